"""Pins for the oracle's forced Cahn-Hilliard step in the frame of the
travelling wave: the fifth-order Hamilton-Jacobi WENO derivative (exact on
linear data, fifth order on smooth periodic data, essentially non-oscillatory
at a jump), the reduction to the plain Cahn-Hilliard step, and the exact
response of the implicit step to the forcing alone."""
import math

import numpy as np
import pytest

from paper_2107_05395_amd import inputs


@pytest.mark.parametrize("plus", [True, False])
def test_weno5_exact_on_linear_data(oracle, plus):
    n = 40
    phi = 0.37 * np.arange(n) - 2.0          # linear away from the periodic wrap
    w = oracle.weno5(phi, plus)
    assert np.allclose(w[4:n - 4], 0.37, rtol=0, atol=1e-14)


@pytest.mark.parametrize("plus", [True, False])
def test_weno5_fifth_order_on_smooth_data(oracle, plus):
    errs = []
    for n in (64, 128, 256):
        x = np.arange(n) / n
        w = oracle.weno5(np.sin(2 * math.pi * x) + 0.3 * np.cos(4 * math.pi * x + 0.2), plus) * n
        exact = 2 * math.pi * np.cos(2 * math.pi * x) - 1.2 * math.pi * np.sin(4 * math.pi * x + 0.2)
        errs.append(np.max(np.abs(w - exact)))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(orders) > 4.3, orders


def test_weno5_is_non_oscillatory_at_a_jump(oracle):
    """A unit step between points 19 and 20: the left-biased derivative at 19
    and the right-biased one at 20 each have one candidate stencil on the flat
    side, whose weight takes over; both stay far below the jump."""
    n = 40
    phi = np.where(np.arange(n) >= 20, 1.0, 0.0)
    assert abs(oracle.weno5(phi, False)[19]) < 1e-10
    assert abs(oracle.weno5(phi, True)[20]) < 1e-10
    # across the jump the upwind stencils see it fully
    assert oracle.weno5(phi, True)[19] > 0.5 and oracle.weno5(phi, False)[20] > 0.5


def test_forced_step_without_forcing_is_the_plain_step(oracle):
    n, m = 64, 6
    sigma, alpha = oracle.ch_coefficients(0.01, 2 * math.pi / n, 1e-3)
    c0 = inputs.uniform_batch(n, m, seed=101, lo=-0.5, hi=0.5)
    assert np.array_equal(oracle.ch_forced_step(c0, sigma, alpha, 0.0, 0.0, 0.3, steps=3),
                          oracle.ch_step(c0, sigma, alpha, steps=3))


def test_forced_step_response_to_the_forcing(oracle):
    """From C = 0 the nonlinear and advection terms vanish, so one step solves
    A C' = dt f0 k cos(k eta_i), eta_i = i dx: on the periodic grid a Fourier
    mode, divided by the eigenvalue 1 + sigma (2 - 2 cos k dx)^2 of the
    left-hand side.  The expected value is built here from dt, f0 and k; the
    oracle goes through its own mapping of (v, f0, k) to the scheme."""
    n, L, gamma = 128, 2 * math.pi, 0.01
    dx = L / n
    dt = 0.1 * dx
    sigma, alpha = oracle.ch_coefficients(gamma, dx, dt)
    k = np.array([1.0, 3.0, 10.0])
    f0 = np.array([0.2, -0.05, 1.0])
    v = np.array([0.4, -0.4, 1.0])
    beta, amp, kdx = oracle.ch_forced_parameters(dt, dx, v, f0, k)
    out = oracle.ch_forced_step(np.zeros((n, 3)), sigma, alpha, beta, amp, kdx)
    eta = np.arange(n)[:, None] * dx
    ref = dt * f0 * k * np.cos(k * eta) / (1 + sigma * (2 - 2 * np.cos(k * dx)) ** 2)
    assert np.max(np.abs(out - ref)) < 1e-15


def _advected(oracle, n, v, steps, dt, L=2 * math.pi):
    """The oracle's forced step with no hyperdiffusion, no nonlinear term and
    no forcing (sigma = alpha = 0, f0 = 0): pure advection of the smooth
    profile sin(eta) + 0.3 cos(2 eta + 0.2) at speed v."""
    dx = L / n
    eta = np.arange(n) * dx
    c0 = np.sin(eta) + 0.3 * np.cos(2 * eta + 0.2)
    beta, amp, kdx = oracle.ch_forced_parameters(dt, dx, np.array([v]), np.array([0.0]),
                                                 np.array([1.0]))
    out = oracle.ch_forced_step(c0[:, None], 0.0, 0.0, beta, amp, kdx, steps=steps)[:, 0]
    return eta, out


@pytest.mark.parametrize("v", [0.5, -0.5])
def test_pure_advection_follows_the_moving_frame_equation(oracle, v):
    """In the frame of the travelling wave the equation carries the term
    v dC/deta on the side of dC/dt, so with nothing else C(eta, t) =
    C0(eta + v t): the profile moves towards -eta for v > 0.  The scheme
    advances it by forward Euler in time with the WENO5 derivative in space;
    with the exact derivative each Fourier mode q would be multiplied by
    (1 + i v q dt) per step, and the oracle must approach that time-discrete
    solution at about fifth order in dx for fixed dt (a dropped dt, dx or v,
    or a wrong sign, breaks the limit).  Over the same time the profile must
    sit at eta + vT, not at eta - vT."""
    dt, steps = 0.01, 20
    T = dt * steps
    errs = []
    for n in (32, 64, 128, 256):
        eta, out = _advected(oracle, n, v, steps, dt)
        g1, g2 = (1 + 1j * v * dt) ** steps, (1 + 2j * v * dt) ** steps
        ref = np.real(-1j * g1 * np.exp(1j * eta)) + 0.3 * np.real(g2 * np.exp(1j * (2 * eta + 0.2)))
        errs.append(np.max(np.abs(out - ref)))
        fwd = np.sin(eta + v * T) + 0.3 * np.cos(2 * (eta + v * T) + 0.2)
        bwd = np.sin(eta - v * T) + 0.3 * np.cos(2 * (eta - v * T) + 0.2)
        # what is left against C0(eta + vT) is the forward-Euler error
        # ~ (v q)^2 dt T / 2 of the modes, far below the shift itself
        assert np.max(np.abs(out - fwd)) < 1e-3 < 0.25 < np.max(np.abs(out - bwd))
    order = math.log2(errs[0] / errs[-1]) / (len(errs) - 1)
    assert order > 4.2, (errs, order)
    assert errs[-1] < 5e-8


def test_forced_step_advection_direction(oracle):
    """Without nonlinearity, hyperdiffusion or forcing (alpha = sigma = 0) a
    step is C + beta W(C), and W is the upwind WENO derivative: beta > 0 uses
    the right-biased one, beta < 0 the left-biased one."""
    n = 48
    c0 = np.where(np.arange(n) >= 20, 1.0, 0.0)[:, None] * np.ones((1, 2))
    out = oracle.ch_forced_step(c0, 0.0, 0.0, [0.25, -0.25], 0.0, 0.0)
    assert np.allclose(out[:, 0], c0[:, 0] + 0.25 * oracle.weno5(c0[:, 0], True), atol=1e-15)
    assert np.allclose(out[:, 1], c0[:, 1] - 0.25 * oracle.weno5(c0[:, 1], False), atol=1e-15)
