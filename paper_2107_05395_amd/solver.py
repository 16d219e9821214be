"""Python face of libbandbatch: shared-matrix factors and batched solves on
torch device tensors.  Argument marshalling only -- every operation on a
batch runs in the library's HIP kernels.

A batch of m systems of size n is an (n, m) tensor, or an (n, m) view with
strides (ld, 1) into a wider array: element i of system k at [i, k], the
interleaved layout of Carroll et al. (arXiv:2107.05395), Section 2.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import BandBatchError, check, dptr, lib

KINDS = ("tri", "tri_cyclic", "penta", "penta_cyclic")


def _stream_ptr(t: torch.Tensor):
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _batch_view(t: torch.Tensor, n: int, dtype: torch.dtype, what: str):
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % what)
    if t.dtype != dtype:
        raise ValueError("%s must be %s, got %s" % (what, dtype, t.dtype))
    if t.dim() != 2 or t.shape[0] != n:
        raise ValueError("%s must have shape (n=%d, m), got %s" % (what, n, tuple(t.shape)))
    m = t.shape[1]
    if m > 1 and t.stride(1) != 1:
        raise ValueError("%s must have unit stride along the batch" % what)
    ld = t.stride(0) if n > 1 else max(m, 1)
    if ld < max(m, 1):
        raise ValueError("%s: leading dimension %d < m = %d" % (what, ld, m))
    return m, ld


class Factor:
    """One shared left-hand-side matrix, factorised once on the host.

    Bands are host sequences of length n (see include/bandbatch.h for which
    entries are ignored or are periodic corners)."""

    def __init__(self, kind: str, bands, n: int, handle):
        self.kind = kind
        self.n = n
        self.nbands = 3 if kind.startswith("tri") else 5
        self.cyclic = kind.endswith("cyclic")
        self._handle = handle
        self._bands = bands   # float64 numpy copies, kept for reference

    @classmethod
    def _make(cls, kind: str, bands, cyclic: bool):
        arrs = [np.ascontiguousarray(np.asarray(b, dtype=np.float64).reshape(-1)) for b in bands]
        n = arrs[0].shape[0]
        if any(a.shape[0] != n for a in arrs):
            raise ValueError("all bands must have the same length")
        full = kind + ("_cyclic" if cyclic else "")
        h = ctypes.c_void_p()
        fn = getattr(lib(), "bb_factor_shared_" + full)
        check(fn(*(dptr(a) for a in arrs), n, ctypes.byref(h)))
        return cls(full, arrs, n, h)

    @classmethod
    def tri(cls, a, b, c, cyclic: bool = False) -> "Factor":
        return cls._make("tri", (a, b, c), cyclic)

    @classmethod
    def penta(cls, a, b, c, d, e, cyclic: bool = False) -> "Factor":
        return cls._make("penta", (a, b, c, d, e), cyclic)

    @classmethod
    def cahn_hilliard(cls, n: int, length: float, gamma: float, dt: float) -> "Factor":
        """The left-hand side of the semi-implicit Cahn-Hilliard scheme on n
        periodic points of a domain of length `length` (bb_factor_ch).  The
        factor carries the scheme's scalars: .sigma, .alpha (dt/dx^2, the
        argument of ch_step), .dt and .dx."""
        h = ctypes.c_void_p()
        sigma, alpha = ctypes.c_double(), ctypes.c_double()
        check(lib().bb_factor_ch(int(n), float(length), float(gamma), float(dt), ctypes.byref(h),
                                 ctypes.byref(sigma), ctypes.byref(alpha)))
        f = cls("penta_cyclic", None, int(n), h)
        f.sigma, f.alpha, f.dt, f.dx, f.gamma = (sigma.value, alpha.value, float(dt),
                                                 float(length) / int(n), float(gamma))
        return f

    def __del__(self):
        h = getattr(self, "_handle", None)
        if h is not None and h.value:
            try:
                lib().bb_factor_destroy(h)
            except Exception:
                pass
            self._handle = None

    @property
    def handle(self):
        return self._handle

    def chunk(self) -> int:
        c = ctypes.c_int32()
        check(lib().bb_factor_info(self._handle, None, None, ctypes.byref(c)))
        return c.value

    def upload(self, device=None) -> None:
        with torch.cuda.device(device if device is not None else torch.cuda.current_device()):
            check(lib().bb_factor_upload(self._handle, None))

    # ------------------------------------------------------------ solves
    def _run(self, fname: str, rhs: torch.Tensor, out, precision: str):
        if precision not in _lib.PRECISION:
            raise ValueError("precision must be one of %s" % list(_lib.PRECISION))
        in_dtype = torch.float32 if precision in ("f32", "f32rhs", "f32rhs_f64") else torch.float64
        out_dtype = torch.float32 if precision == "f32" else torch.float64
        m, ld = _batch_view(rhs, self.n, in_dtype, "rhs")
        if out is None:
            out = torch.empty_like(rhs, dtype=out_dtype)
        m2, ld2 = _batch_view(out, self.n, out_dtype, "out")
        if (m2, ld2) != (m, ld) or out.device != rhs.device:
            raise ValueError("out must match rhs in shape, strides and device")
        with torch.cuda.device(rhs.device):
            check(getattr(lib(), fname)(self._handle, ctypes.c_void_p(rhs.data_ptr()),
                                        ctypes.c_void_p(out.data_ptr()), m, ld,
                                        _lib.PRECISION[precision], _stream_ptr(rhs)))
        return out

    def solve(self, rhs: torch.Tensor, out: torch.Tensor | None = None,
              precision: str = "f64") -> torch.Tensor:
        """x = A^{-1} rhs for every column.

        precision: "f64" (double rhs and x), "f32r" (double rhs and x, float
        sweeps + one double residual refinement), "f32" (float rhs and x, no
        refinement), "f32rhs" (float rhs data, double x, refined like "f32r"),
        "f32rhs_f64" (float rhs data promoted exactly and solved with the FP64
        sweeps, double x).  out may be rhs (in place) except with "f32rhs" and
        "f32rhs_f64"."""
        return self._run("bb_solve_batch_" + self.kind.replace("_cyclic", ""), rhs, out, precision)

    def adjoint(self, g: torch.Tensor, out: torch.Tensor | None = None,
                precision: str = "f64") -> torch.Tensor:
        """lam = A^{-T} g for every column."""
        return self._run("bb_solve_batch_" + self.kind.replace("_cyclic", "") + "_adjoint", g, out,
                         precision)

    def solve_thread_per_system(self, rhs: torch.Tensor, out: torch.Tensor | None = None):
        """The paper's one-thread-per-system sweep (baseline design; tri, double)."""
        m, ld = _batch_view(rhs, self.n, torch.float64, "rhs")
        if out is None:
            out = torch.empty_like(rhs)
        with torch.cuda.device(rhs.device):
            check(lib().bb_solve_batch_tri_thread_per_system(
                self._handle, ctypes.c_void_p(rhs.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                m, ld, _stream_ptr(rhs)))
        return out

    def plan(self, m: int, stepper: bool = False, precision: str = "f64") -> dict:
        """The decomposition a call with m systems takes (host only)."""
        out = [ctypes.c_int32() for _ in range(4)]
        check(lib().bb_plan(self._handle, int(m), 1 if stepper else 0, _lib.PRECISION[precision],
                            *(ctypes.byref(o) for o in out)))
        return dict(chunk=out[0].value, lanes=out[1].value, waves=out[2].value,
                    scalar=bool(out[3].value))

    def band_grad(self, lam: torch.Tensor, x: torch.Tensor,
                  grad: torch.Tensor | None = None) -> torch.Tensor:
        """grad[band, i] += -sum_k lam[i,k] x[i+band-nb/2, k]  ->  (nbands, n) float64."""
        m, ld = _batch_view(lam, self.n, torch.float64, "lam")
        if _batch_view(x, self.n, torch.float64, "x") != (m, ld):
            raise ValueError("x must match lam in shape and strides")
        if grad is None:
            grad = torch.zeros(self.nbands, self.n, dtype=torch.float64, device=lam.device)
        if grad.shape != (self.nbands, self.n) or grad.dtype != torch.float64 or not grad.is_contiguous():
            raise ValueError("grad must be a contiguous (nbands, n) float64 tensor")
        nbytes = lib().bb_band_grad_workspace_bytes(self._handle, m)
        ws = torch.empty(max(nbytes, 8), dtype=torch.uint8, device=lam.device)
        with torch.cuda.device(lam.device):
            check(lib().bb_band_grad(self._handle, ctypes.c_void_p(lam.data_ptr()),
                                     ctypes.c_void_p(x.data_ptr()), m, ld,
                                     ctypes.c_void_p(grad.data_ptr()),
                                     ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(lam)))
        return grad

    def band_grad_noalloc(self, lam: torch.Tensor, x: torch.Tensor,
                          grad: torch.Tensor) -> torch.Tensor:
        """band_grad into a caller-given grad (+=) with the library's own
        device scratch: nothing is allocated (bb_band_grad_noalloc)."""
        m, ld = _batch_view(lam, self.n, torch.float64, "lam")
        if _batch_view(x, self.n, torch.float64, "x") != (m, ld):
            raise ValueError("x must match lam in shape and strides")
        if grad.shape != (self.nbands, self.n) or grad.dtype != torch.float64 or not grad.is_contiguous():
            raise ValueError("grad must be a contiguous (nbands, n) float64 tensor")
        with torch.cuda.device(lam.device):
            check(lib().bb_band_grad_noalloc(self._handle, ctypes.c_void_p(lam.data_ptr()),
                                             ctypes.c_void_p(x.data_ptr()), m, ld,
                                             ctypes.c_void_p(grad.data_ptr()), _stream_ptr(lam)))
        return grad

    def ch_step(self, c: torch.Tensor, alpha: float, steps: int = 1,
                out: torch.Tensor | None = None) -> torch.Tensor:
        """`steps` semi-implicit Cahn-Hilliard steps (cyclic penta factor of the LHS)."""
        m, ld = _batch_view(c, self.n, torch.float64, "c")
        if out is None:
            out = torch.empty_like(c)
        if _batch_view(out, self.n, torch.float64, "out") != (m, ld):
            raise ValueError("out must match c in shape and strides")
        with torch.cuda.device(c.device):
            check(lib().bb_ch_step(self._handle, ctypes.c_void_p(c.data_ptr()),
                                   ctypes.c_void_p(out.data_ptr()), m, ld, float(alpha),
                                   int(steps), _stream_ptr(c)))
        return out

    @property
    def long(self) -> bool:
        """True when n is above what one launch holds on chip (tri 2048,
        penta 1024): solves go through three launches, out of place, and the
        (forced) Cahn-Hilliard step takes one step per call."""
        return self.n > (2048 if self.nbands == 3 else 1024)

    def ch_run(self, c: torch.Tensor, alpha: float, steps: int) -> torch.Tensor:
        """`steps` Cahn-Hilliard steps from c (left unchanged) into a new
        tensor: one fused call, or for long systems one call per step
        alternating between two buffers (the step of a long system is out of
        place)."""
        if not self.long:
            return self.ch_step(c, alpha, steps=steps)
        a, b = torch.empty_like(c), torch.empty_like(c)
        src = c
        for s in range(int(steps)):
            dst = a if s % 2 == 0 else b
            self.ch_step(src, alpha, steps=1, out=dst)
            src = dst
        return src if steps > 0 else c.clone()

    def ch_step_stats(self, c: torch.Tensor, alpha: float, steps: int, every: int = 1,
                      out: torch.Tensor | None = None):
        """Cahn-Hilliard steps plus the ensemble-mean typical domain size
        1/(1 - <C^2>) after every `every` steps -> (state, lbar float64 tensor
        of steps // every entries on the device)."""
        m, ld = _batch_view(c, self.n, torch.float64, "c")
        if out is None:
            out = torch.empty_like(c)
        if _batch_view(out, self.n, torch.float64, "out") != (m, ld):
            raise ValueError("out must match c in shape and strides")
        samples = int(steps) // int(every) if every >= 1 else 0
        lbar = torch.empty(max(samples, 1), dtype=torch.float64, device=c.device)
        with torch.cuda.device(c.device):
            nbytes = lib().bb_ch_stats_workspace_bytes(self._handle, m, samples)
            ws = torch.empty(max(nbytes, 8), dtype=torch.uint8, device=c.device)
            check(lib().bb_ch_step_stats(self._handle, ctypes.c_void_p(c.data_ptr()),
                                         ctypes.c_void_p(out.data_ptr()), m, ld, float(alpha),
                                         int(steps), int(every), ctypes.c_void_p(lbar.data_ptr()),
                                         ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                         _stream_ptr(c)))
        return out, lbar[:samples]

    def ch_forced_step(self, c: torch.Tensor, dt: float, dx: float, v: torch.Tensor,
                       f0: torch.Tensor, k: torch.Tensor, steps: int = 1,
                       out: torch.Tensor | None = None) -> torch.Tensor:
        """Forced Cahn-Hilliard steps in the frame of the travelling wave
        (bb_ch_forced_step); per run: speed v, forcing amplitude f0 and
        wavenumber k (float64 device tensors of m entries); dt, dx shared."""
        m, ld = _batch_view(c, self.n, torch.float64, "c")
        for name, t in (("v", v), ("f0", f0), ("k", k)):
            if (t.dtype != torch.float64 or t.device != c.device or t.numel() != m
                    or not t.is_contiguous()):
                raise ValueError("%s must be a contiguous float64 tensor of m entries on c's device" % name)
        if out is None:
            out = torch.empty_like(c)
        if _batch_view(out, self.n, torch.float64, "out") != (m, ld):
            raise ValueError("out must match c in shape and strides")
        with torch.cuda.device(c.device):
            check(lib().bb_ch_forced_step(self._handle, ctypes.c_void_p(c.data_ptr()),
                                          ctypes.c_void_p(out.data_ptr()), m, ld, float(dt),
                                          float(dx), ctypes.c_void_p(v.data_ptr()),
                                          ctypes.c_void_p(f0.data_ptr()),
                                          ctypes.c_void_p(k.data_ptr()), int(steps),
                                          _stream_ptr(c)))
        return out

    def ch_forced_run(self, c: torch.Tensor, dt: float, dx: float, v: torch.Tensor,
                      f0: torch.Tensor, k: torch.Tensor, steps: int) -> torch.Tensor:
        """`steps` forced Cahn-Hilliard steps from c (left unchanged) into a
        new tensor: one fused call, or for long systems one call per step
        alternating between two buffers."""
        if not self.long:
            return self.ch_forced_step(c, dt, dx, v, f0, k, steps=steps)
        a, b = torch.empty_like(c), torch.empty_like(c)
        src = c
        for s in range(int(steps)):
            dst = a if s % 2 == 0 else b
            self.ch_forced_step(src, dt, dx, v, f0, k, steps=1, out=dst)
            src = dst
        return src if steps > 0 else c.clone()

    def cn_step(self, c: torch.Tensor, w, steps: int = 1,
                out: torch.Tensor | None = None) -> torch.Tensor:
        """`steps` Crank-Nicolson steps A c' = B c with B the constant stencil w
        (3 weights for a tri factor, 5 for a penta one); periodic when the
        factor is cyclic.  out may be c itself (in place)."""
        m, ld = _batch_view(c, self.n, torch.float64, "c")
        if out is None:
            out = torch.empty_like(c)
        if _batch_view(out, self.n, torch.float64, "out") != (m, ld):
            raise ValueError("out must match c in shape and strides")
        if len(w) != self.nbands:
            raise ValueError("need %d stencil weights" % self.nbands)
        wv = (ctypes.c_double * len(w))(*(float(x) for x in w))
        with torch.cuda.device(c.device):
            check(lib().bb_cn_step(self._handle, ctypes.cast(wv, ctypes.c_void_p),
                                   ctypes.c_void_p(c.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                   m, ld, int(steps), _stream_ptr(c)))
        return out

    def cn_trajectory(self, c: torch.Tensor, w, steps: int) -> torch.Tensor:
        """The states after each of `steps` Crank-Nicolson steps from c, as a
        (steps, n, m) tensor whose [s] has c's row stride; bitwise equal to
        `steps` calls of cn_step with steps=1."""
        m, ld = _batch_view(c, self.n, torch.float64, "c")
        if len(w) != self.nbands:
            raise ValueError("need %d stencil weights" % self.nbands)
        if steps < 1:
            raise ValueError("steps must be >= 1")
        traj = torch.empty((steps, self.n, ld), dtype=torch.float64, device=c.device)[:, :, :m]
        wv = (ctypes.c_double * len(w))(*(float(x) for x in w))
        with torch.cuda.device(c.device):
            check(lib().bb_cn_trajectory(self._handle, ctypes.cast(wv, ctypes.c_void_p),
                                         ctypes.c_void_p(c.data_ptr()),
                                         ctypes.c_void_p(traj.data_ptr()), m, ld, int(steps),
                                         _stream_ptr(c)))
        return traj


    def adjoint_trajectory(self, g: torch.Tensor, steps: int) -> torch.Tensor:
        """lam_{s+1} = A^{-T} lam_s from lam_0 = g for s < steps, as a
        (steps, n, m) tensor (bb_adjoint_trajectory): the adjoints of a
        rollout of implicit steps, with the factor's own transposed solve."""
        m, ld = _batch_view(g, self.n, torch.float64, "g")
        if steps < 1:
            raise ValueError("steps must be >= 1")
        traj = torch.empty((steps, self.n, ld), dtype=torch.float64, device=g.device)[:, :, :m]
        with torch.cuda.device(g.device):
            check(lib().bb_adjoint_trajectory(self._handle, ctypes.c_void_p(g.data_ptr()),
                                              ctypes.c_void_p(traj.data_ptr()), m, ld, int(steps),
                                              _stream_ptr(g)))
        return traj

    def adjoint_band_grad(self, g: torch.Tensor, traj: torch.Tensor,
                          grad: torch.Tensor | None = None):
        """Backward over a stretch of the rollout u_t = A^{-1} u_{t-1}, t = 1..T,
        from g = dL/du_T and the forward states traj[t-1] = u_t (a (T, n, m)
        tensor as cn_trajectory returns it): returns (dL/du_0, grad) with
        grad[band, i] += -sum_t sum_k d_{t-1}[i,k] u_t[i+band-nb/2, k],
        d_t = dL/du_t (bb_adjoint_band_grad)."""
        m, ld = _batch_view(g, self.n, torch.float64, "g")
        if traj.dim() != 3 or traj.shape[1:] != (self.n, m) or traj.dtype != torch.float64 \
                or traj.device != g.device or traj.stride() != (self.n * ld, ld, 1):
            raise ValueError("traj must be a (T, n, m) float64 tensor with g's row stride, "
                             "states n * ld apart")
        steps = traj.shape[0]
        if steps < 1:
            raise ValueError("traj holds no state")
        if grad is None:
            grad = torch.zeros(self.nbands, self.n, dtype=torch.float64, device=g.device)
        if grad.shape != (self.nbands, self.n) or grad.dtype != torch.float64 or not grad.is_contiguous():
            raise ValueError("grad must be a contiguous (nbands, n) float64 tensor")
        lam = torch.empty((self.n, ld), dtype=torch.float64, device=g.device)[:, :m]
        nbytes = lib().bb_adjoint_band_grad_workspace_bytes(self._handle, m, ld)
        ws = torch.empty(max(nbytes, 8), dtype=torch.uint8, device=g.device)
        with torch.cuda.device(g.device):
            check(lib().bb_adjoint_band_grad(self._handle, ctypes.c_void_p(g.data_ptr()),
                                             ctypes.c_void_p(traj.data_ptr()),
                                             ctypes.c_void_p(lam.data_ptr()), m, ld, int(steps),
                                             ctypes.c_void_p(grad.data_ptr()),
                                             ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                             _stream_ptr(g)))
        return lam, grad

    def adjoint_band_grad_fused(self, m: int) -> bool:
        """Whether adjoint_band_grad with m systems runs the fused kernel."""
        return bool(lib().bb_adjoint_band_grad_fused(self._handle, int(m)))


TUNING_NAMES = ("max_chunk", "waves_per_system", "waves_per_block", "lockstep", "ch_uniform",
                "grid_linear", "long_spread")


def set_tuning(name: str, value: int | None) -> None:
    """Process-wide override of a decomposition choice (bb_set_tuning); None
    restores the automatic choice."""
    check(lib().bb_set_tuning(name.encode(), -1 if value is None else int(value)))


def get_tuning(name: str) -> int | None:
    v = lib().bb_get_tuning(name.encode())
    if v == -2:
        raise ValueError("unknown tuning name %r" % name)
    return None if v == -1 else int(v)


def mse_loss_grad(u: torch.Tensor, target: torch.Tensor, grad: torch.Tensor | None = None):
    """(loss as a 0-d device tensor, dloss/du) for loss = mean((u - target)^2)."""
    n = u.shape[0]
    m, ld = _batch_view(u, n, torch.float64, "u")
    if _batch_view(target, n, torch.float64, "target") != (m, ld):
        raise ValueError("target must match u in shape and strides")
    if grad is None:
        grad = torch.empty_like(u)
    loss = torch.empty((), dtype=torch.float64, device=u.device)
    nbytes = lib().bb_mse_workspace_bytes(n, m)
    ws = torch.empty(max(nbytes, 8), dtype=torch.uint8, device=u.device)
    with torch.cuda.device(u.device):
        check(lib().bb_mse_loss_grad(ctypes.c_void_p(u.data_ptr()),
                                     ctypes.c_void_p(target.data_ptr()),
                                     ctypes.c_void_p(grad.data_ptr()),
                                     ctypes.c_void_p(loss.data_ptr()), n, m, ld,
                                     ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(u)))
    return loss, grad


def copy_tiles(src: torch.Tensor, dst: torch.Tensor) -> torch.Tensor:
    """dst <- src through bb_copy_tiles (the streaming reference of the
    benchmarks); both contiguous device tensors of the same size in bytes."""
    if not (src.is_cuda and dst.is_cuda and src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("src and dst must be contiguous device tensors")
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("src and dst differ in size")
    with torch.cuda.device(src.device):
        check(lib().bb_copy_tiles(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                  nbytes, _stream_ptr(src)))
    return dst


def copy_rows(src: torch.Tensor, dst: torch.Tensor) -> torch.Tensor:
    """dst <- src (n, m) float64 batches of the same strides through
    bb_copy_rows: the copy with the FP64 sweeps' access pattern, their
    streaming ceiling (n a multiple of 128, m of 32)."""
    n = src.shape[0]
    m, ld = _batch_view(src, n, torch.float64, "src")
    if _batch_view(dst, n, torch.float64, "dst") != (m, ld):
        raise ValueError("dst must match src in shape and strides")
    with torch.cuda.device(src.device):
        check(lib().bb_copy_rows(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                 n, m, ld, _stream_ptr(src)))
    return dst


def empty_batch(n: int, m: int, dtype: torch.dtype = torch.float64, device="cuda",
                pad: int | None = None) -> torch.Tensor:
    """An uninitialised (n, m) batch in the interleaved layout, as a column
    slice of an (n, m + pad) allocation: row stride ld = m + pad.  Every entry
    point takes ld >= m.  By default rows whose byte stride is a multiple of
    64 KiB get 32 elements of padding: with such strides the rows of the
    systems a sweep has in flight fall on fewer memory channels (measured:
    pentadiagonal n = 1024, m = 2^18, 4.27 TB/s at ld = m, 4.73 at m + 32);
    other strides are left alone."""
    esize = torch.empty((), dtype=dtype).element_size()
    if pad is None:
        pad = 32 if (m * esize) % 65536 == 0 else 0
    if pad < 0:
        raise ValueError("pad must be >= 0")
    return torch.empty((n, m + pad), dtype=dtype, device=device)[:, :m]


def max_n() -> int:
    return int(lib().bb_max_n())


__all__ = ["Factor", "BandBatchError", "mse_loss_grad", "copy_tiles", "empty_batch", "max_n", "KINDS",
           "set_tuning", "get_tuning"]
