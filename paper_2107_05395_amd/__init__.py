"""bandbatch for MI355X: batched tridiagonal / pentadiagonal solves with one
shared left-hand-side matrix (Carroll, Gloster, Bustamante, O Naraigh,
arXiv:2107.05395), as hand-written HIP kernels for gfx950 behind a C ABI
(include/bandbatch.h).

    from paper_2107_05395_amd import Factor
    f = Factor.tri(a, b, c)            # host factorisation, once
    x = f.solve(rhs)                   # rhs: (n, m) float64 device tensor

The compiled library is loaded on first use and must have been built in tree
(``python -m paper_2107_05395_amd.build``).
"""
from ._lib import BandBatchError  # noqa: F401  (no library load at import)


def __getattr__(name):
    if name in ("Factor", "mse_loss_grad", "max_n", "KINDS", "set_tuning", "get_tuning",
                "empty_batch"):
        from . import solver
        return getattr(solver, name)
    if name in ("banded_solve", "banded_rollout", "mse_loss", "BandedSolve", "BandedRollout"):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)
