"""LR-SPIKE oracle (FP64, CPU) -- TEST INFRASTRUCTURE ONLY.

A plain C implementation of what the banded LR-SPIKE method computes
(Spring, Polizzi and Sameh, arXiv 2504.11167), wrapped with ctypes:

* ``band_solve``      R0, the plain definition x* = A^{-1} f (or A^{-T} g):
                      band Gaussian elimination with row partial pivoting.
* ``lrspike``         R1, the literal LR-SPIKE solution at rank r: the DS
                      factorization, explicit spikes, rank-r truncated SVD of the
                      whole spikes, the reduced system solved as a band matrix,
                      and solve-based recovery (sections "SPIKE partitioning",
                      "SPIKE reduced system solvers", "SVD representation of the
                      spikes").  With ``transpose=True`` it is R3, the exact
                      transpose of that operator.  ``variant="t"`` is
                      LR-SPIKE-T: the reduced system cut to its independent
                      2 x 2 interface blocks (truncated SPIKE).
* ``band_solve_refined``  x* accurate to about one rounding whatever the
                      condition number (residual in long double).
* ``bicgstab``        BiCGStab right-preconditioned by the LR-SPIKE operator,
                      the outer Krylov solver of the paper's experiments.
* ``lrspike_iter``    LR-SPIKE-I and LR-SPIKE-OTF: the reduced system (its
                      low-rank form, or the true one) solved by BiCGStab
                      preconditioned by the LR-SPIKE-T system.
* ``lrspike_rsvd``    R1 / R3 with the spikes truncated through the randomized
                      SVD (Halko-Martinsson-Tropp proto-algorithm, caller-drawn
                      Gaussian test matrices); ``rsvd_project`` is its range
                      finder Q Q^T a.
* ``reduced_dense``, ``partition_spikes``, ``thin_svd``, ``band_matvec``,
  ``band_grad`` and ``partition`` expose the intermediate objects the pins test.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline
leg may import this package.  It shares no code with the GPU library.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.POINTER(ctypes.c_int64)


def _load():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build(force=False)
        lib = ctypes.CDLL(path)
        i64, i32 = ctypes.c_int64, ctypes.c_int
        lib.orc_band_solve.argtypes = [i64, i32, _D, i32, _D, _D, i32]
        lib.orc_band_solve_refined.argtypes = [i64, i32, _D, i32, _D, _D, i32, i32]
        lib.orc_band_matvec.argtypes = [i64, i32, _D, i32, _D, _D, i32]
        lib.orc_band_matvec.restype = None
        lib.orc_partition.argtypes = [i64, i32, _I64]
        lib.orc_partition.restype = None
        lib.orc_thin_svd.argtypes = [i64, i32, _D, _D, _D]
        lib.orc_lrspike.argtypes = [i64, i32, _D, i32, i32, i32, _D, _D, i32, _D, i32, i32]
        lib.orc_lrspike_rsvd.argtypes = [i64, i32, _D, i32, i32, i32, _D, _D, i32, _D, i32, i32, i32, i32, _D]
        lib.orc_rsvd_project.argtypes = [i64, i32, _D, i32, i32, _D, _D]
        lib.orc_lrspike_iter.argtypes = [i64, i32, _D, i32, i32, i32, _D, _D, i32, ctypes.c_double, i32,
                                         ctypes.POINTER(ctypes.c_int), _D, i32]
        lib.orc_reduced_dense.argtypes = [i64, i32, _D, i32, i32, _D]
        lib.orc_partition_spikes.argtypes = [i64, i32, _D, i32, i32, _D, _D]
        lib.orc_bicgstab.argtypes = [i64, i32, _D, i32, i32, i32, i32, _D, _D, ctypes.c_double, i32, i32,
                                     ctypes.POINTER(ctypes.c_int), _D, i32]
        lib.orc_band_grad.argtypes = [i64, i32, i32, _D, _D, _D]
        lib.orc_band_grad.restype = None
        _lib = lib
    return _lib


class OracleError(RuntimeError):
    pass


def _p(a):
    return a.ctypes.data_as(_D)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _as2d(f):
    f = _f64(f)
    return (f[:, None], True) if f.ndim == 1 else (f, False)


def _check(rc, what):
    if rc != 0:
        raise OracleError(f"{what}: return code {rc}")


def _band_args(bands):
    bands = _f64(bands)
    k2, n = bands.shape
    assert k2 % 2 == 1, "bands must have 2k+1 rows"
    return bands, n, (k2 - 1) // 2


def partition(n, p):
    """Row offsets (p + 1 entries) of the p partitions: floor(n/p) + [j < n mod p] rows."""
    offs = np.zeros(p + 1, dtype=np.int64)
    _load().orc_partition(n, p, offs.ctypes.data_as(_I64))
    return offs


def band_solve(bands, f, transpose=False):
    """R0: A^{-1} f (or A^{-T} f) by band Gaussian elimination with partial pivoting."""
    bands, n, k = _band_args(bands)
    f2, flat = _as2d(f)
    x = np.empty_like(f2)
    _check(_load().orc_band_solve(n, k, _p(bands), f2.shape[1], _p(f2), _p(x), int(transpose)), "band_solve")
    return x[:, 0] if flat else x


def band_solve_refined(bands, f, steps=2, transpose=False):
    """x* (or A^{-T} f) with `steps` long-double-residual corrections (accurate to ~u for any kappa)."""
    bands, n, k = _band_args(bands)
    f2, flat = _as2d(f)
    x = np.empty_like(f2)
    _check(_load().orc_band_solve_refined(n, k, _p(bands), f2.shape[1], _p(f2), _p(x), steps, int(transpose)),
           "band_solve_refined")
    return x[:, 0] if flat else x


def band_matvec(bands, x, transpose=False):
    """A x (or A^T x) from the band-major storage."""
    bands, n, k = _band_args(bands)
    x2, flat = _as2d(x)
    y = np.empty_like(x2)
    _load().orc_band_matvec(n, k, _p(bands), x2.shape[1], _p(x2), _p(y), int(transpose))
    return y[:, 0] if flat else y


_VARIANTS = {"full": 0, "t": 1}


def lrspike(bands, f, p, r, transpose=False, return_sv=False, threads=0, variant="full"):
    """R1 (or R3 with transpose=True): the literal LR-SPIKE solve at rank r.

    variant="full" solves the whole truncated reduced system S~_red;
    variant="t" is LR-SPIKE-T, which keeps only its 2 x 2 interface blocks
    [[I, V~_{j,b}], [W~_{j+1,t}, I]] (the truncated-SPIKE system S~~_red)."""
    bands, n, k = _band_args(bands)
    f2, flat = _as2d(f)
    x = np.empty_like(f2)
    sv = np.zeros((p, 2, k))
    rc = _load().orc_lrspike(n, k, _p(bands), p, r, f2.shape[1], _p(f2), _p(x), int(transpose), _p(sv), threads,
                             _VARIANTS[variant])
    _check(rc, "lrspike")
    x = x[:, 0] if flat else x
    return (x, sv) if return_sv else x


def lrspike_rsvd(bands, f, p, r, omega, q=0, transpose=False, return_sv=False, threads=0, variant="full"):
    """R1 / R3 with every spike truncated through the randomized SVD (the
    proto-algorithm of Halko, Martinsson and Tropp): omega holds the Gaussian
    test matrices, shape (p, 2, k, ell) (V_j then W_j of each partition), q
    the power steps.  Needs r < k."""
    bands, n, k = _band_args(bands)
    f2, flat = _as2d(f)
    om = _f64(omega)
    if om.ndim != 4 or om.shape[:3] != (p, 2, k):
        raise ValueError("omega must have shape (p, 2, k, ell)")
    ell = om.shape[3]
    x = np.empty_like(f2)
    sv = np.zeros((p, 2, k))
    rc = _load().orc_lrspike_rsvd(n, k, _p(bands), p, r, f2.shape[1], _p(f2), _p(x), int(transpose), _p(sv),
                                  threads, _VARIANTS[variant], ell, q, _p(om))
    _check(rc, "lrspike_rsvd")
    x = x[:, 0] if flat else x
    return (x, sv) if return_sv else x


def lrspike_iter(bands, f, p, r, kind="i", tol=1e-13, max_it=100, threads=0):
    """LR-SPIKE-I (kind="i": S~_red) or LR-SPIKE-OTF (kind="otf": the true
    S_red) solved by BiCGStab right-preconditioned by S~~_red at rank r, then
    the solve-based recovery.  Returns (x, iters, relres) per column."""
    bands, n, k = _band_args(bands)
    f2, flat = _as2d(f)
    m = f2.shape[1]
    x = np.empty_like(f2)
    iters = (ctypes.c_int * m)()
    relres = np.zeros(m)
    rc = _load().orc_lrspike_iter(n, k, _p(bands), p, r, m, _p(f2), _p(x), {"i": 0, "otf": 1}[kind], tol, max_it,
                                  iters, _p(relres), threads)
    _check(rc, "lrspike_iter")
    return (x[:, 0] if flat else x), np.array(list(iters)), relres


def rsvd_project(a, omega, q=0):
    """Q Q^T a for Q an orthonormal basis of range((a a^T)^q a omega): the
    randomized range finder of the spike truncation."""
    a = _f64(a)
    om = _f64(omega)
    rows, cols = a.shape
    ell = om.shape[1]
    if om.shape[0] != cols:
        raise ValueError("omega must have a.shape[1] rows")
    out = np.empty_like(a)
    _check(_load().orc_rsvd_project(rows, cols, _p(a), ell, q, _p(om), _p(out)), "rsvd_project")
    return out


def bicgstab(bands, f, p, r, tol=1e-13, max_it=200, transpose=False, variant="full", threads=0):
    """BiCGStab right-preconditioned by the LR-SPIKE operator M_r^{-1} (column by
    column, x_0 = M^{-1} f).  Returns (x, iterations per column, final relative
    residual per column)."""
    bands, n, k = _band_args(bands)
    f2, flat = _as2d(f)
    m = f2.shape[1]
    x = np.empty_like(f2)
    its = (ctypes.c_int * m)()
    res = np.zeros(m)
    rc = _load().orc_bicgstab(n, k, _p(bands), p, r, _VARIANTS[variant], m, _p(f2), _p(x), tol, max_it,
                              int(transpose), its, _p(res), threads)
    _check(rc, "bicgstab")
    return (x[:, 0] if flat else x), list(its), res


def reduced_dense(bands, p, r):
    """The dense truncated reduced system S~_red (order 2kp) at rank r."""
    bands, n, k = _band_args(bands)
    N = 2 * k * p
    S = np.zeros((N, N))
    _check(_load().orc_reduced_dense(n, k, _p(bands), p, r, _p(S)), "reduced_dense")
    return S


def partition_spikes(bands, p, j):
    """Explicit spikes (V_j, W_j), each n_j x k (zeros where the spike does not exist)."""
    bands, n, k = _band_args(bands)
    offs = partition(n, p)
    nj = int(offs[j + 1] - offs[j])
    V = np.zeros((nj, k))
    W = np.zeros((nj, k))
    _check(_load().orc_partition_spikes(n, k, _p(bands), p, j, _p(V), _p(W)), "partition_spikes")
    return V, W


def thin_svd(a):
    """Singular values (descending) and right singular vectors (columns) of a tall matrix."""
    a = _f64(a)
    rows, cols = a.shape
    s = np.zeros(cols)
    vr = np.zeros((cols, cols))
    _check(_load().orc_thin_svd(rows, cols, _p(a), _p(s), _p(vr)), "thin_svd")
    return s, vr


def band_grad(lam, x, k):
    """-lam x^T restricted to the band, in band-major layout ((2k+1) x n)."""
    lam2, _ = _as2d(lam)
    x2, _ = _as2d(x)
    n, m = lam2.shape
    g = np.zeros((2 * k + 1, n))
    _load().orc_band_grad(n, k, m, _p(lam2), _p(x2), _p(g))
    return g
