"""MI355X-native LR-SPIKE banded solver (Spring, Polizzi and Sameh, arXiv 2504.11167).

Thin ctypes binding over ``liblrspike.so`` (the C ABI declared in
``include/lrspike.h``).  Every step of the method runs in the library's HIP
kernels; this module only marshals torch tensors (device memory), the current
HIP stream and autograd plumbing.  There is no CPU fallback: without the built
library or a GPU every call raises.

    plan = factor(bands, p, r, precision="fp64")      # bands: (2k+1, n) float64 CUDA tensor
    x = plan.solve(b)                                  # b: (n,) or (n, m) float64 CUDA tensor
    lam = plan.solve_adjoint(g)
    x = solve(bands, b, p, r)                          # differentiable in bands and b

    bp = factor_batched(systems, bands_base)           # many independent systems
    bp.solve(rhs_base); bp.run(rhs_base)               # eager / one graph replay of factor + solve
"""
import ctypes
import os

import torch

from . import build as _build

__all__ = ["factor", "solve", "Plan", "BatchedPlan", "factor_batched", "pack_systems", "LRSpikeError",
           "library_path", "load_library"]

FP64, FP32_REFINED, FP64_REFINED, FP64_BICGSTAB, FP32_BICGSTAB = 0, 1, 2, 3, 4
_PRECISIONS = {"fp64": FP64, "fp32_refined": FP32_REFINED, "fp64_refined": FP64_REFINED,
               "fp64_bicgstab": FP64_BICGSTAB, "fp32_bicgstab": FP32_BICGSTAB}
VARIANT_FULL, VARIANT_T, VARIANT_I, VARIANT_OTF = 0, 1, 2, 3
_VARIANTS = {"full": VARIANT_FULL, "t": VARIANT_T, "i": VARIANT_I, "otf": VARIANT_OTF}
SVD_EXACT, SVD_RANDOMIZED = 0, 1
_SVDS = {"exact": SVD_EXACT, "randomized": SVD_RANDOMIZED}
_ERRORS = {
    1: "ZERO_PIVOT", 2: "REDUCED_SINGULAR", 3: "NOT_CONVERGED", 4: "NONFINITE",
    5: "HIP_ERROR", 6: "NOT_SUPPORTED", 7: "WORKSPACE",
}


class LRSpikeError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        name = _ERRORS.get(code, f"argument {-code} invalid" if code < 0 else str(code))
        super().__init__(f"{where}: {name} (code {code})")


class _Opts(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int32),
        ("max_refine", ctypes.c_int32),
        ("refine_tol", ctypes.c_double),
        ("stream", ctypes.c_void_p),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
        ("max_nrhs", ctypes.c_int32),
        ("profile", ctypes.c_int32),
        ("variant", ctypes.c_int32),
        ("svd", ctypes.c_int32),
        ("rsvd_ell", ctypes.c_int32),
        ("rsvd_power", ctypes.c_int32),
        ("rsvd_omega", ctypes.c_void_p),
    ]


class _Info(ctypes.Structure):
    _fields_ = [
        ("error", ctypes.c_int32),
        ("partition", ctypes.c_int32),
        ("row", ctypes.c_int64),
        ("refine_iters", ctypes.c_int32),
        ("swapped_blocks", ctypes.c_int32),
        ("last_correction", ctypes.c_double),
        ("min_pivot", ctypes.c_double),
        ("max_abs_entry", ctypes.c_double),
        ("min_sigma_gap", ctypes.c_double),
        ("reduced_growth", ctypes.c_double),
    ]


class _BatchDesc(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("k", ctypes.c_int32),
        ("p", ctypes.c_int32),
        ("r", ctypes.c_int32),
        ("nrhs", ctypes.c_int32),
        ("band_offset", ctypes.c_int64),
        ("rhs_offset", ctypes.c_int64),
    ]


_lib = None
SYMBOLS = (
    "lrspike_default_opts", "lrspike_workspace_size", "lrspike_workspace_size_opts", "lrspike_factor", "lrspike_solve",
    "lrspike_solve_adjoint", "lrspike_band_grad", "lrspike_status", "lrspike_destroy",
    "lrspike_strerror", "lrspike_profile", "lrspike_profile_read", "lrspike_factor_batched",
    "lrspike_solve_batched", "lrspike_run_batched", "lrspike_batch_partitions", "lrspike_solve_noalloc",
)


def library_path():
    return _build.LIB


def load_library():
    """Load liblrspike.so (built in-tree by ``build.py``); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i32, i64 = ctypes.c_int32, ctypes.c_int64
    lib.lrspike_default_opts.argtypes = [ctypes.POINTER(_Opts)]
    lib.lrspike_default_opts.restype = None
    lib.lrspike_workspace_size.argtypes = [i64, i32, i32, i32, i32, i32, ctypes.POINTER(ctypes.c_size_t)]
    lib.lrspike_workspace_size_opts.argtypes = [i64, i32, i32, i32, ctypes.POINTER(_Opts),
                                                ctypes.POINTER(ctypes.c_size_t)]
    lib.lrspike_factor.argtypes = [i64, i32, P, i32, i32, ctypes.POINTER(_Opts), ctypes.POINTER(P)]
    lib.lrspike_solve.argtypes = [P, P, i32]
    lib.lrspike_solve_adjoint.argtypes = [P, P, i32]
    lib.lrspike_band_grad.argtypes = [P, P, P, i32, P]
    lib.lrspike_status.argtypes = [P, ctypes.POINTER(_Info)]
    lib.lrspike_destroy.argtypes = [P]
    lib.lrspike_profile.argtypes = [P, i32]
    lib.lrspike_profile_read.argtypes = [P, i32, ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.lrspike_factor_batched.argtypes = [i32, ctypes.POINTER(_BatchDesc), P, ctypes.POINTER(_Opts), ctypes.POINTER(P)]
    lib.lrspike_solve_batched.argtypes = [P, P]
    lib.lrspike_run_batched.argtypes = [P, P]
    lib.lrspike_batch_partitions.argtypes = [P, i32, ctypes.POINTER(i32)]
    lib.lrspike_solve_noalloc.argtypes = [i64, i32, P, i32, i32, P, i32, P, P]
    lib.lrspike_strerror.argtypes = [i32]
    lib.lrspike_strerror.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check_vec(t, n, name):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if t.shape[0] != n or t.dim() not in (1, 2):
        raise ValueError(f"{name} must have shape (n,) or (n, m) with n = {n}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def workspace_bytes(n, k, p, r, precision="fp64", max_nrhs=32, svd="exact", rsvd_ell=0, variant="full"):
    lib = load_library()
    out = ctypes.c_size_t(0)
    if svd == "exact" and variant in ("full", "t"):
        rc = lib.lrspike_workspace_size(n, k, p, r, _PRECISIONS[precision], max_nrhs, ctypes.byref(out))
    else:
        opts = _Opts()
        lib.lrspike_default_opts(ctypes.byref(opts))
        opts.precision = _PRECISIONS[precision]
        opts.max_nrhs = max_nrhs
        opts.variant = _VARIANTS[variant]
        opts.svd = _SVDS[svd]
        opts.rsvd_ell = rsvd_ell
        rc = lib.lrspike_workspace_size_opts(n, k, p, r, ctypes.byref(opts), ctypes.byref(out))
    if rc:
        raise LRSpikeError(rc, "lrspike_workspace_size")
    return out.value


class Plan:
    """A factored LR-SPIKE plan: the factors live in a caller-owned workspace tensor."""

    def __init__(self, bands, p, r, precision="fp64", max_nrhs=32, max_refine=30, refine_tol=1e-13,
                 workspace=None, profile=False, variant="full", svd="exact", rsvd_ell=None, rsvd_power=0,
                 rsvd_omega=None, rsvd_seed=0):
        """svd="randomized" truncates the spikes through the randomized SVD with
        rsvd_ell sketch columns (default min(k, 2r)) and rsvd_power power steps;
        rsvd_omega, a float64 CUDA tensor of shape (p, 2, k, rsvd_ell), holds the
        Gaussian test matrices (drawn here from rsvd_seed when not given)."""
        lib = load_library()
        if not isinstance(bands, torch.Tensor) or bands.device.type != "cuda" or bands.dtype != torch.float64:
            raise TypeError("bands must be a float64 CUDA tensor of shape (2k+1, n)")
        if bands.dim() != 2 or bands.shape[0] % 2 != 1 or not bands.is_contiguous():
            raise ValueError("bands must be contiguous with shape (2k+1, n)")
        self.k = (bands.shape[0] - 1) // 2
        self.n = bands.shape[1]
        self.p, self.r = int(p), int(r)
        self.precision = precision
        self.variant = variant
        self.max_nrhs = int(max_nrhs)
        self.bands = bands  # borrowed by the library for the plan's lifetime
        self.svd = svd
        ell = 0
        self.rsvd_omega = None
        if svd == "randomized":
            ell = int(rsvd_ell) if rsvd_ell is not None else min(self.k, max(2 * self.r, 1))
            if rsvd_omega is None:
                gen = torch.Generator(device=bands.device)
                gen.manual_seed(int(rsvd_seed))
                rsvd_omega = torch.randn((self.p, 2, self.k, ell), dtype=torch.float64, device=bands.device,
                                         generator=gen)
            if (not isinstance(rsvd_omega, torch.Tensor) or rsvd_omega.device != bands.device or
                    rsvd_omega.dtype != torch.float64 or tuple(rsvd_omega.shape) != (self.p, 2, self.k, ell) or
                    not rsvd_omega.is_contiguous()):
                raise ValueError(f"rsvd_omega must be a contiguous float64 tensor of shape "
                                 f"({self.p}, 2, {self.k}, {ell}) on {bands.device}")
            self.rsvd_omega = rsvd_omega  # read by the factorization's kernels
        elif svd != "exact":
            raise ValueError("svd must be 'exact' or 'randomized'")
        nbytes = workspace_bytes(self.n, self.k, self.p, self.r, precision, self.max_nrhs, svd, ell, variant)
        if workspace is None:
            workspace = torch.empty(nbytes, dtype=torch.uint8, device=bands.device)
        elif workspace.dtype != torch.uint8 or workspace.numel() < nbytes or workspace.device != bands.device:
            raise ValueError(f"workspace must be a uint8 tensor of >= {nbytes} bytes on {bands.device}")
        self.workspace = workspace
        opts = _Opts()
        lib.lrspike_default_opts(ctypes.byref(opts))
        opts.precision = _PRECISIONS[precision]
        opts.max_refine = max_refine
        opts.refine_tol = refine_tol
        opts.stream = torch.cuda.current_stream(bands.device).cuda_stream
        opts.workspace = self.workspace.data_ptr()
        opts.workspace_bytes = nbytes
        opts.max_nrhs = self.max_nrhs
        opts.profile = 1 if profile else 0
        opts.variant = _VARIANTS[variant]
        opts.svd = _SVDS[svd]
        opts.rsvd_ell = ell
        opts.rsvd_power = int(rsvd_power)
        opts.rsvd_omega = self.rsvd_omega.data_ptr() if self.rsvd_omega is not None else None
        handle = ctypes.c_void_p()
        rc = lib.lrspike_factor(self.n, self.k, bands.data_ptr(), self.p, self.r, ctypes.byref(opts),
                                ctypes.byref(handle))
        if rc:
            raise LRSpikeError(rc, "lrspike_factor")
        self._h = handle
        self._lib = lib

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.lrspike_destroy(h)
            self._h = None

    def _apply(self, b, inplace, adjoint, check=False):
        _check_vec(b, self.n, "rhs")
        x = b if inplace else b.clone()
        m = 1 if x.dim() == 1 else x.shape[1]
        fn = self._lib.lrspike_solve_adjoint if adjoint else self._lib.lrspike_solve
        for c0 in range(0, m, self.max_nrhs):
            cols = min(self.max_nrhs, m - c0)
            if m == cols:
                rc = fn(self._h, x.data_ptr(), m)
            else:
                blk = x[:, c0:c0 + cols].contiguous()
                rc = fn(self._h, blk.data_ptr(), cols)
                x[:, c0:c0 + cols] = blk
            if rc:
                raise LRSpikeError(rc, "lrspike_solve_adjoint" if adjoint else "lrspike_solve")
        if check:
            self.status()
        return x

    def solve(self, b, inplace=False, check=False):
        """x = M_r^{-1} b (A^{-1} b at r = k, or refined to tolerance with a refined precision).
        check=True synchronizes and raises LRSpikeError on any device-latched error."""
        return self._apply(b, inplace, False, check)

    def solve_adjoint(self, g, inplace=False, check=False):
        """M_r^{-T} g, the exact transpose of solve (refined against A^T with a refined precision)."""
        return self._apply(g, inplace, True, check)

    def band_grad(self, lam, x):
        """-lam x^T restricted to the band, shape (2k+1, n)."""
        _check_vec(lam, self.n, "lam")
        _check_vec(x, self.n, "x")
        m = 1 if x.dim() == 1 else x.shape[1]
        out = torch.empty_like(self.bands)
        rc = self._lib.lrspike_band_grad(self._h, lam.data_ptr(), x.data_ptr(), m, out.data_ptr())
        if rc:
            raise LRSpikeError(rc, "lrspike_band_grad")
        return out

    def profile(self, enable=True):
        rc = self._lib.lrspike_profile(self._h, 1 if enable else 0)
        if rc:
            raise LRSpikeError(rc, "lrspike_profile")

    def profile_read(self):
        """{kernel name: (total ms, launches)} since the last read (synchronizes)."""
        mx = 64
        names = ctypes.create_string_buffer(32 * mx)
        ms = (ctypes.c_double * mx)()
        cnt = (ctypes.c_int32 * mx)()
        count = ctypes.c_int32(0)
        rc = self._lib.lrspike_profile_read(self._h, mx, names, ms, cnt, ctypes.byref(count))
        if rc:
            raise LRSpikeError(rc, "lrspike_profile_read")
        out = {}
        for i in range(min(mx, count.value)):
            nm = names.raw[32 * i:32 * i + 32].split(b"\0", 1)[0].decode()
            out[nm] = (ms[i], cnt[i])
        return out

    def status(self):
        """Synchronize and return the device-latched state as a dict; raises on a latched error."""
        info = _Info()
        rc = self._lib.lrspike_status(self._h, ctypes.byref(info))
        d = {f: getattr(info, f) for f, _ in _Info._fields_}
        if rc:
            err = LRSpikeError(rc, "lrspike_status")
            err.info = d
            raise err
        return d


def factor(bands, p, r, precision="fp64", max_nrhs=32, **kw):
    """Factor A (bands: (2k+1, n) float64 CUDA tensor) into p partitions at rank r.
    precision: "fp64" (one application of M_r^{-1}), "fp32_refined" / "fp64_refined" (iterative
    refinement preconditioned by M_r^{-1}) or "fp64_bicgstab" / "fp32_bicgstab" (BiCGStab
    right-preconditioned by M_r^{-1}); variant: "full" (LR-SPIKE), "t" (LR-SPIKE-T), "i" (LR-SPIKE-I:
    S~_red by BiCGStab preconditioned by LR-SPIKE-T's system) or "otf" (LR-SPIKE-OTF: the true
    reduced system the same way, products by partition solves; the result is A^{-1} b); for "i"
    and "otf" refine_tol / max_refine are the inner iteration's tolerance and cap."""
    return Plan(bands, p, r, precision=precision, max_nrhs=max_nrhs, **kw)


class LRSpikeSolve(torch.autograd.Function):
    """x = A^{-1} b through LR-SPIKE; backward through the adjoint solve:
    grad_b = A^{-T} grad_x, grad_bands = -lam x^T on the band.

    These are the gradients of the converged solve x = A^{-1} b.  At r = k one
    application of the FP64 plan is that solve; at r < k the plan's operator
    M_r^{-1} differs from A^{-1} (and depends on A through the truncated
    spikes), so the plan is FP64_REFINED: M_r^{-1} preconditions an iterative
    refinement with FP64 residual, forward against A and backward against A^T,
    to refine_tol.  Any device-latched error (zero pivot, non-convergence,
    non-finite data) raises LRSpikeError in forward or backward."""

    @staticmethod
    def forward(ctx, bands, b, p, r, precision, refine_tol):
        m = 1 if b.dim() == 1 else b.shape[1]
        plan = Plan(bands.detach(), p, r, precision=precision, max_nrhs=max(1, m), refine_tol=refine_tol)
        x = plan.solve(b.detach(), check=True)
        ctx.plan = plan
        ctx.save_for_backward(x)
        return x

    @staticmethod
    def backward(ctx, gx):
        (x,) = ctx.saved_tensors
        plan = ctx.plan
        lam = plan.solve_adjoint(gx.contiguous(), check=True)
        gbands = plan.band_grad(lam, x) if ctx.needs_input_grad[0] else None
        return gbands, (lam if ctx.needs_input_grad[1] else None), None, None, None, None


def solve(bands, b, p, r=None, precision=None, refine_tol=1e-13):
    """Differentiable x = A^{-1} b (r defaults to k, where LR-SPIKE is exact).

    precision defaults to "fp64" at r = k and to "fp64_refined" at r < k, so
    that forward and gradients are those of A^{-1} b; "fp32_refined" is also
    accepted.  A plain "fp64" plan at r < k would apply M_r^{-1}, whose band
    gradient is not -lam x^T, and is refused."""
    k = (bands.shape[0] - 1) // 2
    if r is None:
        r = k
    if precision is None:
        precision = "fp64" if r == k else "fp64_refined"
    if precision == "fp64" and r != k:
        raise ValueError("solve(): at r < k the gradient of the one-shot operator is not -lam x^T; "
                         "use precision='fp64_refined' (the default) or 'fp32_refined'")
    return LRSpikeSolve.apply(bands, b, p, r, precision, refine_tol)


def solve_noalloc(bands, b, p, r, status=None):
    """x = M_r^{-1} b (FP64) through ``lrspike_solve_noalloc``: factor and
    solve with the library's static device scratch, nothing allocated (the
    output tensor aside, which this wrapper clones from b).  status: optional
    int32 CUDA tensor of one element that receives the latched error code."""
    lib = load_library()
    if not isinstance(bands, torch.Tensor) or bands.device.type != "cuda" or bands.dtype != torch.float64 or \
            bands.dim() != 2 or not bands.is_contiguous():
        raise TypeError("bands must be a contiguous float64 CUDA tensor of shape (2k+1, n)")
    k = (bands.shape[0] - 1) // 2
    n = bands.shape[1]
    _check_vec(b, n, "rhs")
    x = b.clone()
    m = 1 if x.dim() == 1 else x.shape[1]
    st = None
    if status is not None:
        if status.dtype != torch.int32 or status.device != bands.device or status.numel() < 1:
            raise ValueError("status must be an int32 tensor on the bands' device")
        st = status.data_ptr()
    rc = lib.lrspike_solve_noalloc(n, k, bands.data_ptr(), int(p), int(r), x.data_ptr(), m,
                                   torch.cuda.current_stream(bands.device).cuda_stream, st)
    if rc:
        raise LRSpikeError(rc, "lrspike_solve_noalloc")
    return x


def pack_systems(bands_list, rhs_list, p=None, r=None):
    """Host-side marshalling for the batched calls: concatenates per-system
    band-major bands ((2k_s+1, n_s) arrays) and row-major right-hand sides
    ((n_s, m_s) arrays) into two flat float64 arrays and returns them with the
    descriptor tuples (n, k, p, r, nrhs, band_offset, rhs_offset).  p defaults
    to 0 (autotuned), r to k // 2."""
    import numpy as np
    descs, bo, ro = [], 0, 0
    for s, (b, f) in enumerate(zip(bands_list, rhs_list)):
        k = (b.shape[0] - 1) // 2
        n = b.shape[1]
        f2 = f.reshape(n, -1)
        ps = 0 if p is None else (p[s] if hasattr(p, "__len__") else p)
        rs = k // 2 if r is None else (r[s] if hasattr(r, "__len__") else r)
        descs.append((n, k, int(ps), int(rs), f2.shape[1], bo, ro))
        bo += b.size
        ro += f2.size
    bands = np.concatenate([np.ascontiguousarray(b).ravel() for b in bands_list])
    rhs = np.concatenate([np.ascontiguousarray(f).ravel() for f in rhs_list])
    return bands, rhs, descs


class BatchedPlan:
    """Factored batch of independent banded systems (``lrspike_factor_batched``).

    ``systems``: descriptor tuples (n, k, p, r, nrhs, band_offset, rhs_offset),
    offsets in elements of ``bands_base`` / ``rhs_base`` (flat float64 CUDA
    tensors).  The plan borrows ``bands_base`` and owns its device memory."""

    def __init__(self, systems, bands_base, precision="fp64"):
        lib = load_library()
        if not isinstance(bands_base, torch.Tensor) or bands_base.device.type != "cuda" or \
                bands_base.dtype != torch.float64 or not bands_base.is_contiguous():
            raise TypeError("bands_base must be a contiguous float64 CUDA tensor")
        self.count = len(systems)
        arr = (_BatchDesc * self.count)()
        for i, d in enumerate(systems):
            arr[i] = _BatchDesc(*[int(v) for v in d])
        self.systems = [tuple(int(v) for v in d) for d in systems]
        self.bands_base = bands_base
        self.precision = precision
        opts = _Opts()
        lib.lrspike_default_opts(ctypes.byref(opts))
        opts.precision = _PRECISIONS[precision]
        opts.stream = torch.cuda.current_stream(bands_base.device).cuda_stream
        handle = ctypes.c_void_p()
        rc = lib.lrspike_factor_batched(self.count, arr, bands_base.data_ptr(), ctypes.byref(opts),
                                        ctypes.byref(handle))
        if rc:
            raise LRSpikeError(rc, "lrspike_factor_batched")
        self._h = handle
        self._lib = lib

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.lrspike_destroy(h)
            self._h = None

    def _check_rhs(self, rhs_base):
        if not isinstance(rhs_base, torch.Tensor) or rhs_base.device.type != "cuda" or \
                rhs_base.dtype != torch.float64 or not rhs_base.is_contiguous():
            raise TypeError("rhs_base must be a contiguous float64 CUDA tensor")

    def solve(self, rhs_base):
        """In place: every system's right-hand sides are replaced by its solution."""
        self._check_rhs(rhs_base)
        rc = self._lib.lrspike_solve_batched(self._h, rhs_base.data_ptr())
        if rc:
            raise LRSpikeError(rc, "lrspike_solve_batched")
        return rhs_base

    def run(self, rhs_base):
        """Refactor from bands_base and solve in place, as one HIP graph replay."""
        self._check_rhs(rhs_base)
        rc = self._lib.lrspike_run_batched(self._h, rhs_base.data_ptr())
        if rc:
            raise LRSpikeError(rc, "lrspike_run_batched")
        return rhs_base

    def partitions(self):
        out = (ctypes.c_int32 * self.count)()
        rc = self._lib.lrspike_batch_partitions(self._h, self.count, out)
        if rc:
            raise LRSpikeError(rc, "lrspike_batch_partitions")
        return list(out)

    def status(self):
        info = _Info()
        rc = self._lib.lrspike_status(self._h, ctypes.byref(info))
        d = {f: getattr(info, f) for f, _ in _Info._fields_}
        if rc:
            err = LRSpikeError(rc, "lrspike_status")
            err.info = d
            raise err
        return d


def factor_batched(systems, bands_base, precision="fp64"):
    return BatchedPlan(systems, bands_base, precision=precision)
