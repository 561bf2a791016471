"""Host-only checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching the GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "lrspike.h")).read()
    return sorted(set(re.findall(r"\b(lrspike_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    import paper_2504_11167_amd as lr
    lib = lr.load_library()
    names = _declared()
    assert "lrspike_factor" in names and "lrspike_solve" in names
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) <= set(lr.SYMBOLS) | {"lrspike_default_opts"}


def test_default_opts_and_strerror():
    import paper_2504_11167_amd as lr
    lib = lr.load_library()
    o = lr._Opts()
    lib.lrspike_default_opts(ctypes.byref(o))
    assert o.precision == 0 and o.max_refine == 30 and abs(o.refine_tol - 1e-13) < 1e-30 and o.max_nrhs == 32
    assert lib.lrspike_strerror(0) == b"ok"
    assert b"pivot" in lib.lrspike_strerror(1)
    assert b"invalid" in lib.lrspike_strerror(-3)


@pytest.mark.parametrize("args,code", [
    ((0, 4, 1, 1, 0, 1), -1),
    ((100, 0, 1, 0, 0, 1), -2),
    ((100, 4, 0, 1, 0, 1), -3),
    ((100, 4, 101, 1, 0, 1), -3),
    ((100, 4, 2, 5, 0, 1), -4),
    ((100, 4, 2, -1, 0, 1), -4),
    ((100, 4, 2, 2, 7, 1), -5),
    ((100, 4, 2, 2, 5, 1), -5),
    ((100, 4, 2, 2, 0, 0), -6),
])
def test_workspace_size_argument_codes(args, code):
    import paper_2504_11167_amd as lr
    lib = lr.load_library()
    out = ctypes.c_size_t(0)
    assert lib.lrspike_workspace_size(*args, ctypes.byref(out)) == code


def test_noalloc_rejects_problems_beyond_its_scratch_before_any_gpu_call():
    """The allocation-free entry point checks sizes on the host first: a
    workspace above its 64 MiB scratch returns LRSPIKE_ERR_WORKSPACE (7)."""
    import paper_2504_11167_amd as lr
    lib = lr.load_library()
    assert lib.lrspike_solve_noalloc(1 << 22, 32, None, 1024, 8, None, 16, None, None) == 7
    assert lib.lrspike_solve_noalloc(0, 4, None, 1, 1, None, 1, None, None) == -1
    assert lib.lrspike_solve_noalloc(100, 4, None, 2, 5, None, 1, None, None) == -5
    assert lib.lrspike_solve_noalloc(100, 4, None, 2, 2, None, 0, None, None) == -7


def test_workspace_size_grows_with_problem():
    import paper_2504_11167_amd as lr
    a = lr.workspace_bytes(4096, 8, 4, 8)
    b = lr.workspace_bytes(8192, 8, 4, 8)
    c = lr.workspace_bytes(4096, 8, 4, 8, precision="fp32_refined")
    d = lr.workspace_bytes(4096, 8, 4, 8, precision="fp64_refined")
    assert 0 < a < b
    assert c > 0
    assert d > a  # the refined plans hold the residual and the copy of f


def test_randomized_svd_workspace_and_option_codes():
    """The randomized spike SVD holds the n x 2 ell sketch (and at least 2 ell
    solve columns) in the workspace instead of the spike sweeps' n x 2K
    intermediate; ell outside [r, k], power steps outside [0, 4] and unknown
    svd codes are argument errors (-5), while r = k or r = 0 (nothing
    truncated) needs nothing extra."""
    import paper_2504_11167_amd as lr
    lib = lr.load_library()
    n, k, p, r = 4096, 16, 4, 4
    rs8 = lr.workspace_bytes(n, k, p, r, max_nrhs=2, svd="randomized", rsvd_ell=8)
    rs12 = lr.workspace_bytes(n, k, p, r, max_nrhs=2, svd="randomized", rsvd_ell=12)
    assert rs12 >= rs8 + n * 2 * 4 * 8
    assert lr.workspace_bytes(n, k, p, k, max_nrhs=2, svd="randomized", rsvd_ell=8) == \
        lr.workspace_bytes(n, k, p, k, max_nrhs=2)
    o = lr._Opts()
    lib.lrspike_default_opts(ctypes.byref(o))
    out = ctypes.c_size_t(0)
    for svd, ell, q, code in [(1, 8, 0, 0), (1, 3, 0, -5), (1, 17, 0, -5), (1, 8, 5, -5), (1, 8, -1, -5),
                              (2, 8, 0, -5), (0, 99, 9, 0)]:
        o.svd, o.rsvd_ell, o.rsvd_power = svd, ell, q
        assert lib.lrspike_workspace_size_opts(n, k, p, r, ctypes.byref(o), ctypes.byref(out)) == code


def test_factor_rejects_bad_sizes_before_gpu():
    import paper_2504_11167_amd as lr
    lib = lr.load_library()
    o = lr._Opts()
    lib.lrspike_default_opts(ctypes.byref(o))
    h = ctypes.c_void_p()
    assert lib.lrspike_factor(0, 4, None, 1, 1, ctypes.byref(o), ctypes.byref(h)) == -1
    assert lib.lrspike_factor(100, 0, None, 1, 0, ctypes.byref(o), ctypes.byref(h)) == -2


def test_product_package_does_not_reference_oracle():
    pkg = os.path.join(ROOT, "paper_2504_11167_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".h")):
                text = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in text and "from oracle" not in text, fn
                assert "lrspike_oracle" not in text, fn
