"""LR-SPIKE-T on the GPU through the C ABI, against the oracle.

LR-SPIKE-T keeps only the 2 x 2 interface blocks [[I, V~_{j,b}], [W~_{j+1,t}, I]]
of the truncated reduced system (the truncated-SPIKE system S~~_red of eqs.
truncated_redsys and red_sys_prec_mid_1/2; table solver-list), each solved on
its own, with the same solve-based recovery as LR-SPIKE.  Parity: relative
error <= 1e-12 per column against the oracle's literal variant (band matrix
with the dropped blocks left out), forward and adjoint, over every kernel
width (K = 4 .. 64), ragged partitions, several column chunks, r < k and r = k.
As a preconditioner of the refined precisions it must reach A^{-1} f.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def col_rel(got, ref):
    got = got.reshape(ref.shape[0], -1)
    ref = ref.reshape(ref.shape[0], -1)
    return max(np.linalg.norm(got[:, c] - ref[:, c]) / np.linalg.norm(ref[:, c]) for c in range(ref.shape[1]))


CASES = [  # n, k, p, r, m, rule
    (1000, 3, 5, 2, 2, "weak"),
    (1203, 8, 7, 5, 1, "weak"),
    (2000, 16, 5, 8, 3, "weak"),
    (2000, 16, 4, 16, 40, "weak"),
    (3001, 32, 6, 12, 17, "weak"),
    (4000, 32, 3, 32, 2, "weak"),
    (2600, 50, 4, 20, 5, "strict"),
    (4000, 64, 5, 32, 3, "strict"),
    (600, 10, 2, 4, 2, "weak"),
]


@pytest.mark.parametrize("n,k,p,r,m,rule", CASES)
def test_variant_t_matches_oracle(gpu, n, k, p, r, m, rule):
    print(f"case T n={n} k={k} p={p} r={r} m={m}", flush=True)
    bands, f = synth.make_problem(n, k, m, seed=n + k + r, rule=rule)
    plan = gpu.factor(to_dev(bands), p, r, max_nrhs=m, variant="t")
    x = plan.solve(to_dev(f)).cpu().numpy()
    lam = plan.solve_adjoint(to_dev(f)).cpu().numpy()
    plan.status()
    ref = oracle.lrspike(bands, f, p, r, variant="t")
    reft = oracle.lrspike(bands, f, p, r, transpose=True, variant="t")
    assert col_rel(x, ref) <= 1e-12
    assert col_rel(lam, reft) <= 1e-12


def test_variant_t_differs_from_full_where_the_tips_couple(gpu):
    """Short weakly dominant partitions: the dropped blocks matter, and the GPU
    follows the truncated system, not the whole one."""
    n, k, p, r = 192, 8, 8, 4  # 24-row partitions: T and LR-SPIKE differ by ~1e-4
    bands, f = synth.make_problem(n, k, 1, seed=3, rule="weak")
    x = gpu.factor(to_dev(bands), p, r, max_nrhs=1, variant="t").solve(to_dev(f)).cpu().numpy()
    ref_t = oracle.lrspike(bands, f, p, r, variant="t")
    ref_full = oracle.lrspike(bands, f, p, r)
    assert col_rel(ref_t, ref_full) > 1e-6
    assert col_rel(x, ref_t) <= 1e-12


@pytest.mark.parametrize("precision", ["fp64_refined", "fp32_refined"])
@pytest.mark.parametrize("n,k,p,r,m", [(3000, 8, 4, 3, 2), (4000, 32, 4, 8, 3), (3000, 16, 6, 16, 1)])
def test_variant_t_preconditions_refinement(gpu, precision, n, k, p, r, m):
    """M_T^{-1} as the preconditioner of iterative refinement (FP64 residual):
    the result is A^{-1} f (within 1e-12 in FP64 factors, 1e-11 in FP32)."""
    print(f"case T-refined {precision} n={n} k={k} p={p} r={r} m={m}", flush=True)
    bands, f = synth.make_problem(n, k, m, seed=9, rule="weak")
    plan = gpu.factor(to_dev(bands), p, r, precision=precision, max_nrhs=m, variant="t")
    x = plan.solve(to_dev(f)).cpu().numpy()
    info = plan.status()
    assert info["refine_iters"] >= 1
    tol = 1e-12 if precision == "fp64_refined" else 1e-11
    assert col_rel(x, oracle.band_solve(bands, f)) <= tol
