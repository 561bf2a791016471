"""LR-SPIKE-I and LR-SPIKE-OTF on the GPU through the C ABI, against the oracle.

Table solver-list: LR-SPIKE-I solves S~_red (the spikes' rank-r tips) and
LR-SPIKE-OTF the true reduced system S_red (eq. spikered), both by BiCGStab
right-preconditioned by the LR-SPIKE-T system S~~_red, followed by the
recovery of eqs. recovery1/2.  At convergence LR-SPIKE-I gives the direct
LR-SPIKE result (R1) and LR-SPIKE-OTF gives A^{-1} f for any r; the inner
tolerance is 1e-14 on the reduced residual, so the tips carry about
kappa(S) 1e-14 and the bound is 1e-12 (10x the oracle's own forward error
where A is ill-conditioned).  Cases span every kernel width (K = 4 .. 64),
short partitions (far tips that LR-SPIKE-T drops), ragged partitions,
several column chunks and partitions factored with interchanges.
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


CASES_I = [  # n, k, p, r, m, rule, theta
    (180, 8, 4, 3, 2, "weak", 1.05),
    (200, 8, 4, 3, 1, "theta", 0.3),
    (1000, 3, 5, 2, 3, "weak", 1.05),
    (700, 16, 5, 6, 17, "weak", 1.05),
    (1300, 32, 5, 8, 2, "weak", 1.05),
    (2600, 50, 4, 10, 3, "strict", 1.05),
]


@pytest.mark.parametrize("n,k,p,r,m,rule,theta", CASES_I)
def test_lri_matches_direct_lrspike(gpu, n, k, p, r, m, rule, theta):
    print(f"case I n={n} k={k} p={p} r={r} m={m} {rule}", flush=True)
    bands, f = synth.make_problem(n, k, m, seed=n + k, rule=rule, theta=theta)
    plan = gpu.factor(to_dev(bands), p, r, max_nrhs=m, variant="i", refine_tol=1e-14, max_refine=100)
    x = plan.solve(to_dev(f)).cpu().numpy()
    plan.status()
    ref = oracle.lrspike(bands, f, p, r)
    e0 = col_rel(oracle.band_solve(bands, f), oracle.band_solve_refined(bands, f))
    assert col_rel(x, ref) <= max(1e-12, 10 * e0)


CASES_OTF = [  # n, k, p, r, m, rule, theta
    (200, 8, 4, 3, 2, "theta", 0.3),
    (1200, 4, 3, 1, 1, "theta", 0.3),
    (4000, 16, 4, 4, 3, "weak", 1.05),
    (1200, 16, 3, 4, 2, "theta", 0.3),
    (3001, 32, 6, 8, 17, "weak", 1.05),
    (2400, 32, 3, 8, 2, "theta", 0.15),
    (2600, 50, 4, 10, 2, "strict", 1.05),
]


@pytest.mark.parametrize("n,k,p,r,m,rule,theta", CASES_OTF)
def test_otf_reaches_the_exact_solve(gpu, n, k, p, r, m, rule, theta):
    print(f"case OTF n={n} k={k} p={p} r={r} m={m} {rule}", flush=True)
    bands, f = synth.make_problem(n, k, m, seed=n + 2 * k, rule=rule, theta=theta)
    plan = gpu.factor(to_dev(bands), p, r, max_nrhs=m, variant="otf", refine_tol=1e-14, max_refine=200)
    x = plan.solve(to_dev(f)).cpu().numpy()
    info = plan.status()
    assert info["refine_iters"] >= 1
    ref = oracle.band_solve_refined(bands, f)
    e0 = col_rel(oracle.band_solve(bands, f), ref)
    assert col_rel(x, ref) <= max(1e-12, 10 * e0)
    # the oracle's own OTF converges to the same answer
    xo, _, _ = oracle.lrspike_iter(bands, f, p, r, "otf", tol=1e-14, max_it=200)
    assert col_rel(xo, ref) <= max(1e-12, 10 * e0)


def test_iterative_variants_refuse_the_adjoint_and_report_non_convergence(gpu):
    bands, f = synth.make_problem(1200, 16, 1, seed=3, rule="theta", theta=0.3)
    plan = gpu.factor(to_dev(bands), 3, 4, max_nrhs=1, variant="otf", refine_tol=1e-14, max_refine=200)
    with pytest.raises(gpu.LRSpikeError) as e:
        plan.solve_adjoint(to_dev(f))
    assert e.value.code == 6
    # one inner iteration cannot reach 1e-14 here: NOT_CONVERGED is latched
    plan2 = gpu.factor(to_dev(bands), 3, 4, max_nrhs=1, variant="otf", refine_tol=1e-14, max_refine=1)
    plan2.solve(to_dev(f))
    with pytest.raises(gpu.LRSpikeError) as e:
        plan2.status()
    assert e.value.code == 3
