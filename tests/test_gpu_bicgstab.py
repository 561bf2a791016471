"""BiCGStab right-preconditioned by LR-SPIKE on the GPU, through the C ABI.

* Iterates: with the tolerance out of reach and max_refine = N the plan stops
  after N iterations (latching NOT_CONVERGED); x then equals the oracle's N-th
  BiCGStab iterate (same recurrence, same x_0 = M^{-1} f), forward and
  adjoint, for both reduced-system variants.  The rounding of the two
  preconditioner applications differs at ~1e-15; over a few iterations of a
  non-dominant system that grows by a few orders, hence 1e-10.
* Convergence: on non-dominant systems where plain refinement diverges
  (I - M^{-1} A is not a contraction at small r), BiCGStab reaches A^{-1} f,
  checked against the oracle's extended-precision reference; the bound is
  the refined-precision target 1e-11 (kappa_1 ~ 3e5 workload) or 1e-10 for
  the smaller, harder case whose rounding floor kappa u is ~1e-11.
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


@pytest.mark.parametrize("n,k,p,r,m,variant", [(1500, 5, 3, 2, 2, "full"), (1500, 5, 3, 2, 1, "t"),
                                               (4000, 32, 4, 8, 3, "full"), (3000, 16, 5, 4, 2, "t")])
@pytest.mark.parametrize("iters", [1, 3])
@pytest.mark.parametrize("adjoint", [False, True])
def test_bicgstab_iterates_match_oracle(gpu, n, k, p, r, m, variant, iters, adjoint):
    print(f"case bicg-iterates n={n} k={k} p={p} r={r} m={m} {variant} it={iters} adj={adjoint}", flush=True)
    bands, f = synth.make_problem(n, k, m, seed=41, rule="theta", theta=0.4)
    plan = gpu.factor(to_dev(bands), p, r, precision="fp64_bicgstab", max_nrhs=m, refine_tol=1e-300,
                      max_refine=iters, variant=variant)
    x = (plan.solve_adjoint if adjoint else plan.solve)(to_dev(f)).cpu().numpy()
    with pytest.raises(gpu.LRSpikeError) as e:
        plan.status()
    assert e.value.code == 3 and e.value.info["refine_iters"] == iters
    ref, its, _ = oracle.bicgstab(bands, f, p, r, tol=0.0, max_it=iters, transpose=adjoint, variant=variant)
    assert its == [iters] * m
    assert col_rel(x, ref) <= 1e-10


@pytest.mark.parametrize("precision", ["fp64_bicgstab", "fp32_bicgstab"])
@pytest.mark.parametrize("variant", ["full", "t"])
def test_bicgstab_converges_where_refinement_diverges(gpu, precision, variant):
    n, k, p, r, m = 4096, 8, 8, 2, 2
    print(f"case bicg-converge {precision} {variant}", flush=True)
    bands, f = synth.make_problem(n, k, m, seed=33, rule="theta", theta=0.15)
    xs = oracle.band_solve_refined(bands, f, steps=3)
    plan = gpu.factor(to_dev(bands), p, r, precision=precision, max_nrhs=m, max_refine=300, variant=variant)
    x = plan.solve(to_dev(f)).cpu().numpy()
    info = plan.status()
    assert 1 <= info["refine_iters"] < 300
    assert col_rel(x, xs) <= 1e-10
    lam = plan.solve_adjoint(to_dev(f)).cpu().numpy()
    plan.status()
    assert col_rel(lam, oracle.band_solve(bands, f, transpose=True)) <= 1e-10
    # the plain refinement on the same preconditioner does not converge here
    ref = gpu.factor(to_dev(bands), p, r, precision="fp64_refined", max_nrhs=m, variant=variant)
    ref.solve(to_dev(f))
    with pytest.raises(gpu.LRSpikeError) as e:
        ref.status()
    assert e.value.code == 3


@pytest.mark.parametrize("precision", ["fp64_bicgstab", "fp32_bicgstab"])
def test_bicgstab_ill_conditioned_workload_at_rank_8(gpu, precision):
    """The ill-conditioned refinement workload (n = 2^16, k = 32, p = 16,
    theta = 0.15, kappa_1 ~ 3.1e5) at r = 8, where refinement latches
    NOT_CONVERGED: BiCGStab reaches the extended-precision reference."""
    import json
    import os
    meta = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "c2_nondominant.json")))
    n, k, p, r, m = meta["n"], meta["k"], 16, 8, 2
    print(f"case bicg-c2 {precision}", flush=True)
    bands, f = synth.make_problem(n, k, m, seed=meta["seed"], rule="theta", theta=meta["theta"])
    xs = oracle.band_solve_refined(bands, f, steps=3)
    plan = gpu.factor(to_dev(bands), p, r, precision=precision, max_nrhs=m, max_refine=200)
    x = plan.solve(to_dev(f)).cpu().numpy()
    info = plan.status()
    assert info["refine_iters"] >= 1
    assert col_rel(x, xs) <= 1e-11


def test_bicgstab_exact_preconditioner(gpu):
    """r = k: M^{-1} = A^{-1}, the initial iterate already solves the system."""
    bands, f = synth.make_problem(3000, 8, 2, seed=32, rule="weak")
    plan = gpu.factor(to_dev(bands), 4, 8, precision="fp64_bicgstab", max_nrhs=2)
    x = plan.solve(to_dev(f)).cpu().numpy()
    info = plan.status()
    assert info["refine_iters"] <= 1
    assert col_rel(x, oracle.band_solve(bands, f)) <= 1e-12


def test_bicgstab_refused_for_batches(gpu):
    bands, f = synth.make_problem(2000, 4, 1, seed=1)
    bb, rh, descs = gpu.pack_systems([bands], [f])
    with pytest.raises(gpu.LRSpikeError) as e:
        gpu.factor_batched(descs, to_dev(bb), precision="fp64_bicgstab")
    assert e.value.code < 0
