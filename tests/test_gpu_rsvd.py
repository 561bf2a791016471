"""Randomized spike SVD on the GPU through the C ABI, against the oracle.

The spikes are truncated through the randomized SVD of section "SVD
representation of the spikes" (the Halko-Martinsson-Tropp proto-algorithm:
ell = r + oversampling sketch columns, q power steps), with the same seeded
Gaussian test matrices on both sides.  The oracle forms the explicit spike,
its sketch and a Householder QR; the GPU sketches by block solves with 2 ell
right-hand sides and adjoint solves, and orthonormalizes through the sketch's
Gram (pivoted Cholesky).  The two bases agree to about eps * kappa(Y)^2, and a
power step raises kappa(Y) to its cube: parity is relative error <= 1e-12 per
column at q = 0 and <= 1e-10 at q = 1, forward and adjoint, over every kernel
width (K = 4 .. 64), ragged partitions, several column chunks, both reduced
systems and partitions factored with interchanges.  With ell = k the sketch
spans the whole spike and the result is the exact truncation's, up to the
spike directions the Gram cannot resolve (below 1e-6 sigma_1), which the GPU
drops from the basis.
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


CASES = [  # n, k, p, r, ell, q, m, rule, variant
    (1000, 3, 5, 1, 2, 0, 2, "weak", "full"),
    (1203, 8, 7, 4, 6, 0, 1, "weak", "full"),
    (2000, 16, 5, 8, 12, 0, 3, "weak", "full"),
    (2000, 16, 4, 4, 8, 1, 2, "weak", "t"),
    (3001, 32, 6, 8, 16, 0, 17, "weak", "full"),
    (3001, 32, 6, 8, 12, 1, 2, "strict", "full"),
    (2600, 50, 4, 10, 20, 0, 5, "strict", "full"),
    (4000, 64, 5, 16, 24, 0, 3, "strict", "t"),
]


@pytest.mark.parametrize("n,k,p,r,ell,q,m,rule,variant", CASES)
def test_rsvd_matches_oracle(gpu, n, k, p, r, ell, q, m, rule, variant):
    print(f"case rsvd n={n} k={k} p={p} r={r} ell={ell} q={q} m={m} {variant}", flush=True)
    bands, f = synth.make_problem(n, k, m, seed=n + k + r, rule=rule)
    om = synth.gaussian_test_matrices(p, k, ell, seed=n)
    plan = gpu.factor(to_dev(bands), p, r, max_nrhs=m, variant=variant, svd="randomized", rsvd_ell=ell,
                      rsvd_power=q, rsvd_omega=to_dev(om))
    x = plan.solve(to_dev(f)).cpu().numpy()
    lam = plan.solve_adjoint(to_dev(f)).cpu().numpy()
    plan.status()
    ref = oracle.lrspike_rsvd(bands, f, p, r, om, q=q, variant=variant)
    reft = oracle.lrspike_rsvd(bands, f, p, r, om, q=q, variant=variant, transpose=True)
    tol = 1e-12 if q == 0 else 1e-10
    assert col_rel(x, ref) <= tol
    assert col_rel(lam, reft) <= tol


def test_rsvd_differs_from_the_exact_truncation(gpu):
    """r < ell < k: the sketched truncation is not the exact one (the oracle's
    exact and randomized results differ far above the parity tolerance) and
    the GPU follows the randomized one."""
    n, k, p, r, ell, m = 3000, 16, 5, 4, 6, 2
    bands, f = synth.make_problem(n, k, m, seed=5, rule="weak")
    om = synth.gaussian_test_matrices(p, k, ell, seed=6)
    plan = gpu.factor(to_dev(bands), p, r, max_nrhs=m, svd="randomized", rsvd_ell=ell, rsvd_omega=to_dev(om))
    x = plan.solve(to_dev(f)).cpu().numpy()
    plan.status()
    ref = oracle.lrspike_rsvd(bands, f, p, r, om)
    exact = oracle.lrspike(bands, f, p, r)
    assert col_rel(ref, exact) > 1e-6
    assert col_rel(x, ref) <= 1e-12


def test_rsvd_full_sketch_is_the_exact_truncation(gpu):
    """ell = k: the sketch spans the whole spike and the result is the exact
    truncation's, except for spike directions below the resolution of the
    Gram-based orthonormalization (singular values under 1e-6 sigma_1 are
    dropped from the basis): the deviation is bounded by ten times the
    largest such relative singular value (here about 2e-7)."""
    n, k, p, r, m = 1500, 12, 3, 5, 2
    bands, f = synth.make_problem(n, k, m, seed=8, rule="weak")
    om = synth.gaussian_test_matrices(p, k, k, seed=9)
    plan = gpu.factor(to_dev(bands), p, r, max_nrhs=m, svd="randomized", rsvd_ell=k, rsvd_omega=to_dev(om))
    x = plan.solve(to_dev(f)).cpu().numpy()
    plan.status()
    exact, sv = oracle.lrspike(bands, f, p, r, return_sv=True)
    rel_sv = sv / np.maximum(sv[:, :, :1], 1e-300)
    below = rel_sv[(rel_sv < 1e-6) & (sv > 0)]
    tol = max(1e-12, 10 * below.max()) if below.size else 1e-12
    assert tol <= 1e-5
    assert col_rel(x, exact) <= tol
    # where every spike direction is resolved (smallest relative singular value
    # s_min >= 1e-6), the Gram-based basis errs by about eps / s_min relative
    bands2, f2 = synth.make_problem(n, 4, m, seed=8, rule="weak")
    om2 = synth.gaussian_test_matrices(p, 4, 4, seed=9)
    ex2, sv2 = oracle.lrspike(bands2, f2, p, 2, return_sv=True)
    smin = (sv2[sv2 > 0] / np.repeat(sv2[:, :, :1], 4, axis=2)[sv2 > 0]).min()
    assert smin > 1e-6
    plan2 = gpu.factor(to_dev(bands2), p, 2, max_nrhs=m, svd="randomized", rsvd_ell=4, rsvd_omega=to_dev(om2))
    x2 = plan2.solve(to_dev(f2)).cpu().numpy()
    plan2.status()
    assert col_rel(x2, ex2) <= max(1e-12, 1e-14 / smin)


@pytest.mark.parametrize("k,theta", [(4, 0.3), (16, 0.3), (32, 0.15)])
def test_rsvd_with_interchanges(gpu, k, theta):
    """Non-dominant bands: partitions factored with row interchanges run their
    sketch solves through the interchanging sweeps.  Two backward-stable FP64
    computations differ by about kappa u: the GPU may differ from the oracle
    by 10x the oracle's own forward error on the plain solve (at least 1e-12)."""
    n, p, r, ell, m = (1200 if k <= 16 else 2400), 3, 2, 3, 2
    bands, f = synth.make_problem(n, k, m, seed=3, rule="theta", theta=theta)
    om = synth.gaussian_test_matrices(p, k, ell, seed=k)
    plan = gpu.factor(to_dev(bands), p, r, max_nrhs=m, svd="randomized", rsvd_ell=ell, rsvd_omega=to_dev(om))
    x = plan.solve(to_dev(f)).cpu().numpy()
    lam = plan.solve_adjoint(to_dev(f)).cpu().numpy()
    info = plan.status()
    assert info["swapped_blocks"] > 0
    ref = oracle.lrspike_rsvd(bands, f, p, r, om)
    reft = oracle.lrspike_rsvd(bands, f, p, r, om, transpose=True)
    e0 = col_rel(oracle.band_solve(bands, f), oracle.band_solve_refined(bands, f, steps=2))
    tol = max(1e-12, 10 * e0)
    assert col_rel(x, ref) <= tol
    assert col_rel(lam, reft) <= tol


def test_rsvd_preconditions_refinement(gpu):
    """As the preconditioner of FP64 refinement the randomized operator still
    reaches A^{-1} f."""
    n, k, p, r, ell, m = 4096, 32, 8, 8, 16, 3
    bands, f = synth.make_problem(n, k, m, seed=3, rule="weak")
    plan = gpu.factor(to_dev(bands), p, r, precision="fp64_refined", max_nrhs=m, svd="randomized",
                      rsvd_ell=ell, rsvd_seed=1)
    x = plan.solve(to_dev(f)).cpu().numpy()
    info = plan.status()
    assert info["refine_iters"] >= 1
    assert col_rel(x, oracle.band_solve(bands, f)) <= 1e-12
