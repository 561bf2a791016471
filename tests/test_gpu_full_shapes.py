"""Parity at the workloads' real shapes (slow: full-size oracle runs).

* Large workload (n = 2^22, k = 32, p = 1024, 16 right-hand sides, weakly
  dominant): FP64 LR-SPIKE against the oracle's literal LR-SPIKE (R1) at every
  rank of the plan r in {4, 8, 16, 32}, element by element, <= 1e-12; at
  r = k also against the plain solve (R0).  For r < k the truncation must be
  well defined: a rounding perturbation u ||V^T V|| of the Gram matrix turns
  the retained subspace by about u / (2 gap) (gap = the smallest relative
  singular-value gap (sigma_r - sigma_{r+1}) / sigma_1 over all spikes,
  reported by the library), and that turn moves x by at most its size times
  the truncation's own effect (~1e-4 relative at these ranks); a gap above
  1e-4 keeps both sides' rounding of the subspace below 1e-15 of x.
* Refinement at that shape: FP32 factors + FP64 refinement at r = k against
  the extended-precision reference, <= 1e-11; on the non-dominant variant
  (theta from c2_nondominant_full.json, kappa_1 ~ 1e6 at n = 2^22) with
  BiCGStab on FP32 factors when the stored theta exists.
* Batched workload: a seeded 128-system subset of the 4096 systems (their
  own n, k, r, right-hand sides and seeds), factored and solved as one batch
  with autotuned partition counts, each against the oracle's R1 of that
  system with the same p, <= 1e-12.
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

DEV = "cuda:0"
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def rel(a, b):
    a = np.asarray(a).reshape(len(a), -1)
    b = np.asarray(b).reshape(len(b), -1)
    return max(np.linalg.norm(a[:, c] - b[:, c]) / np.linalg.norm(b[:, c]) for c in range(b.shape[1]))


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.fixture(scope="module")
def large():
    bands, f = synth.make_problem(1 << 22, 32, 16, seed=0, rule="weak")
    return bands, f


@pytest.mark.parametrize("r", [4, 8, 16, 32])
def test_large_workload_every_rank(gpu, large, r):
    bands, f = large
    n, k, p, m = 1 << 22, 32, 1024, 16
    print(f"case full n={n} k={k} p={p} r={r} m={m}", flush=True)
    plan = gpu.factor(to_dev(bands), p, r, max_nrhs=m)
    x = plan.solve(to_dev(f)).cpu().numpy()
    info = plan.status()
    ref = oracle.lrspike(bands, f, p, r)
    assert rel(x, ref) <= 1e-12
    if r < k:
        assert info["min_sigma_gap"] > 1e-4
    else:
        assert rel(x, oracle.band_solve(bands, f)) <= 1e-12


def test_large_workload_refined_fp32(gpu, large):
    bands, f = large
    n, k, p, m = 1 << 22, 32, 1024, 16
    print(f"case full refined n={n} k={k} p={p} r={k} m={m}", flush=True)
    plan = gpu.factor(to_dev(bands), p, k, precision="fp32_refined", max_nrhs=m)
    x = plan.solve(to_dev(f)).cpu().numpy()
    info = plan.status()
    assert info["refine_iters"] >= 1
    assert rel(x, oracle.band_solve_refined(bands, f, steps=2)) <= 1e-11


def test_large_workload_nondominant(gpu):
    path = os.path.join(GOLD, "c2_nondominant_full.json")
    if not os.path.exists(path):
        pytest.skip("c2_nondominant_full.json not written (tests/golden/make_c2_theta.py --full)")
    meta = json.load(open(path))
    n, k, p, m = meta["n"], meta["k"], 1024, 4
    print(f"case full nondominant theta={meta['theta']} n={n} k={k} p={p} m={m}", flush=True)
    bands, f = synth.make_problem(n, k, m, seed=meta["seed"], rule="theta", theta=meta["theta"])
    ref = oracle.band_solve_refined(bands, f, steps=3)
    for precision, r in (("fp32_bicgstab", k), ("fp64_bicgstab", 8)):
        plan = gpu.factor(to_dev(bands), p, r, precision=precision, max_nrhs=m, max_refine=200)
        x = plan.solve(to_dev(f)).cpu().numpy()
        plan.status()
        assert rel(x, ref) <= 1e-11, precision


def test_batched_subset_of_the_4096_systems(gpu):
    systems = synth.batched_systems(4096, seed=0)
    pick = sorted(np.random.default_rng(7).choice(len(systems), size=128, replace=False).tolist())
    bl, fl = [], []
    for s in pick:
        n, k, r, m, seed = systems[s]
        b, f = synth.make_problem(n, k, m, seed=list(seed), rule="strict")
        bl.append(b)
        fl.append(f)
    bands, rhs, descs = gpu.pack_systems(bl, fl)
    print(f"case batched subset of {len(descs)} systems", flush=True)
    plan = gpu.factor_batched(descs, to_dev(bands))
    x = plan.solve(to_dev(rhs)).cpu().numpy()
    plan.status()
    parts = plan.partitions()
    for i, d in enumerate(descs):
        n, k, _, r, m, _, ro = d
        xs = x[ro:ro + n * m].reshape(n, m)
        ref = oracle.lrspike(bl[i], fl[i], parts[i], r)
        assert rel(xs, ref) <= 1e-12, (i, pick[i], n, k, parts[i])
