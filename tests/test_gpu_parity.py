"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerances: plain FP64 rel.err <= 1e-12 against R0 (r = k) or R1 (r < k);
FP32 factors with FP64 refinement <= 1e-11 against R0.  rel.err is the max
over right-hand-side columns of ||x_c - ref_c||_2 / ||ref_c||_2.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def rel(a, b):
    a = np.asarray(a).reshape(len(a), -1)
    b = np.asarray(b).reshape(len(b), -1)
    return max(np.linalg.norm(a[:, c] - b[:, c]) / np.linalg.norm(b[:, c]) for c in range(b.shape[1]))


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def run(lr, bands, f, p, r, precision="fp64", adjoint=False):
    print(f"case n={bands.shape[1]} k={(bands.shape[0]-1)//2} p={p} r={r} m={f.shape[1] if f.ndim > 1 else 1} "
          f"{precision} adjoint={adjoint}", flush=True)
    tb = to_dev(bands)
    plan = lr.factor(tb, p, r, precision=precision, max_nrhs=max(1, f.shape[1] if f.ndim > 1 else 1))
    tf = to_dev(f)
    x = plan.solve_adjoint(tf) if adjoint else plan.solve(tf)
    info = plan.status()
    return x.cpu().numpy(), info


CASES = [
    # n, k, p, r, m, rule
    (4096, 8, 4, 8, 1, "strict"),      # the small exact workload
    (4096, 8, 4, 0, 1, "strict"),
    (4096, 8, 4, 3, 2, "strict"),
    (1000, 3, 7, 3, 3, "strict"),      # k padded to 4, ragged partitions
    (999, 5, 4, 2, 2, "weak"),         # k padded to 8, r < k
    (777, 1, 5, 1, 1, "strict"),       # tridiagonal
    (1500, 16, 3, 16, 33, "weak"),     # two column chunks
    (2000, 32, 4, 32, 5, "weak"),
    (2000, 32, 4, 8, 2, "weak"),
    (300, 2, 1, 2, 1, "strict"),       # p = 1: the base solver
    (64 * 9 + 5, 4, 9, 2, 4, "weak"),
    (128, 8, 2, 8, 1, "strict"),       # p = 2: the 2x2 kernel
    (100, 4, 12, 4, 1, "strict"),      # smallest partitions (n_j = 8 = 2k)
]


@pytest.mark.parametrize("n,k,p,r,m,rule", CASES)
def test_solve_matches_oracle(gpu, n, k, p, r, m, rule):
    bands, f = synth.make_problem(n, k, m, seed=n + k + p + r, rule=rule)
    x, info = run(gpu, bands, f, p, r)
    ref = oracle.lrspike(bands, f, p, r)
    assert rel(x, ref) <= 1e-12
    if r == k:
        assert rel(x, oracle.band_solve(bands, f)) <= 1e-12


@pytest.mark.parametrize("n,k,p,r,m,rule", [c for c in CASES if c[0] <= 2000][:9])
def test_adjoint_matches_oracle(gpu, n, k, p, r, m, rule):
    bands, f = synth.make_problem(n, k, m, seed=7 * n + k, rule=rule)
    x, _ = run(gpu, bands, f, p, r, adjoint=True)
    ref = oracle.lrspike(bands, f, p, r, transpose=True)
    assert rel(x, ref) <= 1e-12


@pytest.mark.parametrize("k,theta", [(4, 0.3), (4, 0.15), (16, 0.3), (32, 0.15), (32, 0.1)])
def test_pivoting_nondominant(gpu, k, theta):
    """Non-dominant matrices make the partition LUs interchange rows (for
    k >= 16 every partition leaves the no-interchange kernel for the general one)."""
    n, p, m = 1200 if k <= 16 else 2400, 3, 2
    bands, f = synth.make_problem(n, k, m, seed=3, rule="theta", theta=theta)
    x, info = run(gpu, bands, f, p, k)
    assert info["swapped_blocks"] > 0
    ref = oracle.band_solve_refined(bands, f, steps=2)
    x0 = oracle.band_solve(bands, f)
    # two backward-stable FP64 solves differ by ~kappa u; allow the GPU 10x the oracle's own error
    tol = max(1e-12, 10 * rel(x0, ref))
    assert rel(x, ref) <= tol
    # the adjoint by the same rule, against the transposed extended-precision reference
    xa, _ = run(gpu, bands, f, p, k, adjoint=True)
    refa = oracle.band_solve_refined(bands, f, steps=2, transpose=True)
    x0a = oracle.band_solve(bands, f, transpose=True)
    assert rel(xa, refa) <= max(1e-12, 10 * rel(x0a, refa))


@pytest.mark.parametrize("n,k,p,r,m,rule", [
    (4096, 8, 4, 8, 2, "strict"),
    (2000, 32, 4, 32, 3, "weak"),
    (2000, 32, 4, 8, 3, "weak"),
    (999, 5, 4, 2, 2, "weak"),
])
def test_fp32_refined_matches_exact(gpu, n, k, p, r, m, rule):
    bands, f = synth.make_problem(n, k, m, seed=11, rule=rule)
    x, info = run(gpu, bands, f, p, r, precision="fp32_refined")
    assert info["refine_iters"] >= 1
    assert rel(x, oracle.band_solve_refined(bands, f)) <= 1e-11


def test_fp32_refined_adjoint(gpu):
    bands, f = synth.make_problem(2000, 16, 2, seed=5, rule="weak")
    x, _ = run(gpu, bands, f, 4, 8, precision="fp32_refined", adjoint=True)
    assert rel(x, oracle.band_solve(bands, f, transpose=True)) <= 1e-11


def test_band_grad_matches_oracle(gpu):
    n, k, m = 700, 3, 2
    bands, f = synth.make_problem(n, k, m, seed=2)
    rng = np.random.default_rng(0)
    lam = rng.standard_normal((n, m))
    x = rng.standard_normal((n, m))
    plan = gpu.factor(to_dev(bands), 2, k, max_nrhs=m)
    g = plan.band_grad(to_dev(lam), to_dev(x)).cpu().numpy()
    assert np.max(np.abs(g - oracle.band_grad(lam, x, k))) <= 1e-13 * np.max(np.abs(g))


def test_zero_pivot_is_latched(gpu):
    n, k, p = 400, 4, 2
    bands, f = synth.make_problem(n, k, 1, seed=1)
    row = 300  # a zero row inside partition 1 makes A_1 singular
    for d in range(-k, k + 1):
        bands[d + k, row] = 0.0
    plan = gpu.factor(to_dev(bands), p, k, max_nrhs=1)
    with pytest.raises(gpu.LRSpikeError) as e:
        plan.status()
    assert e.value.code == 1
    assert e.value.info["partition"] == 1


def test_rejects_host_and_bad_arguments(gpu):
    bands, _ = synth.make_problem(100, 4, 1)
    with pytest.raises(TypeError):
        gpu.factor(torch.from_numpy(bands), 2, 4)
    tb = to_dev(bands)
    with pytest.raises(gpu.LRSpikeError):
        gpu.factor(tb, 20, 4)  # n_j = 5 < 2k
    with pytest.raises(gpu.LRSpikeError):
        gpu.factor(tb, 2, 5)  # r > k


def test_repeat_solves_reuse_factorization(gpu):
    bands, f = synth.make_problem(3000, 8, 4, seed=4, rule="weak")
    plan = gpu.factor(to_dev(bands), 6, 4, max_nrhs=4)
    ref = oracle.lrspike(bands, f, 6, 4)
    x1 = plan.solve(to_dev(f)).cpu().numpy()
    x2 = plan.solve(to_dev(f)).cpu().numpy()
    assert rel(x1, ref) <= 1e-12
    assert np.array_equal(x1, x2)  # deterministic


def test_mixed_interchange_partitions(gpu):
    """Only partition 2 is non-dominant: it alone is refactored with
    interchanges while the others keep the no-interchange factorization."""
    n, k, p, m = 4096, 32, 4, 3
    bands, f = synth.make_problem(n, k, m, seed=8, rule="weak")
    lo, hi = 2 * n // p, 3 * n // p
    off = np.abs(bands[:, lo:hi]).sum(axis=0) - np.abs(bands[k, lo:hi])
    bands[k, lo:hi] = 0.1 * off
    for r in (k, 8):
        x, info = run(gpu, bands, f, p, r)
        assert info["swapped_blocks"] > 0
        ref = oracle.lrspike(bands, f, p, r)
        print(f"mixed interchange r={r}: rel {rel(x, ref):.2e}", flush=True)
        assert rel(x, ref) <= 1e-12


def _c2_problem(m):
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "c2_nondominant.json")) as fh:
        c2 = json.load(fh)
    bands, f = synth.make_problem(c2["n"], c2["k"], m, seed=c2["seed"], rule="theta", theta=c2["theta"])
    return bands, f


@pytest.mark.parametrize("r", [32, 28])
def test_refined_nondominant_cond_1e6(gpu, r):
    """FP32 factors + FP64 refinement on the non-dominant workload (condition
    number ~3e5..3e6, theta from tests/golden/c2_nondominant.json) reach the
    extended-precision reference within 1e-11."""
    bands, f = _c2_problem(4)
    x, info = run(gpu, bands, f, 16, r, precision="fp32_refined")
    assert info["refine_iters"] >= 1
    assert info["swapped_blocks"] > 0
    assert rel(x, oracle.band_solve_refined(bands, f, steps=2)) <= 1e-11


def test_refined_nondominant_low_rank_reports_failure(gpu):
    """At r = 8 the truncated spikes of the non-dominant workload do not make a
    contractive preconditioner: the refinement must stop and latch
    NOT_CONVERGED rather than return a wrong answer silently."""
    bands, f = _c2_problem(2)
    plan = gpu.factor(to_dev(bands), 16, 8, precision="fp32_refined", max_nrhs=2)
    plan.solve(to_dev(f))
    with pytest.raises(gpu.LRSpikeError) as e:
        plan.status()
    assert e.value.code == 3
    assert e.value.info["last_correction"] > 1e-6


def _batch(count, seed, ks=(4, 16, 32), nmax=3000, mmax=6):
    """count systems of the batched workload's kind: k drawn from ks, n up to nmax, 1..mmax right-hand sides."""
    rng = np.random.default_rng(seed)
    bl, fl = [], []
    for s in range(count):
        k = int(rng.choice(ks))
        n = int(rng.integers(max(8 * k, 100), nmax))
        m = int(rng.integers(1, mmax + 1))
        b, f = synth.make_problem(n, k, m, seed=1000 * seed + s, rule="strict")
        bl.append(b)
        fl.append(f)
    return bl, fl


def _unpack(x, descs):
    return [x[d[6]:d[6] + d[0] * d[4]].reshape(d[0], d[4]) for d in descs]


@pytest.mark.parametrize("precision", ["fp64", "fp32_refined"])
def test_batched_matches_per_system_oracle(gpu, precision):
    """Every system of a batch (mixed k, n, nrhs; p autotuned for most, given
    for some) equals the oracle's LR-SPIKE of that system alone."""
    bl, fl = _batch(18, 1)
    bands, rhs, descs = gpu.pack_systems(bl, fl)
    descs = [(d[0], d[1], (3 if s % 4 == 0 else 0), d[3], d[4], d[5], d[6]) for s, d in enumerate(descs)]
    plan = gpu.factor_batched(descs, to_dev(bands), precision=precision)
    tr = to_dev(rhs)
    plan.solve(tr)
    plan.status()
    ps = plan.partitions()
    assert all(ps[s] == 3 for s in range(0, len(descs), 4))
    for s, xs in enumerate(_unpack(tr.cpu().numpy(), descs)):
        n, k, _, r, m = descs[s][:5]
        if precision == "fp64":
            assert rel(xs, oracle.lrspike(bl[s], fl[s], ps[s], r)) <= 1e-12, s
        else:
            assert rel(xs, oracle.band_solve_refined(bl[s], fl[s])) <= 1e-11, s


def test_batched_refinement_stops_per_system(gpu):
    """FP32 factors + FP64 refinement in a batch whose systems share one group
    but differ in scale by 1e6 (one band scaled up, so its solution is 1e6
    smaller): the stopping rule holds per (system, column), so the small
    solution reaches the same relative accuracy as its group-mates."""
    bl, fl = _batch(6, 3, ks=(16,), nmax=2500, mmax=3)
    bl[2] = bl[2] * 1e6
    bands, rhs, descs = gpu.pack_systems(bl, fl)
    plan = gpu.factor_batched(descs, to_dev(bands), precision="fp32_refined")
    tr = to_dev(rhs)
    plan.solve(tr)
    plan.status()
    for s, xs in enumerate(_unpack(tr.cpu().numpy(), descs)):
        assert rel(xs, oracle.band_solve_refined(bl[s], fl[s])) <= 1e-11, s


def test_batched_graph_replays_match_eager(gpu):
    """One HIP graph (factor + solve of every system) replayed several times,
    with eager solves and synchronizations in between, reproduces the eager
    result bit for bit each time."""
    bl, fl = _batch(10, 2)
    bands, rhs, descs = gpu.pack_systems(bl, fl)
    plan = gpu.factor_batched(descs, to_dev(bands))
    eager = to_dev(rhs)
    plan.solve(eager)
    plan.status()
    ref = eager.cpu().numpy()
    tr = to_dev(rhs)
    for rep in range(4):
        tr.copy_(to_dev(rhs))
        plan.run(tr)
        other = to_dev(rhs)
        plan.solve(other)
        torch.cuda.synchronize()
        plan.status()
        assert np.array_equal(tr.cpu().numpy(), ref), rep
        assert np.array_equal(other.cpu().numpy(), ref), rep
    for s, xs in enumerate(_unpack(ref, descs)):
        assert rel(xs, oracle.lrspike(bl[s], fl[s], plan.partitions()[s], descs[s][3])) <= 1e-12


def test_batched_rejects_bad_descriptors(gpu):
    b, f = synth.make_problem(500, 4, 1, seed=0)
    tb = to_dev(b.ravel())
    with pytest.raises(gpu.LRSpikeError) as e:
        gpu.factor_batched([(500, 4, 0, 5, 1, 0, 0)], tb)  # r > k
    assert e.value.code == -2
    with pytest.raises(gpu.LRSpikeError) as e:
        gpu.factor_batched([(500, 4, 100, 2, 1, 0, 0)], tb)  # n / p < 2k
    assert e.value.code == -2


def test_gradient_workload_full_size(gpu):
    """The gradient workload's shape (n = 2^20, k = 16, p = 256, r = 8, one
    right-hand side): forward and adjoint solves against the oracle, and the
    dot-product identity <M^{-1} f, g> = <f, M^{-T} g> at scale."""
    n, k, p, r = 1 << 20, 16, 256, 8
    bands, f = synth.make_problem(n, k, 1, seed=0, rule="strict")
    g = np.random.default_rng(1).standard_normal((n, 1))
    tb = to_dev(bands)
    plan = gpu.factor(tb, p, r, max_nrhs=1)
    x = plan.solve(to_dev(f)).cpu().numpy()
    lam = plan.solve_adjoint(to_dev(g)).cpu().numpy()
    plan.status()
    assert rel(x, oracle.lrspike(bands, f, p, r)) <= 1e-12
    assert rel(lam, oracle.lrspike(bands, g, p, r, transpose=True)) <= 1e-12
    lhs, rhs_ = float(x[:, 0] @ g[:, 0]), float(f[:, 0] @ lam[:, 0])
    assert abs(lhs - rhs_) <= 1e-13 * (np.linalg.norm(x) * np.linalg.norm(g))


@pytest.mark.parametrize("n,k,p,r", [(1, 1, 1, 1), (2, 1, 1, 0), (16, 8, 1, 8), (8, 4, 1, 2)])
def test_tiny_systems(gpu, n, k, p, r):
    """Degenerate sizes: a 1 x 1 system, n = K with a single partition."""
    bands, f = synth.make_problem(n, k, 2, seed=n + k, rule="strict")
    x, _ = run(gpu, bands, f, p, r)
    assert rel(x, oracle.band_solve(bands, f)) <= 1e-12


@pytest.mark.parametrize("n,k,p,r,m", [
    (4000, 64, 4, 32, 3),    # K = 64 with the Gram eigensolver and back-sweeps
    (4000, 64, 5, 8, 2),
    (2600, 50, 4, 25, 5),    # k padded to 64
    (1000, 64, 1, 64, 2),    # a single partition: the exact band solve
    (1200, 40, 2, 20, 1),    # padded, p = 2
    (2000, 64, 3, 16, 20),   # two column chunks (the second ragged)
])
def test_k64_matches_oracle(gpu, n, k, p, r, m):
    bands, f = synth.make_problem(n, k, m, seed=n + k, rule="strict")
    x, _ = run(gpu, bands, f, p, r)
    assert rel(x, oracle.lrspike(bands, f, p, r)) <= 1e-12
    xa, _ = run(gpu, bands, f, p, r, adjoint=True)
    assert rel(xa, oracle.lrspike(bands, f, p, r, transpose=True)) <= 1e-12


def test_k64_refined(gpu):
    bands, f = synth.make_problem(4000, 64, 2, seed=9, rule="strict")
    x, info = run(gpu, bands, f, 4, 32, precision="fp32_refined")
    assert info["refine_iters"] >= 1
    assert rel(x, oracle.band_solve_refined(bands, f)) <= 1e-11


def test_k64_interchanges_reported_unsupported(gpu):
    """At K = 64 partitions are factored without interchanges; one that would
    need them latches NOT_SUPPORTED with its partition instead of a wrong result."""
    bands, f = synth.make_problem(3000, 64, 1, seed=4, rule="theta", theta=0.05)
    plan = gpu.factor(to_dev(bands), 3, 16, max_nrhs=1)
    with pytest.raises(gpu.LRSpikeError) as e:
        plan.status()
    assert e.value.code == 6
    assert 0 <= e.value.info["partition"] < 3


def test_k64_zero_pivot_is_latched(gpu):
    """A zero row makes A_1 singular: the K = 64 factor reaches an exact zero
    pivot at that row and latches ZERO_PIVOT with the partition-local row."""
    n, k, p = 3000, 64, 3
    bands, f = synth.make_problem(n, k, 1, seed=2, rule="strict")
    row = 1500  # partition 1 holds rows 1000..1999
    for d in range(-k, k + 1):
        bands[d + k, row] = 0.0
    plan = gpu.factor(to_dev(bands), p, 32, max_nrhs=1)
    with pytest.raises(gpu.LRSpikeError) as e:
        plan.status()
    assert e.value.code == 1
    assert e.value.info["partition"] == 1
    assert e.value.info["row"] == row - 1000


def test_batched_many_rhs(gpu):
    """Up to 32 right-hand sides per system: several column chunks in every sweep kind."""
    bl, fl = _batch(8, 7, ks=(4, 16, 32, 64), nmax=4000, mmax=32)
    bands, rhs, descs = gpu.pack_systems(bl, fl)
    assert max(d[4] for d in descs) > 16
    plan = gpu.factor_batched(descs, to_dev(bands))
    tr = to_dev(rhs)
    plan.run(tr)
    plan.status()
    for s, xs in enumerate(_unpack(tr.cpu().numpy(), descs)):
        assert rel(xs, oracle.lrspike(bl[s], fl[s], plan.partitions()[s], descs[s][3])) <= 1e-12, s


def test_batched_with_k64_systems(gpu):
    bl, fl = _batch(9, 3, ks=(4, 16, 64), nmax=6000)
    bands, rhs, descs = gpu.pack_systems(bl, fl)
    assert any(d[1] == 64 for d in descs)
    plan = gpu.factor_batched(descs, to_dev(bands))
    tr = to_dev(rhs)
    plan.run(tr)
    plan.status()
    for s, xs in enumerate(_unpack(tr.cpu().numpy(), descs)):
        assert rel(xs, oracle.lrspike(bl[s], fl[s], plan.partitions()[s], descs[s][3])) <= 1e-12, s
