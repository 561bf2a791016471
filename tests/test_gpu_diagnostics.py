"""Failure detection and diagnostics reported by lrspike_status.

* Non-finite band entries latch NONFINITE (code 4) with the partition and the
  row of the pivot they reach, on every factorization path: K < 16
  (interchanging kernel), K = 16 and 32 (single-wave kernel, then the
  interchanging one), K = 64 (LDS-resident kernel).  A non-finite coupling
  entry (outside every A_j) reaches the reduced system and latches there.
* min_sigma_gap equals (sigma_r - sigma_{r+1}) / sigma_1 of the oracle's thin
  SVD of the spikes, minimised over the spikes that exist.
* min_pivot / max_abs_entry / reduced_growth are finite and sensible.
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


@pytest.mark.parametrize("k", [4, 16, 32, 64])
@pytest.mark.parametrize("bad", [float("nan"), float("inf")])
def test_nonfinite_band_entry_is_latched(gpu, k, bad):
    n, p = 3000, 3
    print(f"case nonfinite k={k} value={bad}", flush=True)
    bands, _ = synth.make_problem(n, k, 1, seed=k, rule="strict")
    row = 1500  # partition 1 holds rows 1000..1999
    bands[k, row] = bad
    plan = gpu.factor(to_dev(bands), p, k // 2, max_nrhs=1)
    with pytest.raises(gpu.LRSpikeError) as e:
        plan.status()
    assert e.value.code == 4
    assert e.value.info["partition"] == 1
    assert 0 <= e.value.info["row"] <= row - 1000


@pytest.mark.parametrize("k", [4, 32])
def test_nonfinite_coupling_entry_reaches_reduced_system(gpu, k):
    """A NaN in B_0 (row s_1 - 1, column s_1: outside A_0 and A_1) enters only
    the spike V_0, hence the reduced system: NONFINITE at interface 0."""
    n, p = 2000, 2
    bands, _ = synth.make_problem(n, k, 1, seed=1, rule="strict")
    s1 = n // p
    bands[k + 1, s1 - 1] = np.nan  # A[s1 - 1, s1]
    for r in (k, k // 2):
        plan = gpu.factor(to_dev(bands), p, r, max_nrhs=1)
        with pytest.raises(gpu.LRSpikeError) as e:
            plan.status()
        assert e.value.code == 4
        assert e.value.info["partition"] == 0


def test_nonfinite_rhs_in_refined_solve_is_latched(gpu):
    bands, f = synth.make_problem(1000, 4, 2, seed=3, rule="strict")
    f[10, 1] = np.nan
    plan = gpu.factor(to_dev(bands), 4, 2, precision="fp64_refined", max_nrhs=2)
    plan.solve(to_dev(f))
    with pytest.raises(gpu.LRSpikeError) as e:
        plan.status()
    assert e.value.code == 4


@pytest.mark.parametrize("n,k,p,r,rule", [(4096, 8, 4, 3, "strict"), (4000, 32, 4, 8, "weak"),
                                          (3000, 16, 6, 5, "weak"), (4000, 64, 4, 16, "strict")])
def test_sigma_gap_matches_oracle(gpu, n, k, p, r, rule):
    bands, f = synth.make_problem(n, k, 1, seed=n + r, rule=rule)
    plan = gpu.factor(to_dev(bands), p, r, max_nrhs=1)
    info = plan.status()
    _, sv = oracle.lrspike(bands, f, p, r, return_sv=True)
    gaps = []
    for j in range(p):
        for which in (0, 1):  # V (exists for j < p-1), W (exists for j >= 1)
            if (which == 0 and j == p - 1) or (which == 1 and j == 0):
                continue
            s = sv[j, which]
            gaps.append((s[r - 1] - s[r]) / s[0])
    ref = min(gaps)
    assert abs(info["min_sigma_gap"] - ref) <= 1e-6 * ref
    # the truncation is well defined: the gap is far above rounding level
    assert info["min_sigma_gap"] > 1e-4


def test_pivot_and_growth_diagnostics(gpu):
    n, k, p = 4096, 8, 4
    bands, _ = synth.make_problem(n, k, 1, seed=0, rule="strict")
    info = gpu.factor(to_dev(bands), p, 4, max_nrhs=1).status()
    # the largest entry is a diagonal one; elimination keeps the row
    # dominance margin a_ii - sum_j |a_ij| >= 1 of this matrix, so every pivot is >= 1
    assert info["max_abs_entry"] == np.max(np.abs(bands))
    assert info["min_pivot"] >= 1.0
    assert 0 < info["reduced_growth"] < 10
    assert info["min_sigma_gap"] > 0
    exact = gpu.factor(to_dev(bands), p, k, max_nrhs=1).status()
    assert exact["min_sigma_gap"] == float("inf")  # nothing truncated at r = k
