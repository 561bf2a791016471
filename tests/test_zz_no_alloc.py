"""The allocation-free entry point lrspike_solve_noalloc against the
allocating path (lrspike_factor + lrspike_solve with a caller workspace), on
two calls in a row, the second with a smaller problem, so that the second
reads a scratch the first left filled.  Same kernels in the same order: the
results agree to the FP64 parity bound (they are expected to be identical)."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def test_noalloc_matches_the_allocating_entry_points(gpu):
    status = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    for (n, k, p, r, m) in [(20000, 16, 8, 8, 3), (3000, 8, 3, 4, 2)]:
        print(f"case noalloc n={n} k={k} p={p} r={r} m={m}", flush=True)
        bands, f = synth.make_problem(n, k, m, seed=n, rule="weak")
        tb, tf = to_dev(bands), to_dev(f)
        x_na = gpu.solve_noalloc(tb, tf, p, r, status=status)
        plan = gpu.factor(tb, p, r, max_nrhs=m)
        x_ref = plan.solve(tf, check=True)
        torch.cuda.synchronize()
        assert int(status.item()) == 0
        x_na, x_ref = x_na.cpu().numpy(), x_ref.cpu().numpy()
        err = max(np.linalg.norm(x_na[:, c] - x_ref[:, c]) / np.linalg.norm(x_ref[:, c]) for c in range(m))
        assert err <= 1e-12


def test_noalloc_reports_a_zero_pivot_through_status(gpu):
    n, k, p = 3000, 4, 3
    bands, f = synth.make_problem(n, k, 1, seed=2, rule="strict")
    bands[:, 1500] = 0.0  # a zero row inside partition 1
    status = torch.zeros(1, dtype=torch.int32, device=DEV)
    gpu.solve_noalloc(to_dev(bands), to_dev(f), p, 2, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == 1
