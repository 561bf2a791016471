"""Gradients of the converged solve x = A^{-1} b through the C ABI.

At r < k the autograd path refines the forward solve against A and the
adjoint against A^T (FP64 residual, M_r^{-1} as the preconditioner), so the
returned gradients are those of A^{-1} b: grad_b = lam = A^{-T} dL/dx and
grad_bands = -lam x^T on the band.  They are checked against central finite
differences of the oracle's exact band solve, and at the gradient workload's
shape (n = 2^20, k = 16, p = 256, r = 8) entry by entry against the oracle's
lam = A^{-T}(x - x*) and -lam x^T.
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


def band_mask(n, k):
    mask = np.ones((2 * k + 1, n))
    for d in range(-k, k + 1):
        if d < 0:
            mask[d + k, :-d] = 0
        elif d > 0:
            mask[d + k, n - d:] = 0
    return mask


@pytest.mark.parametrize("r", [4, 2])
def test_autograd_finite_differences(gpu, r):
    """Loss 0.5 ||x - x*||^2 at n = 512, k = 4, p = 4: 8 random band
    directions, 16 single band entries and one direction in b, step 1e-6,
    against the oracle's exact solve, agreement <= 1e-6 relative."""
    n, k, p = 512, 4, 4
    print(f"case fd n={n} k={k} p={p} r={r}", flush=True)
    bands, b = synth.make_problem(n, k, 1, seed=0)
    b = b[:, 0]
    xs = np.random.default_rng(1).standard_normal(n)
    tb = to_dev(bands).requires_grad_(True)
    tbb = to_dev(b).requires_grad_(True)
    x = gpu.solve(tb, tbb, p, r)
    loss = 0.5 * torch.sum((x - to_dev(xs)) ** 2)
    loss.backward()
    gb = tb.grad.cpu().numpy()
    gbb = tbb.grad.cpu().numpy()
    # the forward itself is the exact solve, not the one-shot M_r^{-1} b
    x_ref = oracle.band_solve(bands, b)
    assert np.linalg.norm(x.detach().cpu().numpy() - x_ref) <= 1e-12 * np.linalg.norm(x_ref)

    def L(bd, bb):
        return 0.5 * np.sum((oracle.band_solve(bd, bb) - xs) ** 2)

    rng = np.random.default_rng(2)
    h = 1e-6
    mask = band_mask(n, k)
    dirs = [rng.standard_normal(bands.shape) * mask for _ in range(8)]
    inside = np.argwhere(mask > 0)
    for idx in rng.choice(len(inside), size=16, replace=False):
        e = np.zeros_like(bands)
        e[tuple(inside[idx])] = 1.0
        dirs.append(e)
    for dirn in dirs:
        fd = (L(bands + h * dirn, b) - L(bands - h * dirn, b)) / (2 * h)
        assert abs(fd - np.sum(gb * dirn)) <= 1e-6 * max(1.0, abs(fd))
    db = rng.standard_normal(n)
    fd = (L(bands, b + h * db) - L(bands, b - h * db)) / (2 * h)
    assert abs(fd - np.dot(gbb, db)) <= 1e-6 * max(1.0, abs(fd))


def test_one_shot_fp64_at_low_rank_is_refused_for_autograd(gpu):
    bands, b = synth.make_problem(512, 4, 1, seed=0)
    with pytest.raises(ValueError):
        gpu.solve(to_dev(bands), to_dev(b[:, 0]), 4, 2, precision="fp64")


def test_gradient_workload_against_exact_adjoint(gpu):
    """n = 2^20, k = 16, p = 256, r = 8, one right-hand side (strict
    dominance), loss 0.5 ||x - x*||^2: grad_b and grad_bands entry by entry
    against lam = A^{-T}(x - x*) and -lam x^T from the oracle's band solves,
    within 1e-11 of the largest entry."""
    n, k, p, r = 1 << 20, 16, 256, 8
    print(f"case grad n={n} k={k} p={p} r={r}", flush=True)
    bands, b = synth.make_problem(n, k, 1, seed=0, rule="strict")
    b = b[:, 0]
    xs = np.random.default_rng(1).standard_normal(n)
    tb = to_dev(bands).requires_grad_(True)
    tbb = to_dev(b).requires_grad_(True)
    x = gpu.solve(tb, tbb, p, r)
    loss = 0.5 * torch.sum((x - to_dev(xs)) ** 2)
    loss.backward()
    gb = tb.grad.cpu().numpy()
    gbb = tbb.grad.cpu().numpy()
    x_ref = oracle.band_solve(bands, b)
    lam_ref = oracle.band_solve(bands, x_ref - xs, transpose=True)
    gb_ref = oracle.band_grad(lam_ref, x_ref, k)
    assert np.max(np.abs(x.detach().cpu().numpy() - x_ref)) <= 1e-11 * np.max(np.abs(x_ref))
    assert np.max(np.abs(gbb - lam_ref)) <= 1e-11 * np.max(np.abs(lam_ref))
    assert np.max(np.abs(gb - gb_ref)) <= 1e-11 * np.max(np.abs(gb_ref))


@pytest.mark.parametrize("n,k,p,r,m", [(3000, 8, 4, 3, 2), (4000, 32, 4, 8, 3), (3000, 64, 3, 16, 1)])
def test_fp64_refined_reaches_exact_solve_at_low_rank(gpu, n, k, p, r, m):
    """FP64 factors with M_r^{-1} as preconditioner: the refined solve and
    adjoint equal A^{-1} f and A^{-T} f (weakly dominant, r < k)."""
    print(f"case fp64_refined n={n} k={k} p={p} r={r} m={m}", flush=True)
    bands, f = synth.make_problem(n, k, m, seed=5, rule="weak" if k < 64 else "strict")
    plan = gpu.factor(to_dev(bands), p, r, precision="fp64_refined", max_nrhs=m)
    x = plan.solve(to_dev(f)).cpu().numpy()
    lam = plan.solve_adjoint(to_dev(f)).cpu().numpy()
    info = plan.status()
    assert info["refine_iters"] >= 1
    for got, ref in ((x, oracle.band_solve(bands, f)), (lam, oracle.band_solve(bands, f, transpose=True))):
        err = max(np.linalg.norm(got[:, c] - ref[:, c]) / np.linalg.norm(ref[:, c]) for c in range(m))
        assert err <= 1e-12
