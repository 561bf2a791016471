"""Writes the diagonal weight theta of the non-dominant refinement workloads
(k = 32, seed 0, a_ii = theta x off-diagonal row sum):

* c2_nondominant.json (default): n = 2^16, the largest theta on a 0.01 grid
  below 0.20 whose estimated 1-norm condition number lies in [3e5, 3e6];
* c2_nondominant_full.json (--full): n = 2^22, the large workload's shape;
  theta on a 0.005 grid in [0.100, 0.200], evaluated in parallel, the one
  whose estimate lies in [3e5, 3e6] and is closest to 1e6 (log scale).

The estimate is Hager's 1-norm estimator of ||A^{-1}||_1 (with Higham's extra
alternating-sign test vector) times ||A||_1; every solve goes through the CPU
oracle's band Gaussian elimination.  Run from the repository root:
    python tests/golden/make_c2_theta.py [--full]
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle  # noqa: E402
import synth  # noqa: E402

N, K, SEED = 1 << 16, 32, 0


def norm1(bands):
    k = (bands.shape[0] - 1) // 2
    n = bands.shape[1]
    col = np.zeros(n)
    for d in range(-k, k + 1):  # A[i, i+d] = bands[d+k, i] contributes to column i+d
        i = np.arange(max(0, -d), min(n, n - d))
        np.add.at(col, i + d, np.abs(bands[d + k, i]))
    return col.max()


def inv_norm1_estimate(bands):
    n = bands.shape[1]
    x = np.full(n, 1.0 / n)
    est = 0.0
    for it in range(6):
        y = oracle.band_solve(bands, x)
        new = np.abs(y).sum()
        if it > 0 and new <= est:
            break
        est = new
        xi = np.where(y >= 0, 1.0, -1.0)
        z = oracle.band_solve(bands, xi, transpose=True)
        j = int(np.argmax(np.abs(z)))
        if it > 0 and abs(z[j]) <= z @ x:
            break
        x = np.zeros(n)
        x[j] = 1.0
    alt = np.array([(-1.0) ** i * (1.0 + i / (n - 1.0)) for i in range(n)])
    alt_est = 2.0 * np.abs(oracle.band_solve(bands, alt)).sum() / (3.0 * n)
    return max(est, alt_est)


def cond_at(args):
    n, theta = args
    bands = synth.make_band(n, K, seed=SEED, rule="theta", theta=theta)
    cond = norm1(bands) * inv_norm1_estimate(bands)
    print(f"n={n} theta={theta:.3f} cond1~{cond:.3e}", flush=True)
    return theta, cond


def main_full():
    import math
    from multiprocessing import Pool
    n = 1 << 22
    grid = [round(0.100 + 0.005 * i, 3) for i in range(21)]
    with Pool(4) as pool:
        res = pool.map(cond_at, [(n, t) for t in grid])
    ok = [(t, c) for t, c in res if 3e5 <= c <= 3e6]
    if not ok:
        raise SystemExit("no theta on the grid lands in [3e5, 3e6]: " + repr(res))
    theta, cond = min(ok, key=lambda tc: abs(math.log10(tc[1]) - 6.0))
    out = {"n": n, "k": K, "seed": SEED, "rule": "theta", "theta": theta, "cond1_estimate": cond,
           "method": "Hager-Higham 1-norm estimate with oracle band solves",
           "grid": {f"{t:.3f}": c for t, c in res}}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_nondominant_full.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", path, theta, cond)


def main():
    if "--full" in sys.argv:
        return main_full()
    out = None
    for step in range(1, 16):
        theta = round(0.20 - 0.01 * step, 2)
        bands = synth.make_band(N, K, seed=SEED, rule="theta", theta=theta)
        cond = norm1(bands) * inv_norm1_estimate(bands)
        print(f"theta={theta:.2f} cond1~{cond:.3e}", flush=True)
        if 3e5 <= cond <= 3e6:
            out = {"n": N, "k": K, "seed": SEED, "rule": "theta", "theta": theta, "cond1_estimate": cond,
                   "method": "Hager-Higham 1-norm estimate with oracle band solves"}
            break
    if out is None:
        raise SystemExit("no theta on the grid lands in [3e5, 3e6]")
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_nondominant.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", path, out)


if __name__ == "__main__":
    main()
