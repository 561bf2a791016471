"""Pins of the CPU oracle against facts fixed outside the oracle itself.

Each test names the fact it checks.  A plausible slip in the oracle (dropped
term, wrong sign or index, transposed operand) fails at least one of them:
  * band elimination / solves       -> Thomas, closed forms, scipy's LAPACK band
                                       solver, dense brute force, backward error;
  * spikes                          -> the defining residual A_j V_j = [0; B_j];
  * truncated SVD                   -> numpy's SVD, Eckart-Young;
  * reduced system + recovery       -> exactness at r = k, exactness when the
                                       coupling blocks have rank <= r, the
                                       determinant identity, the p = 2 kernel,
                                       the r = 0 closed form;
  * adjoint                         -> dot-product test, dense transpose;
  * band gradient                   -> central finite differences.
"""
import os

import numpy as np
import pytest
import scipy.linalg

import oracle
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def dense(bands):
    k2, n = bands.shape
    k = (k2 - 1) // 2
    A = np.zeros((n, n))
    for d in range(-k, k + 1):
        for i in range(n):
            if 0 <= i + d < n:
                A[i, i + d] = bands[d + k, i]
    return A


def bands_of(A, k):
    n = A.shape[0]
    b = np.zeros((2 * k + 1, n))
    for d in range(-k, k + 1):
        for i in range(n):
            if 0 <= i + d < n:
                b[d + k, i] = A[i, i + d]
    return b


def thomas(lo, di, up, f):
    """Textbook Thomas recurrence for tridiagonal systems (lo[i] = A[i, i-1], up[i] = A[i, i+1])."""
    n = len(di)
    c = np.zeros(n)
    d = np.zeros(n)
    c[0] = up[0] / di[0]
    d[0] = f[0] / di[0]
    for i in range(1, n):
        den = di[i] - lo[i] * c[i - 1]
        c[i] = up[i] / den if i < n - 1 else 0.0
        d[i] = (f[i] - lo[i] * d[i - 1]) / den
    x = np.zeros(n)
    x[-1] = d[-1]
    for i in range(n - 2, -1, -1):
        x[i] = d[i] - c[i] * x[i + 1]
    return x


def rel(a, b):
    a = np.atleast_2d(np.asarray(a).T).T
    b = np.atleast_2d(np.asarray(b).T).T
    return max(np.linalg.norm(a[:, c] - b[:, c]) / np.linalg.norm(b[:, c]) for c in range(b.shape[1]))


# ---------------------------------------------------------------- R0 pins


def test_p1_thomas_k1():
    bands, f = synth.make_problem(300, 1, 1, seed=3)
    x = oracle.band_solve(bands, f[:, 0])
    xt = thomas(bands[0], bands[1], bands[2], f[:, 0])
    assert rel(x, xt) < 1e-14


def test_p2_golden_poisson_unit_load():
    n = 8
    b = np.zeros((3, n))
    b[0, 1:] = -1.0
    b[1] = 2.0
    b[2, :-1] = -1.0
    x = oracle.band_solve(b, np.ones(n))
    gold = np.loadtxt(os.path.join(GOLD, "tridiag_m1_2_m1_n8_ones.txt"))
    assert np.max(np.abs(x - gold)) < 1e-13


def test_p2_golden_inverse_columns():
    n = 4
    b = np.zeros((3, n))
    b[0, 1:] = -1.0
    b[1] = 2.0
    b[2, :-1] = -1.0
    inv = oracle.band_solve(b, np.eye(n))
    gold = np.loadtxt(os.path.join(GOLD, "tridiag_m1_2_m1_n4_inverse.txt")) / 5.0
    assert np.max(np.abs(inv - gold)) < 1e-14


@pytest.mark.parametrize("a,b", [(3.0, -1.0), (2.5, 0.7)])
def test_p2_toeplitz_eigenvectors(a, b):
    n = 257
    band = np.zeros((3, n))
    band[0, 1:] = b
    band[1] = a
    band[2, :-1] = b
    m = np.arange(1, n + 1)
    for j in (1, 17, 200):
        v = np.sin(j * m * np.pi / (n + 1))
        lam = a + 2 * b * np.cos(j * np.pi / (n + 1))
        x = oracle.band_solve(band, v)
        assert rel(x, v / lam) < 1e-13


@pytest.mark.parametrize("k", [2, 3, 5])
def test_p2_power_of_tridiagonal(k):
    """A = T^k with T = tridiag(-1, 3, -1) has half-bandwidth k; its solve is k Thomas solves."""
    n = 120
    T = 3 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    A = np.linalg.matrix_power(T, k)
    f = np.random.default_rng(k).standard_normal(n)
    y = f.copy()
    lo = np.r_[0.0, -np.ones(n - 1)]
    up = np.r_[-np.ones(n - 1), 0.0]
    for _ in range(k):
        y = thomas(lo, 3 * np.ones(n), up, y)
    x = oracle.band_solve(bands_of(A, k), f)
    assert rel(x, y) < 1e-12


@pytest.mark.parametrize("n,k", [(40, 3), (64, 8), (17, 5)])
def test_p3_dense_bruteforce(n, k):
    bands, f = synth.make_problem(n, k, 3, seed=n + k, rule="theta", theta=0.3)
    A = dense(bands)
    x = oracle.band_solve(bands, f)
    assert rel(x, np.linalg.solve(A, f)) < 1e-11
    xt = oracle.band_solve(bands, f, transpose=True)
    assert rel(xt, np.linalg.solve(A.T, f)) < 1e-11


@pytest.mark.parametrize("rule,theta", [("strict", 0), ("weak", 0), ("theta", 0.2)])
def test_p4_scipy_solve_banded(rule, theta):
    n, k = 3000, 7
    bands, f = synth.make_problem(n, k, 2, seed=11, rule=rule, theta=theta)
    ab = np.zeros_like(bands)
    for d in range(-k, k + 1):  # LAPACK upper-first layout: ab[k - d, i + d] = A[i, i + d]
        for i in range(max(0, -d), min(n, n - d)):
            ab[k - d, i + d] = bands[d + k, i]
    ref = scipy.linalg.solve_banded((k, k), ab, f)
    assert rel(oracle.band_solve(bands, f), ref) < 1e-12


def test_p12_backward_error():
    n, k = 2000, 6
    bands, f = synth.make_problem(n, k, 1, seed=5, rule="theta", theta=0.25)
    x = oracle.band_solve(bands, f)
    r = f - oracle.band_matvec(bands, x)
    A = dense(bands) if n <= 2000 else None
    nrmA = np.abs(A).sum(axis=1).max()
    eta = np.abs(r).max() / (nrmA * np.abs(x).max() + np.abs(f).max())
    assert eta < 8 * (k + 1) * np.finfo(float).eps * 10


def test_refined_reference_exact_on_integer_system():
    """Small-integer band and integer x_true: f = A x_true is exact in double,
    so a solve whose residual is accumulated beyond double precision recovers
    x_true to the last bit, while plain elimination is off by about kappa u
    (kappa_1 ~ 4e5 here).  A residual accumulated in double would leave the
    refined result at the plain one's accuracy."""
    rng = np.random.default_rng(1)
    n, k = 600, 4
    bands = rng.integers(-5, 6, size=(2 * k + 1, n)).astype(float)
    for d in range(-k, k + 1):
        if d < 0:
            bands[d + k, :-d] = 0.0
        elif d > 0:
            bands[d + k, n - d:] = 0.0
    bands[k] = np.round(0.3 * (np.abs(bands).sum(axis=0) - np.abs(bands[k])))
    x_true = rng.integers(-8, 9, size=(n, 2)).astype(float)
    f = dense(bands) @ x_true  # integers well below 2^53: exact
    assert np.array_equal(f, oracle.band_matvec(bands, x_true))
    x0 = oracle.band_solve(bands, f)
    xr = oracle.band_solve_refined(bands, f, steps=3)
    assert rel(x0, x_true) > 1e-14
    assert rel(xr, x_true) <= 2 * np.finfo(float).eps
    # the transposed system: g = A^T x_true, exact in double as well
    g = dense(bands).T @ x_true
    xt0 = oracle.band_solve(bands, g, transpose=True)
    xtr = oracle.band_solve_refined(bands, g, steps=3, transpose=True)
    assert rel(xt0, x_true) > 1e-14
    assert rel(xtr, x_true) <= 2 * np.finfo(float).eps


def test_band_matvec_transpose_is_dense_transpose():
    n, k = 50, 3
    bands, _ = synth.make_problem(n, k, 1, seed=4, rule="theta", theta=0.5)
    x = np.random.default_rng(3).standard_normal((n, 2))
    A = dense(bands)
    assert np.abs(oracle.band_matvec(bands, x) - A @ x).max() < 1e-13
    assert np.abs(oracle.band_matvec(bands, x, transpose=True) - A.T @ x).max() < 1e-13


def test_refined_reference_beats_plain_on_hard_matrix():
    """The long-double-residual reference reaches ~u forward error; check it by
    solving a problem whose exact answer is known (f = A x_true in exact arithmetic
    up to one rounding of the product)."""
    n, k = 600, 4
    bands, _ = synth.make_problem(n, k, 1, seed=2, rule="theta", theta=0.12)
    x_true = np.random.default_rng(1).standard_normal((n, 1))
    f = oracle.band_matvec(bands, x_true)
    xr = oracle.band_solve_refined(bands, f, steps=3)
    # forward error limited by the rounding of f itself times kappa; must not exceed plain R0
    x0 = oracle.band_solve(bands, f)
    assert rel(xr, x_true) <= rel(x0, x_true) * 1.01 + 1e-15


# ---------------------------------------------------------------- spikes / SVD


def test_p13_spike_residual_and_decay():
    n, k, p = 1200, 5, 3
    bands, _ = synth.make_problem(n, k, 1, seed=7, rule="strict")
    A = dense(bands)
    offs = oracle.partition(n, p)
    for j in range(p):
        V, W = oracle.partition_spikes(bands, p, j)
        s, e = offs[j], offs[j + 1]
        Aj = A[s:e, s:e]
        if j < p - 1:
            rhs = np.zeros((e - s, k))
            rhs[-k:] = A[e - k:e, e:e + k]
            assert np.abs(Aj @ V - rhs).max() < 1e-13
            env = np.abs(V).max(axis=1)
            # dominant matrix: envelope decays away from the bottom tip
            assert env[: (e - s) // 2].max() < 1e-3 * env[-k:].max()
        if j > 0:
            rhs = np.zeros((e - s, k))
            rhs[:k] = A[s:s + k, s - k:s]
            assert np.abs(Aj @ W - rhs).max() < 1e-13
            env = np.abs(W).max(axis=1)
            assert env[(e - s) // 2:].max() < 1e-3 * env[:k].max()


def test_p8_thin_svd_vs_numpy_and_eckart_young():
    rng = np.random.default_rng(4)
    a = rng.standard_normal((300, 9)) @ np.diag(2.0 ** -np.arange(9))
    s, vr = oracle.thin_svd(a)
    s_np = np.linalg.svd(a, compute_uv=False)
    assert np.max(np.abs(s - s_np) / s_np[0]) < 1e-14
    assert np.max(np.abs(vr.T @ vr - np.eye(9))) < 1e-13
    for r in (0, 1, 4, 8):
        P = vr[:, :r]
        err = a - a @ P @ P.T
        nxt = s_np[r] if r < 9 else 0.0
        assert abs(np.linalg.norm(err, 2) - nxt) < 1e-12 * s_np[0]
        assert abs(np.linalg.norm(err, "fro") ** 2 - np.sum(s_np[r:] ** 2)) < 1e-12 * s_np[0] ** 2


# ---------------------------------------------------------------- LR-SPIKE (R1) pins


@pytest.mark.parametrize("n,k,p", [(4096, 8, 4), (700, 4, 7), (333, 3, 5), (96, 4, 4)])
def test_p5_exact_at_full_rank(n, k, p):
    bands, f = synth.make_problem(n, k, 2, seed=1, rule="strict")
    x0 = oracle.band_solve(bands, f)
    x1 = oracle.lrspike(bands, f, p, k)
    assert rel(x1, x0) < 1e-13


def test_p5_exact_at_full_rank_weak_and_nondominant():
    for rule, theta in (("weak", 0), ("theta", 0.3)):
        bands, f = synth.make_problem(900, 6, 1, seed=2, rule=rule, theta=theta)
        assert rel(oracle.lrspike(bands, f, 5, 6), oracle.band_solve(bands, f)) < 1e-11


def _low_rank_coupling(bands, p, r):
    """Zero band entries so that every B_j and C_j has rank <= r."""
    b = bands.copy()
    k = (b.shape[0] - 1) // 2
    n = b.shape[1]
    offs = oracle.partition(n, p)
    for j in range(1, p):
        s = offs[j]
        for a in range(k):  # rows of B_{j-1}: s-k+a, columns s+c (c <= a)
            for c in range(k):
                if a < k - r:
                    row, col = s - k + a, s + c
                    d = col - row
                    if -k <= d <= k:
                        b[d + k, row] = 0.0
                if c < k - r:  # C_j rows s+a, columns s-k+c ; keep only its last r columns
                    row, col = s + a, s - k + c
                    d = col - row
                    if -k <= d <= k:
                        b[d + k, row] = 0.0
    return b


@pytest.mark.parametrize("k,r,p", [(6, 2, 4), (8, 3, 3), (5, 1, 6)])
def test_exact_when_coupling_rank_le_r(k, r, p):
    """If B_j and C_j have rank <= r the spikes have rank <= r, the truncation is
    exact and LR-SPIKE at rank r returns A^{-1} f."""
    bands, f = synth.make_problem(100 * p, k, 2, seed=9, rule="strict")
    bands = _low_rank_coupling(bands, p, r)
    x1, sv = oracle.lrspike(bands, f, p, r, return_sv=True)
    assert rel(x1, oracle.band_solve(bands, f)) < 1e-12
    assert np.all(sv[:, :, r:] < 1e-12 * max(1.0, sv.max()))
    # and the truncation really is active: rank r-1 is not exact
    if r > 1:
        x2 = oracle.lrspike(bands, f, p, r - 1)
        assert rel(x2, oracle.band_solve(bands, f)) > 1e-10


def test_p6_one_partition_is_base_solver():
    bands, f = synth.make_problem(500, 5, 3, seed=4, rule="weak")
    for r in (0, 2, 5):
        assert rel(oracle.lrspike(bands, f, 1, r), oracle.band_solve(bands, f)) < 1e-14


def test_p6_two_partitions_2x2_kernel():
    """p = 2: solving only the central kernel [[I, V_{1,b}], [W_{2,t}, I]] for
    (x_{1,b}, x_{2,t}) and recovering gives the same x (paper's 2x2 kernel)."""
    n, k = 80, 4
    bands, f = synth.make_problem(n, k, 1, seed=6, rule="strict")
    A = dense(bands)
    f = f[:, 0]
    h = n // 2
    A1, A2 = A[:h, :h], A[h:, h:]
    B1, C2 = A[h - k:h, h:h + k], A[h:h + k, h - k:h]
    y1, y2 = np.linalg.solve(A1, f[:h]), np.linalg.solve(A2, f[h:])
    V1 = np.linalg.solve(A1, np.r_[np.zeros((h - k, k)), B1])
    W2 = np.linalg.solve(A2, np.r_[C2, np.zeros((n - h - k, k))])
    Kmat = np.block([[np.eye(k), V1[-k:]], [W2[:k], np.eye(k)]])
    t = np.linalg.solve(Kmat, np.r_[y1[-k:], y2[:k]])
    x1b, x2t = t[:k], t[k:]
    x1 = np.linalg.solve(A1, f[:h] - np.r_[np.zeros(h - k), B1 @ x2t])
    x2 = np.linalg.solve(A2, f[h:] - np.r_[C2 @ x1b, np.zeros(n - h - k)])
    assert rel(oracle.lrspike(bands, f, 2, k), np.r_[x1, x2]) < 1e-13


def _blocks(A, offs):
    p = len(offs) - 1
    D = np.zeros_like(A)
    for j in range(p):
        s, e = offs[j], offs[j + 1]
        D[s:e, s:e] = A[s:e, s:e]
    return D


def test_p7_rank_zero_is_two_block_jacobi_sweeps():
    n, k, p = 300, 4, 5
    bands, f = synth.make_problem(n, k, 2, seed=8, rule="weak")
    A = dense(bands)
    D = _blocks(A, oracle.partition(n, p))
    y = np.linalg.solve(D, f)
    ref = y - np.linalg.solve(D, (A - D) @ y)
    assert rel(oracle.lrspike(bands, f, p, 0), ref) < 1e-13


def _woodbury_dense(A, offs, k, r, f, transpose=False, truncated=False):
    """M_r^{-1} f = D^{-1} f - D^{-1} K S~^{-1} E^T D^{-1} f built densely with numpy's SVD.
    truncated=True: S~ with the blocks V~_{j,t} (rows x_{j,t}, columns x_{j+1,t})
    and W~_{j,b} (rows x_{j,b}, columns x_{j-1,b}) zeroed, the truncated-SPIKE
    system S~~_red of LR-SPIKE-T."""
    n = A.shape[0]
    p = len(offs) - 1
    D = _blocks(A, offs)
    N = 2 * k * p
    E = np.zeros((n, N))
    K = np.zeros((n, N))
    Sp = np.zeros((n, N))
    for j in range(p):
        s, e = offs[j], offs[j + 1]
        E[s:s + k, 2 * j * k:2 * j * k + k] = np.eye(k)
        E[e - k:e, (2 * j + 1) * k:(2 * j + 2) * k] = np.eye(k)
        Aj = A[s:e, s:e]
        if j < p - 1:
            K[e - k:e, 2 * (j + 1) * k:2 * (j + 1) * k + k] = A[e - k:e, e:e + k]
            V = np.linalg.solve(Aj, np.r_[np.zeros((e - s - k, k)), A[e - k:e, e:e + k]])
            Pi = np.linalg.svd(V, full_matrices=False)[2][:r].T
            Sp[s:e, 2 * (j + 1) * k:2 * (j + 1) * k + k] = V @ Pi @ Pi.T
        if j > 0:
            K[s:s + k, (2 * j - 1) * k:2 * j * k] = A[s:s + k, s - k:s]
            W = np.linalg.solve(Aj, np.r_[A[s:s + k, s - k:s], np.zeros((e - s - k, k))])
            Psi = np.linalg.svd(W, full_matrices=False)[2][:r].T
            Sp[s:e, (2 * j - 1) * k:2 * j * k] = W @ Psi @ Psi.T
    assert np.abs(A - D - K @ E.T).max() == 0.0  # the DS / Woodbury split of A
    S = np.eye(N) + E.T @ Sp
    if truncated:
        for j in range(p):
            if j < p - 1:
                S[2 * j * k:2 * j * k + k, 2 * (j + 1) * k:2 * (j + 1) * k + k] = 0.0
            if j > 0:
                S[(2 * j + 1) * k:(2 * j + 2) * k, (2 * j - 1) * k:2 * j * k] = 0.0
    Dinv = np.linalg.inv(D)
    M = Dinv - Dinv @ K @ np.linalg.solve(S, E.T @ Dinv)
    return (M.T if transpose else M) @ f, S


@pytest.mark.parametrize("r", [0, 1, 2, 3, 4])
def test_p3_woodbury_dense_all_ranks(r):
    n, k, p = 96, 4, 4
    bands, f = synth.make_problem(n, k, 2, seed=12, rule="weak")
    A = dense(bands)
    offs = oracle.partition(n, p)
    ref, S = _woodbury_dense(A, offs, k, r, f)
    assert rel(oracle.lrspike(bands, f, p, r), ref) < 1e-12
    S_or = oracle.reduced_dense(bands, p, r)
    assert np.abs(S_or - S).max() < 1e-13
    reft, _ = _woodbury_dense(A, offs, k, r, f, transpose=True)
    assert rel(oracle.lrspike(bands, f, p, r, transpose=True), reft) < 1e-12


# ---------------------------------------------------------------- LR-SPIKE-T


@pytest.mark.parametrize("r", [0, 1, 2, 4])
def test_t_variant_dense_truncated_woodbury(r):
    """LR-SPIKE-T = D^{-1} - D^{-1} K S~~^{-1} E^T D^{-1} with S~~ the reduced
    system without V~_{j,t} and W~_{j,b} (eqs. truncated_redsys,
    red_sys_prec_mid_1), built densely with numpy; also its transpose."""
    n, k, p = 96, 4, 4
    bands, f = synth.make_problem(n, k, 2, seed=21, rule="weak")
    A = dense(bands)
    offs = oracle.partition(n, p)
    ref, _ = _woodbury_dense(A, offs, k, r, f, truncated=True)
    full, _ = _woodbury_dense(A, offs, k, r, f)
    assert rel(oracle.lrspike(bands, f, p, r, variant="t"), ref) < 1e-12
    if r > 0:  # (at r = 0 no spike is kept and the two coincide)
        assert rel(ref, full) > 1e-6  # the dropped couplings matter on this matrix
    reft, _ = _woodbury_dense(A, offs, k, r, f, transpose=True, truncated=True)
    assert rel(oracle.lrspike(bands, f, p, r, transpose=True, variant="t"), reft) < 1e-12


@pytest.mark.parametrize("r", [0, 2, 6])
def test_t_variant_two_partitions_equals_full(r):
    """With two partitions the only dropped blocks (V~_{0,t}, W~_{1,b}) sit in
    rows no other unknown depends on: LR-SPIKE-T = LR-SPIKE (the 2 x 2 kernel of eq. 2x2)."""
    bands, f = synth.make_problem(500, 6, 3, seed=22, rule="weak")
    assert rel(oracle.lrspike(bands, f, 2, r, variant="t"), oracle.lrspike(bands, f, 2, r)) < 1e-13


def test_t_variant_exact_when_off_diagonal_tips_vanish():
    """Cut every partition into two halves that do not couple: then V_j lives in
    the bottom half and W_j in the top half, V_{j,t} = W_{j,b} = 0, and the
    truncated reduced system is the whole one (exact at r = k, equal to
    LR-SPIKE at every r)."""
    n, k, p = 180, 5, 6  # 30-row partitions: short enough for the tips to couple
    bands, f = synth.make_problem(n, k, 2, seed=23, rule="weak")
    offs = oracle.partition(n, p)
    for j in range(p):
        mid = (offs[j] + offs[j + 1]) // 2
        for d in range(-k, k + 1):
            for i in range(mid - k, mid + k):
                if (i < mid <= i + d) or (i + d < mid <= i):
                    bands[d + k, i] = 0.0
    x_t = oracle.lrspike(bands, f, p, k, variant="t")
    assert rel(x_t, oracle.band_solve(bands, f)) < 1e-13
    for r in (1, 3):
        assert rel(oracle.lrspike(bands, f, p, r, variant="t"), oracle.lrspike(bands, f, p, r)) < 1e-13
    # without the cut the dropped blocks are not zero and the two differ
    bands2, _ = synth.make_problem(n, k, 2, seed=23, rule="weak")
    assert rel(oracle.lrspike(bands2, f, p, k, variant="t"), oracle.band_solve(bands2, f)) > 1e-10


def test_t_variant_decay_on_strongly_dominant():
    """Strict dominance 2k+1+|u| with n_j = 1024 rows: the spikes decay away from
    their tip (the premise of truncated SPIKE), so V_{j,t} and W_{j,b} are below
    rounding and LR-SPIKE-T equals LR-SPIKE."""
    bands, f = synth.make_problem(4096, 8, 2, seed=24, rule="strict")
    for r in (8, 4):
        assert rel(oracle.lrspike(bands, f, 4, r, variant="t"), oracle.lrspike(bands, f, 4, r)) < 1e-14


@pytest.mark.parametrize("r", [0, 3, 8])
def test_t_variant_adjoint_dot_product(r):
    n, k, p = 2000, 8, 6
    bands, _ = synth.make_problem(n, k, 1, seed=25, rule="weak")
    rng = np.random.default_rng(0)
    f = rng.standard_normal((n, 3))
    g = rng.standard_normal((n, 3))
    x = oracle.lrspike(bands, f, p, r, variant="t")
    lam = oracle.lrspike(bands, g, p, r, transpose=True, variant="t")
    assert abs(np.sum(x * g) - np.sum(f * lam)) <= 1e-13 * np.linalg.norm(x) * np.linalg.norm(g)


def test_p9_determinant_identity():
    """det S_red = det A / prod_j det A_j (A = D S)."""
    n, k, p = 96, 4, 4
    bands, _ = synth.make_problem(n, k, 1, seed=13, rule="weak")
    A = dense(bands)
    offs = oracle.partition(n, p)
    S = oracle.reduced_dense(bands, p, k)
    lhs = np.linalg.slogdet(S)
    la = np.linalg.slogdet(A)
    ld = [np.linalg.slogdet(A[offs[j]:offs[j + 1], offs[j]:offs[j + 1]]) for j in range(p)]
    sign = la[0] * np.prod([s for s, _ in ld])
    assert lhs[0] == sign
    assert abs(lhs[1] - (la[1] - sum(v for _, v in ld))) < 1e-12


@pytest.mark.parametrize("r", [0, 2, 5, 8])
def test_p10_adjoint_dot_product(r):
    n, k, p = 2000, 8, 6
    bands, _ = synth.make_problem(n, k, 1, seed=14, rule="weak")
    rng = np.random.default_rng(0)
    f = rng.standard_normal((n, 3))
    g = rng.standard_normal((n, 3))
    x = oracle.lrspike(bands, f, p, r)
    lam = oracle.lrspike(bands, g, p, r, transpose=True)
    lhs, rhs = np.sum(x * g), np.sum(f * lam)
    assert abs(lhs - rhs) <= 1e-13 * np.linalg.norm(x) * np.linalg.norm(g)


def test_p11_band_gradient_finite_differences():
    """L(bands, b) = 0.5 ||A^{-1} b - x*||^2: dL/db = A^{-T}(x - x*), dL/dA = -lam x^T on the band."""
    n, k = 512, 4
    bands, b = synth.make_problem(n, k, 1, seed=0, rule="strict")
    rng = np.random.default_rng(1)
    xs = rng.standard_normal((n, 1))

    def loss(bd, bb):
        x = oracle.band_solve(bd, bb)
        return 0.5 * np.sum((x - xs) ** 2)

    x = oracle.band_solve(bands, b)
    lam = oracle.band_solve(bands, x - xs, transpose=True)
    grad_band = oracle.band_grad(lam, x, k)
    h = 1e-6
    mask = np.ones_like(bands)
    for d in range(-k, k + 1):
        if d < 0:
            mask[d + k, :-d] = 0
        elif d > 0:
            mask[d + k, n - d:] = 0
    for _ in range(8):
        dirn = rng.standard_normal(bands.shape) * mask
        fd = (loss(bands + h * dirn, b) - loss(bands - h * dirn, b)) / (2 * h)
        an = np.sum(grad_band * dirn)
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))
    for _ in range(16):
        d = int(rng.integers(-k, k + 1))
        i = int(rng.integers(max(0, -d), min(n, n - d)))
        e = np.zeros_like(bands)
        e[d + k, i] = 1.0
        fd = (loss(bands + h * e, b) - loss(bands - h * e, b)) / (2 * h)
        # the loss is O(n), so cancellation limits a central difference to ~u L / h ~ 3e-8 absolute
        assert abs(fd - grad_band[d + k, i]) <= 1e-6 * abs(fd) + 1e-7
    db = rng.standard_normal(b.shape)
    fd = (loss(bands, b + h * db) - loss(bands, b - h * db)) / (2 * h)
    assert abs(fd - np.sum(lam * db)) <= 1e-6 * max(1.0, abs(fd))


def test_partition_rule():
    offs = oracle.partition(10, 3)
    assert list(offs) == [0, 4, 7, 10]
    offs = oracle.partition(4096, 4)
    assert list(np.diff(offs)) == [1024] * 4


def test_argument_errors():
    bands, f = synth.make_problem(40, 4, 1)
    with pytest.raises(oracle.OracleError):
        oracle.lrspike(bands, f, 6, 4)  # n_j = 6 < 2k
    with pytest.raises(oracle.OracleError):
        oracle.lrspike(bands, f, 2, 5)  # r > k


# ---------------------------------------------------------------- BiCGStab (outer Krylov solver)


@pytest.mark.parametrize("variant,transpose", [("full", False), ("t", False), ("full", True)])
@pytest.mark.parametrize("iters", [1, 3])
def test_bicgstab_iterates_match_scipy(variant, transpose, iters):
    """The oracle's preconditioned BiCGStab against scipy's independent
    implementation of the same recurrence (right preconditioner, same x_0),
    iterate by iterate, on a non-dominant matrix where the iterates are far
    from converged."""
    import scipy.sparse.linalg as sl
    n, k, p, r = 1500, 5, 3, 2
    bands, f = synth.make_problem(n, k, 1, seed=31, rule="theta", theta=0.4)
    f = f[:, 0]
    x_or, its, _ = oracle.bicgstab(bands, f, p, r, tol=0.0, max_it=iters, transpose=transpose, variant=variant)
    assert its == [iters]
    A = sl.LinearOperator((n, n), matvec=lambda v: oracle.band_matvec(bands, v.reshape(-1), transpose=transpose))
    M = sl.LinearOperator((n, n), matvec=lambda v: oracle.lrspike(bands, v.reshape(-1), p, r, transpose=transpose,
                                                                  variant=variant))
    x0 = oracle.lrspike(bands, f, p, r, transpose=transpose, variant=variant)
    x_sp, _ = sl.bicgstab(A, f, x0=x0.copy(), rtol=1e-300, atol=0.0, maxiter=iters, M=M)
    assert rel(x_or, x_sp) < 1e-12
    assert rel(x_or, oracle.band_solve(bands, f, transpose=transpose)) > 1e-9  # not converged yet


def test_bicgstab_exact_preconditioner_converges_at_once():
    """At r = k the preconditioner is A^{-1} (LR-SPIKE is exact): x_0 already
    solves the system and at most one iteration is taken."""
    bands, f = synth.make_problem(3000, 8, 2, seed=32, rule="weak")
    x, its, res = oracle.bicgstab(bands, f, 4, 8, tol=1e-13)
    assert max(its) <= 1 and max(res) <= 1e-13
    assert rel(x, oracle.band_solve(bands, f)) < 1e-13


def test_bicgstab_converges_where_refinement_does_not():
    """Non-dominant matrix, strongly truncated spikes: I - M_r^{-1} A is not a
    contraction (the plain refinement iteration x += M^{-1}(f - A x) grows),
    yet BiCGStab reaches A^{-1} f, for both reduced-system variants."""
    n, k, p, r = 4096, 8, 8, 2
    bands, f = synth.make_problem(n, k, 2, seed=33, rule="theta", theta=0.15)
    xs = oracle.band_solve_refined(bands, f, steps=3)
    x = oracle.lrspike(bands, f, p, r)
    errs = []
    for _ in range(4):
        x = x + oracle.lrspike(bands, f - oracle.band_matvec(bands, x), p, r)
        errs.append(rel(x, xs))
    assert errs[-1] > errs[0]  # refinement diverges here
    for variant in ("full", "t"):
        xb, its, res = oracle.bicgstab(bands, f, p, r, tol=1e-13, max_it=300, variant=variant)
        assert max(res) <= 1e-13
        assert rel(xb, xs) < 1e-9
        true_res = np.linalg.norm(f - oracle.band_matvec(bands, xb), axis=0) / np.linalg.norm(f, axis=0)
        assert true_res.max() < 1e-12


# ---------------------------------------------------------------- randomized SVD
def _spectrum_matrix(rows, cols, sig, seed):
    """rows x cols with singular values sig (descending) and random singular vectors."""
    rng = np.random.default_rng(seed)
    u, _ = np.linalg.qr(rng.standard_normal((rows, cols)))
    v, _ = np.linalg.qr(rng.standard_normal((cols, cols)))
    return (u * sig) @ v.T


def test_rsvd_full_sketch_keeps_the_matrix():
    """ell = cols: the test matrix is square and invertible, range(Y) = range(a)
    and Q Q^T a = a."""
    rng = np.random.default_rng(1)
    a = _spectrum_matrix(400, 12, 0.3 ** np.arange(12), 2)
    pr = oracle.rsvd_project(a, rng.standard_normal((12, 12)))
    assert np.abs(pr - a).max() < 1e-12 * np.abs(a).max()


@pytest.mark.parametrize("rank,ell,q", [(3, 5, 0), (6, 6, 0), (4, 8, 1)])
def test_rsvd_exact_on_low_rank(rank, ell, q):
    """rank(a) <= ell: the sketch spans range(a), so the projection is a itself."""
    rng = np.random.default_rng(rank)
    a = rng.standard_normal((300, rank)) @ rng.standard_normal((rank, 16))
    pr = oracle.rsvd_project(a, rng.standard_normal((16, ell)), q=q)
    assert np.abs(pr - a).max() < 1e-11 * np.abs(a).max()


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("decay", [0.5, 0.9])
def test_rsvd_projection_properties_and_hmt_bound(seed, decay):
    """Q Q^T a is an orthogonal projection of a onto an ell-dimensional space:
    rank <= ell, a - proj orthogonal to proj, error >= sigma_{ell+1}
    (Eckart-Young), and the Halko-Martinsson-Tropp bound
    ||a - Q Q^T a|| <= (1 + 11 sqrt(kk + s) sqrt(min(m, n))) sigma_{kk+1}
    for oversampling s >= 4 (failure probability 6 s^-s)."""
    rows, cols, kk, s = 500, 24, 6, 4
    sig = decay ** np.arange(cols)
    a = _spectrum_matrix(rows, cols, sig, 10 + seed)
    om = np.random.default_rng(100 + seed).standard_normal((cols, kk + s))
    pr = oracle.rsvd_project(a, om)
    sp = np.linalg.svd(pr, compute_uv=False)
    assert sp[kk + s] < 1e-12 * sp[0]
    assert np.abs(pr.T @ (a - pr)).max() < 1e-12 * sig[0] ** 2
    err = np.linalg.norm(a - pr, 2)
    assert err >= sig[kk + s] * (1 - 1e-9)
    assert err <= (1 + 11 * np.sqrt(kk + s) * np.sqrt(min(rows, cols))) * sig[kk]


def test_rsvd_power_steps_sharpen_a_flat_spectrum():
    """With a slowly decaying spectrum each power step brings the error
    closer to the optimum sigma_{ell+1}."""
    sig = 1.0 / (1.0 + np.arange(32))
    a = _spectrum_matrix(600, 32, sig, 5)
    om = np.random.default_rng(6).standard_normal((32, 8))
    errs = [np.linalg.norm(a - oracle.rsvd_project(a, om, q=q), 2) for q in (0, 1, 2)]
    assert errs[2] < errs[1] < errs[0]
    assert errs[2] < 1.5 * sig[8]


def test_rsvd_lrspike_full_sketch_is_the_exact_truncation():
    """ell = k: the randomized truncation is the exact rank-r truncation of the
    whole spike (LR-SPIKE at rank r with its thin SVD)."""
    n, k, p, r = 1200, 8, 4, 3
    bands, f = synth.make_problem(n, k, 2, seed=3, rule="weak")
    om = synth.gaussian_test_matrices(p, k, k, seed=1)
    xe = oracle.lrspike(bands, f, p, r)
    xr = oracle.lrspike_rsvd(bands, f, p, r, om)
    assert rel(xr, xe) < 1e-10


@pytest.mark.parametrize("k,r,ell,p", [(6, 2, 3, 4), (8, 3, 5, 3)])
def test_rsvd_lrspike_exact_when_coupling_rank_le_ell(k, r, ell, p):
    """Couplings of rank <= r <= ell: the spikes have rank <= r, the sketch
    captures them whole and LR-SPIKE returns A^{-1} f."""
    bands, f = synth.make_problem(100 * p, k, 2, seed=9, rule="strict")
    bands = _low_rank_coupling(bands, p, r)
    om = synth.gaussian_test_matrices(p, k, ell, seed=2)
    assert rel(oracle.lrspike_rsvd(bands, f, p, r, om), oracle.band_solve(bands, f)) < 1e-12


def test_rsvd_lrspike_between_exact_truncation_and_sketch_error():
    """r < ell < k on a weakly dominant band: the randomized truncation stays
    close to the exact one (within the tips' sketch error) and differs from it."""
    n, k, p, r, ell = 2000, 12, 5, 4, 7
    bands, f = synth.make_problem(n, k, 1, seed=11, rule="weak")
    om = synth.gaussian_test_matrices(p, k, ell, seed=3)
    xe, sve = oracle.lrspike(bands, f, p, r, return_sv=True)
    xr, svr = oracle.lrspike_rsvd(bands, f, p, r, om, return_sv=True)
    x0 = oracle.band_solve(bands, f)
    d = rel(xr, xe)
    assert 1e-14 < d < 10 * rel(xe, x0) + 1e-12
    # the sketched spikes' leading singular values approach the exact ones
    act = sve[:, :, 0] > 0
    assert np.all(np.abs(svr[:, :, :r] - sve[:, :, :r])[act] <= 0.2 * sve[:, :, :r][act])


@pytest.mark.parametrize("variant", ["full", "t"])
def test_rsvd_lrspike_adjoint_dot_product(variant):
    """<M^{-1} f, g> = <f, M^{-T} g> for the randomized operator too."""
    n, k, p, r, ell = 900, 6, 3, 2, 4
    bands, fg = synth.make_problem(n, k, 2, seed=12, rule="weak")
    om = synth.gaussian_test_matrices(p, k, ell, seed=4)
    f, g = fg[:, 0], fg[:, 1]
    x = oracle.lrspike_rsvd(bands, f, p, r, om, variant=variant)
    lam = oracle.lrspike_rsvd(bands, g, p, r, om, variant=variant, transpose=True)
    assert abs(x @ g - f @ lam) < 1e-12 * np.linalg.norm(x) * np.linalg.norm(g)


# ------------------------------------------------ LR-SPIKE-I and LR-SPIKE-OTF
@pytest.mark.parametrize("n,k,p,r,rule,theta", [(180, 8, 4, 3, "weak", 1.05), (200, 8, 4, 3, "theta", 0.3)])
def test_lri_converges_to_the_direct_lrspike(n, k, p, r, rule, theta):
    """LR-SPIKE-I solves the same S~_red as LR-SPIKE, iteratively: at
    convergence the two agree, while the preconditioner's own one-shot answer
    (LR-SPIKE-T) differs from both (short partitions keep the far tips)."""
    bands, f = synth.make_problem(n, k, 2, seed=1, rule=rule, theta=theta)
    xr = oracle.lrspike(bands, f, p, r)
    xi, iters, relres = oracle.lrspike_iter(bands, f, p, r, "i", tol=1e-14)
    assert np.all(iters >= 1) and np.all(relres <= 1e-14)
    assert rel(xi, xr) <= 1e-12
    assert rel(oracle.lrspike(bands, f, p, r, variant="t"), xr) > 1e-8


def test_lri_without_iterations_is_lrspike_t():
    """x_0 = S~~_red^{-1} y_red: with no iteration the result is LR-SPIKE-T's."""
    bands, f = synth.make_problem(200, 8, 2, seed=1, rule="theta", theta=0.3)
    x0, iters, _ = oracle.lrspike_iter(bands, f, 4, 3, "i", max_it=0)
    assert np.all(iters == 0)
    assert rel(x0, oracle.lrspike(bands, f, 4, 3, variant="t")) <= 1e-14


@pytest.mark.parametrize("n,k,p,r,rule,theta", [(200, 8, 4, 3, "theta", 0.3), (240, 6, 5, 2, "weak", 1.05),
                                                (4000, 16, 4, 4, "weak", 1.05), (1200, 16, 3, 4, "theta", 0.3)])
def test_otf_converges_to_the_exact_solve(n, k, p, r, rule, theta):
    """LR-SPIKE-OTF solves the true reduced system: for any r the result is
    A^{-1} f to the inner tolerance (two backward-stable solves differ by
    ~kappa u: 10x the oracle's own forward error, at least 1e-12), where the
    rank-r one-shot operators are off by the truncation."""
    bands, f = synth.make_problem(n, k, 2, seed=2, rule=rule, theta=theta)
    x0 = oracle.band_solve(bands, f)
    ref = oracle.band_solve_refined(bands, f)
    xo, iters, relres = oracle.lrspike_iter(bands, f, p, r, "otf", tol=1e-14)
    assert np.all(iters >= 2) and np.all(relres <= 1e-14)
    assert rel(xo, ref) <= max(1e-12, 10 * rel(x0, ref))
    assert rel(oracle.lrspike(bands, f, p, r), ref) > 1e-6
