"""Pins of the FP64 ALM-SOR-SVD oracle (robust PCA, Table III) against
things other than itself: the soft-thresholding closed form, the initial
values on a matrix with known norms, exact recovery of a low-rank plus sparse
matrix (the regime where the convex program provably recovers both parts),
the same iteration with LAPACK's SVD in place of SOR-SVD, and the optimality
conditions of the convex program at the end (the multiplier Y lies in both
subdifferentials: ||Y||_2 <= 1, ||Y||_max <= lambda)."""
import numpy as np

from oracle import rpca


def problem(n, r, frac, seed, amp=50.0):
    g = np.random.default_rng(seed)
    L = g.standard_normal((n, r)) @ g.standard_normal((r, n))
    S = np.zeros((n, n))
    idx = g.choice(n * n, int(frac * n * n), replace=False)
    S.flat[idx] = g.choice([-amp, amp], size=idx.size)
    return L, S


def test_shrink_closed_form():
    x = np.array([-3.0, -1.0, -0.25, 0.0, 0.25, 1.0, 3.0])
    assert np.array_equal(rpca.shrink(x, 1.0), [-2.0, 0.0, 0.0, 0.0, 0.0, 0.0, 2.0])
    assert np.array_equal(rpca.shrink(x, 0.0), x)


def test_initial_values_on_a_diagonal_matrix():
    X = np.diag([4.0, -2.0, 1.0, 0.5])
    iv = rpca.initial_values(X)
    assert iv["lambda"] == 0.5 and iv["norm2"] == 4.0
    # J = max(||X||_2, ||X||_max / lambda) = max(4, 8) = 8
    assert np.allclose(iv["Y0"], X / 8.0, rtol=0, atol=0)
    assert iv["mu0"] == 1.25 / 4.0 and iv["mu_bar"] == 1e7 * 1.25 / 4.0 and iv["rho"] == 1.5


def test_exact_recovery_of_low_rank_plus_sparse():
    L0, S0 = problem(200, 10, 0.05, 1)
    X = L0 + S0
    L, S, info = rpca.alm_sorsvd(X, 20, q=1, seed=3)
    assert info["xi"] < 1e-7 and info["iters"] < 30
    assert info["rank"] == 10
    assert np.array_equal(np.abs(S) > 1.0, S0 != 0)
    assert np.linalg.norm(L - L0) <= 1e-5 * np.linalg.norm(L0)
    assert np.linalg.norm(S - S0) <= 1e-5 * np.linalg.norm(S0)


def test_sorsvd_step_agrees_with_lapack_svd_step():
    L0, S0 = problem(150, 8, 0.05, 2)
    X = L0 + S0
    La, Sa, ia = rpca.alm_sorsvd(X, 16, q=1, seed=5, svd="sorsvd")
    Lb, Sb, ib = rpca.alm_sorsvd(X, 16, svd="exact")
    assert abs(ia["iters"] - ib["iters"]) <= 1
    assert np.linalg.norm(La - Lb) <= 1e-5 * np.linalg.norm(Lb)
    assert np.linalg.norm(Sa - Sb) <= 1e-5 * np.linalg.norm(Sb)


def test_multiplier_satisfies_the_optimality_conditions():
    L0, S0 = problem(200, 10, 0.05, 4)
    X = L0 + S0
    L, S, info = rpca.alm_sorsvd(X, 20, q=1, seed=1, tol=1e-9)
    Y, lam = info["Y"], info["lambda"]
    assert np.linalg.norm(Y, 2) <= 1.0 + 1e-5          # Y in the subdifferential of ||L||_*
    assert np.abs(Y).max() <= lam * (1.0 + 1e-6)        # Y in lambda times that of ||S||_1
    # on the support of S the multiplier sits at lambda sgn(S)
    on = S != 0
    assert np.allclose(Y[on], lam * np.sign(S[on]), rtol=0, atol=1e-6 * lam)
