"""FP64 reference of robust PCA solved by the ALM-SOR-SVD method (test
infrastructure).

Problem (Sec. V, RPCA): split X = L + S with L low-rank and S sparse by
minimising ||L||_* + lambda ||S||_1 subject to L + S = X. The inexact
augmented-Lagrange-multiplier iteration of Table III replaces the SVD by a
SOR-SVD of width l:

    (U, z, V) = sorsvd(X - S_k + Y_k / mu_k)          width l, q power steps
    L_{k+1}   = U  shrink_{1/mu_k}(z)  V^T             singular value thresholding
    S_{k+1}   = shrink_{lambda/mu_k}(X - L_{k+1} + Y_k / mu_k)
    Y_{k+1}   = Y_k + mu_k (X - L_{k+1} - S_{k+1})
    mu_{k+1}  = min(rho mu_k, mu_bar)

shrink_e(x) = sgn(x) max(|x| - e, 0). The table prints max(rho mu_k, mu_bar),
which would never let mu stop growing; the continuation it cites caps mu, so
min is read (as is Y_k for the Y of the S update). Initial values (those of
the inexact ALM of Lin, Chen and Ma, which the paper adopts): lambda =
1/sqrt(max(m, n)), Y_0 = X / J(X) with J(X) = max(||X||_2, ||X||_max /
lambda), mu_0 = 1.25 / ||X||_2, rho = 1.5, mu_bar = 1e7 mu_0, S_0 = 0. The
iteration stops when ||X - L - S||_F < tol ||X||_F (tol = 1e-7 in the paper's
experiments) or after max_iter steps.

The SVD step is either the oracle's own SOR-SVD (``svd="sorsvd"``, canonical
mode, seed incremented per iteration) or LAPACK's full SVD truncated to l
(``svd="exact"``), which the tests use to pin the iteration itself.
"""
import numpy as np

from . import sorsvd as osvd


def shrink(x, eps):
    """Soft thresholding sgn(x) max(|x| - eps, 0)."""
    return np.sign(x) * np.maximum(np.abs(x) - eps, 0.0)


def initial_values(X):
    X = np.asarray(X, dtype=np.float64)
    m, n = X.shape
    lam = 1.0 / np.sqrt(max(m, n))
    norm2 = float(np.linalg.norm(X, 2))
    J = max(norm2, float(np.abs(X).max()) / lam)
    mu0 = 1.25 / norm2
    return {"lambda": lam, "Y0": X / J, "mu0": mu0, "rho": 1.5, "mu_bar": 1e7 * mu0, "norm2": norm2}


def alm_sorsvd(X, l, q=1, seed=0, tol=1e-7, max_iter=100, svd="sorsvd", norm2=None):
    """Returns (L, S, info) with info = {"iters", "xi" (relative residual),
    "rank" (singular values kept in the last thresholding), "lambda"}."""
    X = np.asarray(X, dtype=np.float64)
    m, n = X.shape
    iv = initial_values(X)
    if norm2 is not None:  # a caller-supplied ||X||_2 (the GPU estimates it)
        iv["mu0"] = 1.25 / norm2
        iv["mu_bar"] = 1e7 * iv["mu0"]
        iv["Y0"] = X / max(norm2, float(np.abs(X).max()) / iv["lambda"])
    lam, mu, rho, mu_bar = iv["lambda"], iv["mu0"], iv["rho"], iv["mu_bar"]
    Y = iv["Y0"]
    S = np.zeros_like(X)
    x_fro = float(np.linalg.norm(X))
    L = np.zeros_like(X)
    it, xi, rank = 0, np.inf, 0
    while it < max_iter:
        W = X - S + Y / mu
        if svd == "sorsvd":
            U, z, V, _ = osvd.sorsvd(W, l, q=q, seed=seed + it)
        else:
            Uf, zf, Vtf = np.linalg.svd(W, full_matrices=False)
            U, z, V = Uf[:, :l], zf[:l], Vtf[:l, :].T
        zt = shrink(z, 1.0 / mu)
        rank = int(np.count_nonzero(zt))
        L = (U * zt[None, :]) @ V.T
        S = shrink(X - L + Y / mu, lam / mu)
        R = X - L - S
        Y = Y + mu * R
        mu = min(rho * mu, mu_bar)
        it += 1
        xi = float(np.linalg.norm(R)) / x_fro
        if xi < tol:
            break
    return L, S, {"iters": it, "xi": xi, "rank": rank, "lambda": lam, "Y": Y, "mu": mu}
