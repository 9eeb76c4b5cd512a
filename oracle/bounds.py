"""Closed forms and theorem bounds of the paper, evaluated in FP64.

  ey_floor         Th. 1 (Eckart-Young / Mirsky): best rank-k error.
  th4_sv_lower     Th. 4, deterministic lower bounds on sigma_j(A_hat).
  th5_err_upper    Th. 5, deterministic upper bound on ||A - A_hat|| (2 and F).
  th6_sv_expect    Th. 6, lower bound on E sigma_j(A_hat) (needs p >= 2).
  th7_err_expect   Th. 7, upper bound on E ||A - A_hat|| (needs p >= 2).

Notation (Sec. IV-A): V1 = first l-p right singular vectors of A, V2 = the
rest; Omega1 = V1^T Omega, Omega2 = V2^T Omega (eq. Omegas); sigma_{l-p+1} is
the first singular value of Sigma_3; 2 <= p + k <= l.

Reading of Th. 5 with the power method: tau = (sigma_k / sigma_{l-p+1}) * beta.
The printed tau = beta / sigma_{l-p+1} is not dimensionless and does not
reduce to the q = 0 value sigma_{l-p+1} / sigma_1; the reading above does, as
eta = (sigma_k / sigma_{l-p+1}) * alpha does for eta.

Test infrastructure only (see ``oracle/__init__``).
"""
import math

import numpy as np


def ey_floor(sigma, k, norm="fro"):
    """||A - A_k|| for singular values ``sigma`` (descending), Th. 1."""
    sigma = np.asarray(sigma, dtype=np.float64)
    if norm == "fro":
        tail = sigma[k:]
        return float(math.sqrt(float(np.sum(tail * tail))))
    return float(sigma[k]) if k < sigma.size else 0.0


def _omega_parts(V, Omega, l, p):
    V1 = V[:, : l - p]
    V2 = V[:, l - p:]
    O1 = V1.T @ Omega
    O2 = V2.T @ Omega
    n2 = np.linalg.norm(O2, 2) if O2.size else 0.0
    n1p = np.linalg.norm(np.linalg.pinv(O1), 2)
    return n2, n1p


def th4_sv_lower(sigma, V, Omega, k, l, p, q):
    """Lower bounds on sigma_j(A_hat), j = 1..k (Th. 4, eqs. Thr1_sv1 / Thr1_sv2)."""
    sigma = np.asarray(sigma, dtype=np.float64)
    if not (2 <= p + k <= l):
        raise ValueError("need 2 <= p + k <= l")
    n2, n1p = _omega_parts(V, Omega, l, p)
    s_lp1 = sigma[l - p]
    sj = sigma[:k]
    return sj / np.sqrt(1.0 + (n2 * n1p) ** 2 * (s_lp1 / sj) ** (4 * q + 4))


def th5_err_upper(sigma, V, Omega, k, l, p, q, norm="fro"):
    """Upper bound on ||A - A_hat||_norm (Th. 5, eq. Thr2_1st and its power-method form)."""
    sigma = np.asarray(sigma, dtype=np.float64)
    if not (2 <= p + k <= l):
        raise ValueError("need 2 <= p + k <= l")
    n2, n1p = _omega_parts(V, Omega, l, p)
    g = (n2 * n1p) ** 2
    s1, sk, slp = sigma[0], sigma[k - 1], sigma[l - p]
    decay = (slp / sk) ** (2 * q)
    alpha = math.sqrt(k) * slp ** 2 / sk * decay
    beta = slp ** 2 / (s1 * sk) * decay
    eta = (sk / slp) * alpha
    tau = (sk / slp) * beta
    a0 = ey_floor(sigma, k, "fro" if norm == "fro" else "2")
    return a0 + math.sqrt(alpha ** 2 * g / (1 + beta ** 2 * g)) + math.sqrt(eta ** 2 * g / (1 + tau ** 2 * g))


def _nu(n, l, p):
    nu1 = math.sqrt(n - l + p) + math.sqrt(l) + 7.0
    nu2 = 4.0 * math.e * math.sqrt(l) / (p + 1)
    return nu1 * nu2


def th6_sv_expect(sigma, n, k, l, p, q):
    """Lower bound on E sigma_j(A_hat), j = 1..k (Th. 6)."""
    if p < 2:
        raise ValueError("Th. 6 needs p >= 2")
    sigma = np.asarray(sigma, dtype=np.float64)
    gam = sigma[l - p] / sigma[:k]
    return sigma[:k] / np.sqrt(1.0 + _nu(n, l, p) ** 2 * gam ** (4 * q + 4))


def th7_err_expect(sigma, n, k, l, p, q, norm="fro"):
    """Upper bound on E ||A - A_hat||_norm (Th. 7)."""
    if p < 2:
        raise ValueError("Th. 7 needs p >= 2")
    sigma = np.asarray(sigma, dtype=np.float64)
    gk = sigma[l - p] / sigma[k - 1]
    a0 = ey_floor(sigma, k, "fro" if norm == "fro" else "2")
    return a0 + (1 + gk) * math.sqrt(k) * _nu(n, l, p) * sigma[l - p] * gk ** (2 * q)
