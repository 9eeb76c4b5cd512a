"""Plain FP64 SOR-SVD, step by step as in Sec. III of the paper.

Alg. 3 (basic SOR-SVD) and Alg. 4 (SOR-SVD with power method):
  1. Omega: n x l standard Gaussian (Alg. 3/4 step 1)       -> ``normal.gaussian_matrix``
  2. T1 = A Omega  (eq. T1),  T2 = A^T T1  (eq. AT1)          -> repeated q+1 times in Alg. 4
  3. T1 = Q1 R1, T2 = Q2 R2  (thin QR)
  4. M = Q1^T A Q2  (eq. M)
  5. rank-k truncated SVD of M: M_k = U~_k S~_k V~_k^T (the transpose is
     implied by the lift in step 6)
  6. A_hat = (Q1 U~_k) S~_k (Q2 V~_k)^T

Step 4 has two forms (``m_form``):
  * ``"exact"`` (default): M = Q1^T A Q2 (eq. M), one more pass over A.
  * ``"approx"``: the pass-efficient M_approx = Q1^T T1 (Q2^T X)^+ (eq.
    M_approx), from A ~ A Q2 Q2^T: X is the operand that produced the last T1
    (Omega when q = 0; in Alg. 4 the non-updated T2 of the last round, in
    the canonical reading the Q2 of the previous round), and ^+ is the
    Moore-Penrose pseudo-inverse.

Two readings of step 2 are offered:
  * ``mode="canonical"`` (default): orthonormalise after every product,
    Q1 = qr(A Q2), Q2 = qr(A^T Q1). By Lemma 1 (Gu) QR(B X) and QR(B X Y) give
    the same projector for non-singular Y, so this spans exactly what Alg. 4's
    T1 = A (A^T A)^q Omega and T2 = (A^T A)^(q+1) Omega span; it is the only
    form that survives the loss of precision of repeated products.
  * ``mode="literal"``: Alg. 4 as printed, T2 <- Omega; q+1 times
    {T1 = A T2; T2 = A^T T1}; QR only at the end.

QR is LAPACK's Householder QR with column signs fixed so that diag(R) > 0
(the unique thin QR of a full-rank matrix). The core SVD is LAPACK's.

Output convention (the paper leaves signs free): singular values descending;
each column of U has its largest-magnitude entry positive (lowest row index on
ties) and the matching column of V is flipped with it.

Test infrastructure only (see ``oracle/__init__``).
"""
import numpy as np

from .normal import gaussian_matrix


def qr_pos(T):
    """Thin QR T = Q R with diag(R) >= 0 (zero pivots keep the LAPACK sign)."""
    Q, R = np.linalg.qr(T, mode="reduced")
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d[None, :], R * d[:, None]


def sign_convention(U, V):
    """Flip column pairs so each U column's largest-|.| entry is positive."""
    U = U.copy()
    V = V.copy()
    if U.shape[0] == 0:
        return U, V
    idx = np.argmax(np.abs(U), axis=0)  # first maximal index on ties
    s = np.sign(U[idx, np.arange(U.shape[1])])
    s[s == 0] = 1.0
    return U * s[None, :], V * s[None, :]


def omega(seed, n, l):
    """Omega of Alg. 3 / Alg. 4 step 1 (stream 0 of the Philox key)."""
    return gaussian_matrix(seed, n, l, stream=0)


def sorsvd(A, k, q=0, seed=0, l=None, mode="canonical", Omega=None, return_all=False, m_form="exact",
           explicit=True):
    """SOR-SVD of A (m x n) to rank k with sketch width l (default l = k) and q power steps.

    Returns (U, s, V, info): U m x k, s length k (descending), V n x k, and
    info = {"err_fro": ||A - U diag(s) V^T||_F / ||A||_F (explicit; with
            explicit=False the identity below instead, which skips forming
            the m x n residual),
            "err_fro_identity": same via ||A||_F^2 - sum s^2 (Th. 2 split),
            "a_fro": ||A||_F}.
    """
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    if l is None or l == 0:
        l = k
    if not (1 <= k <= l <= min(m, n)):
        raise ValueError("need 1 <= k <= l <= min(m, n)")
    if q < 0:
        raise ValueError("q must be >= 0")
    if Omega is None:
        Omega = omega(seed, n, l)

    if m_form not in ("exact", "approx"):
        raise ValueError(m_form)
    if mode == "canonical":
        X = Omega
        T1 = A @ X                                # eq. (T1)
        Q1, _ = qr_pos(T1)
        Q2, R2 = qr_pos(A.T @ Q1)                 # eq. (AT1) + QR (span of A^T T1)
        for _ in range(q):                        # Alg. 4 power loop
            X = Q2
            T1 = A @ X
            Q1, _ = qr_pos(T1)
            Q2, R2 = qr_pos(A.T @ Q1)
    elif mode == "literal":
        T2 = Omega
        for _ in range(q + 1):                    # Alg. 4 loop, no intermediate QR
            X = T2                                # the non-updated T2 of this power iteration
            T1 = A @ X
            T2 = A.T @ T1
        Q1, _ = qr_pos(T1)
        Q2, R2 = qr_pos(T2)
    else:
        raise ValueError(mode)

    if m_form == "exact":
        M = Q1.T @ (A @ Q2)                       # eq. (M)
    else:
        M = (Q1.T @ T1) @ np.linalg.pinv(Q2.T @ X)  # eq. (M_approx)
    Ut, s, Vt = np.linalg.svd(M)                  # core SVD, descending
    Uk, sk, Vk = Ut[:, :k], s[:k], Vt[:k, :].T    # truncation to rank k
    U = Q1 @ Uk                                   # lift (Alg. 3 step 7)
    V = Q2 @ Vk
    U, V = sign_convention(U, V)

    a_fro = float(np.linalg.norm(A))
    info = {"a_fro": a_fro}
    if a_fro > 0:
        info["err_fro_identity"] = float(np.sqrt(max(a_fro ** 2 - float(np.sum(sk ** 2)), 0.0))) / a_fro
        if explicit:
            R = A - (U * sk[None, :]) @ V.T
            info["err_fro"] = float(np.linalg.norm(R)) / a_fro
        else:
            info["err_fro"] = info["err_fro_identity"]
    else:
        info["err_fro"] = 0.0
        info["err_fro_identity"] = 0.0
    if return_all:
        info.update(Q1=Q1, Q2=Q2, M=M, Omega=Omega, R2=R2, s_all=s, X=X, T1=T1)
    return U, sk, V, info


def sketch(A, X):
    """T = A X (eq. T1 / the T1 update of Alg. 4)."""
    return np.asarray(A, dtype=np.float64) @ np.asarray(X, dtype=np.float64)


def orbit(A, Y):
    """T = A^T Y (eq. AT1 / the T2 update of Alg. 4)."""
    return np.asarray(A, dtype=np.float64).T @ np.asarray(Y, dtype=np.float64)


def projection(A, Q1, Q2):
    """M = Q1^T A Q2 (eq. M)."""
    return Q1.T @ (np.asarray(A, dtype=np.float64) @ Q2)
