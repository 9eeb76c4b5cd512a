"""Sketch widths l > 128 (up to 1024): column-blocked passes, the blocked
Cholesky factor of the QR step, the blocked one-sided Jacobi core SVD and the
tiled explicit residual, each against the CPU FP64 oracle (or LAPACK / numpy
for single steps) through the C ABI.

Tolerances:
  FP64 whole method: sigma normwise <= 1e-10, factors equal up to sign to 1e-7
    where the spectrum gap allows (relative gap > 1e-6 on both sides).
  core SVD step: sigma normwise <= 1e-12 against LAPACK (one-sided Jacobi is
    backward stable; the sums over up to 1024 rows round at ~sqrt(l) u).
  QR step: Q^T Q - I <= 1e-13 (two Cholesky-QR steps, or three after a shift),
    Q R = T to 1e-13 |T| cond.
  FP32 / BF16 passes: oracle on the stored values; sigma normwise <= 1e-5 for
    FP32 (backward error ~u32 ||A|| sqrt(K)) and <= 1e-3 for BF16 (operands
    rounded to BF16, the projection to 2^-17 by the hi + lo split).
"""
import numpy as np
import pytest

import workloads as W
from oracle import sorsvd as osvd

from test_gpu_parity import align_signs, check_against_oracle, dev, host, normwise

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("m,n,k,q,l", [
    (700, 600, 256, 1, None),      # two column blocks of 128
    (900, 800, 200, 1, 300),       # ragged width (l = 300: 3 blocks of 112), k < l
    (600, 900, 129, 2, None),      # just above one block, m < n
    (1500, 1200, 512, 1, None),
    (1300, 1100, 1024, 0, None),   # widest sketch
])
def test_wide_fp64_against_oracle(lib, m, n, k, q, l):
    sigma = 1.0 / np.arange(1, min(m, n) + 1) ** 1.5
    A, _, _ = W.spectral(m, n, sigma, m + n + k)
    S, So, info, io = check_against_oracle(lib, A, dev(A), k, q, 3, l=l, tol_s=1e-10, tol_vec=1e-7)
    # identity e^2 = 1 - sum_j s_j^2 / ||A||^2 against the oracle's explicit
    # residual: differences of ~1e-15 ||A||^2 in the two sums over k terms move
    # e by ~k 1e-15 / (2 e)
    assert abs(info["err_fro"] - io["err_fro"]) <= k * 1e-15 / io["err_fro"]
    assert 1 <= info["sweeps"] <= 16


def test_wide_pass_efficient_fp64(lib):
    sigma = 0.995 ** np.arange(1000)
    A, _, _ = W.spectral(1200, 1000, sigma, 8)
    S, So, info, io = check_against_oracle(lib, A, dev(A), 300, 1, 4, tol_s=1e-10, tol_vec=1e-7, pass_efficient=1)


def test_wide_exact_rank_reconstruction(lib):
    gen = W.rng(71)
    A = gen.standard_normal((900, 250)) @ gen.standard_normal((250, 700))
    U, S, V, info = lib.sorsvd(dev(A), 250, q=1, seed=5)
    U, S, V = host(U), host(S), host(V)
    assert np.abs(A - (U * S) @ V.T).max() <= 1e-10 * np.abs(A).max()
    assert info["err_fro"] < 1e-6


@pytest.mark.parametrize("l,k", [(129, 129), (200, 100), (256, 256), (513, 400), (1024, 1024)])
def test_wide_core_svd_against_lapack(lib, l, k):
    gen = W.rng(l * 5 + k)
    Mtx = gen.standard_normal((l, l)) @ np.diag(np.geomspace(1, 1e-6, l)) @ gen.standard_normal((l, l))
    Ut, s, Vt, info = lib.step_core_svd(dev(Mtx), k)
    Ut, s, Vt = host(Ut), host(s), host(Vt)
    Ur, sr, Vrt = np.linalg.svd(Mtx)
    assert normwise(s, sr[:k]) <= 1e-12, normwise(s, sr[:k])
    assert np.all(np.diff(s) <= 0)
    assert info["flags"] == 0 and 1 <= info["sweeps"] <= 40, info
    gap_ok = np.ones(k, dtype=bool)
    rel_gap = np.abs(np.diff(sr)) / sr[0]
    gap_ok[:-1] &= rel_gap[:k - 1] > 1e-6
    gap_ok[1:] &= rel_gap[:k - 1] > 1e-6
    Ua = align_signs(Ut, Ur[:, :k])
    Va = align_signs(Vt, Vrt[:k].T)
    assert np.abs(Ua - Ur[:, :k])[:, gap_ok].max(initial=0) < 1e-8
    assert np.abs(Va - Vrt[:k].T)[:, gap_ok].max(initial=0) < 1e-8
    # (V' accumulates the rotation products of every step: drift ~ steps u)
    assert np.abs(Ut.T @ Ut - np.eye(k)).max() < 5e-12
    assert np.abs(Vt.T @ Vt - np.eye(k)).max() < 5e-12
    # M V = U diag(s)
    assert np.abs(Mtx @ Vt - Ut * s[None, :]).max() < 1e-12 * s[0]


@pytest.mark.parametrize("sweeps", [1, 2, 3])
def test_wide_truncated_sweeps_keep_v_consistent(lib, sweeps):
    """A sweep cap that stops the block Jacobi early: the columns X = M V and V
    carry the same rotations whatever the convergence (V receives each step's
    W one launch later, and one launch after the last step), so A V - U diag(s)
    = (I - P_Q1) A V is as small as in the converged run of the same draw
    (it is the sketch's own approximation error; a W left out of V would
    leave errors of the order of its rotation angle times s_1), and V stays
    orthonormal."""
    m, n, l = 600, 500, 200
    sigma = 0.8 ** np.arange(n, dtype=np.float64)
    A, _, _ = W.spectral(m, n, sigma, 12)

    def relation_error(**opts):
        U, S, V, info = lib.sorsvd(dev(A), l, q=0, seed=3, l=l, **opts)
        U, S, V = host(U), host(S), host(V)
        assert np.abs(V.T @ V - np.eye(l)).max() < 1e-12
        return np.abs(A @ V - U * S[None, :]).max() / S[0], info

    e_full, _ = relation_error()
    e_cut, info = relation_error(max_sweeps=sweeps)
    assert info["sweeps"] <= sweeps
    assert e_cut <= 10 * e_full + 1e-12, (e_cut, e_full)


def test_wide_core_svd_diagonal_is_a_permutation(lib):
    """Orthogonal columns: after the QR preconditioning (which reproduces a
    diagonal M to rounding) no rotation is needed, and V is the permutation
    that sorts the values."""
    l = 300
    d = W.rng(4).permutation(np.arange(1, l + 1)).astype(np.float64)
    Ut, s, Vt, info = lib.step_core_svd(dev(np.diag(d)), l)
    order = np.argsort(-d, kind="stable")
    assert np.max(np.abs(host(s) - d[order]) / d[order]) <= 8 * 2.0 ** -52
    P = np.eye(l)[:, order]
    assert np.abs(np.abs(host(Vt)) - P).max() <= 1e-15
    assert np.abs(np.abs(host(Ut)) - P).max() <= 1e-15
    assert info["sweeps"] <= 2


@pytest.mark.parametrize("rows,l,cond", [(3000, 256, 1e2), (5000, 512, 1e6), (2500, 1024, 1e4),
                                         (4000, 300, 1e11), (2000, 200, 1e9), (1500, 129, 10.0)])
def test_wide_qr_matches_householder(lib, rows, l, cond):
    gen = W.rng(rows + l)
    U = W.haar_columns(rows, l, gen)
    V = W.haar_columns(l, l, gen)
    s = np.geomspace(1.0, 1.0 / cond, l)
    T = (U * s) @ V.T
    Q, R = lib.step_qr(dev(T))
    Q, R = host(Q), host(R)
    Qo, Ro = osvd.qr_pos(T)
    assert np.abs(Q.T @ Q - np.eye(l)).max() <= 1e-13
    assert np.abs(Q @ R - T).max() <= 1e-13 * np.abs(T).max() * cond
    assert np.all(np.diag(R) > 0)
    assert np.abs(np.tril(R, -1)).max() == 0.0
    assert np.abs(Q - Qo).max() <= 1e-15 * cond * 100 * np.sqrt(rows)


@pytest.mark.parametrize("m,n,l", [(3000, 2000, 1024), (1000, 777, 300), (513, 1031, 144)])
def test_wide_sketch_and_orbit_fp64(lib, m, n, l):
    gen = W.rng(m + n + l)
    A = gen.standard_normal((m, n))
    X = gen.standard_normal((n, l))
    Y = gen.standard_normal((m, l))
    Ad = dev(A)
    T = host(lib.step_sketch(Ad, dev(X)))
    assert np.abs(T - A @ X).max() <= 1e-13 * np.abs(A).max() * np.abs(X).max() * n
    T2 = host(lib.step_orbit(Ad, dev(Y)))
    assert np.abs(T2 - A.T @ Y).max() <= 1e-13 * np.abs(A).max() * np.abs(Y).max() * m


@pytest.mark.parametrize("m,n,l", [(2000, 1500, 256), (1200, 900, 300)])
def test_wide_sketch_and_orbit_fp32(lib, m, n, l):
    gen = W.rng(m * 3 + l)
    A32 = gen.standard_normal((m, n)).astype(np.float32)
    A = A32.astype(np.float64)
    X = gen.standard_normal((n, l))
    Y = gen.standard_normal((m, l))
    Ad = dev(A32, torch.float32)
    T = host(lib.step_sketch(Ad, dev(X)))
    ref = A @ X.astype(np.float32).astype(np.float64)
    assert np.abs(T - ref).max() <= 2e-6 * np.sqrt(n) * np.abs(A).max() * np.abs(X).max()
    T2 = host(lib.step_orbit(Ad, dev(Y)))
    ref2 = A.T @ Y.astype(np.float32).astype(np.float64)
    assert np.abs(T2 - ref2).max() <= 2e-6 * np.sqrt(m) * np.abs(A).max() * np.abs(Y).max()


@pytest.mark.parametrize("m,n,k,q", [(2000, 1500, 256, 1), (3000, 2000, 512, 1)])
def test_wide_fp32_against_oracle_on_stored_values(lib, m, n, k, q):
    sigma = 1.0 / np.arange(1, min(m, n) + 1) ** 1.5
    A, _, _ = W.spectral(m, n, sigma, 2)
    A32 = A.astype(np.float32)
    U, S, V, info = lib.sorsvd(dev(A32, torch.float32), k, q=q, seed=9)
    U, S, V = host(U), host(S), host(V)
    Uo, So, Vo, io = osvd.sorsvd(A32.astype(np.float64), k, q=q, seed=9)
    assert normwise(S, So) <= 1e-5, normwise(S, So)
    assert np.abs(U.T @ U - np.eye(k)).max() < 1e-11
    assert info["flags"] == 0


@pytest.mark.parametrize("m,n,k,q,pe", [(3000, 2000, 256, 1, 0), (2500, 1800, 300, 1, 1)])
def test_wide_bf16_against_oracle_on_stored_values(lib, m, n, k, q, pe):
    from test_gpu_bf16 import dev_bf16, to_bf16
    sigma = 0.99 ** np.arange(min(m, n))
    A, _, _ = W.spectral(m, n, sigma, 6)
    A = to_bf16(A)
    U, S, V, info = lib.sorsvd(dev_bf16(A), k, q=q, seed=3, refine=1, pass_efficient=pe)
    U, S, V = host(U), host(S), host(V)
    Uo, So, Vo, io = osvd.sorsvd(A, k, q=q, seed=3, m_form="approx" if pe else "exact")
    assert np.abs(U.T @ U - np.eye(k)).max() < 1e-11
    assert np.all(np.diff(S) <= 0)
    dsig = normwise(S, So)
    print(f"bf16 wide m={m} n={n} k={k} pe={pe}: sigma normwise {dsig:.2e}")
    assert dsig < 1e-3


@pytest.mark.parametrize("m,n,k,q", [(1200, 1000, 300, 1), (900, 1100, 200, 0)])
def test_wide_explicit_residual_fp64(lib, m, n, k, q):
    A = W.low_rank_plus_noise(m, n, 150, 1e-3, m + n + k)
    U, S, V, info = lib.sorsvd(dev(A), k, q=q, seed=5, residual=1)
    _, _, _, io = osvd.sorsvd(A, k, q=q, seed=5)
    e = info["err_fro_explicit"]
    assert abs(e - io["err_fro"]) <= 1e-10 * max(io["err_fro"], 1e-6), (e, io["err_fro"])
    assert abs(e - info["err_fro"]) <= 1e-6


def test_wide_explicit_residual_fp32_on_stored_values(lib):
    sigma = 1.0 / np.arange(1, 1301) ** 1.5
    A, _, _ = W.spectral(1500, 1300, sigma, 17)
    A32 = A.astype(np.float32)
    _, _, _, info = lib.sorsvd(dev(A32, torch.float32), 256, q=1, seed=6, residual=1)
    _, _, _, io = osvd.sorsvd(A32.astype(np.float64), 256, q=1, seed=6)
    assert abs(info["err_fro_explicit"] - io["err_fro"]) <= 1e-3 * io["err_fro"]


def test_wide_deterministic_repeat(lib):
    A, _, _ = W.spectral(800, 700, 0.99 ** np.arange(700), 3)
    Ad = dev(A)
    plan = lib.Plan(800, 700, 300, 1, torch.float64)
    U1, S1, V1 = [t.clone() for t in plan.run(Ad, seed=4)]
    U2, S2, V2 = plan.run(Ad, seed=4)
    assert torch.equal(U1, U2) and torch.equal(S1, S2) and torch.equal(V1, V2)
