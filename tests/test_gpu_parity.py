"""Parity of the HIP path (through the C ABI) with the CPU FP64 oracle.

Tolerances (stated from the arithmetic of each path):
  FP64 passes: sigma normwise max_j |s_j - s_j^or| / s_1^or <= 1e-10; factors
               equal up to column sign to 1e-8 where the spectrum gap allows;
               Q^T Q - I <= 1e-12.
  FP32 passes: the oracle runs on the stored FP32 values (exact in FP64); the
               passes commit a backward error of about u32 ||A|| sqrt(K), so
               sigma normwise <= 1e-4 (observed ~1e-6).
  Omega and other integer-determined results: bitwise.
"""
import numpy as np
import pytest

import workloads as W
from oracle import normal as onormal
from oracle import sorsvd as osvd

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x)).to(dtype).cuda()


def host(t):
    return t.detach().double().cpu().numpy()


def normwise(s, s_ref):
    return float(np.max(np.abs(np.asarray(s) - np.asarray(s_ref))) / np.asarray(s_ref)[0])


def align_signs(X, X_ref):
    d = np.sign(np.sum(X * X_ref, axis=0))
    d[d == 0] = 1
    return X * d[None, :]


def subspace_sin(X, Xo):
    """Sine of the largest principal angle between span(X) and span(Xo)
    (orthonormal columns): sqrt(1 - sigma_min(Xo^T X)^2)."""
    c = np.linalg.svd(Xo.T @ X, compute_uv=False)
    return float(np.sqrt(max(0.0, 1.0 - float(np.min(c)) ** 2)))


def fp32_factor_check(U, V, Uo, Vo, So, K, c=64.0, cap=1e-2):
    """Columns of FP32 factors against the oracle's (on the stored values).

    The FP32 passes commit a backward error of about u32 sqrt(K) ||A||_2
    (K the longest contraction); a singular vector moves by at most that over
    its gap (Wedin), so column j must satisfy
        max |u_j - u_j^or| <= c u32 sqrt(K) sigma_1 / gap_j,
    gap_j = min(sigma_{j-1} - sigma_j, sigma_j - sigma_{j+1}) of the oracle's
    values, checked where that bound is below `cap` (the other columns sit in
    clusters where only their span is determined). Returns the largest
    observed |du_j| gap_j / (u32 sqrt(K) sigma_1) (the margin against c)."""
    k = So.size
    gaps = np.full(k, np.inf)
    d = np.abs(np.diff(So))
    gaps[:-1] = np.minimum(gaps[:-1], d)
    gaps[1:] = np.minimum(gaps[1:], d)
    unit = 2.0 ** -24 * np.sqrt(K) * So[0]
    bound = c * unit / gaps
    ok = (bound < cap) & np.isfinite(gaps)   # k = 1: no neighbour known, no gap
    worst = 0.0
    for X, Xo in ((U, Uo), (V, Vo)):
        dev = np.abs(align_signs(X, Xo) - Xo).max(axis=0)
        assert np.all(dev[ok] <= bound[ok]), (np.nonzero(dev[ok] > bound[ok])[0], dev[ok].max(),
                                              "c needed", float(np.max(dev[ok] * gaps[ok] / unit)))
        if ok.any():
            worst = max(worst, float(np.max(dev[ok] * gaps[ok] / unit)))
    return worst


# ------------------------------------------------------------------ Omega

@pytest.mark.parametrize("seed,rows,cols", [(1, 800, 20), (7, 37, 5), (12345, 1001, 33), (2**63 + 5, 4, 1)])
def test_omega_bitwise_equal_to_oracle(lib, seed, rows, cols):
    got = host(lib.philox_normal(seed, rows, cols))
    ref = onormal.gaussian_matrix(seed, rows, cols)
    assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))


def test_omega_streams_and_word2(lib):
    got = host(lib.philox_normal(3, 50, 4, stream_id=9, word2=2))
    ref = onormal.gaussian_matrix(3, 50, 4, stream=9, word2=2)
    assert np.array_equal(got, ref)


# ------------------------------------------------------------------ single steps

@pytest.mark.parametrize("m,n,l", [(1000, 800, 20), (257, 131, 7), (64, 4000, 48), (3000, 129, 128)])
def test_sketch_and_orbit_fp64(lib, m, n, l):
    gen = W.rng(m + n + l)
    A = gen.standard_normal((m, n))
    X = gen.standard_normal((n, l))
    Y = gen.standard_normal((m, l))
    Ad = dev(A)
    T = host(lib.step_sketch(Ad, dev(X)))
    ref = osvd.sketch(A, X)
    assert np.abs(T - ref).max() <= 1e-13 * np.abs(A).max() * np.abs(X).max() * n
    T2 = host(lib.step_orbit(Ad, dev(Y)))
    ref2 = osvd.orbit(A, Y)
    assert np.abs(T2 - ref2).max() <= 1e-13 * np.abs(A).max() * np.abs(Y).max() * m


def test_sketch_and_orbit_fp64_strided_lda(lib):
    gen = W.rng(5)
    big = gen.standard_normal((300, 211))
    A = big[:, :197]
    Ad = dev(big)[:, :197]
    assert Ad.stride(0) == 211
    X = gen.standard_normal((197, 19))
    Y = gen.standard_normal((300, 19))
    assert np.abs(host(lib.step_sketch(Ad, dev(X))) - A @ X).max() < 1e-11
    assert np.abs(host(lib.step_orbit(Ad, dev(Y))) - A.T @ Y).max() < 1e-11


@pytest.mark.parametrize("m,n,l", [(2000, 1500, 100), (513, 77, 9)])
def test_sketch_and_orbit_fp32(lib, m, n, l):
    gen = W.rng(m * 3 + l)
    A32 = gen.standard_normal((m, n)).astype(np.float32)
    A = A32.astype(np.float64)  # stored values, exact
    X = gen.standard_normal((n, l))
    Y = gen.standard_normal((m, l))
    Ad = dev(A32, torch.float32)
    T = host(lib.step_sketch(Ad, dev(X)))
    ref = A @ X.astype(np.float32).astype(np.float64)
    scale = np.sqrt(n) * np.abs(A).max() * np.abs(X).max()
    assert np.abs(T - ref).max() <= 2e-6 * scale
    T2 = host(lib.step_orbit(Ad, dev(Y)))
    ref2 = A.T @ Y.astype(np.float32).astype(np.float64)
    assert np.abs(T2 - ref2).max() <= 2e-6 * np.sqrt(m) * np.abs(A).max() * np.abs(Y).max()


@pytest.mark.parametrize("rows,l,cond", [(1000, 20, 1e2), (20000, 100, 1e4), (333, 17, 1e7), (64, 64, 10.0),
                                         (5000, 128, 1e9), (3000, 77, 1e11)])
def test_qr_matches_householder_with_positive_diagonal(lib, rows, l, cond):
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
    # unique thin QR: agreement limited by conditioning
    assert np.abs(Q - Qo).max() <= 1e-15 * cond * 100 * np.sqrt(rows)


def test_project_fp64(lib):
    gen = W.rng(11)
    A = gen.standard_normal((700, 500))
    Q1 = W.haar_columns(700, 30, gen)
    Q2 = W.haar_columns(500, 30, gen)
    M = host(lib.step_project(dev(A), dev(Q1), dev(Q2)))
    assert np.abs(M - osvd.projection(A, Q1, Q2)).max() < 1e-12


# widths of every row-block variant (l <= 8, 16, 32, 48, 64, 80, 104, 128) and
# of uneven level ranges of the pair order; V in the kernel up to 32, rebuilt
# from the rotation log above
@pytest.mark.parametrize("l,k", [(20, 20), (100, 100), (64, 10), (128, 128), (7, 3), (1, 1), (2, 2), (3, 3),
                                 (11, 11), (33, 30), (47, 47), (72, 50), (81, 81), (105, 105)])
def test_core_svd_against_lapack(lib, l, k):
    gen = W.rng(l * 7 + k)
    Mtx = gen.standard_normal((l, l)) @ np.diag(np.geomspace(1, 1e-6, l)) @ gen.standard_normal((l, l))
    Ut, s, Vt, info = lib.step_core_svd(dev(Mtx), k)
    Ut, s, Vt = host(Ut), host(s), host(Vt)
    Ur, sr, Vrt = np.linalg.svd(Mtx)
    assert normwise(s, sr[:k]) <= 1e-13
    assert np.all(np.diff(s) <= 0)
    assert info["flags"] == 0 and 1 <= info["sweeps"] <= 40
    gap_ok = np.ones(k, dtype=bool)
    rel_gap = np.abs(np.diff(sr)) / sr[0]
    gap_ok[:-1] &= rel_gap[:k - 1] > 1e-6
    gap_ok[1:] &= rel_gap[:k - 1] > 1e-6
    Ua = align_signs(Ut, Ur[:, :k])
    Va = align_signs(Vt, Vrt[:k].T)
    assert np.abs(Ua - Ur[:, :k])[:, gap_ok].max(initial=0) < 1e-8
    assert np.abs(Va - Vrt[:k].T)[:, gap_ok].max(initial=0) < 1e-8
    assert np.abs(Ut.T @ Ut - np.eye(k)).max() < 1e-12


@pytest.mark.parametrize("l", [33, 65, 99, 127])
def test_core_svd_rotation_log_matches_v_in_kernel(lib, l):
    """Above width 32 V is rebuilt from the logged rotations; a sweep cap above
    the one the workspace log holds (40) keeps V in the Jacobi kernel. Both
    apply the same rotations in the same order to the same start (the
    identity), so they agree to rounding; odd widths add the padding column."""
    gen = W.rng(l)
    Mtx = gen.standard_normal((l, l)) @ np.diag(np.geomspace(1, 1e-3, l)) @ gen.standard_normal((l, l))
    k = l - 3
    Ua, sa, Va, ia = lib.step_core_svd(dev(Mtx), k)
    Ub, sb, Vb, ib = lib.step_core_svd(dev(Mtx), k, max_sweeps=60)
    assert ia["flags"] == ib["flags"] == 0
    assert normwise(host(sa), host(sb)) <= 1e-14
    assert np.abs(host(Ua) - host(Ub)).max() < 1e-11
    assert np.abs(host(Va) - host(Vb)).max() < 1e-11
    Vh = host(Va)
    assert np.abs(Vh.T @ Vh - np.eye(k)).max() < 1e-13
    # M V = U diag(s)
    assert np.abs(Mtx @ Vh - host(Ua) * host(sa)[None, :]).max() < 1e-12 * np.abs(host(sa)).max()


@pytest.mark.parametrize("l", [40, 100, 128])
@pytest.mark.parametrize("sweeps", [1, 2, 3])
def test_core_svd_sweep_cap_replays_every_sweep(lib, l, sweeps):
    """A sweep cap that stops the Jacobi before convergence: the V replay then
    applies every logged sweep (a converged run's last sweep rotates nothing
    and is skipped). Whatever the sweep count, the rotated columns are M V and
    U = (M V) diag(1/s), so M V = U diag(s) to rounding; a sweep left out of V
    would leave errors of the order of its rotation angles times s_1."""
    gen = W.rng(200 + l + sweeps)
    Mtx = gen.standard_normal((l, l)) @ np.diag(np.geomspace(1, 1e-3, l)) @ gen.standard_normal((l, l))
    Ut, s, Vt, info = lib.step_core_svd(dev(Mtx), l, max_sweeps=sweeps)
    Ut, s, Vt = host(Ut), host(s), host(Vt)
    assert info["sweeps"] == sweeps and (info["flags"] & 1)  # stopped at the cap
    assert np.abs(Vt.T @ Vt - np.eye(l)).max() < 1e-13
    assert np.abs(Mtx @ Vt - Ut * s[None, :]).max() <= 1e-12 * s[0]


def test_core_svd_rotation_log_no_rotation_is_a_permutation(lib):
    """A diagonal M (orthogonal columns) takes no rotation: every logged pair
    is the identity and V is the permutation that sorts the values."""
    l = 70
    gen = W.rng(3)
    d = gen.permutation(np.arange(1, l + 1)).astype(np.float64)
    Ut, s, Vt, info = lib.step_core_svd(dev(np.diag(d)), l)
    order = np.argsort(-d, kind="stable")
    assert np.array_equal(host(s), d[order])
    P = np.eye(l)[:, order]
    assert np.array_equal(np.abs(host(Vt)), P)
    # U = M V diag(1/s): a column of M times a reciprocal, exact to one rounding
    assert np.abs(np.abs(host(Ut)) - P).max() <= 2.0 ** -52


# ------------------------------------------------------------------ whole method

def check_against_oracle(lib, A_np, A_dev, k, q, seed, l=None, tol_s=1e-10, tol_vec=1e-8, pass_efficient=0):
    opts = {} if l is None else {"l": l}
    if pass_efficient:
        opts["pass_efficient"] = 1
    U, S, V, info = lib.sorsvd(A_dev, k, q=q, seed=seed, **opts)
    U, S, V = host(U), host(S), host(V)
    Uo, So, Vo, io = osvd.sorsvd(A_np, k, q=q, seed=seed, l=l, m_form="approx" if pass_efficient else "exact")
    assert normwise(S, So) <= tol_s, normwise(S, So)
    assert np.all(np.diff(S) <= 0)
    kk = k
    assert np.abs(U.T @ U - np.eye(kk)).max() < 1e-11
    assert np.abs(V.T @ V - np.eye(kk)).max() < 1e-11
    # sign convention holds on the device result
    idx = np.argmax(np.abs(U), axis=0)
    assert np.all(U[idx, np.arange(kk)] > 0)
    # factors equal up to sign where singular values are separated
    rel_gap = np.abs(np.diff(So)) / So[0]
    ok = np.ones(kk, dtype=bool)
    ok[:-1] &= rel_gap > 1e-6
    ok[1:] &= rel_gap > 1e-6
    if ok.any():
        assert np.abs(align_signs(U, Uo) - Uo)[:, ok].max() < tol_vec
        assert np.abs(align_signs(V, Vo) - Vo)[:, ok].max() < tol_vec
    assert abs(info["a_fro"] - io["a_fro"]) <= 1e-12 * io["a_fro"]
    assert info["flags"] == 0
    return S, So, info, io


def test_c1_fp64_end_to_end(lib):
    A = W.c1()
    S, So, info, io = check_against_oracle(lib, A, dev(A), 20, 0, 1)
    # error record (identity) against the oracle's explicit residual
    assert abs(info["err_fro"] - io["err_fro"]) <= 1e-10 * max(io["err_fro"], 1e-6) + 1e-12


@pytest.mark.parametrize("m,n,k,q,l", [
    (300, 200, 10, 0, None), (300, 200, 10, 2, None), (200, 300, 12, 1, None),
    (517, 389, 17, 1, 29), (1000, 64, 64, 0, None), (64, 1000, 5, 3, 16), (2000, 1200, 128, 1, None),
])
def test_fp64_shapes_and_power_steps(lib, m, n, k, q, l):
    sigma = 1.0 / np.arange(1, min(m, n) + 1) ** 1.5
    A, _, _ = W.spectral(m, n, sigma, m + n + k)
    check_against_oracle(lib, A, dev(A), k, q, 3, l=l, tol_s=1e-10, tol_vec=1e-7)


def test_exact_rank_reconstruction_fp64(lib):
    gen = W.rng(77)
    A = gen.standard_normal((400, 12)) @ gen.standard_normal((12, 300))
    U, S, V, info = lib.sorsvd(dev(A), 12, q=1, seed=5)
    U, S, V = host(U), host(S), host(V)
    assert np.abs(A - (U * S) @ V.T).max() <= 1e-11 * np.abs(A).max()
    assert info["err_fro"] < 1e-6


def test_full_width_sketch_equals_svd(lib):
    A = W.rng(8).standard_normal((90, 70))
    _, S, _, _ = lib.sorsvd(dev(A), 70, q=0, seed=2)
    assert normwise(host(S), np.linalg.svd(A, compute_uv=False)) <= 1e-12


@pytest.mark.parametrize("m,n,k,q", [(2000, 1500, 100, 1), (1500, 2000, 64, 0), (777, 555, 33, 2)])
def test_fp32_against_oracle_on_stored_values(lib, m, n, k, q):
    sigma = 1.0 / np.arange(1, min(m, n) + 1) ** 2
    A, _, _ = W.spectral(m, n, sigma, 2)
    A32 = A.astype(np.float32)
    A64 = A32.astype(np.float64)
    U, S, V, info = lib.sorsvd(dev(A32, torch.float32), k, q=q, seed=9)
    U, S, V = host(U), host(S), host(V)
    Uo, So, Vo, io = osvd.sorsvd(A64, k, q=q, seed=9)
    assert normwise(S, So) <= 1e-5  # bar 1e-4; observed accuracy margin
    assert np.abs(U.T @ U - np.eye(k)).max() < 1e-11 and np.abs(V.T @ V - np.eye(k)).max() < 1e-11
    worst = fp32_factor_check(U, V, Uo, Vo, So, max(m, n))
    print(f"fp32 {m}x{n} k={k} q={q}: factor deviation {worst:.2f} u32 sqrt(K) sigma_1 / gap")


def test_deterministic_repeat(lib):
    A = dev(W.c1())
    plan = lib.Plan(1000, 800, 20, 1, torch.float64)
    U1, S1, V1 = [t.clone() for t in plan.run(A, seed=4)]
    U2, S2, V2 = plan.run(A, seed=4)
    assert torch.equal(U1, U2) and torch.equal(S1, S2) and torch.equal(V1, V2)


def test_nonfinite_input_is_flagged(lib):
    A = W.rng(3).standard_normal((200, 150))
    A[17, 33] = np.nan
    _, _, _, info = lib.sorsvd(dev(A), 5, q=0, seed=1)
    assert info["flags"] & 2


def test_seed_changes_draw_not_leading_values(lib):
    # with l = k the trailing estimates depend on the draw (Th. 4: the factor
    # (sigma_{l-p+1}/sigma_j)^(4q+4) is close to 1 for j near k); the leading
    # ones do not, and all stay below the true values (Th. 3).
    sigma = 0.7 ** np.arange(120)
    A, _, _ = W.spectral(300, 120, sigma, 4)
    _, S1, _, _ = lib.sorsvd(dev(A), 10, q=1, seed=1)
    _, S2, _, _ = lib.sorsvd(dev(A), 10, q=1, seed=2)
    S1, S2 = host(S1), host(S2)
    assert not np.array_equal(S1, S2)
    assert np.all(S1 <= sigma[:10] * (1 + 1e-12)) and np.all(S2 <= sigma[:10] * (1 + 1e-12))
    assert normwise(S1[:5], S2[:5]) < 1e-4


# ------------------------------------------------------------------ explicit residual (error check)

@pytest.mark.parametrize("m,n,k,q", [(1000, 800, 20, 0), (333, 1200, 48, 1), (2500, 700, 128, 1)])
def test_explicit_residual_fp64(lib, m, n, k, q):
    A = W.low_rank_plus_noise(m, n, 30, 1e-3, m + n + k)
    U, S, V, info = lib.sorsvd(dev(A), k, q=q, seed=5, residual=1)
    _, _, _, io = osvd.sorsvd(A, k, q=q, seed=5)
    e = info["err_fro_explicit"]
    assert abs(e - io["err_fro"]) <= 1e-10 * max(io["err_fro"], 1e-6), (e, io["err_fro"])
    assert info["a_noise_rel"] == 0.0
    # the explicit value and the identity agree where the error is not tiny
    assert abs(e - info["err_fro"]) <= 1e-6


def test_explicit_residual_fp32_on_stored_values(lib):
    sigma = 1.0 / np.arange(1, 1301) ** 1.5
    A, _, _ = W.spectral(1500, 1300, sigma, 17)
    A32 = A.astype(np.float32)
    _, _, _, info = lib.sorsvd(dev(A32, torch.float32), 40, q=1, seed=6, residual=1)
    _, _, _, io = osvd.sorsvd(A32.astype(np.float64), 40, q=1, seed=6)
    assert abs(info["err_fro_explicit"] - io["err_fro"]) <= 1e-3 * io["err_fro"]


def test_residual_of_exact_low_rank_is_tiny(lib):
    gen = W.rng(44)
    A = gen.standard_normal((700, 12)) @ gen.standard_normal((12, 530))
    _, _, _, info = lib.sorsvd(dev(A), 12, q=0, seed=2, residual=1)
    assert info["err_fro_explicit"] < 1e-13


# ------------------------------------------------------------------ pass-efficient core matrix

@pytest.mark.parametrize("m,n,k,q,l", [(300, 200, 10, 0, None), (517, 389, 17, 1, 29), (200, 300, 12, 2, None),
                                       (2000, 1200, 128, 1, None)])
def test_pass_efficient_fp64_against_oracle(lib, m, n, k, q, l):
    sigma = 1.0 / np.arange(1, min(m, n) + 1) ** 1.5
    A, _, _ = W.spectral(m, n, sigma, m + 2 * n + k)
    S, So, info, io = check_against_oracle(lib, A, dev(A), k, q, 4, l=l, tol_s=1e-10, tol_vec=1e-7,
                                           pass_efficient=1)
    # the Th. 2 identity stays exact: the core matrix is Q1^T A Q2
    assert abs(info["err_fro"] - io["err_fro"]) <= 1e-9 * max(io["err_fro"], 1e-6)


def test_pass_efficient_fp32_against_oracle_on_stored_values(lib):
    sigma = 1.0 / np.arange(1, 1501) ** 2
    A, _, _ = W.spectral(2000, 1500, sigma, 2)
    A32 = A.astype(np.float32)
    U, S, V, info = lib.sorsvd(dev(A32, torch.float32), 100, q=1, seed=9, pass_efficient=1)
    U, S, V = host(U), host(S), host(V)
    Uo, So, Vo, io = osvd.sorsvd(A32.astype(np.float64), 100, q=1, seed=9, m_form="approx")
    assert normwise(S, So) <= 1e-5
    worst = fp32_factor_check(U, V, Uo, Vo, So, 2000)
    print(f"fp32 pass-efficient: factor deviation {worst:.2f} u32 sqrt(K) sigma_1 / gap")


def test_pass_efficient_equals_exact_core_to_rounding(lib):
    # same Q1, Q2 in both forms; the core matrices agree to FP64 rounding
    A, _, _ = W.spectral(800, 600, 0.97 ** np.arange(600), 5)
    _, S1, _, i1 = lib.sorsvd(dev(A), 40, q=1, seed=3)
    _, S2, _, i2 = lib.sorsvd(dev(A), 40, q=1, seed=3, pass_efficient=1)
    assert normwise(host(S1), host(S2)) <= 1e-12
    assert abs(i1["err_fro"] - i2["err_fro"]) <= 1e-10


# ------------------------------------------------------------------ literal Alg. 4 mode, FP32 outputs

@pytest.mark.parametrize("m,n,k,q,l", [(400, 300, 20, 0, None), (400, 300, 20, 2, None), (350, 500, 16, 1, 24)])
def test_literal_mode_against_oracle_literal(lib, m, n, k, q, l):
    """Alg. 4 as printed (no QR between the products) against the oracle's
    literal mode, on a well-conditioned spectrum: the products' condition
    number (sigma_1 / sigma_l)^(2q+2) stays below ~10, so both QRs are
    accurate to rounding and the results agree to the FP64 bar; the spans
    equal those of the default mode (Lemma 1)."""
    sigma = 0.99 ** np.arange(min(m, n))
    A, _, _ = W.spectral(m, n, sigma, m + n + q)
    U, S, V, info = lib.sorsvd(dev(A), k, q=q, seed=2, l=l or 0, literal=1)
    U, S, V = host(U), host(S), host(V)
    Uo, So, Vo, io = osvd.sorsvd(A, k, q=q, seed=2, l=l, mode="literal")
    assert normwise(S, So) <= 1e-10
    assert abs(info["err_fro"] - io["err_fro"]) <= 1e-9
    _, Sc, _, _ = lib.sorsvd(dev(A), k, q=q, seed=2, l=l or 0)
    assert normwise(host(Sc), S) <= 1e-10
    assert np.abs(U.T @ U - np.eye(k)).max() < 1e-11 and info["flags"] == 0


def test_fp32_outputs_are_the_rounded_fp64_outputs(lib):
    A, _, _ = W.spectral(600, 400, 1.0 / np.arange(1, 401) ** 1.5, 5)
    Ad = dev(A.astype(np.float32), torch.float32)
    U, S, V, _ = lib.sorsvd(Ad, 32, q=1, seed=3)
    U32, S32, V32, _ = lib.sorsvd(Ad, 32, q=1, seed=3, out_f32=1)
    assert U32.dtype == torch.float32 and V32.dtype == torch.float32
    assert torch.equal(S, S32)
    assert torch.equal(U.float(), U32) and torch.equal(V.float(), V32)


@pytest.mark.parametrize("shape,k,q,dt", [((1000, 800), 20, 0, "f64"), ((2000, 1500), 256, 1, "f32")])
def test_graph_replay_equals_eager(lib, shape, k, q, dt):
    """The launch sequence of one SOR-SVD captured in a HIP graph: every replay
    (with eager work and synchronisation between them) reproduces the eager
    result bitwise, also after A changes in place."""
    m, n = shape
    dtype = torch.float64 if dt == "f64" else torch.float32
    A, _, _ = W.spectral(m, n, 1.0 / np.arange(1, min(m, n) + 1), 12)
    Ad = dev(A, dtype)
    plan = lib.Plan(m, n, k, q, dtype)
    U0, S0, V0 = [t.clone() for t in plan.run(Ad, seed=3)]
    g = plan.capture(Ad, seed=3)
    for _ in range(3):
        plan.U.zero_()
        plan.S.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(plan.U, U0) and torch.equal(plan.S, S0) and torch.equal(plan.V, V0)
    Ad.mul_(2.0)  # exact scaling: the replay follows the new contents of A
    g.replay()
    torch.cuda.synchronize()
    assert torch.equal(plan.S, 2.0 * S0)
