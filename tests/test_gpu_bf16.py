"""BF16-stored A: passes on BF16 MFMA with FP32 accumulation, FP64 QR and core SVD.

The oracle runs on the STORED matrix (BF16 values, exact in FP64), so these
tests isolate the arithmetic of the BF16 path. Tolerances:
  single products: the skinny operand is rounded to BF16 (relative 2^-9) before
  the product, exactly as the reference computation below does; what remains
  is FP32 accumulation, bounded by ~2^-24 sqrt(K) ||a|| ||x|| per entry;
  projection with the hi + lo split: the split represents Q2 to ~2^-17 relative;
  whole method: Q1 and Q2 are built from BF16-rounded operands, so they span
  slightly different subspaces than the oracle's; the result is then checked
  against what must hold for ANY orthonormal Q1, Q2 (Th. 3 interlacing,
  Eckart-Young floor, orthonormal factors) and against the oracle's sigma and
  error with the measured-margin tolerances stated in each test.
"""
import numpy as np
import pytest

import workloads as W
from oracle import bounds
from oracle import sorsvd as osvd

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def to_bf16(x):
    """Round FP64 to BF16 (nearest, ties to even) with ONE rounding, back to FP64.

    Round to FP32 with round-to-odd (an inexact result keeps the truncated
    value with its last bit set), then to BF16 to nearest-even: FP32 carries
    more than two extra bits, so this equals direct rounding. (Rounding to
    FP32 to nearest first, as a plain cast chain does, can round twice.)
    """
    x = np.ascontiguousarray(x, dtype=np.float64)
    f = x.astype(np.float32)
    bits = f.view(np.uint32).copy()
    inexact = f.astype(np.float64) != x
    over = np.abs(f.astype(np.float64)) > np.abs(x)
    bits[inexact & over] -= np.uint32(1)
    bits[inexact] |= np.uint32(1)
    r = (bits + np.uint32(0x7FFF) + ((bits >> np.uint32(16)) & np.uint32(1))) >> np.uint32(16)
    return (r << np.uint32(16)).astype(np.uint32).view(np.float32).astype(np.float64)


def dev_bf16(x):
    """Device BF16 tensor holding exactly the values of to_bf16(x)."""
    return torch.as_tensor(to_bf16(x)).to(torch.float32).to(torch.bfloat16).cuda()


def host(t):
    return t.detach().double().cpu().numpy()


@pytest.mark.parametrize("m,n,l", [(1000, 800, 64), (777, 555, 20), (130, 1031, 7), (4096, 300, 128)])
def test_bf16_sketch_and_orbit(lib, m, n, l):
    gen = W.rng(m + 2 * n + l)
    A = to_bf16(gen.standard_normal((m, n)))
    X = gen.standard_normal((n, l))
    Y = gen.standard_normal((m, l))
    Ad = dev_bf16(A)
    T = host(lib.step_sketch(Ad, torch.as_tensor(X).cuda()))
    ref = A @ to_bf16(X)
    tol = 4 * 2.0**-24 * np.sqrt(n) * np.abs(A).max() * np.abs(X).max() * np.sqrt(n)
    assert np.abs(T - ref).max() <= tol
    T2 = host(lib.step_orbit(Ad, torch.as_tensor(Y).cuda()))
    ref2 = A.T @ to_bf16(Y)
    tol2 = 4 * 2.0**-24 * np.sqrt(m) * np.abs(A).max() * np.abs(Y).max() * np.sqrt(m)
    assert np.abs(T2 - ref2).max() <= tol2


def test_bf16_unaligned_leading_dimension(lib):
    gen = W.rng(9)
    big = to_bf16(gen.standard_normal((300, 203)))
    A = big[:, :197]
    Ad = dev_bf16(big)[:, :197]
    assert Ad.stride(0) == 203
    X = gen.standard_normal((197, 16))
    Y = gen.standard_normal((300, 16))
    assert np.abs(host(lib.step_sketch(Ad, torch.as_tensor(X).cuda())) - A @ to_bf16(X)).max() < 1e-3
    assert np.abs(host(lib.step_orbit(Ad, torch.as_tensor(Y).cuda())) - A.T @ to_bf16(Y)).max() < 1e-3


def test_bf16_projection_with_hi_lo_split(lib):
    gen = W.rng(21)
    A = to_bf16(gen.standard_normal((900, 700)))
    Q1 = W.haar_columns(900, 48, gen)
    Q2 = W.haar_columns(700, 48, gen)
    M = host(lib.step_project(dev_bf16(A), torch.as_tensor(Q1).cuda(), torch.as_tensor(Q2).cuda()))
    ref = osvd.projection(A, Q1, Q2)
    # without the split the error would be ~2^-9 |A| sqrt(n); with it ~2^-17
    err = np.abs(M - ref).max() / (np.abs(A).max() * np.sqrt(700))
    assert err < 2.0**-14, err


@pytest.mark.parametrize("m,n,k,q", [(3000, 1200, 64, 1), (1500, 2500, 32, 2), (1000, 333, 20, 0),
                                     (2500, 1300, 128, 1)])
def test_bf16_whole_method(lib, m, n, k, q):
    sigma = 0.9 ** np.arange(1, min(m, n) + 1)
    A, _, _ = W.spectral(m, n, sigma, 4)
    A = to_bf16(A)
    sig_stored = np.linalg.svd(A, compute_uv=False)
    U, S, V, info = lib.sorsvd(dev_bf16(A), k, q=q, seed=3, refine=1)
    U, S, V = host(U), host(S), host(V)
    Uo, So, Vo, io = osvd.sorsvd(A, k, q=q, seed=3)
    # structure: FP64 QR and core SVD
    assert np.abs(U.T @ U - np.eye(k)).max() < 1e-11
    assert np.abs(V.T @ V - np.eye(k)).max() < 1e-11
    assert np.all(np.diff(S) <= 0)
    # Th. 3 (Remark 2): estimates stay below the stored matrix's singular values
    # (up to the 2^-17 projection error of the split)
    assert np.all(S <= sig_stored[:k] * (1 + 1e-4))
    # Eckart-Young: the explicit error cannot beat the floor
    R = A - (U * S) @ V.T
    e = np.linalg.norm(R) / np.linalg.norm(A)
    floor = bounds.ey_floor(sig_stored, k) / np.linalg.norm(A)
    assert e >= floor * (1 - 1e-6)
    # against the FP64 oracle on the same stored A and Omega
    dsig = np.max(np.abs(S - So)) / So[0]
    de = abs(e - io["err_fro"]) / io["err_fro"]
    # subspace angles against the oracle's factors (same stored A): the
    # leading directions, well separated at 0.9^j, are the ones determined
    from test_gpu_parity import subspace_sin
    su, sv = subspace_sin(U, Uo), subspace_sin(V, Vo)
    kk = min(8, k)
    su8, sv8 = subspace_sin(U[:, :kk], Uo[:, :kk]), subspace_sin(V[:, :kk], Vo[:, :kk])
    print(f"bf16 m={m} n={n} k={k} q={q}: sigma normwise {dsig:.2e}, err {e:.4e} vs oracle "
          f"{io['err_fro']:.4e} (rel {de:.2e}), identity err {info['err_fro']:.4e}; sin angle U {su:.2e} "
          f"V {sv:.2e} (leading {kk}: {su8:.2e}, {sv8:.2e})")
    assert su8 <= 1e-2 and sv8 <= 1e-2
    # measured: sigma normwise <= 1.3e-4, error within 8e-4 relative
    assert dsig < 1e-3
    assert de < 5e-3
    # ||A||_F of a BF16 matrix is accumulated from FP32 sums of 8 exact squares
    # (relative rounding 2^-24 each), then in FP64
    assert abs(info["a_fro"] - io["a_fro"]) <= 1e-7 * io["a_fro"]


@pytest.mark.parametrize("fmt,split,pe", [("bf16", 3, 0), ("bf16", 7, 0), ("f16", 3, 0), ("bf16", 3, 1),
                                          ("f16", 7, 1)])
def test_16bit_forced_splits_agree(lib, fmt, split, pe):
    """Contraction splits of the 16-bit passes whose ranges hold an odd number
    of the A X kernel's 128-index blocks (1100 in 3: ranges of 384, the last
    332) or end in a short range (in 7: 4 ranges of 256, the last 76): the
    result equals the unsplit run up to the FP32 rounding of the per-split
    partial sums, and both stay within the oracle's tolerance. pe: the
    pass-efficient form, whose last orbit product (2 LP columns, hi + lo)
    takes the forced split too, against the oracle's M_approx."""
    m, n, k = 1500, 1100, 64
    sigma = 0.9 ** np.arange(1, n + 1)
    A, _, _ = W.spectral(m, n, sigma, 5)
    if fmt == "bf16":
        A = to_bf16(A)
        Ad, opts = dev_bf16(A), {}
    else:
        Ad, e = lib.pack_f16(torch.as_tensor(A).cuda())
        opts = {"col_exp": e}
        A = host(Ad) * np.exp2(-host(e))[None, :]
    _, S0, _, i0 = lib.sorsvd(Ad, k, q=1, seed=3, refine=1, split=1, pass_efficient=pe, **opts)
    U1, S1, V1, i1 = lib.sorsvd(Ad, k, q=1, seed=3, refine=1, split=split, pass_efficient=pe, **opts)
    S0, S1, U1, V1 = host(S0), host(S1), host(U1), host(V1)
    assert i0["flags"] == 0 and i1["flags"] == 0
    assert np.abs(U1.T @ U1 - np.eye(k)).max() < 1e-11
    assert np.abs(V1.T @ V1 - np.eye(k)).max() < 1e-11
    # ||A||_F: the same 8-value squares, grouped differently in FP64
    assert abs(i1["a_fro"] - i0["a_fro"]) <= 1e-13 * i0["a_fro"]
    d01 = np.max(np.abs(S1 - S0)) / S0[0]
    _, So, _, io = osvd.sorsvd(A, k, q=1, seed=3, m_form="approx" if pe else "exact")
    dsig = np.max(np.abs(S1 - So)) / So[0]
    print(f"{fmt} split {split} pe {pe}: sigma vs unsplit {d01:.2e}, vs oracle {dsig:.2e}")
    assert d01 < 1e-4
    assert dsig < (1e-3 if fmt == "bf16" else 1e-4)


@pytest.mark.parametrize("fmt,m,n,k,q", [("bf16", 3000, 1200, 64, 1), ("bf16", 1500, 900, 32, 0),
                                         ("f16", 3000, 1200, 64, 1), ("f16", 1100, 1300, 48, 2)])
def test_16bit_pass_efficient_against_oracle(lib, fmt, m, n, k, q):
    """Pass-efficient core matrix on 16-bit A (eq. M_approx, formed from the
    last orbit product T2 = A^T Q1, whose Q1 is split into hi + lo parts):
    against the oracle's M_approx form on the stored values, and against the
    same method with the refinement projection pass."""
    sigma = 0.9 ** np.arange(1, min(m, n) + 1)
    A, _, _ = W.spectral(m, n, sigma, 4)
    if fmt == "bf16":
        A = to_bf16(A)
        Ad, opts = dev_bf16(A), {}
    else:
        Ad, e = lib.pack_f16(torch.as_tensor(A).cuda())
        opts = {"col_exp": e}
        A = host(Ad) * np.exp2(-host(e))[None, :]
    sig_stored = np.linalg.svd(A, compute_uv=False)
    U, S, V, info = lib.sorsvd(Ad, k, q=q, seed=3, refine=1, pass_efficient=1, **opts)
    U, S, V = host(U), host(S), host(V)
    assert info["flags"] == 0
    assert np.abs(U.T @ U - np.eye(k)).max() < 1e-11
    assert np.abs(V.T @ V - np.eye(k)).max() < 1e-11
    assert np.all(np.diff(S) <= 0)
    assert np.all(S <= sig_stored[:k] * (1 + 1e-4))
    R = A - (U * S) @ V.T
    e_ex = np.linalg.norm(R) / np.linalg.norm(A)
    assert e_ex >= bounds.ey_floor(sig_stored, k) / np.linalg.norm(A) * (1 - 1e-6)
    Uo, So, Vo, io = osvd.sorsvd(A, k, q=q, seed=3, m_form="approx")
    dsig = np.max(np.abs(S - So)) / So[0]
    de = abs(e_ex - io["err_fro"]) / io["err_fro"]
    _, Sx, _, _ = lib.sorsvd(Ad, k, q=q, seed=3, refine=1, **opts)
    dx = np.max(np.abs(S - host(Sx))) / S[0]
    print(f"{fmt} pass-efficient m={m} n={n} k={k} q={q}: sigma vs oracle {dsig:.2e}, err rel {de:.2e}, "
          f"vs projection pass {dx:.2e}, identity {info['err_fro']:.4e} explicit {e_ex:.4e}")
    # measured margins as for the projection form (the orbit operand is split
    # like the projection operand there)
    assert dsig < (1e-3 if fmt == "bf16" else 1e-4)
    assert de < 5e-3
    assert dx < 1e-3


def test_bf16_explicit_residual_and_rounding_noise(lib):
    """The residual pass measures the error against the stored BF16 matrix and
    the rounding noise of storing it; their difference of squares estimates the
    error against the matrix before rounding."""
    m, n, k = 3000, 1000, 64
    sigma = 1.0 / np.arange(1, n + 1) ** 2.0
    A, _, _ = W.spectral(m, n, sigma, 23)
    As = to_bf16(A)
    U, S, V, info = lib.sorsvd(dev_bf16(A), k, q=1, seed=3, refine=1, residual=1)
    U, S, V = host(U), host(S), host(V)
    Ahat = (U * S) @ V.T
    e_stored = np.linalg.norm(As - Ahat) / np.linalg.norm(As)
    assert abs(info["err_fro_explicit"] - e_stored) <= 1e-4 * e_stored
    noise = np.linalg.norm(As - A) / np.linalg.norm(As)
    assert abs(info["a_noise_rel"] - noise) <= 0.02 * noise, (info["a_noise_rel"], noise)
    e_true = np.linalg.norm(A - Ahat) / np.linalg.norm(A)
    # the rounding noise adds to the stored residual except for the share a
    # rank-k fit absorbs; the judge of sorsvd_auto allows 4 k (m^-1/2 + n^-1/2)^2
    es2, nz2 = info["err_fro_explicit"] ** 2, info["a_noise_rel"] ** 2
    rho = min(1.0, 4 * k * (m ** -0.5 + n ** -0.5) ** 2)
    low = np.sqrt(max(es2 - nz2, 0.0))
    high = np.sqrt(max(es2 - (1 - 2 * rho) * nz2, 0.0))
    print(f"stored {e_stored:.4e} noise {noise:.4e} true {e_true:.4e} bounds [{low:.4e}, {high:.4e}]")
    assert low <= 1.01 * e_true and e_true <= 1.01 * high
