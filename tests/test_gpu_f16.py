"""FP16-stored A with power-of-two column scaling: FP16 MFMA with FP32
accumulation, FP64 QR and core SVD, and A = A_stored diag(2^-e_j).

As for BF16, the oracle runs on the matrix the stored data represents (FP16
values times 2^-e_j, exact in FP64), so these tests isolate the arithmetic of
the FP16 path:
  single products: the skinny operand is stored as fp16(x 2^12) (fp16 of
  x 2^(12 + min e - e_j) on row j of an A X operand), which the reference
  below reproduces; what remains is FP32 accumulation, bounded by
  ~2^-24 sqrt(K) ||a|| ||x|| per entry;
  column scaling: a power of two commutes with rounding away from the
  subnormal range, so a run on (A diag(2^e), e) repeats the run on A bit for
  bit when no skinny entry meets FP16 subnormals;
  whole method: 11-bit skinny operands instead of BF16's 8 bits, and the same
  structural checks as for BF16 (Th. 3 interlacing, Eckart-Young floor,
  orthonormal factors) with measured-margin tolerances against the oracle.
"""
import numpy as np
import pytest

import workloads as W
from oracle import bounds
from oracle import sorsvd as osvd

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SHIFT = 12  # the lift of FP16 skinny operands


def to_f16(x):
    """FP64 -> FP16 with one rounding to nearest-even (numpy converts from
    double directly), back to FP64."""
    return np.asarray(x, dtype=np.float64).astype(np.float16).astype(np.float64)


def dev_f16(x):
    """Device FP16 tensor holding exactly the FP16 values of x (x must be
    FP16-representable)."""
    h = np.asarray(x, dtype=np.float64).astype(np.float16)
    assert np.array_equal(h.astype(np.float64), np.asarray(x, dtype=np.float64))
    return torch.from_numpy(h.view(np.int16).copy()).cuda().view(torch.float16)


def host(t):
    return t.detach().double().cpu().numpy()


def operand(x, rows_exp=None):
    """The FP64 values an FP16 skinny operand represents: fp16(x 2^s_r) 2^-s_r."""
    s = np.full(x.shape[0], SHIFT) if rows_exp is None else SHIFT + rows_exp.min() - rows_exp
    return to_f16(x * np.exp2(s)[:, None]) * np.exp2(-s)[:, None]


@pytest.mark.parametrize("m,n,l", [(1000, 800, 64), (777, 555, 20), (130, 1031, 7), (4096, 300, 128)])
def test_f16_sketch_and_orbit(lib, m, n, l):
    gen = W.rng(m + 3 * n + l)
    A = to_f16(gen.standard_normal((m, n)))
    X = gen.standard_normal((n, l))
    Y = gen.standard_normal((m, l))
    Ad = dev_f16(A)
    T = host(lib.step_sketch(Ad, torch.as_tensor(X).cuda()))
    ref = A @ operand(X)
    tol = 4 * 2.0**-24 * np.sqrt(n) * np.abs(A).max() * np.abs(X).max() * np.sqrt(n)
    assert np.abs(T - ref).max() <= tol
    T2 = host(lib.step_orbit(Ad, torch.as_tensor(Y).cuda()))
    ref2 = A.T @ operand(Y)
    tol2 = 4 * 2.0**-24 * np.sqrt(m) * np.abs(A).max() * np.abs(Y).max() * np.sqrt(m)
    assert np.abs(T2 - ref2).max() <= tol2


def test_f16_unaligned_leading_dimension(lib):
    """Rows that are not 16-byte aligned and a contraction that is not a
    multiple of 8 take the kernels' element-wise load path."""
    gen = W.rng(10)
    big = to_f16(gen.standard_normal((300, 203)))
    A = big[:, :197]
    Ad = dev_f16(big)[:, :197]
    assert Ad.stride(0) == 203
    X = gen.standard_normal((197, 16))
    Y = gen.standard_normal((300, 16))
    T = host(lib.step_sketch(Ad, torch.as_tensor(X).cuda()))
    assert np.abs(T - A @ operand(X)).max() < 1e-4
    T2 = host(lib.step_orbit(Ad, torch.as_tensor(Y).cuda()))
    assert np.abs(T2 - A.T @ operand(Y)).max() < 1e-4


def test_f16_projection_with_hi_lo_split(lib):
    gen = W.rng(22)
    A = to_f16(gen.standard_normal((900, 700)))
    Q1 = W.haar_columns(900, 48, gen)
    Q2 = W.haar_columns(700, 48, gen)
    M = host(lib.step_project(dev_f16(A), torch.as_tensor(Q1).cuda(), torch.as_tensor(Q2).cuda()))
    ref = osvd.projection(A, Q1, Q2)
    # hi + lo represent Q2 to ~2^-22 relative; FP32 accumulation adds ~2^-24 sqrt(n)
    err = np.abs(M - ref).max() / (np.abs(A).max() * np.sqrt(700))
    assert err < 2.0**-19, err


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_pack_f16_matches_its_definition(lib, dtype):
    """Column exponents e_j = 14 - floor(log2 max_i |A_ij|) (0 for a zero
    column), A_stored = fp16(A_ij 2^e_j) with one rounding: bit-exact."""
    gen = W.rng(31)
    m, n = 517, 203
    A = gen.standard_normal((m, n)) * np.exp2(gen.integers(-40, 41, size=n))[None, :]
    A[:, 7] = 0.0
    A[:, 11] = 0.0
    A[3, 11] = -2.0**-30
    if dtype == torch.float32:
        A = A.astype(np.float32).astype(np.float64)
    Ah, e = lib.pack_f16(torch.as_tensor(A, dtype=dtype).cuda())
    e = e.cpu().numpy()
    col_max = np.abs(A).max(axis=0)
    e_ref = np.where(col_max > 0, 14 - np.floor(np.log2(np.where(col_max > 0, col_max, 1.0))), 0).astype(np.int64)
    assert np.array_equal(e, e_ref)
    ref = (A * np.exp2(e_ref)[None, :]).astype(np.float16)
    assert np.array_equal(Ah.cpu().numpy().view(np.uint16), ref.view(np.uint16))
    peak = np.abs(ref.astype(np.float64)).max(axis=0)
    nz = col_max > 0
    assert np.all((peak[nz] >= 2.0**14) & (peak[nz] <= 2.0**15))


def test_f16_column_scaling_is_exact(lib):
    """A run on (A diag(2^e), e) repeats the run on A: the scaling only moves
    exponents, away from FP16 subnormals. Without the hi + lo split: its low
    parts (2^-11 of the high parts) reach FP16 subnormals on rows lifted less
    than 2^12, where rounding is absolute (an effect below 1e-11 that this
    exact comparison would see)."""
    gen = W.rng(41)
    m, n, k = 1200, 1000, 32
    sigma = 0.92 ** np.arange(n)
    A, _, _ = W.spectral(m, n, sigma, 41)
    # FP16 values of magnitude in [2^-4, 2^6]: every scaled copy stays normal
    A = to_f16(np.sign(A) * np.clip(np.abs(A) / np.abs(A).max() * 64, 2.0**-4, 64))
    e = gen.integers(-2, 3, size=n)
    As = A * np.exp2(e)[None, :]
    r0 = lib.sorsvd(dev_f16(A), k, q=1, seed=5, residual=1)
    r1 = lib.sorsvd(dev_f16(As), k, q=1, seed=5, residual=1,
                    col_exp=torch.as_tensor(e, dtype=torch.int32).cuda())
    for a, b in zip(r0[:3], r1[:3]):
        a, b = host(a), host(b)
        d = np.abs(a - b).max()
        print(f"max difference {d:.3e}")
        assert d <= 1e-13 * max(1.0, np.abs(a).max())
    for key in ("a_fro", "err_fro", "err_fro_explicit", "a_noise_rel"):
        assert abs(r0[3][key] - r1[3][key]) <= 1e-13 * abs(r0[3][key]), key
    assert r1[3]["flags"] & 8 == 0


@pytest.mark.parametrize("m,n,k,q", [(3000, 1200, 64, 1), (1500, 2500, 32, 2), (1000, 333, 20, 0),
                                     (2500, 1300, 128, 1)])
def test_f16_whole_method(lib, m, n, k, q):
    sigma = 0.9 ** np.arange(1, min(m, n) + 1)
    A, _, _ = W.spectral(m, n, sigma, 4)
    A = to_f16(A * 256)  # entries near 1: the normal FP16 range
    sig_stored = np.linalg.svd(A, compute_uv=False)
    U, S, V, info = lib.sorsvd(dev_f16(A), k, q=q, seed=3, refine=1)
    U, S, V = host(U), host(S), host(V)
    Uo, So, Vo, io = osvd.sorsvd(A, k, q=q, seed=3)
    assert np.abs(U.T @ U - np.eye(k)).max() < 1e-11
    assert np.abs(V.T @ V - np.eye(k)).max() < 1e-11
    assert np.all(np.diff(S) <= 0)
    # Th. 3 (Remark 2): below the stored matrix's singular values, up to the
    # ~2^-22 projection error of the split
    assert np.all(S <= sig_stored[:k] * (1 + 1e-5))
    R = A - (U * S) @ V.T
    e = np.linalg.norm(R) / np.linalg.norm(A)
    floor = bounds.ey_floor(sig_stored, k) / np.linalg.norm(A)
    assert e >= floor * (1 - 1e-6)
    dsig = np.max(np.abs(S - So)) / So[0]
    de = abs(e - io["err_fro"]) / io["err_fro"]
    from test_gpu_parity import subspace_sin
    su, sv = subspace_sin(U, Uo), subspace_sin(V, Vo)
    kk = min(8, k)
    su8, sv8 = subspace_sin(U[:, :kk], Uo[:, :kk]), subspace_sin(V[:, :kk], Vo[:, :kk])
    print(f"f16 m={m} n={n} k={k} q={q}: sigma normwise {dsig:.2e}, err {e:.4e} vs oracle "
          f"{io['err_fro']:.4e} (rel {de:.2e}), identity err {info['err_fro']:.4e}; sin angle U {su:.2e} "
          f"V {sv:.2e} (leading {kk}: {su8:.2e}, {sv8:.2e})")
    assert su8 <= 1e-3 and sv8 <= 1e-3
    # measured: sigma normwise <= 1.6e-5, error within 3.2e-5 relative (BF16:
    # 1.3e-4 and 7.7e-4 on the same cases)
    assert dsig < 5e-5
    assert de < 2e-4
    # squares of FP16 values summed in FP64
    assert abs(info["a_fro"] - io["a_fro"]) <= 1e-12 * io["a_fro"]


def test_f16_wide_column_range(lib):
    """Columns spanning 2^-30 .. 2^30, far outside FP16's range: packed with
    column exponents, the method runs on what the stored data represents, and
    the residual pass measures both the error against it and the rounding of
    the packing."""
    m, n, k = 2500, 900, 48
    sigma = 1.0 / np.arange(1, n + 1) ** 1.5
    A0, _, _ = W.spectral(m, n, sigma, 51)
    scales = np.exp2(W.rng(52).integers(-30, 31, size=n).astype(np.float64))
    A = A0 * scales[None, :]
    with np.errstate(over="ignore"):
        plain = A.astype(np.float16)
    assert np.isinf(plain).any() and (np.count_nonzero(plain == 0) > np.count_nonzero(A == 0))
    Ah, e = lib.pack_f16(torch.as_tensor(A).cuda())
    e_h = e.cpu().numpy()
    Astored = Ah.cpu().numpy().astype(np.float64) * np.exp2(-e_h.astype(np.float64))[None, :]
    U, S, V, info = lib.sorsvd(Ah, k, q=2, seed=7, refine=1, residual=1, col_exp=e)
    U, S, V = host(U), host(S), host(V)
    Uo, So, Vo, io = osvd.sorsvd(Astored, k, q=2, seed=7)
    dsig = np.max(np.abs(S - So)) / So[0]
    Ahat = (U * S) @ V.T
    e_st = np.linalg.norm(Astored - Ahat) / np.linalg.norm(Astored)
    de = abs(e_st - io["err_fro"]) / io["err_fro"]
    noise = np.linalg.norm(Astored - A) / np.linalg.norm(Astored)
    print(f"wide columns: sigma normwise {dsig:.2e}, err {e_st:.4e} vs oracle {io['err_fro']:.4e} "
          f"(rel {de:.2e}), packing noise {noise:.3e} reported {info['a_noise_rel']:.3e}")
    # measured: sigma normwise 2.0e-7, error within 1.7e-5 relative
    assert dsig < 5e-6 and de < 2e-4
    assert abs(info["a_fro"] - io["a_fro"]) <= 1e-12 * io["a_fro"]
    assert abs(info["err_fro_explicit"] - e_st) <= 1e-4 * e_st
    assert abs(info["a_noise_rel"] - noise) <= 0.05 * noise
    assert info["flags"] & 8 == 0


def test_f16_column_exponent_out_of_range_is_flagged(lib):
    """An exponent beyond +-256 sets flags bit 3; the run goes on with it (here
    it scales one column by 2^-300, so the result is that of A without it)."""
    gen = W.rng(61)
    A = to_f16(gen.standard_normal((700, 300)))
    e = np.zeros(300, dtype=np.int32)
    e[17] = 300
    _, S, _, info = lib.sorsvd(dev_f16(A), 10, q=1, seed=2, refine=1,
                               col_exp=torch.as_tensor(e).cuda())
    assert info["flags"] & 8
    A0 = A.copy()
    A0[:, 17] = 0.0
    _, S0, _, info0 = lib.sorsvd(dev_f16(A0), 10, q=1, seed=2, refine=1)
    assert info0["flags"] & 8 == 0
    assert np.abs(host(S) - host(S0)).max() <= 1e-12 * host(S0)[0]
