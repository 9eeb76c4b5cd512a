"""Seeded synthetic inputs shaped like the paper's workloads.

This module only BUILDS INPUT MATRICES. It holds none of SOR-SVD's arithmetic
(no sketch, no orbit product, no projection, no core SVD) and imports neither
the oracle nor the product package; both sides receive the same arrays from it.
The Gaussian Omega that the method itself draws is not made here: each side
generates it from the Philox key (seed, 0).

Workloads (shapes and spectra as in the configurations the library is
measured on; the paper's own datasets are not used):
  c1  A = X Y^T + 1e-3 E, X 1000x20, Y 800x20, E 1000x800, N(0,1), seed 0;
      FP64, k = 20, q = 0, Omega seed 1.
  c2  A = U diag(j^-2) V^T, 20000 x 20000, U, V Haar (QR of Gaussian with the
      sign correction), seed 2; stored FP32, k = 100, q = 1.
  c3  A = U diag(0.9^j) V^T + noise (s.d. 1e-6), 200000 x 4000, stored BF16,
      k = 64, q = 1. 0.9^j < 1e-17 beyond j = 380, so U, V carry the first
      r = 400 Haar columns only; the first r columns of a Haar matrix are the
      Q factor of an r-column Gaussian, so this is exact in distribution.
  c4  512 problems, m ~ U[256, 4096], n ~ U[128, 2048], r ~ U[4, 64] (seed 3);
      L = X Y^T with N(0,1) factors plus Bernoulli(0.05) outliers U[-10, 10];
      FP32, k = r + 8, q = 1.
  c5  A = U diag(j^-1.5) V^T, 32768 x 32768, stored BF16 (the predictor's
      evaluation matrix).

The CPU tests use the numpy builders at reduced sizes. Large matrices are
built on the GPU with torch (plumbing, outside any timed region).
"""
import numpy as np


def rng(seed):
    return np.random.default_rng(seed)


# ----------------------------------------------------------------- numpy side

def haar_columns(rows, cols, gen):
    """First ``cols`` columns of a Haar-distributed orthogonal rows x rows matrix."""
    G = gen.standard_normal((rows, cols))
    Q, R = np.linalg.qr(G, mode="reduced")
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d[None, :]


def spectral(m, n, sigma, seed):
    """A = U diag(sigma) V^T with Haar U (m x r), V (n x r), r = len(sigma)."""
    gen = rng(seed)
    sigma = np.asarray(sigma, dtype=np.float64)
    r = sigma.size
    U = haar_columns(m, r, gen)
    V = haar_columns(n, r, gen)
    return (U * sigma[None, :]) @ V.T, U, V


def c1(seed=0):
    """X Y^T + 1e-3 E (1000 x 800, FP64)."""
    gen = rng(seed)
    X = gen.standard_normal((1000, 20))
    Y = gen.standard_normal((800, 20))
    E = gen.standard_normal((1000, 800))
    return X @ Y.T + 1e-3 * E


def low_rank_plus_noise(m, n, r, noise, seed):
    gen = rng(seed)
    X = gen.standard_normal((m, r))
    Y = gen.standard_normal((n, r))
    E = gen.standard_normal((m, n))
    return X @ Y.T + noise * E


def rpca_problem(m, n, r, seed, frac=0.05, amp=10.0):
    """L = X Y^T (N(0,1) factors, rank r) plus Bernoulli(frac) outliers U[-amp, amp]."""
    gen = rng(seed)
    X = gen.standard_normal((m, r))
    Y = gen.standard_normal((n, r))
    A = X @ Y.T
    mask = gen.random((m, n)) < frac
    A[mask] += gen.uniform(-amp, amp, size=int(mask.sum()))
    return A


def c4_sizes(count=512, seed=3, m_range=(256, 4096), n_range=(128, 2048), r_range=(4, 64)):
    """Per-problem (m, n, r) of the batched workload; k = r + 8."""
    gen = rng(seed)
    m = gen.integers(m_range[0], m_range[1] + 1, size=count)
    n = gen.integers(n_range[0], n_range[1] + 1, size=count)
    r = gen.integers(r_range[0], r_range[1] + 1, size=count)
    return [(int(a), int(b), int(c)) for a, b, c in zip(m, n, r)]


def sigma_power(n, alpha):
    return np.arange(1, n + 1, dtype=np.float64) ** (-alpha)


def sigma_geometric(n, beta):
    return beta ** np.arange(1, n + 1, dtype=np.float64)


# ----------------------------------------------------------------- torch side

def _torch():
    import torch
    return torch


def haar_columns_torch(rows, cols, gen, device):
    torch = _torch()
    G = torch.randn(rows, cols, generator=gen, device=device, dtype=torch.float64)
    Q, R = torch.linalg.qr(G, mode="reduced")
    d = torch.sign(torch.diagonal(R))
    d[d == 0] = 1.0
    return Q * d[None, :]


def spectral_torch(m, n, sigma, seed, device="cuda", out_dtype=None, noise_sd=0.0):
    """Large A = U diag(sigma) V^T (+ Gaussian noise) built on ``device`` in FP64.

    Returns the matrix cast to ``out_dtype`` (row-major, contiguous).
    """
    torch = _torch()
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    sig = torch.as_tensor(np.asarray(sigma, dtype=np.float64), device=device)
    r = sig.numel()
    U = haar_columns_torch(m, r, gen, device)
    V = haar_columns_torch(n, r, gen, device)
    U.mul_(sig[None, :])
    A = U @ V.T
    del U, V
    if noise_sd > 0:
        A.add_(torch.randn(m, n, generator=gen, device=device, dtype=torch.float64), alpha=noise_sd)
    if out_dtype is not None and out_dtype != torch.float64:
        A = A.to(out_dtype)
    return A.contiguous()


def c2_torch(device="cuda", n=20000, seed=2):
    torch = _torch()
    return spectral_torch(n, n, sigma_power(n, 2.0), seed, device, torch.float32)


def c3_torch(device="cuda", m=200000, n=4000, seed=4, r=400, out_dtype=None):
    torch = _torch()
    return spectral_torch(m, n, sigma_geometric(r, 0.9), seed, device, out_dtype or torch.bfloat16, noise_sd=1e-6)


def rpca_problem_torch(m, n, r, seed, device="cuda", frac=0.05, amp=10.0, dtype=None):
    torch = _torch()
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    X = torch.randn(m, r, generator=gen, device=device, dtype=torch.float64)
    Y = torch.randn(n, r, generator=gen, device=device, dtype=torch.float64)
    A = X @ Y.T
    mask = torch.rand(m, n, generator=gen, device=device, dtype=torch.float64) < frac
    vals = (torch.rand(m, n, generator=gen, device=device, dtype=torch.float64) * 2 - 1) * amp
    A = torch.where(mask, A + vals, A)
    return A.to(dtype or torch.float32).contiguous()


def c4_problem_seed(i, seed=3):
    """Generator seed of problem i of the batched workload."""
    return (seed << 20) + i


def c4_torch(device="cuda", count=512, seed=3):
    """The batched workload: FP32 RPCA-style matrices of uneven sizes.

    Returns (mats, ks, qs, omega_seeds, ranks): k = r + 8, q = 1, Omega seed
    of problem i is i + 1.
    """
    sizes = c4_sizes(count, seed)
    mats = [rpca_problem_torch(m, n, r, c4_problem_seed(i, seed), device) for i, (m, n, r) in enumerate(sizes)]
    ks = [r + 8 for (_, _, r) in sizes]
    return mats, ks, [1] * count, [i + 1 for i in range(count)], [r for (_, _, r) in sizes]


def c5_torch(device="cuda", n=32768, seed=5):
    torch = _torch()
    return spectral_torch(n, n, sigma_power(n, 1.5), seed, device, torch.bfloat16)



# ----------------------------------------------------------------- (k, q) predictor spectra

C5_SIZES = (4096, 8192, 16384, 32768)


def c5_training_spectra(count=10000, seed=55, sizes=C5_SIZES):
    """Training spectra of the (k, q) predictor: a third each of
      j^-alpha, alpha ~ U[0.5, 3];  beta^j, beta ~ U[0.8, 0.99];
      rank r ~ U[4, 256] signal (values U[0.2, 1], sorted) plus a noise floor of
      relative Frobenius size 10^U[-6, -2] (quarter-circle profile);
    size n drawn from `sizes`. Returns a list of (kind, n, sigma) with sigma
    descending, FP64."""
    gen = rng(seed)
    out = []
    for i in range(count):
        kind = i % 3
        n = int(gen.choice(sizes))
        j = np.arange(1, n + 1, dtype=np.float64)
        if kind == 0:
            s = j ** (-gen.uniform(0.5, 3.0))
        elif kind == 1:
            s = gen.uniform(0.8, 0.99) ** j
        else:
            r = int(gen.integers(4, 257))
            sig = np.sort(gen.uniform(0.2, 1.0, size=r))[::-1]
            nu = 10.0 ** gen.uniform(-6.0, -2.0)
            x = (np.arange(n - r, dtype=np.float64) + 0.5) / (n - r)
            floor = np.sqrt(np.maximum(1.0 - x * x, 0.0))           # quarter-circle quantile profile
            floor *= nu * np.linalg.norm(sig) / np.linalg.norm(floor)
            s = np.sort(np.concatenate([sig, floor]))[::-1]
        out.append((kind, n, s / s[0]))
    return out


def ey_relative(sigma, kmax):
    """Eckart-Young relative Frobenius floor e_k for k = 0..kmax (Th. 1)."""
    s2 = np.asarray(sigma, dtype=np.float64) ** 2
    tail = np.cumsum(s2[::-1])[::-1]                                # tail[k] = sum_{j >= k} s_j^2
    tot = tail[0]
    ks = np.arange(kmax + 1)
    return np.sqrt(np.where(ks < s2.size, tail[np.minimum(ks, s2.size - 1)], 0.0) / tot)
