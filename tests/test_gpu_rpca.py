"""Robust PCA by the ALM-SOR-SVD iteration on the GPU against the FP64
oracle (same seeds; the oracle takes the GPU's estimate of ||X||_2 so that
both start from the same mu_0 and Y_0): equal iteration counts, L and S to
1e-8 relative, and the paper's recovery criteria on its synthetic setup
(rank(L) = 0.05 n, ||S||_0 = 0.05 n^2 or 0.1 n^2 entries of +-50, l = 2 rank,
q = 1, tol 1e-7): recovered rank and support exact."""
import numpy as np
import pytest

from oracle import rpca as orpca

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def problem(n, r, frac, seed, amp=50.0):
    g = np.random.default_rng(seed)
    L = g.standard_normal((n, r)) @ g.standard_normal((r, n))
    S = np.zeros((n, n))
    idx = g.choice(n * n, int(frac * n * n), replace=False)
    S.flat[idx] = g.choice([-amp, amp], size=idx.size)
    return L, S


@pytest.mark.parametrize("n,frac", [(200, 0.05), (500, 0.05), (500, 0.1)])
def test_rpca_matches_oracle_and_recovers(lib, n, frac):
    r = int(0.05 * n)
    L0, S0 = problem(n, r, frac, 1)
    X = L0 + S0
    L, S, info = lib.rpca(torch.as_tensor(X).cuda(), 2 * r, q=1, seed=3)
    L, S = L.cpu().numpy(), S.cpu().numpy()
    assert info["met"] and info["xi"] < 1e-7
    assert info["rank"] == r
    assert info["nnz_s"] == np.count_nonzero(S0)
    assert np.array_equal(S != 0, S0 != 0)
    assert np.linalg.norm(L - L0) <= 1e-5 * np.linalg.norm(L0)
    # the oracle from the same start
    assert abs(info["norm2"] / np.linalg.norm(X, 2) - 1.0) < 1e-4
    Lo, So, io = orpca.alm_sorsvd(X, 2 * r, q=1, seed=3, norm2=info["norm2"])
    assert info["iters"] == io["iters"]
    assert np.linalg.norm(L - Lo) <= 1e-8 * np.linalg.norm(Lo)
    assert np.linalg.norm(S - So) <= 1e-8 * np.linalg.norm(So)
    assert abs(info["xi"] - io["xi"]) <= 1e-3 * io["xi"]


@pytest.mark.parametrize("n,frac", [(2000, 0.05), (3000, 0.05), (2000, 0.1)])
def test_rpca_paper_sizes_recover(lib, n, frac):
    """The sizes of the paper's Tables IV and V (l = 2 rank = 200, 300: the
    wide-sketch path): rank and support recovered exactly; n = 2000 also
    against the oracle from the same start."""
    r = int(0.05 * n)
    L0, S0 = problem(n, r, frac, 1)
    X = L0 + S0
    L, S, info = lib.rpca(torch.as_tensor(X).cuda(), 2 * r, q=1, seed=3)
    L, S = L.cpu().numpy(), S.cpu().numpy()
    assert info["met"] and info["xi"] < 1e-7
    assert info["rank"] == r
    assert np.array_equal(S != 0, S0 != 0)
    assert np.linalg.norm(L - L0) <= 1e-5 * np.linalg.norm(L0)
    if n == 2000 and frac == 0.05:
        Lo, So, io = orpca.alm_sorsvd(X, 2 * r, q=1, seed=3, norm2=info["norm2"])
        assert info["iters"] == io["iters"]
        assert np.linalg.norm(L - Lo) <= 1e-8 * np.linalg.norm(Lo)
        assert np.linalg.norm(S - So) <= 1e-8 * np.linalg.norm(So)


def test_rpca_stops_at_max_iter_with_the_last_iterate(lib):
    L0, S0 = problem(120, 6, 0.05, 2)
    X = torch.as_tensor(L0 + S0).cuda()
    L, S, info = lib.rpca(X, 12, q=1, seed=1, max_iter=3)
    assert not info["met"] and info["iters"] == 3 and info["xi"] > 1e-7
    assert torch.isfinite(L).all() and torch.isfinite(S).all()
