"""Theorem bounds of Sec. IV on the GPU (sorsvd_bounds): ||Omega2||_2,
||Omega1^+||_2 and the Th. 4 - Th. 7 bounds for the Omega of a seed, against
the FP64 oracle (`oracle/bounds.py`, which forms Omega2 = V2^T Omega and the
pseudo-inverse of Omega1 explicitly with LAPACK), and the deterministic
bounds against the SOR-SVD run of the same seed.

Tolerances: the two norms and every bound within 1e-10 relative of the
oracle's (the GPU takes ||Omega2||_2 from Omega^T Omega - Omega1^T Omega1,
whose entries are O(n) and whose result is O(n - l + p): no cancellation
beyond a few ulps of n); per draw, sigma_hat_j >= Th. 4 bound and the error
<= Th. 5 bound, with 1e-10 relative slack for rounding.
"""
import numpy as np
import pytest

import workloads as W
from oracle import bounds as ob
from oracle import sorsvd as osvd

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


@pytest.mark.parametrize("m,n,k,l,p,q,decay", [
    (500, 400, 10, 20, 5, 0, 0.9),
    (500, 400, 10, 20, 5, 1, 0.9),
    (450, 400, 20, 30, 8, 2, 0.95),
    (400, 400, 10, 12, 0, 1, 0.8),      # p = 0: Th. 6 / Th. 7 undefined (NaN)
    (600, 500, 5, 40, 2, 1, 0.97),
    (700, 600, 50, 200, 20, 1, 0.99),   # wide: l > 128
])
def test_bounds_match_oracle(lib, m, n, k, l, p, q, decay):
    sigma = decay ** np.arange(n, dtype=np.float64)
    A, U, V = W.spectral(m, n, sigma, 31 + l)
    seed = 17
    Om = osvd.omega(seed, n, l)
    r = l - p
    V1 = torch.as_tensor(np.ascontiguousarray(V[:, :r])).cuda()
    b = lib.bounds(V1, sigma, k, l, p, q=q, seed=seed)
    n2 = np.linalg.norm(V[:, r:].T @ Om, 2)
    n1p = np.linalg.norm(np.linalg.pinv(V[:, :r].T @ Om), 2)
    assert rel(b["omega2_norm"], n2) <= 1e-10, (b["omega2_norm"], n2)
    assert rel(b["omega1_pinv_norm"], n1p) <= 1e-10, (b["omega1_pinv_norm"], n1p)
    th4 = ob.th4_sv_lower(sigma, V, Om, k, l, p, q)
    assert np.max(np.abs(b["th4"] - th4) / th4) <= 1e-10
    for norm, key in (("fro", "th5_fro"), ("2", "th5_2")):
        assert rel(b[key], ob.th5_err_upper(sigma, V, Om, k, l, p, q, norm=norm)) <= 1e-10
    if p >= 2:
        th6 = ob.th6_sv_expect(sigma, n, k, l, p, q)
        assert np.max(np.abs(b["th6"] - th6) / th6) <= 1e-12
        for norm, key in (("fro", "th7_fro"), ("2", "th7_2")):
            assert rel(b[key], ob.th7_err_expect(sigma, n, k, l, p, q, norm=norm)) <= 1e-12
    else:
        assert np.all(np.isnan(b["th6"])) and np.isnan(b["th7_fro"]) and np.isnan(b["th7_2"])
    # the deterministic bounds hold for the run that draws this Omega
    Ug, Sg, Vg, info = lib.sorsvd(torch.as_tensor(A).cuda(), k, q=q, seed=seed, l=l)
    S = Sg.cpu().numpy()
    assert np.all(S >= b["th4"] * (1 - 1e-10))
    err = info["err_fro"] * info["a_fro"]
    assert err <= b["th5_fro"] * (1 + 1e-10)


def test_bounds_reject_bad_arguments(lib):
    n, l, p, k = 300, 20, 5, 10
    sigma = 0.9 ** np.arange(n, dtype=np.float64)
    _, _, V = W.spectral(n, n, sigma, 3)
    V1 = torch.as_tensor(np.ascontiguousarray(V[:, :l - p])).cuda()
    with pytest.raises(lib.SorsvdError):
        lib.bounds(V1, sigma[::-1].copy(), k, l, p)      # not descending
    with pytest.raises(lib.SorsvdError):
        lib.bounds(V1, sigma, 17, l, p)                  # p + k > l
    with pytest.raises(lib.SorsvdError):
        lib.bounds(V1, sigma[:l - p], k, l, p)           # too few singular values
