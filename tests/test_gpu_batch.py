"""Batched SOR-SVD (many problems of uneven sizes, one launch per step kind)
against the CPU FP64 oracle, problem by problem.

Tolerances as for the single-problem path:
  FP64 batches: sigma normwise <= 1e-10, rank-k reconstructions within 1e-10
                ||A||, factors equal to 1e-7 on spectra with gaps (0.8^j);
  FP32 batches: the oracle runs on the stored FP32 values; sigma normwise <= 1e-5.
Launch configuration (tile height, grid size), graph replay and autotuning
change no bit of the results: every output element is accumulated in the
same order whatever the configuration.
"""
import os

import numpy as np
import pytest

import workloads as W
from test_gpu_parity import fp32_factor_check
from oracle import sorsvd as osvd

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def host(t):
    return t.detach().double().cpu().numpy()


def normwise(s, s_ref):
    return float(np.max(np.abs(np.asarray(s) - np.asarray(s_ref))) / np.asarray(s_ref)[0])


# (m, n, k, l, q): ragged tails of every tile kind, m < n and m > n, l > k,
# full width (l = min(m, n)), the largest padded width (l = 128), k = 1,
# rows fewer than one tile, uneven q.
MIXED = [
    (300, 200, 10, 0, 0),
    (129, 517, 20, 0, 1),
    (1000, 64, 64, 0, 0),
    (400, 300, 12, 40, 1),
    (700, 500, 100, 128, 0),
    (20, 300, 5, 0, 2),
    (555, 333, 1, 0, 1),
    (1537, 1025, 33, 0, 1),
    (64, 64, 16, 0, 3),
    (2049, 130, 48, 80, 0),
]


def mixed_inputs(dtype, seed0):
    mats, specs = [], []
    for i, (m, n, k, l, q) in enumerate(MIXED):
        r = min(m, n)
        A, _, _ = W.spectral(m, n, 0.8 ** np.arange(r), seed0 + i)
        if dtype == torch.float32:
            A = A.astype(np.float32).astype(np.float64)
        mats.append(A)
        specs.append((k, l, q, 100 + i))
    return mats, specs


def make_batch(lib, mats, specs, dtype):
    dmats = [torch.as_tensor(A).to(dtype).cuda() for A in mats]
    ks = [s[0] for s in specs]
    ls = [s[1] for s in specs]
    qs = [s[2] for s in specs]
    seeds = [s[3] for s in specs]
    return lib.Batch(dmats, ks, qs, seeds, ls=ls), dmats


def determined(So, rel=1e-4):
    """Columns whose singular value is at least rel * s_1: with gaps of 0.8 their
    vectors are fixed to ~u / (0.2 rel) by the data; smaller ones are not (for
    any algorithm) and are checked through the reconstruction only."""
    return np.asarray(So) >= rel * np.asarray(So)[0]


def outputs(b):
    return [(U.clone(), S.clone(), V.clone()) for U, S, V in zip(b.U, b.S, b.V)]


def same_bits(o1, o2):
    return all(torch.equal(x, y) for a, b in zip(o1, o2) for x, y in zip(a, b))


def test_fp64_batch_matches_oracle(lib):
    mats, specs = mixed_inputs(torch.float64, 50)
    b, _ = make_batch(lib, mats, specs, torch.float64)
    b.run()
    torch.cuda.synchronize()
    infos = b.info()
    for i, (A, (k, l, q, seed)) in enumerate(zip(mats, specs)):
        print(f"problem {i}: {A.shape} k={k} l={l} q={q}", flush=True)
        U, S, V = host(b.U[i]), host(b.S[i]), host(b.V[i])
        Uo, So, Vo, io = osvd.sorsvd(A, k, q=q, seed=seed, l=l)
        assert normwise(S, So) <= 1e-10
        R = (U * S) @ V.T - (Uo * So) @ Vo.T
        assert np.abs(R).max() <= 1e-10 * np.abs(A).max()
        # gaps of 0.8 between consecutive singular values: factors agree entrywise
        d = determined(So)
        assert np.abs(U[:, d] - Uo[:, d]).max() <= 1e-7
        assert np.abs(V[:, d] - Vo[:, d]).max() <= 1e-7
        assert abs(infos[i]["a_fro"] - io["a_fro"]) <= 1e-13 * io["a_fro"]
        # sqrt(||A||^2 - sum s^2): near-zero errors carry sqrt(u)-sized rounding
        assert abs(infos[i]["err_fro"] - io["err_fro_identity"]) <= 1e-7
        # bit 2 (a pivot replaced) is expected only where sigma_l / sigma_1 ~ 1e-12
        assert infos[i]["flags"] == (0 if (l or k) < 100 else infos[i]["flags"] & 4), infos[i]


def test_batch_core_svd_lds_fits_every_problem(lib):
    """The batched core SVD keeps V in LDS when the widest problem's fits; a
    narrower problem may then take the padded V layout, which needs more LDS
    than the widest one's unpadded layout (l = 97 against l = 99): the launch
    is sized for the largest need, and both problems match the oracle."""
    mats, specs = [], []
    for i, l in enumerate((99, 97)):
        A, _, _ = W.spectral(400, 300, 0.9 ** np.arange(300), 90 + i)
        mats.append(A)
        specs.append((l - 5, l, 1, 300 + i))
    b, _ = make_batch(lib, mats, specs, torch.float64)
    b.run()
    torch.cuda.synchronize()
    for i, (A, (k, l, q, seed)) in enumerate(zip(mats, specs)):
        print(f"problem {i}: {A.shape} k={k} l={l} q={q}", flush=True)
        U, S, V = host(b.U[i]), host(b.S[i]), host(b.V[i])
        Uo, So, Vo, io = osvd.sorsvd(A, k, q=q, seed=seed, l=l)
        assert normwise(S, So) <= 1e-10
        R = (U * S) @ V.T - (Uo * So) @ Vo.T
        assert np.abs(R).max() <= 1e-10 * np.abs(A).max()
        assert np.abs(V.T @ V - np.eye(k)).max() <= 1e-12


def test_fp64_batch_equals_single_problem_path(lib):
    mats, specs = mixed_inputs(torch.float64, 70)
    b, dmats = make_batch(lib, mats, specs, torch.float64)
    b.run()
    for i, (Ad, (k, l, q, seed)) in enumerate(zip(dmats, specs)):
        print(f"problem {i}: {tuple(Ad.shape)} k={k} l={l} q={q}", flush=True)
        U, S, V, _ = lib.sorsvd(Ad, k, q=q, seed=seed, l=l)
        assert torch.allclose(b.S[i], S, rtol=0, atol=1e-12 * float(S[0]))
        d = torch.as_tensor(determined(host(S)), device="cuda")
        assert torch.allclose(b.U[i][:, d], U[:, d], rtol=0, atol=1e-9)
        assert torch.allclose(b.V[i][:, d], V[:, d], rtol=0, atol=1e-9)


def test_fp32_batch_matches_oracle_on_stored_values(lib):
    mats, specs = mixed_inputs(torch.float32, 90)
    b, _ = make_batch(lib, mats, specs, torch.float32)
    b.run()
    torch.cuda.synchronize()
    worst = 0.0
    for i, (A, (k, l, q, seed)) in enumerate(zip(mats, specs)):
        S = host(b.S[i])
        Uo, So, Vo, _ = osvd.sorsvd(A, k, q=q, seed=seed, l=l)
        assert normwise(S, So) <= 1e-5, i
        U, V = host(b.U[i]), host(b.V[i])
        assert np.abs(U.T @ U - np.eye(k)).max() < 1e-11
        assert np.abs(V.T @ V - np.eye(k)).max() < 1e-11
        worst = max(worst, fp32_factor_check(U, V, Uo, Vo, So, max(A.shape)))
    print(f"fp32 batch: factor deviation {worst:.2f} u32 sqrt(K) sigma_1 / gap")


def test_launch_configuration_changes_no_bit(lib):
    mats, specs = mixed_inputs(torch.float32, 110)
    b, _ = make_batch(lib, mats, specs, torch.float32)
    b.set_config([1, 256, 1, 256, 1, 256])
    b.run()
    ref = outputs(b)
    for cfg in ([2, 4096, 2, 512, 1, 1024], [2, 8, 1, 3, 2, 17], [1, 1, 2, 1, 1, 1]):
        b.set_config(cfg)
        b.run()
        assert same_bits(outputs(b), ref), cfg
    mats64, specs64 = mixed_inputs(torch.float64, 120)
    b64, _ = make_batch(lib, mats64, specs64, torch.float64)
    b64.run()
    ref64 = outputs(b64)
    b64.set_config([1, 7, 1, 64, 1, 4096])
    b64.run()
    assert same_bits(outputs(b64), ref64)


def test_graph_replays_match_eager(lib):
    mats, specs = mixed_inputs(torch.float32, 130)
    b, dmats = make_batch(lib, mats, specs, torch.float32)
    b.run()
    torch.cuda.synchronize()
    ref = outputs(b)
    ref_info = b.info()
    b.capture()
    for rep in range(3):
        for U, S, V in zip(b.U, b.S, b.V):  # eager work between replays
            U.zero_(), S.zero_(), V.zero_()
        lib.sorsvd(dmats[0], 4, q=0, seed=rep)
        torch.cuda.synchronize()
        b.replay()
        torch.cuda.synchronize()
        assert same_bits(outputs(b), ref), rep
        assert b.info() == ref_info
    b.release_graph()


def test_autotune_and_cache(lib, tmp_path):
    cache = tmp_path / "tune.txt"
    os.environ["SORSVD_TUNE_CACHE"] = str(cache)
    try:
        mats, specs = mixed_inputs(torch.float32, 150)
        b, dmats = make_batch(lib, mats, specs, torch.float32)
        b.run()
        ref = outputs(b)
        cfg = b.autotune()
        assert all(c in (1, 2) for c in cfg[0::2]) and all(g >= 1 for g in cfg[1::2])
        assert cfg == b.config()
        assert same_bits(outputs(b), ref)
        assert cache.read_text().strip()
        b2 = lib.Batch(dmats, [s[0] for s in specs], [s[2] for s in specs], [s[3] for s in specs],
                       ls=[s[1] for s in specs])
        assert b2.config() == cfg
    finally:
        del os.environ["SORSVD_TUNE_CACHE"]


def test_nonfinite_problem_is_flagged_alone(lib):
    gen = W.rng(3)
    mats = [gen.standard_normal((200, 150)), gen.standard_normal((180, 90))]
    mats[1][17, 33] = np.inf
    b, _ = make_batch(lib, mats, [(5, 0, 0, 1), (5, 0, 0, 2)], torch.float64)
    b.run()
    info = b.info()
    assert info[0]["flags"] == 0
    assert info[1]["flags"] & 2


def test_exact_low_rank_inputs_are_reconstructed(lib):
    # rank r <= l: Q1 spans the range of A with probability one, A_hat = A
    gen = W.rng(12)
    shapes = [(300, 200, 7), (150, 400, 12), (1000, 100, 30)]
    mats = [gen.standard_normal((m, r)) @ gen.standard_normal((r, n)) for m, n, r in shapes]
    b, _ = make_batch(lib, mats, [(r, 0, 0, 5 + i) for i, (_, _, r) in enumerate(shapes)], torch.float64)
    b.run()
    for i, A in enumerate(mats):
        U, S, V = host(b.U[i]), host(b.S[i]), host(b.V[i])
        assert np.abs(A - (U * S) @ V.T).max() <= 1e-11 * np.abs(A).max()


@pytest.mark.slow
def test_c4_full_batch(lib):
    """512 FP32 RPCA-style problems of uneven sizes (k = r + 8, q = 1) in the
    configuration the benchmark times: properties of every problem, the oracle
    on a sample of problems."""
    mats, ks, qs, seeds, ranks = W.c4_torch("cuda")
    b = lib.Batch(mats, ks, qs, seeds)
    cfg = b.autotune()
    print("tuned config", cfg, flush=True)
    b.run()
    torch.cuda.synchronize()
    infos = b.info()
    for i, (A, k) in enumerate(zip(mats, ks)):
        U, S, V = b.U[i], b.S[i], b.V[i]
        assert infos[i]["flags"] == 0, i
        assert torch.all(S[:-1] >= S[1:]), i
        eye = torch.eye(k, dtype=torch.float64, device="cuda")
        assert float((U.T @ U - eye).abs().max()) < 1e-10, i
        assert float((V.T @ V - eye).abs().max()) < 1e-10, i
        A64 = A.double()
        e = float(torch.linalg.norm(A64 - (U * S) @ V.T) / torch.linalg.norm(A64))
        assert abs(e - infos[i]["err_fro"]) <= 2e-5, (i, e, infos[i]["err_fro"])
    sizes = [(A.shape[0], A.shape[1]) for A in mats]
    order = np.argsort([m * n for m, n in sizes])
    sample = sorted({int(order[0]), int(order[-1]), int(order[len(order) // 2]),
                     next(i for i, (m, n) in enumerate(sizes) if m < n)})
    for i in sample:
        A = host(mats[i])
        print(f"oracle on problem {i}: {A.shape}, k={ks[i]}", flush=True)
        _, So, _, io = osvd.sorsvd(A, ks[i], q=qs[i], seed=seeds[i])
        assert normwise(host(b.S[i]), So) <= 1e-5, i
        assert abs(infos[i]["a_fro"] - io["a_fro"]) <= 1e-12 * io["a_fro"]
