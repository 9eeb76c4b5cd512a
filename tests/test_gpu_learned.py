"""The learned (k, q) part on the GPU: network kernels against the FP64 oracle
(forward <= 1e-5, gradients <= 1e-4 normwise per tensor, the loss over 10
Adam steps on one minibatch stream <= 1e-4 relative), probe features against
the oracle's definition, the diagonal form of the method against the oracle on
the dense diagonal matrix, and the judge / fallback logic of sorsvd_auto."""
import numpy as np
import pytest

import workloads as W
from oracle import mlp as omlp
from oracle import sorsvd as osvd

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev32(x):
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def host(t):
    return t.detach().double().cpu().numpy()


def _params(seed):
    return (omlp.init_params(seed) + 0.05 * np.random.default_rng(seed + 1).standard_normal(omlp.N_PARAMS)).astype(
        np.float32)


def _batch(seed, B):
    gen = np.random.default_rng(seed)
    return (gen.uniform(-1, 0, size=(B, 128)).astype(np.float32), gen.uniform(2, 8, size=(B, 4)).astype(np.float32))


@pytest.mark.parametrize("B", [1, 37, 256])
def test_mlp_forward_matches_oracle(lib, B):
    p = _params(3)
    X, _ = _batch(4, B)
    net = lib.MLP(dev32(p), max_batch=256)
    Y = host(net.forward(dev32(X)))
    Yo, _, _ = omlp.forward(p.astype(np.float64), X.astype(np.float64))
    assert np.abs(Y - Yo).max() <= 1e-5 * max(1.0, np.abs(Yo).max())


def test_mlp_gradient_matches_oracle(lib):
    p = _params(5)
    X, T = _batch(6, 200)
    net = lib.MLP(dev32(p), max_batch=256)
    g, loss = net.backward(dev32(X), dev32(T))
    g = host(g)
    Lo, go = omlp.backward(p.astype(np.float64), X.astype(np.float64), T.astype(np.float64))
    assert abs(float(loss) - Lo) <= 1e-5 * Lo
    off = 0
    for name, shape in omlp.SIZES:
        size = int(np.prod(shape))
        a, b = g[off:off + size], go[off:off + size]
        assert np.linalg.norm(a - b) <= 1e-4 * np.linalg.norm(b), name
        off += size


def test_training_curve_matches_oracle(lib):
    p = _params(7)
    net = lib.MLP(dev32(p), max_batch=256)
    th = p.astype(np.float64)
    m, v = np.zeros_like(th), np.zeros_like(th)
    for step in range(1, 11):
        X, T = _batch(100 + step, 128)
        loss = float(net.train_step(dev32(X), dev32(T), lr=1e-3))
        Lo, go = omlp.backward(th, X.astype(np.float64), T.astype(np.float64))
        th, m, v = omlp.adam_step(th, go, m, v, step, lr=1e-3)
        assert abs(loss - Lo) <= 1e-4 * Lo, (step, loss, Lo)
    assert np.abs(host(net.params) - th).max() <= 1e-5


@pytest.mark.parametrize("shape", [(600, 400), (300, 900), (2000, 128)])
def test_probe_features_match_oracle(lib, shape):
    m, n = shape
    A, _, _ = W.spectral(m, n, 0.9 ** np.arange(min(m, n)), 3 + m)
    f = host(lib.probe_features(torch.as_tensor(A).cuda(), seed=11))
    fo = omlp.probe_features(A, 11)
    assert np.abs(f - fo).max() <= 2e-6


def test_probe_features_of_diagonal(lib):
    sigma = np.arange(1, 1501, dtype=np.float64) ** -1.2
    f = host(lib.probe_features(torch.as_tensor(sigma).cuda(), seed=4))
    fo = omlp.probe_features(np.diag(sigma), 4)
    assert np.abs(f - fo).max() <= 2e-6


@pytest.mark.parametrize("k,q", [(10, 0), (24, 2), (64, 1)])
def test_diagonal_form_matches_oracle(lib, k, q):
    sigma = 0.95 ** np.arange(300)
    U, S, V, info = lib.sorsvd_diag(torch.as_tensor(sigma).cuda(), k, q=q, seed=8)
    Uo, So, Vo, io = osvd.sorsvd(np.diag(sigma), k, q=q, seed=8)
    assert np.max(np.abs(host(S) - So)) <= 1e-10 * So[0]
    assert abs(info["err_fro"] - io["err_fro_identity"]) <= 1e-9
    d = So >= 1e-4 * So[0]
    assert np.abs(host(U)[:, d] - Uo[:, d]).max() <= 1e-7


def test_batched_diagonal_equals_single(lib):
    sig = [torch.as_tensor(0.9 ** np.arange(n)).cuda() for n in (500, 777, 2048)]
    specs = [(8, 0), (40, 1), (128, 3)]
    b = lib.Batch(sig, [k for k, _ in specs], [q for _, q in specs], [5, 6, 7])
    b.run()
    infos = b.info()
    for i, (s, (k, q)) in enumerate(zip(sig, specs)):
        _, S, _, info = lib.sorsvd_diag(s, k, q=q, seed=5 + i)
        assert torch.allclose(b.S[i], S, rtol=0, atol=1e-12)
        # the Th. 2 identity e^2 = 1 - sum_j s_j^2 / ||A||_F^2 is a difference
        # of O(1) terms: two runs that round their s_j differently agree in
        # e^2 to a few k u, not in e (which divides that by 2 e)
        assert abs(infos[i]["err_fro"] ** 2 - info["err_fro"] ** 2) <= 4 * k * 2.0 ** -52


def test_auto_fallback_and_judge(lib):
    # fast decay: the first fixed rung (k = 256, q = 2) meets 1e-3; the identity is the FP32 judge
    n = 1500
    A, _, _ = W.spectral(n, n, np.arange(1, n + 1) ** -2.5, 9)
    U, S, V, info = lib.auto(torch.as_tensor(A, dtype=torch.float32).cuda(), 1e-3, None, seed=1)
    assert info["met"] and info["used_fallback"] == 1 and info["k_used"] == 256 and info["q_used"] == 2
    assert info["runs"] == 1 and info["err"] <= 1e-3
    # j^-1.5: the Eckart-Young floor at 256 is above 1e-3 (2.4e-3), so the
    # ladder doubles the width until the judge accepts (512: floor 1.2e-3; 1024)
    C, _, _ = W.spectral(n, n, np.arange(1, n + 1) ** -1.5, 11)
    _, _, _, info3 = lib.auto(torch.as_tensor(C, dtype=torch.float32).cuda(), 1e-3, None, seed=1)
    assert info3["met"] and info3["k_used"] == 1024 and info3["runs"] == 3 and info3["err"] <= 1e-3
    # slow decay: nothing of width <= 1024 meets 1e-3 -> ETOL with the last rung's result
    B, _, _ = W.spectral(n, n, np.arange(1, n + 1) ** -0.8, 10)
    _, _, _, info2 = lib.auto(torch.as_tensor(B, dtype=torch.float32).cuda(), 1e-3, None, seed=1)
    assert not info2["met"] and info2["err"] > 1e-3 and info2["k_used"] == 1024


def test_auto_run_from_probe_matches_oracle(lib):
    # with the network, the run starts from the probe's Q (its leading k
    # columns are Q1 of the run's first sketch): the result is the oracle's
    # SOR-SVD with the chosen (k, q) and the same seed
    from paper_1804_00462_amd import predictor as PR
    m, n = 1500, 1200
    A, _, _ = W.spectral(m, n, np.arange(1, n + 1) ** -2.5, 21)
    U, S, V, info = lib.auto(torch.as_tensor(A).cuda(), 1e-3, PR.load_params(), seed=3)
    assert info["met"] and info["used_fallback"] == 0 and info["runs"] == 1
    k, q = info["k_used"], info["q_used"]
    assert k < 128
    Uo, So, Vo, io = osvd.sorsvd(A, k, q=q, seed=3)
    S = host(S)
    assert np.linalg.norm(S - So) <= 1e-10 * np.linalg.norm(So)
    # identity e^2 = 1 - sum s^2 / ||A||^2: rounding of ~1e-14 in the two sums moves e by ~1e-14 / (2 e)
    assert abs(info["err"] - io["err_fro"]) <= 1e-10
    U, V = host(U), host(V)
    assert np.abs(U.T @ U - np.eye(k)).max() < 1e-11 and np.abs(V.T @ V - np.eye(k)).max() < 1e-11
    # error record against the explicit residual
    E = A - (U * S) @ V.T
    assert abs(np.linalg.norm(E) / np.linalg.norm(A) - info["err"]) <= 1e-6 * info["err"]


def test_bf16_judge_accepts_only_results_within_tolerance(lib):
    """The BF16 judge subtracts a modelled share of the storage rounding noise
    from the explicit error on the stored values; every result it accepts must
    still meet the tolerance against the FP64 matrix before rounding. At
    16384^2 the noise allowance leaves room to accept fast-decaying spectra;
    j^-1.5 needs k ~ 1000 there, where the allowance (2.5 x 0.25) rejects."""
    from paper_1804_00462_amd import predictor as PR
    n, tol = 16384, 1e-3
    j = np.arange(1, n + 1, dtype=np.float64)
    met = 0
    for i, sigma in enumerate((0.9 ** (j - 1), j ** -2.5, j ** -3.0, j ** -2.0, j ** -1.5)):
        A64 = PR.eval_matrix(n, sigma, 900 + i)
        Ab = A64.to(torch.bfloat16)
        for params in (PR.load_params("bf16"), None):
            U, S, V, info = lib.auto(Ab, tol, params, seed=4)
            e = PR.true_error(A64, U, S, V)
            print(f"spectrum {i} params {params is not None}: k {info['k_used']} q {info['q_used']} "
                  f"runs {info['runs']} judge {info['err']:.3e} stored {info['err_stored']:.3e} true {e:.3e} "
                  f"met {info['met']}", flush=True)
            if info["met"]:
                met += 1
                assert e <= tol, (i, e)
            del U, S, V
        del A64, Ab
        torch.cuda.empty_cache()
    assert met >= 4


@pytest.mark.slow
def test_bf16_learned_beats_fp32_plain_to_tolerance(lib):
    """The headline comparison on held-out 32768 x 32768 matrices (full
    spectra, Haar U, V, seeds unused in training): BF16 storage with the
    learned (k, q) against FP32 with the fixed ladder (256, 2), (512, 2),
    (1024, 2) and the judge. Both must meet 1e-3 against the FP64 matrix, and
    BF16 + learned must take less time to tolerance on each. (On j^-1.5 the
    BF16 storage noise, 1.66e-3, keeps the judge from certifying BF16 results;
    bench.py reports that case with FP32 + learned beside it.)"""
    from paper_1804_00462_amd import predictor as PR
    p16 = PR.load_params("bf16")
    n, tol = 32768, 1e-3
    j = np.arange(1, n + 1, dtype=np.float64)
    for name, sigma, seed in (("j^-2.0", j ** -2.0, 6), ("j^-2.5", j ** -2.5, 8), ("j^-1.8", j ** -1.8, 9)):
        A64 = PR.eval_matrix(n, sigma, seed)
        Ab = A64.to(torch.bfloat16)
        Ub, Sb, Vb, ib = PR.time_to_tolerance(Ab, tol, p16, seed=2, reps=3)
        eb = PR.true_error(A64, Ub, Sb, Vb)
        del Ab, Ub, Sb, Vb
        A = A64.float()
        Up, Sp, Vp, ip = PR.time_to_tolerance(A, tol, None, seed=2, reps=3)
        ep = PR.true_error(A64, Up, Sp, Vp)
        print(f"{name}: bf16+learned k {ib['k_used']} q {ib['q_used']} runs {ib['runs']} {ib['ms']:.2f} ms "
              f"true {eb:.3e} | fp32 plain k {ip['k_used']} runs {ip['runs']} {ip['ms']:.2f} ms true {ep:.3e}",
              flush=True)
        assert ib["met"] and ip["met"]
        assert eb <= tol and ep <= tol
        assert ib["ms"] < ip["ms"]
        del A64, A, Up, Sp, Vp
        torch.cuda.empty_cache()


def test_predict_kq_is_the_first_run_of_auto(lib):
    from paper_1804_00462_amd import predictor as PR
    params = PR.load_params()
    A, _, _ = W.spectral(1500, 1200, np.arange(1, 1201) ** -2.5, 21)
    Ad = torch.as_tensor(A).cuda()
    k, q, kp, predicted = lib.predict_kq(Ad, params, 1e-3, seed=3)
    U, S, V, info = lib.auto(Ad, 1e-3, params, seed=3)
    assert predicted and info["used_fallback"] == 0
    assert (info["k_used"], info["q_used"]) == (k, q)
    assert np.allclose(kp, info["k_pred"], rtol=0, atol=0)
