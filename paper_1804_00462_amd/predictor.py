"""Learned choice of (k, q) for a target tolerance: training data, labels and
training (every step on the GPU through the library's entry points).

* Inputs: the probe features of a matrix (`probe_features`: singular values of
  the sketch A Omega[:, :128], log-scaled).
* Labels: for q = 0..3, log2 of the smallest sketch width k = l whose SOR-SVD
  with q power steps meets the tolerance (relative Frobenius error), found by
  running the method itself. Training spectra are diagonal stand-ins
  A = diag(sigma) (the Gaussian Omega is rotation-invariant, so this is exact in
  distribution for U diag(sigma) V^T with Haar U, V). Two reductions keep the
  labelling cheap without changing the answer:
    - Eckart-Young censoring: the method never beats the rank-k floor (Th. 1),
      so a spectrum whose floor at k = 128 exceeds the tolerance is labelled
      "more than 128" (log2 256) without a run;
    - tail truncation: runs use the leading 2048 diagonal entries and add the
      energy of the rest back into the error identity (those directions are
      outside every rank-128 sketch subspace of the truncated problem).
  Candidate widths are multiples of the Eckart-Young width k_EY; the label is
  the crossing of the tolerance, interpolated in log error between the widest
  failing and the narrowest passing candidate.
* Training: mean squared error on the 4 log2 widths, Adam, minibatches of 256,
  through sorsvd_mlp_train_step.
"""
import math
import os
import sys
import time

import numpy as np

from . import api
from ._lib import SORSVD_DIAG

TOL = 1e-3
KCAP = 128
N_LAB = 2048
CENSORED = 8.0  # log2(256): "needs more than 128"
WIDTH_FACTORS = (1.0, 1.1, 1.25, 1.5, 2.0, 3.0)
PARAMS_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "predictor_params.f32")
PARAMS_FILE_BF16 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "predictor_params_bf16.f32")
# relative Frobenius size of the rounding of a dense matrix with Gaussian-like
# entries to BF16 (as measured by the residual pass on the evaluation matrices)
BF16_NOISE = 1.66e-3


def _torch():
    import torch
    return torch


def ey_floor(sigma, kmax=KCAP):
    """Relative Eckart-Young floors e_0..e_kmax of a spectrum (Th. 1)."""
    s2 = np.asarray(sigma, dtype=np.float64) ** 2
    tail = np.concatenate([np.cumsum(s2[::-1])[::-1], [0.0]])
    return np.sqrt(tail[:kmax + 1] / tail[0])


def candidate_widths(sigma, tol=TOL):
    """(k_EY, candidate widths) or (None, []) if no width <= 128 can meet tol."""
    e = ey_floor(sigma)
    ok = np.nonzero(e <= tol)[0]
    if ok.size == 0:
        return None, []
    k_ey = max(1, int(ok[0]))
    ws = sorted({min(KCAP, max(k_ey, int(math.ceil(f * k_ey)))) for f in WIDTH_FACTORS} | {KCAP})
    return k_ey, ws


def label_spectra(spectra, tol=TOL, batch_bytes=24e9, log=print):
    """Labels (count x 4, log2 widths) from SOR-SVD runs of the diagonal stand-ins."""
    torch = _torch()
    count = len(spectra)
    labels = np.full((count, 4), CENSORED)
    probs = []          # (spectrum, width, q)
    dev = {}
    meta = {}
    for i, (_, n, s) in enumerate(spectra):
        k_ey, ws = candidate_widths(s, tol)
        if k_ey is None:
            continue
        nl = min(n, N_LAB)
        tail = float(np.sum(s[nl:] ** 2))
        meta[i] = (float(np.sum(s ** 2)), float(np.sum(s[:nl] ** 2)), tail, ws)
        for w in ws:
            if w > nl:
                continue
            for q in range(4):
                probs.append((i, w, q))
    log(f"[labels] {len(meta)} of {count} spectra can meet {tol:g} with k <= {KCAP}; {len(probs)} runs")
    err = {}
    t0 = time.perf_counter()
    start = 0
    while start < len(probs):
        # group runs so that the batch workspace stays near batch_bytes
        end, acc = start, 0.0
        while end < len(probs) and (acc == 0.0 or acc < batch_bytes):
            i, w, q = probs[end]
            acc += 8.0 * 8 * min(spectra[i][1], N_LAB) * (16 * ((w + 15) // 16))
            end += 1
        chunk = probs[start:end]
        mats, ks, qs, seeds = [], [], [], []
        for i, w, q in chunk:
            if i not in dev:
                dev[i] = torch.as_tensor(spectra[i][2][:min(spectra[i][1], N_LAB)]).cuda()
            mats.append(dev[i])
            ks.append(w)
            qs.append(q)
            seeds.append(1000 + i)
        b = api.Batch(mats, ks, qs, seeds)
        b.run()
        infos = b.info()
        for (i, w, q), inf in zip(chunk, infos):
            tot, trunc, tail, _ = meta[i]
            e2 = (inf["err_fro"] ** 2) * trunc + tail
            err[(i, w, q)] = math.sqrt(max(e2, 0.0) / tot)
        b.close()
        del b
        start = end
        log(f"[labels] {end}/{len(probs)} runs, {time.perf_counter() - t0:.1f} s")
    for i, (_, _, _, ws) in meta.items():
        for q in range(4):
            prev = None
            for w in ws:
                e = err.get((i, w, q))
                if e is None:
                    continue
                if e <= tol:
                    if prev is None or prev[1] <= tol:
                        labels[i, q] = math.log2(w)
                    else:  # interpolate log(error) between the failing and the passing width
                        w0, e0 = prev
                        t = (math.log(e0) - math.log(tol)) / max(math.log(e0) - math.log(e), 1e-12)
                        labels[i, q] = math.log2(w0 + t * (w - w0))
                    break
                prev = (w, e)
    return labels


def spectrum_features(spectra, seed0=1000, noise_rel=0.0, log=print):
    """Probe features of the diagonal stand-ins at their nominal size (device, count x 128).

    noise_rel > 0: features of the matrix as stored in a reduced precision
    whose rounding adds isotropic noise of that relative Frobenius size: the
    stand-in's spectrum becomes sqrt(sigma_j^2 + noise_rel^2 ||sigma||^2 / n)."""
    torch = _torch()
    feats = torch.empty(len(spectra), 128, dtype=torch.float32, device="cuda")
    t0 = time.perf_counter()
    for i, (_, n, s) in enumerate(spectra):
        if noise_rel > 0.0:
            s = np.sqrt(s * s + (noise_rel ** 2) * float(np.sum(s * s)) / n)
        feats[i] = api.probe_features(torch.as_tensor(s).cuda(), seed0 + i)
        if (i + 1) % 2000 == 0:
            log(f"[features] {i + 1}/{len(spectra)}, {time.perf_counter() - t0:.1f} s")
    return feats


def init_params(seed=0):
    """Glorot-uniform weights, zero biases, in the network's flat layout."""
    gen = np.random.default_rng(seed)
    parts = []
    for fan_out, fan_in in ((64, 128), (64, 64), (4, 64)):
        lim = math.sqrt(6.0 / (fan_in + fan_out))
        parts += [gen.uniform(-lim, lim, size=fan_out * fan_in), np.zeros(fan_out)]
    p = np.concatenate(parts).astype(np.float32)
    # start the output biases at the mean label so that early steps fit the shape
    p[-4:] = 5.0
    return p


def train(X, T, epochs=120, batch=256, lr=2e-3, seed=0, val_frac=0.1, log=print):
    """Train on device features X (N x 128) and labels T (N x 4); returns (params, history)."""
    torch = _torch()
    N = X.shape[0]
    gen = np.random.default_rng(seed)
    perm = gen.permutation(N)
    nval = int(round(val_frac * N))
    val, tr = perm[:nval], perm[nval:]
    params = torch.as_tensor(init_params(seed)).cuda()
    net = api.MLP(params, max_batch=batch)
    Td = T.float().cuda() if hasattr(T, "cuda") else torch.as_tensor(T, dtype=torch.float32).cuda()
    hist = []
    for ep in range(epochs):
        order = tr[gen.permutation(tr.size)]
        tot = 0.0
        for s in range(0, order.size - batch + 1, batch):
            idx = torch.as_tensor(order[s:s + batch]).cuda()
            loss = net.train_step(X.index_select(0, idx), Td.index_select(0, idx), lr=lr)
            tot += float(loss) if s == 0 else 0.0
        if ep % 10 == 9 or ep == epochs - 1:
            vl = _eval_loss(net, X, Td, val, batch)
            hist.append((ep + 1, vl))
            log(f"[train] epoch {ep + 1}: validation mse {vl:.4f} (log2 width units^2)")
    return params, hist


def _eval_loss(net, X, Td, idx, batch):
    torch = _torch()
    tot, cnt = 0.0, 0
    for s in range(0, idx.size, batch):
        ii = torch.as_tensor(idx[s:s + batch]).cuda()
        Y = net.forward(X.index_select(0, ii))
        tot += float(((Y - Td.index_select(0, ii)) ** 2).sum())
        cnt += Y.numel()
    return tot / max(cnt, 1)


def save_params(params, path=PARAMS_FILE):
    params.detach().float().cpu().numpy().astype("<f4").tofile(path)


def load_params(path=PARAMS_FILE, device="cuda"):
    """Network weights (device FP32); path "bf16" selects the weights trained on
    BF16-stored inputs."""
    torch = _torch()
    if path == "bf16":
        path = PARAMS_FILE_BF16
    p = np.fromfile(path, dtype="<f4")
    if p.size != api.mlp_param_count():
        raise ValueError(f"{path}: {p.size} values, expected {api.mlp_param_count()}")
    return torch.as_tensor(p).to(device)


def eval_matrix(n, sigma, seed, rank=2048, device="cuda"):
    """FP64 device matrix U diag(sigma) V^T (n x n) with Haar U, V restricted to the
    leading `rank` singular values (the rest is dropped; for spectra that a width
    <= 128 can resolve to 1e-3 their energy is below 1e-15 relative)."""
    torch = _torch()
    r = min(n, rank)
    g = torch.Generator(device=device)
    g.manual_seed(seed)

    def haar(rows):
        G = torch.randn(rows, r, generator=g, device=device, dtype=torch.float64)
        Q, R = torch.linalg.qr(G, mode="reduced")
        d = torch.sign(torch.diagonal(R))
        d[d == 0] = 1.0
        return Q * d[None, :]
    U, V = haar(n), haar(n)
    s = torch.as_tensor(np.asarray(sigma[:r], dtype=np.float64), device=device)
    return (U * s[None, :]) @ V.T


def time_to_tolerance(A, tol, params, seed=1, reps=3):
    """Median wall time (ms) of sorsvd_auto (probe, network, SOR-SVD, judge,
    fallback) on a device matrix, after one warm-up call, and the last call's
    result."""
    torch = _torch()
    api.auto(A, tol, params, seed)
    times = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        U, S, V, info = api.auto(A, tol, params, seed)
        times.append((time.perf_counter() - t0) * 1e3)
    info["ms"] = sorted(times)[len(times) // 2]
    return U, S, V, info


def true_error(A64, U, S, V):
    torch = _torch()
    return float(torch.linalg.norm(A64 - (U * S) @ V.T) / torch.linalg.norm(A64))


def compare(A64, tol, params, seed=1, log=print, label=""):
    """BF16 + learned against FP32 plain (fixed (128, 2) + judge), and the other
    two combinations, on one FP64 matrix: time-to-tolerance and true error."""
    torch = _torch()
    out = {}
    p16 = load_params("bf16") if os.path.exists(PARAMS_FILE_BF16) else params
    for name, dt, p in (("bf16_learned", torch.bfloat16, p16), ("fp32_plain", torch.float32, None),
                        ("fp32_learned", torch.float32, params), ("bf16_plain", torch.bfloat16, None)):
        A = A64.to(dt)
        U, S, V, info = time_to_tolerance(A, tol, p, seed)
        info["true_err"] = true_error(A64, U, S, V)
        info["met_true"] = info["true_err"] <= tol
        out[name] = info
        del A
        log(f"[{label}] {name}: {info['ms']:.2f} ms, k {info['k_used']} q {info['q_used']}, "
            f"fallback {info['used_fallback']}, judge {info['err']:.3e} ({'met' if info['met'] else 'not met'}), "
            f"true {info['true_err']:.3e}")
    return out


def main(argv=None):
    import argparse
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import workloads as W
    ap = argparse.ArgumentParser(description="train the (k, q) predictor on the GPU")
    ap.add_argument("--count", type=int, default=10000)
    ap.add_argument("--epochs", type=int, default=120)
    ap.add_argument("--seed", type=int, default=55)
    ap.add_argument("--out", default=PARAMS_FILE)
    ap.add_argument("--out-bf16", default=PARAMS_FILE_BF16)
    args = ap.parse_args(argv)
    log = lambda m: print(m, flush=True)
    spectra = W.c5_training_spectra(args.count, args.seed)
    t0 = time.perf_counter()
    T = label_spectra(spectra, log=log)
    log(f"[labels] done in {time.perf_counter() - t0:.1f} s; censored {np.mean(T[:, 0] >= CENSORED):.2%}")
    np.save(os.path.splitext(args.out)[0] + "_labels.npy", T)
    for out, noise in ((args.out, 0.0), (args.out_bf16, BF16_NOISE)):
        X = spectrum_features(spectra, noise_rel=noise, log=log)
        params, hist = train(X, T, epochs=args.epochs, log=log)
        save_params(params, out)
        log(f"[train] saved {out} (input noise {noise:g})")


if __name__ == "__main__":
    main()
