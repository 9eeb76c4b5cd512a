"""Learned choice of (k, q) for a target tolerance: training data, labels and
training (every step on the GPU through the library's entry points).

* Inputs: the probe features of a matrix (`probe_features`: singular values of
  the sketch A Omega[:, :128], log-scaled).
* Labels: for q = 0..3, log2 of the smallest sketch width k = l whose SOR-SVD
  with q power steps meets the tolerance (relative Frobenius error), found by
  running the method itself. Training spectra are diagonal stand-ins
  A = diag(sigma) (the Gaussian Omega is rotation-invariant, so this is exact in
  distribution for U diag(sigma) V^T with Haar U, V). Two reductions keep the
  labelling cheap:
    - Eckart-Young censoring: the method never beats the rank-k floor (Th. 1),
      so a spectrum whose floor at k = 1024 (the widest sketch) exceeds the
      tolerance is labelled "more than 1024" (log2 2048) without a run;
    - tail truncation: runs use the leading 2048 diagonal entries (widths up to
      128; the batched engine) or 4096 (wider; one run each) and add the
      energy of the rest back into the error identity (those directions are
      nearly outside the sketch subspaces of the truncated problem; this is
      an approximation of the labels, not of the method).
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
KCAP = 1024        # widest sketch
NARROW = 128       # widest problem of the batched engine
N_LAB = 2048       # diagonal entries kept for runs of width <= NARROW
N_LAB_WIDE = 4096  # ... and for wider runs
CENSORED = 11.0    # log2(2048): "needs more than 1024"
WIDTH_FACTORS = (1.0, 1.1, 1.25, 1.5, 2.0, 3.0)
WIDE_FACTORS = (1.0, 1.25, 1.6, 2.0)  # fewer candidates where every run is a single wide SOR-SVD
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
    """(k_EY, narrow candidates, wide candidates) or (None, [], []) if no width
    <= KCAP can meet tol. Narrow candidates (<= 128) are multiples of k_EY
    ending with 128; wide ones are taken in increasing order only where every
    narrow one failed: 256, 512, 1024 after a narrow k_EY, or multiples of a
    wide k_EY (rounded up to a multiple of 32) up to 1024."""
    e = ey_floor(sigma)
    ok = np.nonzero(e <= tol)[0]
    if ok.size == 0:
        return None, [], []
    k_ey = max(1, int(ok[0]))
    if k_ey <= NARROW:
        narrow = sorted({min(NARROW, max(k_ey, int(math.ceil(f * k_ey)))) for f in WIDTH_FACTORS} | {NARROW})
        return k_ey, narrow, [256, 512, KCAP]
    wide = sorted({min(KCAP, 32 * int(math.ceil(f * k_ey / 32))) for f in WIDE_FACTORS} | {KCAP})
    return k_ey, [], wide


def _nlab(n, w):
    return min(n, N_LAB if w <= NARROW else N_LAB_WIDE)


def label_spectra(spectra, tol=TOL, batch_bytes=24e9, log=print):
    """Labels (count x 4, log2 widths) from SOR-SVD runs of the diagonal stand-ins."""
    torch = _torch()
    count = len(spectra)
    labels = np.full((count, 4), CENSORED)
    probs = []          # (spectrum, width, q) of width <= NARROW: the batched engine
    dev = {}
    meta = {}
    for i, (_, n, s) in enumerate(spectra):
        k_ey, narrow, wide = candidate_widths(s, tol)
        if k_ey is None:
            continue
        meta[i] = (float(np.sum(s ** 2)), narrow, wide)
        for w in narrow:
            if w > _nlab(n, w):
                continue
            for q in range(4):
                probs.append((i, w, q))
    log(f"[labels] {len(meta)} of {count} spectra can meet {tol:g} with k <= {KCAP}; {len(probs)} batched runs")
    err = {}

    def record(i, w, q, e_run):
        _, n, s = spectra[i]
        nl = _nlab(n, w)
        trunc, tail = float(np.sum(s[:nl] ** 2)), float(np.sum(s[nl:] ** 2))
        err[(i, w, q)] = math.sqrt(max((e_run ** 2) * trunc + tail, 0.0) / meta[i][0])

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
                dev[i] = torch.as_tensor(spectra[i][2][:_nlab(spectra[i][1], w)]).cuda()
            mats.append(dev[i])
            ks.append(w)
            qs.append(q)
            seeds.append(1000 + i)
        b = api.Batch(mats, ks, qs, seeds)
        b.run()
        infos = b.info()
        for (i, w, q), inf in zip(chunk, infos):
            record(i, w, q, inf["err_fro"])
        b.close()
        del b
        start = end
        log(f"[labels] {end}/{len(probs)} batched runs, {time.perf_counter() - t0:.1f} s")
    dev.clear()
    # wide candidates, in increasing width, for the (spectrum, q) that no
    # narrow candidate resolved; one level at a time, grouped by shape so that
    # one plan (workspace) serves a group
    pending = {}
    for i, (_, narrow, wide) in meta.items():
        for q in range(4):
            if not any(err.get((i, w, q), 1.0) <= tol for w in narrow):
                cand = [w for w in wide if w <= _nlab(spectra[i][1], w)]
                if cand:
                    pending[(i, q)] = cand
    nwide = 0
    level = 0
    while pending:
        groups = {}
        for (i, q), cand in pending.items():
            w = cand[0]
            groups.setdefault((_nlab(spectra[i][1], w), w, q), []).append(i)
        t_log = time.perf_counter()
        for (nl, w, q), idx in sorted(groups.items()):
            plan = api.Plan(nl, nl, w, q, SORSVD_DIAG)
            for i in idx:
                plan.run(torch.as_tensor(spectra[i][2][:nl]).cuda(), seed=1000 + i)
                record(i, w, q, plan.info()["err_fro"])
                nwide += 1
                if time.perf_counter() - t_log > 15.0:
                    t_log = time.perf_counter()
                    log(f"[labels] wide level {level + 1}: {nwide} wide runs, {time.perf_counter() - t0:.1f} s")
            del plan
        nxt = {}
        for (i, q), cand in pending.items():
            if err[(i, cand[0], q)] > tol and len(cand) > 1:
                nxt[(i, q)] = cand[1:]
        pending = nxt
        level += 1
        log(f"[labels] wide level {level}: {nwide} wide runs so far, {len(pending)} pending, "
            f"{time.perf_counter() - t0:.1f} s")
    for i, (_, narrow, wide) in meta.items():
        ws = narrow + wide
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


def eval_matrix(n, sigma, seed, rank=None, device="cuda"):
    """FP64 device matrix U diag(sigma) V^T (n x n) with Haar U, V; with `rank`
    only the leading `rank` singular values are kept (the relative Frobenius
    size of what is dropped is sqrt(sum_{j > rank} sigma_j^2) / ||sigma||, which
    the caller must keep well below its tolerance)."""
    torch = _torch()
    r = n if rank is None else min(n, rank)
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


def heldout_eval(params, count=200, seed=77, tol=TOL, log=print):
    """The learned choice against the fixed ladder on held-out spectra (drawn
    like the training spectra, another seed), as diagonal stand-ins at their
    nominal size (exact in distribution for Haar U, V; FP64). Returns the share
    of spectra whose predicted run met the tolerance at once, the share met by
    either, and the mean number of SOR-SVD runs and summed widths (the work)
    of each."""
    import workloads as W
    torch = _torch()
    spectra = W.c5_training_spectra(count, seed)
    first = met_l = met_p = 0
    runs_l = runs_p = 0
    reachable = 0
    for i, (_, n, s) in enumerate(spectra):
        if ey_floor(s, min(KCAP, n))[-1] > tol:
            continue  # no width <= 1024 can meet tol: both end at ETOL
        reachable += 1
        sig = torch.as_tensor(s).cuda()
        _, _, _, il = api.auto(sig, tol, params, seed=1000 + i)
        _, _, _, ip = api.auto(sig, tol, None, seed=1000 + i)
        first += int(il["met"] and not il["used_fallback"])
        met_l += int(il["met"])
        met_p += int(ip["met"])
        runs_l += il["runs"]
        runs_p += ip["runs"]
    r = max(reachable, 1)
    out = {"spectra": count, "reachable": reachable, "first_run_success": first / r, "met_learned": met_l / r,
           "met_plain": met_p / r, "mean_runs_learned": runs_l / r, "mean_runs_plain": runs_p / r}
    log(f"[heldout] {out}")
    return out


def compare(A64, tol, params, seed=1, log=print, label=""):
    """BF16 + learned against FP32 plain (the fixed ladder (256, 2), (512, 2),
    (1024, 2) + judge), and the other two combinations, on one FP64 matrix:
    time-to-tolerance and true error."""
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
    ap.add_argument("--heldout", type=int, default=0, help="held-out spectra to evaluate the FP32 weights on")
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
    if args.heldout > 0:
        heldout_eval(load_params(args.out), count=args.heldout, log=log)


if __name__ == "__main__":
    main()
