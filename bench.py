#!/usr/bin/env python3
"""Throughput of the SOR-SVD hot path on one MI355X.

One step = one complete rank-k SOR-SVD of a device-resident matrix (Philox
Omega, 2q+3 passes over A, the Cholesky QRs of the sketches, the core
projection, the core SVD, the lift with the sign convention and the error
record), enqueued through the C ABI.

Headline workload (the `value` of the JSON line): the plain FP32
configuration, A = U diag(j^-2) V^T with m = n = 20000, Haar U and V (seed 2),
k = l = 100, q = 1, Omega seed 1. The same run also measures, under "extra",
the BF16-stored configuration (200000 x 4000, sigma_j = 0.9^j plus noise of
s.d. 1e-6, k = 64, q = 1, refinement pass) and the small FP64 configuration
(1000 x 800, k = 20, q = 0).

The batched configuration (512 FP32 problems of uneven sizes, k = r + 8,
q = 1) runs as HIP graph replays, one batch per step (extra "c4").

Printed: ONE JSON line with throughput (SOR-SVDs/s), the algorithmic HBM rate
of the passes, the roofline of the dominant kernel (the pass kernel over A,
timed per launch with HIP events that the library records on the same stream
inside the timed region) and the CPU oracle timed on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

WORKLOADS = {
    # name: (m, n, k, q, dtype name, refine, description)
    "c2": (20000, 20000, 100, 1, "float32", 0,
           "plain SOR-SVD FP32: A = U diag(j^-2) V^T, 20000 x 20000, Haar U, V (seed 2), k = 100, q = 1"),
    "c3": (200000, 4000, 64, 1, "bfloat16", 1,
           "BF16-stored A = U diag(0.9^j) V^T + N(0, (1e-6)^2), 200000 x 4000, k = 64, q = 1, "
           "BF16 MFMA passes, hi+lo refinement projection, FP64 QR and core SVD"),
    "c3h": (200000, 4000, 64, 1, "float16", 1,
            "C3's matrix in FP16 with power-of-two column scaling (packed on the GPU from FP64: "
            "e_j = 14 - floor(log2 max_i |a_ij|)), FP16 MFMA passes, hi+lo refinement projection, "
            "FP64 QR and core SVD"),
    "c1": (1000, 800, 20, 0, "float64", 0,
           "plain SOR-SVD FP64: A = X Y^T + 1e-3 E (1000 x 800, seed 0), k = 20, q = 0, Omega seed 1"),
    "c2pe": (20000, 20000, 100, 1, "float32", 0,
             "C2 with the pass-efficient core matrix (eq. M_approx, formed as T2^T Q2 from the last orbit "
             "product: 2q + 2 = 4 passes over A)"),
    "c3pe": (200000, 4000, 64, 1, "bfloat16", 1,
             "C3 with the pass-efficient core matrix (eq. M_approx as T2^T Q2; the last orbit product "
             "takes Q1 split into BF16 hi + lo parts: 2q + 2 = 4 passes over A)"),
    # wide sketches on C5's matrix (32768 x 32768, sigma_j = j^-1.5, Haar U, V, seed 5); for
    # kernel profiles of the widths the C5 comparison runs, not in the default extras
    "c5b": (32768, 32768, 704, 1, "bfloat16", 1,
            "C5's matrix stored in BF16, k = l = 704, q = 1, refinement, pass-efficient core matrix"),
    "c5f": (32768, 32768, 1024, 2, "float32", 0,
            "C5's matrix stored in FP32, k = l = 1024, q = 2 (the top rung of the fixed ladder)"),
}
PASS_EFFICIENT = {"c2pe", "c3pe", "c5b"}

C4_DESC = ("batched SOR-SVD FP32: 512 RPCA-style problems L + S (L = X Y^T, N(0,1) factors of rank r, "
           "S = 5% outliers U[-10, 10]), m ~ U[256, 4096], n ~ U[128, 2048], r ~ U[4, 64] (seed 3), "
           "k = r + 8, q = 1; one launch per step kind, autotuned tiles, HIP graph replay")

# dominant-kernel roofline: (bound, peak, unit)
PEAK = {"float32": ("mfma", 157.3, "TFLOP/s"), "float64": ("mfma", 78.6, "TFLOP/s"),
        "bfloat16": ("hbm", 8000.0, "GB/s"), "float16": ("hbm", 8000.0, "GB/s")}
DTYPE_TAG = {"float32": "f32", "float64": "f64", "bfloat16": "bf16", "float16": "f16"}
MFMA_PEAK = {"float32": 157.3, "float64": 78.6, "bfloat16": 2500.0, "float16": 2500.0}  # dense, TFLOP/s
REDUCED = {"c3", "c3h", "c3pe"}  # 16-bit storage: also the error against the FP64 matrix


HERE = os.path.dirname(os.path.abspath(__file__))
# counter summaries of the pass kernels (FETCH_SIZE + WRITE_SIZE per launch)
# and the sources they were taken from
TRAFFIC = {
    "c2": ("k_skinny_f32_c2_traffic.md", ["common.hpp", "skinny_body.hpp", "gemm.hip"]),
    "c3": ("bf16_passes_c3_traffic.md", ["common.hpp", "half16.hpp", "h16_body.hpp", "gemm_bf16.hip"]),
}


def source_hash(sources):
    import hashlib
    h = hashlib.sha256()
    for f in sources:
        h.update(open(os.path.join(HERE, "paper_1804_00462_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(name):
    """HBM bytes per pass launch from the committed counter summary of this
    workload, or None if there is none or the pass kernel's sources changed
    since the counters were taken."""
    if name not in TRAFFIC:
        return None
    fname, sources = TRAFFIC[name]
    try:
        text = open(os.path.join(HERE, "profiles", fname)).read()
    except OSError:
        return None
    vals = dict(line.split(":", 1) for line in text.splitlines()
                if line.startswith(("traffic_bytes_per_launch:", "source_sha256_16:")))
    if vals.get("source_sha256_16", "").split()[0:1] != [source_hash(sources)]:
        return None
    return float(vals["traffic_bytes_per_launch"])


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_input(name, torch, P, quick=False):
    """(A as stored, plan options, FP64 matrix it stands for or None)."""
    import workloads as W
    m, n, _, _, dname, _, _ = WORKLOADS[name]
    if quick:  # same shape and dtype, N(0, 1) entries: for counter runs where the spectrum does not matter
        g = torch.Generator(device="cuda")
        g.manual_seed(7)
        A = torch.randn(m, n, generator=g, device="cuda", dtype=torch.float32)
        if dname == "float16":
            Ah, e = P.pack_f16(A)
            return Ah, {"col_exp": e}, None
        return A.to(getattr(torch, dname)), {}, None
    if name in ("c2", "c2pe"):
        return W.c2_torch("cuda"), {}, None
    if name in ("c3", "c3h", "c3pe"):
        A64 = W.c3_torch("cuda", out_dtype=torch.float64)
        if name in ("c3", "c3pe"):
            return A64.to(torch.bfloat16), {}, A64
        Ah, e = P.pack_f16(A64)
        return Ah, {"col_exp": e}, A64
    if name == "c1":
        return torch.as_tensor(W.c1()).cuda(), {}, None
    if name in ("c5b", "c5f"):
        import numpy as np
        from paper_1804_00462_amd import predictor as PR
        A64 = PR.eval_matrix(n, np.arange(1, n + 1, dtype=np.float64) ** -1.5, 5)
        return A64.to(getattr(torch, dname)), {}, A64
    raise ValueError(name)


def error_vs_fp64(A64, U, S, V, torch):
    """||A64 - U S V^T||_F / ||A64||_F in FP64 on the device (row blocks)."""
    num = 0.0
    W = (V * S[None, :]).T.contiguous()
    for r0 in range(0, A64.shape[0], 20000):
        R = A64[r0:r0 + 20000] - U[r0:r0 + 20000] @ W
        num += float((R * R).sum())
    return (num ** 0.5) / float(torch.linalg.norm(A64))


def cpu_baseline(A_host, k, q, seed, budget_s=20.0, max_reps=5):
    """The CPU FP64 oracle as it stands, on the same stored matrix."""
    import numpy as np
    from oracle import sorsvd as osvd
    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        cores = os.cpu_count() or 1
    A = np.asarray(A_host, dtype=np.float64)
    times = []
    t_start = time.perf_counter()
    while len(times) < max_reps:
        t0 = time.perf_counter()
        osvd.sorsvd(A, k, q=q, seed=seed, explicit=False)  # the error by the identity, as the GPU step
        times.append(time.perf_counter() - t0)
        if time.perf_counter() - t_start > budget_s:
            break
    med = sorted(times)[len(times) // 2]
    return {"value": 1.0 / med, "unit": "SOR-SVD/s", "cores": int(cores), "kind": "oracle",
            "sample": f"{len(times)} full SOR-SVD(s) of the same stored matrix in FP64 numpy/LAPACK "
                      f"(median {med:.3f} s; error by the identity, as the GPU step: no explicit residual)"}


def run_workload(name, steps, warmup, torch, P, quick=False):
    m, n, k, q, dname, refine, desc = WORKLOADS[name]
    seed = 1
    log(f"[bench] building input {name}: {desc}")
    t0 = time.perf_counter()
    A, extra_opts, A64 = make_input(name, torch, P, quick)
    torch.cuda.synchronize()
    log(f"[bench] input ready in {time.perf_counter() - t0:.1f} s; dtype {A.dtype}")
    pe = 1 if name in PASS_EFFICIENT else 0
    plan = P.Plan(m, n, k, q, A.dtype, refine=refine, pass_efficient=pe, **extra_opts)
    es = A.element_size()

    for _ in range(warmup):
        plan.run(A, seed)
    torch.cuda.synchronize()

    passes = 2 * q + 3 - pe
    P.pass_timing(True, capacity=steps * passes + 8)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(steps):
        plan.run(A, seed)
    ev1.record()
    torch.cuda.synchronize()
    gpu_ms = ev0.elapsed_time(ev1)
    kern_ms, launches, kbytes, kflops = P.pass_timing_read()
    P.pass_timing(False)
    info = plan.info()
    ms_per_step = gpu_ms / steps
    log(f"[bench] {name}: {steps} timed steps, {ms_per_step:.3f} ms/step; pass kernel "
        f"{kern_ms / launches * 1e3:.1f} us/launch")
    # the same step as HIP graph replays (one graph launch per SOR-SVD)
    graph_ms = None
    try:
        S_eager = plan.S.clone()
        g = plan.capture(A, seed)
        for _ in range(warmup):
            g.replay()
        torch.cuda.synchronize()
        g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        g0.record()
        for _ in range(steps):
            g.replay()
        g1.record()
        torch.cuda.synchronize()
        graph_ms = g0.elapsed_time(g1) / steps
        if not torch.equal(S_eager, plan.S):
            raise RuntimeError("graph replay differs from the eager run")
        log(f"[bench] {name}: graph replay {graph_ms:.3f} ms/step")
        del g
    except Exception as ex:  # reported, not fatal
        log(f"[bench] {name}: graph replay not measured ({ex})")

    # bound of the pass kernel by its intensity 2 l / b_A (flop per byte of A)
    # against the ridge of the MFMA peak of its type over 8 TB/s
    intensity = 2.0 * k / es
    if intensity >= MFMA_PEAK[dname] * 1e12 / 8e12:
        bound, peak, unit = "mfma", MFMA_PEAK[dname], "TFLOP/s"
    else:
        bound, peak, unit = "hbm", 8000.0, "GB/s"
    avg_launch_s = kern_ms / launches / 1e3
    per_launch_flops = kflops / launches
    per_launch_bytes = kbytes / launches
    if unit == "GB/s":
        achieved = per_launch_bytes / avg_launch_s / 1e9
    else:
        achieved = per_launch_flops / avg_launch_s / 1e12
    traffic = measured_traffic(name)
    roofline = {"bound": bound, "achieved": round(achieved, 2), "peak": peak, "unit": unit,
                "frac": round(achieved / peak, 4), "traffic": traffic,
                "kernel": "pass kernel over A (sketch, orbit, projection products)",
                "avg_launch_us": round(avg_launch_s * 1e6, 2),
                "per_launch": {"flops": per_launch_flops, "bytes": per_launch_bytes},
                "hbm_gbps_of_that_kernel": round(per_launch_bytes / avg_launch_s / 1e9, 1),
                "tflops_of_that_kernel": round(per_launch_flops / avg_launch_s / 1e12, 2)}
    res = {"workload": desc, "m": m, "n": n, "k": k, "l": k, "q": q, "dtype": DTYPE_TAG[dname],
           "passes_over_A": passes, "ms_per_step": round(ms_per_step, 4),
           "value": round(1000.0 / ms_per_step, 3), "unit": "SOR-SVD/s",
           "hbm_gbps_algorithmic": round(float(m) * n * es * passes / (ms_per_step / 1e3) / 1e9, 1),
           "roofline": roofline, "err_fro": info["err_fro"], "jacobi_sweeps": info["sweeps"],
           "flags": info["flags"],
           "ms_per_step_graph": round(graph_ms, 4) if graph_ms is not None else None}
    if A64 is not None:
        res["err_vs_fp64"] = error_vs_fp64(A64, plan.U, plan.S, plan.V, torch)
        log(f"[bench] {name}: relative error against the FP64 matrix {res['err_vs_fp64']:.4e}")
        del A64
    return res, A


def run_batched(steps, warmup, torch, P):
    """C4: the whole batch is one step; timed as HIP graph replays."""
    import workloads as W
    log(f"[bench] building input c4: {C4_DESC}")
    mats, ks, qs, seeds, _ = W.c4_torch("cuda")
    torch.cuda.synchronize()
    b = P.Batch(mats, ks, qs, seeds)
    cfg = b.autotune()
    log(f"[bench] c4 tuned (rt, grid) per pass kind: {cfg}")
    b.capture()
    for _ in range(warmup):
        b.replay()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(steps):
        b.replay()
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    # pass kernels, timed per launch group on one eager run (graph replays carry no timing events)
    passes = [2 * q + 3 for q in qs]
    P.pass_timing(True, capacity=64)
    b.run()
    torch.cuda.synchronize()
    kern_ms, launches, kbytes, kflops = P.pass_timing_read()
    P.pass_timing(False)
    infos = b.info()
    b.release_graph()
    shapes = [tuple(A.shape) for A in mats]
    bytes_a = sum(p * m * n * 4 for p, (m, n) in zip(passes, shapes))
    flops_a = sum(p * 2.0 * m * n * k for p, (m, n), k in zip(passes, shapes, ks))
    # per-problem roofline: each problem's passes at max(bytes / HBM, flops / FP32 peak)
    t_roof = sum(max(p * m * n * 4 / 8e12, p * 2.0 * m * n * k / 157.3e12)
                 for p, (m, n), k in zip(passes, shapes, ks))
    log(f"[bench] c4: {ms:.3f} ms per batch of {len(mats)}; passes {kern_ms:.3f} ms in {launches} launch groups")
    return {"workload": C4_DESC, "problems": len(mats), "dtype": "f32", "ms_per_step": round(ms, 4),
            "value": round(len(mats) * 1000.0 / ms, 1), "unit": "SOR-SVD/s",
            "tuned_config": cfg,
            "hbm_gbps_algorithmic": round(bytes_a / (ms / 1e3) / 1e9, 1),
            "roofline": {"bound": "mixed (per problem max of HBM and FP32 MFMA time)",
                         "roofline_ms": round(t_roof * 1e3, 4), "frac": round(t_roof * 1e3 / ms, 4),
                         "pass_kernels_ms": round(kern_ms, 4), "pass_launch_groups": launches,
                         "pass_kernels_gbps": round(kbytes / (kern_ms / 1e3) / 1e9, 1),
                         "pass_kernels_tflops": round(kflops / (kern_ms / 1e3) / 1e12, 2),
                         "pass_bytes": kbytes, "pass_flops": kflops, "total_flops_of_passes": flops_a},
            "max_jacobi_sweeps": max(i["sweeps"] for i in infos),
            "flags": sum(i["flags"] for i in infos),
            "err_fro_median": float(sorted(i["err_fro"] for i in infos)[len(infos) // 2])}


RPCA_DESC = ("robust PCA by the ALM-SOR-SVD iteration (Table III): X = L + S, n x n, rank(L) = 0.05 n "
             "(N(0,1) factors), 5% of entries +-50, l = 2 rank, q = 1, tol 1e-7 (the paper's Table IV setup)")


def run_rpca(torch, P, sizes=(1000, 2000, 3000), reps=3):
    """Time to solve one RPCA problem (all iterations, host loop included)."""
    import numpy as np
    out = {"workload": RPCA_DESC, "cases": {}}
    for n in sizes:
        r = int(0.05 * n)
        g = np.random.default_rng(n)
        L0 = g.standard_normal((n, r)) @ g.standard_normal((r, n))
        S0 = np.zeros((n, n))
        idx = g.choice(n * n, int(0.05 * n * n), replace=False)
        S0.flat[idx] = g.choice([-50.0, 50.0], size=idx.size)
        X = torch.as_tensor(L0 + S0).cuda()
        P.rpca(X, 2 * r, q=1, seed=3)
        times = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            L, S, info = P.rpca(X, 2 * r, q=1, seed=3)
            torch.cuda.synchronize()
            times.append((time.perf_counter() - t0) * 1e3)
        ms = sorted(times)[len(times) // 2]
        Lh, Sh = L.cpu().numpy(), S.cpu().numpy()
        case = {"n": n, "rank_true": r, "l": 2 * r, "ms": round(ms, 2), "ms_per_iter": round(ms / info["iters"], 3),
                "iters": info["iters"], "rank": info["rank"], "nnz_s": info["nnz_s"],
                "nnz_true": int(np.count_nonzero(S0)), "xi": info["xi"], "met": info["met"],
                "support_exact": bool(np.array_equal(Sh != 0, S0 != 0)),
                "l_rel_err": float(np.linalg.norm(Lh - L0) / np.linalg.norm(L0))}
        log(f"[rpca n={n}] {ms:.1f} ms, {info['iters']} iterations, rank {info['rank']}/{r}, "
            f"nnz {info['nnz_s']}/{case['nnz_true']}, xi {info['xi']:.2e}")
        out["cases"][str(n)] = case
        del X, L, S
        torch.cuda.empty_cache()
    return out


def run_c5(torch, P):
    """The metric's comparison on its configuration: time to tolerance 1e-3
    (relative Frobenius error against the FP64 matrix) on m = n = 32768,
    A = U diag(j^-1.5) V^T with Haar U, V over the whole spectrum (seed 5):
    BF16 storage + learned (k, q) + judge (sorsvd_auto with the network)
    against FP32 storage + the fixed ladder (256, 2), (512, 2), (1024, 2) +
    judge (sorsvd_auto without it); the other two combinations for context.
    The Eckart-Young floor needs k >= 645 here, so the fixed (256, 2) alone
    cannot meet the tolerance. BF16 storage alone perturbs this matrix by
    1.66e-3 (relative), so the judge, which sees only the stored values,
    cannot certify BF16 results at 1e-3 here; the same comparison on
    sigma_j = j^-2 (seed 6), where it can, follows. Also the success rate of
    the learned first run on 200 held-out spectra (diagonal stand-ins, FP64)."""
    import numpy as np
    from paper_1804_00462_amd import predictor as PR
    params = PR.load_params()
    n = 32768
    j = np.arange(1, n + 1, dtype=np.float64)
    out = {}
    for name, sigma, seed in (("j^-1.5", j ** -1.5, 5), ("j^-2", j ** -2.0, 6)):
        log(f"[bench] c5 {n} x {n}, sigma_j = {name}, full spectrum")
        t0 = time.perf_counter()
        A64 = PR.eval_matrix(n, sigma, seed)
        torch.cuda.synchronize()
        log(f"[bench] c5 input ready in {time.perf_counter() - t0:.1f} s")
        res = PR.compare(A64, 1e-3, params, log=log, label=f"c5 {name}")
        del A64
        torch.cuda.empty_cache()
        bl, fp = res["bf16_learned"], res["fp32_plain"]
        keys = ("k_used", "q_used", "used_fallback", "runs", "err", "true_err", "met", "met_true", "k_pred")
        out[name] = {"bf16_learned_ms": round(bl["ms"], 3), "fp32_plain_ms": round(fp["ms"], 3),
                     "speedup": round(fp["ms"] / bl["ms"], 3),
                     "bf16_learned": {k: bl[k] for k in keys}, "fp32_plain": {k: fp[k] for k in keys},
                     "fp32_learned": {k: res["fp32_learned"][k] for k in keys + ("ms",)},
                     "bf16_plain": {k: res["bf16_plain"][k] for k in keys + ("ms",)}}
    held = PR.heldout_eval(params, 200, log=log)
    return {"workload": "time to relative Frobenius error <= 1e-3 against the FP64 matrix on 32768 x 32768, "
                        "sigma_j = j^-1.5 (whole spectrum, Haar U, V, seed 5; and j^-2, seed 6): BF16 + learned "
                        "(k, q) vs FP32 + fixed ladder (256, 2) -> (512, 2) -> (1024, 2), both judged",
            "cases": out, "heldout": held}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS) + ["c4"])
    ap.add_argument("--extra", default="c3,c3h,c1,c4,c5,c2pe,c3pe,rpca",
                    help="comma-separated extra workloads ('' for none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quick-input", action="store_true",
                    help="N(0, 1) entries of the workload's shape instead of its spectrum (counter runs only)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run 3 plain device copies of 1 GiB (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (run with --gpus 1).",
              file=sys.stderr)
        return 2

    import torch
    import paper_1804_00462_amd as P

    if args.copy_calibration:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("[bench] copy calibration: 3 copies of 1 GiB done")
    if args.workload == "c4":
        head = run_batched(args.steps, args.warmup, torch, P)
        out = {"metric": "rank-k SOR-SVDs/sec + HBM GB/s; BF16+learned vs FP32 plain at ≤1e-3 rel err",
               "value": head["value"], "unit": "SOR-SVD/s", "n_gpus": 1, "steps": args.steps,
               "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True,
               "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
               "config": {"workload": head["workload"], "problems": head["problems"]},
               "roofline": head["roofline"], "cpu_baseline": None, "extra": {}}
        print(json.dumps(out), flush=True)
        return 0
    head, A = run_workload(args.workload, args.steps, args.warmup, torch, P, args.quick_input)
    m, n, k, q = head["m"], head["n"], head["k"], head["q"]
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample")
        A_host = A.double().cpu().numpy()
        del A
        cpu = cpu_baseline(A_host, k, q, 1)
        del A_host
    else:
        del A
    torch.cuda.empty_cache()

    extra = {}
    for name in [x for x in args.extra.split(",") if x and x != args.workload]:
        if name == "c4":
            extra[name] = run_batched(args.steps, args.warmup, torch, P)
        elif name == "c5":
            extra[name] = run_c5(torch, P)
        elif name == "rpca":
            extra[name] = run_rpca(torch, P)
        else:
            res, A = run_workload(name, args.steps, args.warmup, torch, P)
            del A
            extra[name] = res
        torch.cuda.empty_cache()

    out = {
        "metric": "rank-k SOR-SVDs/sec + HBM GB/s; BF16+learned vs FP32 plain at ≤1e-3 rel err",
        "value": head["value"],
        "unit": "SOR-SVD/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head["dtype"],
        "data": "synthetic",
        "config": {"workload": head["workload"], "m": m, "n": n, "k": k, "l": head["l"], "q": q,
                   "passes_over_A": head["passes_over_A"]},
        "hbm_gbps_algorithmic": head["hbm_gbps_algorithmic"],
        "roofline": head["roofline"],
        "cpu_baseline": cpu,
        "err_fro": head["err_fro"],
        "err_vs_fp64": head.get("err_vs_fp64"),
        "jacobi_sweeps": head["jacobi_sweeps"],
        "extra": extra,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
