"""Benchmark: CoR-UTV decompositions per second on one MI355X.

Workload (the paper's plain CoR-UTV, at the 20000 x 15000 size): A =
U0 diag(exp(-i/25)) V0^T + 1e-4 N with Haar U0 (20000 x 300), V0
(15000 x 300), float32; k = 100, p = 10 (l = 110), q = 1 power iteration.
One step = one whole decomposition (test matrix, 2q+3 passes over A, the
CholeskyQR2 bases, the core, its QRCP and the lifts), inputs resident in HBM.

Printed: one JSON line with the throughput, the dominant kernel's roofline
(sketch passes, timed with HIP events on the library's stream inside the
timed region), the float64 oracle timed on the host on a bounded sample, and
a serving leg: a Poisson stream of requests over a pool of device-resident
matrices (log-uniform m in [1000, 40000], n in [500, 20000], k in [5, 150],
sigma_i = exp(-i/k) + 1e-4 noise, p = 10, q in {1, 2}) served one at a time
in FP64 and with continuous batching in FP64, BF16 and split-BF16, with
p50/p99 latency (arrival to completion) and the reconstruction error of the
reduced-precision forms against FP64 on sampled requests.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

M, N, K_RANK, P_OVER = 20000, 15000, 100, 10
PEAK = {"f32": (157.3, "mfma"), "f64": (78.6, "mfma")}  # dense TFLOP/s, MI355X datasheet
HBM_PEAK_GBS = 8000.0
HOST_PANEL_ROWS = 2048  # storage rows per staged panel for the host-resident leg (123 MB)
METRIC = "CoR-UTV/sec + sketch TFLOP/s (20k×15k,k=100); serving p50/p99 at fixed err"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def cpu_threads():
    try:
        from threadpoolctl import threadpool_info

        return max(i.get("num_threads", 1) for i in threadpool_info()) or os.cpu_count()
    except Exception:
        return os.cpu_count()


def measured_traffic():
    """HBM bytes per sketch launch from the committed FETCH_SIZE/WRITE_SIZE
    counter summary, or None when the kernel source changed since then."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "traffic_sketch_f32_20000x15000_k100_q1.txt")
    src = os.path.join(ROOT, "paper_1906_04572_amd", "csrc", "sketch_gemm.hip")
    try:
        text = open(path).read()
        h = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    val, ok = None, False
    for line in text.splitlines():
        if line.startswith("traffic_bytes_per_launch ="):
            val = int(line.split("=")[1])
        if line.startswith("source_sha256(") and line.split("=")[1].strip() == h:
            ok = True
    return val if ok else None


def pct(xs, p):
    xs = sorted(xs)
    if not xs:
        return None
    i = min(len(xs) - 1, max(0, int(np.ceil(p / 100.0 * len(xs))) - 1))
    return xs[i]


def serving_leg(cu, torch, n_req, pool_size, seed=5, load=0.8, slots=3):
    """Serving measurement; returns a dict for the JSON line."""
    from workloads import serving_pool, serving_stream

    dev = torch.device("cuda", 0)
    shapes = serving_pool(pool_size, seed)
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    pool64, pool32 = [], []
    log("serving: generating %d pool matrices on the device" % pool_size)
    for sh in shapes:
        m, n, r, k = sh["m"], sh["n"], sh["r"], sh["k"]
        U0 = torch.linalg.qr(torch.randn(m, r, generator=g, device=dev, dtype=torch.float64)).Q
        V0 = torch.linalg.qr(torch.randn(n, r, generator=g, device=dev, dtype=torch.float64)).Q
        sig = torch.exp(-torch.arange(1, r + 1, device=dev, dtype=torch.float64) / k)
        A = (U0 * sig) @ V0.T.contiguous()
        A += 1e-4 * torch.randn(m, n, generator=g, device=dev, dtype=torch.float64)
        pool64.append(A)
        pool32.append(A.float())
        del U0, V0
    torch.cuda.synchronize()
    p_over = 10
    need = max(cu.workspace_bytes(sh["m"], sh["n"], sh["k"], p_over, 2, "f64") for sh in shapes)
    streams = [torch.cuda.current_stream()] + [torch.cuda.Stream() for _ in range(slots)]
    ctx = cu.Context(workspace_bytes=slots * need, streams=streams)

    def operand(e, prec):
        return pool64[e] if prec == "f64" else pool32[e]

    # saturation throughput of the one-at-a-time FP64 path on the stream's mix
    cal = serving_stream(min(48, n_req), pool_size, 1.0, seed + 1)
    for r in cal[:8]:  # warm the per-shape launch configurations
        sh = shapes[r["entry"]]
        for prec in ("f64", "bf16", "bf16x3"):
            ctx.decompose(operand(r["entry"], prec), sh["k"], p_over, r["q"], r["seed"], prec=prec)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in cal:
        sh = shapes[r["entry"]]
        ctx.decompose(pool64[r["entry"]], sh["k"], p_over, r["q"], r["seed"], prec="f64")
    sat = len(cal) / (time.perf_counter() - t0)
    qps = load * sat
    reqs = serving_stream(n_req, pool_size, qps, seed + 2, tags=("f64", "bf16x3"))

    def one_at_a_time(prec, reqs):
        lat = []
        t0 = time.perf_counter()
        for r in reqs:
            while time.perf_counter() - t0 < r["t"]:
                time.sleep(0.0001)
            sh = shapes[r["entry"]]
            ctx.decompose(operand(r["entry"], prec), sh["k"], p_over, r["q"], r["seed"], prec=prec)
            lat.append(time.perf_counter() - t0 - r["t"])
        return lat, time.perf_counter() - t0

    def batched(prec_of, reqs):
        lat = []
        pend = {}
        i = 0
        t0 = time.perf_counter()
        while i < len(reqs) or pend:
            now = time.perf_counter() - t0
            moved = False
            while i < len(reqs) and reqs[i]["t"] <= now:
                r = reqs[i]
                sh = shapes[r["entry"]]
                prec = prec_of(r)
                try:
                    tk = ctx.submit(operand(r["entry"], prec), sh["k"], p_over, r["q"], r["seed"], prec=prec)
                except cu.CorutvError as e:
                    if e.code == cu.E_BUSY:
                        break
                    raise
                pend[tk] = r["t"]
                i += 1
                moved = True
            for tk in list(pend):
                if ctx.poll(tk) is not None:
                    lat.append(time.perf_counter() - t0 - pend.pop(tk))
                    moved = True
            if not moved:
                if time.perf_counter() - t0 > 300.0:
                    raise RuntimeError("serving leg: %d requests still pending after 300 s" % len(pend))
                time.sleep(0.0001)
        return lat, time.perf_counter() - t0

    def summary(lat, span):
        return {"p50_ms": round(pct(lat, 50) * 1e3, 3), "p99_ms": round(pct(lat, 99) * 1e3, 3),
                "mean_ms": round(float(np.mean(lat)) * 1e3, 3), "decomp_per_s": round(len(lat) / span, 2)}

    modes = {}
    log("serving: %d requests at %.1f/s (%.0f%% of the one-at-a-time FP64 saturation %.1f/s)"
        % (n_req, qps, load * 100, sat))
    modes["f64_one_at_a_time"] = summary(*one_at_a_time("f64", reqs))
    modes["f64_batched"] = summary(*batched(lambda r: "f64", reqs))
    modes["bf16x3_batched"] = summary(*batched(lambda r: "bf16x3", reqs))
    modes["bf16_batched"] = summary(*batched(lambda r: "bf16", reqs))
    modes["mixed_f64_bf16x3_batched"] = summary(*batched(lambda r: r["tag"], reqs))
    # saturation: the same requests all arriving at once
    burst = [dict(r, t=0.0) for r in reqs]
    saturation = {"f64_one_at_a_time": summary(*one_at_a_time("f64", burst))["decomp_per_s"],
                  "f64_batched": summary(*batched(lambda r: "f64", burst))["decomp_per_s"],
                  "bf16x3_batched": summary(*batched(lambda r: "bf16x3", burst))["decomp_per_s"],
                  "bf16_batched": summary(*batched(lambda r: "bf16", burst))["decomp_per_s"]}
    # reconstruction error of the reduced-precision forms on sampled requests
    errs = {"bf16": [], "bf16x3": []}
    for r in reqs[:: max(1, len(reqs) // 12)][:12]:
        sh = shapes[r["entry"]]
        e64 = ctx.decompose(pool64[r["entry"]], sh["k"], p_over, r["q"], r["seed"], prec="f64",
                            want_err=True)[4]["rel_err"]
        for prec in errs:
            e = ctx.decompose(pool32[r["entry"]], sh["k"], p_over, r["q"], r["seed"], prec=prec,
                              want_err=True)[4]["rel_err"]
            errs[prec].append(abs(e - e64))
    ctx.close()
    eq = {prec: {"max_abs_diff_vs_f64": float(max(v)), "within_1e-5": int(sum(x <= 1e-5 for x in v)),
                 "sampled": len(v)} for prec, v in errs.items()}
    return {"requests": n_req, "pool": pool_size, "slots": slots, "qps": round(qps, 2),
            "f64_one_at_a_time_saturation_per_s": round(sat, 2), "load": load, "modes": modes,
            "saturation_decomp_per_s": saturation,
            "equal_error": eq,
            "workload": "Poisson stream; pool of %d device-resident matrices, m log-uniform [1000,40000], "
                        "n log-uniform [500,20000], k uniform [5,150], sigma_i=exp(-i/k)+1e-4 noise, "
                        "p=10, q in {1,2}" % pool_size}


def rpca_leg(cu, torch, runs=3):
    """ALM-CoRUTV robust PCA on the video-frames shape (76800 x 300, rank 5,
    5 % corruption), 50 iterations, k = 5, p = 5, q = 1, M resident in HBM."""
    from workloads import low_rank_plus_sparse

    m, n, k, p, q, iters = 76800, 300, 5, 5, 1, 50
    log("rpca: generating the %d x %d frames input" % (m, n))
    Mh, _, _ = low_rank_plus_sparse(m, n, k, 0.05, 50.0, seed=4, grid=2.0 ** -6)
    Md = torch.from_numpy(np.ascontiguousarray(Mh.T, dtype=np.float32)).cuda().t()
    ctx = cu.Context(workspace_bytes=cu.rpca_workspace_bytes(m, n, k, p, q))
    ctx.rpca(Md, k, p, q, seed=4, max_iter=iters)
    ctx.pass_timing(True, reset=True)
    wall, gpu, step = [], [], []
    for _ in range(runs):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L, S, info = ctx.rpca(Md, k, p, q, seed=4, max_iter=iters)
        torch.cuda.synchronize()
        wall.append((time.perf_counter() - t0) * 1e3)
        gpu.append(info["gpu_ms"])
        step.append(info["step_ms"])
    ctx.pass_timing(False, reset=True)
    ctx.close()
    # fused elementwise kernel, algorithmic bytes: M (4), Y (8 + 8), S (4) and
    # B (8) per entry on all but the last iteration; the last writes L (4) for B
    step_bytes = m * n * (32.0 * (iters - 1) + 28.0)
    step_ms = float(np.median(step))
    achieved = step_bytes / (step_ms * 1e-3) / 1e9
    out = {"workload": "ALM-CoRUTV robust PCA of 76800x300 frames (rank 5, 5% corruption), 50 iterations",
           "m": m, "n": n, "k": k, "p": p, "q": q, "iterations": info["iters"],
           "final_rank": info["final_rank"], "zeta": info["zeta"],
           "ms_per_run": round(float(np.median(wall)), 3), "gpu_ms_per_run": round(float(np.median(gpu)), 3),
           "ms_per_iteration": round(float(np.median(gpu)) / iters, 4),
           "step_kernel": {"kernel": "rpca_step_kernel", "bound": "hbm",
                           "avg_ms": round(step_ms / iters, 4), "achieved": round(achieved, 1),
                           "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                           "algorithmic_bytes_per_run": step_bytes}}
    del Md, L, S
    torch.cuda.empty_cache()
    return out


def achievable_peaks(torch):
    """Achievable rates on this device with vendor kernels (torch's reduction
    and hipBLASLt GEMMs), as context for the datasheet peaks."""
    dev = torch.device("cuda", 0)
    out = {}
    x = torch.ones(1 << 30, dtype=torch.float32, device=dev)  # 4 GiB
    for _ in range(2):
        x.sum()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        x.sum()
    torch.cuda.synchronize()
    out["hbm_read_GBps"] = round(5 * x.numel() * 4 / (time.perf_counter() - t0) / 1e9, 1)
    del x
    for name, dt, n in (("fp64", torch.float64, 8192), ("fp32", torch.float32, 8192),
                        ("bf16", torch.bfloat16, 8192)):
        a = torch.randn(n, n, device=dev).to(dt)
        b = torch.randn(n, n, device=dev).to(dt)
        for _ in range(2):
            a @ b
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = 10
        for _ in range(reps):
            a @ b
        torch.cuda.synchronize()
        out["gemm_%s_TFLOPs" % name] = round(reps * 2.0 * n ** 3 / (time.perf_counter() - t0) / 1e12, 1)
        del a, b
    # the pass shapes themselves: 20000 x 15000 A times a 112-column skinny
    # operand, both orientations (the library's FP32/FP64 passes do the same
    # flops; FP64 here is FP32 data widened, as the F64 form reads an F64 A)
    for name, dt in (("fp32", torch.float32), ("fp64", torch.float64)):
        A = torch.randn(M, N, device=dev).to(dt)
        X = torch.randn(N, 112, device=dev).to(dt)
        Y = torch.randn(M, 112, device=dev).to(dt)
        for lbl, f in (("AX", lambda: A @ X), ("AtY", lambda: A.t() @ Y)):
            for _ in range(2):
                f()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            reps = 10
            for _ in range(reps):
                f()
            torch.cuda.synchronize()
            out["pass_%s_%s_TFLOPs" % (lbl, name)] = round(reps * 2.0 * M * N * 112 / (time.perf_counter() - t0)
                                                          / 1e12, 1)
        del A, X, Y
    torch.cuda.empty_cache()
    out["note"] = ("torch.sum over 4 GiB float32; torch.matmul 8192^3 and the 20000x15000 by 112 pass "
                   "shapes (hipBLASLt)")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--prec", default="f32", choices=["f32", "f64", "bf16x3", "bf16"])
    ap.add_argument("--q", type=int, default=1)
    ap.add_argument("--cpu-sample", type=int, default=2, help="oracle decompositions timed on the host")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=160)
    ap.add_argument("--serving-pool", type=int, default=12)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-rpca", action="store_true")
    ap.add_argument("--rpca-only", action="store_true", help="only run the robust PCA leg")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run 4 plain 1 GiB device copies (calibrates the HBM byte counters)")
    ap.add_argument("--peaks", action="store_true",
                    help="only measure achievable peaks with library kernels (HBM read, GEMM rates)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(requested --gpus %d)" % args.gpus, flush=True)
        sys.exit(2)

    import torch

    if args.peaks:
        print(json.dumps(achievable_peaks(torch)), flush=True)
        return

    if args.copy_calibration:
        # 2^27 doubles = 1 GiB read and 1 GiB written per copy launch
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        print("copied 4 x 1 GiB", flush=True)
        return

    import paper_1906_04572_amd as cu
    from workloads import decaying

    if args.rpca_only:
        print(json.dumps(rpca_leg(cu, torch)), flush=True)
        return

    dev = torch.device("cuda", 0)
    log("generating the 20000 x 15000 float32 input on the host")
    A_h = decaying(M, N, 300, 1e-4, seed=2, kind="exp", tau=25.0, dtype=np.float32)
    A32 = torch.from_numpy(A_h).to(dev)
    ell = K_RANK + P_OVER
    ws = max([cu.workspace_bytes(M, N, K_RANK, P_OVER, 2, p) for p in ("f32", "f64")] +
             [cu.workspace_bytes_host(M, N, K_RANK, P_OVER, 1, "f32", "row", HOST_PANEL_ROWS)])
    ctx = cu.Context(workspace_bytes=ws)

    def timed(A, prec, q, steps, warmup, core="pass"):
        out = ctx.alloc_outputs(A, K_RANK, P_OVER)
        for i in range(warmup):
            ctx.decompose(A, K_RANK, P_OVER, q, seed=1000 + i, prec=prec, out=out, core=core)
        ctx.pass_timing(True, reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            ctx.decompose(A, K_RANK, P_OVER, q, seed=i + 1, prec=prec, out=out, core=core)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = ctx.pass_stats()
        ctx.pass_timing(False, reset=True)
        return dt, st

    log("timing %s q=%d: %d warmup + %d steps" % (args.prec, args.q, args.warmup, args.steps))
    A_main = A32.double() if args.prec == "f64" else A32
    dt, st = timed(A_main, args.prec, args.q, args.steps, args.warmup)
    value = args.steps / dt
    avg_pass_ms = st["total_ms"] / max(st["passes"], 1)
    flops_pass = 2.0 * M * N * ell
    bytes_pass = M * N * (8 if args.prec == "f64" else 4)
    if args.prec in PEAK:
        achieved = flops_pass / (avg_pass_ms * 1e-3) / 1e12
        peak, bound = PEAK[args.prec]
        unit = "TFLOP/s"
    else:
        # bf16 forms read the float32 A at HBM rate; the matrix cores are far from busy
        achieved = bytes_pass / (avg_pass_ms * 1e-3) / 1e9
        peak, bound, unit = HBM_PEAK_GBS, "hbm", "GB/s"
    roof = {"bound": bound, "achieved": round(achieved, 2), "peak": peak, "unit": unit,
            "frac": round(achieved / peak, 4),
            "traffic": measured_traffic() if args.prec == "f32" and args.q == 1 else None,
            "kernel": "sketch_kernel (one pass over A)", "avg_pass_ms": round(avg_pass_ms, 4),
            "min_pass_ms": round(st["min_ms"], 4), "max_pass_ms": round(st["max_ms"], 4),
            "passes_timed": st["passes"], "hbm_GBps": round(bytes_pass / (avg_pass_ms * 1e-3) / 1e9, 1),
            "algorithmic_flops_per_pass": flops_pass, "algorithmic_bytes_per_pass": bytes_pass}
    # accuracy of the timed configuration (untimed decomposition with the residual pass)
    U, T, V, piv, info = ctx.decompose(A_main, K_RANK, P_OVER, args.q, seed=1, prec=args.prec, want_err=True)
    rel_gpu = info["rel_err"]

    variants = {}
    if not args.no_variants:
        for prec, q, core in (("f32", 0, "pass"), ("f32", 2, "pass"), ("f64", 1, "pass"), ("f32", 1, "rz"),
                              ("bf16x3", 1, "pass"), ("bf16", 1, "pass")):
            if prec == args.prec and q == args.q and core == "pass":
                continue
            Av = A32 if prec != "f64" else A32.double()
            vdt, vst = timed(Av, prec, q, 5, 2, core=core)
            vpass = vst["total_ms"] / max(vst["passes"], 1)
            name = "%s_q%d" % (prec, q) + ("_core_rz" if core == "rz" else "")
            peak_v = PEAK.get(prec, PEAK["f32"])[0]
            variants[name] = {
                "corutv_per_s": round(5 / vdt, 2), "ms_per_step": round(vdt / 5 * 1e3, 3),
                "avg_pass_ms": round(vpass, 4),
                "sketch_tflops": round(flops_pass / (vpass * 1e-3) / 1e12, 2),
                "hbm_GBps": round(M * N * (8 if prec == "f64" else 4) / (vpass * 1e-3) / 1e9, 1),
                "passes_per_step": 2 * q + (2 if core == "rz" else 3)}
            if prec in PEAK:
                variants[name]["frac_of_peak"] = round(flops_pass / (vpass * 1e-3) / 1e12 / peak_v, 4)
            del Av
        # A in pinned host memory, streamed through the device in every pass
        # (PCIe-inclusive; not the headline, whose A is resident in HBM)
        A_host = torch.from_numpy(A_h).pin_memory()
        out = ctx.alloc_outputs(A_host, K_RANK, P_OVER)
        ctx.decompose(A_host, K_RANK, P_OVER, 1, seed=7, prec="f32", out=out, panel_rows=HOST_PANEL_ROWS)
        torch.cuda.synchronize()
        hs = 3
        t0 = time.perf_counter()
        for i in range(hs):
            ctx.decompose(A_host, K_RANK, P_OVER, 1, seed=i + 1, prec="f32", out=out, panel_rows=HOST_PANEL_ROWS)
        torch.cuda.synchronize()
        hdt = (time.perf_counter() - t0) / hs
        variants["f32_q1_host_streamed"] = {
            "corutv_per_s": round(1 / hdt, 2), "ms_per_step": round(hdt * 1e3, 2), "passes_per_step": 5,
            "host_to_device_GBps": round(5 * M * N * 4 / hdt / 1e9, 1), "panel_rows": HOST_PANEL_ROWS}
        del A_host, out
        # the same decompositions as a stream through the serving queue with
        # two slots: one request's small steps (thin QRs, QRCP: a few
        # workgroups) overlap the next one's passes
        slots = 2
        pstreams = [torch.cuda.current_stream()] + [torch.cuda.Stream() for _ in range(slots)]
        pctx = cu.Context(workspace_bytes=slots * cu.workspace_bytes(M, N, K_RANK, P_OVER, 1, "f32"),
                          streams=pstreams)
        nreq = 20
        outs = [pctx.alloc_outputs(A32, K_RANK, P_OVER) for _ in range(nreq)]
        for t in [pctx.submit(A32, K_RANK, P_OVER, 1, seed=900 + i, prec="f32", out=outs[i]) for i in range(2)]:
            pctx.wait(t)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tickets = [pctx.submit(A32, K_RANK, P_OVER, 1, seed=i + 1, prec="f32", out=outs[i]) for i in range(nreq)]
        for t in tickets:
            pctx.wait(t)
        torch.cuda.synchronize()
        pdt = (time.perf_counter() - t0) / nreq
        variants["f32_q1_queue_2slots"] = {
            "corutv_per_s": round(1 / pdt, 2), "ms_per_step": round(pdt * 1e3, 3), "passes_per_step": 5,
            "requests": nreq, "slots": slots}
        pctx.close()
        del outs
    ctx.close()
    del A_main, A32
    torch.cuda.empty_cache()

    serving = None
    if not args.no_serving:
        serving = serving_leg(cu, torch, args.serving_requests, args.serving_pool)
    rpca = None if args.no_rpca else rpca_leg(cu, torch)

    cpu = None
    parity = {"rel_err_gpu": rel_gpu}
    if not args.no_cpu_baseline:
        from oracle.corutv import corutv, rel_err

        A64 = A_h.astype(np.float64)
        log("oracle: %d float64 decompositions on the host" % args.cpu_sample)
        t0 = time.perf_counter()
        ref = None
        for i in range(args.cpu_sample):
            r = corutv(A64, K_RANK, P_OVER, args.q, seed=i + 1)
            if i == 0:
                ref = r
        cdt = time.perf_counter() - t0
        cpu = {"value": round(args.cpu_sample / cdt, 4), "unit": "CoR-UTV/s", "cores": cpu_threads(),
               "kind": "oracle",
               "sample": "%d whole float64 decompositions of the same 20000x15000 input (q=%d, l=%d), "
                         "numpy/OpenBLAS" % (args.cpu_sample, args.q, ell)}
        parity["rel_err_oracle"] = rel_err(A64, ref["U"], ref["T"], ref["V"])
        parity["abs_diff"] = abs(parity["rel_err_oracle"] - rel_gpu)

    line = {
        "metric": METRIC, "value": round(value, 3), "unit": "CoR-UTV/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.prec,
        "data": "synthetic",
        "config": {"workload": "CoR-UTV of a 20000x15000 exp-decay(tau=25)+1e-4 noise matrix",
                   "m": M, "n": N, "k": K_RANK, "p": P_OVER, "q": args.q, "prec": args.prec},
        "sketch_tflops": round(flops_pass / (avg_pass_ms * 1e-3) / 1e12, 2),
        "roofline": roof,
        "cpu_baseline": cpu,
        "parity": parity,
        "variants": variants,
        "serving": serving,
        "rpca": rpca,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
