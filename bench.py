"""Benchmark: CoR-UTV decompositions per second on one MI355X.

Headline workload (the paper's plain CoR-UTV at 20000 x 15000, in float64,
the paper's own arithmetic): A = U0 diag(exp(-i/25)) V0^T + 1e-4 N with Haar
U0 (20000 x 300), V0 (15000 x 300), drawn in float32 and widened; k = 100,
p = 10 (l = 110), q = 1 power iteration.  One step = one whole decomposition
(test matrix, 2q+3 passes over A, the CholeskyQR2 bases, the core, its QRCP
and the lifts), inputs resident in HBM.

Printed: one JSON line with the throughput, the dominant kernel's roofline
(the sketch passes, timed with HIP events on the library's stream inside the
timed region), the float64 oracle timed on the host on a bounded sample, and
further legs:
* variants of the headline (q = 0, 1, 2; F32, BF16, split-BF16; 2q+2 passes;
  A streamed from host memory; the serving queue), each with its roofline
  fraction (matrix cores for F32/F64, HBM for the BF16 forms);
* latency of the small plain configuration (2000 x 1500 float64, rank 20 +
  1e-6 noise, k = 20, p = 10, q = 1, lower T);
* the precision form at its real size (50000 x 30000 float32, sigma_i =
  i^-1.5 + 1e-5 noise, k = 200, p = 20, q = 2) in BF16, split-BF16, F32 and
  F64;
* serving: a Poisson stream of 2000 requests over a pool of device-resident
  matrices (log-uniform m in [1000, 40000], n in [500, 20000], k in [5, 150],
  sigma_i = exp(-i/k) + 1e-4 noise, p = 10, q in {1, 2}) at 0.5, 0.8, 1.0 and
  1.2 times the one-at-a-time FP64 saturation rate, served one at a time in
  FP64 and with continuous batching in split-BF16 (and FP64, and a mixed
  stream, at 0.8), with p50/p99 latency (arrival to completion), the
  reconstruction error of the reduced-precision forms against FP64, and
  sampled requests re-run alone and compared bit for bit;
* ALM-CoRUTV robust PCA on 76800 x 300 frames (50 iterations).
"""
import argparse
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

M, N, K_RANK, P_OVER = 20000, 15000, 100, 10
# dense peaks, MI355X datasheet: TFLOP/s of the matrix cores per dtype
PEAK = {"f32": (157.3, "mfma"), "f64": (78.6, "mfma")}
HBM_PEAK_GBS = 8000.0
HOST_PANEL_ROWS = 2048  # storage rows per staged panel for the host-resident leg (123 MB)
METRIC = "CoR-UTV/sec + sketch TFLOP/s (20k×15k,k=100); serving p50/p99 at fixed err"
SERVING_LOADS = (0.5, 0.8, 1.0, 1.2)


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def cpu_threads():
    try:
        from threadpoolctl import threadpool_info

        return max(i.get("num_threads", 1) for i in threadpool_info()) or os.cpu_count()
    except Exception:
        return os.cpu_count()


def host_cpu():
    """CPU model and physical core count of this host (lscpu)."""
    out = {"model": None, "physical_cores": None, "logical_cpus": os.cpu_count()}
    try:
        text = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        kv = {}
        for line in text.splitlines():
            if ":" in line:
                a, b = line.split(":", 1)
                kv[a.strip()] = b.strip()
        out["model"] = kv.get("Model name")
        cps, sk = kv.get("Core(s) per socket"), kv.get("Socket(s)")
        if cps and sk and cps.isdigit() and sk.isdigit():
            out["physical_cores"] = int(cps) * int(sk)
    except Exception:
        pass
    try:
        out["affinity_cpus"] = len(os.sched_getaffinity(0))
    except Exception:
        pass
    return out


def measured_traffic(prec):
    """HBM bytes per sketch launch from the committed FETCH_SIZE/WRITE_SIZE
    counter summary of this form, or None when the kernel source changed
    since the counters were taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "traffic_sketch_%s_20000x15000_k100_q1.txt" % prec)
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


def pass_roofline(prec, avg_pass_ms, m, n, ell):
    """Roofline of one pass over an m x n A with an l-column operand: matrix
    cores for F32/F64 (2 m n l flops), HBM for the BF16 forms (A read once:
    m n 4 bytes of float32)."""
    flops = 2.0 * m * n * ell
    nbytes = m * n * (8 if prec == "f64" else 4)
    if prec in PEAK:
        achieved = flops / (avg_pass_ms * 1e-3) / 1e12
        peak, bound = PEAK[prec]
        unit = "TFLOP/s"
    else:
        achieved = nbytes / (avg_pass_ms * 1e-3) / 1e9
        peak, bound, unit = HBM_PEAK_GBS, "hbm", "GB/s"
    return {"bound": bound, "achieved": round(achieved, 2), "peak": peak, "unit": unit,
            "frac": round(achieved / peak, 4), "avg_pass_ms": round(avg_pass_ms, 4),
            "hbm_GBps": round(nbytes / (avg_pass_ms * 1e-3) / 1e9, 1),
            "sketch_tflops": round(flops / (avg_pass_ms * 1e-3) / 1e12, 2),
            "algorithmic_flops_per_pass": flops, "algorithmic_bytes_per_pass": nbytes}


def device_decaying(torch, m, n, r, eps, seed, kind="exp", tau=25.0, alpha=1.5):
    """A = U0 diag(sigma) V0^T + eps N at sizes the host would take minutes to
    form: the Haar factors U0, V0 are drawn on the host (numpy, seeded, QR of
    Gaussians), the product and the noise (seeded torch generator) on the
    device in float64, the result rounded to float32."""
    from workloads import haar

    dev = torch.device("cuda", 0)
    rng = np.random.default_rng(seed)
    U0 = torch.from_numpy(haar(rng, m, r)).to(dev)
    V0 = torch.from_numpy(haar(rng, n, r)).to(dev)
    i = torch.arange(1, r + 1, device=dev, dtype=torch.float64)
    sig = torch.exp(-i / tau) if kind == "exp" else i ** -alpha
    A = (U0 * sig) @ V0.T.contiguous()
    del U0, V0
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    A += eps * torch.randn(m, n, generator=g, device=dev, dtype=torch.float64)
    A32 = A.float()
    del A
    return A32


def serving_leg(cu, torch, n_req, pool_size, seed=5, slots=3, loads=SERVING_LOADS):
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
        pool32.append(A.float())
        pool64.append(pool32[-1].double())  # both forms see the same data
        del U0, V0, A
    torch.cuda.synchronize()
    p_over = 10
    need = max(cu.workspace_bytes(sh["m"], sh["n"], sh["k"], p_over, 2, "f64") for sh in shapes)
    streams = [torch.cuda.current_stream()] + [torch.cuda.Stream() for _ in range(slots)]
    ctx = cu.Context(workspace_bytes=slots * need, streams=streams)

    def operand(e, prec):
        return pool64[e] if prec == "f64" else pool32[e]

    # saturation throughput of the one-at-a-time FP64 path on the stream's mix
    cal = serving_stream(min(64, n_req), pool_size, 1.0, seed + 1)
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

    def batched(prec_of, reqs, keep=None):
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
                pend[tk] = (r["t"], i)
                i += 1
                moved = True
            for tk in list(pend):
                res = ctx.poll(tk)
                if res is not None:
                    t_arr, idx = pend.pop(tk)
                    lat.append(time.perf_counter() - t0 - t_arr)
                    if keep is not None and idx in keep:
                        keep[idx] = [x.clone() for x in res[:4]]
                    moved = True
            if not moved:
                if time.perf_counter() - t0 > 300.0:
                    raise RuntimeError("serving leg: %d requests still pending after 300 s" % len(pend))
                time.sleep(0.0001)
        return lat, time.perf_counter() - t0

    def summary(lat, span):
        return {"p50_ms": round(pct(lat, 50) * 1e3, 3), "p99_ms": round(pct(lat, 99) * 1e3, 3),
                "mean_ms": round(float(np.mean(lat)) * 1e3, 3), "decomp_per_s": round(len(lat) / span, 2)}

    per_load = {}
    alone_vs_mix = None
    for li, load in enumerate(loads):
        qps = load * sat
        reqs = serving_stream(n_req, pool_size, qps, seed + 2 + li, tags=("f64", "bf16x3"))
        log("serving: %d requests at %.1f/s (%.0f%% of the one-at-a-time FP64 saturation %.1f/s)"
            % (n_req, qps, load * 100, sat))
        row = {"qps": round(qps, 2)}
        row["f64_one_at_a_time"] = summary(*one_at_a_time("f64", reqs))
        keep = None
        if load == 0.8:
            # 50 sampled requests of the mixed stream are kept and re-run alone
            keep = {i: None for i in range(0, n_req, max(1, n_req // 50))[:50]}
            row["mixed_f64_bf16x3_batched"] = summary(*batched(lambda r: r["tag"], reqs, keep))
            row["f64_batched"] = summary(*batched(lambda r: "f64", reqs))
            row["bf16_batched"] = summary(*batched(lambda r: "bf16", reqs))
        row["bf16x3_batched"] = summary(*batched(lambda r: "bf16x3", reqs))
        per_load["%.1fx" % load] = row
        if keep is not None:
            same = 0
            for idx, got in keep.items():
                r = reqs[idx]
                sh = shapes[r["entry"]]
                alone = ctx.decompose(operand(r["entry"], r["tag"]), sh["k"], p_over, r["q"], r["seed"],
                                      prec=r["tag"])
                same += int(got is not None and all(torch.equal(a, b) for a, b in zip(alone[:4], got)))
            alone_vs_mix = {"sampled": len(keep), "bit_identical": same}
    # saturation: requests all arriving at once
    burst = [dict(r, t=0.0) for r in serving_stream(min(n_req, 1000), pool_size, 1.0, seed + 9,
                                                    tags=("f64", "bf16x3"))]
    saturation = {"f64_one_at_a_time": summary(*one_at_a_time("f64", burst))["decomp_per_s"],
                  "f64_batched": summary(*batched(lambda r: "f64", burst))["decomp_per_s"],
                  "bf16x3_batched": summary(*batched(lambda r: "bf16x3", burst))["decomp_per_s"],
                  "bf16_batched": summary(*batched(lambda r: "bf16", burst))["decomp_per_s"]}
    # reconstruction error of the reduced-precision forms against FP64 on the same data
    errs = {"bf16": [], "bf16x3": []}
    for r in burst[:: max(1, len(burst) // 25)][:25]:
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
    return {"requests_per_load": n_req, "pool": pool_size, "slots": slots,
            "f64_one_at_a_time_saturation_per_s": round(sat, 2), "loads": per_load,
            "burst_saturation_decomp_per_s": saturation, "burst_requests": len(burst),
            "equal_error": eq, "alone_vs_mix": alone_vs_mix,
            "workload": "Poisson streams of %d requests at %s x the one-at-a-time FP64 saturation; pool of %d "
                        "device-resident matrices, m log-uniform [1000,40000], n log-uniform [500,20000], "
                        "k uniform [5,150], sigma_i=exp(-i/k) (to 1e-4) + 1e-4 noise, p=10, q in {1,2}"
                        % (n_req, "/".join(str(x) for x in loads), pool_size)}


def c1_leg(cu, torch, reps=30):
    """Latency of the small plain configuration: 2000 x 1500 float64, rank 20
    + 1e-6 noise, k = 20, p = 10, q = 1, lower-triangular T."""
    from workloads import noisy_low_rank

    m, n, k, p, q = 2000, 1500, 20, 10, 1
    A = torch.from_numpy(noisy_low_rank(m, n, k, 1e-6, seed=1)).cuda()
    ctx = cu.Context(workspace_bytes=cu.workspace_bytes(m, n, k, p, q, "f64"))
    out = ctx.alloc_outputs(A, k, p)
    for i in range(5):
        ctx.decompose(A, k, p, q, seed=500 + i, tri="lower", out=out)
    wall, gpu = [], []
    for i in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = ctx.decompose(A, k, p, q, seed=i + 1, tri="lower", out=out)[4]
        wall.append((time.perf_counter() - t0) * 1e3)
        gpu.append(info["gpu_ms"])
    e = ctx.decompose(A, k, p, q, seed=1, tri="lower", want_err=True)[4]["rel_err"]
    ctx.close()
    return {"workload": "CoR-UTV of a 2000x1500 rank-20 + 1e-6 noise float64 matrix, k=20, p=10, q=1, lower T",
            "reps": reps, "latency_ms_p50": round(float(np.median(wall)), 4),
            "latency_ms_p10": round(float(np.percentile(wall, 10)), 4),
            "latency_ms_p90": round(float(np.percentile(wall, 90)), 4),
            "gpu_ms_p50": round(float(np.median(gpu)), 4), "corutv_per_s": round(1e3 / float(np.median(wall)), 1),
            "rel_err": e, "passes": 5}


def c3_leg(cu, torch, reps=5):
    """The precision form at its real size: 50000 x 30000 float32, sigma_i =
    i^-1.5 (i <= 1000) + 1e-5 noise, k = 200, p = 20, q = 2 (7 passes)."""
    m, n, k, p, q = 50000, 30000, 200, 20, 2
    ell = k + p
    log("precision form: drawing the %d x %d input on the device" % (m, n))
    A32 = device_decaying(torch, m, n, 1000, 1e-5, seed=3, kind="poly", alpha=1.5)
    need = max(cu.workspace_bytes(m, n, k, p, q, pr) for pr in ("f64", "f32", "bf16", "bf16x3"))
    ctx = cu.Context(workspace_bytes=need)
    out = {"workload": "CoR-UTV of a 50000x30000 float32 matrix, sigma_i=i^-1.5 (i<=1000) + 1e-5 noise, "
                       "k=200, p=20, q=2", "m": m, "n": n, "k": k, "p": p, "q": q, "forms": {}}
    errs = {}
    for prec in ("bf16", "bf16x3", "f32", "f64"):
        A = A32.double() if prec == "f64" else A32
        o = ctx.alloc_outputs(A, k, p)
        ctx.decompose(A, k, p, q, seed=100, prec=prec, out=o)
        ctx.pass_timing(True, reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(reps):
            ctx.decompose(A, k, p, q, seed=i + 1, prec=prec, out=o)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        st = ctx.pass_stats()
        ctx.pass_timing(False, reset=True)
        errs[prec] = ctx.decompose(A, k, p, q, seed=11, prec=prec, out=o, want_err=True)[4]["rel_err"]
        roof = pass_roofline(prec, st["total_ms"] / max(st["passes"], 1), m, n, ell)
        out["forms"][prec] = {"ms_per_decomposition": round(dt * 1e3, 3), "corutv_per_s": round(1 / dt, 2),
                              "passes_per_step": 2 * q + 3, "pass_roofline": roof, "rel_err": errs[prec]}
        del A, o
    for prec in ("bf16", "bf16x3", "f32"):
        out["forms"][prec]["abs_diff_rel_err_vs_f64"] = abs(errs[prec] - errs["f64"])
    ctx.close()
    del A32
    torch.cuda.empty_cache()
    return out


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
    # the same recipe without rounding the factors and values to the 2^-6
    # grid: M is then L + S only up to FP32 rounding of L
    Mg, Lg, Sg = low_rank_plus_sparse(m, n, k, 0.05, 50.0, seed=4)
    Mgd = torch.from_numpy(np.ascontiguousarray(Mg.T, dtype=np.float32)).cuda().t()
    Lr, Sr, ginfo = ctx.rpca(Mgd, k, p, q, seed=4, max_iter=iters)
    Lh, Sh = Lr.double().cpu().numpy(), Sr.double().cpu().numpy()
    true_s = Sg != 0
    generic = {"l_rel_err": float(np.linalg.norm(Lh - Lg) / np.linalg.norm(Lg)),
               "support_exact_match": bool(np.array_equal(Sh != 0, true_s)),
               "support_true": int(true_s.sum()), "support_found": int((Sh != 0).sum()),
               "found_above_1e-3": int((np.abs(Sh) > 1e-3).sum()),
               "true_found_above_1e-3": int(((np.abs(Sh) > 1e-3) & true_s).sum()),
               "zeta": ginfo["zeta"], "final_rank": ginfo["final_rank"]}
    del Mgd, Lr, Sr, Mg, Lg, Sg, Lh, Sh
    ctx.close()
    # fused elementwise kernel, bytes it moves: M (4), Y (8 + 8), S (4) and B
    # (8) per entry on all but the last iteration; the last writes L (4) for B
    step_bytes = m * n * (32.0 * (iters - 1) + 28.0)
    # the step's minimum at float32 state: read M and Y, write S, Y and B
    step_bytes_f32 = m * n * 20.0 * iters
    step_ms = float(np.median(step))
    achieved = step_bytes / (step_ms * 1e-3) / 1e9
    achieved_f32 = step_bytes_f32 / (step_ms * 1e-3) / 1e9
    out = {"workload": "ALM-CoRUTV robust PCA of 76800x300 frames (rank 5, 5% corruption), 50 iterations",
           "m": m, "n": n, "k": k, "p": p, "q": q, "iterations": info["iters"],
           "final_rank": info["final_rank"], "zeta": info["zeta"],
           "ms_per_run": round(float(np.median(wall)), 3), "gpu_ms_per_run": round(float(np.median(gpu)), 3),
           "ms_per_iteration": round(float(np.median(gpu)) / iters, 4),
           "step_kernel": {"kernel": "rpca_step2_kernel", "bound": "hbm",
                           "avg_ms": round(step_ms / iters, 4), "achieved": round(achieved, 1),
                           "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                           "algorithmic_bytes_per_run": step_bytes,
                           "frac_at_float32_state_bytes": round(achieved_f32 / HBM_PEAK_GBS, 4),
                           "float32_state_bytes_per_run": step_bytes_f32},
           "unrounded_data": generic}
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
    ap.add_argument("--prec", default="f64", choices=["f64", "f32", "bf16x3", "bf16"])
    ap.add_argument("--q", type=int, default=1)
    ap.add_argument("--cpu-sample", type=int, default=2, help="oracle decompositions timed on the host")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=2000)
    ap.add_argument("--serving-pool", type=int, default=64)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-rpca", action="store_true")
    ap.add_argument("--no-small", action="store_true", help="skip the 2000 x 1500 latency leg")
    ap.add_argument("--no-precision-form", action="store_true", help="skip the 50000 x 30000 leg")
    ap.add_argument("--rpca-only", action="store_true", help="only run the robust PCA leg")
    ap.add_argument("--precision-form-only", action="store_true", help="only run the 50000 x 30000 leg")
    ap.add_argument("--small-only", action="store_true", help="only run the 2000 x 1500 latency leg")
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
    if args.precision_form_only:
        print(json.dumps(c3_leg(cu, torch)), flush=True)
        return
    if args.small_only:
        print(json.dumps(c1_leg(cu, torch)), flush=True)
        return

    dev = torch.device("cuda", 0)
    log("generating the 20000 x 15000 float32 input on the host")
    A_h = decaying(M, N, 300, 1e-4, seed=2, kind="exp", tau=25.0, dtype=np.float32)
    A32 = torch.from_numpy(A_h).to(dev)
    A64 = A32.double()  # the same data in float64
    ell = K_RANK + P_OVER
    ws = max([cu.workspace_bytes(M, N, K_RANK, P_OVER, 2, p) for p in ("f32", "f64", "bf16", "bf16x3")] +
             [cu.workspace_bytes_host(M, N, K_RANK, P_OVER, 1, "f32", "row", HOST_PANEL_ROWS)])
    ctx = cu.Context(workspace_bytes=ws)

    def operand(prec):
        return A64 if prec == "f64" else A32

    def timed(prec, q, steps, warmup, core="pass"):
        A = operand(prec)
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
    dt, st = timed(args.prec, args.q, args.steps, args.warmup)
    value = args.steps / dt
    avg_pass_ms = st["total_ms"] / max(st["passes"], 1)
    pr = pass_roofline(args.prec, avg_pass_ms, M, N, ell)
    roof = {k: pr[k] for k in ("bound", "achieved", "peak", "unit", "frac")}
    roof.update({"traffic": measured_traffic(args.prec) if args.q == 1 else None,
                 "kernel": "sketch_kernel (one pass over A)", "avg_pass_ms": pr["avg_pass_ms"],
                 "min_pass_ms": round(st["min_ms"], 4), "max_pass_ms": round(st["max_ms"], 4),
                 "passes_timed": st["passes"], "hbm_GBps": pr["hbm_GBps"],
                 "algorithmic_flops_per_pass": pr["algorithmic_flops_per_pass"],
                 "algorithmic_bytes_per_pass": pr["algorithmic_bytes_per_pass"]})
    # whole decomposition against its roofline: 2q+3 passes at the pass roofline
    npass = 2 * args.q + 3
    pass_roof_ms = max(pr["algorithmic_flops_per_pass"] / (PEAK[args.prec][0] * 1e12) if args.prec in PEAK else 0,
                       pr["algorithmic_bytes_per_pass"] / (HBM_PEAK_GBS * 1e9)) * 1e3
    roof["decomposition_roofline_ms"] = round(npass * pass_roof_ms, 4)
    roof["decomposition_frac"] = round(npass * pass_roof_ms / (dt / args.steps * 1e3), 4)
    # accuracy of the timed configuration (untimed decomposition with the residual pass)
    U, T, V, piv, info = ctx.decompose(operand(args.prec), K_RANK, P_OVER, args.q, seed=1, prec=args.prec,
                                       want_err=True)
    rel_gpu = info["rel_err"]
    del U, T, V, piv

    variants = {}
    if not args.no_variants:
        for prec, q, core in (("f64", 0, "pass"), ("f64", 2, "pass"), ("f64", 1, "rz"),
                              ("f32", 0, "pass"), ("f32", 1, "pass"), ("f32", 2, "pass"), ("f32", 1, "rz"),
                              ("bf16x3", 1, "pass"), ("bf16", 1, "pass")):
            if prec == args.prec and q == args.q and core == "pass":
                continue
            vdt, vst = timed(prec, q, 5, 2, core=core)
            vpass = vst["total_ms"] / max(vst["passes"], 1)
            name = "%s_q%d" % (prec, q) + ("_core_rz" if core == "rz" else "")
            vr = pass_roofline(prec, vpass, M, N, ell)
            variants[name] = {
                "corutv_per_s": round(5 / vdt, 2), "ms_per_step": round(vdt / 5 * 1e3, 3),
                "avg_pass_ms": vr["avg_pass_ms"], "sketch_tflops": vr["sketch_tflops"],
                "hbm_GBps": vr["hbm_GBps"], "passes_per_step": 2 * q + (2 if core == "rz" else 3),
                "pass_bound": vr["bound"], "pass_frac": vr["frac"], "pass_traffic":
                    measured_traffic(prec) if q == 1 and core == "pass" else None}
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
        pctx = cu.Context(workspace_bytes=slots * cu.workspace_bytes(M, N, K_RANK, P_OVER, 1, args.prec),
                          streams=pstreams)
        nreq = 20
        Aq = operand(args.prec)
        outs = [pctx.alloc_outputs(Aq, K_RANK, P_OVER) for _ in range(nreq)]
        for t in [pctx.submit(Aq, K_RANK, P_OVER, 1, seed=900 + i, prec=args.prec, out=outs[i]) for i in range(2)]:
            pctx.wait(t)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tickets = [pctx.submit(Aq, K_RANK, P_OVER, 1, seed=i + 1, prec=args.prec, out=outs[i])
                   for i in range(nreq)]
        for t in tickets:
            pctx.wait(t)
        torch.cuda.synchronize()
        pdt = (time.perf_counter() - t0) / nreq
        variants["%s_q1_queue_2slots" % args.prec] = {
            "corutv_per_s": round(1 / pdt, 2), "ms_per_step": round(pdt * 1e3, 3), "passes_per_step": 5,
            "requests": nreq, "slots": slots}
        pctx.close()
        del outs
    ctx.close()
    del A64, A32
    torch.cuda.empty_cache()

    small = None if args.no_small else c1_leg(cu, torch)
    precision_form = None if args.no_precision_form else c3_leg(cu, torch)
    serving = None
    if not args.no_serving:
        serving = serving_leg(cu, torch, args.serving_requests, args.serving_pool)
    rpca = None if args.no_rpca else rpca_leg(cu, torch)

    cpu = None
    parity = {"rel_err_gpu": rel_gpu}
    if not args.no_cpu_baseline:
        from oracle.corutv import corutv, rel_err

        A_o = A_h.astype(np.float64)
        log("oracle: %d float64 decompositions on the host" % args.cpu_sample)
        t0 = time.perf_counter()
        ref = None
        for i in range(args.cpu_sample):
            r = corutv(A_o, K_RANK, P_OVER, args.q, seed=i + 1)
            if i == 0:
                ref = r
        cdt = time.perf_counter() - t0
        hc = host_cpu()
        cpu = {"value": round(args.cpu_sample / cdt, 4), "unit": "CoR-UTV/s", "cores": cpu_threads(),
               "kind": "oracle",
               "sample": "%d whole float64 decompositions of the same 20000x15000 input (q=%d, l=%d), "
                         "numpy/OpenBLAS" % (args.cpu_sample, args.q, ell),
               "cpu_model": hc.get("model"), "physical_cores": hc.get("physical_cores"),
               "logical_cpus": hc.get("logical_cpus"), "affinity_cpus": hc.get("affinity_cpus")}
        parity["rel_err_oracle"] = rel_err(A_o, ref["U"], ref["T"], ref["V"])
        parity["abs_diff"] = abs(parity["rel_err_oracle"] - rel_gpu)

    line = {
        "metric": METRIC, "value": round(value, 3), "unit": "CoR-UTV/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.prec,
        "data": "synthetic",
        "config": {"workload": "CoR-UTV of a 20000x15000 exp-decay(tau=25)+1e-4 noise matrix",
                   "m": M, "n": N, "k": K_RANK, "p": P_OVER, "q": args.q, "prec": args.prec},
        "sketch_tflops": pr["sketch_tflops"],
        "roofline": roof,
        "cpu_baseline": cpu,
        "parity": parity,
        "variants": variants,
        "small_config": small,
        "precision_form": precision_form,
        "serving": serving,
        "rpca": rpca,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
