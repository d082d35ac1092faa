#!/usr/bin/env python
"""Benchmark of the t-SVD hot path on one MI355X.

Workload (one "step" = one whole t-SVD: Gram, power iteration with deflation
for every triplet, FP64 finishing pass): a dense FP32 matrix of
200,000 x 4,096 resident in HBM, A = U diag(s) V^T with Haar orthonormal
factors (Gaussian QR, seeded) and s_i = 0.97^i, k = 64 triplets.  eps is the
largest stopping tolerance whose predicted sigma error (stopping model of the
power method) is below 1e-6 relative, and the achieved error is checked
against the closed-form s after the run.

Prints ONE JSON line with the headline metric (triplets/s), the roofline of
the dominant kernel, the Gram kernel's MFMA roofline, and a CPU baseline (the
FP64 oracle timed on a bounded sample of the same workload).

``--workload serve`` measures the serving loop instead: Poisson arrivals of
dense t-SVD requests (m log-uniform in [1024, 65536], n in [128, 4096], k in
{8, 16, 32, 64}, s_i = 0.95^i) drawn from a pool of pre-generated matrices,
served by the library's request server (continuous batching, admission by
device footprint); it prints p50/p99 latency and the achieved request rate.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "A-stream GB/s + triplets/s at 1e-6 rel σ error; serving p50/p99 latency"
HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0
FP32_PEAK_TFLOPS = 157.3


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--m", type=int, default=200000)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--k", type=int, default=64)
    ap.add_argument("--q", type=float, default=0.97, help="spectrum s_i = q^i")
    ap.add_argument("--eps", type=float, default=5e-8)
    ap.add_argument("--gram", default="bf16x3", choices=["bf16x3", "fp32"])
    ap.add_argument("--compare-fp32", type=int, default=1, help="also time the plain FP32 Gram mode")
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--workload", default="dense", choices=["dense", "serve", "stream", "sparse", "batch", "oom"])
    ap.add_argument("--legs", default="serve,stream",
                    help="dense: extra legs run after the headline workload (comma list of serve, stream; '' = none)")
    ap.add_argument("--leg-window", type=float, default=8.0, help="serve leg: seconds of measured arrivals")
    ap.add_argument("--leg-stream-m", type=int, default=1_000_000, help="stream leg: rows of the pinned-host A")
    ap.add_argument("--oom-n", type=int, default=8_388_608, help="oom: m = n of the CSR matrix")
    ap.add_argument("--oom-per-row", type=float, default=50.0, help="oom: mean nonzeros per row")
    ap.add_argument("--oom-k", type=int, default=8)
    ap.add_argument("--oom-iters", type=int, default=10, help="oom: fixed iterations per triplet")
    ap.add_argument("--stream-m", type=int, default=2_000_000, help="stream: rows of the pinned-host A")
    ap.add_argument("--stream-n", type=int, default=8192)
    ap.add_argument("--stream-k", type=int, default=32)
    ap.add_argument("--batch-gb", type=float, default=4.0, help="stream: bytes of A per streamed row batch")
    ap.add_argument("--sparse-n", type=int, default=50_000_000, help="sparse: m = n of the CSR matrix")
    ap.add_argument("--sparse-density", type=float, default=1e-6)
    ap.add_argument("--sparse-k", type=int, default=16)
    ap.add_argument("--sparse-iters", type=int, default=100, help="sparse: fixed iterations per triplet")
    ap.add_argument("--sparse-row-bits", type=int, default=0, help="sparse: tile rows 2^bits (0 = library)")
    ap.add_argument("--sparse-col-bits", type=int, default=0, help="sparse: tile columns 2^bits (0 = library)")
    ap.add_argument("--rate", type=float, default=200.0, help="serve: mean arrivals per second")
    ap.add_argument("--window", type=float, default=20.0, help="serve: seconds of measured arrivals")
    ap.add_argument("--warm", type=float, default=2.0, help="serve: seconds of arrivals before the window")
    ap.add_argument("--pool", type=int, default=48, help="serve: distinct pre-generated matrices")
    ap.add_argument("--pool-loc", default="host", choices=["host", "device"],
                    help="serve: pool in pinned host memory (copied per request) or in HBM")
    ap.add_argument("--budget-gb", type=float, default=64.0, help="serve: server device budget")
    ap.add_argument("--team-kib", type=int, default=0, help="serve: batched power team size rule (0 = library)")
    ap.add_argument("--max-batch", type=int, default=0, help="serve: requests per batch launch at most (0 = all)")
    ap.add_argument("--lanes", type=int, default=0, help="serve: batches on the device at once (0 = library)")
    ap.add_argument("--batch-size", type=int, default=64, help="batch: problems per tsvd_dense_batched call")
    ap.add_argument("--gram-units", default="library", choices=["library", "tuned", "64", "128"],
                    help="batch: batched Gram unit shapes per Gram-dimension class (library choice, the "
                         "autotuner's per-class choice measured first, or one tile edge for every class)")
    ap.add_argument("--pool-gen", default="gpu", choices=["gpu", "cpu"],
                    help="serve/batch: build the matrices on the GPU or on the host (then copy)")
    return ap.parse_args()


TRAFFIC_SOURCES = {
    # key -> (file under csrc/, marker that ends the hashed part, or None for the
    # whole file); whole files, since the host-side plans set the launch shapes
    "power.hip": ("power.hip", None),
    "exchange.h": ("exchange.h", None),
    "syrk.hip": ("syrk.hip", None),
    "syrk_dev.h": ("syrk_dev.h", None),
    "common.h": ("common.h", None),
}


def source_hash(key: str) -> str:
    import hashlib
    name, marker = TRAFFIC_SOURCES[key]
    text = open(os.path.join(ROOT, "paper_2208_08410_amd", "csrc", name)).read()
    if marker:
        text = text[:text.index(marker)]
    return hashlib.sha256(text.encode()).hexdigest()[:16]


def measured_mfma():
    """Dense MFMA rates of this GPU from the C++ driver's peak loops (every CU,
    four independent chains per wave), or None when tsvd_bench is not built."""
    exe = os.path.join(ROOT, "paper_2208_08410_amd", "tsvd_bench")
    if not os.path.exists(exe):
        return None
    r = subprocess.run([exe, "mfma"], capture_output=True, text=True, timeout=120)
    if r.returncode != 0:
        return None
    return json.loads(r.stdout.strip().splitlines()[-1])


def measured_exchange(d: int):
    """Microseconds per exchange round of the power kernel's iteration
    exchange alone (the C++ driver's probe: every workgroup publishes its rows
    of a d-vector and two partial sums and gathers all of them, one workgroup
    per CU), or None when tsvd_bench is not built."""
    exe = os.path.join(ROOT, "paper_2208_08410_amd", "tsvd_bench")
    if not os.path.exists(exe):
        return None
    r = subprocess.run([exe, "exchange", str(d), "4000"], capture_output=True, text=True, timeout=120)
    if r.returncode != 0:
        return None
    return json.loads(r.stdout.strip().splitlines()[-1])


def measured_gather():
    """Random 4-byte gather rates of this GPU for gathered sets of 1 MiB to
    1 GiB (the C++ driver's probe), or None when tsvd_bench is not built."""
    exe = os.path.join(ROOT, "paper_2208_08410_amd", "tsvd_bench")
    if not os.path.exists(exe):
        return None
    r = subprocess.run([exe, "gather"], capture_output=True, text=True, timeout=300)
    if r.returncode != 0:
        return None
    return json.loads(r.stdout.strip().splitlines()[-1])


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE, WRITE_SIZE scaled by a reference copy), or None when
    a source file the kernel is built or planned from has changed since the counters
    were taken."""
    path = os.path.join(ROOT, "profiles", "traffic_power_gram_finish_dense_200000x4096_k64.txt")
    try:
        lines = open(path).read().splitlines()
    except OSError:
        return None
    recorded = {}
    for l in lines:
        if l.startswith("sha256-16 "):
            _, key, h = l.split()
            recorded[key] = h
    for l in lines:
        if l.startswith("kernel " + kernel + " "):
            f = dict(kv.split("=") for kv in l.split()[2:])
            for key in f.get("sources", "").split(","):
                if key not in TRAFFIC_SOURCES or recorded.get(key) != source_hash(key):
                    return None
            return float(f["fetch_kib"]) * 1024 * float(f["fetch_scale"]) + \
                float(f["write_kib"]) * 1024 * float(f["write_scale"])
    return None


def power_exchange_rounds(iters, k):
    """Exchange rounds of one power launch: one per iteration, and per triplet
    the re-orthogonalisation all-reduce and the gather of v, plus the gathers
    of w and of v again for every deflation (all triplets but the last)."""
    return int(sum(iters)) + 2 * k + 2 * (k - 1)


def cpu_baseline(A_dev, s, k, eps, v0):
    """The FP64 oracle, as it stands, on the whole workload: one complete
    t-SVD of the same FP32 matrix (read as FP64) with the same start vectors
    (Gram once, k projected power loops, u = A v for every triplet)."""
    import numpy as np
    import oracle as O

    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 0) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    m, n = A_dev.shape
    A_h = A_dev.cpu().double().numpy()
    st = v0.cpu().numpy()
    t0 = time.perf_counter()
    B0 = O.gram_rowblocks(A_h)
    t_gram = time.perf_counter() - t0
    r = O.tsvd_gram(A_h, eps, k, st, B0=B0)
    t_all = time.perf_counter() - t0
    rel = float(np.max(np.abs(r.S - s[:k]) / s[:k]))
    return {
        "value": k / t_all,
        "unit": "triplets/s",
        "cores": int(cores),
        "kind": "oracle",
        "sample": (f"the whole workload: one FP64 NumPy oracle t-SVD of the same {m}x{n} matrix, k={k}, eps={eps}, "
                   f"same start vectors ({int(np.sum(r.iters))} power iterations); Gram {t_gram:.1f} s, total "
                   f"{t_all:.1f} s; sigma within {rel:.1e} of the closed form"),
    }, r


def serve_cpu_baseline(shapes, ks, eps, seed):
    """Saturation throughput of the FP64 oracle serving the same request mix
    one request at a time: the Gram rate, the Gram-vector product rate and the
    u = A v rate are timed on a sample problem, then the mean request time is
    predicted for the actual shapes and k (with the GPU's iteration counts)."""
    import numpy as np
    import oracle as O
    import synth

    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 0) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    m0, n0 = 16384, 1024
    A = synth.gaussian_dense(m0, n0, seed=seed).astype(np.float64)
    t0 = time.perf_counter()
    B = O.gram_rowblocks(A)
    t_gram = time.perf_counter() - t0
    gram_rate = m0 * n0 * n0 / t_gram
    st = synth.start_vectors(1, n0, seed=seed)
    t0 = time.perf_counter()
    r = O.tsvd_gram(A, 0.0, 1, st, B0=B, max_iter=200)
    t_pow = time.perf_counter() - t0
    gemv_rate = 200 * n0 * n0 / t_pow
    t0 = time.perf_counter()
    for _ in range(5):
        A @ r.V[:, 0]
    fin_rate = 5 * m0 * n0 / (time.perf_counter() - t0)
    per = []
    for (m, n), (k, its) in zip(shapes, ks):
        d, K = min(m, n), max(m, n)
        per.append(K * d * d / gram_rate + its * d * d / gemv_rate + k * m * n / fin_rate)
    mean_s = float(np.mean(per))
    return {
        "value": 1.0 / mean_s,
        "unit": "req/s",
        "cores": int(cores),
        "kind": "oracle",
        "sample": (f"FP64 NumPy oracle rates timed on a {m0}x{n0} problem (Gram {gram_rate/1e9:.1f} G mul-add/s, "
                   f"power step {gemv_rate/1e9:.2f} G/s, u = A v {fin_rate/1e9:.2f} G/s), applied to the served "
                   f"shapes, k and iteration counts: mean {mean_s:.2f} s per request, one request at a time"),
    }


def _batch_phases(results):
    """Mean device time per batch phase (every request of a batch reports the
    same batch phase times)."""
    seen = {(x[1]["t_gram_ms"], x[1]["t_eig_ms"], x[1]["t_final_ms"], x[1]["t_total_ms"]) for x in results}
    if not seen:
        return {}
    n = len(seen)
    return {"gram": sum(t[0] for t in seen) / n, "power": sum(t[1] for t in seen) / n,
            "finish": sum(t[2] for t in seen) / n, "total": sum(t[3] for t in seen) / n, "batches_seen": n}


def request_pool(a, dev, loc):
    """The serving mix's matrices: log-uniform shapes m in [1024, 65536], n in
    [128, 4096], A = H_L [diag(0.95^i); 0] H_R, each with 64 start vectors."""
    import torch

    import synth

    q = 0.95
    g = synth.rng(a.seed, 77)
    pool = []
    progress(f"building a pool of {a.pool} matrices on the {a.pool_gen.upper()}")
    gen_dev = dev if a.pool_gen == "gpu" else torch.device("cpu")
    for j in range(a.pool):
        m = int(round(math.exp(g.uniform(math.log(1024), math.log(65536)))))
        n = int(round(math.exp(g.uniform(math.log(128), math.log(4096)))))
        s = synth.spectrum_geometric(q, min(m, n))
        A = synth.householder_known_torch(m, n, s, a.seed * 1000 + j, gen_dev)
        if A.device != dev and loc != "host":
            A = A.to(dev)
        if loc == "host":
            Ah = torch.empty((m, n), dtype=torch.float32, pin_memory=True)
            Ah.copy_(A)
            del A
            A = Ah
        d = min(m, n)
        v0 = torch.from_numpy(synth.start_vectors(64, d, seed=a.seed * 1000 + j)).to(dev)
        pool.append((A, v0, s))
    torch.cuda.synchronize()
    return pool


def batch_main(a):
    """Batched workload: a fixed batch of problems from the serving mix, solved
    by one tsvd_dense_batched call per step (one engine launch over Gram units,
    tile reductions and power-team seats, then the grouped finish), A resident
    in HBM."""
    import numpy as np
    import torch

    import paper_2208_08410_amd as P
    import synth

    dev = torch.device("cuda:0")
    t0 = time.time()
    pool = request_pool(a, dev, "device")
    gen_s = time.time() - t0
    kch = synth.rng(a.seed, 88).choice([8, 16, 32, 64], size=a.batch_size)
    pick = synth.rng(a.seed, 89).integers(0, a.pool, size=a.batch_size)
    probs = [dict(A=pool[j][0], k=int(k), eps=a.eps, v0=pool[j][1][:int(k)], gram="bf16x3") for j, k in zip(pick, kch)]
    ctx = P.Context(0)
    tune = {"team_kib": a.team_kib}
    units = None
    if a.gram_units == "tuned":
        import tempfile

        from paper_2208_08410_amd import autotune as T
        progress("tuning the batched Gram unit shape per Gram-dimension class")
        with tempfile.TemporaryDirectory() as td:
            tuner = T.Tuner(ctx, os.path.join(td, "tuning.json"), reps=2)
            units = {int(c): list(v) for c, v in tuner.tune_gram_classes([tuple(p["A"].shape) for p in probs]).items()}
            tune.update(tuner.class_tuning())
    elif a.gram_units in ("64", "128"):
        tune["group_tile"] = [int(a.gram_units)] * P.GRAM_CLASSES
    P.set_tuning(ctx, **tune)
    progress(f"batch of {a.batch_size}: {a.warmup} warm-up and {a.steps} timed calls")
    for _ in range(a.warmup):
        P.tsvd_dense_batched(ctx, probs)
    torch.cuda.synchronize()
    t_s = time.perf_counter()
    for _ in range(a.steps):
        res = P.tsvd_dense_batched(ctx, probs)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t_s
    statuses, errs = {}, []
    for (U, S, V, info), j, k in zip(res, pick, kch):
        statuses[info["status"]] = statuses.get(info["status"], 0) + 1
        if info["status"] == "TSVD_OK":
            s = pool[j][2]
            errs.append(float(np.max(np.abs(S.cpu().numpy() - s[:k]) / s[:k])))
    info0 = res[0][3]
    ctx.close()
    out = {
        "metric": METRIC,
        "value": a.batch_size * a.steps / dt,
        "unit": "requests/s (batched, A in HBM)",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": dt * 1000 / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16x3/f32acc gram, f64 finish",
        "data": "synthetic",
        "config": {"workload": f"batch of {a.batch_size} problems from the serving mix (m log-uniform [1024, 65536], "
                               f"n [128, 4096], k in {{8,16,32,64}}, s_i = 0.95^i), one tsvd_dense_batched call per "
                               f"step, eps={a.eps}", "batch_size": a.batch_size, "pool": a.pool,
                   "team_kib": a.team_kib, "gram_units": a.gram_units},
        "gram_units_tuned": units,
        "triplets_per_s": float(sum(int(k) for k in kch)) * a.steps / dt,
        "phase_ms": {"gram": info0["t_gram_ms"], "power": info0["t_eig_ms"], "finish": info0["t_final_ms"]},
        "statuses": statuses,
        "sigma_rel_err_max": float(max(errs) if errs else float("nan")),
        "meets_1e-6": bool(errs and max(errs) < 1e-6),
        "gen_seconds": gen_s,
    }
    print(json.dumps(out), flush=True)
    return 0


def serve_main(a):
    out = serve_run(a)
    print(json.dumps(out), flush=True)
    return 0


def serve_run(a):
    """Serving workload: Poisson arrivals into the library's request server."""
    import numpy as np
    import torch

    import paper_2208_08410_amd as P
    import synth

    dev = torch.device("cuda:0")
    eps = a.eps
    t0 = time.time()
    pool = request_pool(a, dev, a.pool_loc)
    gen_s = time.time() - t0
    total = a.warm + a.window
    count = int(a.rate * total * 1.5) + 16
    arrivals = synth.request_stream(count, a.rate, a.seed)
    arrivals = [r for r in arrivals if r.t < total]
    kch = synth.rng(a.seed, 78).choice([8, 16, 32, 64], size=len(arrivals))
    pick = synth.rng(a.seed, 79).integers(0, a.pool, size=len(arrivals))
    ctx = P.Context(0)
    if a.team_kib:
        P.set_tuning(ctx, team_kib=a.team_kib)
    srv = P.Server(ctx, hbm_budget=int(a.budget_gb * (1 << 30)), max_batch=a.max_batch, lanes=a.lanes)
    tickets = []
    progress(f"serving {len(arrivals)} arrivals")
    t_start = time.perf_counter()
    for i, r in enumerate(arrivals):
        now = time.perf_counter() - t_start
        if r.t > now:
            time.sleep(r.t - now)
        A, v0, s = pool[pick[i]]
        k = int(kch[i])
        tickets.append((srv.submit(dict(A=A, k=k, eps=eps, v0=v0[:k], gram="bf16x3")), r.t, i))
    progress("all submitted; collecting")
    results = []
    for tk, t_arr, i in tickets:
        U, S, V, info = srv.wait(tk)
        A, v0, s = pool[pick[i]]
        k = int(kch[i])
        rel = float(np.max(np.abs(S.cpu().numpy() - s[:k]) / s[:k]))
        results.append((t_arr, info, rel, k, tuple(A.shape)))
    t_end = time.perf_counter() - t_start
    st = srv.stats()
    server_error = srv.last_error()
    srv.close()
    ctx.close()
    meas = [x for x in results if x[0] >= a.warm]
    lat = np.array([x[1]["latency_ms"] for x in meas])
    ok = all(x[1]["status"] == "TSVD_OK" for x in results)
    statuses = {}
    for x in results:
        statuses[x[1]["status"]] = statuses.get(x[1]["status"], 0) + 1
    failed = [{"shape": x[4], "k": x[3], "status": x[1]["status"], "k_done": x[1]["k_done"]}
              for x in results if x[1]["status"] != "TSVD_OK"][:10]
    errs = np.array([x[2] for x in meas if x[1]["status"] == "TSVD_OK"] or [float("nan")])
    out = {
        "metric": METRIC,
        "value": float(np.percentile(lat, 99)),
        "unit": "ms (p99 latency)",
        "n_gpus": 1,
        "steps": len(meas),
        "warmup": len(results) - len(meas),
        "ms_per_step": float(np.mean(lat)),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16x3/f32acc gram, f64 finish",
        "data": "synthetic",
        "config": {"workload": f"serving: Poisson {a.rate:g} req/s for {a.window:g} s after {a.warm:g} s; "
                               f"m log-uniform [1024, 65536], n [128, 4096], k in {{8,16,32,64}}, s_i = 0.95^i, "
                               f"pool of {a.pool} matrices in {'pinned host memory' if a.pool_loc == 'host' else 'HBM'}"
                               f", eps={eps}", "rate": a.rate, "window_s": a.window, "pool": a.pool,
                   "pool_loc": a.pool_loc, "budget_gb": a.budget_gb, "team_kib": a.team_kib,
                   "max_batch": a.max_batch, "lanes": a.lanes},
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "max_ms": float(lat.max()),
        "requests": len(meas),
        "offered_rate": a.rate,
        "achieved_rate": len(results) / t_end,
        "all_ok": ok,
        "statuses": statuses,
        "failed_examples": failed,
        "server_error": server_error,
        "sigma_rel_err_max": float(errs.max()),
        "meets_1e-6": bool(errs.max() < 1e-6),
        "batches": st["batches"],
        "mean_batch": st["mean_batch"],
        "lanes_busy_max": st["lanes_busy_max"],
        "overlapped_launches": st["overlapped"],
        "batch_phase_ms_mean": _batch_phases(results),
        "peak_bytes": st["peak_bytes"],
        "gen_seconds": gen_s,
    }
    progress("served; timing the oracle")
    if a.cpu_baseline:
        shapes = [x[4] for x in meas]
        ks = [(x[3], int(sum(x[1]["iters"]))) for x in meas]
        out["cpu_baseline"] = serve_cpu_baseline(shapes, ks, eps, a.seed)
    del pool
    return out


def progress(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def _hip():
    import ctypes
    return ctypes.CDLL("libamdhip64.so")


def pinned_empty(rows, cols):
    """FP32 host tensor in page-locked memory from hipHostMalloc (exact size;
    torch's pinned allocator rounds sizes up to a power of two)."""
    import ctypes
    import torch
    hip = _hip()
    ptr = ctypes.c_void_p()
    nbytes = rows * cols * 4
    if hip.hipHostMalloc(ctypes.byref(ptr), ctypes.c_size_t(nbytes), 0) != 0:
        raise RuntimeError(f"hipHostMalloc({nbytes}) failed")
    buf = (ctypes.c_float * (rows * cols)).from_address(ptr.value)
    return torch.frombuffer(buf, dtype=torch.float32).view(rows, cols), ptr


def stream_main(a):
    out = stream_run(a)
    print(json.dumps(out), flush=True)
    return 0


def stream_run(a):
    """Out-of-HBM dense workload: A in pinned host memory, streamed in row
    batches (pass 1: Gram; pass 2: finishing product), spiked Gaussian rows."""
    import numpy as np
    import torch

    import paper_2208_08410_amd as P
    import synth

    dev = torch.device("cuda:0")
    m, n, k = a.stream_m, a.stream_n, a.stream_k
    R = max(128, int(a.batch_gb * (1 << 30)) // (n * 4) // 128 * 128)
    t0 = time.time()
    progress(f"pinning {m * n * 4 / 1e9:.1f} GB of host memory")
    A, ptr = pinned_empty(m, n)
    progress("filling A")
    y, theta = synth.spiked_factors(m, n, 32, a.seed)
    yd = torch.as_tensor(y, device=dev)
    for r0 in range(0, m, R):
        rows = min(R, m - r0)
        A[r0:r0 + rows].copy_(synth.spiked_rows_torch(m, n, 32, a.seed, r0, rows, dev, yfac=yd))
        progress(f"rows {r0 + rows}/{m}")
    torch.cuda.synchronize()
    gen_s = time.time() - t0
    # plain pinned host -> device copy of one batch: the host link's achievable rate
    dst = torch.empty((R, n), dtype=torch.float32, device=dev)
    best = 1e30
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(A[:R], non_blocking=True)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    copy_gbs = R * n * 4 / (best * 1e-3) / 1e9
    del dst
    v0 = torch.from_numpy(synth.start_vectors(k, n, seed=a.seed + 5)).to(dev)
    ctx = P.Context(0)
    # warm-up on the first two batches (allocates the device buffers)
    progress("warm-up")
    P.tsvd_dense(ctx, A[:2 * R], k, a.eps, v0, rows_per_block=R, queue_depth=2)
    progress("timed run")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    U, S, V, info = P.tsvd_dense(ctx, A, k, a.eps, v0, rows_per_block=R, queue_depth=2)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t1
    Sh = S.cpu().numpy()
    gbs = info["h2d_bytes"] / dt / 1e9
    out = {
        "metric": METRIC,
        "value": gbs,
        "unit": "GB/s (A streamed host->device)",
        "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16x3/f32acc gram, f64 finish", "data": "synthetic",
        "config": {"workload": f"out-of-HBM FP32 A {m}x{n} in pinned host memory, N(0,1) + rank-32 spike "
                               f"(theta_j = 50 sqrt(m) 0.9^j); k={k}, eps={a.eps}; {R}-row batches "
                               f"({R * n * 4 / 2**30:.2f} GiB), 2 device buffers", "m": m, "n": n, "k": k,
                   "rows_per_batch": R},
        "roofline": {"bound": "host link", "achieved": gbs, "peak": 64.0, "unit": "GB/s", "frac": gbs / 64.0,
                     "traffic": None, "note": "PCIe 5.0 x16 per direction, published"},
        "plain_copy_gbs": copy_gbs,
        "frac_of_plain_copy": gbs / copy_gbs,
        "h2d_bytes": info["h2d_bytes"],
        "phase_ms": {"gram_pass": info["t_gram_ms"], "power": info["t_eig_ms"], "finish_pass": info["t_final_ms"]},
        "gram_pass_gbs": m * n * 4 / (info["t_gram_ms"] * 1e-3) / 1e9,
        "overlap": {"copy_ms": info["t_stream_copy_ms"], "compute_ms": info["t_stream_compute_ms"],
                    "overlapped_ms": info["t_stream_overlap_ms"],
                    "frac_of_compute_hidden": info["t_stream_overlap_ms"] / max(info["t_stream_compute_ms"], 1e-9),
                    "frac_of_copy_overlapped": info["t_stream_overlap_ms"] / max(info["t_stream_copy_ms"], 1e-9),
                    "note": "Gram pass: per-batch HIP event intervals on the copy stream and the compute stream "
                            "(the library's own events); overlapped = time both streams were busy at once"},
        "iters_total": int(sum(info["iters"])),
        "sigma_top": [float(x) for x in Sh[:4]],
        "theta_top": [float(x) for x in theta[:4]],
        "gen_seconds": gen_s,
    }
    ctx.close()
    del A
    _hip().hipHostFree(ptr)
    return out


def sparse_main(a):
    """Sparse workload: CSR with uniform random columns, implicit A^T (A x)."""
    import torch

    import paper_2208_08410_amd as P
    import synth

    dev = torch.device("cuda:0")
    n = a.sparse_n
    k = a.sparse_k
    t0 = time.time()
    progress("generating the CSR matrix")
    rowptr, col, val = synth.csr_uniform_torch(n, n, a.sparse_density, a.seed, dev)
    torch.cuda.synchronize()
    gen_s = time.time() - t0
    nnz = col.numel()
    ctx = P.Context(0)
    if a.sparse_row_bits or a.sparse_col_bits:
        P.set_tuning(ctx, sparse_row_bits=a.sparse_row_bits, sparse_col_bits=a.sparse_col_bits)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    progress(f"{nnz} nonzeros; building the CSC copy")
    e0.record()
    csr = P.tsvd_csr_create(ctx, rowptr, col, val, (n, n))
    e1.record()
    e1.synchronize()
    csc_ms = e0.elapsed_time(e1)
    # SpMV rates (FP32 x, FP64 y), both directions
    x = torch.randn(n, dtype=torch.float32, device=dev)
    rates = {}
    for trans in (0, 1):
        P.tsvd_spmv(ctx, csr, x, trans=trans)
        torch.cuda.synchronize()
        best = 1e30
        for _ in range(3):
            e0.record()
            P.tsvd_spmv(ctx, csr, x, trans=trans)
            e1.record()
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1))
        # algorithmic bytes of one product: index + value per nonzero, row
        # pointers, x read once, y written once
        alg = nnz * (4 + 4) + (n + 1) * 8 + n * 4 + n * 8
        rates["csr" if trans == 0 else "csc"] = {"ms": best, "gbs": alg / (best * 1e-3) / 1e9}
    g = torch.Generator(device=dev)
    g.manual_seed(a.seed)
    v0 = torch.randn((k, n), generator=g, dtype=torch.float64, device=dev)
    its = [a.sparse_iters] * k
    progress("SpMV timed; t-SVD warm-up")
    P.tsvd_sparse(ctx, csr, 1, 0.0, v0[:1], fixed_iters=[2])  # warm-up
    progress("timed t-SVD")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    U, S, V, info = P.tsvd_sparse(ctx, csr, k, 0.0, v0, fixed_iters=its)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t1
    per_iter = dt * 1e3 / (k * a.sparse_iters)
    pair = 2 * (nnz * 8 + (n + 1) * 8 + n * 4 + n * 8)
    # the binding ceiling: random gathers of x inside one XCD's L2 (each tile
    # gathers from one 1 MiB slice of FP32 x), measured by the driver's probe
    gp = measured_gather()
    slice_mib = (1 << (a.sparse_col_bits or 18)) * 4 / (1 << 20)
    gpeak = None
    if gp:
        sets = sorted(gp["sets"], key=lambda e: abs(e["set_mib"] - slice_mib))
        gpeak = sets[0]["g_gathers_per_s"]
    gach = nnz / (rates["csr"]["ms"] * 1e-3) / 1e9
    roof_sp = {"kernel": "spmv_tiles_kernel<float> (A x)", "bound": "l2 gather", "achieved": gach, "peak": gpeak,
               "unit": "G gathers/s", "frac": (gach / gpeak) if gpeak else None, "traffic": None,
               "note": "one 4-byte x gather per nonzero; peak = random gathers over a set the size of one column "
                       "slice of x (tsvd_bench gather, same GPU)"}
    out = {
        "metric": METRIC,
        "value": pair / (per_iter * 1e-3) / 1e9,
        "unit": "GB/s (A-stream, SpMV pair per iteration)",
        "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 values, f64 accumulation", "data": "synthetic",
        "config": {"workload": f"sparse CSR {n}x{n}, density {a.sparse_density:g} ({nnz} nnz), uniform random "
                               f"columns, N(0,1) values; k={k}, {a.sparse_iters} fixed iterations per triplet",
                   "n": n, "nnz": nnz, "k": k, "tile_bits": [a.sparse_row_bits, a.sparse_col_bits]},
        "roofline": roof_sp,
        "roofline_hbm_view": {"bound": "hbm", "achieved": rates["csr"]["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": rates["csr"]["gbs"] / HBM_PEAK_GBS,
                              "note": "algorithmic bytes (index + value per nonzero, row pointers, x and y once)"},
        "gather_probe": gp,
        "spmv": rates,
        "ms_per_iteration": per_iter,
        "csc_build_ms": csc_ms,
        "triplets_per_s": k / dt,
        "sigma_top": [float(x) for x in S[:4].cpu()],
        "gen_seconds": gen_s,
    }
    csr.close()
    ctx.close()
    print(json.dumps(out), flush=True)
    return 0


def oom_main(a):
    """Out-of-memory sweep of the sparse path, the paper's degree-1 experiment
    (Sec. VI-B, fixed iterations): A's tiles in HBM and the heavy co-factor V
    in pinned host memory, batched to the device in n_b row batches through
    q_s device buffers for every projection.  Reports time and peak device
    memory per (n_b, q_s) with q_s <= n_b, next to V on the device, and one run
    with A's tiles streamed from pinned host memory as well."""
    import numpy as np
    import torch

    import paper_2208_08410_amd as P
    import synth

    dev = torch.device("cuda:0")
    n, k = a.oom_n, a.oom_k
    progress(f"generating the CSR matrix {n}x{n}, {a.oom_per_row:g} nonzeros per row")
    rowptr, col, val = synth.csr_uniform_torch(n, n, a.oom_per_row / n, a.seed, dev)
    nnz = col.numel()
    ctx = P.Context(0)
    csr = P.tsvd_csr_create(ctx, rowptr, col, val, (n, n))
    g = torch.Generator(device=dev)
    g.manual_seed(a.seed)
    v0 = torch.randn((k, n), generator=g, dtype=torch.float64, device=dev)
    its = [a.oom_iters] * k
    P.tsvd_sparse(ctx, csr, 1, 0.0, v0[:1], fixed_iters=[2])  # warm-up

    def run(handle, **kw):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        U, S, V, info = P.tsvd_sparse(ctx, handle, k, 0.0, v0, fixed_iters=its, **kw)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        peak = info["workspace_bytes"] + handle.info()["device_bytes"]
        return ms, peak, info["h2d_bytes"], S.cpu()

    progress("V on the device")
    ms0, peak0, _, S0 = run(csr)
    sweep = []
    for nb in (2, 4, 8, 16):
        for qs in (1, 2, 4, 8):
            if qs > nb:
                continue
            progress(f"V in pinned host memory: n_b={nb}, q_s={qs}")
            ms, peak, h2d, S1 = run(csr, factor="host", factor_batches=nb, queue_depth=qs)
            sweep.append({"n_b": nb, "q_s": qs, "ms": ms, "peak_device_gb": peak / 1e9, "h2d_gb": h2d / 1e9,
                          "h2d_gbs": h2d / (ms * 1e-3) / 1e9, "bitwise_equal_to_device_V": bool(torch.equal(S0, S1))})
    progress("tiles and V both in pinned host memory")
    pin = P.tsvd_csr_create_pinned(ctx, rowptr.cpu().pin_memory(), col.cpu().pin_memory(), val.cpu().pin_memory(),
                                   (n, n), batch_bytes=256 << 20, queue_depth=2)
    msp, peakp, h2dp, Sp = run(pin, factor="host", factor_batches=8, queue_depth=2)
    all_host = {"ms": msp, "peak_device_gb": peakp / 1e9, "h2d_gb": h2dp / 1e9, "h2d_gbs": h2dp / (msp * 1e-3) / 1e9,
                "tile_batches": pin.info()["batches"], "bitwise_equal_to_device": bool(torch.equal(S0, Sp))}
    pin.close()
    csr.close()
    ctx.close()
    best = min(sweep, key=lambda r: r["ms"])
    out = {
        "metric": METRIC,
        "value": best["ms"],
        "unit": "ms (t-SVD, fastest host-V configuration)",
        "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": best["ms"],
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 values, f64 accumulation and factor", "data": "synthetic",
        "config": {"workload": f"out-of-memory sweep: sparse CSR {n}x{n}, Poisson({a.oom_per_row:g}) uniform columns "
                               f"per row ({nnz} nnz), k={k}, {a.oom_iters} fixed iterations per triplet; V (FP64 "
                               f"{n}x{k}) in pinned host memory, n_b row batches through q_s device buffers",
                   "n": n, "nnz": nnz, "k": k, "iters": a.oom_iters},
        "v_on_device": {"ms": ms0, "peak_device_gb": peak0 / 1e9},
        "sweep": sweep,
        "tiles_and_v_on_host": all_host,
    }
    print(json.dumps(out), flush=True)
    return 0


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py: the library runs on one GPU; multi-GPU (N > 1) is not implemented "
              "(how the path would shard is part of the design notes).", file=sys.stderr)
        return 2
    if a.workload == "batch":
        return batch_main(a)
    if a.workload == "serve":
        return serve_main(a)
    if a.workload == "stream":
        return stream_main(a)
    if a.workload == "sparse":
        return sparse_main(a)
    if a.workload == "oom":
        return oom_main(a)
    import numpy as np
    import torch

    import paper_2208_08410_amd as P
    import synth

    dev = torch.device("cuda:0")
    s = synth.spectrum_geometric(a.q, min(a.m, a.n))
    t0 = time.time()
    A, Utrue, Vtrue = synth.dense_known_torch(a.m, a.n, s, a.seed, dev, keep_factors=a.k)
    v0 = torch.from_numpy(synth.start_vectors(a.k, a.n, seed=a.seed + 100)).to(dev)
    torch.cuda.synchronize()
    gen_s = time.time() - t0
    ctx = P.Context(0)

    def step(gram):
        return P.tsvd_dense(ctx, A, a.k, a.eps, v0, gram=gram)

    def timed(gram):
        for _ in range(a.warmup):
            step(gram)
        torch.cuda.synchronize()
        infos = []
        t0 = time.perf_counter()
        for _ in range(a.steps):
            U, S, V, info = step(gram)
            infos.append(info)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        return dt, infos, (U, S, V)

    dt, infos, (U, S, V) = timed(a.gram)
    ms_step = dt * 1000 / a.steps
    Sh = S.cpu().numpy()
    rel = np.abs(Sh - s[: a.k]) / s[: a.k]
    Vg = V.cpu().numpy()
    Vt = Vtrue.cpu().numpy()
    cosv = np.abs(np.sum(Vg * Vt, axis=0) / np.linalg.norm(Vt, axis=0))
    ang = float(np.max(np.arccos(np.clip(cosv, -1, 1))))
    info = infos[-1]
    t_gram = float(np.mean([i["t_gram_ms"] for i in infos]))
    t_eig = float(np.mean([i["t_eig_ms"] for i in infos]))
    t_fin = float(np.mean([i["t_final_ms"] for i in infos]))
    a_bytes = a.m * a.n * 4
    a_stream = 2 * a_bytes / ((t_gram + t_fin) * 1e-3) / 1e9
    phases = {"gram": t_gram, "power": t_eig, "finish": t_fin}
    dominant = max(phases, key=phases.get)
    # the library's default tiles: 256 x 256 for BF16X3 Grams of dimension >= 1024, else 128 x 128
    bm = 256 if (a.gram == "bf16x3" and a.n >= 1024) else 128
    nt = (a.n + bm - 1) // bm
    gram_flops_hw = (3 if a.gram == "bf16x3" else 1) * 2.0 * a.m * (nt * (nt + 1) // 2) * bm * bm
    # A resident in HBM: 256-wide BF16X3 Grams take the two-pass form (split into
    # BF16 planes, then the direct-to-LDS tile kernel) whenever the planes fit
    gram_kernel = ("split_pack_kernel<0> + syrk_packed_kernel + syrk_reduce_kernel<float,256>" if bm == 256 else
                   "syrk_partial_kernel<%s,0> + syrk_reduce_kernel<float,128>" % a.gram)
    c2_shape = a.n == 4096 and a.m == 200000 and a.k == 64
    gram_flops_alg = 1.0 * a.m * a.n * (a.n + 1)
    gram_peak = BF16_PEAK_TFLOPS if a.gram == "bf16x3" else FP32_PEAK_TFLOPS
    roof_gram = {
        "kernel": gram_kernel,
        "bound": "mfma",
        "achieved": gram_flops_hw / (t_gram * 1e-3) / 1e12,
        "peak": gram_peak,
        "unit": "TFLOP/s",
        "frac": gram_flops_hw / (t_gram * 1e-3) / 1e12 / gram_peak,
        "traffic": measured_traffic("split_pack_kernel<0>+syrk_packed_kernel+syrk_reduce_kernel<float,256>")
        if (c2_shape and bm == 256) else None,
        "traffic_note": "HBM bytes per launch pair from profiles/traffic_*.txt; A alone is m*n*4 bytes",
        "effective_fp32_equiv_tflops": gram_flops_alg / (t_gram * 1e-3) / 1e12,
    }
    traffic = measured_traffic("power_kernel<float,16,2>") if c2_shape else None
    iters_total = int(sum(info["iters"]))
    rounds = power_exchange_rounds(info["iters"], a.k)
    ex = measured_exchange(a.n)
    floor_ms = rounds * ex["exchange_us_per_round"] * 1e-3 if ex else None
    gemv_flops = 2.0 * a.n * a.n * (iters_total + (a.k - 1))
    roof_power = {
        "kernel": "power_kernel<float,16,2>" if a.n == 4096 else "power_kernel<float,...>",
        "bound": "exchange latency",
        "achieved": rounds / (t_eig * 1e-3),
        "peak": (rounds / (floor_ms * 1e-3)) if floor_ms else None,
        "unit": "exchange rounds/s",
        "frac": (floor_ms / t_eig) if floor_ms else None,
        "traffic": traffic,
        "traffic_note": "HBM bytes per launch from profiles/traffic_*.txt (rocprofv3 FETCH_SIZE/WRITE_SIZE, scaled "
                        "by a reference copy); B stays on chip, so HBM traffic is far below n^2 * 4 B per iteration",
        "exchange_rounds_per_launch": rounds,
        "exchange_floor_us_per_round": ex["exchange_us_per_round"] if ex else None,
        "exchange_floor_ms_per_launch": floor_ms,
        "us_per_iteration": t_eig * 1e3 / max(1, iters_total),
        "note": "the kernel's bound: every iteration ends in an all-gather of the iterate among all workgroups; "
                "peak = rounds per launch at the measured latency of that exchange alone (tsvd_bench exchange)",
        "alu_view": {"bound": "alu", "achieved": gemv_flops / (t_eig * 1e-3) / 1e12, "peak": FP32_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": gemv_flops / (t_eig * 1e-3) / 1e12 / FP32_PEAK_TFLOPS,
                     "note": "2 n^2 flops per product (one per iteration, one per deflation) against the FP32 "
                             "vector peak"},
    }
    roofline = roof_power if dominant == "power" else roof_gram
    out = {
        "metric": METRIC,
        "value": a.k * a.steps / dt,
        "unit": "triplets/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16x3/f32acc gram, f64 finish" if a.gram == "bf16x3" else "f32 gram, f64 finish",
        "data": "synthetic",
        "config": {"workload": f"dense in-HBM FP32 A {a.m}x{a.n}, s_i={a.q}^i, Haar factors; k={a.k}, "
                               f"eps={a.eps}", "m": a.m, "n": a.n, "k": a.k, "eps": a.eps, "gram": a.gram},
        "roofline": roofline,
        "roofline_gram": roof_gram,
        "roofline_power": roof_power,
        "a_stream_gbs": a_stream,
        "phase_ms": phases,
        "iters_total": int(sum(info["iters"])),
        "sigma_rel_err_max": float(rel.max()),
        "v_angle_max_rad": ang,
        "meets_1e-6": bool(rel.max() < 1e-6),
        "gen_seconds": gen_s,
    }
    if a.compare_fp32 and a.gram != "fp32":
        dt32, infos32, (U32, S32, V32) = timed("fp32")
        rel32 = np.abs(S32.cpu().numpy() - s[: a.k]) / s[: a.k]
        out["compare_fp32"] = {
            "ms_per_step": dt32 * 1000 / a.steps,
            "value": a.k * a.steps / dt32,
            "gram_ms": float(np.mean([i["t_gram_ms"] for i in infos32])),
            "sigma_rel_err_max": float(rel32.max()),
        }
    # measured HBM rate next to the datasheet peak: a 2 GiB device-to-device copy
    src = torch.empty(1 << 29, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    best = 1e30
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    out["hbm_copy_gbs_measured"] = 2 * src.numel() * 4 / (best * 1e-3) / 1e9
    del src, dst
    # measured dense MFMA rates (the C++ driver's peak loops, run as a child process)
    mm = measured_mfma()
    if mm:
        out["mfma_measured"] = mm
        if a.gram == "bf16x3":
            roof_gram["frac_of_measured_peak"] = roof_gram["achieved"] / mm["mfma_bf16_tflops"]
    if a.cpu_baseline:
        progress("timing the FP64 oracle on the whole workload")
        out["cpu_baseline"], ref = cpu_baseline(A, s, a.k, a.eps, v0)
        # parity with the oracle on this workload: the GPU path in trajectory
        # mode (the oracle's iteration counts, same start vectors), both Gram forms
        import oracle as O
        Ur, Vr = O.canonical(ref.U, ref.V)
        par = {}
        for g in ([a.gram, "fp32"] if a.gram != "fp32" else ["fp32"]):
            Ut, St, Vt_, it_ = P.tsvd_dense(ctx, A, a.k, a.eps, v0, gram=g, fixed_iters=[int(x) for x in ref.iters])
            St, Ut, Vt_ = St.cpu().numpy(), Ut.cpu().numpy(), Vt_.cpu().numpy()
            cv = np.clip(np.abs(np.sum(Vt_ * Vr, axis=0)), 0, 1)
            cu = np.clip(np.abs(np.sum(Ut * Ur, axis=0)), 0, 1)
            sv_ = np.sqrt(np.maximum(0.0, 1 - cv * cv))
            su_ = np.sqrt(np.maximum(0.0, 1 - cu * cu))
            par[g] = {"sigma_rel_vs_oracle": float(np.max(np.abs(St - ref.S) / ref.S)),
                      "v_angle_vs_oracle_rad": float(np.max(np.arctan2(sv_, cv))),
                      "u_angle_vs_oracle_rad": float(np.max(np.arctan2(su_, cu)))}
            par[g]["meets_1e-6_sigma_1e-4_rad"] = bool(par[g]["sigma_rel_vs_oracle"] < 1e-6 and
                                                       par[g]["v_angle_vs_oracle_rad"] < 1e-4 and
                                                       par[g]["u_angle_vs_oracle_rad"] < 1e-4)
        out["parity_vs_oracle"] = par
        out["meets_1e-6"] = bool(out["meets_1e-6"] and par[a.gram]["meets_1e-6_sigma_1e-4_rad"])
    ctx.close()
    del A, Utrue, Vtrue, U, S, V
    torch.cuda.empty_cache()
    legs = [x for x in a.legs.split(",") if x]
    if legs:
        out["legs"] = {}
    if "serve" in legs:
        progress("serving leg")
        sa = argparse.Namespace(**vars(a))
        # the serving workload's own pool (48 matrices of the mix) in pinned host memory
        sa.window, sa.warm, sa.pool, sa.pool_loc = a.leg_window, 2.0, 48, "host"
        r = serve_run(sa)
        out["legs"]["serve"] = {k_: r[k_] for k_ in ("config", "p50_ms", "p99_ms", "max_ms", "requests", "offered_rate",
                                                      "achieved_rate", "all_ok", "sigma_rel_err_max", "meets_1e-6",
                                                      "batches", "mean_batch", "lanes_busy_max",
                                                      "overlapped_launches", "batch_phase_ms_mean",
                                                      "cpu_baseline") if k_ in r}
        torch.cuda.empty_cache()
    if "stream" in legs:
        progress("streaming leg")
        sa = argparse.Namespace(**vars(a))
        sa.stream_m = a.leg_stream_m
        r = stream_run(sa)
        out["legs"]["stream"] = {k_: r[k_] for k_ in ("config", "value", "unit", "ms_per_step", "roofline",
                                                       "plain_copy_gbs", "frac_of_plain_copy", "gram_pass_gbs",
                                                       "overlap", "phase_ms", "h2d_bytes")}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
