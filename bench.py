#!/usr/bin/env python
"""Benchmark of the dual-kernel hot path on one MI355X.

Workload (one step = one pass of the whole hot path): 784-qubit synthetic
28x28 "images" (10 classes, seeded smooth field per class + pixel noise,
scaled to [0, pi]), 4000 training + 1000 test samples, 2 layers, chi_max 64,
cutoff 1e-10. A step builds the MPS of all 5000 samples on the device
(TEBD, FP64), packs them, and runs ONE persistent sweep launch over the
train x train upper triangle (diagonal included) and the test x train
rectangle with the fused epilogue (ln K_q, K_q, K_c with gamma = 1/d, and
K = 0.5 K_q + 0.5 K_c, all FP64). Inputs are resident in HBM before timing.

value = unique pairs per second = (4000*4001/2 + 1000*4000) / seconds per step.

The plain complex-FP64 sweep runs the same step as the comparator; the CPU
oracle is timed on a bounded sample on the host cores (cpu_baseline).
Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAKS = {  # published MI355X figures, TFLOP/s
    "fp64": ("alu", 78.6), "fp32": ("alu", 157.3), "fp32_mfma": ("mfma", 157.3),
    "bf16x2": ("mfma", 2500.0), "bf16x3": ("mfma", 2500.0),
}
# HBM bytes per sweep launch from the rocprofv3 FETCH_SIZE / WRITE_SIZE runs
# summarised under profiles/ (scaled by the copy-kernel calibration), valid
# only for the kernel source they were taken with.
TRAFFIC = {"fp32_mfma": {"source": "paper_2602_01330_amd/csrc/sweep_mfma.hip",
                         "sha256_prefix": "ca4b6e321d0a5d14",
                         "bytes": 296.2e9 + 0.809e9},
           "fp32_mfma_wide": {"source": "paper_2602_01330_amd/csrc/sweep_wide.hip",
                              "sha256_prefix": "d9cf1b83de8347d1",
                              "bytes": 143.1e9 + 0.0027e9},
           # per step of the path-sum leg (both launches)
           "pathsum_l2_step": {"source": "paper_2602_01330_amd/csrc/pathsum.hip",
                               "sha256_prefix": "5a94561d7e8a54e6",
                               "bytes": 24.584e9 + 0.640e9}}
DTYPE = {"fp64": "f64", "fp32": "f32", "fp32_mfma": "f32", "bf16x2": "bf16", "bf16x3": "bf16"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_flops(chi_rows, chi_cols, symmetric):
    """Sum over pairs of sum_k 16 (cA_k cB_k cB_{k+1} + cA_{k+1} cA_k cB_{k+1})
    on realized bond dimensions (8 real FLOP per complex MAC). A symmetric
    job contracts the pairs (i, j), j >= i, with row sample i on the A side."""
    import numpy as np
    A = chi_rows.astype(np.float64)
    B = chi_cols.astype(np.float64)
    u, w = A[:, :-1], A[:, 1:] * A[:, :-1]     # row-side factors per site
    v, z = B[:, :-1] * B[:, 1:], B[:, 1:]      # column-side factors per site
    if not symmetric:
        return 16.0 * float((u.sum(0) * v.sum(0) + w.sum(0) * z.sum(0)).sum())
    # sum over i <= j of u_i v_j = sum_j v_j (u_0 + ... + u_j)
    cu, cw = np.cumsum(u, axis=0), np.cumsum(w, axis=0)
    return 16.0 * float((cu * v).sum() + (cw * z).sum())


def traffic_for(form, shape=None):
    """Measured HBM bytes per launch, or None if the kernel changed since or
    (for an entry taken at one launch shape) the launch used another shape:
    the tile order and the workgroups per CU decide how much of the operand
    stream the L2 caches share."""
    import hashlib
    t = TRAFFIC.get(form)
    if t is None:
        return None
    if "shape" in t and (shape is None or tuple(shape) != tuple(t["shape"])):
        return None
    with open(os.path.join(ROOT, t["source"]), "rb") as f:
        h = hashlib.sha256(f.read()).hexdigest()
    return t["bytes"] if h.startswith(t["sha256_prefix"]) else None


def launch_shape(tune_text, T, nq, form_code):
    """(workgroups per CU, band height) of the tuning entry for bond bound T
    and nq qubits when it was tuned for this form (else the library's
    defaults, 2 and 4), from the text of qk_tune_export: one entry per line,
    'T bucket form wg_per_cu band us_per_tile', bucket = ceil(log2 nq)."""
    bucket = max(0, math.ceil(math.log2(nq))) if nq > 1 else 0
    for line in (tune_text or "").splitlines():
        f = line.split()
        if len(f) >= 5 and int(f[0]) == T and int(f[1]) == bucket and int(f[2]) == form_code:
            return int(f[3]), int(f[4])
    return 2, 4


def gpu_state_held():
    """Reasons this process holds GPU state (empty if none): an open /dev/kfd
    (the HSA runtime has started), torch's CUDA/HIP state initialised, or
    libqk.so mapped. A process in any of these states must not fork: the
    children would share the runtime's queues, signals and device mappings
    copy-on-write with the parent."""
    reasons = []
    try:
        for fd in os.listdir("/proc/self/fd"):
            try:
                if os.readlink(os.path.join("/proc/self/fd", fd)) == "/dev/kfd":
                    reasons.append("/dev/kfd is open")
                    break
            except OSError:
                pass
    except OSError:
        pass
    torch = sys.modules.get("torch")
    if torch is not None and torch.cuda.is_initialized():
        reasons.append("torch's GPU state is initialised")
    try:
        with open("/proc/self/maps") as f:
            if "libqk.so" in f.read():
                reasons.append("libqk.so is loaded")
    except OSError:
        pass
    return reasons


def cpu_model():
    """Host CPU description from /proc/cpuinfo and the sysfs topology."""
    info = {}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if ":" not in line:
                    continue
                k, v = (t.strip() for t in line.split(":", 1))
                if k in ("model name", "vendor_id", "cpu family", "model", "stepping",
                          "cpu MHz", "cache size") and k not in info:
                    info[k] = v
    except OSError:
        pass
    try:
        info["online"] = open("/sys/devices/system/cpu/online").read().strip()
    except OSError:
        pass
    info["affinity_cpus"] = len(os.sched_getaffinity(0))
    return info


# The worker pool is sized to the host threads this process may use, at most
# 16: the CPU share of one GPU on the machines this runs on.
CPU_WORKERS_MAX = 16


def cpu_baseline(x_tr, seconds_target=15.0):
    """Time the FP64 oracle on a bounded sample with a process pool forked
    from this process, which must hold no GPU state (checked: it raises
    otherwise, whatever order the caller runs its legs in)."""
    import multiprocessing as mp
    held = gpu_state_held()
    if held:
        raise RuntimeError("cpu_baseline forks worker processes and must run before anything "
                           "touches the GPU: " + "; ".join(held))
    avail = len(os.sched_getaffinity(0))
    cores = min(avail, CPU_WORKERS_MAX)
    n_build, n_pairs = 8, 24576
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(cores, initializer=_pool_init) as pool:
        res = pool.map(_oracle_chunk, [(x_tr[(4 * w) % (len(x_tr) - 4):][:n_build], n_pairs)
                                       for w in range(cores)])
    wall = time.perf_counter() - t0
    build_s = max(r[0] for r in res)
    sweep_s = max(r[1] for r in res)
    build_rate = cores * n_build / build_s        # samples / s
    sweep_rate = cores * n_pairs / sweep_s        # pairs / s
    pairs = 4000 * 4001 // 2 + 1000 * 4000
    job_s = 5000 / build_rate + pairs / sweep_rate
    cpu = cpu_model()
    return {"value": pairs / job_s, "unit": "entries/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu.get("model name", "unknown"), "cpu": cpu,
            "cpus_available": avail,
            "sample": (f"{cores} processes (one per host thread available, at most "
                       f"{CPU_WORKERS_MAX}) x ({n_build} TEBD builds + {n_pairs} FP64 pair "
                       f"sweeps) at d=784, L=2; wall {wall:.1f}s; whole-job rate "
                       f"extrapolated to 5000 builds + {pairs} pairs")}


def cpu_baseline_pathsum(x_tr, n_layers):
    """The oracle's path-sum timed on a bounded sample of train pairs (one
    process, one core): returns (pairs per second, sample size)."""
    import numpy as np
    from oracle import pathsum as opathsum
    rng = np.random.default_rng(11)
    ns = 1024 if n_layers < 3 else 128  # about 5 s of oracle time either way
    n = x_tr.shape[0]
    sample = np.stack([rng.integers(0, n, ns), rng.integers(0, n, ns)], axis=1)
    t0 = time.perf_counter()
    opathsum.ln_kernel_pairs(x_tr, x_tr, n_layers, sample)
    return len(sample) / (time.perf_counter() - t0), ns


def cpu_baseline_svm(K, y, n_classes, C_box, eps):
    """The oracle's SMO on the same one-against-one problems (one core):
    returns (steps per problem, seconds)."""
    from oracle import svm as osvm
    t0 = time.perf_counter()
    _, _, it_ref = osvm.fit_ovo(K, y, n_classes, C_box, eps)
    return it_ref, time.perf_counter() - t0


def _pool_init():
    os.environ["OMP_NUM_THREADS"] = "1"
    os.environ["OPENBLAS_NUM_THREADS"] = "1"


def _oracle_chunk(args):
    import numpy as np
    from oracle import mps
    xs, n_pairs = args
    t0 = time.perf_counter()
    M = mps.build_batch(xs, 2, 64)
    t1 = time.perf_counter()
    P = mps.pad_batch(M)
    rng = np.random.default_rng(0)
    pairs = rng.integers(len(xs), size=(n_pairs, 2))
    mps.ln_kernel_pairs(P, P, pairs)
    t2 = time.perf_counter()
    return t1 - t0, t2 - t1


def serving(args):
    """Serving against resident support sets (5000 samples per d in
    {16, 64, 256, 784}, L = 2, chi_max 64): requests of 1..64 test rows, d and
    w drawn per request; latency = rows on the host - submission. Three runs
    on one server configuration each:
    - open loop: the Poisson stream (rate --serve-rate, --serve-warmup s of
      warm-up, --serve-seconds s measured) under a 1 GiB budget;
    - budget-bound: the same stream's first part under a budget that admits
      the largest request but only about two of them at once, so requests
      queue for memory (peak reservation reported);
    - closed loop (saturation): --serve-inflight requests always outstanding
      for --serve-sat-seconds s, each completion submitting the next: the
      largest delivered entries/s."""
    import threading
    import queue
    import numpy as np
    import torch

    import paper_2602_01330_amd.qk as qk
    from synthdata import config_inputs, gen_requests
    from synthdata.generators import C5_DIMS

    # the client submits on a Poisson schedule from one thread while another
    # drains results; a short GIL switch interval keeps the schedule on time
    sys.setswitchinterval(2e-4)
    dev = torch.device("cuda:0")
    pools, sups = {}, {}
    for d in C5_DIMS:
        sup, pool, _ = config_inputs("C5", d=d, n_train=5000, n_test=1024)
        sups[d] = torch.as_tensor(sup, device=dev)
        pools[d] = pool
    rng = np.random.default_rng(56)

    def make(budget):
        srv = qk.qk_server_create(budget_bytes=budget, max_rows_per_iter=512, n_streams=2,
                                  prec="auto")
        for d in C5_DIMS:
            qk.qk_server_load_support(srv, sups[d], 2, 64)
        return srv

    def pick(d, n):
        off = int(rng.integers(0, pools[d].shape[0] - n))
        return pools[d][off:off + n]

    def open_loop(budget, warm, dur):
        reqs = gen_requests(55, args.serve_rate, warm + dur, dims=C5_DIMS)
        srv = make(budget)
        try:
            submitted = queue.Queue()
            t_start = time.perf_counter()

            def submitter():
                for r in reqs:
                    delay = t_start + r["t"] - time.perf_counter()
                    if delay > 0:
                        time.sleep(delay)
                    rid = qk.qk_server_submit(srv, pick(r["d"], r["n_rows"]), r["w"])
                    submitted.put((rid, r))
                submitted.put(None)

            th = threading.Thread(target=submitter)
            th.start()
            out = np.empty((64, 5000))
            lat, queued, entries, t_first, t_last, sub = [], [], 0, None, 0.0, []
            while True:
                item = submitted.get()
                if item is None:
                    break
                rid, r = item
                st = qk.qk_server_wait(srv, rid, -1)
                ts, ta, td = qk.qk_server_request_times(srv, rid)
                qk.qk_server_poll(srv, rid, out)
                if st != qk.QK_REQ_DONE:
                    raise RuntimeError(f"request {rid} ended in state {st}: {qk.qk_last_error()}")
                if r["t"] >= warm:
                    sub.append(ts)
                    lat.append(td - ts)
                    queued.append(ta - ts)
                    entries += r["n_rows"] * 5000
                    t_first = ts if t_first is None else min(t_first, ts)
                    t_last = max(t_last, td)
            th.join()
            stats = qk.qk_server_stats(srv)
        finally:
            srv.close()
        lat, queued = np.array(lat) * 1e3, np.array(queued) * 1e3
        meas = [r for r in reqs if r["t"] >= warm]
        return {"rate_per_s": args.serve_rate, "measured_s": dur, "warmup_s": warm,
                "budget_mb": budget / 2**20, "n_requests": int(len(lat)),
                "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "mean_ms": float(lat.mean()),
                "admission_wait_p50_ms": float(np.percentile(queued, 50)),
                "admission_wait_p99_ms": float(np.percentile(queued, 99)),
                "entries_per_s": entries / (t_last - t_first),
                "offered_entries_per_s": sum(r["n_rows"] for r in meas) * 5000 / dur,
                "submit_span_s": float(max(sub) - min(sub)) if sub else 0.0,
                "n_iterations": stats["n_iters"],
                "peak_budget_mb": stats["peak_budget_bytes"] / 2**20}

    def closed_loop(inflight, dur):
        # `inflight` client threads, each with one request outstanding at a
        # time (submit, wait, fetch, repeat): the library's calls release the
        # interpreter lock while they wait or copy
        srv = make(1 << 30)
        lock = threading.Lock()
        tot = {"entries": 0, "lat": []}
        stop_at = time.perf_counter() + dur

        def client(c):
            crng = np.random.default_rng(1000 + c)
            out = np.empty((64, 5000))
            reqs = gen_requests(5700 + c, 1000.0, 60.0, dims=C5_DIMS)  # arrival times unused
            k = 0
            while time.perf_counter() < stop_at and k < len(reqs):
                r = reqs[k]
                k += 1
                off = int(crng.integers(0, pools[r["d"]].shape[0] - r["n_rows"]))
                rid = qk.qk_server_submit(srv, pools[r["d"]][off:off + r["n_rows"]], r["w"])
                st = qk.qk_server_wait(srv, rid, -1)
                ts, _, td = qk.qk_server_request_times(srv, rid)
                qk.qk_server_poll(srv, rid, out)
                if st != qk.QK_REQ_DONE:
                    raise RuntimeError(f"request {rid} ended in state {st}")
                with lock:
                    tot["entries"] += r["n_rows"] * 5000
                    tot["lat"].append(td - ts)

        try:
            t0 = time.perf_counter()
            ths = [threading.Thread(target=client, args=(c,)) for c in range(inflight)]
            for th in ths:
                th.start()
            for th in ths:
                th.join()
            wall = time.perf_counter() - t0
            stats = qk.qk_server_stats(srv)
        finally:
            srv.close()
        lat = np.array(tot["lat"]) * 1e3
        return {"inflight": inflight, "seconds": wall, "n_requests": int(len(lat)),
                "entries_per_s": tot["entries"] / wall, "p50_ms": float(np.percentile(lat, 50)),
                "p99_ms": float(np.percentile(lat, 99)), "n_iterations": stats["n_iters"]}

    res = {"workload": "requests of 1..64 rows, d in {16,64,256,784}, w ~ U[0,1], against "
                       "5000 resident support MPS per d, L=2, chi_max=64"}
    res["open_loop"] = open_loop(1 << 30, args.serve_warmup, args.serve_seconds)
    o = res["open_loop"]
    log(f"serve: open loop {o['n_requests']} requests, p50 {o['p50_ms']:.1f} ms, "
        f"p99 {o['p99_ms']:.1f} ms, {o['entries_per_s']:.3g} entries/s")
    # the largest request (d = 784, 64 rows) reserves about 48 MB: 96 MiB holds two
    res["budget_bound"] = open_loop(96 << 20, 2.0, args.serve_bound_seconds)
    o = res["budget_bound"]
    log(f"serve: 96 MiB budget p50 {o['p50_ms']:.1f} ms, p99 {o['p99_ms']:.1f} ms, "
        f"admission wait p99 {o['admission_wait_p99_ms']:.1f} ms, peak {o['peak_budget_mb']:.1f} MiB")
    res["saturation"] = closed_loop(args.serve_inflight, args.serve_sat_seconds)
    o = res["saturation"]
    log(f"serve: closed loop ({args.serve_inflight} in flight) {o['entries_per_s']:.3g} entries/s, "
        f"p50 {o['p50_ms']:.1f} ms")
    # headline figures of the open-loop run at the top level
    for key in ("p50_ms", "p99_ms", "entries_per_s", "n_requests", "rate_per_s", "measured_s",
                "warmup_s"):
        res[key] = res["open_loop"][key]
    return res


def ragged(args):
    """Ten feature dimensions d in {2, ..., 784}, 1000 cluster samples each,
    L = 2, chi_max = min(2^(d/2), 64), symmetric 1000 x 1000 per d: one
    multi-task call over all of them under AUTO (after the autotuner has
    tuned every (chi_pad, size) key), and each d alone. Every d resolves to
    the same form (the FP32 matrix-core form wherever bonds are <= 4), so the
    call is one persistent sweep launch plus its FP64 refinement pass. Per d:
    entries/s alone, and the largest |d ln K_q| of the AUTO result against
    the plain complex-FP64 sweep of the same MPS (whose parity with the
    oracle the test suite checks). MPS resident."""
    import numpy as np
    import torch

    import paper_2602_01330_amd.qk as qk
    from synthdata import config_inputs
    from synthdata.generators import C4_DIMS, chi_cap

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    batches, outs, tasks = {}, {}, []
    for d in C4_DIMS:
        x, _, _ = config_inputs("C4", d=d, n_train=1000, n_test=0)
        batches[d] = qk.qk_mps_build(torch.as_tensor(x, device=dev), 2, chi_cap("C4", d))
        outs[d] = torch.empty((1000, 1000), dtype=torch.float64, device=dev)
        tasks.append({"rows": batches[d], "cols": batches[d], "symmetric": True,
                      "lnkq": outs[d]})
    pairs = 1000 * 1001 // 2

    def timed(ts, reps=5):
        qk.qk_overlap_gram_multi(ts, "auto")
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            qk.qk_overlap_gram_multi(ts, "auto")
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    for t in tasks:  # tune every (chi_pad, n-bucket) key once
        qk.qk_autotune(t["rows"], t["cols"], True, max_tiles=256)
    forms = {str(d): qk.qk_resolve_precision(batches[d], batches[d]) for d in C4_DIMS}
    n_launch = len(set(forms.values()))  # AUTO runs one sweep launch per distinct form
    all_ms = timed(tasks)
    ln_auto = {d: outs[d].clone() for d in C4_DIMS}
    per_d = {}
    for d, t in zip(C4_DIMS, tasks):
        ms = timed([t])
        per_d[str(d)] = {"ms": ms, "entries_per_s": pairs / (ms / 1e3)}
    for d, t in zip(C4_DIMS, tasks):
        ref = torch.empty_like(outs[d])
        qk.qk_overlap_gram(t["rows"], t["cols"], True, "fp64", None, ref)
        torch.cuda.synchronize()
        a, r = ln_auto[d], ref
        both_inf = torch.isneginf(a) & torch.isneginf(r)
        diff = torch.where(both_inf, torch.zeros_like(a), (a - r).abs())
        iu = torch.triu_indices(1000, 1000, device=diff.device)
        du = diff[iu[0], iu[1]]
        per_d[str(d)]["max_abs_dlnk_vs_fp64"] = float(du.max())
        per_d[str(d)]["pairs_above_ln_gate_1e-3"] = int((du > 1e-3).sum())
    sum_alone = sum(v["ms"] for v in per_d.values())
    log(f"ragged: all ten d in {n_launch} sweep launch(es) {all_ms:.2f} ms, "
        f"sum of per-d launches {sum_alone:.2f} ms, worst |d lnK| vs FP64 "
        f"{max(v['max_abs_dlnk_vs_fp64'] for v in per_d.values()):.2e}")
    return {"workload": "d in {2,4,8,...,512,784}, 1000 samples each, symmetric, L=2, "
                        "chi_max=min(2^(d/2),64); MPS resident",
            "one_launch_ms": all_ms, "one_launch_entries_per_s": 10 * pairs / (all_ms / 1e3),
            "sweep_launches_per_call": n_launch,
            "sum_of_single_d_launches_ms": sum_alone,
            "one_launch_speedup_vs_sum": sum_alone / all_ms, "per_d": per_d,
            "sweep_form_per_d": forms, "tune_table": qk.qk_tune_export()}


def small_configs(args):
    """The two smaller configurations as whole jobs (device builds + one fused
    gram launch, inputs resident): 200 x 8 features at L = 1 (symmetric) and
    2000 + 500 x 64 features at L = 2 (train x train + test x train); the
    chosen form (AUTO) against the plain FP64 sweep."""
    import torch

    import paper_2602_01330_amd.qk as qk
    from synthdata import CONFIGS, config_inputs

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    out = {}
    for name in ("C1", "C2"):
        c = CONFIGS[name]
        x_tr, x_te, _ = config_inputs(name)
        xtr = torch.as_tensor(x_tr, device=dev)
        xte = torch.as_tensor(x_te, device=dev) if len(x_te) else None
        ntr, nte = len(x_tr), len(x_te)
        pairs = ntr * (ntr + 1) // 2 + nte * ntr
        f64 = dict(dtype=torch.float64, device=dev)
        ktr = {k: torch.empty((ntr, ntr), **f64) for k in ("kq", "kc", "k")}
        kte = {k: torch.empty((max(nte, 1), ntr), **f64) for k in ("kq", "kc", "k")}

        def step(prec, store):
            btr = qk.qk_mps_build(xtr, c.n_layers, c.chi_max, c.cutoff, store=store)
            tasks = [{"rows": btr, "cols": btr, "symmetric": True, "kq": ktr["kq"],
                      "fuse": {"x_rows": xtr, "x_cols": xtr, "gamma": 1.0 / c.d, "w": c.w,
                               "kc": ktr["kc"], "k": ktr["k"]}}]
            keep = [btr]
            if xte is not None:
                bte = qk.qk_mps_build(xte, c.n_layers, c.chi_max, c.cutoff, store=store)
                keep.append(bte)
                tasks.append({"rows": bte, "cols": btr, "symmetric": False, "kq": kte["kq"],
                              "fuse": {"x_rows": xte, "x_cols": xtr, "gamma": 1.0 / c.d,
                                       "w": c.w, "kc": kte["kc"], "k": kte["k"]}})
            qk.qk_overlap_gram_multi(tasks, prec)
            return keep

        res = {"workload": f"{ntr} train + {nte} test, d={c.d}, L={c.n_layers}, "
                           f"chi_max={c.chi_max}", "unique_pairs": pairs}
        # the autotuner picks AUTO's form for this size (tiny jobs favour the
        # single-launch FP64 sweep over a reduced form plus its refinement)
        tb = qk.qk_mps_build(xtr, c.n_layers, c.chi_max, c.cutoff, store=qk.QK_STORE_ALL)
        res["auto_form"] = qk.qk_autotune(tb, tb, True, max_tiles=256)
        tb.close()
        # AUTO builds only the tensors its chosen form reads (the reduced forms
        # also read the FP64 ones, for their refinement pass)
        auto_store = qk.QK_STORE_FP64 if res["auto_form"] == "fp64" else qk.QK_STORE_ALL
        for prec, store in (("auto", auto_store), ("fp64", qk.QK_STORE_FP64)):
            step(prec, store)
            torch.cuda.synchronize()
            reps = 5
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                keep = step(prec, store)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            del keep
            res[prec] = {"ms_per_job": ms, "entries_per_s": pairs / (ms / 1e3)}
        res["speedup_vs_plain_fp64"] = res["auto"]["entries_per_s"] / res["fp64"]["entries_per_s"]
        log(f"{name}: auto {res['auto']['ms_per_job']:.2f} ms, fp64 {res['fp64']['ms_per_job']:.2f} ms")
        out[name] = res
    return out


def chi64_sweep(args):
    """The sweep at the truncating regime's shape: 784 sites with every
    interior bond at 64 (bonds 1, 2, 4, ..., 64, ..., 4, 2, 1), on random
    left-canonical MPS (seeded; the device build of such deep circuits is not
    part of this leg), 32 row x 64 column samples = 2048 pairs, inputs
    resident. The complex-FP32 matrix-core sweep over all pairs (with its
    FP64 refinement of pairs above the threshold) and the complex-FP64 sweep
    over all pairs as its comparator."""
    import numpy as np
    import torch

    import paper_2602_01330_amd.qk as qk
    from synthdata import gen_isometry_mps

    nq, T, nr, nc = 784, 64, 32, 64
    log("bench: chi64 leg: generating random left-canonical MPS")
    cr, tr = gen_isometry_mps(nr, nq, T, seed=71)
    cc, tc = gen_isometry_mps(nc, nq, T, seed=72)
    br = qk.qk_mps_import(cr, tr, 8, T, store=qk.QK_STORE_ALL)
    bc = qk.qk_mps_import(cc, tc, 8, T, store=qk.QK_STORE_ALL)
    del tr, tc
    flop_pair = algorithmic_flops(cr[:1], cc[:1], False)
    pairs = nr * nc
    ln = torch.empty((nr, nc), dtype=torch.float64, device="cuda")

    def timed(form, reps):
        qk.qk_set_launch_timing(True)
        ms = []
        for _ in range(reps):
            qk.qk_overlap_gram(br, bc, False, form, None, ln)
            ms.append(qk.qk_last_launch_ms()[0])
        qk.qk_set_launch_timing(False)
        return float(np.median(ms))

    def entry(form, ms, peak, bound, kernel, traffic):
        tf = pairs * flop_pair / (ms / 1e3) / 1e12
        return {"form": form, "kernel": kernel, "kernel_ms": ms,
                "entries_per_s": pairs / (ms / 1e3),
                "roofline": {"bound": bound, "achieved": tf, "peak": peak, "unit": "TFLOP/s",
                             "frac": tf / peak, "traffic": traffic}}

    timed("fp64", 1)  # warmup
    ms64 = timed("fp64", 3)
    res = {"workload": f"{nq} sites, bonds up to {T} (chi_pad {T}), random left-canonical "
                       f"MPS, {nr} x {nc} pairs",
           "algorithmic_flop_per_pair": flop_pair,
           "fp64": entry("fp64", ms64, 78.6, "alu", "sweep_big_kernel<64>", None)}
    timed("fp32_mfma", 1)
    ms32 = timed("fp32_mfma", 3)
    refined = int((ln >= math.log(1e-2)).sum().item())
    res["fp32_mfma"] = entry("fp32_mfma", ms32, 157.3, "mfma",
                             f"sweep_wide_kernel<64> (+ FP64 list pass, {refined} refined)",
                             traffic_for("fp32_mfma_wide"))
    res["speedup_vs_plain_fp64"] = ms64 / ms32
    msg = f"fp64 {ms64:.1f} ms, fp32_mfma {ms32:.1f} ms"
    log(f"bench: chi64 leg ({pairs} pairs): {msg}")
    for b in (br, bc):
        b.close()
    return res


PATHSUM_FLOP_SITE = {1: 14 + 6 + 3 * 6, 2: 12 * 14 + 6 + 7 * 6,
                     3: 80 * 14 + 6 + (4 + 16 + 32) * 6}


def pathsum_flops(d, n_layers, pairs):
    """Algorithmic FLOP of the path-sum chain as written (an FMA counts 2):
    per bond, one butterfly per line and state pair (14 FLOP) and the shared
    line's phase (6); per site the weight's complex products (6 each; the
    first site's only). At L = 3: 80 butterflies, and the weight's q^3, r^3
    (4 products), the 16 products q^a conj(r)^b and one per state (32)."""
    per_site = PATHSUM_FLOP_SITE[n_layers]
    first = {1: 18, 2: 42, 3: (4 + 16 + 32) * 6}[n_layers]
    return float(pairs) * (per_site * (d - 1) + first)


def pathsum_leg(args):
    """The exact path-sum evaluator on the 784-qubit job (4000 train + 1000
    test images, L = 2, the same outputs as the MPS step: K_q, ln K_q, K_c,
    K with w = 0.5, gamma = 1/d), inputs resident; no build. With
    --pathsum-layers 3 the same job at three layers, timed beside the MPS
    route (device build, bonds 8, complex-FP64 sweep) on the same outputs."""
    import numpy as np
    import torch

    import paper_2602_01330_amd.qk as qk
    from synthdata import config_inputs

    x_tr, x_te, _ = config_inputs("C3")
    ntr, nte, d = x_tr.shape[0], x_te.shape[0], x_tr.shape[1]
    L = args.pathsum_layers
    cpu_rate, ns = cpu_baseline_pathsum(x_tr, L)
    xtr = torch.as_tensor(x_tr, device="cuda")
    xte = torch.as_tensor(x_te, device="cuda")
    f64 = dict(dtype=torch.float64, device="cuda")
    o_tr = {k: torch.empty((ntr, ntr), **f64) for k in ("kq", "ln", "kc", "k")}
    o_te = {k: torch.empty((nte, ntr), **f64) for k in ("kq", "ln", "kc", "k")}
    pairs = ntr * (ntr + 1) // 2 + nte * ntr

    def step():
        qk.qk_pathsum_gram(xtr, None, L, True, o_tr["kq"], o_tr["ln"],
                           {"gamma": 1.0 / d, "w": 0.5, "kc": o_tr["kc"], "k": o_tr["k"]})
        qk.qk_pathsum_gram(xte, xtr, L, True, o_te["kq"], o_te["ln"],
                           {"gamma": 1.0 / d, "w": 0.5, "kc": o_te["kc"], "k": o_te["k"]})

    step()
    torch.cuda.synchronize()
    steps = max(1, args.steps)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    ms = e0.elapsed_time(e1) / steps
    flops = pathsum_flops(d, L, pairs)
    tf = flops / (ms / 1e3) / 1e12
    log(f"bench: pathsum leg: {ms:.1f} ms/step ({pairs / (ms / 1e3):.3g} pairs/s, "
        f"{tf:.1f} TFLOP/s)")
    mps = None
    if L == 3:
        ln_ps = o_tr["ln"].clone()
        e0.record()
        btr, bte = qk.qk_mps_build_many([xtr, xte], 3, 64, 1e-10, store=qk.QK_STORE_FP64)
        tasks = [{"rows": btr, "cols": btr, "symmetric": True, "kq": o_tr["kq"],
                  "lnkq": o_tr["ln"], "fuse": {"x_rows": xtr, "x_cols": xtr, "gamma": 1.0 / d,
                                               "w": 0.5, "kc": o_tr["kc"], "k": o_tr["k"]}},
                 {"rows": bte, "cols": btr, "symmetric": False, "kq": o_te["kq"],
                  "lnkq": o_te["ln"], "fuse": {"x_rows": xte, "x_cols": xtr, "gamma": 1.0 / d,
                                               "w": 0.5, "kc": o_te["kc"], "k": o_te["k"]}}]
        qk.qk_overlap_gram_multi(tasks, "fp64")
        e1.record()
        torch.cuda.synchronize()
        mps_ms = e0.elapsed_time(e1)
        dln = float((o_tr["ln"] - ln_ps).abs().max())
        mps = {"ms_per_step": mps_ms, "pairs_per_s": pairs / (mps_ms / 1e3),
               "chi_pad": qk.qk_mps_info(btr)["chi_pad"], "max_abs_dlnk_vs_pathsum": dln,
               "pathsum_speedup": mps_ms / ms}
        log(f"bench: MPS route at L=3 (FP64, bonds 8): {mps_ms:.1f} ms, |d lnK| {dln:.1e}")
        btr.close()
        bte.close()
    return {"workload": f"784-qubit images, 4000 train + 1000 test, L={L}, exact path-sum "
                        "(no MPS build), fused RBF (gamma=1/d) + mix w=0.5",
            "mps_route_fp64": mps,
            "ms_per_step": ms, "wall_ms_per_step": wall, "steps": steps,
            "pairs_per_s": pairs / (ms / 1e3), "algorithmic_flop": flops,
            "roofline": {"bound": "alu", "achieved": tf, "peak": 78.6, "unit": "TFLOP/s",
                         "frac": tf / 78.6,
                         "traffic": traffic_for("pathsum_l2_step") if L == 2 else None,
                         "note": "step time includes the two table kernels and the epilogue"},
            "cpu_oracle": {"pairs_per_s": cpu_rate, "cores": 1, "kind": "oracle",
                           "sample": f"{ns} random train pairs at d=784, L={L} (oracle.pathsum)"}}


def s1_leg(args):
    """The truncating regime end to end: 1000 train + 250 test images (784
    qubits), 8 layers, chi_max 64 (bonds would reach 2^8 without the cap).
    Device build in launches of 250 samples (FP64 tensors and their packed
    FP32 copies), then the sweep of train x train (symmetric) and test x
    train in three calls of about 250k pairs (progress between calls), once
    with the chosen form (complex FP32 on the matrix cores, pairs above the
    refinement threshold redone in FP64) and once with the plain complex-FP64
    sweep; the two are compared on every pair. The first three train
    samples' bond tables, discarded weights and overlaps are checked against
    the oracle's replay (tests/golden/s1_replay_3.json)."""
    import numpy as np
    import torch

    import paper_2602_01330_amd.qk as qk
    from synthdata import config_inputs

    x_tr, x_te, _ = config_inputs("S1")
    ntr, nte, d = x_tr.shape[0], x_te.shape[0], x_tr.shape[1]
    L, chi, B = 8, 64, 250
    xs = [torch.as_tensor(x_tr[k:k + B], device="cuda") for k in range(0, ntr, B)]
    xs.append(torch.as_tensor(x_te, device="cuda"))
    forms = ["fp64"] if args.s1_plain_only else ["fp32_mfma", "fp64"]
    store = qk.QK_STORE_FP64 if args.s1_plain_only else qk.QK_STORE_ALL
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bs = []
    for k, xk in enumerate(xs):
        bs.append(qk.qk_mps_build(xk, L, chi, 1e-10, store=store))
        torch.cuda.synchronize()
        log(f"bench: s1 build {k + 1}/{len(xs)} done at {time.perf_counter() - t0:.1f} s")
    build_s = time.perf_counter() - t0
    tr, te = bs[:-1], bs[-1]
    f64 = dict(dtype=torch.float64, device="cuda")
    chi_tr = np.concatenate([qk.qk_mps_chi(b) for b in tr])
    chi_te = qk.qk_mps_chi(te)
    flops = algorithmic_flops(chi_tr, chi_tr, True) + algorithmic_flops(chi_te, chi_tr, False)
    pairs = ntr * (ntr + 1) // 2 + nte * ntr
    fx = json.load(open(os.path.join(ROOT, "tests", "golden", "s1_replay_3.json")))
    upper = np.triu_indices(ntr)

    def sweep(prec):
        ln_tr = torch.full((ntr, ntr), float("nan"), **f64)
        ln_te = torch.full((nte, ntr), float("nan"), **f64)
        calls = [[(0, 0), (0, 1), (0, 2), (0, 3), (1, 1)],
                 [(1, 2), (1, 3), (2, 2), (2, 3), (3, 3)]]
        t1 = time.perf_counter()
        for n_call, blocks in enumerate(calls):
            tasks = [{"rows": tr[a], "cols": tr[b], "symmetric": a == b, "kq": None,
                      "lnkq": ln_tr[a * B:(a + 1) * B, b * B:(b + 1) * B]} for a, b in blocks]
            qk.qk_overlap_gram_multi(tasks, prec)
            torch.cuda.synchronize()
            log(f"bench: s1 {prec} train sweep {n_call + 1}/2 done at "
                f"{time.perf_counter() - t1:.1f} s")
        tasks = [{"rows": te, "cols": tr[b], "symmetric": False, "kq": None,
                  "lnkq": ln_te[:, b * B:(b + 1) * B]} for b in range(len(tr))]
        qk.qk_overlap_gram_multi(tasks, prec)
        torch.cuda.synchronize()
        sweep_s = time.perf_counter() - t1
        log(f"bench: s1 {prec} test sweep done, sweep {sweep_s:.1f} s")
        ln_all = ln_tr.cpu().numpy()
        lmax = float(np.max(np.abs(ln_all[:3, :3] - np.array(fx["lnkq"]))))
        return ln_tr, ln_te, {
            "sweep_s": sweep_s, "job_s": build_s + sweep_s,
            "pairs_per_s": pairs / (build_s + sweep_s), "sweep_pairs_per_s": pairs / sweep_s,
            "sweep_tflops": flops / sweep_s / 1e12,
            "replay_max_abs_dlnk": lmax, "replay_ln_gate_b": bool(lmax <= 1e-3),
            "diag_max_abs_lnk": float(np.max(np.abs(np.diag(ln_all)))),
            "upper_all_finite": bool(np.isfinite(ln_all[upper]).all())}

    res = {"workload": "truncating regime: 1000 train + 250 test 784-qubit images, L=8, "
                       "chi_max=64, device build (FP64) + sweep, inputs resident",
           "build_s": build_s, "pairs": pairs, "algorithmic_flop": flops,
           "chi_realized_max": int(chi_tr.max())}
    lns = {}
    for prec in forms:
        ln_tr, ln_te, r = sweep(prec)
        res[prec] = r
        lns[prec] = (ln_tr, ln_te)
    if len(forms) == 2:
        a, b = lns["fp32_mfma"], lns["fp64"]
        iu = torch.triu_indices(ntr, ntr, device=a[0].device)
        dd = torch.cat([(a[0][iu[0], iu[1]] - b[0][iu[0], iu[1]]).abs(),
                        (a[1] - b[1]).abs().flatten()])
        res["chosen_vs_plain_all_pairs"] = {
            "max_abs_dlnk": float(dd.max()), "pairs_above_ln_gate_1e-3": int((dd > 1e-3).sum())}
        res["speedup_job"] = res["fp64"]["job_s"] / res["fp32_mfma"]["job_s"]
        res["speedup_sweep"] = res["fp64"]["sweep_s"] / res["fp32_mfma"]["sweep_s"]
    res["replay_check"] = {
        "bond_tables_equal": bool(np.array_equal(chi_tr[:3], np.array(fx["chi"], dtype=np.int32))),
        "discarded_equal": bool(np.allclose(qk.qk_mps_discarded(tr[0])[:3], fx["discarded"],
                                            rtol=1e-6, atol=1e-15))}
    for b in bs:
        b.close()
    return res


def svm_leg(args):
    """SVM training and prediction (Eqs. (1)-(2), (4)-(5), one-against-one)
    on the dual kernel of the 784-feature workload: 4000 train + 1000 test
    images, 10 classes, L = 2, w = 0.5, gamma = 1/d. The Gram matrices come
    from the library (untimed here); timed: the one-launch training of the 45
    problems (C = 10, eps = 1e-3) and the prediction of the 1000 test rows.
    The oracle solves the same 45 problems on the same kernel matrix (copied
    to the host) for the step counts and the CPU time."""
    import numpy as np
    import torch

    import paper_2602_01330_amd.qk as qk
    from synthdata import config_inputs

    x_tr, x_te, lab = config_inputs("C3")
    ntr, nte, d = x_tr.shape[0], x_te.shape[0], x_tr.shape[1]
    y_tr, y_te = lab[:ntr], lab[ntr:]
    xtr = torch.as_tensor(x_tr, device="cuda")
    xte = torch.as_tensor(x_te, device="cuda")
    f64 = dict(dtype=torch.float64, device="cuda")
    k_tr = torch.empty((ntr, ntr), **f64)
    k_te = torch.empty((nte, ntr), **f64)
    btr, bte = qk.qk_mps_build_many([xtr, xte], 2, 64, 1e-10)
    tasks = [{"rows": btr, "cols": btr, "symmetric": True, "kq": None, "lnkq": None,
              "fuse": {"x_rows": xtr, "x_cols": xtr, "gamma": 1.0 / d, "w": 0.5, "k": k_tr}},
             {"rows": bte, "cols": btr, "symmetric": False, "kq": None, "lnkq": None,
              "fuse": {"x_rows": xte, "x_cols": xtr, "gamma": 1.0 / d, "w": 0.5, "k": k_te}}]
    qk.qk_overlap_gram_multi(tasks, "auto")
    torch.cuda.synchronize()
    C_box, eps = 10.0, 1e-3
    qk.qk_svm_fit_ovo(k_tr, y_tr, 10, C_box, eps)  # warmup
    torch.cuda.synchronize()
    fit_ms, pred_ms = [], []
    for _ in range(3):
        t0 = time.perf_counter()
        coef, b, it = qk.qk_svm_fit_ovo(k_tr, y_tr, 10, C_box, eps)
        torch.cuda.synchronize()
        fit_ms.append((time.perf_counter() - t0) * 1e3)
        t0 = time.perf_counter()
        f, pred = qk.qk_svm_predict_ovo(k_te, coef, b, 10)
        torch.cuda.synchronize()
        pred_ms.append((time.perf_counter() - t0) * 1e3)
    it = it.cpu().numpy()
    acc = float((pred.cpu().numpy() == y_te).mean())
    it_ref, cpu_s = cpu_baseline_svm(k_tr.cpu().numpy(), y_tr, 10, C_box, eps)
    log(f"bench: svm leg: fit {np.median(fit_ms):.1f} ms ({int(it.sum())} SMO steps), "
        f"predict {np.median(pred_ms):.2f} ms, oracle fit {cpu_s:.1f} s")
    for bb in (btr, bte):
        bb.close()
    return {"workload": "one-against-one SVMs (45 problems of 800 samples) on the dual kernel "
                        "of 4000 train + 1000 test 784-feature images, C=10, eps=1e-3",
            "fit_ms": float(np.median(fit_ms)), "predict_ms": float(np.median(pred_ms)),
            "smo_steps_total": int(it.sum()), "smo_steps_max": int(it.max()),
            "steps_equal_oracle": bool(np.array_equal(it, it_ref)),
            "test_accuracy_synthetic_labels": acc,
            "cpu_oracle_fit_s": cpu_s, "cpu_oracle_cores": 1}


def all_pairs_gap(chosen, out, out_te, ntr):
    """Largest differences of the chosen form's outputs from the plain FP64
    sweep's over every unique pair of the job (train upper triangle with the
    diagonal, and test x train): |d ln K_q| (and how many pairs exceed the
    stated log gate 1e-3), |d K_q| and |d K| (the stated absolute gate 1e-5)."""
    import torch
    iu = torch.triu_indices(ntr, ntr, device=out["ln"].device)
    res = {}
    for key in ("ln", "kq", "k"):
        a_tr, a_te = chosen[key]
        d_tr = (a_tr[iu[0], iu[1]] - out[key][iu[0], iu[1]]).abs()
        d_te = (a_te - out_te[key]).abs().flatten()
        if key == "ln":  # both -inf (an exactly zero amplitude) count as equal
            z_tr = torch.isneginf(a_tr[iu[0], iu[1]]) & torch.isneginf(out[key][iu[0], iu[1]])
            z_te = (torch.isneginf(a_te) & torch.isneginf(out_te[key])).flatten()
            d_tr = torch.where(z_tr, torch.zeros_like(d_tr), d_tr)
            d_te = torch.where(z_te, torch.zeros_like(d_te), d_te)
        d = torch.cat([d_tr, d_te])
        res[f"max_abs_d{key}"] = float(d.max())
        if key == "ln":
            res["pairs_above_ln_gate_1e-3"] = int((d > 1e-3).sum())
            res["pairs_above_ln_1e-4"] = int((d > 1e-4).sum())
    return res


def run(args):
    import numpy as np

    from synthdata import config_inputs

    log("bench: generating inputs")
    x_tr, x_te, _ = config_inputs("C3")
    cpu = None
    if not args.no_cpu:
        # first, while nothing has touched the GPU: the oracle's worker
        # processes are forked from a process that holds no GPU state
        log("bench: timing the CPU oracle sample")
        cpu = cpu_baseline(x_tr, args.cpu_seconds)

    import torch

    import paper_2602_01330_amd.qk as qk

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    d = x_tr.shape[1]
    xtr = torch.as_tensor(x_tr, device=dev)
    xte = torch.as_tensor(x_te, device=dev)
    ntr, nte = xtr.shape[0], xte.shape[0]
    pairs = ntr * (ntr + 1) // 2 + nte * ntr
    f64 = dict(dtype=torch.float64, device=dev)
    out = {k: torch.empty((ntr, ntr), **f64) for k in ("kq", "ln", "kc", "k")}
    out_te = {k: torch.empty((nte, ntr), **f64) for k in ("kq", "ln", "kc", "k")}
    stream = torch.cuda.current_stream()


    def one_step(prec, timing=None):
        store = qk.QK_STORE_FP64 if prec == "fp64" else qk.QK_STORE_ALL
        # both builds in one launch (as two launches on two streams, the
        # second one ran a third slower than alone)
        btr, bte = qk.qk_mps_build_many([xtr, xte], 2, 64, 1e-10, store=store)
        tasks = [
            {"rows": btr, "cols": btr, "symmetric": True, "kq": out["kq"], "lnkq": out["ln"],
             "fuse": {"x_rows": xtr, "x_cols": xtr, "gamma": 1.0 / d, "w": 0.5,
                      "kc": out["kc"], "k": out["k"]}},
            {"rows": bte, "cols": btr, "symmetric": False, "kq": out_te["kq"],
             "lnkq": out_te["ln"],
             "fuse": {"x_rows": xte, "x_cols": xtr, "gamma": 1.0 / d, "w": 0.5,
                      "kc": out_te["kc"], "k": out_te["k"]}},
        ]
        if timing is not None:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
        qk.qk_overlap_gram_multi(tasks, prec)
        if timing is not None:
            e1.record(stream)
            timing.append((e0, e1))
        return btr, bte

    def measure(prec, steps, warmup):
        for w in range(warmup):
            b = one_step(prec)
            torch.cuda.synchronize()
            del b
            log(f"bench: {prec} warmup {w + 1}/{warmup} done")
        timing = []
        keep = []
        qk.qk_set_launch_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(steps):
            # Batches stay alive until the loop ends (3.5 GB per step): a
            # release drains the device, which would idle it between steps
            # while the host enqueues the next one; long runs release every
            # 16 steps.
            if len(keep) == 16:
                keep.clear()
            keep.append(one_step(prec, timing))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        # the library's own HIP events around the last step's sweep launch
        # and FP64 refinement pass (read after the loop: the query waits)
        kernel_last, refine_last = qk.qk_last_launch_ms()
        qk.qk_set_launch_timing(False)
        sweep_ms = [t[0].elapsed_time(t[1]) for t in timing]
        kernel_ms = [kernel_last]
        refine_ms = [refine_last]
        btr, bte = keep[-1]
        chi_tr = qk.qk_mps_chi(btr)
        chi_te = qk.qk_mps_chi(bte)
        info = qk.qk_mps_info(btr)
        flops = (algorithmic_flops(chi_tr, chi_tr, True)
                 + algorithmic_flops(chi_te, chi_tr, False))
        ms = (t1 - t0) * 1e3 / steps
        log(f"bench: {prec}: {ms:.1f} ms/step, gram call {np.mean(sweep_ms):.1f} ms "
            f"(sweep kernel {np.mean(kernel_ms):.1f} ms, FP64 refinement {np.mean(refine_ms):.1f} ms)")
        return {"ms_per_step": ms, "sweep_ms": float(np.mean(sweep_ms)),
                "kernel_ms": float(np.mean(kernel_ms)), "refine_ms": float(np.mean(refine_ms)),
                "flops": flops,
                "chi_max_realized": info["chi_realized_max"], "chi_pad": info["chi_pad"]}

    chosen = args.prec
    tune = None
    if args.tune_table:
        # a fixed tuning table (';' between entries) instead of the
        # autotuner's run: profiles repeat one launch shape exactly
        qk.qk_tune_import(args.tune_table.replace(";", "\n") + "\n")
        tune = qk.qk_tune_export()
        log(f"bench: tuning table imported: {tune.strip()}")
    if chosen == "auto" and not args.tune_table:
        # the project autotuner times the eligible forms on a slice of the
        # train x train tiles; AUTO then resolves to the winner
        b = qk.qk_mps_build(xtr, 2, 64, 1e-10, store=qk.QK_STORE_ALL)
        chosen = qk.qk_autotune(b, b, True, max_tiles=2048)
        tune = qk.qk_tune_export()
        b.close()
        log(f"bench: autotune chose {chosen}")
    if chosen == "auto":
        b = qk.qk_mps_build(xtr, 2, 64, 1e-10, store=qk.QK_STORE_ALL)
        chosen = qk.qk_resolve_precision(b, b)
        b.close()
    res = measure(chosen, args.steps, args.warmup)
    shape = launch_shape(qk.qk_tune_export(), res["chi_pad"], d, qk.PREC[chosen])
    value = pairs / (res["ms_per_step"] / 1e3)
    bound, peak = PEAKS[chosen]
    achieved = res["flops"] / (res["kernel_ms"] / 1e3) / 1e12
    line = {
        "metric": "Gram kernel entries/sec at 784 qubits chi_max=64 (chosen vs plain FP64)",
        "value": value, "unit": "entries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": res["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[chosen],
        "data": "synthetic (seeded 28x28 smooth-field images, 10 classes)",
        "config": {"workload": "784-qubit images, 4000 train + 1000 test, L=2, chi_max=64, "
                               "cutoff 1e-10, fused RBF (gamma=1/d) + mix w=0.5",
                   "n_train": ntr, "n_test": nte, "d": d, "n_layers": 2, "chi_max": 64,
                   "chi_realized_max": res["chi_max_realized"], "chi_pad": res["chi_pad"],
                   "unique_pairs": pairs, "sweep_form": chosen, "autotune_table": tune},
        "roofline": {"bound": bound, "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": traffic_for(chosen, shape),
                     "launch_shape": {"wg_per_cu": shape[0], "band": shape[1]},
                     "kernel": "sweep (one persistent launch per step)",
                     "kernel_ms": res["kernel_ms"], "algorithmic_flop": res["flops"],
                     "gram_call_ms": res["sweep_ms"], "fp64_refine_ms": res["refine_ms"]},
    }
    if not args.no_plain and chosen != "fp64":
        keep = {k: (out[k].clone(), out_te[k].clone()) for k in ("kq", "ln", "k")}
        p = measure("fp64", max(1, args.steps // 2), 1)
        line["plain_fp64"] = {"value": pairs / (p["ms_per_step"] / 1e3),
                              "ms_per_step": p["ms_per_step"], "sweep_ms": p["sweep_ms"]}
        line["speedup_vs_plain_fp64"] = value / line["plain_fp64"]["value"]
        line["chosen_vs_plain_fp64_all_pairs"] = all_pairs_gap(keep, out, out_te, ntr)
        log(f"bench: chosen vs plain FP64 on all {pairs} pairs: "
            f"{line['chosen_vs_plain_fp64_all_pairs']}")
    def leg(key, fn):
        # an optional leg that raises is recorded as such; the line still prints
        try:
            line[key] = fn(args)
        except Exception as exc:  # noqa: BLE001
            log(f"bench: {key} failed: {exc!r}")
            line[key] = {"error": repr(exc)}

    if args.chi64:
        leg("chi64_sweep", chi64_sweep)
    if not args.no_ragged:
        log("bench: ragged multi-d run")
        leg("ragged", ragged)
    if not args.no_small:
        log("bench: smaller configurations")
        leg("small_configs", small_configs)
    if args.serve_seconds > 0:
        log("bench: serving run")
        leg("serving", serving)
    if args.svm:
        leg("svm", svm_leg)
    if args.pathsum:
        leg("pathsum", pathsum_leg)
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


def hbm_copy():
    """A plain device-to-device copy of exactly 1 GiB, twice: the known byte
    count that scales the FETCH_SIZE / WRITE_SIZE counters of a profiled run
    to HBM bytes."""
    import torch
    n_bytes = 1 << 30
    a = torch.ones(n_bytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
        torch.cuda.synchronize()
    print(json.dumps({"hbm_copy_bytes": n_bytes, "copies": 2}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--prec", default="auto",
                    choices=["auto", "fp64", "fp32", "fp32_mfma", "bf16x2", "bf16x3"])
    ap.add_argument("--tune-table", default=None,
                    help="import this tuning table ('T bucket form wg band us' entries "
                         "separated by ';') instead of running the autotuner")
    ap.add_argument("--no-plain", action="store_true", help="skip the FP64 comparator")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-ragged", action="store_true", help="skip the ten-d ragged run")
    ap.add_argument("--chi64", action="store_true",
                    help="add the 784-site bond-64 sweep leg (FP32 matrix-core form and "
                         "the FP64 comparator)")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the two smaller whole-job configurations")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="measured seconds of the open-loop serving run (0 skips serving)")
    ap.add_argument("--serve-warmup", type=float, default=5.0)
    ap.add_argument("--serve-bound-seconds", type=float, default=15.0,
                    help="measured seconds of the budget-bound serving run")
    ap.add_argument("--serve-sat-seconds", type=float, default=10.0,
                    help="seconds of the closed-loop (saturation) serving run")
    ap.add_argument("--serve-inflight", type=int, default=32,
                    help="requests outstanding in the closed-loop run")
    ap.add_argument("--serve-rate", type=float, default=200.0, help="requests per second")
    ap.add_argument("--pathsum", action="store_true",
                    help="add the exact path-sum leg on the 784-qubit job")
    ap.add_argument("--pathsum-layers", type=int, default=2, choices=[1, 2, 3],
                    help="circuit layers of the path-sum leg (3 also times the MPS route)")
    ap.add_argument("--pathsum-only", action="store_true",
                    help="run only the path-sum leg and print its JSON")
    ap.add_argument("--s1-only", action="store_true",
                    help="run only the truncating-regime job end to end and print its JSON")
    ap.add_argument("--s1-plain-only", action="store_true",
                    help="truncating-regime leg: only the plain FP64 sweep")
    ap.add_argument("--svm", action="store_true",
                    help="add the SVM training / prediction leg on the 784-feature Gram")
    ap.add_argument("--svm-only", action="store_true",
                    help="run only the SVM leg and print its JSON")
    ap.add_argument("--hbm-copy", action="store_true",
                    help="only copy 1 GiB device to device twice (calibrates the HBM byte "
                         "counters FETCH_SIZE / WRITE_SIZE under rocprofv3)")
    ap.add_argument("--chi64-only", action="store_true",
                    help="run only the 784-site bond-64 sweep leg and print its JSON")
    args = ap.parse_args()
    if args.hbm_copy:
        hbm_copy()
        return
    if args.chi64_only:
        print(json.dumps(chi64_sweep(args)), flush=True)
        return
    if args.s1_only:
        print(json.dumps(s1_leg(args)), flush=True)
        return
    if args.pathsum_only:
        print(json.dumps(pathsum_leg(args)), flush=True)
        return
    if args.svm_only:
        print(json.dumps(svm_leg(args)), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the Gram tiles shard across GPUs without "
              "communication in the sweep, but multi-GPU execution is not implemented; "
              "use --gpus 1.", file=sys.stderr)
        sys.exit(2)
    run(args)


if __name__ == "__main__":
    main()
