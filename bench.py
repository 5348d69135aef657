"""Benchmark: p-bit multiply-accumulates per second of the real matrix
product C = A B with N = 2048, p = 512 (512-bit mantissas, exponents
uniform in [-4, 4], exact inputs), on the scaled-integer INT8-MFMA path,
next to the plain limb-window kernel on the same GPU and the exact CPU
oracle on the host cores.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3]

Prints one JSON line.  A step is one arbgpu_mat_mul call (statistics,
slicing, MFMA product, recombination and rounding) with the operands
already resident in device memory.

Two more workloads are measured and reported beside the headline number:
  dot_batch  10^4 complex ball dot products (lengths log-uniform in
             [4, 4096], p log-uniform in [64, 1024], operand precisions in
             [p/2, 2p]) as one resident graph launch after autotuning;
  serving    a Poisson stream (200 requests/s) of complex ball matrix
             products, N log-uniform in [16, 1024], p in {128, ..., 2048},
             over device-resident operands through arbgpu_submit/poll:
             p50/p99 latency from arrival to completion and throughput.
"""

from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1901_04289_amd import gen  # noqa: E402

METRIC = "p-bit MACs/s, sliced-MFMA vs plain limb kernel, N=2048 p=512; p99 latency"
PEAK_INT8_TOPS = 5000.0   # MI355X dense INT8 MFMA, 5.0 POP/s
# 32 x 32 -> 64-bit integer products (v_mad_u64_u32, one per lane per clock
# at the full vector rate): 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
PEAK_LIMB_PRODUCTS = 256 * 4 * 16 * 2.4e9
PEAK_HBM_GBS = 8000.0     # MI355X HBM3E, 8 TB/s

# HBM bytes per launch of the MFMA kernel of each INT8 form at N = 2048,
# p = 512, from FETCH_SIZE (scaled by the copy calibration) and WRITE_SIZE
# counter runs (profiles/mfma_*_matmul2048_p512.txt); each is valid only for
# the kernel source it was taken on (sha256 prefix of that file), else the
# traffic is reported as null.
MFMA_KERNEL = {"residues": "mfma_rns_kernel<256>", "slices": "mfma_diag_kernel"}
MFMA_TRAFFIC = {
    # form: (kernel source, sha256 prefix, bytes per launch)
    "residues": ("mfma_rns.hip", "f01cea3055db3e34", (1777060 * 2 + 645248) * 1024.0),
    # the stored base-256 figure covered the full pair set (before the
    # truncated diagonals): only live counters report that form
    "slices": ("mfma.hip", None, None),
}


def _stored_traffic(n, form):
    import hashlib
    src, want, nbytes = MFMA_TRAFFIC[form]
    with open(os.path.join(ROOT, "paper_1901_04289_amd", "csrc", src), "rb") as f:
        h = hashlib.sha256(f.read()).hexdigest()[:16]
    return nbytes if (want is not None and h == want and n == 2048) else None


# Kernels whose HBM traffic the counter runs report (name as rocprofv3
# prints it, up to the template arguments or the parameter list).
COUNTED_KERNELS = ("mfma_rns_kernel", "mfma_diag_kernel", "rns_slice_kernel", "rns_crt_kernel",
                   "gather_lines_kernel", "slice_kernel", "recombine_kernel")
COPY_KERNEL = "__amd_rocclr_copyBuffer"
CALIBRATION_BYTES = 1 << 30


def traffic_child(n):
    """Body of a counter run: one automatic product at the benchmark size
    and one on base-256 slices, then a 1 GiB device-to-device copy whose
    known byte counts calibrate the counters."""
    import torch
    from paper_1901_04289_amd import arbgpu
    w = gen.config2(n=n)
    ctx = arbgpu.Context(0)
    dA, dB = arbgpu.DeviceArray.from_host(w.A), arbgpu.DeviceArray.from_host(w.B)
    C = arbgpu.DeviceOut.empty(w.M * w.K, w.p, radius=True)
    ctx.mat_mul(C, dA, dB, w.M, w.N, w.K, w.p, 0)
    ctx.mat_mul(C, dA, dB, w.M, w.N, w.K, w.p, arbgpu.ALGO_SLICED)
    torch.cuda.synchronize()
    src = torch.empty(CALIBRATION_BYTES, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    ctx.close()


def _counter_values(csv_path):
    """Per kernel (short name): the counter value of each dispatch, in KiB."""
    import csv
    out = {}
    with open(csv_path, newline="") as f:
        for row in csv.DictReader(f):
            name = row["Kernel_Name"]
            for short in COUNTED_KERNELS + (COPY_KERNEL,):
                if (short + "<") in name or (short + "(") in name or name == short:
                    out.setdefault(short, []).append(float(row["Counter_Value"]))
                    break
    return out


def hbm_counters(n, log):
    """HBM bytes per dispatch of the path's kernels from two rocprofv3
    counter runs of this script (FETCH_SIZE, then WRITE_SIZE), each scaled
    by what the same counter reads for the 1 GiB copy.  None when the
    profiler is missing or a run gives no usable result."""
    import glob
    import shutil
    import subprocess
    import tempfile
    prof = shutil.which("rocprofv3") or "/opt/rocm/bin/rocprofv3"
    if not os.path.exists(prof):
        log("[bench] rocprofv3 not found: traffic from the stored counter runs")
        return None
    tmp = tempfile.mkdtemp(prefix="arbgpu_pmc_", dir="/tmp")
    vals = {}
    for counter in ("FETCH_SIZE", "WRITE_SIZE"):
        d = os.path.join(tmp, counter)
        cmd = ["timeout", "-s", "KILL", "180", prof, "--pmc", counter, "--output-format", "csv", "-d", d,
               "-o", "run", "--", sys.executable, os.path.abspath(__file__), "--traffic-child", "--n", str(n)]
        t0 = time.time()
        r = subprocess.run(cmd, cwd="/tmp", env=dict(os.environ, TMPDIR="/tmp"), stdout=subprocess.DEVNULL,
                           stderr=subprocess.PIPE, text=True)
        csvs = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        got = _counter_values(csvs[0]) if csvs else {}
        log(f"[bench] counter run {counter}: exit {r.returncode}, {time.time() - t0:.1f}s, "
            f"kernels {sorted(got)}")
        if COPY_KERNEL not in got or not any(k in got for k in COUNTED_KERNELS):
            log("[bench] counter run unusable: " + (r.stderr or "")[-500:])
            return None
        vals[counter] = got
    f_read = CALIBRATION_BYTES / (max(vals["FETCH_SIZE"][COPY_KERNEL]) * 1024.0)
    f_write = CALIBRATION_BYTES / (max(vals["WRITE_SIZE"][COPY_KERNEL]) * 1024.0)
    per = {}
    for k in COUNTED_KERNELS:
        if k in vals["FETCH_SIZE"] and k in vals["WRITE_SIZE"]:
            rd = np.mean(vals["FETCH_SIZE"][k]) * 1024.0 * f_read
            wr = np.mean(vals["WRITE_SIZE"][k]) * 1024.0 * f_write
            per[k] = {"read_bytes": rd, "write_bytes": wr, "bytes": rd + wr,
                      "dispatches": len(vals["FETCH_SIZE"][k])}
    return {"per_dispatch": per, "fetch_scale": f_read, "write_scale": f_write,
            "source": "rocprofv3 --pmc FETCH_SIZE and --pmc WRITE_SIZE runs of bench.py --traffic-child "
                      f"(the automatic and the base-256 product at N={n}; counters scaled by a 1 GiB device copy)"}


# ---------------------------------------------------------------------------
# CPU baseline: the exact oracle on a bounded sample of output entries
# ---------------------------------------------------------------------------

_ROWS = None
_COLS = None


def _init_worker(rows, cols):
    global _ROWS, _COLS
    _ROWS, _COLS = rows, cols


def _oracle_entries(args):
    import oracle
    pairs, p, deadline = args
    done = 0
    t = 0.0
    while time.time() < deadline:
        for (i, j) in pairs:
            if time.time() >= deadline:
                break
            t0 = time.perf_counter()
            oracle.dot(_ROWS[i], _COLS[j], p)
            t += time.perf_counter() - t0
            done += 1
    return done, t


def host_cpu():
    """CPU model name (from /proc/cpuinfo), logical CPUs of the host, and
    the CPUs this process may run on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "host_logical_cpus": os.cpu_count(),
            "affinity_cpus": len(os.sched_getaffinity(0))}


def cpu_baseline(w, seconds: float, cores: int):
    """Exact oracle on random output entries: 32 rows and 32 columns are
    decoded up front (not timed); each worker repeatedly evaluates its
    share of the 1024 (row, column) dot products until the deadline."""
    rng = np.random.default_rng(7)
    ri = rng.choice(w.M, 32, replace=False)
    cj = rng.choice(w.K, 32, replace=False)
    rows = [[gen.to_canonical(w.A, int(i) * w.N + k) for k in range(w.N)] for i in ri]
    cols = [[gen.to_canonical(w.B, k * w.K + int(j)) for k in range(w.N)] for j in cj]
    pairs = [(a, b) for a in range(32) for b in range(32)]
    chunks = [pairs[c::cores] for c in range(cores)]
    ctx = mp.get_context("fork")
    pool = ctx.Pool(cores, initializer=_init_worker, initargs=(rows, cols))
    try:
        t0 = time.time()
        res = pool.map(_oracle_entries, [(ch, w.p, time.time() + seconds) for ch in chunks])
        dt = time.time() - t0
    finally:
        pool.close()
        pool.join()
    n = sum(r[0] for r in res)
    host = host_cpu()
    out = {"value": n * w.N / dt, "unit": "p-bit MACs/s", "cores": cores, "kind": "oracle",
           "sample": f"{n} dot products of length {w.N} (entries of the 2048^3 p=512 product from 32 "
                     f"random rows x 32 random columns, {n * w.N} MACs), exact oracle, {cores} worker "
                     f"processes (the CPU share of one GPU, at most 16), {dt:.1f} s wall"}
    out.update(host)
    return out


# ---------------------------------------------------------------------------
# GPU
# ---------------------------------------------------------------------------

def window_limbs(p, terms):
    """Limbs of the accumulation window of a dot product: p bits, the
    extend bits for `terms` terms and the guard bits (Section 3.3)."""
    bc = np.floor(np.log2(np.asarray(terms, dtype=np.float64) + 1)).astype(np.int64) + 1
    return (np.asarray(p) + bc + 1 + 40 + 31) // 32


def limb_products(nx, ny, W):
    """Schoolbook 32 x 32 -> 64-bit limb products of one real term when each
    operand is cut to the W + 1 limbs that can reach the window."""
    return np.minimum(nx, W + 1).astype(np.float64) * np.minimum(ny, W + 1)


def bench_dot_batch(arbgpu, torch, log, launches: int):
    """The 10^4-dot complex ball batch as one graph launch (tuned first)."""
    t0 = time.time()
    w = gen.config3()
    terms = int(w.lengths.sum())
    log(f"[bench] dot batch: {len(w.lengths)} dots, {terms} terms, generated in {time.time() - t0:.1f}s")
    # algorithmic work: per complex term the four real limb products; and
    # the bytes a launch must move: every operand's limbs that can reach its
    # dot's window (W + 1 of them) and its metadata (nls, exp 4 B each, the
    # radius 8 + 4 B), and every output (p bits of limbs, exp, nls, radius,
    # status)
    W = np.repeat(window_limbs(w.precs, 2 * w.lengths + 1), w.lengths)
    n = [o.nls.astype(np.int64) & 0x7FFFFFFF for o in (w.x_re, w.x_im, w.y_re, w.y_im)]
    products = float(np.sum(limb_products(n[0], n[2], W) + limb_products(n[1], n[3], W) +
                            limb_products(n[0], n[3], W) + limb_products(n[1], n[2], W)))
    in_bytes = float(sum(np.sum(4 * np.minimum(nk, W + 1) + 20) for nk in n))
    out_bytes = float(2 * np.sum(4 * ((w.precs + 31) // 32) + 21))
    nbytes = in_bytes + out_bytes
    ctx = arbgpu.Context(0)
    dev = [arbgpu.DeviceArray.from_host(o) for o in (w.x_re, w.x_im, w.y_re, w.y_im)]
    del w.x_re, w.x_im, w.y_re, w.y_im
    stream = torch.cuda.current_stream()

    def timed_batch(flags):
        """Build, tune and time the batch; its outputs and run list."""
        outs = [arbgpu.DeviceOut.empty(len(w.lengths), 1024), arbgpu.DeviceOut.empty(len(w.lengths), 1024)]
        jobs = [arbgpu.dot_job([outs[0].out(), outs[1].out()], i, [dev[0].arr(), dev[1].arr()], int(w.offsets[i]),
                               1, [dev[2].arr(), dev[3].arr()], int(w.offsets[i]), 1, int(w.lengths[i]),
                               int(w.precs[i]), arbgpu.COMPLEX | flags) for i in range(len(w.lengths))]
        b = arbgpu.Batch(ctx, jobs)
        b.launch(stream)
        torch.cuda.synchronize()
        b.tune(stream)
        b.launch(stream)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(launches):
            b.launch(stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        info = b.info()
        b.close()
        return ev0.elapsed_time(ev1) / launches, [o.to_host() for o in outs], info

    # the default path (digit products, the limb kernels for what they hand
    # back), then the limb kernels alone on the same jobs
    ms, res, info = timed_batch(0)
    ms_limb, res_limb, _ = timed_batch(arbgpu.ALGO_LIMB)
    same = all(np.array_equal(a.limbs, c.limbs) and np.array_equal(a.exp, c.exp) and np.array_equal(a.nls, c.nls)
               and np.array_equal(a.rad_m, c.rad_m) and np.array_equal(a.rad_e, c.rad_e) and np.array_equal(sa, sc)
               for (a, sa), (c, sc) in zip(res, res_limb))
    log(f"[bench] dot batch on the limb kernels alone: {ms_limb:.2f} ms/launch; outputs identical: {same}")
    ctx.close()
    cmacs = terms / (ms / 1e3)
    achieved = products / (ms / 1e3)
    gbs = nbytes / (ms / 1e3) / 1e9
    log(f"[bench] dot batch {ms:.2f} ms/launch, {cmacs:.3e} complex MACs/s, {gbs:.0f} GB/s of "
        f"{nbytes / 1e9:.2f} GB algorithmic ({gbs / PEAK_HBM_GBS:.1%} of HBM); limb-product equivalent "
        f"{achieved / PEAK_LIMB_PRODUCTS:.1%} of the v_mad_u64_u32 rate")
    # digit runs report ns = -blocks, na = 1 (real) or 2 (complex)
    return {"dots": len(w.lengths), "terms": terms, "launches": launches, "ms_per_launch": ms,
            "limb_kernels_alone_ms_per_launch": ms_limb, "identical_to_limb_kernels": same,
            "complex_macs_per_s": cmacs, "real_macs_per_s": 4 * cmacs,
            "mean_p": float(np.mean(w.precs)), "shapes": info["shapes"],
            "roofline": {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                         "frac": gbs / PEAK_HBM_GBS, "traffic": None, "bytes_per_launch": nbytes},
            "limb_product_equivalent": {"achieved": achieved / 1e12, "peak": PEAK_LIMB_PRODUCTS / 1e12,
                                        "unit": "T limb products/s", "frac": achieved / PEAK_LIMB_PRODUCTS,
                                        "products_per_launch": products}}


def bench_serving(arbgpu, torch, log, nreq: int, rate: float, slots: int):
    """Open-loop Poisson arrivals of complex ball matrix products; operands
    are taken from resident 1024x1024 pools (the top-left n x n block, row
    stride 1024), outputs from a ring of 8 buffers per precision."""
    reqs = gen.config4_requests(count=nreq, rate=rate)
    ps = sorted({r.p for r in reqs})
    t0 = time.time()
    pools, rings = {}, {}
    for p in ps:
        rng = gen.rng_for(4, 500 + p)
        pools[p] = [arbgpu.DeviceArray.from_host(o) for o in gen.config4_operands(rng, 1024, p)]
        rings[p] = [[arbgpu.DeviceOut.empty(1024 * 1024, p), arbgpu.DeviceOut.empty(1024 * 1024, p)]
                    for _ in range(8)]
    torch.cuda.synchronize()
    log(f"[bench] serving: {nreq} requests at {rate}/s, pools ready in {time.time() - t0:.1f}s")
    ctx = arbgpu.Context(0)
    ctx.serve_config(slots=slots)
    used = {p: 0 for p in ps}

    def job(r):
        P = pools[r.p]
        ring = rings[r.p][used[r.p] % 8]
        used[r.p] += 1
        A = arbgpu.Mat(P[0].arr(), P[1].arr(), r.n, r.n, 0, 1024, 1)
        B = arbgpu.Mat(P[2].arr(), P[3].arr(), r.n, r.n, 0, 1024, 1)
        C = arbgpu.OMat(ring[0].out(), ring[1].out(), r.n, r.n, 0, 1024, 1)
        return arbgpu.matmul_job(C, A, B, r.p, arbgpu.COMPLEX)

    # warm the slots' workspaces and kernels with one request of each precision
    warm = ctx.submit([job(gen.Request(0.0, 256, p)) for p in ps])
    for t in warm:
        ctx.wait(t, 600.0)
    tickets, arrivals = [], []
    start = time.monotonic_ns()
    retries = 0
    for k, r in enumerate(reqs):
        due = start + int(r.arrival_s * 1e9)
        now = time.monotonic_ns()
        if due > now:
            time.sleep((due - now) / 1e9)
        jb = job(r)
        while True:
            rc, t = ctx.submit([jb], check=False)
            if rc == arbgpu.OK:
                break
            if rc != arbgpu.EAGAIN:
                raise RuntimeError(f"submit failed: {rc} {ctx.last_error()}")
            retries += 1
            time.sleep(0.001)
        tickets.append(t[0])
        arrivals.append(due)
        if k % 100 == 99:
            log(f"[bench] serving: {k + 1} submitted")
    last_submit = time.monotonic_ns()
    for k, t in enumerate(tickets):
        ctx.wait(t, 1200.0)
        if k % 100 == 99:
            log(f"[bench] serving: {k + 1} done")
    end = max(ctx.ticket_times(t)[2] for t in tickets)
    lat = np.array([(ctx.ticket_times(t)[2] - a) / 1e6 for t, a in zip(tickets, arrivals)])
    wait = np.array([(ctx.ticket_times(t)[1] - a) / 1e6 for t, a in zip(tickets, arrivals)])
    ctx.close()
    cmacs = float(sum(r.n ** 3 for r in reqs))
    span = (end - start) / 1e9
    log(f"[bench] serving p50 {np.percentile(lat, 50):.1f} ms, p99 {np.percentile(lat, 99):.1f} ms, "
        f"span {span:.1f}s for {reqs[-1].arrival_s:.1f}s of arrivals")
    return {"requests": nreq, "rate_per_s": rate, "slots": slots,
            "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                           "max": float(lat.max())},
            "queue_wait_ms": {"p50": float(np.percentile(wait, 50)), "p99": float(np.percentile(wait, 99))},
            "complex_macs_per_s": cmacs / span, "real_macs_per_s": 4 * cmacs / span,
            "arrival_span_s": reqs[-1].arrival_s, "completion_span_s": span,
            "submit_span_s": (last_submit - start) / 1e9, "eagain_retries": retries}

def bench_largest(arbgpu, torch, log, n: int = 1024, p: int = 2048, reps: int = 5):
    """The largest serving request alone: a complex n x n ball product at
    precision p (operands as in the serving pools), wall time per call and
    per-kernel HIP-event times."""
    rng = gen.rng_for(4, 900 + p)
    dev = [arbgpu.DeviceArray.from_host(o) for o in gen.config4_operands(rng, n, p)]
    C, Ci = arbgpu.DeviceOut.empty(n * n, p, radius=True), arbgpu.DeviceOut.empty(n * n, p, radius=True)
    ctx = arbgpu.Context(0)
    call = lambda: ctx.mat_mul(C, dev[0], dev[2], n, n, n, p, arbgpu.COMPLEX, Ci=Ci, Ai=dev[1], Bi=dev[3])
    call()
    torch.cuda.synchronize()
    ctx.timing(True)
    t = time.perf_counter()
    for _ in range(reps):
        call()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t) * 1e3 / reps
    kern = {k: ctx.timing_read(k)[0] / reps for k in ("stats", "slice", "mfma", "recombine", "rad_gemm")}
    ctx.timing(False)
    plan = ctx.plan_info()
    ctx.close()
    log(f"[bench] largest request n={n} p={p} complex: {ms:.2f} ms, kernels {kern}")
    return {"n": n, "p": p, "complex": True, "ms": ms, "reps": reps, "kernels_ms": kern,
            "primes": plan["primes"], "digit_pairs_per_part": plan["pairs"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--batch-launches", type=int, default=5, help="0 skips the dot batch")
    ap.add_argument("--serve-requests", type=int, default=2000, help="0 skips the serving loop")
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-sweep", default="50,100,400,800,1600,3200",
                    help="further arrival rates (req/s) up to saturation; empty skips")
    ap.add_argument("--sweep-seconds", type=float, default=2.0, help="seconds of arrivals per sweep rate")
    ap.add_argument("--no-counters", action="store_true",
                    help="skip the HBM counter runs (rocprofv3 children); traffic then comes from the stored runs")
    ap.add_argument("--traffic-child", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--no-largest", action="store_true", help="skip timing the largest serving request alone")
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--no-peaks", action="store_true", help="skip the machine-limit microbenchmarks")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also copy a buffer of this many MiB once (reference kernel for HBM counters)")
    a = ap.parse_args()
    if a.traffic_child:
        traffic_child(a.n)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the multi-GPU design is "
                                   "described but not built", "n_gpus": a.gpus}))
        sys.exit(2)

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    t0 = time.time()
    w = gen.config2(n=a.n)
    log(f"[bench] generated {w.name} in {time.time() - t0:.1f}s")

    cpu = None
    if not a.no_cpu:
        cores = len(os.sched_getaffinity(0))
        cores = max(1, min(cores, 16))
        log(f"[bench] oracle baseline on {cores} cores, {a.cpu_seconds:.0f}s")
        cpu = cpu_baseline(w, a.cpu_seconds, cores)
        log(f"[bench] oracle {cpu['value']:.3e} MACs/s")

    import torch
    from paper_1901_04289_amd import arbgpu

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    ctx = arbgpu.Context(0)
    dA, dB = arbgpu.DeviceArray.from_host(w.A), arbgpu.DeviceArray.from_host(w.B)
    M, N, K, p = w.M, w.N, w.K, w.p
    C = arbgpu.DeviceOut.empty(M * K, p, radius=True)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()

    if a.copy_calibration_mib:
        src = torch.empty(a.copy_calibration_mib << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        src.fill_(1)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    peaks = None
    if not a.no_peaks:
        scratch = torch.empty(2 << 30, dtype=torch.uint8, device="cuda")
        peaks = ctx.probe_peaks(scratch, stream)
        del scratch
        torch.cuda.empty_cache()
        log(f"[bench] measured limits {peaks}")

    macs = float(M) * N * K
    KERNELS = ("stats", "slice", "mfma", "recombine")

    def measure(flags, steps, warmup):
        """Steps of one scaled-integer form: wall time per step, HIP-event
        latencies, per-kernel times and the MFMA roofline."""
        for _ in range(warmup):
            ctx.mat_mul(C, dA, dB, M, N, K, p, flags)
        torch.cuda.synchronize()
        ctx.timing(True)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for k in range(steps):
            ev[k][0].record(stream)
            ctx.mat_mul(C, dA, dB, M, N, K, p, flags)
            ev[k][1].record(stream)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        ms_step = (t2 - t1) * 1e3 / steps
        lat = np.array([x.elapsed_time(y) for x, y in ev])
        kern = {k: ctx.timing_read(k) for k in KERNELS}
        ctx.timing(False)
        plan = ctx.plan_info()
        mfma_ms, mfma_n = kern["mfma"]
        mfma_avg_s = mfma_ms / max(mfma_n, 1) / 1e3
        int8_ops = 2.0 * plan["pairs"] * M * K * N   # digit-plane pairs x MACs x 2
        achieved = int8_ops / mfma_avg_s / 1e12
        return {"ms_per_step": ms_step, "value": macs / (ms_step / 1e3), "lat": lat,
                "kernels_ms_per_step": {k: v[0] / steps for k, v in kern.items()},
                "plan": plan, "mfma_avg_ms": mfma_avg_s * 1e3, "int8_ops": int8_ops,
                "mfma_tops": achieved}

    # the library's automatic choice (residues modulo small primes at this
    # shape) is the headline; base-256 slices are measured beside it
    main = measure(0, a.steps, a.warmup)
    log(f"[bench] auto path {main['ms_per_step']:.2f} ms/step, kernels {main['kernels_ms_per_step']}, "
        f"plan {main['plan']}")
    C_main = (C.limbs.clone(), C.exp.clone(), C.nls.clone())
    forms = {}
    for name, flag in (("residues", arbgpu.ALGO_RNS), ("slices", arbgpu.ALGO_SLICED)):
        r = measure(flag, max(2, a.steps // 4), 1)
        forms[name] = {"ms_per_step": r["ms_per_step"], "value": r["value"], "unit": "p-bit MACs/s",
                       "kernels_ms_per_step": r["kernels_ms_per_step"], "digit_pairs": r["plan"]["pairs"],
                       "primes": r["plan"]["primes"], "mfma_avg_ms": r["mfma_avg_ms"],
                       "mfma_frac_of_int8_peak": r["mfma_tops"] / PEAK_INT8_TOPS,
                       "mfma_traffic_bytes": _stored_traffic(a.n, name),
                       "bit_identical_midpoints": bool(torch.equal(C.limbs, C_main[0])
                                                       and torch.equal(C.exp, C_main[1])
                                                       and torch.equal(C.nls, C_main[2]))}
        log(f"[bench] {name} {r['ms_per_step']:.2f} ms/step, mfma {r['mfma_avg_ms']:.2f} ms "
            f"({r['mfma_tops'] / PEAK_INT8_TOPS:.1%} of INT8 peak)")
    ms_step, value, lat, plan = main["ms_per_step"], main["value"], main["lat"], main["plan"]
    mfma_avg_s = main["mfma_avg_ms"] / 1e3
    int8_ops = main["int8_ops"]
    achieved = main["mfma_tops"]
    digits_path = plan["primes"] == 0

    out = {
        "metric": METRIC, "value": value, "unit": "p-bit MACs/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "i8", "data": "synthetic",
        "config": {"workload": "real matrix product 2048x2048 by 2048x2048, p=512, 512-bit mantissas, "
                               "exponents uniform in [-4,4], exact inputs (zero radius)",
                   "N": a.n, "p": p,
                   "path": "scaled-integer block product on INT8 MFMA, " +
                           ("base-256 digit slices" if digits_path else
                            f"residues modulo {plan['primes']} primes below 2^15")},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "max": float(lat.max())},
        "kernels_ms_per_step": main["kernels_ms_per_step"],
        "slice_plan": plan,
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_INT8_TOPS, "unit": "TOP/s",
                     "frac": achieved / PEAK_INT8_TOPS,
                     "traffic": _stored_traffic(a.n, "slices" if digits_path else "residues"),
                     "traffic_source": "stored counter runs on this kernel source (hash-checked)",
                     "kernel": MFMA_KERNEL["slices" if digits_path else "residues"], "ops_per_launch": int8_ops,
                     "avg_launch_ms": mfma_avg_s * 1e3},
        "int8_forms": forms,
        "cpu_baseline": cpu,
    }
    if peaks is not None:
        out["measured_peaks"] = peaks
        out["roofline"]["measured_peak"] = peaks["int8_mfma_tops"]
        out["roofline"]["frac_of_measured_peak"] = achieved / peaks["int8_mfma_tops"]
    ctx.mat_mul(C, dA, dB, M, N, K, p, 0)
    torch.cuda.synchronize()

    # plain limb-window kernel on the same product
    if not a.no_plain:
        Cl = arbgpu.DeviceOut.empty(M * K, p, radius=True)
        ctx.mat_mul(Cl, dA, dB, M, N, K, p, arbgpu.ALGO_LIMB)   # warmup
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        for _ in range(a.plain_steps):
            ctx.mat_mul(Cl, dA, dB, M, N, K, p, arbgpu.ALGO_LIMB)
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        ms_plain = (t4 - t3) * 1e3 / a.plain_steps
        same = bool(torch.equal(C.limbs, Cl.limbs) and torch.equal(C.exp, Cl.exp) and torch.equal(C.nls, Cl.nls))
        # algorithmic work: the limb products of every term of every entry,
        # sum over k of (sum_i m_A(i,k)) (sum_j m_B(k,j))
        Wm = int(window_limbs(p, N + 1))
        mA = np.minimum(w.A.nls.astype(np.int64) & 0x7FFFFFFF, Wm + 1).reshape(M, N).astype(np.float64)
        mB = np.minimum(w.B.nls.astype(np.int64) & 0x7FFFFFFF, Wm + 1).reshape(N, K).astype(np.float64)
        products = float(mA.sum(axis=0) @ mB.sum(axis=1))
        achieved = products / (ms_plain / 1e3)
        out["plain_limb"] = {"value": macs / (ms_plain / 1e3), "unit": "p-bit MACs/s", "ms_per_step": ms_plain,
                             "steps": a.plain_steps, "bit_identical_midpoints": same,
                             "roofline": {"bound": "alu", "achieved": achieved / 1e12,
                                          "peak": PEAK_LIMB_PRODUCTS / 1e12, "unit": "T limb products/s",
                                          "frac": achieved / PEAK_LIMB_PRODUCTS, "traffic": None,
                                          "products_per_launch": products}}
        out["speedup_vs_plain"] = ms_plain / ms_step
        log(f"[bench] plain {ms_plain:.1f} ms/step, identical midpoints: {same}")
        del Cl
    ctx.close()
    del C, dA, dB
    torch.cuda.empty_cache()
    if a.batch_launches:
        out["dot_batch"] = bench_dot_batch(arbgpu, torch, log, a.batch_launches)
        torch.cuda.empty_cache()
    if not a.no_largest:
        out["largest_request"] = bench_largest(arbgpu, torch, log)
        torch.cuda.empty_cache()
    if a.serve_requests:
        out["serving"] = bench_serving(arbgpu, torch, log, a.serve_requests, a.serve_rate, a.serve_slots)
        out["latency_ms"]["serving_p50"] = out["serving"]["latency_ms"]["p50"]
        out["latency_ms"]["serving_p99"] = out["serving"]["latency_ms"]["p99"]
        sweep = []
        for rate in [float(x) for x in a.serve_sweep.split(",") if x.strip()]:
            r = bench_serving(arbgpu, torch, log, max(1, int(round(a.sweep_seconds * rate))), rate,
                              a.serve_slots)
            # keeps pace: every request admitted at once and the completions
            # end within 10% (+50 ms) of the arrivals
            pace = (r["eagain_retries"] == 0 and
                    r["completion_span_s"] <= 1.1 * r["arrival_span_s"] + 0.05)
            sweep.append({"rate_per_s": rate, "requests": r["requests"], "latency_ms": r["latency_ms"],
                          "queue_wait_ms": r["queue_wait_ms"],
                          "completed_req_per_s": r["requests"] / r["completion_span_s"],
                          "complex_macs_per_s": r["complex_macs_per_s"], "eagain_retries": r["eagain_retries"],
                          "keeps_pace": pace})
        if sweep:
            out["serving_sweep"] = sweep
            kept = [x for x in sweep if x["keeps_pace"]]
            over = [x for x in sweep if not x["keeps_pace"]]
            out["serving_capacity"] = {
                "max_rate_kept_per_s": max((x["rate_per_s"] for x in kept), default=None),
                "first_rate_not_kept_per_s": min((x["rate_per_s"] for x in over), default=None),
                "max_completed_req_per_s": max(x["completed_req_per_s"] for x in sweep),
                "max_complex_macs_per_s": max(x["complex_macs_per_s"] for x in sweep)}
    if not a.no_counters:
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        cnt = hbm_counters(a.n, log)
        if cnt is not None:
            kname = "mfma_diag_kernel" if digits_path else "mfma_rns_kernel"
            out["traffic_by_kernel"] = cnt
            if kname in cnt["per_dispatch"]:
                out["roofline"]["traffic"] = cnt["per_dispatch"][kname]["bytes"]
                out["roofline"]["traffic_source"] = cnt["source"]
            for form, kn in (("residues", "mfma_rns_kernel"), ("slices", "mfma_diag_kernel")):
                if kn in cnt["per_dispatch"]:
                    out["int8_forms"][form]["mfma_traffic_bytes"] = cnt["per_dispatch"][kn]["bytes"]
    # no child process outlives the run
    for c in mp.active_children():
        c.join(10)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
