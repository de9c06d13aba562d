#!/usr/bin/env python3
"""Benchmark of the spin summation on one MI355X.

Headline workload: 3D spin summation, FP64, in place, of the amplitude
tensor T[a,b,c,i,j,k] with v = 64 virtual and o = 32 occupied extents,
processed as 8 slabs of 64 x 64 x 8 x 32^3 (1.07G elements, 8.6 GB each);
coefficients identity 4, each transposition -2, each 3-cycle +1.  One step
is one in-place pass over all 8 slabs (8 launches, one per slab).  The
metric is the paper's bandwidth measure (Eq. 12, one read and one write of
every element) in GB/s, and its fraction of the 8 TB/s HBM peak.

Also reported, each against the plain FP64 kernel (``forms``): the 4D
in-place summation, the chained (2 - P_ij)(2 - P_jk) form, the batched
persistent launch replayed from a hipGraph against per-block launches, the
adjoint, and FP32 storage.  ``cpu_baseline`` is the CPU oracle timed on a
bounded sample of the headline workload.

    python bench.py [--steps K] [--warmup W] [--forms all|none] [--no-cpu-baseline]
    python bench.py --profile FORM [--steps K] [--warmup W]   (one form alone)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_GBPS = 8000.0
METRIC = "effective GB/s & % HBM peak, FP64 in-place 3D/4D spinsum; batched/adjoint/FP32 vs plain"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1705_06661_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h", ".cpp")):
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(name: str):
    """HBM bytes per launch of the form `name` (one of PROFILE_FORMS) from
    its committed rocprofv3 counter summary (FETCH_SIZE and WRITE_SIZE, each
    scaled by a plain copy's reading), or None when the counters were taken
    on other kernel sources."""
    path = os.path.join(ROOT, "profiles", f"spinsum_{name}.traffic.txt")
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as f:
        for line in f:
            if line.startswith("#") or ":" not in line:
                continue
            k, v = line.split(":", 1)
            rec[k.strip()] = v.strip()
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    try:
        return float(rec["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def kernel_name(info, dtype="double", chain=False):
    """Name of the device kernel a plan launches, as rocprofv3 lists it."""
    d = info["exec_d"] or info["d"]
    v = info["variant"]
    c = "true" if chain else "false"
    nts = "true" if info["nt_stores"] else "false"
    if info["pair_extent"] > 0:
        return f"k_pair<{dtype}, {d}, {c}, {nts}>"
    if v == 1:
        return f"k_lds<{dtype}, {d}, {c}, {nts}>"
    if v == 4:
        return f"k_ldsp<{dtype}, {d}, {c}, {nts}>"
    if v == 2:
        return f"k_pipe<{dtype}, {d}, {info['vector_width']}, {c}, *>"
    return f"k_exec<{dtype}, {d}, {info['vector_width']}, {c}, {nts}>"


def batched_kernel_name(info):
    """The FP64 3D batched kernel (16-byte chunks), one-shot or persistent."""
    return "k_batched<double, 3, 2, %s>" % ("true" if info["batch_persistent"] else "false")


def warm(fn, seconds=0.25, refill=None):
    """Untimed repeats of a form's call until `seconds` have passed, so that
    a short form is not timed while the GPU clocks are still ramping up
    after host-side set-up (measured: 4D slab 1.11 ms cold, 0.955 ms warm).
    In-place forms pass `refill`, which restores finite input values after
    the warm-up: every in-place pass multiplies magnitudes by up to the
    operator's spectral radius (12 for the 3D set, up to ~85 for 24 random 4D
    coefficients), so hundreds of passes overflow to Inf/NaN, and non-finite
    inputs take the slower term-by-term combine of operators with zero
    coefficients."""
    import torch
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for _ in range(4):
            fn()
        torch.cuda.synchronize()
    if refill is not None:
        refill()
        torch.cuda.synchronize()


def timed(fn, reps, stream):
    import torch
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s.record(stream)
    for _ in range(reps):
        fn()
    e.record(stream)
    torch.cuda.synchronize()
    return s.elapsed_time(e) / reps


def form_entry(nbytes, ms, ref_gbps=None):
    gbps = nbytes / (ms * 1e-3) / 1e9
    d = {"GBps": round(gbps, 1), "frac_peak": round(gbps / PEAK_GBPS, 4), "ms": round(ms, 4)}
    if ref_gbps:
        d["vs_plain_fp64"] = round(gbps / ref_gbps, 3)
    return d


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# The paper's own measurements, quoted for context with its hardware (its
# text gives relative numbers only): Alg. 6 against the NCC / CFOUR
# implementation on Table II, FP64.
PAPER_CONTEXT = {
    "speedup_over_ncc": {"all_sizes": "2.4-5.5x", "small": "2.4-4.3x", "medium": "2.4-3.8x",
                         "large": "3.3-5.5x"},
    "in_place_over_out_of_place": "up to 1.2x",
    "hardware": "2x Intel Xeon E5-2680 v3, 24 threads",
    "stream_copy_GiBps": 101.2,
}


def cpu_baseline(seconds: float, nslabs: int):
    """The oracle on a bounded sample of the headline workload: consecutive
    whole 32^3 spectator cubes of the slabs, regenerated on the host from
    the same seeds, until about `seconds` of oracle time."""
    import numpy as np
    import oracle
    import workloads
    cube = 32 ** 3
    per_slab = 64 * 64 * 8
    threads, nproc, allowed = cpu_threads()
    chunk = 1024
    done, total = 0, 0.0
    while total < seconds and done < nslabs * per_slab:
        slab, c0 = divmod(done, per_slab)
        x = workloads.uniform_numpy(chunk * cube, 1000 + slab, offset=c0 * cube).reshape(chunk, 32, 32, 32)
        t0 = time.perf_counter()
        oracle.spinsum(x, workloads.CONFIG_3D_ALPHA, 1, 3, nthreads=threads)
        total += time.perf_counter() - t0
        done += chunk
    elems = done * cube
    # the same oracle on one thread, over the first chunk (a few seconds)
    x = workloads.uniform_numpy(chunk * cube, 1000, offset=0).reshape(chunk, 32, 32, 32)
    t0 = time.perf_counter()
    oracle.spinsum(x, workloads.CONFIG_3D_ALPHA, 1, 3, nthreads=1)
    t1 = time.perf_counter() - t0
    return {"value": round(2 * elems * 8 / total / 1e9, 4), "unit": "GB/s", "cores": threads,
            "kind": "oracle", "nproc": nproc, "affinity_cpus": allowed,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS"),
            "one_thread_value": round(2 * chunk * cube * 8 / t1 / 1e9, 4),
            "cpu_model": cpu_model(),
            "sample": f"the first {done} spectator cubes (32^3 each, {elems} elements, fp64) of the "
                      f"{nslabs} slabs of the v=64 o=32 in-place workload, in slab order, "
                      f"{total:.1f} s of oracle time on {threads} threads; one_thread_value: "
                      f"the first {chunk} of them on one thread"}


def cpu_threads():
    """Threads for the oracle: every CPU this process may run on
    (sched_getaffinity), capped by OMP_NUM_THREADS where the host sets it
    (the share of a shared GPU host's CPUs that one GPU job is given).
    Returns (threads, os.cpu_count(), CPUs in the affinity mask)."""
    nproc = os.cpu_count() or 1
    try:
        allowed = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        allowed = nproc
    threads = allowed
    omp = os.environ.get("OMP_NUM_THREADS", "")
    if omp.isdigit() and int(omp) > 0:
        threads = min(threads, int(omp))
    return max(1, threads), nproc, allowed


# The paper's three tensor sizes (Sec. 5.1: about 70, 320 and 1200 MiB),
# hyper-square, no spectators: 3D N = 208 / 352 / 544 (rows of whole
# 128-byte lines), 4D N = 54 / 80 / 112.
TABLE2_SIZES = {"small": {3: 208, 4: 54}, "medium": {3: 352, 4: 80}, "large": {3: 544, 4: 112}}


def table2_sweep(ss, workloads, dev, stream, size="medium"):
    """The paper's benchmark (Table II, all 21 spin summations) on hyper-square
    tensors without spectators at one of the sizes of Sec. 5.1, in place,
    FP64, caches flushed before each of 10 reps; the fastest rep (as in the
    paper) and the median.  Eq. 12 bandwidth in GiB/s and Eq. 13 GFLOP/s
    with n = the number of expanded permutations."""
    import torch
    res = {}
    tensors = {}
    flush = torch.empty(1 << 27, dtype=torch.float64, device=dev)
    for case in range(1, 22):
        d, stages = workloads.table2_case(case)
        n = TABLE2_SIZES[size][d]
        shape = (n,) * d
        if d not in tensors:
            tensors[d] = torch.empty(shape, dtype=torch.float64, device=dev)
        x = tensors[d]
        workloads.fill_uniform(x, 5000 + case)
        p = ss.spinsum_plan(shape, 0, d, stages, inplace=True)
        info = ss.spinsum_plan_get_info(p)
        warm(lambda: ss.spinsum_exec(p, x, x, stream), 0.15)
        workloads.fill_uniform(x, 5000 + case)  # thousands of warm-up passes grow the values
        # each rep on cold caches: a 1 GiB scratch write evicts L2 and MALL
        # (the small size fits the MALL) outside the timed region
        times = []
        for _ in range(10):
            flush.fill_(0.0)
            times.append(timed(lambda: ss.spinsum_exec(p, x, x, stream), 1, stream))
        times.sort()
        ms = times[0]
        ms_median = times[len(times) // 2]
        elems = x.numel()
        t = ms * 1e-3
        # [GB/s, fraction of peak, Eq. 12 GiB/s, Eq. 13 GFLOP/s, ms (fastest),
        #  ms (median), expanded terms, tile edge]
        res[str(case)] = [round(2 * elems * 8 / 1e9 / t, 1),
                          round(2 * elems * 8 / 1e9 / t / PEAK_GBPS, 4),
                          round(2 * elems * 8 / 2 ** 30 / t, 1),
                          round(2 * info["nterms_expanded"] * elems / 1e9 / t, 1),
                          round(ms, 4), round(ms_median, 4), info["nterms_expanded"], info["bl"]]
    res["columns"] = ["GBps", "frac_peak", "GiBps_eq12", "GFLOPs_eq13", "ms", "ms_median",
                      "terms", "tile_edge"]
    res["N"] = {"3d": TABLE2_SIZES[size][3], "4d": TABLE2_SIZES[size][4]}
    del tensors, flush
    torch.cuda.empty_cache()
    return res


def accuracy_report(ss, workloads, dev, stream):
    """Errors of the v=48, o=24 forward and adjoint with (2 - P_ij)(2 - P_jk)
    (whose adjoint differs from it), all normwise, max|got - ref| / max|ref|:
      * FP32 storage and accumulation against FP64, on the whole tensor: the
        FP32 kernel on the FP32-rounded input against the FP64 kernel on the
        same rounded values ("rounded", the arithmetic alone) and on the
        unrounded input ("unrounded", storage included);
      * the FP64 and FP32 kernels against the oracle on sampled spectator
        cubes (inputs regenerated on the host from the seeded stream);
      * finite differences of the linear map: <g, (S(x + h v) - S(x)) / h>
        against <S^T g, v> (adjoint kernel) for h = 1 and 1e-3, FP64, whole
        tensor (the gradient check of the autograd form)."""
    import numpy as np
    import torch
    import oracle
    w5 = workloads.WORKLOADS["3d_v48_o24"]
    shape = w5["shape"]
    st = workloads.FACTORED_PIJ_PJK
    cube = 24 ** 3
    ncubes = 48 ** 3
    picks = [0, 1, 4097, 55555, 99991, ncubes - 1]
    p64 = ss.spinsum_plan(shape, 3, 3, st, dtype=torch.float64)
    p32 = ss.spinsum_plan(shape, 3, 3, st, dtype=torch.float32)

    def nerr(a, b):
        return float((a - b).abs().max() / b.abs().max())

    rep = {"workload": "3d_v48_o24 [48,48,48,24,24,24], (2 - P_ij)(2 - P_jk), U(-1,1) seed 4000 "
                       "(upstream gradient seed 4002, direction seed 4001)",
           "norm": "max|got - ref| / max|ref|", "tolerance": {"fp64": 1e-14, "fp32": 2e-6}}
    for name, fn in (("forward", ss.spinsum_exec), ("adjoint", ss.spinsum_adjoint)):
        x = workloads.uniform(shape, 4000, device=dev)
        x32 = x.to(torch.float32)
        y64 = torch.empty_like(x)
        fn(p64, x, y64, stream)
        y32 = torch.empty_like(x32)
        fn(p32, x32, y32, stream)
        yr = torch.empty_like(x)
        fn(p64, x32.to(torch.float64), yr, stream)
        torch.cuda.synchronize()
        y32d = y32.to(torch.float64)
        e = {"fp32_vs_fp64_rounded_input": nerr(y32d, yr),
             "fp32_vs_fp64_unrounded_input": nerr(y32d, y64)}
        del x, x32, yr, y32d
        torch.cuda.empty_cache()
        worst64, worst32 = 0.0, 0.0
        for c in picks:
            xh = workloads.uniform_numpy(cube, 4000, offset=c * cube).reshape(1, 24, 24, 24)
            x32h = xh.astype(np.float32).astype(np.float64)
            f = oracle.spinsum_chain_adjoint if name == "adjoint" else oracle.spinsum_chain
            ref = f(xh, st, 1, 3)
            ref32 = f(x32h, st, 1, 3)
            g64 = y64.view(-1, cube)[c].cpu().numpy().reshape(ref.shape)
            g32 = y32.view(-1, cube)[c].cpu().to(torch.float64).numpy().reshape(ref.shape)
            worst64 = max(worst64, float(np.max(np.abs(g64 - ref)) / np.max(np.abs(ref))))
            worst32 = max(worst32, float(np.max(np.abs(g32 - ref32)) / np.max(np.abs(ref32))))
        e["fp64_vs_oracle_sampled"] = worst64
        e["fp32_vs_oracle_rounded_input_sampled"] = worst32
        e["sampled_cubes"] = picks
        rep[name] = e
        del y64, y32
        torch.cuda.empty_cache()
    # finite differences (FP64)
    x = workloads.uniform(shape, 4000, device=dev)
    v = workloads.uniform(shape, 4001, device=dev)
    g = workloads.uniform(shape, 4002, device=dev)
    y0 = torch.empty_like(x)
    ss.spinsum_exec(p64, x, y0, stream)
    gt = torch.empty_like(g)
    ss.spinsum_adjoint(p64, g, gt, stream)
    torch.cuda.synchronize()
    analytic = float((gt * v).sum(dtype=torch.float64))
    del gt
    fd = {}
    for h in (1.0, 1e-3):
        xp = x + h * v
        y1 = torch.empty_like(x)
        ss.spinsum_exec(p64, xp, y1, stream)
        torch.cuda.synchronize()
        num = float((g * (y1 - y0)).sum(dtype=torch.float64)) / h
        fd[f"h={h:g}"] = {"fd": num, "analytic": analytic,
                          "rel_error": abs(num - analytic) / abs(analytic)}
        del xp, y1
        torch.cuda.empty_cache()
    rep["finite_differences_fp64"] = fd
    del x, v, g, y0
    torch.cuda.empty_cache()
    return rep


PROFILE_FORMS = ("3d_v64_o32_inplace", "4d_v24_o12_inplace", "4d_table2_5_80_premultiplied",
                 "3d_pairs_v48_o24_inplace", "3d_v48_o24_forward_fp64", "3d_coef_grad",
                 "3d_unpack_antisymmetric", "3d_v48_o24_adjoint_fp64", "3d_v48_o24_forward_fp32",
                 "batched_graph", "stream_copy")


def profile_one(name, steps, warmup):
    """One form alone, for a profiler run: its input is filled, then
    `warmup` untimed and `steps` timed launches follow, and one JSON line
    gives the average launch time.  Nothing else touches the GPU, so the
    counters of every spin-summation dispatch belong to this form."""
    import torch
    import workloads
    import paper_1705_06661_amd as ss

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    alpha = [workloads.CONFIG_3D_ALPHA]
    split = {}  # reads and writes where they are not one each of every element
    slab = workloads.WORKLOADS["3d_v64_o32_slab"]["shape"]
    if name in ("3d_v64_o32_inplace", "3d_coef_grad", "stream_copy"):
        x = workloads.uniform(slab, 1000, device=dev)
        y = workloads.uniform(slab, 1001, device=dev) if name != "3d_v64_o32_inplace" else x
        p = ss.spinsum_plan(slab, 3, 3, alpha, inplace=True)
        if name == "3d_coef_grad":
            fn = lambda: ss.spinsum_coef_grad(p, x, y, stream)
        elif name == "stream_copy":
            fn = lambda: ss.spinsum_stream_copy(x, y, stream)
        else:
            fn = lambda: ss.spinsum_exec(p, x, x, stream)
        nbytes = 2 * x.numel() * 8
    elif name == "4d_v24_o12_inplace":
        w4 = workloads.WORKLOADS["4d_v24_o12_slab"]
        x = workloads.uniform(w4["shape"], 2000, device=dev)
        p = ss.spinsum_plan(w4["shape"], 4, 4, [workloads.random_4d_alpha(7)], inplace=True)
        fn = lambda: ss.spinsum_exec(p, x, x, stream)
        nbytes = 2 * x.numel() * 8
    elif name == "4d_table2_5_80_premultiplied":
        x = workloads.uniform((80,) * 4, 5005, device=dev)
        p = ss.spinsum_plan(x.shape, 0, 4, workloads.table2_case(5)[1], inplace=True)
        fn = lambda: ss.spinsum_exec(p, x, x, stream)
        nbytes = 2 * x.numel() * 8
    elif name == "3d_pairs_v48_o24_inplace":
        w5 = workloads.WORKLOADS["3d_v48_o24"]
        x = workloads.uniform(w5["shape"], 5100, device=dev)
        p = ss.spinsum_plan(w5["shape"], 3, 3, alpha, inplace=True,
                            flags=ss.SPINSUM_FLAG_INDEX_PAIRS)
        fn = lambda: ss.spinsum_exec(p, x, x, stream)
        nbytes = 2 * x.numel() * 8
    elif name == "3d_v48_o24_forward_fp64":
        w5 = workloads.WORKLOADS["3d_v48_o24"]
        x = workloads.uniform(w5["shape"], 4000, device=dev)
        y = torch.empty_like(x)
        p = ss.spinsum_plan(w5["shape"], 3, 3, workloads.FACTORED_PIJ_PJK, inplace=False)
        fn = lambda: ss.spinsum_exec(p, x, y, stream)
        nbytes = 2 * x.numel() * 8
    elif name in ("3d_v48_o24_adjoint_fp64", "3d_v48_o24_forward_fp32"):
        w5 = workloads.WORKLOADS["3d_v48_o24"]
        dt = torch.float32 if name.endswith("fp32") else torch.float64
        x = workloads.uniform(w5["shape"], 4000, device=dev, dtype=dt)
        y = torch.empty_like(x)
        p = ss.spinsum_plan(w5["shape"], 3, 3, workloads.FACTORED_PIJ_PJK, dtype=dt, inplace=False)
        if name.startswith("3d_v48_o24_adjoint"):
            fn = lambda: ss.spinsum_adjoint(p, x, y, stream)
        else:
            fn = lambda: ss.spinsum_exec(p, x, y, stream)
        nbytes = 2 * x.numel() * x.element_size()
    elif name == "batched_graph":
        # the 200 power-law blocks, the autotuner's item size and launch
        # style, one graph launch per step (the tuning launches come first;
        # the summaries count the last launches only)
        _, blocks = workloads.batched_blocks()
        shapes = [(v, v, v, o, o, o) for v, o in blocks]
        xs = [workloads.uniform(s, 3000 + k, device=dev) for k, s in enumerate(shapes)]
        p = ss.spinsum_plan_batched(shapes, 3, alpha, inplace=True)
        ss.spinsum_autotune(p, xs, xs)
        for k, x in enumerate(xs):  # finite values again after the tuning passes
            workloads.fill_uniform(x, 3000 + k)
        graph = ss.spinsum_graph_create(p, xs, xs)
        fn = lambda: ss.spinsum_graph_launch(graph, stream)
        nbytes = 2 * 8 * sum(x.numel() for x in xs)
    elif name == "3d_unpack_antisymmetric":
        x = torch.empty(slab, dtype=torch.float64, device=dev)
        p = ss.spinsum_plan(slab, 3, 3, [workloads.antisymmetrizer(3)])
        pk = workloads.uniform(ss.packed_shape(p), 3200, device=dev)
        fn = lambda: ss.spinsum_unpack(p, pk, x, stream)
        split = {"algorithmic_read_bytes": pk.numel() * 8, "algorithmic_write_bytes": x.numel() * 8}
        nbytes = (pk.numel() + x.numel()) * 8
    else:
        raise SystemExit(f"unknown form {name!r}; one of {', '.join(PROFILE_FORMS)}")
    torch.cuda.synchronize()
    for _ in range(warmup):
        fn()
    ms = timed(fn, steps, stream)
    info = ss.spinsum_plan_get_info(p)
    print(json.dumps({"form": name, "launches": warmup + steps, "avg_launch_ms": round(ms, 4),
                      "GBps": round(nbytes / (ms * 1e-3) / 1e9, 1),
                      "algorithmic_bytes_per_launch": nbytes,
                      "kernel": {"stream_copy": "k_copy",
                                 "3d_coef_grad": ("k_cgrad_split<double, 3>" if info["coef_grad_split"]
                                                  else "k_cgrad<double, 3>"),
                                 "batched_graph": batched_kernel_name(info),
                                 "3d_unpack_antisymmetric": "%s<double, 3, %s>" % (
                                     "k_unpack_persist" if info["unpack_persistent"] else "k_unpack",
                                     "true" if info["unpack_nt_stores"] else "false")}.get(
                          name, kernel_name(info, "float" if name.endswith("fp32") else "double")),
                      "tile_edge": info["bl"], "launches_timed": steps, **split,
                      "kernel_source_hash": kernel_source_hash()}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--forms", default="all", choices=["all", "copy", "none"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--slabs", type=int, default=8)
    ap.add_argument("--profile", choices=PROFILE_FORMS, default=None,
                    help="run one form alone (for rocprofv3) and print its launch time")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the spin summation shards over spectator "
              "slabs with no communication, and no multi-GPU path is implemented.",
              file=sys.stderr)
        sys.exit(2)
    if args.profile is not None:
        profile_one(args.profile, args.steps, args.warmup)
        return

    import torch
    import workloads
    import paper_1705_06661_amd as ss

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    alpha = [workloads.CONFIG_3D_ALPHA]
    slab_shape = workloads.WORKLOADS["3d_v64_o32_slab"]["shape"]
    nslabs = args.slabs

    log(f"allocating {nslabs} slabs of {slab_shape} fp64")
    big = torch.empty((nslabs,) + tuple(slab_shape), dtype=torch.float64, device=dev)
    for s in range(nslabs):
        workloads.fill_uniform(big[s], 1000 + s)
    torch.cuda.synchronize()
    plan = ss.spinsum_plan(slab_shape, 3, 3, alpha, inplace=True)
    info = ss.spinsum_plan_get_info(plan)
    log("plan", info)

    def step():
        for s in range(nslabs):
            ss.spinsum_exec(plan, big[s], big[s], stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("timing")
    ms_step = timed(step, args.steps, stream)
    elems_step = nslabs * info["elems"]
    value = 2 * elems_step * 8 / (ms_step * 1e-3) / 1e9
    launch_ms = ms_step / nslabs
    algo_per_launch = 2.0 * info["elems"] * 8
    achieved = algo_per_launch / (launch_ms * 1e-3) / 1e9
    assert bool(torch.isfinite(big[0, 0, 0]).all()), "non-finite output"
    log(f"headline: {ms_step:.3f} ms/step, {value:.1f} GB/s")
    # single launches, after the timed region: each slab (8.6 GB) is far
    # larger than the L2 and MALL, so every launch runs on cold caches
    singles = []
    for _ in range(max(1, min(3, args.steps))):
        for s in range(nslabs):
            singles.append(timed(lambda: ss.spinsum_exec(plan, big[s], big[s], stream), 1, stream))
    singles.sort()

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "3d_v64_o32_inplace", "tensor": [64, 64, 64, 32, 32, 32],
                   "slabs": nslabs, "slab_shape": list(slab_shape), "group": "ijk",
                   "alpha": "id 4, transpositions -2, 3-cycles +1", "inplace": True,
                   "values": "U(-1,1) from seed", "tile_edge": info["bl"],
                   "tile_orbits_per_cube": info["norbits"],
                   "work_items_per_cube": info["items_per_cube"], "tiles_per_item": info["item_tiles"]},
        # the paper's own measures of the same run: Eq. 12 bandwidth in GiB/s
        # and Eq. 13 rate, two flops per term per element
        "paper_measures": {"GiBps_eq12": round(value * 1e9 / 2 ** 30, 1),
                           "GFLOPs_eq13": round(2 * info["nterms_expanded"] * elems_step
                                                / (ms_step * 1e-3) / 1e9, 1)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_GBPS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_GBPS, 4),
                     "traffic": traffic_from_profile("3d_v64_o32_inplace"),
                     "single_launch_ms_min": round(singles[0], 4),
                     "single_launch_ms_median": round(singles[len(singles) // 2], 4),
                     "kernel": kernel_name(info),
                     "algorithmic_bytes_per_launch": algo_per_launch,
                     "avg_launch_ms": round(launch_ms, 4)},
    }

    forms = {}
    if args.forms == "copy":
        dst = torch.empty_like(big[0])
        cms = timed(lambda: ss.spinsum_stream_copy(big[0], dst, stream), 2, stream)
        forms["stream_copy_ceiling"] = form_entry(2 * big[0].numel() * 8, cms)
        out["forms"] = forms
    if args.forms == "all":
        # achievable ceiling: plain copy of one slab with the same instructions
        dst = torch.empty_like(big[0])
        warm(lambda: ss.spinsum_stream_copy(big[0], dst, stream))
        cms = timed(lambda: ss.spinsum_stream_copy(big[0], dst, stream), 5, stream)
        forms["stream_copy_ceiling"] = form_entry(2 * big[0].numel() * 8, cms)
        out["roofline"]["frac_of_copy_ceiling"] = round(
            achieved / forms["stream_copy_ceiling"]["GBps"], 4)
        del dst
        # factorised sums three ways, slab 0: the pre-multiplied operator (one
        # pass), the stages chained in registers (one pass), and one pass per
        # stage through the output (Alg. 3), for (2 - P_ij)(2 - P_jk) and
        # Table II case 1
        for name, stages, flags in [
                ("3d_factored_premultiplied", workloads.FACTORED_PIJ_PJK, 0),
                ("3d_factored_chained", workloads.FACTORED_PIJ_PJK, ss.SPINSUM_FLAG_CHAIN_STAGES),
                ("3d_factored_multi_pass", workloads.FACTORED_PIJ_PJK, ss.SPINSUM_FLAG_MULTI_PASS),
                ("3d_table2_1_premultiplied", workloads.table2_case(1)[1], 0),
                ("3d_table2_1_chained", workloads.table2_case(1)[1], ss.SPINSUM_FLAG_CHAIN_STAGES),
                ("3d_table2_1_multi_pass", workloads.table2_case(1)[1], ss.SPINSUM_FLAG_MULTI_PASS)]:
            pf = ss.spinsum_plan(slab_shape, 3, 3, stages, inplace=True, flags=flags)
            workloads.fill_uniform(big[0], 1000)  # fresh values: repeated passes grow them
            warm(lambda: ss.spinsum_exec(pf, big[0], big[0], stream),
                 refill=lambda: workloads.fill_uniform(big[0], 1000))
            fms = timed(lambda: ss.spinsum_exec(pf, big[0], big[0], stream), 5, stream)
            forms[name] = form_entry(2 * big[0].numel() * 8, fms, value)
        # coefficient gradient <g, pi_p(x)> for all 6 permutations: two slabs
        # read once (no writes)
        workloads.fill_uniform(big[0], 1000)
        warm(lambda: ss.spinsum_coef_grad(plan, big[0], big[1], stream))
        cg = timed(lambda: ss.spinsum_coef_grad(plan, big[0], big[1], stream), 5, stream)
        forms["3d_coef_grad"] = form_entry(2 * big[0].numel() * 8, cg, value)
        forms["3d_coef_grad"]["traffic"] = traffic_from_profile("3d_coef_grad")
        # antisymmetrisation (every permutation weighted by its sign), slab 0
        pa = ss.spinsum_plan(slab_shape, 3, 3, [workloads.antisymmetrizer(3)], inplace=True)
        workloads.fill_uniform(big[0], 1000)
        warm(lambda: ss.spinsum_exec(pa, big[0], big[0], stream),
             refill=lambda: workloads.fill_uniform(big[0], 1000))
        ams = timed(lambda: ss.spinsum_exec(pa, big[0], big[0], stream), 5, stream)
        forms["3d_antisymmetrize"] = form_entry(2 * big[0].numel() * 8, ams, value)
        # pi_123 + pi_213 (Fig. 1b) moves two of the three axes: the plan
        # permutes those two alone (the third moves as whole 256-byte runs),
        # against the tiling under all of S_3 (SPINSUM_FLAG_FULL_GROUP)
        fig1b = [[((0, 1, 2), 1.0), (workloads.P("213"), 1.0)]]
        for name, flags in [("3d_fig1b_subgroup", 0),
                            ("3d_fig1b_full_group", ss.SPINSUM_FLAG_FULL_GROUP)]:
            pf = ss.spinsum_plan(slab_shape, 3, 3, fig1b, inplace=True, flags=flags)
            workloads.fill_uniform(big[0], 1000)
            warm(lambda: ss.spinsum_exec(pf, big[0], big[0], stream),
                 refill=lambda: workloads.fill_uniform(big[0], 1000))
            fms = timed(lambda: ss.spinsum_exec(pf, big[0], big[0], stream), 5, stream)
            forms[name] = form_entry(2 * big[0].numel() * 8, fms, value)
            forms[name]["group_axes"] = ss.spinsum_plan_get_info(pf)["exec_d"]
        # antisymmetric unpacking of slab 0 from its C(32, 3) = 4960 packed
        # values per cube, and packing back (bytes: packed + full tensor)
        pu = ss.spinsum_plan(slab_shape, 3, 3, [workloads.antisymmetrizer(3)])
        pk = workloads.uniform(ss.packed_shape(pu), 3200, device=dev)
        ubytes = (pk.numel() + big[0].numel()) * 8
        warm(lambda: ss.spinsum_unpack(pu, pk, big[0], stream))
        ums = timed(lambda: ss.spinsum_unpack(pu, pk, big[0], stream), 5, stream)
        forms["3d_unpack_antisymmetric"] = form_entry(ubytes, ums, value)
        forms["3d_unpack_antisymmetric"]["traffic"] = traffic_from_profile("3d_unpack_antisymmetric")
        warm(lambda: ss.spinsum_pack(pu, big[0], pk, stream))
        pms = timed(lambda: ss.spinsum_pack(pu, big[0], pk, stream), 5, stream)
        forms["3d_pack_antisymmetric"] = form_entry(ubytes, pms, value)
        del pk
        for name, flags in [("3d_no_nt_stores", ss.SPINSUM_FLAG_NO_NT_STORES),
                            ("3d_no_xcd_grouping", ss.SPINSUM_FLAG_NO_XCD_REMAP)]:
            pf = ss.spinsum_plan(slab_shape, 3, 3, alpha, inplace=True, flags=flags)
            workloads.fill_uniform(big[0], 1000)  # fresh values: repeated passes grow them
            warm(lambda: ss.spinsum_exec(pf, big[0], big[0], stream),
                 refill=lambda: workloads.fill_uniform(big[0], 1000))
            fms = timed(lambda: ss.spinsum_exec(pf, big[0], big[0], stream), 5, stream)
            forms[name] = form_entry(2 * big[0].numel() * 8, fms, value)
        del big
        torch.cuda.empty_cache()

        # Table II case 5 (three stages) on one 80^4 cube, in place: the same
        # three ways (one pass per stage: three passes over the tensor)
        x80 = torch.empty((80,) * 4, dtype=torch.float64, device=dev)
        st5 = workloads.table2_case(5)[1]
        for name, flags in [("4d_table2_5_80_premultiplied", 0),
                            ("4d_table2_5_80_chained", ss.SPINSUM_FLAG_CHAIN_STAGES),
                            ("4d_table2_5_80_multi_pass", ss.SPINSUM_FLAG_MULTI_PASS)]:
            pt = ss.spinsum_plan(x80.shape, 0, 4, st5, inplace=True, flags=flags)
            workloads.fill_uniform(x80, 5005)
            warm(lambda: ss.spinsum_exec(pt, x80, x80, stream),
                 refill=lambda: workloads.fill_uniform(x80, 5005))
            tms = timed(lambda: ss.spinsum_exec(pt, x80, x80, stream), 5, stream)
            forms[name] = form_entry(2 * x80.numel() * 8, tms, value)
            if name == "4d_table2_5_80_premultiplied":
                forms[name]["traffic"] = traffic_from_profile(name)
        del x80
        torch.cuda.empty_cache()

        # 4D in place, one a-slab 1 x 24^3 x 12^4, 24 random integer coefficients
        w4 = workloads.WORKLOADS["4d_v24_o12_slab"]
        x4 = workloads.uniform(w4["shape"], 2000, device=dev)
        a4 = workloads.random_4d_alpha(7)
        p4 = ss.spinsum_plan(w4["shape"], 4, 4, [a4], inplace=True)
        ss.spinsum_exec(p4, x4, x4, stream)
        warm(lambda: ss.spinsum_exec(p4, x4, x4, stream),
             refill=lambda: workloads.fill_uniform(x4, 2000))
        ms4 = timed(lambda: ss.spinsum_exec(p4, x4, x4, stream), 10, stream)
        forms["4d_v24_o12_inplace"] = form_entry(2 * x4.numel() * 8, ms4, value)
        forms["4d_v24_o12_inplace"]["tile_edge"] = ss.spinsum_plan_get_info(p4)["bl"]
        forms["4d_v24_o12_inplace"]["alpha_seed"] = 7
        forms["4d_v24_o12_inplace"]["traffic"] = traffic_from_profile("4d_v24_o12_inplace")
        # 2 - pi_2134 moves two of the four axes: the subgroup plan against S_4
        half = [[((0, 1, 2, 3), 2.0), (workloads.P("2134"), -1.0)]]
        for name, flags in [("4d_2_minus_p2134_subgroup", 0),
                            ("4d_2_minus_p2134_full_group", ss.SPINSUM_FLAG_FULL_GROUP)]:
            ph = ss.spinsum_plan(w4["shape"], 4, 4, half, inplace=True, flags=flags)
            workloads.fill_uniform(x4, 2000)
            warm(lambda: ss.spinsum_exec(ph, x4, x4, stream),
                 refill=lambda: workloads.fill_uniform(x4, 2000))
            hms = timed(lambda: ss.spinsum_exec(ph, x4, x4, stream), 10, stream)
            forms[name] = form_entry(2 * x4.numel() * 8, hms, value)
            forms[name]["group_axes"] = ss.spinsum_plan_get_info(ph)["exec_d"]
        del x4
        torch.cuda.empty_cache()

        # batched: 200 power-law blocks, one persistent launch from a hipGraph
        seed, blocks = workloads.batched_blocks()
        shapes = [(v, v, v, o, o, o) for v, o in blocks]
        xs = [workloads.uniform(s, 3000 + k, device=dev) for k, s in enumerate(shapes)]
        nbytes = 2 * 8 * sum(x.numel() for x in xs)
        bp = ss.spinsum_plan_batched(shapes, 3, alpha, inplace=True)

        def refill_blocks():
            for k, x in enumerate(xs):
                workloads.fill_uniform(x, 3000 + k)

        # item size and launch style picked by the library's autotuner
        tuned, _ = ss.spinsum_autotune(bp, xs, xs)
        graph = ss.spinsum_graph_create(bp, xs, xs)
        ss.spinsum_graph_launch(graph, stream)
        warm(lambda: ss.spinsum_graph_launch(graph, stream), refill=refill_blocks)
        bms = timed(lambda: ss.spinsum_graph_launch(graph, stream), 10, stream)
        singles = [ss.spinsum_plan(s, 3, 3, alpha, inplace=True) for s in shapes]

        def per_block():
            for p, x in zip(singles, xs):
                ss.spinsum_exec(p, x, x, stream)

        per_block()
        warm(per_block, refill=refill_blocks)
        pms = timed(per_block, 5, stream)
        forms["batched_graph"] = form_entry(nbytes, bms, value)
        forms["batched_graph"].update({"blocks": len(blocks), "block_seed": seed,
                                       "item_kib": tuned["cubes_per_wg"],
                                       "persistent": tuned["variant"],
                                       "vs_per_block_launches": round(pms / bms, 3)})
        forms["batched_graph"]["traffic"] = traffic_from_profile("batched_graph")
        forms["batched_per_block_launches"] = form_entry(nbytes, pms, value)
        del xs, graph, singles
        torch.cuda.empty_cache()

        # groups not in the last position: the slab with its group moved in
        # front of an inner spectator run of 8, [64, 64, 32, 32, 32, 8], in place
        xin = workloads.uniform((64, 64, 32, 32, 32, 8), 5000, device=dev)
        pin = ss.spinsum_plan(tuple(xin.shape), 2, 3, alpha, inplace=True)
        ss.spinsum_exec(pin, xin, xin, stream)
        warm(lambda: ss.spinsum_exec(pin, xin, xin, stream),
             refill=lambda: workloads.fill_uniform(xin, 5000))
        ims = timed(lambda: ss.spinsum_exec(pin, xin, xin, stream), 5, stream)
        forms["3d_inner_run8_inplace"] = form_entry(2 * xin.numel() * 8, ims, value)
        forms["3d_inner_run8_inplace"]["tile_edge"] = ss.spinsum_plan_get_info(pin)["bl"]
        del xin
        torch.cuda.empty_cache()
        # index-pair form T[a,b,c,i,j,k], v=48, o=24: (a,i), (b,j), (c,k)
        # permuted together, in place
        w5 = workloads.WORKLOADS["3d_v48_o24"]
        xp = workloads.uniform(w5["shape"], 5100, device=dev)
        pp = ss.spinsum_plan(w5["shape"], 3, 3, alpha, inplace=True,
                             flags=ss.SPINSUM_FLAG_INDEX_PAIRS)
        ss.spinsum_exec(pp, xp, xp, stream)
        warm(lambda: ss.spinsum_exec(pp, xp, xp, stream),
             refill=lambda: workloads.fill_uniform(xp, 5100))
        pms_ = timed(lambda: ss.spinsum_exec(pp, xp, xp, stream), 5, stream)
        forms["3d_pairs_v48_o24_inplace"] = form_entry(2 * xp.numel() * 8, pms_, value)
        forms["3d_pairs_v48_o24_inplace"]["tile_edge"] = ss.spinsum_plan_get_info(pp)["bl"]
        forms["3d_pairs_v48_o24_inplace"]["traffic"] = traffic_from_profile("3d_pairs_v48_o24_inplace")
        del xp
        torch.cuda.empty_cache()

        # adjoint and FP32: v=48, o=24, forward and backward (autograd form)
        w5 = workloads.WORKLOADS["3d_v48_o24"]
        st5 = workloads.FACTORED_PIJ_PJK
        for dt, tag in [(torch.float64, "fp64"), (torch.float32, "fp32")]:
            x5 = workloads.uniform(w5["shape"], 4000, device=dev, dtype=dt)
            y5 = torch.empty_like(x5)
            p5 = ss.spinsum_plan(w5["shape"], 3, 3, st5, dtype=dt, inplace=False)
            ss.spinsum_exec(p5, x5, y5, stream)
            warm(lambda: ss.spinsum_exec(p5, x5, y5, stream))
            fwd = timed(lambda: ss.spinsum_exec(p5, x5, y5, stream), 5, stream)
            warm(lambda: ss.spinsum_adjoint(p5, y5, x5, stream))
            bwd = timed(lambda: ss.spinsum_adjoint(p5, y5, x5, stream), 5, stream)
            nb = 2 * x5.numel() * x5.element_size()
            forms[f"3d_v48_o24_forward_{tag}"] = form_entry(nb, fwd, value)
            forms[f"3d_v48_o24_adjoint_{tag}"] = form_entry(nb, bwd, value)
            if tag == "fp64":
                forms["3d_v48_o24_forward_fp64"]["traffic"] = traffic_from_profile(
                    "3d_v48_o24_forward_fp64")
                forms["3d_v48_o24_adjoint_fp64"]["traffic"] = traffic_from_profile(
                    "3d_v48_o24_adjoint_fp64")
            else:
                forms["3d_v48_o24_forward_fp32"]["traffic"] = traffic_from_profile(
                    "3d_v48_o24_forward_fp32")
            del x5, y5
            torch.cuda.empty_cache()
        accuracy = accuracy_report(ss, workloads, dev, stream)
        # the Table II sweeps first: the forms, the accuracy figures and the
        # CPU baseline then close the line
        for size in ("small", "medium", "large"):
            log(f"table II sweep, {size}")
            out[f"table2_{size}"] = table2_sweep(ss, workloads, dev, stream, size)
        copy_gbps = forms["stream_copy_ceiling"]["GBps"]
        for f in forms.values():
            if "GBps" in f:
                f["frac_copy_ceiling"] = round(f["GBps"] / copy_gbps, 4)
        out["forms"] = forms
        out["accuracy"] = accuracy

    out["paper_context"] = PAPER_CONTEXT
    if not args.no_cpu_baseline:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds, nslabs)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
