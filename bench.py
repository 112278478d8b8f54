#!/usr/bin/env python3
"""Throughput of the co-rank stable merge on one MI355X.

A step is one pass of the whole path over one batch of synthetic input: the
block-boundary co-rank pass and the block-merge kernel of one stable merge
(cm_stable_merge_pairs).  The default workload is the single uneven merge:
m = 2**28, n = 2**26, uint32 keys drawn from 1024 distinct values with
Zipf(1.1) frequencies, each array sorted, uint32 origin payloads.  Inputs are
resident in HBM before the timed region starts.

Output: one JSON line with merged keys/s (whole job), the roofline of the
block-merge kernel (algorithmic bytes = read m + n and write m + n elements,
over its mean duration from HIP events recorded by the library on the
stream it launches on), the CPU oracle timed on the host beside it
(bit-exactness of the GPU output is checked in that leg), a small
warm-cache latency leg, the batched segmented merge against one library call
per merge on the batch workload, and the serving leg.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
METRIC = "merged keys/s & % of HBM peak; batched vs per-merge launches, bit-exact"
# sources of the merge kernels whose HBM counters are stored under profiles/
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1303_4312_amd", "csrc", f)
                  for f in ("kernels.hpp", "merge_device.hpp", "order.hpp", "dispatch.hpp",
                            "launch_impl.hpp", "launch.hip")]
COUNTERS_FILES = {
    "zipf": os.path.join(ROOT, "profiles", "k_merge_blocks_zipf_u32_pairs_counters.md"),
    "segmented": os.path.join(ROOT, "profiles", "k_seg_merge_blocks_segmented_u32_pairs_counters.md"),
    "u64": os.path.join(ROOT, "profiles", "k_merge_blocks_u64_pairs_counters.md"),
    "f32": os.path.join(ROOT, "profiles", "k_merge_blocks_f32_pairs_counters.md"),
    "a_below_b": os.path.join(ROOT, "profiles", "k_merge_blocks_a_below_b_u32_pairs_counters.md"),
    "interleaved": os.path.join(ROOT, "profiles", "k_merge_blocks_interleaved_u32_pairs_counters.md"),
    "all_equal": os.path.join(ROOT, "profiles", "k_merge_blocks_all_equal_u32_pairs_counters.md"),
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def workload_inputs(name):
    from paper_1303_4312_amd import workloads as w
    if name == "zipf":
        d = w.zipf()
        desc = ("single uneven merge m=2^28 n=2^26, uint32 keys Zipf(1.1) over 1024 values, "
                "uint32 payloads")
    elif name == "dup16":
        d = w.dup16()
        desc = "single merge m=n=2^20, uint32 keys uniform in [0,2^16), uint32 payloads"
    elif name == "u64":
        d = w.u64()
        desc = "single merge m=n=2^27, uint64 keys uniform, uint32 payloads"
    elif name == "f32":
        d = w.f32()
        desc = "single merge m=n=2^27, float32 keys N(0,1), uint32 payloads"
    elif name in ("a_below_b", "interleaved", "all_equal"):
        d = w.structured(name)
        desc = f"single merge m=n=2^27, uint32 keys, structured case {name}, uint32 payloads"
    elif name == "segmented":
        d = w.segmented()
        desc = ("segmented batch: 65536 merges, sides log-uniform in [1,2^16], uint32 keys "
                "uniform in [0,2^20) sorted per segment, uint32 payloads")
    else:
        raise SystemExit(f"unknown workload {name}")
    return d, desc


def read_traffic(workload, alg_bytes, nt, e):
    """Measured HBM bytes per launch of the workload's block-merge kernel in
    tile configuration nt x e, from the committed rocprofv3 counter summary
    of this workload, if it was taken on this kernel source; else None."""
    path = COUNTERS_FILES.get(workload)
    if path is None or not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"```json\n(.*?)\n```", text, re.S)
    if not m:
        return None
    rec = json.loads(m.group(1))
    if rec.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    if rec.get("algorithmic_bytes_per_launch") != alg_bytes:
        return None
    row = rec.get("per_config", {}).get(f"{nt}x{e}")
    return None if row is None else row["traffic_bytes_per_launch"]


def cpu_baseline_leg(d, C_gpu, Cv_gpu, seconds):
    """The oracle (plain single-threaded C merge) on the same host arrays,
    repeated until `seconds` of CPU time have passed (at least once); then
    the GPU output is compared with the oracle's byte for byte."""
    import numpy as np
    import oracle
    reps, t_total, out = 0, 0.0, None
    while reps == 0 or t_total < seconds:
        t0 = time.perf_counter()
        if "a_off" in d:
            out = oracle.stable_merge_segmented(d["A"], d["a_off"], d["B"], d["b_off"], d["Av"],
                                                d["Bv"])
        else:
            out = oracle.stable_merge(d["A"], d["B"], d["Av"], d["Bv"])
        t_total += time.perf_counter() - t0
        reps += 1
    n = d["A"].size + d["B"].size
    exact = bool(np.array_equal(out[0].view(np.uint8), C_gpu.view(np.uint8)) and
                 np.array_equal(out[1], Cv_gpu))
    cpu = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = None
    return {
        "value": n * reps / t_total,
        "unit": "keys/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"the full workload arrays ({n} outputs), merged {reps}x by the "
                   f"single-threaded oracle in {t_total:.1f} s on {cpu}"),
        "cpu_model": cpu,
        "host_cores": os.cpu_count(),
        "host_cores_usable": usable,
    }, exact


def batched_leg(steps, warmup, tune):
    """65536 independent merges, sides log-uniform in [1, 2^16]: one batched
    call (co-rank pass + one block-merge launch) against one single-merge call
    per segment; outputs compared byte for byte."""
    import numpy as np
    import torch
    import paper_1303_4312_amd as cm
    from paper_1303_4312_amd import workloads as w

    log("batched: generating 65536 segments")
    d = w.segmented()
    dev = torch.device("cuda:0")
    A, Av, B, Bv = (torch.from_numpy(d[k]).to(dev) for k in ("A", "Av", "B", "Bv"))
    a_off = torch.from_numpy(d["a_off"]).to(dev)
    b_off = torch.from_numpy(d["b_off"]).to(dev)
    n = A.numel() + B.numel()
    C = torch.empty(n, dtype=A.dtype, device=dev)
    Cv = torch.empty(n, dtype=torch.uint32, device=dev)
    ws = torch.empty(cm.segmented_workspace_size("uint32", True, A.numel(), B.numel(),
                                                 a_off.numel() - 1), dtype=torch.uint8, device=dev)
    tuned = cm.autotune_segmented(A, a_off, B, b_off, Av, Bv, reps=5) if tune else None
    if tuned is not None:
        log(f"batched: autotuned choice (config, search, partition): {tuned}")
    choice = cm.tuning_get(cm.OP_SEGMENTED, "uint32", True, n)
    for _ in range(warmup):
        cm.stable_merge_segmented(A, a_off, B, b_off, Av, Bv, C, Cv, workspace=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        cm.stable_merge_segmented(A, a_off, B, b_off, Av, Bv, C, Cv, workspace=ws)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / steps
    log(f"batched: {t_batch * 1e3:.3f} ms per batch; replaying a graph plan")
    plan = cm.plan_segmented(A, a_off, B, b_off, Av, Bv, workspace=ws)
    for _ in range(warmup):
        plan.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.launch()
    torch.cuda.synchronize()
    t_plan = (time.perf_counter() - t0) / steps
    same_plan = bool(torch.equal(plan.C, C) and torch.equal(plan.C_val, Cv))
    plan.close()
    log(f"batched: plan {t_plan * 1e3:.3f} ms per replay; running per-merge launches")
    C2 = torch.empty_like(C)
    Cv2 = torch.empty_like(Cv)
    cm.stable_merge_segmented_each(A, d["a_off"], B, d["b_off"], Av, Bv, C2, Cv2)
    torch.cuda.synchronize()
    reps = 2
    t0 = time.perf_counter()
    for _ in range(reps):
        cm.stable_merge_segmented_each(A, d["a_off"], B, d["b_off"], Av, Bv, C2, Cv2)
    torch.cuda.synchronize()
    t_each = (time.perf_counter() - t0) / reps
    same = bool(np.array_equal(C.cpu().numpy(), C2.cpu().numpy()) and
                np.array_equal(Cv.cpu().numpy(), Cv2.cpu().numpy()))
    return {
        "workload": ("65536 merges, sides log-uniform in [1,2^16], uint32 keys uniform in "
                     "[0,2^20) sorted per segment, uint32 payloads"),
        "outputs": n,
        "batched_keys_per_s": n / t_batch,
        "batched_ms": t_batch * 1e3,
        "plan_replay_ms": t_plan * 1e3,
        "plan_replay_keys_per_s": n / t_plan,
        "plan_identical_output": same_plan,
        "choice": {"config": list(cm.config_info(choice[0])), "search": choice[1],
                   "partition": choice[2], "autotuned": tuned is not None},
        "per_merge_keys_per_s": n / t_each,
        "per_merge_ms": t_each * 1e3,
        "per_merge_calls": a_off.numel() - 1,
        "per_merge_note": ("one cm_stable_merge_pairs call per merge on its sub-arrays, default "
                           "choice per size (below 2^24 outputs: one kernel launch per call)"),
        "speedup": t_each / t_batch,
        "identical_output": same,
    }


def boundary_ab_leg(A, Av, B, Bv, C, Cv, ws, stream, key_dtype, op, reps=10):
    """The boundary pass as an explicit A/B on the step's own arrays, same
    tile as the timed step: synchronised one-level (0), two-level with a
    64- or 16-lane coarse search (1, 2), and synchronisation-free (4: every
    block co-ranks its own ends).  Median per-call times from the library's
    events; the co-rank share is the boundary pass over the whole call."""
    import torch
    import paper_1303_4312_amd as cm
    N = A.numel() + B.numel()
    cls = N.bit_length()
    saved = cm.tuning_get(op, key_dtype, True, N)
    out = []
    try:
        for part in (0, 1, 2, 4):
            cm.tuning_set(op, key_dtype, True, cls, saved[0], saved[1], part)
            for _ in range(2):
                cm.stable_merge_pairs(A, Av, B, Bv, C, Cv, workspace=ws, stream=stream)
            torch.cuda.synchronize()
            cm.timing_start(reps)
            for _ in range(reps):
                cm.stable_merge_pairs(A, Av, B, Bv, C, Cv, workspace=ws, stream=stream)
            torch.cuda.synchronize()
            _, _, _, _, call_each, merge_each = cm.timing_stop(per_call=True)
            call = statistics.median(call_each)
            merge = statistics.median(merge_each)
            out.append({"partition": part,
                        "pass": ["one_level", "two_level_64", "two_level_16", "stream",
                                 "in_block"][part],
                        "call_ms": call, "merge_kernel_ms": merge,
                        "co_rank_share": (call - merge) / call})
    finally:
        cm.tuning_set(op, key_dtype, True, cls, *saved)
    return out


def partition_ablation_leg(A, Av, B, Bv, C, Cv, P=2048, reps=5):
    """The paper's claim against the classic cross-rank partition, on the
    step's own arrays: P workgroups each merge one output segment (the
    streaming kernel), the segments cut by co-ranking (equal lengths) or by
    P/2 equidistant samples of each array cross-ranked in the other.  Same
    kernel, same P; reported: merge kernel and partition times (median of
    the library's events) and the longest segment over the mean."""
    import torch
    import paper_1303_4312_amd as cm
    N = A.numel() + B.numel()
    out = {"P": P}
    ref = None
    for part, name in ((0, "co_rank"), (1, "cross_rank")):
        cm.merge_partition_ablation(A, B, Av, Bv, P=P, partition=part, C=C, C_val=Cv)
        torch.cuda.synchronize()
        cm.timing_start(reps)
        for _ in range(reps):
            _, _, bounds = cm.merge_partition_ablation(A, B, Av, Bv, P=P, partition=part, C=C,
                                                       C_val=Cv)
        torch.cuda.synchronize()
        _, _, _, _, call_each, merge_each = cm.timing_stop(per_call=True)
        b = bounds.cpu().numpy().astype("float64")
        seg = b[1:] - b[:-1]
        if ref is None:
            ref = (C.clone(), Cv.clone())
            same = True
        else:
            same = bool(torch.equal(ref[0], C) and torch.equal(ref[1], Cv))
        merge_ms = statistics.median(merge_each)
        out[name] = {"merge_kernel_ms": merge_ms,
                     "partition_ms": statistics.median(call_each) - merge_ms,
                     "longest_segment_over_mean": float(seg.max() / (N / P)),
                     "shortest_segment_over_mean": float(seg.min() / (N / P)),
                     "identical_output": same}
    out["cross_rank_over_co_rank"] = (out["cross_rank"]["merge_kernel_ms"] /
                                      out["co_rank"]["merge_kernel_ms"])
    return out


def generic_order_leg(A, Av, B, Bv, reps=10):
    """The merge under the reversed key order (the step's arrays reversed,
    CM_KEY_*_DESC) against the same merge ascending, the same keys merged
    without payloads (default tile), and the merge of the same keys carrying
    8-byte records two ways: origin codes merged and the records gathered by
    code, and the records moved by the merge itself as uint64 payloads
    (cm_stable_merge_pairs64; the two outputs must be identical).  Median
    whole-call times from the library's events; the code-and-gather path is
    timed end to end with torch events."""
    import torch
    import paper_1303_4312_amd as cm
    N = A.numel() + B.numel()
    Ad, Bd, Avd, Bvd = A.flip(0), B.flip(0), Av.flip(0), Bv.flip(0)
    C = torch.empty(N, dtype=A.dtype, device=A.device)
    Cv = torch.empty(N, dtype=torch.uint32, device=A.device)

    def calls(fn):
        fn()
        torch.cuda.synchronize()
        cm.timing_start(reps)
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        _, _, _, _, call_each, merge_each = cm.timing_stop(per_call=True)
        return statistics.median(call_each), statistics.median(merge_each)

    asc = calls(lambda: cm.stable_merge_pairs(A, Av, B, Bv, C, Cv))
    desc = calls(lambda: cm.stable_merge_pairs(Ad, Avd, Bd, Bvd, C, Cv, descending=True))
    keys = calls(lambda: cm.stable_merge(A, B, C))  # keys only: 2 K bytes per output
    Arec = torch.arange(A.numel(), dtype=torch.int64, device=A.device)
    Brec = -torch.arange(B.numel(), dtype=torch.int64, device=A.device) - 1
    cm.merge_records(A, B, Arec, Brec)
    torch.cuda.synchronize()
    ts = []
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        cm.merge_records(A, B, Arec, Brec)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    rec_ms = statistics.median(ts)
    _, Crec = cm.merge_records(A, B, Arec, Brec)
    Cn = torch.empty(N, dtype=torch.uint64, device=A.device)
    nat = calls(lambda: cm.stable_merge_pairs(A, Arec.view(torch.uint64), B, Brec.view(torch.uint64), C, Cn))
    same = bool(torch.equal(Cn.view(torch.int64), Crec.view(torch.int64)))
    del Crec, Cn
    return {
        "ascending_call_ms": asc[0], "ascending_merge_kernel_ms": asc[1],
        "descending_call_ms": desc[0], "descending_merge_kernel_ms": desc[1],
        "keys_only_call_ms": keys[0], "keys_only_merge_kernel_ms": keys[1],
        "keys_only_kernel_gbs": 2 * N * A.element_size() / (keys[1] * 1e-3) / 1e9,
        "records_8byte_ms": rec_ms,
        "records_8byte_keys_per_s": N / (rec_ms * 1e-3),
        "records_note": "codes filled, keys merged with codes, 8-byte records gathered by code",
        "records_8byte_native_call_ms": nat[0], "records_8byte_native_merge_kernel_ms": nat[1],
        "records_8byte_native_keys_per_s": N / (nat[0] * 1e-3),
        "records_8byte_native_kernel_gbs": 2 * N * (A.element_size() + 8) / (nat[1] * 1e-3) / 1e9,
        "records_8byte_native_identical": same,
        "records_native_note": "the records as uint64 payloads of the merge (cm_stable_merge_pairs64)",
    }


def sort_leg(lg=28, reps=5, seed=2024):
    """Stable merge sort (NEXT step on from the merge: merge sort's passes
    are batched co-rank merges) of 2^lg uint32 keys uniform on [0, 2^32)
    with uint32 payloads (the input position).  Beside it, the library
    reference torch.sort(stable=True) plus the payload gather, on the same
    arrays; the two results must be identical."""
    import numpy as np
    import torch
    import paper_1303_4312_amd as cm
    dev = torch.device("cuda:0")
    n = 1 << lg
    rng = np.random.default_rng(seed)
    k = torch.from_numpy(rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)).to(dev)
    v = torch.arange(n, dtype=torch.int32, device=dev)
    out = torch.empty_like(k)
    outv = torch.empty_like(v)
    ws = torch.empty(cm.sort_workspace_size("uint32", True, n), dtype=torch.uint8, device=dev)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return statistics.median(ts)

    ms = timed(lambda: cm.stable_sort(k, v.view(torch.uint32), out, outv.view(torch.uint32),
                                      workspace=ws))
    k64 = k.to(torch.int64)  # int64 keeps the uint32 order for torch.sort
    res = {}

    def ref():
        s, idx = torch.sort(k64, stable=True)
        res["k"], res["v"] = s, v[idx]

    ms_ref = timed(ref)
    same = bool(torch.equal(res["k"].to(torch.int32).view(torch.uint32), out) and
                torch.equal(res["v"], outv))
    cfg, search, _ = cm.tuning_get(cm.OP_SORT, "uint32", True, n)
    nt, e = cm.config_info(cfg)
    run = cm.sort_run_length("uint32", True, n)
    passes = 0  # runs sorted in LDS, doubled by each pass until one covers n
    while run << passes < n:
        passes += 1
    return {
        "workload": f"stable sort of 2^{lg} uint32 keys uniform on [0,2^32), uint32 payloads",
        "keys": n,
        "ms": ms,
        "keys_per_s": n / (ms * 1e-3),
        "block": {"threads": nt, "items_per_thread": e},
        "lds_run_length": run,
        "merge_passes": passes,
        "torch_sort_stable_ms": ms_ref,
        "speedup_vs_torch_sort": ms_ref / ms,
        "identical_to_torch_sort": same,
    }


def pcie_ceiling(nbytes=256 << 20, reps=10):
    """Plain pinned-host <-> device copy rates on this machine (GB/s): host to
    device alone, device to host alone, and both at once on two streams.
    The sum of the two one-way rates is the full-duplex bound the serving
    leg is measured against (the two-stream figure is only what plain
    copies reached together; a pipeline can do better)."""
    import torch
    dev = torch.device("cuda:0")
    h_in = torch.empty(nbytes, dtype=torch.uint8).pin_memory()
    h_out = torch.empty(nbytes, dtype=torch.uint8).pin_memory()
    d_in = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    d_out = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    s1, s2 = torch.cuda.Stream(dev), torch.cuda.Stream(dev)

    def run(up, down):
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            if up:
                with torch.cuda.stream(s1):
                    d_in.copy_(h_in, non_blocking=True)
            if down:
                with torch.cuda.stream(s2):
                    h_out.copy_(d_out, non_blocking=True)
        torch.cuda.synchronize()
        return (int(up) + int(down)) * reps * nbytes / (time.perf_counter() - t) / 1e9

    run(True, True)
    return {"h2d_gbs": run(True, False), "d2h_gbs": run(False, True),
            "both_ways_gbs": run(True, True), "bytes_per_copy": nbytes}


def duplex_gbs(ceiling):
    return ceiling["h2d_gbs"] + ceiling["d2h_gbs"]


def host_ingress_leg(pool_size=16, count=400, slots=16, seed=5000):
    """Serving with requests in host memory (beside the device-resident leg),
    two ways.  The runtime's own host ingress (cm_server_submit_host, the
    reported figures): each request's inputs wait in pinned host memory, the
    runtime stages them in its arena over a copy stream, merges, and copies
    the outputs back into pinned host buffers over a second copy stream.
    And a client-side copy loop (client_copy_loop): the client copies the
    inputs to one of `slots` device staging areas on its own stream and
    submits them with inputs_pending, then copies the outputs back itself.
    A request is done once its outputs are on the host.  Closed loop with
    `slots` requests in flight: requests/s, keys/s and PCIe bytes per second
    (both ways together) against the sum of the box's one-way pinned-copy
    rates (the full-duplex bound); latency from entering to outputs on the
    host.  A first pass over the pool (also
    the warm-up) checks every request's host outputs against the same merge
    run alone, byte for byte."""
    import numpy as np
    import torch
    import paper_1303_4312_amd as cm
    from paper_1303_4312_amd import serve, workloads as w
    dev = torch.device("cuda:0")
    pool, alone = [], []
    for r in range(pool_size):
        d = w.request(seed + r)
        pool.append(tuple(torch.from_numpy(d[k]).pin_memory() for k in ("A", "B", "Av", "Bv")))
        A, B, Av, Bv = (t.to(dev) for t in pool[-1])
        C, Cv = cm.stable_merge_pairs(A, Av, B, Bv)
        alone.append((C.cpu().numpy(), Cv.cpu().numpy()))
        del A, B, Av, Bv, C, Cv
    cap = max(p[0].numel() + p[1].numel() for p in pool)
    # per slot: device keys + payloads (A then B), host keys + payloads for the outputs
    stage = [(torch.empty(cap, dtype=torch.uint32, device=dev),
              torch.empty(cap, dtype=torch.uint32, device=dev)) for _ in range(slots)]
    back = [(torch.empty(cap, dtype=torch.uint32).pin_memory(),
             torch.empty(cap, dtype=torch.uint32).pin_memory()) for _ in range(slots)]
    h2d, d2h = torch.cuda.Stream(dev), torch.cuda.Stream(dev)
    srv = serve.NativeServer("uint32", True, arena_bytes=16 * cap * slots, max_batch=64,
                             max_inflight=2, max_requests=slots, device=dev)

    def run(count, check):
        free = list(range(slots))
        merging = {}   # ticket -> (request, slot, outputs, entered)
        copying = []   # (event, ticket, request, slot, outputs, entered)
        lat, done, sub, outputs, moved = [], 0, 0, 0, 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while done < count:
            while sub < count and free:
                slot = free.pop()
                A, B, Av, Bv = pool[sub % pool_size]
                m, n = A.numel(), B.numel()
                sk, sv = stage[slot]
                entered = time.perf_counter()
                with torch.cuda.stream(h2d):
                    sk[:m].copy_(A, non_blocking=True)
                    sk[m:m + n].copy_(B, non_blocking=True)
                    sv[:m].copy_(Av, non_blocking=True)
                    sv[m:m + n].copy_(Bv, non_blocking=True)
                rc = srv.submit_ptrs(sk.data_ptr(), sv.data_ptr(), m, sk.data_ptr() + 4 * m,
                                     sv.data_ptr() + 4 * m, n, h2d.cuda_stream, pending=True)
                if rc != 0:
                    raise cm.CMError(rc, "cm_server_submit")
                merging[srv.last_ticket] = (sub, slot, m + n, entered)
                moved += 8 * (m + n)
                sub += 1
            for d in srv.poll(wait_us=100 if not copying else 0):
                if d.status != 0:
                    raise cm.CMError(d.status, "serving request")
                req, slot, n_out, entered = merging.pop(d.ticket)
                C, Cv = srv.outputs(d, n_out)
                hk, hv = back[slot]
                with torch.cuda.stream(d2h):
                    hk[:n_out].copy_(C, non_blocking=True)
                    hv[:n_out].copy_(Cv, non_blocking=True)
                    ev = torch.cuda.Event()
                    ev.record(d2h)
                copying.append((ev, d.ticket, req, slot, n_out, entered))
            still = []
            for item in copying:
                ev, ticket, req, slot, n_out, entered = item
                if not ev.query():
                    still.append(item)
                    continue
                lat.append(time.perf_counter() - entered)
                if check:
                    Ce, Cve = alone[req % pool_size]
                    hk, hv = back[slot]
                    if not (np.array_equal(hk[:n_out].numpy(), Ce)
                            and np.array_equal(hv[:n_out].numpy(), Cve)):
                        raise AssertionError(f"host-ingress request {req}: outputs differ "
                                             "from the merge run alone")
                srv.release(ticket)
                free.append(slot)
                outputs += n_out
                moved += 8 * n_out
                done += 1
            copying = still
        wall = time.perf_counter() - t0
        lat.sort()

        def pick(q):
            return lat[min(len(lat) - 1, int(round(q * (len(lat) - 1))))]
        return {"requests_per_s": count / wall, "keys_per_s": outputs / wall,
                "pcie_bytes_per_s": moved / wall, "p50_ms": pick(0.5) * 1e3,
                "p99_ms": pick(0.99) * 1e3}

    run(pool_size, check=True)
    loop = run(count, check=False)
    srv.close()
    del stage

    # the runtime's own host ingress (cm_server_submit_host): it stages the
    # inputs in its arena and copies both ways on its own copy streams
    nsrv = serve.NativeServer("uint32", True, arena_bytes=20 * cap * slots, max_batch=64,
                              max_inflight=2, max_requests=slots, device=dev)

    def run_native(count, check):
        free = list(range(slots))
        info = {}  # ticket -> (request, slot, outputs, entered)
        lat, done, sub, outputs, moved = [], 0, 0, 0, 0
        t0 = time.perf_counter()
        while done < count:
            while sub < count and free:
                slot = free.pop()
                A, B, Av, Bv = pool[sub % pool_size]
                N = A.numel() + B.numel()
                hk, hv = back[slot]
                entered = time.perf_counter()
                t = nsrv.submit_host(A, B, Av, Bv, hk[:N], hv[:N])
                info[t] = (sub, slot, N, entered)
                moved += 8 * N
                sub += 1
            for d in nsrv.poll(wait_us=200):
                if d.status != 0:
                    raise cm.CMError(d.status, "serving request")
                req, slot, n_out, entered = info.pop(d.ticket)
                lat.append(time.perf_counter() - entered)
                if check:
                    Ce, Cve = alone[req % pool_size]
                    hk, hv = back[slot]
                    if not (np.array_equal(hk[:n_out].numpy(), Ce)
                            and np.array_equal(hv[:n_out].numpy(), Cve)):
                        raise AssertionError(f"host request {req}: outputs differ from the "
                                             "merge run alone")
                nsrv.release(d.ticket)
                free.append(slot)
                outputs += n_out
                moved += 8 * n_out
                done += 1
        wall = time.perf_counter() - t0
        lat.sort()

        def pick(q):
            return lat[min(len(lat) - 1, int(round(q * (len(lat) - 1))))]
        return {"requests_per_s": count / wall, "keys_per_s": outputs / wall,
                "pcie_bytes_per_s": moved / wall, "p50_ms": pick(0.5) * 1e3,
                "p99_ms": pick(0.99) * 1e3}

    run_native(pool_size, check=True)
    res = run_native(count, check=False)
    nsrv.close()
    del back
    ceiling = pcie_ceiling()
    loop["frac_of_pcie_duplex"] = loop["pcie_bytes_per_s"] / 1e9 / duplex_gbs(ceiling)
    loop["note"] = ("the client copies in and out on two streams of its own around "
                    "cm_server_submit with inputs_pending")
    res.update({
        "workload": ("the serving requests (sides log-uniform in [2^10, 2^24], uint32 key + "
                     "payload) held in pinned host memory"),
        "runtime": ("cm_server_submit_host: the runtime stages inputs in its arena over one "
                    "copy stream and returns outputs over a second"),
        "requests": count,
        "requests_in_flight": slots,
        "alone_vs_mix_checked": pool_size,
        "pcie_ceiling": ceiling,
        "frac_of_pcie_duplex": res["pcie_bytes_per_s"] / 1e9 / duplex_gbs(ceiling),
        "client_copy_loop": loop,
    })
    return res


def latency_leg(reps=200, warmup=20):
    """Small single merge, m = n = 2^20 uint32 keys uniform in [0, 2^16) with
    payloads: it fits in the Infinity Cache, so this is a warm-cache latency
    figure, not a roofline one.  Three views: back-to-back library calls on
    one stream (wall clock per call, no timing events), back-to-back replays
    of a graph plan of the same call, and the device time of one call from
    the library's HIP events (each event boundary adds a few microseconds)."""
    import torch
    import paper_1303_4312_amd as cm
    from paper_1303_4312_amd import workloads as w
    d = w.dup16()
    dev = torch.device("cuda:0")
    A, Av, B, Bv = (torch.from_numpy(d[k]).to(dev) for k in ("A", "Av", "B", "Bv"))
    N = A.numel() + B.numel()
    C = torch.empty(N, dtype=A.dtype, device=dev)
    Cv = torch.empty(N, dtype=torch.uint32, device=dev)
    ws = torch.empty(cm.merge_workspace_size("uint32", True, A.numel(), B.numel()),
                     dtype=torch.uint8, device=dev)

    def wall(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    t_call = wall(lambda: cm.stable_merge_pairs(A, Av, B, Bv, C, Cv, workspace=ws))
    plan = cm.plan_merge(A, B, Av, Bv, C, Cv, workspace=ws)
    t_plan = wall(plan.launch)
    plan.close()
    cm.timing_start(reps)
    for _ in range(reps):
        cm.stable_merge_pairs(A, Av, B, Bv, C, Cv, workspace=ws)
    torch.cuda.synchronize()
    _, _, _, _, call_each, merge_each = cm.timing_stop(per_call=True)
    cfg, search, partition = cm.tuning_get(cm.OP_MERGE, "uint32", True, N)
    return {
        "workload": "single merge m=n=2^20, uint32 keys uniform in [0,2^16), uint32 payloads "
                    "(warm cache)",
        "outputs": N,
        "choice": {"config": list(cm.config_info(cfg)), "search": search, "partition": partition},
        "wall_us_per_call": t_call * 1e6,
        "keys_per_s_back_to_back": N / t_call,
        "wall_us_per_plan_replay": t_plan * 1e6,
        "event_call_us_median": statistics.median(call_each) * 1e3,
        "event_call_us_min": min(call_each) * 1e3,
        "event_merge_kernel_us_median": statistics.median(merge_each) * 1e3,
    }


def copy_ceiling(dev, reps=20):
    """Plain-copy bandwidth of this machine: cm_copy of 1 GiB, mean of reps."""
    import torch
    import paper_1303_4312_amd as cm
    src = torch.empty(1 << 28, dtype=torch.uint32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        cm.copy(src, dst)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        cm.copy(src, dst)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2 * (1 << 30) / (ms * 1e-3) / 1e9


def tile_copy_ceiling(cfg, A, Av, B, Bv, reps=20):
    """GB/s of cm_copy_tiles in tile configuration cfg on the step's arrays:
    the block merge's own data movement (same windows-in-LDS tile structure,
    same bytes) without the merge.  None where it does not apply (keys not
    4 bytes wide, or a side's length not a multiple of 4)."""
    import torch
    import paper_1303_4312_amd as cm
    if A.element_size() != 4 or A.numel() % 4 or B.numel() % 4:
        return None
    a, b = A.view(torch.uint32), B.view(torch.uint32)
    C, Cv = cm.copy_tiles(cfg, a, Av, b, Bv)
    cm.copy_tiles(cfg, a, Av, b, Bv, C, Cv)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        cm.copy_tiles(cfg, a, Av, b, Bv, C, Cv)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del C, Cv
    torch.cuda.empty_cache()
    return 2 * (A.numel() + B.numel()) * 8 / (ms * 1e-3) / 1e9


def serving_leg(pool_size=16, per_point=1000, fractions=(0.25, 0.5, 0.75, 0.9, 1.0, 1.1),
                seed=5000, python_scheduler=True, max_batch=64, max_inflight=2):
    """Serving: requests with sides log-uniform in [2^10, 2^24] (uint32 key +
    payload, uniform keys), staged in HBM before they arrive.  The library's
    serving runtime (cm_server_*: a native scheduler thread) admits them
    against a 16 GiB output arena (the outputs half of a 32 GiB budget for
    inputs plus outputs) and batches them on the fly.  First a closed loop
    (every request at once) gives the saturation rate; then Poisson arrivals
    at fractions of it.  Latency is arrival to completion as seen by the
    scheduler.  The warm-up run checks every finished request's outputs
    against the same merge run alone, bit for bit.  The pure-Python
    scheduler's saturation rate on the same pool is reported beside it."""
    import numpy as np
    import torch
    import paper_1303_4312_amd as cm
    from paper_1303_4312_amd import serve, workloads as w

    log(f"serving: generating {pool_size} requests")
    dev = torch.device("cuda:0")
    pool = []
    for r in range(pool_size):
        d = w.request(seed + r)
        pool.append(tuple(torch.from_numpy(d[k]).to(dev) for k in ("A", "B", "Av", "Bv")))
    sizes = [p[0].numel() + p[1].numel() for p in pool]
    ptrs = [(A.data_ptr(), Av.data_ptr(), A.numel(), B.data_ptr(), Bv.data_ptr(), B.numel())
            for A, B, Av, Bv in pool]
    alone = [tuple(t.view(torch.int32) for t in cm.stable_merge_pairs(A, Av, B, Bv))
             for A, B, Av, Bv in pool]  # each request merged alone
    arena = torch.empty(16 << 30, dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()

    def run_native(arrivals, check=False):
        total = len(arrivals)
        srv = serve.NativeServer("uint32", True, arena=arena, max_batch=max_batch,
                                 max_inflight=max_inflight, max_requests=4096, device=dev)
        submit, poll, release = srv.submit_ptrs, srv.poll, srv.release
        lat, late, outputs, sub = [], {}, 0, 0
        parts = []  # per request: lateness, submit->launch, launch->end seen, device, end seen->report
        t0 = time.perf_counter()
        t_done = t0
        while len(lat) < total:
            now = time.perf_counter()
            while sub < total and t0 + arrivals[sub] <= now:
                rc = submit(*ptrs[sub % pool_size])
                if rc == -9:  # every slot taken: collect results first
                    break
                if rc != 0:
                    raise cm.CMError(rc, "cm_server_submit")
                late[srv.last_ticket] = (now - (t0 + arrivals[sub]), sub % pool_size)
                sub += 1
            wait = 200 if sub >= total else max(0, min(200, int((t0 + arrivals[sub] - now) * 1e6)))
            for d in poll(wait_us=wait):
                if d.status != 0:
                    raise cm.CMError(d.status, "serving request")
                lateness, req = late.pop(d.ticket)
                lat.append(lateness + d.latency_ns * 1e-9)
                parts.append((lateness, d.queued_ns * 1e-9, (d.ended_ns - d.queued_ns) * 1e-9,
                              d.device_ns * 1e-9, (d.latency_ns - d.ended_ns) * 1e-9))
                n_out = sizes[req]
                outputs += n_out
                if check:
                    C, Cv = srv.outputs(d, n_out)
                    if not (torch.equal(C.view(torch.int32), alone[req][0])
                            and torch.equal(Cv.view(torch.int32), alone[req][1])):
                        raise AssertionError(f"serving request {req}: outputs differ from "
                                             "the merge run alone")
                release(d.ticket)
                t_done = time.perf_counter()
        st = srv.stats()
        srv.close()
        wall = t_done - t0 - arrivals[0]
        lat.sort()

        def pick(q):
            return lat[min(len(lat) - 1, int(round(q * (len(lat) - 1))))]
        names = ("client_lateness", "submit_to_launch", "launch_to_end_seen", "batch_device",
                 "end_seen_to_report")
        breakdown = {k: statistics.median(p[x] for p in parts) * 1e3 for x, k in enumerate(names)}
        return {"keys_per_s": outputs / wall, "requests_per_s": total / wall,
                "p50_ms": pick(0.5) * 1e3, "p99_ms": pick(0.99) * 1e3,
                "mean_batch": st["submitted"] / max(st["batches"], 1),
                "gpu_busy_fraction": st["busy_ms"] / (wall * 1e3),
                # bytes moved (read and write one key and one payload per
                # output) over the time some batch was running on the GPU
                "busy_rate_gbs": outputs * 16 / (st["busy_ms"] * 1e-3) / 1e9 if st["busy_ms"] else None,
                "median_breakdown_ms": breakdown}

    run_native([0.0] * per_point, check=True)  # warm-up; every output checked
    sat = run_native([0.0] * per_point)
    sat_rate = sat["requests_per_s"]
    log(f"serving (native): saturation {sat_rate:.0f} req/s, {sat['keys_per_s'] / 1e9:.1f} "
        f"G keys/s, busy {sat['gpu_busy_fraction']:.2f} ({sat['busy_rate_gbs']:.0f} GB/s while busy)")
    rng = np.random.default_rng(seed)
    points = []
    for frac in fractions:
        lam = frac * sat_rate
        gaps = rng.exponential(1.0 / lam, per_point)
        st = run_native(list(np.cumsum(gaps) - gaps[0]))
        st.update({"rate_per_s": lam, "fraction_of_saturation": frac})
        points.append(st)
        log(f"serving (native): rate {lam:.0f}/s p50 {st['p50_ms']:.3f} ms "
            f"p99 {st['p99_ms']:.3f} ms busy {st['gpu_busy_fraction']:.2f} "
            f"({st['busy_rate_gbs']:.0f} GB/s while busy); medians (ms): "
            + ", ".join(f"{k} {v:.3f}" for k, v in st["median_breakdown_ms"].items()))
    del arena, alone
    torch.cuda.empty_cache()

    # the pure-Python scheduler (serve.Server) on the same pool, closed loop
    def run_python(count):
        ex = serve.GpuExecutor(dev)
        srv = serve.Server(ex, budget_bytes=32 << 30, max_batch=64, max_inflight=2)
        torch.cuda.synchronize()
        with srv:
            futs = [srv.submit(*pool[k % pool_size]) for k in range(count)]
            for f in futs:
                f.result(timeout=120)
        return srv.stats()

    native = {
        "workload": ("requests with sides log-uniform in [2^10,2^24], uint32 keys uniform, "
                     "uint32 payloads, device-resident"),
        "runtime": f"cm_server (native scheduler thread), 16 GiB output arena, max_batch {max_batch}, "
                   f"{max_inflight} batches in flight",
        "boundary_pass": ["one_level", "two_level_64", "two_level_16", "two_level_16",
                          "in_block"][cm.tuning_get(cm.OP_BATCH, "uint32", True, 1 << 28)[2]],
        "pool": pool_size,
        "requests_per_point": per_point,
        "alone_vs_mix_checked": per_point,
        "mean_outputs_per_request": float(np.mean(sizes)),
        "saturation": sat,
        "points": points,
    }
    if not python_scheduler:
        return native
    sys.setswitchinterval(1e-4)  # let the scheduler thread in often
    run_python(per_point)
    py = run_python(per_point)
    outputs = sum(sizes[k % pool_size] for k in range(per_point))
    log(f"serving (python scheduler): saturation "
        f"{per_point * py['keys_per_s'] / outputs:.0f} req/s")
    return {
        **native,
        "python_scheduler_saturation": {
            "requests_per_s": per_point * py["keys_per_s"] / outputs,
            "keys_per_s": py["keys_per_s"], "p50_ms": py["p50_s"] * 1e3,
            "p99_ms": py["p99_s"] * 1e3, "mean_batch": py["mean_batch"],
            "note": "serve.Server, 32 GiB budget for inputs plus outputs"},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="zipf")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuner (use the library defaults)")
    ap.add_argument("--no-copy-ceiling", action="store_true",
                    help="skip measuring this box's plain-copy bandwidth")
    ap.add_argument("--no-boundary-ab", action="store_true",
                    help="skip the A/B of boundary passes on the step's arrays")
    ap.add_argument("--no-latency", action="store_true",
                    help="skip the small warm-cache latency leg")
    ap.add_argument("--no-ablation", action="store_true",
                    help="skip the co-rank vs cross-rank partition ablation")
    ap.add_argument("--no-generic", action="store_true",
                    help="skip the descending-order and wide-record legs")
    ap.add_argument("--no-sort", action="store_true",
                    help="skip the stable merge sort leg")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the serving leg (Poisson arrivals, p50/p99)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one cm_copy of 1 GiB (for counter calibration)")
    ap.add_argument("--only-step", action="store_true",
                    help="run the timed step only (no other leg): the form profiled under "
                         "rocprofv3")
    ap.add_argument("--only-sort", action="store_true",
                    help="run the merge-sort leg only and print its record (for profiling)")
    ap.add_argument("--only-serving", action="store_true",
                    help="run the native serving leg only (saturation and the 0.25 and 1.0 "
                         "load points) and print its record (for profiling)")
    args = ap.parse_args()
    if args.only_step:
        for leg in ("cpu_baseline", "batched", "latency", "serving", "boundary_ab", "ablation",
                    "generic", "sort"):
            setattr(args, "no_" + leg, True)

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): the library "
              "has no multi-GPU path; a merge would shard by output range, each GPU "
              "co-ranking its two ends.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1303_4312_amd as cm

    if args.only_serving:
        r = serving_leg(per_point=500, fractions=(0.25, 1.0), python_scheduler=False)
        print(json.dumps({"serving": r}), flush=True)
        return

    if args.only_sort:
        if args.copy_calibration:
            src = torch.empty(1 << 28, dtype=torch.uint32, device="cuda:0")
            dst = torch.empty_like(src)
            cm.copy(src, dst)
            torch.cuda.synchronize()
            del src, dst
        r = sort_leg()
        log(f"sort: {r['ms']:.2f} ms ({r['keys_per_s'] / 1e9:.1f} G keys/s)")
        print(json.dumps({"sort": r}), flush=True)
        return

    log(f"generating workload {args.workload}")
    d, desc = workload_inputs(args.workload)
    dev = torch.device("cuda:0")
    A, Av, B, Bv = (torch.from_numpy(d[k]).to(dev) for k in ("A", "Av", "B", "Bv"))
    m, n = A.numel(), B.numel()
    N = m + n
    key_dtype = str(A.dtype).replace("torch.", "")
    key_bytes = A.element_size()
    C = torch.empty(N, dtype=A.dtype, device=dev)
    Cv = torch.empty(N, dtype=torch.uint32, device=dev)
    stream = torch.cuda.current_stream(dev)
    segmented = args.workload == "segmented"
    if segmented:  # the step is one segmented-batch call
        a_off = torch.from_numpy(d["a_off"]).to(dev)
        b_off = torch.from_numpy(d["b_off"]).to(dev)
        ws = torch.empty(max(cm.segmented_workspace_size(key_dtype, True, m, n,
                                                         a_off.numel() - 1), 1),
                         dtype=torch.uint8, device=dev)
        op = cm.OP_SEGMENTED

        def step():
            cm.stable_merge_segmented(A, a_off, B, b_off, Av, Bv, C, Cv, workspace=ws,
                                      stream=stream)

        def tune():
            return cm.autotune_segmented(A, a_off, B, b_off, Av, Bv, reps=5)
    else:  # the step is one single-merge call
        ws = torch.empty(max(cm.merge_workspace_size(key_dtype, True, m, n), 1),
                         dtype=torch.uint8, device=dev)
        op = cm.OP_MERGE

        def step():
            cm.stable_merge_pairs(A, Av, B, Bv, C, Cv, workspace=ws, stream=stream)

        def tune():
            return cm.autotune_merge(A, B, Av, Bv, reps=5)

    if args.copy_calibration:
        src = torch.empty(1 << 28, dtype=torch.uint32, device=dev)
        dst = torch.empty_like(src)
        cm.copy(src, dst)
        torch.cuda.synchronize()
        del src, dst

    copy_gbs = None
    if not args.no_copy_ceiling:
        copy_gbs = copy_ceiling(dev)
        log(f"box copy ceiling: {copy_gbs:.0f} GB/s")

    tuned = None
    if not args.no_tune:
        # off the timed path: pick the fastest configuration on this machine
        tuned = tune()
        log(f"autotuned choice (config, search, partition): {tuned}")

    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    log(f"timing {args.steps} steps")
    cm.timing_start(args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    calls, co_rank_ms, merge_ms, _, call_each, merge_each = cm.timing_stop(per_call=True)
    assert calls == args.steps
    value = N * args.steps / elapsed
    log(f"{elapsed / args.steps * 1e3:.3f} ms/step; merge kernel {merge_ms:.3f} ms, "
        f"co-rank pass {co_rank_ms:.3f} ms")

    per_elem = 2 * (key_bytes + 4)           # read + write one key and one payload
    alg_bytes = N * per_elem
    achieved = alg_bytes / (merge_ms * 1e-3) / 1e9
    cfg, search, partition = cm.tuning_get(op, key_dtype, True, N)
    nt, e = cm.config_info(cfg)
    streaming = partition == 3 and not segmented
    kernel = ("k_seg_merge_blocks" if segmented else
              "k_merge_stream" if streaming else "k_merge_blocks")
    traffic = None if streaming else read_traffic(args.workload, alg_bytes, nt, e)
    tile_gbs = None if args.no_copy_ceiling else tile_copy_ceiling(cfg, A, Av, B, Bv)
    if tile_gbs:
        log(f"tile-structure copy ceiling ({nt}x{e}): {tile_gbs:.0f} GB/s")
    result = {
        "metric": METRIC,
        "value": value,
        "unit": "keys/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"uint32": "u32", "uint64": "u64", "float32": "f32"}[key_dtype],
        "data": "synthetic",
        "config": {
            "workload": desc,
            "m": m, "n": n, "key": key_dtype, "payload": "uint32",
            "block": {"threads": nt, "items_per_thread": e},
            "search": ["algorithm1", "bisection"][search],
            "autotuned": tuned is not None,
            "boundary_pass": (["one_level", "two_level"][partition != 0] if segmented else
                              ["one_level", "two_level_64", "two_level_16", "stream",
                               "in_block"][partition]),
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel": kernel,
            "kernel_ms": merge_ms,
            "co_rank_pass_ms": co_rank_ms,
            "algorithmic_bytes_per_launch": alg_bytes,
            "box_copy_gbs": copy_gbs,
            "frac_of_box_copy": (achieved / copy_gbs) if copy_gbs else None,
            "tile_copy_gbs": tile_gbs,
            "frac_of_tile_copy": (achieved / tile_gbs) if tile_gbs else None,
            "kernel_ms_median": statistics.median(merge_each),
            "kernel_ms_min": min(merge_each),
        },
        "call_ms": {"mean": statistics.mean(call_each), "median": statistics.median(call_each),
                    "min": min(call_each), "note": "one library call, first kernel start to "
                    "block-merge end, HIP events on the call's stream"},
        "step_hbm_frac": (alg_bytes / (elapsed / args.steps)) / 1e9 / HBM_PEAK_GBS,
    }

    if not segmented and not args.no_boundary_ab:
        result["boundary_ab"] = boundary_ab_leg(A, Av, B, Bv, C, Cv, ws, stream, key_dtype, op)
        log("boundary A/B: " + ", ".join(f"{r['pass']} {r['call_ms']:.3f} ms"
                                         for r in result["boundary_ab"]))

    if not segmented and not args.no_ablation:
        result["partition_ablation"] = partition_ablation_leg(A, Av, B, Bv, C, Cv)
        pa = result["partition_ablation"]
        log(f"partition ablation (P={pa['P']}): co-rank {pa['co_rank']['merge_kernel_ms']:.3f} ms, "
            f"cross-rank {pa['cross_rank']['merge_kernel_ms']:.3f} ms, longest segment "
            f"{pa['cross_rank']['longest_segment_over_mean']:.2f} x mean")

    if not segmented and not args.no_generic:
        result["generic_order"] = generic_order_leg(A, Av, B, Bv)
        go = result["generic_order"]
        log(f"descending merge {go['descending_call_ms']:.3f} ms vs ascending "
            f"{go['ascending_call_ms']:.3f} ms; keys only {go['keys_only_call_ms']:.3f} ms "
            f"({go['keys_only_kernel_gbs']:.0f} GB/s); with 8-byte records "
            f"{go['records_8byte_ms']:.3f} ms by code and gather, "
            f"{go['records_8byte_native_call_ms']:.3f} ms as uint64 payloads "
            f"({go['records_8byte_native_kernel_gbs']:.0f} GB/s, identical: "
            f"{go['records_8byte_native_identical']})")
        torch.cuda.empty_cache()

    if not args.no_cpu_baseline:
        log("cpu baseline: oracle on the host")
        C_h = C.cpu().numpy()
        Cv_h = Cv.cpu().numpy()
        cpu, exact = cpu_baseline_leg(d, C_h, Cv_h, args.cpu_seconds)
        result["cpu_baseline"] = cpu
        result["bit_exact"] = exact
    else:
        result["cpu_baseline"] = None
        result["bit_exact"] = None

    if not args.no_latency:
        result["latency"] = latency_leg()

    if segmented:
        result["config"]["segments"] = int(d["a_off"].size - 1)

    if not args.no_sort:
        torch.cuda.empty_cache()
        result["sort"] = sort_leg()
        log(f"sort: {result['sort']['ms']:.2f} ms ({result['sort']['keys_per_s'] / 1e9:.1f} G keys/s), "
            f"torch.sort stable {result['sort']['torch_sort_stable_ms']:.2f} ms")

    if not args.no_batched:
        del A, Av, B, Bv, C, Cv, ws
        torch.cuda.empty_cache()
        result["batched"] = batched_leg(steps=max(3, min(args.steps, 20)), warmup=2,
                                        tune=not args.no_tune)

    if not args.no_serving:
        torch.cuda.empty_cache()
        result["serving"] = serving_leg()
        torch.cuda.empty_cache()
        result["serving_host_ingress"] = host_ingress_leg()
        hi = result["serving_host_ingress"]
        log(f"serving (host ingress): {hi['requests_per_s']:.0f} req/s, "
            f"{hi['pcie_bytes_per_s'] / 1e9:.1f} GB/s over PCIe "
            f"({hi['frac_of_pcie_duplex']:.2f} of the one-way pinned copy rates added, "
            f"{duplex_gbs(hi['pcie_ceiling']):.1f} GB/s), p50 {hi['p50_ms']:.2f} ms; "
            f"client copy loop {hi['client_copy_loop']['requests_per_s']:.0f} req/s")

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
