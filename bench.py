#!/usr/bin/env python3
"""Benchmark: exact node2vec walk generation on one MI355X.

Default workload (one bench "step" = both runs below, each one launch):
  Chung-Lu power-law graph, 1M nodes, 10M undirected edge samples (degree
  exponent 2.2, mean degree 20, max expected degree 5e4), uint32 weights
  uniform in [1, 100]; node2vec runs (p, q) = (1, 1) and (0.25, 4); 10 walks
  per node; 100 node slots per walk; Philox seed 42.
The graph and outputs are resident in HBM before timing starts.  Throughput
counts transitions actually taken: sum over walks of (len - 1).

Prints ONE JSON line.  Fields beyond the common contract:
  roofline      dominant kernel's algorithmic bytes per launch / its mean
                launch time (HIP events on the launch stream) vs 8 TB/s HBM
  cpu_baseline  the plain single-threaded CPU oracle run on disjoint slices of
                a bounded sample of the same walks, one slice per host thread
  kernels       per-run breakdown (mean ms, steps, algorithmic bytes)
  parity_sample the CPU-baseline sample compared with the GPU output
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "node2vec walk steps/s on 1 MI355X (plain vs batched/served); p50/p99 latency"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target CPU time of the oracle baseline sample (0 = skip)")
    ap.add_argument("--runs", default="1,1;0.25,4", help="(p,q) pairs, ';'-separated")
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--walk-len", type=int, default=100)
    ap.add_argument("--config", default="headline",
                    choices=["headline", "chung_lu_1m", "batched", "served", "big", "corpus", "ef", "gather",
                             "calibrate", "profile_batched"],
                    help="headline (default): 64 graphs x 4096 node2vec requests, batched (one hipGraph replay "
                         "per step) vs one launch per request, and served under Poisson arrivals vs one launch "
                         "per request; chung_lu_1m: plain launches on the 1M-node graph; batched / served: the "
                         "two halves of the headline alone; big: the 20M-node graph; calibrate: copy and "
                         "random-gather kernels of known size for counter calibration")
    ap.add_argument("--plain-passes", type=int, default=3, help="headline: timed one-launch-per-request passes")
    ap.add_argument("--no-served", action="store_true", help="headline: skip the served runs")
    ap.add_argument("--big-slice", type=int, default=0,
                    help="big: walks per bench step (0: every node once per step)")
    ap.add_argument("--rates", default="200,1000,5000", help="served: arrival rates (req/s)")
    ap.add_argument("--approx-k", default="100,10", help="big: sub-sample sizes of approximated node2vec runs")
    ap.add_argument("--big-scale", type=float, default=1.0,
                    help="big: scale of the graph (nodes, edge samples and max expected degree times this)")
    ap.add_argument("--big-runs", default="fo,n2v,approx", help="big: runs to take (fo, n2v, approx)")
    ap.add_argument("--big-upload-flags", type=int, default=0, help="big: n2v_graph_upload flags")
    ap.add_argument("--step-costs", action="store_true",
                    help="big: histogram of the node2vec run's second-order steps by min(d_t, d_v)")
    ap.add_argument("--window", type=int, default=5, help="corpus: SkipGram / CBOW window")
    ap.add_argument("--walklets", default="2,4", help="corpus: Walklets scales")
    ap.add_argument("--negatives", type=int, default=5, help="corpus: negatives per walk position")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (PMC counter calibration)")
    ap.add_argument("--summarize-corpus-profiles", nargs=5, metavar=("TRACE_DIR", "FETCH_DIR", "WRITE_DIR",
                                                                      "CAL_FETCH_DIR", "CAL_WRITE_DIR"),
                    help="write the corpus kernels' rocprofv3 summaries under profiles/")
    ap.add_argument("--summarize-kernel-profiles", nargs=2, metavar=("SET", "DIR"),
                    help="SET = batched, c2 or big: write that kernel's profiles/*.txt from DIR/{trace,fetch,write,sq,"
                         "tcc,cal_fetch,cal_write,cal_tcc} (rocprofv3 output of the commands they name) and exit")
    ap.add_argument("--summarize-profiles", nargs=7, metavar=("TRACE_DIR", "FETCH_DIR", "WRITE_DIR",
                                                              "CAL_FETCH_DIR", "CAL_WRITE_DIR", "SQ_DIR",
                                                              "TCC_DIR"),
                    help="write profiles/*.txt from rocprofv3 output directories and exit")
    return ap.parse_args()


def graph_cache():
    """The 1M-node Chung-Lu graph, generated once and cached on local disk."""
    import synth
    path = os.path.join(ROOT, "_cache", "chung_lu_1m_seed2.npz")
    if os.path.exists(path):
        z = np.load(path)
        return z["O"], z["D"], z["W"]
    O, D, W = synth.chung_lu_1m()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.savez(path + ".tmp.npz", O=O, D=D, W=W)
    os.replace(path + ".tmp.npz", path)
    return O, D, W


WALK_SOURCES = ("n2v_walk.hip", "n2v_device.hpp", "n2v_internal.hpp")
CORPUS_SOURCES = ("n2v_corpus.hip", "n2v_device.hpp", "n2v_internal.hpp")


def kernel_source_hash(files=WALK_SOURCES) -> str:
    """Hash of the device sources the profiled kernels are built from."""
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, "paper_2110_06196_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pmc_traffic_chung_lu_1m.txt")
TRACE_FILE = os.path.join(ROOT, "profiles", "kernel_trace_chung_lu_1m.txt")
KERNEL_OF_PATH = {"generic": "k_walk_n2v", "fo_weighted": "k_walk_lane", "return_only": "k_walk_lane"}
COPY_BYTES = 1 << 30
KERNEL_KEYS = ("k_walk_n2v", "k_walk_lane", "k_walk_queue", "k_contexts_lds", "k_contexts_global", "k_negatives",
               "k_neg_guide", "copy")
CORPUS_TRACE_FILE = os.path.join(ROOT, "profiles", "kernel_trace_corpus_chung_lu_1m.txt")
CORPUS_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pmc_traffic_corpus_chung_lu_1m.txt")


def traffic_from_profiles(kernel: str, path: str = TRAFFIC_FILE, files=WALK_SOURCES):
    """HBM bytes per launch of `kernel` from a committed rocprofv3 PMC summary,
    if it was taken on the current kernel sources (else None)."""
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"source_hash:\s*(\w+)", txt)
    if not m or m.group(1) != kernel_source_hash(files):
        return None
    m = re.search(rf"^{re.escape(kernel)}\s+hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt, re.M)
    return float(m.group(1)) if m else None


COUNTERS_FILE = os.path.join(ROOT, "profiles", "pmc_counters_chung_lu_1m.txt")


def l2_hit_from_profiles(kernel: str, path: str = COUNTERS_FILE, files=WALK_SOURCES):
    """L2 hit rate of `kernel` from the committed rocprofv3 counter summary, if
    it was taken on the current kernel sources (else None)."""
    return _profile_value(path, f"{kernel} l2_hit_rate", files)


def _csvs(d, suffix):
    import glob
    return sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))


def _pmc_per_kernel(d, counter):
    """Mean counter value per dispatch, by kernel-name key."""
    import csv
    vals = {}
    for f in _csvs(d, "counter_collection.csv"):
        for row in csv.DictReader(open(f)):
            if row.get("Counter_Name") != counter:
                continue
            name = row.get("Kernel_Name", "")
            key = next((k for k in KERNEL_KEYS if k in name.lower()), None)
            if key is None:
                key = name[:60]
            vals.setdefault((key, row.get("Dispatch_Id")), 0.0)
            vals[(key, row.get("Dispatch_Id"))] += float(row["Counter_Value"])
    per = {}
    for (key, _), v in vals.items():
        per.setdefault(key, []).append(v)
    return {k: (sum(v) / len(v), len(v)) for k, v in per.items()}


COUNTER_FILE = os.path.join(ROOT, "profiles", "pmc_counters_chung_lu_1m.txt")


def summarize_counters(sq_dir, tcc_dir, cmds):
    """Per-kernel SQ / TCC counters: instruction mix, wait share, L2 hit rate."""
    names = ["SQ_WAVES", "SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES", "SQ_WAIT_ANY", "SQ_WAIT_INST_ANY",
             "SQ_INSTS_VALU", "SQ_INSTS_VMEM_RD", "SQ_INSTS_LDS"]
    per = {n: _pmc_per_kernel(sq_dir, n) for n in names}
    hit = _pmc_per_kernel(tcc_dir, "TCC_HIT_sum")
    miss = _pmc_per_kernel(tcc_dir, "TCC_MISS_sum")
    out = ["# rocprofv3 --pmc counters per dispatch (mean over dispatches), 1M-node Chung-Lu workload",
           f"# sq command: {cmds['sq']}", f"# tcc command: {cmds['tcc']}", f"source_hash: {kernel_source_hash()}"]
    for k in ("k_walk_n2v", "k_walk_lane"):
        if k not in per["SQ_WAVES"]:
            continue
        v = {n: per[n].get(k, (0.0, 0))[0] for n in names}
        waves = max(v["SQ_WAVES"], 1.0)
        h, m = hit.get(k, (0.0, 0))[0], miss.get(k, (0.0, 0))[0]
        out.append(f"{k} " + " ".join(f"{n}: {v[n]:.6e}" for n in names) +
                   f" TCC_HIT_sum: {h:.6e} TCC_MISS_sum: {m:.6e}")
        out.append(f"{k} valu_insts_per_wave: {v['SQ_INSTS_VALU'] / waves:.1f} "
                   f"vmem_rd_insts_per_wave: {v['SQ_INSTS_VMEM_RD'] / waves:.1f} "
                   f"lds_insts_per_wave: {v['SQ_INSTS_LDS'] / waves:.1f} "
                   f"wait_any_share_of_wave_cycles: {v['SQ_WAIT_ANY'] / max(v['SQ_WAVE_CYCLES'], 1.0):.3f} "
                   f"l2_hit_rate: {h / max(h + m, 1.0):.3f}")
    open(COUNTER_FILE, "w").write("\n".join(out) + "\n")
    print(open(COUNTER_FILE).read())


def summarize_profiles(trace_dir, fetch_dir, write_dir, cal_fetch_dir, cal_write_dir, cmds,
                       trace_file=TRACE_FILE, traffic_file=TRAFFIC_FILE,
                       title="1M-node Chung-Lu node2vec workload", files=WALK_SOURCES):
    import csv
    os.makedirs(os.path.dirname(traffic_file), exist_ok=True)
    lines = [f"# rocprofv3 --kernel-trace --stats, {title}",
             f"# command: {cmds['trace']}", "# kernel | calls | total ns | average ns | min ns | max ns"]
    for f in _csvs(trace_dir, "kernel_stats.csv"):
        for row in csv.DictReader(open(f)):
            lines.append(" | ".join([row["Name"][:110], row["Calls"], row["TotalDurationNs"],
                                     row["AverageNs"], row["MinNs"], row["MaxNs"]]))
    open(trace_file, "w").write("\n".join(lines) + "\n")
    fetch = _pmc_per_kernel(fetch_dir, "FETCH_SIZE")
    write = _pmc_per_kernel(write_dir, "WRITE_SIZE")
    cf = _pmc_per_kernel(cal_fetch_dir, "FETCH_SIZE")
    cw = _pmc_per_kernel(cal_write_dir, "WRITE_SIZE")
    cal_f = max(cf.values(), key=lambda x: x[0])[0] if cf else None  # the 1 GiB copy dominates
    cal_w = max(cw.values(), key=lambda x: x[0])[0] if cw else None
    f_scale = COPY_BYTES / (cal_f * 1024.0) if cal_f else 1.0
    w_scale = COPY_BYTES / (cal_w * 1024.0) if cal_w else 1.0
    out = ["# HBM traffic per launch from two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE, KiB",
           "# per dispatch), each scaled by what the same counter reads for a plain 1 GiB copy.",
           f"# fetch command: {cmds['fetch']}", f"# write command: {cmds['write']}",
           f"# calibration commands: {cmds['cal_fetch']} ; {cmds['cal_write']}",
           f"source_hash: {kernel_source_hash(files)}",
           f"copy_fetch_KiB: {cal_f}", f"copy_write_KiB: {cal_w}",
           f"fetch_scale: {f_scale:.6f}", f"write_scale: {w_scale:.6f}"]
    for k in sorted(set(fetch) | set(write)):
        fk = fetch.get(k, (0.0, 0))[0] * 1024.0 * f_scale
        wk = write.get(k, (0.0, 0))[0] * 1024.0 * w_scale
        out.append(f"{k} fetch_bytes_per_launch: {fk:.6e} write_bytes_per_launch: {wk:.6e} "
                   f"dispatches: {fetch.get(k, (0, 0))[1]}")
        out.append(f"{k} hbm_bytes_per_launch: {fk + wk:.6e}")
    open(traffic_file, "w").write("\n".join(out) + "\n")
    print(open(trace_file).read())
    print(open(traffic_file).read())


CAL_USEFUL = 4 << 30


def bench_calibrate(args):
    """Kernels of known size for calibrating memory counters, one dispatch each,
    in this order: a plain 1 GiB device-to-device copy (torch), random 64 B
    gathers over 16 GiB (k_gather<4>), random 128 B gathers over 16 GiB
    (k_gather<8>), random 64 B gathers over 256 MiB (k_gather<4>); each gather
    dispatch reads CAL_USEFUL bytes of distinct random granules' worth of data
    (granules are hashed, so a few repeat within a dispatch)."""
    import torch
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    lib = _membench()
    st = torch.cuda.current_stream().cuda_stream
    x = torch.empty(COPY_BYTES // 4, dtype=torch.int32, device=dev)
    x.fill_(1)
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    del x, y
    sink = torch.zeros(1, dtype=torch.int64, device=dev)
    grid = torch.cuda.get_device_properties(0).multi_processor_count * 32
    done = [{"kernel": "copy", "bytes_read": COPY_BYTES, "bytes_written": COPY_BYTES}]
    for nbytes, gran in ((16 << 30, 64), (16 << 30, 128), (256 << 20, 64)):
        buf = torch.zeros(nbytes // 4, dtype=torch.int32, device=dev)
        torch.cuda.synchronize()
        n_items = CAL_USEFUL // gran
        rc = lib.n2vm_gather(buf.data_ptr(), nbytes // gran, gran, n_items, 777, sink.data_ptr(), grid, st)
        if rc != 0:
            raise RuntimeError(f"n2vm_gather failed ({rc})")
        torch.cuda.synchronize()
        done.append({"kernel": f"k_gather<{gran // 16}>", "buffer_bytes": nbytes, "granule": gran,
                     "items": n_items, "bytes_read": n_items * gran})
        del buf
    print(json.dumps({"calibration_dispatches": done}), flush=True)


def copy_calibration():
    import torch
    x = torch.empty(COPY_BYTES // 4, dtype=torch.int32, device="cuda")
    x.fill_(1)
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": COPY_BYTES, "copies": 3}))


# ---------------------------------------------------------------------------
# Gather roofline: what random reads of a given granule achieve on this GPU
# ---------------------------------------------------------------------------
def _membench():
    import ctypes
    path = os.path.join(ROOT, "paper_2110_06196_amd", "libn2vmembench.so")
    if not os.path.exists(path):
        raise RuntimeError("libn2vmembench.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    u64, vp = ctypes.c_uint64, ctypes.c_void_p
    lib.n2vm_gather.argtypes = [vp, u64, ctypes.c_uint32, u64, u64, vp, ctypes.c_int, vp]
    lib.n2vm_stream.argtypes = [vp, u64, vp, ctypes.c_int, vp]
    lib.n2vm_chase.argtypes = [vp, u64, ctypes.c_uint32, vp, vp]
    for f in (lib.n2vm_gather, lib.n2vm_stream, lib.n2vm_chase):
        f.restype = ctypes.c_int
    return lib


def _timed(torch, fn, reps=3):
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps / 1e3


def gather_bw(torch, nbytes: int, granule: int, useful_bytes: int = 4 << 30) -> float:
    """Useful GB/s of random `granule`-byte reads over a buffer of nbytes (a power of two)."""
    lib = _membench()
    dev = torch.device("cuda:0")
    buf = torch.zeros(nbytes // 4, dtype=torch.int32, device=dev)
    sink = torch.zeros(1, dtype=torch.int64, device=dev)
    grid = torch.cuda.get_device_properties(0).multi_processor_count * 32
    n_items = useful_bytes // granule
    st = torch.cuda.current_stream().cuda_stream

    def run():
        rc = lib.n2vm_gather(buf.data_ptr(), nbytes // granule, granule, n_items, 12345, sink.data_ptr(), grid, st)
        if rc != 0:
            raise RuntimeError(f"n2vm_gather failed ({rc})")
    t = _timed(torch, run)
    del buf
    return n_items * granule / t / 1e9


def bench_gather(args):
    """Random-gather bandwidth at 4/16/64/128 B over buffers resident in L2
    (2 MiB), MALL (128 MiB) and HBM (16 GiB); streaming read of 16 GiB; and
    single-lane pointer-chase latency over 2 MiB, 128 MiB and 1 GiB."""
    import torch
    dev = torch.device("cuda:0")
    lib = _membench()
    st = torch.cuda.current_stream().cuda_stream
    rows = []
    for where, nbytes in (("L2", 2 << 20), ("MALL", 128 << 20), ("HBM", 16 << 30)):
        for gran in (4, 16, 64, 128):
            bw = gather_bw(torch, nbytes, gran)
            rows.append({"buffer": where, "bytes": nbytes, "granule": gran, "useful_GBps": bw})
            print(f"[bench] gather {where} {gran} B: {bw:.1f} GB/s", file=sys.stderr, flush=True)
    buf = torch.zeros((16 << 30) // 4, dtype=torch.int32, device=dev)
    sink = torch.zeros(1, dtype=torch.int64, device=dev)
    grid = torch.cuda.get_device_properties(0).multi_processor_count * 32
    t = _timed(torch, lambda: lib.n2vm_stream(buf.data_ptr(), 16 << 30, sink.data_ptr(), grid, st))
    stream_bw = (16 << 30) / t / 1e9
    del buf
    lat = []
    rng = np.random.default_rng(5)
    for where, n in (("L2", (2 << 20) // 4), ("MALL", (128 << 20) // 4), ("HBM", (1 << 30) // 4)):
        perm = rng.permutation(n).astype(np.uint32)
        nxt = np.empty(n, dtype=np.uint32)
        nxt[perm] = np.roll(perm, -1)  # one cycle through every slot
        d_next = torch.from_numpy(nxt.view(np.int32)).to(dev)
        hops = 100000
        t = _timed(torch, lambda: lib.n2vm_chase(d_next.data_ptr(), hops, int(perm[0]), sink.data_ptr(), st), reps=2)
        lat.append({"buffer": where, "bytes": n * 4, "ns_per_hop": t / hops * 1e9})
        del d_next
    out = {"metric": "memory-system probes (gather roofline)", "value": rows[-4]["useful_GBps"],
           "unit": "GB/s (random 4 B over 16 GiB)", "n_gpus": 1, "steps": 3, "warmup": 1,
           "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
           "data": "synthetic", "config": {"workload": "random gathers / streaming read / pointer chase"},
           "gather": rows, "stream_read_GBps": stream_bw, "chase": lat}
    print(json.dumps(out), flush=True)


def _clog2p1(x, torch):
    """ceil(log2(x + 1)) elementwise for int64 x >= 0."""
    return torch.ceil(torch.log2((x + 1).to(torch.float64))).to(torch.int64)


def algorithmic_bytes(torch, Y, lens, deg, variant: str, lists: bool = False) -> tuple[int, int]:
    """(steps, bytes) the implemented method reads and writes for the walks in Y,
    counting 4 bytes per 32-bit element touched (cache effects ignored).

    Every transition from v (degree d_v): offsets of v 16 B, output slot 4 B,
    selected destination 4 B.  Then
      first order, weighted (also node2vec p = q = 1 and the first step of
      every node2vec walk): ceil(log2(d_v + 1)) prefix probes of 4 B;
      node2vec with 1/q != 1, later steps (previous node t, degree d_t): the row
      sum 4 B, the return weight 4 B, the cheapest classification route
        probe:  N(t) 4 d_t + d_t bisections into N(v), 4 ceil(log2(d_v + 1)) each
        stream: N(v) 4 d_v + d_v bisections into N(t), 4 ceil(log2(d_t + 1)) each
        merge:  both rows once, 4 d_v + 4 d_t
      and the final search over the prefix, 4 ceil(log2(d_v + 1));
      with stored edge lists (lists=True) the step may instead read the edge's
      list record, 16 B, and search the stored list: counted as the record
      alone (a lower bound), so a step costs the cheaper of that and the routes.
      (Weights and prefix entries of common neighbours, a few per step, and
      reuse of N(t) from LDS are not counted.)
    """
    steps = int((lens.to(torch.int64) - 1).clamp(min=0).sum().item())
    total = 0
    chunk = 1 << 19
    for r0 in range(0, Y.shape[0], chunk):
        y = Y[r0:r0 + chunk]
        taken = (y[:, 1:] >= 0)
        dv = deg[y[:, :-1].clamp(min=0).to(torch.int64)]
        lv = _clog2p1(dv, torch)
        b = 24 + 4 * lv
        if variant == "generic":
            dt = deg[y[:, :-2].clamp(min=0).to(torch.int64)]
            dv2 = dv[:, 1:]
            lv2 = lv[:, 1:]
            probe = 4 * dt + 4 * dt * lv2
            stream = 4 * dv2 + 4 * dv2 * _clog2p1(dt, torch)
            merge = 4 * dv2 + 4 * dt
            route = torch.minimum(torch.minimum(probe, stream), merge)
            if lists:
                route = torch.clamp(route, max=16)
            b2 = 24 + 8 + route + 4 * lv2
            b = torch.cat([b[:, :1], b2], dim=1)
        total += int((b * taken).sum().item())
    return steps, total


def main():
    args = parse()
    if args.summarize_profiles:
        t = "cd /tmp && rocprofv3 --kernel-trace --stats --output-format csv -d <dir> -o run -- " \
            "python3 /root/repo/bench.py --steps 2 --warmup 0 --cpu-seconds 0"
        f = "cd /tmp && rocprofv3 --pmc {c} --output-format csv -d <dir> -o run -- " \
            "python3 /root/repo/bench.py --steps 1 --warmup 0 --cpu-seconds 0"
        c = "cd /tmp && rocprofv3 --pmc {c} --output-format csv -d <dir> -o run -- " \
            "python3 /root/repo/bench.py --copy-calibration"
        summarize_profiles(*args.summarize_profiles[:5], cmds={
            "trace": t, "fetch": f.format(c="FETCH_SIZE"), "write": f.format(c="WRITE_SIZE"),
            "cal_fetch": c.format(c="FETCH_SIZE"), "cal_write": c.format(c="WRITE_SIZE")})
        summarize_counters(*args.summarize_profiles[5:], cmds={
            "sq": f.format(c="SQ_WAVES SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_WAIT_ANY SQ_WAIT_INST_ANY SQ_INSTS_VALU "
                           "SQ_INSTS_VMEM_RD SQ_INSTS_LDS"),
            "tcc": f.format(c="TCC_HIT_sum TCC_MISS_sum")})
        return
    if args.summarize_corpus_profiles:
        base = "cd /tmp && rocprofv3 {what} --output-format csv -d <dir> -o run -- " \
               "python3 /root/repo/bench.py --config corpus{extra} --steps {k} --warmup 0 --cpu-seconds 0"
        c = "cd /tmp && rocprofv3 --pmc {c} --output-format csv -d <dir> -o run -- " \
            "python3 /root/repo/bench.py --copy-calibration"
        summarize_profiles(*args.summarize_corpus_profiles, cmds={
            "trace": base.format(what="--kernel-trace --stats", k=2, extra=""),
            "fetch": base.format(what="--pmc FETCH_SIZE", k=1, extra=" --walklets ''"),
            "write": base.format(what="--pmc WRITE_SIZE", k=1, extra=" --walklets ''"),
            "cal_fetch": c.format(c="FETCH_SIZE"), "cal_write": c.format(c="WRITE_SIZE")},
            trace_file=CORPUS_TRACE_FILE, traffic_file=CORPUS_TRAFFIC_FILE,
            title="training corpora of the 1M-node Chung-Lu walks", files=CORPUS_SOURCES)
        return
    if args.summarize_kernel_profiles:
        summarize_kernel_profiles(*args.summarize_kernel_profiles)
        return
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.config == "headline":
        bench_headline(args)
        return
    if args.config == "calibrate":
        bench_calibrate(args)
        return
    if args.config == "profile_batched":
        bench_profile_batched(args)
        return
    if args.config == "batched":
        bench_batched(args)
        return
    if args.config == "served":
        bench_served(args)
        return
    if args.config == "big":
        bench_big(args)
        return
    if args.config == "corpus":
        bench_corpus(args)
        return
    if args.config == "ef":
        bench_ef(args)
        return
    if args.config == "gather":
        bench_gather(args)
        return
    import torch
    import paper_2110_06196_amd as n2v

    assert torch.cuda.is_available(), "bench needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.time()
    O, D, W = graph_cache()
    n = len(O) - 1
    print(f"[bench] graph n={n} m={D.size} gen/load {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    Ot = torch.from_numpy(O.view(np.int64)).to(dev)
    Dt = torch.from_numpy(D).to(dev)
    Wt = torch.from_numpy(W.view(np.int32)).to(dev)
    torch.cuda.synchronize()
    t_up = time.perf_counter()
    g = n2v.n2v_graph_upload(Ot, Dt, Wt)
    torch.cuda.synchronize()
    prep_s = time.perf_counter() - t_up
    info = n2v.n2v_graph_info(g)
    print(f"[bench] graph prep {prep_s:.2f}s, {info['pair_lists']} edge lists, {info['pair_entries']} entries",
          file=sys.stderr, flush=True)
    deg = (Ot[1:] - Ot[:-1]).to(torch.int64)
    starts_np = np.arange(n, dtype=np.int32)
    S = torch.from_numpy(starts_np).to(dev)
    runs = [tuple(float(x) for x in r.split(",")) for r in args.runs.split(";")]
    R, L, seed = args.reps, args.walk_len, 42
    nw = n * R
    outs = [(torch.empty((nw, L), dtype=torch.int32, device=dev),
             torch.empty(nw, dtype=torch.int32, device=dev)) for _ in runs]
    stream = torch.cuda.current_stream()

    def one_step(events=None):
        for i, (p, q) in enumerate(runs):
            Y, lens = outs[i]
            if events is not None:
                events[i][0].record(stream)
            n2v.n2v_walks_node2vec(g, S, R, L, p, q, seed, 0, Y, lens, stream=stream)
            if events is not None:
                events[i][1].record(stream)

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    print(f"[bench] warmup done", file=sys.stderr, flush=True)
    ev = [[[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)] for _ in runs]
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        one_step(ev[k])
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    print(f"[bench] timed {args.steps} steps in {t_total:.3f}s", file=sys.stderr, flush=True)

    kernels = []
    total_steps = 0
    for i, (p, q) in enumerate(runs):
        Y, lens = outs[i]
        ms = float(np.mean([ev[k][i][0].elapsed_time(ev[k][i][1]) for k in range(args.steps)]))
        variant = "fo_weighted" if (p == 1.0 and q == 1.0) else ("return_only" if q == 1.0 else "generic")
        steps, alg = algorithmic_bytes(torch, Y, lens, deg, "generic" if variant == "generic" else "fo_weighted",
                                       lists=info["pair_lists"] > 0)
        total_steps += steps
        kernels.append({"p": p, "q": q, "path": variant, "mean_ms": ms, "steps": steps,
                        "alg_bytes": alg, "steps_per_s": steps / (ms / 1e3),
                        "alg_GBps": alg / (ms / 1e3) / 1e9})
    dom = max(kernels, key=lambda k: k["mean_ms"])
    traffic = traffic_from_profiles(KERNEL_OF_PATH[dom["path"]])
    value = total_steps * args.steps / t_total
    # measured gather roofline at the size of what the walks read (offsets,
    # destinations, weights, row prefix), rounded up to a power of two
    ws = O.nbytes + D.nbytes + W.nbytes + D.size * max(1, info["prefix_bytes"])
    ws2 = 1 << int(np.ceil(np.log2(ws)))
    g4, g64 = gather_bw(torch, ws2, 4), gather_bw(torch, ws2, 64)
    print(f"[bench] gather roofline over {ws2} B: 4 B {g4:.0f} GB/s, 64 B {g64:.0f} GB/s", file=sys.stderr, flush=True)

    # CPU baseline: the oracle on an evenly spaced sample of the same walks.
    cpu = None
    parity = None
    if args.cpu_seconds > 0:
        import oracle
        threads = min(16, os.cpu_count() or 1)
        probe = np.arange(0, nw, max(1, nw // 256), dtype=np.int64)
        t1 = time.perf_counter()
        for (p, q) in runs:
            oracle.walks_threaded(O, D, W, starts_np, R, L, oracle.NODE2VEC, p, q, seed, 0, probe, threads)
        per_walk = (time.perf_counter() - t1) / (len(runs) * probe.size) * threads
        k = int(max(threads, min(nw, args.cpu_seconds * threads / max(per_walk, 1e-9) / len(runs))))
        rows = np.linspace(0, nw - 1, k).astype(np.int64)
        t2 = time.perf_counter()
        csteps = 0
        mism = 0
        for i, (p, q) in enumerate(runs):
            Yo, lo = oracle.walks_threaded(O, D, W, starts_np, R, L, oracle.NODE2VEC, p, q, seed, 0, rows,
                                           threads)
            csteps += int(np.maximum(lo.astype(np.int64) - 1, 0).sum())
            idx = torch.from_numpy(rows).to(dev)
            Yg = outs[i][0].index_select(0, idx).cpu().numpy()
            lg = outs[i][1].index_select(0, idx).cpu().numpy()
            mism += int(((Yg != Yo).any(axis=1) | (lg != lo)).sum())
        tc = time.perf_counter() - t2
        cpu = {"value": csteps / tc, "unit": "walk steps/s", "cores": threads, "kind": "oracle",
               "sample": f"{k} evenly spaced walk rows of each of the {len(runs)} runs "
                         f"({csteps} steps, {tc:.1f} s wall)"}
        parity = {"rows_per_run": int(k), "mismatching_rows": mism}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "walk steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_total / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {
            "workload": "plain node2vec, Chung-Lu 1M nodes / 10M undirected edge samples "
                        "(gamma 2.2, mean deg 20, max expected deg 5e4), weights U[1,100]; "
                        f"runs (p,q) = {runs}; {R} walks per node; {L} slots; seed 42",
            "form": "plain (one launch per request)",
            "n_nodes": n, "n_entries": int(D.size), "max_degree": info["max_degree"],
            "stationary_mean_degree": info["sum_deg_sq"] / max(1, info["n_entries"]),
            "graph_prep": {"seconds": prep_s, "device_bytes": info["device_bytes"], "edge_lists": info["pair_lists"],
                           "list_entries": info["pair_entries"],
                           "note": "upload, outside the timed region: validation, weight prefix, node records, "
                                   "prefix heads and the stored common-neighbour list of every edge"},
        },
        "roofline": {
            "bound": "hbm",
            "achieved": dom["alg_GBps"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": dom["alg_GBps"] / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel": f"node2vec p={dom['p']:g} q={dom['q']:g} ({dom['path']})",
            "note": "achieved = algorithmic bytes (a lower bound with stored edge lists) / kernel time; the "
                    "kernel reads whole cache lines at random (its measured HBM rate, measured_hbm_GBps, is "
                    "far above the algorithmic rate), so line-granular traffic and dependent-load latency "
                    "bound it, not the algorithmic bytes",
            "measured_hbm_GBps": (traffic / (dom["mean_ms"] / 1e3) / 1e9) if traffic else None,
        },
        "gather_roofline": {
            "buffer_bytes": ws2, "random_4B_GBps": g4, "random_64B_GBps": g64,
            "kernel_fetch_GBps": (traffic / (dom["mean_ms"] / 1e3) / 1e9) if traffic else None,
            "kernel_l2_hit_rate": l2_hit_from_profiles(KERNEL_OF_PATH[dom["path"]]),
            "note": "useful GB/s of random 4 B / 64 B reads over a buffer the size of the graph arrays, measured "
                    "in this run, beside the dominant kernel's measured HBM traffic rate (committed PMC profile)",
        },
        "cpu_baseline": cpu,
        "kernels": kernels,
        "parity_sample": parity,
        "kernel_source_hash": kernel_source_hash(),
    }
    print(json.dumps(out), flush=True)
    n2v.n2v_graph_release(g)


# ---------------------------------------------------------------------------
# Many graphs, many requests
# ---------------------------------------------------------------------------
def many_graphs_on_device(torch, n2v, dev):
    import synth
    t0 = time.time()
    ps, host = synth.many_graphs(threads=min(16, os.cpu_count() or 1))
    print(f"[bench] 64 graphs generated in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    graphs = []
    for (O, D, W) in host:
        Ot = torch.from_numpy(O.view(np.int64)).to(dev)
        Dt = torch.from_numpy(D).to(dev)
        Wt = torch.from_numpy(W.view(np.int32)).to(dev)
        graphs.append((n2v.n2v_graph_upload(Ot, Dt, Wt), (Ot, Dt, Wt)))
    return ps, host, graphs


def _requests_on_device(torch, dev, reqs):
    bufs = []
    for r in reqs:
        S = torch.from_numpy(r["starts"]).to(dev)
        nw = r["starts"].size
        bufs.append((S, torch.empty((nw, r["walk_len"]), dtype=torch.int32, device=dev),
                     torch.empty(nw, dtype=torch.int32, device=dev)))
    return bufs


def _oracle_sample(host, reqs, per_req, threads, outs=None, torch=None):
    """Oracle on `per_req` evenly spaced walks of every request; returns
    (steps, seconds, mismatching rows vs outs)."""
    import concurrent.futures as cf
    import oracle
    jobs = []
    for k, r in enumerate(reqs):
        nw = r["starts"].size
        rows = np.unique(np.linspace(0, nw - 1, min(per_req, nw)).astype(np.int64))
        jobs.append((k, rows))

    def one(job):
        k, rows = job
        r = reqs[k]
        O, D, W = host[r["graph"]]
        return k, rows, oracle.walks(O, D, W, r["starts"], 1, r["walk_len"], oracle.NODE2VEC, r["p"], r["q"],
                                     r["seed"], 0, rows)

    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(threads) as ex:
        res = list(ex.map(one, jobs))
    dt = time.perf_counter() - t0
    steps = sum(int(np.maximum(lo.astype(np.int64) - 1, 0).sum()) for _, _, (_, lo) in res)
    mism = 0
    if outs is not None:
        for k, rows, (Yo, lo) in res:
            idx = torch.from_numpy(rows).to(outs[k][1].device)
            Yg = outs[k][1].index_select(0, idx).cpu().numpy()
            lg = outs[k][2].index_select(0, idx).cpu().numpy()
            mism += int(((Yg != Yo).any(axis=1) | (lg != lo)).sum())
    return steps, dt, mism


def section8d_bytes(torch, Y, lens, deg, variant: str) -> tuple[int, int]:
    """(steps, bytes) of the walks in Y by the per-step byte figures of the
    method's statement (4 bytes per 32-bit element the step must touch, cache
    effects ignored), for the variant that ran; d_v is the degree of the node
    a step leaves:
      first order, weighted (also node2vec p = q = 1 and the first step of
      every node2vec walk): offsets 16 + ceil(log2(d_v + 1)) prefix probes of 4
        + destination 4 + output 4;
      node2vec with 1/q == 1 (return bias only): offsets 16 + a bisection for t
        and one over the prefix, 4 ceil(log2(d_v + 1)) each, + weight of t 4
        + destination 4 + output 4;
      node2vec with 1/q != 1: offsets 16 + the row's destinations and weights,
        8 d_v, + output 4 (the streaming statement of the step)."""
    steps = int((lens.to(torch.int64) - 1).clamp(min=0).sum().item())
    if Y.shape[1] < 2 or steps == 0:
        return steps, 0
    total = 0
    chunk = 1 << 19
    for r0 in range(0, Y.shape[0], chunk):
        y = Y[r0:r0 + chunk]
        taken = (y[:, 1:] >= 0)
        dv = deg[y[:, :-1].clamp(min=0).to(torch.int64)]
        fo = 24 + 4 * _clog2p1(dv, torch)
        if variant == "fo_weighted":
            b = fo
        elif variant == "return_only":
            b = torch.cat([fo[:, :1], 28 + 8 * _clog2p1(dv[:, 1:], torch)], dim=1)
        else:
            b = torch.cat([fo[:, :1], 20 + 8 * dv[:, 1:]], dim=1)
        total += int((b * taken).sum().item())
    return steps, total


def variant_of(p: float, q: float) -> str:
    """Kernel family of a node2vec request (the eight specialisations fold
    into three families on weighted graphs)."""
    if q == 1.0:
        return "fo_weighted" if p == 1.0 else "return_only"
    return "generic"


def _fetch_rows(n2v, res, L, rows):
    """Rows of a finished served request (server-owned device memory) on the host."""
    Y = np.empty((rows.size, L), dtype=np.int32)
    lens = np.empty(rows.size, dtype=np.int32)
    hip = n2v._hip()
    for i, r in enumerate(rows.tolist()):
        rc = hip.hipMemcpy(Y[i].ctypes.data, int(res.d_walks) + r * L * 4, L * 4, 2)
        rc |= hip.hipMemcpy(lens.ctypes.data + 4 * i, int(res.d_lens) + r * 4, 4, 2)
        if rc != 0:
            raise RuntimeError("hipMemcpy of a served result failed")
    return Y, lens


def _serve_rate(torch, n2v, graphs, reqs, hdesc, rate, plain_bufs, stream, rows):
    """One open-loop Poisson run (seed 11) at `rate` req/s through the server
    (continuous batching, 200 GB budget), then the same schedule as one plain
    launch per request on one stream.  Latency = done - scheduled arrival; the
    first 5% of arrivals are excluded from the percentiles.  Returns the rate's
    record and the served walks at `rows` of every request."""
    import threading
    import synth
    skip = len(reqs) // 20
    arr = synth.poisson_arrivals(len(reqs), rate)

    def pct(lat):
        lat = np.sort(np.asarray(lat[skip:], dtype=np.float64)) / 1e6
        return float(lat[int(0.5 * (lat.size - 1))]), float(lat[int(np.ceil(0.99 * (lat.size - 1)))])

    def wait_until(t_ns):
        while True:
            d = t_ns - time.monotonic_ns()
            if d <= 0:
                return
            if d > 2_000_000:
                time.sleep((d - 1_000_000) / 1e9)

    srv = n2v.n2v_server_create(200 << 30, 4096)
    for g in graphs:
        n2v.n2v_server_add_graph(srv, g)
    ids = [0] * len(reqs)
    res_of = [None] * len(reqs)
    submitted = [0]
    t0 = time.monotonic_ns() + 20_000_000

    def poller():
        pending, seen, left = set(), 0, len(reqs)
        while left:
            upto = submitted[0]
            pending.update(range(seen, upto))
            seen = upto
            for k in list(pending):
                res = n2v.n2v_request_poll(srv, ids[k])
                if res is not None:
                    res_of[k] = res
                    pending.discard(k)
                    left -= 1
            time.sleep(0.0002)

    th = threading.Thread(target=poller)
    th.start()
    for k in range(len(reqs)):
        ta = t0 + int(arr[k] * 1e9)
        wait_until(ta)
        ids[k] = n2v.n2v_request_submit(srv, hdesc[k], ta)
        submitted[0] = k + 1
    th.join()
    lat = [r.t_done_ns - r.t_arrival_ns for r in res_of]
    s_steps = sum(int(r.steps) for r in res_of)
    s_tput = s_steps / ((max(r.t_done_ns for r in res_of) - t0) / 1e9)
    s50, s99 = pct(lat)
    served_rows = [_fetch_rows(n2v, res_of[k], reqs[k]["walk_len"], rows[k]) for k in range(len(reqs))]
    for k in range(len(reqs)):
        n2v.n2v_request_release(srv, ids[k])
    n2v.n2v_server_destroy(srv)
    print(f"[bench] served {rate:g} req/s: p50 {s50:.1f} ms p99 {s99:.1f} ms, {s_tput:.3e} steps/s",
          file=sys.stderr, flush=True)
    # baseline: one plain launch per request, FIFO, one stream, same schedule
    events = [None] * len(reqs)
    blat = [0] * len(reqs)
    bdone = [0] * len(reqs)
    launched = [0]
    t0 = time.monotonic_ns() + 20_000_000

    def bpoller():
        k = 0
        while k < len(reqs):
            if k >= launched[0]:
                time.sleep(0.0001)
                continue
            if events[k].query():
                now = time.monotonic_ns()
                bdone[k] = now
                blat[k] = now - (t0 + int(arr[k] * 1e9))
                k += 1
            else:
                time.sleep(0.00005)

    th = threading.Thread(target=bpoller)
    th.start()
    for k, (r, (S, Y, lens)) in enumerate(zip(reqs, plain_bufs)):
        wait_until(t0 + int(arr[k] * 1e9))
        n2v.n2v_walks_node2vec(graphs[r["graph"]], S, 1, r["walk_len"], r["p"], r["q"], r["seed"], 0, Y, lens,
                               stream=stream)
        e = torch.cuda.Event()
        e.record(stream)
        events[k] = e
        launched[0] = k + 1
    th.join()
    b50, b99 = pct(blat)
    b_steps = sum(int((l.to(torch.int64) - 1).clamp(min=0).sum().item()) for _, _, l in plain_bufs)
    b_tput = b_steps / ((max(bdone) - t0) / 1e9)
    print(f"[bench] one launch per request {rate:g} req/s: p50 {b50:.1f} ms p99 {b99:.1f} ms, {b_tput:.3e} steps/s",
          file=sys.stderr, flush=True)
    rec = {"rate_rps": rate, "arrival_span_s": float(arr[-1]),
           "served": {"steps_per_s": s_tput, "p50_ms": s50, "p99_ms": s99},
           "one_launch_per_request": {"steps_per_s": b_tput, "p50_ms": b50, "p99_ms": b99},
           "steps": s_steps, "steps_match": s_steps == b_steps}
    return rec, served_rows


SECTOR_FILE = os.path.join(ROOT, "profiles", "pmc_sectors_batched_64_graphs.txt")
BATCHED_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pmc_traffic_batched_64_graphs.txt")
BATCHED_TRACE_FILE = os.path.join(ROOT, "profiles", "kernel_trace_batched_64_graphs.txt")
BATCHED_COUNTERS_FILE = os.path.join(ROOT, "profiles", "pmc_counters_batched_64_graphs.txt")


def _profile_value(path: str, key: str, files=WALK_SOURCES):
    """A `key: value` figure of a committed profile summary taken on the current
    kernel sources (else None)."""
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"source_hash:\s*(\w+)", txt)
    if not m or m.group(1) != kernel_source_hash(files):
        return None
    m = re.search(rf"{re.escape(key)}:\s*([0-9.eE+-]+)", txt)
    return float(m.group(1)) if m else None


def bench_profile_batched(args):
    """The headline's batched half alone, for rocprofv3: the 64 graphs, the
    4096 requests, the plan (autotuned as in the headline), `--warmup` then
    `--steps` replays, and nothing after them, so the last `--steps`
    k_walk_queue dispatches of a profile of this command are the timed
    replays."""
    import torch
    import paper_2110_06196_amd as n2v
    import synth
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log = lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True)  # noqa: E731
    ps, host = synth.many_graphs(threads=min(16, os.cpu_count() or 1))
    log("64 graphs generated")
    keep, graphs = [], []
    for (O, D, W) in host:
        t = (torch.from_numpy(O.view(np.int64)).to(dev), torch.from_numpy(D).to(dev),
             torch.from_numpy(W.view(np.int32)).to(dev))
        keep.append(t)
        graphs.append(n2v.n2v_graph_upload(*t))
    log("64 graphs uploaded")
    reqs = synth.many_requests([p["n"] for p in ps])
    out = _requests_on_device(torch, dev, reqs)
    descs = [n2v.make_request(graphs[r["graph"]], n2v.N2V_NODE2VEC, S, 1, r["walk_len"], r["p"], r["q"],
                              r["seed"], 0, Y, lens) for r, (S, Y, lens) in zip(reqs, out)]
    plan = n2v.n2v_batch_create(descs, autotune=True)
    info = n2v.n2v_batch_info(plan)
    log(f"plan created, shape {info['lanes_per_walker']}/{info['lds_tile']}/{info['list_cap']}")
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        n2v.n2v_batch_launch(plan, stream)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for e0, e1 in ev:
        e0.record(stream)
        n2v.n2v_batch_launch(plan, stream)
        e1.record(stream)
    torch.cuda.synchronize()
    steps = sum(int((lens.to(torch.int64) - 1).clamp(min=0).sum().item()) for _, _, lens in out)
    print(json.dumps({"profile": "batched", "replays": args.steps, "steps_per_replay": steps,
                      "kernel_ms": [a.elapsed_time(b) for a, b in ev],
                      "shape": [int(info["lanes_per_walker"]), int(info["lds_tile"]), int(info["list_cap"])],
                      "kernel_source_hash": kernel_source_hash()}), flush=True)
    n2v.n2v_batch_destroy(plan)
    for g in graphs:
        n2v.n2v_graph_release(g)


def _dispatches(d):
    """Per-dispatch rows of every rocprofv3 CSV under d, in dispatch order:
    [(dispatch id, kernel name, {counter: value} or {"ns": duration})]."""
    import csv
    rows = {}
    for f in _csvs(d, "counter_collection.csv"):
        for r in csv.DictReader(open(f)):
            k = int(r["Dispatch_Id"])
            rec = rows.setdefault(k, (r.get("Kernel_Name", ""), {}))
            rec[1][r["Counter_Name"]] = rec[1].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    for f in _csvs(d, "kernel_trace.csv"):
        for r in csv.DictReader(open(f)):
            k = int(r["Dispatch_Id"])
            rows[k] = (r.get("Kernel_Name", ""), {"ns": float(r["End_Timestamp"]) - float(r["Start_Timestamp"])})
    return [(k, rows[k][0], rows[k][1]) for k in sorted(rows)]


def _last_of(disp, key, n):
    """The last n dispatches whose kernel name contains key."""
    sel = [x for x in disp if key in x[1]]
    return sel[-n:]


def _mean(xs, counter):
    return float(np.mean([x[2].get(counter, 0.0) for x in xs])) if xs else None


PROFILE_SETS = {
    # name: (kernel key, replays in the trace run, replays in the counter runs, program, title, output files)
    "batched": ("k_walk_queue", 3, 2, "python3 /root/repo/bench.py --config profile_batched --warmup 0 --steps {k}",
                "64-graph / 4096-request batched node2vec workload (the headline's batched plan)",
                (BATCHED_TRACE_FILE, BATCHED_TRAFFIC_FILE, BATCHED_COUNTERS_FILE, SECTOR_FILE)),
    "c2": ("k_walk_n2v", 3, 2, "python3 /root/repo/bench.py --config chung_lu_1m --runs 0.25,4 --warmup 0 --steps {k} "
                               "--cpu-seconds 0",
           "1M-node Chung-Lu graph, node2vec (p, q) = (0.25, 4), 10 walks of 100 slots per node",
           (TRACE_FILE, TRAFFIC_FILE, COUNTERS_FILE, os.path.join(ROOT, "profiles", "pmc_sectors_chung_lu_1m.txt"))),
    "c2fo": ("k_walk_lane", 3, 2, "python3 /root/repo/bench.py --config chung_lu_1m --runs 1,1 --warmup 0 --steps {k} "
                                  "--cpu-seconds 0",
             "1M-node Chung-Lu graph, first-order walks ((p, q) = (1, 1)), 10 walks of 100 slots per node",
             tuple(os.path.join(ROOT, "profiles", f) for f in (
                 "kernel_trace_chung_lu_1m_first_order.txt", "pmc_traffic_chung_lu_1m_first_order.txt",
                 "pmc_counters_chung_lu_1m_first_order.txt", "pmc_sectors_chung_lu_1m_first_order.txt"))),
    "ef": ("k_walk_n2v_ef", 1, 1, "python3 /root/repo/bench.py --config ef --warmup 0 --steps {k}",
           "1M-node Chung-Lu graph on the Elias-Fano store (quantum 256), node2vec (p, q) = (0.25, 4), one walk of "
           "100 slots per node",
           tuple(os.path.join(ROOT, "profiles", f) for f in (
               "kernel_trace_ef_chung_lu_1m.txt", "pmc_traffic_ef_chung_lu_1m.txt", "pmc_counters_ef_chung_lu_1m.txt",
               "pmc_sectors_ef_chung_lu_1m.txt")),
           ("n2v_ef.hip", "n2v_device.hpp", "n2v_internal.hpp")),
    "big": ("k_walk_n2v", 1, 1, "python3 /root/repo/bench.py --config big --big-runs n2v --warmup 0 --steps {k} "
                                "--cpu-seconds 0",
            "20M-node Chung-Lu graph, node2vec (p, q) = (1, 2), one walk of 80 slots per node",
            tuple(os.path.join(ROOT, "profiles", f) for f in (
                "kernel_trace_chung_lu_20m.txt", "pmc_traffic_chung_lu_20m.txt", "pmc_counters_chung_lu_20m.txt",
                "pmc_sectors_chung_lu_20m.txt"))),
}


def summarize_kernel_profiles(which, root):
    """profiles/ summaries of one kernel's timed launches (the last few
    dispatches whose name holds the kernel key in each profiled run) and of the
    calibration kernels.  Directory layout under root: trace, fetch, write, sq,
    tcc (profiles of the set's program) and cal_fetch, cal_write, cal_tcc
    (profiles of `bench.py --config calibrate`)."""
    import csv
    KQ, n_trace, n_pmc, prog, title, files = PROFILE_SETS[which][:6]
    sources = PROFILE_SETS[which][6] if len(PROFILE_SETS[which]) > 6 else WALK_SOURCES
    trace_file, traffic_file, counters_file, sector_file = files
    cal = "python3 /root/repo/bench.py --config calibrate"
    cmd = "cd /tmp && rocprofv3 {what} --output-format csv -d <dir> -o run -- {prog}"
    sq_names = ["SQ_WAVES", "SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES", "SQ_WAIT_ANY", "SQ_WAIT_INST_ANY",
                "SQ_INSTS_VALU", "SQ_INSTS_VMEM_RD", "SQ_INSTS_LDS"]
    tcc_names = ["TCC_HIT_sum", "TCC_MISS_sum", "TCP_TCC_READ_REQ_sum", "TCP_TCC_WRITE_REQ_sum"]
    cmds = {
        "trace": cmd.format(what="--kernel-trace --stats", prog=prog.format(k=n_trace)),
        "fetch": cmd.format(what="--pmc FETCH_SIZE", prog=prog.format(k=n_pmc)),
        "write": cmd.format(what="--pmc WRITE_SIZE", prog=prog.format(k=n_pmc)),
        "sq": cmd.format(what="--pmc " + " ".join(sq_names), prog=prog.format(k=n_pmc)),
        "tcc": cmd.format(what="--pmc " + " ".join(tcc_names), prog=prog.format(k=n_pmc)),
        "cal_fetch": cmd.format(what="--pmc FETCH_SIZE", prog=cal),
        "cal_write": cmd.format(what="--pmc WRITE_SIZE", prog=cal),
        "cal_tcc": cmd.format(what="--pmc " + " ".join(tcc_names), prog=cal),
    }
    sub = lambda k: os.path.join(root, k)  # noqa: E731
    h = kernel_source_hash(sources)
    # kernel trace: stats table, and the timed launches' mean duration
    tr = _last_of(_dispatches(sub("trace")), KQ, n_trace)
    lines = [f"# rocprofv3 --kernel-trace --stats, {title}", f"# command: {cmds['trace']}", f"source_hash: {h}",
             f"{KQ} launches: {len(tr)} launch_mean_ns: {_mean(tr, 'ns'):.6e}",
             "# kernel | calls | total ns | average ns | min ns | max ns"]
    for f in _csvs(sub("trace"), "kernel_stats.csv"):
        for row in csv.DictReader(open(f)):
            lines.append(" | ".join([row["Name"][:110], row["Calls"], row["TotalDurationNs"], row["AverageNs"],
                                     row["MinNs"], row["MaxNs"]]))
    open(trace_file, "w").write("\n".join(lines) + "\n")
    # calibration: useful bytes of the random-gather dispatches over what the counters read
    cf, cw, ct = _dispatches(sub("cal_fetch")), _dispatches(sub("cal_write")), _dispatches(sub("cal_tcc"))
    g64 = [x for x in cf if "k_gather<4>" in x[1]]
    g128 = [x for x in cf if "k_gather<8>" in x[1]]
    # the 1 GiB copy: the non-gather dispatch that reads most (fills read nothing);
    # in the write run, the dispatch of the same kernel (fills of the gather
    # buffers write more, in pieces)
    cpy = max((x for x in cf if "gather" not in x[1]), key=lambda x: x[2].get("FETCH_SIZE", 0.0), default=None)
    cpw = max((x for x in cw if cpy is not None and x[1] == cpy[1]), key=lambda x: x[2].get("WRITE_SIZE", 0.0),
              default=None)
    f64 = CAL_USEFUL / (g64[0][2]["FETCH_SIZE"] * 1024.0) if g64 else None
    f128 = CAL_USEFUL / (g128[0][2]["FETCH_SIZE"] * 1024.0) if g128 else None
    fcopy = COPY_BYTES / (cpy[2]["FETCH_SIZE"] * 1024.0) if cpy else None
    wcopy = COPY_BYTES / (cpw[2]["WRITE_SIZE"] * 1024.0) if cpw else None
    t64 = [x for x in ct if "k_gather<4>" in x[1]]
    req_bytes = CAL_USEFUL / t64[0][2]["TCP_TCC_READ_REQ_sum"] if t64 and t64[0][2].get("TCP_TCC_READ_REQ_sum") \
        else None
    # the kernel's traffic, FETCH_SIZE scaled by the 64 B random-gather calibration
    fq = _last_of(_dispatches(sub("fetch")), KQ, n_pmc)
    wq = _last_of(_dispatches(sub("write")), KQ, n_pmc)
    fb = _mean(fq, "FETCH_SIZE") * 1024.0 * (f64 or 1.0) if fq else None
    wb = _mean(wq, "WRITE_SIZE") * 1024.0 * (wcopy or 1.0) if wq else None
    out = [f"# HBM traffic per launch of {KQ}, {title}, from two rocprofv3 --pmc runs (FETCH_SIZE, then "
           "WRITE_SIZE, KiB per dispatch; mean over the timed launches)",
           "# FETCH_SIZE is scaled by what it reads for random 64-byte gathers of known size over a 16 GiB buffer "
           "(fetch_scale), WRITE_SIZE by what it reads for a plain 1 GiB copy (write_scale)",
           f"# fetch command: {cmds['fetch']}", f"# write command: {cmds['write']}",
           f"# calibration commands: {cmds['cal_fetch']} ; {cmds['cal_write']}",
           f"source_hash: {h}",
           f"gather64_fetch_KiB: {g64[0][2]['FETCH_SIZE'] if g64 else None}",
           f"gather128_fetch_KiB: {g128[0][2]['FETCH_SIZE'] if g128 else None}",
           f"gather_useful_bytes: {CAL_USEFUL}",
           f"fetch_scale: {f64}", f"fetch_scale_gather128: {f128}", f"fetch_scale_copy: {fcopy}",
           f"write_scale: {wcopy}",
           f"{KQ} launches: {len(fq)} fetch_bytes_per_launch: {fb} write_bytes_per_launch: {wb}",
           f"{KQ} hbm_bytes_per_launch: {(fb or 0.0) + (wb or 0.0) if fb is not None else None}"]
    open(traffic_file, "w").write("\n".join(out) + "\n")
    # SQ / TCC / TCP counters of the timed launches
    sq = _last_of(_dispatches(sub("sq")), KQ, n_pmc)
    tc = _last_of(_dispatches(sub("tcc")), KQ, n_pmc)
    v = {n: _mean(sq, n) or 0.0 for n in sq_names}
    waves = max(v["SQ_WAVES"], 1.0)
    hit, miss = _mean(tc, "TCC_HIT_sum") or 0.0, _mean(tc, "TCC_MISS_sum") or 0.0
    out = [f"# rocprofv3 --pmc counters of {KQ}, {title} (mean over the timed launches)",
           f"# sq command: {cmds['sq']}", f"# tcc command: {cmds['tcc']}", f"source_hash: {h}",
           f"{KQ} " + " ".join(f"{n}: {v[n]:.6e}" for n in sq_names) + f" TCC_HIT_sum: {hit:.6e} "
           f"TCC_MISS_sum: {miss:.6e}",
           f"{KQ} valu_insts_per_wave: {v['SQ_INSTS_VALU'] / waves:.1f} "
           f"vmem_rd_insts_per_wave: {v['SQ_INSTS_VMEM_RD'] / waves:.1f} "
           f"lds_insts_per_wave: {v['SQ_INSTS_LDS'] / waves:.1f} "
           f"wait_any_share_of_wave_cycles: {v['SQ_WAIT_ANY'] / max(v['SQ_WAVE_CYCLES'], 1.0):.3f}",
           f"{KQ} l2_hit_rate: {hit / max(hit + miss, 1.0):.4f}"]
    open(counters_file, "w").write("\n".join(out) + "\n")
    # L1-to-L2 requests: bytes per request from the 64 B gather calibration
    rd, wr = _mean(tc, "TCP_TCC_READ_REQ_sum"), _mean(tc, "TCP_TCC_WRITE_REQ_sum")
    rb = req_bytes or 64.0
    out = [f"# L1-to-L2 (TCP-to-TCC) requests of {KQ}, {title} (mean over the timed launches); bytes per "
           "request from random 64-byte gathers of known size (request_bytes)",
           f"# command: {cmds['tcc']}", f"# calibration command: {cmds['cal_tcc']}", f"source_hash: {h}",
           f"request_bytes: {rb}",
           f"{KQ} read_requests_per_launch: {rd} write_requests_per_launch: {wr}",
           f"{KQ} l2_request_bytes_per_launch: {((rd or 0.0) + (wr or 0.0)) * rb:.6e}"]
    open(sector_file, "w").write("\n".join(out) + "\n")
    for f in files:
        print(open(f).read())


def bench_headline(args):
    """The default line: 64 resident Chung-Lu graphs and 4096 node2vec requests,
    batched (one replay of the captured persistent launch per bench step)
    against one launch per request, and served under Poisson arrivals at
    200 / 1000 / 5000 req/s against one launch per request on the same
    schedule."""
    import torch
    import paper_2110_06196_amd as n2v
    import synth
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    threads = min(16, os.cpu_count() or 1)
    t0 = time.time()
    ps, host = synth.many_graphs(threads=threads)
    print(f"[bench] 64 graphs generated in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    dev_graphs, graphs, degs = [], [], []
    prep_s = 0.0
    lists = entries = dev_bytes = 0
    for (O, D, W) in host:
        Ot = torch.from_numpy(O.view(np.int64)).to(dev)
        Dt = torch.from_numpy(D).to(dev)
        Wt = torch.from_numpy(W.view(np.int32)).to(dev)
        torch.cuda.synchronize()
        tu = time.perf_counter()
        g = n2v.n2v_graph_upload(Ot, Dt, Wt)
        torch.cuda.synchronize()
        prep_s += time.perf_counter() - tu
        info = n2v.n2v_graph_info(g)
        lists += info["pair_lists"]
        entries += info["pair_entries"]
        dev_bytes += info["device_bytes"]
        graphs.append(g)
        dev_graphs.append((Ot, Dt, Wt))
        degs.append((Ot[1:] - Ot[:-1]).to(torch.int64))
    n_entries = sum(int(D.size) for _, D, _ in host)
    print(f"[bench] uploads {prep_s:.2f}s, {lists} edge lists of {n_entries} entries", file=sys.stderr, flush=True)
    reqs = synth.many_requests([p["n"] for p in ps])
    batch_out = _requests_on_device(torch, dev, reqs)
    plain_out = _requests_on_device(torch, dev, reqs)
    stream = torch.cuda.current_stream()
    descs = [n2v.make_request(graphs[r["graph"]], n2v.N2V_NODE2VEC, S, 1, r["walk_len"], r["p"], r["q"],
                              r["seed"], 0, Y, lens) for r, (S, Y, lens) in zip(reqs, batch_out)]
    t1 = time.perf_counter()
    plan = n2v.n2v_batch_create(descs, autotune=True)
    t_create = time.perf_counter() - t1
    binfo = n2v.n2v_batch_info(plan)
    for _ in range(args.warmup):
        n2v.n2v_batch_launch(plan, stream)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for e0, e1 in ev:
        e0.record(stream)
        n2v.n2v_batch_launch(plan, stream)
        e1.record(stream)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t1
    k_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    steps = sum(int((lens.to(torch.int64) - 1).clamp(min=0).sum().item()) for _, _, lens in batch_out)
    ms_step = t_total / args.steps * 1e3
    value = steps / (ms_step / 1e3)
    print(f"[bench] batched: {args.steps} replays in {t_total:.3f}s, {value:.3e} steps/s (plan {t_create:.2f}s)",
          file=sys.stderr, flush=True)

    # plain: one launch per request
    def plain_pass():
        for r, (S, Y, lens) in zip(reqs, plain_out):
            n2v.n2v_walks_node2vec(graphs[r["graph"]], S, 1, r["walk_len"], r["p"], r["q"], r["seed"], 0,
                                   Y, lens, stream=stream)
    plain_pass()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.plain_passes):
        plain_pass()
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t1) / args.plain_passes
    differ_plain = sum(int(not (torch.equal(a[1], b[1]) and torch.equal(a[2], b[2])))
                       for a, b in zip(plain_out, batch_out))
    print(f"[bench] plain pass {t_plain:.3f}s, {differ_plain} requests differ from batched", file=sys.stderr,
          flush=True)

    # routes only: the same plan on graphs uploaded without stored edge lists
    ro_graphs = [n2v.n2v_graph_upload(Ot, Dt, Wt, flags=n2v.N2V_UPLOAD_NO_PAIR_LISTS) for Ot, Dt, Wt in dev_graphs]
    for _, Y, lens in plain_out:
        Y.fill_(-9)
        lens.fill_(-9)
    ro_descs = [n2v.make_request(ro_graphs[r["graph"]], n2v.N2V_NODE2VEC, S, 1, r["walk_len"], r["p"], r["q"],
                                 r["seed"], 0, Y, lens) for r, (S, Y, lens) in zip(reqs, plain_out)]
    ro_plan = n2v.n2v_batch_create(ro_descs, autotune=True)
    n2v.n2v_batch_launch(ro_plan, stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.plain_passes):
        n2v.n2v_batch_launch(ro_plan, stream)
    torch.cuda.synchronize()
    t_routes = (time.perf_counter() - t1) / args.plain_passes
    differ_routes = sum(int(not (torch.equal(a[1], b[1]) and torch.equal(a[2], b[2])))
                        for a, b in zip(plain_out, batch_out))
    ro_shape = n2v.n2v_batch_info(ro_plan)
    n2v.n2v_batch_destroy(ro_plan)
    for g in ro_graphs:
        n2v.n2v_graph_release(g)
    print(f"[bench] routes only (no stored lists): {t_routes:.3f}s per replay, {differ_routes} requests differ",
          file=sys.stderr, flush=True)

    # oracle rows: 4 evenly spaced walks of every request
    rows = [np.unique(np.linspace(0, r["starts"].size - 1, min(4, r["starts"].size)).astype(np.int64)) for r in reqs]
    served = []
    served_rows = []
    if not args.no_served:
        hdesc = [n2v.host_request(graphs[r["graph"]], n2v.N2V_NODE2VEC, r["starts"], 1, r["walk_len"], r["p"],
                                  r["q"], r["seed"]) for r in reqs]
        for rate in [float(x) for x in args.rates.split(",") if x]:
            rec, srows = _serve_rate(torch, n2v, graphs, reqs, [h[0] for h in hdesc], rate, plain_out, stream, rows)
            served.append(rec)
            served_rows.append(srows)

    # the batched kernel: algorithmic bytes per launch, measured traffic and
    # sector bytes from the committed counter profiles of this command
    alg = 0
    by_variant = {}
    for r, (_, Y, lens) in zip(reqs, batch_out):
        v = variant_of(r["p"], r["q"])
        st, b = section8d_bytes(torch, Y, lens, degs[r["graph"]], v)
        alg += b
        sv = by_variant.setdefault(v, [0, 0])
        sv[0] += st
        sv[1] += b
    achieved = alg / (k_ms / 1e3) / 1e9
    f_scale = _profile_value(BATCHED_TRAFFIC_FILE, "fetch_scale")
    traffic = _profile_value(BATCHED_TRAFFIC_FILE, "k_walk_queue hbm_bytes_per_launch")
    sector_bytes = _profile_value(SECTOR_FILE, "k_walk_queue l2_request_bytes_per_launch")
    l2_hit = _profile_value(BATCHED_COUNTERS_FILE, "k_walk_queue l2_hit_rate")
    # residency of what the walks read: graph arrays, prefix, node records,
    # stored lists (rounded up to a power of two for the gather probe)
    ws = sum(O.nbytes + D.nbytes + W.nbytes for O, D, W in host) + dev_bytes
    ws2 = 1 << int(np.ceil(np.log2(ws)))
    g64 = gather_bw(torch, min(ws2, 16 << 30), 64)
    b_bar = sector_bytes / steps if sector_bytes else None
    print(f"[bench] gather 64 B over {min(ws2, 16 << 30)} B: {g64:.0f} GB/s", file=sys.stderr, flush=True)

    # CPU baseline: the oracle on 4 walks of every request (all host threads)
    # and on the first walk of every 16th request (one thread)
    cpu = None
    parity = {"requests_differing_from_plain": differ_plain, "requests_differing_routes_only": differ_routes}
    if args.cpu_seconds > 0:
        csteps, ct, mism, expect = _oracle_rows(host, reqs, rows, threads, batch_out, torch)
        one = list(range(0, len(reqs), 16))
        c1steps, c1t, _, _ = _oracle_rows(host, [reqs[k] for k in one], [rows[k][:1] for k in one], 1)
        cpu = {"value": csteps / ct, "unit": "walk steps/s", "cores": threads, "kind": "oracle",
               "sample": f"4 evenly spaced walks of each of the {len(reqs)} requests ({csteps} steps, {ct:.1f} s)",
               "one_core": {"value": c1steps / c1t, "sample": f"first walk of every 16th request ({c1steps} steps, "
                                                              f"{c1t:.1f} s)"},
               "nproc": os.cpu_count()}
        parity["oracle_sample_rows"] = int(sum(x.size for x in rows))
        parity["batched_rows_differing_from_oracle"] = mism
        for rec, srows in zip(served, served_rows):
            bad = 0
            for k in range(len(reqs)):
                Yo, lo = expect[k]
                bad += int(((srows[k][0] != Yo).any(axis=1) | (srows[k][1] != lo)).sum())
            rec["served_rows_differing_from_oracle"] = bad
    out = {
        "metric": METRIC, "value": value, "unit": "walk steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {
            "workload": "batched node2vec: 64 resident Chung-Lu graphs (n log-uniform in [1e3, 1e6], mean degree "
                        "U[8, 32], gamma 2.2, max expected degree sqrt(n * mean), weights U[1, 100], seeds 100+g) x "
                        "4096 requests (seed 7: 1..1e4 starts, length U[10, 200], (p, q) in {0.25, 1, 4}^2); one "
                        "bench step = one replay of the captured persistent launch over all requests",
            "form": "batched (persistent queue kernel, hipGraph replay)",
            "n_graphs": len(graphs), "n_nodes": int(sum(p["n"] for p in ps)), "n_entries": n_entries,
            "n_requests": len(reqs), "n_walks": int(binfo["n_walks"]), "steps_per_replay": steps,
            "autotuned_shape": [int(binfo["lanes_per_walker"]), int(binfo["lds_tile"]), int(binfo["list_cap"])],
            "chunks": int(binfo["n_chunks"]),
        },
        "plain": {"value": steps / t_plain, "ms_per_pass": t_plain * 1e3, "passes": args.plain_passes,
                  "form": "one launch per request (4096 launches per pass, one stream)"},
        "batched_vs_plain": t_plain / (ms_step / 1e3),
        "routes_only": {"value": steps / t_routes, "ms_per_replay": t_routes * 1e3,
                        "shape": [int(ro_shape["lanes_per_walker"]), int(ro_shape["lds_tile"]),
                                  int(ro_shape["list_cap"])],
                        "note": "same plan on graphs uploaded with N2V_UPLOAD_NO_PAIR_LISTS: every second-order "
                                "step classifies its candidates by the probe / stream / merge routes"},
        "prep": {"upload_s": prep_s, "plan_create_s": t_create, "device_bytes": dev_bytes, "edge_lists": lists,
                 "list_entries": entries,
                 "amortised_value": steps * args.steps / (t_total + prep_s + t_create),
                 "note": "graph uploads (validation, prefix, node records, heads, stored common-neighbour lists) "
                         "and plan creation (tables, autotuning, capture), outside the timed region; "
                         "amortised_value charges them to the timed replays"},
        "served": served,
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": "k_walk_queue (batched persistent launch)", "kernel_ms": k_ms, "alg_bytes_per_launch": alg,
            "by_variant": {k: {"steps": v[0], "bytes": v[1]} for k, v in by_variant.items()},
            "note": "achieved = per-step bytes of the method's statement for the variant run (first order 24 + 4 "
                    "ceil(log2(d+1)); return only 28 + 8 ceil(log2(d+1)); 1/q != 1: 20 + 8 d, the streamed row) "
                    "summed over the launch's steps / HIP-event launch time; traffic = calibrated FETCH_SIZE + "
                    "WRITE_SIZE per launch from the committed counter profile (null if taken on other sources)",
        },
        "gather_roofline": {
            "b_bar_bytes_per_step": b_bar, "bw_gather_64B_GBps": g64, "buffer_bytes": min(ws2, 16 << 30),
            "working_set_bytes": ws,
            "roofline_steps_per_s": (g64 * 1e9 / b_bar) if b_bar else None,
            "frac": (value * b_bar / (g64 * 1e9)) if b_bar else None,
            "l2_hit_rate": l2_hit, "fetch_scale": f_scale,
            "note": "b_bar = 64-byte sector requests the batched kernel sends to L2 per step (TCP-to-TCC read and "
                    "write requests, committed counter profile of this command) ; roofline = random 64 B gather "
                    "bandwidth over a buffer of the working set's size, measured in this run, / b_bar",
        },
        "cpu_baseline": cpu,
        "parity_sample": parity,
        "kernel_source_hash": kernel_source_hash(),
    }
    print(json.dumps(out), flush=True)
    n2v.n2v_batch_destroy(plan)


def _oracle_rows(host, reqs, rows, threads, outs=None, torch=None):
    """The oracle's walks at rows[k] of every request k on `threads` host
    threads; returns (steps, seconds, rows differing from outs, [(Y, lens)])."""
    import concurrent.futures as cf
    import oracle

    def one(k):
        r = reqs[k]
        O, D, W = host[r["graph"]]
        return oracle.walks(O, D, W, r["starts"], 1, r["walk_len"], oracle.NODE2VEC, r["p"], r["q"], r["seed"], 0,
                            rows[k])

    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(threads) as ex:
        res = list(ex.map(one, range(len(reqs))))
    dt = time.perf_counter() - t0
    steps = sum(int(np.maximum(lo.astype(np.int64) - 1, 0).sum()) for _, lo in res)
    mism = 0
    if outs is not None:
        for k, (Yo, lo) in enumerate(res):
            idx = torch.from_numpy(rows[k]).to(outs[k][1].device)
            Yg = outs[k][1].index_select(0, idx).cpu().numpy()
            lg = outs[k][2].index_select(0, idx).cpu().numpy()
            mism += int(((Yg != Yo).any(axis=1) | (lg != lo)).sum())
    return steps, dt, mism, res


def bench_batched(args):
    import torch
    import paper_2110_06196_amd as n2v
    import synth
    dev = torch.device("cuda:0")
    ps, host, graphs = many_graphs_on_device(torch, n2v, dev)
    reqs = synth.many_requests([p["n"] for p in ps])
    plain_out = _requests_on_device(torch, dev, reqs)
    batch_out = _requests_on_device(torch, dev, reqs)
    stream = torch.cuda.current_stream()

    def plain_pass():
        for r, (S, Y, lens) in zip(reqs, plain_out):
            n2v.n2v_walks_node2vec(graphs[r["graph"]][0], S, 1, r["walk_len"], r["p"], r["q"], r["seed"], 0,
                                   Y, lens, stream=stream)

    descs = [n2v.make_request(graphs[r["graph"]][0], n2v.N2V_NODE2VEC, S, 1, r["walk_len"], r["p"], r["q"],
                              r["seed"], 0, Y, lens) for r, (S, Y, lens) in zip(reqs, batch_out)]
    for _ in range(args.warmup):
        plain_pass()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plain_pass()
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) / args.steps
    print(f"[bench] plain pass {t_plain:.3f}s", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    plan = n2v.n2v_batch_create(descs, autotune=True)
    t_create = time.perf_counter() - t0
    info = n2v.n2v_batch_info(plan)
    for _ in range(args.warmup):
        n2v.n2v_batch_launch(plan, stream)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for e0, e1 in ev:
        e0.record(stream)
        n2v.n2v_batch_launch(plan, stream)
        e1.record(stream)
    torch.cuda.synchronize()
    t_batched = (time.perf_counter() - t0) / args.steps
    k_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    print(f"[bench] batched pass {t_batched:.3f}s (create {t_create:.2f}s)", file=sys.stderr, flush=True)
    steps = sum(int((lens.to(torch.int64) - 1).clamp(min=0).sum().item()) for _, _, lens in batch_out)
    same = sum(int(not (torch.equal(a[1], b[1]) and torch.equal(a[2], b[2]))) for a, b in zip(plain_out, batch_out))
    cpu = None
    parity = {"requests_differing_from_plain": same}
    if args.cpu_seconds > 0:
        threads = min(16, os.cpu_count() or 1)
        csteps, ct, mism = _oracle_sample(host, reqs, 4, threads, batch_out, torch)
        cpu = {"value": csteps / ct, "unit": "walk steps/s", "cores": threads, "kind": "oracle",
               "sample": f"4 evenly spaced walks of each of the {len(reqs)} requests ({csteps} steps, {ct:.1f} s)"}
        parity["oracle_sample_mismatching_rows"] = mism
    out = {
        "metric": METRIC, "value": steps / t_batched, "unit": "walk steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": t_batched * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "batched: 64 Chung-Lu graphs (n log-uniform 1e3..1e6, mean degree U[8,32], "
                               "gamma 2.2, weights U[1,100]); 4096 node2vec requests (1..1e4 starts, length "
                               "U[10,200], (p,q) in {0.25,1,4}^2)",
                   "form": "batched: one persistent hipGraph-captured launch",
                   "n_requests": len(reqs), "n_walks": int(info["n_walks"]), "chunks": int(info["n_chunks"]),
                   "autotuned_shape": [int(info["lanes_per_walker"]), int(info["lds_tile"]), int(info["list_cap"])]},
        "plain": {"value": steps / t_plain, "ms_per_step": t_plain * 1e3, "form": "one launch per request"},
        "speedup_vs_plain": t_plain / t_batched,
        "batched_kernel_ms": k_ms, "plan_create_s": t_create,
        "cpu_baseline": cpu, "parity_sample": parity, "kernel_source_hash": kernel_source_hash(),
    }
    print(json.dumps(out), flush=True)
    n2v.n2v_batch_destroy(plan)


def bench_served(args):
    import threading
    import torch
    import paper_2110_06196_amd as n2v
    import synth
    dev = torch.device("cuda:0")
    ps, host, graphs = many_graphs_on_device(torch, n2v, dev)
    reqs = synth.many_requests([p["n"] for p in ps])
    outs = _requests_on_device(torch, dev, reqs)
    stream = torch.cuda.current_stream()
    hdesc = [n2v.host_request(graphs[r["graph"]][0], n2v.N2V_NODE2VEC, r["starts"], 1, r["walk_len"], r["p"],
                              r["q"], r["seed"])[0] for r in reqs]
    skip = len(reqs) // 20  # the first 5% of arrivals are warm-up

    def pct(lat):
        lat = np.sort(np.asarray(lat[skip:], dtype=np.float64)) / 1e6
        return float(lat[int(0.5 * (lat.size - 1))]), float(lat[int(np.ceil(0.99 * (lat.size - 1)))])

    def wait_until(t_ns):
        while True:
            d = t_ns - time.monotonic_ns()
            if d <= 0:
                return
            if d > 2_000_000:
                time.sleep((d - 1_000_000) / 1e9)

    results = []
    for rate in [float(x) for x in args.rates.split(",")]:
        arr = synth.poisson_arrivals(len(reqs), rate)
        # --- server: continuous batching
        srv = n2v.n2v_server_create(200 << 30, 4096)
        for g, _ in graphs:
            n2v.n2v_server_add_graph(srv, g)
        ids = [0] * len(reqs)
        lat = [0] * len(reqs)
        steps = [0] * len(reqs)
        done_t = [0] * len(reqs)
        submitted = [0]
        t0 = time.monotonic_ns() + 20_000_000

        def poller():
            pending = set()
            seen = 0
            left = len(reqs)
            while left:
                upto = submitted[0]
                pending.update(range(seen, upto))
                seen = upto
                for k in list(pending):
                    res = n2v.n2v_request_poll(srv, ids[k])
                    if res is not None:
                        lat[k] = res.t_done_ns - res.t_arrival_ns
                        done_t[k] = res.t_done_ns
                        steps[k] = res.steps
                        n2v.n2v_request_release(srv, ids[k])
                        pending.discard(k)
                        left -= 1
                time.sleep(0.0002)

        th = threading.Thread(target=poller)
        th.start()
        for k in range(len(reqs)):
            ta = t0 + int(arr[k] * 1e9)
            wait_until(ta)
            ids[k] = n2v.n2v_request_submit(srv, hdesc[k], ta)
            submitted[0] = k + 1
        th.join()
        n2v.n2v_server_destroy(srv)
        s50, s99 = pct(lat)
        s_tput = sum(steps) / ((max(done_t) - t0) / 1e9)
        print(f"[bench] served rate {rate:g}: p50 {s50:.1f} ms p99 {s99:.1f} ms", file=sys.stderr, flush=True)
        # --- baseline: one plain launch per request, FIFO, one stream
        events = [None] * len(reqs)
        blat = [0] * len(reqs)
        bdone = [0] * len(reqs)
        launched = [0]
        t0 = time.monotonic_ns() + 20_000_000

        def bpoller():
            k = 0
            while k < len(reqs):
                if k >= launched[0]:
                    time.sleep(0.0001)
                    continue
                if events[k].query():
                    now = time.monotonic_ns()
                    bdone[k] = now
                    blat[k] = now - (t0 + int(arr[k] * 1e9))
                    k += 1
                else:
                    time.sleep(0.00005)

        th = threading.Thread(target=bpoller)
        th.start()
        for k, (r, (S, Y, lens)) in enumerate(zip(reqs, outs)):
            wait_until(t0 + int(arr[k] * 1e9))
            n2v.n2v_walks_node2vec(graphs[r["graph"]][0], S, 1, r["walk_len"], r["p"], r["q"], r["seed"], 0, Y, lens,
                                   stream=stream)
            e = torch.cuda.Event()
            e.record(stream)
            events[k] = e
            launched[0] = k + 1
        th.join()
        b50, b99 = pct(blat)
        bsteps = sum(int((l.to(torch.int64) - 1).clamp(min=0).sum().item()) for _, _, l in outs)
        b_tput = bsteps / ((max(bdone) - t0) / 1e9)
        print(f"[bench] plain rate {rate:g}: p50 {b50:.1f} ms p99 {b99:.1f} ms", file=sys.stderr, flush=True)
        results.append({"rate_rps": rate, "served": {"steps_per_s": s_tput, "p50_ms": s50, "p99_ms": s99},
                        "one_launch_per_request": {"steps_per_s": b_tput, "p50_ms": b50, "p99_ms": b99},
                        "steps": int(sum(steps)), "steps_match": int(sum(steps)) == bsteps})
    top = results[-1]
    out = {
        "metric": METRIC, "value": top["served"]["steps_per_s"], "unit": "walk steps/s", "n_gpus": 1,
        "steps": len(reqs), "warmup": skip, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "served: same 64 graphs and 4096 requests as the batched workload, open-loop "
                               "Poisson arrivals (seed 11), budget 200 GB, latency = done - scheduled arrival, "
                               "first 5% excluded", "form": "served (continuous batching)",
                   "value_at_rate_rps": top["rate_rps"]},
        "rates": results, "kernel_source_hash": kernel_source_hash(),
    }
    print(json.dumps(out), flush=True)


def bench_big(args):
    """20M nodes, 1e9 undirected edge samples (gamma 2.2, max expected degree 2e6,
    weights U[1,255]), generated on the GPU; first-order and node2vec (1, 2),
    one walk of 80 slots per node, seed 42; 300 sampled walks per run checked
    against the oracle."""
    import torch
    import oracle
    import paper_2110_06196_amd as n2v
    import synth
    dev = torch.device("cuda:0")
    n, ne = int(20_000_000 * args.big_scale), int(1_000_000_000 * args.big_scale)
    t0 = time.time()
    O, D, W = synth.chung_lu_device(n, ne, 2.2, 2.0 * ne / n, 2.0e6 * args.big_scale, (1, 255), seed=3,
                                    log=lambda m: print(f"[bench] {m} ({time.time() - t0:.0f}s)", file=sys.stderr,
                                                        flush=True))
    torch.cuda.synchronize()
    print(f"[bench] graph generated in {time.time() - t0:.1f}s, m={D.numel()}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    tu = time.perf_counter()
    g = n2v.n2v_graph_upload(O, D, W, flags=args.big_upload_flags)
    t_upload = time.perf_counter() - tu
    info = n2v.n2v_graph_info(g)
    print(f"[bench] upload {t_upload:.2f}s, hub sets {info['hub_sets']} (rows of degree >= "
          f"{info['hub_min_degree']})", file=sys.stderr, flush=True)
    L = 80
    S = torch.arange(n, dtype=torch.int32, device=dev)
    Y = torch.empty((n, L), dtype=torch.int32, device=dev)
    lens = torch.empty(n, dtype=torch.int32, device=dev)
    host = (O.cpu().numpy().view(np.uint64), D.cpu().numpy(), W.cpu().numpy().view(np.uint32))
    rows = np.linspace(0, n - 1, 300).astype(np.int64)
    runs = []
    which = set(args.big_runs.split(","))
    plan = [(n2v.N2V_FIRST_ORDER, 1.0, 1.0, 0)] if "fo" in which else []
    plan += [(n2v.N2V_NODE2VEC, 1.0, 2.0, 0)] if "n2v" in which else []
    if "approx" in which:
        plan += [(n2v.N2V_NODE2VEC, 1.0, 2.0, int(k)) for k in args.approx_k.split(",") if k]
    costs = None
    for kind, p, q, ka in plan:
        ms = []
        for k in range(args.warmup + args.steps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            if ka:
                n2v.n2v_walks_approximated(g, kind, S, 1, L, p, q, ka, 42, 0, Y, lens)
            elif kind == n2v.N2V_FIRST_ORDER:
                n2v.n2v_walks_first_order(g, S, 1, L, 42, 0, Y, lens)
            else:
                n2v.n2v_walks_node2vec(g, S, 1, L, p, q, 42, 0, Y, lens)
            e1.record()
            torch.cuda.synchronize()
            if k >= args.warmup:
                ms.append(e0.elapsed_time(e1))
            print(f"[bench] kind {kind} p {p} q {q} k {ka} launch {k}: {e0.elapsed_time(e1):.1f} ms",
                  file=sys.stderr, flush=True)
        steps = int((lens.to(torch.int64) - 1).clamp(min=0).sum().item())
        if args.step_costs and kind == n2v.N2V_NODE2VEC and not ka:
            costs = step_cost_histogram(torch, Y, lens, (O[1:] - O[:-1]).to(torch.int64))
        print(f"[bench] oracle on {rows.size} sampled walks", file=sys.stderr, flush=True)
        idx = torch.from_numpy(rows).to(dev)
        Yg = Y.index_select(0, idx).cpu().numpy()
        lg = lens.index_select(0, idx).cpu().numpy()
        t1 = time.perf_counter()
        Yo, lo = oracle.walks_threaded(*host, S.cpu().numpy(), 1, L, kind, p, q, 42, 0, rows, min(16, os.cpu_count()),
                                       k_approx=ka)
        ct = time.perf_counter() - t1
        csteps = int(np.maximum(lo.astype(np.int64) - 1, 0).sum())
        runs.append({"kind": "first_order" if kind == 0 else "node2vec", "p": p, "q": q, "k_approx": ka,
                     "mean_ms": float(np.mean(ms)), "steps": steps, "steps_per_s": steps / (np.mean(ms) / 1e3),
                     "oracle_sample_mismatching_rows": int(((Yg != Yo).any(1) | (lg != lo)).sum()),
                     "oracle_steps_per_s": csteps / ct})
    main_run = next((r for r in runs if r["kind"] == "node2vec" and not r["k_approx"]), runs[0])
    out = {"metric": METRIC, "value": main_run["steps_per_s"], "unit": "walk steps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": main_run["mean_ms"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
           "config": {"workload": "plain first-order, node2vec (p=1, q=2) and approximated node2vec on a Chung-Lu graph: 20M nodes, 1e9 "
                                  "undirected edge samples (gamma 2.2, max expected degree 2e6), weights U[1,255], "
                                  "one walk of 80 slots per node, seed 42",
                      "n_entries": int(D.numel()), "max_degree": info["max_degree"],
                      "upload_s": t_upload, "upload_flags": args.big_upload_flags, "hub_sets": info["hub_sets"],
                      "hub_min_degree": info["hub_min_degree"], "device_bytes": info["device_bytes"],
                      "stationary_mean_degree": info["sum_deg_sq"] / max(1, info["n_entries"])},
           "runs": runs, "step_costs": costs, "kernel_source_hash": kernel_source_hash()}
    if args.big_scale != 1.0:
        out["config"]["workload"] += f" (at {args.big_scale} of the stated size: {n} nodes, {ne} edge samples)"
    print(json.dumps(out), flush=True)
    n2v.n2v_graph_release(g)


def step_cost_histogram(torch, Y, lens, deg):
    """Second-order steps of a node2vec run (from v after t) by
    floor(log2(min(d_t, d_v))): step count, sum of min(d_t, d_v), and sum of
    min * ceil(log2(max + 1)) (the bisection reads of probing the shorter row
    into the longer) and of d_t + d_v (the entries a merge streams)."""
    nb = 24
    cnt = torch.zeros(nb, dtype=torch.float64, device=Y.device)
    smin = torch.zeros_like(cnt)
    sprobe = torch.zeros_like(cnt)
    smerge = torch.zeros_like(cnt)
    L = Y.shape[1]
    for s in range(2, L):
        ok = lens > s
        t = Y[:, s - 2][ok].to(torch.int64)
        v = Y[:, s - 1][ok].to(torch.int64)
        dt, dv = deg[t], deg[v]
        mn, mx = torch.minimum(dt, dv), torch.maximum(dt, dv)
        b = torch.floor(torch.log2(mn.clamp(min=1).to(torch.float64))).to(torch.int64).clamp(max=nb - 1)
        # bincount keeps per-block histograms (few bins: atomics on a handful
        # of global addresses would serialise)
        cnt += torch.bincount(b, minlength=nb).to(torch.float64)
        smin += torch.bincount(b, weights=mn.to(torch.float64), minlength=nb)
        smerge += torch.bincount(b, weights=(dt + dv).to(torch.float64), minlength=nb)
        smx = mn.to(torch.float64) * torch.ceil(torch.log2(mx.to(torch.float64) + 1))
        sprobe += torch.bincount(b, weights=smx, minlength=nb)
        if s % 20 == 0:
            print(f"[bench] step costs: slot {s}", file=sys.stderr, flush=True)
    rows = []
    for i in range(nb):
        if cnt[i] > 0:
            rows.append({"min_deg_log2": i, "steps": int(cnt[i]), "sum_min": float(smin[i]),
                         "sum_probe_reads": float(sprobe[i]), "sum_merge_entries": float(smerge[i])})
    return rows


def bench_corpus(args):
    """Training corpora of the 1M-node workload's walks (node2vec p=q=1, 10 walks
    per node, 100 slots, seed 42): SkipGram / CBOW context slots of one window,
    Walklets slots of each scale, and scale-free negatives per position.  One
    step runs every corpus kernel once over all 1e9 walk positions; the walks
    are generated once, before timing.  Sampled rows are checked against the
    oracle, which is also timed on them."""
    import torch
    import oracle
    import paper_2110_06196_amd as n2v

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    O, D, W = graph_cache()
    n = len(O) - 1
    Ot = torch.from_numpy(O.view(np.int64)).to(dev)
    Dt = torch.from_numpy(D).to(dev)
    Wt = torch.from_numpy(W.view(np.int32)).to(dev)
    g = n2v.n2v_graph_upload(Ot, Dt, Wt)
    R, L, seed = args.reps, args.walk_len, 42
    nw = n * R
    S = torch.arange(n, dtype=torch.int32, device=dev)
    Y = torch.empty((nw, L), dtype=torch.int32, device=dev)
    lens = torch.empty(nw, dtype=torch.int32, device=dev)
    n2v.n2v_walks_node2vec(g, S, R, L, 1.0, 1.0, seed, 0, Y, lens)
    torch.cuda.synchronize()
    w, n_neg = args.window, args.negatives
    scales = [int(k) for k in args.walklets.split(",") if k]
    C = torch.empty((nw, L, 2 * w), dtype=torch.int32, device=dev)
    Cw = [torch.empty((nw, L, 2), dtype=torch.int32, device=dev) for _ in scales]
    N = torch.empty((nw, L, n_neg), dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    npos = nw * L
    ops = [(f"skipgram_window{w}", lambda: n2v.n2v_walk_contexts(Y, w, 1, C, stream=stream), npos * (4 + 8 * w))]
    for k, buf in zip(scales, Cw):
        ops.append((f"walklets_scale{k}", lambda k=k, buf=buf: n2v.n2v_walk_contexts(Y, 1, k, buf, stream=stream),
                    npos * (4 + 8)))
    ops.append((f"negatives{n_neg}", lambda: n2v.n2v_negative_samples(g, Y, n_neg, seed, 0, N, stream=stream),
                npos * (4 + 4 * n_neg)))
    print(f"[bench] corpus: {npos} walk positions, {len(ops)} kernels", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        for _, f, _ in ops:
            f()
    torch.cuda.synchronize()
    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in ops]
          for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        for i, (_, f, _) in enumerate(ops):
            ev[k][i][0].record(stream)
            f()
            ev[k][i][1].record(stream)
    torch.cuda.synchronize()
    tt = time.perf_counter() - t0
    print(f"[bench] timed {args.steps} steps in {tt:.3f}s", file=sys.stderr, flush=True)
    kernels = []
    for i, (name, _, alg) in enumerate(ops):
        ms = float(np.mean([ev[k][i][0].elapsed_time(ev[k][i][1]) for k in range(args.steps)]))
        kernels.append({"op": name, "kernel": "k_negatives" if name.startswith("negatives") else "k_contexts_lds",
                        "mean_ms": ms, "alg_bytes": alg, "alg_GBps": alg / (ms / 1e3) / 1e9,
                        "positions_per_s": npos / (ms / 1e3)})
    dom = max(kernels, key=lambda k: k["mean_ms"])

    # Fused walk -> contexts (no walk array) against walks then contexts, for
    # the corpus's walks (p = q = 1) and node2vec (0.25, 4); outputs compared
    fused = []
    Cf = torch.empty_like(C)
    lf = torch.empty_like(lens)
    Yu = torch.empty_like(Y)
    lu = torch.empty_like(lens)
    for p, q in ((1.0, 1.0), (0.25, 4.0)):
        def unfused():
            n2v.n2v_walks_node2vec(g, S, R, L, p, q, seed, 0, Yu, lu, stream=stream)
            n2v.n2v_walk_contexts(Yu, w, 1, C, stream=stream)

        def fused_op():
            n2v.n2v_walks_contexts(g, n2v.N2V_NODE2VEC, S, R, L, p, q, seed, 0, w, 1, Cf, lf, stream=stream)
        times = {}
        for name, f in (("unfused", unfused), ("fused", fused_op)):
            f()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(max(1, args.steps)):
                f()
            e1.record(stream)
            torch.cuda.synchronize()
            times[name] = e0.elapsed_time(e1) / max(1, args.steps)
        same = bool(torch.equal(C, Cf) and torch.equal(lu, lf))
        fused.append({"p": p, "q": q, "unfused_ms": times["unfused"], "fused_ms": times["fused"], "identical": same,
                      "unfused_device_bytes": (Yu.numel() + C.numel()) * 4, "fused_device_bytes": C.numel() * 4})
        print(f"[bench] fused contexts (p, q) = ({p}, {q}): {times['fused']:.1f} ms, walks + contexts "
              f"{times['unfused']:.1f} ms, identical {same}", file=sys.stderr, flush=True)
    del Cf, Yu
    # the contexts buffer now holds the (0.25, 4) corpus: recompute the p = q = 1 one for the oracle check
    n2v.n2v_walk_contexts(Y, w, 1, C, stream=stream)
    torch.cuda.synchronize()

    # Oracle on a contiguous block of walk rows (walk ids follow the row index).
    rows = max(1, min(nw, int(20000 * max(args.cpu_seconds, 1.0) / 15.0)))
    r0 = nw // 2 - rows // 2
    Yh = Y[r0:r0 + rows].cpu().numpy()
    mism = {}
    t1 = time.perf_counter()
    Co = oracle.contexts(Yh, w, 1)
    Cwo = [oracle.contexts(Yh, 1, k) for k in scales]
    No = oracle.negatives(O, Yh, n_neg, seed, r0)
    ct = time.perf_counter() - t1
    mism[kernels[0]["op"]] = int((C[r0:r0 + rows].cpu().numpy() != Co).any(axis=(1, 2)).sum())
    for k, buf, ref in zip(scales, Cw, Cwo):
        mism[f"walklets_scale{k}"] = int((buf[r0:r0 + rows].cpu().numpy() != ref).any(axis=(1, 2)).sum())
    mism[kernels[-1]["op"]] = int((N[r0:r0 + rows].cpu().numpy() != No).any(axis=(1, 2)).sum())
    ms_step = tt / args.steps * 1e3
    out = {"metric": "walk positions turned into training corpora per second", "value": npos / (ms_step / 1e3),
           "unit": "walk positions/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "u64", "data": "synthetic",
           "config": {"workload": f"corpora of the walks of node2vec p=q=1 on the Chung-Lu 1M-node graph, {R} walks "
                                  f"per node, {L} slots, seed 42: SkipGram/CBOW window {w}, Walklets scales "
                                  f"{scales}, {n_neg} scale-free negatives per position",
                      "positions": npos},
           "roofline": {"bound": "hbm", "achieved": dom["alg_GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": dom["alg_GBps"] / HBM_PEAK_GBS,
                        "traffic": traffic_from_profiles(dom["kernel"], CORPUS_TRAFFIC_FILE, CORPUS_SOURCES),
                        "kernel": dom["op"]},
           "cpu_baseline": {"value": rows * L / ct, "unit": "walk positions/s", "cores": 1, "kind": "oracle",
                            "sample": f"walk rows [{r0}, {r0 + rows}) through every corpus op ({ct:.1f} s wall)"},
           "kernels": kernels, "fused_contexts": fused, "parity_sample": {"rows": rows, "mismatching_rows": mism},
           "kernel_source_hash": kernel_source_hash(CORPUS_SOURCES)}
    print(json.dumps(out), flush=True)
    n2v.n2v_graph_release(g)


def bench_ef(args):
    """The 1M-node workload on the Elias-Fano store (quantum 256) next to the
    CSR store: device bytes of each, first-order / node2vec (1, 1) walks (10
    per node) and node2vec (0.25, 4) walks (1 per node), 100 slots, seed 42.
    Every EF walk equals the CSR walk of the same request (checked in full)
    and sampled rows equal the oracle."""
    import torch
    import oracle
    import paper_2110_06196_amd as n2v

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    O, D, W = graph_cache()
    n = len(O) - 1
    Ot = torch.from_numpy(O.view(np.int64)).to(dev)
    Dt = torch.from_numpy(D).to(dev)
    Wt = torch.from_numpy(W.view(np.int32)).to(dev)
    gc = n2v.n2v_graph_upload(Ot, Dt, Wt)
    t0 = time.perf_counter()
    ge = n2v.n2v_graph_upload_ef(Ot, Dt, Wt, 256)
    t_build = time.perf_counter() - t0
    ic, ie, ef = n2v.n2v_graph_info(gc), n2v.n2v_graph_info(ge), n2v.n2v_ef_info(ge)
    ef_bytes = 8 * (ef["h_words"] + ef["l_words"] + ef["s1_len"] + ef["s0_len"])
    csr_bytes = 8 * (n + 1) + 4 * D.size
    prefix_bytes = ic["device_bytes"]
    L, seed = args.walk_len, 42
    deg = (Ot[1:] - Ot[:-1]).to(torch.int64)
    S = torch.arange(n, dtype=torch.int32, device=dev)
    runs = []
    for (p, q, R) in [(1.0, 1.0, args.reps), (0.25, 4.0, 1)]:
        nw = n * R
        outs = {}
        for name, g in (("csr", gc), ("ef", ge)):
            Y = torch.empty((nw, L), dtype=torch.int32, device=dev)
            lens = torch.empty(nw, dtype=torch.int32, device=dev)
            ms = []
            for k in range(args.warmup + args.steps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                n2v.n2v_walks_node2vec(g, S, R, L, p, q, seed, 0, Y, lens)
                e1.record()
                torch.cuda.synchronize()
                if k >= args.warmup:
                    ms.append(e0.elapsed_time(e1))
            outs[name] = (Y, lens, float(np.mean(ms)))
            print(f"[bench] ef: {name} p={p} q={q} {np.mean(ms):.1f} ms", file=sys.stderr, flush=True)
        same = bool(torch.equal(outs["csr"][0], outs["ef"][0]) and torch.equal(outs["csr"][1], outs["ef"][1]))
        Y, lens, ms = outs["ef"]
        variant = "generic" if q != 1.0 else "fo_weighted"
        steps, alg = algorithmic_bytes(torch, Y, lens, deg, variant)
        rows = np.linspace(0, nw - 1, 200).astype(np.int64)
        Yo, lo = oracle.walks_threaded(O, D, W, np.arange(n, dtype=np.int32), R, L, oracle.NODE2VEC, p, q, seed, 0,
                                       rows, min(16, os.cpu_count() or 1))
        idx = torch.from_numpy(rows).to(dev)
        mism = int(((Y.index_select(0, idx).cpu().numpy() != Yo).any(1) |
                    (lens.index_select(0, idx).cpu().numpy() != lo)).sum())
        runs.append({"p": p, "q": q, "walks_per_node": R, "steps": steps, "ef_ms": ms, "csr_ms": outs["csr"][2],
                     "ef_steps_per_s": steps / (ms / 1e3), "csr_steps_per_s": steps / (outs["csr"][2] / 1e3),
                     "ef_alg_GBps": alg / (ms / 1e3) / 1e9, "ef_equals_csr": same,
                     "oracle_sample_mismatching_rows": mism})
    dom = runs[-1]
    out = {"metric": METRIC, "value": dom["ef_steps_per_s"], "unit": "walk steps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": dom["ef_ms"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
           "config": {"workload": "node2vec on the Elias-Fano store (quantum 256) of the Chung-Lu 1M-node graph, "
                                  "100 slots, seed 42", "n_entries": int(D.size)},
           "storage": {"csr_topology_bytes": csr_bytes, "ef_topology_bytes": ef_bytes,
                       "ef_bits_per_entry": 8 * ef_bytes / max(1, D.size), "weight_prefix_bytes": prefix_bytes,
                       "ef_k": ef["k"], "ef_l": ef["l"], "ef_build_s": t_build,
                       "ef_bound_bits": 2 * D.size + D.size * int(np.ceil(np.log2(ef["u"] / D.size)))},
           "roofline": {"bound": "hbm", "achieved": dom["ef_alg_GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": dom["ef_alg_GBps"] / HBM_PEAK_GBS, "traffic": None,
                        "kernel": "node2vec p=0.25 q=4 over Elias-Fano (the CSR step's algorithmic bytes)"},
           "runs": runs, "kernel_source_hash": kernel_source_hash(("n2v_ef.hip", "n2v_device.hpp", "n2v_internal.hpp"))}
    print(json.dumps(out), flush=True)
    n2v.n2v_graph_release(ge)
    n2v.n2v_graph_release(gc)


if __name__ == "__main__":
    main()
