"""Benchmark of the LOR assembly hot path on one MI355X.

Workload (the headline configuration): H1 diffusion + mass LOR assembly at
p = 6 on 32^3 curved hexahedra (sinusoidal node map, amplitude 0.1 h),
log-normal kappa (sigma 2) per subelement, beta = 1: 7,189,057 rows,
192,100,033 nonzeros.  Inputs are synthetic and already resident in HBM; the
pattern and schedule are built once outside the timed region (they depend on
the mesh only) and their time is reported separately.

One step = one lor_assemble_h1 call in FP64 with the default kernel (the
owner-computes kernel on this mesh: every subelement integration, row sum
and CSR store of the step).  value = rows / step time in MDOF/s.  Extra
fields report the FP32 form, the coloured kernel for comparison, the
backward (adjoint) at p = 4 with a batch of 8 kappa fields, the H(curl),
H(div) and 2D assemblies, the pattern, the auxiliary kernels, the roofline of
the dominant kernel, and the CPU oracle timed on bounded samples.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes_h1(nel, p, ndofs, nnz, vbytes, batch=1):
    """Every input read once, every value written once (col_idx not read)."""
    q = p + 1
    return (batch * nnz * vbytes           # values
            + ndofs * 3 * 8                # coords (FP64)
            + nel * q ** 3 * 4             # elem_dofs
            + batch * nel * p ** 3 * vbytes  # kappa
            + (ndofs + 1) * 4)             # row_ptr


def algorithmic_bytes_vec(nel, p, nrows, ndofs_h1, nnz, vbytes, nloc_map):
    """H(curl) / H(div): values written once, coords, vertex map, signed edge
    or face map (nloc_map entries per element), kappa and row_ptr read once."""
    q = p + 1
    return (nnz * vbytes + ndofs_h1 * 3 * 8 + nel * q ** 3 * 4 + nel * nloc_map * 4 + nel * p ** 3 * vbytes
            + (nrows + 1) * 4)


def algorithmic_bytes_2d(nel, p, ndofs, nnz, vbytes):
    """2D H1: values written once, 2D coords, vertex map, kappa, row_ptr."""
    q = p + 1
    return nnz * vbytes + ndofs * 2 * 8 + nel * q * q * 4 + nel * p * p * vbytes + (ndofs + 1) * 4


def algorithmic_bytes_backward(nel, p, ndofs, nnz, vbytes, batch):
    """Adjoint: every input read once (the cotangent per batch entry, coords,
    vertex map, row_ptr, kappa per batch entry) and every output written once
    (the kappa gradient per batch entry, the vertex gradient).  The E-vector
    workspace round trip of this implementation is not counted."""
    q = p + 1
    return (batch * nnz * vbytes + ndofs * 24 + nel * q ** 3 * 4 + 2 * batch * nel * p ** 3 * vbytes
            + (ndofs + 1) * 4 + ndofs * 24)


MALL_BYTES = 256 * 2 ** 20   # MI355X Infinity Cache (memory-side, shared by all XCDs)


def roofline_of(bytes_, ms):
    """HBM roofline of a leg.  `mall_resident` flags a working set that fits in
    the 256 MB Infinity Cache: back-to-back calls may then be served partly
    from it, so the figure is a warm one."""
    ach = bytes_ / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
            "algorithmic_bytes": bytes_, "mall_resident": bool(bytes_ < MALL_BYTES)}


def ramp(fn, ms_target):
    """Call fn back to back, untimed, for about ms_target milliseconds of
    device time; returns the device time spent."""
    import torch
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    spent = 0.0
    while spent < ms_target:
        t0.record()
        for _ in range(10):
            fn()
        t1.record()
        torch.cuda.synchronize()
        spent += t0.elapsed_time(t1)
    return spent


def time_it(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(steps):
        fn()
    t1.record()
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / steps


def step_median(fn, steps):
    """Median step time (ms) over `steps` steps, one HIP event between
    consecutive steps on the launch stream (a separate pass after the timed
    region, so the reported mean is untouched)."""
    import torch
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    ev[0].record()
    for i in range(steps):
        fn()
        ev[i + 1].record()
    torch.cuda.synchronize()
    d = sorted(ev[i].elapsed_time(ev[i + 1]) for i in range(steps))
    return d[steps // 2] if steps % 2 else 0.5 * (d[steps // 2 - 1] + d[steps // 2])


def time_graph(fn, steps, reps=20):
    """Device time of one call of fn (ms): `reps` calls captured into one HIP
    graph, the graph replayed `steps` times between HIP events.  For the small
    legs, whose kernels take tens of microseconds, this removes the host
    launch overhead of the Python binding that back-to-back timing includes.
    fn must write preallocated outputs (no allocation, no memset) and be
    repeatable; the caller checks a replay against an eager call."""
    import torch
    fn()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        for _ in range(reps):
            fn()
    g.replay()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(steps):
        g.replay()
    t1.record()
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / (steps * reps)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def cpu_baseline(m, sample_elems, sample_elems_1t):
    """The oracle (unchanged: COO + stable sort + segment sums, FP64) on the
    first elements of the workload, with all host threads and with one, the
    median of 3 runs each, scaled linearly to the whole mesh.  The sort is
    O(n log n), so the linear scaling slightly flatters the CPU."""
    import statistics
    import torch
    from oracle import lor_oracle as orc

    def run(ne):
        t = time.perf_counter()
        R, C, V = orc._coo_h1(m["coords"], m["elem_dofs"][:ne], m["p"], m["kappa"][:ne], m["beta"])
        orc.coo_to_csr(R, C, V, m["ndofs"])
        return time.perf_counter() - t

    threads = torch.get_num_threads()
    out = {}
    for key, ne, nth in (("all", min(sample_elems, m["nel"]), threads), ("one", min(sample_elems_1t, m["nel"]), 1)):
        torch.set_num_threads(nth)
        try:
            ts = [run(ne) for _ in range(3)]
        finally:
            torch.set_num_threads(threads)
        dt = statistics.median(ts)
        out[key] = {"value": m["ndofs"] / (dt * m["nel"] / ne) / 1e6, "cores": nth, "elements": ne,
                    "seconds": ts}
    return {
        "value": out["all"]["value"],
        "unit": "MDOF/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"CPU FP64 oracle (COO + stable sort + segment sums) on the first {out['all']['elements']} of "
                  f"{m['nel']} elements, median of 3, scaled linearly to the whole mesh (the sort is n log n)",
        "one_thread": {"value": out["one"]["value"], "unit": "MDOF/s", "cores": 1,
                       "sample": f"first {out['one']['elements']} elements, median of 3, scaled linearly"},
        "runs_s": {"all": out["all"]["seconds"], "one": out["one"]["seconds"]},
        "cpu": cpu_model(),
    }


KERNEL_SOURCES = ("lor_h1.hip", "lor_h1_owner.hip", "lor_h1_math.hpp", "lor_common.hpp")
TRAFFIC_FILE = "h1_p6_32cubed_traffic.json"
VALU_FILE = "h1_p6_32cubed_valu.json"
# the headline kernels: rocprofv3 names -> keys of the committed records
KERNELS = {
    "owner_f64": "k_h1_owner<6, double, double>",
    "owner_f32": "k_h1_owner<6, float, float>",
    "colored_f64": "k_h1_assemble<6, double, double>",
    "colored_f32": "k_h1_assemble<6, float, float>",
}
# profiled workloads: summary name -> (kernels, their sources); the records
# are written by --summarize-profiles / --summarize-valu with --profile-name
PROFILE_SETS = {
    "h1_p6_32cubed": (KERNELS, KERNEL_SOURCES),
    "backward_p4_16cubed_b8": ({
        "backward_f64": "k_h1_backward<4, double, double>",
        "backward_f32": "k_h1_backward<4, float, float>",
        "gather_vertices": "k_gather_vertices",
    }, ("lor_backward.hip", "lor_h1_adjoint.hpp", "lor_h1_math.hpp", "lor_common.hpp")),
    "h1_2d_p6_512sq": ({
        "owner2d_f64": "k_h1_2d_owner<6, double, double>",
        "owner2d_f32": "k_h1_2d_owner<6, float, float>",
        "colored2d_f64": "k_h1_2d_assemble<6, double, double>",
        "colored2d_f32": "k_h1_2d_assemble<6, float, float>",
    }, ("lor_h1_2d_owner.hip", "lor_h1_2d.hip", "lor_h1_2d_math.hpp", "lor_h1_math.hpp", "lor_common.hpp")),
    "nd_p3_24cubed": ({
        **{f"nd_owner_{n}_{d}": f"k_nd_owner<3, {t}, {t}, {d}>" for n, t in (("f64", "double"), ("f32", "float"))
           for d in range(3)},
        "nd_colored_f64": "k_nd_assemble<3, double, double>",
        "nd_colored_f32": "k_nd_assemble<3, float, float>",
    }, ("lor_nd_owner.hip", "lor_nd.hip", "lor_nd_math.hpp", "lor_h1_math.hpp", "lor_common.hpp")),
}
# VALU wave-instruction counters (one rocprofv3 --pmc pass holds all five)
VALU_COUNTERS = ("SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64", "SQ_INSTS_VALU_FMA_F64",
                 "SQ_INSTS_VALU_TRANS_F64", "SQ_INSTS_VALU")
MI355X_SIMDS = 256 * 4           # 256 CUs x 4 SIMDs
MI355X_CLOCK_HZ = 2.4e9
CYCLES_PER_WAVE_INSTR = 4        # 16 lanes per SIMD per clock (FP64, and FP32 without packed math)
FP64_PEAK_TFLOPS = 78.6          # vector FP64 (an FMA counts as 2 flops)


def kernel_source_hash(sources=KERNEL_SOURCES):
    """Hash of the sources of the profiled kernels: counters taken on other code are stale."""
    import hashlib
    h = hashlib.sha256()
    for name in sources:
        with open(os.path.join(ROOT, "paper_2210_12253_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _load_record(fname, sources=KERNEL_SOURCES):
    path = os.path.join(ROOT, "profiles", fname)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_source_hash") != kernel_source_hash(sources):
        return {"stale": True, "file": fname}
    return t


def load_traffic(key, name="h1_p6_32cubed"):
    """HBM bytes per launch of one profiled kernel from the committed
    FETCH_SIZE / WRITE_SIZE summary: (bytes, detail), or (None, reason)."""
    fname = name + "_traffic.json"
    t = _load_record(fname, PROFILE_SETS[name][1])
    if t is None or t.get("stale"):
        return None, t
    k = t.get("kernels", {}).get(key)
    if k is None:
        return None, {"missing": key, "file": fname}
    return k["bytes_per_launch"], dict(k, fetch_scale=t["fetch_scale"], write_scale=t["write_scale"],
                                       command=t["command"])


def copy_calibration(torch, dev, nbytes=1 << 30, reps=5):
    """A plain 1 GiB device-to-device copy (torch's copy kernel): the achievable
    bandwidth reference and the known-size kernel the HBM counters are scaled by."""
    src = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        dst.copy_(src)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return {"bytes_read": nbytes, "bytes_written": nbytes, "ms": ms,
            "GBs": 2 * nbytes / (ms * 1e-3) / 1e9}


def _read_csvs(d, suffix):
    import glob
    import csv
    rows = []
    for path in sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True)):
        with open(path, newline="") as f:
            rows.extend(csv.DictReader(f))
    return rows


def _kernel_key(name):
    for key, needle in KERNELS.items():
        if needle in name:
            return key
    return None


def summarize_profiles(stats_dir, fetch_dir, write_dir, command, name="h1_p6_32cubed"):
    """Turn rocprofv3 CSV output of this script into the short text summary
    and the traffic record that bench.py reads.  stats_dir: --kernel-trace
    --stats run; fetch_dir / write_dir: --pmc FETCH_SIZE and --pmc WRITE_SIZE
    runs (counters in KiB per dispatch), all of `bench.py --skip-extras` (the
    headline kernels on the headline mesh only) or of `bench.py
    --backward-only` (name backward_p4_16cubed_b8), of `bench.py --h1-2d-only`
    (name h1_2d_p6_512sq) or of `bench.py --nd-only` (name nd_p3_24cubed)."""
    kernels, sources = PROFILE_SETS[name]
    lines = [f"command: {command}", ""]
    stats = _read_csvs(stats_dir, "kernel_stats.csv")
    lines.append(f"{'kernel':70s} {'calls':>6s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s} {'pct':>6s}")
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"])):
        if not ("lor::" in r["Name"] or "copy" in r["Name"].lower() or "elementwise" in r["Name"].lower()):
            continue
        lines.append(f"{r['Name'][:70]:70s} {int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:10.2f} "
                     f"{float(r['MinNs']) / 1e3:10.2f} {float(r['MaxNs']) / 1e3:10.2f} "
                     f"{float(r['Percentage']):6.2f}")
    res = {}
    for key, d, counter in (("fetch", fetch_dir, "FETCH_SIZE"), ("write", write_dir, "WRITE_SIZE")):
        per = {}
        for r in _read_csvs(d, "counter_collection.csv"):
            if r["Counter_Name"] != counter:
                continue
            per.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]) * 1024.0)
        res[key] = per

    def pick(per, needle):
        vals = [v for k, vs in per.items() if needle in k for v in vs]
        return (sum(vals) / len(vals), len(vals)) if vals else (None, 0)

    def pick_copy(per):
        # the calibration copy moves exactly 1 GiB each way; take the dispatch closest to it
        best = None
        for k, vs in per.items():
            if "copy" in k.lower() or "elementwise" in k.lower():
                for v in vs:
                    if best is None or abs(v - (1 << 30)) < abs(best - (1 << 30)):
                        best = v
        return best
    fc, wc = pick_copy(res["fetch"]), pick_copy(res["write"])
    lines.append("")
    lines.append(f"calibration copy (1 GiB each way): FETCH_SIZE {fc}, WRITE_SIZE {wc} bytes")
    out = None
    if None not in (fc, wc):
        sf, sw = (1 << 30) / fc, (1 << 30) / wc
        out = {"kernel_source_hash": kernel_source_hash(sources), "fetch_scale": sf, "write_scale": sw,
               "command": command, "kernels": {}}
        lines.append(f"scale: fetch {sf:.4f}, write {sw:.4f}")
        for key, needle in kernels.items():
            fk, nf = pick(res["fetch"], needle)
            wk, nw = pick(res["write"], needle)
            if fk is None or wk is None:
                continue
            rec = {"kernel": needle, "dispatches": min(nf, nw), "fetch_bytes_per_launch": fk * sf,
                   "write_bytes_per_launch": wk * sw, "bytes_per_launch": fk * sf + wk * sw}
            out["kernels"][key] = rec
            lines.append(f"{needle}: {rec['dispatches']} dispatches, fetch {rec['fetch_bytes_per_launch'] / 1e6:.2f} MB"
                         f" + write {rec['write_bytes_per_launch'] / 1e6:.2f} MB = "
                         f"{rec['bytes_per_launch'] / 1e6:.2f} MB per launch")
    return "\n".join(lines) + "\n", out


def summarize_valu(pmc_dir, command):
    """VALU wave instructions per dispatch of the headline kernels from one
    rocprofv3 --pmc run of VALU_COUNTERS: the competing (arithmetic) bound."""
    per = {}
    for r in _read_csvs(pmc_dir, "counter_collection.csv"):
        key = _kernel_key(r["Kernel_Name"])
        if key and r["Counter_Name"] in VALU_COUNTERS:
            per.setdefault(key, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    rec = {"kernel_source_hash": kernel_source_hash(), "command": command, "kernels": {}}
    lines = [f"command: {command}", ""]
    for key, cs in per.items():
        if any(c not in cs for c in VALU_COUNTERS):
            continue
        avg = {c: sum(v) / len(v) for c, v in cs.items()}
        rec["kernels"][key] = {"kernel": KERNELS[key], "dispatches": len(cs[VALU_COUNTERS[0]]),
                               "wave_instr_per_launch": avg}
        lines.append(f"{KERNELS[key]}: {len(cs[VALU_COUNTERS[0]])} dispatches, wave instructions per dispatch")
        lines += [f"  {c:28s} {avg[c]:16.0f}" for c in VALU_COUNTERS]
    if not rec["kernels"]:
        return "\n".join(lines) + "no VALU counters found for the headline kernels\n", None
    return "\n".join(lines) + "\n", rec


WAVE_COUNTERS = (("SQ_WAVES", "SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES", "SQ_WAIT_INST_LDS", "SQ_LDS_BANK_CONFLICT",
                  "SQ_ACTIVE_INST_VALU", "SQ_WAIT_ANY", "SQ_WAIT_INST_ANY"),
                 ("SQ_INSTS_VALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM", "SQ_ACTIVE_INST_LDS", "SQ_ACTIVE_INST_VMEM",
                  "SQ_INST_LEVEL_VMEM", "SQ_INSTS_SALU", "SQ_ACTIVE_INST_ANY"))


def summarize_waves(pmc_dirs, command, name):
    """Wave-state summary of the profiled kernels from two rocprofv3 --pmc runs
    of WAVE_COUNTERS (one pass each): per dispatch, the counters and the
    shares of the summed wave cycles spent issuing VALU, LDS and any
    instruction, waiting on memory or LDS counters, and waiting for an
    instruction to issue."""
    kernels = PROFILE_SETS[name][0]
    per = {}
    for d in pmc_dirs:
        for r in _read_csvs(d, "counter_collection.csv"):
            for key, needle in kernels.items():
                if needle in r["Kernel_Name"]:
                    per.setdefault(key, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    lines = [f"command: {command}", ""]
    for key, cs in per.items():
        avg = {c: sum(v) / len(v) for c, v in cs.items()}
        lines.append(f"{kernels[key]}: {len(cs.get('SQ_WAVES', []))} dispatches, per dispatch")
        lines += [f"  {c:24s} {avg[c]:16.0f}" for c in sorted(avg)]
        wc = avg.get("SQ_WAVE_CYCLES")
        if wc:
            shares = [(c, avg[c] / wc) for c in ("SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_LDS", "SQ_ACTIVE_INST_ANY",
                                                 "SQ_WAIT_ANY", "SQ_WAIT_INST_ANY", "SQ_WAIT_INST_LDS") if c in avg]
            lines.append("  share of SQ_WAVE_CYCLES: " + ", ".join(f"{c[3:]} {v:.3f}" for c, v in shares))
        lines.append("")
    return "\n".join(lines)


def valu_bound(key, avg_launch_us):
    """Arithmetic bound of one launch from its counted wave instructions: the
    issue time if every VALU wave instruction ran back to back on the chip's
    SIMDs (FP64 and unpacked FP32 issue at the same rate), and the FP64 rate
    counting all 64 lanes of each instruction (an upper bound on useful
    flops: masked lanes are counted)."""
    t = _load_record(VALU_FILE)
    if t is None or t.get("stale"):
        return t
    k = t.get("kernels", {}).get(key)
    if k is None:
        return {"missing": key, "file": VALU_FILE}
    w = k["wave_instr_per_launch"]
    fp64 = sum(w[c] for c in VALU_COUNTERS[:4])
    flops = 64 * (w["SQ_INSTS_VALU_ADD_F64"] + w["SQ_INSTS_VALU_MUL_F64"] + 2 * w["SQ_INSTS_VALU_FMA_F64"]
                  + w["SQ_INSTS_VALU_TRANS_F64"])
    floor_us = w["SQ_INSTS_VALU"] * CYCLES_PER_WAVE_INSTR / (MI355X_SIMDS * MI355X_CLOCK_HZ) * 1e6
    ach = flops / (avg_launch_us * 1e-6) / 1e12
    return {"bound": "alu", "unit": "TFLOP/s", "achieved": ach, "peak": FP64_PEAK_TFLOPS,
            "frac": ach / FP64_PEAK_TFLOPS, "fp64_wave_instr_per_launch": fp64,
            "all_valu_wave_instr_per_launch": w["SQ_INSTS_VALU"],
            "valu_issue_floor_us": floor_us, "valu_issue_floor_frac_of_launch": floor_us / avg_launch_us}


def headline_roofline(key, kernel, bytes_per_step, ms, launches, calib):
    """HBM roofline of a headline kernel: algorithmic bytes per launch over its
    average launch time (HIP events on the launch stream, whole timed region)."""
    avg_us = ms * 1e3 / launches
    ach = (bytes_per_step / launches) / (avg_us * 1e-6) / 1e9
    traffic, detail = load_traffic(key)
    return {
        "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
        "traffic": traffic, "kernel": kernel, "algorithmic_bytes_per_launch": bytes_per_step / launches,
        "avg_launch_us": avg_us, "launches_per_step": launches, "traffic_detail": detail,
        "copy_calibration": calib, "frac_of_measured_copy": ach / calib["GBs"],
        "competing_bound": valu_bound(key, avg_us),
    }


def pattern_algorithmic_bytes(nel, p, nrows, nnz):
    """The pattern step: the element map read once, row_ptr and col_idx written
    once (the schedule it also builds is not counted)."""
    return nel * (p + 1) ** 3 * 4 + (nrows + 1) * 4 + nnz * 4


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-sample", type=int, default=16384, help="elements of the all-threads CPU oracle sample")
    ap.add_argument("--cpu-sample-1t", type=int, default=1024, help="elements of the one-thread CPU oracle sample")
    ap.add_argument("--skip-extras", action="store_true")
    ap.add_argument("--backward-only", action="store_true",
                    help="only the copy calibration and the backward leg (for profiling its kernels)")
    ap.add_argument("--h1-2d-only", action="store_true",
                    help="only the copy calibration and the 2D H1 leg (for profiling its kernels)")
    ap.add_argument("--nd-only", action="store_true",
                    help="only the copy calibration and the H(curl) leg (for profiling its kernels)")
    ap.add_argument("--pencil-small", action="store_true",
                    help="FP32 pencil eigenvalues on the 35,937-row mesh instead of the 274,625-row one")
    ap.add_argument("--summarize-profiles", nargs=3, metavar=("STATS_DIR", "FETCH_DIR", "WRITE_DIR"),
                    help="summarise rocprofv3 CSV output of this script (no GPU use)")
    ap.add_argument("--summarize-valu", metavar="PMC_DIR",
                    help="summarise a rocprofv3 --pmc run of the VALU counters (no GPU use)")
    ap.add_argument("--summarize-waves", nargs=2, metavar=("PMC_DIR_A", "PMC_DIR_B"),
                    help="summarise two rocprofv3 --pmc runs of the wave-state counters (no GPU use)")
    ap.add_argument("--profile-command", default="", help="command recorded in the summary")
    ap.add_argument("--profile-name", default="h1_p6_32cubed")
    args = ap.parse_args()
    if args.summarize_valu:
        text, rec = summarize_valu(args.summarize_valu, args.profile_command)
        os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
        with open(os.path.join(ROOT, "profiles", args.profile_name + "_valu.txt"), "w") as f:
            f.write(text)
        if rec is not None:
            with open(os.path.join(ROOT, "profiles", VALU_FILE), "w") as f:
                json.dump(rec, f, indent=1)
        print(text)
        return
    if args.summarize_waves:
        text = summarize_waves(args.summarize_waves, args.profile_command, args.profile_name)
        os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
        with open(os.path.join(ROOT, "profiles", args.profile_name + "_waves.txt"), "w") as f:
            f.write(text)
        print(text)
        return
    if args.summarize_profiles:
        text, traffic = summarize_profiles(*args.summarize_profiles, args.profile_command, args.profile_name)
        os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
        with open(os.path.join(ROOT, "profiles", args.profile_name + ".txt"), "w") as f:
            f.write(text)
        if traffic is not None:
            with open(os.path.join(ROOT, "profiles", args.profile_name + "_traffic.json"), "w") as f:
                json.dump(traffic, f, indent=1)
        print(text)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU path "
              f"(interface-row exchange between element partitions) is not built", file=sys.stderr)
        sys.exit(2)

    import torch

    import meshgen
    import paper_2210_12253_amd as lor

    dev = torch.device("cuda:0")
    if args.backward_only:
        log("copy calibration")
        calib = copy_calibration(torch, dev)
        log("backward")
        print(json.dumps({"backward": bench_backward(lor, meshgen, args, dev), "copy_calibration": calib}))
        return
    if args.nd_only:
        log("copy calibration")
        calib = copy_calibration(torch, dev)
        log("H(curl)")
        print(json.dumps({"nd": bench_nd(lor, meshgen, args, dev), "copy_calibration": calib}))
        return
    if args.h1_2d_only:
        log("copy calibration")
        calib = copy_calibration(torch, dev)
        log("2D H1")
        print(json.dumps({"h1_2d": bench_2d(lor, meshgen, args, dev), "copy_calibration": calib}))
        return
    log("building the headline inputs")
    m = meshgen.config_mesh("c3_h1_p6_curved")
    p, nel, ndofs = m["p"], m["nel"], m["ndofs"]
    ed = torch.from_numpy(m["elem_dofs"]).to(dev)
    x = torch.from_numpy(m["coords"]).to(dev)
    k64 = m["kappa"].to(dev)
    k32 = k64.float()
    torch.cuda.synchronize()

    log("copy calibration")
    calib = copy_calibration(torch, dev)

    log("pattern")
    # the library's code objects load at its first launch in the process: a
    # one-element mesh takes that cost out of the per-mesh figure
    tiny = meshgen.cartesian_mesh(1, p, 0.0)
    lor.lor_pattern(lor.LOR_H1, p, torch.from_numpy(tiny["elem_dofs"]).to(dev), tiny["ndofs"])
    torch.cuda.synchronize()
    t = time.perf_counter()
    pat = lor.lor_pattern(lor.LOR_H1, p, ed, ndofs)
    torch.cuda.synchronize()
    t_pattern = (time.perf_counter() - t) * 1e3
    t_rebuild = []
    for _ in range(3):  # the same mesh again, its buffers now in the allocator's cache
        t = time.perf_counter()
        lor.lor_pattern(lor.LOR_H1, p, ed, ndofs)
        torch.cuda.synchronize()
        t_rebuild.append((time.perf_counter() - t) * 1e3)
    nnz = pat.nnz
    v64 = torch.empty(nnz, dtype=torch.float64, device=dev)
    v32 = torch.empty(nnz, dtype=torch.float32, device=dev)
    owner = pat.owner
    kind = "owner" if owner else "colored"
    launches = 1 if owner else pat.ncolors

    def f64(kernel="auto"):
        return lor.lor_assemble_h1(pat, ed, x, k64, 1.0, out=v64, kernel=kernel)

    def f32(kernel="auto"):
        return lor.lor_assemble_h1(pat, ed, x, k32, 1.0, dtype=torch.float32, fp64_fallback=True, out=v32,
                                   kernel=kernel)

    # Untimed ramp before the warm-up steps: the first tens of milliseconds of
    # sustained load run at lower clocks (measured: the first timed FP64 block
    # 0.89 ms per step against 0.82 ms for the same kernel a few seconds later)
    log("ramp")
    ramp_ms = ramp(f64, 200.0)
    log("timing fp64")
    ms64 = time_it(f64, args.steps, args.warmup)
    log("timing fp32")
    ms32 = time_it(f32, args.steps, args.warmup)
    med64 = step_median(f64, max(args.steps, 20))
    med32 = step_median(f32, max(args.steps, 20))
    b64 = algorithmic_bytes_h1(nel, p, ndofs, nnz, 8)
    b32 = algorithmic_bytes_h1(nel, p, ndofs, nnz, 4)
    kname64 = "k_h1_owner<6,double,double> (one dispatch per step)" if owner else \
        "k_h1_assemble<6,double,double> (one dispatch per element colour)"
    kname32 = "k_h1_owner<6,float,float> (one dispatch per step)" if owner else \
        "k_h1_assemble<6,float,float> (one dispatch per element colour)"
    out = {
        "metric": "LOR assembly MDOF/s & %HBM roofline, H1 p=6: FP64 vs FP32; backward MDOF/s",
        "value": ndofs / (ms64 * 1e-3) / 1e6,
        "unit": "MDOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms64,
        "ms_per_step_median": med64,
        "untimed_ramp_ms": ramp_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "H1 diffusion+mass LOR assembly, p=6, 32^3 curved hexes (amp 0.1h), "
                        "log-normal kappa sigma=2, beta=1",
            "rows": ndofs, "nnz": nnz, "elements": nel, "subelements": nel * p ** 3,
            "kernel": kind, "launches_per_step": launches,
        },
        "roofline": headline_roofline(f"{kind}_f64", kname64, b64, ms64, launches, calib),
        "fp32": {
            "ms_per_step": ms32,
            "ms_per_step_median": med32,
            "value": ndofs / (ms32 * 1e-3) / 1e6,
            "unit": "MDOF/s",
            "speedup_vs_fp64": ms64 / ms32,
            "roofline": headline_roofline(f"{kind}_f32", kname32, b32, ms32, launches, calib),
        },
        "pattern": {"ms": t_pattern, "ms_cold_total": t_pattern + ms64,
                    "ms_rebuild_median": sorted(t_rebuild)[1], "ncolors": pat.ncolors,
                    "owner_schedule": owner,
                    "roofline": roofline_of(pattern_algorithmic_bytes(nel, p, ndofs, nnz), t_pattern)},
    }
    if owner:
        log("timing the coloured kernel")
        msc64 = time_it(lambda: f64("colored"), args.steps, args.warmup)
        msc32 = time_it(lambda: f32("colored"), args.steps, args.warmup)
        out["colored"] = {
            "f64": {"ms": msc64, "value": ndofs / (msc64 * 1e-3) / 1e6, "unit": "MDOF/s",
                    "roofline": headline_roofline("colored_f64", "k_h1_assemble<6,double,double>", b64, msc64,
                                                  pat.ncolors, calib)},
            "f32": {"ms": msc32, "value": ndofs / (msc32 * 1e-3) / 1e6, "unit": "MDOF/s",
                    "roofline": headline_roofline("colored_f32", "k_h1_assemble<6,float,float>", b32, msc32,
                                                  pat.ncolors, calib)},
            "launches_per_step": pat.ncolors,
            "owner_speedup_f64": msc64 / ms64, "owner_speedup_f32": msc32 / ms32,
        }

    if not args.skip_extras:
        out["elimination"] = bench_elim(lor, meshgen, m, pat, v64, args, dev)
        out["unstructured"] = bench_unstructured(lor, meshgen, m, pat, ms64, args, dev)
        out["aux"] = bench_aux(lor, meshgen, pat, args, dev)
        out["backward"] = bench_backward(lor, meshgen, args, dev)
        out["nd"] = bench_nd(lor, meshgen, args, dev)
        out["rt"] = bench_rt(lor, meshgen, args, dev)
        out["h1_2d"] = bench_2d(lor, meshgen, args, dev)
        out["h1_unstructured_mesh"] = bench_trisplit(lor, meshgen, args, dev)
        log("fp32 pencil eigenvalues")
        out["fp32"]["pencil_eigs"] = bench_fp32_pencil(lor, meshgen, dev, small=args.pencil_small)
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(m, args.cpu_sample, args.cpu_sample_1t)
    print(json.dumps(out))


def _pcg(B, diag, u, tol, maxit):
    """Jacobi-preconditioned conjugate gradients for B x = u (B SPD, CSR)."""
    import torch
    x = torch.zeros_like(u)
    r = u.clone()
    z = r / diag
    p = z.clone()
    rz = torch.dot(r, z)
    stop = float(tol * torch.linalg.norm(u))
    for it in range(1, maxit + 1):
        ap = torch.mv(B, p)
        a = rz / torch.dot(p, ap)
        x += a * p
        r -= a * ap
        if it % 25 == 0 and float(torch.linalg.norm(r)) <= stop:
            return x, it
        z = r / diag
        rz2 = torch.dot(r, z)
        p = z + (rz2 / rz) * p
        rz = rz2
    return x, maxit


def pencil_extreme_eigs(row_ptr, col_idx, v64, v32, n, steps=30, cg_tol=1e-10, cg_maxit=20000):
    """Extreme eigenvalues of the pencil A64 x = lambda A32 x (the FP64 LOR
    matrix preconditioned by its FP32 form, both on the same pattern) by
    Lanczos on the device: lambda - 1 = mu are the eigenvalues of
    A32^-1 (A64 - A32), self-adjoint in the A32 inner product; each step
    solves with A32 by Jacobi-preconditioned CG, and the basis is fully
    re-orthogonalised.  The difference is scaled by 2^24 (the FP32 rounding
    level).  Ritz values lie inside the spectrum, so the reported extremes are
    lower bounds of |lambda - 1|; the residual estimate |beta_k s_k| / |theta|
    of each extreme Ritz pair is reported, and `converged` says whether both
    are below 1e-6."""
    import numpy as np
    import torch
    rp = row_ptr.to(torch.int64)
    ci = col_idx.to(torch.int64)
    a32 = v32.to(torch.float64)
    scale = 2.0 ** 24
    B = torch.sparse_csr_tensor(rp, ci, a32, (n, n))
    E = torch.sparse_csr_tensor(rp, ci, (v64 - a32) * scale, (n, n))
    rows = torch.repeat_interleave(torch.arange(n, device=rp.device), rp[1:] - rp[:-1])
    diag = torch.zeros(n, dtype=torch.float64, device=rp.device)
    diag.index_add_(0, rows, torch.where(rows == ci, a32, torch.zeros_like(a32)))
    del rows
    g = torch.Generator(device="cpu").manual_seed(0)
    v = torch.randn(n, generator=g, dtype=torch.float64).to(rp.device)
    bv = torch.mv(B, v)
    nrm = torch.sqrt(torch.dot(v, bv))
    V, BV = [v / nrm], [bv / nrm]
    alpha, beta, cg_its = [], [], []
    for j in range(steps):
        u = torch.mv(E, V[j])
        w, its = _pcg(B, diag, u, cg_tol, cg_maxit)
        cg_its.append(its)
        alpha.append(float(torch.dot(V[j], u)))
        Vm, BVm = torch.stack(V, 1), torch.stack(BV, 1)
        for _ in range(2):          # full re-orthogonalisation in the A32 inner product
            w = w - Vm @ (BVm.T @ w)
        bw = torch.mv(B, w)
        bj = float(torch.sqrt(torch.dot(w, bw)))
        beta.append(bj)
        if bj == 0.0:
            break
        V.append(w / bj)
        BV.append(bw / bj)
    k = len(alpha)
    T = np.diag(alpha) + np.diag(beta[:k - 1], 1) + np.diag(beta[:k - 1], -1)
    th, S = np.linalg.eigh(T)
    res = {"max": abs(beta[k - 1] * S[-1, -1]) / max(abs(th[-1]), 1e-300),
           "min": abs(beta[k - 1] * S[-1, 0]) / max(abs(th[0]), 1e-300)}
    return {"lambda_max_minus_1": float(th[-1]) / scale, "one_minus_lambda_min": -float(th[0]) / scale,
            "lanczos_steps": k, "cg_iterations_per_solve": int(np.median(cg_its)), "relative_residual": res,
            "converged": all(r <= 1e-6 for r in res.values())}


def bench_fp32_pencil(lor, meshgen, dev, small=False):
    """FP32-form quality on the p=4, 16^3 curved mesh with kappa = exp(2 N(0,1))
    per subelement (seed 0) and beta = 1 (274,625 rows); small=True takes the
    p=4, 8^3 mesh (35,937 rows)."""
    import torch
    n_el = 8 if small else 16
    m = meshgen.cartesian_mesh(n_el, 4, 0.1 / n_el)
    k = meshgen.kappa_field(m["nel"], 4, 2.0, seed=0).to(dev)
    beta = 1.0
    ed = torch.from_numpy(m["elem_dofs"]).to(dev)
    x = torch.from_numpy(m["coords"]).to(dev)
    pat = lor.lor_pattern(lor.LOR_H1, 4, ed, m["ndofs"])
    v64 = lor.lor_assemble_h1(pat, ed, x, k, beta)
    v32 = lor.lor_assemble_h1(pat, ed, x, k.float(), beta, dtype=torch.float32, fp64_fallback=True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    res = pencil_extreme_eigs(pat.row_ptr, pat.col_idx, v64, v32, m["ndofs"])
    res["seconds"] = time.perf_counter() - t
    res["workload"] = (f"H1 p=4, {n_el}^3 curved hexes, kappa sigma=2, beta=1 ({m['ndofs']} rows); "
                       f"Lanczos on the device, FP32 values from the default kernel")
    return res


def bench_backward(lor, meshgen, args, dev):
    import torch
    try:
        m = meshgen.config_mesh("c5_h1_p4_backward")
        ed = torch.from_numpy(m["elem_dofs"]).to(dev)
        x = torch.from_numpy(m["coords"]).to(dev)
        pat = lor.lor_pattern(lor.LOR_H1, m["p"], ed, m["ndofs"])
        res = {}
        for name, dt in (("f64", torch.float64), ("f32", torch.float32)):
            k = m["kappa"].to(dev, dt)
            gv = meshgen.cotangent(8, pat.nnz, seed=1).to(dev, dt)
            ws = torch.empty(lor.load_library().lor_backward_workspace(m["p"], m["nel"], 8, lor.LOR_F64), dtype=torch.uint8,
                             device=dev)
            ms = time_it(lambda: lor.lor_assemble_backward(pat, ed, x, k, 1.0, gv, dtype=dt, workspace=ws),
                         args.steps, args.warmup)
            fwd = time_it(lambda: lor.lor_assemble_h1(pat, ed, x, k, 1.0, dtype=dt), args.steps, args.warmup)
            roof = roofline_of(algorithmic_bytes_backward(m["nel"], m["p"], m["ndofs"], pat.nnz, dt.itemsize, 8), ms)
            # HBM bytes of the backward kernel (and of the vertex gather that
            # follows it) from the committed counter summary, if it is current
            tb, detail = load_traffic(f"backward_{name}", "backward_p4_16cubed_b8")
            tg, _ = load_traffic("gather_vertices", "backward_p4_16cubed_b8")
            roof.update(kernel=f"k_h1_backward<4,{'double' if name == 'f64' else 'float'}> + k_gather_vertices",
                        traffic=None if tb is None or tg is None else tb + tg, traffic_detail=detail)
            res[name] = {"ms": ms, "value": 8 * m["ndofs"] / (ms * 1e-3) / 1e6, "unit": "MDOF/s (batch*rows)",
                         "forward_batch8_ms": fwd, "roofline": roof}
        res["workload"] = "backward of H1 p=4, 16^3 curved hexes, batch 8 kappa fields"
        res["speedup_f32_vs_f64"] = res["f64"]["ms"] / res["f32"]["ms"]
        return res
    except lor.LorError as e:
        return {"error": str(e)}


def elim_algorithmic_bytes(torch, pat, marker, ness, elt, batch=1):
    """Bytes step A4 has to move when the rows and columns of `ness` essential
    dofs (marker [nrows] bool, on the device) are eliminated: the essential
    list (4 B each), the marker (cleared: 1 B per row; set: 1 B per essential
    dof), two row pointers per essential row, its column indices and values
    (written), the marker byte of every off-diagonal column, and per
    transposed entry (c, i) with c not essential: two row pointers, the one
    column index that identifies it and its value (written)."""
    rp = pat.row_ptr.to(torch.int64)
    rows = torch.repeat_interleave(torch.arange(pat.nrows, device=rp.device), rp[1:] - rp[:-1])
    ci = pat.col_idx.to(torch.int64)
    in_row = marker[rows]
    e_rows = int(in_row.sum())
    e_cols = int((marker[ci] & ~marker[rows]).sum())
    del rows, ci, in_row
    return (4 * ness + pat.nrows + ness + 8 * ness + (4 + elt * batch) * e_rows + (e_rows - ness)
            + (8 + 4 + elt * batch) * e_cols), e_rows, e_cols


def bench_elim(lor, meshgen, m, pat, v64, args, dev):
    """Step A4 on the benchmark matrix: the boundary vertices of the cube are
    eliminated (diagonal set to 1) from the assembled FP64 values.  The call
    is idempotent, so repeated calls on the same values time the same work."""
    import torch
    try:
        bnd = torch.from_numpy(meshgen.boundary_vertices(m["n"], m["p"])).to(dev)
        mk = torch.empty(pat.nrows, dtype=torch.uint8, device=dev)
        lor.lor_eliminate_bc(pat, v64, bnd, "one", marker=mk)
        torch.cuda.synchronize()
        bytes_, e_rows, e_cols = elim_algorithmic_bytes(torch, pat, mk.bool(), bnd.numel(), 8)
        fe = lambda: lor.lor_eliminate_bc(pat, v64, bnd, "one", marker=mk)  # noqa: E731
        ms_ev = time_it(fe, args.steps, args.warmup)
        ms = time_graph(fe, args.steps)
        return {
            "ms": ms, "ms_back_to_back": ms_ev, "value": bnd.numel() / (ms * 1e-3) / 1e6,
            "unit": "M essential dofs/s",
            "workload": "eliminate the 221,186 boundary vertices of the H1 p=6 32^3 matrix (FP64, diagonal 1)",
            "essential": bnd.numel(), "row_entries": e_rows, "column_entries": e_cols,
            "roofline": dict(roofline_of(bytes_, ms),
                             kernels="k_elim_clear + k_elim_mark + k_elim_rows<double>"),
        }
    except lor.LorError as e:
        return {"error": str(e)}


def bench_aux(lor, meshgen, pat_h1, args, dev):
    """The auxiliary data of Step S1.2: the discrete gradient of the H(curl)
    p=3 24^3 mesh, and the LOR coordinate vector of the headline mesh (32^3,
    p=6) from degree-2 curved mesh nodes (interpolation to an E-vector, then
    E-vector to T-vector).  Algorithmic bytes per dof: gradient 4 (row
    pointer of the schedule) + 4 (first incidence) + 4 (edge map) + 8 (two
    vertex ids) + 4 + 8 + 16 (row pointer, columns, FP64 values written) =
    48 B per edge; interpolation reads the nodes and writes the E-vector once;
    E->T reads 4 + 4 (row pointer, first incidence) + 24 (E-vector entry) and
    writes 24 B per dof.  "ms" is the device time from graph replays of 20
    captured calls; "ms_back_to_back" the plain event timing of consecutive
    calls, which includes the binding's host launch overhead."""
    import torch

    def rl(bytes_, ms):
        return roofline_of(bytes_, ms)
    res = {}
    try:
        m = meshgen.config_mesh("c4_nd_p3_curved")
        ee = torch.from_numpy(m["elem_edges"]).to(dev)
        ed = torch.from_numpy(m["elem_dofs"]).to(dev)
        pat = lor.lor_pattern(lor.LOR_ND, 3, ee, m["nedges"])
        ned = m["nedges"]
        rp = torch.empty(ned + 1, dtype=torch.int32, device=dev)
        ci = torch.empty(2 * ned, dtype=torch.int32, device=dev)
        v = torch.empty(2 * ned, dtype=torch.float64, device=dev)
        fg = lambda: lor.lor_discrete_gradient(pat, ed, ee, m["ndofs"], out=(rp, ci, v))  # noqa: E731
        ms_ev = time_it(fg, args.steps, args.warmup)
        ms = time_graph(fg, args.steps)
        res["gradient"] = {"ms": ms, "ms_back_to_back": ms_ev, "value": ned / (ms * 1e-3) / 1e9,
                           "unit": "GDOF/s (edges)",
                           "workload": "discrete gradient, H(curl) p=3 24^3 (1,151,064 edges), FP64",
                           "roofline": rl(48 * ned, ms)}
        fm, nf = meshgen.face_map(24, 3)
        fm = torch.from_numpy(fm).to(dev)
        ws = torch.empty(nf, dtype=torch.int32, device=dev)
        crp = torch.empty(nf + 1, dtype=torch.int32, device=dev)
        cci = torch.empty(4 * nf, dtype=torch.int32, device=dev)
        cv = torch.empty(4 * nf, dtype=torch.float64, device=dev)
        fc = lambda: lor.lor_discrete_curl(3, ee, fm, ned, nf, workspace=ws, out=(crp, cci, cv), device=dev)  # noqa: E731
        ms_c_ev = time_it(fc, args.steps, args.warmup)
        ms_c = time_graph(fc, args.steps)
        # face map read twice (owner pass, row pass: 4 + 4 per face incidence,
        # two incidences per interior face) + owner fill/atomic/read 12 +
        # 4 edge-map entries 16 + row pointer 4 + columns 16 + FP64 values 32
        res["curl"] = {"ms": ms_c, "ms_back_to_back": ms_c_ev, "value": nf / (ms_c * 1e-3) / 1e9,
                       "unit": "GDOF/s (faces)",
                       "workload": "discrete curl, p=3 24^3 (%d faces), FP64" % nf,
                       "roofline": rl(int(8 * fm.numel() + (12 + 16 + 4 + 16 + 32) * nf), ms_c)}
        del pat, rp, ci, v, ee, ed, fm, ws, crp, cci, cv
        n, p, q = 32, 6, 2
        X = torch.from_numpy(meshgen.ho_nodes(n, q, 0.1)).to(dev)
        E = torch.empty((n ** 3, (p + 1) ** 3, 3), dtype=torch.float64, device=dev)
        T = torch.empty((pat_h1.nrows, 3), dtype=torch.float64, device=dev)
        fi = lambda: lor.lor_interp_nodes(X, p, q, out=E)  # noqa: E731
        ft = lambda: lor.lor_evec_to_tvec(pat_h1, E, out=T)  # noqa: E731
        ms_i_ev, ms_t_ev = time_it(fi, args.steps, args.warmup), time_it(ft, args.steps, args.warmup)
        ms_i, ms_t = time_graph(fi, args.steps), time_graph(ft, args.steps)
        res["interp_nodes"] = {"ms": ms_i, "ms_back_to_back": ms_i_ev,
                               "value": E.shape[0] * E.shape[1] / (ms_i * 1e-3) / 1e9,
                               "unit": "GDOF/s (E-vector points)",
                               "workload": "degree-2 curved nodes -> p=6 Gauss-Lobatto lattice, 32^3 elements",
                               "roofline": rl(X.numel() * 8 + E.numel() * 8, ms_i)}
        res["evec_to_tvec"] = {"ms": ms_t, "ms_back_to_back": ms_t_ev, "value": pat_h1.nrows / (ms_t * 1e-3) / 1e9,
                               "unit": "GDOF/s (vertices)",
                               "workload": "E-vector of 32^3 p=6 elements -> 7,189,057 vertex coordinates",
                               "roofline": rl(56 * pat_h1.nrows, ms_t)}
    except lor.LorError as e:
        res["error"] = str(e)
    return res


def bench_trisplit(lor, meshgen, args, dev):
    """The headline form (H1 p=6, kappa sigma 2, beta 1) on an unstructured mesh
    of the same size: the unit square cut into 16 x 16 cells, two triangles per
    cell, three quadrilaterals per triangle (vertex valence 3, 4 and 6),
    extruded in 21 layers: 32,256 hexahedra, 7,071,487 rows."""
    import torch
    try:
        log("unstructured mesh: building inputs")
        m = meshgen.config_mesh("c8_h1_p6_trisplit")
        ed = torch.from_numpy(m["elem_dofs"]).to(dev)
        x = torch.from_numpy(m["coords"]).to(dev)
        k64 = m["kappa"].to(dev)
        k32 = k64.float()
        torch.cuda.synchronize()
        t = time.perf_counter()
        pat = lor.lor_pattern(lor.LOR_H1, 6, ed, m["ndofs"])
        torch.cuda.synchronize()
        t_pattern = (time.perf_counter() - t) * 1e3
        res = {"workload": "H1 diffusion+mass LOR assembly, p=6, triangle-split unstructured hex mesh "
                           "(16x16 cells, 21 layers, valence 3/4/6), log-normal kappa sigma=2, beta=1",
               "elements": m["nel"], "rows": m["ndofs"], "nnz": pat.nnz, "ncolors": pat.ncolors,
               "pattern_ms": t_pattern}
        out64 = torch.empty(pat.nnz, dtype=torch.float64, device=dev)
        out32 = torch.empty(pat.nnz, dtype=torch.float32, device=dev)
        for name, kap, dt, out in (("f64", k64, torch.float64, out64), ("f32", k32, torch.float32, out32)):
            log(f"unstructured mesh: timing {name}")
            ms = time_it(lambda: lor.lor_assemble_h1(pat, ed, x, kap, 1.0, dtype=dt, out=out,
                                                     fp64_fallback=dt == torch.float32),
                         args.steps, args.warmup)
            res[name] = {"ms": ms, "value": m["ndofs"] / (ms * 1e-3) / 1e6, "unit": "MDOF/s",
                         "roofline": roofline_of(algorithmic_bytes_h1(m["nel"], 6, m["ndofs"], pat.nnz,
                                                                      dt.itemsize), ms)}
        del out64, out32, pat
        torch.cuda.empty_cache()
        return res
    except lor.LorError as e:
        return {"error": str(e)}


def bench_unstructured(lor, meshgen, m, pat, ms_macro, args, dev):
    """The comparator of the paper's assembly results on the headline mesh:
    the explicit LOR mesh (refined element map, timed once) and the generic
    per-element assembly with atomic adds (timed like the macro kernel)."""
    import torch
    try:
        ed = torch.from_numpy(m["elem_dofs"]).to(dev)
        x = torch.from_numpy(m["coords"]).to(dev)
        k = m["kappa"].to(dev)
        sub = torch.empty((m["nel"] * m["p"] ** 3, 8), dtype=torch.int32, device=dev)
        ms_map = time_it(lambda: lor.lor_refine_map(m["p"], ed, device=dev, out=sub), 3, 1)
        out = torch.empty(pat.nnz, dtype=torch.float64, device=dev)
        ms = time_it(lambda: lor.lor_assemble_h1_unstructured(pat, sub, x, k, m["beta"], out=out),
                     args.steps, args.warmup)
        return {"ms": ms, "value": m["ndofs"] / (ms * 1e-3) / 1e6, "unit": "MDOF/s",
                "refine_map_ms": ms_map, "macro_speedup": ms / ms_macro,
                "workload": "H1 p=6 32^3 as 7,077,888 explicit trilinear elements, FP64, atomic adds"}
    except lor.LorError as e:
        return {"error": str(e)}


def bench_2d(lor, meshgen, args, dev):
    """The paper's 2D workload (Section 4.1): H1 p=6 on 512^2 quadrilaterals,
    9,443,329 rows and 84,953,089 nonzeros."""
    import torch
    try:
        m = meshgen.config_mesh("c7_h1_2d_p6_curved")
        ed = torch.from_numpy(m["elem_dofs"]).to(dev)
        x = torch.from_numpy(m["coords"]).to(dev)
        pat = lor.lor_pattern(lor.LOR_H1_2D, 6, ed, m["ndofs"])
        res = {"kernel": "owner" if pat.owner else "colored", "colored": {}}
        for name, dt in (("f64", torch.float64), ("f32", torch.float32)):
            k = m["kappa"].to(dev, dt)
            out = torch.empty(pat.nnz, dtype=dt, device=dev)
            fb = dt == torch.float32
            ms = time_it(lambda: lor.lor_assemble_h1_2d(pat, ed, x, k, m["beta"], dtype=dt, fp64_fallback=fb, out=out),
                         args.steps, args.warmup)
            roof = roofline_of(algorithmic_bytes_2d(m["nel"], 6, m["ndofs"], pat.nnz, dt.itemsize), ms)
            # HBM bytes of the kernel that ran, from the committed counter
            # summary, if it is current
            key = ("owner2d_" if pat.owner else "colored2d_") + name
            tb, detail = load_traffic(key, "h1_2d_p6_512sq")
            roof.update(traffic=tb, traffic_detail=detail)
            res[name] = {"ms": ms, "value": m["ndofs"] / (ms * 1e-3) / 1e6, "unit": "MDOF/s", "roofline": roof}
            if pat.owner:  # the element-coloured kernel on the same mesh, for comparison
                mc = time_it(lambda: lor.lor_assemble_h1_2d(pat, ed, x, k, m["beta"], dtype=dt, fp64_fallback=fb,
                                                            out=out, kernel="colored"), args.steps, args.warmup)
                res["colored"][name] = {"ms": mc, "owner_speedup": mc / ms}
        res["workload"] = "2D H1 LOR assembly, p=6, 512^2 curved quadrilaterals, kappa sigma=2, beta=1"
        res["rows"], res["nnz"], res["ncolors"] = m["ndofs"], pat.nnz, pat.ncolors
        return res
    except lor.LorError as e:
        return {"error": str(e)}


def bench_rt(lor, meshgen, args, dev):
    import torch
    try:
        m = meshgen.config_mesh("c6_rt_p3_curved")
        ed = torch.from_numpy(m["elem_dofs"]).to(dev)
        fm = torch.from_numpy(m["elem_faces"]).to(dev)
        x = torch.from_numpy(m["coords"]).to(dev)
        pat = lor.lor_pattern(lor.LOR_RT, m["p"], fm, m["nfaces"])
        res = {"kernel": "owner" if pat.owner else "colored", "colored": {}}
        for name, dt in (("f64", torch.float64), ("f32", torch.float32)):
            k = m["kappa"].to(dev, dt)
            out = torch.empty(pat.nnz, dtype=dt, device=dev)
            fb = dt == torch.float32
            ms = time_it(lambda: lor.lor_assemble_rt(pat, ed, fm, x, k, 1.0, m["ndofs"], dtype=dt, fp64_fallback=fb,
                                                     out=out), args.steps, args.warmup)
            p = m["p"]
            res[name] = {"ms": ms, "value": m["nfaces"] / (ms * 1e-3) / 1e6, "unit": "MDOF/s",
                         "roofline": roofline_of(algorithmic_bytes_vec(m["nel"], p, m["nfaces"], m["ndofs"], pat.nnz,
                                                                       dt.itemsize, 3 * p * p * (p + 1)), ms)}
            if pat.owner:  # the element-coloured kernel on the same mesh, for comparison
                mc = time_it(lambda: lor.lor_assemble_rt(pat, ed, fm, x, k, 1.0, m["ndofs"], dtype=dt, fp64_fallback=fb,
                                                         out=out, kernel="colored"), args.steps, args.warmup)
                res["colored"][name] = {"ms": mc, "owner_speedup": mc / ms}
        res["workload"] = "H(div) LOR assembly, p=3, 24^3 curved hexes, kappa sigma=1, beta=1"
        res["rows"], res["nnz"], res["ncolors"] = m["nfaces"], pat.nnz, pat.ncolors
        return res
    except lor.LorError as e:
        return {"error": str(e)}


def bench_nd(lor, meshgen, args, dev):
    import torch
    try:
        m = meshgen.config_mesh("c4_nd_p3_curved")
        ed = torch.from_numpy(m["elem_dofs"]).to(dev)
        ee = torch.from_numpy(m["elem_edges"]).to(dev)
        x = torch.from_numpy(m["coords"]).to(dev)
        pat = lor.lor_pattern(lor.LOR_ND, m["p"], ee, m["nedges"])
        res = {"kernel": "owner" if pat.owner else "colored", "colored": {}}
        for name, dt in (("f64", torch.float64), ("f32", torch.float32)):
            k = m["kappa"].to(dev, dt)
            out = torch.empty(pat.nnz, dtype=dt, device=dev)
            fb = dt == torch.float32
            ms = time_it(lambda: lor.lor_assemble_nd(pat, ed, ee, x, k, 1.0, m["ndofs"], dtype=dt, fp64_fallback=fb,
                                                     out=out), args.steps, args.warmup)
            p = m["p"]
            roof = roofline_of(algorithmic_bytes_vec(m["nel"], p, m["nedges"], m["ndofs"], pat.nnz, dt.itemsize,
                                                     3 * p * (p + 1) ** 2), ms)
            if pat.owner:
                # HBM bytes of the three launches (one per edge direction) from
                # the committed counter summary, if it is current
                parts = [load_traffic(f"nd_owner_{name}_{d}", "nd_p3_24cubed") for d in range(3)]
                tb = sum(t for t, _ in parts) if all(t is not None for t, _ in parts) else None
                roof.update(traffic=tb, traffic_detail=[dd for _, dd in parts])
            res[name] = {"ms": ms, "value": m["nedges"] / (ms * 1e-3) / 1e6, "unit": "MDOF/s", "roofline": roof}
            if pat.owner:  # the element-coloured kernel on the same mesh, for comparison
                mc = time_it(lambda: lor.lor_assemble_nd(pat, ed, ee, x, k, 1.0, m["ndofs"], dtype=dt, fp64_fallback=fb,
                                                         out=out, kernel="colored"), args.steps, args.warmup)
                res["colored"][name] = {"ms": mc, "owner_speedup": mc / ms}
        res["workload"] = "H(curl) LOR assembly, p=3, 24^3 curved hexes, kappa sigma=1, beta=1"
        res["rows"], res["nnz"], res["ncolors"] = m["nedges"], pat.nnz, pat.ncolors
        return res
    except lor.LorError as e:
        return {"error": str(e)}


if __name__ == "__main__":
    main()
