#!/usr/bin/env python3
"""Throughput benchmark of the axisymmetric multiphase LBM step on one MI355X.

A step is one time step of the whole method over every node of the workload:
pull streaming, moments, FP64 EOS and pseudopotential, Kupershtokh force with the
exact-difference shift, axisymmetric force correction and source terms, BGK.
Default workload: the 256-member droplet ensemble in FP32 storage, all members in
one launch per step (per stream group), replayed as hipGraph chunks of up to 10
steps (an even chunk that fits the requested step count, so short runs replay too;
longer chunks start the second stream group later, by the host time of launching the
first group's graph, which costs more than the fewer launches save).  The same line
also reports the single large domain (16384 x 8192) in FP32 and in FP64.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import dataclasses
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
# per node and step: read the 9 populations once and write them once
BYTES_PER_NODE = {"f32": 2 * 9 * 4, "f64": 2 * 9 * 8}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def code_text(src: str) -> str:
    """C++ source without comments and with whitespace collapsed: what the compiler sees."""
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    return " ".join(src.split())


def kernel_source_hash() -> str:
    """Hash of the kernel code (comments and layout excluded), which keys the committed
    byte counters to the code they were taken from."""
    h = hashlib.sha256()
    for f in ("lbm_kernels.hip", "lbm_axi_internal.h"):
        with open(os.path.join(ROOT, "paper_1512_01977_amd", "csrc", f), encoding="utf-8") as fh:
            h.update(code_text(fh.read()).encode())
    return h.hexdigest()[:16]


def traffic_record(workload: str, dtype: str):
    """The committed rocprofv3 counter summary of this workload (HBM bytes per launch and
    the launch shape they were counted in), or None when there is none or the kernel
    source changed since it was taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            data = json.load(fh)
    except (OSError, ValueError):
        return None
    rec = data.get(f"{workload}:{dtype}")
    if not rec or rec.get("kernel_hash") != kernel_source_hash():
        return None
    return rec


def same_launch(a, b) -> bool:
    """Two launch-shape dicts name the same launch (a missing stream count reads as 1)."""
    if not a or not b:
        return False
    keys = set(a) | set(b)
    return all(a.get(k, 1 if k == "streams" else None) == b.get(k, 1 if k == "streams" else None)
               for k in keys)


def settle_device(wl, launch, seconds=0.3):
    """Bring the GPU out of its idle power state before a form's warm-up steps: from idle, a
    step takes ~25 % longer for the first ~100 ms of load, and again after a second of idling
    (the same state then ramps again; a memory-bound copy kernel only half warms it).  A
    throwaway copy of the workload, in the same launch shape, is stepped for `seconds` and
    discarded: the measured state still gets exactly its warm-up steps, and nothing of the
    settling is timed."""
    from paper_1512_01977_amd import lbm
    tmp = lbm.LbmAxi(wl.params if len(wl.params) > 1 else wl.params[0],
                     wl.rho0 if len(wl.params) > 1 else wl.rho0[0], precision=wl.precision)
    try:
        tmp.set_launch(**launch)
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < seconds:
            tmp.step(10)
            tmp.sync()
    finally:
        tmp.close()


def run_form(wl, steps, warmup, graph_chunk, shape, label):
    """shape: "profiled" runs the launch shape the committed byte counters were taken in
    (autotuning when there is none for the current kernel), "tune" autotunes unless the
    tuning cache has this size class, "cached" takes the cache or the library's default."""
    import torch
    from paper_1512_01977_amd import lbm, tuning

    dtype = "f32" if wl.precision == lbm.PREC_FP32 else "f64"
    log(f"[bench] {label}: {wl.name} {dtype}, {wl.nodes} nodes, {len(wl.params)} instance(s)")
    t0 = time.perf_counter()
    sim = lbm.LbmAxi(wl.params if len(wl.params) > 1 else wl.params[0],
                     wl.rho0 if len(wl.params) > 1 else wl.rho0[0], precision=wl.precision)
    log(f"[bench] {label}: state on the device in {time.perf_counter() - t0:.1f} s")
    rec = traffic_record(wl.name, dtype)
    if isinstance(shape, dict):
        sim.set_launch(**shape)
        launch, source = sim.get_launch(), "given"
    elif shape == "profiled" and rec and rec.get("launch"):
        sim.set_launch(**rec["launch"])
        launch, source = sim.get_launch(), "profiled"
    else:
        launch = tuning.choose_launch(sim, wl, tune=shape != "cached", log=log)
        source = "tuner" if shape != "cached" else "cached"
    log(f"[bench] {label}: launch {launch} ({source})")
    if graph_chunk:
        sim.set_graph_chunk(graph_chunk)
    settle_device(wl, launch)
    sim.step(warmup)
    sim.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev_ms = sim.step_timed(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sim.sync()
    mass = float(sim.mass().sum())
    sim.close()
    nodes = wl.nodes
    per_launch_s = ev_ms / 1e3 / steps
    achieved = BYTES_PER_NODE[dtype] * nodes / per_launch_s / 1e9
    # the counted bytes belong to one launch shape: reported only when that shape ran
    traffic = rec.get("bytes_per_launch") if rec and same_launch(rec.get("launch"), launch) else None
    # the bytes the profiler counted crossing the HBM interface in one step, over the same time
    counted = traffic / per_launch_s / 1e9 if traffic else None
    res = {
        "workload": wl.name, "dtype": dtype, "nodes": nodes, "steps": steps,
        "graph_chunk": graph_chunk,
        "ms_per_step": wall * 1e3 / steps, "kernel_ms_per_step": ev_ms / steps,
        "MLUPS": nodes * steps / wall / 1e6,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic},
        "counted_hbm_GBps": counted,
        "counted_hbm_frac": counted / HBM_PEAK_GBPS if counted else None,
        "launch": launch, "launch_source": source, "mass_after": mass,
    }
    log(f"[bench] {label}: {res['MLUPS']:.0f} MLUPS, {achieved:.0f} GB/s algorithmic "
        f"({100 * achieved / HBM_PEAK_GBPS:.1f}% of HBM peak)"
        + (f", {counted:.0f} GB/s counted ({100 * counted / HBM_PEAK_GBPS:.1f}%)" if counted else ""))
    return res


def graph_chunk_for(steps: int, limit: int) -> int:
    """The captured chunk for a run of `steps` steps: an even number of steps (a chunk must
    end on the buffer it starts from) of at most `limit`, chosen to leave the fewest steps
    to eager launches and, among those, the longest; 0 (eager only) below two steps."""
    best = 0
    for c in range(2, min(limit, steps) + 1, 2):
        if best == 0 or (steps % c, -c) < (steps % best, -best):
            best = c
    return best


def guo_workload():
    from paper_1512_01977_amd import inputs, lbm, workloads
    nz, nr = 16384, 8192
    p = dataclasses.replace(workloads.cs_params(nz, nr, 0.8, 0.8), forcing=lbm.FORCING_GUO)
    rv, rl = workloads.coexistence(p)
    rho = inputs.droplet(nz, nr, rv, rl, 2000.0, zc=nz / 2, width=10.0, eps=0.02, noise=1e-4, seed=5)
    return workloads.Workload(f"large_droplet_{nz}x{nr}_guo", [p], [rho], lbm.PREC_FP32, 100)


def cpu_baseline(wl, budget_s=15.0, max_nodes=2_000_000, threads=None):
    """The CPU oracle, as it is, on a bounded sample of the same workload: the first
    members of the workload (or a band of rows of a single domain) for a few steps, on
    all host threads or on the given number of them."""
    import numpy as np

    import oracle as O
    from paper_1512_01977_amd import lbm

    def oparams(p):
        return O.Params(nz=p.nz, nr=p.nr, tau=p.tau, eos=p.eos, T=p.T, eos_a=p.eos_a,
                        eos_b=p.eos_b, eos_R=p.eos_R, lam=p.lam, A=p.A, axisym=p.axisym,
                        faxis_sound=p.faxis_sound, bc_top=p.bc_top, gz=p.gz, forcing=p.forcing)

    members = []
    if len(wl.params) > 1:
        for p, r in zip(wl.params, wl.rho0):
            members.append((oparams(p), r))
            if sum(q.nz * q.nr for q, _ in members) >= max_nodes:
                break
    else:
        p = wl.params[0]
        rows = max(8, min(p.nr, max_nodes // p.nz))
        q = oparams(p)
        q.nr = rows
        members.append((q, np.ascontiguousarray(wl.rho0[0][:rows])))
    states = [(q, O.init(q, r)) for q, r in members]
    nodes = sum(q.nz * q.nr for q, _ in states)
    all_threads = O.threads()
    if threads:
        O.set_threads(threads)
    try:
        t0 = time.perf_counter()
        for q, f in states:
            O.step(q, f, 1)
        per_step = time.perf_counter() - t0
        steps = max(1, int(budget_s / max(per_step, 1e-6)))
        t0 = time.perf_counter()
        for q, f in states:
            O.step(q, f, steps)
        dt = time.perf_counter() - t0
        cores = O.threads()
    finally:
        O.set_threads(all_threads)
    return {"value": nodes * steps / dt / 1e6, "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": f"{len(states)} member(s) of {wl.name} ({nodes} nodes) for {steps} steps, "
                      f"FP64 C oracle, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="batch", choices=["batch", "large", "wave", "mode2", "static"])
    ap.add_argument("--precision", default=None, choices=["fp32", "fp64"])
    ap.add_argument("--forms", default="all", choices=["all", "main"],
                    help="all: also time the large single domain in FP32 and FP64")
    ap.add_argument("--graph-chunk", type=int, default=10,
                    help="longest captured chunk of steps (an even chunk <= this that fits --steps is used)")
    ap.add_argument("--tune", action="store_true",
                    help="autotune the launch shape (unless cached) instead of running the shape "
                         "the committed byte counters were taken in")
    ap.add_argument("--no-tune", action="store_true", help="use the cached or default launch shape")
    ap.add_argument("--launch", default=None, metavar="JSON",
                    help="launch shape of the main form as a JSON object of lbm_axi_launch fields")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--stream-copy", type=int, default=0, metavar="BYTES",
                    help="only run the reference copy kernel on BYTES and print its GB/s")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library steps each domain on one GPU and has "
              "no multi-GPU path; run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU (the HIP library has no CPU path).", file=sys.stderr)
        sys.exit(2)
    from paper_1512_01977_amd import lbm, workloads

    if args.stream_copy:
        gbps = lbm.lbm_axi_stream_copy(args.stream_copy, max(1, args.steps))
        print(json.dumps({"stream_copy_bytes": args.stream_copy, "iters": args.steps,
                          "GBps": gbps}), flush=True)
        return

    prec = {"fp32": lbm.PREC_FP32, "fp64": lbm.PREC_FP64}
    default_prec = {"batch": "fp32", "large": "fp32", "wave": "fp32", "mode2": "fp32",
                    "static": "fp64"}
    main_prec = prec[args.precision or default_prec[args.workload]]
    t_all = time.perf_counter()
    wl = workloads.REGISTRY[args.workload](precision=main_prec)
    chunk = graph_chunk_for(args.steps, args.graph_chunk)
    shape = "cached" if args.no_tune else "tune" if args.tune else "profiled"
    main_res = run_form(wl, args.steps, args.warmup, chunk,
                        json.loads(args.launch) if args.launch else shape, "main")

    forms = [main_res]
    if args.forms == "all":
        for w_name, p_name, steps in (("large", "fp32", 100), ("large", "fp64", 60)):
            if w_name == args.workload and prec[p_name] == main_prec:
                continue
            w = workloads.REGISTRY[w_name](precision=prec[p_name])
            forms.append(run_form(w, steps, 4, 0, shape, f"{w_name}-{p_name}"))
            del w
        # the 16384 x 8192 domain in FP32 with Guo's forcing (Sec. 2.1) in place of the
        # exact-difference method, at T/T_c = 0.8 (density ratio ~14): Guo's term does not
        # hold the ratio-1e3 droplet of the other forms
        try:
            forms.append(run_form(guo_workload(), 100, 4, 0, shape, "large-fp32-guo"))
        except Exception as exc:  # a form that fails is reported, the others still count
            log(f"[bench] large-fp32-guo: failed ({exc})")

    # practical HBM ceiling: a plain 1 GiB device-to-device copy kernel, read + write bytes
    copy_gbps = lbm.lbm_axi_stream_copy(1 << 30, 10)
    log(f"[bench] copy kernel: {copy_gbps:.0f} GB/s ({100 * copy_gbps / HBM_PEAK_GBPS:.1f}% of 8 TB/s)")

    cpu = cpu1 = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline: timing the oracle on a bounded sample")
        cpu = cpu_baseline(wl)
        log(f"[bench] cpu baseline: {cpu['value']:.2f} MLUPS on {cpu['cores']} threads")
        cpu1 = cpu_baseline(wl, budget_s=8.0, max_nodes=250_000, threads=1)
        log(f"[bench] cpu baseline: {cpu1['value']:.2f} MLUPS on {cpu1['cores']} thread")

    out = {
        "metric": "MLUPS + achieved HBM GB/s (% of peak), FP64 plain vs FP32/batched, 1 GPU",
        "value": main_res["MLUPS"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": main_res["dtype"],
        "data": "synthetic (seeded initial conditions of the paper's validation set-ups)",
        "config": {"workload": wl.name, "nodes": wl.nodes, "instances": len(wl.params),
                   "graph_chunk": chunk, "launch": main_res["launch"],
                   "launch_source": main_res["launch_source"]},
        "roofline": main_res["roofline"],
        "stream_copy_GBps": copy_gbps,
        "cpu_baseline": cpu,
        "cpu_baseline_1core": cpu1,
        "counted_hbm_GBps": main_res["counted_hbm_GBps"],
        "forms": [{k: f[k] for k in ("workload", "dtype", "MLUPS", "ms_per_step", "kernel_ms_per_step",
                                     "graph_chunk", "roofline", "counted_hbm_GBps", "launch",
                                     "launch_source")}
                  for f in forms],
        "wall_s": time.perf_counter() - t_all,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
