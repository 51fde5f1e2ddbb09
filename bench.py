"""Throughput of the fluctuating two-component D3Q19 + sphere step on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W]
                [--workload large|single|ensemble|paper|parity|adjoint] [--no-forms] [--no-cpu]

Prints ONE JSON line: MLUPS (replica node updates per second / 1e6, both
components of a node counted once) of the chosen workload, by default the
large channel (192 x 192 x 1024, FP16 relative-deviation storage, FP32
arithmetic), with all inputs resident in HBM, plus
  roofline:     the main kernel's algorithmic HBM bytes per launch (read +
                write of 2 x 19 populations per node) over its mean duration,
                measured with HIP events on the library stream during the
                timed region, against the 8 TB/s HBM peak; `traffic` is the
                HBM bytes per launch from the committed rocprofv3 counters
                when they were taken on the current kernel sources in this
                launch shape;
  valu:         the same kernel's VALU wave-instructions per launch (from
                those counters) over the live duration, against the issue
                peak of 256 CUs x 4 SIMDs x one wave64 instruction per 4
                cycles at 2.4 GHz (614.4 G/s), and its VALU-busy fraction;
  forms:        (default workload) the batched ensemble and the adjoint form
                against the plain single run, timed in the same invocation:
                plain 64x64x256 single-run MLUPS, the 192-replica ensemble's
                MLUPS and its ratio to it, and the adjoint call's cost per
                step over plain steps of its 48x48x192 channel;
  cpu_baseline: the FP64 CPU oracle (OpenMP over z-planes, all the threads
                OMP_NUM_THREADS allows) on a bounded sample of the workload.
--workload adjoint times lbm_adjoint (1000 steps, checkpoint every 50) on
the 48x48x192 channel instead.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# VALU issue peak of MI355X: 256 CUs x 4 SIMDs of 16 lanes, one wave64
# instruction per SIMD every 4 cycles, 2.4 GHz (39.3 T lane operations/s; the
# 157.3 TFLOP/s FP32 vector figure counts a packed FMA as 4 flops per lane)
N_SIMD = 1024
CLOCK_HZ = 2.4e9
VALU_PEAK_GINSTR = N_SIMD * CLOCK_HZ / 4 / 1e9
KERNEL_SOURCES = ["paper_1909_01092_amd/csrc/lbm_kernels_impl.h",
                  "paper_1909_01092_amd/csrc/lbm_math.h",
                  "paper_1909_01092_amd/csrc/lbm_types.h"]


def timing_every(steps):
    """HIP events around every main launch of a short timed region, every
    tenth of a long one (events cost the small single run about 4% a step)."""
    return 1 if steps < 100 else 10


def kernel_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def workload(name):
    from paper_1909_01092_amd import workloads as w
    if name == "single":
        return ([w.SINGLE_RUN], "fp32", "single run 64x64x256 channel, FP32 deviation storage, "
                "R=8, kT=1e-5, g=1e-4, G=1.5, tau=1")
    if name == "ensemble":
        return (w.ensemble(), "fp32", "ensemble 128x(32x32x128,R=4)+32x(24x24x96,R=3)+"
                "32x(48x48x192,R=6), FP32 deviations, kT=1e-5, g=5e-5")
    if name == "large":
        return ([w.LARGE], "fp16", "large single run 192x192x1024, FP16 relative deviations, "
                "R=16, kT=1e-4, g=1e-4, G=1.5, tau=1")
    if name == "paper":
        return ([w.paper_box()], "fp32", "paper geometry: closed 60x60x900 box, rho_A/rho_B = 2.21/0.09, "
                "G = 1.5, R = 8, kT = 1e-4, g = 5e-6, FP32 deviations")
    if name == "parity":
        return ([w.PARITY_SMALL], "fp64", "parity channel 24x24x48, FP64, R=4, kT=1e-5")
    raise SystemExit(f"unknown workload {name}")


def profile_counters(name, block, zchunk):
    """The committed rocprofv3 counters of this workload's main kernel in
    this launch shape (profiles/k_main_<name>_counters.json), if they were
    taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"k_main_{name}_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_hash") != kernel_hash():
        return None
    for e in [d] + d.get("shapes", []):
        if e.get("block") == block and e.get("zchunk") == zchunk:
            return e
    return None


def traffic_from_profile(name, block, zchunk):
    """HBM bytes per launch of the main kernel from the committed counters
    (None unless they match the current sources and this launch shape)."""
    e = profile_counters(name, block, zchunk)
    return e.get("hbm_bytes_per_launch") if e else None


def valu_from_profile(name, block, zchunk, kern_ms):
    """VALU wave-instructions per launch (SQ_INSTS_VALU) and active VALU
    cycles (SQ_ACTIVE_INST_VALU, x 4 per wave instruction) from the committed
    counters, over the live kernel duration."""
    e = profile_counters(name, block, zchunk)
    if not e or "sq_insts_valu" not in e or not kern_ms:
        return None
    s = kern_ms * 1e-3
    achieved = e["sq_insts_valu"] / s / 1e9
    return {"bound": "alu", "achieved": round(achieved, 1), "peak": VALU_PEAK_GINSTR,
            "unit": "G wave64 VALU instr/s", "frac": round(achieved / VALU_PEAK_GINSTR, 4),
            "busy": round(e["sq_active_inst_valu"] * 4 / (N_SIMD * CLOCK_HZ * s), 4),
            "instr_per_launch": e["sq_insts_valu"]}


def make_sim(torch, reps, prec, args=None, tune_steps=100):
    from paper_1909_01092_amd.sim import Simulation
    sim = Simulation(reps, precision=prec, device="cuda:0", stream=torch.cuda.Stream())
    if args is not None and args.zchunk:
        sim.set_launch(args.block, args.zchunk)
    elif tune_steps > 0:
        sim.autotune(steps_per_trial=tune_steps, preserve=False)  # before the warm-up
    return sim


def timed_steps(torch, sim, steps, warmup, every=None):
    """Warm-up, then `steps` plain-launch steps bracketed by device syncs;
    returns (seconds, mean main-kernel ms, timed launches)."""
    sim.step(warmup)
    sim.sync()
    sim.timing(timing_every(steps) if every is None else every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.sync()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    kern_ms, nlaunch = sim.timing_read()
    sim.timing(False)
    return el, kern_ms, nlaunch


def nodes_of(reps):
    return sum(q["nx"] * q["ny"] * q["nz"] for q in reps)


def forms_comparison(torch, steps_single=2000, steps_ensemble=200, steps_adjoint=1000):
    """The batched ensemble and the adjoint form against the plain single-run
    path, each timed here (autotuned launch shapes, plain launches)."""
    out = {}
    reps, prec, desc = workload("single")
    sim = make_sim(torch, reps, prec, tune_steps=100)
    el, _, _ = timed_steps(torch, sim, steps_single, 100, every=0)
    plain = nodes_of(reps) * steps_single / el / 1e6
    sim.close()
    out["plain"] = {"workload": desc, "MLUPS": round(plain, 1), "steps": steps_single}
    reps, prec, desc = workload("ensemble")
    sim = make_sim(torch, reps, prec, tune_steps=50)
    el, _, _ = timed_steps(torch, sim, steps_ensemble, 20, every=0)
    ens = nodes_of(reps) * steps_ensemble / el / 1e6
    # the same steps replayed as HIP graphs of 50 steps (one graph launch per
    # 50 steps of every replica); the first replay instantiates the graph
    sim.set_graph(50)
    el_g, _, _ = timed_steps(torch, sim, steps_ensemble, 50, every=0)
    ens_g = nodes_of(reps) * steps_ensemble / el_g / 1e6
    sim.close()
    del sim
    out["ensemble"] = {"workload": desc, "MLUPS": round(ens, 1), "steps": steps_ensemble,
                       "vs_plain": round(ens / plain, 3),
                       "graph": {"steps_per_graph": 50, "MLUPS": round(ens_g, 1),
                                 "vs_plain_launches": round(ens_g / ens, 3)}}
    from paper_1909_01092_amd import workloads as w
    p = w.ADJOINT
    sim = make_sim(torch, [p], "fp32", tune_steps=100)
    sim.adjoint(50, 50)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.adjoint(steps_adjoint, 50)
    torch.cuda.synchronize()
    el_adj = time.perf_counter() - t0
    el_fwd, _, _ = timed_steps(torch, sim, steps_adjoint, 0, every=0)
    sim.close()
    out["adjoint"] = {"workload": "adjoint 48x48x192 channel, R=6, kT=1e-5, g=5e-5, FP32, 1000 steps, "
                                  "checkpoint every 50",
                      "ms_per_step": round(el_adj * 1e3 / steps_adjoint, 5),
                      "plain_ms_per_step": round(el_fwd * 1e3 / steps_adjoint, 5),
                      "cost_vs_plain": round(el_adj / el_fwd, 3)}
    return out


def oracle_threads():
    """Threads the oracle may use: OMP_NUM_THREADS when set, else every CPU."""
    v = os.environ.get("OMP_NUM_THREADS", "")
    return int(v) if v.isdigit() and int(v) > 0 else (os.cpu_count() or 1)


def cpu_baseline(reps, budget_s=15.0, max_nodes=4_000_000, slab_nz=64):
    """FP64 oracle (OpenMP over z-planes) on the first replica of the
    workload, or on a 64-plane slab of it when the replica has more than
    `max_nodes` nodes: whole steps until the budget is spent (at least one)."""
    from oracle import oracle as om
    from paper_1909_01092_amd import workloads as w
    p = dict(reps[0])
    what = "one replica"
    if p["nx"] * p["ny"] * p["nz"] > max_nodes:
        p = w.full(dict(p, nz=slab_nz, X0=None))
        what = f"a {slab_nz}-plane slab (same cross-section, sphere and parameters)"
    threads = om.set_threads(oracle_threads())
    t0 = time.perf_counter()
    sim = om.OracleSim(p)
    t_init = time.perf_counter() - t0
    steps = 0
    t0 = time.perf_counter()
    while True:
        sim.step(1)
        steps += 1
        el = time.perf_counter() - t0
        if el > budget_s or el / steps * (steps + 1) > 2 * budget_s:
            break
    N = p["nx"] * p["ny"] * p["nz"]
    return {"value": round(N * steps / el / 1e6, 4), "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"{steps} step(s) of {what} of the workload, {p['nx']}x{p['ny']}x{p['nz']}, in "
                      f"FP64 on {threads} thread(s) ({el:.1f} s; init {t_init:.1f} s excluded)"}

# algorithmic bytes per node of the adjoint node kernel (FP32): recorded
# moments (8 values) and adjoint state after the step (8) read, adjoint state
# before the step (8) and node-force adjoint (6) written; the neighbours'
# values are the same arrays read again through the caches
ADJ_LOCAL_BYTES_PER_NODE = (8 + 8 + 8 + 6) * 4


def adjoint_bench(torch, args, steps, segment=50):
    from oracle.oracle import OracleSim
    from paper_1909_01092_amd import workloads as w
    from paper_1909_01092_amd.sim import Simulation
    p = w.ADJOINT
    nodes = p["nx"] * p["ny"] * p["nz"]
    sim = Simulation(p, precision="fp32", device="cuda:0", stream=torch.cuda.Stream())
    if args.zchunk:
        sim.set_launch(args.block, args.zchunk)
    elif args.autotune > 0:
        sim.autotune(steps_per_trial=args.autotune, preserve=False)
    block, cz = sim.get_launch()
    sim.adjoint(min(args.warmup, 50), segment)  # warm-up
    sim.sync()
    sim.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J, grad = sim.adjoint(steps, segment)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    kern_ms, nlaunch = sim.timing_read()
    sim.timing(False)
    # one segment: every step's moments recorded (8 FP32 per node and step),
    # so the forward steps run once
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.adjoint(steps, steps)
    torch.cuda.synchronize()
    el_one = time.perf_counter() - t0
    t0 = time.perf_counter()
    sim.step(steps)
    sim.sync()
    el_fwd = time.perf_counter() - t0
    unstable = sim.particle_state(0, allow_unstable=True)["unstable"]
    sim.close()
    bpl = ADJ_LOCAL_BYTES_PER_NODE * nodes
    achieved = bpl / (kern_ms * 1e-3) / 1e9
    out = {
        "metric": "MLUPS (2-comp D3Q19), adjoint form vs plain", "value": round(nodes * steps / el / 1e6, 2),
        "unit": "MLUPS", "n_gpus": 1, "steps": steps, "warmup": min(args.warmup, 50),
        "ms_per_step": round(el * 1e3 / steps, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "adjoint 48x48x192 channel, R=6, kT=1e-5, g=5e-5, G=1.5, FP32 "
                               f"deviations, checkpoint every {segment} steps",
                   "replicas": 1, "nodes": nodes, "precision": "fp32", "block": block, "zchunk": cz,
                   "unstable": unstable},
        "adjoint": {"J": J, "grad_g_xyz_G_drho": [float(v) for v in grad], "segment": segment,
                    "plain_ms_per_step": round(el_fwd * 1e3 / steps, 5),
                    "cost_vs_plain": round(el / el_fwd, 3),
                    "one_segment_ms_per_step": round(el_one * 1e3 / steps, 5),
                    "one_segment_cost_vs_plain": round(el_one / el_fwd, 3)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": "k_adj_local",
                     "kernel_ms": round(kern_ms, 5), "launches": nlaunch, "bytes_per_launch": bpl},
    }
    if not args.no_cpu:
        from oracle import oracle as om
        k = 2
        om.set_threads(1)  # the oracle's adjoint is sequential
        osim = OracleSim(p)
        t0 = time.perf_counter()
        osim.adjoint(k)
        oel = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(nodes * k / oel / 1e6, 4), "unit": "MLUPS", "cores": 1,
                               "kind": "oracle",
                               "sample": f"oracle adjoint of {k} steps of the same 48x48x192 channel "
                                         f"in FP64 ({oel:.1f} s, every state stored)"}
    print(json.dumps(out), flush=True)


def copy_calibration(torch, mib, steps, warmup):
    """Plain device-to-device copy of `mib` MiB (the runtime's copy kernel):
    under rocprofv3 its FETCH_SIZE / WRITE_SIZE per dispatch give the scale
    between those counters and bytes actually moved.  Also timed: a streaming
    elementwise kernel (dst = src * 1, one read and one write per element),
    the faster of the two and the bandwidth ceiling quoted for read + write
    kernels."""
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(max(warmup, 1)):
        dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    moved = 2 * n * 4
    for _ in range(max(warmup, 1)):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        torch.mul(src, 1.0, out=dst)
    e1.record()
    torch.cuda.synchronize()
    ms_s = e0.elapsed_time(e1) / steps
    print(json.dumps({"copy_mib": mib, "ms_per_copy": round(ms, 5), "bytes_moved": moved,
                      "GB/s": round(moved / (ms * 1e-3) / 1e9, 1),
                      "stream_ms": round(ms_s, 5), "stream_GB/s": round(moved / (ms_s * 1e-3) / 1e9, 1)}),
          flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default 200; adjoint: 1000)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="large")
    ap.add_argument("--zchunk", type=int, default=0, help="fixed main-kernel z-chunk (skips the autotuner)")
    ap.add_argument("--block", type=int, default=256, help="main-kernel block with --zchunk")
    ap.add_argument("--autotune", type=int, default=100,
                    help="steps per candidate of the launch-shape autotuner (0: library default shape)")
    ap.add_argument("--graph", type=int, default=0, help="steps per HIP graph (0: plain launches)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the ensemble / adjoint against plain comparison")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="instead of the step: time a plain device copy of this many MiB "
                         "(calibrates the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the library runs on exactly one GPU (the hot path is one GPU's share); "
              "a multi-GPU run is not supported", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_mib:
        copy_calibration(torch, args.copy_mib, args.steps or 2000, args.warmup)
        return
    if args.workload == "adjoint":
        adjoint_bench(torch, args, args.steps or 1000)
        return
    args.steps = args.steps or 200
    reps, prec, desc = workload(args.workload)
    sim = make_sim(torch, reps, prec, args, tune_steps=args.autotune)
    block, cz = sim.get_launch()
    if args.graph:
        sim.set_graph(args.graph)
    el, kern_ms, nlaunch = timed_steps(torch, sim, args.steps, args.warmup,
                                       every=0 if args.graph else None)
    state = [sim.particle_state(r, allow_unstable=True) for r in range(len(reps))]
    unstable = any(s["unstable"] for s in state)
    nodes = nodes_of(reps)
    mlups = nodes * args.steps / el / 1e6
    step_bytes = sim.step_bytes()
    sim.close()
    del sim
    roof = valu = None
    if kern_ms:
        achieved = step_bytes / (kern_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic_from_profile(args.workload, block, cz),
                "kernel": "k_main", "kernel_ms": round(kern_ms, 5), "launches": nlaunch,
                "bytes_per_launch": step_bytes}
        valu = valu_from_profile(args.workload, block, cz, kern_ms)
    out = {
        "metric": "MLUPS (2-comp D3Q19)", "value": round(mlups, 2), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(el * 1e3 / args.steps, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "fp16": "f16-storage/f32"}[prec], "data": "synthetic",
        "config": {"workload": desc, "replicas": len(reps), "nodes": nodes, "precision": prec,
                   "block": block, "zchunk": cz, "autotuned": not args.zchunk and args.autotune > 0,
                   "graph_steps": args.graph, "unstable": unstable},
        "roofline": roof,
        "valu": valu,
    }
    if args.workload == "large" and not args.no_forms:
        out["forms"] = forms_comparison(torch)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(reps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
