"""Throughput of the fluctuating two-component D3Q19 + sphere step on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload single|ensemble|large|paper|parity|adjoint]

Prints ONE JSON line: MLUPS (replica node updates per second / 1e6, both
components of a node counted once) for the chosen workload with all inputs
resident in HBM, plus
  roofline:     the main kernel's algorithmic HBM bytes per launch (read +
                write of 2 x 19 populations per node) over its mean duration,
                measured with HIP events on the library stream during the
                timed region, against the 8 TB/s HBM peak;
  cpu_baseline: the FP64 CPU oracle timed on a bounded sample of the same
                workload on this host (single thread).
--workload adjoint times lbm_adjoint (1000 steps, checkpoint every 50) on
the 48x48x192 channel instead: MLUPS of the whole adjoint call (forward
sweep, replays and reverse sweep; each step counted once), its cost against
plain steps of the same channel, and the roofline of the adjoint's node
kernel.
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
TIMING_EVERY = 10
KERNEL_SOURCES = ["paper_1909_01092_amd/csrc/lbm_kernels_impl.h",
                  "paper_1909_01092_amd/csrc/lbm_math.h",
                  "paper_1909_01092_amd/csrc/lbm_types.h"]


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
                "R=16, kT=1e-4, g=1e-4")
    if name == "paper":
        return ([w.paper_box()], "fp32", "paper geometry: closed 60x60x900 box, rho_A/rho_B = 2.21/0.09, "
                "G = 1.5, R = 8, kT = 1e-4, g = 5e-6, FP32 deviations")
    if name == "parity":
        return ([w.PARITY_SMALL], "fp64", "parity channel 24x24x48, FP64, R=4, kT=1e-5")
    raise SystemExit(f"unknown workload {name}")


def traffic_from_profile(name, block, zchunk):
    """HBM bytes per launch of the main kernel from the committed rocprofv3
    counter summary, if it was taken on the current kernel sources in the
    same launch shape (the summary's own shape, or one of its per-shape
    entries)."""
    path = os.path.join(ROOT, "profiles", f"k_main_{name}_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_hash") != kernel_hash():
        return None
    for e in [d] + d.get("shapes", []):
        if e.get("block") == block and e.get("zchunk") == zchunk:
            return e.get("hbm_bytes_per_launch")
    return None


def plain_comparison(torch, mlups, steps=1000):
    """The batched form against the plain single-run path: MLUPS of the
    64x64x256 single run (autotuned, plain launches) timed here, and the
    ratio of the batched throughput to it."""
    from paper_1909_01092_amd.sim import Simulation
    reps, prec, _ = workload("single")
    sim = Simulation(reps, precision=prec, device="cuda:0", stream=torch.cuda.Stream())
    sim.autotune(steps_per_trial=10, preserve=False)
    sim.step(100)
    sim.sync()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.sync()
    el = time.perf_counter() - t0
    sim.close()
    plain = reps[0]["nx"] * reps[0]["ny"] * reps[0]["nz"] * steps / el / 1e6
    return {"plain_single_run_MLUPS": round(plain, 1), "batched_over_plain": round(mlups / plain, 3)}


def cpu_baseline(reps, budget_s=15.0):
    """FP64 oracle on the first replica of the workload, whole steps until the
    budget is spent (at least one step)."""
    from oracle.oracle import OracleSim
    p = reps[0]
    t0 = time.perf_counter()
    sim = OracleSim(p)
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
    return {"value": round(N * steps / el / 1e6, 4), "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"{steps} step(s) of one {p['nx']}x{p['ny']}x{p['nz']} replica of the same "
                      f"workload in FP64 ({el:.1f} s; init {t_init:.1f} s excluded)"}


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
        k = 2
        osim = OracleSim(p)
        t0 = time.perf_counter()
        osim.adjoint(k)
        oel = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(nodes * k / oel / 1e6, 4), "unit": "MLUPS", "cores": 1,
                               "kind": "oracle",
                               "sample": f"oracle adjoint of {k} steps of the same 48x48x192 channel "
                                         f"in FP64 ({oel:.1f} s, every state stored)"}
    print(json.dumps(out), flush=True)


def friction_study(torch, steps=12000, tail=1000, wettability=False):
    """Deterministic confinement friction (kT = 0): terminal settling
    velocity of spheres of several d/L in the square channel, one replica per
    radius in one context, and the friction factor relative to Stokes,
    c_m = F_ext / (3 pi eta d U), F_ext = V (rho_p - rho_tot) g (Sec. 3 eq. fp),
    eta = rho_tot nu, nu = (tau - 1/2) / 3.  wettability: the paper's mixture
    (rho 2.21 / 0.09) with each of its three wettabilities instead of the
    0.95 / 0.05 mixture with a neutral sphere."""
    import math
    from paper_1909_01092_amd import workloads as w
    from paper_1909_01092_amd.sim import Simulation
    reps = w.friction_wettability(steps_cap=steps) if wettability else w.friction(steps_cap=steps)
    sim = Simulation(reps, precision="fp32", device="cuda:0", stream=torch.cuda.Stream())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.sync()
    el = time.perf_counter() - t0
    rows = []
    for r, q in enumerate(reps):
        u = sim.u_series(r)[:, 2]
        U, Uprev = u[-tail:].mean(), u[-2 * tail:-tail].mean()
        R = q["radius"]
        rho = q["rho0"][0] + q["rho0"][1]
        Fext = 4.0 / 3.0 * math.pi * R ** 3 * (q["rho_p"] - rho) * q["g"][2]
        eta = rho * (q["tau_shear"] - 0.5) / 3.0
        rows.append({"wettability": q.get("wettability", "neutral"), "drho": q["wet_drho"],
                     "R": R, "d_over_L": 2 * R / q["nx"], "U": float(U),
                     "drift": float(abs(U - Uprev) / abs(U)), "c_m": float(Fext / (3 * math.pi * eta * 2 * R * U)),
                     "Re": float(abs(U) * 2 * R * 3.0 / (q["tau_shear"] - 0.5))})
    nodes = sum(q["nx"] * q["ny"] * q["nz"] for q in reps)
    sim.close()
    mix = f"rho {reps[0]['rho0'][0]:g} / {reps[0]['rho0'][1]:g}"
    return {"study": "confinement friction, kT = 0", "mixture": mix,
            "channel": f"{w.FRICTION_L}x{w.FRICTION_L}x{w.FRICTION_LZ}",
            "steps": steps, "mean_over_last": tail, "seconds": round(el, 3),
            "MLUPS": round(nodes * steps / el / 1e6, 1), "rows": rows}


def interface_height(rho, X, clear):
    """Height of the flat A|B interface far from the sphere: the zero of the
    composition rho_A - rho_B averaged over the (x, y) columns farther than
    `clear` from the sphere's axis, by linear interpolation between planes
    (A below, B above)."""
    import numpy as np
    nz, ny, nx = rho.shape[1:]
    yy, xx = np.mgrid[0:ny, 0:nx]
    far = np.hypot(xx - X[0], yy - X[1]) > clear
    phi = (rho[0] - rho[1])[:, far].mean(1)
    k = np.where((phi[:-1] > 0) & (phi[1:] <= 0))[0]
    if len(k) != 1:
        return float("nan")
    k = int(k[0])
    return k + phi[k] / (phi[k] - phi[k + 1])


def wetting_study(torch, steps=30000, tail=10000, every=500):
    """Contact angle of the wetting layer against Delta rho.  A sphere free to
    move (no noise, no driving) at a flat interface between the two demixed
    phases settles where the interface meets its surface at the contact
    angle theta; with the A phase below, cos theta_A = (z_i - Z) / R (Young's
    condition on a sphere, the interface staying flat).  Z and the far-field
    interface height z_i are averaged over the last `tail` steps (sampled
    every `every` steps): the staircase sphere keeps moving by a fraction of
    a node.  The paper's three wettabilities (Sec. 3: theta = 120.5, 90,
    55 degrees, measured in the majority phase A) are then read off by
    linear interpolation."""
    import math
    import numpy as np
    from paper_1909_01092_amd import workloads as w
    from paper_1909_01092_amd.sim import Simulation
    reps = w.wetting()
    sim = Simulation(reps, precision="fp32", device="cuda:0", stream=torch.cuda.Stream())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps - tail)
    h = [[] for _ in reps]
    for _ in range(tail // every):
        sim.step(every)
        for r, q in enumerate(reps):
            X = sim.particle_state(r)["X"]
            rho, _ = sim.fields(r)
            h[r].append(interface_height(rho, X, q["radius"] + 8.0) - X[2])
    sim.sync()
    el = time.perf_counter() - t0
    rows = []
    for r, q in enumerate(reps):
        d = np.array(h[r])
        c = float(d.mean() / q["radius"])
        rows.append({"drho": q["wet_drho"], "zi_minus_Z": float(d.mean()), "spread": float(d.std()),
                     "cos_theta": c, "theta_deg": math.degrees(math.acos(max(-1.0, min(1.0, c))))})
    cos = np.array([x["cos_theta"] for x in rows])
    drho = np.array([x["drho"] for x in rows])
    calib = {}
    if np.all(np.diff(cos) > 0):
        for th in (120.5, 90.0, 55.0):
            calib[f"{th:g}"] = float(np.interp(math.cos(math.radians(th)), cos, drho))
    nodes = sum(q["nx"] * q["ny"] * q["nz"] for q in reps)
    sim.close()
    return {"study": "contact angle of the wetting layer, kT = 0",
            "box": f"{w.WETTING_N}^3 closed, R = {w.WETTING_R:g}, rho {w.PAPER_RHO0}",
            "steps": steps, "averaged_over_last": tail, "seconds": round(el, 3),
            "MLUPS": round(nodes * steps / el / 1e6, 1), "rows": rows, "drho_for_theta": calib}


def interface_study(torch, steps=30000, tail=10000, every=500):
    """A sphere at a flat interface pushed towards the A phase by a body force
    (the paper's suggested follow-up: settling at the interface between two
    immiscible fluids), for the paper's three wettabilities.  A trapped sphere
    settles where capillarity balances F_ext; its offset from the interface,
    z_i - Z, is averaged over the last `tail` steps.  A sphere whose centre
    gets more than R + 2 below the interface plane has detached and sinks into
    A (it then reaches the bottom wall, which ends that replica)."""
    import numpy as np
    from paper_1909_01092_amd import workloads as w
    from paper_1909_01092_amd.sim import Simulation
    reps = w.interface_trap()
    sim = Simulation(reps, precision="fp32", device="cuda:0", stream=torch.cuda.Stream())
    z0 = (w.WETTING_N - 1) / 2.0
    detached = [None] * len(reps)
    h = [[] for _ in reps]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        sim.step(every)
        done += every
        for r, q in enumerate(reps):
            if detached[r] is not None:
                continue
            st = sim.particle_state(r, allow_unstable=True)
            if st["unstable"] or st["X"][2] < z0 - q["radius"] - 2.0:
                detached[r] = done
            elif done > steps - tail:
                rho, _ = sim.fields(r)
                h[r].append(interface_height(rho, st["X"], q["radius"] + 8.0) - st["X"][2])
    sim.sync()
    el = time.perf_counter() - t0
    rows = []
    for r, q in enumerate(reps):
        row = {"wettability": q["wettability"], "drho": q["wet_drho"], "F_ext": q["force"],
               "detached_by_step": detached[r]}
        if detached[r] is None:
            d = np.array(h[r])
            row.update({"zi_minus_Z": float(d.mean()), "spread": float(d.std())})
        rows.append(row)
    nodes = sum(q["nx"] * q["ny"] * q["nz"] for q in reps)
    sim.close()
    return {"study": "sphere at a flat interface under a body force towards A, kT = 0",
            "box": f"{w.WETTING_N}^3 closed, R = {w.WETTING_R:g}, rho {w.PAPER_RHO0}", "steps": steps,
            "averaged_over_last": tail, "seconds": round(el, 3), "MLUPS": round(nodes * steps / el / 1e6, 1),
            "rows": rows}


def langevin_stats(sim, reps, steps, skip):
    """Per-replica mean and variance of the particle velocity U_z over the
    last steps - skip recorded steps, grouped by lattice size, with the
    variance in units of kT / m_p (the Langevin prediction, Sec. 3)."""
    import math
    import numpy as np
    groups = {}
    for r, q in enumerate(reps):
        if q["radius"] <= 0 or q["series_cap"] < steps:
            continue
        u = sim.u_series(r)[-(steps - skip):, 2]
        mp = 4.0 / 3.0 * math.pi * q["radius"] ** 3 * q["rho_p"]
        key = f"{q['nx']}x{q['ny']}x{q['nz']},R={q['radius']:g},kT={q['kT']:g}"
        groups.setdefault(key, []).append((u.mean(), u.var() / (q["kT"] / mp) if q["kT"] > 0 else float("nan")))
    out = {}
    for key, v in groups.items():
        a = np.array(v)
        out[key] = {"replicas": len(v), "steps_used": steps - skip, "mean_Uz": float(a[:, 0].mean()),
                    "var_Uz_over_kT_mp": float(a[:, 1].mean()),
                    "sem": float(a[:, 1].std() / math.sqrt(len(v)))}
    return out


def fp16_error(torch, steps, every=50, skip=500):
    """FP16 relative-deviation storage against FP32 storage on the large
    channel (192 x 192 x 1024, R = 16), same Philox stream: time average of
    the z-averaged u_z(x, y) over the fluid (sampled every `every` steps) and
    the variance of the particle's U_z after `skip` steps.  FP32 is the
    reference here: FP64 storage of this lattice exceeds the library's 32-bit
    per-component offsets, and FP32 agrees with the FP64 oracle to ~1e-8."""
    import numpy as np
    from paper_1909_01092_amd import workloads as w
    from paper_1909_01092_amd.sim import Simulation
    res = {}
    for prec in ("fp32", "fp16"):
        p = dict(w.LARGE, series_cap=steps)
        sim = Simulation([p], precision=prec, device="cuda:0", stream=torch.cuda.Stream())
        prof, n = None, 0
        t0 = time.perf_counter()
        for k in range(steps // every):
            sim.step(every)
            pr = sim.observables(profile=True)["uz_profile"]
            prof = pr if prof is None else prof + pr
            n += 1
        sim.sync()
        el = time.perf_counter() - t0
        u = sim.u_series()[:, 2]
        res[prec] = dict(profile=prof / n, var=float(u[skip:].var()), mean=float(u[skip:].mean()),
                         U_end=float(u[-1]), sec=el, unstable=sim.particle_state(allow_unstable=True)["unstable"])
        sim.close()
        del sim
    a, b = res["fp16"], res["fp32"]
    return {
        "workload": "large 192x192x1024, R=16, kT=1e-4, g=1e-4, G=1.5", "steps": steps,
        "reference": "fp32 storage (same noise)",
        "uz_profile_rel_l2": float(np.linalg.norm(a["profile"] - b["profile"]) / np.linalg.norm(b["profile"])),
        "uz_profile_rel_max": float(np.abs(a["profile"] - b["profile"]).max() / np.abs(b["profile"]).max()),
        "var_Uz_fp16": a["var"], "var_Uz_fp32": b["var"], "var_Uz_rel": abs(a["var"] - b["var"]) / b["var"],
        "mean_Uz_rel": abs(a["mean"] - b["mean"]) / abs(b["mean"]),
        "U_end_rel": abs(a["U_end"] - b["U_end"]) / abs(b["U_end"]),
        "seconds": {"fp32": round(b["sec"], 1), "fp16": round(a["sec"], 1)},
        "unstable": bool(a["unstable"] or b["unstable"])}


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
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default 2000; adjoint: 1000)")
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="single")
    ap.add_argument("--zchunk", type=int, default=0, help="fixed main-kernel z-chunk (skips the autotuner)")
    ap.add_argument("--block", type=int, default=256, help="main-kernel block with --zchunk")
    ap.add_argument("--autotune", type=int, default=100,
                    help="steps per candidate of the launch-shape autotuner (0: library default shape)")
    ap.add_argument("--graph", type=int, default=0, help="steps per HIP graph (0: plain launches)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--stats", type=int, default=-1, metavar="SKIP",
                    help="add per-replica particle-velocity statistics over the timed steps after "
                         "the first SKIP (needs series_cap >= steps)")
    ap.add_argument("--fp16-error", type=int, default=0, metavar="STEPS",
                    help="instead of timing: run the large workload for STEPS steps in FP16 and in "
                         "FP32 storage on the same noise and report the FP16 error of the mean "
                         "velocity profile and of the particle velocity variance")
    ap.add_argument("--study", default="", choices=["", "friction", "friction-wet", "wetting", "interface"],
                    help="instead of timing: run a physics study and print its table (friction: "
                         "deterministic confinement friction c_m(d/L) at kT = 0; friction-wet: the "
                         "same in the paper's mixture for its three wettabilities; wetting: contact "
                         "angle against Delta rho of a sphere at a flat interface; interface: that "
                         "sphere under a body force, trapped or detached, for three wettabilities)")
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
    if args.fp16_error:
        print(json.dumps(fp16_error(torch, args.fp16_error)), flush=True)
        return
    if args.study == "friction":
        print(json.dumps(friction_study(torch, steps=args.steps or 12000)), flush=True)
        return
    if args.study == "friction-wet":
        print(json.dumps(friction_study(torch, steps=args.steps or 30000, tail=10000, wettability=True)),
              flush=True)
        return
    if args.study == "wetting":
        print(json.dumps(wetting_study(torch, steps=args.steps or 30000)), flush=True)
        return
    if args.study == "interface":
        print(json.dumps(interface_study(torch, steps=args.steps or 30000)), flush=True)
        return
    if args.workload == "adjoint":
        adjoint_bench(torch, args, args.steps or 1000)
        return
    args.steps = args.steps or 2000
    from paper_1909_01092_amd.sim import Simulation
    reps, prec, desc = workload(args.workload)
    stream = torch.cuda.Stream()
    sim = Simulation(reps, precision=prec, device="cuda:0", stream=stream)
    if args.zchunk:
        sim.set_launch(args.block, args.zchunk)
    elif args.autotune > 0:
        sim.autotune(steps_per_trial=args.autotune, preserve=False)  # before the warm-up
    block, cz = sim.get_launch()
    if args.graph:
        sim.set_graph(args.graph)
    sim.step(args.warmup)
    sim.sync()

    nodes = sum(q["nx"] * q["ny"] * q["nz"] for q in reps)
    timed = not args.graph
    # HIP events around one main launch in TIMING_EVERY: the kernel's
    # duration over the timed region without slowing the other steps
    sim.timing(TIMING_EVERY if timed else 0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(args.steps)
    sim.sync()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    kern_ms, nlaunch = sim.timing_read() if timed else (None, 0)
    sim.timing(False)

    stats = langevin_stats(sim, reps, args.steps, args.stats) if args.stats >= 0 else None
    state = [sim.particle_state(r, allow_unstable=True) for r in range(len(reps))]
    unstable = any(s["unstable"] for s in state)
    mlups = nodes * args.steps / el / 1e6
    step_bytes = sim.step_bytes()
    roof = None
    if kern_ms:
        achieved = step_bytes / (kern_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic_from_profile(args.workload, block, cz),
                "kernel": "k_main", "kernel_ms": round(kern_ms, 5), "launches": nlaunch,
                "bytes_per_launch": step_bytes}
    out = {
        "metric": "MLUPS (2-comp D3Q19)", "value": round(mlups, 2), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(el * 1e3 / args.steps, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "fp16": "f16-storage/f32"}[prec], "data": "synthetic",
        "config": {"workload": desc, "replicas": len(reps), "nodes": nodes, "precision": prec,
                   "block": block, "zchunk": cz, "autotuned": not args.zchunk and args.autotune > 0,
                   "graph_steps": args.graph,
                   "unstable": unstable},
        "roofline": roof,
    }
    if stats is not None:
        out["langevin"] = stats
    sim.close()
    del sim
    if args.workload == "ensemble":
        out["vs_plain"] = plain_comparison(torch, mlups)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(reps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
