"""Physics studies on the GPU path (the scope table's next rows), each a
function that runs the library through Simulation and returns a table.

  friction_study    confinement friction c_m(d/L) at kT = 0 (Sec. 3, the
                    friction figure), optionally for the paper's mixture and
                    its three wettabilities;
  wetting_study     contact angle of the wetting layer against Delta rho, from
                    a sphere at a flat interface (Young's condition);
  interface_study   a sphere at a flat interface pushed towards A by a body
                    force (the follow-up of Sec. 5), trapped or detached;
  langevin_stats    per-replica mean and variance of U_z against kT / m_p
                    (Sec. 4, eq. MEANVARIANCE);
  fp16_error        FP16 against FP32 storage on the full large channel over
                    a long run (same noise).

    python -m paper_1909_01092_amd.studies friction|friction-wet|wetting|interface|fp16|langevin [--steps N]
"""
import argparse
import json
import time

def friction_study(torch, steps=12000, tail=1000, wettability=False):
    """Deterministic confinement friction (kT = 0): terminal settling
    velocity of spheres of several d/L in the square channel, one replica per
    radius in one context, and the friction factor relative to Stokes,
    c_m = F_ext / (3 pi eta d U), F_ext = V (rho_p - rho_tot) g (Sec. 3 eq. fp),
    eta = rho_tot nu, nu = (tau - 1/2) / 3.  wettability: the paper's mixture
    (rho 2.21 / 0.09) with each of its three wettabilities instead of the
    0.95 / 0.05 mixture with a neutral sphere."""
    import math
    from . import workloads as w
    from .sim import Simulation
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
    from . import workloads as w
    from .sim import Simulation
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
    from . import workloads as w
    from .sim import Simulation
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
    variance in units of kT / m_p (the Langevin prediction, Sec. 4, eq.
    MEANVARIANCE)."""
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
    from . import workloads as w
    from .sim import Simulation
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("study", choices=["friction", "friction-wet", "wetting", "interface", "fp16",
                                      "langevin"])
    ap.add_argument("--steps", type=int, default=0)
    ap.add_argument("--skip", type=int, default=500, help="langevin: steps left out as transient")
    args = ap.parse_args()
    import torch
    if args.study == "friction":
        out = friction_study(torch, steps=args.steps or 12000)
    elif args.study == "friction-wet":
        out = friction_study(torch, steps=args.steps or 30000, tail=10000, wettability=True)
    elif args.study == "wetting":
        out = wetting_study(torch, steps=args.steps or 30000)
    elif args.study == "interface":
        out = interface_study(torch, steps=args.steps or 30000)
    elif args.study == "fp16":
        out = fp16_error(torch, args.steps or 2000)
    else:
        from . import workloads as w
        from .sim import Simulation
        steps = args.steps or 1500
        reps = w.ensemble(steps_cap=steps)
        sim = Simulation(reps, precision="fp32", device="cuda:0", stream=torch.cuda.Stream())
        sim.step(steps)
        sim.sync()
        out = {"study": "Langevin statistics of the 192-replica ensemble", "steps": steps,
               "skip": args.skip, "groups": langevin_stats(sim, reps, steps, args.skip)}
        sim.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
