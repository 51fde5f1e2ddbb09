"""Run parameters and named workloads (plain data: no arithmetic of the method).

A parameter set is a dict with the fields of lbm_params; missing fields take
DEFAULTS.  The named workloads are the synthetic channels used for parity
tests and benchmarks; they stand in for the paper's 60 x 60 x 900 closed
channel (Sec. 3) at the sizes of each form of the hot path.
"""

DEFAULTS = dict(nx=8, ny=8, nz=8, walls=0, rho0=(0.95, 0.05), init_amp=0.0, G=0.0,
                tau_shear=1.0, tau_bulk=1.0, tau_mom=1.0, tau_ghost=1.0, kT=0.0, seed=0,
                replica=0, g=(0.0, 0.0, 0.0), force_mode=0, radius=0.0, rho_p=2.0,
                wet_drho=0.0, X0=None, U0=(0.0, 0.0, 0.0), W0=(0.0, 0.0, 0.0),
                noise_diffusive=1, fixed_velocity=0, series_cap=4096, init_split=0, shared_fluid=0)

SPHERE_FIELDS = ("radius", "rho_p", "wet_drho", "X0", "U0", "W0")


def full(params: dict) -> dict:
    """Parameters with defaults filled in; X0 defaults to the box centre."""
    q = dict(DEFAULTS)
    q.update(params)
    if q["X0"] is None:
        q["X0"] = ((q["nx"] - 1) / 2.0, (q["ny"] - 1) / 2.0, (q["nz"] - 1) / 2.0)
    return q


def entries(replicas) -> list:
    """lbm_init entries of one replica dict or a list of them.  A replica may
    list further spheres in the same fluid under "spheres" (dicts of
    SPHERE_FIELDS; missing ones as DEFAULTS): each becomes an entry with
    shared_fluid = 1 after the replica's own."""
    if isinstance(replicas, dict):
        replicas = [replicas]
    out = []
    for q in replicas:
        base = full({k: v for k, v in q.items() if k != "spheres"})
        out.append(base)
        for e in q.get("spheres", ()):
            extra = {k: e.get(k, DEFAULTS[k]) for k in SPHERE_FIELDS if k != "X0"}
            extra["X0"] = e["X0"]
            out.append(dict(base, shared_fluid=1, **extra))
    return out


def channel(n: int, nz: int, **kw) -> dict:
    """Square n x n channel (walls in x and y, periodic z), sphere at the centre,
    mixture 0.95 / 0.05 with +-1e-3 initial density noise, G = 1.5, tau = 1."""
    p = dict(nx=n, ny=n, nz=nz, walls=3, rho0=(0.95, 0.05), init_amp=1e-3, G=1.5, rho_p=2.0)
    p.update(kw)
    return full(p)


# FP64 parity case: 24 x 24 x 48, kT = 1e-5, R = 4, g = 1e-5 along z, 200 steps
PARITY_SMALL = channel(24, 48, kT=1e-5, radius=4.0, g=(0.0, 0.0, 1e-5), seed=0)
PARITY_SMALL_STEPS = 200

# single run, FP32 deviations: 64 x 64 x 256, R = 8, kT = 1e-5, g = 1e-4 (timed point)
SINGLE_RUN = channel(64, 256, kT=1e-5, radius=8.0, g=(0.0, 0.0, 1e-4), seed=1, series_cap=16384)
SINGLE_RUN_STEPS = 10000

# the single run's parameter grid: kT x g x Delta rho, one replica each
GRID_KT = (1e-6, 1e-5, 1e-4)
GRID_G = (1e-5, 3e-5, 1e-4)
GRID_DRHO = (-0.5, 0.0, 0.5)


def single_grid(steps_cap: int = 4096) -> list:
    return [dict(SINGLE_RUN, kT=kT, g=(0.0, 0.0, g), wet_drho=d, replica=k, series_cap=steps_cap,
                 grid=(kT, g, d))
            for k, (kT, g, d) in enumerate((kT, g, d) for kT in GRID_KT for g in GRID_G for d in GRID_DRHO)]


def ensemble(steps_cap: int = 8192) -> list:
    """128 replicas of 32x32x128 (R = 4), 32 of 24x24x96 (R = 3), 32 of 48x48x192
    (R = 6); kT = 1e-5, g = 5e-5; independent Philox keys per replica."""
    reps = []
    for k in range(128):
        reps.append(channel(32, 128, kT=1e-5, radius=4.0, g=(0, 0, 5e-5), seed=7, replica=k,
                            series_cap=steps_cap))
    for k in range(32):
        reps.append(channel(24, 96, kT=1e-5, radius=3.0, g=(0, 0, 5e-5), seed=7, replica=128 + k,
                            series_cap=steps_cap))
    for k in range(32):
        reps.append(channel(48, 192, kT=1e-5, radius=6.0, g=(0, 0, 5e-5), seed=7, replica=160 + k,
                            series_cap=steps_cap))
    return reps


# adjoint form: 48 x 48 x 192, R = 6, kT = 1e-5, g = 5e-5
ADJOINT = channel(48, 192, kT=1e-5, radius=6.0, g=(0.0, 0.0, 5e-5), seed=3)

# large single run, FP16 relative deviations: 192 x 192 x 1024, R = 16, kT = 1e-4, g = 1e-4
LARGE = channel(192, 192, kT=1e-4, radius=16.0, g=(0.0, 0.0, 1e-4), seed=5)
LARGE["nz"] = 1024
LARGE = full(dict(LARGE, X0=None))

# deterministic confinement friction (kT = 0): one replica per sphere radius
# in a 32 x 32 x 128 channel, uniform initial densities, g small enough for
# creeping flow (Re = U d / nu below 2e-3)
FRICTION_L, FRICTION_LZ = 32, 128
FRICTION_RADII = (2.5, 3.5, 5.0, 6.5, 8.0, 10.0)
FRICTION_G = 1e-6


def friction(steps_cap: int = 16384) -> list:
    return [channel(FRICTION_L, FRICTION_LZ, kT=0.0, init_amp=0.0, radius=R, g=(0.0, 0.0, FRICTION_G),
                    seed=0, replica=k, series_cap=steps_cap)
            for k, R in enumerate(FRICTION_RADII)]

# the paper's own setup (Sec. 3): closed 60 x 60 x 900 box (walls on every
# axis, neutral), rho_A = 2.21, rho_B = 0.09, G = 1.5 (G rho_tot = 3.45, the
# A-rich side of the miscibility gap, far from its spinodal), rho_p = 2 rho_tot;
# sphere of d / L = 0.27 low in the box, settling along +z
PAPER_RHO0 = (2.21, 0.09)


def paper_box(n: int = 60, nz: int = 900, radius: float = 8.0, kT: float = 1e-4, g: float = 5e-6,
              steps_cap: int = 4096) -> dict:
    rho_tot = PAPER_RHO0[0] + PAPER_RHO0[1]
    return full(dict(nx=n, ny=n, nz=nz, walls=7, rho0=PAPER_RHO0, init_amp=1e-3, G=1.5,
                     rho_p=2.0 * rho_tot, kT=kT, radius=radius, g=(0.0, 0.0, g), seed=9,
                     X0=((n - 1) / 2.0, (n - 1) / 2.0, min(nz / 4.0, 3.0 * radius + 4.0)),
                     series_cap=steps_cap))


# contact angle of the wetting layer: the sphere centred on a flat interface
# between the two demixed phases of PAPER_RHO0 (A below the plane
# z = n/2 - 1/2, B above) in a closed n^3 box with neutral walls, no noise, no
# driving, one replica per wetting offset Delta rho
WETTING_N = 48
WETTING_R = 8.0
WETTING_DRHO = (-0.2, -0.15, -0.1, -0.05, 0.0, 0.05, 0.1, 0.15, 0.2)


def wetting(drhos=WETTING_DRHO, n: int = WETTING_N, radius: float = WETTING_R,
            steps_cap: int = 16384) -> list:
    rho_tot = PAPER_RHO0[0] + PAPER_RHO0[1]
    return [full(dict(nx=n, ny=n, nz=n, walls=7, rho0=PAPER_RHO0, init_amp=0.0, G=1.5,
                      init_split=n // 2, rho_p=2.0 * rho_tot, kT=0.0, radius=radius, wet_drho=d,
                      seed=0, replica=k, series_cap=steps_cap))
            for k, d in enumerate(drhos)]


# the paper's three particle wettabilities (Sec. 3: theta_A = 120.5, 90 and 55
# degrees) as wetting offsets for an R = 8 sphere, read off the contact-angle
# sweep above (python -m paper_1909_01092_amd.studies wetting)
PAPER_WETTING_DRHO = {"hydrophobic": -0.146, "neutral": 0.0, "hydrophilic": 0.167}
INTERFACE_FORCES = (0.0, 0.5, 1.0, 2.0, 3.0)


def interface_trap(forces=INTERFACE_FORCES, n: int = WETTING_N, radius: float = WETTING_R,
                   steps_cap: int = 16384) -> list:
    """The contact-angle box with a body force pushing the sphere towards the A
    phase (-z): F_ext = V (rho_p - rho_tot) g (Sec. 3 eq. fp) equal to each of
    `forces`, for each of the paper's three wettabilities."""
    import math
    rho_tot = PAPER_RHO0[0] + PAPER_RHO0[1]
    V = 4.0 / 3.0 * math.pi * radius ** 3
    reps = []
    for name, d in PAPER_WETTING_DRHO.items():
        for F in forces:
            q = wetting(drhos=(d,), n=n, radius=radius, steps_cap=steps_cap)[0]
            g = F / (V * (q["rho_p"] - rho_tot))
            reps.append(dict(q, g=(0.0, 0.0, -g), replica=len(reps), wettability=name, force=F))
    return reps



# the same channels in the paper's mixture with its three wettabilities: radii
# from d = 10 up (the paper resolves d >= 8); smaller non-neutral spheres
# carry a minority-phase film whose flow outweighs this driving.  g is raised
# so that the settling velocity stands above that flow (Re <= 0.06).
FRICTION_WET_RADII = (5.0, 6.5, 8.0, 10.0)
FRICTION_WET_G = 2e-5


def friction_wettability(steps_cap: int = 32768, g: float = FRICTION_WET_G,
                         radii=FRICTION_WET_RADII) -> list:
    """The friction channels in the paper's mixture (rho 2.21 / 0.09, G = 1.5,
    rho_p = 2 rho_tot) with each of its three wettabilities: one replica per
    (wettability, radius)."""
    rho_tot = PAPER_RHO0[0] + PAPER_RHO0[1]
    reps = []
    for name, d in PAPER_WETTING_DRHO.items():
        for R in radii:
            reps.append(channel(FRICTION_L, FRICTION_LZ, kT=0.0, init_amp=0.0, radius=R,
                                g=(0.0, 0.0, g), rho0=PAPER_RHO0, rho_p=2.0 * rho_tot,
                                wet_drho=d, seed=0, replica=len(reps), series_cap=steps_cap,
                                wettability=name))
    return reps
