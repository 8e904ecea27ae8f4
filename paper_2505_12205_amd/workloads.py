"""Seeded synthetic workloads: lattice-unit parameters and initial fields.

This module is the only code shared by the HIP path and the FP64 oracle.  It
holds no step arithmetic: it produces plain parameter dictionaries and initial
phase-field / velocity arrays (layout [z, y, x], x fastest) from which each
side builds its own initial populations.

Parameter values follow the dimensionless groups of the paper's validation
and jet sections (density ratio, viscosity ratio, Reynolds, Weber, Froude,
Atwood, Peclet and capillary numbers) converted to lattice units with
nu = tau cs^2, cs^2 = 1/3.
"""
from __future__ import annotations

import numpy as np

CS2 = 1.0 / 3.0


def _tanh_profile(signed_dist, xi):
    """Equilibrium kernel of the phase field: 1/2 + 1/2 tanh(2 d / xi)."""
    return 0.5 + 0.5 * np.tanh(2.0 * signed_dist / xi)


def _grid(nx, ny, nz):
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x.astype(np.float64), y.astype(np.float64), z.astype(np.float64)


def perturb(phi0, u0, seed, phi_amp=0.0, u_amp=0.0):
    """Seeded noise added to initial fields (breaks exact symmetries in parity
    runs).  The phase-field noise is weighted by 4 phi (1 - phi), so it lives
    in the interfaces and leaves the bulk phases (and so rho >= rho_L) intact."""
    rng = np.random.default_rng(seed)
    if phi_amp:
        phi = phi0 + phi_amp * 4.0 * phi0 * (1.0 - phi0) * rng.standard_normal(phi0.shape)
    else:
        phi = phi0.copy()
    if u_amp:
        un = u_amp * rng.standard_normal((3,) + phi0.shape)
        u = un if u0 is None else u0 + un
    else:
        u = None if u0 is None else u0.copy()
    return phi, u


# --------------------------------------------------------------------------
# 2D stationary drop (D2Q9, all periodic)
# --------------------------------------------------------------------------

def drop2d(n=128, radius=25.0, xi=4.0, rho_h=1.0, rho_l=1e-3, visc_ratio=100.0,
           nu_h=0.1, sigma=1e-4, mobility=0.02, center=None, kinematic_ratio=True):
    """Heavy drop of radius R centred in an n x n periodic box.

    The viscosity ratio is kinematic, nu_H / nu_L = visc_ratio, by default:
    tau_H = nu_H / cs^2, tau_L = nu_L / cs^2.  (Read as a dynamic ratio
    mu_H / mu_L = 100 at rho_H / rho_L = 1000 it gives nu_L = 1.0; the explicit
    viscous force then moves information across the light side of the
    interface at about 4 nu_L / xi = 1 lattice unit per step and the scheme
    diverges.)  kinematic_ratio=False selects the dynamic reading."""
    if kinematic_ratio:
        nu_l = nu_h / visc_ratio
    else:
        nu_l = (rho_h * nu_h / visc_ratio) / rho_l
    cfg = dict(q=9, nx=n, ny=n, nz=1, rho_h=rho_h, rho_l=rho_l,
               tau_h=nu_h / CS2, tau_l=nu_l / CS2,
               sigma=sigma, xi=xi, mobility=mobility,
               gravity=(0.0, 0.0, 0.0), body_force="rho", bc=("periodic",) * 6,
               name=f"drop2d_{n}x{n}_R{radius:g}")
    cx, cy = center if center is not None else (n / 2.0, n / 2.0)
    x, y, _ = _grid(n, n, 1)
    r = np.sqrt((x - cx) ** 2 + (y - cy) ** 2)
    phi0 = _tanh_profile(radius - r, xi)
    return cfg, phi0, None


# --------------------------------------------------------------------------
# 3D Rayleigh-Taylor (D3Q19; periodic x/z, no-slip walls in y)
# --------------------------------------------------------------------------

def laplace3d(n=100, radius=20.0, sigma=0.005, rho_ratio=1000.0, tau=0.5, xi=4.0, mobility=0.02):
    """Static drop of the stationary-drop test: a heavy sphere of radius R
    centred in an n^3 periodic box at rest, tau_H = tau_L = tau, the given
    surface tension and density ratio (the paper's table: n = 100,
    R = 15 ... 35, sigma = 0.001, 0.005, 0.01, tau = 0.5, xi = 4,
    rho* = 1000).  The paper does not give the mobility; 0.02 as for the
    2D drop."""
    cfg = dict(q=19, nx=n, ny=n, nz=n, rho_h=1.0, rho_l=1.0 / rho_ratio, tau_h=tau, tau_l=tau,
               sigma=sigma, xi=xi, mobility=mobility, gravity=(0.0, 0.0, 0.0), body_force="rho",
               bc=("periodic",) * 6, name=f"laplace3d_{n}_R{radius:g}_s{sigma:g}")
    x, y, z = _grid(n, n, n)
    c = n / 2.0
    r = np.sqrt((x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2)
    return cfg, _tanh_profile(radius - r, xi), None


def rt_params(lref=256, atwood=0.5, reynolds=3000.0, u0=0.04, visc_ratio=1.0,
              peclet=1000.0, capillary=0.26, xi=5.0):
    """Lattice-unit parameters of the Rayleigh-Taylor case.

    U0 = sqrt(g L) (given), At = (rho_H - rho_L)/(rho_H + rho_L), Re = rho_H U0 L / mu_H,
    Pe = U0 L / M, Ca = mu_H U0 / sigma, with rho_H = 1."""
    rho_h = 1.0
    rho_l = rho_h * (1.0 - atwood) / (1.0 + atwood)
    mu_h = rho_h * u0 * lref / reynolds
    mu_l = mu_h / visc_ratio
    g = u0 * u0 / lref
    return dict(rho_h=rho_h, rho_l=rho_l, tau_h=(mu_h / rho_h) / CS2,
                tau_l=(mu_l / rho_l) / CS2, mobility=u0 * lref / peclet,
                sigma=mu_h * u0 / capillary, xi=xi, g=g)


def rt3d(nx=256, ny=1024, nz=256, lref=256, amp_frac=0.1, **kw):
    """Heavy fluid above a cosine-perturbed interface y0(x, z) in a
    nx x ny x nz box; parameters from rt_params(lref) so that a small copy
    (nx < lref) carries the same per-node arithmetic as the full case.
    y0 = ny/2 + amp_frac/2 * nx [cos(2 pi x/nx) + cos(2 pi z/nz)], peak amp_frac * nx."""
    p = rt_params(lref=lref, **kw)
    cfg = dict(q=19, nx=nx, ny=ny, nz=nz, rho_h=p["rho_h"], rho_l=p["rho_l"],
               tau_h=p["tau_h"], tau_l=p["tau_l"], sigma=p["sigma"], xi=p["xi"],
               mobility=p["mobility"], gravity=(0.0, -p["g"], 0.0),
               body_force="rho_minus_rhol",
               bc=("periodic", "periodic", "noslip", "noslip", "periodic", "periodic"),
               name=f"rt3d_{nx}x{ny}x{nz}")
    x, y, z = _grid(nx, ny, nz)
    y0 = ny / 2.0 + 0.5 * amp_frac * nx * (np.cos(2 * np.pi * x / nx) + np.cos(2 * np.pi * z / nz))
    phi0 = _tanh_profile(y - y0, p["xi"])
    return cfg, phi0, None


# the table of Rayleigh-Taylor cases: density ratio, viscosity ratio, Re,
# Pe, Ca (None: no surface tension), interface width, dimension
RT_CASES = {
    "a": dict(rho_ratio=3.0, visc_ratio=1.0, reynolds=3000.0, peclet=1000.0, capillary=0.26, xi=4.0, dim=2),
    "b": dict(rho_ratio=1000.0, visc_ratio=100.0, reynolds=3000.0, peclet=1000.0, capillary=0.44, xi=4.0, dim=2),
    "c": dict(rho_ratio=3.0, visc_ratio=3.0, reynolds=128.0, peclet=744.0, capillary=None, xi=5.0, dim=3),
    "d": dict(rho_ratio=1000.0, visc_ratio=100.0, reynolds=3000.0, peclet=200.0, capillary=8.7, xi=5.0, dim=3),
}


def rt_case(case, n=None, lref=256, amp_frac=0.1):
    """One of the four Rayleigh-Taylor cases of the paper's table: an
    L0 x 4 L0 (2D) or L0 x 4 L0 x L0 (3D) box, walls at the bottom and top,
    periodic sides, heavy fluid above a cosine-perturbed interface.  The
    parameters are those of L0 = lref; n (default lref) sets the lateral
    extent, so that a small copy keeps the per-node arithmetic.  The
    viscosity ratio is dynamic (mu_H / mu_L)."""
    c = RT_CASES[case]
    n = lref if n is None else n
    at = (c["rho_ratio"] - 1.0) / (c["rho_ratio"] + 1.0)
    p = rt_params(lref=lref, atwood=at, reynolds=c["reynolds"], visc_ratio=c["visc_ratio"], peclet=c["peclet"],
                  capillary=c["capillary"] or 1.0, xi=c["xi"])
    sigma = p["sigma"] if c["capillary"] else 0.0
    if c["dim"] == 2:
        nx, ny, nz = n, 4 * n, 1
        bc = ("periodic", "periodic", "noslip", "noslip", "periodic", "periodic")
        grav = (0.0, -p["g"], 0.0)
    else:
        nx, ny, nz = n, 4 * n, n
        bc = ("periodic", "periodic", "noslip", "noslip", "periodic", "periodic")
        grav = (0.0, -p["g"], 0.0)
    cfg = dict(q=9 if c["dim"] == 2 else 19, nx=nx, ny=ny, nz=nz, rho_h=p["rho_h"], rho_l=p["rho_l"],
               tau_h=p["tau_h"], tau_l=p["tau_l"], sigma=sigma, xi=p["xi"], mobility=p["mobility"],
               gravity=grav, body_force="rho_minus_rhol", bc=bc, name=f"rt_case_{case}_{nx}x{ny}x{nz}")
    x, y, z = _grid(nx, ny, nz)
    y0 = ny / 2.0 + amp_frac * nx * np.cos(2 * np.pi * x / nx)
    if c["dim"] == 3:
        y0 = ny / 2.0 + 0.5 * amp_frac * nx * (np.cos(2 * np.pi * x / nx) + np.cos(2 * np.pi * z / nz))
    return cfg, _tanh_profile(y - y0, p["xi"]), None


# --------------------------------------------------------------------------
# 3D liquid jet (D3Q19; free-slip sides, circular velocity inlet at z = 0,
# convective outlet at z = nz - 1, gravity along +z)
# --------------------------------------------------------------------------

def jet_params(diameter, u_jet=0.02, rho_ratio=800.0, visc_ratio=50.0, reynolds=300.0,
               weber=5.0, fr_over_re=0.01728, xi=5.0, mobility=0.01):
    """Re = rho_H u_j D / mu_H, We = rho_H u_j^2 D / sigma, Fr = u_j / sqrt(g D)
    with Fr/Re fixed (the constant ratio across the paper's jet table)."""
    rho_h = 1.0
    rho_l = rho_h / rho_ratio
    mu_h = rho_h * u_jet * diameter / reynolds
    mu_l = mu_h / visc_ratio
    froude = fr_over_re * reynolds
    g = u_jet * u_jet / (froude * froude * diameter)
    return dict(rho_h=rho_h, rho_l=rho_l, tau_h=(mu_h / rho_h) / CS2,
                tau_l=(mu_l / rho_l) / CS2, sigma=rho_h * u_jet * u_jet * diameter / weber,
                xi=xi, mobility=mobility, g=g, u_jet=u_jet)


def jet3d(nx=192, ny=192, nz=768, radius=12.0, stub=16.0, param_radius=None, **kw):
    """Jet domain with the nozzle centred in the inlet face; the liquid column
    initially fills z < stub inside the nozzle radius and moves at u_j.
    param_radius (default: radius) sets the nozzle radius the dimensionless
    groups refer to, so that a small copy keeps the per-node parameters."""
    p = jet_params(2.0 * (radius if param_radius is None else param_radius), **kw)
    cx, cy = nx / 2.0, ny / 2.0
    cfg = dict(q=19, nx=nx, ny=ny, nz=nz, rho_h=p["rho_h"], rho_l=p["rho_l"],
               tau_h=p["tau_h"], tau_l=p["tau_l"], sigma=p["sigma"], xi=p["xi"],
               mobility=p["mobility"], gravity=(0.0, 0.0, p["g"]),
               body_force="rho_minus_rhol",
               bc=("freeslip", "freeslip", "freeslip", "freeslip", "inlet", "outlet"),
               inlet_center=(cx, cy), inlet_radius=radius, inlet_u=p["u_jet"],
               outlet_mode="local", name=f"jet3d_{nx}x{ny}x{nz}_R{radius:g}")
    x, y, z = _grid(nx, ny, nz)
    r = np.sqrt((x - cx) ** 2 + (y - cy) ** 2)
    phi0 = _tanh_profile(radius - r, p["xi"]) * _tanh_profile(stub - z, p["xi"])
    u0 = np.zeros((3, nz, ny, nx))
    u0[2] = p["u_jet"] * phi0
    return cfg, phi0, u0


def sweep_lengths(seed=12205, n=64, lo=256, hi=768):
    """Domain lengths of the batched Weber sweep (uniform integers in [lo, hi])."""
    return np.random.default_rng(seed).integers(lo, hi + 1, n)


def sweep_weber(n=64, lo=0.5, hi=8.0):
    """Log-spaced Weber numbers We_k = lo * (hi/lo)^(k/(n-1))."""
    return lo * (hi / lo) ** (np.arange(n) / (n - 1))


SWEEP_MOBILITY = 0.05


def jet_sweep(n=64, nx=96, ny=96, radius=8.0, reynolds=200.0, lengths=None, webers=None,
              seed=12205, mobility=SWEEP_MOBILITY, **kw):
    """The batched sweep: a list of (cfg, phi0, u0) jet domains of uneven length.

    The sweep's configuration fixes Re, We, the density ratio and the nozzle
    radius but not the mobility.  With M = 0.01 (the precision-form jet's
    value) the low-We end diverges within a few hundred steps in the FP64
    reference and on the GPU alike (at R = 8 and Re = 200 the grid Ohnesorge
    number sqrt(D We)/Re is 0.014 at We = 0.5); M = 0.05 (Peclet number
    u_j D / M = 6.4) keeps every Weber number of the sweep finite for about
    10,300 steps, past the windows the surrogate and the regime calls use;
    later, the domains with We 0.7-1.1 diverge at their first pinch-off."""
    L = sweep_lengths(seed, n) if lengths is None else lengths
    We = sweep_weber(n) if webers is None else webers
    out = []
    for k in range(len(L)):
        out.append(jet3d(nx=nx, ny=ny, nz=int(L[k]), radius=radius, reynolds=reynolds,
                         weber=float(We[k]), mobility=mobility, **kw))
    return out


def breakup_field(nx=192, ny=192, nz=768, radius=12.0, intact=300.0, xi=4.0, seed=7, ndrops=None):
    """A phase field with the structure of a breaking jet, for the drop
    diagnostic: an intact liquid column of the nozzle radius from the inlet
    plane (z = 0) to z = intact, then a train of separated spherical drops
    (radii 0.4 R to 1.4 R, lateral offsets up to R/2) and small satellites
    (radius 2 to 3) towards the outlet, every interface with the tanh
    profile of width xi (a drop's profile is evaluated within 4 xi of its
    surface).  Returns (phi [nz, ny, nx] float32, drops), drops a list of
    (centre (x, y, z), radius) of every sphere placed."""
    rng = np.random.default_rng(seed)
    cx, cy = nx / 2.0, ny / 2.0
    yy, xx = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    r = np.sqrt((xx - cx) ** 2 + (yy - cy) ** 2)
    zz = np.arange(nz)
    phi = (_tanh_profile(intact - zz, xi)[:, None, None] * _tanh_profile(radius - r, xi)[None]).astype(np.float32)
    drops = []
    zc = intact + 2.0 * radius
    while zc < nz - 2.5 * radius and (ndrops is None or len(drops) < ndrops):
        big = len(drops) % 3 != 2
        rd = radius * rng.uniform(0.4, 1.4) if big else rng.uniform(2.0, 3.0)
        c = (cx + rng.uniform(-0.5, 0.5) * radius, cy + rng.uniform(-0.5, 0.5) * radius, zc + rd)
        m = rd + 4.0 * xi
        lo = [max(0, int(np.floor(c[d] - m))) for d in range(3)]
        hi = [min(n, int(np.ceil(c[d] + m)) + 1) for d, n in enumerate((nx, ny, nz))]
        z, y, x = np.meshgrid(np.arange(lo[2], hi[2]), np.arange(lo[1], hi[1]), np.arange(lo[0], hi[0]),
                              indexing="ij")
        d = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2)
        box = (slice(lo[2], hi[2]), slice(lo[1], hi[1]), slice(lo[0], hi[0]))
        phi[box] = np.maximum(phi[box], _tanh_profile(rd - d, xi))
        drops.append((c, rd))
        zc = c[2] + rd + xi + 3.0  # a gap of more than one interface width
    return phi, drops


def phi_in_profile(cfg):
    """Nozzle profile psi(r) on the inlet face (for diagnostics)."""
    x, y, _ = _grid(cfg["nx"], cfg["ny"], 1)
    cx, cy = cfg["inlet_center"]
    r = np.sqrt((x - cx) ** 2 + (y - cy) ** 2)
    return _tanh_profile(cfg["inlet_radius"] - r, cfg["xi"])[0]


def summary(cfg):
    """Human-readable one-line description of a workload."""
    keys = ("q", "nx", "ny", "nz", "rho_h", "rho_l", "tau_h", "tau_l", "sigma", "xi", "mobility")
    return ", ".join(f"{k}={cfg[k]:.6g}" if isinstance(cfg[k], float) else f"{k}={cfg[k]}"
                     for k in keys if k in cfg)


__all__ = ["drop2d", "rt3d", "rt_params", "jet3d", "jet_params", "jet_sweep", "SWEEP_MOBILITY", "sweep_lengths",
           "sweep_weber", "perturb", "phi_in_profile", "summary"]
