"""FP64 CPU oracle of the conservative phase-field LBM step (arXiv 2505.12205).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It shares no code with
the HIP implementation in ``paper_2505_12205_amd``; the two meet only through
the seeded input generators of ``paper_2505_12205_amd.workloads``.

The arithmetic lives in ``ora.c`` (plain C99 + OpenMP, double precision); this
module compiles it with gcc and wraps it with ctypes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ora.c")
_SRC_DROPS = os.path.join(_HERE, "drops.c")
_LIB = os.path.join(_HERE, "libora.so")

PERIODIC, NOSLIP, FREESLIP, INLET, OUTLET = 0, 1, 2, 3, 4
_BC = {"periodic": PERIODIC, "noslip": NOSLIP, "freeslip": FREESLIP,
       "inlet": INLET, "outlet": OUTLET}
_BODY = {"rho": 0, "rho_minus_rhol": 1}
_OUTLET = {"local": 0, "max": 1, "average": 2}


def build(force: bool = True) -> str:
    """Compile ora.c and drops.c into libora.so with gcc (IEEE double, no fast-math)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=gnu99", "-fopenmp", "-fPIC", "-shared", "-Wall",
               "-Wno-unused-function", _SRC, _SRC_DROPS, "-o", _LIB + ".tmp", "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class Params(C.Structure):
    _fields_ = [
        ("q", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("rho_h", C.c_double), ("rho_l", C.c_double),
        ("tau_h", C.c_double), ("tau_l", C.c_double),
        ("sigma", C.c_double), ("xi", C.c_double), ("mobility", C.c_double),
        ("gravity", C.c_double * 3), ("body_force", C.c_int),
        ("bc", C.c_int * 6),
        ("inlet_center", C.c_double * 2), ("inlet_radius", C.c_double),
        ("inlet_u", C.c_double), ("outlet_mode", C.c_int), ("flags", C.c_int),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        fp = C.POINTER(C.c_float)
        lp = C.POINTER(C.c_long)
        L.ora_lattice.argtypes = [C.c_int, ip, dp, ip, dp, dp, ip]
        L.ora_create.restype = C.c_void_p
        L.ora_create.argtypes = [C.POINTER(Params)]
        L.ora_destroy.argtypes = [C.c_void_p]
        L.ora_init.argtypes = [C.c_void_p, dp, dp]
        L.ora_set_state.argtypes = [C.c_void_p, dp, dp, dp]
        L.ora_get_state.argtypes = [C.c_void_p, dp, dp, dp]
        L.ora_step.argtypes = [C.c_void_p, C.c_int]
        L.ora_fields.argtypes = [C.c_void_p, dp, dp, dp]
        L.ora_step_h_prescribed.argtypes = [C.c_void_p, dp, dp, C.c_int]
        L.ora_reduce.argtypes = [C.c_void_p, dp, dp]
        L.ora_step_nodes_f32.argtypes = [C.POINTER(Params), fp, fp, fp, C.c_long, lp, dp, dp, dp]
        L.ora_feq.argtypes = [C.c_int, C.c_double, dp, dp]
        L.ora_heq.argtypes = [C.c_int, C.c_double, dp, dp]
        L.ora_grad_lap.argtypes = [C.c_int, dp, dp, dp]
        L.ora_chem_potential.restype = C.c_double
        L.ora_chem_potential.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double]
        L.ora_viscous_force.argtypes = [C.c_int, C.c_int, dp, dp, C.c_double, dp, dp]
        L.ora_collide_g.argtypes = [C.c_int, C.c_int, dp, dp, dp, C.c_double, C.c_double, dp]
        L.ora_phase_forcing.argtypes = [C.c_int, C.c_double, dp, C.c_double, dp]
        L.ora_collide_h.argtypes = [C.c_int, dp, C.c_double, dp, dp, C.c_double, C.c_double, dp]
        L.ora_collide_node.argtypes = [C.POINTER(Params), dp, dp, dp, dp, dp, dp, dp]
        L.ora_label.argtypes = [fp, C.c_int, C.c_int, C.c_int, C.c_uint, C.c_float, ip]
        L.ora_components.argtypes = [ip, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, ip, ip, ip, ip, dp]
        _lib = L
    return _lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


def make_params(cfg: dict) -> Params:
    """Fill the oracle's parameter block from a plain dict of lattice-unit values."""
    p = Params()
    p.q = int(cfg["q"])
    p.nx, p.ny, p.nz = int(cfg["nx"]), int(cfg["ny"]), int(cfg.get("nz", 1))
    p.rho_h, p.rho_l = float(cfg["rho_h"]), float(cfg["rho_l"])
    p.tau_h, p.tau_l = float(cfg["tau_h"]), float(cfg["tau_l"])
    p.sigma, p.xi, p.mobility = float(cfg["sigma"]), float(cfg["xi"]), float(cfg["mobility"])
    g = cfg.get("gravity", (0.0, 0.0, 0.0))
    for d in range(3):
        p.gravity[d] = float(g[d])
    p.body_force = _BODY[cfg.get("body_force", "rho")]
    bc = cfg.get("bc", ("periodic",) * 6)
    for f in range(6):
        p.bc[f] = _BC[bc[f]]
    c = cfg.get("inlet_center", (0.0, 0.0))
    p.inlet_center[0], p.inlet_center[1] = float(c[0]), float(c[1])
    p.inlet_radius = float(cfg.get("inlet_radius", 0.0))
    p.inlet_u = float(cfg.get("inlet_u", 0.0))
    p.outlet_mode = _OUTLET[cfg.get("outlet_mode", "local")]
    p.flags = (1 if cfg.get("clamp_phi", False) else 0) | (2 if _op(cfg) == "bgk" else 0)
    return p


def _op(cfg):
    """Collision operator of the hydrodynamic set: "wmrt" (default) or "bgk"."""
    op = cfg.get("collision", "wmrt")
    if op not in ("wmrt", "bgk"):
        raise ValueError(f"collision must be 'wmrt' or 'bgk', not {op!r}")
    return op


def lattice(q: int):
    """(e[q,3], w[q], opp[q], M[q,q], Minv[q,q], srel[q]) as the oracle holds them."""
    e = np.zeros((q, 3), np.int32)
    w = np.zeros(q)
    opp = np.zeros(q, np.int32)
    M = np.zeros((q, q))
    Mi = np.zeros((q, q))
    s = np.zeros(q, np.int32)
    ip = C.POINTER(C.c_int)
    dp = C.POINTER(C.c_double)
    rc = lib().ora_lattice(q, e.ctypes.data_as(ip), w.ctypes.data_as(dp), opp.ctypes.data_as(ip),
                           M.ctypes.data_as(dp), Mi.ctypes.data_as(dp), s.ctypes.data_as(ip))
    if rc != 0:
        raise ValueError(f"unknown lattice q={q}")
    return e, w, opp, M, Mi, s


class Oracle:
    """Full-grid FP64 simulation.  Arrays are numpy, layout pop[a, z, y, x]."""

    def __init__(self, cfg: dict):
        self.cfg = dict(cfg)
        self.params = make_params(cfg)
        self.q = self.params.q
        self.shape = (self.params.nz, self.params.ny, self.params.nx)
        self.N = int(np.prod(self.shape))
        self._h = lib().ora_create(C.byref(self.params))
        if not self._h:
            raise ValueError("oracle rejected the parameters")

    def __del__(self):
        if getattr(self, "_h", None):
            lib().ora_destroy(self._h)
            self._h = None

    def init(self, phi0, u0=None):
        phi0, pp = _d(np.asarray(phi0).reshape(-1))
        assert phi0.size == self.N
        if u0 is None:
            up = None
        else:
            u0, up = _d(np.asarray(u0).reshape(-1))
            assert u0.size == 3 * self.N
        lib().ora_init(self._h, pp, up)
        return self

    def step(self, n: int = 1):
        lib().ora_step(self._h, int(n))
        return self

    def step_h_prescribed(self, u_field, scales):
        """Advance only the phase-field set, len(scales) steps, under the
        prescribed velocity scales[k] * u_field (u_field: [3, nz, ny, nx])."""
        u, up = _d(np.asarray(u_field).reshape(-1))
        assert u.size == 3 * self.N
        sc, sp = _d(np.asarray(scales, float).reshape(-1))
        if lib().ora_step_h_prescribed(self._h, up, sp, int(sc.size)) != 0:
            raise ValueError("prescribed-velocity transport needs periodic or wall faces")
        return self

    def state(self):
        q, N = self.q, self.N
        h = np.empty(q * N)
        g = np.empty(q * N)
        u = np.empty(3 * N)
        lib().ora_get_state(self._h, _d(h)[1], _d(g)[1], _d(u)[1])
        sh = (q,) + self.shape
        return h.reshape(sh), g.reshape(sh), u.reshape((3,) + self.shape)

    def set_state(self, h, g, u):
        h, hp = _d(np.asarray(h).reshape(-1))
        g, gp = _d(np.asarray(g).reshape(-1))
        u, up = _d(np.asarray(u).reshape(-1))
        lib().ora_set_state(self._h, hp, gp, up)
        return self

    def fields(self):
        N = self.N
        phi = np.empty(N)
        u = np.empty(3 * N)
        p = np.empty(N)
        lib().ora_fields(self._h, _d(phi)[1], _d(u)[1], _d(p)[1])
        return phi.reshape(self.shape), u.reshape((3,) + self.shape), p.reshape(self.shape)

    def reduce(self):
        m = C.c_double()
        k = C.c_double()
        lib().ora_reduce(self._h, C.byref(m), C.byref(k))
        return m.value, k.value


def step_nodes_f32(cfg: dict, h, g, u, nodes):
    """One oracle step evaluated only at `nodes` (flat indices) from an FP32 state.

    Returns (h_new[k, q], g_new[k, q], u_new[k, 3])."""
    p = make_params(cfg)
    q = p.q
    h = np.ascontiguousarray(h, dtype=np.float32).reshape(-1)
    g = np.ascontiguousarray(g, dtype=np.float32).reshape(-1)
    u = np.ascontiguousarray(u, dtype=np.float32).reshape(-1)
    nodes = np.ascontiguousarray(nodes, dtype=np.int64)
    k = nodes.size
    ho = np.empty(k * q)
    go = np.empty(k * q)
    uo = np.empty(k * 3)
    fp = C.POINTER(C.c_float)
    rc = lib().ora_step_nodes_f32(
        C.byref(p), h.ctypes.data_as(fp), g.ctypes.data_as(fp), u.ctypes.data_as(fp), k,
        nodes.ctypes.data_as(C.POINTER(C.c_long)), _d(ho)[1], _d(go)[1], _d(uo)[1])
    if rc != 0:
        raise ValueError("oracle rejected the parameters")
    return ho.reshape(k, q), go.reshape(k, q), uo.reshape(k, 3)


# ---- single-node building blocks (thin wrappers for the unit pins) ----

def feq(q, pstar, u):
    u, up = _d(np.asarray(u, float).reshape(3))
    out = np.empty(q)
    lib().ora_feq(q, pstar, up, _d(out)[1])
    return out


def heq(q, phi, u):
    u, up = _d(np.asarray(u, float).reshape(3))
    out = np.empty(q)
    lib().ora_heq(q, phi, up, _d(out)[1])
    return out


def grad_lap(q, phin):
    phin, pp = _d(phin)
    grad = np.empty(3)
    lap = C.c_double()
    lib().ora_grad_lap(q, pp, _d(grad)[1], C.byref(lap))
    return grad, lap.value


def chem_potential(phi, lap, sigma, xi):
    return lib().ora_chem_potential(phi, lap, sigma, xi)


_OPS = {"wmrt": 0, "bgk": 1}


def viscous_force(q, g, feq_, tau, gradrho, op="wmrt"):
    g, gp = _d(g)
    f, fp = _d(feq_)
    gr, grp = _d(np.asarray(gradrho, float).reshape(3))
    out = np.empty(3)
    lib().ora_viscous_force(q, _OPS[op], gp, fp, tau, grp, _d(out)[1])
    return out


def collide_g(q, g, feq_, force, rho, tau, op="wmrt"):
    g, gp = _d(g)
    f, fp = _d(feq_)
    F, Fp = _d(np.asarray(force, float).reshape(3))
    out = np.empty(q)
    lib().ora_collide_g(q, _OPS[op], gp, fp, Fp, rho, tau, _d(out)[1])
    return out


def phase_forcing(q, phi, gradphi, xi):
    gr, grp = _d(np.asarray(gradphi, float).reshape(3))
    out = np.empty(q)
    lib().ora_phase_forcing(q, phi, grp, xi, _d(out)[1])
    return out


def collide_h(q, h, phi, u, gradphi, xi, mobility):
    h, hp = _d(h)
    u, up = _d(np.asarray(u, float).reshape(3))
    gr, grp = _d(np.asarray(gradphi, float).reshape(3))
    out = np.empty(q)
    lib().ora_collide_h(q, hp, phi, up, grp, xi, mobility, _d(out)[1])
    return out


def collide_node(cfg, h, g, u_prev, phin):
    p = make_params(cfg)
    q = p.q
    h, hp = _d(h)
    g, gp = _d(g)
    u, up = _d(np.asarray(u_prev, float).reshape(3))
    pn, pnp = _d(phin)
    ho = np.empty(q)
    go = np.empty(q)
    uo = np.empty(3)
    lib().ora_collide_node(C.byref(p), hp, gp, up, pnp, _d(ho)[1], _d(go)[1], _d(uo)[1])
    return ho, go, uo


# ---------------------------------------------------------------------------
# drop-size diagnostic (drops.c)
# ---------------------------------------------------------------------------

def label(phi, periodic=(False, False, False), thr=0.5):
    """Connected components of {phi > thr} of a [nz, ny, nx] field (face
    connectivity, axes x, y, z wrapping where periodic): int32 labels, each
    the smallest node index of its component, -1 outside the liquid."""
    phi = np.ascontiguousarray(np.asarray(phi, dtype=np.float32))
    if phi.ndim == 2:
        phi = phi[None]
    nz, ny, nx = phi.shape
    out = np.empty(phi.shape, np.int32)
    mask = sum(1 << d for d in range(3) if periodic[d])
    rc = lib().ora_label(phi.ctypes.data_as(C.POINTER(C.c_float)), nx, ny, nz, mask, float(thr),
                         out.ctypes.data_as(C.POINTER(C.c_int)))
    if rc != 0:
        raise RuntimeError(f"ora_label failed ({rc})")
    return out


def components(lab, axis=2):
    """Per component, in ascending order of label: dict of root, size (node
    count), lo / hi (extent along axis: 0 = x, 1 = y, 2 = z) and deq (the
    equivalent sphere diameter in 3D, disc diameter when nz = 1)."""
    lab = np.ascontiguousarray(np.asarray(lab, dtype=np.int32))
    nz, ny, nx = lab.shape
    cap = int((lab.reshape(-1) == np.arange(lab.size)).sum())
    ip = C.POINTER(C.c_int)
    arrs = {k: np.zeros(max(cap, 1), np.int32) for k in ("root", "size", "lo", "hi")}
    deq = np.zeros(max(cap, 1))
    nc = lib().ora_components(lab.ctypes.data_as(ip), nx, ny, nz, axis, cap,
                              *[arrs[k].ctypes.data_as(ip) for k in ("root", "size", "lo", "hi")],
                              deq.ctypes.data_as(C.POINTER(C.c_double)))
    if nc != cap:
        raise RuntimeError(f"ora_components: {nc} components, expected {cap}")
    out = {k: v[:nc] for k, v in arrs.items()}
    out["deq"] = deq[:nc]
    return out
