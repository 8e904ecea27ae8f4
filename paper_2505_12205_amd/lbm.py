"""ctypes binding of liblbm.so (include/lbm.h).

Argument marshalling only: every step of the method runs in the HIP kernels
of the library.  PyTorch provides device memory and the stream.  Importing
this module loads the library and raises if it has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "_lib", "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_EUNSTABLE, LBM_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
FIELD_PHI, FIELD_U, FIELD_P = 1, 2, 4
_BC = {"periodic": 0, "noslip": 1, "freeslip": 2, "inlet": 3, "outlet": 4}
_BODY = {"rho": 0, "rho_minus_rhol": 1}
_OUTLET = {"local": 0, "max": 1, "average": 2}
STORAGE = {"fp32": 0, "fp16": 1, "bf16": 2}
VF_CLAMP_PHI = 1
VF_BGK = 2
COLLISION = ("wmrt", "bgk")  # operator of the hydrodynamic set (cfg["collision"])


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"lbm error {code}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [
        ("lattice", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("rho_h", C.c_double), ("rho_l", C.c_double),
        ("tau_h", C.c_double), ("tau_l", C.c_double),
        ("sigma", C.c_double), ("xi", C.c_double), ("mobility", C.c_double),
        ("gravity", C.c_double * 3), ("body_force", C.c_int),
        ("bc", C.c_int * 6),
        ("inlet_center", C.c_double * 2), ("inlet_radius", C.c_double), ("inlet_u", C.c_double),
        ("outlet_mode", C.c_int), ("storage", C.c_int), ("variant_flags", C.c_uint),
    ]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2505_12205_amd.build` (hipcc, gfx950)")
    L = C.CDLL(LIB_PATH)
    vp, sz = C.c_void_p, C.c_size_t
    P = C.POINTER(Params)
    L.lbm_state_bytes.argtypes = [P, C.POINTER(sz)]
    L.lbm_init.argtypes = [P, vp, vp, vp, sz, vp, C.POINTER(vp)]
    L.lbm_step.argtypes = [vp, C.c_int]
    L.lbm_steps_done.argtypes = [vp]
    L.lbm_steps_done.restype = C.c_longlong
    L.lbm_fields.argtypes = [vp, C.c_uint, vp, vp, vp]
    L.lbm_reduce.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.lbm_export_state.argtypes = [vp, vp, vp, vp]
    L.lbm_import_state.argtypes = [vp, vp, vp, vp]
    L.lbm_checkpoint_bytes.argtypes = [vp, C.POINTER(sz)]
    L.lbm_save.argtypes = [vp, vp, sz]
    L.lbm_load.argtypes = [vp, vp, sz]
    L.lbm_set_tile.argtypes = [vp, C.c_int, C.c_int]
    L.lbm_get_tile.argtypes = [vp, C.POINTER(C.c_int), C.POINTER(C.c_int)]
    L.lbm_kernel_times.argtypes = [vp, C.c_int, C.POINTER(C.c_double)]
    L.lbm_set_store_hint.argtypes = [vp, C.c_int]
    L.lbm_set_zchunk.argtypes = [vp, C.c_int]
    L.lbm_get_zchunk.argtypes = [vp, C.POINTER(C.c_int)]
    L.lbm_get_blocks_per_cu.argtypes = [vp, C.POINTER(C.c_int)]
    L.lbm_batch_set_zchunk.argtypes = [vp, C.c_int]
    L.lbm_set_blocks_per_cu.argtypes = [vp, C.c_int]
    L.lbm_autotune.argtypes = [vp, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int),
                               C.POINTER(C.c_int), C.POINTER(C.c_double)]
    L.lbm_destroy.argtypes = [vp]
    L.lbm_batch_state_bytes.argtypes = [C.c_int, P, C.POINTER(sz)]
    L.lbm_batch_init.argtypes = [C.c_int, P, C.POINTER(vp), C.POINTER(vp), vp, sz, vp, C.POINTER(vp)]
    L.lbm_batch_step.argtypes = [vp, C.c_int]
    L.lbm_batch_steps_done.argtypes = [vp]
    L.lbm_batch_steps_done.restype = C.c_longlong
    L.lbm_batch_reduce.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.lbm_batch_reduce_noalloc.argtypes = [vp, vp]
    L.lbm_batch_fields.argtypes = [vp, C.c_int, C.c_uint, vp, vp, vp]
    L.lbm_batch_export_state.argtypes = [vp, C.c_int, vp, vp, vp]
    L.lbm_batch_intact_length.argtypes = [vp, C.c_float, C.POINTER(C.c_int)]
    L.lbm_batch_set_launch.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_int]
    L.lbm_batch_autotune.argtypes = [vp, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int),
                                     C.POINTER(C.c_int), C.POINTER(C.c_double)]
    L.lbm_batch_kernel_times.argtypes = [vp, C.c_int, C.POINTER(C.c_double)]
    L.lbm_batch_destroy.argtypes = [vp]
    L.lbm_last_error.restype = C.c_char_p
    L.lbm_version.restype = C.c_char_p
    return L


lib = _load()

EXPORTED = ("lbm_state_bytes", "lbm_init", "lbm_step", "lbm_steps_done", "lbm_fields", "lbm_reduce",
            "lbm_export_state", "lbm_import_state", "lbm_checkpoint_bytes", "lbm_save", "lbm_load",
            "lbm_set_tile", "lbm_get_tile", "lbm_set_store_hint", "lbm_set_zchunk", "lbm_get_zchunk", "lbm_batch_set_zchunk", "lbm_set_blocks_per_cu", "lbm_get_blocks_per_cu", "lbm_autotune",
            "lbm_kernel_times", "lbm_destroy", "lbm_last_error", "lbm_version",
            "lbm_batch_state_bytes", "lbm_batch_init", "lbm_batch_step", "lbm_batch_steps_done",
            "lbm_batch_reduce", "lbm_batch_reduce_noalloc", "lbm_batch_fields", "lbm_batch_export_state", "lbm_batch_intact_length",
            "lbm_batch_set_launch", "lbm_batch_autotune", "lbm_batch_kernel_times", "lbm_batch_destroy")


def _check(rc):
    if rc != LBM_OK:
        raise LbmError(rc, lib.lbm_last_error().decode())


def make_params(cfg: dict, storage: str = "fp32") -> Params:
    p = Params()
    p.lattice = int(cfg["q"])
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
    p.storage = STORAGE[storage]
    op = cfg.get("collision", "wmrt")
    if op not in COLLISION:
        raise ValueError(f"collision must be one of {COLLISION}, not {op!r}")
    p.variant_flags = (VF_CLAMP_PHI if cfg.get("clamp_phi", False) else 0) | (VF_BGK if op == "bgk" else 0)
    return p


def state_bytes(cfg: dict, storage: str = "fp32") -> int:
    p = make_params(cfg, storage)
    n = C.c_size_t()
    _check(lib.lbm_state_bytes(C.byref(p), C.byref(n)))
    return n.value


class Sim:
    """One simulation on the current CUDA (HIP) device and stream.

    phi0 / u0 are array-likes of shape [nz, ny, nx] / [3, nz, ny, nx]."""

    def __init__(self, cfg: dict, phi0, u0=None, storage: str = "fp32", device="cuda", stream=None):
        self.cfg = dict(cfg)
        self.storage = storage
        self.params = make_params(cfg, storage)
        self.q = self.params.lattice
        self.shape = (self.params.nz, self.params.ny, self.params.nx)
        self.N = self.params.nx * self.params.ny * self.params.nz
        self.device = torch.device(device)
        nbytes = state_bytes(cfg, storage)
        self.state = torch.empty(nbytes // 4 + 64, dtype=torch.float32, device=self.device)
        off = (-self.state.data_ptr()) % 256
        assert off % 4 == 0
        self._base = self.state.data_ptr() + off
        self._nbytes = nbytes
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        phi0 = torch.as_tensor(phi0, dtype=torch.float32).reshape(-1).to(self.device).contiguous()
        assert phi0.numel() == self.N
        if u0 is not None:
            u0 = torch.as_tensor(u0, dtype=torch.float32).reshape(-1).to(self.device).contiguous()
            assert u0.numel() == 3 * self.N
        h = C.c_void_p()
        _check(lib.lbm_init(C.byref(self.params), phi0.data_ptr(),
                            u0.data_ptr() if u0 is not None else None, self._base, nbytes,
                            self.stream.cuda_stream, C.byref(h)))
        self._h = h
        self._keep = (phi0, u0)  # alive until the init kernel has run
        self.synchronize()
        self._keep = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and lib is not None:
            try:
                self.synchronize()
            except Exception:
                pass
            lib.lbm_destroy(h)
            self._h = None

    def synchronize(self):
        self.stream.synchronize()

    def step(self, n: int = 1):
        _check(lib.lbm_step(self._h, int(n)))
        return self

    @property
    def steps_done(self) -> int:
        return int(lib.lbm_steps_done(self._h))

    def fields(self):
        """(phi[nz,ny,nx], u[3,nz,ny,nx], p[nz,ny,nx]) float32 device tensors."""
        phi = torch.empty(self.shape, dtype=torch.float32, device=self.device)
        u = torch.empty((3,) + self.shape, dtype=torch.float32, device=self.device)
        p = torch.empty(self.shape, dtype=torch.float32, device=self.device)
        _check(lib.lbm_fields(self._h, FIELD_PHI | FIELD_U | FIELD_P, phi.data_ptr(), u.data_ptr(),
                              p.data_ptr()))
        self.synchronize()
        return phi, u, p

    def reduce(self):
        m, k = C.c_double(), C.c_double()
        _check(lib.lbm_reduce(self._h, C.byref(m), C.byref(k)))
        return m.value, k.value

    def export_state(self):
        """Canonical FP32 (h[q,nz,ny,nx], g[q,...], u[3,...]) device tensors."""
        h = torch.empty((self.q,) + self.shape, dtype=torch.float32, device=self.device)
        g = torch.empty((self.q,) + self.shape, dtype=torch.float32, device=self.device)
        u = torch.empty((3,) + self.shape, dtype=torch.float32, device=self.device)
        _check(lib.lbm_export_state(self._h, h.data_ptr(), g.data_ptr(), u.data_ptr()))
        self.synchronize()
        return h, g, u

    def import_state(self, h, g, u):
        h = torch.as_tensor(h, dtype=torch.float32).to(self.device).contiguous()
        g = torch.as_tensor(g, dtype=torch.float32).to(self.device).contiguous()
        u = torch.as_tensor(u, dtype=torch.float32).to(self.device).contiguous()
        assert h.numel() == self.q * self.N and g.numel() == self.q * self.N and u.numel() == 3 * self.N
        _check(lib.lbm_import_state(self._h, h.data_ptr(), g.data_ptr(), u.data_ptr()))
        self.synchronize()
        return self

    def save(self) -> bytes:
        n = C.c_size_t()
        _check(lib.lbm_checkpoint_bytes(self._h, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        _check(lib.lbm_save(self._h, C.cast(buf, C.c_void_p), n.value))
        return buf.raw

    def load(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        _check(lib.lbm_load(self._h, C.cast(buf, C.c_void_p), len(blob)))
        return self

    def set_tile(self, bx: int, by: int):
        _check(lib.lbm_set_tile(self._h, int(bx), int(by)))
        return self

    @property
    def tile(self):
        bx, by = C.c_int(), C.c_int()
        _check(lib.lbm_get_tile(self._h, C.byref(bx), C.byref(by)))
        return bx.value, by.value

    def set_store_hint(self, nontemporal: bool):
        _check(lib.lbm_set_store_hint(self._h, 1 if nontemporal else 0))
        return self

    def set_zchunk(self, planes: int):
        """Planes per z-marching task of the D3Q19 interior kernel (0: tiled kernel)."""
        _check(lib.lbm_set_zchunk(self._h, int(planes)))
        return self

    @property
    def zchunk(self) -> int:
        v = C.c_int()
        _check(lib.lbm_get_zchunk(self._h, C.byref(v)))
        return v.value

    @property
    def blocks_per_cu(self) -> int:
        """Blocks per CU of the persistent launches (0: one block per tile)."""
        v = C.c_int()
        _check(lib.lbm_get_blocks_per_cu(self._h, C.byref(v)))
        return v.value

    def set_blocks_per_cu(self, n: int):
        _check(lib.lbm_set_blocks_per_cu(self._h, int(n)))
        return self

    def autotune(self, trial_steps: int = 10):
        """Pick the fastest tile shape and store hint (cached per shape); returns
        (bx, by, nontemporal, ms_per_step).  Advances the state by the trials."""
        bx, by, nt, ms = C.c_int(), C.c_int(), C.c_int(), C.c_double()
        _check(lib.lbm_autotune(self._h, int(trial_steps), C.byref(bx), C.byref(by), C.byref(nt),
                                C.byref(ms)))
        return bx.value, by.value, bool(nt.value), ms.value

    def kernel_times(self, n: int):
        """Mean ms of (phase-field pass, fused step kernel, boundary planes) over n eager steps."""
        out = (C.c_double * 3)()
        _check(lib.lbm_kernel_times(self._h, int(n), out))
        return tuple(out)


class Batch:
    """Many independent domains (same lattice and storage) advanced together.

    domains: list of (cfg, phi0, u0) as produced by workloads."""

    def __init__(self, domains, storage: str = "fp32", device="cuda", stream=None):
        self.storage = storage
        self.device = torch.device(device)
        self.cfgs = [dict(d[0]) for d in domains]
        self.ndom = len(domains)
        arr = (Params * self.ndom)()
        for i, d in enumerate(domains):
            arr[i] = make_params(d[0], storage)
        self.params = arr
        self.shapes = [(p.nz, p.ny, p.nx) for p in arr]
        self.q = arr[0].lattice
        n = C.c_size_t()
        _check(lib.lbm_batch_state_bytes(self.ndom, arr, C.byref(n)))
        self.state = torch.empty(n.value // 4 + 64, dtype=torch.float32, device=self.device)
        off = (-self.state.data_ptr()) % 256
        self._base = self.state.data_ptr() + off
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        keep = []
        phis = (C.c_void_p * self.ndom)()
        us = (C.c_void_p * self.ndom)()
        for i, (cfg, phi0, u0) in enumerate(domains):
            t = torch.as_tensor(phi0, dtype=torch.float32).reshape(-1).to(self.device).contiguous()
            keep.append(t)
            phis[i] = t.data_ptr()
            if u0 is not None:
                tu = torch.as_tensor(u0, dtype=torch.float32).reshape(-1).to(self.device).contiguous()
                keep.append(tu)
                us[i] = tu.data_ptr()
            else:
                us[i] = None
        h = C.c_void_p()
        _check(lib.lbm_batch_init(self.ndom, arr, phis, us, self._base, n.value, self.stream.cuda_stream,
                                  C.byref(h)))
        self._h = h
        self.stream.synchronize()
        del keep

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and lib is not None:
            try:
                self.stream.synchronize()
            except Exception:
                pass
            lib.lbm_batch_destroy(h)
            self._h = None

    @property
    def nodes(self) -> int:
        return sum(int(s[0]) * int(s[1]) * int(s[2]) for s in self.shapes)

    def step(self, n: int = 1):
        _check(lib.lbm_batch_step(self._h, int(n)))
        return self

    @property
    def steps_done(self) -> int:
        return int(lib.lbm_batch_steps_done(self._h))

    def reduce(self, strict: bool = True):
        """(mass[ndom], kinetic[ndom]); strict=False returns non-finite
        values of diverged domains instead of raising."""
        m = (C.c_double * self.ndom)()
        k = (C.c_double * self.ndom)()
        rc = lib.lbm_batch_reduce(self._h, m, k)
        if rc != LBM_EUNSTABLE or strict:
            _check(rc)
        return list(m), list(k)

    def reduce_noalloc(self, out):
        """Allocation-free reduction into a caller device tensor out (float64,
        2 * ndom entries): out[2d] = sum phi, out[2d + 1] = kinetic energy.
        Asynchronous on the batch's stream."""
        if out.dtype != torch.float64 or not out.is_cuda or not out.is_contiguous() or out.numel() < 2 * self.ndom:
            raise ValueError("out must be a contiguous float64 device tensor of 2 * ndom entries")
        _check(lib.lbm_batch_reduce_noalloc(self._h, out.data_ptr()))
        return out

    def fields(self, dom: int):
        sh = self.shapes[dom]
        phi = torch.empty(sh, dtype=torch.float32, device=self.device)
        u = torch.empty((3,) + sh, dtype=torch.float32, device=self.device)
        p = torch.empty(sh, dtype=torch.float32, device=self.device)
        _check(lib.lbm_batch_fields(self._h, dom, FIELD_PHI | FIELD_U | FIELD_P, phi.data_ptr(), u.data_ptr(),
                                    p.data_ptr()))
        self.stream.synchronize()
        return phi, u, p

    def export_state(self, dom: int):
        sh = self.shapes[dom]
        h = torch.empty((self.q,) + sh, dtype=torch.float32, device=self.device)
        g = torch.empty((self.q,) + sh, dtype=torch.float32, device=self.device)
        u = torch.empty((3,) + sh, dtype=torch.float32, device=self.device)
        _check(lib.lbm_batch_export_state(self._h, dom, h.data_ptr(), g.data_ptr(), u.data_ptr()))
        self.stream.synchronize()
        return h, g, u

    def intact_length(self, threshold: float = 0.5):
        out = (C.c_int * self.ndom)()
        _check(lib.lbm_batch_intact_length(self._h, float(threshold), out))
        return list(out)

    def set_launch(self, bx: int, by: int, blocks_per_cu: int = 4, nontemporal: bool = False):
        _check(lib.lbm_batch_set_launch(self._h, bx, by, blocks_per_cu, 1 if nontemporal else 0))
        return self

    def set_zchunk(self, planes: int):
        _check(lib.lbm_batch_set_zchunk(self._h, int(planes)))
        return self

    def autotune(self, trial_steps: int = 4):
        bx, by, bpc, nt, ms = C.c_int(), C.c_int(), C.c_int(), C.c_int(), C.c_double()
        _check(lib.lbm_batch_autotune(self._h, int(trial_steps), C.byref(bx), C.byref(by), C.byref(bpc),
                                      C.byref(nt), C.byref(ms)))
        return bx.value, by.value, bpc.value, bool(nt.value), ms.value

    def kernel_times(self, n: int):
        out = (C.c_double * 3)()
        _check(lib.lbm_batch_kernel_times(self._h, int(n), out))
        return tuple(out)


def version() -> str:
    return lib.lbm_version().decode()
