"""ctypes binding of libdrops.so (include/drops.h): the drop-size diagnostic
of the jet study on the GPU -- connected components of the liquid
{phi > 1/2} and their equivalent diameters d_e.

Argument marshalling only; torch tensors provide device memory and the
stream.  Importing this module loads the library and raises if it has not
been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "_lib", "libdrops.so")

DR_OK, DR_EINVAL, DR_EDEVICE, DR_ECAPACITY, DR_EINTERNAL = 0, -1, -3, -6, -7


class DropsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"drop diagnostic error {code}: {msg}")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2505_12205_amd.build` (hipcc, gfx950)")
    L = C.CDLL(LIB_PATH)
    vp, i, u, f, sz = C.c_void_p, C.c_int, C.c_uint, C.c_float, C.c_size_t
    L.dr_last_error.restype = C.c_char_p
    L.dr_workspace_bytes.argtypes = [i, i, i]
    L.dr_workspace_bytes.restype = sz
    L.dr_label.argtypes = [vp, i, i, i, u, f, vp, vp, sz, vp]
    L.dr_components.argtypes = [vp, i, i, i, i, i, vp, vp, vp, vp, vp, C.POINTER(C.c_int), vp, sz, vp]
    return L


lib = _load()

EXPORTED = ("dr_last_error", "dr_workspace_bytes", "dr_label", "dr_components")


def _check(rc):
    if rc != DR_OK:
        raise DropsError(rc, lib.dr_last_error().decode())


def _s(stream):
    return (stream or torch.cuda.current_stream()).cuda_stream


def workspace(shape, device="cuda"):
    """Device workspace for fields of shape [nz, ny, nx]."""
    nz, ny, nx = shape
    n = lib.dr_workspace_bytes(nx, ny, nz)
    if n == 0:
        raise DropsError(DR_EINVAL, f"invalid extent {shape}")
    return torch.empty(n, dtype=torch.uint8, device=device)


def label(phi, periodic=(False, False, False), thr=0.5, ws=None, out=None, stream=None):
    """phi: float32 device tensor [nz, ny, nx] (or [ny, nx]).  Returns int32
    labels of the same shape: the smallest node index of each node's
    component of {phi > thr} (face connectivity, axes x, y, z wrapping where
    periodic), -1 outside the liquid."""
    assert phi.dtype == torch.float32 and phi.is_cuda and phi.is_contiguous(), "float32 contiguous device tensor"
    shape = (1,) + tuple(phi.shape) if phi.dim() == 2 else tuple(phi.shape)
    nz, ny, nx = shape
    ws = workspace(shape, phi.device) if ws is None else ws
    out = torch.empty(phi.shape, dtype=torch.int32, device=phi.device) if out is None else out
    mask = sum(1 << d for d in range(3) if periodic[d])
    _check(lib.dr_label(phi.data_ptr(), nx, ny, nz, mask, float(thr), out.data_ptr(), ws.data_ptr(), ws.numel(),
                        _s(stream)))
    return out


def components(lab, axis=2, cap=4096, ws=None, stream=None):
    """Per component, in ascending order of label, as numpy arrays: root,
    size (node count), lo / hi (extent along axis: 0 x, 1 y, 2 z) and deq
    (equivalent sphere diameter in 3D, disc diameter for a single plane).
    The capacity grows to the component count if cap is too small."""
    assert lab.dtype == torch.int32 and lab.is_cuda and lab.is_contiguous()
    shape = (1,) + tuple(lab.shape) if lab.dim() == 2 else tuple(lab.shape)
    nz, ny, nx = shape
    ws = workspace(shape, lab.device) if ws is None else ws
    while True:
        bufs = [torch.empty(max(cap, 1), dtype=torch.int32, device=lab.device) for _ in range(4)]
        deq = torch.empty(max(cap, 1), dtype=torch.float32, device=lab.device)
        nc = C.c_int()
        rc = lib.dr_components(lab.data_ptr(), nx, ny, nz, axis, cap, *[b.data_ptr() for b in bufs],
                               deq.data_ptr(), C.byref(nc), ws.data_ptr(), ws.numel(), _s(stream))
        if rc == DR_ECAPACITY:
            cap = nc.value
            continue
        _check(rc)
        n = nc.value
        out = {k: b[:n].cpu().numpy() for k, b in zip(("root", "size", "lo", "hi"), bufs)}
        out["deq"] = deq[:n].cpu().numpy()
        return out


def periodic_axes(cfg):
    bc = cfg.get("bc", ("periodic",) * 6)
    return tuple(bc[2 * d] == "periodic" for d in range(3))


def drop_sizes(phi, cfg, thr=0.5):
    """Drop statistics of a jet's phase field (device tensor [nz, ny, nx]):
    components of the liquid along the jet axis (z in 3D, y in 2D); the one
    that touches the inlet plane is the intact jet, those that touch the
    outlet plane are leaving the domain; the rest are drops.  Returns the
    drops' equivalent diameters d_e, d_e / D_j with D_j = 2 R_inlet, and the
    extent of the intact jet (nodes from the inlet)."""
    axis = 2 if cfg["q"] == 19 else 1
    n_axis = (cfg["nx"], cfg["ny"], cfg.get("nz", 1))[axis]
    c = components(label(phi, periodic_axes(cfg), thr), axis=axis)
    attached = c["lo"] == 0
    leaving = c["hi"] == n_axis - 1
    drops = ~attached & ~leaving
    dj = 2.0 * float(cfg["inlet_radius"])
    de = c["deq"][drops].astype(np.float64)
    return {"d_e": de, "d_e_over_Dj": de / dj, "count": int(drops.sum()),
            "mean_d_e_over_Dj": float(de.mean() / dj) if de.size else float("nan"),
            "intact_extent": int(c["hi"][attached].max() + 1) if attached.any() else 0,
            "components": int(len(c["root"]))}
