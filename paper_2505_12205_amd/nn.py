"""ctypes binding of libsurr.so (include/surrogate.h): the learned
surrogate's gfx950 kernels.

Argument marshalling only; torch tensors provide device memory and the
stream.  Importing this module loads the library and raises if it has not
been built.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "_lib", "libsurr.so")

SG_OK, SG_EINVAL, SG_EDEVICE = 0, -1, -3


class SurrogateError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"surrogate kernel error {code}: {msg}")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2505_12205_amd.build` (hipcc, gfx950)")
    L = C.CDLL(LIB_PATH)
    vp, i, ll, f, sz = C.c_void_p, C.c_int, C.c_longlong, C.c_float, C.c_size_t
    L.sg_last_error.restype = C.c_char_p
    L.sg_conv3d_fwd.argtypes = [vp, i, i, i, i, i, vp, vp, i, i, i, i, vp, vp, vp, vp]
    L.sg_conv3d_bwd_data.argtypes = [vp, i, i, i, i, i, vp, i, i, i, vp, vp, vp, vp, vp]
    L.sg_conv3d_bwd_weight_workspace.argtypes = [i, i, i, i, i, i, i, i]
    L.sg_conv3d_bwd_weight_workspace.restype = sz
    L.sg_conv3d_bwd_weight.argtypes = [vp, i, i, i, i, i, vp, i, i, i, vp, sz, vp, vp, vp]
    L.sg_flip_weights.argtypes = [vp, i, i, vp, vp]
    L.sg_fold_up_weights.argtypes = [vp, i, i, vp, vp]
    L.sg_conv3d_bwd_data_up2.argtypes = [vp, i, i, i, i, i, vp, i, vp, vp, vp, vp, vp]
    L.sg_adam.argtypes = [vp, vp, vp, vp, ll, i, f, f, f, f, vp, vp]
    L.sg_normalize.argtypes = [vp, i, i, ll, vp, vp, vp, vp]
    L.sg_pack.argtypes = [vp, i, i, ll, i, vp, vp]
    L.sg_residual_loss.argtypes = [vp, vp, vp, vp, i, i, ll, i, f, vp, vp, vp, vp]
    L.sg_unpack.argtypes = [vp, vp, vp, i, i, ll, i, vp, vp, vp, vp]
    L.sg_coarsen.argtypes = [vp, vp, vp, i, i, i, i, i, vp, vp]
    L.sg_phi_budget.argtypes = [vp, i, i, i, i, i, vp, vp]
    L.sg_gather.argtypes = [vp, ll, ll, vp, i, vp, vp]
    return L


lib = _load()

EXPORTED = ("sg_last_error", "sg_conv3d_fwd", "sg_conv3d_bwd_data", "sg_conv3d_bwd_weight_workspace",
            "sg_conv3d_bwd_weight", "sg_flip_weights", "sg_fold_up_weights", "sg_conv3d_bwd_data_up2", "sg_adam", "sg_normalize", "sg_pack",
            "sg_residual_loss", "sg_unpack", "sg_coarsen", "sg_phi_budget", "sg_gather")


def _check(rc):
    if rc != SG_OK:
        raise SurrogateError(rc, lib.sg_last_error().decode())


def _p(t):
    return None if t is None else t.data_ptr()


def _s(stream):
    return (stream or torch.cuda.current_stream()).cuda_stream


def _bf(t):
    assert t.dtype == torch.bfloat16 and t.is_cuda and t.is_contiguous(), "bf16 contiguous device tensor"
    return t


def conv3d_fwd(x, w, b, co, stride=1, up=1, relu=True, skip=None, y=None, yr=None, stream=None):
    """x [n, d, h, w, ci] bf16, w [co, 27, ci] bf16, b [co] float -> y [n, od, oh, ow, co]."""
    n, d, h, wd, ci = _bf(x).shape
    od, oh, ow = [-(-(up * e) // stride) for e in (d, h, wd)]
    if y is None:
        y = torch.empty((n, od, oh, ow, co), dtype=torch.bfloat16, device=x.device)
    _check(lib.sg_conv3d_fwd(_p(x), n, d, h, wd, ci, _p(_bf(w)), _p(b), co, stride, up, 1 if relu else 0,
                             _p(skip), _p(y), _p(yr), _s(stream)))
    return y


def conv3d_bwd_data(dz, wf, n, d, h, w, ci, stride=1, up=1, add=None, mask=None, da=None, dzp=None, stream=None):
    """dz [n, od, oh, ow, co] bf16, wf [ci, 27, co] bf16 (flip_weights) -> dzp [n, d, h, w, ci]."""
    co = _bf(dz).shape[-1]
    if dzp is None:
        dzp = torch.empty((n, d, h, w, ci), dtype=torch.bfloat16, device=dz.device)
    _check(lib.sg_conv3d_bwd_data(_p(dz), n, d, h, w, ci, _p(_bf(wf)), co, stride, up, _p(add), _p(mask), _p(da),
                                  _p(dzp), _s(stream)))
    return dzp


def conv3d_bwd_data_up2(dz, wu, n, d, h, w, ci, add=None, mask=None, da=None, dzp=None, stream=None):
    """Data gradient of a x2 upsampling layer: dz [n, 2d, 2h, 2w, co] bf16, wu [ci, 64, co]
    bf16 (fold_up_weights) -> dzp [n, d, h, w, ci]."""
    co = _bf(dz).shape[-1]
    if dzp is None:
        dzp = torch.empty((n, d, h, w, ci), dtype=torch.bfloat16, device=dz.device)
    _check(lib.sg_conv3d_bwd_data_up2(_p(dz), n, d, h, w, ci, _p(_bf(wu)), co, _p(add), _p(mask), _p(da),
                                      _p(dzp), _s(stream)))
    return dzp


def fold_up_weights(w, co, ci, wu=None, stream=None):
    """wu[c][a][o] = sum of w[o][k][c] over the fold set of a (sg_fold_up_weights)."""
    if wu is None:
        wu = torch.empty((ci, 64, co), dtype=torch.bfloat16, device=w.device)
    _check(lib.sg_fold_up_weights(_p(_bf(w)), co, ci, _p(wu), _s(stream)))
    return wu


def bwd_weight_workspace(n, d, h, w, ci, co, stride=1, up=1):
    return int(lib.sg_conv3d_bwd_weight_workspace(n, d, h, w, ci, co, stride, up))


def conv3d_bwd_weight(x, dz, stride, up, ws, dw, db, stream=None):
    n, d, h, wd, ci = _bf(x).shape
    co = _bf(dz).shape[-1]
    _check(lib.sg_conv3d_bwd_weight(_p(x), n, d, h, wd, ci, _p(dz), co, stride, up, _p(ws),
                                    ws.numel() * ws.element_size(), _p(dw), _p(db), _s(stream)))


def flip_weights(w, co, ci, wf, stream=None):
    """wf[c][26 - k][o] = w[o][k][c] (the data gradient's weights)."""
    _check(lib.sg_flip_weights(_p(_bf(w)), co, ci, _p(wf), _s(stream)))


def adam(p, m, v, g, t, lr, beta1=0.9, beta2=0.999, eps=1e-8, pb=None, stream=None):
    _check(lib.sg_adam(_p(p), _p(m), _p(v), _p(g), p.numel(), int(t), lr, beta1, beta2, eps, _p(pb), _s(stream)))


def normalize(x, shift, scale, out=None, stream=None):
    """x [n, c, ...] float -> (x - shift[c]) * scale[c]."""
    n, c = x.shape[:2]
    vox = x[0, 0].numel()
    out = torch.empty_like(x) if out is None else out
    _check(lib.sg_normalize(_p(x), n, c, vox, _p(shift), _p(scale), _p(out), _s(stream)))
    return out


def pack(xn, cpad, out=None, stream=None):
    """[n, c, d, h, w] float -> [n, d, h, w, cpad] bf16."""
    n, c = xn.shape[:2]
    sp = tuple(xn.shape[2:])
    vox = xn[0, 0].numel()
    if out is None:
        out = torch.empty((n,) + sp + (cpad,), dtype=torch.bfloat16, device=xn.device)
    _check(lib.sg_pack(_p(xn), n, c, vox, cpad, _p(out), _s(stream)))
    return out


def residual_loss(xn, tn, r, dr, loss=None, ws=None, rs=None, mass_weight=0.0, stream=None):
    """pred = xn + rs * r; mean squared error against tn (+ the phase-field
    content term weighted by mass_weight) and its gradient dr.  ws: 2048
    doubles."""
    n, c = xn.shape[:2]
    vox = xn[0, 0].numel()
    cpad = r.shape[-1]
    _check(lib.sg_residual_loss(_p(xn), _p(tn), _p(r), _p(rs), n, c, vox, cpad, float(mass_weight), _p(dr),
                                _p(loss), _p(ws), _s(stream)))


def unpack(xn, r, shift, scale, out=None, rs=None, stream=None):
    n, c = xn.shape[:2]
    vox = xn[0, 0].numel()
    out = torch.empty_like(xn) if out is None else out
    _check(lib.sg_unpack(_p(xn), _p(r), _p(rs), n, c, vox, r.shape[-1], _p(shift), _p(scale), _p(out),
                         _s(stream)))
    return out


def coarsen(phi, u, p, nx, ny, nz, z0c, dw, out=None, stream=None):
    if out is None:
        out = torch.empty((5, dw, ny // 2, nx // 2), dtype=torch.float32, device=phi.device)
    _check(lib.sg_coarsen(_p(phi), _p(u), _p(p), nx, ny, nz, z0c, dw, _p(out), _s(stream)))
    return out


def phi_budget(x, out=None, stream=None):
    """x [n, c, d, h, w] float -> [n, 3] double (sum phi, inlet-plane and
    last-plane sums of phi u_z)."""
    n, c, d, h, w = x.shape
    out = torch.empty((n, 3), dtype=torch.float64, device=x.device) if out is None else out
    _check(lib.sg_phi_budget(_p(x), n, c, d, h, w, _p(out), _s(stream)))
    return out


def gather(store, idx, out, stream=None):
    """store [rows, ...] float, idx [n] int64 device -> out [n, ...] float."""
    rows = store.shape[0]
    length = store[0].numel()
    assert store.dtype == torch.float32 and idx.dtype == torch.int64 and idx.is_cuda
    assert out.numel() == idx.numel() * length
    _check(lib.sg_gather(_p(store), rows, length, _p(idx), idx.numel(), _p(out), _s(stream)))
    return out
