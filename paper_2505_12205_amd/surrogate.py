"""Learned surrogate of the jet solver: a 3D convolutional encoder-decoder
that advances coarse (phi, u_x, u_y, u_z, p) fields by a fixed number of
solver steps, trained on snapshots the batched solver produces.

Every arithmetic step runs in the HIP kernels of libsurr.so (binding in
``nn``); this module allocates the tensors and sequences the calls.

Network (the layer list below): 3 x 3 x 3 convolutions with ReLU,
an encoder that halves the grid twice (stride 2), a bottleneck, a decoder
that doubles it twice (nearest-neighbour upsampling fused into the
convolution) with additive skip connections from the encoder, and a linear
output layer whose result, times a fixed increment scale, is added to the
input (the network predicts the increment).  Weights are bf16 with float master copies; accumulation is
FP32; Adam updates the master copies.  Training minimises the mean squared
error of the normalised fields plus a weighted phase-field content term.

The fields are normalised with fixed physical scales: phi as is, velocity by
the jet velocity, pressure by rho_H u_j^2.
"""
from __future__ import annotations

import numpy as np
import torch

from . import nn

FIELDS = ("phi", "u_x", "u_y", "u_z", "p")
CIN = 5
# weight of the phase-field content term of the loss (mean over samples of
# the squared mean residual of the normalised phase field)
MASS_WEIGHT = 2.0e3
# a prediction that violates the phase-field budget by more than this
# (relative) is handed to the solver
FALLBACK_THRESHOLD = 1e-3
# the network's output is multiplied by this before it is added to the
# normalised input: one lag's increments are a few hundredths of the field
# scales, so the last layer works with numbers of order one
INCREMENT_SCALE = 0.05


def layers(cin=CIN, c1=16, c2=32, c3=64):
    """(name, c_in, c_out, stride, upsample, relu, skip-from) per layer."""
    return [
        ("e1", cin, c1, 1, 1, True, None),
        ("e2", c1, c2, 2, 1, True, None),
        ("e3", c2, c2, 1, 1, True, None),
        ("e4", c2, c3, 2, 1, True, None),
        ("b1", c3, c3, 1, 1, True, None),
        ("b2", c3, c3, 1, 1, True, None),
        ("d1", c3, c2, 1, 2, True, "e3"),
        ("d2", c2, c2, 1, 1, True, None),
        ("d3", c2, c1, 1, 2, True, "e1"),
        ("d4", c1, c1, 1, 1, True, None),
        ("out", c1, cin, 1, 1, False, None),
    ]


def pad16(c):
    return max(16, -(-c // 16) * 16)


def norm_scales(u_jet=0.02, rho_h=1.0):
    """(shift, scale) per field: xn = (x - shift) * scale."""
    shift = np.zeros(CIN, dtype=np.float32)
    scale = np.array([1.0, 1.0 / u_jet, 1.0 / u_jet, 1.0 / u_jet, 1.0 / (rho_h * u_jet * u_jet)],
                     dtype=np.float32)
    return shift, scale


class Network:
    """The encoder-decoder on a fixed batch shape [batch, 5, d, h, w]."""

    def __init__(self, batch, d, h, w, widths=(16, 32, 64), device="cuda", seed=0, lr=1e-3,
                 u_jet=0.02, increment_scale=INCREMENT_SCALE, mass_weight=MASS_WEIGHT, stream=None):
        self.dev = torch.device(device)
        self.stream = stream
        self.batch, self.shape = batch, (d, h, w)
        self.spec = layers(CIN, *widths)
        self.lr = lr
        self.t = 0
        sh, sc = norm_scales(u_jet)
        self.shift = torch.tensor(sh, device=self.dev)
        self.scale = torch.tensor(sc, device=self.dev)
        self.rs = torch.full((CIN,), float(increment_scale), dtype=torch.float32, device=self.dev)
        self.mass_weight = float(mass_weight)
        # parameter layout: per layer W [co_p][27][ci_p] then b [co_p], one flat buffer
        self.lay = {}
        off = 0
        ext = (d, h, w)
        self.ext_in = {}
        for (name, ci, co, s, u, relu, skip) in self.spec:
            cip, cop = pad16(ci), pad16(co)
            self.lay[name] = dict(ci=ci, co=co, cip=cip, cop=cop, s=s, u=u, relu=relu, skip=skip,
                                  w=off, b=off + cop * 27 * cip)
            off += cop * 27 * cip + cop
            self.ext_in[name] = ext
            ext = tuple(-(-(u * e) // s) for e in ext)
            if skip is not None:
                src = self.lay[skip]
                src_out = tuple(-(-(src["u"] * e) // src["s"]) for e in self.ext_in[skip])
                if src_out != ext:
                    raise ValueError(f"grid {d}x{h}x{w}: skip {skip}->{name} shapes differ "
                                     f"({src_out} vs {ext}); use extents divisible by 4")
        self.count = off
        f32 = dict(dtype=torch.float32, device=self.dev)
        self.P = torch.zeros(off, **f32)
        self.M = torch.zeros(off, **f32)
        self.V = torch.zeros(off, **f32)
        self.G = torch.zeros(off, **f32)
        self.Pb = torch.zeros(off, dtype=torch.bfloat16, device=self.dev)
        self.WF = {}
        self._alloc()
        self.init_params(seed)

    # ---- memory -----------------------------------------------------------
    def _act(self, name, ext=None, c=None):
        L = self.lay[name]
        e = ext if ext is not None else tuple(-(-(L["u"] * x) // L["s"]) for x in self.ext_in[name])
        return torch.empty((self.batch,) + e + (c or L["cop"],), dtype=torch.bfloat16, device=self.dev)

    def _alloc(self):
        self.y, self.yr, self.dz, self.gskip = {}, {}, {}, {}
        ws = 0
        sources = {L["skip"] for L in self.lay.values() if L["skip"]}
        for (name, *_r) in self.spec:
            L = self.lay[name]
            if L["u"] == 2 and L["s"] == 1:  # folded weights of the x2 upsampling data gradient
                self.WF[name] = torch.empty((L["cip"], 64, L["cop"]), dtype=torch.bfloat16, device=self.dev)
            else:
                self.WF[name] = torch.empty((L["cip"], 27, L["cop"]), dtype=torch.bfloat16, device=self.dev)
            self.y[name] = self._act(name)
            if L["skip"]:
                self.yr[name] = self._act(name)
            self.dz[name] = self._act(name)
            if name in sources:
                self.gskip[name] = self._act(name)
            ws = max(ws, nn.bwd_weight_workspace(self.batch, *self.ext_in[name], L["cip"], L["cop"], L["s"], L["u"]))
        self.ws = torch.empty(ws // 4 + 1, dtype=torch.float32, device=self.dev)
        d, h, w = self.shape
        self.xb = torch.empty((self.batch, d, h, w, pad16(CIN)), dtype=torch.bfloat16, device=self.dev)
        self.loss_ws = torch.empty(2048, dtype=torch.float64, device=self.dev)
        self.loss = torch.zeros(1, dtype=torch.float64, device=self.dev)

    # ---- parameters ---------------------------------------------------------
    def init_params(self, seed=0):
        """He-normal weights (the output layer scaled by 0.1), zero biases."""
        rng = np.random.default_rng(seed)
        params = {}
        for (name, ci, co, *_r) in self.spec:
            std = np.sqrt(2.0 / (ci * 27)) * (0.1 if name == "out" else 1.0)
            params[name + ".w"] = rng.standard_normal((co, ci, 3, 3, 3)) * std
            params[name + ".b"] = np.zeros(co)
        self.set_params(params)

    def set_params(self, params):
        """params: name.w [co, ci, 3, 3, 3] and name.b [co] arrays."""
        flat = np.zeros(self.count, dtype=np.float32)
        for (name, ci, co, *_r) in self.spec:
            L = self.lay[name]
            w = np.asarray(params[name + ".w"], dtype=np.float64).reshape(co, ci, 27)
            W = np.zeros((L["cop"], 27, L["cip"]), dtype=np.float32)
            W[:co, :, :ci] = w.transpose(0, 2, 1)
            flat[L["w"]:L["b"]] = W.reshape(-1)
            flat[L["b"]:L["b"] + co] = np.asarray(params[name + ".b"], dtype=np.float32)
        self.P.copy_(torch.from_numpy(flat))
        self.M.zero_()
        self.V.zero_()
        self.t = 0
        self._refresh_bf16()

    def get_params(self):
        flat = self.P.cpu().numpy()
        out = {}
        for (name, ci, co, *_r) in self.spec:
            L = self.lay[name]
            W = flat[L["w"]:L["b"]].reshape(L["cop"], 27, L["cip"])[:co, :, :ci]
            out[name + ".w"] = W.transpose(0, 2, 1).reshape(co, ci, 3, 3, 3).astype(np.float64)
            out[name + ".b"] = flat[L["b"]:L["b"] + co].astype(np.float64)
        return out

    def _refresh_bf16(self):
        # the bf16 copy is made by the optimiser kernel; a zero-learning-rate
        # step with zero moments copies the master weights exactly
        zero = torch.zeros_like(self.P)
        nn.adam(self.P, zero.clone(), zero.clone(), zero, 1, 0.0, pb=self.Pb, stream=self.stream)
        self._flip()

    def _flip(self):
        for (name, *_r) in self.spec:
            L = self.lay[name]
            if L["u"] == 2 and L["s"] == 1:
                nn.fold_up_weights(self._w(name), L["cop"], L["cip"], self.WF[name], stream=self.stream)
            else:
                nn.flip_weights(self._w(name), L["cop"], L["cip"], self.WF[name], stream=self.stream)

    def _w(self, name):
        L = self.lay[name]
        return self.Pb[L["w"]:L["b"]]

    def _b(self, name, buf=None):
        L = self.lay[name]
        return (self.P if buf is None else buf)[L["b"]:L["b"] + L["cop"]]

    def save(self, path):
        np.savez(path, **{k: v.astype(np.float32) for k, v in self.get_params().items()})

    def load(self, path):
        with np.load(path, allow_pickle=False) as z:
            self.set_params({k: z[k] for k in z.files})

    # ---- passes -------------------------------------------------------------
    def normalize(self, x, out=None):
        return nn.normalize(x, self.shift, self.scale, out=out, stream=self.stream)

    def forward(self, xn):
        """xn: normalised [batch, 5, d, h, w] float; returns the output
        layer's activation (the predicted increment, channels padded)."""
        nn.pack(xn, pad16(CIN), out=self.xb, stream=self.stream)
        h = self.xb
        for (name, *_r) in self.spec:
            L = self.lay[name]
            nn.conv3d_fwd(h, self._w(name), self._b(name), L["cop"], L["s"], L["u"], L["relu"],
                          skip=self.y[L["skip"]] if L["skip"] else None, y=self.y[name],
                          yr=self.yr.get(name), stream=self.stream)
            h = self.y[name]
        return h

    def backward(self):
        """Gradients of the loss into G, from dz['out'] (set by the loss)."""
        names = [s[0] for s in self.spec]
        for i in range(len(names) - 1, -1, -1):
            name = names[i]
            L = self.lay[name]
            x_in = self.xb if i == 0 else self.y[names[i - 1]]
            nn.conv3d_bwd_weight(x_in, self.dz[name], L["s"], L["u"], self.ws,
                                 self.G[L["w"]:L["b"]], self._b(name, self.G), stream=self.stream)
            if i == 0:
                break
            prev = names[i - 1]
            P = self.lay[prev]
            mask = None
            if P["relu"]:
                mask = self.yr[prev] if P["skip"] else self.y[prev]
            if L["u"] == 2 and L["s"] == 1:
                nn.conv3d_bwd_data_up2(self.dz[name], self.WF[name], self.batch, *self.ext_in[name], L["cip"],
                                       add=self.gskip.get(prev), mask=mask,
                                       da=self.gskip[P["skip"]] if P["skip"] else None, dzp=self.dz[prev],
                                       stream=self.stream)
            else:
                nn.conv3d_bwd_data(self.dz[name], self.WF[name], self.batch, *self.ext_in[name], L["cip"],
                                   L["s"], L["u"], add=self.gskip.get(prev), mask=mask,
                                   da=self.gskip[P["skip"]] if P["skip"] else None, dzp=self.dz[prev],
                                   stream=self.stream)

    def step(self):
        self.t += 1
        nn.adam(self.P, self.M, self.V, self.G, self.t, self.lr, pb=self.Pb, stream=self.stream)
        self._flip()

    def train_step(self, xn, tn, with_loss=True):
        """One optimiser step on normalised inputs / targets; returns the
        device scalar of the loss (before the update)."""
        r = self.forward(xn)
        nn.residual_loss(xn, tn, r, self.dz["out"], self.loss if with_loss else None, self.loss_ws,
                         rs=self.rs, mass_weight=self.mass_weight, stream=self.stream)
        self.backward()
        self.step()
        return self.loss

    def loss_and_grad(self, xn, tn):
        """Loss and gradients without an update (G holds the gradients)."""
        r = self.forward(xn)
        nn.residual_loss(xn, tn, r, self.dz["out"], self.loss, self.loss_ws, rs=self.rs,
                         mass_weight=self.mass_weight, stream=self.stream)
        self.backward()
        return self.loss

    def predict(self, x, out=None):
        """Physical fields at t + the training lag from physical fields x."""
        xn = self.normalize(x)
        r = self.forward(xn)
        return nn.unpack(xn, r, self.shift, self.scale, out=out, rs=self.rs, stream=self.stream)

    def grads(self):
        """Gradients in the layout of get_params (host float64)."""
        flat = self.G.cpu().numpy()
        out = {}
        for (name, ci, co, *_r) in self.spec:
            L = self.lay[name]
            W = flat[L["w"]:L["b"]].reshape(L["cop"], 27, L["cip"])[:co, :, :ci]
            out[name + ".w"] = W.transpose(0, 2, 1).reshape(co, ci, 3, 3, 3).astype(np.float64)
            out[name + ".b"] = flat[L["b"]:L["b"] + co].astype(np.float64)
        return out


def phase_mass(x):
    """Sum of phi per sample, FP64 (host array)."""
    return nn.phi_budget(x).cpu().numpy()[:, 0]


def mass_drift(x_prev, x, pred):
    """Relative violation of the phase-field budget by a prediction: the
    jet's liquid content changes by what the inlet injects less what leaves,
    which varies slowly from one lag to the next, so the predicted change
    sum(pred) - sum(x) is compared with the change over the previous lag,
    sum(x) - sum(x_prev), relative to sum(x).  All states are physical
    coarse fields [n, 5, d, h, w] one lag apart; returns [n] (host)."""
    m0, m1, m2 = phase_mass(x_prev), phase_mass(x), phase_mass(pred)
    return np.abs((m2 - m1) - (m1 - m0)) / np.abs(m1)


def fallback_mask(x_prev, x, pred, threshold=FALLBACK_THRESHOLD):
    """Samples whose prediction violates the phase-field budget by more
    than `threshold` (relative): the solver advances those instead."""
    return mass_drift(x_prev, x, pred) > threshold
