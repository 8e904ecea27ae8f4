"""FP64 CPU oracle of the learned surrogate: a 3D convolutional
encoder-decoder that advances coarse (phi, u, v, w, p) fields by a fixed
number of solver steps, its gradients and its optimiser step.

TEST INFRASTRUCTURE ONLY (the tests, the smoke check and the benchmark's
CPU-baseline leg).  It shares no code with the HIP implementation; both
sides take the same network description (layer list below) and the same
seeded inputs.

The paper has no passage on a learned part: the network, its loss and its
optimiser are this project's own definitions, written out plainly here:

* conv3d (3 x 3 x 3 taps, zero padding 1, stride s in {1, 2}, optional
  nearest-neighbour input upsampling by u in {1, 2}):
      y[n, o, p] = b[o] + sum_{c, k} w[o, c, k] * X[n, c, s p + k - 1],
  X the (upsampled, u = 2: X[q] = x[q // 2]) input, zero outside its extent.
* relu(z) = max(z, 0); skip connections add a stored activation after the
  relu; the output is the input plus the last (linear) layer times a fixed
  increment scale: x + scale r(x).
* loss = mean over all elements of (prediction - target)^2, optionally plus
  a weight times the mean over samples of the squared mean residual of the
  phase field (channel 0).
* Adam with bias correction (Kingma & Ba, Algorithm 1).

Everything is float64 numpy: np.einsum over the channel axis is the only
library primitive, applied once per tap.
"""
from __future__ import annotations

import numpy as np

# ---------------------------------------------------------------------------
# network description: (name, c_in, c_out, stride, upsample, relu, skip-from)
# channels (c1, c2, c3) = (16, 32, 64) for the production network
# ---------------------------------------------------------------------------


def layers(cin=5, c1=16, c2=32, c3=64):
    """Layer list of the encoder-decoder.  skip-from names an earlier layer
    whose (post-relu) output is added to this layer's post-relu output."""
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


def n_params(spec):
    return sum(co * ci * 27 + co for (_, ci, co, _, _, _, _) in spec)


def init_params(spec, seed=0):
    """He-normal weights, zero biases, the last layer scaled by 0.1."""
    rng = np.random.default_rng(seed)
    P = {}
    for (name, ci, co, _, _, _, _) in spec:
        std = np.sqrt(2.0 / (ci * 27))
        if name == "out":
            std *= 0.1
        P[name + ".w"] = rng.standard_normal((co, ci, 3, 3, 3)) * std
        P[name + ".b"] = np.zeros(co)
    return P


# ---------------------------------------------------------------------------
# conv3d by its definition
# ---------------------------------------------------------------------------

def out_shape(D, H, W, s, u):
    """Output extent of a padded 3^3 conv with stride s on an input
    upsampled by u: ceil(u n / s)."""
    return tuple(-(-(u * n) // s) for n in (D, H, W))


def _upsample(x, u):
    if u == 1:
        return x
    return x.repeat(u, axis=2).repeat(u, axis=3).repeat(u, axis=4)


def conv3d(x, w, b, s=1, u=1):
    """x [N, Ci, D, H, W], w [Co, Ci, 3, 3, 3], b [Co] -> [N, Co, Do, Ho, Wo]."""
    X = np.pad(_upsample(x, u), ((0, 0), (0, 0), (1, 1), (1, 1), (1, 1)))
    N = x.shape[0]
    Do, Ho, Wo = out_shape(*x.shape[2:], s, u)
    y = np.zeros((N, w.shape[0], Do, Ho, Wo))
    for kz in range(3):
        for ky in range(3):
            for kx in range(3):
                # X index s p + k - 1 of the unpadded input = s p + k here
                xs = X[:, :, kz:kz + s * Do:s, ky:ky + s * Ho:s, kx:kx + s * Wo:s]
                y += np.einsum("oc,ncdhw->nodhw", w[:, :, kz, ky, kx], xs)
    return y + b[None, :, None, None, None]


def conv3d_backward(x, w, dy, s=1, u=1):
    """Gradients of sum(dy * conv3d(x, w, b, s, u)) with respect to x, w, b
    (the adjoint of each term of the definition)."""
    N, Ci, D, H, W = x.shape
    Do, Ho, Wo = dy.shape[2:]
    Xu = _upsample(x, u)
    X = np.pad(Xu, ((0, 0), (0, 0), (1, 1), (1, 1), (1, 1)))
    dX = np.zeros_like(X)
    dw = np.zeros_like(w)
    for kz in range(3):
        for ky in range(3):
            for kx in range(3):
                sl = (slice(None), slice(None), slice(kz, kz + s * Do, s), slice(ky, ky + s * Ho, s),
                      slice(kx, kx + s * Wo, s))
                dw[:, :, kz, ky, kx] = np.einsum("nodhw,ncdhw->oc", dy, X[sl])
                dX[sl] += np.einsum("oc,nodhw->ncdhw", w[:, :, kz, ky, kx], dy)
    dXu = dX[:, :, 1:-1, 1:-1, 1:-1]
    if u == 1:
        dx = dXu
    else:  # adjoint of the repeat: sum over each u^3 block
        dx = dXu.reshape(N, Ci, D, u, H, u, W, u).sum(axis=(3, 5, 7))
    db = dy.sum(axis=(0, 2, 3, 4))
    return dx, dw, db


def conv3d_direct(x, w, b, s=1, u=1):
    """The same definition with explicit loops (tiny inputs only)."""
    N, Ci, D, H, W = x.shape
    Co = w.shape[0]
    Do, Ho, Wo = out_shape(D, H, W, s, u)
    y = np.zeros((N, Co, Do, Ho, Wo))
    for n in range(N):
        for o in range(Co):
            for pz in range(Do):
                for py in range(Ho):
                    for px in range(Wo):
                        acc = b[o]
                        for kz in range(3):
                            qz = s * pz + kz - 1
                            if qz < 0 or qz >= u * D:
                                continue
                            for ky in range(3):
                                qy = s * py + ky - 1
                                if qy < 0 or qy >= u * H:
                                    continue
                                for kx in range(3):
                                    qx = s * px + kx - 1
                                    if qx < 0 or qx >= u * W:
                                        continue
                                    for c in range(Ci):
                                        acc += w[o, c, kz, ky, kx] * x[n, c, qz // u, qy // u, qx // u]
                        y[n, o, pz, py, px] = acc
    return y


# ---------------------------------------------------------------------------
# network forward / backward, loss, optimiser
# ---------------------------------------------------------------------------

def forward(P, spec, x, scale=1.0):
    """Returns (prediction x + scale r(x), cache).  cache[name] = (input,
    pre-activation)."""
    cache = {}
    h = x
    out = {}
    for (name, ci, co, s, u, relu, skip) in spec:
        z = conv3d(h, P[name + ".w"], P[name + ".b"], s, u)
        a = np.maximum(z, 0.0) if relu else z
        if skip is not None:
            a = a + out[skip]
        cache[name] = (h, z)
        out[name] = a
        h = a
    return x + scale * h, cache


def mse(pred, target, mass_weight=0.0):
    """Mean squared error, plus mass_weight * mean over samples of the
    squared mean phase-field residual (channel 0): the prediction should
    carry the target's phase-field content.  Returns (L, dL/dpred)."""
    d = pred - target
    L = float(np.mean(d * d))
    g = 2.0 * d / d.size
    if mass_weight:
        N = d.shape[0]
        V = d[0, 0].size
        m = d[:, 0].reshape(N, -1).sum(axis=1) / V  # mean residual of phi per sample
        L += mass_weight * float(np.mean(m * m))
        g[:, 0] += (mass_weight * 2.0 * m / (N * V))[:, None, None, None]
    return L, g


def backward(P, spec, cache, dpred, scale=1.0):
    """Gradients of the loss given dL/dprediction."""
    G = {}
    dout = {name: None for (name, *_rest) in spec}
    dh = scale * dpred  # into the last layer's output (the scaled residual branch)
    for (name, ci, co, s, u, relu, skip) in reversed(spec):
        da = dh if dout[name] is None else dh + dout[name]
        if skip is not None:  # a = relu(z) + out[skip]
            dout[skip] = da if dout[skip] is None else dout[skip] + da
        h, z = cache[name]
        dz = da * (z > 0.0) if relu else da
        dx, dw, db = conv3d_backward(h, P[name + ".w"], dz, s, u)
        G[name + ".w"] = dw
        G[name + ".b"] = db
        dh = dx
    return G, dh + dpred  # d/dx includes the identity path


def loss_and_grad(P, spec, x, target, scale=1.0, mass_weight=0.0):
    pred, cache = forward(P, spec, x, scale)
    L, dpred = mse(pred, target, mass_weight)
    G, _ = backward(P, spec, cache, dpred, scale)
    return L, G


def adam_step(P, G, state, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update in place; state = {'t': int, 'm': {}, 'v': {}}."""
    state["t"] += 1
    t = state["t"]
    for k in P:
        m = state["m"].get(k, np.zeros_like(P[k]))
        v = state["v"].get(k, np.zeros_like(P[k]))
        m = beta1 * m + (1 - beta1) * G[k]
        v = beta2 * v + (1 - beta2) * G[k] * G[k]
        mh = m / (1 - beta1 ** t)
        vh = v / (1 - beta2 ** t)
        P[k] = P[k] - lr * mh / (np.sqrt(vh) + eps)
        state["m"][k] = m
        state["v"][k] = v
    return P


# ---------------------------------------------------------------------------
# coarse fields from solver output
# ---------------------------------------------------------------------------

def pool2(f):
    """2 x 2 x 2 average of a [..., D, H, W] array (even extents)."""
    *lead, D, H, W = f.shape
    return f.reshape(*lead, D // 2, 2, H // 2, 2, W // 2, 2).mean(axis=(-5, -3, -1))


def relative_mass_drift(pred_phi, ref_phi):
    """|sum pred - sum ref| / sum ref per sample (the fallback criterion)."""
    axes = tuple(range(1, pred_phi.ndim))
    sr = ref_phi.sum(axis=axes)
    return np.abs(pred_phi.sum(axis=axes) - sr) / np.abs(sr)
