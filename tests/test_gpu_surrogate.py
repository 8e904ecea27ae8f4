"""GPU parity of the surrogate's kernels (through the C ABI of libsurr.so)
against the FP64 oracle in oracle/surrogate.py, on bf16-representable
inputs (so both sides start from identical values):

* forward convolution: within half a bf16 ulp of the output plus an FP32
  accumulation bound;
* data and weight gradients: the same, and FP32-level for the float
  weight gradient;
* Adam against the oracle's update;
* the whole network's loss and parameter gradients: the network stores
  activations and activation gradients in bf16 (2^-9 relative per rounding,
  about twenty roundings between the loss and the bottleneck, and ReLU
  decisions that flip on a rounding weigh most where a layer has few voxels),
  so the bound per layer is a relative L2 error <= 6e-2 with cosine >= 0.998;
  the same comparison against the oracle with its skip connections removed
  (a wiring mistake planted in the oracle, on the CPU) must break it;
* a short training run lowers the loss.
Every case covers ragged extents (not multiples of the tiles) and the three
(stride, upsample) forms."""
import sys

import numpy as np
import pytest

from oracle import surrogate as S

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _mods():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("a GPU test ran without a GPU")
    from paper_2505_12205_amd import nn, surrogate
    return torch, nn, surrogate


def _bf(a):
    """Round to the nearest bf16 value (ties to even), as float64."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(torch.bfloat16)
    return t.to(torch.float32).numpy().astype(np.float64)


def _ndhwc(torch, x, cpad):
    """[n, c, d, h, w] float64 -> device bf16 [n, d, h, w, cpad]."""
    n, c = x.shape[:2]
    out = np.zeros((n,) + x.shape[2:] + (cpad,), dtype=np.float32)
    out[..., :c] = np.moveaxis(x, 1, -1)
    return torch.from_numpy(out).to(torch.bfloat16).cuda()


def _ncdhw(t, c):
    return np.moveaxis(t.float().cpu().numpy(), -1, 1)[:, :c].astype(np.float64)


def _wdev(torch, w, cop, cip):
    co, ci = w.shape[:2]
    W = np.zeros((cop, 27, cip), dtype=np.float32)
    W[:co, :, :ci] = w.reshape(co, ci, 27).transpose(0, 2, 1)
    return torch.from_numpy(W).to(torch.bfloat16).cuda()


def _pad(c):
    return max(16, -(-c // 16) * 16)


FORMS = [(1, 1), (2, 1), (1, 2)]
CASES = [  # (ci, co, stride, up, n, d, h, w)
    (16, 16, 1, 1, 2, 5, 6, 7), (16, 32, 2, 1, 2, 7, 6, 5), (32, 64, 2, 1, 1, 6, 9, 4),
    (64, 64, 1, 1, 1, 4, 5, 6), (64, 32, 1, 2, 2, 3, 4, 5), (32, 16, 1, 2, 1, 5, 3, 4),
    (5, 16, 1, 1, 2, 6, 5, 7), (16, 5, 1, 1, 1, 5, 6, 4), (64, 16, 1, 1, 1, 9, 11, 13),
    # several LDS halo tiles / bricks along every axis, with ragged ends
    (32, 32, 1, 1, 2, 5, 19, 37), (16, 16, 1, 1, 1, 9, 17, 33), (64, 64, 1, 1, 1, 5, 11, 21),
    # every (co, ci, upsample) of the halo-brick weight gradient
    (16, 16, 1, 2, 1, 3, 5, 10), (32, 32, 1, 2, 1, 3, 5, 9), (16, 32, 1, 1, 1, 6, 9, 21),
    (32, 16, 1, 1, 2, 7, 12, 20), (16, 32, 1, 2, 1, 4, 3, 9),
    # the upsampling halo-tile forwards over several tiles, ragged
    (32, 16, 1, 2, 2, 5, 9, 20), (64, 32, 1, 2, 1, 4, 9, 17),
    # the stride-2 data gradient by parity class over several waves, ragged
    (16, 32, 2, 1, 1, 9, 20, 37), (64, 32, 2, 1, 1, 5, 17, 33),
]


@pytest.mark.parametrize("case", CASES)
def test_conv_forward(case):
    torch, nn, _ = _mods()
    ci, co, s, u, n, d, h, w = case
    rng = np.random.default_rng(sum(case))
    x = _bf(rng.standard_normal((n, ci, d, h, w)))
    wt = _bf(rng.standard_normal((co, ci, 3, 3, 3)) * np.sqrt(2.0 / (27 * ci)))
    b = rng.standard_normal(co).astype(np.float32).astype(np.float64) * 0.1
    cip, cop = _pad(ci), _pad(co)
    z = S.conv3d(x, wt, b, s, u)
    zabs = S.conv3d(np.abs(x), np.abs(wt), np.abs(b), s, u)
    bias = torch.zeros(cop, dtype=torch.float32, device="cuda")
    bias[:co] = torch.from_numpy(b.astype(np.float32))
    skip_np = _bf(rng.standard_normal(z.shape))
    skip = _ndhwc(torch, skip_np, cop)
    for relu, use_skip in [(True, False), (False, False), (True, True)]:
        _log(f"[gpu] conv fwd {case} relu={relu} skip={use_skip}")
        yr = torch.empty_like(skip) if use_skip else None
        y = nn.conv3d_fwd(_ndhwc(torch, x, cip), _wdev(torch, wt, cop, cip), bias, cop, s, u, relu,
                          skip=skip if use_skip else None, yr=yr)
        ref = np.maximum(z, 0) if relu else z
        full = ref + (skip_np if use_skip else 0.0)
        got = _ncdhw(y, co)
        # half a bf16 ulp of the stored value plus the FP32 accumulation bound
        err = np.abs(got - full)
        _log(f"conv fwd {case} relu={relu} skip={use_skip}: max err {err.max():.3e}, "
             f"max |y| {np.abs(full).max():.3e}")
        assert (err <= 2.0 ** -8 * np.abs(full) + 1e-5 * zabs + 1e-6).all()
        if use_skip:
            assert (np.abs(_ncdhw(yr, co) - ref) <= 2.0 ** -8 * np.abs(ref) + 1e-5 * zabs + 1e-6).all()
        if cop > co:  # padding channels of the output stay zero (no relu of a bias: biases are zero there)
            assert (y[..., co:].float() == 0).all()


@pytest.mark.parametrize("case", CASES)
def test_conv_data_gradient(case):
    torch, nn, _ = _mods()
    ci, co, s, u, n, d, h, w = case
    rng = np.random.default_rng(100 + sum(case))
    wt = _bf(rng.standard_normal((co, ci, 3, 3, 3)) * 0.2)
    od, oh, ow = S.out_shape(d, h, w, s, u)
    dz = _bf(rng.standard_normal((n, co, od, oh, ow)))
    x = np.zeros((n, ci, d, h, w))
    dx, _, _ = S.conv3d_backward(x, wt, dz, s, u)
    dxa, _, _ = S.conv3d_backward(x, np.abs(wt), np.abs(dz), s, u)
    cip, cop = _pad(ci), _pad(co)
    W = _wdev(torch, wt, cop, cip)
    WT = torch.empty((cip, 27, cop), dtype=torch.bfloat16, device="cuda")
    nn.flip_weights(W, cop, cip, WT)
    add = _bf(rng.standard_normal(dx.shape))
    mask = _bf(rng.standard_normal(dx.shape))
    _log(f"[gpu] conv data grad {case}")
    da = torch.empty((n, d, h, w, cip), dtype=torch.bfloat16, device="cuda")
    dzp = nn.conv3d_bwd_data(_ndhwc(torch, dz, cop), WT, n, d, h, w, cip, s, u, add=_ndhwc(torch, add, cip),
                             mask=_ndhwc(torch, mask, cip), da=da)
    g = dx + add
    tol = 2.0 ** -8 * np.abs(g) + 1e-5 * (dxa + np.abs(add)) + 1e-6
    e1 = np.abs(_ncdhw(da, ci) - g)
    _log(f"conv data grad {case}: max err {e1.max():.3e}, max |g| {np.abs(g).max():.3e}")
    assert (e1 <= tol).all()
    assert (np.abs(_ncdhw(dzp, ci) - g * (mask > 0)) <= tol).all()
    plain = nn.conv3d_bwd_data(_ndhwc(torch, dz, cop), WT, n, d, h, w, cip, s, u)
    assert (np.abs(_ncdhw(plain, ci) - dx) <= 2.0 ** -8 * np.abs(dx) + 1e-5 * dxa + 1e-6).all()
    if s == 1 and u == 2:
        # the folded form: the folded weights are rounded once more to bf16
        # (half an ulp, 2^-9 of each, bounded by the gradient of |w| and |dz|)
        WU = nn.fold_up_weights(W, cop, cip)
        da2 = torch.empty_like(da)
        dzp2 = nn.conv3d_bwd_data_up2(_ndhwc(torch, dz, cop), WU, n, d, h, w, cip, add=_ndhwc(torch, add, cip),
                                      mask=_ndhwc(torch, mask, cip), da=da2)
        tol2 = tol + 2.0 ** -9 * dxa
        e2 = np.abs(_ncdhw(da2, ci) - g)
        _log(f"conv data grad {case} (folded): max err {e2.max():.3e}")
        assert (e2 <= tol2).all()
        assert (np.abs(_ncdhw(dzp2, ci) - g * (mask > 0)) <= tol2).all()
        plain2 = nn.conv3d_bwd_data_up2(_ndhwc(torch, dz, cop), WU, n, d, h, w, cip)
        assert (np.abs(_ncdhw(plain2, ci) - dx) <= 2.0 ** -8 * np.abs(dx) + (1e-5 + 2.0 ** -9) * dxa + 1e-6).all()


@pytest.mark.parametrize("case", CASES)
def test_conv_weight_gradient(case):
    torch, nn, _ = _mods()
    ci, co, s, u, n, d, h, w = case
    rng = np.random.default_rng(200 + sum(case))
    x = _bf(rng.standard_normal((n, ci, d, h, w)))
    od, oh, ow = S.out_shape(d, h, w, s, u)
    dz = _bf(rng.standard_normal((n, co, od, oh, ow)))
    _, dw, db = S.conv3d_backward(x, np.zeros((co, ci, 3, 3, 3)), dz, s, u)
    _, dwa, dba = S.conv3d_backward(np.abs(x), np.zeros((co, ci, 3, 3, 3)), np.abs(dz), s, u)
    cip, cop = _pad(ci), _pad(co)
    ws = torch.empty(nn.bwd_weight_workspace(n, d, h, w, cip, cop, s, u) // 4 + 1, device="cuda")
    DW = torch.empty((cop, 27, cip), dtype=torch.float32, device="cuda")
    DB = torch.empty(cop, dtype=torch.float32, device="cuda")
    _log(f"[gpu] conv weight grad {case}")
    nn.conv3d_bwd_weight(_ndhwc(torch, x, cip), _ndhwc(torch, dz, cop), s, u, ws, DW, DB)
    got = DW.cpu().numpy().astype(np.float64)
    got_w = got[:co, :, :ci].transpose(0, 2, 1).reshape(co, ci, 3, 3, 3)
    e = np.abs(got_w - dw)
    _log(f"conv weight grad {case}: max err {e.max():.3e}, max |dw| {np.abs(dw).max():.3e}")
    assert (e <= 1e-5 * dwa + 1e-6).all()
    assert (np.abs(got[co:]) == 0).all() and (np.abs(got[:, :, ci:]) == 0).all()
    gb = DB.cpu().numpy().astype(np.float64)
    assert (np.abs(gb[:co] - db) <= 1e-5 * dba + 1e-6).all() and (gb[co:] == 0).all()


def test_adam_matches_oracle():
    torch, nn, _ = _mods()
    rng = np.random.default_rng(5)
    P = {"a": rng.standard_normal(1000)}
    st = {"t": 0, "m": {}, "v": {}}
    p = torch.tensor(P["a"], dtype=torch.float32, device="cuda")
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    pb = torch.empty(1000, dtype=torch.bfloat16, device="cuda")
    for t in range(1, 6):
        g = rng.standard_normal(1000)
        S.adam_step(P, {"a": g}, st, lr=1e-2)
        nn.adam(p, m, v, torch.tensor(g, dtype=torch.float32, device="cuda"), t, 1e-2, pb=pb)
    got = p.cpu().numpy().astype(np.float64)
    assert np.abs(got - P["a"]).max() < 1e-5
    assert (pb.float().cpu().numpy() == _bf(got)).all()


def _net_case(torch, surrogate, widths=(16, 32, 16), shape=(8, 8, 12), batch=2, seed=3, scale=1.0, mw=0.0):
    net = surrogate.Network(batch, *shape, widths=widths, seed=seed, increment_scale=scale, mass_weight=mw)
    params = net.get_params()
    rng = np.random.default_rng(seed)
    for k in params:  # bf16-representable weights, non-zero biases
        if k.endswith(".w"):
            params[k] = _bf(params[k])
        else:
            params[k] = rng.standard_normal(params[k].shape).astype(np.float32).astype(np.float64) * 0.05
    net.set_params(params)
    x = _bf(rng.standard_normal((batch, 5) + shape))
    t = _bf(x + 0.1 * rng.standard_normal(x.shape))
    return net, params, x, t


def test_network_loss_and_gradients_match_oracle():
    torch, nn, surrogate = _mods()
    net, params, x, t = _net_case(torch, surrogate)
    spec = S.layers(5, *(16, 32, 16))
    Lo, Go = S.loss_and_grad(params, spec, x, t, net.rs[0].item())
    xn = torch.tensor(x, dtype=torch.float32, device="cuda")
    tn = torch.tensor(t, dtype=torch.float32, device="cuda")
    _log("[gpu] network loss and gradients")
    Lg = float(net.loss_and_grad(xn, tn).item())
    Gg = net.grads()
    _log(f"network loss gpu {Lg:.6e} oracle {Lo:.6e}")
    assert abs(Lg - Lo) <= 1e-2 * Lo
    def rel_cos(a, b):
        a, b = a.ravel(), b.ravel()
        return (np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30),
                a @ b / max(np.linalg.norm(a) * np.linalg.norm(b), 1e-30))

    for k in Go:
        rel, cos = rel_cos(Gg[k], Go[k])
        _log(f"grad {k}: rel L2 {rel:.3e} cos {cos:.6f}")
        assert rel <= 6e-2 and cos >= 0.998, k
    # discrimination: an oracle without the skip connections is far outside the bound
    bad = [(n, ci, co, s_, u_, r_, None) for (n, ci, co, s_, u_, r_, _) in spec]
    _, Gb = S.loss_and_grad(params, bad, x, t, net.rs[0].item())
    worst = max(rel_cos(Gg[k], Gb[k])[0] for k in Gb)
    _log(f"against the mis-wired oracle: worst rel L2 {worst:.3e}")
    assert worst > 0.3


def test_training_lowers_the_loss():
    torch, nn, surrogate = _mods()
    rng = np.random.default_rng(11)
    batch, shape = 4, (16, 16, 16)
    net = surrogate.Network(batch, *shape, seed=1, lr=2e-3, increment_scale=1.0, mass_weight=0.0)
    # a learnable map: the target is the input advected by one cell along z
    x = rng.standard_normal((batch, 5) + shape).astype(np.float32)
    t = np.roll(x, 1, axis=2) * 0.9
    xn = torch.tensor(x, device="cuda")
    tn = torch.tensor(t, device="cuda")
    losses = []
    _log("[gpu] training 300 steps")
    for k in range(300):
        losses.append(float(net.train_step(xn, tn).item()))
    _log(f"training loss {losses[0]:.4f} -> {losses[-1]:.4f}")
    assert np.isfinite(losses).all()
    assert losses[-1] < 0.6 * losses[0]


def test_network_increment_scale_and_mass_term():
    """The production increment scale and phase-field content weight enter
    the prediction, the loss and its gradient: loss and the output layer's
    gradients against the oracle with the same settings (the layers below
    are covered at scale 1 without the content term)."""
    torch, nn, surrogate = _mods()
    net, params, x, t = _net_case(torch, surrogate, scale=surrogate.INCREMENT_SCALE, seed=5,
                                  mw=surrogate.MASS_WEIGHT)
    t[:, 0] += 1e-3  # a phase-field content offset, so the mass term matters
    spec = S.layers(5, *(16, 32, 16))
    Lo, Go = S.loss_and_grad(params, spec, x, t, surrogate.INCREMENT_SCALE, surrogate.MASS_WEIGHT)
    xn = torch.tensor(x, dtype=torch.float32, device="cuda")
    tn = torch.tensor(t, dtype=torch.float32, device="cuda")
    _log("[gpu] network increment scale")
    Lg = float(net.loss_and_grad(xn, tn).item())
    Gg = net.grads()
    assert abs(Lg - Lo) <= 1e-3 * Lo
    for k in ("out.w", "out.b", "d4.w"):
        a, b = Gg[k].ravel(), Go[k].ravel()
        rel = np.linalg.norm(a - b) / np.linalg.norm(b)
        _log(f"scale {surrogate.INCREMENT_SCALE}: grad {k} rel L2 {rel:.3e}")
        assert rel <= 2e-2, k
    # predict() takes physical fields and returns physical fields
    sh, sc = surrogate.norm_scales()
    sc5 = sc[None, :, None, None, None].astype(np.float64)
    phys = torch.tensor(x / sc5, dtype=torch.float32, device="cuda")
    pred = net.predict(phys).cpu().numpy().astype(np.float64) * sc5
    po, _ = S.forward(params, spec, x, surrogate.INCREMENT_SCALE)
    e = np.abs(pred - po).max()
    _log(f"predict() in normalised units: max err {e:.3e}")
    assert e < 2e-2
