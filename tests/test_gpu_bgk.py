"""GPU parity of the selectable BGK operator of the hydrodynamic set
(Eqs. bgk_collision and viscous_force_bgk, cfg["collision"] = "bgk") against
the FP64 oracle on the same seeded inputs:

* one even and one odd step at every node from the same FP32 state, for a
  jet (inlet, convective outlet, free-slip sides: the face kernels) and for
  x walls (wall lanes of the tiled kernel), at the FP32 rounding level;
* 1000 steps of a D2Q9 drop (rho* = 10, tau_L = 0.03) and of the
  Rayleigh-Taylor copy (tau_H = 0.01, s = 1.96): max|dphi| <= 1e-5,
  rel_u <= 1e-4;
* FP16 deviation storage on the drop: max|dphi| <= 1e-3;
* the operator switch changes the flow (BGK differs from WMRT);
* a stability map of both operators over density ratio and s_L -> 2."""
import sys

import numpy as np
import pytest

import oracle
from paper_2505_12205_amd import workloads as W

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("a GPU test ran without a GPU")
    from paper_2505_12205_amd import lbm
    return lbm


def _bgk(cfg):
    return dict(cfg, collision="bgk", name=cfg.get("name", "case") + "_bgk")


def _one_step_every_node(cfg, phi0, u0, tile=None):
    lbm = _lbm()
    s = lbm.Sim(cfg, phi0, u0)
    if tile:
        s.set_tile(*tile)
    s.step(5)
    q = cfg["q"]
    for _ in range(2):
        h, g, u = [t.cpu().numpy() for t in s.export_state()]
        _log(f"[gpu] bgk {cfg['name']} one step at parity {s.steps_done % 2}")
        s.step(1)
        h1, g1, u1 = [t.cpu().numpy() for t in s.export_state()]
        nodes = np.arange(h.reshape(q, -1).shape[1])
        ho, go, uo = oracle.step_nodes_f32(cfg, h, g, u, nodes)
        eh = np.abs(h1.reshape(q, -1).T - ho).max()
        eg = np.abs(g1.reshape(q, -1).T - go).max()
        eu = np.abs(u1.reshape(3, -1).T - uo).max()
        _log(f"bgk {cfg['name']}: max|dh|={eh:.3e} max|dg|={eg:.3e} max|du|={eu:.3e}")
        assert eh < 2e-7 and eg < 2e-7 and eu < 2e-7


def test_bgk_one_step_every_node_jet_faces():
    cfg, phi0, u0 = W.jet3d(nx=20, ny=18, nz=30, radius=5.0, param_radius=12.0, stub=10.0)
    phi0, u0 = W.perturb(phi0, u0, 9, 0.01, 1e-3)
    _one_step_every_node(_bgk(cfg), phi0, u0)


@pytest.mark.parametrize("q", (19, 9))
def test_bgk_one_step_every_node_x_walls(q):
    if q == 19:
        cfg, phi0, u0 = W.rt3d(nx=21, ny=26, nz=9, lref=256)
        cfg = dict(cfg, bc=("noslip", "freeslip", "noslip", "noslip", "periodic", "periodic"))
    else:
        cfg, phi0, u0 = W.drop2d(n=32, radius=9.0, center=(13.0, 17.0), rho_l=0.1, visc_ratio=10.0)
        cfg = dict(cfg, bc=("freeslip", "freeslip", "noslip", "noslip", "periodic", "periodic"))
    phi0, u0 = W.perturb(phi0, u0, 11, 0.01, 2e-3)
    _one_step_every_node(_bgk(cfg), phi0, u0, tile=(16, 4))


def _parity(cfg, phi0, u0, steps, uref, storage="fp32"):
    lbm = _lbm()
    _log(f"[gpu] bgk {cfg['name']} storage={storage} steps={steps}")
    o = oracle.Oracle(cfg).init(phi0, u0).step(steps)
    phi_o, u_o, _ = o.fields()
    s = lbm.Sim(cfg, phi0, u0, storage=storage).step(steps)
    phi_g, u_g, _ = [t.cpu().numpy().astype(np.float64) for t in s.fields()]
    ephi = np.abs(phi_g - phi_o).max()
    eu = np.abs(u_g - u_o).max() / max(np.abs(u_o).max(), 1e-30)
    _log(f"bgk {cfg['name']} {storage}: max|dphi|={ephi:.3e} rel_u={eu:.3e}")
    return ephi, eu, u_g


def test_bgk_drop2d_fp32_and_fp16_1000_steps():
    cfg, phi0, u0 = W.drop2d(rho_l=0.1, visc_ratio=10.0)
    cfg = _bgk(cfg)
    uref = cfg["sigma"] / (cfg["rho_h"] * cfg["tau_h"] / 3)
    ephi, eu, u_bgk = _parity(cfg, phi0, u0, 1000, uref)
    assert ephi <= 1e-5 and eu <= 1e-4
    ephi16, _, _ = _parity(cfg, phi0, u0, 1000, uref, storage="fp16")
    assert ephi16 <= 1e-3
    # the switch is live: WMRT on the same input gives another flow
    lbm = _lbm()
    s = lbm.Sim(dict(cfg, collision="wmrt"), phi0, u0).step(1000)
    u_w = s.fields()[1].cpu().numpy()
    assert np.abs(u_w - u_bgk).max() > 1e-3 * np.abs(u_w).max()


def test_bgk_rt3d_copy_fp32_1000_steps():
    cfg, phi0, u0 = W.rt3d(nx=32, ny=48, nz=16, lref=256)
    phi0, u0 = W.perturb(phi0, u0, 21, 0.01, 1e-3)
    ephi, eu, _ = _parity(_bgk(cfg), phi0, u0, 1000, 0.04)
    assert ephi <= 1e-5 and eu <= 1e-4


def _steps_to_divergence(lbm, cfg, phi0, total, chunk):
    s = lbm.Sim(cfg, phi0)
    for k in range(total // chunk):
        s.step(chunk)
        try:
            s.reduce()
        except lbm.LbmError as e:
            if e.code != lbm.LBM_EUNSTABLE:
                raise
            return (k + 1) * chunk
    return None


def test_bgk_and_wmrt_stability_map():
    """Stability of the two operators on the 128 x 128 drop (R = 25,
    tau_H = 0.3) over density ratio and light-fluid relaxation rate
    s_L = 1/(tau_L + 1/2) -> 2: WMRT stays finite for 4000 steps in every
    case; BGK does at rho* = 10 and diverges at rho* = 1000."""
    lbm = _lbm()
    rows = {}
    for rl in (0.1, 0.01, 0.001):
        for vr in (10.0, 100.0, 1000.0):
            cfg, phi0, _ = W.drop2d(rho_l=rl, visc_ratio=vr)
            res = [_steps_to_divergence(lbm, dict(cfg, collision=op), phi0, 4000, 250) for op in ("wmrt", "bgk")]
            rows[(rl, vr)] = res
            _log(f"stability rho*={1 / rl:g} tau_L={cfg['tau_l']:.4g} s_L={1 / (cfg['tau_l'] + 0.5):.4f}: "
                 f"wmrt {'finite' if res[0] is None else 'diverged by %d' % res[0]}, "
                 f"bgk {'finite' if res[1] is None else 'diverged by %d' % res[1]}")
    assert all(r[0] is None for r in rows.values())
    assert all(rows[(0.1, vr)][1] is None for vr in (10.0, 100.0, 1000.0))
    assert all(rows[(0.001, vr)][1] is not None for vr in (10.0, 100.0, 1000.0))
