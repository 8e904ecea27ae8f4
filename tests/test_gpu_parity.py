"""GPU parity: the HIP path (through the C-ABI) against the FP64 oracle on
the same seeded inputs.

Tolerances (FP32 storage and compute, after 1000 steps unless stated):
  max |phi_gpu - phi_oracle| <= 1e-5,
  max |u_gpu - u_oracle| / max |u_oracle| <= 1e-4
(the velocity error relative to the oracle field's own largest speed, also
for the drop at rest, whose speeds are spurious currents of order 1e-5).
16-bit storage: max |phi_gpu - phi_oracle| <= 1e-3."""
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


def _run_gpu(cfg, phi0, u0, steps, storage="fp32", tile=None):
    lbm = _lbm()
    _log(f"[gpu] {cfg.get('name', cfg['q'])} storage={storage} steps={steps} tile={tile}")
    s = lbm.Sim(cfg, phi0, u0, storage=storage)
    if tile:
        s.set_tile(*tile)
    s.step(steps)
    phi, u, p = s.fields()
    return s, phi.cpu().numpy().astype(np.float64), u.cpu().numpy().astype(np.float64), p.cpu().numpy()


def _run_oracle(cfg, phi0, u0, steps):
    o = oracle.Oracle(cfg).init(phi0, u0)
    o.step(steps)
    phi, u, p = o.fields()
    return o, phi, u, p


def _errors(phi_g, u_g, phi_o, u_o, uref=None):
    """max |dphi| and the velocity error relative to max |u_oracle| (uref is
    kept only to name the case's velocity scale in the log)."""
    ephi = np.abs(phi_g - phi_o).max()
    eu = np.abs(u_g - u_o).max() / max(np.abs(u_o).max(), 1e-30)
    return ephi, eu


_ORACLE_CACHE = {}


def _oracle_cached(key, cfg, phi0, u0, steps):
    if key not in _ORACLE_CACHE:
        _ORACLE_CACHE[key] = _run_oracle(cfg, phi0, u0, steps)
    return _ORACLE_CACHE[key]


def test_drop2d_fp32_1000_steps():
    cfg, phi0, u0 = W.drop2d()
    _, phi_o, u_o, _ = _oracle_cached("drop", cfg, phi0, u0, 1000)
    _, phi_g, u_g, _ = _run_gpu(cfg, phi0, u0, 1000)
    ephi, eu = _errors(phi_g, u_g, phi_o, u_o, cfg["sigma"] / (cfg["rho_h"] * cfg["tau_h"] / 3))
    _log(f"drop2d: max|dphi|={ephi:.3e} rel_u={eu:.3e}")
    assert ephi <= 1e-5 and eu <= 1e-4


def _rt_copy(nx, ny, nz, seed=None):
    cfg, phi0, u0 = W.rt3d(nx=nx, ny=ny, nz=nz, lref=256)
    if seed is not None:
        phi0, u0 = W.perturb(phi0, u0, seed, 0.01, 1e-3)
    return cfg, phi0, u0


def test_rt3d_copy_fp32_1000_steps():
    cfg, phi0, u0 = _rt_copy(32, 48, 16, seed=21)
    _, phi_o, u_o, _ = _oracle_cached("rt", cfg, phi0, u0, 1000)
    _, phi_g, u_g, _ = _run_gpu(cfg, phi0, u0, 1000)
    ephi, eu = _errors(phi_g, u_g, phi_o, u_o, 0.04)
    _log(f"rt3d copy: max|dphi|={ephi:.3e} rel_u={eu:.3e}")
    assert ephi <= 1e-5 and eu <= 1e-4


@pytest.mark.parametrize("shape,tile", [((37, 29, 11), (64, 4)), ((37, 29, 11), (32, 8)),
                                        ((3, 5, 4), (16, 4)), ((70, 9, 3), (128, 2))])
def test_rt3d_ragged_tiles(shape, tile):
    cfg, phi0, u0 = _rt_copy(*shape, seed=5)
    _, phi_o, u_o, _ = _run_oracle(cfg, phi0, u0, 101)
    _, phi_g, u_g, _ = _run_gpu(cfg, phi0, u0, 101, tile=tile)
    ephi, eu = _errors(phi_g, u_g, phi_o, u_o, 0.04)
    _log(f"ragged {shape} {tile}: max|dphi|={ephi:.3e} rel_u={eu:.3e}")
    assert ephi <= 1e-5 and eu <= 1e-4


def _jet_copy(nx=24, ny=24, nz=48, radius=6.0, seed=None):
    cfg, phi0, u0 = W.jet3d(nx=nx, ny=ny, nz=nz, radius=radius, param_radius=12.0, stub=10.0)
    if seed is not None:
        phi0, u0 = W.perturb(phi0, u0, seed, 0.01, 1e-3)
    return cfg, phi0, u0


def test_jet_copy_fp32_inlet_outlet_freeslip():
    cfg, phi0, u0 = _jet_copy(seed=3)
    _, phi_o, u_o, _ = _oracle_cached("jet", cfg, phi0, u0, 1000)
    _, phi_g, u_g, _ = _run_gpu(cfg, phi0, u0, 1000)
    ephi, eu = _errors(phi_g, u_g, phi_o, u_o, cfg["inlet_u"])
    _log(f"jet copy fp32: max|dphi|={ephi:.3e} rel_u={eu:.3e}")
    assert ephi <= 1e-5 and eu <= 1e-4


@pytest.mark.parametrize("storage", ["fp16", "bf16"])
def test_jet_copy_16bit_storage(storage):
    cfg, phi0, u0 = _jet_copy(seed=3)
    _, phi_o, u_o, p_o = _oracle_cached("jet", cfg, phi0, u0, 1000)
    _, phi_g, u_g, p_g = _run_gpu(cfg, phi0, u0, 1000, storage=storage)
    ephi, eu = _errors(phi_g, u_g, phi_o, u_o, cfg["inlet_u"])
    ep = np.abs(p_g - p_o).max()
    _log(f"jet copy {storage}: max|dphi|={ephi:.3e} rel_u={eu:.3e} max|dp|={ep:.3e}")
    # both 16-bit forms meet the 1e-3 bar (BF16 through stochastic rounding)
    assert ephi <= 1e-3


def test_drop2d_16bit_storage():
    cfg, phi0, u0 = W.drop2d()
    _, phi_o, u_o, _ = _oracle_cached("drop", cfg, phi0, u0, 1000)
    for storage in ("fp16", "bf16"):
        _, phi_g, u_g, _ = _run_gpu(cfg, phi0, u0, 1000, storage=storage)
        ephi, eu = _errors(phi_g, u_g, phi_o, u_o, 1e-3)
        _log(f"drop2d {storage}: max|dphi|={ephi:.3e} rel_u={eu:.3e}")
        assert ephi <= 1e-3


def test_one_step_both_parities_against_oracle_at_every_node():
    """One even and one odd step from an exported state, every node."""
    lbm = _lbm()
    cfg, phi0, u0 = _jet_copy(nx=20, ny=18, nz=30, radius=5.0, seed=9)
    s = lbm.Sim(cfg, phi0, u0)
    s.step(6)
    for k in range(2):
        h, g, u = [t.cpu().numpy() for t in s.export_state()]
        _log(f"[gpu] one-step parity={s.steps_done % 2}")
        s.step(1)
        h1, g1, u1 = [t.cpu().numpy() for t in s.export_state()]
        nodes = np.arange(h.shape[1] * h.shape[2] * h.shape[3])
        ho, go, uo = oracle.step_nodes_f32(cfg, h, g, u, nodes)
        q = cfg["q"]
        eh = np.abs(h1.reshape(q, -1).T - ho).max()
        eg = np.abs(g1.reshape(q, -1).T - go).max()
        eu = np.abs(u1.reshape(3, -1).T - uo).max()
        _log(f"one step: max|dh|={eh:.3e} max|dg|={eg:.3e} max|du|={eu:.3e}")
        assert eh < 2e-7 and eg < 2e-7 and eu < 2e-7


def test_full_size_rt_sampled_one_step():
    """Rayleigh-Taylor at 256x1024x256 in the benchmark's launch shape: one
    even and one odd step checked at sampled nodes against the oracle's
    one-node evaluation from the exported full state."""
    lbm = _lbm()
    cfg, phi0, u0 = W.rt3d()
    s = lbm.Sim(cfg, phi0, u0)
    del phi0
    s.step(4)
    rng = np.random.default_rng(12205)
    N = 256 * 1024 * 256
    nodes = np.unique(np.concatenate([
        rng.integers(0, N, 400),
        # walls, periodic seams and the interface band
        [0, 255, 256 * 1023, N - 1, 256 * 1024 * 128 + 256 * 512 + 7,
         256 * 511 + 3, 256 * 512 + 255, 256 * 1024 * 255 + 256 * 513]]))
    for k in range(2):
        _log(f"[gpu] full-size RT sampled step, parity={s.steps_done % 2}")
        h, g, u = s.export_state()
        hc, gc, uc = h.cpu().numpy(), g.cpu().numpy(), u.cpu().numpy()
        del h, g, u
        s.step(1)
        h1, g1, u1 = s.export_state()
        import torch
        idx = torch.as_tensor(nodes, device=h1.device)
        h1s = h1.reshape(19, -1)[:, idx].T.cpu().numpy()
        g1s = g1.reshape(19, -1)[:, idx].T.cpu().numpy()
        u1s = u1.reshape(3, -1)[:, idx].T.cpu().numpy()
        del h1, g1, u1
        ho, go, uo = oracle.step_nodes_f32(cfg, hc, gc, uc, nodes)
        del hc, gc, uc
        eh, eg, eu = np.abs(h1s - ho).max(), np.abs(g1s - go).max(), np.abs(u1s - uo).max()
        _log(f"full RT sampled: max|dh|={eh:.3e} max|dg|={eg:.3e} max|du|={eu:.3e}")
        assert eh < 2e-7 and eg < 2e-7 and eu < 2e-7


def test_mass_conservation_fp32():
    lbm = _lbm()
    cfg, phi0, u0 = _rt_copy(64, 128, 32, seed=1)
    s = lbm.Sim(cfg, phi0, u0)
    m0, _ = s.reduce()
    s.step(1000)
    m1, k1 = s.reduce()
    _log(f"mass drift {abs(m1 - m0) / m0:.3e}")
    assert abs(m1 - m0) / m0 <= 1e-6 and np.isfinite(k1)


def test_reduce_matches_oracle():
    lbm = _lbm()
    cfg, phi0, u0 = W.drop2d()
    s = lbm.Sim(cfg, phi0, u0)
    s.step(100)
    o = oracle.Oracle(cfg).init(phi0, u0).step(100)
    mg, kg = s.reduce()
    mo, ko = o.reduce()
    assert abs(mg - mo) / mo < 1e-6
    assert abs(kg - ko) <= 1e-3 * ko + 1e-18


def test_deterministic_and_step_splitting():
    """Two runs are bitwise equal; 1+3+... single/graph splits equal one call."""
    lbm = _lbm()
    cfg, phi0, u0 = _jet_copy(seed=4)
    a = lbm.Sim(cfg, phi0, u0).step(57)
    b = lbm.Sim(cfg, phi0, u0)
    for n in (1, 3, 2, 40, 11):
        b.step(n)
    ha, ga, ua = a.export_state()
    hb, gb, ub = b.export_state()
    assert (ha == hb).all() and (ga == gb).all() and (ua == ub).all()


@pytest.mark.parametrize("storage", ["fp32", "fp16"])
def test_export_import_and_checkpoint_roundtrip(storage):
    lbm = _lbm()
    cfg, phi0, u0 = _jet_copy(seed=6)
    a = lbm.Sim(cfg, phi0, u0, storage=storage).step(31)
    blob = a.save()
    h, g, u = a.export_state()
    b = lbm.Sim(cfg, phi0, u0, storage=storage).import_state(h, g, u)
    h2, g2, u2 = b.export_state()
    if storage == "fp32":
        assert (h2 == h).all() and (g2 == g).all() and (u2 == u).all()
    else:
        assert (h2 - h).abs().max().item() < 1e-3
    a.step(20)
    c = lbm.Sim(cfg, phi0, u0, storage=storage).load(blob).step(20)
    ha, ga, _ = a.export_state()
    hc, gc, _ = c.export_state()
    assert (ha == hc).all() and (ga == gc).all()


def test_zero_steps_and_tiny_domain():
    lbm = _lbm()
    cfg, phi0, u0 = _rt_copy(2, 4, 2, seed=2)
    s = lbm.Sim(cfg, phi0, u0).step(0)
    h0, g0, _ = s.export_state()
    o = oracle.Oracle(cfg).init(phi0, u0)
    ho, go, _ = o.state()
    assert np.abs(h0.cpu().numpy() - ho).max() < 1e-6
    s.step(9)
    o.step(9)
    phi_g, u_g, _ = s.fields()
    phi_o, u_o, _ = o.fields()
    assert np.abs(phi_g.cpu().numpy() - phi_o).max() < 1e-5


@pytest.mark.parametrize("storage", ["fp32", "fp16"])
def test_rest_and_uniform_flow_are_fixed_points(storage):
    """Degenerate states: a single phase at rest stays exactly at rest, and
    a uniform flow through a periodic box keeps its velocity (both are fixed
    points of the step: no gradients, equilibrium populations)."""
    lbm = _lbm()
    cfg, _, _ = W.rt3d(nx=16, ny=20, nz=8, lref=256)
    cfg = dict(cfg, bc=("periodic",) * 6, gravity=(0.0, 0.0, 0.0))
    shape = (8, 20, 16)
    for phi_value in (1.0, 0.0):
        phi0 = np.full(shape, phi_value)
        s = lbm.Sim(cfg, phi0, None, storage=storage).step(50)
        phi, u, _ = s.fields()
        _log(f"[gpu] rest {storage} phi={phi_value}: max|u|={u.abs().max().item():.2e}")
        assert u.abs().max().item() == 0.0
        assert (phi - phi_value).abs().max().item() <= 1e-6
    u0 = np.zeros((3,) + shape)
    u0[0], u0[1], u0[2] = 0.01, -0.005, 0.002
    s = lbm.Sim(cfg, np.ones(shape), u0, storage=storage).step(50)
    phi, u, _ = s.fields()
    du = np.abs(u.cpu().numpy() - u0).max()
    _log(f"[gpu] uniform flow {storage}: max|u-u0|={du:.2e}")
    assert du <= (1e-6 if storage == "fp32" else 2e-5)


@pytest.mark.parametrize("mode", ["max", "average"])
def test_jet_copy_outlet_plane_options(mode):
    """Convective outflow with the plane options of appendix B (U_max and
    U_ave over the layer next to the outlet instead of each node's own
    outward velocity), 400 steps, FP32, against the oracle; the option must
    change the run (compared with the local option in the oracle)."""
    cfg, phi0, u0 = _jet_copy(seed=3)
    cfg = dict(cfg, outlet_mode=mode)
    _, phi_o, u_o, _ = _run_oracle(cfg, phi0, u0, 400)
    _, phi_l, u_l, _ = _oracle_cached("jet_local_400", dict(cfg, outlet_mode="local"), phi0, u0, 400)
    _, phi_g, u_g, _ = _run_gpu(cfg, phi0, u0, 400)
    ephi, eu = _errors(phi_g, u_g, phi_o, u_o)
    dlocal = np.abs(u_o - u_l).max() / np.abs(u_o).max()
    _log(f"jet copy outlet {mode}: max|dphi|={ephi:.3e} rel_u={eu:.3e} (option vs local: {dlocal:.2e})")
    assert dlocal > 1e-6
    assert ephi <= 1e-5 and eu <= 1e-4


def test_drop2d_fp32_2000_steps_and_laplace():
    """The 2D drop workload at its stated 2000 steps: FP32 parity with the
    oracle and the Laplace law on the GPU's own pressure field, dp = sigma / R
    within 5% (mean p inside r < R - 2 xi minus mean p outside r > R + 2 xi).

    Past 1000 steps the drop's centre is ill-conditioned: the heavy bulk sits
    1e-5 off phi = 1 with a vanishing gradient at the symmetry point, where
    the sharpening term's direction is undefined, and the FP64 oracle with
    its state rounded to FP32 after every step drifts by 1.7e-5 there by step
    2000.  The phase field is therefore held to 1e-5 inside the interface band
    (0.02 < phi < 0.98) and to four times that rounded oracle's drift in the
    bulk.  The velocities are spurious currents that decay (max |u| 9.8e-6 at
    1000 steps, 3.1e-6 at 2000) while FP32 rounding of the velocity sums stays
    about 5e-10: the velocity error is bounded by 1e-4 of the run's velocity
    scale, the spurious speed at 1000 steps, i.e. 1e-9."""
    cfg, phi0, u0 = W.drop2d()
    _, phi_o, u_o, _ = _oracle_cached("drop2000", cfg, phi0, u0, 2000)
    r = oracle.Oracle(cfg).init(phi0, u0)
    for _ in range(2000):
        r.step(1)
        h, g, u = r.state()
        r.set_state(*(a.astype(np.float32).astype(np.float64) for a in (h, g, u)))
    env = np.abs(r.fields()[0] - phi_o).max()
    _, phi_g, u_g, p_g = _run_gpu(cfg, phi0, u0, 2000)
    ephi, eu = _errors(phi_g, u_g, phi_o, u_o)
    band = (phi_o > 0.02) & (phi_o < 0.98)
    eband = np.abs(phi_g - phi_o)[band].max()
    du = np.abs(u_g - u_o).max()
    n, R = cfg["nx"], 25.0
    y, x = np.mgrid[0:n, 0:n]
    rr = np.hypot(x - n / 2, y - n / 2)
    dp = p_g[0][rr < R - 2 * cfg["xi"]].mean() - p_g[0][rr > R + 2 * cfg["xi"]].mean()
    lap = dp / (cfg["sigma"] / R) - 1.0
    _log(f"drop2d 2000 steps: max|dphi|={ephi:.3e} (band {eband:.3e}, FP32-rounded oracle {env:.3e}) "
         f"max|du|={du:.3e} (rel_u={eu:.3e}) Laplace dp R/sigma - 1 = {lap:+.4f}")
    assert eband <= 1e-5 and ephi <= max(1e-5, 4.0 * env)
    assert du <= 1e-4 * 9.8e-6
    assert abs(lap) < 0.05


@pytest.mark.timeout(900)
def test_jet_config3_parity_copy_64x64x256():
    """The precision-form jet's stated parity copy: 64 x 64 x 256 with the
    full jet's nozzle radius 12 and per-node parameters (u_j, sigma, tau, M,
    W, g), seeded perturbation, 1000 steps against the FP64 oracle, compared
    every 250 steps: FP32 within 1e-5 in phi and 1e-4 in velocity; FP16 and
    BF16 deviation storage within 1e-3 in phi (velocity and pressure errors
    logged, and where the largest phase-field error sits)."""
    lbm = _lbm()
    cfg, phi0, u0 = W.jet3d(nx=64, ny=64, nz=256, radius=12.0, stub=16.0)
    phi0, u0 = W.perturb(phi0, u0, 3, 0.01, 1e-3)
    _log("[oracle] jet 64x64x256, 1000 steps")
    o = oracle.Oracle(cfg).init(phi0, u0)
    sims = {st: lbm.Sim(cfg, phi0, u0, storage=st) for st in ("fp32", "fp16", "bf16")}
    tol = {"fp32": 1e-5, "fp16": 1e-3, "bf16": 1e-3}
    worst = {st: 0.0 for st in sims}
    for k in range(4):
        o.step(250)
        phi_o, u_o, p_o = o.fields()
        for st, s in sims.items():
            s.step(250)
            phi_g, u_g, p_g = [t.cpu().numpy().astype(np.float64) for t in s.fields()]
            ephi, eu = _errors(phi_g, u_g, phi_o, u_o)
            ep = np.abs(p_g - p_o).max() / np.abs(p_o).max()
            d = np.abs(phi_g - phi_o)
            at = np.unravel_index(d.argmax(), d.shape)
            _log(f"jet 64x64x256 {st} step {250 * (k + 1)}: max|dphi|={ephi:.3e} at (z,y,x)={tuple(map(int, at))} "
                 f"phi={phi_o[at]:.4f} rel_u={eu:.3e} rel_p={ep:.3e}")
            worst[st] = max(worst[st], ephi)
            if st == "fp32":
                assert eu <= 1e-4
    for st in sims:
        assert worst[st] <= tol[st], (st, worst[st])


@pytest.mark.parametrize("storage", ["fp32", "fp16", "bf16"])
@pytest.mark.parametrize("which", ["rt", "jet", "rt-bgk"])
def test_z_marching_kernel_equals_tiled_kernel(which, storage):
    """The D3Q19 interior kernel marching along z with the phase field staged
    in LDS gives bit for bit the state of the tiled kernel that reads the
    stencil from global memory, for several chunk lengths and tiles (ragged
    last chunk, partial tiles, wall lanes and inlet/outlet faces in the jet),
    with persistent launches and with one block per tile or task, for the
    WMRT and the BGK operator and every storage form."""
    lbm = _lbm()
    if which.startswith("rt"):
        cfg, phi0, u0 = _rt_copy(37, 29, 23, seed=5)
        if which == "rt-bgk":
            cfg = dict(cfg, collision="bgk")
    else:
        cfg, phi0, u0 = _jet_copy(nx=24, ny=20, nz=37, seed=3)
    ref = lbm.Sim(cfg, phi0, u0, storage=storage).set_zchunk(0).step(25)
    h0, g0, u_0 = [t.cpu().numpy() for t in ref.export_state()]
    for zc, tile, bpc in ((16, None, 4), (5, (32, 8), 4), (1, (64, 4), 0), (64, (16, 16), 2), (0, None, 0),
                          (7, (32, 4), 0)):
        _log(f"[gpu] z-marching {which} {storage} zc={zc} tile={tile} blocks/CU={bpc}")
        s = lbm.Sim(cfg, phi0, u0, storage=storage)
        if tile:
            s.set_tile(*tile)
        s.set_blocks_per_cu(bpc)
        s.set_zchunk(zc).step(25)
        h, g, u = [t.cpu().numpy() for t in s.export_state()]
        assert np.array_equal(h, h0) and np.array_equal(g, g0) and np.array_equal(u, u_0), (zc, tile, bpc)
