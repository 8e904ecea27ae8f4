"""GPU tests of the batched form: every domain of a batch equals the same
domain run on its own (bitwise: the per-node arithmetic is the same), the
small domains match the FP64 oracle, and the diagnostics are consistent."""
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


def _small_sweep(seed=0):
    doms = []
    for k, (nz, we) in enumerate([(40, 1.0), (52, 3.0), (44, 6.0)]):
        cfg, phi0, u0 = W.jet3d(nx=24, ny=24, nz=nz, radius=6.0, param_radius=12.0, stub=10.0,
                                weber=we)
        phi0, u0 = W.perturb(phi0, u0, seed + k, 0.01, 1e-3)
        doms.append((cfg, phi0, u0))
    return doms


@pytest.mark.parametrize("storage", ["fp32", "fp16"])
def test_batch_equals_standalone_bitwise(storage):
    lbm = _lbm()
    doms = _small_sweep()
    _log(f"[gpu] batch of {len(doms)} storage={storage}")
    b = lbm.Batch(doms, storage=storage).step(37)
    for d, (cfg, phi0, u0) in enumerate(doms):
        s = lbm.Sim(cfg, phi0, u0, storage=storage).step(37)
        hb, gb, ub = b.export_state(d)
        hs, gs, us = s.export_state()
        assert (hb == hs).all() and (gb == gs).all() and (ub == us).all(), d


def test_bgk_batch_equals_standalone_bitwise():
    """The operator flag reaches the batched launches: a batch of BGK domains
    (x-wall lanes, faces, inlet and outlet) equals each domain run alone with
    BGK, and differs from WMRT."""
    lbm = _lbm()
    doms = [(dict(c, collision="bgk"), p, u) for c, p, u in _small_sweep(seed=3)[:2]]
    _log(f"[gpu] BGK batch of {len(doms)}")
    b = lbm.Batch(doms, storage="fp32").step(41)
    for d, (cfg, phi0, u0) in enumerate(doms):
        s = lbm.Sim(cfg, phi0, u0).step(41)
        hb, gb, ub = b.export_state(d)
        hs, gs, us = s.export_state()
        assert (hb == hs).all() and (gb == gs).all() and (ub == us).all(), d
    cfg, phi0, u0 = doms[0]
    w = lbm.Sim(dict(cfg, collision="wmrt"), phi0, u0).step(41)
    assert not (w.export_state()[1] == b.export_state(0)[1]).all()


def test_diverged_domain_is_isolated_and_reported():
    """A non-finite value in one domain stays in that domain: the other
    domain still equals its standalone run bit for bit; reduce() raises
    LBM_EUNSTABLE and reduce(strict=False) returns the per-domain values."""
    lbm = _lbm()
    doms = _small_sweep(seed=5)[:2]
    cfg1, phi1, u1 = doms[1]
    phi1 = phi1.copy()
    phi1[phi1.shape[0] // 2, phi1.shape[1] // 2, phi1.shape[2] // 2] = np.nan
    doms[1] = (cfg1, phi1, u1)
    _log("[gpu] batch with a non-finite domain")
    b = lbm.Batch(doms, storage="fp32").step(12)
    with pytest.raises(lbm.LbmError) as ei:
        b.reduce()
    assert ei.value.code == lbm.LBM_EUNSTABLE
    mass, ke = b.reduce(strict=False)
    assert np.isfinite(mass[0]) and np.isfinite(ke[0]) and not np.isfinite(mass[1])
    cfg0, phi0, u0 = doms[0]
    s = lbm.Sim(cfg0, phi0, u0).step(12)
    hb, gb, ub = b.export_state(0)
    hs, gs, us = s.export_state()
    assert (hb == hs).all() and (gb == gs).all() and (ub == us).all()


def test_batch_domain_matches_oracle():
    lbm = _lbm()
    doms = _small_sweep(seed=7)
    b = lbm.Batch(doms).step(300)
    for d in (0, 2):
        cfg, phi0, u0 = doms[d]
        o = oracle.Oracle(cfg).init(phi0, u0).step(300)
        phi_o, u_o, _ = o.fields()
        phi_g, u_g, _ = b.fields(d)
        ephi = np.abs(phi_g.cpu().numpy() - phi_o).max()
        eu = np.abs(u_g.cpu().numpy() - u_o).max() / max(np.abs(u_o).max(), 1e-30)
        _log(f"batch domain {d}: max|dphi|={ephi:.3e} rel_u={eu:.3e}")
        assert ephi <= 1e-5 and eu <= 1e-4


def test_batch_launch_shapes_agree():
    """Any launch shape gives the same result (bitwise)."""
    lbm = _lbm()
    doms = _small_sweep(seed=3)
    ref = lbm.Batch(doms).step(12)
    for launch in ((16, 16, 2, True), (64, 4, 0, False)):
        alt = lbm.Batch(doms).set_launch(*launch).step(12)
        for d in range(len(doms)):
            for a, r in zip(alt.export_state(d), ref.export_state(d)):
                assert (a == r).all(), launch


def test_batch_fp16_sweep_domain_matches_oracle():
    """The Weber sweep's real configuration (96 x 96 x L_k, FP16 deviation
    storage, the sweep's mobility and walls): the two shortest domains run
    batched for 200 steps, and the shorter one is compared with the FP64
    oracle at every node (phase field within 1e-3)."""
    lbm = _lbm()
    L = W.sweep_lengths()
    We = W.sweep_weber()
    idx = [int(k) for k in np.argsort(L)[:2]]
    doms = W.jet_sweep(lengths=[L[k] for k in idx], webers=[We[k] for k in idx])
    _log(f"[gpu] fp16 sweep domains vs oracle {[(int(L[k]), round(float(We[k]), 3)) for k in idx]}")
    b = lbm.Batch(doms, storage="fp16").step(200)
    cfg, phi0, u0 = doms[0]
    o = oracle.Oracle(cfg).init(phi0, u0).step(200)
    phi_o, u_o, _ = o.fields()
    phi_g, u_g, _ = b.fields(0)
    ephi = np.abs(phi_g.cpu().numpy() - phi_o).max()
    eu = np.abs(u_g.cpu().numpy() - u_o).max() / max(np.abs(u_o).max(), 1e-30)
    _log(f"fp16 sweep domain 0 ({cfg['nx']}x{cfg['ny']}x{cfg['nz']}): max|dphi|={ephi:.3e} rel_u={eu:.3e}")
    assert np.isfinite(eu) and ephi <= 1e-3


def test_batch_full_size_sweep_domains_equal_standalone():
    """The two shortest domains of the Weber sweep (96 x 96 x L, FP16 storage)
    batched and standalone, 20 steps, bitwise."""
    lbm = _lbm()
    L = W.sweep_lengths()
    We = W.sweep_weber()
    idx = np.argsort(L)[:2]
    doms = [W.jet3d(nx=96, ny=96, nz=int(L[k]), radius=8.0, reynolds=200.0, weber=float(We[k]))
            for k in idx]
    _log(f"[gpu] sweep domains {[(int(L[k]), round(float(We[k]), 3)) for k in idx]}")
    b = lbm.Batch(doms, storage="fp16")
    b.autotune(2)
    b.step(20)
    m, ke = b.reduce()
    assert all(np.isfinite(m)) and all(np.isfinite(ke))
    for d, (cfg, phi0, u0) in enumerate(doms):
        s = lbm.Sim(cfg, phi0, u0, storage="fp16").step(b.steps_done)
        hb = b.export_state(d)[0]
        hs = s.export_state()[0]
        assert (hb == hs).all(), d


def test_intact_length_of_initial_stub():
    lbm = _lbm()
    doms = [W.jet3d(nx=32, ny=32, nz=64, radius=8.0, stub=float(s)) for s in (16, 24)]
    b = lbm.Batch(doms)
    assert b.intact_length(0.5) == [16, 24]
