"""What the trained surrogate gains over the solver alone, on jets of held-out
Weber numbers (every fourth Weber number of the sweep, never seen in
training): from a solver state at t0, the network advances the coarse fields
by 8 lags of 32 steps and the solver advances the same domains; both are
timed and compared with the solver's coarse snapshots.

* accuracy: at every lag the network's error is below that of the forecast
  without a model (persistence: the state at t0);
* cost: one network advance of all the domains takes less time than the
  solver's 32 steps of the same domains;
* fallback: a prediction whose phase-field budget is violated beyond the
  threshold is handed to the solver; the solver's own snapshots are not.

Uses the committed weights (paper_2505_12205_amd/weights/jet_surrogate.npz,
written by paper_2505_12205_amd.train_surrogate)."""
import os
import sys
import time

import numpy as np
import pytest

from paper_2505_12205_amd import workloads as W

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.path.join(ROOT, "paper_2505_12205_amd", "weights", "jet_surrogate.npz")
LAG, WINDOW, K0, LAGS = 32, 192, 100, 8


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_surrogate_gain_on_heldout_weber():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("a GPU test ran without a GPU")
    from paper_2505_12205_amd import lbm, nn
    from paper_2505_12205_amd import surrogate as SG

    L = W.sweep_lengths()
    We = W.sweep_weber()
    held = [d for d in range(64) if d % 4 == 3]
    pick = sorted(held, key=lambda d: L[d])[:4]  # the four shortest held-out domains
    doms = W.jet_sweep(lengths=[L[d] for d in pick], webers=[We[d] for d in pick])
    cfgs = [c for c, _, _ in doms]
    _log(f"[gpu] held-out domains We={[round(float(We[d]), 3) for d in pick]} L={[int(L[d]) for d in pick]}")
    b = lbm.Batch(doms, storage="fp16")
    n = len(cfgs)
    shape = (5, WINDOW, cfgs[0]["ny"] // 2, cfgs[0]["nx"] // 2)
    net = SG.Network(n, *shape[1:], u_jet=cfgs[0]["inlet_u"])
    net.load(WEIGHTS)

    def snapshot(out):  # physical coarse fields of every domain
        for d, c in enumerate(cfgs):
            phi, u, p = b.fields(d)
            nn.coarsen(phi, u, p, c["nx"], c["ny"], c["nz"], 0, WINDOW, out=out[d])
        return out

    b.step(K0 * LAG)
    x0 = snapshot(torch.empty((n,) + shape, device="cuda"))
    # solver: LAGS advances, timed, with its coarse snapshots
    ref = []
    torch.cuda.synchronize()
    t_solver = 0.0
    for _ in range(LAGS):
        t0 = time.perf_counter()
        b.step(LAG)
        torch.cuda.synchronize()
        t_solver += time.perf_counter() - t0
        ref.append(snapshot(torch.empty((n,) + shape, device="cuda")))
    # network: LAGS advances from x0, timed
    x = x0.clone()
    preds = []
    net.predict(x)  # warm-up
    torch.cuda.synchronize()
    t_net = 0.0
    for _ in range(LAGS):
        t0 = time.perf_counter()
        x = net.predict(x)
        torch.cuda.synchronize()
        t_net += time.perf_counter() - t0
        preds.append(x.clone())
    sc = torch.tensor(SG.norm_scales(cfgs[0]["inlet_u"])[1], device="cuda").view(1, 5, 1, 1, 1)
    err_net, err_per = [], []
    for j in range(LAGS):
        err_net.append(float((((preds[j] - ref[j]) * sc) ** 2).mean()))
        err_per.append(float((((x0 - ref[j]) * sc) ** 2).mean()))
    _log("normalised MSE per lag, network:     " + " ".join(f"{e:.2e}" for e in err_net))
    _log("normalised MSE per lag, persistence: " + " ".join(f"{e:.2e}" for e in err_per))
    _log(f"time per advance of {n} domains: network {t_net / LAGS * 1e3:.2f} ms, "
         f"solver {t_solver / LAGS * 1e3:.2f} ms (x{t_solver / max(t_net, 1e-9):.1f})")
    assert all(a < p for a, p in zip(err_net, err_per))
    assert t_net < t_solver
    # fallback decisions: the budget compares a lag's change of the liquid
    # content with the previous lag's
    drift_solver = SG.mass_drift(x0, ref[0], ref[1])
    drift_net = SG.mass_drift(x0, ref[0], net.predict(ref[0]))
    bad = ref[1].clone()
    bad[:, 0] *= 1.01  # one per cent more liquid than the solver carries
    _log(f"budget violation: solver {np.round(drift_solver, 6)}, network {np.round(drift_net, 6)} "
         f"(fallback above {SG.FALLBACK_THRESHOLD})")
    assert SG.fallback_mask(x0, ref[0], bad).all()
    assert not SG.fallback_mask(x0, ref[0], ref[1]).any()


def test_hybrid_rollout_with_solver_fallback():
    """The network advances four held-out jets from their initial fields for
    64 lags; every prediction that violates the phase-field budget by more
    than the threshold is replaced by the solver's own advance of that domain
    (from its last synchronised state).  Reported: the fallback share, the
    wall time of the hybrid run against the solver alone, and the coarse
    fields' error against the solver at the last lag, with and without the
    fallback."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("a GPU test ran without a GPU")
    from paper_2505_12205_amd import hybrid as HY
    from paper_2505_12205_amd import lbm
    from paper_2505_12205_amd import surrogate as SG

    lags = 64
    L = W.sweep_lengths()
    We = W.sweep_weber()
    held = [d for d in range(64) if d % 4 == 3]
    pick = sorted(held, key=lambda d: L[d])[:4]
    doms = W.jet_sweep(lengths=[L[d] for d in pick], webers=[We[d] for d in pick])
    cfgs = [c for c, _, _ in doms]
    _log(f"[gpu] hybrid rollout We={[round(float(We[d]), 3) for d in pick]}")
    shape = (5, HY.WINDOW, cfgs[0]["ny"] // 2, cfgs[0]["nx"] // 2)
    net = SG.Network(len(doms), *shape[1:], u_jet=cfgs[0]["inlet_u"])
    net.load(WEIGHTS)
    hy = HY.HybridRollout(net, doms)
    plain = HY.HybridRollout(net, doms)
    t0 = time.perf_counter()
    for _ in range(lags):
        hy.advance()
    torch.cuda.synchronize()
    t_hybrid = time.perf_counter() - t0
    # the network alone (no fallback): the same rollout with the check switched off
    for _ in range(lags):
        plain.x_prev.copy_(plain.x)
        plain.x.copy_(net.predict(plain.x))
    # the solver alone over the same lags
    ref = lbm.Batch(doms, storage="fp16")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ref.step(lags * LAG)
    torch.cuda.synchronize()
    t_solver = time.perf_counter() - t0
    xr = torch.empty((len(doms),) + shape, device="cuda")
    for d, c in enumerate(cfgs):
        phi, u, p = ref.fields(d)
        HY.coarse_fields(phi, u, p, c, xr[d])
    sc = torch.tensor(SG.norm_scales(cfgs[0]["inlet_u"])[1], device="cuda").view(1, 5, 1, 1, 1)
    err_h = float((((hy.x - xr) * sc) ** 2).mean())
    err_p = float((((plain.x - xr) * sc) ** 2).mean())
    dphi_h = float((hy.x[:, 0] - xr[:, 0]).abs().max())
    share = len(hy.fallbacks) / (len(doms) * (lags - 1))
    _log(f"hybrid: {len(hy.fallbacks)} fallbacks of {len(doms) * (lags - 1)} predictions ({share:.1%}), "
         f"network {hy.t_net:.2f} s + solver catch-up {hy.t_solver:.2f} s = {t_hybrid:.2f} s; "
         f"solver alone {t_solver:.2f} s")
    _log(f"coarse-field MSE at lag {lags}: hybrid {err_h:.3e}, network alone {err_p:.3e}; "
         f"hybrid max|dphi| {dphi_h:.3f}")
    # every flagged prediction was replaced by the solver state of that lag
    for lag, d in hy.fallbacks:
        assert hy.sync[d] >= lag
    assert err_h <= err_p * 1.05 + 1e-12
    assert np.isfinite(err_h)


def test_guided_bracket_equals_bisection():
    """The critical Weber number on the sweep's 64-point Weber grid, regimes
    called from the intact length over lags 250..299 (steps 8,000-9,568, the
    window of the training data): solver-only bisection against the
    surrogate-guided search (network rollouts of all 64 domains from their
    initial fields propose the first jetting index, the solver confirms
    around it).  Both must end on the same adjacent pair; both wall times
    are reported."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("a GPU test ran without a GPU")
    from paper_2505_12205_amd import hybrid as HY
    from paper_2505_12205_amd import surrogate as SG

    window = (250, 299)
    doms = HY.weber_grid()
    We = W.sweep_weber()
    n = len(doms)
    cfg0 = doms[0][0]
    net = SG.Network(32, HY.WINDOW, cfg0["ny"] // 2, cfg0["nx"] // 2, u_jet=cfg0["inlet_u"])
    net.load(WEIGHTS)
    probes_s = []

    def probe(i):
        jet, med, dt = HY.solver_regime(*doms[i], window)
        probes_s.append(dt)
        _log(f"solver probe We={We[i]:.3f}: median L_b/D {med:.2f} -> {'jetting' if jet else 'dripping'} ({dt:.1f} s)")
        return jet

    t0 = time.perf_counter()
    first_b, calls_b = HY.bisect(probe, 0, n - 1)
    t_bisect = time.perf_counter() - t0
    t0 = time.perf_counter()
    jet_net, med_net, t_roll = HY.network_regimes(net, doms, window)
    proposal = int(np.argmax(jet_net)) if jet_net.any() else n - 1
    first_g, calls_g = HY.guided_bracket(probe, n, proposal)
    t_guided = time.perf_counter() - t0
    _log(f"bisection: first jetting We={We[first_b]:.3f} after {len(calls_b)} solver probes, {t_bisect:.1f} s")
    _log(f"guided: network proposes We={We[proposal]:.3f} ({t_roll:.1f} s of rollouts), first jetting "
         f"We={We[first_g]:.3f} after {len(calls_g)} solver probes, {t_guided:.1f} s")
    assert first_b is not None and first_g == first_b
