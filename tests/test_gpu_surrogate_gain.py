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
    """The network advances four held-out jets for 65 lags from the solver's
    state at lag 234 (the lead-in of the regime window); every prediction
    that violates the phase-field budget by more than the threshold is
    replaced by the solver's own advance of that domain (from its last
    synchronised state).  Run at the production threshold and at a tenth of
    it, so that the fallback path is exercised.  Reported: the fallback
    shares, wall times against the solver alone, and the coarse fields'
    error against the solver at the last lag, with and without fallback."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("a GPU test ran without a GPU")
    from paper_2505_12205_amd import hybrid as HY
    from paper_2505_12205_amd import lbm
    from paper_2505_12205_amd import surrogate as SG

    start, lags = HY.START, 65
    L = W.sweep_lengths()
    We = W.sweep_weber()
    held = [d for d in range(64) if d % 4 == 3]
    pick = sorted(held, key=lambda d: L[d])[:4]
    doms = W.jet_sweep(lengths=[L[d] for d in pick], webers=[We[d] for d in pick])
    cfgs = [c for c, _, _ in doms]
    _log(f"[gpu] hybrid rollout We={[round(float(We[d]), 3) for d in pick]} from lag {start}")
    shape = (5, HY.WINDOW, cfgs[0]["ny"] // 2, cfgs[0]["nx"] // 2)
    net = SG.Network(len(doms), *shape[1:], u_jet=cfgs[0]["inlet_u"])
    net.load(WEIGHTS)
    runs = {}
    for name, thr in (("production", SG.FALLBACK_THRESHOLD), ("tight", 0.1 * SG.FALLBACK_THRESHOLD)):
        hy = HY.HybridRollout(net, doms, start=start, threshold=thr)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(lags):
            hy.advance()
        torch.cuda.synchronize()
        runs[name] = (hy, time.perf_counter() - t0)
    # the network alone (no fallback) from the same start
    x = runs["production"][0].solver_start.clone()
    for _ in range(lags):
        x = net.predict(x)
    # the solver alone
    ref = lbm.Batch(doms, storage="fp16")
    ref.step(start * LAG)
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

    def mse(a):
        return float((((a - xr) * sc) ** 2).mean())

    err_p = mse(x)
    _log(f"solver alone over the {lags} lags: {t_solver:.2f} s; network alone: MSE {err_p:.3e}, "
         f"max|dphi| {float((x[:, 0] - xr[:, 0]).abs().max()):.3f}")
    total = len(doms) * (lags - 1)
    for name, (hy, t_h) in runs.items():
        _log(f"hybrid ({name}, threshold {hy.threshold:.0e}): {len(hy.fallbacks)} fallbacks of {total} "
             f"predictions, network {hy.t_net:.2f} s + solver catch-up {hy.t_solver:.2f} s = {t_h:.2f} s; "
             f"MSE {mse(hy.x):.3e}, max|dphi| {float((hy.x[:, 0] - xr[:, 0]).abs().max()):.3f}")
        # every flagged prediction was replaced by the solver state of that lag
        for lag, d in hy.fallbacks:
            assert hy.sync[d] >= lag
        assert np.isfinite(mse(hy.x))
        # a fallback can only bring a domain back onto the solver's trajectory
        assert mse(hy.x) <= err_p * 1.05 + 1e-12
    assert len(runs["tight"][0].fallbacks) > 0
    if not runs["production"][0].fallbacks:
        assert runs["production"][1] < t_solver


def test_accelerated_bisection_equals_solver_bisection():
    """The critical Weber number on the sweep's 64-point Weber grid, regimes
    called from the intact length over lags 250..299 (steps 8,000-9,568, the
    window of the training data).  Solver-only bisection, each probe a solver
    run through the window, against the surrogate-accelerated search
    (hybrid.AcceleratedSearch: the solver to lag 234, the network through
    the window, the final pair confirmed by the solver from the kept
    states).  Both must end on the same adjacent pair; the solver steps and
    the wall times of both are reported, and the accelerated search must
    take fewer solver steps."""
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
    calls = []

    def probe(i):
        jet, med, dt = HY.solver_regime(*doms[i], window)
        calls.append(i)
        _log(f"solver probe We={We[i]:.3f}: median L_b/D {med:.2f} -> {'jetting' if jet else 'dripping'} ({dt:.1f} s)")
        return jet

    t0 = time.perf_counter()
    first_b, _ = HY.bisect(probe, 0, n - 1)
    t_bisect = time.perf_counter() - t0
    steps_b = len(calls) * window[1] * LAG
    net = SG.Network(1, HY.WINDOW, cfg0["ny"] // 2, cfg0["nx"] // 2, u_jet=cfg0["inlet_u"])
    net.load(WEIGHTS)
    t0 = time.perf_counter()
    acc = HY.AcceleratedSearch(net, doms, window, HY.START)
    first_a = acc.run()
    torch.cuda.synchronize()
    t_acc = time.perf_counter() - t0
    _log(f"solver bisection: first jetting We={We[first_b]:.3f} after {len(calls)} probes, "
         f"{steps_b} solver steps, {t_bisect:.1f} s")
    _log(f"accelerated: first jetting We={We[first_a]:.3f} after {len(acc.probes)} probes "
         f"(network calls {[(We[i].round(3), acc.netcall[i]) for i in acc.probes]}) and "
         f"{len(acc.confirmations)} confirmations, {acc.solver_steps} solver steps, {t_acc:.1f} s")
    assert first_b is not None and first_a == first_b
    assert acc.solver_steps < steps_b
