"""Train and evaluate the jet surrogate on snapshots of the batched solver.

    python -m paper_2505_12205_amd.train_surrogate --out DIR [--snapshots N] [--epochs E]

1. The batched Weber sweep (64 jet domains 96 x 96 x L_k, FP16 storage)
   runs for N x 32 steps; every 32 steps each domain's fields are averaged
   over 2 x 2 x 2 blocks into a 192-plane window from the inlet (zero beyond
   the outlet), normalised and stored in FP32 on the device (one lag's
   increments are of the order of a bf16 rounding of the fields, so the
   store keeps full precision).
2. Pairs (snapshot k, snapshot k + 1) of every domain with k_index % 4 != 3
   train the network (batch 32, Adam); the other quarter of the Weber
   numbers is held out.
3. Held-out evaluation: error of the prediction against the solver's next
   snapshot, next to the persistence forecast (the input itself); the
   phase-field budget violation of each prediction and the share above the
   fallback threshold (those samples are advanced by the solver instead);
   rollouts of several lags from one snapshot; throughput of the network
   against the solver for the same advance.
4. Regimes: each domain's median intact length over the last 50 snapshots,
   from the solver and from a 50-lag network rollout, classifies it as
   dripping or jetting (more than two nozzle diameters); each proposes the
   critical Weber number of the transition.
Writes DIR/jet_surrogate.npz (weights) and DIR/report.json; progress goes to
stdout.  Every arithmetic step runs in the library kernels (liblbm.so and
libsurr.so); torch holds the buffers and computes the report's summary
statistics.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

from . import lbm, nn
from . import surrogate as SG
from . import workloads as W

LAG = 32          # solver steps per surrogate step
WINDOW = 192      # coarse planes of the window (384 fine planes from the inlet)
FALLBACK = SG.FALLBACK_THRESHOLD  # budget violation above which the solver takes over


def log(msg):
    print(f"[surrogate {time.strftime('%H:%M:%S')}] {msg}", flush=True)


class Recorder:
    """Coarse normalised snapshots of every domain of a batch, float rows
    [5, WINDOW, ny/2, nx/2] in a device store."""

    def __init__(self, batch: lbm.Batch, cfgs, snapshots: int, shift, scale):
        self.b, self.cfgs = batch, cfgs
        self.nd = len(cfgs)
        nx, ny = cfgs[0]["nx"], cfgs[0]["ny"]
        self.shape = (5, WINDOW, ny // 2, nx // 2)
        self.rows = self.nd * snapshots
        self.store = torch.empty((self.rows,) + self.shape, dtype=torch.float32, device="cuda")
        self.buf = torch.empty((1,) + self.shape, dtype=torch.float32, device="cuda")
        self.shift, self.scale = shift, scale
        self.k = 0
        self.snapshots = snapshots
        self.valid = np.ones((snapshots, self.nd), dtype=bool)  # finite snapshot of domain d at k
        self.sums = torch.empty((1, 3), dtype=torch.float64, device="cuda")

    def row(self, d, k):
        return k * self.nd + d

    def record(self):
        for d, c in enumerate(self.cfgs):
            phi, u, p = self.b.fields(d)
            nn.coarsen(phi, u, p, c["nx"], c["ny"], c["nz"], 0, WINDOW, out=self.buf[0])
            nn.phi_budget(self.buf, out=self.sums)
            ok = bool(np.isfinite(self.sums.cpu().numpy()).all())
            # a domain that has left the scheme's stability range stays out
            self.valid[self.k, d] = ok and (self.k == 0 or self.valid[self.k - 1, d])
            r = self.row(d, self.k)
            nn.normalize(self.buf, self.shift, self.scale, out=self.store[r:r + 1])
        self.k += 1


def generate(snapshots: int, seed: int = 12205, autotune: bool = True):
    cfgs_full = W.jet_sweep(seed=seed)
    cfgs = [c for c, _, _ in cfgs_full]
    b = lbm.Batch(cfgs_full, storage="fp16")
    del cfgs_full
    if autotune:
        b.autotune(trial_steps=4)
    shift, scale = SG.norm_scales(cfgs[0]["inlet_u"])
    rec = Recorder(b, cfgs, snapshots, torch.tensor(shift, device="cuda"), torch.tensor(scale, device="cuda"))
    t0 = time.perf_counter()
    rec.record()
    for k in range(1, snapshots):
        b.step(LAG)
        rec.record()
        if k % 25 == 0 or k == snapshots - 1:
            torch.cuda.synchronize()
            log(f"snapshot {k + 1}/{snapshots} (solver step {b.steps_done}, {time.perf_counter() - t0:.0f} s)")
    torch.cuda.synchronize()
    return b, cfgs, rec, time.perf_counter() - t0


def split(nd: int, snapshots: int, rec: Recorder):
    """Training / held-out domains (every fourth Weber number held out) and
    their consecutive-snapshot pairs, finite snapshots only."""
    held = [d for d in range(nd) if d % 4 == 3]
    train = [d for d in range(nd) if d % 4 != 3]

    def pairs(ds):
        return np.array([(rec.row(d, k), rec.row(d, k + 1)) for d in ds for k in range(snapshots - 1)
                         if rec.valid[k + 1, d]], dtype=np.int64).reshape(-1, 2)

    return train, held, pairs(train), pairs(held)


def train(net: SG.Network, rec: Recorder, pairs: np.ndarray, epochs: int, bs: int, seed: int = 0,
          budget_s: float = 1e9):
    rng = np.random.default_rng(seed)
    xb = torch.empty((bs,) + rec.shape, dtype=torch.float32, device="cuda")
    tb = torch.empty_like(xb)
    hist = []
    t0 = time.perf_counter()
    steps = 0
    for ep in range(epochs):
        perm = rng.permutation(len(pairs))
        acc, n = 0.0, 0
        for i in range(0, len(perm) - bs + 1, bs):
            sel = pairs[perm[i:i + bs]]
            idx = torch.from_numpy(sel.T.copy()).cuda()
            nn.gather(rec.store, idx[0], xb)
            nn.gather(rec.store, idx[1], tb)
            L = net.train_step(xb, tb)
            steps += 1
            if steps % 50 == 0:
                v = float(L.item())
                acc += v
                n += 1
                if steps % 200 == 0:
                    log(f"epoch {ep} step {steps} loss {v:.5f} ({time.perf_counter() - t0:.0f} s)")
            if time.perf_counter() - t0 > budget_s:
                break
        hist.append(acc / max(n, 1))
        log(f"epoch {ep} mean sampled loss {hist[-1]:.5f}")
        if time.perf_counter() - t0 > budget_s:
            log("training time budget reached")
            break
    torch.cuda.synchronize()
    return hist, steps, time.perf_counter() - t0


def evaluate(net: SG.Network, rec: Recorder, pairs: np.ndarray, bs: int):
    """Normalised MSE of the network and of persistence, phi errors, budget
    violations (network and solver) and the fallback share on held-out
    pairs whose previous snapshot exists (the budget compares with it)."""
    xb = torch.empty((bs,) + rec.shape, dtype=torch.float32, device="cuda")
    tb = torch.empty_like(xb)
    pb = torch.empty_like(xb)
    zero = torch.zeros((bs,) + rec.shape[1:] + (16,), dtype=torch.bfloat16, device="cuda")
    dr = torch.empty_like(zero)
    ws = torch.empty(2048, dtype=torch.float64, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    pairs = pairs[pairs[:, 0] >= rec.nd]  # k >= 1
    mse_net, mse_per, phi_net, phi_per, drift_net, drift_lbm = [], [], [], [], [], []
    for i in range(0, len(pairs) - bs + 1, bs):
        sel = pairs[i:i + bs]
        idx = torch.from_numpy(np.stack([sel[:, 0] - rec.nd, sel[:, 0], sel[:, 1]])).cuda()
        nn.gather(rec.store, idx[0], pb)
        nn.gather(rec.store, idx[1], xb)
        nn.gather(rec.store, idx[2], tb)
        r = net.forward(xb)
        nn.residual_loss(xb, tb, r, dr, loss, ws, rs=net.rs)
        mse_net.append(float(loss.item()))
        nn.residual_loss(xb, tb, zero, dr, loss, ws)
        mse_per.append(float(loss.item()))
        p_phys = nn.unpack(pb, zero, net.shift, net.scale)
        x_phys = nn.unpack(xb, zero, net.shift, net.scale)
        t_phys = nn.unpack(tb, zero, net.shift, net.scale)
        pred = nn.unpack(xb, r, net.shift, net.scale, rs=net.rs)
        phi_net.append(float((pred[:, 0] - t_phys[:, 0]).abs().max().item()))
        phi_per.append(float((x_phys[:, 0] - t_phys[:, 0]).abs().max().item()))
        drift_net.extend(SG.mass_drift(p_phys, x_phys, pred).tolist())
        drift_lbm.extend(SG.mass_drift(p_phys, x_phys, t_phys).tolist())
    drift_net = np.array(drift_net)
    drift_lbm = np.array(drift_lbm)
    return {
        "pairs": int(len(mse_net) * bs),
        "mse_network": float(np.mean(mse_net)), "mse_persistence": float(np.mean(mse_per)),
        "max_abs_phi_error_network": float(np.max(phi_net)),
        "max_abs_phi_error_persistence": float(np.max(phi_per)),
        "budget_violation_network_median": float(np.median(drift_net)),
        "budget_violation_solver_median": float(np.median(drift_lbm)),
        "budget_violation_solver_p99": float(np.percentile(drift_lbm, 99)),
        "fallback_share": float(np.mean(drift_net > FALLBACK)),
        "fallback_share_solver_itself": float(np.mean(drift_lbm > FALLBACK)),
    }


def rollout(net1: SG.Network, rec: Recorder, held, k0: int, lags: int):
    """Advance held-out domains `lags` surrogate steps from snapshot k0 and
    compare with the solver's snapshots: normalised MSE per lag (network and
    persistence)."""
    x = torch.empty((1,) + rec.shape, dtype=torch.float32, device="cuda")
    t = torch.empty_like(x)
    zero = torch.zeros((1,) + rec.shape[1:] + (16,), dtype=torch.bfloat16, device="cuda")
    dr = torch.empty_like(zero)
    ws = torch.empty(2048, dtype=torch.float64, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    out = {"net": np.zeros(lags), "persistence": np.zeros(lags)}
    for d in held:
        nn.gather(rec.store, torch.tensor([rec.row(d, k0)], device="cuda"), x)
        x0 = x.clone()
        for j in range(lags):
            nn.gather(rec.store, torch.tensor([rec.row(d, k0 + j + 1)], device="cuda"), t)
            r = net1.forward(x)
            nn.residual_loss(x, t, r, dr, loss, ws, rs=net1.rs)
            out["net"][j] += float(loss.item()) / len(held)
            nn.residual_loss(x0, t, zero, dr, loss, ws)
            out["persistence"][j] += float(loss.item()) / len(held)
            nxt = nn.unpack(x, r, torch.zeros_like(net1.shift), torch.ones_like(net1.scale), rs=net1.rs)  # normalised
            x.copy_(nxt)
    return {k: v.tolist() for k, v in out.items()}


def intact_length(phi: np.ndarray) -> np.ndarray:
    """Intact length in fine lattice units of coarse phase fields [n, d, h, w]:
    the planes from the inlet that hold liquid (phi > 1/2) without a gap,
    times 2 (a coarse plane spans two fine planes)."""
    has = (phi > 0.5).reshape(phi.shape[0], phi.shape[1], -1).any(axis=2)
    run = np.where(has.all(axis=1), phi.shape[1], np.argmin(has, axis=1))
    return 2 * run


def critical_weber(we: np.ndarray, jetting: np.ndarray) -> float:
    """The Weber number that best splits dripping (below) from jetting
    (above): the split with the fewest misclassified domains, placed at the
    geometric mean of its two neighbours."""
    o = np.argsort(we)
    w, j = we[o], jetting[o].astype(int)
    best, cut = None, 0
    for i in range(len(w) + 1):
        err = j[:i].sum() + (1 - j[i:]).sum()
        if best is None or err < best:
            best, cut = err, i
    if cut == 0:
        return float(w[0])
    if cut == len(w):
        return float(w[-1])
    return float(np.sqrt(w[cut - 1] * w[cut]))


def regime_study(net: SG.Network, rec: Recorder, cfgs, k_from: int, k_to: int, held):
    """Dripping / jetting per domain (median intact length over snapshots
    k_from..k_to above 2 nozzle diameters = jetting) from the solver's
    snapshots and from network rollouts started at snapshot k_from - 1, and
    the critical Weber number each proposes."""
    We = np.array(W.sweep_weber(len(cfgs)))
    D = 2.0 * cfgs[0]["inlet_radius"]
    ok = np.array([rec.valid[k_to, d] for d in range(rec.nd)])
    ks = list(range(k_from, k_to + 1))
    lb_lbm = np.zeros((rec.nd, len(ks)))
    lb_net = np.zeros((rec.nd, len(ks)))
    bs = net.batch
    x = torch.empty((bs,) + rec.shape, dtype=torch.float32, device="cuda")
    one = torch.ones(5, device="cuda")
    zero5 = torch.zeros(5, device="cuda")
    for d0 in range(0, rec.nd, bs):
        doms = list(range(d0, min(d0 + bs, rec.nd)))
        pad = doms + [doms[-1]] * (bs - len(doms))
        nn.gather(rec.store, torch.tensor([rec.row(d, k_from - 1) for d in pad], device="cuda"), x)
        for j, k in enumerate(ks):
            r = net.forward(x)
            x = nn.unpack(x, r, zero5, one, rs=net.rs)  # next normalised state
            phi_net = x[:len(doms), 0].cpu().numpy()  # phi is normalised by 1
            lb_net[doms, j] = intact_length(phi_net)
            phi_lbm = rec.store[[rec.row(d, k) for d in doms], 0].cpu().numpy()
            lb_lbm[doms, j] = intact_length(phi_lbm)
    med_lbm = np.median(lb_lbm, axis=1)
    med_net = np.median(lb_net, axis=1)
    jet_lbm = med_lbm / D > 2.0
    jet_net = med_net / D > 2.0
    hmask = np.zeros(rec.nd, bool)
    hmask[held] = True
    return {
        "snapshots": [k_from, k_to], "solver_step_range": [k_from * LAG, k_to * LAG],
        "criterion": "median intact length over the snapshots > 2 nozzle diameters",
        "weber": We.tolist(), "finite": ok.tolist(),
        "intact_length_solver": med_lbm.tolist(), "intact_length_network_rollout": med_net.tolist(),
        "jetting_solver": jet_lbm.tolist(), "jetting_network_rollout": jet_net.tolist(),
        "regime_agreement": float(np.mean(jet_lbm[ok] == jet_net[ok])),
        "regime_agreement_heldout": float(np.mean(jet_lbm[ok & hmask] == jet_net[ok & hmask])),
        "we_critical_solver": critical_weber(We[ok], jet_lbm[ok]),
        "we_critical_network": critical_weber(We[ok], jet_net[ok]),
    }


def throughput(net: SG.Network, rec: Recorder, b: lbm.Batch, held, reps: int = 5):
    """Seconds per 32-step advance of the held-out domains: the network on
    the coarse windows (batch = number of held-out domains) and the solver
    (the batch's time scaled by the held-out share of its nodes)."""
    xb = torch.empty((net.batch,) + rec.shape, dtype=torch.float32, device="cuda")
    idx = torch.tensor([rec.row(d, 0) for d in held][:net.batch], device="cuda")
    nn.gather(rec.store, idx, xb[:len(idx)])
    net.forward(xb)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        net.forward(xb)
    torch.cuda.synchronize()
    t_net = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    b.step(LAG)
    torch.cuda.synchronize()
    t_lbm_all = time.perf_counter() - t0
    nodes = [int(np.prod(s)) for s in b.shapes]
    share = sum(nodes[d] for d in held) / sum(nodes)
    return {"network_s_per_advance": t_net, "network_batch": net.batch, "solver_s_per_advance_all": t_lbm_all,
            "solver_s_per_advance_heldout_share": t_lbm_all * share}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--snapshots", type=int, default=300, help="snapshots per domain (every 32 steps)")
    ap.add_argument("--epochs", type=int, default=6)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--train-seconds", type=float, default=360.0)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--weights", default="", help="start from these weights (npz)")
    ap.add_argument("--mass-weight", type=float, default=SG.MASS_WEIGHT,
                    help="weight of the phase-field content term of the loss")
    args = ap.parse_args(argv)
    os.makedirs(args.out, exist_ok=True)
    log(f"generating {args.snapshots} snapshots x 64 domains")
    b, cfgs, rec, t_gen = generate(args.snapshots)
    train_d, held_d, tr_pairs, ho_pairs = split(len(cfgs), args.snapshots, rec)
    log(f"data: {rec.rows} snapshots in {t_gen:.0f} s; {len(tr_pairs)} training pairs, {len(ho_pairs)} held out")
    net = SG.Network(args.batch, *rec.shape[1:], seed=args.seed, lr=args.lr, u_jet=cfgs[0]["inlet_u"],
                     mass_weight=args.mass_weight)
    if args.weights:
        net.load(args.weights)
    hist, steps, t_train = train(net, rec, tr_pairs, args.epochs, args.batch, args.seed, args.train_seconds)
    net.save(os.path.join(args.out, "jet_surrogate.npz"))
    log(f"trained {steps} steps in {t_train:.0f} s")
    ev = evaluate(net, rec, ho_pairs, args.batch)
    log(f"held-out: {ev}")
    net1 = SG.Network(1, *rec.shape[1:], u_jet=cfgs[0]["inlet_u"])
    net1.set_params(net.get_params())
    k0 = args.snapshots // 2
    lags = min(8, args.snapshots - k0 - 1)
    ro = rollout(net1, rec, [d for d in held_d if rec.valid[k0 + lags, d]], k0, lags)
    log(f"rollout: {ro}")
    tp = throughput(SG.Network(len(held_d), *rec.shape[1:], u_jet=cfgs[0]["inlet_u"]), rec, b, held_d)
    log(f"throughput: {tp}")
    k_to = args.snapshots - 1
    k_from = max(1, k_to - 49)
    rg = regime_study(net, rec, cfgs, k_from, k_to, held_d)
    log(f"regimes: We_cr solver {rg['we_critical_solver']:.3f}, network {rg['we_critical_network']:.3f}; "
        f"agreement {rg['regime_agreement']:.3f} (held out {rg['regime_agreement_heldout']:.3f})")
    We = W.sweep_weber()
    report = {
        "domains": len(cfgs), "snapshots_per_domain": args.snapshots, "lag_steps": LAG,
        "window": list(rec.shape), "data_seconds": t_gen, "train_pairs": int(len(tr_pairs)),
        "heldout_pairs": int(len(ho_pairs)), "heldout_weber": [float(We[d]) for d in held_d],
        "batch": args.batch, "lr": args.lr, "train_steps": steps, "train_seconds": t_train,
        "epoch_loss": hist, "heldout": ev, "rollout_mse": ro, "throughput": tp, "regimes": rg,
        "params": int(sum(v.size for v in net.get_params().values())),
        "domains_finite_at_end": int(rec.valid[-1].sum()),
        "mobility": cfgs[0]["mobility"], "mass_weight": args.mass_weight,
        "fallback_threshold": FALLBACK,
    }
    with open(os.path.join(args.out, "report.json"), "w") as f:
        json.dump(report, f, indent=1)
    log("done")
    return 0


if __name__ == "__main__":
    sys.exit(main())
