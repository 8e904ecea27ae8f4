"""Surrogate and solver together on the Weber sweep's jets.

HybridRollout advances jet domains lag by lag (one lag = 32 solver steps)
with the network on their coarse fields.  A prediction whose phase-field
budget is violated beyond the threshold (surrogate.fallback_mask) is not
accepted: the solver, which holds each domain's full-resolution state at the
last lag it was synchronised, advances that domain (lbm_batch_step) to the
current lag, and its coarsened fields replace the prediction.  The solver
cannot restart from a coarse state, so a fallback costs the solver steps
since the domain's last synchronisation.

The critical Weber number of the dripping-to-jetting transition is
bracketed on the sweep's Weber grid by calling each domain's regime from its
intact length over a window of lags (median above two nozzle diameters:
jetting), two ways:
  - solver only: bisection, each probe one solver run of one domain through
    the window;
  - surrogate-accelerated (AcceleratedSearch): each probe runs the solver to
    a lag before the window and the network through it; the adjacent pair
    the search ends on is confirmed by the solver from the kept states, and
    the search repeats with any regime the confirmation corrects.
Both searches end on the same adjacent pair of Weber numbers whenever the
solver's regime is monotone in We, since the regimes of the final pair are
solver calls.  (Network rollouts from the initial fields call every domain
of the sweep jetting: the error of 250 chained predictions is too large for
the intact length.)
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import lbm, nn
from . import surrogate as SG
from . import workloads as W

LAG = 32
WINDOW = 192
# lag at which the accelerated search hands a probe from the solver to the
# network: 16 lags before the regime window of lags 250..299
START = 234


def coarse_fields(phi, u, p, cfg, out):
    """Full-resolution fields of one domain -> coarse physical window [5, 192, ny/2, nx/2]."""
    return nn.coarsen(phi, u, p, cfg["nx"], cfg["ny"], cfg["nz"], 0, WINDOW, out=out)


def initial_coarse(cfg, phi0, u0, out):
    """Coarse window of a domain's initial fields (p = 0)."""
    dev = out.device
    phi = torch.as_tensor(phi0, dtype=torch.float32, device=dev).contiguous()
    u = torch.as_tensor(u0, dtype=torch.float32, device=dev).contiguous()
    p = torch.zeros_like(phi)
    return coarse_fields(phi, u, p, cfg, out)


def intact_length(phi_coarse):
    """Intact length in fine lattice units of coarse phase fields [n, d, h, w]
    (planes from the inlet holding liquid without a gap, times two)."""
    has = (phi_coarse > 0.5).reshape(phi_coarse.shape[0], phi_coarse.shape[1], -1).any(axis=2)
    run = np.where(has.all(axis=1), phi_coarse.shape[1], np.argmin(has, axis=1))
    return 2 * run


class HybridRollout:
    """Network rollout of `doms` (list of (cfg, phi0, u0)) with solver
    fallback, from the solver's state at lag `start` (0: the initial fields);
    predictions whose budget violation exceeds `threshold` fall back."""

    def __init__(self, net: SG.Network, doms, storage="fp16", start=0, threshold=SG.FALLBACK_THRESHOLD):
        self.net, self.cfgs = net, [c for c, _, _ in doms]
        self.n = len(doms)
        self.threshold = threshold
        assert self.n == net.batch
        c0 = self.cfgs[0]
        self.shape = (5, WINDOW, c0["ny"] // 2, c0["nx"] // 2)
        self.solver = [lbm.Batch([d], storage=storage) for d in doms]
        self.sync = np.full(self.n, start, dtype=np.int64)  # lag of each solver state
        self.x = torch.empty((self.n,) + self.shape, device="cuda")
        for d, (c, phi0, u0) in enumerate(doms):
            if start == 0:
                initial_coarse(c, phi0, u0, self.x[d])
            else:
                self.solver[d].step(start * LAG)
                phi, u, p = self.solver[d].fields(0)
                coarse_fields(phi, u, p, c, self.x[d])
        self.x_prev = self.x.clone()
        self.solver_start = self.x.clone()
        self.lag = start
        self.start = start
        self.fallbacks = []              # (lag, domain)
        self.t_net = self.t_solver = 0.0

    def _solver_state(self, d, out):
        b = self.solver[d]
        k = self.lag - int(self.sync[d])
        t0 = time.perf_counter()
        b.step(k * LAG)
        phi, u, p = b.fields(0)
        coarse_fields(phi, u, p, self.cfgs[d], out)
        torch.cuda.synchronize()
        self.t_solver += time.perf_counter() - t0
        self.sync[d] = self.lag

    def advance(self):
        """One lag for every domain; returns the domains that fell back."""
        t0 = time.perf_counter()
        pred = self.net.predict(self.x)
        torch.cuda.synchronize()
        self.t_net += time.perf_counter() - t0
        bad = (np.nonzero(SG.fallback_mask(self.x_prev, self.x, pred, self.threshold))[0]
               if self.lag > self.start else [])
        self.lag += 1
        for d in bad:
            self._solver_state(int(d), pred[int(d)])
            self.fallbacks.append((self.lag, int(d)))
        self.x_prev.copy_(self.x)
        self.x.copy_(pred)
        return list(map(int, bad))


def solver_regime(cfg, phi0, u0, window, storage="fp16"):
    """Regime of one domain from the solver: intact lengths every lag over
    lags window[0]..window[1]; returns (jetting, median L_b / D, seconds)."""
    t0 = time.perf_counter()
    b = lbm.Batch([(cfg, phi0, u0)], storage=storage)
    b.step(window[0] * LAG)
    jet, med = _solver_window(b, cfg, window)
    return jet, med, time.perf_counter() - t0


def _solver_window(b, cfg, window):
    """Regime from a one-domain solver batch standing at lag window[0]."""
    lb = []
    for k in range(window[0], window[1] + 1):
        lb.append(b.intact_length(0.5)[0])
        if k < window[1]:
            b.step(LAG)
    torch.cuda.synchronize()
    med = float(np.median(lb)) / (2.0 * cfg["inlet_radius"])
    return med > 2.0, med


class AcceleratedSearch:
    """Bisection for the first jetting index in which each probe runs the
    solver only to lag `start` and the network (batch 1) from there through
    the window; the probed domain's solver state at lag `start` is kept.
    The adjacent pair the search ends on is then confirmed by the solver,
    continuing the kept states through the window.  A confirmed regime
    overrides the network's call, and the search repeats with it until the
    confirmed pair drips / jets, so the result is the solver-only one
    whenever the solver's regime is monotone in We.  Solver steps are
    counted: start * LAG per probe, (window[1] - start) * LAG per
    confirmation."""

    def __init__(self, net: SG.Network, doms, window, start, storage="fp16"):
        assert net.batch == 1 and start <= window[0]
        self.net, self.doms, self.window, self.start, self.storage = net, doms, window, start, storage
        self.netcall, self.confirmed, self.state = {}, {}, {}
        self.medians = {}
        self.solver_steps = 0
        self.probes, self.confirmations = [], []

    def _network(self, i):
        cfg, phi0, u0 = self.doms[i]
        b = lbm.Batch([(cfg, phi0, u0)], storage=self.storage)
        b.step(self.start * LAG)
        self.solver_steps += self.start * LAG
        x = torch.empty((1, 5, WINDOW, cfg["ny"] // 2, cfg["nx"] // 2), device="cuda")
        coarse_fields(*b.fields(0), cfg, x[0])
        lb = []
        for k in range(self.start + 1, self.window[1] + 1):
            x = self.net.predict(x)
            if k >= self.window[0]:
                lb.append(intact_length(x[:, 0].cpu().numpy())[0])
        med = float(np.median(lb)) / (2.0 * cfg["inlet_radius"])
        self.state[i] = b
        self.probes.append(i)
        self.medians[("net", i)] = med
        return med > 2.0

    def call(self, i):
        if i in self.confirmed:
            return self.confirmed[i]
        if i not in self.netcall:
            self.netcall[i] = self._network(i)
        return self.netcall[i]

    def confirm(self, i):
        if i not in self.confirmed:
            self.call(i)  # the kept state comes from the probe
            b = self.state.pop(i)
            b.step((self.window[0] - self.start) * LAG)
            jet, med = _solver_window(b, self.doms[i][0], self.window)
            self.solver_steps += (self.window[1] - self.start) * LAG
            self.confirmed[i] = jet
            self.medians[("solver", i)] = med
            self.confirmations.append(i)
            del b
        return self.confirmed[i]

    def run(self):
        """First jetting index (None if the last domain drips)."""
        n = len(self.doms)
        while True:
            lo, hi = 0, n - 1
            if not self.call(hi):
                if not self.confirm(hi):
                    return None
                continue
            if self.call(lo):
                if self.confirm(lo):
                    return lo
                continue
            while hi - lo > 1:
                mid = (lo + hi) // 2
                if self.call(mid):
                    hi = mid
                else:
                    lo = mid
            if not self.confirm(lo) and self.confirm(hi):
                return hi


def bisect(probe, lo, hi, known=None):
    """Smallest jetting index on a monotone grid, given that index lo drips
    and index hi jets (either may be None: unknown ends are probed).
    probe(i) -> bool (jetting).  Returns (first jetting index, probes)."""
    known = dict(known or {})
    calls = []

    def call(i):
        if i not in known:
            known[i] = probe(i)
            calls.append(i)
        return known[i]

    if not call(hi):
        return None, calls
    if call(lo):
        return lo, calls
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if call(mid):
            hi = mid
        else:
            lo = mid
    return hi, calls


def weber_grid(n=64):
    """The sweep's domains (lengths, Weber numbers) as (cfg, phi0, u0)."""
    return W.jet_sweep(n=n)
