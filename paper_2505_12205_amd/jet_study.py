"""Breakup length and drop size against the Weber number on the batched jet
sweep (the jet-breakup section's two diagnostics, L_b / D_j and d_e / D_j
against We), all on the GPU: the 64 domains advance together; every `every`
steps from `start` on, each domain's intact length (lbm_batch_intact_length)
and its drops (libdrops: components of phi > 1/2 apart from the intact jet
and from those leaving through the outlet, equivalent diameters) are
sampled.  A domain whose mass turns non-finite is marked and left out from
then on.

    python -m paper_2505_12205_amd.jet_study --steps 9600 --out runs/jet_study.json
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np
import torch

from . import drops as DR
from . import lbm
from . import workloads as W


def run(steps=9600, start=4800, every=320, storage="fp16", n=64, log=print):
    doms = W.jet_sweep(n=n)
    cfgs = [c for c, _, _ in doms]
    we = np.asarray(W.sweep_weber(n))
    dj = 2.0 * cfgs[0]["inlet_radius"]
    b = lbm.Batch(doms, storage=storage)
    t0 = time.perf_counter()
    done = 0
    while done < start:
        k = min(1600, start - done)
        b.step(k)
        done += k
        torch.cuda.synchronize()
        log(f"[jet_study] step {done}: advancing to the first sample, {time.perf_counter() - t0:.0f} s")
    alive = np.ones(n, bool)
    lb = [[] for _ in range(n)]
    de = [[] for _ in range(n)]
    counts = [[] for _ in range(n)]
    t = start
    while True:
        mass, ke = b.reduce(strict=False)
        alive &= np.isfinite(mass) & np.isfinite(ke)
        lengths = b.intact_length(0.5)
        for d in range(n):
            if not alive[d]:
                continue
            st = DR.drop_sizes(b.fields(d)[0], cfgs[d])
            lb[d].append(lengths[d])
            de[d].extend(st["d_e"].tolist())
            counts[d].append(st["count"])
        log(f"[jet_study] step {t}: {int(alive.sum())} finite domains, "
            f"{sum(c[-1] for c in counts if c)} drops, {time.perf_counter() - t0:.0f} s")
        if t + every > steps:
            break
        b.step(every)
        t += every
    mean_de = np.array([np.mean(x) / dj if x else np.nan for x in de])
    mean_lb = np.array([np.mean(x) / dj if x else np.nan for x in lb])
    return {
        "steps": [start, t], "every": every, "storage": storage, "D_j": dj,
        "weber": we.tolist(), "finite": alive.tolist(),
        "lb_over_Dj": mean_lb.tolist(), "de_over_Dj": mean_de.tolist(),
        "drops_per_sample": [float(np.mean(c)) if c else 0.0 for c in counts],
        "drop_observations": [len(x) for x in de],
        "seconds": time.perf_counter() - t0,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=9600)
    ap.add_argument("--start", type=int, default=4800)
    ap.add_argument("--every", type=int, default=320)
    ap.add_argument("--storage", default="fp16")
    ap.add_argument("--out", default="")
    a = ap.parse_args()
    if not torch.cuda.is_available():
        raise SystemExit("jet_study needs a GPU")
    res = run(a.steps, a.start, a.every, a.storage, log=lambda m: print(m, flush=True))
    we, de, lbd = np.array(res["weber"]), np.array(res["de_over_Dj"]), np.array(res["lb_over_Dj"])
    for k in range(0, len(we), 4):
        print(f"We {we[k]:6.3f}  L_b/D_j {lbd[k]:6.2f}  d_e/D_j {de[k]:6.3f}  "
              f"drops/sample {res['drops_per_sample'][k]:5.2f}  finite {res['finite'][k]}", flush=True)
    if a.out:
        os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
        with open(a.out, "w") as f:
            json.dump(res, f)


if __name__ == "__main__":
    main()
