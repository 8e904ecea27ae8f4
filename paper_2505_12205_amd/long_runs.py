"""Long runs of the stated workloads on one GPU, with their diagnostics.

rt: the 3D Rayleigh-Taylor workload at full size (D3Q19, 256 x 1024 x 256,
    FP32) for 20,000 steps (t* = t sqrt(g At / L) reaches 2.2): finiteness,
    the FP64 mass drift, kinetic energy and the bubble-front / spike-tip
    positions (the paper's section "Rayleigh-Taylor instability").

jet: the precision-form jet at full size (192 x 192 x 768, inlet radius 12,
    rho* = 800, We = 5, Re = 300, convective outflow), one domain per
    storage form advanced side by side; sum phi and the intact length
    L_b / D_j of the 16-bit forms against FP32 over the run.

    python -m paper_2505_12205_amd.long_runs rt --steps 20000 --every 2000
    python -m paper_2505_12205_amd.long_runs jet --steps 50000 --every 5000 --forms fp32,fp16,bf16
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np
import torch

from . import lbm
from . import workloads as W


def _fronts(phi, lref):
    """Bubble front (highest y holding light fluid) and spike tip (lowest y
    holding heavy fluid), in units of L relative to the box centre."""
    ny = phi.shape[1]
    heavy = phi > 0.5
    rows = heavy.any(axis=(0, 2))
    light = (~heavy).any(axis=(0, 2))
    spike = int(np.argmax(rows))
    bubble = ny - 1 - int(np.argmax(light[::-1]))
    return (bubble - ny / 2) / lref, (spike - ny / 2) / lref


def rt(steps=20000, every=2000, log=print):
    cfg, phi0, u0 = W.rt3d()
    p = W.rt_params(lref=256)
    t_scale = np.sqrt(256.0 / (p["g"] * 0.5))  # L / sqrt(g At L) in steps
    s = lbm.Sim(cfg, phi0, u0)
    del phi0
    s.autotune(trial_steps=4)
    m0, k0 = s.reduce()
    rows = []
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        k = min(every, steps - done)
        s.step(k)
        done += k
        m, ke = s.reduce()
        phi = s.fields()[0].cpu().numpy()
        b, sp = _fronts(phi, 256.0)
        rows.append({"step": done, "t_star": round(done / t_scale, 3), "mass_drift": (m - m0) / m0,
                     "kinetic": ke, "bubble": b, "spike": sp})
        log(f"[rt] step {done} t*={done / t_scale:.2f} mass drift {(m - m0) / m0:+.2e} "
            f"KE {ke:.4e} bubble {b:+.3f} spike {sp:+.3f} ({time.perf_counter() - t0:.0f} s)")
    return {"workload": cfg["name"], "steps": steps, "wall_s": round(time.perf_counter() - t0, 1),
            "finite": bool(np.isfinite(rows[-1]["kinetic"])), "rows": rows}


def jet(steps=50000, every=5000, forms=("fp32", "fp16"), log=print):
    cfg, phi0, u0 = W.jet3d()
    dj = 2.0 * cfg["inlet_radius"]
    runs = {f: lbm.Batch([(cfg, phi0, u0)], storage=f) for f in forms}
    del phi0, u0
    rows = []
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        k = min(every, steps - done)
        for b in runs.values():
            b.step(k)
        done += k
        row = {"step": done}
        for f, b in runs.items():
            m, ke = b.reduce(strict=False)
            row[f] = {"mass": m[0], "kinetic": ke[0], "L_b_over_D": b.intact_length(0.5)[0] / dj}
        ref = row[forms[0]]
        for f in forms[1:]:
            row[f]["mass_rel_to_" + forms[0]] = row[f]["mass"] / ref["mass"] - 1.0
        rows.append(row)
        log(f"[jet] step {done}: " + " ".join(
            f"{f}: sum phi {row[f]['mass']:.6e} L_b/D {row[f]['L_b_over_D']:.2f}" for f in forms)
            + f" ({time.perf_counter() - t0:.0f} s)")
    return {"workload": cfg["name"], "steps": steps, "forms": list(forms),
            "wall_s": round(time.perf_counter() - t0, 1), "rows": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", choices=["rt", "jet"])
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--every", type=int, default=None)
    ap.add_argument("--forms", default="fp32,fp16,bf16")
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    log = lambda m: print(m, flush=True)  # noqa: E731
    if a.which == "rt":
        res = rt(a.steps or 20000, a.every or 2000, log)
    else:
        res = jet(a.steps or 50000, a.every or 5000, tuple(a.forms.split(",")), log)
    txt = json.dumps(res, indent=1)
    if a.out:
        with open(a.out, "w") as f:
            f.write(txt)
    print(txt, flush=True)


if __name__ == "__main__":
    main()
