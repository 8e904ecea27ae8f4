#!/usr/bin/env python3
"""Benchmark: MLUPS and HBM-roofline fraction of the phase-field LBM step on
one MI355X, on the 3D Rayleigh-Taylor workload (D3Q19, 256 x 1024 x 256,
FP32 populations), next to the FP64 CPU oracle timed on a bounded sample.

One step = phase-field pass + fused macroscopic/collision/AA-streaming kernel
for both population sets.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
METRIC = "MLUPS + % HBM roofline; FP16-stored & batched vs FP32 at ≤1e-3 φ error"


def algorithmic_bytes_per_node(q: int, d: int, pop_bytes: int):
    """Bytes each lattice update must move (populations read and written once,
    velocity state read and written once, phi written once and read once;
    the 16-bit forms also read the previous step's phi, against which the
    stored values were encoded, in both kernels).
    Returns (whole step, fused step kernel, phase-field pass)."""
    ref = 4 if pop_bytes == 2 else 0
    kstep = 2 * 2 * q * pop_bytes + 2 * d * 4 + 4 + ref
    kphi = q * pop_bytes + 4 + ref
    return 2 * 2 * q * pop_bytes + 2 * d * 4 + 8 + ref, kstep, kphi


def run_gpu(cfg, phi0, u0, storage, steps, warmup, tile=None, autotune=True, zchunk=None, bpc=None):
    import torch

    from paper_2505_12205_amd import lbm
    sim = lbm.Sim(cfg, phi0, u0, storage=storage)
    if zchunk is not None:
        sim.set_zchunk(zchunk)
    if bpc is not None:
        sim.set_blocks_per_cu(bpc)
    if tile:
        sim.set_tile(*tile)
    elif autotune:
        choice = sim.autotune(trial_steps=6)
        print(f"[bench] {storage} autotune -> tile {choice[0]}x{choice[1]} nontemporal={choice[2]} "
              f"z-chunk {sim.zchunk} blocks/CU {sim.blocks_per_cu} {choice[3]:.3f} ms/step",
              file=sys.stderr, flush=True)
    sim.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kt = sim.kernel_times(min(steps, 20))
    mass, ke = sim.reduce()
    return sim, dt, kt, mass, ke


def run_jet(steps, warmup, forms=("fp32", "fp16", "bf16"), autotune=True, tile=None, zchunk=None, bpc=None):
    """The precision-form jet at its stated size (192 x 192 x 768, inlet radius
    12, rho* = 800, We = 5, Re = 300, convective outflow) in each storage
    form: MLUPS of the whole step and the fused kernel's algorithmic GB/s."""
    import torch

    from paper_2505_12205_amd import workloads as W
    cfg, phi0, u0 = W.jet3d()
    n = cfg["nx"] * cfg["ny"] * cfg["nz"]
    out = {"nodes": n}
    for st in forms:
        sim, dt, kt, _, _ = run_gpu(cfg, phi0, u0, st, steps, warmup, tile, autotune, zchunk, bpc)
        _, bk, _ = algorithmic_bytes_per_node(19, 3, 4 if st == "fp32" else 2)
        out[st] = {"MLUPS": round(n * steps / dt / 1e6, 1), "ms_per_step": round(dt / steps * 1e3, 4),
                   "step_kernel_ms": round(kt[1], 4), "phi_pass_ms": round(kt[0], 4),
                   "outlet_ms": round(kt[2], 4),
                   "step_kernel_GBs": round(bk * n / (kt[1] * 1e-3) / 1e9, 1)}
        print(f"[bench] jet 192x192x768 {st} {out[st]}", file=sys.stderr, flush=True)
        del sim
        torch.cuda.empty_cache()
    return out


def run_batch(steps, warmup, storage="fp16", autotune=True, launch=None):
    """The batched Weber sweep: 64 jet domains 96 x 96 x L_k (seeded lengths
    256..768), We_k log-spaced 0.5..8, one set of launches per step."""
    import torch

    from paper_2505_12205_amd import lbm
    from paper_2505_12205_amd import workloads as W
    doms = W.jet_sweep()
    bt = lbm.Batch(doms, storage=storage)
    del doms
    if launch:
        bt.set_launch(*launch)
    elif autotune:
        choice = bt.autotune(trial_steps=4)
        print(f"[bench] batch {storage} autotune -> tile {choice[0]}x{choice[1]} blocks/CU={choice[2]} "
              f"nontemporal={choice[3]} {choice[4]:.3f} ms/step", file=sys.stderr, flush=True)
    bt.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bt.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kt = bt.kernel_times(6)
    lb = bt.intact_length(0.5)
    return bt.nodes, dt, kt, lb


MFMA_BF16_PEAK_TFLOPS = 2500.0  # MI355X dense bf16, published


def run_surrogate(steps=10, batch=32):
    """Training-step and forward throughput of the surrogate (batch 32 of
    5 x 192 x 48 x 48 coarse windows) in TFLOP/s of executed MFMA work."""
    import torch

    from paper_2505_12205_amd import surrogate as SG
    net = SG.Network(batch, 192, 48, 48, seed=0)
    g = torch.Generator(device="cuda").manual_seed(0)
    x = torch.randn((batch, 5, 192, 48, 48), device="cuda", generator=g) * 0.1
    t = x + 0.01 * torch.randn(x.shape, device="cuda", generator=g)
    fl = 0
    for (name, *_r) in net.spec:
        L = net.lay[name]
        od, oh, ow = [-(-(L["u"] * e) // L["s"]) for e in net.ext_in[name]]
        fl += 2 * batch * od * oh * ow * L["cip"] * L["cop"] * 27
    for _ in range(3):
        net.train_step(x, t, with_loss=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        net.train_step(x, t, with_loss=False)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    t0 = time.perf_counter()
    for _ in range(steps):
        net.forward(x)
    torch.cuda.synchronize()
    df = (time.perf_counter() - t0) / steps
    return {"train_step_ms": round(dt * 1e3, 2), "train_TFLOPs": round(3 * fl / dt / 1e12, 1),
            "forward_ms": round(df * 1e3, 2), "forward_TFLOPs": round(fl / df / 1e12, 1),
            "forward_flop": fl, "mfma_bf16_peak_TFLOPs": MFMA_BF16_PEAK_TFLOPS,
            "train_frac": round(3 * fl / dt / 1e12 / MFMA_BF16_PEAK_TFLOPS, 4),
            "batch": batch, "window": [5, 192, 48, 48]}


def run_drops(reps=20):
    """Drop-size diagnostic on the breaking-jet field of the jet workload's
    size (192 x 192 x 768): labelling of {phi > 1/2} and the component
    statistics, wall time per call (each call synchronises)."""
    import torch
    from paper_2505_12205_amd import drops as D
    from paper_2505_12205_amd import workloads as W
    phi_h, placed = W.breakup_field()
    phi = torch.from_numpy(phi_h).cuda()
    ws = D.workspace(phi_h.shape)
    lab = torch.empty(phi_h.shape, dtype=torch.int32, device="cuda")
    for _ in range(3):
        D.label(phi, ws=ws, out=lab)
        c = D.components(lab, axis=2, ws=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        D.label(phi, ws=ws, out=lab)
    t_label = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        c = D.components(lab, axis=2, ws=ws)
    t_comp = (time.perf_counter() - t0) / reps
    n = phi.numel()
    return {"nodes": n, "components": int(len(c["root"])), "drops_placed": len(placed),
            "label_ms": round(t_label * 1e3, 3), "components_ms": round(t_comp * 1e3, 3),
            "label_GBs_algorithmic": round(8.0 * n / t_label / 1e9, 1),
            "label_Gnodes_per_s": round(n / t_label / 1e9, 2)}


def counted_traffic(zchunk, tile):
    """HBM bytes per launch of the fused FP32 step from the committed counter
    summaries (FETCH_SIZE and WRITE_SIZE, each scaled by its reading for a copy
    of known size): the record of the interior kernel the run used (tiled for
    z_chunk 0, z-marching otherwise) at the run's tile, or None when there is
    none or the kernel source has changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None, None
    with open(path) as f:
        recs = json.load(f)["records"]
    csrc = os.path.join(ROOT, "paper_2505_12205_amd", "csrc")
    h = hashlib.sha256()
    for name in ("kernels.hpp", "lattice.hpp"):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(f.read())
    for rec in recs:
        if h.hexdigest()[:16] != rec.get("kernel_source_sha256_16"):
            continue
        if (zchunk > 0) != (rec.get("z_chunk", 0) > 0) or list(tile) != rec.get("tile"):
            continue
        return float(rec["traffic_bytes_per_launch"]), rec.get("summary")
    return None, None


def copy_probe(gib: float = 2.0, reps: int = 10):
    """Device-to-device copy of a buffer of known size (torch's copy kernel):
    the practical HBM ceiling, and the calibration run for the byte counters."""
    import torch
    n = int(gib * (1 << 30) // 4)
    a = torch.empty(n, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    return 2 * n * 4 / dt / 1e9


def cpu_baseline(budget_s: float = 15.0):
    """FP64 oracle on a slab of the same Rayleigh-Taylor workload (same
    per-node parameters, 256 x 128 x 32 nodes), timed for about budget_s."""
    import oracle
    from paper_2505_12205_amd import workloads as W
    cfg, phi0, u0 = W.rt3d(nx=256, ny=128, nz=32, lref=256)
    o = oracle.Oracle(cfg).init(phi0, u0)
    t0 = time.perf_counter()
    o.step(1)
    t1 = time.perf_counter() - t0
    n = max(1, int(budget_s / max(t1, 1e-3)))
    t0 = time.perf_counter()
    o.step(n)
    dt = time.perf_counter() - t0
    nodes = 256 * 128 * 32
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": round(nodes * n / dt / 1e6, 4), "unit": "MLUPS", "cores": threads,
            "kind": "oracle",
            "sample": f"FP64 oracle, Rayleigh-Taylor slab 256x128x32 (same per-node parameters), "
                      f"{n} steps in {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms", default="fp16,bf16",
                    help="comma list of 16-bit storage forms to time beside FP32 ('' for none)")
    ap.add_argument("--tile", default="", help="bx,by launch shape of the fused kernel")
    ap.add_argument("--zchunk", type=int, default=None,
                    help="planes per z-marching task of the fused kernel (0: tiled kernel)")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched Weber sweep")
    ap.add_argument("--no-bgk", action="store_true", help="skip the FP32 run with the BGK operator")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the surrogate training step")
    ap.add_argument("--copy-probe-only", action="store_true",
                    help="only run the 2 GiB copy (counter calibration)")
    ap.add_argument("--blocks-per-cu", type=int, default=None,
                    help="blocks per CU of the persistent launches, 0: one block per tile (with --tile; "
                         "the batched launch defaults to 8)")
    ap.add_argument("--surrogate-only", action="store_true",
                    help="only time the surrogate's training step (for profiling it alone)")
    ap.add_argument("--drops-only", action="store_true",
                    help="only run the drop-size diagnostic (for profiling it alone)")
    ap.add_argument("--no-drops", action="store_true", help="skip the drop-size diagnostic")
    ap.add_argument("--no-jet", action="store_true", help="skip the 192x192x768 jet in each storage form")
    ap.add_argument("--jet-only", action="store_true",
                    help="only run the 192x192x768 jet in the storage forms of --forms plus fp32 "
                         "(for profiling it alone)")
    ap.add_argument("--batch-only", action="store_true",
                    help="only run the batched Weber sweep (for profiling it alone)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU slab decomposition is a design note only)", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    from paper_2505_12205_amd import workloads as W
    tile = tuple(int(v) for v in args.tile.split(",")) if args.tile else None
    copy_gbs = copy_probe()
    from paper_2505_12205_amd import probe
    ceil = probe.ceilings()
    print(f"[bench] device copy {copy_gbs:.0f} GB/s (torch); hand-written probes {ceil} GB/s",
          file=sys.stderr, flush=True)
    if args.copy_probe_only:
        return
    if args.surrogate_only:
        print(json.dumps({"surrogate_bf16_mfma": run_surrogate(steps=args.steps)}), flush=True)
        return
    if args.drops_only:
        print(json.dumps({"drops": run_drops()}), flush=True)
        return
    if args.jet_only:
        forms = ["fp32"] + [f for f in args.forms.split(",") if f and f != "fp32"]
        print(json.dumps({"jet_192x192x768": run_jet(args.steps, args.warmup, forms, not args.no_autotune, tile,
                                                     args.zchunk, args.blocks_per_cu)}), flush=True)
        return
    if args.batch_only:
        bpc = 8 if args.blocks_per_cu is None else args.blocks_per_cu
        launch = (tile[0], tile[1], bpc, False) if tile else None
        nb, dtb, ktb, lb = run_batch(args.steps, args.warmup, "fp16", not args.no_autotune, launch)
        print(json.dumps({"batched_fp16_MLUPS": round(nb * args.steps / dtb / 1e6, 1), "nodes": nb,
                          "ms_per_step": round(dtb / args.steps * 1e3, 3), "phi_ms": round(ktb[0], 3),
                          "step_ms": round(ktb[1], 3), "outlet_ms": round(ktb[2], 4)}), flush=True)
        return

    cfg, phi0, u0 = W.rt3d()
    N = cfg["nx"] * cfg["ny"] * cfg["nz"]
    print(f"[bench] workload {cfg['name']} N={N} steps={args.steps} warmup={args.warmup}",
          file=sys.stderr, flush=True)
    sim, dt, kt, mass, ke = run_gpu(cfg, phi0, u0, "fp32", args.steps, args.warmup, tile,
                                    not args.no_autotune, args.zchunk, args.blocks_per_cu)
    mlups = N * args.steps / dt / 1e6
    b_step, b_k, b_phi = algorithmic_bytes_per_node(19, 3, 4)
    achieved = b_k * N / (kt[1] * 1e-3) / 1e9
    print(f"[bench] fp32 {mlups:.1f} MLUPS, kernels phi {kt[0]:.3f} ms step {kt[1]:.3f} ms",
          file=sys.stderr, flush=True)
    tile_used = sim.tile
    zchunk_used = sim.zchunk
    bpc_used = sim.blocks_per_cu
    del sim
    torch.cuda.empty_cache()

    forms = {}
    for st in [f for f in args.forms.split(",") if f]:
        s2, dt2, kt2, _, _ = run_gpu(cfg, phi0, u0, st, max(20, args.steps // 2), 5, tile,
                                     not args.no_autotune, args.zchunk, args.blocks_per_cu)
        n2 = max(20, args.steps // 2)
        _, bk2, _ = algorithmic_bytes_per_node(19, 3, 2)
        forms[st] = {"MLUPS": round(N * n2 / dt2 / 1e6, 1),
                     "step_kernel_ms": round(kt2[1], 4),
                     "step_kernel_GBs": round(bk2 * N / (kt2[1] * 1e-3) / 1e9, 1)}
        print(f"[bench] {st} {forms[st]}", file=sys.stderr, flush=True)
        del s2
        torch.cuda.empty_cache()

    if not args.no_bgk:  # the selectable single-relaxation operator on the same workload
        n2 = max(20, args.steps // 2)
        s2, dt2, kt2, _, _ = run_gpu(dict(cfg, collision="bgk"), phi0, u0, "fp32", n2, 5, tile,
                                     not args.no_autotune, args.zchunk, args.blocks_per_cu)
        forms["bgk_fp32"] = {"MLUPS": round(N * n2 / dt2 / 1e6, 1),
                             "step_kernel_ms": round(kt2[1], 4),
                             "step_kernel_GBs": round(b_k * N / (kt2[1] * 1e-3) / 1e9, 1)}
        print(f"[bench] bgk_fp32 {forms['bgk_fp32']}", file=sys.stderr, flush=True)
        del s2
        torch.cuda.empty_cache()

    if not args.no_jet:
        forms["jet_192x192x768"] = run_jet(max(20, args.steps // 4), 5,
                                           tuple(["fp32"] + [f for f in args.forms.split(",") if f]),
                                           not args.no_autotune)
        torch.cuda.empty_cache()

    if not args.no_batch:
        nb, dtb, ktb, lb = run_batch(max(20, args.steps // 4), 4, "fp16", not args.no_autotune)
        nsb = max(20, args.steps // 4)
        forms["batched_fp16"] = {"MLUPS": round(nb * nsb / dtb / 1e6, 1), "domains": 64, "nodes": nb,
                                 "ms_per_step": round(dtb / nsb * 1e3, 3),
                                 "phi_ms": round(ktb[0], 3), "step_ms": round(ktb[1], 3),
                                 "outlet_ms": round(ktb[2], 4),
                                 "intact_length_range": [min(lb), max(lb)]}
        print(f"[bench] batched_fp16 {forms['batched_fp16']}", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()

    if not args.no_drops:
        forms["drops"] = run_drops()
        print(f"[bench] drops {forms['drops']}", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()

    if not args.no_surrogate:
        forms["surrogate_bf16_mfma"] = run_surrogate()
        print(f"[bench] surrogate {forms['surrogate_bf16_mfma']}", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()

    traffic, traffic_src = counted_traffic(zchunk_used, tile_used)
    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (analytic cosine-perturbed interface, seeded parameters)",
        "config": {"workload": "rayleigh_taylor_3d_d3q19", "nx": 256, "ny": 1024, "nz": 256,
                   "storage": "fp32", "atwood": 0.5, "reynolds": 3000, "W": 5,
                   "tile": list(tile_used), "z_chunk": zchunk_used, "blocks_per_cu": bpc_used},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "traffic_source": traffic_src,
                     "traffic_GBs": round(traffic / (kt[1] * 1e-3) / 1e9, 1) if traffic else None,
                     "kernel": ("kb_march" if zchunk_used else "kb_interior") +
                               " (fused macroscopic update + both collisions + AA streaming)",
                     "bytes_per_node": b_k, "kernel_ms": round(kt[1], 4),
                     "phi_pass_ms": round(kt[0], 4), "device_copy_GBs": round(copy_gbs, 1),
                     "probe_GBs": ceil,
                     "frac_of_inplace_probe": round(achieved / ceil["soa_inplace"], 4)},
        "step_bytes_per_node": b_step,
        "mass": mass,
        "kinetic": ke,
        "forms": forms,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
