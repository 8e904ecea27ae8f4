"""GPU parity of the drop-size diagnostic (libdrops.so through the C-ABI)
against the oracle (oracle/drops.c) on the same float32 phase fields:
labels and component root, size and axial extent bit-exact, equivalent
diameters to float rounding (relative 1e-6).

Fields: smooth random fields at liquid fractions from sparse drops to
near-percolating networks (one component with many branches: heavy union
contention), in shapes that span many waves and blocks with ragged ends, 2D
and single-row cases, every periodicity; the synthetic breaking jet at the
full 192 x 192 x 768 size; the phase field of the solver's own jet; the
degenerate fields; the capacity error path."""
import ctypes as C
import sys

import numpy as np
import pytest
from scipy import ndimage

import oracle
from paper_2505_12205_amd import workloads as W

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dr():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("a GPU test ran without a GPU")
    from paper_2505_12205_amd import drops
    return torch, drops


def _field(shape, frac, seed, smooth=1.0):
    rng = np.random.default_rng(seed)
    f = ndimage.gaussian_filter(rng.standard_normal(shape), smooth, mode="wrap")
    return (f - np.quantile(f, 1.0 - frac) + 0.5).astype(np.float32)


def _check(phi, periodic=(False, False, False), axes=(0, 1, 2)):
    torch, dr = _dr()
    _log(f"[gpu] drops shape={phi.shape} periodic={periodic}")
    g = dr.label(torch.from_numpy(phi).cuda(), periodic)
    got = g.cpu().numpy()
    ref = oracle.label(phi, periodic)
    assert np.array_equal(got, ref.reshape(got.shape)), "labels differ"
    for axis in axes:
        cg = dr.components(g, axis=axis)
        co = oracle.components(ref, axis=axis)
        for k in ("root", "size", "lo", "hi"):
            assert np.array_equal(cg[k], co[k]), (k, axis)
        assert np.allclose(cg["deq"], co["deq"], rtol=1e-6, atol=0)
    return len(np.unique(ref[ref >= 0]))


@pytest.mark.parametrize("shape,frac,seed", [((9, 13, 17), 0.3, 1), ((12, 10, 31), 0.15, 2),
                                             ((33, 47, 65), 0.3, 3), ((5, 70, 130), 0.5, 4),
                                             ((64, 64, 64), 0.12, 5), ((17, 3, 257), 0.3, 6)])
def test_labels_and_components_match_oracle(shape, frac, seed):
    phi = _field(shape, frac, seed)
    for per in ((False, False, False), (True, False, False), (False, True, True), (True, True, True)):
        n = _check(phi, per)
        _log(f"shape {shape} frac {frac} periodic {per}: {n} components")


@pytest.mark.parametrize("shape", [(1, 40, 50), (1, 1, 300), (1, 129, 1), (2, 2, 2), (1, 1, 1)])
def test_planes_rows_and_tiny_fields(shape):
    phi = _field(shape, 0.4, 7) if np.prod(shape) > 8 else np.random.default_rng(8).random(shape).astype(np.float32)
    for per in ((False, False, False), (True, True, False)):
        _check(phi, per)


def test_degenerate_fields():
    _check(np.zeros((4, 5, 70), np.float32))
    _check(np.ones((4, 5, 70), np.float32))
    _check(np.full((3, 3, 3), 0.5, np.float32))  # the threshold is strict


def test_full_size_breakup_field():
    """192 x 192 x 768: the intact column and the drop train; every drop's
    d_e against the diameter of the sphere placed."""
    torch, dr = _dr()
    phi, placed = W.breakup_field()
    _check(phi, axes=(2,))
    cfg, _, _ = W.jet3d()
    st = dr.drop_sizes(torch.from_numpy(phi).cuda(), cfg)
    _log(f"breakup field: {st['components']} components, {st['count']} drops, intact extent "
         f"{st['intact_extent']}, mean d_e/D_j {st['mean_d_e_over_Dj']:.3f}")
    assert st["intact_extent"] == 300
    inside = [2 * r for (c, r) in placed if c[2] + r < cfg["nz"] - 1]
    assert st["count"] == len(inside)
    assert np.allclose(np.sort(st["d_e"]), np.sort(inside), rtol=0.08)


def test_solver_jet_field():
    """The phase field of the solver's jet copy after 600 steps (inlet
    column and its cap), labelled on the GPU and by the oracle."""
    torch, dr = _dr()
    from paper_2505_12205_amd import lbm
    cfg, phi0, u0 = W.jet3d(nx=24, ny=24, nz=48, radius=6.0, param_radius=12.0, stub=10.0)
    s = lbm.Sim(cfg, phi0, u0).step(600)
    phi = s.fields()[0].contiguous()
    _check(phi.cpu().numpy(), dr.periodic_axes(cfg), axes=(2,))
    st = dr.drop_sizes(phi, cfg)
    assert st["intact_extent"] >= 10 and st["components"] >= 1


def test_capacity_error_returns_the_first_components():
    torch, dr = _dr()
    phi = _field((16, 16, 64), 0.1, 9)
    g = dr.label(torch.from_numpy(phi).cuda())
    full = dr.components(g, axis=2)
    n = len(full["root"])
    assert n > 4
    cap = 3
    ws = dr.workspace(phi.shape)
    bufs = [torch.empty(cap, dtype=torch.int32, device="cuda") for _ in range(4)]
    deq = torch.empty(cap, dtype=torch.float32, device="cuda")
    nc = C.c_int()
    rc = dr.lib.dr_components(g.data_ptr(), 64, 16, 16, 2, cap, *[b.data_ptr() for b in bufs], deq.data_ptr(),
                              C.byref(nc), ws.data_ptr(), ws.numel(), torch.cuda.current_stream().cuda_stream)
    assert rc == dr.DR_ECAPACITY and nc.value == n
    assert np.array_equal(bufs[0].cpu().numpy(), full["root"][:cap])
    assert np.array_equal(bufs[1].cpu().numpy(), full["size"][:cap])
