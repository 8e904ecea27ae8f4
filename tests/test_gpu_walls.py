"""GPU parity of wall faces in every position the launches distinguish:
x walls (handled as wall lanes inside the tiled kernel), y walls (face rows)
and z walls (face planes), no-slip and free-slip, in 2D and 3D, against the
FP64 oracle: one even and one odd step at every node from the same FP32
state, and a few hundred steps of the coupled flow."""
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


# (lattice, bc of the x, y, z faces); gravity along y in 3D (the heavy layer
# sits on top), none in 2D
CASES = {
    "x_noslip_y_freeslip": (19, ("noslip", "noslip", "freeslip", "freeslip", "periodic", "periodic")),
    "x_freeslip_y_noslip_z_noslip": (19, ("freeslip", "freeslip", "noslip", "noslip", "noslip", "noslip")),
    "x_mixed_walls": (19, ("noslip", "freeslip", "noslip", "noslip", "periodic", "periodic")),
    "x_walls_only": (19, ("freeslip", "freeslip", "periodic", "periodic", "periodic", "periodic")),
    "2d_x_noslip": (9, ("noslip", "noslip", "periodic", "periodic", "periodic", "periodic")),
    "2d_x_freeslip_y_noslip": (9, ("freeslip", "freeslip", "noslip", "noslip", "periodic", "periodic")),
}


def _case(name, seed=11, shape=(21, 26, 9)):
    q, bc = CASES[name]
    if q == 19:
        cfg, phi0, u0 = W.rt3d(nx=shape[0], ny=shape[1], nz=shape[2], lref=256)
    else:
        cfg, phi0, u0 = W.drop2d(n=32, radius=9.0, center=(13.0, 17.0))
    cfg = dict(cfg)
    cfg["bc"] = bc
    cfg["name"] = name
    phi0, u0 = W.perturb(phi0, u0, seed, 0.01, 2e-3)
    return cfg, phi0, u0


@pytest.mark.parametrize("name", list(CASES))
def test_walls_one_step_every_node(name):
    lbm = _lbm()
    cfg, phi0, u0 = _case(name)
    s = lbm.Sim(cfg, phi0, u0)
    s.set_tile(16, 4)  # several tiles per row: wall lanes at both tile edges
    s.step(5)
    q = cfg["q"]
    for _ in range(2):
        h, g, u = [t.cpu().numpy() for t in s.export_state()]
        _log(f"[gpu] walls {name} one step at parity {s.steps_done % 2}")
        s.step(1)
        h1, g1, u1 = [t.cpu().numpy() for t in s.export_state()]
        nodes = np.arange(h.reshape(q, -1).shape[1])
        ho, go, uo = oracle.step_nodes_f32(cfg, h, g, u, nodes)
        eh = np.abs(h1.reshape(q, -1).T - ho).max()
        eg = np.abs(g1.reshape(q, -1).T - go).max()
        eu = np.abs(u1.reshape(3, -1).T - uo).max()
        _log(f"walls {name}: max|dh|={eh:.3e} max|dg|={eg:.3e} max|du|={eu:.3e}")
        assert eh < 2e-7 and eg < 2e-7 and eu < 2e-7


@pytest.mark.parametrize("name", ["x_noslip_y_freeslip", "x_freeslip_y_noslip_z_noslip", "2d_x_noslip"])
def test_walls_300_steps(name):
    lbm = _lbm()
    cfg, phi0, u0 = _case(name, seed=4)
    o = oracle.Oracle(cfg).init(phi0, u0).step(300)
    phi_o, u_o, _ = o.fields()
    for tile in [(32, 2), (64, 1)]:
        _log(f"[gpu] walls {name} 300 steps tile {tile}")
        s = lbm.Sim(cfg, phi0, u0).set_tile(*tile).step(300)
        phi_g, u_g, _ = s.fields()
        ephi = np.abs(phi_g.cpu().numpy() - phi_o).max()
        eu = np.abs(u_g.cpu().numpy() - u_o).max() / max(np.abs(u_o).max(), 1e-30)
        _log(f"walls {name} {tile}: max|dphi|={ephi:.3e} rel_u={eu:.3e}")
        assert ephi <= 1e-5 and eu <= 1e-4


@pytest.mark.parametrize("storage", ["fp16", "bf16"])
def test_walls_16bit_one_step_decode(storage):
    """16-bit forms on x walls: the value each wall lane stores is encoded
    relative to the phase field of the node that reads it; after a few steps
    the stepped state agrees with the FP32 path to the storage precision."""
    lbm = _lbm()
    cfg, phi0, u0 = _case("x_mixed_walls", seed=8)
    a = lbm.Sim(cfg, phi0, u0, storage="fp32").step(40)
    b = lbm.Sim(cfg, phi0, u0, storage=storage).step(40)
    pa, _, _ = a.fields()
    pb, _, _ = b.fields()
    e = (pa - pb).abs().max().item()
    _log(f"walls 16-bit {storage}: max|dphi| vs fp32 = {e:.3e}")
    assert e <= (2e-4 if storage == "fp16" else 4e-3)
