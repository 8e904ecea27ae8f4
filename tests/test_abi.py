"""CPU checks of the C-ABI library: it loads, exports every symbol that
include/lbm.h declares, and rejects invalid parameter sets on the host
(no GPU call is made)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("lbm_init", "lbm_step", "lbm_fields", "lbm_reduce", "lbm_state_bytes", "lbm_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2505_12205_amd import lbm
    for n in _declared():
        assert hasattr(lbm.lib, n), n
    assert set(_declared()) <= set(lbm.EXPORTED) | {"lbm_init"}


def _cfg(**kw):
    from paper_2505_12205_amd import workloads as W
    cfg, _, _ = W.rt3d(nx=16, ny=32, nz=8)
    cfg.update(kw)
    return cfg


def test_state_bytes_layout():
    from paper_2505_12205_amd import lbm
    cfg = _cfg()
    n32 = lbm.state_bytes(cfg, "fp32")
    n16 = lbm.state_bytes(cfg, "fp16")
    N = 16 * 32 * 8
    assert n32 >= (2 * 19 * 4 + 3 * 4 + 4) * N
    assert n16 >= (2 * 19 * 2 + 3 * 4 + 8) * N
    assert n16 < n32


@pytest.mark.parametrize("bad,code", [
    (dict(q=7), -1),
    (dict(tau_h=-0.6), -1),
    (dict(xi=0.0), -1),
    (dict(rho_l=0.0), -1),
    (dict(bc=("periodic", "noslip", "noslip", "noslip", "periodic", "periodic")), -1),
    (dict(bc=("inlet", "outlet", "noslip", "noslip", "periodic", "periodic")), -5),
])
def test_invalid_parameters_rejected_on_host(bad, code):
    from paper_2505_12205_amd import lbm
    with pytest.raises(lbm.LbmError) as ei:
        lbm.state_bytes(_cfg(**bad))
    assert ei.value.code == code


@pytest.mark.parametrize("mode", ["local", "max", "average"])
def test_outlet_velocity_options_accepted(mode):
    """The three convective-velocity options of appendix B are accepted; an
    unknown one is rejected."""
    from paper_2505_12205_amd import lbm
    cfg = _cfg(bc=("periodic", "periodic", "noslip", "noslip", "inlet", "outlet"), outlet_mode=mode)
    assert lbm.state_bytes(cfg) > 0
    p = lbm.make_params(cfg)
    p.outlet_mode = 7
    n = lbm.C.c_size_t()
    assert lbm.lib.lbm_state_bytes(lbm.C.byref(p), lbm.C.byref(n)) == -1


def _declared_surrogate():
    txt = open(os.path.join(ROOT, "include", "surrogate.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sg_[a-z_0-9]+)\s*\(", txt)))


def test_surrogate_library_exports_every_declared_symbol():
    from paper_2505_12205_amd import nn
    names = _declared_surrogate()
    assert "sg_conv3d_fwd" in names and "sg_conv3d_bwd_weight" in names
    for n in names:
        assert hasattr(nn.lib, n), n
    assert set(names) == set(nn.EXPORTED)


def test_surrogate_rejects_bad_sizes_on_host():
    from paper_2505_12205_amd import nn
    # channels must be 16, 32 or 64; stride 2 with upsampling is not a form
    assert nn.lib.sg_conv3d_fwd(None, 1, 4, 4, 4, 8, None, None, 16, 1, 1, 1, None, None, None, None) == -1
    assert nn.lib.sg_conv3d_fwd(None, 1, 4, 4, 4, 16, None, None, 16, 2, 2, 1, None, None, None, None) == -1
    assert nn.lib.sg_conv3d_bwd_weight_workspace(1, 4, 4, 4, 16, 16, 2, 2) == 0
    assert nn.lib.sg_conv3d_bwd_weight_workspace(2, 8, 8, 8, 16, 32, 2, 1) > 0


def test_drops_library_exports_every_declared_symbol_and_rejects_on_host():
    from paper_2505_12205_amd import drops
    txt = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "drops.h")).read(), flags=re.S)
    names = sorted(set(re.findall(r"\b(dr_[a-z_0-9]+)\s*\(", txt)))
    assert "dr_label" in names and "dr_components" in names
    for n in names:
        assert hasattr(drops.lib, n), n
    assert set(names) == set(drops.EXPORTED)
    # extents and arguments are checked before any device call
    assert drops.lib.dr_workspace_bytes(0, 4, 4) == 0
    assert drops.lib.dr_workspace_bytes(2048, 1024, 1024) == 0  # beyond 2^30 nodes
    n = drops.lib.dr_workspace_bytes(70, 5, 4)
    assert n >= 4 * 70 * 5 * 4
    assert drops.lib.dr_label(None, 70, 5, 4, 0, 0.5, None, None, n, None) == drops.DR_EINVAL
    assert drops.lib.dr_label(1, 70, 5, 4, 8, 0.5, 1, 1, n, None) == drops.DR_EINVAL  # bad periodic bits
    assert drops.lib.dr_label(1, 70, 5, 4, 0, 0.5, 1, 1, n - 1, None) == drops.DR_EINVAL  # small workspace
    nc = C.c_int()
    assert drops.lib.dr_components(1, 70, 5, 4, 3, 8, 1, 1, 1, 1, 1, C.byref(nc), 1, n, None) == drops.DR_EINVAL


def test_probe_library_exports_every_declared_symbol_and_rejects_on_host():
    from paper_2505_12205_amd import probe
    txt = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "probe.h")).read(), flags=re.S)
    names = sorted(set(re.findall(r"\b(pb_[a-z_0-9]+)\s*\(", txt)))
    assert names == sorted(probe.EXPORTED)
    for n in names:
        assert hasattr(probe.lib, n), n
    ms = C.c_double()
    # arguments are checked before any device call
    assert probe.lib.pb_stream(4, 1, 1, 1024, 0, 1, None, C.byref(ms)) == -1   # unknown kind
    assert probe.lib.pb_stream(0, 1, 1, 1022, 0, 1, None, C.byref(ms)) == -1   # n not a multiple of 4
    assert probe.lib.pb_stream(0, 1, None, 1024, 0, 1, None, C.byref(ms)) == -1  # copy without dst
    assert probe.lib.pb_stream(3, 1, None, 19 * 64, 7, 1, None, C.byref(ms)) == -1  # q not 19 or 38
    assert probe.lib.pb_stream(3, 1, None, 1024, 38, 1, None, C.byref(ms)) == -1  # 38 does not divide 1024
    assert probe.lib.pb_stream(0, 1, 1, 1024, 0, 0, None, C.byref(ms)) == -1   # no passes
    assert b"bad argument" in probe.lib.pb_last_error() or b"q must" in probe.lib.pb_last_error()


def test_batch_layout_and_validation_on_host():
    """lbm_batch_state_bytes: the sum of the domains' 256-byte aligned
    layouts; batches of mixed lattice or storage, and empty ones, are
    rejected before any device call."""
    from paper_2505_12205_amd import lbm
    from paper_2505_12205_amd import workloads as W
    doms = [W.jet3d(nx=16, ny=16, nz=nz, radius=4.0) for nz in (24, 40)]
    arr = (lbm.Params * 2)(*[lbm.make_params(d[0], "fp16") for d in doms])
    n = C.c_size_t()
    assert lbm.lib.lbm_batch_state_bytes(2, arr, C.byref(n)) == 0
    each = [lbm.state_bytes(d[0], "fp16") for d in doms]
    assert n.value >= sum(each) and n.value <= sum(each) + 2 * 256
    mixed = (lbm.Params * 2)(lbm.make_params(doms[0][0], "fp16"), lbm.make_params(doms[1][0], "fp32"))
    assert lbm.lib.lbm_batch_state_bytes(2, mixed, C.byref(n)) == -1
    d2, _, _ = W.drop2d(n=16)
    mixed = (lbm.Params * 2)(lbm.make_params(doms[0][0], "fp32"), lbm.make_params(d2, "fp32"))
    assert lbm.lib.lbm_batch_state_bytes(2, mixed, C.byref(n)) == -1
    assert lbm.lib.lbm_batch_state_bytes(0, arr, C.byref(n)) == -1
    # one collision operator per batch
    mixed = (lbm.Params * 2)(lbm.make_params(doms[0][0], "fp16"),
                             lbm.make_params(dict(doms[1][0], collision="bgk"), "fp16"))
    assert lbm.lib.lbm_batch_state_bytes(2, mixed, C.byref(n)) == -1
    assert b"collision operator" in lbm.lib.lbm_last_error()
    both = (lbm.Params * 2)(*[lbm.make_params(dict(d[0], collision="bgk"), "fp16") for d in doms])
    assert lbm.lib.lbm_batch_state_bytes(2, both, C.byref(n)) == 0


def test_collision_operator_selection_on_host():
    """cfg["collision"] sets the BGK variant flag; unknown names and unknown
    flag bits are rejected."""
    from paper_2505_12205_amd import lbm
    from paper_2505_12205_amd import workloads as W
    cfg, _, _ = W.drop2d(n=16)
    assert lbm.make_params(cfg).variant_flags == 0
    assert lbm.make_params(dict(cfg, collision="bgk")).variant_flags == lbm.VF_BGK
    assert lbm.make_params(dict(cfg, collision="bgk", clamp_phi=True)).variant_flags == lbm.VF_BGK | lbm.VF_CLAMP_PHI
    with pytest.raises(ValueError):
        lbm.make_params(dict(cfg, collision="mrt"))
    p = lbm.make_params(cfg)
    p.variant_flags = 4
    n = C.c_size_t()
    assert lbm.lib.lbm_state_bytes(C.byref(p), C.byref(n)) == -1


def test_regime_helpers():
    """Intact length of coarse phase fields and the critical Weber split."""
    import numpy as np

    from paper_2505_12205_amd.train_surrogate import critical_weber, intact_length
    phi = np.zeros((3, 10, 3, 3))
    phi[0, :4, 1, 1] = 1.0     # 4 planes, then a gap, then a detached drop
    phi[0, 6:8, 1, 1] = 1.0
    phi[1, :, 0, 0] = 0.9      # liquid through the whole window
    phi[2, 0, 1, 1] = 0.4      # below the threshold: no liquid
    assert list(intact_length(phi)) == [8, 20, 0]   # fine units: 2 per coarse plane
    we = np.array([0.5, 1.0, 2.0, 4.0, 8.0])
    assert abs(critical_weber(we, np.array([0, 0, 1, 1, 1])) - np.sqrt(2.0)) < 1e-12
    assert critical_weber(we, np.array([1, 1, 1, 1, 1])) == 0.5
    # one outlier: the split with the fewest misclassified domains
    assert abs(critical_weber(we, np.array([0, 1, 0, 1, 1])) - np.sqrt(0.5)) < 1e-12
