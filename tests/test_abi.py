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
    (dict(bc=("periodic", "periodic", "noslip", "noslip", "inlet", "outlet"), outlet_mode="max"), -5),
])
def test_invalid_parameters_rejected_on_host(bad, code):
    from paper_2505_12205_amd import lbm
    with pytest.raises(lbm.LbmError) as ei:
        lbm.state_bytes(_cfg(**bad))
    assert ei.value.code == code


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
