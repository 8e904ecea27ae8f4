"""The allocation-free batch reduction (lbm_batch_reduce_noalloc, called
through the C ABI) against lbm_batch_reduce on the same batches: two calls in
a row, the second on a smaller batch, so the shared static scratch array is
reused with fewer partial sums."""
import sys

import numpy as np
import pytest

from paper_2505_12205_amd import workloads as W

pytestmark = pytest.mark.gpu


def _batch(shapes, seed):
    import torch
    if not torch.cuda.is_available():
        pytest.fail("a GPU test ran without a GPU")
    from paper_2505_12205_amd import lbm
    doms = []
    for k, (nx, ny, nz) in enumerate(shapes):
        cfg, phi0, u0 = W.rt3d(nx=nx, ny=ny, nz=nz, lref=256)
        phi0, u0 = W.perturb(phi0, u0, seed + k, 0.01, 1e-3)
        doms.append((cfg, phi0, u0))
    return lbm.Batch(doms)


@pytest.mark.parametrize("steps", [7, 12])
def test_noalloc_reduce_matches_batch_reduce(steps):
    import torch
    for shapes, seed in (([(32, 48, 16), (48, 64, 24), (16, 40, 8)], 11), ([(16, 24, 8), (24, 16, 12)], 29)):
        print(f"[gpu] noalloc reduce: {len(shapes)} domains {shapes}", flush=True)
        sys.stdout.flush()
        b = _batch(shapes, seed).step(steps)
        out = torch.full((2 * b.ndom,), float("nan"), dtype=torch.float64, device=b.device)
        b.reduce_noalloc(out)
        b.stream.synchronize()
        got = out.cpu().numpy()
        m, k = b.reduce()
        ref = np.stack([np.array(m), np.array(k)], axis=1).reshape(-1)
        print(f"noalloc {got.tolist()} reduce {ref.tolist()}", flush=True)
        assert np.all(np.isfinite(got))
        assert np.array_equal(got, ref)
