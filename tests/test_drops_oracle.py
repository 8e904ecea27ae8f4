"""Pins of the drop-size oracle (oracle/drops.c): the labelling against
scipy.ndimage.label (face connectivity) and its canonical form (each label
the smallest node index of its component), periodic wrap against the shift
invariance of the partition and a bar across the boundary, the component
statistics against an independent numpy evaluation, balls of known volume,
and the degenerate fields."""
import numpy as np
import pytest
from scipy import ndimage

import oracle


def _field(shape, frac, seed, smooth=1.0):
    """A smooth random field; the level frac of its distribution is the
    threshold 1/2 after shifting, so about frac of the nodes are liquid."""
    rng = np.random.default_rng(seed)
    f = ndimage.gaussian_filter(rng.standard_normal(shape), smooth, mode="wrap")
    return (f - np.quantile(f, 1.0 - frac) + 0.5).astype(np.float32)


def _same_partition(a, b):
    """Labellings a, b (-1 = background) define the same partition."""
    if not np.array_equal(a < 0, b < 0):
        return False
    fa, fb = a[a >= 0], b[b >= 0]
    pairs = np.unique(np.stack([fa, fb]), axis=1)
    return len(np.unique(pairs[0])) == pairs.shape[1] == len(np.unique(pairs[1]))


def _min_index_labels(scipy_lab):
    idx = np.arange(scipy_lab.size).reshape(scipy_lab.shape)
    n = scipy_lab.max()
    mins = ndimage.minimum(idx, scipy_lab, index=np.arange(1, n + 1)).astype(np.int64)
    out = np.full(scipy_lab.shape, -1, np.int64)
    out[scipy_lab > 0] = mins[scipy_lab[scipy_lab > 0] - 1]
    return out


@pytest.mark.parametrize("shape,frac,seed", [((9, 13, 17), 0.3, 1), ((12, 10, 31), 0.15, 2),
                                             ((6, 7, 8), 0.5, 3), ((20, 20, 20), 0.25, 4)])
def test_label_matches_scipy_face_connectivity(shape, frac, seed):
    phi = _field(shape, frac, seed)
    lab = oracle.label(phi)
    ref, n = ndimage.label(phi > np.float32(0.5), structure=ndimage.generate_binary_structure(3, 1))
    assert n > 1
    assert _same_partition(lab, np.where(ref > 0, ref, -1))
    assert np.array_equal(lab, _min_index_labels(ref))


def test_label_2d_is_four_connected():
    phi = _field((1, 40, 50), 0.35, 5)
    lab = oracle.label(phi)
    ref, _ = ndimage.label(phi[0] > np.float32(0.5), structure=ndimage.generate_binary_structure(2, 1))
    assert np.array_equal(lab[0], _min_index_labels(ref))
    # diagonal neighbours are not connected
    d = np.zeros((1, 3, 3), np.float32)
    d[0, 0, 0] = d[0, 1, 1] = 1.0
    assert len(oracle.components(oracle.label(d), axis=1)["root"]) == 2


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_periodic_wrap(axis):
    shape = (8, 9, 10)
    phi = np.zeros(shape, np.float32)
    n = shape[2 - axis]
    sl = [slice(3, 5)] * 3
    for pos in (0, 1, n - 2, n - 1):  # a bar cut by the boundary of `axis`
        s = list(sl)
        s[2 - axis] = pos
        phi[tuple(s)] = 1.0
    per = [False] * 3
    assert len(oracle.components(oracle.label(phi))["root"]) == 2
    per[axis] = True
    c = oracle.components(oracle.label(phi, periodic=per))
    assert len(c["root"]) == 1 and c["size"][0] == 16


def test_periodic_partition_is_shift_invariant():
    phi = _field((10, 12, 14), 0.3, 6)
    per = (True, True, True)
    lab = oracle.label(phi, periodic=per)
    for shift in ((3, 0, 0), (0, 5, 0), (0, 0, 7), (4, 11, 2)):
        rolled = oracle.label(np.roll(phi, shift, axis=(0, 1, 2)), periodic=per)
        assert _same_partition(rolled, np.roll(lab, shift, axis=(0, 1, 2)))
    # without wrap the partition is finer or equal, never coarser
    flat = oracle.label(phi)
    assert len(np.unique(flat[flat >= 0])) >= len(np.unique(lab[lab >= 0]))


def test_component_statistics_against_numpy():
    phi = _field((11, 13, 29), 0.25, 7)
    lab = oracle.label(phi)
    for axis in (0, 1, 2):
        c = oracle.components(lab, axis=axis)
        roots = np.unique(lab[lab >= 0])
        assert np.array_equal(c["root"], roots)
        coord = np.indices(lab.shape)[2 - axis]
        for k, r in enumerate(roots):
            m = lab == r
            assert c["size"][k] == m.sum()
            assert c["lo"][k] == coord[m].min() and c["hi"][k] == coord[m].max()
        assert np.allclose(c["deq"], np.cbrt(6.0 * c["size"] / np.pi), rtol=1e-14)


def test_balls_of_known_volume():
    z, y, x = np.indices((40, 40, 64))
    phi = np.zeros(z.shape, np.float32)
    balls = [((20, 20, 14), 9.0), ((20, 20, 46), 5.5)]
    masks = []
    for (cz, cy, cx), r in balls:
        m = (x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2 <= r * r
        phi[m] = 1.0
        masks.append(m)
    c = oracle.components(oracle.label(phi), axis=0)
    assert len(c["root"]) == 2
    assert sorted(c["size"]) == sorted(int(m.sum()) for m in masks)
    for k, (cen, r) in enumerate(balls):  # ordered by root = first node in memory order
        assert abs(c["deq"][k] / (2 * r) - 1) < 0.03
        assert c["lo"][k] == cen[2] - int(r) and c["hi"][k] == cen[2] + int(r)


def test_degenerate_fields():
    empty = np.zeros((3, 4, 5), np.float32)
    assert (oracle.label(empty) == -1).all()
    assert len(oracle.components(oracle.label(empty))["root"]) == 0
    full = np.ones((3, 4, 5), np.float32)
    c = oracle.components(oracle.label(full))
    assert list(c["root"]) == [0] and c["size"][0] == 60 and c["lo"][0] == 0 and c["hi"][0] == 2
    # the threshold is strict and taken in float
    at = np.full((2, 2, 2), 0.5, np.float32)
    assert (oracle.label(at) == -1).all()
    one = np.zeros((1, 1, 1), np.float32) + 1
    assert oracle.label(one)[0, 0, 0] == 0
