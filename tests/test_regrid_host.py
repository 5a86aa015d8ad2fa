"""The library's host-side Berger-Rigoutsos clustering (amr_cluster_boxes,
the rule amr_regrid applies) against the oracle's own clustering: the same
boxes in the same order, on hand-made and random flag sets (no GPU)."""

import numpy as np
import pytest

from oracle import regrid as RG
from paper_1110_1616_amd import amr as A


def _same(mask, adm, eff, maxbox):
    want = RG.cluster(mask, adm if adm is not None else np.ones_like(mask), eff, maxbox)
    got = A.amr_cluster_boxes(mask, adm, eff, maxbox)
    assert got == [(tuple(lo), tuple(hi)) for lo, hi in want]
    return got


def test_l_shape_and_blocks():
    m = np.zeros((16, 16), dtype=bool)
    m[0:8, 0:2] = True
    m[0:2, 0:8] = True
    assert _same(m, None, 0.7, 16) == [((0, 0), (2, 8)), ((2, 0), (8, 2))]
    m = np.zeros((32, 16), dtype=bool)
    m[2:6, 3:9] = True
    m[20:26, 4:7] = True
    _same(m, None, 0.7, 32)
    _same(np.ones((40, 8), dtype=bool), None, 0.7, 16)


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("ndim", [2, 3])
def test_random_sets_match_the_oracle(seed, ndim):
    rng = np.random.default_rng(100 + seed)
    shape = (36, 28, 20)[:ndim]
    m = np.zeros(shape, dtype=bool)
    for _ in range(5):
        c = rng.integers(0, shape)
        r = rng.integers(1, 6, size=ndim)
        m[tuple(slice(max(c[a] - r[a], 0), c[a] + r[a]) for a in range(ndim))] = True
    m |= rng.random(shape) < 0.02
    adm = rng.random(shape) < 2.0  # all True
    adm[tuple(slice(0, 6) for _ in range(ndim))] = False
    m &= adm
    eff = (0.5, 0.7, 0.9)[seed % 3]
    got = _same(m, adm, eff, (8, 12, 16)[seed % 3])
    assert got


def test_empty_mask_gives_no_boxes():
    assert A.amr_cluster_boxes(np.zeros((8, 8), dtype=bool)) == []
