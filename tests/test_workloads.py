"""Seeded input generators: determinism, shapes, recipe properties (no GPU)."""
import json
import os

import numpy as np

from paper_2502_04189_amd import workloads as W
from tests.golden.make_input_hashes import cases

HERE = os.path.dirname(os.path.abspath(__file__))


def test_input_fingerprints_are_stable():
    with open(os.path.join(HERE, "golden", "input_hashes.json")) as f:
        ref = json.load(f)
    got = {name: W.fingerprint(c) for name, c in cases()}
    assert got == ref


def test_config0_recipe():
    c = W.config0()
    g = c.grid
    assert g.shape == (32, 32, 32) and (g.bcx, g.bcy, g.bcz) == (0, 0, 1)
    assert np.all(c.w[-1] == 0.0)
    assert c.rho0 == c.rho.min() and 1.0 <= c.rho0 < 2.0 and c.rho.max() == 1000.0
    dzf = np.diff(g.zf)
    mean = (c.pstar.sum(axis=(1, 2)) * dzf).sum() / (g.nx * g.ny * g.lz)
    assert abs(mean) < 1e-15
    umax = max(np.abs(c.u).max(), np.abs(c.v).max(), np.abs(c.w).max())
    assert abs(c.dt - (8 / 15) * 0.5 * (1 / 32) / umax) < 1e-18


def test_tanh_grid():
    zf = W.zf_tanh(512, 2.0, 1.8)
    dz = np.diff(zf)
    assert zf[0] == 0.0 and zf[-1] == 2.0 and np.all(dz > 0)
    assert abs(dz.min() / (2.0 / 512) - 0.613) < 0.01 and abs(dz.max() / (2.0 / 512) - 1.256) < 0.01
    assert np.max(dz[1:] / dz[:-1]) < 1.006 and np.max(dz[:-1] / dz[1:]) < 1.006


def test_bubbles_do_not_overlap_and_respect_walls():
    rng = np.random.Generator(np.random.PCG64(3))
    g = W.GridSpec(128, 128, 128, 6.28, 6.28, W.zf_tanh(128, 2.0), 0, 0, 1)
    R = 8 * g.dx
    b = np.array(W.place_bubbles(rng, g, [R] * 6))
    assert len(b) == 6
    for i in range(len(b)):
        assert b[i, 2] - R >= 3 * g.dx - 1e-12 and g.lz - b[i, 2] - R >= 3 * g.dx - 1e-12
        for j in range(i):
            d = b[i, :3] - b[j, :3]
            d[:2] = (d[:2] + 0.5 * 6.28) % 6.28 - 0.5 * 6.28
            assert np.sqrt((d**2).sum()) >= 2 * R + 4 * g.dx - 1e-12


def test_config4_batch_mix():
    cs = W.config4(ndom=192)
    assert len(cs) == 192
    assert sum(c.grid.bcz == W.WALL for c in cs) == 96
    cells = sum(c.grid.cells for c in cs)
    assert 40e6 < cells < 90e6
    for c in cs:
        assert c.grid.nx in W.BATCH_XY and c.grid.ny in W.BATCH_XY and c.grid.nz in W.BATCH_Z
        assert 10.0 <= c.rho.max() <= 1000.0 + 1e-9 and c.rho0 >= 1.0 - 1e-12
