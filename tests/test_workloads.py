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


def test_emulsion_recipe():
    """Small emulsion: drop count and density range, rms 1, and the velocity
    is solenoidal in the continuum with its spectrum confined to the shell:
    after undoing the half-cell sampling shifts, k . u_hat = 0 for every mode
    and u_hat = 0 outside 1 <= |k| <= kmax."""
    kmax = 8.0
    c = W.emulsion(64, 64, 32, 6, 77, "e", kmax=kmax)
    g = c.grid
    assert (g.bcx, g.bcy, g.bcz) == (0, 0, 0) and g.shape == (32, 64, 64)
    assert c.meta["drops"] == 6
    assert c.rho.max() == 10.0 and 1.0 <= c.rho.min() < 1.01 and c.rho0 == c.rho.min()
    rms = np.sqrt((np.square(c.u).mean() + np.square(c.v).mean() + np.square(c.w).mean()) / 3.0)
    assert abs(rms - 1.0) < 1e-12
    kz = np.fft.fftfreq(g.nz, d=g.lz / g.nz) * 2 * np.pi
    ky = np.fft.fftfreq(g.ny, d=g.ly / g.ny) * 2 * np.pi
    kx = np.fft.fftfreq(g.nx, d=g.lx / g.nx) * 2 * np.pi
    KZ, KY, KX = np.meshgrid(kz, ky, kx, indexing="ij")
    dz = g.lz / g.nz
    # u sampled at x + dx/2, v at y + dy/2, w at z + dz/2 relative to the centres
    U = np.fft.fftn(c.u) * np.exp(-0.5j * KX * g.dx)
    V = np.fft.fftn(c.v) * np.exp(-0.5j * KY * g.dy)
    Wf = np.fft.fftn(c.w) * np.exp(-0.5j * KZ * dz)
    kk = np.sqrt(KX ** 2 + KY ** 2 + KZ ** 2)
    amp = np.sqrt(np.abs(U) ** 2 + np.abs(V) ** 2 + np.abs(Wf) ** 2)
    inside = (kk >= 1 - 1e-9) & (kk <= kmax + 1e-9)
    assert amp[~inside].max() <= 1e-10 * amp.max()
    kdotu = np.abs(KX * U + KY * V + KZ * Wf)
    assert kdotu.max() <= 1e-10 * (kk * amp).max()
    # the discrete (staggered) divergence is not zero: the RHS velocity term is exercised
    div = ((c.u - np.roll(c.u, 1, 2)) / g.dx + (c.v - np.roll(c.v, 1, 1)) / g.dy
           + (c.w - np.roll(c.w, 1, 0)) / dz)
    assert np.abs(div).max() > 1e-6
    # shell spectrum E(k) ~ k^-5/3: least-squares slope over k = 1..kmax
    ks = np.arange(1, int(kmax) + 1)
    E = np.array([np.sum(amp[(kk >= k - 0.5) & (kk < k + 0.5)] ** 2) for k in ks])
    slope = np.polyfit(np.log(ks), np.log(E), 1)[0]
    assert -2.6 < slope < -0.8, slope
