"""Seeded synthetic inputs for the pressure-correction step.

This module only draws and lays out input fields: grids, a diffuse-interface
phase field of spheres, the density mapped linearly over it, predicted
staggered velocities, an extrapolated-pressure stand-in p*, the time step and
rho0.  It holds none of the step's own arithmetic, and it is the only code the
GPU path and the CPU oracle have in common.

The paper (CaNS-Fizzy) measures on bubbles and droplets in turbulence and on a
weak-scaling emulsion case with no public dataset; these seeded fields stand in
for them, with the shapes, sizes and value distributions of those workloads.

Storage: C-contiguous ``[k][j][i]`` float64; ``u[k][j][i]`` on the +x face of
cell i, ``v`` on +y, ``w`` on +z.  In a wall direction the last face index is
the wall face and is set to 0.  bc codes: 0 periodic, 1 wall.

Recipes (one ``numpy.random.Generator(PCG64(seed))`` per case, draws in the
order listed in each function):
  * phase field  phi = max_b 1/2 [1 + tanh((R_b - d_b) / (2 eps))], eps = dx/2,
    minimum-image distances in periodic directions, and phi = 0 exactly where
    (R_b - d_b)/(2 eps) < -20 for every bubble;
  * density rho = rho_l + (rho_g - rho_l) phi (phi = 1 inside a bubble/drop);
  * rho0 = min(rho); dt = (8/15) * 0.5 * h_min / max|u*|,
    h_min = min(dx, dy, min dzf);
  * p* has its volume-weighted mean removed.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

PERIODIC, WALL = 0, 1


@dataclass
class GridSpec:
    nx: int
    ny: int
    nz: int
    lx: float
    ly: float
    zf: np.ndarray
    bcx: int = PERIODIC
    bcy: int = PERIODIC
    bcz: int = WALL

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def dx(self):
        return self.lx / self.nx

    @property
    def dy(self):
        return self.ly / self.ny

    @property
    def lz(self):
        return float(self.zf[-1] - self.zf[0])

    @property
    def cells(self):
        return self.nx * self.ny * self.nz


@dataclass
class Case:
    name: str
    grid: GridSpec
    dt: float
    rho0: float
    rho: np.ndarray
    pstar: np.ndarray
    u: np.ndarray
    v: np.ndarray
    w: np.ndarray
    meta: dict = field(default_factory=dict)

    def fields(self):
        return self.rho, self.pstar, self.u, self.v, self.w


# ------------------------------------------------------------------ z grids

def zf_uniform(nz: int, lz: float) -> np.ndarray:
    return np.arange(nz + 1, dtype=np.float64) * (lz / nz)


def zf_tanh(nz: int, lz: float, a: float = 1.8) -> np.ndarray:
    """Two-sided tanh clustering towards both walls (stretch factor a)."""
    s = np.arange(nz + 1, dtype=np.float64) / nz
    zf = lz * 0.5 * (1.0 + np.tanh(a * (s - 0.5)) / math.tanh(a / 2.0))
    zf[0], zf[-1] = 0.0, lz
    return zf


def _centres(g: GridSpec):
    x = (np.arange(g.nx) + 0.5) * g.dx
    y = (np.arange(g.ny) + 0.5) * g.dy
    zc = 0.5 * (g.zf[:-1] + g.zf[1:])
    return x, y, zc


# ------------------------------------------------------------- phase field

def _axis_window(c, half, pos, n, L, periodic):
    """Indices of cells whose centre lies within `half` of c, plus the signed
    (minimum-image) distances of those centres from c."""
    if periodic:
        d = (pos - c + 0.5 * L) % L - 0.5 * L
    else:
        d = pos - c
    idx = np.nonzero(np.abs(d) <= half)[0]
    return idx, d[idx]


def phase_field(g: GridSpec, bubbles, cutoff: float = 20.0) -> np.ndarray:
    """phi of a set of spheres (cx, cy, cz, R) with eps = dx/2."""
    eps = 0.5 * g.dx
    x, y, zc = _centres(g)
    phi = np.zeros(g.shape)
    for (cx, cy, cz, R) in bubbles:
        half = R + cutoff * 2.0 * eps
        ii, dxs = _axis_window(cx, half, x, g.nx, g.lx, g.bcx == PERIODIC)
        jj, dys = _axis_window(cy, half, y, g.ny, g.ly, g.bcy == PERIODIC)
        kk, dzs = _axis_window(cz, half, zc, g.nz, g.lz, g.bcz == PERIODIC)
        if len(ii) == 0 or len(jj) == 0 or len(kk) == 0:
            continue
        d = np.sqrt(dzs[:, None, None] ** 2 + dys[None, :, None] ** 2 + dxs[None, None, :] ** 2)
        arg = (R - d) / (2.0 * eps)
        pb = np.where(arg < -cutoff, 0.0, 0.5 * (1.0 + np.tanh(arg)))
        sub = np.ix_(kk, jj, ii)
        phi[sub] = np.maximum(phi[sub], pb)
    return phi


def place_bubbles(rng, g: GridSpec, radii, gap_cells: float = 4.0, wall_cells: float = 3.0,
                  max_tries: int = 20000):
    """Seeded non-overlapping placement by rejection: centre distance at least
    R_a + R_b + gap_cells*dx, and at least R + wall_cells*dx from every wall."""
    h = g.dx
    L = np.array([g.lx, g.ly, g.lz])
    per = np.array([g.bcx == PERIODIC, g.bcy == PERIODIC, g.bcz == PERIODIC])
    lo0 = np.array([0.0, 0.0, float(g.zf[0])])
    placed = []
    tries = 0
    for R in radii:
        ok = False
        while tries < max_tries and not ok:
            tries += 1
            lo = np.where(per, lo0, lo0 + R + wall_cells * h)
            hi = np.where(per, lo0 + L, lo0 + L - R - wall_cells * h)
            if np.any(hi <= lo):
                return placed
            c = lo + rng.random(3) * (hi - lo)
            if placed:
                P = np.array(placed)
                d = P[:, :3] - c
                d = np.where(per, (d + 0.5 * L) % L - 0.5 * L, d)
                dist = np.sqrt((d ** 2).sum(axis=1))
                if np.any(dist < P[:, 3] + R + gap_cells * h):
                    continue
            placed.append([c[0], c[1], c[2], R])
            ok = True
        if not ok:
            break
    return placed


# ----------------------------------------------------------------- helpers

def zero_wall_faces(g: GridSpec, u, v, w):
    if g.bcx == WALL:
        u[:, :, -1] = 0.0
    if g.bcy == WALL:
        v[:, -1, :] = 0.0
    if g.bcz == WALL:
        w[-1, :, :] = 0.0


def remove_volume_mean(g: GridSpec, q):
    dzf = np.diff(g.zf)
    m = float((q.sum(axis=(1, 2)) * dzf).sum() / (g.nx * g.ny * g.lz))
    q -= m
    return q


def dt_rule(g: GridSpec, u, v, w):
    hmin = min(g.dx, g.dy, float(np.diff(g.zf).min()))
    umax = max(float(np.abs(u).max()), float(np.abs(v).max()), float(np.abs(w).max()))
    return (8.0 / 15.0) * 0.5 * hmin / umax


def smooth_pstar(rng, g: GridSpec, nmodes: int = 32, kmax: int = 4, kzmax: int = 4):
    """sum_n a_n cos(kx x + ky y + ph_n) Z_n(z); Z_n = cos(pi kz z / lz) for a
    wall z, cos(2 pi kz z / lz) for a periodic z.  Draws: a, ix, iy, iz, ph."""
    a = rng.standard_normal(nmodes)
    ix = rng.integers(-kmax, kmax + 1, nmodes)
    iy = rng.integers(-kmax, kmax + 1, nmodes)
    iz = rng.integers(0, kzmax + 1, nmodes)
    ph = rng.uniform(0.0, 2.0 * math.pi, nmodes)
    x, y, zc = _centres(g)
    zeta = (zc - g.zf[0]) / g.lz
    zmul = math.pi if g.bcz == WALL else 2.0 * math.pi
    planes = {}
    for n in range(nmodes):
        kx = 2.0 * math.pi * ix[n] / g.lx
        ky = 2.0 * math.pi * iy[n] / g.ly
        pl = a[n] * np.cos(kx * x[None, :] + ky * y[:, None] + ph[n])
        planes[int(iz[n])] = planes.get(int(iz[n]), 0.0) + pl
    p = np.zeros(g.shape)
    for kz, pl in sorted(planes.items()):
        zf_ = np.cos(zmul * kz * zeta)
        p += zf_[:, None, None] * pl[None, :, :]
    return remove_volume_mean(g, p)


def _finish(name, g, rho, pstar, u, v, w, meta):
    zero_wall_faces(g, u, v, w)
    dt = dt_rule(g, u, v, w)
    rho0 = float(rho.min())
    return Case(name, g, dt, rho0, rho, pstar, u, v, w, meta)


# ----------------------------------------------------------------- configs

def config0(seed: int = 1000) -> Case:
    """32^3, unit box, x/y periodic, walls in z (uniform); one sphere R = 0.25
    at the centre; rho_l = 1000, rho_g = 1; u, v, w ~ U(-1, 1); p* ~ N(0, 1).
    Draws: u, v, w, p*."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = 32
    g = GridSpec(n, n, n, 1.0, 1.0, zf_uniform(n, 1.0), PERIODIC, PERIODIC, WALL)
    phi = phase_field(g, [(0.5, 0.5, 0.5, 0.25)])
    rho = 1000.0 + (1.0 - 1000.0) * phi
    u = rng.uniform(-1.0, 1.0, g.shape)
    v = rng.uniform(-1.0, 1.0, g.shape)
    w = rng.uniform(-1.0, 1.0, g.shape)
    pstar = remove_volume_mean(g, rng.standard_normal(g.shape))
    return _finish("config0_32^3_fp64_wallz", g, rho, pstar, u, v, w, {"bubbles": 1})


def channel_bubbles(n: int, nbub: int, seed: int, name: str) -> Case:
    """n^3 cells, 2pi x 2pi x 2, x/y periodic, walls in z on a tanh grid
    (a = 1.8); nbub spheres of R = 8 dx at seeded non-overlapping positions;
    density ratio 1000; u = 1 - (z-1)^2 + N(0, 0.1), v, w ~ N(0, 0.1);
    smooth random p*.  Draws: centres, u noise, v, w, p* modes."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g = GridSpec(n, n, n, 2.0 * math.pi, 2.0 * math.pi, zf_tanh(n, 2.0, 1.8), PERIODIC, PERIODIC, WALL)
    R = 8.0 * g.dx
    bub = place_bubbles(rng, g, [R] * nbub)
    phi = phase_field(g, bub)
    rho = 1000.0 + (1.0 - 1000.0) * phi
    del phi
    _, _, zc = _centres(g)
    u = rng.normal(0.0, 0.1, g.shape)
    u += (1.0 - (zc - 1.0) ** 2)[:, None, None]
    v = rng.normal(0.0, 0.1, g.shape)
    w = rng.normal(0.0, 0.1, g.shape)
    pstar = smooth_pstar(rng, g)
    return _finish(name, g, rho, pstar, u, v, w, {"bubbles": len(bub)})


def config1(seed: int = 1001) -> Case:
    """256^3 wall-bounded channel with 64 bubbles (density ratio 1000)."""
    return channel_bubbles(256, 64, seed, "config1_256^3_fp64_wallz_tanh")


def config3(seed: int = 1003) -> Case:
    """512^3 wall-bounded channel with 512 bubbles (density ratio 1000)."""
    return channel_bubbles(512, 512, seed, "config3_512^3_wallz_tanh")


def solenoidal_velocity(rng, g: GridSpec, kmax: float = 32.0, kmin: float = 1.0):
    """Random-phase Fourier velocity with 1 <= |k| <= kmax (physical
    wavenumbers, multiples of 2 pi / L per axis), |u_k| = |k|^(-11/6) so the
    shell spectrum goes as k^(-5/3), each mode's complex amplitude drawn
    N(0,1)+iN(0,1) per component and projected perpendicular to k (solenoidal
    in the continuum).  The field is the real part of the mode sum (the
    Hermitian-symmetrised spectrum), sampled at the staggered face positions,
    so the discrete divergence is not zero.  Scaled to rms 1 over the three
    components.  Evaluated as a pruned inverse DFT in three stages (x, then
    y, then z) since only the few modes inside the shell are non-zero.
    Draws: the amplitudes, in (kz, ky, kx) order, real parts then imaginary."""
    ax = []
    for n, L in ((g.nz, g.lz), (g.ny, g.ly), (g.nx, g.lx)):
        step = 2.0 * math.pi / L
        m = min(int(math.floor(kmax / step + 1e-12)), n // 2 - 1)
        ax.append(np.arange(-m, m + 1) * step)
    kz, ky, kx = ax
    K = np.stack(np.meshgrid(kz, ky, kx, indexing="ij"), axis=-1)[..., ::-1]  # (kx, ky, kz) per mode
    kk = np.sqrt((K ** 2).sum(axis=-1))
    shell = (kk >= kmin - 1e-12) & (kk <= kmax + 1e-12)
    a = rng.standard_normal(K.shape) + 1j * rng.standard_normal(K.shape)
    with np.errstate(invalid="ignore", divide="ignore"):
        kh = np.where(shell[..., None], K / np.where(shell, kk, 1.0)[..., None], 0.0)
        a = a - kh * (kh * a).sum(axis=-1, keepdims=True)
        norm = np.sqrt((np.abs(a) ** 2).sum(axis=-1))
        amp = np.where(shell, np.where(shell, kk, 1.0) ** (-11.0 / 6.0) / np.where(norm > 0, norm, 1.0), 0.0)
    coef = a * amp[..., None]                        # (nkz, nky, nkx, 3)
    x, y, zc = _centres(g)
    xf = (np.arange(g.nx) + 1.0) * g.dx
    yf = (np.arange(g.ny) + 1.0) * g.dy
    zfc = g.zf[1:] - g.zf[0]
    zc = zc - g.zf[0]
    out = []
    for comp, (xs, ys, zs) in enumerate(((xf, y, zc), (x, yf, zc), (x, y, zfc))):
        C = coef[..., comp]
        A = C.reshape(-1, len(kx)) @ np.exp(1j * np.outer(kx, xs))                 # (nkz*nky, nx)
        B = np.exp(1j * np.outer(ys, ky))[None] @ A.reshape(len(kz), len(ky), -1)  # (nkz, ny, nx)
        B = B.reshape(len(kz), -1)
        Br, Bi = np.ascontiguousarray(B.real), np.ascontiguousarray(B.imag)
        del A, B
        Ez = np.exp(1j * np.outer(zs, kz))                                          # (nz, nkz)
        Er, Ei = np.ascontiguousarray(Ez.real), np.ascontiguousarray(Ez.imag)
        f = np.empty((g.nz, g.ny * g.nx))
        step = 1 << 16
        for c0 in range(0, f.shape[1], step):
            f[:, c0:c0 + step] = Er @ Br[:, c0:c0 + step]
            f[:, c0:c0 + step] -= Ei @ Bi[:, c0:c0 + step]
        del Br, Bi
        out.append(f.reshape(g.shape))
    rms = math.sqrt(sum(float(np.square(c).mean()) for c in out) / 3.0)
    for c in out:
        c /= rms
    return out


def emulsion(nx: int, ny: int, nz: int, ndrops: int, seed: int, name: str, kmax: float = 32.0,
             rlo: float = 4.0, rhi: float = 12.0) -> Case:
    """Triply periodic emulsion in a 2pi x 2pi x pi box (uniform grid when
    nx = ny = 2 nz): ndrops drops with R ~ U[rlo, rhi] dx at seeded
    non-overlapping positions; carrier rho = 10, drop rho = 1; solenoidal
    random-phase velocity with a k^-5/3 shell spectrum for 1 <= |k| <= kmax,
    rms 1; smooth random p* periodic in z.
    Draws: radii, centres, velocity amplitudes, p* modes."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g = GridSpec(nx, ny, nz, 2.0 * math.pi, 2.0 * math.pi, zf_uniform(nz, math.pi), PERIODIC, PERIODIC,
                 PERIODIC)
    radii = list(rng.uniform(rlo, rhi, ndrops) * g.dx)
    bub = place_bubbles(rng, g, radii, max_tries=200000)
    phi = phase_field(g, bub)
    rho = 10.0 + (1.0 - 10.0) * phi
    del phi
    u, v, w = solenoidal_velocity(rng, g, kmax)
    pstar = smooth_pstar(rng, g)
    return _finish(name, g, rho, pstar, u, v, w, {"drops": len(bub)})


def config2(seed: int = 1002) -> Case:
    """1024 x 1024 x 512 triply periodic emulsion: 2000 drops, R ~ U[4, 12] dx,
    density ratio 10, k^-5/3 solenoidal velocity for 1 <= |k| <= 32."""
    return emulsion(1024, 1024, 512, 2000, seed, "config2_1024x1024x512_triply_periodic")


def random_case(seed, nx, ny, nz, bcx=PERIODIC, bcy=PERIODIC, bcz=WALL, stretch=0.0,
                nbub=3, ratio=1000.0, lx=None, ly=None, lz=None) -> Case:
    """Small seeded case of any size/BC for parity tests: a few bubbles,
    u, v, w ~ U(-1, 1), p* ~ N(0, 1).  Draws: radii, centres, u, v, w, p*."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lx = nx / 32.0 if lx is None else lx
    ly = ny / 32.0 if ly is None else ly
    lz = nz / 32.0 if lz is None else lz
    zf = zf_tanh(nz, lz, stretch) if stretch > 0 else zf_uniform(nz, lz)
    g = GridSpec(nx, ny, nz, lx, ly, zf, bcx, bcy, bcz)
    h = g.dx
    rmax = max(1.5, min(nx, ny, nz) / 6.0)
    radii = rng.uniform(1.5, rmax, nbub) * h
    bub = place_bubbles(rng, g, list(radii), gap_cells=2.0, wall_cells=1.0, max_tries=2000)
    phi = phase_field(g, bub)
    rho = ratio + (1.0 - ratio) * phi
    u = rng.uniform(-1.0, 1.0, g.shape)
    v = rng.uniform(-1.0, 1.0, g.shape)
    w = rng.uniform(-1.0, 1.0, g.shape)
    pstar = remove_volume_mean(g, rng.standard_normal(g.shape))
    return _finish(f"random_{nx}x{ny}x{nz}_bc{bcx}{bcy}{bcz}_s{stretch}", g, rho, pstar, u, v, w,
                   {"bubbles": len(bub)})


BATCH_XY = (32, 48, 64, 96, 128)
BATCH_Z = (32, 64, 96)


def config4(seed: int = 1004, ndom: int = 192):
    """Batch of ndom independent domains: nx, ny drawn from BATCH_XY and nz
    from BATCH_Z; box = n/32 (h = 1/32); x, y periodic; half periodic-z and
    half wall-z by a seeded permutation; uniform z; 1-8 bubbles with
    R ~ U[3, max(3, min(n)/6)] h; density ratio log-uniform in [10, 1000],
    rho_g = 1; u, v, w ~ U(-1, 1); p* ~ N(0, 1).
    Draws: nx[], ny[], nz[], bc permutation, then per domain: nbub, ratio,
    radii, centres, u, v, w, p*."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nxs = rng.choice(BATCH_XY, ndom)
    nys = rng.choice(BATCH_XY, ndom)
    nzs = rng.choice(BATCH_Z, ndom)
    bcz = np.zeros(ndom, dtype=int)
    bcz[rng.permutation(ndom)[: ndom // 2]] = WALL
    cases = []
    for d in range(ndom):
        nx, ny, nz = int(nxs[d]), int(nys[d]), int(nzs[d])
        g = GridSpec(nx, ny, nz, nx / 32.0, ny / 32.0, zf_uniform(nz, nz / 32.0), PERIODIC, PERIODIC,
                     int(bcz[d]))
        nb = int(rng.integers(1, 9))
        ratio = float(math.exp(rng.uniform(math.log(10.0), math.log(1000.0))))
        rmax = max(3.0, min(nx, ny, nz) / 6.0)
        radii = list(rng.uniform(3.0, rmax, nb) / 32.0)
        bub = place_bubbles(rng, g, radii, max_tries=2000)
        phi = phase_field(g, bub)
        rho = ratio + (1.0 - ratio) * phi
        u = rng.uniform(-1.0, 1.0, g.shape)
        v = rng.uniform(-1.0, 1.0, g.shape)
        w = rng.uniform(-1.0, 1.0, g.shape)
        pstar = remove_volume_mean(g, rng.standard_normal(g.shape))
        cases.append(_finish(f"batch{d}_{nx}x{ny}x{nz}_bcz{int(bcz[d])}", g, rho, pstar, u, v, w,
                             {"bubbles": len(bub), "ratio": ratio}))
    return cases


def fingerprint(case: Case) -> str:
    """SHA-256 over the raw bytes of every input array plus dt and rho0."""
    import hashlib
    h = hashlib.sha256()
    for a in (case.grid.zf,) + case.fields():
        h.update(np.ascontiguousarray(a).tobytes())
    h.update(np.float64(case.dt).tobytes())
    h.update(np.float64(case.rho0).tobytes())
    return h.hexdigest()
