"""Pins of the Dirichlet (sine-transform) variants of the constant-
coefficient Poisson oracle (oracle/dirichlet.c): the discrete eigenvectors
of each boundary condition with their closed-form eigenvalues, a dense
solve of the assembled operator on tiny grids of every combination, the
operator's agreement with the wall/periodic oracle where both apply,
symmetry, and a library sine transform.  No GPU."""
import itertools
import math

import numpy as np
import pytest
import scipy.fft

from paper_2502_04189_amd import workloads as W


def grid(orc, nx, ny, nz, bc, stretch=0.0, lx=1.0, ly=0.8, lz=0.9):
    zf = W.zf_tanh(nz, lz, stretch) if stretch > 0 else W.zf_uniform(nz, lz)
    return orc.Grid(nx, ny, nz, lx, ly, zf, *bc)


def mode(n, bc, l):
    x = np.arange(n)
    if bc == 0:
        return np.cos(2 * math.pi * l * x / n)  # the real part of the exponential (l and n - l share lambda)
    if bc == 1:
        return np.cos(math.pi * l * (x + 0.5) / n)
    return np.sin(math.pi * (l + 1) * (x + 0.5) / n)


ALL = list(itertools.product((0, 1, 2), repeat=3))
WITH_D = [b for b in ALL if 2 in b]


@pytest.mark.parametrize("bc", ALL)
def test_eigenvectors_with_closed_form_eigenvalues(orc, bc):
    """On a uniform grid the product of the directions' modes is an
    eigenvector of the operator with the sum of the closed-form
    eigenvalues; L applied to it, and (with a Dirichlet direction) the
    solve, reproduce that exactly up to rounding."""
    n = (8, 6, 5)
    g = grid(orc, *n, bc)
    h = (1.0 / 8, 0.8 / 6, 0.9 / 5)
    rng = np.random.default_rng(sum(bc))
    for _ in range(4):
        ls = [int(rng.integers(0, n[d])) for d in range(3)]
        v = mode(n[2], bc[2], ls[2])[:, None, None] * mode(n[1], bc[1], ls[1])[None, :, None] * \
            mode(n[0], bc[0], ls[0])[None, None, :]
        lam = sum(orc.eig_bc(n[d], h[d], bc[d], ls[d]) for d in range(3))
        Lv = orc.apply_L_bc(g, v)
        assert np.abs(Lv - lam * v).max() <= 1e-12 * max(abs(lam), 1.0)
        if 2 in bc:
            p = orc.poisson_bc(g, lam * v)
            assert np.abs(p - v).max() <= 1e-12


@pytest.mark.parametrize("bc", WITH_D)
@pytest.mark.parametrize("stretch", [0.0, 1.4])
def test_dense_solve_of_the_assembled_operator(orc, bc, stretch):
    n = (4, 3, 5) if bc[1] != 0 else (4, 4, 5)
    g = grid(orc, *n, bc, stretch)
    N = n[0] * n[1] * n[2]
    A = np.empty((N, N))
    for c in range(N):
        e = np.zeros(N)
        e[c] = 1.0
        A[:, c] = orc.apply_L_bc(g, e.reshape(g.shape)).ravel()
    f = np.random.default_rng(3).normal(size=g.shape)
    want = np.linalg.solve(A, f.ravel()).reshape(g.shape)
    got = orc.poisson_bc(g, f)
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()
    if stretch == 0.0:
        # uniform spacing: the operator is symmetric and negative definite
        assert np.abs(A - A.T).max() <= 1e-12 * np.abs(A).max()
        assert np.linalg.eigvalsh(0.5 * (A + A.T)).max() < 0


@pytest.mark.parametrize("bc", [b for b in ALL if 2 not in b])
def test_operator_matches_the_wall_oracle(orc, bc):
    """Without Dirichlet directions the operator is the one oracle.c
    assembles from G and D (an independent implementation); the solve
    refers the singular case back to it."""
    g = grid(orc, 6, 4, 5, bc, 1.3)
    p = np.random.default_rng(1).normal(size=g.shape)
    assert np.abs(orc.apply_L_bc(g, p) - orc.apply_L(g, p)).max() <= 1e-12 * np.abs(orc.apply_L(g, p)).max()
    with pytest.raises(RuntimeError):
        orc.poisson_bc(g, p)


def test_sine_modes_match_a_library_sine_transform(orc):
    """The Dirichlet modes are the DST-II basis: projecting random data on
    them gives scipy's DST-II (which carries a factor 2)."""
    n = 12
    x = np.random.default_rng(2).normal(size=n)
    proj = np.array([(x * mode(n, 2, l)).sum() for l in range(n)])
    assert np.abs(2 * proj - scipy.fft.dst(x, type=2)).max() <= 1e-13 * np.abs(x).sum()
    cproj = np.array([(x * mode(n, 1, l)).sum() for l in range(n)])
    assert np.abs(2 * cproj - scipy.fft.dct(x, type=2)).max() <= 1e-13 * np.abs(x).sum()


@pytest.mark.parametrize("bc", [(2, 2, 2), (0, 2, 1), (2, 1, 0)])
def test_apply_then_solve_on_stretched_grids(orc, bc):
    g = grid(orc, 16, 12, 10, bc, 1.5)
    q = np.random.default_rng(5).normal(size=g.shape)
    p = orc.poisson_bc(g, orc.apply_L_bc(g, q))
    assert np.abs(p - q).max() <= 1e-12 * np.abs(q).max()
