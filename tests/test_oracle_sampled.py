"""The oracle's sampled-output evaluators (used by full-size GPU checks)
agree bit for bit with its whole-grid RHS and correction."""
import numpy as np
import pytest

from paper_2502_04189_amd import workloads as W


@pytest.mark.parametrize("dims,bc,stretch", [((12, 10, 8), (0, 0, 1), 1.5), ((8, 9, 6), (1, 1, 0), 0.0),
                                             ((6, 8, 7), (1, 0, 1), 1.2), ((8, 6, 5), (0, 1, 0), 0.0)])
def test_sampled_equal_whole_grid(orc, dims, bc, stretch):
    c = W.random_case(11 + sum(dims), *dims, *bc, stretch=stretch)
    g = orc.Grid.from_workload(c.grid)
    cells = np.arange(c.grid.cells)
    f = orc.rhs(g, c.dt, c.rho0, *c.fields())
    assert np.array_equal(orc.rhs_at(g, c.dt, c.rho0, *c.fields(), cells), f.ravel())
    p = np.random.default_rng(3).standard_normal(c.grid.shape)
    full = orc.correct(g, c.dt, c.rho0, *c.fields(), p)
    for d in range(3):
        got = orc.correct_at(g, c.dt, c.rho0, *c.fields(), p, np.full(len(cells), d), cells)
        assert np.array_equal(got, full[d].ravel())


def test_sampled_rejects_bad_index(orc):
    c = W.random_case(5, 6, 6, 4)
    g = orc.Grid.from_workload(c.grid)
    with pytest.raises(Exception):
        orc.rhs_at(g, c.dt, c.rho0, *c.fields(), np.array([c.grid.cells]))
    with pytest.raises(Exception):
        orc.correct_at(g, c.dt, c.rho0, *c.fields(), c.pstar, np.array([3]), np.array([0]))


@pytest.mark.parametrize("dims,bc,stretch", [((12, 10, 8), (0, 0, 1), 1.5), ((8, 9, 6), (1, 1, 0), 0.0),
                                             ((16, 8, 12), (0, 0, 0), 0.0), ((6, 8, 7), (1, 1, 1), 1.2)])
def test_torch_checkers_match_oracle(orc, dims, bc, stretch):
    """The torch RHS and divergence used by the full-size GPU checks agree
    with the oracle (run here on CPU tensors)."""
    import torch
    from tests import manufactured as M
    c = W.random_case(23 + sum(dims), *dims, *bc, stretch=stretch)
    g = orc.Grid.from_workload(c.grid)
    t = [torch.from_numpy(a) for a in c.fields()]
    f = orc.rhs(g, c.dt, c.rho0, *c.fields())
    ft = M.rhs_t(c.grid, c.dt, c.rho0, *t).numpy()
    assert np.abs(ft - f).max() <= 1e-13 * np.abs(f).max()
    d = orc.div(g, c.u, c.v, c.w)
    dt_ = M.div_t(c.grid, *t[2:]).numpy()
    assert np.abs(dt_ - d).max() <= 1e-13 * np.abs(d).max()
