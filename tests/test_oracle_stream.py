"""Pins of streaming with mid-grid bounce-back (Sec. 2, Eq. LBeqs and the
wall model): on fluid nodes the step is a permutation of the populations;
a free population moves by exactly c_k; a population that would enter a
wall node comes back on the opposite velocity at the node it left."""
import numpy as np

import workloads as W


def _lattice(ora, nx, ny, nz, solid=None):
    return ora.Lattice(W.params(nx, ny, nz, 0.0), solid)


def test_stream_is_permutation_on_fluid(ora):
    nx, ny, nz = 6, 5, 7
    solid = W.walls_mask(nx, ny, nz)
    solid[3, 2, 4] = 1  # an isolated solid node in the bulk
    L = _lattice(ora, nx, ny, nz, solid)
    fluid = solid == 0
    rng = np.random.default_rng(1)
    n_fluid = int(fluid.sum()) * 38
    vals = rng.permutation(n_fluid).astype(np.float64) + 1.0  # distinct integers
    f = np.zeros((nz, ny, nx, 2, 19))
    f[fluid] = vals.reshape(-1, 2, 19)
    out = L.stream(f)
    assert np.all(out[~fluid] == 0.0)
    # every fluid population lands exactly once
    assert np.array_equal(np.sort(out[fluid].ravel()), np.sort(vals))
    assert out[fluid].sum() == vals.sum()


def test_free_population_moves_by_c(ora):
    c, _, _ = ora.tables()
    nx, ny, nz = 5, 6, 7
    L = _lattice(ora, nx, ny, nz)
    for k in range(19):
        f = np.zeros((nz, ny, nx, 2, 19))
        x0, y0, z0 = 4, 0, 3  # next to the periodic wrap in x and y
        f[z0, y0, x0, 1, k] = 1.0
        out = L.stream(f)
        z1, y1, x1 = (z0 + c[k, 2]) % nz, (y0 + c[k, 1]) % ny, (x0 + c[k, 0]) % nx
        assert out[z1, y1, x1, 1, k] == 1.0
        assert out.sum() == 1.0


def test_bounce_back_at_floor(ora):
    c, _, opp = ora.tables()
    nx, ny, nz = 4, 4, 6
    solid = W.walls_mask(nx, ny, nz)
    L = _lattice(ora, nx, ny, nz, solid)
    for k in range(19):
        f = np.zeros((nz, ny, nx, 2, 19))
        f[1, 2, 2, 0, k] = 1.0
        out = L.stream(f)
        if c[k, 2] == -1:  # heads into the floor: reflected in place
            assert out[1, 2, 2, 0, opp[k]] == 1.0
        else:
            z1, y1, x1 = 1 + c[k, 2], (2 + c[k, 1]) % ny, (2 + c[k, 0]) % nx
            assert out[z1, y1, x1, 0, k] == 1.0
        assert out.sum() == 1.0
