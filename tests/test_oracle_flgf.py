"""Pins of the two-grid fast-LGF oracle (the far-field approximation of
Sec. 2.2 / Sec. 5, read from first principles).

* the 4-point weights reproduce cubic polynomials exactly;
* anterpolation is the transpose of interpolation: <I U, f> = <U, A f>;
* with every pair near (D >= the extent) the approximation is the exact
  convolution;
* the far field is the interpolated kernel: its error falls like the
  fourth power of the near radius (cubic interpolation of a kernel whose
  derivatives fall like 1/r), measured against the direct sum.
"""
import numpy as np
import pytest

from oracle import direct, flgf


@pytest.mark.parametrize("nb", [8, 16])
def test_block_local_weights_reproduce_cubics(nb):
    for i in range(nb):
        nodes, w = flgf.node_weights(i, nb)
        assert nodes.min() >= 0 and nodes.max() < nb // 2
        x = (i + 0.5) / 2.0
        for deg in range(4):
            assert abs((w * (nodes + 0.5) ** deg).sum() - x ** deg) < 1e-12 * max(1.0, x ** deg)


def test_anterpolation_is_the_transpose_of_interpolation():
    rng = np.random.default_rng(0)
    cells = np.stack(np.meshgrid(*[np.arange(12)] * 3, indexing="ij"), -1).reshape(-1, 3) + np.array([8, -16, 4])
    f = rng.standard_normal(len(cells))
    nodes, Af = flgf.anterpolate(cells, f, 4)
    U = rng.standard_normal(len(nodes))
    lhs = (flgf.interpolate(nodes, U, cells, 4) * f).sum()
    rhs = (U * Af).sum()
    assert abs(lhs - rhs) < 1e-12 * abs(rhs)


def _problem(nb, nblk, seed):
    b = np.stack(np.meshgrid(*[np.arange(nblk)] * 3, indexing="ij"), -1).reshape(-1, 3)
    r = np.arange(nb)
    local = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3)
    cells = (b[:, None, :] * nb + local[None]).reshape(-1, 3)
    rng = np.random.default_rng(seed)
    c = cells.mean(axis=0)
    f = np.exp(-((cells - c) ** 2).sum(1) / (2 * (nb * nblk / 6.0) ** 2)) + 0.1 * rng.standard_normal(len(cells))
    return cells, f


def test_all_near_is_exact():
    cells, f = _problem(8, 3, 1)
    tgt = cells[::7]
    got = flgf.flgf(cells, f, tgt, 0.5, 8, D=2)
    ref = direct.direct_sum(cells, f, tgt, 0.5)
    assert np.abs(got - ref).max() < 1e-14 * np.abs(ref).max()


def test_far_error_falls_with_the_near_radius():
    cells, f = _problem(8, 5, 2)
    tgt = cells[np.random.default_rng(3).choice(len(cells), 48, replace=False)]
    ref = direct.direct_sum(cells, f, tgt, 1.0)
    errs = []
    for D in (1, 2, 3):
        got = flgf.flgf(cells, f, tgt, 1.0, 8, D)
        errs.append(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    print("FLGF rel L2 vs direct sum for D = 1, 2, 3:", errs)
    assert errs[2] < errs[1] < errs[0] < 1e-3, errs
