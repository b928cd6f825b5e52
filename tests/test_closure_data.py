"""Host-side bookkeeping of the closure dataset (paired fine and coarse runs;
an extension, not in arXiv:2211.06142): cell lookup, target ratios and their
clipping, row assembly, the normaliser, the pull-off density of bonded
contacts, and the initial parameters.  No GPU."""
import math

import numpy as np
import pytest

from paper_2211_06142_amd import closure_train as ct

GRID = ((0.0, 0.0, 0.0), (4.0, 2.0, 1.0), (4, 2, 2))   # cells 1 x 1 x 0.5


def test_cell_index_x_fastest_and_outside():
    x = np.array([[0.5, 0.5, 0.25], [1.5, 0.5, 0.25], [0.5, 1.5, 0.25], [0.5, 0.5, 0.75], [3.9, 1.9, 0.99],
                  [-0.1, 0.5, 0.5], [0.5, 2.0, 0.5], [0.5, 0.5, 1.0]])
    np.testing.assert_array_equal(ct.cell_index(x, GRID), [0, 1, 4, 8, 15, -1, -1, -1])


def test_log_ratio_clips_to_the_closure_range_and_masks():
    fine = np.array([1.0, 8.0, 1.0, 2.0, 0.0, 3.0])
    coarse = np.array([2.0, 1.0, 8.0, 1.0, 1.0, 3.0])
    valid = np.array([True, True, True, True, True, False])
    y = ct.log_ratio(fine, coarse, valid)
    assert y[0] == pytest.approx(-math.log(2.0))
    assert y[1] == pytest.approx(math.log(2.0))       # ln 8 clipped
    assert y[2] == pytest.approx(-math.log(2.0))      # -ln 8 clipped
    assert y[3] == pytest.approx(math.log(2.0))
    assert np.isnan(y[4]) and np.isnan(y[5])          # zero fine value; invalid cell


def test_assemble_keeps_parcels_of_cells_with_both_targets():
    feats = np.arange(5 * 6, dtype=float).reshape(5, 6)
    cells = np.array([0, 1, 2, -1, 1])
    yd = np.array([0.1, 0.2, np.nan])
    yc = np.array([0.3, 0.4, 0.5])
    X, Y = ct.assemble(feats, cells, yd, yc)
    np.testing.assert_array_equal(X, feats[[0, 1, 4]])
    np.testing.assert_array_equal(Y, [[0.1, 0.3], [0.2, 0.4], [0.2, 0.4]])


def test_normaliser_constant_feature_gets_unit_scale():
    rng = np.random.default_rng(0)
    X = rng.normal(size=(1000, 6))
    X[:, 3] = 2.0                                       # the coarse-graining factor: constant
    nm = ct.normaliser(X)
    np.testing.assert_allclose(nm[:6], X.mean(axis=0))
    assert nm[6 + 3] == 1.0
    np.testing.assert_allclose(nm[[6, 7, 8, 10, 11]], X.std(axis=0)[[0, 1, 2, 4, 5]])


def test_pulloff_density_of_bonded_contacts():
    """two bonded pairs in cell 0 and one unbonded pair: density = sum of
    3 pi gamma R* over the bonded ones / (eps_s V_cell)"""
    x = np.array([[0.2, 0.5, 0.2], [0.4, 0.5, 0.2], [0.6, 0.5, 0.2], [0.8, 0.5, 0.2], [2.5, 0.5, 0.2],
                  [2.7, 0.5, 0.2]])
    r = np.array([0.1, 0.1, 0.1, 0.1, 0.1, 0.1])
    pairs = np.array([[0, 1], [2, 3], [4, 5]])
    bonded = np.array([1, 1, 0], np.uint8)
    eps = np.zeros(16)
    eps[0] = 0.5
    eps[2] = 0.5
    gam = 0.7
    A = ct.pulloff_density(x, r, pairs, bonded, gam, GRID, eps)
    expect = 2 * 3 * math.pi * gam * 0.05 / (0.5 * 0.5)
    assert A[0] == pytest.approx(expect)
    assert np.count_nonzero(A) == 1


def test_contact_point_divides_the_centre_line_by_the_radii():
    """unequal radii: the point sits r_a from a's centre, here across a cell face"""
    x = np.array([[0.55, 0.5, 0.2], [1.55, 0.5, 0.2]])
    r = np.array([0.6, 0.4])
    eps = np.ones(16)
    A = ct.pulloff_density(x, r, np.array([[0, 1]]), np.array([1], np.uint8), 1.0, GRID, eps)
    assert A[1] > 0.0 and A[0] == 0.0       # point at x = 1.15: cell 1


def test_he_params_layout():
    p = ct.he_params(3)
    from paper_2211_06142_amd import dem
    assert p.shape == (dem.MLP_NPARAMS,)
    sizes = [6, 64, 64, 64, 2]
    o = 0
    for a, b in zip(sizes[:-1], sizes[1:]):
        W = p[o:o + a * b]
        o += a * b
        assert np.all(p[o:o + b] == 0.0)
        o += b
        assert abs(W.std() / math.sqrt(2.0 / a) - 1.0) < 0.25
    assert o == p.size
