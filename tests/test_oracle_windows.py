"""The sub-box rows of H x (tests/oracle_windows.py) equal the rows of the
oracle's operator on the whole grid, in 2D and 3D, for boxes at the low and
high corners (sides shared with the domain) and inside the domain, with the
absorbing layer and a heterogeneous medium.  This is what lets the full-size
GPU tests compare sampled operator rows with the oracle."""
import numpy as np
import pytest

from oracle.elastic import ElasticSystem
from oracle_windows import window_rows
from workloads import abc_all_but_top


def medium(n, seed):
    rng = np.random.default_rng(seed)
    shape = tuple(reversed(n))
    vp = rng.uniform(2.0, 4.0, shape)
    vs = vp * rng.uniform(0.3, 0.55, shape)
    rho = rng.uniform(0.8, 1.3, shape)
    return vp, vs, rho


@pytest.mark.parametrize("n,h,boxes", [
    ((20, 14), (1.0, 0.5), [((0, 0), (7, 6)), ((13, 8), (7, 6)), ((5, 4), (9, 7))]),
    ((11, 9, 10), (1.0, 1.0, 0.8), [((0, 0, 0), (6, 5, 5)), ((5, 4, 5), (6, 5, 5)),
                                    ((3, 2, 2), (6, 6, 6))]),
])
def test_window_rows_equal_full_operator_rows(n, h, boxes):
    vp, vs, rho = medium(n, 4)
    omega, width, sides = 0.9, 3, abc_all_but_top(len(n))
    s = ElasticSystem(n, h, vp, vs, rho, omega, width, sides)
    rng = np.random.default_rng(5)
    x = rng.standard_normal(s.ndof) + 1j * rng.standard_normal(s.ndof)
    y = s.H() @ x
    seen = 0
    for lo, w in boxes:
        idx, yw = window_rows(n, h, vp, vs, rho, omega, width, sides, x, lo, w)
        assert len(idx) > 0 and len(np.unique(idx)) == len(idx)
        assert np.allclose(yw, y[idx], rtol=0, atol=1e-12 * np.abs(y).max())
        seen += len(idx)
    assert seen > 0


def test_window_margin_is_needed():
    """Rows next to a box side inside the domain do differ (so the margin
    is doing something): with margin 0 some rows disagree."""
    n, h = (16, 12), (1.0, 1.0)
    vp, vs, rho = medium(n, 6)
    s = ElasticSystem(n, h, vp, vs, rho, 0.9, 3, 15)
    rng = np.random.default_rng(7)
    x = rng.standard_normal(s.ndof) + 1j * rng.standard_normal(s.ndof)
    y = s.H() @ x
    idx, yw = window_rows(n, h, vp, vs, rho, 0.9, 3, 15, x, (4, 3), (8, 6), margin=0)
    assert not np.allclose(yw, y[idx], rtol=0, atol=1e-9 * np.abs(y).max())
