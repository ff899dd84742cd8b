"""fpca_cv_select (host code behind the C ABI): the grid minimizer of a CV
curve refined by the vertex of the parabola through its neighbours in log h.
Pinned by closed forms: a curve that is exactly quadratic in log h has its
vertex at the known minimizer; boundary minima keep the grid point; rows on a
ray move together."""
import numpy as np
import pytest

import paper_1510_04439_amd as F


@pytest.fixture(scope="module", autouse=True)
def lib():
    F.load_library()


def test_quadratic_in_log_h_recovers_vertex():
    hs = np.geomspace(0.05, 0.5, 12)
    for hstar in (0.0731, 0.12, 0.2567, 0.41):
        cv = 3.0 * (np.log(hs) - np.log(hstar)) ** 2 + 7.0
        got = F.fpca_cv_select(hs, cv)[0]
        assert abs(got - hstar) <= 1e-12 * hstar, (hstar, got)


def test_boundary_and_concave_keep_grid_point():
    hs = np.geomspace(0.1, 0.4, 6)
    assert F.fpca_cv_select(hs, np.arange(6.0))[0] == hs[0]
    assert F.fpca_cv_select(hs, -np.arange(6.0))[0] == hs[-1]
    # an interior minimum: the vertex stays between its neighbours, and on the
    # side of the lower neighbour
    cv2 = np.array([5.0, 4.0, 2.0, 3.0, 4.0, 6.0])
    got = F.fpca_cv_select(hs, cv2)[0]
    assert hs[2] < got < hs[3]
    # NaN scores never win
    cv3 = np.array([np.nan, 4.0, 2.0, 3.0, np.nan, 1.0])
    assert F.fpca_cv_select(hs, cv3)[0] == hs[5]


def test_rows_on_a_ray_move_together():
    s = np.geomspace(0.08, 0.4, 9)
    rows = np.stack([s, 1.5 * s], axis=1)
    cv = (np.log(s) - np.log(0.17)) ** 2
    got = F.fpca_cv_select(rows, cv, d=2)
    assert abs(got[0] - 0.17) < 1e-12 and abs(got[1] - 1.5 * 0.17) < 1e-12


def test_rejects_rows_off_a_ray_and_unsorted():
    s = np.geomspace(0.1, 0.3, 4)
    bad = np.stack([s, s * np.array([1.0, 1.1, 1.0, 1.0])], axis=1)
    with pytest.raises(F.FpcaError):
        F.fpca_cv_select(bad, np.ones(4), d=2)
    with pytest.raises(F.FpcaError):
        F.fpca_cv_select(s[::-1].copy(), np.ones(4))
