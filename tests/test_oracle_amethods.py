"""Sect. 3.4 one-ray accuracy study: the formal solvers of oracle/amethods.py pinned to
closed forms, to scipy's PCHIP derivative, and to the statements of the section."""
import math

import numpy as np
import pytest
from scipy.interpolate import PchipInterpolator


@pytest.fixture(scope="module")
def am():
    from oracle import amethods
    return amethods


def test_fritsch_butland_is_the_pchip_derivative(am):
    rng = np.random.default_rng(4)
    for _ in range(20):
        x = np.cumsum(rng.uniform(0.2, 2.0, 12))
        y = np.cumsum(rng.normal(size=12))
        want = PchipInterpolator(x, y).derivative()(x[1:-1])
        got = [am.fritsch_butland(y[k - 1], y[k], y[k + 1], x[k] - x[k - 1], x[k + 1] - x[k])
               for k in range(1, 11)]
        np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-14)


def test_parabolic_control_point_reproduces_any_quadratic(orc):
    """Steps 1, 3, 4 alone give the tangent of the parabola through M, O, P, extremum
    or not; BESSER keeps c_M = y_O when O is an extremum."""
    rng = np.random.default_rng(5)
    for _ in range(50):
        a, b, c = rng.normal(size=3)
        hM, hP = rng.uniform(0.3, 2.0, 2)
        q = lambda x: a * x * x + b * x + c
        yM, yO, yP = q(-hM), q(0.0), q(hP)
        # tangent at O, evaluated at the middle of MO
        want = yO - 0.5 * hM * b
        assert orc.parabolic_cm(yM, yO, yP, hM, hP) == pytest.approx(want, abs=1e-12)
    yM, yO, yP = 0.0, 1.0, 0.0        # extremum at O
    assert orc.besser_cm(yM, yO, yP, 1.0, 1.0) == 1.0
    assert orc.parabolic_cm(yM, yO, yP, 1.0, 1.0) == pytest.approx(1.0)   # symmetric case
    assert orc.parabolic_cm(0.0, 1.0, 0.5, 1.0, 1.0) != orc.besser_cm(0.0, 1.0, 0.5, 1.0, 1.0)


def test_parabolic_formal_solution_exact_for_quadratic_source(am):
    """For S(t) quadratic along the ray, I = S - S' + S'' plus the decaying boundary
    term; the parabolic solver is exact at every node but the last, even where S has
    an extremum, and BESSER is not there."""
    z = np.linspace(-3.0, 3.0, 25)
    S = 2.0 - 0.3 * z * z + 0.1 * z            # maximum inside the range
    exact = lambda t: (2.0 - 0.3 * t * t + 0.1 * t) - (-0.6 * t + 0.1) + (-0.6)
    i0 = exact(z[0]) + 0.7                      # plus a boundary transient
    want = exact(z) + 0.7 * np.exp(-(z - z[0]))
    got = am.solve_ray(z, S, i0, "parabolic")
    np.testing.assert_allclose(got[:-1], want[:-1], rtol=1e-12)
    got_b = am.solve_ray(z, S, i0, "besser")
    assert np.abs(got_b[:-1] - want[:-1]).max() > 1e-6


@pytest.fixture(scope="module")
def table(am):
    return am.error_table()


def test_boundary_value_of_the_section(am):
    assert am.intensity(-12.0) == pytest.approx(2.77176e-7, rel=5e-6)


def test_besser_equals_parabolic_without_overshoots(table):
    """Sect. 3.3: the two give identical results when nothing overshoots (fine grids)."""
    for (dt, eb), (_, ep) in zip(table["besser"], table["parabolic"]):
        if dt <= 0.5:
            assert eb == ep
    # and at the coarsest grid the parabola overshoots badly, BESSER does not
    assert table["parabolic"][0][1] > 10 * table["besser"][0][1]


def test_convergence_orders(table):
    """Fine grids: linear interpolation of S is second order, parabolic / BESSER third."""
    def order(m):
        (d1, e1), (d2, e2) = table[m][-2], table[m][-1]
        return math.log(e1 / e2) / math.log(d1 / d2)
    assert 1.8 < order("linear") < 2.2
    assert 2.7 < order("besser") < 3.3
    assert 2.7 < order("parabolic") < 3.3
    for m in ("parabolic", "besser", "bezier", "cbezier"):
        assert table[m][-1][1] < table["linear"][-1][1] / 10


def test_bezier_needs_no_clip_on_a_uniform_grid(table):
    """A property of the reading taken (design reading A25), not a statement of the
    paper, which shows the two solvers apart: with equal spacing the Fritsch-Butland
    derivative is at most twice the smaller slope, so y_O - h/2 y'_O never leaves
    [y_M, y_O] and the clipped and unclipped Bezier solvers coincide."""
    for (_, e1), (_, e2) in zip(table["bezier"], table["cbezier"]):
        assert e1 == e2


READINGS = ("bezier_o", "cbezier_o", "bezier_m", "cbezier_m", "bezier_mo", "cbezier_mo")


def test_no_reading_of_the_bezier_solvers_gives_the_paper_ranking(am, table):
    """Sect. 3.4 states that on fine grids the Bezier solvers (Fritsch-Butland derivative,
    with or without the c_M clip) are less accurate than BESSER and the parabolic solver,
    and that the clip helps on coarse grids.  None of the readings tried reproduces that
    on this problem: the tangent at O (as in the study), the tangent at M, the mean of
    the two, each with and without the clip, with every interval given its full rule
    (ghost nodes) and E over every node.  On every one of them the clip never acts on a
    uniform grid and, for Delta tau <= 0.5, the Bezier solver is more accurate than
    BESSER; this records the evidence behind reading A25."""
    besser = dict(table["besser"])
    for n in (49, 97, 193):
        dt = 24.0 / (n - 1)
        errs = {r: am.solve_ray_reading(n, r) for r in READINGS}
        for r in ("bezier_o", "bezier_m", "bezier_mo"):
            assert errs[r] == errs["c" + r]
            assert errs[r] < besser[dt], (dt, r, errs[r], besser[dt])
