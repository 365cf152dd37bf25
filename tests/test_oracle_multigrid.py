"""Pins of the oracle's multigrid iteration (Sect. 5): the transfer operators against
library interpolation and their defining identities, the statistical-equilibrium
operator against the Jacobi update, and the FAS cycle against a direct solution of
the (linear, two-level) discrete problem on a tiny grid."""
import dataclasses

import numpy as np
import pytest
from scipy.interpolate import RegularGridInterpolator

from paper_1307_4217_amd import inputs


@pytest.fixture(scope="module")
def mg():
    from oracle import multigrid
    return multigrid


def _periodic_trilinear(c, nxc, nyc, nzc):
    """Fine-node values of the piecewise tri-linear interpolant of a coarse grid field,
    by scipy on a grid padded by one periodic column/row in x and y."""
    g = c.reshape(nzc, nyc, nxc)
    g = np.concatenate([g, g[:, :1, :]], axis=1)
    g = np.concatenate([g, g[:, :, :1]], axis=2)
    f = RegularGridInterpolator((np.arange(nzc), np.arange(nyc + 1), np.arange(nxc + 1)), g)
    nx, ny, nz = 2 * nxc, 2 * nyc, 2 * nzc - 1
    kk, jj, ii = np.meshgrid(np.arange(nz) / 2, np.arange(ny) / 2, np.arange(nx) / 2,
                             indexing="ij")
    return f(np.stack([kk.ravel(), jj.ravel(), ii.ravel()], axis=1))


@pytest.mark.parametrize("shape", [(2, 2, 2), (3, 2, 4), (5, 4, 3)])
def test_prolongation_is_trilinear_interpolation(mg, shape):
    nxc, nyc, nzc = shape
    rng = np.random.default_rng(1)
    c = rng.standard_normal((2, nzc * nyc * nxc))
    got = mg.prolong(c, nxc, nyc, nzc)
    for k in range(2):
        np.testing.assert_allclose(got[k], _periodic_trilinear(c[k], nxc, nyc, nzc),
                                   rtol=0, atol=1e-14)
    # injection at the coarse nodes
    np.testing.assert_array_equal(mg.inject(got, 2 * nxc, 2 * nyc, 2 * nzc - 1), c)


def test_restriction_constants_and_linear_z(mg):
    nx, ny, nz = 6, 4, 9
    one = np.full((1, nx * ny * nz), 3.25)
    np.testing.assert_allclose(mg.restrict(one, nx, ny, nz), 3.25, rtol=0, atol=1e-15)
    z = np.repeat(np.arange(nz, dtype=float), nx * ny)[None, :]   # f = k (plane index)
    r = mg.restrict(z, nx, ny, nz).reshape(5, -1)
    # interior coarse planes: full weighting reproduces a linear function
    np.testing.assert_allclose(r[1:-1], np.broadcast_to((2.0 * np.arange(1, 4))[:, None], (3, 6)),
                               atol=1e-14)
    # boundary planes keep 2 x 3^2 nodes with z weights (1, 1/2) / 1.5
    np.testing.assert_allclose(r[0], (1.0 * 0 + 0.5 * 1) / 1.5, atol=1e-15)
    np.testing.assert_allclose(r[-1], (1.0 * 8 + 0.5 * 7) / 1.5, atol=1e-15)


def test_restriction_is_adjoint_of_prolongation_inside(mg):
    """8 <R f, g>_coarse = <f, P g>_fine for coarse fields vanishing on the z boundaries
    (where R is renormalised), and the restriction only sees the 3^3 neighbourhood."""
    nx, ny, nz = 8, 6, 11
    nxc, nyc, nzc = mg.coarse_shape(nx, ny, nz)
    rng = np.random.default_rng(2)
    f = rng.standard_normal((1, nx * ny * nz))
    g = rng.standard_normal((1, nxc * nyc * nzc)).reshape(nzc, nyc, nxc)
    g[0] = g[-1] = 0.0
    g = g.reshape(1, -1)
    lhs = 8.0 * float(np.sum(mg.restrict(f, nx, ny, nz) * g))
    rhs = float(np.sum(f * mg.prolong(g, nxc, nyc, nzc)))
    assert lhs == pytest.approx(rhs, rel=1e-13)
    # a delta at a fine node reaches only the coarse nodes within one fine cell
    d = np.zeros((1, nx * ny * nz))
    d[0, (4 * ny + 3) * nx + 5] = 1.0                  # fine (i, j, k) = (5, 3, 4)
    r = mg.restrict(d, nx, ny, nz).reshape(nzc, nyc, nxc)
    nz_idx = {tuple(i) for i in np.argwhere(r != 0)}
    assert nz_idx == {(2, 1, 2), (2, 1, 3), (2, 2, 2), (2, 2, 3)}
    assert r[2, 1, 2] == pytest.approx(1.0 * 0.5 * 0.5 / 8)


def _atmosphere(nx, ny, nz, nmu=2, nchi=4, nfreq=5, propmat=False, seed=0):
    cfg = inputs.Config("mg", nx, ny, nz, nmu, nchi, nfreq, True)
    atm = inputs.make_atmosphere(cfg, seed=seed)
    if not propmat:
        atm = dataclasses.replace(atm, propmat=0 * atm.propmat)
    return atm, inputs.make_quadrature(cfg)


def test_see_operator_matches_jacobi_update(orc):
    """With J held fixed the Jacobi update solves the K = 2 rows exactly and the K = 0
    row up to the Lambda-bar term: L(S_new) S_new = f + (1-eps) Lbar (S_new - S_old)."""
    atm, q = _atmosphere(4, 4, 5)
    rng = np.random.default_rng(3)
    n = atm.npoints
    jkq = np.vstack([rng.uniform(0.5, 1.5, (1, n)), 0.05 * rng.standard_normal((8, n)),
                     rng.uniform(0.0, 0.9, (1, n))])
    s_old = atm.source
    f = 0.02 * rng.standard_normal((6, n))
    f[0] += atm.eps_c * atm.planck
    s_new, _, _ = orc.see_update(jkq, s_old, atm, rhs=f)
    lhs = orc.see_operator(jkq, s_new, atm)
    want = f.copy()
    want[0] += (1 - atm.eps_c) * jkq[9] * (s_new[0] - s_old[0])
    np.testing.assert_allclose(lhs, want, rtol=0, atol=1e-13)
    # rhs = None is f = (eps B, 0, ...)
    f0 = np.zeros((6, n))
    f0[0] = atm.eps_c * atm.planck
    a, _, _ = orc.see_update(jkq, s_old, atm)
    b, _, _ = orc.see_update(jkq, s_old, atm, rhs=f0)
    np.testing.assert_array_equal(a, b)


@pytest.fixture(scope="module")
def tiny_problem(mg):
    """The 8x8x9 problem iterated to R_c < 1e-15.  (BESSER's limiter makes the formal
    solution non-linear in S, so there is no constant matrix to solve directly; the
    converged iterate is pinned instead by its residual f - L(rho) rho.)"""
    atm, q = _atmosphere(8, 8, 9, nmu=2, nchi=4, nfreq=3)
    lev = mg.make_levels(atm, q, 1)[0]
    f = lev.planck_rhs()
    S = atm.source.copy()
    for _ in range(500):
        S, rc = lev.jacobi(S, f)
        if rc < 1e-15:
            break
    return atm, q, f, S


def test_converged_iterate_solves_the_equations(mg, tiny_problem):
    atm, q, f, s_star = tiny_problem
    lev = mg.make_levels(atm, q, 1)[0]
    r = lev.residual(s_star, f)
    assert np.abs(r).max() < 1e-13
    # and the thermalised deep layers of an isothermal model sit at the Planck value
    deep = s_star[0].reshape(9, -1)[0]
    np.testing.assert_allclose(deep, atm.planck, rtol=1e-2)


def test_fas_cycle_fixed_point(mg, tiny_problem):
    """At the discrete solution the residual vanishes, Eq. mgcsfy is solved by R(rho),
    and the coarse-grid correction is zero: one V-cycle returns the solution."""
    atm, q, f, s_star = tiny_problem
    levels = mg.make_levels(atm, q, 2)
    S = mg.vcycle(levels, s_star.copy(), f, ncoarse=10)
    np.testing.assert_allclose(S, s_star, rtol=0, atol=1e-12 * np.abs(s_star).max())


def test_vcycles_converge_to_the_discrete_solution(mg):
    """On a grid whose coarse level still resolves each decade of optical depth with
    about three points, ten V-cycles drive the K = 0 rows of the residual of Eq. resid
    to 1e-9 and the whole residual 1e5 times below that of the initial guess (the K = 2
    rows, relaxed by plain Lambda iteration in the deep magnetised layers, lag)."""
    atm, q = _atmosphere(16, 16, 33, nfreq=3)
    levels = mg.make_levels(atm, q, 2)
    f = levels[0].planck_rhs()
    S = atm.source.copy()
    r0 = np.abs(levels[0].residual(S, f)).max()
    for _ in range(10):
        S = mg.vcycle(levels, S, f, ncoarse=20)
    r = np.abs(levels[0].residual(S, f))
    assert r[0].max() < 1e-9
    assert r.max() < 1e-5 * r0


def test_coarse_grid_correction_accelerates_smoothing(mg):
    """Sect. 5.1: the same cycle (2 + 4 Jacobi iterations around a residual) reduces
    R_c several times more with the coarse-grid correction than without it."""
    atm, q = _atmosphere(16, 16, 33, nfreq=5)
    levels = mg.make_levels(atm, q, 2)
    f = levels[0].planck_rhs()

    def smoothing_only(S):
        for _ in range(6):
            S, _ = levels[0].jacobi(S, f)
        return S
    ratios = []
    for cycle in (lambda S: mg.vcycle(levels, S, f, ncoarse=40), smoothing_only):
        S = cycle(atm.source.copy())
        S1 = cycle(S)
        S2 = cycle(S1)
        ratios.append(mg.relative_change(S2, S1) / mg.relative_change(S1, S))
    assert ratios[0] < 0.3 * ratios[1]


def test_tricubic_prolongation_reproduces_cubics(mg):
    """The tri-cubic-centred prolongation is exact for cubic polynomials along z (also
    next to the boundaries, where the interpolant shifts inward) and along x away from
    the periodic seam, and takes the coarse values on coarse nodes."""
    nxc, nyc, nzc = 8, 3, 6
    nx, ny, nz = 2 * nxc, 2 * nyc, 2 * nzc - 1
    p3 = lambda t: 0.3 * t ** 3 - 1.1 * t * t + 0.7 * t - 2.0
    kc = np.arange(nzc, dtype=float)
    cz = np.repeat(p3(kc), nyc * nxc)[None, :]
    fz = mg.prolong(cz, nxc, nyc, nzc, order=3).reshape(nz, ny, nx)
    np.testing.assert_allclose(fz[:, 0, 0], p3(np.arange(nz) / 2.0), rtol=1e-13, atol=1e-13)
    ic = np.arange(nxc, dtype=float)
    cx = np.tile(p3(ic), nzc * nyc)[None, :]
    fx = mg.prolong(cx, nxc, nyc, nzc, order=3).reshape(nz, ny, nx)
    inner = np.arange(2, 2 * nxc - 4)          # stencils that do not cross the seam
    np.testing.assert_allclose(fx[0, 0, inner], p3(inner / 2.0), rtol=1e-13, atol=1e-13)
    rng = np.random.default_rng(6)
    c = rng.normal(size=(2, nzc * nyc * nxc))
    f = mg.prolong(c, nxc, nyc, nzc, order=3)
    np.testing.assert_array_equal(mg.inject(f, nx, ny, nz), c)
    # the centred weights (-1, 9, 9, -1)/16 and the boundary ones (5, 15, -5, 1)/16
    e = np.zeros((1, nzc * nyc * nxc))
    e[0, 0] = 1.0                               # coarse node (0, 0, 0)
    g = mg.prolong(e, nxc, nyc, nzc, order=3).reshape(nz, ny, nx)
    assert g[1, 0, 0] == pytest.approx(5 / 16)              # z: first interval
    assert g[0, 0, 1] == pytest.approx(9 / 16)              # x: centred, right of node 0
    assert g[0, 0, 2 * nxc - 1] == pytest.approx(9 / 16)    # x: across the periodic seam
    assert g[0, 0, 3] == pytest.approx(-1 / 16)


@pytest.mark.parametrize("order", [1, 3])
def test_fas_fixed_point_with_either_prolongation(mg, tiny_problem, order):
    atm, q, f, s_star = tiny_problem
    levels = mg.make_levels(atm, q, 2)
    S = mg.vcycle(levels, s_star.copy(), f, ncoarse=10, order=order)
    np.testing.assert_allclose(S, s_star, rtol=0, atol=1e-12 * np.abs(s_star).max())


def test_nested_multigrid_starts_closer_than_a_vcycle(mg):
    """Nested multigrid (coarsest-grid solution prolonged upwards, one V-cycle per grid)
    leaves a smaller residual than one V-cycle from the flat initial guess, for a few
    coarse-grid sweeps more."""
    atm, q = _atmosphere(16, 16, 33, nfreq=3)
    levels = mg.make_levels(atm, q, 3)
    f = levels[0].planck_rhs()
    r_v = np.abs(levels[0].residual(mg.vcycle(levels, atm.source.copy(), f, ncoarse=20), f))
    S = mg.nested(levels, atm.source, cycles=1, ncoarse=20)
    r_n = np.abs(levels[0].residual(S, f))
    assert r_n.max() < 0.5 * r_v.max()
    assert r_n[0].max() < 0.1 * r_v[0].max()


def test_random_propagation_matrix_leaves_isolated_slow_points(mg):
    """Why the V-cycle barely helps on the configured atmosphere (16x16x33, random
    eta_X, rho_X up to 5% of eta_I with no matching emission, magnetic field): in the
    optically thick lower planes each cell's own dichroism raises J above S by
    delta = [(1 + K')^-1]_II - 1, comparable to eps_c, which leaves a local equation with
    a destruction probability eps_c - delta close to zero.  The error that survives the
    cycles sits on a few isolated points of that kind, which no coarser grid represents,
    so a V(2,4) cycle gains about what its own smoothing gains."""
    from oracle import multigrid as mgm
    cfg = inputs.Config("mg", 16, 16, 33, 2, 4, 5, True)
    atm = inputs.make_atmosphere(cfg, seed=0, magnetic=True)
    q = inputs.make_quadrature(cfg)
    levels = mgm.make_levels(atm, q, 3)
    f = levels[0].planck_rhs()
    S = atm.source.copy()
    hist = []
    for _ in range(6):
        new = mgm.vcycle(levels, S.copy(), f)
        hist.append(mgm.relative_change(new, S))
        prev, S = S, new
    factor = (hist[-1] / hist[-3]) ** 0.5
    # slow: about 0.4 per cycle, against 0.86 per Jacobi sweep (0.86^6 = 0.41 for the
    # cycle's six smoothing sweeps)
    assert factor > 0.3, hist
    d = np.abs(S[0] - prev[0]) / np.abs(S[0])
    slow = d > d.max() / 10
    np_ = cfg.nx * cfg.ny
    assert slow.mean() < 0.02                      # a few points carry the change
    sm = slow.reshape(cfg.nz, np_)
    assert sm[6:].sum() == 0                       # all in the optically thick planes
    S3 = S[0].reshape(cfg.nz, np_)
    ratio = np.concatenate([S3[k][sm[k]] / np.median(S3[k]) for k in range(cfg.nz) if sm[k].any()])
    assert np.median(ratio) > 1.3                  # where S00 rose above its plane
    eta = atm.propmat / atm.kappa
    a2, r2 = (eta[:3] ** 2).sum(0), (eta[3:] ** 2).sum(0)
    ar = (eta[:3] * eta[3:]).sum(0)
    delta = (1 + r2) / (1 + r2 - a2 - ar ** 2) - 1
    assert np.median(delta[slow]) > 1.3 * np.median(delta)   # with the larger dichroism
