"""Pins of the oracle's first-face short characteristics (faces = 1, Sect. 3.1: M and P
on the first face of the grid the ray crosses, vertical or horizontal, with the
in-plane dependencies that a vertical face brings closed around the periodic box) and
of its reference, long characteristics through the trilinear medium cut at every face
crossing (lc_fine_sweep).

Closed forms: a source linear in the vertical optical depth (the Eddington-Barbier
solution, linear in z, so bilinear interpolation on vertical faces is exact) and a
thermalized slab; the node-aligned diagonal ray, on which both SC variants and long
characteristics coincide; periodic shift invariance; and the refinement study that
compares the two SC geometries with the exact solution on a smooth atmosphere.
"""
import math
import types

import numpy as np
import pytest

from paper_1307_4217_amd import inputs


def _slab(nx, ny, nz, lx, ly, ztop, kap, S, i_bottom):
    n = nx * ny * nz
    e = np.zeros((6, n))
    e[0] = np.repeat(kap * S, nx * ny) if np.ndim(S) else kap * S
    return types.SimpleNamespace(nx=nx, ny=ny, nz=nz, lx=float(lx), ly=float(ly),
                                 z=np.linspace(0.0, ztop, nz), kappa=np.full(n, kap),
                                 propmat=np.zeros((6, n)), emis=e, i_bottom=float(i_bottom),
                                 w2=1.0, npoints=n)


def _quad(mu, nchi):
    return types.SimpleNamespace(mu=np.array([mu]), wmu=np.array([1.0]), nchi=nchi,
                                 phi=np.array([1.0]), wfreq=np.array([1.0]), x=np.zeros(1))


@pytest.mark.parametrize("mu", [0.06, 0.3, 0.9])
def test_linear_source_is_exact(orc, mu):
    """S = a + b tau_z with constant eta_I: I(z, mu) = a + b (tau_z + mu) at every node, so
    also where M lies on a vertical face (the z interpolation of I there is exact)."""
    nx, ny, nz = 6, 5, 12
    kap, a, b = 0.9, 1.0, 0.3
    z = np.linspace(0.0, 10.0, nz)
    tauz = kap * (z[-1] - z)
    atm = _slab(nx, ny, nz, 3.0, 2.5, 10.0, kap, a + b * tauz, a + b * (tauz[0] + mu))
    q = _quad(mu, 4)
    op = orc.OracleProblem(atm, q, faces=1)
    out = orc.fs_sweep(op, rays=[0, 1, 2, 3], want_full=True)["ifull"][..., 0]
    want = np.repeat(a + b * (tauz + mu), nx * ny)
    np.testing.assert_allclose(out[:, 0], np.broadcast_to(want, (4, want.size)), rtol=1e-13)
    if mu < 0.5:
        # these rays reach a vertical face before the plane below (dx < dz tan(theta))
        assert 3.0 / nx < (z[1] - z[0]) * math.sqrt(1 - mu * mu) / mu / math.sqrt(2)


def test_thermalized_slab_stays_at_its_source(orc):
    """Homogeneous slab whose bottom intensity equals its source function: I = S everywhere
    for every direction, grazing ones included."""
    atm = _slab(5, 4, 9, 2.0, 1.5, 8.0, 0.7, 1.3, 1.3)
    mu, w = np.polynomial.legendre.leggauss(4)
    q = types.SimpleNamespace(mu=0.5 * (mu + 1), wmu=0.5 * w, nchi=6, phi=np.array([1.0, 0.2]),
                              wfreq=np.ones(2), x=np.zeros(2))
    out = orc.fs_sweep(orc.OracleProblem(atm, q, faces=1), want_full=True)["ifull"]
    up = out[: len(q.mu) * q.nchi]
    np.testing.assert_allclose(up[..., 0], 1.3, rtol=1e-12)
    np.testing.assert_array_equal(up[..., 1:], 0.0)


def test_node_aligned_diagonal_ray_equals_long_characteristics(orc):
    """chi = pi/4 and dx = dy = dz tan(theta)/sqrt(2): every characteristic passes through
    grid nodes, so the first face crossed is the plane below at a node, and the
    first-face SC equals the plane-hop SC and both long-characteristics references
    (random atmosphere with polarization)."""
    mu = 0.6
    cfg = inputs.Config("diag", 6, 6, 7, 1, 4, 2, True)
    atm = inputs.make_atmosphere(cfg, seed=8)
    dz = 50.0
    dx = dz * math.sqrt(1 - mu * mu) / mu / math.sqrt(2)
    atm.z = np.arange(cfg.nz) * dz
    atm.lx = atm.ly = cfg.nx * dx
    q = types.SimpleNamespace(mu=np.array([mu]), wmu=np.array([1.0]), nchi=4,
                              phi=np.array([1.0, 0.3]), wfreq=np.ones(2), x=np.zeros(2))
    rays, freqs = [0, 1, 2, 3], [0, 1]
    f1 = orc.fs_sweep(orc.OracleProblem(atm, q, faces=1), rays=rays, freqs=freqs,
                      want_full=True)["ifull"]
    f0 = orc.fs_sweep(orc.OracleProblem(atm, q), rays=rays, freqs=freqs, want_full=True)["ifull"]
    lc = orc.lc_sweep(orc.OracleProblem(atm, q), rays, freqs)
    lcf = orc.lc_fine_sweep(orc.OracleProblem(atm, q), rays, freqs, nsub=1)
    scale = np.abs(f0).max()
    for other in (f0, lc, lcf):
        assert np.abs(f1 - other).max() <= 1e-13 * scale


def test_periodic_shift_invariance(orc):
    """Shifting every input by whole cells shifts the solution (the periodic fixed point
    does not depend on where the passes over a plane start)."""
    cfg = inputs.Config("shift", 6, 5, 8, 2, 4, 2, True)
    atm = inputs.make_atmosphere(cfg, seed=9)
    q = inputs.make_quadrature(cfg)
    rays = [0, 3, 5]
    base = orc.fs_sweep(orc.OracleProblem(atm, q, faces=1), rays=rays, want_full=True)["ifull"]
    di, dj = 2, 3
    sh = lambda a: np.roll(a.reshape(a.shape[:-1] + (cfg.nz, cfg.ny, cfg.nx)), (dj, di),
                           axis=(-2, -1)).reshape(a.shape)
    moved = types.SimpleNamespace(**vars(atm))
    moved.kappa, moved.propmat, moved.emis = sh(atm.kappa), sh(atm.propmat), sh(atm.emis)
    out = orc.fs_sweep(orc.OracleProblem(moved, q, faces=1), rays=rays, want_full=True)["ifull"]
    want = np.moveaxis(sh(np.moveaxis(base, -1, -2)), -1, -2)
    assert np.abs(out - want).max() <= 1e-13 * np.abs(base).max()
    # and grazing rays of this grid do reach vertical faces
    dz, dx = atm.z[1] - atm.z[0], atm.lx / cfg.nx
    assert dz * math.sqrt(1 - q.mu[0] ** 2) / q.mu[0] > dx


def test_fine_long_characteristics_converge(orc):
    """The reference itself: cutting each piece between face crossings into more parts
    changes the emergent intensity less and less (second order)."""
    cfg = inputs.Config("lc", 6, 6, 9, 2, 4, 1, True)
    atm = inputs.make_atmosphere(cfg, seed=10)
    q = inputs.make_quadrature(cfg)
    op = orc.OracleProblem(atm, q)
    top = slice((cfg.nz - 1) * 36, cfg.nz * 36)
    r = {n: orc.lc_fine_sweep(op, [0], [0], nsub=n)[0, 0, top, 0] for n in (2, 4, 8, 16)}
    d = [np.abs(r[n] / r[16] - 1).max() for n in (2, 4)]
    d8 = np.abs(r[8] / r[16] - 1).max()
    assert d[1] < 0.45 * d[0] and d8 < 0.45 * d[1], (d, d8)


def _smooth_atmosphere(n, nz, L=2000.0, H=500.0):
    x = np.arange(n) * L / n
    z = np.linspace(0.0, L, nz)
    Zg, Yg, Xg = np.meshgrid(z, x, x, indexing="ij")
    kap = (100.0 / H) * np.exp(-Zg / H) * (1 + 0.3 * np.sin(2 * np.pi * Xg / L)
                                           * np.cos(2 * np.pi * Yg / L))
    S = 1.0 + 0.4 * np.sin(2 * np.pi * (Xg + Yg) / L) * np.exp(-Zg / 800.0)
    e = np.zeros((6,) + kap.shape)
    e[0] = kap * S
    nn = kap.size
    return types.SimpleNamespace(nx=n, ny=n, nz=nz, lx=L, ly=L, z=z, kappa=kap.reshape(nn),
                                 propmat=np.zeros((6, nn)), emis=e.reshape(6, nn),
                                 i_bottom=1.0, w2=1.0, npoints=nn)


def test_first_face_sc_converges_where_plane_hops_do_not(orc):
    """A smooth atmosphere sampled at 8x8x9 and 16x16x17 (dx = dz), one grazing ray
    (mu = 0.05): against long characteristics through the same trilinear medium, the
    first-face SC error halves with the spacing, while the plane-hop SC (M always on the
    plane below, reading A1) does not decrease: its step crosses about tan(theta) dz/dx =
    20 cells with the medium sampled only at M, O and P, a ratio refinement keeps."""
    q = _quad(0.05, 8)
    err = {}
    for n in (8, 16):
        atm = _smooth_atmosphere(n, n + 1)
        top = slice(n * n * n, (n + 1) * n * n)
        ref = orc.lc_fine_sweep(orc.OracleProblem(atm, q), [1], [0], nsub=8)[0, 0, top, 0]
        for faces in (0, 1):
            sc = orc.fs_sweep(orc.OracleProblem(atm, q, faces=faces), rays=[1], freqs=[0],
                              want_full=True)["ifull"][0, 0, top, 0]
            err[(n, faces)] = float(np.sqrt(np.mean((sc / ref - 1) ** 2)))
    print("rms rel err of I_top, mu = 0.05:", err)
    assert err[(16, 1)] < 0.6 * err[(8, 1)]                 # first order or better
    assert err[(16, 0)] > 0.9 * err[(8, 0)]                 # plane hops: no convergence
    assert err[(16, 0)] > 10 * err[(16, 1)]


def test_faces_option_is_validated(orc):
    cfg = inputs.Config("v", 4, 4, 5, 1, 2, 1, True)
    atm = inputs.make_atmosphere(cfg, seed=1)
    q = inputs.make_quadrature(cfg)
    with pytest.raises(ValueError):
        orc.fs_sweep(orc.OracleProblem(atm, q, interp=1, faces=1))   # bilinear faces only
    with pytest.raises(ValueError):
        orc.fs_sweep(orc.OracleProblem(atm, q, faces=2))
    n = atm.npoints
    with pytest.raises(ValueError):
        orc.fs_sweep_cs(orc.OracleProblem(atm, q, faces=1), np.zeros(n), np.zeros((6, n)),
                        np.zeros((6, n)))
    with pytest.raises(ValueError):
        orc.fs_adjoint(orc.OracleProblem(atm, q, faces=1),
                       np.zeros((2, 1, 4, 4, 4)))
