"""GPU multigrid calls (Sect. 5) against the oracle: grid transfer, the statistical-
equilibrium operator and right-hand side, and whole V-cycles."""
import dataclasses

import numpy as np
import pytest

from paper_1307_4217_amd import inputs, porta

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mgo():
    from oracle import multigrid
    return multigrid


def _dev(a, dtype=None):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype or torch.float64, device="cuda:0")


SHAPES = [(2, 2, 3), (4, 6, 5), (6, 4, 9), (16, 16, 33)]


@pytest.mark.parametrize("shape", SHAPES)
def test_restrict_prolong_inject_match_oracle(mgo, shape):
    import torch
    nx, ny, nz = shape
    nxc, nyc, nzc = mgo.coarse_shape(nx, ny, nz)
    n, nc = nx * ny * nz, nxc * nyc * nzc
    print(f"transfer {shape}", flush=True)
    rng = np.random.default_rng(nx * 100 + nz)
    for k in (1, 6):
        f = rng.standard_normal((k, n))
        got = porta.mg_restrict(_dev(f), nx, ny, nz).cpu().numpy()
        want = mgo.restrict(f, nx, ny, nz)
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-14 * np.abs(f).max())
        a, b = rng.standard_normal((k, nc)), rng.standard_normal((k, nc))
        base = rng.standard_normal((k, n))
        fine = _dev(base)
        porta.mg_prolong(fine, nx, ny, nz, _dev(a), _dev(b))
        np.testing.assert_allclose(fine.cpu().numpy(), base + mgo.prolong(a - b, nxc, nyc, nzc),
                                   rtol=0, atol=1e-14)
        fine = _dev(base)
        porta.mg_prolong(fine, nx, ny, nz, _dev(a))
        np.testing.assert_allclose(fine.cpu().numpy(), base + mgo.prolong(a, nxc, nyc, nzc),
                                   rtol=0, atol=1e-14)
    # emissivities written beside the restricted / prolonged source function
    kap_f = rng.uniform(0.5, 2.0, n)
    kap_c = mgo.inject(kap_f, nx, ny, nz)
    for prec, dt in ((porta.F64, torch.float64), (porta.F32, torch.float32)):
        f = rng.standard_normal((6, n))
        emis_c = torch.empty((6, nc), dtype=dt, device="cuda:0")
        rc_ = porta.mg_restrict(_dev(f), nx, ny, nz, kappa_c=_dev(kap_c, dt), emis_c=emis_c,
                                prec=prec).cpu().numpy()
        tol = 1e-15 if prec == porta.F64 else 1e-6
        kc = kap_c.astype(np.float32).astype(np.float64) if prec == porta.F32 else kap_c
        np.testing.assert_allclose(emis_c.cpu().numpy(), kc * rc_, rtol=tol, atol=tol)
        fine = _dev(f)
        emis = torch.empty((6, n), dtype=dt, device="cuda:0")
        a = rng.standard_normal((6, nc))
        porta.mg_prolong(fine, nx, ny, nz, _dev(a), kappa=_dev(kap_f, dt), emis=emis, prec=prec)
        kf = kap_f.astype(np.float32).astype(np.float64) if prec == porta.F32 else kap_f
        np.testing.assert_allclose(emis.cpu().numpy(), kf * fine.cpu().numpy(), rtol=tol,
                                   atol=tol)
    # injection of float32 and float64 fields
    for dt in (torch.float32, torch.float64):
        f = _dev(rng.standard_normal((3, n)), dt)
        got = porta.mg_inject(f, nx, ny, nz).cpu().numpy()
        np.testing.assert_array_equal(got, mgo.inject(f.cpu().numpy(), nx, ny, nz))
    torch.cuda.synchronize()


@pytest.mark.parametrize("magnetic", [True, False])
def test_see_operator_and_rhs_match_oracle(orc, magnetic):
    import torch
    cfg = inputs.Config("s", 8, 6, 5, 2, 4, 3, magnetic)
    atm = inputs.make_atmosphere(cfg, seed=3)
    n = atm.npoints
    rng = np.random.default_rng(7)
    jkq = np.vstack([rng.uniform(0.5, 1.5, (1, n)), 0.05 * rng.standard_normal((8, n)),
                     rng.uniform(0.0, 0.9, (1, n))])
    S = atm.source
    f = 0.02 * rng.standard_normal((6, n))
    base = rng.standard_normal((6, n))
    hanle = None if atm.hanle is None else _dev(atm.hanle)
    bhat = None if atm.bhat is None else _dev(atm.bhat)
    args = dict(eps_c=atm.eps_c, delta2=atm.delta2, w2=atm.w2, planck=atm.planck, hanle=hanle,
                bhat=bhat)
    lop = orc.see_operator(jkq, S, atm)
    for b, sign in ((None, -1.0), (base, 1.0), (base, -0.5)):
        got = porta.see_operator(_dev(jkq), _dev(S), base=None if b is None else _dev(b),
                                 sign=sign, **args).cpu().numpy()
        bb = b if b is not None else np.vstack([np.full((1, n), atm.eps_c * atm.planck),
                                                np.zeros((5, n))])
        np.testing.assert_allclose(got, bb + sign * lop, rtol=0, atol=1e-13)
    want, _, _ = orc.see_update(jkq, S, atm, rhs=f)
    got, _, _ = porta.see_update(_dev(jkq), _dev(S), rhs=_dev(f), want_rc=False, **args)
    np.testing.assert_allclose(got.cpu().numpy(), want, rtol=1e-13, atol=1e-14)
    # R_c between two iterates
    a, b = rng.uniform(0.5, 1.5, (6, n)), rng.uniform(0.5, 1.5, (6, n))
    rc = porta.rel_change(_dev(a), _dev(b)).item()
    assert rc == np.max(np.abs(a[0] - b[0]) / np.abs(a[0]))
    torch.cuda.synchronize()


def _mg_atmosphere(nx, nz, nfreq=5, seed=0):
    cfg = inputs.Config("mg", nx, nx, nz, 2, 4, nfreq, True)
    atm = inputs.make_atmosphere(cfg, seed=seed)
    return dataclasses.replace(atm, propmat=0 * atm.propmat), inputs.make_quadrature(cfg)


@pytest.mark.parametrize("nlevels", [2, 3])
def test_vcycles_match_oracle_fp64(mgo, nlevels):
    """Two V-cycles on 16x16x33 (2 + 4 smoothing, 10 coarse Jacobi iterations)."""
    import torch
    from paper_1307_4217_amd.multigrid import MultigridSolver
    atm, q = _mg_atmosphere(16, 33)
    print(f"V-cycles FP64, {nlevels} levels", flush=True)
    levels = mgo.make_levels(atm, q, nlevels)
    f = levels[0].planck_rhs()
    solver = MultigridSolver(atm, q, nlevels, porta.F64, ncoarse=10)
    S = atm.source.copy()
    for cycle in range(2):
        S_new = mgo.vcycle(levels, S, f, ncoarse=10)
        rc = solver.vcycle().item()
        got = solver.source.cpu().numpy()
        scale = np.abs(S_new).max(axis=1, keepdims=True)
        err = (np.abs(got - S_new) / scale).max()
        print(f"cycle {cycle + 1}: max err / component scale {err:.2e}, R_c {rc:.3e}", flush=True)
        assert err < 1e-10
        assert rc == pytest.approx(mgo.relative_change(S_new, S), rel=1e-8)
        S = S_new
    torch.cuda.synchronize()


def test_vcycle_fp32_sweep_close_to_oracle(mgo):
    """FP32 formal solutions inside the cycle (FP64 J, SEE and transfers) against the
    oracle on the same single-precision model: the S^0_0 error stays within the FP32
    sweep's 2e-5 relative bound amplified by at most 1/(1 - (1-eps) Lbar) <= 1/eps."""
    import torch
    from paper_1307_4217_amd.multigrid import MultigridSolver
    atm, q = _mg_atmosphere(16, 33)
    atm = dataclasses.replace(atm, kappa=atm.kappa.astype(np.float32).astype(np.float64),
                              source=atm.source)
    levels = mgo.make_levels(atm, q, 2)
    f = levels[0].planck_rhs()
    solver = MultigridSolver(atm, q, 2, porta.F32, ncoarse=10)
    S = mgo.vcycle(levels, atm.source.copy(), f, ncoarse=10)
    solver.vcycle()
    got = solver.source.cpu().numpy()
    rel00 = (np.abs(got[0] - S[0]) / np.abs(S[0])).max()
    k2 = (np.abs(got[1:] - S[1:]).max(axis=1) / np.abs(S[1:]).max(axis=1)).max()
    print(f"FP32 V-cycle: S00 max rel err {rel00:.2e}, K=2 max err / scale {k2:.2e}", flush=True)
    assert rel00 < 2e-5 / atm.eps_c
    assert k2 < 2e-5 / atm.eps_c
    torch.cuda.synchronize()


def test_emissivity_call():
    import torch
    rng = np.random.default_rng(9)
    n = 1000
    s = rng.standard_normal((6, n))
    kap = rng.uniform(0.1, 3.0, n)
    for dt in (torch.float64, torch.float32):
        got = porta.emissivity(_dev(kap, dt), _dev(s)).cpu().numpy().astype(np.float64)
        k = kap.astype(np.float32).astype(np.float64) if dt == torch.float32 else kap
        np.testing.assert_allclose(got, k * s, rtol=1e-15 if dt == torch.float64 else 1e-7,
                                   atol=0)
    torch.cuda.synchronize()


def test_mixed_precision_cycles_reach_fp64_result():
    """Three V-cycles with FP32 sweeps, then three with FP64 sweeps, end where six FP64
    cycles end, to less than what one more cycle still changes (the FP32 cycles only
    move the starting point of the FP64 ones)."""
    import torch
    from paper_1307_4217_amd.multigrid import MultigridSolver
    atm, q = _mg_atmosphere(16, 33)
    a = MultigridSolver(atm, q, 2, porta.F64, ncoarse=10)
    for _ in range(6):
        rc_a = a.vcycle().item()
    b = MultigridSolver(atm, q, 2, porta.F32, ncoarse=10)
    for _ in range(3):
        b.vcycle()
    b.set_precision(porta.F64)
    for _ in range(3):
        rc_b = b.vcycle().item()
    sa, sb = a.source.cpu().numpy(), b.source.cpu().numpy()
    err = (np.abs(sa - sb).max(axis=1) / np.abs(sa).max(axis=1)).max()
    print(f"mixed precision: R_c {rc_b:.2e} (FP64 {rc_a:.2e}), max diff / scale {err:.2e}",
          flush=True)
    assert err < rc_a
    assert rc_b < 2 * rc_a
    torch.cuda.synchronize()


@pytest.mark.parametrize("shape", [(2, 2, 7), (4, 6, 9), (6, 4, 9), (16, 16, 33)])
def test_cubic_prolongation_matches_oracle(mgo, shape):
    import torch
    nx, ny, nz = shape
    nxc, nyc, nzc = mgo.coarse_shape(nx, ny, nz)
    print(f"cubic prolongation {shape}", flush=True)
    rng = np.random.default_rng(nx + 7 * nz)
    for k in (1, 6):
        a, b = rng.standard_normal((k, nxc * nyc * nzc)), rng.standard_normal((k, nxc * nyc * nzc))
        base = rng.standard_normal((k, nx * ny * nz))
        fine = _dev(base)
        porta.mg_prolong(fine, nx, ny, nz, _dev(a), _dev(b), order=3)
        np.testing.assert_allclose(fine.cpu().numpy(),
                                   base + mgo.prolong(a - b, nxc, nyc, nzc, order=3),
                                   rtol=0, atol=1e-14)
    torch.cuda.synchronize()


def test_cubic_vcycles_and_nested_multigrid_match_oracle(mgo):
    """Two V-cycles with tri-cubic prolongation (2 levels) and one nested-multigrid pass
    (3 levels, tri-linear and tri-cubic) on 16x16x33, FP64."""
    import torch
    from paper_1307_4217_amd.multigrid import MultigridSolver
    atm, q = _mg_atmosphere(16, 33)
    levels2 = mgo.make_levels(atm, q, 2)
    f = levels2[0].planck_rhs()
    solver = MultigridSolver(atm, q, 2, porta.F64, ncoarse=10, order=3)
    S = atm.source.copy()
    for cycle in range(2):
        S = mgo.vcycle(levels2, S, f, ncoarse=10, order=3)
        solver.vcycle()
        got = solver.source.cpu().numpy()
        err = (np.abs(got - S) / np.abs(S).max(axis=1, keepdims=True)).max()
        print(f"cubic V-cycle {cycle + 1}: max err / scale {err:.2e}", flush=True)
        assert err < 1e-10
    levels3 = mgo.make_levels(atm, q, 3)
    for order in (1, 3):
        want = mgo.nested(levels3, atm.source, cycles=1, ncoarse=10, order=order)
        s3 = MultigridSolver(atm, q, 3, porta.F64, ncoarse=10, order=order)
        s3.nested()
        got = s3.source.cpu().numpy()
        err = (np.abs(got - want) / np.abs(want).max(axis=1, keepdims=True)).max()
        print(f"nested multigrid, order {order}: max err / scale {err:.2e}", flush=True)
        assert err < 1e-10
    torch.cuda.synchronize()
