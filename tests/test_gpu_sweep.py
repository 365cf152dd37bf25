"""GPU parity of the forward path (C-ABI calls) against the FP64 CPU oracle."""
import dataclasses

import numpy as np
import pytest

from gpu_common import (Case, compare_jkq, compare_stokes, oracle_full, require_gpu, rounded,
                        to_dev, up_rays)
from paper_1307_4217_amd import inputs, porta

pytestmark = pytest.mark.gpu


def test_library_is_in_tree():
    import os
    require_gpu()
    assert os.path.dirname(porta.LIB_PATH).endswith("paper_1307_4217_amd")
    assert "gfx950" in porta.version()


def test_sweep_fp64_c1_matches_oracle():
    atm, q, ref = oracle_full("C1", 0, "f64")
    case = Case(atm, q, porta.F64)
    jkq, itop = case.sweep()
    print("C1 FP64:", compare_stokes(itop, ref["itop"], 1e-10, 1e-12, "itop"),
          compare_jkq(jkq, ref["jkq"], 1e-10, "jkq"))


def test_sweep_fp32_c1_matches_oracle():
    atm, q, ref = oracle_full("C1", 0, "f32")
    case = Case(atm, q, porta.F32)
    jkq, itop = case.sweep()
    print("C1 FP32:", compare_stokes(itop, ref["itop"], 2e-5, 1e-7, "itop"),
          compare_jkq(jkq, ref["jkq"], 2e-5, "jkq"))


@pytest.mark.parametrize("prec", [porta.F64, porta.F32])
@pytest.mark.parametrize("ray_batch, block", [(0, 256), (3, 64), (7, 192)])
def test_sweep_ragged_grid_batches_and_blocks(orc, prec, ray_batch, block):
    """Odd sizes (plane of 7x5 nodes, partial blocks and ray batches, 3 azimuths)."""
    cfg = inputs.Config("ragged", 7, 5, 9, 2, 3, 5, True)
    atm = inputs.make_atmosphere(cfg, seed=3)
    atm = dataclasses.replace(atm, lx=530.0, ly=410.0, z=np.sort(np.random.default_rng(9).uniform(0, 900, 9)))
    if prec == porta.F32:
        atm = rounded(atm, np.float32)
    q = inputs.make_quadrature(cfg)
    ref = orc.fs_sweep(orc.OracleProblem(atm, q))
    case = Case(atm, q, prec)
    jkq, itop = case.sweep(opts=porta.options(ray_batch=ray_batch, block=block))
    tol_i, tol_p = (1e-10, 1e-12) if prec == porta.F64 else (2e-5, 1e-7)
    compare_stokes(itop, up_rays(ref["itop"], q), tol_i, tol_p, "itop")
    compare_jkq(jkq, ref["jkq"], tol_i, "jkq")


@pytest.mark.parametrize("ray_batch, block", [(0, 256), (5, 64), (3, 192)])
def test_sweep_rows_of_whole_wavefronts(orc, ray_batch, block):
    """nx a multiple of 64 (128x3 planes, lx != ly, unequal z steps): the FP32 kernel
    takes the x + 1 corners of the upwind stencil from the next lane, the last lane's
    from a wavefront-uniform load; the wrap of the stencil around x falls inside a
    wavefront for the shifted rays, and blocks of 192 threads put row boundaries
    between wavefronts of one block."""
    cfg = inputs.Config("rows64", 128, 3, 7, 2, 4, 3, True)
    atm = inputs.make_atmosphere(cfg, seed=12)
    z = np.cumsum(np.r_[0.0, np.random.default_rng(13).uniform(30.0, 120.0, cfg.nz - 1)])
    atm = rounded(dataclasses.replace(atm, lx=1700.0, ly=90.0, z=z), np.float32)
    q = inputs.make_quadrature(cfg)
    ref = orc.fs_sweep(orc.OracleProblem(atm, q))
    jkq, itop = Case(atm, q, porta.F32).sweep(opts=porta.options(ray_batch=ray_batch,
                                                                  block=block))
    ei, ep = compare_stokes(itop, up_rays(ref["itop"], q), 2e-5, 1e-7, "itop")
    ej = compare_jkq(jkq, ref["jkq"], 2e-5, "jkq")
    print(f"128x3 FP32 block {block}: I {ei:.2e}, Q/I.. {ep:.2e}, J {ej:.2e}")


@pytest.mark.parametrize("prec", [porta.F64, porta.F32])
@pytest.mark.parametrize("scale", [1e-7, 1e3])
def test_extreme_optical_depths(orc, prec, scale):
    """The whole model scaled to optical steps of 1e-17..1e-2 (every coefficient from
    its Taylor branch) or of up to 6e7 at line centre on the most inclined rays
    (e^-tau underflows, I_O -> S_O): eta and eps scaled together, so the source
    functions are unchanged."""
    cfg = inputs.Config("ext", 6, 5, 8, 2, 3, 5, True)
    atm = inputs.make_atmosphere(cfg, seed=14)
    atm = dataclasses.replace(atm, kappa=atm.kappa * scale, propmat=atm.propmat * scale,
                              emis=atm.emis * scale)
    if prec == porta.F32:
        atm = rounded(atm, np.float32)
    q = inputs.make_quadrature(cfg)
    ref = orc.fs_sweep(orc.OracleProblem(atm, q))
    jkq, itop = Case(atm, q, prec).sweep()
    tol_i, tol_p = (1e-10, 1e-12) if prec == porta.F64 else (2e-5, 1e-7)
    compare_stokes(itop, up_rays(ref["itop"], q), tol_i, tol_p, f"itop x{scale:g}")
    compare_jkq(jkq, ref["jkq"], tol_i, f"jkq x{scale:g}")


def test_single_plane_pair_and_single_column(orc):
    """Degenerate grids: nz = 2 (boundary + last plane only) and a 1x1 column."""
    for (nx, ny, nz) in ((4, 3, 2), (1, 1, 6)):
        cfg = inputs.Config("tiny", nx, ny, nz, 2, 4, 3, False)
        atm = inputs.make_atmosphere(cfg, seed=5)
        q = inputs.make_quadrature(cfg)
        ref = orc.fs_sweep(orc.OracleProblem(atm, q))
        jkq, itop = Case(atm, q, porta.F64).sweep()
        compare_stokes(itop, up_rays(ref["itop"], q), 1e-10, 1e-12, f"itop {nx}x{ny}x{nz}")
        compare_jkq(jkq, ref["jkq"], 1e-10, f"jkq {nx}x{ny}x{nz}")


def test_accumulate_adds_to_existing_j():
    torch = require_gpu()
    atm, q, ref = oracle_full("C1", 0, "f64")
    case = Case(atm, q, porta.F64)
    j0 = torch.full((10, case.hg.N), 0.25, dtype=torch.float64, device="cuda")
    porta.fs_sweep(case.hg, case.kappa, case.prop, case.emis, atm.i_bottom, atm.w2,
                   jkq=j0, accumulate=True, want_itop=False)
    torch.cuda.synchronize()
    compare_jkq(j0.cpu().numpy() - 0.25, ref["jkq"], 1e-10, "accumulated jkq")


def test_sweep_is_deterministic():
    atm, q, _ = oracle_full("C1", 0, "f64")
    for prec in (porta.F64, porta.F32):
        case = Case(atm, q, prec)
        a = case.sweep()
        b = case.sweep()
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_periodic_shift_is_exact_on_gpu():
    atm, q, _ = oracle_full("C1", 0, "f64")
    nx, ny, nz = atm.nx, atm.ny, atm.nz
    di, dj = 5, 11
    roll = lambda a: np.roll(a.reshape(a.shape[:-1] + (nz, ny, nx)), (dj, di),
                             axis=(-2, -1)).reshape(a.shape)
    atm2 = dataclasses.replace(atm, kappa=roll(atm.kappa[None])[0], propmat=roll(atm.propmat),
                               emis=roll(atm.emis))
    j1, t1 = Case(atm, q, porta.F32).sweep()
    j2, t2 = Case(atm2, q, porta.F32).sweep()
    assert np.array_equal(j2, roll(j1))
    assert np.array_equal(t2, np.roll(t1, (dj, di), axis=(2, 3)))


@pytest.mark.parametrize("prec", [porta.F64, porta.F32])
def test_jkq_accumulate_matches_oracle(orc, prec):
    torch = require_gpu()
    cfg = inputs.Config("blk", 6, 5, 4, 3, 4, 7, False)
    atm = inputs.make_atmosphere(cfg, seed=2)
    q = inputs.make_quadrature(cfg)
    op = orc.OracleProblem(atm, q)
    rng = np.random.default_rng(7)
    ray0, nray, f0, nf = 5, 9, 2, 4
    st = rng.normal(size=(nray, nf, op.N, 4))
    st[..., 0] += 3.0
    lam = rng.uniform(0, 1, size=(nray, nf, op.N))
    dt = np.float64 if prec == porta.F64 else np.float32
    st, lam = st.astype(dt).astype(np.float64), lam.astype(dt).astype(np.float64)
    ref = orc.jkq_accumulate(op, ray0, f0, st, lam)
    hg = porta.HostGrid.from_inputs(atm, q)
    tdt = torch.float64 if prec == porta.F64 else torch.float32
    got = porta.jkq_accumulate(hg, ray0, f0, to_dev(st, tdt), to_dev(lam, tdt), prec=prec)
    torch.cuda.synchronize()
    compare_jkq(got.cpu().numpy(), ref, 1e-13, "jkq_accumulate")


@pytest.mark.parametrize("magnetic", [True, False])
def test_see_update_matches_oracle(orc, magnetic):
    torch = require_gpu()
    atm, q, ref = oracle_full("C1", 0, "f64", magnetic)
    s_ref, e_ref, rc_ref = orc.see_update(ref["jkq"], atm.source, atm)
    for prec in (porta.F64, porta.F32):
        tdt = torch.float64 if prec == porta.F64 else torch.float32
        emis = torch.empty((6, atm.npoints), dtype=tdt, device="cuda")
        s_new, _, rc = porta.see_update(
            to_dev(ref["jkq"], torch.float64), to_dev(atm.source, torch.float64), atm.eps_c,
            atm.delta2, atm.w2, atm.planck,
            hanle=None if atm.hanle is None else to_dev(atm.hanle, torch.float64),
            bhat=None if atm.bhat is None else to_dev(atm.bhat, torch.float64),
            kappa=to_dev(atm.kappa, tdt), emis_out=emis, prec=prec)
        torch.cuda.synchronize()
        np.testing.assert_allclose(s_new.cpu().numpy(), s_ref, rtol=1e-12, atol=1e-14)
        # emis_out = kappa * S_new, in the sweep precision
        e = emis.cpu().numpy().astype(np.float64) / atm.kappa.astype(tdt == torch.float32 and
                                                                     np.float32 or np.float64)
        if prec == porta.F64:
            np.testing.assert_allclose(e, s_ref, rtol=1e-12, atol=1e-14)
        else:
            np.testing.assert_allclose(e, s_ref, rtol=1e-6, atol=1e-7 * np.abs(s_ref).max())
        assert rc.item() == pytest.approx(rc_ref, rel=1e-12)


def test_jacobi_iterations_c1_match_oracle(orc):
    """Five Jacobi iterations (sweep + J + SEE) in FP64 on the GPU and on the oracle."""
    torch = require_gpu()
    atm = inputs.make_atmosphere(inputs.CONFIGS["C1"], seed=1, magnetic=True)
    q = inputs.make_quadrature(inputs.CONFIGS["C1"])
    case = Case(atm, q, porta.F64)
    S = to_dev(atm.source, torch.float64)
    hanle, bhat = to_dev(atm.hanle, torch.float64), to_dev(atm.bhat, torch.float64)
    s_host = atm.source.copy()
    emis_host = atm.emis.copy()
    for it in range(5):
        jkq, _ = porta.fs_sweep(case.hg, case.kappa, case.prop, case.emis, atm.i_bottom, atm.w2,
                                want_itop=False)
        S, _, rc = porta.see_update(jkq, S, atm.eps_c, atm.delta2, atm.w2, atm.planck, hanle,
                                    bhat, kappa=case.kappa, emis_out=case.emis)
        torch.cuda.synchronize()
        ref = orc.fs_sweep(orc.OracleProblem(dataclasses.replace(atm, emis=emis_host), q),
                           want_itop=False)
        s_host, emis_host, rc_ref = orc.see_update(ref["jkq"], s_host, atm)
        np.testing.assert_allclose(S.cpu().numpy(), s_host, rtol=1e-10, atol=1e-12)
        assert rc.item() == pytest.approx(rc_ref, rel=1e-8)


@pytest.mark.parametrize("prec", [porta.F64, porta.F32])
def test_bezier2d_mode_matches_oracle(orc, prec):
    """Mode B (9-point monotonic Bezier at M and P) on the 16x16x32 instance and a ragged
    plane, against the oracle's interpolation mode 1: FP64 to the FP64 bars, FP32 on
    Stokes I (2e-5) and J (2e-5 of J00).  The FP32 bar on Q/I, U/I, V/I (1e-7) is not met
    in this mode; test_bezier2d_mode_fp32_polarization_bar records that."""
    import torch
    for cfg, seed in ((inputs.CONFIGS["C1"], 0), (inputs.Config("rag", 7, 5, 9, 2, 3, 5, True), 4)):
        atm = inputs.make_atmosphere(cfg, seed=seed)
        if cfg.name == "rag":
            atm = dataclasses.replace(atm, lx=530.0, ly=410.0)
        if prec == porta.F32:
            atm = rounded(atm, np.float32)
        q = inputs.make_quadrature(cfg)
        ref = orc.fs_sweep(orc.OracleProblem(atm, q, interp=1))
        jkq, itop = Case(atm, q, prec).sweep(interp=porta.BEZIER2D)
        want = up_rays(ref["itop"], q)
        what = f"bezier2d {cfg.name}"
        if prec == porta.F64:
            compare_stokes(itop, want, 1e-10, 1e-12, what)
            compare_jkq(jkq, ref["jkq"], 1e-10, what)
        else:
            rel = np.abs(itop[..., 0] - want[..., 0]) / np.abs(want[..., 0])
            assert rel.max() <= 2e-5, f"{what} Stokes I max rel err {rel.max():.3e}"
            compare_jkq(jkq, ref["jkq"], 2e-5, what)
        # and it is a different interpolation from the bilinear one
        _, it_bl = Case(atm, q, prec).sweep()
        assert np.abs(it_bl - itop).max() > 1e-6
        torch.cuda.synchronize()


@pytest.mark.xfail(strict=True, reason=(
    "FP32 9-point Bezier mode misses the 1e-7 bar on Q/I, U/I, V/I (measured up to 4.2e-7; "
    "2.8e-7 with the interpolation evaluated in FP64 on the FP32 plane states): the "
    "per-component clamps amplify the rounding of the FP32 plane states, so the bar needs "
    "FP64 states, i.e. the FP64 sweep"))
def test_bezier2d_mode_fp32_polarization_bar(orc):
    """The FP32 bar of Q/I, U/I, V/I (1e-7 absolute against the oracle on the same
    FP32-rounded inputs) in the 9-point Bezier mode, 16x16x32 instance."""
    cfg = inputs.CONFIGS["C1"]
    atm = rounded(inputs.make_atmosphere(cfg, seed=0), np.float32)
    q = inputs.make_quadrature(cfg)
    ref = up_rays(orc.fs_sweep(orc.OracleProblem(atm, q, interp=1), want_j=False)["itop"], q)
    _, itop = Case(atm, q, porta.F32).sweep(interp=porta.BEZIER2D, want_jkq=False)
    worst = max(float(np.abs(itop[..., s] / itop[..., 0] - ref[..., s] / ref[..., 0]).max())
                for s in (1, 2, 3))
    print(f"bezier2d FP32 Q/I, U/I, V/I max abs err {worst:.3e}")
    assert worst <= 1e-7


@pytest.mark.parametrize("prec", [porta.F64, porta.F32])
def test_parabolic_control_point_matches_oracle(orc, prec):
    """porta_options.control = PARABOLIC (the parabola through M, O, P, as DELOPAR
    interpolates the source function) against the oracle's control = 1, also combined
    with the 9-point interpolation in FP64."""
    import torch
    tol_i, tol_p = (1e-10, 1e-12) if prec == porta.F64 else (2e-5, 1e-7)
    opts = porta.options(control=porta.CONTROL_PARABOLIC)
    cases = [(inputs.CONFIGS["C1"], 0, porta.BILINEAR),
             (inputs.Config("rag", 7, 5, 9, 2, 3, 5, True), 4, porta.BILINEAR)]
    if prec == porta.F64:
        cases.append((inputs.Config("rag", 7, 5, 9, 2, 3, 5, True), 4, porta.BEZIER2D))
    for cfg, seed, interp in cases:
        atm = inputs.make_atmosphere(cfg, seed=seed)
        if cfg.name == "rag":
            atm = dataclasses.replace(atm, lx=530.0, ly=410.0)
        if prec == porta.F32:
            atm = rounded(atm, np.float32)
        q = inputs.make_quadrature(cfg)
        ref = orc.fs_sweep(orc.OracleProblem(atm, q, interp=interp, control=1))
        jkq, itop = Case(atm, q, prec).sweep(interp=interp, opts=opts)
        what = f"parabolic {cfg.name} interp {interp}"
        compare_stokes(itop, up_rays(ref["itop"], q), tol_i, tol_p, what)
        compare_jkq(jkq, ref["jkq"], tol_i, what)
        _, it_b = Case(atm, q, prec).sweep(interp=interp)
        assert np.abs(it_b - itop).max() > 1e-8       # BESSER clamps somewhere
        torch.cuda.synchronize()


@pytest.mark.parametrize("prec", [porta.F64, porta.F32])
def test_intensity_only_sweep_matches_oracle(orc, prec):
    """opts.stokes = 1 (the unpolarized problem: K' = 0, emission eps^0_0) on the full
    synthetic model, whose propagation matrix and K = 2 emissivities it must ignore,
    against the oracle on the same model with those set to zero (where Q = U = V = 0):
    Stokes I at the top, every J^K_Q (from I alone) and Lambda-bar."""
    import torch
    tol = 1e-10 if prec == porta.F64 else 2e-5
    cases = [(inputs.CONFIGS["C1"], 0, porta.options(stokes=1)),
             (inputs.Config("rag", 7, 5, 9, 2, 3, 5, True), 4,
              porta.options(ray_batch=3, block=64, stokes=1, control=porta.CONTROL_PARABOLIC))]
    for cfg, seed, opts in cases:
        atm = inputs.make_atmosphere(cfg, seed=seed)
        if cfg.name == "rag":
            atm = dataclasses.replace(atm, lx=530.0, ly=410.0)
        if prec == porta.F32:
            atm = rounded(atm, np.float32)
        q = inputs.make_quadrature(cfg)
        emis0 = atm.emis.copy()
        emis0[1:] = 0.0
        ref_atm = dataclasses.replace(atm, propmat=0 * atm.propmat, emis=emis0)
        ref = orc.fs_sweep(orc.OracleProblem(ref_atm, q, control=opts.control))
        want = up_rays(ref["itop"], q)
        assert np.abs(want[..., 1:]).max() == 0.0
        jkq, itop = Case(atm, q, prec).sweep(opts=opts)
        assert itop.shape == want.shape[:-1]
        rel = np.abs(itop - want[..., 0]) / np.abs(want[..., 0])
        assert rel.max() <= tol, f"{cfg.name}: I max rel err {rel.max():.3e}"
        compare_jkq(jkq, ref["jkq"], tol, f"intensity-only {cfg.name}")
        torch.cuda.synchronize()


@pytest.mark.parametrize("prec", [porta.F64, porta.F32])
def test_ray_ranges_sum_to_the_full_sweep(prec):
    """Calls over ray ranges that split the enumeration (one straddles the hemispheres,
    none aligned with the ray batches) give the one-call sweep: each writes its own rows
    of I_top, bitwise, and J summed with accumulate = 1 matches up to summation order."""
    torch = require_gpu()
    cfg = inputs.Config("sub", 7, 5, 9, 2, 3, 5, True)
    atm = dataclasses.replace(inputs.make_atmosphere(cfg, seed=6), lx=530.0, ly=410.0)
    if prec == porta.F32:
        atm = rounded(atm, np.float32)
    q = inputs.make_quadrature(cfg)
    case = Case(atm, q, prec)
    ref_j, ref_t = case.sweep(opts=porta.options(ray_batch=2))
    nh = case.hg.nray_up
    jkq = torch.full((10, case.hg.N), float("nan"), dtype=torch.float64, device="cuda")
    itop = torch.full(ref_t.shape, float("nan"), dtype=case.dt, device="cuda")
    for i, (first, count) in enumerate(((nh + 3, nh - 3), (0, 3), (3, nh))):
        porta.fs_sweep(case.hg, case.kappa, case.prop, case.emis, atm.i_bottom, atm.w2,
                       prec=prec, jkq=jkq, accumulate=i > 0, i_top=itop,
                       opts=porta.options(ray_batch=2, ray_first=first, ray_count=count))
    torch.cuda.synchronize()
    assert np.array_equal(itop.cpu().numpy(), ref_t)
    np.testing.assert_allclose(jkq.cpu().numpy(), ref_j, rtol=1e-13,
                               atol=1e-15 * np.abs(ref_j).max())
    # a downward-only range leaves I_top alone
    itop2 = itop.clone()
    porta.fs_sweep(case.hg, case.kappa, case.prop, case.emis, atm.i_bottom, atm.w2, prec=prec,
                   i_top=itop2, want_jkq=False, opts=porta.options(ray_first=nh, ray_count=nh))
    torch.cuda.synchronize()
    assert torch.equal(itop, itop2)


@pytest.mark.parametrize("prec", [porta.F64, porta.F32])
def test_check_inputs_option(prec):
    """opts.check_inputs: valid fields pass and give the unchecked result; a NaN
    emissivity, an infinite propagation-matrix entry or eta_I <= 0 at one point make
    the sweep and the adjoint return PORTA_ENONFINITE before any other launch; without
    the option nothing is checked."""
    torch = require_gpu()
    atm, q, _ = oracle_full("C1", 0, "f64")
    case = Case(atm, q, prec)
    chk = porta.options(check_inputs=True)
    j0, t0 = case.sweep()
    j1, t1 = case.sweep(opts=chk)
    assert np.array_equal(j0, j1) and np.array_equal(t0, t1)
    seed = torch.ones_like(torch.as_tensor(t0, device="cuda"))
    porta.fs_adjoint(case.hg, case.kappa, case.prop, case.emis, atm.i_bottom, seed, atm.w2,
                     prec=prec, checkpoint_stride=4, opts=chk)
    p = 1234
    for name, field, value in (("emis", case.emis, float("nan")),
                               ("propmat", case.prop, float("inf")),
                               ("kappa", case.kappa, 0.0)):
        saved = field.clone()
        field.view(-1)[p] = value
        for call in ("sweep", "adjoint"):
            with pytest.raises(porta.PortaError) as err:
                if call == "sweep":
                    porta.fs_sweep(case.hg, case.kappa, case.prop, case.emis, atm.i_bottom,
                                   atm.w2, prec=prec, opts=chk)
                else:
                    porta.fs_adjoint(case.hg, case.kappa, case.prop, case.emis, atm.i_bottom,
                                     seed, atm.w2, prec=prec, checkpoint_stride=4, opts=chk)
            assert err.value.status == porta.ENONFINITE, (name, call)
        if name == "emis":
            # unchecked, the sweep runs and the NaN reaches J
            j, _ = porta.fs_sweep(case.hg, case.kappa, case.prop, case.emis, atm.i_bottom,
                                  atm.w2, prec=prec)
            torch.cuda.synchronize()
            assert torch.isnan(j).any()
        field.copy_(saved)
    torch.cuda.synchronize()


def test_jacobi_save_and_resume_is_exact(tmp_path):
    """Six Jacobi iterations in one go equal three, a save to disk, a fresh solver
    loading the file and three more: S^K_Q, emissivities and the R_c history bitwise
    (the iteration is deterministic).  A file for another grid is refused."""
    torch = require_gpu()
    from paper_1307_4217_amd.jacobi import JacobiSolver
    atm, q, _ = oracle_full("C1", 0, "f64")
    for prec in (porta.F64, porta.F32):
        a = JacobiSolver(atm, q, prec)
        a.solve(6, tol=0.0)
        b = JacobiSolver(atm, q, prec)
        b.solve(3, tol=0.0)
        path = str(tmp_path / f"it{prec}.npz")
        b.save(path)
        c = JacobiSolver(atm, q, prec)
        c.load(path)
        assert c.iteration == 3
        c.solve(3, tol=0.0)
        torch.cuda.synchronize()
        assert torch.equal(a.source, c.source) and torch.equal(a.emis, c.emis)
        assert a.history == c.history and c.iteration == 6
    other = dataclasses.replace(atm, nx=atm.nx // 2, kappa=atm.kappa[: atm.npoints // 2],
                                propmat=atm.propmat[:, : atm.npoints // 2],
                                emis=atm.emis[:, : atm.npoints // 2],
                                source=atm.source[:, : atm.npoints // 2],
                                hanle=None, bhat=None)
    with pytest.raises(ValueError):
        JacobiSolver(other, q, porta.F32).load(path)


def test_jacobi_switches_sweep_precision(tmp_path):
    """Three FP32 iterations, set_precision(F64) and three FP64 ones equal three FP32
    iterations saved to disk, loaded by an FP64 solver and continued (the emissivities
    formed from S^K_Q by porta_emissivity in both): S^K_Q, emissivities and R_c history
    bitwise.  After the switch the iterate is the all-FP64 one up to the FP32 rounding
    of the first iterations, which the contraction of the iteration damps."""
    torch = require_gpu()
    from paper_1307_4217_amd.jacobi import JacobiSolver
    atm, q, _ = oracle_full("C1", 0, "f64")
    a = JacobiSolver(atm, q, porta.F32)
    a.solve(3, tol=0.0)
    a.set_precision(porta.F64)
    assert a.prec == porta.F64 and a.emis.dtype == torch.float64
    a.solve(3, tol=0.0)
    b = JacobiSolver(atm, q, porta.F32)
    b.solve(3, tol=0.0)
    path = str(tmp_path / "it32.npz")
    b.save(path)
    c = JacobiSolver(atm, q, porta.F64)
    c.load(path)
    c.solve(3, tol=0.0)
    d = JacobiSolver(atm, q, porta.F64)
    d.solve(6, tol=0.0)
    torch.cuda.synchronize()
    assert torch.equal(a.source, c.source) and torch.equal(a.emis, c.emis)
    assert a.history == c.history and c.iteration == 6
    err = float(((a.source - d.source).abs().max() / d.source[0].abs().max()).item())
    print(f"FP32 x 3 then FP64 x 3 vs FP64 x 6: max |dS| / max S00 = {err:.2e}")
    assert err < 1e-4
