"""GPU sweep with M and P on the first face crossed (options.faces = 1, Sect. 3.1)
against the oracle's first-face mode (faces = 1), through the C ABI.

The oracle solves each plane to its periodic fixed point by passes to 1e-15; the GPU
marches across the plane from a guess started far enough upstream that the guess is
damped below the rounding of the sweep precision.  Bars: FP64 1e-10 relative on I,
1e-12 on Q/I, U/I, V/I and on J (of the J00 scale); FP32 2e-5, 1e-7, 2e-5."""
import dataclasses

import numpy as np
import pytest

from gpu_common import Case, compare_jkq, compare_stokes, require_gpu, rounded, to_dev, up_rays
from paper_1307_4217_amd import inputs, porta

pytestmark = pytest.mark.gpu


def _face_kinds(atm, q):
    """Kind of the first face crossed upwind on the first interior plane, per upward ray:
    0 the plane below, 1 an x face, 2 a y face (uniform z spacing)."""
    dz = atm.z[1] - atm.z[0]
    dx, dy = atm.lx / atm.nx, atm.ly / atm.ny
    kinds = []
    for a, mu in enumerate(q.mu):
        st = np.sqrt(1 - mu * mu)
        for m in range(q.nchi):
            chi = (m + 0.5) * 2 * np.pi / q.nchi
            sz, sx = dz / mu, dx / max(abs(st * np.cos(chi)), 1e-300)
            sy = dy / max(abs(st * np.sin(chi)), 1e-300)
            kinds.append(0 if sz <= min(sx, sy) else (1 if sx <= sy else 2))
    return np.array(kinds)


@pytest.mark.parametrize("prec", [porta.F64, porta.F32])
def test_first_face_sweep_c1_matches_oracle(orc, prec):
    """16x16x32, 80 rays, 21 frequencies: I_top of every upward ray, J^K_Q and
    Lambda-bar.  On this grid the two most inclined of the five inclinations reach
    vertical faces (x and y faces both occur)."""
    cfg = inputs.CONFIGS["C1"]
    atm = inputs.make_atmosphere(cfg, seed=0)
    if prec == porta.F32:
        atm = rounded(atm, np.float32)
    q = inputs.make_quadrature(cfg)
    kinds = _face_kinds(atm, q)
    assert {0, 1, 2} <= set(kinds.tolist())
    ref = orc.fs_sweep(orc.OracleProblem(atm, q, faces=1))
    jkq, itop = Case(atm, q, prec).sweep(opts=porta.options(faces=1))
    tol_i, tol_p = (1e-10, 1e-12) if prec == porta.F64 else (2e-5, 1e-7)
    ei, ep = compare_stokes(itop, up_rays(ref["itop"], q), tol_i, tol_p, "faces C1")
    ej = compare_jkq(jkq, ref["jkq"], tol_i if prec == porta.F64 else 2e-5, "faces C1")
    print(f"first-face sweep C1 {'FP64' if prec == porta.F64 else 'FP32'}: I {ei:.2e}, "
          f"Q/I.. {ep:.2e}, J {ej:.2e}")
    # and it is a different solution from the plane-hop one on the inclined rays
    _, it0 = Case(atm, q, prec).sweep()
    assert np.abs(it0 - itop)[kinds != 0].max() > 1e-3 * np.abs(itop).max()


@pytest.mark.parametrize("prec", [porta.F64, porta.F32])
@pytest.mark.parametrize("ray_batch", [0, 3])
def test_first_face_sweep_ragged_grid(orc, prec, ray_batch):
    """A 7x5 plane (lanes and march of different lengths in the two orientations),
    unequal z steps, lx != ly, 3 azimuths, partial ray batches, parabolic control point
    on one of the cases."""
    cfg = inputs.Config("ragged", 7, 5, 9, 2, 3, 5, True)
    atm = inputs.make_atmosphere(cfg, seed=3)
    z = np.cumsum(np.r_[0.0, np.random.default_rng(9).uniform(40.0, 160.0, cfg.nz - 1)])
    atm = dataclasses.replace(atm, lx=530.0, ly=410.0, z=z)
    if prec == porta.F32:
        atm = rounded(atm, np.float32)
    q = inputs.make_quadrature(cfg)
    control = 1 if ray_batch == 3 else 0
    ref = orc.fs_sweep(orc.OracleProblem(atm, q, faces=1, control=control))
    jkq, itop = Case(atm, q, prec).sweep(opts=porta.options(faces=1, ray_batch=ray_batch,
                                                            control=control))
    tol_i, tol_p = (1e-10, 1e-12) if prec == porta.F64 else (2e-5, 1e-7)
    compare_stokes(itop, up_rays(ref["itop"], q), tol_i, tol_p, "faces ragged")
    compare_jkq(jkq, ref["jkq"], tol_i if prec == porta.F64 else 2e-5, "faces ragged")


@pytest.mark.parametrize("prec", [porta.F64, porta.F32])
def test_first_face_sweep_rows_span_several_wavefronts(orc, prec):
    """A 130x70 plane: 3 wavefronts of lanes for the rays that meet a y face first and 2
    (the exchanged frame) for those that meet an x face first, the last one ragged in
    both, so the in-plane corners of a row cross between wavefronts and around the
    periodic box; the steep rays reach the plane below first."""
    cfg = inputs.Config("wide", 130, 70, 6, 2, 6, 3, True)
    atm = inputs.make_atmosphere(cfg, seed=4)
    atm = dataclasses.replace(atm, lx=13000.0, ly=7000.0, z=np.arange(cfg.nz) * 100.0)
    if prec == porta.F32:
        atm = rounded(atm, np.float32)
    q = inputs.make_quadrature(cfg)
    assert {0, 1, 2} <= set(_face_kinds(atm, q).tolist())
    ref = orc.fs_sweep(orc.OracleProblem(atm, q, faces=1))
    jkq, itop = Case(atm, q, prec).sweep(opts=porta.options(faces=1))
    tol_i, tol_p = (1e-10, 1e-12) if prec == porta.F64 else (2e-5, 1e-7)
    ei, ep = compare_stokes(itop, up_rays(ref["itop"], q), tol_i, tol_p, "faces wide")
    ej = compare_jkq(jkq, ref["jkq"], tol_i if prec == porta.F64 else 2e-5, "faces wide")
    print(f"first-face sweep 130x70 {'FP64' if prec == porta.F64 else 'FP32'}: I {ei:.2e}, "
          f"Q/I.. {ep:.2e}, J {ej:.2e}")


@pytest.mark.parametrize("prec", [porta.F64, porta.F32])
def test_first_face_sweep_widest_rows(orc, prec):
    """A 504x8 plane, the widest rows of the benchmark grids (blocks of 512 lanes, eight
    wavefronts, the last one ragged; in the exchanged frame rows of 8 lanes and a march
    of 504 rows), all three first faces."""
    cfg = inputs.Config("wide504", 504, 8, 6, 2, 6, 3, True)
    atm = inputs.make_atmosphere(cfg, seed=6)
    atm = dataclasses.replace(atm, lx=504 * 100.0, ly=800.0, z=np.arange(cfg.nz) * 100.0)
    if prec == porta.F32:
        atm = rounded(atm, np.float32)
    q = inputs.make_quadrature(cfg)
    assert {0, 1, 2} <= set(_face_kinds(atm, q).tolist())
    ref = orc.fs_sweep(orc.OracleProblem(atm, q, faces=1))
    jkq, itop = Case(atm, q, prec).sweep(opts=porta.options(faces=1))
    tol_i, tol_p = (1e-10, 1e-12) if prec == porta.F64 else (2e-5, 1e-7)
    ei, ep = compare_stokes(itop, up_rays(ref["itop"], q), tol_i, tol_p, "faces 504x8")
    ej = compare_jkq(jkq, ref["jkq"], tol_i if prec == porta.F64 else 2e-5, "faces 504x8")
    print(f"first-face sweep 504x8 {'FP64' if prec == porta.F64 else 'FP32'}: I {ei:.2e}, "
          f"Q/I.. {ep:.2e}, J {ej:.2e}")


def test_first_face_march_goes_around_a_short_plane_many_times(orc):
    """Rows of 16 nodes, 4 of them in the march direction, rays down to mu = 0.047: the
    guess needs ~760 rows of warm-up (t_z = 0.047) to fall below the FP64 unit roundoff,
    i.e. more than 190 times around the box (FP64 bar)."""
    cfg = inputs.Config("short", 16, 4, 6, 5, 8, 2, True)
    atm = inputs.make_atmosphere(cfg, seed=7)
    atm = dataclasses.replace(atm, lx=1600.0, ly=400.0, z=np.arange(cfg.nz) * 100.0)
    q = inputs.make_quadrature(cfg)
    assert q.mu.min() < 0.05 and 2 in set(_face_kinds(atm, q).tolist())
    ref = orc.fs_sweep(orc.OracleProblem(atm, q, faces=1))
    jkq, itop = Case(atm, q, porta.F64).sweep(opts=porta.options(faces=1))
    ei, ep = compare_stokes(itop, up_rays(ref["itop"], q), 1e-10, 1e-12, "faces short")
    compare_jkq(jkq, ref["jkq"], 1e-10, "faces short")
    print(f"first-face sweep 16x4: I {ei:.2e}, Q/I.. {ep:.2e}")


@pytest.mark.parametrize("shape", [(1, 1, 5), (1, 4, 5), (3, 1, 5), (4, 3, 2)])
def test_first_face_sweep_degenerate_grids(orc, shape):
    """A single column, a single row in either direction (the neighbouring row or column
    of a face is the node's own), and one layer (nz = 2): FP64 against the oracle."""
    nx, ny, nz = shape
    cfg = inputs.Config("degenerate", nx, ny, nz, 3, 4, 2, True)
    atm = inputs.make_atmosphere(cfg, seed=8)
    atm = dataclasses.replace(atm, lx=nx * 100.0, ly=ny * 100.0, z=np.arange(nz) * 150.0)
    q = inputs.make_quadrature(cfg)
    assert {0, 1, 2} <= set(_face_kinds(atm, q).tolist())
    ref = orc.fs_sweep(orc.OracleProblem(atm, q, faces=1))
    jkq, itop = Case(atm, q, porta.F64).sweep(opts=porta.options(faces=1))
    compare_stokes(itop, up_rays(ref["itop"], q), 1e-10, 1e-12, f"faces {shape}")
    compare_jkq(jkq, ref["jkq"], 1e-10, f"faces {shape}")


def test_first_face_sweep_over_ray_ranges_adds_up():
    """Two calls over ray ranges (one straddling the hemispheres), J accumulated, give
    the single call's I_top bitwise and its J to its summation order."""
    torch = require_gpu()
    cfg = inputs.Config("ranges", 9, 7, 6, 2, 5, 3, True)
    atm = inputs.make_atmosphere(cfg, seed=9)
    atm = dataclasses.replace(atm, lx=900.0, ly=700.0, z=np.arange(cfg.nz) * 120.0)
    q = inputs.make_quadrature(cfg)
    case = Case(atm, q, porta.F64)
    j1, it1 = case.sweep(opts=porta.options(faces=1))
    nray = 2 * len(q.mu) * q.nchi
    jkq = torch.zeros((10, atm.npoints), dtype=torch.float64, device="cuda")
    itop = torch.full(it1.shape, float("nan"), dtype=torch.float64, device="cuda")
    for k, (first, count) in enumerate(((0, 7), (7, nray - 7))):
        porta.fs_sweep(case.hg, case.kappa, case.prop, case.emis, atm.i_bottom, atm.w2,
                       prec=porta.F64, jkq=jkq, accumulate=k > 0, i_top=itop,
                       opts=porta.options(faces=1, ray_first=first, ray_count=count,
                                          ray_batch=3))
    torch.cuda.synchronize()
    assert np.array_equal(itop.cpu().numpy(), it1)
    np.testing.assert_allclose(jkq.cpu().numpy(), j1, rtol=1e-13, atol=1e-15 * np.abs(j1).max())


def test_first_face_sweep_equals_plane_hops_where_every_face_is_horizontal():
    """Rays that reach the plane below (and above) within one cell on every plane: the
    first face is that plane, so the two sweeps compute the same arithmetic up to
    rounding: the compiler fuses multiply-adds differently in the two kernels, J is summed
    in another order, and a ray that would meet an x face before a y face is solved with
    x and y exchanged, which sums the four terms of each bilinear interpolation in
    another order (relative differences of a few units in the last place per plane)."""
    torch = require_gpu()
    cfg = inputs.Config("steep", 8, 8, 10, 3, 4, 6, True)
    atm = inputs.make_atmosphere(cfg, seed=5)
    q = inputs.make_quadrature(cfg)
    dz = 100.0
    dx = 1.2 * dz * np.sqrt(1 - q.mu.min() ** 2) / q.mu.min()   # wider than the widest hop
    atm = dataclasses.replace(atm, lx=8 * dx, ly=8 * dx, z=np.arange(cfg.nz) * dz)
    assert np.all(_face_kinds(atm, q) == 0)
    case = Case(atm, q, porta.F64)
    j1, it1 = case.sweep(opts=porta.options(faces=1))
    j0, it0 = case.sweep()
    torch.cuda.synchronize()
    np.testing.assert_allclose(it1, it0, rtol=1e-13, atol=1e-15 * np.abs(it0).max())
    np.testing.assert_allclose(j1, j0, rtol=1e-13, atol=1e-15 * np.abs(j0).max())


def test_first_face_sweep_full_size_sampled(orc):
    """256x256x128, 160 rays, 101 frequencies, in the launch configuration the benchmark
    times (a hemisphere of rays per launch, the default frequency chunks): I_top over the
    whole top surface for 8 upward rays (the most inclined ones meeting x faces and y
    faces, intermediate ones, steep ones whose first face is the plane below) at line
    centre and in the wing, FP32 and FP64 sweeps of the same FP32-rounded inputs against
    the oracle's first-face mode on those pairs."""
    torch = require_gpu()
    cfg = inputs.CONFIGS["C3"]
    atm = rounded(inputs.make_atmosphere(cfg, seed=0), np.float32)
    q = inputs.make_quadrature(cfg)
    rays, freqs = [0, 4, 17, 21, 38, 55, 64, 75], [50, 10]
    kinds = _face_kinds(atm, q)[rays]
    assert {0, 1, 2} <= set(kinds.tolist())
    ref = orc.fs_sweep(orc.OracleProblem(atm, q, faces=1), rays=rays, freqs=freqs,
                       want_j=False)["itop"]
    print("  oracle done", flush=True)
    for prec, tol_i, tol_p in ((porta.F32, 2e-5, 1e-7), (porta.F64, 1e-10, 1e-12)):
        case = Case(atm, q, prec)
        _, itop = porta.fs_sweep(case.hg, case.kappa, case.prop, case.emis, atm.i_bottom,
                                 atm.w2, prec=prec, want_jkq=False,
                                 opts=porta.options(faces=1))
        got = itop[rays][:, freqs].cpu().numpy().astype(np.float64)
        name = "FP32" if prec == porta.F32 else "FP64"
        ei, ep = compare_stokes(got, ref, tol_i, tol_p, f"faces C3 {name}")
        print(f"first-face sweep C3 {name}, {len(rays)} rays x {len(freqs)} frequencies x "
              f"{cfg.nx * cfg.ny} top points: I {ei:.2e}, Q/I.. {ep:.2e}", flush=True)
        del case, itop
        torch.cuda.empty_cache()


def test_first_face_fp32_every_output_full_size():
    """256x256x128, 160 rays, 101 frequencies: the FP32 first-face sweep against the FP64
    one of the same FP32-rounded inputs (pinned to the oracle by
    test_first_face_sweep_full_size_sampled) over every top point, upward ray and
    frequency: 2e-5 on I, 1e-7 on Q/I, U/I, V/I.  The line wings of the most inclined
    rays, where the change of I per cell step falls below half a unit in the last place
    of an FP32 I, are where an FP32 in-plane chain fails this (4.4e-5)."""
    torch = require_gpu()
    torch.cuda.empty_cache()
    cfg = inputs.CONFIGS["C3"]
    atm = rounded(inputs.make_atmosphere(cfg, seed=0), np.float32)
    q = inputs.make_quadrature(cfg)
    hg = porta.HostGrid.from_inputs(atm, q)
    its = []
    for prec, dt in ((porta.F32, torch.float32), (porta.F64, torch.float64)):
        _, it = porta.fs_sweep(hg, to_dev(atm.kappa, dt), to_dev(atm.propmat, dt),
                               to_dev(atm.emis, dt), atm.i_bottom, atm.w2, prec=prec,
                               want_jkq=False, opts=porta.options(faces=1))
        its.append(it)
    ei = ep = 0.0
    for r in range(its[1].shape[0]):
        a, b = its[0][r].double(), its[1][r]
        ei = max(ei, float(((a[..., 0] - b[..., 0]).abs() / b[..., 0].abs()).max()))
        ep = max(ep, float((a[..., 1:] / a[..., :1] - b[..., 1:] / b[..., :1]).abs().max()))
    del its
    torch.cuda.empty_cache()
    print(f"first-face C3 FP32 vs FP64, every output: I {ei:.2e}, Q/I.. {ep:.2e}")
    assert ei <= 2e-5 and ep <= 1e-7
