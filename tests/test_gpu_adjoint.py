"""GPU adjoint (porta_fs_adjoint) against complex-step derivatives of the FP64
CPU oracle, central finite differences of the GPU forward, and itself."""
import dataclasses

import numpy as np
import pytest

from gpu_common import (Case, compare_jkq, compare_stokes, require_gpu, rounded, to_dev,
                        up_rays)
from paper_1307_4217_amd import inputs, porta

pytestmark = pytest.mark.gpu


def seed_for(case, rng, sparse=None):
    """Random dL/dI_top in the i_top layout (optionally nonzero only on some (ray, freq))."""
    hg = case.hg
    w = rng.normal(size=(hg.nray_up, hg.nfreq, hg.ny, hg.nx, 4))
    if sparse is not None:
        mask = np.zeros((hg.nray_up, hg.nfreq, 1, 1, 1))
        for r, f in sparse:
            mask[r, f] = 1.0
        w *= mask
    dt = np.float64 if case.prec == porta.F64 else np.float32
    return w.astype(dt).astype(np.float64)


def gpu_grad(case, w, stride=3, opts=None):
    torch = require_gpu()
    g = porta.fs_adjoint(case.hg, case.kappa, case.prop, case.emis, case.atm.i_bottom,
                         to_dev(w, case.dt), case.atm.w2, prec=case.prec,
                         checkpoint_stride=stride, opts=opts)
    torch.cuda.synchronize()
    return [x.cpu().numpy().astype(np.float64) for x in g]


def oracle_directional(orc, atm, q, w, dk, dp, de, pairs=None, control=0):
    """<w, d I_top> along (dk, dp, de) by complex step on the oracle."""
    op = orc.OracleProblem(atm, q, control=control)
    nup = len(q.mu) * q.nchi
    if pairs is None:
        rays, freqs = np.arange(nup), np.arange(len(q.phi))
        _, im = orc.fs_sweep_cs(op, dk, dp, de, h=1e-30, rays=rays, freqs=freqs)
        return float(np.sum(w * im) / 1e-30)
    rays = sorted({r for r, _ in pairs})
    freqs = sorted({f for _, f in pairs})
    _, im = orc.fs_sweep_cs(op, dk, dp, de, h=1e-30, rays=rays, freqs=freqs)
    return float(sum(np.sum(w[r, f] * im[rays.index(r), freqs.index(f)]) for r, f in pairs)
                 / 1e-30)


def tiny_case(prec, seed=11, nx=4, ny=3, nz=5):
    cfg = inputs.Config("adj", nx, ny, nz, 2, 4, 3, False)
    atm = inputs.make_atmosphere(cfg, seed=seed)
    atm = dataclasses.replace(atm, lx=900.0, ly=700.0, z=np.linspace(0, 1000, nz))
    if prec == porta.F32:
        atm = rounded(atm, np.float32)
    return atm, inputs.make_quadrature(cfg)


@pytest.mark.parametrize("stride", [1, 2, 4])
def test_adjoint_fp64_every_component_matches_complex_step(orc, stride):
    atm, q = tiny_case(porta.F64)
    case = Case(atm, q, porta.F64)
    w = seed_for(case, np.random.default_rng(1))
    gk, gp, ge = gpu_grad(case, w, stride=stride)
    got = np.concatenate([gk[None], gp, ge])          # [13][N]
    n = atm.npoints
    ref = np.zeros((13, n))
    zero1, zero6 = np.zeros(n), np.zeros((6, n))
    for c in range(13):
        for pnt in range(n):
            dk, dp, de = zero1.copy(), zero6.copy(), zero6.copy()
            if c == 0:
                dk[pnt] = 1.0
            elif c < 7:
                dp[c - 1, pnt] = 1.0
            else:
                de[c - 7, pnt] = 1.0
            ref[c, pnt] = oracle_directional(orc, atm, q, w, dk, dp, de)
    scale = np.abs(ref).max()
    err = np.abs(got - ref).max(axis=1) / scale
    assert err.max() < 1e-10, err


@pytest.mark.parametrize("prec, tol", [(porta.F64, 1e-10), (porta.F32, 2e-5)])
def test_adjoint_dot_product_c1(orc, prec, tol):
    """<J^T w, v> from the GPU against d/dh <w, I_top(p + h v)> from the oracle (C1)."""
    atm = inputs.make_atmosphere(inputs.CONFIGS["C1"], seed=0)
    if prec == porta.F32:
        atm = rounded(atm, np.float32)
    q = inputs.make_quadrature(inputs.CONFIGS["C1"])
    case = Case(atm, q, prec)
    rng = np.random.default_rng(2)
    w = seed_for(case, rng)
    gk, gp, ge = gpu_grad(case, w, stride=4)
    for trial in range(2):
        v_k = rng.normal(size=atm.npoints) * atm.kappa
        v_p = rng.normal(size=(6, atm.npoints)) * atm.kappa
        v_e = rng.normal(size=(6, atm.npoints)) * atm.emis.std(axis=1, keepdims=True)
        got = np.sum(gk * v_k) + np.sum(gp * v_p) + np.sum(ge * v_e)
        ref = oracle_directional(orc, atm, q, w, v_k, v_p, v_e)
        assert got == pytest.approx(ref, rel=tol), (trial, got, ref)


@pytest.mark.parametrize("prec", [porta.F64, porta.F32])
def test_single_frequency_and_single_inclination(orc, prec):
    """One frequency (the FP32 frequency loops take two per trip) and one inclination per
    hemisphere (4 rays): the forward I_top and J, and the adjoint along random
    directions, against the oracle."""
    cfg = inputs.Config("one", 5, 4, 6, 1, 2, 1, True)
    atm = dataclasses.replace(inputs.make_atmosphere(cfg, seed=21), lx=800.0, ly=600.0,
                              z=np.linspace(0, 1200, 6))
    if prec == porta.F32:
        atm = rounded(atm, np.float32)
    q = inputs.make_quadrature(cfg)
    ref = orc.fs_sweep(orc.OracleProblem(atm, q))
    case = Case(atm, q, prec)
    jkq, itop = case.sweep()
    tol_i, tol_p = (1e-10, 1e-12) if prec == porta.F64 else (2e-5, 1e-7)
    compare_stokes(itop, up_rays(ref["itop"], q), tol_i, tol_p, "itop")
    compare_jkq(jkq, ref["jkq"], tol_i, "jkq")
    rng = np.random.default_rng(22)
    w = seed_for(case, rng)
    for stride in (1, 2):
        g = gpu_grad(case, w, stride=stride)
        v = [rng.normal(size=atm.npoints) * atm.kappa,
             rng.normal(size=(6, atm.npoints)) * atm.kappa,
             rng.normal(size=(6, atm.npoints)) * atm.emis.std(axis=1, keepdims=True)]
        got = sum(np.sum(a * b) for a, b in zip(g, v))
        assert got == pytest.approx(oracle_directional(orc, atm, q, w, *v), rel=tol_i), stride


def test_adjoint_ragged_batches_and_strides(orc):
    """Odd plane (5x3), several ray batches and block sizes give the same gradient."""
    atm, q = tiny_case(porta.F64, seed=12, nx=5, ny=3, nz=7)
    case = Case(atm, q, porta.F64)
    w = seed_for(case, np.random.default_rng(3))
    base = np.concatenate([g.reshape(-1) for g in gpu_grad(case, w, stride=6)])
    for stride, rb, blk in ((1, 3, 64), (3, 5, 128), (2, 0, 192)):
        g = gpu_grad(case, w, stride=stride, opts=porta.options(ray_batch=rb, block=blk))
        np.testing.assert_allclose(np.concatenate([x.reshape(-1) for x in g]), base, rtol=1e-12,
                                   atol=1e-14 * np.abs(base).max())
    rng = np.random.default_rng(4)
    v = [rng.normal(size=atm.npoints), rng.normal(size=(6, atm.npoints)),
         rng.normal(size=(6, atm.npoints))]
    g = gpu_grad(case, w, stride=2)
    got = sum(np.sum(a * b) for a, b in zip(g, v))
    assert got == pytest.approx(oracle_directional(orc, atm, q, w, *v), rel=1e-10)


def test_adjoint_is_deterministic_and_adds_to_outputs():
    torch = require_gpu()
    atm, q = tiny_case(porta.F32, seed=13)
    case = Case(atm, q, porta.F32)
    w = to_dev(seed_for(case, np.random.default_rng(5)), torch.float32)
    a = porta.fs_adjoint(case.hg, case.kappa, case.prop, case.emis, atm.i_bottom, w, atm.w2,
                         prec=porta.F32, checkpoint_stride=2)
    b = porta.fs_adjoint(case.hg, case.kappa, case.prop, case.emis, atm.i_bottom, w, atm.w2,
                         prec=porta.F32, checkpoint_stride=2)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    porta.fs_adjoint(case.hg, case.kappa, case.prop, case.emis, atm.i_bottom, w, atm.w2,
                     prec=porta.F32, checkpoint_stride=2, g_kappa=a[0], g_propmat=a[1],
                     g_emis=a[2])
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        torch.testing.assert_close(x, 2 * y, rtol=1e-6, atol=0)


def _loss_and_seed(case, target):
    torch = require_gpu()
    _, it = porta.fs_sweep(case.hg, case.kappa, case.prop, case.emis, case.atm.i_bottom,
                           case.atm.w2, prec=case.prec, want_jkq=False)
    torch.cuda.synchronize()
    d = it.double() - target
    return float((d * d).sum()), 2 * d


def test_c4_fp32_adjoint_against_fd_and_oracle(orc):
    """Differentiation instance (64^3, 80 rays, 41 frequencies): the loss
    L = sum (I_top - target)^2 with a target from a perturbed atmosphere.  The FP64
    adjoint against central differences (h = 1e-4 relative, FP64 GPU forward) on 32
    random parameters; the FP32 adjoint against the FP64 one (l2 and per component);
    and complex-step derivatives of the oracle for a seed on four (ray, freq) pairs."""
    torch = require_gpu()
    cfg = inputs.CONFIGS["C4"]
    atm = rounded(inputs.make_atmosphere(cfg, seed=0), np.float32)
    q = inputs.make_quadrature(cfg)
    tgt_atm = inputs.perturbed_target_atmosphere(atm, seed=5)
    c64_t = Case(tgt_atm, q, porta.F64)
    _, target = porta.fs_sweep(c64_t.hg, c64_t.kappa, c64_t.prop, c64_t.emis, atm.i_bottom,
                               atm.w2, prec=porta.F64, want_jkq=False)
    case64 = Case(atm, q, porta.F64)
    case32 = Case(atm, q, porta.F32)
    _, seed = _loss_and_seed(case64, target)
    g64 = gpu_grad(case64, seed.cpu().numpy(), stride=8)
    g32 = gpu_grad(case32, seed.cpu().numpy().astype(np.float32).astype(np.float64), stride=8)
    fields = [atm.kappa, atm.propmat, atm.emis]
    # FP32 against FP64 adjoint
    a64 = np.concatenate([g.reshape(-1) for g in g64])
    a32 = np.concatenate([g.reshape(-1) for g in g32])
    l2 = np.linalg.norm(a32 - a64) / np.linalg.norm(a64)
    big = np.abs(a64) > 1e-3 * np.abs(a64).max()
    comp = np.max(np.abs(a32 - a64)[big] / np.abs(a64)[big])
    print(f"C4 FP32 vs FP64 adjoint: l2 rel {l2:.2e}, max rel over large components {comp:.2e}")
    assert l2 < 1e-4 and comp < 1e-3
    # finite differences with the FP64 forward on 32 random parameters
    rng = np.random.default_rng(6)
    checked, worst64, worst32 = 0, 0.0, 0.0
    for _ in range(64):
        which = rng.integers(0, 3)
        shape = fields[which].shape
        idx = tuple(rng.integers(0, s) for s in shape)
        val = fields[which][idx]
        if val == 0.0:
            continue
        h = 1e-4 * abs(val)
        tops = []
        for sgn in (+1, -1):
            f2 = [x.copy() for x in fields]
            f2[which][idx] = val + sgn * h
            c = Case(dataclasses.replace(atm, kappa=f2[0], propmat=f2[1], emis=f2[2]), q,
                     porta.F64)
            tops.append(porta.fs_sweep(c.hg, c.kappa, c.prop, c.emis, atm.i_bottom, atm.w2,
                                       prec=porta.F64, want_jkq=False)[1])
        # L(p+h) - L(p-h) summed term by term, free of the cancellation of two large sums
        fd = float(((tops[0] - tops[1]) * (tops[0] + tops[1] - 2 * target)).sum()) / (2 * h)
        scale = max(abs(fd), 1e-3 * np.abs(g64[which]).max())
        worst64 = max(worst64, abs(g64[which][idx] - fd) / scale)
        worst32 = max(worst32, abs(g32[which][idx] - fd) / scale)
        checked += 1
        if checked == 32:
            break
    print(f"C4 central differences on {checked} parameters: FP64 adjoint {worst64:.2e}, "
          f"FP32 adjoint {worst32:.2e}")
    assert checked == 32
    assert worst64 < 1e-3 and worst32 < 1e-3
    # complex step of the oracle with a seed on four (ray, frequency) pairs only
    pairs = [(3, 20), (17, 10), (29, 33), (38, 2)]
    wr = np.random.default_rng(7).normal(size=seed.shape)
    mask = np.zeros(wr.shape[:2] + (1, 1, 1))
    for r, f in pairs:
        mask[r, f] = 1
    w = (wr * mask).astype(np.float32).astype(np.float64)
    gk, gp, ge = gpu_grad(case32, w, stride=8)
    v = [rng.normal(size=atm.npoints) * atm.kappa, rng.normal(size=(6, atm.npoints)) * atm.kappa,
         rng.normal(size=(6, atm.npoints)) * atm.emis.std(axis=1, keepdims=True)]
    got = np.sum(gk * v[0]) + np.sum(gp * v[1]) + np.sum(ge * v[2])
    ref = oracle_directional(orc, atm, q, w, *v, pairs=pairs)
    assert got == pytest.approx(ref, rel=1e-4)


def test_autograd_function_uses_the_adjoint(orc):
    torch = require_gpu()
    from paper_1307_4217_amd.autograd import emergent_stokes
    atm, q = tiny_case(porta.F64, seed=21, nx=4, ny=4, nz=6)
    case = Case(atm, q, porta.F64)
    k = case.kappa.clone().requires_grad_(True)
    pm = case.prop.clone().requires_grad_(True)
    e = case.emis.clone().requires_grad_(True)
    target = torch.zeros((case.hg.nray_up, case.hg.nfreq, atm.ny, atm.nx, 4),
                         dtype=torch.float64, device="cuda")
    itop = emergent_stokes(case.hg, k, pm, e, atm.i_bottom, atm.w2, prec=porta.F64,
                           checkpoint_stride=2)
    loss = ((itop - target) ** 2).sum()
    loss.backward()
    gk, gp, ge = porta.fs_adjoint(case.hg, case.kappa, case.prop, case.emis, atm.i_bottom,
                                  (2 * (itop - target)).detach(), atm.w2, prec=porta.F64,
                                  checkpoint_stride=2)
    torch.cuda.synchronize()
    assert torch.equal(k.grad, gk) and torch.equal(pm.grad, gp) and torch.equal(e.grad, ge)
    # the same with the forward sweep keeping the checkpoints for the backward pass
    k2, pm2, e2 = (x.detach().clone().requires_grad_(True) for x in (k, pm, e))
    itop2 = emergent_stokes(case.hg, k2, pm2, e2, atm.i_bottom, atm.w2, prec=porta.F64,
                            checkpoint_stride=2, keep_checkpoints=True)
    ((itop2 - target) ** 2).sum().backward()
    torch.cuda.synchronize()
    assert torch.equal(itop2, itop)
    assert torch.equal(k2.grad, gk) and torch.equal(pm2.grad, gp) and torch.equal(e2.grad, ge)
    # the autograd gradient against complex-step derivatives of the oracle
    rng = np.random.default_rng(22)
    v = [rng.normal(size=atm.npoints), rng.normal(size=(6, atm.npoints)),
         rng.normal(size=(6, atm.npoints))]
    got = sum(float(np.sum(x.grad.cpu().numpy() * y)) for x, y in zip((k, pm, e), v))
    w = (2 * (itop - target)).detach().cpu().numpy()
    assert got == pytest.approx(oracle_directional(orc, atm, q, w, *v), rel=1e-10)


def test_autograd_function_in_the_bezier_mode():
    """emergent_stokes(interp=BEZIER2D): the forward is the 9-point sweep and the backward
    its adjoint, bitwise, with and without checkpoints kept by the forward."""
    torch = require_gpu()
    from paper_1307_4217_amd.autograd import emergent_stokes
    atm, q = tiny_case(porta.F64, seed=23, nx=5, ny=4, nz=6)
    case = Case(atm, q, porta.F64)
    target = torch.zeros((case.hg.nray_up, case.hg.nfreq, atm.ny, atm.nx, 4),
                         dtype=torch.float64, device="cuda")
    _, ref_t = case.sweep(interp=porta.BEZIER2D, want_jkq=False)
    for keep in (False, True):
        k, pm, e = (x.clone().requires_grad_(True) for x in (case.kappa, case.prop, case.emis))
        itop = emergent_stokes(case.hg, k, pm, e, atm.i_bottom, atm.w2, prec=porta.F64,
                               checkpoint_stride=2, keep_checkpoints=keep,
                               interp=porta.BEZIER2D)
        ((itop - target) ** 2).sum().backward()
        g = porta.fs_adjoint(case.hg, case.kappa, case.prop, case.emis, atm.i_bottom,
                             (2 * (itop - target)).detach(), atm.w2, prec=porta.F64,
                             interp=porta.BEZIER2D, checkpoint_stride=2)
        torch.cuda.synchronize()
        assert np.array_equal(itop.detach().cpu().numpy(), ref_t)
        assert torch.equal(k.grad, g[0]) and torch.equal(pm.grad, g[1]) and torch.equal(e.grad, g[2])


@pytest.mark.parametrize("interp", [porta.BILINEAR, porta.BEZIER2D])
@pytest.mark.parametrize("prec", [porta.F64, porta.F32])
@pytest.mark.parametrize("stride, rb_fwd, rb_adj", [(2, 0, 3), (3, 5, 0), (1, 2, 7), (6, 0, 0)])
def test_adjoint_with_checkpoints_from_the_sweep(prec, stride, rb_fwd, rb_adj, interp):
    """Checkpoints written by porta_fs_sweep (any ray batch) give the same gradient, bitwise,
    as the adjoint making its own, in either interpolation mode."""
    torch = require_gpu()
    atm, q = tiny_case(prec, seed=31, nx=5, ny=4, nz=7)
    case = Case(atm, q, prec)
    w = to_dev(seed_for(case, np.random.default_rng(8)), case.dt)
    n = porta.checkpoint_size(case.hg, prec, stride)
    ck = torch.full((max(n, 256),), 255, dtype=torch.uint8, device="cuda")
    jkq, itop = porta.fs_sweep(case.hg, case.kappa, case.prop, case.emis, atm.i_bottom, atm.w2,
                               prec=prec, interp=interp, checkpoints=ck,
                               checkpoint_stride=stride, opts=porta.options(ray_batch=rb_fwd))
    ref_j, ref_t = case.sweep(interp=interp)
    torch.cuda.synchronize()
    # I_top is independent of the ray batching; J only up to its summation order
    assert np.array_equal(itop.cpu().numpy(), ref_t)
    np.testing.assert_allclose(jkq.cpu().numpy(), ref_j, rtol=1e-13, atol=1e-15)
    own = porta.fs_adjoint(case.hg, case.kappa, case.prop, case.emis, atm.i_bottom, w, atm.w2,
                           prec=prec, interp=interp, checkpoint_stride=stride,
                           opts=porta.options(ray_batch=rb_adj))
    ext = porta.fs_adjoint(case.hg, case.kappa, case.prop, case.emis, atm.i_bottom, w, atm.w2,
                           prec=prec, interp=interp, checkpoint_stride=stride, checkpoints=ck,
                           opts=porta.options(ray_batch=rb_adj))
    torch.cuda.synchronize()
    for a, b in zip(own, ext):
        assert torch.equal(a, b)


def test_adjoint_with_parabolic_control_point(orc):
    """FP64 adjoint through the parabolic control point (no clamps, so its derivative
    is the linear formula of steps 3-4 and the ratio) against the oracle's complex step."""
    atm, q = tiny_case(porta.F64, seed=14, nx=5, ny=4, nz=6)
    case = Case(atm, q, porta.F64)
    rng = np.random.default_rng(15)
    w = seed_for(case, rng)
    opts = porta.options(control=porta.CONTROL_PARABOLIC)
    for stride in (1, 3):
        g = gpu_grad(case, w, stride=stride, opts=opts)
        v = [rng.normal(size=atm.npoints) * atm.kappa,
             rng.normal(size=(6, atm.npoints)) * atm.kappa,
             rng.normal(size=(6, atm.npoints)) * atm.emis.std(axis=1, keepdims=True)]
        got = sum(np.sum(a * b) for a, b in zip(g, v))
        ref = oracle_directional(orc, atm, q, w, *v, control=1)
        assert got == pytest.approx(ref, rel=1e-10)
    # and it is a different derivative from the BESSER one
    gb = gpu_grad(case, w, stride=1)
    assert max(np.abs(a - b).max() for a, b in zip(g, gb)) > 0


@pytest.mark.parametrize("prec", [porta.F64, porta.F32])
def test_adjoint_over_ray_ranges(prec):
    """Adjoint calls over ray ranges (gradients added into the same arrays) give the
    one-call gradient, with their own checkpoints and with stride-1 checkpoints kept by a
    sweep of the same range just before: the schedule that interleaves forward and reverse
    sweeps range by range without recomputing a plane."""
    torch = require_gpu()
    atm, q = tiny_case(prec, seed=32, nx=5, ny=4, nz=7)
    case = Case(atm, q, prec)
    nh = case.hg.nray_up
    w = to_dev(seed_for(case, np.random.default_rng(9)), case.dt)
    ref = porta.fs_adjoint(case.hg, case.kappa, case.prop, case.emis, atm.i_bottom, w, atm.w2,
                           prec=prec, checkpoint_stride=2)
    _, ref_t = case.sweep()
    torch.cuda.synchronize()
    scale = max(float(x.abs().max()) for x in ref)
    # FP32: each call rounds its share of the gradient to the sweep precision
    tol = 1e-13 if prec == porta.F64 else 2e-6
    ranges = ((0, 3), (3, 2), (5, nh - 5 + 4), (nh + 4, nh - 4))
    g_own = [torch.zeros_like(x) for x in ref]
    g_fused = [torch.zeros_like(x) for x in ref]
    itop = torch.full(ref_t.shape, float("nan"), dtype=case.dt, device="cuda")
    for first, count in ranges:
        o = porta.options(ray_batch=2, ray_first=first, ray_count=count)
        porta.fs_adjoint(case.hg, case.kappa, case.prop, case.emis, atm.i_bottom, w, atm.w2,
                         prec=prec, checkpoint_stride=3, g_kappa=g_own[0], g_propmat=g_own[1],
                         g_emis=g_own[2], opts=o)
        ck = torch.empty(max(porta.checkpoint_size(case.hg, prec, 1, o), 256), dtype=torch.uint8,
                         device="cuda")
        porta.fs_sweep(case.hg, case.kappa, case.prop, case.emis, atm.i_bottom, atm.w2, prec=prec,
                       want_jkq=False, i_top=itop, opts=o, checkpoints=ck, checkpoint_stride=1)
        porta.fs_adjoint(case.hg, case.kappa, case.prop, case.emis, atm.i_bottom, w, atm.w2,
                         prec=prec, checkpoint_stride=1, g_kappa=g_fused[0],
                         g_propmat=g_fused[1], g_emis=g_fused[2], opts=o, checkpoints=ck)
        torch.cuda.synchronize()
    assert np.array_equal(itop.cpu().numpy(), ref_t)
    for g in (g_own, g_fused):
        for a, b in zip(g, ref):
            err = float((a.double() - b.double()).abs().max()) / scale
            assert err <= tol, err


@pytest.mark.parametrize("prec, range_rays, interp", [(porta.F64, 3, porta.BILINEAR),
                                                      (porta.F32, 5, porta.BILINEAR),
                                                      (porta.F64, 4, porta.BEZIER2D)])
def test_interleaved_schedule_matches_separate_calls(prec, range_rays, interp):
    """schedule.InterleavedSweep (ranges of upward rays swept with every plane kept and
    reversed at once, downward rays last) against one sweep of all rays and one adjoint
    call: J, I_top before the seed, the seed rows handed to the callback, and the
    gradients of L = sum (I_top - target)^2, in either interpolation mode."""
    torch = require_gpu()
    from paper_1307_4217_amd import schedule
    atm, q = tiny_case(prec, seed=33, nx=5, ny=4, nz=7)
    case = Case(atm, q, prec)
    hg = case.hg
    ref_j, ref_t = case.sweep(interp=interp)
    target = to_dev(ref_t * 0.9 + 0.01, case.dt)
    seed_ref = 2 * (to_dev(ref_t, case.dt) - target)
    g_ref = porta.fs_adjoint(hg, case.kappa, case.prop, case.emis, atm.i_bottom, seed_ref,
                             atm.w2, prec=prec, interp=interp, checkpoint_stride=2)
    inter = schedule.InterleavedSweep(hg, prec, range_rays, ray_batch=3, interp=interp)
    jkq = torch.full((10, hg.N), float("nan"), dtype=torch.float64, device="cuda")
    itop = torch.full(ref_t.shape, float("nan"), dtype=case.dt, device="cuda")
    g = [torch.zeros_like(x) for x in g_ref]
    seen = []

    def seed(r, n, rows):
        seen.append((r, n, rows.cpu().numpy().copy()))
        rows.sub_(target[r:r + n]).mul_(2.0)

    inter.run(case.kappa, case.prop, case.emis, atm.i_bottom, atm.w2, jkq, itop, seed, *g)
    torch.cuda.synchronize()
    assert [(r, n) for r, n, _ in seen] == inter.ranges
    assert sum(n for _, n in inter.ranges) == hg.nray_up
    for r, n, rows in seen:
        assert np.array_equal(rows, ref_t[r:r + n])
    np.testing.assert_allclose(jkq.cpu().numpy(), ref_j, rtol=1e-13,
                               atol=1e-15 * np.abs(ref_j).max())
    np.testing.assert_allclose(itop.cpu().numpy(), seed_ref.cpu().numpy(), rtol=0, atol=0)
    scale = max(float(x.abs().max()) for x in g_ref)
    tol = 1e-13 if prec == porta.F64 else 2e-6
    for a, b in zip(g, g_ref):
        assert float((a.double() - b.double()).abs().max()) / scale <= tol
    assert inter.launch_ray_counts() == [n for _, n in inter.ranges] + [3, 3, 2]
