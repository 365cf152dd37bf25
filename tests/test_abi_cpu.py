"""C-ABI checks that need no GPU: exported symbols and host-side validation."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1307_4217_amd import inputs, porta

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "porta.h")).read()
    return sorted(set(re.findall(r"^\s*(?:[\w\s\*]+?)\b(porta_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    L = porta.lib()
    names = declared_symbols()
    assert set(names) == set(porta.EXPORTED), names
    for n in names:
        assert hasattr(L, n), n
    assert "gfx950" in porta.version()


def small_hg(**kw):
    cfg = inputs.CONFIGS["C1"]
    atm = inputs.make_atmosphere(cfg)
    q = inputs.make_quadrature(cfg)
    args = dict(nx=atm.nx, ny=atm.ny, nz=atm.nz, lx=atm.lx, ly=atm.ly, z=atm.z, mu=q.mu,
                wmu=q.wmu, nchi=q.nchi, phi=q.phi, wfreq=q.wfreq)
    args.update(kw)
    return porta.HostGrid(**args)


def call_sweep(hg, prec=porta.F64, interp=porta.BILINEAR, ws_bytes=None, fields=True, ws=True):
    L = porta.lib()
    dummy = np.zeros(8)
    f = porta.Fields(dummy.ctypes.data if fields else None, dummy.ctypes.data,
                     dummy.ctypes.data, 1.0, 1.0)
    return L.porta_fs_sweep(C.byref(hg.grid), C.byref(hg.quad), C.byref(f), prec, interp, None,
                            None, 0, None, None, 0, 0, dummy.ctypes.data if ws else None,
                            0 if ws_bytes is None else ws_bytes, None)


@pytest.mark.parametrize("kw, code", [
    (dict(nz=1, z=[0.0]), -1),
    (dict(nx=0), -1),
    (dict(z=np.linspace(1, 0, 32)), -1),
    (dict(z=np.r_[np.linspace(0, 1, 31), np.nan]), -1),
    (dict(lx=-1.0), -1),
    (dict(mu=[0.5, 1.2, 0.3, 0.2, 0.1]), -1),
    (dict(mu=[0.0, 0.5, 0.3, 0.2, 0.1]), -1),
    (dict(wmu=[0.2] * 4 + [0.3]), -1),
    (dict(phi=-np.ones(21)), -1),
    (dict(wfreq=np.zeros(21)), -1),
])
def test_sweep_rejects_bad_geometry(kw, code):
    hg = small_hg(**kw)
    assert call_sweep(hg) == -1
    assert porta.lib().porta_last_error().decode() != ""


def test_sweep_rejects_bad_enums_and_pointers():
    hg = small_hg()
    assert call_sweep(hg, prec=7) == -1
    assert call_sweep(hg, interp=9) == -1
    assert call_sweep(hg, fields=False) == -1
    assert call_sweep(hg, ws=False) == -1


def test_sweep_reports_short_workspace():
    hg = small_hg()
    need = porta.workspace_size(hg, porta.F64, porta.WS_SWEEP)
    assert need > 0
    assert call_sweep(hg, ws_bytes=need - 1) == -3
    assert "workspace" in porta.lib().porta_last_error().decode()


def test_workspace_sizes_scale_with_precision_and_batch():
    hg = small_hg()
    w64 = porta.workspace_size(hg, porta.F64, porta.WS_SWEEP)
    w32 = porta.workspace_size(hg, porta.F32, porta.WS_SWEEP)
    assert w32 < w64
    wb = porta.workspace_size(hg, porta.F64, porta.WS_SWEEP, opts=porta.options(ray_batch=8))
    assert wb < w64
    assert porta.workspace_size(hg, porta.F64, porta.WS_JKQ) < wb
    assert porta.lib().porta_workspace_size(C.byref(hg.grid), C.byref(hg.quad), 5, 0, 1,
                                            None) == 0


def test_other_entry_points_validate():
    L = porta.lib()
    hg = small_hg()
    dummy = np.zeros(8)
    a = porta.Atom(1.5, 0.0, 1.0, 1.0, None, None)
    assert L.porta_see_update(10, dummy.ctypes.data, C.byref(a), None, dummy.ctypes.data,
                              dummy.ctypes.data, None, None, 0, None, None, 0, None) == -1
    a = porta.Atom(0.1, 0.0, 1.0, 1.0, None, None)
    assert L.porta_see_update(0, dummy.ctypes.data, C.byref(a), None, dummy.ctypes.data,
                              dummy.ctypes.data, None, None, 0, None, None, 0, None) == -1
    assert L.porta_see_update(10, dummy.ctypes.data, C.byref(a), None, dummy.ctypes.data,
                              dummy.ctypes.data, None, None, 0, dummy.ctypes.data,
                              dummy.ctypes.data, 1, None) == -3
    assert L.porta_jkq_accumulate(C.byref(hg.grid), C.byref(hg.quad), 70, 20, 0, 1,
                                  dummy.ctypes.data, None, 0, dummy.ctypes.data,
                                  dummy.ctypes.data, 1 << 20, None) == -1
    assert L.porta_jkq_accumulate(C.byref(hg.grid), C.byref(hg.quad), 0, 1, 20, 2,
                                  dummy.ctypes.data, None, 0, dummy.ctypes.data,
                                  dummy.ctypes.data, 1 << 20, None) == -1
    f = porta.Fields(dummy.ctypes.data, dummy.ctypes.data, dummy.ctypes.data, 1.0, 1.0)
    for stride in (0, 32):   # must be in 1..nz-1
        assert L.porta_fs_adjoint(C.byref(hg.grid), C.byref(hg.quad), C.byref(f), 0, 0, None,
                                  dummy.ctypes.data, None, 0, stride, dummy.ctypes.data,
                                  dummy.ctypes.data, dummy.ctypes.data, dummy.ctypes.data,
                                  1 << 40, None) == -1
    # a checkpoint buffer needs a valid stride
    assert L.porta_fs_sweep(C.byref(hg.grid), C.byref(hg.quad), C.byref(f), 0, 0, None, None, 0,
                            None, dummy.ctypes.data, 1 << 40, 0, dummy.ctypes.data, 1 << 40,
                            None) == -1
    assert porta.checkpoint_size(hg, porta.F32, 4) == (30 // 4) * 40 * 21 * 256 * 16
    assert porta.checkpoint_size(hg, porta.F64, 31) == 0
    assert (porta.workspace_size(hg, porta.F32, porta.WS_ADJOINT_CKPT, 4)
            < porta.workspace_size(hg, porta.F32, porta.WS_ADJOINT, 4))
    assert porta.lib().porta_strerror(-3) == b"workspace too small"


def test_adjoint_accepts_both_interpolation_modes():
    """Both modes pass the option checks of the adjoint and reach the workspace check
    (a workspace of 16 bytes: PORTA_ENOMEM before any launch); an unknown mode does not."""
    L = porta.lib()
    hg = small_hg()
    dummy = np.zeros(8)
    f = porta.Fields(dummy.ctypes.data, dummy.ctypes.data, dummy.ctypes.data, 1.0, 1.0)

    def adj(interp):
        return L.porta_fs_adjoint(C.byref(hg.grid), C.byref(hg.quad), C.byref(f), 0, interp,
                                  None, dummy.ctypes.data, None, 0, 4, dummy.ctypes.data,
                                  dummy.ctypes.data, dummy.ctypes.data, dummy.ctypes.data, 16,
                                  None)
    assert adj(porta.BILINEAR) == porta.ENOMEM
    assert adj(porta.BEZIER2D) == porta.ENOMEM
    assert adj(7) == porta.EINVAL


def test_multigrid_entry_points_validate():
    """Shape and argument checks of the multigrid calls (no kernel launch)."""
    L = porta.lib()
    d = np.zeros(8).ctypes.data
    a = porta.Atom(0.1, 0.0, 1.0, 1.0, None, None)
    bad = porta.Atom(-0.1, 0.0, 1.0, 1.0, None, None)
    assert L.porta_see_operator(0, d, C.byref(a), d, None, -1.0, d, None) == -1
    assert L.porta_see_operator(10, d, C.byref(bad), d, None, -1.0, d, None) == -1
    assert L.porta_see_operator(10, None, C.byref(a), d, None, -1.0, d, None) == -1
    assert L.porta_see_operator(10, d, C.byref(a), d, None, float("nan"), d, None) == -1
    # odd nx, even nz, too small, bad ncomp, bad precision, kappa without emis
    for nx, ny, nz, k, prec in ((5, 4, 5, 1, 0), (4, 4, 6, 1, 0), (4, 4, 1, 1, 0), (0, 4, 5, 1, 0),
                                (4, 4, 5, 0, 0), (4, 4, 5, 65, 0), (4, 4, 5, 1, 7)):
        assert L.porta_mg_restrict(nx, ny, nz, k, d, d, None, None, prec, None) == -1
        assert L.porta_mg_prolong(nx, ny, nz, k, 1, d, None, d, None, None, prec, None) == -1
    assert L.porta_mg_restrict(4, 4, 5, 1, d, d, d, None, 0, None) == -1
    assert L.porta_mg_prolong(4, 4, 5, 1, 1, d, None, d, None, d, 0, None) == -1
    assert L.porta_mg_prolong(4, 4, 9, 1, 2, d, None, d, None, None, 0, None) == -1   # order
    assert L.porta_mg_prolong(4, 4, 5, 1, 3, d, None, d, None, None, 0, None) == -1   # nzc < 4
    assert L.porta_mg_restrict(4, 4, 5, 1, None, d, None, None, 0, None) == -1
    assert L.porta_mg_prolong(4, 4, 5, 1, 1, None, None, d, None, None, 0, None) == -1
    assert L.porta_mg_inject(4, 4, 5, 1, 2, d, d, None) == -1
    assert L.porta_mg_inject(4, 4, 4, 1, 8, d, d, None) == -1
    assert L.porta_rel_change(10, d, d, d, d, 4, None) == -3
    assert L.porta_rel_change(10, d, None, d, d, 1 << 20, None) == -1


def test_kernel_code_digest_found_in_built_library():
    """The benchmark keys its committed HBM counters to the machine code of the kernel."""
    import re
    import bench
    for k in ("k_sweep_plane<float, 0>", "k_adjoint_plane<float, 0>"):
        d = bench.kernel_code_sha256(k)
        assert d is not None and re.fullmatch(r"[0-9a-f]{64}", d)
    assert bench.kernel_code_sha256("no such kernel") is None


def test_unknown_control_point_rule_rejected():
    L = porta.lib()
    hg = small_hg()
    d = np.zeros(8).ctypes.data
    f = porta.Fields(d, d, d, 1.0, 1.0)
    bad = porta.options(control=2)
    assert L.porta_fs_sweep(C.byref(hg.grid), C.byref(hg.quad), C.byref(f), 0, 0, C.byref(bad),
                            d, 0, d, None, 0, 0, d, 1 << 40, None) == -1
    assert b"control" in L.porta_last_error()
    assert L.porta_fs_adjoint(C.byref(hg.grid), C.byref(hg.quad), C.byref(f), 0, 0,
                              C.byref(bad), d, None, 0, 2, d, d, d, d, 1 << 40, None) == -1


def test_intensity_only_option_checks():
    L = porta.lib()
    hg = small_hg()
    d = np.zeros(8).ctypes.data
    f = porta.Fields(d, d, d, 1.0, 1.0)
    args = lambda o, interp=0, ck=None, stride=0: (C.byref(hg.grid), C.byref(hg.quad), C.byref(f),
                                                   0, interp, C.byref(o), d, 0, d, ck,
                                                   1 << 40 if ck else 0, stride, d, 1 << 40,
                                                   None)
    assert L.porta_fs_sweep(*args(porta.options(stokes=2))) == -1
    assert L.porta_fs_sweep(*args(porta.options(stokes=1), interp=1)) == -2
    assert L.porta_fs_sweep(*args(porta.options(stokes=1), ck=d, stride=2)) == -2
    assert L.porta_fs_adjoint(C.byref(hg.grid), C.byref(hg.quad), C.byref(f), 0, 0,
                              C.byref(porta.options(stokes=1)), d, None, 0, 2, d, d, d, d,
                              1 << 40, None) == -2
    # the workspace of the intensity-only sweep holds a quarter of the plane states
    w4 = porta.workspace_size(hg, porta.F32, porta.WS_SWEEP, 1, porta.options(ray_batch=4))
    w1 = porta.workspace_size(hg, porta.F32, porta.WS_SWEEP, 1,
                              porta.options(ray_batch=4, stokes=1))
    assert w1 < w4


def test_ray_range_checks_and_sizes():
    """A ray range [ray_first, ray_first + ray_count) beyond the 2 nmu nchi rays is
    rejected before any launch; checkpoints and workspaces are sized for the range."""
    L = porta.lib()
    hg = small_hg()
    nh = hg.nray_up
    d = np.zeros(8).ctypes.data
    f = porta.Fields(d, d, d, 1.0, 1.0)
    for first, count in ((0, 2 * nh + 1), (2 * nh - 5, 6), (-1, 2), (0, -1)):
        o = porta.options(ray_first=first, ray_count=count)
        assert L.porta_fs_sweep(C.byref(hg.grid), C.byref(hg.quad), C.byref(f), 0, 0,
                                C.byref(o), d, 0, d, None, 0, 0, d, 1 << 40, None) == -1
        assert L.porta_fs_adjoint(C.byref(hg.grid), C.byref(hg.quad), C.byref(f), 0, 0,
                                  C.byref(o), d, None, 0, 2, d, d, d, d, 1 << 40, None) == -1
        assert porta.checkpoint_size(hg, porta.F32, 4, o) == 0
    full = porta.checkpoint_size(hg, porta.F32, 4)
    # only the upward rays of the range are kept: 10 of [30, 50), none of the downward
    assert porta.checkpoint_size(hg, porta.F32, 4,
                                 porta.options(ray_first=nh - 10, ray_count=20)) == full // 4
    assert porta.checkpoint_size(hg, porta.F32, 4,
                                 porta.options(ray_first=nh, ray_count=nh)) == 0
    assert porta.checkpoint_size(hg, porta.F32, 1, porta.options(ray_count=8)) == \
        (32 - 2) * 8 * 21 * 256 * 16
    # the batch of a call is at most its rays in one hemisphere
    for kind, stride in ((porta.WS_SWEEP, 1), (porta.WS_ADJOINT_CKPT, 1), (porta.WS_ADJOINT, 3)):
        sub = porta.workspace_size(hg, porta.F32, kind, stride,
                                   porta.options(ray_first=8, ray_count=8))
        assert sub == porta.workspace_size(hg, porta.F32, kind, stride,
                                           porta.options(ray_batch=8))
        assert sub < porta.workspace_size(hg, porta.F32, kind, stride)


def test_short_checkpoint_buffer_rejected():
    """A checkpoint buffer below porta_checkpoint_size() for the call's stride and ray
    range is refused with PORTA_ENOMEM by the sweep and the adjoint before any launch."""
    L = porta.lib()
    hg = small_hg()
    d = np.zeros(8).ctypes.data
    f = porta.Fields(d, d, d, 1.0, 1.0)
    for o in (None, porta.options(ray_first=4, ray_count=10)):
        need = porta.checkpoint_size(hg, porta.F32, 3, o)
        ob = C.byref(o) if o else None
        assert L.porta_fs_sweep(C.byref(hg.grid), C.byref(hg.quad), C.byref(f), 1, 0, ob, d, 0,
                                d, d, need - 1, 3, d, 1 << 40, None) == -3
        assert b"checkpoint buffer" in L.porta_last_error()
        assert L.porta_fs_adjoint(C.byref(hg.grid), C.byref(hg.quad), C.byref(f), 1, 0, ob, d,
                                  d, need - 1, 3, d, d, d, d, 1 << 40, None) == -3
        assert b"checkpoint buffer" in L.porta_last_error()


def test_interleaved_schedule_range_size():
    """schedule.fitting_range_rays: the largest number of rays per range (up to the
    limit) whose stride-1 checkpoints and extra adjoint workspace fit the budget."""
    from paper_1307_4217_amd import schedule
    hg = small_hg()
    prec = porta.F32
    base = porta.workspace_size(hg, prec, porta.WS_SWEEP, 1, porta.options(ray_batch=40))

    def need(n):
        o = porta.options(ray_batch=n, ray_count=n)
        return (porta.checkpoint_size(hg, prec, 1, o)
                + max(0, porta.workspace_size(hg, prec, porta.WS_ADJOINT_CKPT, 1, o) - base))

    assert schedule.fitting_range_rays(hg, prec, 1 << 50, base) == 16
    assert schedule.fitting_range_rays(hg, prec, 1 << 50, base, limit=100) == hg.nray_up
    assert schedule.fitting_range_rays(hg, prec, need(1) - 1, base) == 0
    for n in (1, 5, 11):
        assert schedule.fitting_range_rays(hg, prec, need(n), base) == n
        assert schedule.fitting_range_rays(hg, prec, need(n + 1) - 1, base) == n


def test_check_inputs_option_is_validated():
    L = porta.lib()
    hg = small_hg()
    d = np.zeros(8).ctypes.data
    f = porta.Fields(d, d, d, 1.0, 1.0)
    bad = porta.Options(0, 0, -1, 0, 4, 0, 0, 2)
    assert L.porta_fs_sweep(C.byref(hg.grid), C.byref(hg.quad), C.byref(f), 0, 0, C.byref(bad),
                            d, 0, d, None, 0, 0, d, 1 << 40, None) == porta.EINVAL
    assert b"check_inputs" in L.porta_last_error()
    assert L.porta_strerror(porta.ENONFINITE).startswith(b"non-finite")
    assert porta.options(check_inputs=True).check_inputs == 1


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: asked for several it exits at once with status 2 and
    says why, before touching the GPU."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=root)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


def test_noalloc_sweep_validates_before_touching_the_device():
    """porta_fs_sweep_noalloc checks its arguments, and that the sweep's workspace fits its
    64 MiB static scratch, on the host before any HIP call."""
    L = porta.lib()
    dummy = np.zeros(8)
    f = porta.Fields(dummy.ctypes.data, dummy.ctypes.data, dummy.ctypes.data, 1.0, 1.0)
    hg = small_hg()
    big = small_hg(nx=256, ny=256)
    assert porta.workspace_size(big, porta.F32, porta.WS_SWEEP) > 64 << 20
    assert L.porta_fs_sweep_noalloc(C.byref(big.grid), C.byref(big.quad), C.byref(f), 1, 0,
                                    None, None, 0, None, None) == porta.ENOMEM
    msg = L.porta_last_error().decode()
    assert "static scratch" in msg and str(64 << 20) in msg
    assert L.porta_fs_sweep_noalloc(C.byref(hg.grid), C.byref(hg.quad), None, 1, 0, None, None,
                                    0, None, None) == porta.EINVAL
    assert L.porta_fs_sweep_noalloc(C.byref(hg.grid), C.byref(hg.quad), C.byref(f), 5, 0, None,
                                    None, 0, None, None) == porta.EINVAL


def test_checkpoints_accepted_with_the_bezier_mode():
    """The adjoint differentiates either mode, so a 9-point sweep may leave checkpoints
    (for an adjoint called with the same mode): the call gets past the option checks to
    the workspace check."""
    L = porta.lib()
    hg = small_hg()
    dummy = np.zeros(8)
    f = porta.Fields(dummy.ctypes.data, dummy.ctypes.data, dummy.ctypes.data, 1.0, 1.0)
    assert L.porta_fs_sweep(C.byref(hg.grid), C.byref(hg.quad), C.byref(f), 0, porta.BEZIER2D,
                            None, None, 0, None, dummy.ctypes.data, 1 << 40, 4,
                            dummy.ctypes.data, 16, None) == porta.ENOMEM


def test_faces_option_checks():
    """options.faces = 1 (M and P on the first face crossed): bilinear Stokes-vector sweep
    only, no checkpoints, no adjoint, nx and ny up to 512; other values rejected."""
    L = porta.lib()
    hg = small_hg()
    dummy = np.zeros(8)
    f = porta.Fields(dummy.ctypes.data, dummy.ctypes.data, dummy.ctypes.data, 1.0, 1.0)

    def sweep(opts, interp=porta.BILINEAR, ck=False, g=hg, ws_bytes=1 << 40):
        return L.porta_fs_sweep(C.byref(g.grid), C.byref(g.quad), C.byref(f), 0, interp,
                                C.byref(opts), None, 0, None, dummy.ctypes.data if ck else None,
                                1 << 40, 4, dummy.ctypes.data, ws_bytes, None)

    assert sweep(porta.options(faces=2)) == porta.EINVAL
    assert sweep(porta.options(faces=1), interp=porta.BEZIER2D) == porta.EUNSUPPORTED
    assert sweep(porta.options(faces=1, stokes=1)) == porta.EUNSUPPORTED
    assert sweep(porta.options(faces=1), ck=True) == porta.EUNSUPPORTED
    assert sweep(porta.options(faces=1), g=small_hg(nx=520)) == porta.EUNSUPPORTED
    assert "512" in L.porta_last_error().decode()
    assert L.porta_fs_adjoint(C.byref(hg.grid), C.byref(hg.quad), C.byref(f), 0,
                              porta.BILINEAR, C.byref(porta.options(faces=1)),
                              dummy.ctypes.data, None, 0, 4, dummy.ctypes.data,
                              dummy.ctypes.data, dummy.ctypes.data, dummy.ctypes.data, 1 << 40,
                              None) == porta.EUNSUPPORTED
    # the per-chunk partial sums of J enlarge the workspace, the more the smaller the chunk
    ws = lambda o: porta.workspace_size(hg, porta.F64, porta.WS_SWEEP, 1, o)
    assert ws(porta.options(faces=1)) > ws(porta.options())
    assert ws(porta.options(faces=1, faces_chunk=1)) > ws(porta.options(faces=1))
    # frequencies per block: >= 0, and they must fit in the LDS of a block (FP64, 512
    # lanes: 17 KiB per frequency)
    assert sweep(porta.options(faces=1, faces_chunk=-1)) == porta.EINVAL
    assert sweep(porta.options(faces=1, faces_chunk=10), g=small_hg(nx=500)) == \
        porta.EUNSUPPORTED
    assert "faces_chunk" in L.porta_last_error().decode()
    # three fit: the call gets past the option checks to the workspace check
    assert sweep(porta.options(faces=1, faces_chunk=3), g=small_hg(nx=500), ws_bytes=16) == \
        porta.ENOMEM


def test_bench_precision_report_on_known_differences():
    """bench.precision_report (CPU tensors): the largest relative difference on I, the
    largest absolute one on Q/I, U/I, V/I, J^K_Q rows 0-8 relative to J00 at the same
    point and Lbar relative, each found where it was planted."""
    import torch
    import bench
    rng = np.random.default_rng(3)
    it64 = torch.as_tensor(1.0 + rng.uniform(0, 0.1, size=(3, 5, 4, 6, 4)))
    it64[..., 1:] *= 1e-3
    it32 = it64.float().clone()
    it32[2, 4, 1, 5, 0] = float(it64[2, 4, 1, 5, 0]) * (1 + 3e-5)      # I, relative
    it32[1, 0, 3, 2, 2] += 2e-6 * float(it64[1, 0, 3, 2, 0])            # U/I, absolute
    j64 = torch.as_tensor(1.0 + rng.uniform(0, 1, size=(10, 24)))
    j32 = j64.clone()
    j32[5, 7] += 4e-7 * j64[0, 7]
    j32[9, 11] *= 1 + 5e-8
    r = bench.precision_report(it32, it64, j32, j64, 4)
    assert r["outputs"] == 3 * 5 * 4 * 6
    assert r["i_rel_max"] == pytest.approx(3e-5, rel=0.02)
    assert r["pol_abs_max"] == pytest.approx(2e-6, rel=0.02)
    assert r["jkq_rel_j00_max"] == pytest.approx(4e-7, rel=1e-6)
    assert r["lbar_rel_max"] == pytest.approx(5e-8, rel=1e-6)


def test_bench_algorithmic_bytes():
    """The algorithmic bytes per plane launch that the roofline divides by: per update the
    upwind Stokes vector read and the new one written (16 + 16 B in FP32), per node the
    three coefficient planes (3 x 52 B) and J read and written (160 B); the adjoint reads
    two Stokes vectors and writes one per update and writes 33 partials per node and ray."""
    import bench
    from paper_1307_4217_amd import inputs
    cfg = inputs.CONFIGS["C3"]
    np_ = cfg.nx * cfg.ny
    b, upd = bench.sweep_launch_bytes(cfg, 40, 4)
    assert upd == 40 * 101 * np_
    assert b == 40 * 101 * np_ * 32 + np_ * (3 * 52 + 160)
    a, aupd = bench.adjoint_launch_bytes(cfg, 16, 4)
    assert aupd == 16 * 101 * np_
    assert a == 16 * 101 * np_ * 48 + 16 * np_ * 33 * 4 + 3 * np_ * 13 * 4
