"""The allocation-free sweep entry point (porta_fs_sweep_noalloc) against porta_fs_sweep.

Both run the same kernels with the same launch shapes; only the workspace differs (the
library's static device scratch against a caller buffer), so the results must agree
bit for bit.  Two calls in a row: the second on a smaller problem in the other
precision, so it runs on the scratch the first one left behind."""
import dataclasses

import numpy as np
import pytest

from gpu_common import require_gpu, rounded, to_dev
from paper_1307_4217_amd import inputs, porta

pytestmark = pytest.mark.gpu


def _case(cfg, seed, prec):
    atm = inputs.make_atmosphere(cfg, seed=seed)
    if prec == porta.F32:
        atm = rounded(atm, np.float32)
    return atm, inputs.make_quadrature(cfg)


def _both(atm, q, prec, opts=None, accumulate=False):
    torch = require_gpu()
    dt = torch.float64 if prec == porta.F64 else torch.float32
    hg = porta.HostGrid.from_inputs(atm, q)
    kappa, prop, emis = to_dev(atm.kappa, dt), to_dev(atm.propmat, dt), to_dev(atm.emis, dt)
    j_ref, it_ref = porta.fs_sweep(hg, kappa, prop, emis, atm.i_bottom, atm.w2, prec=prec,
                                   opts=opts)
    jkq = torch.full((10, hg.N), 7.0, dtype=torch.float64, device="cuda")
    it = torch.full(it_ref.shape, 7.0, dtype=dt, device="cuda")
    porta.fs_sweep_noalloc(hg, kappa, prop, emis, atm.i_bottom, jkq, it, atm.w2, prec=prec,
                           opts=opts)
    torch.cuda.synchronize()
    return (jkq.cpu().numpy(), it.cpu().numpy()), (j_ref.cpu().numpy(), it_ref.cpu().numpy())


def test_noalloc_sweep_equals_sweep_twice_second_smaller():
    print("noalloc: 16x16x32, 80 rays, 21 freq, FP64", flush=True)
    atm, q = _case(inputs.CONFIGS["C1"], 0, porta.F64)
    (j1, i1), (jr1, ir1) = _both(atm, q, porta.F64)
    assert np.isfinite(i1).all() and np.abs(i1[..., 0]).min() > 0
    np.testing.assert_array_equal(j1, jr1)
    np.testing.assert_array_equal(i1, ir1)

    print("noalloc: ragged 7x5x9, 12 rays, 5 freq, FP32, ray batches of 3", flush=True)
    cfg = inputs.Config("ragged", 7, 5, 9, 2, 3, 5, True)
    atm, q = _case(cfg, 3, porta.F32)
    atm = dataclasses.replace(atm, lx=530.0, ly=410.0)
    (j2, i2), (jr2, ir2) = _both(atm, q, porta.F32, opts=porta.options(ray_batch=3, block=64))
    assert np.isfinite(i2).all()
    np.testing.assert_array_equal(j2, jr2)
    np.testing.assert_array_equal(i2, ir2)


def test_noalloc_sweep_rejects_a_problem_beyond_its_scratch():
    torch = require_gpu()
    cfg = inputs.CONFIGS["C1"]
    atm, q = _case(cfg, 0, porta.F64)
    hg = porta.HostGrid.from_inputs(atm, q)
    big = porta.HostGrid(256, 256, atm.nz, atm.lx, atm.ly, atm.z, q.mu, q.wmu, q.nchi, q.phi,
                         q.wfreq)
    assert porta.workspace_size(big, porta.F64, porta.WS_SWEEP) > 64 << 20
    x = torch.zeros(16, dtype=torch.float64, device="cuda")
    with pytest.raises(porta.PortaError) as e:
        porta.fs_sweep_noalloc(big, x, x, x, 1.0, x, x)
    assert e.value.status == porta.ENOMEM
    # the same problem fits once its ray batch is small enough
    opts = porta.options(ray_batch=2)
    assert porta.workspace_size(hg, porta.F64, porta.WS_SWEEP, 1, opts) < 64 << 20
