"""Helpers shared by the GPU parity tests (inputs, oracle runs, tolerances)."""
import functools

import numpy as np

from paper_1307_4217_amd import inputs, porta


def require_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    return torch


def to_dev(a, dtype):
    torch = require_gpu()
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def rounded(atm, dtype):
    """Copy of `atm` whose material arrays are rounded to `dtype` (then held in FP64)."""
    import dataclasses
    return dataclasses.replace(
        atm, kappa=atm.kappa.astype(dtype).astype(np.float64),
        propmat=atm.propmat.astype(dtype).astype(np.float64),
        emis=atm.emis.astype(dtype).astype(np.float64))


class Case:
    """One problem on the GPU: host grid plus device fields in the sweep precision."""

    def __init__(self, atm, quad, prec):
        torch = require_gpu()
        self.atm, self.quad, self.prec = atm, quad, prec
        dt = torch.float64 if prec == porta.F64 else torch.float32
        self.dt = dt
        self.hg = porta.HostGrid.from_inputs(atm, quad)
        self.kappa = to_dev(atm.kappa, dt)
        self.prop = to_dev(atm.propmat, dt)
        self.emis = to_dev(atm.emis, dt)

    def sweep(self, **kw):
        import torch
        j, it = porta.fs_sweep(self.hg, self.kappa, self.prop, self.emis, self.atm.i_bottom,
                               self.atm.w2, prec=self.prec, **kw)
        torch.cuda.synchronize()
        return (None if j is None else j.cpu().numpy(), None if it is None else it.cpu().numpy())


def compare_stokes(got, ref, tol_i, tol_pol, what=""):
    """I relative to tol_i; Q/I, U/I, V/I absolute to tol_pol."""
    gi, ri = got[..., 0], ref[..., 0]
    rel = np.abs(gi - ri) / np.abs(ri)
    assert rel.max() <= tol_i, f"{what} Stokes I max rel err {rel.max():.3e} > {tol_i}"
    for s, name in ((1, "Q/I"), (2, "U/I"), (3, "V/I")):
        d = np.abs(got[..., s] / gi - ref[..., s] / ri)
        assert d.max() <= tol_pol, f"{what} {name} max abs err {d.max():.3e} > {tol_pol}"
    return rel.max(), max(np.abs(got[..., s] / gi - ref[..., s] / ri).max() for s in (1, 2, 3))


def compare_jkq(got, ref, tol, what=""):
    """Each J^K_Q component and Lbar to tol relative to the scale of J00."""
    scale = np.abs(ref[0]).max()
    err = np.abs(got - ref).max(axis=1) / scale
    assert err.max() <= tol, f"{what} J max err/scale per component {err}"
    return err.max()


@functools.lru_cache(maxsize=8)
def oracle_full(cfg_name, seed, dtype_name, magnetic=None):
    """Oracle sweep (all rays/frequencies) of a named configuration, cached per session."""
    from oracle import oracle as orc
    cfg = inputs.CONFIGS[cfg_name]
    atm = inputs.make_atmosphere(cfg, seed=seed, magnetic=magnetic)
    if dtype_name == "f32":
        atm = rounded(atm, np.float32)
    q = inputs.make_quadrature(cfg)
    out = orc.fs_sweep(orc.OracleProblem(atm, q))
    out["itop"] = up_rays(out["itop"], q)
    return atm, q, out


def up_rays(itop, q):
    """The oracle returns I_top for every selected ray; keep the upward ones."""
    return itop[: len(q.mu) * q.nchi]
