"""Jacobi iteration of the two-level NLTE problem on the GPU (Sect. 5 of the paper).

Each iteration is one formal solution of every ray and frequency with the
fused J^K_Q / Lambda* integration (porta_fs_sweep), followed by the per-point
statistical-equilibrium update (porta_see_update) that rewrites the
emissivities for the next sweep.  The convergence measure is
R_c = max |dS00| / S00, read back once per iteration.

The iterate (S^K_Q, the emissivities of the next sweep, the iteration count and
the R_c history) can be saved and the iteration resumed from it: the paper's
restart from a stored, partially converged solution (the radiation field itself
is never stored).

    python -m paper_1307_4217_amd.jacobi --config C2 --prec f64 --iters 50 [--save s.npz]
    python -m paper_1307_4217_amd.jacobi --config C2 --prec f64 --iters 20 --resume s.npz
    python -m paper_1307_4217_amd.jacobi --config C5 --fp32-until 1e-4 --tol 1e-5 --iters 400
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import inputs, porta


class JacobiSolver:
    """Device-resident state of the Jacobi iteration for one atmosphere."""

    def __init__(self, atm, quad, prec=porta.F64, device="cuda:0", opts=None):
        import torch
        self.torch = torch
        self.atm, self.quad = atm, quad
        self.dev = torch.device(device)
        self.hg = porta.HostGrid.from_inputs(atm, quad)
        self.opts = opts
        self.S = [self._dev(atm.source, torch.float64),
                  torch.empty((6, atm.npoints), dtype=torch.float64, device=self.dev)]
        self.hanle = None if atm.hanle is None else self._dev(atm.hanle, torch.float64)
        self.bhat = None if atm.bhat is None else self._dev(atm.bhat, torch.float64)
        self.jkq = torch.empty((10, atm.npoints), dtype=torch.float64, device=self.dev)
        self.rc = torch.empty((), dtype=torch.float64, device=self.dev)
        self.ws_see = torch.empty(8 * ((atm.npoints + 255) // 256) + 256, dtype=torch.uint8,
                                  device=self.dev)
        self.prec = None
        self._set_fields(prec)
        self.emis = self._dev(self.atm.emis, porta.dtype_of(prec))
        self.iteration = 0
        self.history = []

    def _dev(self, a, dt):
        return self.torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=self.dev)

    def _set_fields(self, prec):
        """Transfer coefficients and sweep workspace in the precision `prec`."""
        self.prec = prec
        dt = porta.dtype_of(prec)
        self.kappa = self._dev(self.atm.kappa, dt)
        self.prop = self._dev(self.atm.propmat, dt)
        self.ws = None
        self.torch.cuda.empty_cache()
        self.ws = self.torch.empty(porta.workspace_size(self.hg, prec, porta.WS_SWEEP, 1,
                                                        self.opts),
                                   dtype=self.torch.uint8, device=self.dev)

    def set_precision(self, prec):
        """Continue the iteration with formal solutions in `prec`: the transfer
        coefficients are taken again in that precision and the emissivities of the next
        sweep formed from the current S^K_Q (porta_emissivity)."""
        if prec == self.prec:
            return
        self.emis = None
        self._set_fields(prec)
        self.emis = porta.emissivity(self.kappa, self.S[0])

    @property
    def source(self):
        """Current source-function multipoles S^K_Q, [6][N] float64 on the device."""
        return self.S[0]

    def step(self):
        """One Jacobi iteration; returns the device scalar R_c."""
        porta.fs_sweep(self.hg, self.kappa, self.prop, self.emis, self.atm.i_bottom,
                       self.atm.w2, prec=self.prec, jkq=self.jkq, want_itop=False,
                       opts=self.opts, workspace=self.ws)
        porta.see_update(self.jkq, self.S[0], self.atm.eps_c, self.atm.delta2, self.atm.w2,
                         self.atm.planck, self.hanle, self.bhat, kappa=self.kappa,
                         emis_out=self.emis, prec=self.prec, s_new=self.S[1], rc=self.rc,
                         workspace=self.ws_see)
        self.S.reverse()
        self.iteration += 1
        return self.rc

    def solve(self, max_iter=50, tol=1e-6, callback=None, fp32_until=0.0, max_seconds=0.0):
        """Iterate until R_c < tol or max_iter (or, with max_seconds > 0, until that much
        wall time has passed); returns the list of R_c values.  With fp32_until > 0, FP32
        sweeps continue in FP64 once R_c falls below it."""
        hist = []
        t0 = time.perf_counter()
        for _ in range(max_iter):
            if max_seconds > 0 and hist and time.perf_counter() - t0 > max_seconds:
                break
            rc = float(self.step().item())
            hist.append(rc)
            self.history.append(rc)
            if callback:
                callback(self.iteration, rc)
            if rc < tol:
                break
            if fp32_until > 0 and rc < fp32_until:
                self.set_precision(porta.F64)
        return hist

    def save(self, path):
        """Write the iterate to an .npz file: S^K_Q (FP64), the emissivities of the next
        sweep (sweep precision), the iteration count, the R_c history and the shapes
        it belongs to."""
        a = self.atm
        np.savez(path, source=self.S[0].cpu().numpy(), emis=self.emis.cpu().numpy(),
                 iteration=self.iteration, history=np.asarray(self.history, dtype=np.float64),
                 shape=np.asarray([a.nx, a.ny, a.nz, self.hg.nrays, self.hg.nfreq]),
                 prec=self.prec)

    def load(self, path):
        """Resume from a file written by save() for the same grid and quadrature.  In the
        precision it was saved in, the next step() continues the iteration exactly; in
        the other one, the emissivities are formed from the saved S^K_Q as
        set_precision() forms them."""
        with np.load(path, allow_pickle=False) as f:
            a = self.atm
            want = [a.nx, a.ny, a.nz, self.hg.nrays, self.hg.nfreq]
            if list(f["shape"]) != want:
                raise ValueError(f"{path} holds an iterate of shape {list(f['shape'])}, "
                                 f"not {want}")
            self.S[0].copy_(self.torch.as_tensor(f["source"]))
            if int(f["prec"]) == self.prec:
                self.emis.copy_(self.torch.as_tensor(f["emis"]))
            else:
                porta.emissivity(self.kappa, self.S[0], emis=self.emis)
            self.iteration = int(f["iteration"])
            self.history = [float(x) for x in f["history"]]


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--config", default="C2")
    ap.add_argument("--prec", default="f64", choices=["f32", "f64"])
    ap.add_argument("--iters", type=int, default=50)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--ray-batch", type=int, default=0)
    ap.add_argument("--save", default="", help="write the final iterate to this .npz file")
    ap.add_argument("--resume", default="", help="start from an iterate written by --save")
    ap.add_argument("--fp32-until", type=float, default=0.0,
                    help="sweep in FP32 until R_c drops below this value, then in FP64")
    ap.add_argument("--max-seconds", type=float, default=0.0,
                    help="start no iteration after this much wall time")
    args = ap.parse_args(argv)
    cfg = inputs.CONFIGS[args.config]
    atm = inputs.make_atmosphere(cfg, seed=0)
    q = inputs.make_quadrature(cfg)
    prec = porta.F64 if args.prec == "f64" and args.fp32_until <= 0 else porta.F32
    solver = JacobiSolver(atm, q, prec, opts=porta.options(ray_batch=args.ray_batch))
    if args.resume:
        solver.load(args.resume)
    t0 = time.perf_counter()

    def report(it, rc):
        print(json.dumps({"iteration": it, "R_c": rc,
                          "sweep_prec": "f32" if solver.prec == porta.F32 else "f64",
                          "elapsed_s": round(time.perf_counter() - t0, 3)}), flush=True)
    hist = solver.solve(args.iters, args.tol, report, fp32_until=args.fp32_until,
                        max_seconds=args.max_seconds)
    dt = time.perf_counter() - t0
    print(json.dumps({"config": cfg.name, "grid": [cfg.nx, cfg.ny, cfg.nz], "rays": cfg.nrays,
                      "freqs": cfg.nfreq, "prec": args.prec, "fp32_until": args.fp32_until,
                      "iterations": len(hist), "final_R_c": hist[-1],
                      "converged": hist[-1] < args.tol, "seconds": round(dt, 2),
                      "updates_per_s": cfg.updates * len(hist) / dt,
                      "total_iterations": solver.iteration}), flush=True)
    if args.save:
        solver.save(args.save)
    return 0


if __name__ == "__main__":
    sys.exit(main())
