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
        self.atm, self.quad, self.prec = atm, quad, prec
        self.dev = torch.device(device)
        dt = porta.dtype_of(prec)
        t = lambda a, d: torch.as_tensor(np.ascontiguousarray(a), dtype=d, device=self.dev)
        self.hg = porta.HostGrid.from_inputs(atm, quad)
        self.kappa = t(atm.kappa, dt)
        self.prop = t(atm.propmat, dt)
        self.emis = t(atm.emis, dt)
        self.S = [t(atm.source, torch.float64), torch.empty((6, atm.npoints),
                                                            dtype=torch.float64, device=self.dev)]
        self.hanle = None if atm.hanle is None else t(atm.hanle, torch.float64)
        self.bhat = None if atm.bhat is None else t(atm.bhat, torch.float64)
        self.opts = opts
        self.jkq = torch.empty((10, atm.npoints), dtype=torch.float64, device=self.dev)
        self.rc = torch.empty((), dtype=torch.float64, device=self.dev)
        self.ws = torch.empty(porta.workspace_size(self.hg, prec, porta.WS_SWEEP, 1, opts),
                              dtype=torch.uint8, device=self.dev)
        self.ws_see = torch.empty(8 * ((atm.npoints + 255) // 256) + 256, dtype=torch.uint8,
                                  device=self.dev)
        self.iteration = 0
        self.history = []

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

    def solve(self, max_iter=50, tol=1e-6, callback=None):
        """Iterate until R_c < tol or max_iter; returns the list of R_c values."""
        hist = []
        for _ in range(max_iter):
            rc = float(self.step().item())
            hist.append(rc)
            self.history.append(rc)
            if callback:
                callback(self.iteration, rc)
            if rc < tol:
                break
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
        """Resume from a file written by save() for the same grid, quadrature and
        precision; the next step() continues the iteration exactly."""
        with np.load(path, allow_pickle=False) as f:
            a = self.atm
            want = [a.nx, a.ny, a.nz, self.hg.nrays, self.hg.nfreq]
            if list(f["shape"]) != want or int(f["prec"]) != self.prec:
                raise ValueError(f"{path} holds an iterate of shape {list(f['shape'])} "
                                 f"(prec {int(f['prec'])}), not {want} (prec {self.prec})")
            self.S[0].copy_(self.torch.as_tensor(f["source"]))
            self.emis.copy_(self.torch.as_tensor(f["emis"]))
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
    args = ap.parse_args(argv)
    cfg = inputs.CONFIGS[args.config]
    atm = inputs.make_atmosphere(cfg, seed=0)
    q = inputs.make_quadrature(cfg)
    prec = porta.F64 if args.prec == "f64" else porta.F32
    solver = JacobiSolver(atm, q, prec, opts=porta.options(ray_batch=args.ray_batch))
    if args.resume:
        solver.load(args.resume)
    t0 = time.perf_counter()

    def report(it, rc):
        print(json.dumps({"iteration": it, "R_c": rc, "elapsed_s": round(time.perf_counter() - t0,
                                                                        3)}), flush=True)
    hist = solver.solve(args.iters, args.tol, report)
    dt = time.perf_counter() - t0
    print(json.dumps({"config": cfg.name, "grid": [cfg.nx, cfg.ny, cfg.nz], "rays": cfg.nrays,
                      "freqs": cfg.nfreq, "prec": args.prec, "iterations": len(hist),
                      "final_R_c": hist[-1], "converged": hist[-1] < args.tol,
                      "seconds": round(dt, 2),
                      "updates_per_s": cfg.updates * len(hist) / dt,
                      "total_iterations": solver.iteration}), flush=True)
    if args.save:
        solver.save(args.save)
    return 0


if __name__ == "__main__":
    sys.exit(main())
