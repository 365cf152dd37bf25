"""Non-linear multigrid (FAS) iteration of the two-level problem on the GPU (Sect. 5).

Each level is a grid with every second node of the finer one (x, y periodic with even
n_x, n_y; z with odd n_z), its model sampled at those nodes (porta_mg_inject), and the
same quadrature.  A V-cycle on level l (Sect. 5.1):

  nu1 Jacobi iterations           porta_fs_sweep + porta_see_update (rhs f_l)
  residual r = f - L(rho) rho     porta_fs_sweep + porta_see_operator (sign -1)
  rho_c = R(rho), R(r)            porta_mg_restrict (also emis_c = kappa_c rho_c)
  f_c = L_c(rho_c) rho_c + R(r)   porta_fs_sweep + porta_see_operator (sign +1), Eq. mgcsfy
  solve on level l+1              the next V-cycle, or ncoarse Jacobi iterations
  rho += P(rho_c_new - rho_c)     porta_mg_prolong (also emis = kappa rho)
  nu2 Jacobi iterations

The unknowns rho are the source-function multipoles S^K_Q (emissivity = kappa S).  All
arithmetic runs in the library's kernels; this module only holds device buffers and
orders the calls.

    python -m paper_1307_4217_amd.multigrid --nx 128 --nz 97 --levels 3 --cycles 4
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import sys
import time

import numpy as np

from . import inputs, porta


class Level:
    """Device state of one grid of the hierarchy."""

    def __init__(self, hg, kappa, propmat, hanle, bhat, atom, i_bottom, prec, opts, dev):
        import torch
        self.hg, self.prec, self.opts, self.dev = hg, prec, opts, dev
        self.kappa, self.propmat, self.hanle, self.bhat = kappa, propmat, hanle, bhat
        self.atom, self.i_bottom = atom, float(i_bottom)
        n = hg.N
        f64 = dict(dtype=torch.float64, device=dev)
        self.S = torch.empty((6, n), **f64)
        self.S_alt = torch.empty((6, n), **f64)
        self.S0 = torch.empty((6, n), **f64)      # R(rho_fine) while this is a coarse level
        self.f = torch.empty((6, n), **f64)       # right-hand side while a coarse level
        self.r = torch.empty((6, n), **f64)
        self.emis = torch.empty((6, n), dtype=kappa.dtype, device=dev)
        self.jkq = torch.empty((10, n), **f64)
        self.ws = torch.empty(porta.workspace_size(hg, prec, porta.WS_SWEEP, 1, opts),
                              dtype=torch.uint8, device=dev)
        self.ws_see = torch.empty(8 * ((n + 255) // 256) + 256, dtype=torch.uint8, device=dev)

    @property
    def dims(self):
        return self.hg.nx, self.hg.ny, self.hg.nz

    def formal_solution(self):
        """J^K_Q and Lambda-bar of the current emissivities into self.jkq."""
        porta.fs_sweep(self.hg, self.kappa, self.propmat, self.emis, self.i_bottom,
                       self.atom["w2"], prec=self.prec, jkq=self.jkq, want_itop=False,
                       opts=self.opts, workspace=self.ws)

    def jacobi(self, rhs=None):
        """One Jacobi iteration of L(rho) rho = rhs (None: eps_c B)."""
        self.formal_solution()
        porta.see_update(self.jkq, self.S, s_new=self.S_alt, kappa=self.kappa,
                         emis_out=self.emis, prec=self.prec, want_rc=False,
                         workspace=self.ws_see, rhs=rhs, hanle=self.hanle, bhat=self.bhat,
                         **self.atom)
        self.S, self.S_alt = self.S_alt, self.S

    def operator(self, base, sign, out):
        """out = base + sign L(rho) rho, with J from a formal solution of the current S."""
        self.formal_solution()
        porta.see_operator(self.jkq, self.S, base=base, sign=sign, out=out, hanle=self.hanle,
                           bhat=self.bhat, **self.atom)


def _atom_args(atm):
    return dict(eps_c=atm.eps_c, delta2=atm.delta2, w2=atm.w2, planck=atm.planck)


class MultigridSolver:
    """Hierarchy of `nlevels` grids over the atmosphere `atm` (finest first).  The formal
    solutions run in `prec`; set_precision() switches between FP32 and FP64 sweeps
    keeping the current iterate (J, the SEE and the transfers are FP64 either way)."""

    def __init__(self, atm, quad, nlevels=2, prec=porta.F64, device="cuda:0", opts=None,
                 nu1=2, nu2=4, ncoarse=20, order=1):
        import torch
        self.torch = torch
        self.atm, self.quad, self.nlevels, self.opts = atm, quad, nlevels, opts
        self.nu1, self.nu2, self.ncoarse = nu1, nu2, ncoarse
        self.order = order          # prolongation: 1 tri-linear, 3 tri-cubic-centred
        self.dev = torch.device(device)
        self.levels = []
        self._build_levels(prec)
        fine = self.levels[0]
        fine.S.copy_(torch.as_tensor(np.ascontiguousarray(atm.source), dtype=torch.float64,
                                     device=self.dev))
        porta.emissivity(fine.kappa, fine.S, emis=fine.emis)
        self.S_prev = torch.empty_like(fine.S)
        self.rc = torch.empty((), dtype=torch.float64, device=self.dev)
        self.cycles = 0

    def _build_levels(self, prec):
        torch, atm, quad, dev = self.torch, self.atm, self.quad, self.dev
        dt = porta.dtype_of(prec)
        t = lambda a, d: None if a is None else torch.as_tensor(np.ascontiguousarray(a), dtype=d,
                                                                  device=dev)
        atom = _atom_args(atm)
        hg = porta.HostGrid.from_inputs(atm, quad)
        levels = [Level(hg, t(atm.kappa, dt), t(atm.propmat, dt), t(atm.hanle, torch.float64),
                        t(atm.bhat, torch.float64), atom, atm.i_bottom, prec, self.opts, dev)]
        z = np.asarray(atm.z, dtype=np.float64)
        for _ in range(self.nlevels - 1):
            up = levels[-1]
            nx, ny, nz = up.dims
            z = z[::2]
            hgc = porta.HostGrid(nx // 2, ny // 2, (nz + 1) // 2, atm.lx, atm.ly, z, quad.mu,
                                 quad.wmu, quad.nchi, quad.phi, quad.wfreq)
            inj = lambda a: None if a is None else porta.mg_inject(a, nx, ny, nz)
            levels.append(Level(hgc, inj(up.kappa), inj(up.propmat), inj(up.hanle),
                                inj(up.bhat), atom, atm.i_bottom, prec, self.opts, dev))
        self.levels = levels
        self.prec = prec

    def set_precision(self, prec):
        """Continue with formal solutions in `prec` from the current iterate."""
        if prec == self.prec:
            return
        S = self.levels[0].S.clone()
        self.levels = []
        self.torch.cuda.empty_cache()
        self._build_levels(prec)
        fine = self.levels[0]
        fine.S.copy_(S)
        porta.emissivity(fine.kappa, fine.S, emis=fine.emis)

    @property
    def source(self):
        return self.levels[0].S

    def _vcycle(self, l, rhs):
        lev = self.levels[l]
        if l == len(self.levels) - 1:
            for _ in range(self.ncoarse):
                lev.jacobi(rhs)
            return
        for _ in range(self.nu1):
            lev.jacobi(rhs)
        lev.operator(rhs, -1.0, lev.r)                      # r = f - L(rho) rho
        co = self.levels[l + 1]
        nx, ny, nz = lev.dims
        porta.mg_restrict(lev.S, nx, ny, nz, out=co.S0, kappa_c=co.kappa, emis_c=co.emis,
                          prec=lev.prec)
        co.S.copy_(co.S0)
        porta.mg_restrict(lev.r, nx, ny, nz, out=co.r, prec=lev.prec)
        co.operator(co.r, 1.0, co.f)                        # f_c = L_c(R rho) R rho + R r
        self._vcycle(l + 1, co.f)
        porta.mg_prolong(lev.S, nx, ny, nz, co.S, co.S0, kappa=lev.kappa, emis=lev.emis,
                         prec=lev.prec, order=self.order)
        for _ in range(self.nu2):
            lev.jacobi(rhs)

    def vcycle(self):
        """One V-cycle on the finest grid; returns the device scalar R_c of the cycle."""
        fine = self.levels[0]
        self.S_prev.copy_(fine.S)
        self._vcycle(0, None)
        self.cycles += 1
        return porta.rel_change(fine.S, self.S_prev, rc=self.rc, workspace=fine.ws_see)

    def nested(self, cycles=1):
        """Nested multigrid from the current finest-grid S: that S sampled on the
        coarsest grid is relaxed by ncoarse Jacobi iterations, and each finer grid
        starts from the prolonged solution of the grid below and takes `cycles`
        V-cycles (Sect. 5; the nested scheme of Fabiani Bendicho et al.).  Returns the
        device scalar R_c of the last finest-grid cycle."""
        fine = self.levels[0]
        self.S_prev.copy_(fine.S)
        top = len(self.levels) - 1
        for l in range(top):                      # initial guess on every grid
            up, lo = self.levels[l], self.levels[l + 1]
            lo.S.copy_(porta.mg_inject(up.S, *up.dims))
        co = self.levels[top]
        porta.emissivity(co.kappa, co.S, emis=co.emis)
        for _ in range(self.ncoarse):
            co.jacobi(None)
        for l in range(top - 1, -1, -1):
            lev, lo = self.levels[l], self.levels[l + 1]
            lev.S.zero_()
            porta.mg_prolong(lev.S, *lev.dims, lo.S, kappa=lev.kappa, emis=lev.emis,
                             prec=lev.prec, order=self.order)
            for _ in range(cycles):
                self._vcycle(l, None)
        self.cycles += 1
        return porta.rel_change(fine.S, self.S_prev, rc=self.rc, workspace=fine.ws_see)

    def fine_sweeps_per_cycle(self):
        """Work of one V-cycle in units of one formal solution on the finest grid."""
        work, scale = 0.0, 1.0
        for l in range(len(self.levels)):
            if l == len(self.levels) - 1:
                work += scale * self.ncoarse
            else:
                work += scale * (self.nu1 + self.nu2 + 1) + scale / 8.0   # + f_c on l+1
            scale /= 8.0
        return work


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--nx", type=int, default=128)
    ap.add_argument("--nz", type=int, default=97)
    ap.add_argument("--nmu", type=int, default=5)
    ap.add_argument("--nchi", type=int, default=16)
    ap.add_argument("--nfreq", type=int, default=41)
    ap.add_argument("--levels", type=int, default=3)
    ap.add_argument("--cycles", type=int, default=4)
    ap.add_argument("--tol", type=float, default=0.0,
                    help="stop once R_c falls below this (the cycles and the Jacobi iterations)")
    ap.add_argument("--jacobi", type=int, default=0, help="also run this many Jacobi iterations")
    ap.add_argument("--ncoarse", type=int, default=20)
    ap.add_argument("--ray-batch", type=int, default=40)
    ap.add_argument("--cubic", action="store_true", help="tri-cubic-centred prolongation")
    ap.add_argument("--nested", action="store_true",
                    help="start with one nested-multigrid pass instead of a V-cycle")
    ap.add_argument("--prec", default="f64", choices=["f32", "f64"])
    ap.add_argument("--fp32-until", type=float, default=0.0,
                    help="sweep in FP32 until R_c drops below this value, then in FP64")
    ap.add_argument("--with-propmat", action="store_true",
                    help="keep the random dichroism/dispersion terms of the synthetic model")
    args = ap.parse_args(argv)
    cfg = inputs.Config("mg", args.nx, args.nx, args.nz, args.nmu, args.nchi, args.nfreq, True)
    atm = inputs.make_atmosphere(cfg, seed=0)
    if not args.with_propmat:
        atm = dataclasses.replace(atm, propmat=0 * atm.propmat)
    q = inputs.make_quadrature(cfg)
    prec = porta.F64 if args.prec == "f64" else porta.F32
    if args.fp32_until > 0:
        prec = porta.F32
    import torch
    solver = MultigridSolver(atm, q, args.levels, prec, ncoarse=args.ncoarse,
                             opts=porta.options(ray_batch=args.ray_batch),
                             order=3 if args.cubic else 1)
    work = solver.fine_sweeps_per_cycle()
    t0 = time.perf_counter()
    rc = None   # no cycle run (--cycles 0, e.g. to time Jacobi alone)
    for c in range(args.cycles):
        rc = float((solver.nested() if (args.nested and c == 0) else solver.vcycle()).item())
        print(json.dumps({"cycle": c + 1, "R_c": rc, "fine_sweeps": round(work * (c + 1), 2),
                          "sweep_prec": "f32" if solver.prec == porta.F32 else "f64",
                          "elapsed_s": round(time.perf_counter() - t0, 3)}), flush=True)
        if rc < args.tol:
            break
        if args.fp32_until > 0 and rc < args.fp32_until:
            solver.set_precision(porta.F64)
    mg_s = time.perf_counter() - t0
    out = {"grid": [args.nx, args.nx, args.nz], "levels": args.levels, "cycles": solver.cycles,
           "rays": cfg.nrays, "freqs": args.nfreq, "prec": args.prec, "mg_seconds": round(mg_s, 3),
           "final_R_c": rc, "fine_sweeps_per_cycle": round(work, 3)}
    if args.jacobi:
        from .jacobi import JacobiSolver
        js = JacobiSolver(atm, q, prec, opts=porta.options(ray_batch=args.ray_batch))
        t0 = time.perf_counter()
        its = 0
        for it in range(args.jacobi):
            rcj = float(js.step().item())
            its = it + 1
            if its % 10 == 0:
                print(json.dumps({"jacobi": its, "R_c": rcj}), flush=True)
            if rcj < args.tol:
                break
        torch.cuda.synchronize()
        out.update({"jacobi_iterations": its, "jacobi_final_R_c": rcj,
                    "jacobi_seconds": round(time.perf_counter() - t0, 3)})
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
