"""Non-linear multigrid (FAS) iteration of the two-level problem (Sect. 5 of the paper),
written plainly on top of the oracle's formal solver and statistical equilibrium.

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU-baseline leg of the
benchmark may import this module.  The GPU library never calls it.

Grids: the grid of level l-1 keeps every second node of level l along each axis, so
coarse node (i, j, k) is fine node (2i, 2j, 2k) (Sect. 5.1).  x and y are periodic
(n_x, n_y even); z is not (n_z odd, both boundary planes kept).  Fields are [c][N]
arrays with x fastest, N = n_z n_y n_x.

Readings where the paper is silent:
* the unknowns rho are represented by the source-function multipoles S^K_Q of the
  two-level atom (emissivity = kappa S);
* the model atmosphere of a coarse grid (opacities, propagation matrix, field) is the
  fine one sampled at the coarse nodes (injection); the quadrature is the same;
* the restriction is the adjoint of tri-linear prolongation divided by the sum of its
  weights, so that it maps a constant to itself; at a z boundary this leaves the
  2 x 3^2 nodes of Sect. 5.2 with z weights (2/3, 1/3);
* the coarsest grid is "solved" by a fixed number of Jacobi iterations.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import oracle as orc


def coarse_shape(nx, ny, nz):
    if nx % 2 or ny % 2 or nz % 2 == 0 or nz < 3:
        raise ValueError("coarsening needs even n_x, n_y and odd n_z >= 3")
    return nx // 2, ny // 2, (nz + 1) // 2


# ----------------------------------------------------------------- transfer operators
def _linear_1d(c, axis, periodic):
    """Linear interpolation along one axis to twice the resolution: node 2i takes
    c[i], node 2i+1 the mean of c[i] and c[i+1] (periodic axis: n_f = 2 n_c;
    otherwise n_f = 2 n_c - 1)."""
    c = np.moveaxis(c, axis, 0)
    n = c.shape[0]
    nf = 2 * n if periodic else 2 * n - 1
    out = np.empty((nf,) + c.shape[1:])
    for i in range(nf):
        if i % 2 == 0:
            out[i] = c[i // 2]
        else:
            out[i] = 0.5 * (c[i // 2] + c[(i // 2 + 1) % n])
    return np.moveaxis(out, 0, axis)


def _lagrange_weights(nodes, x):
    """Weights of the Lagrange polynomial through `nodes` evaluated at x."""
    w = []
    for a in nodes:
        v = 1.0
        for b in nodes:
            if b != a:
                v *= (x - b) / (a - b)
        w.append(v)
    return w


def _cubic_1d(c, axis, periodic):
    """Cubic interpolation along one axis to twice the resolution: node 2i takes c[i];
    node 2i+1 takes the cubic through the four coarse nodes around it, i-1 .. i+2
    (periodic axis), or, next to the ends of a non-periodic axis, through the four
    nodes nearest to it inside the axis (Sect. 5.2)."""
    c = np.moveaxis(c, axis, 0)
    n = c.shape[0]
    nf = 2 * n if periodic else 2 * n - 1
    out = np.empty((nf,) + c.shape[1:])
    for i in range(nf):
        if i % 2 == 0:
            out[i] = c[i // 2]
            continue
        x = i / 2.0                                  # position in coarse units
        if periodic:
            base = i // 2 - 1
            nodes = [base, base + 1, base + 2, base + 3]
            idx = [m % n for m in nodes]
        else:
            base = min(max(i // 2 - 1, 0), n - 4)
            nodes = [base, base + 1, base + 2, base + 3]
            idx = nodes
        w = _lagrange_weights(nodes, x)
        out[i] = sum(wk * c[m] for wk, m in zip(w, idx))
    return np.moveaxis(out, 0, axis)


def prolong(c, nxc, nyc, nzc, order=1):
    """Prolongation (Sect. 5.2): coarse [k][nzc*nyc*nxc] -> fine [k][N_f].
    order 1, tri-linear: nodes on coarse nodes take the coarse value, nodes on coarse
    lines and planes are interpolated linearly and bilinearly, the rest tri-linearly.
    order 3, tri-cubic-centred: the same with cubic interpolation through four coarse
    nodes per axis (4^3 nodes for the tri-cubic case); needs n_z of the coarse grid
    >= 4.  Both are tensor products of one-dimensional interpolations along z, y, x."""
    c = np.asarray(c, dtype=np.float64)
    k = c.shape[0]
    g = c.reshape(k, nzc, nyc, nxc)
    one_d = _linear_1d if order == 1 else _cubic_1d
    g = one_d(g, 1, periodic=False)
    g = one_d(g, 2, periodic=True)
    g = one_d(g, 3, periodic=True)
    return g.reshape(k, -1)


def restrict(f, nx, ny, nz):
    """Restriction (Sect. 5.2): at each coarse node, the weighted mean of the 3^3 fine
    nodes around it with weights w(dx) w(dy) w(dz), w(0) = 1, w(+-1) = 1/2 (the
    adjoint of tri-linear prolongation), over the nodes that exist."""
    f = np.asarray(f, dtype=np.float64)
    k = f.shape[0]
    nxc, nyc, nzc = coarse_shape(nx, ny, nz)
    g = f.reshape(k, nz, ny, nx)
    out = np.zeros((k, nzc, nyc, nxc))
    w = {-1: 0.5, 0: 1.0, 1: 0.5}
    for kc in range(nzc):
        wsum = 0.0
        for dz in (-1, 0, 1):
            kf = 2 * kc + dz
            if kf < 0 or kf >= nz:
                continue
            for dy in (-1, 0, 1):
                rows = (2 * np.arange(nyc) + dy) % ny
                for dx in (-1, 0, 1):
                    cols = (2 * np.arange(nxc) + dx) % nx
                    wt = w[dz] * w[dy] * w[dx]
                    out[:, kc] += wt * g[:, kf][:, rows][:, :, cols]
                    wsum += wt
        out[:, kc] /= wsum
    return out.reshape(k, -1)


def inject(f, nx, ny, nz):
    """Values of a fine field at the coarse nodes."""
    f = np.asarray(f)
    lead = f.shape[:-1]
    g = f.reshape(lead + (nz, ny, nx))[..., ::2, ::2, ::2]
    return np.ascontiguousarray(g).reshape(lead + (-1,))


def coarse_atmosphere(atm):
    """The model of the next coarser grid: every second node along each axis."""
    nxc, nyc, nzc = coarse_shape(atm.nx, atm.ny, atm.nz)
    ij = lambda a: None if a is None else inject(a, atm.nx, atm.ny, atm.nz)
    return dataclasses.replace(
        atm, nx=nxc, ny=nyc, nz=nzc, z=np.asarray(atm.z)[::2].copy(), kappa=ij(atm.kappa),
        propmat=ij(atm.propmat), emis=ij(atm.emis), source=ij(atm.source), hanle=ij(atm.hanle),
        bhat=ij(atm.bhat))


# ----------------------------------------------------------------- one grid level
class Level:
    """Model, quadrature and interpolation of one grid."""

    def __init__(self, atm, quad, interp=0):
        self.atm, self.quad, self.interp = atm, quad, interp

    @property
    def shape(self):
        return self.atm.nx, self.atm.ny, self.atm.nz

    def planck_rhs(self):
        """f of the problem itself: (eps_c B, 0, 0, 0, 0, 0) at every point."""
        f = np.zeros((6, self.atm.npoints))
        f[0] = self.atm.eps_c * self.atm.planck
        return f

    def radiation(self, S):
        """J^K_Q and Lambda-bar of a formal solution with emissivity kappa S."""
        kap = np.asarray(self.atm.kappa, dtype=np.float64)
        a = dataclasses.replace(self.atm, emis=kap[None, :] * S)
        return orc.fs_sweep(orc.OracleProblem(a, self.quad, interp=self.interp),
                            want_itop=False)["jkq"]

    def jacobi(self, S, f):
        """One Jacobi iteration for L(rho) rho = f; returns (S_new, R_c)."""
        s_new, _, rc = orc.see_update(self.radiation(S), S, self.atm, rhs=f)
        return s_new, rc

    def residual(self, S, f):
        """r = f - L(rho) rho (Eq. resid)."""
        return f - orc.see_operator(self.radiation(S), S, self.atm)


def make_levels(atm, quad, nlevels, interp=0):
    """Finest first."""
    levels = [Level(atm, quad, interp)]
    for _ in range(nlevels - 1):
        levels.append(Level(coarse_atmosphere(levels[-1].atm), quad, interp))
    return levels


def vcycle(levels, S, f, l=0, nu1=2, nu2=4, ncoarse=20, order=1):
    """One V-cycle of the FAS scheme of Sect. 5.1 on levels[l:] (levels[0] finest):
    nu1 Jacobi smoothing iterations, the residual, restriction of rho and of the
    residual, the coarse-grid equation L_c(rho_c) rho_c = L_c(R rho) R rho + R r
    (Eq. mgcsfy) solved by the next V-cycle (Jacobi iterations on the coarsest grid),
    the coarse-grid correction rho += P(rho_c - R rho), and nu2 smoothing iterations."""
    lev = levels[l]
    if l == len(levels) - 1:
        for _ in range(ncoarse):
            S, _ = lev.jacobi(S, f)
        return S
    for _ in range(nu1):
        S, _ = lev.jacobi(S, f)
    r = lev.residual(S, f)
    nx, ny, nz = lev.shape
    coarse = levels[l + 1]
    Sc = restrict(S, nx, ny, nz)
    fc = orc.see_operator(coarse.radiation(Sc), Sc, coarse.atm) + restrict(r, nx, ny, nz)
    Sc_new = vcycle(levels, Sc.copy(), fc, l + 1, nu1, nu2, ncoarse, order)
    S = S + prolong(Sc_new - Sc, *coarse.shape, order=order)
    for _ in range(nu2):
        S, _ = lev.jacobi(S, f)
    return S


def nested(levels, S0, cycles=1, nu1=2, nu2=4, ncoarse=20, order=1):
    """Nested multigrid: solve on the coarsest grid (ncoarse Jacobi iterations from S0
    injected there), then on each finer grid start from the prolonged solution of the
    grid below and apply `cycles` V-cycles on it and the grids below it.  Returns the
    finest-grid S."""
    # the initial guess on every level: S0 sampled at its nodes
    guesses = [np.asarray(S0, dtype=np.float64)]
    for lev in levels[:-1]:
        guesses.append(inject(guesses[-1], *lev.shape))
    top = len(levels) - 1
    S = guesses[top]
    f = levels[top].planck_rhs()
    for _ in range(ncoarse):
        S, _ = levels[top].jacobi(S, f)
    for l in range(top - 1, -1, -1):
        S = prolong(S, *levels[l + 1].shape, order=order)
        f = levels[l].planck_rhs()
        for _ in range(cycles):
            S = vcycle(levels, S, f, l, nu1, nu2, ncoarse, order)
    return S


def relative_change(s_new, s_old):
    """R_c = max |dS00| / |S00| between two iterates."""
    return float(np.max(np.abs(s_new[0] - s_old[0]) / np.abs(s_new[0])))
