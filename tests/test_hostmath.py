"""The per-update arithmetic of the GPU kernels (porta_math.hpp, compiled for the
host) against the oracle and closed forms."""
import ctypes as C
import math
import os

import numpy as np
import pytest

from paper_1307_4217_amd import build as pbuild

_dp = C.POINTER(C.c_double)
_fp = C.POINTER(C.c_float)


@pytest.fixture(scope="module")
def hm():
    if not os.path.exists(pbuild.HOSTTEST_LIB):
        pbuild.build_hostmath()
    L = C.CDLL(pbuild.HOSTTEST_LIB)
    L.hm_coefficients_f32.argtypes = [C.c_float, _fp]
    L.hm_coefficients_f64.argtypes = [C.c_double, _dp]
    L.hm_besser_cm.argtypes = [C.c_double] * 4
    L.hm_besser_cm.restype = C.c_double
    L.hm_parabolic_cm.argtypes = [C.c_double] * 4
    L.hm_parabolic_cm.restype = C.c_double
    L.hm_parabolic_cm_grad.argtypes = [C.c_double] * 4 + [_dp]
    L.hm_parabolic_cm_grad.restype = C.c_double
    L.hm_bezier3_f64.argtypes = [C.c_double] * 4
    L.hm_bezier3_f64.restype = C.c_double
    L.hm_bezier3_f32.argtypes = [C.c_float] * 4
    L.hm_bezier3_f32.restype = C.c_float
    L.hm_bezier3_grad_f64.argtypes = [C.c_double] * 4 + [C.POINTER(C.c_double)]
    L.hm_bezier3_grad_f64.restype = C.c_double
    L.hm_solve_stokes_f64.argtypes = [_dp] * 4
    L.hm_solve_stokes_f32.argtypes = [_fp] * 4
    L.hm_kprime_apply.argtypes = [_dp] * 4
    L.hm_stokes_solve_scaled_f64.argtypes = [_dp, _dp, C.c_double, _dp, C.c_int, _dp]
    L.hm_stokes_solve_scaled_f32.argtypes = [_fp, _fp, C.c_float, _fp, C.c_int, _fp]
    L.hm_ray_consts.argtypes = [C.c_double] * 4 + [_dp]
    L.hm_hanle_solve.argtypes = [C.c_double] * 5 + [_dp, _dp]
    L.hm_solve_pivot5.argtypes = [_dp] * 3
    return L


def p(a):
    return a.ctypes.data_as(_dp if a.dtype == np.float64 else _fp)


def coef(hm, tau, f32=False):
    out = np.zeros(6, np.float32 if f32 else np.float64)
    (hm.hm_coefficients_f32 if f32 else hm.hm_coefficients_f64)(tau, p(out))
    return out.astype(np.float64)


def test_coefficients_f64_match_oracle(hm, orc):
    for tau in np.concatenate([np.logspace(-7, 2.5, 300), [0.1, 0.14, 0.18]]):
        np.testing.assert_allclose(coef(hm, tau), orc.coefficients(tau), rtol=3e-13, atol=0)


def test_coefficients_f32_accuracy(hm, orc):
    worst = 0.0
    for tau in np.logspace(-7, 2, 600):
        t32 = float(np.float32(tau))
        ref = orc.coefficients(t32)
        got = coef(hm, t32, f32=True)
        rel = np.abs(got[1:] / ref[1:] - 1)
        worst = max(worst, rel.max())
        assert got[0] == pytest.approx(ref[0], rel=1e-6, abs=1e-30)
    assert worst < 1.5e-6


def test_scaled_stokes_solve_matches_dense_solve(hm):
    """(1 + p K') x = b and its transpose through the per-node operator and the
    per-frequency scalars, against a dense solve, over p from 1e-6 to 1 and K' entries
    up to the dichroism and dispersion the synthetic models reach (and ten times more)."""
    rng = np.random.default_rng(12)
    worst32 = 0.0
    for trial in range(600):
        amp = 0.05 if trial < 300 else 0.5
        e, r = rng.uniform(-amp, amp, 3), rng.uniform(-amp, amp, 3)
        b = rng.normal(size=4)
        pp = 10.0 ** rng.uniform(-6, 0)
        K = np.array([[0, e[0], e[1], e[2]], [e[0], 0, r[2], -r[1]],
                      [e[1], -r[2], 0, r[0]], [e[2], r[1], -r[0], 0]])
        A = np.eye(4) + pp * K
        for sgn, M in ((1, A), (-1, A.T)):
            want = np.linalg.solve(M, b)
            x = np.zeros(4)
            hm.hm_stokes_solve_scaled_f64(p(e), p(r), pp, p(b), sgn, p(x))
            np.testing.assert_allclose(x, want, rtol=1e-13, atol=1e-14)
            e32, r32, b32 = e.astype(np.float32), r.astype(np.float32), b.astype(np.float32)
            x32 = np.zeros(4, np.float32)
            hm.hm_stokes_solve_scaled_f32(p(e32), p(r32), np.float32(pp), p(b32), sgn, p(x32))
            worst32 = max(worst32, np.abs(x32 - want).max() / np.abs(want).max())
    assert worst32 < 2e-6, worst32


def test_besser_matches_oracle(hm, orc):
    rng = np.random.default_rng(1)
    for _ in range(5000):
        y = rng.normal(size=3)
        if rng.uniform() < 0.5:
            y = np.sort(y) * rng.choice([-1, 1])
        hM, hP = np.exp(rng.uniform(-6, 4, 2))
        ref = orc.besser_cm(*y, hM, hP)
        got = hm.hm_besser_cm(*y, hM / hP)
        assert got == pytest.approx(ref, rel=1e-12, abs=1e-12)


def test_solve_stokes_matches_dense_solve(hm, orc):
    rng = np.random.default_rng(2)
    for _ in range(500):
        e = rng.uniform(-0.3, 0.3, 3)
        r = rng.uniform(-0.3, 0.3, 3)
        b = rng.normal(size=4)
        A = np.eye(4) + np.array([[0, e[0], e[1], e[2]], [e[0], 0, r[2], -r[1]],
                                  [e[1], -r[2], 0, r[0]], [e[2], r[1], -r[0], 0]])
        x = np.zeros(4)
        hm.hm_solve_stokes_f64(p(e), p(r), p(b), p(x))
        np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-12, atol=1e-13)
        np.testing.assert_allclose(x, orc.solve4(A, b), rtol=1e-12, atol=1e-13)
        y = np.zeros(4)
        hm.hm_kprime_apply(p(e), p(r), p(x), p(y))
        np.testing.assert_allclose(y, (A - np.eye(4)) @ x, rtol=1e-13, atol=1e-14)
        x32 = np.zeros(4, np.float32)
        hm.hm_solve_stokes_f32(p(e.astype(np.float32)), p(r.astype(np.float32)),
                               p(b.astype(np.float32)), p(x32))
        np.testing.assert_allclose(x32, x, rtol=2e-5, atol=2e-6)


def test_ray_tables_match_oracle_tensors(hm, orc):
    rng = np.random.default_rng(3)
    for _ in range(40):
        mu, chi, w2 = rng.uniform(-1, 1), rng.uniform(0, 2 * math.pi), rng.uniform(0.3, 1.0)
        out = np.zeros(24 + 36 + 4)
        hm.hm_ray_consts(mu, chi, 0.1, w2, p(out))
        emis = out[:24].reshape(4, 6)
        proj = out[24:60].reshape(9, 4)
        e6 = rng.normal(size=6)
        np.testing.assert_allclose(emis @ e6, orc.emission(mu, chi, e6, w2), rtol=1e-13,
                                   atol=1e-14)
        t = orc.tkq(mu, chi)        # [4][9], slots K0; K1 Q-1..1; K2 Q-2..2
        ref = np.array([t[:, 0].real, t[:, 2].real, t[:, 3].real, t[:, 3].imag, t[:, 6].real,
                        t[:, 7].real, t[:, 7].imag, t[:, 8].real, t[:, 8].imag])
        np.testing.assert_allclose(proj, ref, atol=1e-15)
        st = math.sqrt(1 - mu * mu)
        np.testing.assert_allclose(out[60:], [mu, st * math.cos(chi), st * math.sin(chi), 0.1],
                                   rtol=1e-15, atol=1e-16)


def test_hanle_real_system_matches_complex_solve(hm):
    rng = np.random.default_rng(4)
    Jz = np.diag(np.arange(-2, 3)).astype(complex)
    Jp = np.zeros((5, 5), complex)
    for q in range(-2, 2):
        Jp[q + 3, q + 2] = math.sqrt(6 - q * (q + 1))
    Jm = Jp.conj().T
    for _ in range(200):
        a, h = 1 + rng.uniform(0, 1), rng.uniform(0, 10)
        b = rng.normal(size=3)
        b /= np.linalg.norm(b)
        K = b[0] * (Jp + Jm) / 2 + b[1] * (Jp - Jm) / 2j + b[2] * Jz
        R = np.zeros(5, complex)
        R[2] = rng.normal()
        R[3] = rng.normal() + 1j * rng.normal()
        R[4] = rng.normal() + 1j * rng.normal()
        R[1] = -np.conj(R[3])
        R[0] = np.conj(R[4])
        S = np.linalg.solve(a * np.eye(5) + 1j * h * K, R)
        rhs = np.array([R[2].real, R[3].real, R[3].imag, R[4].real, R[4].imag])
        x = np.zeros(5)
        hm.hm_hanle_solve(a, h, *b, p(rhs), p(x))
        np.testing.assert_allclose(x, [S[2].real, S[3].real, S[3].imag, S[4].real, S[4].imag],
                                   rtol=1e-11, atol=1e-13)


def test_besser_gradient_matches_finite_differences(hm):
    hm.hm_besser_cm_grad.argtypes = [C.c_double] * 4 + [_dp]
    hm.hm_besser_cm_grad.restype = C.c_double
    rng = np.random.default_rng(5)
    branches = set()
    for _ in range(3000):
        y = rng.normal(size=3)
        if rng.uniform() < 0.7:
            y = np.sort(y) * rng.choice([-1, 1])
        r = float(np.exp(rng.uniform(-3, 3)))
        d = np.zeros(4)
        c0 = hm.hm_besser_cm_grad(*y, r, p(d))
        assert c0 == hm.hm_besser_cm(*y, r)
        h = 1e-7
        args = list(y) + [r]
        fd = []
        ok = True
        for k in range(4):
            ap, am = list(args), list(args)
            ap[k] += h * max(1.0, abs(args[k]))
            am[k] -= h * max(1.0, abs(args[k]))
            cp_, cm_ = hm.hm_besser_cm(*ap), hm.hm_besser_cm(*am)
            dp_ = np.zeros(4)
            dm_ = np.zeros(4)
            hm.hm_besser_cm_grad(*ap, p(dp_))
            hm.hm_besser_cm_grad(*am, p(dm_))
            if not (np.allclose(dp_, d) and np.allclose(dm_, d)):
                ok = False     # a branch boundary lies within the step
                break
            fd.append((cp_ - cm_) / (ap[k] - am[k]))
        if ok:
            branches.add(tuple(np.round(d, 12) == 0))
            np.testing.assert_allclose(d, fd, rtol=1e-5, atol=1e-6)
    assert len(branches) >= 4


def test_coefficient_tau_derivatives(hm):
    hm.hm_coef_tau_grad_f64.argtypes = [C.c_double, _dp]
    hm.hm_coef_tau_grad_f64.restype = C.c_double
    hm.hm_coef_tau_grad_f32.argtypes = [C.c_float, _fp]
    hm.hm_coef_tau_grad_f32.restype = C.c_float
    for tau in np.logspace(-6, 2, 80):
        for k in range(6):
            g = np.zeros(6)
            g[k] = 1.0
            got = hm.hm_coef_tau_grad_f64(tau, p(g))
            h = 1e-5 * tau
            fd = (coef(hm, tau + h)[k] - coef(hm, tau - h)[k]) / (2 * h)
            # truncation ~ (h/tau)^2, rounding of the difference ~ ulp(value) / h
            assert got == pytest.approx(fd, rel=1e-6, abs=4e-16 / h), (tau, k)
            got32 = hm.hm_coef_tau_grad_f32(np.float32(tau), p(g.astype(np.float32)))
            assert got32 == pytest.approx(got, rel=2e-4, abs=1e-6), (tau, k)


def test_bezier3_closed_form_equals_branchy_besser(hm, orc):
    """The kernels' branch-free equidistant Bezier (weights in t, limited slope
    min(|d1|, |d2|, |d1 + d2|/4)) against the oracle's BESSER steps with ratio 1, on random
    triples, triples near each branch switch (d2 = 3 d1, d1 = 3 d2, a zero difference) and
    both halves of the interval."""
    rng = np.random.default_rng(11)
    cases = []
    for _ in range(4000):
        y0 = rng.standard_normal()
        d1, d2 = rng.standard_normal(2)
        kind = rng.integers(0, 6)
        if kind == 1:
            d2 = 3 * d1 * (1 + rng.choice([-1, 1]) * 1e-9)
        elif kind == 2:
            d1 = 3 * d2 * (1 + rng.choice([-1, 1]) * 1e-9)
        elif kind == 3:
            d2 = 0.0
        elif kind == 4:
            d1 = abs(d1) * np.sign(d2)   # monotone
        cases.append((y0 - d1, y0, y0 + d2, rng.uniform(-0.5, 0.5)))
    cases += [(0.0, 1.0, 2.0, 0.5), (2.0, 1.0, 0.0, -0.5), (1.0, 1.0, 1.0, 0.3), (0.0, 1.0, 0.0, 0.0)]
    scale = 1.0
    for ym, y0, yp, t in cases:
        ref = orc.bezier1d(ym, y0, yp, t)
        scale = max(abs(ym), abs(y0), abs(yp), 1.0)
        assert hm.hm_bezier3_f64(ym, y0, yp, t) == pytest.approx(ref, abs=4e-16 * scale)
        f = hm.hm_bezier3_f32(ym, y0, yp, t)
        assert f == pytest.approx(ref, abs=3e-6 * scale)


def test_bezier3_gradient_against_differences_and_oracle_branches(hm, orc):
    """The partials of the equidistant Bezier (the adjoint of the 9-point mode) against
    central differences of the oracle's BESSER-based evaluation, on random triples away
    from the branch switches, in both halves of the interval; the value is the
    interpolant itself; at an extremum or a zero difference the control point is y0 and
    only the weights of the quadratic remain."""
    rng = np.random.default_rng(12)
    g = (C.c_double * 3)()
    checked = 0
    for _ in range(3000):
        ym, y0, yp = rng.standard_normal(3)
        t = rng.uniform(-0.5, 0.5)
        d1, d2 = y0 - ym, yp - y0
        a = sorted([abs(d1), abs(d2), 0.25 * abs(d1 + d2)])
        if d1 * d2 > 0 and a[1] - a[0] < 1e-3:
            continue                              # next to a switch of the clamp
        if abs(d1) < 1e-3 or abs(d2) < 1e-3:
            continue
        v = hm.hm_bezier3_grad_f64(ym, y0, yp, t, g)
        assert v == pytest.approx(hm.hm_bezier3_f64(ym, y0, yp, t), abs=1e-15)
        h = 1e-6
        y = [ym, y0, yp]
        for k in range(3):
            yp_, ym_ = list(y), list(y)
            yp_[k] += h
            ym_[k] -= h
            fd = (orc.bezier1d(*yp_, t) - orc.bezier1d(*ym_, t)) / (2 * h)
            assert g[k] == pytest.approx(fd, abs=1e-8), (y, t, k)
        checked += 1
    assert checked > 1500
    for ym, y0, yp, t in [(0.0, 1.0, 0.0, 0.3), (1.0, 1.0, 2.0, -0.2), (2.0, 2.0, 2.0, 0.4)]:
        hm.hm_bezier3_grad_f64(ym, y0, yp, t, g)
        w = (t * t if t < 0 else 0.0, 1 - t * t, t * t if t >= 0 else 0.0)
        assert list(g) == pytest.approx(w, abs=1e-15)


def test_parabolic_control_point_matches_oracle_and_its_gradient(hm, orc):
    rng = np.random.default_rng(21)
    for _ in range(200):
        y = rng.normal(size=3)
        hM, hP = rng.uniform(0.05, 3.0, 2)
        r = hM / hP
        assert hm.hm_parabolic_cm(*y, r) == pytest.approx(orc.parabolic_cm(*y, hM, hP),
                                                          rel=1e-13, abs=1e-14)
        d = np.zeros(4)
        c = hm.hm_parabolic_cm_grad(*y, r, p(d))
        assert c == hm.hm_parabolic_cm(*y, r)
        args = [*y, r]
        for k in range(4):
            h = 1e-6 * max(1.0, abs(args[k]))
            up, dn = list(args), list(args)
            up[k] += h
            dn[k] -= h
            fd = (hm.hm_parabolic_cm(*up) - hm.hm_parabolic_cm(*dn)) / (2 * h)
            assert d[k] == pytest.approx(fd, rel=1e-6, abs=1e-8)


def test_pivoted_solve_needs_and_takes_row_swaps(hm):
    """The SEE's 5x5 elimination with partial pivoting (the pivot row swapped in by
    selects) against numpy on random systems whose rows are permuted so that the
    diagonal is zero or tiny: without the swaps the elimination would divide by it."""
    rng = np.random.default_rng(11)
    for trial in range(300):
        M = rng.normal(size=(5, 5)) + 5 * np.eye(5)
        A = np.ascontiguousarray(M[rng.permutation(5)])
        if trial % 3 == 0:
            A[0, 0] = 0.0
        elif trial % 3 == 1:
            A[np.arange(5), np.arange(5)] *= 1e-12
        b = rng.normal(size=5)
        x = np.zeros(5)
        hm.hm_solve_pivot5(p(A), p(b), p(x))
        np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-9, atol=1e-11)
