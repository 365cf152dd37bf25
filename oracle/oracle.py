"""ctypes wrapper of the FP64 CPU oracle (porta_oracle.cpp).

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this module.  The GPU library never calls it and
shares no code with it.  Inputs are plain NumPy arrays (x-fastest point
order); the oracle defines its own problem struct.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "porta_oracle.cpp")
# PORTA_ORACLE_LIB names another build of the same source (the sanitizer test uses it)
LIB = os.environ.get("PORTA_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")

_lock = threading.Lock()
_lib = None

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


class Problem(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("lx", C.c_double), ("ly", C.c_double), ("z", _dp),
                ("nmu", C.c_int), ("nchi", C.c_int), ("nfreq", C.c_int),
                ("mu", _dp), ("wmu", _dp), ("phi", _dp), ("wfreq", _dp),
                ("i_bottom", C.c_double), ("w2", C.c_double), ("interp", C.c_int),
                ("control", C.c_int), ("faces", C.c_int)]


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (IEEE double, no fast-math)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["g++", "-std=c++17", "-O3", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", SRC, "-o", tmp])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB):
                build()
            L = C.CDLL(LIB)
            L.oracle_fs_sweep.argtypes = [C.POINTER(Problem), _dp, _dp, _dp, C.c_int, _ip, C.c_int,
                                          _ip, _dp, _dp, _dp, _dp, C.c_int]
            L.oracle_fs_sweep_cs.argtypes = [C.POINTER(Problem), _dp, _dp, _dp, _dp, _dp, _dp,
                                             C.c_double, C.c_int, _ip, C.c_int, _ip, _dp, _dp,
                                             C.c_int]
            L.oracle_fs_adjoint.argtypes = [C.POINTER(Problem), _dp, _dp, _dp, C.c_int, _ip,
                                            C.c_int, _ip, _dp, _dp, _dp, _dp, C.c_int]
            L.oracle_lc_fine_sweep.argtypes = [C.POINTER(Problem), _dp, _dp, _dp, C.c_int, _ip,
                                               C.c_int, _ip, C.c_int, _dp, C.c_int]
            L.oracle_lc_sweep.argtypes = [C.POINTER(Problem), _dp, _dp, _dp, C.c_int, _ip,
                                          C.c_int, _ip, _dp]
            L.oracle_jkq_accumulate.argtypes = [C.POINTER(Problem), C.c_int, C.c_int, C.c_int,
                                                C.c_int, _dp, _dp, _dp]
            L.oracle_see_update.argtypes = [C.c_int, _dp, _dp, C.c_double, C.c_double,
                                            C.c_double, C.c_double, _dp, _dp, _dp, _dp, _dp,
                                            _dp, _dp]
            L.oracle_see_operator.argtypes = [C.c_int, _dp, _dp, C.c_double, C.c_double,
                                              C.c_double, _dp, _dp, _dp]
            L.oracle_coefficients.argtypes = [C.c_double, _dp]
            L.oracle_besser_cm.argtypes = [C.c_double] * 5
            L.oracle_besser_cm.restype = C.c_double
            L.oracle_parabolic_cm.argtypes = [C.c_double] * 5
            L.oracle_parabolic_cm.restype = C.c_double
            L.oracle_bezier1d.argtypes = [C.c_double] * 4
            L.oracle_bezier1d.restype = C.c_double
            L.oracle_interp_plane.argtypes = [_dp, C.c_int, C.c_int, C.c_double, C.c_double,
                                              C.c_int]
            L.oracle_interp_plane.restype = C.c_double
            L.oracle_tkq.argtypes = [C.c_double, C.c_double, _dp, _dp]
            L.oracle_emission.argtypes = [C.c_double, C.c_double, _dp, C.c_double, _dp]
            L.oracle_solve4.argtypes = [_dp, _dp, _dp]
            _lib = L
    return _lib


def _d(a):
    """Contiguous float64 array and its pointer (keeps the array alive via the caller)."""
    return a.ctypes.data_as(_dp)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


class OracleProblem:
    """Holds the NumPy arrays behind a Problem struct."""

    def __init__(self, atm, quad, interp: int = 0, i_bottom: float | None = None,
                 control: int = 0, faces: int = 0):
        self.nx, self.ny, self.nz = atm.nx, atm.ny, atm.nz
        self.N = atm.nx * atm.ny * atm.nz
        self.z = _f64(atm.z)
        self.mu = _f64(quad.mu)
        self.wmu = _f64(quad.wmu)
        self.phi = _f64(quad.phi)
        self.wfreq = _f64(quad.wfreq)
        self.nchi = int(quad.nchi)
        self.nfreq = len(self.phi)
        self.nrays = 2 * len(self.mu) * self.nchi
        self.kappa = _f64(atm.kappa)
        self.prop = _f64(atm.propmat)
        self.emis = _f64(atm.emis)
        self.struct = Problem(self.nx, self.ny, self.nz, float(atm.lx), float(atm.ly),
                              _d(self.z), len(self.mu), self.nchi, self.nfreq, _d(self.mu),
                              _d(self.wmu), _d(self.phi), _d(self.wfreq),
                              float(atm.i_bottom if i_bottom is None else i_bottom),
                              float(atm.w2), int(interp), int(control), int(faces))

    def with_fields(self, kappa=None, prop=None, emis=None):
        """Shallow copy with replaced material arrays."""
        o = object.__new__(OracleProblem)
        o.__dict__.update(self.__dict__)
        if kappa is not None:
            o.kappa = _f64(kappa)
        if prop is not None:
            o.prop = _f64(prop)
        if emis is not None:
            o.emis = _f64(emis)
        return o


def fs_sweep(op: OracleProblem, rays=None, freqs=None, want_j=True, want_itop=True,
             want_full=False, want_lambda=False, nthreads: int = 0):
    """Formal solution of the selected (ray, frequency) pairs.

    Returns a dict with 'jkq' [10][N], 'itop' [nr][nf][ny][nx][4], 'ifull'
    [nr][nf][N][4] and 'lam' [nr][nf][N] as requested."""
    L = lib()
    rays = np.arange(op.nrays, dtype=np.int32) if rays is None else np.asarray(rays, np.int32)
    freqs = np.arange(op.nfreq, dtype=np.int32) if freqs is None else np.asarray(freqs, np.int32)
    nr, nf = len(rays), len(freqs)
    np_ = op.nx * op.ny
    out = {}
    jkq = np.zeros((10, op.N)) if want_j else None
    itop = np.zeros((nr, nf, op.ny, op.nx, 4)) if want_itop else None
    ifull = np.zeros((nr, nf, op.N, 4)) if want_full else None
    lam = np.zeros((nr, nf, op.N)) if want_lambda else None
    nul = C.cast(None, _dp)
    rc = L.oracle_fs_sweep(C.byref(op.struct), _d(op.kappa), _d(op.prop), _d(op.emis), nr,
                           rays.ctypes.data_as(_ip), nf, freqs.ctypes.data_as(_ip),
                           _d(jkq) if jkq is not None else nul,
                           _d(itop) if itop is not None else nul,
                           _d(ifull) if ifull is not None else nul,
                           _d(lam) if lam is not None else nul, int(nthreads))
    if rc != 0:
        raise ValueError("oracle_fs_sweep rejected its inputs")
    del np_
    if want_j:
        out["jkq"] = jkq
    if want_itop:
        out["itop"] = itop
    if want_full:
        out["ifull"] = ifull
    if want_lambda:
        out["lam"] = lam
    return out


def fs_sweep_cs(op: OracleProblem, dkappa, dprop, demis, h=1e-30, rays=None, freqs=None,
                nthreads: int = 0):
    """Complex-step emergent Stokes: returns (real, imag) of I_top, [nr][nf][ny][nx][4]."""
    L = lib()
    rays = np.arange(op.nrays // 2, dtype=np.int32) if rays is None else np.asarray(rays, np.int32)
    freqs = np.arange(op.nfreq, dtype=np.int32) if freqs is None else np.asarray(freqs, np.int32)
    nr, nf = len(rays), len(freqs)
    dk, dp_, de = _f64(dkappa), _f64(dprop), _f64(demis)
    re = np.zeros((nr, nf, op.ny, op.nx, 4))
    im = np.zeros_like(re)
    rc = L.oracle_fs_sweep_cs(C.byref(op.struct), _d(op.kappa), _d(op.prop), _d(op.emis),
                              _d(dk), _d(dp_), _d(de), float(h), nr, rays.ctypes.data_as(_ip),
                              nf, freqs.ctypes.data_as(_ip), _d(re), _d(im), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_fs_sweep_cs rejected its inputs")
    return re, im


def fs_adjoint(op: OracleProblem, seed, rays=None, freqs=None, nthreads: int = 0):
    """Reverse-mode gradient of L = sum(seed * I_top) over the selected upward rays and
    frequencies; seed [nr][nf][ny][nx][4].  Returns (g_kappa [N], g_prop [6][N],
    g_emis [6][N])."""
    L = lib()
    rays = np.arange(op.nrays // 2, dtype=np.int32) if rays is None else np.asarray(rays, np.int32)
    freqs = np.arange(op.nfreq, dtype=np.int32) if freqs is None else np.asarray(freqs, np.int32)
    seed = _f64(seed)
    if seed.shape != (len(rays), len(freqs), op.ny, op.nx, 4):
        raise ValueError(f"seed shape {seed.shape} does not match the selection")
    gk, gp, ge = np.zeros(op.N), np.zeros((6, op.N)), np.zeros((6, op.N))
    rc = L.oracle_fs_adjoint(C.byref(op.struct), _d(op.kappa), _d(op.prop), _d(op.emis),
                             len(rays), rays.ctypes.data_as(_ip), len(freqs),
                             freqs.ctypes.data_as(_ip), _d(seed), _d(gk), _d(gp), _d(ge),
                             int(nthreads))
    if rc != 0:
        raise ValueError("oracle_fs_adjoint rejected its inputs")
    return gk, gp, ge


def lc_sweep(op: OracleProblem, rays, freqs):
    """Long-characteristics Stokes vectors at every point, [nr][nf][N][4]."""
    L = lib()
    rays = np.asarray(rays, np.int32)
    freqs = np.asarray(freqs, np.int32)
    out = np.zeros((len(rays), len(freqs), op.N, 4))
    rc = L.oracle_lc_sweep(C.byref(op.struct), _d(op.kappa), _d(op.prop), _d(op.emis),
                           len(rays), rays.ctypes.data_as(_ip), len(freqs),
                           freqs.ctypes.data_as(_ip), _d(out))
    if rc != 0:
        raise ValueError("oracle_lc_sweep rejected its inputs")
    return out


def lc_fine_sweep(op: OracleProblem, rays, freqs, nsub=1, nthreads: int = 0):
    """Long characteristics through the trilinear medium, cut at every face crossing and
    each piece in nsub parts: Stokes vectors at every point, [nr][nf][N][4]."""
    L = lib()
    rays = np.asarray(rays, np.int32)
    freqs = np.asarray(freqs, np.int32)
    out = np.zeros((len(rays), len(freqs), op.N, 4))
    rc = L.oracle_lc_fine_sweep(C.byref(op.struct), _d(op.kappa), _d(op.prop), _d(op.emis),
                                len(rays), rays.ctypes.data_as(_ip), len(freqs),
                                freqs.ctypes.data_as(_ip), int(nsub), _d(out), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_lc_fine_sweep rejected its inputs")
    return out


def jkq_accumulate(op: OracleProblem, ray0, f0, stokes, lam=None, jkq=None):
    """Eq. 1 from a stored block stokes [nray][nf][N][4] (and lam [nray][nf][N])."""
    L = lib()
    stokes = _f64(stokes)
    nray, nf = stokes.shape[0], stokes.shape[1]
    jkq = np.zeros((10, op.N)) if jkq is None else jkq
    lam = _f64(lam)
    rc = L.oracle_jkq_accumulate(C.byref(op.struct), int(ray0), nray, int(f0), nf, _d(stokes),
                                 _d(lam) if lam is not None else C.cast(None, _dp), _d(jkq))
    if rc != 0:
        raise ValueError("oracle_jkq_accumulate rejected its inputs")
    return jkq


def see_update(jkq, s_old, atm, kappa=None, rhs=None):
    """One Jacobi update of the two-level SEE; returns (s_new, emis_new, rc).
    rhs [6][N] replaces the right-hand side (eps B, 0, ...) when given."""
    L = lib()
    jkq = _f64(jkq)
    s_old = _f64(s_old)
    n = s_old.shape[1]
    s_new = np.zeros((6, n))
    emis_new = np.zeros((6, n))
    kap = _f64(atm.kappa if kappa is None else kappa)
    hanle = _f64(atm.hanle)
    bhat = _f64(atm.bhat)
    rhs = _f64(rhs)
    rc = C.c_double(0.0)
    nul = C.cast(None, _dp)
    opt = lambda a: _d(a) if a is not None else nul
    st = L.oracle_see_update(n, _d(jkq), _d(s_old), float(atm.eps_c), float(atm.delta2),
                             float(atm.w2), float(atm.planck), opt(hanle), opt(bhat), opt(rhs),
                             _d(kap), _d(s_new), _d(emis_new), C.byref(rc))
    if st != 0:
        raise ValueError("oracle_see_update rejected its inputs")
    return s_new, emis_new, rc.value


def see_operator(jkq, s, atm):
    """L(rho) rho of the two-level SEE (left-hand side of Eq. nonlte), [6][N]."""
    L = lib()
    jkq = _f64(jkq)
    s = _f64(s)
    out = np.zeros_like(s)
    hanle = _f64(atm.hanle)
    bhat = _f64(atm.bhat)
    nul = C.cast(None, _dp)
    st = L.oracle_see_operator(s.shape[1], _d(jkq), _d(s), float(atm.eps_c), float(atm.delta2),
                               float(atm.w2), _d(hanle) if hanle is not None else nul,
                               _d(bhat) if bhat is not None else nul, _d(out))
    if st != 0:
        raise ValueError("oracle_see_operator rejected its inputs")
    return out


def coefficients(tau: float) -> np.ndarray:
    """(e^-tau, psi'_M, psi'_O, omega_M, omega_O, omega_C)."""
    out = np.zeros(6)
    lib().oracle_coefficients(float(tau), _d(out))
    return out


def besser_cm(yM, yO, yP, hM, hP) -> float:
    return lib().oracle_besser_cm(float(yM), float(yO), float(yP), float(hM), float(hP))


def parabolic_cm(yM, yO, yP, hM, hP) -> float:
    return lib().oracle_parabolic_cm(float(yM), float(yO), float(yP), float(hM), float(hP))


def bezier1d(ym, y0, yp, t) -> float:
    return lib().oracle_bezier1d(float(ym), float(y0), float(yp), float(t))


def interp_plane(f2d, fx, fy, mode=0) -> float:
    f = _f64(f2d)
    ny, nx = f.shape
    return lib().oracle_interp_plane(_d(f), nx, ny, float(fx), float(fy), int(mode))


def tkq(mu, chi) -> np.ndarray:
    """Complex T^K_Q(i, Omega), shape [4][9] (slots K=0; K=1 Q=-1..1; K=2 Q=-2..2)."""
    re = np.zeros(36)
    im = np.zeros(36)
    lib().oracle_tkq(float(mu), float(chi), _d(re), _d(im))
    return (re + 1j * im).reshape(4, 9)


def emission(mu, chi, e6, w2=1.0) -> np.ndarray:
    e = _f64(e6)
    out = np.zeros(4)
    lib().oracle_emission(float(mu), float(chi), _d(e), float(w2), _d(out))
    return out


def solve4(A, b) -> np.ndarray:
    A = _f64(A)
    b = _f64(b)
    x = np.zeros(4)
    lib().oracle_solve4(_d(A), _d(b), _d(x))
    return x


def ray_table(op: OracleProblem):
    """(mu, chi, weight) of every ray in the oracle's enumeration order."""
    nh = len(op.mu) * op.nchi
    out = []
    for r in range(op.nrays):
        a = (r % nh) // op.nchi
        m = r % op.nchi
        mu = op.mu[a] if r < nh else -op.mu[a]
        out.append((mu, (m + 0.5) * 2 * np.pi / op.nchi, 0.5 * op.wmu[a] / op.nchi))
    return out
