"""Thin ctypes binding of the C ABI in include/porta.h.

Only argument marshalling happens here: every step of the computation runs in
the HIP kernels of libporta.so.  PyTorch provides device memory and the
current stream.  Loading fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libporta.so")

F64, F32 = 0, 1
BILINEAR, BEZIER2D = 0, 1
CONTROL_BESSER, CONTROL_PARABOLIC = 0, 1
WS_SWEEP, WS_ADJOINT, WS_JKQ, WS_SEE, WS_ADJOINT_CKPT = 0, 1, 2, 3, 4

_dp = C.POINTER(C.c_double)


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("lx", C.c_double), ("ly", C.c_double), ("z", _dp)]


class Quad(C.Structure):
    _fields_ = [("nmu", C.c_int32), ("nchi", C.c_int32), ("nfreq", C.c_int32),
                ("mu", _dp), ("wmu", _dp), ("phi", _dp), ("wfreq", _dp)]


class Fields(C.Structure):
    _fields_ = [("kappa", C.c_void_p), ("propmat", C.c_void_p), ("emis", C.c_void_p),
                ("i_bottom", C.c_double), ("w2", C.c_double)]


class Atom(C.Structure):
    _fields_ = [("eps_c", C.c_double), ("delta2", C.c_double), ("w2", C.c_double),
                ("planck", C.c_double), ("hanle", C.c_void_p), ("bhat", C.c_void_p)]


class Options(C.Structure):
    _fields_ = [("ray_batch", C.c_int32), ("block", C.c_int32), ("xcd_remap", C.c_int32),
                ("control", C.c_int32), ("stokes", C.c_int32), ("ray_first", C.c_int32),
                ("ray_count", C.c_int32), ("check_inputs", C.c_int32),
                ("faces", C.c_int32), ("faces_chunk", C.c_int32)]


OK, EINVAL, EUNSUPPORTED, ENOMEM, EDEVICE, ENONFINITE = 0, -1, -2, -3, -4, -5


class PortaError(RuntimeError):
    def __init__(self, fn, status, msg):
        super().__init__(f"{fn} failed with status {status}: {msg}")
        self.status = status


_lock = threading.Lock()
_lib = None


def lib():
    """Load libporta.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError(f"{LIB_PATH} is missing: build it with "
                                  "`python -c 'import __graft_entry__ as g; g.build()'`")
            L = C.CDLL(LIB_PATH)
            vp, sz = C.c_void_p, C.c_size_t
            L.porta_workspace_size.argtypes = [C.POINTER(Grid), C.POINTER(Quad), C.c_int, C.c_int,
                                               C.c_int, C.POINTER(Options)]
            L.porta_workspace_size.restype = sz
            L.porta_fs_sweep.argtypes = [C.POINTER(Grid), C.POINTER(Quad), C.POINTER(Fields),
                                         C.c_int, C.c_int, C.POINTER(Options), vp, C.c_int, vp,
                                         vp, sz, C.c_int, vp, sz, vp]
            L.porta_fs_sweep_noalloc.argtypes = [C.POINTER(Grid), C.POINTER(Quad),
                                                 C.POINTER(Fields), C.c_int, C.c_int,
                                                 C.POINTER(Options), vp, C.c_int, vp, vp]
            L.porta_checkpoint_size.argtypes = [C.POINTER(Grid), C.POINTER(Quad), C.c_int,
                                                C.c_int, C.POINTER(Options)]
            L.porta_checkpoint_size.restype = sz
            L.porta_jkq_accumulate.argtypes = [C.POINTER(Grid), C.POINTER(Quad), C.c_int, C.c_int,
                                               C.c_int, C.c_int, vp, vp, C.c_int, vp, vp, sz, vp]
            L.porta_see_update.argtypes = [C.c_int64, vp, C.POINTER(Atom), vp, vp, vp, vp, vp,
                                           C.c_int, vp, vp, sz, vp]
            L.porta_see_operator.argtypes = [C.c_int64, vp, C.POINTER(Atom), vp, vp, C.c_double,
                                             vp, vp]
            ci = C.c_int
            L.porta_mg_restrict.argtypes = [ci, ci, ci, ci, vp, vp, vp, vp, ci, vp]
            L.porta_mg_prolong.argtypes = [ci, ci, ci, ci, ci, vp, vp, vp, vp, vp, ci, vp]
            L.porta_mg_inject.argtypes = [ci, ci, ci, ci, ci, vp, vp, vp]
            L.porta_rel_change.argtypes = [C.c_int64, vp, vp, vp, vp, sz, vp]
            L.porta_emissivity.argtypes = [C.c_int64, ci, vp, vp, vp, ci, vp]
            L.porta_fs_adjoint.argtypes = [C.POINTER(Grid), C.POINTER(Quad), C.POINTER(Fields),
                                           C.c_int, C.c_int, C.POINTER(Options), vp, vp, sz,
                                           C.c_int, vp, vp, vp, vp, sz, vp]
            L.porta_strerror.argtypes = [C.c_int]
            L.porta_strerror.restype = C.c_char_p
            L.porta_last_error.restype = C.c_char_p
            L.porta_version.restype = C.c_char_p
            _lib = L
    return _lib


EXPORTED = ("porta_workspace_size", "porta_checkpoint_size", "porta_fs_sweep",
            "porta_fs_sweep_noalloc",
            "porta_jkq_accumulate", "porta_see_update", "porta_see_operator",
            "porta_mg_restrict", "porta_mg_prolong", "porta_mg_inject", "porta_rel_change",
            "porta_emissivity",
            "porta_fs_adjoint", "porta_strerror", "porta_last_error", "porta_version")


def _check(fn, status):
    if status != 0:
        L = lib()
        raise PortaError(fn, status, f"{L.porta_strerror(status).decode()}: "
                                     f"{L.porta_last_error().decode()}")


def _ptr(t):
    """Device (or host) address of a tensor/array, None for None."""
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


def _nbytes(t):
    """Size in bytes of a tensor/array (0 for None)."""
    if t is None:
        return 0
    if isinstance(t, np.ndarray):
        return int(t.nbytes)
    return int(t.numel()) * int(t.element_size())


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


class HostGrid:
    """Host-side grid/quadrature structs with the arrays they point to."""

    def __init__(self, nx, ny, nz, lx, ly, z, mu, wmu, nchi, phi, wfreq):
        self._z = np.ascontiguousarray(z, np.float64)
        self._mu = np.ascontiguousarray(mu, np.float64)
        self._wmu = np.ascontiguousarray(wmu, np.float64)
        self._phi = np.ascontiguousarray(phi, np.float64)
        self._wfreq = np.ascontiguousarray(wfreq, np.float64)
        self.grid = Grid(int(nx), int(ny), int(nz), float(lx), float(ly),
                         self._z.ctypes.data_as(_dp))
        self.quad = Quad(len(self._mu), int(nchi), len(self._phi), self._mu.ctypes.data_as(_dp),
                         self._wmu.ctypes.data_as(_dp), self._phi.ctypes.data_as(_dp),
                         self._wfreq.ctypes.data_as(_dp))
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.N = self.nx * self.ny * self.nz
        self.nmu, self.nchi, self.nfreq = len(self._mu), int(nchi), len(self._phi)
        self.nrays = 2 * self.nmu * self.nchi
        self.nray_up = self.nmu * self.nchi

    @classmethod
    def from_inputs(cls, atm, quad):
        return cls(atm.nx, atm.ny, atm.nz, atm.lx, atm.ly, atm.z, quad.mu, quad.wmu, quad.nchi,
                   quad.phi, quad.wfreq)


def options(ray_batch=0, block=0, xcd_remap=-1, control=0, stokes=4, ray_first=0,
            ray_count=0, check_inputs=False, faces=0, faces_chunk=0):
    """porta_options; control = CONTROL_BESSER or CONTROL_PARABOLIC; stokes = 4 (Stokes
    vector) or 1 (intensity only, the unpolarized problem); rays [ray_first,
    ray_first + ray_count) of the enumeration (ray_count 0: every ray); check_inputs: the
    sweep and the adjoint first check that the coefficients are finite and eta_I > 0
    (waits on the stream; PORTA_ENONFINITE otherwise); faces = 1: M and P on the first
    face of the grid the ray crosses (0: on the neighbouring horizontal planes), with
    faces_chunk frequencies per block of its kernel (0: 4 in FP32, 7 in FP64, fewer if
    the LDS of a block holds fewer)."""
    return Options(int(ray_batch), int(block), int(xcd_remap), int(control), int(stokes),
                   int(ray_first), int(ray_count), int(bool(check_inputs)), int(faces),
                   int(faces_chunk))


def workspace_size(hg: HostGrid, prec, kind, checkpoint_stride=1, opts=None) -> int:
    n = lib().porta_workspace_size(C.byref(hg.grid), C.byref(hg.quad), int(prec), int(kind),
                                   int(checkpoint_stride), C.byref(opts) if opts else None)
    if n == 0:
        raise PortaError("porta_workspace_size", -1, lib().porta_last_error().decode())
    return int(n)


def checkpoint_size(hg: HostGrid, prec, checkpoint_stride, opts=None) -> int:
    """Bytes of the checkpoint buffer for the upward rays of the options' ray range (0 also
    when no plane is a checkpoint; an invalid stride is reported by fs_sweep /
    fs_adjoint)."""
    return int(lib().porta_checkpoint_size(C.byref(hg.grid), C.byref(hg.quad), int(prec),
                                           int(checkpoint_stride),
                                           C.byref(opts) if opts else None))


def _workspace(nbytes, device):
    import torch
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def dtype_of(prec):
    import torch
    return torch.float64 if prec == F64 else torch.float32


def fs_sweep(hg: HostGrid, kappa, propmat, emis, i_bottom, w2=1.0, prec=F64, interp=BILINEAR,
             jkq=None, accumulate=False, i_top=None, want_jkq=True, want_itop=True,
             opts=None, workspace=None, stream=None, checkpoints=None, checkpoint_stride=0):
    """porta_fs_sweep.  Returns (jkq [10][N] float64, i_top [nray_up][nfreq][ny][nx][4]).
    With `checkpoints` (a device buffer of checkpoint_size() bytes) the states of the
    upward rays every `checkpoint_stride` planes are kept for fs_adjoint."""
    import torch
    dev = kappa.device
    if want_jkq and jkq is None:
        jkq = torch.empty((10, hg.N), dtype=torch.float64, device=dev)
    if want_itop and i_top is None:
        shape = (hg.nray_up, hg.nfreq, hg.ny, hg.nx)
        if not (opts is not None and opts.stokes == 1):
            shape += (4,)
        i_top = torch.empty(shape, dtype=dtype_of(prec), device=dev)
    if workspace is None:
        workspace = _workspace(workspace_size(hg, prec, WS_SWEEP, 1, opts), dev)
    f = Fields(_ptr(kappa), _ptr(propmat), _ptr(emis), float(i_bottom), float(w2))
    st = lib().porta_fs_sweep(C.byref(hg.grid), C.byref(hg.quad), C.byref(f), int(prec),
                              int(interp), C.byref(opts) if opts else None,
                              _ptr(jkq) if want_jkq else None, int(bool(accumulate)),
                              _ptr(i_top) if want_itop else None, _ptr(checkpoints),
                              _nbytes(checkpoints), int(checkpoint_stride), _ptr(workspace), workspace.numel(),
                              _stream(stream))
    _check("porta_fs_sweep", st)
    return (jkq if want_jkq else None), (i_top if want_itop else None)


def fs_sweep_noalloc(hg: HostGrid, kappa, propmat, emis, i_bottom, jkq, i_top, w2=1.0,
                     prec=F64, interp=BILINEAR, accumulate=False, opts=None, stream=None):
    """porta_fs_sweep_noalloc: fs_sweep with the library's static device scratch as its
    workspace.  The caller passes the outputs (jkq [10][N] float64 or None, i_top or
    None); nothing is allocated.  Returns (jkq, i_top)."""
    f = Fields(_ptr(kappa), _ptr(propmat), _ptr(emis), float(i_bottom), float(w2))
    st = lib().porta_fs_sweep_noalloc(C.byref(hg.grid), C.byref(hg.quad), C.byref(f),
                                      int(prec), int(interp), C.byref(opts) if opts else None,
                                      _ptr(jkq), int(bool(accumulate)), _ptr(i_top),
                                      _stream(stream))
    _check("porta_fs_sweep_noalloc", st)
    return jkq, i_top


def jkq_accumulate(hg: HostGrid, ray0, f0, stokes, lambda_star=None, jkq=None, prec=F64,
                   workspace=None, stream=None):
    """porta_jkq_accumulate for stokes [nray][nf][N][4]."""
    import torch
    dev = stokes.device
    if jkq is None:
        jkq = torch.zeros((10, hg.N), dtype=torch.float64, device=dev)
    if workspace is None:
        workspace = _workspace(workspace_size(hg, prec, WS_JKQ), dev)
    nray, nf = stokes.shape[0], stokes.shape[1]
    st = lib().porta_jkq_accumulate(C.byref(hg.grid), C.byref(hg.quad), int(ray0), int(nray),
                                    int(f0), int(nf), _ptr(stokes), _ptr(lambda_star), int(prec),
                                    _ptr(jkq), _ptr(workspace), workspace.numel(),
                                    _stream(stream))
    _check("porta_jkq_accumulate", st)
    return jkq


def see_update(jkq, s_old, eps_c, delta2, w2, planck, hanle=None, bhat=None, kappa=None,
               emis_out=None, prec=F64, want_rc=True, s_new=None, rc=None, workspace=None,
               stream=None, rhs=None):
    """porta_see_update.  Returns (s_new [6][N], emis_out or None, rc device scalar or None).
    rhs [6][N] FP64 replaces the right-hand side (eps_c B, 0, ...) when given."""
    import torch
    dev = jkq.device
    n = s_old.shape[1]
    if s_new is None:
        s_new = torch.empty_like(s_old)
    if want_rc and rc is None:
        rc = torch.empty((), dtype=torch.float64, device=dev)
    if workspace is None:
        workspace = _workspace(8 * ((n + 255) // 256), dev)
    atom = Atom(float(eps_c), float(delta2), float(w2), float(planck), _ptr(hanle), _ptr(bhat))
    st = lib().porta_see_update(int(n), _ptr(jkq), C.byref(atom), _ptr(rhs), _ptr(s_old),
                                _ptr(s_new), _ptr(kappa), _ptr(emis_out), int(prec),
                                _ptr(rc) if want_rc else None, _ptr(workspace),
                                workspace.numel(), _stream(stream))
    _check("porta_see_update", st)
    return s_new, emis_out, (rc if want_rc else None)


def see_operator(jkq, s, eps_c, delta2, w2, planck, hanle=None, bhat=None, base=None,
                 sign=1.0, out=None, stream=None):
    """porta_see_operator: out = base + sign * L(rho) rho (base None: (eps_c B, 0, ...))."""
    import torch
    if out is None:
        out = torch.empty_like(s)
    atom = Atom(float(eps_c), float(delta2), float(w2), float(planck), _ptr(hanle), _ptr(bhat))
    st = lib().porta_see_operator(int(s.shape[1]), _ptr(jkq), C.byref(atom), _ptr(s),
                                  _ptr(base), float(sign), _ptr(out), _stream(stream))
    _check("porta_see_operator", st)
    return out


def coarse_dims(nx, ny, nz):
    return nx // 2, ny // 2, (nz + 1) // 2


def mg_restrict(fine, nx, ny, nz, out=None, kappa_c=None, emis_c=None, prec=F64, stream=None):
    """porta_mg_restrict of a [k][nx*ny*nz] FP64 field; returns the coarse [k][Nc]."""
    import torch
    k = fine.shape[0]
    nxc, nyc, nzc = coarse_dims(nx, ny, nz)
    if out is None:
        out = torch.empty((k, nxc * nyc * nzc), dtype=torch.float64, device=fine.device)
    st = lib().porta_mg_restrict(int(nx), int(ny), int(nz), int(k), _ptr(fine), _ptr(out),
                                 _ptr(kappa_c), _ptr(emis_c), int(prec), _stream(stream))
    _check("porta_mg_restrict", st)
    return out


def mg_prolong(fine, nx, ny, nz, coarse_a, coarse_b=None, kappa=None, emis=None, prec=F64,
               stream=None, order=1):
    """porta_mg_prolong: fine += P(coarse_a - coarse_b), in place (order 1 tri-linear,
    3 tri-cubic-centred); returns fine."""
    st = lib().porta_mg_prolong(int(nx), int(ny), int(nz), int(fine.shape[0]), int(order),
                                _ptr(coarse_a),
                                _ptr(coarse_b), _ptr(fine), _ptr(kappa), _ptr(emis), int(prec),
                                _stream(stream))
    _check("porta_mg_prolong", st)
    return fine


def mg_inject(fine, nx, ny, nz, stream=None):
    """porta_mg_inject of a [k][N] (or [N]) float32/float64 tensor."""
    import torch
    shape = fine.shape
    f2 = fine.reshape(-1, shape[-1])
    nxc, nyc, nzc = coarse_dims(nx, ny, nz)
    out = torch.empty((f2.shape[0], nxc * nyc * nzc), dtype=fine.dtype, device=fine.device)
    st = lib().porta_mg_inject(int(nx), int(ny), int(nz), int(f2.shape[0]),
                               int(fine.element_size()), _ptr(f2), _ptr(out), _stream(stream))
    _check("porta_mg_inject", st)
    return out.reshape(shape[:-1] + (out.shape[-1],))


def emissivity(kappa, s, emis=None, stream=None):
    """porta_emissivity: emis = kappa * s ([k][N], dtype of kappa)."""
    import torch
    if emis is None:
        emis = torch.empty(s.shape, dtype=kappa.dtype, device=s.device)
    prec = F64 if kappa.dtype == torch.float64 else F32
    st = lib().porta_emissivity(int(s.shape[-1]), int(s.shape[0]), _ptr(kappa), _ptr(s),
                                _ptr(emis), int(prec), _stream(stream))
    _check("porta_emissivity", st)
    return emis


def rel_change(s_new, s_old, rc=None, workspace=None, stream=None):
    """porta_rel_change of the S00 rows; returns a device FP64 scalar."""
    import torch
    n = s_new.shape[-1]
    if rc is None:
        rc = torch.empty((), dtype=torch.float64, device=s_new.device)
    if workspace is None:
        workspace = _workspace(8 * ((n + 255) // 256), s_new.device)
    st = lib().porta_rel_change(int(n), _ptr(s_new), _ptr(s_old), _ptr(rc), _ptr(workspace),
                                workspace.numel(), _stream(stream))
    _check("porta_rel_change", st)
    return rc


def fs_adjoint(hg: HostGrid, kappa, propmat, emis, i_bottom, dl_ditop, w2=1.0, prec=F64,
               interp=BILINEAR, checkpoint_stride=8, g_kappa=None, g_propmat=None, g_emis=None,
               opts=None, workspace=None, stream=None, checkpoints=None):
    """porta_fs_adjoint; gradients are added to g_* (allocated as zeros if None).
    `checkpoints`: the buffer fs_sweep filled with the same stride and ray range (its
    size is passed along and checked), or None.  With a ray range in `opts` only its
    upward rays are differentiated."""
    import torch
    dev = kappa.device
    if g_kappa is None:
        g_kappa = torch.zeros_like(kappa)
    if g_propmat is None:
        g_propmat = torch.zeros_like(propmat)
    if g_emis is None:
        g_emis = torch.zeros_like(emis)
    if workspace is None:
        kind = WS_ADJOINT if checkpoints is None else WS_ADJOINT_CKPT
        workspace = _workspace(workspace_size(hg, prec, kind, checkpoint_stride, opts), dev)
    f = Fields(_ptr(kappa), _ptr(propmat), _ptr(emis), float(i_bottom), float(w2))
    st = lib().porta_fs_adjoint(C.byref(hg.grid), C.byref(hg.quad), C.byref(f), int(prec),
                                int(interp), C.byref(opts) if opts else None, _ptr(dl_ditop),
                                _ptr(checkpoints), _nbytes(checkpoints),
                                int(checkpoint_stride), _ptr(g_kappa),
                                _ptr(g_propmat),
                                _ptr(g_emis), _ptr(workspace), workspace.numel(), _stream(stream))
    _check("porta_fs_adjoint", st)
    return g_kappa, g_propmat, g_emis


def version() -> str:
    return lib().porta_version().decode()
