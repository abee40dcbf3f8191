"""ctypes binding of libscdyson.so: argument marshalling only.

Every entry point of ``include/scdyson.h`` is exposed under the same name.
Tensors are PyTorch tensors on the current HIP device (complex128 for Green's
functions, float64 for real inputs); the current torch stream is passed to the
library.  No arithmetic of the method happens here, and there is no fallback:
if the library is missing the first call raises.
"""
import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("SCD_LIBRARY") or os.path.join(_HERE, "libscdyson.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "scdyson.h")

SCD_OK, SCD_EINVAL, SCD_ENOMEM, SCD_EHIP, SCD_ENOTCONV, SCD_EDIVERGED, SCD_ENAN = 0, -1, -2, -3, -4, -5, -6
PREC_FP64, PREC_FP32, PREC_BF16X3 = 0, 1, 2
ERROR_NAMES = {0: "SCD_OK", -1: "SCD_EINVAL", -2: "SCD_ENOMEM", -3: "SCD_EHIP",
               -4: "SCD_ENOTCONV", -5: "SCD_EDIVERGED", -6: "SCD_ENAN"}


class Problem(ctypes.Structure):
    _fields_ = [("Lx", ctypes.c_int32), ("Ly", ctypes.c_int32), ("periodic", ctypes.c_int32),
                ("n_real", ctypes.c_int32), ("n_imag", ctypes.c_int32),
                ("dt", ctypes.c_double), ("beta", ctypes.c_double), ("mu", ctypes.c_double),
                ("t_min", ctypes.c_double)]

    @property
    def n_r(self):
        return self.Lx * self.Ly

    @property
    def n_t(self):
        return 2 * self.n_real + self.n_imag


class Stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("n_blocks", ctypes.c_int32),
                ("sweeps_total", ctypes.c_int32), ("sweeps_max", ctypes.c_int32),
                ("fp64_sweeps", ctypes.c_int32), ("lowp_sweeps", ctypes.c_int32),
                ("final_err", ctypes.c_double), ("rho_est", ctypes.c_double),
                ("gemm_flops", ctypes.c_double), ("seconds", ctypes.c_double),
                ("sweep_kernel_seconds", ctypes.c_double),
                ("lowp_kernel_seconds", ctypes.c_double),
                ("sweep_launches", ctypes.c_int32), ("lowp_launches", ctypes.c_int32),
                ("stream_kernel_seconds", ctypes.c_double), ("stream_bytes", ctypes.c_double),
                ("stream_launches", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class ScdError(RuntimeError):
    def __init__(self, code, message, stats=None):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {message}")
        self.code = code
        self.stats = stats


_lib = None
_P = ctypes.POINTER
_vp = ctypes.c_void_p


def lib():
    """Load libscdyson.so (once; SCD_LIBRARY may name another build).  Raises if it
    has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing; build it with "
                           "`python -m paper_1309_5994_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    L.scd_last_error.restype = ctypes.c_char_p
    L.scd_last_error.argtypes = []
    L.scd_workspace_bytes.restype = ctypes.c_int
    L.scd_workspace_bytes.argtypes = [_P(Problem), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                      _P(ctypes.c_size_t)]
    L.sigma_build.restype = ctypes.c_int
    L.sigma_build.argtypes = [_P(Problem), _vp, _vp, _vp, _vp]
    L.dyson_iterate.restype = ctypes.c_int
    L.dyson_iterate.argtypes = [_P(Problem), _vp, _vp, _P(ctypes.c_int32), ctypes.c_int32,
                                ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                _vp, _vp, _vp, _vp, ctypes.c_size_t, _P(Stats), _vp]
    L.dyson_iterate_trunc.restype = ctypes.c_int
    L.dyson_iterate_trunc.argtypes = [_P(Problem), _vp, _vp, _P(ctypes.c_int32), ctypes.c_int32,
                                      ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                      ctypes.c_int32, _vp, _vp, _vp, _vp, ctypes.c_size_t,
                                      _P(Stats), _vp]
    L.scd_sym_workspace_bytes.restype = ctypes.c_int
    L.scd_sym_workspace_bytes.argtypes = [_P(Problem), _P(ctypes.c_int32), ctypes.c_int32,
                                          ctypes.c_int32, ctypes.c_int32, _P(ctypes.c_size_t)]
    L.dyson_iterate_sym.restype = ctypes.c_int
    L.dyson_iterate_sym.argtypes = L.dyson_iterate.argtypes
    L.scd_gmres_workspace_bytes.restype = ctypes.c_int
    L.scd_gmres_workspace_bytes.argtypes = [_P(Problem), ctypes.c_int32, ctypes.c_int32,
                                            ctypes.c_int32, _P(ctypes.c_size_t)]
    L.dyson_gmres.restype = ctypes.c_int
    L.dyson_gmres.argtypes = [_P(Problem), _vp, _vp, _P(ctypes.c_int32), ctypes.c_int32,
                              ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                              _vp, _vp, _vp, _vp, ctypes.c_size_t, _P(Stats), _vp]
    L.scd_sigma2_workspace_bytes.restype = ctypes.c_int
    L.scd_sigma2_workspace_bytes.argtypes = [_P(Problem), _P(ctypes.c_size_t)]
    L.sigma2_build.restype = ctypes.c_int
    L.sigma2_build.argtypes = [_P(Problem), _vp, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t,
                               _vp]
    L.sigma2_dress.restype = ctypes.c_int
    L.sigma2_dress.argtypes = [_P(Problem), _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]
    L.scd_selfconsistent_workspace_bytes.restype = ctypes.c_int
    L.scd_selfconsistent_workspace_bytes.argtypes = [_P(Problem), ctypes.c_int32, ctypes.c_int32,
                                                     _P(ctypes.c_size_t)]
    L.dyson_selfconsistent.restype = ctypes.c_int
    L.dyson_selfconsistent.argtypes = [_P(Problem), _vp, _vp, _vp, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_int32, ctypes.c_double, ctypes.c_int32, _vp, _vp,
                                       _vp, _vp, _vp, ctypes.c_size_t, _P(ctypes.c_int32),
                                       _P(ctypes.c_double), _P(Stats), _vp]
    L.double_occupancy.restype = ctypes.c_int
    L.double_occupancy.argtypes = [_P(Problem), _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_int32,
                                   _vp, _vp, _vp]
    L.scd_extrapolate_dt.restype = ctypes.c_int
    L.scd_extrapolate_dt.argtypes = [_P(ctypes.c_double), ctypes.c_int32, _P(ctypes.c_double),
                                     ctypes.c_int32, _P(ctypes.c_double)]
    L.local_observables.restype = ctypes.c_int
    L.local_observables.argtypes = [_P(Problem), _vp, _vp, _vp, ctypes.c_int32, _vp, _vp, _vp]
    L.scd_adjoint_workspace_bytes.restype = ctypes.c_int
    L.scd_adjoint_workspace_bytes.argtypes = [_P(Problem), ctypes.c_int32, _P(ctypes.c_size_t)]
    L.dyson_adjoint.restype = ctypes.c_int
    L.dyson_adjoint.argtypes = [_P(Problem), _vp, _vp, _vp, _vp, _vp, ctypes.c_int32,
                                ctypes.c_int32, ctypes.c_double, ctypes.c_int32, _vp, _vp, _vp,
                                _vp, _vp, _vp, ctypes.c_size_t, _P(Stats), _vp]
    _lib = L
    return L


def header_functions():
    """Names of the functions that include/scdyson.h declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", text, flags=re.M)))


def last_error() -> str:
    return lib().scd_last_error().decode()


def _check(rc, stats=None):
    if rc != SCD_OK:
        raise ScdError(rc, last_error(), stats)


def problem(Lx, Ly, n_real, n_imag, dt, beta, mu=0.0, t_min=0.0, periodic=False) -> Problem:
    return Problem(int(Lx), int(Ly), int(bool(periodic)), int(n_real), int(n_imag), float(dt),
                   float(beta), float(mu), float(t_min))


def problem_from_workload(wl) -> Problem:
    return problem(wl.Lx, wl.Ly, wl.n_real, wl.n_imag, wl.dt, wl.beta, wl.mu, wl.t_min,
                   wl.periodic)


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _need(t, dtype, shape, name):
    import torch
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def workspace_bytes(prob: Problem, n_src, block_sites, prec=PREC_FP64) -> int:
    out = ctypes.c_size_t(0)
    _check(lib().scd_workspace_bytes(ctypes.byref(prob), int(n_src), int(block_sites), int(prec),
                                     ctypes.byref(out)))
    return out.value


def sigma_build(prob: Problem, V, U, S=None, stream=None):
    """S[N_r, N_t, N_t] (complex128) from V[N_r], U[n_real] (float64, on device)."""
    import torch
    _need(V, torch.float64, (prob.n_r,), "V")
    _need(U, torch.float64, (prob.n_real,), "U")
    if S is None:
        S = torch.empty((prob.n_r, prob.n_t, prob.n_t), dtype=torch.complex128, device=V.device)
    _need(S, torch.complex128, (prob.n_r, prob.n_t, prob.n_t), "S")
    _check(lib().sigma_build(ctypes.byref(prob), _ptr(V), _ptr(U), _ptr(S), _stream(stream)))
    return S


def dyson_iterate(prob: Problem, S, J, src, block_sites=None, prec=PREC_FP64, tol=1e-12,
                  max_iter=500, want_cols=False, want_nn=True, ws=None, out=None, stream=None):
    """Columns of G for the source sites ``src``.

    Returns dict(G_loc [n_src,N_t,N_t], G_nn [n_src,4,N_t,N_t] or None,
    G_cols [N_r,N_t,n_src*N_t] or None, stats dict).  Raises ScdError on
    failure (the error carries the stats).
    """
    import torch
    n_r, n_t = prob.n_r, prob.n_t
    src = np.ascontiguousarray(np.asarray(src, dtype=np.int32).reshape(-1))
    n_src = int(src.size)
    block_sites = n_src if block_sites is None else int(block_sites)
    _need(S, torch.complex128, (n_r, n_t, n_t), "S")
    _need(J, torch.float64, (prob.n_real,), "J")
    dev = S.device
    out = dict(out or {})
    G_loc = out.get("G_loc")
    if G_loc is None:
        G_loc = torch.empty((n_src, n_t, n_t), dtype=torch.complex128, device=dev)
    G_nn = out.get("G_nn")
    if want_nn and G_nn is None:
        G_nn = torch.empty((n_src, 4, n_t, n_t), dtype=torch.complex128, device=dev)
    G_cols = out.get("G_cols")
    if want_cols and G_cols is None:
        G_cols = torch.empty((n_r, n_t, n_src * n_t), dtype=torch.complex128, device=dev)
    need = workspace_bytes(prob, n_src, block_sites, prec)
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
    st = Stats()
    rc = lib().dyson_iterate(ctypes.byref(prob), _ptr(S), _ptr(J),
                             src.ctypes.data_as(_P(ctypes.c_int32)), n_src, block_sites, int(prec),
                             float(tol), int(max_iter), _ptr(G_cols), _ptr(G_loc), _ptr(G_nn),
                             _ptr(ws), ctypes.c_size_t(ws.numel()), ctypes.byref(st),
                             _stream(stream))
    _check(rc, st.as_dict())
    return {"G_loc": G_loc, "G_nn": G_nn, "G_cols": G_cols, "stats": st.as_dict(), "ws": ws}


def dyson_iterate_trunc(prob: Problem, S, J, src, max_radius, block_sites=None, tol=1e-12,
                        max_iter=500, want_cols=False, want_nn=True, ws=None, out=None,
                        stream=None):
    """``dyson_iterate`` (FP64) restricted to the sites within ``max_radius`` of
    each column's source."""
    import torch
    n_r, n_t = prob.n_r, prob.n_t
    src = np.ascontiguousarray(np.asarray(src, dtype=np.int32).reshape(-1))
    n_src = int(src.size)
    block_sites = n_src if block_sites is None else int(block_sites)
    _need(S, torch.complex128, (n_r, n_t, n_t), "S")
    _need(J, torch.float64, (prob.n_real,), "J")
    G_loc, G_nn, G_cols = _outputs(prob, n_src, S.device, out, want_cols, want_nn)
    need = workspace_bytes(prob, n_src, block_sites, PREC_FP64)
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=S.device)
    st = Stats()
    rc = lib().dyson_iterate_trunc(ctypes.byref(prob), _ptr(S), _ptr(J),
                                   src.ctypes.data_as(_P(ctypes.c_int32)), n_src, block_sites,
                                   int(max_radius), float(tol), int(max_iter), _ptr(G_cols),
                                   _ptr(G_loc), _ptr(G_nn), _ptr(ws), ctypes.c_size_t(ws.numel()),
                                   ctypes.byref(st), _stream(stream))
    _check(rc, st.as_dict())
    return {"G_loc": G_loc, "G_nn": G_nn, "G_cols": G_cols, "stats": st.as_dict(), "ws": ws}


def sym_workspace_bytes(prob: Problem, src, block_sites, prec=PREC_FP64) -> int:
    src = np.ascontiguousarray(np.asarray(src, dtype=np.int32).reshape(-1))
    out = ctypes.c_size_t(0)
    _check(lib().scd_sym_workspace_bytes(ctypes.byref(prob), src.ctypes.data_as(_P(ctypes.c_int32)),
                                         int(src.size), int(block_sites), int(prec),
                                         ctypes.byref(out)))
    return out.value


def dyson_iterate_sym(prob: Problem, S, J, src, block_sites=None, prec=PREC_FP64, tol=1e-12,
                      max_iter=500, want_cols=False, want_nn=True, ws=None, out=None,
                      stream=None):
    """``dyson_iterate`` with only one source per point-group orbit solved (App. A);
    same outputs for every requested source."""
    import torch
    n_r, n_t = prob.n_r, prob.n_t
    src = np.ascontiguousarray(np.asarray(src, dtype=np.int32).reshape(-1))
    n_src = int(src.size)
    block_sites = n_src if block_sites is None else int(block_sites)
    _need(S, torch.complex128, (n_r, n_t, n_t), "S")
    _need(J, torch.float64, (prob.n_real,), "J")
    G_loc, G_nn, G_cols = _outputs(prob, n_src, S.device, out, want_cols, want_nn)
    need = sym_workspace_bytes(prob, src, block_sites, prec)
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=S.device)
    st = Stats()
    rc = lib().dyson_iterate_sym(ctypes.byref(prob), _ptr(S), _ptr(J),
                                 src.ctypes.data_as(_P(ctypes.c_int32)), n_src, block_sites,
                                 int(prec), float(tol), int(max_iter), _ptr(G_cols), _ptr(G_loc),
                                 _ptr(G_nn), _ptr(ws), ctypes.c_size_t(ws.numel()),
                                 ctypes.byref(st), _stream(stream))
    _check(rc, st.as_dict())
    return {"G_loc": G_loc, "G_nn": G_nn, "G_cols": G_cols, "stats": st.as_dict(), "ws": ws}


def gmres_workspace_bytes(prob: Problem, n_src, block_sites, restart) -> int:
    out = ctypes.c_size_t(0)
    _check(lib().scd_gmres_workspace_bytes(ctypes.byref(prob), int(n_src), int(block_sites),
                                           int(restart), ctypes.byref(out)))
    return out.value


def _outputs(prob, n_src, dev, out, want_cols, want_nn):
    import torch
    n_r, n_t = prob.n_r, prob.n_t
    out = dict(out or {})
    G_loc = out.get("G_loc")
    if G_loc is None:
        G_loc = torch.empty((n_src, n_t, n_t), dtype=torch.complex128, device=dev)
    G_nn = out.get("G_nn")
    if want_nn and G_nn is None:
        G_nn = torch.empty((n_src, 4, n_t, n_t), dtype=torch.complex128, device=dev)
    G_cols = out.get("G_cols")
    if want_cols and G_cols is None:
        G_cols = torch.empty((n_r, n_t, n_src * n_t), dtype=torch.complex128, device=dev)
    return G_loc, G_nn, G_cols


def dyson_gmres(prob: Problem, S, J, src, block_sites=None, restart=8, tol=1e-12,
                max_iter=500, want_cols=False, want_nn=True, ws=None, out=None, stream=None):
    """Columns of G for the source sites ``src`` by preconditioned restarted
    GMRES (App. C); same outputs as ``dyson_iterate``."""
    import torch
    n_r, n_t = prob.n_r, prob.n_t
    src = np.ascontiguousarray(np.asarray(src, dtype=np.int32).reshape(-1))
    n_src = int(src.size)
    block_sites = n_src if block_sites is None else int(block_sites)
    _need(S, torch.complex128, (n_r, n_t, n_t), "S")
    _need(J, torch.float64, (prob.n_real,), "J")
    G_loc, G_nn, G_cols = _outputs(prob, n_src, S.device, out, want_cols, want_nn)
    need = gmres_workspace_bytes(prob, n_src, block_sites, restart)
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=S.device)
    st = Stats()
    rc = lib().dyson_gmres(ctypes.byref(prob), _ptr(S), _ptr(J),
                           src.ctypes.data_as(_P(ctypes.c_int32)), n_src, block_sites,
                           int(restart), float(tol), int(max_iter), _ptr(G_cols), _ptr(G_loc),
                           _ptr(G_nn), _ptr(ws), ctypes.c_size_t(ws.numel()), ctypes.byref(st),
                           _stream(stream))
    _check(rc, st.as_dict())
    return {"G_loc": G_loc, "G_nn": G_nn, "G_cols": G_cols, "stats": st.as_dict(), "ws": ws}


def local_observables(prob: Problem, G_loc, G_nn, J, want_ekin=True, stream=None):
    """(n [n_src, n_real], ekin [n_src, n_real] or None) on the device."""
    import torch
    n_src = int(G_loc.shape[0])
    _need(G_loc, torch.complex128, (n_src, prob.n_t, prob.n_t), "G_loc")
    _need(J, torch.float64, (prob.n_real,), "J")
    n = torch.empty((n_src, prob.n_real), dtype=torch.float64, device=G_loc.device)
    ekin = None
    if want_ekin:
        _need(G_nn, torch.complex128, (n_src, 4, prob.n_t, prob.n_t), "G_nn")
        ekin = torch.empty_like(n)
    _check(lib().local_observables(ctypes.byref(prob), _ptr(G_loc), _ptr(G_nn if want_ekin else None),
                                   _ptr(J), n_src, _ptr(n), _ptr(ekin), _stream(stream)))
    return n, ekin


def sigma2_workspace_bytes(prob: Problem) -> int:
    out = ctypes.c_size_t(0)
    _check(lib().scd_sigma2_workspace_bytes(ctypes.byref(prob), ctypes.byref(out)))
    return out.value


def sigma2_build(prob: Problem, V, U, J, S, G_loc_all, out=None, ws=None, stream=None):
    """Sigma~ [N_r, N_t, N_t] (eq. defnSigmatilde) from every site's local G."""
    import torch
    shape = (prob.n_r, prob.n_t, prob.n_t)
    _need(S, torch.complex128, shape, "S")
    _need(G_loc_all, torch.complex128, shape, "G_loc_all")
    _need(V, torch.float64, (prob.n_r,), "V")
    _need(U, torch.float64, (prob.n_real,), "U")
    _need(J, torch.float64, (prob.n_real,), "J")
    out = torch.empty(shape, dtype=torch.complex128, device=S.device) if out is None else out
    need = sigma2_workspace_bytes(prob)
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=S.device)
    _check(lib().sigma2_build(ctypes.byref(prob), _ptr(V), _ptr(U), _ptr(J), _ptr(S),
                              _ptr(G_loc_all), _ptr(out), _ptr(ws), ctypes.c_size_t(ws.numel()),
                              _stream(stream)))
    return out


def sigma2_dress(prob: Problem, S, sig, out=None, ws=None, stream=None):
    """S' = S (S - Sigma~)^-1 S per site (eq. defnSigma, eq. Glatt)."""
    import torch
    shape = (prob.n_r, prob.n_t, prob.n_t)
    _need(S, torch.complex128, shape, "S")
    _need(sig, torch.complex128, shape, "sig")
    out = torch.empty(shape, dtype=torch.complex128, device=S.device) if out is None else out
    need = sigma2_workspace_bytes(prob)
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=S.device)
    _check(lib().sigma2_dress(ctypes.byref(prob), _ptr(S), _ptr(sig), _ptr(out), _ptr(ws),
                              ctypes.c_size_t(ws.numel()), _stream(stream)))
    return out


def dyson_selfconsistent(prob: Problem, V, U, J, lam=0.7, delta_sc=1e-8, max_sc=50,
                         block_sites=None, prec=PREC_FP64, tol=1e-12, max_iter=500, ws=None,
                         stream=None):
    """The self-consistent second-order solution of Sec. III.  Returns dict(S,
    sigma, G_loc, G_nn, iterations, norm, stats)."""
    import torch
    n_r, n_t = prob.n_r, prob.n_t
    _need(V, torch.float64, (n_r,), "V")
    _need(U, torch.float64, (prob.n_real,), "U")
    _need(J, torch.float64, (prob.n_real,), "J")
    block_sites = n_r if block_sites is None else int(block_sites)
    dev = V.device
    S = torch.empty((n_r, n_t, n_t), dtype=torch.complex128, device=dev)
    sig = torch.empty_like(S)
    G_loc = torch.empty_like(S)
    G_nn = torch.empty((n_r, 4, n_t, n_t), dtype=torch.complex128, device=dev)
    out = ctypes.c_size_t(0)
    _check(lib().scd_selfconsistent_workspace_bytes(ctypes.byref(prob), block_sites, int(prec),
                                                    ctypes.byref(out)))
    if ws is None or ws.numel() < out.value:
        ws = torch.empty(out.value, dtype=torch.uint8, device=dev)
    it = ctypes.c_int32(0)
    norm = ctypes.c_double(0.0)
    st = Stats()
    rc = lib().dyson_selfconsistent(ctypes.byref(prob), _ptr(V), _ptr(U), _ptr(J), float(lam),
                                    float(delta_sc), int(max_sc), block_sites, int(prec),
                                    float(tol), int(max_iter), _ptr(S), _ptr(sig), _ptr(G_loc),
                                    _ptr(G_nn), _ptr(ws), ctypes.c_size_t(ws.numel()),
                                    ctypes.byref(it), ctypes.byref(norm), ctypes.byref(st),
                                    _stream(stream))
    _check(rc, st.as_dict())
    return {"S": S, "sigma": sig, "G_loc": G_loc, "G_nn": G_nn, "iterations": it.value,
            "norm": norm.value, "stats": st.as_dict()}


def double_occupancy(prob: Problem, G_loc, G_nn, J, V, U, src, want_fraction=True,
                     stream=None):
    """(D [n_src, n_real], doubly occupied fraction [n_real] or None) on the device
    for the source sites ``src`` of the blocks (eq. docc)."""
    import torch
    n_src = int(G_loc.shape[0])
    _need(G_loc, torch.complex128, (n_src, prob.n_t, prob.n_t), "G_loc")
    _need(G_nn, torch.complex128, (n_src, 4, prob.n_t, prob.n_t), "G_nn")
    _need(J, torch.float64, (prob.n_real,), "J")
    _need(U, torch.float64, (prob.n_real,), "U")
    _need(V, torch.float64, (prob.n_r,), "V")
    src_d = torch.as_tensor(np.asarray(src, dtype=np.int32).reshape(-1), device=G_loc.device)
    if src_d.numel() != n_src:
        raise ValueError("one source site per block")
    D = torch.empty((n_src, prob.n_real), dtype=torch.float64, device=G_loc.device)
    frac = torch.empty(prob.n_real, dtype=torch.float64, device=G_loc.device) if want_fraction \
        else None
    _check(lib().double_occupancy(ctypes.byref(prob), _ptr(G_loc), _ptr(G_nn), _ptr(J), _ptr(V),
                                  _ptr(U), _ptr(src_d), n_src, _ptr(D), _ptr(frac),
                                  _stream(stream)))
    return D, frac


def extrapolate_dt(dts, values):
    """Value at dt -> 0 (linear for two step sizes, quadratic for three) of host
    arrays values[k] sampled at the same physical times."""
    dts = np.ascontiguousarray(np.asarray(dts, dtype=np.float64))
    vals = np.ascontiguousarray(np.asarray(values, dtype=np.float64))
    shape = vals.shape[1:]
    flat = vals.reshape(len(dts), -1)
    out = np.empty(flat.shape[1], dtype=np.float64)
    _check(lib().scd_extrapolate_dt(dts.ctypes.data_as(_P(ctypes.c_double)), int(dts.size),
                                    flat.ctypes.data_as(_P(ctypes.c_double)), int(flat.shape[1]),
                                    out.ctypes.data_as(_P(ctypes.c_double))))
    return out.reshape(shape)


def adjoint_workspace_bytes(prob: Problem, prec=PREC_FP64) -> int:
    out = ctypes.c_size_t(0)
    _check(lib().scd_adjoint_workspace_bytes(ctypes.byref(prob), int(prec), ctypes.byref(out)))
    return out.value


def dyson_adjoint(prob: Problem, S, V, U, J, w=None, t_index=None, prec=PREC_FP64, tol=1e-12,
                  max_iter=500, grads=True, want_n=True, ws=None, stream=None):
    """Densities n_l(t_e) of every site and, with ``grads``, the gradients of
    L = sum_l w_l n_l(t_e) with respect to V, U(t) and J(t).

    Returns dict(n_te, loss, dV, dU, dJ, stats); t_index defaults to the last
    forward time.  Raises ScdError on failure."""
    import torch
    n_r = prob.n_r
    _need(S, torch.complex128, (n_r, prob.n_t, prob.n_t), "S")
    _need(J, torch.float64, (prob.n_real,), "J")
    if grads:
        _need(V, torch.float64, (n_r,), "V")
        _need(U, torch.float64, (prob.n_real,), "U")
    if w is not None:
        _need(w, torch.float64, (n_r,), "w")
    dev = S.device
    t_index = prob.n_real - 1 if t_index is None else int(t_index)
    n_te = torch.empty(n_r, dtype=torch.float64, device=dev) if want_n else None
    loss = torch.empty(1, dtype=torch.float64, device=dev) if w is not None else None
    dV = dU = dJ = None
    if grads:
        if w is None:
            raise ValueError("gradients need loss weights w")
        dV = torch.empty(n_r, dtype=torch.float64, device=dev)
        dU = torch.empty(prob.n_real, dtype=torch.float64, device=dev)
        dJ = torch.empty(prob.n_real, dtype=torch.float64, device=dev)
    need = adjoint_workspace_bytes(prob, prec)
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
    st = Stats()
    rc = lib().dyson_adjoint(ctypes.byref(prob), _ptr(S), _ptr(V if grads else None),
                             _ptr(U if grads else None), _ptr(J), _ptr(w), t_index, int(prec),
                             float(tol), int(max_iter), _ptr(n_te), _ptr(loss), _ptr(dV), _ptr(dU),
                             _ptr(dJ), _ptr(ws), ctypes.c_size_t(ws.numel()), ctypes.byref(st),
                             _stream(stream))
    _check(rc, st.as_dict())
    return {"n_te": n_te, "loss": loss, "dV": dV, "dU": dU, "dJ": dJ, "stats": st.as_dict()}


def _density_fn():
    import torch

    class DysonDensity(torch.autograd.Function):
        """n_l(t_e) for every site as a differentiable function of the trap
        potential V, the interaction U(t) and the hopping J(t).  The backward
        pass is the hand-written adjoint Dyson solve (dyson_adjoint), which
        recomputes the forward columns instead of storing iterates."""

        @staticmethod
        def forward(ctx, V, U, J, prob, t_index, prec, tol):
            S = sigma_build(prob, V, U)
            out = dyson_adjoint(prob, S, V, U, J, w=None, t_index=t_index, prec=prec, tol=tol,
                                grads=False)
            ctx.save_for_backward(V, U, J)
            ctx.cfg = (prob, t_index, prec, tol)
            return out["n_te"]

        @staticmethod
        def backward(ctx, grad_n):
            V, U, J = ctx.saved_tensors
            prob, t_index, prec, tol = ctx.cfg
            S = sigma_build(prob, V, U)
            out = dyson_adjoint(prob, S, V, U, J, w=grad_n.contiguous().to(torch.float64),
                                t_index=t_index, prec=prec, tol=tol, grads=True, want_n=False)
            return out["dV"], out["dU"], out["dJ"], None, None, None, None

    return DysonDensity


_DENSITY_FN = None


def density_at(prob: Problem, V, U, J, t_index=None, prec=PREC_FP64, tol=1e-12):
    """Differentiable n_l(t_e) (torch tensors V, U, J on the device)."""
    global _DENSITY_FN
    if _DENSITY_FN is None:
        _DENSITY_FN = _density_fn()
    t_index = prob.n_real - 1 if t_index is None else int(t_index)
    return _DENSITY_FN.apply(V, U, J, prob, t_index, prec, tol)
