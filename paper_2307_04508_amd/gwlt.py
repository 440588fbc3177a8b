"""ctypes binding of the gwlt C ABI (include/gwlt.h): argument marshalling
only.  Device arrays are torch tensors on the context's device (their data
pointers are passed through); host arrays are numpy arrays.  Every function
has the name of its C entry point and raises ``GwError`` on a non-OK status.
There is no fallback: if libgwlt.so is missing the import fails.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgwlt.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} not found: build it with "
                      "`python paper_2307_04508_amd/build.py`")
# The library must use the HIP runtime that owns the tensors and streams it
# is handed.  torch ships its own libamdhip64.so.7; loading torch first makes
# the dynamic loader resolve the library's libamdhip64.so.7 to that copy
# instead of pulling a second runtime in from the ROCm install.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

GW_OK, GW_EINVAL, GW_ENOMEM, GW_EDEVICE, GW_ENOTSPD, GW_EPADE, GW_ENOCONV, \
    GW_EUNSUPPORTED = range(8)
GW_FP64, GW_FP32, GW_BF16X3 = 0, 1, 2
PRECISIONS = {"fp64": GW_FP64, "fp32": GW_FP32, "bf16x3": GW_BF16X3}

EXPORTS = ["gw_create", "gw_destroy", "gw_set_stream", "gw_sync", "gw_last_error",
           "gw_status_string", "gw_prepare", "gw_freq_grid_mgl", "gw_lt_grid_minimax",
           "gw_minimax_inverse", "gw_profile_enable", "gw_profile_get",
           "gw_naf_compress", "gw_naf_apply", "gw_polarizability_lt", "gw_screen",
           "gw_sigma_diag", "gw_qp_solve", "gw_g0w0",
           "gw_graph_begin", "gw_graph_end", "gw_graph_launch", "gw_graph_destroy",
           "gw_polarizability_lt_batched", "gw_screen_batched", "gw_sigma_diag_batched",
           "gw_qp_solve_batched", "gw_g0w0_batched", "gw_reserve", "gw_naf_compress_batched",
           "gw_naf_apply_batched", "gw_autotune", "gw_evgw", "gw_polarizability_sos",
           "gw_screen_sos", "gw_lt_grid_auto", "gw_sigma_diag_noalloc", "gw_autotune_restrict",
           "gw_autotune_save", "gw_autotune_load"]

c_int, c_i64, c_dbl, c_vp = ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
P_DBL = ctypes.POINTER(ctypes.c_double)
P_INT = ctypes.POINTER(ctypes.c_int)


class GwParams(ctypes.Structure):
    _fields_ = [("n_occ", c_int), ("n_fc", c_int), ("n_virt", c_int), ("n_aux", c_int),
                ("n_lt", c_int), ("n_freq", c_int), ("n_pade", c_int), ("n_qp", c_int),
                ("eps_naf", c_dbl), ("max_keep", c_int), ("x0", c_dbl), ("eta", c_dbl),
                ("tol", c_dbl), ("max_iter", c_int), ("freq_batch", c_int), ("no_lt", c_int),
                ("eps_lt", c_dbl)]


class GwStats(ctypes.Structure):
    _fields_ = [("n_naf", c_int), ("lt_err_norm", c_dbl), ("t_naf_ms", c_dbl),
                ("t_chi_ms", c_dbl), ("t_screen_ms", c_dbl), ("t_sigma_ms", c_dbl),
                ("t_qp_ms", c_dbl), ("t_total_ms", c_dbl), ("n_lt", c_int)]


class ChiJob(ctypes.Structure):
    _fields_ = [("n_naf", c_int), ("n_i", c_int), ("n_virt", c_int), ("x_lt", P_DBL),
                ("w_lt", P_DBL), ("eps_i", P_DBL), ("eps_a", P_DBL), ("R_chunk", c_vp),
                ("ld_R", c_i64), ("M", c_vp)]


class ScreenJob(ctypes.Structure):
    _fields_ = [("n_naf", c_int), ("x_lt", P_DBL), ("M", c_vp), ("n_w", c_int),
                ("omega", P_DBL), ("W_hat", c_vp)]


class SigmaJob(ctypes.Structure):
    _fields_ = [("n_naf", c_int), ("n_qp", c_int), ("n_mo", c_int), ("eps_mo", P_DBL),
                ("eps_F", c_dbl), ("R_qp", c_vp), ("ld_R", c_i64), ("n_w", c_int),
                ("omega", P_DBL), ("w_omega", P_DBL), ("W_hat", c_vp), ("n_pade", c_int),
                ("omega_pade", P_DBL), ("sigma_iw", c_vp), ("W_nm", c_vp)]


class QpJob(ctypes.Structure):
    _fields_ = [("n_qp", c_int), ("eps_n", P_DBL), ("static_n", P_DBL), ("eps_F", c_dbl),
                ("n_pade", c_int), ("omega_pade", P_DBL), ("sigma_iw", c_vp),
                ("eps_qp", P_DBL), ("z_factor", P_DBL), ("status", P_INT)]


class Mol(ctypes.Structure):
    _fields_ = [("n_occ", c_int), ("n_fc", c_int), ("n_virt", c_int), ("n_aux", c_int),
                ("n_qp", c_int), ("eps_naf", c_dbl), ("max_keep", c_int), ("eps", P_DBL),
                ("qp", P_INT), ("static_n", P_DBL), ("R_oo", c_vp), ("R_ov", c_vp),
                ("R_qp", c_vp), ("eps_qp", P_DBL), ("z_factor", P_DBL), ("status", P_INT),
                ("sigma_iw", P_DBL), ("n_naf", c_int)]


class BatchParams(ctypes.Structure):
    _fields_ = [("n_lt", c_int), ("n_freq", c_int), ("n_pade", c_int), ("x0", c_dbl),
                ("eta", c_dbl), ("tol", c_dbl), ("max_iter", c_int)]


class BatchStats(ctypes.Structure):
    _fields_ = [("t_naf_ms", c_dbl), ("t_rest_ms", c_dbl), ("t_total_ms", c_dbl),
                ("graph_replayed", c_int)]


GW_BATCH_GRAPH = 1


class Dims(ctypes.Structure):
    _fields_ = [("n_aux", c_int), ("n_naf", c_int), ("n_occ_act", c_int), ("n_virt", c_int),
                ("n_mo", c_int), ("n_qp", c_int), ("n_lt", c_int), ("n_w", c_int),
                ("n_pade", c_int), ("chunk_i", c_int)]


class NafJob(ctypes.Structure):
    _fields_ = [("n_aux", c_int), ("n_oo_rows", c_i64), ("R_oo", c_vp), ("n_ov_rows", c_i64),
                ("R_ov", c_vp), ("K", c_vp), ("eps_naf", c_dbl), ("max_keep", c_int),
                ("U", c_vp), ("n_naf", c_int), ("eigvals", P_DBL)]


class NafApplyJob(ctypes.Structure):
    _fields_ = [("n_aux", c_int), ("n_naf", c_int), ("U", c_vp), ("n_rows", c_i64),
                ("R_in", c_vp), ("R_out", c_vp), ("ld_out", c_i64)]

_sig = {
    "gw_create": [ctypes.POINTER(c_vp), c_int, c_vp],
    "gw_destroy": [c_vp],
    "gw_set_stream": [c_vp, c_vp],
    "gw_sync": [c_vp],
    "gw_profile_enable": [c_vp, c_int],
    "gw_profile_get": [c_vp, ctypes.c_char_p, P_DBL, ctypes.POINTER(c_i64), P_DBL, P_DBL],
    "gw_prepare": [c_int, c_int, c_int, P_DBL, c_dbl, P_DBL, P_DBL, P_DBL],
    "gw_freq_grid_mgl": [c_int, c_dbl, P_DBL, P_DBL],
    "gw_lt_grid_minimax": [c_int, c_dbl, c_dbl, P_DBL, P_DBL, P_DBL],
    "gw_minimax_inverse": [c_int, c_dbl, P_DBL, P_DBL, P_DBL, P_DBL, P_DBL],
    "gw_naf_compress": [c_vp, c_int, c_int, c_i64, c_vp, c_i64, c_vp, c_vp, c_int, c_int,
                        c_dbl, c_int, P_INT, c_vp, P_DBL],
    "gw_naf_apply": [c_vp, c_int, c_int, c_int, c_vp, c_i64, c_vp, c_vp, c_i64],
    "gw_polarizability_lt": [c_vp, c_int, c_int, c_int, P_DBL, P_DBL, c_int, c_int, P_DBL,
                             P_DBL, c_vp, c_i64, c_int, c_int, c_vp],
    "gw_screen": [c_vp, c_int, c_int, c_int, P_DBL, c_vp, c_int, P_DBL, c_vp],
    "gw_sigma_diag": [c_vp, c_int, c_int, c_int, c_int, P_DBL, c_dbl, c_vp, c_i64, c_int,
                      P_DBL, P_DBL, c_vp, c_int, P_DBL, c_int, c_vp, c_vp],
    "gw_sigma_diag_noalloc": [c_vp, c_int, c_int, c_int, c_int, P_DBL, c_dbl, c_vp, c_i64,
                              c_int, P_DBL, P_DBL, c_vp, c_int, P_DBL, c_int, c_vp, c_vp],
    "gw_qp_solve": [c_vp, c_int, P_DBL, P_DBL, c_dbl, c_int, P_DBL, c_vp, c_dbl, c_dbl, c_int,
                    P_DBL, P_DBL, P_INT],
    "gw_g0w0": [c_vp, c_int, ctypes.POINTER(GwParams), P_DBL, P_INT, P_DBL, c_vp, c_vp, c_vp,
                P_DBL, P_DBL, P_INT, P_DBL, ctypes.POINTER(GwStats)],
    "gw_reserve": [c_vp, c_int, ctypes.POINTER(Dims)],
    "gw_polarizability_sos": [c_vp, c_int, c_int, c_int, P_DBL, c_int, c_int, P_DBL, P_DBL,
                              c_vp, c_i64, c_int, c_int, c_vp],
    "gw_screen_sos": [c_vp, c_int, c_int, c_int, c_vp, c_vp],
    "gw_lt_grid_auto": [c_dbl, c_int, c_dbl, c_dbl, P_INT, P_DBL, P_DBL, P_DBL],
    "gw_evgw": [c_vp, c_int, ctypes.POINTER(GwParams), c_int, P_DBL, P_INT, P_DBL, c_vp, c_vp,
                c_vp, P_DBL, P_DBL, P_INT, P_DBL, ctypes.POINTER(GwStats)],
    "gw_autotune": [c_vp, c_int, P_INT],
    "gw_autotune_restrict": [c_vp, ctypes.c_char_p, c_int, c_int],
    "gw_autotune_save": [c_vp, ctypes.c_char_p],
    "gw_autotune_load": [c_vp, ctypes.c_char_p, P_INT],
    "gw_naf_compress_batched": [c_vp, c_int, c_int, ctypes.POINTER(NafJob)],
    "gw_naf_apply_batched": [c_vp, c_int, c_int, ctypes.POINTER(NafApplyJob)],
    "gw_graph_begin": [c_vp],
    "gw_graph_end": [c_vp, ctypes.POINTER(c_vp)],
    "gw_graph_launch": [c_vp, c_vp],
    "gw_graph_destroy": [c_vp],
    "gw_polarizability_lt_batched": [c_vp, c_int, c_int, c_int, ctypes.POINTER(ChiJob), c_int,
                                     c_int],
    "gw_screen_batched": [c_vp, c_int, c_int, c_int, ctypes.POINTER(ScreenJob)],
    "gw_sigma_diag_batched": [c_vp, c_int, c_int, ctypes.POINTER(SigmaJob), c_int],
    "gw_qp_solve_batched": [c_vp, c_int, ctypes.POINTER(QpJob), c_dbl, c_dbl, c_int],
    "gw_g0w0_batched": [c_vp, c_int, ctypes.POINTER(BatchParams), c_int, ctypes.POINTER(Mol),
                        c_int, ctypes.POINTER(BatchStats)],
}
for _name, _args in _sig.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = c_int
_lib.gw_last_error.argtypes = [c_vp]
_lib.gw_last_error.restype = ctypes.c_char_p
_lib.gw_status_string.argtypes = [c_int]
_lib.gw_status_string.restype = ctypes.c_char_p


class GwError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_lib.gw_status_string(status).decode()}: {msg}")
        self.status = status


def _check(st: int, ctx=None):
    if st != GW_OK:
        msg = _lib.gw_last_error(ctx.handle if ctx is not None else None)
        raise GwError(st, msg.decode() if msg else "")


def _prec(p) -> int:
    return PRECISIONS[p] if isinstance(p, str) else int(p)


def _host(a, dtype=np.float64):
    """Contiguous host array (kept alive by the caller's reference)."""
    return np.ascontiguousarray(a, dtype=dtype)


def _dp(a):
    return a.ctypes.data_as(P_DBL) if a is not None else None


def _ip(a):
    return a.ctypes.data_as(P_INT) if a is not None else None


def _ld(t, n_cols):
    """Row stride (elements) of a device tensor viewed as rows of n_cols."""
    if t is None or t.dim() < 2:
        return 0
    return int(t.stride(-2)) if t.stride(-1) == 1 else n_cols


def _dev(t, strided=False):
    """Device pointer of a torch tensor (or None).  Strided tensors (padded
    rows) are accepted where the C call takes a row stride."""
    if t is None:
        return None
    if not t.is_cuda or (not strided and not t.is_contiguous()):
        raise ValueError("device arguments must be contiguous GPU tensors")
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """A gwlt context bound to a device and a HIP stream (torch stream)."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(device)
        h = c_vp()
        _check(_lib.gw_create(ctypes.byref(h), device, c_vp(stream.cuda_stream)))
        self.handle = h
        self.device = device
        self.stream = stream

    def close(self):
        if self.handle:
            _lib.gw_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gw_create(device: int = 0, stream=None) -> Context:
    return Context(device, stream)


def gw_destroy(ctx: Context):
    ctx.close()


def gw_sync(ctx: Context):
    _check(_lib.gw_sync(ctx.handle), ctx)


def gw_profile_enable(ctx, enable: bool = True):
    _check(_lib.gw_profile_enable(ctx.handle, int(enable)), ctx)


def gw_profile_get(ctx, kernel: str):
    """(total_ms, launches, flops, bytes) recorded for `kernel`."""
    ms, fl, by, n = c_dbl(), c_dbl(), c_dbl(), c_i64()
    _check(_lib.gw_profile_get(ctx.handle, kernel.encode(), ctypes.byref(ms), ctypes.byref(n),
                               ctypes.byref(fl), ctypes.byref(by)), ctx)
    return ms.value, n.value, fl.value, by.value


def gw_prepare(n_occ, n_fc, n_virt, eps, omega_min):
    e = _host(eps)
    out = (c_dbl(), c_dbl(), c_dbl())
    _check(_lib.gw_prepare(n_occ, n_fc, n_virt, _dp(e), omega_min, *map(ctypes.byref, out)))
    return tuple(o.value for o in out)


def gw_freq_grid_mgl(n: int, x0: float = 0.5):
    om, wt = np.empty(n), np.empty(n)
    _check(_lib.gw_freq_grid_mgl(n, x0, _dp(om), _dp(wt)))
    return om, wt


def gw_lt_grid_minimax(n_lt: int, y_min: float, y_max: float):
    x, w, err = np.empty(n_lt), np.empty(n_lt), c_dbl()
    _check(_lib.gw_lt_grid_minimax(n_lt, y_min, y_max, _dp(x), _dp(w), ctypes.byref(err)))
    return x, w, err.value


def gw_lt_grid_auto(eps_lt: float, y_min: float, y_max: float, max_lt: int = 20):
    """Smallest Laplace grid meeting eps_lt: (n_lt, x, w, err)."""
    n = ctypes.c_int(0)
    x, w, err = np.empty(max_lt), np.empty(max_lt), c_dbl()
    _check(_lib.gw_lt_grid_auto(float(eps_lt), int(max_lt), float(y_min), float(y_max),
                                ctypes.byref(n), _dp(x), _dp(w), ctypes.byref(err)))
    return n.value, x[:n.value].copy(), w[:n.value].copy(), err.value


def lt_points_for(eps, cfg, eps_lt: float):
    """The accuracy-driven Laplace grid for a workload's energies (its bounds
    as gw_g0w0 takes them): {"L": n_lt, "err_norm": ...}."""
    om, _ = gw_freq_grid_mgl(cfg.n_freq, cfg.x0)
    _, y_min, y_max = gw_prepare(cfg.n_occ, cfg.n_fc, cfg.n_virt, eps, om[0])
    n, _, _, err = gw_lt_grid_auto(eps_lt, y_min, y_max)
    return {"L": n, "err_norm": err, "y_min": y_min, "y_max": y_max}


def gw_minimax_inverse(n_lt: int, R: float, alpha0=None, omega0=None):
    a0 = None if alpha0 is None else _host(alpha0)
    o0 = None if omega0 is None else _host(omega0)
    al, om, err = np.empty(n_lt), np.empty(n_lt), c_dbl()
    _check(_lib.gw_minimax_inverse(n_lt, R, _dp(a0), _dp(o0), _dp(al), _dp(om),
                                   ctypes.byref(err)))
    return al, om, err.value


def gw_naf_compress(ctx, prec, n_aux, R_oo, R_ov, K, accumulate, finalize, eps_naf,
                    max_keep, U, want_eigvals=True):
    n_oo = 0 if R_oo is None else R_oo.numel() // n_aux
    n_ov = 0 if R_ov is None else R_ov.numel() // n_aux
    n_naf = c_int(0)
    ev = np.empty(n_aux) if (finalize and want_eigvals) else None
    _check(_lib.gw_naf_compress(ctx.handle, _prec(prec), n_aux, n_oo, _dev(R_oo), n_ov,
                                _dev(R_ov), _dev(K), int(accumulate), int(finalize),
                                float(eps_naf), int(max_keep), ctypes.byref(n_naf),
                                _dev(U), _dp(ev)), ctx)
    return n_naf.value, ev


def gw_naf_apply(ctx, prec, n_aux, n_naf, U, R_in, R_out):
    n_rows = R_in.numel() // n_aux
    ld = R_out.shape[-1] if R_out.dim() >= 2 else n_naf
    _check(_lib.gw_naf_apply(ctx.handle, _prec(prec), n_aux, n_naf, _dev(U), n_rows,
                             _dev(R_in), _dev(R_out), ld), ctx)


def gw_polarizability_lt(ctx, prec, n_naf, x_lt, w_lt, n_i, n_virt, eps_i, eps_a, R_chunk,
                         accumulate, finalize, M):
    x, w = _host(x_lt), _host(w_lt)
    ei, ea = _host(eps_i), _host(eps_a)
    _check(_lib.gw_polarizability_lt(ctx.handle, _prec(prec), n_naf, len(x), _dp(x), _dp(w),
                                     n_i, n_virt, _dp(ei), _dp(ea), _dev(R_chunk, True),
                                     _ld(R_chunk, n_naf), int(accumulate), int(finalize),
                                     _dev(M)), ctx)


def gw_polarizability_sos(ctx, prec, n_naf, omega, n_i, n_virt, eps_i, eps_a, R_chunk,
                          accumulate, finalize, P):
    om = _host(omega)
    ei, ea = _host(eps_i), _host(eps_a)
    _check(_lib.gw_polarizability_sos(ctx.handle, _prec(prec), n_naf, len(om), _dp(om), n_i,
                                      n_virt, _dp(ei), _dp(ea), _dev(R_chunk, True),
                                      _ld(R_chunk, n_naf), int(accumulate), int(finalize),
                                      _dev(P)), ctx)


def gw_screen_sos(ctx, prec, n_naf, P, W_hat):
    _check(_lib.gw_screen_sos(ctx.handle, _prec(prec), n_naf, P.shape[0], _dev(P),
                              _dev(W_hat)), ctx)


def gw_screen(ctx, prec, n_naf, x_lt, M, omega, W_hat):
    x, om = _host(x_lt), _host(omega)
    _check(_lib.gw_screen(ctx.handle, _prec(prec), n_naf, len(x), _dp(x), _dev(M), len(om),
                          _dp(om), _dev(W_hat)), ctx)


def gw_sigma_diag(ctx, prec, n_naf, n_qp, n_mo, eps_mo, eps_F, R_qp, omega, w_omega, W_hat,
                  omega_pade, accumulate, sigma_iw, W_nm=None):
    e, om, wt, op = _host(eps_mo), _host(omega), _host(w_omega), _host(omega_pade)
    _check(_lib.gw_sigma_diag(ctx.handle, _prec(prec), n_naf, n_qp, n_mo, _dp(e), float(eps_F),
                              _dev(R_qp, True), _ld(R_qp, n_naf), len(om), _dp(om), _dp(wt),
                              _dev(W_hat), len(op), _dp(op), int(accumulate), _dev(sigma_iw),
                              _dev(W_nm)), ctx)


def gw_sigma_diag_noalloc(ctx, prec, n_naf, n_qp, n_mo, eps_mo, eps_F, R_qp, omega, w_omega,
                          W_hat, omega_pade, accumulate, sigma_iw, W_nm=None):
    e, om, wt, op = _host(eps_mo), _host(omega), _host(w_omega), _host(omega_pade)
    _check(_lib.gw_sigma_diag_noalloc(ctx.handle, _prec(prec), n_naf, n_qp, n_mo, _dp(e),
                                      float(eps_F), _dev(R_qp, True), _ld(R_qp, n_naf), len(om),
                                      _dp(om), _dp(wt), _dev(W_hat), len(op), _dp(op),
                                      int(accumulate), _dev(sigma_iw), _dev(W_nm)), ctx)


def gw_qp_solve(ctx, eps_n, static_n, eps_F, omega_pade, sigma_iw, eta, tol=1e-6,
                max_iter=100):
    en = _host(eps_n)
    st = None if static_n is None else _host(static_n)
    op = _host(omega_pade)
    q = len(en)
    E, Z, S = np.empty(q), np.empty(q), np.empty(q, dtype=np.int32)
    _check(_lib.gw_qp_solve(ctx.handle, q, _dp(en), _dp(st), float(eps_F), len(op), _dp(op),
                            _dev(sigma_iw), float(eta), float(tol), int(max_iter), _dp(E),
                            _dp(Z), _ip(S)), ctx)
    return E, Z, S


def gw_g0w0(ctx, prec, params: GwParams, eps, qp, static_n, R_oo, R_ov, R_qp,
            want_sigma=True):
    e = _host(eps)
    q = _host(qp, np.int32)
    st = None if static_n is None else _host(static_n)
    n = params.n_qp
    E, Z, S = np.empty(n), np.empty(n), np.empty(n, dtype=np.int32)
    sig = np.empty(2 * n * params.n_pade) if want_sigma else None
    stats = GwStats()
    _check(_lib.gw_g0w0(ctx.handle, _prec(prec), ctypes.byref(params), _dp(e), _ip(q), _dp(st),
                        _dev(R_oo), _dev(R_ov), _dev(R_qp), _dp(E), _dp(Z), _ip(S), _dp(sig),
                        ctypes.byref(stats)), ctx)
    sigma = None if sig is None else (sig[0::2] + 1j * sig[1::2]).reshape(n, params.n_pade)
    return E, Z, S, sigma, stats


def gw_evgw(ctx, prec, params: GwParams, n_cycles, eps, qp, static_n, R_oo, R_ov, R_qp):
    """Returns (eps_qp [n_cycles][n_qp], z [n_qp] of the last cycle, status
    [n_cycles][n_qp], energies of the next cycle, stats)."""
    e = _host(eps)
    q = _host(qp, np.int32)
    st = None if static_n is None else _host(static_n)
    n = params.n_qp
    E = np.empty((n_cycles, n))
    Z = np.empty(n)
    S = np.empty((n_cycles, n), dtype=np.int32)
    last = np.empty(len(e))
    stats = GwStats()
    _check(_lib.gw_evgw(ctx.handle, _prec(prec), ctypes.byref(params), int(n_cycles), _dp(e),
                        _ip(q), _dp(st), _dev(R_oo), _dev(R_ov), _dev(R_qp), _dp(E), _dp(Z),
                        _ip(S), _dp(last), ctypes.byref(stats)), ctx)
    return E, Z, S, last, stats


def params_for(cfg, freq_batch: int = 0, tol: float = 1e-6, max_iter: int = 100,
               no_lt: bool = False, eps_lt: float = 0.0) -> GwParams:
    """gw_params from a workload description with the fields of gwsynth.Config;
    eps_lt > 0 asks for the accuracy-driven Laplace grid (n_lt its upper bound)."""
    return GwParams(n_occ=cfg.n_occ, n_fc=cfg.n_fc, n_virt=cfg.n_virt, n_aux=cfg.n_aux,
                    n_lt=cfg.n_lt, n_freq=cfg.n_freq, n_pade=cfg.n_pade, n_qp=cfg.n_qp,
                    eps_naf=cfg.eps_naf, max_keep=cfg.max_keep, x0=cfg.x0, eta=cfg.eta,
                    tol=tol, max_iter=max_iter, freq_batch=freq_batch, no_lt=int(no_lt),
                    eps_lt=float(eps_lt))


# ------------------------------------------------------------------ graphs

class Graph:
    """A captured graph (gw_graph_end); released by close() or gw_graph_destroy."""

    def __init__(self, handle, ctx):
        self.handle = handle
        self.ctx = ctx

    def close(self):
        if self.handle:
            _lib.gw_graph_destroy(self.handle)
            self.handle = None


def gw_graph_begin(ctx):
    _check(_lib.gw_graph_begin(ctx.handle), ctx)


def gw_graph_end(ctx) -> Graph:
    h = c_vp()
    _check(_lib.gw_graph_end(ctx.handle, ctypes.byref(h)), ctx)
    return Graph(h, ctx)


def gw_graph_launch(ctx, graph: Graph):
    _check(_lib.gw_graph_launch(ctx.handle, graph.handle), ctx)


def gw_graph_destroy(graph: Graph):
    graph.close()


# ------------------------------------------------------------------ batched twins
# Job arguments are dicts with the keyword names of the single-molecule call;
# host arrays are converted and kept alive for the duration of the call.

def _jobs(cls, rows):
    arr = (cls * max(len(rows), 1))()
    for i, r in enumerate(rows):
        for k, v in r.items():
            setattr(arr[i], k, v)
    return arr


def gw_polarizability_lt_batched(ctx, prec, n_lt, jobs, accumulate, finalize):
    keep, rows = [], []
    for j in jobs:
        x, w, ei, ea = (_host(j["x_lt"]), _host(j["w_lt"]), _host(j["eps_i"]), _host(j["eps_a"]))
        keep += [x, w, ei, ea]
        R = j.get("R_chunk")
        rows.append(dict(n_naf=j["n_naf"], n_i=j["n_i"], n_virt=j["n_virt"], x_lt=_dp(x),
                         w_lt=_dp(w), eps_i=_dp(ei), eps_a=_dp(ea), R_chunk=_dev(R, True),
                         ld_R=_ld(R, j["n_naf"]), M=_dev(j["M"])))
    arr = _jobs(ChiJob, rows)
    _check(_lib.gw_polarizability_lt_batched(ctx.handle, _prec(prec), n_lt, len(rows), arr,
                                             int(accumulate), int(finalize)), ctx)


def gw_screen_batched(ctx, prec, n_lt, jobs):
    keep, rows = [], []
    for j in jobs:
        x, om = _host(j["x_lt"]), _host(j["omega"])
        keep += [x, om]
        rows.append(dict(n_naf=j["n_naf"], x_lt=_dp(x), M=_dev(j["M"]), n_w=len(om),
                         omega=_dp(om), W_hat=_dev(j["W_hat"])))
    arr = _jobs(ScreenJob, rows)
    _check(_lib.gw_screen_batched(ctx.handle, _prec(prec), n_lt, len(rows), arr), ctx)


def gw_sigma_diag_batched(ctx, prec, jobs, accumulate):
    keep, rows = [], []
    for j in jobs:
        e, om, wt, op = (_host(j["eps_mo"]), _host(j["omega"]), _host(j["w_omega"]),
                         _host(j["omega_pade"]))
        keep += [e, om, wt, op]
        R = j["R_qp"]
        rows.append(dict(n_naf=j["n_naf"], n_qp=j["n_qp"], n_mo=j["n_mo"], eps_mo=_dp(e),
                         eps_F=float(j["eps_F"]), R_qp=_dev(R, True), ld_R=_ld(R, j["n_naf"]),
                         n_w=len(om), omega=_dp(om), w_omega=_dp(wt), W_hat=_dev(j["W_hat"]),
                         n_pade=len(op), omega_pade=_dp(op), sigma_iw=_dev(j["sigma_iw"]),
                         W_nm=_dev(j.get("W_nm"))))
    arr = _jobs(SigmaJob, rows)
    _check(_lib.gw_sigma_diag_batched(ctx.handle, _prec(prec), len(rows), arr, int(accumulate)),
           ctx)


def gw_qp_solve_batched(ctx, jobs, eta, tol=1e-6, max_iter=100):
    """Returns a list of (eps_qp, z_factor, status) per job."""
    keep, rows, outs = [], [], []
    for j in jobs:
        en, op = _host(j["eps_n"]), _host(j["omega_pade"])
        st = None if j.get("static_n") is None else _host(j["static_n"])
        q = len(en)
        E, Z, S = np.empty(q), np.empty(q), np.empty(q, dtype=np.int32)
        keep += [en, op, st]
        outs.append((E, Z, S))
        rows.append(dict(n_qp=q, eps_n=_dp(en), static_n=_dp(st), eps_F=float(j["eps_F"]),
                         n_pade=len(op), omega_pade=_dp(op), sigma_iw=_dev(j["sigma_iw"]),
                         eps_qp=_dp(E), z_factor=_dp(Z), status=_ip(S)))
    arr = _jobs(QpJob, rows)
    _check(_lib.gw_qp_solve_batched(ctx.handle, len(rows), arr, float(eta), float(tol),
                                    int(max_iter)), ctx)
    return outs


def batch_params_for(cfg, tol: float = 1e-6, max_iter: int = 100) -> BatchParams:
    return BatchParams(n_lt=cfg.n_lt, n_freq=cfg.n_freq, n_pade=cfg.n_pade, x0=cfg.x0,
                       eta=cfg.eta, tol=tol, max_iter=max_iter)


def gw_g0w0_batched(ctx, prec, params: BatchParams, mols, graph=True, want_sigma=False):
    """mols: list of dicts with cfg (n_occ, n_fc, n_virt, n_aux, eps_naf, max_keep),
    eps, qp, R_oo, R_ov, R_qp (device) and optionally static_n.  Returns
    (list of (eps_qp, z, status, sigma or None, n_naf), BatchStats)."""
    keep, rows, outs = [], [], []
    for m in mols:
        c = m["cfg"]
        e, q = _host(m["eps"]), _host(m["qp"], np.int32)
        st = None if m.get("static_n") is None else _host(m["static_n"])
        nq = len(q)
        E, Z, S = np.empty(nq), np.empty(nq), np.empty(nq, dtype=np.int32)
        sig = np.empty(2 * nq * params.n_pade) if want_sigma else None
        keep += [e, q, st]
        outs.append((E, Z, S, sig))
        rows.append(dict(n_occ=c.n_occ, n_fc=c.n_fc, n_virt=c.n_virt, n_aux=c.n_aux, n_qp=nq,
                         eps_naf=float(c.eps_naf), max_keep=int(c.max_keep), eps=_dp(e),
                         qp=_ip(q), static_n=_dp(st), R_oo=_dev(m["R_oo"]),
                         R_ov=_dev(m["R_ov"]), R_qp=_dev(m["R_qp"]), eps_qp=_dp(E),
                         z_factor=_dp(Z), status=_ip(S), sigma_iw=_dp(sig), n_naf=0))
    arr = _jobs(Mol, rows)
    stats = BatchStats()
    _check(_lib.gw_g0w0_batched(ctx.handle, _prec(prec), ctypes.byref(params), len(rows), arr,
                                GW_BATCH_GRAPH if graph else 0, ctypes.byref(stats)), ctx)
    res = []
    for i, (E, Z, S, sig) in enumerate(outs):
        s2 = None if sig is None else (sig[0::2] + 1j * sig[1::2]).reshape(len(E), params.n_pade)
        res.append((E, Z, S, s2, arr[i].n_naf))
    return res, stats


def gw_reserve(ctx, prec, **dims):
    """Grow ctx's workspace for per-step calls up to the given sizes (the
    fields of gw_dims as keywords; missing ones are 0)."""
    d = Dims(**dims)
    _check(_lib.gw_reserve(ctx.handle, _prec(prec), ctypes.byref(d)), ctx)


def gw_naf_compress_batched(ctx, prec, jobs):
    """jobs: dicts with n_aux, R_oo, R_ov (device, or None), K, U (device),
    eps_naf, max_keep.  Returns [(n_naf, eigvals)] per job."""
    rows, evs = [], []
    for j in jobs:
        A = j["n_aux"]
        ev = np.empty(A)
        evs.append(ev)
        Roo, Rov = j.get("R_oo"), j.get("R_ov")
        rows.append(dict(n_aux=A, n_oo_rows=0 if Roo is None else Roo.numel() // A,
                         R_oo=_dev(Roo), n_ov_rows=0 if Rov is None else Rov.numel() // A,
                         R_ov=_dev(Rov), K=_dev(j["K"]), eps_naf=float(j["eps_naf"]),
                         max_keep=int(j.get("max_keep", 0)), U=_dev(j["U"]), n_naf=0,
                         eigvals=_dp(ev)))
    arr = _jobs(NafJob, rows)
    _check(_lib.gw_naf_compress_batched(ctx.handle, _prec(prec), len(rows), arr), ctx)
    return [(arr[i].n_naf, evs[i]) for i in range(len(rows))]


def gw_naf_apply_batched(ctx, prec, jobs):
    """jobs: dicts with n_aux, n_naf, U, R_in, R_out (device)."""
    rows = []
    for j in jobs:
        A = j["n_aux"]
        R_out = j["R_out"]
        rows.append(dict(n_aux=A, n_naf=j["n_naf"], U=_dev(j["U"]),
                         n_rows=j["R_in"].numel() // A, R_in=_dev(j["R_in"]),
                         R_out=_dev(R_out), ld_out=R_out.shape[-1]))
    arr = _jobs(NafApplyJob, rows)
    _check(_lib.gw_naf_apply_batched(ctx.handle, _prec(prec), len(rows), arr), ctx)


def gw_autotune_restrict(ctx, family: str, modulus: int, residue: int = 0) -> None:
    """Keep only the candidates c of a kernel family with c % modulus ==
    residue (modulus 0 lifts the restriction)."""
    _check(_lib.gw_autotune_restrict(ctx.handle, family.encode(), int(modulus), int(residue)),
           ctx)


def gw_autotune_save(ctx, path) -> None:
    """Write the context's kept autotuner choices to a text file."""
    _check(_lib.gw_autotune_save(ctx.handle, str(path).encode()), ctx)


def gw_autotune_load(ctx, path) -> int:
    """Read saved autotuner choices into the context; returns their number."""
    n = ctypes.c_int(0)
    _check(_lib.gw_autotune_load(ctx.handle, str(path).encode(), ctypes.byref(n)), ctx)
    return n.value


def gw_autotune(ctx, enable: int = -1) -> int:
    """Switch launch-shape autotuning (0 off, 1 on, 2 on and forget, -1 keep);
    returns the number of kept choices."""
    n = ctypes.c_int(0)
    _check(_lib.gw_autotune(ctx.handle, int(enable), ctypes.byref(n)), ctx)
    return n.value
