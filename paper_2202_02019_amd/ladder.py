"""ctypes binding of libladder.so with the names of the C ABI (include/ladder.h).

Argument marshalling only: every step of the ladder runs in the library's HIP
kernels.  Tensors must be float64, contiguous and on the current HIP device.
Workspace and outputs are allocated with torch when the caller does not pass them
(device memory is the only thing torch provides here).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

PKG = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(PKG, "libladder.so")

FP64 = 0
SPLIT_BF16 = 1
SPLIT_INT8 = 2
FLAG_GENERAL = 1
FLAG_DENSE = 2
DO_FORWARD = 1
DO_ADJOINT = 2
U_TABLE = 0
U_APPENDIX = 1

EXPORTS = (
    "ladder_default_options", "ladder_workspace_size", "ladder_forward", "ladder_adjoint",
    "ladder_tau_gradient_workspace_size", "ladder_tau_gradient", "ladder_autotune", "ladder_autotune_load",
    "ladder_autotune_reset", "ladder_metric_contraction",
    "ladder_back_transform_workspace_size", "ladder_back_transform", "ladder_excited_amplitudes",
    "ladder_ov3_abci_workspace_size", "ladder_ov3_abci", "ladder_ov3_abic_workspace_size", "ladder_ov3_abic",
    "ladder_metric_contraction_pairs", "ladder_mfma_probe",
    "ladder_mp2_amplitudes", "ladder_amplitude_update", "ladder_batched_workspace_size",
    "ladder_batched", "ladder_strerror", "ladder_last_error", "ladder_shutdown",
    "ladder_profile_start", "ladder_profile_stop", "ladder_gemm_workspace_size", "ladder_gemm",
    "ladder_forward_noalloc",
)

STAGE_NAMES = ("gemm_b", "gemm_c", "energy", "gemm_e", "gemm_f", "swap", "mp2", "update", "slice", "pack", "unpack",
               "metric", "back_transform", "ov3_permute", "ov3", "gemm")


class LadderError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__("%s (%d): %s" % (_strerror(code), code, message))
        self.code = code


class _COptions(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("n_slices", ctypes.c_int32), ("n_abatch", ctypes.c_int64),
                ("flags", ctypes.c_uint32), ("n_slices_adjoint", ctypes.c_int32)]


class _CStageStats(ctypes.Structure):
    _fields_ = [("stage", ctypes.c_int32), ("launches", ctypes.c_int32), ("total_ms", ctypes.c_double),
                ("flops", ctypes.c_double), ("bytes", ctypes.c_double)]


class _CInstance(ctypes.Structure):
    _fields_ = [("o", ctypes.c_int64), ("v", ctypes.c_int64), ("n", ctypes.c_int64),
                ("L", ctypes.c_void_p), ("tau", ctypes.c_void_p), ("tbar", ctypes.c_void_p),
                ("R", ctypes.c_void_p), ("E", ctypes.c_void_p), ("X", ctypes.c_void_p)]


@dataclass
class Options:
    precision: int = FP64
    n_slices: int = 0
    n_abatch: int = 0
    flags: int = 0
    n_slices_adjoint: int = 0

    def c(self) -> _COptions:
        return _COptions(self.precision, self.n_slices, self.n_abatch, self.flags, self.n_slices_adjoint)


_lib = None


def library_path() -> str:
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError("libladder.so is not built (%s); run __graft_entry__.build() or "
                           "python -m paper_2202_02019_amd.build" % _LIB_PATH)
    lib = ctypes.CDLL(_LIB_PATH)
    i64, vp, dbl, sz = ctypes.c_int64, ctypes.c_void_p, ctypes.c_double, ctypes.c_size_t
    op = ctypes.POINTER(_COptions)
    lib.ladder_default_options.argtypes = [op]
    lib.ladder_default_options.restype = None
    lib.ladder_workspace_size.argtypes = [i64, i64, i64, op, ctypes.POINTER(sz)]
    lib.ladder_forward.argtypes = [i64, i64, i64, vp, vp, vp, dbl, vp, vp, vp, sz, op, vp]
    lib.ladder_adjoint.argtypes = [i64, i64, i64, vp, vp, vp, dbl, dbl, vp, vp, sz, op, vp]
    lib.ladder_tau_gradient_workspace_size.argtypes = [i64, i64, i64, op, ctypes.POINTER(sz)]
    lib.ladder_tau_gradient.argtypes = [i64, i64, i64, vp, vp, dbl, vp, vp, sz, op, vp]
    lib.ladder_autotune.argtypes = [i64, i64, i64, vp, vp, vp, vp, vp, vp, sz, op, ctypes.c_char_p,
                                    ctypes.POINTER(i64), vp]
    lib.ladder_autotune_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_int)]
    lib.ladder_autotune_reset.argtypes = []
    lib.ladder_autotune_reset.restype = None
    lib.ladder_metric_contraction.argtypes = [i64, i64, vp, vp, dbl, dbl, vp, vp]
    lib.ladder_back_transform_workspace_size.argtypes = [i64, i64, ctypes.POINTER(sz)]
    lib.ladder_back_transform.argtypes = [i64, i64, vp, vp, vp, dbl, dbl, vp, vp, sz, vp]
    lib.ladder_excited_amplitudes.argtypes = [i64, i64, dbl, vp, vp, ctypes.c_int, vp, vp]
    lib.ladder_ov3_abci_workspace_size.argtypes = [i64, i64, i64, ctypes.POINTER(sz)]
    lib.ladder_ov3_abci.argtypes = [i64, i64, i64, vp, vp, vp, vp, dbl, dbl, vp, vp, vp, sz, vp]
    lib.ladder_metric_contraction_pairs.argtypes = [i64, i64, vp, vp, dbl, dbl, vp, vp]
    lib.ladder_mfma_probe.argtypes = [ctypes.c_int, i64, i64, vp, ctypes.POINTER(dbl), vp]
    lib.ladder_ov3_abic_workspace_size.argtypes = [i64, i64, i64, op, ctypes.POINTER(sz)]
    lib.ladder_ov3_abic.argtypes = [i64, i64, i64, dbl, vp, vp, vp, vp, vp, vp, vp, dbl, dbl, vp, vp, vp, sz, op, vp]
    lib.ladder_mp2_amplitudes.argtypes = [i64, i64, i64, vp, vp, vp, vp]
    lib.ladder_amplitude_update.argtypes = [i64, i64, vp, vp, vp, vp]
    lib.ladder_batched_workspace_size.argtypes = [ctypes.c_int, ctypes.POINTER(_CInstance), ctypes.c_uint32, op,
                                                  ctypes.POINTER(sz)]
    lib.ladder_batched.argtypes = [ctypes.c_int, ctypes.POINTER(_CInstance), ctypes.c_uint32, vp, sz, op, vp]
    lib.ladder_forward_noalloc.argtypes = [i64, i64, i64, vp, vp, vp, dbl, vp, vp, op, vp]
    lib.ladder_gemm_workspace_size.argtypes = [i64, i64, i64, op, ctypes.POINTER(sz)]
    lib.ladder_gemm.argtypes = [i64, i64, i64, dbl, vp, i64, vp, i64, dbl, vp, i64, vp, sz, op, vp]
    for f in ("ladder_forward_noalloc", "ladder_gemm_workspace_size", "ladder_gemm", "ladder_workspace_size", "ladder_forward", "ladder_adjoint", "ladder_tau_gradient_workspace_size",
              "ladder_tau_gradient", "ladder_autotune", "ladder_autotune_load", "ladder_metric_contraction",
              "ladder_back_transform_workspace_size",
              "ladder_back_transform", "ladder_excited_amplitudes", "ladder_ov3_abci_workspace_size",
              "ladder_ov3_abci", "ladder_ov3_abic_workspace_size", "ladder_ov3_abic", "ladder_metric_contraction_pairs",
              "ladder_mp2_amplitudes", "ladder_mfma_probe",
              "ladder_amplitude_update", "ladder_batched_workspace_size", "ladder_batched"):
        getattr(lib, f).restype = ctypes.c_int
    lib.ladder_strerror.argtypes = [ctypes.c_int]
    lib.ladder_strerror.restype = ctypes.c_char_p
    lib.ladder_last_error.argtypes = []
    lib.ladder_last_error.restype = ctypes.c_char_p
    lib.ladder_shutdown.argtypes = []
    lib.ladder_shutdown.restype = None
    lib.ladder_profile_start.argtypes = []
    lib.ladder_profile_start.restype = ctypes.c_int
    lib.ladder_profile_stop.argtypes = [ctypes.POINTER(_CStageStats), ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    lib.ladder_profile_stop.restype = ctypes.c_int
    _lib = lib
    return lib


def exported_symbols():
    """Loads the library and returns the C entry points (no GPU call is made)."""
    lib = _load()
    return {name: getattr(lib, name) for name in EXPORTS}


def _strerror(code: int) -> str:
    try:
        return _load().ladder_strerror(code).decode()
    except Exception:  # pragma: no cover
        return "error"


def _check(rc: int):
    if rc != 0:
        raise LadderError(rc, _load().ladder_last_error().decode())


def _opts(opts) -> _COptions:
    if opts is None:
        return Options().c()
    if isinstance(opts, _COptions):
        return opts
    return opts.c()


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _need(t, name, shape=None):
    if t is None:
        raise ValueError("%s is required" % name)
    if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError("%s must be a contiguous float64 tensor on the GPU" % name)
    if shape is not None and t.numel() != int(torch.Size(shape).numel()):
        raise ValueError("%s has %d elements, %s expected" % (name, t.numel(), tuple(shape)))
    return t


def workspace_size(o: int, v: int, n: int, opts=None) -> int:
    b = ctypes.c_size_t(0)
    _check(_load().ladder_workspace_size(o, v, n, ctypes.byref(_opts(opts)), ctypes.byref(b)))
    return b.value


def _workspace(nbytes, device, ws):
    if ws is not None:
        if ws.numel() * ws.element_size() < nbytes:
            raise ValueError("workspace too small: %d < %d bytes" % (ws.numel() * ws.element_size(), nbytes))
        return ws
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)


def forward(L, tau, tbar=None, *, o, v, n, R=None, E=None, beta=0.0, want_energy=True, ws=None, opts=None,
            stream=None):
    """R = beta*R + ladder(L, tau); E = sum tbar*ladder (if tbar given).  Returns (R, E or None)."""
    _need(L, "L", (v, v, n)); _need(tau, "tau", (o, o, v, v))
    if tbar is not None:
        _need(tbar, "tbar", (o, o, v, v))
    dev = L.device
    if R is None:
        R = torch.empty((o, o, v, v), dtype=torch.float64, device=dev)
    _need(R, "R", (o, o, v, v))
    if want_energy and tbar is not None and E is None:
        E = torch.empty((), dtype=torch.float64, device=dev)
    if not want_energy or tbar is None:
        E = None
    c = _opts(opts)
    w = _workspace(workspace_size(o, v, n, c), dev, ws)
    _check(_load().ladder_forward(o, v, n, _ptr(L), _ptr(tau), _ptr(tbar), float(beta), _ptr(R), _ptr(E), _ptr(w),
                                  w.numel() * w.element_size(), ctypes.byref(c), _stream(stream)))
    return R, E


def forward_noalloc(L, tau, tbar=None, *, o, v, n, R, E=None, beta=0.0, opts=None, stream=None):
    """ladder_forward_noalloc: forward() on the library's static device scratch; R (and E, if the
    energy is wanted) must be given, so that nothing is allocated here either."""
    _need(L, "L", (v, v, n)); _need(tau, "tau", (o, o, v, v)); _need(R, "R", (o, o, v, v))
    if tbar is not None:
        _need(tbar, "tbar", (o, o, v, v))
    if E is not None and (not E.is_cuda or E.dtype != torch.float64 or E.numel() != 1):
        raise ValueError("E must be a one-element float64 tensor on the GPU")
    c = _opts(opts)
    _check(_load().ladder_forward_noalloc(o, v, n, _ptr(L), _ptr(tau), _ptr(tbar), float(beta), _ptr(R), _ptr(E),
                                          ctypes.byref(c), _stream(stream)))
    return R, E


def adjoint(L, tau, w, *, o, v, n, X=None, alpha=1.0, beta=0.0, ws=None, opts=None, stream=None):
    """X = beta*X + alpha * d/dL sum(w * ladder(L, tau))."""
    _need(L, "L", (v, v, n)); _need(tau, "tau", (o, o, v, v)); _need(w, "w", (o, o, v, v))
    if X is None:
        X = torch.empty((v, v, n), dtype=torch.float64, device=L.device)
    _need(X, "X", (v, v, n))
    c = _opts(opts)
    wsb = _workspace(workspace_size(o, v, n, c), L.device, ws)
    _check(_load().ladder_adjoint(o, v, n, _ptr(L), _ptr(tau), _ptr(w), float(alpha), float(beta), _ptr(X), _ptr(wsb),
                                  wsb.numel() * wsb.element_size(), ctypes.byref(c), _stream(stream)))
    return X


def gemm_workspace_size(M: int, N: int, K: int, opts=None) -> int:
    b = ctypes.c_size_t(0)
    _check(_load().ladder_gemm_workspace_size(M, N, K, ctypes.byref(_opts(opts)), ctypes.byref(b)))
    return b.value


def gemm(A, B, *, C=None, alpha=1.0, beta=0.0, ws=None, opts=None, stream=None):
    """C = beta*C + alpha * A @ B.T for 2-D float64 tensors A [M][K], B [N][K] (ladder_gemm)."""
    if A.dim() != 2 or B.dim() != 2 or A.shape[1] != B.shape[1]:
        raise ValueError("A [M][K] and B [N][K] expected")
    M, K = A.shape
    N = B.shape[0]
    _need(A, "A"); _need(B, "B")
    if C is None:
        C = torch.empty((M, N), dtype=torch.float64, device=A.device)
    _need(C, "C", (M, N))
    c = _opts(opts)
    nb = gemm_workspace_size(M, N, K, c)
    w = _workspace(nb, A.device, ws) if nb else ws
    _check(_load().ladder_gemm(M, N, K, float(alpha), _ptr(A), K, _ptr(B), K, float(beta), _ptr(C), N, _ptr(w),
                               0 if w is None else w.numel() * w.element_size(), ctypes.byref(c), _stream(stream)))
    return C


def tau_gradient_workspace_size(o: int, v: int, n: int, opts=None) -> int:
    b = ctypes.c_size_t(0)
    _check(_load().ladder_tau_gradient_workspace_size(o, v, n, ctypes.byref(_opts(opts)), ctypes.byref(b)))
    return b.value


def tau_gradient(L, w, *, o, v, n, G=None, beta=0.0, ws=None, opts=None, stream=None):
    """G = beta*G + d/dtau sum(w * ladder(L, tau)) = sum_ab w_ij^ab (ac|bd) (the transposed ladder)."""
    _need(L, "L", (v, v, n)); _need(w, "w", (o, o, v, v))
    if G is None:
        G = torch.empty((o, o, v, v), dtype=torch.float64, device=L.device)
    _need(G, "G", (o, o, v, v))
    c = _opts(opts)
    wsb = _workspace(tau_gradient_workspace_size(o, v, n, c), L.device, ws)
    _check(_load().ladder_tau_gradient(o, v, n, _ptr(L), _ptr(w), float(beta), _ptr(G), _ptr(wsb),
                                       wsb.numel() * wsb.element_size(), ctypes.byref(c), _stream(stream)))
    return G


def autotune(L, tau, tbar, *, o, v, n, ws, R=None, X=None, opts=None, cache_path=None, stream=None):
    """Times candidate virtual-batch sizes within the workspace `ws` and keeps the fastest for later
    calls with n_abatch = 0 (ladder_autotune).  Returns the chosen batch size.  R and X (allocated if
    None) receive partial results."""
    _need(L, "L", (v, v, n)); _need(tau, "tau", (o, o, v, v)); _need(tbar, "tbar", (o, o, v, v))
    if R is None:
        R = torch.empty((o, o, v, v), dtype=torch.float64, device=L.device)
    if X is None:
        X = torch.empty((v, v, n), dtype=torch.float64, device=L.device)
    c = _opts(opts)
    nA = ctypes.c_int64(0)
    path = None if cache_path is None else os.fsencode(cache_path)
    _check(_load().ladder_autotune(o, v, n, _ptr(L), _ptr(tau), _ptr(tbar), _ptr(R), _ptr(X), _ptr(ws),
                                   ws.numel() * ws.element_size(), ctypes.byref(c), path, ctypes.byref(nA),
                                   _stream(stream)))
    return nA.value


def autotune_load(cache_path) -> int:
    """Loads tuned batch sizes of this device from a JSON-lines file; returns the number taken."""
    k = ctypes.c_int(0)
    _check(_load().ladder_autotune_load(os.fsencode(cache_path), ctypes.byref(k)))
    return k.value


def autotune_reset() -> None:
    _load().ladder_autotune_reset()


def w_intermediate(Z, tau, tbar, *, o, v, n, W=None, beta=0.0, ws=None, opts=None, stream=None):
    """W^K_ac = sum_bd d_acbd Z^K_bd (the V^4 block of the density intermediate): ladder_adjoint
    with Z in place of L and alpha = 1/2."""
    return adjoint(Z, tau, tbar, o=o, v=v, n=n, X=W, alpha=0.5, beta=beta, ws=ws, opts=opts, stream=stream)


def metric_contraction(Z, W, *, v, n, V=None, alpha=1.0, beta=0.0, stream=None):
    """V_MN = beta*V + alpha * sum_pq Z^M_pq W^N_pq  ([n][n])."""
    _need(Z, "Z", (v, v, n)); _need(W, "W", (v, v, n))
    if V is None:
        V = torch.empty((n, n), dtype=torch.float64, device=Z.device)
    _need(V, "V", (n, n))
    _check(_load().ladder_metric_contraction(v, n, _ptr(Z), _ptr(W), float(alpha), float(beta), _ptr(V),
                                             _stream(stream)))
    return V


def back_transform_workspace_size(v: int, n: int) -> int:
    b = ctypes.c_size_t(0)
    _check(_load().ladder_back_transform_workspace_size(v, n, ctypes.byref(b)))
    return b.value


def back_transform(x, y, W, *, v, n, Wmo=None, alpha=1.0, beta=0.0, ws=None, stream=None):
    """Wmo^K_pq = beta*Wmo + alpha * sum_rs x_rp y_sq W^K_rs  (x, y: [v][v]; W, Wmo: [v][v][n])."""
    _need(x, "x", (v, v)); _need(y, "y", (v, v)); _need(W, "W", (v, v, n))
    if Wmo is None:
        Wmo = torch.empty((v, v, n), dtype=torch.float64, device=W.device)
    _need(Wmo, "Wmo", (v, v, n))
    wsb = _workspace(back_transform_workspace_size(v, n), W.device, ws)
    _check(_load().ladder_back_transform(v, n, _ptr(x), _ptr(y), _ptr(W), float(alpha), float(beta), _ptr(Wmo),
                                         _ptr(wsb), wsb.numel() * wsb.element_size(), _stream(stream)))
    return Wmo


def excited_amplitudes(T, R2, R0, *, o, v, mode=U_APPENDIX, U=None, stream=None):
    """U for the excited-state V^4 density: U_TABLE: R0 T + R2; U_APPENDIX: R0 T / 2 + R~2, where
    R~2 is R2 with its diagonal elements (i = j, a = b) doubled."""
    _need(T, "T", (o, o, v, v)); _need(R2, "R2", (o, o, v, v))
    if U is None:
        U = torch.empty((o, o, v, v), dtype=torch.float64, device=T.device)
    _need(U, "U", (o, o, v, v))
    _check(_load().ladder_excited_amplitudes(o, v, float(R0), _ptr(T), _ptr(R2), int(mode), _ptr(U), _stream(stream)))
    return U


def ov3_abci_workspace_size(o: int, v: int, n: int) -> int:
    b = ctypes.c_size_t(0)
    _check(_load().ladder_ov3_abci_workspace_size(o, v, n, ctypes.byref(b)))
    return b.value


def ov3_abci(L2, R1, Zvv, Zvo, *, o, v, n, Wab=None, Wci=None, alpha=1.0, beta=0.0, want=(True, True), ws=None,
             stream=None):
    """Both W contributions of the excited-state OV^3 density d_abci = sum_j L_ji^ac R_j^b:
    Wab [v][v][n] (from Zvo [v][o][n]) and Wci [v][o][n] (from Zvv [v][v][n]), each
    beta*W + alpha*W'.  `want` = (ab side, ci side); a side not wanted is returned as None."""
    want_ab, want_ci = bool(want[0]), bool(want[1])
    _need(L2, "L2", (o, o, v, v)); _need(R1, "R1", (o, v))
    if want_ab:
        _need(Zvo, "Zvo", (v, o, n))
        if Wab is None:
            Wab = torch.empty((v, v, n), dtype=torch.float64, device=L2.device)
        _need(Wab, "Wab", (v, v, n))
    if want_ci:
        _need(Zvv, "Zvv", (v, v, n))
        if Wci is None:
            Wci = torch.empty((v, o, n), dtype=torch.float64, device=L2.device)
        _need(Wci, "Wci", (v, o, n))
    wsb = _workspace(ov3_abci_workspace_size(o, v, n), L2.device, ws)
    _check(_load().ladder_ov3_abci(o, v, n, _ptr(L2), _ptr(R1), _ptr(Zvv) if want_ci else None,
                                   _ptr(Zvo) if want_ab else None, float(alpha), float(beta),
                                   _ptr(Wab) if want_ab else None, _ptr(Wci) if want_ci else None, _ptr(wsb),
                                   wsb.numel() * wsb.element_size(), _stream(stream)))
    return (Wab if want_ab else None), (Wci if want_ci else None)


def ov3_abic_workspace_size(o: int, v: int, n: int, opts=None) -> int:
    b = ctypes.c_size_t(0)
    co = _opts(opts)
    _check(_load().ladder_ov3_abic_workspace_size(o, v, n, ctypes.byref(co), ctypes.byref(b)))
    return b.value


def ov3_abic(R0, L1, L2, T, R1, R2, Zvv, Zov, *, o, v, n, Wab=None, Wic=None, alpha=1.0, beta=0.0, want=(True, True),
             ws=None, opts=None, stream=None):
    """Both W contributions of the excited-state OV^3 density d_abic: Wab [v][v][n] (from
    Zov [o][v][n]) and Wic [o][v][n] (from Zvv [v][v][n]), each beta*W + alpha*W'.
    L1, R1: [o][v]; L2, T, R2: [o][o][v][v]; R0 a float.  `want` = (ab side, ic side);
    opts.precision picks FP64 or split BF16 for the o^3 v^3 products."""
    want_ab, want_ic = bool(want[0]), bool(want[1])
    _need(L1, "L1", (o, v)); _need(R1, "R1", (o, v))
    for t, name in ((L2, "L2"), (T, "T"), (R2, "R2")):
        _need(t, name, (o, o, v, v))
    if want_ab:
        _need(Zov, "Zov", (o, v, n))
        if Wab is None:
            Wab = torch.empty((v, v, n), dtype=torch.float64, device=L2.device)
        _need(Wab, "Wab", (v, v, n))
    if want_ic:
        _need(Zvv, "Zvv", (v, v, n))
        if Wic is None:
            Wic = torch.empty((o, v, n), dtype=torch.float64, device=L2.device)
        _need(Wic, "Wic", (o, v, n))
    co = _opts(opts)
    wsb = _workspace(ov3_abic_workspace_size(o, v, n, co), L2.device, ws)
    _check(_load().ladder_ov3_abic(o, v, n, float(R0), _ptr(L1), _ptr(L2), _ptr(T), _ptr(R1), _ptr(R2),
                                   _ptr(Zvv) if want_ic else None, _ptr(Zov) if want_ab else None, float(alpha),
                                   float(beta), _ptr(Wab) if want_ab else None, _ptr(Wic) if want_ic else None,
                                   _ptr(wsb), wsb.numel() * wsb.element_size(), ctypes.byref(co), _stream(stream)))
    return (Wab if want_ab else None), (Wic if want_ic else None)


def metric_contraction_pairs(Z, W, *, pairs, n, V=None, alpha=1.0, beta=0.0, stream=None):
    """V_MN = beta*V + alpha * sum_p Z[p][M] W[p][N] over `pairs` index pairs  (Z, W: [pairs][n])."""
    _need(Z, "Z", (pairs, n)); _need(W, "W", (pairs, n))
    if V is None:
        V = torch.empty((n, n), dtype=torch.float64, device=Z.device)
    _need(V, "V", (n, n))
    _check(_load().ladder_metric_contraction_pairs(pairs, n, _ptr(Z), _ptr(W), float(alpha), float(beta), _ptr(V),
                                                   _stream(stream)))
    return V


PROBE_BF16 = 0
PROBE_FP64 = 1
PROBE_INT8 = 2


def mfma_probe(kind, iters, blocks, out=None, stream=None):
    """Launches the matrix-core ceiling probe; returns (out [blocks*256] checksums, flops)."""
    if out is None:
        out = torch.empty((blocks * 256,), dtype=torch.float64, device="cuda")
    _need(out, "out", (blocks * 256,))
    fl = ctypes.c_double(0.0)
    _check(_load().ladder_mfma_probe(int(kind), int(iters), int(blocks), _ptr(out), ctypes.byref(fl),
                                     _stream(stream)))
    return out, fl.value


def mp2_amplitudes(Lov, eps, *, o, v, n, t=None, stream=None):
    _need(Lov, "Lov", (o, v, n)); _need(eps, "eps", (o + v,))
    if t is None:
        t = torch.empty((o, o, v, v), dtype=torch.float64, device=Lov.device)
    _need(t, "t", (o, o, v, v))
    _check(_load().ladder_mp2_amplitudes(o, v, n, _ptr(Lov), _ptr(eps), _ptr(t), _stream(stream)))
    return t


def amplitude_update(eps, R, t, *, o, v, stream=None):
    """In place: t += R / ((eps_i+eps_j) - (eps_a+eps_b))."""
    _need(eps, "eps", (o + v,)); _need(R, "R", (o, o, v, v)); _need(t, "t", (o, o, v, v))
    _check(_load().ladder_amplitude_update(o, v, _ptr(eps), _ptr(R), _ptr(t), _stream(stream)))
    return t


def _instances(insts):
    arr = (_CInstance * len(insts))()
    for k, d in enumerate(insts):
        arr[k] = _CInstance(d["o"], d["v"], d["n"], d["L"].data_ptr(), d["tau"].data_ptr(),
                            d["tbar"].data_ptr() if d.get("tbar") is not None else None,
                            d["R"].data_ptr() if d.get("R") is not None else None,
                            d["E"].data_ptr() if d.get("E") is not None else None,
                            d["X"].data_ptr() if d.get("X") is not None else None)
    return arr


def batched_workspace_size(insts, what=DO_FORWARD | DO_ADJOINT, opts=None) -> int:
    arr = _instances(insts)
    b = ctypes.c_size_t(0)
    _check(_load().ladder_batched_workspace_size(len(insts), arr, what, ctypes.byref(_opts(opts)), ctypes.byref(b)))
    return b.value


def batched(insts, what=DO_FORWARD | DO_ADJOINT, *, ws=None, opts=None, stream=None):
    """insts: list of dicts with o, v, n, L, tau, tbar, R, E, X (device tensors)."""
    arr = _instances(insts)
    c = _opts(opts)
    b = ctypes.c_size_t(0)
    _check(_load().ladder_batched_workspace_size(len(insts), arr, what, ctypes.byref(c), ctypes.byref(b)))
    dev = insts[0]["L"].device
    w = _workspace(b.value, dev, ws)
    _check(_load().ladder_batched(len(insts), arr, what, _ptr(w), w.numel() * w.element_size(), ctypes.byref(c),
                                  _stream(stream)))


def profile_start():
    """Start bracketing every library launch with HIP events on its stream."""
    _check(_load().ladder_profile_start())


def profile_stop():
    """Stop recording; returns {stage name: dict(launches, total_ms, avg_ms, flops, bytes)}."""
    arr = (_CStageStats * 16)()
    k = ctypes.c_int(0)
    _check(_load().ladder_profile_stop(arr, 16, ctypes.byref(k)))
    out = {}
    for i in range(k.value):
        s = arr[i]
        out[STAGE_NAMES[s.stage]] = dict(launches=s.launches, total_ms=s.total_ms,
                                         avg_ms=s.total_ms / max(1, s.launches), flops=s.flops, bytes=s.bytes)
    return out


class LadderEnergy(torch.autograd.Function):
    """E(L, tau, tbar) = sum tbar * ladder(L, tau) with the library adjoint as backward.

    backward gives dE/dL = X (hand-written adjoint, g recomputed per batch, nothing
    of the forward kept but the inputs), dE/dtau = the transposed ladder of tbar and
    dE/dtbar = R.  With the default options the inputs must be pair-symmetric (the
    +/- packed path); pass Options(flags=FLAG_GENERAL) otherwise.
    """

    @staticmethod
    def forward(ctx, L, tau, tbar, dims, opts=None):
        o, v, n = dims
        R, E = forward(L, tau, tbar, o=o, v=v, n=n, opts=opts)
        ctx.dims, ctx.opts = dims, opts
        ctx.save_for_backward(L, tau, tbar, R if tbar.requires_grad else None)
        return E

    @staticmethod
    def backward(ctx, gE):
        L, tau, tbar, R = ctx.saved_tensors
        o, v, n = ctx.dims
        gL = gtau = gt = None
        if ctx.needs_input_grad[1]:
            gtau = tau_gradient(L, tbar, o=o, v=v, n=n, opts=ctx.opts)
            gtau.mul_(gE)
        if ctx.needs_input_grad[0]:
            # the incoming gradient is the adjoint's alpha: X = gE * dE/dL in one pass
            gL = adjoint(L, tau, tbar, o=o, v=v, n=n, alpha=float(gE), opts=ctx.opts)
        if ctx.needs_input_grad[2]:
            gt = R * gE
        return gL, gtau, gt, None, None


def ladder_energy(L, tau, tbar, dims, opts=None):
    return LadderEnergy.apply(L, tau, tbar, tuple(dims), opts)
