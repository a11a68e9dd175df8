"""ctypes binding of the C oracle in ladder_oracle.c plus the oracle-side input recipe.

See ladder_oracle.c for the definitions and their citations.  ``build()`` compiles
the C file with gcc (-O2, OpenMP, strict IEEE: no -ffast-math).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time

import numpy as np

import synthetic

from . import matrix

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ladder_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

__all__ = [
    "build", "load", "forward", "adjoint", "forward_range", "adjoint_range", "R_sample",
    "X_sample", "tau_gradient", "tau_gradient_range", "w_intermediate", "w_intermediate_range",
    "metric_contraction", "metric_contraction_pairs", "back_transform", "back_transform_range",
    "excited_amplitudes", "ov3_abci", "ov3_abci_wab", "ov3_abci_wci", "ov3_abic", "mp2_amplitudes", "amplitude_update", "make_inputs",
    "num_threads",
    "set_num_threads", "flops_forward", "flops_adjoint", "matrix",
]

_lib = None


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc; returns the path."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-march=x86-64-v3", "-ffp-contract=off", "-fno-fast-math",
               "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall", "-Wextra", "-o", tmp, SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        lib = ctypes.CDLL(LIB)
        i64, dp, vp = ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p
        lib.oracle_ladder_forward_range.argtypes = [i64, i64, i64, dp, dp, dp, i64, i64, dp, dp, dp]
        lib.oracle_ladder_adjoint_range.argtypes = [i64, i64, i64, dp, dp, dp, i64, i64, dp]
        lib.oracle_ladder_R_sample.argtypes = [i64, i64, i64, dp, dp, i64, vp, dp]
        lib.oracle_ladder_X_sample.argtypes = [i64, i64, i64, dp, dp, dp, i64, vp, dp]
        lib.oracle_ladder_tau_gradient_range.argtypes = [i64, i64, i64, dp, dp, i64, i64, dp]
        lib.oracle_w_intermediate_range.argtypes = [i64, i64, i64, dp, dp, dp, i64, i64, dp]
        lib.oracle_metric_contraction.argtypes = [i64, i64, dp, dp, dp]
        lib.oracle_excited_amplitudes.argtypes = [i64, i64, ctypes.c_double, dp, dp, ctypes.c_int, dp]
        lib.oracle_back_transform_range.argtypes = [i64, i64, dp, dp, dp, i64, i64, dp]
        lib.oracle_ov3_abci_wab.argtypes = [i64, i64, i64, dp, dp, dp, i64, vp, dp]
        lib.oracle_ov3_abci_wci.argtypes = [i64, i64, i64, dp, dp, dp, i64, vp, dp]
        lib.oracle_metric_contraction_pairs.argtypes = [i64, i64, dp, dp, dp]
        lib.oracle_ov3_abic.argtypes = [i64, i64, i64, ctypes.c_double, dp, dp, dp, dp, dp, dp, dp, dp, dp]
        lib.oracle_mp2_amplitudes.argtypes = [i64, i64, i64, dp, dp, dp]
        lib.oracle_amplitude_update.argtypes = [i64, i64, dp, dp, dp]
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
        for f in ("oracle_ladder_forward_range", "oracle_ladder_adjoint_range", "oracle_ladder_R_sample",
                  "oracle_ladder_X_sample", "oracle_ladder_tau_gradient_range", "oracle_w_intermediate_range",
                  "oracle_metric_contraction", "oracle_back_transform_range", "oracle_excited_amplitudes",
                  "oracle_ov3_abci_wab", "oracle_ov3_abci_wci", "oracle_metric_contraction_pairs", "oracle_ov3_abic",
                  "oracle_mp2_amplitudes",
                  "oracle_amplitude_update"):
            getattr(lib, f).restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.size != int(np.prod(shape)):
        raise ValueError("array of size %d where %s was expected" % (a.size, shape))
    return a


def num_threads() -> int:
    return int(load().oracle_num_threads())


def set_num_threads(t: int) -> None:
    load().oracle_set_num_threads(int(t))


def forward_range(o, v, n, L, tau, tbar, a_lo, a_hi, R=None):
    """R rows a in [a_lo,a_hi) (other rows of R untouched), per-a energies and their sum."""
    L = _f64(L, (v, v, n)); tau = _f64(tau, (o, o, v, v))
    tbar = None if tbar is None else _f64(tbar, (o, o, v, v))
    if R is None:
        R = np.zeros((o, o, v, v))
    Ep = np.zeros(max(1, a_hi - a_lo)); E = np.zeros(1)
    rc = load().oracle_ladder_forward_range(o, v, n, _p(L), _p(tau), _p(tbar), a_lo, a_hi, _p(R), _p(Ep), _p(E))
    if rc != 0:
        raise RuntimeError("oracle_ladder_forward_range failed")
    return R, Ep[: a_hi - a_lo], float(E[0])


def forward(o, v, n, L, tau, tbar=None):
    """Returns (R [o][o][v][v], E) with E = sum tbar*R (0.0 if tbar is None)."""
    R, _, E = forward_range(o, v, n, L, tau, tbar, 0, v)
    return R, E


def adjoint_range(o, v, n, L, tau, w, p_lo, p_hi, X=None):
    L = _f64(L, (v, v, n)); tau = _f64(tau, (o, o, v, v)); w = _f64(w, (o, o, v, v))
    if X is None:
        X = np.zeros((v, v, n))
    rc = load().oracle_ladder_adjoint_range(o, v, n, _p(L), _p(tau), _p(w), p_lo, p_hi, _p(X))
    if rc != 0:
        raise RuntimeError("oracle_ladder_adjoint_range failed")
    return X


def adjoint(o, v, n, L, tau, w):
    """X [v][v][n] = dE/dL with E = sum w * R(L, tau), general (no symmetry assumed)."""
    return adjoint_range(o, v, n, L, tau, w, 0, v)


def tau_gradient_range(o, v, n, L, w, c_lo, c_hi, G=None):
    """G_ij^cd = sum_ab w_ij^ab (ac|bd) for rows c in [c_lo, c_hi) (others untouched)."""
    L = _f64(L, (v, v, n)); w = _f64(w, (o, o, v, v))
    if G is None:
        G = np.zeros((o, o, v, v))
    rc = load().oracle_ladder_tau_gradient_range(o, v, n, _p(L), _p(w), c_lo, c_hi, _p(G))
    if rc != 0:
        raise RuntimeError("oracle_ladder_tau_gradient_range failed")
    return G


def tau_gradient(o, v, n, L, w):
    """G [o][o][v][v] = dE/dtau with E = sum w * R(L, tau) (the transposed ladder), general L."""
    return tau_gradient_range(o, v, n, L, w, 0, v)


def w_intermediate_range(o, v, n, Z, tau, w, p_lo, p_hi, W=None):
    """W^K_pq = sum_rs d_pqrs Z^K_rs (d_pqrs = sum_ij w_ij^pr tau_ij^qs) for rows p in [p_lo, p_hi)."""
    Z = _f64(Z, (v, v, n)); tau = _f64(tau, (o, o, v, v)); w = _f64(w, (o, o, v, v))
    if W is None:
        W = np.zeros((v, v, n))
    rc = load().oracle_w_intermediate_range(o, v, n, _p(Z), _p(tau), _p(w), p_lo, p_hi, _p(W))
    if rc != 0:
        raise RuntimeError("oracle_w_intermediate_range failed")
    return W


def w_intermediate(o, v, n, Z, tau, w):
    return w_intermediate_range(o, v, n, Z, tau, w, 0, v)


def metric_contraction(v, n, Z, W):
    """V [n][n], V_MN = sum_pq Z^M_pq W^N_pq."""
    Z = _f64(Z, (v, v, n)); W = _f64(W, (v, v, n))
    V = np.zeros((n, n))
    if load().oracle_metric_contraction(v, n, _p(Z), _p(W), _p(V)) != 0:
        raise RuntimeError("oracle_metric_contraction failed")
    return V


def back_transform_range(v, n, x, y, W, K_lo, K_hi, Wmo=None):
    """Wmo^K_pq = sum_rs x_rp y_sq W^K_rs for K in [K_lo, K_hi)."""
    x = _f64(x, (v, v)); y = _f64(y, (v, v)); W = _f64(W, (v, v, n))
    if Wmo is None:
        Wmo = np.zeros((v, v, n))
    if load().oracle_back_transform_range(v, n, _p(x), _p(y), _p(W), K_lo, K_hi, _p(Wmo)) != 0:
        raise RuntimeError("oracle_back_transform_range failed")
    return Wmo


def back_transform(v, n, x, y, W):
    return back_transform_range(v, n, x, y, W, 0, n)


def excited_amplitudes(o, v, R0, T, R2, mode):
    """U for the excited-state V^4 density (mode 0: R0 T + R2; mode 1: R0 T/2 + R~2, R~2 = R2 with its i=j, a=b elements doubled)."""
    T = _f64(T, (o, o, v, v)); R2 = _f64(R2, (o, o, v, v))
    U = np.zeros((o, o, v, v))
    if load().oracle_excited_amplitudes(o, v, float(R0), _p(T), _p(R2), int(mode), _p(U)) != 0:
        raise RuntimeError("oracle_excited_amplitudes failed")
    return U


def metric_contraction_pairs(pairs, n, Z, W):
    """V [n][n], V_MN = sum_p Z^M_p W^N_p over `pairs` index pairs (Z, W: [pairs][n])."""
    Z = _f64(Z, (pairs, n)); W = _f64(W, (pairs, n))
    V = np.zeros((n, n))
    if load().oracle_metric_contraction_pairs(pairs, n, _p(Z), _p(W), _p(V)) != 0:
        raise RuntimeError("oracle_metric_contraction_pairs failed")
    return V


def _pairs(idx):
    idx = np.ascontiguousarray(idx, dtype=np.int64).reshape(-1, 2)
    return idx, (idx.ctypes.data if idx.shape[0] else None)


def ov3_abci_wab(o, v, n, L2, R1, Zvo, ab):
    """Wab^K_ab = sum_ci d_abci Z^K_ci (d_abci = sum_j L_ji^ac R_j^b) for pairs ab (k x 2): [k][n]."""
    L2 = _f64(L2, (o, o, v, v)); R1 = _f64(R1, (o, v)); Zvo = _f64(Zvo, (v, o, n))
    ab, pab = _pairs(ab)
    out = np.zeros((ab.shape[0], n))
    if load().oracle_ov3_abci_wab(o, v, n, _p(L2), _p(R1), _p(Zvo), ab.shape[0], pab, _p(out)) != 0:
        raise RuntimeError("oracle_ov3_abci_wab failed")
    return out


def ov3_abci_wci(o, v, n, L2, R1, Zvv, ci):
    """Wci^K_ci = sum_ab d_abci Z^K_ab for pairs ci (k x 2, c virtual, i occupied): [k][n]."""
    L2 = _f64(L2, (o, o, v, v)); R1 = _f64(R1, (o, v)); Zvv = _f64(Zvv, (v, v, n))
    ci, pci = _pairs(ci)
    out = np.zeros((ci.shape[0], n))
    if load().oracle_ov3_abci_wci(o, v, n, _p(L2), _p(R1), _p(Zvv), ci.shape[0], pci, _p(out)) != 0:
        raise RuntimeError("oracle_ov3_abci_wci failed")
    return out


def ov3_abci(o, v, n, L2, R1, Zvv, Zvo):
    """(Wab [v][v][n], Wci [v][o][n]): both contributions of the OV^3 block d_abci, in full."""
    ab = np.array([(a, b) for a in range(v) for b in range(v)], dtype=np.int64)
    ci = np.array([(c, i) for c in range(v) for i in range(o)], dtype=np.int64)
    return (ov3_abci_wab(o, v, n, L2, R1, Zvo, ab).reshape(v, v, n),
            ov3_abci_wci(o, v, n, L2, R1, Zvv, ci).reshape(v, o, n))


def ov3_abic(o, v, n, R0, L1, L2, T, R1, R2, Zvv, Zov):
    """(Wab [v][v][n], Wic [o][v][n]): both contributions of the excited-state OV^3 block d_abic."""
    L1 = _f64(L1, (o, v)); R1 = _f64(R1, (o, v))
    L2 = _f64(L2, (o, o, v, v)); T = _f64(T, (o, o, v, v)); R2 = _f64(R2, (o, o, v, v))
    Zvv = _f64(Zvv, (v, v, n)); Zov = _f64(Zov, (o, v, n))
    Wab, Wic = np.zeros((v, v, n)), np.zeros((o, v, n))
    if load().oracle_ov3_abic(o, v, n, float(R0), _p(L1), _p(L2), _p(T), _p(R1), _p(R2), _p(Zvv), _p(Zov),
                              _p(Wab), _p(Wic)) != 0:
        raise RuntimeError("oracle_ov3_abic failed")
    return Wab, Wic


def R_sample(o, v, n, L, tau, ab):
    """R_ij^ab for pairs ab (k x 2 int array): returns [k][o*o]."""
    L = _f64(L, (v, v, n)); tau = _f64(tau, (o, o, v, v))
    ab = np.ascontiguousarray(ab, dtype=np.int64).reshape(-1, 2)
    out = np.zeros((ab.shape[0], o * o))
    if load().oracle_ladder_R_sample(o, v, n, _p(L), _p(tau), ab.shape[0], _p(ab), _p(out)) != 0:
        raise RuntimeError("oracle_ladder_R_sample failed")
    return out


def X_sample(o, v, n, L, tau, w, pq):
    """X^J_pq for pairs pq (k x 2): returns [k][n]."""
    L = _f64(L, (v, v, n)); tau = _f64(tau, (o, o, v, v)); w = _f64(w, (o, o, v, v))
    pq = np.ascontiguousarray(pq, dtype=np.int64).reshape(-1, 2)
    out = np.zeros((pq.shape[0], n))
    if load().oracle_ladder_X_sample(o, v, n, _p(L), _p(tau), _p(w), pq.shape[0], _p(pq), _p(out)) != 0:
        raise RuntimeError("oracle_ladder_X_sample failed")
    return out


def mp2_amplitudes(o, v, n, Lov, eps):
    Lov = _f64(Lov, (o, v, n)); eps = _f64(eps, (o + v,))
    t = np.empty((o, o, v, v))
    if load().oracle_mp2_amplitudes(o, v, n, _p(Lov), _p(eps), _p(t)) != 0:
        raise RuntimeError("oracle_mp2_amplitudes failed")
    return t


def amplitude_update(o, v, eps, R, t):
    """Returns a new array t + R/(eps_i+eps_j-eps_a-eps_b)."""
    eps = _f64(eps, (o + v,)); R = _f64(R, (o, o, v, v)); t = np.array(t, dtype=np.float64, copy=True)
    if load().oracle_amplitude_update(o, v, _p(eps), _p(R), _p(t)) != 0:
        raise RuntimeError("oracle_amplitude_update failed")
    return t


def make_inputs(o, v, n, seed, decay=0.0):
    """The oracle-side inputs of the synthetic recipe: (L_vv, tau, tbar, L_ov, eps).

    tau = t with t the first-order amplitudes built by the oracle from the draws,
    tbar = t + 1e-2 * xi with the pair-symmetric noise xi; decay > 0 scales the
    Cholesky vectors by exp(-decay * J / n) first (the stress variant).
    """
    Lvv = synthetic.draw_L_vv(seed, o, v, n)
    Lov = synthetic.draw_L_ov(seed, o, v, n)
    if decay:
        f = synthetic.decay_factors(n, decay)
        Lvv, Lov = Lvv * f, Lov * f
    eps = synthetic.draw_eps(seed, o, v)
    t = mp2_amplitudes(o, v, n, Lov, eps)
    tbar = t + synthetic.NOISE_SCALE * synthetic.draw_noise_full(seed, o, v)
    return Lvv, t, tbar, Lov, eps


def flops_forward(o, v, n):
    """Algorithmic dense flops of g (2 n v^4), R (2 o^2 v^4) and E (2 o^2 v^2)."""
    return 2.0 * n * v ** 4 + 2.0 * o * o * v ** 4 + 2.0 * o * o * v * v


def flops_adjoint(o, v, n):
    """Algorithmic dense flops of D (2 o^2 v^4) and X (2 n v^4), pair-symmetric form."""
    return 2.0 * o * o * v ** 4 + 2.0 * n * v ** 4
