"""Second oracle implementation: the same definitions with numpy matrix products.

Same quantities and citations as ladder_oracle.c (Sec. II A Cholesky expansion,
Sec. II B A2 ladder and V^4 density O^(2), Sec. II C W~, Appendix A pair symmetry
of d), written per virtual index a with library matrix products as steps, so that
the medium workload (o=20, v=150, n=600) finishes in seconds.  Test
infrastructure only; pinned by the same tests as the C version.
"""
from __future__ import annotations

import math

import numpy as np


def forward(o, v, n, L, tau, tbar=None, a_range=None):
    """R [o][o][v][v] and E = sum tbar*R (exactly rounded sum of the products).

    With a_range = (a_lo, a_hi) only the rows a in that range are formed; R is then
    [o][o][a_hi-a_lo][v] and E covers those rows only.
    """
    L = np.ascontiguousarray(L, dtype=np.float64).reshape(v, v, n)
    T = np.ascontiguousarray(tau, dtype=np.float64).reshape(o * o, v * v)  # [ij, (c,d)]
    Lbd = L.reshape(v * v, n)                                              # [(b,d), J]
    a_lo, a_hi = (0, v) if a_range is None else a_range
    R = np.empty((o * o, a_hi - a_lo, v))
    for a in range(a_lo, a_hi):
        g = L[a] @ Lbd.T                                   # g[c, (b,d)] = sum_J L^J_ac L^J_bd
        g = g.reshape(v, v, v).transpose(1, 0, 2).reshape(v, v * v)  # g[b, (c,d)]
        R[:, a - a_lo, :] = T @ g.T                        # R_ij^ab = sum_cd (ac|bd) tau_ij^cd
    R = R.reshape(o, o, a_hi - a_lo, v)
    E = 0.0
    if tbar is not None:
        tb = np.asarray(tbar, dtype=np.float64).reshape(o, o, v, v)[:, :, a_lo:a_hi, :]
        E = math.fsum((tb * R).ravel())
    return R, E


def adjoint(o, v, n, L, tau, w, p_range=None):
    """X^J_pq = sum_bd L^J_bd sum_ij (w_ij^pb tau_ij^qd + w_ij^bp tau_ij^dq), general form.

    With p_range = (p_lo, p_hi) only those rows are formed ([p_hi-p_lo][v][n]).
    """
    L = np.ascontiguousarray(L, dtype=np.float64).reshape(v, v, n)
    T = np.ascontiguousarray(tau, dtype=np.float64).reshape(o * o, v * v)  # [ij, (q,d)] or [ij, (d,q)]
    W = np.ascontiguousarray(w, dtype=np.float64).reshape(o * o, v, v)
    Lbd = L.reshape(v * v, n)
    p_lo, p_hi = (0, v) if p_range is None else p_range
    X = np.empty((p_hi - p_lo, v, n))
    for p in range(p_lo, p_hi):
        D1 = np.ascontiguousarray(W[:, p, :]).T @ T   # D1[b, (q,d)] = sum_ij w_ij^pb tau_ij^qd
        D2 = np.ascontiguousarray(W[:, :, p]).T @ T   # D2[b, (d,q)] = sum_ij w_ij^bp tau_ij^dq
        C = D1.reshape(v, v, v).transpose(1, 0, 2) + D2.reshape(v, v, v).transpose(2, 0, 1)  # C[q, b, d]
        X[p - p_lo] = C.reshape(v, v * v) @ Lbd
    return X


def tau_gradient(o, v, n, L, w, c_range=None):
    """G_ij^cd = sum_ab w_ij^ab (ac|bd), general L (the transposed ladder).

    With c_range = (c_lo, c_hi) only those rows are formed ([o][o][c_hi-c_lo][v]).
    """
    L = np.ascontiguousarray(L, dtype=np.float64).reshape(v, v, n)
    W = np.ascontiguousarray(w, dtype=np.float64).reshape(o * o, v * v)  # [ij, (a,b)]
    Lbd = L.reshape(v * v, n)
    c_lo, c_hi = (0, v) if c_range is None else c_range
    G = np.empty((o * o, c_hi - c_lo, v))
    for c in range(c_lo, c_hi):
        h = np.ascontiguousarray(L[:, c, :]) @ Lbd.T       # h[a, (b,d)] = sum_J L^J_ac L^J_bd
        G[:, c - c_lo, :] = W @ h.reshape(v * v, v)        # G_ij^cd = sum_ab w_ij^ab h[(a,b), d]
    return G.reshape(o, o, c_hi - c_lo, v)


def w_intermediate(o, v, n, Z, tau, w, p_range=None):
    """W^K_pq = sum_rs d_pqrs Z^K_rs with d_pqrs = sum_ij w_ij^pr tau_ij^qs, per row p."""
    Z = np.ascontiguousarray(Z, dtype=np.float64).reshape(v * v, n)        # [(r,s), K]
    T = np.ascontiguousarray(tau, dtype=np.float64).reshape(o * o, v * v)  # [ij, (q,s)]
    Wt = np.ascontiguousarray(w, dtype=np.float64).reshape(o * o, v, v)    # [ij, p, r]
    p_lo, p_hi = (0, v) if p_range is None else p_range
    out = np.empty((p_hi - p_lo, v, n))
    for p in range(p_lo, p_hi):
        d = np.ascontiguousarray(Wt[:, p, :]).T @ T                        # d[r, (q,s)]
        d = d.reshape(v, v, v).transpose(1, 0, 2).reshape(v, v * v)       # d[q, (r,s)]
        out[p - p_lo] = d @ Z
    return out


def metric_contraction(v, n, Z, W):
    """V_MN = sum_pq Z^M_pq W^N_pq."""
    return np.asarray(Z, dtype=np.float64).reshape(v * v, n).T @ np.asarray(W, dtype=np.float64).reshape(v * v, n)


def back_transform(v, n, x, y, W, K_range=None):
    """Wmo^K_pq = sum_rs x_rp y_sq W^K_rs, one K at a time."""
    W = np.asarray(W, dtype=np.float64).reshape(v, v, n)
    K_lo, K_hi = (0, n) if K_range is None else K_range
    out = np.empty((v, v, K_hi - K_lo))
    for K in range(K_lo, K_hi):
        out[:, :, K - K_lo] = x.T @ np.ascontiguousarray(W[:, :, K]) @ y
    return out


def ov3_abci(o, v, n, L2, R1, Zvv, Zvo):
    """Both W contributions of the excited-state OV^3 density d_abci = sum_j L_ji^ac R_j^b:
    Wab^K_ab = sum_ci d_abci Z^K_ci and Wci^K_ci = sum_ab d_abci Z^K_ab, one density slice
    d[a] = d_a[b, (c,i)] at a time (the density is formed, as in the C version)."""
    L2 = np.ascontiguousarray(L2, dtype=np.float64).reshape(o, o, v, v)   # [j, i, a, c]
    R1 = np.ascontiguousarray(R1, dtype=np.float64).reshape(o, v)         # [j, b]
    Zvv = np.ascontiguousarray(Zvv, dtype=np.float64).reshape(v, v, n)    # [a, b, K]
    Zvo = np.ascontiguousarray(Zvo, dtype=np.float64).reshape(v * o, n)   # [(c,i), K]
    Wab = np.empty((v, v, n))
    Wci = np.zeros((v * o, n))
    for a in range(v):
        M = np.ascontiguousarray(L2[:, :, a, :].transpose(0, 2, 1)).reshape(o, v * o)  # M[j, (c,i)] = L_ji^ac
        d = R1.T @ M                                                                    # d[b, (c,i)] = d_abci
        Wab[a] = d @ Zvo
        Wci += d.T @ Zvv[a]
    return Wab, Wci.reshape(v, o, n)


def ov3_abic(o, v, n, R0, L1, L2, T, R1, R2, Zvv, Zov):
    """Both W contributions of the excited-state OV^3 density d_abic (same eight terms and
    intermediates as the C version), the density formed in full with einsum and contracted."""
    f = lambda x, s: np.ascontiguousarray(x, dtype=np.float64).reshape(s)
    ein = lambda spec, *ops: np.einsum(spec, *ops, optimize=True)   # library contractions as steps
    L1, R1 = f(L1, (o, v)), f(R1, (o, v))
    L2, T, R2 = f(L2, (o, o, v, v)), f(T, (o, o, v, v)), f(R2, (o, o, v, v))
    Zvv, Zov = f(Zvv, (v, v, n)), f(Zov, (o, v, n))
    tt = 2.0 * T - T.transpose(1, 0, 2, 3)                      # t~_ij^ab
    eye_o, eye_v = np.eye(o), np.eye(v)
    Rt = R2 * (1.0 + ein("ij,ab->ijab", eye_o, eye_v))      # R~_ij^ab
    X = ein("klad,klbd->ab", L2, T)
    V = ein("lkae,libe->akbi", L2, T)
    Y = ein("klad,ilbd->akbi", L2, T)
    Yt = ein("lkea,liec->akci", L2, tt)
    W = ein("mkad,kd->am", L2, R1)
    B = ein("mnad,id->iamn", L2, R1)
    d = (R0 * ein("ma,imcb->abic", L1, tt)
         + ein("ma,mibc->abic", L1, 2.0 * Rt)
         - ein("ma,micb->abic", L1, Rt)
         + 2.0 * ein("ab,ic->abic", X, R1)
         - ein("akbi,kc->abic", V + Y, R1)
         + ein("am,mibc->abic", W, tt)
         - ein("iamn,mnbc->abic", B, T)
         + ein("akci,kb->abic", Yt, R1)
         - ein("ac,ib->abic", X, R1))
    Wab = ein("abic,icK->abK", d, Zov)
    Wic = ein("abic,abK->icK", d, Zvv)
    return Wab, Wic
