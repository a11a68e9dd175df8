"""Shared test helpers: error metrics and seeded inputs (no ladder arithmetic)."""
import numpy as np


def err_norm(x, ref):
    """max|x - ref| / max|ref| (normwise, infinity norm)."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.abs(ref).max()
    return float(np.abs(x - ref).max() / den) if den > 0 else float(np.abs(x).max())


def err_rel(x, ref):
    return abs(float(x) - float(ref)) / abs(float(ref)) if ref != 0 else abs(float(x))


def pair_sym(x):
    return 0.5 * (x + x.transpose(1, 0, 3, 2))


def gaussian_inputs(seed, o, v, n, symmetric=True):
    """Generic Gaussian L (asymmetric in ac), tau, w; pair-symmetric tau and w if asked."""
    rng = np.random.default_rng(seed)
    L = rng.standard_normal((v, v, n)) * (0.3 / np.sqrt(n))
    tau = rng.standard_normal((o, o, v, v)) * 1e-2
    w = rng.standard_normal((o, o, v, v)) * 1e-2
    if symmetric:
        tau, w = pair_sym(tau), pair_sym(w)
    return L, tau, w


def integer_inputs(seed, o, v, n, symmetric=True, lim=7):
    rng = np.random.default_rng(seed)
    L = rng.integers(-lim, lim + 1, size=(v, v, n)).astype(np.float64)
    tau = rng.integers(-lim, lim + 1, size=(o, o, v, v)).astype(np.float64)
    w = rng.integers(-lim, lim + 1, size=(o, o, v, v)).astype(np.float64)
    if symmetric:
        # make x_ji^ba = x_ij^ab exactly, keeping integers
        for x in (tau, w):
            for i in range(o):
                for j in range(i):
                    x[j, i] = x[i, j].T
                U = np.triu(x[i, i])
                x[i, i] = U + np.triu(U, 1).T
        assert np.array_equal(tau, tau.transpose(1, 0, 3, 2)) and np.array_equal(w, w.transpose(1, 0, 3, 2))
    return L, tau, w
