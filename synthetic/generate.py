"""Counter-based draws for the synthetic ladder inputs (host / numpy side).

Generator: SplitMix64 (G. L. Steele, D. Lea, C. H. Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), used as a stateless hash of a
64-bit counter:

    counter = seed << 48 | stream << 40 | index          (index < 2**40)
    z = counter + 0x9E3779B97F4A7C15
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB
    z = z ^ (z >> 31)                                     (all mod 2**64)
    uniform = (z >> 11) * 2**-53                          in [0, 1)

A Gaussian uses Box-Muller on two uniforms from the streams s and s | 0x80 at the
same index:  sqrt(-2 ln(1 - u1)) * cos(2 pi u2).

Input recipe (molecular shapes o occupied, v virtual, n Cholesky vectors,
N = o + v orbitals, occupied first):
  * L^J_pq = 0.3/sqrt(n) * G_{min(p,q), max(p,q), J}, G ~ N(0,1) from stream 1 at
    index (p*N + q)*n + J with p <= q  (symmetric in pq, like real-orbital CD vectors);
  * eps_i ~ U[-1.5, -0.3] (stream 2, index i), eps_a ~ U[0.1, 3.0] (stream 3, index a);
  * multiplier noise xi_{ij}^{ab} = N(0,1) from stream 4 at index P*(o*v) + Q with
    P = min(i*v+a, j*v+b), Q = max(...), so that xi_ij^ab = xi_ji^ba.
The amplitudes t_ij^ab = (ia|jb)/(eps_i+eps_j-eps_a-eps_b), tau = t and
tbar = t + 1e-2 * xi are formed by the consumer.
Stress variant (decaying Cholesky vectors, as pivoted Cholesky vectors of real
molecules decay with J): every block of L is multiplied by exp(-alpha * J / n)
along J before the amplitudes are formed (alpha = 0: the plain recipe).

The same generator is implemented for the GPU in synth.hip from the definition
above; the two agree bitwise on integers and uniforms and to a few ulps on
Gaussians (libm vs device log/cos).
"""
from __future__ import annotations

import math

import numpy as np

GOLDEN_GAMMA = np.uint64(0x9E3779B97F4A7C15)
MIX1 = np.uint64(0xBF58476D1CE4E5B9)
MIX2 = np.uint64(0x94D049BB133111EB)

STREAM_L = 1
STREAM_EPS_OCC = 2
STREAM_EPS_VIRT = 3
STREAM_NOISE = 4
STREAM_SIZES = 5
STREAM_ASYM = 6
L_SCALE = 0.3
NOISE_SCALE = 1e-2

__all__ = [
    "splitmix64", "uniform", "gaussian", "counter", "draw_L_block", "draw_L_vv", "draw_L_ov",
    "draw_eps", "pair_noise", "draw_noise_full", "asym_noise_full", "batched_sizes", "decay_factors",
    "CONFIGS", "STREAM_L", "STREAM_EPS_OCC", "STREAM_EPS_VIRT", "STREAM_NOISE", "STREAM_SIZES",
    "STREAM_ASYM", "L_SCALE", "NOISE_SCALE",
]

# The five workloads (o occupied, v virtual, n Cholesky vectors, seed).
CONFIGS = {
    "tiny": dict(o=4, v=20, n=60, seed=1),
    "medium": dict(o=20, v=150, n=600, seed=2),
    "retinal": dict(o=78, v=657, n=2200, seed=3),
    "batched": dict(count=64, seed=4),
    "autograd": dict(o=40, v=350, n=1200, seed=5),
    "thymine": dict(o=33, v=228, n=967, seed=6),
    "azobenzene": dict(o=48, v=364, n=1444, seed=7),
}


def splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 output for state x (uint64 array), arithmetic mod 2**64."""
    with np.errstate(over="ignore"):
        z = x.astype(np.uint64) + GOLDEN_GAMMA
        z = (z ^ (z >> np.uint64(30))) * MIX1
        z = (z ^ (z >> np.uint64(27))) * MIX2
        return z ^ (z >> np.uint64(31))


def counter(seed: int, stream: int, index: np.ndarray) -> np.ndarray:
    if not (0 <= seed < 1 << 16 and 0 <= stream < 1 << 8):
        raise ValueError("seed must be < 2**16 and stream < 2**8")
    idx = np.asarray(index, dtype=np.uint64)
    if idx.size and int(idx.max()) >= 1 << 40:
        raise ValueError("counter index must be < 2**40")
    return (np.uint64(seed) << np.uint64(48)) | (np.uint64(stream) << np.uint64(40)) | idx


def uniform(seed: int, stream: int, index) -> np.ndarray:
    z = splitmix64(counter(seed, stream, index))
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def gaussian(seed: int, stream: int, index) -> np.ndarray:
    u1 = uniform(seed, stream, index)
    u2 = uniform(seed, stream | 0x80, index)
    return np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * math.pi * u2)


def draw_L_block(seed: int, N: int, n: int, p0: int, np_: int, q0: int, nq: int) -> np.ndarray:
    """L^J_pq for p in [p0, p0+np_), q in [q0, q0+nq) as a [np_][nq][n] array."""
    p = np.arange(p0, p0 + np_, dtype=np.int64)[:, None, None]
    q = np.arange(q0, q0 + nq, dtype=np.int64)[None, :, None]
    J = np.arange(n, dtype=np.int64)[None, None, :]
    lo = np.minimum(p, q)
    hi = np.maximum(p, q)
    idx = (lo * N + hi) * n + J
    return (L_SCALE / math.sqrt(n)) * gaussian(seed, STREAM_L, idx)


def draw_L_vv(seed: int, o: int, v: int, n: int) -> np.ndarray:
    """Virtual-virtual block, layout [v][v][n] (flat)."""
    out = np.empty((v, v, n), dtype=np.float64)
    step = max(1, (1 << 24) // max(1, v * n))
    for a0 in range(0, v, step):
        a1 = min(v, a0 + step)
        out[a0:a1] = draw_L_block(seed, o + v, n, o + a0, a1 - a0, o, v)
    return out


def draw_L_ov(seed: int, o: int, v: int, n: int) -> np.ndarray:
    """Occupied-virtual block, layout [o][v][n]."""
    return draw_L_block(seed, o + v, n, 0, o, o, v)


def decay_factors(n: int, alpha: float) -> np.ndarray:
    """exp(-alpha * J / n) for J < n: the per-vector scale of the decaying stress variant."""
    return np.exp(-float(alpha) * np.arange(n, dtype=np.float64) / n)


def draw_eps(seed: int, o: int, v: int) -> np.ndarray:
    eo = -1.5 + 1.2 * uniform(seed, STREAM_EPS_OCC, np.arange(o))
    ev = 0.1 + 2.9 * uniform(seed, STREAM_EPS_VIRT, np.arange(v))
    return np.concatenate([eo, ev])


def pair_noise(seed: int, o: int, v: int, i, j, a, b) -> np.ndarray:
    """xi_ij^ab for index arrays (broadcast), symmetric under (i,a) <-> (j,b)."""
    P1 = np.asarray(i, dtype=np.int64) * v + np.asarray(a, dtype=np.int64)
    P2 = np.asarray(j, dtype=np.int64) * v + np.asarray(b, dtype=np.int64)
    lo = np.minimum(P1, P2)
    hi = np.maximum(P1, P2)
    return gaussian(seed, STREAM_NOISE, lo * (o * v) + hi)


def draw_noise_full(seed: int, o: int, v: int) -> np.ndarray:
    """xi as a [o][o][v][v] array."""
    i = np.arange(o)[:, None, None, None]
    j = np.arange(o)[None, :, None, None]
    a = np.arange(v)[None, None, :, None]
    b = np.arange(v)[None, None, None, :]
    out = np.empty((o, o, v, v))
    for ii in range(o):
        out[ii] = pair_noise(seed, o, v, ii, j[0], a[0], b[0])
    return out


def asym_noise_full(seed: int, o: int, v: int, stream: int = STREAM_ASYM) -> np.ndarray:
    """Unsymmetrised N(0,1) draws [o][o][v][v] for tests that break pair symmetry."""
    return gaussian(seed, stream, np.arange(o * o * v * v)).reshape(o, o, v, v)


def batched_sizes(seed: int = 4, count: int = 64, o_range=(8, 40), v_range=(60, 300)):
    """(o, v, n) for a ragged batch: o ~ U{o_range}, v ~ U{v_range} (inclusive), n = 4(o+v).
    The defaults are the 64-instance workload (o in 8..40, v in 60..300)."""
    uo = uniform(seed, STREAM_SIZES, np.arange(count))
    uv = uniform(seed, STREAM_SIZES, np.arange(count) + count)
    o = o_range[0] + np.floor(uo * (o_range[1] - o_range[0] + 1)).astype(np.int64)
    v = v_range[0] + np.floor(uv * (v_range[1] - v_range[0] + 1)).astype(np.int64)
    return [(int(a), int(b), int(4 * (a + b))) for a, b in zip(o, v)]
