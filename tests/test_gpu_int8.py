"""Parity of the INT8-slice split path (LADDER_SPLIT_INT8) with the CPU oracle and with
exact integer arithmetic.

The INT8 slices carry 7 bits each (integers m_p in [-64, 64] under one exponent per row
and 256-long chunk), and every slice pair p + q < S goes to an exact INT32 sum per level
L = p + q; the levels are folded into FP64 per chunk.  The tolerances are the accuracy
targets (1e-8 in R and X, 1e-10 in E); the integer tests are bitwise.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2202_02019_amd as P
from helpers import err_norm, err_rel, integer_inputs

pytestmark = pytest.mark.gpu

TOL_RX, TOL_E = 1e-8, 1e-10
INT8_DEFAULT = P.Options(precision=P.SPLIT_INT8, n_slices=6, n_slices_adjoint=5)


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    oracle.build(force=False)
    return torch.device("cuda:0")


def g(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


def run(dev, o, v, n, L, tau, w, opts):
    Lg, tg, wg = g(L, dev), g(tau, dev), g(w, dev)
    R, E = P.forward(Lg, tg, wg, o=o, v=v, n=n, opts=opts)
    X = P.adjoint(Lg, tg, wg, o=o, v=v, n=n, opts=opts)
    torch.cuda.synchronize()
    return R.cpu().numpy(), float(E.cpu()), X.cpu().numpy()


def _levels_operands(rng, S, M, N, K):
    """A: even integers in [-126, 126] with 126 in every (row, chunk), so the chunk exponent is
    7 and slice 0 alone carries a/2 (|m_0| <= 63).  B: integers of magnitude below 2^(7S-1) with
    a maximum of at least 2^(7S-2) in every (row, chunk), so the exponent is 7S - 1 and all S
    slices are in use with b = sum_p m_p 2^(7(S-1-p)) exactly.  Every product pair (0, q) has
    p + q < S, so nothing is dropped and the split product is exact; the level sums of a chunk
    reach 256 * 63 * 64 (just under 2^20), the top of their range."""
    A = 2 * rng.integers(-63, 64, size=(M, K))
    B = rng.integers(-(2 ** (7 * S - 1) - 1), 2 ** (7 * S - 1), size=(N, K))
    for c0 in range(0, K, 256):
        A[:, c0] = 126 * np.where(rng.random(M) < 0.5, -1, 1)
        B[:, c0] = (2 ** (7 * S - 1) - 1) * np.where(rng.random(N) < 0.5, -1, 1)
    return A.astype(np.int64), B.astype(np.int64)


@pytest.mark.parametrize("S", [2, 3, 4, 5])
def test_int8_gemm_every_level_exact(dev, S):
    """ladder_gemm in INT8 on operands whose product the triangular truncation keeps whole
    (see _levels_operands): the result equals the int64 product bitwise, with the roles of the
    operands swapped too.  M, N span several 128 x 64 tiles with ragged edges; K three whole
    chunks and a ragged one (not a multiple of the 32-k step)."""
    rng = np.random.default_rng(1200 + S)
    M, N, K = 300, 150, 3 * 256 + 100
    A, B = _levels_operands(rng, S, M, N, K)
    ref = A @ B.T
    assert np.abs(ref).max() < 2 ** 53
    opts = P.Options(precision=P.SPLIT_INT8, n_slices=S)
    C = P.gemm(g(A.astype(np.float64), dev), g(B.astype(np.float64), dev), opts=opts)
    Ct = P.gemm(g(B.astype(np.float64), dev), g(A.astype(np.float64), dev), opts=opts)
    torch.cuda.synchronize()
    got, gott = C.cpu().numpy(), Ct.cpu().numpy()
    print("int8 levels S=%d: max|C| %.4e, mismatches %d / %d" % (S, np.abs(got).max(), int((got != ref).sum()),
                                                               int((gott != ref.T).sum())))
    assert np.array_equal(got, ref.astype(np.float64)) and np.array_equal(gott, ref.T.astype(np.float64))


@pytest.mark.parametrize("S", [2, 3, 4, 5, 6])
def test_int8_gemm_alpha_beta_and_bound(dev, S):
    """ladder_gemm in INT8 on Gaussian data against the FP64 MFMA result, within the worst-case
    slice bound: per term the residuals of both operands (each <= 2^-7S of the chunk scale) and
    the dropped pairs p + q >= S (level L holds L + 1 pairs of at most 2^-7L) stay below
    (S + 4) 2^-7S of 2^(eA + eB) <= 4 max|a| max|b|."""
    rng = np.random.default_rng(1250 + S)
    M, N, K = 130, 257, 600
    A, B, C0 = rng.standard_normal((M, K)), rng.standard_normal((N, K)), rng.standard_normal((M, N))
    Ag, Bg = g(A, dev), g(B, dev)
    C = P.gemm(Ag, Bg, C=g(C0, dev), alpha=0.5, beta=-2.0, opts=P.Options(precision=P.SPLIT_INT8, n_slices=S))
    C64 = P.gemm(Ag, Bg, C=g(C0, dev), alpha=0.5, beta=-2.0, opts=P.Options(precision=P.FP64))
    torch.cuda.synchronize()
    bound = 0.5 * K * (S + 4) * 2.0 ** (-7 * S) * 4 * np.abs(A).max() * np.abs(B).max()
    d = np.abs(C.cpu().numpy() - C64.cpu().numpy()).max()
    print("int8 gaussian S=%d: max |C - C_fp64| %.3e, bound %.3e" % (S, d, bound))
    assert d <= bound


@pytest.mark.parametrize("flags", [0, P.FLAG_DENSE])
@pytest.mark.parametrize("o,v,n,seed", [(2, 5, 3, 1), (3, 9, 40, 2), (4, 20, 300, 3)])
def test_int8_integer_inputs_bitwise(dev, o, v, n, seed, flags):
    """Small integers are carried by slice 0 alone and every sum stays below 2^53: forward,
    energy and adjoint equal the oracle bitwise on both paths (n = 300 gives two chunks along J)."""
    L, tau, w = integer_inputs(seed, o, v, n, lim=3)
    opts = P.Options(precision=P.SPLIT_INT8, n_slices=6, n_slices_adjoint=5, flags=flags)
    R, E, X = run(dev, o, v, n, L, tau, w, opts)
    Rr, Er = oracle.forward(o, v, n, L, tau, w)
    Xr = oracle.adjoint(o, v, n, L, tau, w)
    assert np.array_equal(R, Rr) and E == Er and np.array_equal(X, Xr)


@pytest.mark.parametrize("flags", [0, P.FLAG_DENSE])
@pytest.mark.parametrize("decay", [0.0, 8.0])
def test_int8_medium_recipe(dev, flags, decay):
    """The medium recipe workload (o=20, v=150, n=600, decaying vectors too) at the default
    INT8 slice counts (6 forward, 5 adjoint; the long-K GEMMs split K up to 16 ways): R, E
    and X against the oracle (measured 2.7e-12, 1.8e-12, 1.5e-9 without decay)."""
    o, v, n = 20, 150, 600
    L, tau, tbar, _, _ = oracle.make_inputs(o, v, n, 2, decay=decay)
    opts = P.Options(precision=P.SPLIT_INT8, n_slices=6, n_slices_adjoint=5, flags=flags)
    R, E, X = run(dev, o, v, n, L, tau, tbar, opts)
    Rr, Er = oracle.forward(o, v, n, L, tau, tbar)
    Xr = oracle.adjoint(o, v, n, L, tau, tbar)
    eR, eE, eX = err_norm(R, Rr), err_rel(E, Er), err_norm(X, Xr)
    print("int8 medium decay %.0f flags %d: err_R %.3e err_E %.3e err_X %.3e" % (decay, flags, eR, eE, eX))
    assert eR <= TOL_RX and eE <= TOL_E and eX <= TOL_RX


@pytest.mark.parametrize("decay", [4.0, 8.0])
def test_int8_tiny_decaying_vectors(dev, decay):
    """The hardest recipe case for the per-(row, chunk) exponents (n = 60: one chunk per row,
    the smallest entries decay / ln 2 bits below its exponent).  Six forward slices meet the
    energy target (measured 1.2e-11 and 2.2e-11); five do not under decay 8 (2.4e-9), which is
    why the forward takes six INT8 slices."""
    o, v, n = 4, 20, 60
    L, tau, tbar, _, _ = oracle.make_inputs(o, v, n, 1, decay=decay)
    Rr, Er = oracle.forward(o, v, n, L, tau, tbar)
    Xr = oracle.adjoint(o, v, n, L, tau, tbar)
    R, E, X = run(dev, o, v, n, L, tau, tbar, INT8_DEFAULT)
    eR, eE, eX = err_norm(R, Rr), err_rel(E, Er), err_norm(X, Xr)
    print("int8 tiny, decay %.0f: err_R %.3e err_E %.3e err_X %.3e" % (decay, eR, eE, eX))
    assert eR <= TOL_RX and eE <= TOL_E and eX <= TOL_RX
    _, E5, _ = run(dev, o, v, n, L, tau, tbar, P.Options(precision=P.SPLIT_INT8, n_slices=5))
    assert err_rel(E5, Er) > eE


def test_int8_ragged_batches_and_determinism(dev):
    """Batches that leave a ragged last one (n_abatch = 7 of v = 30) and a K that is not a
    multiple of 32: parity with the oracle, and two runs bitwise equal."""
    o, v, n = 5, 30, 90
    L, tau, tbar, _, _ = oracle.make_inputs(o, v, n, 9)
    opts = P.Options(precision=P.SPLIT_INT8, n_slices=6, n_slices_adjoint=5, n_abatch=7)
    R, E, X = run(dev, o, v, n, L, tau, tbar, opts)
    R2, E2, X2 = run(dev, o, v, n, L, tau, tbar, opts)
    Rr, Er = oracle.forward(o, v, n, L, tau, tbar)
    Xr = oracle.adjoint(o, v, n, L, tau, tbar)
    assert err_norm(R, Rr) <= TOL_RX and err_rel(E, Er) <= TOL_E and err_norm(X, Xr) <= TOL_RX
    assert np.array_equal(R, R2) and E == E2 and np.array_equal(X, X2)


def test_int8_mfma_probe(dev):
    """The INT8 ceiling probe runs, reports its operations and writes repeatable checksums."""
    a, ops = P.mfma_probe(P.PROBE_INT8, 64, 16)
    b, ops2 = P.mfma_probe(P.PROBE_INT8, 64, 16)
    torch.cuda.synchronize()
    assert ops == ops2 == 16 * 4 * 64 * 4 * (2 * 32 * 32 * 32)
    assert torch.isfinite(a).all() and torch.equal(a, b) and float(a.abs().sum()) > 0


@pytest.mark.parametrize("flags", [0, P.FLAG_DENSE])
def test_int8_tau_gradient(dev, flags):
    """The transposed ladder (dE/dtau, the forward path with tbar for tau) in INT8 slices against
    the oracle at the R tolerance."""
    o, v, n = 6, 30, 120
    L, tau, tbar, _, _ = oracle.make_inputs(o, v, n, 11)
    opts = P.Options(precision=P.SPLIT_INT8, n_slices=6, n_slices_adjoint=5, flags=flags)
    G = P.tau_gradient(g(L, dev), g(tbar, dev), o=o, v=v, n=n, opts=opts)
    torch.cuda.synchronize()
    eG = err_norm(G.cpu().numpy(), oracle.tau_gradient(o, v, n, L, tbar))
    print("int8 tau gradient flags %d: err %.3e" % (flags, eG))
    assert eG <= TOL_RX
