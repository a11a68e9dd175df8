"""Parity of the HIP ladder (libladder.so, through its C ABI) with the CPU oracle.

Tolerances for the FP64 path: both sides sum the same products in different
orders, so each output differs by rounding only, bounded by about K*u*sum|terms|
with K = n for g and K = v^2 for R (u = 2^-53).  For these inputs that is below
1e-13 of max|R| (max|X|); the tests use 1e-11, which still sits three orders of
magnitude under the 1e-8 accuracy target.  Integer inputs whose sums stay below
2^53 are exact on both sides, so those compare bitwise.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_2202_02019_amd as P
from helpers import err_norm, err_rel, gaussian_inputs, integer_inputs

pytestmark = pytest.mark.gpu

TOL = 1e-11


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    oracle.build(force=False)
    return torch.device("cuda:0")


def g(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


def run(dev, o, v, n, L, tau, w, opts=None):
    Lg, tg, wg = g(L, dev), g(tau, dev), g(w, dev)
    R, E = P.forward(Lg, tg, wg, o=o, v=v, n=n, opts=opts)
    X = P.adjoint(Lg, tg, wg, o=o, v=v, n=n, opts=opts)
    torch.cuda.synchronize()
    return R.cpu().numpy(), float(E.cpu()), X.cpu().numpy()


PATHS = [pytest.param(0, id="pm"), pytest.param(P.FLAG_DENSE, id="dense")]


@pytest.mark.parametrize("flags", PATHS)
@pytest.mark.parametrize("o,v,n,seed", [(2, 5, 3, 1), (3, 4, 2, 2), (1, 3, 1, 3)])
def test_integer_inputs_bitwise(dev, o, v, n, seed, flags):
    L, tau, w = integer_inputs(seed, o, v, n)
    R, E, X = run(dev, o, v, n, L, tau, w, P.Options(flags=flags))
    Rr, Er = oracle.forward(o, v, n, L, tau, w)
    Xr = oracle.adjoint(o, v, n, L, tau, w)
    assert np.array_equal(R, Rr)
    assert E == Er
    assert np.array_equal(X, Xr)


def test_micro_example(dev):
    import json, os
    gd = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "micro_example.json")))
    L, tau, w = np.array(gd["L"]), np.array(gd["tau"]), np.array(gd["tbar"])
    R, E, X = run(dev, 1, 2, 1, L, tau, w, P.Options(flags=P.FLAG_GENERAL))
    assert np.array_equal(R.ravel(), np.array(gd["R"]).ravel()) and E == gd["E"]
    assert np.array_equal(X.ravel(), np.array(gd["X"]).ravel())


@pytest.mark.parametrize("flags", PATHS)
def test_tiny_workload(dev, flags):
    o, v, n = 4, 20, 60
    L, tau, tbar, _, _ = oracle.make_inputs(o, v, n, 1)
    R, E, X = run(dev, o, v, n, L, tau, tbar, P.Options(flags=flags))
    Rr, Er = oracle.forward(o, v, n, L, tau, tbar)
    Xr = oracle.adjoint(o, v, n, L, tau, tbar)
    print("tiny: err_R %.3e err_E %.3e err_X %.3e" % (err_norm(R, Rr), err_rel(E, Er), err_norm(X, Xr)))
    assert err_norm(R, Rr) <= TOL and err_rel(E, Er) <= TOL and err_norm(X, Xr) <= TOL


@pytest.mark.parametrize("flags", PATHS)
@pytest.mark.parametrize("o,v,n,nA", [(5, 37, 70, 4), (3, 41, 130, 0), (7, 19, 257, 19), (2, 129, 17, 64), (1, 23, 9, 5)])
def test_ragged_tiles_and_batches(dev, o, v, n, nA, flags):
    """Shapes whose M, N, K are not tile multiples, several batches with a ragged last one."""
    L, tau, w = gaussian_inputs(100 + v, o, v, n)
    R, E, X = run(dev, o, v, n, L, tau, w, P.Options(n_abatch=nA, flags=flags))
    Rr, Er = oracle.forward(o, v, n, L, tau, w)
    Xr = oracle.adjoint(o, v, n, L, tau, w)
    assert err_norm(R, Rr) <= TOL and err_rel(E, Er) <= TOL and err_norm(X, Xr) <= TOL


def test_general_flag_on_asymmetric_input(dev):
    o, v, n = 3, 23, 40
    L, tau, w = gaussian_inputs(7, o, v, n, symmetric=False)
    R, E, X = run(dev, o, v, n, L, tau, w, P.Options(flags=P.FLAG_GENERAL, n_abatch=5))
    Rr, Er = oracle.forward(o, v, n, L, tau, w)
    Xr = oracle.adjoint(o, v, n, L, tau, w)
    assert err_norm(R, Rr) <= TOL and err_rel(E, Er) <= TOL and err_norm(X, Xr) <= TOL
    # the default (pair-symmetric) adjoint must differ here: the flag matters
    _, _, Xs = run(dev, o, v, n, L, tau, w, P.Options(n_abatch=5))
    assert err_norm(Xs, Xr) > 1e-3


@pytest.mark.parametrize("flags", PATHS)
def test_alpha_beta_accumulation(dev, flags):
    o, v, n = 3, 17, 33
    L, tau, w = gaussian_inputs(8, o, v, n)
    R0 = np.random.default_rng(1).standard_normal((o, o, v, v))
    X0 = np.random.default_rng(2).standard_normal((v, v, n))
    Lg, tg, wg = g(L, dev), g(tau, dev), g(w, dev)
    R = g(R0, dev)
    X = g(X0, dev)
    opts = P.Options(flags=flags)
    P.forward(Lg, tg, wg, o=o, v=v, n=n, R=R, beta=0.5, opts=opts)
    P.adjoint(Lg, tg, wg, o=o, v=v, n=n, X=X, alpha=-2.0, beta=1.5, opts=opts)
    Rr, _ = oracle.forward(o, v, n, L, tau, w)
    Xr = oracle.adjoint(o, v, n, L, tau, w)
    assert err_norm(R.cpu().numpy(), 0.5 * R0 + Rr) <= TOL
    assert err_norm(X.cpu().numpy(), 1.5 * X0 - 2.0 * Xr) <= TOL


def test_beta_zero_ignores_nan_in_output(dev):
    o, v, n = 2, 9, 11
    L, tau, w = gaussian_inputs(9, o, v, n)
    Lg, tg, wg = g(L, dev), g(tau, dev), g(w, dev)
    R = torch.full((o, o, v, v), float("nan"), dtype=torch.float64, device=dev)
    X = torch.full((v, v, n), float("nan"), dtype=torch.float64, device=dev)
    P.forward(Lg, tg, wg, o=o, v=v, n=n, R=R, beta=0.0)
    P.adjoint(Lg, tg, wg, o=o, v=v, n=n, X=X, beta=0.0)
    assert torch.isfinite(R).all() and torch.isfinite(X).all()


@pytest.mark.parametrize("flags", PATHS)
def test_nan_input_propagates_to_energy(dev, flags):
    o, v, n = 2, 9, 11
    L, tau, w = gaussian_inputs(10, o, v, n)
    tau[1, 0, 3, 4] = tau[0, 1, 4, 3] = np.nan  # keeps the pair symmetry the packed path relies on
    _, E, X = run(dev, o, v, n, L, tau, w, P.Options(flags=flags))
    assert np.isnan(E) and np.isnan(X).any()


@pytest.mark.parametrize("flags", PATHS)
def test_deterministic_bitwise(dev, flags):
    o, v, n = 6, 45, 90
    L, tau, w = gaussian_inputs(11, o, v, n)
    a = run(dev, o, v, n, L, tau, w, P.Options(n_abatch=7, flags=flags))
    b = run(dev, o, v, n, L, tau, w, P.Options(n_abatch=7, flags=flags))
    assert np.array_equal(a[0], b[0]) and a[1] == b[1] and np.array_equal(a[2], b[2])


def test_workspace_too_small_raises(dev):
    o, v, n = 2, 5, 3
    L, tau, w = gaussian_inputs(12, o, v, n)
    ws = torch.empty(512, dtype=torch.uint8, device=dev)
    Lg, tg, wg = g(L, dev), g(tau, dev), g(w, dev)
    R = torch.empty((o, o, v, v), dtype=torch.float64, device=dev)
    with pytest.raises(ValueError):
        P.forward(Lg, tg, wg, o=o, v=v, n=n, R=R, ws=ws)


@pytest.mark.parametrize("flags", PATHS)
def test_medium_workload(dev, flags):
    """o=20, v=150, n=600, seed 2: every element of R and X and E against the oracle."""
    o, v, n = 20, 150, 600
    L, tau, tbar, _, _ = oracle.make_inputs(o, v, n, 2)
    R, E, X = run(dev, o, v, n, L, tau, tbar, P.Options(flags=flags))
    Rr, Er = oracle.matrix.forward(o, v, n, L, tau, tbar)
    Xr = oracle.matrix.adjoint(o, v, n, L, tau, tbar)
    print("medium: E %.17g (oracle %.17g) err_R %.3e err_E %.3e err_X %.3e"
          % (E, Er, err_norm(R, Rr), err_rel(E, Er), err_norm(X, Xr)))
    assert err_norm(R, Rr) <= TOL and err_rel(E, Er) <= TOL and err_norm(X, Xr) <= TOL


@pytest.mark.parametrize("o,v,n,seed", [(4, 20, 60, 1), (6, 53, 70, 21)])
def test_amplitudes_and_update(dev, o, v, n, seed):
    import synthetic
    Lov = synthetic.draw_L_ov(seed, o, v, n)
    eps = synthetic.draw_eps(seed, o, v)
    t_ref = oracle.mp2_amplitudes(o, v, n, Lov, eps)
    t = P.mp2_amplitudes(g(Lov, dev), g(eps, dev), o=o, v=v, n=n)
    assert err_norm(t.cpu().numpy(), t_ref) <= 1e-13
    tn = t.cpu().numpy()
    assert np.array_equal(tn, tn.transpose(1, 0, 3, 2))  # pair symmetry is kept bitwise
    R = np.random.default_rng(seed).standard_normal((o, o, v, v)) * 1e-3
    t2_ref = oracle.amplitude_update(o, v, eps, R, t_ref)
    tg = g(t_ref, dev)
    P.amplitude_update(g(eps, dev), g(R, dev), tg, o=o, v=v)
    assert err_norm(tg.cpu().numpy(), t2_ref) <= 1e-15


def test_autograd_backward_matches_oracle(dev):
    o, v, n = 3, 21, 25
    L, tau, w = gaussian_inputs(13, o, v, n)
    Lg = g(L, dev).requires_grad_(True)
    wg = g(w, dev).requires_grad_(True)
    E = P.ladder_energy(Lg, g(tau, dev), wg, (o, v, n))
    E.backward()
    Rr, Er = oracle.forward(o, v, n, L, tau, w)
    Xr = oracle.adjoint(o, v, n, L, tau, w)
    assert err_rel(float(E.detach()), Er) <= TOL
    assert err_norm(Lg.grad.cpu().numpy(), Xr) <= TOL
    assert err_norm(wg.grad.cpu().numpy(), Rr) <= TOL


def test_autograd_finite_differences(dev):
    """E is quadratic along one L entry: the central difference has no truncation error."""
    o, v, n = 4, 30, 40
    L, tau, w = gaussian_inputs(14, o, v, n)
    Lg, tg, wg = g(L, dev), g(tau, dev), g(w, dev)
    X = P.adjoint(Lg, tg, wg, o=o, v=v, n=n).cpu().numpy()
    rng = np.random.default_rng(3)
    h = 1e-6
    worst = 0.0
    for _ in range(200):
        a, c, J = rng.integers(v), rng.integers(v), rng.integers(n)
        Lp = Lg.clone(); Lp[a, c, J] += h
        Lm = Lg.clone(); Lm[a, c, J] -= h
        Ep = P.forward(Lp, tg, wg, o=o, v=v, n=n)[1]
        Em = P.forward(Lm, tg, wg, o=o, v=v, n=n)[1]
        fd = float((Ep - Em).cpu()) / (2 * h)
        worst = max(worst, abs(fd - X[a, c, J]) / np.abs(X).max())
    print("finite differences: worst |fd - X| / max|X| = %.3e" % worst)
    assert worst < 1e-7


# ------------------------------------------------------------------ split BF16
SPLIT5 = P.Options(precision=P.SPLIT_BF16, n_slices=5)
# Accuracy targets of the split path: 1e-8 normwise in R and X, 1e-10 relative in E.
SPLIT_TOL_RX = 1e-8
SPLIT_TOL_E = 1e-10


def err_E_terms(E, Er, w, Rr):
    """|E - E_ref| / sum|w R_ref|: the energy error against the magnitude of its terms.

    The relative target on E is stated for the workload recipe, where E has a
    systematic part; for generic random-sign inputs E itself can cancel to far
    below its terms, and the error is measured against the terms instead."""
    return abs(float(E) - float(Er)) / float(np.abs(np.asarray(w) * np.asarray(Rr)).sum())


@pytest.mark.parametrize("flags", PATHS)
@pytest.mark.parametrize("o,v,n,seed,S", [(2, 5, 3, 1, 3), (3, 4, 2, 2, 2), (2, 33, 21, 4, 3)])
def test_split_integer_inputs_bitwise(dev, o, v, n, seed, S, flags):
    """Small integers (and the half-integers of the +/- packing) are carried exactly
    by two or three slices, and every FP32 chunk sum is exact, so the split path
    must agree bitwise with the oracle."""
    L, tau, w = integer_inputs(seed, o, v, n, lim=3)
    R, E, X = run(dev, o, v, n, L, tau, w, P.Options(precision=P.SPLIT_BF16, n_slices=S, n_abatch=7, flags=flags))
    Rr, Er = oracle.forward(o, v, n, L, tau, w)
    Xr = oracle.adjoint(o, v, n, L, tau, w)
    assert np.array_equal(R, Rr)
    assert E == Er
    assert np.array_equal(X, Xr)


def test_split_tiny_workload(dev):
    o, v, n = 4, 20, 60
    L, tau, tbar, _, _ = oracle.make_inputs(o, v, n, 1)
    R, E, X = run(dev, o, v, n, L, tau, tbar, SPLIT5)
    Rr, Er = oracle.forward(o, v, n, L, tau, tbar)
    Xr = oracle.adjoint(o, v, n, L, tau, tbar)
    print("split tiny: err_R %.3e err_E %.3e err_X %.3e" % (err_norm(R, Rr), err_rel(E, Er), err_norm(X, Xr)))
    assert err_norm(R, Rr) <= SPLIT_TOL_RX and err_rel(E, Er) <= SPLIT_TOL_E and err_norm(X, Xr) <= SPLIT_TOL_RX


@pytest.mark.parametrize("flags", PATHS)
@pytest.mark.parametrize("o,v,n,nA", [(5, 37, 70, 4), (3, 41, 300, 0), (7, 19, 257, 19), (2, 129, 17, 64), (1, 23, 9, 5)])
def test_split_ragged_tiles_chunks_batches(dev, o, v, n, nA, flags):
    """K not a multiple of the 256 chunk nor of 16, several batches, ragged edges."""
    L, tau, w = gaussian_inputs(200 + v, o, v, n)
    R, E, X = run(dev, o, v, n, L, tau, w, P.Options(precision=P.SPLIT_BF16, n_slices=5, n_abatch=nA, flags=flags))
    Rr, Er = oracle.forward(o, v, n, L, tau, w)
    Xr = oracle.adjoint(o, v, n, L, tau, w)
    assert err_norm(R, Rr) <= SPLIT_TOL_RX and err_E_terms(E, Er, w, Rr) <= SPLIT_TOL_E and err_norm(X, Xr) <= SPLIT_TOL_RX


def test_split_general_flag(dev):
    o, v, n = 3, 23, 40
    L, tau, w = gaussian_inputs(17, o, v, n, symmetric=False)
    opts = P.Options(precision=P.SPLIT_BF16, n_slices=5, flags=P.FLAG_GENERAL, n_abatch=6)
    R, E, X = run(dev, o, v, n, L, tau, w, opts)
    Rr, Er = oracle.forward(o, v, n, L, tau, w)
    Xr = oracle.adjoint(o, v, n, L, tau, w)
    assert err_norm(R, Rr) <= SPLIT_TOL_RX and err_E_terms(E, Er, w, Rr) <= SPLIT_TOL_E and err_norm(X, Xr) <= SPLIT_TOL_RX


def test_split_deterministic_bitwise(dev):
    o, v, n = 6, 45, 90
    L, tau, w = gaussian_inputs(18, o, v, n)
    a = run(dev, o, v, n, L, tau, w, P.Options(precision=P.SPLIT_BF16, n_abatch=7))
    b = run(dev, o, v, n, L, tau, w, P.Options(precision=P.SPLIT_BF16, n_abatch=7))
    assert np.array_equal(a[0], b[0]) and a[1] == b[1] and np.array_equal(a[2], b[2])


def test_split_medium_error_versus_slices(dev):
    """o=20, v=150, n=600: error of every output against the oracle for S = 2..6;
    S = 5 (the default) must meet the targets, and more slices must not be worse."""
    o, v, n = 20, 150, 600
    L, tau, tbar, _, _ = oracle.make_inputs(o, v, n, 2)
    Rr, Er = oracle.matrix.forward(o, v, n, L, tau, tbar)
    Xr = oracle.matrix.adjoint(o, v, n, L, tau, tbar)
    errs = {}
    for S in (2, 3, 4, 5, 6):
        R, E, X = run(dev, o, v, n, L, tau, tbar, P.Options(precision=P.SPLIT_BF16, n_slices=S))
        errs[S] = (err_norm(R, Rr), err_rel(E, Er), err_norm(X, Xr))
        print("split medium S=%d: err_R %.3e err_E %.3e err_X %.3e" % ((S,) + errs[S]))
    eR, eE, eX = errs[5]
    assert eR <= SPLIT_TOL_RX and eE <= SPLIT_TOL_E and eX <= SPLIT_TOL_RX
    assert errs[6][0] <= 2 * errs[5][0] and errs[5][0] <= errs[3][0]


@pytest.mark.parametrize("alpha", [4.0, 8.0])
def test_split_medium_decaying_vectors(dev, alpha):
    """Stress variant of the recipe: Cholesky vectors decaying as exp(-alpha J / n) (real pivoted
    vectors do), so the chunk exponents of the slices along J differ by up to alpha / ln 2 bits.
    The default S = 5 still meets the targets on every element of the medium workload."""
    o, v, n = 20, 150, 600
    L, tau, tbar, _, _ = oracle.make_inputs(o, v, n, 2, decay=alpha)
    Rr, Er = oracle.matrix.forward(o, v, n, L, tau, tbar)
    Xr = oracle.matrix.adjoint(o, v, n, L, tau, tbar)
    R, E, X = run(dev, o, v, n, L, tau, tbar, P.Options(precision=P.SPLIT_BF16))
    eR, eE, eX = err_norm(R, Rr), err_rel(E, Er), err_norm(X, Xr)
    print("split medium, decay %.0f: err_R %.3e err_E %.3e err_X %.3e" % (alpha, eR, eE, eX))
    assert eR <= SPLIT_TOL_RX and eE <= SPLIT_TOL_E and eX <= SPLIT_TOL_RX


@pytest.mark.parametrize("decay", [0.0, 8.0])
def test_split_adjoint_with_fewer_slices(dev, decay):
    """n_slices_adjoint = 4 beside the forward's 5 (the benchmark's configuration): the forward
    outputs are bitwise those of the all-5 run (the option reaches only the adjoint), and X stays
    within the 1e-8 target on every element of the medium workload, plain and with decaying
    Cholesky vectors (measured 3.1e-9 and 1.8e-9)."""
    o, v, n = 20, 150, 600
    L, tau, tbar, _, _ = oracle.make_inputs(o, v, n, 2, decay=decay)
    Rr, Er = oracle.matrix.forward(o, v, n, L, tau, tbar)
    Xr = oracle.matrix.adjoint(o, v, n, L, tau, tbar)
    R5, E5, X5 = run(dev, o, v, n, L, tau, tbar, P.Options(precision=P.SPLIT_BF16))
    R, E, X = run(dev, o, v, n, L, tau, tbar, P.Options(precision=P.SPLIT_BF16, n_slices_adjoint=4))
    eX, eX5 = err_norm(X, Xr), err_norm(X5, Xr)
    print("split medium, decay %.0f: err_X with 4 adjoint slices %.3e (5: %.3e)" % (decay, eX, eX5))
    assert np.array_equal(R, R5) and E == E5
    assert err_rel(E, Er) <= SPLIT_TOL_E and err_norm(R, Rr) <= SPLIT_TOL_RX
    assert eX <= SPLIT_TOL_RX and eX5 < eX


@pytest.mark.parametrize("flags", PATHS)
def test_split_mixed_slice_counts_integer_bitwise(dev, flags):
    """Small integers are carried exactly by two slices as well as three, so a forward at 3 and
    an adjoint at 2 slices must both match the oracle bitwise."""
    o, v, n = 3, 33, 21
    L, tau, w = integer_inputs(170, o, v, n, lim=3)
    opts = P.Options(precision=P.SPLIT_BF16, n_slices=3, n_slices_adjoint=2, n_abatch=7, flags=flags)
    R, E, X = run(dev, o, v, n, L, tau, w, opts)
    Rr, Er = oracle.forward(o, v, n, L, tau, w)
    Xr = oracle.adjoint(o, v, n, L, tau, w)
    assert np.array_equal(R, Rr) and E == Er and np.array_equal(X, Xr)


@pytest.mark.parametrize("decay", [4.0, 8.0])
def test_split_tiny_decaying_vectors(dev, decay):
    """The hardest recipe case for the per-(row, 256-chunk) exponents: n = 60 puts every Cholesky
    index of a row in one chunk, so with vectors decaying as exp(-decay J / n) the smallest entries of
    a chunk sit decay / ln 2 bits below its exponent.  The default five slices still meet the
    targets (measured E 9.1e-12 and 5.0e-11)."""
    o, v, n = 4, 20, 60
    L, tau, tbar, _, _ = oracle.make_inputs(o, v, n, 1, decay=decay)
    R, E, X = run(dev, o, v, n, L, tau, tbar, SPLIT5)
    Rr, Er = oracle.forward(o, v, n, L, tau, tbar)
    Xr = oracle.adjoint(o, v, n, L, tau, tbar)
    eR, eE, eX = err_norm(R, Rr), err_rel(E, Er), err_norm(X, Xr)
    print("split tiny, decay %.0f: err_R %.3e err_E %.3e err_X %.3e" % (decay, eR, eE, eX))
    assert eR <= SPLIT_TOL_RX and eE <= SPLIT_TOL_E and eX <= SPLIT_TOL_RX


@pytest.mark.parametrize("o,v,n,seed", [(1, 2, 1, 160), (2, 3, 2, 161)])
def test_autograd_gradcheck(dev, o, v, n, seed):
    """torch.autograd.gradcheck on the FP64 path: central differences of E in every entry of
    L, tau and tbar (E is quadratic in L and bilinear in (tau, tbar), so the differences are
    exact up to rounding) against LadderEnergy's backward (adjoint, transposed ladder, R).
    The perturbations break pair symmetry, so the general path is used."""
    L, tau, w = gaussian_inputs(seed, o, v, n, symmetric=False)
    args = [g(x, dev).requires_grad_(True) for x in (L, tau, w)]
    opts = P.Options(flags=P.FLAG_GENERAL)
    f = lambda L_, t_, w_: P.ladder_energy(L_, t_, w_, (o, v, n), opts)
    assert torch.autograd.gradcheck(f, args, eps=1e-6, atol=1e-9, rtol=1e-7)


@pytest.mark.parametrize("precision,S_fwd,S_adj", [pytest.param(P.SPLIT_INT8, 6, 5, id="int8-6-5"),
                                                 pytest.param(P.SPLIT_BF16, 5, 4, id="bf16-5-4")])
def test_retinal_split_sampled(dev, precision, S_fwd, S_adj):
    """o=78, v=657, n=2200, seed 3, in the configurations the benchmark times (INT8 slices 6
    forward / 5 adjoint, its default, and BF16 5 / 4; +/- packed, the batch size of the committed
    autotune cache): one forward and one adjoint on
    the GPU-drawn recipe inputs, then sampled rows of R (all ij for chosen ab) and of X (all J for
    chosen ac) against the oracle, computed one by one from host copies of the same arrays."""
    import os
    from synthetic import gpu as SG
    torch.cuda.empty_cache()
    o, v, n, seed = 78, 657, 2200, 3
    cache = os.path.join(os.path.dirname(P.library_path()), "tuned_mi355x.jsonl")
    P.autotune_load(cache)
    L = SG.draw_L_vv(seed, o, v, n)
    Lov = SG.draw_L_ov(seed, o, v, n)
    tau = P.mp2_amplitudes(Lov, SG.draw_eps(seed, o, v), o=o, v=v, n=n)
    del Lov
    tbar = SG.add_noise(seed, o, v, tau)
    opts = P.Options(precision=precision, n_slices=S_fwd, n_slices_adjoint=S_adj)
    ws = torch.empty(P.workspace_size(o, v, n, opts), dtype=torch.uint8, device=dev)
    R, E = P.forward(L, tau, tbar, o=o, v=v, n=n, ws=ws, opts=opts)
    X = P.adjoint(L, tau, tbar, o=o, v=v, n=n, ws=ws, opts=opts)
    torch.cuda.synchronize()
    del ws
    print("retinal split: forward + adjoint done, E = %.15g" % float(E), flush=True)
    Lh, th, wh = L.cpu().numpy(), tau.cpu().numpy(), tbar.cpu().numpy()
    ab = np.array([[0, 0], [656, 656], [3, 600], [600, 3], [327, 328]])
    pq = np.array([[0, 0], [656, 1], [100, 540]])
    Rr = oracle.R_sample(o, v, n, Lh, th, ab)
    Xr = oracle.X_sample(o, v, n, Lh, th, wh, pq)
    Rg = np.stack([R[:, :, a, b].cpu().numpy().ravel() for a, b in ab])
    Xg = np.stack([X[p, q].cpu().numpy() for p, q in pq])
    eR, eX = err_norm(Rg, Rr), err_norm(Xg, Xr)
    print("retinal split sampled: err_R %.3e err_X %.3e" % (eR, eX), flush=True)
    assert eR <= SPLIT_TOL_RX and eX <= SPLIT_TOL_RX
    # the energy of two whole rows a (all i, j, b) against the oracle's forward rows: the
    # oracle's own exactly rounded sum of tbar * R over those rows, and the same sum of the GPU R
    rows = (0, 401)
    e_gpu, e_ref = [], []
    for a in rows:
        Rr_a, Er_a = oracle.matrix.forward(o, v, n, Lh, th, wh, a_range=(a, a + 1))
        e_ref.append(Er_a)
        e_gpu.append(math.fsum((wh[:, :, a, :] * R[:, :, a, :].cpu().numpy()).ravel()))
    eErows = err_rel(sum(e_gpu), sum(e_ref))
    print("retinal split: energy of rows a = %s: split %.15e oracle %.15e rel %.2e"
          % (rows, sum(e_gpu), sum(e_ref), eErows), flush=True)
    assert eErows <= SPLIT_TOL_E
    # the whole energy against the FP64 MFMA path on the same device arrays (that path is
    # compared with the oracle element by element at the medium size and on sampled rows here)
    del X, Lh, th, wh
    torch.cuda.empty_cache()
    o64 = P.Options(precision=P.FP64)
    ws64 = torch.empty(P.workspace_size(o, v, n, o64), dtype=torch.uint8, device=dev)
    R64, E64 = P.forward(L, tau, tbar, o=o, v=v, n=n, ws=ws64, opts=o64)
    torch.cuda.synchronize()
    eE = err_rel(float(E), float(E64))
    eR64 = max(float((R[i] - R64[i]).abs().max()) for i in range(o)) / max(float(R64[i].abs().max()) for i in range(o))
    print("retinal split vs FP64 GPU: E %.15e vs %.15e rel %.2e; err_R (all elements) %.2e"
          % (float(E), float(E64), eE, eR64), flush=True)
    assert eE <= SPLIT_TOL_E and eR64 <= SPLIT_TOL_RX


@pytest.mark.parametrize("kind", [P.PROBE_BF16, P.PROBE_FP64])
def test_mfma_probe(dev, kind):
    """The ceiling probe runs, reports the flops of its launch and writes finite, repeatable
    checksums (the same register-only arithmetic twice)."""
    a, fl = P.mfma_probe(kind, 64, 16)
    b, fl2 = P.mfma_probe(kind, 64, 16)
    torch.cuda.synchronize()
    per = 2 * 32 * 32 * 16 if kind == P.PROBE_BF16 else 2 * 16 * 16 * 4
    assert fl == fl2 == 16 * 4 * 64 * 4 * per
    assert torch.isfinite(a).all() and torch.equal(a, b) and float(a.abs().sum()) > 0


# ------------------------------------------------------------------ exactness at the 24-bit edge
def _edge_operands(rng, rows, K, lo, hi, odd=False):
    """Integers of magnitude in [lo, hi] (odd ones only if asked) with one random sign per
    row: every product of a row of A with a row of B then has the same sign within the row
    pair, so the chunk sums of the split product grow monotonically to the top of their range."""
    mag = rng.integers(lo, hi + 1, size=(rows, K))
    if odd:
        mag |= 1
    sign = np.where(rng.random((rows, 1)) < 0.5, -1, 1)
    return (mag * sign).astype(np.int64)


@pytest.mark.parametrize("S,lo,hi", [(2, 241, 255), (3, 65280 + 96, 65280 + 127)])
def test_split_gemm_chunk_sums_at_24_bits(dev, S, lo, hi):
    """The FP32 accumulators of the split GEMM are exact only if every chunk sum fits the
    24-bit significand.  S = 2 with odd-heavy 8-bit integers near 255: slice 0 carries each
    value whole (the chunk exponent is 8), and a 256-long chunk of same-sign products sums to
    at most 256 * 255^2 = 16 646 400 < 2^24 (its odd partial sums use all 24 bits).  S = 3 with
    16-bit integers 65280 + r, r in [96, 127]: slice 0 is 255, slice 1 is r, so the
    (0,1) + (1,0) sums reach 2 * 256 * 255 * 127 = 16 581 120 < 2^24 as well, and (1,1) is
    exact too.  K spans three whole chunks and a ragged one, M and N several tiles with ragged
    edges; the result must equal the int64 product bitwise (it is below 2^53)."""
    rng = np.random.default_rng(900 + S)
    M, N, K = 300, 260, 3 * 256 + 100
    A = _edge_operands(rng, M, K, lo, hi, odd=S == 2)
    B = _edge_operands(rng, N, K, lo, hi, odd=S == 2)
    ref = A @ B.T                                     # int64, exact
    assert np.abs(ref).max() < 2 ** 53
    Ag, Bg = g(A.astype(np.float64), dev), g(B.astype(np.float64), dev)
    for opts in (P.Options(precision=P.SPLIT_BF16, n_slices=S), P.Options(precision=P.FP64)):
        C = P.gemm(Ag, Bg, opts=opts)
        torch.cuda.synchronize()
        got = C.cpu().numpy()
        print("edge S=%d precision %d: max|C| %.4e, mismatches %d" % (S, opts.precision, np.abs(got).max(),
                                                                    int((got != ref).sum())))
        assert np.array_equal(got, ref.astype(np.float64))
    # one chunk alone: its sums are the largest the accumulators ever see
    C = P.gemm(Ag[:, :256].contiguous(), Bg[:, :256].contiguous(), opts=P.Options(precision=P.SPLIT_BF16, n_slices=S))
    torch.cuda.synchronize()
    assert np.array_equal(C.cpu().numpy(), (A[:, :256] @ B[:, :256].T).astype(np.float64))


@pytest.mark.parametrize("S", [2, 3, 4, 5])
def test_split_gemm_alpha_beta_and_fp64_agreement(dev, S):
    """ladder_gemm on Gaussian data: C = beta C + alpha A B^T against the FP64 MFMA result within
    the worst-case slice bound: per term, the residuals of both operands and the dropped pairs
    p + q >= S stay below (S+3)/4 2^-8S of the chunk scale 2^(eA+eB) <= 4 max|a| max|b|."""
    rng = np.random.default_rng(950 + S)
    M, N, K = 130, 257, 600
    A, B, C0 = rng.standard_normal((M, K)), rng.standard_normal((N, K)), rng.standard_normal((M, N))
    Ag, Bg = g(A, dev), g(B, dev)
    C = P.gemm(Ag, Bg, C=g(C0, dev), alpha=0.5, beta=-2.0, opts=P.Options(precision=P.SPLIT_BF16, n_slices=S))
    C64 = P.gemm(Ag, Bg, C=g(C0, dev), alpha=0.5, beta=-2.0, opts=P.Options(precision=P.FP64))
    torch.cuda.synchronize()
    ref = -2.0 * C0 + 0.5 * (A @ B.T)
    assert np.abs(C64.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()
    bound = 0.5 * K * (S + 3) * 2.0 ** (-8 * S) * np.abs(A).max() * np.abs(B).max()
    assert np.abs(C.cpu().numpy() - C64.cpu().numpy()).max() <= bound


def test_split_autograd(dev):
    o, v, n = 3, 21, 25
    L, tau, w = gaussian_inputs(19, o, v, n)
    Lg = g(L, dev).requires_grad_(True)
    E = P.ladder_energy(Lg, g(tau, dev), g(w, dev), (o, v, n), SPLIT5)
    E.backward()
    Rr, Er = oracle.forward(o, v, n, L, tau, w)
    Xr = oracle.adjoint(o, v, n, L, tau, w)
    assert err_E_terms(float(E.detach()), Er, w, Rr) <= SPLIT_TOL_E
    assert err_norm(Lg.grad.cpu().numpy(), Xr) <= SPLIT_TOL_RX


# ------------------------------------------------------------------ ragged batches
def _instances(dev, shapes, seed0):
    insts, refs = [], []
    for k, (o, v, n) in enumerate(shapes):
        L, tau, w = gaussian_inputs(seed0 + k, o, v, n)
        insts.append(dict(o=o, v=v, n=n, L=g(L, dev), tau=g(tau, dev), tbar=g(w, dev),
                          R=torch.empty((o, o, v, v), dtype=torch.float64, device=dev),
                          E=torch.empty((), dtype=torch.float64, device=dev),
                          X=torch.empty((v, v, n), dtype=torch.float64, device=dev)))
        refs.append((L, tau, w))
    return insts, refs


@pytest.mark.parametrize("precision", [P.FP64, P.SPLIT_BF16, P.SPLIT_INT8])
def test_batched_matches_single_calls_and_oracle(dev, precision):
    shapes = [(3, 17, 30), (5, 9, 11), (2, 40, 70), (4, 23, 5), (6, 31, 44), (1, 12, 9), (7, 6, 20), (3, 50, 33),
              (2, 19, 101), (4, 8, 16)]
    insts, refs = _instances(dev, shapes, 300)
    opts = P.Options(precision=precision, n_abatch=4)
    P.batched(insts, P.DO_FORWARD | P.DO_ADJOINT, opts=opts)
    torch.cuda.synchronize()
    tol_rx, tol_e = (TOL, TOL) if precision == P.FP64 else (SPLIT_TOL_RX, SPLIT_TOL_E)
    e_err = err_rel if precision == P.FP64 else (lambda E, Er: err_E_terms(E, Er, w, Rr))
    for d, (L, tau, w) in zip(insts, refs):
        o, v, n = d["o"], d["v"], d["n"]
        R1, E1 = P.forward(d["L"], d["tau"], d["tbar"], o=o, v=v, n=n, opts=opts)
        X1 = P.adjoint(d["L"], d["tau"], d["tbar"], o=o, v=v, n=n, opts=opts)
        assert torch.equal(d["R"], R1) and torch.equal(d["X"], X1) and torch.equal(d["E"], E1)
        Rr, Er = oracle.forward(o, v, n, L, tau, w)
        Xr = oracle.adjoint(o, v, n, L, tau, w)
        assert err_norm(d["R"].cpu().numpy(), Rr) <= tol_rx and err_norm(d["X"].cpu().numpy(), Xr) <= tol_rx
        assert e_err(float(d["E"].cpu()), Er) <= tol_e


def _recipe_instances(dev, sizes, seed0):
    """The ragged-batch recipe on the GPU: per instance m, Cholesky vectors and orbital energies
    drawn with seed seed0 + m, first-order amplitudes by the library, tbar = t + noise."""
    from synthetic import gpu as SG
    insts = []
    for m, (o, v, n) in enumerate(sizes):
        seed = seed0 + m
        L = SG.draw_L_vv(seed, o, v, n)
        Lov = SG.draw_L_ov(seed, o, v, n)
        tau = P.mp2_amplitudes(Lov, SG.draw_eps(seed, o, v), o=o, v=v, n=n)
        del Lov
        tbar = SG.add_noise(seed, o, v, tau)
        insts.append(dict(o=o, v=v, n=n, L=L, tau=tau, tbar=tbar, R=torch.empty_like(tau),
                          E=torch.empty((), dtype=torch.float64, device=dev), X=torch.empty_like(L)))
    return insts


@pytest.mark.parametrize("sizes_seed,o_range,v_range", [(4, (8, 40), (60, 300)), (8, (4, 12), (20, 80))],
                         ids=["config4", "small"])
def test_batched_64_recipe_instances(dev, sizes_seed, o_range, v_range):
    """The 64-instance ragged workload (sizes from seed 4, data seeds 1000 + m; and a set of small
    instances): one ladder_batched graph launch (split precision, 8 virtual indices per batch for
    every instance, so that the single calls run the same plans) against 64 single forward + adjoint
    calls bitwise, and the four smallest instances against the oracle."""
    import synthetic
    sizes = synthetic.batched_sizes(sizes_seed, 64, o_range, v_range)
    insts = _recipe_instances(dev, sizes, 1000)
    opts = P.Options(precision=P.SPLIT_BF16, n_abatch=8)
    P.batched(insts, P.DO_FORWARD | P.DO_ADJOINT, opts=opts)
    torch.cuda.synchronize()
    for d in insts:
        o, v, n = d["o"], d["v"], d["n"]
        R1, E1 = P.forward(d["L"], d["tau"], d["tbar"], o=o, v=v, n=n, opts=opts)
        X1 = P.adjoint(d["L"], d["tau"], d["tbar"], o=o, v=v, n=n, opts=opts)
        torch.cuda.synchronize()
        assert torch.equal(d["R"], R1) and torch.equal(d["E"], E1) and torch.equal(d["X"], X1), (o, v, n)
        del R1, E1, X1
    small = sorted(range(64), key=lambda m: sizes[m][1] ** 4 * (sizes[m][2] + sizes[m][0] ** 2))[:4]
    for m in small:
        d = insts[m]
        o, v, n = d["o"], d["v"], d["n"]
        Lh, th, wh = (d[k].cpu().numpy() for k in ("L", "tau", "tbar"))
        Rr, Er = oracle.matrix.forward(o, v, n, Lh, th, wh)
        Xr = oracle.matrix.adjoint(o, v, n, Lh, th, wh)
        eR, eE, eX = err_norm(d["R"].cpu().numpy(), Rr), err_rel(float(d["E"].cpu()), Er), err_norm(d["X"].cpu().numpy(), Xr)
        print("batched instance %d (%d, %d, %d): err_R %.2e err_E %.2e err_X %.2e" % (m, o, v, n, eR, eE, eX))
        assert eR <= SPLIT_TOL_RX and eE <= SPLIT_TOL_E and eX <= SPLIT_TOL_RX


def test_batched_graph_replay_sees_new_data(dev):
    """The second call with the same shapes and pointers replays the captured graph;
    it must compute on the current contents of the inputs."""
    shapes = [(3, 14, 20), (2, 21, 13), (4, 9, 30)]
    insts, _ = _instances(dev, shapes, 400)
    P.batched(insts, P.DO_FORWARD | P.DO_ADJOINT)
    first = [(d["R"].clone(), d["E"].clone(), d["X"].clone()) for d in insts]
    for d in insts:
        d["tau"].mul_(2.0)   # same pointers, new data
    P.batched(insts, P.DO_FORWARD | P.DO_ADJOINT)
    torch.cuda.synchronize()
    for d, (R0, E0, X0) in zip(insts, first):
        assert torch.allclose(d["R"], 2.0 * R0, rtol=1e-13, atol=0)
        assert torch.allclose(d["X"], 2.0 * X0, rtol=1e-13, atol=0)
        assert torch.allclose(d["E"], 2.0 * E0, rtol=1e-13, atol=0)
    for _ in range(3):  # replays interleaved with eager work stay correct
        P.batched(insts, P.DO_FORWARD)
        R1, _ = P.forward(insts[0]["L"], insts[0]["tau"], insts[0]["tbar"], o=3, v=14, n=20)
        torch.cuda.synchronize()
        assert torch.equal(insts[0]["R"], R1)


def test_batched_forward_only_leaves_X_alone(dev):
    shapes = [(2, 10, 12), (3, 7, 9)]
    insts, _ = _instances(dev, shapes, 500)
    for d in insts:
        d["X"].fill_(7.0)
    P.batched(insts, P.DO_FORWARD)
    torch.cuda.synchronize()
    assert all(bool((d["X"] == 7.0).all()) for d in insts)


def test_autograd_workload_split_forward(dev):
    """o=40, v=350, n=1200, seed 5: LadderEnergy with the split forward and the
    hand-written adjoint.  Checked against the oracle gradient on 200 random
    (J, a, c) entries, against central differences of the FP64 GPU energy on a few
    entries, and E against the FP64 path."""
    import time
    o, v, n = 40, 350, 1200
    t0 = time.time()
    L, tau, tbar, _, _ = oracle.make_inputs(o, v, n, 5)
    print("autograd workload: inputs in %.1fs" % (time.time() - t0), flush=True)
    Lg = g(L, dev).requires_grad_(True)
    tg, wg = g(tau, dev), g(tbar, dev)
    E = P.ladder_energy(Lg, tg, wg, (o, v, n), SPLIT5)
    E.backward()
    X = Lg.grad.detach().cpu().numpy()
    E64 = float(P.forward(Lg.detach(), tg, wg, o=o, v=v, n=n)[1].cpu())
    print("autograd workload: E split %.17g fp64 %.17g rel %.2e" % (float(E.detach()), E64, err_rel(float(E.detach()), E64)))
    assert err_rel(float(E.detach()), E64) <= SPLIT_TOL_E
    rng = np.random.default_rng(5)
    ac = np.stack([rng.integers(v, size=200), rng.integers(v, size=200)], axis=1)
    J = rng.integers(n, size=200)
    t0 = time.time()
    Xs = oracle.X_sample(o, v, n, L, tau, tbar, ac)
    print("autograd workload: 200 oracle gradient rows in %.1fs" % (time.time() - t0), flush=True)
    got = X[ac[:, 0], ac[:, 1], J]
    ref = Xs[np.arange(200), J]
    scale = np.abs(Xs).max()
    print("autograd workload: max |X - X_oracle| / max|X_oracle rows| = %.2e" % (np.abs(got - ref).max() / scale))
    assert np.abs(got - ref).max() <= SPLIT_TOL_RX * scale
    # whole rows too: every J of the sampled (a, c)
    assert np.abs(X[ac[:, 0], ac[:, 1], :] - Xs).max() <= SPLIT_TOL_RX * scale
    h = 1e-6
    Ld = Lg.detach()
    for k in range(4):
        a, c, j = int(ac[k, 0]), int(ac[k, 1]), int(J[k])
        Lp = Ld.clone(); Lp[a, c, j] += h
        Lm = Ld.clone(); Lm[a, c, j] -= h
        Ep = float(P.forward(Lp, tg, wg, o=o, v=v, n=n)[1].cpu())
        Em = float(P.forward(Lm, tg, wg, o=o, v=v, n=n)[1].cpu())
        fd = (Ep - Em) / (2 * h)
        print("autograd workload: FD (%d,%d,%d) %.12e  X %.12e" % (a, c, j, fd, X[a, c, j]))
        assert abs(fd - X[a, c, j]) <= 1e-6 * scale


# ------------------------------------------------------------------ transposed ladder (dE/dtau)
def run_tg(dev, o, v, n, L, w, opts=None, beta=0.0, G0=None):
    Gg = None if G0 is None else g(G0, dev)
    G = P.tau_gradient(g(L, dev), g(w, dev), o=o, v=v, n=n, G=Gg, beta=beta, opts=opts)
    torch.cuda.synchronize()
    return G.cpu().numpy()


@pytest.mark.parametrize("flags", PATHS)
@pytest.mark.parametrize("o,v,n,seed", [(2, 5, 3, 31), (3, 4, 2, 32), (1, 3, 1, 33)])
def test_tau_gradient_integer_bitwise(dev, o, v, n, seed, flags):
    L, _, w = integer_inputs(seed, o, v, n)  # L is not symmetric in (a, c)
    assert not np.array_equal(L, L.transpose(1, 0, 2)) or v == 1
    for S in (0, 3):
        opts = P.Options(flags=flags) if S == 0 else P.Options(precision=P.SPLIT_BF16, n_slices=S, flags=flags)
        G = run_tg(dev, o, v, n, L, w, opts)
        assert np.array_equal(G, oracle.tau_gradient(o, v, n, L, w)), S


@pytest.mark.parametrize("flags", PATHS)
@pytest.mark.parametrize("o,v,n,nA", [(4, 20, 60, 0), (5, 37, 70, 4), (2, 129, 17, 64), (1, 23, 9, 5)])
def test_tau_gradient_matches_oracle(dev, o, v, n, nA, flags):
    L, _, w = gaussian_inputs(34 + v, o, v, n)
    Gr = oracle.tau_gradient(o, v, n, L, w)
    G = run_tg(dev, o, v, n, L, w, P.Options(flags=flags, n_abatch=nA))
    Gs = run_tg(dev, o, v, n, L, w, P.Options(precision=P.SPLIT_BF16, n_slices=5, flags=flags, n_abatch=nA))
    print("tau_gradient o=%d v=%d n=%d: fp64 %.3e split %.3e" % (o, v, n, err_norm(G, Gr), err_norm(Gs, Gr)))
    assert err_norm(G, Gr) <= TOL
    assert err_norm(Gs, Gr) <= SPLIT_TOL_RX


def test_tau_gradient_general_flag_and_beta(dev):
    o, v, n = 3, 17, 23
    L, _, w = gaussian_inputs(35, o, v, n, symmetric=False)
    Gr = oracle.tau_gradient(o, v, n, L, w)
    G0 = np.random.default_rng(36).standard_normal((o, o, v, v))
    G = run_tg(dev, o, v, n, L, w, P.Options(flags=P.FLAG_GENERAL), beta=-0.5, G0=G0)
    assert err_norm(G, Gr - 0.5 * G0) <= TOL


def test_autograd_tau_gradient(dev):
    """dE/dtau from ladder_energy's backward equals the oracle's transposed ladder."""
    o, v, n = 3, 21, 25
    L, tau, w = gaussian_inputs(37, o, v, n)
    tg = g(tau, dev).requires_grad_(True)
    Lg = g(L, dev).requires_grad_(True)
    E = P.ladder_energy(Lg, tg, g(w, dev), (o, v, n))
    (2.0 * E).backward()
    Gr = oracle.tau_gradient(o, v, n, L, w)
    Xr = oracle.adjoint(o, v, n, L, tau, w)
    assert err_norm(tg.grad.cpu().numpy(), 2.0 * Gr) <= TOL
    assert err_norm(Lg.grad.cpu().numpy(), 2.0 * Xr) <= TOL
    # E is linear in tau: <tau, dE/dtau> = E
    assert err_rel(float((tg.detach() * tg.grad).sum()) / 2.0, float(E.detach())) <= TOL


def test_tau_gradient_autograd_workload_sampled(dev):
    """o=40, v=350, n=1200 (the autograd workload): split path, rows c sampled against the oracle."""
    o, v, n = 40, 350, 1200
    L, tau, tbar, _, _ = oracle.make_inputs(o, v, n, 5)
    G = run_tg(dev, o, v, n, L, tbar, P.Options(precision=P.SPLIT_BF16))
    rows = [0, 1, 117, 349]
    for c in rows:
        Gr = oracle.matrix.tau_gradient(o, v, n, L, tbar, c_range=(c, c + 1))
        e = err_norm(G[:, :, c:c + 1, :], Gr)
        print("tau_gradient autograd workload row c=%d: err %.3e" % (c, e))
        assert e <= SPLIT_TOL_RX


# ------------------------------------------------------------------ gradient intermediates W, V, Wmo
@pytest.mark.parametrize("flags", PATHS)
@pytest.mark.parametrize("o,v,n,seed", [(3, 7, 5, 71), (4, 20, 60, 72), (2, 41, 33, 73)])
def test_w_intermediate_matches_oracle(dev, o, v, n, seed, flags):
    _, tau, w = gaussian_inputs(seed, o, v, n)
    Z = np.random.default_rng(seed + 100).standard_normal((v, v, n))
    Wr = oracle.w_intermediate(o, v, n, Z, tau, w)
    for opts, tol in ((P.Options(flags=flags), TOL), (P.Options(precision=P.SPLIT_BF16, flags=flags), SPLIT_TOL_RX)):
        W = P.w_intermediate(g(Z, dev), g(tau, dev), g(w, dev), o=o, v=v, n=n, opts=opts).cpu().numpy()
        print("W o=%d v=%d n=%d precision=%d: err %.3e" % (o, v, n, opts.precision, err_norm(W, Wr)))
        assert err_norm(W, Wr) <= tol


@pytest.mark.parametrize("v,n,seed", [(1, 1, 74), (3, 2, 75), (20, 60, 76), (37, 70, 77), (129, 17, 78)])
def test_metric_and_back_transform_integer_bitwise(dev, v, n, seed):
    rng = np.random.default_rng(seed)
    Z, W = (rng.integers(-5, 6, (v, v, n)).astype(float) for _ in range(2))
    x, y = (rng.integers(-3, 4, (v, v)).astype(float) for _ in range(2))
    V = P.metric_contraction(g(Z, dev), g(W, dev), v=v, n=n).cpu().numpy()
    assert np.array_equal(V, oracle.metric_contraction(v, n, Z, W))
    Wmo = P.back_transform(g(x, dev), g(y, dev), g(W, dev), v=v, n=n).cpu().numpy()
    assert np.array_equal(Wmo, oracle.back_transform(v, n, x, y, W))


@pytest.mark.parametrize("v,n,seed", [(20, 60, 79), (150, 600, 80), (131, 257, 81)])
def test_metric_and_back_transform_match_oracle(dev, v, n, seed):
    rng = np.random.default_rng(seed)
    Z, W = rng.standard_normal((v, v, n)), rng.standard_normal((v, v, n))
    x, y = rng.standard_normal((v, v)) / np.sqrt(v), rng.standard_normal((v, v)) / np.sqrt(v)
    V0, W0 = rng.standard_normal((n, n)), rng.standard_normal((v, v, n))
    V = P.metric_contraction(g(Z, dev), g(W, dev), v=v, n=n, V=g(V0, dev), alpha=2.0, beta=-1.0).cpu().numpy()
    Vr = 2.0 * oracle.matrix.metric_contraction(v, n, Z, W) - V0
    Wmo = P.back_transform(g(x, dev), g(y, dev), g(W, dev), v=v, n=n, Wmo=g(W0, dev), alpha=0.5, beta=3.0)
    Wr = 0.5 * oracle.matrix.back_transform(v, n, x, y, W) + 3.0 * W0
    print("v=%d n=%d: err V %.3e err Wmo %.3e" % (v, n, err_norm(V, Vr), err_norm(Wmo.cpu().numpy(), Wr)))
    assert err_norm(V, Vr) <= TOL and err_norm(Wmo.cpu().numpy(), Wr) <= TOL


def test_metric_and_back_transform_retinal_sampled(dev):
    """v=657, n=2200 (the retinal shape): sampled blocks of V and slices K of Wmo against the oracle."""
    v, n = 657, 2200
    gen = torch.Generator(device=dev)
    gen.manual_seed(82)
    Z = torch.randn((v, v, n), dtype=torch.float64, device=dev, generator=gen)
    W = torch.randn((v, v, n), dtype=torch.float64, device=dev, generator=gen)
    x = torch.randn((v, v), dtype=torch.float64, device=dev, generator=gen) / v ** 0.5
    y = torch.randn((v, v), dtype=torch.float64, device=dev, generator=gen) / v ** 0.5
    V = P.metric_contraction(Z, W, v=v, n=n).cpu().numpy()
    Wmo = P.back_transform(x, y, W, v=v, n=n)
    torch.cuda.synchronize()
    cols = [0, 1, 977, 2199]
    Zs = Z[:, :, cols].cpu().numpy()
    Ws = W[:, :, cols].cpu().numpy()
    Vr = oracle.matrix.metric_contraction(v, len(cols), Zs, Ws)
    eV = err_norm(V[np.ix_(cols, cols)], Vr)
    xh, yh = x.cpu().numpy(), y.cpu().numpy()
    eW = 0.0
    for K in (0, 1500, 2199):
        Wr = oracle.matrix.back_transform(v, 1, xh, yh, W[:, :, K:K + 1].cpu().numpy())
        eW = max(eW, err_norm(Wmo[:, :, K:K + 1].cpu().numpy(), Wr))
    print("retinal shape: err V %.3e err Wmo %.3e" % (eV, eW))
    assert eV <= TOL and eW <= TOL


# ------------------------------------------------------------------ excited-state V^4 density
@pytest.mark.parametrize("mode", [P.U_TABLE, P.U_APPENDIX])
def test_excited_amplitudes_and_density(dev, mode):
    """U on the GPU equals the oracle's (dyadic inputs: exact), and the excited-state V^4
    contribution ladder_adjoint(L, U, L2) matches the oracle chain."""
    o, v, n = 4, 20, 30
    rng = np.random.default_rng(90 + mode)
    T = np.round(rng.standard_normal((o, o, v, v)) * 64) / 64
    R2 = np.round(rng.standard_normal((o, o, v, v)) * 64) / 64
    T, R2 = 0.5 * (T + T.transpose(1, 0, 3, 2)), 0.5 * (R2 + R2.transpose(1, 0, 3, 2))
    U = P.excited_amplitudes(g(T, dev), g(R2, dev), 0.75, o=o, v=v, mode=mode).cpu().numpy()
    Ur = oracle.excited_amplitudes(o, v, 0.75, T, R2, mode)
    assert np.array_equal(U, Ur)
    L, _, L2 = gaussian_inputs(92, o, v, n)
    X = P.adjoint(g(L, dev), g(U, dev), g(L2, dev), o=o, v=v, n=n).cpu().numpy()
    Xr = oracle.adjoint(o, v, n, L, Ur, L2)
    assert err_norm(X, Xr) <= TOL
    # in place: U written over T
    Tg = g(T, dev)
    P.excited_amplitudes(Tg, g(R2, dev), 0.75, o=o, v=v, mode=mode, U=Tg)
    assert np.array_equal(Tg.cpu().numpy(), Ur)


# ------------------------------------------------------------------ excited-state OV^3 density d_abci
def ov3_inputs(seed, o, v, n, integer=False):
    rng = np.random.default_rng(seed)
    if integer:
        return (rng.integers(-3, 4, (o, o, v, v)).astype(float), rng.integers(-3, 4, (o, v)).astype(float),
                rng.integers(-3, 4, (v, v, n)).astype(float), rng.integers(-3, 4, (v, o, n)).astype(float))
    return (rng.standard_normal((o, o, v, v)), rng.standard_normal((o, v)), rng.standard_normal((v, v, n)),
            rng.standard_normal((v, o, n)))


@pytest.mark.parametrize("o,v,n,seed", [(1, 1, 1, 110), (2, 3, 2, 111), (3, 7, 5, 112), (5, 33, 17, 113),
                                        (4, 130, 9, 114), (9, 20, 131, 115)])
def test_ov3_abci_integer_bitwise(dev, o, v, n, seed):
    """Integer inputs: every sum is exact on both sides, so Wab and Wci equal the oracle's
    (density formed element by element) bit for bit; shapes span several 128 tiles and ragged tails."""
    L2, R1, Zvv, Zvo = ov3_inputs(seed, o, v, n, integer=True)
    Wab, Wci = P.ov3_abci(g(L2, dev), g(R1, dev), g(Zvv, dev), g(Zvo, dev), o=o, v=v, n=n)
    Wab_r, Wci_r = oracle.ov3_abci(o, v, n, L2, R1, Zvv, Zvo)
    assert np.array_equal(Wab.cpu().numpy(), Wab_r)
    assert np.array_equal(Wci.cpu().numpy(), Wci_r)


@pytest.mark.parametrize("o,v,n,seed", [(4, 20, 60, 116), (6, 45, 70, 117), (3, 129, 130, 118)])
def test_ov3_abci_matches_oracle(dev, o, v, n, seed):
    """Gaussian inputs with alpha, beta; each side alone (the other output and its Z NULL)
    gives the same result as both together."""
    L2, R1, Zvv, Zvo = ov3_inputs(seed, o, v, n)
    rng = np.random.default_rng(seed + 1)
    A0, C0 = rng.standard_normal((v, v, n)), rng.standard_normal((v, o, n))
    Wab_r, Wci_r = oracle.matrix.ov3_abci(o, v, n, L2, R1, Zvv, Zvo)
    Wab, Wci = P.ov3_abci(g(L2, dev), g(R1, dev), g(Zvv, dev), g(Zvo, dev), o=o, v=v, n=n, Wab=g(A0, dev),
                          Wci=g(C0, dev), alpha=-0.5, beta=2.0)
    ea, ec = err_norm(Wab.cpu().numpy(), 2.0 * A0 - 0.5 * Wab_r), err_norm(Wci.cpu().numpy(), 2.0 * C0 - 0.5 * Wci_r)
    print("OV3 o=%d v=%d n=%d: err Wab %.3e err Wci %.3e" % (o, v, n, ea, ec))
    assert ea <= TOL and ec <= TOL
    a_only, none = P.ov3_abci(g(L2, dev), g(R1, dev), None, g(Zvo, dev), o=o, v=v, n=n, want=(True, False))
    assert none is None and err_norm(a_only.cpu().numpy(), Wab_r) <= TOL
    none, c_only = P.ov3_abci(g(L2, dev), g(R1, dev), g(Zvv, dev), None, o=o, v=v, n=n, want=(False, True))
    assert none is None and err_norm(c_only.cpu().numpy(), Wci_r) <= TOL


@pytest.mark.parametrize("pairs,n,seed", [(1, 1, 119), (35, 17, 120), (300, 129, 121)])
def test_metric_contraction_pairs_bitwise(dev, pairs, n, seed):
    rng = np.random.default_rng(seed)
    Z, W, V0 = (rng.integers(-5, 6, s).astype(float) for s in ((pairs, n), (pairs, n), (n, n)))
    V = P.metric_contraction_pairs(g(Z, dev), g(W, dev), pairs=pairs, n=n, V=g(V0, dev), alpha=2.0, beta=-1.0)
    assert np.array_equal(V.cpu().numpy(), 2.0 * oracle.metric_contraction_pairs(pairs, n, Z, W) - V0)


def test_ov3_abci_retinal_sampled(dev):
    """o=78, v=657, n=2200 (the retinal shape, the launch the benchmark times): sampled rows of
    Wab and Wci against the oracle one by one, and the identity sum Zvv*Wab = sum Zvo*Wci
    (both are sum_abci d_abci (ab|ci) with (ab|ci) = sum_K Zvv^K_ab Zvo^K_ci)."""
    o, v, n = 78, 657, 2200
    gen = torch.Generator(device=dev)
    gen.manual_seed(122)
    L2 = torch.randn((o, o, v, v), dtype=torch.float64, device=dev, generator=gen)
    R1 = torch.randn((o, v), dtype=torch.float64, device=dev, generator=gen)
    Zvv = torch.randn((v, v, n), dtype=torch.float64, device=dev, generator=gen)
    Zvo = torch.randn((v, o, n), dtype=torch.float64, device=dev, generator=gen)
    Wab, Wci = P.ov3_abci(L2, R1, Zvv, Zvo, o=o, v=v, n=n)
    torch.cuda.synchronize()
    s_ab, s_ci = float((Zvv * Wab).sum()), float((Zvo * Wci).sum())
    L2h, R1h, Zvvh, Zvoh = L2.cpu().numpy(), R1.cpu().numpy(), Zvv.cpu().numpy(), Zvo.cpu().numpy()
    ab = np.array([[0, 0], [656, 1], [300, 656], [77, 78]])
    ci = np.array([[0, 0], [656, 77], [123, 40]])
    ra = oracle.ov3_abci_wab(o, v, n, L2h, R1h, Zvoh, ab)
    rc = oracle.ov3_abci_wci(o, v, n, L2h, R1h, Zvvh, ci)
    ea = err_norm(Wab[ab[:, 0], ab[:, 1]].cpu().numpy(), ra)
    ec = err_norm(Wci[ci[:, 0], ci[:, 1]].cpu().numpy(), rc)
    ident = abs(s_ab - s_ci) / (float((Zvv * Wab).abs().sum()))
    print("OV3 retinal shape: err Wab %.3e err Wci %.3e identity %.3e" % (ea, ec, ident))
    assert ea <= TOL and ec <= TOL and ident <= 1e-12


# ------------------------------------------------------------------ excited-state OV^3 density d_abic
def abic_inputs(seed, o, v, n, integer=False):
    rng = np.random.default_rng(seed)
    draw = (lambda *s: rng.integers(-2, 3, s).astype(float)) if integer else (lambda *s: rng.standard_normal(s))
    return dict(R0=0.5 if integer else 0.625, L1=draw(o, v), L2=draw(o, o, v, v), T=draw(o, o, v, v), R1=draw(o, v),
                R2=draw(o, o, v, v), Zvv=draw(v, v, n), Zov=draw(o, v, n))


def gpu_abic(dev, o, v, n, x, **kw):
    return P.ov3_abic(x["R0"], *(g(x[k], dev) if x.get(k) is not None else None
                                 for k in ("L1", "L2", "T", "R1", "R2", "Zvv", "Zov")), o=o, v=v, n=n, **kw)


@pytest.mark.parametrize("o,v,n,seed", [(1, 1, 1, 140), (2, 3, 2, 141), (3, 7, 5, 142), (9, 6, 4, 143),
                                        (10, 13, 3, 144), (4, 33, 17, 145)])
def test_ov3_abic_integer_bitwise(dev, o, v, n, seed):
    """Integer inputs: every intermediate and sum is an exact integer on both sides, so Wab and Wic
    equal the oracle's (Appendix A density formed element by element) bit for bit; o = 9, 10 run
    the S_iacb slab over a full and a ragged group of occupied indices."""
    x = abic_inputs(seed, o, v, n, integer=True)
    Wab, Wic = gpu_abic(dev, o, v, n, x)
    ra, rc = oracle.ov3_abic(o, v, n, x["R0"], x["L1"], x["L2"], x["T"], x["R1"], x["R2"], x["Zvv"], x["Zov"])
    assert np.array_equal(Wab.cpu().numpy(), ra)
    assert np.array_equal(Wic.cpu().numpy(), rc)


@pytest.mark.parametrize("o,v,n,seed", [(4, 20, 30, 146), (11, 17, 40, 147), (3, 130, 9, 148)])
def test_ov3_abic_matches_oracle(dev, o, v, n, seed):
    """Gaussian inputs with alpha and beta; each side alone gives the same as both together."""
    x = abic_inputs(seed, o, v, n)
    rng = np.random.default_rng(seed + 1)
    A0, C0 = rng.standard_normal((v, v, n)), rng.standard_normal((o, v, n))
    ra, rc = oracle.matrix.ov3_abic(o, v, n, x["R0"], x["L1"], x["L2"], x["T"], x["R1"], x["R2"], x["Zvv"], x["Zov"])
    Wab, Wic = gpu_abic(dev, o, v, n, x, Wab=g(A0, dev), Wic=g(C0, dev), alpha=1.5, beta=-1.0)
    ea, ec = err_norm(Wab.cpu().numpy(), 1.5 * ra - A0), err_norm(Wic.cpu().numpy(), 1.5 * rc - C0)
    print("d_abic o=%d v=%d n=%d: err Wab %.3e err Wic %.3e" % (o, v, n, ea, ec))
    assert ea <= TOL and ec <= TOL
    y = dict(x); y["Zvv"] = None
    a_only, none = gpu_abic(dev, o, v, n, y, want=(True, False))
    assert none is None and err_norm(a_only.cpu().numpy(), ra) <= TOL
    y = dict(x); y["Zov"] = None
    none, c_only = gpu_abic(dev, o, v, n, y, want=(False, True))
    assert none is None and err_norm(c_only.cpu().numpy(), rc) <= TOL


def test_ov3_abic_medium_and_identity(dev):
    """o=20, v=150, n=600 (the medium workload) in full against the numpy oracle, and the
    identity sum Zvv*Wab = sum Zov*Wic that holds at any size."""
    o, v, n = 20, 150, 600
    x = abic_inputs(149, o, v, n)
    x["L2"] *= 0.1; x["T"] *= 0.1; x["R2"] *= 0.1
    ra, rc = oracle.matrix.ov3_abic(o, v, n, x["R0"], x["L1"], x["L2"], x["T"], x["R1"], x["R2"], x["Zvv"], x["Zov"])
    Wab, Wic = gpu_abic(dev, o, v, n, x)
    Wab, Wic = Wab.cpu().numpy(), Wic.cpu().numpy()
    ea, ec = err_norm(Wab, ra), err_norm(Wic, rc)
    ident = abs(np.sum(x["Zvv"] * Wab) - np.sum(x["Zov"] * Wic)) / np.sum(np.abs(x["Zvv"] * Wab))
    print("d_abic medium: err Wab %.3e err Wic %.3e identity %.3e" % (ea, ec, ident))
    assert ea <= TOL and ec <= TOL and ident <= 1e-12


@pytest.mark.parametrize("o,v,n,seed", [(2, 3, 2, 150), (9, 6, 4, 151), (4, 33, 17, 152)])
def test_ov3_abic_split_integer_bitwise(dev, o, v, n, seed):
    """Split BF16 for the o^3 v^3 products: small integers are exact in the slices and every
    chunk sum is exact, so the result is still bitwise the oracle's."""
    x = abic_inputs(seed, o, v, n, integer=True)
    Wab, Wic = gpu_abic(dev, o, v, n, x, opts=P.Options(precision=P.SPLIT_BF16))
    ra, rc = oracle.ov3_abic(o, v, n, x["R0"], x["L1"], x["L2"], x["T"], x["R1"], x["R2"], x["Zvv"], x["Zov"])
    assert np.array_equal(Wab.cpu().numpy(), ra)
    assert np.array_equal(Wic.cpu().numpy(), rc)


def test_ov3_abic_split_medium(dev):
    """Split BF16 (S = 5) on the medium workload against the numpy oracle, in full."""
    o, v, n = 20, 150, 600
    x = abic_inputs(153, o, v, n)
    ra, rc = oracle.matrix.ov3_abic(o, v, n, x["R0"], x["L1"], x["L2"], x["T"], x["R1"], x["R2"], x["Zvv"], x["Zov"])
    Wab, Wic = gpu_abic(dev, o, v, n, x, opts=P.Options(precision=P.SPLIT_BF16))
    ea, ec = err_norm(Wab.cpu().numpy(), ra), err_norm(Wic.cpu().numpy(), rc)
    print("d_abic split medium: err Wab %.3e err Wic %.3e" % (ea, ec))
    assert ea <= SPLIT_TOL_RX and ec <= SPLIT_TOL_RX


# ------------------------------------------------------------------ autotuned batch size
@pytest.mark.parametrize("precision", [P.FP64, P.SPLIT_BF16])
def test_autotune_then_default_calls_use_it(dev, tmp_path, precision):
    """The tuner picks a batch size within the workspace it is given, writes a cache line that
    reloads, and the following default calls (n_abatch = 0) run that plan and still match the oracle."""
    o, v, n = 5, 53, 70
    L, tau, w = gaussian_inputs(95, o, v, n)
    Lg, tg, wg = g(L, dev), g(tau, dev), g(w, dev)
    opts = P.Options(precision=precision)
    P.autotune_reset()
    cap = (v + 3) // 4
    ws = torch.empty(P.workspace_size(o, v, n, P.Options(precision=precision, n_abatch=cap)), dtype=torch.uint8,
                     device=dev)
    cache = tmp_path / "tune.jsonl"
    nA = P.autotune(Lg, tg, wg, o=o, v=v, n=n, ws=ws, opts=opts, cache_path=str(cache))
    assert 1 <= nA <= cap
    line = cache.read_text().strip().splitlines()[-1]
    assert '"n_abatch": %d' % nA in line and '"v": 53' in line
    assert P.workspace_size(o, v, n, opts) <= ws.numel()
    R, E, X = run(dev, o, v, n, L, tau, w, opts)
    Rr, Er = oracle.forward(o, v, n, L, tau, w)
    Xr = oracle.adjoint(o, v, n, L, tau, w)
    tol_rx, tol_e = (TOL, TOL) if precision == P.FP64 else (SPLIT_TOL_RX, None)
    assert err_norm(R, Rr) <= tol_rx and err_norm(X, Xr) <= tol_rx
    if tol_e is None:
        assert err_E_terms(E, Er, w, Rr) <= SPLIT_TOL_E
    else:
        assert err_rel(E, Er) <= tol_e
    P.autotune_reset()
    assert P.autotune_load(str(cache)) == 1
    P.autotune_reset()


def test_batched_after_retune_uses_new_sizes_and_stays_correct(dev):
    """A tuned batch size for one instance shape changes that instance's plan inside the
    ragged batch (the graph is recaptured, not replayed) and the results stay right."""
    shapes = [(3, 14, 20), (2, 21, 13), (4, 9, 30)]
    insts, refs = _instances(dev, shapes, 420)
    P.autotune_reset()
    ws0 = P.batched_workspace_size(insts)
    P.batched(insts, P.DO_FORWARD | P.DO_ADJOINT)
    d = insts[1]
    ws = torch.empty(P.workspace_size(d["o"], d["v"], d["n"], P.Options(n_abatch=6)), dtype=torch.uint8, device=dev)
    nA = P.autotune(d["L"], d["tau"], d["tbar"], o=d["o"], v=d["v"], n=d["n"], ws=ws)
    assert 1 <= nA <= 6
    P.batched(insts, P.DO_FORWARD | P.DO_ADJOINT)
    torch.cuda.synchronize()
    for dd, (L, tau, w) in zip(insts, refs):
        o, v, n = dd["o"], dd["v"], dd["n"]
        Rr, Er = oracle.forward(o, v, n, L, tau, w)
        Xr = oracle.adjoint(o, v, n, L, tau, w)
        assert err_norm(dd["R"].cpu().numpy(), Rr) <= TOL and err_norm(dd["X"].cpu().numpy(), Xr) <= TOL
        assert err_rel(float(dd["E"]), Er) <= TOL
    P.autotune_reset()
    assert P.batched_workspace_size(insts) == ws0
