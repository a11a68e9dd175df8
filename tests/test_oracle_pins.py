"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these re-types the oracle's loops: each checks it against an independent
route (hand-derived example, exact integer brute force, a matrix-product closed
form, invariants of the definitions, finite differences) chosen so that a dropped
term, a wrong index or a transposed operand in the oracle fails at least one.
"""
import json
import os

import numpy as np
import pytest

import synthetic

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


class _Matrix:
    """The numpy matrix-product implementation behind the same interface."""

    def __init__(self, c):
        import oracle
        self._m = oracle.matrix
        self._c = c

    def forward(self, o, v, n, L, tau, tbar=None):
        return self._m.forward(o, v, n, L, tau, tbar)

    def adjoint(self, o, v, n, L, tau, w):
        return self._m.adjoint(o, v, n, L, tau, w)

    def tau_gradient(self, o, v, n, L, w):
        return self._m.tau_gradient(o, v, n, L, w)

    def __getattr__(self, name):
        return getattr(self._c, name)


@pytest.fixture(params=["c", "matrix"])
def impl(request, oracle_lib):
    return oracle_lib if request.param == "c" else _Matrix(oracle_lib)


def rnd(seed, *shape):
    return np.random.default_rng(seed).standard_normal(shape)


def pair_sym(x):
    """(x_ij^ab + x_ji^ba)/2: pair-symmetric part."""
    return 0.5 * (x + x.transpose(1, 0, 3, 2))


# ---------------------------------------------------------------- worked example
def test_micro_example(impl):
    g = json.load(open(os.path.join(GOLDEN, "micro_example.json")))
    o, v, n = g["o"], g["v"], g["n"]
    L = np.array(g["L"]); tau = np.array(g["tau"]); tbar = np.array(g["tbar"])
    R, E = impl.forward(o, v, n, L, tau, tbar)
    X = impl.adjoint(o, v, n, L, tau, tbar)
    assert np.array_equal(R, np.array(g["R"]))
    assert E == g["E"]
    assert np.array_equal(X, np.array(g["X"]))


# ---------------------------------------------------------------- exact brute force
def _brute_int(o, v, n, L, tau, w):
    """Six nested loops over the full 4-index g in exact Python integers."""
    g = [[[[sum(L[a][c][J] * L[b][d][J] for J in range(n)) for d in range(v)] for c in range(v)]
          for b in range(v)] for a in range(v)]  # g[a][b][c][d] = (ac|bd)
    R = [[[[sum(g[a][b][c][d] * tau[i][j][c][d] for c in range(v) for d in range(v))
            for b in range(v)] for a in range(v)] for j in range(o)] for i in range(o)]
    E = sum(w[i][j][a][b] * R[i][j][a][b] for i in range(o) for j in range(o) for a in range(v) for b in range(v))
    # X^J_pq = dE/dL^J_pq by the product rule on g_acbd = sum_J L^J_ac L^J_bd:
    # L^J_pq enters as the first factor when (a,c) = (p,q) and as the second when (b,d) = (p,q).
    X = [[[0] * n for _ in range(v)] for _ in range(v)]
    for i in range(o):
        for j in range(o):
            for a in range(v):
                for b in range(v):
                    for c in range(v):
                        for d in range(v):
                            f = w[i][j][a][b] * tau[i][j][c][d]
                            if f == 0:
                                continue
                            for J in range(n):
                                X[a][c][J] += f * L[b][d][J]
                                X[b][d][J] += f * L[a][c][J]
    return R, E, X


@pytest.mark.parametrize("seed,o,v,n", [(11, 2, 3, 2), (12, 1, 4, 3), (13, 3, 2, 1)])
def test_integer_exact_brute_force(impl, seed, o, v, n):
    rng = np.random.default_rng(seed)
    L = rng.integers(-7, 8, size=(v, v, n))
    tau = rng.integers(-7, 8, size=(o, o, v, v))
    w = rng.integers(-7, 8, size=(o, o, v, v))  # deliberately neither symmetric
    R_ref, E_ref, X_ref = _brute_int(o, v, n, L.tolist(), tau.tolist(), w.tolist())
    R, E = impl.forward(o, v, n, L.astype(float), tau.astype(float), w.astype(float))
    X = impl.adjoint(o, v, n, L.astype(float), tau.astype(float), w.astype(float))
    assert np.array_equal(R, np.array(R_ref, dtype=float))
    assert E == float(E_ref)
    assert np.array_equal(X, np.array(X_ref, dtype=float))


# ---------------------------------------------------------------- matrix closed forms
def test_matrix_closed_form(impl):
    o, v, n = 3, 7, 5
    L, tau, w = rnd(1, v, v, n), rnd(2, o, o, v, v), rnd(3, o, o, v, v)
    R, E = impl.forward(o, v, n, L, tau, w)
    X = impl.adjoint(o, v, n, L, tau, w)
    Lj = [np.ascontiguousarray(L[:, :, J]) for J in range(n)]
    R_ref = np.zeros_like(R)
    X_ref = np.zeros_like(X)
    for i in range(o):
        for j in range(o):
            T, W = tau[i, j], w[i, j]
            for J in range(n):
                R_ref[i, j] += Lj[J] @ T @ Lj[J].T                  # R_ij = sum_J L^J T_ij L^J^T
                X_ref[:, :, J] += W @ Lj[J] @ T.T + W.T @ Lj[J] @ T  # X^J = sum_ij W L T^T + W^T L T
    np.testing.assert_allclose(R, R_ref, rtol=0, atol=1e-13 * np.abs(R_ref).max())
    np.testing.assert_allclose(X, X_ref, rtol=0, atol=1e-13 * np.abs(X_ref).max())
    assert abs(E - np.sum(w * R_ref)) <= 1e-13 * np.sum(np.abs(w * R_ref))


def test_rank_one(impl):
    """n=1, L_ac = u_a y_c:  R_ij^ab = u_a u_b (y^T T_ij y)."""
    o, v = 2, 6
    u, y = rnd(4, v), rnd(5, v)
    L = np.einsum("a,c->ac", u, y)[:, :, None]
    tau = rnd(6, o, o, v, v)
    R, _ = impl.forward(o, v, 1, L, tau)
    ref = np.einsum("a,b,ijcd,c,d->ijab", u, u, tau, y, y)
    np.testing.assert_allclose(R, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


def test_zero_inputs(impl):
    o, v, n = 2, 4, 3
    L, tau = rnd(7, v, v, n), rnd(8, o, o, v, v)
    R, E = impl.forward(o, v, n, L, np.zeros_like(tau), tau)
    assert not R.any() and E == 0.0
    R, E = impl.forward(o, v, n, np.zeros_like(L), tau, tau)
    assert not R.any() and E == 0.0
    assert not impl.adjoint(o, v, n, L, tau, np.zeros_like(tau)).any()


# ---------------------------------------------------------------- invariants
def test_pair_symmetry_of_R(impl):
    """tau_ij^ab = tau_ji^ba  =>  R_ij^ab = R_ji^ba for any L (even asymmetric in ac)."""
    o, v, n = 3, 6, 4
    L, tau = rnd(9, v, v, n), pair_sym(rnd(10, o, o, v, v))
    R, _ = impl.forward(o, v, n, L, tau)
    np.testing.assert_allclose(R, R.transpose(1, 0, 3, 2), rtol=0, atol=1e-14 * np.abs(R).max())
    # and the relation is not automatic: it fails for an asymmetric tau
    R2, _ = impl.forward(o, v, n, L, rnd(10, o, o, v, v))
    assert np.abs(R2 - R2.transpose(1, 0, 3, 2)).max() > 1e-3 * np.abs(R2).max()


def test_euler_homogeneity(impl):
    """E is homogeneous of degree 2 in L: sum_{J,ac} L^J_ac X^J_ac = 2E."""
    o, v, n = 3, 5, 4
    L, tau, w = rnd(11, v, v, n), rnd(12, o, o, v, v), rnd(13, o, o, v, v)
    _, E = impl.forward(o, v, n, L, tau, w)
    X = impl.adjoint(o, v, n, L, tau, w)
    assert abs(np.sum(L * X) - 2 * E) <= 1e-13 * np.sum(np.abs(L * X))


def test_scaling_and_bilinearity(impl):
    o, v, n = 2, 5, 3
    L, tau, tau2, w, w2 = rnd(14, v, v, n), rnd(15, o, o, v, v), rnd(16, o, o, v, v), rnd(17, o, o, v, v), rnd(18, o, o, v, v)
    R, E = impl.forward(o, v, n, L, tau, w)
    X = impl.adjoint(o, v, n, L, tau, w)
    Rs, Es = impl.forward(o, v, n, 2.0 * L, tau, w)
    Xs = impl.adjoint(o, v, n, 2.0 * L, tau, w)
    # E is quadratic in L, so its gradient X is linear in L (degree 1, not 3)
    assert np.array_equal(Rs, 4.0 * R) and Es == 4.0 * E and np.array_equal(Xs, 2.0 * X)
    _, Ea = impl.forward(o, v, n, L, tau + 3.0 * tau2, w)
    _, Eb = impl.forward(o, v, n, L, tau2, w)
    _, Ec = impl.forward(o, v, n, L, tau, w2)
    _, Ed = impl.forward(o, v, n, L, tau, w - 0.5 * w2)
    scale = np.abs(R).sum() * np.abs(w).max() * 8
    assert abs(Ea - (E + 3.0 * Eb)) <= 1e-13 * scale
    assert abs(Ed - (E - 0.5 * Ec)) <= 1e-13 * scale


def test_density_route_equals_residual_route(impl):
    """E = sum_abcd (ac|bd) O2_{..} with the V^4 density O^(2) of Appendix A.

    With d_abcd = O^(2)_abcd(L_2, C_2) = L_ij^ac C_ij^bd (Sec. II B, Appendix A;
    R_0 = 1, L_2 = tbar, C_2 = tau) and g_pqrs = (pq|rs) = sum_J L^J_pq L^J_rs,
    the V^4 part of sum_pqrs g_pqrs d_pqrs must equal sum tbar R.
    """
    o, v, n = 3, 5, 4
    L, tau, w = rnd(19, v, v, n), rnd(20, o, o, v, v), rnd(21, o, o, v, v)
    _, E = impl.forward(o, v, n, L, tau, w)
    g = np.einsum("pqJ,rsJ->pqrs", L, L)        # (pq|rs), Mulliken
    d = np.einsum("ijpr,ijqs->pqrs", w, tau)     # O2_pqrs = tbar_ij^pr tau_ij^qs
    E_density = np.einsum("pqrs,pqrs->", g, d)
    assert abs(E - E_density) <= 1e-13 * np.einsum("pqrs,pqrs->", np.abs(g), np.abs(d))


def test_factor_two_form_under_pair_symmetry(impl):
    """d_pqrs = d_rspq (Appendix A): with pair-symmetric tbar and tau,
    X^J_ac = 2 sum_bd L^J_bd D_{ab,cd}, D_{ab,cd} = sum_ij tbar_ij^ab tau_ij^cd."""
    o, v, n = 3, 5, 4
    L, tau, w = rnd(22, v, v, n), pair_sym(rnd(23, o, o, v, v)), pair_sym(rnd(24, o, o, v, v))
    X = impl.adjoint(o, v, n, L, tau, w)
    D = np.einsum("ijab,ijcd->abcd", w, tau)
    X2 = 2.0 * np.einsum("abcd,bdJ->acJ", D, L)
    np.testing.assert_allclose(X, X2, rtol=0, atol=1e-13 * np.abs(X2).max())
    # without pair symmetry the factor-2 form is wrong, and the oracle must not use it
    wa = rnd(25, o, o, v, v)
    Xa = impl.adjoint(o, v, n, L, tau, wa)
    Xa2 = 2.0 * np.einsum("abcd,bdJ->acJ", np.einsum("ijab,ijcd->abcd", wa, tau), L)
    assert np.abs(Xa - Xa2).max() > 1e-3 * np.abs(Xa).max()


# ---------------------------------------------------------------- finite differences
@pytest.mark.parametrize("symmetric", [True, False])
def test_finite_differences(impl, symmetric):
    """E is exactly quadratic along any single L entry, so the central difference
    has zero truncation error and must match X to rounding."""
    o, v, n = 2, 5, 3
    L, tau, w = rnd(26, v, v, n), rnd(27, o, o, v, v), rnd(28, o, o, v, v)
    if symmetric:
        tau, w = pair_sym(tau), pair_sym(w)
    X = impl.adjoint(o, v, n, L, tau, w)
    h = 1e-3
    for (a, c, J) in [(0, 0, 0), (1, 3, 2), (4, 2, 1), (2, 2, 0), (3, 0, 2)]:
        Lp, Lm = L.copy(), L.copy()
        Lp[a, c, J] += h
        Lm[a, c, J] -= h
        fd = (impl.forward(o, v, n, Lp, tau, w)[1] - impl.forward(o, v, n, Lm, tau, w)[1]) / (2 * h)
        assert abs(fd - X[a, c, J]) <= 1e-9 * max(1.0, abs(X).max()), (a, c, J, fd, X[a, c, J])


# ---------------------------------------------------------------- transposed ladder
def test_tau_gradient_contracts_to_energy(impl):
    """E is linear in tau, so sum_ijcd tau_ij^cd dE/dtau_ij^cd = E (generic, non-symmetric L)."""
    o, v, n = 3, 5, 4
    L, tau, w = rnd(41, v, v, n), rnd(42, o, o, v, v), rnd(43, o, o, v, v)
    _, E = impl.forward(o, v, n, L, tau, w)
    G = impl.tau_gradient(o, v, n, L, w)
    assert abs(np.sum(tau * G) - E) <= 1e-13 * np.sum(np.abs(tau * G))
    # a transposed L would give a different contraction: the pin is sensitive to it
    GT = impl.tau_gradient(o, v, n, L.transpose(1, 0, 2), w)
    assert abs(np.sum(tau * GT) - E) > 1e-3 * abs(E)


@pytest.mark.parametrize("seed", [44, 45])
def test_tau_gradient_integer_unit_differences(impl, seed):
    """With integer data every value is exact: E(tau + e_k) - E(tau) = G_k for every k."""
    o, v, n = 2, 3, 2
    rng = np.random.default_rng(seed)
    L = rng.integers(-3, 4, (v, v, n)).astype(float)
    tau = rng.integers(-3, 4, (o, o, v, v)).astype(float)
    w = rng.integers(-3, 4, (o, o, v, v)).astype(float)
    G = impl.tau_gradient(o, v, n, L, w)
    _, E0 = impl.forward(o, v, n, L, tau, w)
    for k in np.ndindex(o, o, v, v):
        t1 = tau.copy()
        t1[k] += 1.0
        _, E1 = impl.forward(o, v, n, L, t1, w)
        assert E1 - E0 == G[k], (k, E1 - E0, G[k])


def test_tau_gradient_symmetric_L_is_the_ladder(impl):
    """With L^J_ac = L^J_ca, (ac|bd) = (ca|db), so G(L, w) equals the forward ladder of w."""
    o, v, n = 2, 6, 3
    L0 = rnd(46, v, v, n)
    L = L0 + L0.transpose(1, 0, 2)
    w = rnd(47, o, o, v, v)
    G = impl.tau_gradient(o, v, n, L, w)
    R, _ = impl.forward(o, v, n, L, w)
    np.testing.assert_allclose(G, R, rtol=0, atol=1e-13 * np.abs(R).max())
    # and it does not hold for a non-symmetric L
    G0 = impl.tau_gradient(o, v, n, L0, w)
    R0, _ = impl.forward(o, v, n, L0, w)
    assert np.abs(G0 - R0).max() > 1e-3 * np.abs(R0).max()


def test_tau_gradient_pair_symmetry(impl):
    """(ac|bd) = (bd|ac) makes G pair-symmetric whenever w is."""
    o, v, n = 3, 4, 3
    L, w = rnd(48, v, v, n), pair_sym(rnd(49, o, o, v, v))
    G = impl.tau_gradient(o, v, n, L, w)
    np.testing.assert_allclose(G, G.transpose(1, 0, 3, 2), rtol=0, atol=1e-13 * np.abs(G).max())


# ---------------------------------------------------------------- gradient intermediates (W, V, MO back-transform)
@pytest.fixture(params=["c", "matrix"])
def gi(request, oracle_lib):
    """The C and numpy versions of W, V and the back-transformation behind one interface."""
    import oracle

    class C:
        w = staticmethod(oracle_lib.w_intermediate)
        v = staticmethod(oracle_lib.metric_contraction)
        bt = staticmethod(oracle_lib.back_transform)

    class M:
        w = staticmethod(oracle.matrix.w_intermediate)
        v = staticmethod(oracle.matrix.metric_contraction)
        bt = staticmethod(oracle.matrix.back_transform)

    return C if request.param == "c" else M


def test_w_intermediate_unit_density(gi):
    """A single amplitude pair: w = e_ij^ab, tau = e_ij^cd gives d_pqrs = [p=a][r=b][q=c][s=d],
    so W^K_pq = [p=a][q=c] Z^K_bd exactly."""
    o, v, n = 2, 5, 3
    Z = rnd(51, v, v, n)
    for (i, j, a, b, c, d) in [(0, 1, 2, 4, 1, 3), (1, 1, 0, 0, 4, 2), (1, 0, 3, 1, 1, 3)]:
        w = np.zeros((o, o, v, v)); w[i, j, a, b] = 1.0
        tau = np.zeros((o, o, v, v)); tau[i, j, c, d] = 1.0
        W = gi.w(o, v, n, Z, tau, w)
        ref = np.zeros((v, v, n)); ref[a, c] = Z[b, d]
        assert np.array_equal(W, ref), (i, j, a, b, c, d)


def test_w_intermediate_with_L_contracts_to_energy(gi, oracle_lib):
    """With Z = L: sum_K sum_pq L^K_pq W^K_pq = sum_pqrs (pq|rs) d_pqrs = E (Sec. II A energy),
    and under pair symmetry 2 W = X = dE/dL."""
    o, v, n = 3, 5, 4
    L, tau, w = rnd(52, v, v, n), pair_sym(rnd(53, o, o, v, v)), pair_sym(rnd(54, o, o, v, v))
    _, E = oracle_lib.forward(o, v, n, L, tau, w)
    W = gi.w(o, v, n, L, tau, w)
    assert abs(np.sum(L * W) - E) <= 1e-13 * np.sum(np.abs(L * W))
    X = oracle_lib.adjoint(o, v, n, L, tau, w)
    np.testing.assert_allclose(2.0 * W, X, rtol=0, atol=1e-13 * np.abs(X).max())
    # the energy identity holds for generic (non pair-symmetric) inputs too
    tau2, w2 = rnd(55, o, o, v, v), rnd(56, o, o, v, v)
    _, E2 = oracle_lib.forward(o, v, n, L, tau2, w2)
    W2 = gi.w(o, v, n, L, tau2, w2)
    assert abs(np.sum(L * W2) - E2) <= 1e-13 * np.sum(np.abs(L * W2))


def test_metric_contraction(gi, oracle_lib):
    """Rank-one closed form, V(Z, W)^T = V(W, Z), and with Z = L, W = W(L): trace V = E."""
    v, n = 4, 3
    u, t = rnd(57, v, v), rnd(58, v, v)
    Z = np.zeros((v, v, n)); Z[:, :, 2] = u
    W = np.zeros((v, v, n)); W[:, :, 0] = t
    V = gi.v(v, n, Z, W)
    ref = np.zeros((n, n)); ref[2, 0] = np.sum(u * t)
    np.testing.assert_allclose(V, ref, rtol=0, atol=1e-14)
    Z, W = rnd(59, v, v, n), rnd(60, v, v, n)
    np.testing.assert_allclose(gi.v(v, n, Z, W).T, gi.v(v, n, W, Z), rtol=0, atol=1e-14)
    o = 2
    L, tau, w = rnd(61, v, v, n), rnd(62, o, o, v, v), rnd(63, o, o, v, v)
    _, E = oracle_lib.forward(o, v, n, L, tau, w)
    Vl = gi.v(v, n, L, gi.w(o, v, n, L, tau, w))
    assert abs(np.trace(Vl) - E) <= 1e-13 * np.abs(Vl).sum()


def test_back_transform(gi):
    """Identity and permutation matrices act exactly; two transformations compose:
    BT(x2, y2, BT(x1, y1, W)) = BT(x1 x2, y1 y2, W); y = 1 leaves x^T W per K."""
    v, n = 5, 3
    W = rnd(64, v, v, n)
    I = np.eye(v)
    assert np.array_equal(gi.bt(v, n, I, I, W), W)
    p1, p2 = np.random.default_rng(65).permutation(v), np.random.default_rng(66).permutation(v)
    P1, P2 = I[p1].T, I[p2].T      # P[r][p] = [r = p1[p]]
    assert np.array_equal(gi.bt(v, n, P1, P2, W), W[p1][:, p2])
    x1, y1, x2, y2 = rnd(67, v, v), rnd(68, v, v), rnd(69, v, v), rnd(70, v, v)
    two = gi.bt(v, n, x2, y2, gi.bt(v, n, x1, y1, W))
    one = gi.bt(v, n, x1 @ x2, y1 @ y2, W)
    np.testing.assert_allclose(two, one, rtol=0, atol=1e-12 * np.abs(one).max())
    xo = gi.bt(v, n, x1, I, W)
    np.testing.assert_allclose(xo, np.einsum("rp,rqK->pqK", x1, W), rtol=0, atol=1e-13 * np.abs(xo).max())
    # x and y are not interchangeable
    assert np.abs(gi.bt(v, n, x1, y1, W) - gi.bt(v, n, y1, x1, W)).max() > 1e-3


# ---------------------------------------------------------------- excited-state amplitudes
def test_excited_amplitudes(oracle_lib):
    """Special cases of both readings: R0 = 0 or R2 = 0 isolate one term; in the Appendix
    reading (R~_aibj = R_aibj (1 + delta_{ai,bj}), Appendix A) a unit R2 off the diagonal is
    carried over unchanged and a unit R2 at i = j, a = b counts twice; pair-symmetric T and
    R2 give a pair-symmetric U."""
    o, v = 3, 4
    T, R2 = rnd(81, o, o, v, v), rnd(82, o, o, v, v)
    assert np.array_equal(oracle_lib.excited_amplitudes(o, v, 0.0, T, R2, 0), R2)
    assert np.array_equal(oracle_lib.excited_amplitudes(o, v, 0.75, T, np.zeros_like(R2), 0), 0.75 * T)
    assert np.array_equal(oracle_lib.excited_amplitudes(o, v, 0.75, T, np.zeros_like(R2), 1), 0.375 * T)
    for (i, j, a, b, f) in [(0, 2, 1, 3, 1.0), (1, 1, 2, 0, 1.0), (0, 2, 3, 3, 1.0), (2, 2, 1, 1, 2.0)]:
        E1 = np.zeros((o, o, v, v)); E1[i, j, a, b] = 1.0
        U = oracle_lib.excited_amplitudes(o, v, 0.3, np.zeros_like(T), E1, 1)
        ref = np.zeros_like(U); ref[i, j, a, b] = f
        assert np.array_equal(U, ref), (i, j, a, b)
    Ts, Rs = pair_sym(T), pair_sym(R2)
    for mode in (0, 1):
        U = oracle_lib.excited_amplitudes(o, v, 0.9, Ts, Rs, mode)
        np.testing.assert_allclose(U, U.transpose(1, 0, 3, 2), rtol=0, atol=1e-15)


# ---------------------------------------------------------------- excited-state OV^3 density d_abci
@pytest.fixture(params=["c", "matrix"])
def ov3(request, oracle_lib):
    """(Wab, Wci) of d_abci = sum_j L_ji^ac R_j^b from the C and the numpy oracle."""
    import oracle
    return oracle_lib.ov3_abci if request.param == "c" else oracle.matrix.ov3_abci


def test_ov3_abci_unit_density(ov3):
    """One multiplier element L_ji^ac = 1 and one singles element R_j'^b = 1: the density is
    [j = j'] at (a, b, c, i) only, so Wab^K_ab = Z^K_ci and Wci^K_ci = Z^K_ab exactly,
    and nothing else is touched; R_2 of another occupied index gives zero."""
    o, v, n = 3, 4, 5
    Zvv, Zvo = rnd(91, v, v, n), rnd(92, v, o, n)
    for (j, i, a, c, b) in [(0, 2, 1, 3, 0), (2, 2, 0, 0, 3), (1, 0, 3, 2, 3)]:
        L2 = np.zeros((o, o, v, v)); L2[j, i, a, c] = 1.0
        R1 = np.zeros((o, v)); R1[j, b] = 1.0
        Wab, Wci = ov3(o, v, n, L2, R1, Zvv, Zvo)
        ref_ab = np.zeros((v, v, n)); ref_ab[a, b] = Zvo[c, i]
        ref_ci = np.zeros((v, o, n)); ref_ci[c, i] = Zvv[a, b]
        assert np.array_equal(Wab, ref_ab) and np.array_equal(Wci, ref_ci), (j, i, a, c, b)
        R1 = np.zeros((o, v)); R1[(j + 1) % o, b] = 1.0
        Wab, Wci = ov3(o, v, n, L2, R1, Zvv, Zvo)
        assert not Wab.any() and not Wci.any()
    # ground state: d^gs_abci = 0 (no singles excitation)
    Wab, Wci = ov3(o, v, n, rnd(93, o, o, v, v), np.zeros((o, v)), Zvv, Zvo)
    assert not Wab.any() and not Wci.any()


def test_ov3_abci_table_chain(ov3):
    """The factored route of Sec. II B and its table of intermediates,
    X_aj^K = L_ji^ac Z_ci^K, Wab = R_j^b X_aj^K, P_aj^K = R_j^b Z_ab^K, Wci = L_ji^ac P_aj^K,
    gives what the oracle gets by forming the density and contracting it."""
    o, v, n = 4, 7, 6
    L2, R1, Zvv, Zvo = rnd(94, o, o, v, v), rnd(95, o, v), rnd(96, v, v, n), rnd(97, v, o, n)
    Wab, Wci = ov3(o, v, n, L2, R1, Zvv, Zvo)
    X = np.einsum("jiac,ciK->ajK", L2, Zvo)
    P = np.einsum("jb,abK->ajK", R1, Zvv)
    np.testing.assert_allclose(Wab, np.einsum("jb,ajK->abK", R1, X), rtol=0, atol=1e-13 * np.abs(Wab).max())
    np.testing.assert_allclose(Wci, np.einsum("jiac,ajK->ciK", L2, P), rtol=0, atol=1e-13 * np.abs(Wci).max())


def test_ov3_abci_energy_and_gradient(ov3, oracle_lib):
    """With Z = L (both blocks), sum L_ab W_ab and sum L_ci W_ci are the same number,
    E' = sum_abci d_abci (ab|ci) (Sec. II A energy over this block); E' is bilinear in the two
    Cholesky blocks, so central differences of E' computed from the ab side reproduce the ci
    side W_ci = dE'/dL_ci to rounding; and V_MN = Z_ab^M W_ab^N + Z_ci^M W_ci^N has trace 2 E'."""
    o, v, n = 3, 5, 4
    L2, R1, Lvv, Lvo = rnd(98, o, o, v, v), rnd(99, o, v), rnd(100, v, v, n), rnd(101, v, o, n)
    Wab, Wci = ov3(o, v, n, L2, R1, Lvv, Lvo)
    Eab, Eci = np.sum(Lvv * Wab), np.sum(Lvo * Wci)
    assert abs(Eab - Eci) <= 1e-13 * np.sum(np.abs(Lvv * Wab))

    def energy(Lvo_):
        W, _ = ov3(o, v, n, L2, R1, Lvv, Lvo_)
        return np.sum(Lvv * W)

    h = 0.5
    for (c, i, K) in [(0, 0, 0), (4, 2, 3), (2, 1, 1)]:
        e = np.zeros_like(Lvo); e[c, i, K] = h
        fd = (energy(Lvo + e) - energy(Lvo - e)) / (2 * h)
        assert abs(fd - Wci[c, i, K]) <= 1e-12 * np.abs(Wci).max(), (c, i, K)
    V = (oracle_lib.metric_contraction(v, n, Lvv, Wab)
         + oracle_lib.metric_contraction_pairs(v * o, n, Lvo.reshape(v * o, n), Wci.reshape(v * o, n)))
    assert abs(np.trace(V) - 2 * Eab) <= 1e-13 * np.abs(V).sum()


def test_ov3_abci_integer_exact(oracle_lib):
    """Small integer inputs: every product and sum is exact in FP64, so the C and the
    numpy oracle (different summation orders) agree bit for bit; both are bilinear."""
    import oracle
    o, v, n = 4, 9, 6
    g = np.random.default_rng(102)
    L2, R1 = g.integers(-3, 4, (o, o, v, v)).astype(float), g.integers(-3, 4, (o, v)).astype(float)
    Zvv, Zvo = g.integers(-3, 4, (v, v, n)).astype(float), g.integers(-3, 4, (v, o, n)).astype(float)
    a1, c1 = oracle_lib.ov3_abci(o, v, n, L2, R1, Zvv, Zvo)
    a2, c2 = oracle.matrix.ov3_abci(o, v, n, L2, R1, Zvv, Zvo)
    assert np.array_equal(a1, a2) and np.array_equal(c1, c2)
    a3, c3 = oracle_lib.ov3_abci(o, v, n, 2 * L2, -R1, Zvv, Zvo)
    assert np.array_equal(a3, -2 * a1) and np.array_equal(c3, -2 * c1)
    ab = np.array([[8, 0], [3, 3]]); ci = np.array([[0, 3], [8, 1]])
    assert np.array_equal(oracle_lib.ov3_abci_wab(o, v, n, L2, R1, Zvo, ab), a1[ab[:, 0], ab[:, 1]])
    assert np.array_equal(oracle_lib.ov3_abci_wci(o, v, n, L2, R1, Zvv, ci), c1[ci[:, 0], ci[:, 1]])


# ---------------------------------------------------------------- excited-state OV^3 density d_abic
@pytest.fixture(params=["c", "matrix"])
def abic(request, oracle_lib):
    """(Wab, Wic) of d_abic from the C and the numpy oracle."""
    import oracle
    return oracle_lib.ov3_abic if request.param == "c" else oracle.matrix.ov3_abic


def abic_inputs(seed, o, v, n):
    g = np.random.default_rng(seed)
    return dict(R0=0.625, L1=g.standard_normal((o, v)), L2=g.standard_normal((o, o, v, v)),
                T=g.standard_normal((o, o, v, v)), R1=g.standard_normal((o, v)), R2=g.standard_normal((o, o, v, v)),
                Zvv=g.standard_normal((v, v, n)), Zov=g.standard_normal((o, v, n)))


def _abic(f, o, v, n, x):
    return f(o, v, n, x["R0"], x["L1"], x["L2"], x["T"], x["R1"], x["R2"], x["Zvv"], x["Zov"])


def test_ov3_abic_ground_state_block(abic):
    """R^a_i = R_ij^ab = 0 leaves the ground-state block d_abic = L^a_m t~_im^cb R_0 (Appendix A):
    a unit L^a0_m0 with a unit t_i0m0^c0b0 gives d = 2 R_0 at (a0, b0, i0, c0) only, and a unit
    t_m0i0^c0b0 gives -R_0 there; the W's are then that number times one Z row."""
    o, v, n = 3, 4, 5
    x = abic_inputs(130, o, v, n)
    x["R1"], x["R2"], x["L2"] = np.zeros((o, v)), np.zeros((o, o, v, v)), np.zeros((o, o, v, v))
    m0, a0, i0, b0, c0 = 1, 2, 0, 3, 1
    x["L1"] = np.zeros((o, v)); x["L1"][m0, a0] = 1.0
    for (pos, dval) in [((i0, m0, c0, b0), 2.0), ((m0, i0, c0, b0), -1.0)]:
        x["T"] = np.zeros((o, o, v, v)); x["T"][pos] = 1.0
        Wab, Wic = _abic(abic, o, v, n, x)
        ref_ab = np.zeros((v, v, n)); ref_ab[a0, b0] = dval * x["R0"] * x["Zov"][i0, c0]
        ref_ic = np.zeros((o, v, n)); ref_ic[i0, c0] = dval * x["R0"] * x["Zvv"][a0, b0]
        assert np.array_equal(Wab, ref_ab) and np.array_equal(Wic, ref_ic), pos


def test_ov3_abic_doubles_term(abic):
    """R_0 = 0, t = 0, R^a_i = 0 leaves L^a_m (2 R~_mi^bc - R~_mi^cb): a unit R_m0i0^b0c0 (b0 != c0)
    gives 2 at (a0, b0, i0, c0) and -1 at (a0, c0, i0, b0); a unit diagonal R_m0m0^bb counts
    twice in R~ and gives 2*2 - 2 = 2 at (a0, b, m0, b)."""
    o, v, n = 3, 4, 2
    x = abic_inputs(131, o, v, n)
    x["R0"], x["T"], x["R1"] = 0.0, np.zeros((o, o, v, v)), np.zeros((o, v))
    m0, a0 = 2, 1
    x["L1"] = np.zeros((o, v)); x["L1"][m0, a0] = 1.0
    cases = [((m0, 0, 3, 1), [((a0, 3, 0, 1), 2.0), ((a0, 1, 0, 3), -1.0)]),
             ((m0, m0, 2, 2), [((a0, 2, m0, 2), 2.0)])]
    for pos, dens in cases:
        x["R2"] = np.zeros((o, o, v, v)); x["R2"][pos] = 1.0
        Wab, Wic = _abic(abic, o, v, n, x)
        ref_ab, ref_ic = np.zeros((v, v, n)), np.zeros((o, v, n))
        for (a, b, i, c), dv in dens:
            ref_ab[a, b] += dv * x["Zov"][i, c]
            ref_ic[i, c] += dv * x["Zvv"][a, b]
        assert np.array_equal(Wab, ref_ab) and np.array_equal(Wic, ref_ic), pos


def test_ov3_abic_table_route(abic):
    """The W_ab and W_ic expressions of Sec. II B, built here from its table of intermediates
    (X_ab, V, Y, W_am, B_iamn, and P^K, P_ik^K, P_ai^K, O^J_ai, Q^K, K_ik^K, U_bm^K, S_iacb), give
    what the oracle gets from the Appendix A density.  Readings: the printed 2 Q_ak^K R^b_k
    (and 2 Y_akci P_ak^K) is taken with Yt_akci, the intermediate of term (7) of d_abic; C^K
    is the table's Q^K = X_ab Z_ab^K; O_bm^K is L^a_m Z_ab^K; the R_2 in Yt_bm^K(U) is R~_2."""
    o, v, n = 3, 5, 4
    x = abic_inputs(132, o, v, n)
    Wab, Wic = _abic(abic, o, v, n, x)
    L1, L2, T, R1, R2, R0, Zvv, Zov = (x[k] for k in ("L1", "L2", "T", "R1", "R2", "R0", "Zvv", "Zov"))
    e = np.einsum
    tt = 2.0 * T - T.transpose(1, 0, 2, 3)
    Rt = R2 * (1.0 + e("ij,ab->ijab", np.eye(o), np.eye(v)))
    X = e("klad,klbd->ab", L2, T)
    VY = e("lkae,libe->akbi", L2, T) + e("klad,ilbd->akbi", L2, T)
    Yt = e("lkea,liec->akci", L2, tt)
    Wam = e("mkad,kd->am", L2, R1)
    B = e("mnad,id->iamn", L2, R1)
    S = e("iamn,mnbc->iacb", B, T)                       # S_iacb = B_iamn t_mn^bc = K_icab
    A = R0 * tt.transpose(1, 0, 2, 3) + 2.0 * Rt.transpose(0, 1, 3, 2) - Rt   # A[m,i,c,b] for L^a_m
    Ytb_U = e("micb,icK->bmK", A, Zov)                   # Yt_bm^K(U): sum_ic (...)_im^cb Z_ic^K
    Ytb_T = e("mibc,icK->bmK", tt, Zov)                  # sum_ic t~_mi^bc Z_ic^K
    PK = e("ic,icK->K", R1, Zov)
    Oai = e("ac,icK->aiK", X, Zov)
    Pik = e("kc,icK->ikK", R1, Zov)
    Qak = e("akci,icK->akK", Yt, Zov)
    ref_ab = (e("ma,bmK->abK", L1, Ytb_U) + 2.0 * e("ab,K->abK", X, PK) - e("aiK,ib->abK", Oai, R1)
              - e("akbi,ikK->abK", VY, Pik) + e("akK,kb->abK", Qak, R1) + e("am,bmK->abK", Wam, Ytb_T)
              - e("iacb,icK->abK", S, Zov))
    Obm = e("ma,abK->bmK", L1, Zvv)
    QK = e("ab,abK->K", X, Zvv)
    Pai = e("ib,abK->aiK", R1, Zvv)
    Kik = e("akbi,abK->ikK", VY, Zvv)
    Ubm = e("am,abK->bmK", Wam, Zvv)
    ref_ic = (e("micb,bmK->icK", A, Obm) + 2.0 * e("K,ic->icK", QK, R1) - e("ac,aiK->icK", X, Pai)
              - e("kc,ikK->icK", R1, Kik) + e("akci,akK->icK", Yt, e("kb,abK->akK", R1, Zvv))
              + e("mibc,bmK->icK", tt, Ubm) - e("iacb,abK->icK", S, Zvv))
    np.testing.assert_allclose(Wab, ref_ab, rtol=0, atol=1e-12 * np.abs(ref_ab).max())
    np.testing.assert_allclose(Wic, ref_ic, rtol=0, atol=1e-12 * np.abs(ref_ic).max())


def test_ov3_abic_identity_gradient_linearity(abic):
    """sum Zvv*Wab = sum Zov*Wic (both are sum_abic d_abic (ab|ic) with (ab|ic) = sum_K Zvv^K_ab
    Zov^K_ic); central differences of that number in Zov give Wic; d is linear in the right vector
    (R_0, R^a_i, R_ij^ab) and in the left one (L^a_m, L_ij^ab): the three parts of R add up, and
    doubling either vector doubles W exactly."""
    o, v, n = 3, 4, 3
    x = abic_inputs(133, o, v, n)
    Wab, Wic = _abic(abic, o, v, n, x)
    s_ab, s_ic = np.sum(x["Zvv"] * Wab), np.sum(x["Zov"] * Wic)
    assert abs(s_ab - s_ic) <= 1e-13 * np.sum(np.abs(x["Zvv"] * Wab))

    def energy(Zov):
        y = dict(x); y["Zov"] = Zov
        return np.sum(x["Zvv"] * _abic(abic, o, v, n, y)[0])

    for (i, c, K) in [(0, 0, 0), (2, 3, 2), (1, 2, 1)]:
        h = np.zeros_like(x["Zov"]); h[i, c, K] = 0.5
        fd = (energy(x["Zov"] + h) - energy(x["Zov"] - h)) / 1.0
        assert abs(fd - Wic[i, c, K]) <= 1e-12 * np.abs(Wic).max(), (i, c, K)
    parts = []
    for keep in ("R0", "R1", "R2"):
        y = dict(x)
        for k in ("R0", "R1", "R2"):
            if k != keep:
                y[k] = 0.0 if k == "R0" else np.zeros_like(x[k])
        parts.append(_abic(abic, o, v, n, y))
    np.testing.assert_allclose(sum(p[0] for p in parts), Wab, rtol=0, atol=1e-13 * np.abs(Wab).max())
    np.testing.assert_allclose(sum(p[1] for p in parts), Wic, rtol=0, atol=1e-13 * np.abs(Wic).max())
    y = dict(x); y["R0"], y["R1"], y["R2"] = 2 * x["R0"], 2 * x["R1"], 2 * x["R2"]
    a2, c2 = _abic(abic, o, v, n, y)
    assert np.array_equal(a2, 2 * Wab) and np.array_equal(c2, 2 * Wic)
    y = dict(x); y["L1"], y["L2"] = 2 * x["L1"], 2 * x["L2"]
    a2, c2 = _abic(abic, o, v, n, y)
    assert np.array_equal(a2, 2 * Wab) and np.array_equal(c2, 2 * Wic)


def test_ov3_abic_integer_exact(oracle_lib):
    """Small integer inputs: both oracles are exact and agree bit for bit."""
    import oracle
    o, v, n = 3, 6, 4
    g = np.random.default_rng(134)
    ints = lambda *s: g.integers(-2, 3, s).astype(float)
    args = (2.0, ints(o, v), ints(o, o, v, v), ints(o, o, v, v), ints(o, v), ints(o, o, v, v), ints(v, v, n), ints(o, v, n))
    a1, c1 = oracle_lib.ov3_abic(o, v, n, *args)
    a2, c2 = oracle.matrix.ov3_abic(o, v, n, *args)
    assert np.array_equal(a1, a2) and np.array_equal(c1, c2)


def test_metric_contraction_pairs(oracle_lib):
    """Over v^2 pairs it is the virtual-virtual contraction; a rank-one Z, W gives one entry."""
    v, n = 4, 3
    Z, W = rnd(103, v, v, n), rnd(104, v, v, n)
    assert np.array_equal(oracle_lib.metric_contraction_pairs(v * v, n, Z, W), oracle_lib.metric_contraction(v, n, Z, W))
    P = 7
    z, w = np.zeros((P, n)), np.zeros((P, n))
    z[:, 1], w[:, 2] = rnd(105, P), rnd(106, P)
    V = oracle_lib.metric_contraction_pairs(P, n, z, w)
    ref = np.zeros((n, n)); ref[1, 2] = np.dot(z[:, 1], w[:, 2])
    np.testing.assert_allclose(V, ref, rtol=0, atol=1e-15)


# ---------------------------------------------------------------- ranges and samples
def test_ranges_and_samples_agree_with_full(oracle_lib):
    o, v, n = 2, 7, 4
    L, tau, w = rnd(29, v, v, n), rnd(30, o, o, v, v), rnd(31, o, o, v, v)
    R, E = oracle_lib.forward(o, v, n, L, tau, w)
    X = oracle_lib.adjoint(o, v, n, L, tau, w)
    Rr, Ep, Er = oracle_lib.forward_range(o, v, n, L, tau, w, 2, 5)
    assert np.array_equal(Rr[:, :, 2:5], R[:, :, 2:5]) and not Rr[:, :, :2].any()
    Xr = oracle_lib.adjoint_range(o, v, n, L, tau, w, 3, 6)
    assert np.array_equal(Xr[3:6], X[3:6])
    ab = np.array([[0, 0], [6, 1], [3, 3], [2, 5]])
    Rs = oracle_lib.R_sample(o, v, n, L, tau, ab)
    for k, (a, b) in enumerate(ab):
        np.testing.assert_allclose(Rs[k], R[:, :, a, b].ravel(), rtol=0, atol=1e-14 * np.abs(R).max())
    Xs = oracle_lib.X_sample(o, v, n, L, tau, w, ab)
    for k, (p, q) in enumerate(ab):
        np.testing.assert_allclose(Xs[k], X[p, q], rtol=0, atol=1e-14 * np.abs(X).max())
    G = oracle_lib.tau_gradient(o, v, n, L, w)
    Gr = oracle_lib.tau_gradient_range(o, v, n, L, w, 1, 4)
    assert np.array_equal(Gr[:, :, 1:4], G[:, :, 1:4]) and not Gr[:, :, :1].any() and not Gr[:, :, 4:].any()
    import oracle
    Gm = oracle.matrix.tau_gradient(o, v, n, L, w, c_range=(1, 4))
    np.testing.assert_allclose(Gm, G[:, :, 1:4], rtol=0, atol=1e-13 * np.abs(G).max())


def test_bad_arguments_raise(oracle_lib):
    with pytest.raises(ValueError):
        oracle_lib.forward(2, 3, 4, np.zeros(5), np.zeros(36), None)
    with pytest.raises(RuntimeError):
        oracle_lib.R_sample(1, 2, 1, np.zeros(4), np.zeros(4), [[0, 2]])


# ---------------------------------------------------------------- amplitude recipe
def test_mp2_amplitudes_and_update(oracle_lib):
    o, v, n, seed = 2, 3, 4, 9
    Lov = synthetic.draw_L_ov(seed, o, v, n)
    eps = synthetic.draw_eps(seed, o, v)
    t = oracle_lib.mp2_amplitudes(o, v, n, Lov, eps)
    for i in range(o):
        for j in range(o):
            for a in range(v):
                for b in range(v):
                    iajb = float(np.dot(Lov[i, a], Lov[j, b]))
                    den = eps[i] + eps[j] - eps[o + a] - eps[o + b]
                    scale = float(np.dot(np.abs(Lov[i, a]), np.abs(Lov[j, b]))) / abs(den)
                    assert abs(t[i, j, a, b] - iajb / den) <= 1e-15 * scale
    assert np.array_equal(t, t.transpose(1, 0, 3, 2))  # bitwise pair symmetry
    R = rnd(32, o, o, v, v)
    t2 = oracle_lib.amplitude_update(o, v, eps, R, t)
    den = (eps[:o, None, None, None] + eps[None, :o, None, None]) - (eps[None, None, o:, None] + eps[None, None, None, o:])
    np.testing.assert_allclose((t2 - t) * den, R, rtol=1e-12, atol=0)


def test_mp2_amplitudes_minimal_basis_h2(oracle_lib):
    """A textbook case independent of the oracle's formula: H2 in the minimal STO-3G basis at
    R = 1.4 bohr (Szabo and Ostlund, Modern Quantum Chemistry, ch. 3 and 6), one occupied and
    one virtual orbital with eps_1 = -0.578, eps_2 = 0.670 and K_12 = (12|21) = 0.1813 Eh,
    whose second-order energy is E(2) = K_12^2 / (2 (eps_1 - eps_2)) = -0.0132 Eh.  With one
    Cholesky vector sqrt(K_12), the oracle's amplitude t_11^22 must give
    E(2) = sum t_ij^ab (2 (ia|jb) - (ib|ja)) = t K_12 at that value (to the table's rounding)."""
    eps1, eps2, K12 = -0.578, 0.670, 0.1813
    Lov = np.full((1, 1, 1), np.sqrt(K12))
    t = oracle_lib.mp2_amplitudes(1, 1, 1, Lov, np.array([eps1, eps2]))
    E2 = float(t[0, 0, 0, 0]) * (2.0 * K12 - K12)
    assert t[0, 0, 0, 0] < 0 and abs(E2 - (-0.0132)) <= 1e-4
