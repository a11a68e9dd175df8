/*
 * ladder_oracle.c -- plain, slow FP64 CPU oracle for the V^4 O^2 particle-particle
 * ladder of Cholesky-decomposed CCSD and its adjoint.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code, header, table or helper with the HIP
 * path.
 *
 * What it computes (Schnack-Petersen, Koch, Coriani, Kjonstad, arXiv 2202.02019):
 *
 *   g_acbd  = sum_J L^J_ac L^J_bd                 Sec. II A: Cholesky expansion
 *                                                 of the ERIs, (pq|rs) = sum_J L^J_pq L^J_rs
 *   R_ij^ab = sum_cd g_acbd tau_ij^cd             the A2 (particle-particle ladder)
 *                                                 term of Omega cited in Sec. II B
 *   E       = sum_ijab tbar_ij^ab R_ij^ab         the V^4 part of sum_pqrs g_pqrs d_pqrs
 *                                                 (Sec. II A energy expression) with the
 *                                                 ground-state density d_abcd = O^(2)_abcd
 *                                                 (Appendix A, R_0 = 1, L_2 = tbar)
 *   X^J_pq  = dE/dL^J_pq
 *           = sum_bd L^J_bd sum_ij ( w_ij^pb tau_ij^qd + w_ij^bp tau_ij^dq )
 *                                                 the L-built three-index intermediate
 *                                                 (2 W~^J_pq of Sec. II C) restricted to
 *                                                 the V^4 density block of Sec. II B.
 *   W^K_pq  = sum_rs d_pqrs Z^K_rs,  d_pqrs = sum_ij w_ij^pr tau_ij^qs
 *                                                 the three-index density intermediate of
 *                                                 Sec. II A (V^4 block, density of Sec. II B)
 *   V_MN    = sum_pq Z^M_pq W^N_pq                its two-index partner (Sec. II A)
 *   Wmo^K_pq = sum_rs x_rp y_sq W^K_rs            the MO back-transformation (Sec. II A)
 *   G_ij^cd = dE/dtau_ij^cd = sum_ab w_ij^ab g_acbd
 *                                                 the transposed ladder: the A2-term part
 *                                                 of the multiplier equations tbar A = -eta
 *                                                 (Sec. II A), E being linear in tau.
 *   Wab^K_ab = sum_ci d_abci Z^K_ci,  Wci^K_ci = sum_ab d_abci Z^K_ab,
 *   d_abci   = sum_j L_ji^ac R_j^b              the excited-state OV^3 density block
 *                                                 (Appendix A) and its contributions to W
 *                                                 (Sec. II B)
 *
 * The adjoint is written in its general form: it does NOT assume the pair
 * symmetry tau_ij^ab = tau_ji^ba (Appendix A, d_pqrs = d_rspq), so a GPU path that
 * relies on that symmetry is caught by a parity test fed asymmetric input.
 *
 * Layouts (row-major, FP64):
 *   L    [v][v][n]   L[(a*v+c)*n+J]        = L^J_ac   (virtual-virtual block)
 *   tau  [o][o][v][v] tau[((i*o+j)*v+c)*v+d] = tau_ij^cd  (also tbar, w, R)
 *   X    [v][v][n]   like L
 *   Lov  [o][v][n]   Lov[(i*v+a)*n+J]      = L^J_ia   (occupied-virtual block)
 *   Zvo  [v][o][n]   Zvo[(c*o+i)*n+K]      = Z^K_ci   (virtual-occupied block, also Wci)
 *   R1   [o][v]      R1[j*v+b]             = R_j^b    (excited-state singles)
 *   eps  [o+v]       occupied orbital energies first, then virtual
 *
 * Every function returns 0 on success and -1 on a bad argument.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_num_threads(int t) {
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/* Neumaier's compensated summation: running sum s with correction c. */
static void neumaier_add(double* s, double* c, double x) {
    double t = *s + x;
    if (fabs(*s) >= fabs(x))
        *c += (*s - t) + x;
    else
        *c += (x - t) + *s;
    *s = t;
}

static int bad_dims(int64_t o, int64_t v, int64_t n) {
    return o < 1 || v < 1 || n < 1 || o > 100000 || v > 100000 || n > 1000000;
}

/*
 * Forward ladder for the virtual range a in [a_lo, a_hi):
 *   R[i][j][a][b] = sum_c sum_d g_a[c][b][d] tau[i][j][c][d],
 *   g_a[c][b][d]  = sum_J L[a][c][J] L[b][d][J].
 * Rows a outside the range are left untouched.  If tbar and E_part are given,
 * E_part[a - a_lo] = sum_ijb tbar_ij^ab R_ij^ab (compensated) and *E (if given)
 * receives the compensated sum of E_part in increasing a.
 */
int oracle_ladder_forward_range(int64_t o, int64_t v, int64_t n, const double* L,
                                const double* tau, const double* tbar, int64_t a_lo,
                                int64_t a_hi, double* R, double* E_part, double* E) {
    if (bad_dims(o, v, n) || !L || !tau || !R || a_lo < 0 || a_hi > v || a_lo > a_hi)
        return -1;
    const int64_t oo = o * o, vv = v * v;
    double* Ea = (double*)calloc((size_t)(a_hi - a_lo) + 1, sizeof(double));
    if (!Ea) return -1;
    int fail = 0;
#pragma omp parallel
    {
        double* g = (double*)malloc((size_t)(v * vv) * sizeof(double));
        if (!g) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t a = a_lo; a < a_hi; ++a) {
            if (!g) continue;
            /* g_a[c][b][d] = (ac|bd) */
            for (int64_t c = 0; c < v; ++c) {
                const double* Lac = L + (a * v + c) * n;
                for (int64_t b = 0; b < v; ++b)
                    for (int64_t d = 0; d < v; ++d) {
                        const double* Lbd = L + (b * v + d) * n;
                        double s = 0.0;
                        for (int64_t J = 0; J < n; ++J) s += Lac[J] * Lbd[J];
                        g[(c * v + b) * v + d] = s;
                    }
            }
            /* R_ij^ab = sum_cd (ac|bd) tau_ij^cd */
            double es = 0.0, ec = 0.0;
            for (int64_t ij = 0; ij < oo; ++ij) {
                const double* t = tau + ij * vv;
                for (int64_t b = 0; b < v; ++b) {
                    double s = 0.0;
                    for (int64_t c = 0; c < v; ++c) {
                        const double* gc = g + (c * v + b) * v;
                        const double* tc = t + c * v;
                        for (int64_t d = 0; d < v; ++d) s += gc[d] * tc[d];
                    }
                    R[ij * vv + a * v + b] = s;
                    if (tbar) neumaier_add(&es, &ec, tbar[ij * vv + a * v + b] * s);
                }
            }
            Ea[a - a_lo] = es + ec;
        }
        free(g);
    }
    if (!fail && tbar) {
        double s = 0.0, c = 0.0;
        for (int64_t a = a_lo; a < a_hi; ++a) {
            if (E_part) E_part[a - a_lo] = Ea[a - a_lo];
            neumaier_add(&s, &c, Ea[a - a_lo]);
        }
        if (E) *E = s + c;
    }
    free(Ea);
    return fail ? -1 : 0;
}

int oracle_ladder_forward(int64_t o, int64_t v, int64_t n, const double* L, const double* tau,
                          const double* tbar, double* R, double* E) {
    return oracle_ladder_forward_range(o, v, n, L, tau, tbar, 0, v, R, NULL, E);
}

/*
 * Transposed ladder for the range c in [c_lo, c_hi), general L (no symmetry of
 * L^J in its two indices assumed):
 *   h_c[a][b][d]  = sum_J L[a][c][J] L[b][d][J]           (= g_acbd)
 *   G[i][j][c][d] = sum_a sum_b w[i][j][a][b] h_c[a][b][d].
 * Rows c outside the range are left untouched.
 */
int oracle_ladder_tau_gradient_range(int64_t o, int64_t v, int64_t n, const double* L,
                                     const double* w, int64_t c_lo, int64_t c_hi, double* G) {
    if (bad_dims(o, v, n) || !L || !w || !G || c_lo < 0 || c_hi > v || c_lo > c_hi) return -1;
    const int64_t oo = o * o, vv = v * v;
    int fail = 0;
#pragma omp parallel
    {
        double* h = (double*)malloc((size_t)(v * vv) * sizeof(double));
        if (!h) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t c = c_lo; c < c_hi; ++c) {
            if (!h) continue;
            for (int64_t a = 0; a < v; ++a) {
                const double* Lac = L + (a * v + c) * n;
                for (int64_t b = 0; b < v; ++b)
                    for (int64_t d = 0; d < v; ++d) {
                        const double* Lbd = L + (b * v + d) * n;
                        double s = 0.0;
                        for (int64_t J = 0; J < n; ++J) s += Lac[J] * Lbd[J];
                        h[(a * v + b) * v + d] = s;
                    }
            }
            for (int64_t ij = 0; ij < oo; ++ij) {
                const double* wij = w + ij * vv;
                for (int64_t d = 0; d < v; ++d) {
                    double s = 0.0;
                    for (int64_t a = 0; a < v; ++a)
                        for (int64_t b = 0; b < v; ++b) s += wij[a * v + b] * h[(a * v + b) * v + d];
                    G[ij * vv + c * v + d] = s;
                }
            }
        }
        free(h);
    }
    return fail ? -1 : 0;
}

int oracle_ladder_tau_gradient(int64_t o, int64_t v, int64_t n, const double* L, const double* w,
                               double* G) {
    return oracle_ladder_tau_gradient_range(o, v, n, L, w, 0, v, G);
}

/*
 * Three-index density intermediate for rows p in [p_lo, p_hi):
 *   d_pqrs = sum_ij w[i][j][p][r] tau[i][j][q][s]     (V^4 density, Mulliken order)
 *   W[p][q][K] = sum_r sum_s d_pqrs Z[r][s][K].
 * Z has the layout of L.  Rows p outside the range are left untouched.
 */
int oracle_w_intermediate_range(int64_t o, int64_t v, int64_t n, const double* Z, const double* tau,
                                const double* w, int64_t p_lo, int64_t p_hi, double* W) {
    if (bad_dims(o, v, n) || !Z || !tau || !w || !W || p_lo < 0 || p_hi > v || p_lo > p_hi) return -1;
    const int64_t oo = o * o, vv = v * v;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t p = p_lo; p < p_hi; ++p) {
        for (int64_t q = 0; q < v; ++q) {
            double* out = W + (p * v + q) * n;
            for (int64_t K = 0; K < n; ++K) out[K] = 0.0;
            for (int64_t r = 0; r < v; ++r)
                for (int64_t s = 0; s < v; ++s) {
                    double d = 0.0;
                    for (int64_t ij = 0; ij < oo; ++ij) d += w[ij * vv + p * v + r] * tau[ij * vv + q * v + s];
                    const double* z = Z + (r * v + s) * n;
                    for (int64_t K = 0; K < n; ++K) out[K] += d * z[K];
                }
        }
    }
    return 0;
}

/* V[M][N] = sum_p sum_q Z[p][q][M] W[p][q][N]. */
int oracle_metric_contraction(int64_t v, int64_t n, const double* Z, const double* W, double* V) {
    if (bad_dims(1, v, n) || !Z || !W || !V) return -1;
    const int64_t vv = v * v;
#pragma omp parallel for schedule(static)
    for (int64_t M = 0; M < n; ++M)
        for (int64_t N = 0; N < n; ++N) {
            double s = 0.0;
            for (int64_t pq = 0; pq < vv; ++pq) s += Z[pq * n + M] * W[pq * n + N];
            V[M * n + N] = s;
        }
    return 0;
}

/* Wmo[p][q][K] = sum_r sum_s x[r][p] y[s][q] W[r][s][K], for K in [K_lo, K_hi). */
int oracle_back_transform_range(int64_t v, int64_t n, const double* x, const double* y, const double* W,
                                int64_t K_lo, int64_t K_hi, double* Wmo) {
    if (bad_dims(1, v, n) || !x || !y || !W || !Wmo || K_lo < 0 || K_hi > n || K_lo > K_hi) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t p = 0; p < v; ++p)
        for (int64_t q = 0; q < v; ++q)
            for (int64_t K = K_lo; K < K_hi; ++K) {
                double s = 0.0;
                for (int64_t r = 0; r < v; ++r)
                    for (int64_t t = 0; t < v; ++t) s += x[r * v + p] * y[t * v + q] * W[(r * v + t) * n + K];
                Wmo[(p * v + q) * n + K] = s;
            }
    return 0;
}

/*
 * Excited-state amplitudes entering the excited-state V^4 density
 * d^es_abcd = O^(2)_abcd(L_2, U) (Appendix A); the paper gives two definitions:
 *   mode 0 (table of intermediates): U_ij^ab = R0 T_ij^ab + R_ij^ab
 *   mode 1 (Appendix A):             U_ij^ab = (R0/2) T_ij^ab + Rt_ij^ab,
 *                                    Rt_ij^ab = R_ij^ab (1 + [i = j][a = b])
 * where Rt is the Appendix's R~_2: the doubles written over all (ai, bj) with the
 * coefficient R_aibj (1 + delta_{ai,bj}), i.e. the diagonal doubles counted twice.
 */
int oracle_excited_amplitudes(int64_t o, int64_t v, double R0, const double* T, const double* R2, int mode,
                              double* U) {
    if (bad_dims(o, v, 1) || !T || !R2 || !U || (mode != 0 && mode != 1)) return -1;
    for (int64_t i = 0; i < o; ++i)
        for (int64_t j = 0; j < o; ++j)
            for (int64_t a = 0; a < v; ++a)
                for (int64_t b = 0; b < v; ++b) {
                    const int64_t x = ((i * o + j) * v + a) * v + b;
                    if (mode == 0)
                        U[x] = R0 * T[x] + R2[x];
                    else
                        U[x] = 0.5 * R0 * T[x] + (i == j && a == b ? 2.0 * R2[x] : R2[x]);
                }
    return 0;
}

/*
 * Adjoint for the range p in [p_lo, p_hi), general (no pair symmetry assumed):
 *   D1[b][q][d] = sum_ij w_ij^pb tau_ij^qd
 *   D2[b][d][q] = sum_ij w_ij^bp tau_ij^dq
 *   X[p][q][J]  = sum_b sum_d (D1[b][q][d] + D2[b][d][q]) L[b][d][J].
 */
int oracle_ladder_adjoint_range(int64_t o, int64_t v, int64_t n, const double* L,
                                const double* tau, const double* w, int64_t p_lo,
                                int64_t p_hi, double* X) {
    if (bad_dims(o, v, n) || !L || !tau || !w || !X || p_lo < 0 || p_hi > v || p_lo > p_hi)
        return -1;
    const int64_t oo = o * o, vv = v * v;
    int fail = 0;
#pragma omp parallel
    {
        double* D1 = (double*)malloc((size_t)(v * vv) * sizeof(double));
        double* D2 = (double*)malloc((size_t)(v * vv) * sizeof(double));
        if (!D1 || !D2) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t p = p_lo; p < p_hi; ++p) {
            if (!D1 || !D2) continue;
            memset(D1, 0, (size_t)(v * vv) * sizeof(double));
            memset(D2, 0, (size_t)(v * vv) * sizeof(double));
            for (int64_t ij = 0; ij < oo; ++ij) {
                const double* t = tau + ij * vv;
                const double* wi = w + ij * vv;
                for (int64_t b = 0; b < v; ++b) {
                    const double w1 = wi[p * v + b]; /* w_ij^pb */
                    const double w2 = wi[b * v + p]; /* w_ij^bp */
                    double* d1 = D1 + b * vv;
                    double* d2 = D2 + b * vv;
                    for (int64_t k = 0; k < vv; ++k) {
                        d1[k] += w1 * t[k]; /* k = q*v+d : tau_ij^qd */
                        d2[k] += w2 * t[k]; /* k = d*v+q : tau_ij^dq */
                    }
                }
            }
            for (int64_t q = 0; q < v; ++q) {
                double* x = X + (p * v + q) * n;
                for (int64_t J = 0; J < n; ++J) x[J] = 0.0;
                for (int64_t b = 0; b < v; ++b)
                    for (int64_t d = 0; d < v; ++d) {
                        const double coef = D1[(b * v + q) * v + d] + D2[(b * v + d) * v + q];
                        const double* Lbd = L + (b * v + d) * n;
                        for (int64_t J = 0; J < n; ++J) x[J] += coef * Lbd[J];
                    }
            }
        }
        free(D1);
        free(D2);
    }
    return fail ? -1 : 0;
}

int oracle_ladder_adjoint(int64_t o, int64_t v, int64_t n, const double* L, const double* tau,
                          const double* w, double* X) {
    return oracle_ladder_adjoint_range(o, v, n, L, tau, w, 0, v, X);
}

/*
 * Sampled forward: for each requested pair (a,b), out[k*o*o + ij] = R_ij^ab.
 * g_ab[c][d] = sum_J L^J_ac L^J_bd is formed for that pair only.
 */
int oracle_ladder_R_sample(int64_t o, int64_t v, int64_t n, const double* L, const double* tau,
                           int64_t npairs, const int64_t* ab, double* out) {
    if (bad_dims(o, v, n) || !L || !tau || !ab || !out || npairs < 0) return -1;
    for (int64_t k = 0; k < npairs; ++k)
        if (ab[2 * k] < 0 || ab[2 * k] >= v || ab[2 * k + 1] < 0 || ab[2 * k + 1] >= v) return -1;
    const int64_t oo = o * o, vv = v * v;
    int fail = 0;
#pragma omp parallel
    {
        double* g = (double*)malloc((size_t)vv * sizeof(double));
        if (!g) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t k = 0; k < npairs; ++k) {
            if (!g) continue;
            const int64_t a = ab[2 * k], b = ab[2 * k + 1];
            for (int64_t c = 0; c < v; ++c)
                for (int64_t d = 0; d < v; ++d) {
                    const double* Lac = L + (a * v + c) * n;
                    const double* Lbd = L + (b * v + d) * n;
                    double s = 0.0;
                    for (int64_t J = 0; J < n; ++J) s += Lac[J] * Lbd[J];
                    g[c * v + d] = s;
                }
            for (int64_t ij = 0; ij < oo; ++ij) {
                const double* t = tau + ij * vv;
                double s = 0.0;
                for (int64_t cd = 0; cd < vv; ++cd) s += g[cd] * t[cd];
                out[k * oo + ij] = s;
            }
        }
        free(g);
    }
    return fail ? -1 : 0;
}

/*
 * Sampled adjoint: for each requested pair (p,q), out[k*n + J] = X^J_pq in the
 * general form of oracle_ladder_adjoint_range.
 */
int oracle_ladder_X_sample(int64_t o, int64_t v, int64_t n, const double* L, const double* tau,
                           const double* w, int64_t npairs, const int64_t* pq, double* out) {
    if (bad_dims(o, v, n) || !L || !tau || !w || !pq || !out || npairs < 0) return -1;
    for (int64_t k = 0; k < npairs; ++k)
        if (pq[2 * k] < 0 || pq[2 * k] >= v || pq[2 * k + 1] < 0 || pq[2 * k + 1] >= v) return -1;
    const int64_t oo = o * o, vv = v * v;
    int fail = 0;
#pragma omp parallel
    {
        double* D = (double*)malloc((size_t)vv * sizeof(double));
        if (!D) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t k = 0; k < npairs; ++k) {
            if (!D) continue;
            const int64_t p = pq[2 * k], q = pq[2 * k + 1];
            /* D[b][d] = sum_ij (w_ij^pb tau_ij^qd + w_ij^bp tau_ij^dq) */
            for (int64_t bd = 0; bd < vv; ++bd) D[bd] = 0.0;
            for (int64_t ij = 0; ij < oo; ++ij) {
                const double* t = tau + ij * vv;
                const double* wi = w + ij * vv;
                for (int64_t b = 0; b < v; ++b) {
                    const double w1 = wi[p * v + b], w2 = wi[b * v + p];
                    for (int64_t d = 0; d < v; ++d)
                        D[b * v + d] += w1 * t[q * v + d] + w2 * t[d * v + q];
                }
            }
            double* x = out + k * n;
            for (int64_t J = 0; J < n; ++J) x[J] = 0.0;
            for (int64_t bd = 0; bd < vv; ++bd) {
                const double* Lbd = L + bd * n;
                for (int64_t J = 0; J < n; ++J) x[J] += D[bd] * Lbd[J];
            }
        }
        free(D);
    }
    return fail ? -1 : 0;
}

/*
 * First-order (MP2-like) doubles amplitudes, the synthetic stand-in for CCSD T2:
 *   t_ij^ab = (ia|jb) / (eps_i + eps_j - eps_a - eps_b),  (ia|jb) = sum_J L^J_ia L^J_jb
 * with the Cholesky expansion of Sec. II A.  The denominator is formed as
 * (eps_i + eps_j) - (eps_a + eps_b) so that t_ij^ab = t_ji^ba holds bitwise.
 */
int oracle_mp2_amplitudes(int64_t o, int64_t v, int64_t n, const double* Lov, const double* eps,
                          double* t) {
    if (bad_dims(o, v, n) || !Lov || !eps || !t) return -1;
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t i = 0; i < o; ++i)
        for (int64_t j = 0; j < o; ++j)
            for (int64_t a = 0; a < v; ++a)
                for (int64_t b = 0; b < v; ++b) {
                    const double* Lia = Lov + (i * v + a) * n;
                    const double* Ljb = Lov + (j * v + b) * n;
                    double s = 0.0;
                    for (int64_t J = 0; J < n; ++J) s += Lia[J] * Ljb[J];
                    const double den = (eps[i] + eps[j]) - (eps[o + a] + eps[o + b]);
                    t[((i * o + j) * v + a) * v + b] = s / den;
                }
    return 0;
}

/*
 * One Jacobi (diagonal-denominator) amplitude update, the standard quasi-Newton
 * step for the amplitude equations Omega = 0 (Sec. II A):
 *   t_ij^ab <- t_ij^ab + R_ij^ab / (eps_i + eps_j - eps_a - eps_b)
 * with the same denominator association as oracle_mp2_amplitudes.
 */
int oracle_amplitude_update(int64_t o, int64_t v, const double* eps, const double* R, double* t) {
    if (o < 1 || v < 1 || !eps || !R || !t) return -1;
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t i = 0; i < o; ++i)
        for (int64_t j = 0; j < o; ++j)
            for (int64_t a = 0; a < v; ++a)
                for (int64_t b = 0; b < v; ++b) {
                    const int64_t k = ((i * o + j) * v + a) * v + b;
                    const double den = (eps[i] + eps[j]) - (eps[o + a] + eps[o + b]);
                    t[k] = t[k] + R[k] / den;
                }
    return 0;
}

/*
 * Excited-state OV^3 density block (Appendix A, excited-state densities):
 *   d_abci = sum_j L_ji^ac R_j^b
 * and its two contributions to the three-index intermediate
 * W^K_pq = sum_rs d_pqrs Z^K_rs (Sec. II A), over the integrals (ab|ci) of this
 * block (Sec. II B, contributions of the OV^3 densities):
 *   Wab^K_ab = sum_ci d_abci Z^K_ci           (the ab side)
 *   Wci^K_ci = sum_ab d_abci Z^K_ab           (the ci side)
 * Each density element is formed on its own (o products) and then contracted;
 * the factored route of Sec. II B through X_aj^K and P_aj^K is deliberately not
 * taken, so that it can be checked against this one.
 * Layouts: L2 [o][o][v][v] with L2[((j*o+i)*v+a)*v+c] = L_ji^ac; R1 [o][v] with
 * R1[j*v+b] = R_j^b; Zvv and Wab [v][v][n]; Zvo and Wci [v][o][n] with
 * Zvo[(c*o+i)*n+K] = Z^K_ci.  The functions fill out[k][n] for the k index pairs
 * given (ab[2t], ab[2t+1]) = (a, b), or (ci[2t], ci[2t+1]) = (c, i).
 */
static double dens_abci(int64_t o, int64_t v, const double* L2, const double* R1, int64_t a, int64_t b,
                        int64_t c, int64_t i) {
    double d = 0.0;
    for (int64_t j = 0; j < o; ++j) d += L2[((j * o + i) * v + a) * v + c] * R1[j * v + b];
    return d;
}

int oracle_ov3_abci_wab(int64_t o, int64_t v, int64_t n, const double* L2, const double* R1, const double* Zvo,
                        int64_t k, const int64_t* ab, double* out) {
    if (bad_dims(o, v, n) || !L2 || !R1 || !Zvo || !out || k < 0 || (k > 0 && !ab)) return -1;
    for (int64_t t = 0; t < k; ++t)
        if (ab[2 * t] < 0 || ab[2 * t] >= v || ab[2 * t + 1] < 0 || ab[2 * t + 1] >= v) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < k; ++t) {
        const int64_t a = ab[2 * t], b = ab[2 * t + 1];
        double* w = out + t * n;
        for (int64_t K = 0; K < n; ++K) w[K] = 0.0;
        for (int64_t c = 0; c < v; ++c)
            for (int64_t i = 0; i < o; ++i) {
                const double d = dens_abci(o, v, L2, R1, a, b, c, i);
                const double* z = Zvo + (c * o + i) * n;
                for (int64_t K = 0; K < n; ++K) w[K] += d * z[K];
            }
    }
    return 0;
}

int oracle_ov3_abci_wci(int64_t o, int64_t v, int64_t n, const double* L2, const double* R1, const double* Zvv,
                        int64_t k, const int64_t* ci, double* out) {
    if (bad_dims(o, v, n) || !L2 || !R1 || !Zvv || !out || k < 0 || (k > 0 && !ci)) return -1;
    for (int64_t t = 0; t < k; ++t)
        if (ci[2 * t] < 0 || ci[2 * t] >= v || ci[2 * t + 1] < 0 || ci[2 * t + 1] >= o) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < k; ++t) {
        const int64_t c = ci[2 * t], i = ci[2 * t + 1];
        double* w = out + t * n;
        for (int64_t K = 0; K < n; ++K) w[K] = 0.0;
        for (int64_t a = 0; a < v; ++a)
            for (int64_t b = 0; b < v; ++b) {
                const double d = dens_abci(o, v, L2, R1, a, b, c, i);
                const double* z = Zvv + (a * v + b) * n;
                for (int64_t K = 0; K < n; ++K) w[K] += d * z[K];
            }
    }
    return 0;
}

/* V[M][N] = sum_p Z[p][M] W[p][N] over any number of index pairs p (for the
 * occupied-virtual block of V_MN = Z^M_ab W^N_ab + Z^M_ci W^N_ci, Sec. II B). */
int oracle_metric_contraction_pairs(int64_t pairs, int64_t n, const double* Z, const double* W, double* V) {
    if (pairs < 1 || n < 1 || !Z || !W || !V) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t M = 0; M < n; ++M)
        for (int64_t N = 0; N < n; ++N) {
            double s = 0.0;
            for (int64_t p = 0; p < pairs; ++p) s += Z[p * n + M] * W[p * n + N];
            V[M * n + N] = s;
        }
    return 0;
}

/*
 * Excited-state OV^3 density block d_abic (Appendix A, excited-state densities)
 * and its two contributions to the three-index intermediate (Sec. II B):
 *   Wab^K_ab = sum_ic d_abic Z^K_ic,   Wic^K_ic = sum_ab d_abic Z^K_ab.
 * With L^a_m the singles and L_ij^ab the doubles multipliers, t the ground-state
 * doubles, R_0, R^a_i, R_ij^ab the excited-state right vector, and the tilde
 * conventions  t~_ij^ab = 2 t_ij^ab - t_ji^ab,  R~_ij^ab = R_ij^ab (1 + [i=j][a=b]):
 *   d_abic = R_0 L^a_m t~_im^cb                               (1)
 *          + L^a_m (2 R~_mi^bc - R~_mi^cb)                     (2)
 *          + 2 X_ab R^c_i                                      (3)
 *          - (V_akbi + Y_akbi) R^c_k                           (4)
 *          + L_mk^ad t~_mi^bc R^d_k                            (5)
 *          - L_mn^ad t_mn^bc R^d_i                             (6)
 *          + Yt_akci R^b_k                                     (7)
 *          - X_ac R^b_i                                        (8)
 * with the intermediates of Sec. II B and Appendix A (all with C_2 = t):
 *   X_ab    = L_kl^ad t_kl^bd
 *   V_akbi  = L_lk^ae t_li^be          (V_ajbi = L_kj^ac C_ki^bc)
 *   Y_akbi  = L_kl^ad t_il^bd          (Y_ajbi = L_jl^ad C_il^bd)
 *   Yt_akci = L_mk^ea t~_mi^ec         (Yt_djak = L_mj^ed t~_mk^ea)
 *   W_am    = L_mk^ad R^d_k            (W_ai = L_il^ad R_dl; term (5) is W_am t~_mi^bc)
 *   B_iamn  = L_mn^ad R^d_i            (term (6) is -B_iamn t_mn^bc)
 * Each intermediate is formed from its definition, then every density element
 * d_abic is assembled from the eight terms and contracted.  Layouts: L1, R1
 * [o][v] (L1[m*v+a] = L^a_m); L2, T, R2 [o][o][v][v] (L2[((i*o+j)*v+a)*v+b] =
 * L_ij^ab); Zvv, Wab [v][v][n]; Zov, Wic [o][v][n] (Zov[(i*v+c)*n+K] = Z^K_ic).
 */
typedef struct {
    int64_t o, v;
    double R0;
    const double *L1, *L2, *T, *R1, *R2;
    double *X, *V, *Y, *Yt, *W, *B;
} abic_ctx;

static double a2(const abic_ctx* q, const double* A, int64_t i, int64_t j, int64_t a, int64_t b) {
    return A[((i * q->o + j) * q->v + a) * q->v + b];
}
static double t_tilde(const abic_ctx* q, int64_t i, int64_t j, int64_t a, int64_t b) {
    return 2.0 * a2(q, q->T, i, j, a, b) - a2(q, q->T, j, i, a, b);
}
static double r_tilde(const abic_ctx* q, int64_t i, int64_t j, int64_t a, int64_t b) {
    const double r = a2(q, q->R2, i, j, a, b);
    return (i == j && a == b) ? 2.0 * r : r;
}

static double abic_density(const abic_ctx* q, int64_t a, int64_t b, int64_t i, int64_t c) {
    const int64_t o = q->o, v = q->v;
    double d = 0.0;
    for (int64_t m = 0; m < o; ++m) {
        const double La = q->L1[m * v + a];
        d += q->R0 * La * t_tilde(q, i, m, c, b);                                       /* (1) */
        d += La * (2.0 * r_tilde(q, m, i, b, c) - r_tilde(q, m, i, c, b));              /* (2) */
        d += q->W[a * o + m] * t_tilde(q, m, i, b, c);                                   /* (5) */
    }
    d += 2.0 * q->X[a * v + b] * q->R1[i * v + c];                                      /* (3) */
    for (int64_t k = 0; k < o; ++k) {
        const int64_t akbi = ((a * o + k) * v + b) * o + i;
        d -= (q->V[akbi] + q->Y[akbi]) * q->R1[k * v + c];                               /* (4) */
        d += q->Yt[((a * o + k) * v + c) * o + i] * q->R1[k * v + b];                    /* (7) */
    }
    for (int64_t m = 0; m < o; ++m)
        for (int64_t nn = 0; nn < o; ++nn)
            d -= q->B[((i * v + a) * o + m) * o + nn] * a2(q, q->T, m, nn, b, c);       /* (6) */
    d -= q->X[a * v + c] * q->R1[i * v + b];                                            /* (8) */
    return d;
}

int oracle_ov3_abic(int64_t o, int64_t v, int64_t n, double R0, const double* L1, const double* L2, const double* T,
                    const double* R1, const double* R2, const double* Zvv, const double* Zov, double* Wab,
                    double* Wic) {
    if (bad_dims(o, v, n) || !L1 || !L2 || !T || !R1 || !R2 || !Zvv || !Zov || !Wab || !Wic) return -1;
    abic_ctx q = {o, v, R0, L1, L2, T, R1, R2, NULL, NULL, NULL, NULL, NULL, NULL};
    const int64_t ovov = o * v * o * v;
    q.X = (double*)calloc((size_t)(v * v), sizeof(double));
    q.V = (double*)calloc((size_t)ovov, sizeof(double));
    q.Y = (double*)calloc((size_t)ovov, sizeof(double));
    q.Yt = (double*)calloc((size_t)ovov, sizeof(double));
    q.W = (double*)calloc((size_t)(v * o), sizeof(double));
    q.B = (double*)calloc((size_t)(o * v * o * o), sizeof(double));
    int rc = 0;
    if (!q.X || !q.V || !q.Y || !q.Yt || !q.W || !q.B) {
        rc = -1;
        goto done;
    }
#pragma omp parallel for schedule(static)
    for (int64_t a = 0; a < v; ++a) {
        for (int64_t b = 0; b < v; ++b) {  /* X_ab = L_kl^ad t_kl^bd */
            double s = 0.0;
            for (int64_t k = 0; k < o; ++k)
                for (int64_t l = 0; l < o; ++l)
                    for (int64_t d = 0; d < v; ++d) s += a2(&q, L2, k, l, a, d) * a2(&q, T, k, l, b, d);
            q.X[a * v + b] = s;
        }
        for (int64_t m = 0; m < o; ++m) {  /* W_am = L_mk^ad R^d_k */
            double s = 0.0;
            for (int64_t k = 0; k < o; ++k)
                for (int64_t d = 0; d < v; ++d) s += a2(&q, L2, m, k, a, d) * R1[k * v + d];
            q.W[a * o + m] = s;
        }
        for (int64_t k = 0; k < o; ++k)
            for (int64_t b = 0; b < v; ++b)
                for (int64_t i = 0; i < o; ++i) {
                    double sv = 0.0, sy = 0.0, st = 0.0;
                    for (int64_t l = 0; l < o; ++l)
                        for (int64_t e = 0; e < v; ++e) {
                            sv += a2(&q, L2, l, k, a, e) * a2(&q, T, l, i, b, e);   /* V_akbi */
                            sy += a2(&q, L2, k, l, a, e) * a2(&q, T, i, l, b, e);   /* Y_akbi */
                            st += a2(&q, L2, l, k, e, a) * t_tilde(&q, l, i, e, b); /* Yt_akbi (b as c) */
                        }
                    const int64_t x = ((a * o + k) * v + b) * o + i;
                    q.V[x] = sv;
                    q.Y[x] = sy;
                    q.Yt[x] = st;
                }
    }
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t i = 0; i < o; ++i)
        for (int64_t a = 0; a < v; ++a)
            for (int64_t m = 0; m < o; ++m)
                for (int64_t nn = 0; nn < o; ++nn) {  /* B_iamn = L_mn^ad R^d_i */
                    double s = 0.0;
                    for (int64_t d = 0; d < v; ++d) s += a2(&q, L2, m, nn, a, d) * R1[i * v + d];
                    q.B[((i * v + a) * o + m) * o + nn] = s;
                }
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t a = 0; a < v; ++a)
        for (int64_t b = 0; b < v; ++b) {
            double* w = Wab + (a * v + b) * n;
            for (int64_t K = 0; K < n; ++K) w[K] = 0.0;
            for (int64_t i = 0; i < o; ++i)
                for (int64_t c = 0; c < v; ++c) {
                    const double d = abic_density(&q, a, b, i, c);
                    const double* z = Zov + (i * v + c) * n;
                    for (int64_t K = 0; K < n; ++K) w[K] += d * z[K];
                }
        }
#pragma omp parallel for collapse(2) schedule(dynamic, 1)
    for (int64_t i = 0; i < o; ++i)
        for (int64_t c = 0; c < v; ++c) {
            double* w = Wic + (i * v + c) * n;
            for (int64_t K = 0; K < n; ++K) w[K] = 0.0;
            for (int64_t a = 0; a < v; ++a)
                for (int64_t b = 0; b < v; ++b) {
                    const double d = abic_density(&q, a, b, i, c);
                    const double* z = Zvv + (a * v + b) * n;
                    for (int64_t K = 0; K < n; ++K) w[K] += d * z[K];
                }
        }
done:
    free(q.X);
    free(q.V);
    free(q.Y);
    free(q.Yt);
    free(q.W);
    free(q.B);
    return rc;
}
