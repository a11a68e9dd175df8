// Host check of the +/- packing index arithmetic (pm_pack.hpp) against the dense
// definitions, run on the CPU (built by tests/test_pm_host.py with AddressSanitizer
// on host code, so any index outside a packed buffer aborts).  The tiled block
// bodies that the device kernels run are executed here with one thread and must
// reproduce the element functions bit for bit.
//   R_ij^ab = sum_cd (ac|bd) tau_ij^cd,  D_{ab,cd} = sum_ij tbar_ij^ab tau_ij^cd.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <vector>

#include "../paper_2202_02019_amd/csrc/pm_pack.hpp"

using namespace ladder;

static double rnd(unsigned long long& s) {
    s = s * 6364136223846793005ULL + 1442695040888963407ULL;
    return ((double)(s >> 11) * 0x1.0p-53) - 0.5;
}

// Runs a block body over every (row, tile pair) like the device grid does.
template <class Body>
static void run_tiled(int64_t v, int64_t rows, Body body) {
    PmTile A, B;
    for (int64_t r = 0; r < rows; ++r)
        for (int64_t t = 0; t < pm_tile_pairs(v); ++t) body(r, t, A, B);
}

static int same(const std::vector<double>& x, const std::vector<double>& y, int64_t count, const char* what) {
    for (int64_t k = 0; k < count; ++k)
        if (!(x[k] == y[k])) {
            printf("tiled %s differs at %lld: %.17g vs %.17g\n", what, (long long)k, x[k], y[k]);
            return 1;
        }
    return 0;
}

int check(int64_t o, int64_t v, int64_t n, int64_t nA, unsigned long long seed) {
    std::vector<double> L(v * v * n), tau(o * o * v * v), tb(o * o * v * v);
    for (auto& x : L) x = rnd(seed);
    for (auto* x : {&tau, &tb})
        for (int64_t i = 0; i < o; ++i)
            for (int64_t j = 0; j < o; ++j)
                for (int64_t a = 0; a < v; ++a)
                    for (int64_t b = 0; b < v; ++b) {
                        const int64_t k1 = ((i * o + j) * v + a) * v + b, k2 = ((j * o + i) * v + b) * v + a;
                        if (k2 < k1) (*x)[k1] = (*x)[k2];
                        else (*x)[k1] = rnd(seed);
                    }
    // dense reference R and D
    auto g = [&](int64_t a, int64_t c, int64_t b, int64_t d) {
        double s = 0;
        for (int64_t J = 0; J < n; ++J) s += L[(a * v + c) * n + J] * L[(b * v + d) * n + J];
        return s;
    };
    std::vector<double> Rref(o * o * v * v, 0.0);
    for (int64_t ij = 0; ij < o * o; ++ij)
        for (int64_t a = 0; a < v; ++a)
            for (int64_t b = 0; b < v; ++b) {
                double s = 0;
                for (int64_t c = 0; c < v; ++c)
                    for (int64_t d = 0; d < v; ++d) s += g(a, c, b, d) * tau[ij * v * v + c * v + d];
                Rref[ij * v * v + a * v + b] = s;
            }
    // packed inputs (exact-size buffers)
    std::vector<double> tp(pm_P2(o) * pm_P2(v)), tm(pm_Q2(o) * pm_Q2(v) + 1), wp(pm_P2(o) * v * v), wm(pm_Q2(o) * v * v + 1);
    for (int64_t t = 0; t < pm_amp_count(o, v); ++t) pm_pack_amp_elem(t, tau.data(), o, v, tp.data(), tm.data());
    for (int64_t t = 0; t < pm_w_count(o, v); ++t) pm_pack_w_elem(t, tb.data(), o, v, wp.data(), wm.data());
    int bad = 0;
    {
        std::vector<double> tp2(tp.size(), NAN), tm2(tm.size(), NAN);
        const PmRows rw{0, o, 0, 0};
        run_tiled(v, pm_P2(o), [&](int64_t r, int64_t t, PmTile& A, PmTile& B) {
            pm_pack_pair_block(tau.data(), v, rw, r, t, tp2.data(), tm2.data(), A, B, 0, 1, PmNoBarrier{});
        });
        bad |= same(tp2, tp, pm_P2(o) * pm_P2(v), "tau+") | same(tm2, tm, pm_Q2(o) * pm_Q2(v), "tau-");
    }
    std::vector<double> R(o * o * v * v, NAN);
    double worstR = 0, worstD = 0, E = 0, Eref = 0;
    for (int64_t a0 = 0; a0 < v; a0 += nA) {
        const int64_t nb = nA < v - a0 ? nA : v - a0;
        std::vector<double> gt(nb * (v - a0) * v * v);  // only b >= a0 is formed
        for (int64_t ap = 0; ap < nb; ++ap)
            for (int64_t b = a0; b < v; ++b)
                for (int64_t c = 0; c < v; ++c)
                    for (int64_t d = 0; d < v; ++d) gt[((ap * (v - a0) + (b - a0)) * v + c) * v + d] = g(a0 + ap, c, b, d);
        const int64_t NP = pm_gp_off(nb, v, a0), NM = pm_gm_off(nb, v, a0);
        std::vector<double> gp(NP * pm_P2(v)), gm(NM * pm_Q2(v) + 1);
        for (int64_t t = 0; t < pm_g_count(v, a0, nb); ++t) pm_pack_g_elem(t, gt.data(), v, a0, nb, gp.data(), gm.data());
        {
            std::vector<double> gp2(gp.size(), NAN), gm2(gm.size(), NAN);
            const PmRows rw{1, 0, a0, nb};
            run_tiled(v, NP, [&](int64_t r, int64_t t, PmTile& A, PmTile& B) {
                pm_pack_pair_block(gt.data(), v, rw, r, t, gp2.data(), pm_Q2(v) > 0 ? gm2.data() : nullptr, A, B, 0, 1,
                                   PmNoBarrier{});
            });
            bad |= same(gp2, gp, NP * pm_P2(v), "g+") | same(gm2, gm, NM * pm_Q2(v), "g-");
        }
        std::vector<double> rp(pm_P2(o) * NP), rm(pm_Q2(o) * NM + 1);
        for (int64_t p = 0; p < pm_P2(o); ++p)
            for (int64_t r = 0; r < NP; ++r) {
                double s = 0;
                for (int64_t k = 0; k < pm_P2(v); ++k) s += tp[p * pm_P2(v) + k] * gp[r * pm_P2(v) + k];
                rp[p * NP + r] = s;
            }
        for (int64_t q = 0; q < pm_Q2(o); ++q)
            for (int64_t r = 0; r < NM; ++r) {
                double s = 0;
                for (int64_t k = 0; k < pm_Q2(v); ++k) s += tm[q * pm_Q2(v) + k] * gm[r * pm_Q2(v) + k];
                rm[q * NM + r] = s;
            }
        for (int pass = 0; pass < 2; ++pass)
            for (int64_t t = 0; t < o * o * nb * v; ++t) {
                double e;
                if (pm_unpack_R_elem(t, rp.data(), rm.data(), o, v, a0, nb, 0.0, tb.data(), R.data(), pass, &e)) E += e;
            }
    }
    for (int64_t k = 0; k < o * o * v * v; ++k) {
        if (isnan(R[k])) { printf("R element %lld never written\n", (long long)k); return 1; }
        worstR = fmax(worstR, fabs(R[k] - Rref[k]));
        Eref += tb[k] * Rref[k];
    }
    // adjoint with packed density rows: Wp/Wm packed on (a<=b) by the mode-2 tiles, D+/D- per
    // batch of b, tiles (alpha) and (beta), and X assembled from both against the dense X
    double worstX = 0;
    {
        std::vector<double> wpp(pm_P2(o) * pm_P2(v), NAN), wmm(pm_Q2(o) * pm_Q2(v) + 1, NAN);
        const PmRows rw{2, o, 0, 0};
        run_tiled(v, pm_P2(o), [&](int64_t r, int64_t t, PmTile& A, PmTile& B) {
            pm_pack_pair_block(tb.data(), v, rw, r, t, wpp.data(), wmm.data(), A, B, 0, 1, PmNoBarrier{});
        });
        for (int64_t p = 0; p < pm_P2(o); ++p)  // Wp[P(i,j)][P(a,b)] = wp[P(i,j)][(a,b)]
            for (int64_t b = 0; b < v; ++b)
                for (int64_t a = 0; a <= b; ++a)
                    if (!(wpp[p * pm_P2(v) + pm_P(a, b)] == wp[p * v * v + a * v + b])) { printf("Wp differs\n"); bad = 1; }
        for (int64_t q = 0; q < pm_Q2(o); ++q)
            for (int64_t b = 0; b < v; ++b)
                for (int64_t a = 0; a < b; ++a)
                    if (!(wmm[q * pm_Q2(v) + pm_Q(a, b)] == wm[q * v * v + a * v + b])) { printf("Wm differs\n"); bad = 1; }
        std::vector<double> X(v * v * n, 0.0), Xref(v * v * n, 0.0);
        for (int64_t a = 0; a < v; ++a)
            for (int64_t c = 0; c < v; ++c)
                for (int64_t b = 0; b < v; ++b)
                    for (int64_t d = 0; d < v; ++d) {
                        double s = 0;
                        for (int64_t ij = 0; ij < o * o; ++ij) s += tb[ij * v * v + a * v + b] * tau[ij * v * v + c * v + d];
                        for (int64_t J = 0; J < n; ++J) Xref[(a * v + c) * n + J] += 2.0 * s * L[(b * v + d) * n + J];
                    }
        for (int64_t b0 = 0; b0 < v; b0 += nA) {
            const int64_t nB = nA < v - b0 ? nA : v - b0, A = b0 + nB;
            const int64_t rp = pm_P2(A) - pm_P2(b0), rm = pm_Q2(A) - pm_Q2(b0);
            std::vector<double> dp(rp * pm_P2(v)), dm(rm * pm_Q2(v) + 1);
            for (int64_t r = 0; r < rp; ++r)
                for (int64_t k = 0; k < pm_P2(v); ++k) {
                    double s = 0;
                    for (int64_t p = 0; p < pm_P2(o); ++p) s += wpp[p * pm_P2(v) + pm_P2(b0) + r] * tp[p * pm_P2(v) + k];
                    dp[r * pm_P2(v) + k] = s;
                }
            for (int64_t r = 0; r < rm; ++r)
                for (int64_t k = 0; k < pm_Q2(v); ++k) {
                    double s = 0;
                    for (int64_t q = 0; q < pm_Q2(o); ++q) s += wmm[q * pm_Q2(v) + pm_Q2(b0) + r] * tm[q * pm_Q2(v) + k];
                    dm[r * pm_Q2(v) + k] = s;
                }
            for (int64_t b = b0; b < A; ++b)  // the packed rows against the dense density
                for (int64_t a = 0; a <= b; ++a)
                    for (int64_t c = 0; c < v; ++c)
                        for (int64_t d = 0; d < v; ++d) {
                            double sd = 0;
                            for (int64_t ij = 0; ij < o * o; ++ij) sd += tb[ij * v * v + a * v + b] * tau[ij * v * v + c * v + d];
                            worstD = fmax(worstD, fabs(pm_density(dp.data(), dm.data(), v, b0, a, b, c, d) - sd));
                        }
            for (int pass = 0; pass < 2; ++pass) {  // 0: alpha, 1: beta
                const bool alpha = pass == 0;
                const int64_t rows = alpha ? nB * v : A * v, K = alpha ? A * v : nB * v;
                std::vector<double> T(rows * K, NAN), T2(rows * K, NAN);
                for (int64_t t = 0; t < rows * K; ++t) {
                    if (alpha) pm_tile_alpha_elem(t, dp.data(), dm.data(), v, b0, nB, T.data());
                    else pm_tile_beta_elem(t, dp.data(), dm.data(), v, b0, nB, T.data());
                }
                run_tiled(v, nB * A, [&](int64_t r, int64_t t, PmTile& Pa, PmTile& Pb) {
                    pm_tile_ab_block(dp.data(), dm.data(), v, b0, nB, r, t, alpha, T2.data(), Pa, Pb, 0, 1, PmNoBarrier{});
                });
                bad |= same(T2, T, rows * K, alpha ? "tile alpha" : "tile beta");
                // the element source of the split tile slicer, (row, k) -> value, equals the tile
                std::vector<double> T3(rows * K, NAN);
                for (int64_t r = 0; r < rows; ++r)
                    for (int64_t k = 0; k < K; ++k) T3[r * K + k] = pm_tile_value(dp.data(), dm.data(), v, b0, nB, alpha, r, k);
                bad |= same(T3, T, rows * K, alpha ? "tile alpha source" : "tile beta source");
                // X rows: alpha (b, y) += T[(b-b0, y)][(a, w)] L[(a, w)];  beta (a, y) += T[(a, y)][(b-b0, w)] L[(b, w)]
                const int64_t row0 = alpha ? b0 * v : 0, k0 = alpha ? 0 : b0 * v;
                for (int64_t r = 0; r < rows; ++r)
                    for (int64_t k = 0; k < K; ++k) {
                        const double tv = T[r * K + k];
                        if (tv == 0.0) continue;
                        for (int64_t J = 0; J < n; ++J) X[(row0 + r) * n + J] += 2.0 * tv * L[(k0 + k) * n + J];
                    }
            }
        }
        for (int64_t k = 0; k < v * v * n; ++k) worstX = fmax(worstX, fabs(X[k] - Xref[k]));
    }
    printf("o=%lld v=%lld n=%lld nA=%lld  max|dR| %.3e  max|dD| %.3e  |dE| %.3e  max|dX| %.3e\n", (long long)o, (long long)v,
           (long long)n, (long long)nA, worstR, worstD, fabs(E - Eref), worstX);
    return (!bad && worstR < 1e-12 && worstD < 1e-12 && fabs(E - Eref) < 1e-11 && worstX < 1e-11) ? 0 : 1;
}

int main() {
    int bad = 0;
    bad |= check(1, 1, 1, 1, 1);
    bad |= check(2, 3, 2, 1, 2);
    bad |= check(3, 5, 3, 2, 3);
    bad |= check(4, 7, 2, 3, 4);
    bad |= check(2, 9, 4, 9, 5);
    bad |= check(5, 6, 3, 4, 6);
    bad |= check(2, 37, 2, 11, 7);   // two tile blocks, ragged
    bad |= check(3, 70, 1, 33, 8);   // three tile blocks, ragged batches
    printf(bad ? "FAIL\n" : "OK\n");
    return bad;
}
