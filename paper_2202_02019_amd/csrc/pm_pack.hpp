// pm_pack.hpp -- symmetric / antisymmetric (+/-) packing of the ladder
// (the strategy of Scuseria, Lee and Schaefer for the A2 term, which Sec. II B
// adapts to the V^4 density).
//
// With pair-symmetric amplitudes (x_ij^ab = x_ji^ba) write
//   x+_ij^cd = (x_ij^cd + x_ij^dc)/2   symmetric in i<->j and in c<->d,
//   x-_ij^cd = (x_ij^cd - x_ij^dc)/2   antisymmetric in both,
// and g+-_{ab,cd} = (ac|bd) +- (ad|bc), symmetric / antisymmetric in a<->b and c<->d.
// Then
//   R_ij^ab = sum_{c<=d} g+_{ab,cd} w_cd tau+_ij^cd + sum_{c<d} g-_{ab,cd} tau-_ij^cd,  w_cc = 1/2, else 1,
// so each of the two products needs only i<=j (resp. i<j), a<=b (a<b) and c<=d
// (c<d): 1/8 of the dense O^2 V^4 work each, 1/4 together.  For the density
//   D_{ab,cd} = sum_ij tbar_ij^ab tau_ij^cd
//             = sum_{i<=j} (2 - delta_ij) tbar+_ij^ab tau+_ij^cd + sum_{i<j} 2 tbar-_ij^ab tau-_ij^cd
// (the mixed terms cancel in the sum over i, j), which halves both the
// contraction and the (c,d) range: 1/2 of the dense work.
//
// Pair indices: P(i,j) = j(j+1)/2 + i for i <= j, Q(i,j) = j(j-1)/2 + i for i < j.
// The element functions below define every packed value; they are host-callable
// so that the index arithmetic can be checked on the CPU against the dense
// definition.  The R unpack kernel is a grid-stride loop over its element
// function; the pack and D-unpack kernels are LDS-tiled (end of file) and the
// host check compares them with the element functions bit for bit.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace ladder {

__host__ __device__ inline int64_t pm_P(int64_t i, int64_t j) { return j * (j + 1) / 2 + i; }  // i <= j
__host__ __device__ inline int64_t pm_Q(int64_t i, int64_t j) { return j * (j - 1) / 2 + i; }  // i < j
__host__ __device__ inline int64_t pm_P2(int64_t x) { return x * (x + 1) / 2; }
__host__ __device__ inline int64_t pm_Q2(int64_t x) { return x * (x - 1) / 2; }

// Inverse of P: p -> (i, j) with i <= j.
__host__ __device__ inline void pm_unP(int64_t p, int64_t& i, int64_t& j) {
    int64_t jj = (int64_t)((sqrt(8.0 * (double)p + 1.0) - 1.0) * 0.5);
    while (jj > 0 && jj * (jj + 1) / 2 > p) --jj;
    while ((jj + 1) * (jj + 2) / 2 <= p) ++jj;
    j = jj;
    i = p - jj * (jj + 1) / 2;
}
// Inverse of Q: q -> (i, j) with i < j.
__host__ __device__ inline void pm_unQ(int64_t q, int64_t& i, int64_t& j) {
    int64_t jj = (int64_t)((sqrt(8.0 * (double)q + 1.0) + 1.0) * 0.5);
    while (jj > 1 && jj * (jj - 1) / 2 > q) --jj;
    while ((jj + 1) * jj / 2 <= q) ++jj;
    j = jj;
    i = q - jj * (jj - 1) / 2;
}

// Rows of the packed g tile of a batch A = [a0, a0+nA): (a', b) with b >= a0+a'
// (plus part) or b > a0+a' (minus part), a' major.
__host__ __device__ inline int64_t pm_gp_off(int64_t ap, int64_t v, int64_t a0) { return ap * (v - a0) - ap * (ap - 1) / 2; }
__host__ __device__ inline int64_t pm_gm_off(int64_t ap, int64_t v, int64_t a0) { return ap * (v - a0 - 1) - ap * (ap - 1) / 2; }

// Packed element counts.
__host__ __device__ inline int64_t pm_amp_count(int64_t o, int64_t v) { return pm_P2(o) * pm_P2(v) + pm_Q2(o) * pm_Q2(v); }
__host__ __device__ inline int64_t pm_w_count(int64_t o, int64_t v) { return (pm_P2(o) + pm_Q2(o)) * v * v; }
__host__ __device__ inline int64_t pm_g_count(int64_t v, int64_t a0, int64_t nA) {
    return pm_gp_off(nA, v, a0) * pm_P2(v) + pm_gm_off(nA, v, a0) * pm_Q2(v);
}

// x[o][o][v][v] -> xp[P(i,j)][P(c,d)] = (x_ij^cd + x_ij^dc)/2, xm[Q(i,j)][Q(c,d)] = (x_ij^cd - x_ij^dc)/2.
__host__ __device__ inline void pm_pack_amp_elem(int64_t t, const double* x, int64_t o, int64_t v, double* xp, double* xm) {
    const int64_t np = pm_P2(o) * pm_P2(v), vv = v * v;
    int64_t i, j, c, d;
    if (t < np) {
        const int64_t cols = pm_P2(v);
        pm_unP(t / cols, i, j);
        pm_unP(t % cols, c, d);
        const double* r = x + (i * o + j) * vv;
        xp[t] = 0.5 * (r[c * v + d] + r[d * v + c]);
    } else {
        const int64_t u = t - np, cols = pm_Q2(v);
        pm_unQ(u / cols, i, j);
        pm_unQ(u % cols, c, d);
        const double* r = x + (i * o + j) * vv;
        xm[u] = 0.5 * (r[c * v + d] - r[d * v + c]);
    }
}

// tbar -> wp[P(i,j)][(a,b)] = (2 - delta_ij) (t_ij^ab + t_ij^ba)/2, wm[Q(i,j)][(a,b)] = t_ij^ab - t_ij^ba
// over all (a, b): the reference the packed-row weights Wp, Wm are checked against.
__host__ __device__ inline void pm_pack_w_elem(int64_t t, const double* x, int64_t o, int64_t v, double* wp, double* wm) {
    const int64_t vv = v * v, np = pm_P2(o) * vv;
    const bool plus = t < np;
    const int64_t u = plus ? t : t - np;
    const int64_t ab = u % vv, a = ab / v, b = ab % v;
    int64_t i, j;
    if (plus) pm_unP(u / vv, i, j); else pm_unQ(u / vv, i, j);
    const double* r = x + (i * o + j) * vv;
    if (plus) wp[u] = (i == j ? 0.5 : 1.0) * (r[a * v + b] + r[b * v + a]);
    else wm[u] = r[a * v + b] - r[b * v + a];
}

// g tile g[(a', b-a0)][(c,d)] of batch [a0, a0+nA) (only b >= a0 is formed) ->
// gp[rowp(a',b)][P(c,d)], gm[rowm(a',b)][Q(c,d)]:
//   gp = (ac|bd) + (ad|bc) for c < d, (ac|bc) for c = d (the w_cc = 1/2 folded in),
//   gm = (ac|bd) - (ad|bc).
__host__ __device__ inline void pm_pack_g_elem(int64_t t, const double* g, int64_t v, int64_t a0, int64_t nA, double* gp,
                                               double* gm) {
    const int64_t cp = pm_P2(v), cm = pm_Q2(v), vv = v * v;
    const int64_t np = pm_gp_off(nA, v, a0) * cp;
    const bool plus = t < np;
    const int64_t u = plus ? t : t - np;
    const int64_t cols = plus ? cp : cm;
    const int64_t row = u / cols, col = u % cols;
    // row -> (a', b): off(a') = a'K - a'(a'-1)/2 <= row < off(a'+1), K = v - a0 (- 1 for minus)
    const double K2 = 2.0 * (double)(plus ? v - a0 : v - a0 - 1) + 1.0;
    int64_t ap = (int64_t)(0.5 * (K2 - sqrt(fmax(K2 * K2 - 8.0 * (double)row, 0.0))));
    if (ap < 0) ap = 0;
    if (ap > nA - 1) ap = nA - 1;
    while (ap > 0 && (plus ? pm_gp_off(ap, v, a0) : pm_gm_off(ap, v, a0)) > row) --ap;
    while (ap + 1 < nA && (plus ? pm_gp_off(ap + 1, v, a0) : pm_gm_off(ap + 1, v, a0)) <= row) ++ap;
    const int64_t b = a0 + ap + (row - (plus ? pm_gp_off(ap, v, a0) : pm_gm_off(ap, v, a0))) + (plus ? 0 : 1);
    int64_t c, d;
    if (plus) pm_unP(col, c, d); else pm_unQ(col, c, d);
    const double* r = g + (ap * (v - a0) + (b - a0)) * vv;
    if (plus) gp[u] = c < d ? r[c * v + d] + r[d * v + c] : r[c * v + c];
    else gm[u] = r[c * v + d] - r[d * v + c];
}

// One R element of batch [a0, a0+nA) from rp[P(i,j)][rowp] and rm[Q(i,j)][rowm]:
//   R_ij^ab = rp + s_ij rm (pass 0, b >= a),  R_ij^ba = rp - s_ij rm (pass 1, b > a),
// s_ij = +1 (i<j), -1 (i>j), 0 (i=j).  Slot t enumerates (i, j, a', b) (pass 0,
// contiguous in b) or (i, j, b, a') (pass 1, contiguous in a); returns false for
// unused slots.  Writes R = beta R + value and returns tbar * value in *e.
__host__ __device__ inline bool pm_unpack_R_elem(int64_t t, const double* rp, const double* rm, int64_t o, int64_t v,
                                                 int64_t a0, int64_t nA, double beta, const double* tbar, double* R,
                                                 int pass, double* e) {
    const int64_t vv = v * v, NP = pm_gp_off(nA, v, a0), NM = pm_gm_off(nA, v, a0);
    const int64_t per_ij = nA * v;
    const int64_t ij = t / per_ij, s = t % per_ij;
    const int64_t i = ij / o, j = ij % o;
    int64_t ap, b;
    if (pass == 0) {
        ap = s / v;
        b = s % v;
    } else {
        b = s / nA;
        ap = s % nA;
    }
    const int64_t a = a0 + ap;
    if (pass == 0 ? b < a : b <= a) return false;
    const int64_t lo = i < j ? i : j, hi = i < j ? j : i;
    const double sij = i < j ? 1.0 : (i > j ? -1.0 : 0.0);
    const double p = rp[pm_P(lo, hi) * NP + pm_gp_off(ap, v, a0) + (b - a)];
    const double m = (b > a && i != j) ? rm[pm_Q(lo, hi) * NM + pm_gm_off(ap, v, a0) + (b - a - 1)] : 0.0;
    const double val = pass == 0 ? p + sij * m : p - sij * m;
    const int64_t idx = ij * vv + (pass == 0 ? a * v + b : b * v + a);
    R[idx] = beta == 0.0 ? val : val + beta * R[idx];
    *e = tbar ? tbar[idx] * val : 0.0;
    return true;
}

// ---- adjoint with packed density rows (a <= b) ----
// The density is symmetric under the pair exchange, D_{ab,cd} = D_{ba,dc}, so the
// adjoint forms only the rows a <= b: D+ = Wp^T Tp on rows P(a,b) and D- = Wm^T Tm
// on rows Q(a,b), for the b of a batch [b0, b0+nB), with
//   Wp[P(i,j)][P(a,b)] = (2 - delta_ij)(t_ij^ab + t_ij^ba)/2,  Wm[Q(i,j)][Q(a,b)] = t_ij^ab - t_ij^ba,
// and X^J_xy = sum_zw D_{xz,yw} L^J_zw is assembled from the two uses of each row:
//   (alpha) X_{b y} += sum_{a<b, w} D_{ab,wy} L_{a w}       rows (b, y), K = (a, w), a < b0 + nB
//   (beta)  X_{a y} += sum_{b, w}   D_{ab,yw} L_{b w}       rows (a, y), K = (b, w), a <= b
// (the z > x terms of X_x come from (beta) with (a, b) = (x, z), the z < x terms from
// (alpha) with (a, b) = (z, x)).

// D_{ab,cd} for a <= b, b in [b0, b0+nB), from the batch's packed rows.
__host__ __device__ inline double pm_density(const double* dp, const double* dm, int64_t v, int64_t b0, int64_t a, int64_t b,
                                             int64_t c, int64_t d) {
    const int64_t lo = c < d ? c : d, hi = c < d ? d : c;
    double x = dp[(pm_P(a, b) - pm_P2(b0)) * pm_P2(v) + pm_P(lo, hi)];
    if (a < b && c != d) x += (c < d ? 1.0 : -1.0) * dm[(pm_Q(a, b) - pm_Q2(b0)) * pm_Q2(v) + pm_Q(lo, hi)];
    return x;
}
// Tile (alpha), [(b - b0) v + y][a v + w] with a < b0 + nB: D_{ab,wy} for a < b, else 0.
__host__ __device__ inline void pm_tile_alpha_elem(int64_t t, const double* dp, const double* dm, int64_t v, int64_t b0,
                                                   int64_t nB, double* T) {
    const int64_t K = (b0 + nB) * v;
    const int64_t row = t / K, col = t % K;
    const int64_t b = b0 + row / v, y = row % v, a = col / v, w = col % v;
    T[t] = a < b ? pm_density(dp, dm, v, b0, a, b, w, y) : 0.0;
}
// Tile (beta), [a v + y][(b - b0) v + w] with a < b0 + nB: D_{ab,yw} for a <= b, else 0.
__host__ __device__ inline void pm_tile_beta_elem(int64_t t, const double* dp, const double* dm, int64_t v, int64_t b0,
                                                  int64_t nB, double* T) {
    const int64_t K = nB * v;
    const int64_t row = t / K, col = t % K;
    const int64_t a = row / v, y = row % v, b = b0 + col / v, w = col % v;
    T[t] = a <= b ? pm_density(dp, dm, v, b0, a, b, y, w) : 0.0;
}

// Element (r, k) of tile (alpha) or (beta) of batch [b0, b0+nB), as pm_tile_alpha_elem /
// pm_tile_beta_elem define it (rows r, contraction index k), read from the packed rows.
__host__ __device__ inline double pm_tile_value(const double* dp, const double* dm, int64_t v, int64_t b0, int64_t nB,
                                                bool alpha, int64_t r, int64_t k) {
    if (alpha) {  // r = (b - b0) v + y, k = a v + w: D_{ab, w y} for a < b
        const int64_t b = b0 + r / v, y = r % v, a = k / v, w = k % v;
        return a < b ? pm_density(dp, dm, v, b0, a, b, w, y) : 0.0;
    }
    // r = a v + y, k = (b - b0) v + w: D_{ab, y w} for a <= b
    const int64_t a = r / v, y = r % v, b = b0 + k / v, w = k % v;
    (void)nB;
    return a <= b ? pm_density(dp, dm, v, b0, a, b, y, w) : 0.0;
}

// Source functor of the split slicer for the density tiles: the slices of a tile are
// written straight from the packed rows, without the FP64 tile in between.
struct PmTileRows {
    const double* dp;
    const double* dm;
    int64_t v, b0, nB;
    int alpha;
    __device__ double operator()(int64_t r, int64_t k) const { return pm_tile_value(dp, dm, v, b0, nB, alpha != 0, r, k); }
};

#define PM_GRID_STRIDE(total) \
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < (total); t += (int64_t)gridDim.x * blockDim.x)

// Needs all threads of the block (it has a barrier); one energy partial per block.
__global__ void pm_unpack_R_kernel(const double* __restrict__ rp, const double* __restrict__ rm, int64_t o, int64_t v,
                                   int64_t a0, int64_t nA, double beta, const double* __restrict__ tbar,
                                   double* __restrict__ R, double* __restrict__ partial, int pass) {
    double e = 0.0;
    PM_GRID_STRIDE(o * o * nA * v) {
        double x;
        if (pm_unpack_R_elem(t, rp, rm, o, v, a0, nA, beta, tbar, R, pass, &x)) e += x;
    }
    if (!tbar) return;
    __shared__ double red[16];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += red[k];
        partial[blockIdx.x] = s;
    }
}

}  // namespace ladder

namespace ladder {

// ---------------------------------------------------------------------------
// Tiled forms of the packing kernels.  A v x v matrix is processed in 32 x 32
// tile pairs (Cb, Db), Cb <= Db: a workgroup stages M[Cb][Db] and M[Db][Cb]
// through LDS with row-contiguous reads and writes the packed (or unpacked)
// values contiguously, so every fetched line is used whole by one workgroup (the
// element-wise kernels above gather with a stride of about v).  Each tile body is
// split at its barrier into host-callable parts taking (tid, nthreads), so the
// host check can run the same code with one thread; the values equal those of
// the element functions above.
constexpr int PM_T = 32;
typedef double PmTile[PM_T][PM_T + 1];

__host__ __device__ inline int64_t pm_tile_pairs(int64_t v) {
    const int64_t nb = (v + PM_T - 1) / PM_T;
    return nb * (nb + 1) / 2;
}

// A[r][q] = M[c0+r][d0+q], B[r][q] = M[d0+r][c0+q] (zero outside v x v).
__host__ __device__ inline void pm_stage_pair(const double* M, int64_t v, int64_t c0, int64_t d0, PmTile& A, PmTile& B,
                                              int tid, int nth) {
    for (int e = tid; e < PM_T * PM_T; e += nth) {
        const int r = e / PM_T, q = e % PM_T;
        A[r][q] = (c0 + r < v && d0 + q < v) ? M[(c0 + r) * v + d0 + q] : 0.0;
        B[r][q] = (d0 + r < v && c0 + q < v) ? M[(d0 + r) * v + c0 + q] : 0.0;
    }
}

// Source matrix of packed row r.  mode 0 (amplitudes) and mode 2 (adjoint weights):
// r = P(i,j) / Q(i,j) of an o x o pair index, source i o + j.  mode 1 (g tile of
// batch [a0, a0+nA)): r = rowp / rowm(a', b), source a'(v - a0) + b - a0.
struct PmRows {
    int mode;
    int64_t o;       // mode 0
    int64_t a0, nA;  // mode 1
};
__host__ __device__ inline int64_t pm_src_row(const PmRows& rw, int64_t v, int64_t r, bool plus) {
    int64_t i, j;
    if (rw.mode != 1) {
        if (plus) pm_unP(r, i, j); else pm_unQ(r, i, j);
        return i * rw.o + j;
    }
    const int64_t a0 = rw.a0, nA = rw.nA;
    const double K2 = 2.0 * (double)(plus ? v - a0 : v - a0 - 1) + 1.0;
    int64_t ap = (int64_t)(0.5 * (K2 - sqrt(fmax(K2 * K2 - 8.0 * (double)r, 0.0))));
    if (ap < 0) ap = 0;
    if (ap > nA - 1) ap = nA - 1;
    while (ap > 0 && (plus ? pm_gp_off(ap, v, a0) : pm_gm_off(ap, v, a0)) > r) --ap;
    while (ap + 1 < nA && (plus ? pm_gp_off(ap + 1, v, a0) : pm_gm_off(ap + 1, v, a0)) <= r) ++ap;
    const int64_t b = a0 + ap + (r - (plus ? pm_gp_off(ap, v, a0) : pm_gm_off(ap, v, a0))) + (plus ? 0 : 1);
    return ap * (v - a0) + (b - a0);
}

// Packed row r, tile pair (c0, d0), from the staged A, B:
//   plus:  out[P(c,d)] = off (M_cd + M_dc) for c < d, dg M_cc for c = d,
//   minus: out[Q(c,d)] = off (M_cd - M_dc).
// Amplitudes (mode 0): off = 1/2, dg = 1.  g (mode 1): off = 1, dg = 1 (the w_cc = 1/2
// folded in).  Adjoint weights (mode 2): plus off = 1/2 (i = j) or 1, dg = 2 off; minus off = 1.
__host__ __device__ inline void pm_pack_sym_tile(const PmTile& A, const PmTile& B, int64_t v, int64_t c0, int64_t d0,
                                                 bool plus, double off, double dg, double* o, int tid, int nth) {
    for (int e = tid; e < PM_T * PM_T; e += nth) {
        const int q = e / PM_T, rr = e % PM_T;  // d offset, c offset (c is contiguous in the packed index)
        const int64_t c = c0 + rr, d = d0 + q;
        if (c >= v || d >= v || (plus ? c > d : c >= d)) continue;
        const double mcd = A[rr][q], mdc = B[q][rr];
        if (plus) o[pm_P(c, d)] = c == d ? dg * mcd : off * (mcd + mdc);
        else o[pm_Q(c, d)] = off * (mcd - mdc);
    }
}

// Whole-block bodies: the kernels below run them with (threadIdx.x, blockDim.x)
// and a barrier, the host check with (0, 1) and no barrier.
struct PmBarrier {
    __device__ void operator()() const { __syncthreads(); }
};
struct PmNoBarrier {
    __host__ __device__ void operator()() const {}
};

// The antisymmetric row that shares plus row r's source matrix, or -1 when the
// source pair is diagonal (i = j, or b = a for g) and has no antisymmetric part.
__host__ __device__ inline int64_t pm_minus_row(const PmRows& rw, int64_t v, int64_t r) {
    if (rw.mode != 1) {
        int64_t i, j;
        pm_unP(r, i, j);
        return i < j ? pm_Q(i, j) : -1;
    }
    const int64_t K = v - rw.a0, src = pm_src_row(rw, v, r, true);  // ap K + (b - a0)
    const int64_t ap = src / K, b = rw.a0 + src % K, a = rw.a0 + ap;
    return b > a ? pm_gm_off(ap, v, rw.a0) + (b - a - 1) : -1;
}

// Plus row r and its minus row (when there is one and outm is not NULL) from one
// staging of tile pair tpair of their common source matrix.
template <class Sync>
__host__ __device__ inline void pm_pack_pair_block(const double* src, int64_t v, const PmRows& rw, int64_t r, int64_t tpair,
                                                   double* outp, double* outm, PmTile& A, PmTile& B, int tid, int nth,
                                                   Sync sync) {
    int64_t cb, db;
    pm_unP(tpair, cb, db);
    const int64_t c0 = cb * PM_T, d0 = db * PM_T;
    pm_stage_pair(src + pm_src_row(rw, v, r, true) * v * v, v, c0, d0, A, B, tid, nth);
    sync();
    const double moff = rw.mode == 0 ? 0.5 : 1.0;
    double off = moff, dg = 1.0;
    if (rw.mode == 2) {
        int64_t i, j;
        pm_unP(r, i, j);
        off = i == j ? 0.5 : 1.0;
        dg = 2.0 * off;
    }
    pm_pack_sym_tile(A, B, v, c0, d0, true, off, dg, outp + r * pm_P2(v), tid, nth);
    const int64_t rm = outm ? pm_minus_row(rw, v, r) : -1;
    if (rm >= 0) pm_pack_sym_tile(A, B, v, c0, d0, false, moff, 1.0, outm + rm * pm_Q2(v), tid, nth);
}

// Tiles (alpha) and (beta) of a batch [b0, b0+nB): block row `row` = (b - b0)(b0 + nB) + a
// for a < b0 + nB, tile pair tpair of (c, d).  The packed row (a, b) is staged when the
// pair contributes (alpha: a < b, beta: a <= b); otherwise zeros are written.
template <class Sync>
__host__ __device__ inline void pm_tile_ab_block(const double* dp, const double* dm, int64_t v, int64_t b0, int64_t nB,
                                                 int64_t row, int64_t tpair, bool alpha, double* T, PmTile& Pp,
                                                 PmTile& Pm, int tid, int nth, Sync sync) {
    int64_t cb, db;
    pm_unP(tpair, cb, db);
    const int64_t c0 = cb * PM_T, d0 = db * PM_T, A = b0 + nB;
    const int64_t bl = row / A, a = row % A, b = b0 + bl;
    const bool live = alpha ? a < b : a <= b;
    if (live) {
        const double* prow = dp + (pm_P(a, b) - pm_P2(b0)) * pm_P2(v);
        const double* mrow = a < b ? dm + (pm_Q(a, b) - pm_Q2(b0)) * pm_Q2(v) : nullptr;
        for (int e = tid; e < PM_T * PM_T; e += nth) {  // Pp[q][rr] = dp[P(x, y')], x = c0 + rr <= y' = d0 + q
            const int q = e / PM_T, rr = e % PM_T;
            const int64_t x = c0 + rr, yy = d0 + q;
            const bool in = x < v && yy < v && x <= yy;
            Pp[q][rr] = in ? prow[pm_P(x, yy)] : 0.0;
            Pm[q][rr] = (in && x < yy && mrow) ? mrow[pm_Q(x, yy)] : 0.0;
        }
    }
    sync();
    const bool same = c0 == d0;
    // D_{ab, x y'} = Pp + Pm and D_{ab, y' x} = Pp - Pm for x = c0 + rr <= y' = d0 + q
    if (alpha) {  // T[(bl v + y)][a v + w] = D_{ab, w y}; K = (b0 + nB) v
        const int64_t K = A * v;
        double* base = T + bl * v * K + a * v;
        for (int e = tid; e < PM_T * PM_T; e += nth) {
            {   // (w, y) = (x, y'): row y', column x (x contiguous)
                const int q = e / PM_T, rr = e % PM_T;
                const int64_t x = c0 + rr, yy = d0 + q;
                if (x < v && yy < v && (!same || rr <= q)) base[yy * K + x] = live ? Pp[q][rr] + Pm[q][rr] : 0.0;
            }
            {   // (w, y) = (y', x), y' > x: row x, column y' (y' contiguous)
                const int rr = e / PM_T, q = e % PM_T;
                const int64_t x = c0 + rr, yy = d0 + q;
                if (x < v && yy < v && (!same || q > rr)) base[x * K + yy] = live ? Pp[q][rr] - Pm[q][rr] : 0.0;
            }
        }
    } else {  // T[(a v + y)][bl v + w] = D_{ab, y w}; K = nB v
        const int64_t K = nB * v;
        double* base = T + a * v * K + bl * v;
        for (int e = tid; e < PM_T * PM_T; e += nth) {
            {   // (y, w) = (x, y'): row x, column y' (y' contiguous)
                const int rr = e / PM_T, q = e % PM_T;
                const int64_t x = c0 + rr, yy = d0 + q;
                if (x < v && yy < v && (!same || rr <= q)) base[x * K + yy] = live ? Pp[q][rr] + Pm[q][rr] : 0.0;
            }
            {   // (y, w) = (y', x), y' > x: row y', column x (x contiguous)
                const int q = e / PM_T, rr = e % PM_T;
                const int64_t x = c0 + rr, yy = d0 + q;
                if (x < v && yy < v && (!same || q > rr)) base[yy * K + x] = live ? Pp[q][rr] - Pm[q][rr] : 0.0;
            }
        }
    }
}

// Launch shape of the tiled kernels: grid.x = tile pairs, rows over (y, z); the
// row test is uniform per block, so every thread of a working block reaches the barrier.
__device__ inline int64_t pm_block_row() { return (int64_t)blockIdx.y + (int64_t)blockIdx.z * gridDim.y; }

// Grid: pm_grid(v, plus rows); outm NULL packs the plus rows only.
__global__ __launch_bounds__(256) void pm_pack_pair_tiled_kernel(const double* __restrict__ src, int64_t v, PmRows rw,
                                                                 int64_t nrows, double* __restrict__ outp,
                                                                 double* __restrict__ outm) {
    __shared__ PmTile A, B;
    const int64_t r = pm_block_row();
    if (r >= nrows) return;
    pm_pack_pair_block(src, v, rw, r, blockIdx.x, outp, outm, A, B, threadIdx.x, blockDim.x, PmBarrier{});
}

__global__ __launch_bounds__(256) void pm_tile_ab_kernel(const double* __restrict__ dp, const double* __restrict__ dm,
                                                          int64_t v, int64_t b0, int64_t nB, int alpha,
                                                          double* __restrict__ T) {
    __shared__ PmTile Pp, Pm;
    const int64_t row = pm_block_row();
    if (row >= nB * (b0 + nB)) return;
    pm_tile_ab_block(dp, dm, v, b0, nB, row, blockIdx.x, alpha != 0, T, Pp, Pm, threadIdx.x, blockDim.x, PmBarrier{});
}

}  // namespace ladder
