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
// Every kernel is a grid-stride loop over one element function; the element
// functions are host-callable so that the index arithmetic can be checked on the
// CPU against the dense definition.
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

// tbar -> wp[P(i,j)][(a,b)] = (2 - delta_ij) (t_ij^ab + t_ij^ba)/2, wm[Q(i,j)][(a,b)] = t_ij^ab - t_ij^ba.
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

// D tile [(a',c)][(b,d)] of a batch from dp[(a',b)][P(c,d)] and dm[(a',b)][Q(c,d)]:
//   D_{ab,cd} = dp[(a,b)][P(min,max)] + s_cd dm[(a,b)][Q(min,max)].
// Slot t enumerates (a', b, c, d) with d fastest: one (a', b) at a time, so the
// packed rows being gathered stay in L2 while whole d-runs of D are written.
__host__ __device__ inline void pm_unpack_D_elem(int64_t t, const double* dp, const double* dm, int64_t v, double* D) {
    const int64_t cp = pm_P2(v), cm = pm_Q2(v);
    const int64_t d = t % v, c = (t / v) % v, row = t / (v * v);  // row = a' v + b
    const int64_t b = row % v, ap = row / v;
    const int64_t lo = c < d ? c : d, hi = c < d ? d : c;
    double x = dp[row * cp + pm_P(lo, hi)];
    if (c != d) x += (c < d ? 1.0 : -1.0) * dm[row * cm + pm_Q(lo, hi)];
    D[((ap * v + c) * v + b) * v + d] = x;
}

#define PM_GRID_STRIDE(total) \
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < (total); t += (int64_t)gridDim.x * blockDim.x)

__global__ void pm_pack_amp_kernel(const double* __restrict__ x, int64_t o, int64_t v, double* __restrict__ xp,
                                   double* __restrict__ xm) {
    PM_GRID_STRIDE(pm_amp_count(o, v)) pm_pack_amp_elem(t, x, o, v, xp, xm);
}
__global__ void pm_pack_w_kernel(const double* __restrict__ x, int64_t o, int64_t v, double* __restrict__ wp,
                                 double* __restrict__ wm) {
    PM_GRID_STRIDE(pm_w_count(o, v)) pm_pack_w_elem(t, x, o, v, wp, wm);
}
__global__ void pm_pack_g_kernel(const double* __restrict__ g, int64_t v, int64_t a0, int64_t nA, double* __restrict__ gp,
                                 double* __restrict__ gm) {
    PM_GRID_STRIDE(pm_g_count(v, a0, nA)) pm_pack_g_elem(t, g, v, a0, nA, gp, gm);
}
__global__ void pm_unpack_D_kernel(const double* __restrict__ dp, const double* __restrict__ dm, int64_t v, int64_t nA,
                                   double* __restrict__ D) {
    PM_GRID_STRIDE(nA * v * v * v) pm_unpack_D_elem(t, dp, dm, v, D);
}
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
