// gemm_f64.hpp -- FP64 MFMA GEMM for gfx950 with layout-permuting epilogues.
//
//   C(m, n) = sum_k A(m, k) * B(k, n)         m < M, n < N, k < K
//
// A is read either K-contiguous, A(m,k) = A[m*lda + k], or M-contiguous,
// A(m,k) = A[k*lda + m]; B either K-contiguous, B(k,n) = B[n*ldb + k], or
// N-contiguous, B(k,n) = B[k*ldb + n].  Both are staged through LDS as [k][m]
// and [k][n] tiles (row stride 129 doubles, so the transposing stores of the
// K-contiguous case spread over the banks), double-buffered with one barrier per
// K-step.  Each of the 4 waves owns a 64x64 sub-tile made of 4x4
// v_mfma_f64_16x16x4_f64 blocks (128 accumulator VGPRs).
//
// The epilogue functor receives every finished element with its (m, n) and
// decides where it goes; tiles on the M/N/K edges are zero-padded on load and
// masked on store, so any M, N, K >= 1 works.
//
// Tiles are walked in an XCD-aware order: the hardware hands workgroup w to XCD
// w % 8, so the linear id is remapped to give each XCD a contiguous range of
// tiles, and that range is walked in groups of GROUP_M tile-rows so that
// neighbouring workgroups share A rows and B columns in the XCD's L2.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ladder {

typedef double dx4 __attribute__((ext_vector_type(4)));

constexpr int F64_BM = 128;
constexpr int F64_BN = 128;
constexpr int F64_BK = 16;
constexpr int F64_LDS = 129;  // LDS row stride in doubles
constexpr int F64_THREADS = 256;
constexpr int GROUP_M = 8;
constexpr int NUM_XCD = 8;

struct TileMap {
    int64_t tiles_m, tiles_n;
};

// Linear workgroup id -> (tile row, tile col), XCD-contiguous and grouped: the tiles an XCD
// runs are consecutive, walked in groups of gm tile rows, column by column.
__device__ inline void map_tile(int64_t w, int64_t T, const TileMap& tm, int64_t& ti, int64_t& tj,
                                int gm = GROUP_M) {
    const int64_t xcd = w % NUM_XCD, local = w / NUM_XCD;
    const int64_t per = T / NUM_XCD, rem = T % NUM_XCD;
    const int64_t tile = xcd * per + (xcd < rem ? xcd : rem) + local;
    const int64_t group = (int64_t)gm * tm.tiles_n;
    const int64_t g = tile / group;
    const int64_t first = g * gm;
    const int64_t gsz = (tm.tiles_m - first) < gm ? (tm.tiles_m - first) : gm;
    const int64_t in = tile - g * group;
    ti = first + in % gsz;
    tj = in / gsz;
}

// Global -> registers for one BMxBK (or BNxBK) tile: 8 doubles per thread.
template <bool KCONTIG>
__device__ inline void f64_load(const double* __restrict__ p, int64_t ld, int64_t r0, int64_t R,
                                int64_t k0, int64_t K, double (&reg)[8], int tid) {
    if constexpr (KCONTIG) {
        const int kk = tid & 15, rr = tid >> 4;
        const int64_t k = k0 + kk;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int64_t r = r0 + rr + 16 * i;
            reg[i] = (r < R && k < K) ? p[r * ld + k] : 0.0;
        }
    } else {
        const int rr = tid & 127, kk = tid >> 7;
        const int64_t r = r0 + rr;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int64_t k = k0 + kk + 2 * i;
            reg[i] = (r < R && k < K) ? p[k * ld + r] : 0.0;
        }
    }
}

template <bool KCONTIG>
__device__ inline void f64_stage(double* s, const double (&reg)[8], int tid) {
    if constexpr (KCONTIG) {
        const int kk = tid & 15, rr = tid >> 4;
#pragma unroll
        for (int i = 0; i < 8; ++i) s[kk * F64_LDS + rr + 16 * i] = reg[i];
    } else {
        const int rr = tid & 127, kk = tid >> 7;
#pragma unroll
        for (int i = 0; i < 8; ++i) s[(kk + 2 * i) * F64_LDS + rr] = reg[i];
    }
}

struct GemmShape {
    const double* A;
    int64_t lda;
    const double* B;
    int64_t ldb;
    int64_t M, N, K;
};

// Finished-tile visitor: calls epi(m, n, value) for every in-range element and
// lets the epilogue fold a per-workgroup scalar (used for energy partials).
// STAGE only names the instantiation (one kernel symbol per stage in profiles).
template <bool A_KCONTIG, bool B_KCONTIG, class Epi, int STAGE>
__global__ __launch_bounds__(F64_THREADS) void gemm_f64_kernel(GemmShape s, Epi epi) {
    __shared__ double As[2][F64_BK * F64_LDS];
    __shared__ double Bs[2][F64_BK * F64_LDS];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    TileMap tmap{(s.M + F64_BM - 1) / F64_BM, (s.N + F64_BN - 1) / F64_BN};
    int64_t ti, tj;
    map_tile(blockIdx.x, (int64_t)gridDim.x, tmap, ti, tj);
    const int64_t m0 = ti * F64_BM, n0 = tj * F64_BN;

    dx4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = dx4{0.0, 0.0, 0.0, 0.0};

    double ra[8], rb[8];
    const int64_t nk = (s.K + F64_BK - 1) / F64_BK;
    f64_load<A_KCONTIG>(s.A, s.lda, m0, s.M, 0, s.K, ra, tid);
    f64_load<B_KCONTIG>(s.B, s.ldb, n0, s.N, 0, s.K, rb, tid);
    f64_stage<A_KCONTIG>(As[0], ra, tid);
    f64_stage<B_KCONTIG>(Bs[0], rb, tid);
    __syncthreads();

    const int lr = lane & 15, lk = lane >> 4;
    for (int64_t kt = 0; kt < nk; ++kt) {
        const int cur = (int)(kt & 1);
        if (kt + 1 < nk) {
            f64_load<A_KCONTIG>(s.A, s.lda, m0, s.M, (kt + 1) * F64_BK, s.K, ra, tid);
            f64_load<B_KCONTIG>(s.B, s.ldb, n0, s.N, (kt + 1) * F64_BK, s.K, rb, tid);
        }
        const double* as = As[cur] + wm * 64 + lr;
        const double* bs = Bs[cur] + wn * 64 + lr;
#pragma unroll
        for (int ks = 0; ks < F64_BK / 4; ++ks) {
            const int k = ks * 4 + lk;
            double a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = as[k * F64_LDS + 16 * i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = bs[k * F64_LDS + 16 * j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        if (kt + 1 < nk) {
            f64_stage<A_KCONTIG>(As[cur ^ 1], ra, tid);
            f64_stage<B_KCONTIG>(Bs[cur ^ 1], rb, tid);
        }
        __syncthreads();
    }

    // D layout of v_mfma_f64_16x16x4_f64 on gfx950 (measured): lane l, element r holds
    // row (l/16) + 4r, column l%16.
    typename Epi::Local loc = epi.begin();
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t m = m0 + wm * 64 + 16 * i + lk + 4 * r;
                const int64_t n = n0 + wn * 64 + 16 * j + lr;
                if (m < s.M && n < s.N) epi.put(loc, m, n, acc[i][j][r]);
            }
    epi.finish(loc, blockIdx.x);
}

// ----------------------------------------------------------------- epilogues

// out[((x1*Y1 + y1)*X2 + x2)*Y2 + y2] = C + beta*out, with m = x1*X2 + x2 and
// n = y1*Y2 + y2: swaps the two middle indices of a 4-index result.
struct EpiSwapMid {
    double* out;
    int64_t X2, Y1, Y2;
    double alpha, beta;
    struct Local {};
    __device__ Local begin() const { return {}; }
    __device__ void put(Local&, int64_t m, int64_t n, double c) const {
        const int64_t x1 = m / X2, x2 = m - x1 * X2;
        const int64_t y1 = n / Y2, y2 = n - y1 * Y2;
        double* p = out + ((x1 * Y1 + y1) * X2 + x2) * Y2 + y2;
        *p = beta == 0.0 ? alpha * c : alpha * c + beta * *p;
    }
    __device__ void finish(Local&, int64_t) const {}
};

// out[m*ldc + n] = alpha*C + beta*out; optionally partial[w] = sum w8[m*ldc+n]*C over the tile.
struct EpiStrided {
    double* out;
    int64_t ldc;
    double alpha, beta;
    const double* weight;  // NULL: no energy partial
    double* partial;       // one slot per workgroup
    struct Local {
        double e;
    };
    __device__ Local begin() const { return {0.0}; }
    __device__ void put(Local& l, int64_t m, int64_t n, double c) const {
        double* p = out + m * ldc + n;
        if (weight) l.e += weight[m * ldc + n] * c;
        *p = beta == 0.0 ? alpha * c : alpha * c + beta * *p;
    }
    // Needs every thread of the block (it has a barrier); any block size up to 1024.
    __device__ void finish(Local& l, int64_t w) const {
        if (!weight) return;
        __shared__ double red[16];
        double e = l.e;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += red[i];
            partial[w] = t;
        }
    }
};

// General placement: m = x1*X2 + x2, n = y1*Y2 + y2 and
// out[x1*sx1 + x2*sx2 + y1*sy1 + y2*sy2] = alpha*C + beta*out, for results written into
// a slab of a larger array (strides independent of the index decomposition).
struct EpiPlace {
    double* out;
    int64_t X2, Y2;
    int64_t sx1, sx2, sy1, sy2;
    double alpha, beta;
    struct Local {};
    __device__ Local begin() const { return {}; }
    __device__ void put(Local&, int64_t m, int64_t n, double c) const {
        const int64_t x1 = m / X2, x2 = m - x1 * X2;
        const int64_t y1 = n / Y2, y2 = n - y1 * Y2;
        double* p = out + x1 * sx1 + x2 * sx2 + y1 * sy1 + y2 * sy2;
        *p = beta == 0.0 ? alpha * c : alpha * c + beta * *p;
    }
    __device__ void finish(Local&, int64_t) const {}
};

// First-order amplitudes: m = i*v + a, n = j*v + b,
// t[((i*o + j)*v + a)*v + b] = C / ((eps_i + eps_j) - (eps_a + eps_b)).
struct EpiMP2 {
    double* t;
    const double* eps;
    int64_t o, v;
    struct Local {};
    __device__ Local begin() const { return {}; }
    __device__ void put(Local&, int64_t m, int64_t n, double c) const {
        const int64_t i = m / v, a = m - i * v;
        const int64_t j = n / v, b = n - j * v;
        const double den = (eps[i] + eps[j]) - (eps[o + a] + eps[o + b]);
        t[((i * o + j) * v + a) * v + b] = c / den;
    }
    __device__ void finish(Local&, int64_t) const {}
};

}  // namespace ladder
