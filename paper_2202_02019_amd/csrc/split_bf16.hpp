// split_bf16.hpp -- exponent-aligned BF16 slicing and the split GEMM on BF16 MFMA.
//
// Representation.  An FP64 operand matrix (rows r, contraction index k) is cut
// along k into chunks of KC = 256.  Each (row, chunk) gets one exponent e with
// max|x| < 2^e over the chunk, and each element is written as
//     x = 2^e * sum_{p<S} s_p + residual,   s_p = m_p * 2^(-8(p+1)),
// with integers |m_0| <= 256 and |m_p| <= 128 (p >= 1) taken by round-to-nearest
// of the running remainder (every step is exact in FP64), |residual| <= 2^(e-8S-1).
// Every s_p is exact in BF16 (8 significant bits).  This is the error-free
// splitting of Ozaki, Ogita, Oishi and Rump (Numer. Algorithms 2012) with a
// shared exponent per row and chunk.
//
// Product.  For a chunk, the slice pairs (p, q) with p + q < S are multiplied on
// v_mfma_f32_32x32x16_bf16 into three FP32 accumulators:
//   acc0 <- (0,0):        terms are multiples of 2^-16 below 1, at most 256 of
//                         them, so every partial sum is a multiple of 2^-16 of
//                         magnitude <= 2^8: exact in FP32 (24-bit significand);
//   acc1 <- (0,1), (1,0): multiples of 2^-24 of magnitude <= 2^-9, 512 terms,
//                         partial sums <= 1: exact in FP32;
//   acc2 <- p + q >= 2:   rounded in FP32; its rounding error is below
//                         2^-24 * 2^-16 * 256 relative to the chunk scale,
//                         i.e. under 2^-32 of the chunk's sum_k |a||b| bound.
// After each chunk the three are combined in FP64 (acc0 + acc1 exact),
// scaled by 2^(eA + eB) and added to an FP64 accumulator.  The pairs with
// p + q >= S are dropped (triangular truncation), an error of about
// (S+1) 2^(-8S) of max|a| max|b| per term.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gemm_f64.hpp"

namespace ladder {

typedef float fx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bx8 __attribute__((ext_vector_type(8)));
typedef unsigned short ux8 __attribute__((ext_vector_type(8)));

constexpr int SPLIT_KC = 256;       // chunk length along k
constexpr int SPLIT_KALIGN = 16;    // k is padded with zeros to a multiple of this
constexpr int SPLIT_MAX_S = 6;
constexpr int SPLIT_BM = 128, SPLIT_BN = 128, SPLIT_BK = 16;
constexpr int SPLIT_LDS_ROW = 24;   // bf16 per LDS row: 16 data + 8 pad (48 bytes, bank-spread)
constexpr int SPLIT_THREADS = 512;

__host__ __device__ inline int64_t split_kpad(int64_t K) { return (K + SPLIT_KALIGN - 1) / SPLIT_KALIGN * SPLIT_KALIGN; }
__host__ __device__ inline int64_t split_nchunk(int64_t K) { return (K + SPLIT_KC - 1) / SPLIT_KC; }

__device__ inline unsigned short bf16_bits_exact(double v) {
    // v has at most 8 significant bits and a normal BF16 exponent: the float
    // conversion is exact and the low 16 bits of the float are zero.
    const float f = (float)v;
    return (unsigned short)(__builtin_bit_cast(uint32_t, f) >> 16);
}

// Exponent of a chunk maximum: smallest e with mx < 2^e (0 for an all-zero chunk).
__device__ inline int chunk_exponent(double mx) {
    if (!(mx > 0.0) || !__builtin_isfinite(mx)) return 0;
    int e;
    (void)frexp(mx, &e);
    return e;
}

// Writes the S slices of x (given the chunk exponent) to out[p * slice_stride].
template <int S>
__device__ inline void write_slices(double x, int e, unsigned short* out, int64_t slice_stride) {
    double y = ldexp(x, -e);
    double sc = 1.0 / 256.0;
#pragma unroll
    for (int p = 0; p < S; ++p) {
        const double u = y * 256.0;
        const double m = rint(u);
        out[p * slice_stride] = bf16_bits_exact(m * sc);
        y = u - m;
        sc *= 1.0 / 256.0;
    }
}

// ---------------------------------------------------------------- slicers
// K-contiguous source: element (r, k) at src[r*ld + k], r < R, k < K.
// One wave per (row, chunk).  slices: [S][R][Kp] (row stride Kp = split_kpad(K));
// exps: [nchunk][R] (chunk stride ldexp_rows).
template <int S>
__global__ __launch_bounds__(256) void slice_rows_kernel(const double* __restrict__ src, int64_t ld, int64_t R,
                                                         int64_t K, unsigned short* __restrict__ slices,
                                                         int* __restrict__ exps, int64_t exp_ld) {
    const int lane = threadIdx.x & 63;
    const int64_t nch = split_nchunk(K), Kp = split_kpad(K);
    const int64_t job = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (job >= R * nch) return;
    const int64_t r = job / nch, ch = job - r * nch;
    double x[SPLIT_KC / 64];
    double mx = 0.0;
    bool bad = false;
#pragma unroll
    for (int t = 0; t < SPLIT_KC / 64; ++t) {
        const int64_t k = ch * SPLIT_KC + lane + 64 * t;
        x[t] = k < K ? src[r * ld + k] : 0.0;
        mx = fmax(mx, fabs(x[t]));
        bad |= !__builtin_isfinite(x[t]);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
    const int e = chunk_exponent(mx);
    if (lane == 0) exps[ch * exp_ld + r] = e;
    (void)bad;
    const int64_t slice_stride = R * Kp;
#pragma unroll
    for (int t = 0; t < SPLIT_KC / 64; ++t) {
        const int64_t k = ch * SPLIT_KC + lane + 64 * t;
        if (k < Kp) write_slices<S>(x[t], e, slices + r * Kp + k, slice_stride);
    }
}

// Transposed source: element (r, k) at src[k*ld + r].  One workgroup per 32 rows
// and one chunk, staged through LDS so that both the reads (along r) and the
// slice writes (along k) are contiguous.
template <int S>
__global__ __launch_bounds__(256) void slice_cols_kernel(const double* __restrict__ src, int64_t ld, int64_t R,
                                                         int64_t K, unsigned short* __restrict__ slices,
                                                         int* __restrict__ exps, int64_t exp_ld) {
    constexpr int RT = 32;
    __shared__ double tile[SPLIT_KC][RT + 1];
    __shared__ int ex[RT];
    const int tid = threadIdx.x;
    const int64_t Kp = split_kpad(K);
    const int64_t rblocks = (R + RT - 1) / RT;
    const int64_t rb = blockIdx.x % rblocks, ch = blockIdx.x / rblocks;
    const int64_t r0 = rb * RT, k0 = ch * SPLIT_KC;
    {
        const int rr = tid & (RT - 1), kk = tid >> 5;  // 8 k rows per pass
        const int64_t r = r0 + rr;
        for (int i = 0; i < SPLIT_KC / 8; ++i) {
            const int64_t k = k0 + kk + 8 * i;
            tile[kk + 8 * i][rr] = (r < R && k < K) ? src[k * ld + r] : 0.0;
        }
    }
    __syncthreads();
    const int rr = tid >> 3, part = tid & 7;  // 8 threads per row, 32 k each
    double mx = 0.0;
    for (int i = 0; i < SPLIT_KC / 8; ++i) mx = fmax(mx, fabs(tile[part * 32 + i][rr]));
#pragma unroll
    for (int off = 4; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
    if (part == 0) ex[rr] = chunk_exponent(mx);
    __syncthreads();
    const int64_t r = r0 + rr;
    if (r >= R) return;
    const int e = ex[rr];
    if (part == 0) exps[ch * exp_ld + r] = e;
    const int64_t slice_stride = R * Kp;
    for (int i = 0; i < 32; ++i) {
        const int64_t k = k0 + part * 32 + i;
        if (k < Kp) write_slices<S>(tile[part * 32 + i][rr], e, slices + r * Kp + k, slice_stride);
    }
}

// ---------------------------------------------------------------- split GEMM
struct SplitOperand {
    const unsigned short* s;  // slice 0 of row 0 of this operand view
    int64_t slice_stride;     // elements between slices
    int64_t ld;               // = Kp
    const int* e;             // exponent of (row 0, chunk 0) of this view
    int64_t e_ld;             // chunk stride of the exponent array
};

struct SplitShape {
    SplitOperand a, b;
    int64_t M, N, K;  // K = real length (chunks and padding follow from it)
};

// 512 threads = 8 waves in a 4 x 2 grid; wave (wm, wn) owns rows wm*32 .. +32 and
// columns wn*64 .. +64 of the 128 x 128 tile (two 32x32 MFMA blocks), so two
// waves share each SIMD and one's MFMAs overlap the other's FP64 combine.
template <int S, class Epi>
__global__ __launch_bounds__(SPLIT_THREADS) void gemm_split_kernel(SplitShape sh, Epi epi) {
    __shared__ unsigned short As[2][S][SPLIT_BM * SPLIT_LDS_ROW];
    __shared__ unsigned short Bs[2][S][SPLIT_BN * SPLIT_LDS_ROW];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    TileMap tmap{(sh.M + SPLIT_BM - 1) / SPLIT_BM, (sh.N + SPLIT_BN - 1) / SPLIT_BN};
    int64_t ti, tj;
    map_tile(blockIdx.x, (int64_t)gridDim.x, tmap, ti, tj);
    const int64_t m0 = ti * SPLIT_BM, n0 = tj * SPLIT_BN;
    const int64_t Kp = split_kpad(sh.K);
    const int64_t nk = Kp / SPLIT_BK;

    // global -> LDS: threads 0..255 move A, 256..511 move B; 16 bytes (8 k) of
    // row (t%256)/2, half t%2, for every slice.
    const bool is_b = tid >= 256;
    const int lrow = (tid & 255) >> 1, lhalf = tid & 1;
    const SplitOperand& op = is_b ? sh.b : sh.a;
    const bool in = (is_b ? n0 : m0) + lrow < (is_b ? sh.N : sh.M);
    const unsigned short* gsrc = op.s + ((is_b ? n0 : m0) + lrow) * op.ld + 8 * lhalf;
    const int64_t gstride = op.slice_stride;
    unsigned short* ldst0 = is_b ? &Bs[0][0][0] : &As[0][0][0];
    constexpr int LDS_SLICE = SPLIT_BM * SPLIT_LDS_ROW;
    const int lds_w = lrow * SPLIT_LDS_ROW + 8 * lhalf;

    ux8 rg[S];
    auto gload = [&](int64_t kt) {
#pragma unroll
        for (int p = 0; p < S; ++p)
            rg[p] = in ? *(const ux8*)(gsrc + p * gstride + kt * SPLIT_BK) : ux8{0, 0, 0, 0, 0, 0, 0, 0};
    };
    auto lstore = [&](int buf) {
#pragma unroll
        for (int p = 0; p < S; ++p) *(ux8*)(ldst0 + (buf * S + p) * LDS_SLICE + lds_w) = rg[p];
    };

    fx16 acc[3][2];
    double acc64[2][16];
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
#pragma unroll
        for (int g = 0; g < 3; ++g) acc[g][bj] = fx16{};
#pragma unroll
        for (int r = 0; r < 16; ++r) acc64[bj][r] = 0.0;
    }

    // MFMA fragment read offsets: row l%32 of the 32-row block, k half l/32.
    const int frag = (lane & 31) * SPLIT_LDS_ROW + 8 * (lane >> 5);
    const int arow = (wm * 32) * SPLIT_LDS_ROW + frag;
    const int brow0 = (wn * 64) * SPLIT_LDS_ROW + frag;
    const int brow1 = (wn * 64 + 32) * SPLIT_LDS_ROW + frag;

    gload(0);
    lstore(0);
    __syncthreads();
    for (int64_t kt = 0; kt < nk; ++kt) {
        const int cur = (int)(kt & 1);
        if (kt + 1 < nk) gload(kt + 1);

        bx8 bq[S][2];
#pragma unroll
        for (int q = 0; q < S; ++q) {
            bq[q][0] = __builtin_bit_cast(bx8, *(const ux8*)(&Bs[cur][q][brow0]));
            bq[q][1] = __builtin_bit_cast(bx8, *(const ux8*)(&Bs[cur][q][brow1]));
        }
#pragma unroll
        for (int p = 0; p < S; ++p) {
            const bx8 ap = __builtin_bit_cast(bx8, *(const ux8*)(&As[cur][p][arow]));
#pragma unroll
            for (int q = 0; q < S - p; ++q) {
                const int g = (p + q) < 2 ? (p + q) : 2;
#pragma unroll
                for (int bj = 0; bj < 2; ++bj)
                    acc[g][bj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ap, bq[q][bj], acc[g][bj], 0, 0, 0);
            }
        }

        // end of a chunk (or of k): fold the exact FP32 chunk sums into FP64
        if (((kt + 1) % (SPLIT_KC / SPLIT_BK)) == 0 || kt + 1 == nk) {
            const int64_t ch = kt / (SPLIT_KC / SPLIT_BK);
            const int* ea_row = sh.a.e + ch * sh.a.e_ld;
            const int* eb_row = sh.b.e + ch * sh.b.e_ld;
            int eb[2];
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) {
                const int64_t n = n0 + wn * 64 + 32 * bj + (lane & 31);
                eb[bj] = n < sh.N ? eb_row[n] : 0;
            }
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t m = m0 + wm * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                const int ea = m < sh.M ? ea_row[m] : 0;
#pragma unroll
                for (int bj = 0; bj < 2; ++bj) {
                    const double t = ((double)acc[0][bj][r] + (double)acc[1][bj][r]) + (double)acc[2][bj][r];
                    acc64[bj][r] += ldexp(t, ea + eb[bj]);
                }
            }
#pragma unroll
            for (int g = 0; g < 3; ++g)
#pragma unroll
                for (int bj = 0; bj < 2; ++bj) acc[g][bj] = fx16{};
        }

        if (kt + 1 < nk) lstore(cur ^ 1);
        __syncthreads();
    }

    // D layout of v_mfma_f32_32x32x16_bf16 (measured on gfx950): lane l, element r
    // holds row 8*(r/4) + 4*(l/32) + r%4, column l%32.
    typename Epi::Local loc = epi.begin();
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int64_t m = m0 + wm * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
            const int64_t n = n0 + wn * 64 + 32 * bj + (lane & 31);
            if (m < sh.M && n < sh.N) epi.put(loc, m, n, acc64[bj][r]);
        }
    epi.finish(loc, blockIdx.x);
}

}  // namespace ladder
