// split_i8.hpp -- exponent-aligned INT8 slicing and the split GEMM on INT8 MFMA.
//
// Representation.  As in split_bf16.hpp, an FP64 operand (rows r, contraction
// index k) is cut along k into chunks of KC = 256 with one exponent e per
// (row, chunk), max|x| < 2^e.  Each element is written as
//     x = 2^e * (m_0 2^-6 + m_1 2^-13 + ... + m_{S-1} 2^-(6+7(S-1))) + residual,
// every m_p an integer in [-64, 64] taken by round-to-nearest of the running
// remainder (each step exact in FP64), so |residual| <= 2^(e-7S).  Every m_p fits
// in a signed byte: seven bits per slice against the eight of a BF16 slice, on a
// matrix core with twice the BF16 rate (v_mfma_i32_32x32x32_i8, 32 k per
// instruction).  This is the error-free splitting of Ozaki, Ogita, Oishi and
// Rump (Numer. Algorithms 2012) on integer slices, as in Ootomo, Ozaki and Yokota
// (IJHPCA 2024), with a shared exponent per row and chunk.
//
// Product.  For a chunk, slice pairs (p, q) with p + q < S are multiplied into
// one INT32 accumulator per level L = p + q.  Level L sums at most (L+1) * 256
// products of magnitude <= 2^12, i.e. below (L+1) 2^20 < 2^31: every level is
// exact.  After each chunk the levels are combined in FP64 as
//     t = sum_L acc_L 2^(-7L)   (fold_levels; exact for S <= 5, whose bits span
//                                at most 2^21 .. 2^-28),
// scaled by 2^(eA + eB - 12) and added to an FP64 accumulator.  Pairs with
// p + q >= S are dropped (triangular truncation); the first dropped level S holds
// no square s_p(x)^2 when S is odd, so a symmetric product (both operands slices
// of the same matrix) gains no sign-coherent bias before level S + 1.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "split_bf16.hpp"

namespace ladder {

typedef int ix4 __attribute__((ext_vector_type(4)));
typedef int ix16 __attribute__((ext_vector_type(16)));

constexpr int SPLIT8_KALIGN = 32;  // k is padded with zeros to a multiple of this
constexpr int SPLIT8_BM = 128, SPLIT8_BN = 64, SPLIT8_BK = 32;
constexpr int SPLIT8_THREADS = 512;
// Tile rows per group of the tile walk: with 64-column tiles twice as many columns share
// an A panel as with the 128-column ones, so smaller groups than GROUP_M (4 against 8:
// 2 % off the retinal step; 16: 2 % slower).
constexpr int SPLIT8_GROUP_M = 4;

__host__ __device__ inline int64_t split8_kpad(int64_t K) { return (K + SPLIT8_KALIGN - 1) / SPLIT8_KALIGN * SPLIT8_KALIGN; }

// Slice layout: as the BF16 one with bytes for elements and 32 k per k-block.
// Element (r, k) of slice p at byte
//   p*slice_stride + ((r/128)*nkb + k/32)*4096 + (r%128)*32 + k%32,
// nkb = Kp/32 (Kp = split8_kpad(K)), slice_stride = panels*128*Kp bytes.  One GEMM
// K-step (32 k) of a 128-row tile is a contiguous 4 KB run, as in BF16.
__host__ __device__ inline int64_t split8_slice_stride(int64_t R, int64_t K) {
    return split_panels(R) * SPLIT_PANEL * split8_kpad(K);
}
__host__ __device__ inline int64_t split8_index(int64_t r, int64_t k, int64_t nkb) {
    return ((r >> 7) * nkb + (k >> 5)) * (SPLIT_PANEL * 32) + (r & 127) * 32 + (k & 31);
}

// The S integer slices of x (given its chunk exponent), as bytes.
template <int S>
__device__ inline void slices_i8(double x, int e, int (&m)[S]) {
    double y = ldexp(x, -e) * 64.0;  // |y| < 64
#pragma unroll
    for (int p = 0; p < S; ++p) {
        const double r = rint(y);
        m[p] = (int)r;
        y = (y - r) * 128.0;  // |y - r| <= 1/2
    }
}

// Four consecutive k of one row: the S words (4 bytes each, k ascending in the
// little-endian byte order) written at out + p * slice_stride.
template <int S>
__device__ inline void write_slices_i8x4(const double (&x)[4], int e, int8_t* out, int64_t slice_stride) {
    int m[4][S];
#pragma unroll
    for (int j = 0; j < 4; ++j) slices_i8<S>(x[j], e, m[j]);
#pragma unroll
    for (int p = 0; p < S; ++p) {
        const uint32_t w = (uint32_t)(m[0][p] & 0xff) | ((uint32_t)(m[1][p] & 0xff) << 8) |
                           ((uint32_t)(m[2][p] & 0xff) << 16) | ((uint32_t)(m[3][p] & 0xff) << 24);
        *(uint32_t*)(out + p * slice_stride) = w;
    }
}

// Row-wise source (DenseRows, PmTileRows).  One workgroup per 16 rows and one
// chunk: thread (rr, q) = (t/16, t%16) holds k = chunk*256 + 64j + 4q + i for
// j < 4, i < 4, so each 32-k block of the 16 rows goes out as one 512-byte run
// per slice.
template <int S, class Src>
__global__ __launch_bounds__(256) void slice8_rows_kernel(Src src, int64_t R, int64_t K, int8_t* __restrict__ slices,
                                                          int* __restrict__ exps, int64_t exp_ld) {
    constexpr int RB = 16;
    const int64_t nch = split_nchunk(K), Kp = split8_kpad(K);
    const int64_t rblocks = (R + RB - 1) / RB;
    const int64_t rb = blockIdx.x % rblocks, ch = blockIdx.x / rblocks;
    const int rr = threadIdx.x >> 4, q = threadIdx.x & 15;
    const int64_t r = rb * RB + rr;
    if (ch >= nch) return;  // uniform per block
    double x[4][4];
    double mx = 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t k = ch * SPLIT_KC + 64 * j + 4 * q + i;
            x[j][i] = (r < R && k < K) ? src(r, k) : 0.0;
            mx = fmax(mx, fabs(x[j][i]));
        }
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));  // the 16 lanes of row rr
    if (r >= R) return;
    const int e = chunk_exponent(mx);
    if (q == 0) exps[ch * exp_ld + r] = e;
    const int64_t slice_stride = split8_slice_stride(R, K), nkb = Kp / 32;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t k = ch * SPLIT_KC + 64 * j + 4 * q;
        if (k < Kp) write_slices_i8x4<S>(x[j], e, slices + split8_index(r, k, nkb), slice_stride);
    }
}

// Transposed source: element (r, k) at src[k*ld + r].  One workgroup per 32 rows
// and one chunk, staged through LDS; thread (row, q) = (t/8, t%8) writes k
// = 32 kb + 4q .. +4 of its row, so each 32-k block of the 32 rows is one 1 KB run.
template <int S>
__global__ __launch_bounds__(256) void slice8_cols_kernel(const double* __restrict__ src, int64_t ld, int64_t R,
                                                          int64_t K, int8_t* __restrict__ slices,
                                                          int* __restrict__ exps, int64_t exp_ld) {
    constexpr int RT = 32;
    __shared__ double tile[SPLIT_KC][RT + 1];
    const int tid = threadIdx.x;
    const int64_t Kp = split8_kpad(K);
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
    const int row = tid >> 3, q = tid & 7;  // 8 threads per row, 32 k each
    double mx = 0.0;
    for (int i = 0; i < SPLIT_KC / 8; ++i) mx = fmax(mx, fabs(tile[q * 32 + i][row]));
#pragma unroll
    for (int off = 4; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
    const int e = chunk_exponent(mx);
    const int64_t r = r0 + row;
    if (r >= R) return;
    if (q == 0) exps[ch * exp_ld + r] = e;
    const int64_t slice_stride = split8_slice_stride(R, K), nkb = Kp / 32;
    for (int kb = 0; kb < SPLIT_KC / 32; ++kb) {
        const int64_t k = k0 + 32 * kb + 4 * q;
        if (k >= Kp) break;
        double x[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) x[i] = tile[32 * kb + 4 * q + i][row];
        write_slices_i8x4<S>(x, e, slices + split8_index(r, k, nkb), slice_stride);
    }
}

// ---------------------------------------------------------------- INT8 split GEMM
// SplitShape as for BF16, with a.s / b.s pointing at the byte slices (cast), slice
// strides in bytes and nkb = Kp/32.
//
// 512 threads = 8 waves in a 4 x 2 grid; wave (wm, wn) owns the 32 x 32 block at
// rows wm*32, columns wn*32 of the 128 x 64 tile: S INT32 level accumulators and
// one FP64 accumulator per element (16 S + 32 registers per lane).  Operands go
// to LDS by LDS-DMA through a 3-deep ring of 32-k steps, with the slot layout of
// the BF16 kernel (a 128-row x 32-byte slice tile is 256 16-byte slots): waves
// 0-3 load A, waves 4-5 load B; waves 0, 1 and 4 load the chunk exponents.
template <int S>
struct Split8Ring {
    unsigned short a[S][SPLIT_TILE_SLOTS * 8];      // 128 rows
    unsigned short b[S][SPLIT_TILE_SLOTS / 2 * 8];  // 64 rows
};

// sum_L acc_L[r] 2^(-7L) for one element.  Levels 1-2 and 3-4 are first paired in
// INT32, u = acc_L 2^7 + acc_(L+1): |u| <= 2^20 (128(L+1) + L + 2) < 2^30, exact, so
// three conversions and two FMAs (exact for S <= 5) replace five and four.
template <int S>
__device__ inline double fold_levels(const ix16 (&acc)[S], int r) {
    constexpr double h7 = 1.0 / 128.0, h14 = 1.0 / 16384.0;
    if constexpr (S == 2) return fma((double)acc[1][r], h7, (double)acc[0][r]);
    const int u12 = acc[1][r] * 128 + acc[2][r];
    if constexpr (S == 3) return fma((double)u12, h14, (double)acc[0][r]);
    double t;
    if constexpr (S == 4) {
        t = fma((double)acc[3][r], h7, (double)u12);
    } else {
        const int u34 = acc[3][r] * 128 + acc[4][r];
        if constexpr (S == 5) t = fma((double)u34, h14, (double)u12);
        else t = fma(fma((double)acc[5][r], h7, (double)u34), h14, (double)u12);
    }
    return fma(t, h14, (double)acc[0][r]);
}

template <int S, class Epi, int STAGE>
__global__ __launch_bounds__(SPLIT8_THREADS) void gemm_i8_kernel(SplitShape sh, Epi epi) {
    __shared__ __attribute__((aligned(16))) Split8Ring<S> ring0, ring1, ring2;
    __shared__ __attribute__((aligned(16))) int lexp[2][2][SPLIT8_BM];  // [chunk parity][A=0/B=1][row]

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave >> 1, wn = wave & 1;
    TileMap tmap{(sh.M + SPLIT8_BM - 1) / SPLIT8_BM, (sh.N + SPLIT8_BN - 1) / SPLIT8_BN};
    const int64_t T = tmap.tiles_m * tmap.tiles_n;
    const int64_t ksplit = sh.ksplit;
    const int64_t split = (int64_t)blockIdx.x / T;
    int64_t ti, tj;
    map_tile((int64_t)blockIdx.x - split * T, T, tmap, ti, tj, SPLIT8_GROUP_M);
    const int64_t m0 = ti * SPLIT8_BM, n0 = tj * SPLIT8_BN;
    const int64_t Kp = split8_kpad(sh.K);
    constexpr int STEPS_PER_CHUNK = SPLIT_KC / SPLIT8_BK;
    int64_t c0, c1;
    split_chunk_range(split_nchunk(sh.K), ksplit, split, c0, c1);
    const int64_t kbeg = c0 * STEPS_PER_CHUNK;
    const int64_t kend = (c1 * STEPS_PER_CHUNK < Kp / SPLIT8_BK) ? c1 * STEPS_PER_CHUNK : Kp / SPLIT8_BK;

    // DMA roles: wave w < 4 loads A rows 32w .. +32 (slots 64w .. +64), waves 4 and 5
    // load B rows 32(w-4) .. +32; lane i fills slot 64 dq + i.
    const int dop = wave >> 2, dq = wave & 3;
    const bool loads = dop == 0 || dq < 2;
    const SplitOperand& op = dop ? sh.b : sh.a;
    const int64_t row0 = dop ? n0 : m0;
    const int64_t last = (dop ? sh.N : sh.M) - 1 - row0;  // last valid row of this tile, >= 0
    const int slot = 64 * dq + lane;
    const int drow = slot >> 1;
    const int dhalf = (slot & 1) ^ (((drow >> 2) ^ (drow >> 3)) & 1);
    const char* sbase = (const char*)op.s;
    const int64_t abs0 = op.row_off + row0;
    const int64_t pbase = abs0 / SPLIT_PANEL;
    const int64_t arow = abs0 + (drow < last ? drow : last);
    const unsigned dvoff = (unsigned)(((arow / SPLIT_PANEL) - pbase) * op.nkb * (SPLIT_PANEL * 32) +
                                      (arow % SPLIT_PANEL) * 32 + 16 * dhalf);
    const char* dbase = (const char*)uniform_ptr(sbase + pbase * op.nkb * (SPLIT_PANEL * 32));
    constexpr int64_t dkstride = SPLIT_PANEL * 32;
    const int64_t dstride = op.slice_stride;
    const int64_t e_ld = op.e_ld;
    // exponents: waves 0, 1 (A rows 64 dq .. +64) and 4 (B rows 0 .. 63)
    const bool eloads = dop == 0 ? dq < 2 : dq == 0;
    const int erow = 64 * dq + lane;
    const unsigned evoff = (unsigned)((erow < last ? erow : last) * 4);
    const int* ebase = (const int*)uniform_ptr(op.e + row0);

    auto dma = [&](Split8Ring<S>& rg, int64_t kt) {
        if (loads) {
#pragma unroll
            for (int p = 0; p < S; ++p) {
                unsigned short* dst = dop ? &rg.b[p][64 * dq * 8] : &rg.a[p][64 * dq * 8];
                lds_dma16(uniform_ptr(dbase + p * dstride + kt * dkstride), dvoff, lds_addr(dst));
            }
        }
        if (eloads && kt % STEPS_PER_CHUNK == 0) {
            const int64_t ch = kt / STEPS_PER_CHUNK;
            lds_dma4(uniform_ptr(ebase + ch * e_ld), evoff, lds_addr(&lexp[ch & 1][dop][64 * dq]));
        }
    };

    ix16 acc[S];
    double acc64[16];
#pragma unroll
    for (int l = 0; l < S; ++l) acc[l] = ix16{};
#pragma unroll
    for (int r = 0; r < 16; ++r) acc64[r] = 0.0;

    const int fr = lane & 31, fh = lane >> 5;
    const int a_off = split_slot(wm * 32 + fr, fh) * 8;
    const int b_off = split_slot(wn * 32 + fr, fh) * 8;

    auto step = [&](Split8Ring<S>& cur, Split8Ring<S>& nxt, int64_t kt) {
        if (kt + 1 < kend)  // this wave's step-kt loads are done once at most S (step kt+1) remain
            __builtin_amdgcn_s_waitcnt((S & 0xF) | ((S >> 4) << 14) | (0x7 << 4) | (0xF << 8));
        else
            __builtin_amdgcn_s_waitcnt((0x7 << 4) | (0xF << 8));
        __builtin_amdgcn_s_barrier();  // every wave's step-kt loads landed; step kt-1 reads are finished
        if (kt + 2 < kend) dma(nxt, kt + 2);

        ix4 af[S], bf[S];
#pragma unroll
        for (int q = 0; q < S; ++q) {
            af[q] = *(const ix4*)(&cur.a[q][a_off]);
            bf[q] = *(const ix4*)(&cur.b[q][b_off]);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int p = 0; p < S; ++p)
#pragma unroll
            for (int q = 0; q < S - p; ++q)
                acc[p + q] = __builtin_amdgcn_mfma_i32_32x32x32_i8(af[p], bf[q], acc[p + q], 0, 0, 0);

        if (((kt + 1) % STEPS_PER_CHUNK) == 0 || kt + 1 == kend) {  // fold the exact level sums into FP64
            const int par = (int)((kt / STEPS_PER_CHUNK) & 1);
            const int eb = lexp[par][1][wn * 32 + (lane & 31)] - 12;
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4) {
                const int4 ea4 = *(const int4*)(&lexp[par][0][wm * 32 + 8 * r4 + 4 * (lane >> 5)]);
                const int ea[4] = {ea4.x, ea4.y, ea4.z, ea4.w};
#pragma unroll
                for (int r1 = 0; r1 < 4; ++r1) {
                    const int r = 4 * r4 + r1;
                    acc64[r] += ldexp(fold_levels<S>(acc, r), ea[r1] + eb);
                }
            }
#pragma unroll
            for (int l = 0; l < S; ++l) acc[l] = ix16{};
        }
    };

    if (kbeg < kend) {
        dma(ring0, kbeg);
        if (kbeg + 1 < kend) dma(ring1, kbeg + 1);
        for (int64_t kt = kbeg; kt < kend; kt += 3) {
            step(ring0, ring2, kt);
            if (kt + 1 < kend) step(ring1, ring0, kt + 1);
            if (kt + 2 < kend) step(ring2, ring1, kt + 2);
        }
    }

    // D layout of the 32x32 MFMA: lane l, element r holds row 8*(r/4) + 4*(l/32) + r%4, column l%32.
    if (ksplit > 1) {
        double* part = sh.part + split * sh.M * sh.N;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int64_t m = m0 + wm * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
            const int64_t n = n0 + wn * 32 + (lane & 31);
            if (m < sh.M && n < sh.N) part[m * sh.N + n] = acc64[r];
        }
        return;
    }
    typename Epi::Local loc = epi.begin();
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int64_t m = m0 + wm * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int64_t n = n0 + wn * 32 + (lane & 31);
        if (m < sh.M && n < sh.N) epi.put(loc, m, n, acc64[r]);
    }
    epi.finish(loc, blockIdx.x);
}

}  // namespace ladder
