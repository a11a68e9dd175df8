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
// Slice layout ("panel-major, k-blocked"): the rows of an operand are grouped in
// panels of 128; slice p stores, panel after panel, the Kp/16 k-blocks of the
// panel as [128 rows][16 k] BF16 (Kp = split_kpad(K), zero beyond K):
//   element (r, k) of slice p at  p*slice_stride + ((r/128)*nkb + k/16)*2048 + (r%128)*16 + k%16,
// nkb = Kp/16, slice_stride = panels*128*Kp (rows padded to whole panels).  One
// GEMM K-step (16 k) of a 128-row tile is then a contiguous 4 KB run (two runs
// when the tile straddles a panel boundary), and a tile's walk over K stays
// inside one or two contiguous panels, which keeps address translation local.
// Exponents: [nchunk][R] (chunk stride exp_ld).
constexpr int SPLIT_PANEL = 128;
__host__ __device__ inline int64_t split_panels(int64_t R) { return (R + SPLIT_PANEL - 1) / SPLIT_PANEL; }
__host__ __device__ inline int64_t split_slice_stride(int64_t R, int64_t K) { return split_panels(R) * SPLIT_PANEL * split_kpad(K); }
__host__ __device__ inline int64_t split_index(int64_t r, int64_t k, int64_t nkb) {
    return ((r >> 7) * nkb + (k >> 4)) * (SPLIT_PANEL * 16) + (r & 127) * 16 + (k & 15);
}

// Row-wise source: element (r, k) = src(r, k), r < R, k < K (DenseRows: src[r*ld + k];
// the +/- path also slices its density tiles straight from their packed rows).
// One workgroup per 16 rows and one chunk: thread (rr, kk) = (t/16, t%16) holds
// k = chunk*256 + 16*kb + kk for kb < 16, so each k-block of the 16 rows is written
// as one 512-byte run per slice.
struct DenseRows {
    const double* p;
    int64_t ld;
    __device__ double operator()(int64_t r, int64_t k) const { return p[r * ld + k]; }
};

template <int S, class Src>
__global__ __launch_bounds__(256) void slice_rows_kernel(Src src, int64_t R, int64_t K,
                                                         unsigned short* __restrict__ slices,
                                                         int* __restrict__ exps, int64_t exp_ld) {
    constexpr int RB = 16, NKB = SPLIT_KC / 16;
    const int64_t nch = split_nchunk(K), Kp = split_kpad(K);
    const int64_t rblocks = (R + RB - 1) / RB;
    const int64_t rb = blockIdx.x % rblocks, ch = blockIdx.x / rblocks;
    const int rr = threadIdx.x >> 4, kk = threadIdx.x & 15;
    const int64_t r = rb * RB + rr;
    if (ch >= nch) return;  // uniform per block
    double x[NKB];
    double mx = 0.0;
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb) {
        const int64_t k = ch * SPLIT_KC + 16 * kb + kk;
        x[kb] = (r < R && k < K) ? src(r, k) : 0.0;
        mx = fmax(mx, fabs(x[kb]));
    }
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));  // the 16 lanes of row rr
    if (r >= R) return;
    const int e = chunk_exponent(mx);
    if (kk == 0) exps[ch * exp_ld + r] = e;
    const int64_t slice_stride = split_slice_stride(R, K), nkb = Kp / 16;
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb) {
        const int64_t k = ch * SPLIT_KC + 16 * kb + kk;
        if (k < Kp) write_slices<S>(x[kb], e, slices + split_index(r, k, nkb), slice_stride);
    }
}

// Transposed source: element (r, k) at src[k*ld + r].  One workgroup per 32 rows
// and one chunk, staged through LDS so that both the reads (along r) and the
// k-blocked slice writes are contiguous.
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
    if (part == 0 && r0 + rr < R) exps[ch * exp_ld + r0 + rr] = ex[rr];
    // writes: thread (wr, kk) = (t/16, t%16) covers rows wr and wr + 16 of every
    // k-block, so a block's 32 rows x 16 k go out as one 1 KB run per slice
    const int64_t slice_stride = split_slice_stride(R, K), nkb = Kp / 16;
    const int wr = tid >> 4, kk = tid & 15;
    for (int kb = 0; kb < SPLIT_KC / 16; ++kb) {
        const int64_t k = k0 + 16 * kb + kk;
        if (k >= Kp) break;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int row = wr + 16 * h;
            const int64_t r = r0 + row;
            if (r < R) write_slices<S>(tile[16 * kb + kk][row], ex[row], slices + split_index(r, k, nkb), slice_stride);
        }
    }
}

// ---------------------------------------------------------------- split GEMM
struct SplitOperand {
    const unsigned short* s;  // slice 0 of the whole sliced buffer (panel-major layout)
    int64_t slice_stride;     // elements between slices (split_slice_stride of the buffer)
    int64_t row_off;          // first buffer row of this view
    int64_t nkb;              // k-blocks per panel, Kp / 16
    const int* e;             // exponent of (row 0, chunk 0) of this view
    int64_t e_ld;             // chunk stride of the exponent array
    bool i8 = false;          // INT8 slices (split_i8.hpp): s holds bytes, strides in bytes, nkb = Kp / 32
};

struct SplitShape {
    SplitOperand a, b;
    int64_t M, N, K;      // K = real length (chunks and padding follow from it)
    int64_t ksplit = 1;   // > 1: the chunks are dealt to ksplit workgroups per tile, each of
    double* part = nullptr;  // which stores its raw FP64 sum at part[split][M][N]
};

// Chunks [c0, c1) of split s out of ksplit (contiguous, as even as possible).
__host__ __device__ inline void split_chunk_range(int64_t nch, int64_t ksplit, int64_t s, int64_t& c0, int64_t& c1) {
    c0 = nch * s / ksplit;
    c1 = nch * (s + 1) / ksplit;
}

// 512 threads = 8 waves in a 4 x 2 grid; wave (wm, wn) owns rows wm*32 .. +32 and
// columns wn*64 .. +64 of the 128 x 128 tile (two 32x32 MFMA blocks), so two
// waves share each SIMD and one's MFMAs overlap the other's FP64 combine.
//
// Operand tiles go from global memory straight into LDS (global_load_lds_dwordx4,
// no VGPR staging) through a 3-deep ring of K-steps, so two K-steps of loads are
// in flight while the third is multiplied.  An LDS slice tile is 128 rows x 16 k
// of BF16 = 256 slots of 16 bytes; row r, k-half h lives in slot
// 2r + (h ^ f(r)) with f(r) = bit2(r) ^ bit3(r), which keeps both the DMA writes
// (one 1 KB run per wave instruction) and the MFMA fragment reads (8 or 16
// consecutive rows per LDS cycle) free of bank conflicts.
constexpr int SPLIT_STAGES = 3;
constexpr int SPLIT_TILE_SLOTS = 256;  // 16-byte slots per slice tile (4 KB)

__device__ inline int split_slot(int r, int h) { return 2 * r + (h ^ (((r >> 2) ^ (r >> 3)) & 1)); }

typedef __attribute__((address_space(3))) void* lds_ptr_t;

// Global memory -> LDS without VGPR staging (global_load_lds): lane i's bytes
// land at lds_base + size*i; the global address is the wave-uniform `base`
// (SGPRs) plus the lane's 32-bit byte offset.  Written as inline assembly on
// purpose: the compiler treats its own LDS-DMA builtin as aliasing every later
// LDS read and would wait for the just-issued loads before each fragment read,
// which serialises the ring.  Ordering is explicit instead: a buffer is read
// only after s_waitcnt vmcnt and s_barrier, and the statement clobbers memory
// so that no LDS access moves across it.  It has no register outputs.  The LDS
// address goes in through an M0 operand constraint, so the compiler itself
// writes M0 (it treats M0 as reserved and would not preserve a value of its own
// across a statement that wrote it); the s_nop is the wait state between that
// write and the LDS DMA that reads it.
__device__ inline void lds_dma16(const void* base, unsigned voff, unsigned lds_base) {
    asm volatile("s_nop 0\n\tglobal_load_lds_dwordx4 %0, %1" ::"v"(voff), "s"(base), "{m0}"(lds_base) : "memory");
}
__device__ inline void lds_dma4(const void* base, unsigned voff, unsigned lds_base) {
    asm volatile("s_nop 0\n\tglobal_load_lds_dword %0, %1" ::"v"(voff), "s"(base), "{m0}"(lds_base) : "memory");
}
__device__ inline const void* uniform_ptr(const void* p) {
    const uint64_t x = (uint64_t)(uintptr_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
    return (const void*)(uintptr_t)(((uint64_t)hi << 32) | lo);
}
__device__ inline unsigned lds_addr(const void* p) {
    return __builtin_amdgcn_readfirstlane((unsigned)(uintptr_t)(lds_ptr_t)p);
}

// The three ring buffers are distinct LDS variables and the K loop is unrolled
// by three, so every access names its buffer statically; the compiler can then
// tell the in-flight DMA of one buffer from the fragment reads of another and
// waits only where a buffer is reused.
template <int S>
struct SplitRing {
    unsigned short t[2][S][SPLIT_TILE_SLOTS * 8];  // [operand A=0/B=1][slice][slots]
};

// STAGE only names the instantiation (one kernel symbol per stage in profiles).
template <int S, class Epi, int STAGE>
__global__ __launch_bounds__(SPLIT_THREADS) void gemm_split_kernel(SplitShape sh, Epi epi) {
    __shared__ __attribute__((aligned(16))) SplitRing<S> ring0, ring1, ring2;
    // chunk exponents, double-buffered by chunk parity: [parity][A=0/B=1][128 rows]
    __shared__ __attribute__((aligned(16))) int lexp[2][2][SPLIT_BM];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform: keeps the roles in SGPRs
    const int wm = wave >> 1, wn = wave & 1;
    TileMap tmap{(sh.M + SPLIT_BM - 1) / SPLIT_BM, (sh.N + SPLIT_BN - 1) / SPLIT_BN};
    const int64_t T = tmap.tiles_m * tmap.tiles_n;
    const int64_t ksplit = sh.ksplit;
    const int64_t split = (int64_t)blockIdx.x / T;  // grid = T * ksplit; one split's tiles are consecutive
    int64_t ti, tj;
    map_tile((int64_t)blockIdx.x - split * T, T, tmap, ti, tj);
    const int64_t m0 = ti * SPLIT_BM, n0 = tj * SPLIT_BN;
    const int64_t Kp = split_kpad(sh.K);
    constexpr int STEPS_PER_CHUNK = SPLIT_KC / SPLIT_BK;
    // K-steps [kbeg, kend) of this workgroup: whole chunks, so chunk parity and exponents are unchanged
    int64_t c0, c1;
    split_chunk_range(split_nchunk(sh.K), ksplit, split, c0, c1);
    const int64_t kbeg = c0 * STEPS_PER_CHUNK;
    const int64_t kend = (c1 * STEPS_PER_CHUNK < Kp / SPLIT_BK) ? c1 * STEPS_PER_CHUNK : Kp / SPLIT_BK;

    // DMA role: waves 0-3 load A, 4-7 load B; wave w%4 covers slots 64*(w%4) .. +64
    // (rows 32*(w%4) .. +32) of every slice.  Lane i fills slot 64*(w%4) + i.
    // Waves with w%4 < 2 also load the chunk exponents of rows 64*(w%4) .. +64.
    const int dop = wave >> 2, dq = wave & 3;
    const SplitOperand& op = dop ? sh.b : sh.a;
    const int64_t row0 = dop ? n0 : m0;
    const int64_t last = (dop ? sh.N : sh.M) - 1 - row0;  // last valid row of this tile, >= 0
    const int slot = 64 * dq + lane;
    const int drow = slot >> 1;
    const int dhalf = (slot & 1) ^ (((drow >> 2) ^ (drow >> 3)) & 1);
    // rows past the edge load a valid row; their results are never stored.  The
    // tile's rows lie in panel pbase or pbase + 1 of the buffer.
    const int64_t abs0 = op.row_off + row0;
    const int64_t pbase = abs0 / SPLIT_PANEL;
    const int64_t arow = abs0 + (drow < last ? drow : last);
    const unsigned dvoff = (unsigned)((((arow / SPLIT_PANEL) - pbase) * op.nkb * (SPLIT_PANEL * 16) +
                                       (arow % SPLIT_PANEL) * 16 + 8 * dhalf) * 2);
    const unsigned short* dbase = (const unsigned short*)uniform_ptr(op.s + pbase * op.nkb * (SPLIT_PANEL * 16));
    constexpr int64_t dkstride = SPLIT_PANEL * 16;
    const int64_t dstride = op.slice_stride;
    const int64_t e_ld = op.e_ld;
    const int erow = 64 * dq + lane;
    const unsigned evoff = (unsigned)((erow < last ? erow : last) * 4);
    const int* ebase = (const int*)uniform_ptr(op.e + row0);

    auto dma = [&](SplitRing<S>& rg, int64_t kt) {
#pragma unroll
        for (int p = 0; p < S; ++p)
            lds_dma16(uniform_ptr(dbase + p * dstride + kt * dkstride), dvoff, lds_addr(&rg.t[dop][p][64 * dq * 8]));
        if (dq < 2 && kt % STEPS_PER_CHUNK == 0) {
            const int64_t ch = kt / STEPS_PER_CHUNK;
            lds_dma4(uniform_ptr(ebase + ch * e_ld), evoff, lds_addr(&lexp[ch & 1][dop][64 * dq]));
        }
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

    // Fragment reads: row (block base + l%32), k-half l/32.
    const int fr = lane & 31, fh = lane >> 5;
    const int a_off = split_slot(wm * 32 + fr, fh) * 8;
    const int b_off0 = split_slot(wn * 64 + fr, fh) * 8;
    const int b_off1 = split_slot(wn * 64 + 32 + fr, fh) * 8;

    // One K-step on ring buffer `cur`, while step kt+2 is loaded into `nxt`.
    auto step = [&](SplitRing<S>& cur, SplitRing<S>& nxt, int64_t kt) {
        if (kt + 1 < kend)  // this wave's step-kt loads are done once at most S (step kt+1) remain
            __builtin_amdgcn_s_waitcnt((S & 0xF) | ((S >> 4) << 14) | (0x7 << 4) | (0xF << 8));
        else
            __builtin_amdgcn_s_waitcnt((0x7 << 4) | (0xF << 8));
        __builtin_amdgcn_s_barrier();  // every wave's step-kt loads landed; step kt-1 reads are finished
        if (kt + 2 < kend) dma(nxt, kt + 2);

        // every fragment of the step is read before the first MFMA, so no LDS wait sits
        // between MFMAs (S A-fragments and 2S B-fragments, 12 S registers)
        bx8 bq[S][2], ap[S];
#pragma unroll
        for (int q = 0; q < S; ++q) {
            bq[q][0] = __builtin_bit_cast(bx8, *(const ux8*)(&cur.t[1][q][b_off0]));
            bq[q][1] = __builtin_bit_cast(bx8, *(const ux8*)(&cur.t[1][q][b_off1]));
            ap[q] = __builtin_bit_cast(bx8, *(const ux8*)(&cur.t[0][q][a_off]));
        }
        __builtin_amdgcn_sched_barrier(0);  // keep the scheduler from sinking reads between the MFMAs
#pragma unroll
        for (int p = 0; p < S; ++p) {
#pragma unroll
            for (int q = 0; q < S - p; ++q) {
                const int g = (p + q) < 2 ? (p + q) : 2;
#pragma unroll
                for (int bj = 0; bj < 2; ++bj)
                    acc[g][bj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ap[p], bq[q][bj], acc[g][bj], 0, 0, 0);
            }
        }

        if (((kt + 1) % STEPS_PER_CHUNK) == 0 || kt + 1 == kend) {  // fold the exact FP32 chunk sums into FP64
            const int par = (int)((kt / STEPS_PER_CHUNK) & 1);
            const int eb0 = lexp[par][1][wn * 64 + (lane & 31)];
            const int eb1 = lexp[par][1][wn * 64 + 32 + (lane & 31)];
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4) {
                const int4 ea4 = *(const int4*)(&lexp[par][0][wm * 32 + 8 * r4 + 4 * (lane >> 5)]);
                const int ea[4] = {ea4.x, ea4.y, ea4.z, ea4.w};
#pragma unroll
                for (int r1 = 0; r1 < 4; ++r1) {
                    const int r = 4 * r4 + r1;
                    const double t0 = ((double)acc[0][0][r] + (double)acc[1][0][r]) + (double)acc[2][0][r];
                    const double t1 = ((double)acc[0][1][r] + (double)acc[1][1][r]) + (double)acc[2][1][r];
                    acc64[0][r] += ldexp(t0, ea[r1] + eb0);
                    acc64[1][r] += ldexp(t1, ea[r1] + eb1);
                }
            }
#pragma unroll
            for (int g = 0; g < 3; ++g)
#pragma unroll
                for (int bj = 0; bj < 2; ++bj) acc[g][bj] = fx16{};
        }
    };

    if (kbeg < kend) {  // uniform per workgroup; a split may own no chunk only when ksplit > chunks
        dma(ring0, kbeg);
        if (kbeg + 1 < kend) dma(ring1, kbeg + 1);
        for (int64_t kt = kbeg; kt < kend; kt += 3) {
            step(ring0, ring2, kt);
            if (kt + 1 < kend) step(ring1, ring0, kt + 1);
            if (kt + 2 < kend) step(ring2, ring1, kt + 2);
        }
    }

    // D layout of v_mfma_f32_32x32x16_bf16 (measured on gfx950): lane l, element r
    // holds row 8*(r/4) + 4*(l/32) + r%4, column l%32.
    if (ksplit > 1) {  // raw partial sums; the reduction kernel applies the epilogue
        double* part = sh.part + split * sh.M * sh.N;
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t m = m0 + wm * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                const int64_t n = n0 + wn * 64 + 32 * bj + (lane & 31);
                if (m < sh.M && n < sh.N) part[m * sh.N + n] = acc64[bj][r];
            }
        return;
    }
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

// Sums the ksplit partial tiles of a split-K GEMM in split order (deterministic)
// and hands every element to the epilogue.  Any grid; needs all threads of a
// block in finish.
template <class Epi>
__global__ __launch_bounds__(256) void splitk_reduce_kernel(const double* __restrict__ part, int64_t M, int64_t N,
                                                            int64_t ksplit, Epi epi) {
    typename Epi::Local loc = epi.begin();
    const int64_t MN = M * N;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < MN; x += (int64_t)gridDim.x * blockDim.x) {
        double s = part[x];
        for (int64_t k = 1; k < ksplit; ++k) s += part[k * MN + x];
        epi.put(loc, x / N, x % N, s);
    }
    epi.finish(loc, blockIdx.x);
}

}  // namespace ladder
