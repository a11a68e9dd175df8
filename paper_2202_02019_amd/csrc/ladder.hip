// ladder.hip -- libladder.so: host side of the C ABI declared in include/ladder.h
// plus the small FP64 kernels (pair swap, energy reduction, amplitude update).
//
// Forward, per virtual batch A = [a0, a0 + nA) (Sec. II B, "albeit with batching"):
//   GEMM-B  g_A[(a,b),(c,d)] = sum_J L[(a,c),J] L[(b,d),J]      M = nA*v, N = v^2, K = n
//           (Cholesky expansion of Sec. II A; the epilogue swaps the middle
//           indices so that (c,d) becomes the contiguous K axis of the next GEMM)
//   GEMM-C  R[(ij),(a,b)] = beta R + sum_(cd) tau[(ij),(cd)] g_A[(a,b),(cd)]
//           M = o^2, N = nA*v, K = v^2; the epilogue folds tbar*R into one energy
//           partial per workgroup; a last kernel sums the partials in a fixed order.
// Adjoint, per batch:
//   GEMM-E  D_A[(a,c),(b,d)] = sum_ij w[(ij),(a,b)] tau[(ij),(c,d)]   M = nA*v, N = v^2, K = o^2
//           (the V^4 density O^(2) of Sec. II B as a batch tile only)
//   GEMM-F  X[(a,c),J] = beta X + 2 alpha sum_(bd) D_A[(a,c),(bd)] L[(bd),J]  M = nA*v, N = n, K = v^2
//           (2 W~ of Sec. II C; the factor 2 is d_pqrs = d_rspq, Appendix A)
#include <hip/hip_runtime.h>

#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ladder.h"
#include "gemm_f64.hpp"

using namespace ladder;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_check(hipError_t e, const char* what) {
    if (e == hipSuccess) return LADDER_OK;
    return fail(LADDER_EHIP, "%s: %s", what, hipGetErrorString(e));
}

constexpr int64_t MAX_DIM = int64_t(1) << 20;

// ------------------------------------------------------------ stage timing
struct StageRec {
    int stage;
    hipEvent_t a, b;
    double flops, bytes;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<StageRec> g_prof;

// Brackets one launch with events on its stream when profiling is on.
struct StageTimer {
    StageRec rec{};
    bool on = false;
    hipStream_t st;
    StageTimer(int stage, double flops, double bytes, hipStream_t s) : st(s) {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        if (!g_prof_on) return;
        rec.stage = stage;
        rec.flops = flops;
        rec.bytes = bytes;
        if (hipEventCreate(&rec.a) != hipSuccess || hipEventCreate(&rec.b) != hipSuccess) return;
        on = hipEventRecord(rec.a, st) == hipSuccess;
    }
    ~StageTimer() {
        if (!on) return;
        (void)hipEventRecord(rec.b, st);
        std::lock_guard<std::mutex> lk(g_prof_mu);
        g_prof.push_back(rec);
    }
};

double gemm_bytes(int64_t M, int64_t N, int64_t K) { return 8.0 * ((double)M * K + (double)K * N + (double)M * N); }
double gemm_flops(int64_t M, int64_t N, int64_t K) { return 2.0 * (double)M * (double)N * (double)K; }

bool mul_ok(int64_t a, int64_t b, int64_t& out) {
    if (a < 0 || b < 0) return false;
    if (a != 0 && b > INT64_MAX / a) return false;
    out = a * b;
    return true;
}

struct Sizes {
    int64_t oo, vv, ovv_elems /* o^2 v^2 */, vvn /* v^2 n */, vvv /* v^3 */;
};

int check_dims(int64_t o, int64_t v, int64_t n, Sizes& s) {
    if (o < 1 || v < 1 || n < 1) return fail(LADDER_EINVAL, "dimensions must be >= 1 (o=%lld v=%lld n=%lld)", (long long)o, (long long)v, (long long)n);
    if (o > MAX_DIM || v > MAX_DIM || n > MAX_DIM) return fail(LADDER_EINVAL, "dimension above 2^20");
    if (!mul_ok(o, o, s.oo) || !mul_ok(v, v, s.vv) || !mul_ok(s.oo, s.vv, s.ovv_elems) || !mul_ok(s.vv, n, s.vvn) ||
        !mul_ok(s.vv, v, s.vvv) || s.ovv_elems > INT64_MAX / 8 || s.vvn > INT64_MAX / 8)
        return fail(LADDER_EINVAL, "array sizes overflow 64-bit byte counts");
    return LADDER_OK;
}

bool aligned8(const void* p) { return ((uintptr_t)p & 7u) == 0; }

bool overlap(const void* a, int64_t abytes, const void* b, int64_t bbytes) {
    if (!a || !b) return false;
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + (uintptr_t)bbytes && y < x + (uintptr_t)abytes;
}

int get_opts(const ladder_options* in, ladder_options& o) {
    ladder_default_options(&o);
    if (in) o = *in;
    if (o.precision != LADDER_FP64 && o.precision != LADDER_SPLIT_BF16)
        return fail(LADDER_EUNSUPPORTED, "unknown precision %d", (int)o.precision);
    if (o.precision == LADDER_SPLIT_BF16)
        return fail(LADDER_EUNSUPPORTED, "split-BF16 precision is not built into this library yet");
    if (o.n_abatch < 0) return fail(LADDER_EINVAL, "n_abatch must be >= 0");
    if (o.flags & ~LADDER_FLAG_GENERAL) return fail(LADDER_EUNSUPPORTED, "unknown flag bits 0x%x", o.flags);
    if (o.reserved != 0) return fail(LADDER_EINVAL, "reserved option field must be 0");
    return LADDER_OK;
}

constexpr size_t ALIGN = 256;
size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

int64_t tiles(int64_t M, int64_t N) { return ((M + F64_BM - 1) / F64_BM) * ((N + F64_BN - 1) / F64_BN); }

// Batch plan and workspace layout shared by forward and adjoint.
struct Plan {
    int64_t nA, nbatch;
    size_t tile_off, tile_bytes;      // g_A or D_A
    size_t part_off, part_per_batch;  // energy partials (doubles per batch)
    size_t swap_off, swap_bytes;      // pair-swapped w and tau (general adjoint)
    size_t total;
};

Plan make_plan(int64_t o, int64_t v, int64_t n, const ladder_options& op, const Sizes& s) {
    (void)n;
    Plan p{};
    int64_t nA = op.n_abatch;
    if (nA == 0) {
        const int64_t per_a = s.vvv * 8;
        nA = (int64_t)(LADDER_DEFAULT_TILE_BYTES / (size_t)per_a);
        // at least two batches, so the whole v^4 array is never held at once
        nA = std::min(nA, (v + 1) / 2);
        if (nA < 1) nA = 1;
    }
    if (nA > v) nA = v;
    p.nA = nA;
    p.nbatch = (v + nA - 1) / nA;
    p.tile_off = 0;
    p.tile_bytes = align_up((size_t)(nA * s.vvv) * 8);
    p.part_off = p.tile_bytes;
    p.part_per_batch = (size_t)tiles(s.oo, nA * v);
    const size_t part_bytes = align_up(p.part_per_batch * (size_t)p.nbatch * 8);
    p.swap_off = p.part_off + part_bytes;
    p.swap_bytes = (op.flags & LADDER_FLAG_GENERAL) ? align_up((size_t)s.ovv_elems * 8) * 2 : 0;
    p.total = p.swap_off + p.swap_bytes;
    (void)o;
    return p;
}

template <bool AK, bool BK, class Epi>
hipError_t launch_gemm(const double* A, int64_t lda, const double* B, int64_t ldb, int64_t M, int64_t N, int64_t K,
                       const Epi& epi, hipStream_t st) {
    GemmShape sh{A, lda, B, ldb, M, N, K};
    const int64_t T = tiles(M, N);
    hipLaunchKernelGGL((gemm_f64_kernel<AK, BK, Epi>), dim3((unsigned)T), dim3(F64_THREADS), 0, st, sh, epi);
    return hipGetLastError();
}

// out_ij^ab = in_ji^ba
__global__ void pair_swap_kernel(const double* __restrict__ in, double* __restrict__ out, int64_t o, int64_t v) {
    const int64_t total = o * o * v * v;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = x % v, a = (x / v) % v, ij = x / (v * v);
        const int64_t j = ij % o, i = ij / o;
        out[x] = in[((j * o + i) * v + b) * v + a];
    }
}

// *E = sum of partials, one block, fixed order: deterministic.
__global__ void reduce_partials_kernel(const double* __restrict__ part, int64_t count, double* __restrict__ E) {
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < count; i += 256) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *E = red[0];
}

__global__ void amplitude_update_kernel(const double* __restrict__ eps, const double* R, double* t, int64_t o, int64_t v) {
    const int64_t total = o * o * v * v;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = x % v, a = (x / v) % v, ij = x / (v * v);
        const int64_t j = ij % o, i = ij / o;
        const double den = (eps[i] + eps[j]) - (eps[o + a] + eps[o + b]);
        t[x] = t[x] + R[x] / den;
    }
}

unsigned grid_for(int64_t total) {
    int64_t g = (total + 255) / 256;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (unsigned)g;
}

}  // namespace

extern "C" {

void ladder_default_options(ladder_options* o) {
    if (!o) return;
    memset(o, 0, sizeof *o);
    o->precision = LADDER_FP64;
}

const char* ladder_strerror(int code) {
    switch (code) {
        case LADDER_OK: return "success";
        case LADDER_EINVAL: return "invalid argument";
        case LADDER_EWORKSPACE: return "workspace too small";
        case LADDER_EUNSUPPORTED: return "unsupported option";
        case LADDER_EHIP: return "HIP runtime error";
        default: return "unknown error code";
    }
}

const char* ladder_last_error(void) { return g_last_error.c_str(); }

int ladder_workspace_size(int64_t o, int64_t v, int64_t n, const ladder_options* opts, size_t* bytes) {
    g_last_error.clear();
    if (!bytes) return fail(LADDER_EINVAL, "bytes is NULL");
    Sizes s;
    ladder_options op;
    int rc;
    if ((rc = check_dims(o, v, n, s)) || (rc = get_opts(opts, op))) return rc;
    *bytes = make_plan(o, v, n, op, s).total;
    return LADDER_OK;
}

int ladder_forward(int64_t o, int64_t v, int64_t n, const double* L, const double* tau, const double* tbar,
                   double beta, double* R, double* E, void* ws, size_t ws_bytes, const ladder_options* opts,
                   void* stream) {
    g_last_error.clear();
    Sizes s;
    ladder_options op;
    int rc;
    if ((rc = check_dims(o, v, n, s)) || (rc = get_opts(opts, op))) return rc;
    if (!L || !tau || !R || !ws) return fail(LADDER_EINVAL, "L, tau, R and ws must be non-NULL");
    if (E && !tbar) return fail(LADDER_EINVAL, "E requested but tbar is NULL");
    if (!aligned8(L) || !aligned8(tau) || !aligned8(R) || (tbar && !aligned8(tbar)) || (E && !aligned8(E)) ||
        ((uintptr_t)ws % ALIGN))
        return fail(LADDER_EINVAL, "misaligned pointer (arrays need 8-byte, ws 256-byte alignment)");
    const Plan p = make_plan(o, v, n, op, s);
    if (ws_bytes < p.total) return fail(LADDER_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, p.total);
    const int64_t tb = s.ovv_elems * 8, lb = s.vvn * 8;
    if (overlap(R, tb, L, lb) || overlap(R, tb, tau, tb) || overlap(R, tb, tbar, tb) || overlap(R, tb, ws, (int64_t)ws_bytes))
        return fail(LADDER_EINVAL, "R overlaps an input or the workspace");
    if (E && (overlap(E, 8, R, tb) || overlap(E, 8, ws, (int64_t)ws_bytes)))
        return fail(LADDER_EINVAL, "E overlaps R or the workspace");

    hipStream_t st = (hipStream_t)stream;
    char* w = (char*)ws;
    double* g = (double*)(w + p.tile_off);
    double* part = (double*)(w + p.part_off);
    for (int64_t bi = 0; bi < p.nbatch; ++bi) {
        const int64_t a0 = bi * p.nA;
        const int64_t nA = std::min(p.nA, v - a0);
        {
            StageTimer tm(LADDER_STAGE_GEMM_B, gemm_flops(nA * v, s.vv, n), gemm_bytes(nA * v, s.vv, n), st);
            EpiSwapMid eg{g, v, v, v, 1.0, 0.0};
            if ((rc = hip_check(launch_gemm<true, true>(L + a0 * v * n, n, L, n, nA * v, s.vv, n, eg, st), "GEMM-B launch")))
                return rc;
        }
        {
            StageTimer tm(LADDER_STAGE_GEMM_C, gemm_flops(s.oo, nA * v, s.vv) + (E ? 2.0 * s.oo * nA * v : 0.0),
                          gemm_bytes(s.oo, nA * v, s.vv) + (E ? 8.0 * s.oo * nA * v : 0.0), st);
            EpiStrided er{R + a0 * v, s.vv, 1.0, beta, E ? tbar + a0 * v : nullptr, part + bi * p.part_per_batch};
            if ((rc = hip_check(launch_gemm<true, true>(tau, s.vv, g, s.vv, s.oo, nA * v, s.vv, er, st), "GEMM-C launch")))
                return rc;
        }
    }
    if (E) {
        // Batch bi writes partial slots [bi*ppb, bi*ppb + tiles of its GEMM-C); every
        // batch but the last fills all ppb of them, so the slots in use are contiguous.
        const int64_t used_last = tiles(s.oo, (v - (p.nbatch - 1) * p.nA) * v);
        const int64_t count = (int64_t)p.part_per_batch * (p.nbatch - 1) + used_last;
        StageTimer tm(LADDER_STAGE_ENERGY, (double)count, 8.0 * (double)count, st);
        hipLaunchKernelGGL(reduce_partials_kernel, dim3(1), dim3(256), 0, st, part, count, E);
        if ((rc = hip_check(hipGetLastError(), "energy reduction launch"))) return rc;
    }
    return LADDER_OK;
}

int ladder_adjoint(int64_t o, int64_t v, int64_t n, const double* L, const double* tau, const double* wt,
                   double alpha, double beta, double* X, void* ws, size_t ws_bytes, const ladder_options* opts,
                   void* stream) {
    g_last_error.clear();
    Sizes s;
    ladder_options op;
    int rc;
    if ((rc = check_dims(o, v, n, s)) || (rc = get_opts(opts, op))) return rc;
    if (!L || !tau || !wt || !X || !ws) return fail(LADDER_EINVAL, "L, tau, w, X and ws must be non-NULL");
    if (!aligned8(L) || !aligned8(tau) || !aligned8(wt) || !aligned8(X) || ((uintptr_t)ws % ALIGN))
        return fail(LADDER_EINVAL, "misaligned pointer (arrays need 8-byte, ws 256-byte alignment)");
    const Plan p = make_plan(o, v, n, op, s);
    if (ws_bytes < p.total) return fail(LADDER_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, p.total);
    const int64_t tb = s.ovv_elems * 8, lb = s.vvn * 8;
    if (overlap(X, lb, L, lb) || overlap(X, lb, tau, tb) || overlap(X, lb, wt, tb) || overlap(X, lb, ws, (int64_t)ws_bytes))
        return fail(LADDER_EINVAL, "X overlaps an input or the workspace");

    hipStream_t st = (hipStream_t)stream;
    char* w = (char*)ws;
    double* D = (double*)(w + p.tile_off);
    const bool general = (op.flags & LADDER_FLAG_GENERAL) != 0;
    double* pw = general ? (double*)(w + p.swap_off) : nullptr;
    double* pt = general ? (double*)(w + p.swap_off + p.swap_bytes / 2) : nullptr;
    if (general) {
        StageTimer tm(LADDER_STAGE_SWAP, 0.0, 32.0 * (double)s.ovv_elems, st);
        hipLaunchKernelGGL(pair_swap_kernel, dim3(grid_for(s.ovv_elems)), dim3(256), 0, st, wt, pw, o, v);
        hipLaunchKernelGGL(pair_swap_kernel, dim3(grid_for(s.ovv_elems)), dim3(256), 0, st, tau, pt, o, v);
        if ((rc = hip_check(hipGetLastError(), "pair swap launch"))) return rc;
    }
    for (int64_t bi = 0; bi < p.nbatch; ++bi) {
        const int64_t a0 = bi * p.nA;
        const int64_t nA = std::min(p.nA, v - a0);
        {
            StageTimer tm(LADDER_STAGE_GEMM_E, gemm_flops(nA * v, s.vv, s.oo), gemm_bytes(nA * v, s.vv, s.oo), st);
            EpiSwapMid ed{D, v, v, v, 1.0, 0.0};
            if ((rc = hip_check(launch_gemm<false, false>(wt + a0 * v, s.vv, tau, s.vv, nA * v, s.vv, s.oo, ed, st), "GEMM-E launch")))
                return rc;
        }
        if (general) {
            StageTimer tm(LADDER_STAGE_GEMM_E, gemm_flops(nA * v, s.vv, s.oo), gemm_bytes(nA * v, s.vv, s.oo), st);
            EpiSwapMid ed2{D, v, v, v, 1.0, 1.0};
            if ((rc = hip_check(launch_gemm<false, false>(pw + a0 * v, s.vv, pt, s.vv, nA * v, s.vv, s.oo, ed2, st), "GEMM-E launch")))
                return rc;
        }
        {
            StageTimer tm(LADDER_STAGE_GEMM_F, gemm_flops(nA * v, n, s.vv), gemm_bytes(nA * v, n, s.vv), st);
            EpiStrided ex{X + a0 * v * n, n, general ? alpha : 2.0 * alpha, beta, nullptr, nullptr};
            if ((rc = hip_check(launch_gemm<true, false>(D, s.vv, L, n, nA * v, n, s.vv, ex, st), "GEMM-F launch")))
                return rc;
        }
    }
    return LADDER_OK;
}

int ladder_mp2_amplitudes(int64_t o, int64_t v, int64_t n, const double* Lov, const double* eps, double* t,
                          void* stream) {
    g_last_error.clear();
    Sizes s;
    int rc;
    if ((rc = check_dims(o, v, n, s))) return rc;
    if (!Lov || !eps || !t) return fail(LADDER_EINVAL, "Lov, eps and t must be non-NULL");
    if (!aligned8(Lov) || !aligned8(eps) || !aligned8(t)) return fail(LADDER_EINVAL, "misaligned pointer");
    if (overlap(t, s.ovv_elems * 8, Lov, o * v * n * 8) || overlap(t, s.ovv_elems * 8, eps, (o + v) * 8))
        return fail(LADDER_EINVAL, "t overlaps an input");
    EpiMP2 ep{t, eps, o, v};
    StageTimer tm(LADDER_STAGE_MP2, gemm_flops(o * v, o * v, n), gemm_bytes(o * v, o * v, n), (hipStream_t)stream);
    return hip_check(launch_gemm<true, true>(Lov, n, Lov, n, o * v, o * v, n, ep, (hipStream_t)stream), "amplitude GEMM launch");
}

int ladder_amplitude_update(int64_t o, int64_t v, const double* eps, const double* R, double* t, void* stream) {
    g_last_error.clear();
    Sizes s;
    int rc;
    if ((rc = check_dims(o, v, 1, s))) return rc;
    if (!eps || !R || !t) return fail(LADDER_EINVAL, "eps, R and t must be non-NULL");
    if (!aligned8(eps) || !aligned8(R) || !aligned8(t)) return fail(LADDER_EINVAL, "misaligned pointer");
    if (R != t && overlap(t, s.ovv_elems * 8, R, s.ovv_elems * 8)) return fail(LADDER_EINVAL, "R partially overlaps t");
    if (overlap(t, s.ovv_elems * 8, eps, (o + v) * 8)) return fail(LADDER_EINVAL, "t overlaps eps");
    StageTimer tm(LADDER_STAGE_UPDATE, 2.0 * (double)s.ovv_elems, 24.0 * (double)s.ovv_elems, (hipStream_t)stream);
    hipLaunchKernelGGL(amplitude_update_kernel, dim3(grid_for(s.ovv_elems)), dim3(256), 0, (hipStream_t)stream, eps, R, t, o, v);
    return hip_check(hipGetLastError(), "amplitude update launch");
}

int ladder_batched_workspace_size(int count, const ladder_instance* inst, uint32_t what, const ladder_options* opts,
                                  size_t* bytes) {
    (void)count; (void)inst; (void)what; (void)opts; (void)bytes;
    return fail(LADDER_EUNSUPPORTED, "ladder_batched is not built into this library yet");
}

int ladder_batched(int count, const ladder_instance* inst, uint32_t what, void* ws, size_t ws_bytes,
                   const ladder_options* opts, void* stream) {
    (void)count; (void)inst; (void)what; (void)ws; (void)ws_bytes; (void)opts; (void)stream;
    return fail(LADDER_EUNSUPPORTED, "ladder_batched is not built into this library yet");
}

int ladder_profile_start(void) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (auto& r : g_prof) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    g_prof.clear();
    g_prof_on = true;
    return LADDER_OK;
}

int ladder_profile_stop(ladder_stage_stats* out, int max_stages, int* n_out) {
    g_last_error.clear();
    std::vector<StageRec> recs;
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        g_prof_on = false;
        recs.swap(g_prof);
    }
    ladder_stage_stats acc[LADDER_NUM_STAGES];
    for (int i = 0; i < LADDER_NUM_STAGES; ++i) acc[i] = ladder_stage_stats{i, 0, 0.0, 0.0, 0.0};
    int rc = LADDER_OK;
    for (auto& r : recs) {
        float ms = 0.f;
        hipError_t e = hipEventSynchronize(r.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
        if (e != hipSuccess && rc == LADDER_OK) rc = hip_check(e, "profile event");
        acc[r.stage].launches += 1;
        acc[r.stage].total_ms += ms;
        acc[r.stage].flops += r.flops;
        acc[r.stage].bytes += r.bytes;
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    int k = 0;
    for (int i = 0; i < LADDER_NUM_STAGES; ++i)
        if (acc[i].launches && out && k < max_stages) out[k++] = acc[i];
    if (n_out) *n_out = k;
    return rc;
}

void ladder_shutdown(void) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (auto& r : g_prof) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    g_prof.clear();
    g_prof_on = false;
}

}  // extern "C"
