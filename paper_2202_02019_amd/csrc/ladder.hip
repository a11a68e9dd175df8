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
//
// Precision LADDER_FP64 runs the four GEMMs on v_mfma_f64_16x16x4_f64.
// Precisions LADDER_SPLIT_INT8 and LADDER_SPLIT_BF16 first cut every GEMM operand
// into S exponent-aligned slices along its contraction index (inputs once per
// call, the g and D tiles once per batch) and run the GEMMs on INT8 MFMA with
// exact INT32 level sums (split_i8.hpp) or on BF16 MFMA with exact FP32 chunk
// sums (split_bf16.hpp), folded into FP64; R, E and X are accumulated and stored
// in FP64.
#include <hip/hip_runtime.h>

#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <string>
#include <vector>

#include "../../include/ladder.h"
#include "gemm_f64.hpp"
#include "split_bf16.hpp"
#include "split_i8.hpp"
#include "pm_pack.hpp"

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
constexpr int DEFAULT_SLICES = 5;       // BF16
constexpr int DEFAULT_SLICES_INT8 = 6;  // seven bits per slice: six meet the energy target where five do not

// ------------------------------------------------------------ stage timing
struct StageRec {
    int stage;
    hipEvent_t a, b;
    double flops, bytes;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<StageRec> g_prof;
thread_local bool g_capturing = false;  // no timing events (graph capture, allocation-free calls)

// Brackets one launch with events on its stream when profiling is on.
struct StageTimer {
    StageRec rec{};
    bool on = false;
    hipStream_t st;
    StageTimer(int stage, double flops, double bytes, hipStream_t s) : st(s) {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        if (!g_prof_on || g_capturing) return;
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

double gemm_flops(int64_t M, int64_t N, int64_t K) { return 2.0 * (double)M * (double)N * (double)K; }
// Algorithmic bytes of an FP64 GEMM: both operands read once, the result written once.
double gemm_bytes(int64_t M, int64_t N, int64_t K) { return 8.0 * ((double)M * K + (double)K * N + (double)M * N); }

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
    if (o < 1 || v < 1 || n < 1)
        return fail(LADDER_EINVAL, "dimensions must be >= 1 (o=%lld v=%lld n=%lld)", (long long)o, (long long)v, (long long)n);
    if (o > MAX_DIM || v > MAX_DIM || n > MAX_DIM) return fail(LADDER_EINVAL, "dimension above 2^20");
    if (!mul_ok(o, o, s.oo) || !mul_ok(v, v, s.vv) || !mul_ok(s.oo, s.vv, s.ovv_elems) || !mul_ok(s.vv, n, s.vvn) ||
        !mul_ok(s.vv, v, s.vvv) || s.ovv_elems > INT64_MAX / 16 || s.vvn > INT64_MAX / 16 || s.vvv > INT64_MAX / 16)
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
    if (o.precision != LADDER_FP64 && o.precision != LADDER_SPLIT_BF16 && o.precision != LADDER_SPLIT_INT8)
        return fail(LADDER_EUNSUPPORTED, "unknown precision %d", (int)o.precision);
    if (o.n_slices_adjoint < 0) return fail(LADDER_EINVAL, "n_slices_adjoint must be >= 0");
    if (o.precision != LADDER_FP64) {
        const int dflt = o.precision == LADDER_SPLIT_INT8 ? DEFAULT_SLICES_INT8 : DEFAULT_SLICES;
        if (o.n_slices == 0) o.n_slices = dflt;
        if (o.n_slices < 2 || o.n_slices > SPLIT_MAX_S)
            return fail(LADDER_EUNSUPPORTED, "n_slices must be 0 (default %d) or in [2, %d], got %d", dflt,
                        SPLIT_MAX_S, (int)o.n_slices);
        if (o.n_slices_adjoint == 0) o.n_slices_adjoint = o.n_slices;
        if (o.n_slices_adjoint < 2 || o.n_slices_adjoint > SPLIT_MAX_S)
            return fail(LADDER_EUNSUPPORTED, "n_slices_adjoint must be 0 (= n_slices) or in [2, %d], got %d",
                        SPLIT_MAX_S, (int)o.n_slices_adjoint);
    } else {
        o.n_slices_adjoint = 0;
    }
    if (o.n_abatch < 0) return fail(LADDER_EINVAL, "n_abatch must be >= 0");
    if (o.flags & ~(LADDER_FLAG_GENERAL | LADDER_FLAG_DENSE))
        return fail(LADDER_EUNSUPPORTED, "unknown flag bits 0x%x", o.flags);
    return LADDER_OK;
}

constexpr size_t ALIGN = 256;
size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

int64_t tiles(int64_t M, int64_t N) { return ((M + F64_BM - 1) / F64_BM) * ((N + F64_BN - 1) / F64_BN); }
static_assert(F64_BM == SPLIT_BM && F64_BN == SPLIT_BN, "energy partial slots assume one tile size");

// Bump allocator over the caller's workspace (offsets only; sizes 256-aligned).
struct Arena {
    size_t top = 0;
    size_t take(size_t bytes) {
        const size_t off = top;
        top += align_up(bytes);
        return off;
    }
};

// A slice specification: the slice count S, with SPLIT_I8 added for INT8 slices
// (split_i8.hpp) instead of BF16 ones (split_bf16.hpp); 0 means FP64.
constexpr int SPLIT_I8 = 16;
int slice_count(int spec) { return spec & (SPLIT_I8 - 1); }
bool slice_is_i8(int spec) { return (spec & SPLIT_I8) != 0; }
int slice_spec(const ladder_options& op, int n) {
    return op.precision == LADDER_FP64 ? 0 : n | (op.precision == LADDER_SPLIT_INT8 ? SPLIT_I8 : 0);
}
// Bytes of one sliced element (all slices).
int slice_elem_bytes(int spec) { return slice_count(spec) * (slice_is_i8(spec) ? 1 : 2); }

// Output tiles of a GEMM launch (one workgroup each) for a slice spec.
int64_t split_tiles(int spec, int64_t M, int64_t N) {
    return slice_is_i8(spec) ? ((M + SPLIT8_BM - 1) / SPLIT8_BM) * ((N + SPLIT8_BN - 1) / SPLIT8_BN) : tiles(M, N);
}

// One sliced operand: S slices of R rows x Kp, and nch x R exponents.
struct SlicedBuf {
    size_t s_off = 0, e_off = 0;
    int64_t R = 0, K = 0;
    bool i8 = false;
};
size_t slice_bytes(int spec, int64_t R, int64_t K) {
    return slice_is_i8(spec) ? (size_t)slice_count(spec) * (size_t)split8_slice_stride(R, K)
                             : (size_t)slice_count(spec) * (size_t)split_slice_stride(R, K) * 2;
}
size_t exp_bytes(int64_t R, int64_t K) { return (size_t)split_nchunk(K) * (size_t)R * 4; }
SlicedBuf take_sliced(Arena& a, int spec, int64_t R, int64_t K) {
    SlicedBuf b;
    b.R = R;
    b.K = K;
    b.i8 = slice_is_i8(spec);
    b.s_off = a.take(slice_bytes(spec, R, K));
    b.e_off = a.take(exp_bytes(R, K));
    return b;
}

// Batch plan and workspace layout.  The batch region (g or D tile, and its
// slices in split mode) is shared by forward and adjoint; the rest holds the
// per-call data of one direction (slices of the inputs, energy partials, the
// pair-swapped copies of the general adjoint), and both directions start at the
// same offset.
struct Plan {
    int S = 0;   // slices of the forward GEMMs (B, C); 0: FP64
    int Sa = 0;  // slices of the adjoint GEMMs (E, F); 0: FP64
    int64_t nA = 0, nbatch = 0;
    int64_t b_lo = 0, b_hi = 0;          // batches this call runs (all of them except when timing samples)
    size_t tile_off = 0;                 // FP64 g_A or D_A, nA*v^3 doubles
    SlicedBuf tile_sl;                   // split: slices of the tile (rows nA*v, K = v^2)
    size_t part_off = 0, part_per_batch = 0;
    SlicedBuf L_J, tau_cd;               // split forward: L along J, tau along (cd)
    SlicedBuf w_ij, tau_ij, L_bd;        // split adjoint: w and tau along (ij) (rows (ab)/(cd)), L along (bd) (rows J)
    size_t swap_off = 0;                 // general adjoint: P w and P tau, FP64
    SlicedBuf pw_ij, ptau_ij;            // general split adjoint: their slices
    // +/- packed path (pair-symmetric inputs): sizes and offsets
    bool pm = false;
    int64_t P2o = 0, Q2o = 0, P2v = 0, Q2v = 0, NP = 0, NM = 0;  // NP, NM: packed g rows of a full batch
    size_t f_tp = 0, f_tm = 0, f_gp = 0, f_gm = 0, f_rp = 0, f_rm = 0;  // forward, FP64
    SlicedBuf tp_cd, tm_cd, gp_sl, gm_sl;                               // forward, split
    size_t a_wp = 0, a_wm = 0, a_tp = 0, a_tm = 0, a_dp = 0, a_dm = 0;  // adjoint, FP64
    SlicedBuf wp_ij, wm_ij, tp_ij, tm_ij;                               // adjoint, split
    SlicedBuf L_b;                                                      // adjoint, split: L rows (b in batch) along K
    // split-K partial tiles of the long-K split GEMMs (GEMM-C on the +/- path, GEMM-F)
    size_t f_skp = 0, a_skp = 0;
    int64_t f_skp_elems = 0, a_skp_elems = 0;
    size_t fwd_total = 0, adj_total = 0, total = 0;
};

constexpr int64_t KSPLIT_MAX = 4;
// INT8 plans: K-splits of the long-K GEMMs (each split at least KSPLIT_I8_CHUNKS chunks).
// The 128 x 64 tiles put twice as many workgroups, and panels, on an XCD as the BF16
// ones; shorter K ranges keep the workgroups that share panels closer together in K,
// so more of the re-read panels are still in L2.
constexpr int64_t KSPLIT_I8_MAX = 16, KSPLIT_I8_CHUNKS = 32;
int64_t ksplit_cap(int spec) { return slice_is_i8(spec) ? KSPLIT_I8_MAX : KSPLIT_MAX; }

constexpr int PM_UNPACK_GRID = 1024;  // blocks of the R unpack kernel (one energy partial each)

Plan make_plan(int64_t o, int64_t v, int64_t n, const ladder_options& op, const Sizes& s) {
    Plan p;
    p.S = slice_spec(op, op.n_slices);
    p.Sa = slice_spec(op, op.n_slices_adjoint);
    const int Smax = std::max(p.S, p.Sa);
    const bool packed = !(op.flags & (LADDER_FLAG_GENERAL | LADDER_FLAG_DENSE));
    int64_t nA = op.n_abatch;
    if (nA == 0) {
        int64_t per_a = s.vvv * 8 * (packed ? 2 : 1);  // the tile, plus its packed halves on the +/- path
        if (Smax) per_a += (int64_t)(slice_bytes(Smax, v, s.vv) + exp_bytes(v, s.vv));
        nA = (int64_t)(LADDER_DEFAULT_TILE_BYTES / (size_t)per_a);
        // several batches, so that no v^4-sized array is ever held at once
        nA = std::min(nA, packed ? (v + 3) / 4 : (v + 1) / 2);
        if (nA < 1) nA = 1;
    }
    if (nA > v) nA = v;
    p.nA = nA;
    p.nbatch = (v + nA - 1) / nA;
    p.b_lo = 0;
    p.b_hi = p.nbatch;

    Arena a;
    p.tile_off = a.take((size_t)(nA * s.vvv) * 8);
    if (p.S) {
        // slices of the batch tile: rows n_A v along K = v^2 (GEMM-F of the dense path and the
        // packed path's tile (alpha)), or rows v^2 along K = n_A v (tile (beta)); room for either
        p.tile_sl.R = nA * v;
        p.tile_sl.K = s.vv;
        p.tile_sl.i8 = slice_is_i8(Smax);
        p.tile_sl.s_off = a.take(std::max(slice_bytes(Smax, nA * v, s.vv), slice_bytes(Smax, s.vv, nA * v)));
        p.tile_sl.e_off = a.take(std::max(exp_bytes(nA * v, s.vv), exp_bytes(s.vv, nA * v)));
    }
    const size_t common = a.top;

    const bool general = (op.flags & LADDER_FLAG_GENERAL) != 0;
    p.pm = !general && !(op.flags & LADDER_FLAG_DENSE);
    if (p.pm) {
        p.P2o = pm_P2(o); p.Q2o = pm_Q2(o); p.P2v = pm_P2(v); p.Q2v = pm_Q2(v);
        p.NP = pm_gp_off(nA, v, 0);
        p.NM = pm_gm_off(nA, v, 0);
    }

    Arena f = a;  // forward-only part
    if (!p.pm) {
        p.part_per_batch = (size_t)split_tiles(p.S, s.oo, nA * v);
        p.part_off = f.take(p.part_per_batch * (size_t)p.nbatch * 8);
        if (p.S) {
            p.L_J = take_sliced(f, p.S, s.vv, n);
            p.tau_cd = take_sliced(f, p.S, s.oo, s.vv);
        }
    } else {
        p.part_per_batch = 2 * PM_UNPACK_GRID;
        p.part_off = f.take(p.part_per_batch * (size_t)p.nbatch * 8);
        p.f_tp = f.take((size_t)(p.P2o * p.P2v) * 8);
        p.f_tm = f.take((size_t)(p.Q2o * p.Q2v) * 8 + 8);
        p.f_gp = f.take((size_t)(p.NP * p.P2v) * 8);
        p.f_gm = f.take((size_t)(p.NM * p.Q2v) * 8 + 8);
        p.f_rp = f.take((size_t)(p.P2o * p.NP) * 8);
        p.f_rm = f.take((size_t)(p.Q2o * p.NM) * 8 + 8);
        if (p.S) {
            p.L_J = take_sliced(f, p.S, s.vv, n);
            p.tp_cd = take_sliced(f, p.S, p.P2o, p.P2v);
            p.tm_cd = take_sliced(f, p.S, std::max<int64_t>(p.Q2o, 1), std::max<int64_t>(p.Q2v, 1));
            p.gp_sl = take_sliced(f, p.S, p.NP, p.P2v);
            p.gm_sl = take_sliced(f, p.S, std::max<int64_t>(p.NM, 1), std::max<int64_t>(p.Q2v, 1));
            p.f_skp_elems = ksplit_cap(p.S) * std::max(p.P2o * p.NP, p.Q2o * p.NM);
            p.f_skp = f.take((size_t)p.f_skp_elems * 8);
        }
    }
    p.fwd_total = f.top;

    Arena d = a;  // adjoint-only part
    if (!p.pm) {
        if (general) p.swap_off = d.take((size_t)s.ovv_elems * 16);
        if (p.S) {
            p.w_ij = take_sliced(d, p.Sa, s.vv, s.oo);
            p.tau_ij = take_sliced(d, p.Sa, s.vv, s.oo);
            p.L_bd = take_sliced(d, p.Sa, n, s.vv);
            if (general) {
                p.pw_ij = take_sliced(d, p.Sa, s.vv, s.oo);
                p.ptau_ij = take_sliced(d, p.Sa, s.vv, s.oo);
            }
        }
    } else {
        p.a_wp = d.take((size_t)(p.P2o * p.P2v) * 8);
        p.a_wm = d.take((size_t)(p.Q2o * p.Q2v) * 8 + 8);
        p.a_tp = d.take((size_t)(p.P2o * p.P2v) * 8);
        p.a_tm = d.take((size_t)(p.Q2o * p.Q2v) * 8 + 8);
        p.a_dp = d.take((size_t)(nA * v * p.P2v) * 8);
        p.a_dm = d.take((size_t)(nA * v * p.Q2v) * 8 + 8);
        if (p.S) {
            p.wp_ij = take_sliced(d, p.Sa, p.P2v, p.P2o);
            p.wm_ij = take_sliced(d, p.Sa, std::max<int64_t>(p.Q2v, 1), std::max<int64_t>(p.Q2o, 1));
            p.tp_ij = take_sliced(d, p.Sa, p.P2v, p.P2o);
            p.tm_ij = take_sliced(d, p.Sa, std::max<int64_t>(p.Q2v, 1), std::max<int64_t>(p.Q2o, 1));
            p.L_bd = take_sliced(d, p.Sa, n, s.vv);
            p.L_b = take_sliced(d, p.Sa, n, nA * v);
        }
    }
    if (p.S) {
        p.a_skp_elems = ksplit_cap(p.Sa) * nA * v * n;  // split-K only where ksplit * M * n fits (choose_ksplit)
        p.a_skp = d.take((size_t)p.a_skp_elems * 8);
    }
    p.adj_total = d.top;
    (void)common;
    p.total = std::max(p.fwd_total, p.adj_total);
    return p;
}

// ---------------------------------------------------------------- autotuned batch sizes
// ladder_autotune measures candidate virtual-batch sizes on the caller's data and
// keeps the fastest per shape and options; later calls with n_abatch = 0 use it
// whenever its workspace fits the one they are given.
struct TuneKey {
    int64_t o, v, n;
    int32_t precision, slices, slices_adj;
    uint32_t flags;
    bool operator<(const TuneKey& b) const {
        return std::tie(o, v, n, precision, slices, slices_adj, flags) <
               std::tie(b.o, b.v, b.n, b.precision, b.slices, b.slices_adj, b.flags);
    }
};
std::mutex g_tune_mu;
std::map<TuneKey, int64_t> g_tuned;
int64_t g_tune_gen = 0;  // bumped on every change: part of the batched graph cache key

TuneKey tune_key(int64_t o, int64_t v, int64_t n, const ladder_options& op) {
    const bool sp = op.precision != LADDER_FP64;
    return TuneKey{o, v, n, op.precision, sp ? op.n_slices : 0, sp ? op.n_slices_adjoint : 0, op.flags};
}

bool tuned_batch(const TuneKey& k, int64_t& nA) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tuned.find(k);
    if (it == g_tuned.end()) return false;
    nA = it->second;
    return true;
}

// The plan of a call.  An explicit n_abatch wins; otherwise the tuned batch size of
// this shape and options when there is one and its workspace fits ws_bytes, else the
// default.  For a size query (sizing = true) the larger of the two plans is returned,
// so that a workspace of that size runs the tuned plan.
Plan choose_plan(int64_t o, int64_t v, int64_t n, const ladder_options& op, const Sizes& s, size_t ws_bytes,
                 bool sizing) {
    Plan def = make_plan(o, v, n, op, s);
    int64_t t = 0;
    if (op.n_abatch != 0 || !tuned_batch(tune_key(o, v, n, op), t)) return def;
    ladder_options o2 = op;
    o2.n_abatch = t;
    Plan tp = make_plan(o, v, n, o2, s);
    if (sizing) return tp.total >= def.total ? tp : def;
    return tp.total <= ws_bytes ? tp : def;
}

// Executed GEMM flops of batch bi of a plan (both directions), the work model that
// turns the timed sample batches into an estimate for the whole call.
double batch_work(const Plan& p, int64_t o, int64_t v, int64_t n, const Sizes& s, bool general, int64_t bi) {
    const int64_t a0 = bi * p.nA, nA = std::min(p.nA, v - a0);
    if (p.pm) {  // forward over a in [a0, a0+nA); adjoint over b in [a0, a0+nA) with rows a <= b
        const double NPb = (double)pm_gp_off(nA, v, a0), NMb = (double)pm_gm_off(nA, v, a0);
        const int64_t A = a0 + nA;
        const double rowsP = (double)(pm_P2(A) - pm_P2(a0)), rowsQ = (double)(pm_Q2(A) - pm_Q2(a0));
        return gemm_flops(nA * v, (v - a0) * v, n) + 2.0 * ((double)p.P2o * NPb * p.P2v + (double)p.Q2o * NMb * p.Q2v) +
               2.0 * (rowsP * p.P2v * p.P2o + rowsQ * p.Q2v * p.Q2o) + 2.0 * gemm_flops(nA * v, n, A * v);
    }
    (void)o;
    return gemm_flops(nA * v, s.vv, n) + gemm_flops(s.oo, nA * v, s.vv) + (general ? 2.0 : 1.0) * gemm_flops(nA * v, s.vv, s.oo) +
           gemm_flops(nA * v, n, s.vv);
}

// "gfx950:256" (architecture and compute units), the device field of the cache file.
std::string device_tag() {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string arch(prop.gcnArchName);
    const size_t c = arch.find(':');
    if (c != std::string::npos) arch.resize(c);
    return arch + ":" + std::to_string(prop.multiProcessorCount);
}

// ---------------------------------------------------------------- launches
template <bool AK, bool BK, int STAGE, class Epi>
hipError_t launch_gemm(const double* A, int64_t lda, const double* B, int64_t ldb, int64_t M, int64_t N, int64_t K,
                       const Epi& epi, hipStream_t st) {
    GemmShape sh{A, lda, B, ldb, M, N, K};
    hipLaunchKernelGGL((gemm_f64_kernel<AK, BK, Epi, STAGE>), dim3((unsigned)tiles(M, N)), dim3(F64_THREADS), 0, st, sh,
                       epi);
    return hipGetLastError();
}

// A view of rows [row0, row0 + rows) of a sliced buffer.
SplitOperand view(char* ws, const SlicedBuf& b, int64_t row0) {
    SplitOperand v;
    v.s = (const unsigned short*)(ws + b.s_off);
    v.i8 = b.i8;
    if (b.i8) {  // byte slices: strides in bytes, 32 k per k-block
        v.slice_stride = split8_slice_stride(b.R, b.K);
        v.nkb = split8_kpad(b.K) / 32;
    } else {
        v.slice_stride = split_slice_stride(b.R, b.K);
        v.nkb = split_kpad(b.K) / 16;
    }
    v.row_off = row0;
    v.e = (const int*)(ws + b.e_off) + row0;
    v.e_ld = b.R;
    return v;
}

template <int S, int STAGE, class Epi>
hipError_t launch_split_s(const SplitShape& sh, const Epi& epi, hipStream_t st) {
    if (sh.a.i8 || sh.b.i8) return hipErrorInvalidValue;  // BF16 views only
    hipLaunchKernelGGL((gemm_split_kernel<S, Epi, STAGE>), dim3((unsigned)(tiles(sh.M, sh.N) * sh.ksplit)),
                       dim3(SPLIT_THREADS), 0, st, sh, epi);
    if (sh.ksplit > 1) {
        const int64_t blocks = std::min<int64_t>((sh.M * sh.N + 255) / 256, 4096);
        hipLaunchKernelGGL((splitk_reduce_kernel<Epi>), dim3((unsigned)blocks), dim3(256), 0, st, sh.part, sh.M, sh.N,
                           sh.ksplit, epi);
    }
    return hipGetLastError();
}

template <int S, int STAGE, class Epi>
hipError_t launch_i8_s(const SplitShape& sh, const Epi& epi, hipStream_t st) {
    if (!sh.a.i8 || !sh.b.i8) return hipErrorInvalidValue;  // INT8 views only
    hipLaunchKernelGGL((gemm_i8_kernel<S, Epi, STAGE>), dim3((unsigned)(split_tiles(SPLIT_I8, sh.M, sh.N) * sh.ksplit)),
                       dim3(SPLIT8_THREADS), 0, st, sh, epi);
    if (sh.ksplit > 1) {
        const int64_t blocks = std::min<int64_t>((sh.M * sh.N + 255) / 256, 4096);
        hipLaunchKernelGGL((splitk_reduce_kernel<Epi>), dim3((unsigned)blocks), dim3(256), 0, st, sh.part, sh.M, sh.N,
                           sh.ksplit, epi);
    }
    return hipGetLastError();
}

// Compute units of the current device (cached per device).
int64_t device_cus() {
    static int64_t cus[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (!cus[dev]) {
        int c = 0;
        cus[dev] = (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && c > 0) ? c : 256;
    }
    return cus[dev];
}

// Split-K factor for a split GEMM whose epilogue needs no per-tile energy partial:
// the number of K-splits s (whole 256-chunks each, at most KSPLIT_MAX, s*M*N partial
// doubles within `room`) that minimises the waves of workgroups per unit of work,
// ceil(tiles*s / CUs) / s, taken only when it saves at least 4% over s = 1.  INT8
// plans take the largest s up to KSPLIT_I8_MAX with at least KSPLIT_I8_CHUNKS chunks
// per split that fits `room`.
int64_t choose_ksplit(int spec, int64_t M, int64_t N, int64_t K, int64_t room) {
    const int64_t T = split_tiles(spec, M, N), cus = device_cus(), nch = split_nchunk(K);
    if (slice_is_i8(spec)) {
        int64_t s = std::min(KSPLIT_I8_MAX, nch / KSPLIT_I8_CHUNKS);
        while (s > 1 && s * M * N > room) --s;
        return std::max<int64_t>(s, 1);
    }
    double best = (double)((T + cus - 1) / cus);
    const double base = best;
    int64_t pick = 1;
    for (int64_t s = 2; s <= std::min(KSPLIT_MAX, nch); ++s) {
        if (s * M * N > room) break;
        const double c = (double)((T * s + cus - 1) / cus) / (double)s;
        if (c < best * 0.99) {
            best = c;
            pick = s;
        }
    }
    return best <= 0.96 * base ? pick : 1;
}

template <int STAGE, class Epi>
hipError_t launch_split(int S, const SplitShape& sh, const Epi& epi, hipStream_t st) {
    if (slice_is_i8(S)) {
        switch (slice_count(S)) {
            case 2: return launch_i8_s<2, STAGE>(sh, epi, st);
            case 3: return launch_i8_s<3, STAGE>(sh, epi, st);
            case 4: return launch_i8_s<4, STAGE>(sh, epi, st);
            case 5: return launch_i8_s<5, STAGE>(sh, epi, st);
            case 6: return launch_i8_s<6, STAGE>(sh, epi, st);
            default: return hipErrorInvalidValue;
        }
    }
    switch (S) {
        case 2: return launch_split_s<2, STAGE>(sh, epi, st);
        case 3: return launch_split_s<3, STAGE>(sh, epi, st);
        case 4: return launch_split_s<4, STAGE>(sh, epi, st);
        case 5: return launch_split_s<5, STAGE>(sh, epi, st);
        case 6: return launch_split_s<6, STAGE>(sh, epi, st);
        default: return hipErrorInvalidValue;
    }
}

template <int S>
hipError_t slice_s(bool transposed, const double* src, int64_t ld, int64_t R, int64_t K, unsigned short* sl, int* ex,
                   hipStream_t st) {
    const int64_t nch = split_nchunk(K);
    if (!transposed) {
        const int64_t blocks = ((R + 15) / 16) * nch;
        hipLaunchKernelGGL((slice_rows_kernel<S, DenseRows>), dim3((unsigned)blocks), dim3(256), 0, st, DenseRows{src, ld},
                           R, K, sl, ex, R);
    } else {
        const int64_t blocks = ((R + 31) / 32) * nch;
        hipLaunchKernelGGL((slice_cols_kernel<S>), dim3((unsigned)blocks), dim3(256), 0, st, src, ld, R, K, sl, ex, R);
    }
    return hipGetLastError();
}

template <int S>
hipError_t slice8_s(bool transposed, const double* src, int64_t ld, int64_t R, int64_t K, int8_t* sl, int* ex,
                    hipStream_t st) {
    const int64_t nch = split_nchunk(K);
    if (!transposed) {
        const int64_t blocks = ((R + 15) / 16) * nch;
        hipLaunchKernelGGL((slice8_rows_kernel<S, DenseRows>), dim3((unsigned)blocks), dim3(256), 0, st,
                           DenseRows{src, ld}, R, K, sl, ex, R);
    } else {
        const int64_t blocks = ((R + 31) / 32) * nch;
        hipLaunchKernelGGL((slice8_cols_kernel<S>), dim3((unsigned)blocks), dim3(256), 0, st, src, ld, R, K, sl, ex, R);
    }
    return hipGetLastError();
}

// Slices src into the buffer b (rows b.R, length b.K).  transposed: element
// (r, k) at src[k*ld + r]; otherwise at src[r*ld + k].
int slice_into(int S, bool transposed, const double* src, int64_t ld, char* ws, const SlicedBuf& b, hipStream_t st) {
    StageTimer tm(LADDER_STAGE_SLICE, 0.0, (8.0 + slice_elem_bytes(S)) * (double)b.R * (double)b.K, st);
    if (slice_is_i8(S) != b.i8) return fail(LADDER_EINVAL, "internal: slice format of the buffer");
    unsigned short* sl = (unsigned short*)(ws + b.s_off);
    int* ex = (int*)(ws + b.e_off);
    hipError_t e;
    if (slice_is_i8(S)) {
        int8_t* s8 = (int8_t*)(ws + b.s_off);
        switch (slice_count(S)) {
            case 2: e = slice8_s<2>(transposed, src, ld, b.R, b.K, s8, ex, st); break;
            case 3: e = slice8_s<3>(transposed, src, ld, b.R, b.K, s8, ex, st); break;
            case 4: e = slice8_s<4>(transposed, src, ld, b.R, b.K, s8, ex, st); break;
            case 5: e = slice8_s<5>(transposed, src, ld, b.R, b.K, s8, ex, st); break;
            case 6: e = slice8_s<6>(transposed, src, ld, b.R, b.K, s8, ex, st); break;
            default: e = hipErrorInvalidValue;
        }
        return hip_check(e, "slice launch");
    }
    switch (S) {
        case 2: e = slice_s<2>(transposed, src, ld, b.R, b.K, sl, ex, st); break;
        case 3: e = slice_s<3>(transposed, src, ld, b.R, b.K, sl, ex, st); break;
        case 4: e = slice_s<4>(transposed, src, ld, b.R, b.K, sl, ex, st); break;
        case 5: e = slice_s<5>(transposed, src, ld, b.R, b.K, sl, ex, st); break;
        case 6: e = slice_s<6>(transposed, src, ld, b.R, b.K, sl, ex, st); break;
        default: e = hipErrorInvalidValue;
    }
    return hip_check(e, "slice launch");
}

// Slices of a density tile of the +/- adjoint (rows b.R, length b.K) computed from its packed
// rows by the row slicer (the same exponents and slices as slicing the FP64 tile).
template <int S>
hipError_t slice_tile_s(const PmTileRows& src, const SlicedBuf& b, char* ws, hipStream_t st) {
    const int64_t blocks = ((b.R + 15) / 16) * split_nchunk(b.K);
    hipLaunchKernelGGL((slice_rows_kernel<S, PmTileRows>), dim3((unsigned)blocks), dim3(256), 0, st, src, b.R, b.K,
                       (unsigned short*)(ws + b.s_off), (int*)(ws + b.e_off), b.R);
    return hipGetLastError();
}
template <int S>
hipError_t slice8_tile_s(const PmTileRows& src, const SlicedBuf& b, char* ws, hipStream_t st) {
    const int64_t blocks = ((b.R + 15) / 16) * split_nchunk(b.K);
    hipLaunchKernelGGL((slice8_rows_kernel<S, PmTileRows>), dim3((unsigned)blocks), dim3(256), 0, st, src, b.R, b.K,
                       (int8_t*)(ws + b.s_off), (int*)(ws + b.e_off), b.R);
    return hipGetLastError();
}
int slice_tile_into(int S, const PmTileRows& src, char* ws, const SlicedBuf& b, hipStream_t st) {
    StageTimer tm(LADDER_STAGE_SLICE, 0.0, (16.0 + slice_elem_bytes(S)) * (double)b.R * (double)b.K, st);
    if (slice_is_i8(S) != b.i8) return fail(LADDER_EINVAL, "internal: slice format of the buffer");
    hipError_t e;
    if (slice_is_i8(S)) {
        switch (slice_count(S)) {
            case 2: e = slice8_tile_s<2>(src, b, ws, st); break;
            case 3: e = slice8_tile_s<3>(src, b, ws, st); break;
            case 4: e = slice8_tile_s<4>(src, b, ws, st); break;
            case 5: e = slice8_tile_s<5>(src, b, ws, st); break;
            case 6: e = slice8_tile_s<6>(src, b, ws, st); break;
            default: e = hipErrorInvalidValue;
        }
        return hip_check(e, "tile slice launch");
    }
    switch (S) {
        case 2: e = slice_tile_s<2>(src, b, ws, st); break;
        case 3: e = slice_tile_s<3>(src, b, ws, st); break;
        case 4: e = slice_tile_s<4>(src, b, ws, st); break;
        case 5: e = slice_tile_s<5>(src, b, ws, st); break;
        case 6: e = slice_tile_s<6>(src, b, ws, st); break;
        default: e = hipErrorInvalidValue;
    }
    return hip_check(e, "tile slice launch");
}

__global__ void fill_zero_kernel(double* __restrict__ x, int64_t count) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += (int64_t)gridDim.x * blockDim.x)
        x[t] = 0.0;
}

__global__ void scale_kernel(double* __restrict__ x, int64_t count, double f) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += (int64_t)gridDim.x * blockDim.x)
        x[t] *= f;
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

// Excited-state amplitudes: mode 0: U = R0 T + R2; mode 1: U = (R0/2) T + R~2 with
// R~_ij^ab = R_ij^ab (1 + [i = j][a = b]) (the diagonal doubles counted twice).
__global__ void excited_amplitudes_kernel(double R0, const double* __restrict__ T, const double* __restrict__ R2,
                                          int mode, double* __restrict__ U, int64_t o, int64_t v) {
    const int64_t total = o * o * v * v, vv = v * v;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
        if (mode == 0) {
            U[x] = R0 * T[x] + R2[x];
        } else {
            const int64_t ab = x % vv, ij = x / vv, i = ij / o, j = ij % o, a = ab / v, b = ab % v;
            U[x] = 0.5 * R0 * T[x] + (i == j && a == b ? 2.0 * R2[x] : R2[x]);
        }
    }
}

// Multipliers L2[j][i][a][c] (= L_ji^ac) to Lp[j][a][c][i]: for every (j, a) the [i][c]
// block (row stride v*v) is written transposed as [c][i] (row stride o) through a
// 32 x 33 LDS tile, so both the reads (along c) and the writes (along i) are
// contiguous.  Tiles are walked grid-stride; every index is checked against o and v.
__global__ __launch_bounds__(256) void ov3_permute_l2_kernel(const double* __restrict__ L2, double* __restrict__ Lp,
                                                             int64_t o, int64_t v) {
    __shared__ double tile[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int64_t ti_n = (o + 31) / 32, tc_n = (v + 31) / 32;
    const int64_t total = o * v * ti_n * tc_n;
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        const int64_t tc = t % tc_n, r1 = t / tc_n;
        const int64_t ti = r1 % ti_n, ja = r1 / ti_n;
        const int64_t j = ja / v, a = ja - j * v;
        const int64_t i0 = ti * 32, c0 = tc * 32;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t i = i0 + ty + 8 * r, c = c0 + tx;
            if (i < o && c < v) tile[ty + 8 * r][tx] = L2[((j * o + i) * v + a) * v + c];
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t c = c0 + ty + 8 * r, i = i0 + tx;
            if (i < o && c < v) Lp[((j * v + a) * v + c) * o + i] = tile[tx][ty + 8 * r];
        }
        __syncthreads();
    }
}

// Zt[b][a][K] = Z[a][b][K]: whole n-long rows moved, one (a, b) row per block step.
__global__ __launch_bounds__(256) void ov3_swap_vv_kernel(const double* __restrict__ Z, double* __restrict__ Zt,
                                                          int64_t v, int64_t n) {
    for (int64_t ab = blockIdx.x; ab < v * v; ab += gridDim.x) {
        const int64_t a = ab / v, b = ab - a * v;
        const double* src = Z + ab * n;
        double* dst = Zt + (b * v + a) * n;
        for (int64_t K = threadIdx.x; K < n; K += blockDim.x) dst[K] = src[K];
    }
}

// Reordering with an optional second term: out is walked in its own order over the
// extents D[0..3] (last index fastest, so the writes are contiguous) and
//   out[x] = c1 * in[sum_k idx_k s[k]] + c2 * in[sum_k idx_k t[k]]   (second read only if c2 != 0).
// The host checks that the largest offset of either stride set lies inside `in`.
struct Perm4 {
    int64_t D[4], s[4], t[4];
    double c1, c2;
};
__global__ __launch_bounds__(256) void permute4_kernel(const double* __restrict__ in, double* __restrict__ out, Perm4 p) {
    const int64_t total = p.D[0] * p.D[1] * p.D[2] * p.D[3];
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
        int64_t r = x;
        const int64_t i3 = r % p.D[3];
        r /= p.D[3];
        const int64_t i2 = r % p.D[2];
        r /= p.D[2];
        const int64_t i1 = r % p.D[1], i0 = r / p.D[1];
        double val = p.c1 * in[i0 * p.s[0] + i1 * p.s[1] + i2 * p.s[2] + i3 * p.s[3]];
        if (p.c2 != 0.0) val += p.c2 * in[i0 * p.t[0] + i1 * p.t[1] + i2 * p.t[2] + i3 * p.t[3]];
        out[x] = val;
    }
}

// Amplitude matrix of the singles-multiplier terms of d_abic, rows (m, b), columns (i, c):
//   A[(m,b),(i,c)] = R0 (2 t_im^cb - t_mi^cb) + 2 R~_mi^bc - R~_mi^cb,
//   R~_mi^pq = R_mi^pq (1 + [m = i][p = q]).
__global__ __launch_bounds__(256) void abic_amp_kernel(double R0, const double* __restrict__ T,
                                                       const double* __restrict__ R2, double* __restrict__ A,
                                                       int64_t o, int64_t v) {
    const int64_t total = o * o * v * v;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = x % v, r1 = x / v;
        const int64_t i = r1 % o, r2 = r1 / o;
        const int64_t b = r2 % v, m = r2 / v;
        const double dg = (m == i && b == c) ? 2.0 : 1.0;
        const double tt = 2.0 * T[((i * o + m) * v + c) * v + b] - T[((m * o + i) * v + c) * v + b];
        A[x] = R0 * tt + dg * (2.0 * R2[((m * o + i) * v + b) * v + c] - R2[((m * o + i) * v + c) * v + b]);
    }
}

// W_am = sum_kd L_mk^ad R^d_k, stored Wma[m][a]: one 64-lane wave per (m, a).
__global__ __launch_bounds__(256) void abic_wam_kernel(const double* __restrict__ L2, const double* __restrict__ R1,
                                                       double* __restrict__ Wma, int64_t o, int64_t v) {
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t w = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); w < o * v; w += waves) {
        const int64_t m = w / v, a = w - m * v;
        double s = 0.0;
        for (int64_t k = 0; k < o; ++k) {
            const double* l = L2 + ((m * o + k) * v + a) * v;
            const double* r = R1 + k * v;
            for (int64_t d = lane; d < v; d += 64) s += l[d] * r[d];
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
        if (lane == 0) Wma[m * v + a] = s;
    }
}

// MFMA ceiling probe: every wave issues `iters` rounds of four independent MFMAs on
// register operands (no memory traffic besides one checksum per thread), so the time
// of a launch is the matrix-core rate the chip sustains under its own clock and power
// limits.  KIND 0: v_mfma_f32_32x32x16_bf16 (32768 flops), KIND 1: v_mfma_f64_16x16x4_f64
// (2048 flops), KIND 2: v_mfma_i32_32x32x32_i8 (65536 operations).  The operands vary per
// lane, like real slice data.
template <int KIND>
__global__ __launch_bounds__(256) void mfma_probe_kernel(int64_t iters, double* __restrict__ out) {
    const int lane = threadIdx.x & 63;
    double sum = 0.0;
    if constexpr (KIND == 0) {
        bx8 a, b;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            a[i] = (__bf16)(1.0f + 0.0078125f * (float)((lane * 8 + i) % 97));
            b[i] = (__bf16)(0.5f - 0.00390625f * (float)((lane * 5 + 3 * i) % 89));
        }
        fx16 acc[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[k][r] = 0.0f;
        for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
            for (int k = 0; k < 4; ++k) acc[k] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[k], 0, 0, 0);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int r = 0; r < 16; ++r) sum += (double)acc[k][r];
    } else if constexpr (KIND == 1) {
        const double a = 1.0 + 0.001 * (double)lane, b = 0.5 - 0.0005 * (double)lane;
        dx4 acc[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[k] = dx4{0.0, 0.0, 0.0, 0.0};
        for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
            for (int k = 0; k < 4; ++k) acc[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[k], 0, 0, 0);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) sum += acc[k][0] + acc[k][1] + acc[k][2] + acc[k][3];
    } else {
        ix4 a, b;  // bytes in [-64, 64], as INT8 slices
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            uint32_t wa = 0, wb = 0;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                wa |= (uint32_t)(((lane * 16 + 4 * i + j) * 37 % 129 - 64) & 0xff) << (8 * j);
                wb |= (uint32_t)(((lane * 11 + 5 * i + 3 * j) * 53 % 129 - 64) & 0xff) << (8 * j);
            }
            a[i] = (int)wa;
            b[i] = (int)wb;
        }
        ix16 acc[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[k] = ix16{};
        for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
            for (int k = 0; k < 4; ++k) acc[k] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, acc[k], 0, 0, 0);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int r = 0; r < 16; ++r) sum += (double)acc[k][r];
    }
    out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = sum;
}

// Grid of the tiled packing kernels: tile pairs in x, rows over (y, z).
dim3 pm_grid(int64_t v, int64_t rows) {
    const int64_t gy = std::min<int64_t>(std::max<int64_t>(rows, 1), 65535);
    return dim3((unsigned)pm_tile_pairs(v), (unsigned)gy, (unsigned)((rows + gy - 1) / gy));
}

// Packs amplitudes x[o][o][v][v] to xp[P(i,j)][P(c,d)] and xm[Q(i,j)][Q(c,d)].
void pm_pack_amp(const double* x, int64_t o, int64_t v, double* xp, double* xm, hipStream_t st) {
    const PmRows rw{0, o, 0, 0};
    hipLaunchKernelGGL(pm_pack_pair_tiled_kernel, pm_grid(v, pm_P2(o)), dim3(256), 0, st, x, v, rw, pm_P2(o), xp,
                       pm_Q2(o) > 0 && pm_Q2(v) > 0 ? xm : nullptr);
}

unsigned grid_for(int64_t total) {
    int64_t g = (total + 255) / 256;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (unsigned)g;
}

// The split GEMM addresses a 128-row operand tile with 32-bit byte offsets.
int check_split_dims(const Sizes& s, int64_t n, const ladder_options& op) {
    if (op.precision == LADDER_FP64) return LADDER_OK;
    // the slicer grids: up to v^2 rows in blocks of 16 times the chunks of the longest k
    const int64_t kmax = std::max(std::max(s.vv, s.oo), n);
    if ((s.vv / 16 + 1) * split_nchunk(kmax) >= (int64_t(1) << 31))
        return fail(LADDER_EUNSUPPORTED, "split precision: v^2 * max(v^2, o^2, n) too large for the slicer grid");
    // the GEMM's 32-bit per-lane offsets span two panels of the longest k
    if (2 * (split_kpad(kmax) / 16) * SPLIT_PANEL * 16 * 2 + 4096 >= (int64_t(1) << 32))
        return fail(LADDER_EUNSUPPORTED, "split precision: max(v^2, o^2, n) too large for the panel offsets");
    return LADDER_OK;
}


// ---------------------------------------------------------------- +/- packed path
// Forward with the symmetric/antisymmetric packing of pm_pack.hpp: per batch the
// g tile is packed to g+ (a<=b, c<=d) and g- (a<b, c<d), the two products
// R+ = tau+ g+^T and R- = tau- g-^T run on (i<=j) and (i<j) rows, and the unpack
// kernel writes R_ij^ab and R_ij^ba for the batch's a (with the energy partials).
int forward_pm(int64_t o, int64_t v, int64_t n, const double* L, const double* tau, const double* tbar, double beta,
               double* R, double* E, char* w, const Plan& p, const Sizes& s, hipStream_t st) {
    int rc;
    const int S = p.S;
    double* g = (double*)(w + p.tile_off);
    double* part = (double*)(w + p.part_off);
    double *tp = (double*)(w + p.f_tp), *tm = (double*)(w + p.f_tm), *gp = (double*)(w + p.f_gp),
           *gm = (double*)(w + p.f_gm), *rp = (double*)(w + p.f_rp), *rm = (double*)(w + p.f_rm);
    {
        StageTimer tm_(LADDER_STAGE_PACK, 0.0, 16.0 * (double)pm_amp_count(o, v), st);
        pm_pack_amp(tau, o, v, tp, tm, st);
        if ((rc = hip_check(hipGetLastError(), "pack launch"))) return rc;
    }
    const bool minus = p.Q2o > 0 && p.Q2v > 0;
    if (S) {
        if ((rc = slice_into(S, false, L, n, w, p.L_J, st))) return rc;
        if ((rc = slice_into(S, false, tp, p.P2v, w, p.tp_cd, st))) return rc;
        if (minus && (rc = slice_into(S, false, tm, p.Q2v, w, p.tm_cd, st))) return rc;
    }
    for (int64_t bi = p.b_lo; bi < p.b_hi; ++bi) {
        const int64_t a0 = bi * p.nA;
        const int64_t nA = std::min(p.nA, v - a0);
        const int64_t NPb = pm_gp_off(nA, v, a0), NMb = pm_gm_off(nA, v, a0);
        {
            // only b >= a0 is needed by the packed g: N = (v - a0) v rows of L
            const int64_t Nb = (v - a0) * v;
            StageTimer tm_(LADDER_STAGE_GEMM_B, gemm_flops(nA * v, Nb, n), gemm_bytes(nA * v, Nb, n), st);
            EpiSwapMid eg{g, v, v - a0, v, 1.0, 0.0};
            hipError_t e;
            if (!S) {
                e = launch_gemm<true, true, LADDER_STAGE_GEMM_B>(L + a0 * v * n, n, L + a0 * v * n, n, nA * v, Nb, n, eg, st);
            } else {
                SplitShape sh{view(w, p.L_J, a0 * v), view(w, p.L_J, a0 * v), nA * v, Nb, n};
                e = launch_split<LADDER_STAGE_GEMM_B>(S, sh, eg, st);
            }
            if ((rc = hip_check(e, "GEMM-B launch"))) return rc;
        }
        {
            const int64_t cnt = pm_g_count(v, a0, nA);
            StageTimer tm_(LADDER_STAGE_PACK, 0.0, 24.0 * (double)cnt, st);
            const PmRows rw{1, 0, a0, nA};
            hipLaunchKernelGGL(pm_pack_pair_tiled_kernel, pm_grid(v, NPb), dim3(256), 0, st, g, v, rw, NPb, gp,
                               NMb > 0 && p.Q2v > 0 ? gm : nullptr);
            if ((rc = hip_check(hipGetLastError(), "pack launch"))) return rc;
        }
        const bool minus_b = minus && NMb > 0;
        SlicedBuf gps = p.gp_sl, gms = p.gm_sl;
        gps.R = NPb;
        gms.R = NMb;
        if (S) {
            if ((rc = slice_into(S, false, gp, p.P2v, w, gps, st))) return rc;
            if (minus_b && (rc = slice_into(S, false, gm, p.Q2v, w, gms, st))) return rc;
        }
        for (int sign = 0; sign < (minus_b ? 2 : 1); ++sign) {
            const int64_t M = sign ? p.Q2o : p.P2o, N = sign ? NMb : NPb, K = sign ? p.Q2v : p.P2v;
            StageTimer tm_(LADDER_STAGE_GEMM_C, gemm_flops(M, N, K), gemm_bytes(M, N, K), st);
            EpiStrided er{sign ? rm : rp, N, 1.0, 0.0, nullptr, nullptr};
            hipError_t e;
            if (!S) {
                e = launch_gemm<true, true, LADDER_STAGE_GEMM_C>(sign ? tm : tp, K, sign ? gm : gp, K, M, N, K, er, st);
            } else {
                SplitShape sh{view(w, sign ? p.tm_cd : p.tp_cd, 0), view(w, sign ? gms : gps, 0), M, N, K};
                sh.ksplit = choose_ksplit(S, M, N, K, p.f_skp_elems);
                sh.part = (double*)(w + p.f_skp);
                e = launch_split<LADDER_STAGE_GEMM_C>(S, sh, er, st);
            }
            if ((rc = hip_check(e, "GEMM-C launch"))) return rc;
        }
        {
            StageTimer tm_(LADDER_STAGE_UNPACK, 2.0 * (double)s.oo * nA * v, 16.0 * (double)s.oo * nA * v, st);
            for (int pass = 0; pass < 2; ++pass)
                hipLaunchKernelGGL(pm_unpack_R_kernel, dim3(PM_UNPACK_GRID), dim3(256), 0, st, rp, rm, o, v, a0, nA, beta,
                                   E ? tbar : nullptr, R, part + bi * p.part_per_batch + pass * PM_UNPACK_GRID, pass);
            if ((rc = hip_check(hipGetLastError(), "unpack launch"))) return rc;
        }
    }
    if (E) {
        const int64_t count = (int64_t)p.part_per_batch * p.nbatch;
        StageTimer tm_(LADDER_STAGE_ENERGY, (double)count, 8.0 * (double)count, st);
        hipLaunchKernelGGL(reduce_partials_kernel, dim3(1), dim3(256), 0, st, part, count, E);
        if ((rc = hip_check(hipGetLastError(), "energy reduction launch"))) return rc;
    }
    return LADDER_OK;
}

// Adjoint with the packing (pm_pack.hpp): the density is formed only on its rows
// a <= b, D+ = Wp^T tau+ on rows P(a,b) and D- = Wm^T tau- on rows Q(a,b), batch by
// batch of b; each batch's rows feed X twice, through tile (alpha) (X rows of the
// batch's b, K over a < b0 + nB) and tile (beta) (X rows a < b0 + nB, K over the
// batch's b).  X is scaled by beta once, then every contribution is added in a fixed
// order (deterministic).
int adjoint_pm(int64_t o, int64_t v, int64_t n, const double* L, const double* tau, const double* wt, double alpha,
               double beta, double* X, char* w, const Plan& p, const Sizes& s, hipStream_t st) {
    int rc;
    const int S = p.Sa;  // the adjoint's slice count
    double* D = (double*)(w + p.tile_off);
    double *wp = (double*)(w + p.a_wp), *wm = (double*)(w + p.a_wm), *tp = (double*)(w + p.a_tp),
           *tm = (double*)(w + p.a_tm), *dp = (double*)(w + p.a_dp), *dm = (double*)(w + p.a_dm);
    {
        StageTimer tm_(LADDER_STAGE_PACK, 0.0, 16.0 * (double)(2 * pm_amp_count(o, v)), st);
        pm_pack_amp(tau, o, v, tp, tm, st);
        const PmRows rw{2, o, 0, 0};
        hipLaunchKernelGGL(pm_pack_pair_tiled_kernel, pm_grid(v, p.P2o), dim3(256), 0, st, wt, v, rw, p.P2o, wp,
                           p.Q2o > 0 && p.Q2v > 0 ? wm : nullptr);
        if ((rc = hip_check(hipGetLastError(), "pack launch"))) return rc;
    }
    {   // X = beta X (not read when beta = 0); every product below adds to it
        if (beta == 0.0) hipLaunchKernelGGL(fill_zero_kernel, dim3(grid_for(s.vvn)), dim3(256), 0, st, X, s.vvn);
        else if (beta != 1.0) hipLaunchKernelGGL(scale_kernel, dim3(grid_for(s.vvn)), dim3(256), 0, st, X, s.vvn, beta);
        if ((rc = hip_check(hipGetLastError(), "scale launch"))) return rc;
    }
    const bool minus = p.Q2o > 0 && p.Q2v > 0;
    if (S) {
        if ((rc = slice_into(S, true, wp, p.P2v, w, p.wp_ij, st))) return rc;
        if ((rc = slice_into(S, true, tp, p.P2v, w, p.tp_ij, st))) return rc;
        if (minus) {
            if ((rc = slice_into(S, true, wm, p.Q2v, w, p.wm_ij, st))) return rc;
            if ((rc = slice_into(S, true, tm, p.Q2v, w, p.tm_ij, st))) return rc;
        }
        if ((rc = slice_into(S, true, L, n, w, p.L_bd, st))) return rc;
    }
    for (int64_t bi = p.b_lo; bi < p.b_hi; ++bi) {
        const int64_t b0 = bi * p.nA;
        const int64_t nB = std::min(p.nA, v - b0), A = b0 + nB;
        const int64_t rowsP = pm_P2(A) - pm_P2(b0), rowsQ = pm_Q2(A) - pm_Q2(b0);
        for (int sign = 0; sign < 2; ++sign) {
            const int64_t M = sign ? rowsQ : rowsP, N = sign ? p.Q2v : p.P2v, K = sign ? p.Q2o : p.P2o;
            if (M == 0 || N == 0) continue;
            if (sign && !minus) {  // o = 1: no antisymmetric part, D- = 0
                hipLaunchKernelGGL(fill_zero_kernel, dim3(grid_for(M * N)), dim3(256), 0, st, dm, M * N);
                if ((rc = hip_check(hipGetLastError(), "fill launch"))) return rc;
                continue;
            }
            StageTimer tm_(LADDER_STAGE_GEMM_E, gemm_flops(M, N, K), gemm_bytes(M, N, K), st);
            EpiStrided ed{sign ? dm : dp, N, 1.0, 0.0, nullptr, nullptr};
            hipError_t e;
            const int64_t r0 = sign ? pm_Q2(b0) : pm_P2(b0);
            if (!S) {
                e = launch_gemm<false, false, LADDER_STAGE_GEMM_E>((sign ? wm : wp) + r0, N, sign ? tm : tp, N, M, N, K, ed, st);
            } else {
                SplitShape sh{view(w, sign ? p.wm_ij : p.wp_ij, r0), view(w, sign ? p.tm_ij : p.tp_ij, 0), M, N, K};
                e = launch_split<LADDER_STAGE_GEMM_E>(S, sh, ed, st);
            }
            if ((rc = hip_check(e, "GEMM-E launch"))) return rc;
        }
        if (S) {  // L rows (b, w) of this batch, the K of tile (beta)
            SlicedBuf lb = p.L_b;
            lb.K = nB * v;
            if ((rc = slice_into(S, true, L + b0 * v * n, n, w, lb, st))) return rc;
        }
        for (int pass = 0; pass < 2; ++pass) {  // 0: tile (alpha), 1: tile (beta)
            const int64_t M = pass ? A * v : nB * v, K = pass ? nB * v : A * v;
            SlicedBuf tl = p.tile_sl;
            tl.R = M;
            tl.K = K;
            if (!S) {  // the FP64 tile for the FP64 GEMM
                StageTimer tm_(LADDER_STAGE_UNPACK, 0.0, 8.0 * (double)(M * K) + 8.0 * (double)(rowsP * p.P2v + rowsQ * p.Q2v), st);
                hipLaunchKernelGGL(pm_tile_ab_kernel, pm_grid(v, nB * A), dim3(256), 0, st, dp, dm, v, b0, nB,
                                   pass ? 0 : 1, D);
                if ((rc = hip_check(hipGetLastError(), "tile launch"))) return rc;
            } else if ((rc = slice_tile_into(S, PmTileRows{dp, dm, v, b0, nB, pass ? 0 : 1}, w, tl, st))) {
                return rc;  // the slices of the tile straight from the packed rows (no FP64 tile)
            }
            StageTimer tm_(LADDER_STAGE_GEMM_F, gemm_flops(M, n, K), gemm_bytes(M, n, K), st);
            // alpha: X rows (b, y), B = L rows (a, w) for a < A;  beta: X rows (a, y), B = L rows (b, w) of the batch
            EpiStrided ex{X + (pass ? 0 : b0 * v * n), n, 2.0 * alpha, 1.0, nullptr, nullptr};
            hipError_t e;
            if (!S) {
                e = launch_gemm<true, false, LADDER_STAGE_GEMM_F>(D, K, pass ? L + b0 * v * n : L, n, M, n, K, ex, st);
            } else {
                SlicedBuf lb = p.L_b;
                lb.K = nB * v;
                SplitShape sh{view(w, tl, 0), pass ? view(w, lb, 0) : view(w, p.L_bd, 0), M, n, K};
                sh.ksplit = choose_ksplit(S, M, n, K, p.a_skp_elems);
                sh.part = (double*)(w + p.a_skp);
                e = launch_split<LADDER_STAGE_GEMM_F>(S, sh, ex, st);
            }
            if ((rc = hip_check(e, "GEMM-F launch"))) return rc;
        }
    }
    return LADDER_OK;
}

// ------------------------------------------------------------ ragged batches
// ladder_batched runs every instance's forward and/or adjoint as parallel
// branches of one hipGraph.  Instances are dealt to branches longest first, each
// to the branch with the least nominal work so far (LPT), each branch owns one
// workspace slot and runs its instances in order, so up to `branches` instances
// share the GPU at a time.  The graph is captured on the first call with a given
// set of shapes, pointers and options and replayed afterwards.
constexpr int BATCH_BRANCHES = 4;
constexpr size_t BATCH_TILE_BYTES = size_t(4) << 30;  // default g/D tile per instance
constexpr size_t MAX_GRAPHS = 8;

struct BatchPlan {
    ladder_options op;
    std::vector<ladder_options> inst_opts;
    std::vector<int> branch_of;  // LPT assignment
    std::vector<int> order;      // launch order: longest first
    size_t slot = 0, total = 0;
    int branches = 0;
};

int batch_plan(int count, const ladder_instance* inst, uint32_t what, const ladder_options* opts, BatchPlan& bp) {
    int rc;
    if (count < 1 || !inst) return fail(LADDER_EINVAL, "count must be >= 1 and inst non-NULL");
    if (what == 0 || (what & ~(LADDER_DO_FORWARD | LADDER_DO_ADJOINT)))
        return fail(LADDER_EINVAL, "what must be a non-empty combination of LADDER_DO_FORWARD and LADDER_DO_ADJOINT");
    if ((rc = get_opts(opts, bp.op))) return rc;
    bp.inst_opts.resize(count);
    for (int i = 0; i < count; ++i) {
        const ladder_instance& x = inst[i];
        Sizes s;
        if ((rc = check_dims(x.o, x.v, x.n, s)) || (rc = check_split_dims(s, x.n, bp.op))) {
            g_last_error = "instance " + std::to_string(i) + ": " + g_last_error;
            return rc;
        }
        if (!x.L || !x.tau) return fail(LADDER_EINVAL, "instance %d: L and tau must be non-NULL", i);
        if ((what & LADDER_DO_FORWARD) && !x.R) return fail(LADDER_EINVAL, "instance %d: R is NULL", i);
        if ((what & LADDER_DO_ADJOINT) && (!x.X || !x.tbar)) return fail(LADDER_EINVAL, "instance %d: X and tbar are needed", i);
        if (x.E && !x.tbar) return fail(LADDER_EINVAL, "instance %d: E requested but tbar is NULL", i);
        ladder_options oi = bp.op;
        int64_t tuned = 0;
        if (oi.n_abatch == 0 && tuned_batch(tune_key(x.o, x.v, x.n, oi), tuned)) oi.n_abatch = tuned;
        if (oi.n_abatch == 0) {
            int64_t per_a = s.vvv * 8;
            if (oi.precision != LADDER_FP64)
                per_a += (int64_t)(slice_bytes(slice_spec(oi, std::max(oi.n_slices, oi.n_slices_adjoint)), x.v, s.vv) +
                                   exp_bytes(x.v, s.vv));
            oi.n_abatch = std::max<int64_t>(1, std::min<int64_t>((int64_t)(BATCH_TILE_BYTES / (size_t)per_a), (x.v + 1) / 2));
        }
        bp.inst_opts[i] = oi;
        const Plan p = make_plan(x.o, x.v, x.n, oi, s);
        bp.slot = std::max(bp.slot, align_up(p.total));
    }
    bp.branches = std::min(count, BATCH_BRANCHES);
    bp.total = bp.slot * (size_t)bp.branches;
    // longest processing time first onto the least loaded branch
    std::vector<double> work(count);
    for (int i = 0; i < count; ++i) {
        const double o = (double)inst[i].o, v = (double)inst[i].v, n = (double)inst[i].n;
        work[i] = v * v * v * v * (n + o * o);
    }
    bp.order.resize(count);
    for (int i = 0; i < count; ++i) bp.order[i] = i;
    std::stable_sort(bp.order.begin(), bp.order.end(), [&](int a, int b) { return work[a] > work[b]; });
    std::vector<double> load(bp.branches, 0.0);
    bp.branch_of.assign(count, 0);
    for (int i : bp.order) {
        const int b = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        bp.branch_of[i] = b;
        load[b] += work[i];
    }
    return LADDER_OK;
}

struct DeviceStreams {
    bool ready = false;
    hipStream_t cap = nullptr;
    hipStream_t branch[BATCH_BRANCHES] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[BATCH_BRANCHES] = {};
};
struct GraphEntry {
    std::vector<int64_t> key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};
std::mutex g_graph_mu;
std::vector<GraphEntry> g_graphs;
DeviceStreams g_streams[64];

// Library-owned streams (default priority) and events used only for capture.
int ensure_branch_streams(int dev) {
    if (dev < 0 || dev >= 64) return fail(LADDER_EUNSUPPORTED, "device index %d", dev);
    DeviceStreams& ds = g_streams[dev];
    if (ds.ready) return LADDER_OK;
    int rc;
    if ((rc = hip_check(hipStreamCreateWithFlags(&ds.cap, hipStreamNonBlocking), "stream create"))) return rc;
    if ((rc = hip_check(hipEventCreateWithFlags(&ds.fork, hipEventDisableTiming), "event create"))) return rc;
    for (int b = 0; b < BATCH_BRANCHES; ++b) {
        if ((rc = hip_check(hipStreamCreateWithFlags(&ds.branch[b], hipStreamNonBlocking), "stream create"))) return rc;
        if ((rc = hip_check(hipEventCreateWithFlags(&ds.join[b], hipEventDisableTiming), "event create"))) return rc;
    }
    ds.ready = true;
    return LADDER_OK;
}

// Forward ladder on validated arguments (ladder_forward, ladder_tau_gradient).
int forward_impl(int64_t o, int64_t v, int64_t n, const double* L, const double* tau, const double* tbar, double beta,
                 double* R, double* E, char* w, const Plan& p, const Sizes& s, hipStream_t st) {
    int rc;
    if (p.pm) return forward_pm(o, v, n, L, tau, tbar, beta, R, E, w, p, s, st);
    double* g = (double*)(w + p.tile_off);
    double* part = (double*)(w + p.part_off);
    const int S = p.S;
    if (S) {
        if ((rc = slice_into(S, false, L, n, w, p.L_J, st))) return rc;
        if ((rc = slice_into(S, false, tau, s.vv, w, p.tau_cd, st))) return rc;
    }
    for (int64_t bi = p.b_lo; bi < p.b_hi; ++bi) {
        const int64_t a0 = bi * p.nA;
        const int64_t nA = std::min(p.nA, v - a0);
        {
            StageTimer tm(LADDER_STAGE_GEMM_B, gemm_flops(nA * v, s.vv, n), gemm_bytes(nA * v, s.vv, n), st);
            EpiSwapMid eg{g, v, v, v, 1.0, 0.0};
            hipError_t e;
            if (!S) {
                e = launch_gemm<true, true, LADDER_STAGE_GEMM_B>(L + a0 * v * n, n, L, n, nA * v, s.vv, n, eg, st);
            } else {
                SplitShape sh{view(w, p.L_J, a0 * v), view(w, p.L_J, 0), nA * v, s.vv, n};
                e = launch_split<LADDER_STAGE_GEMM_B>(S, sh, eg, st);
            }
            if ((rc = hip_check(e, "GEMM-B launch"))) return rc;
        }
        if (S) {
            SlicedBuf tl = p.tile_sl;
            tl.R = nA * v;  // this batch's rows
            if ((rc = slice_into(S, false, g, s.vv, w, tl, st))) return rc;
        }
        {
            StageTimer tm(LADDER_STAGE_GEMM_C, gemm_flops(s.oo, nA * v, s.vv) + (E ? 2.0 * s.oo * nA * v : 0.0),
                          gemm_bytes(s.oo, nA * v, s.vv) + (E ? 8.0 * s.oo * nA * v : 0.0), st);
            EpiStrided er{R + a0 * v, s.vv, 1.0, beta, E ? tbar + a0 * v : nullptr, part + bi * p.part_per_batch};
            hipError_t e;
            if (!S) {
                e = launch_gemm<true, true, LADDER_STAGE_GEMM_C>(tau, s.vv, g, s.vv, s.oo, nA * v, s.vv, er, st);
            } else {
                SlicedBuf tl = p.tile_sl;
                tl.R = nA * v;
                SplitShape sh{view(w, p.tau_cd, 0), view(w, tl, 0), s.oo, nA * v, s.vv};
                e = launch_split<LADDER_STAGE_GEMM_C>(S, sh, er, st);
            }
            if ((rc = hip_check(e, "GEMM-C launch"))) return rc;
        }
    }
    if (E) {
        // Batch bi writes partial slots [bi*ppb, bi*ppb + tiles of its GEMM-C); every
        // batch but the last fills all ppb of them, so the slots in use are contiguous.
        const int64_t used_last = split_tiles(S, s.oo, (v - (p.nbatch - 1) * p.nA) * v);
        const int64_t count = (int64_t)p.part_per_batch * (p.nbatch - 1) + used_last;
        StageTimer tm(LADDER_STAGE_ENERGY, (double)count, 8.0 * (double)count, st);
        hipLaunchKernelGGL(reduce_partials_kernel, dim3(1), dim3(256), 0, st, part, count, E);
        if ((rc = hip_check(hipGetLastError(), "energy reduction launch"))) return rc;
    }
    return LADDER_OK;
}

// Shared argument checks of ladder_forward and ladder_tau_gradient: out (o^2 v^2
// doubles) must not overlap the inputs or the workspace.
int check_forward_args(int64_t o, int64_t v, int64_t n, const double* L, const double* x, const double* tbar, double* out,
                       double* E, void* ws, size_t ws_bytes, size_t need, const char* out_name, const Sizes& s) {
    if (!L || !x || !out || !ws) return fail(LADDER_EINVAL, "L, the amplitudes, %s and ws must be non-NULL", out_name);
    if (E && !tbar) return fail(LADDER_EINVAL, "E requested but tbar is NULL");
    if (!aligned8(L) || !aligned8(x) || !aligned8(out) || (tbar && !aligned8(tbar)) || (E && !aligned8(E)) ||
        ((uintptr_t)ws % ALIGN))
        return fail(LADDER_EINVAL, "misaligned pointer (arrays need 8-byte, ws 256-byte alignment)");
    if (ws_bytes < need) return fail(LADDER_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    const int64_t tb = s.ovv_elems * 8, lb = s.vvn * 8;
    if (overlap(out, tb, L, lb) || overlap(out, tb, x, tb) || overlap(out, tb, tbar, tb) ||
        overlap(out, tb, ws, (int64_t)ws_bytes))
        return fail(LADDER_EINVAL, "%s overlaps an input or the workspace", out_name);
    if (E && (overlap(E, 8, out, tb) || overlap(E, 8, ws, (int64_t)ws_bytes)))
        return fail(LADDER_EINVAL, "E overlaps %s or the workspace", out_name);
    (void)o; (void)v; (void)n;
    return LADDER_OK;
}

// LT[(c v + a) n + J] = L[(a v + c) n + J]: one workgroup per (a, c) row of n.
__global__ void transpose_pairs_kernel(const double* __restrict__ L, int64_t v, int64_t n, double* __restrict__ LT) {
    for (int64_t row = blockIdx.x; row < v * v; row += gridDim.x) {
        const int64_t a = row / v, c = row % v;
        const double* src = L + row * n;
        double* dst = LT + (c * v + a) * n;
        for (int64_t J = threadIdx.x; J < n; J += blockDim.x) dst[J] = src[J];
    }
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
    if ((rc = check_dims(o, v, n, s)) || (rc = get_opts(opts, op)) || (rc = check_split_dims(s, n, op))) return rc;
    *bytes = choose_plan(o, v, n, op, s, SIZE_MAX, true).total;
    return LADDER_OK;
}

int ladder_forward(int64_t o, int64_t v, int64_t n, const double* L, const double* tau, const double* tbar,
                   double beta, double* R, double* E, void* ws, size_t ws_bytes, const ladder_options* opts,
                   void* stream) {
    g_last_error.clear();
    Sizes s;
    ladder_options op;
    int rc;
    if ((rc = check_dims(o, v, n, s)) || (rc = get_opts(opts, op)) || (rc = check_split_dims(s, n, op))) return rc;
    const Plan p = choose_plan(o, v, n, op, s, ws_bytes, false);
    if ((rc = check_forward_args(o, v, n, L, tau, tbar, R, E, ws, ws_bytes, p.fwd_total, "R", s))) return rc;
    return forward_impl(o, v, n, L, tau, tbar, beta, R, E, (char*)ws, p, s, (hipStream_t)stream);
}

}  // extern "C"

namespace {
// Workspace of ladder_forward_noalloc: one file-scope device array.  Each GPU the
// library runs on holds its own copy from the load of the code object until the
// process ends.  In host code `scratch` is only a symbol: its device address is
// taken once per device with hipGetSymbolAddress and kept in g_scratch_ptr.
static __device__ __align__(256) char scratch[LADDER_STATIC_SCRATCH_BYTES];
std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};

// Device address of this device's `scratch` (looked up on the device's first call).
int scratch_address(void** out) {
    int dev = 0;
    int rc;
    if ((rc = hip_check(hipGetDevice(&dev), "hipGetDevice"))) return rc;
    if (dev < 0 || dev >= 64) return fail(LADDER_EUNSUPPORTED, "device index %d", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if ((rc = hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)"))) return rc;
        if (!p || ((uintptr_t)p % ALIGN)) return fail(LADDER_EHIP, "static scratch at an unaligned address %p", p);
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return LADDER_OK;
}

// Plan of ladder_forward_noalloc: an explicit n_abatch as given; otherwise the plan
// ladder_forward would choose if its forward region fits the static scratch, else the
// largest batch whose forward region fits.
int noalloc_plan(int64_t o, int64_t v, int64_t n, const ladder_options& op, const Sizes& s, Plan& p) {
    const size_t cap = LADDER_STATIC_SCRATCH_BYTES;
    p = choose_plan(o, v, n, op, s, cap, false);
    if (p.fwd_total <= cap) return LADDER_OK;
    if (op.n_abatch == 0) {
        for (int64_t nA = std::min(p.nA, v); nA >= 1; --nA) {
            ladder_options o2 = op;
            o2.n_abatch = nA;
            p = make_plan(o, v, n, o2, s);
            if (p.fwd_total <= cap) return LADDER_OK;
        }
    }
    return fail(LADDER_EWORKSPACE,
                "the forward needs %zu bytes of workspace (n_abatch %lld), more than the %zu of the static scratch",
                p.fwd_total, (long long)p.nA, cap);
}
}  // namespace

extern "C" {

int ladder_forward_noalloc(int64_t o, int64_t v, int64_t n, const double* L, const double* tau, const double* tbar,
                           double beta, double* R, double* E, const ladder_options* opts, void* stream) {
    g_last_error.clear();
    Sizes s;
    ladder_options op;
    int rc;
    if ((rc = check_dims(o, v, n, s)) || (rc = get_opts(opts, op)) || (rc = check_split_dims(s, n, op))) return rc;
    Plan p;
    if ((rc = noalloc_plan(o, v, n, op, s, p))) return rc;
    // the argument checks of ladder_forward, against a stand-in for the scratch range (its device
    // address is only looked up once the arguments are known to be valid)
    void* ws = nullptr;
    if ((rc = check_forward_args(o, v, n, L, tau, tbar, R, E, (void*)(uintptr_t)ALIGN, LADDER_STATIC_SCRATCH_BYTES,
                                 p.fwd_total, "R", s)))
        return rc;
    if ((rc = scratch_address(&ws))) return rc;
    const int64_t tb = s.ovv_elems * 8, lb = s.vvn * 8, sb = (int64_t)LADDER_STATIC_SCRATCH_BYTES;
    if (overlap(ws, sb, L, lb) || overlap(ws, sb, tau, tb) || overlap(ws, sb, tbar, tb) || overlap(ws, sb, R, tb) ||
        (E && overlap(ws, sb, E, 8)))
        return fail(LADDER_EINVAL, "an argument lies inside the library's static scratch");
    // no timing events in this call: it must not create host or device objects
    const bool was = g_capturing;
    g_capturing = true;
    rc = forward_impl(o, v, n, L, tau, tbar, beta, R, E, (char*)ws, p, s, (hipStream_t)stream);
    g_capturing = was;
    return rc;
}

int ladder_tau_gradient_workspace_size(int64_t o, int64_t v, int64_t n, const ladder_options* opts, size_t* bytes) {
    g_last_error.clear();
    if (!bytes) return fail(LADDER_EINVAL, "bytes is NULL");
    Sizes s;
    ladder_options op;
    int rc;
    if ((rc = check_dims(o, v, n, s)) || (rc = get_opts(opts, op)) || (rc = check_split_dims(s, n, op))) return rc;
    *bytes = align_up(choose_plan(o, v, n, op, s, SIZE_MAX, true).fwd_total) + align_up((size_t)s.vvn * 8);
    return LADDER_OK;
}

int ladder_tau_gradient(int64_t o, int64_t v, int64_t n, const double* L, const double* w, double beta, double* G,
                        void* ws, size_t ws_bytes, const ladder_options* opts, void* stream) {
    g_last_error.clear();
    Sizes s;
    ladder_options op;
    int rc;
    if ((rc = check_dims(o, v, n, s)) || (rc = get_opts(opts, op)) || (rc = check_split_dims(s, n, op))) return rc;
    // the transposed L sits after the forward region: pick the plan whose region leaves room for it
    Plan p = choose_plan(o, v, n, op, s, ws_bytes, false);
    if (align_up(p.fwd_total) + align_up((size_t)s.vvn * 8) > ws_bytes) p = make_plan(o, v, n, op, s);
    const size_t lt_off = align_up(p.fwd_total);
    const size_t need = lt_off + align_up((size_t)s.vvn * 8);
    if ((rc = check_forward_args(o, v, n, L, w, nullptr, G, nullptr, ws, ws_bytes, need, "G", s))) return rc;
    hipStream_t st = (hipStream_t)stream;
    double* LT = (double*)((char*)ws + lt_off);
    {
        StageTimer tm(LADDER_STAGE_PACK, 0.0, 16.0 * (double)s.vvn, st);
        hipLaunchKernelGGL(transpose_pairs_kernel, dim3((unsigned)std::min<int64_t>(s.vv, 1 << 20)), dim3(256), 0, st, L,
                           v, n, LT);
        if ((rc = hip_check(hipGetLastError(), "transpose launch"))) return rc;
    }
    return forward_impl(o, v, n, LT, w, nullptr, beta, G, nullptr, (char*)ws, p, s, st);
}

}  // extern "C"

namespace {

// Adjoint on validated arguments (ladder_adjoint, ladder_autotune).
int adjoint_impl(int64_t o, int64_t v, int64_t n, const double* L, const double* tau, const double* wt, double alpha,
                 double beta, double* X, char* w, const Plan& p, const Sizes& s, const ladder_options& op,
                 hipStream_t st) {
    int rc;
    if (p.pm) return adjoint_pm(o, v, n, L, tau, wt, alpha, beta, X, w, p, s, st);
    double* D = (double*)(w + p.tile_off);
    const bool general = (op.flags & LADDER_FLAG_GENERAL) != 0;
    double* pw = general ? (double*)(w + p.swap_off) : nullptr;
    double* pt = general ? pw + s.ovv_elems : nullptr;
    const int S = p.Sa;  // the adjoint's slice count
    if (general) {
        StageTimer tm(LADDER_STAGE_SWAP, 0.0, 32.0 * (double)s.ovv_elems, st);
        hipLaunchKernelGGL(pair_swap_kernel, dim3(grid_for(s.ovv_elems)), dim3(256), 0, st, wt, pw, o, v);
        hipLaunchKernelGGL(pair_swap_kernel, dim3(grid_for(s.ovv_elems)), dim3(256), 0, st, tau, pt, o, v);
        if ((rc = hip_check(hipGetLastError(), "pair swap launch"))) return rc;
    }
    if (S) {
        if ((rc = slice_into(S, true, wt, s.vv, w, p.w_ij, st))) return rc;
        if ((rc = slice_into(S, true, tau, s.vv, w, p.tau_ij, st))) return rc;
        if ((rc = slice_into(S, true, L, n, w, p.L_bd, st))) return rc;
        if (general) {
            if ((rc = slice_into(S, true, pw, s.vv, w, p.pw_ij, st))) return rc;
            if ((rc = slice_into(S, true, pt, s.vv, w, p.ptau_ij, st))) return rc;
        }
    }
    for (int64_t bi = p.b_lo; bi < p.b_hi; ++bi) {
        const int64_t a0 = bi * p.nA;
        const int64_t nA = std::min(p.nA, v - a0);
        for (int term = 0; term < (general ? 2 : 1); ++term) {
            StageTimer tm(LADDER_STAGE_GEMM_E, gemm_flops(nA * v, s.vv, s.oo), gemm_bytes(nA * v, s.vv, s.oo), st);
            EpiSwapMid ed{D, v, v, v, 1.0, term ? 1.0 : 0.0};
            hipError_t e;
            if (!S) {
                const double* wa = term ? pw : wt;
                const double* ta = term ? pt : tau;
                e = launch_gemm<false, false, LADDER_STAGE_GEMM_E>(wa + a0 * v, s.vv, ta, s.vv, nA * v, s.vv, s.oo, ed, st);
            } else {
                SplitShape sh{view(w, term ? p.pw_ij : p.w_ij, a0 * v), view(w, term ? p.ptau_ij : p.tau_ij, 0), nA * v,
                              s.vv, s.oo};
                e = launch_split<LADDER_STAGE_GEMM_E>(S, sh, ed, st);
            }
            if ((rc = hip_check(e, "GEMM-E launch"))) return rc;
        }
        if (S) {
            SlicedBuf tl = p.tile_sl;
            tl.R = nA * v;
            if ((rc = slice_into(S, false, D, s.vv, w, tl, st))) return rc;
        }
        {
            StageTimer tm(LADDER_STAGE_GEMM_F, gemm_flops(nA * v, n, s.vv), gemm_bytes(nA * v, n, s.vv), st);
            EpiStrided ex{X + a0 * v * n, n, general ? alpha : 2.0 * alpha, beta, nullptr, nullptr};
            hipError_t e;
            if (!S) {
                e = launch_gemm<true, false, LADDER_STAGE_GEMM_F>(D, s.vv, L, n, nA * v, n, s.vv, ex, st);
            } else {
                SlicedBuf tl = p.tile_sl;
                tl.R = nA * v;
                SplitShape sh{view(w, tl, 0), view(w, p.L_bd, 0), nA * v, n, s.vv};
                sh.ksplit = choose_ksplit(S, nA * v, n, s.vv, p.a_skp_elems);
                sh.part = (double*)(w + p.a_skp);
                e = launch_split<LADDER_STAGE_GEMM_F>(S, sh, ex, st);
            }
            if ((rc = hip_check(e, "GEMM-F launch"))) return rc;
        }
    }
    return LADDER_OK;
}

}  // namespace

extern "C" {

int ladder_adjoint(int64_t o, int64_t v, int64_t n, const double* L, const double* tau, const double* wt,
                   double alpha, double beta, double* X, void* ws, size_t ws_bytes, const ladder_options* opts,
                   void* stream) {
    g_last_error.clear();
    Sizes s;
    ladder_options op;
    int rc;
    if ((rc = check_dims(o, v, n, s)) || (rc = get_opts(opts, op)) || (rc = check_split_dims(s, n, op))) return rc;
    if (!L || !tau || !wt || !X || !ws) return fail(LADDER_EINVAL, "L, tau, w, X and ws must be non-NULL");
    if (!aligned8(L) || !aligned8(tau) || !aligned8(wt) || !aligned8(X) || ((uintptr_t)ws % ALIGN))
        return fail(LADDER_EINVAL, "misaligned pointer (arrays need 8-byte, ws 256-byte alignment)");
    const Plan p = choose_plan(o, v, n, op, s, ws_bytes, false);
    if (ws_bytes < p.adj_total) return fail(LADDER_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, p.adj_total);
    const int64_t tb = s.ovv_elems * 8, lb = s.vvn * 8;
    if (overlap(X, lb, L, lb) || overlap(X, lb, tau, tb) || overlap(X, lb, wt, tb) || overlap(X, lb, ws, (int64_t)ws_bytes))
        return fail(LADDER_EINVAL, "X overlaps an input or the workspace");
    return adjoint_impl(o, v, n, L, tau, wt, alpha, beta, X, (char*)ws, p, s, op, (hipStream_t)stream);
}

int ladder_autotune(int64_t o, int64_t v, int64_t n, const double* L, const double* tau, const double* tbar, double* R,
                    double* X, void* ws, size_t ws_bytes, const ladder_options* opts, const char* cache_path,
                    int64_t* n_abatch, void* stream) {
    g_last_error.clear();
    Sizes s;
    ladder_options op;
    int rc;
    if ((rc = check_dims(o, v, n, s)) || (rc = get_opts(opts, op)) || (rc = check_split_dims(s, n, op))) return rc;
    if (op.n_abatch != 0) return fail(LADDER_EINVAL, "autotune needs n_abatch = 0 (it chooses the batch size)");
    if (!tbar || !X) return fail(LADDER_EINVAL, "tbar and X must be non-NULL");
    const int64_t tb = s.ovv_elems * 8, lb = s.vvn * 8;
    if (!aligned8(X) || overlap(X, lb, L, lb) || overlap(X, lb, tau, tb) || overlap(X, lb, tbar, tb) ||
        overlap(X, lb, R, tb) || overlap(X, lb, ws, (int64_t)ws_bytes))
        return fail(LADDER_EINVAL, "X misaligned or overlapping an input, R or the workspace");
    const bool packed = !(op.flags & (LADDER_FLAG_GENERAL | LADDER_FLAG_DENSE));
    const bool general = (op.flags & LADDER_FLAG_GENERAL) != 0;
    const int64_t cap = std::max<int64_t>(1, packed ? (v + 3) / 4 : (v + 1) / 2);
    std::vector<int64_t> cand{make_plan(o, v, n, op, s).nA};
    for (int64_t c = 1; c < cap; c *= 2) cand.push_back(c);
    cand.push_back(cap);
    std::sort(cand.begin(), cand.end());
    cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
    std::vector<Plan> plans;
    for (int64_t c : cand) {
        ladder_options oc = op;
        oc.n_abatch = c;
        Plan p = make_plan(o, v, n, oc, s);
        if (p.total <= ws_bytes) plans.push_back(p);
    }
    if (plans.empty()) {
        const Plan p1 = make_plan(o, v, n, op, s);
        return fail(LADDER_EWORKSPACE, "workspace of %zu bytes fits no candidate (default needs %zu)", ws_bytes, p1.total);
    }
    if ((rc = check_forward_args(o, v, n, L, tau, tbar, R, nullptr, ws, ws_bytes, 0, "R", s))) return rc;
    hipStream_t st = (hipStream_t)stream;
    char* w = (char*)ws;
    hipEvent_t e0, e1;
    if ((rc = hip_check(hipEventCreate(&e0), "event create"))) return rc;
    if ((rc = hip_check(hipEventCreate(&e1), "event create"))) {
        (void)hipEventDestroy(e0);
        return rc;
    }
    // forward + adjoint over batches [b_lo, b_hi) of plan p; milliseconds
    auto timed = [&](Plan p, int64_t b_lo, int64_t b_hi, float& ms) -> int {
        p.b_lo = b_lo;
        p.b_hi = b_hi;
        int r;
        if ((r = hip_check(hipEventRecord(e0, st), "event record"))) return r;
        if ((r = forward_impl(o, v, n, L, tau, tbar, 0.0, R, nullptr, w, p, s, st))) return r;
        if ((r = adjoint_impl(o, v, n, L, tau, tbar, 1.0, 0.0, X, w, p, s, op, st))) return r;
        if ((r = hip_check(hipEventRecord(e1, st), "event record"))) return r;
        if ((r = hip_check(hipEventSynchronize(e1), "event sync"))) return r;
        return hip_check(hipEventElapsedTime(&ms, e0, e1), "event time");
    };
    float ms = 0.0f;
    double best_est = 0.0;
    int64_t best = plans[0].nA;
    rc = timed(plans[0], 0, std::min<int64_t>(1, plans[0].nbatch), ms);  // warm-up
    for (size_t i = 0; i < plans.size() && !rc; ++i) {
        const Plan& p = plans[i];
        float t_pro = 0.0f;
        if ((rc = timed(p, 0, 0, t_pro))) break;  // per-call work only (packing, slicing of the inputs)
        const int64_t samples[2] = {0, p.nbatch / 2};
        double t_s = 0.0, w_s = 0.0, w_all = 0.0;
        for (int k = 0; k < (p.nbatch > 1 ? 2 : 1); ++k) {
            if ((rc = timed(p, samples[k], samples[k] + 1, ms))) break;
            t_s += std::max(0.0, (double)ms - (double)t_pro);
            w_s += batch_work(p, o, v, n, s, general, samples[k]);
        }
        if (rc) break;
        for (int64_t b = 0; b < p.nbatch; ++b) w_all += batch_work(p, o, v, n, s, general, b);
        const double est = (double)t_pro + (w_s > 0.0 ? t_s / w_s * w_all : 0.0);
        if (i == 0 || est < best_est) {
            best_est = est;
            best = p.nA;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        g_tuned[tune_key(o, v, n, op)] = best;
        ++g_tune_gen;
    }
    if (n_abatch) *n_abatch = best;
    if (cache_path) {
        FILE* f = fopen(cache_path, "a");
        if (!f) return fail(LADDER_EINVAL, "cannot append to %s", cache_path);
        fprintf(f,
                "{\"device\": \"%s\", \"o\": %lld, \"v\": %lld, \"n\": %lld, \"precision\": %d, \"n_slices\": %d, "
                "\"n_slices_adjoint\": %d, \"flags\": %u, \"n_abatch\": %lld, \"est_ms\": %.1f}\n",
                device_tag().c_str(), (long long)o, (long long)v, (long long)n, (int)op.precision,
                op.precision != LADDER_FP64 ? (int)op.n_slices : 0,
                op.precision != LADDER_FP64 ? (int)op.n_slices_adjoint : 0, (unsigned)op.flags, (long long)best,
                best_est);
        fclose(f);
    }
    return LADDER_OK;
}

int ladder_autotune_load(const char* cache_path, int* n_loaded) {
    g_last_error.clear();
    if (!cache_path) return fail(LADDER_EINVAL, "cache_path is NULL");
    FILE* f = fopen(cache_path, "r");
    if (!f) return fail(LADDER_EINVAL, "cannot read %s", cache_path);
    const std::string dev = device_tag();
    char line[1024];
    int count = 0;
    auto field = [&](const char* key, long long& out) -> bool {
        const char* q = strstr(line, key);
        if (!q) return false;
        q = strchr(q + strlen(key), ':');
        return q && sscanf(q + 1, " %lld", &out) == 1;
    };
    while (fgets(line, sizeof line, f)) {
        const char* d = strstr(line, "\"device\"");
        const char* colon = d ? strchr(d + 8, ':') : nullptr;
        if (!colon) continue;
        const char* q1 = strchr(colon, '"');
        const char* q2 = q1 ? strchr(q1 + 1, '"') : nullptr;
        if (!q2 || std::string(q1 + 1, q2) != dev) continue;
        long long o = 0, v = 0, n = 0, prec = 0, sl = 0, fl = 0, nA = 0;
        if (!field("\"o\"", o) || !field("\"v\"", v) || !field("\"n\"", n) || !field("\"precision\"", prec) ||
            !field("\"n_slices\"", sl) || !field("\"flags\"", fl) || !field("\"n_abatch\"", nA) || nA < 1 || nA > v)
            continue;
        long long sla = sl;  // lines without the field: the adjoint uses the forward's count
        (void)field("\"n_slices_adjoint\"", sla);
        std::lock_guard<std::mutex> g(g_tune_mu);
        g_tuned[TuneKey{o, v, n, (int32_t)prec, (int32_t)sl, (int32_t)sla, (uint32_t)fl}] = nA;  // later lines win
        ++g_tune_gen;
        ++count;
    }
    fclose(f);
    if (n_loaded) *n_loaded = count;
    return LADDER_OK;
}

void ladder_autotune_reset(void) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tuned.clear();
    ++g_tune_gen;
}

int ladder_metric_contraction(int64_t v, int64_t n, const double* Z, const double* W, double alpha, double beta,
                              double* V, void* stream) {
    g_last_error.clear();
    if (v < 1 || n < 1 || v > 100000 || n > 1000000) return fail(LADDER_EINVAL, "bad dimensions v=%lld n=%lld", (long long)v, (long long)n);
    if (!Z || !W || !V) return fail(LADDER_EINVAL, "Z, W and V must be non-NULL");
    if (!aligned8(Z) || !aligned8(W) || !aligned8(V)) return fail(LADDER_EINVAL, "misaligned pointer (8-byte alignment)");
    const int64_t zb = v * v * n * 8, vb = n * n * 8;
    if (overlap(V, vb, Z, zb) || overlap(V, vb, W, zb)) return fail(LADDER_EINVAL, "V overlaps Z or W");
    hipStream_t st = (hipStream_t)stream;
    StageTimer tm(LADDER_STAGE_METRIC, gemm_flops(n, n, v * v), gemm_bytes(n, n, v * v), st);
    // A(M, pq) = Z[pq*n + M], B(pq, N) = W[pq*n + N]: both M/N-contiguous
    EpiStrided ev{V, n, alpha, beta, nullptr, nullptr};
    return hip_check(launch_gemm<false, false, LADDER_STAGE_METRIC>(Z, n, W, n, n, n, v * v, ev, st), "metric GEMM launch");
}

int ladder_back_transform_workspace_size(int64_t v, int64_t n, size_t* bytes) {
    g_last_error.clear();
    if (!bytes) return fail(LADDER_EINVAL, "bytes is NULL");
    if (v < 1 || n < 1 || v > 100000 || n > 1000000) return fail(LADDER_EINVAL, "bad dimensions v=%lld n=%lld", (long long)v, (long long)n);
    *bytes = align_up((size_t)(v * v * n) * 8);
    return LADDER_OK;
}

int ladder_back_transform(int64_t v, int64_t n, const double* x, const double* y, const double* W, double alpha,
                          double beta, double* Wmo, void* ws, size_t ws_bytes, void* stream) {
    g_last_error.clear();
    if (v < 1 || n < 1 || v > 100000 || n > 1000000) return fail(LADDER_EINVAL, "bad dimensions v=%lld n=%lld", (long long)v, (long long)n);
    if (!x || !y || !W || !Wmo || !ws) return fail(LADDER_EINVAL, "x, y, W, Wmo and ws must be non-NULL");
    if (!aligned8(x) || !aligned8(y) || !aligned8(W) || !aligned8(Wmo) || ((uintptr_t)ws % ALIGN))
        return fail(LADDER_EINVAL, "misaligned pointer (arrays need 8-byte, ws 256-byte alignment)");
    const size_t need = align_up((size_t)(v * v * n) * 8);
    if (ws_bytes < need) return fail(LADDER_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    const int64_t wb = v * v * n * 8, xb = v * v * 8;
    if (overlap(Wmo, wb, W, wb) || overlap(Wmo, wb, x, xb) || overlap(Wmo, wb, y, xb) ||
        overlap(Wmo, wb, ws, (int64_t)ws_bytes) || overlap(W, wb, ws, (int64_t)ws_bytes))
        return fail(LADDER_EINVAL, "Wmo or W overlaps another array or the workspace");
    hipStream_t st = (hipStream_t)stream;
    double* U = (double*)ws;
    StageTimer tm(LADDER_STAGE_BACKTRANSFORM, 2.0 * gemm_flops(v, v * n, v), 2.0 * gemm_bytes(v, v * n, v), st);
    // U[s][p][K] = sum_r x_rp W[r][s][K]: A(p, r) = x[r*v + p], B(r, (s,K)) = W[r*v*n + s*n + K]
    EpiSwapMid e1{U, v, v, n, 1.0, 0.0};
    hipError_t e = launch_gemm<false, false, LADDER_STAGE_BACKTRANSFORM>(x, v, W, v * n, v, v * n, v, e1, st);
    int rc;
    if ((rc = hip_check(e, "back-transform GEMM launch"))) return rc;
    // Wmo[p][q][K] = sum_s y_sq U[s][p][K]: A(q, s) = y[s*v + q], B(s, (p,K)) = U[s*v*n + p*n + K]
    EpiSwapMid e2{Wmo, v, v, n, alpha, beta};
    return hip_check(launch_gemm<false, false, LADDER_STAGE_BACKTRANSFORM>(y, v, U, v * n, v, v * n, v, e2, st),
                     "back-transform GEMM launch");
}

int ladder_metric_contraction_pairs(int64_t pairs, int64_t n, const double* Z, const double* W, double alpha,
                                    double beta, double* V, void* stream) {
    g_last_error.clear();
    if (pairs < 1 || n < 1 || pairs > (int64_t)1 << 40 || n > 1000000)
        return fail(LADDER_EINVAL, "bad dimensions pairs=%lld n=%lld", (long long)pairs, (long long)n);
    if (!Z || !W || !V) return fail(LADDER_EINVAL, "Z, W and V must be non-NULL");
    if (!aligned8(Z) || !aligned8(W) || !aligned8(V)) return fail(LADDER_EINVAL, "misaligned pointer (8-byte alignment)");
    int64_t zb;
    if (!mul_ok(pairs, n * 8, zb)) return fail(LADDER_EINVAL, "size overflow");
    const int64_t vb = n * n * 8;
    if (overlap(V, vb, Z, zb) || overlap(V, vb, W, zb)) return fail(LADDER_EINVAL, "V overlaps Z or W");
    hipStream_t st = (hipStream_t)stream;
    StageTimer tm(LADDER_STAGE_METRIC, gemm_flops(n, n, pairs), gemm_bytes(n, n, pairs), st);
    EpiStrided ev{V, n, alpha, beta, nullptr, nullptr};
    return hip_check(launch_gemm<false, false, LADDER_STAGE_METRIC>(Z, n, W, n, n, n, pairs, ev, st), "metric GEMM launch");
}

namespace {
// Workspace of ladder_ov3_abci: Lp [o][v][v][o], one [o][v][n] buffer (X, then P) and
// Zt [v][v][n], each 256-byte aligned.
struct Ov3Layout {
    size_t lp, xp, zt, total;
};
int ov3_layout(int64_t o, int64_t v, int64_t n, Ov3Layout& l) {
    Sizes s;
    int rc;
    if ((rc = check_dims(o, v, n, s))) return rc;
    int64_t ovn;
    if (!mul_ok(o * v, n, ovn) || ovn > INT64_MAX / 16) return fail(LADDER_EINVAL, "array sizes overflow 64-bit byte counts");
    // every GEMM grid (one workgroup per 128 x 128 tile) must fit a 32-bit launch
    const int64_t grid_max = (int64_t)1 << 31;
    if (tiles(o * v, n) >= grid_max || tiles(v, v * n) >= grid_max || tiles(o, v * n) >= grid_max)
        return fail(LADDER_EINVAL, "problem too large for one launch per GEMM");
    l.lp = 0;
    l.xp = align_up((size_t)s.ovv_elems * 8);
    l.zt = l.xp + align_up((size_t)ovn * 8);
    l.total = l.zt + align_up((size_t)s.vvn * 8);
    return LADDER_OK;
}
}  // namespace

int ladder_ov3_abci_workspace_size(int64_t o, int64_t v, int64_t n, size_t* bytes) {
    g_last_error.clear();
    if (!bytes) return fail(LADDER_EINVAL, "bytes is NULL");
    Ov3Layout l;
    int rc;
    if ((rc = ov3_layout(o, v, n, l))) return rc;
    *bytes = l.total;
    return LADDER_OK;
}

int ladder_ov3_abci(int64_t o, int64_t v, int64_t n, const double* L2, const double* R1, const double* Zvv,
                    const double* Zvo, double alpha, double beta, double* Wab, double* Wci, void* ws, size_t ws_bytes,
                    void* stream) {
    g_last_error.clear();
    Ov3Layout l;
    int rc;
    if ((rc = ov3_layout(o, v, n, l))) return rc;
    if (!L2 || !R1 || !ws) return fail(LADDER_EINVAL, "L2, R1 and ws must be non-NULL");
    if (!Wab && !Wci) return fail(LADDER_EINVAL, "Wab and Wci are both NULL: nothing to compute");
    if (Wab && !Zvo) return fail(LADDER_EINVAL, "Wab needs Zvo");
    if (Wci && !Zvv) return fail(LADDER_EINVAL, "Wci needs Zvv");
    if (!aligned8(L2) || !aligned8(R1) || !aligned8(Zvv) || !aligned8(Zvo) || !aligned8(Wab) || !aligned8(Wci) ||
        ((uintptr_t)ws % ALIGN))
        return fail(LADDER_EINVAL, "misaligned pointer (arrays need 8-byte, ws 256-byte alignment)");
    if (ws_bytes < l.total) return fail(LADDER_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, l.total);
    const int64_t l2b = o * o * v * v * 8, r1b = o * v * 8, vvb = v * v * n * 8, vob = v * o * n * 8;
    const int64_t wsb = (int64_t)ws_bytes;
    const void* ins[4] = {L2, R1, Zvv, Zvo};
    const int64_t inb[4] = {l2b, r1b, vvb, vob};
    for (int k = 0; k < 4; ++k)
        if (overlap(ins[k], inb[k], ws, wsb) || overlap(Wab, vvb, ins[k], inb[k]) || overlap(Wci, vob, ins[k], inb[k]))
            return fail(LADDER_EINVAL, "an input overlaps an output or the workspace");
    if (overlap(Wab, vvb, ws, wsb) || overlap(Wci, vob, ws, wsb) || overlap(Wab, vvb, Wci, vob))
        return fail(LADDER_EINVAL, "Wab or Wci overlaps the workspace or the other output");
    hipStream_t st = (hipStream_t)stream;
    char* w = (char*)ws;
    double* Lp = (double*)(w + l.lp);
    double* XP = (double*)(w + l.xp);
    double* Zt = (double*)(w + l.zt);
    const int64_t ov = o * v, vn = v * n;
    {
        StageTimer tm(LADDER_STAGE_OV3_PERMUTE, 0.0, 2.0 * (double)(l2b + (Wci ? vvb : 0)), st);
        const int64_t tiles = ov * ((o + 31) / 32) * ((v + 31) / 32);
        hipLaunchKernelGGL(ov3_permute_l2_kernel, dim3((unsigned)std::min<int64_t>(tiles, (int64_t)1 << 20)), dim3(256),
                           0, st, L2, Lp, o, v);
        if ((rc = hip_check(hipGetLastError(), "OV3 permutation launch"))) return rc;
        if (Wci) {
            hipLaunchKernelGGL(ov3_swap_vv_kernel, dim3((unsigned)std::min<int64_t>(v * v, (int64_t)1 << 20)), dim3(256),
                               0, st, Zvv, Zt, v, n);
            if ((rc = hip_check(hipGetLastError(), "OV3 permutation launch"))) return rc;
        }
    }
    const double fl = (Wab ? gemm_flops(ov, n, ov) + gemm_flops(v, vn, o) : 0.0) +
                      (Wci ? gemm_flops(o, vn, v) + gemm_flops(ov, n, ov) : 0.0);
    const double by = (Wab ? gemm_bytes(ov, n, ov) + gemm_bytes(v, vn, o) : 0.0) +
                      (Wci ? gemm_bytes(o, vn, v) + gemm_bytes(ov, n, ov) : 0.0);
    StageTimer tm(LADDER_STAGE_OV3, fl, by, st);
    if (Wab) {
        // X[j][a][K] = sum_(c,i) Lp[j][a][c][i] Zvo[c][i][K]  (X_aj^K of the table of intermediates)
        EpiStrided ex{XP, n, 1.0, 0.0, nullptr, nullptr};
        if ((rc = hip_check(launch_gemm<true, false, LADDER_STAGE_OV3>(Lp, ov, Zvo, n, ov, n, ov, ex, st), "OV3 GEMM launch")))
            return rc;
        // Wab[a][b][K] = beta Wab + alpha sum_j R1[j][b] X[j][a][K]: A(b, j) = R1[j*v + b],
        // B(j, (a,K)) = X[j*v*n + a*n + K]; the epilogue puts (b, (a,K)) at [a][b][K]
        EpiSwapMid ew{Wab, v, v, n, alpha, beta};
        if ((rc = hip_check(launch_gemm<false, false, LADDER_STAGE_OV3>(R1, v, XP, vn, v, vn, o, ew, st), "OV3 GEMM launch")))
            return rc;
    }
    if (Wci) {
        // P[j][a][K] = sum_b R1[j][b] Zt[b][a][K]  (P_aj^K of the table of intermediates)
        EpiStrided ep{XP, vn, 1.0, 0.0, nullptr, nullptr};
        if ((rc = hip_check(launch_gemm<true, false, LADDER_STAGE_OV3>(R1, v, Zt, vn, o, vn, v, ep, st), "OV3 GEMM launch")))
            return rc;
        // Wci[c][i][K] = beta Wci + alpha sum_(j,a) Lp[j][a][c][i] P[j][a][K]: A((c,i), (j,a)) is
        // (c,i)-contiguous with stride v*o between (j,a) rows
        EpiStrided ew{Wci, n, alpha, beta, nullptr, nullptr};
        if ((rc = hip_check(launch_gemm<false, false, LADDER_STAGE_OV3>(Lp, ov, XP, n, ov, n, ov, ew, st), "OV3 GEMM launch")))
            return rc;
    }
    return LADDER_OK;
}

namespace {
// Workspace of ladder_ov3_abic (every slot 256-byte aligned):
//   three o^2 v^2 buffers (reordered operands and the o^2 v^2 intermediates V+Y, Yt and the
//   amplitude matrices), B_iamn (o^3 v), the S_iacb slab of `g` occupied indices (g v^3),
//   Zt (v^2 n), eight [o][v][n] or [o][o][n] buffers, Xvv (v^2), W_am (o v), P^K and Q^K (n).
// Split precision adds the slices of the two operands of the o^3 v^3 GEMMs (rows
// o v, length o v; the slices of t along (mn) for S_iacb reuse the first one) and of one
// B_i.. block (rows v, length o^2).
struct AbicLayout {
    int64_t g;
    size_t bufA, bufB, bufC, Bm, S, Zt, Zvo, OX, Pp, Pk, PKI, KK, QY, YA, OA, Xvv, Wma, PK, QK, total;
    int slices = 0;  // 0: FP64
    SlicedBuf slA, slB, slT, slBm;
};
int abic_layout(int64_t o, int64_t v, int64_t n, const ladder_options* opts, AbicLayout& l) {
    Sizes s;
    ladder_options op;
    int rc;
    if ((rc = check_dims(o, v, n, s)) || (rc = get_opts(opts, op))) return rc;
    l.slices = slice_spec(op, op.n_slices);
    int64_t ovn, oon, ooov, vvv;
    if (!mul_ok(o * v, n, ovn) || !mul_ok(o * o, n, oon) || !mul_ok(o * o, o * v, ooov) || !mul_ok(s.vv, v, vvv) ||
        ovn > INT64_MAX / 16 || ooov > INT64_MAX / 16)
        return fail(LADDER_EINVAL, "array sizes overflow 64-bit byte counts");
    l.g = std::min<int64_t>(o, 8);
    const int64_t grid_max = (int64_t)1 << 31;
    const int64_t shapes[][2] = {{v, v}, {o * v, o * v}, {o * v, n}, {s.vv, n}, {o * o, n}, {v, v * n}, {o, v * n},
                                 {v, o * n}, {o, o * o * v}, {v, s.vv}, {l.g * v, n}, {1, n}};
    for (auto& sh : shapes)
        if (tiles(sh[0], sh[1]) >= grid_max) return fail(LADDER_EINVAL, "problem too large for one launch per GEMM");
    size_t off = 0;
    auto take = [&](size_t elems) {
        const size_t at = off;
        off += align_up(elems * 8);
        return at;
    };
    l.bufA = take((size_t)s.ovv_elems);
    l.bufB = take((size_t)s.ovv_elems);
    l.bufC = take((size_t)s.ovv_elems);
    l.Bm = take((size_t)ooov);
    l.S = take((size_t)(l.g * vvv));
    l.Zt = take((size_t)s.vvn);
    l.Zvo = take((size_t)ovn);
    l.OX = take((size_t)ovn);
    l.Pp = take((size_t)ovn);
    l.Pk = take((size_t)ovn);
    l.PKI = take((size_t)oon);
    l.KK = take((size_t)oon);
    l.QY = take((size_t)ovn);
    l.YA = take((size_t)ovn);
    l.OA = take((size_t)ovn);
    l.Xvv = take((size_t)s.vv);
    l.Wma = take((size_t)(o * v));
    l.PK = take((size_t)n);
    l.QK = take((size_t)n);
    if (l.slices) {
        const int64_t ov = o * v;
        // slicer grids and 32-bit panel offsets of the split GEMM (as for the ladder)
        if ((ov / 16 + 1) * split_nchunk(ov) >= (int64_t(1) << 31) || (s.vv / 32 + 1) * split_nchunk(o * o) >= (int64_t(1) << 31) ||
            2 * (split_kpad(std::max(ov, o * o)) / 16) * SPLIT_PANEL * 16 * 2 + 4096 >= (int64_t(1) << 32))
            return fail(LADDER_EUNSUPPORTED, "split precision: o v too large for the slicer grid or panel offsets");
        auto sliced = [&](int64_t R, int64_t K, size_t at) {
            SlicedBuf b;
            b.R = R;
            b.K = K;
            b.i8 = slice_is_i8(l.slices);
            b.s_off = at;
            b.e_off = at + align_up(slice_bytes(l.slices, R, K));
            return b;
        };
        const size_t a_b = align_up(slice_bytes(l.slices, ov, ov)) + align_up(exp_bytes(ov, ov));
        const size_t t_b = align_up(slice_bytes(l.slices, s.vv, o * o)) + align_up(exp_bytes(s.vv, o * o));
        const size_t r1 = off;
        off += std::max(a_b, t_b);
        l.slA = sliced(ov, ov, r1);
        l.slT = sliced(s.vv, o * o, r1);
        l.slB = sliced(ov, ov, off);
        off += a_b;
        l.slBm = sliced(v, o * o, off);
        off += align_up(slice_bytes(l.slices, v, o * o)) + align_up(exp_bytes(v, o * o));
    }
    l.total = off;
    return LADDER_OK;
}

// Launches permute4_kernel after checking that both stride sets stay inside `in_elems`.
int permute4(const double* in, int64_t in_elems, double* out, const Perm4& p, hipStream_t st) {
    int64_t hi1 = 0, hi2 = 0;
    for (int k = 0; k < 4; ++k) {
        if (p.D[k] < 1) return fail(LADDER_EINVAL, "empty reordering");
        hi1 += (p.D[k] - 1) * p.s[k];
        hi2 += (p.D[k] - 1) * p.t[k];
    }
    if (hi1 >= in_elems || (p.c2 != 0.0 && hi2 >= in_elems)) return fail(LADDER_EINVAL, "reordering out of range");
    const int64_t total = p.D[0] * p.D[1] * p.D[2] * p.D[3];
    hipLaunchKernelGGL(permute4_kernel, dim3(grid_for(total)), dim3(256), 0, st, in, out, p);
    return hip_check(hipGetLastError(), "reordering launch");
}
}  // namespace

int ladder_ov3_abic_workspace_size(int64_t o, int64_t v, int64_t n, const ladder_options* opts, size_t* bytes) {
    g_last_error.clear();
    if (!bytes) return fail(LADDER_EINVAL, "bytes is NULL");
    AbicLayout l;
    int rc;
    if ((rc = abic_layout(o, v, n, opts, l))) return rc;
    *bytes = l.total;
    return LADDER_OK;
}

int ladder_ov3_abic(int64_t o, int64_t v, int64_t n, double R0, const double* L1, const double* L2, const double* T,
                    const double* R1, const double* R2, const double* Zvv, const double* Zov, double alpha, double beta,
                    double* Wab, double* Wic, void* ws, size_t ws_bytes, const ladder_options* opts, void* stream) {
    g_last_error.clear();
    AbicLayout l;
    int rc;
    if ((rc = abic_layout(o, v, n, opts, l))) return rc;
    if (!L1 || !L2 || !T || !R1 || !R2 || !ws) return fail(LADDER_EINVAL, "L1, L2, T, R1, R2 and ws must be non-NULL");
    if (!Wab && !Wic) return fail(LADDER_EINVAL, "Wab and Wic are both NULL: nothing to compute");
    if (Wab && !Zov) return fail(LADDER_EINVAL, "Wab needs Zov");
    if (Wic && !Zvv) return fail(LADDER_EINVAL, "Wic needs Zvv");
    const void* ptrs[] = {L1, L2, T, R1, R2, Zvv, Zov, Wab, Wic};
    for (const void* q : ptrs)
        if (!aligned8(q)) return fail(LADDER_EINVAL, "misaligned pointer (8-byte alignment)");
    if ((uintptr_t)ws % ALIGN) return fail(LADDER_EINVAL, "misaligned workspace (256-byte alignment)");
    if (ws_bytes < l.total) return fail(LADDER_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, l.total);
    const int64_t ov = o * v, vv = v * v, on = o * n, vn = v * n, oo = o * o;
    const int64_t ovvb = oo * vv * 8, ovb = ov * 8, vvnb = vv * n * 8, ovnb = ov * n * 8, wsb = (int64_t)ws_bytes;
    const void* ins[] = {L1, L2, T, R1, R2, Zvv, Zov};
    const int64_t inb[] = {ovb, ovvb, ovvb, ovb, ovvb, vvnb, ovnb};
    for (int k = 0; k < 7; ++k)
        if (overlap(ins[k], inb[k], ws, wsb) || overlap(Wab, vvnb, ins[k], inb[k]) || overlap(Wic, ovnb, ins[k], inb[k]))
            return fail(LADDER_EINVAL, "an input overlaps an output or the workspace");
    if (overlap(Wab, vvnb, ws, wsb) || overlap(Wic, ovnb, ws, wsb) || overlap(Wab, vvnb, Wic, ovnb))
        return fail(LADDER_EINVAL, "Wab or Wic overlaps the workspace or the other output");

    hipStream_t st = (hipStream_t)stream;
    char* w = (char*)ws;
    auto at = [&](size_t off) { return (double*)(w + off); };
    double *bA = at(l.bufA), *bB = at(l.bufB), *bC = at(l.bufC), *Bm = at(l.Bm), *S = at(l.S), *Zt = at(l.Zt);
    double *Zvo = at(l.Zvo), *OX = at(l.OX), *Pp = at(l.Pp), *Pk = at(l.Pk), *PKI = at(l.PKI), *KK = at(l.KK);
    double *QY = at(l.QY), *YA = at(l.YA), *OA = at(l.OA), *Xvv = at(l.Xvv), *Wma = at(l.Wma), *PK = at(l.PK);
    double* QK = at(l.QK);
    const int64_t L2n = oo * vv;
    const bool ab = Wab != nullptr, ic = Wic != nullptr;
#define ABIC_GEMM(AK, BK, A_, lda, B_, ldb, M, N, K, epi)                                                         \
    do {                                                                                                           \
        if ((rc = hip_check(launch_gemm<AK, BK, LADDER_STAGE_OV3>(A_, lda, B_, ldb, M, N, K, epi, st),           \
                            "OV3 GEMM launch")))                                                                   \
            return rc;                                                                                             \
    } while (0)

    // ---- reorderings and the beta scaling of the outputs
    {
        StageTimer tm(LADDER_STAGE_OV3_PERMUTE, 0.0, 16.0 * (double)(ov * n + vv * n), st);
        if (ab) {
            if (beta == 0.0) hipLaunchKernelGGL(fill_zero_kernel, dim3(grid_for(vv * n)), dim3(256), 0, st, Wab, vv * n);
            else if (beta != 1.0) hipLaunchKernelGGL(scale_kernel, dim3(grid_for(vv * n)), dim3(256), 0, st, Wab, vv * n, beta);
            if ((rc = hip_check(hipGetLastError(), "scale launch"))) return rc;
            // Zvo[c][i][K] = Zov[i][c][K]
            if ((rc = permute4(Zov, ov * n, Zvo, Perm4{{1, v, o, n}, {0, n, vn, 1}, {0, 0, 0, 0}, 1.0, 0.0}, st))) return rc;
        }
        if (ic) {
            if (beta == 0.0) hipLaunchKernelGGL(fill_zero_kernel, dim3(grid_for(ov * n)), dim3(256), 0, st, Wic, ov * n);
            else if (beta != 1.0) hipLaunchKernelGGL(scale_kernel, dim3(grid_for(ov * n)), dim3(256), 0, st, Wic, ov * n, beta);
            if ((rc = hip_check(hipGetLastError(), "scale launch"))) return rc;
            // Zt[b][a][K] = Zvv[a][b][K]
            if ((rc = permute4(Zvv, vv * n, Zt, Perm4{{1, v, v, n}, {0, n, vn, 1}, {0, 0, 0, 0}, 1.0, 0.0}, st))) return rc;
        }
    }
    double fl = 0.0, by = 0.0;
    auto acct = [&](int64_t M, int64_t N, int64_t K) {
        fl += gemm_flops(M, N, K);
        by += gemm_bytes(M, N, K);
    };
    // C(m, n) = sum_k A[m*K + k] B[n*K + k] for the (o v)^3 products: FP64 MFMA, or both
    // operands sliced (INT8 or BF16) and the split GEMM (FP64 combine, same epilogue).
    auto rows_gemm = [&](const double* A_, const double* B_, int64_t M, int64_t N, int64_t K, const auto& epi) -> int {
        acct(M, N, K);
        if (!l.slices) return hip_check(launch_gemm<true, true, LADDER_STAGE_OV3>(A_, K, B_, K, M, N, K, epi, st),
                                        "OV3 GEMM launch");
        int r;
        if ((r = slice_into(l.slices, false, A_, K, w, l.slA, st)) || (r = slice_into(l.slices, false, B_, K, w, l.slB, st)))
            return r;
        SplitShape sh{view(w, l.slA, 0), view(w, l.slB, 0), M, N, K};
        return hip_check(launch_split<LADDER_STAGE_OV3>(l.slices, sh, epi, st), "OV3 split GEMM launch");
    };
    StageTimer tm(LADDER_STAGE_OV3, 0.0, 0.0, st);
    // ---- terms (3) and (8): X_ab = L_kl^ad t_kl^bd over rows a, b and columns (kl, d)
    if ((rc = permute4(L2, L2n, bA, Perm4{{1, v, oo, v}, {0, v, vv, 1}, {0, 0, 0, 0}, 1.0, 0.0}, st))) return rc;
    if ((rc = permute4(T, L2n, bB, Perm4{{1, v, oo, v}, {0, v, vv, 1}, {0, 0, 0, 0}, 1.0, 0.0}, st))) return rc;
    {
        EpiStrided e{Xvv, v, 1.0, 0.0, nullptr, nullptr};
        ABIC_GEMM(true, true, bA, oo * v, bB, oo * v, v, v, oo * v, e);
        acct(v, v, oo * v);
    }
    if (ab) {
        // (3): Wab += 2 alpha X_ab P^K, P^K = sum_ic R^c_i Z^K_ic
        EpiStrided e1{PK, n, 1.0, 0.0, nullptr, nullptr};
        ABIC_GEMM(true, false, R1, ov, Zov, n, 1, n, ov, e1);
        EpiStrided e2{Wab, n, 2.0 * alpha, 1.0, nullptr, nullptr};
        ABIC_GEMM(true, false, Xvv, 1, PK, n, vv, n, 1, e2);
        // (8): Wab -= alpha R^b_i O_ai^K, O_ai^K = sum_c X_ac Z^K_ic stored OX[i][a][K]
        EpiSwapMid e3{OX, v, o, n, 1.0, 0.0};
        ABIC_GEMM(true, false, Xvv, v, Zvo, on, v, on, v, e3);
        EpiSwapMid e4{Wab, v, v, n, -alpha, 1.0};
        ABIC_GEMM(false, false, R1, v, OX, vn, v, vn, o, e4);
        acct(1, n, ov); acct(vv, n, 1); acct(v, on, v); acct(v, vn, o);
    }
    if (ic) {
        // (3): Wic += 2 alpha R^c_i Q^K, Q^K = sum_ab X_ab Z^K_ab
        EpiStrided e1{QK, n, 1.0, 0.0, nullptr, nullptr};
        ABIC_GEMM(true, false, Xvv, vv, Zvv, n, 1, n, vv, e1);
        EpiStrided e2{Wic, n, 2.0 * alpha, 1.0, nullptr, nullptr};
        ABIC_GEMM(true, false, R1, 1, QK, n, ov, n, 1, e2);
        // (8): Wic -= alpha X_ac P_ai^K, P_ai^K = sum_b R^b_i Z^K_ab stored Pp[a][i][K]
        EpiSwapMid e3{Pp, o, v, n, 1.0, 0.0};
        ABIC_GEMM(true, false, R1, v, Zt, vn, o, vn, v, e3);
        EpiSwapMid e4{Wic, v, o, n, -alpha, 1.0};
        ABIC_GEMM(false, false, Xvv, v, Pp, on, v, on, v, e4);
        // Pk[k][a][K] for term (7)
        EpiStrided e5{Pk, vn, 1.0, 0.0, nullptr, nullptr};
        ABIC_GEMM(true, false, R1, v, Zt, vn, o, vn, v, e5);
        acct(1, n, vv); acct(ov, n, 1); acct(o, vn, v); acct(v, on, v); acct(o, vn, v);
    }
    // ---- term (4): VY[a][b][k][i] = V_akbi + Y_akbi
    //   V: rows (a,k) of L_lk^ae, columns (b,i) of t_li^be, summed over (l,e)
    if ((rc = permute4(L2, L2n, bA, Perm4{{v, o, o, v}, {v, vv, ov * v, 1}, {0, 0, 0, 0}, 1.0, 0.0}, st))) return rc;
    if ((rc = permute4(T, L2n, bB, Perm4{{v, o, o, v}, {v, vv, ov * v, 1}, {0, 0, 0, 0}, 1.0, 0.0}, st))) return rc;
    if ((rc = rows_gemm(bA, bB, ov, ov, ov, EpiSwapMid{bC, o, v, o, 1.0, 0.0}))) return rc;
    //   Y: rows (a,k) of L_kl^ad, columns (b,i) of t_il^bd, summed over (l,d)
    if ((rc = permute4(L2, L2n, bA, Perm4{{v, o, o, v}, {v, ov * v, vv, 1}, {0, 0, 0, 0}, 1.0, 0.0}, st))) return rc;
    if ((rc = permute4(T, L2n, bB, Perm4{{v, o, o, v}, {v, ov * v, vv, 1}, {0, 0, 0, 0}, 1.0, 0.0}, st))) return rc;
    if ((rc = rows_gemm(bA, bB, ov, ov, ov, EpiSwapMid{bC, o, v, o, 1.0, 1.0}))) return rc;
    if (ab) {
        // Wab -= alpha sum_ik VY[(a,b),(k,i)] P_ik^K, P_ik^K = sum_c R^c_k Z^K_ic stored PKI[k][i][K]
        EpiStrided e1{PKI, on, 1.0, 0.0, nullptr, nullptr};
        ABIC_GEMM(true, false, R1, v, Zvo, on, o, on, v, e1);
        EpiStrided e2{Wab, n, -alpha, 1.0, nullptr, nullptr};
        ABIC_GEMM(true, false, bC, oo, PKI, n, vv, n, oo, e2);
        acct(o, on, v); acct(vv, n, oo);
    }
    if (ic) {
        // Wic -= alpha sum_k R^c_k K_ik^K, K_ik^K = sum_ab VY[(a,b),(k,i)] Z^K_ab stored KK[k][i][K]
        EpiStrided e1{KK, n, 1.0, 0.0, nullptr, nullptr};
        ABIC_GEMM(false, false, bC, oo, Zvv, n, oo, n, vv, e1);
        EpiSwapMid e2{Wic, v, o, n, -alpha, 1.0};
        ABIC_GEMM(false, false, R1, v, KK, on, v, on, o, e2);
        acct(oo, n, vv); acct(v, on, o);
    }
    // ---- term (7): Yt[(k,a),(i,c)] = sum_me L_mk^ea (2 t_mi^ec - t_im^ec)
    if ((rc = permute4(L2, L2n, bA, Perm4{{o, v, o, v}, {vv, 1, ov * v, v}, {0, 0, 0, 0}, 1.0, 0.0}, st))) return rc;
    if ((rc = permute4(T, L2n, bB, Perm4{{o, v, o, v}, {vv, 1, ov * v, v}, {ov * v, 1, vv, v}, 2.0, -1.0}, st)))
        return rc;
    if ((rc = rows_gemm(bA, bB, ov, ov, ov, EpiStrided{bC, ov, 1.0, 0.0, nullptr, nullptr}))) return rc;
    if (ab) {
        // Wab += alpha sum_k R^b_k Q_ak^K, Q_ak^K = sum_ic Yt[(k,a),(i,c)] Z^K_ic stored QY[k][a][K]
        EpiStrided e1{QY, n, 1.0, 0.0, nullptr, nullptr};
        ABIC_GEMM(true, false, bC, ov, Zov, n, ov, n, ov, e1);
        EpiSwapMid e2{Wab, v, v, n, alpha, 1.0};
        ABIC_GEMM(false, false, R1, v, QY, vn, v, vn, o, e2);
        acct(ov, n, ov); acct(v, vn, o);
    }
    if (ic) {
        // Wic += alpha sum_(k,a) Yt[(k,a),(i,c)] P_ak^K
        EpiStrided e1{Wic, n, alpha, 1.0, nullptr, nullptr};
        ABIC_GEMM(false, false, bC, ov, Pk, n, ov, n, ov, e1);
        acct(ov, n, ov);
    }
    // ---- terms (1), (2) and (5): sum_m c[m][a] Amp[(m,b),(i,c)] with (c, Amp) = (L^a_m, A) and (W_am, t~_mi^bc)
    hipLaunchKernelGGL(abic_amp_kernel, dim3(grid_for(L2n)), dim3(256), 0, st, R0, T, R2, bA, o, v);
    if ((rc = hip_check(hipGetLastError(), "amplitude launch"))) return rc;
    if ((rc = permute4(T, L2n, bB, Perm4{{o, v, o, v}, {ov * v, v, vv, 1}, {vv, v, ov * v, 1}, 2.0, -1.0}, st)))
        return rc;
    hipLaunchKernelGGL(abic_wam_kernel, dim3((unsigned)std::min<int64_t>((ov + 3) / 4, 65536)), dim3(256), 0, st, L2, R1,
                       Wma, o, v);
    if ((rc = hip_check(hipGetLastError(), "W_am launch"))) return rc;
    const double* amps[2] = {bA, bB};
    const double* coef[2] = {L1, Wma};
    for (int t = 0; t < 2; ++t) {
        if (ab) {
            // YA[(m,b)][K] = sum_ic Amp[(m,b),(i,c)] Z^K_ic;  Wab[a][(b,K)] += alpha sum_m coef[m][a] YA[m][(b,K)]
            EpiStrided e1{YA, n, 1.0, 0.0, nullptr, nullptr};
            ABIC_GEMM(true, false, amps[t], ov, Zov, n, ov, n, ov, e1);
            EpiStrided e2{Wab, vn, alpha, 1.0, nullptr, nullptr};
            ABIC_GEMM(false, false, coef[t], v, YA, vn, v, vn, o, e2);
            acct(ov, n, ov); acct(v, vn, o);
        }
        if (ic) {
            // OA[m][(b,K)] = sum_a coef[m][a] Z^K_ab;  Wic[(i,c)][K] += alpha sum_(m,b) Amp[(m,b),(i,c)] OA[(m,b)][K]
            EpiStrided e1{OA, vn, 1.0, 0.0, nullptr, nullptr};
            ABIC_GEMM(true, false, coef[t], v, Zvv, vn, o, vn, v, e1);
            EpiStrided e2{Wic, n, alpha, 1.0, nullptr, nullptr};
            ABIC_GEMM(false, false, amps[t], ov, OA, n, ov, n, ov, e2);
            acct(o, vn, v); acct(ov, n, ov);
        }
    }
    // ---- term (6): -B_iamn t_mn^bc, B_iamn = sum_d L_mn^ad R^d_i stored Bm[i][(m,n)][a]
    {
        EpiStrided e{Bm, oo * v, 1.0, 0.0, nullptr, nullptr};
        ABIC_GEMM(true, true, R1, v, L2, v, o, oo * v, v, e);
        acct(o, oo * v, v);
    }
    if (l.slices && (rc = slice_into(l.slices, true, T, vv, w, l.slT, st))) return rc;  // rows (b,c), along (mn)
    for (int64_t i0 = 0; i0 < o; i0 += l.g) {
        const int64_t gl = std::min<int64_t>(l.g, o - i0);
        for (int64_t il = 0; il < gl; ++il) {
            // S[(a,b)][(il,c)] = sum_mn Bm[i][(m,n)][a] t_mn^bc
            EpiPlace e{S + il * v, 1, v, l.g * vv, 0, l.g * v, 1, 1.0, 0.0};
            const double* Bi = Bm + (i0 + il) * oo * v;
            if (l.slices) {
                if ((rc = slice_into(l.slices, true, Bi, v, w, l.slBm, st))) return rc;  // rows a, along (mn)
                SplitShape sh{view(w, l.slBm, 0), view(w, l.slT, 0), v, vv, oo};
                if ((rc = hip_check(launch_split<LADDER_STAGE_OV3>(l.slices, sh, e, st), "OV3 split GEMM launch")))
                    return rc;
            } else {
                ABIC_GEMM(false, false, Bi, v, T, vv, v, vv, oo, e);
            }
            acct(v, vv, oo);
        }
        if (ab) {
            EpiStrided e{Wab, n, -alpha, 1.0, nullptr, nullptr};
            ABIC_GEMM(true, false, S, l.g * v, Zov + i0 * vn, n, vv, n, gl * v, e);
            acct(vv, n, gl * v);
        }
        if (ic) {
            EpiStrided e{Wic + i0 * vn, n, -alpha, 1.0, nullptr, nullptr};
            ABIC_GEMM(false, false, S, l.g * v, Zvv, n, gl * v, n, vv, e);
            acct(gl * v, n, vv);
        }
    }
#undef ABIC_GEMM
    tm.rec.flops = fl;
    tm.rec.bytes = by;
    return LADDER_OK;
}

namespace {
// Workspace of ladder_gemm: the slices and exponents of A (M rows) and B (N rows) along K.
struct GemmLayout {
    SlicedBuf a, b;
    size_t total = 0;
};
int gemm_layout(int64_t M, int64_t N, int64_t K, const ladder_options& op, GemmLayout& l) {
    if (M < 1 || N < 1 || K < 1 || M > (int64_t(1) << 31) || N > (int64_t(1) << 31) || K > (int64_t(1) << 31))
        return fail(LADDER_EINVAL, "dimensions must be in [1, 2^31] (M=%lld N=%lld K=%lld)", (long long)M,
                    (long long)N, (long long)K);
    if ((M / F64_BM + 1) * (N / F64_BN + 1) >= (int64_t(1) << 31))
        return fail(LADDER_EINVAL, "M*N too large for one launch");
    if (op.precision == LADDER_FP64) return LADDER_OK;
    if ((std::max(M, N) / 16 + 1) * split_nchunk(K) >= (int64_t(1) << 31) ||
        2 * (split_kpad(K) / 16) * SPLIT_PANEL * 16 * 2 + 4096 >= (int64_t(1) << 32))
        return fail(LADDER_EUNSUPPORTED, "split precision: K or max(M, N) too large for the slicer grid or panel offsets");
    Arena a;
    l.a = take_sliced(a, slice_spec(op, op.n_slices), M, K);
    l.b = take_sliced(a, slice_spec(op, op.n_slices), N, K);
    l.total = a.top;
    return LADDER_OK;
}
}  // namespace

int ladder_gemm_workspace_size(int64_t M, int64_t N, int64_t K, const ladder_options* opts, size_t* bytes) {
    g_last_error.clear();
    if (!bytes) return fail(LADDER_EINVAL, "bytes is NULL");
    ladder_options op;
    GemmLayout l;
    int rc;
    if ((rc = get_opts(opts, op)) || (rc = gemm_layout(M, N, K, op, l))) return rc;
    *bytes = l.total;
    return LADDER_OK;
}

int ladder_gemm(int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda, const double* B,
                int64_t ldb, double beta, double* C, int64_t ldc, void* ws, size_t ws_bytes, const ladder_options* opts,
                void* stream) {
    g_last_error.clear();
    ladder_options op;
    GemmLayout l;
    int rc;
    if ((rc = get_opts(opts, op)) || (rc = gemm_layout(M, N, K, op, l))) return rc;
    if (!A || !B || !C) return fail(LADDER_EINVAL, "A, B and C must be non-NULL");
    if (lda < K || ldb < K || ldc < N) return fail(LADDER_EINVAL, "leading dimensions must be >= K (A, B) and >= N (C)");
    if (!aligned8(A) || !aligned8(B) || !aligned8(C)) return fail(LADDER_EINVAL, "misaligned pointer (8-byte alignment)");
    int64_t ab, bb, cb;
    if (!mul_ok(M - 1, lda, ab) || !mul_ok(N - 1, ldb, bb) || !mul_ok(M - 1, ldc, cb) || ab > INT64_MAX / 16 - K ||
        bb > INT64_MAX / 16 - K || cb > INT64_MAX / 16 - N)
        return fail(LADDER_EINVAL, "array sizes overflow 64-bit byte counts");
    ab = (ab + K) * 8;
    bb = (bb + K) * 8;
    cb = (cb + N) * 8;
    if (l.total) {
        if (!ws || ((uintptr_t)ws % ALIGN)) return fail(LADDER_EINVAL, "ws must be non-NULL and 256-byte aligned");
        if (ws_bytes < l.total) return fail(LADDER_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, l.total);
    }
    if (overlap(C, cb, A, ab) || overlap(C, cb, B, bb) || (l.total && overlap(C, cb, ws, (int64_t)ws_bytes)) ||
        (l.total && (overlap(A, ab, ws, (int64_t)ws_bytes) || overlap(B, bb, ws, (int64_t)ws_bytes))))
        return fail(LADDER_EINVAL, "C overlaps A, B or the workspace, or an input overlaps the workspace");
    hipStream_t st = (hipStream_t)stream;
    EpiStrided ep{C, ldc, alpha, beta, nullptr, nullptr};
    StageTimer tm(LADDER_STAGE_GEMM, gemm_flops(M, N, K), gemm_bytes(M, N, K), st);
    if (op.precision == LADDER_FP64)
        return hip_check(launch_gemm<true, true, LADDER_STAGE_GEMM>(A, lda, B, ldb, M, N, K, ep, st), "GEMM launch");
    char* w = (char*)ws;
    const int S = slice_spec(op, op.n_slices);
    if ((rc = slice_into(S, false, A, lda, w, l.a, st))) return rc;
    if ((rc = slice_into(S, false, B, ldb, w, l.b, st))) return rc;
    SplitShape sh{view(w, l.a, 0), view(w, l.b, 0), M, N, K};
    return hip_check(launch_split<LADDER_STAGE_GEMM>(S, sh, ep, st), "split GEMM launch");
}

int ladder_mfma_probe(int kind, int64_t iters, int64_t blocks, double* out, double* flops, void* stream) {
    g_last_error.clear();
    if (kind != LADDER_PROBE_BF16 && kind != LADDER_PROBE_FP64 && kind != LADDER_PROBE_INT8)
        return fail(LADDER_EUNSUPPORTED, "probe kind %d", kind);
    if (iters < 1 || iters > ((int64_t)1 << 32) || blocks < 1 || blocks > ((int64_t)1 << 20))
        return fail(LADDER_EINVAL, "iters must be in [1, 2^32] and blocks in [1, 2^20]");
    if (!out || !aligned8(out)) return fail(LADDER_EINVAL, "out must be a non-NULL 8-byte aligned device pointer");
    const double per = kind == LADDER_PROBE_BF16 ? 2.0 * 32 * 32 * 16 : kind == LADDER_PROBE_INT8 ? 2.0 * 32 * 32 * 32
                                                                                                : 2.0 * 16 * 16 * 4;
    if (flops) *flops = (double)blocks * 4.0 * (double)iters * 4.0 * per;  // 4 waves x 4 MFMAs per round
    hipStream_t st = (hipStream_t)stream;
    if (kind == LADDER_PROBE_BF16)
        hipLaunchKernelGGL(mfma_probe_kernel<0>, dim3((unsigned)blocks), dim3(256), 0, st, iters, out);
    else if (kind == LADDER_PROBE_INT8)
        hipLaunchKernelGGL(mfma_probe_kernel<2>, dim3((unsigned)blocks), dim3(256), 0, st, iters, out);
    else
        hipLaunchKernelGGL(mfma_probe_kernel<1>, dim3((unsigned)blocks), dim3(256), 0, st, iters, out);
    return hip_check(hipGetLastError(), "probe launch");
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
    return hip_check(launch_gemm<true, true, LADDER_STAGE_MP2>(Lov, n, Lov, n, o * v, o * v, n, ep, (hipStream_t)stream),
                     "amplitude GEMM launch");
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
    hipLaunchKernelGGL(amplitude_update_kernel, dim3(grid_for(s.ovv_elems)), dim3(256), 0, (hipStream_t)stream, eps, R,
                       t, o, v);
    return hip_check(hipGetLastError(), "amplitude update launch");
}

int ladder_excited_amplitudes(int64_t o, int64_t v, double R0, const double* T, const double* R2, int mode, double* U,
                              void* stream) {
    g_last_error.clear();
    Sizes s;
    int rc;
    if ((rc = check_dims(o, v, 1, s))) return rc;
    if (mode != LADDER_U_TABLE && mode != LADDER_U_APPENDIX) return fail(LADDER_EUNSUPPORTED, "mode %d", mode);
    if (!T || !R2 || !U) return fail(LADDER_EINVAL, "T, R2 and U must be non-NULL");
    if (!aligned8(T) || !aligned8(R2) || !aligned8(U)) return fail(LADDER_EINVAL, "misaligned pointer");
    const int64_t b = s.ovv_elems * 8;
    if (overlap(U, b, R2, b) || (U != T && overlap(U, b, T, b)))
        return fail(LADDER_EINVAL, "U overlaps R2 (or partially overlaps T)");
    StageTimer tm(LADDER_STAGE_UPDATE, 3.0 * (double)s.ovv_elems, 24.0 * (double)s.ovv_elems, (hipStream_t)stream);
    hipLaunchKernelGGL(excited_amplitudes_kernel, dim3(grid_for(s.ovv_elems)), dim3(256), 0, (hipStream_t)stream, R0, T,
                       R2, mode, U, o, v);
    return hip_check(hipGetLastError(), "excited amplitudes launch");
}

int ladder_batched_workspace_size(int count, const ladder_instance* inst, uint32_t what, const ladder_options* opts,
                                  size_t* bytes) {
    g_last_error.clear();
    if (!bytes) return fail(LADDER_EINVAL, "bytes is NULL");
    BatchPlan bp;
    int rc = batch_plan(count, inst, what, opts, bp);
    if (rc) return rc;
    *bytes = bp.total;
    return LADDER_OK;
}

int ladder_batched(int count, const ladder_instance* inst, uint32_t what, void* ws, size_t ws_bytes,
                   const ladder_options* opts, void* stream) {
    g_last_error.clear();
    BatchPlan bp;
    int rc = batch_plan(count, inst, what, opts, bp);
    if (rc) return rc;
    if (!ws || ((uintptr_t)ws % ALIGN)) return fail(LADDER_EINVAL, "ws must be non-NULL and 256-byte aligned");
    if (ws_bytes < bp.total) return fail(LADDER_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, bp.total);

    // Cache key: everything the captured launches depend on.
    int64_t gen;
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        gen = g_tune_gen;
    }
    std::vector<int64_t> key = {count, (int64_t)what, (int64_t)(uintptr_t)ws, (int64_t)ws_bytes, bp.op.precision,
                                bp.op.n_slices, bp.op.n_slices_adjoint, bp.op.n_abatch, (int64_t)bp.op.flags, gen};
    for (int i = 0; i < count; ++i) {
        const ladder_instance& x = inst[i];
        for (int64_t f : {x.o, x.v, x.n, (int64_t)(uintptr_t)x.L, (int64_t)(uintptr_t)x.tau, (int64_t)(uintptr_t)x.tbar,
                          (int64_t)(uintptr_t)x.R, (int64_t)(uintptr_t)x.E, (int64_t)(uintptr_t)x.X})
            key.push_back(f);
    }
    std::lock_guard<std::mutex> lk(g_graph_mu);
    int dev = 0;
    if ((rc = hip_check(hipGetDevice(&dev), "hipGetDevice"))) return rc;
    key.push_back(dev);
    GraphEntry* hit = nullptr;
    for (auto& e : g_graphs)
        if (e.key == key) hit = &e;
    if (!hit) {
        if ((rc = ensure_branch_streams(dev))) return rc;
        DeviceStreams& ds = g_streams[dev];
        GraphEntry e;
        e.key = key;
        hipStream_t cap = ds.cap;
        if ((rc = hip_check(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal), "graph capture begin"))) return rc;
        g_capturing = true;
        int brc = hip_check(hipEventRecord(ds.fork, cap), "fork event");
        for (int b = 0; b < bp.branches && !brc; ++b) brc = hip_check(hipStreamWaitEvent(ds.branch[b], ds.fork, 0), "fork wait");
        for (int k = 0; k < count && !brc; ++k) {
            const int i = bp.order[k];
            const ladder_instance& x = inst[i];
            const int b = bp.branch_of[i];
            char* slot = (char*)ws + (size_t)b * bp.slot;
            if (what & LADDER_DO_FORWARD)
                brc = ladder_forward(x.o, x.v, x.n, x.L, x.tau, x.tbar, 0.0, x.R, x.E, slot, bp.slot, &bp.inst_opts[i],
                                     ds.branch[b]);
            if (!brc && (what & LADDER_DO_ADJOINT))
                brc = ladder_adjoint(x.o, x.v, x.n, x.L, x.tau, x.tbar, 1.0, 0.0, x.X, slot, bp.slot, &bp.inst_opts[i],
                                     ds.branch[b]);
        }
        for (int b = 0; b < bp.branches && !brc; ++b) {
            brc = hip_check(hipEventRecord(ds.join[b], ds.branch[b]), "join event");
            if (!brc) brc = hip_check(hipStreamWaitEvent(cap, ds.join[b], 0), "join wait");
        }
        g_capturing = false;
        const std::string err = g_last_error;
        hipGraph_t graph = nullptr;
        const hipError_t ec = hipStreamEndCapture(cap, &graph);
        if (brc) {
            if (graph) (void)hipGraphDestroy(graph);
            g_last_error = "while capturing the batch: " + err;
            return brc;
        }
        if ((rc = hip_check(ec, "graph capture end"))) return rc;
        hipGraphExec_t exec = nullptr;
        if ((rc = hip_check(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "graph instantiate"))) {
            (void)hipGraphDestroy(graph);
            return rc;
        }
        e.graph = graph;
        e.exec = exec;
        if (g_graphs.size() >= MAX_GRAPHS) {
            (void)hipGraphExecDestroy(g_graphs.front().exec);
            (void)hipGraphDestroy(g_graphs.front().graph);
            g_graphs.erase(g_graphs.begin());
        }
        g_graphs.push_back(e);
        hit = &g_graphs.back();
    }
    return hip_check(hipGraphLaunch(hit->exec, (hipStream_t)stream), "graph launch");
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
    {
        std::lock_guard<std::mutex> gl(g_graph_mu);
        for (auto& e : g_graphs) {
            (void)hipGraphExecDestroy(e.exec);
            (void)hipGraphDestroy(e.graph);
        }
        g_graphs.clear();
        for (auto& ds : g_streams) {
            if (!ds.ready) continue;
            (void)hipStreamDestroy(ds.cap);
            (void)hipEventDestroy(ds.fork);
            for (int b = 0; b < BATCH_BRANCHES; ++b) {
                (void)hipStreamDestroy(ds.branch[b]);
                (void)hipEventDestroy(ds.join[b]);
            }
            ds = DeviceStreams{};
        }
    }
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (auto& r : g_prof) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    g_prof.clear();
    g_prof_on = false;
}

}  // extern "C"
