/*
 * ladder.h -- C ABI of libladder.so: the V^4 O^2 particle-particle ladder of
 * Cholesky-decomposed CCSD and its adjoint, on one AMD Instinct MI355X (gfx950).
 *
 * Quantities (Schnack-Petersen, Koch, Coriani, Kjonstad, arXiv 2202.02019):
 *   L^J_pq   Cholesky vectors, (pq|rs) = sum_J L^J_pq L^J_rs          (Sec. II A)
 *   g_acbd = sum_J L^J_ac L^J_bd, the (ac|bd) integrals, formed per virtual
 *            batch on the device and never stored whole                (Sec. II B)
 *   R_ij^ab = sum_cd g_acbd tau_ij^cd, the A2 ladder term of Omega       (Sec. II B)
 *   E       = sum_ijab tbar_ij^ab R_ij^ab, the V^4 part of sum g d with the
 *             ground-state density d_abcd = O^(2)_abcd(L_2 = tbar, C_2 = tau)
 *                                                                     (Appendix A)
 *   X^J_ac  = dE/dL^J_ac = 2 sum_bd L^J_bd D_{ab,cd},  D_{ab,cd} = sum_ij tbar_ij^ab tau_ij^cd,
 *             i.e. 2 W~^J_ac (Sec. II C) restricted to the V^4 density block
 *             (Sec. II B); the factor 2 is d_pqrs = d_rspq (Appendix A).
 *
 * Index ranges: i,j < o (occupied), a,b,c,d < v (virtual), J < n (Cholesky).
 *
 * Layouts (row-major FP64, all DEVICE pointers owned by the caller):
 *   L, X      [v][v][n]     L[(a*v + c)*n + J]            = L^J_ac
 *   tau, tbar, R, w
 *             [o][o][v][v]  tau[((i*o + j)*v + c)*v + d]  = tau_ij^cd
 *   Lov       [o][v][n]     Lov[(i*v + a)*n + J]           = L^J_ia
 *   eps       [o + v]       occupied orbital energies first, then virtual ones
 *   E         one double on the device
 *
 * Conventions.
 *   * Every call is asynchronous on `stream` (a hipStream_t; NULL = the null
 *     stream).  Results are valid once the stream has been synchronised.
 *   * The library never allocates device memory in these calls: scratch space is
 *     the caller's `ws` buffer (device memory of `ws_bytes` bytes, 256-byte
 *     aligned), sized with ladder_workspace_size().  It holds only per-batch
 *     tiles of g or D (n_abatch * v^3 doubles), never the whole v^4 array.
 *   * Pair symmetry: the library assumes tau_ij^ab = tau_ji^ba and
 *     tbar_ij^ab = tbar_ji^ba (true for closed-shell CCSD amplitudes) unless
 *     LADDER_FLAG_GENERAL is set.  With it, the default path packs the
 *     contractions into symmetric and antisymmetric parts (the strategy the
 *     paper adapts from Scuseria et al. in Sec. II B): the forward O^2 V^4
 *     product runs on i<=j, a<=b, c<=d (1/4 of the dense work) and the density
 *     on i<=j, c<=d (1/2).  LADDER_FLAG_DENSE selects the unpacked contraction;
 *     LADDER_FLAG_GENERAL forms the second density term explicitly and is
 *     always dense.
 *   * L need not be symmetric in (a,c) (T1-transformed vectors are not).
 *   * Results are deterministic: no floating-point atomics; the same inputs and
 *     options give bitwise identical R, E and X.
 *
 * Errors.  Every entry point validates all arguments on the host before any
 * launch and returns LADDER_OK (0) or a negative code; on error nothing has been
 * launched and no output has been touched.  ladder_strerror() names a code,
 * ladder_last_error() gives the message of the last failure on this thread
 * (including the HIP error string for LADDER_EHIP).
 */
#ifndef LADDER_H
#define LADDER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LADDER_OK 0
#define LADDER_EINVAL (-1)       /* null pointer, non-positive or too-large size, misalignment, aliasing */
#define LADDER_EWORKSPACE (-2)   /* ws too small for the requested batch */
#define LADDER_EUNSUPPORTED (-3) /* option value outside the supported range */
#define LADDER_EHIP (-4)         /* HIP launch or runtime failure */

/* Arithmetic of the four contraction stages. */
#define LADDER_FP64 0       /* FP64 MFMA (v_mfma_f64_16x16x4_f64) throughout */
#define LADDER_SPLIT_BF16 1 /* exponent-aligned BF16 slices on BF16 MFMA, exact FP32 chunk sums, FP64 combine */
#define LADDER_SPLIT_INT8 2 /* exponent-aligned INT8 slices (7 bits each) on INT8 MFMA, exact INT32 level sums,
                               FP64 combine */

/* Option flags. */
#define LADDER_FLAG_GENERAL 1u /* adjoint: do not assume pair symmetry of tau and tbar (implies DENSE) */
#define LADDER_FLAG_DENSE 2u   /* contract all (i,j), (a,b), (c,d): skip the +/- packing */

typedef struct {
    int32_t precision;        /* LADDER_FP64, LADDER_SPLIT_BF16 or LADDER_SPLIT_INT8 */
    int32_t n_slices;         /* split modes: slices per operand of the forward's GEMMs (the g tile and
                                 the R update) and of every other split product; 0 = the default, 5 for
                                 BF16 and 6 for INT8 (the counts that meet 1e-10 in E); otherwise 2..6 */
    int64_t n_abatch;         /* virtual indices a per batch, 0 = automatic */
    uint32_t flags;           /* LADDER_FLAG_* */
    int32_t n_slices_adjoint; /* split mode: slices of the adjoint's GEMMs (the density tile and the X
                                 update); 0 = n_slices, otherwise 2..6; ignored (normalised to 0) in FP64 */
} ladder_options;

/* Defaults: precision FP64, automatic batch, no flags.  `opts` may be NULL in
 * every call below, meaning these defaults. */
void ladder_default_options(ladder_options* opts);

/*
 * Bytes of device workspace that ladder_forward / ladder_adjoint need for the
 * shape (o, v, n) and options (the larger of the two).  With n_abatch = 0 the
 * batch is the largest that keeps the per-batch g/D tile (with its packed
 * halves on the +/- path) at or below LADDER_DEFAULT_TILE_BYTES and covers at
 * most half of the virtual range (a quarter on the +/- path), so no v^4-sized
 * array is ever held.
 */
#define LADDER_DEFAULT_TILE_BYTES ((size_t)16 << 30)
int ladder_workspace_size(int64_t o, int64_t v, int64_t n, const ladder_options* opts, size_t* bytes);

/*
 * Forward ladder (A2 term, Sec. II B) and its energy.
 *   R = beta * R + ladder(L, tau)        R_ij^ab (+)= sum_cd (sum_J L^J_ac L^J_bd) tau_ij^cd
 *   *E = sum_ijab tbar_ij^ab * ladder(L, tau)_ij^ab   (if E != NULL; needs tbar)
 * With beta == 0, R is not read (it may hold NaN).  tbar may be NULL only when E
 * is NULL.  R must not overlap L, tau, tbar or ws.
 */
int ladder_forward(int64_t o, int64_t v, int64_t n, const double* L, const double* tau,
                   const double* tbar, double beta, double* R, double* E, void* ws,
                   size_t ws_bytes, const ladder_options* opts, void* stream);

/*
 * ladder_forward for callers that cannot allocate (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): the same computation
 * and arguments as ladder_forward, without ws/ws_bytes.  Its workspace is a
 * static device array of LADDER_STATIC_SCRATCH_BYTES inside the library, one
 * per GPU (held from the library's first use on that GPU until the process
 * ends); the call itself allocates nothing (no hipMalloc, no events, no
 * library routine that allocates).  With n_abatch = 0 it runs the plan
 * ladder_forward would run if that plan's workspace fits the array, else the
 * largest virtual batch that fits; an explicit n_abatch is used as given.
 * Returns LADDER_EWORKSPACE, before any launch, when even that does not fit
 * (the packed amplitudes take about 4 o^2 v^2 bytes, 9 o^2 v^2 with five BF16
 * slices and 7 o^2 v^2 with six INT8 ones, and the batch tile about 16 v^3 bytes
 * per virtual index on the default +/- path; INT8 plans also hold up to 16 K-split
 * partial tiles of the R update).  Every call on one GPU uses that GPU's one array and leaves its
 * contents behind (nothing in it needs clearing between calls): calls that
 * overlap on one GPU (two streams, two threads) race and must be serialised by
 * the caller.  No argument may lie inside the array.
 */
#define LADDER_STATIC_SCRATCH_BYTES ((size_t)256 << 20)
int ladder_forward_noalloc(int64_t o, int64_t v, int64_t n, const double* L, const double* tau,
                           const double* tbar, double beta, double* R, double* E,
                           const ladder_options* opts, void* stream);

/*
 * Adjoint: the L-built three-index intermediate of the V^4 block.
 *   X = beta * X + alpha * d/dL [ sum_ijab w_ij^ab ladder(L, tau)_ij^ab ]
 *     = beta * X + alpha * 2 sum_bd L^J_bd sum_ij w_ij^ab tau_ij^cd      (pair-symmetric)
 * With w = tbar this is dE/dL (Sec. II B V^4 density O^(2), Sec. II C W~).  With
 * LADDER_FLAG_GENERAL the second term sum_ij w_ij^ba tau_ij^dc is formed
 * explicitly instead of being folded into the factor 2 (costs one more density
 * GEMM and 2*o^2*v^2 doubles of extra workspace).  With beta == 0, X is not read.
 * X must not overlap L, tau, w or ws.
 */
int ladder_adjoint(int64_t o, int64_t v, int64_t n, const double* L, const double* tau,
                   const double* w, double alpha, double beta, double* X, void* ws,
                   size_t ws_bytes, const ladder_options* opts, void* stream);

/*
 * Autotuner for the virtual-batch size (the batch of Sec. II B, whose size the
 * paper leaves open).  For this shape and these options (n_abatch must be 0) it
 * times, on the caller's data and stream, each candidate batch size whose
 * workspace fits ws_bytes: the default one, powers of two and the cap (v/4 on the
 * +/- path, v/2 otherwise).  Each candidate runs the per-call work alone and two
 * sample batches (the first and the middle one) of forward + adjoint; the whole
 * call is estimated from the modelled GEMM work of every batch.  The fastest is
 * kept in a process-wide table, returned in *n_abatch (if not NULL) and, when
 * cache_path is not NULL, appended to that file as one JSON line.  R and X are
 * overwritten with partial results (tbar is used as the adjoint weight).
 * From then on, calls with n_abatch = 0 for the same (o, v, n, precision,
 * n_slices, flags) use the tuned size whenever its workspace fits the one they are
 * given, and ladder_workspace_size / ladder_batched_workspace_size report the
 * larger of the tuned and default workspaces.  Synchronises the stream.
 * ladder_autotune_load reads such a file (lines of other devices are skipped,
 * later lines win; *n_loaded = lines taken, may be NULL); ladder_autotune_reset
 * forgets every tuned entry.
 */
int ladder_autotune(int64_t o, int64_t v, int64_t n, const double* L, const double* tau, const double* tbar,
                    double* R, double* X, void* ws, size_t ws_bytes, const ladder_options* opts,
                    const char* cache_path, int64_t* n_abatch, void* stream);
int ladder_autotune_load(const char* cache_path, int* n_loaded);
void ladder_autotune_reset(void);

/*
 * Transposed ladder: the gradient of the ladder energy with respect to the
 * amplitudes, i.e. the A2-term contribution to the multiplier equations
 * (tbar A = -eta, Sec. II A):
 *   G = beta * G + d/dtau [ sum_ijab w_ij^ab ladder(L, tau)_ij^ab ]
 *   G_ij^cd (+)= sum_ab w_ij^ab (sum_J L^J_ac L^J_bd)
 * This is ladder_forward applied to w with every L^J replaced by its transpose
 * (L^J_ac -> L^J_ca); the library writes that transpose into the workspace, so
 * the call needs ladder_tau_gradient_workspace_size bytes (the forward workspace
 * plus v^2 n doubles).  Options as for ladder_forward (the default +/- path needs
 * pair-symmetric w, for which G is pair-symmetric too).  With beta == 0, G is
 * not read.  G must not overlap L, w or ws.
 */
int ladder_tau_gradient_workspace_size(int64_t o, int64_t v, int64_t n, const ladder_options* opts,
                                       size_t* bytes);
int ladder_tau_gradient(int64_t o, int64_t v, int64_t n, const double* L, const double* w, double beta,
                        double* G, void* ws, size_t ws_bytes, const ladder_options* opts, void* stream);

/*
 * Gradient intermediates of Sec. II A built from the V^4 density block.
 *
 * W: ladder_adjoint called with Z in place of L and alpha = 1/2 returns
 *   W^K_ac = sum_bd d_acbd Z^K_bd,   d_acbd = sum_ij w_ij^ab tau_ij^cd,
 * the three-index density intermediate W^K_pq = sum_rs d_pqrs Z^K_rs restricted
 * to the virtual-virtual block (Z^K_rs = sum_L (S^-1)_KL (L|rs), layout [v][v][n]
 * like L; pair-symmetric amplitudes, or LADDER_FLAG_GENERAL, which returns the
 * average of sum_rs d_pqrs Z_rs and sum_rs d_rspq Z_rs).
 *
 * ladder_metric_contraction: the two-index intermediate
 *   V = beta * V + alpha * V',  V'_MN = sum_pq Z^M_pq W^N_pq      (V: [n][n], row M)
 * over the v^2 virtual pairs given (one FP64 MFMA GEMM, M = N = n, K = v^2).
 * V must not overlap Z or W.  With beta == 0, V is not read.
 */
int ladder_metric_contraction(int64_t v, int64_t n, const double* Z, const double* W, double alpha,
                              double beta, double* V, void* stream);

/*
 * MO back-transformation of the three-index intermediate (Sec. II A, applied
 * before the contraction with the differentiated MO integrals):
 *   Wmo = beta * Wmo + alpha * Wmo',  Wmo'^K_pq = sum_rs x_rp y_sq W^K_rs
 * for the virtual-virtual block: x, y are [v][v] row-major (x[r*v + p] = x_rp),
 * W and Wmo [v][v][n].  Two FP64 MFMA GEMMs (2 v^3 n flops each) through a
 * [v][v][n] intermediate in the workspace (ladder_back_transform_workspace_size
 * bytes, 256-byte aligned).  Wmo must not overlap x, y, W or ws.  With
 * beta == 0, Wmo is not read.
 */
int ladder_back_transform_workspace_size(int64_t v, int64_t n, size_t* bytes);
int ladder_back_transform(int64_t v, int64_t n, const double* x, const double* y, const double* W,
                          double alpha, double beta, double* Wmo, void* ws, size_t ws_bytes,
                          void* stream);

/*
 * Excited-state doubles amplitudes U for the excited-state V^4 density
 * d^es_abcd = O^(2)_abcd(L_2, U) (Appendix A), from the ground-state T_2, the
 * excited-state R_2 and the reference weight R_0.  The paper defines U twice:
 *   LADDER_U_TABLE    (0): U = T_2 R_0 + R_2                  (table of intermediates, Sec. II B)
 *   LADDER_U_APPENDIX (1): U = T_2 R_0 / 2 + Rt_2, Rt_ij^ab = R_ij^ab (1 + [i = j][a = b])
 *                          (Appendix A; Rt_2 is its R~_2, the doubles expanded over all
 *                          (ai, bj) with the diagonal ones counted twice)
 * The excited-state V^4 contribution to the three-index intermediate is then
 * ladder_adjoint(Z or L, U, L_2).  U may equal T (in place) but must not overlap
 * R2.  Pair-symmetric T and R2 give pair-symmetric U in both modes.  FP64.
 */
#define LADDER_U_TABLE 0
#define LADDER_U_APPENDIX 1
int ladder_excited_amplitudes(int64_t o, int64_t v, double R0, const double* T, const double* R2, int mode,
                              double* U, void* stream);

/*
 * Excited-state OV^3 density block d_abci = sum_j L_ji^ac R_j^b (Appendix A,
 * excited-state densities; it vanishes in the ground state) and its two
 * contributions to the three-index intermediate W^K_pq = sum_rs d_pqrs Z^K_rs
 * (Sec. II B, contributions of the OV^3 densities), built through the
 * intermediates of the table in Sec. II B without forming the density:
 *   X_aj^K = sum_ci L_ji^ac Z^K_ci,   Wab^K_ab = beta Wab + alpha sum_j R_j^b X_aj^K
 *   P_aj^K = sum_b R_j^b Z^K_ab,      Wci^K_ci = beta Wci + alpha sum_aj L_ji^ac P_aj^K
 * Layouts (row-major FP64, device): L2 [o][o][v][v] (L2[((j*o+i)*v+a)*v+c] =
 * L_ji^ac, like tau); R1 [o][v] (R1[j*v+b] = R_j^b); Zvv, Wab [v][v][n] (like L);
 * Zvo, Wci [v][o][n] (Zvo[(c*o+i)*n+K] = Z^K_ci).  Either output may be NULL to
 * skip that side (Wab needs Zvo, Wci needs Zvv; the other may then be NULL).
 * With beta == 0 the outputs are not read.  Four FP64 MFMA GEMMs,
 * 4 o^2 v^2 n + 4 o v^2 n flops for both sides, after a reordering of L2 (and of
 * Zvv for Wci) into the workspace: ladder_ov3_abci_workspace_size bytes, 256-byte
 * aligned, (o^2 v^2 + o v n + v^2 n) doubles.  No input may overlap an output or
 * the workspace; the outputs may not overlap each other.  The V_MN partner is
 * ladder_metric_contraction (ab side) plus ladder_metric_contraction_pairs over
 * the v*o pairs of the ci side.
 */
int ladder_ov3_abci_workspace_size(int64_t o, int64_t v, int64_t n, size_t* bytes);
int ladder_ov3_abci(int64_t o, int64_t v, int64_t n, const double* L2, const double* R1, const double* Zvv,
                    const double* Zvo, double alpha, double beta, double* Wab, double* Wci, void* ws, size_t ws_bytes,
                    void* stream);

/*
 * Excited-state OV^3 density block d_abic (Appendix A, excited-state densities)
 * and its two contributions to the three-index intermediate (Sec. II B):
 *   Wab^K_ab = beta Wab + alpha sum_ic d_abic Z^K_ic,  Wic^K_ic = beta Wic + alpha sum_ab d_abic Z^K_ab,
 *   d_abic = R_0 L^a_m t~_im^cb + L^a_m (2 R~_mi^bc - R~_mi^cb) + 2 X_ab R^c_i
 *          - (V_akbi + Y_akbi) R^c_k + L_mk^ad t~_mi^bc R^d_k - L_mn^ad t_mn^bc R^d_i
 *          + Yt_akci R^b_k - X_ac R^b_i
 * with t~_ij^ab = 2 t_ij^ab - t_ji^ab, R~_ij^ab = R_ij^ab (1 + [i=j][a=b]) and the
 * intermediates X_ab = L_kl^ad t_kl^bd, V_akbi = L_lk^ae t_li^be, Y_akbi = L_kl^ad t_il^bd,
 * Yt_akci = L_mk^ea t~_mi^ec of Sec. II B and Appendix A (C_2 = t).  The density is
 * never formed: each term is contracted through its own intermediates (the o^3 v^3
 * ones, V + Y, Yt and S_iacb = B_iamn t_mn^bc, are FP64 MFMA GEMMs; S is formed for
 * eight occupied indices at a time).  Inputs (device, row-major FP64): L1, R1 [o][v]
 * (L1[m*v+a] = L^a_m); L2, T, R2 [o][o][v][v] (L2[((i*o+j)*v+a)*v+b] = L_ij^ab);
 * Zvv, Wab [v][v][n]; Zov, Wic [o][v][n] (Zov[(i*v+c)*n+K] = Z^K_ic).  Either output
 * may be NULL to skip that side (Wab needs Zov, Wic needs Zvv).  With beta == 0 the
 * outputs are not read.  opts (may be NULL: FP64) selects the precision of the three
 * o^3 v^3 products V+Y, Yt and S: LADDER_FP64, or LADDER_SPLIT_BF16 / LADDER_SPLIT_INT8
 * with n_slices slices (the split GEMM of the ladder, FP64 combine); everything else is FP64;
 * n_abatch and flags are ignored.  Workspace: ladder_ov3_abic_workspace_size bytes
 * for the same opts, 256-byte aligned (three o^2 v^2 buffers, o^3 v, 8 v^3, v^2 n and
 * a few [o][v][n] arrays; split adds the slices of two o v x o v operands).
 * No input may overlap an output or the workspace; the outputs may not overlap.
 */
int ladder_ov3_abic_workspace_size(int64_t o, int64_t v, int64_t n, const ladder_options* opts, size_t* bytes);
int ladder_ov3_abic(int64_t o, int64_t v, int64_t n, double R0, const double* L1, const double* L2, const double* T,
                    const double* R1, const double* R2, const double* Zvv, const double* Zov, double alpha, double beta,
                    double* Wab, double* Wic, void* ws, size_t ws_bytes, const ladder_options* opts, void* stream);

/*
 * ladder_metric_contraction over any number of index pairs (the two-index
 * intermediate V_MN = Z^M_ab W^N_ab + Z^M_ci W^N_ci of Sec. II B has a
 * virtual-occupied part):  V = beta * V + alpha * sum_p Z[p][M] W[p][N], with
 * Z and W [pairs][n] and V [n][n].  V must not overlap Z or W; with beta == 0
 * it is not read.
 */
int ladder_metric_contraction_pairs(int64_t pairs, int64_t n, const double* Z, const double* W, double alpha,
                                    double beta, double* V, void* stream);

/*
 * First-order doubles amplitudes from the occupied-virtual Cholesky block (the
 * synthetic stand-in for converged T2; Cholesky expansion of Sec. II A):
 *   t_ij^ab = (sum_J L^J_ia L^J_jb) / ((eps_i + eps_j) - (eps_a + eps_b)).
 * FP64 throughout.  t must not overlap Lov or eps.
 */
int ladder_mp2_amplitudes(int64_t o, int64_t v, int64_t n, const double* Lov, const double* eps,
                          double* t, void* stream);

/*
 * Orbital-energy-denominator (Jacobi) amplitude update, FP64:
 *   t_ij^ab += R_ij^ab / ((eps_i + eps_j) - (eps_a + eps_b)).
 * R may equal t only if the caller wants t <- t + t/den.
 */
int ladder_amplitude_update(int64_t o, int64_t v, const double* eps, const double* R, double* t,
                            void* stream);

/* One instance of a ragged batch (all device pointers; tbar/E and X optional). */
typedef struct {
    int64_t o, v, n;
    const double* L;
    const double* tau;
    const double* tbar;
    double* R; /* forward output (overwritten), may be NULL if not LADDER_DO_FORWARD */
    double* E; /* energy (device scalar), may be NULL */
    double* X; /* adjoint output (overwritten), may be NULL if not LADDER_DO_ADJOINT */
} ladder_instance;

#define LADDER_DO_FORWARD 1u
#define LADDER_DO_ADJOINT 2u

/* Workspace for ladder_batched over `count` instances. */
int ladder_batched_workspace_size(int count, const ladder_instance* inst, uint32_t what,
                                  const ladder_options* opts, size_t* bytes);

/*
 * Many independent instances of uneven (o, v, n): forward (R = ladder, E) and/or
 * adjoint (X = dE/dL with w = tbar, pair-symmetric) for each, in one launch
 * sequence captured once into a hipGraph and replayed on later calls with the
 * same shapes, pointers and options.  `inst` is a host array.
 */
int ladder_batched(int count, const ladder_instance* inst, uint32_t what, void* ws, size_t ws_bytes,
                   const ladder_options* opts, void* stream);

/*
 * The contraction primitive of the four ladder stages (the g tile, the R update,
 * the density tile and the X update are each one such product), exposed alone:
 *   C = beta * C + alpha * A B^T,   C_mn (+)= sum_k A_mk B_nk
 * A [M][K] (row stride lda >= K), B [N][K] (row stride ldb >= K), C [M][N] (row
 * stride ldc >= N): row-major FP64 device arrays owned by the caller.
 * opts->precision LADDER_FP64 runs v_mfma_f64_16x16x4_f64 (no workspace);
 * LADDER_SPLIT_BF16 cuts A and B along k into n_slices exponent-aligned BF16
 * slices in the workspace (one exponent per row and 256-long chunk of k) and
 * runs the pairs p + q < n_slices on v_mfma_f32_32x32x16_bf16 with exact FP32
 * chunk sums folded into FP64, so integer inputs that n_slices slices carry
 * exactly give the exact product as long as every chunk sum fits FP32's 24
 * bits (the representation used by every split stage of the ladder).
 * LADDER_SPLIT_INT8 does the same with 7-bit integer slices on
 * v_mfma_i32_32x32x32_i8, one exact INT32 sum per slice level p + q and chunk
 * (no chunk-sum limit), folded into FP64.
 * ladder_gemm_workspace_size gives the bytes (0 for FP64); ws must then be
 * 256-byte aligned.  With beta == 0, C is not read.  C must not overlap A, B or
 * ws, and A and B must not overlap ws.  n_abatch and flags are ignored.
 * M, N, K in [1, 2^31].  Asynchronous on `stream`.
 */
int ladder_gemm_workspace_size(int64_t M, int64_t N, int64_t K, const ladder_options* opts, size_t* bytes);
int ladder_gemm(int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda, const double* B,
                int64_t ldb, double beta, double* C, int64_t ldc, void* ws, size_t ws_bytes,
                const ladder_options* opts, void* stream);

/*
 * Matrix-core ceiling probe (measurement support): `blocks` workgroups of four
 * waves each issue `iters` rounds of four independent MFMAs on register operands
 * and write one checksum per thread to out[blocks * 256] (device, caller-owned).
 * LADDER_PROBE_BF16 runs v_mfma_f32_32x32x16_bf16 (the split GEMM's instruction),
 * LADDER_PROBE_FP64 v_mfma_f64_16x16x4_f64 (the FP64 GEMM's), LADDER_PROBE_INT8
 * v_mfma_i32_32x32x32_i8 (the INT8 split GEMM's).  *flops (host, may be NULL) receives
 * the flops (integer operations for INT8) of the launch; timing it gives the rate the chip sustains
 * under its clock and power limits, beside the published peaks.  Asynchronous on
 * `stream`.  iters in [1, 2^32], blocks in [1, 2^20].
 */
#define LADDER_PROBE_BF16 0
#define LADDER_PROBE_FP64 1
#define LADDER_PROBE_INT8 2
int ladder_mfma_probe(int kind, int64_t iters, int64_t blocks, double* out, double* flops, void* stream);

/*
 * Per-stage timing with HIP events (for measurement, off by default).
 * ladder_profile_start() clears the record and makes every later kernel launch
 * of this library bracketed by two hipEvents recorded on the launch stream.
 * ladder_profile_stop() synchronises those events, fills up to `max_stages`
 * entries of `out` (one per stage that ran; *n_out receives the count) and
 * turns recording off.  Stage ids are LADDER_STAGE_*; `flops` and `bytes` are
 * the algorithmic work of all launches of the stage (2*M*N*K for a GEMM; for
 * bytes, each operand element read once and each result written once).
 */
#define LADDER_STAGE_GEMM_B 0   /* g tile, K = n */
#define LADDER_STAGE_GEMM_C 1   /* R update, K = v^2 */
#define LADDER_STAGE_ENERGY 2   /* energy partial reduction */
#define LADDER_STAGE_GEMM_E 3   /* D tile, K = o^2 */
#define LADDER_STAGE_GEMM_F 4   /* X update, K = v^2 */
#define LADDER_STAGE_SWAP 5     /* pair swap (general adjoint) */
#define LADDER_STAGE_MP2 6      /* first-order amplitudes */
#define LADDER_STAGE_UPDATE 7   /* amplitude update */
#define LADDER_STAGE_SLICE 8    /* split mode: FP64 -> BF16 slices */
#define LADDER_STAGE_PACK 9     /* +/- packing of tau, tbar and the g tile */
#define LADDER_STAGE_UNPACK 10  /* R and D rebuilt from their packed parts */
#define LADDER_STAGE_METRIC 11  /* V = Z^T W (three-index to two-index intermediate) */
#define LADDER_STAGE_BACKTRANSFORM 12 /* MO back-transformation of W */
#define LADDER_STAGE_OV3_PERMUTE 13 /* OV^3 block: multiplier and Z reorderings */
#define LADDER_STAGE_OV3 14     /* OV^3 block: the four GEMMs of W_ab and W_ci */
#define LADDER_STAGE_GEMM 15    /* ladder_gemm, the contraction primitive alone */
#define LADDER_NUM_STAGES 16
typedef struct {
    int32_t stage;
    int32_t launches;
    double total_ms;
    double flops;
    double bytes;
} ladder_stage_stats;
int ladder_profile_start(void);
int ladder_profile_stop(ladder_stage_stats* out, int max_stages, int* n_out);

/* Name of an error code; never NULL. */
const char* ladder_strerror(int code);
/* Message of the last failing call on this thread ("" if none). */
const char* ladder_last_error(void);
/* Frees host-side caches (instantiated graphs).  Safe to call more than once. */
void ladder_shutdown(void);

#ifdef __cplusplus
}
#endif
#endif /* LADDER_H */
