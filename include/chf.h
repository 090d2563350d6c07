/*
 * chf.h -- C ABI of the MI355X (gfx950) library for fourth-kind Chebyshev
 * smoothing with block-FSAI preconditioners inside a Galerkin V-cycle.
 *
 * Problem statement (paper Sec. 2, Def. 2.1 and Def. 2.2): A is symmetric
 * positive definite with a uniform block structure of n block rows of size b;
 * a factor pattern is lower block-triangular and contains the diagonal
 * (Eq. lower_triangular_pattern).
 *
 * Conventions for every call:
 *  - Return value: CHF_OK (0) or a negative chf_status; chf_last_error()
 *    returns a thread-local message describing the last failure.
 *  - Host arrays are read during the call only and never retained.
 *  - Device vectors are caller-owned buffers on the current HIP device;
 *    handles own their device memory and free it in the matching *_destroy.
 *    At block size 10 the products read vectors in pairs, so a vector that
 *    enters a product must start on a 16-byte (double) or 8-byte (float)
 *    boundary, as hipMalloc'd and torch buffers do; other addresses are
 *    rejected with CHF_EINVAL.
 *  - `stream` is the caller's HIP stream (0 = null stream). A call returns
 *    after enqueueing work, except where a scalar must come back to the host
 *    (PCG stop test, Lanczos, set-up calls), which synchronise `stream`.
 *  - Block indices are 0-based; block b x b values are row-major and
 *    contiguous; BSR column indices ascend within each row.
 *  - Vector element types follow the operator's working dtype: CHF_F64 ->
 *    double, CHF_F32 and CHF_BF16 (BF16 factor storage) -> float.
 *
 * Tuning overrides, read from the environment (results stay within the
 * parity bounds of every setting; they exist for tests and measurement):
 *  - CHF_FSAI_CONFIG="<width>,<tile threshold>[,<rr threshold>]": the local
 *    solver of chf_fsai_setup (width 64, 128 or 256; rows wider than the tile
 *    threshold use the tiled MFMA solver, 0 = never; local systems wider than
 *    the rr threshold, up to 240, use the register-resident MFMA kernel,
 *    absent = never) instead of the autotuned choice.
 *  - CHF_SPMV_SPLIT_BELOW=<slices>: SpMV layouts with fewer slices use one
 *    workgroup per slice (default 2048; 0 = never).
 *  - CHF_SPMV_NONTEMPORAL=0: plain instead of non-temporal matrix loads
 *    (read once per process).
 *  - CHF_AI_WG_PER_CU=<n>: at most n rows of chf_pattern_adaptive in flight
 *    per compute unit (default: as many as LDS and registers allow).
 */
#ifndef CHF_H
#define CHF_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CHF_OK = 0,
    CHF_EINVAL = -1,      /* bad argument, malformed pattern, non-finite input */
    CHF_ENOMEM = -2,      /* device allocation failed */
    CHF_ENOTSPD = -3,     /* a local (or coarse) Cholesky pivot was not positive */
    CHF_EDEVICE = -4,     /* HIP runtime error */
    CHF_ENOCONV = -5,     /* PCG did not reach rtol within maxit */
    CHF_EBREAKDOWN = -6   /* PCG breakdown: p^T A p <= 0 or r^T z <= 0 */
} chf_status;

/* Storage and working precision. CHF_F64, CHF_F32, CHF_BF16 name a storage
 * type (and, as a working mode: FP64 throughout; FP32 A with FP32 vectors and
 * G in FP32 or BF16). CHF_F64_BF16G is a working mode only: A, vectors and
 * arithmetic in FP64 with the factor G read from its BF16 copy (a factor set
 * up with g_store = CHF_BF16 keeps both copies). It is accepted by the
 * smoothers, chf_fsai_apply, chf_lmax_lanczos and chf_level_opts.dtype, where
 * it builds every level's G with BF16 storage. */
typedef enum { CHF_F64 = 0, CHF_F32 = 1, CHF_BF16 = 2, CHF_F64_BF16G = 3 } chf_dtype;
typedef enum { CHF_SMOOTH_CHEB4 = 0, CHF_SMOOTH_CHEB1 = 1, CHF_SMOOTH_RICHARDSON = 2 } chf_smoother;
typedef enum { CHF_CYCLE_VKK = 0, CHF_CYCLE_V2K0 = 1 } chf_cycle;

typedef struct chf_bsr_s* chf_bsr;
typedef struct chf_pattern_s* chf_pattern;
typedef struct chf_fsai_s* chf_fsai;
typedef struct chf_levels_s* chf_levels;
typedef struct chf_mlp_s* chf_mlp;

/* Last error message of the calling thread ("" if none). */
const char* chf_last_error(void);
/* Library version string. */
const char* chf_version(void);

/* ---------------------------------------------------------------- BSR ---- */
/* Block-sparse SPD matrix with block structure B = {b,...,b} (Def. 2.1).
 * rowptr: host int64[nb+1]; colidx: host int32[nnzb], ascending per row;
 * vals: nnzb*b*b doubles, host or device (vals_on_device), block e at
 * vals[e*b*b], row-major. The matrix is copied; b must be in [1, 64].
 * EINVAL on bad structure or non-finite values. */
int chf_bsr_create(int64_t nb, int32_t b, const int64_t* rowptr, const int32_t* colidx,
                   const double* vals, int vals_on_device, chf_bsr* out);
int chf_bsr_destroy(chf_bsr A);
int chf_bsr_info(chf_bsr A, int64_t* nb, int32_t* b, int64_t* nnzb);
/* Copy structure (host rowptr[nb+1], colidx[nnzb]) and FP64 values
 * (host vals[nnzb*b*b]) out; any pointer may be NULL. */
int chf_bsr_export(chf_bsr A, int64_t* rowptr, int32_t* colidx, double* vals);
/* y = A x (residual == 0) or y = bvec - A x (residual != 0), on device
 * vectors of `dtype` (CHF_F64: double, CHF_F32: float with FP32 storage of A). */
int chf_bsr_spmv(chf_bsr A, chf_dtype dtype, const void* x, const void* bvec, void* y,
                 int residual, hipStream_t stream);

/* -------------------------------------------------- variable block sizes -- */
/* Block-sparse SPD matrix whose blocks have their own sizes m_i = bsize[i]
 * (Def. 2.1's block structure with unequal blocks, e.g. a higher polynomial
 * degree on the boundary patches, Sec. 5 Ex. 5.1). rowptr/colidx as for
 * chf_bsr_create; block e = (i, colidx[e]) is the bsize[i] x bsize[colidx[e]]
 * array stored row-major at vals + voff_e, voff_e being the running sum of
 * bsize[i] * bsize[colidx[e]] over the preceding blocks in storage order. All
 * arrays are host arrays, copied; 1 <= bsize[i] <= 64; EINVAL on bad
 * structure or non-finite values. The handle is a chf_bsr whose vectors have
 * sum(bsize) entries. Accepted with CHF_F64: chf_bsr_spmv, chf_pattern_lower,
 * chf_fsai_setup (local systems of at most 32 blocks and 160 unknowns, own
 * block at most 16 wide; EINVAL beyond), chf_fsai_apply, chf_fsai_export
 * (G's blocks bsize[k] x bsize[j] in pattern order, flat), chf_lmax_lanczos
 * and the smoothers (chf_cheb4_smooth[_noalloc], chf_cheb1_smooth,
 * chf_richardson_smooth). The adaptive pattern, nested FSAI, the hierarchy,
 * the learned proposer and FP32/BF16 storage take uniform blocks only
 * (EINVAL). chf_bsr_info reports b = the largest block; chf_bsr_export
 * writes the flat values. */
int chf_vbsr_create(int64_t nb, const int32_t* bsize, const int64_t* rowptr, const int32_t* colidx,
                    const double* vals, chf_bsr* out);
/* Unknowns, stored values and block sizes (host int32[nb], may be NULL) of a
 * matrix, uniform or not. */
int chf_vbsr_info(chf_bsr A, int64_t* ndof, int64_t* nvals, int32_t* bsize);

/* ------------------------------------------------------------ patterns ---- */
/* Lower block triangle of A with the diagonal (static pattern, Sec. 2.1). */
int chf_pattern_lower(chf_bsr A, chf_pattern* out);
/* Pattern from host CSR (rowptr int64[nb+1], colidx int32[nnz]); EINVAL
 * unless lower triangular, strictly ascending per row, diagonal present. */
int chf_pattern_from_csr(int64_t nb, const int64_t* rowptr, const int32_t* colidx,
                         chf_pattern* out);
/* Adaptive block-FSAI pattern (Algorithm 1, Lemma 2.4), computed on the GPU.
 * P0: the initial pattern of Algorithm 1 (borrowed, same block count as A;
 * NULL = the diagonal, the choice of Sec. 5). tmax >= 0 adaptive steps after
 * P0; tau in (0, 1]. A candidate c < k, c not in P_k, with structurally
 * nonzero (FA)_kc enters row k when g* = -log rho_c* > -log tau + 1e-12; ties
 * within a relative 1e-9 of g* go to the smallest column. The longest row of
 * P0 plus tmax must not exceed 32 blocks (EINVAL). ENOTSPD if a local matrix
 * is not positive definite. tmax = 0 returns a copy of P0. */
int chf_pattern_adaptive(chf_bsr A, chf_pattern P0, int tmax, double tau, chf_pattern* out);
/* Pattern from a stencil template on an nx x ny x nz patch grid (block
 * index i = ix + nx (iy + ny iz)): row k holds k and every k + (dx, dy, dz)
 * of the noff offsets (host int32[noff][3]) that stays inside the grid. Each
 * offset must point to a smaller index (dx + nx (dy + ny dz) < 0, EINVAL
 * otherwise). Not part of the paper: with a template read off Algorithm 1's
 * pattern of an interior row, it is the translation-invariant baseline that
 * the learned proposer is compared with. */
int chf_pattern_template(int64_t nx, int64_t ny, int64_t nz, int32_t noff, const int32_t* offsets,
                         chf_pattern* out);
int chf_pattern_info(chf_pattern P, int64_t* nb, int64_t* nnz);
int chf_pattern_export(chf_pattern P, int64_t* rowptr, int32_t* colidx);
int chf_pattern_destroy(chf_pattern P);

/* ---------------------------------------------------------------- FSAI ---- */
/* Block-FSAI factor G = S^{-1/2} F on pattern P (Def. 2.2), with S^{-1/2}
 * the inverse Cholesky root of S_kk. All local SPD systems A[P_k, P_k]
 * (size b*|P_k| <= 320) are factorised in FP64 in one persistent launch.
 * g_store: storage of G for the smoother (F64, F32 or BF16); the FP64
 * values are kept for export and Lanczos. On ENOTSPD *bad_row (may be NULL)
 * is the smallest block row whose local factorisation failed. */
int chf_fsai_setup(chf_bsr A, chf_pattern P, chf_dtype g_store, chf_fsai* out,
                   int64_t* bad_row);
int chf_fsai_destroy(chf_fsai G);
/* G's FP64 blocks in pattern order (host double[nnz*b*b]). */
int chf_fsai_export(chf_fsai G, double* vals);
/* z = G^T G r (the preconditioner M r), device vectors of dtype. work: n.
 * For a nested factor (chf_fsai_nest) z = G0^T G1^T G1 G0 r. */
int chf_fsai_apply(chf_fsai G, chf_dtype dtype, const void* r, void* z, void* work,
                   hipStream_t stream);

/* ---------------------------------------------------- nested FSAI -------- */
/* Sec. 2.2 with one nesting level. The inner factor is built for
 * A1 = G0 A G0^T, where G0 is the outer (scaled) factor: block-FSAI and
 * Algorithm 1 are invariant under that block-diagonal congruence, so
 * M = G0^T G1^T G1 G0 equals the F^T S^{-1} F (F = F1 F0) of Sec. 2.2.
 * chf_bsr_triple: *out = G A G^T (FP64, new handle owned by the caller),
 * on the structural block pattern; G must be a plain factor (EINVAL for a
 * nested one or mismatched sizes).
 * chf_fsai_nest: *out = the nested factor of G0 (outer, built for A) and G1
 * (inner, built for chf_bsr_triple(A, G0)); both are borrowed and must
 * outlive *out; they must share nb, b and storage dtype. The nested handle
 * is accepted wherever a factor is used (smoothers, Lanczos, apply, levels);
 * chf_fsai_export refuses it (export its parts). */
int chf_bsr_triple(chf_bsr A, chf_fsai G, chf_bsr* out);
int chf_fsai_nest(chf_fsai G0, chf_fsai G1, chf_fsai* out);

/* Largest eigenvalue of G A G^T (= of M A) by `iters` plain Lanczos steps
 * from the device start vector v0 (double[N], not modified); theta is the
 * largest Ritz value and *beta = safety * theta (Sec. 5: 100 steps, 1.01).
 * dtype selects which stored operators are used (F64, or the rounded F32/BF16
 * ones, evaluated in FP64 arithmetic). Synchronises `stream`. */
int chf_lmax_lanczos(chf_bsr A, chf_fsai G, chf_dtype dtype, int iters, const double* v0,
                     double safety, double* beta, double* theta, hipStream_t stream);

/* ---------------------------------------------------------- smoother ---- */
/* Algorithm 3 (Chebyshev iteration of the fourth kind), degree >= 1, with
 * M = G^T G and beta >= lambda_max(MA). b, x: device vectors (N = nb*b) of
 * dtype; x is updated in place (x_is_zero: x's input is ignored and taken as
 * 0, saving one product with A). work: device buffer of 3N elements. */
int chf_cheb4_smooth(chf_bsr A, chf_fsai G, chf_dtype dtype, double beta, int degree,
                     const void* b, void* x, int x_is_zero, void* work, hipStream_t stream);

/* chf_cheb4_smooth without the work argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): the call performs no allocation. Its
 * three work vectors live in a library-owned device array of 64 MiB that
 * every device the library runs on holds until the process ends, so
 * 3 * N * sizeof(element) must not exceed 64 MiB (EINVAL otherwise: N up to
 * 2,796,202 for CHF_F64, twice that for FP32 vectors). No part of the array
 * needs to start at zero: each call writes every element it reads. Calls
 * that overlap on one device (several streams or host threads) share the
 * array and race; serialise them. For CHF_F32/CHF_BF16 the FP32 layout of A
 * must already exist (one FP32 call of chf_cheb4_smooth or chf_bsr_spmv
 * builds it), since building it allocates (EINVAL otherwise). Results are
 * those of chf_cheb4_smooth with the same arguments. */
int chf_cheb4_smooth_noalloc(chf_bsr A, chf_fsai G, chf_dtype dtype, double beta, int degree,
                             const void* b, void* x, int x_is_zero, hipStream_t stream);

/* Comparators of Sec. 3.1, with the same arguments, layout and work buffer
 * as chf_cheb4_smooth:
 * - chf_cheb1_smooth: Algorithm 2 (Chebyshev iteration of the first kind)
 *   with the preconditioner M, on the smoothing interval [alpha, beta]
 *   (0 < alpha < beta; Sec. 3.1 takes alpha = rho lambda_max, rho in (0,1)).
 * - chf_richardson_smooth: Richardson smoothing x <- x + omega M (b - A x),
 *   `degree` times, i.e. S = (I - omega M A)^degree (omega = 1 in Sec. 3.1).
 * EINVAL for degree < 1 or parameters outside these ranges. */
int chf_cheb1_smooth(chf_bsr A, chf_fsai G, chf_dtype dtype, double alpha, double beta, int degree,
                     const void* b, void* x, int x_is_zero, void* work, hipStream_t stream);
int chf_richardson_smooth(chf_bsr A, chf_fsai G, chf_dtype dtype, double omega, int degree,
                          const void* b, void* x, int x_is_zero, void* work, hipStream_t stream);

/* ----------------------------------------------------------- V-cycle ---- */
typedef struct {
    int degree;          /* Chebyshev degree k of V(k,k) */
    int pattern;         /* 0: lower(A_l), 1: adaptive (Algorithm 1), 2: diagonal */
    int tmax;            /* adaptive steps */
    double tau;          /* adaptive threshold (1.0 in the paper) */
    int lanczos_iters;   /* 100 in the paper */
    double safety;       /* 1.01 in the paper */
    chf_dtype dtype;     /* F64: plain; F32: A_l, G_l FP32; BF16: A_l FP32, G_l BF16 (FP32 vectors);
                            F64_BF16G: A_l and vectors FP64, G_l BF16 */
} chf_level_opts;

/* Empty hierarchy whose finest operator is A0 (borrowed: A0 must outlive L). */
int chf_levels_create(chf_bsr A0, chf_levels* out);
/* Append a coarser level (Sec. 5: Galerkin coarse operators A_c = P^T A P).
 * The prolongation is P = T (P_s (x) I_b): p_* is the scalar patch
 * prolongation P_s (host CSR, nf x nc, nf = current coarsest block count) and
 * `basis` (host double[nf*b*b], may be NULL for T = I) the block-diagonal
 * change from the interpolated local bases to the fine level's local bases.
 * The Galerkin product is formed on the GPU. */
int chf_levels_add_coarse(chf_levels L, int64_t nc, const int64_t* p_rowptr,
                          const int32_t* p_colidx, const double* p_vals, const double* basis);
/* Per level except the coarsest: pattern, G (FSAI), beta (Lanczos from
 * v0[l], device double[N_l]); coarsest: dense FP64 Cholesky-based inverse.
 * v0 may be NULL only if every beta is set afterwards with
 * chf_levels_set_beta. On ENOTSPD *bad_row is set as in chf_fsai_setup
 * (the coarsest level reports -2). Level 0 is set up on the null stream;
 * the coarser levels are set up meanwhile by an internal host thread on a
 * stream of its own, on the calling thread's current device. The call
 * returns when all levels are done. */
int chf_levels_setup(chf_levels L, const chf_level_opts* opts, const double* const* v0,
                     int64_t* bad_row);
/* Use pattern P (copied; lower triangular with the diagonal) on level `level`
 * instead of opts->pattern, e.g. a learned proposal. Before chf_levels_setup. */
int chf_levels_set_pattern(chf_levels L, int level, chf_pattern P);
int chf_levels_destroy(chf_levels L);
int chf_levels_info(chf_levels L, int* nlevels, int64_t* nb_per_level /* [nlevels] or NULL */);
/* Borrowed handles of level l (valid while L lives; G is NULL on the coarsest). */
int chf_levels_get(chf_levels L, int level, chf_bsr* A, chf_fsai* G, chf_pattern* P);
int chf_levels_get_beta(chf_levels L, int level, double* beta);
int chf_levels_set_beta(chf_levels L, int level, double beta);
/* Nested block-FSAI on every smoothed level (Sec. 2.2, one nesting level,
 * the same t_max and tau on both levels as in Sec. 5): nest = 1 builds the
 * outer factor G0 for A_l, the inner factor for G0 A_l G0^T from Algorithm 1,
 * and smooths with M = G0^T G1^T G1 G0; nest = 0 (default) is plain FSAI.
 * Before chf_levels_setup; with nest = 1 opts->pattern must be 1 (EINVAL). */
int chf_levels_set_nesting(chf_levels L, int nest);
/* Smoother and cycle shape of the hierarchy (default: fourth kind, V(k,k)).
 * smoother: CHF_SMOOTH_CHEB4 (Algorithm 3 on [0, beta_l]; param ignored),
 * CHF_SMOOTH_CHEB1 (Algorithm 2 on [param * beta_l, beta_l], 0 < param < 1),
 * CHF_SMOOTH_RICHARDSON (omega = param > 0). cycle: CHF_CYCLE_VKK, or
 * CHF_CYCLE_V2K0 (Sec. 5's non-symmetric cycle: one pre-smoothing application
 * of degree 2k and no post-smoothing; PCG then requires the flexible form).
 * May be called before or after chf_levels_setup; the bounds beta_l stay. */
int chf_levels_set_cycle(chf_levels L, chf_smoother smoother, double param, chf_cycle cycle);
/* One cycle (V(k,k), or V(2k,0) when so set) on level 0: x <- V(b, x);
 * vectors of the hierarchy's working dtype (double for F64, float otherwise). */
int chf_vcycle(chf_levels L, const void* b, void* x, int x_is_zero, hipStream_t stream);
/* Energy-norm convergence factor of the cycle as a stationary iteration on
 * A x = 0 (Ex. 5.1's rho_A, with b = 0): e <- cycle(0, e) from e0 until
 * ||e||_A < tol ||e0||_A or maxit cycles (maxit >= 1, tol >= 0);
 * *rho = (e_n^T A e_n / e0^T A e0)^{1/(2n)} and *cycles = n. e0: device
 * double[N] on level 0, not modified; a mixed hierarchy cycles in FP32 on e0
 * rounded, and every energy norm is formed in FP64 with the FP64 A.
 * Synchronises `stream` once per cycle. */
int chf_levels_energy_factor(chf_levels L, const double* e0, double tol, int maxit, double* rho, int* cycles,
                             hipStream_t stream);
/* FP64 PCG from x = 0 with one cycle as preconditioner (cast to and from
 * the working dtype for mixed hierarchies). Stops when the recursive
 * residual ||r|| <= rtol ||b||. flexible != 0: Polak-Ribiere beta (required,
 * else EINVAL, when the cycle is V(2k,0), which is not symmetric).
 * relres_hist (host, maxit+1, may be NULL) receives ||r_i||/||b||;
 * true_relres (may be NULL) receives ||b - A x|| / ||b|| in FP64.
 * ENOCONV if maxit is reached (x holds the last iterate). */
int chf_pcg_solve(chf_levels L, const double* b, double* x, double rtol, int maxit,
                  int flexible, int* iters, double* relres_hist, double* true_relres,
                  hipStream_t stream);
/* Right-preconditioned BiCGStab (van der Vorst 1992) from x = 0 with one
 * cycle as preconditioner: the outer solver Sec. 6 names for the
 * non-symmetric V(2k,0) cycle (any cycle is accepted). Shadow residual b.
 * Stops when ||r|| <= rtol ||b||, checked at both half steps of an iteration.
 * relres_hist (host, 2*maxit+1, may be NULL) receives the residual norm
 * after every half step; true_relres as for chf_pcg_solve. EBREAKDOWN if
 * (r^, r), (r^, v) or omega vanish; ENOCONV if maxit is reached. */
int chf_bicgstab_solve(chf_levels L, const double* b, double* x, double rtol, int maxit,
                       int* iters, double* relres_hist, double* true_relres, hipStream_t stream);

/* ------------------------------------------------------- learned pattern -- */
/* Not part of the paper: a small network, trained on patterns that Algorithm 1
 * produces, proposes the factor pattern; Algorithm 1 stays the fallback and
 * the reference its patterns are compared against. */
/* Candidate features for the learned pattern proposer: for each block row k
 * and each candidate c in the strictly lower part of the row pattern of A^2,
 * 6 FP32 features: ||A_kc||_F, ||A_cc^{-1} A_ck||_F, the signed patch offset (dx, dy, dz) of c from k
 * measured on the grid given by (nx, ny) (nz implied), and the one-step gain
 * -log rho_c at P = {k} (Lemma 2.4). Features are written to a device buffer
 * (float[ncand*4]); the candidate CSR (host int64 rowptr[nb+1], int32
 * cols[ncand]) is returned through chf_mlp_candidates. */
int chf_mlp_candidates(chf_bsr A, int64_t* ncand, int64_t* rowptr, int32_t* cols);
int chf_mlp_features(chf_bsr A, int32_t nx, int32_t ny, float* feats, hipStream_t stream);
/* 6 -> 64 -> 64 -> 1 MLP with ReLU, FP32 parameters (4673 floats, layout
 * W1[64][4], b1[64], W2[64][64], b2[64], W3[64], b3) and Adam moments. */
int chf_mlp_create(const float* params_host, chf_mlp* out);
int chf_mlp_destroy(chf_mlp net);
int chf_mlp_get_params(chf_mlp net, float* params_host);
/* Logits for n feature rows (device float[n*4] -> float[n]). */
int chf_mlp_forward(chf_mlp net, const float* feats, int64_t n, float* logits, hipStream_t stream);
/* Mean binary cross-entropy-with-logits loss and its gradient (device
 * float[4673] written to grad) over n rows with labels in {0, 1}. */
int chf_mlp_loss_grad(chf_mlp net, const float* feats, const float* labels, int64_t n,
                      float* loss_host, float* grad, hipStream_t stream);
/* One Adam step (lr, beta1, beta2, eps) on the mini-batch. */
int chf_mlp_train_step(chf_mlp net, const float* feats, const float* labels, int64_t n,
                       float lr, float beta1, float beta2, float eps, float* loss_host,
                       hipStream_t stream);
/* Labels for the candidates of chf_mlp_candidates (device float[ncand]):
 * 1 where the candidate belongs to P (e.g. the pattern of Algorithm 1). */
int chf_mlp_labels(chf_bsr A, chf_pattern P, float* labels, hipStream_t stream);
/* `epochs` passes of mini-batch Adam over n rows in the order given by the
 * device permutation perm (int64[n], NULL = identity), `batch` rows per step.
 * loss_hist (host float[epochs], may be NULL) receives each epoch's mean loss. */
int chf_mlp_train(chf_mlp net, const float* feats, const float* labels, int64_t n, const int64_t* perm,
                  int64_t batch, int epochs, float lr, float beta1, float beta2, float eps,
                  float* loss_hist, hipStream_t stream);
/* Pattern from the t highest-scoring candidates per row (ties to the smaller
 * column), diagonal added. */
int chf_mlp_propose(chf_bsr A, chf_mlp net, int32_t nx, int32_t ny, int t, chf_pattern* out);

#ifdef __cplusplus
}
#endif
#endif /* CHF_H */
