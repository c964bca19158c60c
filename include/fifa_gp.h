/*
 * fifa_gp.h -- C ABI of the MI355X FIFA-GP hot path (libfifagp.so).
 *
 * One Gibbs iteration of the fast increased-fidelity approximate GP sampler of
 * Moran & Wheeler (arXiv 2006.06537) on sorted 1-D inputs: build a HODLR
 * approximation K~_1 of the unit-amplitude covariance, factor alpha K~_1 + beta I
 * symmetrically as W W', solve, take log-determinants, draw f by Algorithm 1 and
 * update tau, sigma_f^2 and the length-scale (Section 4.1).
 *
 * Conventions shared by every call
 *   - Memory: every `double*` / `int64_t*` argument is DEVICE memory owned by the
 *     caller unless the comment says "host".  Vectors are FP64, column-major when
 *     they hold several right-hand sides (leading dimension `ld` >= n).
 *   - Handles (fg_hodlr, fg_factor, fg_chain) own device memory allocated by the
 *     library; destroy them with the matching *_destroy call.
 *   - Streams: `stream` is a hipStream_t (NULL = the default stream).  All calls
 *     are stream-ordered and asynchronous unless stated; the return code covers
 *     argument/configuration errors and launch failures only.  Failures found on
 *     the device (a non-positive leaf pivot, a node singular value >= 1, a Gamma
 *     sampler that ran out of tries) are recorded in the handle's status word and
 *     read with hodlr_status / factor_status / gibbs_chain_state (which synchronise
 *     the stream).
 *   - No exception crosses the ABI and nothing aborts.  fg_last_error() returns a
 *     thread-local message for the last non-zero return code.
 *   - Indices are 32-bit inside the library: n must satisfy 1 <= n < 2^31.
 *   - Kernel: k_1(x,x') = exp(-(x-x')^2 / (2 ell^2)) (squared exponential, Section
 *     2.1 / 4.1 with rho = 1/(2 ell^2)) or exp(-|x-x'|/ell) (exponential, a Matern
 *     kernel of Section 2.1).  `nugget` is added to the diagonal before the
 *     H-matrix construction (Section 4.1, "Additional considerations").
 */
#ifndef FIFA_GP_H
#define FIFA_GP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t fg_status;
#define FG_OK 0
#define FG_EINVAL (-1)     /* bad argument or configuration                         */
#define FG_ENOMEM (-2)     /* device allocation failed                              */
#define FG_ENOTSPD (-3)    /* matrix not positive definite (leaf pivot / sigma >= 1) */
#define FG_ETOL (-4)       /* tolerance needs more than 60 interpolation nodes      */
#define FG_ENOTCONV (-5)   /* an iteration (Gamma tries, Jacobi sweeps) ran out     */
#define FG_EDEVICE (-6)    /* HIP runtime error                                     */

typedef void* fg_stream;                 /* hipStream_t */
typedef struct fg_hodlr_s* fg_hodlr;     /* compressed K~_1, device resident */
typedef struct fg_factor_s* fg_factor;   /* W with W W' = alpha K~_1 + beta I + diag(d) */
typedef struct fg_chain_s* fg_chain;     /* one Gibbs chain and its cached factors */
typedef struct fg_tp_chain_s* fg_tp_chain; /* one tensor-product chain (Section 4.2) */

/* Kernels k_1 (Section 2.1; unit amplitude, d = |x - x'|): squared exponential
 * exp(-d^2 / (2 ell^2)); exponential exp(-d / ell); Matern-3/2 (1 + u) exp(-u) with
 * u = sqrt(3) d / ell; Matern-5/2 (1 + u + u^2/3) exp(-u) with u = sqrt(5) d / ell. */
#define FG_KERNEL_SE 0
#define FG_KERNEL_EXP 1
#define FG_KERNEL_MATERN32 2
#define FG_KERNEL_MATERN52 3

typedef struct {
  int32_t kind;          /* FG_KERNEL_SE, _EXP, _MATERN32 or _MATERN52    */
  double lengthscale;    /* ell > 0                                        */
  double nugget;         /* >= 0, added to the diagonal of K_1             */
} fg_kernel;

/* ---------------------------------------------------------------------------
 * hodlr_build -- HODLR approximation K~_1 of K_1 = [k_1(x_i,x_j)] + nugget I.
 * Section 3.2 (HODLR format: recursive 2x2 partition, dense diagonal leaves,
 * low-rank off-diagonal blocks whose max-norm error is bounded by construction)
 * and the inputs of Algorithm 1 (tolerance eps, maximum block size B).
 *   x     device, n values, sorted ascending (non-decreasing); copied.
 *   leaf  maximum leaf size B, 2 <= B <= 128.
 *   tol   absolute max-norm bound on |K_1 - K~_1|, tol > 0.
 * Each off-diagonal block: window rows within R of the split (k_1 < tol/3 beyond
 * it), first-kind Chebyshev interpolation (per-variable error bound tol/6), then
 * truncated SVD at max(tol/3, 8 u s_1).  Node ranks are decided on the device.
 * Synchronises `stream` once (x is copied to the host for the tree plan).
 * Errors: FG_EINVAL (n, leaf, tol, ell, unsorted x), FG_ETOL, FG_ENOMEM.
 * ------------------------------------------------------------------------- */
fg_status hodlr_build(const double* x, int64_t n, fg_kernel kernel, int32_t leaf,
                      double tol, fg_stream stream, fg_hodlr* out);

/* Host copy of the node ranks in heap order (node 0 = root, children 2h+1,
 * 2h+2; 2^L - 1 internal nodes).  `ranks` is host memory of `cap` entries;
 * `*count` receives 2^L - 1.  Synchronises the stream. */
fg_status hodlr_ranks(fg_hodlr A, int32_t* ranks, int32_t cap, int32_t* count,
                      fg_stream stream);

/* Host copy of the tree: *levels = L, *n_out = n.  Either pointer may be NULL. */
fg_status hodlr_info(fg_hodlr A, int32_t* levels, int64_t* n_out);

/* Host copy of each node's singular values of the interpolant (heap order, `cap`
 * doubles per node, zero padded).  For rank-decision diagnostics.  Syncs. */
fg_status hodlr_singular_values(fg_hodlr A, double* sv, int32_t cap, fg_stream stream);

/* out[t] = K~_1[i[t], j[t]] for t < count (device index arrays, int64). */
fg_status hodlr_entries(fg_hodlr A, const int64_t* i, const int64_t* j, int64_t count,
                        double* out, fg_stream stream);

/* y = (alpha K~_1 + beta I) v for nrhs columns (ld >= n).  v and y must not
 * overlap.  O(n log n) per column (Algorithm 1's H-matrix products). */
fg_status hodlr_matvec(fg_hodlr A, double alpha, double beta, const double* v, double* y,
                       int32_t nrhs, int64_t ld, fg_stream stream);

/* ---------------------------------------------------------------------------
 * hodlr_factor -- symmetric factor W W' = alpha K~_1 + beta I + diag(d)
 * (SI "HODLR decomposition and factorization": W = A_L ... A_0, block-diagonal
 * leaf Cholesky factor times one identity-plus-low-rank factor per level).  The
 * node factor is the canonical one, W_nu = [[I, 0], [C', (I - C'C)^(1/2)]] with
 * C the whitened off-diagonal block, so W depends on the matrix only.
 *   alpha > 0, beta >= 0 (host values); diag: device, n values or NULL.
 * The factor keeps a reference to A's data: destroy it before A.
 * Device failures: FG_ENOTSPD in the factor's status word.
 * ------------------------------------------------------------------------- */
fg_status hodlr_factor(fg_hodlr A, double alpha, double beta, const double* diag,
                       fg_stream stream, fg_factor* out);

/* ---------------------------------------------------------------------------
 * Precision of a factor.  FG_MIXED holds the leaf Cholesky factors, their inverses and
 * the whitened panels in FP32 and computes them in FP32 (leaf Cholesky / whitening,
 * panel Gram products on FP32 MFMA, panel updates); node capacitance factors, log-det
 * accumulation and every vector operation stay FP64.  Meant as a preconditioner
 * (hodlr_solve_refined); its W-products and log-det carry FP32-level error, and a node
 * whose 1 - s^2 falls below 16 FP32 ulps (kappa u32 ~ 1) is floored there instead of
 * being reported as not positive definite.
 * ------------------------------------------------------------------------- */
#define FG_FP64 0
#define FG_MIXED 1
/* hodlr_factor with a precision (FG_FP64 is hodlr_factor itself). */
fg_status hodlr_factor_prec(fg_hodlr A, double alpha, double beta, const double* diag,
                            int32_t precision, fg_stream stream, fg_factor* out);
/* ---------------------------------------------------------------------------
 * hodlr_solve_refined -- x = (alpha K~_1 + beta I)^-1 b by preconditioned conjugate
 * gradients: products with the FP64 HODLR matrix A, preconditioner z = W^-T W^-1 r from
 * F (a factor of the same matrix, any precision), FP64 residuals and inner products.
 * Stops when |b - A x|_2 <= rtol |b|_2 for every column (rtol > 0) or after maxit
 * iterations.  nrhs <= 4 columns, ld >= n; b and x must not overlap.
 * *iters (host, may be NULL): iterations used; *relres (host, may be NULL): the largest
 * final relative residual.  Synchronises the stream once per iteration.
 * Errors: FG_EINVAL, FG_ENOMEM (workspace), FG_ENOTCONV (rtol not reached).
 * ------------------------------------------------------------------------- */
fg_status hodlr_solve_refined(fg_hodlr A, fg_factor F, double alpha, double beta,
                              const double* b, double* x, int32_t nrhs, int64_t ld, double rtol,
                              int32_t maxit, int32_t* iters, double* relres, fg_stream stream);
/* ---------------------------------------------------------------------------
 * hodlr_solve_refined_noalloc -- hodlr_solve_refined for callers that cannot allocate
 * (code under graph capture, tight serving loops, harnesses that forbid runtime
 * allocation).  Same arguments, results and errors, but the PCG workspace is a fixed
 * device array of the library (one per GPU, about 32 MiB, held until the process ends)
 * instead of a per-call allocation: the call makes no hipMalloc / hipFree.
 *   - n * nrhs must be at most 2^20 (FG_EINVAL beyond, with a message).
 *   - Every call on one GPU uses that GPU's array: calls that overlap in time on the
 *     same GPU (other host threads, other streams) race; serialise them.
 *   - The record of convergence is read back into host stack memory once per four
 *     iterations (the stream is synchronised then, as in hodlr_solve_refined).
 * ------------------------------------------------------------------------- */
fg_status hodlr_solve_refined_noalloc(fg_hodlr A, fg_factor F, double alpha, double beta,
                                      const double* b, double* x, int32_t nrhs, int64_t ld,
                                      double rtol, int32_t maxit, int32_t* iters, double* relres,
                                      fg_stream stream);
/* x = (W W')^-1 b = W^-T W^-1 b for nrhs columns: the solves of Algorithm 1 (M~ w = Z,
 * M~ r = tau y) with the factor of the SI factorization, one sweep up the tree (W^-1)
 * and one down (W^-T).  b and x may be the same.  Errors: FG_EINVAL (NULL, nrhs < 1,
 * ld < n); device failures of the factor are in its status word. */
fg_status hodlr_solve(fg_factor F, const double* b, double* x, int32_t nrhs, int64_t ld,
                      fg_stream stream);

/* *logdet_dev = log det(W W') = 2 sum log diag(L_leaf) + sum_nodes sum_i
 * log(1 - sigma_i^2) (SI "Determinant computation speedup": block determinants
 * and Sylvester's theorem).  logdet_dev: device, one double. */
fg_status hodlr_logdet(fg_factor F, double* logdet_dev, fg_stream stream);

/* The same log-determinant in its two parts (SI "Determinant computation speedup": the
 * block-diagonal factor and the identity-plus-low-rank level factors contribute
 * separately): parts_dev[0] = 2 sum log diag(L_leaf), parts_dev[1] = sum_nodes sum_i
 * log(1 - sigma_i^2).  parts_dev: device, two doubles.  A diagnostic for parity checks:
 * at large n the two parts nearly cancel, and each can be compared on its own. */
fg_status hodlr_logdet_parts(fg_factor F, double* parts_dev, fg_stream stream);

/* y = op(W) v with op = W (transpose=0, inverse=0), W' (1,0), W^-1 (0,1),
 * W^-T (1,1); nrhs columns.  v and y may be the same.  The factors of W are those of the
 * SI factorization (W = L_D W_(L-1) ... W_(0)); Algorithm 1 uses W b to form Z and
 * W^-1 f in the length-scale conditional.  Errors: FG_EINVAL (NULL, nrhs < 1, ld < n). */
fg_status hodlr_apply_w(fg_factor F, int32_t transpose, int32_t inverse, const double* v,
                        double* y, int32_t nrhs, int64_t ld, fg_stream stream);

/* ---------------------------------------------------------------------------
 * Counter-based normals: Philox4x64-10 (Salmon et al., SC'11), key (seed, 0),
 * counter (block, tag, iteration, stream), uniforms ((w >> 12) + 0.5) 2^-52,
 * Box-Muller in pairs (cos, sin).  out: device, n doubles.
 * ------------------------------------------------------------------------- */
fg_status fg_normals(uint64_t seed, uint64_t tag, uint64_t iteration, uint64_t stream_id,
                     int64_t n, double* out, fg_stream stream);

/* ---------------------------------------------------------------------------
 * gp_draw_f -- Algorithm 1 (Section 4.1.1) with K~ = sigf2 K~_1, W = sqrt(sigf2) W_1,
 * M~ = tau K~ + I:  a, b ~ N(0, I) (tags 1 and 2 of (seed, iteration, stream_id));
 * Z = sqrt(tau) K~ a + W b;  M~ w = Z;  M~ r = tau y;  f = w + K~ r.
 *   K1  compressed K~_1;  W1 factor of K~_1 (alpha 1, beta 0);
 *   WM  factor of K~_1 with alpha = tau*sigf2, beta = 1.
 *   y, f, r device n-vectors; mu (device, n, or NULL) receives K~ r, the
 *   approximate posterior mean of Lemma 4.1; r = Sigma~^-1 y.
 * ------------------------------------------------------------------------- */
fg_status gp_draw_f(fg_hodlr K1, fg_factor W1, fg_factor WM, double sigf2, double tau,
                    const double* y, uint64_t seed, uint64_t iteration, uint64_t stream_id,
                    double* f, double* r, double* mu, fg_stream stream);

/* ---------------------------------------------------------------------------
 * gp_draw_f_hetero -- Algorithm 1.h (Appendix, heteroskedastic noise) for a
 * unit-variance prior K~ = K~_1 and diagonal noise precisions D:
 *   a ~ N(0, D) (a = sqrt(D) a_std), b ~ N(0, I);  Z = K~ a + W b;
 *   Z* = P~^-1 Z;  Z** = D^-1 Z*;  R = K~ P~^-1 y;  f = R + Z**.
 *   K   compressed K~_1;  WK  factor of K~_1 (alpha 1, beta 0);
 *   WP  factor of K~_1 + diag(1/D) (hodlr_factor with alpha 1, beta 0, diag 1/D).
 *   D, y  device n-vectors (D > 0);  f, R  device n-vectors (R may be NULL):
 *   R = K~ P~^-1 y is the approximate posterior mean of the Appendix lemma.
 *   factor  -1: a_std, b on tags 1 and 2 of (seed, iteration, stream_id);
 *           h >= 0: tags 1 + 16 (h+1) and 2 + 16 (h+1) (factor h of a tensor chain).
 * Errors: FG_EINVAL (NULL, size mismatch, factor < -1).
 * ------------------------------------------------------------------------- */
fg_status gp_draw_f_hetero(fg_hodlr K, fg_factor WK, fg_factor WP, const double* D,
                           const double* y, uint64_t seed, uint64_t iteration,
                           uint64_t stream_id, int32_t factor, double* f, double* R,
                           fg_stream stream);

/* ---------------------------------------------------------------------------
 * Gibbs chain (Section 4.1): sweep f -> tau -> sigma_f^-2 -> length-scale.
 *   tau     | - ~ Ga((a1+n)/2, (b1 + |y-f|^2)/2)            (shape, rate)
 *   sf^-2   | - ~ Ga((a2+n)/2, (b2 + f' K~_1^-1 f)/2)
 *   ell on the grid ell_k = ell0 10^((k - center)/50), k = 0..grid_size-1, by a
 *   Metropolis step on neighbours k +- 1 (the paper's suggested replacement for the
 *   discrete conditional): accept with min(1, exp(D)),
 *   D = -1/2 (log|K~_1'| - log|K~_1|) - (q' - q)/(2 sigf2),  q = |W_1^-1 f|^2.
 * Random numbers: tags 1 (a), 2 (b), 3 (tau Gamma), 4 (sigma Gamma), 5
 * (proposal), 6 (acceptance) of (seed, iteration, stream_id).
 * ------------------------------------------------------------------------- */
typedef struct {
  int32_t kind;          /* FG_KERNEL_SE / _EXP / _MATERN32 / _MATERN52 */
  double ell0;           /* grid centre length-scale */
  double nugget;         /* added to K_1's diagonal */
  int32_t leaf;          /* maximum leaf size */
  double tol;            /* max-norm tolerance on K_1 */
  double tau0;           /* initial noise precision */
  double sigf2_0;        /* initial sigma_f^2 */
  double a1, b1, a2, b2; /* Gamma prior parameters (tau ~ Ga(a1/2, b1/2), ...) */
  int32_t grid_size;     /* number of length-scales (e.g. 100) */
  int32_t grid_center;   /* starting index (e.g. 50) */
  uint64_t seed;
  uint64_t stream_id;    /* chain id in the Philox counter */
  int32_t precision;     /* FG_FP64, or FG_MIXED: M~ = tau sigf2 K~_1 + I factored in
                            FP32 and its two solves refined by PCG to a relative residual
                            of 1e-10 (W_1 and everything else stay FP64); falls back to
                            FP64 for good if the FP32 factor fails (see precision_used) */
} fg_chain_cfg;

typedef struct {
  int64_t iteration;     /* completed sweeps */
  double tau, sigf2, ell;
  int32_t k;             /* grid index of ell */
  int32_t last_proposal; /* proposed grid index of the last sweep (-1/grid_size = off grid) */
  int32_t last_accept;   /* 1 if the last proposal was accepted */
  int32_t accepts;       /* accepted proposals so far */
  double logdet_sigma;   /* log|Sigma~| of the last f-draw, Sigma~ = K~ + I/tau */
  double yr;             /* y' Sigma~^-1 y */
  double loglik;         /* Eq. 2 (with 1/2 on log det) at the last f-draw */
  double sse;            /* |y - f|^2 */
  double q;              /* f' K~_1^-1 f at the current length-scale */
  double logdet1;        /* log|K~_1| at the current length-scale */
  double mh_log_ratio;   /* D of the last Metropolis step (0 if off grid) */
  int32_t status;        /* device status word (FG_OK or a negative code) */
  int32_t pcg_iters;     /* FG_MIXED: PCG iterations of the last f-draw (0 in FP64) */
  double pcg_relres;     /* FG_MIXED: its final relative residual */
  int32_t precision_used;/* precision of M~'s factor now: an FG_MIXED chain moves to FG_FP64
                            for good when the FP32 factor fails as a preconditioner
                            (kappa(M~) u32 ~ 1: non-finite or no convergence in 30 steps) */
} fg_chain_snapshot;

/* x, y: device n-vectors (x sorted); copied.  Builds and factors K~_1 at ell0. */
fg_status gibbs_chain_create(const fg_chain_cfg* cfg, const double* x, const double* y,
                             int64_t n, fg_stream stream, fg_chain* out);
/* Runs `iters` sweeps.  Synchronises once per sweep (the accepted length-scale
 * selects which cached factor the next sweep uses). */
fg_status gibbs_step(fg_chain c, int32_t iters, fg_stream stream);
/* ---------------------------------------------------------------------------
 * gibbs_step_batch -- `iters` sweeps of each of `nchains` distinct chains (any sizes and
 * precisions), with one host synchronisation per batched sweep instead of one per chain.
 * `mode`:
 *   FG_BATCH_EAGER    each chain's launches on one of `nstreams` (1..4) library streams
 *                     (round-robin, default priority);
 *   FG_BATCH_GRAPHS   as EAGER, each chain's sweep captured once per (slot, grid index,
 *                     proposal, FP64 fallback, PCG budget) as a HIP graph and replayed (up
 *                     to 48 captured sweeps per chain);
 *   FG_BATCH_GROUPED  every chain's sweep is recorded, then the chains' launches of the
 *                     same kernel at the same point are issued as ONE grouped launch (its
 *                     blocks partitioned among the chains) on one stream: a batch issues
 *                     about as many launches as one chain;
 *   FG_BATCH_AUTO     an autotuner: the first eight sweeps of a batch signature (chain
 *                     count, largest n, precision) try GROUPED and EAGER on 4 and 2
 *                     streams and GRAPHS on 4, two sweeps each, the second timed; the
 *                     fastest is kept for that signature (gibbs_batch_tuning reports it).
 * While a kernel timer runs every mode runs as EAGER.  Results are identical to
 * gibbs_step on each chain in every mode: chains share no buffers, every reduction is
 * deterministic and the same kernels run on the same data.  The batch starts after the
 * work queued on `stream` and has finished when the call returns.
 * Errors: FG_EINVAL (NULL or repeated chain, nstreams or mode out of range), FG_EDEVICE.
 * ------------------------------------------------------------------------- */
#define FG_BATCH_EAGER 0
#define FG_BATCH_GRAPHS 1
#define FG_BATCH_GROUPED 2
#define FG_BATCH_AUTO 3
fg_status gibbs_step_batch(fg_chain* chains, int32_t nchains, int32_t iters, int32_t nstreams,
                           int32_t mode, fg_stream stream);
/* The autotuner's choice for this batch's signature: *mode (-1 while still tuning),
 * *nstreams and *ms_per_sweep (host, may be NULL) of the timed trial sweep. */
fg_status gibbs_batch_tuning(fg_chain* chains, int32_t nchains, int32_t* mode, int32_t* nstreams,
                             double* ms_per_sweep);
/* Host snapshot of the scalars; if f_out (device, n) is not NULL it receives f
 * (and r_out, mu_out likewise: Sigma~^-1 y and K~ r of the last f-draw). */
fg_status gibbs_chain_state(fg_chain c, fg_chain_snapshot* host_out, double* f_out,
                            double* r_out, double* mu_out, fg_stream stream);

/* ---------------------------------------------------------------------------
 * gibbs_chain_create_grid -- as gibbs_chain_create, with the length-scale drawn from its
 * exact discrete conditional (Section 4.1, the fourth conditional; uniform prior over the
 * grid) in place of the Metropolis step: every grid point's K~_1, W_1 and log det K~_1 are
 * built once at creation and kept on the device (grid_size factorizations: memory grows
 * with grid_size, see chain_device_bytes), and each sweep computes q_h = |W_h^-1 f|^2 for
 * every h on four library streams, then draws h with probability proportional to
 * exp(-1/2 log det K~_1(s_h) - q_h / (2 sigma_f^2)) by inverse CDF with the Philox uniform
 * of tag 9 (the first h whose cumulative weight exceeds u times the total).  In the
 * snapshot, last_proposal is the drawn index, last_accept whether it differs from the
 * previous one, mh_log_ratio the drawn index's log-probability and q its q_h.  FP64 only.
 * Errors: as gibbs_chain_create; FG_ENOTSPD if a grid point's K~_1 is not positive
 * definite; FG_ENOMEM when the grid does not fit.
 * ------------------------------------------------------------------------- */
fg_status gibbs_chain_create_grid(const fg_chain_cfg* cfg, const double* x, const double* y,
                                  int64_t n, fg_stream stream, fg_chain* out);

/* ---------------------------------------------------------------------------
 * Non-unique inputs (Appendix, "Non-unique input points").
 * gibbs_chain_create_collapsed -- as gibbs_chain_create, for n observations (x, y on the
 *   device, any order) whose inputs may repeat.  The U distinct inputs (ascending) with
 *   counts |Q_i| and averages ybar_i are formed on the host, and the chain runs on them:
 *   f | - is Algorithm 1.h with noise precisions |Q_i| tau (the mean of |Q_i| independent
 *   observations of precision tau; the paper prints |Q_i|^2 tau), computed on g = f /
 *   sigma_f with prior K~_1 and f = sigma_f g; tau | - ~ Ga((a1 + n)/2, (b1 + SSE)/2)
 *   with the full-data SSE = sum_i |Q_i| (ybar_i - f_i)^2 + the within-group sum of
 *   squares; sigma_f^-2 and the length-scale steps are those of the plain chain on the U
 *   inputs.  The snapshot's loglik is that of the averages, ybar ~ N(0, sigma_f^2 K~_1 +
 *   diag(1 / (tau |Q_i|))), and its sse the full-data SSE; f, r and mu have U entries.
 *   FP64 only.  Errors: as gibbs_chain_create, FG_EINVAL for FG_MIXED or a NaN input.
 * gibbs_chain_inputs -- the chain's input count U, the observation count n (U for a plain
 *   chain), and, when the device pointers are not NULL, its U inputs and counts.
 * ------------------------------------------------------------------------- */
fg_status gibbs_chain_create_collapsed(const fg_chain_cfg* cfg, const double* x, const double* y,
                                       int64_t n, fg_stream stream, fg_chain* out);
fg_status gibbs_chain_inputs(fg_chain c, int64_t* n_points, int64_t* n_obs, double* x_out,
                             double* counts_out, fg_stream stream);

/* ---------------------------------------------------------------------------
 * Function posterior at new inputs (Appendix, "Function posterior at new inputs").
 * Given the chain's state after its last sweep -- f, sigma_f^2 and the length-scale's
 * K~_1 = K_1 + eta I with its factor W_1 -- each new input x*_j has
 *   f*_j | f ~ N(mu*_j, s2*_j),
 *   mu*_j = k1(x*_j, X) K~_1^-1 f,
 *   s2*_j = sigma_f^2 (1 + eta - k1(x*_j, X) K~_1^-1 k1(X, x*_j)),
 * with the nugget read as part of the process (it enters k** as it enters K~_1's diagonal).
 * The points are drawn from their marginals, independently of each other.  Both terms go
 * through the factor: with z = W_1^-1 f and Z_j = W_1^-1 k1(X, x*_j),
 * mu*_j = Z_j . z and s2*_j = sigma_f^2 (1 + eta - |Z_j|^2).
 *
 * gibbs_predict_inputs -- copies `nstar` new inputs (device, any order; 0 clears them)
 *   into the chain.  Z depends on the length-scale only, so the chain keeps it for up to
 *   `max_grid_points` grid points at once (least recently used evicted; each costs
 *   8 n nstar bytes of device memory, owned by the chain and freed with it or by the next
 *   call) -- the pre-solve per grid value the paper suggests.  The first buffer is
 *   allocated here, the others on first use (a failed allocation there evicts instead).
 *   Synchronises `stream` first.
 *   Errors: FG_EINVAL (NULL, nstar < 0 or > 65535 * 4, max_grid_points < 1), FG_ENOMEM.
 * gibbs_predict -- one draw per new input: fstar (device, nstar) receives f*, and mu and
 *   s2 (device, nstar; either may be NULL) the mean and variance.  The normals are the
 *   Philox stream with tag 8 at iteration = the number of sweeps the chain has made.  Each
 *   call costs one W_1^-1 f and two length-n reductions per new input, plus, when Z of the
 *   current grid point is not cached, the kernel columns and nstar / 4 inverse
 *   applications of W_1.  Enqueued on `stream`, no synchronisation.
 *   Errors: FG_EINVAL (NULL fstar, no inputs set), FG_EDEVICE.
 * gibbs_predict_stats -- grid points whose Z is cached, and Z computations so far.
 * ------------------------------------------------------------------------- */
fg_status gibbs_predict_inputs(fg_chain c, const double* xstar, int64_t nstar,
                               int32_t max_grid_points, fg_stream stream);
fg_status gibbs_predict(fg_chain c, double* fstar, double* mu, double* s2, fg_stream stream);
fg_status gibbs_predict_stats(fg_chain c, int32_t* cached_grid_points, int64_t* builds);

/* ---------------------------------------------------------------------------
 * Tensor-product surface chain (Section 4.2): y_i = beta prod_h f_h(x[h,i]) + e_i,
 * e_i ~ N(0, 1/tau), f_h unit-variance GPs (kernel `kind`, length-scale on a grid
 * per factor).  One sweep, in order:
 *   f_h | -  for h = 0..d-1 by Algorithm 1.h on dimension h's sorted inputs, with
 *            g_i = beta prod_{k != h} f_k(x[k,i]), D = tau g^2, observations y/g
 *            (|g| floored at 1e-150, sign kept, zero taken as positive);
 *   beta | - ~ N(tau G'y / p, 1/p), p = tau G'G + 1/s_beta^2, G_i = prod_h f_h;
 *   tau  | - ~ Ga((a1+n)/2, (b1 + |y - beta G|^2)/2);
 *   ell_h | - for h = 0..d-1: grid Metropolis step as in the 1-D chain with the
 *            unit-variance prior, D = -1/2 (log|K~_h'| - log|K~_h|) - (q' - q)/2.
 * Start: f_h = 1, beta = beta0, tau = tau0, every grid index at grid_center.
 * Random numbers: factor h uses the 1-D tags plus 16 (h+1) (a, b, proposal,
 * acceptance); tau uses tag 3; beta the normal of tag 7.
 *
 * Additive tensor products (Sections 4.2 and 5.2), ncomp = C > 1 components:
 * y_i = sum_c beta_c prod_h f_{c,h}(x[h,i]) + e_i.  Factor m = c d + h (C d <= 8).  For
 * c = 0..C-1: component c's factors are drawn as above from the partial residual
 * r_c = y - sum_{c' != c} beta_c' G_c' in place of y, then beta_c | - from r_c; then tau
 * from the full residual; then every factor's length-scale.  beta_c's normal uses tag 7
 * for c = 0 and 7 + 16 (9 + c) otherwise.  With C = 1 this is the sweep above.
 * ------------------------------------------------------------------------- */
typedef struct {
  int32_t kind;          /* FG_KERNEL_SE / _EXP / _MATERN32 / _MATERN52 */
  int32_t d;             /* number of input dimensions, 1..8 */
  double ell0[8];        /* grid centre length-scale per factor m = c d + h */
  double nugget;         /* added to every K_h's diagonal */
  int32_t leaf;          /* maximum leaf size */
  double tol;            /* max-norm tolerance on each K_h */
  double tau0, beta0;    /* start values */
  double a1, b1;         /* tau ~ Ga(a1/2, b1/2) */
  double s_beta;         /* beta ~ N(0, s_beta^2) */
  int32_t grid_size;     /* length-scales per factor */
  int32_t grid_center;   /* starting index */
  uint64_t seed;
  uint64_t stream_id;
  int32_t ncomp;         /* additive components C, 1..4 (0 is read as 1), C d <= 8 */
} fg_tp_cfg;

typedef struct {
  int64_t iteration;
  double tau, beta;
  double sse;                /* |y - beta G|^2 of the last tau step */
  double beta_mean, beta_sd; /* moments of the last beta draw */
  int32_t k[8];              /* grid index per factor */
  int32_t last_proposal[8];
  int32_t last_accept[8];
  int32_t accepts[8];
  double ell[8];
  double logdet[8];          /* log|K~_h| at the current length-scales */
  double q[8];               /* f_h' K~_h^-1 f_h at the current length-scales */
  double mh_log_ratio[8];
  int32_t status;
  int32_t ncomp;
  double betas[4];           /* beta_c per component (betas[0] == beta) */
  double beta_means[4], beta_sds[4];
} fg_tp_snapshot;

/* x: device d x n (row h = dimension h, observation order, any order of values);
 * y: device n.  Both copied; each dimension is sorted on the host (stable).
 * Synchronises the stream.  Errors: FG_EINVAL, FG_ETOL, FG_ENOMEM, FG_EDEVICE. */
fg_status tp_chain_create(const fg_tp_cfg* cfg, const double* x, const double* y, int64_t n,
                          fg_stream stream, fg_tp_chain* out);
/* Runs `iters` sweeps; synchronises once per sweep. */
fg_status tp_step(fg_tp_chain c, int32_t iters, fg_stream stream);
/* Host snapshot; F_out (device (C d) x n, observation order, or NULL) receives
 * f_m(x[m mod d, i]) for every factor m.  The per-factor arrays hold C d entries. */
fg_status tp_chain_state(fg_tp_chain c, fg_tp_snapshot* host_out, double* F_out,
                         fg_stream stream);

/* Host-only count of the device bytes gibbs_chain_create(cfg) takes for these inputs
 * (x host, sorted): every grid point is planned on the host and the buffers are sized
 * for the largest, as the chain does.  A mixed-precision chain's count includes the FP64
 * factor of M~ it allocates if it falls back to FP64.  No device call. */
fg_status fg_footprint_bytes(const fg_chain_cfg* cfg, const double* x_host, int64_t n,
                             uint64_t* bytes);

/* ---------------------------------------------------------------------------
 * Serving (a request loop for GP-regression jobs, with continuous batching).  A job is
 * one Gibbs chain (Section 4.1's sweep) on (x, y) run for `iters` sweeps.
 *   - serve_create allocates the whole device budget once (an arena of mem_budget bytes)
 *     and max_active slots, each with its own streams.
 *   - Planner threads make a submitted job's host plans and its exact device footprint
 *     (fg_footprint_bytes plus the rounding of each allocation).
 *   - A worker thread admits planned jobs in arrival order (head of line) while a slot is
 *     free and a block of the job's footprint can be carved from the arena; the job's
 *     chain lives in that block.  The worker makes no runtime allocation.
 *   - Every running job advances on its own stream: when its last sweep has finished the
 *     worker enqueues the next one, or retires the job (result, block returned) and
 *     admits the next at once.  The sweeps of all running jobs overlap on the device.
 *   - A job that can never fit (footprint above mem_budget) fails with FG_ENOMEM; a
 *     mixed-precision job whose FP32 leaf factor stops being a preconditioner and whose
 *     block has no room for an FP64 factor ends with FG_ENOTCONV.
 * Each job's result is the result of the same chain run alone (gibbs_step).  Times are
 * seconds since serve_create (steady clock).
 * ------------------------------------------------------------------------- */
typedef struct fg_server_s* fg_server;
typedef struct {
  uint64_t mem_budget;   /* device bytes for running jobs (> 0), allocated at creation */
  int32_t max_active;    /* most jobs running at once (1..256) */
} fg_serve_cfg;
typedef struct {
  const double* x;       /* host, n sorted inputs (copied at submission) */
  const double* y;       /* host, n observations (copied) */
  int64_t n;
  int32_t kind;
  double ell0, nugget;
  int32_t leaf;
  double tol, tau0, sigf2_0;
  int32_t iters;         /* sweeps to run */
  uint64_t seed, stream_id;
  int32_t precision;     /* FG_FP64 / FG_MIXED */
  double* f_out;         /* host, n doubles or NULL: the last draw of f; must stay valid
                            until the job's result has been polled */
} fg_job;
typedef struct {
  uint64_t id;
  int32_t status;        /* FG_OK or the job's error */
  fg_chain_snapshot snap;
  double t_submit, t_admit, t_done;
  uint64_t bytes;        /* device bytes the job held */
} fg_result;
typedef struct {
  int64_t pending, outstanding, sweeps;
  uint64_t peak_bytes;   /* most bytes held by running jobs at once */
} fg_serve_stats;
fg_status serve_create(const fg_serve_cfg* cfg, fg_server* out);
/* Copies the request and queues it; *id (may be NULL) receives its id. */
fg_status serve_submit(fg_server s, const fg_job* job, uint64_t* id);
/* Moves up to `max` finished results into out (host); *got = how many. */
fg_status serve_poll(fg_server s, fg_result* out, int32_t max, int32_t* got);
/* Blocks until every submitted job has finished (FG_ENOTCONV after timeout_s). */
fg_status serve_drain(fg_server s, double timeout_s);
fg_status serve_stats(fg_server s, fg_serve_stats* out);
/* Stops the worker after its current sweep and frees every running job. */
void serve_destroy(fg_server s);

/* ---------------------------------------------------------------------------
 * Live kernel timing (diagnostics).  fg_timer_start(id) makes the library record
 * HIP events, on the launch stream, around every following launch of kernel `id`
 * (FG_KID_LEAF: leaf Cholesky and inverse; FG_KID_REDUCE: level Gram reduction;
 * FG_KID_UPDATE: level update of the coarser panels; FG_KID_WHITEN: whitening of every
 * panel row by the leaf inverses, on matrix cores; FG_KID_PREDICT: the per-point
 * reductions of gibbs_predict).  fg_timer_stop
 * synchronises the device and returns the summed kernel time (ms), the launch count
 * and the algorithmic HBM bytes of those launches (each kernel's minimum traffic:
 * every operand read once and every result written once).
 * ------------------------------------------------------------------------- */
#define FG_KID_LEAF 1
#define FG_KID_REDUCE 2
#define FG_KID_UPDATE 3
#define FG_KID_WHITEN 4
#define FG_KID_PREDICT 5
fg_status fg_timer_start(int32_t kernel_id);
fg_status fg_timer_stop(double* total_ms, int64_t* launches, double* bytes);
/* fg_timer_start for several kernels at once: bit k of `mask` times kernel id k
 * (FG_KID_*).  fg_timer_stop then returns the sums over all of them, and
 * fg_timer_result(k, ...) the figures of kernel k alone from that stop.  The timer
 * state is guarded by a mutex; launches from any host thread are recorded. */
fg_status fg_timer_start_mask(uint32_t mask);
fg_status fg_timer_result(int32_t kernel_id, double* total_ms, int64_t* launches, double* bytes);

/* Status word of a handle (synchronises the stream first). */
fg_status hodlr_status(fg_hodlr A, fg_stream stream);
fg_status factor_status(fg_factor F, fg_stream stream);

const char* fg_last_error(void);
void hodlr_destroy(fg_hodlr A);
void factor_destroy(fg_factor F);
void gibbs_chain_destroy(fg_chain c);
void tp_chain_destroy(fg_tp_chain c);

#ifdef __cplusplus
}
#endif
#endif /* FIFA_GP_H */
