/*
 * iht.h -- C ABI of the MI355X (gfx950) hot path of iterative hard thresholding for GWAS.
 *
 * Method: Keys, Chen & Lange, "Iterative hard thresholding for model selection in genome-wide
 * association studies" (arXiv:1608.01398). The library minimises the least-squares loss
 * f(beta) = 1/2 ||y - A beta||^2 (Methods, eq. leastsquaresloss) subject to at most k nonzero SNP
 * effects, with A = [X_st | Z | 1]: X_st the standardised genotype matrix (Methods, "Bandwidth
 * optimization of IHT"), Z dense non-genetic covariates and an intercept, both unpenalised
 * (Results: SexOCPG and principal components enter as covariates). Option IHT_LOGISTIC replaces
 * f by the logistic negative log-likelihood (the extension the Discussion names).
 *
 * Entry points: the resident matrix (iht_geno_*) and its per-subject-set standardisation
 * (iht_stats_*); the gradient pass for one residual (iht_gradient) and for many on the matrix cores
 * (iht_gradient_batch); the projection (iht_project, iht_project_hint); whole fits, one or many in
 * lock-step (iht_fit, iht_fit_batch); model selection by cross-validation (iht_cv) and prediction
 * (iht_predict); a continuous-batching solve server (iht_server_*); introspection
 * (iht_batch_tuning, iht_status_str, iht_last_error).
 *
 * Conventions shared by every entry point:
 *  - Return value: IHT_OK (0) on success; > 0 means a valid result with a warning; < 0 is an error,
 *    raised before any device work is enqueued whenever it is an argument error. Details of the
 *    last error on the calling thread: iht_last_error(). No C++ exception crosses this ABI.
 *  - `stream` is a hipStream_t (NULL = the default stream). All device work is enqueued on it.
 *    Device-pointer outputs are valid once the stream has been synchronised. Calls that return
 *    host-side values (iht_fit's n_iter, the status of iht_project and iht_fit) synchronise the
 *    stream themselves.
 *  - Ownership: the caller owns every input and output buffer and keeps it alive for the call;
 *    handles own their device memory and free it in the matching *_destroy.
 *  - Threading: a handle must not be used by two threads at once, and the calls on one genotype handle
 *    must go to one stream (iht_gradient, iht_gradient_batch and fits without a workspace share the
 *    handle's device scratch); distinct handles are independent.
 *  - Genotypes: PLINK 1 SNP-major .bed rows. SNP j occupies `row_bytes` bytes; subject i is in byte
 *    i/4 at bits 2(i%4) (low) and 2(i%4)+1 (high); two-bit value 0 = homozygous first allele
 *    (dosage 0), 1 = missing, 2 = heterozygous (dosage 1), 3 = homozygous second allele (dosage 2).
 *  - Standardisation (Methods, "Bandwidth optimization of IHT"; Results, "Simulation"): over the
 *    subject set T of a stats handle, u_j is the mean of the observed dosages, sigma_j^2 the
 *    population variance of the mean-imputed column over all |T| subjects, v_j = 1/sigma_j
 *    (v_j = 0 when sigma_j = 0), and x_st(i,j) = v_j (x_ij - u_j) with missing entries exactly 0.
 */
#ifndef IHT_H
#define IHT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define IHT_OK 0
#define IHT_NOT_CONVERGED 1 /* max_iter reached; outputs hold the last iterate          */
#define IHT_STALLED 2       /* backtracking budget exhausted; outputs hold the last accepted iterate */
#define IHT_EINVAL (-1)     /* bad argument (NULL, sizes, k out of range, subset not 0/1) */
#define IHT_ENOMEM (-2)     /* device allocation failed                                   */
#define IHT_EDEVICE (-3)    /* a HIP runtime call or kernel launch failed                 */
#define IHT_ENONFINITE (-4) /* NaN or Inf in y, Z, r or w                                 */
#define IHT_EUNSUPPORTED (-5)

/* arithmetic of the gradient pass */
#define IHT_FP64 0     /* table entries and accumulation in FP64 (default)                          */
#define IHT_FP32 1     /* table entries in FP32, per-tile FP32 sums accumulated in FP64              */
#define IHT_MIXED_I8 2 /* fits only: one matrix-core pass per iteration for all solves (int8 genotype */
                       /* and residual-digit operands, exact int32 sums, FP64 combination), with the */
                       /* FP64 iteration's decisions (see iht_opts)                                  */

/* model family of a fit (iht_opts.family) */
#define IHT_GAUSSIAN 0 /* least squares, f = 1/2 ||y - A beta||^2 (Methods, eq. leastsquaresloss)    */
#define IHT_LOGISTIC 1 /* logistic regression, f = sum_T [log(1 + e^eta) - y eta], eta = A beta, y in */
                       /* [0, 1] (the extension the Discussion names); IHT_FP64 only                 */

/* iht_geno_create flags: where `bed` lives */
#define IHT_HOST_PTR 0
#define IHT_DEVICE_PTR 1

/* Largest sparsity level the device projection accepts. */
#define IHT_MAX_K 4096

typedef struct iht_geno iht_geno;   /* resident, re-tiled genotype matrix on one device */
typedef struct iht_stats iht_stats; /* u, v [p] FP64 and the subject set T they were computed on */

/*
 * Options of iht_fit and iht_fit_batch. The paper fixes none of them (Methods, "IHT step sizes"
 * only asks 0 < c << 1). IHT_MIXED_I8 takes the decisions of the FP64 iteration (Results, "Analysis
 * of compressed data with IHT", weighs single against double precision): the matrix-core gradient
 * is within a bound of the exact one that the pass itself reports (the residual's quantisation
 * error), the gradient on the support is recomputed in FP64 from the decoded support columns, and
 * every projection is certified: the entries whose value lies within that bound of the k-th largest
 * are recomputed in FP64 before the selection. Supports, step sizes, backtracking and the stopping
 * rule (at tol) are then those of IHT_FP64; k <= 512 and n <= 8 454 660 subjects (the int32 sums
 * stay exact while 254 n <= 2^31 - 1), else IHT_EUNSUPPORTED. With IHT_FP32 the
 * iteration stops at max(tol, mixed_tol); each converged solve is then refined in FP64 on its final
 * support to the least-squares fit on S and the unpenalised columns (the fixed point of the IHT map
 * on a fixed support), with at most polish_iter conjugate-gradient steps and the stopping rule at tol.
 * IHT_LOGISTIC: the residual is y - sigma(eta), so the same gradient pass gives A^T r = -grad f; the
 * step is mu = ||g_{S u C}||^2 / sum_T w_i (A_{S u C} g_{S u C})_i^2 with w = sigma(eta)(1 - sigma(eta))
 * at the current beta, and a proposal is taken when f does not increase by more than 1e-12 |f| (the
 * rounding of the loss sums; else mu is halved, at most
 * max_backtrack times; c is not used). A y outside [0, 1] inside the subject set is reported as
 * IHT_ENONFINITE. Only with IHT_FP64 (else IHT_EUNSUPPORTED); not in iht_cv.
 */
typedef struct iht_opts {
    double tol;            /* stop when S+ = S and ||beta+ - beta||_inf <= tol*max(1,||beta+||_inf); default 1e-10 */
    int32_t max_iter;      /* default 200                                                   */
    int32_t max_backtrack; /* step halvings allowed per iteration; default 50               */
    double c;              /* omega = (1-c)||d||^2/||A d||^2, 0 < c < 1; default 0.01        */
    double shrink;         /* mu <- shrink*mu on each backtrack, 0 < shrink < 1; default 0.5 */
    int32_t precision;     /* IHT_FP64, IHT_FP32 or IHT_MIXED_I8; default IHT_FP64          */
    double mixed_tol;      /* iteration tolerance of IHT_FP32; default 1e-6                 */
    int32_t polish_iter;   /* FP64 refinement steps after an IHT_FP32 solve; default 200    */
    int32_t family;        /* IHT_GAUSSIAN (default) or IHT_LOGISTIC                        */
    void *workspace;       /* NULL (default): the solve state lives in the genotype handle (device */
                           /* memory allocated on first use, grown and reused); else device memory */
                           /* of at least iht_workspace_bytes[_batch] bytes, 256-byte aligned     */
    uint64_t workspace_bytes; /* size of workspace                                           */
} iht_opts;

/* Fill *o with the defaults above. */
void iht_opts_default(iht_opts *o);

/*
 * Device memory of one solve's state (Methods, "Penalized regression": the problem is fixed by n,
 * p, the model size k and the unpenalised columns): the size of the workspace that iht_fit takes
 * through iht_opts.workspace for n subjects, p SNPs, k and c unpenalised columns (covariates plus
 * the intercept column), at `precision`. With a workspace, iht_fit and iht_fit_batch allocate no
 * device memory (they keep a small pinned host staging area per genotype handle, allocated on its
 * first use); the caller owns the workspace, keeps it alive until the call returns, and must not
 * use it from two calls at once; its contents on entry do not matter and on return are undefined.
 * iht_cv and the server ignore iht_opts.workspace. Returns 0 for arguments out of range
 * (n, p, k < 1, c < 0 or c > 64).
 */
size_t iht_workspace_bytes(int64_t n, int64_t p, int32_t k, int32_t c, int32_t precision);
/* The same for iht_fit_batch with T solves of model sizes up to kmax. */
size_t iht_workspace_bytes_batch(int64_t n, int64_t p, int32_t T, int32_t kmax, int32_t c, int32_t precision);

/*
 * Upload (if IHT_HOST_PTR) and re-tile a PLINK SNP-major matrix once onto the current device
 * (Methods, "Parallelization of IHT": the compressed matrix is pushed to the device once).
 *   bed        [p][row_bytes] bytes, host or device memory per `flags`; only read during the call.
 *   n, p       subjects and SNPs, n >= 1, p >= 1, n <= 2^24, p <= 2^28 - 8192.
 *   row_bytes  >= ceil(n/4); bits past subject n-1 are ignored.
 *   out        receives the handle.
 * Errors: IHT_EINVAL, IHT_ENOMEM, IHT_EDEVICE. The stream is synchronised before returning.
 */
int iht_geno_create(const uint8_t *bed, int64_t n, int64_t p, int64_t row_bytes, int32_t flags, void *stream, iht_geno **out);
/*
 * The same with device memory the caller owns (for callers whose allocator owns every device
 * buffer, e.g. PyTorch's): bed is device memory ([p][row_bytes]), and the re-tiled matrix is written
 * into dst, at least iht_geno_bytes(n, p) bytes of device memory, 256-byte aligned. The handle
 * borrows dst: creating it allocates no device memory, iht_geno_destroy leaves dst to the caller,
 * and the caller keeps dst alive and unmodified while the handle lives. The work areas that later
 * calls on the handle allocate on first use (iht_fit's solve state without a workspace, the scratch
 * of iht_gradient and iht_gradient_batch) are the handle's own as with iht_geno_create;
 * iht_gradient_noalloc and iht_fit with a workspace need none.
 * Errors: IHT_EINVAL (also dst NULL, misaligned or too small), IHT_EDEVICE. Stream synchronised.
 */
uint64_t iht_geno_bytes(int64_t n, int64_t p); /* 0 for n or p out of range */
int iht_geno_create_in(const uint8_t *bed, int64_t n, int64_t p, int64_t row_bytes, void *dst, uint64_t dst_bytes,
                       void *stream, iht_geno **out);
int iht_geno_destroy(iht_geno *g);
/* n, p of a handle (either output may be NULL). */
int iht_geno_shape(const iht_geno *g, int64_t *n, int64_t *p);

/*
 * Per-SNP standardisation cache u, v over the subject set T (Methods, "Bandwidth optimization of
 * IHT": precompute and cache the means and inverse standard deviations).
 *   subset  host array of n bytes, each 0 or 1 (1 = subject in T), or NULL for all n subjects;
 *           |T| >= 1. A solve on T equals the solve on the matrix restricted to the rows in T.
 * The counts are exact integers and u_j, sigma_j^2, sqrt and 1/sqrt are single IEEE operations,
 * so u and v are bitwise reproducible. Errors: IHT_EINVAL, IHT_ENOMEM, IHT_EDEVICE.
 */
int iht_stats_create(const iht_geno *g, const uint8_t *subset, void *stream, iht_stats **out);
/*
 * The same in device memory the caller owns: u, v, the subject mask and bits are written into dst,
 * at least iht_stats_bytes(g) bytes, 256-byte aligned, which the handle borrows (no device
 * allocation; iht_stats_destroy leaves dst to the caller, who keeps it alive and unmodified while
 * the handle lives). Errors as iht_stats_create, plus IHT_EINVAL for dst NULL, misaligned or too small.
 */
uint64_t iht_stats_bytes(const iht_geno *g); /* 0 for a NULL handle */
int iht_stats_create_in(const iht_geno *g, const uint8_t *subset, void *dst, uint64_t dst_bytes, void *stream,
                        iht_stats **out);
int iht_stats_destroy(iht_stats *s);
/* Copy u and v (device pointers, p doubles each; either may be NULL) out of a stats handle. */
int iht_stats_read(const iht_stats *s, double *u, double *v, void *stream);

/*
 * Gradient pass g = X_st^T r over T (Methods, eq. normal_grad: g = -grad f at r = y - X beta).
 *   r  device [n] FP64 residuals; entries of subjects outside T are ignored.
 *   g  device [p] FP64 output.
 *   precision  IHT_FP64 or IHT_FP32.
 * Every SNP column is decoded and standardised on the fly from the packed bytes (Methods,
 * "Bandwidth optimization of IHT"). Errors: IHT_EINVAL (stats of another matrix, bad precision),
 * IHT_EDEVICE. Asynchronous; r must stay valid until the stream reaches the work.
 */
int iht_gradient(const iht_geno *g, const iht_stats *s, const double *r, double *grad, int32_t precision, void *stream);

/*
 * iht_gradient for callers that cannot allocate device memory (code under stream capture, tight
 * serving loops, harnesses that forbid allocation): the same kernels and bitwise the same result,
 * with the pass's scratch (centring scalars, centred residual, split partial sums) in one fixed
 * array of device memory per GPU (18 MB, held until the process ends) instead of memory the handle
 * allocates on first use. Calls nothing that allocates. The array keeps the last call's contents;
 * every call rewrites what it reads. Calls that overlap on one GPU (other streams, other threads,
 * other handles) race on the array and must be serialised by the caller. The current device must
 * be the handle's.
 *   Arguments as iht_gradient. Limit: the matrix's scratch (8 bytes per padded subject plus the
 *   partial sums of a split pass, at most 16 MB) must fit iht_gradient_noalloc_max_bytes(): every p
 *   with n <= 262,144. Errors: IHT_EINVAL (also past that limit, before any device work),
 *   IHT_EDEVICE. Asynchronous, as iht_gradient.
 */
int iht_gradient_noalloc(const iht_geno *g, const iht_stats *s, const double *r, double *grad, int32_t precision,
                         void *stream);
/* Bytes of the fixed scratch available to iht_gradient_noalloc's gradient work area. */
size_t iht_gradient_noalloc_max_bytes(void);

/*
 * Batched gradient pass G_t = X_st^T r_t for T solves sharing the genotype matrix (the many traits,
 * cross-validation folds and model sizes of Methods, "Model selection"), each over its own subject
 * set and standardisation. Runs on the matrix cores: dosages and missing flags as int8 against the
 * residual split into three int8 digits under a power-of-two scale, with exact int32 sums combined
 * in FP64; the only approximation is that quantisation (relative error ~1e-7 of max|r_t|).
 *   stats  host array of T stats handles of this matrix (handles may repeat).
 *   R      device [T][n] FP64 residuals (row t for solve t); entries outside a solve's set ignored.
 *   G      device [T][p] FP64 output (row t = gradient of solve t).
 *   1 <= T <= 65535; n <= 8 454 660 (the int32 sums stay exact while 254 n <= 2^31 - 1), else
 *   IHT_EUNSUPPORTED. Errors: IHT_EINVAL, IHT_EUNSUPPORTED, IHT_ENOMEM, IHT_EDEVICE. Synchronises
 *   the stream.
 */
int iht_gradient_batch(const iht_geno *g, const iht_stats *const *stats, int32_t T, const double *R, double *G, void *stream);

/*
 * Hard-threshold projection P_Sk (Methods, eq. ihta and the text after it): keep the k entries of
 * largest |w|, ties broken towards the lower index, zero the rest.
 *   w        device [p] FP64, finite.
 *   support  device [k] int64 output, ascending.
 *   w_out    device [p] FP64 output (w on the support, 0 elsewhere) or NULL.
 *   1 <= k <= min(p, IHT_MAX_K).
 * Errors: IHT_EINVAL, IHT_ENONFINITE (detected on the device; the call synchronises), IHT_EDEVICE.
 */
int iht_project(const double *w, int64_t p, int32_t k, int64_t *support, double *w_out, void *stream);

/*
 * The same projection, warm-started (the IHT loop of Methods, eq. ihta, projects beta + mu g whose
 * support moves little between iterations): `hint` holds k distinct indices (e.g. the previous
 * support), so the smallest |w| over them bounds the k-th largest from below and one filtering pass
 * over w keeps the entries at or above it; the k largest are then selected among those. The result
 * is the one of iht_project for any valid hint; the hint only changes the cost.
 *   hint     device [k] int64, distinct indices in [0, p) (an index outside [0, p) gives no bound).
 * Used for k <= 512; larger k take iht_project's path. Errors: as iht_project, and IHT_EINVAL if the
 * hint repeats an index so that fewer than k entries reach its bound.
 */
int iht_project_hint(const double *w, int64_t p, int32_t k, const int64_t *hint, int64_t *support, double *w_out,
                     void *stream);

/*
 * Full IHT solve (Methods, eq. ihta with the normalised step and the omega backtracking rule of
 * "IHT step sizes"): beta <- P_Sk[beta + mu A^T(y - A beta)], beta^0 = 0,
 * mu = ||g_{S u C}||^2 / ||A_{S u C} g_{S u C}||^2 with C the unpenalised columns; when the support
 * changes, mu is halved until mu < omega = (1-c)||beta+ - beta||^2 / ||A(beta+ - beta)||^2.
 *   y          device [n] FP64 trait; entries outside T are ignored.
 *   Z          device FP32 covariates, column-major [n x cz] (covariate c at Z + c*n), or NULL if cz = 0.
 *   intercept  1 to include an unpenalised column of ones.
 *   k          1 <= k <= min(p, IHT_MAX_K) SNPs in the model.
 *   opts       NULL for the defaults.
 *   support    device [k] int64 output, ascending SNP indices.
 *   beta_S     device [k] FP64 output, effects on `support`.
 *   beta_cov   device [cz + intercept] FP64 output (covariates, then intercept), or NULL if empty.
 *   loss_trace device [max_iter + 1] FP64 output: f at beta^0 .. beta^{n_iter}.
 *   n_iter     host int32 output: iterations performed.
 * Returns IHT_OK, IHT_NOT_CONVERGED, IHT_STALLED, or an error (IHT_EINVAL, IHT_ENONFINITE,
 * IHT_ENOMEM, IHT_EDEVICE; IHT_EINVAL also for a workspace smaller than iht_workspace_bytes or not
 * 256-byte aligned). Synchronises the stream. Same as iht_fit_batch with T = 1.
 */
int iht_fit(const iht_geno *g, const iht_stats *s, const double *y, const float *Z, int32_t cz, int32_t intercept, int32_t k,
            const iht_opts *opts, int64_t *support, double *beta_S, double *beta_cov, double *loss_trace, int32_t *n_iter,
            void *stream);

/*
 * Many IHT solves sharing one genotype matrix, advanced in lock-step on the device (the traits,
 * cross-validation folds and model sizes of Methods, "Model selection"). Solve t is exactly the
 * iht_fit of (stats[t], Y + t*ldy, ks[t]) with the shared covariates and options; its result does
 * not depend on the other solves of the call (each one's residual digits, scale and sums are its
 * own), so it is the same alone and in any mix.
 *   stats      host array of T stats handles of this matrix (handles may repeat).
 *   Y          device FP64 traits, row t at Y + t*ldy (ldy >= n).
 *   Z, cz, intercept   as in iht_fit, shared by all solves.
 *   ks         host int32 [T], 1 <= ks[t] <= min(p, IHT_MAX_K); kmax = max ks[t].
 *   support    device int64 [T][kmax]: row t ascending, entries past ks[t] set to -1.
 *   beta_S     device FP64 [T][kmax]: effects on the support, entries past ks[t] set to 0.
 *   beta_cov   device FP64 [T][cz + intercept], or NULL if cz + intercept = 0.
 *   loss_trace device FP64 [T][max_iter + 1]: f at beta^0 .. beta^{n_iter[t]} of each solve (with
 *              IHT_FP32 the last entry is the loss after the FP64 refinement).
 *   n_iter     host int32 [T]: iterations performed by each solve.
 *   status     host int32 [T]: IHT_OK, IHT_NOT_CONVERGED, IHT_STALLED or IHT_ENONFINITE per solve.
 *   precision  IHT_FP64 / IHT_FP32 run one gradient pass per solve and iteration; IHT_MIXED_I8 runs
 *              one matrix-core pass per iteration over the solves that need a new gradient.
 *   1 <= T <= 65535. Returns the most severe per-solve status (an error if any solve had
 *   non-finite input, else the largest warning), or a call-level error (IHT_EINVAL, IHT_ENOMEM,
 *   IHT_EDEVICE). Device memory grows with T (p doubles of beta and gradient per solve, plus the
 *   top-k candidate area of 12 p bytes per solve). Synchronises the stream.
 */
int iht_fit_batch(const iht_geno *g, const iht_stats *const *stats, int32_t T, const double *Y, int64_t ldy, const float *Z,
                  int32_t cz, int32_t intercept, const int32_t *ks, const iht_opts *opts, int64_t *support, double *beta_S,
                  double *beta_cov, double *loss_trace, int32_t *n_iter, int32_t *status, void *stream);

/*
 * q-fold cross-validation over a path of model sizes (Methods, "Model selection"). Subject i is
 * held out in fold folds[i]. For each fold f and each ks[a], IHT is fitted on the other subjects,
 * with the standardisation (u_j, v_j) of those subjects only; the held-out mean squared error is
 * mse[a][f] = (1/|fold f|) sum_{i in fold f} (y_i - x_st,i beta - z_i beta_cov)^2, the held-out
 * genotypes standardised with the training u_j, v_j (a missing genotype counts as 0). The chosen size
 * is the first ks[a] of least mean over the folds; the model of that size is refitted on every
 * subject and returned as by iht_fit.
 *   y, Z, cz, intercept, opts   as in iht_fit (y and Z device memory).
 *   folds      host uint8 [n], each < q; every fold and its complement non-empty.
 *   q          2 <= q <= 64 folds.
 *   ks         host int32 [r], 1 <= ks[a] <= min(p, IHT_MAX_K); 1 <= q * r <= 65535.
 *   mse        host FP64 [r][q] output.
 *   k_best     host int32 output: the chosen model size.
 *   support, beta_S, beta_cov, loss_trace, n_iter   the refit's outputs, as in iht_fit with k = *k_best
 *              (support and beta_S need max ks[a] entries).
 * The q * r training fits run as one batch (iht_fit_batch). Returns the refit's status, or an error
 * (IHT_EINVAL, IHT_ENONFINITE, IHT_ENOMEM, IHT_EDEVICE); warnings of the training fits are not
 * reported. Synchronises the stream.
 */
int iht_cv(const iht_geno *g, const double *y, const float *Z, int32_t cz, int32_t intercept, const uint8_t *folds, int32_t q,
           const int32_t *ks, int32_t r, const iht_opts *opts, double *mse, int32_t *k_best, int64_t *support, double *beta_S,
           double *beta_cov, double *loss_trace, int32_t *n_iter, void *stream);

/*
 * Prediction of every subject by a fitted model: out_i = sum_q x_st(i, support[q]) beta_S[q] +
 * sum_c z_ic beta_cov[c] (+ beta_cov[cz] if intercept), with x_st standardised by the u_j, v_j of s
 * (the X_st beta product of Methods, "Bandwidth optimization of IHT"; a missing dosage is
 * mean-imputed, i.e. 0). The genetic part (cz = 0, intercept = 0) gives the estimated heritability
 * Var(X beta*) / Var(y) of Results, "Simulation"; the subjects of a held-out fold give the MSE of
 * Methods, "Model selection".
 *   s          stats of this matrix whose u, v standardise the columns (e.g. the fit's training set).
 *   support    device int64 [k], entries in [0, p) (any order; repeats add up).
 *   beta_S     device FP64 [k].
 *   k          0 <= k <= p.
 *   Z, cz, intercept   as in iht_fit; beta_cov device FP64 [cz + intercept], or NULL if empty.
 *   out        device FP64 [n] output, every subject (inside s's subject set or not).
 * Errors: IHT_EINVAL (also for a support entry outside [0, p), found on the device; out is then
 * undefined), IHT_ENOMEM, IHT_EDEVICE. Synchronises the stream.
 */
int iht_predict(const iht_geno *g, const iht_stats *s, const int64_t *support, const double *beta_S, int32_t k,
                const float *Z, int32_t cz, int32_t intercept, const double *beta_cov, double *out, void *stream);

/*
 * Solve server with continuous batching (the request loop of many traits, subject subsets and
 * model sizes over one resident matrix; the traits, folds and sizes of Methods, "Model selection",
 * arriving over time). A server owns `slots` solve slots and a pool of per-subject-set statistics
 * blocks, all allocated at creation inside hbm_budget bytes of device memory, so serving allocates
 * nothing. Requests queue in submission order; iht_server_step admits the queued requests that
 * fit (free slots for all their traits and a free statistics block) while the admitted ones
 * iterate, advances every iterating solve by one turn of the solve loop (up to two iterations),
 * and writes the solves that finished into their request's outputs. Each solve is exactly the
 * iht_fit of its (subject set, trait, k) with the server's covariates and options, bitwise the same
 * alone and in any mix of requests. Single-threaded: calls on one server must not overlap.
 *
 * iht_server_create
 *   slots      1 <= slots <= 65535 solves in flight at once.
 *   kmax       largest model size a request may ask for (1 <= kmax <= min(p, IHT_MAX_K)).
 *   hbm_budget device bytes the server may hold: the slot state (p doubles of beta and gradient,
 *              12 p bytes of top-k candidates and 16 kmax n bytes of support columns per slot, ...)
 *              plus as many statistics blocks (16 p + 8 n bytes each) as fit, at most `slots`.
 *              IHT_ENOMEM if not even one block fits beside the slot state.
 *   Z, cz, intercept   covariates shared by every solve (device memory, as in iht_fit; must stay
 *              valid for the server's life).
 *   opts       as in iht_fit (max_iter >= 1); stream: the stream every launch goes to.
 * iht_server_submit
 *   subset     host uint8 [n] of 0/1 (NULL = every subject): the request's subject set.
 *   Y          device FP64 traits, trait j at Y + j*ldy (ldy >= n); read when the request is
 *              admitted, so it must stay valid until then.
 *   T, ks      1 <= T <= slots traits; host int32 [T] model sizes, 1 <= ks[j] <= kmax;
 *              kr = max ks[j].
 *   support, beta_S   device [T][kr] outputs (rows as in iht_fit_batch, -1 / 0 past ks[j]).
 *   beta_cov   device [T][cz + intercept] output, or NULL if empty.
 *   loss_trace device [T][max_iter + 1] output: entries 0 .. n_iter[j] written.
 *   n_iter, status   host int32 [T] outputs (IHT_OK, IHT_NOT_CONVERGED, IHT_STALLED, IHT_ENONFINITE
 *              per trait). Every output must stay valid until the request is done.
 *   id         host int64 output: the request's id (0, 1, 2, ... in submission order).
 * iht_server_step
 *   completed  host int32 output: requests that finished in this step (their outputs are written
 *              when the call returns). Synchronises the stream.
 * iht_server_poll: *done = 1 once request `id` has finished, else 0.
 * iht_server_info: occupancy and footprint.
 * Errors: IHT_EINVAL (arguments; also an unknown id), IHT_ENOMEM, IHT_EDEVICE (after which the
 * server must be destroyed). iht_server_destroy waits for the stream and frees everything.
 */
typedef struct iht_server iht_server;
typedef struct {
  int32_t slots;        /* solve slots                                  */
  int32_t slots_busy;   /* slots holding an admitted solve              */
  int32_t stats_blocks; /* statistics blocks (requests admitted at once) */
  int64_t queued;       /* requests waiting for admission               */
  int64_t running;      /* requests admitted and not finished           */
  int64_t completed;    /* requests finished                            */
  int64_t turns;        /* turns of the solve loop run so far           */
  int64_t device_bytes; /* device memory the server holds               */
} iht_server_info_t;

int iht_server_create(const iht_geno *g, int32_t slots, int32_t kmax, int64_t hbm_budget, const float *Z, int32_t cz,
                      int32_t intercept, const iht_opts *opts, void *stream, iht_server **out);
int iht_server_submit(iht_server *s, const uint8_t *subset, const double *Y, int64_t ldy, int32_t T, const int32_t *ks,
                      int64_t *support, double *beta_S, double *beta_cov, double *loss_trace, int32_t *n_iter,
                      int32_t *status, int64_t *id);
int iht_server_step(iht_server *s, int32_t *completed);
int iht_server_poll(const iht_server *s, int64_t id, int32_t *done);
int iht_server_info(const iht_server *s, iht_server_info_t *info);
int iht_server_destroy(iht_server *s);

/*
 * Block shape of the matrix-core pass (iht_gradient_batch, IHT_MIXED_I8 fits, the server) for this
 * matrix and T solves: the pass is compiled for several shapes (SNPs per workgroup x workgroups per
 * compute unit x 32-solve blocks per workgroup) and the first launch for a (matrix, T) shape times
 * each three times and keeps the one of least median time for the process. Every shape computes the
 * same exact integer sums, so the choice never changes a result. *snps_per_block = the chosen
 * shape's SNPs per workgroup, or 0 if not tuned yet.
 */
int iht_batch_tuning(const iht_geno *g, int32_t T, int32_t *snps_per_block);

const char *iht_status_str(int status);
const char *iht_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* IHT_H */
