/*
 * iht_oracle.c -- plain, slow, obviously correct FP64 reference for the IHT hot path.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the benchmark's CPU-baseline
 * leg may load this library. The device library never links it, includes it or calls it, and it
 * shares no code with the device path.
 *
 * Source of every formula: Keys, Chen & Lange, "Iterative hard thresholding for model selection
 * in genome-wide association studies" (arXiv:1608.01398).
 *   - loss f(beta) = 1/2 ||y - X beta||^2 ............ Methods, Penalized regression, eq. (leastsquaresloss)
 *   - gradient  grad f = -X^T (y - X beta) ............ Methods, Greedy pursuit algorithms, eq. (normal_grad)
 *   - IHT update beta+ = P_Sk[beta - mu grad f] ....... Methods, Greedy pursuit algorithms, eq. (ihta)
 *   - projection: keep the k largest |.|, zero rest .. same subsection, text after eq. (ihta)
 *   - normalised step mu, backtracking omega ......... Methods, IHT step sizes
 *   - standardisation X_st = X diag(v) - 1 u^T diag(v) Methods, Bandwidth optimization of IHT
 *   - missing dosages -> 0 after standardising ....... Results, Simulation
 *   - unpenalised non-genetic covariates ............. Results (SexOCPG + principal components)
 *
 * Readings taken where the paper is silent or garbled (each is listed in the design notes):
 *   R1 step size mu = ||g_{S u C}||^2 / ||A_{S u C} g_{S u C}||^2 (normalised IHT; the printed
 *      ratio of beta-norms is undefined at beta = 0); S at m = 0 is the top-k of |g|.
 *   R2 omega is tested only when the support changes; accept on mu < omega (strict).
 *   R3 c = 0.01, shrink = 0.5, max_backtrack = 50 (defaults; all are arguments here).
 *   R4 beta^0 = 0.   R5 stop when S+ = S and ||beta+ - beta||_inf <= tol * max(1, ||beta+||_inf).
 *   R6 exactly k SNPs kept: |w| descending, ties to the lower index.
 *   R7 u_j = mean of observed dosages over the subject set T; sigma_j^2 = population variance of
 *      the mean-imputed column over all |T| subjects; v_j = 1/sigma_j (0 if sigma_j = 0).
 *   R10 covariates and intercept are unpenalised, always in the model, never projected.
 *   R11 g = A^T r = -grad f; the update is beta + mu g.
 *   R12 a subject subset is solved as the problem restricted to those rows, with its own u, v.
 *   R17 cross-validation: the caller assigns every subject to one of q folds; the held-out MSE is
 *      the mean of (y - prediction)^2 over the fold, predicted with the training fold's u, v; the
 *      model size of least mean MSE wins (the first in the given order on an exact tie).
 *   R18 logistic IHT (Discussion names logistic regression as the extension; no algorithm given):
 *      f = sum_T [log(1 + exp(eta_i)) - y_i eta_i], eta = A beta, so g = A^T (y - sigma(eta)) = -grad f
 *      and the same gradient pass applies; step mu = ||g_{S u C}||^2 / sum_T w_i (A_{S u C} g)_i^2
 *      with w = sigma(eta)(1 - sigma(eta)) at the current beta (the normalised step with the
 *      curvature of f); a proposal is taken when f does not increase beyond 1e-12 |f| (the rounding
 *      of the loss sums, so that a converged iterate is not rejected on rounding alone), else mu is
 *      halved (the omega rule is a least-squares bound and is not used). y in [0, 1].
 *
 * Plain sequential sums everywhere, compiled with -O2 -ffp-contract=off. OpenMP splits only
 * independent per-SNP work (each SNP's sum keeps its own sequential order), as in the paper's
 * shared-memory column split (Methods, Parallelization of IHT).
 */
#define _GNU_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define REF_OK 0
#define REF_NOT_CONVERGED 1
#define REF_STALLED 2
#define REF_EINVAL (-1)
#define REF_ENOMEM (-2)
#define REF_ENONFINITE (-4)

/* ---- PLINK 1 .bed decoding (Methods, Bandwidth optimization of IHT: two bits per genotype) ---- */

/* Two-bit value of subject i in SNP j: byte j*row + i/4, bits 2*(i%4) and 2*(i%4)+1. */
static int code_at(const uint8_t *bed, int64_t row, int64_t j, int64_t i) {
    return (bed[j * row + i / 4] >> (2 * (i % 4))) & 3;
}

/* PLINK value -> dosage of the second allele: 0 -> 0, 2 -> 1, 3 -> 2; 1 (missing) -> -1. */
static int dosage_of(int code) {
    if (code == 0) return 0;
    if (code == 2) return 1;
    if (code == 3) return 2;
    return -1;
}

int iht_ref_decode(const uint8_t *bed, int64_t n, int64_t p, int64_t row_bytes, int8_t *out) {
    if (!bed || !out || n < 1 || p < 1 || row_bytes < (n + 3) / 4) return REF_EINVAL;
    for (int64_t j = 0; j < p; ++j)
        for (int64_t i = 0; i < n; ++i) out[j * n + i] = (int8_t)dosage_of(code_at(bed, row_bytes, j, i));
    return REF_OK;
}

/* Subject set T as an index list; subset == NULL means all n subjects. Returns |T|. */
static int64_t subject_list(int64_t n, const uint8_t *subset, int64_t *idx) {
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i)
        if (!subset || subset[i]) idx[m++] = i;
    return m;
}

/* ---- Standardisation cache u, v (Methods, Bandwidth optimization of IHT; reading R7) ---- */

static void stats_one(const uint8_t *bed, int64_t row, int64_t j, const int64_t *T, int64_t nT, double *u, double *v) {
    int64_t c0 = 0, c1 = 0, c2 = 0;
    for (int64_t t = 0; t < nT; ++t) {
        int d = dosage_of(code_at(bed, row, j, T[t]));
        if (d == 0) c0++;
        else if (d == 1) c1++;
        else if (d == 2) c2++;
    }
    int64_t nobs = c0 + c1 + c2;
    if (nobs == 0) {
        *u = 0.0;
        *v = 0.0;
        return;
    }
    int64_t s1 = c1 + 2 * c2;         /* sum of observed dosages      */
    int64_t s2 = c1 + 4 * c2;         /* sum of squared dosages       */
    int64_t num = nobs * s2 - s1 * s1; /* nobs^2 * (population variance over observed) */
    *u = (double)s1 / (double)nobs;
    if (num == 0) {
        *v = 0.0;
        return;
    }
    /* variance of the mean-imputed column over all nT subjects = num / (nobs * nT) */
    double var = (double)num / (double)(nobs * nT);
    *v = 1.0 / sqrt(var);
}

int iht_ref_stats(const uint8_t *bed, int64_t n, int64_t p, int64_t row_bytes, const uint8_t *subset, double *u, double *v) {
    if (!bed || !u || !v || n < 1 || p < 1 || row_bytes < (n + 3) / 4) return REF_EINVAL;
    int64_t *T = (int64_t *)malloc(sizeof(int64_t) * n);
    if (!T) return REF_ENOMEM;
    int64_t nT = subject_list(n, subset, T);
    if (nT < 1) {
        free(T);
        return REF_EINVAL;
    }
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < p; ++j) stats_one(bed, row_bytes, j, T, nT, &u[j], &v[j]);
    free(T);
    return REF_OK;
}

/* Standardised entry x_st(i, j) = v_j * (x~_ij - u_j), x~ = dosage, or u_j when missing (-> 0). */
static double xst(const uint8_t *bed, int64_t row, int64_t j, int64_t i, const double *u, const double *v) {
    int d = dosage_of(code_at(bed, row, j, i));
    if (d < 0) return 0.0;
    return v[j] * ((double)d - u[j]);
}

int iht_ref_standardize(const uint8_t *bed, int64_t n, int64_t p, int64_t row_bytes, const double *u, const double *v,
                        double *out /* [p][n] */) {
    if (!bed || !u || !v || !out || n < 1 || p < 1 || row_bytes < (n + 3) / 4) return REF_EINVAL;
    for (int64_t j = 0; j < p; ++j)
        for (int64_t i = 0; i < n; ++i) out[j * n + i] = xst(bed, row_bytes, j, i, u, v);
    return REF_OK;
}

/* ---- Gradient g = X_st^T r over the subject set (eq. normal_grad with the sign of reading R11) ---- */

static void gradient_T(const uint8_t *bed, int64_t row, int64_t p, const int64_t *T, int64_t nT, const double *u, const double *v,
                       const double *r /* indexed by subject id */, double *g) {
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < p; ++j) {
        double s = 0.0;
        for (int64_t t = 0; t < nT; ++t) {
            int64_t i = T[t];
            s += xst(bed, row, j, i, u, v) * r[i];
        }
        g[j] = s;
    }
}

int iht_ref_gradient(const uint8_t *bed, int64_t n, int64_t p, int64_t row_bytes, const double *u, const double *v,
                     const uint8_t *subset, const double *r, double *g) {
    if (!bed || !u || !v || !r || !g || n < 1 || p < 1 || row_bytes < (n + 3) / 4) return REF_EINVAL;
    int64_t *T = (int64_t *)malloc(sizeof(int64_t) * n);
    if (!T) return REF_ENOMEM;
    int64_t nT = subject_list(n, subset, T);
    gradient_T(bed, row_bytes, p, T, nT, u, v, r, g);
    free(T);
    return REF_OK;
}

/* ---- Projection P_Sk: keep the k largest |w|, ties to the lower index (eq. ihta; reading R6) ---- */

static int by_abs_desc_then_index(const void *a, const void *b, void *keys) {
    const double *w = (const double *)keys;
    int64_t ia = *(const int64_t *)a, ib = *(const int64_t *)b;
    double xa = fabs(w[ia]), xb = fabs(w[ib]);
    if (xa > xb) return -1;
    if (xa < xb) return 1;
    return (ia < ib) ? -1 : (ia > ib);
}
static int by_index(const void *a, const void *b) {
    int64_t ia = *(const int64_t *)a, ib = *(const int64_t *)b;
    return (ia < ib) ? -1 : (ia > ib);
}

/* support[0..k) ascending = indices of the k largest |w|. */
static int topk_abs(const double *w, int64_t p, int64_t k, int64_t *support) {
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * p);
    if (!order) return REF_ENOMEM;
    for (int64_t j = 0; j < p; ++j) order[j] = j;
    qsort_r(order, (size_t)p, sizeof(int64_t), by_abs_desc_then_index, (void *)w);
    memcpy(support, order, sizeof(int64_t) * k);
    qsort(support, (size_t)k, sizeof(int64_t), by_index);
    free(order);
    return REF_OK;
}

int iht_ref_project(const double *w, int64_t p, int32_t k, int64_t *support, double *w_out) {
    if (!w || !support || p < 1 || k < 1 || k > p) return REF_EINVAL;
    for (int64_t j = 0; j < p; ++j)
        if (!isfinite(w[j])) return REF_ENONFINITE;
    int rc = topk_abs(w, p, k, support);
    if (rc) return rc;
    if (w_out) {
        for (int64_t j = 0; j < p; ++j) w_out[j] = 0.0;
        for (int32_t t = 0; t < k; ++t) w_out[support[t]] = w[support[t]];
    }
    return REF_OK;
}

/* ---- Full IHT fit: eq. (ihta) with the normalised step and backtracking of "IHT step sizes" ---- */

typedef struct {
    const uint8_t *bed;
    int64_t row, n, p;
    const int64_t *T; /* subject set, ascending */
    int64_t nT;
    const double *u, *v;
    const float *Z; /* dense covariates, column-major [n x cz] */
    int32_t cz;     /* number of dense covariates */
    int32_t icpt;   /* 1 if a column of ones is in the model */
} design;

/* Value of unpenalised column c (0..cz-1: covariates, cz: intercept) at subject i. */
static double cov_at(const design *A, int32_t c, int64_t i) {
    if (c < A->cz) return (double)A->Z[(int64_t)c * A->n + i];
    return 1.0;
}

/* out[i] = sum_{j in cols, ascending} x_st(i,j) b[j] + sum_c A_c(i) bc[c], for i in T. */
static void apply_A(const design *A, const int64_t *cols, int64_t ncols, const double *bsnp, const double *bc, double *out) {
    int32_t nc = A->cz + A->icpt;
    for (int64_t t = 0; t < A->nT; ++t) {
        int64_t i = A->T[t];
        double s = 0.0;
        for (int64_t q = 0; q < ncols; ++q) s += xst(A->bed, A->row, cols[q], i, A->u, A->v) * bsnp[cols[q]];
        for (int32_t c = 0; c < nc; ++c) s += cov_at(A, c, i) * bc[c];
        out[i] = s;
    }
}

/* g = A^T r: SNP part over all p (eq. normal_grad), unpenalised part gc. */
static void apply_At(const design *A, const double *r, double *g, double *gc) {
    gradient_T(A->bed, A->row, A->p, A->T, A->nT, A->u, A->v, r, g);
    int32_t nc = A->cz + A->icpt;
    for (int32_t c = 0; c < nc; ++c) {
        double s = 0.0;
        for (int64_t t = 0; t < A->nT; ++t) s += cov_at(A, c, A->T[t]) * r[A->T[t]];
        gc[c] = s;
    }
}

static double sumsq_T(const design *A, const double *x) {
    double s = 0.0;
    for (int64_t t = 0; t < A->nT; ++t) s += x[A->T[t]] * x[A->T[t]];
    return s;
}

static int same_support(const int64_t *a, const int64_t *b, int64_t k) {
    for (int64_t t = 0; t < k; ++t)
        if (a[t] != b[t]) return 0;
    return 1;
}

/* Union of two ascending supports, ascending, without duplicates. Returns its size. */
static int64_t support_union(const int64_t *a, const int64_t *b, int64_t k, int64_t *out) {
    int64_t i = 0, j = 0, m = 0;
    while (i < k || j < k) {
        if (j >= k || (i < k && a[i] < b[j])) out[m++] = a[i++];
        else if (i >= k || b[j] < a[i]) out[m++] = b[j++];
        else { out[m++] = a[i++]; j++; }
    }
    return m;
}

/* Logistic pieces (reading R18): sigma(x) = 1 / (1 + e^-x) evaluated without overflow, and the
 * per-subject loss log(1 + e^x) - y x = max(x, 0) + log1p(e^-|x|) - y x. */
static double sigmoid(double x) {
    if (x >= 0.0) return 1.0 / (1.0 + exp(-x));
    double e = exp(x);
    return e / (1.0 + e);
}

static double logistic_loss(const design *A, const double *y, const double *eta) {
    double s = 0.0;
    for (int64_t t = 0; t < A->nT; ++t) {
        int64_t i = A->T[t];
        double x = eta[i];
        s += ((x > 0.0 ? x : 0.0) + log1p(exp(-fabs(x)))) - y[i] * x;
    }
    return s;
}

/* w = beta + mu g on SNPs and unpenalised columns; S+ = top-k |w|; beta+ = w on S+, 0 elsewhere. */
static int propose(const design *A, int64_t k, double mu, const double *beta, const double *g, const double *bc, const double *gc,
                   double *w, int64_t *Sp, double *betap, double *bcp) {
    for (int64_t j = 0; j < A->p; ++j) w[j] = beta[j] + mu * g[j];
    int rc = topk_abs(w, A->p, k, Sp);
    if (rc) return rc;
    for (int64_t j = 0; j < A->p; ++j) betap[j] = 0.0;
    for (int64_t t = 0; t < k; ++t) betap[Sp[t]] = w[Sp[t]];
    int32_t nc = A->cz + A->icpt;
    for (int32_t c = 0; c < nc; ++c) bcp[c] = bc[c] + mu * gc[c];
    return REF_OK;
}

/* family 0: least squares (eq. leastsquaresloss); family 1: logistic (reading R18). */
int iht_ref_fit_family(const uint8_t *bed, int64_t n, int64_t p, int64_t row_bytes, const uint8_t *subset, const double *y,
                       const float *Z, int32_t cz, int32_t intercept, int32_t k, double tol, int32_t max_iter,
                       int32_t max_backtrack, double c, double shrink, int32_t family, int64_t *support, double *beta_S,
                       double *beta_cov, double *loss_trace, int32_t *n_iter, double *mu_trace) {
    if (!bed || !y || !support || !beta_S || !loss_trace || !n_iter || n < 1 || p < 1 || row_bytes < (n + 3) / 4) return REF_EINVAL;
    if (family != 0 && family != 1) return REF_EINVAL;
    if (k < 1 || k > p || cz < 0 || (cz > 0 && !Z) || max_iter < 0 || max_backtrack < 0) return REF_EINVAL;
    if (!(c > 0.0 && c < 1.0) || !(shrink > 0.0 && shrink < 1.0) || !(tol >= 0.0)) return REF_EINVAL;
    int32_t nc = cz + (intercept ? 1 : 0);
    if (nc > 0 && !beta_cov) return REF_EINVAL;

    int64_t *T = (int64_t *)malloc(sizeof(int64_t) * n);
    double *u = (double *)malloc(sizeof(double) * p), *v = (double *)malloc(sizeof(double) * p);
    double *beta = (double *)calloc(p, sizeof(double)), *betap = (double *)calloc(p, sizeof(double));
    double *g = (double *)malloc(sizeof(double) * p), *w = (double *)malloc(sizeof(double) * p);
    double *dlt = (double *)calloc(p, sizeof(double));
    double *r = (double *)calloc(n, sizeof(double)), *tmp = (double *)calloc(n, sizeof(double));
    double *eta = (double *)calloc(n, sizeof(double)); /* logistic: A beta at the current iterate */
    double bc[64] = {0}, bcp[64] = {0}, gc[64] = {0}, dc[64] = {0};
    int64_t *S = (int64_t *)malloc(sizeof(int64_t) * k), *Sp = (int64_t *)malloc(sizeof(int64_t) * k);
    int64_t *U = (int64_t *)malloc(sizeof(int64_t) * 2 * k);
    int rc = REF_OK;
    if (!T || !u || !v || !beta || !betap || !g || !w || !dlt || !r || !tmp || !eta || !S || !Sp || !U || nc > 64) {
        rc = REF_ENOMEM;
        goto done;
    }
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(y[i]) || (subset && !(subset[i] == 0 || subset[i] == 1))) { rc = REF_ENONFINITE; goto done; }
    if (family == 1)
        for (int64_t i = 0; i < n; ++i)
            if ((!subset || subset[i]) && !(y[i] >= 0.0 && y[i] <= 1.0)) { rc = REF_EINVAL; goto done; }
    for (int64_t q = 0; q < (int64_t)cz * n; ++q)
        if (!isfinite(Z[q])) { rc = REF_ENONFINITE; goto done; }

    int64_t nT = subject_list(n, subset, T);
    if (nT < 1) { rc = REF_EINVAL; goto done; }
    rc = iht_ref_stats(bed, n, p, row_bytes, subset, u, v);
    if (rc) goto done;
    design A = {bed, row_bytes, n, p, T, nT, u, v, Z, cz, intercept ? 1 : 0};

    /* Initialisation (reading R4): beta = 0, r = y (logistic: y - 1/2), g = A^T r, S = top-k |g|
     * (reading R1). */
    for (int64_t t = 0; t < nT; ++t) r[T[t]] = family ? y[T[t]] - sigmoid(0.0) : y[T[t]];
    loss_trace[0] = family ? logistic_loss(&A, y, eta) : 0.5 * sumsq_T(&A, r);
    apply_At(&A, r, g, gc);
    rc = topk_abs(g, p, k, S);
    if (rc) goto done;

    int status = REF_NOT_CONVERGED;
    int32_t m = 0;
    for (; m < max_iter; ++m) {
        /* Normalised step (reading R1): mu = ||g_{S u C}||^2 / ||A_{S u C} g_{S u C}||^2. */
        double num = 0.0;
        for (int64_t t = 0; t < k; ++t) num += g[S[t]] * g[S[t]];
        for (int32_t q = 0; q < nc; ++q) num += gc[q] * gc[q];
        apply_A(&A, S, k, g, gc, tmp);
        double den = 0.0;
        if (family) { /* curvature weights at the current beta (reading R18) */
            for (int64_t t = 0; t < nT; ++t) {
                double sg = sigmoid(eta[T[t]]);
                den += (sg * (1.0 - sg)) * (tmp[T[t]] * tmp[T[t]]);
            }
        } else {
            den = sumsq_T(&A, tmp);
        }
        if (den == 0.0) { status = REF_OK; break; }
        double mu = num / den;

        rc = propose(&A, k, mu, beta, g, bc, gc, w, Sp, betap, bcp);
        if (rc) goto done;

        /* Backtracking (reading R2): only when the support moves; accept when mu < omega.
         * Logistic (reading R18): accept when the loss does not increase. */
        int nbt = 0, stalled = 0;
        double fplus = 0.0;
        while (family) {
            apply_A(&A, Sp, k, betap, bcp, tmp);
            fplus = logistic_loss(&A, y, tmp);
            if (fplus <= loss_trace[m] + 1e-12 * fabs(loss_trace[m])) break;
            if (nbt == max_backtrack) { stalled = 1; break; }
            mu = mu * shrink;
            nbt++;
            rc = propose(&A, k, mu, beta, g, bc, gc, w, Sp, betap, bcp);
            if (rc) goto done;
        }
        while (!family && !same_support(S, Sp, k)) {
            int64_t nu = support_union(S, Sp, k, U);
            double dd = 0.0;
            for (int64_t q = 0; q < nu; ++q) {
                dlt[U[q]] = betap[U[q]] - beta[U[q]];
                dd += dlt[U[q]] * dlt[U[q]];
            }
            for (int32_t q = 0; q < nc; ++q) {
                dc[q] = bcp[q] - bc[q];
                dd += dc[q] * dc[q];
            }
            apply_A(&A, U, nu, dlt, dc, tmp);
            double dA = sumsq_T(&A, tmp);
            for (int64_t q = 0; q < nu; ++q) dlt[U[q]] = 0.0;
            double omega = (1.0 - c) * dd / dA; /* +inf when A Delta = 0 */
            if (mu < omega) break;
            if (nbt == max_backtrack) { stalled = 1; break; }
            mu = mu * shrink;
            nbt++;
            rc = propose(&A, k, mu, beta, g, bc, gc, w, Sp, betap, bcp);
            if (rc) goto done;
        }
        if (stalled) { status = REF_STALLED; break; }
        if (mu_trace) mu_trace[m] = mu;

        /* Residual, loss (eq. leastsquaresloss; logistic: reading R18) and gradient (eq. normal_grad)
         * at beta+. */
        apply_A(&A, Sp, k, betap, bcp, tmp);
        if (family) {
            for (int64_t t = 0; t < nT; ++t) {
                eta[T[t]] = tmp[T[t]];
                r[T[t]] = y[T[t]] - sigmoid(tmp[T[t]]);
            }
            loss_trace[m + 1] = fplus;
        } else {
            for (int64_t t = 0; t < nT; ++t) r[T[t]] = y[T[t]] - tmp[T[t]];
            loss_trace[m + 1] = 0.5 * sumsq_T(&A, r);
        }
        apply_At(&A, r, g, gc);

        /* Convergence (reading R5). */
        int conv = same_support(S, Sp, k);
        double dmax = 0.0, bmax = 0.0;
        int64_t nu = support_union(S, Sp, k, U);
        for (int64_t q = 0; q < nu; ++q) {
            double d = fabs(betap[U[q]] - beta[U[q]]);
            if (d > dmax) dmax = d;
            if (fabs(betap[U[q]]) > bmax) bmax = fabs(betap[U[q]]);
        }
        for (int32_t q = 0; q < nc; ++q) {
            double d = fabs(bcp[q] - bc[q]);
            if (d > dmax) dmax = d;
            if (fabs(bcp[q]) > bmax) bmax = fabs(bcp[q]);
        }
        conv = conv && dmax <= tol * (bmax > 1.0 ? bmax : 1.0);

        for (int64_t t = 0; t < k; ++t) beta[S[t]] = 0.0;
        for (int64_t t = 0; t < k; ++t) beta[Sp[t]] = betap[Sp[t]];
        memcpy(S, Sp, sizeof(int64_t) * k);
        memcpy(bc, bcp, sizeof(double) * nc);
        if (conv) { status = REF_OK; m++; break; }
    }
    *n_iter = m;
    for (int64_t t = 0; t < k; ++t) {
        support[t] = S[t];
        beta_S[t] = beta[S[t]];
    }
    for (int32_t q = 0; q < nc; ++q) beta_cov[q] = bc[q];
    rc = status;
done:
    free(T); free(u); free(v); free(beta); free(betap); free(g); free(w); free(dlt); free(r); free(tmp); free(eta);
    free(S); free(Sp); free(U);
    return rc;
}

int iht_ref_fit(const uint8_t *bed, int64_t n, int64_t p, int64_t row_bytes, const uint8_t *subset, const double *y,
                const float *Z, int32_t cz, int32_t intercept, int32_t k, double tol, int32_t max_iter, int32_t max_backtrack,
                double c, double shrink, int64_t *support /* [k] */, double *beta_S /* [k] */, double *beta_cov /* [cz+icpt] */,
                double *loss_trace /* [max_iter+1] */, int32_t *n_iter, double *mu_trace /* [max_iter] or NULL */) {
    return iht_ref_fit_family(bed, n, p, row_bytes, subset, y, Z, cz, intercept, k, tol, max_iter, max_backtrack, c, shrink, 0,
                              support, beta_S, beta_cov, loss_trace, n_iter, mu_trace);
}

/* ---- prediction by a fitted model (Methods, Bandwidth optimization of IHT: the product X_st beta) ----
 * out[i] = sum_t x_st(i, support[t]) beta_S[t] + sum_c Z[c][i] beta_cov[c] (+ beta_cov[cz] if intercept)
 * for every subject, with the given u, v; a missing dosage contributes 0 (reading R7). */
int iht_ref_predict(const uint8_t *bed, int64_t n, int64_t p, int64_t row_bytes, const double *u, const double *v,
                    const int64_t *support, const double *beta_S, int32_t k, const float *Z, int32_t cz, int32_t intercept,
                    const double *beta_cov, double *out) {
    if (!bed || !u || !v || !out || n < 1 || p < 1 || k < 0 || (k > 0 && (!support || !beta_S)) || cz < 0 ||
        (cz > 0 && !Z) || ((cz > 0 || intercept) && !beta_cov))
        return REF_EINVAL;
    for (int32_t t = 0; t < k; ++t)
        if (support[t] < 0 || support[t] >= p) return REF_EINVAL;
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int32_t t = 0; t < k; ++t) s += xst(bed, row_bytes, support[t], i, u, v) * beta_S[t];
        for (int32_t c = 0; c < cz; ++c) s += (double)Z[(int64_t)c * n + i] * beta_cov[c];
        if (intercept) s += beta_cov[cz];
        out[i] = s;
    }
    return REF_OK;
}

/* ---- q-fold cross-validation over a path of model sizes (Methods, Model selection) ----
 * For fold f the training set is the subjects whose fold is not f: a subset solve (reading R12)
 * with its own u, v. For every k in ks the fitted model predicts the subjects of fold f,
 * standardised with the training u, v (a missing dosage is mean-imputed, i.e. 0 after
 * standardising: reading R7), and their mean squared error goes to mse[ki * q + f].
 * Reading R17: k_best is the k of least mean MSE over the folds (mean = sequential sum over f / q),
 * the first in ks on an exact tie; the refit on every subject is a plain fit with that k. */
int iht_ref_cv(const uint8_t *bed, int64_t n, int64_t p, int64_t row_bytes, const uint8_t *folds, int32_t q,
               const double *y, const float *Z, int32_t cz, int32_t intercept, const int32_t *ks, int32_t r, double tol,
               int32_t max_iter, int32_t max_backtrack, double c, double shrink, double *mse, int32_t *k_best) {
    if (!bed || !folds || !y || !ks || !mse || !k_best || n < 1 || p < 1 || q < 2 || r < 1 || cz < 0 ||
        (cz > 0 && !Z) || max_iter < 1)
        return REF_EINVAL;
    int32_t kmax = 0;
    for (int32_t a = 0; a < r; ++a) {
        if (ks[a] < 1 || ks[a] > p) return REF_EINVAL;
        if (ks[a] > kmax) kmax = ks[a];
    }
    int64_t *count = (int64_t *)calloc((size_t)q, sizeof(int64_t));
    if (!count) return REF_ENOMEM;
    for (int64_t i = 0; i < n; ++i) {
        if (folds[i] >= q) { free(count); return REF_EINVAL; }
        count[folds[i]]++;
    }
    for (int32_t f = 0; f < q; ++f)
        if (count[f] == 0 || count[f] == n) { free(count); return REF_EINVAL; }  /* empty test or training set */
    const int32_t nc = cz + (intercept ? 1 : 0);
    uint8_t *subset = (uint8_t *)malloc((size_t)n);
    double *u = (double *)malloc(sizeof(double) * (size_t)p);
    double *v = (double *)malloc(sizeof(double) * (size_t)p);
    int64_t *sup = (int64_t *)malloc(sizeof(int64_t) * (size_t)kmax);
    double *bS = (double *)malloc(sizeof(double) * (size_t)kmax);
    double *bc = (double *)malloc(sizeof(double) * (size_t)(nc > 0 ? nc : 1));
    double *trace = (double *)malloc(sizeof(double) * (size_t)(max_iter + 1));
    double *mu = (double *)malloc(sizeof(double) * (size_t)max_iter);
    int rc = REF_OK;
    if (!subset || !u || !v || !sup || !bS || !bc || !trace || !mu) { rc = REF_ENOMEM; goto done; }
    for (int32_t f = 0; f < q; ++f) {
        for (int64_t i = 0; i < n; ++i) subset[i] = folds[i] != f;
        rc = iht_ref_stats(bed, n, p, row_bytes, subset, u, v);
        if (rc) goto done;
        for (int32_t a = 0; a < r; ++a) {
            int32_t nit = 0;
            rc = iht_ref_fit(bed, n, p, row_bytes, subset, y, Z, cz, intercept, ks[a], tol, max_iter, max_backtrack, c,
                             shrink, sup, bS, bc, trace, &nit, mu);
            if (rc < 0) goto done;
            double ss = 0.0;
            for (int64_t i = 0; i < n; ++i) {
                if (folds[i] != f) continue;
                double pred = 0.0;
                for (int32_t t = 0; t < ks[a]; ++t) pred += xst(bed, row_bytes, sup[t], i, u, v) * bS[t];
                for (int32_t cc = 0; cc < cz; ++cc) pred += (double)Z[(int64_t)cc * n + i] * bc[cc];
                if (intercept) pred += bc[cz];
                const double d = y[i] - pred;
                ss += d * d;
            }
            mse[(int64_t)a * q + f] = ss / (double)count[f];
        }
    }
    rc = REF_OK;
    {
        double best = 0.0;
        for (int32_t a = 0; a < r; ++a) {
            double s = 0.0;
            for (int32_t f = 0; f < q; ++f) s += mse[(int64_t)a * q + f];
            s /= (double)q;
            if (a == 0 || s < best) { best = s; *k_best = ks[a]; }
        }
    }
done:
    free(count); free(subset); free(u); free(v); free(sup); free(bS); free(bc); free(trace); free(mu);
    return rc;
}
