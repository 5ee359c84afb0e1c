/*
 * Plain CPU reference ("oracle") for the AVU-GSR solver hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this file's library.  It shares
 * no code, header or table with the HIP library and must never be used as a
 * fallback for it.
 *
 * Everything here is slow and written to be checked by eye against the
 * paper (Cesare et al., "The Gaia AVU-GSR solver: a CPU + GPU parallel code
 * toward Exascale systems") and against the LSQR method it cites (Paige &
 * Saunders 1982).  Floating point is FP64 unless a function says otherwise;
 * build with -ffp-contract=off so that no multiply-add is fused.
 *
 * Matrix form (Sec. 2, the "dense" coefficient matrix): every row holds 24
 * coefficients, N_Astro = 5, N_Att = 12, N_Instr = 6, N_Glob = 1, in slot
 * order astro(5) | attitude axis 0 (4) | axis 1 (4) | axis 2 (4) |
 * instrumental (6) | global (1).  Column of slot k in row r of star s:
 *     k < 5       5*s + k
 *     5 <= k < 17 N_A + a*n_att + att_start[r] + j,  a = (k-5)/4, j = (k-5)%4
 *     17 <= k < 23 N_A + 3*n_att + instr_col[r][k-17]
 *     k = 23      N_A + 3*n_att + n_instr            (only when n_glob = 1)
 * with N_A = 5*n_stars.  Rows are sorted by star.
 *
 * Threads (OpenMP) only split work whose result does not depend on the split:
 * aprod 1 by stars (each row's sum is unchanged), and the column sums of
 * aprod 2 / the column norms by fixed chunks of stars (see below): the
 * results are the same for any thread count.
 *
 * Constraint equations (Sec. 2: a set of them makes the solution unique): ncon
 * extra sparse rows after the m observation rows, row i holding the entries
 * con_col[e], con_val[e] for e in [con_ptr[i], con_ptr[i+1]).  The system is
 * then [A; C] x = [b; c], and every m-sized vector has m + ncon entries.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int64_t n_stars, m, n_att, n_instr;
    int32_t n_glob;         /* 0 or 1 */
    int32_t f32;            /* 1: vals are float, else double */
    const void *vals;       /* [m][24] */
    const int64_t *star_row_ptr; /* [n_stars+1] */
    const int32_t *att_start;    /* [m] */
    const int32_t *instr_col;    /* [m][6] */
    int64_t ncon;                /* constraint rows (0: none) */
    const int64_t *con_ptr;      /* [ncon+1] */
    const int64_t *con_col;      /* [con_ptr[ncon]] */
    const double *con_val;       /* [con_ptr[ncon]] */
} orc_sys;

/* product modes */
#define ORC_P64 0   /* a*x in FP64 */
#define ORC_P32 1   /* fl32(fl32(a)*fl32(x)), accumulated in FP64 */
/* LSQR only: FP32 products as ORC_P32, with the operand of each A^T product the
 * unnormalised u' = A S v - alpha u (before the division by beta = ||u'||) and the
 * column sums divided by beta afterwards -- the same vector in exact arithmetic,
 * but the FP32 rounding falls on u'_r instead of u'_r / beta.  This is the order
 * in which a single pass over the rows forms both products of an iteration.
 * ORC_P64_1P: the same order with FP64 products. */
#define ORC_P32_1P 2
#define ORC_P64_1P 3

int64_t orc_n_unknowns(const orc_sys *A)
{
    return 5 * A->n_stars + 3 * A->n_att + A->n_instr + A->n_glob;
}

static int n_slots(const orc_sys *A) { return A->n_glob ? 24 : 23; }

/* Rows of [A; C]. */
int64_t orc_rows(const orc_sys *A) { return A->m + A->ncon; }

int64_t orc_col(const orc_sys *A, int64_t s, int64_t r, int k)
{
    int64_t NA = 5 * A->n_stars;
    if (k < 5)
        return 5 * s + k;
    if (k < 17) {
        int a = (k - 5) / 4, j = (k - 5) % 4;
        return NA + a * A->n_att + A->att_start[r] + j;
    }
    if (k < 23)
        return NA + 3 * A->n_att + A->instr_col[6 * r + (k - 17)];
    return NA + 3 * A->n_att + A->n_instr;
}

static double coef(const orc_sys *A, int64_t r, int k)
{
    if (A->f32)
        return (double)((const float *)A->vals)[24 * r + k];
    return ((const double *)A->vals)[24 * r + k];
}

static double product(const orc_sys *A, int64_t r, int k, double x, int mode)
{
    if (mode == ORC_P32) {
        float a = A->f32 ? ((const float *)A->vals)[24 * r + k]
                         : (float)((const double *)A->vals)[24 * r + k];
        float xf = (float)x;
        float p = a * xf;
        return (double)p;
    }
    return coef(A, r, k) * x;
}

/* Neumaier's compensated summation step. */
static void comp_add(double *sum, double *c, double v)
{
    double t = *sum + v;
    if (fabs(*sum) >= fabs(v))
        *c += (*sum - t) + v;
    else
        *c += (v - t) + *sum;
    *sum = t;
}

/* Threads used by the products (0 or less: the OpenMP default). */
void orc_set_threads(int n)
{
    omp_set_num_threads(n > 0 ? n : omp_get_num_procs());
}

int orc_get_threads(void) { return omp_get_max_threads(); }

/* Eq. (2): y <- scale_y * y + A x.  Each row is summed in slot order.
 * scale_y == 0 overwrites y without reading it. */
void orc_aprod1(const orc_sys *A, const double *x, double *y, double scale_y, int mode)
{
    int ns = n_slots(A);
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t s = 0; s < A->n_stars; ++s) {
        for (int64_t r = A->star_row_ptr[s]; r < A->star_row_ptr[s + 1]; ++r) {
            double acc = 0.0;
            for (int k = 0; k < ns; ++k)
                acc += product(A, r, k, x[orc_col(A, s, r, k)], mode);
            y[r] = (scale_y == 0.0 ? 0.0 : scale_y * y[r]) + acc;
        }
    }
    for (int64_t i = 0; i < A->ncon; ++i) {
        double acc = 0.0;
        for (int64_t e = A->con_ptr[i]; e < A->con_ptr[i + 1]; ++e)
            acc += A->con_val[e] * x[A->con_col[e]];
        y[A->m + i] = (scale_y == 0.0 ? 0.0 : scale_y * y[A->m + i]) + acc;
    }
}

/*
 * Column sums of A^T y (sq == 0) or of the squared coefficients (sq == 1) over
 * the observation rows, each column a compensated sum in row order.  A star's
 * five astrometric columns take only that star's rows, so stars are shared out
 * between threads freely.  The other columns take rows of every star: the
 * stars are cut into NCH fixed chunks of consecutive stars, each chunk sums its
 * rows in row order into its own compensated pair (sum, cmp) per column, and
 * the chunks' pairs are added in chunk order with compensation.  The chunks do
 * not depend on the thread count.
 */
#define NCH 16

static int column_sums(const orc_sys *A, const double *y, int mode, int sq, double *sum, double *cmp)
{
    int64_t NA = 5 * A->n_stars, nt = orc_n_unknowns(A) - NA;
    int ns = n_slots(A);
    int64_t nch = A->n_stars < NCH ? A->n_stars : NCH;
    double *cs = NULL, *cc = NULL;
    if (nch > 0) {
        cs = calloc((size_t)(nch * nt), sizeof(double));
        cc = calloc((size_t)(nch * nt), sizeof(double));
        if (!cs || !cc) {
            free(cs);
            free(cc);
            return -1;
        }
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t ch = 0; ch < nch; ++ch) {
        /* chunk ch: stars [s0, s1) holding about a (1/nch) share of the rows */
        int64_t s0 = 0, s1 = 0, lo = 0, hi = A->n_stars;
        int64_t r0 = A->m * ch / nch, r1 = A->m * (ch + 1) / nch;
        while (lo < hi) { /* first star whose rows start at or after r0 */
            int64_t mid = (lo + hi) / 2;
            if (A->star_row_ptr[mid] < r0) lo = mid + 1; else hi = mid;
        }
        s0 = ch == 0 ? 0 : lo;
        lo = 0;
        hi = A->n_stars;
        while (lo < hi) {
            int64_t mid = (lo + hi) / 2;
            if (A->star_row_ptr[mid] < r1) lo = mid + 1; else hi = mid;
        }
        s1 = ch == nch - 1 ? A->n_stars : lo;
        double *ps = cs + ch * nt, *pc = cc + ch * nt;
        for (int64_t s = s0; s < s1; ++s)
            for (int64_t r = A->star_row_ptr[s]; r < A->star_row_ptr[s + 1]; ++r)
                for (int k = 0; k < ns; ++k) {
                    int64_t c = orc_col(A, s, r, k);
                    double term;
                    if (sq) {
                        double a = coef(A, r, k);
                        term = a * a;
                    } else {
                        term = product(A, r, k, y[r], mode);
                    }
                    if (c < NA)
                        comp_add(&sum[c], &cmp[c], term);
                    else
                        comp_add(&ps[c - NA], &pc[c - NA], term);
                }
    }
    for (int64_t ch = 0; ch < nch; ++ch)
        for (int64_t j = 0; j < nt; ++j) {
            comp_add(&sum[NA + j], &cmp[NA + j], cs[ch * nt + j]);
            comp_add(&sum[NA + j], &cmp[NA + j], cc[ch * nt + j]);
        }
    free(cs);
    free(cc);
    /* constraint rows, after the observation rows */
    for (int64_t i = 0; i < A->ncon; ++i)
        for (int64_t e = A->con_ptr[i]; e < A->con_ptr[i + 1]; ++e) {
            double a = A->con_val[e];
            comp_add(&sum[A->con_col[e]], &cmp[A->con_col[e]], sq ? a * a : a * y[A->m + i]);
        }
    return 0;
}

/* Eq. (3): x <- scale_x * x + A^T y, every column a compensated sum (see
 * column_sums).  scale_x == 0 overwrites x. */
int orc_aprod2(const orc_sys *A, const double *y, double *x, double scale_x, int mode)
{
    int64_t n = orc_n_unknowns(A);
    double *sum = calloc((size_t)n, sizeof(double));
    double *cmp = calloc((size_t)n, sizeof(double));
    if (!sum || !cmp || column_sums(A, y, mode, 0, sum, cmp)) {
        free(sum);
        free(cmp);
        return -1;
    }
    for (int64_t c = 0; c < n; ++c)
        x[c] = (scale_x == 0.0 ? 0.0 : scale_x * x[c]) + (sum[c] + cmp[c]);
    free(sum);
    free(cmp);
    return 0;
}

/* Euclidean norm of every column of [A; C] (compensated sums of squares). */
int orc_colnorms(const orc_sys *A, double *norms)
{
    int64_t n = orc_n_unknowns(A);
    double *sum = calloc((size_t)n, sizeof(double));
    double *cmp = calloc((size_t)n, sizeof(double));
    if (!sum || !cmp || column_sums(A, NULL, ORC_P64, 1, sum, cmp)) {
        free(sum);
        free(cmp);
        return -1;
    }
    for (int64_t c = 0; c < n; ++c)
        norms[c] = sqrt(sum[c] + cmp[c]);
    free(sum);
    free(cmp);
    return 0;
}

static double nrm2(const double *v, int64_t n)
{
    double s = 0.0, c = 0.0;
    for (int64_t i = 0; i < n; ++i)
        comp_add(&s, &c, v[i] * v[i]);
    return sqrt(s + c);
}

typedef struct {
    double damp, atol, btol, conlim;
    int64_t itmax;
    int32_t precond; /* 1: diagonal column scaling S = diag(1/||a_j||) */
    int32_t mode;    /* ORC_P64, ORC_P32, ORC_P32_1P or ORC_P64_1P */
} orc_opts;

typedef struct {
    int32_t istop;
    int64_t itn;
    double rnorm, arnorm, anorm, acond, xnorm, bnorm;
} orc_result;

/*
 * Preconditioned LSQR (Paige & Saunders 1982) following the solver outline
 * of Sec. 2: precondition, set the initial conditions with aprod 2, iterate
 * aprod 1 / aprod 2 / variances / covariance vectors, de-precondition.
 *
 * Solves min || [A S; damp I] y - [r0; 0] || with r0 = b - A x0 (x0 = 0 when
 * NULL) and returns x = x0 + S y.  With constraint rows, A is [A; C] and b
 * has m + ncon entries.  S = diag(1/||a_j||) when precond is set
 * (1 for an empty column), else I.
 *
 * var (nullable): sum_i (S d_i)^2 with d_i = w_i / rho_i, the variances
 * computed every iteration.  dsel (nullable, [itmax][k]): d_i[sel[p]] in the
 * scaled space, stored for every iteration i, for the covariances of Eq. (4).
 * scale_out (nullable, [n]): the column scaling used.
 */
int orc_lsqr(const orc_sys *A, const double *b, const double *x0, double *x, double *var,
             const int64_t *sel, int64_t k, double *dsel, double *scale_out,
             const orc_opts *o, orc_result *res)
{
    int64_t m = orc_rows(A), n = orc_n_unknowns(A);
    double *u = malloc((size_t)m * sizeof(double));
    double *v = malloc((size_t)n * sizeof(double));
    double *w = malloc((size_t)n * sizeof(double));
    double *y = calloc((size_t)n, sizeof(double));
    double *S = malloc((size_t)n * sizeof(double));
    double *t = malloc((size_t)n * sizeof(double));
    int rc = 0;
    if (!u || !v || !w || !y || !S || !t) {
        rc = -1;
        goto out;
    }
    /* preconditioning */
    if (o->precond) {
        if (orc_colnorms(A, S)) {
            rc = -1;
            goto out;
        }
        for (int64_t j = 0; j < n; ++j)
            S[j] = S[j] > 0.0 ? 1.0 / S[j] : 1.0;
    } else {
        for (int64_t j = 0; j < n; ++j)
            S[j] = 1.0;
    }
    if (scale_out)
        memcpy(scale_out, S, (size_t)n * sizeof(double));

    /* u = r0 = b - A x0 */
    memcpy(u, b, (size_t)m * sizeof(double));
    if (x0) {
        for (int64_t j = 0; j < n; ++j)
            t[j] = -x0[j];
        orc_aprod1(A, t, u, 1.0, ORC_P64);
    }
    const int onepass = o->mode == ORC_P32_1P || o->mode == ORC_P64_1P;
    const int pmode = o->mode == ORC_P32_1P ? ORC_P32 : o->mode == ORC_P64_1P ? ORC_P64 : o->mode;
    const double damp = o->damp, dampsq = o->damp * o->damp;
    const double ctol = o->conlim > 0.0 ? 1.0 / o->conlim : 0.0;
    double beta = nrm2(u, m), alpha = 0.0;
    double anorm = 0.0, acond = 0.0, ddnorm = 0.0, res2 = 0.0, xnorm = 0.0;
    int istop = 0;
    int64_t itn = 0;
    /* initial conditions with aprod 2: beta1 u1 = r0, alpha1 v1 = (A S)^T u1 */
    if (beta > 0.0) {
        if (onepass) {
            /* A^T on the unnormalised r0, then divided by beta */
            if (orc_aprod2(A, u, t, 0.0, pmode)) {
                rc = -1;
                goto out;
            }
            const double ib = 1.0 / beta;
            for (int64_t j = 0; j < n; ++j)
                v[j] = S[j] * (ib * t[j]);
            for (int64_t i = 0; i < m; ++i)
                u[i] /= beta;
        } else {
            for (int64_t i = 0; i < m; ++i)
                u[i] /= beta;
            if (orc_aprod2(A, u, t, 0.0, pmode)) {
                rc = -1;
                goto out;
            }
            for (int64_t j = 0; j < n; ++j)
                v[j] = S[j] * t[j];
        }
        alpha = nrm2(v, n);
    } else {
        memset(v, 0, (size_t)n * sizeof(double));
    }
    if (alpha > 0.0)
        for (int64_t j = 0; j < n; ++j)
            v[j] /= alpha;
    memcpy(w, v, (size_t)n * sizeof(double));
    double rhobar = alpha, phibar = beta;
    const double bnorm = beta;
    double rnorm = beta, arnorm = alpha * beta;
    if (var)
        memset(var, 0, (size_t)n * sizeof(double));

    if (arnorm != 0.0) {
        for (;;) {
            ++itn;
            /* aprod 1: beta u = A S v - alpha u */
            for (int64_t j = 0; j < n; ++j)
                t[j] = S[j] * v[j];
            orc_aprod1(A, t, u, -alpha, pmode);
            beta = nrm2(u, m);
            if (beta > 0.0) {
                double ib = 1.0;
                if (onepass) {
                    /* A^T on the unnormalised u', divided by beta below */
                    if (orc_aprod2(A, u, t, 0.0, pmode)) {
                        rc = -1;
                        goto out;
                    }
                    ib = 1.0 / beta;
                }
                for (int64_t i = 0; i < m; ++i)
                    u[i] /= beta;
                anorm = sqrt(anorm * anorm + alpha * alpha + beta * beta + dampsq);
                /* aprod 2: alpha v = S A^T u - beta v */
                if (!onepass && orc_aprod2(A, u, t, 0.0, pmode)) {
                    rc = -1;
                    goto out;
                }
                for (int64_t j = 0; j < n; ++j)
                    v[j] = onepass ? S[j] * (ib * t[j]) - beta * v[j] : S[j] * t[j] - beta * v[j];
                alpha = nrm2(v, n);
                if (alpha > 0.0)
                    for (int64_t j = 0; j < n; ++j)
                        v[j] /= alpha;
            }
            /* plane rotation that eliminates the damping parameter */
            double rhobar1, psi;
            if (damp > 0.0) {
                rhobar1 = sqrt(rhobar * rhobar + dampsq);
                double cs1 = rhobar / rhobar1, sn1 = damp / rhobar1;
                psi = sn1 * phibar;
                phibar = cs1 * phibar;
            } else {
                rhobar1 = rhobar;
                psi = 0.0;
            }
            /* plane rotation that eliminates the subdiagonal beta */
            double rho = sqrt(rhobar1 * rhobar1 + beta * beta);
            double cs = rhobar1 / rho, sn = beta / rho;
            double theta = sn * alpha;
            rhobar = -cs * alpha;
            double phi = cs * phibar;
            phibar = sn * phibar;
            double tau = sn * phi;
            /* update y, w; variances; covariance vectors d = w / rho */
            double t1 = phi / rho, t2 = -theta / rho, t3 = 1.0 / rho;
            if (dsel)
                for (int64_t p = 0; p < k; ++p)
                    dsel[(itn - 1) * k + p] = t3 * w[sel[p]];
            double dd = 0.0, ddc = 0.0;
            for (int64_t j = 0; j < n; ++j) {
                double d = t3 * w[j];
                comp_add(&dd, &ddc, d * d);
                if (var)
                    var[j] += d * d;
                y[j] = y[j] + t1 * w[j];
                w[j] = v[j] + t2 * w[j];
            }
            ddnorm += dd + ddc;
            /* estimates */
            xnorm = nrm2(y, n);
            acond = anorm * sqrt(ddnorm);
            res2 += psi * psi;
            rnorm = sqrt(phibar * phibar + res2);
            arnorm = alpha * fabs(tau);
            double test1 = rnorm / bnorm;
            double test2 = (anorm * rnorm > 0.0) ? arnorm / (anorm * rnorm) : 0.0;
            double test3 = (acond > 0.0) ? 1.0 / acond : INFINITY;
            double tt1 = test1 / (1.0 + anorm * xnorm / bnorm);
            double rtol = o->btol + o->atol * anorm * xnorm / bnorm;
            /* stopping tests; the lowest-numbered satisfied test wins */
            if (itn >= o->itmax) istop = 7;
            if (1.0 + test3 <= 1.0) istop = 6;
            if (1.0 + test2 <= 1.0) istop = 5;
            if (1.0 + tt1 <= 1.0) istop = 4;
            if (test3 <= ctol) istop = 3;
            if (test2 <= o->atol) istop = 2;
            if (test1 <= rtol) istop = 1;
            if (istop)
                break;
        }
    }
    /* de-precondition: x = x0 + S y, var = S^2 var */
    for (int64_t j = 0; j < n; ++j) {
        x[j] = (x0 ? x0[j] : 0.0) + S[j] * y[j];
        if (var)
            var[j] *= S[j] * S[j];
    }
    res->istop = istop;
    res->itn = itn;
    res->rnorm = rnorm;
    res->arnorm = arnorm;
    res->anorm = anorm;
    res->acond = acond;
    res->xnorm = xnorm;
    res->bnorm = bnorm;
out:
    free(u);
    free(v);
    free(w);
    free(y);
    free(S);
    free(t);
    return rc;
}

/*
 * Covariances of the selected unknowns, Eq. (4), read with d_i = w_i / rho_i
 * as the per-iteration vector and factor 1:
 *     C[p][q] = s_p s_q sum_{i < itn} d_i[sel_p] d_i[sel_q]
 * dsel is [itn][k] as written by orc_lsqr; ssel (nullable) is the column
 * scaling at the selected indices.  C is [k][k], full and symmetric.
 */
void orc_covariances(const double *dsel, int64_t itn, int64_t k, const double *ssel, double *C)
{
    for (int64_t p = 0; p < k; ++p)
        for (int64_t q = 0; q < k; ++q) {
            double acc = 0.0;
            for (int64_t i = 0; i < itn; ++i)
                acc += dsel[i * k + p] * dsel[i * k + q];
            double sp = ssel ? ssel[p] : 1.0, sq = ssel ? ssel[q] : 1.0;
            C[p * k + q] = sp * sq * acc;
        }
}

/*
 * FP32 form with FP64 iterative refinement.  A holds FP32-representable
 * coefficients.  Each outer step forms the residual r = b - A x with FP64
 * products on those coefficients (exact upcast), solves A dx ~ r with the
 * inner LSQR options (normally the FP32-product mode and a loose
 * tolerance), and updates x += dx.  Stops once ||dx|| <= outer_tol ||x||,
 * or once the next correction predicted from the observed contraction,
 * ||dx_k||^2 / ||dx_{k-1}|| (when ||dx_k|| < ||dx_{k-1}||), is at most
 * outer_tol ||x||, or after outer_max steps.  x is overwritten (starts from
 * x0 or zero).
 */
int orc_lsqr_refine(const orc_sys *A, const double *b, const double *x0, double *x,
                    const orc_opts *inner, int32_t outer_max, double outer_tol,
                    int64_t *inner_total, int32_t *outer_steps, orc_result *last)
{
    int64_t m = orc_rows(A), n = orc_n_unknowns(A);
    double *r = malloc((size_t)m * sizeof(double));
    double *nx = malloc((size_t)n * sizeof(double));
    double *dx = malloc((size_t)n * sizeof(double));
    int rc = 0;
    if (!r || !nx || !dx) {
        rc = -1;
        goto out;
    }
    for (int64_t j = 0; j < n; ++j)
        x[j] = x0 ? x0[j] : 0.0;
    *inner_total = 0;
    *outer_steps = 0;
    double prev = 0.0;  /* ||dx|| of the previous step */
    for (int32_t it = 0; it < outer_max; ++it) {
        memcpy(r, b, (size_t)m * sizeof(double));
        for (int64_t j = 0; j < n; ++j)
            nx[j] = -x[j];
        orc_aprod1(A, nx, r, 1.0, ORC_P64);
        if (orc_lsqr(A, r, NULL, dx, NULL, NULL, 0, NULL, NULL, inner, last)) {
            rc = -1;
            goto out;
        }
        for (int64_t j = 0; j < n; ++j)
            x[j] += dx[j];
        *inner_total += last->itn;
        *outer_steps = it + 1;
        double d = nrm2(dx, n), lim = outer_tol * nrm2(x, n);
        if (d <= lim || (it > 0 && d < prev && d * (d / prev) <= lim))
            break;
        prev = d;
    }
out:
    free(r);
    free(nx);
    free(dx);
    return rc;
}

/*
 * Per-star input features of the warm-start network (28 values per star):
 *   [0..14]  the 15 upper-triangle entries (row-major) of A_s^T A_s, A_s the
 *            star's rows restricted to its 5 astrometric columns
 *   [15..19] A_s^T bt, with bt = b - A_other xo the known terms minus the
 *            attitude / instrumental / global part evaluated at xo
 *   [20] rows of the star      [21] mean(att_start) / n_att
 *   [22] std(att_start / n_att) (population)
 *   [23] rms of the 12 attitude coefficients   [24] rms of the 6 instrumental
 *   [25] rms of the global coefficient (0 without one)
 *   [26] ||bt_s|| / sqrt(rows)   [27] sum_r a_glob * bt_r / rows
 * xo has the n - 5*n_stars non-astrometric unknowns.  F is [n_stars][28].
 */
void orc_features(const orc_sys *A, const double *b, const double *xo, double *F)
{
    int ns = n_slots(A);
    int64_t NA = 5 * A->n_stars;
    for (int64_t s = 0; s < A->n_stars; ++s) {
        double *f = F + 28 * s;
        for (int i = 0; i < 28; ++i)
            f[i] = 0.0;
        int64_t r0 = A->star_row_ptr[s], r1 = A->star_row_ptr[s + 1];
        double rows = (double)(r1 - r0);
        if (r1 <= r0)
            continue;
        double mean_att = 0.0;
        for (int64_t r = r0; r < r1; ++r)
            mean_att += (double)A->att_start[r] / (double)A->n_att;
        mean_att /= rows;
        double var_att = 0.0, sq_att = 0.0, sq_ins = 0.0, sq_glb = 0.0, sq_bt = 0.0, gb = 0.0;
        for (int64_t r = r0; r < r1; ++r) {
            double bt = b[r];
            for (int k = 5; k < ns; ++k)
                bt -= coef(A, r, k) * xo[orc_col(A, s, r, k) - NA];
            int q = 0;
            for (int k = 0; k < 5; ++k)
                for (int l = k; l < 5; ++l)
                    f[q++] += coef(A, r, k) * coef(A, r, l);
            for (int k = 0; k < 5; ++k)
                f[15 + k] += coef(A, r, k) * bt;
            double da = (double)A->att_start[r] / (double)A->n_att - mean_att;
            var_att += da * da;
            for (int k = 5; k < 17; ++k)
                sq_att += coef(A, r, k) * coef(A, r, k);
            for (int k = 17; k < 23; ++k)
                sq_ins += coef(A, r, k) * coef(A, r, k);
            if (A->n_glob) {
                sq_glb += coef(A, r, 23) * coef(A, r, 23);
                gb += coef(A, r, 23) * bt;
            }
            sq_bt += bt * bt;
        }
        f[20] = rows;
        f[21] = mean_att;
        f[22] = sqrt(var_att / rows);
        f[23] = sqrt(sq_att / (12.0 * rows));
        f[24] = sqrt(sq_ins / (6.0 * rows));
        f[25] = sqrt(sq_glb / rows);
        f[26] = sqrt(sq_bt / rows);
        f[27] = gb / rows;
    }
}
