/*
 * chisao_oracle.c -- plain, slow FP64 CPU oracle for the ChiSao per-cycle
 * population update (Wolfson, "ChiSao: A GPU-Native Parallel Optimizer for
 * Multimodal Black-Box Functions via Convergence-Anticonvergence Oscillation").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
 * this file; only the test suite, the smoke check and the benchmark's CPU
 * baseline use it.  It shares no code, header, table or constant generator with
 * the HIP library: everything here is written from the paper's text.
 *
 * Conventions: every floating-point quantity is double; loops are written in
 * the order the paper states the steps; OpenMP only splits independent
 * per-sample work, and every reduction over samples runs sequentially in
 * ascending sample order after the parallel loop, so results do not depend on
 * the thread count.
 *
 * Where the paper leaves a step open, the reading used is the one named in the
 * comment (the same readings bind the GPU library).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_ESTATE (-4)

/* Philox counter layout: the top byte of the third counter word names the
 * consumer of the stream. */
enum { PH_INIT = 0, PH_RM = 4, PH_GR = 5, PH_HLC = 6, PH_NOISE = 7, PH_GATE = 8 };

/* Per-iteration L-BFGS decision codes (one byte per sample and iteration). */
#define TR_NONE 0xFF      /* sample not iterated */
#define TR_LS_MASK 0x0F   /* accepted backtracking index, 15 = search failed */
#define TR_LS_FAIL 0x0F
#define TR_STORED 0x10    /* curvature pair stored */
#define TR_CONV 0x20      /* converged after this iteration */
#define TR_RESET 0x40     /* direction was not an ascent direction: history cleared */

/* Objective families: the two mixture log-densities, then the closed-form
 * test functions of Appendix D. */
enum { FAM_GAUSS = 0, FAM_STUDENT_T = 1, FAM_RASTRIGIN = 2, FAM_ACKLEY = 3, FAM_SCHWEFEL = 4,
       FAM_STYBLINSKI_TANG = 5, FAM_MICHALEWICZ = 6, FAM_TRID = 7, FAM_BUKIN6 = 8 };

typedef struct {
    int32_t family;   /* FAM_*; the closed forms ignore K, nu, log_w, mu and prec */
    int32_t d, K;
    double nu;        /* Student-t degrees of freedom */
    const double *log_w; /* K    log mixture weights */
    const double *mu;    /* K*d  component centres */
    const double *prec;  /* K*d*d symmetric positive-definite precision (inverse covariance or inverse scale) */
    const double *lo, *hi; /* d  box domain */
    double noise_sigma;
} orc_problem;

typedef struct {
    int32_t N, m, n_osc, n_conv, n_anti, n_cloud, M;
    double eps_grad, eps_dup, log_delta, momentum, alpha, sigma, sigma_c;
    int32_t grad_mode;   /* 0 central finite differences, 1 analytic gradient */
    double fd_h;         /* >0: fixed step; <=0: h_j = 2^-8 max(1,|x_j|) */
    double ls_c1;
    int32_t ls_max;
    double curv_eps;
    int32_t gate_reps;
    uint32_t phase_mask; /* bit p enables phase p (3..6); phases 1, 2 always run */
    uint64_t seed;
    uint32_t problem_id;
    uint32_t flags;      /* bit 2: structured ray seeding of the starting population */
} orc_config;

typedef struct {
    double *X, *F, *G, *V;
    uint8_t *stuck, *active, *conv, *removed;
    double *S, *Y, *rho;
    int32_t *head, *cnt;
    int32_t k;
    int32_t gr_disabled, gr_fail, gr_used_last, gr_prev_modes;
    double f_max, sigma, alpha_c, alpha_a;
    int32_t K_lost, n_stuck, n_modes, reseed_kind, n_free, n_unfrozen;
    double *Fg; /* quality-gate values (noisy objectives only) */
    double *W;       /* N*d preserved inverse-Hessian diagonals (width export), or NULL */
    uint8_t *wvalid; /* N: W holds a value */
    int32_t n_nonfinite; /* samples deactivated by the non-finite guard of the last Phase 2 */
} orc_state;

typedef struct {
    uint8_t *trace_out;        /* (n_conv+1)*N decision codes, or NULL */
    const uint8_t *trace_in;   /* decisions to follow, or NULL */
    const uint8_t *stuck_in;   /* stick decisions to follow (before dedup), or NULL */
    const uint8_t *removed_in; /* dedup decisions to follow, or NULL */
    double tol_f, tol_g, tol_curv, tol_dist;
    int64_t n_decisions, n_borderline, n_hard;
    double worst_hard;
    int32_t first_hard_sample, first_hard_iter, first_hard_kind;
    int64_t border_by_kind[8], hard_by_kind[8];
} orc_replay;

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplies with the */
/* Weyl-sequence key schedule.                                              */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void draw4(const orc_config *C, uint32_t a, uint32_t b, uint32_t c, uint32_t e, uint32_t out[4])
{
    uint32_t key[2] = { (uint32_t)(C->seed & 0xFFFFFFFFu), (uint32_t)(C->seed >> 32) ^ C->problem_id };
    uint32_t ctr[4] = { a, b, c, e };
    orc_philox4x32_10(ctr, key, out);
}

/* Uniform in (0,1): the top 24 bits plus one half, times 2^-24. */
double orc_u01(uint32_t a) { return ((double)(a >> 8) + 0.5) * (1.0 / 16777216.0); }

/* Box-Muller on consecutive uniform pairs: four normals per Philox call. */
static void normals4(const orc_config *C, uint32_t a, uint32_t b, uint32_t c, uint32_t e, double z[4])
{
    uint32_t o[4];
    draw4(C, a, b, c, e, o);
    const double two_pi = 6.283185307179586476925286766559;
    for (int p = 0; p < 2; ++p) {
        double u1 = orc_u01(o[2 * p]), u2 = orc_u01(o[2 * p + 1]);
        double r = sqrt(-2.0 * log(u1));
        z[2 * p] = r * cos(two_pi * u2);
        z[2 * p + 1] = r * sin(two_pi * u2);
    }
}

/* Standard-normal vector of length n from blocks 0..ceil(n/4)-1. */
static void normal_vec(const orc_config *C, uint32_t a, uint32_t b, uint32_t c, int n, double *z)
{
    for (int blk = 0; 4 * blk < n; ++blk) {
        double t[4];
        normals4(C, a, b, c, (uint32_t)blk, t);
        for (int q = 0; q < 4 && 4 * blk + q < n; ++q) z[4 * blk + q] = t[q];
    }
}

/* Integer in [0, n): high word of the 64-bit product. */
static uint32_t uint_below(uint32_t a, uint32_t n) { return (uint32_t)(((uint64_t)a * (uint64_t)n) >> 32); }

/* ------------------------------------------------------------------------ */
/* Objective: mixture log-density (Gaussian mixture of Appendix D, with the  */
/* anisotropic precision of the benchmark configurations; Student-t mixture  */
/* for the noisy-likelihood configuration).                                  */
/* ------------------------------------------------------------------------ */

/* log normaliser + log weight per component; fails if a precision matrix is
 * not symmetric positive definite. */
int orc_prepare(const orc_problem *P, double *logc)
{
    int d = P->d, K = P->K;
    if (P->family >= FAM_RASTRIGIN && P->family <= FAM_BUKIN6)
        return (d < 1 || (P->family == FAM_BUKIN6 && d != 2)) ? ORC_EINVAL : ORC_OK;
    if (d < 1 || K < 1) return ORC_EINVAL;
    double *L = (double *)malloc(sizeof(double) * (size_t)d * d);
    if (!L) return ORC_ENOMEM;
    const double log_2pi = 1.8378770664093454835606594728112;
    for (int k = 0; k < K; ++k) {
        const double *A = P->prec + (size_t)k * d * d;
        /* Cholesky A = L L^T; log|A| = 2 sum log L_ii */
        double logdet = 0.0;
        for (int i = 0; i < d; ++i) {
            for (int j = 0; j <= i; ++j) {
                double s = A[(size_t)i * d + j];
                for (int q = 0; q < j; ++q) s -= L[(size_t)i * d + q] * L[(size_t)j * d + q];
                if (i == j) {
                    if (!(s > 0.0)) { free(L); return ORC_EINVAL; }
                    L[(size_t)i * d + i] = sqrt(s);
                    logdet += 2.0 * log(L[(size_t)i * d + i]);
                } else {
                    L[(size_t)i * d + j] = s / L[(size_t)j * d + j];
                }
            }
        }
        double c;
        if (P->family == 0) {
            c = -0.5 * d * log_2pi + 0.5 * logdet;
        } else {
            double nu = P->nu;
            c = lgamma(0.5 * (nu + d)) - lgamma(0.5 * nu) - 0.5 * d * log(nu * M_PI) + 0.5 * logdet;
        }
        logc[k] = P->log_w[k] + c;
    }
    free(L);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Closed-form test functions (Appendix D, each already negated so that the  */
/* optimum is a maximum) and their analytic gradients.  Coordinates are      */
/* numbered from 1 in the paper; x[i-1] here.  Where a function is not       */
/* differentiable (Ackley at the origin, Bukin N.6 on its ridge, |.| at 0)   */
/* the gradient term is taken as 0.                                          */
/* ------------------------------------------------------------------------ */
static double sgn(double v) { return (v > 0.0) - (v < 0.0); }

static double closed_form(int family, int d, const double *x, double *g)
{
    const double two_pi = 2.0 * M_PI;
    switch (family) {
    case FAM_RASTRIGIN: {
        /* -[A d + sum (x_i^2 - A cos(2 pi x_i))], A = 10 */
        const double A = 10.0;
        double s = A * d;
        for (int i = 0; i < d; ++i) {
            s += x[i] * x[i] - A * cos(two_pi * x[i]);
            if (g) g[i] = -(2.0 * x[i] + two_pi * A * sin(two_pi * x[i]));
        }
        return -s;
    }
    case FAM_ACKLEY: {
        /* -[-a exp(-b sqrt(mean x_i^2)) - exp(mean cos(c x_i)) + a + e],
         * a = 20, b = 0.2, c = 2 pi */
        const double a = 20.0, b = 0.2, c = two_pi;
        double sq = 0.0, sc = 0.0;
        for (int i = 0; i < d; ++i) {
            sq += x[i] * x[i];
            sc += cos(c * x[i]);
        }
        double r = sqrt(sq / d), ea = exp(-b * r), ec = exp(sc / d);
        if (g)
            for (int i = 0; i < d; ++i)
                g[i] = (r > 0.0 ? -a * b * ea * x[i] / (d * r) : 0.0) - ec * c * sin(c * x[i]) / d;
        return -(-a * ea - ec + a + M_E);
    }
    case FAM_SCHWEFEL: {
        /* -[418.9829 d - sum x_i sin(sqrt|x_i|)] */
        double s = 418.9829 * d;
        for (int i = 0; i < d; ++i) {
            double r = sqrt(fabs(x[i]));
            s -= x[i] * sin(r);
            /* d/dx [x sin sqrt|x|] = sin r + x cos(r) sgn(x) / (2 r) = sin r + (r/2) cos r */
            if (g) g[i] = sin(r) + 0.5 * r * cos(r);
        }
        return -s;
    }
    case FAM_STYBLINSKI_TANG: {
        /* -1/2 sum (x_i^4 - 16 x_i^2 + 5 x_i) */
        double s = 0.0;
        for (int i = 0; i < d; ++i) {
            double v = x[i];
            s += v * v * v * v - 16.0 * v * v + 5.0 * v;
            if (g) g[i] = -0.5 * (4.0 * v * v * v - 32.0 * v + 5.0);
        }
        return -0.5 * s;
    }
    case FAM_MICHALEWICZ: {
        /* sum sin(x_i) sin^(2m)(i x_i^2 / pi), m = 10 */
        const int two_m = 20;
        double s = 0.0;
        for (int i = 0; i < d; ++i) {
            double v = x[i], u = (i + 1) * v * v / M_PI, su = sin(u);
            s += sin(v) * pow(su, two_m);
            if (g)
                g[i] = cos(v) * pow(su, two_m) +
                       sin(v) * two_m * pow(su, two_m - 1) * cos(u) * (2.0 * (i + 1) * v / M_PI);
        }
        return s;
    }
    case FAM_TRID: {
        /* -[sum (x_i - 1)^2 - sum_{i>=2} x_i x_{i-1}] */
        double s = 0.0;
        for (int i = 0; i < d; ++i) s += (x[i] - 1.0) * (x[i] - 1.0);
        for (int i = 1; i < d; ++i) s -= x[i] * x[i - 1];
        if (g)
            for (int i = 0; i < d; ++i)
                g[i] = -2.0 * (x[i] - 1.0) + (i > 0 ? x[i - 1] : 0.0) + (i + 1 < d ? x[i + 1] : 0.0);
        return -s;
    }
    case FAM_BUKIN6: {
        /* -[100 sqrt|y - 0.01 x^2| + 0.01 |x + 10|], (x, y) = (x[0], x[1]) */
        double u = x[1] - 0.01 * x[0] * x[0], r = sqrt(fabs(u));
        if (g) {
            double w = r > 0.0 ? sgn(u) / r : 0.0; /* d sqrt|u| / du = sgn(u) / (2 r) */
            g[0] = -(100.0 * 0.5 * w * (-0.02 * x[0]) + 0.01 * sgn(x[0] + 10.0));
            g[1] = -(100.0 * 0.5 * w);
        }
        return -(100.0 * r + 0.01 * fabs(x[0] + 10.0));
    }
    default:
        return NAN;
    }
}

/* f(x) and, if g != NULL, its gradient.  work holds K + K*d doubles. */
static double eval_point(const orc_problem *P, const double *logc, const double *x, double *g, double *work)
{
    if (P->family >= FAM_RASTRIGIN) return closed_form(P->family, P->d, x, g);
    int d = P->d, K = P->K;
    double *lk = work;           /* K log terms */
    double *U = work + K;        /* K*d: P_k (x - mu_k) */
    double delta[512];
    double lmax = -INFINITY;
    for (int k = 0; k < K; ++k) {
        const double *mu = P->mu + (size_t)k * d;
        const double *A = P->prec + (size_t)k * d * d;
        double *u = U + (size_t)k * d;
        for (int j = 0; j < d; ++j) delta[j] = x[j] - mu[j];
        double q = 0.0;
        for (int i = 0; i < d; ++i) {
            double s = 0.0;
            for (int j = 0; j < d; ++j) s += A[(size_t)i * d + j] * delta[j];
            u[i] = s;
            q += delta[i] * s;
        }
        double l;
        if (P->family == 0) {
            l = logc[k] - 0.5 * q;
        } else {
            l = logc[k] - 0.5 * (P->nu + d) * log1p(q / P->nu);
            /* store the Student-t weight (nu+d)/(nu+q) in place of u's scale */
            double s = (P->nu + d) / (P->nu + q);
            for (int i = 0; i < d; ++i) u[i] *= s;
        }
        lk[k] = l;
        if (l > lmax) lmax = l;
    }
    double sum = 0.0;
    for (int k = 0; k < K; ++k) sum += exp(lk[k] - lmax);
    double f = lmax + log(sum);
    if (g) {
        for (int i = 0; i < d; ++i) g[i] = 0.0;
        for (int k = 0; k < K; ++k) {
            double r = exp(lk[k] - f);
            const double *u = U + (size_t)k * d;
            for (int i = 0; i < d; ++i) g[i] -= r * u[i];
        }
    }
    return f;
}

static size_t eval_work_len(const orc_problem *P)
{
    return P->family >= FAM_RASTRIGIN ? 1 : (size_t)P->K * (1 + P->d);
}

/* ------------------------------------------------------------------------ */
/* Likelihood noise (Sec. 5.7): every evaluation the method makes returns    */
/* f(x) + sigma_n z with a fresh standard normal z.  Reading: z is the first */
/* normal of the NOISE stream at counter (sample, cycle, step << 16 | sub);  */
/* sub names the evaluation within the step: the centre value 0, line-search */
/* trial r, and 0x1000 / 0x2000 | probe << 7 / 0x3000 plus the stencil index */
/* (2j for x + h e_j, 2j + 1 for x - h e_j) for the central differences of   */
/* Phase 1, of smoothing probes and of anti-convergence.  The noise does not */
/* depend on x, so the analytic gradient is noise-free.                       */
/* ------------------------------------------------------------------------ */
typedef struct {
    const orc_config *C;
    double sigma;
    uint32_t sample, cycle, step, sub;
} noise_t;

enum { NZ_FD1 = 0x1000, NZ_FD_PROBE = 0x2000, NZ_FD_ANTI = 0x3000 };

static double noise_at(const noise_t *nz, uint32_t sub)
{
    if (!nz || !(nz->sigma > 0.0)) return 0.0;
    double z[4];
    normals4(nz->C, nz->sample, nz->cycle, ((uint32_t)PH_NOISE << 24) | (nz->step << 16) | sub, 0u, z);
    return nz->sigma * z[0];
}

static noise_t noise_for(const orc_problem *P, const orc_config *C, const orc_state *S, int i, int step,
                         uint32_t sub)
{
    noise_t nz = { C, P->noise_sigma, (uint32_t)i, (uint32_t)S->k + 1u, (uint32_t)step, sub };
    return nz;
}

/* Central finite-difference gradient: g_j = (f(x+h_j e_j) - f(x-h_j e_j)) /
 * ((x_j+h_j) - (x_j-h_j)); the stencil points are not clamped. */
static void fd_grad_point(const orc_problem *P, const double *logc, double fd_h, const double *x, double *g,
                          double *work, double *xs, const noise_t *nz)
{
    int d = P->d;
    for (int j = 0; j < d; ++j) xs[j] = x[j];
    for (int j = 0; j < d; ++j) {
        double h = fd_h > 0.0 ? fd_h : ldexp(fmax(1.0, fabs(x[j])), -8);
        double xp = x[j] + h, xm = x[j] - h;
        xs[j] = xp;
        double fp = eval_point(P, logc, xs, NULL, work) + (nz ? noise_at(nz, nz->sub + 2u * j) : 0.0);
        xs[j] = xm;
        double fm = eval_point(P, logc, xs, NULL, work) + (nz ? noise_at(nz, nz->sub + 2u * j + 1u) : 0.0);
        xs[j] = x[j];
        g[j] = (fp - fm) / (xp - xm);
    }
}

void orc_eval_batch(const orc_problem *P, const double *logc, int n, const double *X, double *f, double *G)
{
    int d = P->d;
#pragma omp parallel
    {
        double *work = (double *)malloc(sizeof(double) * eval_work_len(P));
#pragma omp for schedule(dynamic, 4)
        for (int i = 0; i < n; ++i) {
            double v = eval_point(P, logc, X + (size_t)i * d, G ? G + (size_t)i * d : NULL, work);
            if (f) f[i] = v;
        }
        free(work);
    }
}

void orc_fd_grad_batch(const orc_problem *P, const double *logc, double fd_h, int n, const double *X, double *G)
{
    int d = P->d;
#pragma omp parallel
    {
        double *work = (double *)malloc(sizeof(double) * eval_work_len(P));
        double *xs = (double *)malloc(sizeof(double) * d);
#pragma omp for schedule(dynamic, 4)
        for (int i = 0; i < n; ++i)
            fd_grad_point(P, logc, fd_h, X + (size_t)i * d, G + (size_t)i * d, work, xs, NULL);
        free(xs);
        free(work);
    }
}

/* ------------------------------------------------------------------------ */
/* Small vector helpers                                                      */
/* ------------------------------------------------------------------------ */
static double dot(int n, const double *a, const double *b)
{
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}
static double nrm2(int n, const double *a) { return sqrt(dot(n, a, a)); }
static double nrminf(int n, const double *a)
{
    double s = 0.0;
    for (int i = 0; i < n; ++i) s = fmax(s, fabs(a[i]));
    return s;
}
static void clamp_box(const orc_problem *P, double *x)
{
    for (int j = 0; j < P->d; ++j) x[j] = fmin(fmax(x[j], P->lo[j]), P->hi[j]);
}

/* Per-thread scratch for one sample. */
typedef struct {
    double *work, *xs, *p, *r, *xtr, *gtr, *alpha, *margins;
} scratch_t;

static int scratch_alloc(scratch_t *s, const orc_problem *P, const orc_config *C)
{
    int d = P->d;
    s->work = (double *)malloc(sizeof(double) * eval_work_len(P));
    s->xs = (double *)malloc(sizeof(double) * d);
    s->p = (double *)malloc(sizeof(double) * d);
    s->r = (double *)malloc(sizeof(double) * d);
    s->xtr = (double *)malloc(sizeof(double) * d);
    s->gtr = (double *)malloc(sizeof(double) * d);
    s->alpha = (double *)malloc(sizeof(double) * (C->m > 0 ? C->m : 1));
    s->margins = (double *)malloc(sizeof(double) * (C->ls_max > 0 ? C->ls_max : 1));
    return (s->work && s->xs && s->p && s->r && s->xtr && s->gtr && s->alpha && s->margins) ? 0 : -1;
}
static void scratch_free(scratch_t *s)
{
    free(s->work); free(s->xs); free(s->p); free(s->r); free(s->xtr); free(s->gtr); free(s->alpha); free(s->margins);
}

/* The gradient the method uses at x: analytic (noise-free), or central
 * differences of noisy values with the stencil noise named by nz. */
static void method_grad(const orc_problem *P, const double *logc, const orc_config *C, const double *x, double *g,
                        scratch_t *s, const noise_t *nz)
{
    if (C->grad_mode == 1) (void)eval_point(P, logc, x, g, s->work);
    else fd_grad_point(P, logc, C->fd_h, x, g, s->work, s->xs, nz);
}

/* ------------------------------------------------------------------------ */
/* L-BFGS two-loop recursion (Nocedal & Wright, Algorithm 7.4) for the       */
/* minimisation of F = -f.  The ring holds cnt pairs; the newest sits in     */
/* slot head.  Returns the ascent direction p = -H grad F in p.              */
/* ------------------------------------------------------------------------ */
void orc_two_loop(int d, int m, int cnt, int head, const double *S, const double *Y, const double *rho,
                  const double *g, double *p, double *alpha)
{
    double *q = p; /* work in place */
    for (int i = 0; i < d; ++i) q[i] = -g[i]; /* grad F */
    for (int j = 0; j < cnt; ++j) {
        int slot = (head - j + m) % m;
        alpha[j] = rho[slot] * dot(d, S + (size_t)slot * d, q);
        for (int i = 0; i < d; ++i) q[i] -= alpha[j] * Y[(size_t)slot * d + i];
    }
    double gamma;
    if (cnt > 0) {
        const double *s = S + (size_t)head * d, *y = Y + (size_t)head * d;
        gamma = dot(d, s, y) / dot(d, y, y);
    } else {
        gamma = 1.0 / fmax(nrm2(d, g), 1.0);
    }
    for (int i = 0; i < d; ++i) q[i] *= gamma; /* r = H0 q */
    for (int j = cnt - 1; j >= 0; --j) {
        int slot = (head - j + m) % m;
        double beta = rho[slot] * dot(d, Y + (size_t)slot * d, q);
        for (int i = 0; i < d; ++i) q[i] += S[(size_t)slot * d + i] * (alpha[j] - beta);
    }
    for (int i = 0; i < d; ++i) p[i] = -q[i];
}

/* ------------------------------------------------------------------------ */
/* Decision replay bookkeeping: the oracle compares its own decision with    */
/* the one it is told to follow; a disagreement is borderline when the       */
/* oracle's own margin is within tolerance, otherwise it is a hard mismatch. */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t n_dec, n_border, n_hard;
    double worst;
    int32_t hard_iter, hard_kind;
    int32_t border_kind[8], hard_kind_n[8];
} sample_replay_t;

static void note_disagreement(sample_replay_t *sr, int borderline, double margin, int iter, int kind)
{
    if (borderline) {
        sr->n_border++;
        sr->border_kind[kind & 7]++;
    } else {
        if (sr->n_hard == 0) { sr->hard_iter = iter; sr->hard_kind = kind; }
        sr->n_hard++;
        sr->hard_kind_n[kind & 7]++;
        if (fabs(margin) > sr->worst) sr->worst = fabs(margin);
    }
}

enum { KIND_LS = 1, KIND_CURV = 2, KIND_CONV = 3, KIND_STICK = 4, KIND_DEDUP = 5 };

static void fold_replay(orc_replay *R, const sample_replay_t *sr, int N)
{
    if (!R) return;
    for (int i = 0; i < N; ++i) {
        R->n_decisions += sr[i].n_dec;
        R->n_borderline += sr[i].n_border;
        for (int q = 0; q < 8; ++q) {
            R->border_by_kind[q] += sr[i].border_kind[q];
            R->hard_by_kind[q] += sr[i].hard_kind_n[q];
        }
        if (sr[i].n_hard > 0) {
            if (R->n_hard == 0) {
                R->first_hard_sample = i;
                R->first_hard_iter = sr[i].hard_iter;
                R->first_hard_kind = sr[i].hard_kind;
            }
            R->n_hard += sr[i].n_hard;
            if (sr[i].worst > R->worst_hard) R->worst_hard = sr[i].worst;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Phase 1: release all, then n_conv batched L-BFGS ascent iterations.       */
/* Readings: projected Armijo backtracking t = 2^-i (c1, ls_max trials;     */
/* relaxed by 2 sigma_n for noisy objectives),                               */
/* failure means no move and a cleared history; the scaling gamma is         */
/* s'y/y'y of the newest pair (1/max(|g|,1) with none); a pair is stored     */
/* when s'y > curv_eps |s||y|; a sample whose gradient sup-norm falls below  */
/* eps_grad stops moving for the rest of the phase.                          */
/* ------------------------------------------------------------------------ */
static void lbfgs_iteration(const orc_problem *P, const double *logc, const orc_config *C, orc_state *S, int i,
                            int iter, scratch_t *sc, const orc_replay *R, sample_replay_t *sr, uint8_t *code_out)
{
    int d = P->d, m = C->m;
    double *x = S->X + (size_t)i * d, *g = S->G + (size_t)i * d;
    double *Sh = S->S + (size_t)i * m * d, *Yh = S->Y + (size_t)i * m * d, *rh = S->rho + (size_t)i * m;
    double f = S->F[i];
    uint8_t code = 0;
    const uint8_t *forced = (R && R->trace_in) ? &R->trace_in[(size_t)iter * C->N + i] : NULL;
    const noise_t nz = noise_for(P, C, S, i, iter, 0u);
    /* With evaluation noise the sufficient-increase test is relaxed by twice
     * the noise level (the noise-aware Armijo condition of Berahas, Byrd and
     * Nocedal, SIAM J. Optim. 29 (2019)): the plain test on two noisy values
     * rejects most steps once the true gain falls below the noise. */
    const double relax = 2.0 * P->noise_sigma;

    orc_two_loop(d, m, S->cnt[i], S->head[i], Sh, Yh, rh, g, sc->p, sc->alpha);
    double gp = dot(d, g, sc->p);
    if (!(gp > 0.0)) {
        S->cnt[i] = 0;
        S->head[i] = m - 1;
        double g0 = 1.0 / fmax(nrm2(d, g), 1.0);
        for (int j = 0; j < d; ++j) sc->p[j] = g0 * g[j];
        code |= TR_RESET;
    }

    /* backtracking: the first trial whose Armijo margin is >= 0 */
    int own = TR_LS_FAIL;
    int n_eval = 0;
    for (int t = 0; t < C->ls_max; ++t) {
        double step = ldexp(1.0, -t);
        for (int j = 0; j < d; ++j) sc->xtr[j] = x[j] + step * sc->p[j];
        clamp_box(P, sc->xtr);
        double ftr = eval_point(P, logc, sc->xtr, NULL, sc->work) + noise_at(&nz, (uint32_t)t);
        for (int j = 0; j < d; ++j) sc->r[j] = sc->xtr[j] - x[j];
        sc->margins[t] = ftr - f - C->ls_c1 * dot(d, g, sc->r) + relax;
        n_eval = t + 1;
        if (sc->margins[t] >= 0.0) { own = t; break; }
    }
    int use = own;
    if (forced && *forced == TR_NONE) {
        sr->n_dec++;
        note_disagreement(sr, 0, 1.0, iter, KIND_LS);
    }
    if (forced) {
        int gpu = (*forced == TR_NONE) ? -1 : (*forced & TR_LS_MASK);
        sr->n_dec++;
        if (gpu >= 0 && gpu != own) {
            /* make sure the margins the comparison needs are known */
            int need = (gpu == TR_LS_FAIL) ? C->ls_max : gpu + 1;
            for (int t = n_eval; t < need && t < C->ls_max; ++t) {
                double step = ldexp(1.0, -t);
                for (int j = 0; j < d; ++j) sc->xtr[j] = x[j] + step * sc->p[j];
                clamp_box(P, sc->xtr);
                double ftr = eval_point(P, logc, sc->xtr, NULL, sc->work) + noise_at(&nz, (uint32_t)t);
                for (int j = 0; j < d; ++j) sc->r[j] = sc->xtr[j] - x[j];
                sc->margins[t] = ftr - f - C->ls_c1 * dot(d, g, sc->r) + relax;
            }
            double tol = R->tol_f * fmax(1.0, fabs(f));
            double mgn;
            if (gpu != TR_LS_FAIL && (own == TR_LS_FAIL || gpu < own)) mgn = sc->margins[gpu]; /* oracle rejected it */
            else mgn = sc->margins[own];                                                     /* oracle accepted it */
            note_disagreement(sr, fabs(mgn) <= tol, mgn / fmax(1.0, fabs(f)), iter, KIND_LS);
            use = gpu;
        }
    }

    if (use == TR_LS_FAIL) {
        code |= TR_LS_FAIL;
        S->cnt[i] = 0;
        S->head[i] = m - 1;
    } else {
        code |= (uint8_t)use;
        double step = ldexp(1.0, -use);
        for (int j = 0; j < d; ++j) sc->xtr[j] = x[j] + step * sc->p[j];
        clamp_box(P, sc->xtr);
        /* the accepted trial's value, as the search saw it (same noise draw) */
        double fnew = eval_point(P, logc, sc->xtr, C->grad_mode == 1 ? sc->gtr : NULL, sc->work) +
                      noise_at(&nz, (uint32_t)use);
        noise_t nzf = nz;
        nzf.sub = NZ_FD1;
        if (C->grad_mode != 1) fd_grad_point(P, logc, C->fd_h, sc->xtr, sc->gtr, sc->work, sc->xs, &nzf);
        /* curvature pair for F = -f: s = x_new - x, y = grad F(x_new) - grad F(x) */
        double *s = sc->r, *y = sc->p;
        for (int j = 0; j < d; ++j) { s[j] = sc->xtr[j] - x[j]; y[j] = -(sc->gtr[j] - g[j]); }
        double sy = dot(d, s, y), ns = nrm2(d, s), ny = nrm2(d, y);
        int store = sy > C->curv_eps * ns * ny;
        if (forced && *forced != TR_NONE) {
            int gpu_store = (*forced & TR_STORED) ? 1 : 0;
            sr->n_dec++;
            if (gpu_store != store) {
                double cosv = (ns > 0 && ny > 0) ? sy / (ns * ny) : 0.0;
                double mgn = cosv - C->curv_eps;
                /* a step within a few single-precision ulps of x may round to
                 * no move at all in the compared FP32 run (s = 0, nothing to
                 * store): its pair decision is borderline whatever the cosine */
                double srel = 0.0;
                for (int j = 0; j < d; ++j) srel = fmax(srel, fabs(s[j]) / fmax(fabs(x[j]), 1e-30));
                int below_fp32 = srel < 0x1p-21;
                note_disagreement(sr, below_fp32 || fabs(mgn) <= R->tol_curv, mgn, iter, KIND_CURV);
                store = gpu_store;
            }
        }
        if (store && sy != 0.0) {
            int h = (S->head[i] + 1) % m;
            memcpy(Sh + (size_t)h * d, s, sizeof(double) * d);
            memcpy(Yh + (size_t)h * d, y, sizeof(double) * d);
            rh[h] = 1.0 / sy;
            S->head[i] = h;
            if (S->cnt[i] < m) S->cnt[i]++;
            code |= TR_STORED;
        }
        memcpy(x, sc->xtr, sizeof(double) * d);
        memcpy(g, sc->gtr, sizeof(double) * d);
        S->F[i] = fnew;
    }

    double gi = nrminf(d, g);
    int conv = gi < C->eps_grad;
    if (forced && *forced != TR_NONE) {
        int gpu_conv = (*forced & TR_CONV) ? 1 : 0;
        sr->n_dec++;
        if (gpu_conv != conv) {
            double mgn = (gi - C->eps_grad) / C->eps_grad;
            note_disagreement(sr, fabs(mgn) <= R->tol_g, mgn, iter, KIND_CONV);
            conv = gpu_conv;
        }
    }
    if (conv) { S->conv[i] = 1; code |= TR_CONV; }
    *code_out = code;
}

int orc_phase_converge(const orc_problem *P, const double *logc, const orc_config *C, orc_state *S, orc_replay *R)
{
    int N = C->N, d = P->d, m = C->m;
    if (C->ls_max < 1 || C->ls_max > 15) return ORC_EINVAL; /* trace codes keep the index in 4 bits, 15 = failed */
    sample_replay_t *sr = (sample_replay_t *)calloc((size_t)N, sizeof(sample_replay_t));
    if (!sr) return ORC_ENOMEM;
    uint8_t *trace = (R && R->trace_out) ? R->trace_out : NULL;
    int err = 0;
    /* release all: every sample unfrozen, every history emptied */
    for (int i = 0; i < N; ++i) {
        S->stuck[i] = 0;
        S->removed[i] = 0;
        S->conv[i] = 0;
        S->cnt[i] = 0;
        S->head[i] = m - 1;
    }
#pragma omp parallel
    {
        scratch_t sc;
        if (scratch_alloc(&sc, P, C)) {
#pragma omp atomic write
            err = 1;
        }
        /* initial values and gradients at the current positions */
#pragma omp for schedule(dynamic, 2)
        for (int i = 0; i < N; ++i) {
            uint8_t code = TR_NONE;
            if (S->active[i] && !err) {
                double *x = S->X + (size_t)i * d, *g = S->G + (size_t)i * d;
                const noise_t nz0 = noise_for(P, C, S, i, 0, 0u), nzf = noise_for(P, C, S, i, 0, NZ_FD1);
                S->F[i] = eval_point(P, logc, x, C->grad_mode == 1 ? g : NULL, sc.work) + noise_at(&nz0, 0u);
                if (C->grad_mode != 1) fd_grad_point(P, logc, C->fd_h, x, g, sc.work, sc.xs, &nzf);
                double gi = nrminf(d, g);
                int conv = gi < C->eps_grad;
                if (R && R->trace_in && R->trace_in[i] != TR_NONE) {
                    int gpu_conv = (R->trace_in[i] & TR_CONV) ? 1 : 0;
                    sr[i].n_dec++;
                    if (gpu_conv != conv) {
                        double mgn = (gi - C->eps_grad) / C->eps_grad;
                        note_disagreement(&sr[i], fabs(mgn) <= R->tol_g, mgn, 0, KIND_CONV);
                        conv = gpu_conv;
                    }
                }
                S->conv[i] = (uint8_t)conv;
                code = conv ? TR_CONV : 0;
            }
            if (trace) trace[i] = code;
        }
        for (int it = 1; it <= C->n_conv; ++it) {
#pragma omp for schedule(dynamic, 2)
            for (int i = 0; i < N; ++i) {
                uint8_t code = TR_NONE;
                if (S->active[i] && !S->conv[i] && !err)
                    lbfgs_iteration(P, logc, C, S, i, it, &sc, R, &sr[i], &code);
                if (trace) trace[(size_t)it * N + i] = code;
            }
        }
        scratch_free(&sc);
    }
    fold_replay(R, sr, N);
    free(sr);
    return err ? ORC_ENOMEM : ORC_OK;
}

/* Continue Phase 1 from the current state: iterations first..first+n-1 for
 * active samples not yet converged, with the stored histories (no release, no
 * initial evaluation).  Trace rows are indexed by iteration number. */
int orc_lbfgs_iterate(const orc_problem *P, const double *logc, const orc_config *C, orc_state *S, int first, int n,
                      orc_replay *R)
{
    int N = C->N;
    if (first < 1 || first + n - 1 > C->n_conv) return ORC_EINVAL;
    if (C->ls_max < 1 || C->ls_max > 15) return ORC_EINVAL;
    sample_replay_t *sr = (sample_replay_t *)calloc((size_t)N, sizeof(sample_replay_t));
    if (!sr) return ORC_ENOMEM;
    uint8_t *trace = (R && R->trace_out) ? R->trace_out : NULL;
    int err = 0;
#pragma omp parallel
    {
        scratch_t sc;
        if (scratch_alloc(&sc, P, C)) {
#pragma omp atomic write
            err = 1;
        }
        for (int it = first; it < first + n; ++it) {
#pragma omp for schedule(dynamic, 2)
            for (int i = 0; i < N; ++i) {
                uint8_t code = TR_NONE;
                if (S->active[i] && !S->conv[i] && !err)
                    lbfgs_iteration(P, logc, C, S, i, it, &sc, R, &sr[i], &code);
                if (trace) trace[(size_t)it * N + i] = code;
            }
        }
        scratch_free(&sc);
    }
    fold_replay(R, sr, N);
    free(sr);
    return err ? ORC_ENOMEM : ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Phase 2: stick test.  f_max is the largest value over active samples     */
/* (with noise: re-estimated at the sample with the largest gate value);     */
/* stuck = (|grad f|_inf < eps_grad) and (f >= f_max + log delta).           */
/* ------------------------------------------------------------------------ */
/* The value the quality gate, the deduplication order and the mode output
 * use: f as the search saw it, or with noise the gate value. */
static const double *gate_values(const orc_problem *P, const orc_state *S)
{
    return (P->noise_sigma > 0.0 && S->Fg) ? S->Fg : S->F;
}

/* Gate value under noise (reading of Sec. 5.7, whose method the paper leaves
 * to SunBURST): the mean of R fresh noisy evaluations at x_i, R = gate_reps
 * (M when not given), i.e. f(x_i) + sigma_n (1/R) sum_r z_r with z_r the
 * normals of the GATE stream at counter (sample, cycle, GATE << 24, block). */
static int compute_gate_values(const orc_problem *P, const double *logc, const orc_config *C, orc_state *S)
{
    int N = C->N, d = P->d;
    int R = C->gate_reps > 0 ? C->gate_reps : C->M;
    int err = 0;
#pragma omp parallel
    {
        double *work = (double *)malloc(sizeof(double) * eval_work_len(P));
        if (!work) {
#pragma omp atomic write
            err = 1;
        }
#pragma omp for schedule(dynamic, 4)
        for (int i = 0; i < N; ++i) {
            if (!S->active[i] || !work) continue;
            double f = eval_point(P, logc, S->X + (size_t)i * d, NULL, work);
            double zs = 0.0;
            for (int b = 0; 4 * b < R; ++b) {
                double z[4];
                normals4(C, (uint32_t)i, (uint32_t)S->k + 1u, (uint32_t)PH_GATE << 24, (uint32_t)b, z);
                for (int q = 0; q < 4 && 4 * b + q < R; ++q) zs += z[q];
            }
            S->Fg[i] = f + P->noise_sigma * (zs / R);
        }
        free(work);
    }
    return err ? ORC_ENOMEM : ORC_OK;
}

int orc_phase_stick(const orc_problem *P, const double *logc, const orc_config *C, orc_state *S, orc_replay *R)
{
    int N = C->N, d = P->d;
    if (N < 1) return ORC_EINVAL;
    if (P->noise_sigma > 0.0) {
        if (!S->Fg) return ORC_EINVAL;
        int rc = compute_gate_values(P, logc, C, S);
        if (rc) return rc;
    }
    const double *Fv = gate_values(P, S);
    /* A sample whose value, gate value or gradient is not finite leaves the
     * population here, before f_max and every later reduction over samples
     * (the paper is silent on non-finite evaluations; reading). */
    int nbad = 0;
    for (int i = 0; i < N; ++i) {
        if (!S->active[i]) continue;
        int ok = isfinite(S->F[i]) && isfinite(Fv[i]);
        for (int l = 0; ok && l < d; ++l) ok = isfinite(S->G[(size_t)i * d + l]);
        if (!ok) {
            S->active[i] = 0;
            ++nbad;
        }
    }
    S->n_nonfinite = nbad;
    double fmax_ = -INFINITY;
    int best = -1;
    for (int i = 0; i < N; ++i)
        if (S->active[i] && Fv[i] > fmax_) {
            fmax_ = Fv[i];
            best = i;
        }
    if (P->noise_sigma > 0.0 && best >= 0) {
        /* Reading (noise): the largest gate value over many samples, most of
         * them copies of the same peak, overestimates that peak by the
         * largest of their noise terms.  f_max is instead the objective at
         * the sample with the largest gate value, estimated afresh: f there
         * plus sigma_n times the mean of R new normals (GATE stream,
         * sub-stream 1), unbiased for f at that sample. */
        int R = C->gate_reps > 0 ? C->gate_reps : C->M;
        double zs = 0.0;
        for (int b = 0; 4 * b < R; ++b) {
            double z[4];
            normals4(C, (uint32_t)best, (uint32_t)S->k + 1u, ((uint32_t)PH_GATE << 24) | 1u, (uint32_t)b, z);
            for (int q = 0; q < 4 && 4 * b + q < R; ++q) zs += z[q];
        }
        double *work = (double *)malloc(sizeof(double) * eval_work_len(P));
        if (!work) return ORC_ENOMEM;
        double f_best = eval_point(P, logc, S->X + (size_t)best * d, NULL, work);
        free(work);
        fmax_ = f_best + P->noise_sigma * (zs / R);
    }
    S->f_max = fmax_;
    double gate = fmax_ + C->log_delta;
    sample_replay_t *sr = (sample_replay_t *)calloc((size_t)N, sizeof(sample_replay_t));
    if (!sr) return ORC_ENOMEM;
    int n = 0;
    for (int i = 0; i < N; ++i) {
        int st = 0;
        double gi = 0.0;
        if (S->active[i]) {
            gi = nrminf(d, S->G + (size_t)i * d);
            st = (gi < C->eps_grad) && (Fv[i] >= gate);
        }
        if (R && R->stuck_in && S->active[i]) {
            int gpu = R->stuck_in[i] ? 1 : 0;
            sr[i].n_dec++;
            if (gpu != st) {
                double mg = (gi - C->eps_grad) / C->eps_grad;
                double mf = (Fv[i] - gate) / fmax(1.0, fabs(Fv[i]));
                int border = (fabs(mg) <= R->tol_g) || (fabs(mf) <= R->tol_f);
                note_disagreement(&sr[i], border, fabs(mg) < fabs(mf) ? mg : mf, 0, KIND_STICK);
                st = gpu;
            }
        }
        S->stuck[i] = (uint8_t)st;
        n += st;
    }
    S->n_stuck = n;
    fold_replay(R, sr, N);
    free(sr);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Phase 3: L-infinity deduplication among stuck samples (Appendix A).       */
/* Reading of the tie rule: sample j is removed when some other stuck        */
/* sample i lies within eps_dup in the sup-norm and ranks above j in the     */
/* strict order (higher f first, then lower index).  Every stuck sample,     */
/* removed or not, takes part in the comparison.                             */
/* ------------------------------------------------------------------------ */
/* Width export (Phase 3: the surviving sample's inverse Hessian estimate is
 * preserved for width estimation).  The estimate is the L-BFGS inverse
 * Hessian of F = -f that the sample's pairs define, i.e. the matrix the
 * two-loop recursion applies; its diagonal is read off by applying the
 * two-loop to each unit vector.  Survivors with pairs (from this cycle's
 * Phase 1) are refreshed; a survivor without pairs keeps the diagonal it
 * had, or, if it never had one, takes the two-loop's initial matrix for an
 * empty history, 1 / max(|grad f|_2, 1) times I. */
static void preserve_widths(const orc_problem *P, const orc_config *C, orc_state *S)
{
    int d = P->d, m = C->m;
    if (!S->W || !S->wvalid) return;
#pragma omp parallel
    {
        double *e = (double *)malloc(sizeof(double) * d);
        double *p = (double *)malloc(sizeof(double) * d);
        double *al = (double *)malloc(sizeof(double) * m);
#pragma omp for schedule(dynamic, 16)
        for (int i = 0; i < C->N; ++i) {
            if (!(S->stuck[i] && S->active[i])) continue;
            double *w = S->W + (size_t)i * d;
            if (S->cnt[i] > 0) {
                for (int j = 0; j < d; ++j) {
                    /* the two-loop returns -H(-g); with g = -e_j it returns -H e_j */
                    for (int k = 0; k < d; ++k) e[k] = (k == j) ? -1.0 : 0.0;
                    orc_two_loop(d, m, S->cnt[i], S->head[i], S->S + (size_t)i * m * d, S->Y + (size_t)i * m * d,
                                 S->rho + (size_t)i * m, e, p, al);
                    w[j] = -p[j];
                }
                S->wvalid[i] = 1;
            } else if (!S->wvalid[i]) {
                double g0 = 1.0 / fmax(nrm2(d, S->G + (size_t)i * d), 1.0);
                for (int j = 0; j < d; ++j) w[j] = g0;
                S->wvalid[i] = 1;
            }
        }
        free(e);
        free(p);
        free(al);
    }
}

int orc_phase_dedup(const orc_problem *P, const orc_config *C, orc_state *S, orc_replay *R)
{
    int N = C->N, d = P->d;
    int dedup_on = (C->phase_mask >> 3) & 1;
    const double *Fv = gate_values(P, S);
    uint8_t *rem = (uint8_t *)calloc((size_t)N, 1);
    sample_replay_t *sr = (sample_replay_t *)calloc((size_t)N, sizeof(sample_replay_t));
    if (!rem || !sr) { free(rem); free(sr); return ORC_ENOMEM; }
    if (dedup_on) {
#pragma omp parallel for schedule(dynamic, 8)
        for (int j = 0; j < N; ++j) {
            if (!S->stuck[j]) continue;
            const double *xj = S->X + (size_t)j * d;
            int removed = 0, border = 0;
            for (int i = 0; i < N; ++i) {
                if (i == j || !S->stuck[i]) continue;
                const double *xi = S->X + (size_t)i * d;
                double dist = 0.0;
                for (int l = 0; l < d; ++l) dist = fmax(dist, fabs(xi[l] - xj[l]));
                int near = dist < C->eps_dup;
                int above = (Fv[i] > Fv[j]) || (Fv[i] == Fv[j] && i < j);
                if (near && above) removed = 1;
                if (R && (fabs(dist - C->eps_dup) <= R->tol_dist ||
                          (dist < C->eps_dup + R->tol_dist &&
                           fabs(Fv[i] - Fv[j]) <= R->tol_f * fmax(1.0, fabs(Fv[j])))))
                    border = 1;
            }
            if (R && R->removed_in) {
                int gpu = R->removed_in[j] ? 1 : 0;
                sr[j].n_dec++;
                if (gpu != removed) {
                    note_disagreement(&sr[j], border, 1.0, 0, KIND_DEDUP);
                    removed = gpu;
                }
            }
            rem[j] = (uint8_t)removed;
        }
    }
    int lost = 0, modes = 0;
    for (int i = 0; i < N; ++i) {
        S->removed[i] = rem[i];
        if (rem[i]) { S->stuck[i] = 0; lost++; }
        if (S->stuck[i]) modes++;
    }
    S->K_lost = lost;
    S->n_modes = modes;
    fold_replay(R, sr, N);
    free(sr);
    free(rem);
    preserve_widths(P, C, S);
    /* Golden Rooster bookkeeping: a generation that found no new peak counts
     * as a failure; two in a row disable it for good. */
    if (S->gr_used_last) {
        if (modes <= S->gr_prev_modes) S->gr_fail++;
        else S->gr_fail = 0;
        if (S->gr_fail >= 2) S->gr_disabled = 1;
        S->gr_used_last = 0;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Householder QR of a d x d matrix (row-major), returning the orthogonal    */
/* factor with the signs chosen so that diag(R) > 0.                         */
/* ------------------------------------------------------------------------ */
int orc_householder_q(int d, const double *A_in, double *Q, double *R_out)
{
    double *A = (double *)malloc(sizeof(double) * (size_t)d * d);
    double *v = (double *)malloc(sizeof(double) * d);
    if (!A || !v) { free(A); free(v); return ORC_ENOMEM; }
    memcpy(A, A_in, sizeof(double) * (size_t)d * d);
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) Q[(size_t)i * d + j] = (i == j) ? 1.0 : 0.0;
    for (int c = 0; c < d; ++c) {
        double nrm = 0.0;
        for (int i = c; i < d; ++i) nrm += A[(size_t)i * d + c] * A[(size_t)i * d + c];
        nrm = sqrt(nrm);
        if (nrm == 0.0) continue;
        double a0 = A[(size_t)c * d + c];
        double alpha = (a0 > 0.0) ? -nrm : nrm;
        for (int i = 0; i < d; ++i) v[i] = 0.0;
        for (int i = c; i < d; ++i) v[i] = A[(size_t)i * d + c];
        v[c] -= alpha;
        double vn = 0.0;
        for (int i = c; i < d; ++i) vn += v[i] * v[i];
        if (vn == 0.0) continue;
        /* A <- (I - 2 v v^T / v^T v) A */
        for (int j = c; j < d; ++j) {
            double s = 0.0;
            for (int i = c; i < d; ++i) s += v[i] * A[(size_t)i * d + j];
            s *= 2.0 / vn;
            for (int i = c; i < d; ++i) A[(size_t)i * d + j] -= s * v[i];
        }
        /* Q <- Q (I - 2 v v^T / v^T v) */
        for (int i = 0; i < d; ++i) {
            double s = 0.0;
            for (int l = c; l < d; ++l) s += Q[(size_t)i * d + l] * v[l];
            s *= 2.0 / vn;
            for (int l = c; l < d; ++l) Q[(size_t)i * d + l] -= s * v[l];
        }
    }
    /* sign fix: make diag(R) positive by flipping Q's columns and R's rows */
    for (int c = 0; c < d; ++c) {
        if (A[(size_t)c * d + c] < 0.0) {
            for (int i = 0; i < d; ++i) Q[(size_t)i * d + c] = -Q[(size_t)i * d + c];
            for (int j = 0; j < d; ++j) A[(size_t)c * d + j] = -A[(size_t)c * d + j];
        }
    }
    if (R_out) {
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j) R_out[(size_t)i * d + j] = (j >= i) ? A[(size_t)i * d + j] : 0.0;
    }
    free(A);
    free(v);
    return ORC_OK;
}

/* Distance to the box boundary along a ray from o with direction u. */
static double ray_to_box(const orc_problem *P, const double *o, const double *u)
{
    double tmax = INFINITY;
    for (int l = 0; l < P->d; ++l) {
        if (u[l] > 0.0) tmax = fmin(tmax, (P->hi[l] - o[l]) / u[l]);
        else if (u[l] < 0.0) tmax = fmin(tmax, (P->lo[l] - o[l]) / u[l]);
    }
    if (!(tmax >= 0.0)) tmax = 0.0;
    if (isinf(tmax)) tmax = 0.0;
    return tmax;
}

/* ------------------------------------------------------------------------ */
/* Phase 4: reseed the K_lost removed slots.  Repulse Monkey when at least   */
/* five unfrozen samples remain: each slot draws an origin among them, an    */
/* isotropic direction and a uniform position on the ray up to the box       */
/* boundary.  Golden Rooster otherwise: slot j (in ascending order) uses     */
/* peak j mod |peaks| and direction (-1)^q Q[:, floor(q/2) mod d] with       */
/* q = floor(j / |peaks|), Q the orthogonal factor of a Gaussian matrix.     */
/* With Golden Rooster disabled the slots become inactive.                   */
/* ------------------------------------------------------------------------ */
int orc_phase_reseed(const orc_problem *P, const orc_config *C, orc_state *S)
{
    int N = C->N, d = P->d, m = C->m;
    uint32_t k = (uint32_t)S->k + 1;
    S->reseed_kind = 0;
    if (!((C->phase_mask >> 4) & 1) || S->K_lost == 0) return ORC_OK;
    int *freel = (int *)malloc(sizeof(int) * N), *slots = (int *)malloc(sizeof(int) * N),
        *peaks = (int *)malloc(sizeof(int) * N);
    double *u = (double *)malloc(sizeof(double) * d);
    if (!freel || !slots || !peaks || !u) { free(freel); free(slots); free(peaks); free(u); return ORC_ENOMEM; }
    int nf = 0, ns = 0, np = 0;
    for (int i = 0; i < N; ++i) {
        if (S->removed[i]) slots[ns++] = i;
        else if (S->active[i] && !S->stuck[i]) freel[nf++] = i;
        else if (S->active[i] && S->stuck[i]) peaks[np++] = i;
    }
    S->n_free = nf;
    if (nf >= 5) {
        S->reseed_kind = 1;
        for (int j = 0; j < ns; ++j) {
            int s = slots[j];
            uint32_t o4[4];
            draw4(C, (uint32_t)s, k, (uint32_t)PH_RM << 24, 0, o4);
            int origin = freel[uint_below(o4[0], (uint32_t)nf)];
            double frac = orc_u01(o4[1]);
            normal_vec(C, (uint32_t)s, k, ((uint32_t)PH_RM << 24) | (1u << 16), d, u);
            double nu = nrm2(d, u);
            for (int l = 0; l < d; ++l) u[l] /= nu;
            const double *o = S->X + (size_t)origin * d;
            double tmax = ray_to_box(P, o, u);
            double *x = S->X + (size_t)s * d;
            for (int l = 0; l < d; ++l) x[l] = o[l] + frac * tmax * u[l];
            clamp_box(P, x);
        }
    } else if (!S->gr_disabled && np > 0) {
        S->reseed_kind = 2;
        int nq = ns < np ? ns : np; /* peaks that receive at least one slot */
        double *A = (double *)malloc(sizeof(double) * (size_t)d * d);
        double *Q = (double *)malloc(sizeof(double) * (size_t)d * d * nq);
        if (!A || !Q) { free(A); free(Q); free(freel); free(slots); free(peaks); free(u); return ORC_ENOMEM; }
        for (int q = 0; q < nq; ++q) {
            int p = peaks[q];
            normal_vec(C, (uint32_t)p, k, ((uint32_t)PH_GR << 24), d * d, A);
            orc_householder_q(d, A, Q + (size_t)q * d * d, NULL);
        }
        for (int j = 0; j < ns; ++j) {
            int s = slots[j];
            int q = j % np, use = j / np;
            int col = (use / 2) % d;
            double sgn = (use % 2) ? -1.0 : 1.0;
            const double *Qp = Q + (size_t)q * d * d;
            for (int l = 0; l < d; ++l) u[l] = sgn * Qp[(size_t)l * d + col];
            uint32_t o4[4];
            draw4(C, (uint32_t)s, k, ((uint32_t)PH_GR << 24) | (1u << 16), 0, o4);
            double frac = orc_u01(o4[0]);
            const double *o = S->X + (size_t)peaks[q] * d;
            double tmax = ray_to_box(P, o, u);
            double *x = S->X + (size_t)s * d;
            for (int l = 0; l < d; ++l) x[l] = o[l] + frac * tmax * u[l];
            clamp_box(P, x);
        }
        S->gr_used_last = 1;
        S->gr_prev_modes = S->n_modes;
        free(A);
        free(Q);
    } else {
        S->reseed_kind = 3;
        for (int j = 0; j < ns; ++j) S->active[slots[j]] = 0;
    }
    for (int j = 0; j < ns; ++j) {
        int s = slots[j];
        S->removed[s] = 0;
        S->stuck[s] = 0;
        S->cnt[s] = 0;
        S->head[s] = m - 1;
        if (S->wvalid) S->wvalid[s] = 0;
        for (int l = 0; l < d; ++l) S->V[(size_t)s * d + l] = 0.0;
    }
    free(freel);
    free(slots);
    free(peaks);
    free(u);
    return ORC_OK;
}

/* Unfrozen = active and not stuck.  Returns the count. */
static int unfrozen_count(const orc_config *C, const orc_state *S)
{
    int n = 0;
    for (int i = 0; i < C->N; ++i) n += (S->active[i] && !S->stuck[i]);
    return n;
}

/* sigma: given, else c times the pooled standard deviation (square root of
 * the mean per-coordinate population variance) of the unfrozen samples. */
static double choose_sigma(const orc_problem *P, const orc_config *C, const orc_state *S)
{
    if (C->sigma > 0.0) return C->sigma;
    int N = C->N, d = P->d, n = 0;
    double *mean = (double *)calloc((size_t)d, sizeof(double));
    if (!mean) return 0.0;
    for (int i = 0; i < N; ++i) {
        if (!(S->active[i] && !S->stuck[i])) continue;
        n++;
        for (int l = 0; l < d; ++l) mean[l] += S->X[(size_t)i * d + l];
    }
    if (n == 0) { free(mean); return 0.0; }
    for (int l = 0; l < d; ++l) mean[l] /= n;
    double var = 0.0;
    for (int l = 0; l < d; ++l) {
        double v = 0.0;
        for (int i = 0; i < N; ++i) {
            if (!(S->active[i] && !S->stuck[i])) continue;
            double t = S->X[(size_t)i * d + l] - mean[l];
            v += t * t;
        }
        var += v / n;
    }
    free(mean);
    return C->sigma_c * sqrt(var / d);
}

/* ------------------------------------------------------------------------ */
/* Phase 5: Hands Like Clouds.  n_cloud ascent steps along the Monte Carlo   */
/* smoothed gradient (1/M) sum_m grad f(x + sigma z_m), with probes taken in */
/* antithetic pairs (z, -z) and never clamped.  The step length alpha_c is   */
/* fixed at the first step so that the mean first displacement over the     */
/* unfrozen samples equals sigma (a caller's alpha overrides it).            */
/* ------------------------------------------------------------------------ */
int orc_phase_hlc(const orc_problem *P, const double *logc, const orc_config *C, orc_state *S)
{
    int N = C->N, d = P->d, M = C->M;
    S->n_unfrozen = unfrozen_count(C, S);
    S->sigma = choose_sigma(P, C, S);
    S->alpha_c = 0.0;
    if (!((C->phase_mask >> 5) & 1) || S->n_unfrozen == 0) return ORC_OK;
    uint32_t k = (uint32_t)S->k + 1;
    double sigma = S->sigma;
    double *Gh = (double *)malloc(sizeof(double) * (size_t)N * d);
    double *gn = (double *)malloc(sizeof(double) * N);
    if (!Gh || !gn) { free(Gh); free(gn); return ORC_ENOMEM; }
    for (int step = 0; step < C->n_cloud; ++step) {
#pragma omp parallel
        {
            scratch_t sc;
            scratch_alloc(&sc, P, C);
            double *z = (double *)malloc(sizeof(double) * d);
#pragma omp for schedule(dynamic, 2)
            for (int i = 0; i < N; ++i) {
                if (!(S->active[i] && !S->stuck[i])) continue;
                double *gh = Gh + (size_t)i * d;
                const double *x = S->X + (size_t)i * d;
                for (int l = 0; l < d; ++l) gh[l] = 0.0;
                for (int mm = 0; mm < M; ++mm) {
                    int pair = mm / 2;
                    double sgn = (mm % 2) ? -1.0 : 1.0;
                    normal_vec(C, (uint32_t)i, k, ((uint32_t)PH_HLC << 24) | ((uint32_t)step << 16) | (uint32_t)pair,
                               d, z);
                    for (int l = 0; l < d; ++l) sc.xtr[l] = x[l] + sigma * sgn * z[l];
                    const noise_t nzp = noise_for(P, C, S, i, step, NZ_FD_PROBE | ((uint32_t)mm << 7));
                    method_grad(P, logc, C, sc.xtr, sc.gtr, &sc, &nzp);
                    for (int l = 0; l < d; ++l) gh[l] += sc.gtr[l];
                }
                for (int l = 0; l < d; ++l) gh[l] /= M;
                gn[i] = nrm2(d, gh);
            }
            free(z);
            scratch_free(&sc);
        }
        if (step == 0) {
            if (C->alpha > 0.0) {
                S->alpha_c = C->alpha;
            } else {
                double s = 0.0;
                int n = 0;
                for (int i = 0; i < N; ++i)
                    if (S->active[i] && !S->stuck[i]) { s += gn[i]; n++; }
                double mean = s / n;
                S->alpha_c = mean > 0.0 ? sigma / mean : 0.0;
            }
        }
        for (int i = 0; i < N; ++i) {
            if (!(S->active[i] && !S->stuck[i])) continue;
            double *x = S->X + (size_t)i * d;
            for (int l = 0; l < d; ++l) x[l] += S->alpha_c * Gh[(size_t)i * d + l];
            clamp_box(P, x);
        }
    }
    free(Gh);
    free(gn);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Phase 6: anti-convergence.  v <- 0, then n_anti momentum descent steps    */
/* v <- mu v - alpha grad f(x), x <- clamp(x + v).  alpha is fixed at the    */
/* first step to sigma / mean |grad f| over the unfrozen samples unless the  */
/* caller supplies it.                                                       */
/* ------------------------------------------------------------------------ */
int orc_phase_anti(const orc_problem *P, const double *logc, const orc_config *C, orc_state *S)
{
    int N = C->N, d = P->d;
    S->alpha_a = 0.0;
    if (!((C->phase_mask >> 6) & 1)) return ORC_OK;
    int nu = unfrozen_count(C, S);
    if (nu == 0) return ORC_OK;
    double *Gt = (double *)malloc(sizeof(double) * (size_t)N * d);
    double *gn = (double *)malloc(sizeof(double) * N);
    if (!Gt || !gn) { free(Gt); free(gn); return ORC_ENOMEM; }
    for (int i = 0; i < N; ++i)
        if (S->active[i] && !S->stuck[i])
            for (int l = 0; l < d; ++l) S->V[(size_t)i * d + l] = 0.0;
    for (int step = 0; step < C->n_anti; ++step) {
#pragma omp parallel
        {
            scratch_t sc;
            scratch_alloc(&sc, P, C);
#pragma omp for schedule(dynamic, 2)
            for (int i = 0; i < N; ++i) {
                if (!(S->active[i] && !S->stuck[i])) continue;
                const noise_t nza = noise_for(P, C, S, i, step, NZ_FD_ANTI);
                method_grad(P, logc, C, S->X + (size_t)i * d, Gt + (size_t)i * d, &sc, &nza);
                gn[i] = nrm2(d, Gt + (size_t)i * d);
            }
            scratch_free(&sc);
        }
        if (step == 0) {
            if (C->alpha > 0.0) {
                S->alpha_a = C->alpha;
            } else {
                double s = 0.0;
                for (int i = 0; i < N; ++i)
                    if (S->active[i] && !S->stuck[i]) s += gn[i];
                double mean = s / nu;
                S->alpha_a = mean > 0.0 ? S->sigma / mean : 0.0;
            }
        }
        for (int i = 0; i < N; ++i) {
            if (!(S->active[i] && !S->stuck[i])) continue;
            double *x = S->X + (size_t)i * d, *v = S->V + (size_t)i * d;
            const double *g = Gt + (size_t)i * d;
            for (int l = 0; l < d; ++l) {
                v[l] = C->momentum * v[l] - S->alpha_a * g[l];
                x[l] += v[l];
            }
            clamp_box(P, x);
        }
    }
    free(Gt);
    free(gn);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* One oscillation cycle (Algorithm 1 body): phases 1-3 every cycle, phases  */
/* 4-6 only when this is not the last cycle.                                 */
/* ------------------------------------------------------------------------ */
int orc_cycle(const orc_problem *P, const double *logc, const orc_config *C, orc_state *S, orc_replay *R)
{
    if (S->k >= C->n_osc) return ORC_ESTATE;
    int last = (S->k + 1 == C->n_osc);
    int rc;
    S->K_lost = 0; S->reseed_kind = 0; S->sigma = 0.0; S->alpha_c = 0.0; S->alpha_a = 0.0;
    S->n_free = 0; S->n_unfrozen = 0;
    if ((rc = orc_phase_converge(P, logc, C, S, R))) return rc;
    if ((rc = orc_phase_stick(P, logc, C, S, R))) return rc;
    if ((rc = orc_phase_dedup(P, C, S, R))) return rc;
    if (!last) {
        if ((rc = orc_phase_reseed(P, C, S))) return rc;
        if ((rc = orc_phase_hlc(P, logc, C, S))) return rc;
        if ((rc = orc_phase_anti(P, logc, C, S))) return rc;
    }
    S->k += 1;
    return ORC_OK;
}

/* Initial population, uniform in the box from the INIT stream. */
/* Starting population (INIT stream, counter = sample index).  Uniform in the
 * box, or, with flag bit 2, the structured ray seeding the paper names for
 * its carry_tiger runs (Sec. 5.3), which it describes only as rays from the
 * domain's vertices, edges and faces.  Reading: sample i picks an anchor on
 * the boundary -- a vertex, an edge midpoint or a face centre, each with
 * probability 1/3 -- and lies uniformly on the segment from that anchor
 * through the box centre to the opposite anchor.  Draws: counter
 * (i, 0, 0 << 24 | 1, 0) gives the kind (integer below 3), the edge's free or
 * the face's fixed coordinate e (integer below d) and the position t
 * (uniform); counter (i, 0, 0 << 24 | 1, 1) gives one bit per coordinate
 * choosing its bound (hi for 1), from the first word for coordinates 0..31
 * and the second for 32..63. */
static void ray_seed_point(const orc_problem *P, const orc_config *C, int i, double *x)
{
    int d = P->d;
    uint32_t a[4], b[4];
    draw4(C, (uint32_t)i, 0, ((uint32_t)PH_INIT << 24) | 1u, 0, a);
    draw4(C, (uint32_t)i, 0, ((uint32_t)PH_INIT << 24) | 1u, 1, b);
    uint32_t kind = uint_below(a[0], 3);
    int e = (int)uint_below(a[1], (uint32_t)d);
    double t = orc_u01(a[2]);
    for (int c = 0; c < d; ++c) {
        double lo = P->lo[c], hi = P->hi[c];
        /* the anchor's coordinate: at the middle or at a bound */
        int middle = (kind == 1 && c == e) || (kind == 2 && c != e);
        int up = (int)(((c < 32 ? b[0] : b[1]) >> (c & 31)) & 1u);
        double anchor = middle ? 0.5 * (lo + hi) : (up ? hi : lo);
        double centre = 0.5 * (lo + hi);
        /* t along anchor -> opposite anchor (2 centre - anchor) */
        x[c] = anchor + t * (2.0 * centre - 2.0 * anchor);
    }
}

void orc_init_population(const orc_problem *P, const orc_config *C, double *X)
{
    int d = P->d;
    if (C->flags & 4u) {
        for (int i = 0; i < C->N; ++i) ray_seed_point(P, C, i, X + (size_t)i * d);
        return;
    }
    for (int i = 0; i < C->N; ++i) {
        for (int blk = 0; 4 * blk < d; ++blk) {
            uint32_t o[4];
            draw4(C, (uint32_t)i, 0, (uint32_t)PH_INIT << 24, (uint32_t)blk, o);
            for (int q = 0; q < 4 && 4 * blk + q < d; ++q) {
                int l = 4 * blk + q;
                X[(size_t)i * d + l] = P->lo[l] + orc_u01(o[q]) * (P->hi[l] - P->lo[l]);
            }
        }
    }
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count of the parallel per-sample loops (results do not depend on
 * it); n < 1 leaves it unchanged.  Returns the count now in effect. */
int orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
