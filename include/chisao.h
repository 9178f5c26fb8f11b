/*
 * chisao.h -- C ABI of libchisao, the MI355X (gfx950) implementation of the
 * ChiSao per-cycle population update (Wolfson, "ChiSao: A GPU-Native Parallel
 * Optimizer for Multimodal Black-Box Functions via Convergence-Anticonvergence
 * Oscillation").
 *
 * The library finds the significant modes of a mixture log-density
 * f : Theta -> R on a box Theta (Sec. 3.1, eq. 1): a population of N samples
 * goes through n_osc oscillation cycles of six phases (Sec. 3.2, Algorithm 1):
 * batched L-BFGS ascent, the stick test, L-infinity deduplication, Repulse
 * Monkey / Golden Rooster reseeding, Hands Like Clouds smoothed ascent and
 * momentum anti-convergence.  Every phase runs in HIP kernels on one GPU.
 *
 * Conventions for every entry point:
 *  - Return value: CHISAO_OK (0) or a negative CHISAO_E_* code; the message of
 *    the most recent failure on the calling thread is chisao_last_error().
 *  - "host" pointers are read (or written) before the call returns; "device"
 *    pointers must be device memory of the GPU that was current when the handle
 *    was created (for example a torch tensor's data_ptr()).
 *  - Arrays are dense, row-major, float32 unless stated; a sample's d
 *    coordinates are contiguous.
 *  - No partial results are written when a call fails.
 *  - A handle must not be used from two threads at once; distinct handles are
 *    independent.
 */
#ifndef CHISAO_H
#define CHISAO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CHISAO_OK 0
#define CHISAO_E_INVAL (-1)  /* bad sizes, d > 64, N < 1, lo >= hi, non-finite or non-SPD parameters */
#define CHISAO_E_NOMEM (-2)  /* device allocation failed */
#define CHISAO_E_DEVICE (-3) /* a HIP call failed; see chisao_last_error() */
#define CHISAO_E_STATE (-4)  /* cycle requested past n_osc, or call not valid in this state */
#define CHISAO_E_RANGE (-5)  /* output capacity too small; the required size is reported */

#define CHISAO_GAUSS 0     /* Gaussian mixture log-density (Appendix D, with full precision matrices) */
#define CHISAO_STUDENT_T 1 /* multivariate Student-t mixture log-density */
/* Closed-form test functions of Appendix D, each negated so that its optimum
 * is a maximum (constants as stated there: Rastrigin A = 10; Ackley a = 20,
 * b = 0.2, c = 2 pi; Michalewicz m = 10).  Coordinate i of the paper is x[i-1]. */
#define CHISAO_RASTRIGIN 2       /* -[10 d + sum (x_i^2 - 10 cos(2 pi x_i))] */
#define CHISAO_ACKLEY 3          /* 20 exp(-0.2 sqrt(mean x_i^2)) + exp(mean cos(2 pi x_i)) - 20 - e */
#define CHISAO_SCHWEFEL 4        /* -[418.9829 d - sum x_i sin(sqrt|x_i|)] */
#define CHISAO_STYBLINSKI_TANG 5 /* -1/2 sum (x_i^4 - 16 x_i^2 + 5 x_i) */
#define CHISAO_MICHALEWICZ 6     /* sum sin(x_i) sin^20(i x_i^2 / pi) */
#define CHISAO_TRID 7            /* -[sum (x_i - 1)^2 - sum_{i>=2} x_i x_{i-1}] */
#define CHISAO_BUKIN6 8          /* -[100 sqrt|x_2 - 0.01 x_1^2| + 0.01 |x_1 + 10|], d = 2 */

#define CHISAO_GRAD_FD 0      /* central finite differences, 2d evaluations per gradient (Sec. 3.1, Sec. 5) */
#define CHISAO_GRAD_ADJOINT 1 /* analytic gradient fused with the value (reverse mode for the mixtures) */

/* Objective on the box [lo, hi]: a mixture f(x) = log sum_k w_k p_k(x), with
 * p_k N(mu_k, prec_k^-1) (Gaussian) or the Student-t density with nu degrees
 * of freedom and scale matrix prec_k^-1; or one of the closed-form test
 * functions, for which K, nu, log_w, mu and prec are ignored (the arrays may
 * be NULL) and the box is the caller's (Appendix D gives each function's).
 * All arrays are host memory, copied by chisao_init.
 *
 * Form of the mixture parameters.  A component is given by its precision
 * matrix P_k = Sigma_k^-1 and its log weight, not by a whitening factor W_k
 * (P_k = W_k^T W_k) and a precomputed log normaliser: with u = P_k (x - mu_k)
 * one matrix product per component yields both the quadratic form
 * (x - mu_k) . u of the value and the direction -u of the analytic gradient,
 * where W_k would need a second product W_k^T (W_k (x - mu_k)) for the
 * gradient.  The library derives each normaliser itself (an FP64 Cholesky
 * factorisation of P_k at init), so the caller cannot pass one that is
 * inconsistent with P_k.  A caller holding W_k forms W_k^T W_k. */
typedef struct {
    int32_t family;      /* CHISAO_GAUSS, CHISAO_STUDENT_T or a closed form CHISAO_RASTRIGIN..CHISAO_BUKIN6 */
    int32_t d;           /* dimension, 1..64 (2 for CHISAO_BUKIN6) */
    int32_t K;           /* number of components, 1..65536 (mixtures only) */
    float nu;            /* Student-t degrees of freedom (> 0), ignored for Gaussians */
    const float *log_w;  /* [K] log mixture weights */
    const float *mu;     /* [K*d] component centres */
    const float *prec;   /* [K*d*d] exactly symmetric positive-definite precision (inverse covariance / inverse scale) */
    const float *lo;     /* [d] lower box bounds */
    const float *hi;     /* [d] upper box bounds, hi > lo */
    float noise_sigma;   /* >= 0: every value the method evaluates is f(x) + noise_sigma * z, z ~ N(0,1)
                            drawn per evaluation (Sec. 5.7); gradients of the adjoint mode stay exact.
                            chisao_eval returns the noise-free f. */
} chisao_problem;

/* Schedule and hyperparameters (Sec. 3.6, Table 1).  A value <= 0 in a field
 * marked "auto" selects the rule named next to it. */
typedef struct {
    int32_t N;          /* population size, 1..2^30 */
    int32_t m;          /* L-BFGS memory, 1..32 */
    int32_t n_osc;      /* oscillation cycles */
    int32_t n_conv;     /* L-BFGS iterations per cycle, at most 255; auto: max(10, ceil(3 log2 d)) */
    int32_t n_anti;     /* anti-convergence steps, 0..255 */
    int32_t n_cloud;    /* Hands Like Clouds steps, 0..255 (a step index has 8 bits of the random-stream
                           counter, so longer phases would reuse draws) */
    int32_t M;          /* probes per smoothed gradient, 1..32 */
    float eps_grad;     /* stick threshold on the gradient sup-norm */
    float eps_dup;      /* L-infinity deduplication radius */
    float log_delta;    /* log of the quality threshold delta (log 0.1 by default) */
    float momentum;     /* anti-convergence momentum mu */
    float alpha;        /* step length of both exploration phases; auto: sigma / mean |grad| */
    float sigma;        /* smoothing scale; auto: sigma_c * pooled std of unfrozen samples */
    float sigma_c;      /* the constant c of the sigma rule */
    int32_t grad_mode;  /* CHISAO_GRAD_FD or CHISAO_GRAD_ADJOINT */
    float fd_h;         /* finite-difference step; auto: h_j = 2^-8 max(1, |x_j|) */
    float ls_c1;        /* Armijo constant of the backtracking line search */
    int32_t ls_max;     /* backtracking trials t = 1, 1/2, ..., 2^-(ls_max-1); 1..15 (the decision trace
                           stores the accepted index in 4 bits, 15 meaning a failed search) */
    float curv_eps;     /* a pair is stored when s'y > curv_eps |s| |y| */
    int32_t gate_reps;  /* noisy problems: the quality gate compares the mean of this many fresh noisy
                           evaluations per sample (0: M); 0..4096 */
    uint32_t phase_mask;/* bit p enables phase p for p = 3..6 (ablation hook); 0x7E = all */
    uint64_t seed;      /* key of every random stream */
    uint32_t problem_id;/* mixed into the key, so problems draw independent streams */
    uint32_t flags;     /* CHISAO_FLAG_* (handle-wide; taken from the first problem of a batch) */
} chisao_config;

#define CHISAO_FLAG_NO_GRAPH 1u    /* enqueue every cycle's kernels one by one instead of replaying a captured hipGraph */
#define CHISAO_FLAG_NO_AUTOTUNE 2u /* keep the default evaluation schedule (linear tile order, 8192 workgroups,
                                      line-search launches included) */
/* Read per problem: when the problem's starting population is not given, draw
 * it on rays through the centre of the box from its vertices, edge midpoints
 * and face centres (the structured ray seeding of Sec. 5.3) instead of
 * uniformly.  Sample i takes, from Philox counter (i, 0, 0 << 24 | 1, b):
 * block 0 gives the anchor kind (vertex, edge midpoint, face centre; integer
 * below 3 of the first word), the coordinate e that is free (edge) or fixed
 * (face) (integer below d of the second word) and the ray position t (uniform
 * of the third word); block 1 gives one bit per coordinate (bit c of the
 * first word, c < 32, of the second word, c >= 32) choosing the bound hi (1)
 * or lo (0).  The anchor has every coordinate at its chosen bound (vertex),
 * all but e (edge midpoint, e at the middle), or only e (face centre, the
 * others at the middle); the sample lies at t along the segment from the
 * anchor through the centre to the opposite anchor: a bound coordinate is
 * lo + t (hi - lo) or hi - t (hi - lo), a middle one lo + (hi - lo) / 2. */
#define CHISAO_FLAG_RAY_SEEDING 4u
/* Direct evaluations of matrix-core classes in 16-point tiles whatever the
 * autotuner measures (its other tile size; results are the same). */
#define CHISAO_FLAG_HALF_TILES 8u

/* Per-cycle statistics (host struct). */
typedef struct {
    int32_t k;          /* 1-based index of the cycle these figures belong to */
    float f_max;        /* largest value over active samples after Phase 1; with noise, the sample with the largest
                           gate value is re-estimated with gate_reps fresh draws and that estimate is f_max */
    int32_t n_stuck;    /* samples passing the stick test (before deduplication) */
    int32_t K_lost;     /* duplicates removed by Phase 3 */
    int32_t n_modes;    /* stuck samples surviving deduplication */
    int32_t reseed_kind;/* 0 none, 1 Repulse Monkey, 2 Golden Rooster, 3 slots deactivated */
    int32_t n_free;     /* unfrozen samples available as Repulse Monkey origins */
    int32_t n_unfrozen; /* samples moved by Phases 5-6 */
    int32_t n_active;   /* samples still in use */
    float sigma;        /* smoothing scale used in Phase 5 */
    float alpha_c;      /* Hands Like Clouds step length */
    float alpha_a;      /* anti-convergence step length */
    int32_t ls_fail;    /* line searches that failed during Phase 1 */
    int32_t n_nonfinite;/* samples taken out of use at Phase 2 because their value, gate value or gradient
                           was not finite (they join no reduction, are never stuck and are not reseeded) */
    int64_t evals;      /* objective evaluations (points) during the cycle */
} chisao_cycle_stats;

/* Host view of the population state for chisao_get_state / chisao_set_state.
 * Each pointer may be NULL to skip that array. */
typedef struct {
    float *X;           /* [N*d] positions */
    float *F;           /* [N] values after Phase 1 (get only) */
    float *G;           /* [N*d] gradients after Phase 1 (get only) */
    uint8_t *stuck;     /* [N] stuck flags (after deduplication) */
    uint8_t *active;    /* [N] slot-in-use flags */
    uint8_t *stuck_pre; /* [N] stick decisions before deduplication (get only) */
    uint8_t *removed;   /* [N] deduplication decisions (get only) */
    uint8_t *trace;     /* [(n_conv+1)*N] per-iteration L-BFGS decision codes of the last Phase 1 (get only):
                           0xFF not iterated; bits 0-3 accepted backtracking index (15 = failed);
                           bit 4 pair stored; bit 5 converged; bit 6 direction reset */
    int32_t k;          /* cycles completed */
    int32_t gr_disabled, gr_fail, gr_used_last, gr_prev_modes; /* Golden Rooster generation state */
    /* L-BFGS history of the last Phase 1 (get only): pairs (s, y) for F = -f
       in a ring of m slots per sample, newest in slot head, cnt pairs valid */
    float *S;           /* [N*m*d] */
    float *Y;           /* [N*m*d] */
    float *rho;         /* [N*m] 1 / s'y */
    int32_t *head;      /* [N] */
    int32_t *cnt;       /* [N] */
    uint8_t *conv;      /* [N] last Phase 1: 1 converged, 2 stalled (a search from an empty history failed,
                           so every later iteration would repeat it; never with noise), 0 otherwise */
    float *Fg;          /* [N] quality-gate values of a noisy problem after Phase 1 (get only) */
    float *Wd;          /* [N*d] preserved inverse-Hessian diagonals (width export; see chisao_mode_widths) */
    uint8_t *wvalid;    /* [N] 1 where Wd holds a value */
} chisao_state;

/* Kernel timing of the work enqueued by chisao_cycle / chisao_run_phases
 * while profiling is on: HIP events recorded around each launch on the
 * handle's stream, and the number of objective evaluations (points) each
 * evaluation launch processed, counted on the device. */
#define CHISAO_PROF_EVAL_DIRECT 0 /* value and adjoint gradient at the samples */
#define CHISAO_PROF_EVAL_TRIAL 1  /* line-search trial points */
#define CHISAO_PROF_EVAL_PROBE 2  /* Hands Like Clouds smoothing probes */
#define CHISAO_PROF_EVAL_FD 3     /* central-difference stencil points */
#define CHISAO_PROF_LBFGS 4       /* two-loop directions and curvature pairs; points = samples given a direction */
#define CHISAO_PROF_LBFGS_PAIRS 5 /* points only: history pairs those two-loops read (no launches of its own) */
#define CHISAO_PROF_CLASSES 8
typedef struct {
    int32_t launches;
    double ms;       /* summed kernel time */
    int64_t points;  /* evaluations processed (evaluation classes) or samples visited (L-BFGS) */
} chisao_kernel_profile;

typedef struct chisao_ctx *chisao_handle;

/* Create an optimizer for one problem (Sec. 3.1: f, the population, the
 * schedule).  x0_dev: device [N*d] starting population inside the box, or NULL
 * for a uniform draw in the box.  hip_stream: the hipStream_t all work is
 * enqueued on (NULL = default stream).  Allocates the library-owned device
 * workspace, copies every input, and synchronizes before returning. */
int chisao_init(chisao_handle *out, const chisao_problem *p, const chisao_config *c, const float *x0_dev,
                void *hip_stream);

/* Several independent problems in one handle (one per entry of ps/cs, up to
 * 256, uneven d, K and N allowed, equal n_osc): every kernel of a cycle covers
 * all problems, and each problem computes exactly what it would compute in a
 * handle of its own.  Problems are grouped into launch classes (see
 * chisao_tuning); with several classes, each class after the first runs its
 * evaluation and L-BFGS launches on a library-owned stream forked from
 * hip_stream by an event and joined back to it, so the classes run side by
 * side and everything stays ordered on hip_stream as seen by the caller.
 * x0_dev: array of n_problems device pointers (entries may be NULL), or NULL
 * for uniform draws.  Problem indices below refer to the order of ps. */
int chisao_init_batched(chisao_handle *out, int n_problems, const chisao_problem *ps, const chisao_config *cs,
                        const float *const *x0_dev, void *hip_stream);

/* Run n_cycles oscillation cycles (Algorithm 1 body) of every problem.
 * Phases 4-6 are skipped in cycle n_osc.  Work is enqueued asynchronously (by
 * default as one captured hipGraph per cycle); when stats_host is not NULL the
 * call synchronizes and fills n_cycles * n_problems entries, cycle-major.
 * Running past n_osc fails with CHISAO_E_STATE and runs nothing. */
int chisao_cycle(chisao_handle h, int n_cycles, chisao_cycle_stats *stats_host);

/* The estimated mode set {x_i : stuck_i} (Algorithm 1 return value):
 * synchronizes, then writes the stuck active samples in ascending index to
 * x_out (host [cap*d]) and f_out (host [cap], may be NULL).  *n_out receives
 * the count; if cap is smaller, nothing is written and CHISAO_E_RANGE is
 * returned.  problem: index within the handle. */
int chisao_modes(chisao_handle h, int problem, float *x_out, float *f_out, int cap, int *n_out);

/* Widths of the modes (Sec. 3.2 Phase 3: the surviving sample's inverse
 * Hessian estimate is preserved for width estimation).  For each mode, in
 * the order of chisao_modes, the diagonal of the L-BFGS inverse-Hessian
 * approximation H of -f built from the pairs of the Phase 1 in which the
 * sample converged: H = gamma I updated by every stored pair from oldest to
 * newest, gamma = s'y / y'y of the newest pair (1 / max(|grad f|_2, 1) for a
 * sample that stuck without any pair).  For a peak of a Gaussian mixture
 * these approximate the component variances along the coordinates.
 * Synchronizes; writes w_out (host [cap*d]); *n_out receives the mode count;
 * if cap is smaller, nothing is written and CHISAO_E_RANGE is returned. */
int chisao_mode_widths(chisao_handle h, int problem, float *w_out, int cap, int *n_out);

/* Copy the state to / from host memory (synchronizes).  set_state writes X,
 * stuck, active, k, the Golden Rooster state and the preserved widths; F, G,
 * the histories and the decision arrays are recomputed by the next cycle.
 * Every coordinate of X must lie in the box or be NaN; a NaN row stands for a
 * sample whose objective cannot be evaluated, and like any sample whose
 * value or gradient is not finite after Phase 1 it is taken out of use at
 * Phase 2 (counted in chisao_cycle_stats.n_nonfinite).
 * Between cycles this is the whole state a run carries forward: a handle
 * given it continues exactly as the handle it was read from. */
int chisao_get_state(chisao_handle h, int problem, chisao_state *s);
int chisao_set_state(chisao_handle h, int problem, const chisao_state *s);

/* Run a subset of the phases of cycle k+1 of every problem on the current
 * state without advancing k (test hook for per-phase parity).  phase_mask bit
 * p selects phase p (1..6); phases run in ascending order.  Synchronizes. */
int chisao_run_phases(chisao_handle h, uint32_t phase_mask);

/* Batched objective on caller memory (Sec. 3.1 objective, with the gradient
 * the method would use): X_dev device [B*d]; f_dev device [B] (may be NULL);
 * G_dev device [B*d] (may be NULL).  grad_mode selects the adjoint kernel or
 * central differences (fd_h of the handle's config).  Enqueued on the
 * handle's stream; does not synchronize. */
int chisao_eval(chisao_handle h, int problem, const float *X_dev, int B, float *f_dev, float *G_dev,
                int grad_mode);

/* For callers that cannot allocate device memory (serving loops and
 * harnesses that forbid hipMalloc): chisao_eval without a handle.  The
 * problem p (host arrays, as for chisao_init) and the finite-difference step
 * fd_h (<= 0: h_j = 2^-8 max(1, |x_j|), as in chisao_config) replace the
 * handle; X_dev, f_dev, G_dev and grad_mode are as for chisao_eval, and the
 * results are bitwise those of chisao_eval on a handle created for p with
 * that fd_h.  Nothing is allocated: the problem's tables (precision-matrix
 * fragments, centres, log normalisers, descriptors) are built in a static
 * device array of 8 MiB that each GPU holds from library load to process
 * exit.  The tables take 4 (K (DP^2 + d^2 + DP + d + 2) + 2 d) bytes plus
 * about 1 KiB, DP = 8 for a mixture with d <= 8, else d rounded up to 16, 32
 * or 64: up to K = 251 components at d = 64; a larger problem fails with
 * CHISAO_E_RANGE and runs nothing.
 * Enqueued on hip_stream (NULL = default stream) of the current device.  The
 * call synchronizes that stream once, after uploading the problem (a matrix
 * that is not positive definite fails with CHISAO_E_INVAL), and returns with
 * the evaluation kernels enqueued.  Every call on a GPU reuses that GPU's
 * array: calls on one stream are ordered and safe, but calls whose work
 * overlaps on one GPU (other threads, other streams) race on the tables and
 * must be serialized by the caller. */
int chisao_eval_static(const chisao_problem *p, float fd_h, const float *X_dev, int B, float *f_dev, float *G_dev,
                       int grad_mode, void *hip_stream);

/* enable = 1: clear the counters and start recording; enable = 0: stop,
 * synchronize and write CHISAO_PROF_CLASSES entries to out (may be NULL). */
int chisao_profile(chisao_handle h, int enable, chisao_kernel_profile *out);

void chisao_destroy(chisao_handle h);

/* Message of the last failure on this thread ("" if none); valid until the
 * next library call on the same thread. */
const char *chisao_last_error(void);

/* Evaluation launch schedules chosen at init.  Problems are grouped into
 * classes by (padded d, family, gradient mode); for each class the autotuner
 * times CHISAO_TUNE_VARIANTS schedules over the starting population, on a
 * value + adjoint gradient pass (adjoint classes) or a central-difference
 * stencil pass (finite-difference classes): each variant once untimed, then
 * two rounds over the variants, a variant's time its fastest launch.  It
 * keeps the default (variant 0) unless another is at least 3% faster than the
 * best so far: variant v uses
 * tile order v % 2 (0 linear, 1 XCD-chunked) and a grid of 8192 (v < 2) or
 * 1024 workgroups.  Then, for an adjoint mixture class on the matrix cores,
 * it times the value + gradient pass in tiles of 16 and of 32 points under
 * the chosen schedule and keeps 16 for direct evaluations if at least 3%
 * faster.  Last, an adjoint class times the same variants on a smoothing-probe
 * pass (M probes per sample) and picks the probe launches' schedule by the
 * same rule; finite-difference classes use one schedule for all launches.
 * Line-search launches of matrix-core mixture classes take the chosen tile
 * order with a grid of exactly the workgroups the GPU holds at once (the
 * trial kernel's occupancy times the CU count), each workgroup looping over
 * tiles; this is a rule, not a timed choice.  Schedules and tile size change
 * timing only, never results. */
#define CHISAO_TUNE_VARIANTS 4
typedef struct {
    int32_t padded_d;    /* 8 (mixtures with d <= 8, evaluated one point per lane), 16, 32 or 64 */
    int32_t family;
    int32_t grad_mode;
    int32_t n_problems;  /* problems in the class */
    int32_t order;       /* chosen tile order */
    int32_t grid_cap;    /* chosen grid size */
    float ms[CHISAO_TUNE_VARIANTS]; /* measured time per variant (0 when not tuned) */
    int32_t tile_points;            /* points per tile of direct evaluations: 32 or 16 (64 at width 8) */
    float ms_half_tiles;            /* measured time of the pass in 16-point tiles (0 when not tried) */
    float ms_full_tiles;            /* ... and in 32-point tiles, timed alongside (0 when not tried) */
    int32_t probe_order;            /* schedule of the smoothing-probe launches: tile order */
    int32_t probe_grid_cap;         /* ... and grid size */
    float ms_probe[CHISAO_TUNE_VARIANTS]; /* measured probe-pass time per variant (0 when not tuned) */
    int32_t trial_grid_cap;         /* grid of the line-search launches (0: the chosen grid_cap; always 0 with
                                       CHISAO_FLAG_NO_AUTOTUNE) */
} chisao_tuning_entry;

/* Writes one entry per class (at most cap) and the class count to *n_out;
 * cap too small: CHISAO_E_RANGE with *n_out set.  Host memory. */
int chisao_tuning(chisao_handle h, chisao_tuning_entry *out, int cap, int *n_out);

/* Measured ceilings of the GPU the call runs on, against which kernel
 * throughput is priced beside the published figures (FP32 matrix 157.3
 * TFLOP/s, HBM 8 TB/s on MI355X).  fp32_mfma_tflops: a full grid of waves each
 * issuing a long run of v_mfma_f32_16x16x4f32 on independent accumulators;
 * hbm_copy_gbs: a streaming copy between two device buffers of copy_bytes each
 * (read + write bytes over time; 1 MiB .. 32 GiB, a few GiB keeps the caches
 * out of it).  Best of several timed repetitions with HIP events on
 * hip_stream.  Allocates and frees the two copy buffers; synchronizes. */
typedef struct {
    double fp32_mfma_tflops;
    double mfma_flops;  /* flops of one timed matrix launch */
    double mfma_ms;
    double hbm_copy_gbs;
    double copy_bytes;  /* bytes read plus bytes written by one timed copy */
    double copy_ms;
} chisao_peaks;
int chisao_measure_peaks(chisao_peaks *out, size_t copy_bytes, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* CHISAO_H */
