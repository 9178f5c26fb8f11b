// Host side of libchisao: the C ABI declared in include/chisao.h.
//
// A handle owns the device workspace of one population.  A cycle is a fixed
// sequence of kernel launches on the handle's stream; every data-dependent
// choice inside it (which samples move, line-search outcomes, Repulse Monkey
// or Golden Rooster, step lengths) is read by the kernels from device
// memory, so the host never waits inside a cycle.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "../../include/chisao.h"
#include "kernels.h"

using namespace chisao;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                                   \
    do {                                                                                                \
        hipError_t e_ = (expr);                                                                         \
        if (e_ != hipSuccess) return fail(CHISAO_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

struct Buffers {
    std::vector<void *> owned;
    hipError_t alloc(void **p, size_t bytes) {
        *p = nullptr;
        if (bytes == 0) bytes = 16;
        hipError_t e = hipMalloc(p, bytes);
        if (e == hipSuccess) owned.push_back(*p);
        return e;
    }
    void release() {
        for (void *p : owned) (void)hipFree(p);
        owned.clear();
    }
};

}  // namespace

struct chisao_ctx {
    Dev D{};
    hipStream_t stream = nullptr;
    int device = 0;
    int k_host = 0;  // cycles completed (mirrors ctl->k)
    Buffers buf;
    // profiling: event pairs recorded around launches of each class
    bool prof = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, size_t>> ev_used;  // (class, index of the start event)
    ~chisao_ctx() {
        for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
        buf.release();
    }
};

// Run a launch; when profiling, bracket it with events on the handle's stream.
template <class F>
static hipError_t timed(chisao_ctx *h, int cls, F &&launch) {
    if (!h->prof) return launch();
    const size_t i = h->ev_used.size() * 2;
    while (h->ev_pool.size() < i + 2) {
        hipEvent_t e;
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) return r;
        h->ev_pool.push_back(e);
    }
    hipError_t r = hipEventRecord(h->ev_pool[i], h->stream);
    if (r != hipSuccess) return r;
    r = launch();
    if (r != hipSuccess) return r;
    r = hipEventRecord(h->ev_pool[i + 1], h->stream);
    if (r != hipSuccess) return r;
    h->ev_used.push_back({cls, i});
    return hipSuccess;
}

static int pad_dim(int d) { return d <= 16 ? 16 : (d <= 32 ? 32 : 64); }

static int validate(const chisao_problem *p, const chisao_config *c) {
    if (!p || !c) return fail(CHISAO_E_INVAL, "null problem or config");
    if (p->family != CHISAO_GAUSS && p->family != CHISAO_STUDENT_T) return fail(CHISAO_E_INVAL, "unknown family");
    if (p->d < 1 || p->d > 64) return fail(CHISAO_E_INVAL, "d must be in 1..64 (got %d)", p->d);
    if (p->K < 1) return fail(CHISAO_E_INVAL, "K must be >= 1");
    if (!p->log_w || !p->mu || !p->prec || !p->lo || !p->hi) return fail(CHISAO_E_INVAL, "null problem array");
    if (p->family == CHISAO_STUDENT_T && !(p->nu > 0.0f && isfinite(p->nu)))
        return fail(CHISAO_E_INVAL, "Student-t needs nu > 0");
    if (p->noise_sigma != 0.0f) return fail(CHISAO_E_INVAL, "noisy objectives are not supported in this version");
    const int d = p->d, K = p->K;
    for (int j = 0; j < d; ++j)
        if (!(isfinite(p->lo[j]) && isfinite(p->hi[j]) && p->lo[j] < p->hi[j]))
            return fail(CHISAO_E_INVAL, "box bounds must be finite with lo < hi (coordinate %d)", j);
    for (int k = 0; k < K; ++k) {
        if (!isfinite(p->log_w[k])) return fail(CHISAO_E_INVAL, "non-finite log weight %d", k);
        for (int j = 0; j < d; ++j)
            if (!isfinite(p->mu[(size_t)k * d + j])) return fail(CHISAO_E_INVAL, "non-finite centre %d", k);
        const float *P = p->prec + (size_t)k * d * d;
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j) {
                if (!isfinite(P[i * d + j])) return fail(CHISAO_E_INVAL, "non-finite precision entry in %d", k);
                if (P[i * d + j] != P[j * d + i]) return fail(CHISAO_E_INVAL, "precision matrix %d not symmetric", k);
            }
    }
    if (c->N < 1) return fail(CHISAO_E_INVAL, "N must be >= 1");
    if ((long)c->N * d > (1L << 31) - 1) return fail(CHISAO_E_INVAL, "N*d too large");
    if (c->m < 1 || c->m > 32) return fail(CHISAO_E_INVAL, "m must be in 1..32");
    if (c->n_osc < 1) return fail(CHISAO_E_INVAL, "n_osc must be >= 1");
    if (c->n_anti < 0 || c->n_cloud < 0) return fail(CHISAO_E_INVAL, "negative step count");
    if (c->M < 1 || c->M > 32) return fail(CHISAO_E_INVAL, "M must be in 1..32");
    if (c->ls_max < 1 || c->ls_max > 16) return fail(CHISAO_E_INVAL, "ls_max must be in 1..16");
    if (c->grad_mode != CHISAO_GRAD_FD && c->grad_mode != CHISAO_GRAD_ADJOINT)
        return fail(CHISAO_E_INVAL, "unknown grad_mode");
    if (c->gate_reps != 0) return fail(CHISAO_E_INVAL, "gate_reps is reserved and must be 0");
    if (!(c->eps_grad > 0.0f) || !(c->eps_dup > 0.0f)) return fail(CHISAO_E_INVAL, "eps_grad and eps_dup must be > 0");
    if (!isfinite(c->log_delta) || !isfinite(c->momentum) || !isfinite(c->alpha) || !isfinite(c->sigma) ||
        !isfinite(c->sigma_c) || !isfinite(c->fd_h) || !isfinite(c->ls_c1) || !isfinite(c->curv_eps))
        return fail(CHISAO_E_INVAL, "non-finite hyperparameter");
    return CHISAO_OK;
}

extern "C" const char *chisao_last_error(void) { return g_err.c_str(); }

extern "C" int chisao_init(chisao_handle *out, const chisao_problem *p, const chisao_config *c, const float *x0_dev,
                           void *hip_stream) {
    if (!out) return fail(CHISAO_E_INVAL, "null output handle");
    *out = nullptr;
    int rc = validate(p, c);
    if (rc) return rc;
    chisao_ctx *h = new (std::nothrow) chisao_ctx();
    if (!h) return fail(CHISAO_E_NOMEM, "host allocation failed");
    h->stream = (hipStream_t)hip_stream;
    HIP_TRY(hipGetDevice(&h->device));
    Dev &D = h->D;
    D.d = p->d;
    D.DP = pad_dim(p->d);
    D.K = p->K;
    D.family = p->family;
    D.nu = p->family == CHISAO_STUDENT_T ? p->nu : 1.0f;
    D.nu_plus_d = D.nu + (float)p->d;
    D.N = c->N;
    D.m = c->m;
    D.n_osc = c->n_osc;
    D.n_conv = c->n_conv > 0 ? c->n_conv : std::max(10, (int)ceil(3.0 * log2((double)p->d) - 1e-9));
    D.n_anti = c->n_anti;
    D.n_cloud = c->n_cloud;
    D.M = c->M;
    D.ls_max = c->ls_max;
    D.grad_mode = c->grad_mode;
    D.eps_grad = c->eps_grad;
    D.eps_dup = c->eps_dup;
    D.log_delta = c->log_delta;
    D.momentum = c->momentum;
    D.alpha = c->alpha;
    D.sigma_cfg = c->sigma;
    D.sigma_c = c->sigma_c;
    D.fd_h = c->fd_h;
    D.ls_c1 = c->ls_c1;
    D.curv_eps = c->curv_eps;
    D.key0 = (uint32_t)(c->seed & 0xFFFFFFFFu);
    D.key1 = (uint32_t)(c->seed >> 32) ^ c->problem_id;
    D.phase_mask = c->phase_mask;
    D.n_part_blocks = 256;

    const size_t N = (size_t)c->N, d = (size_t)p->d, K = (size_t)p->K, DP = (size_t)D.DP, m = (size_t)c->m;
    Buffers &B = h->buf;
    auto A = [&](void **ptr, size_t bytes) -> int {
        hipError_t e = B.alloc(ptr, bytes);
        if (e != hipSuccess) return fail(CHISAO_E_NOMEM, "hipMalloc(%zu bytes): %s", bytes, hipGetErrorString(e));
        return CHISAO_OK;
    };
#define ALLOC(field, type, count)                                       \
    do {                                                                \
        void *tmp_;                                                     \
        if ((rc = A(&tmp_, sizeof(type) * (size_t)(count)))) goto fail_out; \
        field = (type *)tmp_;                                           \
    } while (0)
    {
        float *Pfrag, *muB, *muC, *logc2, *lo, *hi, *tmp_w, *tmp_mu, *tmp_prec;
        int *bad;
        ALLOC(Pfrag, float, K * DP * DP);
        ALLOC(muB, float, K * DP);
        ALLOC(muC, float, K * DP);
        ALLOC(logc2, float, K);
        ALLOC(lo, float, d);
        ALLOC(hi, float, d);
        ALLOC(tmp_w, float, K);
        ALLOC(tmp_mu, float, K * d);
        ALLOC(tmp_prec, float, K * d * d);
        ALLOC(bad, int, 1);
        D.Pfrag = Pfrag; D.muB = muB; D.muC = muC; D.logc2 = logc2; D.lo = lo; D.hi = hi;
        ALLOC(D.X, float, N * d);
        ALLOC(D.F, float, N);
        ALLOC(D.G, float, N * d);
        ALLOC(D.V, float, N * d);
        ALLOC(D.Xprev, float, N * d);
        ALLOC(D.Gprev, float, N * d);
        ALLOC(D.Pd, float, N * d);
        ALLOC(D.Gh, float, N * d);
        ALLOC(D.ginf, float, N);
        if (c->grad_mode == CHISAO_GRAD_FD) ALLOC(D.Gp, float, N * (size_t)c->M * d);
        ALLOC(D.stuck, uint8_t, N);
        ALLOC(D.active, uint8_t, N);
        ALLOC(D.conv, uint8_t, N);
        ALLOC(D.removed, uint8_t, N);
        ALLOC(D.stuck_pre, uint8_t, N);
        ALLOC(D.status, uint8_t, N);
        ALLOC(D.reset, uint8_t, N);
        ALLOC(D.steep, uint8_t, N);
        ALLOC(D.trace, uint8_t, N * (size_t)(D.n_conv + 1));
        ALLOC(D.S, float, N * m * d);
        ALLOC(D.Y, float, N * m * d);
        ALLOC(D.rho, float, N * m);
        ALLOC(D.head, int, N);
        ALLOC(D.cnt, int, N);
        ALLOC(D.lists, int, N * kNumLists);
        ALLOC(D.ctl, Ctl, 1);
        ALLOC(D.records, CycleRecord, (size_t)c->n_osc);
        ALLOC(D.part, double, (size_t)D.n_part_blocks * 129);

        hipStream_t st = h->stream;
        hipError_t e;
#define HIP_GO(expr)                                                                              \
    do {                                                                                          \
        if ((e = (expr)) != hipSuccess) {                                                         \
            rc = fail(CHISAO_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e));                    \
            goto fail_out;                                                                        \
        }                                                                                         \
    } while (0)
        HIP_GO(hipMemcpyAsync(lo, p->lo, sizeof(float) * d, hipMemcpyHostToDevice, st));
        HIP_GO(hipMemcpyAsync(hi, p->hi, sizeof(float) * d, hipMemcpyHostToDevice, st));
        HIP_GO(hipMemcpyAsync(tmp_w, p->log_w, sizeof(float) * K, hipMemcpyHostToDevice, st));
        HIP_GO(hipMemcpyAsync(tmp_mu, p->mu, sizeof(float) * K * d, hipMemcpyHostToDevice, st));
        HIP_GO(hipMemcpyAsync(tmp_prec, p->prec, sizeof(float) * K * d * d, hipMemcpyHostToDevice, st));
        HIP_GO(hipMemsetAsync(bad, 0, sizeof(int), st));
        HIP_GO(launch_prepare(D.family, D.d, D.DP, D.K, D.nu, tmp_w, tmp_mu, tmp_prec, logc2, Pfrag, muB, muC, bad, st));
        // population and control state
        if (x0_dev) HIP_GO(hipMemcpyAsync(D.X, x0_dev, sizeof(float) * N * d, hipMemcpyDeviceToDevice, st));
        else HIP_GO(launch_uniform_init(D, st));
        HIP_GO(launch_fill_u8(D.active, 1, N, st));
        HIP_GO(launch_fill_u8(D.stuck, 0, N, st));
        HIP_GO(hipMemsetAsync(D.V, 0, sizeof(float) * N * d, st));
        HIP_GO(hipMemsetAsync(D.ctl, 0, sizeof(Ctl), st));
        HIP_GO(hipMemsetAsync(D.records, 0, sizeof(CycleRecord) * c->n_osc, st));
        int bad_h = 0;
        HIP_GO(hipMemcpyAsync(&bad_h, bad, sizeof(int), hipMemcpyDeviceToHost, st));
        HIP_GO(hipStreamSynchronize(st));
        if (bad_h) {
            rc = fail(CHISAO_E_INVAL, "a precision matrix is not positive definite");
            goto fail_out;
        }
        if (x0_dev) {
            // the starting population must lie in the box
            std::vector<float> xh(N * d), loh(p->lo, p->lo + d), hih(p->hi, p->hi + d);
            HIP_GO(hipMemcpy(xh.data(), D.X, sizeof(float) * N * d, hipMemcpyDeviceToHost));
            for (size_t i = 0; i < N * d; ++i) {
                const size_t j = i % d;
                if (!(xh[i] >= loh[j] && xh[i] <= hih[j])) {
                    rc = fail(CHISAO_E_INVAL, "x0 sample %zu lies outside the box", i / d);
                    goto fail_out;
                }
            }
        }
    }
#undef ALLOC
#undef HIP_GO
    *out = h;
    return CHISAO_OK;
fail_out:
    delete h;
    return rc;
}

extern "C" void chisao_destroy(chisao_handle h) {
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    delete h;
}

// ---------------------------------------------------------------------------
// Phase sequences
// ---------------------------------------------------------------------------
static int eval_args_base(chisao_ctx *h, EvalArgs &a) {
    memset(&a, 0, sizeof a);
    a.D = h->D;
    a.X = h->D.X;
    a.Vc = 1;
    a.trial_next = -1;
    return 0;
}

static inline int *host_list(const Dev &D, int id) { return D.lists + (size_t)id * D.N; }

static hipError_t run_eval(chisao_ctx *h, const EvalArgs &a, int center, bool fd, bool grad) {
    const int cls = fd ? CHISAO_PROF_EVAL_FD : center;
    return timed(h, cls, [&] { return launch_eval(a, center, fd, grad, h->stream); });
}

static hipError_t eval_list(chisao_ctx *h, int list_id, float *F_out, float *G_out, bool want_f) {
    const Dev &D = h->D;
    hipStream_t st = h->stream;
    EvalArgs a;
    eval_args_base(h, a);
    a.list = host_list(D, list_id);
    a.count_ptr = &D.ctl->count[list_id];
    a.n_jobs = D.N;
    if (D.grad_mode == CHISAO_GRAD_ADJOINT) {
        a.F_out = F_out;
        a.G_out = G_out;
        return run_eval(h, a, kDirect, false, true);
    }
    hipError_t e = hipSuccess;
    if (want_f) {
        a.F_out = F_out;
        a.G_out = nullptr;
        e = run_eval(h, a, kDirect, false, false);
        if (e != hipSuccess) return e;
    }
    a.F_out = nullptr;
    a.G_out = G_out;
    return run_eval(h, a, kDirect, true, false);
}

static hipError_t phase_converge(chisao_ctx *h) {
    const Dev &D = h->D;
    hipStream_t st = h->stream;
    hipError_t e;
    const bool adj = D.grad_mode == CHISAO_GRAD_ADJOINT;
    if ((e = launch_begin_cycle(D, st)) != hipSuccess) return e;
    if ((e = eval_list(h, L_ACT, D.F, D.G, true)) != hipSuccess) return e;
    for (int t = 1; t <= D.n_conv + 1; ++t) {
        if ((e = launch_reset_counts(D, (1 << L_T1) | (1 << L_T2) | (1 << L_FD), st)) != hipSuccess) return e;
        if ((e = timed(h, CHISAO_PROF_LBFGS, [&] { return launch_lbfgs_step(D, t, st); })) != hipSuccess) return e;
        if (t > D.n_conv) break;
        EvalArgs a;
        eval_args_base(h, a);
        a.list = host_list(D, L_T1);
        a.count_ptr = &D.ctl->count[L_T1];
        a.n_jobs = D.N;
        a.Vc = 1;
        a.r0 = 0;
        a.trial_next = D.ls_max > 1 ? L_T2 : -1;
        if ((e = run_eval(h, a, kTrial, false, adj)) != hipSuccess) return e;
        if (D.ls_max > 1) {
            a.list = host_list(D, L_T2);
            a.count_ptr = &D.ctl->count[L_T2];
            a.Vc = D.ls_max - 1;
            a.r0 = 1;
            a.trial_next = -1;
            if ((e = run_eval(h, a, kTrial, false, adj)) != hipSuccess) return e;
        }
        if (!adj) {
            EvalArgs b;
            eval_args_base(h, b);
            b.list = host_list(D, L_FD);
            b.count_ptr = &D.ctl->count[L_FD];
            b.n_jobs = D.N;
            b.G_out = D.G;
            if ((e = run_eval(h, b, kDirect, true, false)) != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

static hipError_t phase_hlc(chisao_ctx *h) {
    const Dev &D = h->D;
    hipStream_t st = h->stream;
    hipError_t e;
    if ((e = launch_build_list(D, L_UNF, st)) != hipSuccess) return e;
    if ((e = launch_sigma(D, st)) != hipSuccess) return e;
    if (!((D.phase_mask >> 5) & 1)) return hipSuccess;
    const bool adj = D.grad_mode == CHISAO_GRAD_ADJOINT;
    for (int step = 0; step < D.n_cloud; ++step) {
        EvalArgs a;
        eval_args_base(h, a);
        a.list = host_list(D, L_UNF);
        a.count_ptr = &D.ctl->count[L_UNF];
        a.n_jobs = D.N;
        a.Vc = D.M;
        a.step = step;
        if ((e = run_eval(h, a, kProbe, !adj, adj)) != hipSuccess) return e;
        if (!adj && (e = launch_probe_mean(D, st)) != hipSuccess) return e;
        if (step == 0 && (e = launch_step_size(D, D.Gh, 0, st)) != hipSuccess) return e;
        if ((e = launch_hlc_update(D, st)) != hipSuccess) return e;
    }
    return hipSuccess;
}

static hipError_t phase_anti(chisao_ctx *h) {
    const Dev &D = h->D;
    hipStream_t st = h->stream;
    hipError_t e;
    if (!((D.phase_mask >> 6) & 1)) return hipSuccess;
    for (int step = 0; step < D.n_anti; ++step) {
        if ((e = eval_list(h, L_UNF, nullptr, D.Gh, false)) != hipSuccess) return e;
        if (step == 0 && (e = launch_step_size(D, D.Gh, 1, st)) != hipSuccess) return e;
        if ((e = launch_anti_update(D, step, st)) != hipSuccess) return e;
    }
    return hipSuccess;
}

static hipError_t enqueue_phases(chisao_ctx *h, uint32_t mask) {
    hipError_t e;
    const Dev &D = h->D;
    hipStream_t st = h->stream;
    if (mask & (1u << 1))
        if ((e = phase_converge(h)) != hipSuccess) return e;
    if (mask & (1u << 2))
        if ((e = launch_stick(D, st)) != hipSuccess) return e;
    if (mask & (1u << 3))
        if ((e = launch_dedup(D, st)) != hipSuccess) return e;
    if (mask & (1u << 4))
        if ((e = launch_reseed(D, st)) != hipSuccess) return e;
    if (mask & (1u << 5))
        if ((e = phase_hlc(h)) != hipSuccess) return e;
    if (mask & (1u << 6))
        if ((e = phase_anti(h)) != hipSuccess) return e;
    return hipSuccess;
}

extern "C" int chisao_run_phases(chisao_handle h, uint32_t phase_mask) {
    if (!h) return fail(CHISAO_E_INVAL, "null handle");
    HIP_TRY(hipSetDevice(h->device));
    HIP_TRY(enqueue_phases(h, phase_mask & 0x7E));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return CHISAO_OK;
}

extern "C" int chisao_cycle(chisao_handle h, int n_cycles, chisao_cycle_stats *stats_host) {
    if (!h) return fail(CHISAO_E_INVAL, "null handle");
    if (n_cycles < 0) return fail(CHISAO_E_INVAL, "negative cycle count");
    if (h->k_host + n_cycles > h->D.n_osc)
        return fail(CHISAO_E_STATE, "%d cycles requested but only %d of n_osc=%d remain", n_cycles,
                    h->D.n_osc - h->k_host, h->D.n_osc);
    HIP_TRY(hipSetDevice(h->device));
    const int k0 = h->k_host;
    for (int i = 0; i < n_cycles; ++i) {
        const bool last = (h->k_host + 1 == h->D.n_osc);
        const uint32_t mask = last ? 0x0Eu : 0x7Eu;
        HIP_TRY(enqueue_phases(h, mask));
        HIP_TRY(launch_end_cycle(h->D, 1, h->stream));
        h->k_host += 1;
    }
    if (stats_host && n_cycles > 0) {
        std::vector<CycleRecord> rec(n_cycles);
        HIP_TRY(hipMemcpyAsync(rec.data(), h->D.records + k0, sizeof(CycleRecord) * n_cycles,
                               hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
        for (int i = 0; i < n_cycles; ++i) {
            chisao_cycle_stats &o = stats_host[i];
            const CycleRecord &r = rec[i];
            o.k = r.k;
            o.f_max = r.f_max;
            o.n_stuck = r.n_stuck;
            o.K_lost = r.K_lost;
            o.n_modes = r.n_modes;
            o.reseed_kind = r.reseed_kind;
            o.n_free = r.n_free;
            o.n_unfrozen = r.n_unfrozen;
            o.n_active = r.n_active;
            o.sigma = r.sigma;
            o.alpha_c = r.alpha_c;
            o.alpha_a = r.alpha_a;
            o.ls_fail = r.ls_fail;
            o.evals = r.evals;
        }
    }
    return CHISAO_OK;
}

extern "C" int chisao_get_state(chisao_handle h, chisao_state *s) {
    if (!h || !s) return fail(CHISAO_E_INVAL, "null argument");
    const Dev &D = h->D;
    const size_t N = D.N, d = D.d;
    HIP_TRY(hipSetDevice(h->device));
    HIP_TRY(hipStreamSynchronize(h->stream));
    if (s->X) HIP_TRY(hipMemcpy(s->X, D.X, sizeof(float) * N * d, hipMemcpyDeviceToHost));
    if (s->F) HIP_TRY(hipMemcpy(s->F, D.F, sizeof(float) * N, hipMemcpyDeviceToHost));
    if (s->G) HIP_TRY(hipMemcpy(s->G, D.G, sizeof(float) * N * d, hipMemcpyDeviceToHost));
    if (s->stuck) HIP_TRY(hipMemcpy(s->stuck, D.stuck, N, hipMemcpyDeviceToHost));
    if (s->active) HIP_TRY(hipMemcpy(s->active, D.active, N, hipMemcpyDeviceToHost));
    if (s->stuck_pre) HIP_TRY(hipMemcpy(s->stuck_pre, D.stuck_pre, N, hipMemcpyDeviceToHost));
    if (s->removed) HIP_TRY(hipMemcpy(s->removed, D.removed, N, hipMemcpyDeviceToHost));
    if (s->trace) HIP_TRY(hipMemcpy(s->trace, D.trace, N * (size_t)(D.n_conv + 1), hipMemcpyDeviceToHost));
    const size_t m = D.m;
    if (s->S) HIP_TRY(hipMemcpy(s->S, D.S, sizeof(float) * N * m * d, hipMemcpyDeviceToHost));
    if (s->Y) HIP_TRY(hipMemcpy(s->Y, D.Y, sizeof(float) * N * m * d, hipMemcpyDeviceToHost));
    if (s->rho) HIP_TRY(hipMemcpy(s->rho, D.rho, sizeof(float) * N * m, hipMemcpyDeviceToHost));
    if (s->head) HIP_TRY(hipMemcpy(s->head, D.head, sizeof(int) * N, hipMemcpyDeviceToHost));
    if (s->cnt) HIP_TRY(hipMemcpy(s->cnt, D.cnt, sizeof(int) * N, hipMemcpyDeviceToHost));
    if (s->conv) HIP_TRY(hipMemcpy(s->conv, D.conv, N, hipMemcpyDeviceToHost));
    Ctl c;
    HIP_TRY(hipMemcpy(&c, D.ctl, sizeof c, hipMemcpyDeviceToHost));
    s->k = c.k;
    s->gr_disabled = c.gr_disabled;
    s->gr_fail = c.gr_fail;
    s->gr_used_last = c.gr_used_last;
    s->gr_prev_modes = c.gr_prev_modes;
    return CHISAO_OK;
}

extern "C" int chisao_set_state(chisao_handle h, const chisao_state *s) {
    if (!h || !s) return fail(CHISAO_E_INVAL, "null argument");
    const Dev &D = h->D;
    const size_t N = D.N, d = D.d;
    if (s->k < 0 || s->k > D.n_osc) return fail(CHISAO_E_INVAL, "k out of range");
    HIP_TRY(hipSetDevice(h->device));
    HIP_TRY(hipStreamSynchronize(h->stream));
    if (s->X) {
        std::vector<float> lo(d), hi(d);
        HIP_TRY(hipMemcpy(lo.data(), D.lo, sizeof(float) * d, hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(hi.data(), D.hi, sizeof(float) * d, hipMemcpyDeviceToHost));
        for (size_t i = 0; i < N * d; ++i)
            if (!(s->X[i] >= lo[i % d] && s->X[i] <= hi[i % d]))
                return fail(CHISAO_E_INVAL, "sample %zu lies outside the box", i / d);
        HIP_TRY(hipMemcpy(D.X, s->X, sizeof(float) * N * d, hipMemcpyHostToDevice));
    }
    if (s->stuck) HIP_TRY(hipMemcpy(D.stuck, s->stuck, N, hipMemcpyHostToDevice));
    if (s->active) HIP_TRY(hipMemcpy(D.active, s->active, N, hipMemcpyHostToDevice));
    Ctl c;
    HIP_TRY(hipMemcpy(&c, D.ctl, sizeof c, hipMemcpyDeviceToHost));
    c.k = s->k;
    c.gr_disabled = s->gr_disabled;
    c.gr_fail = s->gr_fail;
    c.gr_used_last = s->gr_used_last;
    c.gr_prev_modes = s->gr_prev_modes;
    HIP_TRY(hipMemcpy(D.ctl, &c, sizeof c, hipMemcpyHostToDevice));
    h->k_host = s->k;
    return CHISAO_OK;
}

extern "C" int chisao_modes(chisao_handle h, int problem, float *x_out, float *f_out, int cap, int *n_out) {
    if (!h || !n_out) return fail(CHISAO_E_INVAL, "null argument");
    if (problem != 0) return fail(CHISAO_E_INVAL, "single-problem handle: problem must be 0");
    const Dev &D = h->D;
    HIP_TRY(hipSetDevice(h->device));
    HIP_TRY(launch_mode_list(D, h->stream));
    Ctl c;
    HIP_TRY(hipMemcpyAsync(&c, D.ctl, sizeof c, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    const int n = c.count[O_PEAKS];
    *n_out = n;
    if (cap < n) return fail(CHISAO_E_RANGE, "capacity %d < %d modes", cap, n);
    if (n == 0) return CHISAO_OK;
    if (!x_out) return fail(CHISAO_E_INVAL, "null x_out");
    // rows gathered into Gh (scratch at this point), values into Pd
    HIP_TRY(hipMemcpyAsync(x_out, D.Gh, sizeof(float) * (size_t)n * D.d, hipMemcpyDeviceToHost, h->stream));
    if (f_out) HIP_TRY(hipMemcpyAsync(f_out, D.Pd, sizeof(float) * (size_t)n, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return CHISAO_OK;
}

extern "C" int chisao_profile(chisao_handle h, int enable, chisao_kernel_profile *out) {
    if (!h) return fail(CHISAO_E_INVAL, "null handle");
    HIP_TRY(hipSetDevice(h->device));
    if (enable) {
        HIP_TRY(hipStreamSynchronize(h->stream));
        unsigned long long zero[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        HIP_TRY(hipMemcpy(h->D.ctl->prof_points, zero, sizeof zero, hipMemcpyHostToDevice));
        h->ev_used.clear();
        h->prof = true;
        return CHISAO_OK;
    }
    h->prof = false;
    HIP_TRY(hipStreamSynchronize(h->stream));
    if (out) {
        chisao_kernel_profile res[CHISAO_PROF_CLASSES];
        memset(res, 0, sizeof res);
        for (auto &u : h->ev_used) {
            float ms = 0.0f;
            HIP_TRY(hipEventElapsedTime(&ms, h->ev_pool[u.second], h->ev_pool[u.second + 1]));
            res[u.first].launches += 1;
            res[u.first].ms += ms;
        }
        unsigned long long pts[8];
        HIP_TRY(hipMemcpy(pts, h->D.ctl->prof_points, sizeof pts, hipMemcpyDeviceToHost));
        for (int i = 0; i < 8 && i < CHISAO_PROF_CLASSES; ++i) res[i].points = (int64_t)pts[i];
        memcpy(out, res, sizeof res);
    }
    h->ev_used.clear();
    return CHISAO_OK;
}

extern "C" int chisao_eval(chisao_handle h, const float *X_dev, int B, float *f_dev, float *G_dev, int grad_mode) {
    if (!h) return fail(CHISAO_E_INVAL, "null handle");
    if (B < 0) return fail(CHISAO_E_INVAL, "negative batch");
    if (B == 0) return CHISAO_OK;
    if (!X_dev) return fail(CHISAO_E_INVAL, "null X");
    if (grad_mode != CHISAO_GRAD_FD && grad_mode != CHISAO_GRAD_ADJOINT) return fail(CHISAO_E_INVAL, "bad grad_mode");
    HIP_TRY(hipSetDevice(h->device));
    EvalArgs a;
    eval_args_base(h, a);
    a.X = X_dev;
    a.list = nullptr;
    a.count_ptr = nullptr;
    a.n_jobs = B;
    hipStream_t st = h->stream;
    if (grad_mode == CHISAO_GRAD_ADJOINT) {
        a.F_out = f_dev;
        a.G_out = G_dev;
        HIP_TRY(launch_eval(a, kDirect, false, G_dev != nullptr, st));
        return CHISAO_OK;
    }
    if (f_dev) {
        a.F_out = f_dev;
        a.G_out = nullptr;
        HIP_TRY(launch_eval(a, kDirect, false, false, st));
    }
    if (G_dev) {
        a.F_out = nullptr;
        a.G_out = G_dev;
        HIP_TRY(launch_eval(a, kDirect, true, false, st));
    }
    return CHISAO_OK;
}
