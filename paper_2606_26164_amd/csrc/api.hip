// Host side of libchisao: the C ABI declared in include/chisao.h.
//
// A handle owns the device workspace of P independent problems.  A cycle is
// a fixed sequence of kernel launches; every data-dependent choice inside it
// (which samples move, line-search outcomes, Repulse Monkey or Golden
// Rooster, step lengths) is read by the kernels from device memory, so the
// host never waits inside a cycle and the sequence can be captured once into
// a hipGraph and replayed for every cycle.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "chisao.h"
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

#define HIP_TRY(expr)                                                                               \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess) return fail(CHISAO_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
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

// Launch schedules the autotuner tries per evaluation class: tile order
// (linear, XCD-chunked) x grid (8192 workgroups, dispatched as slots free up;
// 1024, one resident wave per SIMD looping over tiles).
constexpr int kTuneVariants = 4;
constexpr int kMaxTrials = 15;  // upper bound of ls_max
constexpr int kTuneOrder[kTuneVariants] = {0, 1, 0, 1};
constexpr int kTuneCap[kTuneVariants] = {8192, 8192, 1024, 1024};
constexpr float kTuneMargin = 0.97f;
int coords_per_lane(int d) { return d <= 16 ? 1 : (d <= 32 ? 2 : 4); }

}  // namespace

// A group of problems served by one evaluation launch.
struct EvalClass {
    int DP, family, grad_mode;
    const int *pids_dev;  // into the handle's class table
    std::vector<int> pids;
    int g0 = 0, n = 0;    // the class's samples: a contiguous range
    int cpl = 1;          // L-BFGS lane layout of its largest d
    int nconv = 0;        // most L-BFGS iterations among its problems
    int order = 0, grid_cap = 0;  // launch schedule (set by the autotuner)
    int half = 0;                 // 16-point tiles for direct launches (set by the autotuner)
    int p_order = 0, p_grid_cap = 0;  // schedule of the smoothing-probe launches (set by the autotuner)
    int t_grid_cap = 0;               // grid of the line-search launches: the resident workgroups (0: grid_cap)
    float tune_ms[kTuneVariants] = {};
    float tune_half_ms = 0.0f, tune_full_ms = 0.0f;
    float tune_probe_ms[kTuneVariants] = {};
};

struct chisao_ctx {
    Dev D{};
    hipStream_t stream = nullptr;  // the caller's stream: all work runs here
    hipStream_t cur = nullptr;     // where launches are enqueued (stream, or the capture stream)
    hipStream_t cap = nullptr;     // private stream for graph capture
    // side streams and events that fork the launches of several classes off
    // `cur` and join them back (one stream per class after the first)
    std::vector<hipStream_t> side;
    hipEvent_t ev_fork = nullptr;
    std::vector<hipEvent_t> ev_join;
    int device = 0;
    int k_host = 0;  // cycles completed
    uint32_t flags = 0;
    bool any_noise = false;
    std::vector<ProblemDesc> pdh;  // host copy of the descriptors
    std::vector<EvalClass> eclasses;
    const int *pid_seq = nullptr;  // device [P]: 0, 1, ..., P-1
    Buffers buf;
    hipGraphExec_t graph[2] = {nullptr, nullptr};  // [0]: cycles before n_osc, [1]: the last cycle
    // profiling: event pairs recorded around launches of each class
    bool prof = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, size_t>> ev_used;
    ~chisao_ctx() {
        for (hipGraphExec_t g : graph)
            if (g) (void)hipGraphExecDestroy(g);
        for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
        for (hipEvent_t e : ev_join) (void)hipEventDestroy(e);
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        for (hipStream_t s : side) (void)hipStreamDestroy(s);
        if (cap) (void)hipStreamDestroy(cap);
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
    hipError_t r = hipEventRecord(h->ev_pool[i], h->cur);
    if (r != hipSuccess) return r;
    r = launch();
    if (r != hipSuccess) return r;
    r = hipEventRecord(h->ev_pool[i + 1], h->cur);
    if (r != hipSuccess) return r;
    h->ev_used.push_back({cls, i});
    return hipSuccess;
}

// Side streams for n classes.  The launches of different classes touch
// disjoint samples (the counters they share are updated atomically), so with
// more than one class every class after the first goes to a side stream
// forked from the current one by an event and joined back by another: in a
// captured cycle these are parallel branches of the graph, and the classes'
// launches run side by side instead of one after another.  When profiling,
// everything stays on the current stream, in order.
static bool forks(const chisao_ctx *h, size_t n) { return n > 1 && !h->prof && h->side.size() + 1 >= n; }
static hipStream_t branch(const chisao_ctx *h, bool forked, size_t j) {
    return (forked && j > 0) ? h->side[j - 1] : h->cur;
}
static hipError_t fork_open(chisao_ctx *h, size_t n) {
    hipError_t e = hipEventRecord(h->ev_fork, h->cur);
    for (size_t j = 1; j < n && e == hipSuccess; ++j) e = hipStreamWaitEvent(h->side[j - 1], h->ev_fork, 0);
    return e;
}
static hipError_t fork_close(chisao_ctx *h, size_t n) {
    hipError_t e = hipSuccess;
    for (size_t j = 1; j < n && e == hipSuccess; ++j) e = hipEventRecord(h->ev_join[j - 1], h->side[j - 1]);
    for (size_t j = 1; j < n && e == hipSuccess; ++j) e = hipStreamWaitEvent(h->cur, h->ev_join[j - 1], 0);
    return e;
}

// ---------------------------------------------------------------------------
// Validation
// ---------------------------------------------------------------------------
static int validate_problem(const chisao_problem *p, int idx) {
    if (!p) return fail(CHISAO_E_INVAL, "null problem");
    if (p->family < CHISAO_GAUSS || p->family > CHISAO_BUKIN6)
        return fail(CHISAO_E_INVAL, "problem %d: unknown family %d", idx, p->family);
    const bool closed = p->family >= CHISAO_RASTRIGIN;
    if (p->d < 1 || p->d > 64) return fail(CHISAO_E_INVAL, "problem %d: d must be in 1..64 (got %d)", idx, p->d);
    if (p->family == CHISAO_BUKIN6 && p->d != 2) return fail(CHISAO_E_INVAL, "problem %d: Bukin N.6 needs d = 2", idx);
    // (component tables are addressed with 32-bit byte offsets: K d_pad^2 4 < 2^31)
    if (!closed && (p->K < 1 || p->K > 65536)) return fail(CHISAO_E_INVAL, "problem %d: K must be in 1..65536", idx);
    if ((!closed && (!p->log_w || !p->mu || !p->prec)) || !p->lo || !p->hi)
        return fail(CHISAO_E_INVAL, "problem %d: null problem array", idx);
    if (p->family == CHISAO_STUDENT_T && !(p->nu > 0.0f && isfinite(p->nu)))
        return fail(CHISAO_E_INVAL, "problem %d: Student-t needs nu > 0", idx);
    if (!(p->noise_sigma >= 0.0f && isfinite(p->noise_sigma)))
        return fail(CHISAO_E_INVAL, "problem %d: noise_sigma must be finite and >= 0", idx);
    const int d = p->d, K = closed ? 0 : p->K;
    for (int j = 0; j < d; ++j)
        if (!(isfinite(p->lo[j]) && isfinite(p->hi[j]) && p->lo[j] < p->hi[j]))
            return fail(CHISAO_E_INVAL, "problem %d: box bounds must be finite with lo < hi (coordinate %d)", idx, j);
    for (int k = 0; k < K; ++k) {
        if (!isfinite(p->log_w[k])) return fail(CHISAO_E_INVAL, "problem %d: non-finite log weight %d", idx, k);
        for (int j = 0; j < d; ++j)
            if (!isfinite(p->mu[(size_t)k * d + j])) return fail(CHISAO_E_INVAL, "problem %d: non-finite centre %d", idx, k);
        const float *P = p->prec + (size_t)k * d * d;
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j) {
                if (!isfinite(P[i * d + j]))
                    return fail(CHISAO_E_INVAL, "problem %d: non-finite precision entry in component %d", idx, k);
                if (P[i * d + j] != P[j * d + i])
                    return fail(CHISAO_E_INVAL, "problem %d: precision matrix %d not symmetric", idx, k);
            }
    }
    return CHISAO_OK;
}

static int validate(const chisao_problem *p, const chisao_config *c, int idx) {
    if (!p || !c) return fail(CHISAO_E_INVAL, "null problem or config");
    int rc = validate_problem(p, idx);
    if (rc) return rc;
    if (c->N < 1 || c->N > (1 << 30)) return fail(CHISAO_E_INVAL, "problem %d: N must be in 1..2^30", idx);
    if (c->m < 1 || c->m > 32) return fail(CHISAO_E_INVAL, "problem %d: m must be in 1..32", idx);
    if (c->n_osc < 1) return fail(CHISAO_E_INVAL, "problem %d: n_osc must be >= 1", idx);
    if (c->n_anti < 0 || c->n_cloud < 0) return fail(CHISAO_E_INVAL, "problem %d: negative step count", idx);
    // the step index occupies bits 16..23 of a random-stream counter word
    if (c->n_conv > 255 || c->n_anti > 255 || c->n_cloud > 255)
        return fail(CHISAO_E_INVAL, "problem %d: n_conv, n_anti and n_cloud must be at most 255", idx);
    if (c->M < 1 || c->M > 32) return fail(CHISAO_E_INVAL, "problem %d: M must be in 1..32", idx);
    if (c->ls_max < 1 || c->ls_max > 15) return fail(CHISAO_E_INVAL, "problem %d: ls_max must be in 1..15", idx);
    if (c->grad_mode != CHISAO_GRAD_FD && c->grad_mode != CHISAO_GRAD_ADJOINT)
        return fail(CHISAO_E_INVAL, "problem %d: unknown grad_mode", idx);
    if (c->gate_reps < 0 || c->gate_reps > 4096) return fail(CHISAO_E_INVAL, "problem %d: gate_reps must be in 0..4096", idx);
    if (!(c->eps_grad > 0.0f) || !(c->eps_dup > 0.0f))
        return fail(CHISAO_E_INVAL, "problem %d: eps_grad and eps_dup must be > 0", idx);
    if (!isfinite(c->log_delta) || !isfinite(c->momentum) || !isfinite(c->alpha) || !isfinite(c->sigma) ||
        !isfinite(c->sigma_c) || !isfinite(c->fd_h) || !isfinite(c->ls_c1) || !isfinite(c->curv_eps))
        return fail(CHISAO_E_INVAL, "problem %d: non-finite hyperparameter", idx);
    return CHISAO_OK;
}

extern "C" const char *chisao_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------------------
// Creation
// ---------------------------------------------------------------------------
static int autotune(chisao_ctx *h);

extern "C" int chisao_init_batched(chisao_handle *out, int n_problems, const chisao_problem *ps,
                                   const chisao_config *cs, const float *const *x0_dev, void *hip_stream) {
    if (!out) return fail(CHISAO_E_INVAL, "null output handle");
    *out = nullptr;
    if (n_problems < 1 || n_problems > 256) return fail(CHISAO_E_INVAL, "n_problems must be in 1..256");
    if (!ps || !cs) return fail(CHISAO_E_INVAL, "null problem or config array");
    int rc;
    long NT = 0;
    int DS = 1, mmax = 1, Mmax = 1, ncmax = 0;
    std::vector<int> n_conv(n_problems);
    for (int p = 0; p < n_problems; ++p) {
        if ((rc = validate(&ps[p], &cs[p], p))) return rc;
        if (cs[p].n_osc != cs[0].n_osc) return fail(CHISAO_E_INVAL, "all problems of a batch need the same n_osc");
        NT += cs[p].N;
        DS = std::max(DS, ps[p].d);
        mmax = std::max(mmax, cs[p].m);
        Mmax = std::max(Mmax, cs[p].M);
        n_conv[p] = cs[p].n_conv > 0 ? cs[p].n_conv
                                      : std::max(10, (int)ceil(3.0 * log2((double)ps[p].d) - 1e-9));
        ncmax = std::max(ncmax, n_conv[p]);
    }
    DS = (DS + 3) / 4 * 4;  // row stride: a multiple of four floats (aligned vector row access)
    if (NT * (long)DS * std::max(mmax, Mmax) > (1L << 31) - 1)
        return fail(CHISAO_E_INVAL, "population too large for 32-bit indexing");
    chisao_ctx *h = new (std::nothrow) chisao_ctx();
    if (!h) return fail(CHISAO_E_NOMEM, "host allocation failed");
    h->stream = (hipStream_t)hip_stream;
    h->cur = h->stream;
    h->flags = cs[0].flags;
    Dev &D = h->D;
    D.P = n_problems;
    D.NT = (int)NT;
    D.DS = DS;
    D.mmax = mmax;
    D.Mmax = Mmax;
    D.n_conv_max = ncmax;
    D.n_osc = cs[0].n_osc;
    D.n_part_blocks = 64;
    bool any_fd = false;
    for (int p = 0; p < n_problems; ++p) any_fd |= cs[p].grad_mode == CHISAO_GRAD_FD;

    const size_t N = (size_t)NT, P = (size_t)n_problems;
    Buffers &B = h->buf;
    hipError_t e;
    auto A = [&](void **ptr, size_t bytes) -> int {
        hipError_t r = B.alloc(ptr, bytes);
        if (r != hipSuccess) return fail(CHISAO_E_NOMEM, "hipMalloc(%zu bytes): %s", bytes, hipGetErrorString(r));
        return CHISAO_OK;
    };
#define ALLOC(field, type, count)                                           \
    do {                                                                    \
        void *tmp_;                                                         \
        if ((rc = A(&tmp_, sizeof(type) * (size_t)(count)))) goto fail_out; \
        field = (type *)tmp_;                                               \
    } while (0)
#define HIP_GO(expr)                                                           \
    do {                                                                       \
        if ((e = (expr)) != hipSuccess) {                                      \
            rc = fail(CHISAO_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e)); \
            goto fail_out;                                                     \
        }                                                                      \
    } while (0)
    {
        hipStream_t st = h->stream;
        HIP_GO(hipGetDevice(&h->device));
        int *bad;
        ALLOC(bad, int, 1);
        HIP_GO(hipMemsetAsync(bad, 0, sizeof(int), st));
        // ---- per-problem constants ----
        // Samples are laid out problem after problem, ordered by (padded d,
        // family, gradient mode), so the problems of each launch class own a
        // contiguous range of samples.
        std::vector<int> order(P);
        for (int p = 0; p < n_problems; ++p) order[p] = p;
        // Within a class the problems go in decreasing order of K (a tile's
        // time grows with its components), so the longest tiles are dealt
        // out first and the short ones fill in behind them.
        auto key = [&](int p) {
            const int K = ps[p].family >= CHISAO_RASTRIGIN ? 0 : ps[p].K;
            return std::make_tuple(pad_dim(ps[p].d, ps[p].family), ps[p].family, cs[p].grad_mode, -K);
        };
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return key(a) < key(b); });
        std::vector<int> s0_of(P);
        {
            int acc = 0;
            for (int p : order) {
                s0_of[p] = acc;
                acc += cs[p].N;
            }
        }
        h->pdh.resize(P);
        size_t rk_total = 0;
        for (int p = 0; p < n_problems; ++p) {
            const chisao_problem &pr = ps[p];
            const chisao_config &c = cs[p];
            // closed-form functions have no component arrays
            const bool closed = pr.family >= CHISAO_RASTRIGIN;
            const size_t d = pr.d, K = closed ? 0 : pr.K, DP = pad_dim(pr.d, pr.family);
            ProblemDesc &q = h->pdh[p];
            memset(&q, 0, sizeof q);
            float *Pfrag = nullptr, *muB = nullptr, *logc2 = nullptr, *lo, *hi;
            ALLOC(lo, float, d);
            ALLOC(hi, float, d);
            HIP_GO(hipMemcpyAsync(lo, pr.lo, sizeof(float) * d, hipMemcpyHostToDevice, st));
            HIP_GO(hipMemcpyAsync(hi, pr.hi, sizeof(float) * d, hipMemcpyHostToDevice, st));
            const float nu = pr.family == CHISAO_STUDENT_T ? pr.nu : 1.0f;
            if (!closed) {
                float *tw, *tmu, *tprec;
                ALLOC(Pfrag, float, K * DP * DP);
                ALLOC(muB, float, K * DP);
                ALLOC(logc2, float, K);
                ALLOC(tw, float, K);
                ALLOC(tmu, float, K * d);
                ALLOC(tprec, float, K * d * d);
                HIP_GO(hipMemcpyAsync(tw, pr.log_w, sizeof(float) * K, hipMemcpyHostToDevice, st));
                HIP_GO(hipMemcpyAsync(tmu, pr.mu, sizeof(float) * K * d, hipMemcpyHostToDevice, st));
                HIP_GO(hipMemcpyAsync(tprec, pr.prec, sizeof(float) * K * d * d, hipMemcpyHostToDevice, st));
                HIP_GO(launch_prepare(pr.family, pr.d, (int)DP, pr.K, nu, tw, tmu, tprec, logc2, Pfrag, muB, bad, st));
            }
            q.d = pr.d;
            q.DP = (int)DP;
            q.K = (int)K;
            q.family = pr.family;
            q.nu = nu;
            q.nu_plus_d = nu + (float)pr.d;
            q.Pfrag = Pfrag;
            q.muB = muB;
            q.logc2 = logc2;
            q.lo = lo;
            q.hi = hi;
            q.N = c.N;
            q.s0 = s0_of[p];
            q.m = c.m;
            q.n_conv = n_conv[p];
            q.n_anti = c.n_anti;
            q.n_cloud = c.n_cloud;
            q.M = c.M;
            q.ls_max = c.ls_max;
            q.grad_mode = c.grad_mode;
            q.eps_grad = c.eps_grad;
            q.eps_dup = c.eps_dup;
            q.log_delta = c.log_delta;
            q.momentum = c.momentum;
            q.alpha = c.alpha;
            q.sigma_cfg = c.sigma;
            q.sigma_c = c.sigma_c;
            q.fd_h = c.fd_h;
            q.ls_c1 = c.ls_c1;
            q.curv_eps = c.curv_eps;
            q.key0 = (uint32_t)(c.seed & 0xFFFFFFFFu);
            q.key1 = (uint32_t)(c.seed >> 32) ^ c.problem_id;
            q.phase_mask = c.phase_mask;
            q.ray_seed = (c.flags & CHISAO_FLAG_RAY_SEEDING) != 0;
            q.noise_sigma = pr.noise_sigma;
            q.gate_reps = c.gate_reps > 0 ? c.gate_reps : c.M;
            {
                int lb = 0;  // about four stuck samples per bucket at most
                while ((4 << lb) < c.N) ++lb;
                q.hash_lb = lb;
                q.hk0 = (int)rk_total;
                rk_total += ((size_t)1 << lb) + 1;
            }
            h->any_noise |= pr.noise_sigma > 0.0f;
        }
        ProblemDesc *pd_dev;
        ALLOC(pd_dev, ProblemDesc, P);
        HIP_GO(hipMemcpyAsync(pd_dev, h->pdh.data(), sizeof(ProblemDesc) * P, hipMemcpyHostToDevice, st));
        D.pd = pd_dev;
        std::vector<uint16_t> pid(N);
        for (int p = 0; p < n_problems; ++p)
            for (int i = 0; i < h->pdh[p].N; ++i) pid[h->pdh[p].s0 + i] = (uint16_t)p;
        uint16_t *pid_dev;
        ALLOC(pid_dev, uint16_t, N);
        HIP_GO(hipMemcpyAsync(pid_dev, pid.data(), sizeof(uint16_t) * N, hipMemcpyHostToDevice, st));
        D.pid = pid_dev;
        // ---- launch classes ----
        std::map<std::tuple<int, int, int>, std::vector<int>> ecl;
        for (int p = 0; p < n_problems; ++p) {
            ecl[{h->pdh[p].DP, h->pdh[p].family, h->pdh[p].grad_mode}].push_back(p);
        }
        std::vector<int> table;
        for (int p = 0; p < n_problems; ++p) table.push_back(p);  // pid_seq
        for (auto &kv : ecl) table.insert(table.end(), kv.second.begin(), kv.second.end());
        int *tab_dev;
        ALLOC(tab_dev, int, table.size());
        HIP_GO(hipMemcpyAsync(tab_dev, table.data(), sizeof(int) * table.size(), hipMemcpyHostToDevice, st));
        HIP_GO(hipStreamSynchronize(st));  // the host vector goes out of scope
        h->pid_seq = tab_dev;
        size_t off = P;
        for (auto &kv : ecl) {
            EvalClass c;
            std::tie(c.DP, c.family, c.grad_mode) = kv.first;
            c.pids = kv.second;
            c.pids_dev = tab_dev + off;
            off += kv.second.size();
            c.g0 = (int)N;
            int dmax = 1;
            for (int p : c.pids) {
                const ProblemDesc &q = h->pdh[p];
                c.g0 = std::min(c.g0, q.s0);
                c.n += q.N;
                dmax = std::max(dmax, q.d);
                c.nconv = std::max(c.nconv, q.n_conv);
            }
            c.cpl = coords_per_lane(dmax);
            // (CHISAO_FLAG_NO_AUTOTUNE keeps every launch at the default grid)
            c.t_grid_cap = (h->flags & CHISAO_FLAG_NO_AUTOTUNE)
                               ? 0
                               : trial_resident_blocks(c.DP, c.family, c.grad_mode == CHISAO_GRAD_ADJOINT);
            h->eclasses.push_back(c);
        }
        // ---- population state ----
        const size_t DSz = (size_t)DS;
        ALLOC(D.X, float, N * DSz);
        ALLOC(D.F, float, N);
        ALLOC(D.G, float, N * DSz);
        ALLOC(D.V, float, N * DSz);
        ALLOC(D.Xprev, float, N * DSz);
        ALLOC(D.Gprev, float, N * DSz);
        ALLOC(D.Pd, float, N * DSz);
        ALLOC(D.Gh, float, N * DSz);
        ALLOC(D.ginf, float, N);
        ALLOC(D.Fg, float, N);
        ALLOC(D.Wd, float, N * DSz);
        ALLOC(D.wvalid, uint8_t, N);
        if (any_fd) ALLOC(D.Gp, float, N * (size_t)Mmax * DSz);
        ALLOC(D.stuck, uint8_t, N);
        ALLOC(D.active, uint8_t, N);
        ALLOC(D.conv, uint8_t, N);
        ALLOC(D.removed, uint8_t, N);
        ALLOC(D.stuck_pre, uint8_t, N);
        ALLOC(D.status, uint8_t, N);
        ALLOC(D.reset, uint8_t, N);
        ALLOC(D.steep, uint8_t, N);
        ALLOC(D.trace, uint8_t, N * (size_t)(ncmax + 1));
        ALLOC(D.S, float, N * (size_t)mmax * DSz);
        ALLOC(D.Y, float, N * (size_t)mmax * DSz);
        ALLOC(D.rho, float, N * (size_t)mmax);
        ALLOC(D.head, int, N);
        ALLOC(D.cnt, int, N);
        ALLOC(D.lists, int, N * kNumLists);
        ALLOC(D.flag, uint8_t, N);
        ALLOC(D.hoff, int, rk_total);
        ALLOC(D.hcur, int, rk_total);
        ALLOC(D.hcell, int, N);
        ALLOC(D.ctl, Ctl, P);
        ALLOC(D.records, CycleRecord, P * (size_t)D.n_osc);
        ALLOC(D.part, double, P * (size_t)D.n_part_blocks * 129);
        ALLOC(D.prof, unsigned long long, kProfClasses);
        HIP_GO(hipMemsetAsync(D.X, 0, sizeof(float) * N * DSz, st));
        // row arrays start at zero: the L-BFGS kernel reads whole aligned
        // chunks and relies on the columns past each problem's d being zero
        HIP_GO(hipMemsetAsync(D.G, 0, sizeof(float) * N * DSz, st));
        HIP_GO(hipMemsetAsync(D.Xprev, 0, sizeof(float) * N * DSz, st));
        HIP_GO(hipMemsetAsync(D.Gprev, 0, sizeof(float) * N * DSz, st));
        HIP_GO(hipMemsetAsync(D.Pd, 0, sizeof(float) * N * DSz, st));
        HIP_GO(hipMemsetAsync(D.S, 0, sizeof(float) * N * (size_t)mmax * DSz, st));
        HIP_GO(hipMemsetAsync(D.Y, 0, sizeof(float) * N * (size_t)mmax * DSz, st));
        HIP_GO(hipMemsetAsync(D.Wd, 0, sizeof(float) * N * DSz, st));
        HIP_GO(hipMemsetAsync(D.wvalid, 0, N, st));
        HIP_GO(launch_uniform_init(D, st));
        if (x0_dev) {
            for (int p = 0; p < n_problems; ++p)
                if (x0_dev[p]) {
                    const ProblemDesc &q = h->pdh[p];
                    HIP_GO(hipMemcpy2DAsync(D.X + (size_t)q.s0 * DSz, DSz * sizeof(float), x0_dev[p],
                                            (size_t)q.d * sizeof(float), (size_t)q.d * sizeof(float), (size_t)q.N,
                                            hipMemcpyDeviceToDevice, st));
                }
        }
        HIP_GO(launch_fill_u8(D.active, 1, N, st));
        HIP_GO(launch_fill_u8(D.stuck, 0, N, st));
        HIP_GO(hipMemsetAsync(D.V, 0, sizeof(float) * N * DSz, st));
        HIP_GO(hipMemsetAsync(D.ctl, 0, sizeof(Ctl) * P, st));
        HIP_GO(hipMemsetAsync(D.records, 0, sizeof(CycleRecord) * P * D.n_osc, st));
        HIP_GO(hipMemsetAsync(D.prof, 0, sizeof(unsigned long long) * kProfClasses, st));
        int bad_h = 0;
        HIP_GO(hipMemcpyAsync(&bad_h, bad, sizeof(int), hipMemcpyDeviceToHost, st));
        HIP_GO(hipStreamSynchronize(st));
        if (bad_h) {
            rc = fail(CHISAO_E_INVAL, "a precision matrix is not positive definite");
            goto fail_out;
        }
        if (x0_dev) {
            // starting populations must lie in their boxes
            for (int p = 0; p < n_problems; ++p) {
                if (!x0_dev[p]) continue;
                const ProblemDesc &q = h->pdh[p];
                std::vector<float> xh((size_t)q.N * q.d);
                HIP_GO(hipMemcpy(xh.data(), x0_dev[p], sizeof(float) * xh.size(), hipMemcpyDeviceToHost));
                for (size_t i = 0; i < xh.size(); ++i) {
                    const size_t j = i % q.d;
                    if (!(xh[i] >= ps[p].lo[j] && xh[i] <= ps[p].hi[j])) {
                        rc = fail(CHISAO_E_INVAL, "problem %d: x0 sample %zu lies outside the box", p, i / q.d);
                        goto fail_out;
                    }
                }
            }
        }
        HIP_GO(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
        {
            const int n_side = (int)h->eclasses.size() - 1;
            if (n_side > 0) HIP_GO(hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming));
            for (int i = 0; i < n_side; ++i) {
                hipStream_t s;
                hipEvent_t ev;
                HIP_GO(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
                h->side.push_back(s);
                HIP_GO(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
                h->ev_join.push_back(ev);
            }
        }
        if (!(h->flags & CHISAO_FLAG_NO_AUTOTUNE) && (rc = autotune(h))) goto fail_out;
        if (h->flags & CHISAO_FLAG_HALF_TILES)
            for (EvalClass &c : h->eclasses) c.half = (c.DP != kAluDP && c.family < kFamClosed) ? 1 : 0;
    }
#undef ALLOC
#undef HIP_GO
    *out = h;
    return CHISAO_OK;
fail_out:
    (void)hipStreamSynchronize(h->stream);
    delete h;
    return rc;
}

extern "C" int chisao_init(chisao_handle *out, const chisao_problem *p, const chisao_config *c, const float *x0_dev,
                           void *hip_stream) {
    const float *x0s[1] = {x0_dev};
    return chisao_init_batched(out, 1, p, c, x0_dev ? x0s : nullptr, hip_stream);
}

extern "C" void chisao_destroy(chisao_handle h) {
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    delete h;
}

// ---------------------------------------------------------------------------
// Phase sequences
// ---------------------------------------------------------------------------
static EvalArgs base_args(chisao_ctx *h, const EvalClass &c) {
    EvalArgs a;
    memset(&a, 0, sizeof a);
    a.D = h->D;
    a.cls = c.pids_dev;
    a.n_cls = (int)c.pids.size();
    a.X = h->D.X;
    a.x_stride = h->D.DS;
    a.out_stride = h->D.DS;
    a.ext_n = -1;
    a.list_id = -1;
    a.trial_next = -1;
    a.nz_kind = -1;
    return a;
}

// Upper bound on the tiles of a launch (sizes its grid).
static long tile_bound(chisao_ctx *h, const EvalClass &c, int vc_kind, bool fd, int trial_lo = 0, int trial_cnt = 0) {
    long t = 0;
    for (int p : c.pids) {
        const ProblemDesc &q = h->pdh[p];
        const int Vc = vc_kind == kVcTrialRest ? std::max(0, std::min(trial_cnt, q.ls_max - trial_lo))
                                               : (vc_kind == kVcProbes ? q.M : 1);
        const long V = (long)Vc * (fd ? 2 * q.d : 1);
        if (V <= 0) continue;
        t += V <= 32 ? (q.N + (32 / V) - 1) / (32 / V) : (long)q.N * ((V + 31) / 32);
    }
    return t;
}

static hipError_t run_eval(chisao_ctx *h, const EvalClass &c, EvalArgs &a, int center, bool fd, bool grad,
                           hipStream_t st) {
    a.max_tiles = tile_bound(h, c, a.vc_kind, fd, a.trial_lo, a.trial_cnt);
    a.order = center == kProbe ? c.p_order : c.order;
    // line-search launches: one round of resident workgroups looping over the
    // tiles (their launches come one per stage and iteration, each a few
    // tiles per CU; a queue of one-tile workgroups leaves a tail per launch,
    // and in a batch it crowds out the other classes' concurrent launches)
    a.grid_cap = center == kProbe ? c.p_grid_cap : (center == kTrial && c.t_grid_cap > 0 ? c.t_grid_cap : c.grid_cap);
    a.half_tiles = (center == kDirect && !fd) ? c.half : 0;
    const int cls = fd ? CHISAO_PROF_EVAL_FD : center;
    return timed(h, cls, [&] { return launch_eval(a, c.DP, c.family, center, fd, grad, st); });
}

// Times n launch variants of one pass: every variant once untimed (clocks
// and caches settle, so the first variant measured is not the coldest), then
// kTuneRounds rounds over the variants in turn, each launch between its own
// events; a variant's time is its fastest launch.
constexpr int kTuneRounds = 2;
template <class F>
static hipError_t time_variants(chisao_ctx *h, hipEvent_t e0, hipEvent_t e1, int n, F &&launch, float *ms_out) {
    hipError_t e = hipSuccess;
    for (int v = 0; v < n && e == hipSuccess; ++v) e = launch(v);
    for (int v = 0; v < n; ++v) ms_out[v] = 0.0f;
    for (int r = 0; r < kTuneRounds && e == hipSuccess; ++r)
        for (int v = 0; v < n && e == hipSuccess; ++v) {
            e = hipEventRecord(e0, h->stream);
            if (e == hipSuccess) e = launch(v);
            if (e == hipSuccess) e = hipEventRecord(e1, h->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e == hipSuccess && (r == 0 || ms < ms_out[v])) ms_out[v] = ms;
        }
    return e;
}

// The default variant 0 stays unless another is clearly faster than the one
// kept so far: near-ties are timing noise.
static int pick_variant(const float *ms, int n) {
    int best = 0;
    for (int v = 1; v < n; ++v)
        if (ms[v] < kTuneMargin * ms[best]) best = v;
    return best;
}

// Autotuner: per evaluation class, time each launch schedule on a value +
// gradient pass over every sample of the class's problems (the starting
// population; F and G are recomputed by the first cycle) and keep the
// fastest; then, for matrix-core classes with the adjoint gradient, time the
// direct launches in half tiles (16 points, one MFMA column block) under that
// schedule.  A class whose launches hold few full tiles leaves SIMDs idle,
// and half tiles double the waves.  Last, adjoint classes time the four
// schedules again on a smoothing-probe pass (M probes per sample), whose
// launches are the largest of a cycle and can rank the schedules differently
// (finite-difference classes keep the stencil pass's choice: a stencil probe
// pass would take seconds).  Every point's arithmetic is the same in every
// schedule and tile size, so results do not depend on the choice.
static int autotune(chisao_ctx *h) {
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    hipError_t e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(CHISAO_E_DEVICE, "hipEventCreate: %s", hipGetErrorString(e));
    }
    for (EvalClass &c : h->eclasses) {
        // the pass the class runs most: value and adjoint gradient, or the
        // central-difference stencils (a value-only pass is far shorter and
        // does not rank the schedules of the stencil launches)
        const bool adj = c.grad_mode == CHISAO_GRAD_ADJOINT, fd = !adj;
        EvalArgs a = base_args(h, c);
        a.vc_kind = kVcOne;
        a.F_out = adj ? h->D.F : nullptr;
        a.G_out = h->D.G;
        a.max_tiles = tile_bound(h, c, kVcOne, fd);
        e = time_variants(h, e0, e1, kTuneVariants, [&](int v) {
            a.order = kTuneOrder[v];
            a.grid_cap = kTuneCap[v];
            return launch_eval(a, c.DP, c.family, kDirect, fd, adj, h->stream);
        }, c.tune_ms);
        if (e != hipSuccess) break;
        const int best_v = pick_variant(c.tune_ms, kTuneVariants);
        c.order = kTuneOrder[best_v];
        c.grid_cap = kTuneCap[best_v];
        c.p_order = c.order;
        c.p_grid_cap = c.grid_cap;
        if (!adj) continue;
        if (c.DP != kAluDP && c.family < kFamClosed) {
            // full against half tiles under the chosen schedule
            float ms2[2];
            a.order = c.order;
            a.grid_cap = c.grid_cap;
            e = time_variants(h, e0, e1, 2, [&](int v) {
                a.half_tiles = v;
                return launch_eval(a, c.DP, c.family, kDirect, false, true, h->stream);
            }, ms2);
            if (e != hipSuccess) break;
            c.tune_full_ms = ms2[0];
            c.tune_half_ms = ms2[1];
            c.half = pick_variant(ms2, 2);
        }
        // the probe launches: every sample of the class's problems, probe
        // step 0 (sigma is still 0 at init: the probes sit on the samples,
        // the work is the same); the smoothed gradients land in scratch rows
        EvalArgs b = base_args(h, c);
        b.vc_kind = kVcProbes;
        b.max_tiles = tile_bound(h, c, kVcProbes, false);
        e = time_variants(h, e0, e1, kTuneVariants, [&](int v) {
            b.order = kTuneOrder[v];
            b.grid_cap = kTuneCap[v];
            return launch_eval(b, c.DP, c.family, kProbe, false, true, h->stream);
        }, c.tune_probe_ms);
        if (e != hipSuccess) break;
        const int pv = pick_variant(c.tune_probe_ms, kTuneVariants);
        c.p_order = kTuneOrder[pv];
        c.p_grid_cap = kTuneCap[pv];
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return fail(CHISAO_E_DEVICE, "autotuning launch failed: %s", hipGetErrorString(e));
    return CHISAO_OK;
}

// value and gradient of one class's samples on a list, on st: adjoint in one
// pass; with finite differences the value (if wanted) and the stencil gradient.  Values
// of noisy problems carry noise (sub-stream 0 for the value, fd_base plus the
// stencil index for the differences).
static hipError_t eval_list_class(chisao_ctx *h, const EvalClass &c, hipStream_t st, int list_id, float *F_out,
                                  float *G_out, bool want_f, int need_bit, int step_limit, int step, uint32_t fd_base) {
    EvalArgs a = base_args(h, c);
    a.list_id = list_id;
    a.vc_kind = kVcOne;
    a.need_bit = need_bit;
    a.step_limit = step_limit;
    a.step = step;
    a.nz_kind = 0;
    a.nz_base = 0;
    hipError_t e;
    if (c.grad_mode == CHISAO_GRAD_ADJOINT) {
        a.F_out = F_out;
        a.G_out = G_out;
        return run_eval(h, c, a, kDirect, false, true, st);
    }
    if (want_f) {
        a.F_out = F_out;
        a.G_out = nullptr;
        if ((e = run_eval(h, c, a, kDirect, false, false, st)) != hipSuccess) return e;
    }
    a.F_out = nullptr;
    a.G_out = G_out;
    a.nz_base = fd_base;
    return run_eval(h, c, a, kDirect, true, false, st);
}

// Iteration t of Phase 1 for one evaluation class, on the stream st (t runs
// to the class's own n_conv + 1, which closes the last iteration).
static hipError_t converge_iteration(chisao_ctx *h, const EvalClass &c, hipStream_t st, int t) {
    const Dev &D = h->D;
    const bool adj = c.grad_mode == CHISAO_GRAD_ADJOINT;
    hipError_t e;
    // the steppers of iteration t go to list_out; t+1 reads them back
    const int list_in = t == 1 ? L_ACT : ((t - 1) % 2 ? L_T1 : L_T1B);
    const int list_out = t % 2 ? L_T1 : L_T1B;
    if ((e = launch_reset_counts(D, (1 << list_out) | (1 << L_T2) | (1 << L_T3) | (1 << L_FD), st, c.pids_dev,
                                 (int)c.pids.size())) != hipSuccess)
        return e;
    if ((e = timed(h, CHISAO_PROF_LBFGS,
                   [&] { return launch_lbfgs_step(D, t, c.cpl, list_in, c.g0, c.n, st); })) != hipSuccess)
        return e;
    if (t > c.nconv) return hipSuccess;
    // (the L-BFGS step and history-pair tallies are kept only when profiling)
    if ((e = launch_compact(D, list_in, list_out, -1, false, h->prof ? D.prof + CHISAO_PROF_LBFGS : nullptr, st,
                            h->prof ? D.prof + CHISAO_PROF_LBFGS_PAIRS : nullptr, c.g0, c.n)) != hipSuccess)
        return e;
    // first trial t = 1 for every stepper
    {
        EvalArgs a = base_args(h, c);
        a.list_id = list_out;
        a.vc_kind = kVcTrialFirst;
        a.trial_next = L_T2;
        a.step = t;
        a.nz_kind = 0;
        if ((e = run_eval(h, c, a, kTrial, false, adj, st)) != hipSuccess) return e;
    }
    if ((e = launch_compact(D, list_out, L_T2, L_FD, true, nullptr, st, nullptr, c.g0, c.n)) != hipSuccess) return e;
    // the remaining trials in two stages: t = 1/2, 1/4, then the rest only
    // for searches that rejected those too.  Most searches that reject t = 1
    // accept one of the next two, so evaluating every remaining trial at once
    // would mostly compute points that are never used.
    for (int stage = 0; stage < 2; ++stage) {
        const int lst = stage ? L_T3 : L_T2;
        EvalArgs a = base_args(h, c);
        a.list_id = lst;
        a.vc_kind = kVcTrialRest;
        a.trial_lo = stage ? 3 : 1;
        a.trial_cnt = stage ? kMaxTrials : 2;
        a.trial_next = stage ? -1 : L_T3;
        a.step = t;
        a.nz_kind = 0;
        if ((e = run_eval(h, c, a, kTrial, false, adj, st)) != hipSuccess) return e;
        if ((e = launch_compact(D, lst, stage ? -1 : L_T3, L_FD, true, nullptr, st, nullptr, c.g0, c.n)) !=
            hipSuccess)
            return e;
    }
    if (!adj) {
        EvalArgs b = base_args(h, c);
        b.list_id = L_FD;
        b.vc_kind = kVcOne;
        b.G_out = D.G;
        b.step = t;
        b.nz_kind = 0;
        b.nz_base = kNzFd1;
        if ((e = run_eval(h, c, b, kDirect, true, false, st)) != hipSuccess) return e;
    }
    return hipSuccess;
}

// Phase 1.  The classes' problems share no samples, lists or counters, so
// each class runs its whole L-BFGS loop, for as many iterations as its
// problems need, on a stream of its own: in a captured cycle the classes are
// parallel chains that never wait for each other (one fork before, one join
// after).  The launches are enqueued iteration by iteration across the
// classes, so every chain has work queued from the start.  When profiling,
// everything runs in that order on the current stream.
static hipError_t phase_converge(chisao_ctx *h) {
    const Dev &D = h->D;
    hipError_t e;
    if ((e = launch_begin_cycle(D, h->cur)) != hipSuccess) return e;
    const size_t n = h->eclasses.size();
    const bool forked = forks(h, n);
    auto stream_of = [&](size_t i) { return branch(h, forked, i); };
    if (forked && (e = fork_open(h, n)) != hipSuccess) return e;
    int tmax = 0;
    for (size_t i = 0; i < n; ++i) {
        const EvalClass &c = h->eclasses[i];
        tmax = std::max(tmax, c.nconv + 1);
        if ((e = eval_list_class(h, c, stream_of(i), L_ACT, D.F, D.G, true, 0, 0, 0, kNzFd1)) != hipSuccess) return e;
    }
    for (int t = 1; t <= tmax; ++t)
        for (size_t i = 0; i < n; ++i)
            if (t <= h->eclasses[i].nconv + 1)
                if ((e = converge_iteration(h, h->eclasses[i], stream_of(i), t)) != hipSuccess) return e;
    // quality-gate values of noisy problems (the other problems have no jobs)
    if (h->any_noise)
        for (size_t i = 0; i < n; ++i) {
            const EvalClass &c = h->eclasses[i];
            EvalArgs a = base_args(h, c);
            a.list_id = L_ACT;
            a.vc_kind = kVcOne;
            a.F_out = D.Fg;
            a.nz_kind = 1;
            if ((e = run_eval(h, c, a, kDirect, false, false, stream_of(i))) != hipSuccess) return e;
        }
    return forked ? fork_close(h, n) : hipSuccess;
}

static int max_over(chisao_ctx *h, int ProblemDesc::*f) {
    int v = 0;
    for (const ProblemDesc &q : h->pdh) v = std::max(v, q.*f);
    return v;
}

// Phases 5 and 6 run as per-class chains, like Phase 1: a class's smoothing
// (or anti-convergence) steps read and write only its own problems' samples,
// lists and step lengths, so each class runs all of its steps on a stream of
// its own (one fork before the steps, one join after) instead of every step
// waiting for the slowest class.  The population statistics the steps start
// from (the unfrozen lists, sigma) are taken before the fork.
static hipError_t phase_hlc(chisao_ctx *h) {
    const Dev &D = h->D;
    hipError_t e;
    if ((e = launch_build_unfrozen(D, h->cur)) != hipSuccess) return e;
    if ((e = launch_sigma(D, h->cur)) != hipSuccess) return e;
    const size_t n = h->eclasses.size();
    const bool forked = forks(h, n);
    if (forked && (e = fork_open(h, n)) != hipSuccess) return e;
    const int n_cloud = max_over(h, &ProblemDesc::n_cloud);
    for (int step = 0; step < n_cloud; ++step)
        for (size_t i = 0; i < n; ++i) {
            const EvalClass &c = h->eclasses[i];
            const hipStream_t es = branch(h, forked, i);
            const int np = (int)c.pids.size();
            const bool adj = c.grad_mode == CHISAO_GRAD_ADJOINT;
            EvalArgs a = base_args(h, c);
            a.list_id = L_UNF;
            a.vc_kind = kVcProbes;
            a.step = step;
            a.need_bit = 1 << 5;
            a.step_limit = 1;
            a.nz_kind = adj ? -1 : 0;
            a.nz_base = kNzFdProbe;
            if ((e = run_eval(h, c, a, kProbe, !adj, adj, es)) != hipSuccess) return e;
            // (the finite-difference probes' mean; adjoint probes average in the kernel)
            if (!adj && (e = launch_probe_mean(D, step, es, c.pids_dev, np)) != hipSuccess) return e;
            if (step == 0 && (e = launch_step_size(D, D.Gh, 0, es, c.pids_dev, np)) != hipSuccess) return e;
            if ((e = launch_hlc_update(D, step, es, c.pids_dev, np)) != hipSuccess) return e;
        }
    return forked ? fork_close(h, n) : hipSuccess;
}

static hipError_t phase_anti(chisao_ctx *h) {
    const Dev &D = h->D;
    hipError_t e;
    const size_t n = h->eclasses.size();
    const bool forked = forks(h, n);
    if (forked && (e = fork_open(h, n)) != hipSuccess) return e;
    const int n_anti = max_over(h, &ProblemDesc::n_anti);
    for (int step = 0; step < n_anti; ++step)
        for (size_t i = 0; i < n; ++i) {
            const EvalClass &c = h->eclasses[i];
            const hipStream_t es = branch(h, forked, i);
            const int np = (int)c.pids.size();
            if ((e = eval_list_class(h, c, es, L_UNF, nullptr, D.Gh, false, 1 << 6, 2, step, kNzFdAnti)) !=
                hipSuccess)
                return e;
            if (step == 0 && (e = launch_step_size(D, D.Gh, 1, es, c.pids_dev, np)) != hipSuccess) return e;
            if ((e = launch_anti_update(D, step, es, c.pids_dev, np)) != hipSuccess) return e;
        }
    return forked ? fork_close(h, n) : hipSuccess;
}

static hipError_t enqueue_phases(chisao_ctx *h, uint32_t mask) {
    hipError_t e;
    const Dev &D = h->D;
    hipStream_t st = h->cur;
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

static hipError_t enqueue_cycle(chisao_ctx *h, bool last) {
    hipError_t e = enqueue_phases(h, last ? 0x0Eu : 0x7Eu);
    if (e != hipSuccess) return e;
    return launch_end_cycle(h->D, 1, h->cur);
}

// Capture one cycle (the kernels read every varying quantity, including the
// cycle index, from device memory) and instantiate it.
static int capture_cycle(chisao_ctx *h, bool last, hipGraphExec_t *out) {
    hipGraph_t g = nullptr;
    h->cur = h->cap;
    hipError_t e = hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t e2 = enqueue_cycle(h, last);
        e = hipStreamEndCapture(h->cap, &g);
        if (e2 != hipSuccess) e = e2;
    }
    h->cur = h->stream;
    if (e == hipSuccess) e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(CHISAO_E_DEVICE, "graph capture of a cycle failed: %s", hipGetErrorString(e));
    return CHISAO_OK;
}

extern "C" int chisao_run_phases(chisao_handle h, uint32_t phase_mask) {
    if (!h) return fail(CHISAO_E_INVAL, "null handle");
    HIP_TRY(hipSetDevice(h->device));
    h->cur = h->stream;
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
    const bool graphs = !(h->flags & CHISAO_FLAG_NO_GRAPH) && !h->prof;
    for (int i = 0; i < n_cycles; ++i) {
        const bool last = (h->k_host + 1 == h->D.n_osc);
        if (graphs) {
            hipGraphExec_t &g = h->graph[last ? 1 : 0];
            if (!g) {
                int rc = capture_cycle(h, last, &g);
                if (rc) return rc;
            }
            HIP_TRY(hipGraphLaunch(g, h->stream));
        } else {
            h->cur = h->stream;
            HIP_TRY(enqueue_cycle(h, last));
        }
        h->k_host += 1;
    }
    if (stats_host && n_cycles > 0) {
        const int P = h->D.P;
        std::vector<CycleRecord> rec((size_t)P * h->D.n_osc);
        HIP_TRY(hipMemcpyAsync(rec.data(), h->D.records, sizeof(CycleRecord) * rec.size(), hipMemcpyDeviceToHost,
                               h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
        for (int i = 0; i < n_cycles; ++i)
            for (int p = 0; p < P; ++p) {
                chisao_cycle_stats &o = stats_host[(size_t)i * P + p];
                const CycleRecord &r = rec[(size_t)p * h->D.n_osc + k0 + i];
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
                o.n_nonfinite = r.n_nonfinite;
                o.evals = (int64_t)r.evals;
            }
    }
    return CHISAO_OK;
}

// ---------------------------------------------------------------------------
// State, modes, evaluation, profiling
// ---------------------------------------------------------------------------
static int check_problem(chisao_ctx *h, int p) {
    if (p < 0 || p >= h->D.P) return fail(CHISAO_E_INVAL, "problem index %d out of range", p);
    return CHISAO_OK;
}

// rows [s0, s0+N) of a stride-DS device array to a dense host array of stride w
static hipError_t rows_d2h(void *dst, const void *src, size_t elem, size_t w, size_t DS, size_t s0, size_t N) {
    return hipMemcpy2D(dst, w * elem, (const char *)src + s0 * DS * elem, DS * elem, w * elem, N,
                       hipMemcpyDeviceToHost);
}

extern "C" int chisao_get_state(chisao_handle h, int problem, chisao_state *s) {
    if (!h || !s) return fail(CHISAO_E_INVAL, "null argument");
    int rc = check_problem(h, problem);
    if (rc) return rc;
    const Dev &D = h->D;
    const ProblemDesc &q = h->pdh[problem];
    const size_t N = q.N, d = q.d, DS = D.DS, s0 = q.s0, m = q.m, mx = D.mmax;
    HIP_TRY(hipSetDevice(h->device));
    HIP_TRY(hipStreamSynchronize(h->stream));
    if (s->X) HIP_TRY(rows_d2h(s->X, D.X, 4, d, DS, s0, N));
    if (s->F) HIP_TRY(hipMemcpy(s->F, D.F + s0, sizeof(float) * N, hipMemcpyDeviceToHost));
    if (s->G) HIP_TRY(rows_d2h(s->G, D.G, 4, d, DS, s0, N));
    if (s->stuck) HIP_TRY(hipMemcpy(s->stuck, D.stuck + s0, N, hipMemcpyDeviceToHost));
    if (s->active) HIP_TRY(hipMemcpy(s->active, D.active + s0, N, hipMemcpyDeviceToHost));
    if (s->stuck_pre) HIP_TRY(hipMemcpy(s->stuck_pre, D.stuck_pre + s0, N, hipMemcpyDeviceToHost));
    if (s->removed) HIP_TRY(hipMemcpy(s->removed, D.removed + s0, N, hipMemcpyDeviceToHost));
    if (s->trace)
        HIP_TRY(hipMemcpy2D(s->trace, N, D.trace + s0, (size_t)D.NT, N, (size_t)q.n_conv + 1, hipMemcpyDeviceToHost));
    if (s->S || s->Y) {
        std::vector<float> tmp(N * mx * DS);
        for (int which = 0; which < 2; ++which) {
            float *dst = which ? s->Y : s->S;
            if (!dst) continue;
            HIP_TRY(hipMemcpy(tmp.data(), (which ? D.Y : D.S) + s0 * mx * DS, sizeof(float) * tmp.size(),
                              hipMemcpyDeviceToHost));
            for (size_t i = 0; i < N; ++i)
                for (size_t j = 0; j < m; ++j)
                    memcpy(dst + (i * m + j) * d, tmp.data() + (i * mx + j) * DS, sizeof(float) * d);
        }
    }
    if (s->rho) HIP_TRY(rows_d2h(s->rho, D.rho, 4, m, mx, s0, N));
    if (s->head) HIP_TRY(hipMemcpy(s->head, D.head + s0, sizeof(int) * N, hipMemcpyDeviceToHost));
    if (s->cnt) HIP_TRY(hipMemcpy(s->cnt, D.cnt + s0, sizeof(int) * N, hipMemcpyDeviceToHost));
    if (s->conv) HIP_TRY(hipMemcpy(s->conv, D.conv + s0, N, hipMemcpyDeviceToHost));
    if (s->Fg) HIP_TRY(hipMemcpy(s->Fg, D.Fg + s0, sizeof(float) * N, hipMemcpyDeviceToHost));
    if (s->Wd) HIP_TRY(rows_d2h(s->Wd, D.Wd, 4, d, DS, s0, N));
    if (s->wvalid) HIP_TRY(hipMemcpy(s->wvalid, D.wvalid + s0, N, hipMemcpyDeviceToHost));
    Ctl c;
    HIP_TRY(hipMemcpy(&c, D.ctl + problem, sizeof c, hipMemcpyDeviceToHost));
    s->k = c.k;
    s->gr_disabled = c.gr_disabled;
    s->gr_fail = c.gr_fail;
    s->gr_used_last = c.gr_used_last;
    s->gr_prev_modes = c.gr_prev_modes;
    return CHISAO_OK;
}

extern "C" int chisao_set_state(chisao_handle h, int problem, const chisao_state *s) {
    if (!h || !s) return fail(CHISAO_E_INVAL, "null argument");
    int rc = check_problem(h, problem);
    if (rc) return rc;
    const Dev &D = h->D;
    const ProblemDesc &q = h->pdh[problem];
    const size_t N = q.N, d = q.d, DS = D.DS, s0 = q.s0;
    if (s->k < 0 || s->k > D.n_osc) return fail(CHISAO_E_INVAL, "k out of range");
    if (h->D.P > 1 && s->k != h->k_host) return fail(CHISAO_E_INVAL, "a batch keeps one cycle count for all problems");
    HIP_TRY(hipSetDevice(h->device));
    HIP_TRY(hipStreamSynchronize(h->stream));
    if (s->X) {
        std::vector<float> lo(d), hi(d);
        HIP_TRY(hipMemcpy(lo.data(), q.lo, sizeof(float) * d, hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(hi.data(), q.hi, sizeof(float) * d, hipMemcpyDeviceToHost));
        // NaN marks a sample whose objective cannot be evaluated (it leaves the
        // population at the next Phase 2); anything else must lie in the box
        for (size_t i = 0; i < N * d; ++i)
            if (!(isnan(s->X[i]) || (s->X[i] >= lo[i % d] && s->X[i] <= hi[i % d])))
                return fail(CHISAO_E_INVAL, "sample %zu lies outside the box", i / d);
        HIP_TRY(hipMemcpy2D(D.X + s0 * DS, DS * 4, s->X, d * 4, d * 4, N, hipMemcpyHostToDevice));
    }
    if (s->stuck) HIP_TRY(hipMemcpy(D.stuck + s0, s->stuck, N, hipMemcpyHostToDevice));
    if (s->active) HIP_TRY(hipMemcpy(D.active + s0, s->active, N, hipMemcpyHostToDevice));
    if (s->Wd) HIP_TRY(hipMemcpy2D(D.Wd + s0 * DS, DS * 4, s->Wd, d * 4, d * 4, N, hipMemcpyHostToDevice));
    if (s->wvalid) HIP_TRY(hipMemcpy(D.wvalid + s0, s->wvalid, N, hipMemcpyHostToDevice));
    Ctl c;
    HIP_TRY(hipMemcpy(&c, D.ctl + problem, sizeof c, hipMemcpyDeviceToHost));
    c.k = s->k;
    c.gr_disabled = s->gr_disabled;
    c.gr_fail = s->gr_fail;
    c.gr_used_last = s->gr_used_last;
    c.gr_prev_modes = s->gr_prev_modes;
    HIP_TRY(hipMemcpy(D.ctl + problem, &c, sizeof c, hipMemcpyHostToDevice));
    h->k_host = s->k;
    return CHISAO_OK;
}

extern "C" int chisao_modes(chisao_handle h, int problem, float *x_out, float *f_out, int cap, int *n_out) {
    if (!h || !n_out) return fail(CHISAO_E_INVAL, "null argument");
    int rc = check_problem(h, problem);
    if (rc) return rc;
    const Dev &D = h->D;
    const ProblemDesc &q = h->pdh[problem];
    HIP_TRY(hipSetDevice(h->device));
    HIP_TRY(launch_mode_list(D, problem, q.s0, q.N, h->stream));
    Ctl c;
    HIP_TRY(hipMemcpyAsync(&c, D.ctl + problem, sizeof c, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    const int n = c.count[O_PEAKS];
    *n_out = n;
    if (cap < n) return fail(CHISAO_E_RANGE, "capacity %d < %d modes", cap, n);
    if (n == 0) return CHISAO_OK;
    if (!x_out) return fail(CHISAO_E_INVAL, "null x_out");
    HIP_TRY(hipMemcpyAsync(x_out, D.Gh + (size_t)q.s0 * D.DS, sizeof(float) * (size_t)n * q.d, hipMemcpyDeviceToHost,
                           h->stream));
    if (f_out) HIP_TRY(hipMemcpyAsync(f_out, D.Pd + q.s0, sizeof(float) * (size_t)n, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return CHISAO_OK;
}

extern "C" int chisao_mode_widths(chisao_handle h, int problem, float *w_out, int cap, int *n_out) {
    if (!h || !n_out) return fail(CHISAO_E_INVAL, "null argument");
    int rc = check_problem(h, problem);
    if (rc) return rc;
    const Dev &D = h->D;
    const ProblemDesc &q = h->pdh[problem];
    HIP_TRY(hipSetDevice(h->device));
    HIP_TRY(launch_width_list(D, problem, q.N, h->stream));
    Ctl c;
    HIP_TRY(hipMemcpyAsync(&c, D.ctl + problem, sizeof c, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    const int n = c.count[O_PEAKS];
    *n_out = n;
    if (cap < n) return fail(CHISAO_E_RANGE, "capacity %d < %d modes", cap, n);
    if (n == 0) return CHISAO_OK;
    if (!w_out) return fail(CHISAO_E_INVAL, "null w_out");
    HIP_TRY(hipMemcpyAsync(w_out, D.Gh + (size_t)q.s0 * D.DS, sizeof(float) * (size_t)n * q.d, hipMemcpyDeviceToHost,
                           h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return CHISAO_OK;
}

// The launches of an evaluation on caller memory: value and adjoint gradient
// in one pass, or the value and the central-difference stencils.  `a` carries
// the device descriptors; results go to f_dev / G_dev (either may be null).
static hipError_t ext_eval_launches(EvalArgs a, int d, int DP, int family, const float *X_dev, int B, float *f_dev,
                                    float *G_dev, int grad_mode, hipStream_t st) {
    a.X = X_dev;
    a.x_stride = d;
    a.out_stride = d;
    a.ext_n = B;
    a.vc_kind = kVcOne;
    const long Vfd = 2 * d;
    hipError_t e;
    if (grad_mode == CHISAO_GRAD_ADJOINT) {
        a.F_out = f_dev;
        a.G_out = G_dev;
        a.max_tiles = (B + 31) / 32;
        return launch_eval(a, DP, family, kDirect, false, G_dev != nullptr, st);
    }
    if (f_dev) {
        a.F_out = f_dev;
        a.G_out = nullptr;
        a.max_tiles = (B + 31) / 32;
        if ((e = launch_eval(a, DP, family, kDirect, false, false, st)) != hipSuccess) return e;
    }
    if (G_dev) {
        a.F_out = nullptr;
        a.G_out = G_dev;
        a.max_tiles = Vfd <= 32 ? (B + (32 / Vfd) - 1) / (32 / Vfd) : (long)B * ((Vfd + 31) / 32);
        if ((e = launch_eval(a, DP, family, kDirect, true, false, st)) != hipSuccess) return e;
    }
    return hipSuccess;
}

extern "C" int chisao_eval(chisao_handle h, int problem, const float *X_dev, int B, float *f_dev, float *G_dev,
                           int grad_mode) {
    if (!h) return fail(CHISAO_E_INVAL, "null handle");
    int rc = check_problem(h, problem);
    if (rc) return rc;
    if (B < 0) return fail(CHISAO_E_INVAL, "negative batch");
    if (grad_mode != CHISAO_GRAD_FD && grad_mode != CHISAO_GRAD_ADJOINT) return fail(CHISAO_E_INVAL, "bad grad_mode");
    if (B == 0) return CHISAO_OK;
    if (!X_dev) return fail(CHISAO_E_INVAL, "null X");
    HIP_TRY(hipSetDevice(h->device));
    const ProblemDesc &q = h->pdh[problem];
    EvalClass c;
    c.DP = q.DP;
    c.family = q.family;
    c.grad_mode = grad_mode;
    c.pids = {problem};
    c.pids_dev = h->pid_seq + problem;
    HIP_TRY(ext_eval_launches(base_args(h, c), q.d, q.DP, q.family, X_dev, B, f_dev, G_dev, grad_mode, h->stream));
    return CHISAO_OK;
}

extern "C" int chisao_tuning(chisao_handle h, chisao_tuning_entry *out, int cap, int *n_out) {
    if (!h || !n_out) return fail(CHISAO_E_INVAL, "null argument");
    const int n = (int)h->eclasses.size();
    *n_out = n;
    if (cap < n) return fail(CHISAO_E_RANGE, "capacity %d < %d classes", cap, n);
    if (!out) return fail(CHISAO_E_INVAL, "null output");
    for (int i = 0; i < n; ++i) {
        const EvalClass &c = h->eclasses[i];
        chisao_tuning_entry &o = out[i];
        o.padded_d = c.DP;
        o.family = c.family;
        o.grad_mode = c.grad_mode;
        o.n_problems = (int)c.pids.size();
        o.order = c.order;
        o.grid_cap = c.grid_cap > 0 ? c.grid_cap : 8192;
        for (int v = 0; v < CHISAO_TUNE_VARIANTS; ++v) o.ms[v] = v < kTuneVariants ? c.tune_ms[v] : 0.0f;
        o.tile_points = c.DP == kAluDP ? kWave : (c.half ? 16 : 32);
        o.ms_half_tiles = c.tune_half_ms;
        o.ms_full_tiles = c.tune_full_ms;
        o.probe_order = c.p_order;
        o.probe_grid_cap = c.p_grid_cap > 0 ? c.p_grid_cap : 8192;
        for (int v = 0; v < CHISAO_TUNE_VARIANTS; ++v) o.ms_probe[v] = v < kTuneVariants ? c.tune_probe_ms[v] : 0.0f;
        o.trial_grid_cap = c.t_grid_cap;
    }
    return CHISAO_OK;
}

extern "C" int chisao_profile(chisao_handle h, int enable, chisao_kernel_profile *out) {
    if (!h) return fail(CHISAO_E_INVAL, "null handle");
    HIP_TRY(hipSetDevice(h->device));
    if (enable) {
        HIP_TRY(hipStreamSynchronize(h->stream));
        unsigned long long zero[kProfClasses] = {};
        HIP_TRY(hipMemcpy(h->D.prof, zero, sizeof zero, hipMemcpyHostToDevice));
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
        unsigned long long pts[kProfClasses];
        HIP_TRY(hipMemcpy(pts, h->D.prof, sizeof pts, hipMemcpyDeviceToHost));
        for (int i = 0; i < kProfClasses && i < CHISAO_PROF_CLASSES; ++i) res[i].points = (int64_t)pts[i];
        memcpy(out, res, sizeof res);
    }
    h->ev_used.clear();
    return CHISAO_OK;
}

// ---------------------------------------------------------------------------
// Evaluation without device allocation
//
// chisao_eval reads tables that chisao_init allocated: the fragment layouts of
// the precision matrices, the centres, the log normalisers and the problem
// descriptor.  chisao_eval_static builds the same tables for a problem given
// directly, in a fixed device array instead, and runs the same kernels.  The
// array is process-wide: each GPU holds one copy from library load to process
// exit, and every call on that GPU overwrites it.
// ---------------------------------------------------------------------------
namespace {
constexpr size_t kScratchBytes = (size_t)8 << 20;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_dev[kMaxDevices];  // device address of each GPU's copy, once looked up
}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// The device address of the current GPU's copy of `scratch`.  In host code the
// array's name is only a stand-in; the runtime gives each device's address,
// looked up once per device with that device current.
static int scratch_base(unsigned char **out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(CHISAO_E_DEVICE, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(CHISAO_E_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_dev[dev] = (unsigned char *)ptr;
    }
    *out = g_scratch_dev[dev];
    return CHISAO_OK;
}

extern "C" int chisao_eval_static(const chisao_problem *p, float fd_h, const float *X_dev, int B, float *f_dev,
                                  float *G_dev, int grad_mode, void *hip_stream) {
    int rc = validate_problem(p, 0);
    if (rc) return rc;
    if (B < 0) return fail(CHISAO_E_INVAL, "negative batch");
    if (grad_mode != CHISAO_GRAD_FD && grad_mode != CHISAO_GRAD_ADJOINT) return fail(CHISAO_E_INVAL, "bad grad_mode");
    if (!isfinite(fd_h)) return fail(CHISAO_E_INVAL, "non-finite fd_h");
    const bool closed = p->family >= CHISAO_RASTRIGIN;
    const size_t d = p->d, K = closed ? 0 : p->K, DP = pad_dim(p->d, p->family);
    // scratch layout: descriptors, then the tables, each section 256-byte aligned
    size_t used = 0;
    auto take = [&](size_t bytes) {
        const size_t at = used;
        used = (used + bytes + 255) & ~(size_t)255;
        return at;
    };
    const size_t o_pd = take(sizeof(ProblemDesc)), o_cls = take(sizeof(int)), o_ctl = take(sizeof(Ctl));
    const size_t o_bad = take(sizeof(int)), o_lo = take(4 * d), o_hi = take(4 * d);
    size_t o_pf = 0, o_mub = 0, o_lc = 0, o_w = 0, o_mu = 0, o_prec = 0;
    if (!closed) {
        o_pf = take(4 * K * DP * DP);
        o_mub = take(4 * K * DP);
        o_lc = take(4 * K);
        o_w = take(4 * K);
        o_mu = take(4 * K * d);
        o_prec = take(4 * K * d * d);
    }
    if (used > kScratchBytes)
        return fail(CHISAO_E_RANGE,
                    "problem tables need %zu bytes, more than the %zu-byte static scratch (K = %zu at d = %zu)", used,
                    kScratchBytes, K, d);
    if (B == 0) return CHISAO_OK;
    if (!X_dev) return fail(CHISAO_E_INVAL, "null X");
    unsigned char *base = nullptr;
    if ((rc = scratch_base(&base))) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    const float nu = p->family == CHISAO_STUDENT_T ? p->nu : 1.0f;
    ProblemDesc q;
    memset(&q, 0, sizeof q);
    q.d = p->d;
    q.DP = (int)DP;
    q.K = (int)K;
    q.family = p->family;
    q.nu = nu;
    q.nu_plus_d = nu + (float)p->d;
    q.Pfrag = closed ? nullptr : (const float *)(base + o_pf);
    q.muB = closed ? nullptr : (const float *)(base + o_mub);
    q.logc2 = closed ? nullptr : (const float *)(base + o_lc);
    q.lo = (const float *)(base + o_lo);
    q.hi = (const float *)(base + o_hi);
    q.N = B;
    q.fd_h = fd_h;
    q.noise_sigma = p->noise_sigma;  // recorded only: evaluations on caller memory carry no noise
    Ctl ctl;
    memset(&ctl, 0, sizeof ctl);
    const int zero = 0;
    // every section that must start at zero is written from the host: a fill
    // of the same bytes would also do, this keeps the call to copies only
    HIP_TRY(hipMemcpyAsync(base + o_pd, &q, sizeof q, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(base + o_cls, &zero, sizeof zero, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(base + o_ctl, &ctl, sizeof ctl, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(base + o_bad, &zero, sizeof zero, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(base + o_lo, p->lo, 4 * d, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(base + o_hi, p->hi, 4 * d, hipMemcpyHostToDevice, st));
    if (!closed) {
        HIP_TRY(hipMemcpyAsync(base + o_w, p->log_w, 4 * K, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(base + o_mu, p->mu, 4 * K * d, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(base + o_prec, p->prec, 4 * K * d * d, hipMemcpyHostToDevice, st));
        HIP_TRY(launch_prepare(p->family, p->d, (int)DP, p->K, nu, (const float *)(base + o_w),
                               (const float *)(base + o_mu), (const float *)(base + o_prec), (float *)(base + o_lc),
                               (float *)(base + o_pf), (float *)(base + o_mub), (int *)(base + o_bad), st));
    }
    // one synchronization: the host descriptors above stay alive until their
    // copies are done, and a matrix that is not positive definite is reported
    // before anything is evaluated
    int bad = 0;
    HIP_TRY(hipMemcpyAsync(&bad, base + o_bad, sizeof bad, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (bad) return fail(CHISAO_E_INVAL, "a precision matrix is not positive definite");
    EvalArgs a;
    memset(&a, 0, sizeof a);
    a.D.P = 1;
    a.D.NT = B;
    a.D.DS = (int)d;
    a.D.mmax = 1;
    a.D.Mmax = 1;
    a.D.pd = (const ProblemDesc *)(base + o_pd);
    a.D.ctl = (Ctl *)(base + o_ctl);
    a.cls = (const int *)(base + o_cls);
    a.n_cls = 1;
    a.list_id = -1;
    a.trial_next = -1;
    a.nz_kind = -1;
    HIP_TRY(ext_eval_launches(a, p->d, (int)DP, p->family, X_dev, B, f_dev, G_dev, grad_mode, st));
    return CHISAO_OK;
}
