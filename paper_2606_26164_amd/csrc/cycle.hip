// Kernels of the oscillation cycle other than the objective evaluation:
// L-BFGS directions and curvature pairs (Phase 1), the stick test (Phase 2),
// L-infinity deduplication (Phase 3), Repulse Monkey / Golden Rooster
// reseeding (Phase 4), the smoothing and anti-convergence updates (Phases
// 5-6), and the reductions that feed the data-dependent decisions.
//
// Every decision is taken on the device; reductions over samples use fixed
// block partitions and a fixed combination order, so results do not depend
// on scheduling.
#include <math.h>

#include "kernels.h"

namespace chisao {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;

static inline unsigned grid_for(long n, long per_block, long cap = 16384) {
    long g = (n + per_block - 1) / per_block;
    if (g < 1) g = 1;
    return (unsigned)(g < cap ? g : cap);
}

// ---------------------------------------------------------------------------
// small utilities
// ---------------------------------------------------------------------------
__global__ void fill_u8_kernel(uint8_t *p, uint8_t v, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

hipError_t launch_fill_u8(uint8_t *p, uint8_t v, size_t n, hipStream_t st) {
    hipLaunchKernelGGL(fill_u8_kernel, dim3(grid_for((long)n, kBlock)), dim3(kBlock), 0, st, p, v, n);
    return hipGetLastError();
}

__device__ __forceinline__ void append(const Dev &D, int id, int s) {
    const int slot = atomicAdd(&D.ctl->count[id], 1);
    list_ptr(D, id)[slot] = s;
}

// Uniform starting population in the box from the INIT stream.
__global__ void uniform_init_kernel(Dev D) {
    const int nb = (D.d + 3) / 4;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < (long)D.N * nb; e += (long)gridDim.x * blockDim.x) {
        const int s = (int)(e / nb), blk = (int)(e % nb);
        uint4 o = philox((uint32_t)s, 0u, kInit << 24, (uint32_t)blk, D.key0, D.key1);
        const uint32_t w[4] = {o.x, o.y, o.z, o.w};
        for (int q = 0; q < 4; ++q) {
            const int c = 4 * blk + q;
            if (c < D.d) D.X[(size_t)s * D.d + c] = D.lo[c] + u01(w[q]) * (D.hi[c] - D.lo[c]);
        }
    }
}

hipError_t launch_uniform_init(const Dev &D, hipStream_t st) {
    hipLaunchKernelGGL(uniform_init_kernel, dim3(grid_for((long)D.N * ((D.d + 3) / 4), kBlock)), dim3(kBlock), 0,
                       st, D);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Cycle start: release every sample (Phase 1 "release all"), empty the
// histories, and list the active samples.
// ---------------------------------------------------------------------------
__global__ void begin_ctl_kernel(Dev D) {
    Ctl *c = D.ctl;
    for (int i = 0; i < kNumLists; ++i) c->count[i] = 0;
    c->fmax_ord = float_to_ordered(-INFINITY);
    c->n_stuck = c->K_lost = c->n_modes = c->n_active = 0;
    c->reseed_kind = 0;
    c->ls_fail = 0;
    c->evals = 0;
    c->f_max = -INFINITY;
    c->sigma = c->alpha_c = c->alpha_a = 0.0f;
}

__global__ void begin_samples_kernel(Dev D) {
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < D.N; s += gridDim.x * blockDim.x) {
        D.stuck[s] = 0;
        D.removed[s] = 0;
        D.stuck_pre[s] = 0;
        D.conv[s] = 0;
        D.status[s] = 0;
        D.reset[s] = 0;
        D.steep[s] = 0;
        D.cnt[s] = 0;
        D.head[s] = D.m - 1;
        if (D.active[s]) {
            append(D, L_ACT, s);
            atomicAdd(&D.ctl->n_active, 1);
        }
    }
}

hipError_t launch_begin_cycle(const Dev &D, hipStream_t st) {
    hipLaunchKernelGGL(begin_ctl_kernel, dim3(1), dim3(1), 0, st, D);
    hipLaunchKernelGGL(begin_samples_kernel, dim3(grid_for(D.N, kBlock)), dim3(kBlock), 0, st, D);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_fill_u8(D.trace, kTrNone, (size_t)(D.n_conv + 1) * D.N, st);
}

__global__ void reset_counts_kernel(Dev D, int mask) {
    for (int i = 0; i < kNumLists; ++i)
        if (mask & (1 << i)) D.ctl->count[i] = 0;
}

hipError_t launch_reset_counts(const Dev &D, int mask, hipStream_t st) {
    hipLaunchKernelGGL(reset_counts_kernel, dim3(1), dim3(1), 0, st, D, mask);
    return hipGetLastError();
}

// Unfrozen list (active and not stuck) for Phases 5-6.
__global__ void build_unfrozen_kernel(Dev D) {
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < D.N; s += gridDim.x * blockDim.x)
        if (D.active[s] && !D.stuck[s]) append(D, L_UNF, s);
}

hipError_t launch_build_list(const Dev &D, int which, hipStream_t st) {
    if (which != L_UNF) return hipErrorInvalidValue;
    hipLaunchKernelGGL(reset_counts_kernel, dim3(1), dim3(1), 0, st, D, 1 << L_UNF);
    hipLaunchKernelGGL(build_unfrozen_kernel, dim3(grid_for(D.N, kBlock)), dim3(kBlock), 0, st, D);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Phase 1: one wave per sample, one lane per coordinate.
// Part A closes iteration t-1: curvature pair for F = -f
// (s = x - x_prev, y = -(g - g_prev)), stored when s'y > curv_eps |s||y|;
// a failed line search empties the history; the convergence flag is set when
// |g|_inf < eps_grad.  Part B opens iteration t: the two-loop recursion
// (newest to oldest, scale s'y/y'y of the newest pair, 1/max(|g|,1) without
// history), the ascent check, and the sample joins the first-trial list.
// ---------------------------------------------------------------------------
template <int MM>
__global__ __launch_bounds__(kBlock) void lbfgs_step_kernel(Dev D, int t) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x / kWave;
    const int d = D.d, m = D.m;
    const bool on = lane < d;
    for (int s = blockIdx.x * kWavesPerBlock + wv; s < D.N; s += gridDim.x * kWavesPerBlock) {
        if (!D.active[s]) continue;
        const size_t row = (size_t)s * d + lane;
        const float gv = on ? D.G[row] : 0.0f;
        int cnt = D.cnt[s], head = D.head[s];
        bool conv = D.conv[s] != 0;
        if (t == 1) {
            const float gi = wave_max(fabsf(gv));
            conv = gi < D.eps_grad;
            if (lane == 0) {
                D.ginf[s] = gi;
                D.conv[s] = conv;
                D.trace[s] = conv ? kTrConv : 0;
            }
        } else if (conv && D.conv[s] == 2) {
            // stalled: the failed search started from an empty history, so
            // every later iteration repeats it exactly and fails the same way
            if (lane == 0) D.trace[(size_t)(t - 1) * D.N + s] = kTrFail;
        } else {
            const uint8_t stt = D.status[s];
            if (stt != 0) {
                uint8_t code = D.reset[s] ? kTrReset : 0;
                if (stt & kStAccept) {
                    code |= (uint8_t)(stt & 0x0F);
                    const float sv = on ? D.X[row] - D.Xprev[row] : 0.0f;
                    const float yv = on ? -(gv - D.Gprev[row]) : 0.0f;
                    const float sy = wave_sum(sv * yv);
                    const float ss = wave_sum(sv * sv);
                    const float yy = wave_sum(yv * yv);
                    if (sy > D.curv_eps * sqrtf(ss) * sqrtf(yy) && sy != 0.0f) {
                        head = (head + 1) % m;
                        if (on) {
                            D.S[((size_t)s * m + head) * d + lane] = sv;
                            D.Y[((size_t)s * m + head) * d + lane] = yv;
                        }
                        if (lane == 0) D.rho[(size_t)s * m + head] = 1.0f / sy;
                        cnt = cnt < m ? cnt + 1 : m;
                        code |= kTrStored;
                    }
                } else {
                    code |= kTrFail;
                    cnt = 0;
                    head = m - 1;
                }
                const float gi = wave_max(fabsf(gv));
                const bool converged = gi < D.eps_grad;
                if (converged) code |= kTrConv;
                const bool stall = !converged && !(stt & kStAccept) && D.steep[s];
                conv = converged || stall;  // either way no further direction in this phase
                if (lane == 0) {
                    D.ginf[s] = gi;
                    D.conv[s] = converged ? 1 : (stall ? 2 : 0);
                    D.trace[(size_t)(t - 1) * D.N + s] = code;
                    D.status[s] = 0;
                    D.reset[s] = 0;
                    D.cnt[s] = cnt;
                    D.head[s] = head;
                }
            }
        }
        if (t > D.n_conv || conv) continue;
        if (lane == 0) atomicAdd(&D.ctl->prof_points[4], 1ull);
        // ---- two-loop recursion on registers ----
        float hs[MM], hy[MM], al[MM], rh[MM];
#pragma unroll
        for (int j = 0; j < MM; ++j) {
            hs[j] = hy[j] = 0.0f;
            rh[j] = 0.0f;
            if (j < cnt) {
                const int slot = (head - j + m) % m;
                if (on) {
                    hs[j] = D.S[((size_t)s * m + slot) * d + lane];
                    hy[j] = D.Y[((size_t)s * m + slot) * d + lane];
                }
                rh[j] = D.rho[(size_t)s * m + slot];
            }
        }
        float qv = -gv;
#pragma unroll
        for (int j = 0; j < MM; ++j) {
            al[j] = 0.0f;
            if (j < cnt) {
                al[j] = rh[j] * wave_sum(hs[j] * qv);
                qv -= al[j] * hy[j];
            }
        }
        const float gnorm = sqrtf(wave_sum(gv * gv));
        float gamma;
        if (cnt > 0) gamma = wave_sum(hs[0] * hy[0]) / wave_sum(hy[0] * hy[0]);
        else gamma = 1.0f / fmaxf(gnorm, 1.0f);
        float r = gamma * qv;
#pragma unroll
        for (int j = MM - 1; j >= 0; --j) {
            if (j < cnt) {
                const float b = rh[j] * wave_sum(hy[j] * r);
                r += hs[j] * (al[j] - b);
            }
        }
        float p = -r;
        const float gp = wave_sum(gv * p);
        bool rst = false;
        if (!(gp > 0.0f)) {
            rst = true;
            p = gv / fmaxf(gnorm, 1.0f);
        }
        if (on) D.Pd[row] = p;
        if (lane == 0) {
            D.steep[s] = (cnt == 0) || rst;
            if (rst) {
                D.cnt[s] = 0;
                D.head[s] = m - 1;
                D.reset[s] = 1;
            }
            append(D, L_T1, s);
        }
    }
}

hipError_t launch_lbfgs_step(const Dev &D, int t, hipStream_t st) {
    const dim3 grid(grid_for(D.N, kWavesPerBlock, 8192)), block(kBlock);
    if (D.m <= 8) hipLaunchKernelGGL(lbfgs_step_kernel<8>, grid, block, 0, st, D, t);
    else if (D.m <= 16) hipLaunchKernelGGL(lbfgs_step_kernel<16>, grid, block, 0, st, D, t);
    else hipLaunchKernelGGL(lbfgs_step_kernel<32>, grid, block, 0, st, D, t);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Phase 2: f_max over active samples, then the stick test.
// ---------------------------------------------------------------------------
__global__ void fmax_kernel(Dev D) {
    __shared__ float red[kBlock];
    float v = -INFINITY;
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < D.N; s += gridDim.x * blockDim.x)
        if (D.active[s]) v = fmaxf(v, D.F[s]);
    red[threadIdx.x] = v;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(&D.ctl->fmax_ord, float_to_ordered(red[0]));
}

__global__ void stick_kernel(Dev D) {
    const float fmax = ordered_to_float(D.ctl->fmax_ord);
    const float gate = fmax + D.log_delta;
    if (blockIdx.x == 0 && threadIdx.x == 0) D.ctl->f_max = fmax;
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < D.N; s += gridDim.x * blockDim.x) {
        if (!D.active[s]) continue;
        const bool st = (D.ginf[s] < D.eps_grad) && (D.F[s] >= gate);
        D.stuck_pre[s] = st;
        if (st) {
            append(D, L_STK, s);
            atomicAdd(&D.ctl->n_stuck, 1);
        }
    }
}

__global__ void stick_reset_kernel(Dev D) {
    D.ctl->count[L_STK] = 0;
    D.ctl->n_stuck = 0;
    D.ctl->fmax_ord = float_to_ordered(-INFINITY);
}

hipError_t launch_stick(const Dev &D, hipStream_t st) {
    const dim3 grid(grid_for(D.N, kBlock, 1024)), block(kBlock);
    hipLaunchKernelGGL(stick_reset_kernel, dim3(1), dim3(1), 0, st, D);
    hipLaunchKernelGGL(fmax_kernel, grid, block, 0, st, D);
    hipLaunchKernelGGL(stick_kernel, grid, block, 0, st, D);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Phase 3: sample j is removed when another stuck sample i lies within
// eps_dup in the sup-norm and ranks above it (higher f, then lower index).
// All stuck samples take part, removed or not.  Candidate first coordinates
// are staged through LDS; the full row is compared only when the first
// coordinates are within eps_dup.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void dedup_kernel(Dev D) {
    __shared__ float t_x0[kBlock];
    __shared__ float t_f[kBlock];
    __shared__ int t_i[kBlock];
    const int ns = D.ctl->count[L_STK];
    const int *lst = list_ptr(D, L_STK);
    const int d = D.d;
    const float eps = D.eps_dup;
    for (int base = blockIdx.x * kBlock; base < ns; base += gridDim.x * kBlock) {
        const int jj = base + threadIdx.x;
        const int j = jj < ns ? lst[jj] : -1;
        const float xj0 = j >= 0 ? D.X[(size_t)j * d] : 0.0f;
        const float fj = j >= 0 ? D.F[j] : 0.0f;
        bool rem = false;
        for (int tb = 0; tb < ns; tb += kBlock) {
            __syncthreads();
            const int ii = tb + threadIdx.x;
            if (ii < ns) {
                const int i = lst[ii];
                t_i[threadIdx.x] = i;
                t_x0[threadIdx.x] = D.X[(size_t)i * d];
                t_f[threadIdx.x] = D.F[i];
            }
            __syncthreads();
            const int nt = min(kBlock, ns - tb);
            if (j >= 0 && !rem) {
                for (int u = 0; u < nt; ++u) {
                    const int i = t_i[u];
                    if (i == j || !(fabsf(t_x0[u] - xj0) < eps)) continue;
                    const float fi = t_f[u];
                    if (!(fi > fj || (fi == fj && i < j))) continue;
                    bool near = true;
                    for (int c = 1; c < d && near; ++c)
                        near = fabsf(D.X[(size_t)i * d + c] - D.X[(size_t)j * d + c]) < eps;
                    if (near) {
                        rem = true;
                        break;
                    }
                }
            }
        }
        if (j >= 0 && rem) D.removed[j] = 1;
    }
}

__global__ void dedup_reset_kernel(Dev D) {
    D.ctl->K_lost = 0;
    D.ctl->n_modes = 0;
}

__global__ void clear_removed_kernel(Dev D) {
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < D.N; s += gridDim.x * blockDim.x) D.removed[s] = 0;
}

__global__ void dedup_finalize_kernel(Dev D) {
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < D.N; s += gridDim.x * blockDim.x) {
        const bool st = D.stuck_pre[s] && !D.removed[s];
        D.stuck[s] = st;
        if (D.removed[s]) atomicAdd(&D.ctl->K_lost, 1);
        if (st) atomicAdd(&D.ctl->n_modes, 1);
    }
}

// Golden Rooster generations: a generation that found no new peak counts
// as a failure; two in a row disable it for the rest of the run.
__global__ void gr_book_kernel(Dev D) {
    Ctl *c = D.ctl;
    if (c->gr_used_last) {
        if (c->n_modes <= c->gr_prev_modes) c->gr_fail += 1;
        else c->gr_fail = 0;
        if (c->gr_fail >= 2) c->gr_disabled = 1;
        c->gr_used_last = 0;
    }
}

hipError_t launch_dedup(const Dev &D, hipStream_t st) {
    hipLaunchKernelGGL(dedup_reset_kernel, dim3(1), dim3(1), 0, st, D);
    hipLaunchKernelGGL(clear_removed_kernel, dim3(grid_for(D.N, kBlock, 1024)), dim3(kBlock), 0, st, D);
    if ((D.phase_mask >> 3) & 1)
        hipLaunchKernelGGL(dedup_kernel, dim3(grid_for(D.N, kBlock, 2048)), dim3(kBlock), 0, st, D);
    hipLaunchKernelGGL(dedup_finalize_kernel, dim3(grid_for(D.N, kBlock, 1024)), dim3(kBlock), 0, st, D);
    hipLaunchKernelGGL(gr_book_kernel, dim3(1), dim3(1), 0, st, D);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Phase 4: reseeding.
// ---------------------------------------------------------------------------
// Ordered lists (ascending index) of the removed slots, the unfrozen samples
// and the surviving peaks, from one workgroup: per-thread contiguous chunks,
// exclusive scans of the chunk counts, then in-order writes.
constexpr int kScanThreads = 1024;

__global__ __launch_bounds__(kScanThreads) void ordered_lists_kernel(Dev D, int only_peaks) {
    __shared__ int sc[3][kScanThreads];
    if (!only_peaks && (D.ctl->K_lost == 0 || !((D.phase_mask >> 4) & 1))) return;
    const int tid = threadIdx.x;
    const int chunk = (D.N + kScanThreads - 1) / kScanThreads;
    const int b = tid * chunk, e = min(D.N, b + chunk);
    int c0 = 0, c1 = 0, c2 = 0;
    for (int s = b; s < e; ++s) {
        if (D.removed[s]) ++c0;
        else if (D.active[s] && !D.stuck[s]) ++c1;
        else if (D.active[s] && D.stuck[s]) ++c2;
    }
    sc[0][tid] = c0;
    sc[1][tid] = c1;
    sc[2][tid] = c2;
    __syncthreads();
    // inclusive Hillis-Steele scan on the three arrays
    for (int o = 1; o < kScanThreads; o <<= 1) {
        int v0 = 0, v1 = 0, v2 = 0;
        if (tid >= o) {
            v0 = sc[0][tid - o];
            v1 = sc[1][tid - o];
            v2 = sc[2][tid - o];
        }
        __syncthreads();
        sc[0][tid] += v0;
        sc[1][tid] += v1;
        sc[2][tid] += v2;
        __syncthreads();
    }
    int o0 = sc[0][tid] - c0, o1 = sc[1][tid] - c1, o2 = sc[2][tid] - c2;
    int *l0 = list_ptr(D, O_SLOTS), *l1 = list_ptr(D, O_FREE), *l2 = list_ptr(D, O_PEAKS);
    for (int s = b; s < e; ++s) {
        if (D.removed[s]) l0[o0++] = s;
        else if (D.active[s] && !D.stuck[s]) l1[o1++] = s;
        else if (D.active[s] && D.stuck[s]) l2[o2++] = s;
    }
    if (tid == kScanThreads - 1) {
        D.ctl->count[O_SLOTS] = sc[0][tid];
        D.ctl->count[O_FREE] = sc[1][tid];
        D.ctl->count[O_PEAKS] = sc[2][tid];
    }
}

// Repulse Monkey when at least five unfrozen samples remain, Golden Rooster
// otherwise (unless disabled), else the slots are taken out of use.
__global__ void reseed_decide_kernel(Dev D) {
    Ctl *c = D.ctl;
    if (c->K_lost == 0 || !((D.phase_mask >> 4) & 1)) {
        c->reseed_kind = 0;
        return;
    }
    if (c->count[O_FREE] >= 5) c->reseed_kind = 1;
    else if (!c->gr_disabled && c->count[O_PEAKS] > 0) c->reseed_kind = 2;
    else c->reseed_kind = 3;
}

// Shared ray step: x = o + frac * t_max * u, t_max the distance to the box
// boundary along u, then clamped to the box.
__device__ __forceinline__ void ray_fill(const Dev &D, int s, const float *o_row, float u, float frac, int lane) {
    const bool on = lane < D.d;
    float ratio = INFINITY;
    if (on) {
        const float o = o_row[lane];
        if (u > 0.0f) ratio = (D.hi[lane] - o) / u;
        else if (u < 0.0f) ratio = (D.lo[lane] - o) / u;
    }
    float tmax = wave_min(ratio);
    if (!(tmax >= 0.0f) || isinf(tmax)) tmax = 0.0f;
    if (on) {
        const float x = o_row[lane] + frac * tmax * u;
        D.X[(size_t)s * D.d + lane] = fminf(fmaxf(x, D.lo[lane]), D.hi[lane]);
    }
}

__global__ __launch_bounds__(kBlock) void rm_kernel(Dev D) {
    if (D.ctl->reseed_kind != 1) return;
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int nslots = D.ctl->count[O_SLOTS], nfree = D.ctl->count[O_FREE];
    const uint32_t k = (uint32_t)D.ctl->k + 1u;
    const int *slots = list_ptr(D, O_SLOTS), *freel = list_ptr(D, O_FREE);
    for (int j = blockIdx.x * kWavesPerBlock + wv; j < nslots; j += gridDim.x * kWavesPerBlock) {
        const int s = slots[j];
        const uint4 o4 = philox((uint32_t)s, k, kRM << 24, 0u, D.key0, D.key1);
        const int origin = freel[uint_below(o4.x, (uint32_t)nfree)];
        const float frac = u01(o4.y);
        float z[4];
        const int blk = lane >> 2;
        box_muller4(philox((uint32_t)s, k, (kRM << 24) | (1u << 16), (uint32_t)blk, D.key0, D.key1), z);
        const float zv = lane < D.d ? z[lane & 3] : 0.0f;
        const float nz = sqrtf(wave_sum(zv * zv));
        ray_fill(D, s, D.X + (size_t)origin * D.d, zv / nz, frac, lane);
    }
}

// Golden Rooster: slot j (ascending) takes peak j mod n_peaks and the
// direction (-1)^q Q[:, floor(q/2) mod d], q = floor(j / n_peaks), where Q is
// the orthogonal factor (diag R > 0) of a Gaussian d x d matrix drawn for the
// peak.  One wave per slot: Householder QR in LDS, then Q e_col is formed by
// applying the reflectors to e_col in reverse order.
__global__ __launch_bounds__(kWave) void gr_kernel(Dev D) {
    if (D.ctl->reseed_kind != 2) return;
    __shared__ float A[64 * 65];
    __shared__ float vn[64], alpha[64];
    const int lane = threadIdx.x;
    const int d = D.d, LDA = 65;
    const int nslots = D.ctl->count[O_SLOTS], np = D.ctl->count[O_PEAKS];
    const uint32_t k = (uint32_t)D.ctl->k + 1u;
    const int *slots = list_ptr(D, O_SLOTS), *peaks = list_ptr(D, O_PEAKS);
    for (int j = blockIdx.x; j < nslots; j += gridDim.x) {
        const int s = slots[j];
        const int q = j % np, use = j / np;
        const int col = (use / 2) % d;
        const float sgn = (use & 1) ? -1.0f : 1.0f;
        const int p = peaks[q];
        __syncthreads();
        for (int b = lane; b * 4 < d * d; b += kWave) {
            float z[4];
            box_muller4(philox((uint32_t)p, k, kGR << 24, (uint32_t)b, D.key0, D.key1), z);
            for (int t = 0; t < 4; ++t) {
                const int e = 4 * b + t;
                if (e < d * d) A[(e / d) * LDA + (e % d)] = z[t];
            }
        }
        __syncthreads();
        for (int c = 0; c < d; ++c) {
            // reflector for column c: v = A[c:, c] - alpha e_c, alpha = -sign(a_cc) |A[c:, c]|
            const float a = (lane >= c && lane < d) ? A[lane * LDA + c] : 0.0f;
            const float nrm = sqrtf(wave_sum(a * a));
            const float a0 = A[c * LDA + c];
            const float al = a0 > 0.0f ? -nrm : nrm;
            const float v = (lane == c) ? a - al : a;
            const float vv = wave_sum(v * v);
            __syncthreads();
            if (lane >= c && lane < d) A[lane * LDA + c] = v;  // keep v in place of the column
            if (lane == 0) {
                vn[c] = vv;
                alpha[c] = al;
            }
            __syncthreads();
            if (nrm != 0.0f && vv != 0.0f) {
                // apply to the remaining columns, one lane per column
                const int cc = lane;
                if (cc > c && cc < d) {
                    float dotv = 0.0f;
                    for (int i = c; i < d; ++i) dotv += A[i * LDA + c] * A[i * LDA + cc];
                    const float f = 2.0f * dotv / vv;
                    for (int i = c; i < d; ++i) A[i * LDA + cc] -= f * A[i * LDA + c];
                }
            }
            __syncthreads();
        }
        // y = H_0 H_1 ... H_{d-1} e_col
        float y = (lane == col) ? 1.0f : 0.0f;
        for (int c = d - 1; c >= 0; --c) {
            const float vv = vn[c];
            const float nrm_ok = (alpha[c] != 0.0f || vv != 0.0f) ? 1.0f : 0.0f;
            if (vv != 0.0f && nrm_ok != 0.0f) {
                const float v = (lane >= c && lane < d) ? A[lane * LDA + c] : 0.0f;
                const float f = 2.0f * wave_sum(v * y) / vv;
                y -= f * v;
            }
        }
        if (alpha[col] < 0.0f) y = -y;
        const float u = lane < d ? sgn * y : 0.0f;
        const uint4 o4 = philox((uint32_t)s, k, (kGR << 24) | (1u << 16), 0u, D.key0, D.key1);
        ray_fill(D, s, D.X + (size_t)p * d, u, u01(o4.x), lane);
    }
}

__global__ void reseed_finalize_kernel(Dev D) {
    const int kind = D.ctl->reseed_kind;
    if (kind == 0) return;
    const int nslots = D.ctl->count[O_SLOTS];
    const int *slots = list_ptr(D, O_SLOTS);
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < nslots; j += gridDim.x * blockDim.x) {
        const int s = slots[j];
        if (kind == 3) D.active[s] = 0;
        D.stuck[s] = 0;  // removed[] keeps the deduplication decisions until the next cycle
        D.cnt[s] = 0;
        D.head[s] = D.m - 1;
        for (int c = 0; c < D.d; ++c) D.V[(size_t)s * D.d + c] = 0.0f;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && kind == 2) {
        D.ctl->gr_used_last = 1;
        D.ctl->gr_prev_modes = D.ctl->n_modes;
    }
}

hipError_t launch_reseed(const Dev &D, hipStream_t st) {
    hipLaunchKernelGGL(ordered_lists_kernel, dim3(1), dim3(kScanThreads), 0, st, D, 0);
    hipLaunchKernelGGL(reseed_decide_kernel, dim3(1), dim3(1), 0, st, D);
    hipLaunchKernelGGL(rm_kernel, dim3(grid_for(D.N, kWavesPerBlock, 4096)), dim3(kBlock), 0, st, D);
    hipLaunchKernelGGL(gr_kernel, dim3(grid_for(D.N, 1, 4096)), dim3(kWave), 0, st, D);
    hipLaunchKernelGGL(reseed_finalize_kernel, dim3(grid_for(D.N, kBlock, 1024)), dim3(kBlock), 0, st, D);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Phase 5-6 scalars.  sigma: given, or sigma_c times the pooled standard
// deviation (root of the mean per-coordinate population variance) of the
// unfrozen samples.  Step lengths: sigma / mean |g|_2 over the unfrozen
// samples at the first step of each phase (a configured alpha overrides).
// Sums are taken in float64 over fixed sample ranges, then over ranges in
// order.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void sigma_partial_kernel(Dev D) {
    __shared__ double red[kWavesPerBlock][129];
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int chunk = (D.N + gridDim.x - 1) / gridDim.x;
    const int b = blockIdx.x * chunk, e = min(D.N, b + chunk);
    double sx = 0.0, sxx = 0.0, cnt = 0.0;
    for (int s = b + wv; s < e; s += kWavesPerBlock) {
        if (!(D.active[s] && !D.stuck[s])) continue;
        cnt += 1.0;
        if (lane < D.d) {
            const double x = D.X[(size_t)s * D.d + lane];
            sx += x;
            sxx += x * x;
        }
    }
    red[wv][lane] = sx;
    red[wv][64 + lane] = sxx;
    if (lane == 0) red[wv][128] = cnt;
    __syncthreads();
    if (wv == 0) {
        double a = 0.0, c2 = 0.0, n = 0.0;
        for (int w = 0; w < kWavesPerBlock; ++w) {
            a += red[w][lane];
            c2 += red[w][64 + lane];
            n += red[w][128];
        }
        double *part = D.part + (size_t)blockIdx.x * 129;
        part[lane] = a;
        part[64 + lane] = c2;
        if (lane == 0) part[128] = n;
    }
}

__global__ void sigma_final_kernel(Dev D, int nblocks) {
    const int lane = threadIdx.x;
    if (D.sigma_cfg > 0.0f) {
        if (lane == 0) D.ctl->sigma = D.sigma_cfg;
        return;
    }
    double a = 0.0, c2 = 0.0, n = 0.0;
    for (int b = 0; b < nblocks; ++b) {
        const double *part = D.part + (size_t)b * 129;
        a += part[lane];
        c2 += part[64 + lane];
        n += part[128];
    }
    double var = 0.0;
    if (n > 0.0 && lane < D.d) {
        const double mean = a / n;
        var = c2 / n - mean * mean;
        if (var < 0.0) var = 0.0;
    }
    // fixed-order sum of the 64 lane values
    __shared__ double v[64];
    v[lane] = var;
    __syncthreads();
    if (lane == 0) {
        double tot = 0.0;
        for (int i = 0; i < 64; ++i) tot += v[i];
        D.ctl->sigma = n > 0.0 ? (float)((double)D.sigma_c * sqrt(tot / D.d)) : 0.0f;
    }
}

hipError_t launch_sigma(const Dev &D, hipStream_t st) {
    if (D.sigma_cfg <= 0.0f)
        hipLaunchKernelGGL(sigma_partial_kernel, dim3(D.n_part_blocks), dim3(kBlock), 0, st, D);
    hipLaunchKernelGGL(sigma_final_kernel, dim3(1), dim3(64), 0, st, D, D.n_part_blocks);
    return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void norm_partial_kernel(Dev D, const float *Gs) {
    __shared__ double red[kWavesPerBlock][2];
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int chunk = (D.N + gridDim.x - 1) / gridDim.x;
    const int b = blockIdx.x * chunk, e = min(D.N, b + chunk);
    double acc = 0.0, cnt = 0.0;
    for (int s = b + wv; s < e; s += kWavesPerBlock) {
        if (!(D.active[s] && !D.stuck[s])) continue;
        const float gv = lane < D.d ? Gs[(size_t)s * D.d + lane] : 0.0f;
        const float nn = sqrtf(wave_sum(gv * gv));
        acc += (double)nn;
        cnt += 1.0;
    }
    if (lane == 0) {
        red[wv][0] = acc;
        red[wv][1] = cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, n = 0.0;
        for (int w = 0; w < kWavesPerBlock; ++w) {
            a += red[w][0];
            n += red[w][1];
        }
        D.part[(size_t)blockIdx.x * 2] = a;
        D.part[(size_t)blockIdx.x * 2 + 1] = n;
    }
}

__global__ void step_final_kernel(Dev D, int nblocks, int which) {
    double a = 0.0, n = 0.0;
    for (int b = 0; b < nblocks; ++b) {
        a += D.part[(size_t)b * 2];
        n += D.part[(size_t)b * 2 + 1];
    }
    float alpha;
    if (D.alpha > 0.0f) alpha = D.alpha;
    else {
        const double mean = n > 0.0 ? a / n : 0.0;
        alpha = mean > 0.0 ? (float)((double)D.ctl->sigma / mean) : 0.0f;
    }
    if (which == 0) D.ctl->alpha_c = alpha;
    else D.ctl->alpha_a = alpha;
}

hipError_t launch_step_size(const Dev &D, const float *Gsrc, int which, hipStream_t st) {
    if (D.alpha <= 0.0f) hipLaunchKernelGGL(norm_partial_kernel, dim3(D.n_part_blocks), dim3(kBlock), 0, st, D, Gsrc);
    else hipLaunchKernelGGL(reset_counts_kernel, dim3(1), dim3(1), 0, st, D, 0);
    hipLaunchKernelGGL(step_final_kernel, dim3(1), dim3(1), 0, st, D, D.alpha <= 0.0f ? D.n_part_blocks : 0, which);
    return hipGetLastError();
}

// Finite-difference smoothing: mean of the per-probe gradients, probe order.
__global__ void probe_mean_kernel(Dev D) {
    const int n = D.ctl->count[L_UNF];
    const int *lst = list_ptr(D, L_UNF);
    const float invM = 1.0f / (float)D.M;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < (long)n * D.d; e += (long)gridDim.x * blockDim.x) {
        const int s = lst[e / D.d], c = (int)(e % D.d);
        float acc = 0.0f;
        for (int mm = 0; mm < D.M; ++mm) acc += D.Gp[((size_t)s * D.M + mm) * D.d + c];
        D.Gh[(size_t)s * D.d + c] = acc * invM;
    }
}

hipError_t launch_probe_mean(const Dev &D, hipStream_t st) {
    hipLaunchKernelGGL(probe_mean_kernel, dim3(grid_for((long)D.N * D.d, kBlock, 8192)), dim3(kBlock), 0, st, D);
    return hipGetLastError();
}

// x <- clamp(x + alpha_c * smoothed gradient)
__global__ void hlc_update_kernel(Dev D) {
    const int n = D.ctl->count[L_UNF];
    const int *lst = list_ptr(D, L_UNF);
    const float a = D.ctl->alpha_c;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < (long)n * D.d; e += (long)gridDim.x * blockDim.x) {
        const int s = lst[e / D.d], c = (int)(e % D.d);
        const size_t o = (size_t)s * D.d + c;
        D.X[o] = fminf(fmaxf(D.X[o] + a * D.Gh[o], D.lo[c]), D.hi[c]);
    }
}

hipError_t launch_hlc_update(const Dev &D, hipStream_t st) {
    hipLaunchKernelGGL(hlc_update_kernel, dim3(grid_for((long)D.N * D.d, kBlock, 8192)), dim3(kBlock), 0, st, D);
    return hipGetLastError();
}

// v <- mu v - alpha_a g (v = 0 before the first step); x <- clamp(x + v)
__global__ void anti_update_kernel(Dev D, int step) {
    const int n = D.ctl->count[L_UNF];
    const int *lst = list_ptr(D, L_UNF);
    const float a = D.ctl->alpha_a;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < (long)n * D.d; e += (long)gridDim.x * blockDim.x) {
        const int s = lst[e / D.d], c = (int)(e % D.d);
        const size_t o = (size_t)s * D.d + c;
        const float v0 = step == 0 ? 0.0f : D.V[o];
        const float v = D.momentum * v0 - a * D.Gh[o];
        D.V[o] = v;
        D.X[o] = fminf(fmaxf(D.X[o] + v, D.lo[c]), D.hi[c]);
    }
}

hipError_t launch_anti_update(const Dev &D, int step, hipStream_t st) {
    hipLaunchKernelGGL(anti_update_kernel, dim3(grid_for((long)D.N * D.d, kBlock, 8192)), dim3(kBlock), 0, st, D,
                       step);
    return hipGetLastError();
}

// Cycle end: record the statistics of cycle k+1 and optionally advance k.
__global__ void end_cycle_kernel(Dev D, int advance) {
    Ctl *c = D.ctl;
    const int k = c->k;
    if (k < D.n_osc) {
        CycleRecord &r = D.records[k];
        r.k = k + 1;
        r.f_max = c->f_max;
        r.n_stuck = c->n_stuck;
        r.K_lost = c->K_lost;
        r.n_modes = c->n_modes;
        r.reseed_kind = c->reseed_kind;
        r.n_free = c->reseed_kind ? c->count[O_FREE] : 0;
        r.n_unfrozen = c->count[L_UNF];
        r.n_active = c->n_active;
        r.sigma = c->sigma;
        r.alpha_c = c->alpha_c;
        r.alpha_a = c->alpha_a;
        r.ls_fail = c->ls_fail;
        r.evals = c->evals;
    }
    if (advance) c->k = k + 1;
}

hipError_t launch_end_cycle(const Dev &D, int advance, hipStream_t st) {
    hipLaunchKernelGGL(end_cycle_kernel, dim3(1), dim3(1), 0, st, D, advance);
    return hipGetLastError();
}

// Mode export: ordered list of stuck active samples, rows gathered into Gh
// and values into Pd (both free between cycles).
__global__ void gather_modes_kernel(Dev D) {
    const int n = D.ctl->count[O_PEAKS];
    const int *lst = list_ptr(D, O_PEAKS);
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < (long)n * D.d; e += (long)gridDim.x * blockDim.x) {
        const int j = (int)(e / D.d), c = (int)(e % D.d);
        const int s = lst[j];
        D.Gh[(size_t)j * D.d + c] = D.X[(size_t)s * D.d + c];
        if (c == 0) D.Pd[j] = D.F[s];
    }
}

hipError_t launch_mode_list(const Dev &D, hipStream_t st) {
    hipLaunchKernelGGL(ordered_lists_kernel, dim3(1), dim3(kScanThreads), 0, st, D, 1);
    hipLaunchKernelGGL(gather_modes_kernel, dim3(grid_for((long)D.N * D.d, kBlock, 4096)), dim3(kBlock), 0, st, D);
    return hipGetLastError();
}

}  // namespace chisao
