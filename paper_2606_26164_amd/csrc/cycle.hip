// Kernels of the oscillation cycle other than the objective evaluation:
// L-BFGS directions and curvature pairs (Phase 1), the stick test (Phase 2),
// L-infinity deduplication (Phase 3), Repulse Monkey / Golden Rooster
// reseeding (Phase 4), the smoothing and anti-convergence updates (Phases
// 5-6), and the reductions that feed the data-dependent decisions.
//
// A launch covers every problem of the handle (Phase 1's L-BFGS steps, list
// resets and compactions: the problems of one evaluation class, whose samples
// form a contiguous range).  Kernels whose work is per
// problem use gridDim.y = P (block (x, p) works on problem p); reductions over
// a problem's samples use fixed block partitions of that problem and a fixed
// combination order, so results depend neither on scheduling nor on which
// other problems share the launch.  Every decision is taken on the device.
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

// Starting population from the INIT stream (counter = sample index within its
// problem): uniform in the box, or on rays through the box centre from its
// vertices, edge midpoints and face centres (structured ray seeding, Sec.
// 5.3; the layout of the draws is stated with CHISAO_FLAG_RAY_SEEDING).
__global__ void uniform_init_kernel(Dev D) {
    const int nb = (D.DS + 3) / 4;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < (long)D.NT * nb; e += (long)gridDim.x * blockDim.x) {
        const int s = (int)(e / nb), blk = (int)(e % nb);
        const ProblemDesc &pd = D.pd[D.pid[s]];
        if (4 * blk >= pd.d) continue;
        const uint32_t i = (uint32_t)(s - pd.s0);
        if (!pd.ray_seed) {
            uint4 o = philox(i, 0u, kInit << 24, (uint32_t)blk, pd.key0, pd.key1);
            const uint32_t w[4] = {o.x, o.y, o.z, o.w};
            for (int q = 0; q < 4; ++q) {
                const int c = 4 * blk + q;
                if (c < pd.d) D.X[(size_t)s * D.DS + c] = pd.lo[c] + u01(w[q]) * (pd.hi[c] - pd.lo[c]);
            }
            continue;
        }
        const uint4 a = philox(i, 0u, (kInit << 24) | 1u, 0u, pd.key0, pd.key1);
        const uint4 b = philox(i, 0u, (kInit << 24) | 1u, 1u, pd.key0, pd.key1);
        const uint32_t kind = uint_below(a.x, 3u);  // 0 vertex, 1 edge midpoint, 2 face centre
        const int ec = (int)uint_below(a.y, (uint32_t)pd.d);
        const float t = u01(a.z);
        for (int q = 0; q < 4; ++q) {
            const int c = 4 * blk + q;
            if (c >= pd.d) break;
            const float lo = pd.lo[c], w = pd.hi[c] - lo;
            const bool middle = (kind == 1u && c == ec) || (kind == 2u && c != ec);
            const bool up = (((c < 32 ? b.x : b.y) >> (c & 31)) & 1u) != 0u;
            D.X[(size_t)s * D.DS + c] = middle ? lo + 0.5f * w : (up ? pd.hi[c] - t * w : lo + t * w);
        }
    }
}

hipError_t launch_uniform_init(const Dev &D, hipStream_t st) {
    hipLaunchKernelGGL(uniform_init_kernel, dim3(grid_for((long)D.NT * ((D.DS + 3) / 4), kBlock)), dim3(kBlock), 0,
                       st, D);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Cycle start: release every sample (Phase 1 "release all"), empty the
// histories, and list the active samples.
// ---------------------------------------------------------------------------
__global__ void begin_ctl_kernel(Dev D) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= D.P) return;
    Ctl *c = &D.ctl[p];
    for (int i = 0; i < kNumLists; ++i) c->count[i] = 0;
    c->fmax_ord = float_to_ordered(-INFINITY);
    c->n_stuck = c->K_lost = c->n_modes = c->n_active = 0;
    c->reseed_kind = 0;
    c->ls_fail = 0;
    c->n_nonfinite = 0;
    c->evals = 0;
    c->f_max = -INFINITY;
    c->sigma = c->alpha_c = c->alpha_a = 0.0f;
}

__global__ void begin_samples_kernel(Dev D) {
    // the loop bound is uniform per wave: the list appends are wave-wide
    for (int b = blockIdx.x * blockDim.x; b < D.NT; b += gridDim.x * blockDim.x) {
        const int s = b + threadIdx.x;
        const bool in = s < D.NT;
        const int p = in ? D.pid[s] : 0;
        const bool act = in && D.active[s];
        if (in) {
            D.stuck[s] = 0;
            D.removed[s] = 0;
            D.stuck_pre[s] = 0;
            D.conv[s] = 0;
            D.status[s] = 0;
            D.reset[s] = 0;
            D.steep[s] = 0;
            D.cnt[s] = 0;
            D.head[s] = D.pd[p].m - 1;
        }
        wave_append(D, L_ACT, act, p, s);
        wave_claim(act, p, [&](int q) { return &D.ctl[q].n_active; });
    }
}

hipError_t launch_begin_cycle(const Dev &D, hipStream_t st) {
    hipLaunchKernelGGL(begin_ctl_kernel, dim3(grid_for(D.P, 64)), dim3(64), 0, st, D);
    hipLaunchKernelGGL(begin_samples_kernel, dim3(grid_for(D.NT, kBlock)), dim3(kBlock), 0, st, D);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_fill_u8(D.trace, kTrNone, (size_t)(D.n_conv_max + 1) * D.NT, st);
}

// the problems pids[0 .. np) (pids null: problems 0 .. np)
__global__ void reset_counts_kernel(Dev D, int mask, const int *pids, int np) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    const int p = pids ? pids[i] : i;
    for (int l = 0; l < kNumLists; ++l)
        if (mask & (1 << l)) D.ctl[p].count[l] = 0;
}

hipError_t launch_reset_counts(const Dev &D, int mask, hipStream_t st, const int *pids, int np) {
    const int n = pids ? np : D.P;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(reset_counts_kernel, dim3(grid_for(n, 64)), dim3(64), 0, st, D, mask, pids, n);
    return hipGetLastError();
}

// List compaction.  A block takes 256 consecutive list positions; per problem
// present among them (positions are grouped by problem, so usually one) it
// scans the flags with wave ballots and claims room in the destination list
// with one global atomic, instead of one atomic per producing wave: atomics on
// one address serialise in the L2, which made per-wave appends the dominant
// cost of the L-BFGS step.
__global__ __launch_bounds__(kBlock) void compact_kernel(Dev D, int src, int dst1, int dst2, int count_fail,
                                                         unsigned long long *tally, unsigned long long *tally_pairs,
                                                         int pos0, int pos1) {
    __shared__ int s_pmin;
    __shared__ int s_wc[3][kWavesPerBlock];
    __shared__ int s_base[3];
    // profile tallies, summed over the block and added to memory once at the
    // end: one counter hit by every wave of a large population serializes
    __shared__ unsigned long long s_tally, s_pairs;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
    const unsigned long long below = (1ull << lane) - 1ull;
    if (tid == 0) s_tally = s_pairs = 0ull;
    for (int b = pos0 + blockIdx.x * kBlock; b < pos1; b += gridDim.x * kBlock) {
        const int j = b + tid;
        int p = 0, v = 0, s = -1;
        if (j < pos1) {
            p = D.pid[j];
            if (j - D.pd[p].s0 < D.ctl[p].count[src]) {
                v = D.flag[j];
                if (v) s = D.lists[(size_t)src * D.NT + j];
            }
        }
        bool pending = v != 0;
        for (;;) {
            if (tid == 0) s_pmin = 0x7FFFFFFF;
            __syncthreads();
            if (pending) atomicMin(&s_pmin, p);
            __syncthreads();
            const int pl = s_pmin;
            if (pl == 0x7FFFFFFF) break;
            const bool mine = pending && p == pl;
            unsigned long long bal[3];
#pragma unroll
            for (int o = 0; o < 3; ++o) {
                bal[o] = __ballot(mine && v == o + 1);
                if (lane == 0) s_wc[o][w] = (int)__popcll(bal[o]);
            }
            __syncthreads();
            if (tid < 3) {
                int tot = 0;
                for (int k = 0; k < kWavesPerBlock; ++k) tot += s_wc[tid][k];
                int base = 0;
                if (tot > 0) {
                    const int dst = tid == 0 ? dst1 : (tid == 1 ? dst2 : -1);
                    if (dst >= 0) base = atomicAdd(&D.ctl[pl].count[dst], tot);
                    else if (tid == 2 && count_fail) atomicAdd(&D.ctl[pl].ls_fail, tot);
                    if (tid == 0 && tally) s_tally += (unsigned long long)tot;
                }
                s_base[tid] = base;
            }
            __syncthreads();
            if (mine && v <= 2) {
                const int dst = v == 1 ? dst1 : dst2;
                if (dst >= 0) {
                    int off = s_base[v - 1] + (int)__popcll(bal[v - 1] & below);
                    for (int k = 0; k < w; ++k) off += s_wc[v - 1][k];
                    list_ptr(D, dst, D.pd[pl].s0)[off] = s;
                }
            }
            // L-BFGS accounting: history pairs the steppers' two-loops used
            if (tally_pairs) {
                float cnt = (mine && v == 1) ? (float)D.cnt[s] : 0.0f;
                cnt = wave_sum(cnt);
                if (lane == 0 && cnt > 0.0f) atomicAdd(&s_pairs, (unsigned long long)cnt);
            }
            pending = pending && !mine;
            __syncthreads();
        }
    }
    __syncthreads();
    if (tid == 0 && tally && s_tally) atomicAdd(tally, s_tally);
    if (tid == 0 && tally_pairs && s_pairs) atomicAdd(tally_pairs, s_pairs);
}

hipError_t launch_compact(const Dev &D, int src, int dst1, int dst2, bool count_fail, unsigned long long *tally,
                          hipStream_t st, unsigned long long *tally_pairs, int g0, int n) {
    if (n < 0) {
        g0 = 0;
        n = D.NT;
    }
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(compact_kernel, dim3(grid_for(n, kBlock, 4096)), dim3(kBlock), 0, st, D, src, dst1, dst2,
                       (int)count_fail, tally, tally_pairs, g0, g0 + n);
    return hipGetLastError();
}

// Unfrozen list (active and not stuck) for Phases 5-6.
__global__ void build_unfrozen_kernel(Dev D) {
    for (int b = blockIdx.x * blockDim.x; b < D.NT; b += gridDim.x * blockDim.x) {
        const int s = b + threadIdx.x;
        const bool in = s < D.NT;
        wave_append(D, L_UNF, in && D.active[s] && !D.stuck[s], in ? D.pid[s] : 0, s);
    }
}

hipError_t launch_build_unfrozen(const Dev &D, hipStream_t st) {
    hipLaunchKernelGGL(reset_counts_kernel, dim3(grid_for(D.P, 64)), dim3(64), 0, st, D, 1 << L_UNF,
                       (const int *)nullptr, D.P);
    hipLaunchKernelGGL(build_unfrozen_kernel, dim3(grid_for(D.NT, kBlock)), dim3(kBlock), 0, st, D);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Phase 1: four samples per wave.  Sample r of a wave owns the 16 lanes of
// DPP row r and each lane CPL consecutive coordinates, so every dot product
// is a 16-lane DPP reduction (no LDS traffic) and the history stays in
// registers between the two loops.
// Part A closes iteration t-1: curvature pair for F = -f
// (s = x - x_prev, y = -(g - g_prev)), stored when s'y > curv_eps |s||y|;
// a failed line search empties the history; the convergence flag is set when
// |g|_inf < eps_grad.  Part B opens iteration t: the two-loop recursion
// (newest to oldest, scale s'y/y'y of the newest pair, 1/max(|g|,1) without
// history), the ascent check, and the sample joins the first-trial list.
// ---------------------------------------------------------------------------
template <int CPL>
__device__ __forceinline__ void row_load(const float *base, int d, int c0, bool ok, float v[CPL]) {
    // rows are DS floats apart; with DS a multiple of CPL every chunk that
    // starts inside the row lies inside it and is aligned, so it is read in
    // one vector access.  The row arrays are zeroed at creation and no writer
    // puts anything but zeros past d, so a chunk that straddles d reads zeros
    // there (a mask here would make every load wait before the next issues).
    if constexpr (CPL > 1) {
        if (ok && c0 < d) {
            if constexpr (CPL == 4) {
                const float4 w = *reinterpret_cast<const float4 *>(base + c0);
                v[0] = w.x; v[1] = w.y; v[2] = w.z; v[3] = w.w;
            } else {
                const float2 w = *reinterpret_cast<const float2 *>(base + c0);
                v[0] = w.x; v[1] = w.y;
            }
        } else {
#pragma unroll
            for (int i = 0; i < CPL; ++i) v[i] = 0.0f;
        }
    } else {
        v[0] = (ok && c0 < d) ? base[c0] : 0.0f;
    }
}
template <int CPL>
__device__ __forceinline__ void row_store(float *base, int d, int c0, bool ok, const float v[CPL]) {
    if (!ok || c0 >= d) return;
    if constexpr (CPL == 4) {
        *reinterpret_cast<float4 *>(base + c0) = make_float4(v[0], v[1], v[2], v[3]);
    } else if constexpr (CPL == 2) {
        *reinterpret_cast<float2 *>(base + c0) = make_float2(v[0], v[1]);
    } else {
        base[c0] = v[0];
    }
}
template <int CPL>
__device__ __forceinline__ float row_dot(const float a[CPL], const float b[CPL]) {
    float p = 0.0f;
#pragma unroll
    for (int i = 0; i < CPL; ++i) p = fmaf(a[i], b[i], p);
    return row16_sum(p);
}

template <int MM, int CPL>
__global__ __launch_bounds__(kBlock) void lbfgs_step_kernel(Dev D, int t, int list_in, int g0, int n) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x / kWave;
    const int rr = lane >> 4, l16 = lane & 15;
    const int c0 = l16 * CPL;
    const int DS = D.DS, mx = D.mmax;
    const int groups = (n + 3) / 4;
    for (int grp = blockIdx.x * kWavesPerBlock + wv; grp < groups; grp += gridDim.x * kWavesPerBlock) {
        // slot j of the list segment of problem pid[j] (segments start at s0)
        const int pos = g0 + grp * 4 + rr;
        int s = -1, p = 0;
        if (pos < g0 + n) {
            p = D.pid[pos];
            if (pos - D.pd[p].s0 < D.ctl[p].count[list_in]) s = D.lists[(size_t)list_in * D.NT + pos];
        }
        if (__ballot(s >= 0) == 0) continue;
        const bool act = s >= 0 && D.active[s];
        const ProblemDesc &pd = D.pd[p];
        const int d = pd.d, m = pd.m;
        const size_t row = (size_t)(act ? s : 0) * DS;
        float gv[CPL];
        row_load<CPL>(D.G + row, d, c0, act, gv);
        int cnt = act ? D.cnt[s] : 0, head = act ? D.head[s] : m - 1;
        const int cflag = act ? D.conv[s] : 1;
        bool done = cflag != 0;  // converged, stalled or inactive: no direction
        float gabs = 0.0f;
#pragma unroll
        for (int i = 0; i < CPL; ++i) gabs = fmaxf(gabs, fabsf(gv[i]));
        if (t == 1) {
            const float gi = row16_max(gabs);
            const bool converged = gi < pd.eps_grad;
            done = !act || converged;
            if (act && l16 == 0) {
                D.ginf[s] = gi;
                D.conv[s] = converged;
                D.trace[s] = converged ? kTrConv : 0;
            }
        } else {
            const uint8_t stt = act ? D.status[s] : 0;
            const bool accepted = (stt & kStAccept) != 0;
            float sv[CPL], yv[CPL];
            {
                float xa[CPL], xp[CPL], gp_[CPL];
                row_load<CPL>(D.X + row, d, c0, accepted, xa);
                row_load<CPL>(D.Xprev + row, d, c0, accepted, xp);
                row_load<CPL>(D.Gprev + row, d, c0, accepted, gp_);
#pragma unroll
                for (int i = 0; i < CPL; ++i) {
                    sv[i] = xa[i] - xp[i];
                    yv[i] = accepted ? -(gv[i] - gp_[i]) : 0.0f;
                }
            }
            const float sy = row_dot<CPL>(sv, yv);
            const float ss = row_dot<CPL>(sv, sv);
            const float yy = row_dot<CPL>(yv, yv);
            const float gi = row16_max(gabs);
            if (stt != 0) {
                uint8_t code = D.reset[s] ? kTrReset : 0;
                if (accepted) {
                    code |= (uint8_t)(stt & 0x0F);
                    if (sy > pd.curv_eps * sqrtf(ss) * sqrtf(yy) && sy != 0.0f) {
                        head = head + 1 == m ? 0 : head + 1;
                        const size_t slot = ((size_t)s * mx + head) * DS;
                        row_store<CPL>(D.S + slot, d, c0, true, sv);
                        row_store<CPL>(D.Y + slot, d, c0, true, yv);
                        if (l16 == 0) D.rho[(size_t)s * mx + head] = 1.0f / sy;
                        cnt = cnt < m ? cnt + 1 : m;
                        code |= kTrStored;
                    }
                } else {
                    code |= kTrFail;
                    cnt = 0;
                    head = m - 1;
                }
                const bool converged = gi < pd.eps_grad;
                if (converged) code |= kTrConv;
                // (with evaluation noise a repeated search draws fresh values)
                const bool stall = !converged && !accepted && D.steep[s] && !(pd.noise_sigma > 0.0f);
                done = converged || stall;
                if (l16 == 0) {
                    D.ginf[s] = gi;
                    D.conv[s] = converged ? 1 : (stall ? 2 : 0);
                    D.trace[(size_t)(t - 1) * D.NT + s] = code;
                    // the failed search started from an empty history: every
                    // later iteration would repeat it exactly and fail alike
                    if (stall)
                        for (int r = t; r <= pd.n_conv; ++r) D.trace[(size_t)r * D.NT + s] = kTrFail;
                    D.status[s] = 0;
                    D.reset[s] = 0;
                    D.cnt[s] = cnt;
                    D.head[s] = head;
                }
            }
        }
        // ---- two-loop recursion (all four rows take part in the reductions) --
        const bool go = !done && t <= pd.n_conv;
        if (__ballot(go) == 0) {
            if (s >= 0 && l16 == 0) D.flag[pos] = 0;
            continue;
        }
        const int cnt_go = go ? cnt : 0;
        const int cmax = (int)wave_max((float)cnt_go);
        float hs[MM][CPL], hy[MM][CPL], rh[MM], al[MM];
        // the sample's ring of pairs: one 64-bit base per row, 32-bit slot
        // offsets (slot j back from head wraps once: j < cnt <= m)
        const size_t hb = (size_t)(go ? s : 0) * mx;
        const float *Sb = D.S + hb * DS, *Yb = D.Y + hb * DS, *Rb = D.rho + hb;
#pragma unroll
        for (int j = 0; j < MM; ++j) {
            const bool ok = go && j < cnt;
            const int slot = ok ? (head >= j ? head - j : head - j + m) : 0;
            row_load<CPL>(Sb + slot * DS, d, c0, ok, hs[j]);
            row_load<CPL>(Yb + slot * DS, d, c0, ok, hy[j]);
            rh[j] = ok ? Rb[slot] : 0.0f;
        }
        float q[CPL];
#pragma unroll
        for (int i = 0; i < CPL; ++i) q[i] = -gv[i];
#pragma unroll
        for (int j = 0; j < MM; ++j) {
            al[j] = 0.0f;
            if (j < cmax) {
                al[j] = rh[j] * row_dot<CPL>(hs[j], q);
#pragma unroll
                for (int i = 0; i < CPL; ++i) q[i] -= al[j] * hy[j][i];
            }
        }
        const float gnorm = sqrtf(row_dot<CPL>(gv, gv));
        const float s0y0 = row_dot<CPL>(hs[0], hy[0]);
        const float y0y0 = row_dot<CPL>(hy[0], hy[0]);
        const float gamma = cnt_go > 0 ? s0y0 / y0y0 : 1.0f / fmaxf(gnorm, 1.0f);
        float rv[CPL];
#pragma unroll
        for (int i = 0; i < CPL; ++i) rv[i] = gamma * q[i];
#pragma unroll
        for (int j = MM - 1; j >= 0; --j) {
            if (j < cmax) {
                const float b = rh[j] * row_dot<CPL>(hy[j], rv);
#pragma unroll
                for (int i = 0; i < CPL; ++i) rv[i] += hs[j][i] * (al[j] - b);
            }
        }
        float pv[CPL];
#pragma unroll
        for (int i = 0; i < CPL; ++i) pv[i] = -rv[i];
        const float gp = row_dot<CPL>(gv, pv);
        const bool rst = !(gp > 0.0f);
        if (rst) {
#pragma unroll
            for (int i = 0; i < CPL; ++i) pv[i] = gv[i] / fmaxf(gnorm, 1.0f);
        }
        row_store<CPL>(D.Pd + row, d, c0, go, pv);
        if (go && l16 == 0) {
            D.steep[s] = (cnt == 0) || rst;
            if (rst) {
                D.cnt[s] = 0;
                D.head[s] = m - 1;
                D.reset[s] = 1;
            }
        }
        if (s >= 0 && l16 == 0) D.flag[pos] = go ? 1 : 0;
    }
}

template <int CPL>
static void launch_lbfgs_cpl(const Dev &D, int t, int li, int g0, int n, hipStream_t st) {
    const dim3 grid(grid_for((n + 3) / 4, kWavesPerBlock, 8192)), block(kBlock);
    if (D.mmax <= 4) hipLaunchKernelGGL((lbfgs_step_kernel<4, CPL>), grid, block, 0, st, D, t, li, g0, n);
    else if (D.mmax <= 8) hipLaunchKernelGGL((lbfgs_step_kernel<8, CPL>), grid, block, 0, st, D, t, li, g0, n);
    else if (D.mmax <= 12) hipLaunchKernelGGL((lbfgs_step_kernel<12, CPL>), grid, block, 0, st, D, t, li, g0, n);
    else if (D.mmax <= 16) hipLaunchKernelGGL((lbfgs_step_kernel<16, CPL>), grid, block, 0, st, D, t, li, g0, n);
    else hipLaunchKernelGGL((lbfgs_step_kernel<32, CPL>), grid, block, 0, st, D, t, li, g0, n);
}

hipError_t launch_lbfgs_step(const Dev &D, int t, int cpl, int list_in, int g0, int n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (cpl <= 1) launch_lbfgs_cpl<1>(D, t, list_in, g0, n, st);
    else if (cpl <= 2) launch_lbfgs_cpl<2>(D, t, list_in, g0, n, st);
    else launch_lbfgs_cpl<4>(D, t, list_in, g0, n, st);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Phase 2: f_max over a problem's active samples, then the stick test.
// ---------------------------------------------------------------------------
__global__ void stick_reset_kernel(Dev D) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= D.P) return;
    D.ctl[p].count[L_STK] = 0;
    D.ctl[p].n_stuck = 0;
    D.ctl[p].fmax_ord = float_to_ordered(-INFINITY);
    D.ctl[p].fmax_key = 0ull;
}

// A sample whose value, gate value or gradient is not finite leaves the
// population here, before f_max and every later reduction over samples.
__device__ __forceinline__ bool sample_finite(const Dev &D, const ProblemDesc &pd, int s) {
    bool ok = isfinite(D.F[s]) && isfinite(gate_values(D, pd)[s]);
    const float *g = D.G + (size_t)s * D.DS;
    for (int c = 0; c < pd.d; ++c) ok = ok && isfinite(g[c]);
    return ok;
}

// (value, lower index first) as one unsigned key: the largest key is the
// sample with the largest value, the lowest index among equal ones
__device__ __forceinline__ unsigned long long value_index_key(float v, int i) {
    const uint32_t ord = (uint32_t)float_to_ordered(v) ^ 0x80000000u;
    return ((unsigned long long)ord << 32) | (unsigned long long)(0xFFFFFFFFu - (uint32_t)i);
}

__global__ void fmax_kernel(Dev D) {
    __shared__ unsigned long long red[kBlock];
    const int p = blockIdx.y;
    const ProblemDesc &pd = D.pd[p];
    unsigned long long key = 0ull;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < pd.N; i += gridDim.x * blockDim.x) {
        const int s = pd.s0 + i;
        if (!D.active[s]) continue;
        if (sample_finite(D, pd, s)) {
            const unsigned long long k = value_index_key(gate_values(D, pd)[s], i);
            key = k > key ? k : key;
        } else {
            D.active[s] = 0;
            atomicAdd(&D.ctl[p].n_nonfinite, 1);
        }
    }
    red[threadIdx.x] = key;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o && red[threadIdx.x + o] > red[threadIdx.x]) red[threadIdx.x] = red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0 && red[0]) {
        atomicMax(&D.ctl[p].fmax_key, red[0]);
        atomicMax(&D.ctl[p].fmax_ord, float_to_ordered(gate_values(D, pd)[pd.s0 + (int)(0xFFFFFFFFu - (uint32_t)red[0])]));
    }
}

// Noisy problems: the largest gate value over many copies of one peak
// overestimates it by the largest of their noise terms, so f_max is the
// gate value of the best sample with its noise replaced by the mean of
// gate_reps new draws (GATE stream, sub-stream 1): an unbiased estimate of f
// there.  One thread per problem.
__global__ void fmax_redraw_kernel(Dev D) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= D.P) return;
    const ProblemDesc &pd = D.pd[p];
    const unsigned long long key = D.ctl[p].fmax_key;
    if (!(pd.noise_sigma > 0.0f) || key == 0ull) return;
    const int i = (int)(0xFFFFFFFFu - (uint32_t)key);
    const uint32_t kcyc = (uint32_t)D.ctl[p].k + 1u;
    float zs_old = 0.0f, zs_new = 0.0f;
    for (int b = 0; 4 * b < pd.gate_reps; ++b) {
        float zo[4], zn[4];
        box_muller4(philox((uint32_t)i, kcyc, kGate << 24, (uint32_t)b, pd.key0, pd.key1), zo);
        box_muller4(philox((uint32_t)i, kcyc, (kGate << 24) | 1u, (uint32_t)b, pd.key0, pd.key1), zn);
        for (int q = 0; q < 4 && 4 * b + q < pd.gate_reps; ++q) {
            zs_old += zo[q];
            zs_new += zn[q];
        }
    }
    const float R = (float)pd.gate_reps;
    const float fmax = D.Fg[pd.s0 + i] + pd.noise_sigma * (zs_new / R - zs_old / R);
    D.ctl[p].fmax_ord = float_to_ordered(fmax);
}

__global__ void stick_kernel(Dev D) {
    const int p = blockIdx.y;
    const ProblemDesc &pd = D.pd[p];
    const float fmax = ordered_to_float(D.ctl[p].fmax_ord);
    const float gate = fmax + pd.log_delta;
    if (blockIdx.x == 0 && threadIdx.x == 0) D.ctl[p].f_max = fmax;
    for (int b = blockIdx.x * blockDim.x; b < pd.N; b += gridDim.x * blockDim.x) {
        const int i = b + threadIdx.x, s = pd.s0 + i;
        const bool act = i < pd.N && D.active[s];
        const bool st = act && (D.ginf[s] < pd.eps_grad) && (gate_values(D, pd)[s] >= gate);
        if (act) D.stuck_pre[s] = st;
        wave_append(D, L_STK, st, p, s);
        wave_claim(st, p, [&](int q) { return &D.ctl[q].n_stuck; });
    }
}

hipError_t launch_stick(const Dev &D, hipStream_t st) {
    const dim3 grid(grid_for(D.NT / D.P + 1, kBlock, 256), D.P), block(kBlock);
    hipLaunchKernelGGL(stick_reset_kernel, dim3(grid_for(D.P, 64)), dim3(64), 0, st, D);
    hipLaunchKernelGGL(fmax_kernel, grid, block, 0, st, D);
    hipLaunchKernelGGL(fmax_redraw_kernel, dim3(grid_for(D.P, 64)), dim3(64), 0, st, D);
    hipLaunchKernelGGL(stick_kernel, grid, block, 0, st, D);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Phase 3: sample j is removed when another stuck sample i of its problem
// lies within eps_dup in the sup-norm and ranks above it (higher f, then
// lower index).  All stuck samples take part, removed or not.
// ---------------------------------------------------------------------------
// Deduplication through an L-infinity spatial hash (the hashing of
// Appendix A): j is removed iff some stuck sample i of its problem lies
// within eps_dup and ranks above it, (f_i, -i) > (f_j, -j).  The decision
// only asks whether such an i exists, so any candidate order gives the same
// answer; candidates come from j's own and the two adjacent hash cells, which
// makes the phase O(N) in the expected case instead of O(N^2).
//
// The hash is one fixed projection p(x) = sum_c v_c x_c with weights
// v_c = 1/2 + frac((c + 1) phi) (a Weyl sequence: no two coordinates weigh
// alike, so the distinct maxima of lattice-like landscapes, which share
// coordinate values, still land in different cells), cut into cells of width
// 2 eps |v|_1 (1 + 2^-20).  Two samples within eps in the sup-norm differ in
// p by less than eps |v|_1 (FP32 coordinate differences round by at most one
// ulp, inside the margin), so they lie in the same or adjacent cells.  p is
// formed in FP64: its rounding (~d 2^-53 |v|_1 max|x|) is far inside the
// margin.  Hashing every coordinate on its own grid instead would need 3^d
// neighbouring cells.
//
// Cells go to B = 2^hash_lb >= N/4 buckets by multiplicative hashing; a
// counting sort (count, exclusive scan, scatter) groups a problem's stuck
// samples by bucket in its L_HASH list.  Buckets may hold several cells; a
// candidate is compared only when its cell is the one being visited.
__device__ __forceinline__ double hash_weight(int c) {
    const double w = (double)(c + 1) * 0.61803398874989484820;
    return 0.5 + (w - floor(w));
}

// cell of row x; clamping to the int range keeps adjacent cells adjacent
__device__ __forceinline__ int hash_cell(const float *x, int d, double inv_width) {
    double p = 0.0;
    for (int c = 0; c < d; ++c) p += hash_weight(c) * (double)x[c];
    const double q = floor(p * inv_width);
    return (int)fmin(fmax(q, -2147483647.0), 2147483646.0);
}

__device__ __forceinline__ double hash_inv_width(int d, float eps) {
    double v1 = 0.0;
    for (int c = 0; c < d; ++c) v1 += hash_weight(c);
    return 1.0 / (2.0 * (double)eps * v1 * (1.0 + 0x1p-20));
}

__device__ __forceinline__ uint32_t hash_bucket(int cell, int lb) {
    return lb == 0 ? 0u : ((uint32_t)cell * 0x9E3779B1u) >> (32 - lb);
}

__global__ void dedup_clear_kernel(Dev D) {
    const int p = blockIdx.y;
    const ProblemDesc &pd = D.pd[p];
    int *cnt = D.hoff + pd.hk0;
    const int nb = (1 << pd.hash_lb) + 1;
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += gridDim.x * blockDim.x) cnt[b] = 0;
}

__global__ void dedup_count_kernel(Dev D) {
    const int p = blockIdx.y;
    const ProblemDesc &pd = D.pd[p];
    if (!((pd.phase_mask >> 3) & 1)) return;
    const int ns = D.ctl[p].count[L_STK];
    const int *lst = list_ptr(D, L_STK, pd.s0);
    const double inv_w = hash_inv_width(pd.d, pd.eps_dup);
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < ns; t += gridDim.x * blockDim.x) {
        const int s = lst[t];
        const int cell = hash_cell(D.X + (size_t)s * D.DS, pd.d, inv_w);
        D.hcell[s] = cell;
        atomicAdd(&D.hoff[pd.hk0 + hash_bucket(cell, pd.hash_lb)], 1);
    }
}

// exclusive scan of the bucket counts, one workgroup per problem; the
// scatter cursors start as a copy of the offsets
constexpr int kScanBlock = 1024;
__global__ __launch_bounds__(kScanBlock) void dedup_offsets_kernel(Dev D) {
    __shared__ int part[kScanBlock];
    const int p = blockIdx.x;
    const ProblemDesc &pd = D.pd[p];
    if (!((pd.phase_mask >> 3) & 1)) return;
    int *off = D.hoff + pd.hk0, *cur = D.hcur + pd.hk0;
    const int nb = 1 << pd.hash_lb;
    int carry = 0;
    for (int b0 = 0; b0 < nb; b0 += kScanBlock) {
        const int b = b0 + threadIdx.x;
        const int v = b < nb ? off[b] : 0;
        part[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < kScanBlock; o <<= 1) {
            const int add = (int)threadIdx.x >= o ? part[threadIdx.x - o] : 0;
            __syncthreads();
            part[threadIdx.x] += add;
            __syncthreads();
        }
        const int excl = carry + part[threadIdx.x] - v;
        if (b < nb) {
            off[b] = excl;
            cur[b] = excl;
        }
        carry += part[kScanBlock - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) off[nb] = carry;
}

__global__ void dedup_scatter_kernel(Dev D) {
    const int p = blockIdx.y;
    const ProblemDesc &pd = D.pd[p];
    if (!((pd.phase_mask >> 3) & 1)) return;
    const int ns = D.ctl[p].count[L_STK];
    const int *lst = list_ptr(D, L_STK, pd.s0);
    int *ent = list_ptr(D, L_HASH, pd.s0);
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < ns; t += gridDim.x * blockDim.x) {
        const int s = lst[t];
        const int pos = atomicAdd(&D.hcur[pd.hk0 + hash_bucket(D.hcell[s], pd.hash_lb)], 1);
        ent[pos] = s;
    }
}

// One wave per stuck sample: the lanes go through the candidates of a bucket
// 64 at a time, so the few samples whose buckets hold a whole cluster of
// converged copies (the best copy of a cluster finds no better one and
// checks them all) do not serialise the phase.
__global__ __launch_bounds__(kBlock) void dedup_scan_kernel(Dev D) {
    const int p = blockIdx.y;
    const ProblemDesc &pd = D.pd[p];
    if (!((pd.phase_mask >> 3) & 1)) return;
    const int ns = D.ctl[p].count[L_STK];
    const int *lst = list_ptr(D, L_STK, pd.s0);
    const int *ent = list_ptr(D, L_HASH, pd.s0);
    const int *off = D.hoff + pd.hk0;
    const float *Fv = gate_values(D, pd);
    const int d = pd.d, DS = D.DS;
    const float eps = pd.eps_dup;
    const int lane = threadIdx.x % kWave;
    const int wpb = blockDim.x / kWave;
    for (int t = blockIdx.x * wpb + threadIdx.x / kWave; t < ns; t += gridDim.x * wpb) {
        const int j = lst[t];
        const int cj = D.hcell[j];
        const float fj = Fv[j];
        const float *xj = D.X + (size_t)j * DS;
        bool rem = false;
        for (int dc = -1; dc <= 1 && !rem; ++dc) {
            const int c = cj + dc;
            const uint32_t b = hash_bucket(c, pd.hash_lb);
            const int q1 = off[b + 1];
            for (int q0 = off[b]; q0 < q1 && !rem; q0 += kWave) {
                const int q = q0 + lane;
                bool hit = false;
                if (q < q1) {
                    const int i = ent[q];
                    const float fi = Fv[i];
                    if (D.hcell[i] == c && i != j && (fi > fj || (fi == fj && i < j))) {
                        const float *xi = D.X + (size_t)i * DS;
                        hit = true;
                        for (int k = 0; k < d && hit; ++k) hit = fabsf(xi[k] - xj[k]) < eps;
                    }
                }
                rem = __any(hit);
            }
        }
        if (rem && lane == 0) D.removed[j] = 1;
    }
}

__global__ void dedup_reset_kernel(Dev D) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= D.P) return;
    D.ctl[p].K_lost = 0;
    D.ctl[p].n_modes = 0;
}

__global__ void clear_removed_kernel(Dev D) {
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < D.NT; s += gridDim.x * blockDim.x) D.removed[s] = 0;
}

__global__ void dedup_finalize_kernel(Dev D) {
    for (int b = blockIdx.x * blockDim.x; b < D.NT; b += gridDim.x * blockDim.x) {
        const int s = b + threadIdx.x;
        const bool in = s < D.NT;
        const bool rm = in && D.removed[s];
        const bool st = in && D.stuck_pre[s] && !rm;
        if (in) D.stuck[s] = st;
        const int p = in ? D.pid[s] : 0;
        wave_claim(rm, p, [&](int q) { return &D.ctl[q].K_lost; });
        wave_claim(st, p, [&](int q) { return &D.ctl[q].n_modes; });
    }
}

// Width export.  The survivor of deduplication keeps its inverse-Hessian
// estimate for width estimation (Phase 3): H approximates the inverse
// Hessian of F = -f from the sample's L-BFGS pairs, and diag(H) is kept.  H
// is formed by the BFGS recursion
//   H <- H - rho (H y s^T + s y^T H) + (rho^2 y^T H y + rho) s s^T
// over the pairs from oldest to newest, from gamma I with gamma = s'y / y'y
// of the newest pair (the two-loop's initial matrix), held in LDS by one
// workgroup per survivor.  Only survivors whose pairs come from this cycle's
// Phase 1 are recomputed: a sample that was stuck before is released with an
// empty history and sticks again without a step, so it keeps the diagonal it
// had; a survivor that never had a pair gets gamma0 = 1 / max(|g|_2, 1).
constexpr int kWidthBlock = 256;
__global__ __launch_bounds__(kWidthBlock) void width_kernel(Dev D) {
    __shared__ float H[64 * 64];
    __shared__ float sv[64], yv[64], wv[64];
    __shared__ float red[kWidthBlock];
    const int tid = threadIdx.x;
    for (int s = blockIdx.x; s < D.NT; s += gridDim.x) {
        if (!(D.stuck[s] && D.active[s])) continue;
        const ProblemDesc &pd = D.pd[D.pid[s]];
        if (!((pd.phase_mask >> 3) & 1)) continue;
        const int d = pd.d, m = pd.m, cnt = D.cnt[s], head = D.head[s];
        const size_t mx = (size_t)D.mmax;
        float *wrow = D.Wd + (size_t)s * D.DS;
        if (cnt == 0) {
            if (D.wvalid[s]) continue;
            float g2 = 0.0f;
            for (int c = tid; c < d; c += kWidthBlock) g2 += D.G[(size_t)s * D.DS + c] * D.G[(size_t)s * D.DS + c];
            red[tid] = g2;
            __syncthreads();
            for (int o = kWidthBlock / 2; o > 0; o >>= 1) {
                if (tid < o) red[tid] += red[tid + o];
                __syncthreads();
            }
            const float gamma0 = 1.0f / fmaxf(sqrtf(red[0]), 1.0f);
            for (int c = tid; c < d; c += kWidthBlock) wrow[c] = gamma0;
            if (tid == 0) D.wvalid[s] = 1;
            __syncthreads();
            continue;
        }
        // gamma from the newest pair
        {
            const size_t off = ((size_t)s * mx + head) * D.DS;
            float a = 0.0f, b = 0.0f;
            for (int c = tid; c < d; c += kWidthBlock) {
                const float y = D.Y[off + c];
                a += D.S[off + c] * y;
                b += y * y;
            }
            red[tid] = a;
            __syncthreads();
            for (int o = kWidthBlock / 2; o > 0; o >>= 1) {
                if (tid < o) red[tid] += red[tid + o];
                __syncthreads();
            }
            const float sy = red[0];
            __syncthreads();
            red[tid] = b;
            __syncthreads();
            for (int o = kWidthBlock / 2; o > 0; o >>= 1) {
                if (tid < o) red[tid] += red[tid + o];
                __syncthreads();
            }
            const float gamma = sy / red[0];
            for (int e = tid; e < d * d; e += kWidthBlock) H[e] = (e / d == e % d) ? gamma : 0.0f;
            __syncthreads();
        }
        for (int k = cnt - 1; k >= 0; --k) {
            const int slot = (head - k + m) % m;
            const size_t off = ((size_t)s * mx + slot) * D.DS;
            const float rho = D.rho[(size_t)s * mx + slot];
            for (int c = tid; c < d; c += kWidthBlock) {
                sv[c] = D.S[off + c];
                yv[c] = D.Y[off + c];
            }
            __syncthreads();
            // w = H y
            for (int r = tid; r < d; r += kWidthBlock) {
                float acc = 0.0f;
                for (int c = 0; c < d; ++c) acc += H[r * d + c] * yv[c];
                wv[r] = acc;
            }
            __syncthreads();
            float yw = 0.0f;
            for (int c = 0; c < d; ++c) yw += yv[c] * wv[c];
            const float coef = rho * rho * yw + rho;
            for (int e = tid; e < d * d; e += kWidthBlock) {
                const int r = e / d, c = e % d;
                H[e] += -rho * (wv[r] * sv[c] + sv[r] * wv[c]) + coef * sv[r] * sv[c];
            }
            __syncthreads();
        }
        for (int c = tid; c < d; c += kWidthBlock) wrow[c] = H[c * d + c];
        if (tid == 0) D.wvalid[s] = 1;
        __syncthreads();
    }
}

// Golden Rooster generations: a generation that found no new peak counts
// as a failure; two in a row disable it for the rest of the run.
__global__ void gr_book_kernel(Dev D) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= D.P) return;
    Ctl *c = &D.ctl[p];
    if (c->gr_used_last) {
        if (c->n_modes <= c->gr_prev_modes) c->gr_fail += 1;
        else c->gr_fail = 0;
        if (c->gr_fail >= 2) c->gr_disabled = 1;
        c->gr_used_last = 0;
    }
}

hipError_t launch_dedup(const Dev &D, hipStream_t st) {
    hipLaunchKernelGGL(dedup_reset_kernel, dim3(grid_for(D.P, 64)), dim3(64), 0, st, D);
    hipLaunchKernelGGL(clear_removed_kernel, dim3(grid_for(D.NT, kBlock, 1024)), dim3(kBlock), 0, st, D);
    const dim3 per_sample(grid_for(D.NT / D.P + 1, kBlock, 256), D.P);
    const dim3 per_wave(grid_for(D.NT / D.P + 1, kBlock / kWave, 4096), D.P);
    hipLaunchKernelGGL(dedup_clear_kernel, dim3(grid_for(D.NT / D.P + 2, kBlock, 256), D.P), dim3(kBlock), 0, st, D);
    hipLaunchKernelGGL(dedup_count_kernel, per_sample, dim3(kBlock), 0, st, D);
    hipLaunchKernelGGL(dedup_offsets_kernel, dim3(D.P), dim3(kScanBlock), 0, st, D);
    hipLaunchKernelGGL(dedup_scatter_kernel, per_sample, dim3(kBlock), 0, st, D);
    hipLaunchKernelGGL(dedup_scan_kernel, per_wave, dim3(kBlock), 0, st, D);
    hipLaunchKernelGGL(dedup_finalize_kernel, dim3(grid_for(D.NT, kBlock, 1024)), dim3(kBlock), 0, st, D);
    hipLaunchKernelGGL(width_kernel, dim3(grid_for(D.NT, 1, 2048)), dim3(kWidthBlock), 0, st, D);
    hipLaunchKernelGGL(gr_book_kernel, dim3(grid_for(D.P, 64)), dim3(64), 0, st, D);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Phase 4: reseeding.
// ---------------------------------------------------------------------------
// Ordered lists (ascending index) of a problem's removed slots, unfrozen
// samples and surviving peaks, from one workgroup per problem: per-thread
// contiguous chunks, exclusive scans of the chunk counts, then in-order writes.
constexpr int kScanThreads = 1024;

__global__ __launch_bounds__(kScanThreads) void ordered_lists_kernel(Dev D, int only_p) {
    __shared__ int sc[3][kScanThreads];
    const int p = only_p >= 0 ? only_p : blockIdx.x;
    const ProblemDesc &pd = D.pd[p];
    if (only_p < 0 && (D.ctl[p].K_lost == 0 || !((pd.phase_mask >> 4) & 1))) return;
    const int tid = threadIdx.x;
    const int chunk = (pd.N + kScanThreads - 1) / kScanThreads;
    const int b = pd.s0 + tid * chunk, e = min(pd.s0 + pd.N, b + chunk);
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
    int *l0 = list_ptr(D, O_SLOTS, pd.s0), *l1 = list_ptr(D, O_FREE, pd.s0), *l2 = list_ptr(D, O_PEAKS, pd.s0);
    for (int s = b; s < e; ++s) {
        if (D.removed[s]) l0[o0++] = s;
        else if (D.active[s] && !D.stuck[s]) l1[o1++] = s;
        else if (D.active[s] && D.stuck[s]) l2[o2++] = s;
    }
    if (tid == kScanThreads - 1) {
        D.ctl[p].count[O_SLOTS] = sc[0][tid];
        D.ctl[p].count[O_FREE] = sc[1][tid];
        D.ctl[p].count[O_PEAKS] = sc[2][tid];
    }
}

// Repulse Monkey when at least five unfrozen samples remain, Golden Rooster
// otherwise (unless disabled), else the slots are taken out of use.
__global__ void reseed_decide_kernel(Dev D) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= D.P) return;
    Ctl *c = &D.ctl[p];
    if (c->K_lost == 0 || !((D.pd[p].phase_mask >> 4) & 1)) {
        c->reseed_kind = 0;
        return;
    }
    if (c->count[O_FREE] >= 5) c->reseed_kind = 1;
    else if (!c->gr_disabled && c->count[O_PEAKS] > 0) c->reseed_kind = 2;
    else c->reseed_kind = 3;
}

// Shared ray step: x = o + frac * t_max * u, t_max the distance to the box
// boundary along u, then clamped to the box.
__device__ __forceinline__ void ray_fill(const Dev &D, const ProblemDesc &pd, int s, const float *o_row, float u,
                                         float frac, int lane) {
    const bool on = lane < pd.d;
    float ratio = INFINITY;
    if (on) {
        const float o = o_row[lane];
        if (u > 0.0f) ratio = (pd.hi[lane] - o) / u;
        else if (u < 0.0f) ratio = (pd.lo[lane] - o) / u;
    }
    float tmax = wave_min(ratio);
    if (!(tmax >= 0.0f) || isinf(tmax)) tmax = 0.0f;
    if (on) {
        const float x = o_row[lane] + frac * tmax * u;
        D.X[(size_t)s * D.DS + lane] = fminf(fmaxf(x, pd.lo[lane]), pd.hi[lane]);
    }
}

__global__ __launch_bounds__(kBlock) void rm_kernel(Dev D) {
    const int p = blockIdx.y;
    if (D.ctl[p].reseed_kind != 1) return;
    const ProblemDesc &pd = D.pd[p];
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int nslots = D.ctl[p].count[O_SLOTS], nfree = D.ctl[p].count[O_FREE];
    const uint32_t k = (uint32_t)D.ctl[p].k + 1u;
    const int *slots = list_ptr(D, O_SLOTS, pd.s0), *freel = list_ptr(D, O_FREE, pd.s0);
    for (int j = blockIdx.x * kWavesPerBlock + wv; j < nslots; j += gridDim.x * kWavesPerBlock) {
        const int s = slots[j];
        const uint32_t sl = (uint32_t)(s - pd.s0);
        const uint4 o4 = philox(sl, k, kRM << 24, 0u, pd.key0, pd.key1);
        const int origin = freel[uint_below(o4.x, (uint32_t)nfree)];
        const float frac = u01(o4.y);
        float z[4];
        const int blk = lane >> 2;
        box_muller4(philox(sl, k, (kRM << 24) | (1u << 16), (uint32_t)blk, pd.key0, pd.key1), z);
        const float zv = lane < pd.d ? z[lane & 3] : 0.0f;
        const float nz = sqrtf(wave_sum(zv * zv));
        ray_fill(D, pd, s, D.X + (size_t)origin * D.DS, zv / nz, frac, lane);
    }
}

// Golden Rooster: slot j (ascending) takes peak j mod n_peaks and the
// direction (-1)^q Q[:, floor(q/2) mod d], q = floor(j / n_peaks), where Q is
// the orthogonal factor (diag R > 0) of a Gaussian d x d matrix drawn for the
// peak.  One wave per slot: Householder QR in LDS, then Q e_col is formed by
// applying the reflectors to e_col in reverse order.
__global__ __launch_bounds__(kWave) void gr_kernel(Dev D) {
    const int p = blockIdx.y;
    if (D.ctl[p].reseed_kind != 2) return;
    const ProblemDesc &pd = D.pd[p];
    __shared__ float A[64 * 65];
    __shared__ float vn[64], alpha[64];
    const int lane = threadIdx.x;
    const int d = pd.d, LDA = 65;
    const int nslots = D.ctl[p].count[O_SLOTS], np = D.ctl[p].count[O_PEAKS];
    const uint32_t k = (uint32_t)D.ctl[p].k + 1u;
    const int *slots = list_ptr(D, O_SLOTS, pd.s0), *peaks = list_ptr(D, O_PEAKS, pd.s0);
    for (int j = blockIdx.x; j < nslots; j += gridDim.x) {
        const int s = slots[j];
        const int q = j % np, use = j / np;
        const int col = (use / 2) % d;
        const float sgn = (use & 1) ? -1.0f : 1.0f;
        const int pk = peaks[q];
        __syncthreads();
        for (int b = lane; b * 4 < d * d; b += kWave) {
            float z[4];
            box_muller4(philox((uint32_t)(pk - pd.s0), k, kGR << 24, (uint32_t)b, pd.key0, pd.key1), z);
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
            if (vv != 0.0f) {
                const float v = (lane >= c && lane < d) ? A[lane * LDA + c] : 0.0f;
                const float f = 2.0f * wave_sum(v * y) / vv;
                y -= f * v;
            }
        }
        if (alpha[col] < 0.0f) y = -y;
        const float u = lane < d ? sgn * y : 0.0f;
        const uint4 o4 = philox((uint32_t)(s - pd.s0), k, (kGR << 24) | (1u << 16), 0u, pd.key0, pd.key1);
        ray_fill(D, pd, s, D.X + (size_t)pk * D.DS, u, u01(o4.x), lane);
    }
}

__global__ void reseed_finalize_kernel(Dev D) {
    const int p = blockIdx.y;
    const int kind = D.ctl[p].reseed_kind;
    if (kind == 0) return;
    const ProblemDesc &pd = D.pd[p];
    const int nslots = D.ctl[p].count[O_SLOTS];
    const int *slots = list_ptr(D, O_SLOTS, pd.s0);
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < nslots; j += gridDim.x * blockDim.x) {
        const int s = slots[j];
        if (kind == 3) D.active[s] = 0;
        D.stuck[s] = 0;  // removed[] keeps the deduplication decisions until the next cycle
        D.cnt[s] = 0;
        D.head[s] = pd.m - 1;
        D.wvalid[s] = 0;
        for (int c = 0; c < pd.d; ++c) D.V[(size_t)s * D.DS + c] = 0.0f;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && kind == 2) {
        D.ctl[p].gr_used_last = 1;
        D.ctl[p].gr_prev_modes = D.ctl[p].n_modes;
    }
}

hipError_t launch_reseed(const Dev &D, hipStream_t st) {
    const unsigned per = grid_for(D.NT / D.P + 1, kWavesPerBlock, 1024);
    hipLaunchKernelGGL(ordered_lists_kernel, dim3(D.P), dim3(kScanThreads), 0, st, D, -1);
    hipLaunchKernelGGL(reseed_decide_kernel, dim3(grid_for(D.P, 64)), dim3(64), 0, st, D);
    hipLaunchKernelGGL(rm_kernel, dim3(per, D.P), dim3(kBlock), 0, st, D);
    hipLaunchKernelGGL(gr_kernel, dim3(grid_for(D.NT / D.P + 1, 1, 2048), D.P), dim3(kWave), 0, st, D);
    hipLaunchKernelGGL(reseed_finalize_kernel, dim3(grid_for(D.NT / D.P + 1, kBlock, 256), D.P), dim3(kBlock), 0, st,
                       D);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Phase 5-6 scalars.  sigma: given, or sigma_c times the pooled standard
// deviation (root of the mean per-coordinate population variance) of the
// unfrozen samples.  Step lengths: sigma / mean |g|_2 over the unfrozen
// samples at the first step of each phase (a configured alpha overrides).
// Sums are taken in float64 over fixed ranges of the problem's samples, then
// over ranges in order.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void sigma_partial_kernel(Dev D) {
    __shared__ double red[kWavesPerBlock][129];
    const int p = blockIdx.y;
    const ProblemDesc &pd = D.pd[p];
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int chunk = (pd.N + gridDim.x - 1) / gridDim.x;
    const int b = pd.s0 + blockIdx.x * chunk, e = min(pd.s0 + pd.N, b + chunk);
    double sx = 0.0, sxx = 0.0, cnt = 0.0;
    if (pd.sigma_cfg <= 0.0f) {
        for (int s = b + wv; s < e; s += kWavesPerBlock) {
            if (!(D.active[s] && !D.stuck[s])) continue;
            cnt += 1.0;
            if (lane < pd.d) {
                const double x = D.X[(size_t)s * D.DS + lane];
                sx += x;
                sxx += x * x;
            }
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
        double *part = D.part + ((size_t)p * gridDim.x + blockIdx.x) * 129;
        part[lane] = a;
        part[64 + lane] = c2;
        if (lane == 0) part[128] = n;
    }
}

__global__ void sigma_final_kernel(Dev D, int nblocks) {
    const int p = blockIdx.x;
    const ProblemDesc &pd = D.pd[p];
    const int lane = threadIdx.x;
    if (pd.sigma_cfg > 0.0f) {
        if (lane == 0) D.ctl[p].sigma = pd.sigma_cfg;
        return;
    }
    double a = 0.0, c2 = 0.0, n = 0.0;
    for (int b = 0; b < nblocks; ++b) {
        const double *part = D.part + ((size_t)p * nblocks + b) * 129;
        a += part[lane];
        c2 += part[64 + lane];
        n += part[128];
    }
    double var = 0.0;
    if (n > 0.0 && lane < pd.d) {
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
        D.ctl[p].sigma = n > 0.0 ? (float)((double)pd.sigma_c * sqrt(tot / pd.d)) : 0.0f;
    }
}

hipError_t launch_sigma(const Dev &D, hipStream_t st) {
    hipLaunchKernelGGL(sigma_partial_kernel, dim3(D.n_part_blocks, D.P), dim3(kBlock), 0, st, D);
    hipLaunchKernelGGL(sigma_final_kernel, dim3(D.P), dim3(64), 0, st, D, D.n_part_blocks);
    return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void norm_partial_kernel(Dev D, const float *Gs, const int *pids) {
    __shared__ double red[kWavesPerBlock][2];
    const int p = pids ? pids[blockIdx.y] : blockIdx.y;
    const ProblemDesc &pd = D.pd[p];
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int chunk = (pd.N + gridDim.x - 1) / gridDim.x;
    const int b = pd.s0 + blockIdx.x * chunk, e = min(pd.s0 + pd.N, b + chunk);
    double acc = 0.0, cnt = 0.0;
    if (pd.alpha <= 0.0f) {
        // four samples per pass, loaded together and added in sample order
        constexpr int kIlp = 4;
        for (int s0 = b + wv; s0 < e; s0 += kIlp * kWavesPerBlock) {
            float nn[kIlp];
            bool use[kIlp];
#pragma unroll
            for (int u = 0; u < kIlp; ++u) {
                const int s = s0 + u * kWavesPerBlock;
                use[u] = s < e && D.active[s] && !D.stuck[s];
                const float gv = (use[u] && lane < pd.d) ? Gs[(size_t)s * D.DS + lane] : 0.0f;
                nn[u] = gv * gv;
            }
#pragma unroll
            for (int u = 0; u < kIlp; ++u) nn[u] = sqrtf(wave_sum(nn[u]));
#pragma unroll
            for (int u = 0; u < kIlp; ++u)
                if (use[u]) {
                    acc += (double)nn[u];
                    cnt += 1.0;
                }
        }
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
        double *part = D.part + ((size_t)p * gridDim.x + blockIdx.x) * 2;
        part[0] = a;
        part[1] = n;
    }
}

__global__ void step_final_kernel(Dev D, int nblocks, int which, const int *pids, int np) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    const int p = pids ? pids[i] : i;
    const ProblemDesc &pd = D.pd[p];
    double a = 0.0, n = 0.0;
    for (int b = 0; b < nblocks; ++b) {
        a += D.part[((size_t)p * nblocks + b) * 2];
        n += D.part[((size_t)p * nblocks + b) * 2 + 1];
    }
    float alpha;
    if (pd.alpha > 0.0f) alpha = pd.alpha;
    else {
        const double mean = n > 0.0 ? a / n : 0.0;
        alpha = mean > 0.0 ? (float)((double)D.ctl[p].sigma / mean) : 0.0f;
    }
    if (which == 0) D.ctl[p].alpha_c = alpha;
    else D.ctl[p].alpha_a = alpha;
}

hipError_t launch_step_size(const Dev &D, const float *Gsrc, int which, hipStream_t st, const int *pids, int np) {
    // 256 blocks per problem (2 partials each: within the partial buffer)
    constexpr int kNormBlocks = 256;
    const int n = pids ? np : D.P;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(norm_partial_kernel, dim3(kNormBlocks, n), dim3(kBlock), 0, st, D, Gsrc, pids);
    hipLaunchKernelGGL(step_final_kernel, dim3(grid_for(n, 64)), dim3(64), 0, st, D, kNormBlocks, which, pids, n);
    return hipGetLastError();
}

// Workgroups per problem of the element-wise update kernels (gridDim.y = P,
// grid-stride over a problem's unfrozen rows): enough for the average
// problem, and about 8192 in all, so a batch of many problems does not
// dispatch thousands of workgroups per problem that find nothing to do.
static int per_problem_blocks(const Dev &D) {
    const int need = grid_for((long)(D.NT / D.P + 1) * D.DS, kBlock, 2048);
    return std::max(1, std::min(need, std::max(16, 8192 / D.P)));
}

// Finite-difference smoothing: mean of the per-probe gradients, probe order.
__global__ void probe_mean_kernel(Dev D, int step, const int *pids) {
    const int p = pids ? pids[blockIdx.y] : blockIdx.y;
    const ProblemDesc &pd = D.pd[p];
    if (pd.grad_mode != 0 || !((pd.phase_mask >> 5) & 1) || step >= pd.n_cloud) return;
    const int n = D.ctl[p].count[L_UNF];
    const int *lst = list_ptr(D, L_UNF, pd.s0);
    const float invM = 1.0f / (float)pd.M;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < (long)n * pd.d; e += (long)gridDim.x * blockDim.x) {
        const int s = lst[e / pd.d], c = (int)(e % pd.d);
        float acc = 0.0f;
        for (int mm = 0; mm < pd.M; ++mm) acc += D.Gp[((size_t)s * D.Mmax + mm) * D.DS + c];
        D.Gh[(size_t)s * D.DS + c] = acc * invM;
    }
}

hipError_t launch_probe_mean(const Dev &D, int step, hipStream_t st, const int *pids, int np) {
    const int n = pids ? np : D.P;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(probe_mean_kernel, dim3(per_problem_blocks(D), n), dim3(kBlock), 0, st, D, step, pids);
    return hipGetLastError();
}

// x <- clamp(x + alpha_c * smoothed gradient)
__global__ void hlc_update_kernel(Dev D, int step, const int *pids) {
    const int p = pids ? pids[blockIdx.y] : blockIdx.y;
    const ProblemDesc &pd = D.pd[p];
    if (!((pd.phase_mask >> 5) & 1) || step >= pd.n_cloud) return;
    const int n = D.ctl[p].count[L_UNF];
    const int *lst = list_ptr(D, L_UNF, pd.s0);
    const float a = D.ctl[p].alpha_c;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < (long)n * pd.d; e += (long)gridDim.x * blockDim.x) {
        const int s = lst[e / pd.d], c = (int)(e % pd.d);
        const size_t o = (size_t)s * D.DS + c;
        D.X[o] = fminf(fmaxf(D.X[o] + a * D.Gh[o], pd.lo[c]), pd.hi[c]);
    }
}

hipError_t launch_hlc_update(const Dev &D, int step, hipStream_t st, const int *pids, int np) {
    const int n = pids ? np : D.P;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(hlc_update_kernel, dim3(per_problem_blocks(D), n), dim3(kBlock), 0, st, D, step, pids);
    return hipGetLastError();
}

// v <- mu v - alpha_a g (v = 0 before the first step); x <- clamp(x + v)
__global__ void anti_update_kernel(Dev D, int step, const int *pids) {
    const int p = pids ? pids[blockIdx.y] : blockIdx.y;
    const ProblemDesc &pd = D.pd[p];
    if (!((pd.phase_mask >> 6) & 1) || step >= pd.n_anti) return;
    const int n = D.ctl[p].count[L_UNF];
    const int *lst = list_ptr(D, L_UNF, pd.s0);
    const float a = D.ctl[p].alpha_a;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < (long)n * pd.d; e += (long)gridDim.x * blockDim.x) {
        const int s = lst[e / pd.d], c = (int)(e % pd.d);
        const size_t o = (size_t)s * D.DS + c;
        const float v0 = step == 0 ? 0.0f : D.V[o];
        const float v = pd.momentum * v0 - a * D.Gh[o];
        D.V[o] = v;
        D.X[o] = fminf(fmaxf(D.X[o] + v, pd.lo[c]), pd.hi[c]);
    }
}

hipError_t launch_anti_update(const Dev &D, int step, hipStream_t st, const int *pids, int np) {
    const int n = pids ? np : D.P;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(anti_update_kernel, dim3(per_problem_blocks(D), n), dim3(kBlock), 0, st, D, step, pids);
    return hipGetLastError();
}

// Cycle end: record the statistics of cycle k+1 and optionally advance k.
__global__ void end_cycle_kernel(Dev D, int advance) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= D.P) return;
    Ctl *c = &D.ctl[p];
    const int k = c->k;
    if (k < D.n_osc) {
        CycleRecord &r = D.records[(size_t)p * D.n_osc + k];
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
        r.n_nonfinite = c->n_nonfinite;
        r.evals = c->evals;
    }
    if (advance) c->k = k + 1;
}

hipError_t launch_end_cycle(const Dev &D, int advance, hipStream_t st) {
    hipLaunchKernelGGL(end_cycle_kernel, dim3(grid_for(D.P, 64)), dim3(64), 0, st, D, advance);
    return hipGetLastError();
}

// Mode export of problem p: ordered list of its stuck active samples, rows
// gathered densely (stride d) into Gh from row s0 and values into Pd from s0
// (both free between cycles).
__global__ void gather_modes_kernel(Dev D, int p) {
    const ProblemDesc &pd = D.pd[p];
    const int n = D.ctl[p].count[O_PEAKS];
    const int *lst = list_ptr(D, O_PEAKS, pd.s0);
    float *xo = D.Gh + (size_t)pd.s0 * D.DS;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < (long)n * pd.d; e += (long)gridDim.x * blockDim.x) {
        const int j = (int)(e / pd.d), c = (int)(e % pd.d);
        const int s = lst[j];
        xo[(size_t)j * pd.d + c] = D.X[(size_t)s * D.DS + c];
        if (c == 0) D.Pd[pd.s0 + j] = gate_values(D, pd)[s];
    }
}

// the preserved inverse-Hessian diagonals of problem p's modes, in the mode order
__global__ void gather_widths_kernel(Dev D, int p) {
    const ProblemDesc &pd = D.pd[p];
    const int n = D.ctl[p].count[O_PEAKS];
    const int *lst = list_ptr(D, O_PEAKS, pd.s0);
    float *wo = D.Gh + (size_t)pd.s0 * D.DS;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < (long)n * pd.d; e += (long)gridDim.x * blockDim.x) {
        const int j = (int)(e / pd.d), c = (int)(e % pd.d);
        wo[(size_t)j * pd.d + c] = D.Wd[(size_t)lst[j] * D.DS + c];
    }
}

hipError_t launch_width_list(const Dev &D, int p, int N, hipStream_t st) {
    hipLaunchKernelGGL(ordered_lists_kernel, dim3(1), dim3(kScanThreads), 0, st, D, p);
    hipLaunchKernelGGL(gather_widths_kernel, dim3(grid_for((long)N * D.DS, kBlock, 4096)), dim3(kBlock), 0, st, D, p);
    return hipGetLastError();
}

hipError_t launch_mode_list(const Dev &D, int p, int s0, int N, hipStream_t st) {
    (void)s0;
    hipLaunchKernelGGL(ordered_lists_kernel, dim3(1), dim3(kScanThreads), 0, st, D, p);
    hipLaunchKernelGGL(gather_modes_kernel, dim3(grid_for((long)N * D.DS, kBlock, 4096)), dim3(kBlock), 0, st, D, p);
    return hipGetLastError();
}

}  // namespace chisao
