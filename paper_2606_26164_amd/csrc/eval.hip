// Batched mixture objective and adjoint gradient on FP32 MFMA (gfx950).
//
// For a point x and component k the kernel forms delta = x - mu_k (centring
// before the product keeps FP32 cancellation out of the contraction) and
// u_k = P_k delta with P_k the precision matrix.  Then
//   q_k = delta . u_k,   l_k = log c_k - q_k / 2           (Gaussian)
//                        l_k = log c_k - (nu+d)/2 log1p(q_k/nu)  (Student-t)
//   f = log sum_k exp(l_k),   grad f = -sum_k r_k s_k u_k,
// with r = softmax(l) and s_k = 1 (Gaussian) or (nu+d)/(nu+q_k) (Student-t).
// The same contraction therefore yields the value and its reverse-mode
// gradient: 2 K d^2 MFMA flops per point whether or not the gradient is kept.
//
// Work layout: a tile of 32 points in two 16-point blocks per wave (direct
// evaluations may take 16-point half tiles; four waves share a line-search
// tile, each contracting a contiguous quarter of the components, and their
// partial states are merged in wave order).  v_mfma_f32_16x16x4f32 computes U^T (DP x 16) = P' (DP x DP) *
// Delta^T (DP x 16), P' the precision matrix with its rows permuted: lane l
// supplies P[pi(16mb + l%16)][4ks + l/16] (A operand), pi(16mb + 4a + b) =
// 4(4mb + b) + a, and delta[point l%16][4ks + l/16] (B operand), and receives
// u at point l%16 and coordinate pi(16mb + 4(l/16) + r) = 4(4mb + r) + l/16,
// r = 0..3.  So each lane holds u at the very coordinates it holds delta at,
// and the quadratic form delta . u needs no second copy of delta.
// Components are streamed; the log-sum-exp runs online in base 2, and its
// reference moves (rescaling the gradient sums) only when a term exceeds it
// by 2^kLseSlack.  Mixtures with d <= 8 take a VALU path instead, one point
// per lane in 64-point tiles.
//
// The closed-form test functions of Appendix D share the kernel's tiling,
// point generation and epilogues; their value (and analytic gradient) is a
// sum over coordinates evaluated on the VALU, two lanes per point.
#include <math.h>

#include <type_traits>

#include "kernels.h"

namespace chisao {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

constexpr int NB = 2;          // 16-point blocks per wave
constexpr int kTilePts = 32;  // points per wave in the MFMA tiles
using AllBlocks = std::integral_constant<int, NB>;
using OneBlock = std::integral_constant<int, 1>;
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;
// online log-sum-exp: headroom (log2) a term may exceed the running reference
// before the reference moves
constexpr float kLseSlack = 8.0f;
// Student-t kernel in base 2: log2(1 + q / nu) with the hardware log2.
// Rounding 1 + q / nu costs at most 2^-24 absolute in the argument, i.e.
// 1.7e-7 in the log, which the factor (nu + d) / 2 scales to a few 1e-6:
// well inside the FP32 error of the quadratic form itself.
__device__ __forceinline__ float student_log2(float q, float inv_nu) { return __log2f(fmaf(q, inv_nu, 1.0f)); }

// Pointers into the global address space (plain loads through them compile
// to global_load, which only the vector-memory counter tracks).
typedef const float __attribute__((address_space(1))) gfloat;
typedef const f32x4 __attribute__((address_space(1))) gf32x4;
typedef const f32x2 __attribute__((address_space(1))) gf32x2;
__device__ __forceinline__ const gfloat *as_global(const float *p) { return (const gfloat *)p; }
// A read-only table whose address is the same in every lane, in the constant
// address space: loads at wave-uniform offsets compile to scalar loads.
typedef const float __attribute__((address_space(4))) cfloat;
__device__ __forceinline__ const cfloat *uniform_const(const float *p) {
    const uint64_t a = reinterpret_cast<uint64_t>(p);
    const uint64_t u = (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)a) |
                       ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(a >> 32)) << 32);
    return reinterpret_cast<const cfloat *>(u);
}

template <int MB>
__device__ __forceinline__ void load_frag(const gfloat *p, float out[MB]) {
    if constexpr (MB == 4) {
        const f32x4 v = *reinterpret_cast<const gf32x4 *>(p);
        out[0] = v[0]; out[1] = v[1]; out[2] = v[2]; out[3] = v[3];
    } else if constexpr (MB == 2) {
        const f32x2 v = *reinterpret_cast<const gf32x2 *>(p);
        out[0] = v[0]; out[1] = v[1];
    } else {
        out[0] = *p;
    }
}

// Raw buffer resource over a read-only table of `bytes` bytes (gfx9
// descriptor; loads past the end return zero).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t table_rsrc(const float *base, uint32_t bytes) {
    // the table pointer is the same in every lane; passing it through
    // readfirstlane puts the resource in scalar registers
    const uint64_t a = reinterpret_cast<uint64_t>(base);
    const uint64_t u = (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)a) |
                       ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(a >> 32)) << 32);
    return __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<float *>(u), (short)0,
                                             __builtin_amdgcn_readfirstlane((int)bytes), 0x00020000);
}

template <int MB>
__device__ __forceinline__ void load_frag_buf(__amdgpu_buffer_rsrc_t rs, int voff, int soff, float out[MB]) {
    if constexpr (MB == 4) {
        const f32x4 v = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, voff, soff, 0));
        out[0] = v[0]; out[1] = v[1]; out[2] = v[2]; out[3] = v[3];
    } else if constexpr (MB == 2) {
        const f32x2 v = __builtin_bit_cast(f32x2, __builtin_amdgcn_raw_buffer_load_b64(rs, voff, soff, 0));
        out[0] = v[0]; out[1] = v[1];
    } else {
        out[0] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, voff, soff, 0));
    }
}

// One component's operands in registers: precision-matrix fragments,
// centre coordinates in B-operand lane order, log2 weight.
template <int KS, int MB>
struct CompRegs {
    float pa[KS][MB];
    float muB[KS];
    float lc2;
};

// ---------------------------------------------------------------------------
// Closed-form test functions (Appendix D; each negated so that its optimum is
// a maximum).  cf_partial sums one lane's share of the coordinates, c = c0,
// c0 + 2, ... < d, into two accumulators (Ackley needs two sums, the others
// one); cf_value turns the totals into f; cf_grad gives df/dx_c from the
// totals.  Non-differentiable points (Ackley's origin, Bukin N.6's ridge)
// get a zero gradient term.
// ---------------------------------------------------------------------------
constexpr float kTwoPi = 6.283185307179586f;
constexpr float kInvPi = 0.3183098861837907f;
constexpr float kInvPi2 = 0.10132118364233778f;  // 1 / pi^2

__device__ __forceinline__ float sign_of(float v) { return (float)((v > 0.0f) - (v < 0.0f)); }

// sin(u)^20 and sin(u)^19 (Michalewicz, m = 10)
__device__ __forceinline__ void pow20(float su, float &p20, float &p19) {
    const float s2 = su * su, s4 = s2 * s2, s8 = s4 * s4, s16 = s8 * s8;
    p20 = s16 * s4;
    p19 = s16 * s2 * su;
}

__device__ __forceinline__ void cf_partial(int fam, int d, const float *x, int c0, float &a, float &b) {
    a = 0.0f;
    b = 0.0f;
    switch (fam) {
        case CHISAO_RASTRIGIN:
            for (int c = c0; c < d; c += 2) a += x[c] * x[c] - 10.0f * cospif(2.0f * x[c]);
            break;
        case CHISAO_ACKLEY:
            for (int c = c0; c < d; c += 2) {
                a += x[c] * x[c];
                b += cospif(2.0f * x[c]);
            }
            break;
        case CHISAO_SCHWEFEL:
            for (int c = c0; c < d; c += 2) a += x[c] * sinf(sqrtf(fabsf(x[c])));
            break;
        case CHISAO_STYBLINSKI_TANG:
            for (int c = c0; c < d; c += 2) {
                const float v = x[c], v2 = v * v;
                a += v2 * v2 - 16.0f * v2 + 5.0f * v;
            }
            break;
        case CHISAO_MICHALEWICZ:
            for (int c = c0; c < d; c += 2) {
                const float v = x[c];
                float p20, p19;
                // sin(i x^2 / pi) = sinpi(i x^2 / pi^2): exact range reduction
                pow20(sinpif((float)(c + 1) * v * v * kInvPi2), p20, p19);
                a += sinf(v) * p20;
            }
            break;
        case CHISAO_TRID:
            for (int c = c0; c < d; c += 2) {
                a += (x[c] - 1.0f) * (x[c] - 1.0f);
                if (c > 0) b += x[c] * x[c - 1];
            }
            break;
        case CHISAO_BUKIN6:
            if (c0 == 0) a = 100.0f * sqrtf(fabsf(x[1] - 0.01f * x[0] * x[0])) + 0.01f * fabsf(x[0] + 10.0f);
            break;
    }
}

__device__ __forceinline__ float cf_value(int fam, int d, float a, float b) {
    switch (fam) {
        case CHISAO_RASTRIGIN: return -(10.0f * (float)d + a);
        case CHISAO_ACKLEY: {
            const float r = sqrtf(a / (float)d);
            return 20.0f * expf(-0.2f * r) + expf(b / (float)d) - 20.0f - 2.718281828459045f;
        }
        case CHISAO_SCHWEFEL: return -(418.9829f * (float)d - a);
        case CHISAO_STYBLINSKI_TANG: return -0.5f * a;
        case CHISAO_MICHALEWICZ: return a;
        case CHISAO_TRID: return -(a - b);
        case CHISAO_BUKIN6: return -a;
        default: return __builtin_nanf("");
    }
}

__device__ __forceinline__ float cf_grad(int fam, int d, const float *x, int c, float a, float b) {
    const float v = x[c];
    switch (fam) {
        case CHISAO_RASTRIGIN: return -(2.0f * v + 10.0f * kTwoPi * sinpif(2.0f * v));
        case CHISAO_ACKLEY: {
            const float r = sqrtf(a / (float)d);
            const float t1 = r > 0.0f ? -20.0f * 0.2f * expf(-0.2f * r) * v / ((float)d * r) : 0.0f;
            return t1 - expf(b / (float)d) * kTwoPi * sinpif(2.0f * v) / (float)d;
        }
        case CHISAO_SCHWEFEL: {
            const float r = sqrtf(fabsf(v));
            return sinf(r) + 0.5f * r * cosf(r);
        }
        case CHISAO_STYBLINSKI_TANG: return -0.5f * (4.0f * v * v * v - 32.0f * v + 5.0f);
        case CHISAO_MICHALEWICZ: {
            const float ci = (float)(c + 1), un = ci * v * v * kInvPi2;  // u / pi
            float p20, p19;
            pow20(sinpif(un), p20, p19);
            return cosf(v) * p20 + sinf(v) * 20.0f * p19 * cospif(un) * (2.0f * ci * v * kInvPi);
        }
        case CHISAO_TRID:
            return -2.0f * (v - 1.0f) + (c > 0 ? x[c - 1] : 0.0f) + (c + 1 < d ? x[c + 1] : 0.0f);
        case CHISAO_BUKIN6: {
            const float u = x[1] - 0.01f * x[0] * x[0], r = sqrtf(fabsf(u));
            const float w = r > 0.0f ? sign_of(u) / r : 0.0f;  // d sqrt|u| / du = w / 2
            return c == 0 ? x[0] * w - 0.01f * sign_of(x[0] + 10.0f) : -50.0f * w;
        }
        default: return __builtin_nanf("");
    }
}

constexpr int kMaxClass = 256;  // problems per class (LDS budget: 2 waves per SIMD)
// waves per line-search tile: line-search launches are small, so their time
// is one tile's pass over the components, which four waves share; the closed
// forms have no component loop to split
template <int DP, int FAM>
constexpr int trial_split() { return (FAM < kFamClosed && DP != kAluDP) ? 4 : 1; }

__device__ __forceinline__ int job_count(const EvalArgs &a, int p, const ProblemDesc &pd) {
    if (a.ext_n >= 0) return a.ext_n;
    if (a.nz_kind == 1 && !(pd.noise_sigma > 0.0f)) return 0;
    if (a.need_bit && !(pd.phase_mask & (uint32_t)a.need_bit)) return 0;
    if ((a.step_limit == 1 && a.step >= pd.n_cloud) || (a.step_limit == 2 && a.step >= pd.n_anti)) return 0;
    return a.list_id >= 0 ? a.D.ctl[p].count[a.list_id] : pd.N;
}
__device__ __forceinline__ int centres(const EvalArgs &a, const ProblemDesc &pd) {
    switch (a.vc_kind) {
        case kVcTrialRest: return max(0, min(a.trial_cnt, pd.ls_max - a.trial_lo));
        case kVcProbes: return pd.M;
        default: return 1;
    }
}
// inclusive prefix sum over the wave
__device__ __forceinline__ int wave_scan(int v) {
    const int l = threadIdx.x % kWave;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int u = __shfl_up(v, o, kWave);
        if (l >= o) v += u;
    }
    return v;
}
// tiles of ppw points: jpw jobs per tile, or wpj tiles per job
__device__ __forceinline__ long tiles_of(int count, int V, int ppw, int &jpw, int &wpj) {
    if (V <= 0 || count <= 0) {
        jpw = 1;
        wpj = 1;
        return 0;
    }
    if (V <= ppw) {
        jpw = ppw / V;
        wpj = 1;
        return (count + jpw - 1) / jpw;
    }
    jpw = 1;
    wpj = (V + ppw - 1) / ppw;
    return (long)count * wpj;
}
// Line-search launches of at most this many full tiles run half tiles (16
// points, one MFMA column block): twice the tiles, each with half the matrix
// work per component, still one workgroup per CU, so the launch, whose time is
// one tile's pass over the components, takes about half as long.
constexpr int kHalfTileMax = 128;

// SPLIT waves share a tile: each contracts a contiguous part of the
// components and the first (lead) wave merges the partial log-sum-exp states
// in wave order, then runs the epilogue.  Line-search launches are small (a
// few thousand points), so their time is the latency of one tile's pass over
// all K components; splitting the components cuts that latency.
template <int DP, int FAM, bool GRAD, int CENTER, bool FD, int SPLIT, bool HT = false>
__global__ __launch_bounds__(64 * SPLIT) __attribute__((amdgpu_waves_per_eu(2))) void eval_kernel(EvalArgs a) {
    constexpr int KS = DP / 4;
    constexpr int MB = DP / 16;
    constexpr bool CLOSED = FAM >= kFamClosed;
    // small mixtures: one lane per point on the VALU, 64 points per tile
    constexpr bool ALU = !CLOSED && DP == kAluDP;
    constexpr int PPW = ALU ? kWave : kTilePts;
    constexpr int LD = DP + 1;  // padded row: conflict-free column reads
    constexpr int NP = SPLIT > 1 ? SPLIT - 1 : 1;
    __shared__ float s_pm[NP][NB][kWave], s_ps[NP][NB][kWave];       // partial max / sum of waves 1..
    __shared__ float s_pg[(SPLIT > 1 && GRAD) ? NP * NB * KS : 1][kWave];  // partial gradient sums
    __shared__ float s_pts[PPW * LD];
    __shared__ float s_g[GRAD ? PPW * LD : 1];
    __shared__ float s_f[PPW];
    __shared__ float s_den[PPW];
    __shared__ int s_s[PPW];    // sample (or caller row) per point, -1 when the lane is idle
    __shared__ int s_c[PPW];    // centre index within the job
    __shared__ int s_st[PPW];   // stencil index within the centre
    __shared__ int s_pass[PPW];
    __shared__ int s_acc[PPW];
    __shared__ int s_pref[kMaxClass + 1];
    __shared__ int s_ppw;  // points per tile in this launch
    // line search: each point's sample row and gradient before the step, and
    // the partial sums of g . (x_trial - x) over blocks of four coordinates,
    // all gathered while the points are generated
    constexpr bool TRIAL = CENTER == kTrial;
    // half tiles: only split line-search tiles, whose launches are latency-bound
    static_assert(!(TRIAL && FD), "line-search trials take no finite differences");
    constexpr bool HALF = TRIAL && SPLIT > 1;
    // HT: half tiles throughout (direct evaluations; the autotuner's choice
    // for classes whose launches hold too few full tiles to fill the chip)
    static_assert(!HT || (CENTER == kDirect && !FD && SPLIT == 1 && !CLOSED && !ALU), "half tiles: direct MFMA only");
    __shared__ int s_pref2[HALF ? kMaxClass + 1 : 1];  // tile prefix in half tiles
    __shared__ float s_x0[TRIAL ? PPW * LD : 1];
    __shared__ float s_g0[TRIAL ? PPW * LD : 1];
    __shared__ float s_dp[TRIAL ? PPW * KS : 1];

    const Dev &D = a.D;
    const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
    const bool lead = SPLIT == 1 || wv == 0;
    const int g = lane >> 4, n = lane & 15;
    const bool ext = a.ext_n >= 0;
    // Tile prefix over the problems of the class.  Line-search launches are
    // short and many, and a VALU-path launch is short whatever its kind, so
    // there the first wave computes it, one problem per lane: the problems'
    // counts are read in parallel, not one dependent load after another.  The
    // other launches are long; there one thread walks the problems (the wave
    // version's extra scalar registers cost the long launches' component loop
    // more than the walk takes).
    if constexpr (TRIAL || ALU) {
        if (threadIdx.x < kWave) {
            int carry = 0, carry2 = 0;
            if (lane == 0) s_pref[0] = s_pref2[0] = 0;
            for (int j0 = 0; j0 < a.n_cls; j0 += kWave) {
                const int j = j0 + lane;
                int t = 0, t2 = 0;
                if (j < a.n_cls) {
                    const int p = a.cls[j];
                    const ProblemDesc &pd = D.pd[p];
                    const int jobs = job_count(a, p, pd);
                    const int V = centres(a, pd) * (FD ? 2 * pd.d : 1);
                    int jpw, wpj;
                    t = (int)tiles_of(jobs, V, PPW, jpw, wpj);
                    if constexpr (HALF) t2 = (int)tiles_of(jobs, V, PPW / 2, jpw, wpj);
                    // evaluation counts, once per launch (block 0) rather than per tile
                    if (blockIdx.x == 0 && !ext && jobs > 0) {
                        const unsigned long long nv = (unsigned long long)jobs * (unsigned long long)V;
                        atomicAdd(&D.ctl[p].evals, nv);
                        atomicAdd(&D.prof[FD ? 3 : CENTER], nv);
                    }
                }
                const int inc = wave_scan(t), inc2 = HALF ? wave_scan(t2) : 0;
                if (j < a.n_cls) {
                    s_pref[j + 1] = carry + inc;
                    if constexpr (HALF) s_pref2[j + 1] = carry2 + inc2;
                }
                carry += __shfl(inc, kWave - 1, kWave);
                if constexpr (HALF) carry2 += __shfl(inc2, kWave - 1, kWave);
            }
            if (HALF && lane == 0) s_ppw = carry <= kHalfTileMax ? PPW / 2 : PPW;
        }
    } else if (threadIdx.x == 0) {
        int acc = 0;
        unsigned long long pts = 0;
        s_pref[0] = 0;
        for (int j = 0; j < a.n_cls; ++j) {
            const int p = a.cls[j];
            const ProblemDesc &pd = D.pd[p];
            const int Vs = FD ? 2 * pd.d : 1;
            const int jobs = job_count(a, p, pd);
            int jpw, wpj;
            acc += (int)tiles_of(jobs, centres(a, pd) * Vs, HT ? PPW / 2 : PPW, jpw, wpj);
            s_pref[j + 1] = acc;
            // evaluation counts, once per launch (block 0) rather than per tile
            if (blockIdx.x == 0 && !ext && jobs > 0) {
                const unsigned long long nv = (unsigned long long)jobs * centres(a, pd) * Vs;
                atomicAdd(&D.ctl[p].evals, nv);
                pts += nv;
            }
        }
        if (blockIdx.x == 0 && pts) atomicAdd(&D.prof[FD ? 3 : CENTER], pts);
    }
    __syncthreads();
    const int ppw = HALF ? s_ppw : (HT ? PPW / 2 : PPW);
    const int *pref = (HALF && ppw < PPW) ? s_pref2 : s_pref;
    const int n_tiles = pref[a.n_cls];

    // Tile order.  Linear: block b takes tiles b, b + G, ...  XCD-chunked:
    // workgroups are dispatched round-robin over the 8 XCDs, so block b runs on
    // XCD b % 8; that XCD's blocks take a contiguous eighth of the tile range,
    // which in class order spans fewer problems, so each XCD's L2 holds the
    // precision matrices of fewer problems.
    int t0 = 0, first = blockIdx.x, stride = gridDim.x, span = n_tiles;
    if (a.order == 1) {
        constexpr int kXcd = 8;
        span = (n_tiles + kXcd - 1) / kXcd;
        t0 = (blockIdx.x % kXcd) * span;
        first = blockIdx.x / kXcd;
        stride = gridDim.x / kXcd;
    }
    for (int it = first; it < span; it += stride) {
        const int tile = t0 + it;
        if (tile >= n_tiles) break;
        // ---- the tile's problem ---------------------------------------------
        int lo_j = 0, hi_j = a.n_cls - 1;
        while (lo_j < hi_j) {
            const int mid = (lo_j + hi_j + 1) >> 1;
            if (pref[mid] <= tile) lo_j = mid;
            else hi_j = mid - 1;
        }
        // every lane finds the same problem; saying so keeps its descriptor,
        // table pointers and the component loop's addressing in scalar
        // registers instead of per-lane 64-bit arithmetic
        const int p = __builtin_amdgcn_readfirstlane(a.cls[lo_j]);
        const ProblemDesc &pd = D.pd[p];
        const int ltile = tile - pref[lo_j];
        const int d = pd.d;
        const int count = job_count(a, p, pd);
        const int Vc = centres(a, pd);
        const int r0 = a.vc_kind == kVcTrialRest ? a.trial_lo : 0;
        const int Vs = FD ? 2 * d : 1;
        const int V = Vc * Vs;
        int jpw, wpj;
        (void)tiles_of(count, V, ppw, jpw, wpj);
        const uint32_t kcyc = (uint32_t)D.ctl[p].k + 1u;
        const float sigma = (CENTER == kProbe) ? D.ctl[p].sigma : 0.0f;
        const int xs = a.x_stride;
        const int *lst = (!ext && a.list_id >= 0) ? list_ptr(D, a.list_id, pd.s0) : nullptr;
        // ---- point metadata ------------------------------------------------
        if (lead && lane < PPW) {
            const int pt = lane;
            int job, v;
            bool valid;
            if (V <= ppw) {
                job = (int)(ltile * jpw) + pt / V;
                v = pt % V;
                valid = (pt < jpw * V) && job < count;
            } else {
                job = (int)(ltile / wpj);
                v = (int)(ltile % wpj) * ppw + pt;
                valid = pt < ppw && v < V;
            }
            s_s[pt] = valid ? (ext ? job : (lst ? lst[job] : pd.s0 + job)) : -1;
            s_c[pt] = v / Vs;
            s_st[pt] = v % Vs;
            s_den[pt] = 1.0f;
        }
        __syncthreads();
        // ---- generate the points (zero padded to DP), all waves -------------
        // rows are read in 16-byte chunks when the row stride and base allow it
        // (the library's own rows always do; a caller's array may not)
        const bool vrow = (xs & 3) == 0 && (reinterpret_cast<uintptr_t>(a.X) & 15) == 0;
        // Smoothing probes come in antithetic pairs x + sigma z, x - sigma z
        // (centres 2i and 2i + 1 of a job).  When a job's probe count is even
        // the two points of a pair sit side by side in the tile, from an even
        // slot on, so one read of the sample row and one draw of z serve both
        // (the same values the per-point loop below computes for each).
        bool paired = false;
        if constexpr (CENTER == kProbe && !FD) paired = (Vc & 1) == 0;
        if (paired) {
            for (int e = threadIdx.x; e < (PPW / 2) * KS; e += blockDim.x) {
                const int pt = 2 * (e / KS), blk = e % KS, c0 = 4 * blk;
                const int s = s_s[pt];  // the same sample as slot pt + 1
                float xp[4] = {0.f, 0.f, 0.f, 0.f}, xm[4] = {0.f, 0.f, 0.f, 0.f};
                if (s >= 0 && c0 < d) {
                    const uint32_t pair = (uint32_t)(s_c[pt] >> 1);
                    float z[4];
                    box_muller4(philox((uint32_t)(s - pd.s0), kcyc, (kHLC << 24) | ((uint32_t)a.step << 16) | pair,
                                       (uint32_t)blk, pd.key0, pd.key1),
                                z);
                    float xr[4] = {0.f, 0.f, 0.f, 0.f};
                    if (vrow) {
                        const f32x4 w = *reinterpret_cast<const f32x4 *>(a.X + (size_t)s * xs + c0);
                        xr[0] = w[0]; xr[1] = w[1]; xr[2] = w[2]; xr[3] = w[3];
                    } else {
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            if (c0 + q < d) xr[q] = a.X[(size_t)s * xs + c0 + q];
                    }
                    const float sp = sigma, sm = -sigma;
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        if (c0 + q < d) {
                            xp[q] = xr[q] + sp * z[q];
                            xm[q] = xr[q] + sm * z[q];
                        }
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    s_pts[pt * LD + c0 + q] = xp[q];
                    s_pts[(pt + 1) * LD + c0 + q] = xm[q];
                }
            }
        }
        for (int e = paired ? PPW * KS : threadIdx.x; e < PPW * KS; e += blockDim.x) {
            const int pt = e / KS, blk = e % KS, c0 = 4 * blk;
            const int s = s_s[pt];
            float x[4] = {0.f, 0.f, 0.f, 0.f};
            float x0[4] = {0.f, 0.f, 0.f, 0.f}, g0[4] = {0.f, 0.f, 0.f, 0.f};
            float dp = 0.0f;
            if (s >= 0) {
                const int ci = s_c[pt];
                float z[4] = {0.f, 0.f, 0.f, 0.f};
                if constexpr (CENTER == kProbe) {
                    const uint32_t pair = (uint32_t)(ci >> 1);
                    uint4 o = philox((uint32_t)(s - pd.s0), kcyc,
                                     (kHLC << 24) | ((uint32_t)a.step << 16) | pair, (uint32_t)blk, pd.key0, pd.key1);
                    box_muller4(o, z);
                }
                float xr[4] = {0.f, 0.f, 0.f, 0.f}, gr[4] = {0.f, 0.f, 0.f, 0.f}, pr[4] = {0.f, 0.f, 0.f, 0.f};
                if (c0 < d) {
                    if (vrow) {
                        const f32x4 w = *reinterpret_cast<const f32x4 *>(a.X + (size_t)s * xs + c0);
                        xr[0] = w[0]; xr[1] = w[1]; xr[2] = w[2]; xr[3] = w[3];
                    } else {
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            if (c0 + q < d) xr[q] = a.X[(size_t)s * xs + c0 + q];
                    }
                    if constexpr (CENTER == kTrial) {
                        // the library's rows: stride a multiple of four floats
                        const f32x4 wg = *reinterpret_cast<const f32x4 *>(D.G + (size_t)s * D.DS + c0);
                        const f32x4 wp = *reinterpret_cast<const f32x4 *>(D.Pd + (size_t)s * D.DS + c0);
                        gr[0] = wg[0]; gr[1] = wg[1]; gr[2] = wg[2]; gr[3] = wg[3];
                        pr[0] = wp[0]; pr[1] = wp[1]; pr[2] = wp[2]; pr[3] = wp[3];
                    }
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int c = c0 + q;
                    if (c < d) {
                        float xv = xr[q];
                        if constexpr (CENTER == kTrial) {
                            const float t = ldexpf(1.0f, -(r0 + ci));
                            x0[q] = xv;
                            g0[q] = gr[q];
                            xv = fminf(fmaxf(xv + t * pr[q], pd.lo[c]), pd.hi[c]);
                            dp += g0[q] * (xv - x0[q]);
                        } else if constexpr (CENTER == kProbe) {
                            const float sgn = (ci & 1) ? -1.0f : 1.0f;
                            xv = xv + sigma * sgn * z[q];
                        }
                        x[q] = xv;
                    }
                }
                if constexpr (FD) {
                    const int st = s_st[pt];
                    const int cs = st >> 1;
                    if (cs >= c0 && cs < c0 + 4) {
                        const float xc = x[cs - c0];
                        const float h = pd.fd_h > 0.0f ? pd.fd_h : ldexpf(fmaxf(1.0f, fabsf(xc)), -8);
                        const float xp = xc + h, xm = xc - h;
                        x[cs - c0] = (st & 1) ? xm : xp;
                        s_den[pt] = xp - xm;
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) s_pts[pt * LD + c0 + q] = x[q];
            if constexpr (TRIAL) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    s_x0[pt * LD + c0 + q] = x0[q];
                    s_g0[pt * LD + c0 + q] = g0[q];
                }
                s_dp[pt * KS + blk] = dp;
            }
        }
        __syncthreads();
        // Noisy problems: every value the method sees carries sigma_n z, z the
        // first normal of the NOISE stream at (sample, cycle, step << 16 |
        // sub); the gate value carries sigma_n times the mean of gate_reps
        // normals of the GATE stream.  The gradient stays noise-free.
        const bool noisy = !ext && a.nz_kind >= 0 && pd.noise_sigma > 0.0f;
        auto noise_of = [&](int pt) -> float {
            const uint32_t ls = (uint32_t)(s_s[pt] - pd.s0);
            if (a.nz_kind == 0) {
                uint32_t sub = a.nz_base;
                if constexpr (CENTER == kTrial) sub += (uint32_t)(r0 + s_c[pt]);
                if constexpr (CENTER == kProbe) sub |= (uint32_t)s_c[pt] << 7;
                if constexpr (FD) sub += (uint32_t)s_st[pt];
                float z[4];
                box_muller4(philox(ls, kcyc, (kNoise << 24) | ((uint32_t)a.step << 16) | sub, 0u, pd.key0, pd.key1), z);
                return pd.noise_sigma * z[0];
            }
            float zs = 0.0f;
            for (int b = 0; 4 * b < pd.gate_reps; ++b) {
                float z[4];
                box_muller4(philox(ls, kcyc, kGate << 24, (uint32_t)b, pd.key0, pd.key1), z);
                for (int q = 0; q < 4 && 4 * b + q < pd.gate_reps; ++q) zs += z[q];
            }
            return pd.noise_sigma * (zs / (float)pd.gate_reps);
        };
        if constexpr (CLOSED) {
            // ---- closed-form value (and gradient), two lanes per point ------
            const int pt = lane >> 1, c0 = lane & 1;
            const float *x = s_pts + pt * LD;
            float sa, sb;
            cf_partial(pd.family, d, x, c0, sa, sb);
            sa += __shfl_xor(sa, 1, kWave);
            sb += __shfl_xor(sb, 1, kWave);
            if (s_s[pt] >= 0) {
                if (c0 == 0) {
                    float f = cf_value(pd.family, d, sa, sb);
                    if (noisy) f += noise_of(pt);
                    s_f[pt] = f;
                }
                if constexpr (GRAD)
                    for (int c = c0; c < d; c += 2) s_g[pt * LD + c] = cf_grad(pd.family, d, x, c, sa, sb);
            }
            __syncthreads();
        } else if constexpr (ALU) {
            // ---- small mixtures: one lane per point on the VALU ----------------
            // A few coordinates give the matrix core too little to do: padded
            // to 16, a d = 2 component would cost its full 16-wide tile.  Here
            // each lane carries one point through the components; the tile's
            // problem is the same in every lane, so a component's record (P's
            // upper triangle, mu, log2 weight) is read with scalar loads and
            // enters each instruction as its scalar operand.
            const int W = alu_width(d);
            const int K = __builtin_amdgcn_readfirstlane(pd.K);
            const cfloat *tab = uniform_const(pd.Pfrag);
            const float nu = pd.nu, nupd = pd.nu_plus_d, inv_nu = 1.0f / nu;
            auto run = [&](auto wc) {
                constexpr int Wc = decltype(wc)::value, T = Wc * (Wc + 1) / 2, R = alu_record(Wc);
                const int pt = lane;
                float xr[Wc], ga[GRAD ? Wc : 1];
#pragma unroll
                for (int i = 0; i < Wc; ++i) {
                    xr[i] = s_pts[pt * LD + i];
                    if constexpr (GRAD) ga[i] = 0.0f;
                }
                float m = -INFINITY, sm = 0.0f;
                for (int k = 0; k < K; ++k) {
                    const cfloat *rec = tab + k * R;
                    float dl[Wc], u[Wc];
#pragma unroll
                    for (int i = 0; i < Wc; ++i) dl[i] = xr[i] - rec[T + i];
                    // u = P (x - mu) from the upper triangle, q = (x - mu) . u
                    float q = 0.0f;
#pragma unroll
                    for (int i = 0; i < Wc; ++i) {
                        float acc = 0.0f;
#pragma unroll
                        for (int j = 0; j < Wc; ++j) {
                            const int lo = i < j ? i : j, hi = i < j ? j : i;
                            acc = fmaf(rec[lo * Wc - lo * (lo - 1) / 2 + (hi - lo)], dl[j], acc);
                        }
                        u[i] = acc;
                        q = fmaf(dl[i], acc, q);
                    }
                    float l2, w = 1.0f;
                    if constexpr (FAM == 0) {
                        l2 = rec[T + Wc] - q * (0.5f * kLog2e);
                    } else {
                        l2 = rec[T + Wc] - (0.5f * nupd) * student_log2(q, inv_nu);
                        w = nupd * __builtin_amdgcn_rcpf(nu + q);
                    }
                    // the same online log-sum-exp as the tiles: the reference
                    // moves only when a term exceeds it by 2^kLseSlack, which
                    // few components do, so the rescale is a rare branch
                    const bool moved = l2 > m + kLseSlack;
                    if (__any(moved)) {
                        const float mnew = moved ? l2 : m;
                        const float sc = moved ? __builtin_amdgcn_exp2f(m - mnew) : 1.0f;
                        sm *= sc;
                        if constexpr (GRAD)
#pragma unroll
                            for (int i = 0; i < Wc; ++i) ga[i] *= sc;
                        m = mnew;
                    }
                    const float pk = __builtin_amdgcn_exp2f(l2 - m);
                    sm += pk;
                    if constexpr (GRAD) {
                        const float pw = pk * w;
#pragma unroll
                        for (int i = 0; i < Wc; ++i) ga[i] = fmaf(pw, u[i], ga[i]);
                    }
                }
                float f = (m + __log2f(sm)) * kLn2;
                if (noisy && s_s[pt] >= 0) f += noise_of(pt);
                s_f[pt] = f;
                if constexpr (GRAD) {
                    const float inv = -1.0f / sm;
#pragma unroll
                    for (int i = 0; i < Wc; ++i) s_g[pt * LD + i] = ga[i] * inv;
                }
            };
            if (W == 2) run(std::integral_constant<int, 2>{});
            else if (W == 4) run(std::integral_constant<int, 4>{});
            else run(std::integral_constant<int, 8>{});
            __syncthreads();
        } else {
            // ---- operand registers ---------------------------------------------
            float xB[NB][KS];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const float *row = s_pts + (nb * 16 + n) * LD;
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) xB[nb][ks] = row[4 * ks + g];
            }
            float mrun[NB], srun[NB];
            float gacc[NB][GRAD ? KS : 1];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                mrun[nb] = -INFINITY;
                srun[nb] = 0.0f;
                if constexpr (GRAD)
#pragma unroll
                    for (int i = 0; i < KS; ++i) gacc[nb][i] = 0.0f;
            }
            // ---- stream the components -----------------------------------------
            // Two waves per SIMD: while one waits for a component's operands or
            // works through the log-sum-exp epilogue on the VALU, the other keeps
            // the matrix core busy; a wave raises its priority for the duration of
            // its MFMA block so the arbiter keeps the matrix core fed.  Operands
            // come through buffer loads, which only the vector-memory counter
            // tracks: flat loads would also count against the LDS counter, and
            // the cross-lane reductions of the epilogue would then wait for them.
            const float nu = pd.nu, nupd = pd.nu_plus_d, inv_nu = 1.0f / nu;
            CompRegs<KS, MB> ra;
            // Buffer loads: a scalar resource per table and the component's
            // byte offset in a scalar register, each lane's fixed offset in a
            // vector register, so the loop advances one scalar per table
            // instead of per-lane 64-bit addresses.
            const int Kc = pd.K;
            const __amdgpu_buffer_rsrc_t rs_pf = table_rsrc(pd.Pfrag, (uint32_t)Kc * DP * DP * 4u);
            const __amdgpu_buffer_rsrc_t rs_mu = table_rsrc(pd.muB, (uint32_t)Kc * DP * 4u);
            const __amdgpu_buffer_rsrc_t rs_lc = table_rsrc(pd.logc2, (uint32_t)Kc * 4u);
            const int pf_lane = lane * MB * 4, mu_lane = g * KS * 4;
            auto load = [&](int k, CompRegs<KS, MB> &r) {
                const int pf_k = k * DP * DP * 4, mu_k = k * DP * 4;
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) load_frag_buf<MB>(rs_pf, pf_lane + ks * kWave * MB * 4, pf_k, r.pa[ks]);
#pragma unroll
                for (int i = 0; i < KS; i += 4) {
                    const f32x4 vb = __builtin_bit_cast(
                        f32x4, __builtin_amdgcn_raw_buffer_load_b128(rs_mu, mu_lane + i * 4, mu_k, 0));
                    r.muB[i] = vb[0]; r.muB[i + 1] = vb[1]; r.muB[i + 2] = vb[2]; r.muB[i + 3] = vb[3];
                }
                r.lc2 = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs_lc, 0, k * 4, 0));
            };
            // contracts one component for the first NBA column blocks of the tile
            // log-sum-exp state of the lane's own block in the two-block path
            float m_own = -INFINITY, s_own = 0.0f;
            auto own_to_blocks = [&](auto nba) {
                if constexpr (decltype(nba)::value == 2) {
                    rows_pair_split(m_own, mrun[0], mrun[1]);
                    rows_pair_split(s_own, srun[0], srun[1]);
                }
            };
            auto step = [&](const CompRegs<KS, MB> &r, auto nba) {
                constexpr int NBA = decltype(nba)::value;
                f32x4 acc[NB][MB];
#pragma unroll
                for (int nb = 0; nb < NBA; ++nb)
#pragma unroll
                    for (int mb = 0; mb < MB; ++mb) acc[nb][mb] = f32x4{0.f, 0.f, 0.f, 0.f};
                // delta = x - mu_k in B-operand order; with the rows of P
                // permuted at init, the accumulator of lane (n, g) holds u at
                // the same coordinates 4 ks + g, so delta also serves the
                // quadratic form below
                float bv[NB][KS];
                __builtin_amdgcn_s_setprio(1);
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) {
#pragma unroll
                    for (int nb = 0; nb < NBA; ++nb) {
                        bv[nb][ks] = xB[nb][ks] - r.muB[ks];
#pragma unroll
                        for (int mb = 0; mb < MB; ++mb)
                            acc[nb][mb] =
                                __builtin_amdgcn_mfma_f32_16x16x4f32(r.pa[ks][mb], bv[nb][ks], acc[nb][mb], 0, 0, 0);
                    }
                }
                __builtin_amdgcn_s_setprio(0);
                if constexpr (NBA == 2) {
                    // Both blocks' quadratic forms reduced in one exchange;
                    // rows 0 and 2 then carry block 0's log-sum-exp state and
                    // rows 1 and 3 block 1's (the same arithmetic as the
                    // per-block path below, half the lanes' work each), and
                    // the gradient weights are exchanged back to every lane.
                    float q0 = 0.0f, q1 = 0.0f;
#pragma unroll
                    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                        for (int rr = 0; rr < 4; ++rr) {
                            q0 = fmaf(bv[0][4 * mb + rr], acc[0][mb][rr], q0);
                            q1 = fmaf(bv[1][4 * mb + rr], acc[1][mb][rr], q1);
                        }
                    const float q = rows4_sum_pair(q0, q1);
                    float l2, w = 1.0f;
                    if constexpr (FAM == 0) {
                        l2 = r.lc2 - q * (0.5f * kLog2e);
                    } else {
                        l2 = r.lc2 - (0.5f * nupd) * student_log2(q, inv_nu);
                        w = nupd * __builtin_amdgcn_rcpf(nu + q);
                    }
                    const bool moved = l2 > m_own + kLseSlack;
                    const float mnew = moved ? l2 : m_own;
                    const float sc = __builtin_amdgcn_exp2f(m_own - mnew);
                    const float pk = __builtin_amdgcn_exp2f(l2 - mnew);
                    s_own = fmaf(s_own, sc, pk);
                    m_own = mnew;
                    if constexpr (GRAD) {
                        if (__any(moved)) {
                            // sc is exactly 1 in the block that did not move
                            float sc0, sc1;
                            rows_pair_split(sc, sc0, sc1);
#pragma unroll
                            for (int i = 0; i < KS; ++i) {
                                gacc[0][i] *= sc0;
                                gacc[1][i] *= sc1;
                            }
                        }
                    }
                    if constexpr (GRAD) {
                        float pw0, pw1;
                        rows_pair_split(pk * w, pw0, pw1);
#pragma unroll
                        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                            for (int rr = 0; rr < 4; ++rr) {
                                gacc[0][mb * 4 + rr] = fmaf(pw0, acc[0][mb][rr], gacc[0][mb * 4 + rr]);
                                gacc[1][mb * 4 + rr] = fmaf(pw1, acc[1][mb][rr], gacc[1][mb * 4 + rr]);
                            }
                    }
                    return;
                }
#pragma unroll
                for (int nb = 0; nb < NBA; ++nb) {
                    float q = 0.0f;
#pragma unroll
                    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                        for (int rr = 0; rr < 4; ++rr) q = fmaf(bv[nb][4 * mb + rr], acc[nb][mb][rr], q);
                    q = rows4_sum(q);
                    float l2, w = 1.0f;
                    if constexpr (FAM == 0) {
                        l2 = r.lc2 - q * (0.5f * kLog2e);
                    } else {
                        l2 = r.lc2 - (0.5f * nupd) * student_log2(q, inv_nu);
                        w = nupd * __builtin_amdgcn_rcpf(nu + q);
                    }
                    // the reference moves only when a term exceeds it by more
                    // than 2^kLseSlack: terms stay below 2^kLseSlack, and the
                    // gradient sums are rescaled far less often
                    const bool moved = l2 > mrun[nb] + kLseSlack;
                    const float mnew = moved ? l2 : mrun[nb];
                    const float sc = __builtin_amdgcn_exp2f(mrun[nb] - mnew);
                    const float pk = __builtin_amdgcn_exp2f(l2 - mnew);
                    srun[nb] = fmaf(srun[nb], sc, pk);
                    mrun[nb] = mnew;
                    if constexpr (GRAD) {
                        if (__any(moved)) {
#pragma unroll
                            for (int i = 0; i < KS; ++i) gacc[nb][i] *= sc;
                        }
                        const float pw = pk * w;
#pragma unroll
                        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                            for (int rr = 0; rr < 4; ++rr)
                                gacc[nb][mb * 4 + rr] = fmaf(pw, acc[nb][mb][rr], gacc[nb][mb * 4 + rr]);
                    }
                }
            };
            const int K = __builtin_amdgcn_readfirstlane(pd.K);
            const int wvu = __builtin_amdgcn_readfirstlane(wv);
            const int kb = SPLIT == 1 ? 0 : (wvu * K) / SPLIT, ke = SPLIT == 1 ? K : ((wvu + 1) * K) / SPLIT;
            if constexpr (DP < 64) {
                // small components: too little work per component to hide its load
                // latency behind the other wave, so the next one is loaded into a
                // second register set while this one is contracted (the set is
                // small at DP <= 32); the prefetch past the end reloads the last
                // component, which keeps the loop branch-free
                auto run = [&](auto nba) {
                    if (kb < ke) {
                        CompRegs<KS, MB> rb;
                        load(kb, ra);
                        for (int k = kb; k < ke; k += 2) {
                            load(min(k + 1, ke - 1), rb);
                            step(ra, nba);
                            if (k + 1 >= ke) break;
                            load(min(k + 2, ke - 1), ra);
                            step(rb, nba);
                        }
                    }
                    own_to_blocks(nba);
                };
                if constexpr (HALF) {
                    if (ppw < PPW) run(OneBlock{});
                    else run(AllBlocks{});
                } else if constexpr (HT) {
                    run(OneBlock{});
                } else {
                    run(AllBlocks{});
                }
            } else {
                auto run = [&](auto nba) {
                    for (int k = kb; k < ke; ++k) {
                        load(k, ra);
                        step(ra, nba);
                    }
                    own_to_blocks(nba);
                };
                if constexpr (HALF) {
                    if (ppw < PPW) run(OneBlock{});
                    else run(AllBlocks{});
                } else if constexpr (HT) {
                    run(OneBlock{});
                } else {
                    run(AllBlocks{});
                }
            }
            if constexpr (SPLIT > 1) {
                // merge: m = max(m0, m_v), s = s0 2^(m0-m) + s_v 2^(m_v-m), the
                // gradient sums alike, for v = 1, 2, ... in order
                if (!lead) {
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb) {
                        s_pm[wv - 1][nb][lane] = mrun[nb];
                        s_ps[wv - 1][nb][lane] = srun[nb];
                        if constexpr (GRAD)
#pragma unroll
                            for (int i = 0; i < KS; ++i) s_pg[((wv - 1) * NB + nb) * KS + i][lane] = gacc[nb][i];
                    }
                }
                __syncthreads();
                if (lead) {
                    for (int v = 0; v < SPLIT - 1; ++v) {
#pragma unroll
                        for (int nb = 0; nb < NB; ++nb) {
                            const float mv = s_pm[v][nb][lane];
                            if (!(mv > -INFINITY)) continue;  // no components in that part
                            const float mn = fmaxf(mrun[nb], mv);
                            const float a0 = __builtin_amdgcn_exp2f(mrun[nb] - mn);
                            const float a1 = __builtin_amdgcn_exp2f(mv - mn);
                            srun[nb] = fmaf(srun[nb], a0, s_ps[v][nb][lane] * a1);
                            if constexpr (GRAD)
#pragma unroll
                                for (int i = 0; i < KS; ++i)
                                    gacc[nb][i] = fmaf(gacc[nb][i], a0, s_pg[(v * NB + nb) * KS + i][lane] * a1);
                            mrun[nb] = mn;
                        }
                    }
                }
            }
            // ---- results to LDS --------------------------------------------
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                if (!lead || ((HALF || HT) && nb * 16 >= ppw)) break;
                const int pt = nb * 16 + n;
                float f = (mrun[nb] + __log2f(srun[nb])) * kLn2;
                if (noisy && g == 0 && s_s[pt] >= 0) f += noise_of(pt);
                if (g == 0) s_f[pt] = f;
                if constexpr (GRAD) {
                    const float inv = -1.0f / srun[nb];
#pragma unroll
                    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                        for (int r = 0; r < 4; ++r) s_g[pt * LD + 4 * (4 * mb + r) + g] = gacc[nb][mb * 4 + r] * inv;
                }
            }
            __syncthreads();
        }
        // ---- epilogues -----------------------------------------------------
        const int os = a.out_stride;
        if constexpr (CENTER == kDirect && !FD) {
            if (lead && lane < PPW && s_s[lane] >= 0 && a.F_out) a.F_out[s_s[lane]] = s_f[lane];
            if constexpr (GRAD) {
                if (lead && a.G_out)
                    for (int e = lane; e < PPW * d; e += kWave) {
                        const int pt = e / d, c = e % d, s = s_s[pt];
                        if (s >= 0) a.G_out[(size_t)s * os + c] = s_g[pt * LD + c];
                    }
            }
        } else if constexpr (FD) {
            if (lead && lane < PPW) {
                const int pt = lane, s = s_s[pt], st = s_st[pt];
                if (s >= 0 && (st & 1) == 0) {
                    const float gv = (s_f[pt] - s_f[pt + 1]) / s_den[pt];
                    const int c = st >> 1;
                    if constexpr (CENTER == kDirect) a.G_out[(size_t)s * os + c] = gv;
                    else D.Gp[((size_t)s * D.Mmax + s_c[pt]) * D.DS + c] = gv;
                }
            }
        } else if constexpr (CENTER == kProbe) {
            // mean over the job's probes, summed in probe order
            const float invM = 1.0f / (float)Vc;
            for (int e = lead ? lane : jpw * d; e < jpw * d; e += kWave) {
                const int j = e / d, c = e % d, p0 = j * Vc, s = s_s[p0];
                if (s >= 0) {
                    float acc = 0.0f;
                    for (int mm = 0; mm < Vc; ++mm) acc += s_g[(p0 + mm) * LD + c];
                    D.Gh[(size_t)s * D.DS + c] = acc * invM;
                }
            }
        } else if constexpr (CENTER == kTrial) {
            // Armijo margins f_tr - f - c1 g.(x_tr - x), two lanes per point
            const int DS = D.DS;
            if (lead) {
                for (int pt0 = 0; pt0 < PPW; pt0 += kWave / 2) {
                    const int pt = pt0 + (lane >> 1), h = lane & 1, s = s_s[pt];
                    float dot = 0.0f;
                    if (s >= 0)
                        for (int b = h; b < KS; b += 2) dot += s_dp[pt * KS + b];
                    dot += __shfl_xor(dot, 1, kWave);
                    // (relaxed by twice the noise level for noisy objectives: the
                    // noise-aware Armijo test of Berahas, Byrd and Nocedal 2019)
                    if (h == 0)
                        s_pass[pt] =
                            (s >= 0) && (s_f[pt] - D.F[s] - pd.ls_c1 * dot + 2.0f * pd.noise_sigma >= 0.0f);
                }
            }
            __syncthreads();
            if (lead && lane < jpw) {
                int r = -1;
                const int p0 = lane * Vc;
                if (s_s[p0] >= 0)
                    for (int i = 0; i < Vc; ++i)
                        if (s_pass[p0 + i]) { r = i; break; }
                s_acc[lane] = r;
            }
            __syncthreads();
            for (int e = threadIdx.x; e < jpw * d; e += blockDim.x) {
                const int j = e / d, c = e % d, p0 = j * Vc, s = s_s[p0];
                if (s >= 0 && s_acc[j] >= 0) {
                    const int pa = p0 + s_acc[j];
                    const size_t o = (size_t)s * DS + c;
                    D.Xprev[o] = s_x0[p0 * LD + c];
                    D.X[o] = s_pts[pa * LD + c];
                    D.Gprev[o] = s_g0[p0 * LD + c];
                    if constexpr (GRAD) D.G[o] = s_g[pa * LD + c];
                }
            }
            // verdict per list position for the compaction that follows:
            // 1 try the remaining trials, 2 accepted (the finite-difference
            // gradient is still due), 3 the search failed, 0 nothing to do
            if (lead && lane < jpw) {
                const int p0 = lane * Vc, sl = s_s[p0];
                if (sl >= 0) {
                    const int r = s_acc[lane];
                    uint8_t verdict;
                    if (r >= 0) {
                        D.F[sl] = s_f[p0 + r];
                        D.status[sl] = (uint8_t)(kStAccept | (r0 + r));
                        verdict = GRAD ? 0 : 2;
                    } else if (a.trial_next >= 0 && r0 + Vc < pd.ls_max) {
                        verdict = 1;
                    } else {
                        D.status[sl] = kStFail;
                        verdict = 3;
                    }
                    D.flag[pd.s0 + (int)(ltile * jpw) + lane] = verdict;
                }
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Dispatch
// ---------------------------------------------------------------------------
template <int DP, int FAM>
static hipError_t dispatch_modes(const EvalArgs &a, int center, bool fd, bool grad, dim3 grid, hipStream_t st) {
    const dim3 block(kWave);
#define CHISAO_GO(C, G, F) hipLaunchKernelGGL((eval_kernel<DP, FAM, G, C, F, 1>), grid, block, 0, st, a)
#define CHISAO_GO_HALF(G) hipLaunchKernelGGL((eval_kernel<DP, FAM, G, kDirect, false, 1, true>), grid, block, 0, st, a)
#define CHISAO_GO_SPLIT(C, G, F)                                                                       \
    hipLaunchKernelGGL((eval_kernel<DP, FAM, G, C, F, trial_split<DP, FAM>()>), grid, dim3(kWave * trial_split<DP, FAM>()), 0, \
                       st, a)
    constexpr bool kHalfOk = FAM < kFamClosed && DP != kAluDP;  // tiles of two MFMA column blocks
    if (center == kDirect) {
        if (fd) CHISAO_GO(kDirect, false, true);
        else if (kHalfOk && a.half_tiles) {
            if constexpr (kHalfOk) {
                if (grad) CHISAO_GO_HALF(true);
                else CHISAO_GO_HALF(false);
            }
        } else if (grad) CHISAO_GO(kDirect, true, false);
        else CHISAO_GO(kDirect, false, false);
    } else if (center == kTrial) {
        if (grad) CHISAO_GO_SPLIT(kTrial, true, false);
        else CHISAO_GO_SPLIT(kTrial, false, false);
    } else {
        if (fd) CHISAO_GO(kProbe, false, true);
        else CHISAO_GO(kProbe, true, false);
    }
#undef CHISAO_GO
#undef CHISAO_GO_HALF
#undef CHISAO_GO_SPLIT
    return hipGetLastError();
}

// Workgroups of a line-search launch resident at once on the current device
// (the occupancy of the class's split trial kernel times the CU count), or 0
// where line-search tiles are not split.
template <int DP, int FAM>
static int trial_resident(bool grad) {
    constexpr int S = trial_split<DP, FAM>();
    if constexpr (S == 1) {
        return 0;
    } else {
        int nb = 0, dev = 0, cus = 0;
        const hipError_t e = grad ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                        &nb, eval_kernel<DP, FAM, true, kTrial, false, S>, kWave * S, 0)
                                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                        &nb, eval_kernel<DP, FAM, false, kTrial, false, S>, kWave * S, 0);
        if (e != hipSuccess || hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
            (void)hipGetLastError();  // no limit then; leave no error for later launches to report
            return 0;
        }
        return nb * cus;
    }
}

int trial_resident_blocks(int DP, int family, bool grad) {
    if (family >= kFamClosed) return 0;
    switch (DP) {
        case 16: return family == 0 ? trial_resident<16, 0>(grad) : trial_resident<16, 1>(grad);
        case 32: return family == 0 ? trial_resident<32, 0>(grad) : trial_resident<32, 1>(grad);
        case 64: return family == 0 ? trial_resident<64, 0>(grad) : trial_resident<64, 1>(grad);
        default: return 0;
    }
}

hipError_t launch_eval(const EvalArgs &a, int DP, int family, int center, bool fd, bool grad, hipStream_t st) {
    if (a.max_tiles <= 0 || a.n_cls <= 0) return hipSuccess;
    if (a.n_cls > kMaxClass) return hipErrorInvalidValue;
    const long cap = a.grid_cap > 0 ? a.grid_cap : 8192;
    // max_tiles counts 32-point tiles; half tiles are twice as many
    const long tiles = (center == kDirect && !fd && a.half_tiles) ? 2 * a.max_tiles : a.max_tiles;
    long g = tiles < cap ? tiles : cap;
    if (a.order == 1) g = (g + 7) / 8 * 8;  // whole rounds over the XCDs
    const dim3 grid((unsigned)g);
    // the closed forms share one instantiation per padded dimension and
    // select the function per problem
    const int fam = family >= kFamClosed ? kFamClosed : family;
#define CHISAO_FAMS(DPV)                                                                  \
    fam == 0   ? dispatch_modes<DPV, 0>(a, center, fd, grad, grid, st)                   \
    : fam == 1 ? dispatch_modes<DPV, 1>(a, center, fd, grad, grid, st)                   \
               : dispatch_modes<DPV, kFamClosed>(a, center, fd, grad, grid, st)
    switch (DP) {
        case kAluDP:  // mixtures only
            return fam == 0   ? dispatch_modes<kAluDP, 0>(a, center, fd, grad, grid, st)
                   : fam == 1 ? dispatch_modes<kAluDP, 1>(a, center, fd, grad, grid, st)
                              : hipErrorInvalidValue;
        case 16: return CHISAO_FAMS(16);
        case 32: return CHISAO_FAMS(32);
        case 64: return CHISAO_FAMS(64);
        default: return hipErrorInvalidValue;
    }
#undef CHISAO_FAMS
}

// ---------------------------------------------------------------------------
// Per-component constants.  One workgroup per component: float64 Cholesky of
// the precision matrix for log|P_k| (setup only), then the MFMA fragment
// layouts (or, at the VALU width, the component records).  bad[0] is set when
// a matrix is not positive definite.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void prepare_kernel(int family, int d, int DP, int K, float nu, const float *log_w,
                                                     const float *mu, const float *prec, float *logc2, float *Pfrag,
                                                     float *muB, int *bad) {
    const int k = blockIdx.x;
    const int lane = threadIdx.x;
    __shared__ double L[64 * 64];
    __shared__ double diag_log[64];
    const float *A = prec + (size_t)k * d * d;
    for (int e = lane; e < d * d; e += 64) L[e] = (double)A[e];
    __syncthreads();
    // right-looking Cholesky, one column at a time
    for (int j = 0; j < d; ++j) {
        if (lane == 0) {
            double v = L[j * d + j];
            if (!(v > 0.0)) {
                atomicExch(bad, 1);
                v = 1.0;
            }
            L[j * d + j] = sqrt(v);
            diag_log[j] = log(L[j * d + j]);
        }
        __syncthreads();
        for (int i = j + 1 + lane; i < d; i += 64) L[i * d + j] /= L[j * d + j];
        __syncthreads();
        for (int e = lane; e < (d - j - 1) * (d - j - 1); e += 64) {
            const int i = j + 1 + e / (d - j - 1), c = j + 1 + e % (d - j - 1);
            if (c <= i) L[i * d + c] -= L[i * d + j] * L[c * d + j];
        }
        __syncthreads();
    }
    if (lane == 0) {
        double logdet = 0.0;
        for (int j = 0; j < d; ++j) logdet += 2.0 * diag_log[j];
        const double log_2pi = 1.8378770664093454835606594728112;
        double c;
        if (family == 0) {
            c = -0.5 * d * log_2pi + 0.5 * logdet;
        } else {
            c = lgamma(0.5 * ((double)nu + d)) - lgamma(0.5 * (double)nu) - 0.5 * d * log((double)nu * M_PI) +
                0.5 * logdet;
        }
        logc2[k] = (float)(((double)log_w[k] + c) * 1.4426950408889634);
        if (DP == kAluDP) {
            const int W = alu_width(d), T = W * (W + 1) / 2;
            Pfrag[(size_t)k * alu_record(W) + T + W] = logc2[k];
        }
    }
    if (DP == kAluDP) {
        // one record per component: upper triangle of P row by row, mu, and
        // (above) the log2 weight; coordinates past d are zero
        const int W = alu_width(d), T = W * (W + 1) / 2, R = alu_record(W);
        float *rec = Pfrag + (size_t)k * R;
        for (int e = lane; e < T; e += 64) {
            int i = 0, r = e;
            while (r >= W - i) {
                r -= W - i;
                ++i;
            }
            const int j = i + r;
            rec[e] = (i < d && j < d) ? A[i * d + j] : 0.0f;
        }
        if (lane < W) rec[T + lane] = lane < d ? mu[(size_t)k * d + lane] : 0.0f;
        if (lane > 0 && lane < R - T - W) rec[T + W + lane] = 0.0f;
        return;
    }
    // fragments with permuted rows: Pfrag[k][ks][lane][mb] = P[pi][4 ks + lane/16],
    // pi = 4 (4 mb + rho % 4) + rho / 4 for rho = lane % 16
    const int KS = DP / 4, MB = DP / 16;
    for (int ks = 0; ks < KS; ++ks)
        for (int mb = 0; mb < MB; ++mb) {
            const int rho = lane & 15;
            const int row = 4 * (4 * mb + (rho & 3)) + (rho >> 2), col = 4 * ks + (lane >> 4);
            const float v = (row < d && col < d) ? A[row * d + col] : 0.0f;
            Pfrag[(((size_t)k * KS + ks) * 64 + lane) * MB + mb] = v;
        }
    // centres in B-operand order: muB[k][g][ks] = mu[4 ks + g]
    if (lane < 4 * KS) {
        const int gg = lane / KS, i = lane % KS;
        const int cb = 4 * i + gg;
        muB[((size_t)k * 4 + gg) * KS + i] = cb < d ? mu[(size_t)k * d + cb] : 0.0f;
    }
}

hipError_t launch_prepare(int family, int d, int DP, int K, float nu, const float *log_w, const float *mu,
                          const float *prec, float *logc2, float *Pfrag, float *muB, int *bad, hipStream_t st) {
    hipLaunchKernelGGL(prepare_kernel, dim3(K), dim3(64), 0, st, family, d, DP, K, nu, log_w, mu, prec, logc2,
                       Pfrag, muB, bad);
    return hipGetLastError();
}

}  // namespace chisao
