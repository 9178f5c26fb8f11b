// Device-side definitions shared by the libchisao kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "chisao.h"

namespace chisao {

constexpr int kWave = 64;
// objective families from here on are closed-form test functions
constexpr int kFamClosed = CHISAO_RASTRIGIN;

// Evaluation width.  Mixtures with d <= 8 run on the VALU, one lane per
// point (padded width kAluDP); larger d, and the closed forms, run in tiles
// padded to 16, 32 or 64 coordinates.
constexpr int kAluDP = 8;
__host__ __device__ constexpr int pad_dim(int d, int family) {
    return (family < kFamClosed && d <= kAluDP) ? kAluDP : (d <= 16 ? 16 : (d <= 32 ? 32 : 64));
}
// Within the VALU path a problem's components are W = 2, 4 or 8 wide and
// stored as one record each: the upper triangle of P_k row by row
// (W (W + 1) / 2 values), then mu_k (W), then log2 of weight times
// normaliser, padded to a multiple of four floats.  At most 48 floats, so a
// record table fits the K * 8 * 8 floats of a width-8 fragment table.
__host__ __device__ constexpr int alu_width(int d) { return d <= 2 ? 2 : (d <= 4 ? 4 : 8); }
__host__ __device__ constexpr int alu_record(int W) { return (W * (W + 1) / 2 + W + 1 + 3) / 4 * 4; }

// ---------------------------------------------------------------------------
// Counter-based random streams: Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
// SC'11), ten rounds with the Weyl key schedule.  The counter words are
// (index, cycle, consumer << 24 | step << 16 | sub, block); the key is the
// 64-bit seed with the problem id folded into the high word.
// ---------------------------------------------------------------------------
enum Stream : uint32_t { kInit = 0, kRM = 4, kGR = 5, kHLC = 6, kNoise = 7, kGate = 8 };

__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                        uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    return make_uint4(c0, c1, c2, c3);
}

// (top 24 bits + 1/2) * 2^-24: exact in float, strictly inside (0, 1).
__device__ __forceinline__ float u01(uint32_t a) { return ((float)(a >> 8) + 0.5f) * (1.0f / 16777216.0f); }

// Box-Muller on the uniform pairs (o.x, o.y) and (o.z, o.w).
__device__ __forceinline__ void box_muller4(uint4 o, float z[4]) {
    float s, c;
    float r = sqrtf(-2.0f * logf(u01(o.x)));
    sincospif(2.0f * u01(o.y), &s, &c);
    z[0] = r * c;
    z[1] = r * s;
    r = sqrtf(-2.0f * logf(u01(o.z)));
    sincospif(2.0f * u01(o.w), &s, &c);
    z[2] = r * c;
    z[3] = r * s;
}

// integer in [0, n): high word of the 64-bit product
__device__ __forceinline__ uint32_t uint_below(uint32_t a, uint32_t n) { return __umulhi(a, n); }

// ---------------------------------------------------------------------------
// Wave-wide reductions (all 64 lanes participate and receive the result).
// ---------------------------------------------------------------------------
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, kWave));
    return v;
}
__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, kWave));
    return v;
}

// Reductions over the 16 lanes of a DPP row (lanes 16r .. 16r+15), with
// every lane of the row receiving the same, bitwise identical result:
// quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror, row_mirror.
// All 64 lanes must be active.
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ float row16_sum(float v) {
    v += dpp_mov<0xB1>(v);
    v += dpp_mov<0x4E>(v);
    v += dpp_mov<0x141>(v);
    v += dpp_mov<0x140>(v);
    return v;
}
__device__ __forceinline__ float row16_max(float v) {
    v = fmaxf(v, dpp_mov<0xB1>(v));
    v = fmaxf(v, dpp_mov<0x4E>(v));
    v = fmaxf(v, dpp_mov<0x141>(v));
    v = fmaxf(v, dpp_mov<0x140>(v));
    return v;
}

// Sum over the four 16-lane rows (lanes l, l^16, l^32, l^48) with the gfx950
// row-swap permutes (no LDS traffic); every lane receives the same bits.
__device__ __forceinline__ float rows4_sum(float v) {
    const auto a = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    v = __uint_as_float(a[0]) + __uint_as_float(a[1]);
    const auto b = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return __uint_as_float(b[0]) + __uint_as_float(b[1]);
}

// Two values per lane summed over the four rows at once: on return rows 0
// and 2 hold the row sum of a, rows 1 and 3 that of b, each added in the
// order of rows4_sum ((r0 + r1) + (r2 + r3)), so bitwise the same.
__device__ __forceinline__ float rows4_sum_pair(float a, float b) {
    const auto s = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    const float h = __uint_as_float(s[0]) + __uint_as_float(s[1]);
    const auto t = __builtin_amdgcn_permlane32_swap(__float_as_uint(h), __float_as_uint(h), false, false);
    return __uint_as_float(t[0]) + __uint_as_float(t[1]);
}
// The inverse split: x holds a value of block 0 in rows 0 and 2 and one of
// block 1 in rows 1 and 3; every lane receives both.
__device__ __forceinline__ void rows_pair_split(float x, float &b0, float &b1) {
    const auto s = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(x), false, false);
    b0 = __uint_as_float(s[0]);
    b1 = __uint_as_float(s[1]);
}

// Total order on floats as signed ints, for exact atomic max.
__device__ __forceinline__ int float_to_ordered(float f) {
    int i = __float_as_int(f);
    return i >= 0 ? i : i ^ 0x7FFFFFFF;
}
__host__ __device__ inline float ordered_to_float(int i) {
    int b = i >= 0 ? i : i ^ 0x7FFFFFFF;
    union {
        int i;
        float f;
    } u;
    u.i = b;
    return u.f;
}

// ---------------------------------------------------------------------------
// Problems.  A handle holds P independent problems; problem p owns the global
// samples [s0, s0 + N).  All per-sample arrays are concatenated, rows have
// the handle-wide stride DS >= d.
// ---------------------------------------------------------------------------
struct ProblemDesc {
    int d, DP, K, family;
    float nu, nu_plus_d;
    const float *Pfrag;  // [K][DP/4][64][DP/16] MFMA A-operand fragments of the precision matrices;
                         // at DP = kAluDP the component records [K][alu_record(W)] instead
    const float *muB;    // [K][4][DP/4]  centre coordinates in B-operand lane order (unused at DP = kAluDP)
    const float *logc2;  // [K] log2 of weight times normaliser
    const float *lo, *hi;
    int N, s0;
    int m, n_conv, n_anti, n_cloud, M, ls_max, grad_mode;
    float eps_grad, eps_dup, log_delta, momentum, alpha, sigma_cfg, sigma_c, fd_h, ls_c1, curv_eps;
    uint32_t key0, key1, phase_mask;
    int ray_seed;       // starting population on rays through the box centre (when none is given)
    float noise_sigma;  // additive evaluation noise (0: none)
    int gate_reps;      // noisy evaluations averaged by the quality gate
    int hk0;            // offset of the problem's 2^hash_lb + 1 deduplication bucket offsets in Dev::hoff
    int hash_lb;        // log2 of the deduplication bucket count (a power of two >= N/4)
};

// ---------------------------------------------------------------------------
// Per-problem control block: counters and scalars that decide the
// data-dependent control flow of a cycle without a host round trip.
// ---------------------------------------------------------------------------
// L_T1 and L_T1B alternate between L-BFGS iterations: one holds the samples
// that took a step in the previous iteration, the other collects this one's.
// L_T2 / L_T3: searches still open after the first trial / after trials 1-2.
// L_HASH: a problem's stuck samples grouped by deduplication hash bucket.
enum ListId { L_ACT = 0, L_T1, L_T1B, L_T2, L_T3, L_FD, L_UNF, L_STK, L_HASH, O_SLOTS, O_FREE, O_PEAKS, kNumLists };

struct Ctl {
    int k;  // cycles completed
    int count[kNumLists];
    int fmax_ord;  // ordered-int image of f_max
    unsigned long long fmax_key;  // largest (value, -index) over the gate values: finds the best sample
    int n_stuck, K_lost, n_modes, n_active;
    int reseed_kind;  // 0 none, 1 RM, 2 GR, 3 deactivate
    int gr_disabled, gr_fail, gr_used_last, gr_prev_modes;
    int ls_fail;
    int n_nonfinite;  // samples deactivated by the non-finite guard of Phase 2
    unsigned long long evals;
    float f_max, sigma, alpha_c, alpha_a;
};

// Per-cycle record kept on the device, copied out on request.
struct CycleRecord {
    int k;
    float f_max;
    int n_stuck, K_lost, n_modes, reseed_kind, n_free, n_unfrozen, n_active;
    float sigma, alpha_c, alpha_a;
    int ls_fail, n_nonfinite;
    unsigned long long evals;
};

// Status bytes written by the line-search epilogue.
constexpr uint8_t kStAccept = 0x80;  // | accepted trial index
constexpr uint8_t kStFail = 0x40;

// Decision-trace codes (one byte per sample and L-BFGS iteration).
constexpr uint8_t kTrNone = 0xFF;
constexpr uint8_t kTrFail = 0x0F;
constexpr uint8_t kTrStored = 0x10;
constexpr uint8_t kTrConv = 0x20;
constexpr uint8_t kTrReset = 0x40;

constexpr int kProfClasses = 8;

// Everything a kernel needs, passed by value.
struct Dev {
    int P, NT, DS, mmax, Mmax, n_conv_max, n_osc;
    const ProblemDesc *pd;   // [P]
    const uint16_t *pid;     // [NT] problem of each sample
    // population state (rows of stride DS)
    float *X, *F, *G, *V, *Xprev, *Gprev, *Pd, *Gh, *Gp, *ginf;
    float *Fg;  // quality-gate values of noisy problems
    float *Wd;         // [NT][DS] preserved inverse-Hessian diagonal of each surviving mode (width export)
    uint8_t *wvalid;   // [NT] Wd holds a value
    uint8_t *stuck, *active, *conv, *removed, *stuck_pre, *status, *reset, *steep, *trace;
    float *S, *Y, *rho;      // [NT][mmax][DS], [NT][mmax]
    int *head, *cnt;
    int *lists;              // kNumLists x NT; problem p's list occupies [s0, s0 + N)
    uint8_t *flag;           // [NT] per list position: a producer's verdict, read by the compaction
    int *hoff;   // deduplication bucket offsets (exclusive scan of the counts), per problem at hk0
    int *hcur;   // scatter cursors, same layout
    int *hcell;  // deduplication hash cell of each stuck sample
    Ctl *ctl;                // [P]
    CycleRecord *records;    // [P][n_osc]
    double *part;            // [P][n_part_blocks][129] reduction partials
    int n_part_blocks;
    unsigned long long *prof;  // [kProfClasses] evaluations per kernel class
};

__device__ __forceinline__ int *list_ptr(const Dev &D, int id, int s0) { return D.lists + (size_t)id * D.NT + s0; }

// The values the quality gate, the deduplication order and the mode output
// use: f as the search saw it, or the gate values of a noisy problem.
__device__ __forceinline__ const float *gate_values(const Dev &D, const ProblemDesc &pd) {
    return pd.noise_sigma > 0.0f ? D.Fg : D.F;
}

// Noise sub-stream offsets (low 16 bits of the third counter word): the
// centre value 0, line-search trial r, and these bases plus the stencil index
// for central differences in Phase 1, smoothing probes (| probe << 7) and
// anti-convergence.
constexpr uint32_t kNzFd1 = 0x1000, kNzFdProbe = 0x2000, kNzFdAnti = 0x3000;

// Lanes with `want` each take one unit of a per-problem counter (counter(p)
// gives its address): one atomic per distinct problem among the wave's lanes
// instead of one per lane.  Returns the counter's previous value plus the
// lane's rank among the lanes of its problem, or -1 without `want`.  Every
// lane of the wave must make the call.
template <class F>
__device__ __forceinline__ int wave_claim(bool want, int p, F counter) {
    const int lane = __lane_id();
    unsigned long long pending = __ballot(want);
    int slot = -1;
    while (pending) {
        const int leader = __ffsll((unsigned long long)pending) - 1;
        const int pl = __shfl(p, leader, kWave);
        const bool mine = want && p == pl;
        const unsigned long long grp = __ballot(mine);
        int base = 0;
        if (lane == leader) base = atomicAdd(counter(pl), (int)__popcll(grp));
        base = __shfl(base, leader, kWave);
        if (mine) slot = base + (int)__popcll(grp & ((1ull << lane) - 1ull));
        pending &= ~grp;
    }
    return slot;
}

// Wave-aggregated append of sample s to list `id` of problem p.
__device__ __forceinline__ void wave_append(const Dev &D, int id, bool want, int p, int s) {
    const int slot = wave_claim(want, p, [&](int q) { return &D.ctl[q].count[id]; });
    if (want) list_ptr(D, id, D.pd[p].s0)[slot] = s;
}

}  // namespace chisao
