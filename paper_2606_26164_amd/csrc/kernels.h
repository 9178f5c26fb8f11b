// Host-side launchers of the libchisao kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"

namespace chisao {

enum Center { kDirect = 0, kTrial = 1, kProbe = 2 };

// One batched evaluation of the objective at generated points, over the
// problems of one class (same padded dimension and family).  A job is one sample; it expands
// into Vc centres (the sample itself, line-search trials, or smoothing probes)
// and, with finite differences, each centre into a 2d-point stencil.  Tiles
// of 32 points never straddle two problems.
enum VcKind { kVcOne = 0, kVcTrialFirst = 1, kVcTrialRest = 2, kVcProbes = 3 };

struct EvalArgs {
    Dev D;
    const int *cls;       // device: problem ids of this class
    int n_cls;
    long max_tiles;       // upper bound on the tile count (sizes the grid)
    const float *X;       // rows the centres are built from
    int x_stride;         // DS for the population, d for caller memory
    int ext_n;            // >= 0: caller memory, jobs 0..ext_n-1 of problem cls[0]; -1: population lists
    int list_id;          // population jobs: list id, or -1 for every sample of the problem
    int vc_kind;          // VcKind
    int step;             // step index: smoothing/anti step, L-BFGS iteration (noise stream)
    float *F_out;         // direct centres: value per job row (may be null)
    float *G_out;         // direct centres: gradient rows (may be null)
    int out_stride;
    int trial_next;       // trial centres: -1 when no later stage follows (a search none of whose trials passes fails)
    int trial_lo, trial_cnt;  // kVcTrialRest: trials trial_lo .. trial_lo + trial_cnt - 1, capped at ls_max
    int need_bit;         // phase_mask bit a problem must have set to take part (0: none)
    int step_limit;       // 1: only problems with step < n_cloud, 2: step < n_anti, 0: all
    int order;            // tile order: 0 linear, 1 XCD-chunked (block b runs on XCD b % 8)
    int grid_cap;         // most workgroups launched (0: 8192); a multiple of 8 with order 1
    int nz_kind;          // evaluation noise of noisy problems: -1 none, 0 one draw per value, 1 gate mean
    int half_tiles;       // direct value (+ gradient) launches of matrix-core classes: 16-point tiles
    uint32_t nz_base;     // noise sub-stream base (kind 0); the noise step is `step`
};

// center: kDirect / kTrial / kProbe; fd: stencil around each centre;
// grad: accumulate the adjoint gradient.
hipError_t launch_eval(const EvalArgs &a, int DP, int family, int center, bool fd, bool grad, hipStream_t st);

// Workgroups of a class's line-search launch that are resident at once on the
// current GPU (0: no limit applies).  Line-search launches use that many
// workgroups, each looping over tiles: one round of persistent workgroups
// instead of a queue of one-tile workgroups.
int trial_resident_blocks(int DP, int family, bool grad);

// Per-component constants: log2 normalisers (float64 Cholesky of each
// precision matrix) and the fragment layouts of the precision matrices and
// centres.  Writes D.logc2/Pfrag/muB (device buffers passed as mutable).
hipError_t launch_prepare(int family, int d, int DP, int K, float nu, const float *log_w, const float *mu,
                          const float *prec, float *logc2, float *Pfrag, float *muB, int *bad, hipStream_t st);

// Cycle kernels (phases 1-6 and their bookkeeping).
hipError_t launch_fill_u8(uint8_t *p, uint8_t v, size_t n, hipStream_t st);
hipError_t launch_uniform_init(const Dev &D, hipStream_t st);
hipError_t launch_begin_cycle(const Dev &D, hipStream_t st);
// Zero the counts of the lists in `mask` of the problems pids[0 .. np)
// (device array), or of every problem when pids is null.
hipError_t launch_reset_counts(const Dev &D, int mask, hipStream_t st, const int *pids = nullptr, int np = 0);
// Stream compaction of the list `src` by D.flag: for each problem, position j
// of src's segment (j < its count) with flag[j] == v is appended to list
// dst[v - 1] (v = 1, 2; -1: none); positions with flag == 3 are counted into
// the problem's ls_fail.  Entries keep ascending position order within a
// block.  The number appended for v = 1 is added to *tally when not null, and
// the history pair counts (D.cnt) of those samples to *tally_pairs.  Only the
// positions [g0, g0 + n) are scanned (n < 0: all), which must hold whole
// problems.
hipError_t launch_compact(const Dev &D, int src, int dst1, int dst2, bool count_fail, unsigned long long *tally,
                          hipStream_t st, unsigned long long *tally_pairs = nullptr, int g0 = 0, int n = -1);
hipError_t launch_build_unfrozen(const Dev &D, hipStream_t st);
// Iteration t of the L-BFGS loop for the samples on list `list_in` (all
// active samples at t = 1, the previous iteration's steppers after), over the
// list positions [g0, g0 + n) of a set of whole problems, all with
// d <= 16 cpl; D.flag of a position is set to 1 when its sample was given a
// direction, else 0.
hipError_t launch_lbfgs_step(const Dev &D, int t, int cpl, int list_in, int g0, int n, hipStream_t st);
hipError_t launch_stick(const Dev &D, hipStream_t st);
hipError_t launch_dedup(const Dev &D, hipStream_t st);
hipError_t launch_reseed(const Dev &D, hipStream_t st);
hipError_t launch_sigma(const Dev &D, hipStream_t st);
// The per-problem exploration kernels below cover the problems pids[0 .. np)
// (device array), or every problem when pids is null.
hipError_t launch_probe_mean(const Dev &D, int step, hipStream_t st, const int *pids = nullptr, int np = 0);
hipError_t launch_step_size(const Dev &D, const float *Gsrc, int which, hipStream_t st, const int *pids = nullptr,
                            int np = 0);
hipError_t launch_hlc_update(const Dev &D, int step, hipStream_t st, const int *pids = nullptr, int np = 0);
hipError_t launch_anti_update(const Dev &D, int step, hipStream_t st, const int *pids = nullptr, int np = 0);
hipError_t launch_end_cycle(const Dev &D, int advance, hipStream_t st);
hipError_t launch_mode_list(const Dev &D, int p, int s0, int N, hipStream_t st);
hipError_t launch_width_list(const Dev &D, int p, int N, hipStream_t st);
// Mode export of problem p: its stuck active samples in ascending index, rows
// to D.Gh and values to D.Pd from row/element s0, count in ctl[p].count[O_PEAKS].

}  // namespace chisao
