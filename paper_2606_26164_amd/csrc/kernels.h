// Host-side launchers of the libchisao kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"

namespace chisao {

enum Center { kDirect = 0, kTrial = 1, kProbe = 2 };

// One batched evaluation of the objective at generated points.
// A job is one sample (list[job], or job itself without a list); it expands
// into Vc centres (the sample itself, line-search trials, or smoothing
// probes), and with finite differences each centre into a 2d-point stencil.
struct EvalArgs {
    Dev D;
    const float *X;         // rows of the samples the centres are built from (stride d)
    const int *list;        // job -> sample index (nullptr: identity)
    const int *count_ptr;   // device job count (nullptr: n_jobs)
    int n_jobs;             // upper bound on the job count (sizes the grid)
    int Vc;                 // centres per job
    int r0;                 // backtracking index of the first trial centre
    int step;               // smoothing step index (probe stream)
    float *F_out;           // direct centres: value per sample (may be null)
    float *G_out;           // direct centres: gradient rows per sample (may be null)
    int trial_next;         // trial centres: list receiving rejected samples (-1: mark failed)
};

// center: kDirect / kTrial / kProbe; fd: stencil around each centre;
// grad: accumulate the adjoint gradient.
hipError_t launch_eval(const EvalArgs &a, int center, bool fd, bool grad, hipStream_t st);

// Per-component constants: log2 normalisers (float64 Cholesky of each
// precision matrix) and the fragment layouts of the precision matrices and
// centres.  Writes D.logc2/Pfrag/muB/muC (device buffers passed as mutable).
hipError_t launch_prepare(int family, int d, int DP, int K, float nu, const float *log_w, const float *mu,
                          const float *prec, float *logc2, float *Pfrag, float *muB, float *muC, int *bad,
                          hipStream_t st);

// Cycle kernels (phases 1-6 and their bookkeeping).
hipError_t launch_fill_u8(uint8_t *p, uint8_t v, size_t n, hipStream_t st);
hipError_t launch_uniform_init(const Dev &D, hipStream_t st);
hipError_t launch_begin_cycle(const Dev &D, hipStream_t st);
hipError_t launch_reset_counts(const Dev &D, int mask, hipStream_t st);
hipError_t launch_build_list(const Dev &D, int which, hipStream_t st);
hipError_t launch_lbfgs_step(const Dev &D, int t, hipStream_t st);
hipError_t launch_stick(const Dev &D, hipStream_t st);
hipError_t launch_dedup(const Dev &D, hipStream_t st);
hipError_t launch_reseed(const Dev &D, hipStream_t st);
hipError_t launch_sigma(const Dev &D, hipStream_t st);
hipError_t launch_probe_mean(const Dev &D, hipStream_t st);
hipError_t launch_step_size(const Dev &D, const float *Gsrc, int which, hipStream_t st);
hipError_t launch_hlc_update(const Dev &D, hipStream_t st);
hipError_t launch_anti_update(const Dev &D, int step, hipStream_t st);
hipError_t launch_end_cycle(const Dev &D, int advance, hipStream_t st);
// Mode export: stuck active samples in ascending index; rows to D.Gh, values to D.Pd,
// count in ctl->count[O_PEAKS].
hipError_t launch_mode_list(const Dev &D, hipStream_t st);

}  // namespace chisao
