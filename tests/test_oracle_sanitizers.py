"""The oracle under the host sanitizers: a small C driver, compiled together
with oracle/chisao_oracle.c by gcc with AddressSanitizer and
UndefinedBehaviorSanitizer (host code only, no OpenMP), runs whole cycles of
several problem shapes that reach every phase: both gradient modes, Student-t
with evaluation noise and the quality gate, a single-component mixture that
forces Golden Rooster, a closed form, and the structured ray seeding.  Any
invalid access, leak or undefined operation aborts the driver."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "chisao_oracle.c")

DRIVER = r"""
#include <stdio.h>
#include "chisao_oracle.c"

static uint64_t lcg = 88172645463325252ull;
static double urand(void)
{
    lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(lcg >> 11) * (1.0 / 9007199254740992.0);
}

/* family, d, K, N, grad_mode, noise, flags: one run of n_osc cycles */
static int run(int family, int d, int K, int N, int grad_mode, double noise, uint32_t flags, int n_osc)
{
    int closed = family >= FAM_RASTRIGIN;
    int Kc = closed ? 0 : K;
    double *log_w = malloc(sizeof(double) * (Kc + 1)), *mu = malloc(sizeof(double) * (Kc * d + 1));
    double *prec = malloc(sizeof(double) * (Kc * d * d + 1)), *lo = malloc(sizeof(double) * d);
    double *hi = malloc(sizeof(double) * d), *logc = malloc(sizeof(double) * (Kc + 1));
    for (int c = 0; c < d; ++c) { lo[c] = closed ? -5.12 : -3.0; hi[c] = closed ? 5.12 : 3.0; }
    for (int k = 0; k < Kc; ++k) {
        log_w[k] = log(1.0 / Kc);
        for (int c = 0; c < d; ++c) mu[k * d + c] = -2.0 + 4.0 * urand();
        for (int i = 0; i < d * d; ++i) prec[(size_t)k * d * d + i] = 0.0;
        for (int c = 0; c < d; ++c) prec[(size_t)k * d * d + c * d + c] = 1.0 / (0.3 + 0.7 * urand());
        if (d > 1) { /* a symmetric off-diagonal pair, still diagonally dominant */
            prec[(size_t)k * d * d + 1] = 0.1;
            prec[(size_t)k * d * d + d] = 0.1;
        }
    }
    orc_problem P = {family, d, K, 3.0, log_w, mu, prec, lo, hi, noise};
    int m = 5, n_conv = 10, M = 6;
    orc_config C = {N, m, n_osc, n_conv, 5, 3, M, 1e-3, 1e-3, log(0.1), 0.9, 0.0, 0.0, 0.1, grad_mode,
                    0.0, 1e-4, 10, 1e-10, noise > 0 ? 8 : 0, 0x7E, 12345ull, 7u, flags};
    if (!closed && orc_prepare(&P, logc)) return 10;
    size_t Nd = (size_t)N * d;
    orc_state S;
    memset(&S, 0, sizeof S);
    S.X = calloc(Nd, sizeof(double)); S.F = calloc(N, sizeof(double)); S.G = calloc(Nd, sizeof(double));
    S.V = calloc(Nd, sizeof(double));
    S.stuck = calloc(N, 1); S.active = malloc(N); S.conv = calloc(N, 1); S.removed = calloc(N, 1);
    S.S = calloc(Nd * m, sizeof(double)); S.Y = calloc(Nd * m, sizeof(double));
    S.rho = calloc((size_t)N * m, sizeof(double));
    S.head = malloc(sizeof(int32_t) * N); S.cnt = calloc(N, sizeof(int32_t));
    S.Fg = calloc(N, sizeof(double)); S.W = calloc(Nd, sizeof(double)); S.wvalid = calloc(N, 1);
    for (int i = 0; i < N; ++i) { S.active[i] = 1; S.head[i] = m - 1; }
    uint8_t *trace = malloc((size_t)(n_conv + 1) * N);
    orc_init_population(&P, &C, S.X);
    int rc = 0, kinds = 0;
    for (int k = 0; k < n_osc && !rc; ++k) {
        orc_replay R;
        memset(&R, 0, sizeof R);
        R.trace_out = trace;
        R.tol_f = 1e-4; R.tol_g = 0.2; R.tol_curv = 1e-2; R.tol_dist = 1e-5;
        R.first_hard_sample = R.first_hard_iter = -1;
        rc = orc_cycle(&P, logc, &C, &S, &R);
        kinds |= 1 << S.reseed_kind;
    }
    /* batched evaluation, finite differences and the QR on the final state */
    double *f = malloc(sizeof(double) * N), *G = malloc(sizeof(double) * Nd);
    orc_eval_batch(&P, logc, N, S.X, f, G);
    orc_fd_grad_batch(&P, logc, 0.0, N, S.X, G);
    double *A = malloc(sizeof(double) * d * d), *Q = malloc(sizeof(double) * d * d), *Rm = malloc(sizeof(double) * d * d);
    for (int i = 0; i < d * d; ++i) A[i] = urand() - 0.5;
    if (!rc) rc = orc_householder_q(d, A, Q, Rm) ? 11 : 0;
    printf("family %d d %d K %d N %d grad %d noise %g flags %u: rc %d, k %d, modes %d, reseed kinds %d\n", family, d,
           K, N, grad_mode, noise, flags, rc, S.k, S.n_modes, kinds);
    free(A); free(Q); free(Rm); free(f); free(G); free(trace);
    free(S.X); free(S.F); free(S.G); free(S.V); free(S.stuck); free(S.active); free(S.conv); free(S.removed);
    free(S.S); free(S.Y); free(S.rho); free(S.head); free(S.cnt); free(S.Fg); free(S.W); free(S.wvalid);
    free(log_w); free(mu); free(prec); free(lo); free(hi); free(logc);
    return rc;
}

int main(void)
{
    int rc = 0;
    rc |= run(FAM_GAUSS, 3, 4, 96, 1, 0.0, 0u, 4);          /* adjoint */
    rc |= run(FAM_GAUSS, 4, 3, 48, 0, 0.0, 0u, 3);          /* central differences */
    rc |= run(FAM_STUDENT_T, 5, 3, 64, 1, 0.5, 0u, 3);      /* noise, the quality gate, Repulse Monkey */
    rc |= run(FAM_GAUSS, 6, 1, 40, 1, 0.0, 0u, 4);          /* one peak: Golden Rooster, then disabled */
    rc |= run(FAM_RASTRIGIN, 4, 0, 64, 0, 0.0, 0u, 3);      /* a closed form */
    rc |= run(FAM_GAUSS, 6, 5, 64, 1, 0.0, 4u, 3);          /* structured ray seeding */
    return rc;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_cycles_are_clean_under_address_and_undefined_behavior_sanitizers():
    with tempfile.TemporaryDirectory() as td:
        c = os.path.join(td, "driver.c")
        with open(c, "w") as fh:
            fh.write(DRIVER)
        exe = os.path.join(td, "driver")
        cmd = ["gcc", "-std=c11", "-D_GNU_SOURCE", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
               "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-I", os.path.dirname(SRC), c, "-o",
               exe, "-lm"]
        subprocess.run(cmd, check=True, capture_output=True)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
        r = subprocess.run([exe], capture_output=True, text=True, timeout=240, env=env)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.startswith("family")]
    assert len(lines) == 6 and all("rc 0" in ln for ln in lines)
    # the runs reached every reseeding outcome (bit 1: Repulse Monkey, bit 2:
    # Golden Rooster, bit 3: Golden Rooster disabled and the slots deactivated)
    kinds = [int(ln.rsplit(" ", 1)[1]) for ln in lines]
    assert all(any(k & b for k in kinds) for b in (2, 4, 8)), kinds
