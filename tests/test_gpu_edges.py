"""Edge cases of the boundary: degenerate problems (one sample, one
dimension, one component), the largest history / probe / line-search sizes
the ABI accepts, and a batch mixing them with noisy and finite-difference
problems."""
import numpy as np
import pytest

import workloads as W
from oracle import oracle as O

from test_gpu_batch import _assert_same, _state
from test_gpu_phases import REPLAY, _gpu, _oracle_from, _rows_close

pytestmark = pytest.mark.gpu


def _tiny():
    p = W.mixture_problem(61, 1, 1, 2.0, lam_range=(0.5, 0.5))
    c = W.RunConfig(N=1, m=3, n_osc=3, n_conv=10, M=2, eps_grad=1e-4, grad_mode=1, seed=2)
    return p, c, W.uniform_population(61, 1, p.lo, p.hi)


def test_one_sample_one_dimension_one_component():
    """N = d = K = 1: the single sample climbs to the single centre, sticks,
    and is the mode set."""
    from paper_2606_26164_amd.api import Optimizer

    prob, cfg, x0 = _tiny()
    with Optimizer(prob, cfg, x0) as opt:
        stats = opt.cycle(cfg.n_osc, stats=True)
        ms = opt.modes()
    assert [s["k"] for s in stats] == [1, 2, 3]
    assert len(ms.X) == 1
    np.testing.assert_allclose(ms.X[0], prob.mu[0], atol=1e-4)
    f_peak = O.OracleProblem(prob).eval(prob.mu.astype(np.float64), grad=False)[0]
    assert ms.F[0] == pytest.approx(f_peak, abs=1e-5)


def test_largest_history_probe_and_search_sizes():
    """m = 32, M = 32, ls_max = 15 (the ABI's limits) at d = 64: Phase 1 with
    replay and Phases 5-6 against the oracle; ls_max = 16 is refused."""
    prob = W.mixture_problem(62, 64, 6, 10.0, lam_range=(0.2, 1.0))
    from paper_2606_26164_amd import _lib as L

    # one smoothing and one anti step: after 40 iterations most samples sit at
    # modes, the step length rule gives sigma / mean |g| in the hundreds, and
    # further steps would compound FP32 rounding by that factor
    cfg = W.RunConfig(N=96, m=32, n_osc=3, n_conv=40, M=32, ls_max=15, sigma=0.2, eps_grad=1e-3, grad_mode=1,
                      n_cloud=1, n_anti=1, seed=8)
    x0 = W.uniform_population(62, 96, prob.lo, prob.hi)
    with pytest.raises(L.ChisaoError) as ei:
        _gpu(prob, cfg.with_(ls_max=16), x0)
    assert ei.value.code == L.E_INVAL
    with _gpu(prob, cfg, x0) as opt:
        opt.run_phases(1 << 1)
        g1 = opt.get_state(history=True)
        opt.run_phases((1 << 2) | (1 << 3) | (1 << 4))
        g4 = opt.get_state()
        opt.run_phases((1 << 5) | (1 << 6))
        g6 = opt.get_state()
    assert g1["cnt"].max() > 10  # histories longer than the default m were used
    run = O.OracleRun(prob, cfg, x0)
    rep = run.phase_converge(trace_in=g1["trace"], **REPLAY)
    assert rep.n_hard == 0, rep
    _rows_close(g1["X"], run.X, 1e-4, "X after phase 1 (m=32, ls_max=15)")
    later = _oracle_from(prob, cfg, g4)
    later.phase_hlc()
    later.phase_anti()
    # The smoothed gradient of a sample sitting at a mode is a small mean of
    # antithetic probe gradients of size ~ lam_max sigma sqrt(d): FP32
    # cancellation there costs ~64 u (lam_max sigma sqrt(d)) / |g_hat|
    # relative, which the step length sigma / mean |g_hat| carries into the
    # displacement.
    moved = g4["stuck"] == 0
    lam_max = max(np.linalg.eigvalsh(prob.prec[k].astype(np.float64)).max() for k in range(prob.K))
    probe_scale = lam_max * cfg.sigma * np.sqrt(prob.d)
    d_gpu = (g6["X"][moved].astype(np.float64) - g4["X"][moved])
    d_or = later.X[moved] - g4["X"][moved]
    g_hat = np.abs(d_or).max(1) / later.st.alpha_c  # |g_hat|_inf of the first smoothing step, up to the anti step
    tol = 1e-4 + 64 * 2.0 ** -24 * probe_scale / np.maximum(g_hat, 1e-30)
    err = np.abs(d_gpu - d_or).max(1) / np.maximum(np.abs(d_or).max(1), 1e-3)
    print(f"\nphase 5-6 (M=32): relative error max {err.max():.2e}, bound at that row {tol[np.argmax(err)]:.2e}")
    assert np.all(err <= tol)


def test_batch_mixing_degenerate_noisy_and_fd_problems():
    """A batch of a one-sample problem, a noisy Student-t problem and a
    finite-difference problem gives each exactly its single-handle result."""
    from paper_2606_26164_amd.api import Optimizer

    tiny = _tiny()
    pn = W.mixture_problem(63, 12, 8, 4.0, lam_range=(0.3, 1.0), family=W.STUDENT_T, nu=3.0, noise_sigma=0.5)
    cn = W.RunConfig(N=400, m=6, n_osc=3, n_conv=10, M=8, eps_grad=1e-3, grad_mode=1, gate_reps=16, seed=5,
                     problem_id=1)
    pf = W.mixture_problem(64, 20, 6, 5.0, lam_range=(0.3, 1.0))
    cf = W.RunConfig(N=300, m=5, n_osc=3, n_conv=10, M=4, eps_grad=1e-3, grad_mode=0, seed=5, problem_id=2)
    items = [tiny, (pn, cn, W.uniform_population(63, 400, pn.lo, pn.hi)),
             (pf, cf, W.uniform_population(64, 300, pf.lo, pf.hi))]
    with Optimizer.batched(items) as opt:
        opt.cycle(3)
        got = [_state(opt, p) for p in range(len(items))]
    for p, (prob, cfg, x0) in enumerate(items):
        with Optimizer(prob, cfg, x0) as one:
            one.cycle(3)
            _assert_same(got[p], _state(one), f"problem {p}")
