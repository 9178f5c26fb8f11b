"""Pins of the oracle's likelihood-noise model (Sec. 5.7: every evaluation
returns f(x) + sigma_n z with a fresh standard normal z) and of the quality
gate's averaging reading (the mean of R fresh noisy evaluations).  The noise
is recovered by subtracting the noise-free value computed independently, so a
wrong amplitude, a reused draw, a missing division by R or a gradient that
picked up noise each fails a distribution test."""
import numpy as np
import scipy.stats

import workloads as W
from oracle import oracle as O

SIGMA = 0.7


def _noisy_problem(family=W.GAUSS):
    return W.mixture_problem(31, 6, 5, 4.0, lam_range=(0.3, 1.0), family=family, nu=3.0, noise_sigma=SIGMA)


def _run(prob, N=20000, **kw):
    cfg = W.RunConfig(N=N, n_conv=1, M=8, eps_grad=1e-3, seed=9, **kw)
    x0 = W.uniform_population(5, N, prob.lo, prob.hi)
    run = O.OracleRun(prob, cfg, x0)
    run.cc.n_conv = 0  # Phase 1 reduced to its starting evaluation (value and gradient at x0)
    return run, cfg, x0


def _assert_standard_normal(z, var=1.0):
    n = len(z)
    assert abs(z.mean()) < 5.0 * np.sqrt(var / n)
    assert abs(z.var() / var - 1.0) < 5.0 * np.sqrt(2.0 / n)
    assert scipy.stats.kstest(z / np.sqrt(var), "norm").pvalue > 1e-4


def test_value_noise_is_sigma_times_fresh_standard_normal_and_gradient_exact():
    prob = _noisy_problem()
    run, cfg, x0 = _run(prob, grad_mode=1)
    run.phase_converge()
    f_clean, g_clean = O.OracleProblem(prob).eval(x0)
    z = (run.F - f_clean) / SIGMA
    _assert_standard_normal(z)
    # noise does not depend on x: the analytic gradient is untouched
    np.testing.assert_array_equal(run.G, g_clean)
    # the next cycle draws independent values at the same positions
    run.st.k = 1
    run.X[:] = x0
    run.phase_converge()
    z1 = (run.F - f_clean) / SIGMA
    _assert_standard_normal(z1)
    assert abs(np.corrcoef(z, z1)[0, 1]) < 5.0 / np.sqrt(len(z))


def test_finite_differences_use_two_independent_draws():
    prob = _noisy_problem()
    h = 1e-2
    run, cfg, x0 = _run(prob, N=4000, grad_mode=0, fd_h=h)
    run.phase_converge()
    g_clean = O.OracleProblem(prob).fd_grad(x0, fd_h=h)
    # (f+ + s z+ - f- - s z-) / ((x+h)-(x-h)): the noise part is N(0, 2 s^2) / (2h)
    den = (x0 + h) - (x0 - h)
    z = ((run.G - g_clean) * den / SIGMA).ravel()
    _assert_standard_normal(z, var=2.0)


def test_gate_value_is_mean_of_R_noisy_evaluations():
    prob = _noisy_problem(W.STUDENT_T)
    for reps in (16, 0):
        run, cfg, x0 = _run(prob, grad_mode=1, gate_reps=reps)
        R = reps if reps > 0 else cfg.M
        run.phase_converge()
        run.phase_stick()
        f_clean = O.OracleProblem(prob).eval(x0, grad=False)
        z = (run.Fg - f_clean) / SIGMA
        _assert_standard_normal(z, var=1.0 / R)
        # the gate value and the line-search value are different draws
        zf = (run.F - f_clean) / SIGMA
        assert abs(np.corrcoef(z, zf)[0, 1]) < 5.0 / np.sqrt(len(z))
        # the stick test compares gate values with f_max, which is estimated
        # afresh at the sample with the largest gate value
        best = int(np.argmax(np.where(run.active == 1, run.Fg, -np.inf)))
        fm = run.stats()["f_max"]
        assert fm != run.Fg.max() and abs(fm - f_clean[best]) < 6 * SIGMA / np.sqrt(R)
        gate = fm + cfg.log_delta
        np.testing.assert_array_equal(run.stuck, (np.abs(run.G).max(1) < cfg.eps_grad) & (run.Fg >= gate))


def test_f_max_is_an_unbiased_fresh_estimate_at_the_best_gate_sample():
    """With many samples near one peak, the largest gate value overestimates
    the peak by the largest of their noise terms.  f_max is f at the sample
    with the largest gate value plus sigma_n times the mean of R new draws:
    over independent runs its residual is N(0, sigma_n^2 / R), unbiased, and
    uncorrelated with that sample's gate noise, while the largest gate value's
    residual is biased upward."""
    prob = _noisy_problem()
    R = 8
    fresh, maxg, own = [], [], []
    for seed in range(400):
        cfg = W.RunConfig(N=256, n_conv=1, M=8, eps_grad=1e-3, seed=1000 + seed, gate_reps=R)
        x0 = W.uniform_population(5, 256, prob.lo, prob.hi)
        run = O.OracleRun(prob, cfg, x0)
        run.cc.n_conv = 0
        run.phase_converge()
        run.phase_stick()
        f_clean = O.OracleProblem(prob).eval(x0, grad=False)
        best = int(np.argmax(run.Fg))
        fresh.append((run.stats()["f_max"] - f_clean[best]) / SIGMA)
        maxg.append((run.Fg[best] - f_clean[best]) / SIGMA)
    fresh, maxg = np.array(fresh), np.array(maxg)
    _assert_standard_normal(fresh, var=1.0 / R)
    assert abs(np.corrcoef(fresh, maxg)[0, 1]) < 5.0 / np.sqrt(len(fresh))
    assert maxg.mean() > 5.0 * np.sqrt(1.0 / R / len(maxg))


def test_noise_free_problem_ignores_gate_reps():
    prob = W.mixture_problem(31, 6, 5, 4.0, lam_range=(0.3, 1.0))
    a, cfg, x0 = _run(prob, N=2000, grad_mode=1)
    a.phase_converge()
    a.phase_stick()
    b, _, _ = _run(prob, N=2000, grad_mode=1, gate_reps=7)
    b.phase_converge()
    b.phase_stick()
    np.testing.assert_array_equal(a.F, b.F)
    np.testing.assert_array_equal(a.stuck, b.stuck)
    assert a.stats()["f_max"] == a.F.max()


def test_noise_aware_line_search_converges_under_unit_noise():
    """Unit noise on a single Gaussian (d=6): with the sufficient-increase test
    relaxed by twice the noise level, Phase 1 with exact gradients still
    drives every sample to |grad|_inf < eps_grad; the plain test on two noisy
    values would reject most steps once the gain falls below the noise."""
    prob = W.mixture_problem(33, 6, 1, 3.0, lam_range=(0.3, 1.0), noise_sigma=1.0)
    N = 400
    cfg = W.RunConfig(N=N, n_conv=40, m=8, eps_grad=1e-6, grad_mode=1, seed=3)
    run = O.OracleRun(prob, cfg, W.uniform_population(8, N, prob.lo, prob.hi))
    run.phase_converge()
    assert run.conv.mean() > 0.99
    np.testing.assert_allclose(run.X, np.broadcast_to(prob.mu[0], run.X.shape), atol=1e-5)
