"""Pins of the FP64 oracle against facts outside itself.

Each test checks one oracle function against a library routine, a closed form,
a published known-answer vector, or a brute-force definition on tiny inputs,
chosen so that a dropped term, a wrong sign or a transposed operand fails.
"""
import os

import numpy as np
import pytest
import scipy.optimize
import scipy.special
import scipy.stats
import torch

import workloads as W
from oracle import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# Random streams
# --------------------------------------------------------------------------

def test_philox_known_answers():
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) if ln.strip()
            and not ln.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        vals = [int(v, 16) for v in r if v != "->"]
        ctr, key, want = vals[:4], vals[4:6], vals[6:10]
        assert O.philox4x32_10(ctr, key) == want


def test_uniform_is_exact_and_open():
    L = O.lib()
    assert L.orc_u01(0) == 0.5 / 2 ** 24
    assert L.orc_u01(0xFFFFFFFF) == (2 ** 24 - 0.5) / 2 ** 24
    # the low 8 bits are dropped, values are exact multiples of 2^-25
    assert L.orc_u01(0x12345678) == ((0x12345678 >> 8) + 0.5) / 2 ** 24


def test_normals_moments_and_uniform_population():
    """The INIT stream fills the box uniformly: mean and variance of a uniform."""
    p = W.mixture_problem(0, 4, 1, 3.0, isotropic_var=1.0, dirichlet=None)
    cfg = W.RunConfig(N=20000, seed=11)
    run = O.OracleRun(p, cfg)
    X = run.X
    lo, hi = p.lo.astype(float), p.hi.astype(float)
    assert np.all(X >= lo) and np.all(X <= hi)
    np.testing.assert_allclose(X.mean(0), 0.5 * (lo + hi), atol=4 * (hi - lo).max() / np.sqrt(12 * 20000))
    np.testing.assert_allclose(X.var(0), (hi - lo) ** 2 / 12, rtol=0.05)


# --------------------------------------------------------------------------
# Objective and gradients
# --------------------------------------------------------------------------

def _scipy_logpdf(prob, X):
    K = prob.K
    cols = []
    for k in range(K):
        P = prob.prec[k].astype(np.float64)
        cov = np.linalg.inv(P)
        cov = 0.5 * (cov + cov.T)
        if prob.family == W.GAUSS:
            lp = scipy.stats.multivariate_normal.logpdf(X, mean=prob.mu[k].astype(np.float64), cov=cov)
        else:
            lp = scipy.stats.multivariate_t.logpdf(X, loc=prob.mu[k].astype(np.float64), shape=cov, df=prob.nu)
        cols.append(np.atleast_1d(lp) + float(prob.log_w[k]))
    return scipy.special.logsumexp(np.stack(cols, 1), axis=1)


@pytest.mark.parametrize("family", [W.GAUSS, W.STUDENT_T])
def test_value_matches_scipy(family):
    prob = W.mixture_problem(5, 6, 5, 3.0, lam_range=(0.2, 1.0), family=family, nu=3.0)
    X = np.random.default_rng(0).uniform(-4, 4, size=(50, 6))
    f = O.OracleProblem(prob).eval(X, grad=False)
    np.testing.assert_allclose(f, _scipy_logpdf(prob, X), rtol=1e-12, atol=1e-12)


def test_single_gaussian_reduces_to_quadratic():
    """K=1: f is the concave quadratic log N(x; mu, P^-1) with gradient -P(x-mu)."""
    prob = W.mixture_problem(6, 5, 1, 2.0, lam_range=(0.3, 2.0), dirichlet=None)
    P = prob.prec[0].astype(np.float64)
    mu = prob.mu[0].astype(np.float64)
    X = np.random.default_rng(1).normal(size=(7, 5))
    f, G = O.OracleProblem(prob).eval(X)
    _, logdet = np.linalg.slogdet(P)
    want = -0.5 * 5 * np.log(2 * np.pi) + 0.5 * logdet - 0.5 * np.einsum("ni,ij,nj->n", X - mu, P, X - mu)
    np.testing.assert_allclose(f, want, rtol=1e-13)
    np.testing.assert_allclose(G, -(X - mu) @ P, rtol=1e-12, atol=1e-13)
    # stationary at the centre
    _, g0 = O.OracleProblem(prob).eval(mu[None, :])
    assert np.abs(g0).max() < 1e-14


@pytest.mark.parametrize("family", [W.GAUSS, W.STUDENT_T])
def test_gradient_matches_autograd_and_fd(family):
    prob = W.mixture_problem(7, 8, 6, 3.0, lam_range=(0.1, 1.0), family=family, nu=3.0)
    op = O.OracleProblem(prob)
    X = np.random.default_rng(2).uniform(-3, 3, size=(20, 8))
    f, G = op.eval(X)
    # torch autograd of the mixture density written with scipy-checked pieces
    x = torch.tensor(X, requires_grad=True)
    mu = torch.tensor(prob.mu, dtype=torch.float64)
    Pm = torch.tensor(prob.prec, dtype=torch.float64)
    delta = x[:, None, :] - mu[None]
    q = torch.einsum("nki,kij,nkj->nk", delta, Pm, delta)
    logdet = torch.logdet(Pm)
    d = 8
    if family == W.GAUSS:
        comp = -0.5 * d * np.log(2 * np.pi) + 0.5 * logdet - 0.5 * q
    else:
        nu = prob.nu
        comp = (torch.lgamma(torch.tensor((nu + d) / 2, dtype=torch.float64))
                - torch.lgamma(torch.tensor(nu / 2, dtype=torch.float64))
                - 0.5 * d * np.log(nu * np.pi) + 0.5 * logdet - 0.5 * (nu + d) * torch.log1p(q / nu))
    ft = torch.logsumexp(comp + torch.tensor(prob.log_w, dtype=torch.float64), 1)
    np.testing.assert_allclose(ft.detach().numpy(), _scipy_logpdf(prob, X), rtol=1e-12)
    ft.sum().backward()
    np.testing.assert_allclose(G, x.grad.numpy(), rtol=1e-10, atol=1e-12)
    # central differences of the oracle's own value, h = 1e-6
    Gfd = op.fd_grad(X, fd_h=1e-6)
    np.testing.assert_allclose(Gfd, G, rtol=1e-6, atol=1e-7)


def test_fd_gradient_exact_on_quadratic_and_relative_rule():
    """Central differences are exact for a quadratic, for any step."""
    prob = W.mixture_problem(8, 6, 1, 5.0, lam_range=(0.5, 1.0), dirichlet=None)
    op = O.OracleProblem(prob)
    X = np.random.default_rng(3).uniform(-6, 6, size=(10, 6))
    _, G = op.eval(X)
    for h in (1e-5, 0.0):  # fixed step, then the 2^-8 max(1,|x|) rule
        np.testing.assert_allclose(op.fd_grad(X, fd_h=h), G, rtol=1e-7, atol=1e-7)


def test_prepare_rejects_indefinite_precision():
    prob = W.mixture_problem(9, 3, 2, 1.0, isotropic_var=1.0)
    prob.prec = prob.prec.copy()
    prob.prec[1, 2, 2] = -1.0
    with pytest.raises(ValueError):
        O.OracleProblem(prob)


# --------------------------------------------------------------------------
# L-BFGS
# --------------------------------------------------------------------------

def test_two_loop_equals_dense_bfgs_update():
    """The two-loop product equals the explicit inverse-BFGS recursion
    H <- (I - rho s y^T) H (I - rho y s^T) + rho s s^T from H0 = gamma I."""
    rng = np.random.default_rng(4)
    d, m = 6, 4
    A = rng.normal(size=(d, d))
    A = A @ A.T + d * np.eye(d)  # SPD Hessian of F = -f
    for cnt in range(0, m + 1):
        S = np.zeros((m, d)); Y = np.zeros((m, d)); rho = np.zeros(m)
        head = m - 1
        pairs = []
        for _ in range(cnt + 2):  # overfill to exercise the ring wrap
            s = rng.normal(size=d); y = A @ s
            head = (head + 1) % m
            S[head], Y[head], rho[head] = s, y, 1 / (s @ y)
            pairs.append((s, y))
        n = min(cnt, m) if cnt < m else m
        g = rng.normal(size=d)
        if n == 0:
            p = O.two_loop(g, S, Y, rho, 0, head)
            np.testing.assert_allclose(p, g / max(np.linalg.norm(g), 1.0), rtol=1e-14)
            continue
        used = pairs[-n:]
        s_new, y_new = used[-1]
        H = (s_new @ y_new) / (y_new @ y_new) * np.eye(d)
        for s, y in used:
            r = 1 / (s @ y)
            V = np.eye(d) - r * np.outer(y, s)
            H = V.T @ H @ V + r * np.outer(s, s)
        p = O.two_loop(g, S, Y, rho, n, head)
        np.testing.assert_allclose(p, H @ g, rtol=1e-11, atol=1e-12)


def _quad_problem(d=5, seed=10):
    return W.mixture_problem(seed, d, 1, 2.0, lam_range=(0.2, 1.0), dirichlet=None)


def test_lbfgs_converges_on_quadratic_like_scipy():
    """Prop. 1 setting: one concave quadratic.  Every sample reaches the
    centre, matching scipy's L-BFGS-B endpoint."""
    prob = _quad_problem()
    # 1e-7: below ~1e-8 the Armijo test can no longer resolve the FP64 value gain
    cfg = W.RunConfig(N=16, m=10, n_osc=1, n_conv=40, eps_grad=1e-7, grad_mode=1, seed=3)
    x0 = W.uniform_population(3, 16, prob.lo, prob.hi)
    run = O.OracleRun(prob, cfg, x0)
    run.phase_converge()
    mu = prob.mu[0].astype(np.float64)
    assert run.conv.all()
    np.testing.assert_allclose(run.X, np.broadcast_to(mu, run.X.shape), atol=1e-7)
    op = O.OracleProblem(prob)
    res = scipy.optimize.minimize(lambda x: -op.eval(x[None], grad=False)[0], x0[0].astype(np.float64),
                                  jac=lambda x: -op.eval(x[None])[1][0], method="L-BFGS-B",
                                  options=dict(gtol=1e-12, ftol=1e-15))
    np.testing.assert_allclose(run.X[0], res.x, atol=1e-6)


def test_one_cycle_unimodal_collapses_to_one_mode():
    """Prop. 1 and its remark: after one cycle every sample is stuck at the
    single peak and deduplication leaves exactly one mode."""
    prob = _quad_problem(d=4, seed=12)
    cfg = W.RunConfig(N=64, m=8, n_osc=1, n_conv=30, eps_grad=1e-6, grad_mode=1, seed=4)
    run = O.OracleRun(prob, cfg, W.uniform_population(4, 64, prob.lo, prob.hi))
    run.cycle()
    X, F, idx = run.modes()
    assert len(idx) == 1
    np.testing.assert_allclose(X[0], prob.mu[0], atol=1e-6)
    assert run.stats()["K_lost"] == 63


def test_line_search_respects_box_and_armijo():
    """Peak outside the box: iterates stay in the box, values never decrease
    (Armijo with c1 > 0), and the iterates end on the nearest face."""
    prob = W.mixture_problem(13, 3, 1, 1.0, isotropic_var=1.0, dirichlet=None)
    prob.mu = np.array([[5.0, 0.0, 0.0]], np.float32)  # outside [-1.2,1.2]^3
    lo, hi = prob.lo.astype(float), prob.hi.astype(float)
    cfg = W.RunConfig(N=4, m=5, n_osc=1, n_conv=1, eps_grad=1e-12, grad_mode=1)
    x0 = np.array([[-1.2, 0.3, 0.1], [0.0, 0.0, 0.0], [1.2, 1.2, -1.2], [0.5, -0.5, 0.2]], np.float32)
    run = O.OracleRun(prob, cfg, x0)
    fprev = None
    for _ in range(6):  # one iteration per call (each call releases the history)
        run.phase_converge()
        assert np.all(run.X <= hi) and np.all(run.X >= lo)
        if fprev is not None:
            assert np.all(run.F >= fprev)
        fprev = run.F.copy()
    run.cc.n_conv = 40
    run.phase_converge()
    np.testing.assert_allclose(run.X[:, 0], hi[0], atol=0)
    np.testing.assert_allclose(run.X[:, 1:], 0.0, atol=1e-6)


# --------------------------------------------------------------------------
# Stick and deduplication on hand-made sets
# --------------------------------------------------------------------------

def _manual_run(X, F, G, eps_grad=1e-3, eps_dup=1e-3, log_delta=np.log(0.1)):
    X = np.asarray(X, float)
    N, d = X.shape
    prob = W.mixture_problem(14, d, 1, 1.0, isotropic_var=1.0)
    cfg = W.RunConfig(N=N, m=2, eps_grad=eps_grad, eps_dup=eps_dup, log_delta=log_delta)
    run = O.OracleRun(prob, cfg, X)
    run.F[:] = F
    run.G[:] = G
    return run


def test_stick_gate():
    X = np.zeros((5, 2))
    F = np.array([0.0, -1.0, -2.5, -0.5, 0.0])
    G = np.zeros((5, 2))
    G[4, 1] = 2e-3  # fails the gradient test
    G[3, 0] = -9e-4  # passes (sup-norm below 1e-3)
    run = _manual_run(X, F, G)
    run.phase_stick()
    # gate = 0 + log 0.1 = -2.3026
    assert run.stuck.tolist() == [1, 1, 0, 1, 0]
    assert run.st.f_max == 0.0


def test_stick_deactivates_non_finite_samples():
    """Reading: a sample whose value or gradient is not finite leaves the
    population at Phase 2, before f_max; the rest of the phase is the
    brute-force definition over the remaining samples."""
    X = np.zeros((6, 2))
    F = np.array([0.0, np.nan, -0.5, np.inf, -1.0, -3.0])
    G = np.zeros((6, 2))
    G[2, 1] = np.inf
    G[4, 0] = -np.nan
    run = _manual_run(X, F, G)
    run.phase_stick()
    assert run.active.tolist() == [1, 0, 0, 0, 0, 1]
    assert run.st.n_nonfinite == 4
    assert run.st.f_max == 0.0  # +inf no longer dominates
    assert run.stuck.tolist() == [1, 0, 0, 0, 0, 0]  # -3 is below the gate 0 + log 0.1


def test_non_finite_sample_equals_an_empty_slot():
    """A whole cycle with one NaN row ends, for every other sample, exactly as
    a cycle in which that slot was inactive from the start: the guard keeps
    it out of every reduction (f_max, the smoothing scale, the step lengths,
    the reseeding lists)."""
    prob = W.mixture_problem(3, 4, 6, 3.0, lam_range=(0.3, 1.0))
    cfg = W.RunConfig(N=64, m=4, n_conv=8, M=4, eps_grad=1e-6, seed=5)
    x0 = W.uniform_population(4, 64, prob.lo, prob.hi).astype(np.float64)
    bad = 17
    a = O.OracleRun(prob, cfg, x0)
    a.X[bad] = np.nan
    b = O.OracleRun(prob, cfg, x0)
    b.active[bad] = 0
    for _ in range(2):
        a.cycle()
        b.cycle()
    keep = np.arange(64) != bad
    assert a.active[bad] == 0
    np.testing.assert_array_equal(a.X[keep], b.X[keep])
    np.testing.assert_array_equal(a.stuck, b.stuck)
    np.testing.assert_array_equal(a.active, b.active)
    assert np.isfinite(a.st.sigma) and a.st.sigma == b.st.sigma
    assert a.st.alpha_a == b.st.alpha_a


def test_dedup_ties_chains_and_clusters():
    eps = 1e-3
    X = np.array([
        [0.0, 0.0],        # 0: f=1   cluster A
        [0.0005, 0.0],     # 1: f=1   tie with 0 -> lower index (0) survives
        [0.0009, 0.0009],  # 2: f=2   within eps of 0 and 1 -> survives, removes 0 and 1
        [5.0, 5.0],        # 3: chain a
        [5.0009, 5.0],     # 4: chain b (near a and c)
        [5.0018, 5.0],     # 5: chain c (near b only)
        [9.0, 9.0],        # 6: isolated
        [9.0, 9.0011],     # 7: just outside eps of 6
    ])
    F = np.array([1.0, 1.0, 2.0, 3.0, 2.0, 1.0, 0.0, 0.0])
    run = _manual_run(X, F, np.zeros_like(X))
    run.stuck[:] = 1
    run.phase_dedup()
    # 0 removed by 2; 1 removed by 0 (tie, lower index) and 2; 4 removed by 3;
    # 5 removed by 4 even though 4 itself is removed (all stuck samples compare)
    assert run.removed.tolist() == [1, 1, 0, 0, 1, 1, 0, 0]
    assert run.stuck.tolist() == [0, 0, 1, 1, 0, 0, 1, 1]
    assert run.st.K_lost == 4 and run.st.n_modes == 4


def test_dedup_brute_force_random():
    rng = np.random.default_rng(5)
    centers = rng.uniform(-1, 1, size=(6, 3))
    X = centers[rng.integers(0, 6, 60)] + rng.uniform(-3e-4, 3e-4, size=(60, 3))
    F = rng.normal(size=60)
    F[10] = F[11]  # an exact tie
    stuck = (rng.uniform(size=60) < 0.8).astype(np.uint8)
    run = _manual_run(X, F, np.zeros_like(X))
    run.stuck[:] = stuck
    run.phase_dedup()
    want = np.zeros(60, np.uint8)
    for j in range(60):
        if not stuck[j]:
            continue
        for i in range(60):
            if i != j and stuck[i] and np.abs(X[i] - X[j]).max() < 1e-3 and (F[i] > F[j] or (F[i] == F[j] and i < j)):
                want[j] = 1
    np.testing.assert_array_equal(run.removed, want)
    # one survivor per cluster of stuck samples
    lab = np.argmin(np.abs(X[:, None, :] - centers[None]).max(2), 1)
    for c in range(6):
        members = np.nonzero((lab == c) & (stuck == 1))[0]
        if len(members):
            assert run.stuck[members].sum() == 1


def test_disabled_dedup_removes_nothing():
    X = np.zeros((4, 2))
    run = _manual_run(X, np.zeros(4), np.zeros_like(X))
    run.stuck[:] = 1
    run.cc.phase_mask = 0x7E & ~(1 << 3)
    run.phase_dedup()
    assert run.removed.sum() == 0 and run.st.K_lost == 0


# --------------------------------------------------------------------------
# Reseeding
# --------------------------------------------------------------------------

def test_householder_q_matches_numpy_qr_sign_fixed():
    A = np.random.default_rng(6).normal(size=(9, 9))
    Q, R = O.householder_q(A)
    q, r = np.linalg.qr(A)
    s = np.sign(np.diag(r))
    np.testing.assert_allclose(Q, q * s[None, :], atol=1e-12)
    np.testing.assert_allclose(R, r * s[:, None], atol=1e-12)
    np.testing.assert_allclose(Q.T @ Q, np.eye(9), atol=1e-13)
    assert np.all(np.diag(R) > 0)
    np.testing.assert_allclose(Q @ R, A, atol=1e-12)


def _on_ray(x, o, u_unit):
    v = x - o
    t = v @ u_unit
    return t >= -1e-12 and np.linalg.norm(v - t * u_unit) <= 1e-9 * max(1.0, np.linalg.norm(v))


def test_repulse_monkey_invariants():
    rng = np.random.default_rng(7)
    N, d = 40, 3
    X = rng.uniform(-1, 1, size=(N, d))
    run = _manual_run(X, np.zeros(N), np.zeros((N, d)))
    run.stuck[:] = 0
    run.stuck[:4] = 1            # survivors (peaks)
    run.removed[4:10] = 1        # six duplicates to reseed
    run.st.K_lost = 6
    run.st.n_modes = 4
    before = run.X.copy()
    free = [i for i in range(N) if not run.removed[i] and not run.stuck[i]]
    run.phase_reseed()
    assert run.st.reseed_kind == 1 and run.st.n_free == len(free)
    lo, hi = run.P.lo, run.P.hi
    for s in range(4, 10):
        x = run.X[s]
        assert np.all(x >= lo) and np.all(x <= hi)
        # lies on a ray from some free sample's (unchanged) position
        ok = False
        for o in before[free]:
            v = x - o
            if np.linalg.norm(v) == 0:
                ok = True
                break
            if _on_ray(x, o, v / np.linalg.norm(v)):
                ok = True
                break
        assert ok
        assert run.stuck[s] == 0 and run.removed[s] == 0 and run.active[s] == 1
    np.testing.assert_array_equal(run.X[10:], before[10:])


def test_golden_rooster_directions_and_disable():
    d, N = 4, 12
    X = np.zeros((N, d))
    X[0] = [0.3, -0.2, 0.1, 0.0]
    X[1] = [-0.5, 0.4, 0.0, 0.2]
    run = _manual_run(X, np.zeros(N), np.zeros((N, d)))
    run.stuck[:] = 0
    run.stuck[0] = run.stuck[1] = 1
    run.removed[2:12] = 1  # ten slots, no free samples -> Golden Rooster
    run.st.K_lost = 10
    run.st.n_modes = 2
    peaks = X[:2].copy()
    run.phase_reseed()
    assert run.st.reseed_kind == 2
    # slot j uses peak j mod 2, direction (-1)^q Q[:, q//2] with q = j // 2
    dirs = {0: [], 1: []}
    for j, s in enumerate(range(2, 12)):
        o = peaks[j % 2]
        v = run.X[s] - o
        n = np.linalg.norm(v)
        if n > 0:
            dirs[j % 2].append((j // 2, v / n))
    for p in (0, 1):
        for q, u in dirs[p]:
            for q2, u2 in dirs[p]:
                if q2 // 2 != q // 2:
                    assert abs(u @ u2) < 1e-10  # orthogonal columns
                elif q2 != q:
                    np.testing.assert_allclose(u, -u2, atol=1e-10)  # opposite signs of one column
    # bookkeeping: two generations without a new peak disable GR
    assert run.st.gr_used_last == 1
    for _ in range(2):
        run.stuck[:] = 0
        run.stuck[0] = run.stuck[1] = 1
        run.phase_dedup()
        run.st.gr_used_last = 1
        run.st.gr_prev_modes = 2
    assert run.st.gr_disabled == 1
    run.stuck[:] = 0
    run.stuck[0] = run.stuck[1] = 1
    run.removed[2:12] = 1
    run.st.K_lost = 10
    run.phase_reseed()
    assert run.st.reseed_kind == 3 and run.active[2:12].sum() == 0 and run.active[:2].all()


# --------------------------------------------------------------------------
# Hands Like Clouds and anti-convergence on a quadratic
# --------------------------------------------------------------------------

def test_hlc_antithetic_exact_on_quadratic():
    """For a quadratic the gradient is affine, so each antithetic pair
    averages to the exact gradient at x."""
    prob = W.mixture_problem(15, 5, 1, 1.0, lam_range=(0.5, 1.0), dirichlet=None, box_scale=50.0)
    cfg = W.RunConfig(N=8, M=6, n_cloud=1, sigma=0.3, alpha=0.01, grad_mode=1)
    x0 = np.random.default_rng(8).uniform(-3, 3, size=(8, 5)).astype(np.float32)
    run = O.OracleRun(prob, cfg, x0)
    run.stuck[:] = 0
    run.phase_hlc()
    P, mu = prob.prec[0].astype(float), prob.mu[0].astype(float)
    x = x0.astype(float)
    np.testing.assert_allclose(run.X, x + 0.01 * (-(x - mu) @ P), rtol=1e-12, atol=1e-12)


def test_hlc_estimator_unbiased():
    """Appendix B: the Monte Carlo mean of grad f(x + sigma z) estimates
    grad f_sigma; for a Gaussian component f_sigma has a closed form."""
    # single isotropic Gaussian with variance v: f_sigma gradient = -(x-mu)/v ... only for
    # the log-density the smoothing is of log N, a quadratic, whose smoothed gradient is
    # the gradient itself; use a two-component mixture and compare with quadrature instead.
    prob = W.mixture_problem(16, 1, 2, 1.0, isotropic_var=0.3, dirichlet=None, box_scale=50.0)
    op = O.OracleProblem(prob)
    x, sigma = 0.2, 0.4
    # Gauss-Hermite quadrature of E[f'(x + sigma z)]
    t, w = np.polynomial.hermite_e.hermegauss(80)
    _, g = op.eval((x + sigma * t)[:, None])
    want = (w * g[:, 0]).sum() / np.sqrt(2 * np.pi)
    M, n_rep = 10, 2000
    cfg = W.RunConfig(N=n_rep, M=M, n_cloud=1, sigma=sigma, alpha=1.0, grad_mode=1, seed=21)
    run = O.OracleRun(prob, cfg, np.full((n_rep, 1), x, np.float32))
    run.stuck[:] = 0
    run.phase_hlc()
    est = run.X[:, 0] - x  # alpha = 1: displacement equals the estimate
    se = est.std() / np.sqrt(n_rep)
    assert abs(est.mean() - want) < 4 * se


def test_anti_convergence_closed_form():
    """On a quadratic the momentum recursion is linear:
    [e; v] <- [[I + a P, mu I], [a P, mu I]] [e; v] with e = x - centre."""
    prob = W.mixture_problem(17, 3, 1, 1.0, lam_range=(0.5, 1.0), dirichlet=None, box_scale=1e4)
    P, mu = prob.prec[0].astype(float), prob.mu[0].astype(float)
    a, mom, T = 0.05, 0.9, 5
    cfg = W.RunConfig(N=3, n_anti=T, alpha=a, momentum=mom, grad_mode=1)
    x0 = np.random.default_rng(9).uniform(-1, 1, size=(3, 3)).astype(np.float32)
    run = O.OracleRun(prob, cfg, x0)
    run.stuck[:] = 0
    run.st.sigma = 0.1
    run.phase_anti()
    A = np.block([[np.eye(3) + a * P, mom * np.eye(3)], [a * P, mom * np.eye(3)]])
    for i in range(3):
        z = np.concatenate([x0[i].astype(float) - mu, np.zeros(3)])
        zT = np.linalg.matrix_power(A, T) @ z
        np.testing.assert_allclose(run.X[i], zT[:3] + mu, rtol=1e-12, atol=1e-12)


def test_auto_step_sizes_follow_scale_estimate():
    """alpha_a = sigma / mean |grad f| over unfrozen samples, so the mean first
    displacement equals sigma; sigma = 0.1 * pooled std when not given."""
    prob = W.mixture_problem(18, 3, 1, 1.0, lam_range=(0.5, 1.0), dirichlet=None, box_scale=1e4)
    cfg = W.RunConfig(N=50, n_anti=1, n_cloud=1, M=2, grad_mode=1, seed=2)
    x0 = np.random.default_rng(10).uniform(-2, 2, size=(50, 3)).astype(np.float32)
    run = O.OracleRun(prob, cfg, x0)
    run.stuck[:] = 0
    run.stuck[:5] = 1
    run.phase_hlc()
    xs = x0[5:].astype(float)
    assert np.isclose(run.st.sigma, 0.1 * np.sqrt(xs.var(0).mean()), rtol=1e-12)
    before = run.X.copy()
    run.phase_anti()
    disp = np.linalg.norm(run.X[5:] - before[5:], axis=1)
    assert np.isclose(disp.mean(), run.st.sigma, rtol=1e-12)
    np.testing.assert_array_equal(run.X[:5], before[:5])  # stuck samples do not move


# --------------------------------------------------------------------------
# Whole runs
# --------------------------------------------------------------------------

def _grid_modes(prob, spacing=4e-3):
    """Brute force at d=2: local maxima of f on a grid over the box, polished
    by Newton steps on the analytic gradient and Hessian of the mixture."""
    op = O.OracleProblem(prob)
    g1 = np.arange(prob.lo[0], prob.hi[0] + spacing / 2, spacing)
    g2 = np.arange(prob.lo[1], prob.hi[1] + spacing / 2, spacing)
    XX, YY = np.meshgrid(g1, g2, indexing="ij")
    f = op.eval(np.stack([XX.ravel(), YY.ravel()], 1), grad=False).reshape(XX.shape)
    c = f[1:-1, 1:-1]
    is_max = np.ones_like(c, bool)
    for di in (-1, 0, 1):
        for dj in (-1, 0, 1):
            if di or dj:
                is_max &= c > f[1 + di:f.shape[0] - 1 + di, 1 + dj:f.shape[1] - 1 + dj]
    ii, jj = np.nonzero(is_max)
    pts = np.stack([g1[ii + 1], g2[jj + 1]], 1)
    out = []
    P = prob.prec.astype(float)
    mu = prob.mu.astype(float)
    for x in pts:
        for _ in range(50):
            lk = np.array([float(prob.log_w[k]) - 0.5 * (x - mu[k]) @ P[k] @ (x - mu[k]) for k in range(prob.K)])
            r = np.exp(lk - scipy.special.logsumexp(lk))
            gk = np.array([-(P[k] @ (x - mu[k])) for k in range(prob.K)])
            g = r @ gk
            H = sum(r[k] * (np.outer(gk[k], gk[k]) - P[k]) for k in range(prob.K)) - np.outer(g, g)
            x = x - np.linalg.solve(H, g)
        out.append(x)
    return np.array(out), op.eval(np.array(out), grad=False)


def test_gauss4_d2_modes_match_brute_force_grid():
    prob, cfg, x0 = W.gauss4_d2()
    run = O.OracleRun(prob, cfg, x0)
    run.run()
    X, F, _ = run.modes()
    gm, gf = _grid_modes(prob)
    sig = gf >= gf.max() + np.log(0.1)
    gm = gm[sig]
    assert len(X) == len(gm)
    for x in X:
        assert np.abs(gm - x).max(1).min() < 1e-3
    for x in gm:
        assert np.abs(X - x).max(1).min() < 1e-3


def test_newton_reference_modes_match_grid_at_d2():
    """The Newton reference used to score recall agrees with the brute-force
    grid on gauss4_d2, and with the oracle's own full run."""
    from oracle.modes import newton_modes

    prob, cfg, x0 = W.gauss4_d2()
    Xn, Fn = newton_modes(prob)
    gm, gf = _grid_modes(prob)
    gm = gm[gf >= gf.max() + np.log(0.1)]
    assert len(Xn) == len(gm)
    for x in Xn:
        assert np.abs(gm - x).max(1).min() < 1e-6


def test_newton_reference_student_t_hessian():
    """Student-t Hessian of the reference against central differences of the
    analytic gradient."""
    from oracle.modes import value_grad_hess

    prob = W.mixture_problem(19, 5, 3, 2.0, lam_range=(0.3, 1.0), family=W.STUDENT_T, nu=3.0)
    x = np.random.default_rng(3).normal(size=5)
    f, g, H = value_grad_hess(prob, x)
    op = O.OracleProblem(prob)
    f2, g2 = op.eval(x[None])
    assert np.isclose(f, f2[0], rtol=1e-12)
    np.testing.assert_allclose(g, g2[0], rtol=1e-10, atol=1e-12)
    h = 1e-5
    Hfd = np.array([(op.eval((x + h * e)[None])[1][0] - op.eval((x - h * e)[None])[1][0]) / (2 * h)
                    for e in np.eye(5)])
    np.testing.assert_allclose(H, Hfd.T, rtol=1e-5, atol=1e-6)
