"""Pins of the oracle's width export (the survivor's inverse-Hessian
estimate, Phase 3): the diagonal it reports is checked against a dense
inverse-BFGS recursion written here with numpy (a different algorithm from
the two-loop the oracle uses), against the exact answer on an isotropic
quadratic, and against the rules for samples without pairs and for
reseeded samples."""
import numpy as np

import workloads as W
from oracle import oracle as O


def _dense_bfgs_diag(S, Y, rho, cnt, head, m):
    """H = gamma I updated by each pair from oldest to newest:
    H <- (I - rho s y^T) H (I - rho y s^T) + rho s s^T."""
    d = S.shape[1]
    newest = head
    gamma = S[newest] @ Y[newest] / (Y[newest] @ Y[newest])
    H = gamma * np.eye(d)
    for k in range(cnt - 1, -1, -1):
        sl = (head - k + m) % m
        s, y, r = S[sl], Y[sl], rho[sl]
        V = np.eye(d) - r * np.outer(y, s)
        H = V.T @ H @ V + r * np.outer(s, s)
    return np.diag(H)


def _state_with_pairs(d=6, N=5, m=4, seed=0):
    prob = W.mixture_problem(5, d, 1, 3.0, isotropic_var=1.0)
    cfg = W.RunConfig(N=N, m=m, eps_dup=1e-3, seed=seed)
    rng = np.random.default_rng(seed)
    run = O.OracleRun(prob, cfg, rng.uniform(-3, 3, size=(N, d)))
    A = rng.normal(size=(d, d))
    A = A @ A.T + d * np.eye(d)  # SPD curvature: y = A s gives s'y > 0
    for i in range(N):
        cnt = int(rng.integers(1, m + 1))
        head = int(rng.integers(0, m))
        for k in range(cnt):
            sl = (head - k + m) % m
            s = rng.normal(size=d)
            y = A @ s + 0.1 * rng.normal(size=d)
            run.S[i, sl], run.Y[i, sl], run.rho[i, sl] = s, y, 1.0 / (s @ y)
        run.cnt[i], run.head[i] = cnt, head
    run.stuck[:] = 1
    run.active[:] = 1
    run.G[:] = rng.normal(size=(N, d))
    return run, m


def test_width_is_diagonal_of_the_dense_bfgs_recursion():
    run, m = _state_with_pairs()
    run.phase_dedup()
    for i in range(run.cfg.N):
        want = _dense_bfgs_diag(run.S[i], run.Y[i], run.rho[i], int(run.cnt[i]), int(run.head[i]), m)
        np.testing.assert_allclose(run.W[i], want, rtol=1e-12, atol=1e-14)
        assert run.wvalid[i] == 1


def test_isotropic_quadratic_gives_the_exact_variance():
    run, m = _state_with_pairs()
    sig2 = 0.37
    for i in range(run.cfg.N):
        for k in range(int(run.cnt[i])):
            sl = (int(run.head[i]) - k + m) % m
            run.Y[i, sl] = run.S[i, sl] / sig2
            run.rho[i, sl] = 1.0 / (run.S[i, sl] @ run.Y[i, sl])
    run.phase_dedup()
    np.testing.assert_allclose(run.W, sig2, rtol=1e-12)


def test_samples_without_pairs_keep_or_initialise_their_width():
    run, m = _state_with_pairs()
    run.phase_dedup()
    kept = run.W.copy()
    # released and stuck again without a step: the diagonal is kept
    run.cnt[:] = 0
    run.phase_dedup()
    np.testing.assert_array_equal(run.W, kept)
    # never had one: 1 / max(|g|_2, 1)
    run.wvalid[:] = 0
    run.phase_dedup()
    want = 1.0 / np.maximum(np.linalg.norm(run.G, axis=1), 1.0)
    np.testing.assert_allclose(run.W, np.repeat(want[:, None], run.P.d, 1), rtol=1e-15)
