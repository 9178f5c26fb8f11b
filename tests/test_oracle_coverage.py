"""Statistical check of the mode-coverage statement (Prop. 2, d=2): with N
independent uniform starts, mode k is missed by the first convergence phase
with probability (1 - V_k / vol(Theta))^N, V_k the volume of its basin of
attraction under the method's L-BFGS.  The basin fractions are measured on a
grid of starts; the miss frequencies come from independent random groups of
N starts.  Both go through the oracle's Phase 1."""
import numpy as np

import workloads as W
from oracle import oracle as O
from oracle.modes import newton_modes


def _phase1_modes(prob, X, maxima):
    cfg = W.RunConfig(N=len(X), m=6, n_osc=3, n_conv=80, eps_grad=1e-9, grad_mode=1, seed=1)
    run = O.OracleRun(prob, cfg, X)
    run.phase_converge()
    dist = np.abs(run.X[:, None, :] - maxima[None]).max(2)
    k = np.argmin(dist, 1)
    k[dist.min(1) > 1e-4] = -1  # not converged to a maximum
    return k


def test_miss_probability_follows_the_coverage_formula():
    prob = W.mixture_problem(17, 2, 4, 3.0, lam_range=(0.3, 1.0))
    maxima, _ = newton_modes(prob, log_delta=None)
    K = len(maxima)
    lo, hi = prob.lo.astype(np.float64), prob.hi.astype(np.float64)
    n = 120
    g = (np.arange(n) + 0.5) / n
    G1, G2 = np.meshgrid(lo[0] + g * (hi[0] - lo[0]), lo[1] + g * (hi[1] - lo[1]), indexing="ij")
    kg = _phase1_modes(prob, np.stack([G1.ravel(), G2.ravel()], 1), maxima)
    p = np.array([np.mean(kg == k) for k in range(K)])
    assert np.mean(kg >= 0) > 0.99 and K >= 2
    N, R = 4, 2500
    X = W.uniform_population(5, N * R, prob.lo, prob.hi).astype(np.float64)
    kr = _phase1_modes(prob, X, maxima).reshape(R, N)
    for k in range(K):
        miss = np.mean(~(kr == k).any(1))
        want = (1.0 - p[k]) ** N
        sd = np.sqrt(want * (1 - want) / R) + 1e-3
        print(f"mode {k}: basin fraction {p[k]:.4f}, miss {miss:.4f} vs (1-p)^N {want:.4f}")
        assert abs(miss - want) < 5 * sd + 0.01
