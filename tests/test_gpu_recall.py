"""Mode recall of full GPU runs against the FP64 reference mode set (Newton
refinement from every centre, Hessian test and delta-gate; pinned to the
brute-force grid at d=2).

A recovered mode x passed the stick test, so its gradient sup-norm is below
eps_grad; it then lies within |H^-1|_inf * eps_grad (L-infinity) of the exact
maximum x*, H the Hessian at x*.  A recovered mode matches reference mode k
when their L-infinity distance is below twice that bound (and at least
1e-4, for float32 rounding of x); matching is one-to-one."""
import time

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _tolerances(prob, Xref, eps_grad):
    from oracle.modes import value_grad_hess

    tol = []
    for x in Xref:
        _, _, H = value_grad_hess(prob, x)
        tol.append(max(1e-4, 2.0 * np.abs(np.linalg.inv(H)).sum(1).max() * eps_grad))
    return np.array(tol)


def _score(X, Xref, tol):
    hit = np.zeros(len(Xref), bool)
    spurious = 0
    for x in X:
        dist = np.abs(Xref - x).max(1)
        j = int(np.argmin(dist))
        if dist[j] < tol[j] and not hit[j]:
            hit[j] = True
        else:
            spurious += 1
    return hit.mean() if len(Xref) else 1.0, spurious


def _report(prob, X, F, Xall, Fall):
    """Where each recovered mode sits among all reference local maxima."""
    order = np.argsort(-Fall)
    rank = np.empty(len(Fall), int)
    rank[order] = np.arange(len(Fall))
    lines = [f"  top reference values: {np.round(Fall[order[:5]], 4).tolist()}"]
    for x, f in zip(X, F):
        dist = np.abs(Xall - x).max(1)
        j = int(np.argmin(dist))
        lines.append(f"  recovered f={f:.4f}: nearest reference rank {rank[j]} (f={Fall[j]:.4f}), "
                     f"L-inf distance {dist[j]:.2e}")
    return "\n".join(lines)


@pytest.mark.parametrize("name,make", [
    ("config2 (d=16, K=32, N=16384, 200 cycles, finite differences)", W.config2),
    ("config3 (d=64, K=128, N=65536, 300 cycles, adjoint)", W.config3),
])
def test_full_run_mode_recall(name, make):
    from oracle.modes import newton_modes
    from paper_2606_26164_amd.api import Optimizer

    prob, cfg, x0 = make()
    Xall, Fall = newton_modes(prob, log_delta=None)
    keep = Fall >= Fall.max() + cfg.log_delta
    Xref = Xall[keep]
    tol = _tolerances(prob, Xref, cfg.eps_grad)
    t = time.perf_counter()
    with Optimizer(prob, cfg, x0) as opt:
        stats = opt.cycle(cfg.n_osc, stats=True)
        ms = opt.modes()
    dt = time.perf_counter() - t
    recall, spurious = _score(ms.X.astype(np.float64), Xref, tol)
    first_full = next((s["k"] for s in stats if s["n_modes"] >= len(Xref)), None)
    print(f"\n{name}: {len(Xref)} reference modes, {len(ms.X)} recovered, recall {recall:.3f}, spurious {spurious}, "
          f"{dt:.1f} s, first cycle with all modes stuck: {first_full}, match tolerance {tol.max():.2e}")
    print(_report(prob, ms.X.astype(np.float64), ms.F, Xall, Fall))
    assert spurious == 0
    assert recall == 1.0
