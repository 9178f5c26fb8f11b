"""End-to-end GPU runs through the C ABI: recovered mode sets against the
FP64 oracle, error handling of the boundary, and reproducibility."""
import numpy as np
import pytest

import workloads as W
from oracle import oracle as O

pytestmark = pytest.mark.gpu


def _match(A, B, tol=1e-3):
    """One-to-one L-infinity matching within tol (clusters are far apart)."""
    if len(A) != len(B):
        return False
    used = set()
    for a in A:
        dist = np.abs(B - a).max(1) if len(B) else np.array([])
        j = int(np.argmin(dist)) if len(dist) else -1
        if j < 0 or dist[j] >= tol or j in used:
            return False
        used.add(j)
    return True


def test_gauss4_d2_mode_set_matches_oracle():
    from paper_2606_26164_amd.api import Optimizer

    prob, cfg, x0 = W.gauss4_d2()
    run = O.OracleRun(prob, cfg, x0)  # the configuration's own FP64 finite-difference run
    run.run()
    Xo, Fo, _ = run.modes()
    # FP32 on the GPU: adjoint and central differences, threshold at the FP32 floor
    for mode in (1, 0):
        gcfg = cfg.with_(grad_mode=mode, eps_grad=1e-4, fd_h=0.0)
        with Optimizer(prob, gcfg, x0) as opt:
            stats = opt.cycle(cfg.n_osc, stats=True)
            ms = opt.modes()
        assert stats[-1]["k"] == cfg.n_osc
        assert _match(ms.X.astype(np.float64), Xo), (mode, ms.X, Xo)
        np.testing.assert_allclose(ms.F, Fo, rtol=1e-5, atol=1e-5)


def test_cycle_past_schedule_is_rejected_and_state_kept():
    from paper_2606_26164_amd import _lib as L
    from paper_2606_26164_amd.api import Optimizer

    prob, cfg, x0 = W.gauss4_d2(N=32)
    cfg = cfg.with_(n_osc=2, grad_mode=1, eps_grad=1e-4)
    with Optimizer(prob, cfg, x0) as opt:
        opt.cycle(2)
        before = opt.get_state()["X"].copy()
        with pytest.raises(L.ChisaoError) as ei:
            opt.cycle(1)
        assert ei.value.code == L.E_STATE
        np.testing.assert_array_equal(opt.get_state()["X"], before)


def test_modes_capacity_error_reports_count():
    import ctypes as C

    from paper_2606_26164_amd import _lib as L
    from paper_2606_26164_amd.api import Optimizer

    prob, cfg, x0 = W.gauss4_d2(N=64)
    cfg = cfg.with_(n_osc=3, grad_mode=1, eps_grad=1e-4)
    with Optimizer(prob, cfg, x0) as opt:
        opt.cycle(3)
        n = C.c_int(-1)
        X = np.zeros((1, 2), np.float32)
        rc = opt.lib.chisao_modes(opt.h, 0, X.ctypes.data, None, 0, C.byref(n))
        assert rc == L.E_RANGE and n.value == len(opt.modes().X) and n.value >= 1
        assert np.all(X == 0)


def test_invalid_problems_are_rejected():
    from paper_2606_26164_amd import _lib as L
    from paper_2606_26164_amd.api import Optimizer

    prob, cfg, x0 = W.gauss4_d2(N=16)
    bad = W.mixture_problem(0, 2, 4, 5.0, isotropic_var=0.25, dirichlet=None)
    bad.prec = bad.prec.copy()
    bad.prec[0, 0, 1] += 0.5  # not symmetric
    with pytest.raises(L.ChisaoError) as ei:
        Optimizer(bad, cfg, x0)
    assert ei.value.code == L.E_INVAL
    bad2 = W.mixture_problem(0, 2, 4, 5.0, isotropic_var=0.25, dirichlet=None)
    bad2.prec = bad2.prec.copy()
    bad2.prec[1] = -bad2.prec[1]  # symmetric, not positive definite
    with pytest.raises(L.ChisaoError) as ei:
        Optimizer(bad2, cfg, x0)
    assert ei.value.code == L.E_INVAL
    with pytest.raises(L.ChisaoError):
        Optimizer(prob, cfg.with_(M=33), x0)
    outside = x0.copy()
    outside[3, 0] = 100.0
    with pytest.raises(L.ChisaoError):
        Optimizer(prob, cfg, outside)


def test_same_seed_same_state_bitwise():
    from paper_2606_26164_amd.api import Optimizer

    prob, cfg, x0 = W.gauss128_d64(N=256, n_osc=3)
    outs = []
    for _ in range(2):
        with Optimizer(prob, cfg, x0) as opt:
            opt.cycle(2)
            outs.append(opt.get_state())
    for key in ("X", "F", "G", "stuck", "active", "trace"):
        np.testing.assert_array_equal(outs[0][key], outs[1][key], err_msg=key)


def test_gauss128_d64_shape_runs_every_phase():
    """d=64, K=128 at a small population: every phase executes and the state
    stays inside the box; sample counts are consistent."""
    from paper_2606_26164_amd.api import Optimizer

    prob, cfg, x0 = W.gauss128_d64(N=512, n_osc=4)
    with Optimizer(prob, cfg, x0) as opt:
        stats = opt.cycle(4, stats=True)
        st = opt.get_state()
    X = st["X"]
    assert np.all(X >= prob.lo) and np.all(X <= prob.hi)
    for s in stats:
        assert s["n_modes"] + s["K_lost"] == s["n_stuck"]
    for s in stats[:-1]:  # phases 4-6 do not run in the last cycle
        assert s["sigma"] == pytest.approx(0.1)
        assert s["n_unfrozen"] > 0 and s["alpha_c"] > 0 and s["alpha_a"] > 0
    assert stats[0]["evals"] > 512 * 18


def _distinct(X, tol=1e-2):
    out = []
    for x in X:
        if not any(np.max(np.abs(x - y)) < tol for y in out):
            out.append(x)
    return len(out)


def test_ablation_without_deduplication_saturates_the_population():
    """The ablation of Sec. 5.6 (Phase 3 off): nothing is removed, so nothing
    is reseeded, every converged sample stays frozen and the unfrozen
    population drains; the mode list fills with copies of the first modes.
    With Phase 3 the list holds each mode once."""
    import workloads as W
    from paper_2606_26164_amd.api import Optimizer

    prob = W.mixture_problem(31, 8, 12, 4.0, lam_range=(0.3, 1.0))
    res = {}
    for name, mask in (("full", 0x7E), ("no dedup", 0x7E & ~(1 << 3))):
        cfg = W.RunConfig(N=600, m=6, n_osc=6, n_conv=25, eps_grad=1e-3, grad_mode=1, seed=9, phase_mask=mask)
        with Optimizer(prob, cfg, W.uniform_population(9, 600, prob.lo, prob.hi)) as opt:
            st = opt.cycle(cfg.n_osc, stats=True)
            ms = opt.modes()
        res[name] = (st, len(ms.F), _distinct(ms.X))
        print(f"\n{name}: stuck per cycle {[s['n_stuck'] for s in st]}, K_lost {[s['K_lost'] for s in st]}, "
              f"modes {len(ms.F)} ({res[name][2]} distinct), unfrozen {st[-2]['n_unfrozen']}")
    st, n, nd = res["no dedup"]
    assert all(s["K_lost"] == 0 for s in st)
    assert n >= 10 * nd
    assert st[-2]["n_unfrozen"] <= 6
    st, n, nd = res["full"]
    assert n == nd and any(s["K_lost"] > 0 for s in st)


def test_non_finite_sample_is_taken_out_of_use():
    """A NaN row given through set_state is deactivated at Phase 2 and
    counted; every other sample then ends the run bitwise as in a handle where
    that slot was inactive from the start (the guard keeps it out of f_max,
    the smoothing scale, the step lengths and the reseeding lists).  The FP64
    oracle does the same (test_non_finite_sample_equals_an_empty_slot)."""
    from paper_2606_26164_amd.api import Optimizer

    prob = W.mixture_problem(3, 16, 12, 4.0, lam_range=(0.3, 1.0))
    cfg = W.RunConfig(N=700, m=6, n_osc=3, n_conv=14, M=8, eps_grad=1e-3, grad_mode=1, seed=5)
    x0 = W.uniform_population(4, 700, prob.lo, prob.hi)
    bad = 301
    out = []
    for variant in ("nan", "inactive"):
        with Optimizer(prob, cfg, x0) as opt:
            if variant == "nan":
                X = x0.copy()
                X[bad] = np.nan
                opt.set_state(X=X)
            else:
                act = np.ones(700, np.uint8)
                act[bad] = 0
                opt.set_state(active=act)
            stats = opt.cycle(3, stats=True)
            out.append((stats, opt.get_state(), opt.modes()))
    (s_nan, st_nan, m_nan), (s_off, st_off, m_off) = out
    assert [s["n_nonfinite"] for s in s_nan] == [1, 0, 0]
    assert all(s["n_nonfinite"] == 0 for s in s_off)
    assert st_nan["active"][bad] == 0 and st_nan["stuck"][bad] == 0
    keep = np.arange(700) != bad
    np.testing.assert_array_equal(st_nan["X"][keep], st_off["X"][keep])
    np.testing.assert_array_equal(st_nan["active"], st_off["active"])
    np.testing.assert_array_equal(st_nan["stuck"], st_off["stuck"])
    for a, b in zip(s_nan, s_off):
        assert np.isfinite(a["sigma"]) and a["sigma"] == b["sigma"] and a["alpha_a"] == b["alpha_a"]
        assert a["f_max"] == b["f_max"] and a["n_modes"] == b["n_modes"]
    np.testing.assert_array_equal(m_nan.X, m_off.X)


def test_step_counts_above_the_counter_field_are_rejected():
    """The step index has 8 bits of a random-stream counter word."""
    from paper_2606_26164_amd import _lib as L
    from paper_2606_26164_amd.api import Optimizer

    prob, cfg, x0 = W.gauss4_d2(N=16)
    for field in ("n_conv", "n_cloud", "n_anti"):
        with pytest.raises(L.ChisaoError) as ei:
            Optimizer(prob, cfg.with_(**{field: 256}), x0)
        assert ei.value.code == L.E_INVAL
    with Optimizer(prob, cfg.with_(n_conv=255, n_cloud=255, n_anti=255, n_osc=1), x0):
        pass
