"""Per-phase and per-cycle parity of the GPU cycle against the FP64 oracle.

Protocol: the GPU runs a phase (or a cycle) from a state; the oracle runs the
same phase from the same state (float32 values widened exactly), following the
GPU's discrete decisions (line-search index, curvature store, convergence,
stick, deduplication).  Each decision on which the oracle disagrees must be
borderline by the oracle's own margin; continuous results must agree within
the stated tolerance.
"""
import numpy as np
import pytest

import workloads as W
from oracle import oracle as O

pytestmark = pytest.mark.gpu

# borderline widths of the replay (relative Armijo margin, relative distance of
# |g|_inf to eps_grad, cosine margin of the curvature test, absolute L-inf
# distance to eps_dup)
REPLAY = dict(tol_f=1e-4, tol_g=0.2, tol_curv=1e-2, tol_dist=1e-5)


def _gpu(prob, cfg, x0):
    from paper_2606_26164_amd.api import Optimizer

    return Optimizer(prob, cfg, x0)


def _oracle_from(prob, cfg, st):
    run = O.OracleRun(prob, cfg, st["X"])
    run.F[:] = st["F"]
    run.G[:] = st["G"]
    run.stuck[:] = st["stuck"]
    run.active[:] = st["active"]
    run.st.k = st["k"]
    for f in ("gr_disabled", "gr_fail", "gr_used_last", "gr_prev_modes"):
        setattr(run.st, f, st[f])
    return run


def _close(got, want, rtol, atol, what):
    err = np.abs(np.asarray(got, np.float64) - want)
    tol = rtol * np.abs(want) + atol
    bad = err > tol
    assert not bad.any(), f"{what}: {bad.sum()} entries off, worst {err.max():.3g} (tol at worst {tol.flat[np.argmax(err)]:.3g})"


def _rows_close(got, want, rel, what, floor=1.0):
    """Norm-wise per-sample check: |got_i - want_i|_inf <= rel * max(|want_i|_inf, floor)."""
    got = np.asarray(got, np.float64).reshape(len(want), -1)
    want = np.asarray(want, np.float64).reshape(len(want), -1)
    err = np.abs(got - want).max(1)
    scale = np.maximum(np.abs(want).max(1), floor)
    ratio = err / scale
    assert np.all(ratio <= rel), f"{what}: {np.sum(ratio > rel)} rows off, worst relative {ratio.max():.3g} > {rel:g}"
    return ratio


PH1 = [
    ("cfg3-shape", lambda: W.gauss128_d64(N=256, n_osc=3)),
    ("few wide modes", lambda: (lambda p: (p, W.RunConfig(N=300, m=6, n_osc=3, n_conv=15, eps_grad=1e-3,
                                                          grad_mode=1, seed=5),
                                          W.uniform_population(5, 300, p.lo, p.hi)))(
        W.mixture_problem(31, 8, 6, 4.0, lam_range=(0.3, 1.0)))),
]


@pytest.mark.parametrize("name,make", PH1, ids=[p[0] for p in PH1])
def test_phase1_adjoint_parity_with_replay(name, make):
    """All n_conv adjoint L-BFGS iterations of Phase 1 against the oracle:
    per-sample states within relative 1e-4 (sup-norm, the state's own scale)."""
    prob, cfg, x0 = make()
    with _gpu(prob, cfg, x0) as opt:
        opt.run_phases(1 << 1)
        g = opt.get_state()
    run = O.OracleRun(prob, cfg, x0)
    rep = run.phase_converge(trace_in=g["trace"], **REPLAY)
    print(f"\n{name}: decisions {rep.n_decisions} borderline by kind {rep.border_by_kind} hard {rep.n_hard}")
    assert rep.n_hard == 0, rep
    iterated = g["trace"] != O.TR_NONE
    assert np.array_equal(iterated, run.trace != O.TR_NONE)
    r = _rows_close(g["X"], run.X, 1e-4, "X after phase 1")
    print(f"  X relative error: max {r.max():.2e}, 99% {np.quantile(r, 0.99):.2e}")
    # values and gradients are those of the GPU's own positions
    f_at, G_at = run.P.eval(g["X"].astype(np.float64))
    _rows_close(g["F"][:, None], f_at[:, None], 1e-5, "F after phase 1")
    _rows_close(g["G"], G_at, 1e-4, "G after phase 1", floor=1.0)


@pytest.mark.parametrize("grad_mode", [1, 0])
def test_lbfgs_single_iteration_parity(grad_mode):
    """One L-BFGS iteration from the GPU's own state (positions, gradients,
    histories), so FP32 differences cannot compound: the oracle continues from
    the state after t iterations and must reproduce the GPU's state after t+1.
    With central differences this is the only meaningful per-step comparison:
    curvature pairs difference two FP32 finite-difference gradients, whose
    rounding (~1e-3 relative at |f| ~ 1e3) the BFGS update amplifies."""
    prob, cfg, x0 = W.gauss32_d16(N=256, n_osc=3) if grad_mode == 0 else W.gauss128_d64(N=192, n_osc=3)
    cfg = cfg.with_(grad_mode=grad_mode)
    op = O.OracleProblem(prob)
    for t in (1, 2, 5, cfg.n_conv - 1):
        with _gpu(prob, cfg.with_(n_conv=t), x0) as opt:
            opt.run_phases(1 << 1)
            a = opt.get_state(history=True)
        with _gpu(prob, cfg.with_(n_conv=t + 1), x0) as opt:
            opt.run_phases(1 << 1)
            b = opt.get_state(history=True)
        ccfg = cfg.with_(n_conv=t + 1)
        run = _oracle_from(prob, ccfg, a)
        run.S[:] = a["S"]
        run.Y[:] = a["Y"]
        run.rho[:] = a["rho"]
        run.head[:] = a["head"]
        run.cnt[:] = a["cnt"]
        run.conv[:] = a["conv"] == 1  # stalled samples (2) are iterated by the oracle and fail again
        rep = run.iterate(t + 1, 1, trace_in=b["trace"], **REPLAY)
        moved = b["trace"][t + 1] != O.TR_NONE
        print(f"\nmode {grad_mode} t={t}: iterated {moved.sum()} borderline {rep.border_by_kind} hard {rep.n_hard}")
        assert rep.n_hard == 0, rep
        assert moved.sum() > 0
        rx = _rows_close(b["X"][moved], run.X[moved], 1e-5, f"X after iteration {t + 1}")
        f_or = run.F[moved]
        _rows_close(b["F"][moved][:, None], f_or[:, None], 1e-5, f"F after iteration {t + 1}")
        if grad_mode == 1:
            _rows_close(b["G"][moved], run.G[moved], 1e-3, f"G after iteration {t + 1}")
        else:
            # per-component bound of the FP32 central difference (see test_gpu_eval):
            # 2 * 64 u (|f| + q_max/2 + 1) / (2 h_j), plus the step's own relative error
            Xd = run.X[moved]
            qmax = np.zeros(len(Xd))
            for k in range(op.K):
                dl = Xd - op.mu[k]
                qmax = np.maximum(qmax, np.einsum("ni,ij,nj->n", dl, op.prec[k], dl))
            fb = 64 * 2.0 ** -24 * (np.abs(f_or) + 0.5 * qmax + 1.0)
            h = np.ldexp(np.maximum(1.0, np.abs(Xd)), -8)
            gs = np.abs(run.G[moved]).max(1, keepdims=True)
            bound = 2 * fb[:, None] / (2 * h) + 1e-4 * gs + 1e-5
            err = np.abs(b["G"][moved] - run.G[moved])
            assert np.all(err <= bound), f"FD gradient after iteration {t + 1}: worst {err.max():.3g}"
        print(f"  X relative error max {rx.max():.2e}")


def _many_stuck_case(grad_mode=1):
    """Eight dimensions, six wide components: most samples converge, so the
    stick test, deduplication and reseeding all have work."""
    prob = W.mixture_problem(31, 8, 6, 4.0, lam_range=(0.3, 1.0))
    cfg = W.RunConfig(N=600, m=6, n_osc=4, n_conv=25, eps_grad=1e-3, grad_mode=grad_mode, seed=9)
    return prob, cfg, W.uniform_population(9, 600, prob.lo, prob.hi)


def test_phases_2_3_stick_and_dedup_parity():
    prob, cfg, x0 = _many_stuck_case()
    with _gpu(prob, cfg, x0) as opt:
        opt.run_phases((1 << 1))
        g1 = opt.get_state()
        opt.run_phases((1 << 2) | (1 << 3))
        g3 = opt.get_state()
    assert g3["stuck_pre"].sum() > 50 and g3["removed"].sum() > 20
    run = _oracle_from(prob, cfg, g1)
    r2 = run.phase_stick(stuck_in=g3["stuck_pre"], **REPLAY)
    r3 = run.phase_dedup(removed_in=g3["removed"], **REPLAY)
    print(f"\nstick: {r2}\ndedup: {r3}")
    assert r2.n_hard == 0 and r3.n_hard == 0
    np.testing.assert_array_equal(run.stuck, g3["stuck"])
    # without replay the oracle's own decisions differ only on borderline samples
    free = _oracle_from(prob, cfg, g1)
    free.phase_stick()
    assert (free.stuck != g3["stuck_pre"]).sum() <= r2.n_borderline


@pytest.mark.parametrize("N", [3000, 12000])
def test_dedup_rank_order_matches_oracle_many_stuck(N):
    """Deduplication with thousands of stuck samples in a few loose clusters
    (d=2, wide components): the sorted path in LDS (3000) and in global
    memory (12000, above the LDS capacity of 8192) against the oracle's
    all-pairs rule, decisions replayed only where borderline."""
    prob = W.mixture_problem(7, 2, 5, 3.0, lam_range=(0.5, 1.0))
    cfg = W.RunConfig(N=N, m=6, n_osc=3, n_conv=30, eps_grad=1e-3, grad_mode=1, seed=4)
    x0 = W.uniform_population(7, N, prob.lo, prob.hi)
    with _gpu(prob, cfg, x0) as opt:
        opt.run_phases(1 << 1)
        g1 = opt.get_state()
        opt.run_phases((1 << 2) | (1 << 3))
        g3 = opt.get_state()
    n_stuck = int(g3["stuck_pre"].sum())
    print(f"\nN={N}: stuck {n_stuck}, removed {int(g3['removed'].sum())}, modes {int(g3['stuck'].sum())}")
    assert n_stuck > 0.6 * N
    run = _oracle_from(prob, cfg, g1)
    r2 = run.phase_stick(stuck_in=g3["stuck_pre"], **REPLAY)
    r3 = run.phase_dedup(removed_in=g3["removed"], **REPLAY)
    assert r2.n_hard == 0 and r3.n_hard == 0, (r2, r3)
    np.testing.assert_array_equal(run.stuck, g3["stuck"])


def test_phase4_repulse_monkey_parity():
    prob, cfg, x0 = _many_stuck_case()
    with _gpu(prob, cfg, x0) as opt:
        opt.run_phases((1 << 1) | (1 << 2) | (1 << 3))
        g3 = opt.get_state()
        opt.run_phases(1 << 4)
        g4 = opt.get_state()
    run = _oracle_from(prob, cfg, g3)
    run.removed[:] = g3["removed"]
    run.st.K_lost = int(g3["removed"].sum())
    run.st.n_modes = int(g3["stuck"].sum())
    run.phase_reseed()
    assert run.st.reseed_kind == 1
    slots = np.nonzero(g3["removed"])[0]
    assert len(slots) > 0
    # origin indices and uniform fractions are exact; directions differ by the
    # FP32 Box-Muller rounding
    span = (prob.hi - prob.lo).max()
    _close(g4["X"][slots], run.X[slots], 0.0, 2e-5 * span, "reseeded positions")
    others = np.setdiff1d(np.arange(cfg.N), slots)
    np.testing.assert_array_equal(g4["X"][others], g3["X"][others])
    assert np.all(g4["stuck"][slots] == 0) and np.all(g4["active"][slots] == 1)


def test_phase4_golden_rooster_parity():
    """One component: every sample sticks at the centre and all but one are
    duplicates, so fewer than five samples stay free and Golden Rooster
    reseeds along orthonormal directions from the single peak."""
    prob = W.mixture_problem(41, 12, 1, 3.0, lam_range=(0.3, 1.0), dirichlet=None)
    cfg = W.RunConfig(N=200, m=8, n_osc=4, n_conv=30, eps_grad=1e-3, grad_mode=1, seed=4)
    x0 = W.uniform_population(41, 200, prob.lo, prob.hi)
    with _gpu(prob, cfg, x0) as opt:
        opt.run_phases((1 << 1) | (1 << 2) | (1 << 3))
        g3 = opt.get_state()
        opt.run_phases(1 << 4)
        g4 = opt.get_state()
    assert g3["stuck"].sum() == 1 and g3["removed"].sum() == 199
    run = _oracle_from(prob, cfg, g3)
    run.removed[:] = g3["removed"]
    run.st.K_lost = 199
    run.st.n_modes = 1
    run.phase_reseed()
    assert run.st.reseed_kind == 2
    slots = np.nonzero(g3["removed"])[0]
    span = (prob.hi - prob.lo).max()
    _close(g4["X"][slots], run.X[slots], 0.0, 2e-4 * span, "Golden Rooster positions")
    assert np.all(g4["active"][slots] == 1) and np.all(g4["stuck"][slots] == 0)


# an even probe count generates each antithetic pair in one pass; an odd one
# leaves the last probe unpaired and takes the per-point path
@pytest.mark.parametrize("sigma,grad_mode,M", [(0.0, 1, 10), (0.3, 1, 10), (0.0, 0, 10), (0.3, 0, 10), (0.3, 1, 7)])
def test_phases_5_6_smoothing_and_anti_parity(sigma, grad_mode, M):
    prob = W.mixture_problem(51, 16, 12, 5.0, lam_range=(0.2, 1.0))
    cfg = W.RunConfig(N=300, m=6, n_osc=4, n_conv=12, M=M, sigma=sigma, eps_grad=1e-3, grad_mode=grad_mode, seed=6)
    x0 = W.uniform_population(51, 300, prob.lo, prob.hi)
    stuck = np.zeros(300, np.uint8)
    stuck[::7] = 1
    with _gpu(prob, cfg, x0) as opt:
        opt.set_state(stuck=stuck, k=1)
        g0 = opt.get_state()
        opt.run_phases((1 << 5) | (1 << 6))
        g6 = opt.get_state()
    run = _oracle_from(prob, cfg, g0)
    run.phase_hlc()
    run.phase_anti()
    moved = stuck == 0
    np.testing.assert_array_equal(g6["X"][~moved], g0["X"][~moved])
    disp_or = run.X[moved] - g0["X"][moved]
    disp_gpu = g6["X"][moved].astype(np.float64) - g0["X"][moved]
    # adjoint: FP32 rounding of gradients and step lengths, relative 1e-4 of each
    # sample's displacement; central differences add their FP32 rounding,
    # ~64 u (|f| + q/2) / (2 h |g|) ~ 2e-3 of the gradient at these points
    rel = 1e-4 if grad_mode == 1 else 5e-3
    r = _rows_close(disp_gpu, disp_or, rel, "phase 5-6 displacement", floor=1e-3)
    print(f"\nsigma={sigma} mode={grad_mode} M={M}: displacement relative error max {r.max():.2e}")
    assert run.st.sigma == pytest.approx(float(sigma) if sigma > 0 else run.st.sigma)


def test_full_cycle_parity_with_replay():
    """Two cycles of the many-mode case: each GPU cycle is replayed by the
    oracle from the GPU's state at the start of that cycle."""
    prob, cfg, x0 = _many_stuck_case()
    with _gpu(prob, cfg, x0) as opt:
        for _ in range(2):
            s0 = opt.get_state()
            opt.cycle(1)
            s1 = opt.get_state()
            run = _oracle_from(prob, cfg, s0)
            rep = run.cycle(trace_in=s1["trace"], stuck_in=s1["stuck_pre"], removed_in=s1["removed"], **REPLAY)
            print(f"\ncycle {s1['k']}: {rep} {run.stats()}")
            assert rep.n_hard == 0
            assert run.k == s1["k"]
            np.testing.assert_array_equal(run.active, s1["active"])
            np.testing.assert_array_equal(run.stuck, s1["stuck"])
            r = _rows_close(s1["X"], run.X, 1e-4, f"X after cycle {s1['k']}")
            print(f"  X relative error max {r.max():.2e}")


@pytest.mark.parametrize("N,eps_dup", [(20000, 1e-3), (6000, 0.7)])
def test_dedup_lattice_of_maxima_matches_oracle(N, eps_dup):
    """Styblinski-Tang in d=16 has 2^16 local maxima on a lattice whose
    points share coordinate values, with the quality gate opened
    (log_delta = -1e30) so that every stationary sample sticks: thousands of
    distinct maxima plus duplicates, the case the spatial hash is for.  With
    eps_dup = 0.7 converged copies and near-converged samples chain across
    hash cells.  Decisions against the oracle's all-pairs rule."""
    prob = W.closed_form_problem("styblinski_tang", 16)
    cfg = W.RunConfig(N=N, m=8, n_osc=3, n_conv=30, eps_grad=1e-2, eps_dup=eps_dup, log_delta=-1e30,
                      grad_mode=1, seed=2)
    x0 = W.uniform_population(2, N, prob.lo, prob.hi)
    with _gpu(prob, cfg, x0) as opt:
        opt.run_phases(1 << 1)
        g1 = opt.get_state()
        opt.run_phases((1 << 2) | (1 << 3))
        g3 = opt.get_state()
    n_stuck = int(g3["stuck_pre"].sum())
    print(f"\nN={N} eps_dup={eps_dup}: stuck {n_stuck}, removed {int(g3['removed'].sum())}, "
          f"modes {int(g3['stuck'].sum())}")
    assert n_stuck > 0.5 * N and g3["removed"].sum() > 0
    run = _oracle_from(prob, cfg, g1)
    r2 = run.phase_stick(stuck_in=g3["stuck_pre"], **REPLAY)
    r3 = run.phase_dedup(removed_in=g3["removed"], **REPLAY)
    assert r2.n_hard == 0 and r3.n_hard == 0, (r2, r3)
    np.testing.assert_array_equal(run.stuck, g3["stuck"])


def test_dedup_pairs_across_hash_cells_match_oracle():
    """Designed positions: 1500 pairs whose members lie 0.5-0.9 eps_dup apart
    in the sup-norm (must be merged), 500 pairs 1.1-1.5 eps_dup apart (must
    not be), random directions, so that a large share of the merged pairs
    straddle a boundary of the deduplication hash's cells.  The phase-1 state
    of a unimodal problem with the stick test opened (every sample sticks)
    supplies values and gradients; the positions are then replaced.  Exact
    agreement with the oracle's all-pairs rule."""
    from paper_2606_26164_amd.api import Optimizer

    d, eps = 8, 1e-3
    prob = W.mixture_problem(3, d, 1, 2.0, isotropic_var=4.0)
    N = 4000
    cfg = W.RunConfig(N=N, m=6, n_osc=3, n_conv=10, eps_grad=1e9, eps_dup=eps, log_delta=-1e30, grad_mode=1,
                      seed=3)
    rng = np.random.default_rng(8)
    base = rng.uniform(-2.0, 2.0, size=(2000, d))
    sign = rng.choice([-1.0, 1.0], size=(2000, d))
    mag = np.where(np.arange(2000)[:, None] < 1500, rng.uniform(0.5, 0.9, size=(2000, d)),
                   rng.uniform(1.1, 1.5, size=(2000, d)))
    # far pairs: one coordinate beyond eps, the others anywhere inside
    far = np.arange(2000) >= 1500
    mag[far, 1:] = rng.uniform(0.0, 0.9, size=(far.sum(), d - 1))
    X = np.concatenate([base, base + sign * mag * eps]).astype(np.float32)
    x0 = W.uniform_population(3, N, prob.lo, prob.hi)
    with Optimizer(prob, cfg, x0) as opt:
        opt.run_phases(1 << 1)
        opt.set_state(X=X)
        g1 = opt.get_state()
        opt.run_phases((1 << 2) | (1 << 3))
        g3 = opt.get_state()
    assert g3["stuck_pre"].all()
    removed = g3["removed"].astype(bool)
    pair_removed = removed[:2000] | removed[2000:]
    assert pair_removed[:1500].all() and not pair_removed[1500:].any()
    run = _oracle_from(prob, cfg, g1)
    run.phase_stick()
    run.phase_dedup()
    np.testing.assert_array_equal(run.removed.astype(bool), removed)


def test_mode_widths_match_oracle_from_the_same_history():
    """Width export: after Phases 1-3 the GPU's preserved inverse-Hessian
    diagonals of the modes (BFGS recursion in LDS, FP32) against the oracle's
    (two-loop on unit vectors, FP64) from the GPU's own pairs."""
    prob, cfg, x0 = _many_stuck_case()
    with _gpu(prob, cfg, x0) as opt:
        opt.run_phases(1 << 1)
        g1 = opt.get_state(history=True)
        opt.run_phases((1 << 2) | (1 << 3))
        g3 = opt.get_state()
        ms = opt.modes()
        wg = opt.mode_widths().astype(np.float64)
    run = _oracle_from(prob, cfg, g1)
    for f in ("S", "Y", "rho", "head", "cnt"):
        getattr(run, f)[:] = g1[f]
    r2 = run.phase_stick(stuck_in=g3["stuck_pre"], **REPLAY)
    r3 = run.phase_dedup(removed_in=g3["removed"], **REPLAY)
    assert r2.n_hard == 0 and r3.n_hard == 0
    wo = run.mode_widths()
    assert wg.shape == wo.shape and len(wo) == len(ms.F) and len(wo) > 0
    assert np.all(wg > 0) and np.all(np.isfinite(wg))
    rel = np.abs(wg - wo).max(1) / np.abs(wo).max(1)
    print(f"\n{len(wo)} modes: width relative error max {rel.max():.2e}")
    assert rel.max() < 1e-3


def test_mode_widths_of_isotropic_peaks_are_the_variance():
    """Well separated isotropic Gaussian peaks (variance 0.5): near a peak the
    curvature pairs satisfy y = s / 0.5, so every preserved diagonal is the
    variance.  A whole run (3 cycles): modes found in earlier cycles keep the
    diagonal from the cycle they converged in."""
    from paper_2606_26164_amd.api import Optimizer

    prob = W.mixture_problem(12, 6, 4, 8.0, isotropic_var=0.5, dirichlet=None)
    cfg = W.RunConfig(N=400, m=8, n_osc=3, n_conv=20, eps_grad=1e-3, grad_mode=1, seed=12)
    x0 = W.uniform_population(12, 400, prob.lo, prob.hi)
    with Optimizer(prob, cfg, x0) as opt:
        opt.cycle(cfg.n_osc)
        ms = opt.modes()
        wg = opt.mode_widths().astype(np.float64)
    print(f"\n{len(ms.F)} modes, widths in [{wg.min():.4f}, {wg.max():.4f}]")
    assert len(ms.F) >= 2
    assert np.all(np.abs(wg - 0.5) < 0.05 * 0.5)


def test_resume_from_saved_state_continues_bitwise():
    """Checkpoint and resume: the state read between cycles (positions,
    masks, cycle count, Golden Rooster state, preserved widths) given to a new
    handle continues the run exactly as the uninterrupted one."""
    from paper_2606_26164_amd.api import Optimizer

    prob, cfg, x0 = _many_stuck_case()
    with Optimizer(prob, cfg, x0) as a:
        a.cycle(cfg.n_osc)
        ref = a.get_state()
        ref_m, ref_w = a.modes(), a.mode_widths()
    with Optimizer(prob, cfg, x0) as b:
        b.cycle(2)
        st = b.get_state(history=True)
    with Optimizer(prob, cfg, st["X"]) as c:
        c.set_state(stuck=st["stuck"], active=st["active"], k=st["k"],
                    gr={f: st[f] for f in ("gr_disabled", "gr_fail", "gr_used_last", "gr_prev_modes")},
                    Wd=st["Wd"], wvalid=st["wvalid"])
        c.cycle(cfg.n_osc - 2)
        got = c.get_state()
        got_m, got_w = c.modes(), c.mode_widths()
    for f in ("X", "F", "G", "stuck", "active", "removed"):
        np.testing.assert_array_equal(got[f], ref[f], err_msg=f)
    np.testing.assert_array_equal(got_m.X, ref_m.X)
    np.testing.assert_array_equal(got_w, ref_w)
    assert len(ref_m.F) > 0
