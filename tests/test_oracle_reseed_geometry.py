"""Pins of the oracle's reseeding geometry (Sec. 3.2, Phase 4: Repulse Monkey
and Golden Rooster place new samples uniformly along rays inside the domain).

The checks use facts outside the oracle's reseeding code:
- the exit distance of a ray from the box is found by bisection on the
  "inside the box" predicate, not by any face formula;
- the random words come from the Philox function pinned to the published
  known-answer vectors, read through the stream layout of the readings
  (counter = slot, cycle, consumer << 24 | step << 16, block);
- distributions are tested against closed forms: the distance fraction along
  the ray is U(0, 1), each coordinate of an isotropic direction in three
  dimensions is U(-1, 1) (Archimedes), origins are uniform over the unfrozen
  samples (chi-square).

A mutation test compiles copies of the oracle with one planted mistake each
(zero exit distance, the wrong bound, an unscaled distance, a biased origin
draw) and checks that these pins reject every one.
"""
import shutil
import subprocess

import numpy as np
import pytest
import scipy.stats

import workloads as W
from oracle import oracle as O

PH_RM, PH_GR = 4, 5
LO = np.array([-1.0, -2.0, 0.5])
HI = np.array([3.0, 1.0, 4.0])
CYCLE = 5  # state cycle count k; the reseeding streams use k + 1


def _u01(a: int) -> float:
    return ((a >> 8) + 0.5) / 2.0 ** 24


def _words(cfg, slot: int, k: int, c2: int, block: int = 0):
    key = (cfg.seed & 0xFFFFFFFF, (cfg.seed >> 32) ^ cfg.problem_id)
    return O.philox4x32_10((slot, k, c2, block), key)


def exit_distance(o, u, lo=LO, hi=HI):
    """Largest t with o + t u inside [lo, hi], row by row, by bisection on the
    inside predicate (the box is convex and every o lies inside it)."""
    o, u = np.atleast_2d(o), np.atleast_2d(u)

    def inside(t):
        p = o + t[:, None] * u
        return np.all((p >= lo) & (p <= hi), axis=1)

    a = np.zeros(len(o))
    b = np.full(len(o), 4.0 * np.linalg.norm(hi - lo) + 1.0)
    assert inside(a).all() and not inside(b).any()
    for _ in range(200):
        mid = 0.5 * (a + b)
        ins = inside(mid)
        a, b = np.where(ins, mid, a), np.where(ins, b, mid)
    return a


def _case(roles, pos, seed=11):
    """An oracle state on the test box: 'p' = stuck survivor (peak), 'f' =
    unfrozen sample, 's' = slot removed by deduplication."""
    N, d = len(roles), LO.size
    prob = W.mixture_problem(14, d, 1, 1.0, isotropic_var=1.0)
    cfg = W.RunConfig(N=N, m=2, seed=seed, problem_id=3)
    run = O.OracleRun(prob, cfg, pos)
    run.P.lo[:] = LO  # the C problem points at these arrays
    run.P.hi[:] = HI
    run.stuck[:] = [r == "p" for r in roles]
    run.removed[:] = [r == "s" for r in roles]
    run.st.k = CYCLE
    run.st.K_lost = roles.count("s")
    run.st.n_modes = roles.count("p")
    return run, cfg


def _roles(n_peaks, n_free, n_slots, seed):
    roles = ["p"] * n_peaks + ["f"] * n_free + ["s"] * n_slots
    np.random.default_rng(seed).shuffle(roles)
    return roles


def _rm_runs(n_free=7, n_slots=1400):
    """The same slots and draws twice: every unfrozen sample at one point
    (the origin's position is then known), and at distinct points."""
    roles = _roles(2, n_free, n_slots, 21)
    rng = np.random.default_rng(22)
    pos = rng.uniform(LO + 0.1, HI - 0.1, size=(len(roles), 3))
    o_common = np.array([0.2, -0.5, 1.7])
    pos_a = pos.copy()
    pos_a[[r == "f" for r in roles]] = o_common
    run_a, cfg = _case(roles, pos_a)
    run_a.phase_reseed()
    run_b, _ = _case(roles, pos)
    run_b.phase_reseed()
    return roles, pos, o_common, run_a, run_b, cfg


def check_rm_distance():
    roles, _, o, run, _, cfg = _rm_runs()
    assert run.st.reseed_kind == 1
    slots = [i for i, r in enumerate(roles) if r == "s"]
    v = run.X[slots] - o
    r = np.linalg.norm(v, axis=1)
    assert np.all(r > 0), "a reseeded sample sits on its origin"
    u = v / r[:, None]
    t = exit_distance(np.broadcast_to(o, u.shape), u)
    frac = np.array([_u01(_words(cfg, s, CYCLE + 1, PH_RM << 24)[1]) for s in slots])
    np.testing.assert_allclose(r, frac * t, rtol=1e-12, atol=1e-13)
    # distributions that hold whatever the draws
    assert scipy.stats.kstest(r / t, "uniform").pvalue > 1e-4
    for c in range(3):
        assert scipy.stats.kstest((u[:, c] + 1) / 2, "uniform").pvalue > 1e-4


def check_rm_origins():
    roles, pos, o_common, run_a, run_b, cfg = _rm_runs()
    assert run_b.st.reseed_kind == 1
    free = [i for i, r in enumerate(roles) if r == "f"]
    slots = [i for i, r in enumerate(roles) if r == "s"]
    # direction and fraction of each slot from the common-origin run
    v = run_a.X[slots] - o_common
    r = np.linalg.norm(v, axis=1)
    u = v / r[:, None]
    frac = r / exit_distance(np.broadcast_to(o_common, u.shape), u)
    # every (slot, unfrozen sample) pair at once: where the drawn ray from that
    # origin would put the slot
    nf, ns = len(free), len(slots)
    o = np.repeat(pos[free][None], ns, axis=0).reshape(-1, 3)
    uu = np.repeat(u, nf, axis=0)
    t = exit_distance(o, uu).reshape(ns, nf)
    pred = pos[free][None] + (frac[:, None] * t)[..., None] * u[:, None, :]
    hits = np.abs(pred - run_b.X[slots][:, None, :]).max(2) <= 1e-11
    assert np.all(hits.sum(1) == 1), "a new point lies on the drawn ray from no origin or from several"
    idx = hits.argmax(1)
    a0 = np.array([_words(cfg, s, CYCLE + 1, PH_RM << 24)[0] for s in slots], dtype=np.uint64)
    np.testing.assert_array_equal(idx, (a0 * np.uint64(nf)) >> np.uint64(32))  # position in ascending order
    counts = np.bincount(idx, minlength=nf)
    assert scipy.stats.chisquare(counts).pvalue > 1e-4


def check_gr_distance():
    n_peaks, n_slots = 2, 600
    roles = _roles(n_peaks, 3, n_slots, 31)  # three unfrozen samples: too few for Repulse Monkey
    pos = np.random.default_rng(32).uniform(LO + 0.1, HI - 0.1, size=(len(roles), 3))
    run, cfg = _case(roles, pos)
    run.phase_reseed()
    assert run.st.reseed_kind == 2
    peaks = [i for i, r in enumerate(roles) if r == "p"]
    slots = [i for i, r in enumerate(roles) if r == "s"]
    o = pos[[peaks[j % n_peaks] for j in range(n_slots)]]
    v = run.X[slots] - o
    r = np.linalg.norm(v, axis=1)
    assert np.all(r > 0)
    u = v / r[:, None]
    t = exit_distance(o, u)
    frac = np.array([_u01(_words(cfg, s, CYCLE + 1, (PH_GR << 24) | (1 << 16))[0]) for s in slots])
    np.testing.assert_allclose(r, frac * t, rtol=1e-12, atol=1e-13)
    assert scipy.stats.kstest(r / t, "uniform").pvalue > 1e-4
    # each peak's directions: column (q // 2) mod d of one orthogonal matrix, sign (-1)^q
    for p in range(n_peaks):
        js = np.arange(p, n_slots, n_peaks)
        q = js // n_peaks
        cols = np.stack([u[js[np.nonzero((q // 2) % 3 == c)[0][0]]] for c in range(3)], axis=1)
        np.testing.assert_allclose(cols.T @ cols, np.eye(3), atol=1e-12)
        want = ((-1.0) ** q)[:, None] * cols[:, (q // 2) % 3].T
        np.testing.assert_allclose(u[js], want, atol=1e-12)


def check_gr_haar_first_columns():
    """With one slot per peak every slot takes its peak's first column; over
    many peaks these are uniform on the sphere when Q is Haar distributed."""
    n = 400
    roles = _roles(n, 2, n, 41)
    pos = np.random.default_rng(42).uniform(LO + 0.1, HI - 0.1, size=(len(roles), 3))
    run, _ = _case(roles, pos)
    run.phase_reseed()
    assert run.st.reseed_kind == 2
    peaks = [i for i, r in enumerate(roles) if r == "p"]
    slots = [i for i, r in enumerate(roles) if r == "s"]
    v = run.X[slots] - pos[peaks]
    r = np.linalg.norm(v, axis=1)
    assert np.all(r > 0)
    u = v / r[:, None]
    for c in range(3):
        assert scipy.stats.kstest((u[:, c] + 1) / 2, "uniform").pvalue > 1e-4


CHECKS = [check_rm_distance, check_rm_origins, check_gr_distance, check_gr_haar_first_columns]


@pytest.mark.parametrize("check", CHECKS, ids=lambda c: c.__name__)
def test_reseed_geometry(check):
    check()


# planted mistakes: (name, text in the oracle source, replacement)
MUTATIONS = [
    ("zero exit distance", "    if (isinf(tmax)) tmax = 0.0;\n    return tmax;",
     "    if (isinf(tmax)) tmax = 0.0;\n    return 0.0;"),
    ("half the exit distance", "    if (isinf(tmax)) tmax = 0.0;\n    return tmax;",
     "    if (isinf(tmax)) tmax = 0.0;\n    return 0.5 * tmax;"),
    ("upper bound for negative directions", "tmax = fmin(tmax, (P->lo[l] - o[l]) / u[l]);",
     "tmax = fmin(tmax, (P->hi[l] - o[l]) / u[l]);"),
    ("distance not scaled by the exit distance", "x[l] = o[l] + frac * tmax * u[l];",
     "x[l] = o[l] + frac * u[l];"),
    ("origin never the last unfrozen sample", "freel[uint_below(o4[0], (uint32_t)nf)]",
     "freel[uint_below(o4[0], (uint32_t)(nf - 1))]"),
    ("origin and fraction from the same word", "double frac = orc_u01(o4[1]);",
     "double frac = orc_u01(o4[0]);"),
]


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_reject_planted_mistakes(tmp_path, name, old, new):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    src = open(O.SRC).read()
    assert old in src, f"mutation site for '{name}' not found"
    bad = tmp_path / "oracle_mutant.c"
    bad.write_text(src.replace(old, new))
    so = tmp_path / "liboracle_mutant.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                    "-fno-fast-math", "-o", str(so), str(bad), "-lm"], check=True)
    caught = None
    with O.using_library(str(so)):
        for check in CHECKS:
            try:
                check()
            except AssertionError:
                caught = check.__name__
                break
    assert caught, f"no pin rejects the planted mistake '{name}'"
    check_gr_distance()  # the unmutated build is back in use
