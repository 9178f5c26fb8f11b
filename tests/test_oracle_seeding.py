"""Pins of the oracle's starting populations: the structured ray seeding
(rays through the box centre from vertices, edge midpoints and face centres)
is checked against its geometry and the distributions of its draws, so a
wrong anchor, a ray that misses the centre, a biased kind, position or bound
choice fails."""
import numpy as np
import scipy.stats

import workloads as W
from oracle import oracle as O


def _rays(d, N=30000, lo=-3.0, hi=5.0, seed=4):
    prob = W.closed_form_problem("ackley", d)
    prob.lo = np.full(d, lo, np.float32)
    prob.hi = np.full(d, hi, np.float32)
    run = O.OracleRun(prob, W.RunConfig(N=N, seed=seed, flags=4))
    return (run.X - 0.5 * (lo + hi)) / (0.5 * (hi - lo))  # box mapped to [-1, 1]^d


def test_every_sample_lies_on_a_ray_through_the_centre():
    for d in (1, 2, 7, 40, 64):
        u = _rays(d, N=5000)
        a = np.abs(u)
        r = a.max(1)
        off = a > 1e-12
        # off-middle coordinates all share one distance |1 - 2t| from the centre
        assert np.all(np.abs(np.where(off, a, r[:, None]) - r[:, None]) < 1e-12)
        n_off = off.sum(1)
        if d >= 3:
            kinds = {d: "vertex", d - 1: "edge", 1: "face"}
            assert set(np.unique(n_off)) <= set(kinds), np.unique(n_off)


def test_anchor_kinds_positions_and_bounds_are_uniform():
    d, N = 9, 30000
    u = _rays(d, N=N)
    n_off = (np.abs(u) > 1e-12).sum(1)
    for k in (d, d - 1, 1):
        frac = np.mean(n_off == k)
        assert abs(frac - 1 / 3) < 5 * np.sqrt(2 / 9 / N), (k, frac)
    # the distance from the centre is |1 - 2t| with t uniform: uniform on [0, 1]
    r = np.abs(u).max(1)
    assert scipy.stats.kstest(r, "uniform").pvalue > 1e-4
    # bound choices: fair and independent across coordinates (vertex samples)
    v = u[n_off == d]
    sg = np.sign(v)
    assert np.all(np.abs(sg.mean(0)) < 5 / np.sqrt(len(v)))
    c = np.corrcoef(sg.T)[np.triu_indices(d, 1)]
    assert np.all(np.abs(c) < 5 / np.sqrt(len(v)))


def test_free_coordinate_is_uniform_and_ray_seeding_is_off_by_default():
    d, N = 6, 30000
    u = _rays(d, N=N)
    a = np.abs(u) > 1e-12
    face = a.sum(1) == 1
    e = np.argmax(a[face], 1)
    counts = np.bincount(e, minlength=d)
    assert scipy.stats.chisquare(counts).pvalue > 1e-4
    prob = W.closed_form_problem("ackley", d)
    x = O.OracleRun(prob, W.RunConfig(N=2000, seed=4)).X
    assert (np.abs(x - 0.0) > 1e-9).all(1).mean() > 0.99  # uniform: no coordinate at the middle
