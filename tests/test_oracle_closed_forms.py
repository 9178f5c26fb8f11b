"""Pins of the oracle's closed-form test functions (Appendix D).

Each function is checked against facts that do not come from its own code:
optimum locations and values the paper states, exact special values (integer
points of Rastrigin, the point pi/2 of Michalewicz), brute-force grid maxima,
symmetries, and for every gradient a Richardson-extrapolated numerical
derivative of the value.  A sign flip, a dropped term, a wrong constant or an
off-by-one coordinate index fails at least one of them.
"""
import numpy as np
import pytest

import workloads as W
from oracle import oracle as O

FAMS = ["rastrigin", "ackley", "schwefel", "styblinski_tang", "michalewicz", "trid", "bukin6"]


def _op(name, d):
    return O.OracleProblem(W.closed_form_problem(name, d))


def _f(op, X):
    return op.eval(np.atleast_2d(X), grad=False)


def _num_grad(op, x, h):
    """Richardson-extrapolated central differences of the oracle's value."""
    d = x.size
    g = np.empty(d)
    for j in range(d):
        e = np.zeros(d)
        e[j] = 1.0
        pts = np.stack([x + 2 * h * e, x + h * e, x - h * e, x - 2 * h * e])
        fp2, fp1, fm1, fm2 = _f(op, pts)
        g[j] = (-fp2 + 8 * fp1 - 8 * fm1 + fm2) / (12 * h)
    return g


# --------------------------------------------------------------------------
# values and optima the paper states
# --------------------------------------------------------------------------

@pytest.mark.parametrize("d", [1, 2, 7, 64])
def test_rastrigin_origin_and_integer_points(d):
    op = _op("rastrigin", d)
    f, g = op.eval(np.zeros((1, d)))
    assert f[0] == 0.0 and np.all(g == 0.0)
    # cos(2 pi k) = 1 at integers: f = -sum k^2
    k = np.random.default_rng(d).integers(-5, 6, size=(4, d)).astype(float)
    np.testing.assert_allclose(_f(op, k), -(k ** 2).sum(1), rtol=0, atol=1e-9)


@pytest.mark.parametrize("d", [1, 3, 64])
def test_ackley_origin_is_zero_maximum_and_symmetric(d):
    op = _op("ackley", d)
    f, g = op.eval(np.zeros((1, d)))
    assert abs(f[0]) < 1e-12 and np.all(g == 0.0)
    rng = np.random.default_rng(1)
    X = rng.uniform(-32.768, 32.768, size=(64, d))
    fx = _f(op, X)
    assert np.all(fx < 0.0)
    # invariant under coordinate permutations and sign flips
    perm = rng.permutation(d)
    sign = rng.choice([-1.0, 1.0], size=d)
    np.testing.assert_allclose(_f(op, X[:, perm] * sign), fx, rtol=1e-13, atol=1e-12)


def test_schwefel_optimum_near_420_97():
    # the paper: global maximum near theta_i = 420.97, and the constant
    # 418.9829 d makes its value (almost) zero
    for d in (1, 2, 16, 64):
        op = _op("schwefel", d)
        f = _f(op, np.full(d, 420.9687))[0]
        assert abs(f) < 1e-4 * d
        assert _f(op, np.zeros(d))[0] == pytest.approx(-418.9829 * d, abs=1e-9)
    # brute force in one dimension over the whole box
    op = _op("schwefel", 1)
    t = np.linspace(-500, 500, 1_000_001)
    assert abs(t[np.argmax(_f(op, t[:, None]))] - 420.97) < 0.01


def test_styblinski_tang_optimum():
    # the stationary points solve 4 t^3 - 32 t + 5 = 0; the maximum of the
    # negated function sits at the smallest root (numpy's companion-matrix
    # root finder, independent of the oracle)
    r = np.sort(np.roots([4.0, 0.0, -32.0, 5.0]).real)[0]
    for d in (1, 5, 64):
        op = _op("styblinski_tang", d)
        f, g = op.eval(np.full((1, d), r))
        assert np.max(np.abs(g)) < 1e-12
        assert f[0] == pytest.approx(39.16616570377142 * d, rel=1e-12)
    op = _op("styblinski_tang", 1)
    t = np.linspace(-5, 5, 1_000_001)
    assert abs(t[np.argmax(_f(op, t[:, None]))] - r) < 2e-5


def test_michalewicz_exact_point_and_coordinate_index():
    # at x_i = pi/2: sin x_i = 1 and sin(i pi / 4)^20 = 2^-10, 1, 2^-10, 0, ...
    op = _op("michalewicz", 4)
    assert _f(op, np.full(4, np.pi / 2))[0] == pytest.approx(1.0 + 2.0 ** -9, abs=1e-14)
    op8 = _op("michalewicz", 8)
    assert _f(op8, np.full(8, np.pi / 2))[0] == pytest.approx(2.0 * (1.0 + 2.0 ** -9), abs=1e-14)
    # the index i enters: swapping two coordinates changes the value
    x = np.array([[2.2, 1.57]])
    assert _f(_op("michalewicz", 2), x)[0] != pytest.approx(_f(_op("michalewicz", 2), x[:, ::-1])[0], abs=1e-3)
    # separable: the 2-d maximum on a grid is the sum of per-coordinate maxima
    t = np.linspace(0, np.pi, 2001)
    T1, T2 = np.meshgrid(t, t, indexing="ij")
    f2 = _f(_op("michalewicz", 2), np.stack([T1.ravel(), T2.ravel()], 1)).max()
    per = [np.max(np.sin(t) * np.sin((i + 1) * t ** 2 / np.pi) ** 20) for i in range(2)]
    assert f2 == pytest.approx(sum(per), abs=1e-12)
    assert 1.80 < f2 < 1.81


@pytest.mark.parametrize("d", [2, 3, 6, 10, 64])
def test_trid_optimum_stated_in_the_paper(d):
    op = _op("trid", d)
    i = np.arange(1, d + 1, dtype=float)
    xs = i * (d + 1 - i)
    f, g = op.eval(xs[None, :])
    assert f[0] == pytest.approx(d * (d + 4) * (d - 1) / 6.0, rel=1e-13)
    assert np.max(np.abs(g)) < 1e-9
    dx = np.random.default_rng(d).normal(size=(16, d))
    assert np.all(_f(op, xs + dx) < f[0])


def test_bukin6_optimum_and_ridge():
    op = _op("bukin6", 2)
    assert _f(op, np.array([-10.0, 1.0]))[0] == 0.0
    X = np.random.default_rng(2).uniform([-15, -3], [-5, 3], size=(256, 2))
    assert np.all(_f(op, X) < 0.0)
    # on the ridge y = 0.01 x^2 only the linear term remains
    xr = np.array([[-12.0, 1.44], [-6.0, 0.36]])
    np.testing.assert_allclose(_f(op, xr), [-0.02, -0.04], rtol=0, atol=1e-12)


@pytest.mark.parametrize("name,opt", [("rastrigin", 0.0), ("ackley", 0.0), ("styblinski_tang", -2.903534)])
def test_two_dimensional_grid_maximum(name, opt):
    op = _op(name, 2)
    lo, hi = W.closed_form_box(W.CLOSED_FORMS[name], 2)
    t = np.linspace(lo[0], hi[0], 1025)
    T1, T2 = np.meshgrid(t, t, indexing="ij")
    X = np.stack([T1.ravel(), T2.ravel()], 1)
    best = X[np.argmax(_f(op, X))]
    step = t[1] - t[0]
    assert np.all(np.abs(best - opt) <= step)


# --------------------------------------------------------------------------
# gradients
# --------------------------------------------------------------------------

@pytest.mark.parametrize("name", FAMS)
def test_gradient_matches_numerical_derivative(name):
    d = 2 if name == "bukin6" else 9
    op = _op(name, d)
    lo, hi = W.closed_form_box(W.CLOSED_FORMS[name], d)
    rng = np.random.default_rng(11)
    for _ in range(6):
        x = rng.uniform(lo.astype(float), hi.astype(float))
        if name == "bukin6":
            x[1] = 0.01 * x[0] ** 2 + rng.choice([-1, 1]) * rng.uniform(0.5, 2.0)  # off the ridge
        h = 1e-4 * max(1.0, float(np.max(np.abs(x))))
        g = op.eval(x[None, :])[1][0]
        gn = _num_grad(op, x, h)
        scale = max(1.0, float(np.max(np.abs(g))))
        assert np.max(np.abs(g - gn)) < 1e-6 * scale, (name, x, g, gn)


@pytest.mark.parametrize("name", FAMS)
def test_oracle_fd_gradient_approaches_the_analytic_one(name):
    d = 2 if name == "bukin6" else 5
    op = _op(name, d)
    lo, hi = W.closed_form_box(W.CLOSED_FORMS[name], d)
    rng = np.random.default_rng(5)
    X = rng.uniform(lo.astype(float), hi.astype(float), size=(8, d))
    if name == "bukin6":
        X[:, 1] = 0.01 * X[:, 0] ** 2 + 1.0
    g = op.eval(X)[1]
    gfd = op.fd_grad(X, fd_h=1e-6)
    np.testing.assert_allclose(gfd, g, rtol=1e-5, atol=1e-5 * max(1.0, np.abs(g).max()))
