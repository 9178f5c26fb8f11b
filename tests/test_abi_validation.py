"""Argument validation of the C ABI, on the host: every call below is
rejected before the library touches a device, so these run without a GPU.
Each case checks the return code and that the last-error message names what
was wrong."""
import ctypes as C

import numpy as np
import pytest

import workloads as W
from paper_2606_26164_amd import _lib as L
from paper_2606_26164_amd.api import _Spec


def _lib():
    return L.load()


def _err():
    return _lib().chisao_last_error().decode()


def _init(items, n_problems=None, patch=None):
    """chisao_init_batched on (problem, config) pairs; returns (rc, handle).
    patch(struct) edits the first problem's struct (fields that the host
    arrays' shapes cannot express, such as d = 0)."""
    specs = [_Spec(p, c) for p, c in items]
    if patch:
        patch(specs[0].cp)
    n = len(specs) if n_problems is None else n_problems
    probs = (L.Problem * max(1, len(specs)))(*[s.cp for s in specs])
    cfgs = (L.Config * max(1, len(specs)))(*[s.cc for s in specs])
    h = C.c_void_p(1)
    rc = _lib().chisao_init_batched(C.byref(h), n, probs, cfgs, None, None)
    return rc, h


def _base(d=4, K=3, family=W.GAUSS):
    p = W.mixture_problem(3, d, K, 2.0, lam_range=(0.5, 1.0), family=family, nu=3.0)
    c = W.RunConfig(N=64, eps_grad=1e-3, seed=1)
    return p, c


def _copy(p, **kw):
    q = type(p).__new__(type(p))
    q.__dict__.update({k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in p.__dict__.items()})
    for k, v in kw.items():
        setattr(q, k, v)
    return q


def _bad_problem(kind):
    p, c = _base()
    if kind == "family":
        return p, c, "unknown family", lambda s: setattr(s, "family", 42)
    if kind == "d0":
        return p, c, "d must be in 1..64", lambda s: setattr(s, "d", 0)
    if kind == "K0":
        return p, c, "K must be in 1..65536", lambda s: setattr(s, "K", 0)
    if kind == "box":
        lo = p.lo.copy()
        lo[2] = p.hi[2]
        return _copy(p, lo=lo), c, "lo < hi", None
    if kind == "mu":
        mu = p.mu.copy()
        mu[1, 0] = np.nan
        return _copy(p, mu=mu), c, "non-finite centre 1", None
    if kind == "weight":
        lw = p.log_w.copy()
        lw[2] = np.inf
        return _copy(p, log_w=lw), c, "non-finite log weight 2", None
    if kind == "asym":
        prec = p.prec.copy()
        prec[0, 0, 1] += 0.25
        return _copy(p, prec=prec), c, "not symmetric", None
    if kind == "nu":
        q, c = _base(family=W.STUDENT_T)
        return _copy(q, nu=0.0), c, "nu > 0", None
    if kind == "noise":
        return _copy(p, noise_sigma=-1.0), c, "noise_sigma", None
    raise KeyError(kind)


@pytest.mark.parametrize("kind", ["family", "d0", "K0", "box", "mu", "weight", "asym", "nu", "noise"])
def test_bad_problem_is_rejected(kind):
    p, c, msg, patch = _bad_problem(kind)
    rc, h = _init([(p, c)], patch=patch)
    assert rc == L.E_INVAL
    assert h.value is None  # the output handle is cleared
    assert msg in _err()


def test_component_count_above_65536_is_rejected():
    p, c = _base(d=2, K=1)
    k = 65537
    big = W.Problem(family=W.GAUSS, d=2, K=k, log_w=np.zeros(k, np.float32), mu=np.zeros((k, 2), np.float32),
                    prec=np.broadcast_to(np.eye(2, dtype=np.float32), (k, 2, 2)).copy(), lo=p.lo, hi=p.hi)
    rc, _ = _init([(big, c)])
    assert rc == L.E_INVAL and "1..65536" in _err()


def test_dimension_above_64_is_rejected():
    p, c = _base(d=65, K=1)
    rc, _ = _init([(p, c)])
    assert rc == L.E_INVAL and "1..64" in _err()


def test_bukin_needs_d2():
    p2 = W.closed_form_problem(W.BUKIN6, 2)
    p = W.Problem(family=W.BUKIN6, d=3, K=0, log_w=p2.log_w, mu=np.zeros((0, 3), np.float32),
                  prec=np.zeros((0, 3, 3), np.float32), lo=np.full(3, -5.0, np.float32),
                  hi=np.full(3, 5.0, np.float32))
    c = W.RunConfig(N=16, grad_mode=0, eps_grad=1e-2)
    rc, _ = _init([(p, c)])
    assert rc == L.E_INVAL and "Bukin" in _err()


@pytest.mark.parametrize("field,value,msg", [
    ("N", 0, "N must be"),
    ("m", 0, "m must be"),
    ("m", 33, "m must be"),
    ("M", 0, "M must be"),
    ("M", 33, "M must be"),
    ("n_osc", 0, "n_osc"),
    ("n_anti", -1, "negative step count"),
    ("n_conv", 256, "at most 255"),
    ("n_cloud", 256, "at most 255"),
    ("ls_max", 0, "ls_max"),
    ("ls_max", 16, "ls_max"),
    ("grad_mode", 2, "grad_mode"),
    ("gate_reps", -1, "gate_reps"),
    ("eps_grad", 0.0, "eps_grad"),
    ("eps_dup", -1.0, "eps_dup"),
    ("momentum", float("nan"), "non-finite hyperparameter"),
    ("sigma", float("inf"), "non-finite hyperparameter"),
])
def test_bad_config_is_rejected(field, value, msg):
    p, c = _base()
    rc, _ = _init([(p, c.with_(**{field: value}))])
    assert rc == L.E_INVAL
    assert msg in _err()


def test_population_beyond_32_bit_indexing_is_rejected():
    p, c = _base(d=64, K=1)
    rc, _ = _init([(p, c.with_(N=1 << 30, m=32))])
    assert rc == L.E_INVAL and "32-bit" in _err()


def test_batch_shape_checks():
    p, c = _base()
    rc, _ = _init([(p, c)], n_problems=0)
    assert rc == L.E_INVAL and "n_problems" in _err()
    rc, _ = _init([(p, c), (p, c.with_(n_osc=c.n_osc + 1))])
    assert rc == L.E_INVAL and "same n_osc" in _err()
    # the problem index is reported
    q, _, _, _ = _bad_problem("mu")
    rc, _ = _init([(p, c), (p, c), (q, c)])
    assert rc == L.E_INVAL and "problem 2" in _err()


def test_null_arguments():
    lib = _lib()
    p, c = _base()
    sp = _Spec(p, c)
    assert lib.chisao_init_batched(None, 1, C.byref(sp.cp), C.byref(sp.cc), None, None) == L.E_INVAL
    h = C.c_void_p()
    assert lib.chisao_init_batched(C.byref(h), 1, None, C.byref(sp.cc), None, None) == L.E_INVAL
    assert lib.chisao_cycle(None, 1, None) == L.E_INVAL
    n = C.c_int(-7)
    assert lib.chisao_modes(None, 0, None, None, 0, C.byref(n)) == L.E_INVAL
    assert lib.chisao_tuning(None, None, 0, C.byref(n)) == L.E_INVAL
    lib.chisao_destroy(None)  # a no-op


def test_eval_static_limits():
    """The allocation-free evaluation checks its table size against the static
    array before any device work: K = 300 components at d = 64 need more than
    8 MiB of tables; an empty batch of a problem that fits is a no-op."""
    lib = _lib()
    big = W.mixture_problem(5, 64, 300, 2.0, lam_range=(0.5, 1.0))
    sp = _Spec(big, W.RunConfig(N=1))
    assert lib.chisao_eval_static(C.byref(sp.cp), 0.0, None, 0, None, None, L.GRAD_ADJOINT, None) == L.E_RANGE
    assert "static scratch" in _err() and "K = 300" in _err()
    small = _Spec(*_base())
    assert lib.chisao_eval_static(C.byref(small.cp), 0.0, None, -1, None, None, L.GRAD_ADJOINT, None) == L.E_INVAL
    assert lib.chisao_eval_static(C.byref(small.cp), 0.0, None, 0, None, None, 5, None) == L.E_INVAL
    assert lib.chisao_eval_static(C.byref(small.cp), float("nan"), None, 0, None, None, L.GRAD_FD, None) == L.E_INVAL
    assert lib.chisao_eval_static(C.byref(small.cp), 0.0, None, 0, None, None, L.GRAD_ADJOINT, None) == L.OK
