"""The allocation-free evaluation entry point (chisao_eval_static) against
chisao_eval on a handle created for the same problem: values and gradients
must be bitwise equal (the same kernels on the same tables), call after call,
with the static device array reused by problems of different sizes."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _cases():
    # (name, problem, batch): each call reuses the array the previous one filled
    return [
        ("gauss d=64 K=128", W.mixture_problem(2, 64, 128, 20.0, lam_range=(0.05, 1.0)), 2000),
        ("student-t d=32 K=48", W.mixture_problem(4, 32, 48, 20.0, lam_range=(0.05, 1.0), family=W.STUDENT_T,
                                                  nu=3.0), 700),
        ("gauss d=5 K=3", W.mixture_problem(9, 5, 3, 4.0, lam_range=(0.3, 1.0)), 333),
        ("rastrigin d=7", W.closed_form_problem("rastrigin", 7), 100),
    ]


def _points(prob, B, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(prob.lo, prob.hi, size=(B, prob.d)).astype(np.float32)


def _handle_eval(prob, X, grad_mode, fd_h):
    import torch

    from paper_2606_26164_amd.api import Optimizer

    cfg = W.RunConfig(N=64, grad_mode=grad_mode, fd_h=fd_h, eps_grad=1e-3, seed=1)
    x0 = W.uniform_population(1, 64, prob.lo, prob.hi)
    with Optimizer(prob, cfg, x0) as opt:
        f, G = opt.eval(torch.from_numpy(X).cuda(), grad_mode=grad_mode)
        torch.cuda.synchronize()
        return f.cpu().numpy(), G.cpu().numpy()


@pytest.mark.parametrize("grad_mode,fd_h", [(1, 0.0), (0, 0.0), (0, 1e-2)])
def test_static_eval_equals_handle_eval_call_after_call(grad_mode, fd_h):
    import torch

    from paper_2606_26164_amd.api import eval_static

    cases = _cases()
    want = []
    for i, (name, prob, B) in enumerate(cases):
        X = _points(prob, B, 100 + i)
        want.append((X,) + _handle_eval(prob, X, grad_mode, fd_h))
    # consecutive calls, each smaller than the one before, then the first again
    for i in list(range(len(cases))) + [0]:
        name, prob, B = cases[i]
        X, f_want, G_want = want[i]
        f, G = eval_static(prob, torch.from_numpy(X).cuda(), grad_mode=grad_mode, fd_h=fd_h)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(f.cpu().numpy(), f_want, err_msg=f"{name}: values")
        np.testing.assert_array_equal(G.cpu().numpy(), G_want, err_msg=f"{name}: gradients")
        assert np.all(np.isfinite(f_want)) and np.all(np.isfinite(G_want))


def test_static_eval_rejects_tables_beyond_the_static_array():
    import torch

    from paper_2606_26164_amd import _lib as L
    from paper_2606_26164_amd.api import eval_static

    prob = W.mixture_problem(5, 64, 260, 5.0, isotropic_var=1.0)
    X = torch.zeros(8, 64, device="cuda")
    with pytest.raises(L.ChisaoError) as ei:
        eval_static(prob, X)
    assert ei.value.code == L.E_RANGE and "static scratch" in str(ei.value)
    # the largest problem that fits at d = 64 still runs
    ok = W.mixture_problem(5, 64, 251, 5.0, isotropic_var=1.0)
    f, G = eval_static(ok, X)
    torch.cuda.synchronize()
    assert torch.isfinite(f).all() and torch.isfinite(G).all()


def test_static_eval_rejects_a_matrix_that_is_not_positive_definite():
    import torch

    from paper_2606_26164_amd import _lib as L
    from paper_2606_26164_amd.api import eval_static

    prob = W.mixture_problem(6, 4, 2, 3.0, isotropic_var=1.0)
    prob.prec = prob.prec.copy()
    prob.prec[1] = -prob.prec[1]
    with pytest.raises(L.ChisaoError) as ei:
        eval_static(prob, torch.zeros(4, 4, device="cuda"))
    assert ei.value.code == L.E_INVAL
