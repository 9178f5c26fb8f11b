"""Problem instances and starting populations for the five benchmark workloads.

Every array is drawn from ``numpy.random.default_rng(seed)`` and rounded to
float32 once; both the FP64 oracle and the FP32 GPU library receive exactly
these values.  The mixture components follow the paper's Gaussian-mixture test
function (Appendix D) extended to anisotropic components: covariance
``Q diag(lam) Q^T`` with a Haar-random rotation ``Q`` (QR of a Gaussian matrix
with the signs of ``diag(R)`` folded into ``Q``, Mezzadri 2007) and ``lam``
log-uniform.  Problems are handed over as log weights, centres and precision
matrices ``Q diag(1/lam) Q^T``; the box domain is ``[-1.2 a, 1.2 a]^d`` for
centres drawn in ``[-a, a]^d``.
"""
from __future__ import annotations

from dataclasses import dataclass, replace
from typing import List

import numpy as np

GAUSS = 0
STUDENT_T = 1
# closed-form test functions (Appendix D)
RASTRIGIN = 2
ACKLEY = 3
SCHWEFEL = 4
STYBLINSKI_TANG = 5
MICHALEWICZ = 6
TRID = 7
BUKIN6 = 8
CLOSED_FORMS = {"rastrigin": RASTRIGIN, "ackley": ACKLEY, "schwefel": SCHWEFEL,
                "styblinski_tang": STYBLINSKI_TANG, "michalewicz": MICHALEWICZ, "trid": TRID, "bukin6": BUKIN6}


@dataclass
class Problem:
    family: int
    d: int
    K: int
    log_w: np.ndarray  # (K,) float32
    mu: np.ndarray  # (K, d) float32
    prec: np.ndarray  # (K, d, d) float32, symmetric positive definite
    lo: np.ndarray  # (d,) float32
    hi: np.ndarray  # (d,) float32
    nu: float = 0.0
    noise_sigma: float = 0.0
    # the covariance factors the instance was drawn from (diagnostics only)
    lam: np.ndarray | None = None


@dataclass
class RunConfig:
    N: int
    m: int = 10
    n_osc: int = 3
    n_conv: int = 10
    n_anti: int = 5
    n_cloud: int = 3
    M: int = 10
    eps_grad: float = 1e-6
    eps_dup: float = 1e-3
    log_delta: float = float(np.log(0.1))
    momentum: float = 0.9
    alpha: float = 0.0  # <= 0: chosen from the scale estimate
    sigma: float = 0.0  # <= 0: c * pooled std of the unfrozen samples
    sigma_c: float = 0.1
    grad_mode: int = 1  # 0 central differences, 1 analytic (adjoint)
    fd_h: float = 0.0  # > 0 fixed step; <= 0 relative rule
    ls_c1: float = 1e-4
    ls_max: int = 10
    curv_eps: float = 1e-10
    gate_reps: int = 0
    phase_mask: int = 0x7E
    seed: int = 0
    problem_id: int = 0
    flags: int = 0  # bit 0: run cycles without graph replay

    def with_(self, **kw) -> "RunConfig":
        return replace(self, **kw)


def _haar(rng: np.random.Generator, d: int) -> np.ndarray:
    a = rng.standard_normal((d, d))
    q, r = np.linalg.qr(a)
    return q * np.sign(np.diag(r))[None, :]


def mixture_problem(
    seed: int,
    d: int,
    K: int,
    mean_range: float,
    lam_range=(1.0, 1.0),
    isotropic_var: float | None = None,
    dirichlet: float | None = 5.0,
    family: int = GAUSS,
    nu: float = 0.0,
    noise_sigma: float = 0.0,
    box_scale: float = 1.2,
) -> Problem:
    """Draw one mixture instance.

    ``isotropic_var`` gives every component covariance ``var * I`` (the paper's
    Appendix D form); otherwise covariances are ``Q diag(lam) Q^T`` with
    ``lam`` log-uniform in ``lam_range``.  ``dirichlet=None`` gives equal weights.
    """
    rng = np.random.default_rng(seed)
    mu = rng.uniform(-mean_range, mean_range, size=(K, d))
    prec = np.empty((K, d, d))
    lam_all = np.empty((K, d))
    for k in range(K):
        if isotropic_var is not None:
            lam = np.full(d, isotropic_var)
            q = np.eye(d)
        else:
            lo, hi = np.log(lam_range[0]), np.log(lam_range[1])
            lam = np.exp(rng.uniform(lo, hi, size=d))
            q = _haar(rng, d)
        p = (q / lam[None, :]) @ q.T
        prec[k] = 0.5 * (p + p.T)
        lam_all[k] = lam
    if dirichlet is None:
        w = np.full(K, 1.0 / K)
    else:
        w = rng.dirichlet(np.full(K, dirichlet))
    a = box_scale * mean_range
    prob = Problem(
        family=family,
        d=d,
        K=K,
        log_w=np.log(w).astype(np.float32),
        mu=mu.astype(np.float32),
        prec=prec.astype(np.float32),
        lo=np.full(d, -a, dtype=np.float32),
        hi=np.full(d, a, dtype=np.float32),
        nu=float(nu),
        noise_sigma=float(noise_sigma),
        lam=lam_all,
    )
    # float32 rounding keeps the matrices symmetric (elementwise rounding of a
    # symmetric array); make sure nothing upstream broke that.
    assert np.array_equal(prob.prec, np.transpose(prob.prec, (0, 2, 1)))
    return prob


def closed_form_box(family: int, d: int):
    """The search domain Appendix D gives for each closed-form function."""
    if family == RASTRIGIN:
        lo, hi = np.full(d, -5.12), np.full(d, 5.12)
    elif family == ACKLEY:
        lo, hi = np.full(d, -32.768), np.full(d, 32.768)
    elif family == SCHWEFEL:
        lo, hi = np.full(d, -500.0), np.full(d, 500.0)
    elif family == STYBLINSKI_TANG:
        lo, hi = np.full(d, -5.0), np.full(d, 5.0)
    elif family == MICHALEWICZ:
        lo, hi = np.zeros(d), np.full(d, np.pi)
    elif family == TRID:
        lo, hi = np.full(d, -float(d * d)), np.full(d, float(d * d))
    elif family == BUKIN6:
        if d != 2:
            raise ValueError("Bukin N.6 is two-dimensional")
        lo, hi = np.array([-15.0, -3.0]), np.array([-5.0, 3.0])
    else:
        raise ValueError(f"not a closed-form family: {family}")
    return lo.astype(np.float32), hi.astype(np.float32)


def closed_form_problem(name_or_family, d: int, noise_sigma: float = 0.0) -> Problem:
    """One of the closed-form test functions on its Appendix D domain."""
    fam = CLOSED_FORMS[name_or_family] if isinstance(name_or_family, str) else int(name_or_family)
    lo, hi = closed_form_box(fam, d)
    empty = np.zeros(0, np.float32)
    return Problem(family=fam, d=d, K=0, log_w=empty, mu=empty.reshape(0, d), prec=empty.reshape(0, d, d),
                   lo=lo, hi=hi, noise_sigma=float(noise_sigma))


def two_peak_problem(noise_sigma: float, d: int = 6, sep: float = 2.0, box: float = 6.0) -> Problem:
    """Two equal isotropic unit-variance Gaussians at +-sep e_1 (the noise
    experiment of Sec. 5.7: d = 6, peaks at +-2 e_1, four standard deviations
    apart)."""
    mu = np.zeros((2, d))
    mu[0, 0], mu[1, 0] = sep, -sep
    prec = np.broadcast_to(np.eye(d), (2, d, d)).copy()
    return Problem(family=GAUSS, d=d, K=2, log_w=np.log(np.full(2, 0.5)).astype(np.float32),
                   mu=mu.astype(np.float32), prec=prec.astype(np.float32),
                   lo=np.full(d, -box, np.float32), hi=np.full(d, box, np.float32),
                   noise_sigma=float(noise_sigma), lam=np.ones((2, d)))


def uniform_population(seed: int, N: int, lo: np.ndarray, hi: np.ndarray) -> np.ndarray:
    rng = np.random.default_rng(seed + 7919)
    x = rng.uniform(lo.astype(np.float64), hi.astype(np.float64), size=(N, lo.shape[0]))
    return np.clip(x.astype(np.float32), lo, hi)


# --------------------------------------------------------------------------
# The benchmark workloads.  Each returns (problem, config, x0).
# --------------------------------------------------------------------------

def gauss4_d2(N: int = 256):
    """d=2, four isotropic components of standard deviation 0.5, equal weights,
    centres in [-5,5]^2, population in [-6,6]^2; FP64 finite differences h=1e-5,
    m=5, 50 cycles."""
    p = mixture_problem(0, 2, 4, 5.0, isotropic_var=0.25, dirichlet=None)
    c = RunConfig(N=N, m=5, n_osc=50, n_conv=10, n_anti=5, n_cloud=3, M=10, eps_grad=1e-6,
                  grad_mode=0, fd_h=1e-5, seed=0)
    return p, c, uniform_population(0, N, p.lo, p.hi)


def gauss32_d16(N: int = 16384, n_osc: int = 200):
    """d=16, 32 anisotropic components (lam in [0.1,1]), centres in [-10,10]^16,
    Dirichlet(5) weights; central differences, m=8, 200 cycles."""
    p = mixture_problem(1, 16, 32, 10.0, lam_range=(0.1, 1.0))
    c = RunConfig(N=N, m=8, n_osc=n_osc, n_conv=12, M=10, eps_grad=1e-3, grad_mode=0, seed=1)
    return p, c, uniform_population(1, N, p.lo, p.hi)


def gauss128_d64(N: int = 65536, n_osc: int = 300, grad_mode: int = 1):
    """d=64, 128 anisotropic components (lam in [0.05,1]), centres in
    [-20,20]^64; m=10, 300 cycles, n_conv=18, M=16 probes at sigma=0.1."""
    p = mixture_problem(2, 64, 128, 20.0, lam_range=(0.05, 1.0))
    c = RunConfig(N=N, m=10, n_osc=n_osc, n_conv=18, M=16, sigma=0.1, eps_grad=1e-3,
                  grad_mode=grad_mode, seed=2)
    return p, c, uniform_population(2, N, p.lo, p.hi)


def batch64(n_problems: int = 64, seed: int = 3):
    """64 independent problems: d in {2,4,8,16,32,64}, K in 4..64, N in
    1024..16384, generated like gauss32_d16; m=8, 50 cycles."""
    rng = np.random.default_rng(seed)
    out: List = []
    for pid in range(n_problems):
        d = int(rng.choice([2, 4, 8, 16, 32, 64]))
        K = int(rng.integers(4, 65))
        N = int(rng.integers(1024, 16385))
        p = mixture_problem(1000 + pid, d, K, 10.0, lam_range=(0.1, 1.0))
        n_conv = max(10, int(np.ceil(3 * np.log2(d))))
        c = RunConfig(N=N, m=8, n_osc=50, n_conv=n_conv, M=10, eps_grad=1e-3, grad_mode=1,
                      seed=3, problem_id=pid)
        out.append((p, c, uniform_population(1000 + pid, N, p.lo, p.hi)))
    return out


def student48_d32(N: int = 131072, n_osc: int = 400):
    """d=32, 48 Student-t components (nu=3), lam in [0.05,1], centres in
    [-20,20]^32, unit additive noise per evaluation; M=32 probes at sigma=0.2,
    m=10, 400 cycles, n_conv=15."""
    p = mixture_problem(4, 32, 48, 20.0, lam_range=(0.05, 1.0), family=STUDENT_T, nu=3.0,
                        noise_sigma=1.0)
    c = RunConfig(N=N, m=10, n_osc=n_osc, n_conv=15, M=32, sigma=0.2, eps_grad=1e-3,
                  grad_mode=1, gate_reps=32, seed=4)
    return p, c, uniform_population(4, N, p.lo, p.hi)
