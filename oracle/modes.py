"""Reference mode set of a mixture log-density (FP64, CPU): damped Newton
ascent from every component centre with the analytic Hessian, kept when the
Hessian is negative definite (the second condition of the significant-mode
definition, eq. 1), deduplicated, and gated by f >= f_max + log(delta).

TEST INFRASTRUCTURE ONLY (test suite, smoke check): it is the reference the
optimizer's recovered modes are scored against.
"""
from __future__ import annotations

import numpy as np
from scipy.special import logsumexp


def _terms(prob, x):
    """log-weighted component terms, their gradients and Hessians at x."""
    d, K = prob.d, prob.K
    mu = prob.mu.astype(np.float64).reshape(K, d)
    P = prob.prec.astype(np.float64).reshape(K, d, d)
    lw = prob.log_w.astype(np.float64)
    _, logdet = np.linalg.slogdet(P)
    delta = x[None, :] - mu
    u = np.einsum("kij,kj->ki", P, delta)
    q = np.einsum("ki,ki->k", delta, u)
    if prob.family == 0:
        l = lw - 0.5 * d * np.log(2 * np.pi) + 0.5 * logdet - 0.5 * q
        gk = -u
        Hk = -P
    else:
        from scipy.special import gammaln

        nu = float(prob.nu)
        l = (lw + gammaln(0.5 * (nu + d)) - gammaln(0.5 * nu) - 0.5 * d * np.log(nu * np.pi) + 0.5 * logdet
             - 0.5 * (nu + d) * np.log1p(q / nu))
        w = (nu + d) / (nu + q)
        gk = -w[:, None] * u
        # d/dx of -w u = -w P + (2 w^2/(nu+d)) u u^T
        Hk = -w[:, None, None] * P + (2 * w ** 2 / (nu + d))[:, None, None] * np.einsum("ki,kj->kij", u, u)
    return l, gk, Hk


def value_grad_hess(prob, x):
    l, gk, Hk = _terms(prob, x)
    f = logsumexp(l)
    r = np.exp(l - f)
    g = r @ gk
    H = np.einsum("k,kij->ij", r, Hk + np.einsum("ki,kj->kij", gk, gk)) - np.outer(g, g)
    return f, g, H


def newton_modes(prob, log_delta=np.log(0.1), iters=60, tol=1e-10):
    """Local maxima reached from the component centres; with log_delta None
    the whole set, else those with f >= max f + log_delta."""
    d = prob.d
    lo, hi = prob.lo.astype(np.float64), prob.hi.astype(np.float64)
    found = []
    for k in range(prob.K):
        x = prob.mu[k].astype(np.float64).reshape(d).copy()
        f, g, H = value_grad_hess(prob, x)
        for _ in range(iters):
            try:
                step = -np.linalg.solve(H, g)
            except np.linalg.LinAlgError:
                break
            if not np.all(np.linalg.eigvalsh(0.5 * (H + H.T)) < 0):
                step = g / max(np.linalg.norm(g), 1.0)  # ascent step outside concave regions
            t = 1.0
            while t > 1e-12:
                xn = np.clip(x + t * step, lo, hi)
                fn, gn, Hn = value_grad_hess(prob, xn)
                if fn >= f - 1e-14 * abs(f):
                    break
                t *= 0.5
            x, f, g, H = xn, fn, gn, Hn
            if np.abs(g).max() < tol:
                break
        if np.abs(g).max() < 1e-7 and np.all(np.linalg.eigvalsh(0.5 * (H + H.T)) < 0):
            if not any(np.abs(x - y).max() < 1e-6 for y, _ in found):
                found.append((x, f))
    if not found:
        return np.zeros((0, d)), np.zeros(0)
    X = np.array([x for x, _ in found])
    F = np.array([f for _, f in found])
    if log_delta is None:  # every local maximum found, ungated
        return X, F
    keep = F >= F.max() + log_delta
    return X[keep], F[keep]
