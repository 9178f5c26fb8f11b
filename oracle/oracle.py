"""ctypes binding of the FP64 CPU oracle (``chisao_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the product library.  Inputs are the
float32 arrays of ``workloads`` widened to float64.
"""
from __future__ import annotations

import contextlib
import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "chisao_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

TR_NONE = 0xFF
TR_LS_MASK = 0x0F
TR_LS_FAIL = 0x0F
TR_STORED = 0x10
TR_CONV = 0x20
TR_RESET = 0x40
# objective families from 2 on are the closed-form test functions of Appendix D
CLOSED_FORM_FIRST = 2


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", "-o", tmp, SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


class _Problem(C.Structure):
    _fields_ = [("family", C.c_int32), ("d", C.c_int32), ("K", C.c_int32), ("nu", C.c_double),
                ("log_w", C.c_void_p), ("mu", C.c_void_p), ("prec", C.c_void_p), ("lo", C.c_void_p),
                ("hi", C.c_void_p), ("noise_sigma", C.c_double)]


class _Config(C.Structure):
    _fields_ = [("N", C.c_int32), ("m", C.c_int32), ("n_osc", C.c_int32), ("n_conv", C.c_int32),
                ("n_anti", C.c_int32), ("n_cloud", C.c_int32), ("M", C.c_int32),
                ("eps_grad", C.c_double), ("eps_dup", C.c_double), ("log_delta", C.c_double),
                ("momentum", C.c_double), ("alpha", C.c_double), ("sigma", C.c_double),
                ("sigma_c", C.c_double), ("grad_mode", C.c_int32), ("fd_h", C.c_double),
                ("ls_c1", C.c_double), ("ls_max", C.c_int32), ("curv_eps", C.c_double),
                ("gate_reps", C.c_int32), ("phase_mask", C.c_uint32), ("seed", C.c_uint64),
                ("problem_id", C.c_uint32), ("flags", C.c_uint32)]


class _State(C.Structure):
    _fields_ = [("X", C.c_void_p), ("F", C.c_void_p), ("G", C.c_void_p), ("V", C.c_void_p),
                ("stuck", C.c_void_p), ("active", C.c_void_p), ("conv", C.c_void_p), ("removed", C.c_void_p),
                ("S", C.c_void_p), ("Y", C.c_void_p), ("rho", C.c_void_p), ("head", C.c_void_p),
                ("cnt", C.c_void_p), ("k", C.c_int32), ("gr_disabled", C.c_int32), ("gr_fail", C.c_int32),
                ("gr_used_last", C.c_int32), ("gr_prev_modes", C.c_int32), ("f_max", C.c_double),
                ("sigma", C.c_double), ("alpha_c", C.c_double), ("alpha_a", C.c_double),
                ("K_lost", C.c_int32), ("n_stuck", C.c_int32), ("n_modes", C.c_int32),
                ("reseed_kind", C.c_int32), ("n_free", C.c_int32), ("n_unfrozen", C.c_int32),
                ("Fg", C.c_void_p), ("W", C.c_void_p), ("wvalid", C.c_void_p), ("n_nonfinite", C.c_int32)]


class _Replay(C.Structure):
    _fields_ = [("trace_out", C.c_void_p), ("trace_in", C.c_void_p), ("stuck_in", C.c_void_p),
                ("removed_in", C.c_void_p), ("tol_f", C.c_double), ("tol_g", C.c_double),
                ("tol_curv", C.c_double), ("tol_dist", C.c_double), ("n_decisions", C.c_int64),
                ("n_borderline", C.c_int64), ("n_hard", C.c_int64), ("worst_hard", C.c_double),
                ("first_hard_sample", C.c_int32), ("first_hard_iter", C.c_int32),
                ("first_hard_kind", C.c_int32), ("border_by_kind", C.c_int64 * 8), ("hard_by_kind", C.c_int64 * 8)]


_lib = None


def _bind(L):
    """Declare the argument types of the exported functions on a loaded build."""
    P = C.POINTER
    L.orc_philox4x32_10.argtypes = [P(C.c_uint32), P(C.c_uint32), P(C.c_uint32)]
    L.orc_u01.argtypes = [C.c_uint32]
    L.orc_u01.restype = C.c_double
    L.orc_prepare.argtypes = [P(_Problem), C.c_void_p]
    L.orc_eval_batch.argtypes = [P(_Problem), C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]
    L.orc_fd_grad_batch.argtypes = [P(_Problem), C.c_void_p, C.c_double, C.c_int, C.c_void_p, C.c_void_p]
    L.orc_two_loop.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                               C.c_void_p, C.c_void_p, C.c_void_p]
    L.orc_householder_q.argtypes = [C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]
    for name in ("orc_phase_converge", "orc_cycle"):
        getattr(L, name).argtypes = [P(_Problem), C.c_void_p, P(_Config), P(_State), P(_Replay)]
    L.orc_lbfgs_iterate.argtypes = [P(_Problem), C.c_void_p, P(_Config), P(_State), C.c_int, C.c_int,
                                    P(_Replay)]
    L.orc_phase_stick.argtypes = [P(_Problem), C.c_void_p, P(_Config), P(_State), P(_Replay)]
    L.orc_phase_dedup.argtypes = [P(_Problem), P(_Config), P(_State), P(_Replay)]
    L.orc_phase_reseed.argtypes = [P(_Problem), P(_Config), P(_State)]
    L.orc_phase_hlc.argtypes = [P(_Problem), C.c_void_p, P(_Config), P(_State)]
    L.orc_phase_anti.argtypes = [P(_Problem), C.c_void_p, P(_Config), P(_State)]
    L.orc_init_population.argtypes = [P(_Problem), P(_Config), C.c_void_p]
    L.orc_num_threads.restype = C.c_int
    L.orc_set_num_threads.argtypes = [C.c_int]
    L.orc_set_num_threads.restype = C.c_int
    return L


def lib():
    global _lib
    if _lib is None:
        _lib = _bind(C.CDLL(build()))
    return _lib


@contextlib.contextmanager
def using_library(path: str):
    """Route every oracle call to another build of the oracle for the duration
    of the block.  Used by the mutation tests, which compile a copy of the
    source with one planted mistake and check that the pins catch it."""
    global _lib
    saved = _lib
    _lib = _bind(C.CDLL(os.path.abspath(path)))
    try:
        yield _lib
    finally:
        _lib = saved


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data


def philox4x32_10(ctr, key):
    L = lib()
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    L.orc_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> int:
    """Thread count of the oracle's per-sample loops (results do not depend on it)."""
    return int(lib().orc_set_num_threads(int(n)))


class OracleProblem:
    """A mixture problem in float64, with its per-component log constants."""

    def __init__(self, prob):
        self.d, self.K, self.family = prob.d, prob.K, prob.family
        if self.d > 512:
            raise ValueError("oracle supports d <= 512")
        if self.family >= CLOSED_FORM_FIRST:
            # closed-form test function: no mixture arrays
            self.K = 0
        self.log_w = np.ascontiguousarray(prob.log_w if self.K else np.zeros(0), dtype=np.float64)
        self.mu = np.ascontiguousarray(prob.mu if self.K else np.zeros(0), dtype=np.float64).reshape(self.K, self.d)
        self.prec = np.ascontiguousarray(prob.prec if self.K else np.zeros(0),
                                         dtype=np.float64).reshape(self.K, self.d, self.d)
        self.lo = np.ascontiguousarray(prob.lo, dtype=np.float64)
        self.hi = np.ascontiguousarray(prob.hi, dtype=np.float64)
        self.nu = float(prob.nu)
        self.noise_sigma = float(prob.noise_sigma)
        self.c = _Problem(self.family, self.d, self.K, self.nu, _ptr(self.log_w), _ptr(self.mu), _ptr(self.prec),
                          _ptr(self.lo), _ptr(self.hi), self.noise_sigma)
        self.logc = np.zeros(max(self.K, 1))
        rc = lib().orc_prepare(C.byref(self.c), _ptr(self.logc))
        if rc != 0:
            raise ValueError(f"orc_prepare failed ({rc}): precision matrix not positive definite?")

    def eval(self, X: np.ndarray, grad: bool = True):
        X = np.ascontiguousarray(X, dtype=np.float64).reshape(-1, self.d)
        n = X.shape[0]
        f = np.empty(n)
        G = np.empty((n, self.d)) if grad else None
        lib().orc_eval_batch(C.byref(self.c), _ptr(self.logc), n, _ptr(X), _ptr(f), _ptr(G))
        return (f, G) if grad else f

    def fd_grad(self, X: np.ndarray, fd_h: float = 0.0):
        X = np.ascontiguousarray(X, dtype=np.float64).reshape(-1, self.d)
        G = np.empty_like(X)
        lib().orc_fd_grad_batch(C.byref(self.c), _ptr(self.logc), float(fd_h), X.shape[0], _ptr(X), _ptr(G))
        return G


def conv_steps(cfg, d: int) -> int:
    """n_conv, with the Table 1 default max(10, 3 log2 d) when it is not given
    (3 log2 d rounded up)."""
    if cfg.n_conv > 0:
        return int(cfg.n_conv)
    return max(10, int(np.ceil(3.0 * np.log2(d) - 1e-9)))


def make_config(cfg, d: int) -> _Config:
    return _Config(cfg.N, cfg.m, cfg.n_osc, conv_steps(cfg, d), cfg.n_anti, cfg.n_cloud, cfg.M, cfg.eps_grad,
                   cfg.eps_dup, cfg.log_delta, cfg.momentum, cfg.alpha, cfg.sigma, cfg.sigma_c, cfg.grad_mode,
                   cfg.fd_h, cfg.ls_c1, cfg.ls_max, cfg.curv_eps, cfg.gate_reps, cfg.phase_mask, cfg.seed,
                   cfg.problem_id, int(getattr(cfg, "flags", 0)))


@dataclass
class ReplayReport:
    n_decisions: int
    n_borderline: int
    n_hard: int
    worst_hard: float
    first_hard_sample: int
    first_hard_iter: int
    first_hard_kind: int
    # indices: 1 line search, 2 curvature store, 3 convergence, 4 stick, 5 dedup
    border_by_kind: tuple = ()
    hard_by_kind: tuple = ()


class OracleRun:
    """Population state of one optimizer run, advanced a cycle or a phase at a time."""

    def __init__(self, prob, cfg, x0: np.ndarray | None = None):
        self.P = prob if isinstance(prob, OracleProblem) else OracleProblem(prob)
        self.cfg = cfg
        self.cc = make_config(cfg, self.P.d)
        N, d, m = cfg.N, self.P.d, cfg.m
        self.X = np.zeros((N, d))
        if x0 is None:
            lib().orc_init_population(C.byref(self.P.c), C.byref(self.cc), _ptr(self.X))
        else:
            self.X[:] = np.asarray(x0, dtype=np.float64).reshape(N, d)
        self.F = np.zeros(N)
        self.G = np.zeros((N, d))
        self.V = np.zeros((N, d))
        self.stuck = np.zeros(N, np.uint8)
        self.active = np.ones(N, np.uint8)
        self.conv = np.zeros(N, np.uint8)
        self.removed = np.zeros(N, np.uint8)
        self.S = np.zeros((N, m, d))
        self.Y = np.zeros((N, m, d))
        self.rho = np.zeros((N, m))
        self.head = np.full(N, m - 1, np.int32)
        self.cnt = np.zeros(N, np.int32)
        self.trace = np.full((self.cc.n_conv + 1, N), TR_NONE, np.uint8)
        self.Fg = np.zeros(N)
        self.W = np.zeros((N, d))
        self.wvalid = np.zeros(N, np.uint8)
        self.st = _State(_ptr(self.X), _ptr(self.F), _ptr(self.G), _ptr(self.V), _ptr(self.stuck),
                         _ptr(self.active), _ptr(self.conv), _ptr(self.removed), _ptr(self.S), _ptr(self.Y),
                         _ptr(self.rho), _ptr(self.head), _ptr(self.cnt), 0, 0, 0, 0, 0)
        self.st.Fg = _ptr(self.Fg)
        self.st.W = _ptr(self.W)
        self.st.wvalid = _ptr(self.wvalid)

    @property
    def k(self) -> int:
        return int(self.st.k)

    def _replay(self, trace_in=None, stuck_in=None, removed_in=None, tol_f=1e-4, tol_g=0.2, tol_curv=1e-2,
                tol_dist=1e-5):
        n_rows = int(self.cc.n_conv) + 1
        if self.trace.shape != (n_rows, self.cfg.N):  # the schedule may be changed between calls
            self.trace = np.full((n_rows, self.cfg.N), TR_NONE, np.uint8)
        if trace_in is not None and np.shape(trace_in) != self.trace.shape:
            raise ValueError("trace_in must have shape (n_conv+1, N)")
        for a in (stuck_in, removed_in):
            if a is not None and np.shape(a) != (self.cfg.N,):
                raise ValueError("decision arrays must have shape (N,)")
        self._keep = [np.ascontiguousarray(a, dtype=np.uint8) if a is not None else None
                      for a in (trace_in, stuck_in, removed_in)]
        return _Replay(_ptr(self.trace), _ptr(self._keep[0]), _ptr(self._keep[1]), _ptr(self._keep[2]), tol_f,
                       tol_g, tol_curv, tol_dist, 0, 0, 0, 0.0, -1, -1, 0)  # per-kind counters start at zero

    @staticmethod
    def _report(r: _Replay) -> ReplayReport:
        return ReplayReport(int(r.n_decisions), int(r.n_borderline), int(r.n_hard), float(r.worst_hard),
                            int(r.first_hard_sample), int(r.first_hard_iter), int(r.first_hard_kind),
                            tuple(int(v) for v in r.border_by_kind), tuple(int(v) for v in r.hard_by_kind))

    def _check(self, rc, what):
        if rc != 0:
            raise RuntimeError(f"oracle {what} failed with code {rc}")

    def cycle(self, **replay) -> ReplayReport:
        r = self._replay(**replay)
        self._check(lib().orc_cycle(C.byref(self.P.c), _ptr(self.P.logc), C.byref(self.cc), C.byref(self.st),
                                    C.byref(r)), "cycle")
        return self._report(r)

    def run(self, n_cycles: int | None = None):
        n = self.cfg.n_osc - self.k if n_cycles is None else n_cycles
        for _ in range(n):
            self.cycle()

    # individual phases (the cycle index used by the random streams is k+1)
    def phase_converge(self, **replay) -> ReplayReport:
        r = self._replay(**replay)
        self._check(lib().orc_phase_converge(C.byref(self.P.c), _ptr(self.P.logc), C.byref(self.cc),
                                             C.byref(self.st), C.byref(r)), "converge")
        return self._report(r)

    def iterate(self, first: int, n: int = 1, **replay) -> ReplayReport:
        """Continue Phase 1 (iterations first..first+n-1) from the current
        positions, gradients and histories, without releasing."""
        r = self._replay(**replay)
        self._check(lib().orc_lbfgs_iterate(C.byref(self.P.c), _ptr(self.P.logc), C.byref(self.cc),
                                            C.byref(self.st), int(first), int(n), C.byref(r)), "iterate")
        return self._report(r)

    def phase_stick(self, **replay) -> ReplayReport:
        r = self._replay(**replay)
        self._check(lib().orc_phase_stick(C.byref(self.P.c), _ptr(self.P.logc), C.byref(self.cc), C.byref(self.st),
                                          C.byref(r)),
                    "stick")
        return self._report(r)

    def phase_dedup(self, **replay) -> ReplayReport:
        r = self._replay(**replay)
        self._check(lib().orc_phase_dedup(C.byref(self.P.c), C.byref(self.cc), C.byref(self.st), C.byref(r)),
                    "dedup")
        return self._report(r)

    def phase_reseed(self):
        self._check(lib().orc_phase_reseed(C.byref(self.P.c), C.byref(self.cc), C.byref(self.st)), "reseed")

    def phase_hlc(self):
        self._check(lib().orc_phase_hlc(C.byref(self.P.c), _ptr(self.P.logc), C.byref(self.cc), C.byref(self.st)),
                    "hlc")

    def phase_anti(self):
        self._check(lib().orc_phase_anti(C.byref(self.P.c), _ptr(self.P.logc), C.byref(self.cc),
                                         C.byref(self.st)), "anti")

    def modes(self):
        """Stuck active samples, their values (gate values when noisy) and indices."""
        idx = np.nonzero(self.stuck & self.active)[0]
        fv = self.Fg if self.P.noise_sigma > 0 else self.F
        return self.X[idx].copy(), fv[idx].copy(), idx

    def mode_widths(self):
        """Preserved inverse-Hessian diagonals of the modes, in the order of modes()."""
        idx = np.nonzero(self.stuck & self.active)[0]
        return self.W[idx].copy()

    def stats(self) -> dict:
        s = self.st
        return dict(k=s.k, f_max=s.f_max, sigma=s.sigma, alpha_c=s.alpha_c, alpha_a=s.alpha_a, K_lost=s.K_lost,
                    n_stuck=s.n_stuck, n_modes=s.n_modes, reseed_kind=s.reseed_kind, n_free=s.n_free,
                    n_unfrozen=s.n_unfrozen, gr_disabled=s.gr_disabled, gr_fail=s.gr_fail,
                    n_nonfinite=s.n_nonfinite)


def two_loop(g, S, Y, rho, cnt, head):
    """Two-loop recursion on one sample's history (arrays of shape (m, d))."""
    m, d = S.shape
    S = np.ascontiguousarray(S, dtype=np.float64)
    Y = np.ascontiguousarray(Y, dtype=np.float64)
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    p = np.zeros(d)
    alpha = np.zeros(max(m, 1))
    lib().orc_two_loop(d, m, int(cnt), int(head), _ptr(S), _ptr(Y), _ptr(rho), _ptr(g), _ptr(p), _ptr(alpha))
    return p


def householder_q(A: np.ndarray):
    d = A.shape[0]
    A = np.ascontiguousarray(A, dtype=np.float64)
    Q = np.zeros((d, d))
    R = np.zeros((d, d))
    lib().orc_householder_q(d, _ptr(A), _ptr(Q), _ptr(R))
    return Q, R
