"""Python face of libchisao: marshals arguments for the C ABI; all work runs in its kernels.

``Optimizer`` wraps one handle.  ``problem`` and ``config`` may be any objects
with the fields of ``chisao_problem`` / ``chisao_config`` (numpy arrays for the
problem arrays).  torch supplies device memory and the stream.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L


def _f32(a, shape):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32).reshape(shape))


@dataclass
class ModeSet:
    X: np.ndarray
    F: np.ndarray


def _problem_struct(problem):
    """A ``chisao_problem`` for ``problem`` and the host arrays it points to
    (which must stay alive while the struct is used)."""
    d, K = int(problem.d), int(problem.K)
    keep = dict(log_w=_f32(problem.log_w, (K,)), mu=_f32(problem.mu, (K, d)), prec=_f32(problem.prec, (K, d, d)),
                lo=_f32(problem.lo, (d,)), hi=_f32(problem.hi, (d,)))
    cp = L.Problem(int(problem.family), d, K, float(getattr(problem, "nu", 0.0)), keep["log_w"].ctypes.data,
                   keep["mu"].ctypes.data, keep["prec"].ctypes.data, keep["lo"].ctypes.data, keep["hi"].ctypes.data,
                   float(getattr(problem, "noise_sigma", 0.0)))
    return cp, keep


class _Spec:
    """Host copies of one problem's arrays, kept alive while the handle is created."""

    def __init__(self, problem, config):
        d, K = int(problem.d), int(problem.K)
        self.d, self.K, self.N, self.m = d, K, int(config.N), int(config.m)
        self.cp, self.keep = _problem_struct(problem)
        c = config
        self.cc = L.Config(int(c.N), int(c.m), int(c.n_osc), int(c.n_conv), int(c.n_anti), int(c.n_cloud), int(c.M),
                           float(c.eps_grad), float(c.eps_dup), float(c.log_delta), float(c.momentum),
                           float(c.alpha), float(c.sigma), float(c.sigma_c), int(c.grad_mode), float(c.fd_h),
                           float(c.ls_c1), int(c.ls_max), float(c.curv_eps), int(c.gate_reps), int(c.phase_mask),
                           int(c.seed), int(c.problem_id), int(getattr(c, "flags", 0)))
        self.n_conv = int(c.n_conv) if int(c.n_conv) > 0 else max(10, int(np.ceil(3 * np.log2(d) - 1e-9)))


class Optimizer:
    """One handle over one problem (``Optimizer(problem, config, x0)``) or a
    batch of independent problems (``Optimizer.batched([(problem, config, x0), ...])``).
    Methods that concern one problem take its index ``problem`` (default 0)."""

    def __init__(self, problem, config, x0: torch.Tensor | np.ndarray | None = None, device=None, stream=None,
                 flags: int | None = None):
        self._create([(problem, config, x0)], device, stream, flags)

    @classmethod
    def batched(cls, items, device=None, stream=None, flags: int | None = None) -> "Optimizer":
        self = cls.__new__(cls)
        self._create(list(items), device, stream, flags)
        return self

    def _create(self, items, device, stream, flags):
        self.lib = L.load()
        if not torch.cuda.is_available():
            raise RuntimeError("libchisao needs a ROCm GPU (torch.cuda.is_available() is False)")
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.specs = [_Spec(p, c) for p, c, _ in items]
        if flags is not None:
            for sp in self.specs:
                sp.cc.flags = int(flags)
        self.P = len(self.specs)
        s0 = self.specs[0]
        self.d, self.K, self.N, self.n_conv = s0.d, s0.K, s0.N, s0.n_conv
        self.cc = s0.cc
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._x0 = []
        ptrs = (C.c_void_p * self.P)()
        for i, (sp, (_, _, x0)) in enumerate(zip(self.specs, items)):
            if x0 is None:
                continue
            x0t = torch.as_tensor(np.asarray(x0, np.float32) if isinstance(x0, np.ndarray) else x0)
            x0t = x0t.to(self.device, torch.float32).contiguous().reshape(sp.N, sp.d)
            self._x0.append(x0t)
            ptrs[i] = x0t.data_ptr()
        probs = (L.Problem * self.P)(*[sp.cp for sp in self.specs])
        cfgs = (L.Config * self.P)(*[sp.cc for sp in self.specs])
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            L.check(self.lib.chisao_init_batched(C.byref(h), self.P, probs, cfgs, ptrs, self.stream.cuda_stream),
                    "chisao_init_batched")
        self.h = h

    # ------------------------------------------------------------------
    def close(self):
        if getattr(self, "h", None):
            self.lib.chisao_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ------------------------------------------------------------------
    def cycle(self, n: int = 1, stats: bool = False):
        """Run n cycles.  With ``stats``: one dict per cycle (one problem), or
        per cycle a list of one dict per problem (a batch)."""
        arr = (L.CycleStats * max(n * self.P, 1))() if stats else None
        L.check(self.lib.chisao_cycle(self.h, n, arr), "chisao_cycle")
        if not stats:
            return None
        rows = [[{f: getattr(arr[i * self.P + p], f) for f, _ in L.CycleStats._fields_} for p in range(self.P)]
                for i in range(n)]
        return [r[0] for r in rows] if self.P == 1 else rows

    def profile_begin(self):
        L.check(self.lib.chisao_profile(self.h, 1, None), "chisao_profile")

    def profile_end(self) -> dict:
        arr = (L.KernelProfile * L.PROF_CLASSES)()
        L.check(self.lib.chisao_profile(self.h, 0, arr), "chisao_profile")
        return {L.PROF_NAMES[i]: dict(launches=arr[i].launches, ms=arr[i].ms, points=arr[i].points)
                for i in range(L.PROF_CLASSES) if arr[i].launches or arr[i].points}

    def tuning(self) -> list:
        """The evaluation schedule the autotuner chose for each problem class."""
        arr = (L.TuningEntry * 64)()
        n = C.c_int(0)
        L.check(self.lib.chisao_tuning(self.h, arr, 64, C.byref(n)), "chisao_tuning")
        return [dict(padded_d=e.padded_d, family=e.family, grad_mode=e.grad_mode, n_problems=e.n_problems,
                     order=e.order, grid_cap=e.grid_cap, ms=list(e.ms), tile_points=e.tile_points,
                     ms_half_tiles=e.ms_half_tiles, ms_full_tiles=e.ms_full_tiles, probe_order=e.probe_order, probe_grid_cap=e.probe_grid_cap,
                     ms_probe=list(e.ms_probe), trial_grid_cap=e.trial_grid_cap) for e in arr[:n.value]]

    def run_phases(self, mask: int):
        L.check(self.lib.chisao_run_phases(self.h, mask), "chisao_run_phases")

    def modes(self, problem: int = 0) -> ModeSet:
        n = C.c_int(0)
        rc = self.lib.chisao_modes(self.h, problem, None, None, 0, C.byref(n))
        if rc not in (L.OK, L.E_RANGE):
            L.check(rc, "chisao_modes")
        X = np.zeros((n.value, self.specs[problem].d), np.float32)
        F = np.zeros(n.value, np.float32)
        L.check(self.lib.chisao_modes(self.h, problem, X.ctypes.data, F.ctypes.data, n.value, C.byref(n)),
                "chisao_modes")
        return ModeSet(X, F)

    def mode_widths(self, problem: int = 0) -> np.ndarray:
        """Per mode (in the order of ``modes``) the preserved inverse-Hessian
        diagonal of -f: squared widths along the coordinates."""
        n = C.c_int(0)
        rc = self.lib.chisao_mode_widths(self.h, problem, None, 0, C.byref(n))
        if rc not in (L.OK, L.E_RANGE):
            L.check(rc, "chisao_mode_widths")
        Wd = np.zeros((n.value, self.specs[problem].d), np.float32)
        L.check(self.lib.chisao_mode_widths(self.h, problem, Wd.ctypes.data, n.value, C.byref(n)),
                "chisao_mode_widths")
        return Wd

    def get_state(self, history: bool = False, problem: int = 0) -> dict:
        sp = self.specs[problem]
        N, d, m = sp.N, sp.d, sp.m
        out = dict(X=np.zeros((N, d), np.float32), F=np.zeros(N, np.float32), G=np.zeros((N, d), np.float32),
                   stuck=np.zeros(N, np.uint8), active=np.zeros(N, np.uint8), stuck_pre=np.zeros(N, np.uint8),
                   removed=np.zeros(N, np.uint8), trace=np.zeros((sp.n_conv + 1, N), np.uint8))
        s = L.State(*[out[f].ctypes.data for f in ("X", "F", "G", "stuck", "active", "stuck_pre", "removed", "trace")])
        if history:
            out.update(S=np.zeros((N, m, d), np.float32), Y=np.zeros((N, m, d), np.float32),
                       rho=np.zeros((N, m), np.float32), head=np.zeros(N, np.int32), cnt=np.zeros(N, np.int32),
                       conv=np.zeros(N, np.uint8), Fg=np.zeros(N, np.float32), Wd=np.zeros((N, d), np.float32),
                       wvalid=np.zeros(N, np.uint8))
            for f in ("S", "Y", "rho", "head", "cnt", "conv", "Fg", "Wd", "wvalid"):
                setattr(s, f, out[f].ctypes.data)
        L.check(self.lib.chisao_get_state(self.h, problem, C.byref(s)), "chisao_get_state")
        out.update(k=s.k, gr_disabled=s.gr_disabled, gr_fail=s.gr_fail, gr_used_last=s.gr_used_last,
                   gr_prev_modes=s.gr_prev_modes)
        return out

    def set_state(self, X=None, stuck=None, active=None, k=None, gr=None, Wd=None, wvalid=None, problem: int = 0):
        sp = self.specs[problem]
        cur = self.get_state(problem=problem)
        keep = []

        def ptr(a, dt, shape):
            if a is None:
                return None
            a = np.ascontiguousarray(np.asarray(a, dt).reshape(shape))
            keep.append(a)
            return a.ctypes.data

        gr = gr or {}
        s = L.State(ptr(X, np.float32, (sp.N, sp.d)), None, None, ptr(stuck, np.uint8, (sp.N,)),
                    ptr(active, np.uint8, (sp.N,)), None, None, None, cur["k"] if k is None else int(k),
                    gr.get("gr_disabled", cur["gr_disabled"]), gr.get("gr_fail", cur["gr_fail"]),
                    gr.get("gr_used_last", cur["gr_used_last"]), gr.get("gr_prev_modes", cur["gr_prev_modes"]))
        s.Wd = ptr(Wd, np.float32, (sp.N, sp.d))
        s.wvalid = ptr(wvalid, np.uint8, (sp.N,))
        L.check(self.lib.chisao_set_state(self.h, problem, C.byref(s)), "chisao_set_state")

    def eval(self, X: torch.Tensor, grad_mode: int = L.GRAD_ADJOINT, want_f: bool = True, want_g: bool = True,
             problem: int = 0):
        """Objective (and gradient) of one problem at the rows of X (a float32 CUDA tensor)."""
        d = self.specs[problem].d
        X = X.to(self.device, torch.float32).contiguous().reshape(-1, d)
        B = X.shape[0]
        f = torch.empty(B, device=self.device, dtype=torch.float32) if want_f else None
        G = torch.empty(B, d, device=self.device, dtype=torch.float32) if want_g else None
        with torch.cuda.stream(self.stream):
            L.check(self.lib.chisao_eval(self.h, problem, X.data_ptr(), B, f.data_ptr() if f is not None else None,
                                         G.data_ptr() if G is not None else None, grad_mode), "chisao_eval")
        return f, G


def eval_static(problem, X: torch.Tensor, grad_mode: int = L.GRAD_ADJOINT, fd_h: float = 0.0, want_f: bool = True,
                want_g: bool = True, stream=None):
    """Objective (and gradient) of ``problem`` at the rows of X (a float32 CUDA
    tensor) without a handle: ``chisao_eval_static``, which allocates no device
    memory (the problem's tables go to the library's static device array)."""
    lib = L.load()
    cp, keep = _problem_struct(problem)
    d = int(problem.d)
    X = X.to(torch.float32).contiguous().reshape(-1, d)
    B = X.shape[0]
    f = torch.empty(B, device=X.device, dtype=torch.float32) if want_f else None
    G = torch.empty(B, d, device=X.device, dtype=torch.float32) if want_g else None
    st = stream if stream is not None else torch.cuda.current_stream(X.device)
    with torch.cuda.device(X.device):
        L.check(lib.chisao_eval_static(C.byref(cp), float(fd_h), X.data_ptr(), B,
                                       f.data_ptr() if f is not None else None,
                                       G.data_ptr() if G is not None else None, grad_mode, st.cuda_stream),
                "chisao_eval_static")
    del keep  # the call synchronized after copying the problem
    return f, G
