"""Thin Python layer over the C ABI: torch tensors supply device memory and the
HIP stream; every step of the hot path runs in the library's HIP kernels.

Functions keep the C names (rsr_sample, rsr_classify, rsr_eval_unknown,
rsr_estimate, rsr_grad); the small classes own the C handles.
"""
import ctypes
import os

import numpy as np
import torch

from . import _abi as A


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class Context:
    """rsr_ctx on a device, enqueueing on the given torch stream (default: the
    current stream of that device)."""

    def __init__(self, device=0, stream=None):
        lib = A.lib()
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible: the RSR library runs on the GPU only")
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        st = lib.rsr_ctx_create(int(device), ctypes.c_void_p(self.stream.cuda_stream),
                                ctypes.byref(h))
        if st != A.RSR_OK:
            raise A.RSRError(st, "rsr_ctx_create failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            A.lib().rsr_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, st):
        A.check(self.h, st)


class Model:
    """rsr_model: independent components with state probabilities p [n][K] (fp64)."""

    def __init__(self, ctx, p):
        p = np.ascontiguousarray(np.asarray(p, dtype=np.float64))
        if p.ndim != 2:
            raise ValueError("p must be [n][K]")
        self.ctx = ctx
        self.n, self.K = p.shape
        self.p = p
        h = ctypes.c_void_p()
        ctx.check(A.lib().rsr_model_create(ctx.h, self.n, self.K, p.ctypes.data_as(ctypes.c_void_p),
                                           ctypes.byref(h)))
        self.h = h

    @property
    def words(self):
        return int(A.lib().rsr_words(self.n, self.K))

    def update(self, p):
        """rsr_model_update: new probabilities of the same shape, uploaded on the
        context stream without allocating."""
        p = np.ascontiguousarray(np.asarray(p, dtype=np.float64))
        if p.shape != (self.n, self.K):
            raise ValueError(f"p must be [{self.n}][{self.K}]")
        self.ctx.check(A.lib().rsr_model_update(self.h, p.ctypes.data_as(ctypes.c_void_p)))
        self.p = p

    def close(self):
        if getattr(self, "h", None):
            A.lib().rsr_model_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Refs:
    """rsr_refs: lower [R_L][n] and upper [R_U][n] uint8 reference states."""

    @property
    def consistent(self):
        out = ctypes.c_int32(0)
        self.ctx.check(A.lib().rsr_refs_consistent(self.h, ctypes.byref(out)))
        return bool(out.value)

    def __init__(self, ctx, n, K, lower, upper):
        lower = np.ascontiguousarray(np.asarray(lower, dtype=np.uint8).reshape(-1, n))
        upper = np.ascontiguousarray(np.asarray(upper, dtype=np.uint8).reshape(-1, n))
        self.ctx, self.n, self.K = ctx, int(n), int(K)
        self.R_L, self.R_U = lower.shape[0], upper.shape[0]
        h = ctypes.c_void_p()
        ctx.check(A.lib().rsr_refs_create(
            ctx.h, self.n, self.K, lower.ctypes.data_as(ctypes.c_void_p) if self.R_L else None,
            self.R_L, upper.ctypes.data_as(ctypes.c_void_p) if self.R_U else None, self.R_U,
            ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            A.lib().rsr_refs_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class System:
    """rsr_system: s-t connectivity of a graph at a level (kind "st"), global
    connectivity at level 1 (connected) or 2 (two-edge-connected) (kind
    "global"), max s-t flow >= level with capacities = states (kind "flow"),
    or any coherent system function given as a host callback (kind
    "callback": `phi` maps a uint8 state vector [n] to the system state, and
    Phi = [phi(x) >= level]; `graph` may then be None, with n given)."""

    def __init__(self, ctx, graph, K=2, level=1, kind="st", phi=None, n=None):
        self._phi_fn = None
        if kind == "callback":
            if phi is None or n is None:
                raise ValueError("a callback system needs phi and n")
            n = int(n)

            def trampoline(x_ptr, n_c, _user):
                x = np.ctypeslib.as_array(x_ptr, shape=(n_c,)).copy()
                try:
                    return int(phi(x))
                except Exception:   # an exception cannot cross the C ABI
                    return -1

            self._phi_fn = A.PHI_FN(trampoline)
            desc = A.rsr_system_desc(A.RSR_SYS_HOST_CALLBACK, 0, n, int(K), None, None, 0, 0,
                                     int(level), self._phi_fn, None)
        else:
            eu = np.ascontiguousarray(graph["edge_u"], dtype=np.int32)
            ev = np.ascontiguousarray(graph["edge_v"], dtype=np.int32)
            code = {"st": A.RSR_SYS_ST_CONNECTIVITY, "global": A.RSR_SYS_GLOBAL_CONNECTIVITY,
                    "flow": A.RSR_SYS_MAX_FLOW}[kind]
            desc = A.rsr_system_desc(
                code, int(graph["n_nodes"]), eu.size, int(K),
                eu.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                ev.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                int(graph.get("source", 0)), int(graph.get("sink", 0)), int(level))
            n = eu.size
        self.kind = kind
        self.ctx, self.n, self.K, self.level = ctx, int(n), int(K), int(level)
        h = ctypes.c_void_p()
        ctx.check(A.lib().rsr_system_create(ctx.h, ctypes.byref(desc), ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            A.lib().rsr_system_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def alloc_samples(ctx, model_or_n, K=None, N=0):
    if isinstance(model_or_n, Model):
        W = model_or_n.words
    else:
        W = int(A.lib().rsr_words(int(model_or_n), int(K)))
    return torch.empty((W, int(N)), dtype=torch.int32, device=ctx.device)


def rsr_sample(ctx, model, seed, stream_id, first, N, out=None):
    out = alloc_samples(ctx, model, N=N) if out is None else out
    ctx.check(A.lib().rsr_sample(ctx.h, model.h, int(seed), int(stream_id), int(first), int(N),
                                 _ptr(out)))
    return out


def rsr_classify(ctx, refs, samples, N, mode=A.RSR_LABEL, form=A.RSR_AUTO, flags=None,
                 match=None, want_match=False):
    flags = torch.empty(int(N), dtype=torch.uint8, device=ctx.device) if flags is None else flags
    if want_match and match is None:
        match = torch.empty((int(N), 2), dtype=torch.int32, device=ctx.device)
    ctx.check(A.lib().rsr_classify(ctx.h, refs.h, _ptr(samples), int(N), int(mode), int(form),
                                   _ptr(flags), _ptr(match)))
    return (flags, match) if want_match else flags


def rsr_eval_unknown(ctx, system, samples, N, flags, which=A.RSR_UNKNOWN_ONLY, Y=None,
                     n_evaluated=None):
    Y = torch.empty(int(N), dtype=torch.uint8, device=ctx.device) if Y is None else Y
    ctx.check(A.lib().rsr_eval_unknown(ctx.h, system.h, _ptr(samples), int(N), _ptr(flags),
                                       int(which), _ptr(Y), _ptr(n_evaluated)))
    return Y


def rsr_estimate(ctx, flags, Y, N):
    est = A.rsr_estimate_t()
    ctx.check(A.lib().rsr_estimate(ctx.h, _ptr(flags), _ptr(Y), int(N), ctypes.byref(est)))
    return est.as_dict()


def rsr_grad(ctx, model, samples, Y, N, G=None, counts=None, want_counts=False):
    G = torch.empty((model.n, model.K), dtype=torch.float32, device=ctx.device) if G is None else G
    if want_counts and counts is None:
        counts = torch.empty((model.n, model.K), dtype=torch.int64, device=ctx.device)
    ctx.check(A.lib().rsr_grad(ctx.h, model.h, _ptr(samples), _ptr(Y), int(N), _ptr(G),
                               _ptr(counts)))
    return (G, counts) if want_counts else G


def rsr_importance(ctx, model, samples, Y, N, I=None):
    """Binary Birnbaum importance dP/dp_i (K = 2) as fp32 [n]."""
    I = torch.empty(model.n, dtype=torch.float32, device=ctx.device) if I is None else I
    ctx.check(A.lib().rsr_importance(ctx.h, model.h, _ptr(samples), _ptr(Y), int(N), _ptr(I)))
    return I


def rsr_boundary_search(ctx, system, samples, N, picks, rows=None, side=None):
    """Boundary states from the samples picks (device int64 indices): returns
    (rows [n_pick][n] u8, side [n_pick] u8: 0 lower, 1 upper)."""
    n_pick = int(picks.numel())
    if rows is None:
        rows = torch.empty((n_pick, system.n), dtype=torch.uint8, device=ctx.device)
    if side is None:
        side = torch.empty(n_pick, dtype=torch.uint8, device=ctx.device)
    ctx.check(A.lib().rsr_boundary_search(ctx.h, system.h, _ptr(samples), int(N), _ptr(picks),
                                          n_pick, _ptr(rows), _ptr(side)))
    return rows, side


def stage1(ctx, model, system, N, picks, eps_u, max_rows, max_iters, seed, lower0=None,
           upper0=None):
    """Stage-1 loop (rsr_stage1): returns (lower rows, upper rows, result dict),
    rows as uint8 numpy arrays [R][n] in discovery order."""
    n = model.n

    def rows(a):
        if a is None:
            return np.zeros((0, n), dtype=np.uint8)
        return np.ascontiguousarray(a, dtype=np.uint8).reshape(-1, n)

    lo0, up0 = rows(lower0), rows(upper0)
    cap_l = max(int(max_rows), lo0.shape[0])
    cap_u = max(int(max_rows), up0.shape[0])
    lower = np.zeros((cap_l, n), dtype=np.uint8)
    upper = np.zeros((cap_u, n), dtype=np.uint8)
    prm = A.rsr_stage1_params(int(N), int(picks), float(eps_u), int(max_rows), int(max_iters),
                              int(seed))
    res = A.rsr_stage1_result()
    ctx.check(A.lib().rsr_stage1(ctx.h, model.h, system.h, ctypes.byref(prm),
                                 lo0.ctypes.data if lo0.size else None, lo0.shape[0],
                                 up0.ctypes.data if up0.size else None, up0.shape[0],
                                 lower.ctypes.data, cap_l, upper.ctypes.data, cap_u,
                                 ctypes.byref(res)))
    out = res.as_dict()
    return lower[: out["R_L"]].copy(), upper[: out["R_U"]].copy(), out


class Buffers:
    """Device buffers for one Stage-2 pass of N samples of an n x K model."""

    def __init__(self, ctx, n, K, N):
        W = int(A.lib().rsr_words(int(n), int(K)))
        dev = ctx.device
        self.N = int(N)
        self.samples = torch.empty((W, self.N), dtype=torch.int32, device=dev)
        self.flags = torch.empty(self.N, dtype=torch.uint8, device=dev)
        self.Y = torch.empty(self.N, dtype=torch.uint8, device=dev)
        self.G = torch.empty((n, K), dtype=torch.float32, device=dev)
        self.n_eval = torch.zeros(1, dtype=torch.int64, device=dev)


def stage2(ctx, model, refs, system, N, seed, stream_id=0, first=0, form=A.RSR_AUTO, grad=True,
           buffers=None, estimate=True):
    """One pass of the hot path: sample -> classify (LABEL) -> evaluate the
    unclassified samples -> estimate (-> gradient).  Returns (estimate dict or
    None, buffers)."""
    b = buffers or Buffers(ctx, model.n, model.K, N)
    lib, h = A.lib(), ctx.h
    ctx.check(lib.rsr_sample(h, model.h, int(seed), int(stream_id), int(first), int(N),
                             _ptr(b.samples)))
    ctx.check(lib.rsr_classify(h, refs.h, _ptr(b.samples), int(N), A.RSR_LABEL, int(form),
                               _ptr(b.flags), None))
    ctx.check(lib.rsr_eval_unknown(h, system.h, _ptr(b.samples), int(N), _ptr(b.flags),
                                   A.RSR_UNKNOWN_ONLY, _ptr(b.Y), _ptr(b.n_eval)))
    if grad:
        ctx.check(lib.rsr_grad(h, model.h, _ptr(b.samples), _ptr(b.Y), int(N), _ptr(b.G), None))
    est = rsr_estimate(ctx, b.flags, b.Y, N) if estimate else None
    return est, b


class Plan:
    """rsr_plan over a list of jobs.  Each job is a dict with keys model, refs,
    system, seed, N, buffers (a Buffers) and optionally stream_id and grad
    (default True: the job's gradient goes to buffers.G).  tune: False (no
    timing, default configurations), True (time every segment), or the path
    of a JSON tuning cache (reuse stored choices, time and store the rest)."""

    def __init__(self, ctx, jobs, tune=True):
        self.ctx = ctx
        self.jobs = list(jobs)
        arr = (A.rsr_job * len(self.jobs))()
        for k, jb in enumerate(self.jobs):
            b = jb["buffers"]
            arr[k] = A.rsr_job(jb["model"].h.value, jb["refs"].h.value, jb["system"].h.value,
                               int(jb["seed"]), int(jb.get("stream_id", 0)), int(jb["N"]),
                               b.samples.data_ptr(), b.flags.data_ptr(), b.Y.data_ptr(),
                               b.G.data_ptr() if jb.get("grad", True) else None)
        self._arr = arr
        h = ctypes.c_void_p()
        if tune is True:
            cache = b""
        elif tune is False or tune is None:
            cache = None
        else:
            cache = os.fsencode(tune)
        ctx.check(A.lib().rsr_plan_create(ctx.h, arr, len(self.jobs), cache, ctypes.byref(h)))
        self.h = h

    def run(self):
        self.ctx.check(A.lib().rsr_plan_run(self.h))

    def results(self, want_grad=True):
        est = (A.rsr_estimate_t * len(self.jobs))()
        sizes = [jb["model"].n * jb["model"].K for jb in self.jobs]
        G = np.zeros(sum(sizes), dtype=np.float32) if want_grad else None
        self.ctx.check(A.lib().rsr_plan_results(
            self.h, est, G.ctypes.data_as(ctypes.c_void_p) if want_grad else None))
        out = [e.as_dict() for e in est]
        if not want_grad:
            return out, None
        grads, off = [], 0
        for jb, sz in zip(self.jobs, sizes):
            grads.append(G[off:off + sz].reshape(jb["model"].n, jb["model"].K).copy())
            off += sz
        return out, grads

    def close(self):
        if getattr(self, "h", None):
            A.lib().rsr_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
