"""MI355X sketched Tucker-ALS (Ma & Solomonik, arXiv 2104.01101).

Python face of libtsk (include/tsk.h): thin wrappers that marshal torch device
tensors into the C ABI.  Nothing here computes; there is no CPU fallback -- if
the HIP library is missing every call raises.

    T = Tensor.coo(idx, val, dims)            # or Tensor.dense(x)
    core, factors, fits = tucker_sketch_als(T, ranks, m=1600, sweeps=10)
    cp_factors, fit = cp_via_tucker(T, 20, (30, 30, 30), m=14400, ...)
"""
import ctypes

import torch

from . import _lib as L

__all__ = ["Tensor", "tucker_sketch_als", "cp_via_tucker", "hash_tables", "sketch_rhs_ts",
           "rsvd_solve_noalloc",
           "sketch_lhs_ts", "rc_solve", "rrf_init", "leverage_sample", "leverage_select", "sketch_lev",
           "FiberIndex", "fiber_index", "sketch_lev_coo", "fit",
           "sketched_residual", "sketched_residual_grads", "SketchedResidual", "lib"]

lib = L.lib

_PREC_DTYPE = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}


class Tensor:
    """Device tensor in the library's layout: dense row-major, or COO with one
    int32 index vector per mode (0-based, unsorted, duplicates add)."""

    def __init__(self, dims, values, idx=None):
        self.dims = tuple(int(d) for d in dims)
        self.values = values
        self.idx = idx
        if values.dtype not in (torch.float32, torch.float64):
            raise TypeError("values must be float32 or float64")
        if not values.is_cuda:
            raise ValueError("values must be a device tensor")

    @classmethod
    def dense(cls, x):
        return cls(x.shape, x.contiguous())

    @classmethod
    def coo(cls, idx, val, dims):
        """idx: (nnz, N) or a list of N index vectors."""
        if isinstance(idx, torch.Tensor):
            cols = [idx[:, k].to(torch.int32).contiguous() for k in range(idx.shape[1])]
        else:
            cols = [c.to(torch.int32).contiguous() for c in idx]
        return cls(dims, val.contiguous(), cols)

    @property
    def order(self):
        return len(self.dims)

    @property
    def device(self):
        return self.values.device

    def c_struct(self):
        t = L._Tensor()
        t.order = self.order
        for k, d in enumerate(self.dims):
            t.dims[k] = d
        t.dtype = L.F64 if self.values.dtype == torch.float64 else L.F32
        t.values = self.values.data_ptr()
        if self.idx is None:
            t.layout = L.DENSE
            t.nnz = self.values.numel()
        else:
            t.layout = L.COO
            t.nnz = self.values.numel()
            for k, c in enumerate(self.idx):
                t.idx[k] = c.data_ptr()
        return t


def _options(m, sweeps, sketch, init, prec, seed, rrf_k1, rrf_k2, record_fit, solve="exact",
             rsvd_k=0, first_sweep=0, tol=0.0):
    o = L._Options()
    o.sketch = L.SKETCH[sketch]
    o.m = int(m)
    o.init = L.INIT[init]
    o.rrf_k1, o.rrf_k2 = int(rrf_k1), int(rrf_k2)
    o.sweeps = int(sweeps)
    o.prec = L.PREC[prec]
    o.seed = int(seed)
    o.stream = L.stream_ptr()
    o.flags = (L.FLAG_FINAL_FIT if record_fit == "final"
               else L.FLAG_RECORD_FIT if record_fit else 0)
    o.solve = L.SOLVE[solve]
    o.rsvd_k = int(rsvd_k)
    o.first_sweep = int(first_sweep)
    o.tol = float(tol)
    return o


class TuckerPlan:
    """Pre-allocated outputs and workspace for repeated calls with one shape
    (keeps allocation out of timed loops).  record_fit: True (residual after
    every sweep), "final" (after the last sweep only; earlier entries NaN) or
    False.  first_sweep: absolute index of the first sweep (resume, with
    init="user"); tol: stop when the residual changes by less (needs
    record_fit=True)."""

    def __init__(self, T, ranks, m, sweeps, sketch="ts", init="rrf", prec="f32", seed=0,
                 rrf_k1=0, rrf_k2=0, record_fit=True, solve="exact", rsvd_k=0, first_sweep=0,
                 tol=0.0):
        self.T, self.ranks = T, tuple(int(r) for r in ranks)
        self.opt = _options(m, sweeps, sketch, init, prec, seed, rrf_k1, rrf_k2, record_fit,
                            solve, rsvd_k, first_sweep, tol)
        self.ct = T.c_struct()
        self.cr = L.i32_array(self.ranks)
        nb = ctypes.c_size_t(0)
        L.check(L.lib().tsk_workspace_size(ctypes.byref(self.ct), self.cr, ctypes.byref(self.opt),
                                           ctypes.byref(nb)))
        self._ws, wp, n = L.workspace(nb.value, T.device)
        self.opt.workspace, self.opt.workspace_bytes = wp, n
        dev = T.device
        self.core = torch.zeros(self.ranks, dtype=torch.float64, device=dev)
        self.factors = [torch.zeros((s, r), dtype=torch.float64, device=dev)
                        for s, r in zip(T.dims, self.ranks)]
        self.fits = (ctypes.c_double * max(1, int(sweeps)))()
        self.sweeps = int(sweeps)
        self.record_fit = record_fit

    def run(self, init_factors=None):
        if init_factors is not None:
            for F, G in zip(self.factors, init_factors):
                F.copy_(G)
        self.opt.stream = L.stream_ptr()
        done = ctypes.c_int32(0)
        L.check(L.lib().tsk_tucker_sketch_als(
            ctypes.byref(self.ct), self.cr, ctypes.byref(self.opt), L.ptr(self.core),
            L.ptr_array(self.factors), self.fits if self.record_fit else None,
            ctypes.byref(done)))
        self.sweeps_done = done.value
        fits = list(self.fits)[:done.value] if self.record_fit else []
        return self.core, self.factors, fits


def tucker_sketch_als(T, ranks, m, sweeps, sketch="ts", init="rrf", prec="f32", seed=0,
                      rrf_k1=0, rrf_k2=0, record_fit=True, init_factors=None, solve="exact",
                      rsvd_k=0, first_sweep=0, tol=0.0):
    """Sketch-Tucker-ALS (Alg. 4).  Returns (core, factors, fits) -- FP64 device
    tensors and the per-sweep relative residuals.  solve = "exact" (truncated
    SVD of Z^+ Y) or "rsvd" (RSVD-LRLS, Alg. 5, rsvd_k test-matrix columns,
    0 = min(R + 10, r))."""
    plan = TuckerPlan(T, ranks, m, sweeps, sketch, init, prec, seed, rrf_k1, rrf_k2, record_fit,
                      solve, rsvd_k, first_sweep, tol)
    return plan.run(init_factors)


def cp_via_tucker(T, cp_rank, tucker_ranks, m, tucker_sweeps, cp_sweeps, sketch="lev",
                  init="rrf", prec="f32", seed=0, rrf_k1=0, rrf_k2=0, solve="exact", rsvd_k=0):
    """CP-Sketch-Tucker (Alg. 6).  Returns (cp_factors, cp relative residual)."""
    o = _options(m, tucker_sweeps, sketch, init, prec, seed, rrf_k1, rrf_k2, False, solve, rsvd_k)
    ct = T.c_struct()
    tr = L.i32_array(tucker_ranks)
    nb = ctypes.c_size_t(0)
    L.check(L.lib().tsk_cp_workspace_size(ctypes.byref(ct), int(cp_rank), tr, ctypes.byref(o),
                                          ctypes.byref(nb)))
    keep, wp, n = L.workspace(nb.value, T.device)
    o.workspace, o.workspace_bytes = wp, n
    out = [torch.zeros((s, cp_rank), dtype=torch.float64, device=T.device) for s in T.dims]
    fit_v = ctypes.c_double(0)
    L.check(L.lib().tsk_cp_via_tucker(ctypes.byref(ct), int(cp_rank), tr, int(cp_sweeps),
                                      ctypes.byref(o), L.ptr_array(out), ctypes.byref(fit_v)))
    del keep
    return out, fit_v.value


# -------------------------------------------------------------- components ----
def hash_tables(dims, n, m, seed, device="cuda"):
    """TensorSketch maps of subproblem n: lists (index k) of int32 h and int8 sign
    (None at k = n)."""
    N = len(dims)
    h = [None if k == n else torch.empty(dims[k], dtype=torch.int32, device=device) for k in range(N)]
    s = [None if k == n else torch.empty(dims[k], dtype=torch.int8, device=device) for k in range(N)]
    L.check(L.lib().tsk_hash_tables(N, L.i64_array(dims), n, int(m), int(seed), L.ptr_array(h),
                                    L.ptr_array(s), L.stream_ptr()))
    return h, s


def sketch_rhs_ts(T, n, m, h, s):
    """Y = S^(n) T_(n)^T (m x s_n, dtype of T)."""
    Y = torch.empty((int(m), T.dims[n]), dtype=T.values.dtype, device=T.device)
    ct = T.c_struct()
    keep = L.query_and_alloc(L.lib().tsk_sketch_rhs_ts,
                             (ctypes.byref(ct), int(n), int(m), L.ptr_array(h), L.ptr_array(s),
                              L.ptr(Y)), (L.stream_ptr(),), T.device)
    del keep
    return Y


def sketch_lhs_ts(dims, ranks, n, m, h, s, factors, prec="f64"):
    """Z = S^(n) kron_{k != n} A^(k) (m x r) in the operand precision."""
    r = 1
    for k, R in enumerate(ranks):
        if k != n:
            r *= R
    Z = torch.empty((int(m), r), dtype=_PREC_DTYPE[prec], device=factors[0 if n else 1].device)
    facs = [None if k == n else factors[k].contiguous() for k in range(len(dims))]
    keep = L.query_and_alloc(L.lib().tsk_sketch_lhs_ts,
                             (len(dims), L.i64_array(dims), L.i32_array(ranks), int(n), int(m),
                              L.ptr_array(h), L.ptr_array(s), L.ptr_array(facs), L.PREC[prec],
                              L.ptr(Z)), (L.stream_ptr(),), Z.device)
    del keep
    return Z


def rc_solve(Z, Y, R, prec=None):
    """Exact sketched rank-constrained solve -> (A s x R, W r x R), FP64."""
    if prec is None:
        prec = {torch.float64: "f64", torch.float32: "f32", torch.bfloat16: "bf16"}[Z.dtype]
    m, r = Z.shape
    s = Y.shape[1]
    A = torch.empty((s, R), dtype=torch.float64, device=Z.device)
    W = torch.empty((r, R), dtype=torch.float64, device=Z.device)
    keep = L.query_and_alloc(L.lib().tsk_rc_solve,
                             (L.ptr(Z.contiguous()), L.ptr(Y.contiguous()), m, r, s, int(R),
                              L.PREC[prec], L.ptr(A), L.ptr(W)), (L.stream_ptr(),), Z.device)
    del keep
    return A, W


def rsvd_solve_noalloc(Z, Y, R, Omega, prec=None):
    """rsvd_solve through the entry point that allocates no device memory (its
    scratch is the library's static per-GPU buffer); the outputs A and W are
    the only allocations, made here by the caller's side."""
    if prec is None:
        prec = {torch.float64: "f64", torch.float32: "f32", torch.bfloat16: "bf16"}[Z.dtype]
    m, r = Z.shape
    s = Y.shape[1]
    Om = Omega.to(torch.float64).contiguous()
    A = torch.empty((s, R), dtype=torch.float64, device=Z.device)
    W = torch.empty((r, R), dtype=torch.float64, device=Z.device)
    Zc, Yc = Z.contiguous(), Y.contiguous()
    L.check(L.lib().tsk_rsvd_solve_noalloc(L.ptr(Zc), L.ptr(Yc), m, r, s, int(R), L.PREC[prec],
                                           L.ptr(Om), int(Om.shape[1]), L.ptr(A), L.ptr(W),
                                           L.stream_ptr()))
    return A, W


def rsvd_solve(Z, Y, R, Omega, prec=None):
    """RSVD-LRLS (Alg. 5) with the given s x k Gaussian test matrix ->
    (A s x R, W r x R), FP64."""
    if prec is None:
        prec = {torch.float64: "f64", torch.float32: "f32", torch.bfloat16: "bf16"}[Z.dtype]
    m, r = Z.shape
    s = Y.shape[1]
    Om = Omega.to(torch.float64).contiguous()
    A = torch.empty((s, R), dtype=torch.float64, device=Z.device)
    W = torch.empty((r, R), dtype=torch.float64, device=Z.device)
    keep = L.query_and_alloc(L.lib().tsk_rsvd_solve,
                             (L.ptr(Z.contiguous()), L.ptr(Y.contiguous()), m, r, s, int(R),
                              L.PREC[prec], L.ptr(Om), int(Om.shape[1]), L.ptr(A), L.ptr(W)),
                             (L.stream_ptr(),), Z.device)
    del keep
    return A, W


def rrf_init(T, n, R, k1, k2, seed):
    """Init-RRF (Alg. 3) of mode n -> A (s_n x R, FP64)."""
    A = torch.empty((T.dims[n], R), dtype=torch.float64, device=T.device)
    ct = T.c_struct()
    keep = L.query_and_alloc(L.lib().tsk_rrf_init,
                             (ctypes.byref(ct), int(n), int(R), int(k1), int(k2), int(seed),
                              L.ptr(A)), (L.stream_ptr(),), T.device)
    del keep
    return A


def leverage_sample(dims, ranks, n, m, seed, sweep, factors):
    """-> (idx int32 m x (N-1), w float64 m)."""
    dev = factors[0 if n else 1].device
    idx = torch.empty((int(m), len(dims) - 1), dtype=torch.int32, device=dev)
    w = torch.empty(int(m), dtype=torch.float64, device=dev)
    facs = [None if k == n else factors[k].contiguous() for k in range(len(dims))]
    keep = L.query_and_alloc(L.lib().tsk_leverage_sample,
                             (len(dims), L.i64_array(dims), L.i32_array(ranks), int(n), int(m),
                              int(seed), int(sweep), L.ptr_array(facs), L.ptr(idx), L.ptr(w)),
                             (L.stream_ptr(),), dev)
    del keep
    return idx, w


def leverage_select(dims, ranks, n, m, factors):
    """Deterministic leverage selection -> idx int32 m x (N-1) (weights are 1)."""
    dev = factors[0 if n else 1].device
    idx = torch.empty((int(m), len(dims) - 1), dtype=torch.int32, device=dev)
    facs = [None if k == n else factors[k].contiguous() for k in range(len(dims))]
    keep = L.query_and_alloc(L.lib().tsk_leverage_select,
                             (len(dims), L.i64_array(dims), L.i32_array(ranks), int(n), int(m),
                              L.ptr_array(facs), L.ptr(idx)), (L.stream_ptr(),), dev)
    del keep
    return idx


def sketch_lev(T, ranks, n, m, idx, w, factors, prec="f64"):
    """Sampled rows: Z (m x r), Y (m x s_n) in the operand precision."""
    r = 1
    for k, R in enumerate(ranks):
        if k != n:
            r *= R
    dt = _PREC_DTYPE[prec]
    Z = torch.empty((int(m), r), dtype=dt, device=T.device)
    Y = torch.empty((int(m), T.dims[n]), dtype=dt, device=T.device)
    facs = [None if k == n else factors[k].contiguous() for k in range(T.order)]
    ct = T.c_struct()
    L.check(L.lib().tsk_sketch_lev(ctypes.byref(ct), L.i32_array(ranks), int(n), int(m),
                                   L.ptr(idx), L.ptr(w), L.ptr_array(facs), L.PREC[prec],
                                   L.ptr(Z), L.ptr(Y), L.stream_ptr()))
    return Z, Y


class FiberIndex:
    """Mode-n fibre index of a COO tensor (device buffer owned by this object)."""

    def __init__(self, T, n, keep, pointer, nbytes):
        self.T, self.n, self._keep, self.ptr, self.nbytes = T, int(n), keep, pointer, nbytes


def fiber_index(T, n):
    """Build the mode-n fibre index of COO tensor T (sorted keys + values)."""
    ct = T.c_struct()
    ib, wb = ctypes.c_size_t(0), ctypes.c_size_t(0)
    L.check(L.lib().tsk_fiber_index(ctypes.byref(ct), int(n), None, ctypes.byref(ib), None,
                                    ctypes.byref(wb), L.stream_ptr()))
    keep, ip, ni = L.workspace(ib.value, T.device)
    wkeep, wp, nw = L.workspace(wb.value, T.device)
    ib2, wb2 = ctypes.c_size_t(ni), ctypes.c_size_t(nw)
    L.check(L.lib().tsk_fiber_index(ctypes.byref(ct), int(n), ip, ctypes.byref(ib2), wp,
                                    ctypes.byref(wb2), L.stream_ptr()))
    torch.cuda.current_stream().synchronize()
    del wkeep
    return FiberIndex(T, n, keep, ip, ni)


def sketch_lev_coo(T, index, m, idx, w, prec="f64"):
    """Sampled mode-n fibres of COO tensor T through its fibre index: Y (m x s_n)."""
    n = index.n
    Y = torch.empty((int(m), T.dims[n]), dtype=_PREC_DTYPE[prec], device=T.device)
    ct = T.c_struct()
    L.check(L.lib().tsk_sketch_lev_coo(ctypes.byref(ct), n, index.ptr, int(m), L.ptr(idx),
                                       L.ptr(w), L.PREC[prec], L.ptr(Y), L.stream_ptr()))
    return Y


def fit(T, core, factors):
    """Relative residual ||T - T~|| / ||T|| (FP64)."""
    ct = T.c_struct()
    ranks = [F.shape[1] for F in factors]
    out = ctypes.c_double(0)
    keep = L.query_and_alloc(L.lib().tsk_fit,
                             (ctypes.byref(ct), L.i32_array(ranks), L.ptr(core.contiguous()),
                              L.ptr_array([F.contiguous() for F in factors]),
                              ctypes.byref(out)), (L.stream_ptr(),), T.device)
    del keep
    return out.value


def _ydtype(Y):
    return L.F64 if Y.dtype == torch.float64 else L.F32


def sketched_residual(dims, ranks, n, m, h, s, factors, core, Y):
    """L = ||Z W A^T - Y||_F^2 (device scalar, FP64)."""
    out = torch.empty((), dtype=torch.float64, device=Y.device)
    keep = L.query_and_alloc(L.lib().tsk_sketched_residual_fwd,
                             (len(dims), L.i64_array(dims), L.i32_array(ranks), int(n), int(m),
                              L.ptr_array(h), L.ptr_array(s),
                              L.ptr_array([F.contiguous() for F in factors]),
                              L.ptr(core.contiguous()), L.ptr(Y.contiguous()), _ydtype(Y),
                              L.ptr(out)), (L.stream_ptr(),), Y.device)
    del keep
    return out


def sketched_residual_grads(dims, ranks, n, m, h, s, factors, core, Y):
    """(dL/dA^(k) for every k, dL/dC), FP64."""
    grads = [torch.empty_like(F, dtype=torch.float64) for F in factors]
    gC = torch.empty_like(core, dtype=torch.float64)
    keep = L.query_and_alloc(L.lib().tsk_sketched_residual_bwd,
                             (len(dims), L.i64_array(dims), L.i32_array(ranks), int(n), int(m),
                              L.ptr_array(h), L.ptr_array(s),
                              L.ptr_array([F.contiguous() for F in factors]),
                              L.ptr(core.contiguous()), L.ptr(Y.contiguous()), _ydtype(Y),
                              L.ptr_array(grads), L.ptr(gC)), (L.stream_ptr(),), Y.device)
    del keep
    return grads, gC


class SketchedResidual(torch.autograd.Function):
    """L_n(A^(1..N), C) = ||S^(n) P^(n) C_(n)^T A^(n)T - S^(n) T_(n)^T||_F^2 with the
    hand-written HIP adjoint as backward (sketched intermediates recomputed).

    apply(ctx_tuple, core, *factors) where ctx_tuple = (dims, ranks, n, m, h, s, Y)."""

    @staticmethod
    def forward(ctx, spec, core, *factors):
        dims, ranks, n, m, h, s, Y = spec
        ctx.spec = spec
        ctx.save_for_backward(core, *factors)
        return sketched_residual(dims, ranks, n, m, h, s, [f.detach() for f in factors],
                                 core.detach(), Y)

    @staticmethod
    def backward(ctx, gout):
        core, *factors = ctx.saved_tensors
        dims, ranks, n, m, h, s, Y = ctx.spec
        grads, gC = sketched_residual_grads(dims, ranks, n, m, h, s, factors, core, Y)
        return (None, gout * gC, *[gout * g for g in grads])
