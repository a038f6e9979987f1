"""ALS-based truncated HOSVD (t-HOSVD-ALS / st-HOSVD-ALS) on MI355X.

Python surface over libtucker_als.so.  Inputs and outputs are torch tensors
on the GPU; every computation runs in the library's HIP kernels on the
current torch stream.

Method: Xiao, Yang & Li, "Efficient Alternating Least Squares Algorithms for
Low Multilinear Rank Approximation of Tensors" (arXiv 2004.02583).
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib as L
from ._lib import TuckerALSError, load_library  # noqa: F401

__all__ = [
    "als_sthosvd", "als_thosvd", "hooi", "st_order", "ttm", "tucker_reconstruct", "contract_allbut",
    "als_init_step", "als_sweep_step", "als_sweep_kernel", "qr_f64", "batched_sthosvd",
    "BatchedPlan",
    "TuckerALSError", "load_library", "TuckerProject", "TuckerReconstruct",
]

_DT = {torch.float64: L.TK_F64, torch.float32: L.TK_F32, torch.bfloat16: L.TK_BF16}


def _dtcode(t: torch.Tensor) -> int:
    if t.dtype not in _DT:
        raise TuckerALSError(-2, f"dtype {t.dtype}")
    return _DT[t.dtype]


def _factor_dtype(a_dtype: torch.dtype) -> torch.dtype:
    return torch.float64 if a_dtype == torch.float64 else torch.float32


def _stream(dev) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _require_gpu(*ts):
    for t in ts:
        if not (isinstance(t, torch.Tensor) and t.is_cuda):
            raise TuckerALSError(-1, "inputs must be CUDA (HIP) tensors")
        if not t.is_contiguous():
            raise TuckerALSError(-1, "inputs must be contiguous")


_RESID = {"auto": L.TK_RESID_AUTO, "trace": L.TK_RESID_TRACE,
          "explicit": L.TK_RESID_EXPLICIT}
_RESID_NAME = {v: k for k, v in _RESID.items()}


def _opts(tol, max_iters, seed, order, resid_mode, singular_vectors=False, init_ptrs=None):
    o = L.tk_als_opts()
    o.struct_size = ctypes.sizeof(L.tk_als_opts)
    o.tol = float(tol)
    o.max_iters = int(max_iters)
    o.seed = int(seed) & ((1 << 64) - 1)
    if resid_mode not in _RESID:
        raise TuckerALSError(-1, f"resid_mode {resid_mode!r}")
    o.resid_mode = _RESID[resid_mode]
    o.singular_vectors = 1 if singular_vectors else 0
    o.compute = L.TK_COMPUTE_AS_STORAGE
    keep = []
    if order is not None:
        arr = L.i32arr(order)
        keep.append(arr)
        o.order = ctypes.cast(arr, ctypes.POINTER(ctypes.c_int32))
    if init_ptrs is not None:
        arr = (ctypes.c_void_p * len(init_ptrs))(*init_ptrs)
        keep.append(arr)
        o.init_U = ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p))
    return o, keep


def _info_dict(info: L.tk_als_info, N: int) -> dict:
    return dict(
        iters=[info.iters[n] for n in range(N)],
        converged=[bool(info.converged[n]) for n in range(N)],
        resid=[info.resid[n] for n in range(N)],
        norm_a=info.norm_a,
        sweeps=info.sweeps,
        status=L.STATUS.get(info.status, info.status),
        mode_status=[L.STATUS.get(info.mode_status[n], info.mode_status[n]) for n in range(N)],
        resid_form=[_RESID_NAME.get(info.resid_form[n], info.resid_form[n]) for n in range(N)],
    )


def _driver(which, A, ranks, tol, max_iters, seed, order, resid_mode, workspace,
            singular_vectors=False, init=None):
    lib = L.lib()
    _require_gpu(A)
    N = A.dim()
    dims = L.i64arr(A.shape)
    rk = L.i32arr(ranks) if len(ranks) == N else None
    if rk is None:
        raise TuckerALSError(-1, "len(ranks) must equal A.dim()")
    adt = _dtcode(A)
    need = lib.als_workspace_bytes(which, adt, N, dims, rk)
    if need == 0:
        raise TuckerALSError(-1, "als_workspace_bytes")
    fdt = _factor_dtype(A.dtype)
    dev = A.device
    Us = [torch.empty((A.shape[n], ranks[n]), dtype=fdt, device=dev) for n in range(N)]
    G = torch.empty(tuple(ranks), dtype=fdt, device=dev)
    ws = workspace
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
    init_keep, init_ptrs = [], None
    if init is not None:
        if len(init) != N:
            raise TuckerALSError(-1, "init: one entry (or None) per mode")
        init_ptrs = []
        for n, L0 in enumerate(init):
            if L0 is None:
                init_ptrs.append(None)
                continue
            _require_gpu(L0)
            if tuple(L0.shape) != (A.shape[n], ranks[n]) or L0.dtype != fdt:
                raise TuckerALSError(-1, f"init[{n}]: expected {fdt} of shape "
                                         f"{(A.shape[n], ranks[n])}")
            init_keep.append(L0)
            init_ptrs.append(L0.data_ptr())
    o, keep = _opts(tol, max_iters, seed, order, resid_mode, singular_vectors, init_ptrs)
    info = L.tk_als_info()
    fn = lib.als_sthosvd if which == 1 else lib.als_thosvd
    rc = fn(ctypes.c_void_p(A.data_ptr()), adt, N, dims, rk, ctypes.byref(o),
            L.ptrarr([u.data_ptr() for u in Us]), ctypes.c_void_p(G.data_ptr()),
            ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.byref(info), _stream(dev))
    del keep, init_keep
    L.check(rc, "als_sthosvd" if which == 1 else "als_thosvd", allow=(0, 1))
    return G, Us, _info_dict(info, N)


def st_order(dims, ranks):
    """Processing order of least eq. 2.2 cost (Prop. 1), computed by the library on the
    host (no GPU needed)."""
    lib = L.lib()
    N = len(dims)
    out = L.i32arr([0] * N)
    L.check(lib.st_order_auto(N, L.i64arr(dims), L.i32arr(ranks), out), "st_order_auto")
    return [int(x) for x in out]


def als_sthosvd(A, ranks, tol=1e-4, max_iters=50, seed=0, order=None,
                resid_mode="auto", workspace=None, init=None):
    """st-HOSVD-ALS (Algorithm 3.5).  Returns (G, [U_n], info).  order: None (natural),
    a permutation, or "auto" (``st_order``).  resid_mode: "auto", "trace" or "explicit"
    (the residual form of the eq. E5.01 stop test).  init: None, or one I_n x R_n
    initial guess L_0 (or None) per mode, in the factor dtype (a warm start of
    Algorithm 3.3)."""
    if isinstance(order, str):
        if order != "auto":
            raise TuckerALSError(-1, "order must be None, a permutation or 'auto'")
        order = st_order(list(A.shape), list(ranks))
    return _driver(1, A, list(ranks), tol, max_iters, seed, order, resid_mode, workspace,
                   init=init)


def als_thosvd(A, ranks, tol=1e-4, max_iters=50, seed=0, resid_mode="auto",
               workspace=None, singular_vectors=False, init=None):
    """t-HOSVD-ALS (Algorithm 3.4).  Returns (G, [U_n], info).  With singular_vectors the
    factors are the singular vectors of A_(n) inside the ALS subspaces (Section 3).
    init as for ``als_sthosvd``."""
    return _driver(0, A, list(ranks), tol, max_iters, seed, None, resid_mode, workspace,
                   singular_vectors, init=init)


def hooi(A, factors, tol=1e-10, max_iters=50, als_tol=1e-8, als_max_iters=50, seed=0,
         resid_mode="auto", workspace=None):
    """HOOI refinement (Section 6.3) started from ``factors`` (orthonormal I_n x R_n
    tensors, left unchanged).  Returns (G, [U_n], info) with the refined factors;
    als_tol / als_max_iters drive the warm-started inner ALS."""
    lib = L.lib()
    _require_gpu(A)
    N = A.dim()
    if len(factors) != N:
        raise TuckerALSError(-1, "one factor per mode")
    ranks = [int(U.shape[1]) for U in factors]
    dims = L.i64arr(A.shape)
    rk = L.i32arr(ranks)
    adt = _dtcode(A)
    need = lib.hooi_workspace_bytes(adt, N, dims, rk)
    if need == 0:
        raise TuckerALSError(-1, "hooi_workspace_bytes")
    fdt = _factor_dtype(A.dtype)
    dev = A.device
    Us = []
    for n, U in enumerate(factors):
        _require_gpu(U)
        if tuple(U.shape) != (A.shape[n], ranks[n]):
            raise TuckerALSError(-1, "factor shape")
        Us.append(U.to(fdt).clone().contiguous())
    G = torch.empty(tuple(ranks), dtype=fdt, device=dev)
    ws = workspace
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
    o, keep = _opts(als_tol, als_max_iters, seed, None, resid_mode)
    info = L.tk_hooi_info()
    rc = lib.hooi_refine(ctypes.c_void_p(A.data_ptr()), adt, N, dims, rk, ctypes.byref(o),
                         float(tol), int(max_iters), L.ptrarr([u.data_ptr() for u in Us]),
                         ctypes.c_void_p(G.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                         ws.numel(), ctypes.byref(info), _stream(dev))
    del keep
    L.check(rc, "hooi_refine", allow=(0, 1))
    return G, Us, dict(iters=info.iters, converged=bool(info.converged),
                       relerr_init=info.relerr_init, relerr=info.relerr, norm_a=info.norm_a,
                       sweeps=info.sweeps, status=L.STATUS.get(info.status, info.status))


def workspace_bytes(which: str, A_shape, dtype, ranks) -> int:
    lib = L.lib()
    return lib.als_workspace_bytes(1 if which == "st" else 0, _DT[dtype], len(A_shape),
                                   L.i64arr(A_shape), L.i32arr(ranks))


def ttm(X, M, mode, transpose=False, out=None):
    """Y = X x_mode op(M) (Section 2); op(M) = M (J x I) or M^T when
    transpose=True (M stored I x J)."""
    lib = L.lib()
    _require_gpu(X, M)
    J = M.shape[1] if transpose else M.shape[0]
    Iin = M.shape[0] if transpose else M.shape[1]
    if Iin != X.shape[mode]:
        raise TuckerALSError(-1, "ttm: matrix does not match mode size")
    shape = list(X.shape)
    shape[mode] = J
    ydt = _factor_dtype(X.dtype)
    Y = out if out is not None else torch.empty(shape, dtype=ydt, device=X.device)
    rc = lib.ttm(ctypes.c_void_p(X.data_ptr()), _dtcode(X), X.dim(), L.i64arr(X.shape), mode,
                 ctypes.c_void_p(M.data_ptr()), _dtcode(M), J, 1 if transpose else 0,
                 ctypes.c_void_p(Y.data_ptr()), _dtcode(Y), _stream(X.device))
    L.check(rc, "ttm")
    return Y


def tucker_reconstruct(G, Us, workspace=None):
    """A_hat = G x_1 U_1 ... x_N U_N (Section 2)."""
    lib = L.lib()
    _require_gpu(G, *Us)
    N = G.dim()
    dims = [u.shape[0] for u in Us]
    ranks = list(G.shape)
    dt = _dtcode(G)
    need = lib.tucker_reconstruct_workspace_bytes(dt, N, L.i32arr(ranks), L.i64arr(dims))
    ws = workspace
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=G.device)
    out = torch.empty(dims, dtype=G.dtype, device=G.device)
    rc = lib.tucker_reconstruct(ctypes.c_void_p(G.data_ptr()), dt, N, L.i32arr(ranks),
                                L.i64arr(dims), L.ptrarr([u.data_ptr() for u in Us]),
                                ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                                ws.numel(), _stream(G.device))
    L.check(rc, "tucker_reconstruct")
    return out


def contract_allbut(X, Y, mode):
    """K = X_(mode) Y_(mode)^T: contraction over every mode but ``mode``."""
    lib = L.lib()
    _require_gpu(X, Y)
    J = Y.shape[mode]
    dt = _dtcode(X)
    need = lib.contract_allbut_workspace_bytes(dt, X.dim(), L.i64arr(X.shape), mode, J)
    if need == 0:
        raise TuckerALSError(-1, "contract_allbut_workspace_bytes")
    ws = torch.empty(need, dtype=torch.uint8, device=X.device)
    K = torch.empty((X.shape[mode], J), dtype=X.dtype, device=X.device)
    rc = lib.contract_allbut(ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(Y.data_ptr()), dt,
                             X.dim(), L.i64arr(X.shape), mode, J, ctypes.c_void_p(K.data_ptr()),
                             ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(X.device))
    L.check(rc, "contract_allbut")
    return K


def _step_ws(A, mode, R):
    lib = L.lib()
    dims = list(A.shape)
    ranks = [min(R, d) for d in dims]
    ranks[mode] = R
    # the st query covers a mode solve on the input shape
    need = lib.als_workspace_bytes(1, _dtcode(A), A.dim(), L.i64arr(dims),
                                   L.i32arr([R] * A.dim()) if R <= min(dims) else L.i32arr(ranks))
    return torch.empty(max(need, 1 << 20) * 2, dtype=torch.uint8, device=A.device)


def als_init_step(A, mode, R, seed=0):
    """Section 5 initial guess on the mode view: returns (Y = A_(n) S, L0, ||A||^2)."""
    lib = L.lib()
    _require_gpu(A)
    ws = _step_ws(A, mode, R)
    Y = torch.empty((A.shape[mode], R), dtype=torch.float64, device=A.device)
    L0 = torch.empty_like(Y)
    n2 = ctypes.c_double(0.0)
    rc = lib.als_init_step(ctypes.c_void_p(A.data_ptr()), _dtcode(A), A.dim(),
                           L.i64arr(A.shape), mode, R, int(seed), ctypes.c_void_p(Y.data_ptr()),
                           ctypes.c_void_p(L0.data_ptr()), ctypes.byref(n2),
                           ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(A.device))
    L.check(rc, "als_init_step")
    return Y, L0, n2.value


def als_sweep_step(A, mode, Lk, norm2, resid_mode="trace"):
    """One ALS sweep (Algorithm 3.3) from L_k: returns (L_{k+1}, res_k^2)."""
    lib = L.lib()
    _require_gpu(A, Lk)
    R = Lk.shape[1]
    ws = _step_ws(A, mode, R)
    Ln = torch.empty_like(Lk)
    r2 = ctypes.c_double(0.0)
    rm = _RESID[resid_mode]
    rc = lib.als_sweep_step(ctypes.c_void_p(A.data_ptr()), _dtcode(A), A.dim(),
                            L.i64arr(A.shape), mode, R, ctypes.c_void_p(Lk.data_ptr()),
                            ctypes.c_void_p(Ln.data_ptr()), float(norm2), rm, ctypes.byref(r2),
                            ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(A.device))
    L.check(rc, "als_sweep_step")
    return Ln, r2.value


def als_sweep_kernel(A, mode, Lq, reduce=True, workspace=None):
    """The tensor-streaming part of one sweep: with Lq = L (L^T L)^{-1}
    (FP32), returns (Lacc = A_(n) V, GV = V^T V) for V = A_(n)^T Lq
    (FP64), or (None, None) when reduce=False (kernel only, for timing)."""
    lib = L.lib()
    _require_gpu(A, Lq)
    R = Lq.shape[1]
    ws = workspace if workspace is not None else _step_ws(A, mode, R)
    dev = A.device
    Lacc = torch.empty((A.shape[mode], R), dtype=torch.float64, device=dev) if reduce else None
    GV = torch.empty((R, R), dtype=torch.float64, device=dev) if reduce else None
    rc = lib.als_sweep_kernel(ctypes.c_void_p(A.data_ptr()), _dtcode(A), A.dim(),
                              L.i64arr(A.shape), mode, R, ctypes.c_void_p(Lq.data_ptr()),
                              ctypes.c_void_p(Lacc.data_ptr()) if reduce else None,
                              ctypes.c_void_p(GV.data_ptr()) if reduce else None,
                              1 if reduce else 0, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                              _stream(dev))
    L.check(rc, "als_sweep_kernel")
    return Lacc, GV


def step_workspace(A, mode, R):
    """A workspace large enough for the single-step entry points."""
    return _step_ws(A, mode, R)


def qr_f64(Lm):
    """Reduced QR (FP64) with diag(R_hat) > 0; returns Q."""
    lib = L.lib()
    _require_gpu(Lm)
    m, r = Lm.shape
    ws = torch.empty(m * r * 8 + 3 * 65536, dtype=torch.uint8, device=Lm.device)
    Q = torch.empty_like(Lm)
    rc = lib.qr_f64(ctypes.c_void_p(Lm.data_ptr()), m, r, ctypes.c_void_p(Q.data_ptr()), None,
                    ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(Lm.device))
    L.check(rc, "qr_f64")
    return Q


class BatchedPlan:
    """Packed device buffers of a batch of order-3 FP32 tensors for
    ``als_sthosvd_batched``.  ``run`` decomposes the tensors in place (the
    packed inputs stay unchanged) and can be called again: with the same
    buffers and options the library replays the HIP graph it captured."""

    def __init__(self, tensors, ranks_list):
        lib = L.lib()
        self.count = len(tensors)
        if self.count == 0:
            raise TuckerALSError(-1, "batched: no tensors")
        dev = tensors[0].device
        dims3, ranks3, a_off, u_off, g_off = [], [], [], [], []
        ao = uo = go = 0
        for A, rk in zip(tensors, ranks_list):
            if A.dim() != 3 or A.dtype != torch.float32:
                raise TuckerALSError(-1, "batched: order-3 float32 tensors only")
            dims3 += list(A.shape)
            ranks3 += list(rk)
            a_off.append(ao)
            ao += A.numel()
            for n in range(3):
                u_off.append(uo)
                uo += A.shape[n] * rk[n]
            g_off.append(go)
            go += rk[0] * rk[1] * rk[2]
        self.dims3, self.ranks3 = dims3, ranks3
        self.a_off, self.u_off, self.g_off = a_off, u_off, g_off
        self.A = torch.cat([t.reshape(-1) for t in tensors]).contiguous()
        self.U = torch.empty(uo, dtype=torch.float32, device=dev)
        self.G = torch.empty(go, dtype=torch.float32, device=dev)
        self._d3, self._r3 = L.i64arr(dims3), L.i32arr(ranks3)
        self._ao, self._uo, self._go = L.i64arr(a_off), L.i64arr(u_off), L.i64arr(g_off)
        need = lib.als_sthosvd_batched_workspace_bytes(self.count, self._d3, self._r3)
        if need == 0:
            raise TuckerALSError(-1, "als_sthosvd_batched_workspace_bytes")
        self.ws = torch.empty(need, dtype=torch.uint8, device=dev)
        self.iters = (ctypes.c_int32 * (3 * self.count))()
        self.status = (ctypes.c_int32 * self.count)()

    @property
    def algorithmic_bytes_per_pass(self):
        """Bytes of one read of every input tensor (FP32)."""
        return 4 * self.A.numel()

    def run(self, tol=1e-4, max_iters=50, seed=0, resid_mode="auto"):
        lib = L.lib()
        o, keep = _opts(tol, max_iters, seed, None, resid_mode)
        rc = lib.als_sthosvd_batched(ctypes.c_void_p(self.A.data_ptr()), L.TK_F32, self.count,
                                     self._d3, self._r3, self._ao, ctypes.byref(o),
                                     ctypes.c_void_p(self.U.data_ptr()), self._uo,
                                     ctypes.c_void_p(self.G.data_ptr()), self._go, self.iters,
                                     self.status, ctypes.c_void_p(self.ws.data_ptr()),
                                     self.ws.numel(), _stream(self.A.device))
        del keep
        sts = [self.status[t] for t in range(self.count)]
        # a member's own failure (e.g. rank deficiency) is reported in its status;
        # only call-level failures raise
        if rc not in (0, 1) and rc not in sts:
            L.check(rc, "als_sthosvd_batched")
        return sts

    def results(self):
        out = []
        for t in range(self.count):
            d = self.dims3[3 * t:3 * t + 3]
            rk = self.ranks3[3 * t:3 * t + 3]
            Us = [self.U[self.u_off[3 * t + n]:self.u_off[3 * t + n] + d[n] * rk[n]]
                  .view(d[n], rk[n]) for n in range(3)]
            G = self.G[self.g_off[t]:self.g_off[t] + rk[0] * rk[1] * rk[2]].view(*rk)
            out.append((G, Us, [self.iters[3 * t + n] for n in range(3)]))
        return out


def batched_sthosvd(tensors, ranks_list, tol=1e-4, max_iters=50, seed=0, resid_mode="auto"):
    """st-HOSVD-ALS of many small order-3 FP32 tensors in one batched call.

    Returns a list of (G, [U1, U2, U3], iters) and the per-tensor statuses."""
    if len(tensors) == 0:
        return [], []
    plan = BatchedPlan(tensors, ranks_list)
    sts = plan.run(tol=tol, max_iters=max_iters, seed=seed, resid_mode=resid_mode)
    return plan.results(), sts


from .autograd import TuckerProject, TuckerReconstruct  # noqa: E402
