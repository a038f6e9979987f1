"""torch.autograd Functions over the Tucker projection / reconstruction chain.

Forward and backward run in the library's kernels: mode-n products (ttm) for
the chains and contract_allbut for the factor gradients.

For Y = X x_n M (Section 2 mode-n product) the adjoints are
    dX = dY x_n M^T,      dM = dY_(n) X_(n)^T.
Chaining them through
    project:      G = A x_1 U_1^T x_2 ... x_N U_N^T          (eq. best)
    reconstruct:  A_hat = G x_1 U_1 x_2 ... x_N U_N           (Tucker format)
gives
    project:      dA = dG x_1 U_1 ... x_N U_N,
                  dU_n = X^(n)_(n) dG_(n)^T,  X^(n) = A x_{m != n} U_m^T
    reconstruct:  dG = dY x_1 U_1^T ... x_N U_N^T,
                  dU_n = Z^(n)_(n) G_(n)^T,   Z^(n) = dY x_{m != n} U_m^T.

The projection saves its prefix intermediates T_k = A x_{m<k} U_m^T for the
backward pass only while their total size stays within the memory budget;
otherwise the backward pass recomputes them from A.
"""
from __future__ import annotations

import torch

_BUDGET = [1 << 30]   # bytes of saved intermediates (default 1 GiB)


def set_memory_budget(nbytes: int) -> None:
    """Bytes the projection may keep between forward and backward."""
    _BUDGET[0] = int(nbytes)


def get_memory_budget() -> int:
    return _BUDGET[0]


def _ttm(X, U, mode, transpose):
    from . import ttm
    return ttm(X.contiguous(), U.contiguous(), mode, transpose=transpose)


def _prefixes(A, Us, upto):
    """[T_0 = A, T_1, ..., T_upto] with T_k = A x_{m<k} U_m^T."""
    out = [A]
    X = A
    for m in range(upto):
        X = _ttm(X, Us[m], m, True)
        out.append(X)
    return out


class TuckerProject(torch.autograd.Function):
    """G = A x_1 U_1^T ... x_N U_N^T."""

    @staticmethod
    def forward(ctx, A, *Us):
        N = A.dim()
        pre = _prefixes(A.contiguous(), Us, N)
        G = pre[N]
        mid = pre[1:N]
        saved_bytes = sum(t.numel() * t.element_size() for t in mid)
        keep = saved_bytes <= _BUDGET[0]
        ctx.kept = keep
        ctx.N = N
        if keep:
            ctx.save_for_backward(A, *Us, *mid)
        else:
            ctx.save_for_backward(A, *Us)
        return G

    @staticmethod
    def backward(ctx, dG):
        from . import contract_allbut, tucker_reconstruct
        N = ctx.N
        saved = ctx.saved_tensors
        A, Us = saved[0], list(saved[1:N + 1])
        dG = dG.contiguous()
        dA = tucker_reconstruct(dG, Us) if ctx.needs_input_grad[0] else None
        dUs = [None] * N
        if any(ctx.needs_input_grad[1:]):
            pre = [A] + list(saved[N + 1:]) if ctx.kept else None
            for n in range(N):
                if not ctx.needs_input_grad[1 + n]:
                    continue
                # T_n = A x_{m<n} U_m^T (saved or recomputed), then the rest
                X = pre[n] if pre is not None else _prefixes(A, Us, n)[n]
                for m in range(n + 1, N):
                    X = _ttm(X, Us[m], m, True)
                dUs[n] = contract_allbut(X.contiguous(), dG, n)
        return (dA, *dUs)


class TuckerReconstruct(torch.autograd.Function):
    """A_hat = G x_1 U_1 ... x_N U_N."""

    @staticmethod
    def forward(ctx, G, *Us):
        from . import tucker_reconstruct
        ctx.N = G.dim()
        ctx.save_for_backward(G, *Us)
        return tucker_reconstruct(G.contiguous(), [u.contiguous() for u in Us])

    @staticmethod
    def backward(ctx, dY):
        from . import contract_allbut
        N = ctx.N
        saved = ctx.saved_tensors
        G, Us = saved[0], list(saved[1:])
        pre = _prefixes(dY.contiguous(), Us, N)   # P_k = dY x_{m<k} U_m^T
        dG = pre[N] if ctx.needs_input_grad[0] else None
        dUs = [None] * N
        for n in range(N):
            if not ctx.needs_input_grad[1 + n]:
                continue
            Z = pre[n]
            for m in range(n + 1, N):
                Z = _ttm(Z, Us[m], m, True)
            dUs[n] = contract_allbut(Z.contiguous(), G.contiguous(), n)
        return (dG, *dUs)
