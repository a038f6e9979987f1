"""GPU parity of two driver options against the FP64 oracle, on the values the GPU holds:

* singular vectors for t-HOSVD-ALS (Section 3, after Algorithm 3.4): each factor column
  against the oracle's SVD of Q^T A_(n) (up to sign; singular values are distinct in these
  inputs), and the core against the oracle's core with the same column signs;
* the automatic st-HOSVD processing order (eq. 2.2, Prop. 1): the order the library picks
  equals the oracle's, and st-HOSVD-ALS in that order matches the oracle run in that order.

Tolerances: a singular vector moves by at most ||dM|| / gap_c under an error dM of the
Gram M = Q^T A_(n) A_(n)^T Q (Davis-Kahan), gap_c the distance of its eigenvalue to the
others.  The device forms M from V = A_(n)^T Q in the storage's compute type, so ||dM|| is
a few roundings of that type times lambda_1: the gate on column c is
1e-5 + 2^-22 lambda_1 / gap_c rad for FP32/BF16 storage and 1e-9 + 2^-50 lambda_1 / gap_c
for FP64, with the eigenvalues from the oracle.  Cores agree within 1e-5 ||A||
(FP32/BF16) and 1e-10 ||A|| (FP64).
"""
import numpy as np
import pytest
import torch

from oracle import tucker_oracle as o
from workloads import synth

pytestmark = pytest.mark.gpu

TDT = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}


def to_gpu(a, dt):
    return torch.from_numpy(np.ascontiguousarray(a)).to(TDT[dt]).cuda().contiguous()


def held(a, dt):
    return to_gpu(a, dt).double().cpu().numpy()


def np64(t):
    return t.detach().double().cpu().numpy()


def flush(msg):
    print(msg, flush=True)


SVEC_CASES = [
    # dims, ranks (= core dims), dtype, core decay; the paths: fused sweep kernel
    # (I <= 256), generic FP64 kernels, chunked large-mode kernels (I = 700), two-pass
    # kernels (I = 1100), a mode with R_n = I_n (the basis is the identity), and R = 20
    # (two rank tiles)
    ((24, 30, 36, 20), (6, 5, 7, 4), "f32", 0.6),
    ((24, 30, 36, 20), (6, 5, 7, 4), "bf16", 0.6),
    ((24, 30, 36, 20), (6, 5, 7, 4), "f64", 0.6),
    ((700, 24, 30), (12, 6, 8), "f32", 0.6),
    ((1100, 24, 20), (10, 6, 8), "f32", 0.6),
    ((8, 30, 40), (8, 5, 6), "f32", 0.6),
    ((40, 50, 30), (20, 17, 3), "bf16", 0.8),
]


@pytest.mark.parametrize("dims,ranks,dt,decay", SVEC_CASES)
def test_singular_vectors_parity(gpu_lib, dims, ranks, dt, decay):
    tk = gpu_lib
    flush(f"singular vectors {dims} {ranks} {dt}")
    rng = np.random.default_rng(50)
    A = synth.tucker_lowrank(rng, dims, ranks, 1e-4, decay=synth.decay_geom(ranks, decay))[0]
    Ah = held(A, dt)
    G, Us, info = tk.als_thosvd(to_gpu(A, dt), ranks, tol=1e-6, seed=3, singular_vectors=True)
    assert info["status"] in ("TK_OK", "TK_NOT_CONVERGED")
    ref = o.thosvd_als(Ah, ranks, tol=1e-6, seed=3, singular_vectors=True)
    nA = o.frob(Ah)
    floor, eps = (1e-9, 2.0 ** -50) if dt == "f64" else (1e-5, 2.0 ** -22)
    g_tol = 1e-10 if dt == "f64" else 1e-5
    Gref = ref.G
    for n, U in enumerate(Us):
        Ug = np64(U)
        R = ranks[n]
        np.testing.assert_allclose(Ug.T @ Ug, np.eye(R), atol=1e-5 if dt != "f64" else 1e-12)
        C = ref.U[n].T @ o.unfold(Ah, n)
        lam = np.sum(C * C, axis=1)          # eigenvalues of M, descending
        gap = np.array([np.min(np.abs(np.delete(lam, c) - lam[c])) if R > 1 else lam[0]
                        for c in range(R)])
        cos = np.sum(Ug * ref.U[n], axis=0)
        sg = np.where(cos < 0, -1.0, 1.0)
        ang = np.linalg.norm(Ug - ref.U[n] * sg, axis=0)
        tol = floor + eps * lam[0] / gap
        flush(f"  mode {n}: max angle {ang.max():.2e}, max angle/tol {np.max(ang / tol):.2e}")
        assert np.all(ang <= tol), (n, ang, tol)
        Gref = o.ttm(Gref, np.diag(sg), n)
    assert np.linalg.norm(np64(G) - Gref) <= g_tol * nA
    # the span is that of the QR basis: same error as without the option
    G0, U0, _ = tk.als_thosvd(to_gpu(A, dt), ranks, tol=1e-6, seed=3)
    e_sv = o.relerr(Ah, np64(G), [np64(u) for u in Us])
    e_qr = o.relerr(Ah, np64(G0), [np64(u) for u in U0])
    assert abs(e_sv - e_qr) <= (1e-12 if dt == "f64" else 1e-6)


def test_singular_vectors_core_all_orthogonal(gpu_lib):
    """On an exactly low-rank FP64 tensor the core of the singular-vector factors is
    all-orthogonal: G_(n) G_(n)^T = diag(sigma^2) of A_(n) (HOSVD property)."""
    tk = gpu_lib
    rng = np.random.default_rng(51)
    dims, ranks = (30, 26, 22), (6, 5, 4)
    A = synth.tucker_lowrank(rng, dims, ranks, 0.0, decay=synth.decay_geom(ranks, 0.6))[0]
    G, Us, info = tk.als_thosvd(to_gpu(A, "f64"), ranks, tol=1e-10, seed=1,
                                singular_vectors=True)
    Gh = np64(G)
    nA2 = o.frob(A) ** 2
    for n in range(3):
        s = np.linalg.svd(o.unfold(A, n), compute_uv=False)[:ranks[n]]
        Gn = o.unfold(Gh, n)
        np.testing.assert_allclose(Gn @ Gn.T, np.diag(s ** 2), atol=1e-10 * nA2)


ORDER_CASES = [
    # dims, ranks, dtype
    ((40, 40, 40), (12, 3, 7), "f32"),
    ((60, 20, 90, 16), (5, 8, 6, 4), "f32"),
    ((120, 24, 30), (6, 10, 12), "bf16"),
]


@pytest.mark.parametrize("dims,ranks,dt", ORDER_CASES)
def test_st_order_auto_parity(gpu_lib, dims, ranks, dt):
    tk = gpu_lib
    flush(f"st order auto {dims} {ranks} {dt}")
    order = o.st_order_auto(dims, ranks)
    assert tk.st_order(dims, ranks) == order
    rng = np.random.default_rng(52)
    A = synth.tucker_lowrank(rng, dims, ranks, 1e-3)[0]
    Ah = held(A, dt)
    G, Us, info = tk.als_sthosvd(to_gpu(A, dt), ranks, tol=1e-6, seed=4, order="auto")
    ref = o.sthosvd_als(Ah, ranks, order=order, tol=1e-6, seed=4)
    e_gpu = o.relerr(Ah, np64(G), [np64(u) for u in Us])
    assert abs(e_gpu - o.relerr(Ah, ref.G, ref.U)) <= 1e-5
    for n in range(len(dims)):
        assert np.max(o.principal_angles(np64(Us[n]), ref.U[n])) < 1e-3
