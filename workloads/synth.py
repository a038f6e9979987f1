"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws random numbers and assembles test tensors; it computes
none of the decomposition's results and holds no expected values.  Both the
CPU oracle tests and the GPU path take their inputs from here.

Recipe (noise is relative: the noise tensor E is rescaled so that
||E||_F = rho * ||A0||_F exactly):

* ``tucker_lowrank``: core of the given dims with i.i.d. N(0,1) entries times
  an optional per-entry decay, factors U_n = Q of the QR of an I_n x R_n
  Gaussian matrix, A = A0 + E.  Low multilinear rank signal plus noise, as in
  the Tucker-model experiment of Section 6.1.2 (where the core is U[5,10] and
  the noise absolute).
* ``cp_lowrank``: the CP-model experiment of Section 6.1.1, lambda_r in
  U[5,10] and unit-norm random vectors, plus relative noise.

* ``cp_paper`` / ``tucker_paper`` (and their ``_torch`` device versions): the
  two experiments of Section 6.1 as the paper states them: A_hat = A + delta E
  with E i.i.d. N(0,1) and ABSOLUTE noise level delta = 1e-4; the CP model of
  Section 6.1.1 on I x I x 100I with R = 0.2 I terms, lambda_r ~ U[5,10] and
  unit-norm Gaussian vectors; the Tucker model of Section 6.1.2 on
  I x 100 x 100 x 100 with core (0.01 I, 10, 10, 10) ~ U[5,10] and orthonormal
  factors.  Both return (A_hat, A): the paper measures errors against the
  noise-free A.

Seeds: ``2004025830 + k`` for the k-th named workload.
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 2004025830


def rng_for(k: int) -> np.random.Generator:
    return np.random.default_rng(SEED_BASE + k)


def orthonormal(rng: np.random.Generator, n: int, r: int) -> np.ndarray:
    """Q factor of the QR decomposition of an n x r standard Gaussian."""
    q, _ = np.linalg.qr(rng.standard_normal((n, r)))
    return q


def _mode_product(X: np.ndarray, U: np.ndarray, n: int) -> np.ndarray:
    # generator-side assembly of the synthetic signal (tensordot over mode n)
    Y = np.tensordot(U, X, axes=([1], [n]))
    return np.moveaxis(Y, 0, n)


def decay_exp(shape, scale: float) -> np.ndarray:
    """Per-entry factor exp(-(i1+...+iN)/scale), 0-based indices."""
    idx = np.indices(shape).sum(axis=0)
    return np.exp(-idx / scale)


def decay_geom(shape, ratio: float) -> np.ndarray:
    """Per-entry factor ratio^(i1+...+iN), 0-based indices."""
    idx = np.indices(shape).sum(axis=0)
    return ratio ** idx


def tucker_lowrank(rng: np.random.Generator, dims, core_dims, noise_rel: float,
                   decay: np.ndarray | None = None):
    """A = G x_1 U_1 ... x_N U_N + E with ||E|| = noise_rel ||A0||.

    Returns (A, A0, G, Us) in float64."""
    G = rng.standard_normal(tuple(core_dims))
    if decay is not None:
        G = G * decay
    Us = [orthonormal(rng, d, r) for d, r in zip(dims, core_dims)]
    A0 = G
    for n, U in enumerate(Us):
        A0 = _mode_product(A0, U, n)
    A = A0.copy()
    if noise_rel > 0:
        E = rng.standard_normal(A0.shape)
        E *= noise_rel * np.linalg.norm(A0.ravel()) / np.linalg.norm(E.ravel())
        A = A0 + E
    return A, A0, G, Us


def cp_lowrank(rng: np.random.Generator, dims, rank: int, noise_rel: float):
    """Sum of ``rank`` rank-one terms lambda_r a_r o b_r o c_r (Section 6.1.1)
    with lambda_r ~ U[5,10] and unit-norm Gaussian vectors, plus noise."""
    lam = rng.uniform(5.0, 10.0, size=rank)
    vecs = []
    for d in dims:
        V = rng.standard_normal((d, rank))
        vecs.append(V / np.linalg.norm(V, axis=0, keepdims=True))
    A0 = np.zeros(tuple(dims))
    for r in range(rank):
        t = lam[r]
        for n, V in enumerate(vecs):
            shp = [1] * len(dims)
            shp[n] = dims[n]
            t = t * V[:, r].reshape(shp)
        A0 = A0 + t
    A = A0.copy()
    if noise_rel > 0:
        E = rng.standard_normal(A0.shape)
        E *= noise_rel * np.linalg.norm(A0.ravel()) / np.linalg.norm(E.ravel())
        A = A0 + E
    return A, A0


def _cp_terms(rng, dims, rank):
    lam = rng.uniform(5.0, 10.0, size=rank)
    vecs = []
    for d in dims:
        V = rng.standard_normal((d, rank))
        vecs.append(V / np.linalg.norm(V, axis=0, keepdims=True))
    return lam, vecs


def cp_paper(rng: np.random.Generator, I: int, rank: int | None = None, delta: float = 1e-4,
             K: int | None = None):
    """Section 6.1.1: dims (I, I, K = 100 I), R = 0.2 I rank-one terms, absolute noise
    delta * N(0,1).  Returns (A_hat, A) in float64."""
    R = rank if rank is not None else max(1, int(round(0.2 * I)))
    dims = (I, I, K if K is not None else 100 * I)
    lam, (a, b, c) = _cp_terms(rng, dims, R)
    A = np.einsum("r,ir,jr,kr->ijk", lam, a, b, c, optimize=True)
    return A + delta * rng.standard_normal(dims), A


def tucker_paper(rng: np.random.Generator, I: int, J: int = 100, delta: float = 1e-4,
                 R1: int | None = None, R: int = 10):
    """Section 6.1.2: dims (I, J, J, J) with J = 100, core (R1 = 0.01 I, R, R, R) with
    U[5,10] entries, orthonormal factors, absolute noise delta * N(0,1).
    Returns (A_hat, A) in float64."""
    core = (R1 if R1 is not None else max(1, int(round(0.01 * I))), R, R, R)
    dims = (I, J, J, J)
    G = rng.uniform(5.0, 10.0, size=core)
    A = G
    for n in range(4):
        A = _mode_product(A, orthonormal(rng, dims[n], core[n]), n)
    return A + delta * rng.standard_normal(dims), A


def gaussian(rng: np.random.Generator, dims) -> np.ndarray:
    return rng.standard_normal(tuple(dims))


# ---------------------------------------------------------------------------
# The five named workloads (small and full sizes)
# ---------------------------------------------------------------------------

def workload_small_fp64(k: int = 0):
    """64x64x64, core 8^3 N(0,1), orthonormal 64x8 factors, 1e-3 relative
    noise; ranks (8,8,8); tol 1e-8; float64."""
    rng = rng_for(k)
    A, A0, G, Us = tucker_lowrank(rng, (64, 64, 64), (8, 8, 8), 1e-3)
    return dict(A=A, A0=A0, ranks=(8, 8, 8), tol=1e-8)


def workload_4way(dims=(200, 200, 200, 200), R=20, noise_rel=1e-4, k: int = 1):
    """Core R^4 with entries N(0,1) exp(-(i+j+k+l)/10), orthonormal I_n x R
    factors, relative noise 1e-4 (4th-order decaying-core workload)."""
    rng = rng_for(k)
    core = (R,) * 4
    A, A0, G, Us = tucker_lowrank(rng, dims, core, noise_rel,
                                  decay=decay_exp(core, 10.0))
    return dict(A=A, A0=A0, ranks=(R,) * 4)


def workload_cube_geom(I=1024, C=64, R=48, noise_rel=1e-3, k: int = 2):
    """Core C^3 with entries N(0,1) 0.9^(i+j+k), orthonormal I x C factors,
    relative noise 1e-3; target ranks (R,R,R)."""
    rng = rng_for(k)
    core = (C,) * 3
    A, A0, G, Us = tucker_lowrank(rng, (I,) * 3, core, noise_rel,
                                  decay=decay_geom(core, 0.9))
    return dict(A=A, A0=A0, ranks=(R,) * 3)


def workload_autograd(I=256, R=32, k: int = 3):
    """A i.i.d. N(0,1) of size I^3 and orthonormal I x R factors."""
    rng = rng_for(k)
    A = gaussian(rng, (I,) * 3)
    Us = [orthonormal(rng, I, R) for _ in range(3)]
    return dict(A=A, U=Us)


def workload_batched(count=512, lo=16, hi=128, rlo=4, rhi=16, noise_rel=1e-3,
                     k: int = 4):
    """``count`` 3rd-order tensors with I_n ~ U{lo..hi} and R_n ~ U{rlo..rhi}
    per mode, N(0,1) core of dims R_n times orthonormal factors plus 1e-3
    relative noise.  Ranks are capped so each is a realisable multilinear
    rank (R_n <= prod of the other two)."""
    rng = rng_for(k)
    items = []
    for _ in range(count):
        dims = tuple(int(x) for x in rng.integers(lo, hi + 1, size=3))
        ranks = [int(x) for x in rng.integers(rlo, rhi + 1, size=3)]
        for n in range(3):
            others = ranks[(n + 1) % 3] * ranks[(n + 2) % 3]
            ranks[n] = min(ranks[n], others, dims[n])
        A, _, _, _ = tucker_lowrank(rng, dims, tuple(ranks), noise_rel)
        items.append(dict(A=A, ranks=tuple(ranks)))
    return items


# ---------------------------------------------------------------------------
# Device-side generation of the large workloads (same recipe, drawn with
# torch on the GPU so multi-GB tensors never pass through the host).

def tucker_lowrank_torch(k: int, dims, core_dims, noise_rel: float, decay=None,
                         device="cuda", out_dtype=None):
    """Core (numpy, seeded with rng_for(k)) times orthonormal factors plus
    relative Gaussian noise drawn on ``device`` (torch generator seeded with
    SEED_BASE + k), assembled in float64 and returned as ``out_dtype``
    (default float64).  Returns (A, core, factors)."""
    import torch
    rng = rng_for(k)
    G = rng.standard_normal(tuple(core_dims))
    if decay is not None:
        G = G * decay
    Us = [orthonormal(rng, d, r) for d, r in zip(dims, core_dims)]
    X = torch.from_numpy(G).to(device)
    for n, U in enumerate(Us):
        Ut = torch.from_numpy(U).to(device)
        X = torch.movedim(torch.tensordot(Ut, X, dims=([1], [n])), 0, n).contiguous()
    gen = torch.Generator(device=device)
    gen.manual_seed(SEED_BASE + k)
    nrm0 = torch.linalg.vector_norm(X).item()
    E = torch.randn(X.shape, generator=gen, device=device, dtype=torch.float64)
    E *= noise_rel * nrm0 / torch.linalg.vector_norm(E).item()
    X += E
    del E
    if out_dtype is not None:
        X = X.to(out_dtype)
    return X, G, Us


def cp_paper_torch(k: int, I: int, delta: float = 1e-4, device="cuda", out_dtype=None):
    """``cp_paper`` at full size on the device: terms drawn with numpy (rng_for(k)),
    assembled and noised (torch generator seeded SEED_BASE + k) in float64 on ``device``.
    Returns (A_hat, A) as ``out_dtype`` / float64."""
    import torch
    rng = rng_for(k)
    R = max(1, int(round(0.2 * I)))
    dims = (I, I, 100 * I)
    lam, (a, b, c) = _cp_terms(rng, dims, R)
    at, bt, ct = (torch.from_numpy(x).to(device) for x in (a * lam, b, c))
    A = torch.einsum("ir,jr,kr->ijk", at, bt, ct).contiguous()
    gen = torch.Generator(device=device)
    gen.manual_seed(SEED_BASE + k)
    Ah = A + delta * torch.randn(dims, generator=gen, device=device, dtype=torch.float64)
    if out_dtype is not None:
        Ah = Ah.to(out_dtype)
    return Ah, A


def tucker_paper_torch(k: int, I: int, delta: float = 1e-4, device="cuda", out_dtype=None):
    """``tucker_paper`` at full size on the device; the noise-free tensor is returned in
    ``out_dtype`` too (float64 would double the memory at I = 5000).
    Returns (A_hat, A, core, factors)."""
    import torch
    rng = rng_for(k)
    core = (max(1, int(round(0.01 * I))), 10, 10, 10)
    dims = (I, 100, 100, 100)
    G = rng.uniform(5.0, 10.0, size=core)
    Us = [orthonormal(rng, d, r) for d, r in zip(dims, core)]
    X = torch.from_numpy(G).to(device)
    for n in range(1, 4):
        Ut = torch.from_numpy(Us[n]).to(device)
        X = torch.movedim(torch.tensordot(Ut, X, dims=([1], [n])), 0, n).contiguous()
    # the largest mode last, in slabs, so float64 never holds the whole tensor twice
    odt = out_dtype if out_dtype is not None else torch.float64
    A = torch.empty(dims, dtype=odt, device=device)
    Ah = torch.empty(dims, dtype=odt, device=device)
    U0 = torch.from_numpy(Us[0]).to(device)
    gen = torch.Generator(device=device)
    gen.manual_seed(SEED_BASE + k)
    Xf = X.reshape(core[0], -1)
    for s in range(0, I, 256):
        e = min(I, s + 256)
        slab = (U0[s:e] @ Xf).reshape((e - s,) + dims[1:])
        A[s:e] = slab.to(odt)
        Ah[s:e] = (slab + delta * torch.randn(slab.shape, generator=gen, device=device,
                                              dtype=torch.float64)).to(odt)
        del slab
    return Ah, A, G, Us


def workload_4way_torch(dims=(200, 200, 200, 200), R=20, noise_rel=1e-4, device="cuda"):
    """The 4th-order decaying-core workload generated on the device (FP32)."""
    import torch
    core = (R,) * 4
    A, _, Us = tucker_lowrank_torch(1, dims, core, noise_rel, decay=decay_exp(core, 10.0),
                                    device=device, out_dtype=torch.float32)
    return dict(A=A, ranks=(R,) * 4, factors=Us)
