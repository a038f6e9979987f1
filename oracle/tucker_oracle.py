"""Plain FP64 CPU oracle for ALS-based truncated HOSVD.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  The product path
(the HIP library and its Python binding) never calls it and shares no code,
tables or helpers with it.

Source: Xiao, Yang & Li, "Efficient Alternating Least Squares Algorithms for
Low Multilinear Rank Approximation of Tensors" (arXiv 2004.02583).  Every
function names the passage it follows.  The arithmetic is NumPy/SciPy in
float64, written to be checked against the paper by eye: no blocking, no
fusion, no reordering beyond what the cited definition or algorithm states.

Readings of places where the paper is silent or ambiguous (each is also listed
in the design notes of the repository):

* Unfolding column order: C order over the remaining modes instead of the
  paper's column-major index formula (Section 2).  Left singular subspaces,
  factors, core and reconstruction do not depend on the column order; only the
  row order of the right ALS factor does.  ``unfold_paper`` implements the
  paper's own formula so a test can check the equivalence.
* The random matrix S of the initial guess (Section 5, item 1) has J x R_n
  entries with no oversampling, drawn from the counter-based SplitMix64
  generator in ``splitmix_uniform``; j is the C-order column index.
* The stop test (eq. E5.01) is evaluated after each R-update, first at k = 1,
  against the Frobenius norm of the ORIGINAL input tensor for every mode, and
  Algorithm 3.3 returns (L_k, R_k) with R_k the least-squares solution for L_k.
  k counts L-updates; after ``max_iters`` L-updates without convergence the
  result is returned with ``converged=False``.
* Residuals are computed by explicit difference (slow by design).
* R_n == I_n: the dominant subspace is the whole space; U_n = identity with
  zero iterations.
* A Gram matrix whose Cholesky factor has a squared pivot at or below
  1e-13 times the Gram's largest diagonal entry (or that fails Cholesky)
  means R_n exceeds the numerical rank (Remark 3): ``RankDeficient`` is
  raised, no regularisation.
* QR sign convention: diag(R_hat) >= 0.
* Singular vectors for t-HOSVD-ALS (the optional replacement of the factor
  step of Algorithm 3.4, Section 3): columns in descending order of the
  singular values of Q_hat^T A_(n); each column of the small left factor U is
  signed so that its entry of largest magnitude is positive.
* st-HOSVD processing order: the automatic order is the permutation of least
  cost under eq. 2.2 (Prop. 1) over all N! orders, the first in lexicographic
  order among equal costs.
"""
from __future__ import annotations

import dataclasses
import itertools
import numpy as np
import scipy.linalg as sla

# --------------------------------------------------------------------------
# Section 2: tensor primitives
# --------------------------------------------------------------------------


def frob(A: np.ndarray) -> float:
    """Frobenius norm (Section 2): sqrt of the sum of squared entries."""
    A = np.asarray(A, dtype=np.float64)
    return float(np.sqrt(np.sum(A * A)))


def unfold(A: np.ndarray, n: int) -> np.ndarray:
    """Mode-n matricization A_(n), I_n x prod_{k!=n} I_k (Section 2).

    Columns are ordered in C order over the remaining modes (reading above).
    """
    return np.moveaxis(np.asarray(A), n, 0).reshape(A.shape[n], -1)


def fold(M: np.ndarray, n: int, shape) -> np.ndarray:
    """Inverse of ``unfold``: put the rows of M back as mode n of ``shape``."""
    shape = list(shape)
    moved = [shape[n]] + shape[:n] + shape[n + 1:]
    return np.moveaxis(M.reshape(moved), 0, n)


def unfold_paper(A: np.ndarray, n: int) -> np.ndarray:
    """Mode-n matricization with the paper's column-major column index
    j = sum_{k != n} i_k J_k, J_k = prod_{m<k, m!=n} I_m (Section 2, 0-based).

    Written as an explicit loop over entries; only for tiny tensors.
    """
    A = np.asarray(A)
    dims = A.shape
    cols = int(np.prod([d for k, d in enumerate(dims) if k != n]))
    out = np.zeros((dims[n], cols), dtype=A.dtype)
    for idx in np.ndindex(*dims):
        j = 0
        stride = 1
        for k in range(len(dims)):
            if k == n:
                continue
            j += idx[k] * stride
            stride *= dims[k]
        out[idx[n], j] = A[idx]
    return out


def ttm(A: np.ndarray, M: np.ndarray, n: int) -> np.ndarray:
    """Mode-n product A x_n M with M of shape J x I_n (Section 2):
    (A x_n M)_{..j..} = sum_{i_n} A_{..i_n..} M_{j, i_n}."""
    A = np.asarray(A, dtype=np.float64)
    M = np.asarray(M, dtype=np.float64)
    shape = list(A.shape)
    shape[n] = M.shape[0]
    return fold(M @ unfold(A, n), n, shape)


def tucker_to_tensor(G: np.ndarray, Us) -> np.ndarray:
    """Tucker format G x_1 U^(1) x_2 ... x_N U^(N) (Section 2)."""
    X = np.asarray(G, dtype=np.float64)
    for n, U in enumerate(Us):
        X = ttm(X, U, n)
    return X


def core_from_factors(A: np.ndarray, Us) -> np.ndarray:
    """Optimal core for given orthonormal factors (Section 2, eq. best):
    G = A x_1 U^(1)T ... x_N U^(N)T."""
    X = np.asarray(A, dtype=np.float64)
    for n, U in enumerate(Us):
        X = ttm(X, np.asarray(U).T, n)
    return X


def relerr(A: np.ndarray, G: np.ndarray, Us) -> float:
    """||A - G x U|| / ||A|| computed by explicit difference (never through
    1 - ||G||^2/||A||^2, which cancels)."""
    A = np.asarray(A, dtype=np.float64)
    return frob(A - tucker_to_tensor(G, Us)) / frob(A)


# --------------------------------------------------------------------------
# Reduced QR with the sign convention diag(R_hat) >= 0 (Algorithms 3.4/3.5)
# --------------------------------------------------------------------------


def qr_signfix(L: np.ndarray):
    """Reduced QR of L; column signs flipped so that diag(R_hat) >= 0."""
    Q, R = np.linalg.qr(np.asarray(L, dtype=np.float64), mode="reduced")
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s[None, :], R * s[:, None]


# --------------------------------------------------------------------------
# Section 5, initial guess: the random matrix S
# --------------------------------------------------------------------------

_MASK = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15


def splitmix64(state: int) -> int:
    """One SplitMix64 output for the given 64-bit state value (Steele, Lea and
    Flood, OOPSLA 2014): the state is first advanced by the golden-ratio
    increment, then passed through the variant-13 finaliser."""
    z = (state + _GAMMA) & _MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
    return z ^ (z >> 31)


def splitmix_stream(seed: int, count: int):
    """The first ``count`` outputs of a SplitMix64 generator seeded with
    ``seed`` (the k-th output uses state seed + k * gamma)."""
    out = []
    s = seed & _MASK
    for _ in range(count):
        out.append(splitmix64(s))
        s = (s + _GAMMA) & _MASK
    return out


def splitmix_uniform(seed: int, counter: np.ndarray) -> np.ndarray:
    """Uniform [0,1) values at the given 64-bit counters: the counter-th
    SplitMix64 output of the stream seeded with ``seed``, top 24 bits times
    2^-24 (exact in float32 and float64)."""
    c = np.asarray(counter, dtype=np.uint64)
    with np.errstate(over="ignore"):
        state = np.uint64(seed & _MASK) + c * np.uint64(_GAMMA)
        z = state + np.uint64(_GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(40)).astype(np.float64) * (2.0 ** -24)


def init_sketch(seed: int, mode: int, J: int, R: int) -> np.ndarray:
    """S in R^{J x R} with entries U[0,1) (Section 5, item 1).

    Entry (j, r) of the sketch for mode ``mode`` (0-based) uses counter
    mode * 2^48 + j * R + r.
    """
    j = np.arange(J, dtype=np.uint64)[:, None]
    r = np.arange(R, dtype=np.uint64)[None, :]
    counter = np.uint64(mode) * np.uint64(1 << 48) + j * np.uint64(R) + r
    return splitmix_uniform(seed, counter)


# --------------------------------------------------------------------------
# Algorithm 3.3: ALS for the matrix low-rank problem
# --------------------------------------------------------------------------


class RankDeficient(np.linalg.LinAlgError):
    """A Gram matrix L^T L or R^T R is not positive definite in float64:
    the truncation exceeds the numerical rank (Remark 3)."""


# A Gram whose smallest Cholesky pivot (squared diagonal entry of the factor)
# falls to PIVOT_TOL times its largest diagonal entry or below is treated as
# singular: Remark 3's "close to singular" made concrete.
PIVOT_TOL = 1e-13


def _chol_solve(Gram: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Solve Gram X = B for symmetric positive definite Gram (Remark 2)."""
    Gram = np.asarray(Gram, dtype=np.float64)
    try:
        C = np.linalg.cholesky(Gram)
    except np.linalg.LinAlgError as e:  # not positive definite
        raise RankDeficient(str(e)) from None
    piv = np.diag(C) ** 2
    if not np.all(np.isfinite(piv)) or piv.min() <= PIVOT_TOL * np.max(np.diag(Gram)):
        raise RankDeficient("Gram matrix numerically singular")
    Y = sla.solve_triangular(C, B, lower=True)
    return sla.solve_triangular(C.T, Y, lower=False)


@dataclasses.dataclass
class ALSResult:
    L: np.ndarray          # L_k, m x r
    R: np.ndarray          # R_k, n x r, least-squares solution for L_k
    iters: int             # k = number of L-updates performed
    converged: bool
    residuals: list        # res_0 .. res_k, explicit ||A - L_j R_j^T||_F


def als_r_update(A: np.ndarray, L: np.ndarray) -> np.ndarray:
    """Algorithm 3.3, R-update: R = (A^T L)(L^T L)^{-1}."""
    return _chol_solve(L.T @ L, L.T @ A).T


def als_l_update(A: np.ndarray, R: np.ndarray) -> np.ndarray:
    """Algorithm 3.3, L-update: L = (A R)(R^T R)^{-1}."""
    return _chol_solve(R.T @ R, R.T @ A.T).T


def als(A: np.ndarray, r: int, L0: np.ndarray, tol: float, max_iters: int,
        norm_ref: float) -> ALSResult:
    """Algorithm 3.3 with the stop criterion of eq. E5.01.

    ``norm_ref`` is ||A||_F of the original input tensor (right-hand side of
    E5.01).  R_k is computed from L_k; res_k = ||A - L_k R_k^T||_F by explicit
    difference; for k >= 1 the iteration returns (L_k, R_k) when
    |res_{k-1} - res_k| <= tol * norm_ref.
    """
    A = np.asarray(A, dtype=np.float64)
    L = np.asarray(L0, dtype=np.float64)
    R = als_r_update(A, L)
    res = [frob(A - L @ R.T)]
    k = 0
    while True:
        if k >= 1 and abs(res[-2] - res[-1]) <= tol * norm_ref:
            return ALSResult(L, R, k, True, res)
        if k >= max_iters:
            return ALSResult(L, R, k, False, res)
        L = als_l_update(A, R)
        k += 1
        R = als_r_update(A, L)
        res.append(frob(A - L @ R.T))


def als_initial_guess(A: np.ndarray, S: np.ndarray) -> np.ndarray:
    """Section 5, items 2-3: L_0 = Q of the reduced QR of A S."""
    Q, _ = qr_signfix(np.asarray(A, dtype=np.float64) @ S)
    return Q


# --------------------------------------------------------------------------
# Algorithms 3.4 and 3.5: t-HOSVD-ALS and st-HOSVD-ALS
# --------------------------------------------------------------------------


@dataclasses.dataclass
class ModeInfo:
    iters: int
    converged: bool
    residuals: list       # ALS residual history for this mode
    resid: float          # final ALS residual ||B_(n) - L R^T||_F


@dataclasses.dataclass
class TuckerResult:
    G: np.ndarray
    U: list
    info: list            # ModeInfo per mode, indexed by the original mode
    norm_a: float


def _mode_factor(Bn: np.ndarray, R: int, seed: int, mode: int, tol: float,
                 max_iters: int, norm_ref: float, L0=None):
    """One mode of Algorithms 3.4/3.5: ALS on B_(n), then reduced QR of L.
    ``L0`` is Algorithm 3.3's initial guess when given (a warm start); the
    Section 5 sketch otherwise.

    Returns (U_n, R_hat, R_k, ModeInfo)."""
    In, J = Bn.shape
    if R == In:
        # Whole space: any orthonormal basis is exact (reading above).
        U = np.eye(In)
        resid = 0.0
        return U, np.eye(In), Bn.T.copy(), ModeInfo(0, True, [resid], resid)
    if L0 is None:
        S = init_sketch(seed, mode, J, R)
        L0 = als_initial_guess(Bn, S)
    res = als(Bn, R, L0, tol, max_iters, norm_ref)
    Q, Rhat = qr_signfix(res.L)
    return Q, Rhat, res.R, ModeInfo(res.iters, res.converged, res.residuals,
                                    res.residuals[-1])


def singular_vectors_from_basis(An: np.ndarray, Q: np.ndarray):
    """Singular vectors from an orthonormal basis Q of the dominant subspace
    (Section 3, after Algorithm 3.4): the SVD U S V^T of C = Q^T A_(n), then
    Q U.  Singular values come out in descending order; each column of U is
    signed so that its entry of largest magnitude is positive (reading above).
    Returns (Q U, singular values of C)."""
    C = Q.T @ An
    U, s, _ = np.linalg.svd(C, full_matrices=False)
    cols = np.arange(U.shape[1])
    U = U * np.sign(U[np.argmax(np.abs(U), axis=0), cols])
    return Q @ U, s


def thosvd_als(A: np.ndarray, ranks, tol: float = 1e-4, max_iters: int = 50,
               seed: int = 0, singular_vectors: bool = False,
               init=None) -> TuckerResult:
    """Algorithm 3.4 (t-HOSVD-ALS): per mode, ALS on A_(n), U^(n) = Q of the
    reduced QR of L; then G = A x_1 U^(1)T ... x_N U^(N)T.  With
    ``singular_vectors`` the factor step is replaced by the singular vectors
    of A_(n) within that basis (``singular_vectors_from_basis``).  ``init``:
    None, or per mode an I_n x R_n initial guess L_0 of Algorithm 3.3 (or
    None for the Section 5 sketch)."""
    A = np.asarray(A, dtype=np.float64)
    nA = frob(A)
    Us, infos = [], []
    for n in range(A.ndim):
        L0 = None if init is None else init[n]
        U, _, _, info = _mode_factor(unfold(A, n), ranks[n], seed, n, tol,
                                     max_iters, nA, L0)
        if singular_vectors:
            U, _ = singular_vectors_from_basis(unfold(A, n), U)
        Us.append(U)
        infos.append(info)
    G = core_from_factors(A, Us)
    return TuckerResult(G, Us, infos, nA)


def sthosvd_als(A: np.ndarray, ranks, order=None, tol: float = 1e-4,
                max_iters: int = 50, seed: int = 0,
                check_identity: bool = True, init=None) -> TuckerResult:
    """Algorithm 3.5 (st-HOSVD-ALS) with the literal truncation
    B_(n) <- R_hat R^T.

    With ``check_identity`` the literal truncation is compared with the
    mode-n product B x_n U^(n)T; the two agree because R is the
    least-squares solution for the very L that was QR-factorised.
    ``init`` as for ``thosvd_als`` (L_0 of mode n has I_n rows whatever the
    truncation of the other modes).
    """
    A = np.asarray(A, dtype=np.float64)
    N = A.ndim
    order = list(range(N)) if order is None else list(order)
    nA = frob(A)
    B = A.copy()
    Us = [None] * N
    infos = [None] * N
    for n in order:
        Bn = unfold(B, n)
        L0 = None if init is None else init[n]
        U, Rhat, Rk, info = _mode_factor(Bn, ranks[n], seed, n, tol,
                                         max_iters, nA, L0)
        newshape = list(B.shape)
        newshape[n] = ranks[n]
        Bnew = fold(Rhat @ Rk.T, n, newshape)
        if check_identity:
            Bttm = ttm(B, U.T, n)
            scale = max(frob(Bttm), 1e-300)
            d = frob(Bnew - Bttm) / scale
            if d > 1e-10:
                raise AssertionError(f"R_hat R^T differs from B x_n U^T: {d}")
        B = Bnew
        Us[n] = U
        infos[n] = info
    return TuckerResult(B, Us, infos, nA)


def st_order_cost(dims, ranks, order) -> int:
    """Cost model of eq. 2.2 (proof of Prop. 1) for processing the modes of
    st-HOSVD in ``order`` = (i_1, ..., i_N): the sum over n of
    R_{i_1} ... R_{i_n} times I_{i_n} ... I_{i_N}, in exact integers."""
    order = list(order)
    total = 0
    for n in range(len(order)):
        r = 1
        for k in order[:n + 1]:
            r *= int(ranks[k])
        i = 1
        for k in order[n:]:
            i *= int(dims[k])
        total += r * i
    return total


def st_order_auto(dims, ranks) -> list:
    """The st-HOSVD processing order of least eq. 2.2 cost over all N!
    permutations, the first in lexicographic order among equal costs (reading
    above).  With equal dimensions this is the order of ascending ranks
    (Prop. 1)."""
    best, best_cost = None, None
    for perm in itertools.permutations(range(len(dims))):
        c = st_order_cost(dims, ranks, perm)
        if best_cost is None or c < best_cost:
            best, best_cost = list(perm), c
    return best


# --------------------------------------------------------------------------
# Algorithms 3.1 and 3.2: SVD/EIG-based t-HOSVD and st-HOSVD (comparison)
# --------------------------------------------------------------------------


def leading_left_singular_vectors(M: np.ndarray, R: int,
                                  method: str = "auto") -> np.ndarray:
    """Leading R left singular vectors of M (the SVD step of Algorithm 3.1).  The EIG
    route uses eigenvectors of the Gram M M^T (the remark after Alg. 3.1)."""
    M = np.asarray(M, dtype=np.float64)
    if method == "auto":
        method = "svd" if M.size <= (1 << 26) else "eig"
    if method == "svd":
        U, _, _ = np.linalg.svd(M, full_matrices=False)
        return U[:, :R]
    w, V = np.linalg.eigh(M @ M.T)
    return V[:, np.argsort(w)[::-1][:R]]


def singular_values(M: np.ndarray) -> np.ndarray:
    M = np.asarray(M, dtype=np.float64)
    if M.size <= (1 << 26):
        return np.linalg.svd(M, compute_uv=False)
    w = np.linalg.eigvalsh(M @ M.T)[::-1]
    return np.sqrt(np.clip(w, 0.0, None))


def thosvd_svd(A: np.ndarray, ranks, method: str = "auto") -> TuckerResult:
    """Algorithm 3.1 (t-HOSVD)."""
    A = np.asarray(A, dtype=np.float64)
    Us = [leading_left_singular_vectors(unfold(A, n), ranks[n], method)
          for n in range(A.ndim)]
    return TuckerResult(core_from_factors(A, Us), Us, [], frob(A))


def sthosvd_svd(A: np.ndarray, ranks, order=None, method: str = "auto"):
    """Algorithm 3.2 (st-HOSVD), truncation B <- B x_n U^(n)T.

    Returns (TuckerResult, discarded) where discarded[n] is the sum of the
    squared singular values of B_(n) beyond R_n at the time mode n is
    processed."""
    A = np.asarray(A, dtype=np.float64)
    N = A.ndim
    order = list(range(N)) if order is None else list(order)
    B = A.copy()
    Us = [None] * N
    disc = [0.0] * N
    for n in order:
        Bn = unfold(B, n)
        s = singular_values(Bn)
        disc[n] = float(np.sum(s[ranks[n]:] ** 2))
        U = leading_left_singular_vectors(Bn, ranks[n], method)
        B = ttm(B, U.T, n)
        Us[n] = U
    return TuckerResult(B, Us, [], frob(A)), disc


def hooi(A: np.ndarray, Us0, tol: float = 1e-12, max_iters: int = 50):
    """HOOI, the higher-order orthogonal iteration (De Lathauwer, De Moor and
    Vandewalle 2000; the refinement the paper runs from t-/st-HOSVD results,
    Section 6.3, Table 6.3-2), from the orthonormal factors Us0.  One outer
    iteration sets, for n = 0..N-1 in turn, U_n to the leading R_n left
    singular vectors of Y_(n) with Y = A x_{k != n} U_k^T; then
    G = A x_1 U_1^T ... x_N U_N^T and e = ||A - A_hat|| / ||A|| (explicit
    reconstruction).  Stops when |e_prev - e| <= tol.
    Returns (G, Us, errors, converged); errors[0] is the error of Us0."""
    A = np.asarray(A, dtype=np.float64)
    N = A.ndim
    Us = [np.array(U, dtype=np.float64) for U in Us0]
    G = core_from_factors(A, Us)
    errs = [relerr(A, G, Us)]
    converged = max_iters == 0
    for _ in range(max_iters):
        for n in range(N):
            Y = A
            for k in range(N):
                if k != n:
                    Y = ttm(Y, Us[k].T, k)
            Us[n] = leading_left_singular_vectors(unfold(Y, n), Us[n].shape[1])
        G = core_from_factors(A, Us)
        errs.append(relerr(A, G, Us))
        if abs(errs[-2] - errs[-1]) <= tol:
            converged = True
            break
    return G, Us, errs, converged


def tail_energies(A: np.ndarray, ranks):
    """gamma_n = sum_{r > R_n} sigma_r(A_(n))^2 (Lemma 2, eq. E5.1)."""
    return [float(np.sum(singular_values(unfold(A, n))[ranks[n]:] ** 2))
            for n in range(np.ndim(A))]


def principal_angles(U1: np.ndarray, U2: np.ndarray) -> np.ndarray:
    """Principal angles (radians) between the column spaces of U1 and U2."""
    Q1, _ = np.linalg.qr(U1)
    Q2, _ = np.linalg.qr(U2)
    # Bjorck-Golub: cosines from Q1^T Q2, sines from the part of Q2 outside
    # span(Q1); small angles are taken from the sines (accurate near 0).
    c = np.linalg.svd(Q1.T @ Q2, compute_uv=False)               # descending
    s = np.linalg.svd(Q2 - Q1 @ (Q1.T @ Q2), compute_uv=False)[::-1]
    k = min(len(c), len(s))
    c, s = np.clip(c[:k], 0.0, 1.0), np.clip(s[:k], 0.0, 1.0)
    return np.where(c > np.sqrt(0.5), np.arcsin(s), np.arccos(c))


def subspace_distance(U1: np.ndarray, U2: np.ndarray) -> float:
    """sin of the largest principal angle = ||U1 U1^T - U2 U2^T||_2 for
    orthonormal bases of equal dimension."""
    return float(np.sin(np.max(principal_angles(U1, U2))))


# --------------------------------------------------------------------------
# Gradients of the Tucker projection / reconstruction chain
# --------------------------------------------------------------------------


def project(A: np.ndarray, Us) -> np.ndarray:
    """G = A x_1 U_1^T ... x_N U_N^T (eq. best)."""
    return core_from_factors(A, Us)


def project_vjp(A: np.ndarray, Us, dG: np.ndarray):
    """Adjoint of G = A x_1 U_1^T ... x_N U_N^T for cotangent dG.

    For Y = X x_n M: dX = dY x_n M^T and dM = dY_(n) X_(n)^T.  With
    M = U_n^T this gives dU_n = X_(n) dG_(n)^T where X is A projected on
    every mode except n, and dA = dG x_1 U_1 ... x_N U_N.
    """
    A = np.asarray(A, dtype=np.float64)
    N = A.ndim
    dA = tucker_to_tensor(dG, Us)
    dUs = []
    for n in range(N):
        X = A
        for m in range(N):
            if m != n:
                X = ttm(X, np.asarray(Us[m]).T, m)
        dUs.append(unfold(X, n) @ unfold(dG, n).T)
    return dA, dUs


def reconstruct_vjp(G: np.ndarray, Us, dY: np.ndarray):
    """Adjoint of Y = G x_1 U_1 ... x_N U_N for cotangent dY.

    dG = dY x_1 U_1^T ... x_N U_N^T and dU_n = Z_(n) G_(n)^T, where Z is dY
    projected by U_m^T on every mode m != n.
    """
    G = np.asarray(G, dtype=np.float64)
    N = G.ndim
    dG = core_from_factors(dY, Us)
    dUs = []
    for n in range(N):
        Z = np.asarray(dY, dtype=np.float64)
        for m in range(N):
            if m != n:
                Z = ttm(Z, np.asarray(Us[m]).T, m)
        dUs.append(unfold(Z, n) @ unfold(G, n).T)
    return dG, dUs


def tucker_loss(A: np.ndarray, Us) -> float:
    """L(A, U) = ||A - (A x_n U_n^T ...) x_n U_n ...||_F^2."""
    G = project(A, Us)
    return frob(np.asarray(A, dtype=np.float64) - tucker_to_tensor(G, Us)) ** 2


def tucker_loss_grads(A: np.ndarray, Us):
    """Gradients of ``tucker_loss`` by chaining the two adjoints above:
    E = A - A_hat, dL/dA_hat = -2E, dL/dA = 2E + (project adjoint of dG)."""
    A = np.asarray(A, dtype=np.float64)
    G = project(A, Us)
    E = A - tucker_to_tensor(G, Us)
    dY = -2.0 * E
    dG, dUr = reconstruct_vjp(G, Us, dY)
    dA_p, dUp = project_vjp(A, Us, dG)
    dA = 2.0 * E + dA_p
    dUs = [a + b for a, b in zip(dUr, dUp)]
    return dA, dUs
