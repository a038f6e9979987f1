"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: the
elementwise definitions written as loops, library SVD/QR, closed forms of the
ALS iteration (Appendix A), exact recovery, the st-HOSVD error identity and
the bounds of Lemma 2 / Theorem 4, finite differences, published generator
outputs.  No GPU needed.
"""
import os

import numpy as np
import pytest

from oracle import tucker_oracle as o
from workloads import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- P1: TTM

def _ttm_loops(A, M, n):
    """Mode-n product by the elementwise definition of Section 2."""
    shape = list(A.shape)
    shape[n] = M.shape[0]
    out = np.zeros(shape)
    for idx in np.ndindex(*shape):
        s = 0.0
        for i in range(A.shape[n]):
            src = list(idx)
            src[n] = i
            s += A[tuple(src)] * M[idx[n], i]
        out[idx] = s
    return out


@pytest.mark.parametrize("dims", [(2, 3, 4), (3, 1, 5, 2)])
def test_ttm_matches_elementwise_definition(dims):
    rng = np.random.default_rng(1)
    A = rng.standard_normal(dims)
    for n in range(len(dims)):
        M = rng.standard_normal((3, dims[n]))
        np.testing.assert_allclose(o.ttm(A, M, n), _ttm_loops(A, M, n),
                                   rtol=0, atol=1e-14)


def test_unfold_fold_roundtrip_and_paper_order():
    rng = np.random.default_rng(2)
    A = rng.standard_normal((3, 4, 2, 5))
    for n in range(4):
        U = o.unfold(A, n)
        np.testing.assert_array_equal(o.fold(U, n, A.shape), A)
        Up = o.unfold_paper(A, n)
        # same multiset of columns: the orders differ only by a permutation
        assert sorted(map(tuple, U.T.round(12))) == sorted(map(tuple, Up.T.round(12)))
        # left singular subspace and Gram do not depend on the column order
        np.testing.assert_allclose(U @ U.T, Up @ Up.T, atol=1e-13)
        # element (i_n, j) placement by the explicit column-major formula
        for idx in np.ndindex(*A.shape):
            j, stride = 0, 1
            for k in range(4):
                if k != n:
                    j += idx[k] * stride
                    stride *= A.shape[k]
            assert Up[idx[n], j] == A[idx]


def test_ttm_identity_composition_commutation():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((4, 5, 6))
    np.testing.assert_allclose(o.ttm(A, np.eye(5), 1), A, atol=1e-15)
    M1 = rng.standard_normal((3, 5))
    M2 = rng.standard_normal((2, 3))
    np.testing.assert_allclose(o.ttm(o.ttm(A, M1, 1), M2, 1),
                               o.ttm(A, M2 @ M1, 1), atol=1e-13)
    P = rng.standard_normal((2, 4))
    np.testing.assert_allclose(o.ttm(o.ttm(A, M1, 1), P, 0),
                               o.ttm(o.ttm(A, P, 0), M1, 1), atol=1e-13)


# --------------------------------------------- generator (published outputs)

def test_splitmix64_reference_outputs():
    with open(os.path.join(GOLDEN, "splitmix64.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    for row in rows:
        seed = int(row[0])
        want = [int(x, 16) for x in row[1:]]
        assert o.splitmix_stream(seed, len(want)) == want
        # the vectorised counter form gives the same stream
        got = o.splitmix_uniform(seed, np.arange(len(want)))
        np.testing.assert_array_equal(
            got, np.array([(w >> 40) * 2.0 ** -24 for w in want]))


def test_sketch_is_uniform_dense_full_rank():
    S = o.init_sketch(7, 2, 5000, 20)
    assert S.min() >= 0.0 and S.max() < 1.0
    assert abs(S.mean() - 0.5) < 0.01 and abs(S.var() - 1 / 12) < 0.005
    assert np.linalg.matrix_rank(S) == 20
    # values are exact multiples of 2^-24 (representable in float32)
    np.testing.assert_array_equal(S, S.astype(np.float32).astype(np.float64))
    # distinct modes draw distinct sketches
    assert not np.allclose(S, o.init_sketch(7, 3, 5000, 20))


# ------------------------------------------------- P2: SVD-based HOSVDs

def test_exact_recovery_svd_hosvd():
    rng = np.random.default_rng(4)
    A, A0, G, Us = synth.tucker_lowrank(rng, (12, 10, 9), (3, 4, 2), 0.0)
    for res in (o.thosvd_svd(A, (3, 4, 2)), o.sthosvd_svd(A, (3, 4, 2))[0]):
        assert o.relerr(A, res.G, res.U) <= 1e-13


def test_svd_methods_agree_with_eig():
    rng = np.random.default_rng(5)
    A = rng.standard_normal((10, 8, 6))
    a = o.thosvd_svd(A, (4, 3, 2), method="svd")
    b = o.thosvd_svd(A, (4, 3, 2), method="eig")
    for Ua, Ub in zip(a.U, b.U):
        assert o.subspace_distance(Ua, Ub) < 1e-10


def test_sthosvd_error_identity_and_bounds():
    """st-HOSVD: ||A - A_hat||^2 equals the sum of the discarded squared
    singular values of the successive B_(n) (the successive projections are
    orthogonal; Lemma 2's reference).  t-HOSVD error^2 <= sum gamma_n
    (eq. E5.1); the optimum is bounded below by max gamma_n."""
    rng = np.random.default_rng(6)
    A = rng.standard_normal((9, 8, 7, 6))
    ranks = (4, 3, 5, 2)
    st, disc = o.sthosvd_svd(A, ranks, order=[2, 0, 3, 1])
    err2 = o.relerr(A, st.G, st.U) ** 2 * o.frob(A) ** 2
    assert abs(err2 - sum(disc)) <= 1e-10 * o.frob(A) ** 2
    gam = o.tail_energies(A, ranks)
    t = o.thosvd_svd(A, ranks)
    et2 = o.relerr(A, t.G, t.U) ** 2 * o.frob(A) ** 2
    assert et2 <= sum(gam) * (1 + 1e-12)
    assert err2 <= sum(gam) * (1 + 1e-12)
    assert min(err2, et2) >= max(gam) * (1 - 1e-12)


# ------------------------------------------- P3: the ALS iteration itself

def test_als_closed_form_on_diagonal_matrix():
    """Appendix A, eq. E2.5: for A = diag(sigma) the block ratio
    T_k = L_k^(2) (L_k^(1))^{-1} evolves as T_{k+1} = S2^2 T_k S1^{-2}, hence
    T_k[i,j] = (sigma_{r+i}/sigma_j)^{2k} T_0[i,j]."""
    m, n, r = 7, 9, 3
    sig = np.array([5.0, 4.0, 3.0, 2.0, 1.5, 1.0, 0.5])
    A = np.zeros((m, n))
    A[np.arange(m), np.arange(m)] = sig
    rng = np.random.default_rng(7)
    L = rng.standard_normal((m, r))
    T0 = L[r:] @ np.linalg.inv(L[:r])
    ratio = sig[r:, None] / sig[None, :r]
    for k in range(1, 6):
        R = o.als_r_update(A, L)
        L = o.als_l_update(A, R)
        Tk = L[r:] @ np.linalg.inv(L[:r])
        np.testing.assert_allclose(Tk, ratio ** (2 * k) * T0, rtol=1e-9,
                                   atol=1e-13)


def test_als_r_update_is_least_squares_projection():
    """Algorithm 3.3 R-update is the least-squares solution, so L R^T equals
    the orthogonal projection of A onto span(L) (eq. E5.5), computed here
    through an SVD basis of L."""
    rng = np.random.default_rng(8)
    A = rng.standard_normal((20, 30))
    L = rng.standard_normal((20, 4))
    R = o.als_r_update(A, L)
    Ub = np.linalg.svd(L, full_matrices=False)[0]
    np.testing.assert_allclose(L @ R.T, Ub @ (Ub.T @ A), atol=1e-12)
    # L-update: least squares in the other factor
    L2 = o.als_l_update(A, R)
    Vb = np.linalg.svd(R, full_matrices=False)[0]
    np.testing.assert_allclose(L2 @ R.T, (A @ Vb) @ Vb.T, atol=1e-12)


def test_residual_trace_identity():
    """For R the least-squares solution given L:
    ||A - L R^T||^2 = ||A||^2 - tr(L^T L R^T R) (from eq. E5.5)."""
    rng = np.random.default_rng(9)
    A = rng.standard_normal((25, 40))
    L = rng.standard_normal((25, 5))
    R = o.als_r_update(A, L)
    lhs = o.frob(A - L @ R.T) ** 2
    rhs = o.frob(A) ** 2 - np.trace((L.T @ L) @ (R.T @ R))
    assert abs(lhs - rhs) <= 1e-12 * o.frob(A) ** 2


def test_als_converges_to_leading_subspace_with_gap():
    """Theorem 2: with sigma_r > sigma_{r+1} the ALS subspace converges to
    the leading left singular subspace (principal angles < 1e-6)."""
    rng = np.random.default_rng(10)
    U, _ = np.linalg.qr(rng.standard_normal((40, 40)))
    V, _ = np.linalg.qr(rng.standard_normal((60, 40)))
    s = np.concatenate([np.linspace(10, 6, 5), np.linspace(3, 0.1, 35)])
    A = (U * s) @ V.T
    L0 = o.als_initial_guess(A, o.init_sketch(0, 0, 60, 5))
    res = o.als(A, 5, L0, tol=1e-15, max_iters=200, norm_ref=o.frob(A))
    ang = o.principal_angles(res.L, U[:, :5])
    assert np.max(ang) < 1e-6
    # q-linear rate sigma_{r+1}^2/sigma_r^2 = 0.25: residual gaps shrink
    d = np.abs(np.diff(res.residuals))
    d = d[d > 1e-13]
    assert len(d) >= 3 and np.all(d[2:] <= d[1:-1] * 0.5)


def test_convergence_region_theorem3():
    """Theorem 3: an initial guess with
    ||L0^(2) (L0^(1))^{-1}||_2 below the bound converges."""
    m, n, r = 8, 10, 3
    sig = np.array([6.0, 5.0, 4.0, 2.0, 1.5, 1.0, 0.8, 0.5])
    A = np.zeros((m, n))
    A[np.arange(m), np.arange(m)] = sig
    eps = 1.0
    bound = np.sqrt((sig[r - 1] ** 2 - (sig[r - 1] - eps) ** 2)
                    / ((sig[r - 1] - eps) ** 2 - sig[-1] ** 2))
    rng = np.random.default_rng(11)
    L1 = rng.standard_normal((r, r)) + 3 * np.eye(r)
    T = rng.standard_normal((m - r, r))
    T *= 0.99 * bound / np.linalg.norm(T, 2)
    L0 = np.vstack([L1, T @ L1])
    res = o.als(A, r, L0, tol=1e-15, max_iters=300, norm_ref=o.frob(A))
    assert np.max(o.principal_angles(res.L, np.eye(m)[:, :r])) < 1e-6


def test_init_exact_rank_gives_zero_residual():
    """Section 5: R(L_0) lies in R(A_(n)); with exact rank r, L_0 already
    spans the dominant subspace, res_0 = 0 and the stop test fires at k=1."""
    rng = np.random.default_rng(12)
    A = rng.standard_normal((30, 4)) @ rng.standard_normal((4, 50))
    L0 = o.als_initial_guess(A, o.init_sketch(3, 0, 50, 4))
    Ub = np.linalg.svd(A)[0][:, :4]
    assert np.max(o.principal_angles(L0, Ub)) < 1e-12
    res = o.als(A, 4, L0, tol=1e-4, max_iters=50, norm_ref=o.frob(A))
    assert res.residuals[0] < 1e-12 * o.frob(A)
    assert res.iters == 1 and res.converged


def test_rank_deficient_raises():
    """Remark 3: truncation above the numerical rank makes a Gram singular."""
    rng = np.random.default_rng(13)
    A = rng.standard_normal((20, 3)) @ rng.standard_normal((3, 30))
    L0 = o.als_initial_guess(A, o.init_sketch(0, 0, 30, 5))
    with pytest.raises(np.linalg.LinAlgError):
        o.als(A, 5, L0, tol=1e-4, max_iters=5, norm_ref=o.frob(A))


def test_not_converged_flag():
    rng = np.random.default_rng(14)
    A = rng.standard_normal((30, 40))
    L0 = o.als_initial_guess(A, o.init_sketch(0, 0, 40, 6))
    res = o.als(A, 6, L0, tol=1e-14, max_iters=2, norm_ref=o.frob(A))
    assert res.iters == 2 and not res.converged and len(res.residuals) == 3


# ------------------------------------------------------------- P6: QR

def test_qr_signfix():
    rng = np.random.default_rng(15)
    L = rng.standard_normal((30, 6))
    Q, R = o.qr_signfix(L)
    np.testing.assert_allclose(Q.T @ Q, np.eye(6), atol=1e-14)
    assert np.all(np.diag(R) > 0)
    np.testing.assert_allclose(Q @ R, L, atol=1e-13)
    assert o.subspace_distance(Q, L) < 1e-13


# --------------------------------------------------------- P7: drivers

def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


@pytest.mark.parametrize("order", [None, [2, 0, 1]])
def test_sthosvd_als_identities(order):
    """st-HOSVD-ALS: the literal truncation R_hat R^T equals B x_n U^T (checked
    inside), ||A - A_hat||^2 = sum of the per-mode ALS residuals^2 and
    Pythagoras ||A||^2 = ||G||^2 + ||A - A_hat||^2."""
    rng = np.random.default_rng(16)
    A = synth.tucker_lowrank(rng, (14, 12, 10), (5, 4, 3), 0.05)[0]
    res = o.sthosvd_als(A, (5, 4, 3), order=order, tol=1e-6)
    err2 = (o.relerr(A, res.G, res.U) * o.frob(A)) ** 2
    assert _rel(err2, sum(i.resid ** 2 for i in res.info)) < 1e-10
    assert _rel(o.frob(A) ** 2, o.frob(res.G) ** 2 + err2) < 1e-12
    for U in res.U:
        np.testing.assert_allclose(U.T @ U, np.eye(U.shape[1]), atol=1e-13)


def test_thosvd_als_bounds():
    """t-HOSVD-ALS: error^2 <= sum_n res_n^2 for orthonormal factors, and the
    corrected Theorem 4 bound sqrt(sum (eta_n + sqrt(gamma_n)/||A||)^2)."""
    rng = np.random.default_rng(17)
    A = synth.tucker_lowrank(rng, (14, 12, 10), (5, 4, 3), 0.05)[0]
    ranks = (5, 4, 3)
    eta = 1e-3
    res = o.thosvd_als(A, ranks, tol=eta)
    nA = o.frob(A)
    err = o.relerr(A, res.G, res.U)
    assert (err * nA) ** 2 <= sum(i.resid ** 2 for i in res.info) * (1 + 1e-12)
    gam = o.tail_energies(A, ranks)
    # E5.0 is what Theorem 4 assumes; check it on the computed factors
    for n in range(3):
        ropt = np.sqrt(gam[n])
        assert res.info[n].resid >= ropt * (1 - 1e-12)
    bound = np.sqrt(sum((abs(i.resid - np.sqrt(g)) / nA + np.sqrt(g) / nA) ** 2
                        for i, g in zip(res.info, gam)))
    assert err <= bound * (1 + 1e-12)


def test_als_matches_svd_at_tight_tolerance():
    w = synth.workload_small_fp64()
    A, ranks = w["A"], w["ranks"]
    als_t = o.thosvd_als(A, ranks, tol=1e-12)
    svd_t = o.thosvd_svd(A, ranks)
    assert _rel(o.relerr(A, als_t.G, als_t.U), o.relerr(A, svd_t.G, svd_t.U)) < 1e-10
    for Ua, Us in zip(als_t.U, svd_t.U):
        assert np.max(o.principal_angles(Ua, Us)) < 1e-6
    als_s = o.sthosvd_als(A, ranks, tol=1e-12)
    svd_s = o.sthosvd_svd(A, ranks)[0]
    assert _rel(o.relerr(A, als_s.G, als_s.U), o.relerr(A, svd_s.G, svd_s.U)) < 1e-10


def test_warm_start_from_dominant_subspace():
    """Algorithm 3.3 takes L_0 as input (a warm start).  Started from any basis of
    the dominant subspace (here the SVD's, mixed by a random invertible matrix),
    res_0 is already the Eckart-Young residual of the unfolding, the stop test
    fires at k = 1, and the result is the SVD-based t-/st-HOSVD."""
    rng = np.random.default_rng(19)
    A = synth.tucker_lowrank(rng, (14, 12, 16), (4, 3, 5), 0.05)[0]
    ranks = (4, 3, 5)
    svd_t = o.thosvd_svd(A, ranks)
    init = [U @ rng.standard_normal((U.shape[1], U.shape[1])) for U in svd_t.U]
    t = o.thosvd_als(A, ranks, tol=1e-10, init=init)
    for n in range(3):
        sv = np.linalg.svd(o.unfold(A, n), compute_uv=False)
        tail = np.sqrt(np.sum(sv[ranks[n]:] ** 2))
        assert t.info[n].iters == 1 and t.info[n].converged
        assert abs(t.info[n].residuals[0] - tail) <= 1e-10 * o.frob(A)
        assert np.max(o.principal_angles(t.U[n], svd_t.U[n])) < 1e-9
    assert _rel(o.relerr(A, t.G, t.U), o.relerr(A, svd_t.G, svd_t.U)) < 1e-10
    svd_s = o.sthosvd_svd(A, ranks, order=[2, 0, 1])[0]
    s_ = o.sthosvd_als(A, ranks, order=[2, 0, 1], tol=1e-10, init=svd_s.U)
    assert all(i.iters == 1 for i in s_.info)
    assert _rel(o.relerr(A, s_.G, s_.U), o.relerr(A, svd_s.G, svd_s.U)) < 1e-10
    # a None entry keeps the Section 5 sketch for that mode
    part = o.thosvd_als(A, ranks, tol=1e-8, seed=4, init=[None, init[1], None])
    full = o.thosvd_als(A, ranks, tol=1e-8, seed=4)
    assert part.info[0].residuals == full.info[0].residuals
    assert part.info[1].iters == 1


def test_full_rank_mode_is_identity():
    rng = np.random.default_rng(18)
    A = rng.standard_normal((4, 9, 8))
    res = o.sthosvd_als(A, (4, 3, 5), tol=1e-6)
    np.testing.assert_array_equal(res.U[0], np.eye(4))
    assert res.info[0].iters == 0


def test_singular_vectors_exact_low_rank():
    """Singular vectors from the ALS basis (Section 3, after Algorithm 3.4) on an exactly
    low-rank tensor: each U^(n) matches the leading left singular vectors of A_(n) from
    numpy's SVD of the unfolding (up to sign), the core is all-orthogonal with
    G_(n) G_(n)^T = diag(sigma_1^2, ..., sigma_R^2) of A_(n) (the HOSVD property), and the
    error equals that of the plain ALS basis (same subspaces)."""
    rng = np.random.default_rng(31)
    dims, ranks = (12, 10, 9), (5, 4, 3)
    A = synth.tucker_lowrank(rng, dims, ranks, 0.0,
                             decay=synth.decay_geom(ranks, 0.6))[0]
    sv = o.thosvd_als(A, ranks, tol=1e-12, singular_vectors=True)
    plain = o.thosvd_als(A, ranks, tol=1e-12)
    nA = o.frob(A)
    for n in range(3):
        X, s, _ = np.linalg.svd(o.unfold(A, n), full_matrices=False)
        R = ranks[n]
        d = np.abs(np.sum(X[:, :R] * sv.U[n], axis=0))
        np.testing.assert_allclose(d, np.ones(R), atol=1e-9)
        np.testing.assert_allclose(sv.U[n].T @ sv.U[n], np.eye(R), atol=1e-13)
        Gn = o.unfold(sv.G, n)
        np.testing.assert_allclose(Gn @ Gn.T, np.diag(s[:R] ** 2), atol=1e-10 * nA ** 2)
        # same subspace as the QR basis
        assert np.max(o.principal_angles(sv.U[n], plain.U[n])) < 1e-7
    assert abs(o.relerr(A, sv.G, sv.U) - o.relerr(A, plain.G, plain.U)) < 1e-12


def test_singular_vectors_from_basis_order_and_sign():
    """Columns follow descending singular values of Q^T A_(n) (checked against the
    eigenvalues of the Gram) and the small factor W = Q^T U^(n) has its largest-magnitude
    entry positive in every column."""
    rng = np.random.default_rng(32)
    An = rng.standard_normal((15, 40))
    Q = synth.orthonormal(rng, 15, 6)
    U, s = o.singular_vectors_from_basis(An, Q)
    ev = np.linalg.eigvalsh(Q.T @ An @ An.T @ Q)[::-1]
    np.testing.assert_allclose(s ** 2, ev, rtol=1e-12)
    assert np.all(np.diff(s) <= 0)
    W = Q.T @ U
    np.testing.assert_allclose(W.T @ W, np.eye(6), atol=1e-13)
    for c in range(6):
        assert W[np.argmax(np.abs(W[:, c])), c] > 0
    # U^T A_(n) A_(n)^T U is diagonal: the columns are the singular directions
    M = U.T @ An @ An.T @ U
    np.testing.assert_allclose(M, np.diag(s ** 2), atol=1e-10 * s[0] ** 2)


def _st_cost_by_shapes(dims, ranks, order):
    """Work of st-HOSVD (Algorithm 3.2) counted on the shrinking tensor: mode n costs
    R_n times the number of entries of the tensor it is applied to, which then has its
    mode n cut to R_n."""
    shape = list(dims)
    total = 0
    for n in order:
        total += ranks[n] * int(np.prod(shape, dtype=object))
        shape[n] = ranks[n]
    return total


def test_st_order_cost_matches_shrinking_shapes():
    import itertools
    rng = np.random.default_rng(33)
    for N in (2, 3, 4, 5):
        for _ in range(5):
            dims = [int(x) for x in rng.integers(2, 40, N)]
            ranks = [int(rng.integers(1, d + 1)) for d in dims]
            for perm in itertools.permutations(range(N)):
                assert o.st_order_cost(dims, ranks, perm) == _st_cost_by_shapes(dims, ranks, perm)
    # worked by hand: dims (10, 20, 30), ranks (5, 2, 3), natural order:
    # 5*6000 + 10*600 + 30*30
    assert o.st_order_cost((10, 20, 30), (5, 2, 3), (0, 1, 2)) == 36900


def test_st_order_auto_prop1_and_ties():
    """Prop. 1: with equal dimensions the order of ascending ranks is cheapest; equal costs
    resolve to the first order in lexicographic order; the result is a true minimiser."""
    import itertools
    rng = np.random.default_rng(34)
    for N in (3, 4, 5):
        for _ in range(4):
            ranks = [int(x) for x in rng.choice(np.arange(1, 30), N, replace=False)]
            assert o.st_order_auto([40] * N, ranks) == list(np.argsort(ranks))
    assert o.st_order_auto([16] * 4, [3] * 4) == [0, 1, 2, 3]
    assert o.st_order_auto([16, 16, 16], [5, 2, 2]) == [1, 2, 0]
    for _ in range(10):
        dims = [int(x) for x in rng.integers(2, 60, 4)]
        ranks = [int(rng.integers(1, d + 1)) for d in dims]
        best = o.st_order_auto(dims, ranks)
        costs = {p: _st_cost_by_shapes(dims, ranks, p) for p in itertools.permutations(range(4))}
        m = min(costs.values())
        assert costs[tuple(best)] == m
        assert tuple(best) == min(p for p, c in costs.items() if c == m)


def _hooi_stationarity(A, Us):
    """max_n ||(I - U_n U_n^T) Y_(n) Y_(n)^T U_n|| / ||Y||^2, Y = A x_{k != n} U_k^T: zero
    at a stationary point of ||G||^2 over orthonormal factors (first-order condition)."""
    worst = 0.0
    for n in range(A.ndim):
        Y = A
        for k in range(A.ndim):
            if k != n:
                Y = o.ttm(Y, Us[k].T, k)
        Yn = o.unfold(Y, n)
        M = Yn @ Yn.T
        U = Us[n]
        worst = max(worst, np.linalg.norm(M @ U - U @ (U.T @ M @ U)) / np.linalg.norm(M))
    return worst


def test_hooi_monotone_stationary_and_bounded():
    """HOOI from t-HOSVD on a noisy tensor: the error never increases, ends strictly below
    the t-HOSVD error, is bounded below by every single-mode Eckart-Young error, and the
    final factors satisfy the first-order stationarity condition."""
    rng = np.random.default_rng(35)
    dims, ranks = (14, 12, 10), (4, 3, 3)
    A = synth.tucker_lowrank(rng, dims, ranks, 0.3)[0]
    start = o.thosvd_svd(A, ranks)
    G, Us, errs, conv = o.hooi(A, start.U, tol=1e-13, max_iters=500)
    assert conv
    assert all(b <= a * (1 + 1e-13) for a, b in zip(errs, errs[1:]))
    assert errs[-1] < errs[0] - 1e-6
    nA = o.frob(A)
    gam = o.tail_energies(A, ranks)
    assert errs[-1] * nA >= max(gam) ** 0.5 * (1 - 1e-12)
    assert _hooi_stationarity(A, Us) < 1e-6
    # the t-HOSVD start itself is not stationary here
    assert _hooi_stationarity(A, start.U) > 1e-4
    for U in Us:
        np.testing.assert_allclose(U.T @ U, np.eye(U.shape[1]), atol=1e-13)


def test_hooi_recovers_exact_low_rank_from_random_start():
    rng = np.random.default_rng(36)
    dims, ranks = (10, 9, 8), (3, 2, 3)
    A = synth.tucker_lowrank(rng, dims, ranks, 0.0)[0]
    Us0 = [synth.orthonormal(rng, d, r) for d, r in zip(dims, ranks)]
    G, Us, errs, conv = o.hooi(A, Us0, tol=1e-15, max_iters=200)
    assert errs[0] > 0.1
    assert errs[-1] < 1e-7


# ---------------------------------------------------------- P8: gradients

def _fd(f, x, d, h=1e-3):
    """Central difference at h and h/2 combined by Richardson extrapolation
    (error O(h^4) instead of O(h^2))."""
    c1 = (f(x + h * d) - f(x - h * d)) / (2 * h)
    h2 = h / 2
    c2 = (f(x + h2 * d) - f(x - h2 * d)) / (2 * h2)
    return (4 * c2 - c1) / 3


def test_tucker_loss_gradients_finite_difference():
    rng = np.random.default_rng(19)
    A = rng.standard_normal((7, 6, 5))
    Us = [synth.orthonormal(rng, d, r) for d, r in zip(A.shape, (3, 2, 4))]
    dA, dUs = o.tucker_loss_grads(A, Us)
    D = rng.standard_normal(A.shape)
    fd = _fd(lambda X: o.tucker_loss(X, Us), A, D)
    assert _rel(np.sum(dA * D), fd) < 1e-8
    for n in range(3):
        Dn = rng.standard_normal(Us[n].shape)

        def f(Un, n=n):
            V = list(Us)
            V[n] = Un
            return o.tucker_loss(A, V)
        assert _rel(np.sum(dUs[n] * Dn), _fd(f, Us[n], Dn)) < 1e-8
    # at orthonormal factors dL/dA = 2E
    E = A - o.tucker_to_tensor(o.project(A, Us), Us)
    np.testing.assert_allclose(dA, 2 * E, atol=1e-12)


def test_project_and_reconstruct_vjp_finite_difference():
    rng = np.random.default_rng(20)
    A = rng.standard_normal((6, 5, 4))
    Us = [rng.standard_normal((d, r)) for d, r in zip(A.shape, (3, 2, 2))]
    W = rng.standard_normal((3, 2, 2))
    dA, dUs = o.project_vjp(A, Us, W)
    f = lambda X: np.sum(o.project(X, Us) * W)
    D = rng.standard_normal(A.shape)
    assert _rel(np.sum(dA * D), _fd(f, A, D)) < 1e-8
    for n in range(3):
        Dn = rng.standard_normal(Us[n].shape)

        def g(Un, n=n):
            V = list(Us)
            V[n] = Un
            return np.sum(o.project(A, V) * W)
        assert _rel(np.sum(dUs[n] * Dn), _fd(g, Us[n], Dn)) < 1e-8
    G = rng.standard_normal((3, 2, 2))
    Y = rng.standard_normal(A.shape)
    dG, dU2 = o.reconstruct_vjp(G, Us, Y)
    h = lambda X: np.sum(o.tucker_to_tensor(X, Us) * Y)
    DG = rng.standard_normal(G.shape)
    assert _rel(np.sum(dG * DG), _fd(h, G, DG)) < 1e-8
    for n in range(3):
        Dn = rng.standard_normal(Us[n].shape)

        def k(Un, n=n):
            V = list(Us)
            V[n] = Un
            return np.sum(o.tucker_to_tensor(G, V) * Y)
        assert _rel(np.sum(dU2[n] * Dn), _fd(k, Us[n], Dn)) < 1e-8


def test_loss_gradient_symmetry():
    """The loss depends on U_n only through U_n U_n^T, so U_n^T dL/dU_n is
    symmetric."""
    rng = np.random.default_rng(21)
    A = rng.standard_normal((7, 6, 5))
    Us = [synth.orthonormal(rng, d, r) for d, r in zip(A.shape, (3, 2, 4))]
    _, dUs = o.tucker_loss_grads(A, Us)
    for U, dU in zip(Us, dUs):
        M = U.T @ dU
        np.testing.assert_allclose(M, M.T, atol=1e-12)


# ------------------------------------------- principal angles, tail energies

def _planes_at_angles(rng, n, thetas):
    """Two k-dimensional subspaces of R^n whose principal angles are exactly
    ``thetas`` (by construction: the j-th basis vectors of the two spaces span
    a plane of their own, orthogonal to every other pair's), then turned by a
    random rotation of R^n and given non-orthonormal bases."""
    k = len(thetas)
    assert n >= 2 * k
    X = np.zeros((n, k))
    Y = np.zeros((n, k))
    for j, t in enumerate(thetas):
        X[2 * j, j] = 1.0
        Y[2 * j, j] = np.cos(t)
        Y[2 * j + 1, j] = np.sin(t)
    Qr, _ = np.linalg.qr(rng.standard_normal((n, n)))
    Mx = rng.standard_normal((k, k)) + 3.0 * np.eye(k)
    My = rng.standard_normal((k, k)) + 3.0 * np.eye(k)
    return Qr @ X @ Mx, Qr @ Y @ My


def test_principal_angles_constructed():
    """Principal angles (used by Theorem 2's subspace statement) against
    subspaces built at known angles: one of 1e-9 rad (the sine branch), one
    of 1.2 rad (the cosine branch), and 0.35 rad in between."""
    rng = np.random.default_rng(11)
    thetas = np.array([1e-9, 0.35, 1.2])
    U1, U2 = _planes_at_angles(rng, 8, thetas)
    got = np.sort(o.principal_angles(U1, U2))
    # the rotation and the mixing matrices cost a few ulps of the sines
    assert abs(got[0] - 1e-9) <= 2e-15, got[0]
    np.testing.assert_allclose(got[1:], thetas[1:], rtol=0, atol=1e-14)
    # symmetric in its arguments
    np.testing.assert_allclose(np.sort(o.principal_angles(U2, U1)), got, rtol=0, atol=2e-15)


def test_principal_angles_extremes():
    """Equal spans give zero angles; orthogonal spans give pi/2."""
    rng = np.random.default_rng(12)
    U, _ = np.linalg.qr(rng.standard_normal((9, 3)))
    M = rng.standard_normal((3, 3)) + 3.0 * np.eye(3)
    assert np.max(o.principal_angles(U, U @ M)) <= 1e-15
    U1, U2 = _planes_at_angles(rng, 6, [np.pi / 2] * 3)
    np.testing.assert_allclose(o.principal_angles(U1, U2), np.pi / 2, rtol=0, atol=1e-14)


def test_subspace_distance_is_projector_gap():
    """For equal-dimension subspaces, sin of the largest principal angle equals
    the spectral norm of the difference of the orthogonal projectors, computed
    here directly from the projectors."""
    rng = np.random.default_rng(13)
    for thetas in ([1e-7, 0.2], [0.4, 0.9, 1.5], [0.0, 0.0]):
        U1, U2 = _planes_at_angles(rng, 7, thetas)
        Q1, _ = np.linalg.qr(U1)
        Q2, _ = np.linalg.qr(U2)
        gap = np.linalg.norm(Q1 @ Q1.T - Q2 @ Q2.T, 2)
        assert abs(o.subspace_distance(U1, U2) - gap) <= 1e-14
        assert abs(o.subspace_distance(U1, U2) - np.sin(max(thetas))) <= 1e-14


def test_tail_energies_closed_form():
    """gamma_n of Lemma 2 (eq. E5.1) on a tensor with a diagonal core and
    orthonormal factors: every unfolding has exactly the core's diagonal
    entries as singular values (the Khatri-Rao columns of orthonormal factors
    are orthonormal), so gamma_n is the sum of the squares of the diagonal
    entries beyond the R_n largest."""
    rng = np.random.default_rng(14)
    lam = np.array([9.0, -7.0, 5.5, 4.0, 2.5, 1.0])
    dims = (10, 8, 12)
    Us = [np.linalg.qr(rng.standard_normal((d, len(lam))))[0] for d in dims]
    G = np.zeros((len(lam),) * 3)
    for r, v in enumerate(lam):
        G[r, r, r] = v
    A = o.tucker_to_tensor(G, Us)
    sq = np.sort(lam ** 2)[::-1]
    for ranks in ((2, 3, 1), (5, 1, 4), (6, 6, 6)):
        want = [float(np.sum(sq[R:])) for R in ranks]
        np.testing.assert_allclose(o.tail_energies(A, ranks), want, rtol=1e-12, atol=1e-12)


def test_tail_energies_first_mode_of_sthosvd():
    """The st-HOSVD discarded energy of the first processed mode is that
    mode's gamma_n (Algorithm 3.2 starts from A itself), and every later mode's
    discarded energy is at most its gamma_n (projection can only remove
    energy)."""
    rng = np.random.default_rng(15)
    A = rng.standard_normal((7, 6, 5))
    ranks = (3, 2, 4)
    gam = o.tail_energies(A, ranks)
    for order in ((0, 1, 2), (2, 0, 1), (1, 2, 0)):
        _, disc = o.sthosvd_svd(A, ranks, order=order)
        assert abs(disc[order[0]] - gam[order[0]]) <= 1e-12 * gam[order[0]]
        for n in order[1:]:
            assert disc[n] <= gam[n] * (1 + 1e-12)
