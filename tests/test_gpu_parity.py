"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Both sides receive the same seeded input: the oracle runs in FP64 on exactly
the values the GPU holds (the FP32 or BF16 rounding of the FP64 master, or
the FP64 master itself).  Tolerances:
  * FP64 storage: 1e-10 relative on contractions, relerr within 1e-10;
  * FP32 storage: contractions within a few FP32 roundings of an I-term sum
    (rtol 2e-5 with an absolute floor scaled by the operands' norms),
    relative reconstruction error within 1e-5 of the oracle's;
  * BF16 storage: relerr (against the FP64 master) within 1e-2 of the
    oracle's FP64 result.
Subspaces are compared through principal angles (only span(U_n) is defined).
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
    """FP64 copy of exactly the values the GPU holds."""
    return to_gpu(a, dt).double().cpu().numpy()


def np64(t):
    return t.detach().double().cpu().numpy()


def flush(msg):
    print(msg, flush=True)


# ------------------------------------------------------------------ TTM

TTM_CASES = [
    ((7, 9, 11), 1, 5, False),
    ((7, 9, 11), 2, 13, True),      # Q == 1 (last mode), expansion
    ((70, 3, 130), 0, 4, True),     # P == 1, ragged tiles
    ((5, 200, 66), 1, 20, True),    # truncation 200 -> 20, ragged fibre tiles
    ((3, 4, 5, 6), 3, 2, False),
    ((65, 129), 0, 70, False),      # order 2, more outputs than one chunk
    ((300, 150), 1, 37, True),      # Q == 1, 48-wide rank padding, ragged fibre tiles
    ((33, 256, 17), 1, 48, False),  # largest mode and output width of the MFMA TTM
    ((40, 520, 9), 1, 48, True),    # large-mode TTM (chunked rows)
    ((33, 700), 1, 20, False),      # large-mode TTM, Q == 1
    ((9, 70, 40), 1, 19, True),     # TTM width 16 < J <= 20
    ((33, 60), 1, 17, False),       # TTM width 16 < J <= 20, Q == 1
    # Q a multiple of 8, I <= 224: the BF16 16-byte prefetch form
    ((6, 200, 48), 1, 20, True),    # tiles straddle p
    ((3, 128, 1000), 1, 16, False), # 23.4 BF16 tiles, ragged end
]


@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("dims,mode,J,trans", TTM_CASES)
def test_ttm_parity(gpu_lib, dims, mode, J, trans, dt):
    tk = gpu_lib
    flush(f"ttm {dims} mode={mode} J={J} trans={trans} {dt}")
    rng = np.random.default_rng(100 + mode)
    X = rng.standard_normal(dims)
    I = dims[mode]
    M = rng.standard_normal((I, J) if trans else (J, I))
    mdt = "f64" if dt == "f64" else "f32"
    Y = tk.ttm(to_gpu(X, dt), to_gpu(M, mdt), mode, transpose=trans)
    Mh = held(M, mdt)
    want = o.ttm(held(X, dt), Mh.T if trans else Mh, mode)
    got = np64(Y)
    assert got.shape == want.shape
    if dt == "f64":
        np.testing.assert_allclose(got, want, rtol=1e-11, atol=1e-11 * np.abs(want).max())
    else:
        # FP32 accumulation of I products: error <~ I * 2^-24 * sum |x||m|
        bound = I * 2.0 ** -24 * o.ttm(np.abs(held(X, dt)), np.abs(Mh.T if trans else Mh), mode)
        assert np.all(np.abs(got - want) <= 4 * bound + 1e-30)


def test_tucker_reconstruct_parity(gpu_lib):
    tk = gpu_lib
    rng = np.random.default_rng(5)
    ranks, dims = (3, 5, 2, 4), (9, 7, 6, 70)
    G = rng.standard_normal(ranks)
    Us = [rng.standard_normal((d, r)) for d, r in zip(dims, ranks)]
    for dt in ("f64", "f32"):
        out = tk.tucker_reconstruct(to_gpu(G, dt), [to_gpu(u, dt) for u in Us])
        want = o.tucker_to_tensor(held(G, dt), [held(u, dt) for u in Us])
        tol = 1e-12 if dt == "f64" else 2e-5
        assert np.max(np.abs(np64(out) - want)) <= tol * np.abs(want).max()


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_contract_allbut_parity(gpu_lib, dt):
    tk = gpu_lib
    rng = np.random.default_rng(6)
    X = rng.standard_normal((13, 70, 9))
    for mode, J in ((0, 5), (1, 33), (2, 7)):
        shp = list(X.shape)
        shp[mode] = J
        Y = rng.standard_normal(shp)
        K = tk.contract_allbut(to_gpu(X, dt), to_gpu(Y, dt), mode)
        want = o.unfold(held(X, dt), mode) @ o.unfold(held(Y, dt), mode).T
        tol = 1e-11 if dt == "f64" else 3e-5
        assert np.max(np.abs(np64(K) - want)) <= tol * np.abs(want).max()


# --------------------------------------------------- single steps of ALS

STEP_CASES = [((20, 30, 40), 0, 5), ((20, 30, 40), 1, 7), ((20, 30, 40), 2, 6),
              ((100, 9, 70), 0, 20), ((12, 11, 10, 9), 2, 4),
              ((30, 64, 50), 1, 18),      # second rank tile mostly padding, I = 64, tiles straddle p
              ((40, 150, 30), 1, 19),     # second rank tile mostly padding, ragged row tiles
              ((1024, 60), 0, 48)]        # m r^2 > 10^6: the mode step on a grid of workgroups


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("dims,mode,R", STEP_CASES)
def test_init_step_parity(gpu_lib, dims, mode, R, dt):
    tk = gpu_lib
    flush(f"init {dims} mode={mode} R={R} {dt}")
    rng = np.random.default_rng(7)
    A = rng.standard_normal(dims)
    seed = 1234
    Y, L0, n2 = tk.als_init_step(to_gpu(A, dt), mode, R, seed=seed)
    Ah = held(A, dt)
    An = o.unfold(Ah, mode)
    S = o.init_sketch(seed, mode, An.shape[1], R)
    want = An @ S
    tol = 1e-12 if dt == "f64" else 1e-5
    assert np.max(np.abs(np64(Y) - want)) <= tol * np.abs(want).max()
    assert abs(n2 - o.frob(Ah) ** 2) <= 1e-12 * o.frob(Ah) ** 2
    Q = np64(L0)
    np.testing.assert_allclose(Q.T @ Q, np.eye(R), atol=1e-12)
    Qo, _ = o.qr_signfix(np64(Y))
    np.testing.assert_allclose(Q, Qo, atol=1e-10)


# modes of 256 < I <= 1024 rows: the chunked sketch kernels (BF16 storage on
# the BF16 matrix cores when Q, or I when Q == 1, is a multiple of 8)
INIT_LARGE_CASES = [
    ((16, 520, 24), 1, 48),     # R = 48, five chunks (the last ragged), Q = 24
    ((33, 392), 1, 20),         # Q == 1 (fibres are rows), one ragged fibre tile
    ((3, 1000, 8), 1, 5),       # R = 5, Q = 8, J = 24
    ((2, 1024, 40), 1, 48),     # I = 1024, ragged fibre tiles, several tiles per sketch set
    ((300, 20, 40), 0, 12),     # P == 1, I = 300 (last chunk 44 rows)
    ((7, 600, 33), 1, 40),      # Q = 33: BF16 widened to FP32 on the FP32 matrix core
]


def check_init_step(tk, dims, mode, R, dt):
    """Initial sketch pass (Section 5): Y = A_(n) S and ||A||^2 against FP64
    on the same stored values (FP32 accumulation of up to J products per
    entry), and L_0 the QR of Y."""
    rng = np.random.default_rng(17)
    A = rng.standard_normal(dims)
    seed = 99
    Y, L0, n2 = tk.als_init_step(to_gpu(A, dt), mode, R, seed=seed)
    Ah = held(A, dt)
    An = o.unfold(Ah, mode)
    S = o.init_sketch(seed, mode, An.shape[1], R)
    want = An @ S
    assert np.max(np.abs(np64(Y) - want)) <= 1e-5 * np.abs(want).max()
    assert abs(n2 - o.frob(Ah) ** 2) <= 1e-12 * o.frob(Ah) ** 2
    Q = np64(L0)
    np.testing.assert_allclose(Q.T @ Q, np.eye(R), atol=1e-12)
    Qo, _ = o.qr_signfix(np64(Y))
    np.testing.assert_allclose(Q, Qo, atol=1e-10)


@pytest.mark.parametrize("dt", ["f32", "bf16"])
@pytest.mark.parametrize("dims,mode,R", INIT_LARGE_CASES)
def test_init_step_parity_large(gpu_lib, dims, mode, R, dt):
    """The sketch pass on large modes (chunked kernels)."""
    flush(f"init large {dims} mode={mode} R={R} {dt}")
    check_init_step(gpu_lib, dims, mode, R, dt)


# BF16 storage on modes of up to 224 rows (the register-buffered BF16 kernel)
INIT_BF16_CASES = [
    ((40, 200, 48), 1, 20),     # Q = 48: 16-byte loads, tiles straddle p
    ((6, 200, 1000), 1, 20),    # Q = 1000: 16-byte loads, 46.9 tiles, ragged end
    ((200, 40, 30), 0, 16),     # P == 1, Q = 1200, one rank tile
    ((9, 100, 64), 1, 30),      # I = 100, two rank tiles, Q = 64
    ((20, 200, 50), 1, 20),     # Q = 50: dword loads
]


@pytest.mark.parametrize("dims,mode,R", INIT_BF16_CASES)
def test_init_step_parity_bf16(gpu_lib, dims, mode, R):
    """The sketch pass with BF16 storage on modes of up to 224 rows."""
    flush(f"init bf16 {dims} mode={mode} R={R}")
    check_init_step(gpu_lib, dims, mode, R, "bf16")


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("resid", ["trace", "explicit"])
@pytest.mark.parametrize("dims,mode,R", STEP_CASES)
def test_sweep_step_parity(gpu_lib, dims, mode, R, dt, resid):
    """One fused sweep from a given L_k equals one literal iteration of
    Algorithm 3.3: R_k = A^T L (L^T L)^{-1}, L_{k+1} = A R_k (R_k^T R_k)^{-1},
    res_k = ||A - L_k R_k^T||."""
    tk = gpu_lib
    flush(f"sweep {dims} mode={mode} R={R} {dt} {resid}")
    rng = np.random.default_rng(8)
    A = synth.tucker_lowrank(rng, dims, tuple(min(R + 2, d) for d in dims), 0.05)[0]
    Ah = held(A, dt)
    An = o.unfold(Ah, mode)
    Lk = rng.standard_normal((An.shape[0], R)) + 0.0
    Lk, _ = np.linalg.qr(Lk)
    Lk = Lk + 0.01 * rng.standard_normal(Lk.shape)
    n2 = o.frob(Ah) ** 2
    Ln, res2 = tk.als_sweep_step(to_gpu(Ah, dt), mode, torch.from_numpy(Lk).cuda(), n2,
                                 resid_mode=resid)
    Rk = o.als_r_update(An, Lk)
    Lw = o.als_l_update(An, Rk)
    rw = o.frob(An - Lk @ Rk.T)
    got = np64(Ln)
    tol = 1e-9 if dt == "f64" else 2e-4
    assert np.max(np.abs(got - Lw)) <= tol * np.abs(Lw).max()
    rg = np.sqrt(max(res2, 0.0))
    rtol = 1e-9 if dt == "f64" else (1e-3 if resid == "explicit" else 5e-2)
    assert abs(rg - rw) <= rtol * rw + 1e-6 * np.sqrt(n2) * (dt != "f64")


def test_qr_parity(gpu_lib):
    tk = gpu_lib
    rng = np.random.default_rng(9)
    for m, r in ((50, 7), (1024, 48), (64, 64)):
        Lm = rng.standard_normal((m, r)) @ np.diag(np.logspace(0, 3, r))
        Q = np64(tk.qr_f64(torch.from_numpy(Lm).cuda()))
        Qo, _ = o.qr_signfix(Lm)
        np.testing.assert_allclose(Q, Qo, atol=1e-9)
        np.testing.assert_allclose(Q.T @ Q, np.eye(r), atol=1e-12)


# ------------------------------------------------------- drivers

def _relerr_of(A64, G, Us):
    return o.relerr(A64, np64(G), [np64(u) for u in Us])


def test_small_fp64_workload_parity(gpu_lib):
    """64^3 FP64, ranks (8,8,8), tol 1e-8: t- and st-HOSVD-ALS."""
    tk = gpu_lib
    w = synth.workload_small_fp64()
    A, ranks, tol = w["A"], w["ranks"], w["tol"]
    Ag = to_gpu(A, "f64")
    for which in ("st", "t"):
        flush(f"driver small fp64 {which}")
        if which == "st":
            G, Us, info = tk.als_sthosvd(Ag, ranks, tol=tol, seed=11)
            ref = o.sthosvd_als(A, ranks, tol=tol, seed=11)
        else:
            G, Us, info = tk.als_thosvd(Ag, ranks, tol=tol, seed=11)
            ref = o.thosvd_als(A, ranks, tol=tol, seed=11)
        e_gpu = _relerr_of(A, G, Us)
        e_ref = o.relerr(A, ref.G, ref.U)
        assert abs(e_gpu - e_ref) <= 1e-10
        for n in range(3):
            assert np.max(o.principal_angles(np64(Us[n]), ref.U[n])) < 1e-6
            assert info["iters"][n] == ref.info[n].iters
            assert abs(info["resid"][n] - ref.info[n].resid) <= 1e-8 * ref.norm_a
        assert abs(info["norm_a"] - ref.norm_a) <= 1e-12 * ref.norm_a


DRIVER_CASES = [
    # dims, ranks, noise, order
    ((24, 30, 36, 20), (6, 5, 7, 4), 1e-4, None),
    ((70, 66, 40), (12, 9, 10), 1e-3, [2, 0, 1]),
    ((130, 20, 33), (16, 8, 8), 1e-3, None),
]


@pytest.mark.parametrize("dt", ["f32", "bf16"])
@pytest.mark.parametrize("dims,ranks,noise,order", DRIVER_CASES)
@pytest.mark.parametrize("which", ["st", "t"])
def test_driver_parity(gpu_lib, dims, ranks, noise, order, dt, which):
    """FP32 / BF16 storage against the oracle run in FP64 on exactly the values the
    GPU holds: relative errors within 1e-5 and the same iteration count per mode
    (+-1: the last step of the stop test may fall either side of eta under
    different rounding).  BF16 also against the oracle on the FP64 tensor (1e-2)."""
    tk = gpu_lib
    flush(f"driver {which} {dims} {ranks} {dt}")
    rng = np.random.default_rng(20)
    A, A0, _, _ = synth.tucker_lowrank(rng, dims, ranks, noise)
    Ah = held(A, dt)
    tol = 1e-6
    if which == "st":
        G, Us, info = tk.als_sthosvd(to_gpu(A, dt), ranks, tol=tol, seed=3, order=order)
        ref = o.sthosvd_als(Ah, ranks, order=order, tol=tol, seed=3)
    else:
        G, Us, info = tk.als_thosvd(to_gpu(A, dt), ranks, tol=tol, seed=3)
        ref = o.thosvd_als(Ah, ranks, tol=tol, seed=3)
    e_gpu = _relerr_of(Ah, G, Us)
    e_ref = o.relerr(Ah, ref.G, ref.U)
    assert abs(e_gpu - e_ref) <= 1e-5, (e_gpu, e_ref)
    gi, oi = info["iters"], [m.iters for m in ref.info]
    flush(f"  iters gpu={gi} oracle={oi} forms={info['resid_form']}")
    assert all(abs(a - b) <= 1 for a, b in zip(gi, oi)), (gi, oi)
    assert info["mode_status"] == ["TK_OK"] * len(dims)
    if dt == "bf16":
        ref64 = (o.sthosvd_als(A, ranks, order=order, tol=tol, seed=3) if which == "st"
                 else o.thosvd_als(A, ranks, tol=tol, seed=3))
        assert abs(_relerr_of(A, G, Us) - o.relerr(A, ref64.G, ref64.U)) <= 1e-2
    for U in Us:
        Uh = np64(U)
        np.testing.assert_allclose(Uh.T @ Uh, np.eye(Uh.shape[1]), atol=1e-5)


@pytest.mark.parametrize("dt", ["f32", "bf16"])
def test_tight_tol_iteration_counts(gpu_lib, dt):
    """A small tensor at eta = 1e-6: the trace form's rounding (a few 2^-24 ||B||^2
    over sqrt(J / I)) would exceed eta ||A|| here, so the stop test runs on the
    explicit residual and the iteration counts follow the oracle's."""
    tk = gpu_lib
    rng = np.random.default_rng(2004025830)
    A = synth.tucker_lowrank(rng, (40, 36, 44), (6, 5, 7), 1e-3)[0]
    Ah = held(A, dt)
    for which in ("st", "t"):
        flush(f"tight tol {which} {dt}")
        run = tk.als_sthosvd if which == "st" else tk.als_thosvd
        G, Us, info = run(to_gpu(A, dt), (6, 5, 7), tol=1e-6, seed=1)
        ref = (o.sthosvd_als if which == "st" else o.thosvd_als)(Ah, (6, 5, 7), tol=1e-6, seed=1)
        gi, oi = info["iters"], [m.iters for m in ref.info]
        flush(f"  iters gpu={gi} oracle={oi}")
        assert info["resid_form"] == ["explicit"] * 3
        assert all(abs(a - b) <= 1 for a, b in zip(gi, oi)), (gi, oi)
        assert abs(_relerr_of(Ah, G, Us) - o.relerr(Ah, ref.G, ref.U)) <= 1e-5
        for n in range(3):
            # the explicit residual is free of the trace form's cancellation
            assert abs(info["resid"][n] - ref.info[n].resid) <= 1e-6 * ref.norm_a


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("which", ["st", "t"])
def test_warm_start_parity(gpu_lib, dt, which):
    """init_U: Algorithm 3.3 started from a given L_0 per mode (one mode left on the
    sketch), against the oracle started from the same L_0 values.  FP64: identical
    iteration counts and residuals to 1e-9 ||A||; FP32: counts +-1, errors 1e-5."""
    tk = gpu_lib
    flush(f"warm start {which} {dt}")
    rng = np.random.default_rng(24)
    dims, ranks = (30, 26, 34), (6, 5, 7)
    A = synth.tucker_lowrank(rng, dims, ranks, 0.05)[0]
    svd = o.thosvd_svd(A, ranks)
    # a perturbed basis of the dominant subspace, mixed by an invertible matrix
    init = [U + 0.2 * rng.standard_normal(U.shape) for U in svd.U]
    init = [L0 @ (np.eye(L0.shape[1]) + 0.3 * rng.standard_normal((L0.shape[1],) * 2))
            for L0 in init]
    init[1] = None
    fdt = "f64" if dt == "f64" else "f32"
    Ah = held(A, dt)
    init_h = [None if L0 is None else held(L0, fdt) for L0 in init]
    init_g = [None if L0 is None else to_gpu(L0, fdt) for L0 in init]
    run = tk.als_sthosvd if which == "st" else tk.als_thosvd
    G, Us, info = run(to_gpu(A, dt), ranks, tol=1e-8, seed=2, init=init_g)
    ref = (o.sthosvd_als if which == "st" else o.thosvd_als)(Ah, ranks, tol=1e-8, seed=2,
                                                             init=init_h)
    gi, oi = info["iters"], [m.iters for m in ref.info]
    flush(f"  iters gpu={gi} oracle={oi}")
    if dt == "f64":
        assert gi == oi
        for n in range(3):
            assert abs(info["resid"][n] - ref.info[n].resid) <= 1e-9 * ref.norm_a
            assert np.max(o.principal_angles(np64(Us[n]), ref.U[n])) < 1e-8
        assert abs(_relerr_of(Ah, G, Us) - o.relerr(Ah, ref.G, ref.U)) <= 1e-10
    else:
        assert all(abs(a - b) <= 1 for a, b in zip(gi, oi)), (gi, oi)
        assert abs(_relerr_of(Ah, G, Us) - o.relerr(Ah, ref.G, ref.U)) <= 1e-5
    assert abs(info["norm_a"] - ref.norm_a) <= 1e-6 * ref.norm_a


def test_rank_deficient_status(gpu_lib):
    tk = gpu_lib
    rng = np.random.default_rng(30)
    A = synth.tucker_lowrank(rng, (20, 22, 24), (3, 3, 3), 0.0)[0]
    with pytest.raises(tk.TuckerALSError) as e:
        tk.als_sthosvd(to_gpu(A, "f64"), (6, 3, 3), tol=1e-6)
    assert e.value.code == -4


def test_rank_deficient_status_grid_mode_step(gpu_lib):
    """Remark 3's rank test inside the mode step that runs on a grid of
    workgroups (m R^2 >= 10^6): a mode of exact rank 3 asked for R = 48 fails
    its initial QR on every workgroup alike, and the call reports it for that
    mode (the modes after it are skipped)."""
    import ctypes
    from paper_2004_02583_amd import _lib as L
    tk = gpu_lib
    flush("rank deficient, grid mode step")
    rng = np.random.default_rng(31)
    A = to_gpu(synth.tucker_lowrank(rng, (1024, 8, 8), (3, 3, 3), 0.0)[0], "f64")
    ranks = (48, 8, 8)
    lib = L.lib()
    dims = L.i64arr(A.shape)
    rk = L.i32arr(ranks)
    need = lib.als_workspace_bytes(1, L.TK_F64, 3, dims, rk)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    Us = [torch.empty((A.shape[n], ranks[n]), dtype=torch.float64, device="cuda") for n in range(3)]
    G = torch.empty(ranks, dtype=torch.float64, device="cuda")
    info = L.tk_als_info()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.als_sthosvd(ctypes.c_void_p(A.data_ptr()), L.TK_F64, 3, dims, rk, None,
                         L.ptrarr([u.data_ptr() for u in Us]), ctypes.c_void_p(G.data_ptr()),
                         ctypes.c_void_p(ws.data_ptr()), need, ctypes.byref(info), stream)
    torch.cuda.synchronize()
    assert rc == -4 and info.status == -4
    assert list(info.mode_status)[:3] == [-4, 2, 2]
    with pytest.raises(tk.TuckerALSError) as e:
        tk.als_thosvd(A, ranks, tol=1e-6)
    assert e.value.code == -4


@pytest.mark.parametrize("dt", ["f64"])
def test_mode_status_report(gpu_lib, dt):
    """Per-mode status through the C ABI: the failing mode carries the error (Remark 3),
    modes before it their own result, modes after it TK_SKIPPED."""
    import ctypes
    from paper_2004_02583_amd import _lib as L
    tk = gpu_lib
    rng = np.random.default_rng(30)
    A = to_gpu(synth.tucker_lowrank(rng, (20, 22, 24), (3, 3, 3), 0.0)[0], dt)
    lib = L.lib()
    for ranks, want in (((6, 3, 3), [-4, 2, 2]), ((3, 6, 3), [0, -4, 2])):
        flush(f"mode status {ranks} {dt}")
        dims = L.i64arr(A.shape)
        rk = L.i32arr(ranks)
        need = lib.als_workspace_bytes(1, L.TK_F64 if dt == "f64" else L.TK_F32, 3, dims, rk)
        ws = torch.empty(need, dtype=torch.uint8, device="cuda")
        fdt = torch.float64 if dt == "f64" else torch.float32
        Us = [torch.empty((A.shape[n], ranks[n]), dtype=fdt, device="cuda") for n in range(3)]
        G = torch.empty(ranks, dtype=fdt, device="cuda")
        info = L.tk_als_info()
        stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        rc = lib.als_sthosvd(ctypes.c_void_p(A.data_ptr()),
                             L.TK_F64 if dt == "f64" else L.TK_F32, 3, dims, rk, None,
                             L.ptrarr([u.data_ptr() for u in Us]), ctypes.c_void_p(G.data_ptr()),
                             ctypes.c_void_p(ws.data_ptr()), need, ctypes.byref(info), stream)
        assert rc == -4 and info.status == -4
        assert list(info.mode_status)[:3] == want


@pytest.mark.parametrize("resid", ["trace", "explicit"])
@pytest.mark.parametrize("max_iters", [0, 1, 2])
def test_small_max_iters_parity(gpu_lib, max_iters, resid):
    """Every status-read arrangement of a mode solve: with max_iters = 0 a read follows the
    initial step; otherwise the initial step and sweeps 0 and 1 share one read, and later sweeps
    have their own.  FP64 against the oracle: iteration counts, residuals and subspaces."""
    tk = gpu_lib
    rng = np.random.default_rng(23)
    ranks = (6, 5, 4)
    A = synth.tucker_lowrank(rng, (30, 26, 22), ranks, 0.3)[0]
    G, Us, info = tk.als_thosvd(to_gpu(A, "f64"), ranks, tol=1e-15, max_iters=max_iters,
                                seed=3, resid_mode=resid)
    ref = o.thosvd_als(A, ranks, tol=1e-15, max_iters=max_iters, seed=3)
    assert info["status"] == "TK_NOT_CONVERGED"
    for n in range(3):
        assert info["iters"][n] == ref.info[n].iters == max_iters
        assert not info["converged"][n]
        assert abs(info["resid"][n] - ref.info[n].resid) <= 1e-9 * ref.norm_a
        assert np.max(o.principal_angles(np64(Us[n]), ref.U[n])) < 1e-8
    assert abs(info["norm_a"] - ref.norm_a) <= 1e-12 * ref.norm_a


def test_not_converged_status(gpu_lib):
    tk = gpu_lib
    rng = np.random.default_rng(31)
    A = rng.standard_normal((30, 30, 30))
    G, Us, info = tk.als_sthosvd(to_gpu(A, "f64"), (5, 5, 5), tol=1e-15, max_iters=2)
    assert info["status"] == "TK_NOT_CONVERGED"
    assert info["iters"][0] == 2 and not info["converged"][0]


def test_nonfinite_input(gpu_lib):
    tk = gpu_lib
    A = np.ones((8, 9, 10))
    A[3, 4, 5] = np.nan
    with pytest.raises(tk.TuckerALSError) as e:
        tk.als_sthosvd(to_gpu(A, "f32"), (2, 2, 2))
    assert e.value.code == -5


def test_full_rank_mode_identity(gpu_lib):
    tk = gpu_lib
    rng = np.random.default_rng(32)
    A = rng.standard_normal((4, 9, 8))
    G, Us, info = tk.als_sthosvd(to_gpu(A, "f64"), (4, 3, 5), tol=1e-8)
    np.testing.assert_array_equal(np64(Us[0]), np.eye(4))
    ref = o.sthosvd_als(A, (4, 3, 5), tol=1e-8)
    assert abs(_relerr_of(A, G, Us) - o.relerr(A, ref.G, ref.U)) <= 1e-10


def test_determinism(gpu_lib):
    tk = gpu_lib
    rng = np.random.default_rng(33)
    A = to_gpu(rng.standard_normal((40, 50, 60)), "f32")
    G1, U1, _ = tk.als_sthosvd(A, (5, 6, 7), tol=1e-6)
    G2, U2, _ = tk.als_sthosvd(A, (5, 6, 7), tol=1e-6)
    assert torch.equal(G1, G2) and all(torch.equal(a, b) for a, b in zip(U1, U2))


KERNEL_CASES = [
    # dims, mode, R : covers Q > 64, medium Q, Q == 1, ragged tiles, I > 256
    ((200, 40, 30), 0, 20),     # P == 1, Q = 1200
    ((20, 200, 50), 1, 20),     # Q = 50 < 64: tiles straddle p
    ((30, 40, 200), 2, 20),     # Q == 1 (last mode)
    ((17, 33, 65), 1, 3),       # R not a multiple of 4, ragged everything
    ((64, 256, 9), 1, 32),      # I = 256, R = 32
    ((9, 100, 70), 1, 48),      # R = 48 (largest fused rank)
    ((300, 20, 40), 0, 12),     # I > 256: chunked large-mode kernel
    ((7, 600, 33), 1, 40),      # I = 600: ragged last chunk, tiles straddle p
    ((50, 1024), 1, 48),        # I = 1024, Q == 1, R = 48, one ragged tile
    ((1100, 8, 9), 0, 5),       # I > 1024: generic two-pass kernels
    ((20, 200, 50), 1, 17),     # 16 < R <= 20 (second rank tile mostly padding), Q < 64
    ((30, 40, 200), 2, 19),     # 16 < R <= 20, Q == 1
    ((64, 37, 70), 1, 18),      # 16 < R <= 20, ragged small mode
    # BF16 storage, 256 < I <= 1024: the BF16-matrix-core large-mode sweep
    ((16, 520, 24), 1, 48),     # R = 48, five chunks (the last ragged), Q = 24
    ((48, 264, 16), 1, 33),     # R = 33 (third rank tile mostly padding), last chunk 8 rows
    ((33, 392), 1, 20),         # Q == 1 (fibres are rows), one ragged fibre tile
    ((3, 1000, 8), 1, 5),       # R = 5, Q = 8, J = 24
    ((2, 1024, 40), 1, 48),     # I = 1024, R = 48, ragged fibre tiles
    # modes of up to 224 rows with Q a multiple of 4, R up to 32, many tiles per workgroup
    ((40, 200, 36), 1, 20),     # I = 200 (seven 32-row blocks), Q = 36 < 64: tiles straddle p
    ((13, 64, 12), 1, 16),      # I = 64, one rank tile, ragged last tile
    ((8, 100, 20), 1, 3),       # I = 100 (four blocks, the last ragged), R = 3
    ((5, 224, 8), 1, 32),       # I = 224, R = 32 (largest), J = 40 < one tile
    ((6, 1, 16), 1, 1),         # I = 1, R = 1
    ((1, 150, 4), 1, 4),        # J = 4: one group of four fibres
    ((40, 200, 1004), 1, 20),   # 627.5 tiles: both prefetch buffers cycle, ragged end
    # Q a multiple of 8: the BF16 16-byte prefetch form
    ((40, 200, 1000), 1, 20),   # 312.5 BF16 tiles: both buffers cycle, ragged end
    ((24, 200, 40), 1, 9),      # Q = 40 < one BF16 tile: tiles straddle p
]


def bf16_round(x):
    """Round float32 values to BF16 precision (nearest even), kept as float64."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("dt", ["f32", "bf16"])
@pytest.mark.parametrize("dims,mode,R", KERNEL_CASES)
def test_sweep_kernel_parity(gpu_lib, dims, mode, R, dt):
    """Lacc = A_(n) V and GV = V^T V for V = A_(n)^T Lq, against FP64 on the
    same values (FP32 accumulation: a few roundings of I-term and
    J-term sums).  For BF16 storage Lq enters rounded to BF16 precision."""
    tk = gpu_lib
    flush(f"sweep_kernel {dims} mode={mode} R={R} {dt}")
    rng = np.random.default_rng(40)
    A = rng.standard_normal(dims)
    Lq = rng.standard_normal((dims[mode], R)).astype(np.float32)
    Lacc, GV = tk.als_sweep_kernel(to_gpu(A, dt), mode, torch.from_numpy(Lq).cuda())
    An = o.unfold(held(A, dt), mode)
    Lh = bf16_round(Lq) if dt == "bf16" else Lq.astype(np.float64)
    V = An.T @ Lh
    want_l = An @ V
    want_g = V.T @ V
    # scale-aware bounds: |V| from |A||Lq|, then |A||V|
    Vabs = np.abs(An).T @ np.abs(Lh)
    bl = (dims[mode] + 64) * 2.0 ** -24 * (np.abs(An) @ Vabs)
    bg = (dims[mode] + 64) * 2.0 ** -24 * (Vabs.T @ Vabs)
    assert np.all(np.abs(np64(Lacc) - want_l) <= 4 * bl + 1e-30)
    assert np.all(np.abs(np64(GV) - want_g) <= 4 * bg + 1e-30)
    np.testing.assert_array_equal(np64(GV), np64(GV).T)


@pytest.mark.parametrize("resid", ["auto", "trace"])
@pytest.mark.parametrize("dt", ["f32", "bf16"])
@pytest.mark.parametrize("which", ["t", "st"])
def test_large_mode_driver_parity(gpu_lib, which, dt, resid):
    """A 700-row mode runs the chunked large-mode kernels (sketch, sweeps, TTM); with
    the trace residual its BF16 sweeps run on the BF16-matrix-core large-mode kernel
    (the explicit residual, which the automatic choice takes at this J, runs the
    two-pass kernels).  Errors against the oracle on the values the GPU holds."""
    tk = gpu_lib
    flush(f"large-mode driver {which} {dt} {resid}")
    rng = np.random.default_rng(42)
    A = synth.tucker_lowrank(rng, (700, 24, 32), (20, 6, 8), 1e-3)[0]
    Ah = held(A, dt)
    run = tk.als_thosvd if which == "t" else tk.als_sthosvd
    G, Us, info = run(to_gpu(A, dt), (20, 6, 8), tol=1e-5, seed=3, resid_mode=resid)
    ref = (o.thosvd_als if which == "t" else o.sthosvd_als)(Ah, (20, 6, 8), tol=1e-5, seed=3)
    flush(f"  iters gpu={info['iters']} oracle={[m.iters for m in ref.info]}")
    assert abs(_relerr_of(Ah, G, Us) - o.relerr(Ah, ref.G, ref.U)) <= 1e-5
    if dt == "bf16":
        ref64 = (o.thosvd_als if which == "t" else o.sthosvd_als)(A, (20, 6, 8), tol=1e-5, seed=3)
        assert abs(_relerr_of(A, G, Us) - o.relerr(A, ref64.G, ref64.U)) <= 1e-2


def test_two_pass_driver_parity(gpu_lib):
    """I_1 = 1100 > 1024 runs the generic two-pass kernels for mode 1."""
    tk = gpu_lib
    rng = np.random.default_rng(41)
    A = synth.tucker_lowrank(rng, (1100, 24, 20), (10, 6, 8), 1e-3)[0]
    Ah = held(A, "f32")
    G, Us, info = tk.als_sthosvd(to_gpu(A, "f32"), (10, 6, 8), tol=1e-6, seed=5)
    ref = o.sthosvd_als(Ah, (10, 6, 8), tol=1e-6, seed=5)
    assert abs(_relerr_of(Ah, G, Us) - o.relerr(Ah, ref.G, ref.U)) <= 1e-5
