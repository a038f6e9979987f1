"""GPU parity of HOOI refinement (Section 6.3, Table 6.3-2) against the FP64 oracle.

Both sides start from the same factors, the oracle's t-HOSVD-ALS result on the values the GPU
holds (computed on the CPU), and iterate to the same stationary point: the device solves each
mode by warm-started ALS, the oracle by an exact SVD, so iteration counts differ (reported,
not gated) while the limit is the same.  Gates: the final error within 1e-9 (FP64) or 1e-5
(FP32/BF16 storage) of the oracle's, subspaces within 1e-5 / 1e-3 rad, the error of the
given factors equal to the oracle's, and no increase over the start.
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


HOOI_CASES = [
    # dims, core dims, ranks, core decay, dtype: the truncation cuts through a slowly
    # decaying core, so HOOI lowers the t-HOSVD error by 0.3 to 2 per cent in 6 to 32
    # iterations (oracle)
    ((24, 20, 16), (8, 8, 8), (5, 4, 3), 0.8, "f64"),
    ((40, 36, 30), (10, 9, 8), (6, 5, 4), 0.8, "f32"),
    ((40, 36, 30), (10, 9, 8), (6, 5, 4), 0.9, "bf16"),
    ((30, 20, 16, 12), (6, 5, 5, 4), (4, 3, 3, 2), 0.8, "f32"),
    ((300, 24, 20), (12, 8, 8), (8, 5, 4), 0.8, "f32"),
]


@pytest.mark.parametrize("dims,core,ranks,decay,dt", HOOI_CASES)
def test_hooi_parity(gpu_lib, dims, core, ranks, decay, dt):
    tk = gpu_lib
    flush(f"hooi {dims} {ranks} {dt}")
    rng = np.random.default_rng(70)
    A = synth.tucker_lowrank(rng, dims, core, 1e-3, decay=synth.decay_geom(core, decay))[0]
    Ah = held(A, dt)
    start = o.thosvd_als(Ah, ranks, tol=1e-4, seed=2)
    fdt = "f64" if dt == "f64" else "f32"
    U0 = [to_gpu(U, fdt) for U in start.U]
    # the error is flat at the optimum, so a stop on its change leaves the subspace about
    # sqrt(tol) away: FP64 stops at 1e-12; FP32/BF16 storage, whose error carries FP32
    # rounding, runs a fixed 60 iterations (the oracle needs 12 to 32 to reach 1e-13)
    if dt == "f64":
        G, Us, info = tk.hooi(to_gpu(A, dt), U0, tol=1e-12, max_iters=300, als_max_iters=3)
        assert info["status"] == "TK_OK"
    else:
        G, Us, info = tk.hooi(to_gpu(A, dt), U0, tol=0.0, max_iters=60, als_max_iters=3)
        assert info["status"] in ("TK_OK", "TK_NOT_CONVERGED")
    Gr, Ur, errs, conv = o.hooi(Ah, [np64(U) for U in U0], tol=1e-13, max_iters=1000)
    assert conv
    flush(f"  device: {info['iters']} iterations, {info['sweeps']} sweeps, "
          f"error {info['relerr_init']:.6e} -> {info['relerr']:.6e}; "
          f"oracle: {len(errs) - 1} iterations, {errs[0]:.6e} -> {errs[-1]:.6e}")
    g_err, g_ang = (1e-9, 1e-5) if dt == "f64" else (1e-5, 1e-3)
    assert abs(info["relerr_init"] - errs[0]) <= (1e-12 if dt == "f64" else 1e-6)
    e_gpu = o.relerr(Ah, np64(G), [np64(u) for u in Us])
    assert abs(e_gpu - errs[-1]) <= g_err, (e_gpu, errs[-1])
    assert abs(info["relerr"] - e_gpu) <= (1e-12 if dt == "f64" else 1e-6)
    assert e_gpu <= errs[0] + g_err
    assert errs[-1] < errs[0] - 1e-3
    for n in range(len(dims)):
        Ug = np64(Us[n])
        np.testing.assert_allclose(Ug.T @ Ug, np.eye(ranks[n]), atol=1e-12 if dt == "f64" else 1e-5)
        ang = np.max(o.principal_angles(Ug, Ur[n]))
        flush(f"  mode {n}: largest principal angle {ang:.2e}")
        assert ang < g_ang
    # the input factors are left unchanged by the binding
    for U, Us0 in zip(U0, start.U):
        np.testing.assert_allclose(np64(U), Us0, atol=1e-6)


def test_hooi_zero_iterations_is_the_start(gpu_lib):
    """max_iters = 0: the core and error of the given factors, returned unchanged."""
    tk = gpu_lib
    rng = np.random.default_rng(71)
    A = synth.tucker_lowrank(rng, (20, 18, 16), (4, 4, 3), 0.1)[0]
    Us0 = [synth.orthonormal(rng, d, r) for d, r in zip((20, 18, 16), (4, 4, 3))]
    G, Us, info = tk.hooi(to_gpu(A, "f64"), [to_gpu(U, "f64") for U in Us0], max_iters=0)
    assert info["status"] == "TK_OK" and info["iters"] == 0
    Gr = o.core_from_factors(A, Us0)
    np.testing.assert_allclose(np64(G), Gr, atol=1e-12 * o.frob(A))
    assert abs(info["relerr_init"] - o.relerr(A, Gr, Us0)) <= 1e-12
    for U, U0 in zip(Us, Us0):
        np.testing.assert_array_equal(np64(U), U0)
