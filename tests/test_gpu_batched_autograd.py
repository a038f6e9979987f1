"""GPU checks of the batched persistent st-HOSVD-ALS and of the autograd
Functions over the Tucker projection / reconstruction chain."""
import os

import numpy as np
import pytest
import torch

from oracle import tucker_oracle as o
from workloads import synth

pytestmark = pytest.mark.gpu


def np64(t):
    return t.detach().double().cpu().numpy()


def flush(msg):
    print(msg, flush=True)


# ------------------------------------------------------------ batched

def _batch(count, hi, rhi, k=4):
    return synth.workload_batched(count=count, lo=16, hi=hi, rlo=4, rhi=rhi, k=k)


def test_batched_matches_oracle_and_single(gpu_lib, tmp_path, monkeypatch):
    tk = gpu_lib
    monkeypatch.setenv("TK_AUTOTUNE_CACHE", str(tmp_path / "tune.txt"))
    items = _batch(24, 48, 8)
    As = [torch.from_numpy(it["A"]).float().cuda() for it in items]
    ranks = [it["ranks"] for it in items]
    flush("batched 24 tensors")
    out, status = tk.batched_sthosvd(As, ranks, tol=1e-6, seed=9)
    # 0 converged, 1 stopped at max_iters (slow gap): both are valid results
    assert all(s in (0, 1) for s in status), status
    for t, (A, rk) in enumerate(zip(As, ranks)):
        G, Us, iters = out[t]
        Ah = A.double().cpu().numpy()
        e_b = o.relerr(Ah, np64(G), [np64(u) for u in Us])
        ref = o.sthosvd_als(Ah, rk, tol=1e-6, seed=9)
        e_o = o.relerr(Ah, ref.G, ref.U)
        assert abs(e_b - e_o) <= 1e-5, (t, e_b, e_o)
        G1, U1, info = tk.als_sthosvd(A, rk, tol=1e-6, seed=9)
        e_s = o.relerr(Ah, np64(G1), [np64(u) for u in U1])
        assert abs(e_b - e_s) <= 1e-6 * max(1.0, e_s) + 1e-7, (t, e_b, e_s)
        for U in Us:
            Uh = np64(U)
            np.testing.assert_allclose(Uh.T @ Uh, np.eye(Uh.shape[1]), atol=1e-5)
    # the autotuner recorded its choice
    txt = (tmp_path / "tune.txt").read_text()
    assert "gfx950/batched" in txt


def test_batched_rank_deficient_member(gpu_lib):
    tk = gpu_lib
    rng = np.random.default_rng(50)
    good = synth.tucker_lowrank(rng, (20, 24, 18), (4, 5, 3), 1e-3)[0]
    bad = synth.tucker_lowrank(rng, (20, 22, 24), (2, 2, 2), 0.0)[0]   # rank 2 < 4
    As = [torch.from_numpy(x).float().cuda() for x in (good, bad, good)]
    # eta = 1e-5: with 1e-3 noise, |res_k - res_k+1| carries ~5e-7 ||A|| of FP32
    # rounding from the trace form, so a tighter eta sits inside that noise
    out, status = tk.batched_sthosvd(As, [(4, 5, 3), (4, 4, 4), (4, 5, 3)], tol=1e-5)
    assert status[0] == 0 and status[2] == 0
    assert status[1] == -4


def test_batched_full_workload_sampled(gpu_lib):
    """The 512-tensor workload (I_n in [16,128], R_n in [4,16]): every member
    converges with orthonormal factors; a sample matches single-tensor runs."""
    tk = gpu_lib
    items = _batch(512, 128, 16)
    As = [torch.from_numpy(it["A"]).float().cuda() for it in items]
    ranks = [it["ranks"] for it in items]
    flush("batched 512 tensors")
    out, status = tk.batched_sthosvd(As, ranks, tol=1e-4)
    assert all(s in (0, 1) for s in status)
    for t in range(0, 512, 37):
        G, Us, _ = out[t]
        A = As[t]
        Ah = A.double().cpu().numpy()
        e_b = o.relerr(Ah, np64(G), [np64(u) for u in Us])
        G1, U1, _ = tk.als_sthosvd(A, ranks[t], tol=1e-4)
        e_s = o.relerr(Ah, np64(G1), [np64(u) for u in U1])
        assert abs(e_b - e_s) <= 1e-6 + 1e-6 * e_s, (t, e_b, e_s)
        assert e_b < 2e-3


def test_batched_plan_graph_replays(gpu_lib):
    """BatchedPlan.run replays the HIP graph it captured on the first call: three calls with
    eager device work between them give bitwise the results of the first, which equal a
    fresh batched call's and stay within 1e-6 of single-tensor runs."""
    tk = gpu_lib
    items = _batch(40, 64, 10, k=7)
    As = [torch.from_numpy(it["A"]).float().cuda() for it in items]
    ranks = [it["ranks"] for it in items]
    plan = tk.BatchedPlan(As, ranks)
    flush("batched plan: first call (capture)")
    st0 = plan.run(tol=1e-6, seed=2)
    first = [(G.clone(), [u.clone() for u in Us], it) for G, Us, it in plan.results()]
    for rep in range(3):
        junk = torch.randn(1 << 20, device="cuda")
        junk = (junk * 2.0).sum()                     # eager work between the replays
        plan.U.fill_(float("nan"))
        plan.G.fill_(float("nan"))
        torch.cuda.synchronize()
        flush(f"batched plan: replay {rep}")
        st = plan.run(tol=1e-6, seed=2)
        assert st == st0
        for (G0, U0, it0), (G1, U1, it1) in zip(first, plan.results()):
            assert it0 == it1
            assert torch.equal(G0, G1) and all(torch.equal(a, b) for a, b in zip(U0, U1))
    fresh, sts = tk.batched_sthosvd(As, ranks, tol=1e-6, seed=2)
    assert sts == st0
    for (G0, U0, _), (G1, U1, _) in zip(first, fresh):
        assert torch.equal(G0, G1) and all(torch.equal(a, b) for a, b in zip(U0, U1))
    for t in range(0, 40, 7):
        Ah = As[t].double().cpu().numpy()
        G, Us, _ = first[t]
        e_b = o.relerr(Ah, np64(G), [np64(u) for u in Us])
        G1, U1, _ = tk.als_sthosvd(As[t], ranks[t], tol=1e-6, seed=2)
        e_s = o.relerr(Ah, np64(G1), [np64(u) for u in U1])
        assert abs(e_b - e_s) <= 1e-6 * max(1.0, e_s) + 1e-7, (t, e_b, e_s)


# ------------------------------------------------------------ autograd

def _loss(tk, A, Us):
    G = tk.TuckerProject.apply(A, *Us)
    Ah = tk.TuckerReconstruct.apply(G, *Us)
    return ((A - Ah) ** 2).sum()


@pytest.mark.parametrize("budget", [1 << 30, 0])
def test_autograd_fp64_matches_oracle(gpu_lib, budget):
    tk = gpu_lib
    from paper_2004_02583_amd import autograd as ag
    old = ag.get_memory_budget()
    ag.set_memory_budget(budget)
    try:
        rng = np.random.default_rng(60)
        A = rng.standard_normal((9, 7, 8))
        Us = [synth.orthonormal(rng, d, r) for d, r in zip(A.shape, (3, 4, 2))]
        At = torch.from_numpy(A).cuda().requires_grad_(True)
        Ut = [torch.from_numpy(u).cuda().requires_grad_(True) for u in Us]
        L = _loss(tk, At, Ut)
        L.backward()
        dA, dUs = o.tucker_loss_grads(A, Us)
        assert abs(L.item() - o.tucker_loss(A, Us)) <= 1e-10 * abs(L.item())
        np.testing.assert_allclose(np64(At.grad), dA, atol=1e-10)
        for g, want in zip(Ut, dUs):
            np.testing.assert_allclose(np64(g.grad), want, atol=1e-10)
        # separate Functions against their oracle adjoints
        W = rng.standard_normal((3, 4, 2))
        At.grad = None
        for u in Ut:
            u.grad = None
        G = tk.TuckerProject.apply(At, *Ut)
        (G * torch.from_numpy(W).cuda()).sum().backward()
        dA2, dU2 = o.project_vjp(A, Us, W)
        np.testing.assert_allclose(np64(At.grad), dA2, atol=1e-11)
        for g, want in zip(Ut, dU2):
            np.testing.assert_allclose(np64(g.grad), want, atol=1e-11)
    finally:
        ag.set_memory_budget(old)


def test_autograd_central_difference_fp64(gpu_lib):
    tk = gpu_lib
    rng = np.random.default_rng(61)
    A = rng.standard_normal((6, 5, 7))
    Us = [rng.standard_normal((d, r)) for d, r in zip(A.shape, (2, 3, 2))]
    Ut = [torch.from_numpy(u).cuda().requires_grad_(True) for u in Us]
    At = torch.from_numpy(A).cuda().requires_grad_(True)
    L = _loss(tk, At, Ut)
    L.backward()
    h = 1e-3
    D = rng.standard_normal(A.shape)
    Dt = torch.from_numpy(D).cuda()
    with torch.no_grad():
        fd = (_loss(tk, At + h * Dt, Ut) - _loss(tk, At - h * Dt, Ut)).item() / (2 * h)
    assert abs(fd - float((At.grad * Dt).sum())) <= 1e-6 * abs(fd) + 1e-8
    for n in range(3):
        Dn = torch.from_numpy(rng.standard_normal(Us[n].shape)).cuda()
        with torch.no_grad():
            up = [u.clone() for u in Ut]
            dn = [u.clone() for u in Ut]
            up[n] += h * Dn
            dn[n] -= h * Dn
            fd = (_loss(tk, At, up) - _loss(tk, At, dn)).item() / (2 * h)
        an = float((Ut[n].grad * Dn).sum())
        # central differences on a degree-8 polynomial: O(h^2) truncation
        assert abs(fd - an) <= 1e-4 * abs(an) + 1e-6


def test_autograd_workload_fp32_vs_fp64_reference(gpu_lib):
    """256^3 FP32 tensor, orthonormal 256x32 factors: forward core and loss
    gradients against the FP64 oracle on the same values."""
    tk = gpu_lib
    w = synth.workload_autograd()
    A, Us = w["A"], w["U"]
    At = torch.from_numpy(A).float().cuda().requires_grad_(True)
    Ut = [torch.from_numpy(u).float().cuda().requires_grad_(True) for u in Us]
    flush("autograd 256^3")
    L = _loss(tk, At, Ut)
    L.backward()
    Ah = At.detach().double().cpu().numpy()
    Uh = [np64(u) for u in Ut]
    G = np64(tk.TuckerProject.apply(At.detach(), *[u.detach() for u in Ut]))
    Gw = o.core_from_factors(Ah, Uh)
    assert np.max(np.abs(G - Gw)) <= 1e-4 * np.max(np.abs(Gw))
    dA, dUs = o.tucker_loss_grads(Ah, Uh)
    ga = np64(At.grad)
    assert np.linalg.norm(ga - dA) <= 1e-4 * np.linalg.norm(dA)
    for g, want in zip(Ut, dUs):
        assert np.linalg.norm(np64(g.grad) - want) <= 1e-3 * np.linalg.norm(want)
    # element by element under an FP32 accumulation bound: the same chain of
    # products run on |A| and |U_n|, with E = A - A_hat bounded by |A| + |A_hat|
    # terms, times gamma = 2 n u for n the summed lengths along the chain
    # (project 3 x 256, reconstruct 3 x 32, their two adjoints, and the
    # 32 x 32 contraction of dU_n)
    a, u = np.abs(Ah), [np.abs(x) for x in Uh]
    Gm = o.project(a, u)
    Em = a + o.tucker_to_tensor(Gm, u)
    dGm, dUrm = o.reconstruct_vjp(Gm, u, 2.0 * Em)
    dApm, dUpm = o.project_vjp(a, u, dGm)
    gamma = 2.0 * (2 * (3 * 256 + 3 * 32) + 32 * 32) * 2.0 ** -24
    bound_a = gamma * (2.0 * Em + dApm)
    ra = np.abs(ga - dA) / bound_a
    flush(f"  dA: max |err| / bound = {ra.max():.3e}")
    assert np.all(np.abs(ga - dA) <= bound_a)
    for n, g in enumerate(Ut):
        bound_u = gamma * (dUrm[n] + dUpm[n])
        err = np.abs(np64(g.grad) - dUs[n])
        flush(f"  dU_{n}: max |err| / bound = {(err / bound_u).max():.3e}")
        assert np.all(err <= bound_u)
    # that bound is rigorous but loose (absolute values compound along the
    # chain); element by element against the rounding scale of the chain as
    # well: sqrt(n) u (|g| + rms g) for the n summed terms, with a margin of 64
    n_chain = 2 * (3 * 256 + 3 * 32) + 32 * 32
    tau = 64.0 * np.sqrt(n_chain) * 2.0 ** -24
    for name, got, want in [("dA", ga, dA)] + [(f"dU_{n}", np64(g.grad), dUs[n])
                                               for n, g in enumerate(Ut)]:
        scale = np.abs(want) + np.sqrt(np.mean(want ** 2))
        r = np.abs(got - want) / scale
        flush(f"  {name}: max |err| / (|g| + rms g) = {r.max():.3e} (tolerance {tau:.2e})")
        assert np.all(r <= tau), name
