"""Oracle parity at the full size of the benchmark workload: the 200^4 FP32 tensor
(core 20^4 with exp(-(i+j+k+l)/10) decay, orthonormal 200x20 factors, 1e-4 relative
noise), st-HOSVD-ALS (Algorithm 3.5) to ranks 20 with eta = 1e-4 in natural order,
exactly the call bench.py times.  The FP64 oracle runs its literal Algorithm 3.3 on the
host, on the FP64 copy of the very FP32 values the GPU holds (12.8 GB; about a minute of
host time and ~60 GB of host memory), and both errors are computed by the oracle's
explicit-difference relerr."""
import time

import numpy as np
import pytest
import torch

from oracle import tucker_oracle as o
from workloads import synth

pytestmark = pytest.mark.gpu

DIMS = (200, 200, 200, 200)
R = 20
TOL = 1e-4


def flush(msg):
    print(msg, flush=True)


def test_fullsize_sthosvd_matches_oracle(gpu_lib):
    tk = gpu_lib
    flush("fullsize oracle parity: generating the 200^4 FP32 workload")
    w = synth.workload_4way_torch(DIMS, R, 1e-4)
    A = w["A"]
    torch.cuda.synchronize()
    flush("fullsize oracle parity: GPU st-HOSVD-ALS")
    G, Us, info = tk.als_sthosvd(A, (R,) * 4, tol=TOL, seed=0)
    assert info["status"] == "TK_OK"
    Gh = G.double().cpu().numpy()
    Uh = [u.double().cpu().numpy() for u in Us]
    Ah = A.cpu().numpy().astype(np.float64)
    del A, w, G, Us
    torch.cuda.empty_cache()
    t0 = time.perf_counter()
    flush("fullsize oracle parity: oracle st-HOSVD-ALS on the host (FP64)")
    ref = o.sthosvd_als(Ah, (R,) * 4, tol=TOL, seed=0, check_identity=False)
    flush(f"  oracle done in {time.perf_counter() - t0:.1f} s")
    e_gpu = o.relerr(Ah, Gh, Uh)
    e_ref = o.relerr(Ah, ref.G, ref.U)
    gi, oi = info["iters"], [m.iters for m in ref.info]
    angles = [float(np.max(o.principal_angles(Uh[n], ref.U[n]))) for n in range(4)]
    flush(f"  relerr gpu={e_gpu:.9e} oracle={e_ref:.9e} diff={abs(e_gpu - e_ref):.3e}")
    flush(f"  iters gpu={gi} oracle={oi} forms={info['resid_form']}")
    flush(f"  max principal angle per mode: {['%.2e' % a for a in angles]}")
    flush(f"  resid gpu={['%.6e' % r for r in info['resid']]} "
          f"oracle={['%.6e' % m.resid for m in ref.info]}")
    assert abs(e_gpu - e_ref) <= 1e-5, (e_gpu, e_ref)
    assert all(abs(a - b) <= 1 for a, b in zip(gi, oi)), (gi, oi)
    assert abs(info["norm_a"] - ref.norm_a) <= 1e-6 * ref.norm_a
    # the subspaces carry the signal (gap ~ exp(-1.9) against 1e-4 noise): they agree
    # with the oracle's far below the noise level
    assert max(angles) < 1e-3, angles
