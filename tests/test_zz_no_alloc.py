"""The allocation-free coupling entry point (static per-device scratch)
against the handle-based one through the C ABI.

Both run the same kernels; the handle is created with max_mm = n_mm, so the
MM-atoms-per-wave chunk is the same and the results agree bitwise.  The bar
is nevertheless the coupling tests' FP32 / FP64 parity bar (relative to the
size of the forces), which is what the contract promises.  Two calls in a
row, the second with a smaller system, show that what the first call left in
the shared scratch does not leak into the second."""
import numpy as np
import pytest

from paper_2201_08110_amd import synth
from tests.gpu_util import torch_cuda

pytestmark = pytest.mark.gpu
K = synth.COULOMB_K


def _dev(torch, a, dt):
    return torch.tensor(np.ascontiguousarray(np.reshape(a, (-1, 3))), dtype=dt, device="cuda")


def _system(n_mm):
    s = synth.coupling_system(seed=5, n_mm=n_mm)
    return s.x_nnp, s.par_nnp, s.x_mm, s.par_mm


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_noalloc_matches_handle(prec):
    torch = torch_cuda()
    from paper_2201_08110_amd.nnp import Coupling, coupling_noalloc
    dt = torch.float64 if prec == "fp64" else torch.float32
    for n_mm, cutoff in ((47648, 0.0), (3000, 9.0)):      # second call smaller
        xn, pn, xm, pm = (_dev(torch, a, dt) for a in _system(n_mm))
        print(f"noalloc {prec}: n_nnp={xn.shape[0]} n_mm={n_mm} cutoff={cutoff}", flush=True)
        c = Coupling(xn.shape[0], n_mm, K, cutoff, prec)
        E0, Fn0, Fm0 = c(xn, pn, xm, pm)
        # outputs pre-filled with garbage: the call must overwrite them
        E1 = torch.full((1,), 7.0, dtype=torch.float64, device="cuda")
        Fn1 = torch.full_like(xn, 3.0)
        Fm1 = torch.full_like(xm, -2.0)
        coupling_noalloc(xn, pn, xm, pm, K, cutoff, out=(E1, Fn1, Fm1))
        torch.cuda.synchronize()
        E0, E1 = float(E0.cpu()[0]), float(E1.cpu()[0])
        Fn0, Fm0, Fn1, Fm1 = (t.double().cpu().numpy() for t in (Fn0, Fm0, Fn1, Fm1))
        scale = max(np.abs(Fn0).max(), np.abs(Fm0).max())
        tol_e, tol_f = (1e-11, 1e-10) if prec == "fp64" else (5e-6, 1e-4)
        assert abs(E1 - E0) <= tol_e * abs(E0)
        np.testing.assert_allclose(Fn1, Fn0, rtol=0, atol=tol_f * scale)
        np.testing.assert_allclose(Fm1, Fm0, rtol=0, atol=tol_f * scale)
        # the same chunk rule on both sides: the sums run in the same order
        assert E1 == E0 and np.array_equal(Fn1, Fn0) and np.array_equal(Fm1, Fm0)
        # accumulating onto the previous result doubles it exactly (x + x)
        acc = (torch.tensor([E1], dtype=torch.float64, device="cuda"),
               torch.tensor(Fn1, dtype=dt, device="cuda"), torch.tensor(Fm1, dtype=dt, device="cuda"))
        coupling_noalloc(xn, pn, xm, pm, K, cutoff, out=acc, accumulate=True)
        torch.cuda.synchronize()
        assert float(acc[0].cpu()[0]) == 2 * E1
        assert np.array_equal(acc[1].double().cpu().numpy(), 2 * Fn1)
        assert np.array_equal(acc[2].double().cpu().numpy(), 2 * Fm1)
        c.close()


def test_noalloc_rejects_oversize():
    torch = torch_cuda()
    from paper_2201_08110_amd.nnp import NNPError, coupling_noalloc
    # 1024 NNP atoms x 2^22 MM atoms needs far more than the 8 MiB scratch
    xn = torch.zeros((1024, 3), dtype=torch.float64, device="cuda")
    xm = torch.zeros((1 << 22, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(NNPError) as ei:
        coupling_noalloc(xn, xn, xm, xm, K, 0.0)
    assert ei.value.code == 3
