"""Training backward (parameter gradients) through the C ABI and the
torch.autograd.Function, against the FP64 oracle and finite differences.

Loss of the training workload: L = mean_b (E_b - Et_b)^2 + 0.1 mean (F - Ft)^2
with seeded targets; its cotangents are gE = 2 (E - Et) / B and
gF = 0.2 (F - Ft) / (3 A).
"""
import numpy as np
import pytest

from paper_2201_08110_amd import synth
from tests.gpu_util import make_handle, oracle_inputs, to_device, torch_cuda

pytestmark = pytest.mark.gpu


def _cotangents(seed, B, A):
    rng = np.random.default_rng(seed)
    return rng.normal(size=B) * 1e-2, rng.normal(size=(A, 3)) * 1e-2


def _relerr(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("with_force_term,chunk", [(False, 0), (True, 0), (True, 16)])
def test_param_grad_fp64_matches_oracle(orc, hp, with_force_term, chunk):
    torch = torch_cuda()
    b = synth.random_batch(31, [7, 12, 9])
    M = 2
    w = synth.xavier_weights(M, hp["widths"], seed=41)
    h = make_handle(hp, w, M, "fp64", b)
    if chunk:
        h.set_knob("atom_chunk", chunk)
    x, sp, off = to_device(torch, b, torch.float64)
    gE, gF = _cotangents(1, b.n_mols, b.n_atoms)
    if not with_force_term:
        gF = np.zeros_like(gF)
    gEt = torch.tensor(gE, dtype=torch.float64, device="cuda")
    gFt = torch.tensor(gF, dtype=torch.float64, device="cuda") if with_force_term else None
    gp, _ = h.backward(x, sp, off, gEt, gFt)
    torch.cuda.synchronize()
    assert h.device_status() == 0
    go = orc.param_grad(hp, w, M, b.species, b.coords, b.mol_offsets, gE, gF)
    err = _relerr(gp.cpu().numpy(), go)
    print("fp64 param grad rel err", err)
    assert err < 1e-10
    np.testing.assert_allclose(gp.cpu().numpy(), go, rtol=1e-8, atol=1e-10 * np.abs(go).max())


def test_param_grad_fp32_training_batch(orc, hp):
    """Workload 4 shape (molecules of 30-80 atoms, 8 models), FP32, 8 molecules."""
    torch = torch_cuda()
    b = synth.config_batch(4, n_mols=8)
    M = 8
    w = synth.xavier_weights(M, hp["widths"])
    h = make_handle(hp, w, M, "fp32", b)
    x, sp, off = to_device(torch, b, torch.float32)
    gE, gF = _cotangents(2, b.n_mols, b.n_atoms)
    gp, _ = h.backward(x, sp, off, torch.tensor(gE, dtype=torch.float64, device="cuda"),
                       torch.tensor(gF, dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()
    assert h.device_status() == 0
    xo, wo = oracle_inputs(b, w, "fp32")
    go = orc.param_grad(hp, wo, M, b.species, xo, b.mol_offsets, gE, synth.round_to_fp32(gF))
    err = _relerr(gp.cpu().numpy().astype(np.float64), go)
    print("fp32 param grad rel err", err)
    assert err < 1e-4


def test_grad_coords_energy_only(orc, hp):
    torch = torch_cuda()
    b = synth.random_batch(33, [10, 6])
    M = 2
    w = synth.xavier_weights(M, hp["widths"], seed=43)
    h = make_handle(hp, w, M, "fp64", b)
    x, sp, off = to_device(torch, b, torch.float64)
    gE = np.array([0.3, -1.1])
    gp, gx = h.backward(x, sp, off, torch.tensor(gE, dtype=torch.float64, device="cuda"), None,
                        want_coords=True)
    torch.cuda.synchronize()
    _, Fo = orc.energy_forces(hp, w, M, b.species, b.coords, b.mol_offsets)
    mol = np.repeat(np.arange(b.n_mols), np.diff(b.mol_offsets))
    np.testing.assert_allclose(gx.cpu().numpy(), -gE[mol][:, None] * Fo, rtol=1e-9, atol=1e-9)


def test_autograd_function_and_finite_differences(hp):
    """torch autograd over the library: parameter gradients of the training
    loss and coordinate gradients of an energy-only loss, checked by central
    differences of the same FP64 evaluation (16 weights, 16 coordinates)."""
    torch = torch_cuda()
    from paper_2201_08110_amd.autograd import nnp_energy_forces
    b = synth.random_batch(35, [8, 11])
    M = 2
    w = synth.xavier_weights(M, hp["widths"], seed=44)
    h = make_handle(hp, w, M, "fp64", b)
    x, sp, off = to_device(torch, b, torch.float64)
    rng = np.random.default_rng(5)
    Et = torch.tensor(rng.normal(size=b.n_mols) * 50.0, dtype=torch.float64, device="cuda")
    Ft = torch.tensor(rng.normal(size=(b.n_atoms, 3)) * 20.0, dtype=torch.float64, device="cuda")
    params = torch.tensor(w, dtype=torch.float64, requires_grad=True)

    def loss_fn(p, xx):
        E, F = nnp_energy_forces(h, xx, p, sp, off)
        return ((E - Et) ** 2).mean() + 0.1 * ((F - Ft) ** 2).mean()

    L = loss_fn(params, x)
    L.backward()
    g = params.grad.numpy()
    hw = 1e-5
    idx = np.concatenate([np.argsort(-np.abs(g))[:8], rng.integers(0, w.size, 8)])
    for k in idx:
        wp, wm = w.copy(), w.copy()
        wp[k] += hw
        wm[k] -= hw
        with torch.no_grad():
            lp = loss_fn(torch.tensor(wp), x).item()
            lm = loss_fn(torch.tensor(wm), x).item()
        fd = (lp - lm) / (2 * hw)
        assert g[k] == pytest.approx(fd, rel=1e-5, abs=1e-9), k

    # energy-only loss: dL/dx through the function, vs central differences (h = 1e-4 A)
    xg = x.clone().requires_grad_(True)
    E, _ = nnp_energy_forces(h, xg, params.detach(), sp, off)
    LE = ((E - Et) ** 2).sum()
    LE.backward()
    gx = xg.grad.cpu().numpy()
    hx = 1e-4
    for a, c in zip(rng.integers(0, b.n_atoms, 16), rng.integers(0, 3, 16)):
        xp, xm = x.clone(), x.clone()
        xp[a, c] += hx
        xm[a, c] -= hx
        with torch.no_grad():
            Ep, _ = nnp_energy_forces(h, xp, params.detach(), sp, off)
            Em, _ = nnp_energy_forces(h, xm, params.detach(), sp, off)
        fd = (((Ep - Et) ** 2).sum() - ((Em - Et) ** 2).sum()).item() / (2 * hx)
        assert gx[a, c] == pytest.approx(fd, rel=1e-5, abs=1e-6)


@pytest.mark.parametrize("prec,which,knobs", [
    ("fp64", "ani2x", {}), ("fp64", "ani1x_elements", {}), ("fp32", "ani2x", {}),
    ("fp64", "ani2x", {"cell_min": 16, "atom_chunk": 16})])
def test_force_loss_coordinate_gradient(hp, prec, which, knobs):
    """dL/dx = -gE F - H gF against the FP64 Hessian-vector oracle (torch,
    pinned to the C oracle and to differences of its forces).  FP64: 1e-9
    relative in norm; FP32: 2e-4 (second derivatives of single-precision
    featuriser terms)."""
    torch = torch_cuda()
    pytest.importorskip("torch")
    from oracle import hessian
    if which == "ani2x":
        h_, ratio = hp, synth.LIGAND_RATIO
        w = synth.xavier_weights(2, hp["widths"], seed=45)
    else:
        h_, ratio = synth.ani1x_hparams(), (30, 20, 5, 5)
        w = synth.xavier_weights(2, h_["species_widths"], n_species=4, seed=45)
    b = synth.random_batch(36, [9, 14, 1, 6], box_scale=1.9, ratio=ratio)
    h = make_handle(h_, w, 2, prec, b)
    for k, v in knobs.items():   # cutoff-cell neighbour lists above 16 atoms, 16-atom chunks
        h.set_knob(k, v)
    dt = torch.float64 if prec == "fp64" else torch.float32
    x, sp, off = to_device(torch, b, dt)
    gE, gF = _cotangents(4, b.n_mols, b.n_atoms)
    _, gx = h.backward(x, sp, off, torch.tensor(gE, dtype=torch.float64, device="cuda"),
                       torch.tensor(gF, dtype=dt, device="cuda"), want_coords=True)
    torch.cuda.synchronize()
    assert h.device_status() == 0
    xo, wo = oracle_inputs(b, w, prec)
    gFo = gF if prec == "fp64" else synth.round_to_fp32(gF)
    go = hessian.coord_grad(h_, wo, 2, b.species, xo, b.mol_offsets, gE, gFo)
    err = _relerr(gx.double().cpu().numpy(), go)
    print(prec, which, "force-loss dL/dx rel err", err)
    assert err < (1e-9 if prec == "fp64" else 2e-4)


def test_force_loss_autograd_double_backward(hp):
    """Through the autograd Function: d/dx of a force loss equals the C ABI's
    coordinate gradient (FP64)."""
    torch = torch_cuda()
    from paper_2201_08110_amd.autograd import nnp_energy_forces
    b = synth.random_batch(37, [7, 5])
    w = synth.xavier_weights(1, hp["widths"], seed=46)
    h = make_handle(hp, w, 1, "fp64", b)
    x, sp, off = to_device(torch, b, torch.float64)
    xg = x.clone().requires_grad_(True)
    params = torch.tensor(w, dtype=torch.float64)
    E, F = nnp_energy_forces(h, xg, params, sp, off)
    ((F ** 2).sum() + 0.3 * E.sum()).backward()
    gE = torch.full((b.n_mols,), 0.3, dtype=torch.float64, device="cuda")
    _, gx = h.backward(x, sp, off, gE, 2 * F.detach(), want_coords=True)
    torch.cuda.synchronize()
    np.testing.assert_allclose(xg.grad.cpu().numpy(), gx.cpu().numpy(), rtol=1e-12, atol=1e-12)
