"""Parity at the full sizes of the ragged-batch and training workloads, and
the neighbour-list overflow flag.

Ragged batch: 512 molecules of 10-120 atoms (31,719 atoms), 8 models, FP32
and BF16 networks, one handle sized for the whole batch and evaluated through
captured-graph replays (as the benchmark runs it).  34 molecules (the
smallest, the largest and 32 seeded ones) are compared with the FP64 oracle
at the FP32 bars (|dE|/atom <= 1e-4 kcal/mol, force RMSE <= 1e-3 kcal/mol/A)
or the BF16 bars; every molecule's net force vanishes (translation
invariance: each pair and triple term acts on its atoms with opposite signs).

Training: all 64 molecules of 30-80 atoms (3,514 atoms), 8 models, FP32, the
loss of the workload (energy MSE + 0.1 force MSE against the energies and
forces of a second seeded ensemble).  dL/dW is compared with the oracle block
by block -- every (model, element, layer) weight matrix and bias vector on
its own -- so that an error in one element's or one layer's gradient cannot
hide in the norm of 19 M parameters.
"""
import numpy as np
import pytest

from paper_2201_08110_amd import synth
from tests.gpu_util import (BF16_FORCE_RMS_FRAC, bf16_de_bar, errors, sub_batch, to_device,
                            torch_cuda)

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_ragged_512_full_size(orc, hp, prec):
    torch = torch_cuda()
    from paper_2201_08110_amd.nnp import NNP
    b = synth.config_batch(3)
    assert b.n_mols == 512
    sizes = np.diff(b.mol_offsets)
    M = 8
    w = synth.xavier_weights(M, hp["widths"])
    h = NNP(hp, w, M, prec, max_atoms=b.n_atoms, max_mols=b.n_mols, max_atoms_per_mol=120)
    x, sp, off = to_device(torch, b, torch.float32)
    s = torch.cuda.Stream()
    E = torch.empty(b.n_mols, dtype=torch.float64, device="cuda")
    F = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(3):                       # eager + capture, then two replays
        with torch.cuda.stream(s):
            E.fill_(float("nan"))
            F.fill_(float("nan"))
            h.energy_forces(x, sp, off, out=(E, F), graph=True, stream=s)
        s.synchronize()
    assert h.device_status() == 0
    E, F = E.cpu().numpy(), F.double().cpu().numpy()
    assert np.all(np.isfinite(E)) and np.all(np.isfinite(F))
    o = np.asarray(b.mol_offsets)
    net = np.add.reduceat(F, o[:-1], axis=0)
    print(prec, "ragged 512: max |net force| / max |F|", np.abs(net).max() / np.abs(F).max())
    assert np.abs(net).max() <= 1e-5 * np.abs(F).max()
    pick = sorted({int(np.argmin(sizes)), int(np.argmax(sizes))}
                  | set(np.random.default_rng(13).choice(b.n_mols, 32, replace=False).tolist()))
    assert len(pick) >= 33
    spc, xc, soff, rows = sub_batch(b, pick)
    Eo, Fo = orc.energy_forces(hp, synth.round_to_fp32(w), M, spc, synth.round_to_fp32(xc), soff)
    dE, rmse = errors(E[pick], F[rows], Eo, Fo, soff)
    frms = np.sqrt(np.mean(Fo ** 2))
    print(prec, f"ragged 512, {len(pick)} sampled molecules ({sizes[pick].min()}-{sizes[pick].max()} atoms):",
          "|dE|/atom max", dE.max(), "median", np.median(dE), "force RMSE max", rmse.max(), "RMS(F)", frms)
    if prec == "fp32":
        assert dE.max() <= 1e-4 and rmse.max() <= 1e-3
    else:
        assert dE.max() <= bf16_de_bar(M) and rmse.max() <= BF16_FORCE_RMS_FRAC * frms


def _blocks(hp, M, S=7):
    """(model, element, name, start, stop) of every weight matrix and bias
    vector in the packed parameter layout."""
    wd = hp["widths"]
    net = synth.net_size(wd)
    out = []
    for m in range(M):
        for s in range(S):
            p = (m * S + s) * net
            for layer in range(len(wd) - 1):
                nW = wd[layer] * wd[layer + 1]
                out.append((m, s, f"W{layer + 1}", p, p + nW))
                p += nW
                out.append((m, s, f"b{layer + 1}", p, p + wd[layer + 1]))
                p += wd[layer + 1]
    return out


def test_training_full_size_param_grad_per_block(orc, hp):
    torch = torch_cuda()
    from paper_2201_08110_amd.nnp import NNP
    b = synth.config_batch(4)
    assert b.n_mols == 64
    M = 8
    w = synth.xavier_weights(M, hp["widths"])
    wt = synth.xavier_weights(M, hp["widths"], seed=synth.W_SEED + 1)
    xo, wo = synth.round_to_fp32(b.coords), synth.round_to_fp32(w)
    # the workload's loss: targets from a second seeded ensemble (FP64 oracle)
    Et, Ft = orc.energy_forces(hp, wt, M, b.species, b.coords, b.mol_offsets)
    E0, F0 = orc.energy_forces(hp, wo, M, b.species, xo, b.mol_offsets)
    gE = 2.0 * (E0 - Et) / b.n_mols
    gF = synth.round_to_fp32(0.2 * (F0 - Ft) / (3 * b.n_atoms))
    h = NNP(hp, w, M, "fp32", max_atoms=b.n_atoms, max_mols=b.n_mols, max_atoms_per_mol=80,
            training=True)
    x, sp, off = to_device(torch, b, torch.float32)
    gp, _ = h.backward(x, sp, off, torch.tensor(gE, dtype=torch.float64, device="cuda"),
                       torch.tensor(gF, dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()
    assert h.device_status() == 0
    gp = gp.cpu().numpy().astype(np.float64)
    go = orc.param_grad(hp, wo, M, b.species, xo, b.mol_offsets, gE, gF)
    worst = (0.0, None)
    for m, s, name, a, z in _blocks(hp, M):
        g, r = gp[a:z], go[a:z]
        nr = np.linalg.norm(r)
        assert nr > 0, (m, s, name)
        rel = np.linalg.norm(g - r) / nr
        if rel > worst[0]:
            worst = (rel, (m, s, name))
        # per block: relative error of the block, then every element against
        # FP32 rounding of its row sum (1e-3 relative) plus 1e-4 of the block's
        # largest entry for elements that cancel to near zero
        assert rel <= 1e-4, (m, s, name, rel)
        np.testing.assert_allclose(g, r, rtol=1e-3, atol=1e-4 * np.abs(r).max(), err_msg=f"{(m, s, name)}")
    print("training full size: worst per-block relative error", worst,
          "global", np.linalg.norm(gp - go) / np.linalg.norm(go))


@pytest.mark.parametrize("cell_min", [0, 1024])
def test_neighbour_overflow_sets_capacity_flag(hp, cell_min):
    """An atom with more neighbours within rcr than a list holds (192 here)
    raises NNP_E_CAPACITY on the device flag; both neighbour kernels (cutoff
    cells above cell_min atoms, all pairs below) bound their writes by the
    list length.  300 atoms uniform in a 6 A cube (no minimum distance) give
    ~250 neighbours to a central atom.  A normal batch afterwards runs clean."""
    torch = torch_cuda()
    from paper_2201_08110_amd.nnp import NNP, NNP_E_CAPACITY
    rng = np.random.default_rng(21)
    n = 300
    xd = rng.uniform(0.0, 6.0, size=(n, 3))
    spd = rng.integers(0, 7, size=n).astype(np.int32)
    w = synth.xavier_weights(1, hp["widths"], seed=81)
    h = NNP(hp, w, 1, "fp32", max_atoms=n, max_mols=2, max_atoms_per_mol=n)
    if cell_min:
        h.set_knob("cell_min", cell_min)
    x = torch.tensor(xd, dtype=torch.float32, device="cuda")
    sp = torch.tensor(spd, dtype=torch.int32, device="cuda")
    off = torch.tensor([0, n], dtype=torch.int32, device="cuda")
    h.energy_forces(x, sp, off)
    assert h.device_status() == NNP_E_CAPACITY
    ok = synth.random_batch(22, [40, 60])
    x2, sp2, off2 = to_device(torch, ok, torch.float32)
    E, F = h.energy_forces(x2, sp2, off2)
    assert h.device_status() == 0
    assert np.all(np.isfinite(E.cpu().numpy())) and np.all(np.isfinite(F.cpu().numpy()))
