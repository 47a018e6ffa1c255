"""Ragged batches with device-side counts replaying one captured graph.

A caller keeps capacity-sized device buffers, writes each new batch
(coordinates, element labels, offsets and the {molecules, atoms} counts) into
them and calls with NNP_FLAG_DEVICE_COUNTS | NNP_FLAG_GRAPH.  The graph is
keyed on the rounded launch bounds, so batches of different sizes within the
bounds replay the graph captured for the first one, with no re-capture.  Each
batch matches the FP64 oracle on sampled molecules (FP32 bars) and, with
fixed-point force sums, equals bitwise an eager evaluation with host counts.
"""
import numpy as np
import pytest

from paper_2201_08110_amd import synth
from tests.gpu_util import (BF16_FORCE_RMS_FRAC, bf16_de_bar, errors, sub_batch, to_device,
                            torch_cuda)

pytestmark = pytest.mark.gpu

MAX_MOLS, MAX_ATOMS, MAX_APM = 512, 40000, 120


def _batches():
    b3 = synth.config_batch(3)
    rng = np.random.default_rng(17)
    return [
        b3,                                                          # 512 molecules, 31,719 atoms
        synth.random_batch(91, rng.integers(10, 121, size=300)),     # 300 molecules
        synth.random_batch(92, rng.integers(10, 121, size=357)),     # 357 molecules
    ]


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_device_counts_replay_one_graph(orc, hp, prec):
    torch = torch_cuda()
    from paper_2201_08110_amd.nnp import NNP
    M = 8
    w = synth.xavier_weights(M, hp["widths"])
    h = NNP(hp, w, M, prec, max_atoms=MAX_ATOMS, max_mols=MAX_MOLS, max_atoms_per_mol=MAX_APM)
    ref = NNP(hp, w, M, prec, max_atoms=MAX_ATOMS, max_mols=MAX_MOLS, max_atoms_per_mol=MAX_APM)
    for hh in (h, ref):
        hh.set_knob("force_sum", 2)
    dev = "cuda"
    xb = torch.zeros((MAX_ATOMS, 3), dtype=torch.float32, device=dev)
    spb = torch.zeros(MAX_ATOMS, dtype=torch.int32, device=dev)
    offb = torch.zeros(MAX_MOLS + 1, dtype=torch.int32, device=dev)
    cnt = torch.zeros(2, dtype=torch.int32, device=dev)
    Eb = torch.zeros(MAX_MOLS, dtype=torch.float64, device=dev)
    Fb = torch.zeros((MAX_ATOMS, 3), dtype=torch.float32, device=dev)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    for it, b in enumerate(_batches()):
        A, B = b.n_atoms, b.n_mols
        print(f"{prec} batch {it}: {B} molecules, {A} atoms", flush=True)
        x, sp, off = to_device(torch, b, torch.float32)
        with torch.cuda.stream(s):
            xb[:A].copy_(x)
            spb[:A].copy_(sp)
            offb[:B + 1].copy_(off)
            cnt.copy_(torch.tensor([B, A], dtype=torch.int32))
            Eb.fill_(float("nan"))
            h.energy_forces(xb, spb, offb, out=(Eb, Fb), graph=True, stream=s, counts=cnt,
                            bounds=(MAX_MOLS, MAX_ATOMS))
        s.synchronize()
        assert h.device_status() == 0
        st = h.graph_stats()
        # the first call runs eagerly and captures; every later batch replays
        assert st["captures"] == 1 and st["replays"] == it, st
        E = Eb[:B].cpu().numpy()
        F = Fb[:A].double().cpu().numpy()
        assert np.all(np.isnan(Eb[B:].cpu().numpy()))           # nothing written past the batch
        Er, Fr = ref.energy_forces(x, sp, off)
        torch.cuda.synchronize()
        assert np.array_equal(E, Er.cpu().numpy()) and np.array_equal(F, Fr.double().cpu().numpy())
        sizes = np.diff(b.mol_offsets)
        pick = sorted({int(np.argmin(sizes)), int(np.argmax(sizes))}
                      | set(np.random.default_rng(it).choice(B, 12, replace=False).tolist()))
        spc, xc, soff, rows = sub_batch(b, pick)
        Eo, Fo = orc.energy_forces(hp, synth.round_to_fp32(w), M, spc, synth.round_to_fp32(xc), soff)
        dE, rmse = errors(E[pick], F[rows], Eo, Fo, soff)
        print(f"  |dE|/atom max {dE.max():.3g}, force RMSE max {rmse.max():.3g}")
        if prec == "fp32":
            assert dE.max() <= 1e-4 and rmse.max() <= 1e-3
        else:
            assert dE.max() <= bf16_de_bar(M) and rmse.max() <= BF16_FORCE_RMS_FRAC * np.sqrt(np.mean(Fo ** 2))


def test_device_counts_out_of_bounds_flagged(hp):
    torch = torch_cuda()
    from paper_2201_08110_amd.nnp import NNP, NNP_E_CAPACITY
    b = synth.random_batch(93, [20, 30, 25])
    w = synth.xavier_weights(1, hp["widths"], seed=94)
    h = NNP(hp, w, 1, "fp32", max_atoms=256, max_mols=8, max_atoms_per_mol=64)
    x, sp, off = to_device(torch, b, torch.float32)
    E = torch.zeros(8, dtype=torch.float64, device="cuda")
    F = torch.zeros((256, 3), dtype=torch.float32, device="cuda")
    xb = torch.zeros((256, 3), dtype=torch.float32, device="cuda")
    xb[:b.n_atoms] = x
    spb = torch.zeros(256, dtype=torch.int32, device="cuda")
    spb[:b.n_atoms] = sp
    offb = torch.zeros(9, dtype=torch.int32, device="cuda")
    offb[:4] = off
    for counts, ok in (([3, b.n_atoms], True), ([3, b.n_atoms - 1], False), ([9, b.n_atoms], False),
                       ([3, 300], False), ([-1, 0], False), ([0, 0], True)):
        cnt = torch.tensor(counts, dtype=torch.int32, device="cuda")
        h.energy_forces(xb, spb, offb, out=(E, F), counts=cnt, bounds=(8, 256))
        assert h.device_status() == (0 if ok else NNP_E_CAPACITY), counts
