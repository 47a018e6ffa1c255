"""The pipelined evaluation (two halves of the batch on two streams) against
the single-stream evaluation of the same handle: bitwise equal with
fixed-point force sums (the parts are independent sub-batches; every result
is summed in a fixed order), eager and graph-replayed, for ragged batches,
odd molecule counts, an empty half, accumulation and an element table; and
against the FP64 oracle on sampled molecules."""
import numpy as np
import pytest

from paper_2201_08110_amd import synth
from tests.gpu_util import (BF16_FORCE_RMS_FRAC, bf16_de_bar, errors, sub_batch, to_device,
                            torch_cuda)

pytestmark = pytest.mark.gpu


def _pair(hp, w, M, prec, b, apm, **kw):
    from paper_2201_08110_amd.nnp import NNP
    hs = []
    for pipe in (1, 2):
        h = NNP(hp, w, M, prec, max_atoms=max(b.n_atoms, 4096), max_mols=b.n_mols,
                max_atoms_per_mol=apm, **kw)
        h.set_knob("pipeline", pipe)
        h.set_knob("force_sum", 2)
        assert h.get_knob("pipeline") == pipe
        hs.append(h)
    return hs


@pytest.mark.parametrize("prec,sizes", [
    ("bf16", None),                                  # the 512-molecule ragged workload
    ("fp32", [37, 120, 1, 64, 99]),                  # odd molecule count
    ("fp32", [150, 0]),                              # the second half empty
    ("bf16", [0, 3, 48, 48, 48, 11, 130]),
])
def test_pipeline_equals_single_stream(orc, hp, prec, sizes):
    torch = torch_cuda()
    b = synth.config_batch(3) if sizes is None else synth.random_batch(101, sizes)
    M = 8 if sizes is None else 4
    w = synth.xavier_weights(M, hp["widths"], seed=102)
    apm = max(int(np.diff(b.mol_offsets).max()), 1)
    h1, h2 = _pair(hp, w, M, prec, b, apm)
    x, sp, off = to_device(torch, b, torch.float32)
    E1, F1 = h1.energy_forces(x, sp, off)
    E2, F2 = h2.energy_forces(x, sp, off)
    torch.cuda.synchronize()
    assert h1.device_status() == 0 and h2.device_status() == 0
    assert np.array_equal(E1.cpu().numpy(), E2.cpu().numpy())
    assert np.array_equal(F1.cpu().numpy(), F2.cpu().numpy())
    # graph replays and accumulation through the pipelined path
    s = torch.cuda.Stream()
    Eg = torch.zeros(b.n_mols, dtype=torch.float64, device="cuda")
    Fg = torch.zeros_like(x)
    torch.cuda.synchronize()
    for it in range(3):
        with torch.cuda.stream(s):
            h2.energy_forces(x, sp, off, out=(Eg, Fg), graph=True, stream=s, accumulate=True)
        s.synchronize()
    assert h2.device_status() == 0
    np.testing.assert_allclose(Eg.cpu().numpy(), 3 * E1.cpu().numpy(), rtol=1e-14,
                               atol=1e-12 * max(1.0, float(E1.abs().max())))
    np.testing.assert_allclose(Fg.cpu().numpy(), 3 * F1.cpu().numpy(), rtol=1e-6,
                               atol=1e-5 * float(F1.abs().max()))
    # the oracle on sampled molecules
    sizes_ = np.diff(b.mol_offsets)
    pick = [m for m in sorted({0, b.n_mols - 1, int(np.argmax(sizes_)), b.n_mols // 2}) if sizes_[m] > 0]
    spc, xc, soff, rows = sub_batch(b, pick)
    Eo, Fo = orc.energy_forces(hp, synth.round_to_fp32(w), M, spc, synth.round_to_fp32(xc), soff)
    dE, rmse = errors(E2.cpu().numpy()[pick], F2.double().cpu().numpy()[rows], Eo, Fo, soff)
    print(prec, "pipelined: |dE|/atom", dE.max(), "RMSE", rmse.max())
    if prec == "fp32":
        assert dE.max() <= 1e-4 and rmse.max() <= 1e-3
    else:
        assert dE.max() <= bf16_de_bar(M) and rmse.max() <= BF16_FORCE_RMS_FRAC * np.sqrt(np.mean(Fo ** 2))


def test_pipeline_with_element_table(hp):
    torch = torch_cuda()
    b = synth.random_batch(103, [40, 61, 7, 90])
    w = synth.xavier_weights(2, hp["widths"], seed=104)
    Z = np.array((1, 6, 7, 8, 9, 16, 17), dtype=np.int32)
    h1, h2 = _pair(hp, w, 2, "bf16", b, 90, atomic_numbers=Z)
    x, _, off = to_device(torch, b, torch.float32)
    zt = torch.tensor(Z[b.species], dtype=torch.int32, device="cuda")
    E1, F1 = h1.energy_forces(x, zt, off)
    E2, F2 = h2.energy_forces(x, zt, off)
    torch.cuda.synchronize()
    assert h1.device_status() == 0 and h2.device_status() == 0
    assert np.array_equal(E1.cpu().numpy(), E2.cpu().numpy())
    assert np.array_equal(F1.cpu().numpy(), F2.cpu().numpy())
    bad = zt.clone()
    bad[45] = 2
    h2.energy_forces(x, bad, off)
    from paper_2201_08110_amd.nnp import NNP_E_SPECIES
    assert h2.device_status() == NNP_E_SPECIES
