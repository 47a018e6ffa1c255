"""Tunable kernel variants and the autotuner, through the C ABI.

Every candidate of every knob must reproduce the FP64 oracle to the same
bar as the default path (the knobs change speed, not results), and the
autotuner's choice must round-trip through its cache file."""
import itertools
import json

import numpy as np
import pytest

from paper_2201_08110_amd import synth
from tests.gpu_util import BF16_FORCE_RMS_FRAC, bf16_de_bar, errors, make_handle, oracle_inputs, to_device, torch_cuda

pytestmark = pytest.mark.gpu

# molecules above and below the cell thresholds tried, plus a one-atom one
SIZES = [70, 1, 33, 150]
VARIANTS = [dict(mlp_path=m, gemm_stages=g, cell_min=c, tail_tile=1)
            for m, g, c in itertools.product([1, 2], [2, 3], [32, 1024])]
VARIANTS += [dict(mlp_path=1, gemm_stages=2, cell_min=128, tail_tile=t) for t in (2, 3)]
VARIANTS += [dict(mlp_path=1, gemm_stages=g, cell_min=128, tail_tile=1, gemm_waves=8) for g in (2, 3)]
VARIANTS += [dict(mlp_path=2, gemm_stages=2, cell_min=c, tail_tile=1, gemm_waves=4, atom_chunk=a)
             for a, c in ((16, 32), (8, 1024), (4, 128))]
# the force kernel with the dE/dAEV row staged in LDS (global reads by default)
VARIANTS += [dict(mlp_path=1, gemm_stages=2, cell_min=c, tail_tile=1, atom_chunk=a, force_path=1)
             for a, c in ((16, 32), (4, 1024))]


def _batch():
    return synth.random_batch(71, SIZES)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_every_variant_matches_oracle(orc, hp, prec):
    torch = torch_cuda()
    b = _batch()
    M = 2
    w = synth.xavier_weights(M, hp["widths"], seed=47)
    # FP32 handles above 256 atoms batch with 128-row tiles
    h = make_handle(hp, w, M, prec, b, max_atoms=512 if prec == "fp32" else None)
    xo, wo = oracle_inputs(b, w, prec)
    Eo, Fo = orc.energy_forces(hp, wo, M, b.species, xo, b.mol_offsets)
    dt = torch.float64 if prec == "fp64" else torch.float32
    x, sp, off = to_device(torch, b, dt)
    for var in VARIANTS:
        for k, v in var.items():
            h.set_knob(k, v)
        assert {k: h.get_knob(k) for k in var} == var
        E, F = h.energy_forces(x, sp, off)
        torch.cuda.synchronize()
        assert h.device_status() == 0
        E, F = E.cpu().numpy(), F.double().cpu().numpy()
        case = f"{prec} " + " ".join(f"{k}={v}" for k, v in var.items())
        if prec == "fp64":
            np.testing.assert_allclose(E, Eo, rtol=1e-10, err_msg=case)
            np.testing.assert_allclose(F, Fo, rtol=1e-8, atol=1e-9 * np.abs(Fo).max(), err_msg=case)
        else:
            dE, rmse = errors(E, F, Eo, Fo, b.mol_offsets)
            print(case, "|dE|/atom", dE.max(), "RMSE", rmse.max())
            assert dE.max() <= 1e-4 and rmse.max() <= 1e-3, case


def test_bf16_paths_agree(hp):
    """BF16 fused and per-layer network paths round the same operands: their
    energies agree far inside the BF16-vs-oracle bound."""
    torch = torch_cuda()
    b = synth.config_batch(5, n_mols=12)
    w = synth.xavier_weights(8, hp["widths"])
    h = make_handle(hp, w, 8, "bf16", b, max_atoms=1024)
    x, sp, off = to_device(torch, b, torch.float32)
    out = {}
    for mlp in (1, 2):
        h.set_knob("mlp_path", mlp)
        E, F = h.energy_forces(x, sp, off)
        torch.cuda.synchronize()
        out[mlp] = (E.cpu().numpy(), F.double().cpu().numpy())
    dE = np.abs(out[1][0] - out[2][0]) / 48.0
    print("bf16 fused vs per-layer |dE|/atom", dE.max())
    assert dE.max() <= 0.05
    frms = np.sqrt(np.mean(out[2][1] ** 2))
    assert np.sqrt(np.mean((out[1][1] - out[2][1]) ** 2)) <= 5e-3 * frms


def test_knob_validation(hp):
    torch_cuda()
    from paper_2201_08110_amd.nnp import NNP_E_INVALID, NNPError
    b = _batch()
    w = synth.xavier_weights(1, hp["widths"])
    h = make_handle(hp, w, 1, "fp32", b)
    for name, bad in (("mlp_path", 3), ("gemm_stages", 4), ("cell_min", 8), ("cell_min", 5000)):
        with pytest.raises(NNPError) as ei:
            h.set_knob(name, bad)
        assert ei.value.code == NNP_E_INVALID
    h.set_knob("cell_min", 0)
    assert h.get_knob("cell_min") == 128


def test_autotune_choice_and_cache(orc, hp, tmp_path):
    torch = torch_cuda()
    b = _batch()
    M = 2
    w = synth.xavier_weights(M, hp["widths"], seed=47)
    cache = tmp_path / "tune.jsonl"
    x, sp, off = to_device(torch, b, torch.float32)
    h = make_handle(hp, w, M, "fp32", b, max_atoms=512)
    rep = h.autotune(x, sp, off, reps=2, cache_path=str(cache))
    print(json.dumps(rep))
    assert rep["cached"] is False
    for k, v in rep["chosen"].items():
        assert h.get_knob(k) == v
    assert any(k.startswith("mlp_path=") for k in rep["timings_us"])
    lines = cache.read_text().strip().splitlines()
    assert len(lines) == 1 and json.loads(lines[0])["key"] == rep["key"]
    # a second handle of the same shape takes the cached choice without timing
    h2 = make_handle(hp, w, M, "fp32", b, max_atoms=512)
    rep2 = h2.autotune(x, sp, off, reps=2, cache_path=str(cache))
    assert rep2["cached"] is True and rep2["chosen"] == rep["chosen"] and rep2["timings_us"] == {}
    assert len(cache.read_text().strip().splitlines()) == 1
    # the tuned handle still meets the FP32 bar
    xo, wo = oracle_inputs(b, w, "fp32")
    Eo, Fo = orc.energy_forces(hp, wo, M, b.species, xo, b.mol_offsets)
    E, F = h2.energy_forces(x, sp, off)
    torch.cuda.synchronize()
    dE, rmse = errors(E.cpu().numpy(), F.double().cpu().numpy(), Eo, Fo, b.mol_offsets)
    assert dE.max() <= 1e-4 and rmse.max() <= 1e-3


def test_bf16_layer1_paths(orc, hp):
    """Layer-1 GEMMs with both operands staged through LDS (path 1) and with
    the weights in registers (path 2, 2 and 3 LDS stages) on a ragged batch of
    several element buckets: each against the FP64 oracle at the BF16 bar, and
    against each other (same BF16 operands, FP32 sums in another order)."""
    torch = torch_cuda()
    b = synth.random_batch(72, [64, 300, 17, 219, 150])
    M = 8
    w = synth.xavier_weights(M, hp["widths"], seed=48)
    h = make_handle(hp, w, M, "bf16", b, max_atoms=1024)
    assert h.get_knob("l1_path") == 2
    x, sp, off = to_device(torch, b, torch.float32)
    xo, wo = oracle_inputs(b, w, "bf16")
    Eo, Fo = orc.energy_forces(hp, wo, M, b.species, xo, b.mol_offsets)
    frms = np.sqrt(np.mean(Fo ** 2))
    out = {}
    for path, stages in ((1, 2), (2, 2), (2, 3)):
        h.set_knob("l1_path", path)
        h.set_knob("gemm_stages", stages)
        E, F = h.energy_forces(x, sp, off)
        torch.cuda.synchronize()
        assert h.device_status() == 0
        E, F = E.cpu().numpy(), F.double().cpu().numpy()
        dE, rmse = errors(E, F, Eo, Fo, b.mol_offsets)
        print("bf16 l1_path", path, "stages", stages, "|dE|/atom", dE.max(), "RMSE", rmse.max(), "RMS(F)", frms)
        assert dE.max() <= bf16_de_bar(M) and rmse.max() <= BF16_FORCE_RMS_FRAC * frms
        out[(path, stages)] = (E, F)
    n_at = np.diff(b.mol_offsets)
    for key in ((2, 2), (2, 3)):
        dE = np.abs(out[key][0] - out[(1, 2)][0]) / np.maximum(n_at, 1)
        assert dE.max() <= 0.05, key
        assert np.sqrt(np.mean((out[key][1] - out[(1, 2)][1]) ** 2)) <= 5e-3 * frms, key


def test_layer1_path_knob_support(hp):
    """The register-weight layer-1 path exists for BF16 handles only: FP32
    handles run path 1 and refuse path 2 with NNP_E_UNSUPPORTED."""
    torch_cuda()
    from paper_2201_08110_amd import nnp
    b = synth.config_batch(5, n_mols=8)
    w = synth.xavier_weights(2, hp["widths"])
    h32 = make_handle(hp, w, 2, "fp32", b, max_atoms=1024)
    assert h32.get_knob("l1_path") == 1
    with pytest.raises(nnp.NNPError) as ei:
        h32.set_knob("l1_path", 2)
    assert ei.value.code == nnp.NNP_E_UNSUPPORTED
    h16 = make_handle(hp, w, 2, "bf16", b, max_atoms=1024)
    assert h16.get_knob("l1_path") == 2
    h16.set_knob("l1_path", 1)
    assert h16.get_knob("l1_path") == 1
