"""Helpers of the GPU tests: build a library handle and the matching oracle call."""
from __future__ import annotations

import numpy as np

from paper_2201_08110_amd import synth


def torch_cuda():
    import pytest
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def make_handle(hp, weights, M, precision, batch, max_atoms=None, max_mols=None, max_apm=None,
                sae=None):
    from paper_2201_08110_amd.nnp import NNP
    sizes = np.diff(batch.mol_offsets)
    return NNP(hp, weights, M, precision,
               max_atoms=max_atoms or max(int(batch.n_atoms), 1),
               max_mols=max_mols or int(batch.n_mols),
               max_atoms_per_mol=max_apm or max(int(sizes.max()) if len(sizes) else 1, 1),
               sae=sae)


def to_device(torch, batch, dtype):
    x = torch.tensor(batch.coords, dtype=dtype, device="cuda")
    sp = torch.tensor(batch.species, dtype=torch.int32, device="cuda")
    off = torch.tensor(batch.mol_offsets, dtype=torch.int32, device="cuda")
    return x, sp, off


def oracle_inputs(batch, weights, precision):
    """What the GPU path really computes with: FP32-rounded coordinates and
    weights for FP32/BF16 handles (BF16 errors are stated against the FP32
    rounding of the FP64 master weights), exact values for FP64."""
    if precision == "fp64":
        return batch.coords, weights
    return synth.round_to_fp32(batch.coords), synth.round_to_fp32(weights)


def errors(E, F, Eo, Fo, offsets):
    """Per-molecule |dE|/atoms and force RMSE (kcal/mol, kcal/mol/A)."""
    sizes = np.diff(offsets)
    dE = np.abs(E - Eo) / np.maximum(sizes, 1)
    rmse = np.array([np.sqrt(np.mean((F[a:b] - Fo[a:b]) ** 2)) if b > a else 0.0
                     for a, b in zip(offsets[:-1], offsets[1:])])
    return dE, rmse
