"""Helpers of the GPU tests: build a library handle and the matching oracle call."""
from __future__ import annotations

import math

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


# ---------------------------------------------------------------------------
# Parity bars of BF16 network GEMMs (FP32 accumulation) against the FP64
# oracle.  Rounding an operand to bf16 (8 significant bits) changes it by a
# relative error uniform in +-2^-9, standard deviation 2^-9/sqrt(3) = 1.13e-3;
# a pre-activation sum_k W_nk a_k with both operands rounded and random-sign
# terms then carries a relative error of sqrt(2) * 1.13e-3 = 1.6e-3.  The three
# BF16 GEMM layers on the way to an atomic energy add such errors
# independently (gain ~1 through random weights and CELU), so a network output
# e_m is off by ~sqrt(3) * 1.6e-3 = 2.8e-3 of its typical size.  The weights'
# rounding is shared by every atom of an element, so the errors of a
# molecule's atoms add coherently: per atom the ensemble mean is off by
# ~2.8e-3 * rms(e_m) / sqrt(M).  With the seeded Xavier networks rms(e_m) is
# ~30 kcal/mol per atom (64-atom ligand, 8 models), giving sigma ~0.03 kcal/mol
# per atom at M = 8 (measured: 0.018-0.029).  The bar is ~3 sigma: 0.1
# kcal/mol per atom at M = 8, scaled by sqrt(8 / M).  Forces: the same
# relative error on a sum dominated by a few large terms, ~0.7% of RMS(F)
# measured; the bar is 1% of RMS(F).
BF16_FORCE_RMS_FRAC = 1e-2


def bf16_de_bar(M: int) -> float:
    """|dE|/atom bar (kcal/mol) of BF16 network GEMMs, M-model ensemble."""
    return 0.1 * math.sqrt(8.0 / M)


def sub_batch(batch, mols):
    """Species, coordinates, offsets and atom rows of the molecules `mols`
    of a batch (for oracle calls on a sample)."""
    o = np.asarray(batch.mol_offsets)
    rows = np.concatenate([np.arange(o[m], o[m + 1]) for m in mols]) if len(mols) else np.zeros(0, int)
    sizes = np.array([o[m + 1] - o[m] for m in mols], dtype=np.int64)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    return np.asarray(batch.species)[rows], np.asarray(batch.coords)[rows], off, rows
