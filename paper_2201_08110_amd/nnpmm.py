"""The NNP-region force step of an NNP/MM simulation (Methods, Eq. 1): the
NNP energy and forces of the ligand (Eq. 2-3) plus the NNP-MM coupling term
(Eq. 4) added onto them and onto the caller's MM forces, all stream-ordered on
one stream and allocation-free per step, so that an MD engine can run its MM
work concurrently on another stream.

Argument marshalling only: the work runs in the library's kernels (one
captured graph for the NNP evaluation, two coupling launches)."""
from __future__ import annotations

from .nnp import NNP, Coupling


class NNPMMStep:
    """E [1] (float64), F_nnp [n, 3] and F_mm [m, 3] of one NNP/MM force step.

    F_mm is accumulated into (it normally holds the MM engine's forces);
    E and F_nnp are overwritten with V_NNP + V_coupling and its forces."""

    def __init__(self, model: NNP, coupling: Coupling, species, mol_offsets, par_nnp, par_mm):
        if int(mol_offsets.numel()) != 2:
            raise ValueError("the NNP region is one molecule")
        self.model, self.coupling = model, coupling
        self.species, self.mol_offsets = species, mol_offsets
        self.par_nnp, self.par_mm = par_nnp, par_mm

    def __call__(self, x_nnp, x_mm, E, F_nnp, F_mm, stream, graph: bool = True):
        self.model.energy_forces(x_nnp, self.species, self.mol_offsets, out=(E, F_nnp), graph=graph,
                                 stream=stream)
        self.coupling(x_nnp, self.par_nnp, x_mm, self.par_mm, out=(E[0:1], F_nnp, F_mm),
                      accumulate=True, stream=stream)
        return E, F_nnp, F_mm
