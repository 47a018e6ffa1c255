"""torch.autograd.Function over the C ABI: energies and forces with a
hand-written backward that returns parameter gradients.

    E, F = nnp_energy_forces(model, coords, params, species, mol_offsets)

E [B] (float64) and F [A, 3] (coordinate dtype) are differentiable with
respect to `params` (the packed FP64 master weights, any device) and to
`coords` for any loss of E and F (F = -dE/dx, Methods, Eq. 3: a loss of the
forces reaches the coordinates through the energy Hessian, whose products
with dL/dF the library forms exactly).  All arithmetic runs in the HIP
library; this module only moves tensors across the ABI.
"""
from __future__ import annotations

import torch

from .nnp import NNP


class NNPFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, coords, params, model: NNP, species, mol_offsets):
        model.sync_params(params)
        E, F = model.energy_forces(coords.detach().contiguous(), species, mol_offsets)
        ctx.model = model
        ctx.params_meta = (params.dtype, params.device)
        # params is saved so that torch's version check refuses a backward
        # after an in-place change of the weights this forward used
        ctx.save_for_backward(coords, params, species, mol_offsets)
        ctx.set_materialize_grads(False)
        return E, F

    @staticmethod
    def backward(ctx, gE, gF):
        coords, params, species, mol_offsets = ctx.saved_tensors
        model: NNP = ctx.model
        # another forward on the same model may have loaded other weights
        # since: the backward differentiates at this forward's weights
        model.sync_params(params)
        need_x, need_w = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        if gE is None and gF is None:
            return None, None, None, None, None
        gE_ = gE.detach().to(torch.float64).contiguous() if gE is not None else None
        gF_ = gF.detach().to(coords.dtype).contiguous() if gF is not None else None
        gp, gx = model.backward(coords.detach().contiguous(), species, mol_offsets, gE_, gF_,
                                want_coords=need_x)
        dtype, device = ctx.params_meta
        gw = gp.to(device=device, dtype=dtype) if need_w else None
        return (gx if need_x else None), gw, None, None, None


def nnp_energy_forces(model: NNP, coords, params, species, mol_offsets):
    return NNPFunction.apply(coords, params, model, species, mol_offsets)
