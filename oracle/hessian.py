"""FP64 Hessian-vector products of the NNP energy (test infrastructure only).

The coordinate gradient of a loss that depends on the forces needs the
Hessian of the energy: F = -dE/dx (Methods, Eq. 3), so for L(E, F)

    dL/dx = sum_b gE_b dE_b/dx + sum gF . dF/dx = -gE_b(i) F_i - H gF,

with H = d^2E/dx^2.  Here the energy is written out once more in plain torch
FP64 operations (all pairs and all unordered triples of a small molecule, the
same published ANI form as `nnp_oracle.c`; the per-element networks as
Linear / CELU) and differentiated twice by autograd.  It shares no code with
the C oracle or the HIP library; its energies and forces are pinned to the C
oracle and its Hessian-vector products to central differences of the C
oracle's forces.
"""
from __future__ import annotations

import math

import numpy as np


def _torch():
    import torch
    return torch


def _fc(torch, r, rc):
    return torch.where(r < rc, 0.5 * torch.cos(math.pi * r / rc) + 0.5, torch.zeros_like(r))


def _aev(torch, hp, species, x):
    """AEV rows [n, D] of one molecule as a differentiable function of x."""
    n = x.shape[0]
    S = hp["n_species"]
    shf_r = torch.tensor(hp["shf_r"], dtype=torch.float64)
    shf_a = torch.tensor(hp["shf_a"], dtype=torch.float64)
    shf_z = torch.tensor(hp["shf_z"], dtype=torch.float64)
    nR, nA, nZ = len(hp["shf_r"]), len(hp["shf_a"]), len(hp["shf_z"])
    sp = torch.as_tensor(species, dtype=torch.long)
    eye = torch.eye(n, dtype=torch.bool)
    d = x[None, :, :] - x[:, None, :]                                # d[i, j] = x_j - x_i
    r = torch.sqrt((d * d).sum(-1) + eye.to(torch.float64))          # diagonal set to 1 (masked)
    # radial: G_i[nR s_j + k] += pref exp(-etaR (r - ShfR_k)^2) fc(r; Rcr)
    fr = _fc(torch, r, hp["rcr"]) * (~eye)
    rad = hp["radial_pref"] * torch.exp(-hp["eta_r"] * (r[..., None] - shf_r) ** 2) * fr[..., None]
    onehot = torch.nn.functional.one_hot(sp, S).to(torch.float64)     # [n, S]
    G_rad = torch.einsum("ijk,js->isk", rad, onehot).reshape(n, S * nR)
    # angular: every unordered {j, k} of neighbours of i
    fa = _fc(torch, r, hp["rca"]) * (~eye)
    iu = torch.triu_indices(n, n, offset=1)
    j, k = iu[0], iu[1]
    dj, dk = d[:, j, :], d[:, k, :]                                  # [n, P, 3]
    rj, rk = r[:, j], r[:, k]
    cos = (dj * dk).sum(-1) / (rj * rk)
    cp = hp["angle_scale"] * cos
    sn = torch.sqrt(1.0 - cp * cp)
    # cos(theta' - t) with theta' = arccos(c'), written without arccos
    cz = cp[..., None] * torch.cos(shf_z) + sn[..., None] * torch.sin(shf_z)
    ang = 2.0 * ((1.0 + cz) / 2.0) ** hp["zeta"]                      # [n, P, nZ]
    rad_a = torch.exp(-hp["eta_a"] * ((rj + rk)[..., None] / 2.0 - shf_a) ** 2)   # [n, P, nA]
    w = fa[:, j] * fa[:, k]                                           # zero when j or k is i
    term = (rad_a[..., :, None] * ang[..., None, :]) * w[..., None, None]          # [n, P, nA, nZ]
    # species-pair block p(b, c), b <= c, row-major upper triangle
    sj, sk = sp[j], sp[k]
    b, c = torch.minimum(sj, sk), torch.maximum(sj, sk)
    pidx = b * S - (b * (b - 1)) // 2 + (c - b)
    NB = S * (S + 1) // 2
    onep = torch.nn.functional.one_hot(pidx, NB).to(torch.float64)   # [P, NB]
    G_ang = torch.einsum("ipaz,pb->ibaz", term, onep).reshape(n, NB * nA * nZ)
    return torch.cat([G_rad, G_ang], dim=1)


def _networks(torch, hp, weights, n_models):
    """Per (model, element) list of (W, b) layers from the packed FP64 weights."""
    S = hp["n_species"]
    per = hp.get("species_widths") or [hp["widths"]] * S
    w = torch.as_tensor(np.asarray(weights, dtype=np.float64))
    nets, off = {}, 0
    for m in range(n_models):
        for s in range(S):
            wd = per[s]
            layers = []
            for l in range(len(wd) - 1):
                W = w[off:off + wd[l + 1] * wd[l]].view(wd[l + 1], wd[l])
                off += wd[l + 1] * wd[l]
                bb = w[off:off + wd[l + 1]]
                off += wd[l + 1]
                layers.append((W, bb))
            nets[(m, s)] = layers
    return nets


def _energy(torch, hp, nets, n_models, species, x):
    G = _aev(torch, hp, species, x)
    al = hp["celu_alpha"]
    e = torch.zeros((), dtype=torch.float64)
    for i, s in enumerate(np.asarray(species).tolist()):
        for m in range(n_models):
            a = G[i]
            layers = nets[(m, s)]
            for l, (W, bb) in enumerate(layers):
                a = W @ a + bb
                if l + 1 < len(layers):
                    a = torch.where(a >= 0, a, al * torch.expm1(torch.clamp(a, max=0.0) / al))
            e = e + a[0]
    return hp["energy_scale"] * e / n_models


def energy_forces_hvp(hp, weights, n_models, species, coords, v):
    """E, F = -dE/dx and H v for one molecule (all FP64)."""
    torch = _torch()
    nets = _networks(torch, hp, weights, n_models)
    x = torch.tensor(np.asarray(coords, dtype=np.float64), requires_grad=True)
    E = _energy(torch, hp, nets, n_models, species, x)
    (g,) = torch.autograd.grad(E, x, create_graph=True)
    vv = torch.as_tensor(np.asarray(v, dtype=np.float64).reshape(-1, 3))
    (hv,) = torch.autograd.grad((g * vv).sum(), x)
    return float(E.detach()), -g.detach().numpy(), hv.numpy()


def coord_grad(hp, weights, n_models, species, coords, mol_offsets, gE, gF):
    """dL/dx = -gE_b(i) F_i - H gF per molecule of a batch (FP64)."""
    coords = np.asarray(coords, dtype=np.float64).reshape(-1, 3)
    gF = np.asarray(gF, dtype=np.float64).reshape(-1, 3)
    out = np.zeros_like(coords)
    for b in range(len(mol_offsets) - 1):
        a0, a1 = int(mol_offsets[b]), int(mol_offsets[b + 1])
        if a1 == a0:
            continue
        _, F, hv = energy_forces_hvp(hp, weights, n_models, np.asarray(species)[a0:a1], coords[a0:a1],
                                     gF[a0:a1])
        out[a0:a1] = -gE[b] * F - hv
    return out
