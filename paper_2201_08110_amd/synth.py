"""Seeded synthetic inputs: model hyper-parameters, molecules, weights, targets.

This module is the only thing the GPU library's tests and the oracle share.
It holds no arithmetic of the method itself (no symmetry function, network or
derivative): only the numbers a user would hand to the library — the
ANI-2x-shaped hyper-parameters, random molecules of the sizes the paper
simulates, Xavier-initialised weights — drawn from fixed seeds.

Workloads (the paper's ligands are 48-75 atoms over H,C,N,O,F,S,Cl, Results,
Table 1; its timings are single-ligand energy+force calls, Table 2):

  cfg 1  one 24-atom molecule, H12 C8 N2 O2, 6 A cube, one model, FP64
  cfg 2  one 64-atom ligand, 30:20:5:5:2:1:1 over H..Cl, 9 A cube, 8 models, FP32
  cfg 3  512 molecules of U{10..120} atoms, ratio-sampled elements,
         cube edge N^(1/3) * 2.2 A, 8 models, FP32
  cfg 4  64 molecules of U{30..80} atoms with seeded target energies/forces
  cfg 5  1024 Gaussian (sigma 0.05 A) replicas of one 48-atom ligand
         (22:15:4:4:1:1:1), 8 models, BF16 MLP

Geometry: sequential rejection sampling, a uniform candidate in the cube is
accepted when it is at least 1.0 A from every accepted atom; element labels are
exact counts (shuffled) where given, else drawn from the ratio.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

#: base seed of every workload; cfg k draws from SeedSequence(BASE_SEED + k)
BASE_SEED = 220108110
#: seed of the model weights, shared by every workload (model 0 of the
#: ensemble is the single model of cfg 1)
W_SEED = 220108110

#: atomic numbers of the element table, index order = species index
ELEMENTS = (1, 6, 7, 8, 9, 16, 17)
ELEMENT_NAMES = ("H", "C", "N", "O", "F", "S", "Cl")
#: element ratio of a drug-like ligand over H,C,N,O,F,S,Cl
LIGAND_RATIO = (30, 20, 5, 5, 2, 1, 1)

#: Hartree -> kcal/mol
HARTREE_TO_KCALMOL = 627.5094740631


def ani2x_hparams() -> dict:
    """ANI-2x-shaped featuriser and network hyper-parameters.

    Shift grids are half-open: 16 radial shifts from 0.8 A in steps of
    (5.1-0.8)/16, 8 angular-distance shifts from 0.8 A in steps of (3.5-0.8)/8,
    4 angle shifts at the bin midpoints (2z+1) pi / 8 of (0, pi).
    """
    return dict(
        n_species=7,
        rcr=5.1, rca=3.5,
        eta_r=19.7, eta_a=12.5, zeta=14.1,
        shf_r=[0.8 + k * (5.1 - 0.8) / 16.0 for k in range(16)],
        shf_a=[0.8 + a * (3.5 - 0.8) / 8.0 for a in range(8)],
        shf_z=[(2 * z + 1) * math.pi / 8.0 for z in range(4)],
        angle_scale=0.95,
        radial_pref=0.25,
        widths=[1008, 256, 192, 160, 1],
        celu_alpha=0.1,
        energy_scale=HARTREE_TO_KCALMOL,
    )


def ani2x_element_widths(hp: dict) -> list:
    """Per-element layer widths of the ANI-2x element networks (H, C, N, O,
    F, S, Cl): larger networks for the more frequent elements."""
    D = aev_dim(hp)
    hidden = {0: (256, 192, 160), 1: (224, 192, 160), 2: (192, 160, 128), 3: (192, 160, 128),
              4: (160, 128, 96), 5: (160, 128, 96), 6: (160, 128, 96)}
    return [[D, *hidden[s], 1] for s in range(hp["n_species"])]


def ani2x_heterogeneous_hparams() -> dict:
    """ANI-2x featuriser with element networks of their own widths; `widths`
    keeps the largest width of every layer."""
    hp = ani2x_hparams()
    hp["species_widths"] = ani2x_element_widths(hp)
    hp["widths"] = [max(w[l] for w in hp["species_widths"]) for l in range(5)]
    return hp


def ani1x_hparams() -> dict:
    """ANI-1x-shaped featuriser over H, C, N, O (384-dim AEV): 16 radial
    shifts on 0.9..5.2 A, 4 angular-distance shifts on 0.9..3.5 A, 8 angle
    shifts, eta_r 16, eta_a 8, zeta 32, and element networks
    384-160-128-96-1 (H), 384-144-112-96-1 (C), 384-128-112-96-1 (N, O)."""
    hp = dict(
        n_species=4,
        rcr=5.2, rca=3.5,
        eta_r=16.0, eta_a=8.0, zeta=32.0,
        shf_r=[0.9 + k * (5.2 - 0.9) / 16.0 for k in range(16)],
        shf_a=[0.9 + a * (3.5 - 0.9) / 4.0 for a in range(4)],
        shf_z=[(2 * z + 1) * math.pi / 16.0 for z in range(8)],
        angle_scale=0.95,
        radial_pref=0.25,
        celu_alpha=0.1,
        energy_scale=HARTREE_TO_KCALMOL,
    )
    D = aev_dim(hp)
    hp["species_widths"] = [[D, 160, 128, 96, 1], [D, 144, 112, 96, 1], [D, 128, 112, 96, 1],
                            [D, 128, 112, 96, 1]]
    hp["widths"] = [max(w[l] for w in hp["species_widths"]) for l in range(5)]
    return hp


def aev_dim(hp: dict) -> int:
    s = hp["n_species"]
    return s * len(hp["shf_r"]) + (s * (s + 1) // 2) * len(hp["shf_a"]) * len(hp["shf_z"])


def net_size(widths) -> int:
    return sum(widths[l + 1] * widths[l] + widths[l + 1] for l in range(len(widths) - 1))


# --------------------------------------------------------------------------
# geometry


def random_molecule(rng: np.random.Generator, counts, box: float, min_dist: float = 1.0):
    """Rejection-sampled coordinates (Angstrom) and shuffled species indices."""
    counts = list(counts)
    n = int(sum(counts))
    species = np.repeat(np.arange(len(counts), dtype=np.int32), counts)
    rng.shuffle(species)
    pos = np.empty((n, 3), dtype=np.float64)
    k = 0
    tries = 0
    while k < n:
        c = rng.uniform(0.0, box, size=3)
        tries += 1
        if tries > 200000 * max(n, 1):
            raise RuntimeError("rejection sampling did not converge")
        if k == 0 or np.min(np.sum((pos[:k] - c) ** 2, axis=1)) >= min_dist * min_dist:
            pos[k] = c
            k += 1
    return pos, species


def ratio_counts(rng: np.random.Generator, n: int, ratio=LIGAND_RATIO):
    p = np.asarray(ratio, dtype=np.float64)
    p /= p.sum()
    lab = rng.choice(len(ratio), size=n, p=p)
    return np.bincount(lab, minlength=len(ratio))


def rounded_counts(n: int, ratio):
    """Largest-remainder rounding of n * ratio to integers summing to n."""
    r = np.asarray(ratio, dtype=np.float64)
    q = n * r / r.sum()
    base = np.floor(q).astype(int)
    rem = n - base.sum()
    order = np.argsort(-(q - base), kind="stable")
    base[order[:rem]] += 1
    return base


# --------------------------------------------------------------------------
# weights


def xavier_weights(n_models: int, widths, n_species: int = 7, seed: int = W_SEED):
    """FP64 master weights, packed [model][species][layer]{W (out x in), b (out)}.

    W ~ U(+-sqrt(6/(fan_in+fan_out))), b ~ U(+-1/sqrt(fan_in)); model m draws
    from SeedSequence(seed).spawn(m+1)[m] so that model m is the same for any
    ensemble size.  `widths` is one list of layer widths for every element, or
    one list per element (networks of different sizes per element).
    """
    per = [list(w) for w in widths] if isinstance(widths[0], (list, tuple)) else [list(widths)] * n_species
    if len(per) != n_species:
        raise ValueError("one list of widths per element")
    children = np.random.SeedSequence(seed).spawn(max(n_models, 8))
    chunks = []
    for m in range(n_models):
        rng = np.random.Generator(np.random.PCG64(children[m]))
        for s in range(n_species):
            wd = per[s]
            for l in range(len(wd) - 1):
                fin, fout = wd[l], wd[l + 1]
                bw = math.sqrt(6.0 / (fin + fout))
                chunks.append(rng.uniform(-bw, bw, size=fout * fin))
                bb = 1.0 / math.sqrt(fin)
                chunks.append(rng.uniform(-bb, bb, size=fout))
    return np.concatenate(chunks).astype(np.float64)


# --------------------------------------------------------------------------
# batches


@dataclass
class Batch:
    name: str
    coords: np.ndarray          # [A, 3] float64
    species: np.ndarray         # [A] int32 species indices
    mol_offsets: np.ndarray     # [B+1] int32
    n_models: int
    precision: str              # "fp64" | "fp32" | "bf16"
    target_E: np.ndarray | None = None
    target_F: np.ndarray | None = None
    extra: dict = field(default_factory=dict)

    @property
    def n_atoms(self) -> int:
        return int(self.mol_offsets[-1])

    @property
    def n_mols(self) -> int:
        return len(self.mol_offsets) - 1


def _streams(cfg: int):
    ss = np.random.SeedSequence(BASE_SEED + cfg).spawn(4)
    return [np.random.Generator(np.random.PCG64(s)) for s in ss]   # geom, species, spare, targets


def _pack(mols):
    coords = np.concatenate([m[0] for m in mols]) if mols else np.zeros((0, 3))
    species = np.concatenate([m[1] for m in mols]).astype(np.int32) if mols else np.zeros(0, np.int32)
    off = np.zeros(len(mols) + 1, dtype=np.int32)
    off[1:] = np.cumsum([len(m[1]) for m in mols])
    return coords, species, off


def config_batch(cfg: int, n_mols: int | None = None) -> Batch:
    """The seeded batch of workload cfg (1..5); n_mols truncates cfg 3/4/5."""
    g_geom, g_spec, _g_spare, g_tgt = _streams(cfg)
    if cfg == 1:
        pos, sp = random_molecule(g_geom, [12, 8, 2, 2], 6.0)
        c, s, o = _pack([(pos, sp)])
        return Batch("single 24-atom molecule", c, s, o, 1, "fp64")
    if cfg == 2:
        pos, sp = random_molecule(g_geom, [30, 20, 5, 5, 2, 1, 1], 9.0)
        c, s, o = _pack([(pos, sp)])
        return Batch("single 64-atom ligand", c, s, o, 8, "fp32")
    if cfg in (3, 4):
        nb = 512 if cfg == 3 else 64
        lo, hi = (10, 120) if cfg == 3 else (30, 80)
        nb = nb if n_mols is None else n_mols
        mols = []
        for _ in range(nb):
            n = int(g_spec.integers(lo, hi + 1))
            counts = ratio_counts(g_spec, n)
            mols.append(random_molecule(g_geom, counts, n ** (1.0 / 3.0) * 2.2))
        c, s, o = _pack(mols)
        if cfg == 3:
            return Batch(f"{nb} molecules of {lo}-{hi} atoms", c, s, o, 8, "fp32")
        return Batch(f"{nb} molecules of {lo}-{hi} atoms, seeded targets", c, s, o, 8, "fp32",
                     extra={"target_seed": int(g_tgt.integers(1 << 30))})
    if cfg == 5:
        nrep = 1024 if n_mols is None else n_mols
        counts = rounded_counts(48, LIGAND_RATIO)
        base, sp = random_molecule(g_geom, counts, 48 ** (1.0 / 3.0) * 2.2)
        mols = [(base + g_geom.normal(0.0, 0.05, size=base.shape), sp) for _ in range(nrep)]
        c, s, o = _pack(mols)
        return Batch(f"{nrep} replicas of a 48-atom ligand", c, s, o, 8, "bf16")
    raise ValueError(f"unknown workload {cfg}")


def replica_batch(n_mols: int, n_atoms: int = 48, ratio=LIGAND_RATIO, seed: int = BASE_SEED + 50,
                  sigma: float = 0.05) -> Batch:
    """n_mols jittered replicas (Gaussian sigma in A) of one seeded molecule of
    n_atoms atoms with the given element ratio (workload 5 for other models)."""
    g = np.random.Generator(np.random.PCG64(seed))
    counts = rounded_counts(n_atoms, ratio)
    base, sp = random_molecule(g, counts, n_atoms ** (1.0 / 3.0) * 2.2)
    mols = [(base + g.normal(0.0, sigma, size=base.shape), sp) for _ in range(n_mols)]
    c, s, o = _pack(mols)
    return Batch(f"{n_mols} replicas of a {n_atoms}-atom molecule", c, s, o, 8, "bf16")


def random_batch(seed: int, sizes, box_scale: float = 2.2, ratio=LIGAND_RATIO) -> Batch:
    """Free-form seeded batch (tests): molecules of the given atom counts."""
    g = np.random.Generator(np.random.PCG64(seed))
    mols = []
    for n in sizes:
        counts = ratio_counts(g, int(n), ratio)
        mols.append(random_molecule(g, counts, max(int(n), 1) ** (1.0 / 3.0) * box_scale))
    c, s, o = _pack(mols)
    return Batch(f"random batch seed {seed}", c, s, o, 8, "fp32")


def round_to_fp32(a: np.ndarray) -> np.ndarray:
    """FP32-rounded values widened back to FP64 (what an FP32 path really sees)."""
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


# --------------------------------------------------------------------------
# NNP-MM coupling workload (mechanical embedding, Methods, Eq. 4).
#
# e^2 / (4 pi eps0) from the SI defining constants, in kcal/mol * A / e^2
# (the unit system of the energies here): e = 1.602176634e-19 C,
# eps0 = 8.8541878128e-12 F/m, N_A = 6.02214076e23 /mol, 1 kcal = 4184 J.
COULOMB_K = (1.602176634e-19 ** 2 / (4.0 * math.pi * 8.8541878128e-12)
             * 6.02214076e23 / 4184.0 * 1e10)

# atoms of the protein-ligand systems the paper simulates (Results, Table 1:
# 1HPO has a 64-atom ligand in 47,712 atoms in all)
COUPLING_TOTAL_ATOMS = 47712


@dataclass
class CouplingSystem:
    x_nnp: np.ndarray     # [n_nnp, 3] A
    par_nnp: np.ndarray   # [n_nnp, 3] (charge e, sigma A, epsilon kcal/mol)
    x_mm: np.ndarray      # [n_mm, 3]
    par_mm: np.ndarray    # [n_mm, 3]


def _neutral_charges(rng, n, scale):
    q = rng.normal(0.0, scale, size=n)
    return q - q.mean()


def coupling_system(seed: int = BASE_SEED + 100, n_mm: int | None = None,
                    density: float = 0.1, min_dist: float = 2.2) -> CouplingSystem:
    """A ligand (the 64-atom ligand of workload 2) at the centre of a cube of
    MM atoms at liquid density (0.1 atoms per A^3), MM atoms kept at least
    `min_dist` from every ligand atom.  Charges are seeded normals made
    neutral per region; Lennard-Jones sigma in U(2.4, 3.6) A and epsilon in
    U(0.02, 0.2) kcal/mol.  Synthetic stand-ins for the force-field
    parameters the paper's systems carry."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    lig = config_batch(2)
    x_nnp = lig.coords - lig.coords.mean(axis=0)
    n_nnp = len(x_nnp)
    if n_mm is None:
        n_mm = COUPLING_TOTAL_ATOMS - n_nnp
    # the cube holds the ligand with room to spare even for a few MM atoms
    extent = float(np.abs(x_nnp).max())
    edge = max((n_mm / density) ** (1.0 / 3.0), 2.0 * (extent + min_dist) + 8.0)
    keep = []
    total = 0
    for _ in range(1000):
        if total >= n_mm:
            break
        cand = rng.uniform(-edge / 2, edge / 2, size=(max(2 * (n_mm - total), 64), 3))
        d2 = ((cand[:, None, :] - x_nnp[None, :, :]) ** 2).sum(-1).min(axis=1)
        cand = cand[d2 >= min_dist ** 2]
        keep.append(cand[: n_mm - total])
        total += len(keep[-1])
    if total < n_mm:
        raise RuntimeError("could not place the MM atoms")
    x_mm = np.concatenate(keep)[:n_mm] if keep else np.zeros((0, 3))
    par_nnp = np.stack([_neutral_charges(rng, n_nnp, 0.25), rng.uniform(2.4, 3.6, n_nnp),
                        rng.uniform(0.02, 0.2, n_nnp)], axis=1)
    par_mm = np.stack([_neutral_charges(rng, n_mm, 0.35), rng.uniform(2.4, 3.6, n_mm),
                       rng.uniform(0.02, 0.2, n_mm)], axis=1)
    return CouplingSystem(x_nnp, par_nnp, x_mm, par_mm)
