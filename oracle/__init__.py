"""FP64 CPU oracle (test infrastructure only).

Only the tests, the package smoke check and the benchmark's CPU-baseline leg
may import this.  It wraps `nnp_oracle.c` (plain C, built with gcc by
`build()`) through ctypes and shares no code with the HIP library.
`oracle.hessian` writes the energy once more in plain torch FP64 operations
for Hessian-vector products (coordinate gradients of force-dependent losses).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nnp_oracle.c")
_SRC_COUPLING = os.path.join(_HERE, "coupling_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, OpenMP over molecules/atoms)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, _SRC, _SRC_COUPLING, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _AEV(C.Structure):
    _fields_ = [("n_species", C.c_int32), ("n_shf_r", C.c_int32), ("n_shf_a", C.c_int32),
                ("n_shf_z", C.c_int32), ("rcr", C.c_double), ("rca", C.c_double),
                ("eta_r", C.c_double), ("eta_a", C.c_double), ("zeta", C.c_double),
                ("angle_scale", C.c_double), ("radial_pref", C.c_double),
                ("shf_r", C.POINTER(C.c_double)), ("shf_a", C.POINTER(C.c_double)),
                ("shf_z", C.POINTER(C.c_double))]


class _Net(C.Structure):
    _fields_ = [("n_models", C.c_int32), ("n_species", C.c_int32), ("n_layers", C.c_int32),
                ("widths", C.POINTER(C.c_int32)), ("celu_alpha", C.c_double),
                ("weights", C.POINTER(C.c_double)), ("species_widths", C.POINTER(C.c_int32))]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = C.CDLL(_LIB)
        P = C.POINTER
        d, i32 = C.c_double, C.c_int32
        lib.orc_aev_dim.restype = i32
        lib.orc_aev_dim.argtypes = [P(_AEV)]
        lib.orc_fc.restype = d
        lib.orc_fc.argtypes = [d, d]
        lib.orc_dfc.restype = d
        lib.orc_dfc.argtypes = [d, d]
        for name in ("orc_aev", "orc_aev_vjp", "orc_aev_jvp"):
            f = getattr(lib, name)
            f.restype = None
        lib.orc_aev.argtypes = [P(_AEV), i32, P(i32), P(d), P(d)]
        lib.orc_aev_vjp.argtypes = [P(_AEV), i32, P(i32), P(d), P(d), P(d)]
        lib.orc_aev_jvp.argtypes = [P(_AEV), i32, P(i32), P(d), P(d), P(d)]
        lib.orc_atomic_nn.restype = d
        lib.orc_atomic_nn.argtypes = [P(_Net), i32, i32, P(d), P(d)]
        lib.orc_energy_forces.restype = None
        lib.orc_energy_forces.argtypes = [P(_AEV), P(_Net), d, P(d), i32, P(i32), P(i32), P(d),
                                          P(d), P(d)]
        lib.orc_param_grad.restype = None
        lib.orc_param_grad.argtypes = [P(_AEV), P(_Net), d, i32, P(i32), P(i32), P(d), P(d),
                                       P(d), P(d)]
        lib.orc_num_threads.restype = i32
        lib.orc_coupling.restype = None
        lib.orc_coupling.argtypes = [i32, P(d), P(d), i32, P(d), P(d), d, d, P(d), P(d), P(d),
                                     P(d)]
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


class _Keep:
    """Holds the numpy buffers a ctypes struct points into."""

    def __init__(self, struct, *bufs):
        self.struct = struct
        self.bufs = bufs


def _aev_struct(hp: dict) -> _Keep:
    sr = np.ascontiguousarray(hp["shf_r"], dtype=np.float64)
    sa = np.ascontiguousarray(hp["shf_a"], dtype=np.float64)
    sz = np.ascontiguousarray(hp["shf_z"], dtype=np.float64)
    s = _AEV(hp["n_species"], len(sr), len(sa), len(sz), hp["rcr"], hp["rca"], hp["eta_r"],
             hp["eta_a"], hp["zeta"], hp["angle_scale"], hp["radial_pref"], _dp(sr), _dp(sa),
             _dp(sz))
    return _Keep(s, sr, sa, sz)


def species_widths(hp: dict) -> list:
    """Layer widths of every element's networks: hp["species_widths"] (one
    list per element) when given, else hp["widths"] for all."""
    sw = hp.get("species_widths")
    return [list(x) for x in sw] if sw is not None else [list(hp["widths"])] * hp["n_species"]


def _net_struct(hp: dict, weights: np.ndarray, n_models: int) -> _Keep:
    w = np.ascontiguousarray(weights, dtype=np.float64)
    wd = np.ascontiguousarray(hp["widths"], dtype=np.int32)
    per = species_widths(hp)
    if len(per) != hp["n_species"] or any(len(x) != len(wd) for x in per):
        raise ValueError("species_widths needs one list of len(widths) per element")
    swd = np.ascontiguousarray(per, dtype=np.int32).reshape(-1)
    s = _Net(n_models, hp["n_species"], len(wd) - 1, _ip(wd), hp["celu_alpha"], _dp(w),
             _ip(swd) if hp.get("species_widths") is not None else None)
    expect = n_models * sum(sum(x[l + 1] * x[l] + x[l + 1] for l in range(len(x) - 1)) for x in per)
    if w.size != expect:
        raise ValueError(f"weights have {w.size} values, expected {expect}")
    return _Keep(s, w, wd, swd)


def _mol(species, coords):
    sp = np.ascontiguousarray(species, dtype=np.int32)
    x = np.ascontiguousarray(coords, dtype=np.float64).reshape(-1, 3)
    if sp.shape[0] != x.shape[0]:
        raise ValueError("species and coords disagree in length")
    return sp, x


def aev_dim(hp: dict) -> int:
    k = _aev_struct(hp)
    return int(_load().orc_aev_dim(C.byref(k.struct)))


def fc(r: float, rc: float) -> float:
    return float(_load().orc_fc(r, rc))


def dfc(r: float, rc: float) -> float:
    return float(_load().orc_dfc(r, rc))


def aev(hp: dict, species, coords) -> np.ndarray:
    """AEV of one molecule, [n, D]."""
    sp, x = _mol(species, coords)
    k = _aev_struct(hp)
    out = np.zeros((sp.shape[0], aev_dim(hp)), dtype=np.float64)
    _load().orc_aev(C.byref(k.struct), sp.shape[0], _ip(sp), _dp(x), _dp(out))
    return out


def aev_vjp(hp: dict, species, coords, gG) -> np.ndarray:
    """sum_i gG_i . dG_i/dx, [n, 3]."""
    sp, x = _mol(species, coords)
    k = _aev_struct(hp)
    g = np.ascontiguousarray(gG, dtype=np.float64)
    out = np.zeros((sp.shape[0], 3), dtype=np.float64)
    _load().orc_aev_vjp(C.byref(k.struct), sp.shape[0], _ip(sp), _dp(x), _dp(g), _dp(out))
    return out


def aev_jvp(hp: dict, species, coords, v) -> np.ndarray:
    """(dG/dx) v, [n, D]."""
    sp, x = _mol(species, coords)
    k = _aev_struct(hp)
    vv = np.ascontiguousarray(v, dtype=np.float64).reshape(-1, 3)
    out = np.zeros((sp.shape[0], aev_dim(hp)), dtype=np.float64)
    _load().orc_aev_jvp(C.byref(k.struct), sp.shape[0], _ip(sp), _dp(x), _dp(vv), _dp(out))
    return out


def atomic_nn(hp: dict, weights, n_models: int, model: int, species: int, G):
    """(e, de/dG) of network (model, species) at AEV G."""
    nk = _net_struct(hp, weights, n_models)
    g = np.ascontiguousarray(G, dtype=np.float64)
    dG = np.zeros_like(g)
    e = _load().orc_atomic_nn(C.byref(nk.struct), model, species, _dp(g), _dp(dG))
    return float(e), dG


def energy_forces(hp: dict, weights, n_models: int, species, coords, mol_offsets=None,
                  sae=None, energy_scale=None):
    """Per-molecule energies [B] and forces [A, 3] (FP64)."""
    sp, x = _mol(species, coords)
    off = np.ascontiguousarray(
        mol_offsets if mol_offsets is not None else [0, sp.shape[0]], dtype=np.int32)
    ak = _aev_struct(hp)
    nk = _net_struct(hp, weights, n_models)
    scale = hp["energy_scale"] if energy_scale is None else energy_scale
    sae_a = None if sae is None else np.ascontiguousarray(sae, dtype=np.float64)
    E = np.zeros(off.shape[0] - 1, dtype=np.float64)
    F = np.zeros((sp.shape[0], 3), dtype=np.float64)
    _load().orc_energy_forces(C.byref(ak.struct), C.byref(nk.struct), scale,
                              None if sae_a is None else _dp(sae_a), off.shape[0] - 1, _ip(off),
                              _ip(sp), _dp(x), _dp(E), _dp(F))
    return E, F


def param_grad(hp: dict, weights, n_models: int, species, coords, mol_offsets, gE, gF,
               energy_scale=None) -> np.ndarray:
    """dL/dW for loss cotangents gE = dL/dE [B], gF = dL/dF [A, 3] (packed like weights)."""
    sp, x = _mol(species, coords)
    off = np.ascontiguousarray(mol_offsets, dtype=np.int32)
    ak = _aev_struct(hp)
    nk = _net_struct(hp, weights, n_models)
    scale = hp["energy_scale"] if energy_scale is None else energy_scale
    ge = np.ascontiguousarray(gE, dtype=np.float64)
    gf = np.ascontiguousarray(gF, dtype=np.float64).reshape(-1, 3)
    out = np.zeros(nk.bufs[0].size, dtype=np.float64)
    _load().orc_param_grad(C.byref(ak.struct), C.byref(nk.struct), scale, off.shape[0] - 1,
                           _ip(off), _ip(sp), _dp(x), _dp(ge), _dp(gf), _dp(out))
    return out


def num_threads() -> int:
    return int(_load().orc_num_threads())


def coupling(x_nnp, par_nnp, x_mm, par_mm, k, cutoff=0.0, with_abs=False):
    """NNP-MM mechanical-embedding coupling (Methods, Eq. 4): energy, forces
    on the NNP atoms and on the MM atoms.  par_* are [n][3] = (q, sigma,
    eps); Lorentz-Berthelot pair parameters; cutoff 0 = every pair."""
    lib = _load()
    xn = np.ascontiguousarray(x_nnp, dtype=np.float64).reshape(-1, 3)
    pn = np.ascontiguousarray(par_nnp, dtype=np.float64).reshape(-1, 3)
    xm = np.ascontiguousarray(x_mm, dtype=np.float64).reshape(-1, 3)
    pm = np.ascontiguousarray(par_mm, dtype=np.float64).reshape(-1, 3)
    E = np.zeros(1)
    A = np.zeros(1)
    Fn = np.zeros_like(xn)
    Fm = np.zeros_like(xm)
    lib.orc_coupling(len(xn), _dp(xn), _dp(pn), len(xm), _dp(xm), _dp(pm), float(k), float(cutoff),
                     _dp(E), _dp(Fn), _dp(Fm), _dp(A))
    if with_abs:
        return float(E[0]), Fn, Fm, float(A[0])
    return float(E[0]), Fn, Fm
