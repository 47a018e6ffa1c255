"""The C ABI library loads, exports every declared symbol and rejects bad
arguments on the host before touching a GPU (runs without one)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2201_08110_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2201_08110_amd import nnp
    if not os.path.exists(nnp.LIB_PATH):
        pytest.skip("libnnp_hip.so not built")
    return nnp, nnp.load_library()


def test_exports_match_header():
    nnp, lib = _lib()
    hdr = open(os.path.join(ROOT, "include", "nnp.h")).read()
    declared = set(re.findall(r"\b(nnp_[a-z0-9_]+)\s*\(", hdr))
    assert declared == set(nnp.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name


def _params(nnp, hp, w, **over):
    keep = []

    def darr(v):
        a = np.ascontiguousarray(v, dtype=np.float64)
        keep.append(a)
        return a.ctypes.data_as(C.POINTER(C.c_double))

    wd = np.ascontiguousarray(hp["widths"], dtype=np.int32)
    keep.append(wd)
    p = nnp.ModelParams(n_species=7, n_shf_r=16, n_shf_a=8, n_shf_z=4, rcr=5.1, rca=3.5,
                        eta_r=19.7, eta_a=12.5, zeta=14.1, angle_scale=0.95, radial_pref=0.25,
                        shf_r=darr(hp["shf_r"]), shf_a=darr(hp["shf_a"]), shf_z=darr(hp["shf_z"]),
                        n_models=1, n_layers=4, widths=wd.ctypes.data_as(C.POINTER(C.c_int32)),
                        celu_alpha=0.1, weights=darr(w), sae=None, energy_scale=627.5,
                        precision=1, max_atoms=64, max_mols=4, max_atoms_per_mol=64, device=0)
    for k, v in over.items():
        setattr(p, k, v)
    return p, keep


@pytest.mark.parametrize("over,code", [
    ({"n_species": 0}, 1), ({"n_species": 9}, 1), ({"n_shf_r": 8}, 6), ({"rca": 6.0}, 1),
    ({"angle_scale": 1.0}, 1), ({"zeta": 0.5}, 1), ({"celu_alpha": 0.0}, 1),
    ({"n_models": 0}, 1), ({"n_layers": 3}, 6), ({"precision": 7}, 1), ({"max_atoms": 0}, 1),
    ({"max_atoms_per_mol": 5000}, 6),
])
def test_create_rejects_bad_params(hp, over, code):
    nnp, lib = _lib()
    w = np.zeros(synth.net_size(hp["widths"]) * 7)
    p, keep = _params(nnp, hp, w, **over)
    h = C.c_void_p(123)
    rc = lib.nnp_create(C.byref(p), C.byref(h))
    assert rc == code
    assert h.value is None
    assert len(lib.nnp_last_error()) > 0


@pytest.mark.parametrize("change,code", [((0, 0, 1000), 1), ((2, 4, 2), 1), ((3, 1, 0), 6),
                                         ((6, 2, 5000), 6)])
def test_create_rejects_bad_element_widths(hp, change, code):
    """species_widths: first width must be D, last 1, hidden 1..4096."""
    nnp, lib = _lib()
    sw = np.array([[1008, 256, 192, 160, 1]] * 7, dtype=np.int32)
    s, l, v = change
    sw[s, l] = v
    w = np.zeros(synth.net_size(hp["widths"]) * 7)
    p, keep = _params(nnp, hp, w, species_widths=sw.ctypes.data_as(C.POINTER(C.c_int32)))
    keep.append(sw)
    h = C.c_void_p(123)
    assert lib.nnp_create(C.byref(p), C.byref(h)) == code
    assert h.value is None


@pytest.mark.parametrize("table,code", [([1, 6, 7, 8, 9, 16, 6], 2), ([1, 6, 7, 8, 9, 16, 0], 2),
                                        ([1, 6, 7, 8, 9, 16, 128], 2), ([-1, 6, 7, 8, 9, 16, 17], 2)])
def test_create_rejects_bad_element_table(hp, table, code):
    """An element table with a repeated or impossible atomic number is
    refused at creation with NNP_E_SPECIES, before any device work."""
    nnp, lib = _lib()
    z = np.array(table, dtype=np.int32)
    w = np.zeros(synth.net_size(hp["widths"]) * 7)
    p, keep = _params(nnp, hp, w, atomic_numbers=z.ctypes.data_as(C.POINTER(C.c_int32)))
    keep.append(z)
    h = C.c_void_p(123)
    assert lib.nnp_create(C.byref(p), C.byref(h)) == code
    assert h.value is None
    assert b"atomic number" in lib.nnp_last_error()


@pytest.mark.parametrize("flags,prec,code", [(2, 1, 1), (1, 2, 6)])
def test_create_rejects_bad_creation_flags(hp, flags, prec, code):
    """Unknown creation flags; a training workspace on a BF16 handle."""
    nnp, lib = _lib()
    w = np.zeros(synth.net_size(hp["widths"]) * 7)
    p, keep = _params(nnp, hp, w, create_flags=flags, precision=prec)
    h = C.c_void_p(123)
    assert lib.nnp_create(C.byref(p), C.byref(h)) == code
    assert h.value is None


def test_noalloc_coupling_rejects_on_host():
    """The allocation-free coupling call validates everything on the host
    before it looks up its scratch (no GPU needed to get these errors)."""
    nnp, lib = _lib()
    E = (C.c_double * 1)()
    x = (C.c_double * 3)()
    call = lib.nnp_coupling_eval_noalloc
    assert call(7, 332.0, 0.0, 1, x, x, 1, x, x, E, x, x, None, 0) == nnp.NNP_E_INVALID      # precision
    assert call(0, float("inf"), 0.0, 1, x, x, 1, x, x, E, x, x, None, 0) == nnp.NNP_E_INVALID
    assert call(0, 332.0, -1.0, 1, x, x, 1, x, x, E, x, x, None, 0) == nnp.NNP_E_INVALID
    assert call(0, 332.0, 0.0, 1, x, x, 1, x, x, None, x, x, None, 0) == nnp.NNP_E_INVALID    # out_E
    assert call(0, 332.0, 0.0, 1, None, x, 1, x, x, E, x, x, None, 0) == nnp.NNP_E_INVALID
    assert call(0, 332.0, 0.0, -1, x, x, 1, x, x, E, x, x, None, 0) == nnp.NNP_E_INVALID
    assert call(0, 332.0, 0.0, 1, x, x, 1, x, x, E, x, x, None, 4) == nnp.NNP_E_INVALID       # flag
    assert call(0, 332.0, 0.0, 1025, x, x, 1, x, x, E, x, x, None, 0) == nnp.NNP_E_CAPACITY
    assert call(0, 332.0, 0.0, 1, x, x, (1 << 22) + 1, x, x, E, x, x, None, 0) == nnp.NNP_E_CAPACITY


def test_null_arguments():
    nnp, lib = _lib()
    h = C.c_void_p()
    assert lib.nnp_create(None, C.byref(h)) == nnp.NNP_E_INVALID
    assert lib.nnp_energy_forces(None, None, None, None, None) == nnp.NNP_E_INVALID
    assert lib.nnp_energy_forces_f64(None, None, None, None, None) == nnp.NNP_E_INVALID
    assert lib.nnp_aev(None, None, None, None) == nnp.NNP_E_INVALID
    assert lib.nnp_set_weights(None, None) == nnp.NNP_E_INVALID
    assert lib.nnp_set_params(None, None, 0, None) == nnp.NNP_E_INVALID
    assert lib.nnp_num_params(None) == -1
    assert lib.nnp_aev_dim(None) == -1
    v = C.c_int32(0)
    assert lib.nnp_set_knob(None, 0, 0) == nnp.NNP_E_INVALID
    assert lib.nnp_get_knob(None, 0, C.byref(v)) == nnp.NNP_E_INVALID
    assert lib.nnp_autotune(None, None, None, 1, None, None, 0) == nnp.NNP_E_INVALID
    h2 = C.c_void_p(7)
    assert lib.nnp_coupling_create(1, 64, 100, 332.0, 0.0, 0, None) == nnp.NNP_E_INVALID
    for prec, n_nnp, n_mm, k, rc in ((7, 64, 100, 332.0, 0.0), (2, 64, 100, 332.0, 0.0),
                                     (1, 0, 100, 332.0, 0.0), (1, 2000, 100, 332.0, 0.0),
                                     (1, 64, 0, 332.0, 0.0), (1, 64, 100, float("nan"), 0.0),
                                     (1, 64, 100, 332.0, -1.0)):
        assert lib.nnp_coupling_create(prec, n_nnp, n_mm, k, rc, 0, C.byref(h2)) == nnp.NNP_E_INVALID
        assert h2.value is None
    assert lib.nnp_coupling_eval(None, 0, None, None, 0, None, None, None, None, None, None, 0) == \
        nnp.NNP_E_INVALID
    lib.nnp_coupling_destroy(None)
    lib.nnp_destroy(None)


def test_knob_ids_match_header():
    nnp, _ = _lib()
    hdr = open(os.path.join(ROOT, "include", "nnp.h")).read()
    ids = dict((k, int(v)) for k, v in re.findall(r"\bNNP_KNOB_([A-Z0-9_]+)\s*=\s*(\d+)", hdr))
    assert ids == {"MLP_PATH": nnp.KNOB_MLP_PATH, "GEMM_STAGES": nnp.KNOB_GEMM_STAGES,
                   "CELL_MIN": nnp.KNOB_CELL_MIN, "TAIL_TILE": nnp.KNOB_TAIL_TILE,
                   "GEMM_WAVES": nnp.KNOB_GEMM_WAVES, "ATOM_CHUNK": nnp.KNOB_ATOM_CHUNK,
                   "L1_PATH": nnp.KNOB_L1_PATH, "FORCE_SUM": nnp.KNOB_FORCE_SUM,
                   "FORCE_PATH": nnp.KNOB_FORCE_PATH, "PIPELINE": nnp.KNOB_PIPELINE}
    assert set(nnp.KNOBS.values()) == set(ids.values())


def test_product_path_has_no_oracle_dependency():
    """The package never imports, links or reads the oracle."""
    pkg = os.path.join(ROOT, "paper_2201_08110_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in src.lower() or f == "synth.py", f
