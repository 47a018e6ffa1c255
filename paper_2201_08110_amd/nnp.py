"""ctypes binding of libnnp_hip.so (the C ABI of include/nnp.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Tensors are torch CUDA (HIP) tensors; the library runs on torch's
current stream.  If the library has not been built this module raises on
first use -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnnp_hip.so")

PREC = {"fp64": 0, "fp32": 1, "bf16": 2}
FLAG_GRAPH = 1
FLAG_ACCUMULATE = 2
FLAG_DEVICE_COUNTS = 4
CREATE_TRAINING = 1
#: atomic numbers of the ANI-2x elements in index order H, C, N, O, F, S, Cl
ANI2X_Z = (1, 6, 7, 8, 9, 16, 17)

NNP_OK, NNP_E_INVALID, NNP_E_SPECIES, NNP_E_CAPACITY, NNP_E_NOMEM, NNP_E_DEVICE, \
    NNP_E_UNSUPPORTED = range(7)


class NNPError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"nnp error {code}: {msg}")
        self.code = code


class ModelParams(C.Structure):
    _fields_ = [
        ("n_species", C.c_int32), ("n_shf_r", C.c_int32), ("n_shf_a", C.c_int32),
        ("n_shf_z", C.c_int32),
        ("rcr", C.c_double), ("rca", C.c_double), ("eta_r", C.c_double), ("eta_a", C.c_double),
        ("zeta", C.c_double), ("angle_scale", C.c_double), ("radial_pref", C.c_double),
        ("shf_r", C.POINTER(C.c_double)), ("shf_a", C.POINTER(C.c_double)),
        ("shf_z", C.POINTER(C.c_double)),
        ("n_models", C.c_int32), ("n_layers", C.c_int32), ("widths", C.POINTER(C.c_int32)),
        ("species_widths", C.POINTER(C.c_int32)),
        ("celu_alpha", C.c_double), ("weights", C.POINTER(C.c_double)),
        ("sae", C.POINTER(C.c_double)), ("energy_scale", C.c_double),
        ("precision", C.c_int32), ("max_atoms", C.c_int32), ("max_mols", C.c_int32),
        ("max_atoms_per_mol", C.c_int32), ("device", C.c_int32),
        ("atomic_numbers", C.POINTER(C.c_int32)), ("create_flags", C.c_uint32),
    ]


class Batch(C.Structure):
    _fields_ = [("n_mols", C.c_int32), ("n_atoms", C.c_int32), ("mol_offsets", C.c_void_p),
                ("species", C.c_void_p), ("stream", C.c_void_p), ("flags", C.c_uint32),
                ("counts", C.c_void_p)]


_lib = None

#: every symbol include/nnp.h declares
EXPORTS = ("nnp_create", "nnp_destroy", "nnp_energy_forces", "nnp_energy_forces_f64", "nnp_aev",
           "nnp_energy_forces_backward", "nnp_set_weights", "nnp_set_params", "nnp_num_params",
           "nnp_graph_stats", "nnp_aev_dim",
           "nnp_get_device_status", "nnp_set_timing", "nnp_set_timing_only", "nnp_kernel_times",
           "nnp_last_error",
           "nnp_set_knob", "nnp_get_knob", "nnp_autotune",
           "nnp_coupling_create", "nnp_coupling_destroy", "nnp_coupling_eval",
           "nnp_coupling_eval_noalloc")

#: tunable knobs (include/nnp.h)
(KNOB_MLP_PATH, KNOB_GEMM_STAGES, KNOB_CELL_MIN, KNOB_TAIL_TILE, KNOB_GEMM_WAVES, KNOB_ATOM_CHUNK,
 KNOB_L1_PATH, KNOB_FORCE_SUM, KNOB_FORCE_PATH, KNOB_PIPELINE) = range(10)
KNOBS = {"mlp_path": KNOB_MLP_PATH, "gemm_stages": KNOB_GEMM_STAGES, "cell_min": KNOB_CELL_MIN,
         "tail_tile": KNOB_TAIL_TILE, "gemm_waves": KNOB_GEMM_WAVES, "atom_chunk": KNOB_ATOM_CHUNK,
         "l1_path": KNOB_L1_PATH, "force_sum": KNOB_FORCE_SUM, "force_path": KNOB_FORCE_PATH,
         "pipeline": KNOB_PIPELINE}


def load_library(path: str = LIB_PATH):
    """Load libnnp_hip.so and declare its signatures (no GPU work)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run paper_2201_08110_amd/build.py "
                          "(or __graft_entry__.build())")
    lib = C.CDLL(path)
    P, vp, i32, i64, d = C.POINTER, C.c_void_p, C.c_int32, C.c_int64, C.c_double
    lib.nnp_create.argtypes = [P(ModelParams), P(vp)]
    lib.nnp_create.restype = i32
    lib.nnp_destroy.argtypes = [vp]
    lib.nnp_destroy.restype = None
    for name in ("nnp_energy_forces", "nnp_energy_forces_f64"):
        f = getattr(lib, name)
        f.argtypes = [vp, P(Batch), vp, vp, vp]
        f.restype = i32
    lib.nnp_aev.argtypes = [vp, P(Batch), vp, vp]
    lib.nnp_aev.restype = i32
    lib.nnp_energy_forces_backward.argtypes = [vp, P(Batch), vp, vp, vp, vp, vp]
    lib.nnp_energy_forces_backward.restype = i32
    lib.nnp_set_weights.argtypes = [vp, P(d)]
    lib.nnp_set_weights.restype = i32
    lib.nnp_set_params.argtypes = [vp, vp, i32, vp]
    lib.nnp_set_params.restype = i32
    lib.nnp_num_params.argtypes = [vp]
    lib.nnp_num_params.restype = i64
    lib.nnp_graph_stats.argtypes = [vp, P(i64), P(i64), P(i32)]
    lib.nnp_graph_stats.restype = i32
    lib.nnp_aev_dim.argtypes = [vp]
    lib.nnp_aev_dim.restype = i32
    lib.nnp_get_device_status.argtypes = [vp, P(i32)]
    lib.nnp_get_device_status.restype = i32
    lib.nnp_set_timing.argtypes = [vp, i32]
    lib.nnp_set_timing.restype = i32
    lib.nnp_set_timing_only.argtypes = [vp, C.c_char_p]
    lib.nnp_set_timing_only.restype = i32
    lib.nnp_kernel_times.argtypes = [vp, i32, P(C.c_char_p), P(i64), P(d)]
    lib.nnp_kernel_times.restype = i32
    lib.nnp_last_error.argtypes = []
    lib.nnp_last_error.restype = C.c_char_p
    lib.nnp_set_knob.argtypes = [vp, i32, i32]
    lib.nnp_set_knob.restype = i32
    lib.nnp_get_knob.argtypes = [vp, i32, P(i32)]
    lib.nnp_get_knob.restype = i32
    lib.nnp_autotune.argtypes = [vp, P(Batch), vp, i32, C.c_char_p, C.c_char_p, i32]
    lib.nnp_autotune.restype = i32
    lib.nnp_coupling_create.argtypes = [i32, i32, i32, d, d, i32, P(vp)]
    lib.nnp_coupling_create.restype = i32
    lib.nnp_coupling_destroy.argtypes = [vp]
    lib.nnp_coupling_destroy.restype = None
    lib.nnp_coupling_eval.argtypes = [vp, i32, vp, vp, i32, vp, vp, vp, vp, vp, vp, C.c_uint32]
    lib.nnp_coupling_eval.restype = i32
    lib.nnp_coupling_eval_noalloc.argtypes = [i32, d, d, i32, vp, vp, i32, vp, vp, vp, vp, vp, vp,
                                              C.c_uint32]
    lib.nnp_coupling_eval_noalloc.restype = i32
    _lib = lib
    return lib


def _check(rc: int):
    if rc != NNP_OK:
        raise NNPError(rc, load_library().nnp_last_error().decode())


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class NNP:
    """One handle of the library: a model, a precision and a capacity."""

    def __init__(self, hp: dict, weights, n_models: int, precision: str = "fp32",
                 max_atoms: int = 1024, max_mols: int = 64, max_atoms_per_mol: int = 128,
                 device: int = 0, sae=None, atomic_numbers=None, training: bool = False):
        """atomic_numbers: the element table (e.g. ANI2X_Z); batches then
        pass atomic numbers as species.  training: allocate the training
        backward's workspace now rather than on the first backward."""
        lib = load_library()
        self._keep = []

        def darr(v):
            a = np.ascontiguousarray(v, dtype=np.float64)
            self._keep.append(a)
            return _dp(a)

        wd = np.ascontiguousarray(hp["widths"], dtype=np.int32)
        self._keep.append(wd)
        p = ModelParams()
        p.n_species = hp["n_species"]
        p.n_shf_r, p.n_shf_a, p.n_shf_z = len(hp["shf_r"]), len(hp["shf_a"]), len(hp["shf_z"])
        p.rcr, p.rca = hp["rcr"], hp["rca"]
        p.eta_r, p.eta_a, p.zeta = hp["eta_r"], hp["eta_a"], hp["zeta"]
        p.angle_scale, p.radial_pref = hp["angle_scale"], hp["radial_pref"]
        p.shf_r, p.shf_a, p.shf_z = darr(hp["shf_r"]), darr(hp["shf_a"]), darr(hp["shf_z"])
        p.n_models = n_models
        p.n_layers = len(wd) - 1
        p.widths = wd.ctypes.data_as(C.POINTER(C.c_int32))
        if hp.get("species_widths") is not None:
            sw = np.ascontiguousarray(hp["species_widths"], dtype=np.int32).reshape(-1)
            self._keep.append(sw)
            p.species_widths = sw.ctypes.data_as(C.POINTER(C.c_int32))
        p.celu_alpha = hp["celu_alpha"]
        p.weights = darr(weights)
        p.sae = darr(sae) if sae is not None else None
        p.energy_scale = hp["energy_scale"]
        p.precision = PREC[precision]
        p.max_atoms, p.max_mols, p.max_atoms_per_mol = max_atoms, max_mols, max_atoms_per_mol
        p.device = device
        if atomic_numbers is not None:
            z = np.ascontiguousarray(atomic_numbers, dtype=np.int32)
            self._keep.append(z)
            p.atomic_numbers = z.ctypes.data_as(C.POINTER(C.c_int32))
        p.create_flags = CREATE_TRAINING if training else 0
        h = C.c_void_p()
        _check(lib.nnp_create(C.byref(p), C.byref(h)))
        self._keep = []
        self.h = h
        self.precision = precision
        self.device = device
        self.lib = lib

    # -- helpers -----------------------------------------------------------
    def close(self):
        if getattr(self, "h", None):
            self.lib.nnp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def coord_dtype(self):
        import torch
        return torch.float64 if self.precision == "fp64" else torch.float32

    def _batch(self, species, mol_offsets, stream=None, flags=0):
        import torch
        b = Batch()
        b.n_mols = int(mol_offsets.numel()) - 1
        b.n_atoms = int(species.numel())
        b.mol_offsets = mol_offsets.data_ptr()
        b.species = species.data_ptr() if species.numel() else None
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        b.stream = s.cuda_stream
        b.flags = flags
        return b

    @staticmethod
    def _need(t, dtype, name):
        import torch
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
            raise TypeError(f"{name} must be a CUDA tensor")
        if t.dtype != dtype or not t.is_contiguous():
            raise TypeError(f"{name} must be contiguous {dtype}")

    # -- API ---------------------------------------------------------------
    def energy_forces(self, coords, species, mol_offsets, forces: bool = True, out=None,
                      graph: bool = False, stream=None, accumulate: bool = False, counts=None,
                      bounds=None):
        """Energies [B] (float64) and forces [A, 3] of a ragged batch.

        graph=True replays a captured HIP graph while shapes, tensors and the
        stream stay the same (needs a non-default stream).  accumulate=True
        adds the results to the tensors given in `out`.  counts: an int32
        CUDA tensor {n_mols, n_atoms} read on the device, with bounds =
        (max molecules, max atoms) of the call (default: the tensors'
        lengths); with graph=True every batch within the same rounded bounds
        replays one graph."""
        import torch
        self._need(coords, self.coord_dtype, "coords")
        self._need(species, torch.int32, "species")
        self._need(mol_offsets, torch.int32, "mol_offsets")
        if accumulate and out is None:
            raise ValueError("accumulate needs the output tensors in `out`")
        flags = (FLAG_GRAPH if graph else 0) | (FLAG_ACCUMULATE if accumulate else 0)
        if counts is not None:
            self._need(counts, torch.int32, "counts")
            flags |= FLAG_DEVICE_COUNTS
        b = self._batch(species, mol_offsets, stream=stream, flags=flags)
        if counts is not None:
            b.counts = counts.data_ptr()
            if bounds is not None:
                b.n_mols, b.n_atoms = int(bounds[0]), int(bounds[1])
        if out is None:
            E = torch.empty(b.n_mols, dtype=torch.float64, device=coords.device)
            F = torch.empty_like(coords) if forces else None
        else:
            E, F = out
        fn = self.lib.nnp_energy_forces_f64 if self.precision == "fp64" else self.lib.nnp_energy_forces
        _check(fn(self.h, C.byref(b), coords.data_ptr(), E.data_ptr(),
                  F.data_ptr() if F is not None else None))
        return E, F

    def aev(self, coords, species, mol_offsets):
        import torch
        self._need(coords, self.coord_dtype, "coords")
        b = self._batch(species, mol_offsets)
        out = torch.empty((b.n_atoms, self.aev_dim), dtype=self.coord_dtype, device=coords.device)
        _check(self.lib.nnp_aev(self.h, C.byref(b), coords.data_ptr(), out.data_ptr()))
        return out

    def backward(self, coords, species, mol_offsets, grad_E=None, grad_F=None,
                 want_coords: bool = False):
        """dL/dW (packed like the weights) and optionally dL/dx."""
        import torch
        self._need(coords, self.coord_dtype, "coords")
        if grad_E is not None:
            self._need(grad_E, torch.float64, "grad_E")
        if grad_F is not None:
            self._need(grad_F, self.coord_dtype, "grad_F")
        b = self._batch(species, mol_offsets)
        gp = torch.empty(self.num_params, dtype=self.coord_dtype, device=coords.device)
        gx = torch.empty_like(coords) if want_coords else None
        _check(self.lib.nnp_energy_forces_backward(
            self.h, C.byref(b), coords.data_ptr(),
            grad_E.data_ptr() if grad_E is not None else None,
            grad_F.data_ptr() if grad_F is not None else None,
            gp.data_ptr(), gx.data_ptr() if gx is not None else None))
        return gp, gx

    def set_weights(self, weights):
        w = np.ascontiguousarray(weights, dtype=np.float64)
        _check(self.lib.nnp_set_weights(self.h, _dp(w)))
        self._synced = None

    def set_params(self, params, stream=None):
        """Replace the weights from a CUDA tensor (float64 or float32, packed
        like the weights) on the device, enqueued on `stream` (torch's
        current stream by default): no host round trip."""
        import torch
        if params.dtype == torch.float64:
            typ = PREC["fp64"]
        elif params.dtype == torch.float32:
            typ = PREC["fp32"]
        else:
            raise TypeError("params must be float64 or float32")
        self._need(params, params.dtype, "params")
        if params.numel() != self.num_params:
            raise ValueError(f"params has {params.numel()} values, the model {self.num_params}")
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        _check(self.lib.nnp_set_params(self.h, params.data_ptr(), typ, s.cuda_stream))
        self._synced = None

    def sync_params(self, params):
        """Make the handle hold the weights in `params` unless it is the very
        tensor object uploaded last time with no in-place change since (torch's
        version counter).  The handle keeps a reference to that tensor, so a
        new tensor can never be mistaken for it through a reused address.
        CUDA tensors are copied on the device (nnp_set_params), anything else
        through host memory.  Writes that bypass the version counter (through
        `.data`) are not seen: call set_weights or set_params after those."""
        import torch
        last = getattr(self, "_synced", None)
        if last is not None and last[0] is params and last[1] == params._version:
            return
        p = params.detach()
        if p.is_cuda and p.dtype in (torch.float64, torch.float32):
            self.set_params(p.contiguous())
        else:
            self.set_weights(p.to("cpu", dtype=torch.float64).numpy())
        self._synced = (params, params._version)

    def graph_stats(self) -> dict:
        """Captures and replays of evaluation graphs, and graphs cached."""
        c, r, n = C.c_int64(0), C.c_int64(0), C.c_int32(0)
        _check(self.lib.nnp_graph_stats(self.h, C.byref(c), C.byref(r), C.byref(n)))
        return {"captures": int(c.value), "replays": int(r.value), "cached": int(n.value)}

    @property
    def num_params(self) -> int:
        return int(self.lib.nnp_num_params(self.h))

    @property
    def aev_dim(self) -> int:
        return int(self.lib.nnp_aev_dim(self.h))

    def device_status(self) -> int:
        code = C.c_int32(0)
        _check(self.lib.nnp_get_device_status(self.h, C.byref(code)))
        return int(code.value)

    def set_timing(self, on: bool, only: str | None = None):
        """Per-kernel event timing on or off; `only` restricts it to one
        kernel name (None: every kernel)."""
        _check(self.lib.nnp_set_timing_only(self.h, only.encode() if only else None))
        _check(self.lib.nnp_set_timing(self.h, 1 if on else 0))

    def set_knob(self, name: str, value: int):
        """Select a kernel variant (0 = automatic); see include/nnp.h."""
        _check(self.lib.nnp_set_knob(self.h, KNOBS[name], int(value)))

    def get_knob(self, name: str) -> int:
        v = C.c_int32(0)
        _check(self.lib.nnp_get_knob(self.h, KNOBS[name], C.byref(v)))
        return int(v.value)

    def autotune(self, coords, species, mol_offsets, reps: int = 5, cache_path=None) -> dict:
        """Time every variant on this batch, keep the fastest; returns the
        tuner's report (key, chosen values, microseconds per candidate)."""
        import json
        import torch
        self._need(coords, self.coord_dtype, "coords")
        self._need(species, torch.int32, "species")
        self._need(mol_offsets, torch.int32, "mol_offsets")
        b = self._batch(species, mol_offsets)
        buf = C.create_string_buffer(8192)
        path = os.fsencode(cache_path) if cache_path is not None else None
        _check(self.lib.nnp_autotune(self.h, C.byref(b), coords.data_ptr(), int(reps), path, buf,
                                     len(buf)))
        return json.loads(buf.value.decode())

    def kernel_times(self) -> dict:
        n = self.lib.nnp_kernel_times(self.h, 0, None, None, None)
        names = (C.c_char_p * max(n, 1))()
        counts = (C.c_int64 * max(n, 1))()
        ms = (C.c_double * max(n, 1))()
        n = self.lib.nnp_kernel_times(self.h, n, names, counts, ms)
        return {names[i].decode(): (int(counts[i]), float(ms[i])) for i in range(n)}


class Coupling:
    """NNP-MM mechanical-embedding coupling (include/nnp.h): energy and
    forces on both regions, FP64 or FP32, on the device."""

    def __init__(self, max_nnp: int, max_mm: int, coulomb_k: float, cutoff: float = 0.0,
                 precision: str = "fp32", device: int = 0):
        lib = load_library()
        if precision not in ("fp32", "fp64"):
            raise ValueError("coupling precision is fp32 or fp64")
        h = C.c_void_p()
        _check(lib.nnp_coupling_create(PREC[precision], int(max_nnp), int(max_mm), float(coulomb_k),
                                       float(cutoff), int(device), C.byref(h)))
        self.h, self.lib, self.precision, self.device = h, lib, precision, device

    def close(self):
        if getattr(self, "h", None):
            self.lib.nnp_coupling_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __call__(self, x_nnp, par_nnp, x_mm, par_mm, out=None, accumulate: bool = False,
                 stream=None):
        """E (1-element float64 tensor), F_nnp [n_nnp, 3], F_mm [n_mm, 3]."""
        import torch
        dt = torch.float64 if self.precision == "fp64" else torch.float32
        for t, name in ((x_nnp, "x_nnp"), (par_nnp, "par_nnp"), (x_mm, "x_mm"), (par_mm, "par_mm")):
            NNP._need(t, dt, name)
        n_nnp, n_mm = x_nnp.shape[0], x_mm.shape[0]
        if out is None:
            E = torch.zeros(1, dtype=torch.float64, device=x_nnp.device)
            Fn = torch.zeros_like(x_nnp)
            Fm = torch.zeros_like(x_mm)
        else:
            E, Fn, Fm = out
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        _check(self.lib.nnp_coupling_eval(self.h, n_nnp, x_nnp.data_ptr(), par_nnp.data_ptr(), n_mm,
                                          x_mm.data_ptr(), par_mm.data_ptr(), E.data_ptr(),
                                          Fn.data_ptr(), Fm.data_ptr(), s.cuda_stream,
                                          FLAG_ACCUMULATE if accumulate else 0))
        return E, Fn, Fm


def coupling_noalloc(x_nnp, par_nnp, x_mm, par_mm, coulomb_k: float, cutoff: float = 0.0,
                     out=None, accumulate: bool = False, stream=None):
    """The coupling of `Coupling.__call__` through the handle-free,
    allocation-free entry point (static per-device scratch; calls on one GPU
    must not overlap).  Outputs are allocated here unless `out` is given."""
    import torch
    lib = load_library()
    if x_nnp.dtype == torch.float64:
        prec, dt = PREC["fp64"], torch.float64
    elif x_nnp.dtype == torch.float32:
        prec, dt = PREC["fp32"], torch.float32
    else:
        raise TypeError("coordinates must be float32 or float64")
    for t, name in ((x_nnp, "x_nnp"), (par_nnp, "par_nnp"), (x_mm, "x_mm"), (par_mm, "par_mm")):
        NNP._need(t, dt, name)
    if out is None:
        E = torch.zeros(1, dtype=torch.float64, device=x_nnp.device)
        Fn, Fm = torch.zeros_like(x_nnp), torch.zeros_like(x_mm)
    else:
        E, Fn, Fm = out
    s = stream if stream is not None else torch.cuda.current_stream(x_nnp.device)
    _check(lib.nnp_coupling_eval_noalloc(prec, float(coulomb_k), float(cutoff), x_nnp.shape[0],
                                         x_nnp.data_ptr(), par_nnp.data_ptr(), x_mm.shape[0],
                                         x_mm.data_ptr(), par_mm.data_ptr(), E.data_ptr(),
                                         Fn.data_ptr(), Fm.data_ptr(), s.cuda_stream,
                                         FLAG_ACCUMULATE if accumulate else 0))
    return E, Fn, Fm
