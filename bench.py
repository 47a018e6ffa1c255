#!/usr/bin/env python3
"""Throughput of the NNP energy+force path on one MI355X.

Headline (value): atom energy+force evaluations per second of the 8-model
ensemble on 1024 Gaussian replicas of a 48-atom ligand, BF16 network GEMMs
with FP32 accumulation, FP32 featuriser and forces (inputs resident in HBM).
Beside it, in the same JSON line:
  plain_fp32   the single 64-atom ligand in FP32, one call per evaluation
               (the paper's own MD workload: one molecule, low latency),
               timed as graph replays and as one-by-one launches (value:
               the faster); plain_bf16 the same with BF16 networks
  roofline     the dominant kernel's algorithmic FLOP rate from HIP events
               recorded around every launch inside the timed region
  cpu_baseline the FP64 C oracle on a bounded sample of the same workload
  accuracy     errors of the timed GPU results against that oracle sample

A step = one full evaluation (neighbour lists, AEVs, element bucketing,
ensemble networks forward and backward, force scatter, energy sums).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "atom energy+force evals/s (8-model ensemble), batched BF16 vs plain FP32"

# MI355X published peaks
PEAK = {"bf16": 2.5e15, "fp32": 157.3e12, "fp64": 78.6e12}
HBM_BW = 8.0e12            # bytes/s
# plain (non-packed) FP32 VALU: 256 CUs x 64 lanes x 2 FLOP x 2.4 GHz; the
# transcendental unit (exp2, log2, sin, cos, sqrt, rcp) runs at a quarter of
# the lane rate: 256 x 16 x 2.4 GHz
VALU_FP32 = 78.6e12
TRANS_RATE = 256 * 16 * 2.4e9

# Algorithmic work of the featuriser terms (counted once per unordered pair
# and per angular triple, whatever the kernels recompute):
#   radial, per unordered pair within rcr: 16 Gaussians + the cosine cutoff
#     forward (17 transcendentals), the same with its derivative backward (18);
#   angular, per triple (i; {j,k}) within rca: 8 distance Gaussians, 4 powers
#     (log2 + exp2 each) and one square root forward (17, ~110 FLOP), the same
#     recomputed with their derivatives backward (18, ~250 FLOP);
#   per-pair distance geometry ~10 FLOP each way.
TRANS_PAIR_FWD, TRANS_PAIR_BWD = 17, 18
TRANS_TRIPLE_FWD, TRANS_TRIPLE_BWD = 17, 18
FLOP_PAIR_FWD, FLOP_PAIR_BWD = 60, 90
FLOP_TRIPLE_FWD, FLOP_TRIPLE_BWD = 110, 250


def geometry_counts(batch, rcr, rca):
    """Unordered pairs within rcr and angular triples (i; {j<k}) with both
    r_ij, r_ik < rca, counted from the batch's coordinates."""
    o = np.asarray(batch.mol_offsets)
    x = np.asarray(batch.coords)
    pairs = triples = 0
    sizes = np.diff(o)
    # molecules of one size in one vectorised block
    for n in np.unique(sizes):
        if n < 2:
            continue
        idx = np.nonzero(sizes == n)[0]
        xs = np.stack([x[o[m]:o[m] + n] for m in idx])             # [k, n, 3]
        d2 = ((xs[:, :, None, :] - xs[:, None, :, :]) ** 2).sum(-1)
        eye = np.eye(n, dtype=bool)[None]
        pairs += int(((d2 < rcr * rcr) & ~eye).sum()) // 2
        na = ((d2 < rca * rca) & ~eye).sum(-1)
        triples += int((na * (na - 1) // 2).sum())
    return pairs, triples


def stage_floors(hp, M, n_atoms, pairs, triples, g_bytes, dg_bytes, mfma_peak=PEAK["bf16"]):
    """Per-stage lower bounds (seconds) of one evaluation: the larger of the
    MFMA time (networks), the VALU and transcendental times (featuriser,
    forces, CELU) and the HBM time of the bytes each stage must move in this
    staging (AEV rows out of the featuriser, dE/dAEV rows into the force
    kernel).  The sum over stages is the step floor."""
    f = mlp_flops_per_atom(hp, M)
    w = hp["widths"]
    mlp_flops = (f["mlp_l1_fwd"] + f["mlp_tail"] + f["mlp_l1_bwd"]) * n_atoms
    celu_exps = M * sum(w[1:-1]) * n_atoms
    aev_trans = TRANS_PAIR_FWD * pairs + TRANS_TRIPLE_FWD * triples
    aev_flops = FLOP_PAIR_FWD * pairs + FLOP_TRIPLE_FWD * triples
    frc_trans = TRANS_PAIR_BWD * pairs + TRANS_TRIPLE_BWD * triples
    frc_flops = FLOP_PAIR_BWD * pairs + FLOP_TRIPLE_BWD * triples
    st = {
        "networks": {"mfma_s": mlp_flops / mfma_peak, "trans_s": celu_exps / TRANS_RATE},
        "aev": {"trans_s": aev_trans / TRANS_RATE, "valu_s": aev_flops / VALU_FP32,
                "hbm_s": (g_bytes + 12 * n_atoms) / HBM_BW},
        "forces": {"trans_s": frc_trans / TRANS_RATE, "valu_s": frc_flops / VALU_FP32,
                   "hbm_s": (dg_bytes + 24 * n_atoms) / HBM_BW},
    }
    for v in st.values():
        v["floor_s"] = max(v.values())
    return st


def mlp_flops_per_atom(hp, M):
    """Algorithmic FLOPs per atom of each network kernel (unpadded widths)."""
    w = hp["widths"]
    f = {
        "mlp_l1_fwd": 2 * M * w[0] * w[1],
        "mlp_l2_fwd": 2 * M * w[1] * w[2],
        "mlp_l3_fwd": 2 * M * w[2] * w[3] + 2 * M * w[3],
        "mlp_l3_bwd": 2 * M * w[3] * w[2],
        "mlp_l2_bwd": 2 * M * w[2] * w[1],
        "mlp_l1_bwd": 2 * M * w[1] * w[0],
    }
    # the fused tail runs layers 2-3 forward and backward in one kernel
    f["mlp_tail"] = f["mlp_l2_fwd"] + f["mlp_l3_fwd"] + f["mlp_l3_bwd"] + f["mlp_l2_bwd"]
    return f


def run_form(torch, h, batch, steps, warmup, timing, graph=False, per_step=False, only=None):
    """Time `steps` evaluations after `warmup` (inputs already on the device).
    Returns mean seconds per evaluation, per-kernel totals (timing=True),
    the last E and F, and (per_step=True) per-evaluation milliseconds from
    HIP events recorded between evaluations on the evaluation stream."""
    dev = torch.device("cuda:0")
    x = torch.tensor(batch.coords, dtype=torch.float32, device=dev)
    sp = torch.tensor(batch.species, dtype=torch.int32, device=dev)
    off = torch.tensor(batch.mol_offsets, dtype=torch.int32, device=dev)
    E = torch.empty(batch.n_mols, dtype=torch.float64, device=dev)
    F = torch.empty_like(x)
    stream = torch.cuda.Stream() if graph else torch.cuda.current_stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        for _ in range(warmup):
            h.energy_forces(x, sp, off, out=(E, F), graph=graph, stream=stream)
    torch.cuda.synchronize()
    if h.device_status() != 0:
        raise RuntimeError("device flagged an error during warmup")
    h.set_timing(timing, only)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)] if per_step else None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        for i in range(steps):
            if ev:
                ev[i].record(stream)
            h.energy_forces(x, sp, off, out=(E, F), graph=graph, stream=stream)
        if ev:
            ev[steps].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = h.kernel_times() if timing else {}
    h.set_timing(False)
    steps_ms = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)] if ev else None
    return (t1 - t0) / steps, kt, E.cpu().numpy(), F.double().cpu().numpy(), steps_ms


def source_digest(files):
    """sha256 over kernel source files (ties stored counter readings to the
    exact code they were taken from)."""
    import hashlib
    hsh = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            hsh.update(fh.read())
    return hsh.hexdigest()


def stored_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE per dispatch, normalised by a plain copy of
    known size), or None if absent or taken from other kernel sources."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic_bf16_replicas_1024x48.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    meta = dict(l.split(":", 1) for l in txt.splitlines() if l.startswith(("sources:", "sha256:")))
    files = meta.get("sources", "").split()
    if not files or source_digest(files) != meta.get("sha256", "").strip():
        return None
    for line in txt.splitlines():
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) >= 5 and cells[0] == kernel:
            try:
                return float(cells[4])
            except ValueError:
                return None
    return None


def _omp_threads(n):
    """OpenMP thread count of the calling thread (the oracle's parallel
    regions use it)."""
    import ctypes
    try:
        ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(n))
    except (OSError, AttributeError):
        pass


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _sub_batch(batch, mols):
    """Species, coordinates, offsets and atom rows of some molecules."""
    o = np.asarray(batch.mol_offsets)
    rows = np.concatenate([np.arange(o[m], o[m + 1]) for m in mols])
    off = np.concatenate([[0], np.cumsum([o[m + 1] - o[m] for m in mols])]).astype(np.int64)
    return np.asarray(batch.species)[rows], np.asarray(batch.coords)[rows], off, rows


def accuracy_of(E, F, Eo, Fo, offsets):
    """Per-molecule |dE|/atom, force RMSE and largest force-component error
    (kcal/mol, kcal/mol/A) against the oracle."""
    sizes = np.diff(offsets)
    dE = np.abs(E - Eo) / np.maximum(sizes, 1)
    rmse = np.array([np.sqrt(np.mean((F[a:b] - Fo[a:b]) ** 2)) for a, b in zip(offsets[:-1], offsets[1:])
                     if b > a])
    dF = np.abs(F - Fo)
    return {"molecules": int(len(sizes)), "dE_per_atom_max": float(dE.max()),
            "dE_per_atom_median": float(np.median(dE)), "force_rmse_max": float(rmse.max()),
            "force_rmse_median": float(np.median(rmse)), "force_component_abs_err_max": float(dF.max()),
            "force_rms": float(np.sqrt(np.mean(Fo ** 2)))}


def cpu_leg(hp, w, M, b5, jobs, synth):
    """The FP64 C oracle as the CPU baseline (the whole headline batch once
    on every host thread, and the 64-atom ligand on one and on every thread)
    and, from the same oracle, the accuracy of each timed form: its energies
    and forces against the oracle on the inputs the path receives
    (FP32-rounded coordinates and weights)."""
    import oracle
    n_all = oracle.num_threads()
    wo = synth.round_to_fp32(w)
    t0 = time.perf_counter()
    E5o, F5o = oracle.energy_forces(hp, wo, M, b5.species, synth.round_to_fp32(b5.coords), b5.mol_offsets)
    t_all = time.perf_counter() - t0
    b2 = synth.config_batch(2)

    def ligand_rate(threads, budget):
        _omp_threads(threads)
        n, t = 0, 0.0
        while t < budget:
            t0 = time.perf_counter()
            oracle.energy_forces(hp, w, M, b2.species, b2.coords, b2.mol_offsets)
            t += time.perf_counter() - t0
            n += 1
        return t / n

    t1 = ligand_rate(1, 3.0)
    tn = ligand_rate(n_all, 1.0)
    _omp_threads(n_all)
    base = {"value": b5.n_atoms / t_all, "unit": "atom-evals/s", "cores": n_all, "kind": "oracle",
            "sample": f"the whole headline batch ({b5.n_atoms} atoms) once on {n_all} threads: {t_all:.1f} s, FP64",
            "cpu_model": cpu_model(),
            "one_core": {"value": b2.n_atoms / t1, "unit": "atom-evals/s",
                         "sample": f"the 64-atom ligand, 8 models, 1 thread: {t1 * 1e3:.1f} ms per evaluation"},
            "ligand_64_all_cores": {"value": b2.n_atoms / tn, "unit": "atom-evals/s",
                                    "sample": f"the 64-atom ligand on {n_all} threads: {tn * 1e3:.1f} ms"}}
    acc = {}
    for where, b, prec, E, F, mols in jobs:
        if b is b5 and mols is None:
            Eo, Fo, Es, Fs, off = E5o, F5o, E, F, np.asarray(b5.mol_offsets)
        else:
            mols = list(range(b.n_mols)) if mols is None else mols
            sp, xc, off, rows = _sub_batch(b, mols)
            Eo, Fo = oracle.energy_forces(hp, wo, M, sp, synth.round_to_fp32(xc), off)
            Es, Fs = np.asarray(E)[mols], np.asarray(F)[rows]
        a = accuracy_of(Es, Fs, Eo, Fo, np.asarray(off))
        a["vs"] = "FP64 oracle on the FP32-rounded coordinates and weights the path receives"
        a["precision"] = prec
        acc[where] = a
    return base, acc


# flops of one coupling pair as counted here: distance (8), reciprocal and
# reciprocal square root (2), Coulomb (2), Lennard-Jones powers and energy
# (9), dV/dr (6), force components (6).  One evaluation per pair is the
# algorithmic count (Newton's third law serves both sides); the kernels
# evaluate every pair once per side, twice that
COUPLING_FLOPS_PER_PAIR = 33


def coupling_form(torch, nnp, synth, args):
    s = synth.coupling_system()
    n_pairs = len(s.x_nnp) * len(s.x_mm)
    res = {"workload": f"{len(s.x_nnp)}-atom ligand in {len(s.x_mm)} MM atoms (all pairs)",
           "pairs": n_pairs}
    for prec in ("fp32", "fp64"):
        dt = torch.float32 if prec == "fp32" else torch.float64
        c = nnp.Coupling(len(s.x_nnp), len(s.x_mm), synth.COULOMB_K, 0.0, prec)
        xs = [torch.tensor(a, dtype=dt, device="cuda") for a in (s.x_nnp, s.par_nnp, s.x_mm, s.par_mm)]
        out = c(*xs)
        # time the C ABI call itself: arguments marshalled once
        args_ = (c.h, len(s.x_nnp), xs[0].data_ptr(), xs[1].data_ptr(), len(s.x_mm), xs[2].data_ptr(),
                 xs[3].data_ptr(), out[0].data_ptr(), out[1].data_ptr(), out[2].data_ptr(),
                 torch.cuda.current_stream().cuda_stream, 0)
        fn = c.lib.nnp_coupling_eval
        for _ in range(5):
            fn(*args_)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        reps = 200
        for _ in range(reps):
            fn(*args_)
        e1.record()
        torch.cuda.synchronize()
        us = 1e3 * e0.elapsed_time(e1) / reps
        fl = COUPLING_FLOPS_PER_PAIR * n_pairs
        peak = PEAK["fp32"] if prec == "fp32" else PEAK["fp64"]
        res[prec] = {"us_per_eval": us, "pair_evals_per_s": n_pairs / (us * 1e-6),
                     "roofline": {"bound": "alu", "achieved": fl / (us * 1e-6) / 1e12,
                                  "peak": peak / 1e12, "unit": "TFLOP/s",
                                  "frac": fl / (us * 1e-6) / peak,
                                  "flops_per_launch": fl, "executed_flops": 2 * fl}}
        c.close()
    if not args.no_cpu:
        import oracle
        t0 = time.perf_counter()
        oracle.coupling(s.x_nnp, s.par_nnp, s.x_mm, s.par_mm, synth.COULOMB_K)
        t = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": n_pairs / t, "unit": "pair-evals/s", "cores": 1,
                               "kind": "oracle", "sample": "the whole system once, FP64"}
    return res


def overlap_form(torch, nnp, synth, hp, w, M, reps=200, n_probe=1024):
    """The ligand's NNP/MM force step (V_NNP graph + coupling, FP32) alone,
    an MM stand-in alone (Coulomb terms of n_probe MM atoms with the rest of
    the environment), both on one stream, and both on two streams joined every
    step; overlap = (t_step + t_mm - t_concurrent) / min(t_step, t_mm)."""
    from paper_2201_08110_amd.nnpmm import NNPMMStep
    s = synth.coupling_system()
    lig = synth.config_batch(2)
    f32 = torch.float32
    dev = lambda a, dt=f32: torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    x_nnp, x_mm, p_nnp, p_mm = dev(s.x_nnp), dev(s.x_mm), dev(s.par_nnp), dev(s.par_mm)
    sp, off = dev(lig.species, torch.int32), dev(lig.mol_offsets, torch.int32)
    model = nnp.NNP(hp, w, M, "fp32", max_atoms=len(s.x_nnp), max_mols=1, max_atoms_per_mol=len(s.x_nnp))
    coup = nnp.Coupling(len(s.x_nnp), len(s.x_mm), synth.COULOMB_K, 0.0, "fp32")
    probe = nnp.Coupling(n_probe, len(s.x_mm) - n_probe, synth.COULOMB_K, 0.0, "fp32")
    step = NNPMMStep(model, coup, sp, off, p_nnp, p_mm)
    E = torch.empty(1, dtype=torch.float64, device="cuda")
    Fn, Fm = torch.empty_like(x_nnp), torch.zeros_like(x_mm)
    Ep = torch.zeros(1, dtype=torch.float64, device="cuda")
    pq = s.par_mm[:n_probe].copy()
    pq[:, 2] = 0.0   # no LJ between the unscreened MM stand-in atoms
    xp, pp, xe, pe = dev(s.x_mm[:n_probe]), dev(pq), dev(s.x_mm[n_probe:]), dev(s.par_mm[n_probe:])
    Fpn, Fpm = torch.zeros((n_probe, 3), dtype=f32, device="cuda"), torch.zeros_like(xe)
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    ev = [torch.cuda.Event() for _ in range(2)]

    def run(mode):
        for i in range(reps):
            if mode == "conc":
                # both start when the previous step has joined; a waits for b
                ev[0].record(sa)
                sb.wait_event(ev[0])
            if mode in ("step", "seq", "conc"):
                step(x_nnp, x_mm, E, Fn, Fm, sa)
            if mode in ("mm", "seq"):
                probe(xp, pp, xe, pe, out=(Ep, Fpn, Fpm), stream=sa)
            if mode == "conc":
                probe(xp, pp, xe, pe, out=(Ep, Fpn, Fpm), stream=sb)
                ev[1].record(sb)
                sa.wait_event(ev[1])

    res = {"workload": f"{len(s.x_nnp)}-atom ligand NNP/MM force step (8-model FP32 NNP graph + coupling "
                       f"with {len(s.x_mm)} MM atoms) || MM stand-in ({n_probe} x {len(s.x_mm) - n_probe} Coulomb terms)"}
    for mode in ("step", "mm", "seq", "conc"):
        run(mode)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run(mode)
        torch.cuda.synchronize()
        res[f"us_{mode}"] = (time.perf_counter() - t0) / reps * 1e6
    res["overlap"] = (res["us_step"] + res["us_mm"] - res["us_conc"]) / min(res["us_step"], res["us_mm"])
    model.close(); coup.close(); probe.close()
    return res


def training_form(torch, nnp, synth, hp, w, M, reps=20):
    """Workload 4 (64 molecules of 30-80 atoms, 8 models, FP32): one training
    step = energies and forces, then dL/dW of a loss of both (force term
    included); and the same with dL/dx (the Hessian-vector product)."""
    b = synth.config_batch(4)
    h = nnp.NNP(hp, w, M, "fp32", max_atoms=b.n_atoms, max_mols=b.n_mols, max_atoms_per_mol=80)
    x = torch.tensor(b.coords, dtype=torch.float32, device="cuda")
    sp = torch.tensor(b.species, dtype=torch.int32, device="cuda")
    off = torch.tensor(b.mol_offsets, dtype=torch.int32, device="cuda")
    rng = np.random.default_rng(4)
    gE = torch.tensor(rng.normal(size=b.n_mols) * 1e-2, dtype=torch.float64, device="cuda")
    gF = torch.tensor(rng.normal(size=(b.n_atoms, 3)) * 1e-2, dtype=torch.float32, device="cuda")
    res = {"workload": f"{b.n_mols} molecules of 30-80 atoms ({b.n_atoms} atoms), 8-model ensemble, FP32",
           "atoms": int(b.n_atoms)}
    for name, want_x in (("param_grad", False), ("param_and_coord_grad", True)):
        def step():
            h.energy_forces(x, sp, off)
            h.backward(x, sp, off, gE, gF, want_coords=want_x)
        for _ in range(3):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            step()
        torch.cuda.synchronize()
        res[f"ms_per_step_{name}"] = (time.perf_counter() - t0) / reps * 1e3
    h.set_timing(True)
    for _ in range(5):
        h.energy_forces(x, sp, off)
        h.backward(x, sp, off, gE, gF, want_coords=True)
    torch.cuda.synchronize()
    res["kernels_us"] = {k: 1e3 * ms / c for k, (c, ms) in h.kernel_times().items()}
    h.set_timing(False)
    h.close()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--replicas", type=int, default=1024)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain FP32 form")
    ap.add_argument("--no-forms", action="store_true", help="skip the like-for-like batched forms")
    ap.add_argument("--no-coupling", action="store_true", help="skip the NNP-MM coupling form")
    ap.add_argument("--no-overlap", action="store_true",
                    help="skip the NNP/MM step overlapped with an MM stand-in")
    ap.add_argument("--profile-only", choices=["ligand_fp32", "ligand_bf16", "ragged_fp32", "ragged_bf16"],
                    default=None,
                    help="run only this workload (steps evaluations after warmup, graph replays) and "
                         "print its timing: a short run for a kernel trace of that form")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first run one elementwise copy (negation) of this many MiB (a "
                         "reference dispatch for HBM traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(molecules shard across GPUs with no exchange between them)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2201_08110_amd import nnp, synth
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    hp = synth.ani2x_hparams()
    M = 8
    w = synth.xavier_weights(M, hp["widths"])
    if args.copy_mib:
        # one elementwise pass that reads and writes copy_mib MiB each: a
        # dispatch of known traffic (its own kernel name) for normalising HBM
        # byte counters
        src = torch.ones(args.copy_mib * (1 << 20) // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst

    accuracy_jobs = []   # (where, batch, precision, E, F, molecules compared or None = all)

    if args.profile_only:
        wl, prec = args.profile_only.split("_")
        b = synth.config_batch(2 if wl == "ligand" else 3)
        apm = 64 if wl == "ligand" else 120
        hq = nnp.NNP(hp, w, M, prec, max_atoms=b.n_atoms, max_mols=b.n_mols, max_atoms_per_mol=apm)
        secq, _, _, _, _ = run_form(torch, hq, b, args.steps, args.warmup, timing=False, graph=True)
        print(json.dumps({"profile_only": args.profile_only, "atoms": int(b.n_atoms),
                          "us_per_eval": secq * 1e6, "steps": args.steps}))
        hq.close()
        return

    # ---- headline: batched BF16-MLP replicas -----------------------------
    b5 = synth.config_batch(5, n_mols=args.replicas)
    h5 = nnp.NNP(hp, w, M, "bf16", max_atoms=b5.n_atoms, max_mols=b5.n_mols, max_atoms_per_mol=48)
    # Calibration: every kernel bracketed by HIP events, to name the slowest
    # kernel and report the per-kernel split.  The timed region then records
    # events around that kernel only (each event record between kernels
    # costs GPU time, ~60 us per evaluation for all of them), plus
    # per-evaluation events; `value` and the roofline come from it.
    cal_steps = min(args.steps, 20)
    _, kt_all, _, _, _ = run_form(torch, h5, b5, cal_steps, args.warmup, timing=True)
    flops = mlp_flops_per_atom(hp, M)
    # per evaluation: the pipelined evaluation launches each kernel once per
    # half-batch (the two launches of one kernel never overlap), so a
    # kernel's time per evaluation is the sum of its launches
    per_kernel = {k: {"launches_per_eval": c / cal_steps, "avg_us": 1e3 * ms / cal_steps}
                  for k, (c, ms) in kt_all.items()}
    gemms = {k: v for k, v in per_kernel.items() if k in flops}
    dom = max(per_kernel, key=lambda k: per_kernel[k]["avg_us"]) if per_kernel else None
    sec, kt, E5, F5, steps_ms = run_form(torch, h5, b5, args.steps, args.warmup, timing=True,
                                         per_step=True, only=dom)
    value = b5.n_atoms / sec
    dom_us = 1e3 * kt[dom][1] / args.steps if dom in kt else None
    roof = None
    if dom in flops and dom_us:
        achieved = flops[dom] * b5.n_atoms / (dom_us * 1e-6)
        roof = {"kernel": dom, "bound": "mfma", "achieved": achieved / 1e12,
                "peak": PEAK["bf16"] / 1e12, "unit": "TFLOP/s",
                "frac": achieved / PEAK["bf16"], "traffic": stored_traffic(dom),
                "flops_per_launch": flops[dom] * b5.n_atoms}
    mlp_total_us = sum(v["avg_us"] for v in gemms.values())
    mlp_flops = sum(flops[k] for k in gemms) * b5.n_atoms
    # every kernel against its own bound; the step against the sum of the
    # stage floors (Sigma_stages max(flops / peak, transcendentals / rate,
    # bytes / HBM) / measured time)
    pairs5, triples5 = geometry_counts(b5, hp["rcr"], hp["rca"])
    D = synth.aev_dim(hp)
    # BF16 handles keep both the AEV rows and the dE/dAEV rows in bf16
    st5 = stage_floors(hp, M, b5.n_atoms, pairs5, triples5, g_bytes=2 * D * b5.n_atoms,
                       dg_bytes=2 * D * b5.n_atoms)
    for k, v in per_kernel.items():
        if k in flops:
            v["tflops"] = flops[k] * b5.n_atoms / (v["avg_us"] * 1e-6) / 1e12
            v["bound"], v["floor_us"] = "mfma", flops[k] * b5.n_atoms / PEAK["bf16"] * 1e6
        elif k in ("aev", "forces"):
            fl = st5[k]
            v["bound"] = max(("trans", fl["trans_s"]), ("valu", fl["valu_s"]), ("hbm", fl["hbm_s"]),
                             key=lambda t: t[1])[0]
            v["floor_us"] = fl["floor_s"] * 1e6
        elif k == "neighbours":
            # per atom: coordinates and element in (16 B), its list out (2 B per
            # neighbour within Rcr) with its count (4 B), its force row cleared
            # (12 B); the candidate tests (pairs of a molecule, ~8 FLOP each,
            # both orders) are far below the VALU peak
            nbytes = b5.n_atoms * (16 + 4 + 12) + 2 * 2 * pairs5
            v["bound"], v["floor_us"] = "hbm", nbytes / HBM_BW * 1e6
        elif k == "prep":
            # per atom: element in, molecule, row and the row's atom out (16 B)
            v["bound"], v["floor_us"] = "hbm", b5.n_atoms * 16 / HBM_BW * 1e6
        else:
            continue
        v["frac"] = v["floor_us"] / v["avg_us"]
    step_floor = sum(v["floor_s"] for v in st5.values())

    out = {
        "metric": METRIC, "value": value, "unit": "atom-evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": sec * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
        "data": "synthetic (seeded replicas, Xavier weights)",
        "config": {"workload": f"{b5.n_mols} replicas x 48-atom ligand (H,C,N,O,F,S,Cl 22:15:4:4:1:1:1), "
                               "sigma 0.05 A, 8-model ensemble, BF16 MLP / FP32 AEV+forces",
                   "atoms_per_eval": int(b5.n_atoms), "precision": "bf16-mlp"},
        "roofline": roof,
        "ms_per_eval_p10_p50_p90": [float(np.percentile(steps_ms, q)) for q in (10, 50, 90)],
        "kernels": per_kernel,
        "kernels_timing": "calibration pass with every launch timed (microseconds per evaluation, summed "
                          "over its launches); the timed region times only "
                          f"{dom} ({dom_us:.1f} us per evaluation there)" if dom_us else None,
        "pipeline": h5.get_knob("pipeline"),
        "mlp_gemm_tflops": mlp_flops / (mlp_total_us * 1e-6) / 1e12 if mlp_total_us else None,
        "step_roofline": {
            "floor_us": step_floor * 1e6, "frac": step_floor / sec,
            "stages_us": {k: {kk.replace("_s", "_us"): vv * 1e6 for kk, vv in v.items()}
                          for k, v in st5.items()},
            "pairs": pairs5, "triples": triples5,
            "definition": "sum over stages (networks, featuriser, forces) of max(MFMA FLOPs / 2.5 PFLOP/s, "
                          "transcendentals / 9.83 T/s, VALU FLOPs / 78.6 TFLOP/s, bytes crossing HBM between "
                          "stages / 8 TB/s), divided by ms_per_step"},
    }

    # ---- plain FP32 single ligand ----------------------------------------
    if not args.no_plain:
        b2 = synth.config_batch(2)
        # the single molecule is bound by streaming the weights of the
        # elements it holds once per evaluation (all 7 here)
        n_el = len(np.unique(b2.species))
        net_params = synth.net_size(hp["widths"])
        h2 = nnp.NNP(hp, w, M, "fp32", max_atoms=b2.n_atoms, max_mols=1, max_atoms_per_mol=64)
        # both launch modes of the library: one captured graph per evaluation,
        # and the kernels launched one by one (back to back on one stream the
        # latter measured a few microseconds faster per evaluation here: a
        # graph launch adds its own completion step); the faster one is the
        # form's value
        for prec, esize in (("fp32", 4), ("bf16", 2)):
            h2 = nnp.NNP(hp, w, M, prec, max_atoms=b2.n_atoms, max_mols=1, max_atoms_per_mol=64)
            sec_e, _, _, _, _ = run_form(torch, h2, b2, max(args.steps, 200), args.warmup, timing=False)
            sec_g, _, E2, F2, _ = run_form(torch, h2, b2, max(args.steps, 200), args.warmup,
                                           timing=False, graph=True)
            sec2 = min(sec_e, sec_g)
            wbytes = esize * n_el * M * net_params
            nets = "FP32" if prec == "fp32" else "BF16 networks"
            out["plain_" + prec] = {
                "workload": f"single 64-atom ligand, 8-model ensemble, {nets}",
                "value": b2.n_atoms / sec2, "unit": "atom-evals/s",
                "us_per_eval": sec2 * 1e6, "us_per_eval_graph": sec_g * 1e6, "us_per_eval_eager": sec_e * 1e6,
                "launch": ("one captured HIP graph per evaluation" if sec_g <= sec_e
                           else "kernels launched one by one on one stream"),
                "roofline": {"bound": "hbm", "achieved": wbytes / sec2 / 1e9,
                             "peak": HBM_BW / 1e9, "unit": "GB/s",
                             "frac": wbytes / HBM_BW / sec2, "bytes_per_eval": wbytes,
                             "what": f"{prec.upper()} weights of the {n_el} elements present, read once"}}
            accuracy_jobs.append(("plain_" + prec, b2, prec, E2, F2, None))
            h2.close()

    # ---- like-for-like batched forms: both precisions on the replica batch
    # and on the ragged batch of 512 molecules (10-120 atoms) ---------------
    if not args.no_forms:
        forms = {}
        b3 = synth.config_batch(3)
        sizes3 = np.diff(b3.mol_offsets)
        pick3 = sorted({int(np.argmin(sizes3)), int(np.argmax(sizes3))}
                       | set(np.random.default_rng(13).choice(b3.n_mols, 32, replace=False).tolist()))
        pairs3, triples3 = geometry_counts(b3, hp["rcr"], hp["rca"])
        D = synth.aev_dim(hp)
        for name, b, apm in (("replicas_1024x48", b5, 48), ("ragged_512", b3, 120)):
            for prec in ("fp32", "bf16"):
                if name == "replicas_1024x48" and prec == "bf16":
                    forms[f"{name}_{prec}"] = {"atom_evals_per_s": value, "ms_per_eval": sec * 1e3,
                                               "atoms": int(b.n_atoms), "note": "the headline"}
                    continue
                hf = nnp.NNP(hp, w, M, prec, max_atoms=b.n_atoms, max_mols=b.n_mols,
                             max_atoms_per_mol=apm)
                entry = {}
                if name == "ragged_512":
                    # the ragged batch as its workload runs it: variants chosen
                    # by the autotuner, then one captured graph per evaluation
                    dev = torch.device("cuda:0")
                    rep_ = hf.autotune(torch.tensor(b.coords, dtype=torch.float32, device=dev),
                                       torch.tensor(b.species, dtype=torch.int32, device=dev),
                                       torch.tensor(b.mol_offsets, dtype=torch.int32, device=dev), reps=3)
                    entry["autotuned"] = rep_.get("chosen")
                secf, _, Ef, Ff, _ = run_form(torch, hf, b, 20, 3, timing=False, graph=True)
                p_, t_ = (pairs3, triples3) if name == "ragged_512" else (pairs5, triples5)
                gb = (2 if prec == "bf16" else 4) * D * b.n_atoms
                stf = stage_floors(hp, M, b.n_atoms, p_, t_, g_bytes=gb, dg_bytes=gb,
                                   mfma_peak=PEAK["bf16" if prec == "bf16" else "fp32"])
                fl = sum(v["floor_s"] for v in stf.values())
                entry.update({"atom_evals_per_s": b.n_atoms / secf, "ms_per_eval": secf * 1e3,
                              "atoms": int(b.n_atoms), "launch": "one captured HIP graph per evaluation",
                              "step_roofline_frac": fl / secf, "step_floor_us": fl * 1e6})
                forms[f"{name}_{prec}"] = entry
                accuracy_jobs.append((f"batched_forms.{name}_{prec}", b, prec, Ef, Ff,
                                      pick3 if name == "ragged_512" else list(range(16))))
                hf.close()
        out["batched_forms"] = forms

    # ---- model variants on the replica layout: ANI-2x element networks of
    # their own widths, and the ANI-1x-shaped model (4 elements, 384-dim AEV)
    if not args.no_forms:
        variants = {}
        hp_el = synth.ani2x_heterogeneous_hparams()
        hp_1x = synth.ani1x_hparams()
        b1x = synth.replica_batch(args.replicas, 48, (30, 20, 5, 5))
        for name, hpv, bv, prec in (("ani2x_element_widths_bf16", hp_el, b5, "bf16"),
                                    ("ani1x_bf16", hp_1x, b1x, "bf16"),
                                    ("ani1x_fp32", hp_1x, b1x, "fp32")):
            wv = synth.xavier_weights(M, hpv["species_widths"], n_species=hpv["n_species"])
            hv = nnp.NNP(hpv, wv, M, prec, max_atoms=bv.n_atoms, max_mols=bv.n_mols, max_atoms_per_mol=48)
            secv, _, _, _, _ = run_form(torch, hv, bv, 20, 3, timing=False)
            variants[name] = {"atom_evals_per_s": bv.n_atoms / secv, "ms_per_eval": secv * 1e3,
                              "atoms": int(bv.n_atoms),
                              "widths": [list(x) for x in hpv["species_widths"]]}
            hv.close()
        out["model_variants"] = variants

    # ---- training step (workload 4) ---------------------------------------
    if not args.no_forms:
        out["training"] = training_form(torch, nnp, synth, hp, w, M)

    # ---- NNP/MM step overlapped with MM work on a second stream ----------
    if not args.no_coupling and not args.no_overlap:
        out["nnpmm_overlap"] = [overlap_form(torch, nnp, synth, hp, w, M, n_probe=n) for n in (128, 1024)]

    # ---- NNP-MM coupling (Eq. 4): the 64-atom ligand in 47,648 MM atoms --
    if not args.no_coupling:
        out["coupling"] = coupling_form(torch, nnp, synth, args)

    # ---- CPU leg: the oracle as the CPU baseline, and the accuracy of every
    # timed form against it ------------------------------------------------
    if not args.no_cpu:
        accuracy_jobs.insert(0, ("accuracy", b5, "bf16", E5, F5, None))
        out["cpu_baseline"], acc = cpu_leg(hp, w, M, b5, accuracy_jobs, synth)
        for key, a in acc.items():
            if key == "accuracy":
                out["accuracy"] = a
            elif key.startswith("batched_forms."):
                out["batched_forms"][key.split(".", 1)[1]]["accuracy"] = a
            else:
                out[key]["accuracy"] = a
    h5.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
