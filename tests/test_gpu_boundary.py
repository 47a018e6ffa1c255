"""The boundary of Eq. 2 through the C ABI: an element table of atomic
numbers, weights replaced from device memory, results accumulated onto the
outputs, fixed-point (bitwise reproducible) force sums, the training
workspace allocated at creation, and the autograd Function with several
parameter sets on one model."""
import numpy as np
import pytest

from paper_2201_08110_amd import synth
from tests.gpu_util import errors, make_handle, oracle_inputs, to_device, torch_cuda

pytestmark = pytest.mark.gpu

# atomic numbers of the elements in index order H, C, N, O, F, S, Cl
Z = np.array((1, 6, 7, 8, 9, 16, 17), dtype=np.int32)


def _batch():
    # ragged: an empty molecule, a one-atom molecule, cutoff-cell sizes
    return synth.random_batch(61, [23, 0, 1, 140, 48])


def _eval(torch, h, x, sp, off, **kw):
    E, F = h.energy_forces(x, sp, off, **kw)
    torch.cuda.synchronize()
    assert h.device_status() == 0
    return E.cpu().numpy(), F.double().cpu().numpy()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_atomic_number_table_equals_indices(hp, prec):
    """A handle with the table {1,6,7,8,9,16,17} fed atomic numbers computes
    bitwise what an index handle computes (fixed-point force sums, so the
    forces are reproducible too)."""
    torch = torch_cuda()
    from paper_2201_08110_amd.nnp import NNP
    b = _batch()
    M = 2
    w = synth.xavier_weights(M, hp["widths"], seed=71)
    hi = make_handle(hp, w, M, prec, b)
    hz = NNP(hp, w, M, prec, max_atoms=b.n_atoms, max_mols=b.n_mols, max_atoms_per_mol=140,
             atomic_numbers=Z)
    for h in (hi, hz):
        h.set_knob("force_sum", 2)
    x, sp, off = to_device(torch, b, torch.float32)
    zt = torch.tensor(Z[b.species], dtype=torch.int32, device="cuda")
    Ei, Fi = _eval(torch, hi, x, sp, off)
    Ez, Fz = _eval(torch, hz, x, zt, off)
    assert np.array_equal(Ei, Ez) and np.array_equal(Fi, Fz)
    # the same through the graph path (eager + capture, then replays)
    s = torch.cuda.Stream()
    Eg = torch.empty(b.n_mols, dtype=torch.float64, device="cuda")
    Fg = torch.empty_like(x)
    with torch.cuda.stream(s):
        for _ in range(3):
            Eg.zero_()
            Fg.zero_()
            hz.energy_forces(x, zt, off, graph=True, stream=s, out=(Eg, Fg))
    s.synchronize()
    assert np.array_equal(Eg.cpu().numpy(), Ei) and np.array_equal(Fg.double().cpu().numpy(), Fi)


@pytest.mark.parametrize("bad", [2, 0, 53, 127, -5, 1000])
def test_unknown_atomic_number_sets_species_flag(hp, bad):
    torch = torch_cuda()
    from paper_2201_08110_amd.nnp import NNP, NNP_E_SPECIES
    b = synth.random_batch(62, [9, 5])
    w = synth.xavier_weights(1, hp["widths"], seed=72)
    h = NNP(hp, w, 1, "fp32", max_atoms=b.n_atoms, max_mols=b.n_mols, max_atoms_per_mol=9,
            atomic_numbers=Z)
    x, _, off = to_device(torch, b, torch.float32)
    z = Z[b.species].copy()
    z[3] = bad
    h.energy_forces(x, torch.tensor(z, dtype=torch.int32, device="cuda"), off)
    assert h.device_status() == NNP_E_SPECIES
    # the flag is cleared by the read; a valid batch runs clean again
    h.energy_forces(x, torch.tensor(Z[b.species], dtype=torch.int32, device="cuda"), off)
    assert h.device_status() == 0


@pytest.mark.parametrize("prec,src", [("fp32", "fp64"), ("fp32", "fp32"), ("bf16", "fp64"),
                                      ("fp64", "fp64"), ("het_fp64", "fp64")])
def test_set_params_from_device_equals_creation(hp, prec, src):
    """Weights replaced from a device tensor give bitwise the results of a
    handle created with those weights (the same rounding to the handle's
    precision), also for element networks of their own widths."""
    torch = torch_cuda()
    from paper_2201_08110_amd.nnp import NNP
    b = _batch()
    M = 2
    if prec == "het_fp64":
        h_ = synth.ani2x_heterogeneous_hparams()
        w0 = synth.xavier_weights(M, h_["species_widths"], seed=73)
        w1 = synth.xavier_weights(M, h_["species_widths"], seed=74)
        p = "fp64"
    else:
        h_, p = hp, prec
        w0 = synth.xavier_weights(M, hp["widths"], seed=73)
        w1 = synth.xavier_weights(M, hp["widths"], seed=74)
    if src == "fp32":
        w1 = synth.round_to_fp32(w1)
    kw = dict(max_atoms=b.n_atoms, max_mols=b.n_mols, max_atoms_per_mol=140)
    h = NNP(h_, w0, M, p, **kw)
    ref = NNP(h_, w1, M, p, **kw)
    for hh in (h, ref):
        hh.set_knob("force_sum", 2)
    dt = torch.float64 if p == "fp64" else torch.float32
    x, sp, off = to_device(torch, b, dt)
    E0, _ = _eval(torch, h, x, sp, off)
    h.set_params(torch.tensor(w1, dtype=torch.float64 if src == "fp64" else torch.float32,
                              device="cuda"))
    E1, F1 = _eval(torch, h, x, sp, off)
    Er, Fr = _eval(torch, ref, x, sp, off)
    assert not np.array_equal(E0, E1)
    assert np.array_equal(E1, Er) and np.array_equal(F1, Fr)


def test_set_params_keeps_captured_graph_valid(hp):
    torch = torch_cuda()
    from paper_2201_08110_amd.nnp import NNP
    b = synth.config_batch(2)
    M = 8
    w0 = synth.xavier_weights(M, hp["widths"], seed=75)
    w1 = synth.xavier_weights(M, hp["widths"], seed=76)
    kw = dict(max_atoms=b.n_atoms, max_mols=1, max_atoms_per_mol=b.n_atoms)
    h = NNP(hp, w0, M, "fp32", **kw)
    ref = NNP(hp, w1, M, "fp32", **kw)
    for hh in (h, ref):
        hh.set_knob("force_sum", 2)
    x, sp, off = to_device(torch, b, torch.float32)
    s = torch.cuda.Stream()
    out = (torch.empty(1, dtype=torch.float64, device="cuda"), torch.empty_like(x))
    p1 = torch.tensor(w1, dtype=torch.float64, device="cuda")
    with torch.cuda.stream(s):
        h.energy_forces(x, sp, off, out=out, graph=True, stream=s)    # eager + capture
        h.energy_forces(x, sp, off, out=out, graph=True, stream=s)    # replay
        h.set_params(p1, stream=s)                                     # stream-ordered
        h.energy_forces(x, sp, off, out=out, graph=True, stream=s)    # replay, new weights
    s.synchronize()
    Er, Fr = _eval(torch, ref, x, sp, off)
    assert np.array_equal(out[0].cpu().numpy(), Er)
    assert np.array_equal(out[1].double().cpu().numpy(), Fr)


@pytest.mark.parametrize("prec,force_sum", [("fp32", 1), ("fp32", 2), ("fp64", 1), ("bf16", 2)])
def test_accumulate_flag(hp, prec, force_sum):
    """NNP_FLAG_ACCUMULATE adds E and F onto what the outputs hold (eager and
    graph-replayed)."""
    torch = torch_cuda()
    b = _batch()
    M = 2
    w = synth.xavier_weights(M, hp["widths"], seed=77)
    h = make_handle(hp, w, M, prec, b)
    h.set_knob("force_sum", force_sum)
    dt = torch.float64 if prec == "fp64" else torch.float32
    x, sp, off = to_device(torch, b, dt)
    E, F = _eval(torch, h, x, sp, off)
    rng = np.random.default_rng(3)
    E0 = rng.normal(size=E.shape) * 100.0
    F0 = rng.normal(size=F.shape) * 10.0
    E0t = torch.tensor(E0, dtype=torch.float64, device="cuda")
    F0t = torch.tensor(F0, dtype=dt, device="cuda")
    out = (torch.empty_like(E0t), torch.empty_like(F0t))
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    for graph in (False, True, True, True):     # eager, eager + capture, replays
        with torch.cuda.stream(s):
            out[0].copy_(E0t)
            out[1].copy_(F0t)
            h.energy_forces(x, sp, off, out=out, accumulate=True, graph=graph, stream=s)
        s.synchronize()
        assert h.device_status() == 0
        Ea, Fa = out[0].cpu().numpy(), out[1].double().cpu().numpy()
        np.testing.assert_allclose(Ea, E0 + E, rtol=1e-15, atol=1e-12 * np.abs(E).max())
        # F0 as the output tensor stored it, plus the forces (whose last bits
        # move between evaluations with floating-point atomic sums)
        F0s = F0 if prec == "fp64" else F0.astype(np.float32).astype(np.float64)
        eps = 1e-13 if prec == "fp64" else 1e-6
        np.testing.assert_allclose(Fa, F0s + F, rtol=0, atol=4 * eps * (np.abs(F0).max() + np.abs(F).max()))


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp64"])
def test_fixed_point_forces_bitwise_reproducible(orc, hp, prec):
    """force_sum = 2: forces bitwise identical over repeated evaluations, over
    graph replays, and between two handles evaluated concurrently on two
    streams; within the parity bars of the oracle."""
    torch = torch_cuda()
    b = synth.random_batch(63, [48] * 40 + [130, 17])
    M = 4
    w = synth.xavier_weights(M, hp["widths"], seed=78)
    hs = [make_handle(hp, w, M, prec, b) for _ in range(2)]
    for h in hs:
        h.set_knob("force_sum", 2)
    dt = torch.float64 if prec == "fp64" else torch.float32
    x, sp, off = to_device(torch, b, dt)
    E, F = _eval(torch, hs[0], x, sp, off)
    for _ in range(3):
        E2, F2 = _eval(torch, hs[0], x, sp, off)
        assert np.array_equal(E2, E) and np.array_equal(F2, F)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = [(torch.empty(b.n_mols, dtype=torch.float64, device="cuda"), torch.empty_like(x)) for _ in hs]
    torch.cuda.synchronize()
    for _ in range(4):
        for h, s, o in zip(hs, streams, outs):
            with torch.cuda.stream(s):
                h.energy_forces(x, sp, off, out=o, graph=True, stream=s)
    torch.cuda.synchronize()
    for o in outs:
        assert np.array_equal(o[0].cpu().numpy(), E) and np.array_equal(o[1].double().cpu().numpy(), F)
    # accuracy: the same bars as the floating-point sums
    xo, wo = oracle_inputs(b, w, prec)
    Eo, Fo = orc.energy_forces(hp, wo, M, b.species, xo, b.mol_offsets)
    dE, rmse = errors(E, F, Eo, Fo, b.mol_offsets)
    print(prec, "fixed-point forces: max |dE|/atom", dE.max(), "max force RMSE", rmse.max())
    if prec == "fp64":
        assert np.abs(F - Fo).max() <= 1e-8 * np.abs(Fo).max()
    elif prec == "fp32":
        assert dE.max() <= 1e-4 and rmse.max() <= 1e-3
    else:
        assert rmse.max() <= 1e-2 * np.sqrt(np.mean(Fo ** 2))


def test_training_workspace_at_creation(hp):
    """NNP_CREATE_TRAINING: the first backward allocates no device memory
    (free memory unchanged), while a handle without it allocates its
    workspace then."""
    torch = torch_cuda()
    b = synth.config_batch(4, n_mols=16)
    M = 8
    w = synth.xavier_weights(M, hp["widths"])
    from paper_2201_08110_amd.nnp import NNP
    drops = {}
    for training in (True, False):
        h = NNP(hp, w, M, "fp32", max_atoms=b.n_atoms, max_mols=b.n_mols, max_atoms_per_mol=80,
                training=training)
        x, sp, off = to_device(torch, b, torch.float32)
        gE = torch.ones(b.n_mols, dtype=torch.float64, device="cuda")
        gF = torch.full_like(x, 1e-3)
        h.backward(x, sp, off, gE, gF)            # warm torch's allocator for the outputs
        torch.cuda.synchronize()
        del h
        torch.cuda.synchronize()
        h = NNP(hp, w, M, "fp32", max_atoms=b.n_atoms, max_mols=b.n_mols, max_atoms_per_mol=80,
                training=training)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        h.backward(x, sp, off, gE, gF)
        torch.cuda.synchronize()
        drops[training] = free0 - torch.cuda.mem_get_info()[0]
        h.close()
    print("free-memory drop on the first backward (bytes):", drops)
    assert drops[True] <= 2 << 20
    assert drops[False] >= 16 << 20


def test_autograd_two_parameter_sets_on_one_model(hp):
    """Two forwards with different parameter tensors on one model: each
    backward differentiates at its own forward's weights; an in-place change
    of the weights between forward and backward is refused by torch."""
    torch = torch_cuda()
    from paper_2201_08110_amd.autograd import nnp_energy_forces
    b = synth.random_batch(64, [8, 11])
    M = 2
    w1 = synth.xavier_weights(M, hp["widths"], seed=79)
    w2 = synth.xavier_weights(M, hp["widths"], seed=80)
    h = make_handle(hp, w1, M, "fp64", b)
    x, sp, off = to_device(torch, b, torch.float64)

    def grad_alone(w):
        p = torch.tensor(w, dtype=torch.float64, device="cuda", requires_grad=True)
        E, F = nnp_energy_forces(h, x, p, sp, off)
        (E.sum() + 0.1 * (F ** 2).sum()).backward()
        return p.grad.cpu().numpy()

    g1, g2 = grad_alone(w1), grad_alone(w2)
    p1 = torch.tensor(w1, dtype=torch.float64, device="cuda", requires_grad=True)
    p2 = torch.tensor(w2, dtype=torch.float64, device="cuda", requires_grad=True)
    E1, F1 = nnp_energy_forces(h, x, p1, sp, off)
    E2, F2 = nnp_energy_forces(h, x, p2, sp, off)       # the handle now holds w2
    (E1.sum() + 0.1 * (F1 ** 2).sum()).backward()        # must use w1
    (E2.sum() + 0.1 * (F2 ** 2).sum()).backward()
    # equal up to the last bits that the forces' atomic sums move (the loss
    # reads F); gradients at the other weights would differ at O(1)
    np.testing.assert_allclose(p1.grad.cpu().numpy(), g1, rtol=1e-9, atol=1e-12 * np.abs(g1).max())
    np.testing.assert_allclose(p2.grad.cpu().numpy(), g2, rtol=1e-9, atol=1e-12 * np.abs(g2).max())
    assert np.abs(g1 - g2).max() > 1e-3 * np.abs(g1).max()
    # in-place update between forward and backward
    p3 = torch.tensor(w1, dtype=torch.float64, device="cuda", requires_grad=True)
    E3, _ = nnp_energy_forces(h, x, p3, sp, off)
    with torch.no_grad():
        p3.add_(1e-3)
    with pytest.raises(RuntimeError):
        E3.sum().backward()
