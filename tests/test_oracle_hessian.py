"""Pins of the FP64 Hessian-vector oracle (oracle/hessian.py), which serves
the coordinate gradient of force-dependent losses (F = -dE/dx, Methods, Eq. 3,
so dL/dx = -gE F - H gF):

* its energy and forces equal the C oracle's (itself pinned by closed forms
  and finite differences);
* H v equals central differences of the C oracle's forces along v;
* H is symmetric (u . H v = v . H u) and annihilates rigid translations;
* with a zero force cotangent the coordinate gradient is -gE F.
"""
import numpy as np
import pytest

from paper_2201_08110_amd import synth


def _mol(seed=3, n=11):
    b = synth.random_batch(seed, [n], box_scale=1.9)
    return b.species, b.coords


@pytest.fixture(scope="module")
def hes():
    pytest.importorskip("torch")
    from oracle import hessian
    return hessian


def test_energy_forces_match_c_oracle(orc, hp, hes):
    sp, x = _mol()
    w = synth.xavier_weights(2, hp["widths"], seed=61)
    E, F, _ = hes.energy_forces_hvp(hp, w, 2, sp, x, np.zeros_like(x))
    Eo, Fo = orc.energy_forces(hp, w, 2, sp, x)
    assert E == pytest.approx(Eo[0], rel=1e-12)
    np.testing.assert_allclose(F, Fo, rtol=1e-10, atol=1e-11 * np.abs(Fo).max())


@pytest.mark.parametrize("which", ["ani2x", "ani1x_elements"])
def test_hvp_matches_force_differences(orc, hp, hes, which):
    if which == "ani2x":
        h, ratio, w = hp, synth.LIGAND_RATIO, synth.xavier_weights(2, hp["widths"], seed=62)
    else:
        h, ratio = synth.ani1x_hparams(), (30, 20, 5, 5)
        w = synth.xavier_weights(2, h["species_widths"], n_species=4, seed=62)
    b = synth.random_batch(9, [10], box_scale=1.9, ratio=ratio)
    sp, x = b.species, b.coords
    v = np.random.default_rng(1).normal(size=x.shape)
    _, _, hv = hes.energy_forces_hvp(h, w, 2, sp, x, v)

    def dF(step):
        Fp = orc.energy_forces(h, w, 2, sp, x + step * v)[1]
        Fm = orc.energy_forces(h, w, 2, sp, x - step * v)[1]
        return (Fp - Fm) / (2 * step)

    # H v = -dF/dt.  CELU'' jumps at z = 0 (1/alpha below, 0 above), so H is
    # discontinuous where a pre-activation changes sign: the step must be
    # small enough that no unit's z crosses 0 (at 1e-4 A several of the ~12k
    # units do, and the difference is off by ~1e-3)
    fd = -dF(2e-6)
    np.testing.assert_allclose(hv, fd, rtol=0, atol=1e-7 * np.abs(fd).max())


def test_hessian_symmetric_and_translation_free(hp, hes):
    sp, x = _mol(4, 9)
    w = synth.xavier_weights(1, hp["widths"], seed=63)
    rng = np.random.default_rng(2)
    u, v = rng.normal(size=x.shape), rng.normal(size=x.shape)
    _, _, hu = hes.energy_forces_hvp(hp, w, 1, sp, x, u)
    _, _, hv = hes.energy_forces_hvp(hp, w, 1, sp, x, v)
    assert np.sum(u * hv) == pytest.approx(np.sum(v * hu), rel=1e-10)
    shift = np.tile(rng.normal(size=3), (len(sp), 1))
    _, _, hs = hes.energy_forces_hvp(hp, w, 1, sp, x, shift)
    assert np.abs(hs).max() < 1e-10 * np.abs(hv).max()


def test_coord_grad_energy_only_is_minus_gE_F(orc, hp, hes):
    b = synth.random_batch(5, [6, 8], box_scale=1.9)
    w = synth.xavier_weights(1, hp["widths"], seed=64)
    gE = np.array([0.7, -1.3])
    gx = hes.coord_grad(hp, w, 1, b.species, b.coords, b.mol_offsets, gE, np.zeros((b.n_atoms, 3)))
    _, F = orc.energy_forces(hp, w, 1, b.species, b.coords, b.mol_offsets)
    mol = np.repeat(np.arange(2), np.diff(b.mol_offsets))
    np.testing.assert_allclose(gx, -gE[mol][:, None] * F, rtol=1e-10, atol=1e-12)
