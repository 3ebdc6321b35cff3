"""Pins of the seeded input generators and the Stillinger-Weber teacher."""
import math

import numpy as np
import pytest

from paper_2107_08119_amd import inputs as I


def test_accel_unit():
    # 1 eV/A on 1 amu = 9.6485e-3 A/fs^2, and 1 amu A^2/fs^2 = 103.6427 eV
    assert I.ACCEL_UNIT == pytest.approx(9.648533e-3, rel=1e-6)
    assert 1.0 / I.ACCEL_UNIT == pytest.approx(103.6427, rel=1e-6)


def test_diamond_lattice():
    pos, box = I.diamond_supercell(3, 3, 3)
    assert pos.shape == (216, 3)
    d = pos[:, None, :] - pos[None, :, :]
    d -= np.round(d / 16.29) * 16.29
    r = np.sqrt((d ** 2).sum(-1))
    r[r == 0] = np.inf
    assert r.min() == pytest.approx(5.43 * math.sqrt(3) / 4, rel=1e-12)


def test_maxwell_boltzmann_temperature():
    v = I.maxwell_boltzmann(1000, 300.0, 2)
    np.testing.assert_allclose(v.mean(0), 0.0, atol=1e-16)
    t = 2 * I.kinetic_energy(v) / ((3 * 1000 - 3) * I.BOLTZMANN_EV)
    assert t == pytest.approx(300.0, rel=1e-12)


def test_random_packing_min_distance_and_density():
    L = 20.0
    pos = I.random_packing(300, L, 2.0, seed=3, batch=512)
    d = pos[:, None, :] - pos[None, :, :]
    d -= L * np.round(d / L)
    r = np.sqrt((d ** 2).sum(-1)) + np.eye(len(pos)) * 1e9
    assert r.min() >= 2.0
    assert np.all((pos >= 0) & (pos < L))
    # deterministic given the seed
    np.testing.assert_array_equal(pos, I.random_packing(300, L, 2.0, seed=3, batch=512))


def test_training_structures_shapes():
    st = I.training_structures(20, 8, 64, seed=4)
    for s in st:
        assert 8 <= len(s.pos) <= 64
        frac = s.pos @ np.linalg.inv(s.box)
        assert np.all(frac >= 0) and np.all(frac < 1)


def test_sw_diamond_equilibrium():
    """SW dimer minimum at 2^(1/6) sigma with depth -epsilon gives diamond at
    a = 4 r0 / sqrt(3) = 5.43095 A with E = -2 epsilon per atom, zero forces and virial."""
    r0 = 2 ** (1 / 6) * I.SW_SIGMA
    a = 4 * r0 / math.sqrt(3)
    assert a == pytest.approx(5.43095, abs=1e-5)
    pos, box = I.diamond_supercell(2, 2, 2, a)
    e, f, w = I.stillinger_weber(pos, box)
    assert e / len(pos) == pytest.approx(-2 * I.SW_EPSILON, rel=1e-9)
    assert np.abs(f).max() < 1e-12
    assert np.abs(w).max() < 1e-6
    # bond-stretched lattice: compressive virial (negative: attractive restoring)
    e2, _, w2 = I.stillinger_weber(pos * 1.01, box * 1.01)
    assert e2 > e and np.all(np.diag(w2) < 0)


def test_sw_three_body_vanishes_at_tetrahedral_angle():
    """Isolated centre with four tetrahedral neighbours at 2.35 A; the leaves are
    3.84 A apart, beyond the 3.771 A cutoff, so only the four pair terms remain
    (the three-body factor (cos + 1/3)^2 is zero at the tetrahedral angle)."""
    r = 2.35
    tet = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]]) / math.sqrt(3) * r
    assert r * math.sqrt(8 / 3) > I.SW_CUT * I.SW_SIGMA
    pos = np.vstack([[0, 0, 0], tet]) + 15.0
    e, f, _ = I.stillinger_weber(pos, np.eye(3) * 30.0)
    sr = I.SW_SIGMA / r
    rc = I.SW_CUT * I.SW_SIGMA
    phi2 = I.SW_A * I.SW_EPSILON * (I.SW_B * sr ** 4 - 1) * math.exp(I.SW_SIGMA / (r - rc))
    assert e == pytest.approx(4 * phi2, rel=1e-12)
    np.testing.assert_allclose(f[0], 0.0, atol=1e-12)
    # bending one bond switches the three-body term on
    pos[1] += np.array([0.3, -0.2, 0.1])
    e_bent, _, _ = I.stillinger_weber(pos, np.eye(3) * 30.0)
    r1 = np.linalg.norm(pos[1] - pos[0])
    sr1 = I.SW_SIGMA / r1
    phi2_1 = I.SW_A * I.SW_EPSILON * (I.SW_B * sr1 ** 4 - 1) * math.exp(I.SW_SIGMA / (r1 - rc))
    assert e_bent > 3 * phi2 + phi2_1


def test_sw_forces_and_virial_finite_difference():
    rng = np.random.default_rng(0)
    pos, box = I.diamond_supercell(1, 1, 1)
    pos = pos + rng.standard_normal(pos.shape) * 0.1
    e, f, w = I.stillinger_weber(pos, box)
    h = 1e-5
    for i in range(len(pos)):
        for c in range(3):
            p = pos.copy()
            p[i, c] += h
            ep = I.stillinger_weber(p, box)[0]
            p[i, c] -= 2 * h
            em = I.stillinger_weber(p, box)[0]
            assert -(ep - em) / (2 * h) == pytest.approx(f[i, c], abs=1e-7)
    np.testing.assert_allclose(f.sum(0), 0.0, atol=1e-12)
    fd = np.zeros((3, 3))
    for a in range(3):
        for b in range(3):
            D = np.eye(3)
            D[a, b] += h
            ep = I.stillinger_weber(pos @ D, box @ D)[0]
            D[a, b] -= 2 * h
            em = I.stillinger_weber(pos @ D, box @ D)[0]
            fd[a, b] = -(ep - em) / (2 * h)
    np.testing.assert_allclose(w, fd.T, atol=1e-7)


def test_labelled_set_layout():
    ds = I.labelled_set(5, 8, 30, seed=1)
    assert ds.pos.shape == (ds.n_atoms.sum(), 3)
    assert ds.forces.shape == ds.pos.shape
    assert ds.virial.shape == (5, 6) and ds.boxes.shape == (5, 9)
    e = ds.energy / ds.n_atoms  # vacancies and strain raise it above -2 epsilon
    assert np.all(e > -2 * I.SW_EPSILON - 1e-9) and np.all(e < -1.0)
