"""The shipped SNES-trained silicon model: format, size and hyperparameters, and its
error against the Stillinger-Weber teacher recomputed by the oracle."""
import numpy as np
import pytest

import oracle as O
from paper_2107_08119_amd import inputs as I
from paper_2107_08119_amd import train as T


def test_trained_model_file():
    z, meta = T.load_model(T.MODEL_SI_SW)
    # Eq. N_par for N_des = 9 + 5 * 4 and 30 hidden neurons
    assert z.dtype == np.float32 and z.shape == ((9 + 5 * 4 + 2) * 30 + 1,)
    assert np.isfinite(z).all()
    assert (meta["n_max_radial"], meta["n_max_angular"], meta["l_max"], meta["n_neuron"]) == (8, 4, 4, 30)
    assert (meta["rc_radial"], meta["rc_angular"]) == (5.0, 4.0)
    # the teacher judged the model on held-out structures
    assert meta["held_out"]["rmse_force_meV_per_A"] < 0.1 * meta["held_out"]["force_rms_meV_per_A"]


def test_teacher_judges_the_trained_model():
    """The float64 oracle recomputes the model's energy, force and virial RMSE (Sec. II E
    loss terms) against Stillinger-Weber labels of the 200 held-out structures (seed 7,
    never used in training), and the result must match what the training run recorded
    and stay far below the spread of the labels."""
    z, meta = T.load_model(T.MODEL_SI_SW)
    held = meta["held_out"]
    ls = I.labelled_set(held["structures"], 8, 256, seed=held["seed"])
    _, le, lf, lv, _, _ = O.loss(O.hyper(), z, ls)
    assert 1e3 * le == pytest.approx(held["rmse_energy_meV_per_atom"], rel=1e-3)
    assert 1e3 * lf == pytest.approx(held["rmse_force_meV_per_A"], rel=1e-3)
    assert 1e3 * lv == pytest.approx(held["rmse_virial_meV_per_atom"], rel=1e-3)
    force_rms = float(np.sqrt(np.mean(ls.forces ** 2)))
    assert lf < 0.05 * force_rms
    # a model that predicts no force at all has an RMSE equal to the label RMS
    assert O.loss(O.hyper(), np.zeros_like(z), ls)[2] == pytest.approx(force_rms, rel=1e-12)


def test_model_round_trip(tmp_path):
    z = np.random.default_rng(0).standard_normal(931).astype(np.float32)
    path = tmp_path / "m.txt"
    T.save_model(str(path), z, {"note": "round trip"})
    z2, meta = T.load_model(str(path))
    np.testing.assert_array_equal(z, z2)
    assert meta == {"note": "round trip"}
