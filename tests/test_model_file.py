"""The shipped SNES-trained silicon model: format, size and hyperparameters."""
import numpy as np

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


def test_model_round_trip(tmp_path):
    z = np.random.default_rng(0).standard_normal(931).astype(np.float32)
    path = tmp_path / "m.txt"
    T.save_model(str(path), z, {"note": "round trip"})
    z2, meta = T.load_model(str(path))
    np.testing.assert_array_equal(z, z2)
    assert meta == {"note": "round trip"}
