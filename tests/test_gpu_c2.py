"""The 512,000-atom disordered cube (2.33 g/cm^3, random packing with a
2.0 A minimum distance) under the SNES-trained silicon model: bit-exact
neighbour list, sampled per-atom parity, the heat current summed over a
4,096-atom cut, and 500 MD steps that write per-atom virials and heat currents
every step, with the cut's summed heat current checked against the oracle at
steps 100, 200, ..., 500 on the GPU's own positions and velocities.

The random packing relaxes violently under a physical model (the oracle's own
4,096-atom run of the same recipe heats to several thousand kelvin and moves
atoms up to 0.6 A in 10 fs), so the run uses a 1 A skin and rebuilds every 5
steps; the library's skin/2 displacement check (NEP_ESKIN from synchronize)
confirms after every chunk that the lists stayed complete."""
import numpy as np
import pytest

import oracle as O
from paper_2107_08119_amd import inputs as I
from paper_2107_08119_amd import train as T

pytestmark = pytest.mark.gpu

TOL = 1e-5
OH = O.hyper()
SKIN, REBUILD, CAP = 1.0, 5, 128


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


@pytest.fixture(scope="module")
def c2():
    pos, box = I.disordered_cell(512000, seed=3)
    vel = I.maxwell_boltzmann(len(pos), 300.0, seed=2)
    z, _ = T.load_model(T.MODEL_SI_SW)
    return pos, box, vel, z


@pytest.fixture(scope="module")
def c2_gpu(c2):
    from paper_2107_08119_amd import nep
    pos, box, vel, z = c2
    ctx = nep.Context(0)
    ctx.load_params(nep.hyper(), z)
    p, v = nep.soa(pos), nep.soa(vel)
    ctx.build_neighbors(p, box, skin=SKIN, max_neighbors=CAP)
    out = ctx.compute(p, v)
    ctx.synchronize()
    nb = ctx.get_neighbors()
    return ctx, p, v, out, nb


def cut_4096(pos, box):
    """The 4,096 atoms closest to the box centre in the max norm (ties by index)."""
    dev = np.abs(pos - 0.5 * np.diag(box)).max(axis=1)
    return np.lexsort((np.arange(len(pos)), dev))[:4096]


def test_c2_list_bit_exact(c2, c2_gpu):
    from tests.test_gpu_force import list_keys_gpu, list_keys_oracle
    pos, box, _, _ = c2
    _, _, _, _, nb = c2_gpu
    np.testing.assert_array_equal(list_keys_gpu(nb, "radial"),
                                  list_keys_oracle(pos, box, 5.0 + SKIN, cap=CAP))
    np.testing.assert_array_equal(list_keys_gpu(nb, "angular"),
                                  list_keys_oracle(pos, box, 4.0 + SKIN, cap=CAP))


def test_c2_sampled_atoms(c2, c2_gpu):
    from paper_2107_08119_amd import nep
    pos, box, vel, z = c2
    _, _, _, out, _ = c2_gpu
    sel = np.sort(np.random.default_rng(9).choice(len(pos), 400, replace=False))
    ref = O.nep_eval(OH, z, pos, box, vel=vel, sel=sel)
    assert rel(out["U"].cpu().numpy()[sel], ref["U"]) < TOL
    assert rel(nep.aos(out["F"])[sel], ref["F"]) < TOL
    assert rel(nep.aos(out["W"]).reshape(-1, 3, 3)[sel], ref["W"]) < TOL
    assert rel(nep.aos(out["J"])[sel], ref["J"]) < TOL


def test_c2_heat_current_on_cut(c2, c2_gpu):
    from paper_2107_08119_amd import nep
    pos, box, vel, z = c2
    _, _, _, out, _ = c2_gpu
    cut = cut_4096(pos, box)
    J = nep.aos(out["J"]).astype(np.float64)
    ref = O.nep_eval(OH, z, pos, box, vel=vel, sel=cut)
    assert rel(J[cut].sum(axis=0), ref["J"].sum(axis=0)) < TOL


def test_c2_heat_current_snapshots(c2, c2_gpu):
    """500 steps in chunks of 100 (dt 1 fs).  At the end of each chunk the
    per-atom W_i and J_i that the last step wrote belong to the positions and
    end-of-step velocities the call returns; the oracle evaluates those same
    float64 states and sums J_i = W_i . v_i (Sec. II B) over the cut."""
    import torch
    from paper_2107_08119_amd import nep
    _, box, _, z = c2
    ctx, p0, v0, _, _ = c2_gpu
    p, v = p0.clone(), v0.clone()
    n = p.shape[1]
    W = torch.zeros((9, n), dtype=torch.float32, device="cuda")
    J = torch.zeros((3, n), dtype=torch.float32, device="cuda")
    thermo = torch.empty((100, 5), dtype=torch.float64, device="cuda")
    for snap in range(1, 6):
        ctx.md_step(100, 1.0, REBUILD, I.MASS_SI, p, v, thermo, W, J)
        ctx.synchronize()  # raises on a latched overflow, image or skin violation
        th = thermo.cpu().numpy()
        assert np.all(np.isfinite(th)), snap
        pos, vel = nep.aos(p), nep.aos(v)
        cut = cut_4096(pos, box)
        ref = O.nep_eval(OH, z, pos, box, vel=vel, sel=cut)
        Jg = nep.aos(J).astype(np.float64)
        Wg = nep.aos(W).astype(np.float64).reshape(-1, 3, 3)
        assert rel(Jg[cut].sum(axis=0), ref["J"].sum(axis=0)) < TOL, (snap, "sum J")
        assert rel(Jg[cut], ref["J"]) < TOL, (snap, "J_i")
        assert rel(Wg[cut], ref["W"]) < TOL, (snap, "W_i")
        # the summed per-atom heat current of the last step equals its thermo row
        np.testing.assert_allclose(Jg.sum(axis=0), th[-1, 2:], rtol=1e-5,
                                   atol=1e-6 * np.abs(th[-1, 2:]).max())
