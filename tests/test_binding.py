"""Host-side argument checks of the Python binding (no GPU needed).

The library writes the documented extent of every output buffer, so the
binding must refuse a buffer of the wrong dtype or shape before it calls into
libnep.  A context is assembled around a stand-in library that records calls;
every bad buffer must raise with no call made.
"""
import pytest
import torch

from paper_2107_08119_amd import nep


class _RecordingLib:
    def __init__(self):
        self.calls = []

    def __getattr__(self, name):
        def call(*args):
            self.calls.append(name)
            return 0
        return call


@pytest.fixture
def ctx():
    c = nep.Context.__new__(nep.Context)
    c._lib = _RecordingLib()
    c._h = None
    c.device = 0
    c.n, c.cap = 8, 16
    c.hyper = nep.hyper()
    yield c
    assert c._lib.calls == [], "the library was called despite a bad buffer"


def f32(*shape):
    return torch.zeros(shape, dtype=torch.float32)


def f64(*shape):
    return torch.zeros(shape, dtype=torch.float64)


class _Ds:
    n_struct, n_atoms, _h = 3, 8, None


def test_md_step_thermo_needs_a_row_per_step(ctx):
    with pytest.raises(ValueError, match="thermo"):
        ctx.md_step(20, 1.0, 10, 28.0, f64(3, 8), f64(3, 8), thermo=f64(19, 5))
    with pytest.raises(TypeError, match="thermo"):
        ctx.md_step(20, 1.0, 10, 28.0, f64(3, 8), f64(3, 8), thermo=f32(20, 5))


def test_md_step_per_atom_outputs(ctx):
    with pytest.raises(ValueError, match="W"):
        ctx.md_step(2, 1.0, 10, 28.0, f64(3, 8), f64(3, 8), thermo=f64(2, 5), W=f32(9, 7))
    with pytest.raises(ValueError, match="J"):
        ctx.md_step(2, 1.0, 10, 28.0, f64(3, 8), f64(3, 8), thermo=f64(2, 5), J=f32(8, 3))
    # right shapes on the host are still refused: the library needs device memory
    with pytest.raises(TypeError, match="CUDA"):
        ctx.md_step(2, 1.0, 10, 28.0, f64(3, 8), f64(3, 8), thermo=f64(2, 5))


def test_compute_outputs(ctx):
    with pytest.raises(ValueError, match="F"):
        ctx.compute(f64(3, 8), out={"F": f32(3, 7), "totals": f64(13)})
    with pytest.raises(ValueError, match="totals"):
        ctx.compute(f64(3, 8), out={"F": f32(3, 8), "totals": f64(12)})
    with pytest.raises(ValueError, match="J needs vel"):
        ctx.compute(f64(3, 8), out={"F": f32(3, 8), "J": f32(3, 8)})


def test_snes_buffers(ctx):
    n_par = nep.num_params(ctx.hyper)
    m, s = f32(n_par), f32(n_par)
    with pytest.raises(ValueError, match="r"):
        ctx.snes_sample(m, s, 1, 0, 4, r=f32(3, n_par), Z=f32(4, n_par))
    with pytest.raises(ValueError, match="Z"):
        ctx.snes_sample(m, s, 1, 0, 4, r=f32(4, n_par), Z=f32(4, n_par - 1))
    with pytest.raises(ValueError, match="s"):
        ctx.snes_update(m, f32(n_par - 1), f32(4, n_par), f64(4, 6))
    with pytest.raises(ValueError, match="loss"):
        ctx.snes_update(m, s, f32(4, n_par), f64(3, 6))
    with pytest.raises(ValueError, match="best"):
        ctx.snes_run(_Ds(), m, s, 1, 0, 5, f32(4, n_par), f32(4, n_par), f64(4, 6),
                     best=f64(4, 6))
    with pytest.raises(ValueError, match="Z"):
        ctx.eval_population(_Ds(), f32(4, n_par + 1))
    with pytest.raises(ValueError, match="out"):
        ctx.eval_population(_Ds(), f32(4, n_par), out=f64(5, 6))


def test_dataset_buffers(ctx):
    n_par = nep.num_params(ctx.hyper)
    with pytest.raises(ValueError, match="z"):
        ctx.dataset_compute(_Ds(), f32(n_par - 1))
    with pytest.raises(ValueError, match="F"):
        ctx.dataset_backward(_Ds(), f32(n_par), F=f32(3, 7), want_pos=True)
    with pytest.raises(ValueError, match="needs the forces"):
        ctx.dataset_backward(_Ds(), f32(n_par), want_pos=True)


def test_correlation_sample_buffers(ctx):
    corr = nep.Correlation.__new__(nep.Correlation)
    corr.ctx, corr._h, corr.n_atoms, corr.n_lags = ctx, None, 8, 4
    with pytest.raises(ValueError, match="W"):
        corr.sample(f32(9, 7), f64(3, 8))
    with pytest.raises(ValueError, match="vel"):
        corr.sample(f32(9, 8), f64(8, 3))
