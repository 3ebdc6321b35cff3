"""nep_evaluate_static (list build and one evaluation in the library's static
workspace, no device allocation) against nep_build_neighbors + nep_compute on
the same inputs, through the C ABI: two calls in a row, the second with a
smaller system, then the context's own list is used again unchanged."""
import numpy as np
import pytest

from paper_2107_08119_amd import inputs as I

pytestmark = pytest.mark.gpu

KEYS = ("U", "F", "W", "J")


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def system(cells, jitter_seed):
    pos, box = I.diamond_supercell(cells, cells, cells)
    rng = np.random.default_rng(jitter_seed)
    pos = pos + rng.normal(0.0, 0.05, pos.shape)
    vel = I.maxwell_boltzmann(len(pos), 300.0, seed=2)
    return pos, box, vel


def reference(nep, z, pos, box, vel):
    """The existing entry points: nep_build_neighbors then nep_compute."""
    ctx = nep.Context(0)
    ctx.load_params(nep.hyper(), z)
    p, v = nep.soa(pos), nep.soa(vel)
    ctx.build_neighbors(p, box, skin=0.5, max_neighbors=64)
    out = ctx.compute(p, v)
    ctx.synchronize()
    return {k: t.cpu().numpy() for k, t in out.items()}


def outputs(torch, n):
    dev = torch.device("cuda", 0)
    return {"U": torch.full((n,), np.nan, dtype=torch.float32, device=dev),
            "F": torch.full((3, n), np.nan, dtype=torch.float32, device=dev),
            "W": torch.full((9, n), np.nan, dtype=torch.float32, device=dev),
            "J": torch.full((3, n), np.nan, dtype=torch.float32, device=dev),
            "totals": torch.full((13,), np.nan, dtype=torch.float64, device=dev)}


def check(got, ref, what):
    for k in KEYS:
        e = rel(got[k], ref[k])
        assert e < 1e-6, "%s %s rel err %.3e" % (what, k, e)
    et = rel(got["totals"], ref["totals"])
    assert et < 1e-6, "%s totals rel err %.3e" % (what, et)


def test_static_evaluation_matches_build_and_compute():
    import torch
    from paper_2107_08119_amd import nep
    z = I.random_parameters(931, seed=1)
    big = system(8, 11)    # 4,096 atoms, 43.4 A box: the cell-list builder
    small = system(3, 12)  # 216 atoms, 16.3 A box: the all-pairs builder
    ref_big = reference(nep, z, *big)
    ref_small = reference(nep, z, *small)

    ctx = nep.Context(0)
    ctx.load_params(nep.hyper(), z)
    # the context's own system (the small cell), evaluated before and after
    own_p, own_v = nep.soa(small[0]), nep.soa(small[2])
    ctx.build_neighbors(own_p, small[1], skin=0.5, max_neighbors=64)
    own_before = {k: t.cpu().numpy() for k, t in ctx.compute(own_p, own_v).items()}

    for what, (pos, box, vel), ref in (("first call, 4096 atoms", big, ref_big),
                                       ("second call, 216 atoms", small, ref_small)):
        print(what, flush=True)
        n = len(pos)
        out = outputs(torch, n)
        ctx.evaluate_static(nep.soa(pos), box, out, vel=nep.soa(vel), skin=0.5, max_neighbors=64)
        ctx.synchronize()
        check({k: t.cpu().numpy() for k, t in out.items()}, ref, what)

    own_after = {k: t.cpu().numpy() for k, t in ctx.compute(own_p, own_v).items()}
    ctx.synchronize()
    for k in own_before:
        np.testing.assert_array_equal(own_after[k], own_before[k], err_msg=k)


def test_static_evaluation_rejects_a_system_beyond_the_workspace():
    import torch
    from paper_2107_08119_amd import nep
    ctx = nep.Context(0)
    ctx.load_params(nep.hyper(), I.random_parameters(931, seed=1))
    assert nep.lib().nep_static_workspace_bytes() == 32 << 20
    pos, box = I.diamond_supercell(20, 20, 20)  # 64,000 atoms
    n = len(pos)
    out = {"F": torch.empty((3, n), dtype=torch.float32, device="cuda")}
    with pytest.raises(nep.NepError) as e:
        ctx.evaluate_static(nep.soa(pos), box, out, skin=0.5, max_neighbors=64)
    assert e.value.status == nep.NEP_EINVAL
    assert "workspace" in str(e.value)
