"""Train a NEP by separable natural evolution (SNES) on the GPU.

The training set is the one the library's SNES path is built for: strained,
jittered diamond-silicon cells of 8-256 atoms labelled in float64 by the
Stillinger-Weber teacher (inputs.labelled_set).  Every generation samples a
population around the mean m with per-parameter scale s, evaluates the loss
of every individual over the whole set in one batched call
(snes_eval_population: energy, force and virial RMSE plus L1/L2 terms,
Sec. II E), and moves m and s by the rank-based natural-gradient update
(Sec. II E).  The generations run on the device (snes_run: one captured
graph per generation, replayed), with the population kernels' tile shape
picked by snes_autotune.  The result is the final mean m.

The teacher stays the judge of the error: `evaluate` reports the RMSE of the
trained model against Stillinger-Weber labels on a held-out set.

Usage:
    python -m paper_2107_08119_amd.train --generations 20000 --out model.txt
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
MODEL_SI_SW = os.path.join(HERE, "data", "nep_si_sw.txt")


def train(ctx, n_struct=1000, n_min=8, n_max=256, data_seed=4, snes_seed=5, n_pop=50,
          generations=20000, lam=(1.0, 1.0, 1.0, 0.05, 0.05), log_every=1000, log=None):
    """SNES from m ~ U(-1/2, 1/2), s = 0.1; returns (m as float32 numpy, history)."""
    import torch

    from . import inputs as I
    from . import nep

    h = nep.hyper()
    n_par = nep.num_params(h)
    ls = I.labelled_set(n_struct, n_min, n_max, seed=data_seed)
    ds = ctx.dataset_create(ls, max_neighbors=64)
    rng = np.random.default_rng(snes_seed)
    dev = torch.device("cuda", ctx.device)
    m = torch.from_numpy(rng.uniform(-0.5, 0.5, n_par).astype(np.float32)).to(dev)
    s = torch.full((n_par,), 0.1, dtype=torch.float32, device=dev)
    r = torch.empty((n_pop, n_par), dtype=torch.float32, device=dev)
    Z = torch.empty_like(r)
    loss = torch.empty((n_pop, 6), dtype=torch.float64, device=dev)
    # tile shape for this dataset, timed on the first generation's population
    ctx.snes_sample(m, s, snes_seed, 0, n_pop, r, Z)
    atoms, _ = ctx.snes_autotune(ds, Z, reps=3)
    history = []
    t0 = time.perf_counter()
    g = 0
    while g < generations:
        n = min(log_every, generations - g)
        best = ctx.snes_run(ds, m, s, snes_seed, g, n, r, Z, loss, lam)
        g += n
        b = best[n - 1].cpu().numpy()
        rec = {"generation": g, "seconds": time.perf_counter() - t0, "atoms_per_wave": atoms,
               "loss": float(b[0]), "rmse_e": float(b[1]), "rmse_f": float(b[2]),
               "rmse_v": float(b[3])}
        history.append(rec)
        if log:
            log(rec)
    ctx.synchronize()
    return m.cpu().numpy().astype(np.float32), history


def evaluate(ctx, z, n_struct=200, n_min=8, n_max=256, seed=7):
    """RMSE of model z against Stillinger-Weber labels on a held-out set:
    energy and virial per atom (meV/atom), force components (meV/A)."""
    import torch

    from . import inputs as I

    ls = I.labelled_set(n_struct, n_min, n_max, seed=seed)
    ds = ctx.dataset_create(ls, max_neighbors=64)
    zt = torch.from_numpy(np.asarray(z, np.float32)).cuda(ctx.device)
    out = ctx.dataset_compute(ds, zt, virial=True)
    n = ls.n_atoms.astype(np.float64)
    e = out["E"].cpu().numpy()
    f = out["F"].cpu().numpy().T
    w = out["W"].cpu().numpy()  # [S, 9] row-major
    w6 = w[:, [0, 4, 8, 1, 5, 6]]  # xx yy zz xy yz zx
    rmse_e = np.sqrt(np.mean(((e - ls.energy) / n) ** 2))
    rmse_f = np.sqrt(np.mean((f - ls.forces) ** 2))
    rmse_v = np.sqrt(np.mean(((w6 - ls.virial) / n[:, None]) ** 2))
    return {"structures": n_struct, "seed": seed, "rmse_energy_meV_per_atom": 1e3 * rmse_e,
            "rmse_force_meV_per_A": 1e3 * rmse_f, "rmse_virial_meV_per_atom": 1e3 * rmse_v,
            "force_rms_meV_per_A": 1e3 * float(np.sqrt(np.mean(ls.forces ** 2)))}


def save_model(path, z, meta):
    """Text model: one JSON header line, then the parameters, one per line."""
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    with open(path, "w") as fh:
        fh.write("# " + json.dumps(meta, sort_keys=True) + "\n")
        for v in np.asarray(z, np.float32):
            fh.write("%.9g\n" % v)


def load_model(path=MODEL_SI_SW):
    """(z as float32 numpy, header dict) of a text model written by save_model."""
    with open(path) as fh:
        head = fh.readline()
        if not head.startswith("# "):
            raise ValueError("%s: not a model file" % path)
        meta = json.loads(head[2:])
        z = np.array([float(x) for x in fh if x.strip()], dtype=np.float32)
    return z, meta


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--generations", type=int, default=20000)
    ap.add_argument("--structures", type=int, default=1000)
    ap.add_argument("--out", default=MODEL_SI_SW)
    ap.add_argument("--log-every", type=int, default=1000)
    args = ap.parse_args(argv)
    from . import nep

    ctx = nep.Context(0)
    ctx.load_params(nep.hyper(), np.zeros(nep.num_params(nep.hyper()), np.float32))
    z, hist = train(ctx, n_struct=args.structures, generations=args.generations,
                    log_every=args.log_every, log=lambda r: print(json.dumps(r), flush=True))
    ctx.load_params(nep.hyper(), z)
    test = evaluate(ctx, z)
    print(json.dumps({"held_out": test}), flush=True)
    h = nep.hyper()
    meta = {"model": "NEP 29-30-1 Si, trained by SNES on Stillinger-Weber labels",
            "rc_radial": h.rc_radial, "rc_angular": h.rc_angular,
            "n_max_radial": h.n_max_radial, "n_max_angular": h.n_max_angular,
            "l_max": h.l_max, "n_neuron": h.n_neuron, "generations": args.generations,
            "train_structures": args.structures, "data_seed": 4, "snes_seed": 5,
            "population": 50, "final": hist[-1], "held_out": test}
    save_model(args.out, z, meta)
    print("wrote", args.out, flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
