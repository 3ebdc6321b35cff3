"""Throughput of the NEP molecular-dynamics hot path on one MI355X.

One step = one velocity-Verlet NVE step of the whole path: half-kick and
drift, neighbour-list rebuild every 10 steps (amortised), descriptor, network
and partial forces (pass 1), scatter-free gather of forces, per-atom virials
and heat currents with the second half-kick and thermo sums (pass 2).

Workload: 64,000-atom silicon diamond (20x20x20 conventional cells,
a = 5.43 A), Maxwell-Boltzmann velocities at 300 K, dt = 1 fs, skin 0.5 A,
NEP 29-30-1 (r_c 5/4 A, Chebyshev 0-8 / 0-4, Legendre 1-4), float32
arithmetic with float64 positions, velocities and totals.  The paper's speed
test (Sec. III D: bulk Si, 8000 atoms, 100 NVT steps) is the analogue.

Prints ONE JSON line with the metric (K uninstrumented steps), a roofline for
the dominant kernel (HIP events on the library's stream around back-to-back
launches at the state the timed region ended in) and the FP64 CPU oracle timed
on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "atom-steps/s (NEP MD, 64k–512k atoms) + SNES gen/s, vs plain path at 1e-5 rel err"
PEAK_FP32_TFLOPS = 157.3  # MI355X published dense FP32 vector peak
# Without packed float32 (disabled in every kernel here): 256 CUs x 4 SIMDs x
# 16 lanes x 2 flops (FMA) x 2.4 GHz
PEAK_FP32_NONPACKED_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
PEAK_HBM_GBS = 8000.0

# Algorithmic float32 work of the descriptor/network/partial-force kernel,
# counted from its arithmetic (a fused multiply-add counts 2, a square root,
# reciprocal or exponential 1):
#   every list slot (geometry in both loops)                   29
#   every pair inside r_c^R (f_c T_n sums, partial force from
#                            T_n, T_n' sums)                   181
#   every pair inside r_c^A (basis, harmonics, moments,
#                            partial force from T_n, T_n' sums)  1177
#   every atom (angular invariants, 30-neuron network with
#               derivative, moment scaling, n = 0 folds)      4390
FLOP_SLOT, FLOP_RADIAL, FLOP_ANGULAR, FLOP_ATOM = 29, 181, 1177, 4390
# Algorithmic HBM bytes of the same kernel per atom: own position 24, counts 8,
# list 4 per slot, partial force written 12 per slot, pair vector written 12
# per slot (for pass 2), site energy 4.
BYTE_ATOM, BYTE_SLOT = 36, 28
# Measured HBM traffic of one k_partials launch of this workload: rocprofv3
# --pmc FETCH_SIZE and --pmc WRITE_SIZE runs of this bench (KiB per dispatch;
# profiles/k_partials_nve64k_counters.md), each scaled by what the counter
# reads for a plain device copy of known size (--copy-probe-mib: FETCH_SIZE
# reports half the bytes read, WRITE_SIZE all bytes written), one entry per
# tile shape (lanes per atom: FETCH_SIZE, WRITE_SIZE).  They hold only for the
# kernel sources they were taken with (hash below); otherwise, or for a tile
# without an entry, the bench reports traffic null.
COUNTERS = {"sources_sha256": "bb68c64c1c1252629b018d61938ea9669370a28693b87a7445000bca64b64e45",
            "kib": {
                    "2": [12099.1, 81810.2],
                    "4": [10776.8, 76409.1],
                    "8": [10932.5, 76255.0]}}
FETCH_SCALE, WRITE_SCALE = 2.0, 1.0
KERNEL_SOURCES = ["force.hip", "nep_terms.h", "nep_device.h", "nep_internal.h"]


def kernel_sources_hash():
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2107_08119_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(lanes):
    """HBM bytes per k_partials launch of the chosen tile shape (lanes per atom)
    from the recorded counters, or None."""
    if COUNTERS["sources_sha256"] is None or COUNTERS["sources_sha256"] != kernel_sources_hash():
        return None
    kib = COUNTERS["kib"].get(str(lanes))
    if kib is None:
        return None
    return 1024.0 * (FETCH_SCALE * kib[0] + WRITE_SCALE * kib[1])


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--cells", type=int, default=20, help="diamond cells per edge")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target CPU time of the oracle sample")
    ap.add_argument("--no-snes", action="store_true", help="skip the SNES generation rate")
    ap.add_argument("--md-only", action="store_true",
                    help="run only the 64,000-atom MD line (no HNEMD, Table I models, "
                         "autograd, PbTe, 512k or SNES entries; profiling)")
    ap.add_argument("--snes-only", action="store_true",
                    help="run only the SNES generation rate and print its entry (profiling)")
    ap.add_argument("--no-disordered", action="store_true",
                    help="skip the 512,000-atom disordered heat-current run")
    ap.add_argument("--disordered-steps", type=int, default=500)
    ap.add_argument("--snes-structures", type=int, default=1000)
    ap.add_argument("--snes-generations", type=int, default=200)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="finish with 5 plain device copies of this many MiB (a known-size "
                         "kernel that scales the HBM byte counters of a profiler run)")
    return ap.parse_args()


def disordered_rate(args, nep, I, torch, z):
    """512,000-atom random Si cube at 2.33 g/cm^3: NVE steps that write the
    per-atom virial and heat current every step.  The random packing relaxes
    violently (atoms move up to about 0.6 A in 10 fs under the trained model),
    so the lists use a 1 A skin and are rebuilt every 5 steps; synchronize
    raises if any step saw an atom farther than skin/2 from its list-build
    position."""
    pos, box = I.disordered_cell(512000, seed=3)
    vel = I.maxwell_boltzmann(len(pos), 300.0, seed=2)
    skin, rebuild, cap = 1.0, 5, 128
    ctx = nep.Context(0)
    ctx.load_params(nep.hyper(), z)
    p, v = nep.soa(pos), nep.soa(vel)
    ctx.build_neighbors(p, box, skin=skin, max_neighbors=cap)
    n = len(pos)
    W = torch.empty((9, n), dtype=torch.float32, device="cuda")
    J = torch.empty((3, n), dtype=torch.float32, device="cuda")
    K = args.disordered_steps
    thermo = torch.empty((max(K, 20), 5), dtype=torch.float64, device="cuda")
    ctx.md_step(20, 1.0, rebuild, I.MASS_SI, p, v, thermo, W, J)
    lanes, _ = ctx.autotune(p, reps=5)
    ctx.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.md_step(K, 1.0, rebuild, I.MASS_SI, p, v, thermo, W, J)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    ctx.synchronize()
    ms = nep.time_partials(ctx, p, reps=50)
    h = nep.hyper()
    mean_slots = float(ctx.get_neighbors()["cnt_radial"].double().mean())
    pos_end = nep.aos(p)
    nr = pair_counts(pos_end, box, h.rc_radial)
    na = pair_counts(pos_end, box, h.rc_angular)
    flop_atom = FLOP_SLOT * mean_slots + FLOP_RADIAL * nr + FLOP_ANGULAR * na + FLOP_ATOM
    achieved = flop_atom * n / (ms / 1e3) / 1e12
    return {"workload": "NVE MD of a 512,000-atom random Si cube (2.33 g/cm^3, 2.0 A minimum "
                        "distance), per-atom W and J written every step, dt 1 fs, rebuild every "
                        "%d steps, skin %.1f A" % (rebuild, skin),
            "atom_steps_per_s": n * K / t, "ms_per_step": t / K * 1e3,
            "steps": K, "k_partials_us": ms * 1e3, "tile_lanes_per_atom": lanes,
            "roofline": {"kernel": "k_partials", "bound": "alu", "achieved": achieved,
                         "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                         "frac": achieved / PEAK_FP32_TFLOPS,
                         "frac_nonpacked": achieved / PEAK_FP32_NONPACKED_TFLOPS,
                         "flop_per_atom": flop_atom,
                         "neighbours_radial": nr, "neighbours_angular": na,
                         "list_slots": mean_slots,
                         "algorithmic_GBps": (BYTE_ATOM + BYTE_SLOT * mean_slots) * n
                         / (ms / 1e3) / 1e9}}


def spectral_rate(ctx, nep, torch, p, v, n, box, dt, rebuild, mass, fe, n_lags=250,
                  every=2, samples=300):
    """HNEMD with the virial-velocity correlation (Sec. II B): per-atom W_i and
    v_i sampled every `every` steps into a ring of n_lags samples, then the
    spectral conductivity and its quantum correction.  Reports the MD rate
    with sampling, the sampling kernels' time at a full ring and their HBM
    rate (n_lags x 36 B of virials read per atom and sample)."""
    W = torch.empty((9, n), dtype=torch.float32, device="cuda")
    corr = nep.Correlation(ctx, n, n_lags)
    ctx.md_step(every, dt, rebuild, mass, p, v, W=W, fe=fe)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(samples):
        ctx.md_step(every, dt, rebuild, mass, p, v, W=W, fe=fe)
        corr.sample(W, v)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    # the sampling kernels alone, ring full (n_lags lags per sample)
    reps = 20
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(reps):
        corr.sample(W, v)
    torch.cuda.synchronize()
    t_s = (time.perf_counter() - t1) / reps
    K, n_s = corr.get()
    volume = float(abs(np.linalg.det(box)))
    nu = np.linspace(0.0, 25.0, 251)
    kap, kq = corr.spectrum(every * dt, 300.0, volume, fe[0], nu)
    kx = float(np.trapezoid(kap[0], nu))
    kqx = float(np.trapezoid(kq[0], nu))
    corr.close()
    bytes_sample = n_lags * 36.0 * n + 24.0 * n + 72.0 * n  # ring reads, v, W copy in and out
    return {"workload": "HNEMD of the 64,000-atom diamond (F_e = 1e-4 1/A along x) with W_i and "
                        "v_i sampled every %d steps into a %d-sample correlation ring, %d samples; "
                        "spectrum 0-25 THz with the quantum correction" % (every, n_lags, samples),
            "atom_steps_per_s": n * every * samples / t,
            "us_per_sample_full_ring": t_s * 1e6,
            "sample_GBps": bytes_sample / t_s / 1e9,
            "sample_hbm_frac": bytes_sample / t_s / 8.0e12,
            "samples": n_s,
            "kappa_xx_W_per_mK_0_25THz": kx, "kappa_q_xx_W_per_mK_0_25THz": kqx,
            "note": "kappa from %d fs of correlation: a throughput run, not a converged "
                    "conductivity" % int(n_lags * every * dt)}


def paper_model_rate(nep, I, torch, steps=100):
    """The paper's speed test (Sec. III D) in kind, for the three models of
    Table I: 100 MD steps (NVE here) of bulk Si (8000 atoms, 80-50-1:
    r_c 5/5 A, n_max 15/15, 50 neurons), 2D silicene (6000 atoms, 65-40-1:
    r_c 5.5/5.5 A, n_max 12/12, 40 neurons) and bulk PbTe (8000 atoms,
    41-40-1: r_c 8/4 A, n_max 12/6, 40 neurons, sqrt(Z_i Z_j) weights and
    per-atom masses); l_max 4 throughout, random parameters (the work does
    not depend on their values)."""
    cases = []
    pos, box = I.diamond_supercell(10, 10, 10)
    cases.append(("si_80_50_1_8000", nep.hyper(5.0, 5.0, 15, 15, 4, 50), pos, box, None,
                  I.MASS_SI, 0.02))
    pos, box = I.silicene_sheet(50, 30)
    cases.append(("silicene_65_40_1_6000", nep.hyper(5.5, 5.5, 12, 12, 4, 40), pos, box, None,
                  I.MASS_SI, 0.02))
    pos, box, Z, masses = I.rocksalt_supercell(10, 10, 10)
    cases.append(("pbte_41_40_1_8000", nep.hyper(8.0, 4.0, 12, 6, 4, 40), pos, box, (Z, masses),
                  150.0, 0.05))
    out = {"workload": "the paper's speed test in kind: %d NVE steps, dt 1 fs, rebuild every 10 "
                       "steps, for the three models of Table I (one-wave-per-atom kernel with "
                       "each model's sizes compiled in)" % steps,
           "paper_v100_atom_steps_per_s": ">1e7 for each (context: another GPU)"}
    for name, h, pos, box, species, mass, std in cases:
        z = I.random_parameters(nep.num_params(h), seed=1, std=std)
        if species is not None:
            z[:h.n_neuron * nep.num_descriptors(h)] *= np.float32(1.0 / 300.0)
        vel = I.maxwell_boltzmann(len(pos), 300.0, seed=2,
                                  mass=mass if species is None else species[1])
        ctx = nep.Context(0)
        ctx.load_params(h, z)
        p, v = nep.soa(pos), nep.soa(vel)
        ctx.build_neighbors(p, box, skin=0.5, max_neighbors=128)
        if species is not None:
            ctx.set_species(species[0], species[1])
        ctx.md_step(10, 1.0, 10, mass, p, v)
        ctx.synchronize()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.md_step(steps, 1.0, 10, mass, p, v)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        ctx.synchronize()
        ms = nep.time_partials(ctx, p, reps=50)
        rate = len(pos) * steps / t
        out[name] = {"atoms": len(pos), "atom_steps_per_s": rate, "ms_per_step": t / steps * 1e3,
                     "k_partials_us": ms * 1e3, "ratio_to_1e7": rate / 1e7}
    return out


def pbte_rate(nep, I, torch, steps=100):
    """A two-species system (Sec. II C, multicomponent weighting sqrt(Z_i Z_j)):
    64,000-atom rock-salt PbTe with the PbTe-like model sizes of Table I
    (r_c 8/4 A, n_max 12/6, l_max 4, 40 neurons: 41-40-1, 1721 parameters),
    random parameters N(0, 0.05^2), per-atom masses; NVE, dt 1 fs, rebuild every
    10 steps.  Multicomponent systems take the float64-descriptor kernel."""
    h = nep.hyper(8.0, 4.0, 12, 6, 4, 40)
    z = I.random_parameters(nep.num_params(h), seed=1, std=0.05)
    pos, box, Z, masses = I.rocksalt_supercell(20, 20, 20)
    vel = I.maxwell_boltzmann(len(pos), 300.0, seed=2, mass=masses)
    ctx = nep.Context(0)
    ctx.load_params(h, z)
    p, v = nep.soa(pos), nep.soa(vel)
    ctx.build_neighbors(p, box, skin=0.5, max_neighbors=128)
    ctx.set_species(Z, masses)
    ctx.md_step(10, 1.0, 10, 150.0, p, v)
    ctx.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.md_step(steps, 1.0, 10, 150.0, p, v)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    ctx.synchronize()
    ms = nep.time_partials(ctx, p, reps=20)
    nb = ctx.get_neighbors()
    return {"workload": "64,000-atom rock-salt PbTe (20x20x20 cells), NEP 41-40-1 (r_c 8/4 A, "
                        "n_max 12/6, l_max 4, 40 neurons), pair weights sqrt(Z_i Z_j), per-atom "
                        "masses, %d NVE steps, dt 1 fs, rebuild every 10 steps" % steps,
            "atom_steps_per_s": len(pos) * steps / t, "ms_per_step": t / steps * 1e3,
            "k_partials_us": ms * 1e3,
            "list_slots": float(nb["cnt_radial"].double().mean())}


def snes_rate(args, ctx, nep, I, torch):
    """SNES generations/s on 1000 SW-labelled Si structures of 8-256 atoms,
    population 50, and the plain per-structure GPU path as the yardstick."""
    h = nep.hyper()
    n_par = nep.num_params(h)
    ls = I.labelled_set(args.snes_structures, 8, 256, seed=4)
    ds = ctx.dataset_create(ls, max_neighbors=64)
    n_pop, seed, lam = 50, 5, (1.0, 1.0, 1.0, 0.05, 0.05)
    rng = np.random.default_rng(seed)
    m = torch.from_numpy(rng.uniform(-0.5, 0.5, n_par).astype(np.float32)).cuda()
    s = torch.full((n_par,), 0.1, dtype=torch.float32, device="cuda")
    r = torch.empty((n_pop, n_par), dtype=torch.float32, device="cuda")
    Z = torch.empty_like(r)
    loss = torch.empty((n_pop, 6), dtype=torch.float64, device="cuda")

    # tile shape of the population kernels for this dataset (autotuner), then
    # generations on the device: one captured graph per generation, replayed
    ctx.snes_sample(m, s, seed, 0, n_pop, r, Z)
    lanes, tile_ms = ctx.snes_autotune(ds, Z, reps=3)
    ctx.snes_run(ds, m, s, seed, 0, 2, r, Z, loss, lam)
    ctx.synchronize()
    G = args.snes_generations
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.snes_run(ds, m, s, seed, 2, G, r, Z, loss, lam)
    torch.cuda.synchronize()
    t_gen = (time.perf_counter() - t0) / G
    ctx.synchronize()
    best = float(loss[:, 0].min())
    # algorithmic flops of one generation (population pass only; sampling,
    # sort and update are O(n_pop N_par)):
    #   network, per (individual, atom): the hidden layer and dU/dq, two
    #     N_neu x N_des products, plus output and sech^2 terms: 4 N_neu N_des + 4 N_neu;
    #   contraction, per (individual, pair): p_ij from the radial rows,
    #     2 * 3 (n_R + 1), and for angular pairs from the angular rows,
    #     2 * 3 (n_A + 1) l_max; then F_i += p_ij, F_j -= p_ij (6) and the
    #     structure virial r_ij (x) p_ij (18)
    n_r, n_a = ds.pairs()
    n_des, n_neu = nep.num_descriptors(h), h.n_neuron
    nr1, na1 = h.n_max_radial + 1, h.n_max_angular + 1
    f_net = n_pop * ds.n_atoms * (4 * n_neu * n_des + 4 * n_neu)
    f_con = n_pop * (n_r * (6 * nr1 + 24) + n_a * 6 * na1 * h.l_max)
    peak = 157.3e12  # MI355X dense FP32 matrix-core peak
    achieved = (f_net + f_con) / t_gen
    # plain path: per individual, per structure nep_build_neighbors + nep_compute,
    # loss assembled on the host; timed on two individuals, scaled to the population
    Zh = Z.cpu().numpy()
    off = np.concatenate([[0], np.cumsum(ls.n_atoms)])
    pos_dev = [nep.soa(ls.pos[off[k]:off[k + 1]]) for k in range(len(ls.n_atoms))]
    boxes = [ls.boxes[k].reshape(3, 3) for k in range(len(ls.n_atoms))]
    pctx = nep.Context(0)
    n_plain = 2
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(n_plain):
        pctx.load_params(h, Zh[k])
        e = []
        for st in range(len(ls.n_atoms)):
            pctx.build_neighbors(pos_dev[st], boxes[st], skin=0.0, max_neighbors=64)
            out = pctx.compute(pos_dev[st], W=True, U=False)
            e.append((out["totals"], out["F"]))
        [(t.cpu(), f.cpu()) for t, f in e]
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) / n_plain * n_pop
    return {
        "workload": "SNES, population %d x %d SW-labelled Si structures (8-256 atoms, "
                    "%d atoms), NEP 29-30-1, loss E+F+V+L1+L2" % (n_pop, len(ls.n_atoms),
                                                                 int(ls.n_atoms.sum())),
        "gen_per_s": 1.0 / t_gen,
        "ms_per_gen": t_gen * 1e3,
        "generations": G,
        "tile_atoms_per_wave": lanes,
        "tile_ms_per_eval": {"16": tile_ms[0], "32": tile_ms[1], "64": tile_ms[2]},
        "launch": "snes_run: sample, population loss and update of a generation captured as "
                  "one HIP graph, replayed per generation",
        "best_loss_last_gen": best,
        "plain_per_structure_gen_per_s": 1.0 / t_plain,
        "plain_path": "host loop of nep_build_neighbors + nep_compute per (structure, "
                      "individual), timed on %d individuals and scaled to %d" % (n_plain, n_pop),
        "speedup_vs_plain": t_plain / t_gen,
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": peak / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / peak,
                     "gflop_per_gen": (f_net + f_con) / 1e9,
                     "gflop_network": f_net / 1e9, "gflop_contraction": f_con / 1e9,
                     "pairs_radial": n_r, "pairs_angular": n_a,
                     "note": "algorithmic FP32 flops of the population pass per generation "
                             "over the generation's wall time"},
    }


def autograd_rate(nep, I, torch, z, reps=20, n_plain=32):
    """The differentiable form: 256 SW-labelled Si structures of 64-512 atoms,
    one call = NEPEnergy forward (E, F; dE/dr = -F) and the hand-written
    backward of an energy + force loss to dL/dz; against the same objective
    per structure from a host loop (one single-structure dataset each)."""
    ls = I.labelled_set(256, 64, 512, seed=6)
    ctx = nep.Context(0)
    ctx.load_params(nep.hyper(), z)
    ds = ctx.dataset_create(ls, max_neighbors=96)
    zt = torch.from_numpy(np.asarray(z, np.float32)).cuda().requires_grad_(True)

    def objective(d, lab):
        pos = ctx.dataset_positions(d)
        n_s = torch.from_numpy(lab.n_atoms.astype(np.float64)).cuda()
        e_tar = torch.from_numpy(lab.energy).cuda()
        f_tar = torch.from_numpy(np.ascontiguousarray(lab.forces.T)).float().cuda()

        def call():
            zt.grad = None
            E, F = nep.NEPEnergy.apply(pos, zt, ctx, d)
            loss = (((E - e_tar) / n_s) ** 2).sum() + ((F - f_tar) ** 2).mean()
            loss.backward()
        return call

    call = objective(ds, ls)
    call()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        call()
    torch.cuda.synchronize()
    t_call = (time.perf_counter() - t0) / reps
    # per-structure path: the first n_plain structures, each its own dataset
    off = np.concatenate([[0], np.cumsum(ls.n_atoms)])
    calls = []
    for k in range(n_plain):
        sub = I.LabelledSet(n_atoms=ls.n_atoms[k:k + 1], pos=ls.pos[off[k]:off[k + 1]],
                            boxes=ls.boxes[k:k + 1], energy=ls.energy[k:k + 1],
                            forces=ls.forces[off[k]:off[k + 1]], virial=ls.virial[k:k + 1],
                            has_virial=ls.has_virial[k:k + 1])
        calls.append(objective(ctx.dataset_create(sub, max_neighbors=96), sub))
    for c in calls:
        c()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c in calls:
        c()
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) / n_plain * len(ls.n_atoms)
    # algorithmic flops of one call: the forward pass (descriptor, network,
    # partial forces per pair, as counted for the MD kernel with the dataset's
    # own pair counts, no skin) and the backward, which forms q and the
    # directional derivative of q along dL/dF (the same per-pair work) and
    # contracts per atom 4 N_neu N_des terms into the parameter gradient
    n_at = int(ls.n_atoms.sum())
    n_r, n_a = ds.pairs()
    h = nep.hyper()
    f_fwd = FLOP_SLOT * n_r + FLOP_RADIAL * n_r + FLOP_ANGULAR * n_a + FLOP_ATOM * n_at
    f_call = 2 * f_fwd + 4 * h.n_neuron * nep.num_descriptors(h) * n_at
    achieved = f_call / t_call / 1e12
    return {"workload": "NEPEnergy autograd over 256 SW-labelled Si structures of 64-512 atoms "
                        "(%d atoms), NEP 29-30-1: forward E, F and backward dL/dz of an "
                        "energy + force loss" % int(ls.n_atoms.sum()),
            "structures_per_s": len(ls.n_atoms) / t_call, "ms_per_call": t_call * 1e3,
            "plain_per_structure_structures_per_s": len(ls.n_atoms) / t_plain,
            "plain_path": "the same call per structure on single-structure datasets, timed on "
                          "%d structures and scaled to 256" % n_plain,
            "speedup_vs_plain": t_plain / t_call,
            "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                         "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                         "gflop_per_call": f_call / 1e9,
                         "note": "algorithmic float32 flops of forward + backward over the "
                                 "whole call (host-side autograd and launches included)"}}


def pair_counts(pos, box, rc):
    """Mean number of neighbours within rc (periodic orthorhombic box)."""
    from scipy.spatial import cKDTree
    L = np.diag(box)
    tree = cKDTree(np.mod(pos, L), boxsize=L)
    return 2.0 * len(tree.query_pairs(rc, output_type="ndarray")) / len(pos)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# The one-core leg runs in a child process so that OpenMP starts with one thread.
_ONE_CORE = """
import json, sys, time
import numpy as np
sys.path.insert(0, {root!r})
import oracle as O
d = np.load({path!r})
h = O.hyper({hyper})
pos, box, vel, z = d["pos"], d["box"], d["vel"], d["z"]
t0 = time.perf_counter()
O.md_nve(h, z, pos, box, vel, {mass!r}, {dt!r}, {steps})
print(json.dumps({{"seconds": time.perf_counter() - t0}}))
"""


def cpu_baseline(h_np, z, pos, box, vel, mass, dt, target_s):
    """The FP64 oracle as it stands: velocity-Verlet steps of the same system,
    on every host thread, then on one core (a child process with
    OMP_NUM_THREADS=1)."""
    import subprocess
    import tempfile
    import oracle as O
    h = O.hyper(h_np.rc_radial, h_np.rc_angular, h_np.n_max_radial, h_np.n_max_angular,
                h_np.l_max, h_np.n_neuron)
    # one evaluation sizes the sample; the oracle's MD step costs two evaluations
    # of the first step and one per later step
    t0 = time.perf_counter()
    O.nep_eval(h, z, pos, box)
    t_eval = time.perf_counter() - t0
    steps = int(max(1, min(500, target_s / max(t_eval, 1e-9) - 1)))
    t0 = time.perf_counter()
    O.md_nve(h, z, pos, box, vel, mass, dt, steps)
    t = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    out = {"value": len(pos) * steps / t, "unit": "atom-steps/s", "cores": threads,
           "kind": "oracle", "cpu_model": cpu_model(),
           "sample": "%d velocity-Verlet steps of the same %d-atom system by the FP64 oracle "
                     "(plain C, literal angular double sum, OpenMP %d threads), %.1f s"
                     % (steps, len(pos), threads, t)}
    # one core: a sample sized from the threaded rate (about target_s / 2)
    per_step_1 = t / (steps + 1) * threads
    steps1 = int(max(1, min(20, 0.5 * target_s / max(per_step_1, 1e-9) - 1)))
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "system.npz")
        np.savez(path, pos=pos, box=box, vel=vel, z=np.asarray(z, np.float32))
        code = _ONE_CORE.format(
            root=ROOT, path=path, mass=float(mass), dt=float(dt), steps=steps1,
            hyper="%r, %r, %d, %d, %d, %d" % (h_np.rc_radial, h_np.rc_angular, h_np.n_max_radial,
                                              h_np.n_max_angular, h_np.l_max, h_np.n_neuron))
        env = dict(os.environ, OMP_NUM_THREADS="1")
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                           timeout=600)
    if r.returncode == 0:
        t1 = json.loads(r.stdout.strip().splitlines()[-1])["seconds"]
        out["one_core"] = {"value": len(pos) * steps1 / t1, "unit": "atom-steps/s", "cores": 1,
                           "sample": "%d velocity-Verlet steps of the same system, OpenMP 1 "
                                     "thread, %.1f s" % (steps1, t1)}
    else:
        out["one_core"] = {"value": None, "error": r.stderr[-300:]}
    return out


def copy_probe(torch, mib):
    """Five plain device copies of mib MiB: a kernel of known traffic that
    scales the HBM byte counters of a profiler run."""
    src = torch.ones(mib << 18, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    return src.numel() * 4


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU; this build has no multi-GPU path (--gpus %d refused)"
              % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2107_08119_amd import inputs as I
    from paper_2107_08119_amd import nep

    if args.snes_only:
        ctx = nep.Context(0)
        ctx.load_params(nep.hyper(), I.random_parameters(931, seed=1))
        line = {"snes": snes_rate(args, ctx, nep, I, torch)}
        if args.copy_probe_mib:
            line["copy_probe_bytes"] = copy_probe(torch, args.copy_probe_mib)
        print(json.dumps(line), flush=True)
        return

    n_cells = args.cells
    pos, box = I.diamond_supercell(n_cells, n_cells, n_cells)
    n = len(pos)
    vel = I.maxwell_boltzmann(n, 300.0, seed=2)
    h = nep.hyper()
    z_random = I.random_parameters(nep.num_params(h), seed=1)
    # the SNES-trained silicon model (Stillinger-Weber labels) when it is present:
    # the lattice then stays crystalline and the energy drift means something
    from paper_2107_08119_amd import train as T
    if os.path.exists(T.MODEL_SI_SW):
        z, _ = T.load_model(T.MODEL_SI_SW)
        params = "SNES-trained on Stillinger-Weber Si labels"
    else:
        z, params = z_random, "random parameters N(0, 0.1^2)"
    dt, rebuild, skin, cap, mass = 1.0, 10, 0.5, 96, I.MASS_SI

    ctx = nep.Context(0)
    ctx.load_params(h, z)
    p, v = nep.soa(pos), nep.soa(vel)
    ctx.build_neighbors(p, box, skin=skin, max_neighbors=cap)
    thermo = torch.empty((max(args.steps, args.warmup, 1), 5), dtype=torch.float64,
                         device="cuda")
    if args.warmup:
        ctx.md_step(args.warmup, dt, rebuild, mass, p, v, thermo)
    ctx.synchronize()
    # pass-1 tile shape for this system (the library's autotuner)
    lanes, tile_ms = ctx.autotune(p, reps=20)
    nb = ctx.get_neighbors()
    mean_slots = float(nb["cnt_radial"].double().mean())
    # timed region: K steps, no instrumentation
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.md_step(args.steps, dt, rebuild, mass, p, v, thermo)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ctx.synchronize()
    th = thermo[: args.steps].cpu().numpy()
    e_tot = th[:, 0] + th[:, 1]
    # dominant kernel: HIP events around back-to-back launches on the library's
    # stream, at the state the timed region ended in
    ms_partials = nep.time_partials(ctx, p, reps=200)
    # per-kernel-class event times over further steps (events attached to the
    # dispatches; they add gaps between kernels, so these steps are not timed)
    k_diag = min(args.steps, 200)
    nep.set_timing(ctx, True)
    ctx.md_step(k_diag, dt, rebuild, mass, p, v, thermo)
    kt = nep.get_timing(ctx)
    nep.set_timing(ctx, False)

    pos_end = nep.aos(p)
    nr = 0.5 * (pair_counts(pos, box, h.rc_radial) + pair_counts(pos_end, box, h.rc_radial))
    na = 0.5 * (pair_counts(pos, box, h.rc_angular) + pair_counts(pos_end, box, h.rc_angular))
    flop_atom = FLOP_SLOT * mean_slots + FLOP_RADIAL * nr + FLOP_ANGULAR * na + FLOP_ATOM
    avg_s = ms_partials / 1e3
    achieved = flop_atom * n / avg_s / 1e12
    value = n * args.steps / elapsed
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "NEP NVE velocity-Verlet MD, Si diamond %dx%dx%d cells (%d atoms), "
                        "dt 1 fs, rebuild every %d steps, skin %.1f A, NEP 29-30-1 "
                        "(r_c 5/4 A), %s" % (n_cells, n_cells, n_cells, n, rebuild, skin,
                                             params),
            "atoms": n, "dt_fs": dt, "rebuild_every": rebuild, "skin_A": skin,
            "neighbours_radial": nr, "neighbours_angular": na, "list_slots": mean_slots,
        },
        "roofline": {
            "kernel": "k_partials (descriptor, network, partial forces)",
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS,
            "peak_nonpacked": PEAK_FP32_NONPACKED_TFLOPS,
            "frac_nonpacked": achieved / PEAK_FP32_NONPACKED_TFLOPS,
            "traffic": measured_traffic(lanes),
            "flop_per_atom": flop_atom,
            "avg_launch_us": avg_s * 1e6,
            "timing": "HIP events around 200 back-to-back launches on the library stream",
            "algorithmic_GBps": (BYTE_ATOM + BYTE_SLOT * mean_slots) * n / avg_s / 1e9,
        },
        "tile": {"lanes_per_atom": lanes,
                 "us_per_launch": {"2": tile_ms[0] * 1e3, "4": tile_ms[1] * 1e3,
                                   "8": tile_ms[2] * 1e3}},
        "kernel_us_per_launch_instrumented": {
            k: (val[0] * 1e3 / val[1] if val[1] else None) for k, val in kt.items()},
        "energy_drift_meV_per_atom": float((e_tot.max() - e_tot.min()) / n * 1e3),
    }
    if args.md_only:
        if args.copy_probe_mib:
            line["copy_probe_bytes"] = copy_probe(torch, args.copy_probe_mib)
        print(json.dumps(line), flush=True)
        return
    # HNEMD (Sec. II B): the same system driven by F_e . W_i, F_e = 1 um^-1 along x
    fe = (1.0e-4, 0.0, 0.0)
    k_h = min(args.steps, 200)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    th_h = ctx.md_step(k_h, dt, rebuild, mass, p, v, thermo, fe=fe)
    torch.cuda.synchronize()
    t_h = time.perf_counter() - t0
    ctx.synchronize()
    line["hnemd_64k"] = {
        "workload": "the same 64,000-atom system with the HNEMD driving force F_e . W_i, "
                    "F_e = (1e-4, 0, 0) 1/A (1 um^-1)",
        "atom_steps_per_s": n * k_h / t_h, "steps": k_h,
        "mean_Jx_eV_A_per_fs": float(th_h[:k_h, 2].mean().item())}
    line["hnemd_spectral_64k"] = spectral_rate(ctx, nep, torch, p, v, n, box, dt, rebuild, mass,
                                               fe)
    line["paper_models"] = paper_model_rate(nep, I, torch)
    line["autograd_256"] = autograd_rate(nep, I, torch, z)
    line["pbte_64k"] = pbte_rate(nep, I, torch)
    if not args.no_disordered:
        line["disordered_512k"] = disordered_rate(args, nep, I, torch, z)
    if not args.no_snes:
        line["snes"] = snes_rate(args, ctx, nep, I, torch)
    if not args.no_cpu_baseline:
        # the oracle's work does not depend on the parameter values; it is timed
        # with the seeded random ones, which no GPU run produced
        line["cpu_baseline"] = cpu_baseline(h, z_random, pos, box, vel, mass, dt,
                                            args.cpu_seconds)
    if args.copy_probe_mib:
        line["copy_probe_bytes"] = copy_probe(torch, args.copy_probe_mib)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
