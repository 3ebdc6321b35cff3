"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds no NEP arithmetic. It builds atomic configurations
(diamond silicon supercells, random dense packings, strained small cells with
vacancies), Maxwell-Boltzmann velocities, random parameter vectors, and the
Stillinger-Weber silicon labels used as training targets for the SNES loss.

The paper's own training sets (DFT data for general Si, silicene and PbTe,
Sec. III A) are not available; silicon structures labelled by the
Stillinger-Weber potential stand in for them.  The MD speed test of Sec. III D
(bulk Si, 8000 atoms, 100 steps) is stood in for by a 64,000-atom diamond cell.

Conventions: positions in Angstrom as float64 arrays of shape [N, 3]; a box is
a float64 [3, 3] array whose ROWS are the cell vectors a, b, c, so that a
lattice translation is n @ box; velocities in Angstrom/fs; masses in amu;
energies in eV.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# ---------------------------------------------------------------------------
# Physical constants (CODATA 2018 exact/recommended values)
# ---------------------------------------------------------------------------
ELEMENTARY_CHARGE = 1.602176634e-19  # C
ATOMIC_MASS_UNIT = 1.66053906660e-27  # kg
BOLTZMANN_EV = 8.617333262e-5  # eV/K
# acceleration of 1 eV/Angstrom acting on 1 amu, in Angstrom/fs^2
ACCEL_UNIT = ELEMENTARY_CHARGE / ATOMIC_MASS_UNIT * 1.0e-10  # (1e10 m^-1 per A^-1) x (1e-20 A/fs^2 per m/s^2)
MASS_SI = 28.0855  # amu
DIAMOND_SI_A = 5.43  # Angstrom, lattice constant used by the workloads

# ---------------------------------------------------------------------------
# Lattices
# ---------------------------------------------------------------------------
_DIAMOND_BASIS = np.array(
    [
        [0.00, 0.00, 0.00],
        [0.00, 0.50, 0.50],
        [0.50, 0.00, 0.50],
        [0.50, 0.50, 0.00],
        [0.25, 0.25, 0.25],
        [0.25, 0.75, 0.75],
        [0.75, 0.25, 0.75],
        [0.75, 0.75, 0.25],
    ]
)


def diamond_supercell(n1: int, n2: int, n3: int, a: float = DIAMOND_SI_A):
    """Conventional 8-atom diamond cells repeated n1 x n2 x n3 (orthorhombic box)."""
    cells = np.array(
        [[i, j, k] for i in range(n1) for j in range(n2) for k in range(n3)], dtype=np.float64
    )
    frac = (cells[:, None, :] + _DIAMOND_BASIS[None, :, :]).reshape(-1, 3)
    pos = frac * a
    box = np.diag([n1 * a, n2 * a, n3 * a]).astype(np.float64)
    return pos, box


# Two-species test system: rock-salt PbTe (Pb on the fcc sites, Te on the
# octahedral sites), the kind of ionic crystal the paper fits with a longer
# radial than angular cutoff.
PBTE_A = 6.46  # Angstrom, room-temperature lattice constant of PbTe
Z_PB, Z_TE = 82, 52  # atomic numbers
MASS_PB, MASS_TE = 207.2, 127.60  # amu
_ROCKSALT_A = np.array([[0.0, 0.0, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5], [0.5, 0.5, 0.0]])
_ROCKSALT_B = _ROCKSALT_A + np.array([0.5, 0.0, 0.0])


def rocksalt_supercell(n1: int, n2: int, n3: int, a: float = PBTE_A):
    """Conventional 8-atom rock-salt cells repeated n1 x n2 x n3: (pos, box,
    Z, masses), four Pb then four Te per cell."""
    cells = np.array(
        [[i, j, k] for i in range(n1) for j in range(n2) for k in range(n3)], dtype=np.float64
    )
    basis = np.concatenate([_ROCKSALT_A, _ROCKSALT_B % 1.0])
    frac = (cells[:, None, :] + basis[None, :, :]).reshape(-1, 3)
    n_cells = len(cells)
    Z = np.tile(np.array([Z_PB] * 4 + [Z_TE] * 4, dtype=np.int32), n_cells)
    masses = np.where(Z == Z_PB, MASS_PB, MASS_TE).astype(np.float64)
    box = np.diag([n1 * a, n2 * a, n3 * a]).astype(np.float64)
    return frac * a, box, Z, masses


# Buckled honeycomb silicene (2D): in-plane lattice constant and buckling
# height are standard literature values, not the paper's.
SILICENE_A = 3.86  # Angstrom
SILICENE_BUCKLE = 0.44  # Angstrom


def silicene_sheet(n1: int, n2: int, a: float = SILICENE_A, buckle: float = SILICENE_BUCKLE,
                   height: float = 20.0):
    """Rectangular 4-atom cells (a x sqrt(3) a) of buckled silicene repeated
    n1 x n2 in the plane, one sheet in a box of the given height (vacuum
    along z, periodic in all three directions)."""
    r3 = math.sqrt(3.0)
    d = a / r3  # in-plane nearest-neighbour distance
    basis = np.array([[0.0, 0.0, 0.5 * buckle],
                      [0.5 * a, 0.5 * d, -0.5 * buckle],
                      [0.5 * a, 0.5 * r3 * a, 0.5 * buckle],
                      [0.0, 0.5 * r3 * a + 0.5 * d, -0.5 * buckle]])
    cells = np.array([[i * a, j * r3 * a, 0.0] for i in range(n1) for j in range(n2)])
    pos = (cells[:, None, :] + basis[None, :, :]).reshape(-1, 3)
    pos[:, 2] += 0.5 * height
    box = np.diag([n1 * a, n2 * r3 * a, height]).astype(np.float64)
    return pos, box


def wrap_positions(pos: np.ndarray, box: np.ndarray) -> np.ndarray:
    """Map positions into the cell spanned by the box rows (fractional in [0,1))."""
    frac = pos @ np.linalg.inv(box)
    frac -= np.floor(frac)
    return frac @ box


def perpendicular_widths(box: np.ndarray) -> np.ndarray:
    """Distance between opposite faces of the cell, one per cell vector."""
    vol = abs(np.linalg.det(box))
    a, b, c = box
    return np.array(
        [vol / np.linalg.norm(np.cross(b, c)), vol / np.linalg.norm(np.cross(c, a)),
         vol / np.linalg.norm(np.cross(a, b))]
    )


# ---------------------------------------------------------------------------
# Random numbers for the model and the dynamics
# ---------------------------------------------------------------------------
def random_parameters(n_par: int, seed: int, std: float = 0.1) -> np.ndarray:
    """Parameter vector z with entries N(0, std^2), rounded to float32."""
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(n_par) * std).astype(np.float32)


def maxwell_boltzmann(n_atoms: int, temperature: float, seed: int, mass=MASS_SI):
    """Velocities (Angstrom/fs) drawn from the Maxwell-Boltzmann distribution;
    mass is one value in amu or one per atom.

    The centre-of-mass velocity is removed and the result is rescaled so that
    the kinetic temperature with 3N-3 degrees of freedom equals `temperature`.
    """
    rng = np.random.default_rng(seed)
    if np.ndim(mass) == 0:
        sigma = math.sqrt(BOLTZMANN_EV * temperature / mass * ACCEL_UNIT)
        v = rng.standard_normal((n_atoms, 3)) * sigma
        v -= v.mean(axis=0, keepdims=True)
        m = float(mass)
    else:
        m = np.asarray(mass, dtype=np.float64).reshape(n_atoms, 1)
        v = rng.standard_normal((n_atoms, 3)) * np.sqrt(BOLTZMANN_EV * temperature / m * ACCEL_UNIT)
        v -= (m * v).sum(axis=0, keepdims=True) / m.sum()
    if n_atoms > 1:
        if np.ndim(m) == 0:
            ekin = 0.5 * m * float(np.sum(v * v)) / ACCEL_UNIT
        else:
            ekin = 0.5 * float(np.sum(m * v * v)) / ACCEL_UNIT
        t_now = 2.0 * ekin / ((3 * n_atoms - 3) * BOLTZMANN_EV)
        v *= math.sqrt(temperature / t_now)
    return v


def kinetic_energy(vel: np.ndarray, mass=MASS_SI) -> float:
    """Kinetic energy in eV of velocities in Angstrom/fs (one mass or one per atom)."""
    if np.ndim(mass) == 0:
        return 0.5 * mass * float(np.sum(vel * vel)) / ACCEL_UNIT
    m = np.asarray(mass, dtype=np.float64).reshape(len(vel), 1)
    return 0.5 * float(np.sum(m * vel * vel)) / ACCEL_UNIT


# ---------------------------------------------------------------------------
# Random dense packing (random sequential addition with a hard minimum distance)
# ---------------------------------------------------------------------------
def random_packing(n_atoms: int, box_length: float, d_min: float, seed: int,
                   batch: int = 65536) -> np.ndarray:
    """Uniform random points in a periodic cube, no two closer than d_min.

    Candidates are drawn uniformly in batches.  A candidate is kept iff it is
    at least d_min away (minimum image) from every atom kept before its batch
    and from every earlier candidate of its batch that passed that first test.
    Kept candidates are appended in draw order until n_atoms are placed.  The
    result depends only on the seed.
    """
    rng = np.random.default_rng(seed)
    L = float(box_length)
    ncell = max(3, int(L // d_min))
    cw = L / ncell
    cap = 5  # cells are about d_min wide; more than 5 members raises
    grid = -np.ones((ncell, ncell, ncell, cap), dtype=np.int64)
    fill = np.zeros((ncell, ncell, ncell), dtype=np.int64)
    pos = np.empty((n_atoms, 3), dtype=np.float64)
    n = 0
    d2min = d_min * d_min
    offs = np.array([[i, j, k] for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1)])

    def clashes(points, cells, g, pts, earlier_only):
        """True where a point has a grid member closer than d_min."""
        hit = np.zeros(len(points), dtype=bool)
        me = np.arange(len(points))
        for o in offs:
            c = (cells + o) % ncell
            ids = g[c[:, 0], c[:, 1], c[:, 2]]
            valid = ids >= 0
            if earlier_only:
                valid &= ids < me[:, None]
            p = pts[np.where(valid, ids, 0)]
            d = p - points[:, None, :]
            d -= L * np.round(d / L)
            hit |= np.any(valid & (np.sum(d * d, axis=-1) < d2min), axis=1)
        return hit

    def ranks_in_cells(cells):
        """Order of points by cell (then by index) and each point's rank in its cell."""
        order = np.lexsort((np.arange(len(cells)), cells[:, 2], cells[:, 1], cells[:, 0]))
        key = (cells[order, 0] * ncell + cells[order, 1]) * ncell + cells[order, 2]
        rank = np.arange(len(key)) - np.searchsorted(key, key, side="left")
        return order, rank

    sgrid = -np.ones((ncell, ncell, ncell, cap), dtype=np.int64)
    while n < n_atoms:
        cand = rng.random((batch, 3)) * L
        cc = np.minimum((cand // cw).astype(np.int64), ncell - 1)
        ok = ~clashes(cand, cc, grid, pos, False)
        surv = cand[ok]
        sc = cc[ok]
        # survivors of this batch binned by cell; earlier survivors win
        order, rank = ranks_in_cells(sc)
        if len(rank) and rank.max() >= cap:
            raise RuntimeError("packing grid cell overflow")
        sgrid[sc[order, 0], sc[order, 1], sc[order, 2], rank] = order
        keep = ~clashes(surv, sc, sgrid, surv, True)
        sgrid[sc[:, 0], sc[:, 1], sc[:, 2], :] = -1
        kept = surv[keep][: n_atoms - n]
        kc = sc[keep][: n_atoms - n]
        order, rank = ranks_in_cells(kc)
        slot = fill[kc[order, 0], kc[order, 1], kc[order, 2]] + rank
        if len(slot) and slot.max() >= cap:
            raise RuntimeError("packing grid cell overflow")
        grid[kc[order, 0], kc[order, 1], kc[order, 2], slot] = n + order
        np.add.at(fill, (kc[:, 0], kc[:, 1], kc[:, 2]), 1)
        pos[n:n + len(kept)] = kept
        n += len(kept)
    return pos


# ---------------------------------------------------------------------------
# Small strained training cells with vacancies
# ---------------------------------------------------------------------------
def smallest_supercell(n_atoms: int, max_rep: int = 8):
    """Smallest n1<=n2<=n3 conventional diamond supercell holding >= n_atoms atoms.

    Ties in size are broken towards the most compact shape (largest n1, then n2).
    """
    best = None
    for n1 in range(1, max_rep + 1):
        for n2 in range(n1, max_rep + 1):
            for n3 in range(n2, max_rep + 1):
                size = 8 * n1 * n2 * n3
                if size < n_atoms:
                    continue
                key = (size, -n1, -n2)
                if best is None or key < best[0]:
                    best = (key, (n1, n2, n3))
    if best is None:
        raise ValueError("structure too large")
    return best[1]


def random_strain(rng, max_strain: float) -> np.ndarray:
    """Symmetric strain tensor with six independent components U(-max, max)."""
    e = rng.uniform(-max_strain, max_strain, size=6)
    return np.array([[e[0], e[5], e[4]], [e[5], e[1], e[3]], [e[4], e[3], e[2]]])


@dataclass
class Structure:
    pos: np.ndarray  # [n, 3]
    box: np.ndarray  # [3, 3] rows are cell vectors


def training_structures(n_struct: int, n_min: int, n_max: int, seed: int,
                        max_strain: float = 0.03, jitter: float = 0.1,
                        a: float = DIAMOND_SI_A) -> list:
    """Strained, jittered diamond-Si cells with random vacancies.

    Each structure draws N_s ~ U{n_min..n_max}, takes the smallest conventional
    supercell that holds N_s atoms, deletes random atoms down to N_s, applies a
    random symmetric strain (H' = H (I + eps)) and adds N(0, jitter^2) noise to
    every coordinate.  Positions are wrapped into the strained cell.
    """
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_struct):
        ns = int(rng.integers(n_min, n_max + 1))
        n1, n2, n3 = smallest_supercell(ns)
        pos, box = diamond_supercell(n1, n2, n3, a)
        keep = np.sort(rng.permutation(len(pos))[:ns])
        pos = pos[keep]
        eps = random_strain(rng, max_strain)
        deform = np.eye(3) + eps
        pos = pos @ deform
        box = box @ deform
        pos = pos + rng.standard_normal(pos.shape) * jitter
        out.append(Structure(wrap_positions(pos, box), box))
    return out


# ---------------------------------------------------------------------------
# Stillinger-Weber silicon (the teacher that labels training structures)
# ---------------------------------------------------------------------------
# Stillinger & Weber, Phys. Rev. B 31, 5262 (1985), silicon parameter set.
SW_EPSILON = 2.1683  # eV
SW_SIGMA = 2.0951  # Angstrom
SW_A = 7.049556277
SW_B = 0.6022245584
SW_P = 4.0
SW_Q = 0.0
SW_CUT = 1.80  # in units of sigma
SW_LAMBDA = 21.0
SW_GAMMA = 1.20


def _image_pairs(pos: np.ndarray, box: np.ndarray, rc: float):
    """All ordered (i, j, image) with 0 < |r_j + n.H - r_i| < rc (brute force)."""
    n = len(pos)
    inv = np.linalg.inv(box)
    frac = pos @ inv
    widths = perpendicular_widths(box)
    kmax = [int(math.floor(0.5 + rc / w)) + 1 for w in widths]
    ds = frac[None, :, :] - frac[:, None, :]
    shift0 = -np.round(ds)
    I, J = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    ii, jj, dd = [], [], []
    for m0 in range(-kmax[0], kmax[0] + 1):
        for m1 in range(-kmax[1], kmax[1] + 1):
            for m2 in range(-kmax[2], kmax[2] + 1):
                nshift = shift0 + np.array([m0, m1, m2], dtype=np.float64)
                d = (ds + nshift) @ box
                r2 = np.sum(d * d, axis=-1)
                sel = (r2 < rc * rc) & (r2 > 1e-20)
                if np.any(sel):
                    ii.append(I[sel])
                    jj.append(J[sel])
                    dd.append(d[sel])
    if not ii:
        return np.zeros(0, int), np.zeros(0, int), np.zeros((0, 3))
    return np.concatenate(ii), np.concatenate(jj), np.concatenate(dd)


def stillinger_weber(pos: np.ndarray, box: np.ndarray):
    """Energy (eV), forces (eV/A, [n,3]) and virial (eV, [3,3]) of a periodic cell.

    E = sum_{i<j} phi2(r_ij) + sum_i sum_{j<k} phi3(r_ij, r_ik, theta_jik).
    The virial is W_ab = -sum over pair vectors d of d_a (dE/dd)_b, which for
    an isolated cluster equals sum_i r_i (x) F_i.
    """
    eps, sig = SW_EPSILON, SW_SIGMA
    rc = SW_CUT * sig
    n = len(pos)
    ii, jj, d = _image_pairs(pos, box, rc)
    r = np.sqrt(np.sum(d * d, axis=1))
    u = d / r[:, None]
    forces = np.zeros((n, 3))
    virial = np.zeros((3, 3))
    # two-body: each unordered pair appears twice among ordered pairs
    sr = sig / r
    ex = np.exp(sig / (r - rc))
    bracket = SW_B * sr ** SW_P - sr ** SW_Q
    phi2 = SW_A * eps * bracket * ex
    dbracket = (-SW_P * SW_B * sr ** SW_P + SW_Q * sr ** SW_Q) / r
    dex = ex * (-sig / (r - rc) ** 2)
    dphi2 = SW_A * eps * (dbracket * ex + bracket * dex)
    energy = 0.5 * float(np.sum(phi2))
    g = 0.5 * dphi2[:, None] * u  # dE/dd for each ordered pair (half weight)
    np.add.at(forces, ii, g)
    np.add.at(forces, jj, -g)
    virial -= d.T @ g
    # three-body: for each centre i, unordered pairs (j, k) of its neighbours
    order = np.argsort(ii, kind="stable")
    ii, jj, d, r, u = ii[order], jj[order], d[order], r[order], u[order]
    # all (a, b) with a < b inside each centre's group of consecutive pairs
    same = []
    for gap in range(1, len(ii)):
        first = np.arange(len(ii) - gap)
        hit = ii[first] == ii[first + gap]
        if not np.any(hit):
            break
        same.append((first[hit], first[hit] + gap))
    a_list = [x[0] for x in same]
    b_list = [x[1] for x in same]
    energy3 = 0.0
    if a_list:
        A = np.concatenate(a_list)
        B = np.concatenate(b_list)
        c = np.sum(u[A] * u[B], axis=1)
        e1 = np.exp(SW_GAMMA * sig / (r[A] - rc))
        e2 = np.exp(SW_GAMMA * sig / (r[B] - rc))
        de1 = e1 * (-SW_GAMMA * sig / (r[A] - rc) ** 2)
        de2 = e2 * (-SW_GAMMA * sig / (r[B] - rc) ** 2)
        cc = c + 1.0 / 3.0
        h = SW_LAMBDA * eps * cc * cc * e1 * e2
        energy3 = float(np.sum(h))
        dc_dA = (u[B] - c[:, None] * u[A]) / r[A][:, None]
        dc_dB = (u[A] - c[:, None] * u[B]) / r[B][:, None]
        pref = SW_LAMBDA * eps
        gA = pref * (2 * cc * e1 * e2)[:, None] * dc_dA + (pref * cc * cc * de1 * e2)[:, None] * u[A]
        gB = pref * (2 * cc * e1 * e2)[:, None] * dc_dB + (pref * cc * cc * e1 * de2)[:, None] * u[B]
        centre = ii[A]
        np.add.at(forces, centre, gA + gB)
        np.add.at(forces, jj[A], -gA)
        np.add.at(forces, jj[B], -gB)
        virial -= d[A].T @ gA + d[B].T @ gB
    return energy + energy3, forces, virial


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------
VIRIAL_COMPONENTS = ((0, 0), (1, 1), (2, 2), (0, 1), (1, 2), (2, 0))  # xx yy zz xy yz zx


def parity_cell(seed: int = 0):
    """216-atom Si diamond 3x3x3, a = 5.43 A, every coordinate jittered N(0, 0.05^2)."""
    pos, box = diamond_supercell(3, 3, 3)
    rng = np.random.default_rng(seed)
    pos = pos + rng.standard_normal(pos.shape) * 0.05
    return pos, box


def nve_cell():
    """64,000-atom Si diamond 20x20x20, a = 5.43 A, perfect lattice."""
    return diamond_supercell(20, 20, 20)


def disordered_cell(n_atoms: int = 512000, seed: int = 3, density_gcc: float = 2.33,
                    d_min: float = 2.0):
    """Random periodic cube of silicon at the given mass density, min distance d_min."""
    number_density = density_gcc / (MASS_SI * ATOMIC_MASS_UNIT * 1e3) * 1e-24  # per A^3
    L = (n_atoms / number_density) ** (1.0 / 3.0)
    pos = random_packing(n_atoms, L, d_min, seed)
    return pos, np.diag([L, L, L]).astype(np.float64)


@dataclass
class LabelledSet:
    n_atoms: np.ndarray  # [S] int32
    boxes: np.ndarray  # [S, 9] float64 (row-major box rows)
    pos: np.ndarray  # [sum N, 3]
    energy: np.ndarray  # [S] total energy, eV
    forces: np.ndarray  # [sum N, 3] eV/A
    virial: np.ndarray  # [S, 6] total virial xx yy zz xy yz zx, eV
    has_virial: np.ndarray  # [S] uint8


def labelled_set(n_struct: int, n_min: int, n_max: int, seed: int) -> LabelledSet:
    """Training structures labelled by the Stillinger-Weber teacher in float64."""
    structs = training_structures(n_struct, n_min, n_max, seed)
    n_atoms = np.array([len(s.pos) for s in structs], dtype=np.int32)
    boxes = np.stack([s.box.reshape(9) for s in structs])
    pos = np.concatenate([s.pos for s in structs])
    energy = np.empty(n_struct)
    forces = np.empty_like(pos)
    virial = np.empty((n_struct, 6))
    off = 0
    for k, s in enumerate(structs):
        e, f, w = stillinger_weber(s.pos, s.box)
        energy[k] = e
        forces[off:off + len(s.pos)] = f
        virial[k] = [w[a, b] for a, b in VIRIAL_COMPONENTS]
        off += len(s.pos)
    return LabelledSet(n_atoms, boxes, pos, energy, forces, virial,
                       np.ones(n_struct, dtype=np.uint8))
