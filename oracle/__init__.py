"""FP64 CPU oracle for the NEP hot path -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this package.  It is a thin ctypes wrapper over ``nep_oracle.c`` (plain C,
float64, literal double sums), which shares no code with the GPU library.
See the header of ``nep_oracle.c`` for the passages of the paper each
function follows.  ``spectral.py`` (plain numpy, float64) holds the spectral
heat-current analysis of Sec. II B.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nep_oracle.c")
_LIB = os.path.join(_HERE, "libnep_oracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (float64, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", "-std=c99",
             "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Hyper(C.Structure):
    _fields_ = [("rc_radial", C.c_double), ("rc_angular", C.c_double),
                ("n_max_radial", C.c_int), ("n_max_angular", C.c_int),
                ("l_max", C.c_int), ("n_neuron", C.c_int)]

    def __repr__(self):
        return ("Hyper(rc_radial=%g, rc_angular=%g, n_max_radial=%d, n_max_angular=%d, "
                "l_max=%d, n_neuron=%d)" % (self.rc_radial, self.rc_angular, self.n_max_radial,
                                            self.n_max_angular, self.l_max, self.n_neuron))


def hyper(rc_radial=5.0, rc_angular=4.0, n_max_radial=8, n_max_angular=4, l_max=4,
          n_neuron=30) -> Hyper:
    return Hyper(rc_radial, rc_angular, n_max_radial, n_max_angular, l_max, n_neuron)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
        fp = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
        ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
        up = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
        bp = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
        H = C.POINTER(Hyper)
        L.or_n_des.argtypes = [H]
        L.or_n_par.argtypes = [H]
        L.or_chebyshev.argtypes = [C.c_double, C.c_int, dp, dp]
        L.or_radial_basis.argtypes = [C.c_double, C.c_double, C.c_int, dp, dp]
        L.or_legendre.argtypes = [C.c_double, C.c_int, dp, dp]
        L.or_neighbors.argtypes = [C.c_int, dp, dp, C.c_double, C.c_int, ip, ip, ip]
        L.or_nep_eval.argtypes = [H, dp, C.c_int, dp, dp, C.c_void_p, C.c_int, C.c_void_p, C.c_int,
                                  dp, dp, dp, dp, C.c_void_p]
        L.or_nep_eval_species.argtypes = [H, dp, C.c_int, dp, dp, C.c_void_p, C.c_void_p, C.c_int,
                                          C.c_void_p, C.c_int, dp, dp, dp, dp, C.c_void_p]
        L.or_md_nve.argtypes = [H, dp, C.c_int, dp, dp, dp, C.c_double, C.c_double, C.c_int,
                                C.c_int, dp]
        L.or_md_driven.argtypes = [H, dp, C.c_int, dp, dp, dp, C.c_double, C.c_double, C.c_int,
                                   C.c_int, C.c_void_p, dp]
        L.or_md_species.argtypes = [H, dp, C.c_int, dp, dp, C.c_void_p, C.c_void_p, dp,
                                    C.c_double, C.c_double, C.c_int, C.c_int, C.c_void_p, dp]
        L.or_loss.argtypes = [H, dp, C.c_int, ip, dp, dp, dp, dp, dp, bp, dp, C.c_int, dp]
        L.or_grad_params.argtypes = [H, dp, C.c_int, ip, dp, dp, dp, dp, C.c_int, dp]
        L.or_philox4x32_10.argtypes = [up, up, up]
        L.or_snes_sample.argtypes = [C.c_int, C.c_int, fp, fp, C.c_uint64, C.c_int, fp, fp]
        L.or_snes_utilities.argtypes = [C.c_int, dp]
        L.or_snes_order.argtypes = [C.c_int, dp, ip]
        L.or_snes_update.argtypes = [C.c_int, C.c_int, fp, fp, fp, dp, C.c_double, C.c_double]
        L.or_snes_eta_s.argtypes = [C.c_int]
        L.or_snes_eta_s.restype = C.c_double
        _lib = L
    return _lib


_ERR = {-1: "neighbour capacity exceeded", -2: "reverse pair missing", -3: "out of memory"}


def _check(rc):
    if rc != 0:
        raise RuntimeError("oracle: " + _ERR.get(rc, str(rc)))


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ------------------------------------------------------------------ sizes
def n_des(h: Hyper) -> int:
    return lib().or_n_des(C.byref(h))


def n_par(h: Hyper) -> int:
    return lib().or_n_par(C.byref(h))


# -------------------------------------------------------- special functions
def chebyshev(x: float, nmax: int):
    T = np.zeros(nmax + 1)
    U = np.zeros(nmax + 1)
    lib().or_chebyshev(x, nmax, T, U)
    return T, U


def radial_basis(r: float, rc: float, nmax: int):
    g = np.zeros(nmax + 1)
    dg = np.zeros(nmax + 1)
    lib().or_radial_basis(r, rc, nmax, g, dg)
    return g, dg


def legendre(c: float, lmax: int):
    P = np.zeros(max(lmax, 1) + 1)
    dP = np.zeros(max(lmax, 1) + 1)
    lib().or_legendre(c, lmax, P, dP)
    return P[: lmax + 1], dP[: lmax + 1]


# -------------------------------------------------------------- neighbours
def neighbor_arrays(pos, box, rc: float, cap: int = 256):
    """Counts [N], atom indices [N, cap] and images [N, cap, 3] (unspecified order)."""
    pos = _d(pos)
    N = len(pos)
    cnt = np.zeros(max(N, 1), np.int32)
    jl = np.zeros(max(N, 1) * cap, np.int32)
    img = np.zeros(max(N, 1) * cap * 3, np.int32)
    _check(lib().or_neighbors(N, pos, _d(box), rc, cap, cnt, jl, img))
    return cnt[:N], jl.reshape(-1, cap)[:N], img.reshape(-1, cap, 3)[:N]


def neighbors(pos, box, rc: float, cap: int = 256):
    """Per atom: sorted list of (j, n0, n1, n2) with 0 < |r_j + n.H - r_i| < rc."""
    pos = _d(pos)
    N = len(pos)
    cnt = np.zeros(max(N, 1), np.int32)
    jl = np.zeros(max(N, 1) * cap, np.int32)
    img = np.zeros(max(N, 1) * cap * 3, np.int32)
    _check(lib().or_neighbors(N, pos, _d(box), rc, cap, cnt, jl, img))
    jl = jl.reshape(-1, cap)
    img = img.reshape(-1, cap, 3)
    out = []
    for i in range(N):
        c = cnt[i]
        out.append(sorted(zip(jl[i, :c].tolist(), *(img[i, :c, a].tolist() for a in range(3)))))
    return out


# --------------------------------------------------------------------- NEP
def _params(z, exact: bool):
    """z as float64: the float32 values promoted, or (exact) as given."""
    if exact:
        return _d(z)
    return _d(np.asarray(z, dtype=np.float32).astype(np.float64))


def nep_eval(h: Hyper, z, pos, box, vel=None, sel=None, cap: int = 256, want_q: bool = False,
             exact: bool = False, Z=None):
    """Per-atom U, F, W (3x3), J and optionally q for atoms sel (default: all).
    Z: atomic numbers [N] of a multicomponent system (pair weight sqrt(Z_i Z_j))."""
    pos = _d(pos)
    N = len(pos)
    z = _params(z, exact)
    if sel is None:
        n_sel, sel_arr = N, None
    else:
        sel_arr = np.ascontiguousarray(sel, dtype=np.int32)
        n_sel = len(sel_arr)
    U = np.zeros(max(n_sel, 1))
    F = np.zeros((max(n_sel, 1), 3))
    W = np.zeros((max(n_sel, 1), 9))
    J = np.zeros((max(n_sel, 1), 3))
    q = np.zeros((max(n_sel, 1), n_des(h))) if want_q else None
    v = _d(vel) if vel is not None else None
    Zi = None if Z is None else np.ascontiguousarray(Z, dtype=np.int32)
    if Zi is not None and len(Zi) != N:
        raise ValueError("Z must have one entry per atom")
    _check(lib().or_nep_eval_species(
        C.byref(h), z, N, pos, _d(box), None if Zi is None else Zi.ctypes.data,
        v.ctypes.data if v is not None else None, n_sel,
        sel_arr.ctypes.data if sel_arr is not None else None, cap, U, F, W, J,
        q.ctypes.data if q is not None else None))
    out = {"U": U[:n_sel], "F": F[:n_sel], "W": W[:n_sel].reshape(-1, 3, 3), "J": J[:n_sel]}
    if want_q:
        out["q"] = q[:n_sel]
    return out


def md_nve(h: Hyper, z, pos, box, vel, mass, dt: float, n_steps: int, cap: int = 256,
           fe=None, Z=None):
    """Velocity-Verlet NVE (with the HNEMD driving force F_e . W_i when fe is
    given, Sec. II B); returns (thermo [n_steps, 5], pos, vel).  mass is one
    value in amu or one per atom; Z: atomic numbers of a multicomponent system."""
    pos = _d(pos).copy()
    vel = _d(vel).copy()
    thermo = np.zeros((max(n_steps, 1), 5))
    z = _d(np.asarray(z, dtype=np.float32).astype(np.float64))
    fe_arr = None if fe is None else _d(np.asarray(fe, dtype=np.float64).reshape(3))
    m = np.asarray(mass, dtype=np.float64)
    masses = None if m.ndim == 0 else _d(m)
    if masses is not None and len(masses) != len(pos):
        raise ValueError("one mass per atom")
    Zi = None if Z is None else np.ascontiguousarray(Z, dtype=np.int32)
    _check(lib().or_md_species(C.byref(h), z, len(pos), pos, _d(box),
                               None if Zi is None else Zi.ctypes.data,
                               None if masses is None else masses.ctypes.data, vel,
                               float(m) if masses is None else 0.0, dt, n_steps, cap,
                               None if fe_arr is None else fe_arr.ctypes.data, thermo))
    return thermo[:n_steps], pos, vel


def grad_params(h: Hyper, z, ds, gE, gF, cap: int = 256, exact: bool = False):
    """d/dz of sum_s gE_s E_s + sum_i gF_i . F_i over a structure set."""
    grad = np.zeros(n_par(h))
    _check(lib().or_grad_params(
        C.byref(h), _params(z, exact), len(ds.n_atoms), np.ascontiguousarray(ds.n_atoms, np.int32),
        _d(ds.boxes), _d(ds.pos), _d(gE), _d(gF), cap, grad))
    return grad


def loss(h: Hyper, z, ds, lam=(1.0, 1.0, 1.0, 0.05, 0.05), cap: int = 256):
    """(L, L_e, L_f, L_v, L_1, L_2) of parameter vector z on a labelled set."""
    out = np.zeros(6)
    z = _d(np.asarray(z, dtype=np.float32).astype(np.float64))
    _check(lib().or_loss(
        C.byref(h), z, len(ds.n_atoms), np.ascontiguousarray(ds.n_atoms, np.int32),
        _d(ds.boxes), _d(ds.pos), _d(ds.energy), _d(ds.forces), _d(ds.virial),
        np.ascontiguousarray(ds.has_virial, np.uint8), _d(lam), cap, out))
    return out


# -------------------------------------------------------------------- SNES
def philox4x32_10(ctr, key):
    out = np.zeros(4, np.uint32)
    lib().or_philox4x32_10(np.ascontiguousarray(ctr, np.uint32),
                           np.ascontiguousarray(key, np.uint32), out)
    return out


def snes_sample(m, s, seed: int, gen: int, n_pop: int):
    m = np.ascontiguousarray(m, np.float32)
    s = np.ascontiguousarray(s, np.float32)
    r = np.zeros((n_pop, len(m)), np.float32)
    z = np.zeros((n_pop, len(m)), np.float32)
    lib().or_snes_sample(len(m), n_pop, m, s, seed, gen, r, z)
    return r, z


def snes_utilities(n_pop: int):
    u = np.zeros(n_pop)
    lib().or_snes_utilities(n_pop, u)
    return u


def snes_order(losses):
    losses = _d(losses)
    order = np.zeros(len(losses), np.int32)
    lib().or_snes_order(len(losses), losses, order)
    return order


def snes_update(m, s, r, losses, eta_m: float = 1.0, eta_s: float | None = None):
    m = np.array(m, np.float32)
    s = np.array(s, np.float32)
    r = np.ascontiguousarray(r, np.float32)
    if eta_s is None:
        eta_s = snes_eta_s(len(m))
    lib().or_snes_update(len(m), r.shape[0], m, s, r, _d(losses), eta_m, eta_s)
    return m, s


def snes_eta_s(n_par: int) -> float:
    return lib().or_snes_eta_s(n_par)
