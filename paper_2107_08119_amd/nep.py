"""Thin Python binding of libnep (the C ABI declared in include/nep.h).

Only argument marshalling happens here: torch tensors provide device memory
and the current HIP stream, every step of the computation runs in the HIP
kernels of libnep.so.  The library must be built (``__graft_entry__.build()``
or ``python -m paper_2107_08119_amd.build``); nothing falls back to the CPU.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libnep.so")

NEP_OK, NEP_EINVAL, NEP_ESTATE, NEP_ENOMEM, NEP_EOVERFLOW = 0, 1, 2, 3, 4
NEP_ENONFINITE, NEP_EDEVICE, NEP_ENOTIMPL, NEP_EIMAGE, NEP_ESKIN = 5, 6, 7, 8, 9
STATUS_NAMES = {0: "NEP_OK", 1: "NEP_EINVAL", 2: "NEP_ESTATE", 3: "NEP_ENOMEM",
                4: "NEP_EOVERFLOW", 5: "NEP_ENONFINITE", 6: "NEP_EDEVICE", 7: "NEP_ENOTIMPL",
                8: "NEP_EIMAGE", 9: "NEP_ESKIN"}

EXPORTED = [
    "nep_create", "nep_destroy", "nep_last_error", "nep_set_stream", "nep_synchronize",
    "nep_num_descriptors", "nep_num_params", "nep_load_params", "nep_build_neighbors",
    "nep_get_neighbors", "nep_compute", "nep_md_step", "nep_set_timing", "nep_get_timing",
    "nep_time_partials", "nep_dataset_create", "nep_dataset_destroy", "snes_eval_population",
    "snes_sample", "snes_update", "nep_dataset_set_positions", "nep_dataset_get_positions",
    "nep_dataset_compute", "nep_dataset_backward", "snes_autotune", "snes_run",
    "snes_set_tile", "nep_dataset_pairs", "nep_autotune", "nep_set_tile", "nep_md_step_driven",
    "nep_set_species",
    "nep_vvcf_create", "nep_vvcf_destroy", "nep_vvcf_sample", "nep_vvcf_get", "nep_vvcf_spectrum",
    "nep_evaluate_static", "nep_static_workspace_bytes",
]


class NepError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, str(status)), message))
        self.status = status


class Hyper(C.Structure):
    """nep_hyper: cutoffs (A), Chebyshev orders, Legendre order, hidden neurons."""
    _fields_ = [("rc_radial", C.c_double), ("rc_angular", C.c_double),
                ("n_max_radial", C.c_int), ("n_max_angular", C.c_int),
                ("l_max", C.c_int), ("n_neuron", C.c_int)]


def hyper(rc_radial=5.0, rc_angular=4.0, n_max_radial=8, n_max_angular=4, l_max=4,
          n_neuron=30) -> Hyper:
    return Hyper(rc_radial, rc_angular, n_max_radial, n_max_angular, l_max, n_neuron)


_lib = None


def lib() -> C.CDLL:
    """Load libnep.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError("libnep.so is not built: run __graft_entry__.build()")
        L = C.CDLL(_LIB_PATH)
        vp, ip, dp, fp = C.c_void_p, C.c_int, C.c_double, C.c_void_p
        H = C.POINTER(Hyper)
        L.nep_create.argtypes = [C.POINTER(vp), ip, vp]
        L.nep_destroy.argtypes = [vp]
        L.nep_destroy.restype = None
        L.nep_last_error.argtypes = [vp]
        L.nep_last_error.restype = C.c_char_p
        L.nep_set_stream.argtypes = [vp, vp]
        L.nep_synchronize.argtypes = [vp]
        L.nep_num_descriptors.argtypes = [H]
        L.nep_num_params.argtypes = [H]
        L.nep_load_params.argtypes = [vp, H, vp, ip]
        L.nep_build_neighbors.argtypes = [vp, ip, vp, C.POINTER(C.c_double), dp, ip]
        L.nep_get_neighbors.argtypes = [vp, vp, vp, vp, vp, vp]
        L.nep_compute.argtypes = [vp, vp, vp, vp, fp, vp, vp, vp]
        L.nep_md_step.argtypes = [vp, ip, dp, ip, dp, vp, vp, vp, vp, vp]
        L.nep_md_step_driven.argtypes = [vp, ip, dp, ip, dp, vp, vp, vp, vp, vp, vp]
        L.nep_set_species.argtypes = [vp, ip, vp, vp]
        L.nep_vvcf_create.argtypes = [vp, ip, ip, C.POINTER(vp)]
        L.nep_vvcf_destroy.argtypes = [vp]
        L.nep_vvcf_destroy.restype = None
        L.nep_vvcf_sample.argtypes = [vp, vp, vp, vp]
        L.nep_vvcf_get.argtypes = [vp, vp, vp, C.POINTER(C.c_longlong)]
        L.nep_vvcf_spectrum.argtypes = [vp, vp, dp, dp, dp, dp, ip, vp, vp, vp]
        L.nep_set_timing.argtypes = [vp, ip]
        L.nep_get_timing.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int)]
        L.nep_time_partials.argtypes = [vp, vp, ip, C.POINTER(C.c_double)]
        L.nep_dataset_create.argtypes = [vp, ip, vp, vp, vp, vp, vp, vp, vp, ip, C.POINTER(vp)]
        L.nep_dataset_destroy.argtypes = [vp]
        L.nep_dataset_destroy.restype = None
        L.nep_dataset_pairs.argtypes = [vp, vp, vp]
        L.snes_eval_population.argtypes = [vp, vp, ip, vp, vp, vp]
        L.snes_sample.argtypes = [vp, ip, ip, vp, vp, C.c_ulonglong, ip, vp, vp]
        L.snes_update.argtypes = [vp, ip, ip, vp, vp, vp, vp, dp, dp]
        L.snes_autotune.argtypes = [vp, vp, ip, vp, ip, C.POINTER(C.c_int),
                                    C.POINTER(C.c_double)]
        L.snes_set_tile.argtypes = [vp, vp, ip]
        L.nep_autotune.argtypes = [vp, vp, ip, C.POINTER(C.c_int), C.POINTER(C.c_double)]
        L.nep_set_tile.argtypes = [vp, ip]
        L.snes_run.argtypes = [vp, vp, ip, ip, vp, vp, C.c_ulonglong, ip, ip, vp, dp, dp, vp, vp,
                               vp, vp]
        L.nep_dataset_set_positions.argtypes = [vp, vp, vp]
        L.nep_dataset_get_positions.argtypes = [vp, vp, vp]
        L.nep_dataset_compute.argtypes = [vp, vp, vp, vp, vp, vp]
        L.nep_dataset_backward.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.nep_evaluate_static.argtypes = [vp, ip, vp, C.POINTER(C.c_double), dp, ip, vp, vp,
                                          vp, vp, vp, vp]
        L.nep_static_workspace_bytes.argtypes = []
        L.nep_static_workspace_bytes.restype = C.c_size_t
        for name in EXPORTED:
            if name not in ("nep_destroy", "nep_last_error", "nep_num_descriptors",
                            "nep_num_params", "nep_dataset_destroy", "nep_vvcf_destroy",
                            "nep_static_workspace_bytes"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _ptr(t):
    """Device address of a tensor handed to the library (None for NULL)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise TypeError("the library needs CUDA tensors, got one on %s" % t.device)
    return C.c_void_p(t.data_ptr())


def _require(t, dtype, shape=None, name="tensor", min_rows=None):
    """Check a buffer handed to the library before any call is made: a tensor of
    `dtype`, contiguous, of exactly `shape` (None entries match any size), or
    with at least `min_rows` rows where given.  The library writes exactly the
    documented extent of each output, so a smaller buffer would be written past
    its end.  That the tensor lives on the GPU is checked by _ptr."""
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if shape is not None:
        ok = t.dim() == len(shape) and all(
            want is None or got == want for got, want in zip(t.shape, shape))
        if ok and min_rows is not None:
            ok = t.shape[0] >= min_rows
        if not ok:
            want = tuple("*" if w is None else w for w in shape)
            if min_rows is not None:
                want = ">= %d rows of %s" % (min_rows, want)
            raise ValueError("%s must have shape %s, got %s" % (name, want, tuple(t.shape)))
    return t


def num_params(h: Hyper) -> int:
    return lib().nep_num_params(C.byref(h))


def num_descriptors(h: Hyper) -> int:
    return lib().nep_num_descriptors(C.byref(h))


class Context:
    """A libnep context bound to one device and the current torch stream."""

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None):
        self._lib = lib()
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = C.c_void_p()
        st = self._lib.nep_create(C.byref(h), device, C.c_void_p(stream.cuda_stream))
        if st != NEP_OK:
            raise NepError(st, "nep_create failed")
        self._h = h
        self.n = 0
        self.cap = 0
        self.hyper = None

    def close(self):
        if getattr(self, "_h", None):
            self._lib.nep_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int):
        if st != NEP_OK:
            raise NepError(st, self._lib.nep_last_error(self._h).decode())

    # -- C ABI calls ---------------------------------------------------------
    def synchronize(self):
        self._check(self._lib.nep_synchronize(self._h))

    def load_params(self, h: Hyper, z) -> None:
        z = np.ascontiguousarray(z, dtype=np.float32)
        self._check(self._lib.nep_load_params(self._h, C.byref(h), z.ctypes.data, len(z)))
        self.hyper = h

    def build_neighbors(self, pos: torch.Tensor, box, skin: float = 0.5,
                        max_neighbors: int = 64) -> None:
        n = pos.shape[1] if pos.dim() == 2 else 0
        _require(pos, torch.float64, (3, n), "pos")
        b = np.ascontiguousarray(box, dtype=np.float64).reshape(9)
        self._check(self._lib.nep_build_neighbors(
            self._h, n, _ptr(pos), b.ctypes.data_as(C.POINTER(C.c_double)), skin, max_neighbors))
        self.n, self.cap = n, max_neighbors  # cap > 0 marks a built list

    def get_neighbors(self) -> dict:
        dev = torch.device("cuda", self.device)
        n, cap = self.n, self.cap
        out = {
            "cnt_radial": torch.zeros(n, dtype=torch.int32, device=dev),
            "cnt_angular": torch.zeros(n, dtype=torch.int32, device=dev),
            "nbr": torch.zeros((cap, n), dtype=torch.int32, device=dev),
            "img": torch.zeros((cap, n, 3), dtype=torch.int32, device=dev),
            "rev": torch.zeros((cap, n), dtype=torch.int32, device=dev),
        }
        self._check(self._lib.nep_get_neighbors(
            self._h, _ptr(out["cnt_radial"]), _ptr(out["cnt_angular"]), _ptr(out["nbr"]),
            _ptr(out["img"]), _ptr(out["rev"])))
        return out

    def compute(self, pos: torch.Tensor, vel: torch.Tensor | None = None, *, U: bool = True,
                W: bool = True, J: bool | None = None, out: dict | None = None) -> dict:
        n = self.n
        dev = torch.device("cuda", self.device)
        _require(pos, torch.float64, (3, n) if self.cap else None, "pos")
        if vel is not None:
            _require(vel, torch.float64, (3, n), "vel")
        if J is None:
            J = vel is not None
        if out is None:
            out = {"F": torch.empty((3, n), dtype=torch.float32, device=dev),
                   "totals": torch.empty(13, dtype=torch.float64, device=dev)}
            if U:
                out["U"] = torch.empty(n, dtype=torch.float32, device=dev)
            if W:
                out["W"] = torch.empty((9, n), dtype=torch.float32, device=dev)
            if J:
                out["J"] = torch.empty((3, n), dtype=torch.float32, device=dev)
        _require(out["F"], torch.float32, (3, n), "F")
        for key, shape in (("U", (n,)), ("W", (9, n)), ("J", (3, n))):
            if out.get(key) is not None:
                _require(out[key], torch.float32, shape, key)
        if out.get("J") is not None and vel is None:
            raise ValueError("J needs vel")
        if out.get("totals") is not None:
            _require(out["totals"], torch.float64, (13,), "totals")
        self._check(self._lib.nep_compute(
            self._h, _ptr(pos), _ptr(vel), _ptr(out.get("U")), _ptr(out["F"]),
            _ptr(out.get("W")), _ptr(out.get("J")), _ptr(out.get("totals"))))
        return out

    def evaluate_static(self, pos: torch.Tensor, box, out: dict, vel: torch.Tensor | None = None,
                        skin: float = 0.5, max_neighbors: int = 64) -> dict:
        """nep_evaluate_static: list build and one evaluation of the system at
        `pos` in the library's static workspace (no device allocation in the
        call).  `out` holds the caller's output tensors: "F" [3][N] float32
        (required), and optionally "U" [N], "W" [9][N], "J" [3][N] float32 and
        "totals" [13] float64.  The context's own list is left as it was."""
        n = pos.shape[1] if pos.dim() == 2 else 0
        _require(pos, torch.float64, (3, n), "pos")
        if vel is not None:
            _require(vel, torch.float64, (3, n), "vel")
        _require(out["F"], torch.float32, (3, n), "F")
        for key, shape in (("U", (n,)), ("W", (9, n)), ("J", (3, n))):
            if out.get(key) is not None:
                _require(out[key], torch.float32, shape, key)
        if out.get("J") is not None and vel is None:
            raise ValueError("J needs vel")
        if out.get("totals") is not None:
            _require(out["totals"], torch.float64, (13,), "totals")
        b = np.ascontiguousarray(box, dtype=np.float64).reshape(9)
        self._check(self._lib.nep_evaluate_static(
            self._h, n, _ptr(pos), b.ctypes.data_as(C.POINTER(C.c_double)), skin, max_neighbors,
            _ptr(vel), _ptr(out.get("U")), _ptr(out["F"]), _ptr(out.get("W")),
            _ptr(out.get("J")), _ptr(out.get("totals"))))
        return out

    def autotune(self, pos: torch.Tensor, reps: int = 20):
        """Time the pass-1 tile shapes on the current system and keep the
        fastest; returns (lanes per atom chosen, ms per launch of the 2-, 4-
        and 8-lane shapes)."""
        _require(pos, torch.float64, (3, self.n), "pos")
        lanes = C.c_int(0)
        ms = (C.c_double * 3)()
        self._check(self._lib.nep_autotune(self._h, _ptr(pos), reps, C.byref(lanes), ms))
        return lanes.value, list(ms)

    def set_tile(self, lanes: int) -> None:
        self._check(self._lib.nep_set_tile(self._h, lanes))

    def set_species(self, atomic_numbers=None, masses=None) -> None:
        """Atomic numbers [N] (caller order) of a multicomponent system, whose
        pair weights are sqrt(Z_i Z_j), and optional per-atom masses [N] (amu)
        for md_step; None returns to one species (nep_set_species)."""
        if atomic_numbers is None:
            self._check(self._lib.nep_set_species(self._h, 0, None, None))
            return
        Z = np.ascontiguousarray(atomic_numbers, np.int32)
        m = None if masses is None else np.ascontiguousarray(masses, np.float64)
        self._check(self._lib.nep_set_species(self._h, len(Z), Z.ctypes.data,
                                              None if m is None else m.ctypes.data))

    # -- training ------------------------------------------------------------
    def dataset_create(self, ls, max_neighbors: int = 64) -> "Dataset":
        """Copy a labelled set (inputs.LabelledSet layout) to the device."""
        n_atoms = np.ascontiguousarray(ls.n_atoms, np.int32)
        arrays = [n_atoms, np.ascontiguousarray(ls.boxes, np.float64),
                  np.ascontiguousarray(ls.pos, np.float64),
                  np.ascontiguousarray(ls.energy, np.float64),
                  np.ascontiguousarray(ls.forces, np.float64),
                  np.ascontiguousarray(ls.virial, np.float64),
                  np.ascontiguousarray(ls.has_virial, np.uint8)]
        h = C.c_void_p()
        self._check(self._lib.nep_dataset_create(
            self._h, len(n_atoms), *[a.ctypes.data for a in arrays], max_neighbors, C.byref(h)))
        return Dataset(self, h, len(n_atoms), int(n_atoms.sum()))

    def _n_par(self) -> int:
        if self.hyper is None:
            raise NepError(NEP_ESTATE, "no parameters loaded")
        return num_params(self.hyper)

    def eval_population(self, ds: "Dataset", Z: torch.Tensor,
                        lam=(1.0, 1.0, 1.0, 0.05, 0.05), out: torch.Tensor | None = None):
        _require(Z, torch.float32, (None, self._n_par()), "Z")
        n_pop = Z.shape[0]
        if out is None:
            out = torch.empty((n_pop, 6), dtype=torch.float64, device=Z.device)
        _require(out, torch.float64, (n_pop, 6), "out")
        lam = np.ascontiguousarray(lam, np.float64)
        self._check(self._lib.snes_eval_population(self._h, ds._h, n_pop, _ptr(Z),
                                                   lam.ctypes.data, _ptr(out)))
        return out

    def snes_sample(self, m: torch.Tensor, s: torch.Tensor, seed: int, generation: int,
                    n_pop: int, r: torch.Tensor | None = None, Z: torch.Tensor | None = None):
        n_par = m.shape[0]
        _require(m, torch.float32, (n_par,), "m")
        _require(s, torch.float32, (n_par,), "s")
        if r is None:
            r = torch.empty((n_pop, n_par), dtype=torch.float32, device=m.device)
        if Z is None:
            Z = torch.empty((n_pop, n_par), dtype=torch.float32, device=m.device)
        _require(r, torch.float32, (n_pop, n_par), "r")
        _require(Z, torch.float32, (n_pop, n_par), "Z")
        self._check(self._lib.snes_sample(self._h, n_par, n_pop, _ptr(m), _ptr(s), seed,
                                          generation, _ptr(r), _ptr(Z)))
        return r, Z

    def snes_update(self, m: torch.Tensor, s: torch.Tensor, r: torch.Tensor,
                    loss: torch.Tensor, eta_m: float = 0.0, eta_s: float = 0.0) -> None:
        _require(r, torch.float32, (None, None), "r")
        n_pop, n_par = r.shape
        _require(m, torch.float32, (n_par,), "m")
        _require(s, torch.float32, (n_par,), "s")
        _require(loss, torch.float64, (n_pop, 6), "loss")
        self._check(self._lib.snes_update(self._h, n_par, n_pop, _ptr(m), _ptr(s), _ptr(r),
                                          _ptr(loss), eta_m, eta_s))

    def snes_autotune(self, ds: "Dataset", Z: torch.Tensor, reps: int = 3):
        """Time the network-kernel shapes of the population evaluation on this
        dataset and keep the fastest; returns (atoms per wave chosen, ms per
        evaluation of the 16-, 32- and 64-atom shapes)."""
        _require(Z, torch.float32, (None, self._n_par()), "Z")
        atoms = C.c_int(0)
        ms = (C.c_double * 3)()
        self._check(self._lib.snes_autotune(self._h, ds._h, Z.shape[0], _ptr(Z), reps,
                                            C.byref(atoms), ms))
        return atoms.value, list(ms)

    def snes_set_tile(self, ds: "Dataset", atoms: int) -> None:
        self._check(self._lib.snes_set_tile(self._h, ds._h, atoms))

    def snes_run(self, ds: "Dataset", m: torch.Tensor, s: torch.Tensor, seed: int,
                 generation: int, n_gen: int, r: torch.Tensor, Z: torch.Tensor,
                 loss: torch.Tensor, lam=(1.0, 1.0, 1.0, 0.05, 0.05), eta_m: float = 0.0,
                 eta_s: float = 0.0, best: torch.Tensor | None = None):
        """n_gen SNES generations on the device (sample, evaluate, update per
        generation, replayed as a HIP graph); returns best [n_gen][6]."""
        _require(r, torch.float32, (None, None), "r")
        n_pop, n_par = r.shape
        _require(m, torch.float32, (n_par,), "m")
        _require(s, torch.float32, (n_par,), "s")
        _require(Z, torch.float32, (n_pop, n_par), "Z")
        _require(loss, torch.float64, (n_pop, 6), "loss")
        if best is None:
            best = torch.empty((max(n_gen, 1), 6), dtype=torch.float64, device=m.device)
        _require(best, torch.float64, (None, 6), "best", min_rows=n_gen)
        lam = np.ascontiguousarray(lam, np.float64)
        self._check(self._lib.snes_run(self._h, ds._h, n_par, n_pop, _ptr(m), _ptr(s), seed,
                                       generation, n_gen, lam.ctypes.data, eta_m, eta_s, _ptr(r),
                                       _ptr(Z), _ptr(loss), _ptr(best)))
        return best

    def dataset_positions(self, ds: "Dataset") -> torch.Tensor:
        out = torch.empty((3, ds.n_atoms), dtype=torch.float64,
                          device=torch.device("cuda", self.device))
        self._check(self._lib.nep_dataset_get_positions(self._h, ds._h, _ptr(out)))
        return out

    def dataset_set_positions(self, ds: "Dataset", pos: torch.Tensor) -> None:
        _require(pos, torch.float64, (3, ds.n_atoms), "pos")
        self._check(self._lib.nep_dataset_set_positions(self._h, ds._h, _ptr(pos)))

    def dataset_compute(self, ds: "Dataset", z: torch.Tensor, virial: bool = False) -> dict:
        _require(z, torch.float32, (self._n_par(),), "z")
        dev = z.device
        out = {"E": torch.empty(ds.n_struct, dtype=torch.float64, device=dev),
               "F": torch.empty((3, ds.n_atoms), dtype=torch.float32, device=dev)}
        if virial:
            out["W"] = torch.empty((ds.n_struct, 9), dtype=torch.float64, device=dev)
        self._check(self._lib.nep_dataset_compute(self._h, ds._h, _ptr(z), _ptr(out["E"]),
                                                  _ptr(out["F"]), _ptr(out.get("W"))))
        return out

    def dataset_backward(self, ds: "Dataset", z: torch.Tensor, gE=None, gF=None, F=None,
                         want_pos: bool = False) -> dict:
        _require(z, torch.float32, (self._n_par(),), "z")
        dev = z.device
        if gE is not None:
            _require(gE, torch.float64, (ds.n_struct,), "gE")
        if gF is not None:
            _require(gF, torch.float32, (3, ds.n_atoms), "gF")
        if F is not None:
            _require(F, torch.float32, (3, ds.n_atoms), "F")
        elif want_pos:
            raise ValueError("the position gradient needs the forces F of the same z")
        out = {"z": torch.empty(z.shape[0], dtype=torch.float64, device=dev),
               "z32": torch.empty(z.shape[0], dtype=torch.float32, device=dev)}
        if want_pos:
            out["pos"] = torch.empty((3, ds.n_atoms), dtype=torch.float64, device=dev)
        self._check(self._lib.nep_dataset_backward(
            self._h, ds._h, _ptr(z), _ptr(gE), _ptr(gF), _ptr(F), _ptr(out.get("pos")),
            _ptr(out["z"]), _ptr(out["z32"])))
        return out

    def md_step(self, n_steps: int, dt: float, rebuild_every: int, mass: float,
                pos: torch.Tensor, vel: torch.Tensor, thermo: torch.Tensor | None = None,
                W: torch.Tensor | None = None, J: torch.Tensor | None = None,
                fe=None) -> torch.Tensor:
        """Velocity-Verlet steps; with fe = (Fx, Fy, Fz) in 1/Angstrom the HNEMD
        driving force F_e . W_i acts on every atom (nep_md_step_driven)."""
        n = self.n
        _require(pos, torch.float64, (3, n), "pos")
        _require(vel, torch.float64, (3, n), "vel")
        if thermo is None:
            thermo = torch.empty((max(n_steps, 1), 5), dtype=torch.float64, device=pos.device)
        _require(thermo, torch.float64, (None, 5), "thermo", min_rows=n_steps)
        if W is not None:
            _require(W, torch.float32, (9, n), "W")
        if J is not None:
            _require(J, torch.float32, (3, n), "J")
        if fe is None:
            self._check(self._lib.nep_md_step(self._h, n_steps, dt, rebuild_every, mass,
                                              _ptr(pos), _ptr(vel), _ptr(thermo), _ptr(W),
                                              _ptr(J)))
        else:
            f = np.ascontiguousarray(fe, np.float64).reshape(3)
            self._check(self._lib.nep_md_step_driven(
                self._h, n_steps, dt, rebuild_every, mass, f.ctypes.data, _ptr(pos), _ptr(vel),
                _ptr(thermo), _ptr(W), _ptr(J)))
        return thermo


class Dataset:
    """A training set resident on the device (nep_dataset)."""

    def __init__(self, ctx: Context, handle, n_struct: int, n_atoms: int):
        self.ctx, self._h, self.n_struct, self.n_atoms = ctx, handle, n_struct, n_atoms
        self._pos_key = None  # (data pointer, version) of the positions last uploaded

    def pairs(self) -> tuple[int, int]:
        """Ordered pairs inside the radial and inside the angular cutoff."""
        r, a = C.c_longlong(), C.c_longlong()
        self.ctx._check(self.ctx._lib.nep_dataset_pairs(self._h, C.byref(r), C.byref(a)))
        return r.value, a.value

    def close(self):
        if getattr(self, "_h", None):
            self.ctx._lib.nep_dataset_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Correlation:
    """Virial-velocity correlation of an HNEMD run and its spectral
    conductivity (nep_vvcf_*, Sec. II B)."""

    def __init__(self, ctx: Context, n_atoms: int, n_lags: int):
        h = C.c_void_p()
        ctx._check(ctx._lib.nep_vvcf_create(ctx._h, n_atoms, n_lags, C.byref(h)))
        self.ctx, self._h, self.n_atoms, self.n_lags = ctx, h, n_atoms, n_lags

    def sample(self, W: torch.Tensor, vel: torch.Tensor) -> None:
        """W [9][N] float32 and vel [3][N] float64 device tensors (caller order)."""
        _require(W, torch.float32, (9, self.n_atoms), "W")
        _require(vel, torch.float64, (3, self.n_atoms), "vel")
        self.ctx._check(self.ctx._lib.nep_vvcf_sample(self.ctx._h, self._h, _ptr(W), _ptr(vel)))

    def get(self):
        """(K [n_lags, 3] in eV A/fs as numpy, number of samples)."""
        K = np.zeros((self.n_lags, 3))
        n = C.c_longlong()
        self.ctx._check(self.ctx._lib.nep_vvcf_get(self.ctx._h, self._h, K.ctypes.data,
                                                   C.byref(n)))
        return K, n.value

    def spectrum(self, dt_fs: float, temperature: float, volume: float, fe: float, nu_thz):
        """(kappa, kappa_q) [3, len(nu)] in W/(m K THz) at frequencies nu_thz."""
        nu = np.ascontiguousarray(nu_thz, np.float64)
        kap = np.zeros((3, len(nu)))
        kq = np.zeros((3, len(nu)))
        self.ctx._check(self.ctx._lib.nep_vvcf_spectrum(
            self.ctx._h, self._h, dt_fs, temperature, volume, fe, len(nu), nu.ctypes.data,
            kap.ctypes.data, kq.ctypes.data))
        return kap, kq

    def close(self):
        if getattr(self, "_h", None):
            self.ctx._lib.nep_vvcf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class NEPEnergy(torch.autograd.Function):
    """Energies and forces of a dataset's structures as a differentiable function.

    ``E, F = NEPEnergy.apply(pos, z, ctx, ds)`` with pos [3][N] float64 (the
    dataset's atoms) and z [N_par] float32.  E is [S] float64 (structure
    energies), F is [3][N] float32.  The backward pass runs the library's
    hand-written gradient: dG/dz for G = sum gE.E + sum gF.F, and the position
    gradient of the energy part, -gE F.  The position gradient of the force
    part would need second derivatives of U and raises NotImplementedError.
    """

    @staticmethod
    def forward(actx, pos, z, ctx, ds):
        if ds._pos_key != (pos.data_ptr(), pos._version):
            ctx.dataset_set_positions(ds, pos.detach())
            ds._pos_key = (pos.data_ptr(), pos._version)
        out = ctx.dataset_compute(ds, z.detach())
        actx.save_for_backward(z, out["F"])
        actx.nep = (ctx, ds)
        actx.pos_needs_grad = pos.requires_grad
        return out["E"], out["F"]

    @staticmethod
    def backward(actx, gE, gF):
        z, F = actx.saved_tensors
        ctx, ds = actx.nep
        gE = None if gE is None else gE.detach().contiguous()
        gF = None if gF is None else gF.detach().contiguous()
        if gF is not None and actx.pos_needs_grad and bool(gF.abs().max() > 0):
            raise NotImplementedError("position gradient of the force part needs the Hessian")
        g = ctx.dataset_backward(ds, z.detach(), gE, gF, F, want_pos=actx.pos_needs_grad)
        return g.get("pos"), g["z32"], None, None


KERNEL_CLASSES = ("partials", "gather", "neighbors", "integrator")


def set_timing(ctx: "Context", enable: bool) -> None:
    ctx._check(ctx._lib.nep_set_timing(ctx._h, 1 if enable else 0))


def get_timing(ctx: "Context") -> dict:
    """{class: (milliseconds, launches)} since timing was enabled or last read."""
    ms = (C.c_double * 4)()
    cnt = (C.c_int * 4)()
    ctx._check(ctx._lib.nep_get_timing(ctx._h, ms, cnt))
    return {k: (ms[i], cnt[i]) for i, k in enumerate(KERNEL_CLASSES)}


def time_partials(ctx: "Context", pos: torch.Tensor, reps: int = 200) -> float:
    """Mean milliseconds of one descriptor/network/partial-force launch."""
    ms = C.c_double()
    ctx._check(ctx._lib.nep_time_partials(ctx._h, _ptr(pos), reps, C.byref(ms)))
    return ms.value


def soa(x: np.ndarray, device: int = 0) -> torch.Tensor:
    """[N, 3] host array -> [3, N] contiguous float64 device tensor."""
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x, np.float64).T)).to(
        torch.device("cuda", device))


def aos(t: torch.Tensor) -> np.ndarray:
    """[k, N] device tensor -> [N, k] host array."""
    return t.detach().cpu().numpy().T.copy()
