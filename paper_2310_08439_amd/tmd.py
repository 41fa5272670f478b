"""ctypes binding of libtmd.so (include/tmd.h).

Argument marshalling only: torch tensors supply device memory and the HIP
stream; every step of the computation runs in the library's HIP kernels.
The library must have been built (paper_2310_08439_amd/build.py); importing
this module on a machine without it raises instead of falling back to
anything else.
"""
from __future__ import annotations

import ctypes
import weakref
import math
import os
from typing import Optional, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtmd.so")

TMD_OK = 0
STATUS_NAMES = {0: "OK", 1: "INVALID_ARGUMENT", 2: "CAPACITY", 3: "OUT_OF_MEMORY", 4: "DEVICE",
                5: "NUMERICAL", 6: "NOT_READY", 7: "REJECTED"}
TMD_ERR_CAPACITY = 2
FP32 = 0
BF16_MLP = 1
MAX_HIDDEN = 4

# Every exported symbol of include/tmd.h, checked by the CPU test-suite.
EXPORTS = (
    "tmd_context_create", "tmd_context_destroy", "tmd_context_set_stream", "tmd_last_error",
    "tmd_model_create", "tmd_model_set_params", "tmd_model_set_precision", "tmd_model_params_per_species",
    "tmd_model_n_features", "tmd_model_destroy",
    "tmd_nlist_create", "tmd_nlist_destroy", "tmd_build_neighbors", "tmd_nlist_export", "tmd_nlist_capacity",
    "tmd_nlist_stats",
    "tmd_descriptors", "tmd_energy_forces", "tmd_energy_forces_async", "tmd_energy_forces_noalloc",
    "tmd_noalloc_scratch_bytes", "tmd_energy_forces_batch",
    "tmd_profile_enable", "tmd_profile_reset", "tmd_profile_read",
    "tmd_model_get_params", "tmd_batch_create", "tmd_batch_destroy", "tmd_train_step", "tmd_batch_read",
    "tmd_serve_create", "tmd_serve_add_system", "tmd_serve_submit", "tmd_serve_poll", "tmd_serve_wait",
    "tmd_serve_fetch", "tmd_serve_release", "tmd_serve_read_system", "tmd_serve_memory", "tmd_serve_system_memory",
    "tmd_serve_last_error",
    "tmd_serve_destroy",
    "tmd_md_create", "tmd_md_run", "tmd_md_read", "tmd_md_thermostat_state", "tmd_md_destroy",
    "tmd_model_tabulate", "tmd_model_tab_spacing",
)
ENSEMBLE_NVE = 0
ENSEMBLE_NVT_NOSE_HOOVER = 1
TMD_ERR_NOT_READY = 6
REQ_ENERGY_FORCES = 0
REQ_MD = 1

OPT_ADAM = 0
OPT_SGD = 1
BATCH_G, BATCH_ENERGY, BATCH_FORCES, BATCH_RESIDUAL, BATCH_TANGENT = 0, 1, 2, 3, 4


class TMDError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"tmd status {STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
        self.message = message


class SystemView(ctypes.Structure):
    _fields_ = [("n_atoms", ctypes.c_int64), ("pos", ctypes.c_void_p), ("species", ctypes.c_void_p),
                ("box", ctypes.c_double * 3)]


class ModelSpecC(ctypes.Structure):
    _fields_ = [("n_species", ctypes.c_int32), ("n_radial", ctypes.c_int32), ("max_moment", ctypes.c_int32),
                ("n_hidden", ctypes.c_int32), ("hidden", ctypes.c_int32 * MAX_HIDDEN),
                ("activation", ctypes.c_int32), ("reserved", ctypes.c_int32), ("rcut", ctypes.c_double),
                ("mu", ctypes.c_void_p), ("eta", ctypes.c_void_p)]


class TrainOpts(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.c_double), ("lr", ctypes.c_double), ("beta1", ctypes.c_double),
                ("beta2", ctypes.c_double), ("eps", ctypes.c_double), ("optimizer", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class MDOpts(ctypes.Structure):
    _fields_ = [("dt_fs", ctypes.c_double), ("temperature_K", ctypes.c_double), ("tau_fs", ctypes.c_double),
                ("skin", ctypes.c_double), ("ensemble", ctypes.c_int32), ("rebuild_every", ctypes.c_int32)]


class Thermo(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("time_fs", ctypes.c_double), ("epot", ctypes.c_double),
                ("ekin", ctypes.c_double), ("etotal", ctypes.c_double), ("temperature_K", ctypes.c_double),
                ("pressure_GPa", ctypes.c_double), ("pxx_GPa", ctypes.c_double), ("pyy_GPa", ctypes.c_double),
                ("pzz_GPa", ctypes.c_double), ("volume_A3", ctypes.c_double), ("conserved", ctypes.c_double),
                ("xi", ctypes.c_double), ("rebuilds", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "reserved"}


class ServeOpts(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_int64), ("max_slots", ctypes.c_int32), ("device", ctypes.c_int32),
                ("max_atoms", ctypes.c_int64), ("skin", ctypes.c_double), ("capacity", ctypes.c_int32),
                ("batch_atoms", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("system_id", ctypes.c_int64), ("kind", ctypes.c_int32), ("n_steps", ctypes.c_int32),
                ("dt_fs", ctypes.c_double), ("velocities", ctypes.c_void_p)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("kind", ctypes.c_int32), ("system_id", ctypes.c_int64),
                ("n_atoms", ctypes.c_int64), ("n_steps", ctypes.c_int32), ("rebuilds", ctypes.c_int32),
                ("energy", ctypes.c_double), ("kinetic", ctypes.c_double), ("virial", ctypes.c_double * 6),
                ("t_submit", ctypes.c_double), ("t_start", ctypes.c_double), ("t_done", ctypes.c_double),
                ("batch_size", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {"status": self.status, "kind": self.kind, "system_id": self.system_id, "n_atoms": self.n_atoms,
                "n_steps": self.n_steps, "rebuilds": self.rebuilds, "energy": self.energy, "kinetic": self.kinetic,
                "virial": list(self.virial), "t_submit": self.t_submit, "t_start": self.t_start,
                "t_done": self.t_done, "batch_size": self.batch_size}


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libtmd.so; raises FileNotFoundError when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} is missing: run paper_2310_08439_amd/build.py (hipcc, gfx950)")
    # torch first: the library then binds to the HIP runtime torch has loaded
    # (one runtime per process; loading ours first leaves torch a second one)
    _torch()
    L = ctypes.CDLL(path)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    L.tmd_context_create.argtypes = [ctypes.c_int, vp, P(vp)]
    L.tmd_context_destroy.argtypes = [vp]
    L.tmd_context_destroy.restype = None
    L.tmd_context_set_stream.argtypes = [vp, vp]
    L.tmd_last_error.argtypes = [vp]
    L.tmd_last_error.restype = ctypes.c_char_p
    L.tmd_model_create.argtypes = [vp, P(ModelSpecC), vp, P(vp)]
    L.tmd_model_set_params.argtypes = [vp, vp]
    L.tmd_model_set_precision.argtypes = [vp, ctypes.c_int]
    L.tmd_model_params_per_species.argtypes = [vp]
    L.tmd_model_params_per_species.restype = i64
    L.tmd_model_n_features.argtypes = [vp]
    L.tmd_model_n_features.restype = i32
    L.tmd_model_destroy.argtypes = [vp]
    L.tmd_model_destroy.restype = None
    L.tmd_model_tabulate.argtypes = [vp, dbl]
    L.tmd_model_tab_spacing.argtypes = [vp]
    L.tmd_model_tab_spacing.restype = dbl
    L.tmd_nlist_create.argtypes = [vp, i64, i32, i32, P(vp)]
    L.tmd_nlist_destroy.argtypes = [vp]
    L.tmd_nlist_destroy.restype = None
    L.tmd_build_neighbors.argtypes = [vp, P(SystemView), dbl, dbl, vp, P(i32)]
    L.tmd_nlist_export.argtypes = [vp, vp, vp, vp, vp]
    L.tmd_nlist_capacity.argtypes = [vp]
    L.tmd_nlist_capacity.restype = i32
    L.tmd_nlist_stats.argtypes = [vp, vp, P(i64), P(i32)]
    L.tmd_descriptors.argtypes = [vp, vp, P(SystemView), vp, vp]
    L.tmd_energy_forces.argtypes = [vp, vp, P(SystemView), vp, P(dbl), vp, vp, vp]
    L.tmd_energy_forces_async.argtypes = [vp, vp, P(SystemView), vp, vp, vp, vp]
    L.tmd_energy_forces_noalloc.argtypes = [vp, vp, P(SystemView), vp, vp, vp, vp]
    L.tmd_noalloc_scratch_bytes.argtypes = []
    L.tmd_energy_forces_batch.argtypes = [vp, vp, i32, P(SystemView), P(vp), vp, P(vp)]
    L.tmd_noalloc_scratch_bytes.restype = i64
    L.tmd_profile_enable.argtypes = [vp, ctypes.c_int]
    L.tmd_profile_reset.argtypes = [vp]
    L.tmd_profile_read.argtypes = [vp, i32, vp, vp, vp]
    L.tmd_profile_read.restype = i32
    L.tmd_model_get_params.argtypes = [vp, vp]
    L.tmd_batch_create.argtypes = [vp, vp, i32, vp, vp, vp, vp, vp, vp, i32, P(vp)]
    L.tmd_batch_destroy.argtypes = [vp]
    L.tmd_batch_destroy.restype = None
    L.tmd_train_step.argtypes = [vp, vp, vp, P(TrainOpts), vp, vp]
    L.tmd_batch_read.argtypes = [vp, vp, i32, vp]
    L.tmd_md_create.argtypes = [vp, vp, P(SystemView), vp, vp, P(MDOpts), P(vp)]
    L.tmd_md_run.argtypes = [vp, i64, i32, vp, i32, P(i32)]
    L.tmd_md_read.argtypes = [vp, vp, vp]
    L.tmd_md_thermostat_state.argtypes = [vp, vp]
    L.tmd_md_destroy.argtypes = [vp]
    L.tmd_md_destroy.restype = None
    L.tmd_serve_create.argtypes = [vp, P(ServeOpts), P(vp)]
    L.tmd_serve_add_system.argtypes = [vp, i64, vp, vp, vp, vp, P(i64)]
    L.tmd_serve_submit.argtypes = [vp, P(Request), P(ctypes.c_uint64)]
    L.tmd_serve_poll.argtypes = [vp, ctypes.c_uint64, P(Result)]
    L.tmd_serve_wait.argtypes = [vp, ctypes.c_uint64, dbl, P(Result)]
    L.tmd_serve_fetch.argtypes = [vp, ctypes.c_uint64, vp, vp, vp, vp, vp]
    L.tmd_serve_release.argtypes = [vp, ctypes.c_uint64]
    L.tmd_serve_read_system.argtypes = [vp, i64, vp, vp]
    L.tmd_serve_memory.argtypes = [vp, P(i64), P(i64)]
    L.tmd_serve_system_memory.argtypes = [vp, i64, P(i64), P(i64)]
    L.tmd_serve_last_error.argtypes = [vp]
    L.tmd_serve_last_error.restype = ctypes.c_char_p
    L.tmd_serve_destroy.argtypes = [vp]
    L.tmd_serve_destroy.restype = None
    for name in EXPORTS:
        getattr(L, name)
    _lib = L
    return L


def _torch():
    import torch
    return torch


def _ptr(t) -> Optional[int]:
    return None if t is None else int(t.data_ptr())


class Context:
    """A library context bound to one device and the current torch stream."""

    def __init__(self, device: int = 0, stream=None):
        torch = _torch()
        self.lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible to torch")
        self.device = device
        torch.cuda.set_device(device)
        s = stream if stream is not None else torch.cuda.current_stream(device)
        self.stream = s
        h = ctypes.c_void_p()
        st = self.lib.tmd_context_create(device, ctypes.c_void_p(s.cuda_stream), ctypes.byref(h))
        if st != TMD_OK:
            raise TMDError(st, "tmd_context_create failed")
        self.h = h
        # handles made on this context (models, lists, batches, MD runs), closed
        # before the context itself so that none outlives it
        self._children = weakref.WeakSet()

    def adopt(self, obj):
        self._children.add(obj)

    def check(self, st: int, what: str = ""):
        if st != TMD_OK:
            msg = self.lib.tmd_last_error(self.h).decode()
            raise TMDError(st, f"{what}: {msg}" if what else msg)

    def profile(self, on: bool):
        self.check(self.lib.tmd_profile_enable(self.h, 1 if on else 0), "tmd_profile_enable")

    def profile_reset(self):
        self.check(self.lib.tmd_profile_reset(self.h), "tmd_profile_reset")

    def profile_read(self) -> dict:
        """{kernel name: (total ms, launches)} of the launches timed since the last reset."""
        maxk = 64
        names = ctypes.create_string_buffer(32 * maxk)
        tot = (ctypes.c_double * maxk)()
        cnt = (ctypes.c_int64 * maxk)()
        k = self.lib.tmd_profile_read(self.h, maxk, names, tot, cnt)
        out = {}
        for q in range(min(k, maxk)):
            nm = names.raw[32 * q:32 * (q + 1)].split(b"\0", 1)[0].decode()
            out[nm] = (float(tot[q]), int(cnt[q]))
        return out

    def close(self):
        if getattr(self, "h", None):
            for child in list(getattr(self, "_children", ())):
                child.close()
            self.lib.tmd_context_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def system_view(pos, species, box) -> SystemView:
    torch = _torch()
    if pos.dtype != torch.float64 or not pos.is_cuda or not pos.is_contiguous() or pos.dim() != 2 or pos.shape[1] != 3:
        raise ValueError("pos must be a contiguous [n,3] float64 device tensor")
    if species.dtype != torch.int32 or not species.is_cuda or not species.is_contiguous():
        raise ValueError("species must be a contiguous int32 device tensor")
    v = SystemView()
    v.n_atoms = pos.shape[0]
    v.pos = _ptr(pos)
    v.species = _ptr(species)
    for a in range(3):
        v.box[a] = float(box[a])
    return v


class Model:
    """Device copy of a model (ModelSpec from paper_2310_08439_amd.inputs)."""

    def __init__(self, ctx: Context, spec, precision: int = FP32):
        self.ctx = ctx
        ctx.adopt(self)
        self.spec = spec
        c = ModelSpecC()
        c.n_species = spec.n_species
        c.n_radial = spec.n_radial
        c.max_moment = spec.max_moment
        c.n_hidden = len(spec.hidden)
        for q, h in enumerate(spec.hidden):
            c.hidden[q] = h
        c.activation = spec.activation
        c.rcut = spec.rcut
        self._mu = np.ascontiguousarray(spec.mu, dtype=np.float64)
        self._eta = np.ascontiguousarray(spec.eta, dtype=np.float64)
        c.mu = self._mu.ctypes.data
        c.eta = self._eta.ctypes.data
        params = np.ascontiguousarray(spec.params, dtype=np.float32)
        h = ctypes.c_void_p()
        ctx.check(ctx.lib.tmd_model_create(ctx.h, ctypes.byref(c), params.ctypes.data, ctypes.byref(h)),
                  "tmd_model_create")
        self.h = h
        self.set_precision(precision)
        if getattr(spec, "tab_dr", 0.0) > 0.0:
            self.tabulate(spec.tab_dr)

    def tabulate(self, dr: float) -> float:
        """Interpolate the radial functions from a node table of spacing at
        most dr (0: direct evaluation); returns the spacing in use."""
        self.ctx.check(self.ctx.lib.tmd_model_tabulate(self.h, ctypes.c_double(dr)), "tmd_model_tabulate")
        return self.tab_spacing

    @property
    def tab_spacing(self) -> float:
        return float(self.ctx.lib.tmd_model_tab_spacing(self.h))

    @property
    def n_features(self) -> int:
        return int(self.ctx.lib.tmd_model_n_features(self.h))

    def set_precision(self, precision: int):
        self.ctx.check(self.ctx.lib.tmd_model_set_precision(self.h, int(precision)), "tmd_model_set_precision")
        self.precision = precision

    def set_params(self, params: np.ndarray):
        p = np.ascontiguousarray(params, dtype=np.float32)
        self.ctx.check(self.ctx.lib.tmd_model_set_params(self.h, p.ctypes.data), "tmd_model_set_params")

    @property
    def n_params(self) -> int:
        return int(self.ctx.lib.tmd_model_params_per_species(self.h)) * self.spec.n_species

    def get_params(self) -> np.ndarray:
        """Current weights (host float32, tmd_model_create layout)."""
        out = np.empty(self.n_params, dtype=np.float32)
        self.ctx.check(self.ctx.lib.tmd_model_get_params(self.h, out.ctypes.data), "tmd_model_get_params")
        return out

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.tmd_model_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def default_capacity(n_atoms: int, box, rlist: float, n_species: int) -> int:
    vol = float(box[0]) * float(box[1]) * float(box[2])
    mean = n_atoms / vol * 4.0 / 3.0 * math.pi * rlist ** 3
    cap = int(mean * (1.0 / n_species + 0.3)) + 16
    return max(16, (cap + 7) // 8 * 8)


class NeighborList:
    def __init__(self, ctx: Context, n_atoms: int, n_species: int, capacity: int):
        self.ctx = ctx
        ctx.adopt(self)
        self.n_atoms = n_atoms
        self.n_species = n_species
        h = ctypes.c_void_p()
        ctx.check(ctx.lib.tmd_nlist_create(ctx.h, n_atoms, n_species, capacity, ctypes.byref(h)), "tmd_nlist_create")
        self.h = h
        self.capacity = int(ctx.lib.tmd_nlist_capacity(h))

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.tmd_nlist_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_neighbors(ctx: Context, pos, species, box, rcut: float, skin: float, nl: NeighborList) -> int:
    """Returns the largest per-species row length; raises TMDError (status CAPACITY) on overflow."""
    v = system_view(pos, species, box)
    need = ctypes.c_int32(0)
    st = ctx.lib.tmd_build_neighbors(ctx.h, ctypes.byref(v), float(rcut), float(skin), nl.h, ctypes.byref(need))
    if st == TMD_ERR_CAPACITY:
        err = TMDError(st, ctx.lib.tmd_last_error(ctx.h).decode())
        err.required = int(need.value)
        raise err
    ctx.check(st, "tmd_build_neighbors")
    return int(need.value)


def export_neighbors(ctx: Context, nl: NeighborList):
    """(nbr [n,S,cap], img [n,S,cap,3], cnt [n,S]) as device int32 tensors, original numbering."""
    torch = _torch()
    n, S, cap = nl.n_atoms, nl.n_species, nl.capacity
    dev = torch.device("cuda", ctx.device)
    nbr = torch.empty((n, S, cap), dtype=torch.int32, device=dev)
    img = torch.empty((n, S, cap, 3), dtype=torch.int32, device=dev)
    cnt = torch.empty((n, S), dtype=torch.int32, device=dev)
    ctx.check(ctx.lib.tmd_nlist_export(ctx.h, nl.h, _ptr(nbr), _ptr(img), _ptr(cnt)), "tmd_nlist_export")
    return nbr, img, cnt


def nlist_stats(ctx: Context, nl: NeighborList) -> Tuple[int, int]:
    """(total list entries, longest per-species row) of the last build."""
    tot = ctypes.c_int64(0)
    mx = ctypes.c_int32(0)
    ctx.check(ctx.lib.tmd_nlist_stats(ctx.h, nl.h, ctypes.byref(tot), ctypes.byref(mx)), "tmd_nlist_stats")
    return int(tot.value), int(mx.value)


def descriptors(ctx: Context, model: Model, pos, species, box, nl: NeighborList):
    torch = _torch()
    v = system_view(pos, species, box)
    G = torch.empty((pos.shape[0], model.n_features), dtype=torch.float32, device=pos.device)
    ctx.check(ctx.lib.tmd_descriptors(ctx.h, model.h, ctypes.byref(v), nl.h, _ptr(G)), "tmd_descriptors")
    return G


def energy_forces(ctx: Context, model: Model, pos, species, box, nl: NeighborList, atom_energy: bool = True,
                  out_forces=None, out_atom_energy=None) -> Tuple[float, object, object, np.ndarray]:
    """(E, E_atoms or None, F [n,3] float32, virial (xx,yy,zz,xy,xz,yz))."""
    torch = _torch()
    v = system_view(pos, species, box)
    n = pos.shape[0]
    F = out_forces if out_forces is not None else torch.empty((n, 3), dtype=torch.float32, device=pos.device)
    Ea = None
    if atom_energy:
        Ea = out_atom_energy if out_atom_energy is not None else torch.empty(n, dtype=torch.float32, device=pos.device)
    E = ctypes.c_double(0.0)
    W = (ctypes.c_double * 6)()
    ctx.check(ctx.lib.tmd_energy_forces(ctx.h, model.h, ctypes.byref(v), nl.h, ctypes.byref(E), _ptr(Ea), _ptr(F),
                                        W), "tmd_energy_forces")
    return float(E.value), Ea, F, np.array(list(W), dtype=np.float64)


def energy_forces_async(ctx: Context, model: Model, pos, species, box, nl: NeighborList, totals7, forces,
                        atom_energy=None):
    v = system_view(pos, species, box)
    ctx.check(ctx.lib.tmd_energy_forces_async(ctx.h, model.h, ctypes.byref(v), nl.h, _ptr(totals7), _ptr(atom_energy),
                                              _ptr(forces)), "tmd_energy_forces_async")


def energy_forces_noalloc(ctx: Context, model: Model, pos, species, box, nl: NeighborList, totals7, forces,
                          atom_energy=None):
    """tmd_energy_forces_noalloc: the evaluation in the library's static scratch (no allocation)."""
    v = system_view(pos, species, box)
    ctx.check(ctx.lib.tmd_energy_forces_noalloc(ctx.h, model.h, ctypes.byref(v), nl.h, _ptr(totals7),
                                                _ptr(atom_energy), _ptr(forces)), "tmd_energy_forces_noalloc")


def energy_forces_batch(ctx: Context, model: Model, systems, lists, totals7, forces) -> None:
    """tmd_energy_forces_batch: systems is a sequence of (pos, species, box),
    lists the matching NeighborLists, totals7 a [n, 7] float64 device tensor,
    forces a sequence of [n_s, 3] float32 device tensors."""
    n = len(systems)
    if len(lists) != n or len(forces) != n:
        raise ValueError("systems, lists and forces must have the same length")
    views = (SystemView * n)(*[system_view(p, s, b) for p, s, b in systems])
    hl = (ctypes.c_void_p * n)(*[nl.h for nl in lists])
    hf = (ctypes.c_void_p * n)(*[_ptr(f) for f in forces])
    ctx.check(ctx.lib.tmd_energy_forces_batch(ctx.h, model.h, n, views, hl, _ptr(totals7), hf),
              "tmd_energy_forces_batch")


def virial_matrix(w6) -> np.ndarray:
    xx, yy, zz, xy, xz, yz = w6
    return np.array([[xx, xy, xz], [xy, yy, yz], [xz, yz, zz]])


class Evaluator:
    """Context + model + neighbour list for one system, regrowing the list on overflow."""

    def __init__(self, spec, n_atoms: int, box, skin: float = 0.0, precision: int = FP32, device: int = 0,
                 capacity: Optional[int] = None, ctx: Optional[Context] = None):
        self.ctx = ctx if ctx is not None else Context(device)
        self.model = Model(self.ctx, spec, precision)
        self.spec = spec
        self.skin = skin
        cap = capacity or default_capacity(n_atoms, box, spec.rcut + skin, spec.n_species)
        self.nl = NeighborList(self.ctx, n_atoms, spec.n_species, cap)

    def build(self, pos, species, box) -> int:
        try:
            return build_neighbors(self.ctx, pos, species, box, self.spec.rcut, self.skin, self.nl)
        except TMDError as e:
            if e.status != TMD_ERR_CAPACITY:
                raise
            need = (e.required + 8 + 7) // 8 * 8
            self.nl.close()
            self.nl = NeighborList(self.ctx, self.nl.n_atoms, self.spec.n_species, need)
            return build_neighbors(self.ctx, pos, species, box, self.spec.rcut, self.skin, self.nl)

    def energy_forces(self, pos, species, box, rebuild: bool = True, atom_energy: bool = True):
        if rebuild:
            self.build(pos, species, box)
        return energy_forces(self.ctx, self.model, pos, species, box, self.nl, atom_energy=atom_energy)

    def descriptors(self, pos, species, box, rebuild: bool = True):
        if rebuild:
            self.build(pos, species, box)
        return descriptors(self.ctx, self.model, pos, species, box, self.nl)


# ---------------------------------------------------------------- training


class Batch:
    """A labelled batch of periodic systems on the device (tmd_batch_create)."""

    def __init__(self, ctx: Context, model: Model, sys_off, pos, species, boxes, energy_labels, force_labels,
                 capacity: int = 0):
        torch = _torch()
        self.ctx = ctx
        ctx.adopt(self)
        self.sys_off = np.ascontiguousarray(sys_off, dtype=np.int64)
        self.boxes = np.ascontiguousarray(boxes, dtype=np.float64).reshape(-1, 3)
        self.energy_labels = np.ascontiguousarray(energy_labels, dtype=np.float64)
        if pos.dtype != torch.float64 or not pos.is_cuda or not pos.is_contiguous():
            raise ValueError("pos must be a contiguous [N,3] float64 device tensor")
        if species.dtype != torch.int32 or not species.is_cuda or not species.is_contiguous():
            raise ValueError("species must be a contiguous int32 device tensor")
        if force_labels.dtype != torch.float32 or not force_labels.is_cuda or not force_labels.is_contiguous():
            raise ValueError("force_labels must be a contiguous [N,3] float32 device tensor")
        self.n = int(self.sys_off[-1])
        self.n_systems = int(self.sys_off.shape[0] - 1)
        self.n_features = model.n_features
        h = ctypes.c_void_p()
        ctx.check(ctx.lib.tmd_batch_create(ctx.h, model.h, self.n_systems, self.sys_off.ctypes.data, _ptr(pos),
                                           _ptr(species), self.boxes.ctypes.data, self.energy_labels.ctypes.data,
                                           _ptr(force_labels), int(capacity), ctypes.byref(h)), "tmd_batch_create")
        self.h = h

    def read(self, field: int):
        """Device float32 copy of an intermediate of the last step (BATCH_* fields)."""
        torch = _torch()
        shape = {BATCH_G: (self.n, self.n_features), BATCH_ENERGY: (self.n,), BATCH_FORCES: (self.n, 3),
                 BATCH_RESIDUAL: (self.n, 3), BATCH_TANGENT: (self.n, self.n_features)}[field]
        out = torch.empty(shape, dtype=torch.float32, device=torch.device("cuda", self.ctx.device))
        self.ctx.check(self.ctx.lib.tmd_batch_read(self.ctx.h, self.h, int(field), _ptr(out)), "tmd_batch_read")
        return out

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.tmd_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def train_step(ctx: Context, model: Model, batch: Batch, lam: float = 0.1, lr: float = 0.0,
               optimizer: int = OPT_ADAM, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8,
               grad=None) -> Tuple[float, float, float]:
    """(loss, energy term, force term) before the update; grad (device float32) receives dL/dtheta."""
    o = TrainOpts()
    o.lambda_ = float(lam)
    o.lr = float(lr)
    o.beta1 = float(beta1)
    o.beta2 = float(beta2)
    o.eps = float(eps)
    o.optimizer = int(optimizer)
    loss = (ctypes.c_double * 3)()
    ctx.check(ctx.lib.tmd_train_step(ctx.h, model.h, batch.h, ctypes.byref(o), loss, _ptr(grad)), "tmd_train_step")
    return float(loss[0]), float(loss[1]), float(loss[2])


# ---------------------------------------------------------------- autograd


def _energy_function():
    torch = _torch()

    class TMDEnergy(torch.autograd.Function):
        """Total energy E(x) (FP64 scalar) whose gradient dE/dx = -F comes from the
        library's hand-written adjoint kernels (the forces of the same call)."""

        @staticmethod
        def forward(fctx, pos, species, box, evaluator, rebuild):
            E, _, F, _ = evaluator.energy_forces(pos.detach().contiguous(), species, box, rebuild=rebuild,
                                                 atom_energy=False)
            fctx.save_for_backward(F)
            return torch.tensor(E, dtype=torch.float64, device=pos.device)

        @staticmethod
        def backward(fctx, grad_e):
            (F,) = fctx.saved_tensors
            return -F.to(torch.float64) * grad_e, None, None, None, None

    return TMDEnergy


_TMDEnergy = None


def energy(pos, species, box, evaluator: "Evaluator", rebuild: bool = True):
    """Differentiable total energy: torch.autograd sees dE/dpos = -forces."""
    global _TMDEnergy
    if _TMDEnergy is None:
        _TMDEnergy = _energy_function()
    return _TMDEnergy.apply(pos, species, box, evaluator, rebuild)


# ---------------------------------------------------------------- serving


class Server:
    """Persistent request loop (tmd_serve_*): resident systems, worker slots with
    their own streams, admission by memory budget."""

    def __init__(self, model: Model, max_slots: int = 8, hbm_budget_bytes: int = 0, max_atoms: int = 0,
                 skin: float = 1.0, device: int = 0, batch_atoms: int = 0):
        self.lib = model.ctx.lib
        self.model = model  # must outlive the server
        o = ServeOpts()
        o.hbm_budget_bytes = int(hbm_budget_bytes)
        o.max_slots = int(max_slots)
        o.device = int(device)
        o.max_atoms = int(max_atoms)
        o.skin = float(skin)
        o.batch_atoms = int(batch_atoms)
        h = ctypes.c_void_p()
        st = self.lib.tmd_serve_create(model.h, ctypes.byref(o), ctypes.byref(h))
        if st != TMD_OK:
            raise TMDError(st, "tmd_serve_create failed")
        self.h = h
        self.n_atoms = {}

    def _check(self, st: int, what: str):
        if st != TMD_OK:
            raise TMDError(st, f"{what}: {self.lib.tmd_serve_last_error(self.h).decode()}")

    def add_system(self, pos, species, box, masses) -> int:
        pos = np.ascontiguousarray(pos, dtype=np.float64)
        species = np.ascontiguousarray(species, dtype=np.int32)
        box = np.ascontiguousarray(box, dtype=np.float64)
        masses = np.ascontiguousarray(masses, dtype=np.float64)
        sid = ctypes.c_int64(0)
        self._check(self.lib.tmd_serve_add_system(self.h, pos.shape[0], pos.ctypes.data, species.ctypes.data,
                                                  box.ctypes.data, masses.ctypes.data, ctypes.byref(sid)),
                    "tmd_serve_add_system")
        self.n_atoms[int(sid.value)] = int(pos.shape[0])
        return int(sid.value)

    def submit(self, system_id: int, kind: int = REQ_ENERGY_FORCES, n_steps: int = 0, dt_fs: float = 1.0,
               velocities: Optional[np.ndarray] = None) -> int:
        r = Request()
        r.system_id = int(system_id)
        r.kind = int(kind)
        r.n_steps = int(n_steps)
        r.dt_fs = float(dt_fs)
        vel = None
        if velocities is not None:
            vel = np.ascontiguousarray(velocities, dtype=np.float64)
            if vel.shape != (self.n_atoms[int(system_id)], 3):
                raise ValueError("velocities must be [n_atoms, 3]")
            r.velocities = vel.ctypes.data
        t = ctypes.c_uint64(0)
        self._check(self.lib.tmd_serve_submit(self.h, ctypes.byref(r), ctypes.byref(t)), "tmd_serve_submit")
        return int(t.value)

    def poll(self, ticket: int) -> Optional[dict]:
        res = Result()
        st = self.lib.tmd_serve_poll(self.h, ticket, ctypes.byref(res))
        if st == TMD_ERR_NOT_READY:
            return None
        self._check(st, "tmd_serve_poll")
        return res.as_dict()

    def wait(self, ticket: int, timeout_s: float = -1.0) -> Optional[dict]:
        res = Result()
        st = self.lib.tmd_serve_wait(self.h, ticket, float(timeout_s), ctypes.byref(res))
        if st == TMD_ERR_NOT_READY:
            return None
        self._check(st, "tmd_serve_wait")
        return res.as_dict()

    def fetch(self, ticket: int, result: dict) -> dict:
        """Host arrays of a finished request: forces, and for MD pos, vel, epot, ekin."""
        n = result["n_atoms"]
        out = {"forces": np.empty((n, 3), dtype=np.float32), "epot": np.empty(result["n_steps"] + 1)}
        ptrs = [out["forces"].ctypes.data, None, None, out["epot"].ctypes.data, None]
        if result["kind"] == REQ_MD:
            out["pos"] = np.empty((n, 3))
            out["vel"] = np.empty((n, 3))
            out["ekin"] = np.empty(result["n_steps"] + 1)
            ptrs[1], ptrs[2], ptrs[4] = out["pos"].ctypes.data, out["vel"].ctypes.data, out["ekin"].ctypes.data
        self._check(self.lib.tmd_serve_fetch(self.h, ticket, *ptrs), "tmd_serve_fetch")
        return out

    def release(self, ticket: int):
        self._check(self.lib.tmd_serve_release(self.h, ticket), "tmd_serve_release")

    def read_system(self, system_id: int):
        n = self.n_atoms[int(system_id)]
        pos = np.empty((n, 3))
        vel = np.empty((n, 3))
        self._check(self.lib.tmd_serve_read_system(self.h, int(system_id), pos.ctypes.data, vel.ctypes.data),
                    "tmd_serve_read_system")
        return pos, vel

    def memory(self) -> Tuple[int, int]:
        a = ctypes.c_int64(0)
        b = ctypes.c_int64(0)
        self._check(self.lib.tmd_serve_memory(self.h, ctypes.byref(a), ctypes.byref(b)), "tmd_serve_memory")
        return int(a.value), int(b.value)

    def system_memory(self, system_id: int) -> Tuple[int, int]:
        """(state bytes, resident list bytes) of one system."""
        a = ctypes.c_int64(0)
        b = ctypes.c_int64(0)
        self._check(self.lib.tmd_serve_system_memory(self.h, system_id, ctypes.byref(a), ctypes.byref(b)),
                    "tmd_serve_system_memory")
        return int(a.value), int(b.value)

    def close(self):
        if getattr(self, "h", None):
            self.lib.tmd_serve_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- molecular dynamics


class MD:
    """Molecular dynamics of one system (tmd_md_*): velocity Verlet, NVE or
    Nose-Hoover NVT, neighbour list on a fixed period or a displacement rule."""

    def __init__(self, ctx: Context, model: Model, pos, species, box, masses, velocities=None, dt_fs: float = 1.0,
                 ensemble: int = ENSEMBLE_NVT_NOSE_HOOVER, temperature_K: float = 300.0, tau_fs: float = 100.0,
                 skin: float = 1.0, rebuild_every: int = 5):
        self.ctx = ctx
        ctx.adopt(self)
        self.model = model  # must outlive the MD handle
        self.n = int(pos.shape[0])
        v = system_view(pos, species, box)
        masses = np.ascontiguousarray(masses, dtype=np.float64)
        o = MDOpts()
        o.dt_fs, o.temperature_K, o.tau_fs, o.skin = float(dt_fs), float(temperature_K), float(tau_fs), float(skin)
        o.ensemble, o.rebuild_every = int(ensemble), int(rebuild_every)
        if velocities is not None:
            torch = _torch()
            if velocities.dtype != torch.float64 or not velocities.is_cuda or not velocities.is_contiguous():
                raise ValueError("velocities must be a contiguous [n,3] float64 device tensor")
        h = ctypes.c_void_p()
        ctx.check(ctx.lib.tmd_md_create(ctx.h, model.h, ctypes.byref(v), masses.ctypes.data, _ptr(velocities),
                                        ctypes.byref(o), ctypes.byref(h)), "tmd_md_create")
        self.h = h

    def run(self, n_steps: int, thermo_every: int = 0) -> list:
        """Advance n_steps; returns the thermo records (dicts) written."""
        cap = (n_steps // thermo_every + 2) if thermo_every > 0 else 0
        buf = (Thermo * max(cap, 1))()
        nt = ctypes.c_int32(0)
        self.ctx.check(self.ctx.lib.tmd_md_run(self.h, int(n_steps), int(thermo_every), buf, cap, ctypes.byref(nt)),
                       "tmd_md_run")
        return [buf[q].as_dict() for q in range(nt.value)]

    def state(self):
        torch = _torch()
        dev = torch.device("cuda", self.ctx.device)
        pos = torch.empty((self.n, 3), dtype=torch.float64, device=dev)
        vel = torch.empty((self.n, 3), dtype=torch.float64, device=dev)
        self.ctx.check(self.ctx.lib.tmd_md_read(self.h, _ptr(pos), _ptr(vel)), "tmd_md_read")
        return pos, vel

    def thermostat(self) -> Tuple[float, float]:
        xe = (ctypes.c_double * 2)()
        self.ctx.check(self.ctx.lib.tmd_md_thermostat_state(self.h, xe), "tmd_md_thermostat_state")
        return float(xe[0]), float(xe[1])

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.tmd_md_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
