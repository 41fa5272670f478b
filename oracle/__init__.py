"""ctypes front-end of the FP64 CPU oracle (oracle/tmd_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of bench.py, never by the product package.  Every function
here is argument marshalling; the arithmetic is in tmd_oracle.c.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

from . import build as _build

_lib = None

MAXL = 8


class OrcModel(ctypes.Structure):
    _fields_ = [
        ("n_species", ctypes.c_int32),
        ("n_radial", ctypes.c_int32),
        ("max_moment", ctypes.c_int32),
        ("n_hidden", ctypes.c_int32),
        ("hidden", ctypes.c_int32 * MAXL),
        ("activation", ctypes.c_int32),
        ("pad_", ctypes.c_int32),
        ("rcut", ctypes.c_double),
        ("mu", ctypes.c_void_p),
        ("eta", ctypes.c_void_p),
        ("params", ctypes.c_void_p),
    ]


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build(force=True)
        L = ctypes.CDLL(path)
        i64, i32, vp, dbl = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p, ctypes.c_double
        L.orc_neighbors.argtypes = [i64, vp, vp, vp, dbl, i32, vp, vp, vp]
        L.orc_neighbors.restype = i32
        L.orc_atom_neighbors.argtypes = [i64, i64, vp, vp, vp, dbl, i32, vp, vp, vp]
        L.orc_atom_neighbors.restype = i32
        L.orc_descriptors.argtypes = [vp, i64, vp, vp, vp, i64, vp, vp]
        L.orc_descriptors.restype = i32
        L.orc_energy_forces.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp]
        L.orc_energy_forces.restype = i32
        L.orc_forces_subset.argtypes = [vp, i64, vp, vp, vp, i64, vp, vp, vp]
        L.orc_forces_subset.restype = i32
        L.orc_mlp.argtypes = [vp, i64, vp, vp, vp, vp]
        L.orc_mlp.restype = i32
        L.orc_wrap_positions.argtypes = [i64, vp, vp, vp]
        L.orc_wrap_positions.restype = None
        L.orc_neumaier_sum.argtypes = [i64, vp]
        L.orc_neumaier_sum.restype = dbl
        L.orc_num_threads.argtypes = []
        L.orc_num_threads.restype = i32
        _lib = L
    return _lib


def _p(a: np.ndarray) -> int:
    return a.ctypes.data


class _ModelRef:
    """Keeps the numpy arrays a C model struct points at alive."""

    def __init__(self, spec):
        self.mu = np.ascontiguousarray(spec.mu, dtype=np.float64)
        self.eta = np.ascontiguousarray(spec.eta, dtype=np.float64)
        self.params = np.ascontiguousarray(spec.params, dtype=np.float64)
        m = OrcModel()
        m.n_species = spec.n_species
        m.n_radial = spec.n_radial
        m.max_moment = spec.max_moment
        m.n_hidden = len(spec.hidden)
        for q, h in enumerate(spec.hidden):
            m.hidden[q] = h
        m.activation = spec.activation
        m.rcut = spec.rcut
        m.mu = _p(self.mu)
        m.eta = _p(self.eta)
        m.params = _p(self.params)
        self.struct = m

    @property
    def ref(self):
        return ctypes.byref(self.struct)


def _sys_arrays(pos, species, box):
    return (np.ascontiguousarray(pos, dtype=np.float64), np.ascontiguousarray(species, dtype=np.int32),
            np.ascontiguousarray(box, dtype=np.float64))


def wrap_positions(pos, box) -> np.ndarray:
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    box = np.ascontiguousarray(box, dtype=np.float64)
    out = np.empty_like(pos)
    lib().orc_wrap_positions(pos.shape[0], _p(pos), _p(box), _p(out))
    return out


def neighbors(pos, species, box, rlist: float, cap: int = 256):
    """Canonical brute-force list: (nbr [n,cap] (-1 pad), img [n,cap,3], cnt [n])."""
    pos, species, box = _sys_arrays(pos, species, box)
    n = pos.shape[0]
    while True:
        nbr = np.empty((n, cap), dtype=np.int32)
        img = np.empty((n, cap, 3), dtype=np.int32)
        cnt = np.empty(n, dtype=np.int32)
        mx = lib().orc_neighbors(n, _p(pos), _p(species), _p(box), float(rlist), cap, _p(nbr), _p(img), _p(cnt))
        if mx <= cap:
            return nbr, img, cnt
        cap = mx


def atom_neighbors(i: int, pos, species, box, rlist: float, cap: int = 4096):
    """(j [c], img [c,3], D [c,3]) of one atom in canonical order."""
    pos, species, box = _sys_arrays(pos, species, box)
    js = np.empty(cap, dtype=np.int32)
    imgs = np.empty((cap, 3), dtype=np.int32)
    ds = np.empty((cap, 3), dtype=np.float64)
    c = lib().orc_atom_neighbors(int(i), pos.shape[0], _p(pos), _p(species), _p(box), float(rlist), cap,
                                 _p(js), _p(imgs), _p(ds))
    if c > cap:
        return atom_neighbors(i, pos, species, box, rlist, cap=c)
    return js[:c].copy(), imgs[:c].copy(), ds[:c].copy()


def descriptors(spec, pos, species, box, sel: Optional[np.ndarray] = None) -> np.ndarray:
    pos, species, box = _sys_arrays(pos, species, box)
    mref = _ModelRef(spec)
    n = pos.shape[0]
    if sel is not None:
        sel = np.ascontiguousarray(sel, dtype=np.int64)
        nsel = sel.shape[0]
    else:
        nsel = n
    G = np.empty((nsel, spec.n_features), dtype=np.float64)
    rc = lib().orc_descriptors(mref.ref, n, _p(pos), _p(species), _p(box), nsel,
                               _p(sel) if sel is not None else None, _p(G))
    if rc != 0:
        raise ValueError(f"oracle descriptors failed ({rc})")
    return G


def energy_forces(spec, pos, species, box):
    """(E, E_atoms [n], F [n,3], W [3,3]) for the whole system."""
    pos, species, box = _sys_arrays(pos, species, box)
    mref = _ModelRef(spec)
    n = pos.shape[0]
    E = np.zeros(1, dtype=np.float64)
    Ea = np.empty(n, dtype=np.float64)
    F = np.empty((n, 3), dtype=np.float64)
    W = np.empty(9, dtype=np.float64)
    rc = lib().orc_energy_forces(mref.ref, n, _p(pos), _p(species), _p(box), _p(E), _p(Ea), _p(F), _p(W))
    if rc != 0:
        raise ValueError(f"oracle energy_forces failed ({rc})")
    return float(E[0]), Ea, F, W.reshape(3, 3)


def forces_subset(spec, pos, species, box, sel):
    """(E_atoms [k], F [k,3]) for the selected atoms of a large system."""
    pos, species, box = _sys_arrays(pos, species, box)
    mref = _ModelRef(spec)
    sel = np.ascontiguousarray(sel, dtype=np.int64)
    Ea = np.empty(sel.shape[0], dtype=np.float64)
    F = np.empty((sel.shape[0], 3), dtype=np.float64)
    rc = lib().orc_forces_subset(mref.ref, pos.shape[0], _p(pos), _p(species), _p(box), sel.shape[0], _p(sel),
                                 _p(Ea), _p(F))
    if rc != 0:
        raise ValueError(f"oracle forces_subset failed ({rc})")
    return Ea, F


def mlp(spec, species, G):
    """(E [n], dE/dG [n,F]) of the per-element MLPs on given descriptors."""
    species = np.ascontiguousarray(species, dtype=np.int32)
    G = np.ascontiguousarray(G, dtype=np.float64)
    mref = _ModelRef(spec)
    n = G.shape[0]
    E = np.empty(n, dtype=np.float64)
    dG = np.empty_like(G)
    rc = lib().orc_mlp(mref.ref, n, _p(species), _p(G), _p(E), _p(dG))
    if rc != 0:
        raise ValueError(f"oracle mlp failed ({rc})")
    return E, dG


def neumaier_sum(x) -> float:
    x = np.ascontiguousarray(x, dtype=np.float64)
    return float(lib().orc_neumaier_sum(x.shape[0], _p(x)))


def num_threads() -> int:
    return int(lib().orc_num_threads())
