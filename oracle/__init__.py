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
        ("mlp_bf16", ctypes.c_int32),
        ("rcut", ctypes.c_double),
        ("tab_dr", ctypes.c_double),
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
        L.orc_descriptor_jvp.argtypes = [vp, i64, vp, vp, vp, vp, vp]
        L.orc_descriptor_jvp.restype = i32
        L.orc_mlp_second.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp]
        L.orc_mlp_second.restype = i32
        L.orc_train_loss_grad.argtypes = [vp, ctypes.c_int32, vp, vp, vp, vp, vp, vp, dbl, vp, vp, vp, vp]
        L.orc_train_loss_grad.restype = i32
        L.orc_nve.argtypes = [vp, i64, vp, vp, vp, vp, vp, dbl, i32, vp, vp]
        L.orc_nve.restype = i32
        L.orc_nvt.argtypes = [vp, i64, vp, vp, vp, vp, vp, dbl, dbl, dbl, i32, vp, vp, vp, vp]
        L.orc_nvt.restype = i32
        L.orc_pressure.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp]
        L.orc_pressure.restype = i32
        L.orc_radial.argtypes = [vp, dbl, vp, vp]
        L.orc_radial.restype = None
        L.orc_params_per_species.argtypes = [vp]
        L.orc_params_per_species.restype = i32
        L.orc_num_threads.argtypes = []
        L.orc_num_threads.restype = i32
        L.orc_set_num_threads.argtypes = [i32]
        L.orc_set_num_threads.restype = None
        L.orc_round_bf16.argtypes = [i64, vp, vp]
        L.orc_round_bf16.restype = None
        _lib = L
    return _lib


def _p(a: np.ndarray) -> int:
    return a.ctypes.data


class _ModelRef:
    """Keeps the numpy arrays a C model struct points at alive.  bf16: the
    model's BF16 form (MLP matrix-product operands rounded to BF16)."""

    def __init__(self, spec, bf16: bool = False):
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
        m.mlp_bf16 = 1 if bf16 else 0
        m.rcut = spec.rcut
        m.tab_dr = float(getattr(spec, "tab_dr", 0.0))
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


def radial(spec, R: float):
    """(h [K], h' [K]) of the model's radial functions at distance R (direct
    or, when spec.tab_dr > 0, interpolated from the node table)."""
    mref = _ModelRef(spec)
    h = np.empty(spec.n_radial, dtype=np.float64)
    dh = np.empty(spec.n_radial, dtype=np.float64)
    lib().orc_radial(mref.ref, float(R), _p(h), _p(dh))
    return h, dh


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


def energy_forces(spec, pos, species, box, bf16: bool = False):
    """(E, E_atoms [n], F [n,3], W [3,3]) for the whole system (bf16: the
    BF16 form of the MLP)."""
    pos, species, box = _sys_arrays(pos, species, box)
    mref = _ModelRef(spec, bf16)
    n = pos.shape[0]
    E = np.zeros(1, dtype=np.float64)
    Ea = np.empty(n, dtype=np.float64)
    F = np.empty((n, 3), dtype=np.float64)
    W = np.empty(9, dtype=np.float64)
    rc = lib().orc_energy_forces(mref.ref, n, _p(pos), _p(species), _p(box), _p(E), _p(Ea), _p(F), _p(W))
    if rc != 0:
        raise ValueError(f"oracle energy_forces failed ({rc})")
    return float(E[0]), Ea, F, W.reshape(3, 3)


def forces_subset(spec, pos, species, box, sel, bf16: bool = False):
    """(E_atoms [k], F [k,3]) for the selected atoms of a large system."""
    pos, species, box = _sys_arrays(pos, species, box)
    mref = _ModelRef(spec, bf16)
    sel = np.ascontiguousarray(sel, dtype=np.int64)
    Ea = np.empty(sel.shape[0], dtype=np.float64)
    F = np.empty((sel.shape[0], 3), dtype=np.float64)
    rc = lib().orc_forces_subset(mref.ref, pos.shape[0], _p(pos), _p(species), _p(box), sel.shape[0], _p(sel),
                                 _p(Ea), _p(F))
    if rc != 0:
        raise ValueError(f"oracle forces_subset failed ({rc})")
    return Ea, F


def mlp(spec, species, G, bf16: bool = False):
    """(E [n], dE/dG [n,F]) of the per-element MLPs on given descriptors."""
    species = np.ascontiguousarray(species, dtype=np.int32)
    G = np.ascontiguousarray(G, dtype=np.float64)
    mref = _ModelRef(spec, bf16)
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


def set_num_threads(n: int) -> None:
    """OpenMP threads of the following oracle calls."""
    lib().orc_set_num_threads(int(n))


def round_bf16(x) -> np.ndarray:
    """The oracle's BF16 rounding (FP32 first, then 8 significant bits, ties to even)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.empty_like(x)
    lib().orc_round_bf16(x.size, _p(x), _p(out))
    return out


def descriptor_jvp(spec, pos, species, box, r) -> np.ndarray:
    """Descriptor tangents w [n,F] = d/de G(x + e r) along the field r [n,3]."""
    pos, species, box = _sys_arrays(pos, species, box)
    r = np.ascontiguousarray(r, dtype=np.float64)
    mref = _ModelRef(spec)
    w = np.empty((pos.shape[0], spec.n_features), dtype=np.float64)
    rc = lib().orc_descriptor_jvp(mref.ref, pos.shape[0], _p(pos), _p(species), _p(box), _p(r), _p(w))
    if rc != 0:
        raise ValueError(f"oracle descriptor_jvp failed ({rc})")
    return w


def mlp_second(spec, species, G, w, e):
    """(E [n], q [n], grad [S*P]) with q = grad_G E . w and grad = d/dtheta sum(e E - q)."""
    species = np.ascontiguousarray(species, dtype=np.int32)
    G = np.ascontiguousarray(G, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    e = np.ascontiguousarray(e, dtype=np.float64)
    mref = _ModelRef(spec)
    n = G.shape[0]
    E = np.empty(n, dtype=np.float64)
    q = np.empty(n, dtype=np.float64)
    grad = np.empty(spec.params.shape[0], dtype=np.float64)
    rc = lib().orc_mlp_second(mref.ref, n, _p(species), _p(G), _p(w), _p(e), _p(E), _p(q), _p(grad))
    if rc != 0:
        raise ValueError(f"oracle mlp_second failed ({rc})")
    return E, q, grad


def train_loss_grad(spec, sys_off, pos, species, boxes, E_label, F_label, lam: float):
    """(loss, loss_E, loss_F, grad [S*P]) of the force-matching loss over a batch."""
    sys_off = np.ascontiguousarray(sys_off, dtype=np.int64)
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    species = np.ascontiguousarray(species, dtype=np.int32)
    boxes = np.ascontiguousarray(boxes, dtype=np.float64)
    E_label = np.ascontiguousarray(E_label, dtype=np.float64)
    F_label = np.ascontiguousarray(F_label, dtype=np.float64)
    mref = _ModelRef(spec)
    out = np.zeros(3, dtype=np.float64)
    grad = np.empty(spec.params.shape[0], dtype=np.float64)
    rc = lib().orc_train_loss_grad(mref.ref, len(sys_off) - 1, _p(sys_off), _p(pos), _p(species), _p(boxes),
                                   _p(E_label), _p(F_label), float(lam), _p(out[0:]), _p(out[1:]), _p(out[2:]),
                                   _p(grad))
    if rc != 0:
        raise ValueError(f"oracle train_loss_grad failed ({rc})")
    return float(out[0]), float(out[1]), float(out[2]), grad


def nve(spec, pos, vel, species, masses, box, dt: float, n_steps: int):
    """Velocity-Verlet NVE: (pos, vel, epot [n_steps+1], ekin [n_steps+1])."""
    pos = np.array(pos, dtype=np.float64, copy=True)
    vel = np.array(vel, dtype=np.float64, copy=True)
    species = np.ascontiguousarray(species, dtype=np.int32)
    masses = np.ascontiguousarray(masses, dtype=np.float64)
    box = np.ascontiguousarray(box, dtype=np.float64)
    mref = _ModelRef(spec)
    epot = np.empty(n_steps + 1, dtype=np.float64)
    ekin = np.empty(n_steps + 1, dtype=np.float64)
    rc = lib().orc_nve(mref.ref, pos.shape[0], _p(pos), _p(vel), _p(species), _p(masses), _p(box), float(dt),
                       int(n_steps), _p(epot), _p(ekin))
    if rc != 0:
        raise ValueError(f"oracle nve failed ({rc})")
    return pos, vel, epot, ekin


def nvt(spec, pos, vel, species, masses, box, dt: float, T: float, tau_fs: float, n_steps: int, xi_eta=(0.0, 0.0)):
    """Nose-Hoover NVT: (pos, vel, (xi, eta), epot, ekin, conserved), arrays [n_steps+1]."""
    pos = np.array(pos, dtype=np.float64, copy=True)
    vel = np.array(vel, dtype=np.float64, copy=True)
    species = np.ascontiguousarray(species, dtype=np.int32)
    masses = np.ascontiguousarray(masses, dtype=np.float64)
    box = np.ascontiguousarray(box, dtype=np.float64)
    mref = _ModelRef(spec)
    xe = np.array(xi_eta, dtype=np.float64)
    epot = np.empty(n_steps + 1)
    ekin = np.empty(n_steps + 1)
    cons = np.empty(n_steps + 1)
    rc = lib().orc_nvt(mref.ref, pos.shape[0], _p(pos), _p(vel), _p(species), _p(masses), _p(box), float(dt),
                       float(T), float(tau_fs), int(n_steps), _p(xe), _p(epot), _p(ekin), _p(cons))
    if rc != 0:
        raise ValueError(f"oracle nvt failed ({rc})")
    return pos, vel, (float(xe[0]), float(xe[1])), epot, ekin, cons


def pressure(spec, pos, vel, species, masses, box):
    """(p_xx, p_yy, p_zz, P) in GPa."""
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    vel = np.ascontiguousarray(vel, dtype=np.float64)
    species = np.ascontiguousarray(species, dtype=np.int32)
    masses = np.ascontiguousarray(masses, dtype=np.float64)
    box = np.ascontiguousarray(box, dtype=np.float64)
    mref = _ModelRef(spec)
    p4 = np.empty(4)
    rc = lib().orc_pressure(mref.ref, pos.shape[0], _p(pos), _p(vel), _p(species), _p(masses), _p(box), _p(p4))
    if rc != 0:
        raise ValueError(f"oracle pressure failed ({rc})")
    return p4
