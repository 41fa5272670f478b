"""Seeded synthetic inputs shared by the FP64 oracle tests and the HIP path.

This module holds no arithmetic of the potential itself: it only builds
lattices, draws random displacements, species, velocities and MLP weights,
and lays out the radial-basis parameters.  Both sides of every parity test
read the arrays it returns; neither side imports the other.

Workloads stand in for the paper's bulk-metal MD configurations (bcc W at
a = 3.1887 A and 2.8 A, Sec. IV.C and IV.D): Gaussian-displaced perfect
lattices replace thermal snapshots and randomly initialised MLPs replace the
trained potentials (the DFT training set and weights are not available).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

# Fractional basis of the conventional cubic cells and of the orthorhombic
# four-atom hcp cell (a, a*sqrt(3), c).
_BASIS = {
    "fcc": np.array([[0.0, 0.0, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5], [0.5, 0.5, 0.0]]),
    "bcc": np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.5]]),
    "hcp": np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.0], [0.5, 5.0 / 6.0, 0.5], [0.0, 1.0 / 3.0, 0.5]]),
}

ACT_TANH = 0
ACT_SQUAREPLUS = 1


def cell_lengths(kind: str, a: float, c_over_a: float = math.sqrt(8.0 / 3.0)) -> np.ndarray:
    """Edge lengths of one conventional cell of the lattice."""
    if kind in ("fcc", "bcc"):
        return np.array([a, a, a], dtype=np.float64)
    if kind == "hcp":
        return np.array([a, a * math.sqrt(3.0), a * c_over_a], dtype=np.float64)
    raise ValueError(f"unknown lattice {kind!r}")


def lattice(kind: str, a: float, cells: Sequence[int]) -> Tuple[np.ndarray, np.ndarray]:
    """Perfect periodic lattice: positions [N,3] (float64) and box [3].

    Atoms are ordered cell by cell (x fastest), basis atom innermost.
    """
    cells = tuple(int(c) for c in cells)
    basis = _BASIS[kind]
    edge = cell_lengths(kind, a)
    iz, iy, ix = np.meshgrid(np.arange(cells[2]), np.arange(cells[1]), np.arange(cells[0]), indexing="ij")
    origins = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.float64)
    frac = (origins[:, None, :] + basis[None, :, :]).reshape(-1, 3)
    pos = frac * edge[None, :]
    box = edge * np.array(cells, dtype=np.float64)
    return pos, box


@dataclasses.dataclass
class System:
    pos: np.ndarray        # [N,3] float64, wrapped into [0, L)
    species: np.ndarray    # [N] int32
    box: np.ndarray        # [3] float64, orthorhombic, periodic in x, y, z
    masses: np.ndarray     # [S] float64, amu

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])


def make_system(kind: str, a: float, cells: Sequence[int], sigma: float, n_species: int = 1,
                seed: int = 0, masses: Optional[Sequence[float]] = None) -> System:
    """Gaussian-displaced lattice with species split exactly evenly at random.

    Displacements are i.i.d. N(0, sigma^2) per Cartesian component; positions
    are then wrapped into the box.  Species: N//S atoms of each species (the
    remainder goes to the lowest species), assigned by a random permutation.
    """
    rng = np.random.default_rng(seed)
    pos, box = lattice(kind, a, cells)
    n = pos.shape[0]
    if sigma > 0:
        pos = pos + rng.normal(0.0, sigma, size=pos.shape)
    pos = np.mod(pos, box[None, :])
    pos[pos >= box[None, :]] = 0.0
    base = n // n_species
    counts = [base + (1 if s < n % n_species else 0) for s in range(n_species)]
    species = np.repeat(np.arange(n_species, dtype=np.int32), counts)
    species = rng.permutation(species).astype(np.int32)
    if masses is None:
        masses = [183.84] * n_species
    return System(pos=np.ascontiguousarray(pos), species=np.ascontiguousarray(species),
                  box=box.astype(np.float64), masses=np.asarray(masses, dtype=np.float64))


@dataclasses.dataclass
class ModelSpec:
    n_species: int
    n_radial: int              # K
    max_moment: int            # M, 0..3
    hidden: List[int]          # hidden widths, e.g. [64, 64]
    rcut: float
    mu: np.ndarray             # [K]
    eta: np.ndarray            # [K]
    params: np.ndarray         # float64, all species packed (see param_layout)
    activation: int = ACT_TANH
    tab_dr: float = 0.0        # > 0: radial functions interpolated from nodes at most this far apart

    @property
    def n_features(self) -> int:
        return self.n_species * self.n_radial * (self.max_moment + 1)


def param_layout(n_features: int, hidden: Sequence[int]) -> List[Tuple[str, Tuple[int, ...]]]:
    """Per-species parameter blocks, in storage order.

    Layer l maps width w_{l-1} to w_l with W_l stored row-major [w_l][w_{l-1}]
    followed by its bias b_l [w_l]; the last layer maps the last hidden width
    to one output (the atomic energy).
    """
    widths = [n_features] + list(hidden) + [1]
    out = []
    for li in range(len(widths) - 1):
        out.append((f"W{li + 1}", (widths[li + 1], widths[li])))
        out.append((f"b{li + 1}", (widths[li + 1],)))
    return out


def params_per_species(n_features: int, hidden: Sequence[int]) -> int:
    return sum(int(np.prod(s)) for _, s in param_layout(n_features, hidden))


def radial_grid(n_radial: int, rcut: float, r_min: float = 2.0) -> Tuple[np.ndarray, np.ndarray]:
    """Gaussian centres mu_k = r_min + k*delta and widths eta = 1/(2 delta^2)."""
    delta = (rcut - r_min) / n_radial
    mu = r_min + delta * np.arange(n_radial, dtype=np.float64)
    eta = np.full(n_radial, 1.0 / (2.0 * delta * delta), dtype=np.float64)
    return mu, eta


def make_model(n_species: int, n_radial: int, max_moment: int, hidden: Sequence[int], rcut: float,
               seed: int, activation: int = ACT_TANH, weight_scale: float = 1.0,
               r_min: float = 2.0) -> ModelSpec:
    """Random per-element MLPs: W ~ N(0, 1/fan_in) * weight_scale, biases 0.

    Draw order: species 0 layer 1, 2, ..., then species 1, ... (PCG64 stream
    of numpy.default_rng(seed)).
    """
    rng = np.random.default_rng(seed)
    nf = n_species * n_radial * (max_moment + 1)
    layout = param_layout(nf, hidden)
    blocks = []
    for _s in range(n_species):
        for name, shape in layout:
            if name.startswith("W"):
                fan_in = shape[1]
                blocks.append(rng.normal(0.0, 1.0 / math.sqrt(fan_in), size=shape).ravel() * weight_scale)
            else:
                blocks.append(np.zeros(shape, dtype=np.float64).ravel())
    mu, eta = radial_grid(n_radial, rcut, r_min)
    return ModelSpec(n_species=n_species, n_radial=n_radial, max_moment=max_moment, hidden=list(hidden),
                     rcut=float(rcut), mu=mu, eta=eta, params=np.concatenate(blocks).astype(np.float64),
                     activation=activation)


def maxwell_boltzmann(masses_amu: np.ndarray, temperature_k: float, seed: int) -> np.ndarray:
    """Velocities in A/fs with the centre-of-mass velocity removed (no rescale)."""
    kb_ev = 8.617333262e-5
    mvv2e = 103.6427  # amu*(A/fs)^2 -> eV
    rng = np.random.default_rng(seed)
    sd = np.sqrt(kb_ev * temperature_k / (mvv2e * masses_amu))[:, None]
    v = rng.normal(0.0, 1.0, size=(masses_amu.shape[0], 3)) * sd
    p = (masses_amu[:, None] * v).sum(0) / masses_amu.sum()
    return v - p[None, :]


# ---------------------------------------------------------------------------
# Named workloads (sizes of the paper-derived configurations)
# ---------------------------------------------------------------------------

def workload(name: str):
    """(System, ModelSpec, skin) for a named workload.

    oracle32   : 32-atom fcc (2x2x2, a=3.61), sigma 0.1, rc 5.0, K 8, M 3, MLP 64-64.
    fcc32k     : 32,000-atom fcc (20^3, a=3.61), sigma 0.05, rc 6.0, K 8, M 3, MLP 64-64.
    bcc1m      : 1,024,000-atom bcc alloy (80^3, a=3.16, 50/50), sigma 0.08, rc 6.0, K 12, M 3, 128-128.
    bcc4k      : 4,096-atom sub-cell of the bcc alloy workload (8 x 16 x 16 cells, 25.3 x 50.6 x 50.6 A), own seed.
    w_k32[_hp] : bcc W 35^3 (N 85,750), a 3.1887 (2.8 for _hp), rc 6, K 32, M 3, SquarePlus 128-128-128.
    w_k128[_hp]: bcc W 24x24x20 (N 23,040), a 3.1887 (2.8), rc 6, K 128, M 3, SquarePlus 128x4.
    """
    if name == "oracle32":
        sysm = make_system("fcc", 3.61, (2, 2, 2), 0.1, 1, seed=0, masses=[63.546])
        model = make_model(1, 8, 3, [64, 64], 5.0, seed=100)
        return sysm, model, 0.0
    if name == "fcc32k":
        sysm = make_system("fcc", 3.61, (20, 20, 20), 0.05, 1, seed=1, masses=[63.546])
        model = make_model(1, 8, 3, [64, 64], 6.0, seed=101)
        return sysm, model, 0.0
    if name == "bcc1m":
        sysm = make_system("bcc", 3.16, (80, 80, 80), 0.08, 2, seed=2, masses=[183.84, 95.95])
        model = make_model(2, 12, 3, [128, 128], 6.0, seed=102)
        return sysm, model, 0.0
    if name == "bcc4k":
        sysm = make_system("bcc", 3.16, (8, 16, 16), 0.08, 2, seed=20, masses=[183.84, 95.95])
        model = make_model(2, 12, 3, [128, 128], 6.0, seed=102)
        return sysm, model, 0.0
    # Shapes of the paper's own tungsten potentials (Sec. IV: bcc W, one species,
    # K = 32 or 128 radial functions, M = 3, SquarePlus networks), at 0 GPa
    # (a = 3.1887 A) and ~270 GPa (a = 2.8 A); N = 2*35^3 and 2*24*24*20.
    if name in ("w_k32", "w_k32_hp"):
        a = 3.1887 if name == "w_k32" else 2.8
        sysm = make_system("bcc", a, (35, 35, 35), 0.08, 1, seed=30, masses=[183.84])
        model = make_model(1, 32, 3, [128, 128, 128], 6.0, seed=130, activation=ACT_SQUAREPLUS)
        return sysm, model, 0.0
    if name in ("w_k128", "w_k128_hp"):
        a = 3.1887 if name == "w_k128" else 2.8
        sysm = make_system("bcc", a, (24, 24, 20), 0.08, 1, seed=31, masses=[183.84])
        model = make_model(1, 128, 3, [128, 128, 128, 128], 6.0, seed=131, activation=ACT_SQUAREPLUS)
        return sysm, model, 0.0
    if name == "train_teacher":
        model = make_model(1, 8, 3, [64, 64], 5.0, seed=1003)
        return None, model, 0.0
    if name == "train_student":
        model = make_model(1, 8, 3, [64, 64], 5.0, seed=2003)
        return None, model, 0.0
    raise KeyError(name)


# Cell choices of the force-matching batch: single-element fcc (a = 3.61),
# bcc (a = 3.16) and orthorhombic hcp (a = 2.553, c/a = sqrt(8/3)) supercells
# of 108 to 500 atoms, every box edge longer than twice the 5 A cutoff.
TRAIN_CELLS = (
    ("fcc", 3.61, (3, 3, 3)), ("fcc", 3.61, (4, 4, 4)), ("fcc", 3.61, (5, 5, 5)),
    ("bcc", 3.16, (4, 4, 4)), ("bcc", 3.16, (5, 5, 5)), ("bcc", 3.16, (6, 6, 6)),
    ("hcp", 2.553, (4, 3, 3)), ("hcp", 2.553, (6, 4, 5)),
)


@dataclasses.dataclass
class Batch:
    """Ragged batch of periodic systems, concatenated."""
    pos: np.ndarray        # [N,3] float64
    species: np.ndarray    # [N] int32
    sys_off: np.ndarray    # [B+1] int64
    boxes: np.ndarray      # [B,3] float64
    kinds: List[str]

    @property
    def n_systems(self) -> int:
        return int(self.sys_off.shape[0] - 1)

    @property
    def n(self) -> int:
        return int(self.sys_off[-1])

    def system(self, s: int) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
        a, b = int(self.sys_off[s]), int(self.sys_off[s + 1])
        return self.pos[a:b], self.species[a:b], self.boxes[s]


def train_batch(n_cells: int = 64, seed: int = 3, sigma: float = 0.15,
                cells: Sequence[Tuple[str, float, Tuple[int, int, int]]] = TRAIN_CELLS) -> Batch:
    """n_cells systems, each a uniformly drawn entry of `cells` with its own
    Gaussian displacements (one species)."""
    rng = np.random.default_rng(seed)
    pos, sps, offs, boxes, kinds = [], [], [0], [], []
    for c in range(n_cells):
        kind, a, cl = cells[int(rng.integers(0, len(cells)))]
        s = make_system(kind, a, cl, sigma, 1, seed=seed * 1000 + c)
        pos.append(s.pos)
        sps.append(s.species)
        offs.append(offs[-1] + s.n)
        boxes.append(s.box)
        kinds.append(f"{kind}{cl[0]}x{cl[1]}x{cl[2]}")
    return Batch(pos=np.ascontiguousarray(np.concatenate(pos)), species=np.concatenate(sps).astype(np.int32),
                 sys_off=np.asarray(offs, dtype=np.int64), boxes=np.asarray(boxes, dtype=np.float64), kinds=kinds)


def cluster_cut(s: System, centre: int, n_sample: int, reach: float):
    """A non-periodic piece of a periodic system for sampled comparisons.

    The `n_sample` atoms nearest to atom `centre` (minimum image) form the
    sample; every atom within `reach` of the centre's sample sphere (so within
    `reach` of each sampled atom) is kept, unwrapped around the centre, in a box
    wide enough that no periodic image of the piece comes within reach of it.
    With reach >= 2 rcut the atomic energies and forces of the sampled atoms are
    those of the periodic system.  Returns (piece, sample indices in s, sample
    indices in the piece).  Requires the box edges to exceed twice the piece's
    radius (the minimum-image step)."""
    d = s.pos - s.pos[centre]
    d -= s.box[None, :] * np.round(d / s.box[None, :])
    r = np.sqrt((d * d).sum(1))
    order = np.argsort(r, kind="stable")
    sample = np.sort(order[:n_sample])
    r_s = float(r[sample].max())
    radius = r_s + reach
    if np.any(2.0 * radius >= s.box):
        raise ValueError("piece wider than half the box")
    keep = np.nonzero(r <= radius)[0]
    L = 2.0 * radius + reach + 1.0
    piece = System(pos=d[keep] + L / 2.0, species=s.species[keep].copy(), box=np.array([L, L, L]),
                   masses=s.masses)
    where = np.searchsorted(keep, sample)
    return piece, sample, where
