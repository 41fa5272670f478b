"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Neighbour lists bit-exact (as sets, counts equal).  Descriptors
|dG| <= 2e-5 (|G_ref| + 1).  Energies, forces and virial: the FP32 and BF16
bars of tests/parity.py (the configuration targets, per-atom and per-component
bars, and the BF16 path against both the FP64 oracle and its BF16 form).
"""
import math
import sys

import numpy as np
import pytest

import oracle
import parity
from paper_2310_08439_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    return _t


@pytest.fixture(scope="module")
def tmd(torch):
    from paper_2310_08439_amd import tmd as _tmd
    _tmd.load_library()
    return _tmd


@pytest.fixture(scope="module")
def ctx(tmd):
    c = tmd.Context(0)
    yield c
    c.close()


def _note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def _dev(torch, s):
    pos = torch.tensor(s.pos, dtype=torch.float64, device="cuda")
    sp = torch.tensor(s.species, dtype=torch.int32, device="cuda")
    return pos, sp


def _gpu_eval(tmd, ctx, spec, s, prec, skin=0.0, capacity=None):
    import torch
    pos, sp = _dev(torch, s)
    ev = tmd.Evaluator(spec, s.n, s.box, skin=skin, precision=prec, ctx=ctx, capacity=capacity)
    E, Ea, F, W = ev.energy_forces(pos, sp, s.box)
    return E, Ea.cpu().numpy().astype(np.float64), F.cpu().numpy().astype(np.float64), W, ev


def _check_ef(E, Ea, F, W, s, spec, prec):
    if prec == 0:
        parity.check_fp32(E, Ea, F, W, s, spec)
    else:
        parity.check_bf16(E, Ea, F, W, s, spec)


# ------------------------------------------------------------------ neighbour lists

def _gpu_pairs(tmd, ctx, nl, species):
    nbr, img, cnt = tmd.export_neighbors(ctx, nl)
    nbr, img, cnt = nbr.cpu().numpy(), img.cpu().numpy(), cnt.cpu().numpy()
    rows = []
    n, S, cap = nbr.shape
    for b in range(S):
        for c in range(cap):
            m = cnt[:, b] > c
            i = np.nonzero(m)[0]
            j = nbr[m, b, c]
            assert np.all(species[j] == b)
            rows.append(np.stack([i, j, img[m, b, c, 0], img[m, b, c, 1], img[m, b, c, 2]], 1))
    keys = np.concatenate(rows) if rows else np.zeros((0, 5), np.int64)
    order = np.lexsort(keys.T[::-1])
    return keys[order], cnt


def _oracle_pairs(s, rlist):
    nbr, img, cnt = oracle.neighbors(s.pos, s.species, s.box, rlist)
    rows = []
    for i in range(s.n):
        c = cnt[i]
        rows.append(np.concatenate([np.full((c, 1), i), nbr[i, :c, None], img[i, :c]], 1))
    keys = np.concatenate(rows)
    order = np.lexsort(keys.T[::-1])
    per = np.zeros((s.n, int(s.species.max()) + 1), np.int64)
    np.add.at(per, (keys[:, 0], s.species[keys[:, 1]]), 1)
    return keys[order], per


NB_CASES = {
    "fcc32_rc5": lambda: (inputs.workload("oracle32")[0], 5.0, 0.0),
    "bcc4k_rc6": lambda: (inputs.workload("bcc4k")[0], 6.0, 0.0),
    "bcc4k_rc6_skin1": lambda: (inputs.workload("bcc4k")[0], 6.0, 1.0),
    "fcc4_tiny_box_rc6": lambda: (inputs.make_system("fcc", 3.61, (1, 1, 1), 0.05, 1, seed=31), 6.0, 0.0),
    "hcp_ortho_rc5": lambda: (inputs.make_system("hcp", 2.553, (3, 2, 2), 0.1, 3, seed=32), 5.0, 0.5),
    "fcc32k_rc6": lambda: (inputs.workload("fcc32k")[0], 6.0, 0.0),
    # cells of ~107 atoms: more than one wave tracks, so the build falls back
    # to the per-atom fill
    "fcc2916_rc10_crowded_cells": lambda: (inputs.make_system("fcc", 3.61, (9, 9, 9), 0.05, 2, seed=33), 10.0, 0.0),
    # one cell of 108 atoms: the per-atom fill with the positions staged in LDS
    "fcc108_one_crowded_cell_rc6": lambda: (inputs.make_system("fcc", 3.61, (3, 3, 3), 0.05, 2, seed=34), 6.0, 0.0),
}


@pytest.mark.parametrize("case", list(NB_CASES))
def test_neighbors_bitexact(tmd, ctx, torch, case):
    s, rc, skin = NB_CASES[case]()
    _note(f"neighbors {case} n={s.n} rc={rc} skin={skin}")
    pos, sp = _dev(torch, s)
    S = int(s.species.max()) + 1
    cap = tmd.default_capacity(s.n, s.box, rc + skin, S)
    nl = tmd.NeighborList(ctx, s.n, S, cap)
    try:
        tmd.build_neighbors(ctx, pos, sp, s.box, rc, skin, nl)
    except tmd.TMDError as e:
        nl = tmd.NeighborList(ctx, s.n, S, e.required)
        tmd.build_neighbors(ctx, pos, sp, s.box, rc, skin, nl)
    got, gcnt = _gpu_pairs(tmd, ctx, nl, s.species)
    want, wcnt = _oracle_pairs(s, rc + skin)
    assert np.array_equal(gcnt, wcnt)
    assert got.shape == want.shape
    assert np.array_equal(got, want)
    pairs, max_row = tmd.nlist_stats(ctx, nl)  # the on-device reduction of the row counts
    assert pairs == int(wcnt.sum()) and max_row == int(wcnt.max())


def test_capacity_overflow_reports_requirement(tmd, ctx, torch):
    s = inputs.workload("oracle32")[0]
    _note("capacity overflow n=32")
    pos, sp = _dev(torch, s)
    nl = tmd.NeighborList(ctx, s.n, 1, 8)
    with pytest.raises(tmd.TMDError) as ei:
        tmd.build_neighbors(ctx, pos, sp, s.box, 5.0, 0.0, nl)
    assert ei.value.status == tmd.TMD_ERR_CAPACITY
    _, _, cnt = oracle.neighbors(s.pos, s.species, s.box, 5.0)
    assert ei.value.required == cnt.max()


@pytest.mark.parametrize("kind", ["nan", "coincident", "species"])
def test_input_errors(tmd, ctx, torch, kind):
    s = inputs.workload("oracle32")[0]
    _note(f"input error {kind}")
    p = s.pos.copy()
    spc = s.species.copy()
    if kind == "nan":
        p[3, 1] = np.nan
    elif kind == "coincident":
        p[5] = p[4]
    else:
        spc[7] = 3
    pos = torch.tensor(p, dtype=torch.float64, device="cuda")
    sp = torch.tensor(spc, dtype=torch.int32, device="cuda")
    nl = tmd.NeighborList(ctx, s.n, 1, 64)
    with pytest.raises(tmd.TMDError) as ei:
        tmd.build_neighbors(ctx, pos, sp, s.box, 5.0, 0.0, nl)
    assert ei.value.status == {"nan": 5, "coincident": 5, "species": 1}[kind]


def test_empty_system_is_rejected(tmd, ctx, torch):
    _note("empty system")
    pos = torch.zeros((0, 3), dtype=torch.float64, device="cuda")
    sp = torch.zeros(0, dtype=torch.int32, device="cuda")
    with pytest.raises(tmd.TMDError) as ei:
        tmd.NeighborList(ctx, 0, 1, 16)
    assert ei.value.status == 1
    nl = tmd.NeighborList(ctx, 4, 1, 16)
    with pytest.raises(tmd.TMDError) as ei:
        tmd.build_neighbors(ctx, pos, sp, [10.0, 10.0, 10.0], 5.0, 0.0, nl)
    assert ei.value.status == 1


@pytest.mark.parametrize("box", [30.0, 3.0])
def test_single_atom(tmd, ctx, torch, box):
    """One atom: in a large box it has no neighbours (G = 0, E = network at 0);
    in a 3 A box only its own periodic images (zero force by symmetry)."""
    _note(f"single atom box {box}")
    spec = inputs.make_model(1, 8, 3, [32], 5.0, seed=57)
    s = inputs.System(pos=np.array([[0.3, 1.1, 2.2]]), species=np.zeros(1, dtype=np.int32),
                      box=np.array([box, box, box]), masses=np.array([63.546]))
    E, Ea, F, W, _ = _gpu_eval(tmd, ctx, spec, s, tmd.FP32)
    Er, _, Fr, Wr = oracle.energy_forces(spec, s.pos, s.species, s.box)
    assert abs(E - Er) <= 1e-5
    assert np.abs(F).max() <= 1e-4 and np.abs(Fr).max() <= 1e-9
    if box == 30.0:
        E0, _ = oracle.mlp(spec, s.species, np.zeros((1, spec.n_features)))
        assert abs(E - E0[0]) <= 1e-5


# ------------------------------------------------------------------ descriptors

@pytest.mark.parametrize("name", ["oracle32", "bcc4k"])
def test_descriptors_parity(tmd, ctx, torch, name):
    s, spec, _ = inputs.workload(name)
    _note(f"descriptors {name} n={s.n}")
    pos, sp = _dev(torch, s)
    ev = tmd.Evaluator(spec, s.n, s.box, ctx=ctx)
    G = ev.descriptors(pos, sp, s.box).cpu().numpy().astype(np.float64)
    Gr = oracle.descriptors(spec, s.pos, s.species, s.box)
    err = np.abs(G - Gr) / (np.abs(Gr) + 1.0)
    print(f"  max scaled G err {err.max():.3e}", flush=True)
    assert err.max() <= 2e-5


@pytest.mark.parametrize("K,M,S", [(4, 0, 1), (8, 1, 2), (12, 2, 3), (16, 3, 1), (24, 3, 2), (32, 3, 1),
                                   (1, 3, 1), (10, 3, 2), (100, 2, 1)])
def test_descriptor_shapes(tmd, ctx, torch, K, M, S):
    s = inputs.make_system("bcc", 3.16, (3, 3, 3), 0.12, S, seed=40 + K)
    spec = inputs.make_model(S, K, M, [32], 5.5, seed=41)
    _note(f"descriptor shape K={K} M={M} S={S} n={s.n}")
    pos, sp = _dev(torch, s)
    ev = tmd.Evaluator(spec, s.n, s.box, ctx=ctx)
    G = ev.descriptors(pos, sp, s.box).cpu().numpy().astype(np.float64)
    Gr = oracle.descriptors(spec, s.pos, s.species, s.box)
    assert (np.abs(G - Gr) / (np.abs(Gr) + 1.0)).max() <= 2e-5


# ------------------------------------------------------------------ energy / forces / virial

@pytest.mark.parametrize("name", ["oracle32", "bcc4k", "fcc32k"])
def test_energy_forces_fp32(tmd, ctx, torch, name):
    s, spec, _ = inputs.workload(name)
    _note(f"energy_forces fp32 {name} n={s.n}")
    E, Ea, F, W, _ = _gpu_eval(tmd, ctx, spec, s, tmd.FP32)
    _check_ef(E, Ea, F, W, s, spec, 0)


@pytest.mark.parametrize("name", ["oracle32", "bcc4k"])
def test_energy_forces_bf16(tmd, ctx, torch, name):
    s, spec, _ = inputs.workload(name)
    _note(f"energy_forces bf16 {name} n={s.n}")
    E, Ea, F, W, _ = _gpu_eval(tmd, ctx, spec, s, tmd.BF16_MLP)
    _check_ef(E, Ea, F, W, s, spec, 1)


@pytest.mark.parametrize("hidden,act,K,M", [([32], 0, 8, 3), ([64, 64, 64], 1, 8, 2), ([128, 128, 128, 128], 0, 4, 3),
                                            ([64], 1, 16, 1)])
@pytest.mark.parametrize("prec", [0, 1])
def test_energy_forces_model_shapes(tmd, ctx, torch, hidden, act, K, M, prec):
    s = inputs.make_system("bcc", 3.16, (3, 3, 3), 0.12, 2, seed=50)
    spec = inputs.make_model(2, K, M, hidden, 5.5, seed=51, activation=act)
    _note(f"energy_forces shapes hidden={hidden} act={act} K={K} M={M} prec={prec}")
    E, Ea, F, W, _ = _gpu_eval(tmd, ctx, spec, s, prec)
    _check_ef(E, Ea, F, W, s, spec, prec)


@pytest.mark.parametrize("S,K,M,hidden", [(1, 1, 3, [16]), (2, 10, 3, [50, 20]), (2, 20, 2, [100]),
                                          (1, 100, 3, [7, 128, 33]), (2, 13, 1, [128, 1])])
@pytest.mark.parametrize("prec", [0, 1])
def test_energy_forces_any_k_and_widths(tmd, ctx, torch, S, K, M, hidden, prec):
    """Any K in 1..128 and any hidden widths in 1..128 per layer (the kernels
    run K rounded up to 4, 6 or 8 times a power of two and one padded width;
    the padding meets zero weights)."""
    s = inputs.make_system("bcc", 3.16, (3, 3, 3), 0.12, S, seed=50)
    spec = inputs.make_model(S, K, M, hidden, 5.5, seed=51)
    _note(f"energy_forces any shape S={S} K={K} M={M} hidden={hidden} prec={prec}")
    E, Ea, F, W, ev = _gpu_eval(tmd, ctx, spec, s, prec)
    assert ev.model.n_features == spec.n_features
    _check_ef(E, Ea, F, W, s, spec, prec)


@pytest.mark.parametrize("prec", [0, 1])
def test_energy_forces_feature_count_not_multiple_of_4(tmd, ctx, torch, prec):
    """F = 3 species x K 6 x (M+1) 3 = 54: descriptor rows are not 16-byte multiples."""
    s = inputs.make_system("bcc", 3.16, (3, 3, 3), 0.12, 3, seed=52)
    spec = inputs.make_model(3, 6, 2, [64, 64], 5.5, seed=53)
    assert spec.n_features % 4 != 0
    _note(f"energy_forces F={spec.n_features} prec={prec}")
    E, Ea, F, W, _ = _gpu_eval(tmd, ctx, spec, s, prec)
    _check_ef(E, Ea, F, W, s, spec, prec)


@pytest.mark.parametrize("grid", ["jittered_mu", "varied_eta"])
def test_energy_forces_non_uniform_radial_grid(tmd, ctx, torch, grid):
    """Radial centres or widths off a uniform grid: the kernels evaluate every
    Gaussian directly instead of by the uniform-grid recurrence."""
    import dataclasses
    s = inputs.make_system("bcc", 3.16, (4, 4, 4), 0.1, 2, seed=54)
    spec = inputs.make_model(2, 12, 3, [64, 64], 6.0, seed=55)
    rng = np.random.default_rng(56)
    if grid == "jittered_mu":
        spec = dataclasses.replace(spec, mu=spec.mu + rng.uniform(-0.05, 0.05, size=spec.mu.shape))
    else:
        spec = dataclasses.replace(spec, eta=spec.eta * rng.uniform(0.8, 1.2, size=spec.eta.shape))
    _note(f"energy_forces non-uniform radial grid ({grid})")
    E, Ea, F, W, _ = _gpu_eval(tmd, ctx, spec, s, tmd.FP32)
    _check_ef(E, Ea, F, W, s, spec, 0)


@pytest.mark.parametrize("K", [8, 12, 16])
@pytest.mark.parametrize("radial", ["uniform", "jittered_mu", "table"])
def test_matrix_core_shapes(tmd, ctx, torch, K, radial):
    """M = 3 with K = 8, 12 and 16 on 6 x 6 x 6 bcc cells with r_c 6 A: three
    list cells per edge, so the list has a work order and the descriptor and
    adjoint run on the matrix cores (K / 4 groups of radial functions per lane).
    Uniform grid (stride-four recurrence), jittered centres (direct Gaussians)
    and the table; G element by element and E, F, virial against the oracle."""
    import dataclasses
    s = inputs.make_system("bcc", 3.16, (6, 6, 6), 0.1, 2, seed=60 + K)
    spec = inputs.make_model(2, K, 3, [64, 64], 6.0, seed=61)
    if radial == "jittered_mu":
        rng = np.random.default_rng(62)
        spec = dataclasses.replace(spec, mu=spec.mu + rng.uniform(-0.05, 0.05, size=spec.mu.shape))
    elif radial == "table":
        spec = dataclasses.replace(spec, tab_dr=0.01)
    _note(f"matrix-core path K={K} M=3 radial={radial} n={s.n}")
    pos, sp = _dev(torch, s)
    ev = tmd.Evaluator(spec, s.n, s.box, ctx=ctx)
    G = ev.descriptors(pos, sp, s.box).cpu().numpy().astype(np.float64)
    Gr = oracle.descriptors(spec, s.pos, s.species, s.box)
    err = np.abs(G - Gr) / (np.abs(Gr) + 1.0)
    print(f"  max scaled G err {err.max():.3e}", flush=True)
    assert err.max() <= 2e-5
    E, Ea, F, W = ev.energy_forces(pos, sp, s.box)
    _check_ef(E, Ea.cpu().numpy().astype(np.float64), F.cpu().numpy().astype(np.float64), W, s, spec, 0)


@pytest.mark.parametrize("S", [1, 3, 4])
def test_matrix_core_species(tmd, ctx, torch, S):
    """The 4x4x1 matrix-core descriptor and adjoint with one, three and four
    species (one P tile, list row and dE/dG slice per neighbour species), K = 12
    on 6 x 6 x 6 bcc cells with species drawn at random; E, F and virial
    against the oracle."""
    s = inputs.make_system("bcc", 3.16, (6, 6, 6), 0.1, S, seed=80 + S)
    spec = inputs.make_model(S, 12, 3, [64, 64], 6.0, seed=81)
    _note(f"matrix-core adjoint, {S} species, K=12 M=3 n={s.n}")
    pos, sp = _dev(torch, s)
    ev = tmd.Evaluator(spec, s.n, s.box, ctx=ctx)
    E, Ea, F, W = ev.energy_forces(pos, sp, s.box)
    _check_ef(E, Ea.cpu().numpy().astype(np.float64), F.cpu().numpy().astype(np.float64), W, s, spec, 0)


@pytest.mark.parametrize("K", [24, 32, 64, 128])
@pytest.mark.parametrize("radial", ["uniform_wide", "uniform", "jittered_mu", "table"])
def test_matrix_core_large_k(tmd, ctx, torch, K, radial):
    """M = 3 with K = 24 .. 128 on 6 x 6 x 6 bcc cells (two species, r_c 6 A,
    three list cells per edge): the 16x16x4 matrix-core adjoint with the
    atom-major P.  Radial functions: a uniform grid of wide Gaussians (eta 2,
    where the stride-four recurrence holds), the default narrow uniform grid
    (direct Gaussians), jittered centres and the table."""
    import dataclasses
    s = inputs.make_system("bcc", 3.1887, (6, 6, 6), 0.08, 2, seed=70 + K, masses=[183.84, 95.95])
    spec = inputs.make_model(2, K, 3, [32], 6.0, seed=71, activation=inputs.ACT_SQUAREPLUS)
    if radial == "uniform_wide":
        spec = dataclasses.replace(spec, eta=np.full(K, 2.0))
    elif radial == "jittered_mu":
        rng = np.random.default_rng(72)
        spec = dataclasses.replace(spec, mu=spec.mu + rng.uniform(-0.02, 0.02, size=spec.mu.shape))
    elif radial == "table":
        spec = dataclasses.replace(spec, tab_dr=0.01)
    _note(f"matrix-core large K={K} radial={radial} n={s.n}")
    E, Ea, F, W, _ = _gpu_eval(tmd, ctx, spec, s, 0)
    _check_ef(E, Ea, F, W, s, spec, 0)


@pytest.mark.parametrize("K,hidden", [(32, [128, 128, 128]), (128, [128, 128, 128, 128])])
@pytest.mark.parametrize("a", [3.1887, 2.8])
@pytest.mark.parametrize("prec", [0, 1])
def test_paper_shaped_tungsten_models(tmd, ctx, torch, K, hidden, a, prec):
    """The paper's potential shapes (one species, K = 32 or 128, M = 3, SquarePlus
    128-wide networks) on a 4^3 bcc W cell at 0 GPa and ~270 GPa lattice constants."""
    s = inputs.make_system("bcc", a, (4, 4, 4), 0.08, 1, seed=58, masses=[183.84])
    spec = inputs.make_model(1, K, 3, hidden, 6.0, seed=59, activation=inputs.ACT_SQUAREPLUS)
    _note(f"paper-shaped K={K} a={a} prec={prec}")
    E, Ea, F, W, _ = _gpu_eval(tmd, ctx, spec, s, prec)
    _check_ef(E, Ea, F, W, s, spec, prec)


def test_ragged_and_absent_species(tmd, ctx, torch):
    """61 atoms (ragged MLP tiles), species 1 of 2 absent, one isolated atom."""
    rng = np.random.default_rng(60)
    pos = rng.uniform(0, 11.0, size=(60, 3))
    pos = np.concatenate([pos, [[30.0, 30.0, 30.0]]])
    box = np.array([40.0, 40.0, 40.0])
    pos[:60] *= 1.0
    # spread the 60 atoms so no two are closer than 1.8 A
    keep = [0]
    for q in range(1, 60):
        if np.min(np.linalg.norm(pos[keep] - pos[q], axis=1)) > 1.8:
            keep.append(q)
    pos = np.concatenate([pos[keep], pos[60:]])
    s = inputs.System(pos=pos, species=np.zeros(len(pos), np.int32), box=box, masses=np.array([63.5, 58.7]))
    spec = inputs.make_model(2, 8, 3, [64, 64], 5.0, seed=61)
    _note(f"ragged n={s.n}")
    E, Ea, F, W, _ = _gpu_eval(tmd, ctx, spec, s, tmd.FP32)
    _check_ef(E, Ea, F, W, s, spec, 0)
    assert np.all(F[-1] == 0.0)


@pytest.mark.parametrize("case", ["tiny_box_wide_stencil", "two_cells_per_edge", "three_cells_per_edge"])
def test_energy_forces_cell_geometries(tmd, ctx, torch, case):
    """Box shapes that exercise the force-scatter variants: an edge shorter than
    the cutoff (stencil wider than 3x3x3, device atomics), and 2 or 3 cells per
    edge (halo cells that are periodic copies of interior cells)."""
    if case == "tiny_box_wide_stencil":
        s = inputs.make_system("fcc", 3.61, (1, 1, 2), 0.08, 1, seed=90)
        spec = inputs.make_model(1, 8, 3, [32], 5.0, seed=91)
    elif case == "two_cells_per_edge":
        s = inputs.make_system("fcc", 3.61, (4, 4, 4), 0.08, 2, seed=92)
        spec = inputs.make_model(2, 8, 3, [64, 64], 6.0, seed=93)
    else:
        s = inputs.make_system("bcc", 3.16, (6, 6, 6), 0.08, 2, seed=94)
        spec = inputs.make_model(2, 12, 3, [64, 64], 5.5, seed=95)
    _note(f"cell geometry {case} n={s.n} box={s.box}")
    E, Ea, F, W, _ = _gpu_eval(tmd, ctx, spec, s, tmd.FP32)
    _check_ef(E, Ea, F, W, s, spec, 0)


def test_energy_forces_crowded_cells(tmd, ctx, torch):
    """r_c = 10 A on fcc: ~107 atoms per cell (per-atom fill fallback) and
    halos too large for the preferred cell block of the adjoint."""
    s = inputs.make_system("fcc", 3.61, (9, 9, 9), 0.05, 2, seed=34)
    spec = inputs.make_model(2, 8, 3, [32, 32], 10.0, seed=35)
    _note(f"crowded cells n={s.n} rc=10")
    E, Ea, F, W, _ = _gpu_eval(tmd, ctx, spec, s, tmd.FP32)
    _check_ef(E, Ea, F, W, s, spec, 0)


def test_skin_entries_contribute_nothing(tmd, ctx, torch):
    s, spec, _ = inputs.workload("oracle32")
    _note("skin 1.5")
    E0, _, F0, W0, _ = _gpu_eval(tmd, ctx, spec, s, tmd.FP32, skin=0.0)
    E1, _, F1, W1, _ = _gpu_eval(tmd, ctx, spec, s, tmd.FP32, skin=1.5)
    assert abs(E0 - E1) <= 1e-9 * abs(E0)
    assert np.abs(F0 - F1).max() <= 1e-5


def test_list_reuse_after_small_moves(tmd, ctx, torch):
    """A list built with a skin stays valid for moves < skin/2 (positions refreshed each call)."""
    s, spec, _ = inputs.workload("oracle32")
    _note("list reuse")
    pos, sp = _dev(torch, s)
    ev = tmd.Evaluator(spec, s.n, s.box, skin=1.0, ctx=ctx)
    ev.build(pos, sp, s.box)
    moved = s.pos + np.random.default_rng(70).uniform(-0.3, 0.3, s.pos.shape)
    pm = torch.tensor(moved, dtype=torch.float64, device="cuda")
    E, Ea, F, W = ev.energy_forces(pm, sp, s.box, rebuild=False)
    s2 = inputs.System(pos=moved, species=s.species, box=s.box, masses=s.masses)
    _check_ef(E, Ea.cpu().numpy().astype(np.float64), F.cpu().numpy().astype(np.float64), W, s2, spec, 0)


@pytest.mark.parametrize("tab_dr", [0.0, 0.01])
def test_pruned_rows_after_moves(tmd, ctx, torch, tab_dr):
    """Skin lists are pruned to the cutoff at the current positions before the
    descriptor and adjoint loops: two species, rows spanning several batches,
    atoms moved by up to 0.3 A since the build, direct and tabulated radial
    functions, against the oracle."""
    import dataclasses
    s = inputs.make_system("bcc", 3.16, (7, 7, 7), 0.06, 2, seed=96)
    spec = dataclasses.replace(inputs.make_model(2, 16, 3, [64, 64], 5.5, seed=97), tab_dr=tab_dr)
    _note(f"pruned rows n={s.n} tab_dr={tab_dr}")
    pos, sp = _dev(torch, s)
    ev = tmd.Evaluator(spec, s.n, s.box, skin=1.2, ctx=ctx)
    ev.build(pos, sp, s.box)
    for it in range(2):
        moved = s.pos + np.random.default_rng(98 + it).uniform(-0.3, 0.3, s.pos.shape)
        pm = torch.tensor(moved, dtype=torch.float64, device="cuda")
        E, Ea, F, W = ev.energy_forces(pm, sp, s.box, rebuild=False)
        s2 = inputs.System(pos=moved, species=s.species, box=s.box, masses=s.masses)
        _check_ef(E, Ea.cpu().numpy().astype(np.float64), F.cpu().numpy().astype(np.float64), W, s2, spec, 0)


def test_forces_match_gpu_energy_differences(tmd, ctx, torch):
    s, spec, _ = inputs.workload("oracle32")
    _note("finite differences of the GPU energy")
    pos, sp = _dev(torch, s)
    ev = tmd.Evaluator(spec, s.n, s.box, ctx=ctx)
    E, _, F, _ = ev.energy_forces(pos, sp, s.box)
    F = F.cpu().numpy()
    h = 2e-3
    for i, x in ((0, 0), (11, 1), (27, 2)):
        vals = []
        for sgn in (1, -1):
            p = s.pos.copy()
            p[i, x] += sgn * h
            pt = torch.tensor(p, dtype=torch.float64, device="cuda")
            vals.append(ev.energy_forces(pt, sp, s.box)[0])
        fd = -(vals[0] - vals[1]) / (2 * h)
        assert abs(fd - F[i, x]) <= 2e-3 * max(1.0, abs(F[i, x])) + 1e-3


def test_repeat_runs(tmd, ctx, torch):
    s, spec, _ = inputs.workload("bcc4k")
    _note("repeat runs bcc4k")
    pos, sp = _dev(torch, s)
    ev = tmd.Evaluator(spec, s.n, s.box, ctx=ctx, precision=tmd.BF16_MLP)
    E1, Ea1, F1, _ = ev.energy_forces(pos, sp, s.box)
    E2, Ea2, F2, _ = ev.energy_forces(pos, sp, s.box)
    assert E1 == E2
    assert torch.equal(Ea1, Ea2)
    assert torch.equal(F1, F2)  # fixed-point force sums: independent of the atomics' order


def test_bcc1m_skin_list_sampled_parity(tmd, ctx, torch):
    """The 1,024,000-atom alloy on a list with a 1 A skin: 7 A cells, whose
    4x4x2- and 4x2x2-cell blocks have halos beyond the LDS budget, so the work
    order takes 3x2x2 blocks.  FP32, 2,000 sampled atoms against the oracle,
    and every atom's energy against the evaluation on the skin-free list (6 A
    cells, 4x4x2 blocks) within the FP32 rounding of the LDS position offsets."""
    s, spec, _ = inputs.workload("bcc1m")
    _note(f"bcc1m n={s.n} fp32, 1 A skin list, sampled atoms vs oracle")
    pos, sp = _dev(torch, s)
    ev0 = tmd.Evaluator(spec, s.n, s.box, ctx=ctx, precision=tmd.FP32)
    E0, Ea0, _, _ = ev0.energy_forces(pos, sp, s.box)
    ev0.model.close()
    ev0.nl.close()
    ev = tmd.Evaluator(spec, s.n, s.box, ctx=ctx, skin=1.0, precision=tmd.FP32)
    E, Ea, F, _ = ev.energy_forces(pos, sp, s.box)
    Ea = Ea.cpu().numpy().astype(np.float64)
    F = F.cpu().numpy().astype(np.float64)
    parity.check_sampled(Ea, F, s, spec, False, seeds=(82,))
    dEa = np.abs(Ea - Ea0.cpu().numpy().astype(np.float64))
    print(f"  skin 1 vs skin 0: |dE|/N={abs(E - E0) / s.n:.3e}  max|dE_i|={dEa.max():.3e}", flush=True)
    assert abs(E - E0) / s.n <= 1e-6 and dEa.max() <= 1e-5
    ev.model.close()
    ev.nl.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_rebuild_bitwise_reproducible_bcc1m(tmd, ctx, torch, prec):
    """Every output bit for bit across list rebuilds at 1,024,000 atoms.  The
    rebuild also remakes the work order; its slots within one row length used
    to be handed out by LDS atomics, and the atoms grouped with one another
    then changed from build to build, which moved ~800 atoms' FP32 energies
    and ~28,000 atoms' forces at rounding level."""
    s, spec, _ = inputs.workload("bcc1m")
    _note(f"bcc1m rebuild reproducibility prec={prec}")
    pos, sp = _dev(torch, s)
    ev = tmd.Evaluator(spec, s.n, s.box, ctx=ctx, precision=tmd.FP32 if prec == 0 else tmd.BF16_MLP)
    runs = [ev.energy_forces(pos, sp, s.box, rebuild=True) for _ in range(3)]
    E0, Ea0, F0, W0 = runs[0]
    for E, Ea, F, W in runs[1:]:
        assert E == E0
        assert torch.equal(Ea, Ea0)
        assert torch.equal(F, F0)
        assert np.array_equal(np.asarray(W), np.asarray(W0))
    ev.model.close()
    ev.nl.close()


@pytest.mark.parametrize("hidden", [[64, 64], [64, 64, 64], [128]])
def test_bf16_resident_weight_mlp(tmd, ctx, torch, hidden):
    """Systems of 64k+ atoms run the BF16 network with every weight resident in
    LDS (one workgroup per CU looping over 16-atom tiles): 2,000 sampled atoms
    against the oracle and its BF16 form, and the whole system's BF16 - FP32
    energy shift against the BF16 form's mean shift on the sample (this
    network's atomic energies are ~1 eV, so BF16 rounding alone moves the
    energy by up to ~2e-3 eV per atom; the shift is the arithmetic's, which
    the BF16 form reproduces)."""
    s = inputs.make_system("fcc", 3.61, (26, 26, 26), 0.05, 2, seed=96)
    spec = inputs.make_model(2, 8, 3, hidden, 5.5, seed=97)
    _note(f"bf16 resident MLP hidden={hidden} n={s.n}")
    E16, Ea16, F16, W16, ev = _gpu_eval(tmd, ctx, spec, s, tmd.BF16_MLP)
    shift = parity.check_sampled(Ea16, F16, s, spec, True)
    ev.model.set_precision(tmd.FP32)
    pos, sp = _dev(torch, s)
    E32, Ea32, F32, _ = ev.energy_forces(pos, sp, s.box)
    Ea32 = Ea32.cpu().numpy().astype(np.float64)
    F32 = F32.cpu().numpy().astype(np.float64)
    parity.check_sampled(Ea32, F32, s, spec, False)
    # the sample's mean of the form's shift estimates the whole system's to
    # within sigma(shift_i) / sqrt(2000) ~ 2e-5 eV; bar 1e-4 eV
    full = (E16 - E32) / s.n
    print(f"  (E16-E32)/N={full:+.3e}  sampled BF16-form shift={shift:+.3e}", flush=True)
    assert abs(full - shift) <= 1e-4
    assert math.sqrt(np.mean((F16 - F32) ** 2)) <= parity.F_BF16


# ------------------------------------------------------------------ full size (1,024,000 atoms)

def test_bcc1m_sampled_parity(tmd, ctx, torch):
    """The 1,024,000-atom alloy in both precisions: 2 x 2,000 sampled atoms
    against the oracle (and the oracle's BF16 form), and properties of the
    whole system."""
    s, spec, _ = inputs.workload("bcc1m")
    _note(f"bcc1m n={s.n} fp32 + bf16, sampled atoms vs oracle")
    pos, sp = _dev(torch, s)
    ev = tmd.Evaluator(spec, s.n, s.box, ctx=ctx, precision=tmd.FP32)
    E32, Ea32, F32, W32 = ev.energy_forces(pos, sp, s.box)
    Ea32 = Ea32.cpu().numpy().astype(np.float64)
    F32 = F32.cpu().numpy().astype(np.float64)
    ev.model.set_precision(tmd.BF16_MLP)
    E16, Ea16, F16, W16 = ev.energy_forces(pos, sp, s.box, rebuild=False)
    Ea16 = Ea16.cpu().numpy().astype(np.float64)
    F16 = F16.cpu().numpy().astype(np.float64)
    parity.check_sampled(Ea32, F32, s, spec, False, seeds=(80, 81))
    shift = parity.check_sampled(Ea16, F16, s, spec, True, seeds=(80, 81))
    # properties at full size
    assert abs(E32 - oracle.neumaier_sum(Ea32)) <= 1e-9 * abs(E32) + 1e-6
    assert np.abs(F32.sum(0)).max() <= 1e-3
    full = (E16 - E32) / s.n
    print(f"  E/N fp32={E32 / s.n:.6f} bf16={E16 / s.n:.6f}; (E16-E32)/N={full:+.3e}, "
          f"sampled BF16-form shift={shift:+.3e}", flush=True)
    assert abs(full) <= parity.E_BF16
    assert abs(full - shift) <= 1e-4
    assert math.sqrt(np.mean((F16 - F32) ** 2)) <= parity.F_BF16
