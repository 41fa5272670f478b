"""Tabulated radial functions (tmd_model_tabulate) on the GPU.

Parity: the GPU with a table against the oracle with the same table (same
spacing rule, cubic Hermite nodes) at the direct path's bars (tests/parity.py:
FP32 bars, and BF16 against the oracle and its BF16 form).  Static accuracy (the
paper's static test): GPU tabulated against GPU direct forces, RMS error
falling with the spacing down to the FP32 floor.  Dynamics: an NVE run with
the table conserves energy as well as the direct one.
"""
import dataclasses
import math
import sys

import numpy as np
import pytest

import oracle
import parity
from paper_2310_08439_amd import inputs

pytestmark = pytest.mark.gpu

CU = 63.546


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


def _eval(tmd, ctx, torch, spec, s, prec=0):
    pos = torch.tensor(s.pos, dtype=torch.float64, device="cuda")
    sp = torch.tensor(s.species, dtype=torch.int32, device="cuda")
    ev = tmd.Evaluator(spec, s.n, s.box, precision=prec, ctx=ctx)
    E, Ea, F, W = ev.energy_forces(pos, sp, s.box)
    return E, Ea.cpu().numpy().astype(np.float64), F.cpu().numpy().astype(np.float64), W, ev


@pytest.mark.parametrize("name,dr", [("oracle32", 0.05), ("oracle32", 0.0625), ("bcc4k", 0.01), ("fcc32k", 0.003)])
def test_tabulated_matches_oracle_table(tmd, ctx, torch, name, dr):
    s, spec, _ = inputs.workload(name)
    tab = dataclasses.replace(spec, tab_dr=dr)
    _note(f"tabulated {name} dr={dr} n={s.n}")
    E, Ea, F, W, ev = _eval(tmd, ctx, torch, tab, s)
    assert ev.model.tab_spacing == spec.rcut / math.ceil(spec.rcut / dr)
    parity.check_fp32(E, Ea, F, W, s, tab)


@pytest.mark.parametrize("prec", [0, 1])
def test_tabulated_model_shapes(tmd, ctx, torch, prec):
    """kc 4 (K 4), 6 (K 12) and 8 (K 32) chunks, M 1..3, two species, both MLP precisions."""
    s = inputs.make_system("bcc", 3.16, (3, 3, 3), 0.12, 2, seed=150)
    for K, M in ((4, 3), (12, 1), (32, 3)):
        spec = dataclasses.replace(inputs.make_model(2, K, M, [64, 64], 5.5, seed=151), tab_dr=0.02)
        _note(f"tabulated K={K} M={M} prec={prec}")
        E, Ea, F, W, _ = _eval(tmd, ctx, torch, spec, s, prec)
        if prec == 0:
            parity.check_fp32(E, Ea, F, W, s, spec)
        else:
            parity.check_bf16(E, Ea, F, W, s, spec)


def test_tabulated_non_uniform_grid_and_wide_stencil(tmd, ctx, torch):
    """Jittered centres (no recurrence in the direct path; the table does not
    care) and a box edge shorter than the cutoff (atomic force scatter)."""
    s = inputs.make_system("fcc", 3.61, (1, 1, 2), 0.08, 1, seed=152)
    spec = inputs.make_model(1, 8, 3, [32], 5.0, seed=153)
    rng = np.random.default_rng(154)
    spec = dataclasses.replace(spec, mu=spec.mu + rng.uniform(-0.05, 0.05, size=spec.mu.shape), tab_dr=0.01)
    _note("tabulated, jittered mu, wide stencil")
    E, Ea, F, W, _ = _eval(tmd, ctx, torch, spec, s)
    parity.check_fp32(E, Ea, F, W, s, spec)


def test_static_error_against_direct(tmd, ctx, torch):
    """Force RMS error of the tabulated GPU path against the direct GPU path on
    16,000 atoms (the paper's static test size) for several spacings."""
    s = inputs.make_system("bcc", 3.16, (20, 20, 20), 0.08, 2, seed=155)
    _, spec, _ = inputs.workload("bcc1m")
    E0, _, F0, _, ev = _eval(tmd, ctx, torch, spec, s)
    errs = []
    for dr in (0.1, 0.05, 0.01, 0.001):
        ev.model.tabulate(dr)
        E, _, F, _ = ev.energy_forces(torch.tensor(s.pos, device="cuda"),
                                      torch.tensor(s.species, dtype=torch.int32, device="cuda"), s.box)
        F = F.cpu().numpy().astype(np.float64)
        errs.append((abs(E - E0) / s.n, math.sqrt(np.mean((F - F0) ** 2))))
        print(f"  dr={dr}: |dE|/N={errs[-1][0]:.3e}  F rms={errs[-1][1]:.3e}", flush=True)
    assert errs[0][1] > 4 * errs[1][1]          # O(dr^3) while above the FP32 floor
    assert errs[2][1] <= 2e-5 and errs[3][1] <= 2e-5
    assert errs[2][0] <= 1e-6 and errs[3][0] <= 1e-6
    ev.model.tabulate(0.0)
    assert ev.model.tab_spacing == 0.0
    E1 = ev.energy_forces(torch.tensor(s.pos, device="cuda"),
                          torch.tensor(s.species, dtype=torch.int32, device="cuda"), s.box)[0]
    assert E1 == E0


def test_bcc1m_tabulated_sampled(tmd, ctx, torch):
    s, spec, _ = inputs.workload("bcc1m")
    tab = dataclasses.replace(spec, tab_dr=0.01)
    _note(f"bcc1m tabulated n={s.n}")
    E, Ea, F, W, _ = _eval(tmd, ctx, torch, tab, s)
    parity.check_sampled(Ea, F, s, tab, False, n_sample=1000, seeds=(156,))


def test_tabulated_md_conserves_energy(tmd, ctx, torch):
    s = inputs.make_system("fcc", 3.61, (3, 3, 3), 0.1, 1, seed=157, masses=[CU])
    _, spec, _ = inputs.workload("oracle32")
    v0 = inputs.maxwell_boltzmann(np.full(s.n, CU), 300.0, seed=158)
    drift = {}
    for dr in (0.0, 0.01):
        model = tmd.Model(ctx, dataclasses.replace(spec, tab_dr=dr))
        pos = torch.tensor(s.pos, dtype=torch.float64, device="cuda")
        sp = torch.tensor(s.species, dtype=torch.int32, device="cuda")
        vel = torch.tensor(v0, dtype=torch.float64, device="cuda")
        md = tmd.MD(ctx, model, pos, sp, s.box, s.masses, vel, dt_fs=1.0, ensemble=tmd.ENSEMBLE_NVE, skin=1.0,
                    rebuild_every=5)
        th = md.run(1000, thermo_every=10)
        e = np.array([t["etotal"] for t in th])
        drift[dr] = np.abs(e - e[0]).max() / s.n
        md.close()
    _note(f"NVE drift per atom: direct {drift[0.0]:.2e}, tabulated {drift[0.01]:.2e}")
    assert drift[0.01] <= max(2 * drift[0.0], 2e-5)


def test_tabulated_errors_and_training_guard(tmd, ctx, torch):
    _, spec, _ = inputs.workload("oracle32")
    model = tmd.Model(ctx, spec)
    for dr in (-0.01, 6.0, float("inf"), float("nan"), 4e-6):
        with pytest.raises(tmd.TMDError) as ei:
            model.tabulate(dr)
        assert ei.value.status == 1
        assert model.tab_spacing == 0.0
    assert model.tabulate(0.07) == 5.0 / 72
    b = inputs.train_batch(n_cells=2, seed=159)
    tm = tmd.Model(ctx, inputs.workload("train_teacher")[1])
    tm.tabulate(0.01)
    batch = tmd.Batch(ctx, tm, b.sys_off, torch.tensor(b.pos, dtype=torch.float64, device="cuda"),
                      torch.tensor(b.species, dtype=torch.int32, device="cuda"), b.boxes,
                      np.zeros(b.n_systems), torch.zeros((b.n, 3), dtype=torch.float32, device="cuda"))
    with pytest.raises(tmd.TMDError) as ei:
        tmd.train_step(ctx, tm, batch, lr=0.0)
    assert ei.value.status == 1 and "table" in ei.value.message
    tm.tabulate(0.0)
    loss, _, _ = tmd.train_step(ctx, tm, batch, lr=0.0)
    assert math.isfinite(loss)
    batch.close()
