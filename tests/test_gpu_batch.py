"""tmd_energy_forces_batch: several small systems in one launch chain.

* Against the FP64 oracle, per system, to the FP32 bars of tests/parity.py
  (whole-system energy, per-atom energies, forces, virial), and in BF16 to the
  BF16 bars against the oracle and its BF16 form.
* Against tmd_energy_forces_async run per system.  The single-system path
  may take the blocked descriptor and adjoint, which form displacements from
  FP32 offsets held in LDS (about 3e-7 A of rounding per coordinate) and sum in
  another order, while the batch forms them from the FP64 positions: forces
  within the FP32 force bars, energies within 1e-6 eV per atom and virials
  within rcut x 1e-6 eV per atom (a tenth of the FP32 energy target and a
  hundredth of the FP32 virial bar; FP32 rounding of the displacements moves a
  bcc atom's energy by ~1e-7 eV).
* A system's results do not depend on its batch mates: alone in a batch of
  one and in the full batch they agree bit for bit (fixed-point force sums,
  per-system totals over segments that no workgroup crosses).
* Lists built with a skin (rows with entries beyond the cutoff) give the
  same results as lists built without one, within the FP32 bars.
"""
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


# small systems of the two-element bcc alloy and its fcc/hcp relatives, all
# evaluated with the alloy's model (two species, K 12, M 3, rc 6): boxes from
# below twice the cutoff (periodic self-images) to several cells per edge
SYSTEMS = [
    ("bcc", 3.16, (3, 3, 3), 0.08, 2, 11),
    ("bcc", 3.16, (4, 4, 5), 0.08, 2, 12),
    ("fcc", 3.61, (3, 3, 3), 0.05, 2, 13),
    ("bcc", 3.16, (7, 6, 6), 0.10, 2, 14),
    ("hcp", 2.553, (4, 3, 3), 0.05, 2, 15),
    ("bcc", 3.16, (2, 2, 2), 0.08, 2, 16),
]


def _systems():
    return [inputs.make_system(k, a, c, sg, ns, seed=sd) for k, a, c, sg, ns, sd in SYSTEMS]


def _model():
    return inputs.make_model(2, 12, 3, [128, 128], 6.0, seed=102)


def _lists(tmd, ctx, torch, spec, systems, skin):
    out = []
    for s in systems:
        pos = torch.tensor(s.pos, dtype=torch.float64, device="cuda")
        sp = torch.tensor(s.species, dtype=torch.int32, device="cuda")
        cap = tmd.default_capacity(s.n, s.box, spec.rcut + skin, spec.n_species)
        nl = tmd.NeighborList(ctx, s.n, spec.n_species, cap)
        tmd.build_neighbors(ctx, pos, sp, s.box, spec.rcut, skin, nl)
        out.append((pos, sp, nl))
    return out


def _batch(tmd, ctx, torch, model, systems, lists, idx=None):
    idx = list(range(len(systems))) if idx is None else idx
    tot = torch.zeros((len(idx), 7), dtype=torch.float64, device="cuda")
    F = [torch.zeros((systems[i].n, 3), dtype=torch.float32, device="cuda") for i in idx]
    tmd.energy_forces_batch(ctx, model, [(lists[i][0], lists[i][1], systems[i].box) for i in idx],
                            [lists[i][2] for i in idx], tot, F)
    torch.cuda.synchronize()
    return tot.cpu().numpy(), [f.cpu().numpy().astype(np.float64) for f in F]


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_batch_matches_oracle(tmd, ctx, torch, prec):
    spec = _model()
    systems = _systems()
    _note(f"batch of {len(systems)} systems ({[s.n for s in systems]} atoms) vs oracle, {prec}")
    model = tmd.Model(ctx, spec, tmd.FP32 if prec == "fp32" else tmd.BF16_MLP)
    lists = _lists(tmd, ctx, torch, spec, systems, 0.0)
    tot, F = _batch(tmd, ctx, torch, model, systems, lists)
    for s, t, f in zip(systems, tot, F):
        E64, Ea64, F64, W64 = oracle.energy_forces(spec, s.pos, s.species, s.box)
        dW = np.abs(parity._virial_matrix(t[1:]) - W64).max() / s.n
        if prec == "fp32":
            frms = parity._rms(f - F64)
            print(f"  n={s.n}: |dE|/N={abs(t[0] - E64) / s.n:.3e}  F rms={frms:.3e}  "
                  f"max|dF|={np.abs(f - F64).max():.3e}  |dW|/N={dW:.3e}", flush=True)
            assert abs(t[0] - E64) / s.n <= parity.E_FP32
            assert frms <= parity.F_FP32
            assert np.abs(f - F64).max() <= parity.FMAX_FP32
            assert dW <= spec.rcut * parity.F_FP32
        else:
            E16, Ea16, F16, _ = oracle.energy_forces(spec, s.pos, s.species, s.box, bf16=True)
            form_dE = abs(E16 - E64) / s.n
            print(f"  n={s.n}: |dE|/N vs FP64={abs(t[0] - E64) / s.n:.3e} (form {form_dE:.3e}) "
                  f"F rms vs form={parity._rms(f - F16):.3e}  |dW|/N={dW:.3e}", flush=True)
            assert abs(t[0] - E64) / s.n <= max(parity.E_BF16, form_dE + parity.E_FP32)
            assert parity._rms(f - F16) <= parity.BF16_FORM_FRMS
            assert parity._rms(f - F64) <= max(parity.F_BF16, parity._rms(F16 - F64) + parity.F_FP32)
            assert dW <= spec.rcut * max(parity.F_BF16, parity._rms(F16 - F64) + parity.F_FP32)
    model.close()
    for _, _, nl in lists:
        nl.close()


def test_batch_matches_single_system_path(tmd, ctx, torch):
    spec = _model()
    systems = _systems()
    _note("batch vs tmd_energy_forces_async per system, FP32")
    model = tmd.Model(ctx, spec, tmd.FP32)
    lists = _lists(tmd, ctx, torch, spec, systems, 0.0)
    tot, F = _batch(tmd, ctx, torch, model, systems, lists)
    for i, s in enumerate(systems):
        pos, sp, nl = lists[i]
        t1 = torch.zeros(7, dtype=torch.float64, device="cuda")
        f1 = torch.zeros((s.n, 3), dtype=torch.float32, device="cuda")
        tmd.energy_forces_async(ctx, model, pos, sp, s.box, nl, t1, f1)
        torch.cuda.synchronize()
        t1 = t1.cpu().numpy()
        f1 = f1.cpu().numpy().astype(np.float64)
        print(f"  n={s.n}: |dE|={abs(tot[i][0] - t1[0]):.3e}  max|dF|={np.abs(F[i] - f1).max():.3e}  "
              f"max|dW|={np.abs(tot[i][1:] - t1[1:]).max():.3e}", flush=True)
        assert abs(tot[i][0] - t1[0]) / s.n <= 1e-6
        assert parity._rms(F[i] - f1) <= parity.F_FP32 and np.abs(F[i] - f1).max() <= parity.FMAX_FP32
        assert np.abs(tot[i][1:] - t1[1:]).max() / s.n <= spec.rcut * 1e-6
    model.close()
    for _, _, nl in lists:
        nl.close()


def test_batch_independent_of_batch_mates(tmd, ctx, torch):
    spec = _model()
    systems = _systems()
    _note("each system alone vs in the full batch, bit for bit, BF16")
    model = tmd.Model(ctx, spec, tmd.BF16_MLP)
    lists = _lists(tmd, ctx, torch, spec, systems, 0.0)
    tot, F = _batch(tmd, ctx, torch, model, systems, lists)
    for i in range(len(systems)):
        t1, f1 = _batch(tmd, ctx, torch, model, systems, lists, idx=[i])
        assert np.array_equal(t1[0], tot[i])
        assert np.array_equal(f1[0], F[i])
    # a reordered batch with a repeated system
    order = [3, 0, 5, 3, 1]
    t2, f2 = _batch(tmd, ctx, torch, model, systems, lists, idx=order)
    for k, i in enumerate(order):
        assert np.array_equal(t2[k], tot[i])
        assert np.array_equal(f2[k], F[i])
    model.close()
    for _, _, nl in lists:
        nl.close()


def test_batch_with_skin_lists(tmd, ctx, torch):
    spec = _model()
    systems = _systems()
    _note("skin 1 A lists vs skin 0 lists in the batch, FP32")
    model = tmd.Model(ctx, spec, tmd.FP32)
    l0 = _lists(tmd, ctx, torch, spec, systems, 0.0)
    l1 = _lists(tmd, ctx, torch, spec, systems, 1.0)
    t0, f0 = _batch(tmd, ctx, torch, model, systems, l0)
    t1, f1 = _batch(tmd, ctx, torch, model, systems, l1)
    for i, s in enumerate(systems):
        assert abs(t0[i][0] - t1[i][0]) / s.n <= parity.E_FP32
        assert parity._rms(f0[i] - f1[i]) <= parity.F_FP32
    model.close()
    for _, _, nl in l0 + l1:
        nl.close()


def test_batch_rejects_bad_arguments(tmd, ctx, torch):
    spec = _model()
    systems = _systems()[:2]
    model = tmd.Model(ctx, spec, tmd.FP32)
    lists = _lists(tmd, ctx, torch, spec, systems, 0.0)
    tot = torch.zeros((2, 7), dtype=torch.float64, device="cuda")
    F = [torch.zeros((s.n, 3), dtype=torch.float32, device="cuda") for s in systems]
    # a list paired with another system's atoms
    with pytest.raises(tmd.TMDError):
        tmd.energy_forces_batch(ctx, model, [(lists[1][0], lists[1][1], systems[1].box),
                                             (lists[0][0], lists[0][1], systems[0].box)],
                                [lists[0][2], lists[1][2]], tot, F[::-1])
    model.close()
    for _, _, nl in lists:
        nl.close()
