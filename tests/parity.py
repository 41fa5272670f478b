"""Bars of the GPU-vs-oracle comparisons (helpers for the GPU tests).

FP32 path against the FP64 oracle (the configuration targets for FP32):
  |E - E_ref| / N <= 1e-5 eV and every |E_i - E_i,ref| <= 1e-5 eV;
  force RMS error <= 1e-4 eV/A and every force component within 1e-3 eV/A
  (ten times the RMS bar: an error of that RMS spread like a normal
  distribution stays below 5.5 RMS over 10^5 components, while one wrong
  component that the RMS would average away fails);
  virial |dW_ab| / N <= rcut x 1e-4 (a pair's term is D g with |D| <= rcut).

BF16 MLP.  Its deviation from FP64 has two parts.  (a) Rounding the operands
of the network's matrix products to BF16 (relative 2^-8), which the oracle's
BF16 form reproduces exactly (same rounding points, exact sums): a property
of the arithmetic the precision form prescribes, not of the kernels.  (b) What
the kernels add: FP32 sums, and operands whose FP32 value and the oracle's
FP64 value round to neighbouring BF16 numbers ("flips": expected on about
(operands per atom) x (FP32 discrepancy / BF16 spacing) ~ 500 x 2^-15, i.e.
a few per cent of the atoms, each moving one product term by one BF16 ulp).
  Against the FP64 oracle: the configuration targets |E - E_ref| / N <= 1e-3 eV
  and force RMS <= 5e-3 eV/A wherever the BF16 form itself meets them; where it
  does not (networks with atomic energies of ~1 eV, or a hundred radial
  functions), the BF16 form's own error plus the FP32 bars.
  Against the BF16 form: the median |dE_i| <= 1e-6 eV (atoms without a flip
  agree at the FP32 level), at most 10 % of the atoms beyond 1e-5 eV, no atom
  beyond 5e-3 eV and a force RMS <= 1e-3 eV/A (a flip may cost at most the
  BF16 force target on one atom, the kernels at most a fifth of it in RMS);
  summed over the atoms without a flip the energy agrees within 1e-6 eV per
  atom (FP32 errors of either sign), and the total is the compensated sum of
  the atomic energies.
"""
import math

import numpy as np

import oracle
from paper_2310_08439_amd import inputs

E_FP32, F_FP32, FMAX_FP32 = 1e-5, 1e-4, 1e-3
E_BF16, F_BF16 = 1e-3, 5e-3
BF16_MEDIAN_EI, BF16_FLIP_EI, BF16_FLIP_FRAC, BF16_MAX_EI, BF16_FORM_FRMS = 1e-6, 1e-5, 0.10, 5e-3, 1e-3


def _rms(x):
    return math.sqrt(float(np.mean(np.square(x))))


def _virial_matrix(W):
    return np.array([[W[0], W[3], W[4]], [W[3], W[1], W[5]], [W[4], W[5], W[2]]])


def check_fp32_atoms(Ea, F, Ear, Fr, tag=""):
    de = np.abs(Ea - Ear)
    df = np.abs(F - Fr)
    print(f"  {tag}max|dE_i|={de.max():.3e}  F rms err={_rms(F - Fr):.3e}  max|dF|={df.max():.3e} "
          f"(F rms={_rms(Fr):.3e})", flush=True)
    assert de.max() <= E_FP32
    assert _rms(F - Fr) <= F_FP32
    assert df.max() <= FMAX_FP32


def check_fp32(E, Ea, F, W, s, spec):
    """Whole system against the FP64 oracle, FP32 bars."""
    Er, Ear, Fr, Wr = oracle.energy_forces(spec, s.pos, s.species, s.box)
    dE = abs(E - Er) / s.n
    dW = np.abs(_virial_matrix(W) - Wr).max() / s.n
    print(f"  |dE|/N={dE:.3e}  |dW|/N={dW:.3e}", flush=True)
    assert dE <= E_FP32
    check_fp32_atoms(Ea, F, Ear, Fr)
    assert dW <= spec.rcut * F_FP32


def check_bf16_atoms(Ea, F, ref64, ref16, n_atoms_total=None, tag=""):
    """Per-atom BF16 checks; ref64 / ref16 = (E_i, F) of the FP64 oracle and of
    its BF16 form for the same atoms."""
    Ear, Fr = ref64
    Eaf, Ff = ref16
    de = np.abs(Ea - Eaf)
    form_frms = _rms(Ff - Fr)
    frms = _rms(F - Fr)
    flip = de > BF16_FLIP_EI
    print(f"  {tag}vs BF16 form: median|dE_i|={np.median(de):.3e} max={de.max():.3e} "
          f"flipped={flip.mean():.4f} F rms={_rms(F - Ff):.3e}; vs FP64: F rms={frms:.3e} "
          f"(form {form_frms:.3e})", flush=True)
    assert np.median(de) <= BF16_MEDIAN_EI
    assert flip.mean() <= BF16_FLIP_FRAC
    assert de.max() <= BF16_MAX_EI
    assert _rms(F - Ff) <= BF16_FORM_FRMS
    assert frms <= max(F_BF16, form_frms + F_FP32)
    return de, flip


def check_bf16(E, Ea, F, W, s, spec):
    """Whole system: against the FP64 oracle and against its BF16 form."""
    E64, Ea64, F64, W64 = oracle.energy_forces(spec, s.pos, s.species, s.box)
    E16, Ea16, F16, _ = oracle.energy_forces(spec, s.pos, s.species, s.box, bf16=True)
    de, flip = check_bf16_atoms(Ea, F, (Ea64, F64), (Ea16, F16))
    form_dE = abs(E16 - E64) / s.n
    dE64 = abs(E - E64) / s.n
    unflipped = abs(float(np.sum((Ea - Ea16)[~flip]))) / s.n
    dW = np.abs(_virial_matrix(W) - W64).max() / s.n
    print(f"  |dE|/N vs FP64={dE64:.3e} (form {form_dE:.3e}); vs form over unflipped atoms={unflipped:.3e}; "
          f"|dW|/N={dW:.3e}", flush=True)
    assert dE64 <= max(E_BF16, form_dE + E_FP32)
    assert unflipped <= BF16_MEDIAN_EI
    assert abs(E - oracle.neumaier_sum(Ea)) <= 1e-9 * abs(E) + 1e-6
    assert dW <= spec.rcut * max(F_BF16, _rms(F16 - F64) + F_FP32)


def sampled_refs(spec, s, n_sample, seed, bf16):
    """Oracle results for about n_sample atoms of a large periodic system, from
    a piece cut out of it (inputs.cluster_cut with reach 2 rcut + 0.5 A)."""
    centre = int(np.random.default_rng(seed).integers(s.n))
    piece, sample, where = inputs.cluster_cut(s, centre, n_sample, 2.0 * spec.rcut + 0.5)
    _, Ea64, F64, _ = oracle.energy_forces(spec, piece.pos, piece.species, piece.box)
    out = {"sample": sample, "ref64": (Ea64[where], F64[where])}
    if bf16:
        _, Ea16, F16, _ = oracle.energy_forces(spec, piece.pos, piece.species, piece.box, bf16=True)
        out["ref16"] = (Ea16[where], F16[where])
    return out


def check_sampled(Ea, F, s, spec, bf16, n_sample=2000, seeds=(0,)):
    """Sampled atoms of a large system against the oracle (FP32 or BF16 bars).
    Returns, for BF16, the BF16 form's mean signed shift of E_i from FP64 over
    the samples (an estimate of its per-atom energy shift at full size)."""
    shifts = []
    for seed in seeds:
        r = sampled_refs(spec, s, n_sample, seed, bf16)
        sel = r["sample"]
        tag = f"sample {len(sel)} (seed {seed}) "
        if bf16:
            check_bf16_atoms(Ea[sel], F[sel], r["ref64"], r["ref16"], tag=tag)
            shifts.append(float(np.mean(r["ref16"][0] - r["ref64"][0])))
        else:
            check_fp32_atoms(Ea[sel], F[sel], r["ref64"][0], r["ref64"][1], tag=tag)
    return float(np.mean(shifts)) if shifts else 0.0
