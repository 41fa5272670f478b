"""Pins of the oracle's tabulated radial functions (Sec. III.B: H and H'
interpolated from a 1-D table with the cutoff folded in; cubic Hermite
interpolation stands in for the unprinted rational formula).

The checks come from the interpolation theory, not from the oracle's formula:
exactness at the nodes, the cubic Hermite error bound
|f - p| <= delta^4 / 384 max|f''''| with f'''' taken by finite differences of
the direct functions, the convergence orders 4 (value) and 3 (derivative),
value/derivative consistency by central differences, continuity across
nodes, the forced end points, and forces that are minus the gradient of the
tabulated energy.
"""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2310_08439_amd import inputs


def _spec(dr):
    _, spec, _ = inputs.workload("oracle32")  # rc 5.0, K 8
    return dataclasses.replace(spec, tab_dr=dr)


def _radial_many(spec, Rs):
    h = np.empty((len(Rs), spec.n_radial))
    dh = np.empty_like(h)
    for q, R in enumerate(Rs):
        h[q], dh[q] = oracle.radial(spec, float(R))
    return h, dh


def test_exact_at_nodes():
    # rc = 5.0 and dr = 0.0625 give 80 intervals of exactly 0.0625 A: every
    # node is a binary fraction, so t = 0 exactly there.
    tab, direct = _spec(0.0625), _spec(0.0)
    for j in (1, 7, 32, 41, 79):
        R = j * 0.0625
        h, dh = oracle.radial(tab, R)
        h0, dh0 = oracle.radial(direct, R)
        np.testing.assert_allclose(h, h0, rtol=0, atol=1e-15)
        np.testing.assert_allclose(dh, dh0, rtol=0, atol=1e-14)


def test_spacing_rule_puts_cutoff_on_a_node():
    # dr = 0.07 does not divide 5.0: the spacing becomes 5.0 / ceil(5.0 / 0.07) = 5/72
    tab, direct = _spec(0.07), _spec(0.0)
    delta = 5.0 / 72
    for j in (3, 36, 71):
        h, dh = oracle.radial(tab, j * delta)
        h0, dh0 = oracle.radial(direct, j * delta)
        np.testing.assert_allclose(h, h0, rtol=0, atol=1e-12)
        np.testing.assert_allclose(dh, dh0, rtol=0, atol=1e-11)
    # a point between the nodes of a 0.07 grid is not a node of this one
    h, _ = oracle.radial(tab, 36 * 0.07)
    h0, _ = oracle.radial(direct, 36 * 0.07)
    assert np.abs(h - h0).max() > 0.0


def _fourth_derivative_max(spec, lo, hi):
    """max |f''''| over [lo, hi] for each k by 4th central differences of the
    direct functions (step 2e-3: truncation ~1e-6 relative, roundoff ~1e-4)."""
    s = 2e-3
    Rs = np.arange(lo, hi, s / 4)
    out = np.zeros(spec.n_radial)
    for R in Rs:
        v = [oracle.radial(spec, R + q * s)[0] for q in (-2, -1, 0, 1, 2)]
        d4 = (v[0] - 4 * v[1] + 6 * v[2] - 4 * v[3] + v[4]) / s**4
        out = np.maximum(out, np.abs(d4))
    return out


def test_hermite_error_bound():
    """Cubic Hermite interpolation of a C^4 function on nodes delta apart
    errs by at most delta^4/384 max|f''''| (Burden & Faires, Thm 3.9)."""
    direct = _spec(0.0)
    delta = 5.0 / 40  # dr = 0.125
    tab = _spec(0.125)
    # sample the interior intervals [1, 4.5] (the first interval is forced to 0 at r = 0)
    f4 = _fourth_derivative_max(direct, 1.0 - 0.01, 4.5 + 0.01)
    Rs = np.linspace(1.0, 4.5, 3001)
    h, _ = _radial_many(tab, Rs)
    h0, _ = _radial_many(direct, Rs)
    err = np.abs(h - h0).max(0)
    bound = delta**4 / 384 * f4
    assert np.all(err <= 1.02 * bound + 1e-15), (err, bound)
    # and the bound is not vacuous: the error reaches a good part of it
    assert np.all(err >= 0.2 * bound)


def test_convergence_orders():
    direct = _spec(0.0)
    Rs = np.linspace(0.9, 5.1, 6007)
    h0, dh0 = _radial_many(direct, Rs)
    ev, ed = [], []
    for dr in (0.1, 0.05, 0.025):
        h, dh = _radial_many(_spec(dr), Rs)
        ev.append(np.abs(h - h0).max())
        ed.append(np.abs(dh - dh0).max())
    for q in range(2):
        assert 13.0 <= ev[q] / ev[q + 1] <= 19.0, ev  # O(delta^4)
        assert 6.5 <= ed[q] / ed[q + 1] <= 9.5, ed    # O(delta^3)


def test_derivative_is_derivative_of_value():
    tab = _spec(0.1)
    rng = np.random.default_rng(5)
    delta = 0.1
    for _ in range(40):
        j = rng.integers(1, 49)
        R = (j + rng.uniform(0.05, 0.95)) * delta  # inside one cubic piece
        e = 1e-6
        hp, _ = oracle.radial(tab, R + e)
        hm, _ = oracle.radial(tab, R - e)
        _, dh = oracle.radial(tab, R)
        np.testing.assert_allclose((hp - hm) / (2 * e), dh, rtol=0, atol=1e-8)


def test_continuous_across_nodes():
    tab = _spec(0.1)
    for j in (5, 20, 33, 49):
        R = j * 0.1
        e = 1e-9
        hl, dl = oracle.radial(tab, R - e)
        hr, dr = oracle.radial(tab, R + e)
        np.testing.assert_allclose(hl, hr, rtol=0, atol=1e-8)
        np.testing.assert_allclose(dl, dr, rtol=0, atol=1e-6)


def test_end_points():
    tab = _spec(0.05)
    h, dh = oracle.radial(tab, 0.0)
    assert np.all(h == 0.0) and np.all(dh == 0.0)  # forced node at r = 0
    for R in (5.0, 5.0 + 1e-12, 7.3):
        h, dh = oracle.radial(tab, R)
        assert np.all(h == 0.0) and np.all(dh == 0.0)
    h, dh = oracle.radial(tab, 5.0 - 1e-7)
    assert np.abs(h).max() < 1e-12 and np.abs(dh).max() < 1e-5


def test_tabulated_forces_are_gradient_of_tabulated_energy():
    s, _, _ = inputs.workload("oracle32")
    tab = _spec(0.05)
    E, Ea, F, W = oracle.energy_forces(tab, s.pos, s.species, s.box)
    h = 1e-5
    for i in (0, 13, 30):
        for x in range(3):
            p = s.pos.copy()
            p[i, x] += h
            Ep = oracle.energy_forces(tab, p, s.species, s.box)[0]
            p[i, x] -= 2 * h
            Em = oracle.energy_forces(tab, p, s.species, s.box)[0]
            assert abs(-(Ep - Em) / (2 * h) - F[i, x]) <= 1e-6 * max(1.0, abs(F[i, x]))


def test_tabulated_energy_converges_to_direct():
    s, _, _ = inputs.workload("oracle32")
    E0, _, F0, _ = oracle.energy_forces(_spec(0.0), s.pos, s.species, s.box)
    errs = []
    for dr in (0.1, 0.01):
        E, _, F, _ = oracle.energy_forces(_spec(dr), s.pos, s.species, s.box)
        errs.append((abs(E - E0), np.abs(F - F0).max()))
    assert errs[1][0] < errs[0][0] * 1e-2 and errs[1][1] < errs[0][1] * 1e-1
    assert errs[1][0] < 1e-6 * s.n and errs[1][1] < 1e-5


def test_invalid_spacing_rejected():
    s, _, _ = inputs.workload("oracle32")
    for dr in (-0.1, 6.0, float("nan")):
        with pytest.raises(ValueError):
            oracle.energy_forces(_spec(dr), s.pos, s.species, s.box)
