"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these re-type the oracle's own formulas: they use closed forms
(single neighbour, perfect lattices), the paper's angular double-sum identity,
a textbook radial symmetry function, torch autograd, invariances, finite
differences and exact rational sums.
"""
import fractions
import itertools
import math
import os

import numpy as np
import pytest

import oracle
from paper_2310_08439_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _h(R, spec):
    """Radial function times cutoff for the test's closed forms (Gaussian x cosine cutoff)."""
    fc = 0.5 * (np.cos(np.pi * R / spec.rcut) + 1.0) if R < spec.rcut else 0.0
    return np.exp(-spec.eta * (R - spec.mu) ** 2) * fc


def _tdm_golden():
    rows = []
    with open(os.path.join(GOLDEN, "tdm_table.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            parts = line.split()
            rows.append((parts[0], [int(v) for v in parts[1:]]))
    return rows


# ---------------------------------------------------------------- T_dm table

def test_tdm_table_is_multinomial():
    """The printed T_dm are the multinomial coefficients m!/(px! py! pz!) of each monomial."""
    for name, t in _tdm_golden():
        if name == "1":
            p = (0, 0, 0)
        else:
            p = tuple(name.count(c) for c in "xyz")
        m = sum(p)
        expect = math.factorial(m) // (math.factorial(p[0]) * math.factorial(p[1]) * math.factorial(p[2]))
        assert t[m] == expect and sum(t) == expect


# ---------------------------------------------------------------- T1 neighbours

def _shell_counts(kind, a, rcut):
    """Number of lattice vectors shorter than rcut, by integer enumeration of the
    infinite lattice (independent of any periodic box)."""
    basis = {"fcc": [(0, 0, 0), (0, .5, .5), (.5, 0, .5), (.5, .5, 0)], "bcc": [(0, 0, 0), (.5, .5, .5)]}[kind]
    n = int(math.ceil(rcut / a)) + 1
    cnt = 0
    for i, j, k in itertools.product(range(-n, n + 1), repeat=3):
        for b in basis:
            r = a * math.sqrt((i + b[0]) ** 2 + (j + b[1]) ** 2 + (k + b[2]) ** 2)
            if 0 < r < rcut:
                cnt += 1
    return cnt


@pytest.mark.parametrize("kind,a,cells,rc", [("fcc", 3.61, (2, 2, 2), 5.0), ("fcc", 3.61, (4, 4, 4), 6.0),
                                             ("bcc", 3.16, (4, 4, 4), 6.0), ("fcc", 3.61, (1, 1, 1), 5.0)])
def test_neighbor_counts_perfect_lattice(kind, a, cells, rc):
    pos, box = inputs.lattice(kind, a, cells)
    sp = np.zeros(len(pos), dtype=np.int32)
    nbr, img, cnt = oracle.neighbors(pos, sp, box, rc)
    expect = _shell_counts(kind, a, rc)
    assert expect == {("fcc", 5.0): 42, ("fcc", 6.0): 78, ("bcc", 6.0): 58}[(kind, rc)]
    assert (cnt == expect).all()


def test_neighbor_list_matches_python_bruteforce_and_is_symmetric():
    s = inputs.make_system("bcc", 3.16, (2, 2, 2), 0.2, 2, seed=7)
    rl = 5.5
    nbr, img, cnt = oracle.neighbors(s.pos, s.species, s.box, rl)
    w = np.mod(s.pos, s.box)
    want = set()
    for i in range(s.n):
        for j in range(s.n):
            for n in itertools.product(range(-3, 4), repeat=3):
                if i == j and n == (0, 0, 0):
                    continue
                d = w[j] - w[i] + np.array(n) * s.box
                if d @ d < rl * rl:
                    want.add((i, j, n))
    got = set()
    for i in range(s.n):
        for c in range(cnt[i]):
            got.add((i, int(nbr[i, c]), tuple(int(v) for v in img[i, c])))
    assert got == want
    for (i, j, n) in got:
        assert (j, i, tuple(-v for v in n)) in got
    # canonical order: species of j, then j, then image
    for i in range(s.n):
        keys = [(s.species[nbr[i, c]], nbr[i, c], tuple(img[i, c])) for c in range(cnt[i])]
        assert keys == sorted(keys)


# ---------------------------------------------------------------- T2 single neighbour

@pytest.mark.parametrize("R", [2.3, 3.1, 4.7])
def test_dimer_closed_form(R):
    """One neighbour: G_{k,0} = h_k(R) and G_{k,m} = h_k(R)^2 for m >= 1
    (sum_d T_dm M_d(u)^2 = |u|^{2m} = 1 by the multinomial theorem)."""
    spec = inputs.make_model(1, 8, 3, [8], 5.0, seed=1)
    box = np.array([30.0, 30.0, 30.0])
    u = np.array([0.36, -0.48, 0.8])
    pos = np.array([[10.0, 11.0, 12.0], [10.0, 11.0, 12.0] + R * u])
    G = oracle.descriptors(spec, pos, np.zeros(2, np.int32), box)
    h = _h(R, spec)
    Gk = G[0].reshape(8, 4)
    np.testing.assert_allclose(Gk[:, 0], h, rtol=1e-13, atol=1e-300)
    for m in (1, 2, 3):
        np.testing.assert_allclose(Gk[:, m], h * h, rtol=1e-12, atol=1e-300)


def test_dimer_two_species_slots():
    """The neighbour's species selects the b block; other blocks stay zero."""
    spec = inputs.make_model(3, 4, 2, [8], 5.0, seed=2)
    box = np.array([30.0, 30.0, 30.0])
    pos = np.array([[5.0, 5.0, 5.0], [7.5, 5.0, 5.0]])
    G = oracle.descriptors(spec, pos, np.array([0, 2], np.int32), box).reshape(2, 3, 4, 3)
    h = _h(2.5, spec)
    assert np.all(G[0, :2] == 0) and np.all(G[1, 1:] == 0)
    np.testing.assert_allclose(G[0, 2, :, 0], h, rtol=1e-13)
    np.testing.assert_allclose(G[1, 0, :, 2], h * h, rtol=1e-12)


# ---------------------------------------------------------------- T3 perfect cubic lattices

@pytest.mark.parametrize("kind,a,cells,rc", [("fcc", 3.61, (3, 3, 3), 6.0), ("bcc", 3.16, (3, 3, 3), 6.0)])
def test_perfect_cubic_lattice(kind, a, cells, rc):
    """Inversion symmetry kills odd moments; cubic symmetry makes the second
    moment isotropic (S_k2 = P_k0^2 / 3); every atom is equivalent; forces vanish."""
    pos, box = inputs.lattice(kind, a, cells)
    sp = np.zeros(len(pos), dtype=np.int32)
    spec = inputs.make_model(1, 8, 3, [16, 16], rc, seed=3)
    G = oracle.descriptors(spec, pos, sp, box).reshape(len(pos), 8, 4)
    scale = G[:, :, 0].max() ** 2
    assert np.abs(G[:, :, 1]).max() < 1e-12 * scale
    assert np.abs(G[:, :, 3]).max() < 1e-12 * scale
    np.testing.assert_allclose(G[:, :, 2], G[:, :, 0] ** 2 / 3.0, rtol=1e-10, atol=1e-14 * scale)
    E, Ea, F, W = oracle.energy_forces(spec, pos, sp, box)
    np.testing.assert_allclose(Ea, Ea[0], rtol=1e-12)
    assert np.abs(F).max() < 1e-10
    # cubic symmetry: isotropic virial
    np.testing.assert_allclose(np.diag(W), W[0, 0], rtol=1e-10)
    assert np.abs(W - np.diag(np.diag(W))).max() < 1e-9 * abs(W[0, 0])


# ---------------------------------------------------------------- T4 MEAM double-sum identity

def test_meam_angular_identity():
    """S[b,k,m] = sum_j sum_l h_k(R_j) h_k(R_l) cos^m(theta_jl), j = l included
    (the paper's double-to-single-sum identity, Sec. II.A, eqn moment_s_formalism)."""
    s = inputs.make_system("bcc", 3.16, (2, 2, 2), 0.15, 2, seed=11)
    spec = inputs.make_model(2, 6, 3, [8], 5.0, seed=4)
    G = oracle.descriptors(spec, s.pos, s.species, s.box).reshape(s.n, 2, 6, 4)
    for i in (0, 5, 13):
        js, imgs, D = oracle.atom_neighbors(i, s.pos, s.species, s.box, spec.rcut)
        R = np.linalg.norm(D, axis=1)
        u = D / R[:, None]
        H = np.stack([_h(r, spec) for r in R])          # [c, K]
        cos = u @ u.T                                    # [c, c]
        for b in range(2):
            sel = s.species[js] == b
            Hb, cb = H[sel], cos[np.ix_(sel, sel)]
            for m in range(4):
                S = np.einsum("jk,lk,jl->k", Hb, Hb, cb ** m)
                got = G[i, b, :, m] ** 2 if m == 0 else G[i, b, :, m]
                np.testing.assert_allclose(got, S, rtol=1e-11, atol=1e-12)


# ---------------------------------------------------------------- T5 BPNN radial function

def test_m0_is_bpnn_radial_g2():
    """With only m = 0 the descriptor is the Behler-Parrinello radial G2 sum
    sum_j exp(-eta (R_ij - mu)^2) f_c(R_ij), per neighbour species."""
    s = inputs.make_system("fcc", 3.61, (2, 2, 2), 0.1, 2, seed=5)
    spec = inputs.make_model(2, 5, 0, [8], 5.0, seed=6)
    G = oracle.descriptors(spec, s.pos, s.species, s.box).reshape(s.n, 2, 5)
    w = np.mod(s.pos, s.box)
    for i in (0, 7, 31):
        g2 = np.zeros((2, 5))
        for j in range(s.n):
            for n in itertools.product(range(-2, 3), repeat=3):
                if i == j and n == (0, 0, 0):
                    continue
                r = np.linalg.norm(w[j] - w[i] + np.array(n) * s.box)
                if r < spec.rcut:
                    fc = 0.5 * (math.cos(math.pi * r / spec.rcut) + 1.0)
                    g2[s.species[j]] += np.exp(-spec.eta * (r - spec.mu) ** 2) * fc
        np.testing.assert_allclose(G[i], g2, rtol=1e-12)


# ---------------------------------------------------------------- T6 MLP vs autograd

@pytest.mark.parametrize("act", [inputs.ACT_TANH, inputs.ACT_SQUAREPLUS])
def test_mlp_matches_torch_autograd(act):
    torch = pytest.importorskip("torch")
    spec = inputs.make_model(2, 4, 3, [24, 16, 8], 5.0, seed=8, activation=act)
    F = spec.n_features
    rng = np.random.default_rng(9)
    G = rng.normal(0, 2.0, size=(10, F))
    sp = rng.integers(0, 2, size=10).astype(np.int32)
    E, dG = oracle.mlp(spec, sp, G)
    per = inputs.params_per_species(F, spec.hidden)
    layout = inputs.param_layout(F, spec.hidden)
    for a in range(10):
        p = torch.tensor(spec.params[sp[a] * per:(sp[a] + 1) * per], dtype=torch.float64)
        x = torch.tensor(G[a], dtype=torch.float64, requires_grad=True)
        off, h, tensors = 0, x, {}
        for name, shape in layout:
            size = int(np.prod(shape))
            tensors[name] = p[off:off + size].reshape(shape)
            off += size
        nl = len(spec.hidden) + 1
        for l in range(1, nl + 1):
            h = tensors[f"W{l}"] @ h + tensors[f"b{l}"]
            if l < nl:
                h = torch.tanh(h) if act == inputs.ACT_TANH else 0.5 * (h + torch.sqrt(h * h + 4.0))
        h.sum().backward()
        np.testing.assert_allclose(E[a], h.item(), rtol=1e-13, atol=1e-13)
        np.testing.assert_allclose(dG[a], x.grad.numpy(), rtol=1e-12, atol=1e-14)


# ---------------------------------------------------------------- T7-T9 invariances

def _small():
    s, spec, _ = inputs.workload("oracle32")
    return s, spec


def test_translation_and_permutation_invariance():
    s, spec = _small()
    E, Ea, F, W = oracle.energy_forces(spec, s.pos, s.species, s.box)
    shifted = s.pos + np.array([1.7, -0.3, 5.9])
    E2, _, F2, W2 = oracle.energy_forces(spec, shifted, s.species, s.box)
    np.testing.assert_allclose(E2, E, rtol=1e-12)
    np.testing.assert_allclose(F2, F, atol=1e-11)
    perm = np.random.default_rng(1).permutation(s.n)
    E3, Ea3, F3, _ = oracle.energy_forces(spec, s.pos[perm], s.species[perm], s.box)
    np.testing.assert_allclose(E3, E, rtol=1e-12)
    np.testing.assert_allclose(F3, F[perm], atol=1e-11)
    np.testing.assert_allclose(Ea3, Ea[perm], rtol=1e-12)


def test_cubic_rotation_of_periodic_cell():
    """A 90-degree rotation maps the cubic periodic cell onto itself."""
    s, spec = _small()
    E, Ea, F, W = oracle.energy_forces(spec, s.pos, s.species, s.box)
    Q = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    rp = s.pos @ Q.T
    E2, Ea2, F2, W2 = oracle.energy_forces(spec, rp, s.species, s.box)
    np.testing.assert_allclose(E2, E, rtol=1e-12)
    np.testing.assert_allclose(F2, F @ Q.T, atol=1e-11)
    np.testing.assert_allclose(W2, Q @ W @ Q.T, rtol=1e-10, atol=1e-10)


def test_random_rotation_of_cluster():
    """Isolated cluster in a box larger than twice (extent + cutoff): E(QX) = E(X), F(QX) = Q F(X)."""
    rng = np.random.default_rng(12)
    spec = inputs.make_model(2, 6, 3, [16, 16], 5.0, seed=13)
    pos, _ = inputs.lattice("bcc", 3.16, (2, 2, 2))
    pos = pos - pos.mean(0) + rng.normal(0, 0.1, pos.shape)
    sp = rng.integers(0, 2, len(pos)).astype(np.int32)
    box = np.array([40.0, 40.0, 40.0])
    A = rng.normal(size=(3, 3))
    Q, _ = np.linalg.qr(A)
    c = np.array([20.0, 20.0, 20.0])
    E, _, F, _ = oracle.energy_forces(spec, pos + c, sp, box)
    E2, _, F2, _ = oracle.energy_forces(spec, pos @ Q.T + c, sp, box)
    np.testing.assert_allclose(E2, E, rtol=1e-12)
    np.testing.assert_allclose(F2, F @ Q.T, atol=1e-11)
    G1 = oracle.descriptors(spec, pos + c, sp, box)
    G2 = oracle.descriptors(spec, pos @ Q.T + c, sp, box)
    np.testing.assert_allclose(G2, G1, rtol=1e-10, atol=1e-12)


def test_net_force_zero():
    s = inputs.make_system("bcc", 3.16, (3, 3, 3), 0.15, 2, seed=14)
    spec = inputs.make_model(2, 6, 3, [16, 16], 5.0, seed=15)
    _, _, F, _ = oracle.energy_forces(spec, s.pos, s.species, s.box)
    assert np.abs(F.sum(0)).max() < 1e-12 * max(1.0, np.abs(F).sum())


# ---------------------------------------------------------------- T10 forces = -dE/dx

def test_forces_central_differences():
    s, spec = _small()
    E, Ea, F, W = oracle.energy_forces(spec, s.pos, s.species, s.box)
    h = 1e-5
    for i in (0, 9, 31):
        for x in range(3):
            p = s.pos.copy()
            p[i, x] += h
            Ep = oracle.energy_forces(spec, p, s.species, s.box)[0]
            p[i, x] -= 2 * h
            Em = oracle.energy_forces(spec, p, s.species, s.box)[0]
            fd = -(Ep - Em) / (2 * h)
            assert abs(fd - F[i, x]) <= 1e-7 * max(1.0, abs(F[i, x]))


def test_forces_central_differences_two_species_squareplus():
    s = inputs.make_system("bcc", 3.16, (2, 2, 2), 0.1, 2, seed=16)
    spec = inputs.make_model(2, 5, 3, [12, 10], 5.5, seed=17, activation=inputs.ACT_SQUAREPLUS)
    _, _, F, _ = oracle.energy_forces(spec, s.pos, s.species, s.box)
    h = 1e-5
    for i in (1, 6):
        for x in range(3):
            p = s.pos.copy()
            p[i, x] += h
            Ep = oracle.energy_forces(spec, p, s.species, s.box)[0]
            p[i, x] -= 2 * h
            Em = oracle.energy_forces(spec, p, s.species, s.box)[0]
            assert abs(-(Ep - Em) / (2 * h) - F[i, x]) <= 1e-7 * max(1.0, abs(F[i, x]))


# ---------------------------------------------------------------- T11 virial

def test_virial_is_strain_derivative():
    """Diagonal W_aa = -dE/d(eps_aa) for a periodic cell stretched along a
    (positions and box scaled together); W symmetric."""
    s, spec = _small()
    E, _, _, W = oracle.energy_forces(spec, s.pos, s.species, s.box)
    assert np.abs(W - W.T).max() < 1e-10 * np.abs(W).max()
    h = 1e-6
    for a in range(3):
        vals = []
        for sgn in (+1, -1):
            T = np.eye(3)
            T[a, a] += sgn * h
            vals.append(oracle.energy_forces(spec, s.pos @ T.T, s.species, s.box * np.diag(T))[0])
        np.testing.assert_allclose(-(vals[0] - vals[1]) / (2 * h), W[a, a], rtol=1e-6, atol=1e-6)


def test_virial_shear_via_cluster():
    """Off-diagonal virial of an isolated cluster: W_ab = -dE/d(eps_ab)."""
    rng = np.random.default_rng(18)
    spec = inputs.make_model(1, 6, 3, [16], 5.0, seed=19)
    pos, _ = inputs.lattice("fcc", 3.61, (2, 2, 1))
    pos = pos - pos.mean(0) + rng.normal(0, 0.1, pos.shape)
    sp = np.zeros(len(pos), np.int32)
    box = np.array([50.0, 50.0, 50.0])
    c = np.array([25.0, 25.0, 25.0])
    _, _, _, W = oracle.energy_forces(spec, pos + c, sp, box)
    h = 1e-6
    for a, b in ((0, 1), (1, 2), (2, 0), (0, 0)):
        vals = []
        for sgn in (+1, -1):
            T = np.eye(3)
            T[a, b] += sgn * h
            vals.append(oracle.energy_forces(spec, pos @ T.T + c, sp, box)[0])
        np.testing.assert_allclose(-(vals[0] - vals[1]) / (2 * h), W[a, b], rtol=1e-6, atol=1e-7)


# ---------------------------------------------------------------- T14 compensated sum

def test_neumaier_sum_exact():
    rng = np.random.default_rng(21)
    x = np.concatenate([rng.normal(0, 1, 1000) * 10.0 ** rng.integers(-8, 8, 1000), [1e16, -1e16, 3.0]])
    exact = sum(fractions.Fraction(v) for v in x)
    got = oracle.neumaier_sum(x)
    assert abs(fractions.Fraction(got) - exact) <= abs(exact) * 2.0 ** -52


def test_total_energy_is_compensated_sum_of_atomic_energies():
    s, spec = _small()
    E, Ea, _, _ = oracle.energy_forces(spec, s.pos, s.species, s.box)
    exact = sum(fractions.Fraction(v) for v in Ea)
    assert abs(fractions.Fraction(E) - exact) <= abs(exact) * 2.0 ** -52


def test_subset_forces_match_full_evaluation():
    s = inputs.make_system("bcc", 3.16, (3, 3, 3), 0.1, 2, seed=22)
    spec = inputs.make_model(2, 6, 3, [16, 16], 5.0, seed=23)
    _, Ea, F, _ = oracle.energy_forces(spec, s.pos, s.species, s.box)
    sel = np.array([0, 7, 30, 53])
    Ea2, F2 = oracle.forces_subset(spec, s.pos, s.species, s.box, sel)
    np.testing.assert_allclose(Ea2, Ea[sel], rtol=1e-13)
    np.testing.assert_allclose(F2, F[sel], atol=1e-12)
