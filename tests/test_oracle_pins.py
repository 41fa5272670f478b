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


# ---------------------------------------------------------------- BF16 form of the MLP

def test_bf16_rounding_matches_torch():
    """The oracle's BF16 rounding (FP64 -> FP32 -> nearest 8-bit significand,
    ties to even) against torch's FP32 -> bfloat16 conversion, including exact
    halfway cases, subnormal-range FP32 values and signed zeros."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(11)
    x = rng.normal(size=20000) * np.exp(rng.uniform(-30.0, 30.0, 20000))
    ties = []
    for e in range(-20, 21):
        for m in range(128, 256):
            base = m * 2.0 ** (e - 7)
            ties += [base + 2.0 ** (e - 8), -(base + 2.0 ** (e - 8))]  # exactly halfway to the next bf16
    x = np.concatenate([x, np.array(ties), [0.0, -0.0, 1e-40, -3e-39, 1.0 + 2.0 ** -30]])
    want = torch.tensor(x, dtype=torch.float64).to(torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    got = oracle.round_bf16(x)
    assert np.array_equal(got, want)
    # halfway cases go to the even neighbour: 1 + 2^-8 -> 1, 1 + 3 * 2^-8 -> 1 + 2^-6
    assert oracle.round_bf16(np.array([1 + 2.0 ** -8]))[0] == 1.0
    assert oracle.round_bf16(np.array([1 + 3 * 2.0 ** -8]))[0] == 1 + 2.0 ** -6


def _bf16_exact(rng, shape, scale):
    return oracle.round_bf16(rng.normal(0, scale, size=shape))


def test_bf16_form_is_exact_on_bf16_operands():
    """One hidden layer whose weights and inputs are already BF16 numbers: the
    forward pass of the BF16 form rounds nothing, so its energies equal the
    exact network's bit for bit (the input gradient still rounds the deltas)."""
    spec = inputs.make_model(1, 4, 3, [24], 5.0, seed=12)
    rng = np.random.default_rng(13)
    spec.params[:] = oracle.round_bf16(spec.params)
    G = _bf16_exact(rng, (16, spec.n_features), 1.5)
    sp = np.zeros(16, dtype=np.int32)
    E64, dG64 = oracle.mlp(spec, sp, G)
    E16, dG16 = oracle.mlp(spec, sp, G, bf16=True)
    assert np.array_equal(E16, E64)
    assert not np.array_equal(dG16, dG64)
    # the deltas' rounding moves dG_q by at most u sum_o |W_oq delta_o| with
    # |delta_o| <= |w_out,o| (tanh' <= 1) and u = 2^-8 (1 + 2^-15)
    F = spec.n_features
    W1 = spec.params[:24 * F].reshape(24, F)
    wout = spec.params[24 * F + 24:24 * F + 48]
    bound = 2.0 ** -8 * (1 + 2.0 ** -15) * (np.abs(W1) * np.abs(wout)[:, None]).sum(0)
    assert np.all(np.abs(dG16 - dG64) <= bound[None, :])


def _first_order_bound(spec, s, G):
    """First-order bound on |E_bf16 - E| for one atom: each rounded operand x
    carries a relative error of at most u = 2^-8 (1 + 2^-15) (FP32, then BF16),
    a product of two rounded operands at most 2u, and the activations are
    1-Lipschitz (tanh, squareplus)."""
    u = 2.0 ** -8 * (1 + 2.0 ** -15)
    per = inputs.params_per_species(spec.n_features, spec.hidden)
    p = spec.params[s * per:(s + 1) * per]
    off, a, err = 0, np.asarray(G, dtype=np.float64), np.zeros(len(G))
    win = spec.n_features
    for h in spec.hidden:
        W = p[off:off + h * win].reshape(h, win)
        off += h * win
        b = p[off:off + h]
        off += h
        z = W @ a + b
        err = np.abs(W) @ err + 2 * u * (np.abs(W) @ np.abs(a))
        a = np.tanh(z) if spec.activation == inputs.ACT_TANH else 0.5 * (z + np.sqrt(z * z + 4.0))
        win = h
    wout = p[off:off + win]
    return float(np.abs(wout) @ err)


def test_bf16_form_error_within_rounding_bound():
    """Two hidden layers on random descriptors: the BF16 form differs from the
    exact network by no more than the first-order rounding bound, and on every
    atom by something (so the rounding is applied)."""
    spec = inputs.make_model(2, 6, 3, [32, 24], 5.0, seed=14)
    rng = np.random.default_rng(15)
    G = rng.uniform(0.0, 3.0, size=(40, spec.n_features))
    sp = rng.integers(0, 2, size=40).astype(np.int32)
    E64, _ = oracle.mlp(spec, sp, G)
    E16, _ = oracle.mlp(spec, sp, G, bf16=True)
    bound = np.array([_first_order_bound(spec, int(sp[a]), G[a]) for a in range(40)])
    err = np.abs(E16 - E64)
    assert np.all(err <= 1.01 * bound)
    assert np.all(err > 0.0)


def test_cluster_cut_reproduces_periodic_atoms():
    """A piece cut out of a periodic system with reach 2 rcut (+ margin) gives the
    sampled atoms' energies and forces of the whole periodic system: an atom's
    energy depends on neighbours within rcut, its force on their energies."""
    s = inputs.make_system("bcc", 3.16, (10, 10, 10), 0.1, 2, seed=24)
    spec = inputs.make_model(2, 6, 3, [16, 16], 4.0, seed=25)
    _, Ea, F, _ = oracle.energy_forces(spec, s.pos, s.species, s.box)
    piece, sample, where = inputs.cluster_cut(s, 123, 60, 2 * spec.rcut + 0.5)
    assert piece.n < s.n
    _, Ea_p, F_p, _ = oracle.energy_forces(spec, piece.pos, piece.species, piece.box)
    np.testing.assert_allclose(Ea_p[where], Ea[sample], rtol=0, atol=1e-11)
    np.testing.assert_allclose(F_p[where], F[sample], rtol=0, atol=1e-11)
    # too small a reach changes the forces of the outer sampled atoms
    piece2, sample2, where2 = inputs.cluster_cut(s, 123, 60, spec.rcut)
    _, _, F2, _ = oracle.energy_forces(spec, piece2.pos, piece2.species, piece2.box)
    assert np.abs(F2[where2] - F[sample2]).max() > 1e-6
