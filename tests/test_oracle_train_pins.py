"""Pins of the oracle's force-matching gradient and NVE integrator.

The training gradient has no printed reference (the paper trained its
potentials elsewhere), so it is pinned by finite differences of the loss,
by torch's double backward on the network, by finite differences of the
descriptors along a displacement field, and by the exact zero at the teacher.
The integrator is pinned by free flight, time reversibility and energy
conservation.
"""
import numpy as np
import pytest

import oracle
from paper_2310_08439_amd import inputs


def _with_params(spec, params):
    import dataclasses
    return dataclasses.replace(spec, params=np.ascontiguousarray(params, dtype=np.float64))


# ---------------------------------------------------------------- descriptor tangent

@pytest.mark.parametrize("case", ["oracle32", "two_species_squareplus"])
def test_descriptor_tangent_is_directional_derivative(case):
    if case == "oracle32":
        s, spec, _ = inputs.workload("oracle32")
    else:
        s = inputs.make_system("bcc", 3.16, (2, 2, 2), 0.15, 2, seed=31)
        spec = inputs.make_model(2, 6, 3, [16], 5.2, seed=32, activation=inputs.ACT_SQUAREPLUS)
    r = np.random.default_rng(33).normal(size=(s.n, 3))
    w = oracle.descriptor_jvp(spec, s.pos, s.species, s.box, r)
    eps = 1e-5
    gp = oracle.descriptors(spec, s.pos + eps * r, s.species, s.box)
    gm = oracle.descriptors(spec, s.pos - eps * r, s.species, s.box)
    fd = (gp - gm) / (2 * eps)
    assert np.abs(fd - w).max() <= 1e-7 * np.abs(w).max()


def test_descriptor_tangent_of_rigid_translation_is_zero():
    s, spec, _ = inputs.workload("oracle32")
    r = np.tile(np.array([[0.3, -1.1, 0.7]]), (s.n, 1))
    w = oracle.descriptor_jvp(spec, s.pos, s.species, s.box, r)
    assert np.abs(w).max() <= 1e-12 * max(1.0, np.abs(oracle.descriptors(spec, s.pos, s.species, s.box)).max())


def test_descriptor_tangent_of_homogeneous_scaling():
    """Along r = x (a uniform dilation of a cluster), each pair tangent is D itself,
    so w = d/de G((1+e) x) = d/ds G at s = 1 for the scaled cluster."""
    rng = np.random.default_rng(34)
    n = 12
    x = rng.uniform(0, 6.0, size=(n, 3)) + 20.0
    sp = rng.integers(0, 2, size=n).astype(np.int32)
    box = np.array([60.0, 60.0, 60.0])
    spec = inputs.make_model(2, 6, 3, [8], 5.0, seed=35)
    w = oracle.descriptor_jvp(spec, x, sp, box, x)
    eps = 1e-6
    c = x.mean(0)
    gp = oracle.descriptors(spec, c + (1 + eps) * (x - c), sp, box)
    gm = oracle.descriptors(spec, c + (1 - eps) * (x - c), sp, box)
    np.testing.assert_allclose(w, (gp - gm) / (2 * eps), rtol=1e-6, atol=1e-8 * np.abs(w).max())


# ---------------------------------------------------------------- second-order network pass

@pytest.mark.parametrize("act", [inputs.ACT_TANH, inputs.ACT_SQUAREPLUS])
def test_mlp_second_matches_torch_double_backward(act):
    torch = pytest.importorskip("torch")
    spec = inputs.make_model(2, 4, 3, [24, 16, 8], 5.0, seed=36, activation=act)
    F = spec.n_features
    rng = np.random.default_rng(37)
    n = 9
    G = rng.normal(0, 1.5, size=(n, F))
    w = rng.normal(0, 1.0, size=(n, F))
    e = rng.normal(0, 1.0, size=n)
    sp = rng.integers(0, 2, size=n).astype(np.int32)
    E, q, grad = oracle.mlp_second(spec, sp, G, w, e)
    per = inputs.params_per_species(F, spec.hidden)
    layout = inputs.param_layout(F, spec.hidden)
    theta = torch.tensor(spec.params, dtype=torch.float64, requires_grad=True)
    J = torch.zeros((), dtype=torch.float64)
    for a in range(n):
        p = theta[sp[a] * per:(sp[a] + 1) * per]
        x = torch.tensor(G[a], dtype=torch.float64, requires_grad=True)
        off, h, t = 0, x, {}
        for name, shape in layout:
            size = int(np.prod(shape))
            t[name] = p[off:off + size].reshape(shape)
            off += size
        nl = len(spec.hidden) + 1
        for l in range(1, nl + 1):
            h = t[f"W{l}"] @ h + t[f"b{l}"]
            if l < nl:
                h = torch.tanh(h) if act == inputs.ACT_TANH else 0.5 * (h + torch.sqrt(h * h + 4.0))
        Ea = h.sum()
        (dEdG,) = torch.autograd.grad(Ea, x, create_graph=True)
        qa = (dEdG * torch.tensor(w[a])).sum()
        np.testing.assert_allclose(E[a], Ea.item(), rtol=1e-13, atol=1e-13)
        np.testing.assert_allclose(q[a], qa.item(), rtol=1e-12, atol=1e-13)
        J = J + e[a] * Ea - qa
    (gt,) = torch.autograd.grad(J, theta)
    np.testing.assert_allclose(grad, gt.numpy(), rtol=1e-11, atol=1e-12 * np.abs(gt.numpy()).max())


# ---------------------------------------------------------------- loss and gradient

def _labels(teacher, batch):
    E = np.empty(batch.n_systems)
    F = np.empty((batch.n, 3))
    for s in range(batch.n_systems):
        x, sp, box = batch.system(s)
        E[s], _, f, _ = oracle.energy_forces(teacher, x, sp, box)
        F[batch.sys_off[s]:batch.sys_off[s + 1]] = f
    return E, F


def _cell32_batch():
    s, _, _ = inputs.workload("oracle32")
    return inputs.Batch(pos=s.pos, species=s.species, sys_off=np.array([0, s.n], dtype=np.int64),
                        boxes=s.box[None, :].copy(), kinds=["fcc2x2x2"])


def _small_batch():
    cells = (("fcc", 3.61, (3, 3, 3)), ("bcc", 3.16, (4, 4, 4)), ("hcp", 2.553, (4, 3, 3)))
    return inputs.train_batch(n_cells=3, seed=41, cells=cells)


def _loss(spec, batch, E_l, F_l, lam, params):
    return oracle.train_loss_grad(_with_params(spec, params), batch.sys_off, batch.pos, batch.species,
                                  batch.boxes, E_l, F_l, lam)


def test_train_gradient_central_differences_32_atom_cell():
    """Configuration-3 check: dL/dtheta by central differences of L on the 32-atom cell."""
    _, teacher, _ = inputs.workload("train_teacher")
    _, student, _ = inputs.workload("train_student")
    b = _cell32_batch()
    E_l, F_l = _labels(teacher, b)
    loss, le, lf, grad = _loss(student, b, E_l, F_l, 0.1, student.params)
    assert le > 0 and lf > 0 and abs(loss - le - lf) <= 1e-15 * loss
    rng = np.random.default_rng(42)
    eps = 1e-6
    for _ in range(3):
        v = rng.normal(size=grad.shape)
        v /= np.linalg.norm(v)
        lp = _loss(student, b, E_l, F_l, 0.1, student.params + eps * v)[0]
        lm = _loss(student, b, E_l, F_l, 0.1, student.params - eps * v)[0]
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - grad @ v) <= 1e-7 * abs(fd) + 1e-12, (fd, grad @ v)
    # single elements: first-layer weight, a second-layer bias, the output bias
    F = student.n_features
    for idx in (5, F * 64 + 64 + 3, student.params.shape[0] - 1):
        e_i = np.zeros_like(student.params)
        e_i[idx] = eps
        fd = (_loss(student, b, E_l, F_l, 0.1, student.params + e_i)[0] -
              _loss(student, b, E_l, F_l, 0.1, student.params - e_i)[0]) / (2 * eps)
        assert abs(fd - grad[idx]) <= 1e-6 * max(abs(grad[idx]), np.abs(grad).max() * 1e-3), (idx, fd, grad[idx])


def test_force_term_gradient_central_differences():
    """Energy labels equal to the student's own energies: the energy term and its
    gradient vanish, leaving the double-backward force term alone."""
    _, teacher, _ = inputs.workload("train_teacher")
    _, student, _ = inputs.workload("train_student")
    b = _small_batch()
    _, F_l = _labels(teacher, b)
    E_own, _ = _labels(student, b)
    loss, le, lf, grad = _loss(student, b, E_own, F_l, 0.1, student.params)
    assert le == 0.0 and lf > 0.0
    rng = np.random.default_rng(47)
    eps = 1e-6
    for _ in range(2):
        v = rng.normal(size=grad.shape)
        v /= np.linalg.norm(v)
        fd = (_loss(student, b, E_own, F_l, 0.1, student.params + eps * v)[0] -
              _loss(student, b, E_own, F_l, 0.1, student.params - eps * v)[0]) / (2 * eps)
        assert abs(fd - grad @ v) <= 1e-6 * abs(fd) + 1e-12, (fd, grad @ v)


def test_train_gradient_central_differences_ragged_batch():
    _, teacher, _ = inputs.workload("train_teacher")
    _, student, _ = inputs.workload("train_student")
    b = _small_batch()
    E_l, F_l = _labels(teacher, b)
    loss, le, lf, grad = _loss(student, b, E_l, F_l, 0.1, student.params)
    v = np.random.default_rng(43).normal(size=grad.shape)
    v /= np.linalg.norm(v)
    eps = 1e-6
    fd = (_loss(student, b, E_l, F_l, 0.1, student.params + eps * v)[0] -
          _loss(student, b, E_l, F_l, 0.1, student.params - eps * v)[0]) / (2 * eps)
    assert abs(fd - grad @ v) <= 1e-7 * abs(fd) + 1e-12


def test_train_loss_and_gradient_vanish_at_the_teacher():
    _, teacher, _ = inputs.workload("train_teacher")
    b = _small_batch()
    E_l, F_l = _labels(teacher, b)
    loss, le, lf, grad = _loss(teacher, b, E_l, F_l, 0.1, teacher.params)
    assert loss == 0.0 and le == 0.0 and lf == 0.0
    assert np.abs(grad).max() == 0.0


def test_energy_only_gradient_matches_torch_backprop():
    """lambda = 0: dL/dtheta = sum_s (2/B)(E_s - Ehat_s)/N_s^2 dE_s/dtheta, with
    dE_s/dtheta from torch autograd of the network on the oracle's descriptors."""
    torch = pytest.importorskip("torch")
    _, teacher, _ = inputs.workload("train_teacher")
    _, student, _ = inputs.workload("train_student")
    b = _small_batch()
    E_l, F_l = _labels(teacher, b)
    _, _, _, grad = _loss(student, b, E_l, F_l, 0.0, student.params)
    F = student.n_features
    layout = inputs.param_layout(F, student.hidden)
    theta = torch.tensor(student.params, dtype=torch.float64, requires_grad=True)
    L = torch.zeros((), dtype=torch.float64)
    for s in range(b.n_systems):
        x, sp, box = b.system(s)
        G = torch.tensor(oracle.descriptors(student, x, sp, box))
        off, h, t = 0, G.T, {}
        for name, shape in layout:
            size = int(np.prod(shape))
            t[name] = theta[off:off + size].reshape(shape)
            off += size
        nl = len(student.hidden) + 1
        for l in range(1, nl + 1):
            h = t[f"W{l}"] @ h + t[f"b{l}"][:, None]
            if l < nl:
                h = torch.tanh(h)
        Es = h.sum()
        L = L + ((Es - E_l[s]) / x.shape[0]) ** 2 / b.n_systems
    (gt,) = torch.autograd.grad(L, theta)
    np.testing.assert_allclose(grad, gt.numpy(), rtol=1e-9, atol=1e-12 * np.abs(gt.numpy()).max())


# ---------------------------------------------------------------- velocity Verlet

def test_nve_free_flight_with_zero_network():
    s, spec, _ = inputs.workload("oracle32")
    spec0 = _with_params(spec, np.zeros_like(spec.params))
    v = inputs.maxwell_boltzmann(np.full(s.n, 63.546), 300.0, seed=44)
    x, vv, epot, ekin = oracle.nve(spec0, s.pos, v, s.species, np.array([63.546]), s.box, 1.0, 25)
    np.testing.assert_allclose(x, s.pos + 25.0 * v, rtol=0, atol=1e-12)
    np.testing.assert_array_equal(vv, v)
    assert np.all(epot == 0.0)


def test_nve_time_reversible():
    s, spec, _ = inputs.workload("oracle32")
    m = np.array([63.546])
    v = inputs.maxwell_boltzmann(np.full(s.n, 63.546), 300.0, seed=45)
    x1, v1, _, _ = oracle.nve(spec, s.pos, v, s.species, m, s.box, 1.0, 20)
    x2, v2, _, _ = oracle.nve(spec, x1, -v1, s.species, m, s.box, 1.0, 20)
    np.testing.assert_allclose(x2, s.pos, rtol=0, atol=1e-9)
    np.testing.assert_allclose(-v2, v, rtol=0, atol=1e-11)


def test_nve_conserves_energy():
    """1,000 steps of 1 fs at 300 K on the 32-atom cell: total-energy drift
    per atom stays far below k_B T (target 1e-4 eV)."""
    s, spec, _ = inputs.workload("oracle32")
    m = np.array([63.546])
    v = inputs.maxwell_boltzmann(np.full(s.n, 63.546), 300.0, seed=46)
    _, _, epot, ekin = oracle.nve(spec, s.pos, v, s.species, m, s.box, 1.0, 1000)
    etot = epot + ekin
    assert np.abs(etot - etot[0]).max() / s.n <= 1e-4
    assert np.std(ekin) > 1e-3  # the dynamics actually exchanged energy


# ---------------------------------------------------------------- Nose-Hoover NVT

KB = 8.617333262e-5


def test_nvt_conserves_extended_energy_and_holds_temperature():
    s, spec, _ = inputs.workload("oracle32")
    v = inputs.maxwell_boltzmann(np.full(s.n, 63.546), 300.0, seed=48)
    for tau in (20.0, 50.0):
        _, _, _, epot, ekin, cons = oracle.nvt(spec, s.pos, v, s.species, s.masses, s.box, 1.0, 300.0, tau, 1000)
        assert np.abs(cons - cons[0]).max() / s.n <= 1e-4
        T = 2.0 * ekin / (3 * s.n * KB)
        assert 255.0 <= T[500:].mean() <= 345.0
    # without the thermostat the random network heats the lattice far above 300 K
    _, _, epot, ekin = oracle.nve(spec, s.pos, v, s.species, s.masses, s.box, 1.0, 1000)
    assert (2.0 * ekin / (3 * s.n * KB))[500:].mean() > 1000.0


def test_nvt_with_a_very_slow_thermostat_is_nve():
    s, spec, _ = inputs.workload("oracle32")
    v = inputs.maxwell_boltzmann(np.full(s.n, 63.546), 300.0, seed=49)
    x1, v1, xe, *_ = oracle.nvt(spec, s.pos, v, s.species, s.masses, s.box, 1.0, 300.0, 1e7, 50)
    x2, v2, _, _ = oracle.nve(spec, s.pos, v, s.species, s.masses, s.box, 1.0, 50)
    assert abs(xe[0]) < 1e-10
    np.testing.assert_allclose(x1, x2, rtol=0, atol=1e-9)
    np.testing.assert_allclose(v1, v2, rtol=0, atol=1e-10)


def test_nvt_time_reversible():
    s, spec, _ = inputs.workload("oracle32")
    v = inputs.maxwell_boltzmann(np.full(s.n, 63.546), 300.0, seed=50)
    x1, v1, (xi, eta), *_ = oracle.nvt(spec, s.pos, v, s.species, s.masses, s.box, 1.0, 300.0, 20.0, 20,
                                       xi_eta=(0.003, 0.0))
    x2, v2, (xi2, _), *_ = oracle.nvt(spec, x1, -v1, s.species, s.masses, s.box, 1.0, 300.0, 20.0, 20,
                                      xi_eta=(-xi, eta))
    np.testing.assert_allclose(x2, s.pos, rtol=0, atol=1e-9)
    np.testing.assert_allclose(-v2, v, rtol=0, atol=1e-11)
    assert abs(-xi2 - 0.003) <= 1e-11


def test_pressure_of_a_free_gas_is_ideal():
    """Zero network: W = 0, so P = 2 KE / (3 V) = N kB T_kin / V."""
    import dataclasses
    s, spec, _ = inputs.workload("oracle32")
    spec0 = dataclasses.replace(spec, params=np.zeros_like(spec.params))
    v = inputs.maxwell_boltzmann(np.full(s.n, 63.546), 300.0, seed=51)
    p = oracle.pressure(spec0, s.pos, v, s.species, s.masses, s.box)
    ke = 0.5 * 103.6427 * 63.546 * (v ** 2).sum(0)
    V = np.prod(s.box)
    np.testing.assert_allclose(p[:3], 2 * ke / V * 160.21766208, rtol=1e-12)
    np.testing.assert_allclose(p[3], 2 * ke.sum() / (3 * V) * 160.21766208, rtol=1e-12)
