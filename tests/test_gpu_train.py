"""Force-matching training step and the autograd energy, HIP path vs the oracle.

Bars (FP32 training path against the FP64 oracle): descriptors as in the
inference tests; forces RMS <= 1e-4 eV/A; loss terms within 1e-3 relative;
gradient max error <= 2e-3 of the largest gradient component and relative L2
error <= 2e-3 (the force term is linear in the residual F - Fhat, whose FP32
error is ~1e-4 of its size, and the MLP runs in FP32 with FP32 weight-gradient
sums over up to 500 atoms per system); descriptor tangents within
1e-4 x (|w| + max|w|).
"""
import math
import sys

import numpy as np
import pytest

import oracle
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


def _labels(teacher, batch):
    E = np.empty(batch.n_systems)
    F = np.empty((batch.n, 3))
    for s in range(batch.n_systems):
        x, sp, box = batch.system(s)
        E[s], _, f, _ = oracle.energy_forces(teacher, x, sp, box)
        F[batch.sys_off[s]:batch.sys_off[s + 1]] = f
    return E, F


def _small_batch():
    cells = (("fcc", 3.61, (3, 3, 3)), ("bcc", 3.16, (4, 4, 4)), ("hcp", 2.553, (4, 3, 3)))
    return inputs.train_batch(n_cells=3, seed=41, cells=cells)


def _cell32_batch():
    s, _, _ = inputs.workload("oracle32")
    return inputs.Batch(pos=s.pos, species=s.species, sys_off=np.array([0, s.n], dtype=np.int64),
                        boxes=s.box[None, :].copy(), kinds=["fcc2x2x2"])


def _device_batch(tmd, ctx, torch, model, b, E_l, F_l, capacity=0):
    pos = torch.tensor(b.pos, dtype=torch.float64, device="cuda")
    sp = torch.tensor(b.species, dtype=torch.int32, device="cuda")
    fl = torch.tensor(F_l, dtype=torch.float32, device="cuda")
    return tmd.Batch(ctx, model, b.sys_off, pos, sp, b.boxes, E_l, fl, capacity=capacity)


def _grad_close(g, gr, bar=2e-3):
    err = np.abs(g - gr).max() / np.abs(gr).max()
    rel = np.linalg.norm(g - gr) / np.linalg.norm(gr)
    print(f"  grad max err/max={err:.3e} rel L2={rel:.3e}", flush=True)
    assert err <= bar and rel <= bar


def test_train_step_any_k_and_widths(tmd, ctx, torch):
    """A model whose K (10) and hidden widths (40, 24) are padded inside the
    kernels: loss and gradient (ABI layout, padded entries dropped) against the
    oracle, and an SGD step that leaves the model's own parameters consistent."""
    _note("train step, padded model K=10 hidden [40, 24]")
    teacher = inputs.make_model(1, 10, 3, [40, 24], 5.0, seed=1005)
    student = inputs.make_model(1, 10, 3, [40, 24], 5.0, seed=2005)
    b = _small_batch()
    E_l, F_l = _labels(teacher, b)
    model = tmd.Model(ctx, student)
    assert model.n_params == student.params.shape[0]
    bt = _device_batch(tmd, ctx, torch, model, b, E_l, F_l)
    grad = torch.empty(model.n_params, dtype=torch.float32, device="cuda")
    loss, le, lf = tmd.train_step(ctx, model, bt, lam=0.1, lr=0.0, grad=grad)
    lr_, le_r, lf_r, gr = oracle.train_loss_grad(student, b.sys_off, b.pos, b.species, b.boxes, E_l, F_l, 0.1)
    print(f"  loss {loss:.8e} vs {lr_:.8e}", flush=True)
    assert abs(loss - lr_) <= 1e-3 * lr_
    _grad_close(grad.cpu().numpy().astype(np.float64), gr)
    G = bt.read(tmd.BATCH_G).cpu().numpy().astype(np.float64)
    x, sp, box = b.system(0)
    Gr = oracle.descriptors(student, x, sp, box)
    assert G.shape[1] == student.n_features
    assert (np.abs(G[:b.sys_off[1]] - Gr) / (np.abs(Gr) + 1.0)).max() <= 2e-5
    # one SGD step: the model's parameters move by -lr * grad exactly (FP32)
    p0 = model.get_params()
    tmd.train_step(ctx, model, bt, lam=0.1, lr=1e-2, optimizer=tmd.OPT_SGD)
    p1 = model.get_params()
    g = grad.cpu().numpy()
    np.testing.assert_allclose(p1, (p0 - np.float32(1e-2) * g).astype(np.float32), rtol=0, atol=1e-6)
    # and the updated model evaluates as the oracle does with those parameters
    import dataclasses
    upd = dataclasses.replace(student, params=p1.astype(np.float64))
    ev_pos = torch.tensor(x, dtype=torch.float64, device="cuda")
    ev_sp = torch.tensor(sp, dtype=torch.int32, device="cuda")
    nl = tmd.NeighborList(ctx, len(x), 1, 96)
    tmd.build_neighbors(ctx, ev_pos, ev_sp, box, student.rcut, 0.0, nl)
    E, _, F, _ = tmd.energy_forces(ctx, model, ev_pos, ev_sp, box, nl)
    Er, _, Fr, _ = oracle.energy_forces(upd, x, sp, box)
    assert abs(E - Er) / len(x) <= 1e-5
    assert math.sqrt(np.mean((F.cpu().numpy() - Fr) ** 2)) <= 1e-4
    nl.close()
    bt.close()
    model.close()


@pytest.mark.parametrize("case", ["cell32", "three_cells"])
def test_train_step_matches_oracle(tmd, ctx, torch, case):
    _note(f"train step vs oracle: {case}")
    _, teacher, _ = inputs.workload("train_teacher")
    _, student, _ = inputs.workload("train_student")
    b = _cell32_batch() if case == "cell32" else _small_batch()
    E_l, F_l = _labels(teacher, b)
    model = tmd.Model(ctx, student)
    bt = _device_batch(tmd, ctx, torch, model, b, E_l, F_l)
    grad = torch.empty(model.n_params, dtype=torch.float32, device="cuda")
    loss, le, lf = tmd.train_step(ctx, model, bt, lam=0.1, lr=0.0, grad=grad)
    lr_, le_r, lf_r, gr = oracle.train_loss_grad(student, b.sys_off, b.pos, b.species, b.boxes, E_l, F_l, 0.1)
    print(f"  loss {loss:.8e} vs {lr_:.8e}; E term {le:.6e} vs {le_r:.6e}; F term {lf:.6e} vs {lf_r:.6e}",
          flush=True)
    assert abs(le - le_r) <= 1e-3 * le_r + 1e-12
    assert abs(lf - lf_r) <= 1e-3 * lf_r + 1e-12
    assert abs(loss - lr_) <= 1e-3 * lr_
    _grad_close(grad.cpu().numpy().astype(np.float64), gr)
    # intermediate results: descriptors, forces, tangent along the GPU's own residual
    G = bt.read(tmd.BATCH_G).cpu().numpy().astype(np.float64)
    F = bt.read(tmd.BATCH_FORCES).cpu().numpy().astype(np.float64)
    r = bt.read(tmd.BATCH_RESIDUAL).cpu().numpy().astype(np.float64)
    w = bt.read(tmd.BATCH_TANGENT).cpu().numpy().astype(np.float64)
    for s in range(b.n_systems):
        x, sp, box = b.system(s)
        a0, a1 = int(b.sys_off[s]), int(b.sys_off[s + 1])
        Gr = oracle.descriptors(student, x, sp, box)
        assert (np.abs(G[a0:a1] - Gr) / (np.abs(Gr) + 1.0)).max() <= 2e-5
        _, _, Fr, _ = oracle.energy_forces(student, x, sp, box)
        frms = math.sqrt(np.mean((F[a0:a1] - Fr) ** 2))
        assert frms <= 1e-4, frms
        wr = oracle.descriptor_jvp(student, x, sp, box, r[a0:a1])
        werr = (np.abs(w[a0:a1] - wr) / (np.abs(wr) + np.abs(wr).max())).max()
        assert werr <= 1e-4, werr
    bt.close()
    model.close()


@pytest.mark.parametrize("shape", ["two_species", "hidden128"])
def test_train_step_other_shapes(tmd, ctx, torch, shape):
    """Two species (tiles and reduction chunks of each species apart), and
    128-wide hidden layers (8-atom sub-tiles, hidden weights in 16 LDS blocks)."""
    _note(f"train step vs oracle: {shape}")
    if shape == "two_species":
        # the 64-cell batch: several sub-tiles per workgroup on each side of
        # the species boundary
        b = inputs.train_batch()
        b.species[:] = np.random.default_rng(7).integers(0, 2, b.n).astype(np.int32)
        teacher = inputs.make_model(2, 8, 3, [64, 64], 5.0, seed=1013)
        student = inputs.make_model(2, 8, 3, [64, 64], 5.0, seed=2013)
    else:
        b = _small_batch()
        teacher = inputs.make_model(1, 8, 3, [128, 128], 5.0, seed=1023)
        student = inputs.make_model(1, 8, 3, [128, 128], 5.0, seed=2023)
    E_l, F_l = _labels(teacher, b)
    model = tmd.Model(ctx, student)
    bt = _device_batch(tmd, ctx, torch, model, b, E_l, F_l)
    grad = torch.empty(model.n_params, dtype=torch.float32, device="cuda")
    loss, le, lf = tmd.train_step(ctx, model, bt, lam=0.1, lr=0.0, grad=grad)
    lr_, le_r, lf_r, gr = oracle.train_loss_grad(student, b.sys_off, b.pos, b.species, b.boxes, E_l, F_l, 0.1)
    print(f"  loss {loss:.8e} vs {lr_:.8e}", flush=True)
    assert abs(le - le_r) <= 1e-3 * le_r + 1e-12
    assert abs(lf - lf_r) <= 1e-3 * lf_r + 1e-12
    _grad_close(grad.cpu().numpy().astype(np.float64), gr)
    bt.close()
    model.close()


def test_train_step_full_batch_64_cells(tmd, ctx, torch):
    """The 64-cell fcc/bcc/hcp batch (about 18k atoms) against the oracle."""
    _note("train step 64-cell batch vs oracle")
    _, teacher, _ = inputs.workload("train_teacher")
    _, student, _ = inputs.workload("train_student")
    b = inputs.train_batch()
    E_l, F_l = _labels(teacher, b)
    model = tmd.Model(ctx, student)
    bt = _device_batch(tmd, ctx, torch, model, b, E_l, F_l)
    grad = torch.empty(model.n_params, dtype=torch.float32, device="cuda")
    loss, le, lf = tmd.train_step(ctx, model, bt, lam=0.1, lr=0.0, grad=grad)
    lr_, le_r, lf_r, gr = oracle.train_loss_grad(student, b.sys_off, b.pos, b.species, b.boxes, E_l, F_l, 0.1)
    print(f"  N={b.n} loss {loss:.8e} vs {lr_:.8e}", flush=True)
    assert abs(le - le_r) <= 1e-3 * le_r and abs(lf - lf_r) <= 1e-3 * lf_r
    _grad_close(grad.cpu().numpy().astype(np.float64), gr)
    bt.close()
    model.close()


def test_train_step_large_batch_repeated_cells(tmd, ctx, torch):
    """The 64-cell batch repeated 15 times (276,420 atoms): at this size the
    pair-table kernels keep the model's eight radial functions per thread.
    Both loss terms are means over systems and atoms, so the repeated batch
    has exactly the loss and gradient of the 64-cell batch, which the oracle
    gives."""
    _note("train step, 64-cell batch repeated 15 times")
    rep = 15
    _, teacher, _ = inputs.workload("train_teacher")
    _, student, _ = inputs.workload("train_student")
    b = inputs.train_batch()
    E_l, F_l = _labels(teacher, b)
    off = np.concatenate([[0]] + [b.sys_off[1:] + k * b.n for k in range(rep)]).astype(np.int64)
    big = inputs.Batch(pos=np.tile(b.pos, (rep, 1)), species=np.tile(b.species, rep), sys_off=off,
                       boxes=np.tile(b.boxes, (rep, 1)), kinds=list(b.kinds) * rep)
    assert big.n >= 256 * 1024  # N * K / 8 threads with K = 8
    model = tmd.Model(ctx, student)
    bt = _device_batch(tmd, ctx, torch, model, big, np.tile(E_l, rep), np.tile(F_l, (rep, 1)))
    grad = torch.empty(model.n_params, dtype=torch.float32, device="cuda")
    loss, le, lf = tmd.train_step(ctx, model, bt, lam=0.1, lr=0.0, grad=grad)
    lr_, le_r, lf_r, gr = oracle.train_loss_grad(student, b.sys_off, b.pos, b.species, b.boxes, E_l, F_l, 0.1)
    print(f"  loss {loss:.8e} vs {lr_:.8e}", flush=True)
    assert abs(le - le_r) <= 1e-3 * le_r + 1e-12
    assert abs(lf - lf_r) <= 1e-3 * lf_r + 1e-12
    _grad_close(grad.cpu().numpy().astype(np.float64), gr)
    bt.close()
    model.close()


def test_train_step_is_deterministic(tmd, ctx, torch):
    _note("train step bitwise repeat")
    _, teacher, _ = inputs.workload("train_teacher")
    _, student, _ = inputs.workload("train_student")
    b = _small_batch()
    E_l, F_l = _labels(teacher, b)
    model = tmd.Model(ctx, student)
    bt = _device_batch(tmd, ctx, torch, model, b, E_l, F_l)
    g1 = torch.empty(model.n_params, dtype=torch.float32, device="cuda")
    g2 = torch.empty_like(g1)
    l1 = tmd.train_step(ctx, model, bt, grad=g1)
    l2 = tmd.train_step(ctx, model, bt, grad=g2)
    assert l1 == l2
    assert torch.equal(g1, g2)


@pytest.mark.parametrize("optimizer", ["adam", "sgd"])
def test_update_matches_reference_optimizer(tmd, ctx, torch, optimizer):
    _note(f"optimizer step {optimizer}")
    _, teacher, _ = inputs.workload("train_teacher")
    _, student, _ = inputs.workload("train_student")
    b = _cell32_batch()
    E_l, F_l = _labels(teacher, b)
    model = tmd.Model(ctx, student)
    bt = _device_batch(tmd, ctx, torch, model, b, E_l, F_l)
    theta = model.get_params().astype(np.float64)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    lr, b1, b2, eps = 1e-3, 0.9, 0.999, 1e-8
    grad = torch.empty(model.n_params, dtype=torch.float32, device="cuda")
    opt = tmd.OPT_ADAM if optimizer == "adam" else tmd.OPT_SGD
    for t in range(1, 4):
        tmd.train_step(ctx, model, bt, lr=lr, optimizer=opt, grad=grad)
        g = grad.cpu().numpy().astype(np.float64)
        if opt == tmd.OPT_ADAM:
            m = b1 * m + (1 - b1) * g
            v = b2 * v + (1 - b2) * g * g
            theta = theta - lr * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps)
        else:
            theta = theta - lr * g
        got = model.get_params().astype(np.float64)
        np.testing.assert_allclose(got, theta, rtol=2e-6, atol=2e-7)
        theta = got  # follow the device's FP32 state
    # inference with the updated model uses the regenerated operand copies
    spec_new = inputs.make_model(1, 8, 3, [64, 64], 5.0, seed=2003)
    spec_new.params = model.get_params().astype(np.float64)
    s, _, _ = inputs.workload("oracle32")
    pos = torch.tensor(s.pos, dtype=torch.float64, device="cuda")
    sp = torch.tensor(s.species, dtype=torch.int32, device="cuda")
    nl = tmd.NeighborList(ctx, s.n, 1, 96)
    tmd.build_neighbors(ctx, pos, sp, s.box, spec_new.rcut, 0.0, nl)
    E, _, _, _ = tmd.energy_forces(ctx, model, pos, sp, s.box, nl)
    Er, _, _, _ = oracle.energy_forces(spec_new, s.pos, s.species, s.box)
    assert abs(E - Er) / s.n <= 1e-5
    # BF16 operand copies regenerated on the device equal a fresh host upload
    fresh = tmd.Model(ctx, spec_new)
    for mm in (model, fresh):
        mm.set_precision(tmd.BF16_MLP)
    E_dev, Ea_dev, F_dev, _ = tmd.energy_forces(ctx, model, pos, sp, s.box, nl)
    E_host, Ea_host, F_host, _ = tmd.energy_forces(ctx, fresh, pos, sp, s.box, nl)
    assert E_dev == E_host
    assert torch.equal(Ea_dev, Ea_host)


def test_training_reduces_loss(tmd, ctx, torch):
    _note("30 Adam steps")
    _, teacher, _ = inputs.workload("train_teacher")
    _, student, _ = inputs.workload("train_student")
    b = _small_batch()
    E_l, F_l = _labels(teacher, b)
    model = tmd.Model(ctx, student)
    bt = _device_batch(tmd, ctx, torch, model, b, E_l, F_l)
    losses = [tmd.train_step(ctx, model, bt, lr=2e-3)[0] for _ in range(30)]
    print(f"  loss {losses[0]:.4e} -> {losses[-1]:.4e}", flush=True)
    assert losses[-1] < 0.5 * losses[0]


def test_batch_input_errors(tmd, ctx, torch):
    _note("batch input errors")
    _, student, _ = inputs.workload("train_student")
    b = _cell32_batch()
    model = tmd.Model(ctx, student)
    E_l = np.zeros(1)
    F_l = np.zeros((b.n, 3))
    bad = inputs.Batch(pos=b.pos, species=np.full(b.n, 3, dtype=np.int32), sys_off=b.sys_off, boxes=b.boxes,
                       kinds=b.kinds)
    with pytest.raises(tmd.TMDError) as ei:
        _device_batch(tmd, ctx, torch, model, bad, E_l, F_l)
    assert ei.value.status == 1
    bt = _device_batch(tmd, ctx, torch, model, b, E_l, F_l)
    other = tmd.Model(ctx, inputs.make_model(1, 8, 3, [64, 64], 5.5, seed=2003))
    with pytest.raises(tmd.TMDError) as ei:
        tmd.train_step(ctx, other, bt)
    assert ei.value.status == 1
    # same descriptor shape, wider or deeper network than the batch was sized for:
    # rejected on the host (its per-step buffers are sized by the creation model)
    for hidden in ([128, 128], [64, 64, 64]):
        wider = tmd.Model(ctx, inputs.make_model(1, 8, 3, hidden, student.rcut, seed=2004))
        with pytest.raises(tmd.TMDError) as ei:
            tmd.train_step(ctx, wider, bt)
        assert ei.value.status == 1
        wider.close()
    with pytest.raises(tmd.TMDError):
        tmd.train_step(ctx, model, bt, lr=-1.0)


def test_tmd_energy_autograd(tmd, ctx, torch):
    """torch.autograd through the hand-written adjoint: dE/dx = -F, and central
    differences of the GPU energy agree."""
    _note("TMDEnergy autograd")
    s, spec, _ = inputs.workload("oracle32")
    ev = tmd.Evaluator(spec, s.n, s.box, ctx=ctx)
    pos = torch.tensor(s.pos, dtype=torch.float64, device="cuda", requires_grad=True)
    sp = torch.tensor(s.species, dtype=torch.int32, device="cuda")
    E = tmd.energy(pos, sp, s.box, ev)
    (g,) = torch.autograd.grad(2.0 * E, pos)
    _, _, F, _ = ev.energy_forces(pos.detach(), sp, s.box)
    assert (g + 2.0 * F.double()).abs().max().item() <= 1e-5
    _, _, Fr, _ = oracle.energy_forces(spec, s.pos, s.species, s.box)
    assert math.sqrt(np.mean((-g.cpu().numpy() / 2.0 - Fr) ** 2)) <= 1e-4
    h = 2e-3
    for i, x in ((3, 0), (17, 2)):
        vals = []
        for sgn in (1, -1):
            p = pos.detach().clone()
            p[i, x] += sgn * h
            vals.append(tmd.energy(p, sp, s.box, ev).item())
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - g[i, x].item() / 2.0) <= 2e-3 * max(1.0, abs(fd)) + 1e-3
