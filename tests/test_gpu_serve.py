"""The serving loop (tmd_serve_*) on the GPU: results against the oracle, NVE
energy conservation, results alone vs in a concurrent mix, per-system order,
admission by memory budget.

Bars: energies and forces as in the inference tests (FP32: |dE|/N <= 1e-5 eV,
force RMS <= 1e-4 eV/A); MD trajectories of 10 steps of 1 fs against the FP64
oracle's velocity Verlet: positions within 1e-6 A and velocities within
1e-7 A/fs (a force error of 1e-4 eV/A moves a 63.5 amu atom by ~1e-7 A in
10 fs); alone vs mix: the same request on the same state gives the same
forces, energies, positions and kinetic energies bit for bit (forces are
summed in fixed point, totals in a fixed order).
"""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_2310_08439_amd import inputs

pytestmark = pytest.mark.gpu

CU_MASS = 63.546


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


def _fcc108():
    return inputs.make_system("fcc", 3.61, (3, 3, 3), 0.1, 1, seed=71, masses=[CU_MASS])


def test_serve_energy_forces_matches_oracle(tmd, ctx):
    _note("serve EF vs oracle")
    _, spec, _ = inputs.workload("oracle32")
    model = tmd.Model(ctx, spec)
    srv = tmd.Server(model, max_slots=2, max_atoms=4096, skin=1.0)
    systems = [_fcc108(), inputs.make_system("bcc", 3.16, (4, 4, 4), 0.1, 1, seed=72, masses=[CU_MASS])]
    ids = [srv.add_system(s.pos, s.species, s.box, s.masses) for s in systems]
    tickets = [srv.submit(i) for i in ids]
    for s, t in zip(systems, tickets):
        r = srv.wait(t, 60.0)
        assert r is not None and r["status"] == 0
        out = srv.fetch(t, r)
        Er, _, Fr, Wr = oracle.energy_forces(spec, s.pos, s.species, s.box)
        assert abs(r["energy"] - Er) / s.n <= 1e-5
        assert math.sqrt(np.mean((out["forces"] - Fr) ** 2)) <= 1e-4
        W = np.array(r["virial"])
        Wr6 = np.array([Wr[0, 0], Wr[1, 1], Wr[2, 2], Wr[0, 1], Wr[0, 2], Wr[1, 2]])
        assert np.abs(W - Wr6).max() / s.n <= spec.rcut * 1e-4
    srv.close()


def test_serve_md_matches_oracle_velocity_verlet(tmd, ctx):
    _note("serve MD vs oracle NVE")
    _, spec, _ = inputs.workload("oracle32")
    model = tmd.Model(ctx, spec)
    srv = tmd.Server(model, max_slots=2, max_atoms=4096, skin=0.3)
    s = _fcc108()
    v0 = inputs.maxwell_boltzmann(np.full(s.n, CU_MASS), 300.0, seed=73)
    sid = srv.add_system(s.pos, s.species, s.box, s.masses)
    t = srv.submit(sid, tmd.REQ_MD, n_steps=10, dt_fs=1.0, velocities=v0)
    r = srv.wait(t, 60.0)
    assert r["status"] == 0
    out = srv.fetch(t, r)
    x, v, epot, ekin = oracle.nve(spec, s.pos, v0, s.species, s.masses, s.box, 1.0, 10)
    print(f"  max |dx|={np.abs(out['pos'] - x).max():.3e}  max |dv|={np.abs(out['vel'] - v).max():.3e}", flush=True)
    np.testing.assert_allclose(out["pos"], x, rtol=0, atol=1e-6)
    np.testing.assert_allclose(out["vel"], v, rtol=0, atol=1e-7)
    assert np.abs(out["epot"] - epot).max() / s.n <= 1e-5
    np.testing.assert_allclose(out["ekin"], ekin, rtol=1e-5, atol=1e-8)
    # the resident state is the final state
    xs, vs = srv.read_system(sid)
    np.testing.assert_array_equal(xs, out["pos"])
    np.testing.assert_array_equal(vs, out["vel"])
    srv.close()


def test_serve_md_in_queued_chunks_matches_oracle(tmd, ctx):
    """40 NVE steps of 4,000 atoms (160,000 atom-steps): the server queues them
    in chunks of at least 65,536 atom-steps (17 steps here) and waits for the
    end of the first chunk once the third is queued; the trajectory still
    follows the FP64 oracle's velocity Verlet.  With a 1 A skin no atom moves
    beyond skin/2, so no step rebuilds the list that registration built.
    Bars: a force error of 5e-6 eV/A (the FP32 path's largest) acting for the
    whole 40 fs moves an atom by 0.5 * 9.65e-3 * 5e-6 / 63.5 * 40^2 = 6e-7 A
    and changes its velocity by 3e-8 A/fs; the bars allow three times that."""
    _note("serve MD in chunks vs oracle NVE")
    _, spec, _ = inputs.workload("oracle32")
    model = tmd.Model(ctx, spec)
    srv = tmd.Server(model, max_slots=2, max_atoms=4096, skin=1.0)
    s = inputs.make_system("fcc", 3.61, (10, 10, 10), 0.05, 1, seed=74, masses=[CU_MASS])
    v0 = inputs.maxwell_boltzmann(np.full(s.n, CU_MASS), 300.0, seed=75)
    sid = srv.add_system(s.pos, s.species, s.box, s.masses)
    t = srv.submit(sid, tmd.REQ_MD, n_steps=40, dt_fs=1.0, velocities=v0)
    r = srv.wait(t, 60.0)
    assert r["status"] == 0 and r["rebuilds"] == 0
    out = srv.fetch(t, r)
    x, v, epot, ekin = oracle.nve(spec, s.pos, v0, s.species, s.masses, s.box, 1.0, 40)
    print(f"  max |dx|={np.abs(out['pos'] - x).max():.3e}  max |dv|={np.abs(out['vel'] - v).max():.3e}", flush=True)
    np.testing.assert_allclose(out["pos"], x, rtol=0, atol=2e-6)
    np.testing.assert_allclose(out["vel"], v, rtol=0, atol=1e-7)
    assert np.abs(out["epot"] - epot).max() / s.n <= 1e-5
    np.testing.assert_allclose(out["ekin"], ekin, rtol=1e-5, atol=1e-8)
    srv.close()


def test_serve_nve_conserves_energy_across_list_rebuilds(tmd, ctx):
    _note("serve NVE 400 steps")
    _, spec, _ = inputs.workload("oracle32")
    model = tmd.Model(ctx, spec)
    srv = tmd.Server(model, max_slots=1, max_atoms=4096, skin=0.2)
    s = _fcc108()
    v0 = inputs.maxwell_boltzmann(np.full(s.n, CU_MASS), 300.0, seed=74)
    sid = srv.add_system(s.pos, s.species, s.box, s.masses)
    t = srv.submit(sid, tmd.REQ_MD, n_steps=400, dt_fs=1.0, velocities=v0)
    r = srv.wait(t, 120.0)
    assert r["status"] == 0
    out = srv.fetch(t, r)
    etot = out["epot"] + out["ekin"]
    drift = np.abs(etot - etot[0]).max() / s.n
    print(f"  rebuilds={r['rebuilds']} drift/N={drift:.3e}", flush=True)
    assert r["rebuilds"] >= 2
    assert drift <= 1e-4
    srv.close()


def _mix_systems():
    return [
        inputs.make_system("bcc", 3.16, (6, 6, 6), 0.08, 2, seed=80, masses=[183.84, 95.95]),
        inputs.make_system("fcc", 3.61, (8, 8, 8), 0.08, 2, seed=81, masses=[183.84, 95.95]),
        inputs.make_system("bcc", 3.16, (10, 10, 10), 0.08, 2, seed=82, masses=[183.84, 95.95]),
        inputs.make_system("fcc", 3.61, (12, 12, 12), 0.08, 2, seed=83, masses=[183.84, 95.95]),
        inputs.make_system("bcc", 3.16, (16, 16, 16), 0.08, 2, seed=84, masses=[183.84, 95.95]),
    ]


def _a_sequence(tmd, srv, sid, v0):
    ts = [srv.submit(sid), srv.submit(sid, tmd.REQ_MD, 10, 1.0, v0), srv.submit(sid),
          srv.submit(sid, tmd.REQ_MD, 10, 1.0, None)]
    return ts


def test_serve_results_same_alone_and_in_the_mix(tmd, ctx):
    _note("serve alone vs mix")
    s_all = _mix_systems()
    A = s_all[0]
    spec = inputs.make_model(2, 12, 3, [128, 128], 6.0, seed=102)
    model = tmd.Model(ctx, spec, precision=tmd.BF16_MLP)
    mA = np.where(A.species == 0, 183.84, 95.95)
    v0 = inputs.maxwell_boltzmann(mA, 300.0, seed=85)

    srv = tmd.Server(model, max_slots=4, max_atoms=20000, skin=1.0)
    sid = srv.add_system(A.pos, A.species, A.box, A.masses)
    alone = []
    for t in _a_sequence(tmd, srv, sid, v0):
        r = srv.wait(t, 60.0)
        assert r["status"] == 0
        alone.append((r, srv.fetch(t, r)))
    srv.close()

    srv = tmd.Server(model, max_slots=4, max_atoms=20000, skin=1.0)
    ids = [srv.add_system(s.pos, s.species, s.box, s.masses) for s in s_all]
    rng = np.random.default_rng(86)
    others = []
    for k in range(12):
        j = 1 + k % 4
        s = s_all[j]
        if k % 2:
            m = np.where(s.species == 0, 183.84, 95.95)
            others.append(srv.submit(ids[j], tmd.REQ_MD, 10, 1.0,
                                     inputs.maxwell_boltzmann(m, 300.0, seed=int(rng.integers(1 << 30)))))
        else:
            others.append(srv.submit(ids[j]))
        if k == 2:
            a_tickets = _a_sequence(tmd, srv, ids[0], v0)
    mixed = []
    for t in a_tickets:
        r = srv.wait(t, 120.0)
        assert r["status"] == 0
        mixed.append((r, srv.fetch(t, r)))
    spans = []
    for t in others + a_tickets:
        r = srv.wait(t, 120.0)
        assert r["status"] == 0
        spans.append((r["t_start"], r["t_done"]))
    srv.close()
    # forces are summed in fixed point and energies in a fixed order, so the
    # same request on the same state gives the same bits alone and in the mix
    for (ra, oa), (rm, om) in zip(alone, mixed):
        assert ra["energy"] == rm["energy"]
        assert np.array_equal(oa["forces"], om["forces"])
        if ra["kind"] == tmd.REQ_MD:
            assert np.array_equal(oa["pos"], om["pos"])
            assert ra["kinetic"] == rm["kinetic"]
    # requests ran concurrently: some pair of execution intervals overlaps
    spans.sort()
    overlap = any(spans[i + 1][0] < spans[i][1] for i in range(len(spans) - 1))
    assert overlap


def test_serve_same_system_requests_keep_order(tmd, ctx):
    _note("serve per-system order")
    _, spec, _ = inputs.workload("oracle32")
    model = tmd.Model(ctx, spec)
    s = _fcc108()
    v0 = inputs.maxwell_boltzmann(np.full(s.n, CU_MASS), 300.0, seed=87)
    srv = tmd.Server(model, max_slots=4, max_atoms=4096, skin=1.0)
    sid = srv.add_system(s.pos, s.species, s.box, s.masses)
    t1 = srv.submit(sid, tmd.REQ_MD, 10, 1.0, v0)
    t2 = srv.submit(sid, tmd.REQ_MD, 10, 1.0, None)
    r1, r2 = srv.wait(t1, 60.0), srv.wait(t2, 60.0)
    assert r2["t_start"] >= r1["t_done"]
    o2 = srv.fetch(t2, r2)
    srv.close()
    srv = tmd.Server(model, max_slots=1, max_atoms=4096, skin=1.0)
    sid = srv.add_system(s.pos, s.species, s.box, s.masses)
    t = srv.submit(sid, tmd.REQ_MD, 20, 1.0, v0)
    r = srv.wait(t, 60.0)
    o = srv.fetch(t, r)
    srv.close()
    assert np.abs(o["pos"] - o2["pos"]).max() <= 1e-6
    assert np.abs(o["vel"] - o2["vel"]).max() <= 1e-7


def test_serve_admission_by_memory_budget(tmd, ctx):
    _note("serve memory budget")
    _, spec, _ = inputs.workload("oracle32")
    model = tmd.Model(ctx, spec)
    systems = [inputs.make_system("fcc", 3.61, (c, c, c), 0.05, 1, seed=90 + c, masses=[CU_MASS]) for c in (5, 6, 7)]
    # measure the fixed part and the largest list with an unconstrained server,
    # which builds every system's list at registration
    srv = tmd.Server(model, max_slots=2, max_atoms=2048, skin=1.0)
    ids = [srv.add_system(s.pos, s.species, s.box, s.masses) for s in systems]
    total, _ = srv.memory()
    lists = [srv.system_memory(i)[1] for i in ids]
    assert min(lists) > 0
    for i in ids:
        r = srv.wait(srv.submit(i), 60.0)
        assert r["status"] == 0 and r["rebuilds"] == 0  # the list was resident
    assert srv.memory()[0] == total
    srv.close()
    base = total - sum(lists)  # workspaces and system states
    budget = base + max(lists) + 1024  # room for about one list at a time
    srv = tmd.Server(model, max_slots=2, max_atoms=2048, skin=1.0, hbm_budget_bytes=budget)
    ids = [srv.add_system(s.pos, s.species, s.box, s.masses) for s in systems]
    resident = [srv.system_memory(i)[1] > 0 for i in ids]
    assert resident[0] and not all(resident)  # the others wait for their first request
    tickets = [srv.submit(i) for i in ids for _ in range(2)]
    for t, s in zip(tickets, [s for s in systems for _ in range(2)]):
        r = srv.wait(t, 60.0)
        assert r["status"] == 0
        Er, _, _, _ = oracle.energy_forces(spec, s.pos, s.species, s.box)
        assert abs(r["energy"] - Er) / s.n <= 1e-5
    _, peak = srv.memory()
    assert peak <= budget
    srv.close()


def test_serve_input_errors(tmd, ctx):
    _note("serve input errors")
    _, spec, _ = inputs.workload("oracle32")
    model = tmd.Model(ctx, spec)
    srv = tmd.Server(model, max_slots=1, max_atoms=200, skin=1.0)
    s = _fcc108()
    sid = srv.add_system(s.pos, s.species, s.box, s.masses)
    big = inputs.make_system("fcc", 3.61, (4, 4, 4), 0.05, 1, seed=95, masses=[CU_MASS])
    with pytest.raises(tmd.TMDError) as ei:
        srv.add_system(big.pos, big.species, big.box, big.masses)
    assert ei.value.status == 7
    with pytest.raises(tmd.TMDError) as ei:
        srv.submit(sid + 100)
    assert ei.value.status == 1
    with pytest.raises(tmd.TMDError) as ei:
        srv.system_memory(sid + 100)
    assert ei.value.status == 1
    state, lst = srv.system_memory(sid)
    assert state > 0 and lst > 0  # registration built the list
    with pytest.raises(tmd.TMDError) as ei:
        srv.submit(sid, tmd.REQ_MD, 10, 0.0)
    assert ei.value.status == 1
    with pytest.raises(tmd.TMDError) as ei:
        srv.add_system(s.pos, np.full(s.n, 5, dtype=np.int32), s.box, s.masses)
    assert ei.value.status == 1
    srv.close()


def test_serve_batches_small_energy_force_requests(tmd, ctx):
    """Energy-and-force requests on small resident systems are evaluated together
    (batch_atoms): results against the oracle to the FP32 bars, and the same
    bit for bit whatever they were batched with."""
    _note("serve EF batching of small systems vs oracle")
    _, spec, _ = inputs.workload("oracle32")
    model = tmd.Model(ctx, spec)
    srv = tmd.Server(model, max_slots=1, max_atoms=8192, skin=1.0, batch_atoms=1024)
    systems = [_fcc108(), inputs.make_system("bcc", 3.16, (4, 4, 4), 0.1, 1, seed=73, masses=[CU_MASS]),
               inputs.make_system("fcc", 3.61, (2, 2, 3), 0.1, 1, seed=74, masses=[CU_MASS]),
               inputs.make_system("bcc", 3.16, (3, 3, 5), 0.1, 1, seed=75, masses=[CU_MASS]),
               inputs.make_system("fcc", 3.61, (4, 4, 4), 0.05, 1, seed=76, masses=[CU_MASS])]
    ids = [srv.add_system(s.pos, s.species, s.box, s.masses) for s in systems]
    # a larger system whose MD runs keep the one slot busy while a wave queues
    big = inputs.make_system("fcc", 3.61, (6, 6, 6), 0.05, 1, seed=77, masses=[CU_MASS])
    big_id = srv.add_system(big.pos, big.species, big.box, big.masses)
    v0 = inputs.maxwell_boltzmann(np.full(big.n, CU_MASS), 300.0, seed=78)
    # first requests build the resident lists (not batched: no list yet)
    for t in [srv.submit(i) for i in ids]:
        assert srv.wait(t, 60.0)["status"] == 0
    refs = [oracle.energy_forces(spec, s.pos, s.species, s.box) for s in systems]
    seen = {}
    sizes = []
    for wave in range(3):
        order = ids if wave != 1 else ids[::-1]
        order = order if wave != 2 else order[1::2]
        busy = srv.submit(big_id, tmd.REQ_MD, 100, 1.0, v0)
        tickets = [(i, srv.submit(i)) for i in order]
        assert srv.wait(busy, 60.0)["status"] == 0
        for i, t in tickets:
            r = srv.wait(t, 60.0)
            assert r is not None and r["status"] == 0
            sizes.append(r["batch_size"])
            out = srv.fetch(t, r)
            k = ids.index(i)
            s = systems[k]
            Er, _, Fr, Wr = refs[k]
            assert abs(r["energy"] - Er) / s.n <= 1e-5
            assert math.sqrt(np.mean((out["forces"] - Fr) ** 2)) <= 1e-4
            W = np.array(r["virial"])
            Wr6 = np.array([Wr[0, 0], Wr[1, 1], Wr[2, 2], Wr[0, 1], Wr[0, 2], Wr[1, 2]])
            assert np.abs(W - Wr6).max() / s.n <= spec.rcut * 1e-4
            if r["batch_size"] > 1:
                key = (i, "batched")
                if key in seen:
                    assert seen[key][0] == r["energy"]
                    assert np.array_equal(seen[key][1], out["forces"])
                seen[key] = (r["energy"], out["forces"])
    print(f"  batch sizes seen: {sorted(set(sizes))}", flush=True)
    assert max(sizes) > 1
    srv.close()
