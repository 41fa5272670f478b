"""Molecular dynamics driver (tmd_md_*) on the GPU against the FP64 oracle.

Bars: 20 steps of 1 fs against the oracle's velocity Verlet / Nose-Hoover
integrators: positions within 1e-6 A, velocities within 1e-7 A/fs (the FP32
forces differ from FP64 by ~1e-6 eV/A here, which moves a 63.5 amu atom by
~1e-9 A in 20 fs), energies per atom within 1e-5 eV; the thermostat
variable integrates the kinetic energy's error: each step adds
dt G = dt (2 KE - 3 N kB T) / Q to xi, so xi - xi_ref is at most
2 dt sum_steps |KE - KE_ref| / Q (bar: 1.5 times that, the kinetic energies
of the thermo records standing in for those of the half steps, plus 1e-6 of
|xi|), and eta - eta_ref at most n dt times xi's bar; pressure within
N r_c F_tol / V (the virial bar) converted to GPa; a 2,000-step NVT run keeps
its extended energy within 2e-4 eV/atom and its mean temperature within
15 % of the target (32 to 108 atoms fluctuate by ~10 %).
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2310_08439_amd import inputs

pytestmark = pytest.mark.gpu

CU = 63.546
KB = 8.617333262e-5
GPA = 160.21766208


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


def _dev(torch, s, v):
    return (torch.tensor(s.pos, dtype=torch.float64, device="cuda"),
            torch.tensor(s.species, dtype=torch.int32, device="cuda"),
            torch.tensor(v, dtype=torch.float64, device="cuda"))


@pytest.mark.parametrize("ensemble", ["nvt", "nve"])
def test_md_matches_oracle_integrator(tmd, ctx, torch, ensemble):
    _note(f"MD {ensemble} vs oracle, 20 steps")
    s, spec, _ = inputs.workload("oracle32")
    v0 = inputs.maxwell_boltzmann(np.full(s.n, CU), 300.0, seed=60)
    model = tmd.Model(ctx, spec)
    pos, sp, vel = _dev(torch, s, v0)
    ens = tmd.ENSEMBLE_NVT_NOSE_HOOVER if ensemble == "nvt" else tmd.ENSEMBLE_NVE
    md = tmd.MD(ctx, model, pos, sp, s.box, s.masses, vel, dt_fs=1.0, ensemble=ens, temperature_K=300.0,
                tau_fs=20.0, skin=1.0, rebuild_every=0)
    th = md.run(20, thermo_every=1)
    x, v = (t.cpu().numpy() for t in md.state())
    if ensemble == "nvt":
        xr, vr, (xi, eta), epot, ekin, cons = oracle.nvt(spec, s.pos, v0, s.species, s.masses, s.box, 1.0, 300.0,
                                                          20.0, 20)
        xi_g, eta_g = md.thermostat()
        ek_g = np.array([t["ekin"] for t in th])
        Q = 3 * s.n * KB * 300.0 * 20.0 ** 2
        xi_bar = 1.5 * 2.0 * 1.0 * np.abs(ek_g - ekin).sum() / Q + 1e-6 * abs(xi)
        print(f"  |dxi|={abs(xi_g - xi):.3e} (bar {xi_bar:.3e})  |deta|={abs(eta_g - eta):.3e}", flush=True)
        assert abs(xi_g - xi) <= xi_bar
        assert abs(eta_g - eta) <= 20 * 1.0 * xi_bar + 1e-6 * abs(eta)
    else:
        xr, vr, epot, ekin = oracle.nve(spec, s.pos, v0, s.species, s.masses, s.box, 1.0, 20)
        cons = epot + ekin
    print(f"  max |dx|={np.abs(x - xr).max():.3e}  max |dv|={np.abs(v - vr).max():.3e}", flush=True)
    np.testing.assert_allclose(x, xr, rtol=0, atol=1e-6)
    np.testing.assert_allclose(v, vr, rtol=0, atol=1e-7)
    assert len(th) == 21 and [t["step"] for t in th] == list(range(21))
    ep = np.array([t["epot"] for t in th])
    ek = np.array([t["ekin"] for t in th])
    co = np.array([t["conserved"] for t in th])
    assert np.abs(ep - epot).max() / s.n <= 1e-5
    np.testing.assert_allclose(ek, ekin, rtol=1e-5, atol=1e-9)
    assert np.abs(co - cons).max() / s.n <= 1e-5
    T = np.array([t["temperature_K"] for t in th])
    np.testing.assert_allclose(T, 2 * ekin / (3 * s.n * KB), rtol=1e-5)
    md.close()


def test_md_pressure_matches_oracle(tmd, ctx, torch):
    _note("MD thermo pressure")
    s, spec, _ = inputs.workload("oracle32")
    v0 = inputs.maxwell_boltzmann(np.full(s.n, CU), 300.0, seed=61)
    model = tmd.Model(ctx, spec)
    pos, sp, vel = _dev(torch, s, v0)
    md = tmd.MD(ctx, model, pos, sp, s.box, s.masses, vel, ensemble=tmd.ENSEMBLE_NVE)
    th = md.run(0, thermo_every=1)
    p = oracle.pressure(spec, s.pos, v0, s.species, s.masses, s.box)
    V = float(np.prod(s.box))
    bar = s.n * spec.rcut * 1e-4 / V * GPA
    got = np.array([th[0]["pxx_GPa"], th[0]["pyy_GPa"], th[0]["pzz_GPa"], th[0]["pressure_GPa"]])
    print(f"  P={got[3]:.4f} GPa vs {p[3]:.4f} (bar {bar:.2e})", flush=True)
    assert np.abs(got - p).max() <= bar
    assert abs(th[0]["volume_A3"] - V) <= 1e-9 * V
    md.close()


def test_md_periodic_rebuild_equals_displacement_rule(tmd, ctx, torch):
    """With a 1 A skin, rebuilding every 5 steps and rebuilding on displacement
    give the same trajectory (skin entries contribute exactly zero)."""
    _note("MD rebuild policies")
    s = inputs.make_system("fcc", 3.61, (3, 3, 3), 0.1, 1, seed=62, masses=[CU])
    _, spec, _ = inputs.workload("oracle32")
    v0 = inputs.maxwell_boltzmann(np.full(s.n, CU), 300.0, seed=63)
    model = tmd.Model(ctx, spec)
    out = []
    for every in (5, 0):
        pos, sp, vel = _dev(torch, s, v0)
        md = tmd.MD(ctx, model, pos, sp, s.box, s.masses, vel, skin=1.0, rebuild_every=every, tau_fs=50.0)
        th = md.run(50, thermo_every=10)
        out.append((md.state()[0].cpu().numpy(), th[-1]))
        md.close()
    assert out[0][1]["rebuilds"] == 11  # the first build and one every 5 steps
    assert np.abs(out[0][0] - out[1][0]).max() <= 1e-6
    assert abs(out[0][1]["etotal"] - out[1][1]["etotal"]) <= 1e-6 * s.n


@pytest.mark.parametrize("rebuild_every", [0, 30])
def test_md_reused_pruned_rows_follow_a_fast_atom(tmd, ctx, torch, rebuild_every):
    """The MD driver prunes a skin list to r_c + skin/5 and reuses those rows
    until the displacement since the build could have brought a dropped pair
    inside r_c.  One atom crosses 0.75 A in 15 steps (the threshold is 0.2 A,
    and the list itself is rebuilt only after 1 A or 30 steps): the trajectory
    must still follow the oracle's, which has no lists to reuse."""
    _note(f"MD fast atom, pruned rows reused, rebuild_every={rebuild_every}")
    s, spec, _ = inputs.workload("oracle32")
    v0 = inputs.maxwell_boltzmann(np.full(s.n, CU), 300.0, seed=66)
    v0[5] = [0.05, -0.01, 0.02]  # A/fs
    model = tmd.Model(ctx, spec)
    pos, sp, vel = _dev(torch, s, v0)
    md = tmd.MD(ctx, model, pos, sp, s.box, s.masses, vel, dt_fs=1.0, ensemble=tmd.ENSEMBLE_NVE, skin=2.0,
                rebuild_every=rebuild_every)
    th = md.run(15, thermo_every=15)
    x, v = (t.cpu().numpy() for t in md.state())
    xr, vr, epot, ekin = oracle.nve(spec, s.pos, v0, s.species, s.masses, s.box, 1.0, 15)
    print(f"  max |dx|={np.abs(x - xr).max():.3e}  rebuilds={th[-1]['rebuilds']}", flush=True)
    assert th[-1]["rebuilds"] == 1  # the first build only: every other step reused the list
    np.testing.assert_allclose(x, xr, rtol=0, atol=1e-6)
    np.testing.assert_allclose(v, vr, rtol=0, atol=1e-7)
    assert abs(th[-1]["epot"] - epot[-1]) / s.n <= 1e-5
    md.close()


def test_md_nvt_long_run(tmd, ctx, torch):
    _note("MD NVT 2000 steps")
    s = inputs.make_system("fcc", 3.61, (3, 3, 3), 0.1, 1, seed=64, masses=[CU])
    _, spec, _ = inputs.workload("oracle32")
    v0 = inputs.maxwell_boltzmann(np.full(s.n, CU), 300.0, seed=65)
    model = tmd.Model(ctx, spec)
    pos, sp, vel = _dev(torch, s, v0)
    md = tmd.MD(ctx, model, pos, sp, s.box, s.masses, vel, tau_fs=50.0, skin=1.0, rebuild_every=5)
    th = md.run(2000, thermo_every=10)
    co = np.array([t["conserved"] for t in th])
    T = np.array([t["temperature_K"] for t in th])
    drift = np.abs(co - co[0]).max() / s.n
    print(f"  drift/N={drift:.3e}  <T>={T[len(T) // 2:].mean():.1f} K  rebuilds={th[-1]['rebuilds']}", flush=True)
    assert drift <= 2e-4
    assert 255.0 <= T[len(T) // 2:].mean() <= 345.0
    md.close()


def test_md_input_errors(tmd, ctx, torch):
    _note("MD input errors")
    s, spec, _ = inputs.workload("oracle32")
    model = tmd.Model(ctx, spec)
    pos = torch.tensor(s.pos, dtype=torch.float64, device="cuda")
    sp = torch.tensor(s.species, dtype=torch.int32, device="cuda")
    for kw in ({"dt_fs": 0.0}, {"temperature_K": -1.0}, {"rebuild_every": -1}, {"skin": -0.5}):
        with pytest.raises(tmd.TMDError) as ei:
            tmd.MD(ctx, model, pos, sp, s.box, s.masses, **kw)
        assert ei.value.status == 1
