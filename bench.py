#!/usr/bin/env python3
"""Benchmark of one TensorMD energy+force step on one MI355X.

A step is the whole hot path on one batch of synthetic input: on-device
cell-list neighbour rebuild, descriptors, per-element MLP forward+backward,
adjoint forces and virial, FP64 totals.  The workload is the 1,024,000-atom
two-element bcc alloy (80^3 cells, a = 3.16 A, sigma = 0.08 A, rcut 6 A,
K = 12, M = 3, MLP 96-128-128-1): value = ns/step/atom with the MLP in BF16
on MFMA; the FP32 path is timed beside it.

Prints one JSON line.  Usage: python bench.py [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ns/step/atom (E+F) at 1M atoms, BF16-MLP vs FP32; serving p50/p99 latency"
PEAK_FP32_VECTOR_TFLOPS = 157.3     # published MI355X FP32 vector peak
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_BF16_MFMA_TFLOPS = 2500.0
PEAK_HBM_GBS = 8000.0
# device memory the serving leg's server may hold: every resident system's
# neighbour list (about 30 GB for the pool of 256) plus the slots' workspaces,
# well within the 288 GB of one MI355X
SERVE_HBM_BUDGET = 96 << 30


def padded_k(K: int) -> int:
    """The radial functions the kernels run for a model of K: the smallest 4, 6
    or 8 times a power of two (at most 64 chunks) that is at least K."""
    def chunked(k):
        return any(k % kc == 0 and (k // kc) & (k // kc - 1) == 0 and k // kc <= 64 for kc in (8, 6, 4))
    return next(k for k in range(max(K, 4), 129) if chunked(k))


def adjoint_unit(spec):
    """The unit that sets the adjoint's pace on a list with a work order: the
    library runs its contractions on the FP32 matrix cores for M = 3 and a
    padded K of 8 or more (4x4x1 MFMAs up to K = 16, 16x16x4 beyond), else on
    the vector ALUs; both peaks are 157.3 TFLOP/s."""
    if spec.max_moment == 3 and padded_k(spec.n_radial) >= 8:
        return "mfma", PEAK_FP32_MFMA_TFLOPS
    return "alu", PEAK_FP32_VECTOR_TFLOPS


def descriptor_unit(spec):
    """The descriptor's contraction runs on the FP32 matrix cores (4x4x1
    MFMAs) for M = 3 and a padded K of 8, 12 or 16, else on the vector ALUs."""
    if spec.max_moment == 3 and padded_k(spec.n_radial) in (8, 12, 16):
        return "mfma", PEAK_FP32_MFMA_TFLOPS
    return "alu", PEAK_FP32_VECTOR_TFLOPS


def algorithmic_flops(spec, n_atoms: int, pairs: int) -> dict:
    """Flops each kernel must perform by the method's definition (2 per FMA).

    descriptor: P = sum_c h_k M_d          -> 2*K*D per pair
    adjoint:    U = P' M and V = P' h       -> 4*K*D per pair
    mlp:        forward 2*(F*H + (L-1)*H*H + H) + backward 2*((L-1)*H*H + H*F) per atom
    """
    K, M = spec.n_radial, spec.max_moment
    D = (M + 1) * (M + 2) * (M + 3) // 6
    F = spec.n_features
    H = spec.hidden[0]
    L = len(spec.hidden)
    mlp = 2 * (F * H + (L - 1) * H * H + H) + 2 * ((L - 1) * H * H + H * F)
    return {"descriptor": 2 * K * D * pairs, "adjoint": 4 * K * D * pairs, "mlp": mlp * n_atoms}


# Profiler scope name -> (rocprofv3 kernel-name prefix, source file of that kernel)
KERNEL_OF_SCOPE = {
    "adjoint": ("k_adjoint", "paper_2310_08439_amd/csrc/descriptor.hip"),
    "descriptor": ("k_descriptor", "paper_2310_08439_amd/csrc/descriptor.hip"),
    "mlp": (("k_mlp_resident", "k_mlp<true"), "paper_2310_08439_amd/csrc/mlp.hip"),  # BF16: resident or staged
    "nb_fill": ("k_fill", "paper_2310_08439_amd/csrc/neighbors.hip"),
}


def measured_traffic(workload: str, scope: str):
    """HBM bytes per launch of a kernel from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary, each counter scaled by its copy-kernel calibration factor.
    None when there is no summary or the kernel's source changed since it was taken."""
    import hashlib
    import re
    if scope not in KERNEL_OF_SCOPE:
        return None
    prefix, src = KERNEL_OF_SCOPE[scope]
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"`" + re.escape(src) + r"`: `([0-9a-f]{64})`", text)
    cur = hashlib.sha256(open(os.path.join(ROOT, src), "rb").read()).hexdigest()
    if not m or m.group(1) != cur:
        return None
    prefixes = (prefix,) if isinstance(prefix, str) else prefix
    for pre in prefixes:
        for line in text.splitlines():
            f = line.split()
            if len(f) == 6 and f[0] == "traffic" and f[1].startswith(pre.replace(" ", "")):
                fetch_kib, write_kib, ff, wf = map(float, f[2:])
                return int(fetch_kib * 1024 * ff + write_kib * 1024 * wf)
    return None


def kernel_rooflines(workload: str, spec, flops: dict, avg_ms: dict) -> dict:
    """Per kernel of the BF16 step: algorithmic TFLOP/s against its unit's peak
    and, from the committed FETCH/WRITE summary (when it matches the source),
    HBM GB/s against 8 TB/s."""
    out = {}
    adj_unit, adj_peak = adjoint_unit(spec)
    desc_unit, desc_peak = descriptor_unit(spec)
    for name, unit, peak in (("adjoint", adj_unit, adj_peak), ("descriptor", desc_unit, desc_peak),
                             ("mlp", "mfma", PEAK_BF16_MFMA_TFLOPS)):
        if name not in avg_ms:
            continue
        sec = avg_ms[name] * 1e-3
        tf = flops[name] / sec / 1e12
        row = {"ms": round(avg_ms[name], 4), "tflops": round(tf, 3), "unit": unit, "peak_tflops": peak,
               "frac_compute": round(tf / peak, 4)}
        traffic = measured_traffic(workload, name) if workload else None
        if traffic is not None:
            gbs = traffic / sec / 1e9
            row.update({"hbm_bytes": traffic, "gb_per_s": round(gbs, 1), "frac_hbm": round(gbs / PEAK_HBM_GBS, 4)})
        out[name] = row
    return out


def _oracle_rate(spec, s, threads: int, seconds: float):
    """(ns/step/atom of the oracle's full E+F, share of it in its brute-force
    neighbour search, repetitions) with `threads` OpenMP threads."""
    import oracle
    oracle.set_num_threads(threads)
    reps, t0 = 0, time.perf_counter()
    while True:
        oracle.energy_forces(spec, s.pos, s.species, s.box)
        reps += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    t1 = time.perf_counter()
    oracle.neighbors(s.pos, s.species, s.box, spec.rcut)
    tn = time.perf_counter() - t1
    return el / (reps * s.n) * 1e9, tn / (el / reps), reps


def cpu_baseline(seconds: float) -> dict:
    """The FP64 oracle (full E+F incl. its brute-force O(N^2) neighbour search)
    on the 4,096-atom sub-cell of the same alloy and model, on every host core
    (value), plus one thread and the other sizes: the 32-atom cell, the
    4,096-atom sub-cell and the 32,000-atom fcc cell (all cores only)."""
    import oracle
    from paper_2310_08439_amd import inputs
    oracle.lib()
    cores = len(os.sched_getaffinity(0))
    s, spec, _ = inputs.workload("bcc4k")
    value, nshare, reps = _oracle_rate(spec, s, cores, seconds)
    runs = []
    for name, thr, secs in (("oracle32", 1, 1.0), ("oracle32", cores, 1.0), ("bcc4k", 1, 2.0), ("fcc32k", cores, 0.0)):
        sx, specx, _ = inputs.workload(name)
        v, sh, r = _oracle_rate(specx, sx, thr, secs)
        runs.append({"workload": name, "atoms": sx.n, "threads": thr, "ns_per_step_atom": round(v, 1),
                     "neighbour_search_share": round(sh, 3), "repetitions": r})
    runs.append({"workload": "bcc4k", "atoms": s.n, "threads": cores, "ns_per_step_atom": round(value, 1),
                 "neighbour_search_share": round(nshare, 3), "repetitions": reps})
    oracle.set_num_threads(cores)
    cpu = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": value, "unit": "ns/step/atom", "cores": cores, "kind": "oracle",
            "sample": f"full FP64 E+F (brute-force neighbours included) of the 4,096-atom bcc sub-cell with the "
                      f"1M-atom workload's model on {cores} threads, {reps} repetitions in about {seconds:.0f} s; "
                      f"host CPU {cpu}",
            "runs": runs}


def train_leg(tmd, torch, ctx, steps: int, warmup: int) -> dict:
    """Force-matching training on the 64-cell fcc/bcc/hcp batch (about 18k atoms,
    descriptor K 8 M 3 rc 5, MLP 32-64-64-1).  Labels come from the GPU FP32
    path with the teacher network (the oracle is not used outside the CPU
    baseline); each timed step is tmd_train_step with an Adam update."""
    import numpy as np
    from paper_2310_08439_amd import inputs
    b = inputs.train_batch()
    _, teacher, _ = inputs.workload("train_teacher")
    _, student, _ = inputs.workload("train_student")
    mt = tmd.Model(ctx, teacher)
    E_l = np.empty(b.n_systems)
    F_l = torch.empty((b.n, 3), dtype=torch.float32, device="cuda")
    pos = torch.tensor(b.pos, dtype=torch.float64, device="cuda")
    sp = torch.tensor(b.species, dtype=torch.int32, device="cuda")
    for s in range(b.n_systems):
        a0, a1 = int(b.sys_off[s]), int(b.sys_off[s + 1])
        nl = tmd.NeighborList(ctx, a1 - a0, 1, 96)
        x, spp = pos[a0:a1].contiguous(), sp[a0:a1].contiguous()
        tmd.build_neighbors(ctx, x, spp, b.boxes[s], teacher.rcut, 0.0, nl)
        E_l[s], _, f, _ = tmd.energy_forces(ctx, mt, x, spp, b.boxes[s], nl, atom_energy=False)
        F_l[a0:a1] = f
        nl.close()
    ms = tmd.Model(ctx, student)
    t0 = time.perf_counter()
    bt = tmd.Batch(ctx, ms, b.sys_off, pos, sp, b.boxes, E_l, F_l)
    t_create = time.perf_counter() - t0
    for _ in range(warmup):
        tmd.train_step(ctx, ms, bt, lr=1e-3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    last = None
    for _ in range(steps):
        last = tmd.train_step(ctx, ms, bt, lr=1e-3)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    bt.close()
    return {"workload": f"{b.n_systems} periodic fcc/bcc/hcp cells, {b.n} atoms, MLP 32-64-64-1, lambda 0.1, Adam lr 1e-3",
            "ms_per_train_step": round(sec * 1e3, 4), "atoms_per_s": round(b.n / sec, 1),
            "batch_setup_ms": round(t_create * 1e3, 2), "loss_after_warmup_and_steps": last[0]}


def serve_leg(tmd, ctx, spec, n_requests: int, n_warmup: int, pool: int, rate: float, slots: int,
              batch_atoms: int = 4096) -> dict:
    """Open-loop Poisson stream against the serving loop: systems are fcc
    (species 0, a = 3.61) or 50/50 bcc alloy (a = 3.16) cells with atom counts
    log-uniform in 64..262,144 (nearest cubic supercell), a pool of `pool`
    resident systems; requests are 50/50 energy+forces or 10 velocity-Verlet
    steps of 1 fs from Maxwell-Boltzmann velocities at 300 K; BF16 MLP.  The
    same systems and request stream are served twice: with energy-and-force
    requests on systems of at most batch_atoms atoms evaluated together
    (reported) and without ("without_batching")."""
    import numpy as np
    from paper_2310_08439_amd import inputs
    rng = np.random.default_rng(4)
    systems = []
    for q in range(pool):
        target = math.exp(rng.uniform(math.log(64), math.log(262144)))
        if rng.random() < 0.5:
            c = min(40, max(2, int(round((target / 4) ** (1 / 3)))))
            s = inputs.make_system("fcc", 3.61, (c, c, c), 0.05, 1, seed=1000 + q, masses=[63.546])
            masses = np.array([63.546, 95.95])
        else:
            c = min(50, max(2, int(round((target / 2) ** (1 / 3)))))
            s = inputs.make_system("bcc", 3.16, (c, c, c), 0.08, 2, seed=1000 + q, masses=[183.84, 95.95])
            masses = np.array([183.84, 95.95])
        systems.append((s, masses, np.where(s.species == 0, masses[0], masses[1])))
    total = n_warmup + n_requests
    plan = []
    t = 0.0
    for k in range(total):
        t += rng.exponential(1.0 / rate)
        q = int(rng.integers(pool))
        md = rng.random() < 0.5
        vel = inputs.maxwell_boltzmann(systems[q][2], 300.0, seed=int(rng.integers(1 << 31))) if md else None
        plan.append((t, q, md, vel))
    # closed loop: a burst of requests drawn the same way, all queued at once,
    # so that every slot stays busy; peak atom-steps/s over the burst
    burst = []
    for k in range(max(1, n_requests // 3)):
        q = int(rng.integers(pool))
        md = rng.random() < 0.5
        vel = inputs.maxwell_boltzmann(systems[q][2], 300.0, seed=int(rng.integers(1 << 31))) if md else None
        burst.append((q, md, vel))
    # small systems only: every system of at most batch_atoms atoms gets four
    # energy-and-force requests, all queued at once (shuffled)
    small = [q for q, (s, _, _) in enumerate(systems) if s.n <= batch_atoms]
    small_burst = [small[k] for k in rng.permutation(np.repeat(np.arange(len(small)), 4))]
    runs = {}
    for ba in (batch_atoms, 0):
        runs[ba] = _serve_run(tmd, ctx, spec, systems, plan, burst, small_burst, n_warmup, slots, ba)
        print(f"[bench] serving batch_atoms={ba}: p50 {runs[ba]['p50_latency_ms']} ms, "
              f"saturation {runs[ba]['closed_loop_saturation']['atom_steps_per_s']:.3g} atom-steps/s",
              file=sys.stderr, flush=True)
    sizes = np.array([s.n for (s, _, _) in systems])
    out = {"workload": f"Poisson {rate:g} req/s, {n_requests} requests after {n_warmup} warm-up, pool of {pool} "
                       f"resident fcc/bcc systems of {sizes.min()}..{sizes.max()} atoms (mean {sizes.mean():.0f}), "
                       f"50% E+F / 50% 10 VV steps, {slots} slots, BF16 MLP, E+F on systems of <= {batch_atoms} "
                       f"atoms batched, HBM budget {SERVE_HBM_BUDGET >> 30} GiB"}
    out.update(runs[batch_atoms])
    out["without_batching"] = runs[0]
    return out


def _serve_run(tmd, ctx, spec, systems, plan, burst, small_burst, n_warmup, slots, batch_atoms) -> dict:
    import numpy as np
    model = tmd.Model(ctx, spec, precision=tmd.BF16_MLP)
    srv = tmd.Server(model, max_slots=slots, max_atoms=262144, skin=1.0, batch_atoms=batch_atoms,
                     hbm_budget_bytes=SERVE_HBM_BUDGET)
    t_reg = time.perf_counter()
    ids = [srv.add_system(s.pos, s.species, s.box, masses) for (s, masses, _) in systems]
    t_reg = time.perf_counter() - t_reg  # uploads and first list builds of the pool
    tickets = []
    start = time.perf_counter()
    for (ta, q, md, vel) in plan:
        delay = start + ta - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        tickets.append(srv.submit(ids[q], tmd.REQ_MD, 10, 1.0, vel) if md else srv.submit(ids[q]))
    results = []
    for tk in tickets:
        r = srv.wait(tk, 300.0)
        if r is None or r["status"] != 0:
            raise RuntimeError(f"serving request failed: {r}")
        results.append(r)
        srv.release(tk)
    t0 = time.perf_counter()
    btk = [srv.submit(ids[q], tmd.REQ_MD, 10, 1.0, vel) if md else srv.submit(ids[q]) for (q, md, vel) in burst]
    bres = []
    for tk in btk:
        r = srv.wait(tk, 300.0)
        if r is None or r["status"] != 0:
            raise RuntimeError(f"serving request failed: {r}")
        bres.append(r)
        srv.release(tk)
    bwall = time.perf_counter() - t0
    saturation = {"requests": len(burst), "wall_s": round(bwall, 3),
                  "atom_steps_per_s": round(sum(r["n_atoms"] * max(1, r["n_steps"]) for r in bres) / bwall, 1)}
    t0 = time.perf_counter()
    stk = [srv.submit(ids[q]) for q in small_burst]
    sres = []
    for tk in stk:
        r = srv.wait(tk, 300.0)
        if r is None or r["status"] != 0:
            raise RuntimeError(f"serving request failed: {r}")
        sres.append(r)
        srv.release(tk)
    swall = time.perf_counter() - t0
    slat = np.array([r["t_done"] - r["t_submit"] for r in sres]) * 1e3
    ssz = np.array([r["batch_size"] for r in sres])
    small_systems = {"requests": len(sres), "wall_s": round(swall, 4),
                     "requests_per_s": round(len(sres) / swall, 1),
                     "atom_steps_per_s": round(sum(r["n_atoms"] for r in sres) / swall, 1),
                     "p50_ms": round(float(np.percentile(slat, 50)), 3),
                     "p99_ms": round(float(np.percentile(slat, 99)), 3),
                     "mean_batch_size": round(float(ssz.mean()), 2),
                     # the server's own span (first start to last completion) and
                     # service time per request; the client's submit and wait calls
                     # (Python, ~30 us per request) bound requests_per_s here
                     "server_span_s": round(max(r["t_done"] for r in sres) - min(r["t_start"] for r in sres), 4),
                     "mean_service_ms": round(float(np.mean([r["t_done"] - r["t_start"] for r in sres])) * 1e3, 3)}
    mem, peak = srv.memory()
    srv.close()
    model.close()
    meas = results[n_warmup:]
    lat = np.array([r["t_done"] - r["t_submit"] for r in meas]) * 1e3
    wall = max(r["t_done"] for r in meas) - min(r["t_submit"] for r in meas)
    atom_steps = sum(r["n_atoms"] * max(1, r["n_steps"]) for r in meas)
    # latency per system-size bucket and request kind
    buckets = {}
    natoms = np.array([r["n_atoms"] for r in meas])
    kinds = np.array([r["kind"] for r in meas])
    for lo, hi in ((0, 1000), (1000, 10000), (10000, 100000), (100000, 1 << 40)):
        for kname, kv in (("ef", tmd.REQ_ENERGY_FORCES), ("md10", tmd.REQ_MD)):
            sel = (natoms >= lo) & (natoms < hi) & (kinds == kv)
            if sel.sum() == 0:
                continue
            key = f"{lo}-{hi if hi < (1 << 40) else 'max'}_atoms_{kname}"
            buckets[key] = {"requests": int(sel.sum()), "p50_ms": round(float(np.percentile(lat[sel], 50)), 3),
                            "p99_ms": round(float(np.percentile(lat[sel], 99)), 3)}
    bsteps = sum(r["n_atoms"] * max(1, r["n_steps"]) for r in bres)
    saturation["ns_per_atom_step"] = round(bwall / bsteps * 1e9, 3)
    bsz = np.array([r["batch_size"] for r in meas + bres])
    return {"p50_latency_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_latency_ms": round(float(np.percentile(lat, 99)), 3),
            "mean_latency_ms": round(float(lat.mean()), 3),
            "atom_steps_per_s": round(atom_steps / wall, 1),
            "closed_loop_saturation": saturation,
            "small_system_ef_burst": small_systems,
            "latency_by_size": buckets,
            "requests_batched": round(float((bsz > 1).mean()), 3),
            "registration_s": round(t_reg, 3),
            "mean_batch_size_of_batched": round(float(bsz[bsz > 1].mean()), 2) if (bsz > 1).any() else None,
            "device_bytes_peak": int(peak)}


def paper_shapes_leg(tmd, torch, ctx, steps: int, warmup: int) -> dict:
    """The paper's own potential shapes (bcc W, one species, K = 32 or 128,
    SquarePlus 128-wide networks; 0 GPa and ~270 GPa lattice constants): E+F with
    the on-device rebuild, ns/step/atom in BF16 and FP32 MLP precision."""
    from paper_2310_08439_amd import inputs
    out = {}
    for name in ("w_k32", "w_k32_hp", "w_k128", "w_k128_hp"):
        s, spec, skin = inputs.workload(name)
        pos = torch.tensor(s.pos, dtype=torch.float64, device="cuda")
        sp = torch.tensor(s.species, dtype=torch.int32, device="cuda")
        ev = tmd.Evaluator(spec, s.n, s.box, skin=skin, precision=tmd.BF16_MLP, ctx=ctx)
        ev.build(pos, sp, s.box)
        pairs, _ = tmd.nlist_stats(ctx, ev.nl)
        row = {"atoms": s.n, "a_A": round(float(s.box[0] / 35 if s.n == 85750 else s.box[0] / 24), 4),
               "K": spec.n_radial, "mlp": f"{spec.n_features}-{'-'.join(map(str, spec.hidden))}-1 squareplus",
               "pairs_per_atom": round(pairs / s.n, 2)}
        flops = algorithmic_flops(spec, s.n, pairs)
        for pname, prec in (("bf16", tmd.BF16_MLP), ("fp32", tmd.FP32)):
            sec, prof, _ = time_precision(tmd, torch, ev, pos, sp, s.box, prec, steps, warmup)
            row[f"ns_per_step_atom_{pname}"] = round(sec / s.n * 1e9, 3)
            if pname == "bf16":
                avg = {k: v[0] / v[1] for k, v in prof.items()}
                row["kernels_roofline_bf16"] = kernel_rooflines(None, spec, flops, avg)
        out[name] = row
        ev.model.close()
        ev.nl.close()
    return out


def md_leg(tmd, torch, ctx, s, spec, steps: int) -> dict:
    """The paper's MD protocol on the 1M-atom alloy: Nose-Hoover NVT at 300 K
    (tau 100 fs), 1 fs steps, 1 A skin rebuilt every 5 steps, thermodynamic
    output every 10 steps, BF16 MLP; whole MD steps timed."""
    import numpy as np
    from paper_2310_08439_amd import inputs
    model = tmd.Model(ctx, spec, precision=tmd.BF16_MLP)
    m = np.where(s.species == 0, s.masses[0], s.masses[1])
    v0 = inputs.maxwell_boltzmann(m, 300.0, seed=7)
    pos = torch.tensor(s.pos, dtype=torch.float64, device="cuda")
    sp = torch.tensor(s.species, dtype=torch.int32, device="cuda")
    vel = torch.tensor(v0, dtype=torch.float64, device="cuda")
    md = tmd.MD(ctx, model, pos, sp, s.box, s.masses, vel, dt_fs=1.0, temperature_K=300.0, tau_fs=100.0,
                skin=1.0, rebuild_every=5)
    md.run(10, thermo_every=10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    th = md.run(steps, thermo_every=10)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    last = th[-1] if th else None  # no record when steps < 10
    md.close()
    model.close()
    return {"workload": f"{s.n} atoms, NVT Nose-Hoover 300 K tau 100 fs, dt 1 fs, skin 1 A rebuilt every 5 steps, "
                        f"thermo every 10 steps, BF16 MLP, {steps} steps",
            "ns_per_step_atom": round(sec / s.n * 1e9, 4), "ms_per_step": round(sec * 1e3, 4),
            "last_thermo": None if last is None else
            {k: (round(v, 6) if isinstance(v, float) else v) for k, v in last.items()}}


def interpolation_leg(tmd, torch, ev, pos, sp, s, spec, steps: int, warmup: int) -> dict:
    """Tabulated radial functions (cubic Hermite table, cutoff folded in) against
    direct evaluation: speed on the main workload (BF16 MLP), for the uniform
    grid (two exponentials per chunk) and for jittered centres (one exponential
    per radial function); static error on 16,000 atoms; dynamic error of E, T
    and P over a 54,000-atom NVT run (the paper's static and dynamic test sizes)."""
    import dataclasses
    import numpy as np
    from paper_2310_08439_amd import inputs
    out = {"scheme": "cubic Hermite, nodes rcut/ceil(rcut/dr) apart, FP32 coefficients"}
    speed = {}

    def timed(evx, label):
        sec, prof, _ = time_precision(tmd, torch, evx, pos, sp, s.box, tmd.BF16_MLP, steps, warmup)
        speed[label] = {"ns_per_step_atom": round(sec / s.n * 1e9, 4),
                        "descriptor_ms": round(prof["descriptor"][0] / prof["descriptor"][1], 4),
                        "adjoint_ms": round(prof["adjoint"][0] / prof["adjoint"][1], 4)}

    timed(ev, "direct_uniform_grid")
    for dr in (0.01, 0.001):
        ev.model.tabulate(dr)
        timed(ev, f"table_dr{dr:g}")
    ev.model.tabulate(0.0)
    rng = np.random.default_rng(9)
    jit = dataclasses.replace(spec, mu=spec.mu + rng.uniform(-0.02, 0.02, size=spec.mu.shape))
    evj = tmd.Evaluator(jit, s.n, s.box, precision=tmd.BF16_MLP, ctx=ev.ctx)
    timed(evj, "direct_jittered_grid")
    evj.model.tabulate(0.01)
    timed(evj, "table_dr0.01_jittered_grid")
    evj.model.close()
    evj.nl.close()
    out["speed"] = speed

    st = inputs.make_system("bcc", 3.16, (20, 20, 20), 0.08, 2, seed=155)
    pst = torch.tensor(st.pos, dtype=torch.float64, device="cuda")
    sst = torch.tensor(st.species, dtype=torch.int32, device="cuda")
    evs = tmd.Evaluator(spec, st.n, st.box, precision=tmd.FP32, ctx=ev.ctx)
    E0, _, F0, _ = evs.energy_forces(pst, sst, st.box)
    F0 = F0.cpu().numpy().astype(np.float64)
    static = {}
    for dr in (0.1, 0.05, 0.01, 0.005, 0.001):
        evs.model.tabulate(dr)
        E, _, F, _ = evs.energy_forces(pst, sst, st.box)
        F = F.cpu().numpy().astype(np.float64)
        static[f"{dr:g}"] = {"force_rmse_eV_per_A": float(math.sqrt(np.mean((F - F0) ** 2))),
                             "energy_err_eV_per_atom": float(abs(E - E0) / st.n)}
    evs.model.close()
    evs.nl.close()
    out["static_16000_atoms_fp32"] = static

    sd = inputs.make_system("bcc", 3.16, (30, 30, 30), 0.05, 2, seed=160, masses=[183.84, 95.95])
    m = np.where(sd.species == 0, sd.masses[0], sd.masses[1])
    v0 = inputs.maxwell_boltzmann(m, 300.0, seed=161)
    series = {}
    for dr in (0.0, 0.01, 0.001):
        model = tmd.Model(ev.ctx, dataclasses.replace(spec, tab_dr=dr), precision=tmd.FP32)
        md = tmd.MD(ev.ctx, model, torch.tensor(sd.pos, dtype=torch.float64, device="cuda"),
                    torch.tensor(sd.species, dtype=torch.int32, device="cuda"), sd.box, sd.masses,
                    torch.tensor(v0, dtype=torch.float64, device="cuda"), dt_fs=1.0, temperature_K=300.0,
                    tau_fs=100.0, skin=1.0, rebuild_every=5)
        th = md.run(1000, thermo_every=10)
        series[dr] = np.array([[t["etotal"] / sd.n, t["temperature_K"], t["pressure_GPa"]] for t in th])
        md.close()
        model.close()
    dyn = {}
    for dr in (0.01, 0.001):
        d = series[dr] - series[0.0]
        dyn[f"{dr:g}"] = {"etotal_rmse_eV_per_atom": float(math.sqrt(np.mean(d[:, 0] ** 2))),
                          "temperature_rmse_K": float(math.sqrt(np.mean(d[:, 1] ** 2))),
                          "pressure_rmse_GPa": float(math.sqrt(np.mean(d[:, 2] ** 2)))}
    out["dynamic_54000_atoms_nvt_1000_steps_fp32"] = dyn
    return out


def accuracy(tmd, ev, pos, sp, s, spec, n_sample: int, precision: int) -> dict:
    """Per-atom energy and force errors against the FP64 oracle on n_sample
    atoms: a compact sample cut out of the system with every atom within
    2 rcut + 0.5 A of it (inputs.cluster_cut), so that the oracle evaluates the
    piece exactly as it would the whole periodic system for those atoms.
    Reports the mean signed error of E_i (the energy bias per atom at full
    size, sampled) and, for BF16, the oracle's BF16 form beside it."""
    import numpy as np
    import oracle
    from paper_2310_08439_amd import inputs
    ev.model.set_precision(precision)
    E, Ea, F, _ = ev.energy_forces(pos, sp, s.box)
    Ea = Ea.cpu().numpy().astype(np.float64)
    F = F.cpu().numpy().astype(np.float64)
    centre = int(np.random.default_rng(1234).integers(s.n))
    t0 = time.perf_counter()
    piece, sample, where = inputs.cluster_cut(s, centre, n_sample, 2.0 * spec.rcut + 0.5)
    _, Ear, Fr, _ = oracle.energy_forces(spec, piece.pos, piece.species, piece.box)
    Ear, Fr = Ear[where], Fr[where]
    dE = Ea[sample] - Ear
    dF = F[sample] - Fr
    out = {"sampled_atoms": int(len(sample)), "piece_atoms": int(piece.n),
           "mean_signed_dE_atom_eV": float(dE.mean()), "max_abs_dE_atom_eV": float(np.abs(dE).max()),
           "force_rms_err_eV_per_A": float(math.sqrt(np.mean(dF ** 2))),
           "force_max_abs_err_eV_per_A": float(np.abs(dF).max()),
           "force_rms_eV_per_A": float(math.sqrt(np.mean(Fr ** 2)))}
    if precision == tmd.BF16_MLP:
        _, Ea16, F16, _ = oracle.energy_forces(spec, piece.pos, piece.species, piece.box, bf16=True)
        out["oracle_bf16_form_mean_signed_dE_atom_eV"] = float((Ea16[where] - Ear).mean())
        out["vs_bf16_form_median_abs_dE_atom_eV"] = float(np.median(np.abs(Ea[sample] - Ea16[where])))
    out["oracle_seconds"] = round(time.perf_counter() - t0, 2)
    return out


def time_precision(tmd, torch, ev, pos, sp, box, precision, steps, warmup):
    ev.model.set_precision(precision)
    for _ in range(warmup):
        ev.build(pos, sp, box)
        ev.energy_forces(pos, sp, box, rebuild=False, atom_energy=False)
    torch.cuda.synchronize()
    ev.ctx.profile_reset()
    ev.ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ev.build(pos, sp, box)
        E, _, F, W = ev.energy_forces(pos, sp, box, rebuild=False, atom_energy=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ev.ctx.profile(False)
    prof = ev.ctx.profile_read()
    return (t1 - t0) / steps, prof, E


def time_no_rebuild(tmd, torch, ev, pos, sp, box, precision, steps, warmup):
    """E+F alone on the list built beforehand (no rebuild inside the timed region)."""
    ev.model.set_precision(precision)
    ev.build(pos, sp, box)
    for _ in range(warmup):
        ev.energy_forces(pos, sp, box, rebuild=False, atom_energy=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ev.energy_forces(pos, sp, box, rebuild=False, atom_energy=False)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def whole_path_bound(spec, n_atoms: int, pairs: int) -> float:
    """Seconds the E+F path needs at the published peaks: the contraction flops
    of descriptor and adjoint (6*K*D per pair) on the FP32 vector units or the
    minimum bytes per atom (positions 24, species 4, list 4 per pair, forces 12,
    energy 4) from HBM, whichever is longer, plus the MLP flops on BF16 MFMA."""
    f = algorithmic_flops(spec, n_atoms, pairs)
    desc = (f["descriptor"] + f["adjoint"]) / (PEAK_FP32_VECTOR_TFLOPS * 1e12)
    hbm = n_atoms * (24 + 4 + 12 + 4 + 4 * pairs / n_atoms) / (PEAK_HBM_GBS * 1e9)
    return max(desc, hbm) + f["mlp"] / (PEAK_BF16_MFMA_TFLOPS * 1e12)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="bcc1m", choices=["bcc1m", "fcc32k", "bcc4k"])
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--accuracy-samples", type=int, default=2000)
    ap.add_argument("--train-steps", type=int, default=20)
    ap.add_argument("--md-steps", type=int, default=50)
    ap.add_argument("--serve-requests", type=int, default=600)
    ap.add_argument("--serve-warmup", type=int, default=100)
    ap.add_argument("--serve-pool", type=int, default=256)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--no-extra", action="store_true", help="skip the training and serving legs")
    ap.add_argument("--mode", default="step", choices=["step", "copy", "paper"],
                    help="copy: 3 device copies of 1 GiB, to calibrate HBM byte counters; "
                         "paper: only the paper-shaped workloads (for profiling their kernels)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the multi-GPU (spatial decomposition) path is a design, "
              "not part of this build; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2310_08439_amd import inputs, tmd

    if args.mode == "copy":
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "copy", "bytes_read_per_copy": src.numel() * 4,
                          "bytes_written_per_copy": dst.numel() * 4}), flush=True)
        return
    if args.mode == "paper":
        ctx = tmd.Context(0)
        print(json.dumps({"mode": "paper", "paper_shapes": paper_shapes_leg(tmd, torch, ctx, args.steps,
                                                                             args.warmup)}), flush=True)
        ctx.close()
        return

    s, spec, skin = inputs.workload(args.workload)
    pos = torch.tensor(s.pos, dtype=torch.float64, device="cuda")
    sp = torch.tensor(s.species, dtype=torch.int32, device="cuda")
    ev = tmd.Evaluator(spec, s.n, s.box, skin=skin, precision=tmd.BF16_MLP)
    ev.build(pos, sp, s.box)
    pairs, max_row = tmd.nlist_stats(ev.ctx, ev.nl)

    res = {}
    for name, prec in (("bf16", tmd.BF16_MLP), ("fp32", tmd.FP32)):
        sec, prof, E = time_precision(tmd, torch, ev, pos, sp, s.box, prec, args.steps, args.warmup)
        res[name] = {"sec": sec, "prof": prof, "E": E}

    no_rebuild = {name: time_no_rebuild(tmd, torch, ev, pos, sp, s.box, prec, args.steps, args.warmup)
                  for name, prec in (("bf16", tmd.BF16_MLP), ("fp32", tmd.FP32))}
    ev.model.set_precision(tmd.BF16_MLP)
    t_bound = whole_path_bound(spec, s.n, pairs)

    flops = algorithmic_flops(spec, s.n, pairs)
    prof = res["bf16"]["prof"]
    avg_ms = {k: v[0] / v[1] for k, v in prof.items()}
    dom = max(avg_ms, key=avg_ms.get)
    if dom in flops:
        if dom == "mlp":
            bound, peak = "mfma", PEAK_BF16_MFMA_TFLOPS
        elif dom == "adjoint":
            bound, peak = adjoint_unit(spec)
        else:
            bound, peak = "alu", PEAK_FP32_VECTOR_TFLOPS
        achieved = flops[dom] / (avg_ms[dom] * 1e-3) / 1e12
        roof = {"bound": bound, "kernel": dom, "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4), "traffic": measured_traffic(args.workload, dom),
                "algorithmic_flops_per_launch": int(flops[dom]), "avg_launch_ms": round(avg_ms[dom], 4)}
    else:
        roof = {"bound": "hbm", "kernel": dom, "achieved": None, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": None,
                "traffic": None}

    acc = {}
    if args.accuracy_samples > 0:
        for name, prec in (("bf16", tmd.BF16_MLP), ("fp32", tmd.FP32)):
            acc[name] = accuracy(tmd, ev, pos, sp, s, spec, args.accuracy_samples, prec)

    training = serving = shapes = md = interp = None
    if not args.no_extra:
        md = md_leg(tmd, torch, ev.ctx, s, spec, args.md_steps)
        print(f"[bench] md {md}", file=sys.stderr, flush=True)
        interp = interpolation_leg(tmd, torch, ev, pos, sp, s, spec, 10, 2)
        print(f"[bench] interpolation {interp}", file=sys.stderr, flush=True)
        shapes = paper_shapes_leg(tmd, torch, ev.ctx, 10, 2)
        print(f"[bench] paper shapes {shapes}", file=sys.stderr, flush=True)
        training = train_leg(tmd, torch, ev.ctx, args.train_steps, 2)
        print(f"[bench] training {training}", file=sys.stderr, flush=True)
        serving = serve_leg(tmd, ev.ctx, spec, args.serve_requests, args.serve_warmup, args.serve_pool,
                            args.serve_rate, args.serve_slots)
        print(f"[bench] serving {serving}", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.cpu_seconds)

    ns_bf16 = res["bf16"]["sec"] / s.n * 1e9
    ns_fp32 = res["fp32"]["sec"] / s.n * 1e9
    kernels = {}
    for name in ("bf16", "fp32"):
        kernels[name] = {k: round(v[0] / v[1], 4) for k, v in sorted(res[name]["prof"].items())}
    line = {
        "metric": METRIC,
        "value": round(ns_bf16, 4),
        "unit": "ns/step/atom",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(res["bf16"]["sec"] * 1e3, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16-mlp/fp32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {s.n} atoms, box {s.box[0]:.2f} A, rcut {spec.rcut}, "
                               f"K {spec.n_radial}, M {spec.max_moment}, S {spec.n_species}, "
                               f"MLP {spec.n_features}-{'-'.join(map(str, spec.hidden))}-1, neighbour rebuild each step",
                   "atoms": s.n, "pairs": pairs, "max_row": max_row, "parallelism": "single GPU"},
        "fp32": {"ns_per_step_atom": round(ns_fp32, 4), "ms_per_step": round(res["fp32"]["sec"] * 1e3, 4)},
        "bf16_speedup_vs_fp32": round(ns_fp32 / ns_bf16, 4),
        "without_rebuild": {name: {"ns_per_step_atom": round(t / s.n * 1e9, 4), "ms_per_step": round(t * 1e3, 4)}
                            for name, t in no_rebuild.items()},
        "whole_path_bound": {"t_bound_ms": round(t_bound * 1e3, 4),
                             "frac_with_rebuild": round(t_bound / res["bf16"]["sec"], 4),
                             "frac_without_rebuild": round(t_bound / no_rebuild["bf16"], 4),
                             "basis": f"max(6KD flops/pair on 157.3 TF FP32 vector, "
                                      f"{44 + 4 * pairs / s.n:.0f} B/atom on 8 TB/s) + MLP flops on 2.5 PF BF16 MFMA"},
        "energy_per_atom": {"bf16": res["bf16"]["E"] / s.n, "fp32": res["fp32"]["E"] / s.n},
        "kernels_avg_ms": kernels,
        "accuracy_vs_oracle": acc,
        "roofline": roof,
        "kernels_roofline": kernel_rooflines(args.workload, spec, flops, avg_ms),
        "cpu_baseline": cpu,
        "serving": serving,
        "training": training,
        "paper_shapes": shapes,
        "md": md,
        "interpolation": interp,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
