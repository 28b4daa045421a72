#!/usr/bin/env python
"""Benchmark: grid solves per second + energies at 256^3 (FP32 vs FP64) on one MI355X.

Workload (mixed_256): periodic 256^3 cell, 80 nm side, cubic iron-like stiffness
C11/C12/C44 = 243/145/116 GPa, 2000 synthetic defects (70 % 1/2<111> loops,
10 % <100> loops, 20 % dilatational spheres; seeded).  One step is the whole
hot path from the defect list: rasterise, forward FFT, Green operator, inverse
FFT + stress, per-defect self terms and the compensated energy reduction,
ending with the energies on the host.  Nothing in the step reads the stress
away from the defects, so the solves store it at the covered voxels only (the
library forms the rest when a call needs it; see include/ec.h).  ``value`` is FP32-storage steps/s;
FP64 steps/s and the per-defect FP32 error against the FP64 path are reported
beside it.  Inputs are resident on the device when timing starts.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak, GB/s


# sources of the FFT-pass kernels (the families the roofline line can name)
FFT_SOURCES = ("ec_internal.h", "fft_core.h", "k_fft.hip")


def kernel_source_sha():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2403_09158_amd", "csrc")
    for f in FFT_SOURCES:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_for(family, sha):
    """HBM bytes per launch of `family` from committed rocprofv3 counter runs,
    or None if absent or taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            t = json.load(fh)
    except OSError:
        return None
    if t.get("source_sha") != sha or family not in t.get("families", {}):
        return None
    return t["families"][family]


def timed_steps(st, defs, steps, warmup, profile, families=None):
    """`steps` solve + energies steps after `warmup` untimed ones; with
    `profile`, HIP events bracket the launches of `families` (None: all)."""
    import torch

    for _ in range(warmup):
        st.solve(defs)
        st.energies()
    torch.cuda.synchronize()
    st.profile(profile, families)
    st.profile_read()  # drop warmup records
    t0 = time.perf_counter()
    for _ in range(steps):
        st.solve(defs)
        E = st.energies()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = st.profile_read() if profile else None
    st.profile(False)
    return dt, E, prof


def cpu_baseline(prob, defs, green_planes=16, self_sample=100):
    """The FP64 oracle on a bounded sample of the same workload, extrapolated to
    one full solve + energies: full rasterisation and FFTs, the Green step on
    `green_planes` of n z-planes (scaled by n/green_planes), the stress, the
    footprint sums for all defects and the self terms of `self_sample` defects
    (scaled).  The kernel window G (a per-problem setup, six extra solves) is
    excluded."""
    import numpy as np

    from oracle import elastic, energy, raster, solve

    n = prob.n
    C = elastic.stiffness_of(prob)
    T = {}
    t = time.perf_counter()
    fps, Es = raster.rasterise(prob, defs)
    es = raster.eigenstrain_field(n, fps, Es)
    T["raster"] = time.perf_counter() - t
    t = time.perf_counter()
    tau = np.einsum("ijkl,kl...->ij...", C, es)
    t_f = time.perf_counter()
    th = solve.fft3(tau)
    fft_many = time.perf_counter() - t_f
    T["forward"] = time.perf_counter() - t
    # the transforms are the only multi-threaded stages: timed again on one worker
    T1 = {}
    t = time.perf_counter()
    solve.fft3(tau, workers=1)
    T1["forward_fft"] = time.perf_counter() - t
    del tau
    planes = list(range(0, n, n // green_planes))[:green_planes]
    t = time.perf_counter()
    eh = solve.apply_green(C, prob.L, th, es.sum(axis=(-3, -2, -1)), prob.bc, planes=planes)
    T["green"] = (time.perf_counter() - t) * n / len(planes)
    del th
    t = time.perf_counter()
    solve.fft3(eh, inverse=True, workers=1)
    T1["inverse_fft"] = time.perf_counter() - t
    t = time.perf_counter()
    eps_c = solve.fft3(eh, inverse=True)
    fft_many += time.perf_counter() - t
    eps = eps_c.real
    del eh, eps_c
    sig = np.einsum("ijkl,kl...->ij...", C, eps - es)
    T["inverse_stress"] = time.perf_counter() - t
    del eps
    t = time.perf_counter()
    sf = sig.reshape(3, 3, -1)
    S = [sf[:, :, ids].sum(axis=-1) for ids in fps]
    T["footprint_sums"] = time.perf_counter() - t
    # self terms need G; time them on a small synthetic window (values irrelevant)
    D = energy.window_halfwidth(fps, n)
    G = np.zeros((3, 3, 3, 3, 2 * D + 1, 2 * D + 1, 2 * D + 1))
    idx = np.linspace(0, len(fps) - 1, self_sample).astype(int)
    h3c = prob.h**3 * elastic.GPA_NM3_EV
    t = time.perf_counter()
    for i in idx:
        energy.self_term(fps[i], Es[i], G, D, n, h3c)
    T["self_terms"] = (time.perf_counter() - t) * len(fps) / len(idx)
    del sig, S
    total = sum(T.values())
    # one worker: the transform time of the forward and inverse stages replaced
    # by their single-worker time (the rest of the oracle runs on one thread)
    t_fft_many = T1["forward_fft"] + T1["inverse_fft"]
    total_1 = total - fft_many + t_fft_many
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {
        "value": 1.0 / total,
        "unit": "solves/s",
        "cores": int(os.environ.get("ORACLE_FFT_WORKERS", "0")) or (os.cpu_count() or 1),
        "cpu_model": cpu,
        "one_worker": {"value": 1.0 / total_1, "fft_s": {k: round(v, 2) for k, v in T1.items()},
                       "fft_s_all_workers": round(fft_many, 2)},
        "kind": "oracle",
        "sample": (
            f"mixed_256 workload at 256^3: full rasterisation, FFTs and footprint sums; Green step on "
            f"{len(planes)}/{n} z-planes and self terms of {len(idx)}/{len(fps)} defects, scaled; "
            f"G-window setup excluded; per-stage s: " + ", ".join(f"{k}={v:.2f}" for k, v in T.items())
        ),
    }


def family_table(prof):
    return {k: {"launches": v["launches"], "avg_ms": round(v["ms"] / max(v["launches"], 1), 5),
                "GBps": round(v["bytes_per_launch"] / max(v["ms"] / max(v["launches"], 1), 1e-9) / 1e6, 1)}
            for k, v in prof.items() if v["launches"]}


def energy_errors(E32, E64):
    import numpy as np

    err = np.abs(E32 - E64)
    tol = np.maximum(1e-4 * np.abs(E64), 1e-5)
    return {
        "max_abs_eV": float(err.max()),
        "p50_abs_eV": float(np.median(err)),
        "p99_abs_eV": float(np.quantile(err, 0.99)),
        "pass_fraction": float(np.mean(err <= tol)),
        "max_err_over_tol": float(np.max(err / tol)),
    }


def serving_block(nreq=4000, rate=2000.0, slots=4, plain_req=1000, budget_gb=200.0):
    """Serving workload: 64 replicas (grids 64-240, 50-1500 defects), Poisson
    arrivals, 90 % one-defect hops, 10 % re-solves, admitted against a 200 GB
    HBM budget; ready hops of one grid shape are batched and replayed from HIP
    graphs."""
    import numpy as np

    from paper_2403_09158_amd import ec, inputs, serve

    reps = inputs.serving_replicas(64, prec=1)
    out = {
        "workload": "serving: 64 replicas, n ~ U{64,96,128,160,240}, 50-1500 defects each (mixed_256 mix), "
        f"Poisson {rate:.0f} req/s, 90% (+-1,+-1,+-1) hops of a random defect, 10% re-solves",
        "slots": slots,
    }
    out["hbm_budget_gb"] = budget_gb
    ctx = ec.Context(0, budget_bytes=int(budget_gb * 1e9))
    srv = serve.Server(ctx, reps, slots=slots)
    srv.warm()
    st = srv.run(serve.serving_requests(reps, nreq, rate), realtime=True)
    out["fp32_served"] = {"requests": nreq, "throughput_req_s": round(st.throughput, 1), "p50_ms": round(st.p50_ms, 4),
                          "p99_ms": round(st.p99_ms, 4), "mean_ms": round(st.mean_ms, 4), "batches": st.batches,
                          "by_grid": st.by_grid()}
    st = srv.run(serve.serving_requests(reps, 3000, 1e9), realtime=False)
    out["fp32_saturated"] = {"requests": 3000, "throughput_req_s": round(st.throughput, 1),
                             "p99_ms_queued_at_t0": round(st.p99_ms, 2), "batches": st.batches}
    out["hip_graphs"] = ctx.graphs()
    used, budget = ctx.ledger()
    out["ledger_gb"] = {"used": round(used / 1e9, 3), "budget": round(budget / 1e9, 1)}
    srv.close()
    ctx.close()
    ctx = ec.Context(0)
    reps64 = [(p.with_(prec=0), d) for p, d in reps]
    thr, svc, _ = serve.run_plain(ctx, reps64, serve.serving_requests(reps, plain_req, rate))
    ctx.close()
    out["fp64_plain"] = {"requests": plain_req, "throughput_req_s": round(thr, 1),
                         "service_p50_ms": round(float(np.median(svc)), 4),
                         "service_p99_ms": round(float(np.quantile(svc, 0.99)), 4)}
    out["saturated_fp32_over_plain_fp64"] = round(out["fp32_saturated"]["throughput_req_s"] / thr, 3)
    return out


def mixed_512_block(steps=3):
    """512^3, 20000 defects: FP32 and FP64 solve + energies, per-pass rates and
    the FP32 energy error against the FP64 path."""
    import torch

    from paper_2403_09158_amd import ec, inputs

    prob, defs = inputs.mixed_512(prec=1)
    ctx = ec.Context(0)
    out = {"workload": "mixed_512: 512^3 periodic cell, 160 nm, 20000 defects (mixed_256 mix, loops up to 8 nm)"}
    E = {}
    for prec, name in ((1, "fp32"), (0, "fp64")):
        st = ec.State(ctx, prob.with_(prec=prec))
        st.solve(defs)
        st.energies()
        torch.cuda.synchronize()
        st.profile(True)
        st.profile_read()
        t0 = time.perf_counter()
        for _ in range(steps):
            st.solve(defs)
            E[prec] = st.energies()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        out[name] = {"ms_per_resolve": round(dt * 1e3, 3), "per_family": family_table(st.profile_read())}
        st.close()
    out["fp32_vs_fp64"] = energy_errors(E[1], E[0])
    ctx.close()
    return out


def paper_129_block(steps=10, warmup=3):
    """The paper's odd grid (129^3 voxels in a cube of 500 a0, 300 defects):
    FP32 and FP64 solve + energies, and both against the stored oracle."""
    import numpy as np
    import torch

    from paper_2403_09158_amd import ec, inputs

    prob, defs = inputs.paper_129(prec=1)
    ctx = ec.Context(0)
    out = {"workload": "paper_129: 129^3 cell of 500 a0 (143.3 nm), cubic C 243/145/116 GPa, 300 defects"}
    g = np.load(os.path.join(ROOT, "tests", "golden", "oracle_paper_129.npz"))
    for prec, name in ((1, "fp32"), (0, "fp64")):
        st = ec.State(ctx, prob.with_(prec=prec))
        dt, E, _ = timed_steps(st, defs, steps, warmup, profile=False)
        out[name] = {"solves_per_s": round(steps / dt, 2), "ms_per_step": round(1e3 * dt / steps, 4),
                     "vs_oracle": energy_errors(E, g["E"])}
        st.close()
    ctx.close()
    return out


def stored_type_block(reps=10):
    """Stored defect types translated by the shift theorem on mixed_256 (FP32
    storage): storing a type, and the energies of one type at 16 and at 64
    sub-voxel positions with the resident stress (the mover excluded)."""
    import numpy as np
    import torch

    from paper_2403_09158_amd import ec, inputs

    prob, defs = inputs.mixed_256(prec=1)
    ctx = ec.Context(0)
    st = ec.State(ctx, prob)
    st.solve(defs)
    torch.cuda.synchronize()
    i = 5
    t0 = time.perf_counter()
    t = st.type_store(defs[i : i + 1])
    store_ms = (time.perf_counter() - t0) * 1e3
    rng = np.random.default_rng(0)
    out = {"workload": "mixed_256 FP32, type = defect 5 (a 1/2<111> loop), positions within 2 voxels",
           "store_ms": round(store_ms, 3)}
    for k in (16, 64):
        X = defs[i]["c"] + rng.uniform(-2, 2, (k, 3)) * prob.h
        st.type_energies(t, X, X_excl=defs[i]["c"])
        t0 = time.perf_counter()
        for _ in range(reps):
            st.type_energies(t, X, X_excl=defs[i]["c"])
        ms = (time.perf_counter() - t0) * 1e3 / reps
        out[f"positions_{k}"] = {"ms_per_call": round(ms, 3), "us_per_position": round(1e3 * ms / k, 2)}
    st.close()
    ctx.close()
    return out


def frame_block(steps=10, warmup=3):
    """mixed_256 with the crystal in the orientation of the paper's simulations
    (cell x, y, z along [111], [-1-12], [1-10]): solve + energies per step in
    FP32 and FP64, per-pass times, and the FP32 energy error against FP64."""
    from paper_2403_09158_amd import ec, inputs

    prob, defs = inputs.mixed_256(prec=1)
    prob = prob.with_(frame=inputs.FRAME_111)
    ctx = ec.Context(0)
    out = {
        "workload": "mixed_256 (256^3, 2000 defects) in a crystal rotated to cell axes [111], [-1-12], [1-10]: "
        "the Green step applied in the cube frame"
    }
    E = {}
    for prec, name in ((1, "fp32"), (0, "fp64")):
        st = ec.State(ctx, prob.with_(prec=prec))
        dt, E[prec], prof = timed_steps(st, defs, steps, warmup, True)
        out[name] = {"ms_per_step": round(dt / steps * 1e3, 4), "per_family": family_table(prof)}
        st.close()
    out["fp32_vs_fp64"] = energy_errors(E[1], E[0])
    ctx.close()
    return out


def dislocation_block(steps=10, warmup=3):
    """An edge dislocation in the paper's rotated frame (line along the cell z
    axis [1-10], Burgers vector 1/2[111] along x): the cost of setting the line
    and of solve + energies of mixed_256 with it present (FP32), and the
    interaction energy of a 1/2[111] loop (R = 1 nm) hopping along its glide
    direction x, 5 nm above the dislocation's glide plane (128^3, FP64)."""
    import numpy as np
    import torch

    from paper_2403_09158_amd import ec, inputs

    h = inputs.H_VOXEL
    bx = 0.5 * inputs.A_FE * np.sqrt(3.0) * np.array([1.0, 0.0, 0.0])
    ctx = ec.Context(0)
    prob, defs = inputs.mixed_256(prec=1)
    prob = prob.with_(frame=inputs.FRAME_111)
    line = inputs.line(np.array([128.0, 128.0, 0.0]) * h, 2, 1, bx)
    st = ec.State(ctx, prob)
    st.solve(defs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st.set_dislocations(line)
    torch.cuda.synchronize()
    t_set = time.perf_counter() - t0
    dt, _, prof = timed_steps(st, defs, steps, warmup, True)
    st.close()
    out = {
        "workload": "edge dislocation (line [1-10], b 1/2[111]) in the rotated frame: mixed_256 solve + energies with the "
        "line present (FP32), and a 1/2[111] loop (R 1 nm) hopping along x 5 nm above the glide plane (128^3, FP64)",
        "set_line_ms": round(t_set * 1e3, 3),
        "fp32_ms_per_step_with_line": round(dt / steps * 1e3, 4),
        "per_family": family_table(prof),
    }
    n = 128
    pp = inputs.Problem(n, n * h, *inputs.CUBIC_FE, prec=0, frame=inputs.FRAME_111)
    st = ec.State(ctx, pp)
    st.set_dislocations(inputs.line(np.array([64.0, 64.0, 0.0]) * h, 2, 1, bx))
    loop = inputs.loop(np.array([64.0 - 32.0 + 0.5, 64.0 + 16.0 + 0.5, 64.5]) * h, 1.0, bx, bx)
    st.solve(loop)
    xs, Es = [], []
    for k in range(17):
        if k:
            loop["c"][0] = loop["c"][0] + np.array([4.0 * h, 0.0, 0.0])
            E = st.update(0, loop[0])
        else:
            E = st.energies()
        xs.append(round(float(loop["c"][0][0] - 64.0 * h), 4))
        Es.append(float(E[0]))
    st.close()
    ctx.close()
    out["loop_profile"] = {"x_nm_from_line": xs, "E_eV": Es, "E_min_eV": min(Es), "E_max_eV": max(Es)}
    # dislocation loops and a line in a general direction by field dislocation
    # mechanics (ec_set_dislocation_paths): 16 hexagonal 1/2<111> loops of
    # radius 2 nm in their (111) planes and one mixed line along [1 1 0] through
    # the cell, on mixed_256 (FP32)
    prob, defs = inputs.mixed_256(prec=1)
    rng = np.random.default_rng(7)
    L = prob.L
    paths = []
    for k in range(16):
        s = np.array([1.0, 1.0, 1.0]) * rng.choice([-1.0, 1.0], 3)
        nrm = s / np.sqrt(3.0)
        e1 = np.cross(nrm, [1.0, 0.0, 0.0] if abs(nrm[0]) < 0.9 else [0.0, 1.0, 0.0])
        e1 /= np.linalg.norm(e1)
        e2 = np.cross(nrm, e1)
        ang = np.arange(6) * np.pi / 3.0
        c = rng.uniform(0.0, L, 3)
        paths.append((c + 2.0 * (np.cos(ang)[:, None] * e1 + np.sin(ang)[:, None] * e2), np.zeros(3),
                      0.5 * inputs.A_FE * s))
    paths.append((np.array([[1.3, 7.9, 40.6]]), np.array([L, L, 0.0]), np.array([0.12, 0.0, 0.21])))
    ctx = ec.Context(0)
    st = ec.State(ctx, prob)
    st.solve(defs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st.set_dislocation_paths(paths)
    torch.cuda.synchronize()
    t_paths = time.perf_counter() - t0
    dt, _, _ = timed_steps(st, defs, steps, warmup, False)
    st.close()
    ctx.close()
    out["paths"] = {"workload": "16 hexagonal 1/2<111> loops (R 2 nm) and a mixed line along [1 1 0], mixed_256 FP32",
                    "set_paths_ms": round(t_paths * 1e3, 3), "fp32_ms_per_step_with_paths": round(dt / steps * 1e3, 4)}
    return out


def jump_probe_block(steps=10):
    """Jump probes on mixed_256 (2000 defects, two glide jumps each): energy
    changes of all candidate jumps, biased frequencies and the frequency-line
    choice per defect; FP32 against FP64 and, for a few defects, against the
    energy change of actually making the move."""
    import numpy as np
    import torch

    from paper_2403_09158_amd import ec, inputs

    prob, defs = inputs.mixed_256(prec=1)
    J = inputs.glide_jumps(defs)
    rng = np.random.default_rng(inputs.SEED_BASE + 50)
    Em = np.full(len(defs), 0.1)  # eV
    kT, nu0 = 0.0258, 1.0e13  # eV (300 K), 1/s
    ctx = ec.Context(0)
    out = {
        "workload": "mixed_256 jump probes: 2000 defects, 2 glide jumps each (one voxel forward and back along b), "
        "biased frequencies (Em 0.1 eV, kT 0.0258 eV, nu0 1e13/s) and the frequency-line choice",
        "jumps_per_defect": int(J.shape[1]),
    }
    dE, E = {}, {}
    for prec, name in ((1, "fp32"), (0, "fp64")):
        st = ec.State(ctx, prob.with_(prec=prec))
        st.solve(defs)
        E[prec] = st.energies().copy()
        for _ in range(2):
            st.jump_energies(J)
            st.jump_select(Em, nu0, kT, 1.0 - rng.uniform(size=len(defs)))
        torch.cuda.synchronize()
        st.profile(True)
        st.profile_read()
        # a probe of a new configuration: the jump order alternates, so the
        # stored cross parts (kept while footprints only translate) are not reused
        Jr = np.ascontiguousarray(J[:, ::-1])
        t0 = time.perf_counter()
        for k in range(steps):
            st.jump_energies(Jr if k % 2 else J)
            nu, choice = st.jump_select(Em, nu0, kT, 1.0 - rng.uniform(size=len(defs)))
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        fam = family_table(st.profile_read())
        # the same jumps again (as after an OkMC step): cross parts reused
        dE[prec] = st.jump_energies(J)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            dE[prec] = st.jump_energies(J)
            nu, choice = st.jump_select(Em, nu0, kT, 1.0 - rng.uniform(size=len(defs)))
        torch.cuda.synchronize()
        dt_warm = (time.perf_counter() - t0) / steps
        # pair sums actually formed: one per jump up to sign (X(-l) = X(l)), none for l = 0
        m = np.array([len(f) for f in st.footprints()], dtype=np.float64)
        distinct = np.array([len({min(tuple(v), tuple(-v)) for v in J[i] if v.any()}) for i in range(len(defs))])
        pairs = float((m * m * distinct).sum())
        out[name] = {
            "ms_per_probe": round(dt * 1e3, 3),
            "ms_per_probe_cross_parts_reused": round(dt_warm * 1e3, 3),
            "pairs_per_probe": pairs,
            "per_family": fam,
        }
        if prec == 0:
            # a few defects: the energy change of making the move
            diffs = []
            for i in range(0, len(defs), 400):
                moved = defs[i].copy()
                moved["c"] = moved["c"] + J[i, 0].astype(np.float64) * prob.h
                E1 = st.update(i, moved)
                diffs.append(abs((E1[i] - E[0][i]) - dE[0][i, 0]))
                st.update(i, defs[i])
            out["fp64_vs_move_max_abs_eV"] = float(max(diffs))
        st.close()
    tol = 2.0 * np.maximum(1e-4 * np.abs(E[0]), 1e-5)[:, None]
    err = np.abs(dE[1] - dE[0])
    out["fp32_vs_fp64"] = {
        "max_abs_eV": float(err.max()),
        "pass_fraction": float(np.mean(err <= tol)),
        "max_err_over_tol": float((err / tol).max()),
    }
    ctx.close()
    return out


def okmc_block(steps=20, warmup=3):
    """OkMC time steps on mixed_256 (Sec. 5, App. B): Poisson gate over the
    fixed step, jump probes and choice for every defect, the chosen jumps made
    and the field solved again; the 1/2<111> loop migration barrier of the
    paper's loop runs (0.1 eV at 300 K) for every defect, two glide jumps each."""
    import numpy as np
    import torch

    from paper_2403_09158_amd import ec, inputs

    prob, defs = inputs.mixed_256(prec=1)
    J = inputs.glide_jumps(defs)
    nd = len(defs)
    Em = np.full(nd, 0.1)  # eV
    kT, nu0 = 8.617333262e-5 * 300.0, 1.0e13
    dt_s = 1.0 / (nu0 * np.exp(-0.1 / kT))
    ctx = ec.Context(0)
    out = {
        "workload": "mixed_256 OkMC steps: 2000 defects, 2 glide jumps each, Em 0.1 eV, 300 K, nu0 1e13/s, "
        "fixed step 1/nu_max; per step: Poisson gate, jump probes of all defects, frequency-line choice, "
        "chosen jumps made and the field solved again",
        "dt_ps": round(dt_s * 1e12, 4),
    }
    for prec, name in ((1, "fp32"), (0, "fp64")):
        rng = np.random.default_rng(inputs.SEED_BASE + 60)
        st = ec.State(ctx, prob.with_(prec=prec))
        st.solve(defs)
        for _ in range(warmup):
            st.okmc_step(J, Em, nu0, kT, 1.0 - rng.uniform(size=nd), 1.0 - rng.uniform(size=nd))
        torch.cuda.synchronize()
        moved = 0
        t0 = time.perf_counter()
        for _ in range(steps):
            ch = st.okmc_step(J, Em, nu0, kT, 1.0 - rng.uniform(size=nd), 1.0 - rng.uniform(size=nd))
            moved += int((ch >= 0).sum())
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / steps
        st.close()
        out[name] = {
            "ms_per_step": round(t * 1e3, 3),
            "steps_per_s": round(1.0 / t, 1),
            "moved_fraction": round(moved / (steps * nd), 4),
            "simulated_ns_per_wall_s": round(dt_s / t * 1e9, 3),
        }
        if prec == 1:
            # short steps (dt = 1e-3 / nu_max): about two defects act per step and
            # are moved one by one with the incremental update
            st = ec.State(ctx, prob.with_(prec=prec))
            st.solve(defs)
            dts = 1e-3 * dt_s
            for _ in range(warmup):
                st.okmc_step(J, Em, nu0, kT, 1.0 - rng.uniform(size=nd), 1.0 - rng.uniform(size=nd), dt=dts)
            torch.cuda.synchronize()
            acted = 0
            t0 = time.perf_counter()
            for _ in range(steps):
                ch = st.okmc_step(J, Em, nu0, kT, 1.0 - rng.uniform(size=nd), 1.0 - rng.uniform(size=nd), dt=dts)
                acted += int((ch >= 0).sum())
            torch.cuda.synchronize()
            tf = (time.perf_counter() - t0) / steps
            st.close()
            out["fp32_short_steps"] = {"dt_ps": round(dts * 1e12, 6), "ms_per_step": round(tf * 1e3, 3),
                                       "acting_per_step": round(acted / steps, 2)}
    ctx.close()
    return out


def _nearest_separation(prob, defs):
    """Per defect: the smallest min-image centre distance to another defect over
    the sum of the two radii (below 1 the bounding spheres overlap)."""
    import numpy as np

    c, R, L = defs["c"], defs["radius"], prob.L
    out = np.full(len(defs), np.inf)
    for i in range(len(defs)):
        dx = c - c[i]
        dx -= L * np.round(dx / L)
        s = np.sqrt((dx * dx).sum(1)) / (R + R[i])
        s[i] = np.inf
        out[i] = s.min()
    return out


def dipole_block(steps=10):
    """Dipole-tensor energies against the exact ones (FP64 states): on mixed_256,
    binned by each defect's nearest-neighbour separation, and for two coaxial
    1/2[111] loops moved apart along [111] (the loop-loop comparison of the
    paper's discussion), as the ratio exact / dipole."""
    import numpy as np
    import torch

    from paper_2403_09158_amd import ec, inputs

    prob, defs = inputs.mixed_256(prec=0)
    ctx = ec.Context(0)
    st = ec.State(ctx, prob)
    st.solve(defs)
    E = st.energies().copy()
    Ed = st.dipole_energies()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        Ed = st.dipole_energies()
    dt = (time.perf_counter() - t0) / steps
    st.close()
    sep = _nearest_separation(prob, defs)
    rel = np.abs(Ed - E) / np.maximum(np.abs(E), 1e-12)
    bins = {}
    for name, lo, hi in (("overlapping (<1)", 0.0, 1.0), ("1-2", 1.0, 2.0), (">=2", 2.0, np.inf)):
        m = (sep >= lo) & (sep < hi)
        if m.any():
            bins[name] = {"count": int(m.sum()), "rel_err_p50": float(np.median(rel[m])), "rel_err_p90": float(np.quantile(rel[m], 0.9))}

    # two coaxial loops, R = 4 voxels, in a 128^3 cell
    n = 128
    h = inputs.H_VOXEL
    pp = inputs.Problem(n, n * h, *inputs.CUBIC_FE, prec=0)
    b = 0.5 * inputs.A_FE * np.array([1.0, 1.0, 1.0])
    c0 = np.array([0.5, 0.5, 0.5]) * h
    R = 4.0
    sweep = []
    st = ec.State(ctx, pp)
    for k in (3, 5, 9, 14, 18, 27):
        d = np.concatenate([inputs.loop(c0, R * h, b, b), inputs.loop(c0 + k * h, R * h, b, b)])
        st.solve(d)
        Ex = st.energies().copy()
        Edp = st.dipole_energies()
        sweep.append({"d_over_R": round(k * 3**0.5 / R, 2), "E_exact_eV": float(Ex[1]), "E_dipole_eV": float(Edp[1]), "exact_over_dipole": float(Ex[1] / Edp[1])})
    st.close()
    ctx.close()
    return {
        "workload": "dipole-tensor energies -P:eps_others(x_c) against the exact energies (FP64 states): mixed_256 by nearest-neighbour separation |x_i - x_j| / (R_i + R_j), and two coaxial 1/2[111] loops (R = 4 voxels, 128^3) along [111]",
        "ms_per_call_mixed_256": round(dt * 1e3, 3),
        "mixed_256_by_separation": bins,
        "coaxial_loops": sweep,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--fp64-steps", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--skip-fp64", action="store_true", help="time the FP32 path only (profiling runs)")
    ap.add_argument("--no-serving", action="store_true", help="skip the many-replica serving workload")
    ap.add_argument("--no-512", action="store_true", help="skip the 512^3 / 20000-defect workload")
    ap.add_argument("--no-jumps", action="store_true", help="skip the jump-probe workload")
    ap.add_argument("--jumps-only", action="store_true", help="run the jump-probe, dipole and OkMC workloads alone")
    ap.add_argument("--okmc-only", action="store_true", help="run the OkMC-step workload alone (profiling runs)")
    ap.add_argument("--probe-only", action="store_true", help="run the jump-probe workload alone (profiling runs)")
    ap.add_argument("--dipole-only", action="store_true", help="run the dipole-tensor workload alone (profiling runs)")
    ap.add_argument("--no-frame", action="store_true", help="skip the rotated-crystal and dislocation workloads")
    ap.add_argument("--frame-only", action="store_true", help="run the rotated-crystal and dislocation workloads alone")
    ap.add_argument("--no-f4", action="store_true", help="skip the odd-grid and stored-type workloads")
    ap.add_argument("--f4-only", action="store_true", help="run the odd-grid and stored-type workloads alone")
    ap.add_argument(
        "--calibrate-copy",
        action="store_true",
        help="run one plain 1 GiB device copy and exit (reference for HBM byte counters)",
    )
    args = ap.parse_args()
    if args.gpus != 1:
        print(
            json.dumps({"error": "this solver runs on one GPU per process; multi-GPU runs are not supported"}),
            flush=True,
        )
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2403_09158_amd import ec, inputs

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)  # reads and writes exactly 2^30 bytes each
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": 1 << 30}), flush=True)
        return
    if args.f4_only:
        print(json.dumps({"paper_129": paper_129_block(), "stored_type": stored_type_block()}), flush=True)
        return
    if args.frame_only:
        print(json.dumps({"frame_111": frame_block(), "dislocation": dislocation_block()}), flush=True)
        return
    if args.dipole_only:
        print(json.dumps({"dipole": dipole_block()}), flush=True)
        return
    if args.probe_only:
        print(json.dumps({"jump_probe": jump_probe_block()}), flush=True)
        return
    if args.okmc_only:
        print(json.dumps({"okmc": okmc_block()}), flush=True)
        return
    if args.jumps_only:
        print(json.dumps({"jump_probe": jump_probe_block(), "dipole": dipole_block(), "okmc": okmc_block()}), flush=True)
        return
    prob32, defs = inputs.mixed_256(prec=1)
    prob64 = prob32.with_(prec=0)
    ctx = ec.Context(0)

    E64 = None
    if not args.skip_fp64:
        st64 = ec.State(ctx, prob64)
        k64 = args.fp64_steps if args.fp64_steps is not None else max(1, args.steps // 2)
        dt64, E64, _ = timed_steps(st64, defs, k64, max(1, args.warmup), profile=False)
        st64.close()

    st = ec.State(ctx, prob32)
    # Every family's launches timed over a few untimed steps give the
    # per-family table and the roofline kernel (the FFT-pass family with the
    # longest launches: the fused z pass); in the timed steps events bracket
    # that family's launches only, so that the others' events do not stretch
    # the step.
    prof_all, fam = None, None
    if not args.no_profile:
        _, _, prof_all = timed_steps(st, defs, 5, args.warmup, True)
        fam = max((k for k in prof_all
                   if k not in ("raster", "self_term", "energy_reduce", "other") and prof_all[k]["launches"]),
                  key=lambda k: prof_all[k]["ms"] / prof_all[k]["launches"])
    dt, E32, prof = timed_steps(st, defs, args.steps, args.warmup, profile=not args.no_profile,
                                families=None if fam is None else [fam])
    sps = args.steps / dt

    precision = {}
    if E64 is not None:
        err = np.abs(E32 - E64)
        tol = np.maximum(1e-4 * np.abs(E64), 1e-5)
        precision = {
            "fp32_vs_fp64_max_abs_eV": float(err.max()),
            "fp32_vs_fp64_p50_abs_eV": float(np.median(err)),
            "fp32_vs_fp64_p99_abs_eV": float(np.quantile(err, 0.99)),
            "fp32_pass_fraction": float(np.mean(err <= tol)),
            "fp32_max_err_over_tol": float(np.max(err / tol)),
        }
    golden = os.path.join(ROOT, "tests", "golden", "oracle_mixed_256.npz")
    if os.path.exists(golden):
        g = np.load(golden)
        if E64 is not None:
            precision["fp64_vs_oracle_max_rel"] = float(np.max(np.abs(E64 - g["E"])) / np.max(np.abs(g["E"])))
        e32 = np.abs(E32 - g["E"])
        precision["fp32_vs_oracle_pass_fraction"] = float(np.mean(e32 <= np.maximum(1e-4 * np.abs(g["E"]), 1e-5)))

    roofline = None
    if prof:
        n = prob32.n
        p = prof[fam]
        avg_ms = p["ms"] / max(p["launches"], 1)
        achieved = p["bytes_per_launch"] / (avg_ms * 1e-3) / 1e9
        sha = kernel_source_sha()
        roofline = {
            "bound": "hbm",
            "kernel": fam,
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic_for(fam, sha),
            "avg_launch_ms": round(avg_ms, 5),
            "bytes_per_launch": p["bytes_per_launch"],
            "source_sha": sha,
            "per_family": family_table(prof_all),
            # solve-level fraction against the minimal fused schedule: 240 n^3 bytes at FP32 storage
            "solve_frac_240N": round(240.0 * n**3 / (dt / args.steps) / 1e9 / HBM_PEAK_GBS, 4),
        }

    line = {
        "metric": "grid-solves/sec + energies at 256^3 (FP32 vs FP64), served p50/p99 latency",
        "value": round(sps, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * dt / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-storage/f64-arith",
        "data": "synthetic",
        "config": {
            "workload": "mixed_256: 256^3 periodic cell, 80 nm, cubic C 243/145/116 GPa, 2000 defects "
            "(70% 1/2<111> loops, 10% <100> loops, 20% dilatational spheres)",
            "n": prob32.n,
            "ndef": int(len(defs)),
            "parallelism": "single GPU",
            "stress": "stored by each solve at the voxels the defects cover (the energies read no other)",
        },
        "fp64": None if E64 is None else {"value": round(k64 / dt64, 3), "unit": "solves/s",
                                           "ms_per_step": round(1e3 * dt64 / k64, 4)},
        "precision": precision,
        "roofline": roofline,
    }
    st.close()
    ctx.close()
    if not args.no_serving:
        line["serving"] = serving_block()
    if not args.no_512:
        line["mixed_512"] = mixed_512_block()
    if not args.no_jumps:
        line["jump_probe"] = jump_probe_block()
        line["dipole"] = dipole_block()
        line["okmc"] = okmc_block()
    if not args.no_frame:
        line["frame_111"] = frame_block()
        line["dislocation"] = dislocation_block()
    if not args.no_f4:
        line["paper_129"] = paper_129_block()
        line["stored_type"] = stored_type_block()
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(prob64, defs)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
