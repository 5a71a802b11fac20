#!/usr/bin/env python3
"""Benchmark: DOF-timesteps/s of one full misfit + gradient evaluation
(forward + stored/checkpointed states + float64 misfit + adjoint fused with the
float64 gradient accumulation) on the layered KMV4 workload, on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

A "step" is one complete evaluation of J and dJ/dc for one shot over the whole
time window (every time step counted once):  value = N_dofs * N_t / seconds.
Prints one JSON line (plus progress lines on stderr).  The roofline object is
computed live from HIP events around sampled launches of the dominant kernel;
cpu_baseline times the FP64 oracle on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "DOF-timesteps/s fwd+adj+grad (FP32 vs FP64 oracle-matched); p50/p99 shot latency"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_hash():
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_2108_10946_amd", "csrc", "kernels.hip"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(variant, n_dofs, n_cells, dim, ts, shots=1):
    """Bytes the method must move per launch of `shots` shots on one mesh and model:
    per DOF and shot  forward step: read u^n, du^n; write u^{n+1}, du^{n+1}
                      adjoint step: the same for lambda, plus read u^m and a
                                    float64 read-modify-write of the gradient
                                    accumulator
    per DOF           c^2, gamma, beta (shared by the shots)
    per cell          compact topology (vertex + edge [+ face] ids, 4 B each) and
                      the symmetric geometry factor |det J| J^-1 J^-T (3 or 6 values)."""
    topo = 4 * (6 if dim == 2 else 14)
    geom = (3 if dim == 2 else 6) * ts
    per_cell = n_cells * (topo + geom)
    shared = n_dofs * 3 * ts
    if variant == "patch_forward":
        return shots * n_dofs * 4 * ts + shared + per_cell
    if variant == "patch_adjoint":
        return shots * n_dofs * (5 * ts + 16) + shared + per_cell
    raise ValueError(variant)


FP32_VECTOR_PEAK_TFLOPS = 157.3   # MI355X, packed FP32
FP32_NONPACKED_TFLOPS = 78.6      # 256 CUs x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz (no packed FP32 here)


def algorithmic_flops(variant, n_cells, dim, degree):
    """Flops per launch of the element work: the two reference-gradient
    contractions over the nonzero table entries (2 flops per multiply-add), the
    geometry product at each node, and in the adjoint the forward-state gradient
    and the pairing."""
    from paper_2108_10946_amd import kmv_element_tables
    nodes, w, g = kmv_element_tables(dim, degree)
    nnz = int(np.count_nonzero(np.abs(g) > 1e-14 * np.abs(g).max()))
    nd = len(w)
    per_cell = 2 * 2 * nnz + nd * 2 * (dim * dim + dim)
    if variant == "patch_adjoint":
        per_cell += 2 * nnz + nd * 2 * dim
    return per_cell * n_cells


def traffic_from_profiles(variant, hash_, precision="fp32", path=None):
    """HBM bytes per launch of a kernel variant in one precision ("fp32" or "fp64")
    from the committed counter summary, or None when there is no record for that
    variant and precision, or it was taken on another version of kernels.hip.  The
    record's kernel name must also be the instance of that precision
    (k_step<float, ...> or k_step<double, ...>)."""
    path = path or os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("kernels_hip_sha") != hash_:
        return None
    rec = (d.get(precision) or {}).get(variant)
    if not rec:
        return None
    ctype = {"fp32": "float", "fp64": "double"}.get(precision)
    if ctype is None or f"k_step<{ctype}," not in rec.get("kernel", "").replace(" ", ""):
        return None
    return rec.get("bytes_per_launch")


WORKLOADS = ("layered_kmv4", "layered_tet_kmv3")


def setup_workload(precision, budget_frac=0.75, window=0, workload="layered_kmv4", checkpoint_every=0,
                   mesh_cache={}, problem=True, gradient_every=1, absorbing=False, pml=False, patch_cells=0):
    import torch
    from paper_2108_10946_amd import Mesh, Problem
    from synth import configs
    w = getattr(configs, workload)()
    cache = mesh_cache.setdefault((workload, patch_cells), {})  # one mesh and step per workload
    if "mesh" not in cache:
        t = time.time()
        cache["mesh"] = Mesh(w.coords, w.cells, w.degree, patch_cells=patch_cells)
        log(f"mesh: {len(w.cells)} cells, {cache['mesh'].n_dofs} DOFs, "
            f"{cache['mesh'].n_patches} patches ({time.time() - t:.1f}s)")
    m = cache["mesh"]
    x = m.dof_coords()
    c_cur = torch.tensor(w.vp(*x.T), dtype=torch.float64, device="cuda")
    c_obs = torch.tensor(w.vp_obs(*x.T), dtype=torch.float64, device="cuda")
    eta = w.eta(*x.T)
    free, _ = torch.cuda.mem_get_info()
    budget = int(free * budget_frac)
    if "dt" not in cache:
        probe = Problem(m, 1e-4, 4, precision="fp64")
        rho = max(probe.spectral_radius(c_cur, iters=300), probe.spectral_radius(c_obs, iters=300))
        probe.close()
        nt = int(np.ceil(w.T / (w.cfl_fraction * 2.0 / np.sqrt(rho)) - 1e-12))
        cache["dt"] = (w.T / nt, nt)
        log(f"CFL: rho={rho:.6g}, dt={w.T / nt * 1e3:.4f} ms, N_t={nt}")
    dt, nt = cache["dt"]
    if window:
        nt = window
    if not problem:
        return w, m, None, c_cur, None, dt, nt
    prob = Problem(m, dt, nt, precision=precision, mem_budget=budget, checkpoint_every=checkpoint_every,
                   gradient_every=gradient_every)
    if pml:
        prob.set_pml(w.extra["sigma"](*x.T))
    else:
        prob.set_damping(eta)
    if absorbing:
        prob.set_absorbing_boundary(True)
    prob.set_sources(w.sources, f0=w.f0, t0=w.t0, amp=w.amp)
    prob.set_receivers(w.receivers)
    obs = prob.forward(c_obs)
    torch.cuda.synchronize()
    return w, m, prob, c_cur, obs, dt, nt


def time_gpu(precision, steps, warmup, every, window=0, workload="layered_kmv4", checkpoint_every=0,
             gradient_every=1, absorbing=False, pml=False, patch_cells=0):
    import torch
    from paper_2108_10946_amd import kmvwave as K
    w, m, prob, c, obs, dt, nt = setup_workload(precision, window=window, workload=workload,
                                                checkpoint_every=checkpoint_every, gradient_every=gradient_every,
                                                absorbing=absorbing, pml=pml, patch_cells=patch_cells)
    K.kmv_profile_enable(prob.handle, every)
    for i in range(warmup):
        t = time.time()
        J, g, _ = prob.misfit_gradient(c, obs)
        log(f"{precision} warmup {i}: J={J:.6g} ({time.time() - t:.2f}s)")
    K.kmv_profile_enable(prob.handle, every)  # reset counters, keep events
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        J, g, tr = prob.misfit_gradient(c, obs, keep_traces=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sec = (t1 - t0) / steps
    log(f"{precision}: {sec * 1e3:.1f} ms per misfit+gradient, J={J:.6g}, "
        f"|g|={float(torch.linalg.vector_norm(g)):.6g}")
    prof = {K.PROFILE_VARIANTS[v]: K.kmv_profile_read(prob.handle, v) for v in K.PROFILE_VARIANTS}
    info = prob.info()
    out = dict(sec=sec, J=J, n_dofs=m.n_dofs, n_cells=m.n_cells, nt=nt, dt=dt, prof=prof,
               checkpoint_every=info["checkpoint_every"], n_patches=m.n_patches,
               n_shared=m.n_shared_dofs, grad=g.cpu().numpy(), traces=tr.double().cpu().numpy())
    prob.close()
    del g, tr
    torch.cuda.empty_cache()
    return out


def roofline(res, ts, dim=2, shots=1):
    hash_ = kernel_hash()
    best = None
    for variant in ("patch_forward", "patch_adjoint"):
        p = res["prof"][variant]
        if p["timed"] == 0:
            continue
        total = p["launches"] * p["mean_ms"]
        b = algorithmic_bytes(variant, res["n_dofs"], res["n_cells"], dim, ts, shots)
        achieved = b / (p["mean_ms"] * 1e-3) / 1e9
        r = {"kernel": f"k_step ({variant.split('_')[1]})", "bound": "hbm", "achieved": round(achieved, 1),
             "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
             "traffic": (traffic_from_profiles(variant, hash_, "fp32" if ts == 4 else "fp64")
                         if shots == 1 else None),
             "algorithmic_bytes": int(b),
             "mean_launch_us": round(p["mean_ms"] * 1e3, 3), "launches": p["launches"],
             "timed_launches": p["timed"], "total_ms": total}
        if best is None or total > best["total_ms"]:
            best = r
        res.setdefault("rooflines", {})[variant] = r
    return best


def _oracle_sample(n_sample, quiet=False):
    """FP64 oracle (one thread) on the first n_sample forward and adjoint steps of the
    layered KMV4 workload; setup (DOF numbering, assembly) is not timed.  Returns
    (n_dofs, n_sample, seconds)."""
    from threadpoolctl import threadpool_limits
    from oracle.fem import Discretization
    from oracle import solver
    from synth import configs
    w = configs.layered_kmv4()
    with threadpool_limits(1):
        t = time.time()
        d = Discretization(w.coords, w.cells, w.degree)
        c = d.nodal_values(w.vp)
        K = d.stiffness(c)
        M = d.lumped_mass()
        P = d.interpolation_matrix(w.receivers)
        s = np.asarray(d.interpolation_matrix(w.sources).sum(0)).ravel()
        eta = d.nodal_values(w.eta)
        if not quiet:
            log(f"oracle setup {time.time() - t:.1f}s (not timed)")
        dt = 2.5e-4
        a = eta * dt / 2
        wav = solver.ricker(np.arange(n_sample) * dt, w.f0, w.t0, w.amp)
        t0 = time.perf_counter()
        tr, st = solver.forward(K, M, a, dt, n_sample, solver.point_source_load(s, wav), P=P,
                                keep_states=True)
        J, g, _ = solver.gradient(d, c, K, M, a, dt, P, 1.01 * tr, st)
        sec = time.perf_counter() - t0
    return d.n_dofs, n_sample, sec


def host_cpu():
    """The host the oracle ran on: logical CPUs the OS reports, the CPUs this process
    may run on, and the processor model."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        allowed = None
    return {"os_cpu_count": os.cpu_count(), "cpus_allowed": allowed, "cpu_model": model}


def _oracle_sample_quiet(n_sample):
    return _oracle_sample(n_sample, quiet=True)


def cpu_baseline(n_sample=120, processes=None):
    """The oracle on the host: one thread (value, cores = 1), and the aggregate of a
    process pool running the same sample concurrently, one thread each (at most 16
    processes, the host share of one GPU)."""
    N, n, sec = _oracle_sample(n_sample)
    value = N * n / sec
    log(f"oracle: {n} steps fwd+adj+grad in {sec:.1f}s -> {value:.3g} DOF-timesteps/s")
    out = {"value": round(value, 1), "unit": "DOF-timesteps/s", "cores": 1, "kind": "oracle",
           "sample": f"layered_kmv4 mesh (N={N}), first {n} steps of forward + "
                     f"adjoint + gradient, FP64 assembled CSR, one thread; {sec:.1f}s",
           "host": host_cpu()}
    procs = processes if processes is not None else min(16, os.cpu_count() or 1)
    if procs > 1:
        import multiprocessing as mp
        t = time.time()
        with mp.get_context("spawn").Pool(procs) as pool:  # fresh interpreters: no GPU state
            res = pool.map(_oracle_sample_quiet, [n_sample] * procs)
        agg = sum(Nw * nw / sw for Nw, nw, sw in res)
        log(f"oracle x {procs} processes: {agg:.3g} DOF-timesteps/s aggregate ({time.time() - t:.1f}s)")
        out["aggregate"] = {"value": round(agg, 1), "unit": "DOF-timesteps/s", "processes": procs,
                            "cores": procs, "sample": f"the same sample in {procs} concurrent processes, "
                                                      "one thread each; sum of their rates"}
    return out


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - np.asarray(b, np.float64)) / np.linalg.norm(b))


def serving_bench(n_requests=32, t_scale=1.0, slots=6, load=0.7, seed=11, mode="full", solo=3):
    """The serving mix: Poisson arrivals of shot requests over three seeded layered
    meshes (about 20k, 80k and 300k triangles), KMV degree uniform in {2,3,4,5},
    duration uniform in [1, 4] s x t_scale, 10% forward-only, the rest misfit +
    gradient against FP64 observed data of the model with anomalies (four shot
    positions per mesh, cached).  The offered load is `load` x the saturation
    throughput of the FP32 server (all requests submitted at once); the same
    arrival trace is then replayed through the FP32 server and through the plain
    per-shot FP64 path (one solve at a time, in arrival order).

    mode "burst": only the burst (for a kernel trace of the mix at full occupancy).
    mode "solo": only the first `solo` requests on the smallest discretisation (the
    23k-cell mesh, KMV2), one at a time on an idle server, each alone on the GPU (the
    case where per-launch cost shows most)."""
    import torch
    from paper_2108_10946_amd import Mesh, Problem, Server
    from synth import configs
    from synth.models import sponge_eta, surface_receivers
    rng = np.random.default_rng(seed)
    rec = surface_receivers(300, 0.1, 7.9, 0.1)
    positions = [np.array([[x, 0.01]]) for x in np.linspace(0.5, 7.5, 4)]
    cuda = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    disc = {}
    t = time.time()
    for i in range(3):
        coords, cells, vp, vpo = configs.serving_mesh(i)
        for k in (2, 3, 4, 5):
            m = Mesh(coords, cells, k)
            x = m.dof_coords()
            c, co = vp(x[:, 0], x[:, 1]), vpo(x[:, 0], x[:, 1])
            eta = sponge_eta(x[:, 0], x[:, 1], 0.0, 8.0, 3.0, 0.75, c_max=4.5)
            probe = Problem(m, 1e-4, 4, precision="fp64")
            rho = max(probe.spectral_radius(cuda(c), iters=100), probe.spectral_radius(cuda(co), iters=100))
            probe.close()
            disc[(i, k)] = dict(mesh=m, c=c, c_obs=co, eta=eta, dt=0.9 * 2.0 / np.sqrt(rho),
                                cells=len(cells))
    log(f"serving: 12 discretisations ready ({time.time() - t:.1f}s)")
    reqs = []
    for r in range(n_requests):
        key = (int(rng.integers(3)), int(rng.choice([2, 3, 4, 5])))
        T = rng.uniform(1.0, 4.0) * t_scale
        d = disc[key]
        reqs.append(dict(key=key, pos=int(rng.integers(4)), nt=max(1, int(round(T / d["dt"]))),
                         fwd=bool(rng.random() < 0.1)))
    if mode == "solo":
        reqs = [q for q in reqs if q["key"] == (0, 2)][:solo]
    # observed data, FP64, per (mesh, degree, position) at the longest window used
    t = time.time()
    obs = {}
    for (key, pos) in sorted({(q["key"], q["pos"]) for q in reqs}):
        d = disc[key]
        nt = max(q["nt"] for q in reqs if q["key"] == key and q["pos"] == pos)
        pr = Problem(d["mesh"], d["dt"], nt, precision="fp64")
        pr.set_damping(d["eta"])
        pr.set_sources(positions[pos], f0=5.0, t0=0.2)
        pr.set_receivers(rec)
        obs[(key, pos)] = pr.forward(cuda(d["c_obs"])).cpu().numpy()
        pr.close()
    torch.cuda.synchronize()
    log(f"serving: observed data for {len(obs)} shots ({time.time() - t:.1f}s)")

    def submit(srv, q, precision):
        d = disc[q["key"]]
        o = None if q["fwd"] else obs[(q["key"], q["pos"])][:q["nt"]]
        return srv.submit(d["mesh"], d["c"], positions[q["pos"]], rec, d["dt"], q["nt"], precision=precision,
                          eta=d["eta"], observed=o, forward_only=q["fwd"], f0=5.0, t0=0.2)

    dof_steps = sum(disc[q["key"]]["mesh"].n_dofs * q["nt"] for q in reqs)
    if mode == "solo":
        srv = Server(max_slots=slots)
        rows = []
        for q in reqs:
            t1 = time.perf_counter()
            r = srv.result(submit(srv, q, "fp32"))
            assert r["status"] == 0, r.get("error")
            rows.append({"n_dofs": disc[q["key"]]["mesh"].n_dofs, "n_steps": q["nt"], "forward_only": q["fwd"],
                         "seconds": round(time.perf_counter() - t1, 4)})
            log(f"serving solo: {rows[-1]}")
        srv.close()
        return {"mesh_cells": disc[(0, 2)]["cells"], "degree": 2, "requests": rows}

    def collect(srv, tickets, what):  # results in order, with a progress line every 10
        out = []
        for i, x in enumerate(tickets):
            out.append(srv.result(x))
            if (i + 1) % 10 == 0:
                log(f"serving {what}: {i + 1}/{len(tickets)} done")
        return out

    # saturation: every request at once
    srv = Server(max_slots=slots)
    t0 = time.perf_counter()
    tk = [submit(srv, q, "fp32") for q in reqs]
    res_sat = collect(srv, tk, "saturation")
    t_sat = time.perf_counter() - t0
    srv.close()
    assert all(r["status"] == 0 for r in res_sat), [r.get("error") for r in res_sat if r["status"]]
    sat = n_requests / t_sat
    lam = load * sat
    arrivals = np.cumsum(rng.exponential(1.0 / lam, n_requests))
    log(f"serving: saturation {sat:.2f} shots/s over {t_sat:.1f}s; offered load {lam:.2f}/s")
    if mode == "burst":
        return {"requests": n_requests, "duration_scale": t_scale, "slots": slots,
                "saturation_shots_per_s": round(sat, 3), "seconds": round(t_sat, 3),
                "dof_timesteps_total": int(dof_steps), "dof_timesteps_per_s": round(dof_steps / t_sat, 1)}

    # FP32 server, Poisson arrivals
    srv = Server(max_slots=slots)
    start = time.perf_counter()
    tk = []
    for q, ta in zip(reqs, arrivals):
        wait = start + ta - time.perf_counter()
        if wait > 0:
            time.sleep(wait)
        tk.append(submit(srv, q, "fp32"))
        if len(tk) % 20 == 0:
            log(f"serving fp32: {len(tk)}/{n_requests} submitted")
    res = collect(srv, tk, "fp32")
    srv.close()
    lat = np.array([r["t_done"] - r["t_submit"] for r in res])
    span = max(r["t_done"] for r in res) - min(r["t_submit"] for r in res)
    # the served results equal the saturation run's (same requests, other mix)
    same = all(np.array_equal(a["traces"], b["traces"]) and a["J"] == b["J"] for a, b in zip(res, res_sat))
    log(f"serving fp32: p50 {np.median(lat):.3f}s p99 {np.percentile(lat, 99):.3f}s, "
        f"{n_requests / span:.2f} shots/s; equal across mixes: {same}")

    # plain per-shot FP64, same arrival trace
    start = time.perf_counter()
    lat64 = []
    for q, ta in zip(reqs, arrivals):
        now = time.perf_counter() - start
        if now < ta:
            time.sleep(ta - now)
        d = disc[q["key"]]
        pr = Problem(d["mesh"], d["dt"], q["nt"], precision="fp64", mem_budget=64 << 30)
        pr.set_damping(d["eta"])
        pr.set_sources(positions[q["pos"]], f0=5.0, t0=0.2)
        pr.set_receivers(rec)
        if q["fwd"]:
            pr.forward(cuda(d["c"]))
        else:
            pr.misfit_gradient(cuda(d["c"]), cuda(obs[(q["key"], q["pos"])][:q["nt"]]))
        torch.cuda.synchronize()
        pr.close()
        lat64.append(time.perf_counter() - start - ta)
        if len(lat64) % 10 == 0:
            log(f"plain fp64: {len(lat64)}/{n_requests} done")
    lat64 = np.array(lat64)
    span64 = time.perf_counter() - start - arrivals[0]
    log(f"plain fp64: p50 {np.median(lat64):.3f}s p99 {np.percentile(lat64, 99):.3f}s, "
        f"{n_requests / span64:.2f} shots/s")
    return {
        "workload": f"{n_requests} Poisson shot requests over 3 layered meshes "
                    f"({', '.join(str(disc[(i, 2)]['cells']) for i in range(3))} cells), KMV k in {{2,3,4,5}}, "
                    f"T ~ U[{1.0 * t_scale:g}, {4.0 * t_scale:g}] s, 10% forward-only, FP64 observed data",
        "duration_scale": t_scale,
        "offered_load_shots_per_s": round(lam, 3),
        "saturation_shots_per_s": round(sat, 3),
        "dof_timesteps_total": int(dof_steps),
        "fp32_server": {"slots": slots, "p50_latency_s": round(float(np.median(lat)), 4),
                        "p99_latency_s": round(float(np.percentile(lat, 99)), 4),
                        "shots_per_s": round(n_requests / span, 3),
                        "results_equal_across_mixes": bool(same)},
        "fp64_plain": {"p50_latency_s": round(float(np.median(lat64)), 4),
                       "p99_latency_s": round(float(np.percentile(lat64, 99)), 4),
                       "shots_per_s": round(n_requests / span64, 3)},
    }


def trace_busy_summary(path):
    """GPU occupancy of a serving run from a rocprofv3 kernel trace (its
    kernel_trace.csv): over the window in which the server's streams run (from the
    first kernel on a stream other than the set-up stream to the last kernel end),
    the time covered by at least one kernel, the idle rest, and per stream the
    kernel time and the gaps between consecutive kernels of that stream."""
    import csv
    per = {}
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            if row.get("Kind", "KERNEL_DISPATCH") != "KERNEL_DISPATCH":
                continue
            sid = row["Stream_Id"]
            a, b = int(row["Start_Timestamp"]), int(row["End_Timestamp"])
            per.setdefault(sid, []).append((a, b, "k_step" in row["Kernel_Name"]))
    first = {sid: min(x[0] for x in v) for sid, v in per.items()}
    setup = min(first, key=first.get)
    others = [sid for sid in per if sid != setup]
    if not others:
        raise ValueError("no kernels outside the set-up stream")
    lo = min(first[sid] for sid in others)
    iv = sorted((a, b) for v in per.values() for a, b, _ in v if b > lo)
    hi = max(b for _, b in iv)
    busy, cur_a, cur_b = 0, None, None
    for a, b in iv:
        a = max(a, lo)
        if cur_b is None or a > cur_b:
            if cur_b is not None:
                busy += cur_b - cur_a
            cur_a, cur_b = a, b
        else:
            cur_b = max(cur_b, b)
    busy += cur_b - cur_a
    streams = {}
    for sid in others:
        v = sorted(per[sid])
        ker = sum(b - a for a, b, _ in v)
        gaps = [max(0, v[i + 1][0] - v[i][1]) for i in range(len(v) - 1)]
        steps = [b - a for a, b, st in v if st]
        streams[sid] = {"kernels": len(v), "kernel_ms": round(ker * 1e-6, 3), "gap_ms": round(sum(gaps) * 1e-6, 3),
                        "gap_frac": round(sum(gaps) / max(1, sum(gaps) + ker), 4),
                        "median_gap_us": round(float(np.median(gaps)) * 1e-3, 3) if gaps else None,
                        "median_step_us": round(float(np.median(steps)) * 1e-3, 3) if steps else None}
    span = hi - lo
    return {"window_ms": round(span * 1e-6, 3), "busy_ms": round(busy * 1e-6, 3),
            "idle_frac": round(1.0 - busy / span, 4), "streams": streams}


def c5_leg(steps, warmup, every, window=0, patch_cells=0):
    """The 3D workload: layered model with anomalies on 1.33 M graded tetrahedra,
    KMV3tet (16.9 M DOFs), T = 2 s, FP32 fields, float64 misfit and gradient,
    reverse sweep from checkpoints (segments of sqrt(2 N_t) steps).  The element
    work dominates here, so the roofline is the FP32 vector ALU.  Returns the timing
    result, its value and its rooflines."""
    res = time_gpu("fp32", steps, warmup, every, window, workload="layered_tet_kmv3", checkpoint_every=-1,
                   patch_cells=patch_cells)
    N, nt = res["n_dofs"], res["nt"]
    value = N * nt / res["sec"]
    roof = {}
    for variant in ("patch_forward", "patch_adjoint"):
        p = res["prof"][variant]
        if not p["timed"]:
            continue
        fl = algorithmic_flops(variant, res["n_cells"], 3, 3)
        ach = fl / (p["mean_ms"] * 1e-3) / 1e12
        roof[variant] = {"kernel": f"k_step ({variant.split('_')[1]})", "bound": "alu",
                         "achieved": round(ach, 2), "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(ach / FP32_VECTOR_PEAK_TFLOPS, 4),
                         "frac_of_nonpacked_peak": round(ach / FP32_NONPACKED_TFLOPS, 4),
                         "traffic": None, "algorithmic_flops": int(fl),
                         "mean_launch_us": round(p["mean_ms"] * 1e3, 3)}
    return res, value, roof


def bench_3d(args):
    """The 3D workload as a bench line of its own."""
    res, value, roof = c5_leg(args.steps, args.warmup, args.profile_every, args.window, args.patch_cells)
    N, nt = res["n_dofs"], res["nt"]
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "DOF-timesteps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(res["sec"] * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "layered_tet_kmv3: 3D 4x4x2 km, 8 layers 1.5-4.5 km/s + 3 seeded anomalies, "
                               "500 m sponge on five faces, graded Kuhn/Maubach tetrahedra, KMV3tet, 1 Ricker "
                               "shot (5 Hz), 40x40 receivers, T=2 s at 0.9x the power-iteration CFL step, "
                               "checkpointed reverse sweep",
                   "n_cells": res["n_cells"], "n_dofs": N, "n_steps": nt, "dt_s": res["dt"],
                   "checkpoint_every": res["checkpoint_every"], "n_patches": res["n_patches"]},
        "roofline": roof.get("patch_adjoint"),
        "rooflines": roof,
        "kernel_mean_us": {k: round(v["mean_ms"] * 1e3, 3) for k, v in res["prof"].items()},
        "note": "the 3D workload; the bench line is the default (layered_kmv4) run",
    }
    print(json.dumps(out), flush=True)


def five_gaussians(x, seed=17, n=5, radius=0.5, box=(0.0, 8.0, 0.0, 3.0)):
    """The seeded smooth perturbation direction of the 40-shot check: a sum of n
    Gaussians of the given radius (km) with seeded centres and signs in the physical
    box, scaled to a maximum of 1 km/s and zero outside the box (the sponge)."""
    rng = np.random.default_rng(seed)
    x0, x1, z0, z1 = box
    cx = x0 + (x1 - x0) * rng.random(n)
    cz = z0 + (z1 - z0) * rng.random(n)
    sg = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    d = sum(s * np.exp(-((x[:, 0] - a) ** 2 + (x[:, 1] - b) ** 2) / radius ** 2) for s, a, b in zip(sg, cx, cz))
    inside = (x[:, 0] >= x0) & (x[:, 0] <= x1) & (x[:, 1] >= z0) & (x[:, 1] <= z1)
    d = np.where(inside, d, 0.0)
    return d / np.abs(d).max()


def c3_bench(n_shots=40, batch=8, h=1e-3, every=16, subsample=10, checks=True):
    """The 40-shot FWI gradient of the layered KMV4 workload: shots at
    x_s = linspace(0.1, 7.9, 40), 10 m deep, T = 4 s; observed data from the model
    with anomalies (FP64), current model the layers.  J and dJ/dc are summed over
    the shots through the torch.autograd.Function (fwi_misfit) over 5 problems of 8
    shots (one launch per step for 8 shots, J and the gradient accumulated in the
    library), FP32 fields with FP64 accumulation, checkpointed reverse sweep.
    Checks: central differences of J at h along the seeded five-Gaussian direction
    (zero in the sponge) against the gradient; the adjoint's dot-product identity
    on one 8-shot problem; the FP32 J and gradient against the same 40 shots in
    FP64; and the 40 shots with the paper's gradient subsampling (r = 10).
    checks=False stops after the timed FP32 evaluation (for a kernel trace)."""
    import torch
    from paper_2108_10946_amd import Problem, kmvwave as K
    from paper_2108_10946_amd.autograd import fwi_misfit
    w, m, _, c_cur, _, dt, nt = setup_workload("fp32", workload="layered_kmv4", problem=False)
    x = m.dof_coords()
    eta = w.eta(*x.T)
    c_obs = torch.tensor(w.vp_obs(*x.T), dtype=torch.float64, device="cuda")
    line = np.linspace(0.1, 7.9, n_shots)
    groups = [np.stack([[[xx, 0.01]] for xx in line[k:k + batch]]) for k in range(0, n_shots, batch)]

    def make(prec, xs, budget, r=1, ck=-1):
        p = Problem(m, dt, nt, precision=prec, n_shots=len(xs), checkpoint_every=ck, mem_budget=budget,
                    gradient_every=r)
        p.set_damping(eta)
        p.set_sources(xs, f0=w.f0, t0=w.t0, amp=w.amp)
        p.set_receivers(w.receivers)
        return p

    free, _ = torch.cuda.mem_get_info()
    # FP64: observed data and the reference J and gradient, one 8-shot problem at a time
    t = time.time()
    obs64, J64, g64 = [], 0.0, torch.zeros(m.n_dofs, dtype=torch.float64, device="cuda")
    for xs in groups:
        p = make("fp64", xs, int(free * 0.4))
        obs64.append(p.forward(c_obs))
        if checks:
            J64 = p.misfit_gradient_accumulate(c_cur, obs64[-1], J64, g64)
        p.close()
    torch.cuda.synchronize()
    sec64 = time.time() - t
    log(f"c3: FP64 observed data and 40-shot J, gradient ({sec64:.1f}s)")
    # FP32 through the autograd Function, 5 problems of 8 shots
    free, _ = torch.cuda.mem_get_info()
    probs = [make("fp32", xs, int(free * 0.15)) for xs in groups]
    obs32 = [o.float().contiguous() for o in obs64]
    K.kmv_profile_enable(probs[0].handle, every)
    cg = c_cur.clone().requires_grad_(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J = fwi_misfit(cg, probs, obs32)
    J.backward()
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    J32, g32 = float(J), cg.grad.detach().clone()
    prof = {K.PROFILE_VARIANTS[v]: K.kmv_profile_read(probs[0].handle, v) for v in K.PROFILE_VARIANTS}
    info = probs[0].info()
    value = m.n_dofs * nt * n_shots / sec
    log(f"c3: 40 shots FP32 misfit + gradient in {sec:.2f}s -> {value:.4g} DOF-timesteps/s")
    if not checks:
        for p in probs:
            p.close()
        return {"shots": n_shots, "value": round(value, 1), "sec_per_misfit_gradient": round(sec, 3),
                "kernel_mean_us": {k: round(v["mean_ms"] * 1e3, 3) for k, v in prof.items()}}
    # central differences (J only) along the five-Gaussian direction
    ct = torch.as_tensor(five_gaussians(x), dtype=torch.float64, device="cuda")
    with torch.no_grad():
        Jp = float(fwi_misfit(c_cur + h * ct, probs, obs32))
        Jm = float(fwi_misfit(c_cur - h * ct, probs, obs32))
    fd = (Jp - Jm) / (2 * h)
    an = float(torch.dot(ct, g32))
    log(f"c3: central differences {fd:.9e} vs gradient {an:.9e} ({abs(fd - an) / abs(an):.2e})")
    # dot-product identity on one 8-shot problem
    p0 = probs[0]
    u = p0.forward(c_cur)
    y = torch.randn(u.shape, generator=torch.Generator(device="cuda").manual_seed(3), device="cuda",
                    dtype=torch.float32)
    _, st = p0.adjoint(c_cur, y, src_trace=True)
    wav = torch.as_tensor(np.asarray([w.amp * (1 - 2 * (np.pi * w.f0 * (n * dt - w.t0)) ** 2)
                                      * np.exp(-(np.pi * w.f0 * (n * dt - w.t0)) ** 2) for n in range(nt)]),
                          dtype=torch.float64, device="cuda")
    lhs = float((y.double() * u.double()).sum())
    rhs = dt * dt * float((wav[None, :, None] * st.double()).sum())
    for p in probs:
        p.close()
    del probs
    torch.cuda.empty_cache()
    # the paper's gradient subsampling over the 40 shots, r = 10 (every 10th state kept)
    sub = None
    if subsample > 1:
        free, _ = torch.cuda.mem_get_info()
        t = time.time()
        Js, gs = 0.0, torch.zeros_like(g32)
        for xs, o in zip(groups, obs32):
            p = make("fp32", xs, int(free * 0.6), r=subsample, ck=0)
            Js = p.misfit_gradient_accumulate(c_cur, o, Js, gs)
            p.close()
        torch.cuda.synchronize()
        secs = time.time() - t
        sub = {"gradient_every": subsample, "value": round(m.n_dofs * nt * n_shots / secs, 1),
               "sec_per_misfit_gradient": round(secs, 3),
               "gradient_rel_l2_vs_exact": float(torch.linalg.vector_norm(gs - g32) / torch.linalg.vector_norm(g32)),
               "note": "problems of 8 shots one after another, every 10th state kept (no recompute); "
                       "allocation included"}
        log(f"c3: gradient every {subsample} steps: {secs:.2f}s, gradient vs exact {sub['gradient_rel_l2_vs_exact']:.2e}")
    res = dict(n_dofs=m.n_dofs, n_cells=m.n_cells, prof=prof)
    roofline(res, 4, shots=batch)
    us = {k: round(v["mean_ms"] * 1e3, 3) for k, v in prof.items()}
    return {
        "workload": f"{n_shots} shots (x_s = linspace(0.1, 7.9, {n_shots}), 10 m deep) of the layered KMV4 "
                    "workload, T = 4 s; J and dJ/dc summed over the shots through the torch.autograd.Function "
                    f"over {len(groups)} problems of {batch} shots (one launch per step for {batch} shots), "
                    "FP32 fields with float64 misfit and gradient accumulation, checkpointed reverse sweep",
        "shots": n_shots, "value": round(value, 1), "unit": "DOF-timesteps/s", "sec_per_misfit_gradient": round(sec, 3),
        "n_steps": nt, "checkpoint_every": info["checkpoint_every"],
        "J": J32,
        "fp32_vs_fp64": {"J": abs(J32 - J64) / abs(J64),
                         "grad": float(torch.linalg.vector_norm(g32 - g64) / torch.linalg.vector_norm(g64))},
        "central_differences": {"h": h, "direction": "five seeded Gaussians (r = 0.5 km), max 1 km/s, zero in "
                                                     "the sponge", "fd": fd, "gradient": an,
                                "rel_err": abs(fd - an) / abs(an)},
        "dot_product": {"problem": f"one {batch}-shot problem, FP32, seeded normal adjoint data",
                        "lhs": lhs, "rhs": rhs, "rel_err": abs(lhs - rhs) / abs(lhs)},
        "fp64_reference_sec": round(sec64, 3),
        "kernel_mean_us": us,
        "per_shot_step_us": {"forward": round(us["patch_forward"] / batch, 3),
                             "adjoint": round(us["patch_adjoint"] / batch, 3)},
        "rooflines": {k: {kk: vv for kk, vv in v.items() if kk != "total_ms"}
                      for k, v in res.get("rooflines", {}).items()},
        "gradient_subsampling": sub,
    }


def gradient_check_bench(le3d=0.0):
    """The paper's gradient verification (2D: KMV2 on 20 m triangles, 2000 steps;
    with the sponge and with the PML) in FP64 and FP32: d^co = c~^T M G along the
    masked gradient against forward differences at h = 1e-3, 1e-4, 1e-5.  le3d > 0
    adds the 3D KMV2tet analogue with that box edge (sponge and PML)."""
    import torch
    from paper_2108_10946_amd import Mesh, Problem
    from paper_2108_10946_amd.fwi import directional_derivative_check
    from synth import configs
    cases = [("2d", "sponge", configs.gradient_check_2d()), ("2d", "pml", configs.gradient_check_2d())]
    if le3d > 0:
        cases += [("3d", "sponge", configs.gradient_check_3d(le=le3d)), ("3d", "pml", configs.gradient_check_3d(le=le3d))]
    out = {}
    for dim, layer, w in cases:
        t = time.time()
        m = Mesh(w.coords, w.cells, w.degree)
        x = m.dof_coords()
        nt = int(round(w.T / w.dt))
        c = torch.as_tensor(w.vp(*x.T), dtype=torch.float64, device="cuda")
        c_true = torch.as_tensor(w.vp_obs(*x.T), dtype=torch.float64, device="cuda")
        inside = w.eta(*x.T) == 0.0
        rows = {}
        obs = None
        for prec in ("fp64", "fp32"):
            p = Problem(m, w.dt, nt, precision=prec, mem_budget=64 << 30)
            if layer == "pml":
                p.set_pml(w.extra["sigma"](*x.T))
            else:
                p.set_damping(w.eta(*x.T))
            p.set_sources(w.sources, f0=w.f0, t0=w.t0)
            p.set_receivers(w.receivers)
            if obs is None:
                obs = p.forward(c_true)  # FP64 observed data
            r = directional_derivative_check(p, c, obs.to(p.dtype), mask=inside)
            p.close()
            rows[prec] = {"d_co": r["d_co"], "d_fd": {f"{h:g}": v for h, v in r["d_fd"].items()},
                          "rel_err": {f"{h:g}": v for h, v in r["rel_err"].items()}, "J": r["J"]}
        key = f"{dim}_{layer}"
        out[key] = dict(rows, n_cells=len(w.cells), n_dofs=m.n_dofs, n_steps=nt)
        log(f"gradient check {key}: d_co {rows['fp64']['d_co']:.6g}, rel err "
            + ", ".join(f"{h}: {v:.1e}" for h, v in rows["fp64"]["rel_err"].items()) + f" ({time.time() - t:.1f}s)")
        m.close()
    return out


def pml3d_leg(le=0.05):
    """The PML on tetrahedra against the sponge on the 3D gradient-verification box
    (KMV2 tetrahedra of edge le, T = 1 s at dt = 0.5 ms, layer on five faces), FP32:
    seconds per misfit + gradient with each layer (one warm-up, then one timed)."""
    import torch
    from paper_2108_10946_amd import Mesh, Problem
    from synth import configs
    w = configs.gradient_check_3d(le=le)
    m = Mesh(w.coords, w.cells, w.degree)
    x = m.dof_coords()
    nt = int(round(w.T / w.dt))
    c = torch.as_tensor(w.vp(*x.T), dtype=torch.float64, device="cuda")
    c_obs = torch.as_tensor(w.vp_obs(*x.T), dtype=torch.float64, device="cuda")
    out = {"workload": f"gradient_check_3d(le={le}): {len(w.cells)} KMV2 tetrahedra, {m.n_dofs} DOFs, "
                       f"{nt} steps, FP32", "n_dofs": m.n_dofs, "n_steps": nt}
    for layer in ("sponge", "pml"):
        p = Problem(m, w.dt, nt, precision="fp32", mem_budget=64 << 30)
        if layer == "pml":
            p.set_pml(w.extra["sigma"](*x.T))
        else:
            p.set_damping(w.eta(*x.T))
        p.set_sources(w.sources, f0=w.f0, t0=w.t0)
        p.set_receivers(w.receivers)
        obs = p.forward(c_obs)
        p.misfit_gradient(c, obs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p.misfit_gradient(c, obs)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        p.close()
        out[layer] = {"sec_per_misfit_gradient": round(sec, 4), "value": round(m.n_dofs * nt / sec, 1)}
        log(f"3D {layer}: {sec * 1e3:.1f} ms per misfit + gradient")
    out["overhead_vs_sponge"] = round(out["pml"]["sec_per_misfit_gradient"] / out["sponge"]["sec_per_misfit_gradient"] - 1.0, 4)
    m.close()
    return out


def copy_bandwidth(n_bytes=2 << 30, reps=10):
    """Achievable HBM bandwidth: a plain device-to-device copy of n_bytes (read +
    write = 2 n_bytes per copy, far above the 256 MB Infinity Cache), timed with
    events; the second roofline denominator beside the datasheet 8 TB/s."""
    import torch
    a = torch.ones(n_bytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2 * n_bytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbs


def copy_calibration(n_bytes=1 << 30, reps=3):
    """A plain device copy of known size, for scaling the FETCH_SIZE / WRITE_SIZE
    counters of a profiled run to bytes."""
    import torch
    a = torch.ones(n_bytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"bytes_read": n_bytes, "bytes_written": n_bytes,
                                           "dispatches": reps}}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--profile-every", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--window", type=int, default=0,
                    help="run only the first WINDOW time steps (hardware-counter runs: the "
                         "per-launch traffic does not depend on the window); not a bench line")
    ap.add_argument("--workload", choices=WORKLOADS, default="layered_kmv4",
                    help="layered_tet_kmv3: the 3D workload (FP32, checkpointed reverse sweep, "
                         "ALU roofline); not the bench line")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-c3", action="store_true", help="skip the 40-shot leg")
    ap.add_argument("--no-3d", action="store_true", help="skip the 3D (KMV3 tetrahedra) leg")
    ap.add_argument("--patch-cells", type=int, default=0,
                    help="cells per patch of the main legs' mesh (layered_kmv4, or layered_tet_kmv3 with "
                         "--workload; 0: the library's choice)")
    ap.add_argument("--c3-batch", type=int, default=8, help="shots per problem in the 40-shot leg")
    ap.add_argument("--no-pml", action="store_true", help="skip the leg with the PML in place of the sponge")
    ap.add_argument("--pml-only", action="store_true", help="run only the PML leg (for a kernel-trace profile)")
    ap.add_argument("--no-gradient-check", action="store_true")
    ap.add_argument("--gradient-check-only", action="store_true",
                    help="run only the gradient verification (with --gradient-check-3d for the 3D case)")
    ap.add_argument("--gradient-check-3d", type=float, default=0.0,
                    help="box edge (km) of the 3D gradient verification (0: skip; 0.02: the full size)")
    ap.add_argument("--subsample", type=int, default=10,
                    help="also time the paper's gradient subsampling with this ratio (1: skip)")
    ap.add_argument("--no-absorbing", action="store_true",
                    help="skip the leg with the absorbing boundary term on")
    ap.add_argument("--absorbing-only", action="store_true",
                    help="run only the absorbing-boundary leg (for a kernel-trace profile)")
    ap.add_argument("--c3-timing-only", action="store_true",
                    help="run only the FP64 observed data and the timed FP32 40-shot evaluation (kernel traces)")
    ap.add_argument("--c3-only", action="store_true",
                    help="run only the 40-shot leg and print its object (profiling runs)")
    ap.add_argument("--serving-only", action="store_true", help="run only the serving mix")
    ap.add_argument("--serving-requests", type=int, default=32)
    ap.add_argument("--serving-burst-only", action="store_true",
                    help="run only the serving mix's burst (all requests at once), for a kernel trace")
    ap.add_argument("--serving-solo", type=int, default=0,
                    help="run only this many of the mix's smallest requests, one at a time, for a kernel trace")
    ap.add_argument("--trace-summary", default="",
                    help="print the GPU busy / idle summary of a rocprofv3 kernel_trace.csv and exit (no GPU)")
    ap.add_argument("--serving-scale", type=float, default=1.0,
                    help="request durations are U[1,4] s times this (1.0: the configuration's own mix)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.trace_summary:
        print(json.dumps({"trace_summary": trace_busy_summary(args.trace_summary)}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); shots would shard "
              "across GPUs with one float64 all-reduce of the gradient, which is not implemented",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.workload == "layered_tet_kmv3":
        bench_3d(args)
        return
    if args.c3_only or args.c3_timing_only:
        print(json.dumps({"c3_40_shots": c3_bench(batch=args.c3_batch, subsample=args.subsample,
                                                  checks=not args.c3_timing_only)}), flush=True)
        return
    if args.gradient_check_only:
        print(json.dumps({"gradient_check": gradient_check_bench(args.gradient_check_3d)}), flush=True)
        return
    if args.serving_burst_only or args.serving_solo > 0:
        mode = "burst" if args.serving_burst_only else "solo"
        print(json.dumps({f"serving_{mode}": serving_bench(n_requests=args.serving_requests,
                                                           t_scale=args.serving_scale, mode=mode,
                                                           solo=args.serving_solo)}), flush=True)
        return
    if args.serving_only:
        print(json.dumps({"serving": serving_bench(n_requests=args.serving_requests,
                                                   t_scale=args.serving_scale)}), flush=True)
        return
    import paper_2108_10946_amd as kmv
    kmv.lib()

    def absorbing_leg(ref_sec=None):
        a = time_gpu("fp32", args.steps, min(1, args.warmup), 0, absorbing=True)
        out = {"value": round(a["n_dofs"] * a["nt"] / a["sec"], 1), "ms_per_step": round(a["sec"] * 1e3, 3),
               "storage": ("all states kept in HBM" if a["checkpoint_every"] == 0
                           else f"checkpoints every {a['checkpoint_every']} steps"),
               "note": "first-order absorbing boundary (du/dt + c du/dn = 0) on every boundary facet, "
                       "with its gradient term; observed data from the same boundary"}
        if ref_sec:
            out["overhead_vs_neumann"] = round(a["sec"] / ref_sec - 1.0, 4)
        return out

    if args.absorbing_only:
        print(json.dumps({"absorbing_boundary": absorbing_leg()}), flush=True)
        return

    def pml_leg(ref_sec=None):
        a = time_gpu("fp32", args.steps, min(1, args.warmup), args.profile_every, pml=True)
        out = {"value": round(a["n_dofs"] * a["nt"] / a["sec"], 1), "ms_per_step": round(a["sec"] * 1e3, 3),
               "kernel_mean_us": {k: round(v["mean_ms"] * 1e3, 3) for k, v in a["prof"].items()},
               "note": "the 750 m layer as the paper's PML (auxiliary p on the patches touching the layer, "
                       "their own kernel instance) in place of the sponge; observed data with the same "
                       "layer; kernel_mean_us times the launch over the patches away from the layer"}
        if ref_sec:
            out["overhead_vs_sponge"] = round(a["sec"] / ref_sec - 1.0, 4)
        out["tetrahedra"] = pml3d_leg()
        return out

    if args.pml_only:
        print(json.dumps({"pml": pml_leg()}), flush=True)
        return

    res32 = time_gpu("fp32", args.steps, args.warmup, args.profile_every, args.window, patch_cells=args.patch_cells)
    rl = roofline(res32, 4)
    sub1 = None
    if not args.window and args.subsample > 1:
        sub1 = time_gpu("fp32", args.steps, min(1, args.warmup), 0, gradient_every=args.subsample)
    absorb = None
    if not args.window and not args.no_absorbing:
        absorb = absorbing_leg(res32["sec"])
    pml = None
    if not args.window and not args.no_pml:
        pml = pml_leg(res32["sec"])
    res64 = None
    if not args.no_fp64:
        res64 = time_gpu("fp64", max(1, args.steps // 2), min(1, args.warmup), args.profile_every,
                         args.window, patch_cells=args.patch_cells)
        roofline(res64, 8)
    multi = None
    if not args.no_c3 and not args.window:
        multi = c3_bench(batch=args.c3_batch, subsample=args.subsample)
    gcheck = None
    if not args.no_gradient_check and not args.window:
        gcheck = gradient_check_bench()
    c5 = None
    if not args.no_3d and not args.window:
        r3, v3, roof3 = c5_leg(1, 1, args.profile_every)
        c5 = {"value": round(v3, 1), "unit": "DOF-timesteps/s", "sec_per_misfit_gradient": round(r3["sec"], 3),
              "workload": "layered_tet_kmv3: 3D 4x4x2 km, 8 layers + 3 seeded anomalies, 500 m sponge on five "
                          "faces, graded Kuhn/Maubach tetrahedra, KMV3tet, 1 Ricker shot (5 Hz), 40x40 receivers, "
                          "T=2 s, FP32 fields, float64 misfit and gradient, checkpointed reverse sweep",
              "n_cells": r3["n_cells"], "n_dofs": r3["n_dofs"], "n_steps": r3["nt"],
              "checkpoint_every": r3["checkpoint_every"], "roofline": roof3.get("patch_adjoint"),
              "rooflines": roof3}
        log(f"3D: {v3:.3e} DOF-timesteps/s ({r3['sec']:.2f}s)")
    serving = None
    if not args.no_serving and not args.window:
        serving = serving_bench(n_requests=args.serving_requests, t_scale=args.serving_scale)
    cpu = None if args.no_cpu_baseline else cpu_baseline()

    N, nt = res32["n_dofs"], res32["nt"]
    value = N * nt / res32["sec"]
    copy_gbs = copy_bandwidth()
    log(f"device copy: {copy_gbs:.0f} GB/s (read + write)")
    rls = list(res32.get("rooflines", {}).values()) + (list(multi["rooflines"].values()) if multi else [])
    for r in rls:
        r["measured_copy_GBs"] = round(copy_gbs, 1)
        r["frac_of_measured_copy"] = round(r["achieved"] / copy_gbs, 4)
    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "DOF-timesteps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(res32["sec"] * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "layered_kmv4: 2D 8x3 km, 8 layers 1.5-4.5 km/s + 3 seeded anomalies, "
                        "750 m sponge, graded NVB mesh, KMV4, 1 Ricker shot (5 Hz), 300 receivers, "
                        "T=4 s at 0.9x the power-iteration CFL step",
            "n_cells": res32["n_cells"], "n_dofs": N, "n_steps": nt, "dt_s": res32["dt"],
            "precision": "fp32 wavefields/operators, fp64 misfit and gradient accumulation",
            "state_storage": ("all states kept in HBM" if res32["checkpoint_every"] == 0
                              else f"checkpoints every {res32['checkpoint_every']} steps + recompute"),
            "n_patches": res32["n_patches"], "n_shared_dofs": res32["n_shared"],
            "patch_cells": args.patch_cells or "library default",
        },
        "roofline": {k: v for k, v in rl.items() if k != "total_ms"} if rl else None,
        "rooflines": {k: {kk: vv for kk, vv in v.items() if kk != "total_ms"}
                      for k, v in res32.get("rooflines", {}).items()},
        "kernel_mean_us": {k: round(v["mean_ms"] * 1e3, 3) for k, v in res32["prof"].items()},
        "cpu_baseline": cpu,
    }
    if multi:
        out["c3_40_shots"] = multi
    if pml:
        out["pml"] = pml
    if gcheck:
        out["gradient_check"] = gcheck
    if c5:
        out["c5_3d"] = c5
    if sub1:
        out["gradient_subsampling"] = {
            "gradient_every": args.subsample,
            "value": round(N * nt / sub1["sec"], 1), "ms_per_step": round(sub1["sec"] * 1e3, 3),
            "storage": ("every r-th state kept, no recompute" if sub1["checkpoint_every"] == 0
                        else f"checkpoints every {sub1['checkpoint_every']} steps"),
            "gradient_rel_l2_vs_exact": _rel(sub1["grad"], res32["grad"]),
            "note": "the paper's gradient subsampling (pairing and stored states every r-th step, "
                    "scaled by r); an approximation of the exact gradient that value is quoted on"}
    if absorb:
        out["absorbing_boundary"] = absorb
    if serving:
        out["p50_shot_latency_s"] = serving["fp32_server"]["p50_latency_s"]
        out["p99_shot_latency_s"] = serving["fp32_server"]["p99_latency_s"]
        out["serving"] = serving
    if res64:
        out["fp32_vs_fp64"] = {"J": abs(res32["J"] - res64["J"]) / abs(res64["J"]),
                               "traces": _rel(res32["traces"], res64["traces"]),
                               "grad": _rel(res32["grad"], res64["grad"])}
    if args.window:
        out["window"] = args.window
        out["note"] = "time window cut for a hardware-counter run: not a bench line"
    if res64:
        out["fp64"] = {"value": round(N * nt / res64["sec"], 1), "ms_per_step": round(res64["sec"] * 1e3, 3),
                       "state_storage": ("all states kept in HBM" if res64["checkpoint_every"] == 0
                                         else f"checkpoints every {res64['checkpoint_every']} steps"),
                       "rooflines": {k: {kk: vv for kk, vv in v.items() if kk != "total_ms"}
                                     for k, v in res64.get("rooflines", {}).items()}}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
