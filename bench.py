#!/usr/bin/env python3
"""Throughput of the entropic (KBC) lattice Boltzmann hot path on one MI355X.

A step is one pass of the whole path (geometry, pull streaming, moments, entropic equilibrium,
KBC collision with the per-node stabiliser, wall reconstruction and forces where the workload has
walls, store) over the workload's lattice.  The headline workload is ``turb512``: the 512^3
periodic box of seeded divergence-free turbulence (E(k) ~ k^4 exp(-2 (k/k0)^2), k0 = 8, rms 0.04,
Re_lambda ~ 100), FP32 populations -- the box the 70 % roofline target is stated on.  ``value`` is
whole-job MLUPS (lattice-node updates per second / 1e6) with the populations already resident in HBM.

Also reported on the same JSON line:
  roofline      -- the bulk sweep kernel's algorithmic HBM bytes per launch (216 per node) / its
                   average launch duration (HIP events recorded around each launch on the library's
                   stream), against the MI355X HBM peak of 8 TB/s; ``traffic`` comes from the
                   committed rocprofv3 counter summary when it was taken on the current kernel
                   source at this size.
  cpu_baseline  -- the FP64 CPU oracle, as it stands, on the headline recipe at 64^3 (the rerun the
                   reduced-storage error is stated on; per-node cost does not depend on the box
                   size): all host threads over the rerun's full 500 steps, one thread on a sample of
                   it, and the full 32^3 Taylor-Green workload.
  forms         -- the other forms: FP16 / BF16 storage on 512^3, FP32 on 256^3, the stabiliser
                   variants, the moving-sphere channel (384x192x192), the settling sphere, the
                   deforming swimmer, the adjoint rollout, and a plain copy kernel.
Progress goes to stderr; stdout carries the one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
BYTES_PER_NODE = {"f32": 216, "f16": 108, "bf16": 108}
SWEEP_SOURCES = ["paper_1608_04658_amd/csrc/sweep.hip", "paper_1608_04658_amd/csrc/elbm_internal.hpp"]
TRAFFIC_PROFILES = {"turb512": os.path.join(ROOT, "profiles", "sweep_turb512_traffic.md"),
                    "turb256": os.path.join(ROOT, "profiles", "sweep_f32_turb256_traffic.md")}


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def sweep_source_hash() -> str:
    h = hashlib.sha256()
    for rel in SWEEP_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(workload: str, nodes: int):
    """HBM bytes per sweep launch from the committed counter summary, or None when the summary is
    missing, for another size, or was taken on a different kernel source."""
    path = TRAFFIC_PROFILES.get(workload)
    if path is None or not os.path.exists(path):
        return None
    text = open(path).read()
    m_hash = re.search(r"source_sha256:\s*([0-9a-f]+)", text)
    m_bytes = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", text)
    m_nodes = re.search(r"nodes:\s*(\d+)", text)
    if not (m_hash and m_bytes and m_nodes):
        return None
    if m_hash.group(1) != sweep_source_hash() or int(m_nodes.group(1)) != nodes:
        return None
    return float(m_bytes.group(1))


def run_form(elbm, torch, shape, nu, storage, steps, warmup, init, bodies=None, channel=False, u_in=(0, 0, 0),
             flags=0):
    """Time ``steps`` steps of one form; returns (MLUPS, ms/step, sweep GB/s, fp64 nodes, lattice)."""
    lat = elbm.Lattice(shape, nu, storage=storage, channel=channel, u_inlet=u_in,
                       max_bodies=len(bodies) if bodies else 0, flags=flags)
    init(lat)
    if bodies:
        lat.set_bodies(bodies)
    lat.step(warmup)
    torch.cuda.synchronize()
    elbm.elbm_set_timing(lat.ctx, True)
    s = lat.stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s)
    lat.step(steps)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    sweep_ms, launches = elbm.elbm_get_timing(lat.ctx)
    elbm.elbm_set_timing(lat.ctx, False)
    n = lat.N
    mlups = n * steps / (ms / 1e3) / 1e6
    gbps = BYTES_PER_NODE[storage] * n / (sweep_ms / launches / 1e3) / 1e9
    info = lat.info()
    return mlups, ms / steps, gbps, sweep_ms / launches, info, lat


def copy_probe(torch, nbytes=8 << 30, reps=20):
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2 * nbytes / (ms / 1e3) / 1e9


def adjoint_form(torch, WL):
    """The differentiable workload: 300-step rollout of the 128x64x64 oscillating-sphere channel with
    a body-force field, loss = mean drag over steps 100..300; forward with checkpoints every 20
    steps, then the reverse sweep (recompute of each segment + hand-written adjoint steps).
    Bytes per node and reverse step: recompute 228 + adjoint 360 = 588."""
    import numpy as np
    from paper_1608_04658_amd.adjoint import ForceRollout, window_weights
    w = WL.WORKLOADS["adj128"]
    steps = 300
    rho, u = WL.uniform_flow(w["shape"], w["u_in"])
    F = torch.tensor(WL.body_force(w["shape"], w["force_seed"], w["force_amp"]), dtype=torch.float32, device="cuda")
    ro = ForceRollout(w["shape"], w["nu"], w["bodies"][0], steps, window_weights(steps, *w["loss_window"]),
                      checkpoint=w["checkpoint"], channel=True, u_in=w["u_in"], rho=rho, u=u)
    ro.forward(F, w["bodies"][0]["amp"])  # warm-up
    ro.backward()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    torch.cuda.synchronize()
    e[0].record()
    L = ro.forward(F, w["bodies"][0]["amp"])
    e[1].record()
    gF, gA = ro.backward()
    e[2].record()
    torch.cuda.synchronize()
    fwd, bwd = e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2])
    n = int(np.prod(w["shape"]))
    return {"MLUPS": round(n * steps / (bwd / 1e3) / 1e6, 1), "ms_per_step": round(bwd / steps, 4),
            "GBps_588B": round(588 * n * steps / (bwd / 1e3) / 1e9, 1), "forward_ms_per_step": round(fwd / steps, 4),
            "loss": L, "dL_damp": gA, "dL_dF_norm": float(gF.double().norm().item())}


def settle_form(elbm, torch, WL, steps: int = 500):
    """Two-way coupling: a sphere (R = 10, density ratio 2) settling under gravity in a fluid at rest,
    384 x 96 x 96 channel with the inlet wall at rest, FP32.  Every step reads the previous step's
    force back to the host for the Euler update of the sphere."""
    shape = (384, 96, 96)
    rho, u = WL.uniform_flow(shape, (0.0, 0.0, 0.0))
    lat = elbm.Lattice(shape, 0.004, channel=True, u_inlet=(0.0, 0.0, 0.0), max_bodies=1)
    lat.init_equilibrium(rho, u)
    lat.set_bodies([WL.free_sphere((40.0, 47.5, 47.5), 10.0, 2.0, gravity=(2e-5, 0.0, 0.0))])
    lat.step(100)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(lat.stream)
    lat.step(steps)
    e1.record(lat.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    x, v = lat.body_state(0)
    n = shape[0] * shape[1] * shape[2]
    return {"MLUPS": round(n * steps / (ms / 1e3) / 1e6, 1), "ms_per_step": round(ms / steps, 4),
            "position_x": round(float(x[0]), 4), "velocity_x": float(v[0])}


def swimmer_form(elbm, torch, steps: int = 20, warmup: int = 3, L: int = 200):
    """Deforming triangulated body (Sec. IV.C): the anguilliform swimmer of length L = 200 in the
    paper's 8L x 4L x L domain (1600 x 800 x 200, 256 M nodes, FP32), undulation period T = 10^4,
    Re = (L^2/T)/nu = 7142, held in place in a channel stream at its swimming speed 0.415 L/T, at full
    amplitude.  The surface (150 segments x 16 points) of every step is generated beforehand and
    held on the device; each step uploads nothing from the host."""
    import numpy as np
    from workloads import meshes as M
    T = 1.0e4
    nu = (L * L / T) / 7142.0
    shape = (8 * L, 4 * L, L)
    u_in = (0.415 * L / T, 0.0, 0.0)
    head = (2.0 * L, 2.0 * L + 0.35, 0.5 * L + 0.4)
    t0 = T
    levels = [M.swimmer_mesh(head, L, T, t0 + k) for k in range(warmup + steps + 1)]
    tris = levels[0][1]
    Xs = torch.as_tensor(np.stack([lv[0] for lv in levels])).cuda()
    Vs = torch.as_tensor(np.stack([lv[2] for lv in levels])).cuda()
    lo = (head[0] - 2.0, head[1] - 0.2 * L, head[2] - 0.1 * L)
    hi = (head[0] + L + 2.0, head[1] + 0.2 * L, head[2] + 0.1 * L)
    ctr = (head[0] + 0.5 * L, head[1], head[2])
    lat = elbm.Lattice(shape, nu, channel=True, u_inlet=u_in, max_bodies=1, max_mesh_vertices=Xs.shape[1],
                       max_mesh_triangles=len(tris))
    nx, ny, nz = shape
    u = torch.zeros((3, nz, ny, nx), dtype=torch.float64, device="cuda")
    u[0] = u_in[0]
    elbm.elbm_init_equilibrium(lat.ctx, None, u)
    del u
    lat.set_mesh(levels[0][0], tris, lo, hi, vels=levels[0][2], center=ctr)
    lat.set_bodies([dict(kind="mesh")])
    for k in range(warmup):
        lat.mesh_next(Xs[k + 1], Vs[k + 1], center=ctr)
        lat.step(1)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(lat.stream)
    for k in range(warmup, warmup + steps):
        lat.mesh_next(Xs[k + 1], Vs[k + 1], center=ctr)
        lat.step(1)
    e1.record(lat.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    info = lat.info()
    F = lat.force_history(0, info.t - steps + 1, steps)
    n = nx * ny * nz
    out = {"MLUPS": round(n * steps / (ms / 1e3) / 1e6, 1), "ms_per_step": round(ms / steps, 4),
           "nodes": n, "triangles": int(len(tris)), "boundary_nodes_last_step": int(info.boundary_nodes),
           "fp64_nodes_last_step": int(info.fp64_nodes), "thrust_x_mean": float(F[:, 0].mean())}
    del lat
    torch.cuda.empty_cache()
    return out


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_run(workload: str, n: int, steps: int, budget_s: float | None):
    """Step the FP64 oracle on `workload`'s recipe at n^3 (the workload's own size if n = 0) from its
    initial field: `steps` steps, or fewer if budget_s seconds of stepping are reached first (at
    least 2).  Returns (nodes, steps done, seconds, threads)."""
    import oracle
    import workloads as WL
    w = WL.WORKLOADS[workload]
    shape = w["shape"] if n == 0 else (n, n, n)
    rho, u = WL.initial_field(workload, shape)
    sim = oracle.Simulation(shape, w["nu"], rho, u)
    done = 0
    t0 = time.perf_counter()
    while done < steps:
        sim.step(1)
        done += 1
        el = time.perf_counter() - t0
        if done % 50 == 0 or done <= 2:
            log(f"cpu_baseline: {workload} at {shape[0]}^3, oracle step {done} at {el:.1f}s "
                f"({oracle.max_threads()} threads)")
        if budget_s is not None and done >= 2 and el >= budget_s:
            break
    return sim.N, done, time.perf_counter() - t0, oracle.max_threads()


def cpu_baseline(workload: str, budget_s: float = 10.0):
    """The FP64 oracle, unmodified, on the host cores.  The headline recipe is run as the 64^3 rerun
    (the turbulence recipe of the headline box at 64^3, its 500 steps in full): the oracle's cost per
    node does not depend on the box size, and the 512^3 box would need about 90 GB of host memory
    and 16 s per step.  Also: one host thread on a bounded sample of the same rerun (a child process
    with OMP_NUM_THREADS=1), and the 32^3 Taylor-Green workload in full."""
    import subprocess
    import workloads as WL
    w = WL.WORKLOADS[workload]
    n_rerun = 64 if w["shape"][0] > 64 else 0
    nodes, steps, el, threads = oracle_run(workload, n_rerun, w["steps"], None)
    value = nodes * steps / el / 1e6
    env = dict(os.environ, OMP_NUM_THREADS="1")
    one = subprocess.run([sys.executable, os.path.abspath(__file__), "--oracle-sample", workload, str(n_rerun),
                          str(w["steps"]), str(budget_s)], env=env, capture_output=True, text=True, timeout=600)
    if one.returncode != 0:
        raise RuntimeError(f"one-thread oracle run failed: {one.stderr[-500:]}")
    n1, s1, e1, t1 = json.loads(one.stdout.strip().splitlines()[-1])
    tg_nodes, tg_steps, tg_s, _ = oracle_run("tg32", 0, WL.WORKLOADS["tg32"]["steps"], None)
    side = w["shape"][0] if n_rerun == 0 else n_rerun
    return {"value": round(value, 3), "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"{workload} recipe at {side}^3 (FP64 C oracle): all {steps} steps in {el:.1f} s "
                      f"on {threads} threads; MLUPS per node does not depend on the box size",
            "cpu_model": cpu_model(), "host_threads_available": len(os.sched_getaffinity(0)),
            "one_thread": {"value": round(n1 * s1 / e1 / 1e6, 4), "unit": "MLUPS",
                           "sample": f"{s1} steps of the same {side}^3 rerun, {e1:.1f} s, {t1} thread"},
            "tg32_full": {"steps": tg_steps, "seconds": round(tg_s, 2), "MLUPS": round(tg_nodes * tg_steps / tg_s / 1e6, 3)},
            "rerun_full": {"steps": steps, "seconds": round(el, 2)}}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default: the workload's step count)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="turb512")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--form-steps", type=int, default=100)
    ap.add_argument("--forms", default="copy,turb512_2byte,turb256,stabilisers,sphere384,settle,swimmer,adj128",
                    help="comma-separated subset of the extra forms to run")
    ap.add_argument("--probe-copy-mib", type=int, default=0,
                    help="after the headline run, copy a buffer of this many MiB 5 times (a plain copy kernel "
                         "of known size, used to scale the HBM byte counters of a rocprofv3 --pmc run)")
    ap.add_argument("--oracle-sample", nargs=4, metavar=("WORKLOAD", "N", "STEPS", "BUDGET_S"),
                    help="internal: time the FP64 oracle only (no GPU) and print [nodes, steps, s, threads]")
    args = ap.parse_args()

    if args.oracle_sample:
        wl, n, st, bud = args.oracle_sample
        print(json.dumps(list(oracle_run(wl, int(n), int(st), float(bud)))), flush=True)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on exactly one GPU: the library has no multi-GPU path (asked for --gpus "
              f"{args.gpus}, WORLD_SIZE={world}).", file=sys.stderr)
        sys.exit(2)

    import numpy as np  # noqa: F401
    import torch
    import workloads as WL
    from paper_1608_04658_amd import elbm

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(3)
    torch.cuda.set_device(0)
    elbm.load()

    def make_init(workload):
        """Initial equilibrium of a workload's field: the 512^3 turbulence drawn on the device (the
        host FFT at that size is slow), the others from the host recipe."""
        wl = WL.WORKLOADS[workload]
        if workload == "turb512":
            log("turb512: generating the initial field on the device")
            r_, u_ = WL.turbulence_device(512, wl["k0"], wl["urms"], wl["seed"])

            def init_dev(lat):
                elbm.elbm_init_equilibrium(lat.ctx, r_, u_)
                torch.cuda.synchronize()
            return init_dev, (r_, u_)
        log(f"{workload}: generating the initial field")
        r_, u_ = WL.initial_field(workload)

        def init_host(lat):
            lat.init_equilibrium(r_, u_)
        return init_host, (r_, u_)

    w = WL.WORKLOADS[args.workload]
    steps = args.steps if args.steps is not None else w["steps"]
    shape = w["shape"]
    init, keep = make_init(args.workload)
    log(f"workload {args.workload} {shape}: timing {steps} steps after {args.warmup} warm-up steps")
    mlups, ms_step, gbps, sweep_ms, info, lat = run_form(elbm, torch, shape, w["nu"], "f32", steps, args.warmup,
                                                         init, bodies=w.get("bodies"), channel=w.get("channel", False),
                                                         u_in=w.get("u_in", (0, 0, 0)))
    # the stored FP32 deviations, checked in place (an FP64 copy of 512^3 would take 29 GB)
    finite = bool(torch.isfinite(lat.population_view()).all().item())
    healthy = info.nonfinite == 0
    del lat
    torch.cuda.empty_cache()
    log(f"{args.workload}: {mlups:.0f} MLUPS, sweep {gbps:.0f} GB/s, {ms_step:.3f} ms/step, finite={finite}, "
        f"no failed state={healthy}, fp64 nodes last step={info.fp64_nodes}")
    n_nodes = shape[0] * shape[1] * shape[2]
    roof = {"bound": "hbm", "achieved": round(gbps, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(gbps / HBM_PEAK_GBPS, 4), "traffic": traffic_from_profile(args.workload, n_nodes),
            "kernel": "k_sweep<f32> (bulk stream-collide)", "bytes_per_launch": BYTES_PER_NODE["f32"] * n_nodes,
            "avg_launch_ms": round(sweep_ms, 4), "sweep_source_sha16": sweep_source_hash()}

    if args.probe_copy_mib:
        nb = args.probe_copy_mib << 20
        a = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"copy probe: 5 copies of {args.probe_copy_mib} MiB (read {nb} B + write {nb} B each)")
        del a, b

    forms = {}
    which = set(args.forms.split(",")) if not args.no_forms else set()
    try:
        if "copy" in which:
            forms["copy_probe_GBps"] = round(copy_probe(torch), 1)
            log(f"copy probe {forms['copy_probe_GBps']} GB/s")
            # the library's stream-only mode: the sweep's pull and store, no collision -- the
            # attainable bandwidth of exactly this access pattern
            _, _, gb, _, _, lat = run_form(elbm, torch, shape, w["nu"], "f32", args.form_steps, 5, init,
                                           flags=elbm.FLAG_STREAM_ONLY)
            del lat
            torch.cuda.empty_cache()
            forms["pull_copy_GBps"] = round(gb, 1)
            roof["attainable_pull_copy"] = round(gb, 1)
            log(f"stream-only pull copy ({args.workload}) {gb:.0f} GB/s")
        if "turb512_2byte" in which:
            w5 = WL.WORKLOADS["turb512"]
            init5, keep5 = (init, keep) if args.workload == "turb512" else make_init("turb512")
            stores = ("f16", "bf16") if args.workload == "turb512" else ("f32", "f16", "bf16")
            for st in stores:
                m, msps, gb, _, inf, lat = run_form(elbm, torch, w5["shape"], w5["nu"], st, args.form_steps, 5, init5)
                del lat
                torch.cuda.empty_cache()
                forms[f"turb512_{st}"] = {"MLUPS": round(m, 1), "ms_per_step": round(msps, 4),
                                          "sweep_GBps": round(gb, 1), "frac": round(gb / HBM_PEAK_GBPS, 4),
                                          "vs_f32_MLUPS": round(m / mlups, 3) if args.workload == "turb512" else None,
                                          "fp64_nodes_last_step": int(inf.fp64_nodes)}
                log(f"turb512 {st}: {m:.0f} MLUPS, sweep {gb:.0f} GB/s")
            del init5, keep5
            torch.cuda.empty_cache()
        if "turb256" in which and args.workload != "turb256":
            w1 = WL.WORKLOADS["turb256"]
            init1, keep1 = make_init("turb256")
            m, msps, gb, sms, inf, lat = run_form(elbm, torch, w1["shape"], w1["nu"], "f32", 2 * args.form_steps, 5,
                                                  init1)
            del lat, init1, keep1
            torch.cuda.empty_cache()
            forms["turb256_f32"] = {"MLUPS": round(m, 1), "ms_per_step": round(msps, 4), "sweep_GBps": round(gb, 1),
                                    "frac": round(gb / HBM_PEAK_GBPS, 4), "avg_launch_ms": round(sms, 4),
                                    "traffic": traffic_from_profile("turb256", 256 ** 3)}
            log(f"turb256 f32: {m:.0f} MLUPS, sweep {gb:.0f} GB/s")
        if "stabilisers" in which:
            # the headline run with the exact stabiliser, LBGK and the central-moment shear part
            for name, fl in (("exact_gamma", elbm.FLAG_EXACT_GAMMA), ("lbgk", elbm.FLAG_LBGK),
                             ("central", elbm.FLAG_CENTRAL)):
                m, msps, gb, _, _, lat = run_form(elbm, torch, shape, w["nu"], "f32", max(10, args.form_steps // 5), 3,
                                                  init, flags=fl)
                del lat
                torch.cuda.empty_cache()
                forms[f"{args.workload}_{name}"] = {"MLUPS": round(m, 1), "ms_per_step": round(msps, 4),
                                                    "sweep_GBps": round(gb, 1)}
                log(f"{args.workload} {name}: {m:.0f} MLUPS, sweep {gb:.0f} GB/s")
        if "sphere384" in which:
            w2 = WL.WORKLOADS["sphere384"]
            r2, u2 = WL.initial_field("sphere384")

            def init2(lat):
                lat.init_equilibrium(r2, u2)

            m, msps, gb, _, inf, lat = run_form(elbm, torch, w2["shape"], w2["nu"], "f32", 2 * args.form_steps, 5,
                                                init2, bodies=w2["bodies"], channel=True, u_in=w2["u_in"])
            F, _ = lat.force(0, lat.info().t)
            del lat
            torch.cuda.empty_cache()
            forms["sphere384_f32"] = {"MLUPS": round(m, 1), "ms_per_step": round(msps, 4), "sweep_GBps": round(gb, 1),
                                      "boundary_nodes": int(inf.boundary_nodes), "fp64_nodes_last_step": int(inf.fp64_nodes),
                                      "drag_last_step": F[0]}
            log(f"sphere384: {m:.0f} MLUPS, boundary nodes {inf.boundary_nodes}, drag {F[0]:.4e}")
        if "settle" in which:
            forms["settle_f32"] = settle_form(elbm, torch, WL)
            log(f"settling sphere: {forms['settle_f32']}")
        if "swimmer" in which:
            forms["swimmer_f32"] = swimmer_form(elbm, torch)
            log(f"deforming swimmer: {forms['swimmer_f32']}")
        if "adj128" in which:
            forms["adj128_adjoint"] = adjoint_form(torch, WL)
            log(f"adj128 adjoint: {forms['adj128_adjoint']}")
    except Exception as exc:  # a failing extra form must not hide the headline number
        forms["error"] = repr(exc)
        log(f"forms failed: {exc!r}")
    del init, keep
    torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.workload)
        log(f"cpu_baseline {cpu['value']:.2f} MLUPS on {cpu['cores']} threads, "
            f"{cpu['one_thread']['value']:.3f} MLUPS on one ({cpu['cpu_model']})")

    line = {
        "metric": "MLUPS and % of HBM roofline, FP32 vs reduced-storage vs adjoint, 1 MI355X",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "lattice": "D3Q27", "shape": list(shape), "nu": w["nu"],
                   "collision": "KBC entropic", "storage": "f32", "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "forms": forms,
        "finite": finite,
        "failed_state": not healthy,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
