#!/usr/bin/env python3
"""Throughput of the entropic (KBC) lattice Boltzmann hot path on one MI355X.

A step is one pass of the whole path (geometry, pull streaming, moments, entropic equilibrium,
KBC collision with the per-node stabiliser, wall reconstruction and forces where the workload has
walls, store) over the workload's lattice.  The headline workload is ``turb256``: 256^3 periodic
box, seeded divergence-free turbulence (E(k) ~ k^4 exp(-2 (k/k0)^2), k0 = 4, rms 0.04), FP32
populations.  ``value`` is whole-job MLUPS (lattice-node updates per second / 1e6) with the
populations already resident in HBM.

Also reported on the same JSON line:
  roofline      -- the bulk sweep kernel's algorithmic HBM bytes per launch / its average launch
                   duration (HIP events recorded around each launch on the library's stream),
                   against the MI355X HBM peak of 8 TB/s; ``traffic`` comes from the committed
                   rocprofv3 counter summary when it was taken on the current kernel source.
  cpu_baseline  -- the FP64 CPU oracle, as it stands, on a bounded sample of the same workload.
  forms         -- the other forms at their workloads: FP32 / FP16 / BF16 storage on 512^3, the
                   moving-sphere channel (384x192x192), and a plain copy kernel as the measured
                   achievable HBM bandwidth.
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
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "sweep_f32_turb256_traffic.md")


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def sweep_source_hash() -> str:
    h = hashlib.sha256()
    for rel in SWEEP_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(nodes: int):
    """HBM bytes per sweep launch from the committed counter summary, or None when the summary is
    missing, for another size, or was taken on a different kernel source."""
    if not os.path.exists(TRAFFIC_PROFILE):
        return None
    text = open(TRAFFIC_PROFILE).read()
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
    """Deforming triangulated body (Sec. IV.B): the anguilliform swimmer of length L = 200 in the
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


def cpu_baseline(workload: str, budget_s: float = 15.0):
    """The FP64 oracle, unmodified, stepping the workload's own lattice on the host cores for a
    bounded number of steps (at least 2, until ~budget_s seconds of stepping)."""
    import oracle
    import workloads as WL
    w = WL.WORKLOADS[workload]
    rho, u = WL.initial_field(workload)
    sim = oracle.Simulation(w["shape"], w["nu"], rho, u)
    del rho, u
    steps = 0
    t0 = time.perf_counter()
    while True:
        sim.step(1)
        steps += 1
        el = time.perf_counter() - t0
        log(f"cpu_baseline: oracle step {steps} at {el:.1f}s")
        if steps >= 2 and el >= budget_s:
            break
    n = sim.N
    return {"value": n * steps / el / 1e6, "unit": "MLUPS", "cores": oracle.max_threads(), "kind": "oracle",
            "sample": f"{workload} ({w['shape'][0]}x{w['shape'][1]}x{w['shape'][2]}, FP64 C oracle): "
                      f"{steps} of its {w['steps']} steps, {el:.1f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default: the workload's step count)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="turb256")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--form-steps", type=int, default=100)
    ap.add_argument("--forms", default="copy,stabilisers,turb512,sphere384,settle,swimmer,adj128",
                    help="comma-separated subset of the extra forms to run")
    ap.add_argument("--probe-copy-mib", type=int, default=0,
                    help="after the headline run, copy a buffer of this many MiB 5 times (a plain copy kernel "
                         "of known size, used to scale the HBM byte counters of a rocprofv3 --pmc run)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on exactly one GPU: this build has no multi-GPU path (asked for --gpus "
              f"{args.gpus}, WORLD_SIZE={world}).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import workloads as WL
    from paper_1608_04658_amd import elbm

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(3)
    torch.cuda.set_device(0)
    elbm.load()

    w = WL.WORKLOADS[args.workload]
    steps = args.steps if args.steps is not None else w["steps"]
    shape = w["shape"]
    log(f"workload {args.workload} {shape}, generating the initial field")
    rho, u = WL.initial_field(args.workload)

    def init(lat):
        lat.init_equilibrium(rho, u)

    log(f"timing {steps} steps after {args.warmup} warm-up steps")
    mlups, ms_step, gbps, sweep_ms, info, lat = run_form(elbm, torch, shape, w["nu"], "f32", steps, args.warmup,
                                                         init, bodies=w.get("bodies"), channel=w.get("channel", False),
                                                         u_in=w.get("u_in", (0, 0, 0)))
    pops = lat.populations()
    finite = bool(torch.isfinite(pops).all().item())
    mass = float(pops.sum().item()) / lat.N
    del pops, lat
    torch.cuda.empty_cache()
    log(f"{args.workload}: {mlups:.0f} MLUPS, sweep {gbps:.0f} GB/s, {ms_step:.3f} ms/step, finite={finite}, "
        f"mean rho={mass:.6f}, fp64 nodes last step={info.fp64_nodes}")
    n_nodes = shape[0] * shape[1] * shape[2]
    roof = {"bound": "hbm", "achieved": round(gbps, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(gbps / HBM_PEAK_GBPS, 4), "traffic": traffic_from_profile(n_nodes),
            "kernel": "k_sweep<f32> (bulk stream-collide)", "bytes_per_launch": BYTES_PER_NODE["f32"] * n_nodes,
            "avg_launch_ms": round(sweep_ms, 4)}

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
            _, _, gb, _, _, lat = run_form(elbm, torch, shape, w["nu"], "f32", 100, 5, init,
                                           flags=elbm.FLAG_STREAM_ONLY)
            del lat
            torch.cuda.empty_cache()
            forms["pull_copy_GBps"] = round(gb, 1)
            roof["attainable_pull_copy"] = round(gb, 1)
            log(f"stream-only pull copy ({args.workload}) {gb:.0f} GB/s")
        if "turb512" in which:
            w5 = WL.WORKLOADS["turb512"]
            log("turb512: generating the initial field on the device")
            r5, u5 = WL.turbulence_device(512, w5["k0"], w5["urms"], w5["seed"])

            def init5(lat):
                elbm.elbm_init_equilibrium(lat.ctx, r5, u5)
                torch.cuda.synchronize()

            for st in ("f32", "f16", "bf16"):
                m, msps, gb, _, inf, lat = run_form(elbm, torch, w5["shape"], w5["nu"], st, args.form_steps, 5, init5)
                del lat
                torch.cuda.empty_cache()
                forms[f"turb512_{st}"] = {"MLUPS": round(m, 1), "ms_per_step": round(msps, 4),
                                          "sweep_GBps": round(gb, 1), "frac": round(gb / HBM_PEAK_GBPS, 4),
                                          "fp64_nodes_last_step": int(inf.fp64_nodes)}
                log(f"turb512 {st}: {m:.0f} MLUPS, sweep {gb:.0f} GB/s")
            del r5, u5
            torch.cuda.empty_cache()
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
        if "stabilisers" in which:
            # the same turb256 run with the exact stabiliser and with LBGK, for comparison
            for name, fl in (("exact_gamma", elbm.FLAG_EXACT_GAMMA), ("lbgk", elbm.FLAG_LBGK),
                             ("central", elbm.FLAG_CENTRAL)):
                m, msps, gb, _, _, lat = run_form(elbm, torch, shape, w["nu"], "f32", 100, 5, init, flags=fl)
                del lat
                torch.cuda.empty_cache()
                forms[f"{args.workload}_{name}"] = {"MLUPS": round(m, 1), "ms_per_step": round(msps, 4),
                                                    "sweep_GBps": round(gb, 1)}
                log(f"{args.workload} {name}: {m:.0f} MLUPS, sweep {gb:.0f} GB/s")
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

    cpu = None
    if not args.no_cpu_baseline:
        del rho, u
        cpu = cpu_baseline(args.workload)
        log(f"cpu_baseline {cpu['value']:.2f} MLUPS on {cpu['cores']} threads")

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
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
