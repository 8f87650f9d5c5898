"""Benchmark of the coupled ternary phase-field LB step on one MI355X.

Default workload: the porous-medium displacement, a 4096 x 2048 D2Q9 domain
of seeded random non-overlapping circles (radius U[8, 24], porosity 0.6,
diffuse solid of width 3), FP32 storage and arithmetic, contact angle 45
deg, density ratio 1, viscosity ratio 5, body force 1e-6 along x.  A step is
one coupled update of both lattices at every node (one launch of the fused
kernel).  Inputs are resident in HBM before the timed region.

Between the warmup steps and the timed region a settle phase keeps the device
stepping for --settle-s seconds (reported as settle_s / settle_steps): after
an idle gap the first few dozen launches run slower than the steady state.

Prints one JSON line: coupled MLUPS (whole-job), the roofline of the fused
kernel (algorithmic bytes per launch / HIP-event kernel time against the
8 TB/s HBM peak) and the CPU oracle timed on a bounded sample.  roofline.traffic
is null: the HBM traffic counters need a profiler run of their own; their
figures for each kernel are kept with its profile summary.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "coupled MLUPS + % HBM roofline; time-to-equilibrium learned vs plain"

def workload(name: str, nx: int = 4096, ny: int = 2048):
    from paper_2311_05091_amd import geometry as G
    if name == "porous_displacement":
        return [G.porous_medium(nx=nx, ny=ny)], "porous_displacement_%dx%d" % (nx, ny)
    if name == "cylinder_droplet":
        return [G.cylinder_droplet()], "cylinder_droplet_1024x1024"
    if name == "flat_wall_droplet":
        return [G.flat_wall_droplet()], "flat_wall_droplet_128x64"
    if name == "batched_sweep":
        # 512 independent rough-wall droplets, sides U{128..512}: the batched
        # workload of the warm-start data sweep, stepped without retirement
        specs = G.batched_sweep(n_domains=512, smin=128, smax=512)
        return specs, "batched_sweep_512_domains_%d_nodes" % sum(s.nx * s.ny for s in specs)
    raise SystemExit("unknown workload %s" % name)


def cpu_baseline(spec, steps: int):
    """The FP64 oracle on the host cores: `steps` steps of the full domain."""
    import oracle
    oracle.build(force=False)
    p = oracle.make_params(spec.nx, spec.ny, periodic_x=spec.periodic_x, periodic_y=spec.periodic_y,
                           d0=spec.d0, D=spec.D, sigma12=spec.sigma12, theta_deg=spec.theta_deg,
                           kappa=spec.kappa, rho=spec.rho, mu=spec.mu, M_cst=spec.M_cst,
                           M_deg=spec.M_deg, tau_phi=spec.tau_phi, Fb=spec.Fb)
    sim = oracle.Sim(p, spec.phi0, spec.phi1)
    sim.step(1)  # first-touch of the pass buffers
    t0 = time.perf_counter()
    sim.step(steps)
    dt = time.perf_counter() - t0
    n = spec.nx * spec.ny
    return {"value": round(n * steps / dt / 1e6, 4), "unit": "MLUPS", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": "%d FP64 steps of the full %dx%d domain (after 1 untimed step)" % (steps, spec.nx, spec.ny)}


def cpu_baseline3(spec, steps: int):
    """The FP64 3D oracle on the host cores: `steps` steps of a 64^3 block of
    the same workload (the full domain would take minutes per step)."""
    import oracle
    oracle.build(force=False)
    n = 64
    phi0 = np.ascontiguousarray(spec.phi0[:n, :n, :n])
    phi1 = np.ascontiguousarray(spec.phi1[:n, :n, :n])
    p = oracle.make_params3(n, n, n, periodic=spec.periodic, d0=spec.d0, D=spec.D, sigma12=spec.sigma12,
                            theta_deg=spec.theta_deg, rho=spec.rho, mu=spec.mu, M_cst=spec.M_cst,
                            M_deg=spec.M_deg, tau_phi=spec.tau_phi, Fb=spec.Fb)
    sim = oracle.Sim3(p, phi0, phi1)
    sim.step(1)
    t0 = time.perf_counter()
    sim.step(steps)
    dt = time.perf_counter() - t0
    return {"value": round(n ** 3 * steps / dt / 1e6, 4), "unit": "MLUPS", "cores": oracle.num_threads(),
            "kind": "oracle", "sample": "%d FP64 steps of a 64^3 block of the workload (after 1 untimed step)" % steps}


def run3d(args, copy_gbs):
    """The 3D (D3Q15) coupled step on the porous-spheres workload."""
    import torch
    from paper_2311_05091_amd import geometry3d as G3
    from paper_2311_05091_amd.lbm3 import Context3
    spec = G3.porous_spheres(n=args.n3)
    nodes = spec.nx * spec.ny * spec.nz
    wname = "porous_spheres_3d_%d^3" % args.n3
    print("[bench] workload %s, %d nodes, precision %d, solid share %.3f" %
          (wname, nodes, args.precision, float((spec.phi0 > 0.5).mean())), flush=True)
    ctx = Context3(precision=args.precision)
    ctx.add_domain(spec)
    ctx.finalize()
    if args.tile:
        ctx.set_tile(args.tile)
    tx, ty, tz = ctx.tile()
    print("[bench] tile %dx%dx%d" % (tx, ty, tz), flush=True)
    ctx.step(args.warmup)
    torch.cuda.synchronize()
    settle_steps = 0
    t_settle = time.perf_counter()
    while time.perf_counter() - t_settle < args.settle_s:
        ctx.step(5)
        settle_steps += 5
    torch.cuda.synchronize()
    settle_s = time.perf_counter() - t_settle
    ctx.kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kern_ms, launches = ctx.kernel_timing(False)
    mass = ctx.mass(0)
    print("[bench] %d steps in %.3f s, kernel avg %.4f ms over %d launches, mass %.10e" %
          (args.steps, dt, kern_ms, launches, mass), flush=True)
    if not math.isfinite(mass):
        raise SystemExit("bench: the 3D state is not finite after the timed steps; no figure reported")
    bpn = ctx.bytes_per_node(0)
    achieved = bpn * nodes / (kern_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "bytes_per_node": bpn,
            "kernel_ms": round(kern_ms, 5)}
    if copy_gbs:
        roof["copy_GBs"] = round(copy_gbs, 1)
        roof["frac_of_copy"] = round(achieved / copy_gbs, 4)
    out = {
        "metric": METRIC, "value": round(nodes * args.steps / dt / 1e6, 2), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "settle_s": round(settle_s, 3), "settle_steps": settle_steps,
        "ms_per_step": round(dt / args.steps * 1e3, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if args.precision == 32 else "f64", "data": "synthetic",
        "config": {"workload": wname, "nodes": nodes, "lattice": "D3Q15 x 2 (CH + NS)", "tile": [tx, ty, tz],
                   "precision": args.precision},
        "roofline": roof,
    }
    ctx.close()
    if not args.no_cpu:
        print("[bench] cpu baseline: 3D oracle, %d steps" % args.cpu_steps, flush=True)
        out["cpu_baseline"] = cpu_baseline3(spec, args.cpu_steps)
    print(json.dumps(out), flush=True)


def run3f(args, copy_gbs):
    """The 3f model (two CH lattices, phi0 evolving) on drops in layers."""
    import torch
    from paper_2311_05091_amd import geometry3f as G3F
    from paper_2311_05091_amd.lbm3f import Context3F
    spec = G3F.drops_in_layers(n=args.n3f, n_drops=max(8, (args.n3f // 128) ** 2 // 2), rmin=12.0, rmax=48.0,
                               rho=(2.0, 3.0, 1.0), mu=(0.2, 0.3, 0.1), sigma01=0.012, sigma02=0.008, sigma12=0.01)
    nodes = spec.nx * spec.ny
    wname = "drops_in_layers_3f_%dx%d" % (spec.nx, spec.ny)
    print("[bench] workload %s, %d nodes, precision %d" % (wname, nodes, args.precision), flush=True)
    ctx = Context3F(precision=args.precision)
    ctx.add_domain(spec)
    ctx.finalize()
    ctx.step(args.warmup)
    torch.cuda.synchronize()
    settle_steps = 0
    t_settle = time.perf_counter()
    while time.perf_counter() - t_settle < args.settle_s:
        ctx.step(10)
        settle_steps += 10
    torch.cuda.synchronize()
    settle_s = time.perf_counter() - t_settle
    ctx.kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kern_ms, launches = ctx.kernel_timing(False)
    mass = ctx.mass(0)
    print("[bench] %d steps in %.3f s, kernel avg %.4f ms over %d launches, masses %.10e %.10e" %
          (args.steps, dt, kern_ms, launches, mass[0], mass[1]), flush=True)
    if not np.isfinite(mass).all():
        raise SystemExit("bench: the 3f state is not finite after the timed steps; no figure reported")
    bpn = ctx.bytes_per_node(0)
    achieved = bpn * nodes / (kern_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "bytes_per_node": bpn,
            "kernel_ms": round(kern_ms, 5)}
    if copy_gbs:
        roof["copy_GBs"] = round(copy_gbs, 1)
        roof["frac_of_copy"] = round(achieved / copy_gbs, 4)
    out = {
        "metric": METRIC, "value": round(nodes * args.steps / dt / 1e6, 2), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "settle_s": round(settle_s, 3), "settle_steps": settle_steps,
        "ms_per_step": round(dt / args.steps * 1e3, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if args.precision == 32 else "f64", "data": "synthetic",
        "config": {"workload": wname, "nodes": nodes, "lattice": "D2Q9 x 3 (two CH + NS), 3f model",
                   "tile": [64, 32], "precision": args.precision},
        "roofline": roof,
    }
    ctx.close()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="porous_displacement")
    ap.add_argument("--nx", type=int, default=4096, help="porous workload width")
    ap.add_argument("--ny", type=int, default=2048, help="porous workload height")
    ap.add_argument("--precision", type=int, default=32)
    ap.add_argument("--n3", type=int, default=256, help="edge of the 3D porous workload (--workload porous3d)")
    ap.add_argument("--n3f", type=int, default=2048, help="edge of the 3f workload (--workload drops3f)")
    ap.add_argument("--tile", type=int, default=0, help="tile code; 0 = autotune (per size class for batches)")
    ap.add_argument("--tile-cache", default=None, help="JSON cache of the per-size-class autotuner")
    ap.add_argument("--launch-mode", type=int, default=0,
                    help="0: one launch per step; 1: one persistent launch for all steps (strip tiles)")
    ap.add_argument("--to-residual", type=float, default=0.0,
                    help="> 0: run the batch from its initial state to this residual (run_to_residual, "
                         "at most --steps steps) and report the wall time instead of the step rate")
    ap.add_argument("--check-every", type=int, default=100, help="residual check interval for --to-residual")
    ap.add_argument("--settle-s", type=float, default=0.3,
                    help="seconds of untimed steps run right before the timed region, after the "
                         "warmup steps: after an idle gap of even 50 ms the device runs the first "
                         "~60 launches 5-18%% slower than in steady state")
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-copy-ceiling", dest="copy_ceiling", action="store_false",
                    help="skip the 1 GiB device copy that measures the achievable HBM bandwidth")
    ap.add_argument("--copy-mib", type=int, default=256,
                    help="size of the plain device copy run once before the steps; its "
                         "FETCH_SIZE/WRITE_SIZE counters calibrate the HBM traffic figures")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the library runs on one GPU only (no multi-GPU path); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2311_05091_amd.lbm import Context, size_class

    if args.copy_mib > 0:
        # reference copy kernel of known size (reads and writes copy_mib MiB)
        src = torch.ones(args.copy_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    copy_gbs = None
    if args.copy_ceiling:
        # achievable HBM bandwidth: the library's non-temporal device copy
        from paper_2311_05091_amd.lbm import copy_bandwidth
        copy_gbs = copy_bandwidth(1 << 30, nontemporal=True) / 1e9
        print("[bench] device copy (1 GiB, non-temporal): %.1f GB/s" % copy_gbs, flush=True)

    if args.workload == "porous3d":
        return run3d(args, copy_gbs)
    if args.workload == "drops3f":
        return run3f(args, copy_gbs)
    specs, wname = workload(args.workload, args.nx, args.ny)
    if args.to_residual > 0:
        return run_residual(args, specs, wname)
    nodes = sum(s.nx * s.ny for s in specs)
    print("[bench] workload %s, %d nodes, precision %d" % (wname, nodes, args.precision), flush=True)
    ctx = Context(precision=args.precision)
    for s in specs:
        ctx.add_domain(s)
    ctx.finalize()
    per_class = None
    if args.tile:
        ctx.set_tile(args.tile)
    elif len(specs) > 1 and args.launch_mode == 0:
        # a batch of many sizes: one tile code per size class, or the best
        # single code for the whole batch, whichever steps the batch faster
        # (each class is timed alone, which does not see how the classes
        # share the device)
        import tempfile
        cache = args.tile_cache or os.path.join(tempfile.mkdtemp(prefix="tpf_tiles_"), "tiles.json")

        def batch_ms(n=20):
            ctx.step(5)
            torch.cuda.synchronize()
            t = time.perf_counter()
            ctx.step(n)
            torch.cuda.synchronize()
            return (time.perf_counter() - t) / n * 1e3

        ctx.autotune_classes(steps=10, cache_path=cache)
        t_class = batch_ms()
        ctx.autotune(steps=10)
        t_single = batch_ms()
        print("[bench] batch step with per-class codes %.3f ms, one code %.3f ms" % (t_class, t_single), flush=True)
        if t_class <= t_single:
            ctx.autotune_classes(steps=10, cache_path=cache)   # the cached choice, no timing
            per_class = {}
            for i, sp in enumerate(specs):
                key = size_class(args.precision, sp.nx, sp.ny, sp.rho[1] != sp.rho[2])
                per_class.setdefault(key, [ctx.domain_tile(i), 0])[1] += 1
            print("[bench] tile per size class (code, domains): %s" % per_class, flush=True)
    else:
        ctx.autotune(steps=30)
    code, tx, ty = ctx.tile()
    if args.launch_mode:
        ctx.set_launch_mode(args.launch_mode)
    print("[bench] tile %d (%dx%d), launch mode %d" % (code, tx, ty, args.launch_mode), flush=True)
    ctx.step(args.warmup)
    torch.cuda.synchronize()
    # settle: keep the device busy until its clocks hold their steady state, so
    # that the timed launches do not start on a ramp (each call returns after
    # the stream has drained; the gaps between calls are microseconds)
    settle_steps = 0
    t_settle = time.perf_counter()
    while time.perf_counter() - t_settle < args.settle_s:
        ctx.step(25)
        settle_steps += 25
    torch.cuda.synchronize()
    settle_s = time.perf_counter() - t_settle

    ctx.kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kern_ms, launches = ctx.kernel_timing(False)
    d = ctx.diag(0)
    print("[bench] %d steps in %.3f s, kernel avg %.4f ms over %d launches, mass %.10e" %
          (args.steps, dt, kern_ms, launches, d["mass"]), flush=True)
    if not math.isfinite(d["mass"]):
        raise SystemExit("bench: the state is not finite after the timed steps; no figure reported")

    mlups = nodes * args.steps / dt / 1e6
    bpn = ctx.bytes_per_node(0)
    achieved = bpn * nodes / (kern_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None,
            "bytes_per_node": bpn, "kernel_ms": round(kern_ms, 5)}
    if copy_gbs:
        roof["copy_GBs"] = round(copy_gbs, 1)
        roof["frac_of_copy"] = round(achieved / copy_gbs, 4)
    out = {
        "metric": METRIC, "value": round(mlups, 2), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "settle_s": round(settle_s, 3),
        "settle_steps": settle_steps, "ms_per_step": round(dt / args.steps * 1e3, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if args.precision == 32 else "f64", "data": "synthetic",
        "config": {"workload": wname, "nodes": nodes, "lattice": "D2Q9 x 2 (CH + NS)",
                   "tile": [tx, ty] if per_class is None else per_class, "precision": args.precision,
                   "launch_mode": args.launch_mode},
        "roofline": roof,
    }
    ctx.close()
    if not args.no_cpu:
        print("[bench] cpu baseline: oracle, %d steps" % args.cpu_steps, flush=True)
        out["cpu_baseline"] = cpu_baseline(specs[0], args.cpu_steps)
    print(json.dumps(out), flush=True)


def run_residual(args, specs, wname):
    """Wall time of one run_to_residual call over the whole batch from its
    initial state: every domain steps until its residual falls below the
    tolerance (checked every --check-every steps) or --steps steps have run.
    A first context of the same batch warms the kernels up."""
    import torch
    from paper_2311_05091_amd.lbm import Context

    def make():
        ctx = Context(precision=args.precision)
        for s in specs:
            ctx.add_domain(s)
        ctx.finalize()
        if args.tile:
            ctx.set_tile(args.tile)
        elif args.launch_mode == 0:
            ctx.autotune_classes(steps=10, cache_path=args.tile_cache)
        if args.launch_mode:
            ctx.set_launch_mode(args.launch_mode)
        return ctx

    warm = make()
    warm.run_to_residual(args.to_residual, check_every=args.check_every, max_steps=max(args.warmup, 1))
    warm.close()
    ctx = make()
    code, tx, ty = ctx.tile()
    print("[bench] %s to residual %.1e, check every %d, at most %d steps, tile %d, launch mode %d"
          % (wname, args.to_residual, args.check_every, args.steps, code, args.launch_mode), flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, steps = ctx.run_to_residual(args.to_residual, check_every=args.check_every, max_steps=args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    node_steps = sum(s.nx * s.ny * int(n) for s, n in zip(specs, steps))
    retired = sum(1 for n in steps if n < args.steps)
    out = {"metric": "batch wall time to residual", "value": round(dt, 4), "unit": "s",
           "higher_is_better": False, "rc": int(rc), "domains": len(specs), "retired": retired,
           "steps_min": int(min(steps)), "steps_max": int(max(steps)),
           "node_updates_per_s": round(node_steps / dt, 1),
           "config": {"workload": wname, "tol": args.to_residual, "check_every": args.check_every,
                      "max_steps": args.steps, "tile": code, "precision": args.precision,
                      "launch_mode": args.launch_mode}}
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
