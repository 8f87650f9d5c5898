"""Batched sweep, surrogate training and the learned warm start.

1. ``sweep``: many independent rough-wall droplet domains advance together in
   the batched launcher until each one's residual drops below a tolerance (or
   a step cap); their equilibrium phase fields become training data.
2. ``train``: the encoder-decoder of ``surrogate.py`` learns phi1 from (phi0,
   contact angle, volume) on 256 x 256 resamplings, with x-mirror augmentation
   (the problem is symmetric under x -> -x).
3. ``evaluate``: on held-out geometries, the time to reach the tolerance from
   the plain initial condition is compared with the time for inference +
   mass-projected warm start + relaxation; a warm start that fails (non-finite
   values, or the step cap) falls back to the plain initial condition.

All LB and network arithmetic runs in the HIP libraries; this module is
orchestration (timing with device synchronisation, bookkeeping).
"""
from __future__ import annotations

import json
import math
import time
from typing import Dict, List, Optional

import numpy as np

from . import geometry as G
from .lbm import Context, TPF_ENAN, TPF_OK
from . import surrogate as S


def _sync():
    import torch
    torch.cuda.synchronize()


def sweep(specs: List[G.DomainSpec], tol: float, check_every: int, max_steps: int, precision: int = 32,
          tile: Optional[int] = None, launch_mode: int = 2, group: int = 0, log=None) -> Dict:
    """Advances the domains to r < tol (batched; converged domains retire) and
    returns their fields and statistics.  group > 0 runs consecutive groups of
    that many domains one after another (one context each) and logs after
    each; the wall time is then the sum over groups."""
    if group and group < len(specs):
        parts = [sweep(specs[i:i + group], tol, check_every, max_steps, precision, tile, launch_mode, 0, log)
                 for i in range(0, len(specs), group)]
        out = {"phi1": [], "steps": [], "status": [], "residual": []}
        wall = 0.0
        for part in parts:
            for key in out:
                out[key].extend(list(part[key]))
            wall += part["wall_s"]
        out = {k: (v if k == "phi1" else np.array(v)) for k, v in out.items()}
        out["rc"] = min(p["rc"] for p in parts)
        out["wall_s"] = wall
        out["nodes"] = sum(sp.nx * sp.ny for sp in specs)
        node_steps = float(sum(int(out["steps"][i]) * specs[i].nx * specs[i].ny for i in range(len(specs))))
        out["mlups"] = node_steps / wall / 1e6
        return out
    ctx = Context(precision=precision)
    for sp in specs:
        ctx.add_domain(sp)
    ctx.finalize()
    if tile:
        ctx.set_tile(tile)
    if launch_mode:
        ctx.set_launch_mode(launch_mode)
    _sync()
    t0 = time.perf_counter()
    rc, steps = ctx.run_to_residual(tol, check_every=check_every, max_steps=max_steps)
    _sync()
    wall = time.perf_counter() - t0
    phi, status, res = [], [], []
    for i in range(len(specs)):
        d = ctx.diag(i)
        status.append(d["status"])
        res.append(d["residual"])
        phi.append(ctx.moments(i)[0])
    nodes = sum(sp.nx * sp.ny for sp in specs)
    node_steps = float(sum(int(steps[i]) * specs[i].nx * specs[i].ny for i in range(len(specs))))
    out = {"phi1": phi, "steps": np.asarray(steps), "status": np.array(status), "residual": np.array(res),
           "wall_s": wall, "rc": rc, "nodes": nodes, "mlups": node_steps / wall / 1e6}
    ctx.close()
    if log:
        log(json.dumps({"sweep_group": len(specs), "nodes": nodes, "wall_s": round(wall, 3),
                        "steps_mean": float(np.mean(steps)), "mlups": round(out["mlups"], 1)}))
    return out


def build_dataset(specs: List[G.DomainSpec], phi_eq: List[np.ndarray], status) -> Dict[str, np.ndarray]:
    """Network inputs/targets on the 256 x 256 grid (GPU bilinear resampling)."""
    X0, X1, TH, VOL, Y = [], [], [], [], []
    for s, phi, st in zip(specs, phi_eq, status):
        if st == TPF_ENAN or not np.isfinite(phi).all():
            continue
        X0.append(S.resample(s.phi0[None], S.RES, S.RES)[0])
        X1.append(S.resample(s.phi1[None], S.RES, S.RES)[0])
        TH.append(s.theta_deg)
        VOL.append(S.volume_feature(s.phi1))
        Y.append(np.clip(S.resample(phi[None], S.RES, S.RES)[0], 0.0, 1.0))
    return {"phi0": np.array(X0, np.float32), "phi1_init": np.array(X1, np.float32),
            "theta": np.array(TH, np.float32), "vol": np.array(VOL, np.float32),
            "target": np.array(Y, np.float32)}


def predict_fields(net: S.UNet, specs: List[G.DomainSpec], batch: int = 32):
    """Warm-start fields (mass-projected, on each domain's grid) for the
    domains; None where the prediction is unusable."""
    def to_res(fields):
        # one resampling call per group of equal-size domains; a field already
        # at the network's resolution is kept as it is (the corner-aligned
        # bilinear map is then the identity)
        shape = fields[0].shape
        if all(f.shape == shape for f in fields):
            a = np.stack(fields).astype(np.float32)
            return a if shape == (S.RES, S.RES) else S.resample(a, S.RES, S.RES)
        return np.stack([S.resample(f[None], S.RES, S.RES)[0] for f in fields])

    fields = []
    for b0 in range(0, len(specs), batch):
        grp = specs[b0:b0 + batch]
        phi0 = to_res([sp.phi0 for sp in grp])
        phi1 = to_res([sp.phi1 for sp in grp])
        th = np.array([sp.theta_deg for sp in grp], np.float32)
        vol = np.array([S.volume_feature(sp.phi1) for sp in grp], np.float32)
        pred = net.predict_device(phi0, th, vol, phi1)
        fields.extend(S.warm_start_fields(pred, [sp.phi0 for sp in grp], [float(np.sum(sp.phi1)) for sp in grp]))
    return fields


def rel_l2(a: np.ndarray, b: np.ndarray) -> float:
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def calibrate_gate(net: S.UNet, specs: List[G.DomainSpec], phi_eq: List[np.ndarray], q: float = 0.75) -> float:
    """Gate of the warm start from validation domains (not trained on): the
    q-quantile of the surrogate's error (rel. L2 of the warm-start field
    against the swept equilibrium).  A prediction that lies closer than this
    to the plain initial condition carries no information beyond it, and the
    plain start is kept."""
    fields = predict_fields(net, specs)
    errs = [rel_l2(f, e) for f, e in zip(fields, phi_eq) if f is not None and np.isfinite(e).all()]
    return float(np.quantile(errs, q)) if errs else 0.0


def train(data: Dict[str, np.ndarray], epochs: int = 30, batch: int = 8, lr: float = 3e-4, seed: int = 0,
          log=print, time_budget_s: float = 1e9, warmup_steps: int = 100) -> S.UNet:
    """Adam on the cross-entropy loss.  The learning rate ramps up linearly over
    the first ``warmup_steps`` updates (the network has no normalisation
    layers, and a full-size first step can push the decoder into saturation)
    and decays along a half cosine to zero at the last planned update."""
    import torch
    net = S.UNet(seed=seed)
    n = len(data["theta"])
    rng = np.random.default_rng(seed)
    t0 = time.perf_counter()
    hist = []
    n_upd = max(epochs * (n // batch), 1)
    for ep in range(epochs):
        perm = rng.permutation(n)
        losses = []
        for b0 in range(0, n - batch + 1, batch):
            idx = perm[b0:b0 + batch]
            flip = rng.random(batch) < 0.5

            def mirrored(a):
                return np.ascontiguousarray(np.where(flip[:, None, None], a[:, :, ::-1], a))

            phi0 = mirrored(data["phi0"][idx])
            phi1 = mirrored(data["phi1_init"][idx])
            tgt = mirrored(data["target"][idx])
            net.pack(phi0, data["theta"][idx], data["vol"][idx], phi1)
            t = torch.tensor(np.ascontiguousarray(tgt).ravel(), device=net.dev)
            # linear warm-up, then cosine decay to zero over the planned updates
            k = net.t + 1
            step_lr = lr * min(1.0, k / max(warmup_steps, 1)) * 0.5 * (1.0 + math.cos(math.pi * min(k / n_upd, 1.0)))
            losses.append(net.train_step(batch, t, lr=step_lr).clone())
        ep_loss = float(torch.stack(losses).mean().item()) if losses else float("nan")
        hist.append(ep_loss)
        log(json.dumps({"epoch": ep, "loss": ep_loss, "t": round(time.perf_counter() - t0, 1)}))
        if time.perf_counter() - t0 > time_budget_s:
            break
    net.history = hist
    return net


def warm_kernels(precision: int = 32, launch_mode: int = 2):
    """Loads every LB kernel either timed side may run (the tile shapes launch
    mode 2 picks from, the reductions, the moments kernel) in an untimed
    throwaway context, so that neither side pays for first-launch loading."""
    sp = G.held_out_set(n_domains=1, s=128, seed0=987654)[0]
    ctx = Context(precision=precision)
    ctx.add_domain(sp)
    ctx.finalize()
    for code in (17, 9, 8, 2, 1):
        ctx.set_tile(code)
        ctx.step(2)
    ctx.set_tile(0)
    if launch_mode:
        ctx.set_launch_mode(launch_mode)
    ctx.run_to_residual(1e-30, check_every=2, max_steps=4)
    ctx.moments(0)
    ctx.diag(0)
    ctx.close()
    _sync()


def steps_to_reference(ctx: Context, ref: List[np.ndarray], eps_list: List[float], check_every: int,
                       cap: int) -> np.ndarray:
    """Steps each domain of ctx takes until its phi1 lies within each eps of
    ``eps_list`` (rel. L2) of ref, checked every ``check_every`` steps (and at
    step 0); a domain leaves the batch once it is within the smallest eps.
    Returns [len(eps_list), domains], -1 where a threshold is not reached
    within ``cap`` steps (or the domain turns non-finite)."""
    n = len(ref)
    eps = sorted(eps_list, reverse=True)
    steps = np.full((len(eps), n), -1, dtype=np.int64)
    t = 0
    while True:
        for i in range(n):
            if steps[-1, i] < 0:
                phi = ctx.moments(i)[0]
                if not np.isfinite(phi).all():
                    continue
                d = rel_l2(phi, ref[i])
                for k, e in enumerate(eps):
                    if steps[k, i] < 0 and d < e:
                        steps[k, i] = t
                if steps[-1, i] >= 0:
                    ctx.set_active(i, False)
        if (steps[-1] >= 0).all() or t >= cap:
            return steps
        ctx.step(check_every)
        t += check_every


def equilibrium_eval(net: S.UNet, specs: List[G.DomainSpec], ref_steps: int, eps_list: List[float],
                     check_every: int, cap: int, gate: float = 0.0, precision: int = 32, launch_mode: int = 2,
                     log=print) -> Dict:
    """Time to equilibrium measured on the state itself, not on its change per
    step: the reference of each domain is its plain start advanced by
    ``ref_steps`` steps (its per-step residual at that point is reported);
    then the plain start and the warm start (the surrogate's mass-projected
    prediction, kept where it passes the gate) each run until phi1 is within
    eps (rel. L2) of that reference, for each eps of ``eps_list``.  A side
    that does not get there within ``cap`` counts as slower; domains whose
    reference is not finite are left out."""
    ctx = Context(precision=precision)
    for sp in specs:
        ctx.add_domain(sp)
    ctx.finalize()
    if launch_mode:
        ctx.set_launch_mode(launch_mode)
    ctx.step(ref_steps - 1000)
    before = [ctx.moments(i)[0] for i in range(len(specs))]
    ctx.step(1000)
    ref = [ctx.moments(i)[0] for i in range(len(specs))]
    ctx.close()
    res = [rel_l2(a, b) / 1000.0 if np.isfinite(b).all() else float("nan") for a, b in zip(before, ref)]
    keep = [i for i in range(len(specs)) if np.isfinite(ref[i]).all()]
    specs = [specs[i] for i in keep]
    ref = [ref[i] for i in keep]
    res = [res[i] for i in keep]
    log(json.dumps({"reference_steps": ref_steps, "domains": len(specs), "dropped_nonfinite": len(before) - len(keep),
                    "reference_residual_median": float(np.median(res)), "reference_residual_max": float(np.max(res))}))
    sides = {}
    gated = 0
    for side in ("plain", "learned"):
        ctx = Context(precision=precision)
        for sp in specs:
            ctx.add_domain(sp)
        ctx.finalize()
        if launch_mode:
            ctx.set_launch_mode(launch_mode)
        if side == "learned":
            for i, f in enumerate(predict_fields(net, specs)):
                if f is None or rel_l2(f, specs[i].phi1) < gate:
                    gated += 1
                else:
                    ctx.set_phi1(i, f)
        sides[side] = steps_to_reference(ctx, ref, eps_list, check_every, cap)
        ctx.close()
    eps = sorted(eps_list, reverse=True)
    big = float(cap + check_every)
    per_eps = []
    for k, e in enumerate(eps):
        ps, ls = sides["plain"][k].astype(float), sides["learned"][k].astype(float)
        pinf, linf = np.where(ps < 0, big, ps), np.where(ls < 0, big, ls)
        both = (ps >= 0) & (ls >= 0)
        per_eps.append({"eps": e, "plain_reached": int((ps >= 0).sum()), "learned_reached": int((ls >= 0).sum()),
                        "learned_slower_share": float(np.mean(linf > pinf)),
                        "learned_faster_share": float(np.mean(linf < pinf)),
                        "work_ratio_reached_both": float(ps[both].sum() / max(ls[both].sum(), 1.0))
                        if both.any() else float("nan"),
                        "work_ratio_cap_counted": float(pinf.sum() / max(linf.sum(), 1.0)),
                        "plain_steps_median": float(np.median(pinf)),
                        "learned_steps_median": float(np.median(linf))})
    out = {"domains": len(specs), "reference_steps": ref_steps,
           "reference_residual_median": float(np.median(res)), "check_every": check_every, "cap": cap,
           "gate": gate, "gated_to_plain": gated, "per_eps": per_eps,
           "per_domain": {"plain": sides["plain"].tolist(), "learned": sides["learned"].tolist(),
                          "theta": [sp.theta_deg for sp in specs], "eps": eps}}
    log(json.dumps({k: v for k, v in out.items() if k != "per_domain"}))
    return out


def evaluate(net: S.UNet, specs: List[G.DomainSpec], tol: float, check_every: int, max_steps: int,
             precision: int = 32, launch_mode: int = 2, gate: float = 0.0, probe_steps: int = 0,
             log=print) -> Dict:
    """Plain vs learned time to r < tol on the same held-out domains, each side
    one batch (converged domains retire).

    Learned side, timed as a whole: an optional probe (all domains relax from
    the plain initial condition for ``probe_steps`` steps; those that converge
    within it need no surrogate), then inference for the others, the
    mass-projected warm start (kept only where it differs from the plain
    initial condition by at least ``gate`` in relative L2; elsewhere the plain
    relaxation simply continues) and relaxation to the tolerance.  Steps of
    the probe count for every domain.  A domain that turns non-finite restarts
    from the plain initial condition afterwards (its wasted steps count
    against it).  Work is compared as node-steps (each domain's steps x its
    nodes), which is what the batched GPU time follows once the batch is
    large; the batch wall times are reported beside it."""
    warm_kernels(precision, launch_mode)
    plain = sweep(specs, tol, check_every, max_steps, precision=precision, launch_mode=launch_mode)
    log(json.dumps({"plain_wall_s": round(plain["wall_s"], 3), "plain_rc": plain["rc"],
                    "plain_steps_mean": float(np.mean(plain["steps"]))}))
    ctx = Context(precision=precision)
    for sp in specs:
        ctx.add_domain(sp)
    ctx.finalize()
    if launch_mode:
        ctx.set_launch_mode(launch_mode)
    # the network's kernels are loaded by an untimed pass first, as the LB
    # kernels were by the plain run
    predict_fields(net, specs[:1])
    _sync()
    t0 = time.perf_counter()
    n = len(specs)
    steps = np.zeros(n, dtype=np.int64)
    todo = list(range(n))
    if probe_steps > 0:
        rc1, s1 = ctx.run_to_residual(tol, check_every=check_every, max_steps=probe_steps)
        steps += s1
        nan = {i for i in range(n) if rc1 == TPF_ENAN and ctx.diag(i)["status"] == TPF_ENAN}
        todo = [i for i in range(n) if s1[i] >= probe_steps and i not in nan]
        for i in range(n):
            if s1[i] < probe_steps and i not in nan:
                ctx.set_active(i, False)  # converged within the probe: done
    t_probe = time.perf_counter() - t0
    fields: List = [None] * n
    for i, f in zip(todo, predict_fields(net, [specs[i] for i in todo]) if todo else []):
        fields[i] = f
    empty = sum(fields[i] is None for i in todo)
    gated = 0
    for i in todo:
        f = fields[i]
        if f is not None and rel_l2(f, specs[i].phi1) < gate:
            gated += 1
        elif f is not None:
            ctx.set_phi1(i, f)
    _sync()
    t_inf = time.perf_counter() - t0 - t_probe
    if todo:
        _, s2 = ctx.run_to_residual(tol, check_every=check_every, max_steps=max(max_steps - probe_steps, 0))
        steps += s2
    _sync()
    t_learn = time.perf_counter() - t0
    phi_l = [ctx.moments(i)[0] for i in range(len(specs))]
    status_l = [ctx.diag(i)["status"] for i in range(len(specs))]
    ctx.close()
    # domains whose warm start failed (non-finite) restart from the plain
    # initial condition in a batch of their own; their wasted steps and that
    # batch's time count against the learned side
    bad = [i for i in range(len(specs)) if status_l[i] == TPF_ENAN]
    if bad:
        re = sweep([specs[i] for i in bad], tol, check_every, max_steps, precision=precision,
                   launch_mode=launch_mode)
        t_learn += re["wall_s"]
        for k, i in enumerate(bad):
            steps[i] += int(re["steps"][k])
            phi_l[i] = re["phi1"][k]
            status_l[i] = int(re["status"][k])
    err = [float(np.linalg.norm(fields[i] - plain["phi1"][i]) / np.linalg.norm(plain["phi1"][i]))
           if fields[i] is not None else float("nan") for i in range(len(specs))]
    agree = [float(np.linalg.norm(phi_l[i] - plain["phi1"][i]) / np.linalg.norm(plain["phi1"][i]))
             for i in range(len(specs))]
    nodes = np.array([sp.nx * sp.ny for sp in specs], dtype=float)
    ps = np.asarray(plain["steps"], dtype=float)
    ls = steps.astype(float)
    ok = np.array([plain["status"][i] != TPF_ENAN and status_l[i] != TPF_ENAN for i in range(len(specs))])
    ratio = ps[ok] / np.maximum(ls[ok], 1.0)
    finite_err = [e for e in err if np.isfinite(e)]
    out = {"domains": len(specs), "tol": tol, "check_every": check_every, "cap": max_steps,
           "plain_wall_s": plain["wall_s"], "learned_wall_s": t_learn, "inference_s": t_inf,
           "probe_steps": probe_steps, "probe_s": t_probe, "probe_converged": n - len(todo),
           "wall_speedup": plain["wall_s"] / t_learn,
           "work_speedup": float((ps[ok] * nodes[ok]).sum() / max((ls[ok] * nodes[ok]).sum(), 1.0)),
           "plain_steps_mean": float(ps.mean()), "learned_steps_mean": float(ls.mean()),
           "steps_ratio_median": float(np.median(ratio)) if ratio.size else float("nan"),
           "faster_share": float(np.mean(ratio > 1.0)) if ratio.size else float("nan"),
           "plain_capped": int((ps >= max_steps).sum()), "learned_capped": int((ls >= max_steps).sum()),
           "empty_predictions": empty, "gate": gate, "gated_to_plain": gated, "restarted": len(bad),
           "plain_nan": int(np.sum(np.asarray(plain["status"]) == TPF_ENAN)),
           "learned_nan": int(np.sum(np.asarray(status_l) == TPF_ENAN)),
           "surrogate_rel_l2_mean": float(np.mean(finite_err)) if finite_err else float("nan"),
           "surrogate_rel_l2_median": float(np.median(finite_err)) if finite_err else float("nan"),
           "final_state_rel_l2_median": float(np.median(agree)), "final_state_rel_l2_max": float(np.max(agree)),
           "per_domain": {"plain_steps": ps.astype(int).tolist(), "learned_steps": ls.astype(int).tolist(),
                          "theta": [sp.theta_deg for sp in specs], "surrogate_rel_l2": err,
                          "final_state_rel_l2": agree}}
    log(json.dumps({k: v for k, v in out.items() if k != "per_domain"}))
    return out


def save_params(net: S.UNet, path: str, gate: float = 0.0):
    p = net.params_numpy()
    flat = {"gate": np.array(gate)}
    for k, (w, b) in p.items():
        flat[k + ".w"] = w.astype(np.float32)
        flat[k + ".b"] = b.astype(np.float32)
    np.savez_compressed(path, **flat)


def load_params(path: str):
    """(params, gate) from a file written by save_params."""
    z = np.load(path)
    names = sorted({k.rsplit(".", 1)[0] for k in z.files if "." in k})
    gate = float(z["gate"]) if "gate" in z.files else 0.0
    return {k: (z[k + ".w"].astype(np.float64), z[k + ".b"].astype(np.float64)) for k in names}, gate


def main(argv=None):
    import argparse
    import os
    ap = argparse.ArgumentParser(description="batched sweep -> surrogate training -> warm-start evaluation")
    ap.add_argument("--train-domains", type=int, default=1536)
    ap.add_argument("--smin", type=int, default=128)
    ap.add_argument("--smax", type=int, default=512)
    ap.add_argument("--eval-domains", type=int, default=256)
    ap.add_argument("--tol", type=float, default=1e-5)
    ap.add_argument("--check-every", type=int, default=100)
    ap.add_argument("--sweep-cap", type=int, default=60000)
    ap.add_argument("--eval-cap", type=int, default=100000)
    ap.add_argument("--epochs", type=int, default=250)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=5e-4)
    ap.add_argument("--train-budget-s", type=float, default=420.0)
    ap.add_argument("--sweep-group", type=int, default=64, help="domains per sweep context (logged per group)")
    ap.add_argument("--launch-mode", type=int, default=2,
                    help="0: one launch per step, fixed tiles; 1: persistent; 2: tiles follow the live work")
    ap.add_argument("--gate", type=float, default=-1.0,
                    help="warm-start gate (rel. L2 to the plain start); < 0: calibrated on validation domains")
    ap.add_argument("--weights", default="", help="load trained weights instead of sweeping and training")
    ap.add_argument("--probe-steps", type=int, default=500,
                    help="learned side: steps of the plain start before the surrogate is consulted (0: none)")
    ap.add_argument("--eps-domains", type=int, default=0,
                    help="held-out domains of the time-to-equilibrium measurement (0: skip)")
    ap.add_argument("--ref-steps", type=int, default=300000,
                    help="steps of the plain start that give the reference state of a domain")
    ap.add_argument("--eps", default="0.1,0.03,0.01,0.003",
                    help="rel. L2 distances to the reference counted as reached (comma-separated)")
    ap.add_argument("--out", default="warmstart_out")
    args = ap.parse_args(argv)
    os.makedirs(args.out, exist_ok=True)
    logf = open(os.path.join(args.out, "log.jsonl"), "a")

    def log(msg):
        print(msg, flush=True)
        logf.write(msg + "\n")
        logf.flush()

    result = {"config": vars(args)}
    if args.weights:
        params, gate = load_params(args.weights)
        net = S.UNet(params=params)
        if args.gate >= 0:
            gate = args.gate
    else:
        specs = G.batched_sweep(n_domains=args.train_domains, smin=args.smin, smax=args.smax)
        log(json.dumps({"phase": "sweep", "domains": len(specs), "nodes": sum(s.nx * s.ny for s in specs)}))
        sw = sweep(specs, args.tol, args.check_every, args.sweep_cap, launch_mode=args.launch_mode,
                   group=args.sweep_group, log=log)
        conv = int(np.sum(np.array(sw["steps"]) < args.sweep_cap))
        result["sweep"] = {"wall_s": sw["wall_s"], "mlups": sw["mlups"], "nodes": sw["nodes"],
                           "converged": conv, "nan": int(np.sum(sw["status"] == TPF_ENAN)),
                           "steps_mean": float(np.mean(sw["steps"]))}
        log(json.dumps({"phase": "sweep_done", **result["sweep"]}))
        # the last tenth of the domains is validation (calibrates the gate), not trained on
        n_val = max(1, len(specs) // 10)
        val_specs, val_eq = specs[-n_val:], sw["phi1"][-n_val:]
        data = build_dataset(specs[:-n_val], sw["phi1"][:-n_val], sw["status"][:-n_val])
        del sw
        log(json.dumps({"phase": "train", "samples": int(len(data["theta"]))}))
        net = train(data, epochs=args.epochs, batch=args.batch, lr=args.lr, log=log,
                    time_budget_s=args.train_budget_s)
        result["train"] = {"samples": int(len(data["theta"])), "loss_first": net.history[0],
                           "loss_last": net.history[-1], "epochs": len(net.history),
                           "params": net.n_params(), "gflop_fwd_per_sample": net.flops_per_sample() / 1e9}
        gate = calibrate_gate(net, val_specs, val_eq) if args.gate < 0 else args.gate
        result["train"]["gate"] = gate
        result["train"]["validation_domains"] = n_val
        save_params(net, os.path.join(args.out, "unet_weights.npz"), gate)
        log(json.dumps({"phase": "train_done", **result["train"]}))
    held = G.held_out_set(n_domains=args.eval_domains, s=256)
    log(json.dumps({"phase": "evaluate", "domains": len(held)}))
    result["evaluate"] = evaluate(net, held, args.tol, args.check_every, args.eval_cap,
                                  launch_mode=args.launch_mode, gate=gate, probe_steps=args.probe_steps, log=log)
    if args.eps_domains:
        log(json.dumps({"phase": "equilibrium", "domains": args.eps_domains}))
        eps = [float(e) for e in args.eps.split(",")]
        result["equilibrium"] = equilibrium_eval(net, held[:args.eps_domains], args.ref_steps, eps, 500,
                                                 args.eval_cap, gate=gate, launch_mode=args.launch_mode, log=log)
    with open(os.path.join(args.out, "result.json"), "w") as f:
        json.dump(result, f, indent=1, default=float)
    ev = result["evaluate"]
    log(json.dumps({"phase": "done", "work_speedup": ev["work_speedup"], "wall_speedup": ev["wall_speedup"]}))
    return result


if __name__ == "__main__":
    main()
