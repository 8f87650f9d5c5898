"""Runtime behaviour of the HIP library on an MI355X: batching, retirement,
checkpoints, failure isolation, the autotuner, edge cases and full-size
parity on the benchmark workload."""
import ctypes
import math
import os
import sys
import tempfile
import time

import numpy as np
import pytest

from paper_2311_05091_amd import geometry as G
from paper_2311_05091_amd import lbm
from _util import gpu_context, oracle_run, rel_l2

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _mixed_batch():
    return [
        G.solid_disk_box(n=67, ny=23, Rs=5.0, R0=6.0, periodic_y=0),
        G.solid_disk_box(n=40, ny=52, Rs=6.0, R0=7.0, periodic_y=1, rho=(1.0, 1.0, 0.1),
                         mu=(0.15, 0.15, 0.015)),
        G.flat_wall_droplet(nx=128, ny=48, wall_rows=6, R0=14, theta_deg=120.0),
    ]


@pytest.mark.parametrize("prec", [32, 64])
def test_batched_equals_single(prec):
    """Domains advanced together in one launch per step match each domain run
    alone, bit for bit (mixed sizes, walls/periodic, with and without S)."""
    specs = _mixed_batch()
    _say("batched", prec)
    ctx = gpu_context(specs, precision=prec)
    ctx.step(120)
    for i, sp in enumerate(specs):
        one = gpu_context([sp], precision=prec)
        one.step(120)
        a, b = ctx.populations(i), one.populations(0)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), i
        one.close()
    ctx.close()


def test_restart_bitwise():
    """N steps, checkpoint, restore into a fresh context, N more == 2N steps."""
    specs = _mixed_batch()[:2]
    _say("restart")
    ref = gpu_context(specs, precision=32)
    ref.step(200)
    a = gpu_context(specs, precision=32)
    a.step(100)
    with tempfile.TemporaryDirectory() as td:
        path = os.path.join(td, "ck.bin")
        a.save(path)
        a.close()
        b = gpu_context(specs, precision=32)
        b.load(path)
        b.step(100)
    for i in range(len(specs)):
        x, y = ref.populations(i), b.populations(i)
        assert np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1])
        assert b.diag(i)["steps"] == 200
    ref.close()
    b.close()


def test_load_rejects_other_parameters_and_truncated_files():
    """A checkpoint of domains with another contact angle, or a truncated one,
    is refused (TPF_EINVAL, TPF_EIO) and leaves the context's state as it was."""
    from paper_2311_05091_amd.lbm import TpfError, TPF_EINVAL, TPF_EIO
    specs = _mixed_batch()[:2]
    _say("load rejection")
    a = gpu_context(specs, precision=32)
    a.step(50)
    other = [G.with_params(specs[0], theta_deg=specs[0].theta_deg + 1.0), specs[1]]
    b = gpu_context(other, precision=32)
    b.step(20)
    before = [b.populations(i) for i in range(2)]
    with tempfile.TemporaryDirectory() as td:
        path = os.path.join(td, "ck.bin")
        a.save(path)
        with pytest.raises(TpfError) as e:
            b.load(path)
        assert e.value.status == TPF_EINVAL
        c = gpu_context(specs, precision=32)
        c.step(20)
        before_c = [c.populations(i) for i in range(2)]
        data = open(path, "rb").read()
        short = os.path.join(td, "short.bin")
        open(short, "wb").write(data[:len(data) - 100])
        with pytest.raises(TpfError) as e:
            c.load(short)
        assert e.value.status == TPF_EIO
        for i in range(2):
            x, y = c.populations(i), before_c[i]
            assert np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1])
        c.load(path)
        assert c.diag(0)["steps"] == 50
        c.close()
    for i in range(2):
        x, y = b.populations(i), before[i]
        assert np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1])
    a.close()
    b.close()


def test_deterministic_replay():
    """Two identical runs give identical bits (no races in the LDS staging)."""
    sp = G.solid_disk_box(n=200, ny=120, Rs=20, R0=25, periodic_y=0, rho=(1.0, 1.0, 0.1),
                          mu=(0.15, 0.15, 0.015))
    _say("replay")
    out = []
    for _ in range(2):
        c = gpu_context([sp], precision=32)
        c.step(300)
        out.append(c.populations(0))
        c.close()
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


def test_nan_domain_is_isolated():
    """A domain poisoned with NaN is retired with TPF_ENAN; the others keep
    running and still match their single-domain runs."""
    specs = _mixed_batch()[:2]
    bad = G.with_params(specs[0], phi1=specs[0].phi1.copy())
    bad.phi1[5, 7] = np.nan
    _say("nan isolation")
    ctx = gpu_context([bad, specs[1]], precision=32)
    rc, steps = ctx.run_to_residual(1e-30, check_every=50, max_steps=200)
    assert rc == lbm.TPF_ENAN
    assert ctx.diag(0)["status"] == lbm.TPF_ENAN
    assert ctx.diag(1)["status"] == lbm.TPF_OK
    assert steps[1] == 200 and steps[0] < 200
    one = gpu_context([specs[1]], precision=32)
    one.step(200)
    assert np.array_equal(ctx.populations(1)[0], one.populations(0)[0])
    ctx.close()
    one.close()


def test_run_to_residual_retires_domains():
    specs = [G.flat_wall_droplet(nx=64, ny=32, wall_rows=5, R0=10, theta_deg=t) for t in (60.0, 90.0)]
    _say("run to residual")
    ctx = gpu_context(specs, precision=32)
    rc, steps = ctx.run_to_residual(1e-6, check_every=100, max_steps=200000)
    assert rc == lbm.TPF_OK
    for i in range(2):
        d = ctx.diag(i)
        assert d["residual"] < 1e-6 and steps[i] % 100 == 0 and steps[i] >= 200
    # budget exhaustion is reported
    rc2, steps2 = ctx.run_to_residual(1e-30, check_every=100, max_steps=300)
    assert rc2 == lbm.TPF_EBUDGET and (steps2 == 300).all()
    ctx.close()


def test_residual_definition():
    """r = ||phi^n - phi^(n-K)|| / (K ||phi^n||) from the device reductions equals
    the same quantity computed from read-back fields."""
    sp = G.flat_wall_droplet(nx=96, ny=40, wall_rows=6, R0=14)
    _say("residual definition")
    ctx = gpu_context([sp], precision=64)
    ctx.step(100)
    ctx.run_to_residual(0.0, check_every=1, max_steps=0)  # snapshot only
    a = ctx.moments(0)[0]
    ctx.run_to_residual(0.0, check_every=37, max_steps=37)
    b = ctx.moments(0)[0]
    r = ctx.diag(0)["residual"]
    expect = np.linalg.norm(b - a) / (37 * np.linalg.norm(b))
    assert abs(r / expect - 1) < 1e-10
    assert abs(ctx.diag(0)["mass"] - b.sum()) < 1e-12 * b.sum()
    ctx.close()


def test_autotune_restores_state_and_picks_known_tile():
    sp = G.solid_disk_box(n=300, ny=200, Rs=20, R0=25, periodic_y=0)
    _say("autotune")
    ctx = gpu_context([sp], precision=32)
    ctx.step(10)
    before = ctx.populations(0)
    ctx.autotune(steps=5)
    code, tx, ty = ctx.tile()
    assert code in [c for c, _, _ in lbm.tile_codes()]
    after = ctx.populations(0)
    assert np.array_equal(before[0], after[0]) and np.array_equal(before[1], after[1])
    assert ctx.diag(0)["steps"] == 10
    ctx.close()


def test_class_autotune_cache_is_reused_and_state_restored(tmp_path):
    """Per-size-class autotuning: three classes (128^2 without S, 300 x 200
    without S, 128^2 with S) are timed, each domain gets its class's code, the
    state is restored, and the JSON cache written for this device makes a
    second context take the same codes without timing and step to the same
    bits.  A cache of another device is ignored and replaced."""
    ratio10 = dict(rho=(1.0, 1.0, 0.1), mu=(0.15, 0.15, 0.015))
    specs = [G.solid_disk_box(n=128, Rs=12, R0=15), G.solid_disk_box(n=128, Rs=10, R0=17),
             G.solid_disk_box(n=300, ny=200, Rs=20, R0=25, periodic_y=0),
             G.solid_disk_box(n=300, ny=200, Rs=24, R0=20, periodic_y=0),
             G.solid_disk_box(n=128, Rs=12, R0=15, **ratio10)]
    cache = str(tmp_path / "tiles.json")
    with open(cache, "w") as f:
        f.write('{\n  "format": "tpf-autotune-1",\n  "device": "other:1",\n  "entries": {\n'
                '    "p32_s0_w128_h128": {"code": 1, "ms_per_step": 0.001}\n  }\n}\n')
    _say("class autotune")
    runs = []
    for attempt in range(2):
        ctx = gpu_context(specs, precision=32)
        ctx.step(10)
        before = [ctx.populations(i) for i in range(len(specs))]
        n_timed = ctx.autotune_classes(steps=3, cache_path=cache)
        assert n_timed == (3 if attempt == 0 else 0)
        for i in range(len(specs)):
            f, g = ctx.populations(i)
            assert np.array_equal(f, before[i][0]) and np.array_equal(g, before[i][1]), (attempt, i)
            assert ctx.diag(i)["steps"] == 10
        codes = [ctx.domain_tile(i) for i in range(len(specs))]
        assert codes[0] == codes[1] and codes[2] == codes[3]
        ctx.step(20)
        runs.append((codes, [ctx.populations(i) for i in range(len(specs))]))
        ctx.close()
    text = open(cache).read()
    assert '"device": "other:1"' not in text and text.count('"code"') == 3
    for key in ("p32_s0_w128_h128", "p32_s0_w512_h256", "p32_s1_w128_h128"):
        assert key in text
    assert runs[0][0] == runs[1][0]
    for a, b in zip(runs[0][1], runs[1][1]):
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    # mixed codes in one step agree with one code for all to FP32 rounding
    one = gpu_context(specs, precision=32, tile=9)
    one.step(30)
    for i, (f, g) in enumerate(runs[0][1]):
        f1, g1 = one.populations(i)
        assert np.abs(f - f1).max() <= 2e-6 * np.abs(f1).max(), i
        assert np.abs(g - g1).max() <= 2e-6 * max(np.abs(g1).max(), 1e-3), i
    one.close()


def test_step_reads_no_memory_initialisation_left_unwritten():
    """The same batch (walls, periodic, the S flux, ragged sizes, a moving
    solid) in arenas filled with zeros and with NaN bytes before
    tpf_finalize, stepped in every launch mode: bitwise equal states, so no
    kernel reads arena memory that initialisation did not write."""
    from paper_2311_05091_amd.lbm import Context
    ratio10 = dict(rho=(1.0, 1.0, 0.1), mu=(0.15, 0.15, 0.015))
    specs = [G.solid_disk_box(n=67, ny=23, Rs=5.0, R0=6.0, periodic_y=0),
             G.solid_disk_box(n=131, ny=37, Rs=7.0, R0=9.0, periodic_y=0, **ratio10),
             G.with_params(G.solid_disk_box(n=40, ny=33, **ratio10), u_wall=(1e-3, 0.0), omega_wall=1e-4,
                           wall_center=(12.0, 13.2))]
    _say("arena fill")
    for mode in (0, 1, 2):
        out = []
        for fill in (0x00, 0xFF):
            ctx = Context(precision=32)
            for sp in specs:
                ctx.add_domain(sp)
            ctx.finalize(fill=fill)
            ctx.set_launch_mode(mode)
            ctx.step(60)
            ctx.run_to_residual(1e-30, check_every=20, max_steps=40)
            out.append([ctx.populations(i) for i in range(len(specs))])
            ctx.close()
        for i, (a, b) in enumerate(zip(*out)):
            assert np.isfinite(a[0]).all() and np.isfinite(a[1]).all(), (mode, i)
            assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), (mode, i)


EDGE = [
    ("min_3x3_periodic", lambda: G.DomainSpec(nx=3, ny=3, phi0=np.zeros((3, 3)),
                                              phi1=np.array([[0.1, 0.5, 0.9]] * 3), periodic_y=1)),
    ("min_3x3_walls", lambda: G.DomainSpec(nx=3, ny=3, phi0=np.full((3, 3), 0.2),
                                           phi1=np.array([[0.1, 0.5, 0.7]] * 3), periodic_x=0,
                                           periodic_y=0)),
    ("closed_box_walls_xy", lambda: G.with_params(G.solid_disk_box(n=30, ny=22, periodic_y=0), periodic_x=0)),
    ("theta90_kappa", lambda: G.with_params(G.solid_disk_box(n=33, ny=29, periodic_y=0), theta_deg=90.0,
                                            kappa=0.8)),
    ("textbook_d0", lambda: G.with_params(G.solid_disk_box(n=33, ny=29), d0=1.0 / 3.0)),
    ("all_solid_row", lambda: G.with_params(G.flat_wall_droplet(nx=40, ny=30, wall_rows=10, R0=8, D=2.0),
                                            mu=(0.2, 0.15, 0.05), M_cst=0.002)),
]


@pytest.mark.parametrize("name,factory", EDGE, ids=[e[0] for e in EDGE])
def test_edge_cases_fp64(orc, name, factory):
    sp = factory()
    _say("edge", name)
    ctx = gpu_context([sp], precision=64)
    ctx.step(60)
    sim = oracle_run(orc, sp, 60)
    for a, b in zip(ctx.moments(0), sim.moments()):
        # relative to the field maximum, with an absolute floor for fields that
        # are rounding noise (the 3x3 cases have |u| ~ 1e-12)
        assert np.abs(a - b).max() <= 1e-11 * np.abs(b).max() + 1e-15
    ctx.close()


def test_invalid_parameters_rejected():
    from paper_2311_05091_amd.lbm import Context, TpfError
    ctx = Context(precision=32)
    base = G.solid_disk_box(n=8)
    for change in ({"theta_deg": 0.0}, {"theta_deg": 180.0}, {"tau_phi": 0.5}, {"d0": 1.0},
                   {"rho": (1.0, 0.0, 1.0)}, {"M_deg": 0.0, "M_cst": 0.0}):
        with pytest.raises(TpfError) as e:
            ctx.add_domain(G.with_params(base, **change))
        assert e.value.status == lbm.TPF_EINVAL
    with pytest.raises(TpfError) as e:
        ctx.add_domain(G.DomainSpec(nx=2, ny=8, phi0=np.zeros((8, 2)), phi1=np.zeros((8, 2))))
    assert e.value.status == lbm.TPF_EINVAL
    # more nodes than the 32-bit index space of one domain: rejected before any copy
    p = lbm.params_from_spec(base)
    p.nx, p.ny = 20000, 20000
    dummy = np.zeros(4)
    did = ctypes.c_int32()
    rc = ctx.lib.tpf_add_domain(ctx._h, ctypes.byref(p), dummy.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                dummy.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(did))
    assert rc == lbm.TPF_EINVAL
    # no domains: finalize is refused, as is stepping before finalize
    assert ctx.lib.tpf_finalize(ctx._h, None, 0) == lbm.TPF_ESTATE
    assert ctx.lib.tpf_step(ctx._h, 1) == lbm.TPF_ESTATE
    ctx.close()


@pytest.mark.parametrize("nontemporal", [False, True])
def test_copy_bandwidth_copies_and_times(nontemporal):
    """The roofline's reference copy moves the data unchanged (checked inside
    copy_bandwidth) at a plausible HBM rate."""
    from paper_2311_05091_amd.lbm import copy_bandwidth
    _say("copy", nontemporal)
    bw = copy_bandwidth(64 << 20, nontemporal=nontemporal, reps=5)
    assert 1e11 < bw < 2e13, bw


def test_inactive_domain_is_left_out_and_resumes():
    """An inactive domain keeps its state through steps and runs to a
    residual (0 steps counted); the others advance as they would alone; once
    active again it continues as if it had not been paused."""
    a = G.solid_disk_box(n=40, ny=24, periodic_y=0)
    b = G.solid_disk_box(n=67, ny=23, Rs=5.0, R0=6.0, periodic_y=0)
    _say("set_active")
    ctx = gpu_context([a, b], precision=64)
    ref = gpu_context([b], precision=64)
    ctx.set_active(0, False)
    fa0 = ctx.populations(0)
    ctx.step(30)
    ref.step(30)
    assert np.array_equal(ctx.populations(0)[0], fa0[0]) and np.array_equal(ctx.populations(0)[1], fa0[1])
    assert np.array_equal(ctx.populations(1)[0], ref.populations(0)[0])
    rc, steps = ctx.run_to_residual(1e-30, check_every=10, max_steps=20)
    assert steps[0] == 0 and steps[1] == 20
    ctx.set_active(0, True)
    ctx.step(15)
    alone = gpu_context([a], precision=64)
    alone.step(15)
    assert np.array_equal(ctx.populations(0)[0], alone.populations(0)[0])
    with pytest.raises(lbm.TpfError):
        ctx.set_active(5, True)
    for c in (ctx, ref, alone):
        c.close()


def test_zero_steps_is_noop():
    sp = G.solid_disk_box(n=20)
    ctx = gpu_context([sp], precision=64)
    a = ctx.populations(0)
    ctx.step(0)
    b = ctx.populations(0)
    assert np.array_equal(a[0], b[0]) and ctx.diag(0)["steps"] == 0
    ctx.close()


@pytest.mark.parametrize("prec,tile", [(64, 24), (32, 23), (32, 0)])
def test_full_size_porous_workload(orc, prec, tile):
    """The benchmark workload (4096 x 2048 porous medium) at full size, in the
    tile shapes the benchmark's autotuner takes on it (FP32 23, FP64 24: groups
    of four 64 x 64 strips with non-temporal loads) and in whatever a short
    autotune picks (tile 0): 3 steps against the oracle at every node.
    FP64: <= 1e-11 of the field maximum.  FP32: phi within 2e-6 absolute
    (a few FP32 ulps of O(1) populations per step); u and p within 1e-3 of
    their maxima (they come from O(1e-6) differences of FP32 values)."""
    sp = G.porous_medium()
    _say("full size porous", prec, tile)
    ctx = gpu_context([sp], precision=prec)
    if tile:
        ctx.set_tile(tile)
    else:
        ctx.autotune(steps=3)
    ctx.step(3)
    g = ctx.moments(0)
    ctx.close()
    sim = oracle_run(orc, sp, 3)
    o = sim.moments()
    del sim
    if prec == 64:
        for a, b in zip(g, o):
            assert np.abs(a - b).max() <= 1e-11 * np.abs(b).max()
    else:
        assert np.abs(g[0] - o[0]).max() <= 2e-6
        for a, b in zip(g[1:], o[1:]):
            assert np.abs(a - b).max() <= 1e-3 * np.abs(b).max()


@pytest.mark.parametrize("prec,tile", [(64, 9), (32, 8), (32, 10)])
def test_persistent_launch_matches_per_step_launch(prec, tile):
    """One persistent launch per chunk (work queue over (step, tile) with
    per-domain step barriers) gives the same state as one launch per step:
    to rounding, since the persistent and the per-step strip kernels are
    separate compilations of the node update whose multiply-add contraction
    may differ (FP32: within 1e-5 of the largest population after 77 steps,
    measured 2.5e-6 for the NS offsets; FP64: 1e-13)."""
    specs = _mixed_batch() + [G.flat_wall_droplet(nx=200, ny=90, wall_rows=6, R0=20)]
    _say("persistent", prec, tile)
    a = gpu_context(specs, precision=prec, tile=tile)
    a.step(77)
    b = gpu_context(specs, precision=prec, tile=tile)
    assert b.lib.tpf_set_launch_mode(b._h, 1) == 0  # noqa: via the raw ABI
    b.step(77)
    tol = 1e-13 if prec == 64 else 1e-5
    for i in range(len(specs)):
        fa, ga = a.populations(i)
        fb, gb = b.populations(i)
        assert b.diag(i)["steps"] == 77
        assert np.abs(fa - fb).max() <= tol * np.abs(fa).max()
        assert np.abs(ga - gb).max() <= tol * max(np.abs(ga).max(), 1e-12)
    # residual-driven runs work in this mode too
    rc, steps = b.run_to_residual(1e-30, check_every=50, max_steps=100)
    assert rc == lbm.TPF_EBUDGET and (steps == 100).all()
    a.close()
    b.close()


def _converging_batch():
    return [
        G.flat_wall_droplet(nx=64, ny=32, wall_rows=5, R0=10, theta_deg=60.0),
        G.flat_wall_droplet(nx=96, ny=40, wall_rows=6, R0=12, theta_deg=90.0),
        G.flat_wall_droplet(nx=150, ny=45, wall_rows=5, R0=12, theta_deg=120.0),
    ]


@pytest.mark.parametrize("prec,tile", [(64, 9), (64, 21), (64, 23), (32, 9), (32, 21), (32, 23)])
def test_persistent_run_to_residual_retires_inside_the_launch(prec, tile):
    """Launch mode 1 runs the residual checks of run_to_residual inside the
    persistent launch (one check item per live domain and step, active at
    every check_every-th step of the call and at its last step); a domain
    whose residual falls below tol leaves the work queue there while the
    others go on.  Against one launch per step with checks on the host: the
    same retirement steps (FP64; FP32 within one check interval, since the
    two kernels round differently), the same residual (FP64 to 1e-8
    relative), the same state (FP64 1e-13; FP32 1e-5 of the largest
    population where the steps agree), and the budget case ends at
    max_steps with the final check taken at that step."""
    specs = _converging_batch()
    _say("persistent residual", prec, tile)
    tol, every = 1e-5, 100
    a = gpu_context(specs, precision=prec, tile=tile)
    t0 = time.perf_counter()
    rc_a, st_a = a.run_to_residual(tol, check_every=every, max_steps=100000)
    t1 = time.perf_counter()
    b = gpu_context(specs, precision=prec, tile=tile)
    b.set_launch_mode(1)
    rc_b, st_b = b.run_to_residual(tol, check_every=every, max_steps=100000)
    t2 = time.perf_counter()
    print("steps per domain %s (per-step launches, %.2f s) %s (persistent, %.2f s)"
          % (st_a.tolist(), t1 - t0, st_b.tolist(), t2 - t1), flush=True)
    assert rc_a == lbm.TPF_OK and rc_b == lbm.TPF_OK
    assert len(set(st_a.tolist())) > 1, st_a      # the domains leave at different steps
    if prec == 64:
        assert (st_a == st_b).all(), (st_a, st_b)
    else:
        assert np.abs(st_a - st_b).max() <= every, (st_a, st_b)
    ptol = 1e-13 if prec == 64 else 1e-5
    for i in range(len(specs)):
        da, db = a.diag(i), b.diag(i)
        assert db["status"] == lbm.TPF_OK and db["steps"] == st_b[i] and st_b[i] % every == 0
        assert db["residual"] < tol and da["residual"] < tol
        if st_a[i] == st_b[i]:
            if prec == 64:
                assert abs(db["residual"] / da["residual"] - 1) < 1e-8, (da, db)
                assert abs(db["mass"] / da["mass"] - 1) < 1e-13
            fa, ga = a.populations(i)
            fb, gb = b.populations(i)
            assert np.abs(fa - fb).max() <= ptol * np.abs(fa).max()
            assert np.abs(ga - gb).max() <= ptol * max(np.abs(ga).max(), 1e-12)
    # budget: no domain converges; the last check falls on max_steps = 130
    # (not a multiple of check_every), and later calls step every domain again
    for c in (a, b):
        rc, st = c.run_to_residual(1e-30, check_every=50, max_steps=130)
        assert rc == lbm.TPF_EBUDGET and (st == 130).all()
    for i in range(len(specs)):
        da, db = a.diag(i), b.diag(i)
        assert da["steps"] == st_a[i] + 130 and db["steps"] == st_b[i] + 130
        if st_a[i] == st_b[i] and prec == 64:
            assert abs(db["residual"] / da["residual"] - 1) < 1e-8, (i, da, db)
    a.close()
    b.close()


def test_persistent_run_to_residual_isolates_a_nan_domain():
    """In launch mode 1 a domain that turns non-finite leaves at its first
    check with TPF_ENAN while the others run to max_steps, as in mode 0."""
    specs = _mixed_batch()[:2]
    bad = G.with_params(specs[0], phi1=specs[0].phi1.copy())
    bad.phi1[5, 7] = 2.0e3     # finite at entry, non-finite within a few steps
    _say("persistent nan isolation")
    out = []
    for mode in (0, 1):
        ctx = gpu_context([bad, specs[1]], precision=32, tile=9)
        ctx.set_launch_mode(mode)
        rc, steps = ctx.run_to_residual(1e-30, check_every=50, max_steps=200)
        out.append((rc, steps.tolist(), ctx.diag(0)["status"], ctx.diag(1)["status"]))
        ctx.close()
    assert out[0] == out[1], out
    rc, steps, s0, s1 = out[1]
    assert rc == lbm.TPF_ENAN and s0 == lbm.TPF_ENAN and s1 == lbm.TPF_OK
    assert steps[1] == 200 and steps[0] < 200


@pytest.mark.parametrize("prec", [64, 32])
def test_adaptive_tile_mode_matches_fixed_tiles(prec):
    """Launch mode 2 re-chooses the tile shape from the live work at every
    call: same state as fixed tiles up to the rounding differences between
    the kernels (FP64 1e-13, FP32 1e-5 of the largest population), and
    residual-driven runs retire domains as in mode 0."""
    specs = _mixed_batch()
    _say("adaptive", prec)
    a = gpu_context(specs, precision=prec, tile=9)
    a.step(60)
    b = gpu_context(specs, precision=prec)
    b.set_launch_mode(2)
    b.step(60)
    code, _, _ = b.tile()
    assert code in (17, 9, 8, 2, 1)
    tol = 1e-13 if prec == 64 else 1e-5
    for i in range(len(specs)):
        fa, ga = a.populations(i)
        fb, gb = b.populations(i)
        assert np.abs(fa - fb).max() <= tol * np.abs(fa).max()
        assert np.abs(ga - gb).max() <= tol * max(np.abs(ga).max(), 1e-12)
    rc, steps = b.run_to_residual(1e-30, check_every=20, max_steps=40)
    assert rc == lbm.TPF_EBUDGET and (steps == 40).all()
    a.close()
    b.close()
