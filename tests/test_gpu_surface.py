"""Compensated surface (eta stored as an FP32 pair) on the GPU: parity with
the FP64 oracle at the bar on closed, open-channel, masked and
implicit-link-depth cases; exact state round trip; still water; execution
variants and batches bit for bit.
"""
import sys

import numpy as np
import pytest

from helpers import compare, oracle_from_spec
from paper_1902_02999_amd import workloads as wl

pytestmark = pytest.mark.gpu

H_TOL, U_TOL = 1e-5, 1e-4


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_1902_02999_amd import mlb
    c = mlb.Context(0)
    yield c
    c.close()


def bumpy(nx, ny, seed, amp=0.3):
    rng = np.random.default_rng(seed)
    X, Y = np.meshgrid(np.arange(nx), np.arange(ny))
    zb = np.zeros((ny, nx))
    for _ in range(3):
        cx, cy = rng.uniform(0, nx), rng.uniform(0, ny)
        s = rng.uniform(nx / 12, nx / 4)
        zb += amp * rng.uniform(0.3, 1) * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2 * s * s))
    return zb


def comp(spec):
    spec.compensated = True
    return spec


def run_gpu(ctx, spec, nsteps, state=None, opts=None):
    from paper_1902_02999_amd import mlb
    g = mlb.grid_from_spec(ctx, spec)
    if state is not None:
        g.set_state(*state)
    if opts:
        g.set_exec_opts(**opts)
    g.step(nsteps)
    out = g.get_state()
    g.close()
    return out


def closed(nx, ny, seed, **kw):
    return comp(wl.Spec("closed_%dx%d" % (nx, ny), nx, ny, 1.0, 10.0 / 6.0, bumpy(nx, ny, seed), 2.0,
                        wind_speed=(9.0, -4.0), chezy=45.0, **kw))


def check(ctx, spec, nsteps, state=None):
    state = spec.initial() if state is None else state
    say("case", spec.name, spec.nx, spec.ny, "steps", nsteps)
    got = run_gpu(ctx, spec, nsteps, state)
    ref = oracle_from_spec(spec, *state)
    ref.run(nsteps)
    where = None if spec.kind is None else spec.kind != wl.SOLID
    dh, du = compare(*got, ref.h, ref.qx, ref.qy, where=where)
    say("dh", dh, "du", du)
    assert dh <= H_TOL and du <= U_TOL


@pytest.mark.parametrize("case", ["closed", "periodic", "channel1", "channel2", "masked", "implicit", "tidal"])
def test_compensated_parity(ctx, case):
    if case == "closed":
        spec = closed(125, 70, 1, omega=1e-3)
    elif case == "periodic":
        spec = closed(70, 40, 5, edges=(wl.PERIODIC,) * 4)
    elif case.startswith("channel"):
        spec = comp(wl.bump_channel(150, 67, sigma=12.0))
        spec.extrap_order = int(case[-1])
    elif case == "masked":
        spec = closed(130, 67, 4, kind=wl.random_geometry(np.random.Generator(np.random.PCG64(4)), 130, 67))
    elif case == "implicit":
        spec = closed(90, 61, 6)
        spec.hbar_implicit = True
    else:
        spec = comp(wl.tidal_strip())
        check(ctx, spec, 10800)
        return
    state = None if case.startswith("channel") else wl.seeded_state(spec, 3, eta_amp=0.05, q_amp=0.1)
    check(ctx, spec, 300 if not case.startswith("channel") else 600, state)


def test_state_round_trip_is_exact(ctx):
    from paper_1902_02999_amd import mlb
    spec = closed(70, 45, 2)
    rng = np.random.default_rng(3)
    h = spec.H + 3.0 + 1e-3 * rng.standard_normal(spec.H.shape)   # eta ~ 3 m, detail at 1e-3
    g = mlb.grid_from_spec(ctx, spec)
    g.set_state(h, np.zeros_like(h), np.zeros_like(h))
    h2, _, _ = g.get_state()
    g.set_surface(False)          # plain FP32: eta rounded
    g.set_state(h, np.zeros_like(h), np.zeros_like(h))
    h3, _, _ = g.get_state()
    g.close()
    e2 = np.abs(h2 - h).max()
    e3 = np.abs(h3 - h).max()
    say("round trip error: compensated", e2, "FP32", e3)
    assert e2 <= 1e-12 and e3 >= 1e-8


def test_compensated_still_water_bitwise(ctx):
    spec = comp(wl.Spec("rest", 130, 77, 1.0, 10.0 / 6.0, bumpy(130, 77, 1, amp=0.8), 2.0))
    h, qx, qy = run_gpu(ctx, spec, 500)
    assert np.all(qx == 0.0) and np.all(qy == 0.0)
    assert np.array_equal(h, run_gpu(ctx, spec, 0)[0])


def test_compensated_variants_and_batch_bitwise(ctx):
    from paper_1902_02999_amd import mlb
    spec = closed(150, 80, 7)
    state = wl.seeded_state(spec, 7, q_amp=0.1)
    base = run_gpu(ctx, spec, 101, state, dict(tile_rows=15, tblock=1, use_graph=0))
    for o in (dict(tile_rows=4), dict(tile_rows=9, use_graph=1, graph_chunk=8), dict(tile_rows=15, tblock=2),
              dict(tile_rows=12, persistent=1)):
        say("variant", o)
        got = run_gpu(ctx, spec, 101, state, o)
        for u, v in zip(base, got):
            assert np.array_equal(u, v)
    specs = [closed(90, 70, 2), closed(64, 130, 3)]
    states = [wl.seeded_state(s, i) for i, s in enumerate(specs)]
    singles = [run_gpu(ctx, s, 61, st) for s, st in zip(specs, states)]
    gs = [mlb.grid_from_spec(ctx, s) for s in specs]
    for g, st in zip(gs, states):
        g.set_state(*st)
    b = mlb.Batch(ctx, gs)
    with pytest.raises(mlb.MlbError):
        gs[0].set_surface(False)      # grid inside a live batch
    b.step(61)
    b.close()
    for g, want in zip(gs, singles):
        for u, v in zip(g.get_state(), want):
            assert np.array_equal(u, v)
    gs[1].set_surface(False)
    with pytest.raises(mlb.MlbError):
        mlb.Batch(ctx, gs)            # the surface modes differ
    for g in gs:
        g.close()
