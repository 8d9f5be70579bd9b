"""Implicit link depth on the GPU (the static per-node sums, one or two steps
per pass) against the oracle's exact solve, and its invariants.

Bar as for the other parity tests: max |dh| <= 1e-5 max h, max |du| <= 1e-4
max |u|.  Over a flat bed the implicit form is Eq. h-bar's map bit for bit
(1/(1+0) = 1 and a zero correction); execution variants are bit for bit.
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


def bumpy(nx, ny, seed, amp=0.4):
    rng = np.random.default_rng(seed)
    X, Y = np.meshgrid(np.arange(nx), np.arange(ny))
    zb = np.zeros((ny, nx))
    for _ in range(3):
        cx, cy = rng.uniform(0, nx), rng.uniform(0, ny)
        s = rng.uniform(nx / 12, nx / 4)
        zb += amp * rng.uniform(0.3, 1) * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2 * s * s))
    return zb


def implicit(spec):
    spec.hbar_implicit = True
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
    return got, ref


def closed(nx, ny, seed, **kw):
    return implicit(wl.Spec("closed_%dx%d" % (nx, ny), nx, ny, 1.0, 10.0 / 6.0, bumpy(nx, ny, seed), 2.0,
                            wind_speed=(9.0, -4.0), chezy=45.0, **kw))


@pytest.mark.parametrize("nx,ny,seed", [(125, 70, 1), (61, 9, 2), (4, 133, 3)])
def test_implicit_closed_basin_parity(ctx, nx, ny, seed):
    spec = closed(nx, ny, seed, omega=1e-3)
    check(ctx, spec, 300, wl.seeded_state(spec, seed, eta_amp=0.05, q_amp=0.1))


def test_implicit_periodic_parity(ctx):
    spec = closed(70, 40, 5, edges=(wl.PERIODIC,) * 4)
    check(ctx, spec, 300, wl.seeded_state(spec, 5, q_amp=0.2))


@pytest.mark.parametrize("order", [1, 2])
def test_implicit_open_channel_parity(ctx, order):
    spec = implicit(wl.bump_channel(150, 67, sigma=12.0, bump=0.4))
    spec.extrap_order = order
    check(ctx, spec, 500)


def test_implicit_masked_parity(ctx):
    kind = wl.random_geometry(np.random.Generator(np.random.PCG64(4)), 130, 67, holes=4)
    spec = closed(130, 67, 4, kind=kind)
    check(ctx, spec, 300, wl.seeded_state(spec, 4, q_amp=0.1))


def test_implicit_tidal_strip_parity(ctx):
    spec = implicit(wl.tidal_strip())
    check(ctx, spec, 1500)


def test_implicit_hump_parity_at_paper_size(ctx):
    check(ctx, implicit(wl.hump_channel()), 300)


def test_flat_bed_forms_agree_bitwise(ctx):
    a = wl.Spec("flat", 97, 66, 1.0, 10.0 / 6.0, np.zeros((66, 97)), 2.0, wind_speed=(6.0, 8.0), chezy=40.0)
    state = wl.seeded_state(a, 2, q_amp=0.2)
    ga = run_gpu(ctx, a, 200, state, dict(tblock=1))
    gb = run_gpu(ctx, implicit(a), 200, state)
    for u, v in zip(ga, gb):
        assert np.array_equal(u, v)


def test_implicit_still_water_bitwise(ctx):
    spec = implicit(wl.Spec("rest", 130, 77, 1.0, 10.0 / 6.0, bumpy(130, 77, 1, amp=0.8), 2.0))
    h, qx, qy = run_gpu(ctx, spec, 500)
    assert np.all(qx == 0.0) and np.all(qy == 0.0)
    assert np.array_equal(h, run_gpu(ctx, spec, 0)[0])


def test_implicit_execution_variants_bitwise(ctx):
    spec = closed(150, 80, 7)
    state = wl.seeded_state(spec, 7, q_amp=0.1)
    base = run_gpu(ctx, spec, 101, state, dict(tile_rows=15, tblock=1, use_graph=0))
    for o in (dict(tile_rows=4), dict(tile_rows=9, use_graph=1, graph_chunk=8), dict(tile_rows=15, tblock=2),
              dict(tile_rows=12, persistent=1), dict(tile_rows=33, blocks_per_cu=2)):
        say("variant", o)
        got = run_gpu(ctx, spec, 101, state, o)
        for u, v in zip(base, got):
            assert np.array_equal(u, v)


def _two_step_cases():
    """(name, spec, state, steps, tile_rows): every edge kind (the open S edge's
    deferred row carries its coefficients through the queue), both
    extrapolation orders, a node mask, narrow and odd strips."""
    cases = []
    for nx, ny, rows in ((125, 70, 15), (5, 4, 4), (61, 9, 6), (59, 31, 30)):
        sp = closed(nx, ny, nx + ny, omega=1e-3)
        cases.append(("closed%dx%d_rows%d" % (nx, ny, rows), sp, wl.seeded_state(sp, 2, q_amp=0.1), 37, rows))
    sp = closed(70, 40, 5, edges=(wl.PERIODIC,) * 4)
    cases.append(("periodic70x40", sp, wl.seeded_state(sp, 5, q_amp=0.2), 101, 9))
    kind = wl.random_geometry(np.random.Generator(np.random.PCG64(4)), 130, 67, holes=4)
    sp = closed(130, 67, 4, kind=kind)
    cases.append(("masked130x67", sp, wl.seeded_state(sp, 4, q_amp=0.1), 61, 14))
    for order in (1, 2):
        sp = implicit(wl.bump_channel(150, 67, sigma=12.0, bump=0.4))
        sp.extrap_order = order
        cases.append(("channel_order%d" % order, sp, None, 120, 15))
        nx, ny = 40, 90
        sp = implicit(wl.Spec("ychannel", nx, ny, 1.0, 25.0 / 6.0, bumpy(nx, ny, 7, amp=0.2), 2.0,
                              edges=(wl.PERIODIC, wl.PERIODIC, wl.DISCHARGE, wl.DEPTH), extrap_order=order,
                              depth_bc={wl.N: (2.0, 0.05, 30.0, 0.0)}, discharge_bc={wl.S: (0.1, 1.5)},
                              qy0=np.full((ny, nx), 1.5)))
        cases.append(("ychannel_order%d" % order, sp, None, 99, 12))
    sp = implicit(wl.Spec("ydepth", 70, 46, 1.0, 25.0 / 6.0, bumpy(70, 46, 9, amp=0.2), 2.0,
                          edges=(wl.WALL, wl.WALL, wl.DEPTH, wl.DISCHARGE), extrap_order=2,
                          depth_bc={wl.S: (2.0, 0.03, 20.0, 0.5)}, discharge_bc={wl.N: (0.0, 0.5)}))
    cases.append(("ydepth_walls", sp, None, 66, 15))
    cases.append(("hump", implicit(wl.hump_channel()), None, 51, 17))
    return cases


_TB2 = _two_step_cases()


@pytest.mark.parametrize("case", _TB2, ids=[c[0] for c in _TB2])
def test_implicit_two_step_passes_bitwise(ctx, case):
    """Two steps per pass give the bits of one step per pass (whose parity
    with the oracle the tests above check)."""
    name, spec, state, steps, rows = case
    say("implicit two-step case", name, spec.nx, spec.ny, "steps", steps, "rows", rows)
    one = run_gpu(ctx, spec, steps, state, {"tile_rows": rows, "tblock": 1})
    for opts in ({"tile_rows": rows, "tblock": 2}, {"tile_rows": rows, "tblock": 2, "use_graph": True, "graph_chunk": 8}):
        two = run_gpu(ctx, spec, steps, state, opts)
        for a, b in zip(two, one):
            assert np.array_equal(a, b), (name, opts)


def test_implicit_batch_and_errors(ctx):
    from paper_1902_02999_amd import mlb
    specs = [closed(90, 70, 2), closed(64, 130, 3)]
    states = [wl.seeded_state(s, i) for i, s in enumerate(specs)]
    singles = [run_gpu(ctx, s, 61, st) for s, st in zip(specs, states)]
    gs = [mlb.grid_from_spec(ctx, s) for s in specs]
    for g, st in zip(gs, states):
        g.set_state(*st)
    b = mlb.Batch(ctx, gs)
    with pytest.raises(mlb.MlbError):
        gs[0].set_hbar(False)        # grid inside a live batch
    b.set_exec_opts(tile_rows=12, tblock=2)
    b.step(61)
    b.close()
    for g, want in zip(gs, singles):
        for u, v in zip(g.get_state(), want):
            assert np.array_equal(u, v)
    gs[1].set_hbar(False)
    with pytest.raises(mlb.MlbError):
        mlb.Batch(ctx, gs)           # the forms differ
    for g in gs:
        g.close()
    g = mlb.grid_from_spec(ctx, specs[0])
    from paper_1902_02999_amd.mlb import lib
    assert lib().mlb_set_hbar(g.h, 7) != 0
    g.close()


def test_implicit_checked_step_and_volume(ctx):
    """The checked step (fused reduction) of the implicit form matches the
    oracle's diagnostics; its volume moves as the oracle's does, while Eq.
    h-bar keeps it."""
    from paper_1902_02999_amd import mlb
    spec = closed(64, 48, 9)
    state = wl.seeded_state(spec, 9, eta_amp=0.1, q_amp=0.1)
    g = mlb.grid_from_spec(ctx, spec)
    g.set_state(*state)
    m0 = g.diag()["mass"]
    ok, d = g.run_steady(0.0, 2000, 1000)
    h, qx, qy = g.get_state()
    g.close()
    ref = oracle_from_spec(spec, *state)
    r0 = ref.diag()["mass"]
    ref.run(2000)
    r = ref.diag()
    say("gpu mass drift", (d["mass"] - m0) / m0, "oracle", (r["mass"] - r0) / r0)
    assert d["nonfinite"] == 0
    assert d["mass"] == pytest.approx(r["mass"], rel=1e-9)
    assert abs((d["mass"] - m0) - (r["mass"] - r0)) <= 0.05 * abs(r["mass"] - r0) + 1e-6
    dh, du = compare(h, qx, qy, ref.h, ref.qx, ref.qy)
    assert dh <= H_TOL and du <= U_TOL
