"""GPU (FP32 HIP kernels, through the C ABI) against the FP64 oracle.

Bar (after equal step counts): max |dh| <= 1e-5 max h and max |du| <= 1e-4 max |u|;
still water bitwise; every execution variant (tile rows, graph chunks,
batching) bitwise equal to every other.
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


def run_gpu(ctx, spec, nsteps, state=None, opts=None, step0=0):
    from paper_1902_02999_amd import mlb
    g = mlb.grid_from_spec(ctx, spec)
    if state is not None:
        g.set_state(*state, step0=step0)
    if opts:
        g.set_exec_opts(**opts)
    g.step(nsteps)
    out = g.get_state()
    g.close()
    return out


def run_both(ctx, spec, nsteps, state=None, threads=0):
    say("case", spec.name, spec.nx, spec.ny, "steps", nsteps)
    got = run_gpu(ctx, spec, nsteps, state)
    ref = oracle_from_spec(spec, *(state if state is not None else spec.initial()))
    ref.threads = threads
    ref.run(nsteps)
    return got, (ref.h, ref.qx, ref.qy)


def bumpy(nx, ny, seed, amp=0.3, depth=2.0):
    rng = np.random.default_rng(seed)
    X, Y = np.meshgrid(np.arange(nx), np.arange(ny))
    zb = np.zeros((ny, nx))
    for _ in range(3):
        cx, cy = rng.uniform(0, nx), rng.uniform(0, ny)
        s = rng.uniform(nx / 12, nx / 4)
        zb += amp * rng.uniform(0.3, 1) * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2 * s * s))
    return zb


def closed_spec(nx, ny, seed, wind=(9.0, -4.0), chezy=45.0):
    return wl.Spec("closed_%dx%d" % (nx, ny), nx, ny, 1.0, 10.0 / 6.0, bumpy(nx, ny, seed), 2.0,
                   wind_speed=wind, chezy=chezy)


# ----------------------------------------------------------------------------- invariants
def test_lake_at_rest_is_bitwise(ctx):
    say("lake at rest 130x77")
    spec = wl.Spec("rest", 130, 77, 1.0, 10.0 / 6.0, bumpy(130, 77, 1, amp=0.8), 2.0)
    h, qx, qy = run_gpu(ctx, spec, 500)
    assert np.all(qx == 0.0) and np.all(qy == 0.0)
    assert np.array_equal(h, run_gpu(ctx, spec, 0)[0])


# ----------------------------------------------------------------------------- parity vs oracle
# The 5 x 4 basin runs few steps: its flow dies within ~100 steps, after which
# u is the residual of wind stress against surface tilt (|u| ~ 1e-6 m/s) and
# the FP32 quantum of eta (~1e-9 m) dominates any relative velocity measure.
@pytest.mark.parametrize("nx,ny,seed,steps", [(64, 64, 0, 300), (125, 70, 1, 300), (61, 9, 2, 300),
                                              (5, 4, 3, 30), (4, 133, 4, 300)])
def test_closed_basin_parity(ctx, nx, ny, seed, steps):
    spec = closed_spec(nx, ny, seed)
    state = wl.seeded_state(spec, seed, eta_amp=0.05, q_amp=0.1)
    got, ref = run_both(ctx, spec, steps, state)
    dh, du = compare(*got, *ref)
    say("dh", dh, "du", du)
    assert dh <= H_TOL and du <= U_TOL



def test_small_closed_basin_long_run(ctx):
    """The 5 x 4 closed basin over 3000 steps, long after its flow has died:
    the velocity error is measured against the flow's own scale (its largest
    speed, at the start), since the wind-driven remainder (|u| ~ 7e-7 m/s)
    makes the bar's max |u| of the final state ill-conditioned.  The steady
    surface tilt, which balances the wind stress, is compared on its own
    range after removing each side's mean level."""
    spec = closed_spec(5, 4, 3)
    state = wl.seeded_state(spec, 3, eta_amp=0.05, q_amp=0.1)
    h0, qx0, qy0 = state
    scale = (np.hypot(qx0, qy0) / h0).max()
    ref = oracle_from_spec(spec, *state)
    done = 0
    for n in (30, 300, 3000):
        got = run_gpu(ctx, spec, n, state)
        ref.run(n - done)
        done = n
        h, qx, qy = got
        dh = np.abs(h - ref.h).max() / np.abs(ref.h).max()
        du = max(np.abs(qx / h - ref.qx / ref.h).max(), np.abs(qy / h - ref.qy / ref.h).max())
        umax = (np.hypot(ref.qx, ref.qy) / ref.h).max()
        tg, tr = h - spec.H, ref.h - spec.H
        tg, tr = tg - tg.mean(), tr - tr.mean()
        dt_rel = np.abs(tg - tr).max() / (tr.max() - tr.min())
        say("steps", n, "dh", dh, "du/scale", du / scale, "du/max|u|", du / umax, "max|u|", umax,
            "tilt", dt_rel, "tilt range", tr.max() - tr.min())
        assert dh <= H_TOL and du / scale <= U_TOL
        # the steady tilt spans ~9e-5 m; 1e-3 of it is ~90 FP32 ulps of
        # |eta| ~ 0.01 m (measured: 7e-5 of it)
        assert dt_rel <= 1e-3


def test_periodic_parity(ctx):
    spec = wl.Spec("periodic", 70, 40, 1.0, 10.0 / 6.0, bumpy(70, 40, 5), 2.0,
                   edges=(wl.PERIODIC,) * 4, wind_speed=(5.0, 3.0), chezy=50.0, omega=1e-3)
    state = wl.seeded_state(spec, 5, q_amp=0.2)
    got, ref = run_both(ctx, spec, 400, state)
    dh, du = compare(*got, *ref)
    say("dh", dh, "du", du)
    assert dh <= H_TOL and du <= U_TOL


@pytest.mark.parametrize("order", [1, 2])
def test_open_channel_parity(ctx, order):
    spec = wl.bump_channel(150, 67, sigma=12.0)
    spec.extrap_order = order
    got, ref = run_both(ctx, spec, 600)
    dh, du = compare(*got, *ref)
    say("dh", dh, "du", du)
    assert dh <= H_TOL and du <= U_TOL


@pytest.mark.parametrize("order", [1, 2])
def test_open_channel_periodic_y_two_step_parity(ctx, order):
    """Open W / E edges with periodic S / N, two steps per pass (the edge
    tiles take the interior arithmetic and replace the open-edge nodes)."""
    spec = wl.bump_channel(190, 64, sigma=9.0)
    spec.edges = (wl.DISCHARGE, wl.DEPTH, wl.PERIODIC, wl.PERIODIC)
    spec.extrap_order = order
    say("case periodic-y channel, order", order)
    got = run_gpu(ctx, spec, 400, opts={"tblock": 2, "tile_rows": 14})
    ref = oracle_from_spec(spec)
    ref.run(400)
    dh, du = compare(*got, ref.h, ref.qx, ref.qy)
    say("dh", dh, "du", du)
    assert dh <= H_TOL and du <= U_TOL


def test_open_edges_on_y_parity(ctx):
    """Inflow on the south edge, outflow depth on the north edge (row pipeline
    deferral / history), periodic across."""
    nx, ny = 40, 90
    zb = bumpy(nx, ny, 7, amp=0.2)
    spec = wl.Spec("ychannel", nx, ny, 1.0, 25.0 / 6.0, zb, 2.0,
                   edges=(wl.PERIODIC, wl.PERIODIC, wl.DISCHARGE, wl.DEPTH), extrap_order=2,
                   depth_bc={wl.N: (2.0, 0.05, 30.0, 0.0)}, discharge_bc={wl.S: (0.1, 1.5)},
                   qy0=np.full((ny, nx), 1.5))
    got, ref = run_both(ctx, spec, 500)
    dh, du = compare(*got, *ref)
    say("dh", dh, "du", du)
    assert dh <= H_TOL and du <= U_TOL


def test_wind_lake_256_steady_state(ctx):
    """The 256 x 256 wind-driven dish lake from rest to a per-step residual of
    1e-6 (checks every 100 steps), FP32 on the GPU against the FP64 oracle:
    both cross 1e-6 at the same check and agree there at the parity bar; the
    GPU's state is within the residual-implied distance R / (1 - rho) of the
    oracle's fixed point (the oracle run on to R <= 1e-10), with rho the
    oracle's per-step contraction over its last checks."""
    from paper_1902_02999_amd import mlb
    spec = wl.wind_lake(256)
    g = mlb.grid_from_spec(ctx, spec)
    say("wind lake 256 to 1e-6 on the GPU")
    ok, dg = g.run_steady(1e-6, 400000, 100)
    got = g.get_state()
    g.close()
    assert ok and dg["residual"] <= 1e-6
    say("gpu steps", dg["step"], "residual", dg["residual"])
    ref = oracle_from_spec(spec)
    at_tol, hist = None, []
    while True:
        ref.run(99)
        q0 = (ref.qx.copy(), ref.qy.copy())
        ref.run(1)
        r = ref.diag(*q0)["residual"]
        hist.append(r)
        if at_tol is None and r <= 1e-6:
            at_tol = (ref.step_index, ref.h.copy(), ref.qx.copy(), ref.qy.copy())
            say("oracle crosses 1e-6 at", ref.step_index)
        if r <= 1e-10 or ref.step_index >= 400000:
            break
    say("oracle fixed point: steps", ref.step_index, "residual", hist[-1])
    assert hist[-1] <= 1e-10
    # same check, same state at the bar
    assert dg["step"] == at_tol[0]
    dh, du = compare(*got, *at_tol[1:])
    say("at 1e-6: dh", dh, "du", du)
    assert dh <= H_TOL and du <= U_TOL
    # residual-implied distance to the fixed point
    rho = (hist[-1] / hist[-11]) ** (1.0 / 1000.0)
    bound = dg["residual"] / (1.0 - rho)
    qg = np.concatenate([got[1].ravel(), got[2].ravel()])
    qr = np.concatenate([ref.qx.ravel(), ref.qy.ravel()])
    dist = np.linalg.norm(qg - qr) / np.linalg.norm(qr)
    say("rho", rho, "bound", bound, "distance", dist)
    assert dist <= 2.0 * bound


def test_tidal_strip_parity(ctx):
    spec = wl.tidal_strip()
    got, ref = run_both(ctx, spec, 10800)
    dh, du = compare(*got, *ref)
    say("dh", dh, "du", du)
    assert dh <= H_TOL and du <= U_TOL


def test_wind_lake_parity(ctx):
    spec = wl.wind_lake(64)
    got, ref = run_both(ctx, spec, 2000)
    dh, du = compare(*got, *ref)
    say("dh", dh, "du", du)
    assert dh <= H_TOL and du <= U_TOL


# ----------------------------------------------------------------------------- execution variants
def test_tile_rows_and_graphs_bitwise(ctx):
    spec = wl.bump_channel(190, 150, sigma=15.0)
    spec.extrap_order = 2
    base = None
    for opts in ({"tile_rows": 4, "use_graph": False}, {"tile_rows": 64, "use_graph": False},
                 {"tile_rows": 37, "use_graph": True, "graph_chunk": 8},
                 {"tile_rows": 256, "use_graph": True, "graph_chunk": 64}):
        say("variant", opts)
        out = run_gpu(ctx, spec, 131, opts=opts)
        if base is None:
            base = out
        else:
            for a, b in zip(out, base):
                assert np.array_equal(a, b)


def _two_step_cases():
    """(name, spec, state, steps, tile_rows): every edge kind, extrapolation
    order, narrow and odd strips, tiles shifted to row 1, odd step counts."""
    cases = []
    sp = closed_spec(64, 64, 0)
    cases.append(("closed64", sp, wl.seeded_state(sp, 0, q_amp=0.1), 131, 15))
    sp = closed_spec(125, 70, 1)
    cases.append(("closed125x70_rows21", sp, wl.seeded_state(sp, 1, q_amp=0.1), 64, 21))
    for nx, ny, rows in ((5, 4, 4), (4, 133, 9), (61, 9, 6), (121, 22, 21), (59, 31, 30), (60, 25, 12)):
        sp = closed_spec(nx, ny, nx + ny)
        cases.append(("closed%dx%d_rows%d" % (nx, ny, rows), sp, wl.seeded_state(sp, 2, q_amp=0.1), 37, rows))
    sp = wl.Spec("periodic", 70, 40, 1.0, 10.0 / 6.0, bumpy(70, 40, 5), 2.0,
                 edges=(wl.PERIODIC,) * 4, wind_speed=(5.0, 3.0), chezy=50.0, omega=1e-3)
    cases.append(("periodic70x40", sp, wl.seeded_state(sp, 5, q_amp=0.2), 101, 9))
    sp = wl.Spec("periodic_narrow", 3, 5, 1.0, 10.0 / 6.0, bumpy(3, 5, 6), 2.0,
                 edges=(wl.PERIODIC,) * 4, wind_speed=(5.0, 3.0))
    cases.append(("periodic3x5", sp, wl.seeded_state(sp, 6, q_amp=0.2), 40, 4))
    for order in (1, 2):
        sp = wl.bump_channel(150, 67, sigma=12.0)
        sp.extrap_order = order
        cases.append(("channel_order%d" % order, sp, None, 120, 15))
        sp = wl.bump_channel(181, 22, sigma=6.0)
        sp.extrap_order = order
        cases.append(("channel181x22_rows21_order%d" % order, sp, None, 77, 21))
    for order in (1, 2):
        # open W / E edges with periodic S / N: every edge tile takes the
        # interior arithmetic plus the open-edge replacement
        sp = wl.bump_channel(190, 64, sigma=9.0)
        sp.edges = (wl.DISCHARGE, wl.DEPTH, wl.PERIODIC, wl.PERIODIC)
        sp.extrap_order = order
        cases.append(("channel_periodic_y_order%d" % order, sp, None, 91, 17))
    nx, ny = 40, 90
    for order in (1, 2):
        sp = wl.Spec("ychannel", nx, ny, 1.0, 25.0 / 6.0, bumpy(nx, ny, 7, amp=0.2), 2.0,
                     edges=(wl.PERIODIC, wl.PERIODIC, wl.DISCHARGE, wl.DEPTH), extrap_order=order,
                     depth_bc={wl.N: (2.0, 0.05, 30.0, 0.0)}, discharge_bc={wl.S: (0.1, 1.5)},
                     qy0=np.full((ny, nx), 1.5))
        cases.append(("ychannel_order%d" % order, sp, None, 99, 12))
    sp = wl.Spec("ydepth", 70, 46, 1.0, 25.0 / 6.0, bumpy(70, 46, 9, amp=0.2), 2.0,
                 edges=(wl.WALL, wl.WALL, wl.DEPTH, wl.DISCHARGE), extrap_order=2,
                 depth_bc={wl.S: (2.0, 0.03, 20.0, 0.5)}, discharge_bc={wl.N: (0.0, 0.5)})
    cases.append(("ydepth_walls", sp, None, 66, 15))
    cases.append(("ydepth_walls_rows4", sp, None, 66, 4))
    cases.append(("tidal_strip", wl.tidal_strip(), None, 500, 15))
    # four-row tiles (the shortest the tuner tries) on grids of many tiles
    sp = closed_spec(64, 64, 0)
    cases.append(("closed64_rows4", sp, wl.seeded_state(sp, 0, q_amp=0.1), 131, 4))
    sp = wl.bump_channel(150, 67, sigma=12.0)
    sp.extrap_order = 2
    cases.append(("channel_order2_rows4", sp, None, 120, 4))
    sp = wl.Spec("ychannel", 40, 90, 1.0, 25.0 / 6.0, bumpy(40, 90, 7, amp=0.2), 2.0,
                 edges=(wl.PERIODIC, wl.PERIODIC, wl.DISCHARGE, wl.DEPTH), extrap_order=2,
                 depth_bc={wl.N: (2.0, 0.05, 30.0, 0.0)}, discharge_bc={wl.S: (0.1, 1.5)},
                 qy0=np.full((90, 40), 1.5))
    cases.append(("ychannel_order2_rows4", sp, None, 99, 4))
    return cases


_TB2 = _two_step_cases()


@pytest.mark.parametrize("case", _TB2, ids=[c[0] for c in _TB2])
def test_two_step_passes_bitwise(ctx, case):
    """Two steps per pass (temporal blocking) give the bits of one step per pass."""
    name, spec, state, steps, rows = case
    say("two-step case", name, spec.nx, spec.ny, "steps", steps, "rows", rows)
    one = run_gpu(ctx, spec, steps, state, opts={"tile_rows": rows, "tblock": 1})
    for opts in ({"tile_rows": rows, "tblock": 2},
                 {"tile_rows": rows, "tblock": 2, "use_graph": True, "graph_chunk": 8}):
        two = run_gpu(ctx, spec, steps, state, opts=opts)
        for a, b in zip(two, one):
            assert np.array_equal(a, b), (name, opts)


def test_two_step_diag_and_steady_match(ctx):
    """Steady-state runs stop at the same check with the same state bit for
    bit with one or two steps per pass.  The two-step run's checks are fused
    into its closing two-step pass (the residual against the level it holds
    in registers): its FP64 sums run over the two-step tiles, so they agree
    with the one-step checks to summation order (1e-13), and the per-node
    maximum and the count exactly."""
    from paper_1902_02999_amd import mlb
    spec = closed_spec(90, 70, 4)
    res = []
    for tb in (1, 2):
        g = mlb.grid_from_spec(ctx, spec)
        g.set_exec_opts(tblock=tb, tile_rows=12)
        ok, d = g.run_steady(1e-5, 200000, 100)
        g.step(4)
        res.append((ok, d, g.diag(), g.get_state()))
        g.close()
    (ok1, d1, e1, s1), (ok2, d2, e2, s2) = res
    assert ok1 and ok2
    for k in ("step", "max_speed", "nonfinite"):
        assert d1[k] == d2[k] and e1[k] == e2[k], k
    for k in ("mass", "residual"):
        assert d2[k] == pytest.approx(d1[k], rel=1e-13) and e2[k] == pytest.approx(e1[k], rel=1e-13), k
    for a, b in zip(s1, s2):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("case", ["closed", "channel", "dish", "implicit", "friction_periodic"])
@pytest.mark.parametrize("n", [50, 51, 2])
def test_fused_two_step_diag_equals_one_step_diag(ctx, case, n):
    """A call of n steps ends with a checked pass of its own kind: with two
    steps per pass the residual of the last step is taken against the level
    the pass holds in registers.  It equals the one-step run's (same fields
    bit for bit) to FP64 summation order; the bulk passes are timed alone."""
    from paper_1902_02999_amd import mlb
    if case == "closed":
        spec = closed_spec(130, 90, 5)
    elif case == "channel":
        spec = wl.bump_channel(150, 70, sigma=9.0)
    elif case == "dish":
        spec = wl.circular_dish(120, 400.0 / 120)
    elif case == "implicit":
        spec = wl.bump_channel(96, 80, sigma=8.0, bump=0.4)
        spec.hbar_implicit = True
    else:
        spec = closed_spec(100, 64, 6)
        spec.edges = (wl.PERIODIC,) * 4
    out = []
    for tb in (1, 2):
        g = mlb.grid_from_spec(ctx, spec)
        g.set_exec_opts(tblock=tb, tile_rows=11, graph_chunk=8)
        g.step(7)
        say(case, "n", n, "tblock", tb)
        g.step(n)
        d = g.diag()
        if tb == 2 and n == 50:
            ms, passes, k = ctx.last_pass_ms()
            assert (passes, k) == (24, 2) and ms > 0
        out.append((d, g.get_state()))
        g.close()
    (d1, s1), (d2, s2) = out
    for a, b in zip(s1, s2):
        assert np.array_equal(a, b)
    assert d1["step"] == d2["step"] == 7 + n
    assert d1["nonfinite"] == d2["nonfinite"] == 0
    assert d2["max_speed"] == d1["max_speed"]
    assert d2["mass"] == pytest.approx(d1["mass"], rel=1e-13)
    assert d1["residual"] > 0
    assert d2["residual"] == pytest.approx(d1["residual"], rel=1e-12)


def test_two_step_batch_bitwise(ctx):
    from paper_1902_02999_amd import mlb
    specs = [closed_spec(n, m, s) for (n, m, s) in ((64, 64, 0), (200, 97, 1), (33, 150, 2))]
    specs.append(wl.bump_channel(130, 60, sigma=10.0))
    solo = [run_gpu(ctx, s, 77) for s in specs]
    grids = [mlb.grid_from_spec(ctx, s) for s in specs]
    b = mlb.Batch(ctx, grids)
    b.set_exec_opts(tile_rows=15, tblock=2, graph_chunk=8)
    say("two-step batch of", len(grids))
    b.step(77)
    b.close()
    for g, ref in zip(grids, solo):
        for a, r in zip(g.get_state(), ref):
            assert np.array_equal(a, r)
        g.close()
    # the closed basins on their own take the kernel without open-edge logic,
    # in the batch with the open channel the general one: same bits
    for s, ref in zip(specs[:3], solo):
        got = run_gpu(ctx, s, 77, opts=dict(tile_rows=15, tblock=2, graph_chunk=8))
        for a, r in zip(got, ref):
            assert np.array_equal(a, r)


_PERSIST = [c for c in _TB2 if c[0] in ("closed64", "closed61x9_rows6", "periodic70x40", "channel_order2",
                                          "ychannel_order2", "ydepth_walls", "tidal_strip")]


@pytest.mark.parametrize("persistent", [1, 2], ids=["cooperative", "workqueue"])
@pytest.mark.parametrize("case", _PERSIST, ids=[c[0] for c in _PERSIST])
def test_persistent_launches_bitwise(ctx, case, persistent):
    """All passes of a call in one persistent launch, separated by grid
    barriers (1) or ordered per tile by the work queue's epoch flags (2), give
    the bits of one launch per pass, for one and two steps per pass (the
    work queue also with a workgroup cap: fewer waves than tiles)."""
    name, spec, state, steps, rows = case
    say("persistent", persistent, "case", name, spec.nx, spec.ny, "steps", steps)
    for tb in (1, 2):
        ref = run_gpu(ctx, spec, steps, state, opts={"tile_rows": rows, "tblock": tb})
        caps = (0, 1) if persistent == 2 else (0,)
        for cap in caps:
            say("  tblock", tb, "cap", cap)
            got = run_gpu(ctx, spec, steps, state,
                          opts={"tile_rows": rows, "tblock": tb, "persistent": persistent, "blocks_per_cu": cap})
            for a, b in zip(got, ref):
                assert np.array_equal(a, b), (name, tb, cap)


@pytest.mark.parametrize("persistent", [1, 2], ids=["cooperative", "workqueue"])
def test_persistent_steady_and_batch(ctx, persistent):
    from paper_1902_02999_amd import mlb
    spec = closed_spec(90, 70, 4)
    res = []
    for ps in (0, persistent):
        g = mlb.grid_from_spec(ctx, spec)
        g.set_exec_opts(tblock=2, tile_rows=6, persistent=ps)
        ok, d = g.run_steady(1e-5, 200000, 100)
        res.append((ok, d, g.get_state()))
        g.close()
    assert res[0][0] and res[1][0]
    for k in ("step", "mass", "residual"):
        assert res[0][1][k] == res[1][1][k], k
    for a, b in zip(res[0][2], res[1][2]):
        assert np.array_equal(a, b)
    specs = [closed_spec(n, m, s) for (n, m, s) in ((64, 64, 0), (100, 37, 1), (33, 150, 2))]
    solo = [run_gpu(ctx, s, 45) for s in specs]
    grids = [mlb.grid_from_spec(ctx, s) for s in specs]
    b = mlb.Batch(ctx, grids)
    b.set_exec_opts(tile_rows=9, tblock=2, persistent=persistent)
    b.step(45)
    b.close()
    for g, ref in zip(grids, solo):
        for x, y in zip(g.get_state(), ref):
            assert np.array_equal(x, y)
        g.close()


def test_workqueue_wait_timeout_is_reported(ctx, monkeypatch):
    """A work-queue launch whose waits may poll zero times gives up at its
    first wait (forced from the host); every state call reports it, later
    launches of the plan do nothing until then, and the grid works again once
    its state is set."""
    from paper_1902_02999_amd import mlb
    monkeypatch.setenv("MLB_SPIN_LIMIT", "0")
    c = mlb.Context(0)
    monkeypatch.delenv("MLB_SPIN_LIMIT")
    spec = closed_spec(150, 90, 0)
    state = wl.seeded_state(spec, 0, q_amp=0.1)
    g = mlb.grid_from_spec(c, spec)
    g.set_state(*state)
    g.set_exec_opts(tile_rows=8, tblock=2, persistent=2)
    for call in (lambda: g.diag(), lambda: g.get_state(), lambda: c.sync()):
        g.set_state(*state)
        g.step(20)
        with pytest.raises(mlb.MlbError) as ei:
            call()
        assert ei.value.name == "MLB_E_DEVICE"
        c.sync()   # reported and cleared
    g.set_state(*state)
    g.set_exec_opts(tile_rows=8, tblock=2, persistent=0)
    g.step(20)
    got = g.get_state()
    g.close()
    c.close()
    ref = run_gpu(ctx, spec, 20, state)
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)


def test_workqueue_ensemble_512_bitwise(ctx):
    """The 512-basin ensemble (sizes 64^2 .. 512^2, seed 1902) in one
    work-queue launch per call gives the bits of one graph-launched pass per
    two steps; states compared on the device."""
    import torch
    from paper_1902_02999_amd import mlb
    specs = wl.ensemble(512, 1902)
    outs = []
    for ps in (0, 2):
        grids = [mlb.grid_from_spec(ctx, s) for s in specs]
        b = mlb.Batch(ctx, grids)
        b.set_exec_opts(tile_rows=17, tblock=2, persistent=ps, graph_chunk=100, blocks_per_cu=0)
        say("ensemble, persistent", ps)
        b.step(7)
        b.step(30)
        b.close()
        fields = []
        for g, sp in zip(grids, specs):
            f = torch.empty((3, sp.ny, sp.nx), dtype=torch.float32, device="cuda")
            g.get_state_device(f[0], f[1], f[2])
            fields.append(f)
            g.close()
        ctx.sync()
        outs.append(fields)
    for a, b in zip(*outs):
        assert torch.equal(a, b)



def test_ensemble_512_sampled_against_oracle(ctx):
    """The 512-basin ensemble (sizes 64^2 .. 512^2, seed 1902) in the launch
    configuration its benchmark times (one batch, two steps per pass, 17-row
    tiles, 4 workgroups per CU, graph chunks of 100 steps; closed basins, so
    the two-step kernel without open-edge logic) against the oracle on a
    sample of its basins: the largest, the smallest and six drawn at random
    (seeded), 41 steps from seeded perturbed states, each at the bar.  The
    other basins start from rest and share every launch."""
    from paper_1902_02999_amd import mlb
    specs = wl.ensemble(512, 1902)
    sizes = np.array([s.nx for s in specs])
    rng = np.random.default_rng(7)
    pick = sorted({int(np.argmax(sizes)), int(np.argmin(sizes))} |
                  {int(i) for i in rng.choice(len(specs), 6, replace=False)})
    states = {i: wl.seeded_state(specs[i], i, q_amp=0.1) for i in pick}
    grids = [mlb.grid_from_spec(ctx, s) for s in specs]
    for i in pick:
        grids[i].set_state(*states[i])
    b = mlb.Batch(ctx, grids)
    b.set_exec_opts(tile_rows=17, tblock=2, use_graph=True, graph_chunk=100, blocks_per_cu=4)
    say("ensemble 512 basins, 41 steps; sampled", [(i, specs[i].nx) for i in pick])
    b.step(41)
    b.close()
    got = {i: grids[i].get_state() for i in pick}
    for g in grids:
        g.close()
    for i in pick:
        ref = oracle_from_spec(specs[i], *states[i])
        ref.run(41)
        dh, du = compare(*got[i], ref.h, ref.qx, ref.qy)
        say("basin", i, specs[i].nx, "dh", dh, "du", du)
        assert dh <= H_TOL and du <= U_TOL, (i, specs[i].nx)


def test_persistent_barrier_timeout_is_reported(ctx, monkeypatch):
    """A barrier wait forced to give up at once (spin limit 0, set from the
    host) ends the launch; the next check reports it, and the grid works
    again once its state is set."""
    from paper_1902_02999_amd import mlb
    monkeypatch.setenv("MLB_SPIN_LIMIT", "0")
    c = mlb.Context(0)
    monkeypatch.delenv("MLB_SPIN_LIMIT")
    spec = closed_spec(64, 64, 0)
    state = wl.seeded_state(spec, 0, q_amp=0.1)
    g = mlb.grid_from_spec(c, spec)
    g.set_state(*state)
    g.set_exec_opts(tile_rows=4, tblock=1, persistent=1)   # 32 tiles, 8 workgroups
    g.step(20)
    with pytest.raises(mlb.MlbError) as ei:
        g.diag()
    assert ei.value.name == "MLB_E_DEVICE"
    # every call that hands out state reports the give-up, once
    for call in (lambda: g.get_state(), lambda: c.sync()):
        g.set_state(*state)
        g.step(20)
        with pytest.raises(mlb.MlbError) as ei:
            call()
        assert ei.value.name == "MLB_E_DEVICE"
        c.sync()   # reported and cleared
    # the autotuner never keeps a persistent candidate whose launches gave up
    g.set_state(*state)
    best = g.autotune(steps=8)
    assert best["persistent"] == 0
    g.step(20)
    g.get_state()
    # recovered: ordinary launches from a fresh state match a fresh grid
    g.set_state(*state)
    g.set_exec_opts(tile_rows=4, tblock=1, persistent=0)
    g.step(20)
    got = g.get_state()
    g.close()
    c.close()
    ref = run_gpu(ctx, spec, 20, state)
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)


def test_batch_equals_solo_bitwise(ctx):
    from paper_1902_02999_amd import mlb
    specs = [closed_spec(n, m, s) for (n, m, s) in ((64, 64, 0), (200, 97, 1), (33, 150, 2))]
    specs.append(wl.bump_channel(130, 60, sigma=10.0))
    solo = [run_gpu(ctx, s, 77) for s in specs]
    grids = [mlb.grid_from_spec(ctx, s) for s in specs]
    b = mlb.Batch(ctx, grids)
    say("batch of", len(grids))
    b.step(77)
    b.close()
    for g, ref in zip(grids, solo):
        got = g.get_state()
        for a, r in zip(got, ref):
            assert np.array_equal(a, r)
        g.close()


# ----------------------------------------------------------------------------- diagnostics
def test_diag_matches_oracle_on_same_fields(ctx):
    from paper_1902_02999_amd import mlb
    spec = closed_spec(150, 90, 3)
    state = wl.seeded_state(spec, 3, q_amp=0.1)
    g = mlb.grid_from_spec(ctx, spec)
    g.set_state(*state)
    g.step(49)
    h0, qx0, qy0 = g.get_state()
    g.step(1)
    d = g.diag()
    h1, qx1, qy1 = g.get_state()
    ref = oracle_from_spec(spec, h1, qx1, qy1)
    r = ref.diag(qx0, qy0)
    assert d["step"] == 50
    assert d["mass"] == pytest.approx(r["mass"], rel=1e-13)
    assert d["residual"] == pytest.approx(r["residual"], rel=1e-12)
    # the device divides by the stored FP32 still-water depth plus eta
    assert d["max_speed"] == pytest.approx(r["max_speed"], rel=1e-6)
    assert d["nonfinite"] == 0
    g.close()


def test_mass_conserved_in_closed_basin(ctx):
    from paper_1902_02999_amd import mlb
    spec = closed_spec(256, 256, 4)
    g = mlb.grid_from_spec(ctx, spec)
    g.set_state(*wl.seeded_state(spec, 4, q_amp=0.1))
    m0 = g.diag()["mass"]
    g.step(2000)
    m1 = g.diag()["mass"]
    say("mass drift", (m1 - m0) / m0)
    # FP32 storage: each step rounds eta to 2^-24 relative of |eta| per node
    assert abs(m1 - m0) / m0 <= 1e-6
    g.close()


def test_run_steady_and_nonfinite(ctx):
    from paper_1902_02999_amd import mlb
    spec = closed_spec(48, 40, 6, wind=(8.0, 0.0))
    g = mlb.grid_from_spec(ctx, spec)
    ok, d = g.run_steady(1e-6, 200000, 100)
    say("steady", ok, d["step"], d["residual"])
    assert ok and d["residual"] <= 1e-6 and d["step"] % 100 == 0
    h, qx, qy = g.get_state()
    h[5, 7] = np.nan
    g.set_state(h, qx, qy)
    with pytest.raises(mlb.MlbError) as ei:
        g.run_steady(1e-6, 1000, 10)
    assert ei.value.name == "MLB_E_NONFINITE"
    g.close()


def test_unstable_parameters_rejected(ctx):
    from paper_1902_02999_amd import mlb
    p = mlb.make_params(20, 20, 1.0, 1.0, zeta_ref=10.0)  # e = 6 m/s
    g = mlb.Grid(ctx, p)                                    # default bed: H = 1 m, stable
    with pytest.raises(mlb.MlbError) as ei:
        g.set_bathymetry(np.zeros((20, 20)))                # H = 10 m: g H = 98 > e^2 = 36
    assert ei.value.name == "MLB_E_UNSTABLE"
    g.close()


# ----------------------------------------------------------------------------- full size, whole field
def test_full_size_bump_channel_whole_field(ctx):
    """4096 x 4096 channel in the benchmark's launch configuration (two steps
    per pass, 26-row tiles, 4 workgroups per CU, graphs): four GPU steps from
    a GPU state against four oracle steps from the same state, every one of
    the 16.8 M nodes at the bar (and at 1e-6 of the field scales, the FP32
    rounding of four steps), and the fused diagnostics of the last step."""
    from paper_1902_02999_amd import mlb
    spec = wl.bump_channel(4096)
    say("full size, whole field", spec.name)
    g = mlb.grid_from_spec(ctx, spec)
    g.set_exec_opts(tblock=2, tile_rows=26, blocks_per_cu=4, use_graph=True, graph_chunk=100)
    g.step(20)
    h0, qx0, qy0 = g.get_state()
    g.step(4)
    d = g.diag()
    h4, qx4, qy4 = g.get_state()
    g.close()
    ref = oracle_from_spec(spec, h0, qx0, qy0, step0=20)
    ref.run(3)
    rq = (ref.qx.copy(), ref.qy.copy())
    ref.run(1)
    dh, du = compare(h4, qx4, qy4, ref.h, ref.qx, ref.qy)
    say("dh", dh, "du", du)
    assert dh <= H_TOL and du <= U_TOL
    hmax, qmax = np.abs(ref.h).max(), max(np.abs(ref.qx).max(), np.abs(ref.qy).max())
    assert np.abs(h4 - ref.h).max() <= 1e-6 * hmax
    assert np.abs(qx4 - ref.qx).max() <= 1e-6 * qmax and np.abs(qy4 - ref.qy).max() <= 1e-6 * qmax
    r = ref.diag(*rq)
    say("diag gpu", d["mass"], d["residual"], "oracle", r["mass"], r["residual"])
    assert d["step"] == 24 and d["nonfinite"] == 0
    assert d["mass"] == pytest.approx(r["mass"], rel=1e-9)
    # the residual is a difference of FP32 fields: their rounding, not the sums, limits it
    assert d["residual"] == pytest.approx(r["residual"], rel=1e-2)


def test_full_size_two_step_bitwise(ctx):
    """4096 x 4096 channel: two steps per pass give the bits of one step per
    pass (whose single steps the sampled oracle test checks)."""
    from paper_1902_02999_amd import mlb
    spec = wl.bump_channel(4096)
    outs = []
    for tb in (1, 2):
        say("full size tblock", tb)
        g = mlb.grid_from_spec(ctx, spec)
        g.set_exec_opts(tile_rows=15, tblock=tb, blocks_per_cu=3)
        g.step(21)
        outs.append(g.get_state())
        g.close()
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


# ----------------------------------------------------------------------------- tuning
def test_blocks_per_cu_bitwise(ctx):
    spec = wl.bump_channel(200, 130, sigma=12.0)
    outs = [run_gpu(ctx, spec, 64, opts={"blocks_per_cu": cap, "tile_rows": 21}) for cap in (0, 1, 3, 8)]
    for o in outs[1:]:
        for a, b in zip(o, outs[0]):
            assert np.array_equal(a, b)


def test_autotune_keeps_state_and_caches(ctx, tmp_path):
    from paper_1902_02999_amd import mlb
    spec = closed_spec(300, 170, 8)
    g = mlb.grid_from_spec(ctx, spec)
    g.set_state(*wl.seeded_state(spec, 8, q_amp=0.1), step0=5)
    before = g.get_state()
    cache = str(tmp_path / "tune.txt")
    say("autotune", spec.name)
    best = g.autotune(steps=8, cache_path=cache)
    assert best["tile_rows"] in (4, 6, 9, 12, 15, 21, 27, 33, 45, 5, 8, 11, 14, 17, 20, 23, 26, 32, 44)
    assert best["blocks_per_cu"] in (0, 2, 3, 4, 5)
    assert best["tblock"] in (1, 2)
    after = g.get_state()
    for a, b in zip(before, after):
        assert np.array_equal(a, b)
    assert g.diag()["step"] == 5
    lines = open(cache).read().split()
    assert len(lines) == 6 and lines[0].endswith("_g300x170") and int(lines[3]) in (1, 2)
    assert int(lines[4]) in (0, 1)
    # second call: served from the cache, same choice
    assert g.autotune(steps=8, cache_path=cache) == g.exec_opts().as_dict()
    # stepping after tuning equals stepping an untuned copy
    g.step(33)
    ref = run_gpu(ctx, spec, 33, state=wl.seeded_state(spec, 8, q_amp=0.1), step0=5)
    for a, b in zip(g.get_state(), ref):
        assert np.array_equal(a, b)
    g.close()


def test_batch_autotune_keeps_state(ctx):
    from paper_1902_02999_amd import mlb
    specs = [closed_spec(n, n, s) for n, s in ((70, 1), (130, 2), (64, 3))]
    grids = [mlb.grid_from_spec(ctx, s) for s in specs]
    for g, s in zip(grids, specs):
        g.set_state(*wl.seeded_state(s, 1, q_amp=0.1))
    before = [g.get_state() for g in grids]
    b = mlb.Batch(ctx, grids)
    best = b.autotune(steps=6)
    assert best["tile_rows"] in (4, 6, 9, 12, 15, 21, 27, 33, 45, 5, 8, 11, 14, 17, 20, 23, 26, 32, 44)
    b.close()
    for g, bf in zip(grids, before):
        for x, y in zip(g.get_state(), bf):
            assert np.array_equal(x, y)
        g.close()
