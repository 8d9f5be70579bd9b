"""Node-kind mask on the GPU (one-step kernel, masked tiles on the edge path)
against the FP64 oracle, bitwise invariants, and the paper's own geometries
(Section 4): the circular wind-driven basin and the 2D hump channel.

Bar as for the other parity tests (max |dh| <= 1e-5 max h, max |du| <= 1e-4
max |u|) over the water; SOLID nodes keep their stored values bit for bit.
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


def masked_spec(nx, ny, seed, edges=(wl.WALL,) * 4, chezy=45.0, omega=0.0):
    kind = wl.random_geometry(np.random.Generator(np.random.PCG64(seed)), nx, ny, holes=4)
    return wl.Spec("masked_%dx%d_%d" % (nx, ny, seed), nx, ny, 1.0, 10.0 / 6.0, bumpy(nx, ny, seed), 2.0,
                   edges=edges, wind_speed=(9.0, -4.0), chezy=chezy, omega=omega, kind=kind)


def seeded(spec, seed, solid_h=None):
    h, qx, qy = wl.seeded_state(spec, seed, eta_amp=0.05, q_amp=0.1)
    if solid_h is not None and spec.kind is not None:
        h = np.where(spec.kind == wl.SOLID, solid_h, h)
    return h, qx, qy


def run_gpu(ctx, spec, nsteps, state=None, opts=None, grid_out=False):
    from paper_1902_02999_amd import mlb
    g = mlb.grid_from_spec(ctx, spec)
    if state is not None:
        g.set_state(*state)
    if opts:
        g.set_exec_opts(**opts)
    g.step(nsteps)
    out = g.get_state()
    if grid_out:
        return out, g
    g.close()
    return out


def check_parity(ctx, spec, nsteps, state, opts=None):
    say("case", spec.name, spec.nx, spec.ny, "steps", nsteps, "opts", opts)
    got = run_gpu(ctx, spec, nsteps, state, opts)
    ref = oracle_from_spec(spec, *state)
    ref.run(nsteps)
    water = spec.kind != wl.SOLID
    dh, du = compare(*got, ref.h, ref.qx, ref.qy, where=water)
    say("dh", dh, "du", du)
    assert dh <= H_TOL and du <= U_TOL
    solid = ~water
    # SOLID nodes: the stored FP32 state, untouched
    g0 = run_gpu(ctx, spec, 0, state)
    for a, b in zip(got, g0):
        assert np.array_equal(a[solid], b[solid])
    wall = spec.kind == wl.WALL_NODE
    assert (got[1][wall] == 0).all() and (got[2][wall] == 0).all()
    return got


# ----------------------------------------------------------------------------- parity vs oracle
@pytest.mark.parametrize("nx,ny,seed,chezy", [(70, 45, 1, 45.0), (130, 67, 2, 0.0), (20, 133, 3, 45.0),
                                              (190, 30, 4, 60.0)])
def test_masked_basin_parity(ctx, nx, ny, seed, chezy):
    spec = masked_spec(nx, ny, seed, chezy=chezy)
    check_parity(ctx, spec, 300, seeded(spec, seed, solid_h=-1.0))


def test_masked_periodic_parity(ctx):
    """A mask on a periodic grid: islands and a wrapped basin shape."""
    spec = masked_spec(96, 50, 6, edges=(wl.PERIODIC,) * 4, omega=1e-3)
    check_parity(ctx, spec, 300, seeded(spec, 6))


def test_islands_in_an_open_channel_parity(ctx):
    """SOLID islands and a WALL-lined breakwater in a channel with a
    prescribed inflow discharge and outflow depth (open edges kept FLUID)."""
    spec = wl.bump_channel(180, 60, sigma=10.0)
    Y, X = np.mgrid[0:60, 0:180].astype(float)
    inside = ((X - 70) ** 2 + (Y - 25) ** 2 > 36) & ((X - 120) ** 2 + (Y - 40) ** 2 > 20)
    inside &= ~((X >= 95) & (X < 98) & (Y < 22))
    spec.kind = wl.staircase_kinds(np.pad(inside[1:-1, 3:-3], ((1, 1), (3, 3)), constant_values=True))
    spec.kind[0, :] = wl.FLUID
    spec.kind[-1, :] = wl.FLUID
    spec.kind[:, :3] = wl.FLUID
    spec.kind[:, -3:] = wl.FLUID
    check_parity(ctx, spec, 400, spec.initial())


def test_dish_parity_at_paper_size(ctx):
    spec = wl.circular_dish()
    state = wl.seeded_state(spec, 9, eta_amp=0.02, q_amp=0.02)
    check_parity(ctx, spec, 300, state)


def test_hump_parity_at_paper_size(ctx):
    spec = wl.hump_channel()
    spec.kind = None
    got = run_gpu(ctx, spec, 300)
    ref = oracle_from_spec(spec)
    ref.run(300)
    dh, du = compare(*got, ref.h, ref.qx, ref.qy)
    say("hump dh", dh, "du", du)
    assert dh <= H_TOL and du <= U_TOL


# ----------------------------------------------------------------------------- bitwise invariants
@pytest.mark.parametrize("nx,ny,outer", [(150, 97, wl.WALL), (61, 9, wl.PERIODIC), (64, 64, wl.WALL)])
def test_ring_mask_is_the_rectangular_basin_bitwise(ctx, nx, ny, outer):
    """(nx+2) x (ny+2) with a SOLID ring around a WALL ring runs the nx x ny
    wall basin bit for bit (bounce flags from the mask instead of the edges)."""
    rect = wl.Spec("rect", nx, ny, 1.0, 10.0 / 6.0, bumpy(nx, ny, 3), 2.0, wind_speed=(7.0, 3.0),
                   chezy=40.0, omega=2e-3)
    state = seeded(rect, 3)
    inside = np.zeros((ny + 2, nx + 2), bool)
    inside[1:-1, 1:-1] = True
    pad = lambda a, v: np.pad(a, 1, constant_values=v)
    big = wl.Spec("ring", nx + 2, ny + 2, 1.0, 10.0 / 6.0, pad(rect.zb, 0.0), 2.0, edges=(outer,) * 4,
                  wind_speed=(7.0, 3.0), chezy=40.0, omega=2e-3, kind=wl.staircase_kinds(inside))
    bstate = (pad(state[0], 2.5), pad(state[1], 1.0), pad(state[2], -1.0))
    a, ga = run_gpu(ctx, rect, 200, state, grid_out=True)
    b, gb = run_gpu(ctx, big, 200, bstate, grid_out=True)
    for u, v in zip(a, b):
        assert np.array_equal(u, v[1:-1, 1:-1])
    da, db = ga.diag(), gb.diag()
    ga.close()
    gb.close()
    assert db["mass"] == pytest.approx(da["mass"], rel=1e-12)
    assert db["nonfinite"] == 0


def test_masked_execution_variants_bitwise(ctx):
    from paper_1902_02999_amd import mlb
    spec = masked_spec(150, 80, 7)
    state = seeded(spec, 7, solid_h=-3.0)
    base = run_gpu(ctx, spec, 101, state, dict(tile_rows=15, tblock=1, use_graph=0))
    for o in (dict(tile_rows=4), dict(tile_rows=7, use_graph=1, graph_chunk=8), dict(tile_rows=40),
              dict(tile_rows=15, tblock=2), dict(tile_rows=12, persistent=1), dict(tile_rows=9, blocks_per_cu=2)):
        got = run_gpu(ctx, spec, 101, state, o)
        say("variant", o)
        for u, v in zip(base, got):
            assert np.array_equal(u, v)
    # the mask removed again: the plain grid, bit for bit
    plain = wl.Spec(spec.name, spec.nx, spec.ny, spec.dx, spec.nu, spec.zb, spec.zeta_ref, edges=spec.edges,
                    wind_speed=spec.wind_speed, chezy=spec.chezy)
    state = seeded(spec, 7)   # wet everywhere: SOLID nodes join the water
    g = mlb.grid_from_spec(ctx, spec)
    g.set_mask(None)
    g.set_state(*state)
    g.step(50)
    a = g.get_state()
    g.close()
    b = run_gpu(ctx, plain, 50, state)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


def test_masked_batch_bitwise(ctx):
    from paper_1902_02999_amd import mlb
    specs = [masked_spec(130, 67, 2), wl.Spec("plain", 90, 70, 1.0, 10.0 / 6.0, bumpy(90, 70, 5), 2.0,
                                               wind_speed=(3.0, 8.0), chezy=50.0), wl.circular_dish(120, 400.0 / 120)]
    states = [seeded(s, i) for i, s in enumerate(specs)]
    singles = [run_gpu(ctx, s, 77, st) for s, st in zip(specs, states)]
    gs = [mlb.grid_from_spec(ctx, s) for s in specs]
    for g, st in zip(gs, states):
        g.set_state(*st)
    b = mlb.Batch(ctx, gs)
    b.set_exec_opts(tile_rows=12, tblock=2)   # two steps per pass, masked tiles included
    b.step(77)
    b.close()
    for g, want in zip(gs, singles):
        got = g.get_state()
        g.close()
        for u, v in zip(got, want):
            assert np.array_equal(u, v)


def test_masked_diagnostics_skip_solid_nodes(ctx):
    from paper_1902_02999_amd import mlb
    spec = masked_spec(70, 45, 1)
    state = seeded(spec, 1, solid_h=-1.0)   # dry SOLID nodes: not counted as bad
    g = mlb.grid_from_spec(ctx, spec)
    g.set_state(*state)
    g.step(9)
    h0, qx0, qy0 = g.get_state()
    g.step(1)
    d = g.diag()
    h1, qx1, qy1 = g.get_state()
    ok, dd = g.run_steady(0.0, 10, 10)
    g.close()
    ref = oracle_from_spec(spec, h1, qx1, qy1)
    r = ref.diag(qx0, qy0)
    say("gpu", d, "oracle", r)
    assert d["nonfinite"] == 0 and dd["nonfinite"] == 0
    assert d["mass"] == pytest.approx(r["mass"], rel=1e-9)
    assert d["residual"] == pytest.approx(r["residual"], rel=1e-6)
    assert d["max_speed"] == pytest.approx(r["max_speed"], rel=1e-6)


def test_mask_argument_errors(ctx):
    from paper_1902_02999_amd import mlb
    spec = masked_spec(40, 30, 2)
    g = mlb.grid_from_spec(ctx, spec)
    bad = spec.kind.copy()
    bad[5, 5] = 3
    with pytest.raises(mlb.MlbError):
        g.set_mask(bad)
    with pytest.raises(mlb.MlbError):
        g.set_mask(np.full((30, 40), wl.SOLID, np.uint8))
    b = mlb.Batch(ctx, [g])
    with pytest.raises(mlb.MlbError):
        g.set_mask(spec.kind)
    b.close()
    g.close()
    ch = wl.bump_channel(60, 20)
    ch.extrap_order = 2
    g = mlb.grid_from_spec(ctx, ch)
    k = np.zeros((20, 60), np.uint8)
    k[10, 2] = wl.SOLID          # within two nodes of the inflow edge
    with pytest.raises(mlb.MlbError):
        g.set_mask(k)
    k[10, 2] = 0
    k[10, 3] = wl.SOLID
    g.set_mask(k)
    g.close()
    net = mlb.Net(ctx, 64, 64, base_ch=32, levels=2, in_ch=32, max_batch=1, seed=1)
    g = mlb.grid_from_spec(ctx, masked_spec(64, 64, 2))
    with pytest.raises(mlb.MlbError):
        net.infer(g)
    with pytest.raises(mlb.MlbError):
        net.warm_start_run(g, 1e-6, 100, 10)
    g.close()
    net.close()


def islands_channel():
    spec = wl.bump_channel(180, 60, sigma=10.0)
    Y, X = np.mgrid[0:60, 0:180].astype(float)
    inside = ((X - 70) ** 2 + (Y - 25) ** 2 > 36) & ((X - 120) ** 2 + (Y - 40) ** 2 > 20)
    inside &= ~((X >= 95) & (X < 98) & (Y < 22))
    spec.kind = wl.staircase_kinds(np.pad(inside[1:-1, 3:-3], ((1, 1), (3, 3)), constant_values=True))
    spec.kind[0, :] = wl.FLUID
    spec.kind[-1, :] = wl.FLUID
    spec.kind[:, :3] = wl.FLUID
    spec.kind[:, -3:] = wl.FLUID
    return spec


@pytest.mark.parametrize("case", ["basin", "periodic", "islands_channel", "dish", "narrow"])
def test_masked_two_step_passes_bitwise(ctx, case):
    """Two steps per pass on masked grids (the kinds travel with the first
    stage's rows to the second) give the one-step result bit for bit, for
    odd step counts, several tile heights and with open edges."""
    if case == "basin":
        spec, state = masked_spec(150, 80, 7), None
    elif case == "periodic":
        spec, state = masked_spec(96, 50, 6, edges=(wl.PERIODIC,) * 4, omega=1e-3), None
    elif case == "islands_channel":
        spec, state = islands_channel(), None
    elif case == "dish":
        spec, state = wl.circular_dish(), None
    else:
        spec, state = masked_spec(20, 133, 3), None
    state = seeded(spec, 5, solid_h=-2.0) if case in ("basin", "periodic", "narrow") else spec.initial()
    one = run_gpu(ctx, spec, 211, state, dict(tile_rows=15, tblock=1))
    for tr in (8, 17, 44):
        two = run_gpu(ctx, spec, 211, state, dict(tile_rows=tr, tblock=2))
        say(case, "two-step tile rows", tr)
        for u, v in zip(one, two):
            assert np.array_equal(u, v)


# ----------------------------------------------------------------------------- the paper's geometries
def test_dish_steady_gyres_at_paper_size(ctx):
    """Section 4's wind-driven basin (200 x 200, dx = 2 m, nu = 5.33 m^2/s,
    5 m/s wind from the south-west): the steady state has flow with the wind
    over the shallow margins and against it over the deep centre along the
    cross-wind diagonal, keeps its volume, and is symmetric about x = y."""
    from paper_1902_02999_amd import mlb
    spec = wl.circular_dish()
    g = mlb.grid_from_spec(ctx, spec)
    m0 = g.diag()["mass"]
    ok, d = g.run_steady(1e-6, 3_000_000, 2000)
    h, qx, qy = g.get_state()
    g.close()
    say("dish steady", ok, d["step"], d["residual"], d["max_speed"])
    assert ok
    assert abs(d["mass"] - m0) <= 1e-6 * m0
    water = spec.kind != wl.SOLID
    dh, du = compare(h, qx, qy, h.T, qy.T, qx.T, where=water)
    say("transpose asymmetry", dh, du)
    assert dh <= H_TOL and du <= 1e-3
    n = spec.nx
    i = np.arange(n)
    j = n - 1 - i
    s = ((qx[j, i] + qy[j, i]) / h[j, i])[water[j, i]]
    m = len(s)
    say("along-wind velocity on the cross-wind diagonal", np.round(s[::8] * 1e3, 3))
    assert s[m // 2 - 1] < 0 and s[m // 2] < 0
    assert s[2:m // 5].min() > 0 and s[-m // 5:-2].min() > 0


def test_hump_steady_flow(ctx):
    """Section 4's hump channel (200 x 200, dx = 5 m, q = 10 m^2/s in, h = 10 m
    out): at the steady state every cross-section carries the inflow, and the
    subcritical surface dips over the hump."""
    from paper_1902_02999_amd import mlb
    spec = wl.hump_channel()
    g = mlb.grid_from_spec(ctx, spec)
    ok, d = g.run_steady(1e-6, 2_000_000, 2000)
    h, qx, qy = g.get_state()
    g.close()
    say("hump steady", ok, d["step"], d["residual"], d["max_speed"])
    assert ok
    flux = qx[1:-1, :].sum(axis=0) / (spec.ny - 2)   # per unit width, wall rows excluded
    say("section discharge min/max", flux.min(), flux.max())
    assert np.abs(flux - 10.0).max() <= 0.02 * 10.0
    zeta = h + spec.zb
    c = spec.nx // 2
    assert zeta[c, int(400 / spec.dx)] < zeta[c, int(200 / spec.dx)]
