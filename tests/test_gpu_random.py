"""Randomised configurations on the GPU against the FP64 oracle.

Forty seeded draws of grid shape (4 to 150 nodes a side, ragged against the
tile sizes), edge kinds (walls, periodic pairs, or one open axis with a depth
and a discharge edge), node mask, implicit link depth, compensated surface,
forcing, tile height and steps per pass.  Each draw must meet the parity bar
against the oracle, and its two-step passes must give the bits of one-step
passes.  The draws cover combinations no hand-written case lists: masks with
periodic edges, the implicit link depth on narrow open channels, tile heights
that leave ragged last bands, and so on.
"""
import copy
import sys

import numpy as np
import pytest

from helpers import compare, oracle_from_spec
from paper_1902_02999_amd import workloads as wl

pytestmark = pytest.mark.gpu

H_TOL, U_TOL = 1e-5, 1e-4
DRAWS = 40


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_1902_02999_amd import mlb
    c = mlb.Context(0)
    yield c
    c.close()


def draw(i):
    rng = np.random.Generator(np.random.PCG64(7000 + i))
    layout = rng.choice(["walls", "periodic", "periodic_x", "open_x", "open_y"])
    lo = 5 if layout.startswith("open") else 4
    nx, ny = int(rng.integers(lo, 151)), int(rng.integers(lo, 101))
    X, Y = np.meshgrid(np.arange(nx), np.arange(ny))
    zb = np.zeros((ny, nx))
    for _ in range(2):
        cx, cy, s = rng.uniform(0, nx), rng.uniform(0, ny), rng.uniform(2.0, max(3.0, nx / 4))
        zb += rng.uniform(0.0, 0.3) * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2 * s * s))
    W, P, D, Q = wl.WALL, wl.PERIODIC, wl.DEPTH, wl.DISCHARGE
    depth_bc, discharge_bc = {}, {}
    if layout == "walls":
        edges = (W, W, W, W)
    elif layout == "periodic":
        edges = (P, P, P, P)
    elif layout == "periodic_x":
        edges = (P, P, W, W)
    elif layout == "open_x":
        edges = (Q, D, W, W) if rng.random() < 0.5 else (Q, D, P, P)
        discharge_bc[wl.W] = (float(rng.uniform(0.05, 0.4)), 0.0)
        depth_bc[wl.E] = (2.0, float(rng.uniform(0.0, 0.02)), 40.0, 0.0)
    else:
        edges = (W, W, Q, D) if rng.random() < 0.5 else (P, P, Q, D)
        discharge_bc[wl.S] = (0.0, float(rng.uniform(0.05, 0.4)))
        depth_bc[wl.N] = (2.0, float(rng.uniform(0.0, 0.02)), 40.0, 0.0)
    kind = None
    if layout in ("walls", "periodic", "periodic_x") and nx >= 12 and ny >= 12 and rng.random() < 0.35:
        kind = wl.random_geometry(rng, nx, ny, holes=int(rng.integers(0, 4)))
    spec = wl.Spec("draw%02d_%s_%dx%d" % (i, layout, nx, ny), nx, ny, 1.0, 10.0 / 6.0, zb, 2.0, edges=edges,
                   extrap_order=int(rng.integers(1, 3)), depth_bc=depth_bc, discharge_bc=discharge_bc,
                   wind_speed=(float(rng.uniform(-12, 12)), float(rng.uniform(-12, 12))),
                   chezy=float(rng.choice([0.0, 40.0, 60.0])), omega=float(rng.choice([0.0, 1e-3])), kind=kind)
    spec.hbar_implicit = bool(rng.random() < 0.25)
    spec.compensated = bool(rng.random() < 0.2)
    closed_state = layout in ("walls", "periodic", "periodic_x")
    state = wl.seeded_state(spec, 100 + i, eta_amp=0.05, q_amp=0.1) if closed_state else None
    if state is not None and kind is not None:
        h, qx, qy = state
        solid = kind == wl.SOLID
        state = (np.where(solid, spec.H, h), np.where(solid, 0.0, qx), np.where(solid, 0.0, qy))
    rows = int(rng.choice([4, 5, 8, 9, 14, 17, 26]))
    steps = int(rng.integers(15, 61))
    return spec, state, rows, steps


CASES = [draw(i) for i in range(DRAWS)]


def run_gpu(ctx, spec, steps, state, opts):
    from paper_1902_02999_amd import mlb
    g = mlb.grid_from_spec(ctx, spec)
    if state is not None:
        g.set_state(*state)
    g.set_exec_opts(**opts)
    g.step(steps)
    out = g.get_state()
    g.close()
    return out


@pytest.mark.parametrize("case", CASES, ids=[c[0].name for c in CASES])
def test_random_configuration(ctx, case):
    spec, state, rows, steps = case
    say("draw", spec.name, "rows", rows, "steps", steps, "implicit", spec.hbar_implicit,
        "compensated", spec.compensated, "mask", spec.kind is not None)
    one = run_gpu(ctx, spec, steps, state, dict(tile_rows=rows, tblock=1))
    two = run_gpu(ctx, spec, steps, state, dict(tile_rows=rows, tblock=2, use_graph=True, graph_chunk=8))
    for a, b in zip(one, two):
        assert np.array_equal(a, b)
    ref = oracle_from_spec(spec, *(state if state is not None else spec.initial()))
    ref.run(steps)
    where = None if spec.kind is None else spec.kind != wl.SOLID
    dh, du = compare(*one, ref.h, ref.qx, ref.qy, where=where)
    say("dh", dh, "du", du)
    assert dh <= H_TOL and du <= U_TOL


def _plain(spec):
    s = copy.copy(spec)
    s.hbar_implicit = False
    s.compensated = False
    return s


@pytest.mark.parametrize("group", range(4))
def test_random_batches_bitwise(ctx, group):
    """Ten of the draws (old-time link depth, FP32 surface) in one batch give
    the bits of each basin run on its own.  A batch holding an open or a
    masked basin launches the general or masked kernel for every basin, while
    a closed, unmasked basin on its own takes the kernel without open-edge
    logic, so this also checks that the kernel variants agree bit for bit."""
    from paper_1902_02999_amd import mlb
    members = CASES[10 * group:10 * group + 10]
    rows = (5, 9, 14, 17)[group]
    steps = 24
    opts = dict(tile_rows=rows, tblock=2, use_graph=True, graph_chunk=8)
    say("batch group", group, "rows", rows, [c[0].name for c in members])
    specs = [_plain(c[0]) for c in members]
    solo = [run_gpu(ctx, s, steps, c[1], opts) for s, c in zip(specs, members)]
    grids = []
    for s, c in zip(specs, members):
        g = mlb.grid_from_spec(ctx, s)
        if c[1] is not None:
            g.set_state(*c[1])
        grids.append(g)
    b = mlb.Batch(ctx, grids)
    b.set_exec_opts(**opts)
    b.step(steps)
    b.close()
    for g, ref, s in zip(grids, solo, specs):
        for a, r in zip(g.get_state(), ref):
            assert np.array_equal(a, r), s.name
        g.close()
