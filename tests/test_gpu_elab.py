"""The eLABSWE baseline on the GPU (nine FP32 distributions per node)
against the oracle's FP64 eLABSWE, through the C ABI.

Bar on the macroscopic fields as for the streaming-only step (max |dh| <= 1e-5
max h, max |du| <= 1e-4 max |u|), after a few hundred steps, for relaxation
times below, at and above 1, on closed, periodic, staircase-masked and
island geometries.  At tau = 1 the baseline and the streaming-only step agree
to the same bar.  Tile rows do not change the result (bit for bit).
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


def islands(nx, ny):
    Y, X = np.mgrid[0:ny, 0:nx].astype(float)
    kind = np.zeros((ny, nx), np.uint8)
    kind[((X - nx / 3) ** 2 + (Y - ny / 2) ** 2 <= 9) | ((X - 2 * nx / 3) ** 2 + (Y - ny / 3) ** 2 <= 4)] = wl.SOLID
    return kind


def make_spec(case, nx, ny, seed):
    edges, kind = (wl.WALL,) * 4, None
    if case == "periodic":
        edges = (wl.PERIODIC,) * 4
    elif case == "masked":
        kind = wl.random_geometry(np.random.Generator(np.random.PCG64(seed)), nx, ny, holes=3)
    elif case == "islands":
        edges, kind = (wl.PERIODIC,) * 4, islands(nx, ny)
    return wl.Spec("%s_%dx%d" % (case, nx, ny), nx, ny, 1.0, 10.0 / 6.0, bumpy(nx, ny, seed), 2.0, edges=edges,
                   wind_speed=(8.0, -5.0), chezy=45.0, omega=1e-3, kind=kind)


def run_elab(ctx, spec, tau, steps, state, tile_rows=None):
    from paper_1902_02999_amd import mlb
    g = mlb.grid_from_spec(ctx, spec)
    g.set_state(*state)
    if tile_rows:
        g.set_exec_opts(tile_rows=tile_rows)
    el = mlb.Elab(g, tau)
    el.step(steps)
    out = el.get_state()
    el.close()
    g.close()
    return out


@pytest.mark.parametrize("case,nx,ny,tau", [("walls", 125, 70, 0.8), ("walls", 61, 9, 1.0),
                                            ("periodic", 70, 40, 1.6), ("masked", 130, 67, 1.2),
                                            ("islands", 96, 50, 0.7)])
def test_elab_parity(ctx, case, nx, ny, tau):
    import oracle
    spec = make_spec(case, nx, ny, 3)
    state = wl.seeded_state(spec, 3, eta_amp=0.05, q_amp=0.1)
    say("case", case, nx, ny, "tau", tau)
    got = run_elab(ctx, spec, tau, 300, state)
    ref = oracle.ElabBasin(oracle_from_spec(spec, *state), tau)
    ref.run(300)
    rh, rqx, rqy = ref.macro()
    where = None if spec.kind is None else spec.kind != wl.SOLID
    dh, du = compare(*got, rh, rqx, rqy, where=where)
    say("dh", dh, "du", du)
    assert dh <= H_TOL and du <= U_TOL


def test_tau_one_matches_the_streaming_only_step(ctx):
    from paper_1902_02999_amd import mlb
    spec = make_spec("walls", 150, 97, 5)
    state = wl.seeded_state(spec, 5, q_amp=0.1)
    a = run_elab(ctx, spec, 1.0, 400, state)
    g = mlb.grid_from_spec(ctx, spec)
    g.set_state(*state)
    g.step(400)
    b = g.get_state()
    g.close()
    dh, du = compare(*a, *b)
    say("elab(tau=1) vs streaming-only: dh", dh, "du", du)
    assert dh <= H_TOL and du <= U_TOL


def test_elab_tile_rows_bitwise(ctx):
    spec = make_spec("masked", 150, 80, 7)
    state = wl.seeded_state(spec, 7, q_amp=0.1)
    a = run_elab(ctx, spec, 0.9, 120, state, tile_rows=15)
    for tr in (4, 9, 40):
        b = run_elab(ctx, spec, 0.9, 120, state, tile_rows=tr)
        for u, v in zip(a, b):
            assert np.array_equal(u, v)


def test_elab_distributions_and_errors(ctx):
    import torch
    import oracle
    from paper_1902_02999_amd import mlb
    spec = make_spec("walls", 64, 40, 2)
    state = wl.seeded_state(spec, 2, q_amp=0.1)
    g = mlb.grid_from_spec(ctx, spec)
    g.set_state(*state)
    el = mlb.Elab(g, 1.3)
    with pytest.raises(mlb.MlbError):
        g.close()                   # the baseline still uses the grid
    el.step(50)
    f = torch.empty((9, 40, 64), dtype=torch.float32, device="cuda")
    el.get_dist(f)
    ctx.sync()
    ref = oracle.ElabBasin(oracle_from_spec(spec, *state), 1.3)
    ref.run(50)
    fr = ref.dist()
    err = np.abs(f.cpu().numpy() - fr).max() / np.abs(fr).max()
    say("distribution error", err)
    assert err <= 1e-5
    el.close()
    with pytest.raises(mlb.MlbError):
        mlb.Elab(g, 0.5)
    g.set_hbar(True)
    with pytest.raises(mlb.MlbError):
        mlb.Elab(g, 1.0)
    g.close()
    ch = mlb.grid_from_spec(ctx, wl.bump_channel(80, 20))
    with pytest.raises(mlb.MlbError):
        mlb.Elab(ch, 1.0)
    ch.close()
