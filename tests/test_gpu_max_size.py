"""The largest grid the library accepts, on the GPU.

A field plane is addressed with 32-bit byte offsets, so the padded plane must
hold fewer than 2^30 values: a 32768 x 32704 periodic grid is within 0.2 % of
that limit and puts byte offsets near 2^32.  Its state is a 64 x 64 periodic
pattern tiled 512 x 511 times, so after any number of steps it must still be
that pattern, bit for bit equal to the 64 x 64 periodic grid run on its own
(every node's update is the same arithmetic on the same values); the small
grid is checked against the FP64 oracle in the same test.  Both the two-step
pass of the benchmark's launch configuration and the one-step pass with ragged
row tiles are checked.
"""
import sys

import numpy as np
import pytest

from helpers import compare, oracle_from_spec
from paper_1902_02999_amd import workloads as wl

pytestmark = pytest.mark.gpu

P = 64                       # period of the pattern
NX, NY = 32768, 32704        # 512 x 511 periods; pitch x ny = 1 071 644 672 < 2^30
STEPS = 40


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def small_spec():
    x = np.arange(P) * 2 * np.pi / P
    X, Y = np.meshgrid(x, x)
    zb = 0.3 * np.sin(X) * np.cos(2 * Y) + 0.2 * np.cos(3 * X + Y)
    return wl.Spec("periodic_pattern_64", P, P, 1.0, 10.0 / 6.0, zb, 2.0, edges=(wl.PERIODIC,) * 4,
                   wind_speed=(9.0, -4.0), chezy=45.0, omega=1e-3)


def test_max_size_grid_is_the_tiled_small_grid():
    import torch
    from paper_1902_02999_amd import mlb
    spec = small_spec()
    state = wl.seeded_state(spec, 11, eta_amp=0.05, q_amp=0.1)
    ctx = mlb.Context(0)
    dev = torch.device("cuda", 0)

    # the small periodic grid, against the oracle
    gs = mlb.grid_from_spec(ctx, spec)
    gs.set_state(*state)
    f0 = [torch.empty((P, P), device=dev) for _ in range(3)]
    gs.get_state_device(*f0)
    gs.step(STEPS)
    got = gs.get_state()
    f1 = [torch.empty((P, P), device=dev) for _ in range(3)]
    gs.get_state_device(*f1)
    mass_small = gs.diag()["mass"]
    ctx.sync()
    gs.close()
    ref = oracle_from_spec(spec, *state)
    ref.run(STEPS)
    dh, du = compare(*got, ref.h, ref.qx, ref.qy)
    say("64 x 64 periodic vs oracle after", STEPS, "steps: dh", dh, "du", du)
    assert dh <= 1e-5 and du <= 1e-4

    # the same pattern on the largest grid
    p = mlb.make_params(NX, NY, spec.dx, spec.nu, spec.zeta_ref, spec.edges, omega=spec.omega)
    say("creating the", NX, "x", NY, "grid")
    g = mlb.Grid(ctx, p)
    try:
        g.set_bathymetry(np.tile(spec.zb, (NY // P, NX // P)))
        g.set_wind(*spec.wind_speed)
        g.set_chezy(spec.chezy)
        reps = (NY // P, NX // P)
        for opts in (dict(tblock=2, tile_rows=17, blocks_per_cu=3), dict(tblock=1, tile_rows=9, blocks_per_cu=0)):
            big = [f.tile(reps) for f in f0]
            g.set_state_device(*big)
            del big
            g.set_exec_opts(use_graph=True, graph_chunk=20, **opts)
            say("max size", opts, "stepping", STEPS)
            g.step(STEPS)
            d = g.diag()
            assert d["nonfinite"] == 0
            # FP64 sums over 5.3e5 copies of the small grid, in another order
            assert d["mass"] == pytest.approx(mass_small * reps[0] * reps[1], rel=1e-9)
            for k, name in enumerate(("eta", "qx", "qy")):
                out = torch.empty((NY, NX), device=dev)
                args = [None, None, None]
                args[k] = out
                g.get_state_device(*args)
                ctx.sync()
                diff = int((out.view(reps[0], P, reps[1], P) != f1[k].view(1, P, 1, P)).sum().item())
                say("  ", name, "nodes differing from the small grid:", diff)
                assert diff == 0
                del out
    finally:
        g.close()
        ctx.close()
