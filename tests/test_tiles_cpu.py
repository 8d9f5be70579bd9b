"""Host logic of the tile plans (no GPU): every node is stored by exactly one
wave, windows stay inside the grid, two-step tiles never start at row 1, and
with a node mask the masked flag and the dropped tiles match a brute-force
reading of each tile's window."""
import numpy as np
import pytest

from paper_1902_02999_amd import mlb, workloads as wl

STRIP = {1: 62, 2: 60}


def owned(t, tb, nx):
    x0, y0, rows, xo, yo, _ = t
    xs = range(max(x0, xo), min(x0 + STRIP[tb], nx))
    ys = range(yo, y0 + rows)
    return xs, ys


def window(t, tb, nx, ny, px, py):
    x0, y0, rows = t[0], t[1], t[2]
    k = tb
    cols = [c % nx if px else min(max(c, 0), nx - 1) for c in range(x0 - k, x0 - k + 64)]
    rws = [r % ny if py else min(max(r, 0), ny - 1) for r in range(y0 - k, y0 + rows + k)]
    return cols, rws


CASES = [(100, 50, (wl.WALL,) * 4), (4, 133, (wl.WALL,) * 4), (300, 7, (wl.PERIODIC,) * 4),
         (61, 62, (wl.DISCHARGE, wl.DEPTH, wl.WALL, wl.WALL)), (123, 77, (wl.PERIODIC, wl.PERIODIC, wl.DEPTH, wl.WALL)),
         (5, 5, (wl.WALL,) * 4), (200, 200, (wl.WALL,) * 4)]


@pytest.mark.parametrize("nx,ny,edges", CASES)
@pytest.mark.parametrize("tb", [1, 2])
def test_every_node_stored_once(nx, ny, edges, tb):
    p = mlb.make_params(nx, ny, 1.0, 1.0, 2.0, edges)
    for rows in (4, 5, 6, 9, 14, 17, 44):
        t = mlb.plan_tiles(p, rows, tb)
        count = np.zeros((ny, nx), int)
        for tile in t:
            xs, ys = owned(tile, tb, nx)
            for y in ys:
                count[y, list(xs)] += 1
            x0, y0, r = tile[0], tile[1], tile[2]
            assert x0 >= 0 and (x0 + STRIP[tb] <= nx or x0 == 0)
            assert y0 >= 0 and y0 + r <= ny and r >= 1
            assert tile[5] == 0
            if tb == 2:
                assert y0 != 1
        assert (count == 1).all(), (rows, np.argwhere(count != 1)[:5])


@pytest.mark.parametrize("tb", [1, 2])
@pytest.mark.parametrize("seed,nx,ny,edges", [(1, 130, 67, (wl.WALL,) * 4), (2, 96, 50, (wl.PERIODIC,) * 4),
                                              (3, 200, 200, (wl.WALL,) * 4), (4, 20, 133, (wl.WALL,) * 4)])
def test_masked_plans_match_brute_force(tb, seed, nx, ny, edges):
    kind = wl.random_geometry(np.random.Generator(np.random.PCG64(seed)), nx, ny, holes=4)
    if seed == 3:
        kind = wl.circular_dish().kind
    px = py = edges[0] == wl.PERIODIC
    p = mlb.make_params(nx, ny, 1.0, 1.0, 2.0, edges)
    for rows in (4, 5, 9, 17):
        t = mlb.plan_tiles(p, rows, tb, kind)
        full = mlb.plan_tiles(p, rows, tb)
        count = np.zeros((ny, nx), int)
        for tile in t:
            xs, ys = owned(tile, tb, nx)
            sub = kind[np.ix_(list(ys), list(xs))]
            assert (sub != wl.SOLID).any()                 # kept tiles own water
            for y in ys:
                count[y, list(xs)] += 1
            cols, rws = window(tile, tb, nx, ny, px, py)
            masked = (kind[np.ix_(rws, cols)] != wl.FLUID).any()
            assert bool(tile[5] & 1) == masked
        water = kind != wl.SOLID
        assert (count[water] == 1).all()
        assert (count[~water] <= 1).all()
        # the dropped tiles are exactly those owning only SOLID nodes
        kept = {tuple(x[:5]) for x in t}
        for tile in full:
            xs, ys = owned(tile, tb, nx)
            all_solid = (kind[np.ix_(list(ys), list(xs))] == wl.SOLID).all()
            assert (tuple(tile[:5]) not in kept) == all_solid


def test_plan_argument_errors():
    p = mlb.make_params(50, 40, 1.0, 1.0, 2.0)
    with pytest.raises(mlb.MlbError):
        mlb.plan_tiles(p, 3, 1)
    with pytest.raises(mlb.MlbError):
        mlb.plan_tiles(p, 9, 3)
    bad = np.zeros((40, 50), np.uint8)
    bad[3, 3] = 7
    with pytest.raises(mlb.MlbError):
        mlb.plan_tiles(p, 9, 1, bad)


def test_size_limit_is_the_plane_addressing_limit():
    """A field plane is addressed with 32-bit byte offsets: nx rounded up to
    64, times ny, must stay below 2^30 nodes."""
    ok = [(32768, 32767), (32769, 32704), (32704, 32831), (1 << 20, 1023)]
    bad = [(32768, 32768), (32769, 32705), (32705, 32769), (1 << 20, 1024), (1 << 30, 4)]
    for nx, ny in ok:
        assert ((nx + 63) // 64 * 64) * ny < (1 << 30)
        t = mlb.plan_tiles(mlb.make_params(nx, ny, 1.0, 1.0, 2.0), 4096, 2)
        assert len(t) > 0
    for nx, ny in bad:
        assert ((nx + 63) // 64 * 64) * ny >= (1 << 30)
        with pytest.raises(mlb.MlbError, match="too large"):
            mlb.plan_tiles(mlb.make_params(nx, ny, 1.0, 1.0, 2.0), 4096, 2)


@pytest.mark.parametrize("tb", [1, 2])
def test_costly_tiles_are_dispatched_first(tb):
    """Edge and masked tiles lead the list (they overlap the pass instead of
    forming its tail); each group keeps band order."""
    k, strip = tb, STRIP[tb]
    for nx, ny, edges, kind in ((300, 170, (wl.WALL,) * 4, None),
                                (200, 200, (wl.WALL,) * 4, wl.circular_dish().kind),
                                (130, 90, (wl.PERIODIC,) * 4, None)):
        p = mlb.make_params(nx, ny, 1.0, 1.0, 2.0, edges)
        t = mlb.plan_tiles(p, 9, tb, kind)
        per = edges[0] == wl.PERIODIC
        costly = [bool(x[5] & 1) or (not per and (x[0] < k or x[0] + strip + k > nx or x[1] < k
                                                   or x[1] + x[2] + k > ny)) for x in t]
        n = sum(costly)
        assert all(costly[:n]) and not any(costly[n:])
        for part in (t[:n], t[n:]):
            keys = [(x[4], x[3]) for x in part]       # (band, strip) in list order
            assert keys == sorted(keys)
        if per:
            assert n == 0


def _wq_brute_force(t, tb, nx, ny, px, py):
    """Dependency sets of the work queue from a node-level owner map: D(t) =
    {t} + tiles owning a node of t's window + tiles whose window holds a node
    t owns."""
    owner = -np.ones((ny, nx), int)
    for i, tile in enumerate(t):
        xs, ys = owned(tile, tb, nx)
        for y in ys:
            owner[y, list(xs)] = i
    reads = []
    for tile in t:
        cols, rws = window(tile, tb, nx, ny, px, py)
        u = owner[np.ix_(sorted(set(rws)), sorted(set(cols)))]
        reads.append(set(int(v) for v in np.unique(u) if v >= 0))
    dep = [{i} | r for i, r in enumerate(reads)]
    for i, r in enumerate(reads):
        for u in r:
            dep[u].add(i)
    return dep


@pytest.mark.parametrize("tb", [1, 2])
@pytest.mark.parametrize("nx,ny,edges,masked", [
    (200, 130, (wl.WALL,) * 4, False), (300, 7, (wl.PERIODIC,) * 4, False), (5, 5, (wl.WALL,) * 4, False),
    (61, 62, (wl.DISCHARGE, wl.DEPTH, wl.WALL, wl.WALL), False), (130, 121, (wl.PERIODIC,) * 4, False),
    (123, 77, (wl.PERIODIC, wl.PERIODIC, wl.DEPTH, wl.WALL), False), (64, 200, (wl.WALL,) * 4, False),
    (150, 96, (wl.WALL,) * 4, True), (121, 90, (wl.PERIODIC,) * 4, True)])
def test_workqueue_dependencies_match_brute_force(tb, nx, ny, edges, masked):
    """The work queue's dependency lists are exactly the brute-force sets:
    every tile whose owned nodes a tile reads, and every tile reading what it
    owns (so no item overwrites what a pass still reads, nor reads before the
    previous pass wrote), ascending, the tile itself included."""
    p = mlb.make_params(nx, ny, 1.0, 1.0, 2.0, edges)
    kind = wl.random_geometry(np.random.default_rng(nx + ny), nx, ny) if masked else None
    if kind is not None and edges[0] == wl.PERIODIC:
        kind = np.where(kind == wl.SOLID, wl.SOLID, wl.FLUID).astype(np.uint8)
    for rows in (4, 5, 9, 17, 26, 44):
        t = mlb.plan_tiles(p, rows, tb, kind=kind)
        off, nbr = mlb.plan_workqueue(p, rows, tb, kind=kind)
        assert off.size == len(t) + 1 and off[0] == 0 and off[-1] == nbr.size
        want = _wq_brute_force(t, tb, nx, ny, edges[0] == wl.PERIODIC, edges[2] == wl.PERIODIC)
        for i in range(len(t)):
            got = nbr[off[i]:off[i + 1]]
            assert list(got) == sorted(want[i]), (rows, i)
            assert len(got) <= 64
