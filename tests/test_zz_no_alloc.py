"""The allocation-free diagnostics entry point (mlb_diag_noalloc) against
mlb_diag, through the C ABI: two calls in a row, the second on a smaller grid
(the fixed scratch array keeps the first call's partial sums), each for a
state just set (the state reduction through the scratch array) and after
steps (the sums the last checked pass kept); and the size limit."""
import ctypes as C

import numpy as np
import pytest

from paper_1902_02999_amd import workloads as wl

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def _read(out):
    from paper_1902_02999_amd import mlb
    return mlb.Diag.from_buffer_copy(out.cpu().numpy().tobytes()).as_dict()


def _pair(ctx, spec, state):
    """Two grids with the same problem and state."""
    from paper_1902_02999_amd import mlb
    gs = []
    for _ in range(2):
        g = mlb.grid_from_spec(ctx, spec)
        g.set_state(*state)
        g.set_exec_opts(tblock=2, tile_rows=17)
        gs.append(g)
    return gs


def _specs():
    nx, ny = 700, 530
    X, Y = np.meshgrid(np.arange(nx), np.arange(ny))
    zb = 0.3 * np.exp(-((X - 300.0) ** 2 + (Y - 200.0) ** 2) / (2 * 60.0 ** 2))
    inside = (X - nx / 2) ** 2 / (0.45 * nx) ** 2 + (Y - ny / 2) ** 2 / (0.45 * ny) ** 2 <= 1.0
    big = wl.Spec("masked_700x530", nx, ny, 1.0, 10.0 / 6.0, zb, 2.0, wind_speed=(8.0, -3.0), chezy=45.0,
                  kind=wl.staircase_kinds(inside))
    small = wl.bump_channel(130, 90, sigma=9.0)
    return [big, small]


def test_noalloc_diag_equals_mlb_diag_on_two_calls():
    import torch
    from paper_1902_02999_amd import mlb
    ctx = mlb.Context(0)
    out = torch.zeros(C.sizeof(mlb.Diag), dtype=torch.uint8, device="cuda")
    try:
        for k, spec in enumerate(_specs()):   # the second call has the smaller grid
            state = wl.seeded_state(spec, 3 + k, eta_amp=0.05, q_amp=0.1)
            ga, gb = _pair(ctx, spec, state)
            # just set: the state reduction, its partials in the scratch array
            say("noalloc, state just set:", spec.name)
            torch.cuda.synchronize()
            ga.diag_noalloc(out)
            ctx.sync()
            a, b = _read(out), gb.diag()
            for key in ("step", "nonfinite", "max_speed", "residual", "e", "dt", "gh_over_e2", "rle", "t"):
                assert a[key] == b[key], key
            assert a["mass"] == pytest.approx(b["mass"], rel=1e-13)
            assert a["residual"] == 0.0 and a["max_speed"] > 0
            # after steps: the sums of the closing checked pass, bit for bit
            for n in (37, 12):
                say("noalloc after", n, "steps:", spec.name)
                ga.step(n)
                gb.step(n)
                ga.diag_noalloc(out)
                ctx.sync()
                a, b = _read(out), gb.diag()
                assert a == b
                assert a["residual"] > 0 and a["step"] == 37 + (12 if n == 12 else 0)
            # mlb_diag on the grid the entry point served agrees with it
            assert ga.diag() == a
            for g in (ga, gb):
                g.close()
    finally:
        ctx.close()


def test_noalloc_diag_rejects_grids_beyond_its_array():
    import torch
    from paper_1902_02999_amd import mlb
    ctx = mlb.Context(0)
    out = torch.zeros(C.sizeof(mlb.Diag), dtype=torch.uint8, device="cuda")
    try:
        # 128 x 129 tiles of 64 x 64 nodes: one row of tiles too many
        spec = wl.Spec("flat_8192x8256", 8192, 8256, 1.0, 10.0 / 6.0, np.zeros((8256, 8192)), 1.0)
        say("noalloc size limit:", spec.name)
        g = mlb.grid_from_spec(ctx, spec)
        with pytest.raises(mlb.MlbError) as ei:
            g.diag_noalloc(out)
        assert ei.value.name == "MLB_E_INVAL" and "16384" in str(ei.value)
        g.close()
        spec = wl.Spec("flat_8192x8192", 8192, 8192, 1.0, 10.0 / 6.0, np.zeros((8192, 8192)), 1.0)   # 16384 tiles
        say("noalloc at the limit:", spec.name)
        g = mlb.grid_from_spec(ctx, spec)
        g.diag_noalloc(out)
        ctx.sync()
        a = _read(out)
        assert a["nonfinite"] == 0 and a["residual"] == 0.0
        assert a["mass"] == pytest.approx(8192 * 8192 * 1.0, rel=1e-12)   # flat bed one metre down
        g.close()
    finally:
        ctx.close()
