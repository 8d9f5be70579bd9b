"""Host state hand-over through the C-ABI on grids large enough for the
library's threaded conversion: set then get returns the state as stored
(FP32 perturbation, or the exact pair of the compensated surface), a caller
pitch larger than nx is honoured on both sides and leaves the padding alone,
and missing discharge arrays mean zero discharge."""
import ctypes as C
import sys

import numpy as np
import pytest

from paper_1902_02999_amd import workloads as wl

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_1902_02999_amd import mlb
    c = mlb.Context(0)
    yield c
    c.close()


def _ptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


@pytest.mark.parametrize("nx,ny,comp", [(1000, 700, False), (777, 1001, True), (1024, 513, False)])
def test_round_trip(ctx, nx, ny, comp):
    from paper_1902_02999_amd import mlb
    say("round trip", nx, ny, "compensated" if comp else "fp32")
    spec = wl.bump_channel(nx, ny, sigma=50.0)
    spec.compensated = comp
    g = mlb.grid_from_spec(ctx, spec)
    try:
        rng = np.random.Generator(np.random.PCG64(nx + ny))
        H = spec.initial()[0]
        h0 = H + 0.01 * rng.standard_normal((ny, nx))
        qx = rng.standard_normal((ny, nx))
        qy = rng.standard_normal((ny, nx))
        g.set_state(h0, qx, qy)
        h, a, b = g.get_state()
        assert np.array_equal(a, qx.astype(np.float32).astype(np.float64))
        assert np.array_equal(b, qy.astype(np.float32).astype(np.float64))
        # FP32: the perturbation h - H rounded once; compensated: an exact pair
        err = np.abs(h - h0).max()
        bound = 1e-14 if comp else np.abs(h0 - H).max() * 2.0 ** -24 * 1.01 + 1e-15
        assert err <= bound, err
    finally:
        g.close()


def test_caller_pitch_and_missing_discharge(ctx):
    from paper_1902_02999_amd import mlb
    nx, ny, ld = 900, 600, 1037
    spec = wl.bump_channel(nx, ny, sigma=40.0)
    g = mlb.grid_from_spec(ctx, spec)
    try:
        rng = np.random.Generator(np.random.PCG64(3))
        H = spec.initial()[0]
        hbuf = np.full((ny, ld), -7.0)
        hbuf[:, :nx] = H + 0.02 * rng.standard_normal((ny, nx))
        ubuf = np.full((ny, ld), -7.0)
        ubuf[:, :nx] = rng.standard_normal((ny, nx))
        lib = mlb.lib()
        # hu from the pitched buffer, hv absent (zero)
        assert lib.mlb_set_state(g.h, _ptr(hbuf), _ptr(ubuf), None, ld, 0) == 0
        out_h = np.full((ny, ld), 5.0)
        out_u = np.full((ny, ld), 5.0)
        out_v = np.full((ny, ld), 5.0)
        assert lib.mlb_get_state(g.h, _ptr(out_h), _ptr(out_u), _ptr(out_v), ld) == 0
        assert np.all(out_h[:, nx:] == 5.0) and np.all(out_u[:, nx:] == 5.0) and np.all(out_v[:, nx:] == 5.0)
        assert np.array_equal(out_u[:, :nx], ubuf[:, :nx].astype(np.float32).astype(np.float64))
        assert np.all(out_v[:, :nx] == 0.0)
        assert np.abs(out_h[:, :nx] - hbuf[:, :nx]).max() < 1e-8
        # the same state read back with the binding's dense arrays
        h, a, b = g.get_state()
        assert np.array_equal(h, out_h[:, :nx]) and np.array_equal(a, out_u[:, :nx])
        # a pitch below nx is refused
        assert lib.mlb_get_state(g.h, _ptr(out_h), _ptr(out_u), _ptr(out_v), nx - 1) != 0
        assert lib.mlb_set_state(g.h, _ptr(hbuf), None, None, nx - 1, 0) != 0
    finally:
        g.close()
