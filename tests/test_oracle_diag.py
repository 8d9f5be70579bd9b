"""Pins of the oracle's diagnostics (mass, residual, max speed, bad count).

The paper declares its runs steady without giving a criterion (Section 4.2,
4.3: "steady solution is obtained"); the residual read from it is
R = |q_n - q_(n-1)|_2 / |q_n|_2 over both discharge components and every node
that is not SOLID, 0 when q did not change.  Mass is the sum of h dx^2 over
the same nodes; max speed is max |q| / h; the bad count is the number of
nodes with a non-finite value or h <= 0 (those are left out of the sums).

None of these re-types the oracle's sums.  Each checks a value the dynamics
or the construction fixes in closed form:
  * the flat periodic shear wave decays by exactly G = 2/3 + cos(theta)/3 per
    step (pinned in test_oracle_pins), so its residual is (1 - G) / G at
    every step, for either orientation of the wave;
  * a uniform flow has speed q / h at every node, a single fast node sets the
    maximum, and SOLID nodes (whatever they hold) change nothing;
  * planted NaN / infinite / dry nodes are counted one each and leave the
    other sums as without them;
  * uniform depth gives mass = h N dx^2 exactly.
A last test applies plausible mistakes to a copy of the oracle's C source
and checks that every one of them fails at least one of these pins.
"""
import ctypes as C
import math
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOLID = 2


def diag_fn(L):
    """mref_diag of the library L as a Python function."""
    dp = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
    L.mref_diag.argtypes = [C.c_int32, C.c_int32, C.c_double, dp, dp, dp, C.c_void_p, C.c_void_p, C.c_void_p, dp]
    L.mref_diag.restype = None

    def diag(h, qx, qy, qx0=None, qy0=None, kind=None, dx=1.0):
        ny, nx = h.shape
        h, qx, qy = (np.ascontiguousarray(a, np.float64) for a in (h, qx, qy))
        a = None if qx0 is None else np.ascontiguousarray(qx0, np.float64)
        b = None if qy0 is None else np.ascontiguousarray(qy0, np.float64)
        k = None if kind is None else np.ascontiguousarray(kind, np.uint8)
        out = np.zeros(4)
        L.mref_diag(nx, ny, dx, h, qx, qy, None if a is None else a.ctypes.data,
                    None if b is None else b.ctypes.data, None if k is None else k.ctypes.data, out)
        return {"mass": out[0], "residual": out[1], "max_speed": out[2], "bad": int(out[3])}
    return diag


# ----------------------------------------------------------------------------- pins
def pin_residual_shear_wave(diag, oracle):
    """Shear wave along either axis: R_n = (1 - G) / G exactly at every step."""
    H, U, lam, n_ax = 2.0, 1e-3, 16, 32
    G = 2.0 / 3.0 + math.cos(2 * math.pi / lam) / 3.0
    want = (1.0 - G) / G
    for axis in ("x", "y"):
        s = H * U * np.sin(2 * np.pi * np.arange(n_ax) / lam)
        if axis == "x":   # hu varies along y
            nx, ny, qx, qy = 4, n_ax, np.tile(s[:, None], (1, 4)), np.zeros((n_ax, 4))
        else:             # hv varies along x
            nx, ny, qx, qy = n_ax, 4, np.zeros((4, n_ax)), np.tile(s[None, :], (4, 1))
        b = oracle.Basin(nx, ny, 1.0, 10.0 / 6.0, np.zeros((ny, nx)), edges=(oracle.PERIODIC,) * 4,
                         h=np.full((ny, nx), H), qx=qx, qy=qy)
        for _ in range(3):
            qx0, qy0 = b.qx.copy(), b.qy.copy()
            b.run(1)
            d = diag(b.h, b.qx, b.qy, qx0, qy0)
            assert abs(d["residual"] - want) <= 1e-9 * want, (axis, d["residual"], want)
        if axis == "y":
            # the four rows are equal copies, so leaving one out keeps R; a
            # SOLID row is not water, whatever it holds and however it changed
            kind = np.zeros((ny, nx), np.uint8)
            kind[1, :] = SOLID
            jx, jy = b.qx.copy(), b.qy.copy()
            jx[1, :] = 7.0; jy[1, :] = -3.0
            d = diag(b.h, jx, jy, qx0, qy0, kind)
            assert abs(d["residual"] - want) <= 1e-9 * want, d


def pin_residual_zero_and_rest(diag, oracle):
    """No change gives R = 0 exactly (also for a basin at rest, 0 / 0)."""
    h = np.full((5, 6), 3.0)
    q = np.linspace(-1, 1, 30).reshape(5, 6)
    assert diag(h, q, 2 * q, q, 2 * q)["residual"] == 0.0
    z = np.zeros((5, 6))
    assert diag(h, z, z, z, z)["residual"] == 0.0


def pin_max_speed(diag, oracle):
    """Uniform flow: |q| / h; a single fast node sets the maximum; SOLID
    nodes with any value are ignored."""
    ny, nx = 7, 9
    h = np.full((ny, nx), 2.5)
    qx = np.full((ny, nx), 3.0)
    qy = np.full((ny, nx), -4.0)
    d = diag(h, qx, qy)
    assert abs(d["max_speed"] - 5.0 / 2.5) <= 1e-15
    h2 = h.copy(); qx2 = qx.copy(); qy2 = qy.copy()
    h2[3, 4] = 0.5; qx2[3, 4] = 6.0; qy2[3, 4] = 8.0      # speed 20 at one node
    assert abs(diag(h2, qx2, qy2)["max_speed"] - 20.0) <= 1e-14
    kind = np.zeros((ny, nx), np.uint8)
    kind[3, 4] = SOLID
    assert abs(diag(h2, qx2, qy2, kind=kind)["max_speed"] - 2.0) <= 1e-15
    # depth, not a unit depth: the same discharge over twice the depth is half as fast
    assert abs(diag(2 * h, qx, qy)["max_speed"] - 1.0) <= 1e-15


def pin_bad_count_and_mass(diag, oracle):
    """Planted non-finite and dry nodes are counted once each and left out of
    the mass and the residual; SOLID nodes are neither counted nor summed;
    uniform depth gives h N dx^2."""
    ny, nx, H, dx = 6, 10, 1.75, 2.5
    h = np.full((ny, nx), H)
    q0 = np.zeros((ny, nx))
    qx = np.full((ny, nx), 0.5)
    qy = np.zeros((ny, nx))
    d = diag(h, qx, qy, q0, q0, dx=dx)
    assert d["bad"] == 0
    assert abs(d["mass"] - H * nx * ny * dx * dx) <= 1e-12 * d["mass"]
    assert abs(d["residual"] - 1.0) <= 1e-15   # |q - 0| / |q|
    hb, xb, yb = h.copy(), qx.copy(), qy.copy()
    hb[0, 0] = np.nan          # non-finite depth
    xb[1, 2] = np.inf          # non-finite discharge
    yb[2, 3] = -np.inf
    hb[3, 4] = 0.0             # dry
    hb[4, 5] = -1.0            # negative depth
    xb[4, 5] = 1e6             # (and a huge discharge there: left out)
    kind = np.zeros((ny, nx), np.uint8)
    kind[5, :] = SOLID         # a SOLID row holding garbage
    hb[5, 7] = np.nan; xb[5, 8] = np.inf; hb[5, 9] = -5.0
    d = diag(hb, xb, yb, q0, q0, kind=kind, dx=dx)
    assert d["bad"] == 5, d
    good = nx * (ny - 1) - 5
    assert abs(d["mass"] - H * good * dx * dx) <= 1e-12 * d["mass"], d
    assert abs(d["residual"] - 1.0) <= 1e-15, d
    assert abs(d["max_speed"] - 0.5 / H) <= 1e-15, d


PINS = [pin_residual_shear_wave, pin_residual_zero_and_rest, pin_max_speed, pin_bad_count_and_mass]


@pytest.mark.parametrize("pin", PINS, ids=lambda f: f.__name__)
def test_diag_pin(oracle, pin):
    pin(diag_fn(oracle.lib()), oracle)


def test_residual_of_a_run_matches_the_shear_wave_decay(oracle):
    """Basin.run_steady stops at the first check whose residual is <= tol,
    and the residual it reports is the closed form (1 - G) / G."""
    H, U, lam = 1.0, 1e-3, 8
    G = 2.0 / 3.0 + math.cos(2 * math.pi / lam) / 3.0
    s = H * U * np.sin(2 * np.pi * np.arange(16) / lam)
    b = oracle.Basin(3, 16, 1.0, 10.0 / 6.0, np.zeros((16, 3)), edges=(oracle.PERIODIC,) * 4,
                     h=np.full((16, 3), H), qx=np.tile(s[:, None], (1, 3)))
    d = b.run_steady((1.0 - G) / G * 1.0001, 1000, 10)
    assert d is not None and b.step_index == 10
    assert abs(d["residual"] - (1.0 - G) / G) <= 1e-9 * (1.0 - G) / G


# ----------------------------------------------------------------------------- planted mistakes
MISTAKES = {
    "normalised by the old discharge": ("den += a * a + b * b;",
                                        "den += (qx0 ? qx0[x] * qx0[x] + qy0[x] * qy0[x] : a * a + b * b);"),
    "SOLID nodes counted": ("if (kind && kind[x] == NODE_SOLID) continue;", ";"),
    "h <= 0 not checked": ("|| hh <= 0.0)", ")"),
    "speed not divided by depth": ("double sp = sqrt(a * a + b * b) / hh;", "double sp = sqrt(a * a + b * b);"),
    "residual of one component": ("num += da * da + db * db;", "num += da * da;"),
    "mass without the cell area": ("mass += hh * dx * dx;", "mass += hh;"),
    "norm ratio without the root": ("sqrt(num) / sqrt(den)", "num / den"),
}


def _mutant(tmp, name, old, new):
    src = open(os.path.join(ROOT, "oracle", "maclab_ref.c")).read()
    body = re.search(r"void mref_diag\(.*?\n}\n", src, re.S)
    assert body and body.group(0).count(old) == 1, name
    mutated = src[:body.start()] + body.group(0).replace(old, new) + src[body.end():]
    path = os.path.join(tmp, "m%d.c" % abs(hash(name)))
    with open(path, "w") as f:
        f.write(mutated)
    so = path[:-2] + ".so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fPIC", "-shared", "-fopenmp",
                           "-ffp-contract=off", "-o", so, path, "-lm"])
    return C.CDLL(so)


@pytest.mark.parametrize("name", sorted(MISTAKES))
def test_planted_mistake_fails_a_pin(oracle, name):
    old, new = MISTAKES[name]
    with tempfile.TemporaryDirectory() as tmp:
        diag = diag_fn(_mutant(tmp, name, old, new))
        failed = []
        for pin in PINS:
            try:
                pin(diag, oracle)
            except AssertionError:
                failed.append(pin.__name__)
        assert failed, "no pin catches: " + name
