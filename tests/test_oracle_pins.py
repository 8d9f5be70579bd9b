"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these re-types the oracle's formulas: each checks a property the
paper states (moments of the equilibrium, Eqs. fea-0-h / fea-0-v and the
second moment the recovery in the Appendix relies on; the viscosity relation
Eq. mlb-viscosity; bounce-back no-slip; Dirichlet boundaries taken as given)
or an exact consequence of the discrete map (conservation, well-balancing,
closed-form linear modes, special cases that reduce to explicit Euler).
"""
import math

import numpy as np
import pytest

from paper_1902_02999_amd import workloads as wl

G = 9.81


def flat_periodic(o, nx, ny, dx=1.0, nu=10.0 / 6.0, **kw):
    return o.Basin(nx, ny, dx, nu, np.zeros((ny, nx)), edges=(o.PERIODIC,) * 4, **kw)


# ----------------------------------------------------------------------------- equilibrium
def test_lattice_directions(oracle):
    ex, ey, ca, lam, opp = oracle.lattice()
    vecs = set(zip(ex.tolist(), ey.tolist()))
    assert vecs == {(a, b) for a in (-1, 0, 1) for b in (-1, 0, 1)}
    # Section 3: C = 1/3, lambda = 1 on alpha = 1,3,5,7 (axis); 1/12, 1/4 on 2,4,6,8.
    for a in range(1, 9):
        axis = abs(ex[a]) + abs(ey[a]) == 1
        assert axis == (a % 2 == 1)
        # the opposite direction is the bounce-back partner
        assert ex[opp[a]] == -ex[a] and ey[opp[a]] == -ey[a]
    # Section 3 bounce-back example: at a south wall f2, f3, f4 are the unknowns,
    # i.e. the directions pointing into the fluid (north), paired with 6, 7, 8.
    assert {a for a in range(1, 9) if ey[a] > 0} == {2, 3, 4}
    assert [opp[a] for a in (2, 3, 4)] == [6, 7, 8]


@pytest.mark.parametrize("seed", range(5))
def test_feq_moments(oracle, seed):
    """Eqs. (fea-0-h), (fea-0-v): sum f = h, sum e f = h u; and the second
    moment sum e_i e_j f = g h^2/2 delta_ij + h u_i u_j used in the recovery."""
    rng = np.random.default_rng(seed)
    ex, ey, *_ = oracle.lattice()
    e = rng.uniform(5, 40)
    h = rng.uniform(0.5, 30)
    u, v = rng.uniform(-0.1, 0.1, 2) * e
    f = np.array([oracle.feq(a, G, e, h, u, v) for a in range(9)])
    cx, cy = e * ex, e * ey
    assert abs(f.sum() - h) <= 1e-13 * h
    assert abs((cx * f).sum() - h * u) <= 1e-12 * h * e
    assert abs((cy * f).sum() - h * v) <= 1e-12 * h * e
    scale = G * h * h + h * e * e
    assert abs((cx * cx * f).sum() - (G * h * h / 2 + h * u * u)) <= 1e-13 * scale
    assert abs((cy * cy * f).sum() - (G * h * h / 2 + h * v * v)) <= 1e-13 * scale
    assert abs((cx * cy * f).sum() - h * u * v) <= 1e-13 * scale


def test_params_and_forcing(oracle):
    # Eq. (mlb-viscosity): e = 6 nu / dx and dt = dx / e; the paper's tidal case
    # (dx = 7.5, nu = 31.25) has e = 25 m/s, dt = 0.3 s.
    e, dt = oracle.params_from_nu(7.5, 31.25)
    assert e == pytest.approx(25.0, rel=1e-15) and dt == pytest.approx(0.3, rel=1e-15)
    # Eq. (wind_u-stress): rho_a = 1.293, C_w = 0.0026; 10 m/s east wind.
    tx, ty = oracle.wind_stress(10.0, 0.0, rho_w=1000.0)
    assert tx == pytest.approx(1.293 * 0.0026 * 100 / 1000, rel=1e-15) and ty == 0.0
    tx, ty = oracle.wind_stress(3.0, 4.0, rho_w=1.0)
    assert math.hypot(tx, ty) == pytest.approx(1.293 * 0.0026 * 25, rel=1e-14)
    assert ty / tx == pytest.approx(4 / 3, rel=1e-14)
    # Eq. (bed-stress): C_b = g / C_z^2.
    assert oracle.bed_coeff(50.0) == pytest.approx(9.81 / 2500, rel=1e-15)


def test_tidal_boundary_formula(oracle):
    """Eq. (veri-Ini-Bc.3r): h(0,t) = 20 - 4 sin(pi (4t/86400 + 1/2))."""
    b = oracle.Basin(5, 3, 7.5, 31.25, np.zeros((3, 5)),
                     edges=(oracle.DEPTH, oracle.WALL, oracle.PERIODIC, oracle.PERIODIC),
                     depth_bc={0: (16.0, 4.0, 43200.0, math.pi / 2)})
    p = b.problem()
    for t in (0.0, 10800.0, 21600.0, 32400.0, 1234.5):
        ref = 20 - 4 * math.sin(math.pi * (4 * t / 86400 + 0.5))
        assert oracle.lib().mref_depth_bc(p, 0, t) == pytest.approx(ref, abs=1e-13)


# ----------------------------------------------------------------------------- uniform states
def test_uniform_state_is_fixed(oracle):
    b = flat_periodic(oracle, 7, 6, h=np.full((6, 7), 3.0), qx=np.full((6, 7), 0.4),
                      qy=np.full((6, 7), -0.25))
    b.run(50)
    assert np.abs(b.h - 3.0).max() <= 1e-14 * 3
    assert np.abs(b.qx - 0.4).max() <= 1e-14
    assert np.abs(b.qy + 0.25).max() <= 1e-14


def test_uniform_wind_is_explicit_euler(oracle):
    """Uniform wind on a flat periodic domain: the momentum sum reduces to
    q_{n+1} = q_n + dt tau/rho (sum C_a e_ai e_aj = e^2 delta_ij), the mass is
    unchanged (sum C_a e_a = 0)."""
    tx, ty = 2e-4, -1e-4
    b = flat_periodic(oracle, 5, 5, h=np.full((5, 5), 2.0), tx=tx, ty=ty)
    n = 200
    b.run(n)
    assert np.abs(b.h - 2.0).max() <= 1e-13
    # round-off: each step sums O(h e) terms, so allow n * eps * h * e absolute
    tol = n * 2.2e-16 * 2.0 * b.e
    assert np.abs(b.qx - n * b.dt * tx).max() <= tol
    assert np.abs(b.qy - n * b.dt * ty).max() <= tol


def test_uniform_friction_and_coriolis_is_explicit_euler(oracle):
    """Bed friction (Eq. bed-stress) and Coriolis on a uniform state: explicit
    Euler of dq/dt = -C_b u|u| + Omega (qy, -qx) (Eq. SWE-force)."""
    cb, om, h = 9.81 / 40.0 ** 2, 1e-3, 1.5
    b = flat_periodic(oracle, 4, 4, h=np.full((4, 4), h), qx=np.full((4, 4), 0.6),
                      qy=np.full((4, 4), 0.2), cb=cb, omega=om)
    qx, qy = 0.6, 0.2
    for _ in range(300):
        u, v = qx / h, qy / h
        s = math.hypot(u, v)
        qx, qy = qx + b.dt * (-cb * u * s + om * qy), qy + b.dt * (-cb * v * s - om * qx)
    b.run(300)
    assert np.abs(b.h - h).max() <= 1e-13
    assert np.abs(b.qx - qx).max() <= 1e-12
    assert np.abs(b.qy - qy).max() <= 1e-12


# ----------------------------------------------------------------------------- well-balancing, mass
def bumpy_bed(nx, ny, seed=0):
    rng = np.random.default_rng(seed)
    X, Y = np.meshgrid(np.arange(nx), np.arange(ny))
    zb = np.zeros((ny, nx))
    for _ in range(3):
        cx, cy = rng.uniform(0, nx), rng.uniform(0, ny)
        zb += rng.uniform(0.2, 0.8) * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / rng.uniform(4, 20))
    return zb


def test_lake_at_rest_over_bumps(oracle):
    """Still water over an uneven bed with walls stays at rest: the bed-slope
    term with the centred depth cancels the hydrostatic part of f^eq."""
    nx, ny = 24, 17
    zb = bumpy_bed(nx, ny)
    b = oracle.Basin(nx, ny, 1.0, 10.0 / 6.0, zb, h=2.0 - zb)
    b.run(2000)
    assert np.abs(b.qx).max() <= 1e-12 and np.abs(b.qy).max() <= 1e-12
    assert np.abs(b.h + zb - 2.0).max() <= 1e-12


def test_closed_basin_conserves_mass(oracle):
    nx, ny = 21, 18
    zb = bumpy_bed(nx, ny, 1)
    spec = wl.Spec("t", nx, ny, 1.0, 10.0 / 6.0, zb, 2.0)
    h, qx, qy = wl.seeded_state(spec, 3, eta_amp=0.1, q_amp=0.1)
    tx, ty = oracle.wind_stress(12.0, 5.0)
    b = oracle.Basin(nx, ny, 1.0, 10.0 / 6.0, zb, h=h, qx=qx, qy=qy, tx=tx, ty=ty,
                     cb=oracle.bed_coeff(40.0))
    m0 = b.diag()["mass"]
    b.run(3000)
    m1 = b.diag()["mass"]
    assert abs(m1 - m0) <= 1e-12 * m0
    assert np.abs(b.qx[:, 0]).max() == 0.0 and np.abs(b.qy[0, :]).max() == 0.0  # no-slip walls


def test_open_boundaries_keep_uniform_flow(oracle):
    """Uniform flow through a channel with a prescribed inflow discharge
    (west) and a prescribed outflow depth (east) is a fixed point: the
    Dirichlet values are imposed directly and the free variable extrapolated."""
    nx, ny, h0, q0 = 30, 6, 2.0, 0.8
    for order in (1, 2):
        b = oracle.Basin(nx, ny, 1.0, 25.0 / 6.0, np.zeros((ny, nx)),
                         edges=(oracle.DISCHARGE, oracle.DEPTH, oracle.PERIODIC, oracle.PERIODIC),
                         extrap_order=order, depth_bc={1: (h0, 0.0, 0.0, 0.0)},
                         discharge_bc={0: (q0, 0.0)},
                         h=np.full((ny, nx), h0), qx=np.full((ny, nx), q0))
        b.run(100)
        assert np.abs(b.h - h0).max() <= 1e-13
        assert np.abs(b.qx - q0).max() <= 1e-13
        assert np.abs(b.qy).max() <= 1e-13


def test_dirichlet_values_imposed(oracle):
    nx, ny = 12, 5
    zb = bumpy_bed(nx, ny, 4) * 0.3
    spec = wl.Spec("t", nx, ny, 1.0, 10.0 / 6.0, zb, 2.0)
    h, qx, qy = wl.seeded_state(spec, 5)
    b = oracle.Basin(nx, ny, 1.0, 10.0 / 6.0, zb, h=h, qx=qx, qy=qy,
                     edges=(oracle.DISCHARGE, oracle.DEPTH, oracle.WALL, oracle.WALL),
                     depth_bc={1: (2.1, 0.05, 50.0, 0.3)}, discharge_bc={0: (0.3, -0.02)})
    b.run(7)
    p = b.problem()
    hbc = oracle.lib().mref_depth_bc(p, 1, b.t)
    assert np.all(b.h[1:-1, -1] == hbc)
    assert np.all(b.qx[1:-1, 0] == 0.3) and np.all(b.qy[1:-1, 0] == -0.02)
    # corners are walls (precedence WALL > DISCHARGE > DEPTH)
    for j, i in ((0, 0), (0, nx - 1), (ny - 1, 0), (ny - 1, nx - 1)):
        assert b.qx[j, i] == 0.0 and b.qy[j, i] == 0.0
    # discharge edge: free surface copied from the inner neighbour (order 1)
    h_pre = b.step_from(b.h, b.qx, b.qy)  # next step from here
    nb = oracle.Basin(nx, ny, 1.0, 10.0 / 6.0, zb, h=b.h, qx=b.qx, qy=b.qy,
                      edges=(oracle.WALL, oracle.WALL, oracle.WALL, oracle.WALL))
    inner = nb.step_from(b.h, b.qx, b.qy)[0][1:-1, 1]  # interior update does not see edge kinds
    assert np.allclose(h_pre[0][1:-1, 0] + zb[1:-1, 0], inner + zb[1:-1, 1], rtol=0, atol=1e-13)


# ----------------------------------------------------------------------------- linear modes
def test_shear_wave_exact_decay(oracle):
    """Flat periodic shear wave u = U sin(2 pi y / lam): the discrete map gives
    hu' = (2/3) hu + (1/6)(hu(y-dx) + hu(y+dx)) exactly, so the amplitude
    decays by G = 2/3 + cos(theta)/3 per step and h stays uniform."""
    nx, ny, H, U = 4, 32, 2.0, 1e-3
    lam = 16
    y = np.arange(ny)
    q0 = H * U * np.sin(2 * np.pi * y / lam)
    b = flat_periodic(oracle, nx, ny, h=np.full((ny, nx), H), qx=np.tile(q0[:, None], (1, nx)))
    n = 120
    b.run(n)
    Gf = 2.0 / 3.0 + math.cos(2 * np.pi / lam) / 3.0
    assert np.abs(b.qx - np.tile((q0 * Gf ** n)[:, None], (1, nx))).max() <= 1e-12 * H * U
    assert np.abs(b.h - H).max() <= 1e-13 * H
    assert np.abs(b.qy).max() <= n * 2.2e-16 * H * b.e  # zero up to round-off


def test_viscosity_second_order(oracle):
    """Eq. (mlb-viscosity) and the (at least) second-order recovery (Appendix):
    at fixed nu and physical time the shear-wave amplitude tends to
    exp(-nu k^2 t).  For this mode the discrete factor G = 1 - (2/3) sin^2(theta/2)
    has ln G = -theta^2/6 + O(theta^6), so the error actually falls as dx^4."""
    nu, lamL, T = 0.5, 8.0, 6.0
    errs = []
    for ny in (16, 32, 64):
        dx = lamL / ny
        e, dt = oracle.params_from_nu(dx, nu)
        steps = int(round(T / dt))
        assert abs(steps * dt - T) < 1e-9
        y = np.arange(ny) * dx
        q0 = 1e-4 * np.sin(2 * np.pi * y / lamL)
        b = oracle.Basin(3, ny, dx, nu, np.zeros((ny, 3)), edges=(oracle.PERIODIC,) * 4,
                         h=np.ones((ny, 3)), qx=np.tile(q0[:, None], (1, 3)))
        b.run(steps)
        amp = (b.qx[:, 0] @ np.sin(2 * np.pi * y / lamL)) / (ny / 2) / 1e-4
        errs.append(abs(amp - math.exp(-nu * (2 * np.pi / lamL) ** 2 * T)))
    order = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(3.8 <= o <= 4.2 for o in order), (errs, order)


def test_gravity_wave_linear_map(oracle):
    """Small standing wave on a flat periodic 1D domain follows the linear
    amplification matrix M(theta) = [[1 - r(1-c), -i s/e], [-i gH s/e, c]],
    r = gH/e^2, c = cos theta, s = sin theta (derived from Eqs. feq-full,
    Mac.lb.6, Mac.lb.7 by linearising)."""
    nx, H, A = 24, 2.0, 1e-6
    k = 3
    th = 2 * np.pi * k / nx
    b = flat_periodic(oracle, nx, 3, nu=10.0 / 6.0)
    i = np.arange(nx)
    b.h[:] = H + A * np.cos(th * i)[None, :]
    e = b.e
    r = G * H / e ** 2
    M = np.array([[1 - r * (1 - math.cos(th)), -1j * math.sin(th) / e],
                  [-1j * G * H * math.sin(th) / e, math.cos(th)]])
    n = 40
    b.run(n)
    z = np.linalg.matrix_power(M, n) @ np.array([A, 0.0])
    eta = np.real(z[0] * np.exp(1j * th * i))
    q = np.real(z[1] * np.exp(1j * th * i))
    assert np.abs(b.h[1] - H - eta).max() <= 1e-5 * A
    assert np.abs(b.qx[1] - q).max() <= 1e-5 * A * e


def test_unstable_when_gH_exceeds_e2(oracle):
    """The linear map has |eigenvalue| = |1 - 2r| > 1 at theta = pi once gH > e^2:
    the odd-even mode grows; below the bound it does not."""
    nx, A = 16, 1e-7
    for H, grows in ((0.9 * 100 / G, False), (1.3 * 100 / G, True)):
        b = flat_periodic(oracle, nx, 3, nu=10.0 / 6.0)  # e = 10
        b.h[:] = H + A * np.cos(np.pi * np.arange(nx))[None, :]
        b.run(60)
        amp = np.abs(b.h - H).max()
        assert (amp > 10 * A) == grows


def test_mirror_symmetry(oracle):
    """y -> -y maps direction (1,2,3,4,5,6,7,8) to (1,8,7,6,5,4,3,2) and leaves
    C and lambda unchanged: a mirror-symmetric problem stays symmetric."""
    nx, ny = 20, 15
    X, Y = np.meshgrid(np.arange(nx), np.arange(ny) - (ny - 1) / 2)
    zb = 0.5 * np.exp(-((X - 8) ** 2 + Y ** 2) / 10)
    tx, _ = oracle.wind_stress(10.0, 0.0)
    h0 = 2.0 - zb + 0.05 * np.exp(-((X - 12) ** 2 + Y ** 2) / 6)
    b = oracle.Basin(nx, ny, 1.0, 10.0 / 6.0, zb, h=h0, tx=tx, cb=oracle.bed_coeff(45.0))
    b.run(400)
    assert np.abs(b.h - b.h[::-1]).max() <= 1e-12
    assert np.abs(b.qx - b.qx[::-1]).max() <= 1e-12
    assert np.abs(b.qy + b.qy[::-1]).max() <= 1e-12
    assert np.abs(b.qy).max() > 1e-5  # the flow is genuinely 2D


# ----------------------------------------------------------------------------- tidal flow
def tidal_exact(x, t, L, level, amp=4.0):
    """Long-wave asymptotic solution of Eqs. (swe-con), (swe-mom) for the tidal
    inflow h(0,t) = level + amp - amp sin(omega t + pi/2), closed at x = L: the
    surface stays flat, zeta(t) = level + amp - amp sin(omega t + pi/2), and
    continuity gives hu = (L - x) dzeta/dt."""
    om = 4 * np.pi / 86400
    zeta = level + amp - amp * np.sin(om * t + np.pi / 2)
    q = (L - x) * (-amp * om * np.cos(om * t + np.pi / 2))
    return zeta, q


def run_tidal(oracle, spec, t_end):
    h, qx, qy = spec.initial()
    b = oracle.Basin(spec.nx, spec.ny, spec.dx, spec.nu, spec.zb, edges=spec.edges,
                     extrap_order=spec.extrap_order, depth_bc=spec.depth_bc, h=h, qx=qx, qy=qy)
    n = int(round(t_end / b.dt))
    assert abs(n * b.dt - t_end) < 1e-6
    b.run(n)
    return b


def test_tidal_strip_vs_asymptotic(oracle):
    spec = wl.tidal_strip()
    b = run_tidal(oracle, spec, 10800.0)
    x = np.arange(spec.nx) * spec.dx
    L = x[-1]
    zeta, q = tidal_exact(x, b.t, L, spec.zeta_ref)
    lvl = b.h[1] + spec.zb[1]
    assert np.abs(lvl - zeta).max() / zeta <= 5e-4     # measured 3.5e-4 (quasi-static tilt)
    u = b.qx[1] / b.h[1]
    ue = q / (zeta - spec.zb[1])
    assert np.abs(u - ue).max() <= 0.07 * np.abs(ue).max()  # measured 4.7 % (start-up seiche)


def load_table1():
    import os
    p = os.path.join(os.path.dirname(__file__), "golden", "tidal_table1_bed.txt")
    d = np.loadtxt(p, comments="#")
    return d[:, 0], d[:, 1]


@pytest.mark.parametrize("t_end", [10800.0, 32400.0])
def test_paper_tidal_case_vs_asymptotic(oracle, t_end):
    """The paper's own tidal test (Section 4.1, Table 1): level and velocity
    against the analytical solution.  The paper reports < 0.005 % level error;
    the flat-surface asymptotic solution itself carries O(eps^2) error plus a
    start-up seiche, so the velocity gate is looser than its 0.05 %."""
    xs, zs = load_table1()
    spec = wl.tidal_table_bed(xs, zs)
    b = run_tidal(oracle, spec, t_end)
    x = np.arange(spec.nx) * spec.dx
    zeta, q = tidal_exact(x, t_end, 1500.0, 16.0)
    lvl = b.h[1] + spec.zb[1]
    # the paper's own bound on the level error: 0.005 % (measured 1.0e-5, 1.9e-5)
    assert np.abs(lvl - zeta).max() / zeta <= 5e-5
    u = b.qx[1] / b.h[1]
    ue = q / (zeta - spec.zb[1])
    assert np.abs(u - ue).max() <= 0.015 * np.abs(ue).max()  # measured 0.9 % of max |u|
