"""Seeded synthetic inputs for the MacLABSWE step (numpy only).

These generators describe problems: grid size, lattice size, bed elevation,
still-water level, edge kinds and boundary data, wind and Chezy coefficient,
and the initial state.  They contain none of the method's arithmetic (no
equilibria, no force evaluation, no parameter derivation), so the GPU library
and the FP64 oracle can both be fed from them.

Edge kinds use the numbering WALL=0, PERIODIC=1, DEPTH=2, DISCHARGE=3 and the
edge order (W, E, S, N).  An optional node-kind mask describes irregular
geometry: FLUID=0, WALL_NODE=1 (no-slip boundary node), SOLID=2 (outside the
water).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

import numpy as np

WALL, PERIODIC, DEPTH, DISCHARGE = 0, 1, 2, 3
W, E, S, N = 0, 1, 2, 3
FLUID, WALL_NODE, SOLID = 0, 1, 2


@dataclass
class Spec:
    name: str
    nx: int
    ny: int
    dx: float
    nu: float
    zb: np.ndarray                       # bed elevation [ny][nx], FP64
    zeta_ref: float                      # still-water level; H = zeta_ref - zb
    edges: Tuple[int, int, int, int] = (WALL, WALL, WALL, WALL)
    extrap_order: int = 1
    depth_bc: Dict[int, Tuple[float, float, float, float]] = field(default_factory=dict)
    discharge_bc: Dict[int, Tuple[float, float]] = field(default_factory=dict)
    wind_speed: Optional[Tuple[float, float]] = None       # (u_wx, u_wy) [m/s]
    wind_stress: Optional[Tuple[float, float]] = None      # tau_w / rho [m^2/s^2]
    chezy: float = 0.0                                     # <= 0: no bed friction
    omega: float = 0.0
    h0: Optional[np.ndarray] = None      # initial depth; default still water
    qx0: Optional[np.ndarray] = None
    qy0: Optional[np.ndarray] = None
    kind: Optional[np.ndarray] = None    # node kinds [ny][nx] (uint8), None: all FLUID
    hbar_implicit: bool = False          # link depth with the node's new-time depth
    compensated: bool = False            # GPU: surface stored as a compensated FP32 pair

    def __post_init__(self):
        self.zb = np.ascontiguousarray(self.zb, np.float64).reshape(self.ny, self.nx)
        if self.kind is not None:
            self.kind = np.ascontiguousarray(np.asarray(self.kind, np.uint8).reshape(self.ny, self.nx))

    @property
    def H(self) -> np.ndarray:
        return self.zeta_ref - self.zb

    def initial(self):
        h = (np.maximum(self.H, 0.0) if self.h0 is None else np.asarray(self.h0, np.float64))
        qx = np.zeros_like(h) if self.qx0 is None else np.asarray(self.qx0, np.float64)
        qy = np.zeros_like(h) if self.qy0 is None else np.asarray(self.qy0, np.float64)
        return (np.ascontiguousarray(h.reshape(self.ny, self.nx)),
                np.ascontiguousarray(qx.reshape(self.ny, self.nx) * np.ones((self.ny, self.nx))),
                np.ascontiguousarray(qy.reshape(self.ny, self.nx) * np.ones((self.ny, self.nx))))

    @property
    def nodes(self) -> int:
        return self.nx * self.ny


def nu_for_speed(e: float, dx: float) -> float:
    """The eddy viscosity that gives lattice speed e on lattice size dx
    (inverse of e = 6 nu / dx; used only to state the chosen e)."""
    return e * dx / 6.0


# ----------------------------------------------------------------------------- 1D tidal strip
def tidal_strip(nx: int = 400, ny: int = 3, L: float = 14000.0, dx: float = 35.0,
                dt: float = 1.0, zeta_ref: float = 60.5, amp: float = 4.0) -> Spec:
    """1D tidal flow as a D2Q9 strip, periodic across.  Bed
    zb = 10 + 40 x/L + 10 sin(pi (4x/L - 1/2)); still level zeta_ref; west depth
    h(0,t) = H(0) + 4 - 4 sin(pi (4t/86400 + 1/2)); east end closed (wall)."""
    x = np.arange(nx) * dx
    zb1 = 10.0 + 40.0 * x / L + 10.0 * np.sin(np.pi * (4.0 * x / L - 0.5))
    zb = np.tile(zb1, (ny, 1))
    e = dx / dt
    H0 = zeta_ref - zb1[0]
    return Spec("tidal_strip_%dx%d" % (nx, ny), nx, ny, dx, nu_for_speed(e, dx), zb, zeta_ref,
                edges=(DEPTH, WALL, PERIODIC, PERIODIC), extrap_order=2,
                depth_bc={W: (H0, amp, 43200.0, np.pi / 2)})


def tidal_table_bed(x_pts, z_pts, nx: int = 201, dx: float = 7.5, ny: int = 3,
                    nu: float = 31.25, level: float = 16.0, amp: float = 4.0) -> Spec:
    """The paper's 1D tidal case over an irregular bed given as a table of
    (x, zb) points, interpolated linearly; h(x,0) = level - zb, u = 0,
    h(0,t) = level + amp - amp sin(pi (4t/86400 + 1/2)), u(end) = 0."""
    x = np.arange(nx) * dx
    zb1 = np.interp(x, np.asarray(x_pts, float), np.asarray(z_pts, float))
    zb = np.tile(zb1, (ny, 1))
    return Spec("tidal_table_%d" % nx, nx, ny, dx, nu, zb, level,
                edges=(DEPTH, WALL, PERIODIC, PERIODIC), extrap_order=2,
                depth_bc={W: (level - zb1[0], amp, 43200.0, np.pi / 2)})


# ----------------------------------------------------------------------------- wind-driven lake
def wind_lake(n: int = 256, side: float = 8000.0, h0: float = 10.0, R: float = 4000.0,
              shelf: float = 0.5, tau_pa: Tuple[float, float] = (0.1, 0.0), rho_w: float = 1000.0,
              chezy: float = 50.0, e: float = 20.0) -> Spec:
    """Dish-shaped lake in a square basin: H = h0 max(0, 1 - r^2/R^2) + shelf,
    cell-centred nodes, uniform wind stress, Chezy friction, walls all round."""
    dx = side / n
    c = (np.arange(n) + 0.5) * dx - side / 2
    X, Y = np.meshgrid(c, c)
    r2 = X * X + Y * Y
    H = h0 * np.maximum(0.0, 1.0 - r2 / (R * R)) + shelf
    zeta_ref = h0 + shelf
    return Spec("wind_lake_%d" % n, n, n, dx, nu_for_speed(e, dx), zeta_ref - H, zeta_ref,
                wind_stress=(tau_pa[0] / rho_w, tau_pa[1] / rho_w), chezy=chezy)


# ----------------------------------------------------------------------------- bump channel
def bump_channel(nx: int = 4096, ny: Optional[int] = None, dx: float = 1.0, depth: float = 2.0,
                 bump: float = 0.2, sigma: Optional[float] = None, q_in: float = 4.42,
                 e: float = 25.0) -> Spec:
    """Subcritical channel flow over a Gaussian bump at the centre: discharge
    q_in at the west edge, fixed depth at the east edge, walls north and south.
    Initial state: still level, uniform discharge q_in."""
    ny = nx if ny is None else ny
    sigma = 100.0 * nx / 4096.0 if sigma is None else sigma
    sigma = max(sigma, 2.0 * dx)
    x = (np.arange(nx) - (nx - 1) / 2.0) * dx
    y = (np.arange(ny) - (ny - 1) / 2.0) * dx
    X, Y = np.meshgrid(x, y)
    zb = bump * np.exp(-(X * X + Y * Y) / (2.0 * sigma * sigma))
    qx0 = np.full((ny, nx), q_in)
    return Spec("bump_channel_%dx%d" % (nx, ny), nx, ny, dx, nu_for_speed(e, dx), zb, depth,
                edges=(DISCHARGE, DEPTH, WALL, WALL),
                depth_bc={E: (depth, 0.0, 0.0, 0.0)}, discharge_bc={W: (q_in, 0.0)},
                qx0=qx0)


# ----------------------------------------------------------------------------- irregular geometry
def staircase_kinds(inside: np.ndarray) -> np.ndarray:
    """Node kinds of a staircase boundary: nodes outside the water are SOLID;
    water nodes with an outside node (or the grid's edge) among their eight
    neighbours are WALL_NODE; the rest FLUID."""
    inside = np.asarray(inside, bool)
    pad = np.pad(inside, 1, constant_values=False)
    ny, nx = inside.shape
    all_in = np.ones_like(inside)
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            all_in &= pad[1 + dy:1 + dy + ny, 1 + dx:1 + dx + nx]
    kind = np.full(inside.shape, SOLID, np.uint8)
    kind[inside] = WALL_NODE
    kind[inside & all_in] = FLUID
    return kind


def circular_dish(n: int = 200, dx: float = 2.0, nu: float = 5.33, wind: float = 5.0,
                  chezy: float = 0.0) -> Spec:
    """Wind-driven circulation in a circular basin (Section 4): still-water
    depth H = (1/1.3) (1/2 + sqrt(1/2 - r/386.4)) for r <= 193.2 m, bed
    z_b = H(0,0) - H, wind u_w m/s from south-west to north-east.  Nodes sit at
    cell centres of an n x n square of side n dx centred on the basin; nodes
    with r > 193.2 m are SOLID (their H is the rim depth), the water's outer
    ring is WALL_NODE (staircase bounce-back).  The paper gives no bed
    friction for this case: none by default."""
    c = (np.arange(n) - (n - 1) / 2.0) * dx
    X, Y = np.meshgrid(c, c)
    r = np.hypot(X, Y)
    R = 193.2
    inside = r <= R
    H = (1.0 / 1.3) * (0.5 + np.sqrt(np.maximum(0.5 - np.minimum(r, R) / 386.4, 0.0)))
    H0 = (1.0 / 1.3) * (0.5 + np.sqrt(0.5))
    w = wind / np.sqrt(2.0)
    return Spec("circular_dish_%d" % n, n, n, dx, nu, H0 - H, H0, wind_speed=(w, w), chezy=chezy,
                kind=staircase_kinds(inside))


def hump_channel(n: int = 200, length: float = 1000.0, q: float = 10.0, depth: float = 10.0,
                 e: float = 25.0) -> Spec:
    """Steady flow over a 2D hump (Section 4): z_b = sin^2(pi (x-300)/200)
    sin^2(pi (y-400)/200) on [300,500] x [400,600], 0 elsewhere, in a square
    channel of side `length` on n x n cell-centred nodes; discharge q m^2/s
    in at the west edge, depth `depth` at the east (outflow) edge, walls
    north and south.  Initial state: still level `depth`, uniform q.  The
    paper gives no viscosity for this case: e (hence nu = e dx / 6) is chosen
    with g H <= e^2 and a small lattice Reynolds number."""
    dx = length / n
    c = (np.arange(n) + 0.5) * dx
    X, Y = np.meshgrid(c, c)
    om = (X >= 300.0) & (X <= 500.0) & (Y >= 400.0) & (Y <= 600.0)
    zb = np.where(om, np.sin(np.pi * (X - 300.0) / 200.0) ** 2 * np.sin(np.pi * (Y - 400.0) / 200.0) ** 2, 0.0)
    return Spec("hump_channel_%d" % n, n, n, dx, nu_for_speed(e, dx), zb, depth,
                edges=(DISCHARGE, DEPTH, WALL, WALL),
                depth_bc={E: (depth, 0.0, 0.0, 0.0)}, discharge_bc={W: (q, 0.0)},
                qx0=np.full((n, n), q))


def random_geometry(rng: np.random.Generator, nx: int, ny: int, holes: int = 3) -> np.ndarray:
    """Node kinds of a random closed basin: an ellipse-and-rectangle union
    with islands (SOLID discs) punched out, staircase boundary."""
    Y, X = np.mgrid[0:ny, 0:nx].astype(float)
    cx, cy = rng.uniform(0.35, 0.65) * nx, rng.uniform(0.35, 0.65) * ny
    ax, ay = rng.uniform(0.3, 0.48) * nx, rng.uniform(0.3, 0.48) * ny
    inside = ((X - cx) / ax) ** 2 + ((Y - cy) / ay) ** 2 <= 1.0
    x0, y0 = int(rng.integers(1, nx // 3)), int(rng.integers(1, ny // 3))
    inside |= (X >= x0) & (X < x0 + nx // 3) & (Y >= y0) & (Y < y0 + ny // 2)
    for _ in range(holes):
        hx, hy, hr = rng.uniform(0.2, 0.8) * nx, rng.uniform(0.2, 0.8) * ny, rng.uniform(1.0, 3.5)
        inside &= (X - hx) ** 2 + (Y - hy) ** 2 > hr * hr
    return staircase_kinds(inside)


# ----------------------------------------------------------------------------- ensemble basins
def random_basin(rng: np.random.Generator, n: int, dx: float = 1.0, depth: float = 2.0,
                 e: float = 10.0, name: str = "basin") -> Spec:
    """A closed square basin: 1-3 Gaussian bumps (height U(0,0.3) m, width
    U(n/16, n/6) nodes, centre U(0.2n, 0.8n)), wind speed U(0,15) m/s at a
    random heading, Chezy U(30,70), walls all round."""
    nb = int(rng.integers(1, 4))
    c = np.arange(n) * dx
    X, Y = np.meshgrid(c, c)
    zb = np.zeros((n, n))
    for _ in range(nb):
        hgt = rng.uniform(0.0, 0.3)
        sig = rng.uniform(n / 16.0, n / 6.0) * dx
        cx, cy = rng.uniform(0.2 * n, 0.8 * n, size=2) * dx
        zb += hgt * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2.0 * sig * sig))
    speed = rng.uniform(0.0, 15.0)
    head = rng.uniform(0.0, 2.0 * np.pi)
    chezy = rng.uniform(30.0, 70.0)
    return Spec("%s_%d" % (name, n), n, n, dx, nu_for_speed(e, dx), zb, depth,
                wind_speed=(speed * np.cos(head), speed * np.sin(head)), chezy=chezy)


def ensemble(count: int = 512, seed: int = 1902, nmin: int = 64, nmax: int = 512) -> List[Spec]:
    """Closed basins with sizes drawn uniformly from nmin..nmax (square)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = rng.integers(nmin, nmax + 1, size=count)
    return [random_basin(rng, int(n), name="basin%03d" % i) for i, n in enumerate(sizes)]


def learned_set(count: int, seed: int, n: int = 256) -> List[Spec]:
    """Fixed-size basins from the ensemble distributions (warm-start data)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return [random_basin(rng, n, name="ws%04d" % i) for i in range(count)]


# ----------------------------------------------------------------------------- small fields
def seeded_state(spec: Spec, seed: int, eta_amp: float = 0.05, q_amp: float = 0.05):
    """A smooth random perturbation of still water (for parity tests)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ny, nx = spec.ny, spec.nx
    def smooth():
        f = rng.standard_normal((ny, nx))
        for _ in range(3):
            f = 0.25 * (np.roll(f, 1, 0) + np.roll(f, -1, 0) + np.roll(f, 1, 1) + np.roll(f, -1, 1))
        return f / max(1e-12, np.abs(f).max())
    h = np.maximum(spec.H, 0.0) + eta_amp * smooth()
    qx = q_amp * smooth()
    qy = q_amp * smooth()
    return h, qx, qy
