"""FP64 CPU oracle of the MacLABSWE step (Zhou, arXiv 1902.02999).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product path never does.  It
shares no code with the GPU library.

The arithmetic lives in ``maclab_ref.c`` (plain C, double precision, the
paper's Eqs. (feq-full), (Mac.lb.3), (Mac.lb.6), (Mac.lb.7), (force-CS)); this
module only compiles it with gcc, loads it with ctypes and marshals numpy
arrays.  ``nn_ref`` holds the numpy oracle of the learned warm-start network.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "maclab_ref.c")
_LIB = os.path.join(_HERE, "libmaclab_ref.so")
_lock = threading.Lock()
_lib = None

WALL, PERIODIC, DEPTH, DISCHARGE = 0, 1, 2, 3
W, E, S, N = 0, 1, 2, 3
FLUID, WALL_NODE, SOLID = 0, 1, 2   # node kinds of an optional geometry mask


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fPIC", "-shared",
                               "-fopenmp", "-fno-fast-math", "-ffp-contract=off",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Problem(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32),
                ("e", C.c_double), ("dt", C.c_double), ("g", C.c_double),
                ("tx", C.c_double), ("ty", C.c_double), ("cb", C.c_double),
                ("omega", C.c_double),
                ("edge", C.c_int32 * 4), ("extrap_order", C.c_int32), ("pad_", C.c_int32),
                ("bc_h_mean", C.c_double * 4), ("bc_amp", C.c_double * 4),
                ("bc_period", C.c_double * 4), ("bc_phase", C.c_double * 4),
                ("bc_qx", C.c_double * 4), ("bc_qy", C.c_double * 4),
                ("kind", C.c_void_p), ("hbar_implicit", C.c_int32), ("pad2_", C.c_int32)]


def lib():
    global _lib
    with _lock:
        if _lib is None:
            L = C.CDLL(build())
            dp = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
            L.mref_feq.restype = C.c_double
            L.mref_feq.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double]
            L.mref_params_from_nu.argtypes = [C.c_double, C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double)]
            L.mref_wind_stress.argtypes = [C.c_double] * 5 + [C.POINTER(C.c_double)] * 2
            L.mref_bed_coeff.restype = C.c_double
            L.mref_bed_coeff.argtypes = [C.c_double, C.c_double]
            L.mref_depth_bc.restype = C.c_double
            L.mref_depth_bc.argtypes = [C.POINTER(Problem), C.c_int, C.c_double]
            L.mref_step.argtypes = [C.POINTER(Problem), dp, dp, dp, dp, C.c_double, dp, dp, dp, C.c_int]
            L.mref_node.argtypes = [C.POINTER(Problem), dp, dp, dp, dp, C.c_double, C.c_int, C.c_int, dp]
            L.mref_node_trial.argtypes = [C.POINTER(Problem), dp, dp, dp, dp, C.c_int, C.c_int, C.c_double, dp]
            L.mref_run.argtypes = [C.POINTER(Problem), dp, dp, dp, dp, C.c_int64, C.c_int64, dp, C.c_int]
            L.mref_diag.argtypes = [C.c_int32, C.c_int32, C.c_double, dp, dp, dp,
                                    C.c_void_p, C.c_void_p, C.c_void_p, dp]
            L.mref_lattice.argtypes = [C.c_void_p] * 5
            L.mref_elab_init.argtypes = [C.POINTER(Problem), dp, dp, dp, dp]
            L.mref_elab_macro.argtypes = [C.POINTER(Problem), dp, dp, dp, dp]
            L.mref_elab_step.argtypes = [C.POINTER(Problem), C.c_double, dp, dp, dp, C.c_int]
            L.mref_elab_run.argtypes = [C.POINTER(Problem), C.c_double, dp, dp, C.c_int64, dp, C.c_int]
            L.mref_max_threads.restype = C.c_int
            _lib = L
    return _lib


def lattice():
    """The oracle's D2Q9 table: (ex, ey, C, lambda, opposite)."""
    ex = np.zeros(9, np.int32); ey = np.zeros(9, np.int32)
    ca = np.zeros(9); lam = np.zeros(9); opp = np.zeros(9, np.int32)
    lib().mref_lattice(ex.ctypes.data, ey.ctypes.data, ca.ctypes.data, lam.ctypes.data, opp.ctypes.data)
    return ex, ey, ca, lam, opp


def feq(a: int, g: float, e: float, h: float, u: float, v: float) -> float:
    """Eq. (feq-full) for one direction."""
    return lib().mref_feq(int(a), g, e, h, u, v)


def params_from_nu(dx: float, nu: float):
    """Eq. (mlb-viscosity): (e, dt)."""
    e = C.c_double(); dt = C.c_double()
    lib().mref_params_from_nu(dx, nu, C.byref(e), C.byref(dt))
    return e.value, dt.value


def wind_stress(uwx: float, uwy: float, rho_air=1.293, c_w=0.0026, rho_w=1000.0):
    """Eq. (wind_u-stress) over the water density."""
    tx = C.c_double(); ty = C.c_double()
    lib().mref_wind_stress(rho_air, c_w, rho_w, uwx, uwy, C.byref(tx), C.byref(ty))
    return tx.value, ty.value


def bed_coeff(cz: float, g: float = 9.81) -> float:
    """Eq. (bed-stress): C_b = g / C_z^2."""
    return lib().mref_bed_coeff(g, cz)


def default_threads() -> int:
    return int(os.environ.get("ORACLE_THREADS", "0")) or lib().mref_max_threads()


@dataclass
class Basin:
    """One problem for the oracle: FP64 fields [ny][nx] and the parameters.

    ``zb`` is the bed, ``h, qx, qy`` the depth and discharge (hu, hv).
    Edge kinds are (W, E, S, N) with WALL/PERIODIC/DEPTH/DISCHARGE.
    ``kind`` is an optional uint8 [ny][nx] node-kind mask (FLUID, WALL_NODE,
    SOLID).  ``hbar_implicit`` selects the link depth with the node's new-time
    depth (the definition given with Eq. feq-full) instead of Eq. h-bar.
    """
    nx: int
    ny: int
    dx: float
    nu: float
    zb: np.ndarray
    g: float = 9.81
    tx: float = 0.0
    ty: float = 0.0
    cb: float = 0.0
    omega: float = 0.0
    edges: tuple = (WALL, WALL, WALL, WALL)
    extrap_order: int = 1
    depth_bc: dict = field(default_factory=dict)     # edge -> (h_mean, amp, period, phase)
    discharge_bc: dict = field(default_factory=dict)  # edge -> (qx, qy)
    h: np.ndarray = None
    qx: np.ndarray = None
    qy: np.ndarray = None
    step_index: int = 0
    threads: int = 0
    kind: np.ndarray = None
    hbar_implicit: bool = False

    def __post_init__(self):
        self.zb = np.ascontiguousarray(self.zb, np.float64).reshape(self.ny, self.nx)
        self.e, self.dt = params_from_nu(self.dx, self.nu)
        for name in ("h", "qx", "qy"):
            a = getattr(self, name)
            a = np.zeros((self.ny, self.nx)) if a is None else np.array(a, np.float64, copy=True)
            setattr(self, name, np.ascontiguousarray(a.reshape(self.ny, self.nx)))
        if self.kind is not None:
            self.kind = np.ascontiguousarray(np.asarray(self.kind, np.uint8).reshape(self.ny, self.nx))
        self._work = np.zeros(3 * self.nx * self.ny)

    def problem(self) -> Problem:
        p = Problem()
        p.nx, p.ny = self.nx, self.ny
        p.e, p.dt, p.g = self.e, self.dt, self.g
        p.tx, p.ty, p.cb, p.omega = self.tx, self.ty, self.cb, self.omega
        for k in range(4):
            p.edge[k] = int(self.edges[k])
        p.extrap_order = int(self.extrap_order)
        for k, (hm, amp, per, ph) in self.depth_bc.items():
            p.bc_h_mean[k], p.bc_amp[k], p.bc_period[k], p.bc_phase[k] = hm, amp, per, ph
        for k, (a, b) in self.discharge_bc.items():
            p.bc_qx[k], p.bc_qy[k] = a, b
        p.kind = None if self.kind is None else self.kind.ctypes.data
        p.hbar_implicit = int(bool(self.hbar_implicit))
        return p

    @property
    def t(self) -> float:
        return self.step_index * self.dt

    def run(self, nsteps: int) -> None:
        """Advance nsteps steps in place (t = n dt at step n)."""
        p = self.problem()
        rc = lib().mref_run(C.byref(p), self.zb, self.h, self.qx, self.qy,
                            self.step_index, int(nsteps), self._work,
                            self.threads or default_threads())
        if rc:
            raise ValueError("oracle rejected the problem (rc=%d)" % rc)
        self.step_index += int(nsteps)

    def step_from(self, h, qx, qy, step_index=None):
        """One step from an arbitrary state; returns (h, qx, qy) new arrays."""
        p = self.problem()
        n = self.step_index if step_index is None else step_index
        h = np.ascontiguousarray(h, np.float64); qx = np.ascontiguousarray(qx, np.float64)
        qy = np.ascontiguousarray(qy, np.float64)
        o = [np.empty_like(h) for _ in range(3)]
        rc = lib().mref_step(C.byref(p), self.zb, h, qx, qy, n * self.dt, o[0], o[1], o[2],
                             self.threads or default_threads())
        if rc:
            raise ValueError("oracle rejected the problem (rc=%d)" % rc)
        return tuple(o)

    def node_from(self, h, qx, qy, i: int, j: int, step_index=None):
        """The new (h, hu, hv) of node (i, j) after one step from the given state."""
        p = self.problem()
        n = self.step_index if step_index is None else step_index
        out = np.zeros(3)
        rc = lib().mref_node(C.byref(p), self.zb, np.ascontiguousarray(h, np.float64),
                             np.ascontiguousarray(qx, np.float64),
                             np.ascontiguousarray(qy, np.float64), n * self.dt, int(i), int(j), out)
        if rc:
            raise ValueError("bad node")
        return out

    def node_trial(self, h, qx, qy, i: int, j: int, trial: float):
        """Node (i, j)'s update (before boundary overrides) with its new-time
        depth in h-bar taken as `trial` (the map the implicit h-bar solves)."""
        p = self.problem()
        out = np.zeros(3)
        rc = lib().mref_node_trial(C.byref(p), self.zb, np.ascontiguousarray(h, np.float64),
                                   np.ascontiguousarray(qx, np.float64), np.ascontiguousarray(qy, np.float64),
                                   int(i), int(j), float(trial), out)
        if rc:
            raise ValueError("bad node")
        return out

    def diag(self, qx0=None, qy0=None):
        """(mass, residual, max speed, bad count); residual needs the previous q."""
        out = np.zeros(4)
        a = None if qx0 is None else np.ascontiguousarray(qx0, np.float64)
        b = None if qy0 is None else np.ascontiguousarray(qy0, np.float64)
        lib().mref_diag(self.nx, self.ny, self.dx, self.h, self.qx, self.qy,
                        None if a is None else a.ctypes.data,
                        None if b is None else b.ctypes.data,
                        None if self.kind is None else self.kind.ctypes.data, out)
        return {"mass": out[0], "residual": out[1], "max_speed": out[2], "bad": int(out[3])}

    def run_steady(self, tol: float, max_steps: int, check_every: int = 100):
        """Step until the per-step residual at a check falls to tol."""
        while self.step_index < max_steps:
            self.run(check_every - 1)
            qx0, qy0 = self.qx.copy(), self.qy.copy()
            self.run(1)
            d = self.diag(qx0, qy0)
            if d["bad"]:
                raise FloatingPointError("non-finite or dry node at step %d" % self.step_index)
            if d["residual"] <= tol:
                return d
        return None


def from_spec(spec, h=None, qx=None, qy=None, step0=0) -> "Basin":
    """The oracle problem described by a workload spec (any object with the
    attributes of ``paper_1902_02999_amd.workloads.Spec``: shape, dx, nu, bed,
    forcing, edges and their data, node kinds, link-depth form).  The oracle
    derives its own e, dt, wind stress and friction coefficient from them."""
    if h is None:
        h, qx, qy = spec.initial()
    tx = ty = 0.0
    if spec.wind_speed is not None:
        tx, ty = wind_stress(*spec.wind_speed)
    if spec.wind_stress is not None:
        tx, ty = spec.wind_stress
    b = Basin(spec.nx, spec.ny, spec.dx, spec.nu, spec.zb, tx=tx, ty=ty,
              cb=bed_coeff(spec.chezy) if spec.chezy > 0 else 0.0,
              omega=spec.omega, edges=spec.edges, extrap_order=spec.extrap_order,
              depth_bc=dict(spec.depth_bc), discharge_bc=dict(spec.discharge_bc),
              h=h, qx=qx, qy=qy, kind=spec.kind, hbar_implicit=spec.hbar_implicit)
    b.step_index = step0
    return b


class ElabBasin:
    """The eLABSWE baseline (Eq. lb.1; nine stored distributions, relaxation
    time tau) on the problem of a ``Basin``: same bed, forcing, edges (walls
    and periodic only) and node kinds.  Starts from f = f^eq of the basin's
    state."""

    def __init__(self, basin: Basin, tau: float):
        self.b = basin
        self.tau = float(tau)
        n = basin.nx * basin.ny
        self.f = np.zeros(9 * n)
        self._work = np.zeros(9 * n)
        p = basin.problem()
        if lib().mref_elab_init(C.byref(p), basin.h, basin.qx, basin.qy, self.f):
            raise ValueError("oracle rejected the problem")
        self.step_index = basin.step_index

    def run(self, nsteps: int) -> None:
        p = self.b.problem()
        rc = lib().mref_elab_run(C.byref(p), self.tau, self.b.zb, self.f, int(nsteps), self._work,
                                 self.b.threads or default_threads())
        if rc:
            raise ValueError("oracle rejected the eLABSWE problem (rc=%d)" % rc)
        self.step_index += int(nsteps)

    def macro(self):
        """(h, hu, hv) [ny][nx] of the stored distributions."""
        b = self.b
        h = np.zeros((b.ny, b.nx)); qx = np.zeros_like(h); qy = np.zeros_like(h)
        p = b.problem()
        lib().mref_elab_macro(C.byref(p), self.f, h, qx, qy)
        return h, qx, qy

    def dist(self):
        """The distributions as [9][ny][nx]."""
        return self.f.reshape(9, self.b.ny, self.b.nx)
