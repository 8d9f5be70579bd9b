"""ctypes binding of the C ABI in include/mlb.h (argument marshalling only).

Every step of the method runs in the HIP kernels of libmlb.so; this module
only converts numpy / torch arguments and raises on error codes.  Loading
fails loudly if libmlb.so has not been built (python -m
paper_1902_02999_amd.build); there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmlb.so")

WALL, PERIODIC, DEPTH, DISCHARGE = 0, 1, 2, 3
NODE_FLUID, NODE_WALL, NODE_SOLID = 0, 1, 2   # MLB_NODE_*
HBAR_SEMI_IMPLICIT, HBAR_IMPLICIT = 0, 1       # MLB_HBAR_*
SURFACE_FP32, SURFACE_COMPENSATED = 0, 1       # MLB_SURFACE_*
W, E, S, N = 0, 1, 2, 3

STATUS = {0: "MLB_OK", -1: "MLB_E_INVAL", -2: "MLB_E_NOMEM", -3: "MLB_E_DEVICE",
          -4: "MLB_E_UNSTABLE", -5: "MLB_E_NONFINITE", -6: "MLB_E_STATE",
          -7: "MLB_E_NOTCONVERGED", -8: "MLB_E_STALLED"}


class MlbError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__("%s failed: %s (%s)" % (where, STATUS.get(code, code), msg))
        self.code = code
        self.name = STATUS.get(code, str(code))


class Params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("dx", C.c_double), ("nu", C.c_double),
                ("g", C.c_double), ("rho_w", C.c_double), ("rho_air", C.c_double),
                ("c_w", C.c_double), ("omega", C.c_double), ("zeta_ref", C.c_double),
                ("edge", C.c_int32 * 4), ("extrap_order", C.c_int32)]


class Diag(C.Structure):
    _fields_ = [("step", C.c_int64), ("t", C.c_double), ("mass", C.c_double),
                ("residual", C.c_double), ("max_speed", C.c_double), ("nonfinite", C.c_int64),
                ("e", C.c_double), ("dt", C.c_double), ("gh_over_e2", C.c_double),
                ("rle", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ExecOpts(C.Structure):
    _fields_ = [("tile_rows", C.c_int32), ("tblock", C.c_int32), ("use_graph", C.c_int32),
                ("graph_chunk", C.c_int32), ("blocks_per_cu", C.c_int32), ("persistent", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class NetCfg(C.Structure):
    _fields_ = [("height", C.c_int32), ("width", C.c_int32), ("in_ch", C.c_int32), ("out_ch", C.c_int32),
                ("base_ch", C.c_int32), ("levels", C.c_int32), ("max_batch", C.c_int32)]


NET_FEATURES = 8   # MLB_NET_FEATURES


class NetNorm(C.Structure):
    _fields_ = [("in_mean", C.c_float * 5), ("in_std", C.c_float * 5), ("s_eta", C.c_float), ("s_q", C.c_float),
                ("tau_ref", C.c_float)]


class AdamWCfg(C.Structure):
    _fields_ = [("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("weight_decay", C.c_float)]


class TrainCfg(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_float), ("lr_min", C.c_float),
                ("warmup_steps", C.c_int32), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("weight_decay", C.c_float), ("seed", C.c_uint64)]


class WarmReport(C.Structure):
    _fields_ = [("used_guess", C.c_int32), ("fallback", C.c_int32), ("r0_guess", C.c_double),
                ("r0_cold", C.c_double), ("infer_ms", C.c_double), ("wall_s", C.c_double),
                ("steps", C.c_int64), ("steps_total", C.c_int64), ("guess_err", C.c_double * 3),
                ("diag", Diag)]

    def as_dict(self) -> dict:
        out = {k: getattr(self, k) for k, _ in self._fields_ if k not in ("guess_err", "diag")}
        out["guess_err"] = list(self.guess_err)
        out["diag"] = self.diag.as_dict()
        return out


WARM_NONE, WARM_NONFINITE_GUESS, WARM_WORSE_THAN_COLD, WARM_DIVERGING = 0, 1, 2, 3

# Every exported symbol of include/mlb.h with its ctypes signature.
_VP = C.c_void_p
_DP = C.POINTER(C.c_double)
SIGNATURES = {
    "mlb_status_str": (C.c_char_p, [C.c_int]),
    "mlb_last_error": (C.c_char_p, []),
    "mlb_ctx_create": (C.c_int, [C.c_int, _VP, C.POINTER(_VP)]),
    "mlb_ctx_destroy": (C.c_int, [_VP]),
    "mlb_ctx_sync": (C.c_int, [_VP]),
    "mlb_grid_workspace_bytes": (C.c_int, [C.POINTER(Params), C.POINTER(C.c_size_t)]),
    "mlb_grid_create": (C.c_int, [_VP, C.POINTER(Params), _VP, C.c_size_t, C.POINTER(_VP)]),
    "mlb_grid_destroy": (C.c_int, [_VP]),
    "mlb_set_bathymetry": (C.c_int, [_VP, _DP, C.c_int64]),
    "mlb_set_mask": (C.c_int, [_VP, C.POINTER(C.c_uint8), C.c_int64]),
    "mlb_set_hbar": (C.c_int, [_VP, C.c_int32]),
    "mlb_plan_tiles": (C.c_int, [C.POINTER(Params), C.POINTER(C.c_uint8), C.c_int64, C.c_int32, C.c_int32,
                                 C.POINTER(C.c_int32), C.c_int64, C.POINTER(C.c_int64)]),
    "mlb_plan_workqueue": (C.c_int, [C.POINTER(Params), C.POINTER(C.c_uint8), C.c_int64, C.c_int32, C.c_int32,
                                     C.POINTER(C.c_int32), C.c_int64, C.POINTER(C.c_int32), C.c_int64,
                                     C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "mlb_set_surface": (C.c_int, [_VP, C.c_int32]),
    "mlb_set_wind": (C.c_int, [_VP, C.c_double, C.c_double]),
    "mlb_set_wind_stress": (C.c_int, [_VP, C.c_double, C.c_double]),
    "mlb_set_chezy": (C.c_int, [_VP, C.c_double]),
    "mlb_set_edge_depth": (C.c_int, [_VP, C.c_int, C.c_double, C.c_double, C.c_double, C.c_double]),
    "mlb_set_edge_discharge": (C.c_int, [_VP, C.c_int, C.c_double, C.c_double]),
    "mlb_set_state": (C.c_int, [_VP, _DP, _DP, _DP, C.c_int64, C.c_int64]),
    "mlb_set_state_device": (C.c_int, [_VP, _VP, _VP, _VP]),
    "mlb_get_state": (C.c_int, [_VP, _DP, _DP, _DP, C.c_int64]),
    "mlb_get_state_device": (C.c_int, [_VP, _VP, _VP, _VP, _VP]),
    "mlb_step": (C.c_int, [_VP, C.c_int64]),
    "mlb_diag": (C.c_int, [_VP, C.POINTER(Diag)]),
    "mlb_run_steady": (C.c_int, [_VP, C.c_double, C.c_int64, C.c_int32, C.POINTER(Diag)]),
    "mlb_get_exec_opts": (C.c_int, [_VP, C.POINTER(ExecOpts)]),
    "mlb_set_exec_opts": (C.c_int, [_VP, C.POINTER(ExecOpts)]),
    "mlb_batch_create": (C.c_int, [_VP, C.POINTER(_VP), C.c_int32, C.POINTER(_VP)]),
    "mlb_batch_step": (C.c_int, [_VP, C.c_int64]),
    "mlb_batch_run_steady": (C.c_int, [_VP, C.c_double, C.c_int64, C.c_int32, C.POINTER(Diag)]),
    "mlb_batch_set_exec_opts": (C.c_int, [_VP, C.POINTER(ExecOpts)]),
    "mlb_batch_destroy": (C.c_int, [_VP]),
    "mlb_last_step_ms": (C.c_int, [_VP, _DP]),
    "mlb_last_pass_ms": (C.c_int, [_VP, _DP, C.POINTER(C.c_int64), C.POINTER(C.c_int32)]),
    "mlb_diag_noalloc": (C.c_int, [_VP, _VP]),
    "mlb_copy_probe": (C.c_int, [_VP, C.c_size_t, C.c_int32, _DP]),
    "mlb_autotune": (C.c_int, [_VP, C.c_int32, C.c_char_p, C.POINTER(ExecOpts)]),
    "mlb_batch_autotune": (C.c_int, [_VP, C.c_int32, C.c_char_p, C.POINTER(ExecOpts)]),
    "mlb_net_create": (C.c_int, [_VP, C.POINTER(NetCfg), C.c_uint64, C.POINTER(_VP)]),
    "mlb_net_destroy": (C.c_int, [_VP]),
    "mlb_net_param_count": (C.c_int, [_VP, C.POINTER(C.c_int64)]),
    "mlb_net_get_params": (C.c_int, [_VP, C.POINTER(C.c_float), C.c_int64]),
    "mlb_net_set_params": (C.c_int, [_VP, C.POINTER(C.c_float), C.c_int64]),
    "mlb_net_set_norm": (C.c_int, [_VP, C.POINTER(NetNorm)]),
    "mlb_net_get_norm": (C.c_int, [_VP, C.POINTER(NetNorm)]),
    "mlb_net_forward": (C.c_int, [_VP, _VP, C.c_int32, _VP]),
    "mlb_net_loss_grad": (C.c_int, [_VP, _VP, _VP, _VP, C.c_double, C.c_int32, _DP, C.POINTER(C.c_float)]),
    "mlb_net_adamw": (C.c_int, [_VP, C.POINTER(AdamWCfg)]),
    "mlb_net_features": (C.c_int, [_VP, _VP, _VP]),
    "mlb_net_targets": (C.c_int, [_VP, _VP, _VP]),
    "mlb_net_infer": (C.c_int, [_VP, _VP]),
    "mlb_net_save": (C.c_int, [_VP, C.c_char_p]),
    "mlb_net_load": (C.c_int, [_VP, C.c_char_p]),
    "mlb_net_train": (C.c_int, [_VP, _VP, _VP, _VP, C.c_int32, C.POINTER(TrainCfg), _DP]),
    "mlb_warm_start_run": (C.c_int, [_VP, _VP, C.c_double, C.c_int64, C.c_int32, C.POINTER(WarmReport)]),
    "mlb_set_stall_checks": (C.c_int, [_VP, C.c_int32]),
    "mlb_elab_create": (C.c_int, [_VP, C.c_double, C.POINTER(_VP)]),
    "mlb_elab_step": (C.c_int, [_VP, C.c_int64]),
    "mlb_elab_get_state": (C.c_int, [_VP, _DP, _DP, _DP, C.c_int64]),
    "mlb_elab_get_dist_device": (C.c_int, [_VP, _VP]),
    "mlb_elab_destroy": (C.c_int, [_VP]),
}

_lib = None


def lib():
    """Load libmlb.so (raises if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libmlb.so is not built; run `python -m paper_1902_02999_amd.build`")
        L = C.CDLL(LIB_PATH, mode=C.RTLD_GLOBAL)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(code: int, where: str):
    if code != 0:
        raise MlbError(code, where, lib().mlb_last_error().decode())


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(_DP)


def _f64(a, shape):
    return np.ascontiguousarray(np.broadcast_to(np.asarray(a, np.float64), shape))


def _tensor_ptr(t):
    """Device pointer of a torch tensor or an int."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


class Context:
    """One GPU and one HIP stream.  stream: None (library-owned stream) or a
    torch.cuda.Stream / raw hipStream_t int (not the legacy default stream if
    graphs are used)."""

    def __init__(self, device: int = 0, stream=None):
        h = _VP()
        s = None
        if stream is not None:
            s = stream if isinstance(stream, int) else stream.cuda_stream
        _check(lib().mlb_ctx_create(device, s, C.byref(h)), "mlb_ctx_create")
        self.h = h
        self.device = device

    def sync(self):
        _check(lib().mlb_ctx_sync(self.h), "mlb_ctx_sync")

    def set_stall_checks(self, checks: int):
        """Steady-state runs stop (stalled) after `checks` checks without a
        new lowest residual; 0 turns the rule off."""
        _check(lib().mlb_set_stall_checks(self.h, int(checks)), "mlb_set_stall_checks")

    def last_step_ms(self) -> float:
        v = C.c_double()
        _check(lib().mlb_last_step_ms(self.h, C.byref(v)), "mlb_last_step_ms")
        return v.value

    def last_pass_ms(self):
        """(ms per pass, passes, steps per pass) of the last call's bulk passes."""
        v = C.c_double()
        n = C.c_int64()
        k = C.c_int32()
        _check(lib().mlb_last_pass_ms(self.h, C.byref(v), C.byref(n), C.byref(k)), "mlb_last_pass_ms")
        return v.value, n.value, k.value

    def copy_probe(self, nbytes: int, reps: int = 10) -> float:
        """Read + write GB/s of a plain device copy of nbytes."""
        v = C.c_double()
        _check(lib().mlb_copy_probe(self.h, int(nbytes), int(reps), C.byref(v)), "mlb_copy_probe")
        return v.value

    def close(self):
        if self.h:
            _check(lib().mlb_ctx_destroy(self.h), "mlb_ctx_destroy")
            self.h = None


def make_params(nx, ny, dx, nu, zeta_ref=0.0, edges=(WALL, WALL, WALL, WALL), extrap_order=1,
                g=9.81, rho_w=1000.0, rho_air=1.293, c_w=0.0026, omega=0.0) -> Params:
    p = Params()
    p.nx, p.ny, p.dx, p.nu = int(nx), int(ny), float(dx), float(nu)
    p.g, p.rho_w, p.rho_air, p.c_w, p.omega, p.zeta_ref = g, rho_w, rho_air, c_w, omega, zeta_ref
    for k in range(4):
        p.edge[k] = int(edges[k])
    p.extrap_order = int(extrap_order)
    return p


def workspace_bytes(p: Params) -> int:
    n = C.c_size_t()
    _check(lib().mlb_grid_workspace_bytes(C.byref(p), C.byref(n)), "mlb_grid_workspace_bytes")
    return n.value


class Grid:
    """A basin on the GPU.  workspace: optional torch uint8 CUDA tensor of at
    least workspace_bytes(params) bytes (kept alive by this object)."""

    def __init__(self, ctx: Context, params: Params, workspace=None):
        self.ctx = ctx
        self.params = params
        self.nx, self.ny = params.nx, params.ny
        self._ws = workspace
        h = _VP()
        ptr, nbytes = None, 0
        if workspace is not None:
            ptr = _tensor_ptr(workspace)
            nbytes = workspace.numel() * workspace.element_size()
        _check(lib().mlb_grid_create(ctx.h, C.byref(params), ptr, nbytes, C.byref(h)), "mlb_grid_create")
        self.h = h

    # -- setup
    def set_bathymetry(self, zb):
        a = _f64(zb, (self.ny, self.nx))
        _check(lib().mlb_set_bathymetry(self.h, _dptr(a), self.nx), "mlb_set_bathymetry")

    def set_mask(self, kind):
        """Node kinds [ny][nx] (NODE_FLUID / NODE_WALL / NODE_SOLID); None removes the mask."""
        if kind is None:
            _check(lib().mlb_set_mask(self.h, None, self.nx), "mlb_set_mask")
            return
        a = np.ascontiguousarray(np.asarray(kind).reshape(self.ny, self.nx), np.uint8)
        _check(lib().mlb_set_mask(self.h, a.ctypes.data_as(C.POINTER(C.c_uint8)), self.nx), "mlb_set_mask")

    def set_hbar(self, implicit: bool):
        """Link depth: Eq. h-bar (False, default) or the implicit new-time form (True)."""
        _check(lib().mlb_set_hbar(self.h, HBAR_IMPLICIT if implicit else HBAR_SEMI_IMPLICIT), "mlb_set_hbar")

    def set_surface(self, compensated: bool):
        """Surface perturbation in FP32 (False, default) or as a compensated FP32 pair (True)."""
        _check(lib().mlb_set_surface(self.h, SURFACE_COMPENSATED if compensated else SURFACE_FP32),
               "mlb_set_surface")

    def set_wind(self, uwx, uwy):
        _check(lib().mlb_set_wind(self.h, uwx, uwy), "mlb_set_wind")

    def set_wind_stress(self, tx, ty):
        _check(lib().mlb_set_wind_stress(self.h, tx, ty), "mlb_set_wind_stress")

    def set_chezy(self, cz):
        _check(lib().mlb_set_chezy(self.h, cz), "mlb_set_chezy")

    def set_edge_depth(self, edge, h_mean, amp=0.0, period=0.0, phase=0.0):
        _check(lib().mlb_set_edge_depth(self.h, edge, h_mean, amp, period, phase), "mlb_set_edge_depth")

    def set_edge_discharge(self, edge, qx, qy=0.0):
        _check(lib().mlb_set_edge_discharge(self.h, edge, qx, qy), "mlb_set_edge_discharge")

    def set_state(self, h, hu=None, hv=None, step0: int = 0):
        shape = (self.ny, self.nx)
        a = _f64(h, shape)
        b = None if hu is None else _f64(hu, shape)
        c = None if hv is None else _f64(hv, shape)
        _check(lib().mlb_set_state(self.h, _dptr(a), None if b is None else _dptr(b),
                                   None if c is None else _dptr(c), self.nx, int(step0)),
               "mlb_set_state")

    def set_state_device(self, eta, qx, qy):
        _check(lib().mlb_set_state_device(self.h, _tensor_ptr(eta), _tensor_ptr(qx), _tensor_ptr(qy)),
               "mlb_set_state_device")

    def get_state(self):
        shape = (self.ny, self.nx)
        h, hu, hv = np.empty(shape), np.empty(shape), np.empty(shape)
        _check(lib().mlb_get_state(self.h, _dptr(h), _dptr(hu), _dptr(hv), self.nx), "mlb_get_state")
        return h, hu, hv

    def get_state_device(self, eta=None, qx=None, qy=None, H=None):
        _check(lib().mlb_get_state_device(self.h, _tensor_ptr(eta), _tensor_ptr(qx), _tensor_ptr(qy),
                                          _tensor_ptr(H)), "mlb_get_state_device")

    # -- execution
    def exec_opts(self) -> ExecOpts:
        o = ExecOpts()
        _check(lib().mlb_get_exec_opts(self.h, C.byref(o)), "mlb_get_exec_opts")
        return o

    def set_exec_opts(self, tile_rows=None, tblock=None, use_graph=None, graph_chunk=None,
                      blocks_per_cu=None, persistent=None):
        o = self.exec_opts()
        if tile_rows is not None: o.tile_rows = tile_rows
        if tblock is not None: o.tblock = tblock
        if use_graph is not None: o.use_graph = int(use_graph)
        if graph_chunk is not None: o.graph_chunk = graph_chunk
        if blocks_per_cu is not None: o.blocks_per_cu = blocks_per_cu
        if persistent is not None: o.persistent = int(persistent)
        _check(lib().mlb_set_exec_opts(self.h, C.byref(o)), "mlb_set_exec_opts")

    def autotune(self, steps: int = 40, cache_path: Optional[str] = None) -> dict:
        """Time the candidate execution options, apply the fastest; state kept."""
        o = ExecOpts()
        _check(lib().mlb_autotune(self.h, int(steps), None if cache_path is None else cache_path.encode(),
                                  C.byref(o)), "mlb_autotune")
        return o.as_dict()

    def step(self, n: int = 1):
        _check(lib().mlb_step(self.h, int(n)), "mlb_step")

    def diag_noalloc(self, out_dev):
        """mlb_diag_noalloc into a device buffer of at least 80 bytes (a torch
        tensor or a device pointer); enqueued, returns without waiting."""
        ptr = out_dev if isinstance(out_dev, int) else out_dev.data_ptr()
        _check(lib().mlb_diag_noalloc(self.h, C.c_void_p(ptr)), "mlb_diag_noalloc")

    def diag(self) -> dict:
        d = Diag()
        _check(lib().mlb_diag(self.h, C.byref(d)), "mlb_diag")
        return d.as_dict()

    def run_steady(self, tol: float, max_steps: int, check_every: int = 100):
        """Returns (converged, diag dict); raises on non-finite values."""
        d = Diag()
        rc = lib().mlb_run_steady(self.h, tol, int(max_steps), int(check_every), C.byref(d))
        if rc in (-7, -8):
            out = d.as_dict()
            out["stalled"] = rc == -8
            return False, out
        _check(rc, "mlb_run_steady")
        out = d.as_dict()
        out["stalled"] = False
        return True, out

    def close(self):
        if self.h:
            _check(lib().mlb_grid_destroy(self.h), "mlb_grid_destroy")
            self.h = None


class Batch:
    """Many grids stepped by one persistent launch per step."""

    def __init__(self, ctx: Context, grids: Sequence[Grid]):
        self.ctx = ctx
        self.grids = list(grids)
        arr = (_VP * len(grids))(*[g.h for g in grids])
        h = _VP()
        _check(lib().mlb_batch_create(ctx.h, arr, len(grids), C.byref(h)), "mlb_batch_create")
        self.h = h

    def set_exec_opts(self, tile_rows=27, tblock=1, use_graph=True, graph_chunk=64, blocks_per_cu=3,
                      persistent=0):
        o = ExecOpts(tile_rows, tblock, int(use_graph), graph_chunk, blocks_per_cu, int(persistent))
        _check(lib().mlb_batch_set_exec_opts(self.h, C.byref(o)), "mlb_batch_set_exec_opts")

    def autotune(self, steps: int = 20, cache_path: Optional[str] = None) -> dict:
        o = ExecOpts()
        _check(lib().mlb_batch_autotune(self.h, int(steps), None if cache_path is None else cache_path.encode(),
                                        C.byref(o)), "mlb_batch_autotune")
        return o.as_dict()

    def step(self, n: int = 1):
        _check(lib().mlb_batch_step(self.h, int(n)), "mlb_batch_step")

    def run_steady(self, tol: float, max_steps: int, check_every: int = 100):
        ds = (Diag * len(self.grids))()
        rc = lib().mlb_batch_run_steady(self.h, tol, int(max_steps), int(check_every), ds)
        if rc == -7:
            return False, [d.as_dict() for d in ds]
        _check(rc, "mlb_batch_run_steady")
        return True, [d.as_dict() for d in ds]

    def close(self):
        if self.h:
            _check(lib().mlb_batch_destroy(self.h), "mlb_batch_destroy")
            self.h = None


def plan_tiles(params: Params, tile_rows: int, tblock: int, kind=None) -> np.ndarray:
    """The wave tiles of a grid (no device needed): rows of (x0, y0, rows, xo, yo, flags)."""
    kp, kld = None, 0
    if kind is not None:
        ka = np.ascontiguousarray(np.asarray(kind).reshape(params.ny, params.nx), np.uint8)
        kp, kld = ka.ctypes.data_as(C.POINTER(C.c_uint8)), params.nx
    n = C.c_int64()
    _check(lib().mlb_plan_tiles(C.byref(params), kp, kld, int(tile_rows), int(tblock), None, 0, C.byref(n)),
           "mlb_plan_tiles")
    out = np.zeros((max(n.value, 1), 6), np.int32)
    _check(lib().mlb_plan_tiles(C.byref(params), kp, kld, int(tile_rows), int(tblock),
                                out.ctypes.data_as(C.POINTER(C.c_int32)), n.value, C.byref(n)), "mlb_plan_tiles")
    return out[:n.value]


def plan_workqueue(params: Params, tile_rows: int, tblock: int, kind=None):
    """The work-queue dependency lists of a grid (no device needed): (off, nbr)
    with tile t's list nbr[off[t]:off[t+1]] over the tiles of plan_tiles."""
    kp, kld = None, 0
    if kind is not None:
        ka = np.ascontiguousarray(np.asarray(kind).reshape(params.ny, params.nx), np.uint8)
        kp, kld = ka.ctypes.data_as(C.POINTER(C.c_uint8)), params.nx
    nt, nn = C.c_int64(), C.c_int64()
    _check(lib().mlb_plan_workqueue(C.byref(params), kp, kld, int(tile_rows), int(tblock), None, 0, None, 0,
                                    C.byref(nt), C.byref(nn)), "mlb_plan_workqueue")
    off = np.zeros(nt.value + 1, np.int32)
    nbr = np.zeros(max(nn.value, 1), np.int32)
    _check(lib().mlb_plan_workqueue(C.byref(params), kp, kld, int(tile_rows), int(tblock),
                                    off.ctypes.data_as(C.POINTER(C.c_int32)), off.size,
                                    nbr.ctypes.data_as(C.POINTER(C.c_int32)), nbr.size, C.byref(nt), C.byref(nn)),
           "mlb_plan_workqueue")
    return off, nbr[:nn.value]


def grid_from_spec(ctx: Context, spec, workspace=None) -> Grid:
    """A Grid set up from a workloads.Spec (bed, forcing, edges, initial state)."""
    p = make_params(spec.nx, spec.ny, spec.dx, spec.nu, spec.zeta_ref, spec.edges, spec.extrap_order,
                    omega=spec.omega)
    g = Grid(ctx, p, workspace)
    g.set_bathymetry(spec.zb)
    if getattr(spec, "kind", None) is not None:
        g.set_mask(spec.kind)
    if getattr(spec, "hbar_implicit", False):
        g.set_hbar(True)
    if getattr(spec, "compensated", False):
        g.set_surface(True)
    if spec.wind_speed is not None:
        g.set_wind(*spec.wind_speed)
    if spec.wind_stress is not None:
        g.set_wind_stress(*spec.wind_stress)
    g.set_chezy(spec.chezy)
    for k, (hm, amp, per, ph) in spec.depth_bc.items():
        g.set_edge_depth(k, hm, amp, per, ph)
    for k, (a, b) in spec.discharge_bc.items():
        g.set_edge_discharge(k, a, b)
    h, qx, qy = spec.initial()
    g.set_state(h, qx, qy)
    return g


class Elab:
    """The eLABSWE baseline (nine stored distributions, relaxation time tau)
    on a grid's geometry and forcing; starts from f = f^eq of its state."""

    def __init__(self, grid: "Grid", tau: float):
        self.grid = grid
        h = _VP()
        _check(lib().mlb_elab_create(grid.h, float(tau), C.byref(h)), "mlb_elab_create")
        self.h = h

    def step(self, n: int):
        _check(lib().mlb_elab_step(self.h, int(n)), "mlb_elab_step")

    def get_state(self):
        g = self.grid
        h = np.empty((g.ny, g.nx)); qx = np.empty_like(h); qy = np.empty_like(h)
        _check(lib().mlb_elab_get_state(self.h, _dptr(h), _dptr(qx), _dptr(qy), g.nx), "mlb_elab_get_state")
        return h, qx, qy

    def get_dist(self, out):
        """Distributions [9][ny][nx] into a torch CUDA float32 tensor (or a device pointer)."""
        ptr = out if isinstance(out, int) else out.data_ptr()
        _check(lib().mlb_elab_get_dist_device(self.h, ptr), "mlb_elab_get_dist_device")

    def close(self):
        if self.h:
            _check(lib().mlb_elab_destroy(self.h), "mlb_elab_destroy")
            self.h = None


class Net:
    """The warm-start encoder-decoder (BF16 MFMA kernels, FP32 masters).
    Tensors passed in are torch CUDA float32 tensors (or raw device pointers)."""

    def __init__(self, ctx: Context, height: int, width: int, base_ch: int = 32, levels: int = 4,
                 in_ch: int = 32, max_batch: int = 8, seed: int = 0):
        self.ctx = ctx
        self.cfg = NetCfg(height, width, in_ch, 3, base_ch, levels, max_batch)
        h = _VP()
        _check(lib().mlb_net_create(ctx.h, C.byref(self.cfg), int(seed), C.byref(h)), "mlb_net_create")
        self.h = h
        n = C.c_int64()
        _check(lib().mlb_net_param_count(self.h, C.byref(n)), "mlb_net_param_count")
        self.nparam = n.value

    def get_params(self) -> np.ndarray:
        a = np.empty(self.nparam, np.float32)
        _check(lib().mlb_net_get_params(self.h, a.ctypes.data_as(C.POINTER(C.c_float)), self.nparam),
               "mlb_net_get_params")
        return a

    def set_params(self, theta):
        a = np.ascontiguousarray(theta, np.float32)
        _check(lib().mlb_net_set_params(self.h, a.ctypes.data_as(C.POINTER(C.c_float)), a.size),
               "mlb_net_set_params")

    def set_norm(self, in_mean, in_std, s_eta, s_q, tau_ref=0.0):
        """in_mean / in_std: H, tau_x/rho, tau_y/rho, |tau|/rho, C_b."""
        nm = NetNorm()
        for k in range(5):
            nm.in_mean[k], nm.in_std[k] = float(in_mean[k]), float(in_std[k])
        nm.s_eta, nm.s_q, nm.tau_ref = float(s_eta), float(s_q), float(tau_ref)
        _check(lib().mlb_net_set_norm(self.h, C.byref(nm)), "mlb_net_set_norm")

    def get_norm(self) -> dict:
        nm = NetNorm()
        _check(lib().mlb_net_get_norm(self.h, C.byref(nm)), "mlb_net_get_norm")
        return {"in_mean": list(nm.in_mean), "in_std": list(nm.in_std), "s_eta": nm.s_eta, "s_q": nm.s_q,
                "tau_ref": nm.tau_ref}

    def forward(self, x, n, y):
        _check(lib().mlb_net_forward(self.h, _tensor_ptr(x), int(n), _tensor_ptr(y)), "mlb_net_forward")

    def loss_grad(self, x, t, n, mask=None, mask_count=0.0, want_grad=False):
        """Returns (loss, gradient as numpy or None)."""
        loss = C.c_double()
        g = np.empty(self.nparam, np.float32) if want_grad else None
        _check(lib().mlb_net_loss_grad(self.h, _tensor_ptr(x), _tensor_ptr(t), _tensor_ptr(mask),
                                       float(mask_count), int(n), C.byref(loss),
                                       None if g is None else g.ctypes.data_as(C.POINTER(C.c_float))),
               "mlb_net_loss_grad")
        return loss.value, g

    def adamw(self, lr, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0):
        a = AdamWCfg(lr, beta1, beta2, eps, weight_decay)
        _check(lib().mlb_net_adamw(self.h, C.byref(a)), "mlb_net_adamw")

    def features(self, grid, x):
        _check(lib().mlb_net_features(self.h, grid.h, _tensor_ptr(x)), "mlb_net_features")

    def targets(self, grid, t):
        _check(lib().mlb_net_targets(self.h, grid.h, _tensor_ptr(t)), "mlb_net_targets")

    def infer(self, grid):
        _check(lib().mlb_net_infer(self.h, grid.h), "mlb_net_infer")

    def train(self, x, t, n, epochs, batch, lr, lr_min=0.0, warmup_steps=0, beta1=0.9, beta2=0.999,
              eps=1e-8, weight_decay=0.0, seed=0, mask=None):
        """AdamW training over device-resident samples; returns the per-epoch mean loss."""
        cfg = TrainCfg(int(epochs), int(batch), lr, lr_min, int(warmup_steps), beta1, beta2, eps,
                       weight_decay, int(seed))
        el = np.zeros(int(epochs))
        _check(lib().mlb_net_train(self.h, _tensor_ptr(x), _tensor_ptr(t), _tensor_ptr(mask), int(n),
                                   C.byref(cfg), _dptr(el)), "mlb_net_train")
        return el

    def warm_start_run(self, grid, tol, max_steps, check_every=100):
        """Returns (converged, report dict); raises on errors other than
        MLB_E_NOTCONVERGED."""
        r = WarmReport()
        rc = lib().mlb_warm_start_run(grid.h, self.h, tol, int(max_steps), int(check_every), C.byref(r))
        if rc in (-7, -8):
            out = r.as_dict()
            out["stalled"] = rc == -8
            return False, out
        _check(rc, "mlb_warm_start_run")
        out = r.as_dict()
        out["stalled"] = False
        return True, out

    def save(self, path):
        _check(lib().mlb_net_save(self.h, path.encode()), "mlb_net_save")

    def load(self, path):
        _check(lib().mlb_net_load(self.h, path.encode()), "mlb_net_load")

    def close(self):
        if self.h:
            _check(lib().mlb_net_destroy(self.h), "mlb_net_destroy")
            self.h = None
