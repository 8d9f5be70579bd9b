"""Shared test plumbing: build the oracle and the GPU grid from one workload spec."""
import numpy as np

import oracle
from paper_1902_02999_amd import workloads as wl


def oracle_from_spec(spec: wl.Spec, h=None, qx=None, qy=None, step0=0) -> "oracle.Basin":
    """The FP64 oracle problem described by a workload spec (the oracle derives
    its own e, dt, wind stress and friction coefficient)."""
    if h is None:
        h, qx, qy = spec.initial()
    tx = ty = 0.0
    if spec.wind_speed is not None:
        tx, ty = oracle.wind_stress(*spec.wind_speed)
    if spec.wind_stress is not None:
        tx, ty = spec.wind_stress
    b = oracle.Basin(spec.nx, spec.ny, spec.dx, spec.nu, spec.zb, tx=tx, ty=ty,
                     cb=oracle.bed_coeff(spec.chezy) if spec.chezy > 0 else 0.0,
                     omega=spec.omega, edges=spec.edges, extrap_order=spec.extrap_order,
                     depth_bc=dict(spec.depth_bc), discharge_bc=dict(spec.discharge_bc),
                     h=h, qx=qx, qy=qy, kind=spec.kind, hbar_implicit=spec.hbar_implicit)
    b.step_index = step0
    return b


def compare(h_gpu, qx_gpu, qy_gpu, h_ref, qx_ref, qy_ref, where=None):
    """Errors in the form the parity bar is stated in: max |dh| / max h and
    max |du| / max |u| (u = q / h, both components); `where` selects the
    nodes compared (default all)."""
    if where is not None:
        h_gpu, qx_gpu, qy_gpu = h_gpu[where], qx_gpu[where], qy_gpu[where]
        h_ref, qx_ref, qy_ref = h_ref[where], qx_ref[where], qy_ref[where]
    dh = np.abs(h_gpu - h_ref).max() / np.abs(h_ref).max()
    u_ref = np.hypot(qx_ref, qy_ref) / h_ref
    du = max(np.abs(qx_gpu / h_gpu - qx_ref / h_ref).max(), np.abs(qy_gpu / h_gpu - qy_ref / h_ref).max())
    umax = u_ref.max()
    return dh, (du / umax if umax > 0 else du)


def gpu_state_as_f64(grid):
    return grid.get_state()
