"""Shared test plumbing: build the oracle and the GPU grid from one workload spec."""
import numpy as np

import oracle


# the oracle problem of a workload spec (kept under this name for the tests)
oracle_from_spec = oracle.from_spec


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
