"""MI355X-native MacLABSWE streaming-only D2Q9 step (Zhou, arXiv 1902.02999).

The step runs in hand-written HIP kernels for gfx950 behind a C ABI
(``include/mlb.h``, built into ``libmlb.so`` next to this file).  ``mlb`` is a
thin ctypes binding with the same call names; ``workloads`` holds the seeded
input generators.  Nothing here falls back to a CPU path: if the library is
missing, loading it raises.
"""
__all__ = ["mlb", "workloads"]


def __getattr__(name):
    if name in ("mlb", "workloads", "warmstart"):
        import importlib
        return importlib.import_module("." + name, __name__)
    raise AttributeError(name)
