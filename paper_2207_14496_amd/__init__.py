"""MI355X-native free-surface lattice Boltzmann step (Schwarzmeier & Ruede,
arXiv 2207.14496): HIP kernels for gfx950 behind a small C ABI.

Submodules:
  ``fslbm``   ctypes binding of the C ABI (loads ``libfslbm.so``; raises if missing)
  ``setups``  seeded synthetic initial states of the workloads
The binding is imported lazily so that ``setups`` can be used without a GPU.
"""
__all__ = ["fslbm", "setups"]


def __getattr__(name):
    if name in __all__:
        import importlib
        return importlib.import_module(f".{name}", __name__)
    raise AttributeError(name)
