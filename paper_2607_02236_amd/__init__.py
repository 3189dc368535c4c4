"""MI355X-native TACAW spectral hot path (exit-wave series -> S(k, omega) -> detector spectra).

The compute path is the HIP library libtacaw.so (C ABI in include/tacaw.h);
``tacaw`` is its thin ctypes binding, ``detectors`` builds mask arrays,
``axes`` gives the frequency/energy coordinates of the output bins and
``autograd`` wraps the hand-written adjoint as a torch.autograd.Function and
``workloads`` names plan shapes (benchmark workloads, the paper's settings).
"""

from . import axes, detectors, workloads  # noqa: F401

__all__ = ["axes", "detectors", "workloads", "tacaw", "autograd"]


def __getattr__(name):
    if name in ("tacaw", "autograd"):
        import importlib

        return importlib.import_module(f".{name}", __name__)
    raise AttributeError(name)
