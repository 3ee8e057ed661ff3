"""lbch: anisotropic Cahn-Hilliard MRT lattice Boltzmann on AMD MI355X (gfx950).

The compute path is the C-ABI shared library ``liblbch.so`` built from
``csrc/`` (hand-written HIP kernels); ``lbch`` is its thin ctypes binding.
``inputs`` holds the seeded synthetic workload generators and nothing of the
method's arithmetic.  Submodules are imported lazily so that importing the
package does not load the GPU runtime.
"""
import importlib

__all__ = ["lbch", "inputs", "build"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f".{name}", __name__)
    raise AttributeError(name)
