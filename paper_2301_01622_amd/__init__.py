"""MI355X-native lattice Boltzmann without populations.

The time step runs in hand-written HIP kernels behind the C ABI of
include/lbm.h (liblbm.so); ``LBM`` is its Python handle.  Importing the
package does not load the library; ``LBM`` does, and raises if it is not
built.
"""

__all__ = ["LBM"]


def __getattr__(name):
    if name == "LBM":
        from .lbm import LBM
        return LBM
    raise AttributeError(name)
