"""MI355X-native D2Q9 lattice Boltzmann hot path (PortLBM paper, arXiv 2607.20650).

The update runs in hand-written gfx950 HIP kernels behind the C ABI of
``include/lbm.h`` (``liblbm.so``); :mod:`.lbm` is its ctypes binding and
:mod:`.workloads` generates the seeded synthetic inputs.  Importing the
package loads nothing; the library is loaded on first use.
"""

__all__ = ["lbm", "workloads"]
