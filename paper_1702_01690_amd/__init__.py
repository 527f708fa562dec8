"""MI355X (gfx950) implementation of the D2Q25 off-lattice thermal Boltzmann
stage update of Busuioc, Ambrus, Biciusca and Sofonea (arXiv:1702.01690).

The compute path is the HIP library ``libolb.so`` (sources in ``csrc/``,
C-ABI in ``include/olb.h``); ``olb`` is its ctypes binding.
"""
from .olb import (OLB_BC_DIFFUSE, OLB_BC_PERIODIC, OLB_FP32_MIXED, OLB_FP64, Batch, Lattice,  # noqa: F401
                  OlbError, lib, make_params)
