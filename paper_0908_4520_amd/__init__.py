"""MI355X (gfx950) BGK step for high-order lattice Boltzmann and discrete-velocity models.

The compute path is the HIP library ``liblbm.so`` behind the C ABI in ``include/lbm.h``;
``paper_0908_4520_amd.lbm`` is its ctypes binding.  Build with ``paper_0908_4520_amd.build``.
"""
