"""MI355X-native coupled photon/electron Monte Carlo dose engine (gDPM method).

The transport runs in hand-written HIP kernels behind the C-ABI library
``libgdpm.so`` (declared in include/gdpm.h); ``paper_1107_3355_amd.gdpm`` is its
ctypes binding.  ``paper_1107_3355_amd.inputs`` builds seeded synthetic inputs.
Importing the package loads nothing; the binding loads the library on first use.
"""
__all__ = ["inputs", "gdpm"]
