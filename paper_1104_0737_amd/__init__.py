"""MI355X-native modified block BiCGSTAB with SAP preconditioning for the
Wilson-Dirac equation (Nakamura et al., Sec. 2): HIP kernels for gfx950 behind
a C ABI (include/mbbs.h), with a thin ctypes binding in `binding`.

Importing the package loads nothing; `binding.lib()` loads libmbbs.so and
raises if it has not been built.
"""
