"""MI355X-native F-statistic search for periodic gravitational waves.

The device path is the HIP library libfstat.so (C ABI in include/fstat.h);
`paper_1410_3677_amd.fstat` is its Python binding.  Importing the package
does not load the library.
"""
