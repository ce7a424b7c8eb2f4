"""MI355X-native FFT angular-spectrum PSF engine (libdop) and its Python binding.

The propagation itself runs in hand-written HIP kernels behind the C ABI in
include/dop.h; ``paper_2505_22313_amd.api`` loads that library
(paper_2505_22313_amd/libdop.so) on first use and marshals arguments.  It
raises if the library is not built: there is no fallback path.
"""
