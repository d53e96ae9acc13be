"""MI355X-native path tracer: HIP kernels behind a C ABI (libpt.so) with a thin ctypes binding.

Importing the package does not load the native library; `paper_2407_19977_amd.pt`
does, and fails loudly if it has not been built.
"""
