"""MI355X-native batched FP16 FFT on the matrix cores (tcFFT method).

The product path is the HIP library ``libtcfft.so`` (kernels + C-ABI) and the
thin ctypes binding in :mod:`paper_2104_11471_amd.tcfft`.  Importing this
package loads nothing; :mod:`paper_2104_11471_amd.tcfft` loads the library and
fails loudly when it is missing.
"""
__all__ = ["tcfft", "inputs"]
