"""MI355X-native hot path of FL-MISR's SCG solve (multi-image super-resolution).

``misr``   -- ctypes binding over the C ABI of ``libmisr.so`` (HIP kernels).
``synth``  -- seeded synthetic inputs (phantoms, shifts, PSF taps, noise).
"""
