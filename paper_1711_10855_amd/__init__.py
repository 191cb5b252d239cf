"""FDAS correlation step (overlap-and-save matched filter) for AMD MI355X.

Submodules:
  fdas   -- ctypes binding of the C ABI in include/fdas.h (libfdas.so)
  synth  -- seeded synthetic inputs (time series, spectra, workload recipes)
  build  -- compiles libfdas.so in-tree with hipcc for gfx950

Importing the package loads nothing; ``fdas.load()`` loads the library.
"""
