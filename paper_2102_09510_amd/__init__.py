"""MI355X-native quasi-greedy many-clone 3-XORSAT solver (arXiv 2102.09510).

Submodules
  xorsat     ctypes binding of libxorsat.so (the C ABI in include/xorsat.h)
  instances  seeded synthetic planted instances (inputs only)
  build      hipcc build of libxorsat.so for gfx950

Importing the package loads nothing; ``xorsat.load()`` loads the HIP library.
"""
