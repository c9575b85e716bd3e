"""MI355X-native Newton-system solve for arrowhead LPs with local linking.

Submodules (imported explicitly; nothing heavy is loaded here):
  gen   seeded synthetic instances with a known optimum
  ahlp  ctypes binding of the C-ABI library libahlp.so (HIP kernels, gfx950)
"""
