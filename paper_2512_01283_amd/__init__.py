"""MI355X-native polarized Monte Carlo radiative transfer (two-step imaging).

Submodules:
  polrad     ctypes binding of libpolrad.so (the HIP kernels behind a C ABI)
  workloads  seeded synthetic inputs shared by the HIP path and the oracle
  build      hipcc build of libpolrad.so for gfx950

Nothing is imported eagerly: importing `polrad` loads the compiled library
and fails if it has not been built.
"""
