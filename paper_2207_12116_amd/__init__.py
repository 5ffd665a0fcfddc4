"""MI355X-native propagate-and-search after "A Variant of Concurrent Constraint
Programming on GPU" (Talbot, Pinel, Bouvry, AAAI 2022).

Modules:
  instances  seeded synthetic models (tiny CSP, RCPSP family)
  pccp       ctypes binding of libpccp.so (HIP kernels + C-ABI)
  build      hipcc build of libpccp.so
"""
