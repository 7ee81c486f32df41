"""MI355X-native ladder dual-fermion hot path (HIP kernels behind a C ABI).

Submodules:
  inputs   seeded synthetic inputs (Hubbard-atom g, Delta, vertices; dispersion)
  binding  ctypes binding of libdf.so (df_dual_gf, df_bubble, df_ladder_solve,
           df_sigma, df_iterate)
  build    in-tree build of libdf.so for gfx950

Importing the package loads nothing; the binding loads libdf.so on first use.
"""
__all__ = ["inputs", "binding", "build"]
