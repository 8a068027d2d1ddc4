"""MI355X-native multigrid interpolative separable density fitting (ISDF)
exchange path: a HIP library (libisdf.so, C ABI in include/isdf.h) plus a
thin ctypes binding.  Importing the package loads nothing; use
``paper_2404_09373_amd.binding``."""
__all__ = ["binding", "build"]
