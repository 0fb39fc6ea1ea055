"""MI355X-native SU(Nc) pure-gauge configuration generation (Wilson action,
checkerboard heatbath / overrelaxation sweep), after Cardoso & Bicudo,
arXiv:1112.4533.

The compute path is the HIP library libsun (C ABI in include/sun.h); the
`sun` module binds it.  Importing this package does not load the library;
`paper_1112_4533_amd.sun.load()` does, and raises if it is not built.
"""
__all__ = ["sun", "workloads", "build"]
