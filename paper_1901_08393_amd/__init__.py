"""MI355X (gfx950) P0 Galerkin BEM for the electrostatic capacity of
polyhedra: dense single-layer assembly and persistent Krylov solves in
hand-written HIP behind a C ABI (include/bemcap.h).

Importing the package does not load the library or touch the GPU; the
first call into :mod:`paper_1901_08393_amd.api` does, and fails loudly if
the library is not built.
"""

__all__ = ["api", "adaptive", "serve"]
