"""MI355X (gfx950) SpAMM and Newton-Schulz square-root iteration.

``spamm`` is the binding over the HIP library (include/spamm.h); ``inputs``
builds the seeded synthetic workloads; ``build`` compiles the library.
Importing the package loads nothing; the library is loaded on first use.
"""
__all__ = ["spamm", "inputs", "build"]
