"""MI355X-native cyclic coordinate descent for the Bayesian self-controlled
case series model (Suchard et al., "Massive parallelization of serial
inference algorithms for a complex generalized linear model").

The compute path is the HIP library ``libsccs.so`` behind the C ABI declared
in ``include/sccs.h``; ``paper_1208_0945_amd.sccs`` is its thin ctypes
binding.  Importing this package loads nothing; the library is opened on
first use.
"""
__all__ = ["synth", "sccs"]
