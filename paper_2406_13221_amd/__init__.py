"""MI355X (gfx950) encrypted quadratic-gradient NAG logistic regression (RNS-CKKS).

The compute path is libheqg.so (HIP kernels behind the C ABI in include/heqg.h);
`heqg` is its ctypes binding and `train` drives the paper's pipeline (section 4.3)
on top of it.  Importing the binding loads the library and fails loudly when
it has not been built.
"""
__all__ = ["heqg"]
