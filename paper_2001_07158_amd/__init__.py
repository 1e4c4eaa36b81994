"""MI355X-native temporal path-motif sieve (constrained multilinear sieving over
GF(2^8), hand-written HIP for gfx950) behind the C ABI in include/tpm.h.

`paper_2001_07158_amd.tpm` is the ctypes binding; it raises at import if the HIP
library has not been built.
"""

__all__ = ["tpm"]
