"""MI355X-native Bloch-CAP transmission: T(E,k) = 4 Tr[Gamma_L G Gamma_R G^+]
by Krylov solves over the absorbing-boundary columns, in hand-written gfx950
HIP kernels behind the C-ABI library librst.so.

Importing the package is cheap; the HIP library is loaded by
``paper_2208_02783_amd.rst`` on first use and raises if it is missing.
"""
__version__ = "0.1.0"
