"""Electron-phonon scattering self-energy (SSE) on one AMD MI355X.

Hot path of the dissipative NEGF solver of Ziogas et al. (SC'19): the
contraction Sigma^{<>}(E, kz) of Eq. 3, behind a C-ABI HIP library
(``libsse.so``, declared in ``include/sse.h``).  This package holds the seeded
input generators, the flop model and the thin Python binding.
"""
