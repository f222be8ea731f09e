"""nusht: nonuniform spherical harmonic transforms (spin 0 and spin s) on one MI355X (gfx950).

Thin Python binding over the C ABI of ``libnusht.so`` (declared in ``include/nusht.h``):
argument marshalling only.  Every step of a transform runs in the library's HIP kernels
and rocFFT; torch supplies device memory and the current stream.  Importing this package
does not load the library; the first call does, and raises if it is missing.

Method: arXiv:2406.14542 (cuNUSHT), Sec. II.B: synthesis Y = N F D S (Eq. 5) and its
adjoint Y^H = S^H D^H F^H N^H (Eq. 6); spin-weighted fields through Wigner's d in place of
the Legendre step (the spin-n extension named in Sec. V).
"""
from __future__ import annotations

from ._binding import (  # noqa: F401
    NUSHT_DFS_FUSED, NUSHT_DFS_PAPER, NUSHT_EDEVICE, NUSHT_EINVAL, NUSHT_ENOCONV, NUSHT_ENOMEM,
    NUSHT_EPRECISION, NUSHT_F64, NUSHT_MAX_SPIN, NUSHT_MIXED, NUSHT_OK, NushtError, Plan, adam_step, deflect,
    density_map, density_map_noalloc, geometry, lib, library_path, mlp_backward, mlp_forward,
    mlp_param_count, nalm, point_features,
)
