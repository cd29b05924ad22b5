"""CPU FP64 oracle for the real-space spherical convolution (test infrastructure).

This package is test infrastructure only. It is imported by the tests, by
the package's smoke check and by the benchmark's CPU-baseline leg, and by
nothing else. The library never calls it and shares no code with it.

What it computes is the plain definition of the operator that the paper's
kernel splitting hands to real space (Estimating Errors section, Eq. 1:
the real-space part of the split kernel, truncated at theta_cut):

    y_p = Omega * sum_{q : d_pq <= d_cut} Ktilde(d_pq) * x_q

with Omega = 4 pi / Npix the pixel area of the equal-area pixelization,
d_pq = |v_p - v_q| the chord between pixel centres, d_cut = 2 sin(theta_cut/2),
and Ktilde the kernel interpolated from a table sampled on a uniform chord grid
(Results section: the real-space convolver interpolates the kernel from a table
of nodes). Every function is written from that definition in FP64, with
no blocking or reordering beyond what the definition needs.

Modules:
  geometry  ring table and pixel centres of the ring-ordered pixelization
  kernel    Legendre-series tabulation of K on chord nodes, 4-point
            interpolation, truncated transfer function k_l^trunc
  convolve  brute-force and ring-exhaustive sampled sums, pair counts
"""
from . import geometry, kernel, convolve  # noqa: F401
