"""Deflected point sets for the tests, computed with the oracle only (test
infrastructure; not a test module).

The lensing potential comes from the seeded generators; the deflection field is the
spin-1 synthesis of sqrt(L (L + 1)) phi_LM at the undeflected points (eq. deflect),
by the direct sum for small sets and by the plain CPU NUFFT-based SHT for large
ones, and the points move along great circles (end of Sect. 3) with the oracle's
own formula.
"""
import numpy as np

import oracle
from oracle import lensing as ol
from oracle import nufft_sht


def deflect_small(theta, phi, lmax_p: int, seed: int):
    """Direct-sum deflection of a few thousand points by a potential of band limit lmax_p."""
    from paper_2304_10431_amd import workloads as wl
    plm = wl.lensing_potential(lmax_p, seed)
    alpha = ol.deflection_field(plm, lmax_p, lmax_p, theta, phi)
    th, ph, _ = ol.deflect(theta, phi, alpha)
    return th, ph


def deflect_large(theta, phi, plm, lmax_p: int, eps: float = 1e-12):
    """Deflection of millions of points: the spin-1 field by the plain CPU NUFFT-based
    SHT at accuracy eps (FP64), then the great-circle step."""
    g = np.zeros((2, oracle.nalm(lmax_p, lmax_p)), dtype=np.complex128)
    g[0] = plm
    g = ol.lscale(g, lmax_p, lmax_p)
    p = nufft_sht.default_params(lmax_p, lmax_p, eps)
    alpha = nufft_sht.synth(g, lmax_p, lmax_p, 1, theta, phi, **p)
    th, ph, _ = ol.deflect(theta, phi, alpha)
    return th, ph
