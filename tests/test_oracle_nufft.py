"""Pins of the plain CPU NUFFT-based SHT (``oracle.nufft_sht``).

The module follows Sect. 3 step by step in FP64.  It is tied here to facts outside
itself: the kernel's Fourier transform against a 30-digit adaptive quadrature
(mpmath), both NUFFT steps against brute-force Fourier sums on small grids, the
type-1 step as the exact transpose of the type-2 step, the whole transform against
the direct-sum oracle (which has its own pins), and adjointness of the pair.  A
wrong doubling sign, a missing normalisation, a transposed grid or an off-by-one
window breaks one of them.
"""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle
from oracle import nufft_sht as o8

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


@pytest.mark.parametrize("w,n", [(7, 64), (12, 96), (16, 200)])
def test_kernel_transform_vs_adaptive_quadrature(w, n):
    beta = 2.3 * w
    ks = np.array([0, 1, 5, n // 8, n // 4])
    J = o8.kernel_ft(ks, n, w, beta)
    with mp.workdps(30):
        for k, j in zip(ks, J):
            ref = mp.quad(lambda z: mp.exp(beta * (mp.sqrt(1 - z * z) - 1))
                          * mp.cos(mp.pi * int(k) * w * z / n), [-1, 0, 1])
            assert abs(j - float(ref)) <= 2e-14 * abs(float(ref)), (w, k, j, ref)


def _fourier_sum(c, th, ph):
    K, M = (c.shape[0] - 1) // 2, (c.shape[1] - 1) // 2
    E1 = np.exp(1j * np.outer(th, np.arange(-K, K + 1)))
    E2 = np.exp(1j * np.outer(ph, np.arange(-M, M + 1)))
    return np.einsum("ik,km,im->i", E1, c, E2)


# (w, measured 2-D type-2 error at oversampling ~2 is below this bound)
@pytest.mark.parametrize("w,bound", [(7, 3e-6), (12, 5e-11)])
def test_nufft_steps_vs_brute_force(w, bound):
    rng = np.random.default_rng(11)
    K, M = 20, 15
    c = rng.standard_normal((2 * K + 1, 2 * M + 1)) + 1j * rng.standard_normal((2 * K + 1, 2 * M + 1))
    th = rng.uniform(0, np.pi, 1000)
    ph = rng.uniform(-1.0, 7.0, 1000)        # phi outside [0, 2 pi) wraps
    th[:2] = [0.0, np.pi]
    n1, n2 = 82, 62
    ref = _fourier_sum(c, th, ph)
    f = o8.nufft_type2(c, th, ph, n1, n2, w, 2.3 * w)
    assert np.linalg.norm(f - ref) <= bound * np.linalg.norm(ref)
    y = rng.standard_normal(1000) + 1j * rng.standard_normal(1000)
    c1 = o8.nufft_type1(y, th, ph, K, M, n1, n2, w, 2.3 * w)
    E1 = np.exp(-1j * np.outer(th, np.arange(-K, K + 1)))
    E2 = np.exp(-1j * np.outer(ph, np.arange(-M, M + 1)))
    ref1 = np.einsum("ik,i,im->km", E1, y, E2)
    assert np.linalg.norm(c1 - ref1) <= bound * np.linalg.norm(ref1)
    # the type-1 step is the exact transpose of the type-2 step
    lhs = np.vdot(y, f)
    rhs = np.vdot(c1, c)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


@pytest.mark.parametrize("spin,lmax,mmax", [(0, 40, 40), (1, 33, 20), (2, 40, 33), (3, 25, 25)])
def test_nufft_sht_vs_direct_sum(spin, lmax, mmax):
    rng = np.random.default_rng(100 + spin)
    nc = oracle.ncomp(spin)
    na = oracle.nalm(lmax, mmax)
    a = rng.standard_normal((nc, na)) + 1j * rng.standard_normal((nc, na))
    th = np.arccos(rng.uniform(-1, 1, 1500))
    ph = rng.uniform(0, 2 * np.pi, 1500)
    th[:4] = [0.0, np.pi, 1e-9, np.pi - 1e-7]
    p = o8.default_params(lmax, mmax, 1e-10)
    assert p["w"] == 12
    ref = oracle.synth(a, lmax, mmax, spin, th, ph)
    f = o8.synth(a, lmax, mmax, spin, th, ph, **p)
    assert oracle.eps_eff(f, ref) <= 1e-10
    y = rng.standard_normal((nc, th.size))
    wts = np.sqrt(oracle.alm_weights(lmax, mmax))[None, :]
    ra = oracle.adjoint(y, lmax, mmax, spin, th, ph)
    b = o8.adjoint(y, lmax, mmax, spin, th, ph, **p)
    assert oracle.eps_eff(wts * b, wts * ra) <= 1e-10
    # the pair is adjoint under the coefficient inner product with w_0 = 1, w_m>0 = 2
    lhs = float(np.sum(y * f))
    rhs = oracle.alm_inner(a, b, lmax, mmax)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_nufft_sht_accuracy_follows_kernel_width():
    """At w = 7 the same steps give the 1e-5 class of accuracy, and never better than
    the kernel allows: the error is the NUFFT's, not the Legendre step's."""
    rng = np.random.default_rng(5)
    lmax = mmax = 48
    a = rng.standard_normal((2, oracle.nalm(lmax, mmax))) * (1 + 1j)
    th = np.arccos(rng.uniform(-1, 1, 1000))
    ph = rng.uniform(0, 2 * np.pi, 1000)
    ref = oracle.synth(a, lmax, mmax, 2, th, ph)
    p = o8.default_params(lmax, mmax, 1e-5)
    assert p["w"] == 7
    e7 = oracle.eps_eff(o8.synth(a, lmax, mmax, 2, th, ph, **p), ref)
    assert 1e-8 < e7 <= 1e-5
    p["ntheta"] += 7           # any ntheta >= lmax + 2 is exact
    e7b = oracle.eps_eff(o8.synth(a, lmax, mmax, 2, th, ph, **p), ref)
    assert abs(e7b - e7) <= 0.05 * e7


def test_nufft_sht_grid_round_trip():
    """Undeflected Gauss-Legendre grid: adjoint(W * synth(a)) = a to the NUFFT's
    accuracy (W = quadrature weight x 2 pi / nphi)."""
    lmax = mmax = 30
    spin = 2
    x, wq = np.polynomial.legendre.leggauss(lmax + 1)
    nphi = 2 * mmax + 2
    th = np.repeat(np.arccos(x), nphi)
    ph = np.tile(2 * np.pi * np.arange(nphi) / nphi, lmax + 1)
    W = np.repeat(wq, nphi) * 2 * np.pi / nphi
    rng = np.random.default_rng(9)
    a = rng.standard_normal((2, oracle.nalm(lmax, mmax))) + 1j * rng.standard_normal((2, oracle.nalm(lmax, mmax)))
    for blk in a:
        for m in range(mmax + 1):
            i0 = oracle.alm_index(m, m, lmax)
            if m == 0:
                blk[i0:i0 + lmax + 1] = blk[i0:i0 + lmax + 1].real
            blk[i0:i0 + max(0, spin - m)] = 0
    p = o8.default_params(lmax, mmax, 1e-10)
    f = o8.synth(a, lmax, mmax, spin, th, ph, **p)
    back = o8.adjoint(W[None, :] * f, lmax, mmax, spin, th, ph, **p)
    wts = np.sqrt(oracle.alm_weights(lmax, mmax))[None, :]
    assert oracle.eps_eff(wts * back, wts * a) <= 1e-10
