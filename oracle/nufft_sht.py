"""Plain FP64 CPU NUFFT-based general SHT -- TEST INFRASTRUCTURE ONLY.

Only ``tests/`` and the CPU-baseline leg of ``bench.py`` use this module; it shares
no code with the GPU library and never imports it.

It computes the general synthesis and its adjoint the way Sect. 3 of Reinecke,
Belkner & Carron (2023) describes, one step after the other, in FP64:

1. synthesis onto ``ntheta`` equidistant rings theta_j = pi j / (ntheta - 1), both
   poles included, in (theta, m) space (the direct-sum ring synthesis of this
   package, ``ring_synth``);
2. doubling of the theta range to [0, 2 pi): F_m(2 pi - theta) = (-1)^(s+m) F_m(theta),
   the continuation that turns every F_m into a trigonometric polynomial of degree
   lmax in theta;
3. FFT over the nd = 2 ntheta - 2 doubled rings: c_km = (1/nd) sum_j F_m(theta_j)
   e^{-i k theta_j}, kept for |k| <= lmax, so that the map is
   f(theta, phi) = sum_{k,m} c_km e^{i (k theta + m phi)};
4. deconvolution by the kernel's Fourier transform and zero padding onto the
   N1 x N2 torus, inverse FFT, and interpolation with the kernel (type-2 NUFFT).

The adjoint applies the transposes in reverse: spreading (type-1), forward FFT,
truncation and the same real deconvolution factors, inverse length-nd transform,
folding of the doubled rings back onto [0, pi], and the ring adjoint.

Type-2 step, in cell units t (t = theta N / 2 pi): with the kernel
psi(t) = exp(beta (sqrt(1 - (2t/w)^2) - 1)) on |t| <= w/2 and its transform
psihat(k) = int psi(t) e^{-2 pi i k t / N} dt, the trapezoidal rule on the grid
turns the convolution identity f = (f / psihat) * psi into
f(x) = sum_cells g_cell psi(x - cell) with g = inverse DFT of c_k / psihat(k); the
quadrature (aliasing) error is what the kernel parameters control.  Integrated in
z = 2t/w: psihat(k) = (w/2) J(k), J(k) = int_{-1}^{1} phi(z) cos(pi k w z / N) dz, so
the factor applied per dimension is 2 / (w J(k)).  J is computed after the
substitution z = sin(x), which removes the square-root endpoint behaviour of the
kernel, with Gauss-Legendre quadrature.

All parameters (ntheta, N1, N2, w, beta) are explicit arguments.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.fft

from . import _check, _load, _p, ncomp, ring_adjoint, ring_synth


def kernel_ft(k, n: int, w: int, beta: float, nodes: int = 0) -> np.ndarray:
    """J(k) = int_{-1}^{1} exp(beta (sqrt(1 - z^2) - 1)) cos(pi k w z / n) dz, for an
    array of integer frequencies k on a length-n grid."""
    k = np.asarray(k, dtype=np.float64)
    nq = nodes or (4 * w + 60)
    x, wt = np.polynomial.legendre.leggauss(nq)
    t = 0.5 * math.pi * x                 # z = sin(t), t in [-pi/2, pi/2]
    wt = 0.5 * math.pi * wt
    f = np.exp(beta * (np.cos(t) - 1.0)) * np.cos(t)
    z = np.sin(t)
    return (wt * f)[None, :].dot(np.cos(np.pi * w / n * np.outer(z, k))).ravel()


def deconv_factor(kmax: int, n: int, w: int, beta: float) -> np.ndarray:
    """h / psihat(k) = 2 / (w J(k)) for k = -kmax..kmax."""
    k = np.arange(-kmax, kmax + 1)
    return 2.0 / (w * kernel_ft(k, n, w, beta))


def nufft_type2(c, theta, phi, n1: int, n2: int, w: int, beta: float, nthreads: int = 0):
    """f_i ~= sum_{|k|<=K, |m|<=M} c[k + K][m + M] e^{i (k theta_i + m phi_i)}.
    c is [2K+1][2M+1] complex; returns complex [npts]."""
    c = np.asarray(c, dtype=np.complex128)
    K, M = (c.shape[0] - 1) // 2, (c.shape[1] - 1) // 2
    if 2 * K + 1 > n1 or 2 * M + 1 > n2:
        raise ValueError("grid smaller than the band limit")
    ch = c * deconv_factor(K, n1, w, beta)[:, None] * deconv_factor(M, n2, w, beta)[None, :]
    spec = np.zeros((n1, n2), dtype=np.complex128)
    ka = np.arange(-K, K + 1) % n1
    ma = np.arange(-M, M + 1) % n2
    spec[np.ix_(ka, ma)] = ch
    g = np.ascontiguousarray(scipy.fft.ifft2(spec, norm="forward", workers=nthreads or -1))
    del spec
    th = np.ascontiguousarray(theta, dtype=np.float64)
    ph = np.ascontiguousarray(phi, dtype=np.float64)
    out = np.zeros(th.size, dtype=np.complex128)
    _check(_load().gsht_oracle_nufft_interp(_p(g.view(np.float64)), n1, n2, w, float(beta),
                                            th.size, _p(th), _p(ph), _p(out.view(np.float64)),
                                            nthreads), "nufft_interp")
    return out


def nufft_type1(y, theta, phi, K: int, M: int, n1: int, n2: int, w: int, beta: float,
                nthreads: int = 0):
    """Transpose of nufft_type2: c'[k + K][m + M] ~= sum_i y_i e^{-i (k theta_i + m phi_i)}."""
    if 2 * K + 1 > n1 or 2 * M + 1 > n2:
        raise ValueError("grid smaller than the band limit")
    th = np.ascontiguousarray(theta, dtype=np.float64)
    ph = np.ascontiguousarray(phi, dtype=np.float64)
    yc = np.ascontiguousarray(np.asarray(y, dtype=np.complex128).ravel())
    g = np.zeros((n1, n2), dtype=np.complex128)
    _check(_load().gsht_oracle_nufft_spread(_p(yc.view(np.float64)), n1, n2, w, float(beta),
                                            th.size, _p(th), _p(ph), _p(g.view(np.float64))),
           "nufft_spread")
    C = scipy.fft.fft2(g, norm="backward", workers=nthreads or -1)
    del g
    ka = np.arange(-K, K + 1) % n1
    ma = np.arange(-M, M + 1) % n2
    return (C[np.ix_(ka, ma)] * deconv_factor(K, n1, w, beta)[:, None]
            * deconv_factor(M, n2, w, beta)[None, :])


def ring_thetas(ntheta: int) -> np.ndarray:
    """Equidistant rings including both poles: theta_j = pi j / (ntheta - 1)."""
    return np.pi * np.arange(ntheta) / (ntheta - 1)


def _mirror_sign(mmax: int, spin: int) -> np.ndarray:
    m = np.arange(-mmax, mmax + 1)
    return np.where((m + spin) % 2 == 0, 1.0, -1.0)


def synth(alm, lmax: int, mmax: int, spin: int, theta, phi, ntheta: int, n1: int, n2: int,
          w: int, beta: float, nthreads: int = 0) -> np.ndarray:
    """General synthesis through the steps of Sect. 3; returns [ncomp][npts] float64."""
    if ntheta < lmax + 2:
        raise ValueError("need ntheta >= lmax + 2")
    nd = 2 * ntheta - 2
    F = ring_synth(alm, lmax, mmax, spin, ring_thetas(ntheta), nthreads)   # [2mmax+1][ntheta]
    FD = np.empty((2 * mmax + 1, nd), dtype=np.complex128)
    FD[:, :ntheta] = F
    j = np.arange(ntheta, nd)
    FD[:, ntheta:] = _mirror_sign(mmax, spin)[:, None] * F[:, nd - j]
    del F
    ck = scipy.fft.fft(FD, axis=1, workers=nthreads or -1) / nd           # [m][k mod nd]
    del FD
    c = ck[:, np.arange(-lmax, lmax + 1) % nd].T                          # [k][m]
    del ck
    f = nufft_type2(c, theta, phi, n1, n2, w, beta, nthreads)
    if spin == 0:
        return f.real[None, :].copy()
    return np.stack([f.real, f.imag])


def adjoint(maps, lmax: int, mmax: int, spin: int, theta, phi, ntheta: int, n1: int, n2: int,
            w: int, beta: float, nthreads: int = 0) -> np.ndarray:
    """Adjoint of ``synth`` (the transposed steps in reverse); returns [ncomp][nalm]."""
    if ntheta < lmax + 2:
        raise ValueError("need ntheta >= lmax + 2")
    nd = 2 * ntheta - 2
    y = np.asarray(maps, dtype=np.float64).reshape(ncomp(spin), -1)
    yc = y[0] + 1j * y[1] if spin else y[0].astype(np.complex128)
    c = nufft_type1(yc, theta, phi, lmax, mmax, n1, n2, w, beta, nthreads)   # [k][m]
    ck = np.zeros((2 * mmax + 1, nd), dtype=np.complex128)
    ck[:, np.arange(-lmax, lmax + 1) % nd] = c.T
    del c
    HD = scipy.fft.ifft(ck, axis=1, norm="forward", workers=nthreads or -1) / nd
    del ck
    H = HD[:, :ntheta].copy()
    j = np.arange(1, ntheta - 1)
    H[:, j] += _mirror_sign(mmax, spin)[:, None] * HD[:, nd - j]
    del HD
    return ring_adjoint(H, lmax, mmax, spin, ring_thetas(ntheta), nthreads)


def _smooth7(n: int) -> bool:
    for f in (2, 3, 5, 7):
        while n % f == 0:
            n //= f
    return n == 1


def default_params(lmax: int, mmax: int, eps: float) -> dict:
    """This module's own parameter choice: the smallest ntheta >= lmax + 2 with a
    7-smooth doubled length, oversampling 2 with even 7-smooth grid lengths,
    w = ceil(log10(1/eps)) + 2 (one cell above the 1-D rule for the two dimensions),
    beta = 2.3 w."""
    nt = max(lmax + 2, 2)
    while not _smooth7(2 * nt - 2):
        nt += 1
    w = int(math.ceil(math.log10(1.0 / eps))) + 2

    def grid(L):
        n = max(2 * (2 * L + 1), 2 * w + 4)
        while n % 2 or not _smooth7(n):
            n += 1
        return n
    return dict(ntheta=nt, n1=grid(lmax), n2=grid(mmax), w=w, beta=2.3 * w)
