"""FP64 CPU reference of the lensing geometry -- TEST INFRASTRUCTURE ONLY.

Only ``tests/`` use this module; it shares no code with the GPU library.

Sect. 2: the lensed field at n is the unlensed field at n', the point at distance
|alpha| from n along the great circle in the direction of the deflection alpha,
times e^{i s chi} for a spin-s field, where chi = beta - beta' is the difference of
the angles that great circle makes with the local e_theta at n and at n'.  The end
of Sect. 3 gives n' = cos(a) n + (sin(a)/a) (alpha_theta e_theta + alpha_phi e_phi)
and the deflection as the spin-1 synthesis of sqrt(L (L+1)) (phi_LM + i Omega_LM)
in the sign convention of eq. forwardpol (eq. deflect).

Everything here is plain numpy in global Cartesian coordinates.
"""
from __future__ import annotations

import numpy as np

from . import adjoint, alm_index, nalm, ncomp, synth


def basis(theta, phi):
    """Unit vector n and the local basis (e_theta, e_phi), each [3][npts]."""
    st, ct, sp, cp = np.sin(theta), np.cos(theta), np.sin(phi), np.cos(phi)
    n = np.array([st * cp, st * sp, ct])
    et = np.array([ct * cp, ct * sp, -st])
    ep = np.array([-sp, cp, np.zeros_like(st)])
    return n, et, ep


def lscale(alm, lmax: int, mmax: int):
    """sqrt(l (l + 1)) alm for every stored coefficient ([ncomp][nalm])."""
    out = np.array(alm, dtype=np.complex128, copy=True)
    for m in range(mmax + 1):
        i0 = alm_index(m, m, lmax)
        ls = np.arange(m, lmax + 1)
        out[..., i0:i0 + ls.size] *= np.sqrt(ls * (ls + 1.0))
    return out


def deflection_field(plm, lmax: int, mmax: int, theta, phi, olm=None, nthreads: int = 0):
    """(alpha_theta, alpha_phi) [2][npts]: spin-1 direct-sum synthesis of
    sqrt(L (L+1)) (phi_LM, Omega_LM) as gradient and curl coefficients."""
    g = np.zeros((2, nalm(lmax, mmax)), dtype=np.complex128)
    g[0] = plm
    if olm is not None:
        g[1] = olm
    return synth(lscale(g, lmax, mmax), lmax, mmax, 1, theta, phi, nthreads)


def deflect(theta, phi, alpha):
    """Deflected positions (theta', phi' in [0, 2 pi)) and the spin phase chi."""
    at, ap = np.asarray(alpha[0], float), np.asarray(alpha[1], float)
    n, et, ep = basis(theta, phi)
    a = np.hypot(at, ap)
    safe = np.where(a > 0, a, 1.0)
    sinc = np.where(a > 0, np.sin(a) / safe, 1.0)
    d = at * et + ap * ep                                   # alpha as a 3-vector
    n2 = np.cos(a) * n + sinc * d
    th2 = np.arctan2(np.hypot(n2[0], n2[1]), n2[2])
    ph2 = np.mod(np.arctan2(n2[1], n2[0]), 2 * np.pi)
    # direction of the great circle: at n along alpha (beta from e_theta towards e_phi);
    # at n' the tangent d/ds [cos(s) n + sin(s) ahat] at s = a
    ahat = np.where(a > 0, d / safe, et)
    beta = np.arctan2(ap, at)
    t2 = -np.sin(a) * n + np.cos(a) * ahat
    _, et2, ep2 = basis(th2, ph2)
    beta2 = np.arctan2(np.sum(t2 * ep2, axis=0), np.sum(t2 * et2, axis=0))
    chi = np.angle(np.exp(1j * (beta - beta2)))
    chi = np.where(a > 0, chi, 0.0)
    return th2, ph2, chi


def lensed_synth(alm, lmax: int, mmax: int, spin: int, theta, phi, alpha, nthreads: int = 0):
    """Eq. forward / eq. forwardpol: the unlensed field at n', times e^{i s chi}."""
    th2, ph2, chi = deflect(theta, phi, alpha)
    m = synth(alm, lmax, mmax, spin, th2, ph2, nthreads)
    if spin:
        p = (m[0] + 1j * m[1]) * np.exp(1j * spin * chi)
        m = np.stack([p.real, p.imag])
    return m


def lensed_adjoint(maps, lmax: int, mmax: int, spin: int, theta, phi, alpha, nthreads: int = 0):
    """Adjoint of lensed_synth (eq. adjoint and its spin-s form with e^{-i s chi})."""
    th2, ph2, chi = deflect(theta, phi, alpha)
    y = np.asarray(maps, float).reshape(ncomp(spin), -1)
    if spin:
        p = (y[0] + 1j * y[1]) * np.exp(-1j * spin * chi)
        y = np.stack([p.real, p.imag])
    return adjoint(y, lmax, mmax, spin, th2, ph2, nthreads)


def transport(v, n, ahat, a, steps: int = 2000):
    """Parallel transport of the tangent vectors v (at n) along the great circles
    n(s) = cos(s) n + sin(s) ahat, s in [0, a], by integrating dv/ds = -(v . t) n(s)
    (t = dn/ds) with classical Runge-Kutta steps: a brute-force reference that uses
    no closed form of the transport."""
    v = np.array(v, float)
    h = a / steps

    def f(s, vv):
        ns = np.cos(s) * n + np.sin(s) * ahat
        ts = -np.sin(s) * n + np.cos(s) * ahat
        return -np.sum(vv * ts, axis=0) * ns

    s = np.zeros_like(a)
    for _ in range(steps):
        k1 = f(s, v)
        k2 = f(s + h / 2, v + h / 2 * k1)
        k3 = f(s + h / 2, v + h / 2 * k2)
        k4 = f(s + h, v + h * k3)
        v = v + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
        s = s + h
    return v


def lfactor(alm, lmax: int, mmax: int, kind: int):
    """f_l alm: kind 1 -> l (l+1) / 2, kind 2 -> sqrt((l-1) l (l+1) (l+2)) / 2."""
    out = np.array(alm, dtype=np.complex128, copy=True)
    for m in range(mmax + 1):
        i0 = alm_index(m, m, lmax)
        ls = np.arange(m, lmax + 1).astype(float)
        f = 0.5 * ls * (ls + 1) if kind == 1 else 0.5 * np.sqrt(np.maximum((ls - 1) * ls * (ls + 1) * (ls + 2), 0))
        out[..., i0:i0 + ls.size] *= f
    return out


def magnification(plm, lmax: int, mmax: int, theta, phi, olm=None):
    """Appendix B: |A| from the convergence kappa (+ i omega) = (1/2) eth-bar of the
    spin-1 deflection and the shear gamma = (1/2) eth of it, i.e. the spin-0 synthesis
    of l(l+1)/2 (phi, Omega) and the spin-2 synthesis of sqrt((l-1)l(l+1)(l+2))/2
    (phi, Omega) in the sign convention of eq. forwardpol."""
    alpha = deflection_field(plm, lmax, mmax, theta, phi, olm)
    kappa = synth(lfactor(plm[None, :], lmax, mmax, 1), lmax, mmax, 0, theta, phi)[0]
    omega = 0.0 if olm is None else synth(lfactor(olm[None, :], lmax, mmax, 1), lmax, mmax, 0, theta, phi)[0]
    g = np.zeros((2, nalm(lmax, mmax)), complex)
    g[0] = plm
    if olm is not None:
        g[1] = olm
    gam = synth(lfactor(g, lmax, mmax, 2), lmax, mmax, 2, theta, phi)
    a = np.hypot(alpha[0], alpha[1])
    safe = np.where(a > 0, a, 1.0)
    sc = np.where(a > 0, np.sin(a) / safe, 1.0)
    beta = np.arctan2(alpha[1], alpha[0])
    return (sc * ((1 - kappa) ** 2 + omega ** 2 - gam[0] ** 2 - gam[1] ** 2)
            + (np.cos(a) - sc) * (1 - kappa - np.cos(2 * beta) * gam[0] - np.sin(2 * beta) * gam[1]))


def magnification_fd(plm, lmax: int, mmax: int, theta, phi, olm=None, h: float = 1e-5):
    """The Jacobian determinant d^2 n' / d^2 n (signed: negative where the remapping
    folds) by central differences of the deflected point (unit vectors):
    ((dn'/dtheta x dn'/dphi) . n') / sin(theta)."""
    def npos(t, p):
        al = deflection_field(plm, lmax, mmax, t, p, olm)
        t2, p2, _ = deflect(t, p, al)
        return basis(t2, p2)[0]
    dt = (npos(theta + h, phi) - npos(theta - h, phi)) / (2 * h)
    dp = (npos(theta, phi + h) - npos(theta, phi - h)) / (2 * h)
    n2 = npos(theta, phi)
    cr = np.cross(dt.T, dp.T).T
    return np.sum(cr * n2, axis=0) / np.sin(theta)
