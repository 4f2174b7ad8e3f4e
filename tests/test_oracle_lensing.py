"""Pins of the CPU lensing-geometry reference (``oracle.lensing``).

* the deflected point lies on the great circle through n along alpha, at distance
  |alpha| (spherical geometry, independent of the formula's form);
* the deflection field is the gradient of the potential field (eq. deflect with the
  spin-1 sign of eq. forwardpol), checked against the oracle's own derivatives;
* chi = beta - beta' against a brute-force parallel transport (Runge-Kutta on the
  transport equation along the great circle);
* the e^{i s chi} convention against the transport of a genuine vector field: the
  gradient of a scalar field, carried from n' back to n, must equal
  e^{i chi} (d_theta T + i / sin(theta) d_phi T)(n');
* adjointness of the lensed synthesis and its adjoint.
"""
import numpy as np
import pytest

import oracle
from oracle import lensing as ol


def _alm(spin, lmax, mmax, seed, decay=1.0):
    rng = np.random.default_rng(seed)
    nc = oracle.ncomp(spin)
    a = rng.standard_normal((nc, oracle.nalm(lmax, mmax))) + 1j * rng.standard_normal((nc, oracle.nalm(lmax, mmax)))
    for blk in a:
        for m in range(mmax + 1):
            i0 = oracle.alm_index(m, m, lmax)
            ls = np.arange(m, lmax + 1)
            blk[i0:i0 + ls.size] /= (ls + 1.0) ** decay
            if m == 0:
                blk[i0:i0 + ls.size] = blk[i0:i0 + ls.size].real
            blk[i0:i0 + max(0, spin - m)] = 0
    return a


def _points(n, seed):
    rng = np.random.default_rng(seed)
    return np.arccos(rng.uniform(-0.98, 0.98, n)), rng.uniform(0, 2 * np.pi, n)


def test_deflected_point_geometry():
    th, ph = _points(500, 1)
    rng = np.random.default_rng(2)
    alpha = rng.normal(0, 0.05, (2, 500))
    th2, ph2, _ = ol.deflect(th, ph, alpha)
    n, et, ep = ol.basis(th, ph)
    n2, _, _ = ol.basis(th2, ph2)
    a = np.hypot(alpha[0], alpha[1])
    # distance along the sphere
    assert np.max(np.abs(np.arccos(np.clip(np.sum(n * n2, axis=0), -1, 1)) - a)) < 1e-7
    assert np.max(np.abs(np.arctan2(np.linalg.norm(np.cross(n.T, n2.T), axis=1),
                                    np.sum(n * n2, axis=0)) - a)) < 1e-14
    # direction: n' - cos(a) n is sin(a) times the unit deflection direction
    d = (alpha[0] * et + alpha[1] * ep) / a
    assert np.max(np.abs(n2 - np.cos(a) * n - np.sin(a) * d)) < 1e-14
    # first order: theta' - theta ~ alpha_theta, (phi' - phi) sin(theta) ~ alpha_phi
    small = 1e-6 * alpha
    th3, ph3, _ = ol.deflect(th, ph, small)
    dphi = np.angle(np.exp(1j * (ph3 - ph)))
    assert np.max(np.abs(th3 - th - small[0])) < 1e-10
    assert np.max(np.abs(dphi * np.sin(th) - small[1])) < 1e-10


def test_deflection_is_gradient_of_potential():
    lmax = mmax = 40
    plm = _alm(0, lmax, mmax, 3)[0]
    th, ph = _points(300, 4)
    alpha = ol.deflection_field(plm, lmax, mmax, th, ph)
    dth, dph = oracle.synth_deriv(plm[None, :], lmax, mmax, 0, th, ph)
    s = np.max(np.abs(alpha))
    assert np.max(np.abs(alpha[0] - dth[0])) < 1e-12 * s
    assert np.max(np.abs(alpha[1] - dph[0] / np.sin(th))) < 1e-12 * s


def test_chi_against_brute_force_transport():
    th, ph = _points(200, 5)
    th[:4] = [0.05, 0.2, np.pi - 0.1, np.pi - 0.02]   # near the poles chi is large
    rng = np.random.default_rng(6)
    alpha = rng.normal(0, 0.03, (2, 200))
    th2, ph2, chi = ol.deflect(th, ph, alpha)
    n, et, ep = ol.basis(th, ph)
    a = np.hypot(alpha[0], alpha[1])
    ahat = (alpha[0] * et + alpha[1] * ep) / a
    E1 = ol.transport(et, n, ahat, a)
    _, et2, ep2 = ol.basis(th2, ph2)
    chi_bf = -np.arctan2(np.sum(E1 * ep2, axis=0), np.sum(E1 * et2, axis=0))
    assert np.max(np.abs(np.angle(np.exp(1j * (chi - chi_bf))))) < 1e-11
    assert np.max(np.abs(chi)) > 0.01          # the test exercises non-trivial phases


def test_spin_phase_moves_vectors_by_parallel_transport():
    """Spin 1: the gradient of a scalar field, evaluated at n' and carried back to n
    along the great circle, is e^{i chi} times its spin-1 value at n'."""
    lmax = mmax = 24
    tlm = _alm(0, lmax, mmax, 7)
    th, ph = _points(120, 8)
    th[:2] = [0.1, np.pi - 0.15]
    rng = np.random.default_rng(9)
    alpha = rng.normal(0, 0.04, (2, 120))
    th2, ph2, chi = ol.deflect(th, ph, alpha)
    dth, dph = oracle.synth_deriv(tlm, lmax, mmax, 0, th2, ph2)
    f1 = dth[0] + 1j * dph[0] / np.sin(th2)                 # spin-1 value at n'
    n2, et2, ep2 = ol.basis(th2, ph2)
    v = dth[0] * et2 + dph[0] / np.sin(th2) * ep2            # the gradient as a 3-vector
    # great circle from n' back to n: direction minus the arrival tangent
    n, et, ep = ol.basis(th, ph)
    a = np.hypot(alpha[0], alpha[1])
    ahat = (alpha[0] * et + alpha[1] * ep) / a
    back = -(-np.sin(a) * n + np.cos(a) * ahat)
    vb = ol.transport(v, n2, back, a)
    c = np.sum(vb * et, axis=0) + 1j * np.sum(vb * ep, axis=0)
    assert np.max(np.abs(c - np.exp(1j * chi) * f1)) < 1e-10 * np.max(np.abs(f1))


@pytest.mark.parametrize("spin", [0, 2])
def test_lensed_pair_is_adjoint(spin):
    lmax = mmax = 30
    a = _alm(spin, lmax, mmax, 10 + spin)
    th, ph = _points(400, 11)
    rng = np.random.default_rng(12)
    alpha = rng.normal(0, 0.02, (2, 400))
    f = ol.lensed_synth(a, lmax, mmax, spin, th, ph, alpha)
    y = rng.standard_normal(f.shape)
    b = ol.lensed_adjoint(y, lmax, mmax, spin, th, ph, alpha)
    lhs = float(np.sum(y * f))
    rhs = oracle.alm_inner(a, b, lmax, mmax)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


@pytest.mark.parametrize("curl", [False, True])
def test_magnification_closed_form_vs_jacobian(curl):
    """Appendix B's |A| (from kappa, omega and the shear) equals the Jacobian
    determinant of n -> n' taken by central differences."""
    lmax = mmax = 20
    plm = _alm(0, lmax, mmax, 13, decay=2.0)[0] * 0.03
    olm = _alm(0, lmax, mmax, 14, decay=2.0)[0] * 0.01 if curl else None
    th, ph = _points(100, 15)
    det = ol.magnification(plm, lmax, mmax, th, ph, olm)
    fd = ol.magnification_fd(plm, lmax, mmax, th, ph, olm)
    assert np.max(np.abs(det - 1)) > 0.05                 # non-trivial magnification
    assert np.max(np.abs(det - fd)) < 1e-7
