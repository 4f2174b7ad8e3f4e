"""GPU lensing geometry and operator against the CPU reference ``oracle.lensing``.

* gsht_deflect: deflected positions and spin phase vs the reference (itself pinned
  against spherical geometry and brute-force parallel transport);
* gsht_deflect_vjp: exact Jacobian products vs central differences of the reference;
* the lensing operator (spin-1 deflection synthesis, deflection, synthesis at the
  deflected points, spin phase) and its adjoint vs the reference within epsilon;
* gradients with respect to the lensing potential vs central differences of the GPU
  FP64 operator, and with respect to the unlensed coefficients vs w_m times the
  adjoint.
"""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
from oracle import lensing as ol

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def G():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2304_10431_amd import gsht
    return gsht


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


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
    th = np.arccos(rng.uniform(-1, 1, n))
    ph = rng.uniform(0, 2 * np.pi, n)
    return th, ph


def _potential(lmax_p, seed, rms):
    """A potential whose deflection has roughly the given rms (radians)."""
    plm = _alm(0, lmax_p, lmax_p, seed, decay=2.5)[0]
    plm[:oracle.alm_index(0, 0, lmax_p) + 2] = 0.0       # no monopole / dipole
    th, ph = _points(2000, seed + 1)
    a = ol.deflection_field(plm, lmax_p, lmax_p, th, ph)
    return plm * (rms / math.sqrt(np.mean(a[0] ** 2 + a[1] ** 2)))


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_deflect_vs_reference(G, prec):
    say("deflect", prec)
    th, ph = _points(20000, 1)
    th[:3] = [1e-3, math.pi - 1e-3, math.pi / 2]
    rng = np.random.default_rng(2)
    alpha = rng.normal(0, 0.01, (2, th.size))
    alpha[:, 3] = 0.0                                       # no deflection
    alpha[:, 4] = [1e-9, -2e-9]                            # series branch
    rdt = torch.float64 if prec == "f64" else torch.float32
    al_d = dev(alpha).to(rdt)
    al = al_d.double().cpu().numpy()                       # the values the GPU sees
    t2, p2, chi = G.deflect(dev(th), dev(ph), al_d)
    rt, rp, rc = ol.deflect(th, ph, al)
    t2, p2, chi = t2.cpu().numpy(), p2.cpu().numpy(), chi.cpu().numpy()
    assert np.max(np.abs(t2 - rt)) < 2e-14
    dphi = np.angle(np.exp(1j * (p2 - rp)))
    assert np.max(np.abs(dphi * np.sin(rt))) < 2e-14
    assert np.all((p2 >= 0) & (p2 < 2 * math.pi))
    away = (np.sin(rt) > 1e-2) & (np.sin(th) > 1e-2)
    assert np.max(np.abs(np.angle(np.exp(1j * (chi - rc))))[away]) < 1e-11
    assert chi[3] == 0.0 and t2[3] == th[3]


def test_deflect_vjp_vs_central_differences(G):
    say("deflect vjp")
    th, ph = _points(3000, 3)
    th = np.clip(th, 0.05, math.pi - 0.05)
    rng = np.random.default_rng(4)
    alpha = rng.normal(0, 0.01, (2, th.size))
    alpha[:, 0] = 0.0
    gt, gp, gc = rng.standard_normal((3, th.size))
    ga = G.deflect_vjp(dev(th), dev(alpha), dev(gt), dev(gp), dev(gc)).cpu().numpy()
    h = 1e-7
    ref = np.zeros_like(alpha)
    for c in range(2):
        e = np.zeros_like(alpha)
        e[c] = h
        a1 = ol.deflect(th, ph, alpha + e)
        a0 = ol.deflect(th, ph, alpha - e)
        dt = (a1[0] - a0[0]) / (2 * h)
        dp = np.angle(np.exp(1j * (a1[1] - a0[1]))) / (2 * h)
        dc = np.angle(np.exp(1j * (a1[2] - a0[2]))) / (2 * h)
        ref[c] = gt * dt + gp * dp + gc * dc
    assert np.max(np.abs(ga - ref)) < 1e-6 * np.max(np.abs(ref))


@pytest.mark.parametrize("prec,eps", [("f64", 1e-10), ("f32", 1e-5)])
@pytest.mark.parametrize("spin", [0, 2])
def test_lensing_operator_vs_reference(G, prec, eps, spin):
    from paper_2304_10431_amd.lensing import Lensing
    say("lensing operator", prec, eps, spin)
    lmax = mmax = 96
    lmax_p = 64
    th, ph = _points(20000, 10 + spin)
    plm = _potential(lmax_p, 20, 3e-3)
    a = _alm(spin, lmax, mmax, 30 + spin)
    cdt = torch.complex128 if prec == "f64" else torch.complex64
    rdt = torch.float64 if prec == "f64" else torch.float32
    L = Lensing(dev(th), dev(ph), dev(plm), lmax, mmax, spin, eps, prec, lmax_p=lmax_p)
    m = L.forward(dev(a).to(cdt)).double().cpu().numpy()
    alpha = ol.deflection_field(plm, lmax_p, lmax_p, th, ph)
    ref = ol.lensed_synth(a, lmax, mmax, spin, th, ph, alpha)
    e_f = oracle.eps_eff(m, ref)
    y = np.random.default_rng(40).standard_normal(ref.shape)
    b = L.adjoint(dev(y).to(rdt)).to(torch.complex128).cpu().numpy()
    rb = ol.lensed_adjoint(y, lmax, mmax, spin, th, ph, alpha)
    w = np.sqrt(oracle.alm_weights(lmax, mmax))[None, :]
    e_a = oracle.eps_eff(w * b, w * rb)
    L.close()
    say("  forward %.3e adjoint %.3e" % (e_f, e_a))
    assert e_f <= eps
    assert e_a <= eps


@pytest.mark.parametrize("spin", [0, 2])
def test_lensing_gradients(G, spin):
    from paper_2304_10431_amd.lensing import Lensing
    say("lensing gradients", spin)
    lmax = mmax = 64
    lmax_p = 32
    th, ph = _points(4000, 50 + spin)
    plm = _potential(lmax_p, 60, 5e-3)
    a = _alm(spin, lmax, mmax, 70 + spin)
    g = np.random.default_rng(80).standard_normal((oracle.ncomp(spin), th.size))
    tht, pht, ad, gd = dev(th), dev(ph), dev(a), dev(g)

    def loss(p):
        L = Lensing(tht, pht, dev(p), lmax, mmax, spin, 1e-10, "f64", lmax_p=lmax_p)
        v = float(torch.sum(L.forward(ad) * gd))
        L.close()
        return v

    L = Lensing(tht, pht, dev(plm), lmax, mmax, spin, 1e-10, "f64", lmax_p=lmax_p)
    galm, gp, go = L.vjp(ad, gd)
    b = L.adjoint(gd)
    L.close()
    w = torch.from_numpy(oracle.alm_weights(lmax, mmax)).cuda()
    bw = b * w[None, :]
    assert float(torch.max(torch.abs(galm - bw))) <= 1e-13 * float(torch.max(torch.abs(bw)))
    gp = gp.cpu().numpy()
    rng = np.random.default_rng(90)
    idx = rng.choice(np.arange(oracle.alm_index(2, 0, lmax_p), plm.size), 6, replace=False)
    scale = np.max(np.abs(gp))
    worst = 0.0
    for i in idx:
        for part in (1.0, 1j):
            m_of_i = next(m for m in range(lmax_p + 1) if oracle.alm_index(m, m, lmax_p) <= i <
                          oracle.alm_index(m, m, lmax_p) + lmax_p + 1 - m)
            if m_of_i == 0 and part == 1j:
                continue                                     # Im of m = 0 is ignored
            h = 1e-6 * np.max(np.abs(plm))
            e = np.zeros_like(plm)
            e[i] = h * part
            fd = (loss(plm + e) - loss(plm - e)) / (2 * h)
            got = gp[i].real if part == 1.0 else gp[i].imag
            worst = max(worst, abs(fd - got) / scale)
    say("  worst |fd - grad| / max|grad| = %.3e" % worst)
    assert worst <= 1e-5


def _gl_grid(nring, nphi):
    x, wq = np.polynomial.legendre.leggauss(nring)
    th = np.repeat(np.arccos(x), nphi)
    ph = np.tile(2 * np.pi * np.arange(nphi) / nphi, nring)
    return th, ph, np.repeat(wq, nphi) * 2 * np.pi / nphi


@pytest.mark.parametrize("spin", [0, 2])
def test_lensed_alm_pipeline(G, spin):
    """Undeflected: the Gauss-Legendre analysis returns the input (exact quadrature).
    Deflected: against the CPU chain (reference lensed map, weights, direct adjoint),
    and the FP64 pipeline and its adjoint are adjoint to 1e-12."""
    from paper_2304_10431_amd.lensing import LensedAlm
    say("lensed alm", spin)
    lmax = mmax = 40
    lmax_len = mmax_len = 32
    lmax_p = 24
    th, ph, w = _gl_grid(lmax + 1, 2 * mmax + 2)
    a = _alm(spin, lmax, mmax, 100 + spin)
    zero = np.zeros(oracle.nalm(lmax_p, lmax_p), complex)
    P = LensedAlm(dev(th), dev(ph), dev(w), dev(zero), lmax, mmax, lmax, mmax, spin, 1e-10, "f64",
                  lmax_p=lmax_p)
    back = P.forward(dev(a)).cpu().numpy()
    P.close()
    wm = np.sqrt(oracle.alm_weights(lmax, mmax))[None, :]
    e0 = oracle.eps_eff(wm * back, wm * a)
    plm = _potential(lmax_p, 110, 4e-3)
    P = LensedAlm(dev(th), dev(ph), dev(w), dev(plm), lmax, mmax, lmax_len, mmax_len, spin, 1e-10,
                  "f64", lmax_p=lmax_p)
    got = P.forward(dev(a)).cpu().numpy()
    alpha = ol.deflection_field(plm, lmax_p, lmax_p, th, ph)
    ref = oracle.adjoint(w[None, :] * ol.lensed_synth(a, lmax, mmax, spin, th, ph, alpha),
                         lmax_len, mmax_len, spin, th, ph)
    wl = np.sqrt(oracle.alm_weights(lmax_len, mmax_len))[None, :]
    e1 = oracle.eps_eff(wl * got, wl * ref)
    b = _alm(spin, lmax_len, mmax_len, 120 + spin)
    fb = P.adjoint(dev(b)).cpu().numpy()
    P.close()
    lhs = oracle.alm_inner(b, got, lmax_len, mmax_len)
    rhs = oracle.alm_inner(fb, a, lmax, mmax)
    say("  undeflected %.3e  deflected %.3e  adjointness %.3e" % (e0, e1, abs(lhs - rhs) / abs(lhs)))
    assert e0 <= 1e-10
    assert e1 <= 1e-10
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


@pytest.mark.parametrize("prec,tol", [("f64", 1e-9), ("f32", 2e-5)])
@pytest.mark.parametrize("curl", [False, True])
def test_magnification_vs_reference(G, prec, tol, curl):
    from paper_2304_10431_amd.lensing import Lensing
    say("magnification", prec, curl)
    lmax_p = 48
    th, ph = _points(5000, 130)
    plm = _potential(lmax_p, 131, 2e-2)
    olm = _potential(lmax_p, 132, 5e-3) if curl else None
    eps = 1e-10 if prec == "f64" else 1e-5
    L = Lensing(dev(th), dev(ph), dev(plm), 16, 16, 0, eps, prec,
                olm=None if olm is None else dev(olm), lmax_p=lmax_p)
    det = L.magnification().cpu().numpy()
    L.close()
    ref = ol.magnification(plm, lmax_p, lmax_p, th, ph, olm)
    say("  max |A - 1| %.3e, max diff %.3e" % (np.max(np.abs(ref - 1)), np.max(np.abs(det - ref))))
    assert np.max(np.abs(ref - 1)) > 1e-2
    assert np.max(np.abs(det - ref)) <= tol


def test_inverse_lensing(G):
    """Appendix B: the adjoint applied to the lensed map times quadrature weights and
    |A| recovers the unlensed coefficients (approximately: the lensed map is not band
    limited); the GPU result equals the CPU chain (reference |A|, weights, direct
    adjoint) within epsilon."""
    from paper_2304_10431_amd.lensing import Lensing
    say("inverse lensing")
    lmax = mmax = 24
    lmax_p = 16
    th, ph, w = _gl_grid(3 * lmax, 6 * lmax)
    a = _alm(0, lmax, mmax, 140, decay=1.5)
    plm = _potential(lmax_p, 141, 1e-2)
    L = Lensing(dev(th), dev(ph), dev(plm), lmax, mmax, 0, 1e-10, "f64", lmax_p=lmax_p)
    t_len = L.forward(dev(a))
    back = L.inverse(t_len, dev(w)).cpu().numpy()
    L.close()
    alpha = ol.deflection_field(plm, lmax_p, lmax_p, th, ph)
    det = ol.magnification(plm, lmax_p, lmax_p, th, ph)
    ref = ol.lensed_adjoint((w * det)[None, :] * t_len.cpu().numpy(), lmax, mmax, 0, th, ph, alpha)
    wm = np.sqrt(oracle.alm_weights(lmax, mmax))[None, :]
    e_ref = oracle.eps_eff(wm * back, wm * ref)
    e_unl = oracle.eps_eff(wm * back, wm * a)
    say("  vs CPU chain %.3e, vs unlensed %.3e" % (e_ref, e_unl))
    assert e_ref <= 1e-9
    assert e_unl <= 1e-3
