"""GPU derivatives: position derivatives of the synthesis, vector-Jacobian products
and the torch.autograd wrappers, through the C ABI.

References:
* the oracle's derivative synthesis (d/dphi: factor i m; d/dtheta: the spin ladder
  relation; itself pinned against finite differences and, for spin 0, against the
  spin-1 synthesis of sqrt(l (l+1)) a_lm);
* w_m times the oracle's adjoint for the coefficient gradient, and the synthesis of
  galm / w_m for the adjoint's map gradient (the inner product of O6 / Sect. 2);
* central differences of the GPU's own FP64 synthesis at 32 coordinates.

Bars: the derivative maps are interpolated from the same oversampled grid with the
kernel's derivative, which carries the kernel error amplified by the derivative
(measured with the plain CPU steps: 4.8e-6 to 6.3e-6 relative at w = 7,
6e-11 to 1.4e-10 at w = 12), so they are held to 3 epsilon relative to the
derivative field's norm.
"""
import math
import sys

import numpy as np
import pytest
import torch

import oracle

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


def _alm(spin, lmax, mmax, seed):
    rng = np.random.default_rng(5000 + seed)
    nc = oracle.ncomp(spin)
    na = oracle.nalm(lmax, mmax)
    a = (rng.standard_normal((nc, na)) + 1j * rng.standard_normal((nc, na))) / math.sqrt(2)
    for blk in a:
        for m in range(mmax + 1):
            i0 = oracle.alm_index(m, m, lmax)
            if m == 0:
                blk[i0:i0 + lmax + 1] = blk[i0:i0 + lmax + 1].real
            blk[i0:i0 + max(0, spin - m)] = 0
    return a


def _points(npts, seed):
    rng = np.random.default_rng(6000 + seed)
    th = np.arccos(rng.uniform(-1, 1, npts))
    ph = rng.uniform(0, 2 * np.pi, npts)
    th[:2] = [1e-6, np.pi - 1e-6]
    ph[2:4] = [-0.3, 7.0]
    return th, ph


CASES = [
    # spin, lmax, mmax, npts, seed
    (0, 127, 127, 4000, 1),
    (2, 200, 150, 4000, 2),
    (1, 64, 64, 2000, 3),
]
FORMS = [("f64", 1e-10), ("f32", 1e-5)]
CDT = {"f64": torch.complex128, "f32": torch.complex64}
RDT = {"f64": torch.float64, "f32": torch.float32}


@pytest.mark.parametrize("prec,eps", FORMS)
@pytest.mark.parametrize("spin,lmax,mmax,npts,seed", CASES)
def test_synth_deriv_vs_oracle(G, prec, eps, spin, lmax, mmax, npts, seed):
    say("synth_deriv", prec, eps, spin, lmax, mmax, npts)
    th, ph = _points(npts, seed)
    a = _alm(spin, lmax, mmax, seed)
    plan = G.Plan(dev(th), dev(ph), lmax, mmax, spin, eps, prec)
    ad = dev(a).to(CDT[prec])
    m, dth, dph = plan.synth_deriv(ad)
    m0 = plan.synth(ad)
    plan.close()
    rt, rp = oracle.synth_deriv(a, lmax, mmax, spin, th, ph)
    e_t = oracle.eps_eff(dth.double().cpu().numpy(), rt)
    e_p = oracle.eps_eff(dph.double().cpu().numpy(), rp)
    e_m = oracle.eps_eff(m.double().cpu().numpy(), m0.double().cpu().numpy())
    say("  dtheta %.3e  dphi %.3e  map vs synth %.3e" % (e_t, e_p, e_m))
    assert e_t <= 3 * eps
    assert e_p <= 3 * eps
    # same grid and taps as the plain synthesis; only the kernel's exp may differ
    assert e_m <= (1e-13 if prec == "f64" else 1e-6)


@pytest.mark.parametrize("prec,eps", FORMS)
@pytest.mark.parametrize("spin,lmax,mmax,npts,seed", CASES)
def test_synth_vjp_vs_oracle(G, prec, eps, spin, lmax, mmax, npts, seed):
    say("synth_vjp", prec, eps, spin, lmax, mmax, npts)
    th, ph = _points(npts, seed)
    a = _alm(spin, lmax, mmax, seed)
    nc = oracle.ncomp(spin)
    gm = np.random.default_rng(7100 + seed).standard_normal((nc, npts))
    plan = G.Plan(dev(th), dev(ph), lmax, mmax, spin, eps, prec)
    ad = dev(a).to(CDT[prec])
    gd = dev(gm).to(RDT[prec])
    galm, gth, gph = plan.synth_vjp(ad, gd)
    b = plan.adjoint(gd)
    only_t = plan.synth_vjp(ad, gd, want_alm=False, want_theta=True, want_phi=False)
    plan.close()
    w = torch.from_numpy(oracle.alm_weights(lmax, mmax)).cuda()
    # the coefficient gradient is the adjoint scaled by exactly w_m (a power of two)
    assert torch.equal(galm, b * w.to(RDT[prec])[None, :])
    wm = oracle.alm_weights(lmax, mmax)[None, :]
    ref_adj = oracle.adjoint(gm, lmax, mmax, spin, th, ph)
    # galm / w_m is the adjoint; its accuracy is measured as for the adjoint itself
    e_a = oracle.eps_eff(np.sqrt(wm) * galm.to(torch.complex128).cpu().numpy() / wm,
                         np.sqrt(wm) * ref_adj)
    rt, rp = oracle.synth_deriv(a, lmax, mmax, spin, th, ph)
    e_t = oracle.eps_eff(gth.cpu().numpy(), np.sum(gm * rt, axis=0))
    e_p = oracle.eps_eff(gph.cpu().numpy(), np.sum(gm * rp, axis=0))
    say("  galm %.3e  gtheta %.3e  gphi %.3e" % (e_a, e_t, e_p))
    assert e_a <= eps
    assert e_t <= 3 * eps
    assert e_p <= 3 * eps
    assert only_t[0] is None and only_t[2] is None
    assert torch.equal(only_t[1], gth)


@pytest.mark.parametrize("spin,lmax,mmax", [(0, 96, 96), (2, 80, 64)])
def test_position_gradient_vs_central_differences(G, spin, lmax, mmax):
    """d L / d theta_k and d L / d phi_k for L = sum g * map at 32 coordinates, against
    central differences (step 1e-6) of the FP64 synthesis at the displaced point."""
    say("position gradient FD", spin, lmax, mmax)
    npts = 500
    th, ph = _points(npts, 10 + spin)
    th[:2] = [0.4, 2.1]
    a = _alm(spin, lmax, mmax, 10 + spin)
    nc = oracle.ncomp(spin)
    gm = np.random.default_rng(7200 + spin).standard_normal((nc, npts))
    plan = G.Plan(dev(th), dev(ph), lmax, mmax, spin, 1e-10, "f64")
    ad = dev(a)
    _, gth, gph = plan.synth_vjp(ad, dev(gm), want_alm=False)
    plan.close()
    gth, gph = gth.cpu().numpy(), gph.cpu().numpy()
    h = 1e-6
    ks = np.random.default_rng(7300 + spin).choice(npts, 16, replace=False)
    scale = max(np.max(np.abs(gth)), np.max(np.abs(gph)))
    worst = 0.0
    for k in ks:
        for which, ref in (("theta", gth[k]), ("phi", gph[k])):
            dt, dp = (h, 0.0) if which == "theta" else (0.0, h)
            pt = np.array([th[k] + dt, th[k] - dt])
            pp = np.array([ph[k] + dp, ph[k] - dp])
            p2 = G.Plan(dev(pt), dev(pp), lmax, mmax, spin, 1e-10, "f64")
            f = p2.synth(ad).cpu().numpy()
            p2.close()
            fd = float(np.sum(gm[:, k] * (f[:, 0] - f[:, 1]))) / (2 * h)
            worst = max(worst, abs(fd - ref) / scale)
    say("  worst |fd - grad| / max|grad| = %.3e" % worst)
    assert worst <= 1e-6


@pytest.mark.parametrize("prec,eps", FORMS)
def test_autograd_synth_and_adjoint(G, prec, eps):
    from paper_2304_10431_amd import autograd as ag
    spin, lmax, mmax, npts = 2, 100, 100, 3000
    say("autograd", prec, eps)
    th, ph = _points(npts, 20)
    a = _alm(spin, lmax, mmax, 20)
    plan = G.Plan(dev(th), dev(ph), lmax, mmax, spin, eps, prec)
    W = np.random.default_rng(7400).standard_normal((2, npts))
    at = dev(a).to(CDT[prec]).requires_grad_(True)
    tt = dev(th).requires_grad_(True)
    pt = dev(ph).requires_grad_(True)
    loss = (ag.synth(plan, at, tt, pt) * dev(W).to(RDT[prec])).sum()
    loss.backward()
    wm = oracle.alm_weights(lmax, mmax)[None, :]
    ref_adj = oracle.adjoint(W, lmax, mmax, spin, th, ph)
    e_a = oracle.eps_eff(np.sqrt(wm) * at.grad.to(torch.complex128).cpu().numpy() / wm,
                         np.sqrt(wm) * ref_adj)
    rt, rp = oracle.synth_deriv(a, lmax, mmax, spin, th, ph)
    e_t = oracle.eps_eff(tt.grad.cpu().numpy(), np.sum(W * rt, axis=0))
    e_p = oracle.eps_eff(pt.grad.cpu().numpy(), np.sum(W * rp, axis=0))
    # adjoint: L = sum Re(conj(Z) b), dL/dmap = synthesis of Z / w_m
    Z = _alm(spin, lmax, mmax, 21)
    mt = dev(W).to(RDT[prec]).requires_grad_(True)
    b = ag.adjoint(plan, mt)
    (torch.real(torch.conj(dev(Z).to(CDT[prec])) * b)).sum().backward()
    ref_m = oracle.synth(Z / wm, lmax, mmax, spin, th, ph)
    e_m = oracle.eps_eff(mt.grad.double().cpu().numpy(), ref_m)
    plan.close()
    say("  alm %.3e theta %.3e phi %.3e map %.3e" % (e_a, e_t, e_p, e_m))
    assert e_a <= eps and e_m <= eps
    assert e_t <= 3 * eps and e_p <= 3 * eps
