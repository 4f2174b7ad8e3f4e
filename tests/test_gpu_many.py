"""Several maps on one plan (gsht_plan_synth_many): the group Legendre kernel shares
the recurrence between up to four maps; every map must equal its own single-map
synthesis up to rounding, for group sizes 4, 2 and 1 and both synthesis launch
shapes that have a group kernel (and the fallback for the other), and stay within
epsilon of the oracle."""
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


def _alms(nmaps, spin, lmax, mmax, seed):
    rng = np.random.default_rng(seed)
    nc = oracle.ncomp(spin)
    a = (rng.standard_normal((nmaps, nc, oracle.nalm(lmax, mmax)))
         + 1j * rng.standard_normal((nmaps, nc, oracle.nalm(lmax, mmax)))) / math.sqrt(2)
    for m in range(mmax + 1):
        i0 = oracle.alm_index(m, m, lmax)
        if m == 0:
            a[..., i0:i0 + lmax + 1] = a[..., i0:i0 + lmax + 1].real
        a[..., i0:i0 + max(0, spin - m)] = 0
    return a


@pytest.mark.parametrize("syn_r", [1, 2, 4])
@pytest.mark.parametrize("prec,eps,tol", [("f64", 1e-10, 1e-13), ("f32", 1e-5, 1e-6)])
@pytest.mark.parametrize("spin,lmax,mmax,npts", [(2, 260, 200, 20000), (0, 300, 300, 20000)])
def test_many_equals_single(G, monkeypatch, syn_r, prec, eps, tol, spin, lmax, mmax, npts):
    say("synth_many", syn_r, prec, spin, lmax, mmax)
    monkeypatch.setenv("GSHT_SYN_R", str(syn_r))
    rng = np.random.default_rng(lmax + spin)
    th = np.arccos(rng.uniform(-1, 1, npts))
    ph = rng.uniform(0, 2 * np.pi, npts)
    th[:2] = [0.0, np.pi]
    nmaps = 7                                   # groups of 4, 2 and 1
    a = _alms(nmaps, spin, lmax, mmax, 77)
    cdt = torch.complex128 if prec == "f64" else torch.complex64
    plan = G.Plan(torch.from_numpy(th).cuda(), torch.from_numpy(ph).cuda(), lmax, mmax, spin, eps,
                  prec)
    ad = torch.from_numpy(a).cuda().to(cdt)
    many = plan.synth_many(ad).double().cpu().numpy()
    worst = 0.0
    for k in range(nmaps):
        one = plan.synth(ad[k].contiguous()).double().cpu().numpy()
        worst = max(worst, oracle.eps_eff(many[k], one))
    ref = oracle.synth(a[5], lmax, mmax, spin, th, ph)
    e_o = oracle.eps_eff(many[5], ref)
    plan.close()
    say("  worst vs single %.3e, map 5 vs oracle %.3e" % (worst, e_o))
    assert worst <= tol
    assert e_o <= eps


def _spectrum_alms(nmaps, spin, lmax, mmax, seed):
    """Gaussian a_lm with C_l = 1 / (l + 1)^2 (large dynamic range over l), map
    amplitudes spread over eight decades, and one all-zero map."""
    a = _alms(nmaps, spin, lmax, mmax, seed)
    for m in range(mmax + 1):
        i0 = oracle.alm_index(m, m, lmax)
        a[..., i0:i0 + lmax + 1 - m] /= np.arange(m, lmax + 1) + 1.0
    a *= np.logspace(-4, 4, nmaps)[:, None, None]
    a[3] = 0
    return a


@pytest.mark.parametrize("spin,lmax,mmax,npts,nmaps", [(2, 260, 200, 20000, 16),
                                                       (0, 300, 300, 20000, 16),
                                                       (1, 131, 131, 8000, 8),
                                                       (3, 77, 50, 6000, 21),
                                                       (2, 40, 40, 3000, 11)])
def test_many_mfma(G, monkeypatch, spin, lmax, mmax, npts, nmaps):
    """FP32 plans run groups of 8 to 16 maps through the matrix-core Legendre step
    (FP16 hi/lo products, FP32 accumulation); every map must stay within a few
    1e-7 of its own single-map synthesis (FP64 Legendre step) and within epsilon of
    the oracle, whatever its amplitude; GSHT_MANY_MFMA=0 falls back to the FP64
    group kernel."""
    say("synth_many mfma", spin, lmax, mmax, npts, nmaps)
    rng = np.random.default_rng(lmax + 10 * spin)
    th = np.arccos(rng.uniform(-1, 1, npts))
    ph = rng.uniform(0, 2 * np.pi, npts)
    th[:2] = [0.0, np.pi]
    a = _spectrum_alms(nmaps, spin, lmax, mmax, 91)
    plan = G.Plan(torch.from_numpy(th).cuda(), torch.from_numpy(ph).cuda(), lmax, mmax, spin, 1e-5,
                  "f32")
    ad = torch.from_numpy(a).cuda().to(torch.complex64)
    many = plan.synth_many(ad).double().cpu().numpy()
    monkeypatch.setenv("GSHT_MANY_MFMA", "0")
    valu = plan.synth_many(ad).double().cpu().numpy()
    worst = worst_valu = 0.0
    for k in range(nmaps):
        one = plan.synth(ad[k].contiguous()).double().cpu().numpy()
        if k == 3:
            assert np.all(many[k] == 0) and np.all(one == 0)
            continue
        worst = max(worst, oracle.eps_eff(many[k], one))
        worst_valu = max(worst_valu, oracle.eps_eff(valu[k], one))
    plan.close()
    e_o = [oracle.eps_eff(many[k], oracle.synth(a[k], lmax, mmax, spin, th, ph)) for k in (0, nmaps - 1)]
    say("  worst vs single: mfma %.3e, fp64 group %.3e; vs oracle %.3e %.3e"
        % (worst, worst_valu, e_o[0], e_o[1]))
    assert worst <= 1e-6
    assert worst_valu <= 1e-6
    assert max(e_o) <= 1e-5


@pytest.mark.parametrize("spin,lmax,mmax,npts,nmaps", [(2, 260, 200, 20000, 16),
                                                       (0, 300, 300, 20000, 16),
                                                       (1, 131, 131, 8000, 8),
                                                       (3, 77, 50, 6000, 21),
                                                       (2, 40, 40, 3000, 11)])
def test_adjoint_many_mfma(G, monkeypatch, spin, lmax, mmax, npts, nmaps):
    """FP32 plans run the adjoint of 8 to 16 maps through the matrix-core Legendre
    step; every map's coefficients must stay within about 1e-6 of its own adjoint
    (FP64 Legendre step) and within epsilon of the oracle, whatever the map's
    amplitude; GSHT_MANY_MFMA=0 gives the single-map results."""
    say("adjoint_many mfma", spin, lmax, mmax, npts, nmaps)
    rng = np.random.default_rng(lmax + 20 * spin)
    th = np.arccos(rng.uniform(-1, 1, npts))
    ph = rng.uniform(0, 2 * np.pi, npts)
    th[:2] = [0.0, np.pi]
    nc = oracle.ncomp(spin)
    y = rng.standard_normal((nmaps, nc, npts)) * np.logspace(-4, 4, nmaps)[:, None, None]
    y[3] = 0
    plan = G.Plan(torch.from_numpy(th).cuda(), torch.from_numpy(ph).cuda(), lmax, mmax, spin, 1e-5,
                  "f32")
    yd = torch.from_numpy(y).cuda().float()
    many = plan.adjoint_many(yd).to(torch.complex128).cpu().numpy()
    monkeypatch.setenv("GSHT_MANY_MFMA", "0")
    plain = plan.adjoint_many(yd).to(torch.complex128).cpu().numpy()
    w = np.sqrt(oracle.alm_weights(lmax, mmax))[None, :]
    worst = worst_plain = 0.0
    for k in range(nmaps):
        one = plan.adjoint(yd[k].contiguous()).to(torch.complex128).cpu().numpy()
        if k == 3:
            assert np.all(many[k] == 0) and np.all(one == 0)
            continue
        worst = max(worst, oracle.eps_eff(w * many[k], w * one))
        worst_plain = max(worst_plain, oracle.eps_eff(w * plain[k], w * one))
    plan.close()
    e_o = [oracle.eps_eff(w * many[k], w * oracle.adjoint(y[k], lmax, mmax, spin, th, ph))
           for k in (0, nmaps - 1)]
    say("  worst vs single: mfma %.3e, plain %.3e; vs oracle %.3e %.3e"
        % (worst, worst_plain, e_o[0], e_o[1]))
    assert worst <= 2e-6
    assert worst_plain <= 1e-12
    assert max(e_o) <= 1e-5
    # m = 0 imaginary parts and l < spin entries stay exactly zero
    for m in range(min(spin, mmax + 1)):
        i0 = oracle.alm_index(m, m, lmax)
        assert np.all(many[:, :, i0:i0 + spin - m] == 0)
    assert np.all(many[:, :, :lmax + 1].imag == 0)


@pytest.mark.parametrize("spin,lmax,mmax,npts", [(2, 2, 2, 500), (0, 5, 0, 700), (3, 3, 1, 400),
                                                 (1, 17, 17, 1)])
def test_many_edge_cases(G, spin, lmax, mmax, npts):
    """Degenerate several-map cases on the matrix-core paths: lmax = spin (one degree
    per m, most m empty), mmax = 0, a single point, and zero maps (a no-op)."""
    say("many edge", spin, lmax, mmax, npts)
    rng = np.random.default_rng(5 + lmax)
    th = np.arccos(rng.uniform(-1, 1, npts))
    ph = rng.uniform(0, 2 * np.pi, npts)
    nm = 9
    a = _spectrum_alms(nm, spin, lmax, mmax, 3)
    plan = G.Plan(torch.from_numpy(th).cuda(), torch.from_numpy(ph).cuda(), lmax, mmax, spin, 1e-5,
                  "f32")
    ad = torch.from_numpy(a).cuda().to(torch.complex64)
    many = plan.synth_many(ad)
    y = torch.from_numpy(rng.standard_normal((nm, oracle.ncomp(spin), npts))).cuda().float()
    back = plan.adjoint_many(y)
    w = np.sqrt(oracle.alm_weights(lmax, mmax))[None, :]
    for k in (0, 4, 8):
        one = plan.synth(ad[k].contiguous()).double().cpu().numpy()
        assert oracle.eps_eff(many[k].double().cpu().numpy(), one) <= 1e-6
        ref = oracle.adjoint(y[k].double().cpu().numpy(), lmax, mmax, spin, th, ph)
        assert oracle.eps_eff(w * back[k].to(torch.complex128).cpu().numpy(), w * ref) <= 1e-5
    empty_a = torch.zeros((0,) + tuple(ad.shape[1:]), dtype=ad.dtype, device="cuda")
    assert plan.synth_many(empty_a).shape[0] == 0
    empty_m = torch.zeros((0,) + tuple(y.shape[1:]), dtype=y.dtype, device="cuda")
    assert plan.adjoint_many(empty_m).shape[0] == 0
    plan.close()
