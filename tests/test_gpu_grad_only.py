"""Gradient-only spin-s transforms (C = 0 on input, G only on output).

The gradient-only kernels share the products of G with both spin channels, so
their arithmetic differs from the general path's; the results must agree with it
(C set to zero, or the G block of the general adjoint) to rounding, and with the
oracle within epsilon, for every Legendre launch shape.
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


def _glm(spin, lmax, mmax, seed):
    rng = np.random.default_rng(seed)
    a = (rng.standard_normal(oracle.nalm(lmax, mmax)) + 1j * rng.standard_normal(oracle.nalm(lmax, mmax))) / math.sqrt(2)
    for m in range(mmax + 1):
        i0 = oracle.alm_index(m, m, lmax)
        if m == 0:
            a[i0:i0 + lmax + 1] = a[i0:i0 + lmax + 1].real
        a[i0:i0 + max(0, spin - m)] = 0
    return a


SHAPES = [(1, 1, 8), (2, 3, 8), (4, 2, 4), (2, 4, 4), (2, 3, 4)]


@pytest.mark.parametrize("syn_r,adj_r,adj_b", SHAPES)
@pytest.mark.parametrize("prec,eps", [("f64", 1e-10), ("f32", 1e-5)])
@pytest.mark.parametrize("spin,lmax,mmax,npts", [(2, 300, 300, 20000), (1, 200, 130, 8000),
                                                 (3, 130, 130, 5000)])
def test_gradient_only_matches_general(G, monkeypatch, syn_r, adj_r, adj_b, prec, eps, spin,
                                       lmax, mmax, npts):
    say("gradient only", syn_r, adj_r, adj_b, prec, eps, spin, lmax, mmax, npts)
    monkeypatch.setenv("GSHT_SYN_R", str(syn_r))
    monkeypatch.setenv("GSHT_ADJ_R", str(adj_r))
    monkeypatch.setenv("GSHT_ADJ_B", str(adj_b))
    rng = np.random.default_rng(lmax + spin)
    th = np.arccos(rng.uniform(-1, 1, npts))
    ph = rng.uniform(0, 2 * np.pi, npts)
    th[:2] = [0.0, np.pi]
    g = _glm(spin, lmax, mmax, 7 + spin)
    cdt = torch.complex128 if prec == "f64" else torch.complex64
    rdt = torch.float64 if prec == "f64" else torch.float32
    plan = G.Plan(dev(th), dev(ph), lmax, mmax, spin, eps, prec)
    gd = dev(g[None, :]).to(cdt)
    m_grad = plan.synth_grad(gd)
    m_full = plan.synth(torch.cat([gd, torch.zeros_like(gd)]).contiguous())
    y = dev(rng.standard_normal((2, npts))).to(rdt)
    b_grad = plan.adjoint_grad(y)
    b_full = plan.adjoint(y)
    plan.close()
    tight = 1e-13 if prec == "f64" else 2e-6
    e_m = oracle.eps_eff(m_grad.double().cpu().numpy(), m_full.double().cpu().numpy())
    wts = np.sqrt(oracle.alm_weights(lmax, mmax))[None, :]
    e_b = oracle.eps_eff(wts * b_grad.to(torch.complex128).cpu().numpy(),
                         wts * b_full[:1].to(torch.complex128).cpu().numpy())
    ref = oracle.synth(np.stack([g, np.zeros_like(g)]), lmax, mmax, spin, th, ph)
    e_o = oracle.eps_eff(m_grad.double().cpu().numpy(), ref)
    ref_b = oracle.adjoint(y.double().cpu().numpy(), lmax, mmax, spin, th, ph)[:1]
    e_ob = oracle.eps_eff(wts * b_grad.to(torch.complex128).cpu().numpy(), wts * ref_b)
    say("  vs general: synth %.2e adjoint %.2e; vs oracle: %.2e %.2e" % (e_m, e_b, e_o, e_ob))
    assert e_m <= tight and e_b <= tight
    assert e_o <= eps and e_ob <= eps
    assert float(torch.max(torch.abs(b_grad[0, :lmax + 1].imag))) == 0.0   # m = 0 real


def test_gradient_only_rejects_spin0(G):
    plan = G.Plan(dev(np.array([0.5])), dev(np.array([0.1])), 8, 8, 0, 1e-10, "f64")
    with pytest.raises(G.GshtError):
        plan.synth_grad(dev(_glm(0, 8, 8, 1)[None, :]))
    plan.close()
