"""Minimal-ring analysis (Appendix A) on the GPU.

For a band-limited map the method is exact, so the expected result is the input:
a_lm -> map on the lmax + 2 equiangular rings (the oracle's ring synthesis and an
FFT in phi, i.e. the definition of the synthesis at those points) -> GPU analysis
-> a_lm.  Cases cover spins 0..3, mmax < lmax, the smallest allowed nphi
(2 mmax + 1, odd) and an even one, both precisions, and lmax 512.
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


def _alm(spin, lmax, mmax, seed):
    rng = np.random.default_rng(seed)
    nc = oracle.ncomp(spin)
    a = (rng.standard_normal((nc, oracle.nalm(lmax, mmax))) + 1j * rng.standard_normal((nc, oracle.nalm(lmax, mmax)))) / math.sqrt(2)
    for blk in a:
        for m in range(mmax + 1):
            i0 = oracle.alm_index(m, m, lmax)
            if m == 0:
                blk[i0:i0 + lmax + 1] = blk[i0:i0 + lmax + 1].real
            blk[i0:i0 + max(0, spin - m)] = 0
    return a


def grid_map(a, lmax, mmax, spin, nphi):
    """The synthesis on the minimal grid: F_m(theta_j) from the oracle's ring sums,
    then sum_m F_m e^{i m phi_k}."""
    ntheta = lmax + 2
    th = np.pi * np.arange(ntheta) / (ntheta - 1)
    F = oracle.ring_synth(a, lmax, mmax, spin, th)            # [2 mmax + 1][ntheta]
    spec = np.zeros((ntheta, nphi), complex)
    for m in range(-mmax, mmax + 1):
        spec[:, m % nphi] += F[m + mmax]
    P = np.fft.ifft(spec, axis=1) * nphi
    if spin == 0:
        return P.real[None]
    return np.stack([P.real, P.imag])


CASES = [
    # spin, lmax, mmax, nphi
    (0, 64, 64, 129),
    (0, 33, 20, 50),
    (1, 40, 40, 90),
    (2, 100, 80, 161),
    (3, 31, 20, 41),
]


@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", 2e-6)])
@pytest.mark.parametrize("spin,lmax,mmax,nphi", CASES)
def test_minimal_ring_analysis_round_trip(G, prec, tol, spin, lmax, mmax, nphi):
    say("analysis", prec, spin, lmax, mmax, nphi)
    a = _alm(spin, lmax, mmax, 300 + lmax + spin)
    m = grid_map(a, lmax, mmax, spin, nphi)
    rdt = torch.float64 if prec == "f64" else torch.float32
    b = G.analysis_minimal(torch.from_numpy(np.ascontiguousarray(m)).cuda().to(rdt), lmax, mmax,
                           spin).to(torch.complex128).cpu().numpy()
    w = np.sqrt(oracle.alm_weights(lmax, mmax))[None, :]
    e = oracle.eps_eff(w * b, w * a)
    say("  eps %.3e" % e)
    assert e <= tol


def test_minimal_ring_analysis_lmax512(G):
    spin, lmax, mmax = 2, 512, 512
    nphi = 2 * mmax + 2
    say("analysis lmax 512")
    a = _alm(spin, lmax, mmax, 999)
    m = grid_map(a, lmax, mmax, spin, nphi)
    b = G.analysis_minimal(torch.from_numpy(m).cuda(), lmax, mmax, spin).cpu().numpy()
    w = np.sqrt(oracle.alm_weights(lmax, mmax))[None, :]
    e = oracle.eps_eff(w * b, w * a)
    say("  eps %.3e" % e)
    assert e <= 1e-11


def test_minimal_ring_analysis_rejects_small_nphi(G):
    m = torch.zeros((1, 10, 14), dtype=torch.float64, device="cuda")
    with pytest.raises(G.GshtError):
        G.analysis_minimal(m, 8, 8, 0)          # nphi 14 < 2 mmax + 1
