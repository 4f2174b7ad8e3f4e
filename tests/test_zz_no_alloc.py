"""The allocation-free stage entry point (gsht_legendre_rings_adjoint_noalloc) against
the allocating one (gsht_legendre_rings_adjoint) through the C ABI: calls in a row on
the device's shared scratch, each later call smaller than the one before, so stale
tables or accumulators left by a larger call would show.  Both entry points run the
same kernels and sum with atomics in unspecified order, so FP64 results agree to
rounding (1e-13 relative) and FP32 results to one FP32 rounding (1e-6)."""
import sys

import numpy as np
import pytest
import torch

from paper_2304_10431_amd import workloads as wl

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def G():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2304_10431_amd import gsht
    return gsht


def rel(a, b):
    a, b = a.to(torch.complex128), b.to(torch.complex128)
    return float(torch.linalg.norm(a - b) / torch.linalg.norm(b))


@pytest.mark.parametrize("prec,tol", [("f64", 1e-13), ("f32", 1e-6)])
def test_noalloc_equals_allocating_entry(G, prec, tol):
    cdt = torch.complex128 if prec == "f64" else torch.complex64
    # (lmax, mmax, spin, ntheta): each call smaller than the previous one
    cases = [(1024, 1024, 2, 1030), (300, 250, 2, 520), (130, 130, 0, 140), (20, 5, 3, 23)]
    for k, (lmax, mmax, spin, ntheta) in enumerate(cases):
        say("noalloc", prec, lmax, mmax, spin, ntheta)
        rng = np.random.default_rng(100 + k)
        ncol = mmax + 1 if spin == 0 else 2 * mmax + 1
        F = torch.from_numpy(rng.standard_normal((ncol, 2 * ntheta - 2))
                             + 1j * rng.standard_normal((ncol, 2 * ntheta - 2))).cuda().to(cdt)
        ref = G.legendre_rings_adjoint(F, lmax, mmax, spin, ntheta, prec)
        ncomp = 1 if spin == 0 else 2
        out = torch.full((ncomp, wl.nalm(lmax, mmax)), complex(np.nan, np.nan), dtype=cdt,
                         device="cuda")
        G.legendre_rings_adjoint_noalloc(F, lmax, mmax, spin, ntheta, out, prec)
        torch.cuda.synchronize()
        e = rel(out, ref)
        say("  relative difference %.2e" % e)
        assert torch.isfinite(torch.view_as_real(out)).all()
        assert e <= tol, e
        # exact zeros where the convention puts them: Im of m = 0, and l < spin
        assert torch.all(out[:, :lmax + 1].imag == 0)
        for l in range(min(spin, lmax + 1)):
            assert torch.all(out[:, l] == 0)
