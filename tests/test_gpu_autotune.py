"""Launch-shape autotuning: the chosen shapes are supported ones and the plan's
results after tuning equal those before it up to rounding."""
import sys

import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("spin,lmax,prec", [(2, 700, "f64"), (0, 900, "f32")])
def test_autotune_keeps_results(spin, lmax, prec):
    from paper_2304_10431_amd import gsht
    say("autotune", spin, lmax, prec)
    rng = np.random.default_rng(lmax)
    npts = 50000
    th = torch.from_numpy(np.arccos(rng.uniform(-1, 1, npts))).cuda()
    ph = torch.from_numpy(rng.uniform(0, 2 * np.pi, npts)).cuda()
    nc = oracle.ncomp(spin)
    a = rng.standard_normal((nc, oracle.nalm(lmax, lmax))) + 1j * rng.standard_normal((nc, oracle.nalm(lmax, lmax)))
    for m in range(lmax + 1):
        i0 = oracle.alm_index(m, m, lmax)
        if m == 0:
            a[:, i0:i0 + lmax + 1] = a[:, i0:i0 + lmax + 1].real
        a[:, i0:i0 + max(0, spin - m)] = 0
    cdt = torch.complex128 if prec == "f64" else torch.complex64
    rdt = torch.float64 if prec == "f64" else torch.float32
    eps = 1e-10 if prec == "f64" else 1e-5
    plan = gsht.Plan(th, ph, lmax, lmax, spin, eps, prec)
    ad = torch.from_numpy(a).cuda().to(cdt)
    y = torch.from_numpy(rng.standard_normal((nc, npts))).cuda().to(rdt)
    m0, b0 = plan.synth(ad), plan.adjoint(y)
    shape = plan.autotune()
    m1, b1 = plan.synth(ad), plan.adjoint(y)
    plan.close()
    say("  chosen", shape)
    assert shape[0] in (1, 2, 4)
    assert (shape[1], shape[2]) in ((1, 8), (2, 8), (2, 4), (4, 4), (3, 8), (3, 4), (4, 8))
    tol = 1e-13 if prec == "f64" else 1e-6
    assert oracle.eps_eff(m1.double().cpu().numpy(), m0.double().cpu().numpy()) <= tol
    w = np.sqrt(oracle.alm_weights(lmax, lmax))[None, :]
    assert oracle.eps_eff(w * b1.to(torch.complex128).cpu().numpy(),
                          w * b0.to(torch.complex128).cpu().numpy()) <= tol
