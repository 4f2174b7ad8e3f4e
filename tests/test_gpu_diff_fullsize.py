"""Differentiation at the full size of the stated workload: chi^2 = |A(a, n') - y|^2
with A the spin-2 general synthesis at lmax 2048 on a 2049 x 4097 Gauss-Legendre grid
(8,394,753 points) displaced along great circles by a deflection field (the spin-1
gradient of a Gaussian potential, C_l ~ l^-4 above l = 60, scaled to 2.5 arcmin rms),
y a noisy forward run, FP64.  The backward pass is the hand-written adjoint (gradient
in a_lm) and the position-gradient kernel chained through the deflection's
vector-Jacobian product (gradient in the deflection).  Both are checked against
central differences of chi^2 (step 1e-6 for the deflection) at 32 random
coordinates (Richardson-combined for the deflection); the oracle gradient at small
lmax is in test_gpu_deriv.py."""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
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


def test_chi2_gradients_full_size(G):
    lmax, spin, eps = 2048, 2, 1e-10
    rng = np.random.default_rng(2024)
    th0n, ph0n, _ = wl.gl_grid(lmax + 1, 2 * lmax + 1)
    th0 = torch.from_numpy(th0n).cuda()
    ph0 = torch.from_numpy(ph0n).cuda()
    npts = th0.numel()
    say("chi2 full size: %d points" % npts)
    # deflection: spin-1 synthesis of sqrt(l (l + 1)) phi_lm, scaled to 2.5 arcmin rms
    lp = 2048
    ell = np.arange(lp + 1, dtype=float)
    clp = np.where(ell > 60, (np.maximum(ell, 1) / 60.0) ** -4.0, 1.0)   # C_l of the potential
    clp[0] = 0.0
    plm = wl.gaussian_alm(lp, lp, 0, rng, cl=clp)[0]
    g1 = np.zeros((2, plm.size), complex)
    g1[0] = plm
    p1 = G.Plan(th0, ph0, lp, lp, 1, eps, "f64")
    alpha = p1.synth(G.alm_lscale(torch.from_numpy(g1).cuda(), lp, lp))
    p1.close()
    alpha *= (2.5 / 60.0 * math.pi / 180.0) / float(torch.sqrt(torch.mean(alpha ** 2) * 2))
    th, ph, _ = G.deflect(th0, ph0, alpha, want_chi=False)
    # data and model
    a_true = torch.from_numpy(wl.gaussian_alm(lmax, lmax, spin, rng)).cuda()
    plan = G.Plan(th, ph, lmax, lmax, spin, eps, "f64")
    y = plan.synth(a_true)
    y += 0.1 * float(torch.sqrt(torch.mean(y ** 2))) * torch.from_numpy(
        rng.standard_normal((2, npts))).cuda()
    a = a_true + 0.05 * torch.from_numpy(wl.gaussian_alm(lmax, lmax, spin, rng)).cuda()
    r = plan.synth(a) - y
    galm, gth, gph = plan.synth_vjp(a, 2.0 * r)
    galpha = G.deflect_vjp(th0, alpha, g_theta=gth, g_phi=gph)
    h_a = 1e-3 * float(torch.sqrt(torch.mean(torch.abs(a) ** 2)))
    # coefficient coordinates (chi^2 is quadratic in a: central differences are exact
    # up to rounding; differences of residuals avoid cancellation in chi^2 itself)
    worst_a, scale_a = 0.0, float(torch.max(torch.abs(galm)))
    nal = oracle.nalm(lmax, lmax)
    for _ in range(16):
        c = int(rng.integers(0, 2))
        m = int(rng.integers(0, lmax + 1))
        l = int(rng.integers(max(m, spin), lmax + 1))
        i = oracle.alm_index(l, m, lmax)
        part = 1.0 if (m == 0 or rng.random() < 0.5) else 1j
        e = torch.zeros((2, nal), dtype=torch.complex128, device="cuda")
        e[c, i] = h_a * part
        rp = plan.synth(a + e) - y
        rm = plan.synth(a - e) - y
        fd = float(torch.sum((rp - rm) * (rp + rm))) / (2 * h_a)
        got = float(galm[c, i].real) if part == 1.0 else float(galm[c, i].imag)
        worst_a = max(worst_a, abs(fd - got) / scale_a)
    # deflection coordinates: only point k moves, so chi^2 changes by its residual
    # alone.  Central differences at steps 1e-6 and 5e-7, combined by Richardson
    # extrapolation (at lmax 2048 the plain step-1e-6 difference carries a relative
    # h^2 term of order 1e-5).
    h = 1e-6
    ks = rng.choice(npts, 16, replace=False)
    comps = rng.integers(0, 2, 16)
    steps = (h, -h, h / 2, -h / 2)
    pts_al = []
    for k, c in zip(ks, comps):
        for st in steps:
            al = alpha[:, k].clone()
            al[c] += st
            pts_al.append(al)
    al_t = torch.stack(pts_al, dim=1).contiguous()
    sel = torch.from_numpy(np.repeat(ks, len(steps))).cuda()
    thd, phd, _ = G.deflect(th0[sel].contiguous(), ph0[sel].contiguous(), al_t, want_chi=False)
    small = G.Plan(thd, phd, lmax, lmax, spin, eps, "f64")
    fk = small.synth(a)
    small.close()
    plan.close()
    res = (fk - y[:, sel]).cpu().numpy()
    scale_p = float(torch.max(torch.abs(galpha)))
    worst_p = 0.0
    ga = galpha.cpu().numpy()
    for j, (k, c) in enumerate(zip(ks, comps)):
        q = res[:, 4 * j:4 * j + 4]
        fd1 = float(np.sum(q[:, 0] ** 2 - q[:, 1] ** 2)) / (2 * h)
        fd2 = float(np.sum(q[:, 2] ** 2 - q[:, 3] ** 2)) / h
        fd = (4 * fd2 - fd1) / 3
        worst_p = max(worst_p, abs(fd - ga[c, k]) / scale_p)
    say("  worst |fd - grad| / max|grad|: coefficients %.2e, deflection %.2e" % (worst_a, worst_p))
    assert worst_a <= 1e-8
    assert worst_p <= 1e-6
