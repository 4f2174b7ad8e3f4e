"""The FP64 fused column stage (mode 2) is compiled once per count of register slots
per thread (the transform lengths nd and n1 / 2 over the workgroup's threads) and
launched with the smallest count that holds the plan's transforms.  Each case below
lands on a different count, up to the largest column the mode takes, and is checked
against the same plan's library-FFT column stage (mode 0), synthesis and adjoint,
and against the FP64 oracle on a few points (Sect. 3, the FFT step of the method).
"""
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


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# (lmax, sigma, eps): slot counts per thread (1024 threads) of the forward and the
# adjoint kernel, ceil(n1 / 2 / 1024) and ceil(max(nd, n1 / 2) / 1024): (1, 1), (2, 3),
# (3, 4), (4, 5), (5, 6), (6, 7), (8, 8), (6, 9) and (8, 10), the last at the largest
# column the fused stage takes (sigma 1.25 reaches 1e-9, not 1e-10)
@pytest.mark.parametrize("lmax,sigma,eps", [(300, 2.0, 1e-10), (1100, 1.5, 1e-10),
                                            (1600, 1.5, 1e-10), (2100, 1.5, 1e-10),
                                            (2800, 1.5, 1e-10), (3500, 1.5, 1e-10),
                                            (3100, 2.0, 1e-10), (4200, 1.25, 1e-9),
                                            (4800, 1.5, 1e-10)])
def test_column_slot_instances(G, monkeypatch, lmax, sigma, eps):
    say("column slots", lmax, sigma, eps)
    rng = np.random.default_rng(900 + lmax)
    th, ph = wl.uniform_sphere(3000, rng)
    spin = 2
    a = wl.gaussian_alm(lmax, lmax, spin, rng)
    y = rng.standard_normal((oracle.ncomp(spin), th.size))
    w = np.sqrt(oracle.alm_weights(lmax, lmax))[None, :]
    outs = {}
    for mode in (2, 0):
        monkeypatch.setenv("GSHT_COLUMN_MODE", str(mode))
        plan = G.Plan(dev(th), dev(ph), lmax, lmax, spin, eps, "f64", sigma=sigma)
        inf = plan.info()
        assert inf["column_mode"] == mode
        if mode == 2:
            nd, nh = inf["ndouble"], inf["n1"] // 2
            say("  nd %d, n1 %d: slots %d / %d" % (nd, inf["n1"], -(-nh // 1024),
                                                  -(-max(nd, nh) // 1024)))
        m = plan.synth(dev(a)).cpu().numpy()
        b = plan.adjoint(dev(y)).cpu().numpy()
        plan.close()
        outs[mode] = (m, b)
    assert rel_l2(outs[2][0], outs[0][0]) <= 1e-12
    assert rel_l2(outs[2][1] * w, outs[0][1] * w) <= 1e-12
    # a few points against the oracle's direct sum (its cost grows as lmax^2 per point)
    sel = np.arange(0, th.size, 300)
    ref = oracle.synth(a, lmax, lmax, spin, th[sel], ph[sel])
    assert oracle.eps_eff(outs[2][0][:, sel], ref) <= eps
