"""Graph capture: a plan's synthesis and adjoint (and the several-map synthesis,
after its first call has allocated its buffers) issue only kernel launches and
library FFT launches on the caller's stream, so they can be captured in a HIP graph
and replayed.  Each replay gets new input values (copied into the captured input
buffers), runs with other eager work of the same plan in between, and must match an
eager run on the same input (the adjoint's atomic sums may differ in the order of
additions, hence a rounding tolerance there)."""
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


def rel(a, b):
    dt = torch.complex128 if a.is_complex() else torch.float64
    a, b = a.to(dt), b.to(dt)
    return float(torch.linalg.norm((a - b).flatten()) / max(torch.linalg.norm(b.flatten()), 1e-300))


@pytest.mark.parametrize("spin,lmax,npts,prec,eps", [(2, 200, 30000, "f32", 1e-5),
                                                     (0, 150, 20000, "f64", 1e-10),
                                                     (1, 97, 10000, "f64", 1e-12)])
def test_graph_replays_match_eager(G, spin, lmax, npts, prec, eps):
    say("graph", spin, lmax, npts, prec, eps)
    rng = np.random.default_rng(700 + lmax)
    th, ph = wl.uniform_sphere(npts, rng)
    cdt = torch.complex128 if prec == "f64" else torch.complex64
    rdt = torch.float64 if prec == "f64" else torch.float32
    plan = G.Plan(torch.from_numpy(th).cuda(), torch.from_numpy(ph).cuda(), lmax, lmax, spin, eps,
                  prec)
    inputs = [torch.from_numpy(wl.gaussian_alm(lmax, lmax, spin, np.random.default_rng(k))).cuda()
              .to(cdt) for k in range(4)]
    a_s = inputs[0].clone()
    m_s = plan.synth(a_s)
    b_s = plan.adjoint(m_s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.synth(a_s, out=m_s)
        plan.adjoint(m_s, out=b_s)
    torch.cuda.synchronize()
    tol_b = 1e-13 if prec == "f64" else 1e-6
    w = torch.from_numpy(np.sqrt(oracle.alm_weights(lmax, lmax))).cuda()
    for k in (1, 2, 3, 1):
        a_s.copy_(inputs[k])
        graph.replay()
        # eager work of the same plan between replays (same workspace)
        m_e = plan.synth(inputs[k])
        b_e = plan.adjoint(m_e)
        torch.cuda.synchronize()
        e_m, e_b = rel(m_s, m_e), rel(b_s * w, b_e * w)
        say("  replay input %d: synth %.2e adjoint %.2e" % (k, e_m, e_b))
        assert e_m == 0.0
        assert e_b <= tol_b
    # the replays compute the transform itself, not a stale copy
    ref = oracle.synth(inputs[1][:, :].cpu().numpy().astype(np.complex128), lmax, lmax, spin,
                       th[:2000], ph[:2000])
    a_s.copy_(inputs[1])
    graph.replay()
    torch.cuda.synchronize()
    assert oracle.eps_eff(m_s[:, :2000].double().cpu().numpy(), ref) <= eps
    plan.close()


def test_graph_many_maps(G):
    """Several-map synthesis on the matrix cores, captured after a first eager call."""
    spin, lmax, npts, nm = 2, 130, 8000, 12
    say("graph many", spin, lmax, npts, nm)
    rng = np.random.default_rng(77)
    th, ph = wl.uniform_sphere(npts, rng)
    plan = G.Plan(torch.from_numpy(th).cuda(), torch.from_numpy(ph).cuda(), lmax, lmax, spin, 1e-5,
                  "f32")
    alms = [torch.from_numpy(np.stack([wl.gaussian_alm(lmax, lmax, spin, np.random.default_rng(10 * j + k))
                                       for k in range(nm)])).cuda().to(torch.complex64) for j in range(3)]
    a_s = alms[0].clone()
    m_s = plan.synth_many(a_s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.synth_many(a_s, out=m_s)
    for j in (1, 2, 1):
        a_s.copy_(alms[j])
        graph.replay()
        m_e = plan.synth_many(alms[j])
        torch.cuda.synchronize()
        e = rel(m_s, m_e)
        say("  replay %d: %.2e" % (j, e))
        assert e == 0.0
    plan.close()
