"""Moving an existing plan to new points (gsht_plan_set_points): only the bin sort is
redone, so a moved plan must give what a plan built on the new points gives — the
synthesis bit for bit (same sort, same per-point arithmetic), the adjoint to rounding
(spreading may flush with atomics) — for fewer and as many points as the plan was
built with; counts beyond that capacity and invalid points are refused; and
Lensing.update (new potential, same pixels) must equal a lensing operator built on
the new potential."""
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


def _points(n, seed):
    rng = np.random.default_rng(seed)
    return np.arccos(rng.uniform(-1, 1, n)), rng.uniform(0, 2 * np.pi, n)


def _alm(spin, lmax, mmax, seed, decay=0.0):
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


@pytest.mark.parametrize("prec,eps,tol", [("f64", 1e-10, 1e-13), ("f32", 1e-5, 1e-6)])
@pytest.mark.parametrize("spin,lmax,mmax", [(0, 200, 200), (2, 257, 190)])
def test_moved_plan_equals_fresh_plan(G, prec, eps, tol, spin, lmax, mmax):
    say("set_points", prec, spin, lmax, mmax)
    cap = 30000
    th0, ph0 = _points(cap, 1)
    cdt = torch.complex128 if prec == "f64" else torch.complex64
    rdt = torch.float64 if prec == "f64" else torch.float32
    a = dev(_alm(spin, lmax, mmax, 2)).to(cdt)
    plan = G.Plan(dev(th0), dev(ph0), lmax, mmax, spin, eps, prec)
    w = np.sqrt(oracle.alm_weights(lmax, mmax))[None, :]
    # fewer points, clustered in one cap (other tiles empty), then as many as the capacity
    th1, ph1 = _points(12345, 3)
    th1 = th1 * 0.2
    th1[:2] = [0.0, 0.2]
    th2, ph2 = _points(cap, 4)
    th2[:2] = [0.0, math.pi]
    for th, ph in ((th1, ph1), (th2, ph2)):
        plan.set_points(dev(th), dev(ph))
        assert plan.npts == th.size
        fresh = G.Plan(dev(th), dev(ph), lmax, mmax, spin, eps, prec)
        m_moved = plan.synth(a).cpu()
        m_fresh = fresh.synth(a).cpu()
        assert torch.equal(m_moved, m_fresh)
        y = dev(np.random.default_rng(th.size).standard_normal((oracle.ncomp(spin), th.size))).to(rdt)
        b_moved = plan.adjoint(y).to(torch.complex128).cpu().numpy()
        b_fresh = fresh.adjoint(y).to(torch.complex128).cpu().numpy()
        fresh.close()
        e = oracle.eps_eff(w * b_moved, w * b_fresh)
        ref = oracle.synth(a.to(torch.complex128).cpu().numpy(), lmax, mmax, spin, th[:500], ph[:500])
        e_o = oracle.eps_eff(m_moved.double().numpy()[:, :500], ref)
        say("  npts %d: adjoint moved vs fresh %.3e, synth vs oracle %.3e" % (th.size, e, e_o))
        assert e <= tol
        assert e_o <= eps
    # back to an empty point set and out again
    plan.set_points(dev(th1[:0]), dev(ph1[:0]))
    assert plan.synth(a).shape == (oracle.ncomp(spin), 0)
    plan.set_points(dev(th0), dev(ph0))
    fresh = G.Plan(dev(th0), dev(ph0), lmax, mmax, spin, eps, prec)
    assert torch.equal(plan.synth(a).cpu(), fresh.synth(a).cpu())
    fresh.close()
    plan.close()


def test_set_points_refusals(G):
    say("set_points refusals")
    th, ph = _points(5000, 7)
    plan = G.Plan(dev(th), dev(ph), 64, 64, 1, 1e-10, "f64")
    a = dev(_alm(1, 64, 64, 8))
    before = plan.synth(a).cpu()
    big_t, big_p = _points(5001, 9)
    with pytest.raises(G.GshtError, match="capacity"):
        plan.set_points(dev(big_t), dev(big_p))
    bad = th.copy()
    bad[17] = 4.0
    with pytest.raises(G.GshtError, match="theta outside"):
        plan.set_points(dev(bad), dev(ph))
    # the refused sort left no valid points: every transform is refused on the host
    y = dev(np.random.default_rng(3).standard_normal((2, 5000)))
    for call in (lambda: plan.synth(a), lambda: plan.adjoint(y),
                 lambda: plan.synth_many(a.unsqueeze(0)), lambda: plan.adjoint_many(y.unsqueeze(0)),
                 lambda: plan.synth_deriv(a), lambda: plan.synth_vjp(a, y)):
        with pytest.raises(G.GshtError, match="no valid points"):
            call()
    plan.set_points(dev(th), dev(ph))             # valid points again: same results as before
    assert torch.equal(plan.synth(a).cpu(), before)
    plan.close()


@pytest.mark.parametrize("spin", [0, 2])
def test_lensing_update_equals_new_operator(G, spin):
    from paper_2304_10431_amd.lensing import Lensing
    say("lensing update", spin)
    lmax = mmax = 96
    lmax_p = 64
    th, ph = _points(20000, 20 + spin)
    a = dev(_alm(spin, lmax, mmax, 21))

    def pot(seed):
        p = _alm(0, lmax_p, lmax_p, seed, decay=2.5)[0]
        p[:2] = 0.0
        return dev(p * 2e-3)

    p1, p2 = pot(22), pot(23)
    L = Lensing(dev(th), dev(ph), p1, lmax, mmax, spin, 1e-10, "f64", lmax_p=lmax_p)
    first = L.forward(a).cpu()
    L.update(p2)
    M = Lensing(dev(th), dev(ph), p2, lmax, mmax, spin, 1e-10, "f64", lmax_p=lmax_p)
    assert torch.equal(L.theta_d.cpu(), M.theta_d.cpu())
    moved, new = L.forward(a).cpu(), M.forward(a).cpu()
    assert torch.equal(moved, new)
    assert not torch.equal(moved, first)
    y = dev(np.random.default_rng(24).standard_normal((oracle.ncomp(spin), th.size)))
    e = oracle.eps_eff(L.adjoint(y).cpu().numpy(), M.adjoint(y).cpu().numpy())
    say("  adjoint updated vs new %.3e" % e)
    assert e <= 1e-13
    with pytest.raises(ValueError):
        L.update(p1, olm=p2)
    L.close()
    M.close()
