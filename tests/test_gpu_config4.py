"""The batched uneven workload at its stated sizes (Sect. 4: many maps, and many maps
deflected with one set of angles), FP32 at epsilon 1e-5 on plans that pick their
oversampling by timing.

* Four instances of the 64-instance mix (lmax uniform in [512, 3000], spin 0 or 2,
  10^6 to 6x10^6 uniformly random points): the largest band limit, the most points,
  and the first remaining instance of each spin, run as one batch over worker
  streams, eagerly and as a captured graph replayed with new inputs.  Replays must
  equal eager batch calls; every instance is checked against the oracle on sampled
  points (synthesis) and with the adjoint's input supported on sampled points.
* Two geometries of the four-geometry reading (16 maps each) through the several-map
  calls, whose Legendre step runs on the matrix cores: every map against the oracle
  on sampled points, in both directions.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2304_10431_amd import workloads as wl

pytestmark = pytest.mark.gpu

EPS = 1e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def G():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2304_10431_amd import gsht
    return gsht


def picked_instances():
    specs = wl.batched_instances()
    pick = [int(np.argmax([s["lmax"] for s in specs])), int(np.argmax([s["npts"] for s in specs]))]
    for spin in (0, 2):
        pick.append(next(i for i, s in enumerate(specs) if s["spin"] == spin and i not in pick))
    return [(i, specs[i]) for i in pick]


def adjoint_err(got, ref, lmax):
    w = np.sqrt(oracle.alm_weights(lmax, lmax))[None, :]
    return oracle.eps_eff(got.astype(np.complex128) * w, ref * w)


def test_config4_batch_graph(G):
    inst = picked_instances()
    plans, alms, ys, pts, samples = [], [], [], [], []
    rng = np.random.default_rng(41)
    for i, s in inst:
        th, ph = wl.instance_points(s)
        say("instance %d: lmax %d spin %d npts %d" % (i, s["lmax"], s["spin"], s["npts"]))
        plans.append(G.Plan(torch.from_numpy(th).cuda(), torch.from_numpy(ph).cuda(), s["lmax"],
                            s["mmax"], s["spin"], EPS, "f32", sigma="tuned"))
        alms.append(torch.from_numpy(wl.instance_alm(s, s["alm_seed"])).cuda().to(torch.complex64))
        nc = oracle.ncomp(s["spin"])
        idx = np.sort(rng.choice(s["npts"], 600, replace=False))
        ysup = idx[:300]
        y = torch.zeros((nc, s["npts"]), dtype=torch.float32, device="cuda")
        yv = rng.standard_normal((nc, ysup.size))
        y[:, torch.from_numpy(ysup).cuda()] = torch.from_numpy(yv).cuda().float()
        ys.append(y)
        pts.append((th, ph))
        samples.append((idx, ysup, yv))
    batch = G.Batch(4)
    outs_s = batch.synth(plans, alms)
    outs_a = batch.adjoint(plans, ys)
    torch.cuda.synchronize()
    for k, (i, s) in enumerate(inst):
        th, ph = pts[k]
        idx, ysup, yv = samples[k]
        a_h = alms[k].cpu().numpy().astype(np.complex128)
        ref = oracle.synth(a_h, s["lmax"], s["mmax"], s["spin"], th[idx], ph[idx])
        e_s = oracle.eps_eff(outs_s[k][:, torch.from_numpy(idx).cuda()].double().cpu().numpy(), ref)
        refa = oracle.adjoint(yv.astype(np.float32).astype(np.float64), s["lmax"], s["mmax"],
                              s["spin"], th[ysup], ph[ysup])
        e_a = adjoint_err(outs_a[k].cpu().numpy(), refa, s["lmax"])
        say("  instance %d: eps_eff synthesis %.2e, adjoint %.2e (sigma %.2f)"
            % (i, e_s, e_a, plans[k].info()["sigma"]))
        assert e_s <= EPS and e_a <= EPS
    # one graph: the whole batch's synthesis and adjoint, replayed with new inputs
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        batch.synth(plans, alms, outs_s)
        batch.adjoint(plans, ys, outs_a)
    for rep in range(2):
        for a, y in zip(alms, ys):
            a.mul_(-0.5)
            y.mul_(2.0)
        graph.replay()
        torch.cuda.synchronize()
        eag_s = batch.synth(plans, alms)
        eag_a = batch.adjoint(plans, ys)
        torch.cuda.synchronize()
        for k in range(len(plans)):
            assert torch.equal(outs_s[k], eag_s[k])
            d = float(torch.linalg.norm((outs_a[k] - eag_a[k]).to(torch.complex128))
                      / torch.linalg.norm(eag_a[k].to(torch.complex128)))
            assert d <= 1e-6, d
        say("  replay %d equals eager batch calls" % rep)
    batch.close()
    for p in plans:
        p.close()


@pytest.mark.parametrize("group", [0, 2])
def test_config4_geometry_group_matrix_core(G, group):
    g = wl.batched_groups()[group]
    lmax, mmax, spin = g["lmax"], g["mmax"], g["spin"]
    nm = len(g["alm_seeds"])
    nc = oracle.ncomp(spin)
    th, ph = wl.instance_points(g)
    say("group %d: lmax %d spin %d npts %d, %d maps" % (group, lmax, spin, g["npts"], nm))
    plan = G.Plan(torch.from_numpy(th).cuda(), torch.from_numpy(ph).cuda(), lmax, mmax, spin,
                  EPS, "f32", sigma="tuned")
    a_h = np.stack([wl.instance_alm(g, sd) for sd in g["alm_seeds"]])
    mm = plan.synth_many(torch.from_numpy(a_h).cuda().to(torch.complex64))
    rng = np.random.default_rng(43 + group)
    idx = np.sort(rng.choice(g["npts"], 200, replace=False))
    got = mm[:, :, torch.from_numpy(idx).cuda()].double().cpu().numpy()
    del mm
    worst_s = max(oracle.eps_eff(got[k], oracle.synth(a_h[k], lmax, mmax, spin, th[idx], ph[idx]))
                  for k in range(nm))
    ysup = idx[:100]
    yv = rng.standard_normal((nm, nc, ysup.size)).astype(np.float32)
    ym = torch.zeros((nm, nc, g["npts"]), dtype=torch.float32, device="cuda")
    ym[:, :, torch.from_numpy(ysup).cuda()] = torch.from_numpy(yv).cuda()
    bm = plan.adjoint_many(ym).cpu().numpy()
    plan.close()
    worst_a = max(adjoint_err(bm[k], oracle.adjoint(yv[k].astype(np.float64), lmax, mmax, spin,
                                                    th[ysup], ph[ysup]), lmax)
                  for k in range(nm))
    say("  worst eps_eff over %d maps: synthesis %.2e, adjoint %.2e" % (nm, worst_s, worst_a))
    assert worst_s <= EPS and worst_a <= EPS
