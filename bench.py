"""Benchmark: general spin-2 synthesis + adjoint at lmax 4096 on ~48M deflected points.

One step = one synthesis (a_lm -> map) plus one adjoint (map -> a_lm) through the
C ABI (plan API, geometry reused as in the paper's lensing use), with all inputs
resident in HBM.  Forms timed:

  * FP64 form, epsilon = 1e-10  (headline ``value``: seconds per step, the paper's
    double precision)
  * FP32 form, epsilon = 1e-5   (FFT/NUFFT in FP32, Legendre recurrence in FP64)
  * FP64 form, epsilon = 1e-5   (for the FP32-vs-FP64 speed-up at equal accuracy)

Workload: spin 2, lmax = mmax = 4096, Gaussian E/B a_lm, points of a 6144-ring
longitude-thinned Gauss-Legendre grid displaced along great circles by the gradient
of a Gaussian lensing potential (C_L ~ L^-4 above L = 60, 2.5 arcmin rms; about
4.8e7 points, the "~5e7 pixel" intermediate grid of the paper's Sect. 4 benchmark).
The deflection is computed by the library (FP64 spin-1 synthesis, great-circle
step).  Synthetic data, generated with fixed seeds.

Reported beside the headline: synthesis and adjoint times of each form (HIP events
on the stream the library launches on, timed with the library's profiling off);
per-stage times from a separate profiled pass of the same steps; the dominant
kernel's achieved fraction of its MI355X roofline (``roofline``) and the same figure
for the other main kernels; the spreading stage's HBM fraction and LDS atomic rate;
the several-map (matrix-core) forms; the batched uneven workload (64 instances as
one captured graph, and 4 geometries x 16 maps); the FP64 CPU oracle timed on a
bounded sample of points on the host cores, with each form's effective accuracy
against the oracle's values at 10^4 sampled points; and the plain CPU NUFFT-based
SHT timed at lmax 2048 on 8.4M deflected points.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "synth+adjoint s @ lmax4096 spin2 ~50M pts: FP32 eps1e-5 vs FP64 eps1e-10; %roof"
FP64_VECTOR_PEAK_TFLOPS = 78.6   # MI355X: 256 CU x 2.4 GHz x 128 FP64 flop/clk/CU
HBM_PEAK_GBS = 8000.0
CALIB_BYTES = 1 << 30            # plain copy used to calibrate the HBM byte counters
GOLDEN = os.path.join(ROOT, "tests", "golden")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_%s.json")
CSRC = os.path.join(ROOT, "paper_2304_10431_amd", "csrc")
# sources that define each stage's kernels (a traffic record holds only for them)
STAGE_SOURCES = {
    "legendre_synth": ["legendre_kernels.hip", "legendre_device.hpp"],
    "legendre_adj": ["legendre_kernels.hip", "legendre_device.hpp"],
    "spread": ["nufft.hip"],
    "interp": ["nufft.hip"],
    "column_fwd": ["colfft.hip"],
    "column_adj": ["colfft.hip"],
}
HEADLINE = "f64_eps1e-10"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sources_sha(stage):
    h = hashlib.sha256()
    for f in STAGE_SOURCES[stage]:
        h.update(open(os.path.join(CSRC, f), "rb").read())
    return h.hexdigest()


def measured_traffic(workload, form, stage, w=None):
    """HBM bytes per call of a stage (summed over its launches) from the committed
    counter runs, or None if they were taken on another workload or form, on a
    different version of the stage's kernel sources, or (NUFFT stages) with another
    kernel support w."""
    try:
        rec = json.load(open(TRAFFIC_FILE % workload))[form][stage]
    except (OSError, ValueError, KeyError):
        return None
    if rec.get("kernel_source_sha256") != sources_sha(stage):
        return None
    if "w" in rec and w is not None and rec["w"] != w:
        return None
    return rec.get("bytes_per_call")


def legendre_flops(lmax, mmax, spin):
    """Algorithmic FP64 flops of one Legendre launch: per (l, m, ring pair) unit,
    8 flop for spin 0 (2 FMA recurrence + 2 FMA accumulation) and 24 flop for
    spin > 0 (2 recurrences + 4 complex-by-real accumulations), over
    max(m, s) <= l <= lmax, 0 <= m <= mmax and the (lmax + 2) / 2 ring pairs of the
    smallest ring grid that is exact (lmax + 2 rings)."""
    units = 0
    for m in range(mmax + 1):
        l0 = max(m, spin)
        if l0 <= lmax:
            units += lmax - l0 + 1
    per = 8 if spin == 0 else 24
    return per * units * ((lmax + 3) // 2)


def stage_bytes(stage, info, npts, ncomp, prec):
    """Algorithmic HBM bytes of one call of an HBM-bound stage.
    spread: per point its sorted FP64 (theta, phi) (16 B), 4 B permutation entry and
    ncomp map values, plus one read and one write of every kept grid cell, times the
    patch halo factor ((T + w - 1) / T)^2.  interp: the same with one read of the grid.
    column_fwd: the doubled columns read once (ncol x nd complex) and the kept rows of
    the oversampled columns written once (ncol x nrows complex); column_adj: the
    reverse."""
    rs = 8 if prec == "f64" else 4
    cs = 2 * rs
    w, t1, t2 = info["w"], info["tile1"], info["tile2"]
    halo = (t1 + w - 1) * (t2 + w - 1) / float(t1 * t2)
    grid = info["nrows"] * info["n2"] * ncomp * rs
    pts = npts * (16 + 4 + ncomp * rs)
    ncol = 2 * info["mmax"] + 1 if ncomp == 2 else info["mmax"] + 1
    if stage == "spread":
        return pts + 2 * grid * halo
    if stage == "interp":
        return pts + grid * halo
    if stage in ("column_fwd", "column_adj"):
        return ncol * (info["ndouble"] + info["nrows"]) * cs
    return None


def roofline_entry(stage, form_key, r, spec, npts, workload):
    info, st = r["info"], r["stages"]
    ms, cnt = st[stage]
    if not cnt:
        return None
    avg_s = ms / cnt / 1e3
    ncomp = 2 if spec["spin"] else 1
    if stage.startswith("legendre"):
        flops = legendre_flops(spec["lmax"], spec["mmax"], spec["spin"])
        ach = flops / avg_s / 1e12
        e = {"kernel": stage, "bound": "alu", "achieved": ach, "peak": FP64_VECTOR_PEAK_TFLOPS,
             "unit": "TFLOP/s", "frac": ach / FP64_VECTOR_PEAK_TFLOPS, "flops_per_launch": flops}
    else:
        nb = stage_bytes(stage, info, npts, ncomp, form_key[:3])
        if nb is None:
            return None
        ach = nb / avg_s / 1e9
        e = {"kernel": stage, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
             "unit": "GB/s", "frac": ach / HBM_PEAK_GBS, "bytes_per_launch": nb}
    e["avg_launch_ms"] = avg_s * 1e3
    e["traffic"] = measured_traffic(workload, form_key, stage, info["w"])
    return e


def time_form(gsht, torch, th, ph, alm, spec, prec, eps, steps, warmup, many=0, autotune=False,
              check=None, sigma="tuned"):
    lmax, mmax, spin = spec["lmax"], spec["mmax"], spec["spin"]
    cdt = torch.complex128 if prec == "f64" else torch.complex64
    t0 = time.time()
    plan = gsht.Plan(th, ph, lmax, mmax, spin, eps, prec, sigma=sigma)
    if autotune:
        plan.autotune()
    torch.cuda.synchronize()
    t_plan = time.time() - t0
    a = alm.to(cdt)
    m = plan.synth(a)
    b = plan.adjoint(m)
    for _ in range(warmup):
        plan.synth(a, out=m)
        plan.adjoint(m, out=b)
    torch.cuda.synchronize()
    # timed steps, library profiling off; the library launches on torch's current
    # stream, so events recorded there bracket exactly one synthesis and one adjoint
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        ev[k][0].record()
        plan.synth(a, out=m)
        ev[k][1].record()
        plan.adjoint(m, out=b)
        ev[k][2].record()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    syn_ms = sum(e[0].elapsed_time(e[1]) for e in ev) / steps
    adj_ms = sum(e[1].elapsed_time(e[2]) for e in ev) / steps
    # per-stage times: a separate pass of the same steps with the library's events on
    plan.set_profiling(True)
    for _ in range(steps):
        plan.synth(a, out=m)
        plan.adjoint(m, out=b)
    torch.cuda.synchronize()
    stages = plan.stage_times()
    plan.set_profiling(False)
    info = plan.info()
    r = dict(s_per_step=dt, synth_ms=syn_ms, adjoint_ms=adj_ms, plan_s=t_plan, stages=stages,
             info=info)
    if check is not None:
        r["check_synth"] = m[:, check["idx"]].double().cpu().numpy()
        rdt = torch.float64 if prec == "f64" else torch.float32
        r["check_adjoint"] = plan.adjoint(check["yfull"].to(rdt)).to(torch.complex128).cpu().numpy()
    if spin > 0:
        # the gradient-only setting (C = 0): same plan, same step count
        g = a[:1].contiguous()
        bg = plan.adjoint_grad(m)
        plan.synth_grad(g, out=m)
        torch.cuda.synchronize()
        evg = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
        for k in range(steps):
            evg[k][0].record()
            plan.synth_grad(g, out=m)
            evg[k][1].record()
            plan.adjoint_grad(m, out=bg)
            evg[k][2].record()
        torch.cuda.synchronize()
        r["gradient_only"] = {
            "synth_ms": sum(e[0].elapsed_time(e[1]) for e in evg) / steps,
            "adjoint_ms": sum(e[1].elapsed_time(e[2]) for e in evg) / steps}
        del g, bg
    del m, b
    if many > 1:
        r.update(time_many(plan, torch, a, prec, steps, many, check))
    return plan, r


def time_many(plan, torch, a, prec, steps, many, check):
    """Several maps on the same plan: FP32 plans take groups of 8..16 maps through the
    matrix-core Legendre step, smaller groups (and FP64) through the FP64 group kernel."""
    out = {}
    fac = torch.linspace(0.5, 2.0, many, device=a.device)
    am = (a.unsqueeze(0) * fac.to(a.dtype)[:, None, None]).contiguous()
    mm = plan.synth_many(am)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        plan.synth_many(am, out=mm)
    e1.record()
    torch.cuda.synchronize()
    kind = "mfma" if (prec == "f32" and many >= 8) else "fp64"
    out["synth_many"] = {"maps": many, "synth_ms_per_map": e0.elapsed_time(e1) / steps / many,
                         "legendre": kind}
    plan.set_profiling(True)
    plan.synth_many(am, out=mm)
    st = plan.stage_times()
    plan.set_profiling(False)
    out["synth_many"]["legendre_ms_per_map"] = st["legendre_synth"][0] / many
    out["synth_many"]["prep_ms_per_map"] = st["prep_alm"][0] / many
    one = plan.synth(am[many - 1].contiguous())
    out["synth_many"]["eps_vs_single"] = float(torch.linalg.norm((mm[many - 1] - one).double())
                                               / torch.linalg.norm(one.double()))
    del am, one
    if check is not None:
        out["many_check"] = {"synth": (mm[many - 1][:, check["idx"]] / fac[-1]).double().cpu().numpy()}
    bm = plan.adjoint_many(mm)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        plan.adjoint_many(mm, out=bm)
    e1.record()
    torch.cuda.synchronize()
    out["adjoint_many"] = {"maps": many, "adjoint_ms_per_map": e0.elapsed_time(e1) / steps / many,
                           "legendre": kind}
    plan.set_profiling(True)
    plan.adjoint_many(mm, out=bm)
    st = plan.stage_times()
    plan.set_profiling(False)
    out["adjoint_many"]["legendre_ms_per_map"] = st["legendre_adj"][0] / many
    out["adjoint_many"]["prep_ms_per_map"] = st["prep_alm"][0] / many
    one = plan.adjoint(mm[many - 1].contiguous())
    out["adjoint_many"]["eps_vs_single"] = float(
        torch.linalg.norm((bm[many - 1] - one).to(torch.complex128))
        / torch.linalg.norm(one.to(torch.complex128)))
    del bm, one
    if check is not None:
        ym = (check["yfull"].to(mm.dtype).unsqueeze(0) * fac[:, None, None]).contiguous()
        bmy = plan.adjoint_many(ym)
        out["many_check"]["adjoint"] = (bmy[many - 1] / fac[-1]).to(torch.complex128).cpu().numpy()
        del ym, bmy
    del mm
    return out


def load_samples(workload):
    """The committed oracle values at 10^4 sampled points of the workload (written by
    tests/golden/make_fullsize_samples.py), or None."""
    path = os.path.join(GOLDEN, "%s_samples.npz" % workload)
    if not os.path.exists(path):
        return None
    with np.load(path) as f:
        return {k: f[k] for k in ("idx", "theta", "phi", "synth")}


def adjoint_columns(mmax, seed=17):
    rng = np.random.default_rng(seed)
    mid = rng.choice(np.arange(4, mmax), 20, replace=False)
    return np.concatenate([[0, 1, 2, 3], np.sort(mid), [mmax]]).astype(np.int32)


def accuracy_and_cpu_baseline(spec, alm_h, fx, sup, y_s, results, time_sample):
    """Each form's effective accuracy against the oracle (synthesis at the 10^4 sampled
    points; adjoint of an input supported on 5000 of them, on 25 columns m), and the
    oracle (FP64 direct sum, all host cores) timed on a bounded sample of the points:
    synthesis and full adjoint on time_sample points, scaled linearly to the workload."""
    import oracle
    lmax, mmax, spin = spec["lmax"], spec["mmax"], spec["spin"]
    cores = len(os.sched_getaffinity(0))
    th_s, ph_s = fx["theta"][sup], fx["phi"][sup]
    ms = adjoint_columns(mmax)
    ref_adj = oracle.adjoint_cols(y_s, lmax, mmax, spin, th_s, ph_s, ms, nthreads=cores)
    sel = np.zeros(oracle.nalm(lmax, mmax), bool)
    for m in ms:
        i0 = oracle.alm_index(m, m, lmax)
        sel[i0:i0 + lmax + 1 - m] = True
    wts = np.sqrt(oracle.alm_weights(lmax, mmax))[sel][None, :]
    err = {}
    for k, r in results.items():
        err[k] = {"synthesis": oracle.eps_eff(r["check_synth"], fx["synth"]),
                  "adjoint": oracle.eps_eff(wts * r["check_adjoint"][:, sel], wts * ref_adj[:, sel])}
        mc = r.get("many_check")
        if mc:
            err[k]["synthesis_many"] = oracle.eps_eff(mc["synth"], fx["synth"])
            err[k]["adjoint_many"] = oracle.eps_eff(wts * mc["adjoint"][:, sel], wts * ref_adj[:, sel])
    # timing sample: spread over the three groups
    pick = np.random.default_rng(12345).choice(fx["idx"].size, time_sample, replace=False)
    th_t, ph_t = fx["theta"][pick], fx["phi"][pick]
    t0 = time.time()
    oracle.synth(alm_h, lmax, mmax, spin, th_t, ph_t, nthreads=cores)
    t_syn = time.time() - t0
    log("oracle synthesis on %d points: %.1f s" % (time_sample, t_syn))
    y_t = np.random.default_rng(7).standard_normal((2 if spin else 1, time_sample))
    t0 = time.time()
    oracle.adjoint(y_t, lmax, mmax, spin, th_t, ph_t, nthreads=cores)
    t_adj = time.time() - t0
    log("oracle adjoint on %d points: %.1f s" % (time_sample, t_adj))
    npts = spec["npts_total"]
    per_step = (t_syn + t_adj) * npts / time_sample
    cb = dict(value=per_step, unit="s", cores=cores, kind="oracle",
              sample="%d of the sampled points of the %d-point workload: synthesis %.1f s + "
                     "adjoint %.1f s on %d threads, scaled linearly to all points"
                     % (time_sample, npts, t_syn, t_adj, cores))
    return cb, err


def cpu_nufft_baseline(eps=1e-10):
    """The plain CPU NUFFT-based SHT of the oracle package (FP64, all host cores), one
    synthesis and one adjoint at lmax 2048, spin 0, on the 2049 x 4097 Gauss-Legendre
    grid deflected by the workload's potential (deflection computed by the same CPU
    code, untimed), with its own parameter choice for eps."""
    import oracle
    from oracle import lensing as ol
    from oracle import nufft_sht
    from paper_2304_10431_amd import workloads as wl
    spec = wl.WORKLOADS["tlens_l2048"]
    lmax, mmax, spin = spec["lmax"], spec["mmax"], spec["spin"]
    cores = len(os.sched_getaffinity(0))
    th0, ph0 = wl.base_points(spec)
    g = np.zeros((2, oracle.nalm(lmax, lmax)), dtype=np.complex128)
    g[0] = wl.make_potential(spec)
    t0 = time.time()
    alpha = nufft_sht.synth(ol.lscale(g, lmax, lmax), lmax, lmax, 1, th0, ph0, nthreads=cores,
                            **nufft_sht.default_params(lmax, lmax, 1e-12))
    th, ph, _ = ol.deflect(th0, ph0, alpha)
    del alpha, th0, ph0
    log("cpu nufft: deflected %d points (%.1f s, untimed)" % (th.size, time.time() - t0))
    alm_h = wl.make_alm(spec)
    p = nufft_sht.default_params(lmax, mmax, eps)
    t0 = time.time()
    m = nufft_sht.synth(alm_h, lmax, mmax, spin, th, ph, nthreads=cores, **p)
    t_syn = time.time() - t0
    log("cpu nufft synthesis %.1f s" % t_syn)
    t0 = time.time()
    nufft_sht.adjoint(m, lmax, mmax, spin, th, ph, nthreads=cores, **p)
    t_adj = time.time() - t0
    log("cpu nufft adjoint %.1f s" % t_adj)
    return dict(value=t_syn + t_adj, unit="s", cores=cores, kind="oracle (plain CPU NUFFT SHT)",
                eps=eps, params=p, workload="tlens_l2048: spin 0, lmax 2048, %d deflected "
                "Gauss-Legendre points" % th.size,
                sample="whole workload, one synthesis (%.1f s) + one adjoint (%.1f s), FP64"
                       % (t_syn, t_adj))


def batched(gsht, torch, steps, warmup, nstreams=4):
    """The batched uneven workload, FP32 at eps 1e-5 on plans that pick their
    oversampling by timing: (a) 64 independent instances, synthesis + adjoint of all of
    them as one captured graph over worker streams; (b) 4 geometries x 16 maps through
    the several-map calls (matrix-core Legendre step)."""
    from paper_2304_10431_amd import workloads as wl
    out = {}
    specs = wl.batched_instances()
    t0 = time.time()
    plans, alms, maps, adjs = [], [], [], []
    for k, s in enumerate(specs):
        th, ph = wl.instance_points(s)
        plans.append(gsht.Plan(torch.from_numpy(th).cuda(), torch.from_numpy(ph).cuda(), s["lmax"],
                               s["mmax"], s["spin"], 1e-5, "f32", sigma="tuned"))
        alms.append(torch.from_numpy(wl.instance_alm(s, s["alm_seed"])).cuda().to(torch.complex64))
        if k % 16 == 15:
            log("batch: %d plans (%.0f s)" % (k + 1, time.time() - t0))
    torch.cuda.synchronize()
    t_plans = time.time() - t0
    batch = gsht.Batch(nstreams)
    maps = batch.synth(plans, alms)
    adjs = batch.adjoint(plans, maps)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        batch.synth(plans, alms, maps)
        batch.adjoint(plans, maps, adjs)
    for _ in range(warmup):
        graph.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        graph.replay()
    e1.record()
    torch.cuda.synchronize()
    out["instances_graph"] = {
        "instances": len(specs), "points": int(sum(s["npts"] for s in specs)),
        "ms_per_step": e0.elapsed_time(e1) / steps, "streams": nstreams, "plans_s": t_plans,
        "sigma": sorted({p.info()["sigma"] for p in plans})}
    log("batch: 64 instances, %.1f ms per synthesis + adjoint (graph)"
        % out["instances_graph"]["ms_per_step"])
    del graph
    batch.close()
    for p in plans:
        p.close()
    del plans, alms, maps, adjs
    torch.cuda.empty_cache()
    groups = wl.batched_groups()
    tot, t_plans = 0.0, 0.0
    for g in groups:
        th, ph = wl.instance_points(g)
        t0 = time.time()
        plan = gsht.Plan(torch.from_numpy(th).cuda(), torch.from_numpy(ph).cuda(), g["lmax"],
                         g["mmax"], g["spin"], 1e-5, "f32", sigma="tuned")
        t_plans += time.time() - t0
        am = torch.from_numpy(np.stack([wl.instance_alm(g, sd) for sd in g["alm_seeds"]])).cuda()
        am = am.to(torch.complex64)
        mm = plan.synth_many(am)
        bm = plan.adjoint_many(mm)
        for _ in range(warmup):
            plan.synth_many(am, out=mm)
            plan.adjoint_many(mm, out=bm)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(steps):
            plan.synth_many(am, out=mm)
            plan.adjoint_many(mm, out=bm)
        e1.record()
        torch.cuda.synchronize()
        tot += e0.elapsed_time(e1) / steps
        plan.close()
        del am, mm, bm
        torch.cuda.empty_cache()
    out["groups_many"] = {"groups": len(groups), "maps": sum(len(g["alm_seeds"]) for g in groups),
                          "ms_per_step": tot, "plans_s": t_plans,
                          "shapes": [[g["lmax"], g["spin"], g["npts"]] for g in groups]}
    log("batch: 4 x 16 maps, %.1f ms per synthesis + adjoint" % tot)
    return out


def point_desc(spec):
    if spec["points"] == "thin":
        return ("%d-ring longitude-thinned Gauss-Legendre grid deflected by a 2.5 arcmin rms "
                "Gaussian lensing potential" % spec["nring"])
    if spec["points"] == "gl":
        return ("%d x %d Gauss-Legendre grid deflected by a 2.5 arcmin rms Gaussian lensing "
                "potential" % (spec["nring"], spec["nphi"]))
    return "uniform random points"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="pollens_thin6144")
    ap.add_argument("--cpu-sample", type=int, default=2048)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle leg")
    ap.add_argument("--no-cpu-nufft", action="store_true",
                    help="skip the plain CPU NUFFT-based SHT baseline")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched uneven workload")
    ap.add_argument("--autotune", action="store_true",
                    help="let each plan time the Legendre launch shapes and keep the fastest")
    ap.add_argument("--many", type=int, default=16,
                    help="maps per call for the several-map timing (FP32 form; 0: off)")
    ap.add_argument("--forms", default="f64:1e-10,f32:1e-5,f64:1e-5",
                    help="comma-separated precision:epsilon forms (the headline is f64:1e-10)")
    ap.add_argument("--sigma", default="tuned",
                    help="oversampling factor of the plans: tuned (gsht_plan_create_tuned picks "
                         "the fastest of 2, 1.5, 1.25 at plan time) or one of 2, 1.5, 1.25")
    ap.add_argument("--copy-calib", action="store_true",
                    help="run one plain 1 GiB device-to-device copy first (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on exactly one GPU; --gpus %d is not supported "
              "(the multi-GPU sharding is described, not built)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    log("importing torch")
    import torch
    from paper_2304_10431_amd import gsht
    from paper_2304_10431_amd import workloads as wl
    from paper_2304_10431_amd.lensing import deflected_points

    spec = dict(wl.WORKLOADS[args.workload])
    lmax, mmax, spin = spec["lmax"], spec["mmax"], spec["spin"]
    ncomp = 2 if spin else 1
    if args.copy_calib:
        src = torch.ones(CALIB_BYTES // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    t0 = time.time()
    log("generating %s points" % args.workload)
    th0, ph0 = wl.base_points(spec)
    th = torch.from_numpy(th0).cuda()
    ph = torch.from_numpy(ph0).cuda()
    del th0, ph0
    if spec["points"] != "uniform":
        plm = torch.from_numpy(wl.make_potential(spec)).cuda()
        th, ph = deflected_points(th, ph, plm, lmax)
        del plm
    fx = None if args.no_cpu else load_samples(args.workload)
    chk, sup, y_s = None, None, None
    if fx is not None:
        # the 10^4 sampled points take the oracle's deflected coordinates (within 1e-14
        # of the library's), so that both sides evaluate the same points
        idx = torch.from_numpy(fx["idx"]).cuda()
        th[idx] = torch.from_numpy(fx["theta"]).cuda()
        ph[idx] = torch.from_numpy(fx["phi"]).cuda()
        sup = wl.adjoint_support()
        y_s = wl.adjoint_check_input(ncomp, sup.size, 9)
        yfull = torch.zeros((ncomp, th.numel()), dtype=torch.float64, device="cuda")
        yfull[:, idx[torch.from_numpy(sup).cuda()]] = torch.from_numpy(y_s).cuda()
        chk = {"idx": idx, "yfull": yfull}
    alm_h = wl.make_alm(spec)
    alm = torch.from_numpy(alm_h).cuda()
    torch.cuda.synchronize()
    npts = th.numel()
    spec["npts_total"] = npts
    log("inputs ready: %d points, %.1f s" % (npts, time.time() - t0))

    forms = []
    for f in args.forms.split(","):
        p, e = f.split(":")
        forms.append((p, float(e)))
    results = {}
    for prec, eps in forms:
        key = "%s_eps%.0e" % (prec, eps)
        log("timing %s" % key)
        plan, r = time_form(gsht, torch, th, ph, alm, spec, prec, eps, args.steps, args.warmup,
                            many=args.many if prec == "f32" else 0, autotune=args.autotune,
                            check=chk,
                            sigma=args.sigma if args.sigma == "tuned" else float(args.sigma))
        results[key] = r
        log("%s: %.2f ms/step (synthesis %.2f, adjoint %.2f; plan %.2f s)" %
            (key, 1e3 * r["s_per_step"], r["synth_ms"], r["adjoint_ms"], r["plan_s"]))
        plan.close()
        del plan
        torch.cuda.empty_cache()

    head_key = HEADLINE if HEADLINE in results else next(iter(results))
    head = results[head_key]
    # roofline of the main kernels of the headline form; the dominant one (longest
    # stage) is the line's roofline
    roofs = {}
    for stage in STAGE_SOURCES:
        e = roofline_entry(stage, head_key, head, spec, npts, args.workload)
        if e is not None:
            roofs[stage] = e
    dom = max(roofs, key=lambda s: roofs[s]["avg_launch_ms"])
    roof = dict(roofs[dom])
    roof["form"] = head_key
    roof["others"] = {s: {"frac": v["frac"], "bound": v["bound"], "avg_launch_ms": v["avg_launch_ms"],
                          "traffic": v["traffic"]}
                      for s, v in roofs.items() if s != dom}
    f32 = results.get("f32_eps1e-05")
    out = {
        "metric": METRIC,
        "value": head["s_per_step"],
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * head["s_per_step"],
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if head_key.startswith("f64") else "f32 (FFT/NUFFT), f64 Legendre",
        "data": "synthetic",
        "config": {"workload": "%s: spin %d, lmax=mmax=%d, %d points (%s), %s"
                               % (args.workload, spin, lmax, npts, point_desc(spec),
                                  head_key.replace("_", " ")),
                   "npts": npts, "lmax": lmax, "mmax": mmax, "spin": spin},
        "f32_eps1e-5_s": f32["s_per_step"] if f32 else None,
        "forms": {k: {"s_per_step": v["s_per_step"], "synth_ms": v["synth_ms"],
                      "adjoint_ms": v["adjoint_ms"], "plan_s": v["plan_s"],
                      "sigma": v["info"]["sigma"],
                      "w": v["info"]["w"], "n1": v["info"]["n1"], "n2": v["info"]["n2"],
                      "column_mode": v["info"]["column_mode"], "tile": v["info"]["tile1"],
                      "legendre_shapes": [v["info"]["syn_r"], v["info"]["adj_r"], v["info"]["adj_b"]],
                      "gradient_only_ms": v.get("gradient_only"),
                      "synth_many": v.get("synth_many"),
                      "adjoint_many": v.get("adjoint_many"),
                      "stage_ms": {n: (t / c if c else None) for n, (t, c) in v["stages"].items()}}
                  for k, v in results.items()},
        "roofline": roof,
    }
    out["spreading"] = {}
    for k, v in results.items():
        e = roofline_entry("spread", k, v, spec, npts, args.workload)
        if e is not None:
            # patch word updates of point-by-point spreading (w^2 cells per point; FP64
            # complex cells are two words, FP32 complex cells one packed word); FP64
            # couples of neighbouring points issue fewer LDS atomics than this
            w = v["info"]["w"]
            words = ncomp if k.startswith("f64") else 1
            upd = npts * w * w * words
            e["patch_words_point_by_point"] = upd
            e["patch_word_rate_g_per_s"] = upd / (e["avg_launch_ms"] / 1e3) / 1e9
            out["spreading"][k] = e
    if "f64_eps1e-05" in results and f32:
        out["speedup_f32_vs_f64_eps1e-5"] = results["f64_eps1e-05"]["s_per_step"] / f32["s_per_step"]
        sm, am_ = f32.get("synth_many"), f32.get("adjoint_many")
        if sm and am_ and sm.get("legendre") == "mfma":
            # per map: FP32 form with the matrix-core Legendre step (16-map groups) against
            # the plain FP64 form, synthesis + adjoint
            out["speedup_f32_mfma_many_vs_f64_eps1e-5"] = (
                results["f64_eps1e-05"]["s_per_step"] * 1e3
                / (sm["synth_ms_per_map"] + am_["adjoint_ms_per_map"]))
    del th, ph, alm
    if chk is not None:
        del chk
    torch.cuda.empty_cache()
    if not args.no_batch:
        log("batched uneven workload")
        out["batched"] = batched(gsht, torch, max(1, args.steps // 2), 1)
        torch.cuda.empty_cache()
    if fx is not None:
        cb, err = accuracy_and_cpu_baseline(spec, alm_h, fx, sup, y_s, results, args.cpu_sample)
        out["cpu_baseline"] = cb
        out["eps_eff_on_sample"] = err
    if not args.no_cpu_nufft:
        out["cpu_nufft_baseline"] = cpu_nufft_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
