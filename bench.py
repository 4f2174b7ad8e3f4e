"""Benchmark: general spin-2 synthesis + adjoint at lmax 4096 on ~48M deflected points.

One step = one synthesis (a_lm -> map) plus one adjoint (map -> a_lm) through the
C ABI (plan API, geometry reused as in the paper's lensing use), with all inputs
resident in HBM.  Forms timed:

  * FP32 form, epsilon = 1e-5   (headline ``value``: seconds per step)
  * FP64 form, epsilon = 1e-5   (for the FP32-vs-FP64 speed-up at equal accuracy)
  * FP64 form, epsilon = 1e-10

Workload: spin 2, lmax = mmax = 4096, Gaussian E/B a_lm, points of a 6144-ring
longitude-thinned Gauss-Legendre grid displaced by a 2.5 arcmin rms deflection
field (about 4.8e7 points; the "~5e7 pixel" intermediate grid of the paper's
Sect. 4 benchmark).  Synthetic data, generated with fixed seeds.

Also reported: synthesis and adjoint times of each form (HIP events), the dominant
kernel's achieved fraction of the MI355X FP64 vector peak (Legendre recurrence),
the spreading kernel's HBM fraction and LDS atomic rate, per-stage times from HIP
events inside the library, and the FP64 CPU oracle timed on a bounded sample of
points on the host cores, with each form's effective accuracy against it
(synthesis on the sampled points, adjoint of an input supported on them).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_legendre_synth_pollens_thin6144.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2304_10431_amd", "csrc", f)
                  for f in ("legendre_kernels.hip", "legendre_device.hpp")]


def measured_traffic(workload):
    """HBM bytes per launch of the Legendre synthesis from the committed counter
    runs, or None if they were taken on another workload or on a different version
    of the kernel source."""
    import hashlib
    try:
        rec = json.load(open(TRAFFIC_FILE))
        sha = hashlib.sha256(b"".join(open(f, "rb").read() for f in KERNEL_SOURCES)).hexdigest()
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256") != sha or rec.get("workload", "").split()[0] != workload:
        return None
    return rec.get("bytes_per_launch")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def legendre_flops(lmax, mmax, spin, npairs):
    """Algorithmic FP64 flops of one Legendre launch: per (l, m, ring pair) unit,
    8 flop for spin 0 (2 FMA recurrence + 2 FMA accumulation) and 24 flop for
    spin > 0 (2 recurrences + 4 complex-by-real accumulations), over
    max(m, s) <= l <= lmax, 0 <= m <= mmax."""
    units = 0
    for m in range(mmax + 1):
        l0 = max(m, spin)
        if l0 <= lmax:
            units += lmax - l0 + 1
    per = 8 if spin == 0 else 24
    return per * units * npairs


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
    plan.set_profiling(True)
    # the library launches on torch's current stream, so events recorded there
    # bracket exactly one synthesis and one adjoint
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
    stages = plan.stage_times()
    plan.set_profiling(False)
    info = plan.info()
    r = dict(s_per_step=dt, synth_ms=syn_ms, adjoint_ms=adj_ms, plan_s=t_plan, stages=stages,
             info=info)
    if spec["spin"] > 0:
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
        m = plan.synth(a, out=m)
    if many > 1:
        # several maps on the same plan: FP32 plans take groups of 8..16 maps through the
        # matrix-core Legendre step, smaller groups (and FP64) through the FP64 group kernel
        am = a.unsqueeze(0).repeat(many, 1, 1).contiguous()
        am *= torch.linspace(0.5, 2.0, many, device=am.device).to(am.dtype)[:, None, None]
        mm = plan.synth_many(am)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            plan.synth_many(am, out=mm)
        e1.record()
        torch.cuda.synchronize()
        r["synth_many"] = {"maps": many, "synth_ms_per_map": e0.elapsed_time(e1) / steps / many,
                           "legendre": "mfma" if (prec == "f32" and many >= 8) else "fp64"}
        plan.set_profiling(True)
        plan.synth_many(am, out=mm)
        st = plan.stage_times()
        plan.set_profiling(False)
        r["synth_many"]["legendre_ms_per_map"] = st["legendre_synth"][0] / many
        r["synth_many"]["prep_ms_per_map"] = st["prep_alm"][0] / many
        # accuracy of the last map against its own single-map synthesis
        one = plan.synth(am[many - 1].contiguous())
        r["synth_many"]["eps_vs_single"] = float(torch.linalg.norm((mm[many - 1] - one).double())
                                                 / torch.linalg.norm(one.double()))
        del am, one
        fac = torch.linspace(0.5, 2.0, many, device=mm.device)
        if check is not None:
            # the last map's values on the oracle's sample points, undone the scaling
            r["many_check"] = {"synth": (mm[many - 1][:, check["idx"]] / fac[-1]).double().cpu().numpy()}
        # adjoint of the same maps (matrix-core Legendre step for 8..16 FP32 maps)
        bm = plan.adjoint_many(mm)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(steps):
            plan.adjoint_many(mm, out=bm)
        e1.record()
        torch.cuda.synchronize()
        r["adjoint_many"] = {"maps": many, "adjoint_ms_per_map": e0.elapsed_time(e1) / steps / many,
                             "legendre": "mfma" if (prec == "f32" and many >= 8) else "fp64"}
        plan.set_profiling(True)
        plan.adjoint_many(mm, out=bm)
        st = plan.stage_times()
        plan.set_profiling(False)
        r["adjoint_many"]["legendre_ms_per_map"] = st["legendre_adj"][0] / many
        r["adjoint_many"]["prep_ms_per_map"] = st["prep_alm"][0] / many
        one = plan.adjoint(mm[many - 1].contiguous())
        r["adjoint_many"]["eps_vs_single"] = float(
            torch.linalg.norm((bm[many - 1] - one).to(torch.complex128))
            / torch.linalg.norm(one.to(torch.complex128)))
        del bm, one
        if check is not None:
            # adjoint of scaled copies of the oracle's sampled input
            ym = (check["yfull"].to(mm.dtype).unsqueeze(0) * fac[:, None, None]).contiguous()
            bmy = plan.adjoint_many(ym)
            r["many_check"]["adjoint"] = (bmy[many - 1] / fac[-1]).to(torch.complex128).cpu().numpy()
            del ym, bmy
        del mm
    return plan, m, r


def spreading_figures(info, stages, npts, ncomp, prec):
    """Spreading (type-1 NUFFT) throughput.  Algorithmic HBM bytes per launch:
    per point its sorted FP64 (theta, phi) (16 B), its 4 B permutation entry and its
    ncomp map values; per grid cell one read and one write of the grid value (complex
    for spin > 0, real for spin 0), times the halo factor ((T + w - 1) / T)^2 of a
    tile's patch.  LDS integer atomics: w^2 taps x ncomp per point."""
    rs = 8 if prec == "f64" else 4
    w, t1, t2 = info["w"], info["tile1"], info["tile2"]
    halo = (t1 + w - 1) * (t2 + w - 1) / float(t1 * t2)
    grid = info["nrows"] * info["n2"] * ncomp * rs
    nbytes = npts * (16 + 4 + ncomp * rs) + 2 * grid * halo
    ms, cnt = stages["spread"]
    avg_s = ms / max(cnt, 1) / 1e3
    atomics = npts * w * w * ncomp
    return {"kernel": "spread", "bound": "hbm", "achieved": nbytes / avg_s / 1e9,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": nbytes / avg_s / 1e9 / HBM_PEAK_GBS,
            "bytes_per_launch": nbytes, "avg_launch_ms": avg_s * 1e3,
            "lds_atomics_per_launch": atomics, "lds_atomic_gops": atomics / avg_s / 1e9}


def sample_points(npts, nsample, ncomp):
    """The bounded sample the oracle is timed on: sorted random point indices and an
    adjoint input supported on them."""
    rng = np.random.default_rng(12345)
    idx = np.sort(rng.choice(npts, nsample, replace=False))
    y = np.random.default_rng(7).standard_normal((ncomp, nsample))
    return idx, y


def cpu_baseline(spec, th_h, ph_h, alm_h, idx, y, m_gpu_h, adj_gpu_h, many_checks=None):
    """Oracle (FP64 direct sum, all host cores) on a bounded random sample of the
    workload's points, scaled linearly to the full point count.  Also returns the
    GPU forms' effective accuracy against it: synthesis on the sampled points, and the
    adjoint of an input supported on them (w_m-weighted over a_lm)."""
    import oracle
    lmax, mmax, spin = spec["lmax"], spec["mmax"], spec["spin"]
    nsample = idx.size
    cores = len(os.sched_getaffinity(0))
    t0 = time.time()
    ref = oracle.synth(alm_h, lmax, mmax, spin, th_h[idx], ph_h[idx], nthreads=cores)
    t_syn = time.time() - t0
    t0 = time.time()
    ref_adj = oracle.adjoint(y, lmax, mmax, spin, th_h[idx], ph_h[idx], nthreads=cores)
    t_adj = time.time() - t0
    npts = th_h.size
    per_step = (t_syn + t_adj) * npts / nsample
    wts = np.sqrt(oracle.alm_weights(lmax, mmax))[None, :]
    err = {k: {"synthesis": oracle.eps_eff(v[:, idx], ref),
               "adjoint": oracle.eps_eff(wts * adj_gpu_h[k], wts * ref_adj)}
           for k, v in m_gpu_h.items()}
    for k, mc in (many_checks or {}).items():
        # several-map paths: the last map of the group against the same oracle values
        if "synth" in mc:
            err[k]["synthesis_many"] = oracle.eps_eff(mc["synth"], ref)
        if "adjoint" in mc:
            err[k]["adjoint_many"] = oracle.eps_eff(wts * mc["adjoint"], wts * ref_adj)
    return dict(value=per_step, unit="s", cores=cores, kind="oracle",
                sample="%d random points of the %d-point workload: synthesis %.1f s + adjoint "
                       "%.1f s on %d threads, scaled linearly to all points" %
                       (nsample, npts, t_syn, t_adj, cores)), err


def cpu_nufft_baseline(spec, th_h, ph_h, alm_h, eps):
    """The plain CPU NUFFT-based SHT (FP64, all host cores), one synthesis and one
    adjoint at the full workload, with its own parameter choice for eps."""
    from oracle import nufft_sht
    lmax, mmax, spin = spec["lmax"], spec["mmax"], spec["spin"]
    p = nufft_sht.default_params(lmax, mmax, eps)
    cores = len(os.sched_getaffinity(0))
    t0 = time.time()
    m = nufft_sht.synth(alm_h, lmax, mmax, spin, th_h, ph_h, nthreads=cores, **p)
    t_syn = time.time() - t0
    log("cpu nufft synthesis %.1f s" % t_syn)
    t0 = time.time()
    nufft_sht.adjoint(m, lmax, mmax, spin, th_h, ph_h, nthreads=cores, **p)
    t_adj = time.time() - t0
    log("cpu nufft adjoint %.1f s" % t_adj)
    return dict(value=t_syn + t_adj, unit="s", cores=cores, kind="oracle (plain CPU NUFFT SHT)",
                eps=eps, params=p,
                sample="whole workload, one synthesis (%.1f s) + one adjoint (%.1f s), FP64"
                       % (t_syn, t_adj))


def point_desc(spec):
    if spec["points"] == "thin":
        return ("%d-ring longitude-thinned Gauss-Legendre grid, 2.5 arcmin rms deflection"
                % spec["nring"])
    if spec["points"] == "gl":
        return ("%d x %d Gauss-Legendre grid, 2.5 arcmin rms deflection"
                % (spec["nring"], spec["nphi"]))
    return "uniform random points"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="pollens_thin6144")
    ap.add_argument("--cpu-sample", type=int, default=2048)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--autotune", action="store_true",
                    help="let each plan time the Legendre launch shapes and keep the fastest")
    ap.add_argument("--many", type=int, default=16,
                    help="maps per call for the several-map synthesis timing (FP32 form; 0: off)")
    ap.add_argument("--cpu-nufft", action="store_true",
                    help="also time the plain CPU NUFFT-based SHT on the whole workload "
                         "(FP64, eps 1e-10; minutes at lmax 2048)")
    ap.add_argument("--no-f64", action="store_true")
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

    spec = wl.WORKLOADS[args.workload]
    lmax, mmax, spin = spec["lmax"], spec["mmax"], spec["spin"]
    if args.copy_calib:
        src = torch.ones(CALIB_BYTES // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    t0 = time.time()
    log("generating %s points" % args.workload)
    if spec["points"] == "thin":
        th0, ph0 = wl.thinned_gl_grid(spec["nring"])
    elif spec["points"] == "gl":
        th0, ph0, _ = wl.gl_grid(spec["nring"], spec["nphi"])
    else:
        th0, ph0 = wl.uniform_sphere(spec["npts"], np.random.default_rng(wl.seed_for(spec["id"])))
    th = torch.from_numpy(th0).cuda()
    ph = torch.from_numpy(ph0).cuda()
    del th0, ph0
    if spec["points"] != "uniform":
        th, ph = wl.deflect(th, ph, wl.seed_for(spec["id"]) + 500)
    alm_h = wl.make_alm(spec)
    alm = torch.from_numpy(alm_h).cuda()
    torch.cuda.synchronize()
    npts = th.numel()
    log("inputs ready: %d points, %.1f s" % (npts, time.time() - t0))

    ncomp = 2 if spin else 1
    if not args.no_cpu:
        idx, ysam = sample_points(npts, args.cpu_sample, ncomp)
        yfull = torch.zeros((ncomp, npts), dtype=torch.float64, device="cuda")
        yfull[:, torch.from_numpy(idx).cuda()] = torch.from_numpy(ysam).cuda()
    adj_maps = {}
    forms = [("f32", 1e-5)]
    if not args.no_f64:
        forms += [("f64", 1e-5), ("f64", 1e-10)]
    results = {}
    maps = {}
    for prec, eps in forms:
        log("timing %s eps %.0e" % (prec, eps))
        chk = None if args.no_cpu else {"idx": torch.from_numpy(idx).cuda(), "yfull": yfull}
        plan, m, r = time_form(gsht, torch, th, ph, alm, spec, prec, eps, args.steps, args.warmup,
                               many=args.many if prec == "f32" else 0, autotune=args.autotune,
                               check=chk,
                               sigma=args.sigma if args.sigma == "tuned" else float(args.sigma))
        key = "%s_eps%.0e" % (prec, eps)
        results[key] = r
        maps[key] = m.detach().to(torch.float64).cpu().numpy()
        if not args.no_cpu:
            rdt = torch.float64 if prec == "f64" else torch.float32
            adj_maps[key] = plan.adjoint(yfull.to(rdt)).to(torch.complex128).cpu().numpy()
        log("%s: %.2f ms/step (synthesis %.2f, adjoint %.2f; plan %.2f s)" %
            (key, 1e3 * r["s_per_step"], r["synth_ms"], r["adjoint_ms"], r["plan_s"]))
        plan.close()
        del plan, m
        torch.cuda.empty_cache()

    head = results["f32_eps1e-05"]
    info = head["info"]
    st = head["stages"]
    leg_ms, leg_n = st["legendre_synth"]
    leg_avg_s = leg_ms / max(leg_n, 1) / 1e3
    flops = legendre_flops(lmax, mmax, spin, (info["ntheta"] + 1) // 2)
    achieved = flops / leg_avg_s / 1e12
    adj_ms, adj_n = st["legendre_adj"]
    adj_avg_s = adj_ms / max(adj_n, 1) / 1e3

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
        "dtype": "f32 (FFT/NUFFT), f64 Legendre",
        "data": "synthetic",
        "config": {"workload": "%s: spin %d, lmax=mmax=%d, %d points (%s), FP32 eps 1e-5"
                               % (args.workload, spin, lmax, npts, point_desc(spec)),
                   "npts": npts, "lmax": lmax, "mmax": mmax, "spin": spin},
        "forms": {k: {"s_per_step": v["s_per_step"], "synth_ms": v["synth_ms"],
                      "adjoint_ms": v["adjoint_ms"], "plan_s": v["plan_s"],
                      "sigma": v["info"]["sigma"],
                      "w": v["info"]["w"], "n1": v["info"]["n1"], "n2": v["info"]["n2"],
                      "column_mode": v["info"]["column_mode"],
                      "legendre_shapes": [v["info"]["syn_r"], v["info"]["adj_r"], v["info"]["adj_b"]],
                      "gradient_only_ms": v.get("gradient_only"),
                      "synth_many": v.get("synth_many"),
                      "adjoint_many": v.get("adjoint_many"),
                      "stage_ms": {n: (t / c if c else None) for n, (t, c) in v["stages"].items()}}
                  for k, v in results.items()},
        "roofline": {"kernel": "legendre_synth", "bound": "alu",
                     "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "traffic": measured_traffic(args.workload),
                     "flops_per_launch": flops, "avg_launch_ms": leg_avg_s * 1e3,
                     "legendre_adj_frac": flops / adj_avg_s / 1e12 / FP64_VECTOR_PEAK_TFLOPS},
    }
    out["spreading"] = {k: spreading_figures(v["info"], v["stages"], npts, ncomp, k[:3])
                        for k, v in results.items()}
    if "f64_eps1e-05" in results:
        out["speedup_f32_vs_f64_eps1e-5"] = results["f64_eps1e-05"]["s_per_step"] / head["s_per_step"]
        sm, am_ = head.get("synth_many"), head.get("adjoint_many")
        if sm and am_ and sm.get("legendre") == "mfma":
            # per map: FP32 form with the matrix-core Legendre step (16-map groups) against
            # the plain FP64 form, synthesis + adjoint
            out["speedup_f32_mfma_many_vs_f64_eps1e-5"] = (
                results["f64_eps1e-05"]["s_per_step"] * 1e3
                / (sm["synth_ms_per_map"] + am_["adjoint_ms_per_map"]))
    if "f64_eps1e-10" in results:
        out["f64_eps1e-10_s"] = results["f64_eps1e-10"]["s_per_step"]
    if not args.no_cpu:
        th_h = th.cpu().numpy()
        ph_h = ph.cpu().numpy()
        mchk = {k: v.pop("many_check") for k, v in results.items() if "many_check" in v}
        cb, err = cpu_baseline(spec, th_h, ph_h, alm_h, idx, ysam, maps, adj_maps, mchk)
        out["cpu_baseline"] = cb
        out["eps_eff_on_sample"] = err
    if args.cpu_nufft:
        out["cpu_nufft_baseline"] = cpu_nufft_baseline(spec, th.cpu().numpy(), ph.cpu().numpy(),
                                                       alm_h, 1e-10)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
