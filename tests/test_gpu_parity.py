"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

* Legendre stage (exact up to rounding): F[col][j] on the doubled meridian vs the
  oracle's ring synthesis plus the doubling rule of Sect. 3; its adjoint vs the
  oracle's ring adjoint after the undoubling rule.
* Bin sort: bit-exact vs a stable argsort of the oracle's tile keys.
* End to end: synthesis and adjoint within the requested epsilon (relative L2,
  the effective accuracy of Sect. 4), both precisions, spins 0..3, ragged sizes,
  poles, phi wrap-around, mmax < lmax, empty point sets.
* Adjointness of the GPU pair in FP64.
"""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
from lensed_points import deflect_small
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


def ring_thetas(ntheta):
    return np.pi * np.arange(ntheta) / (ntheta - 1)


def doubled_reference(alm, lmax, mmax, spin, ntheta):
    th = ring_thetas(ntheta)
    F = oracle.ring_synth(alm, lmax, mmax, spin, th)       # [2mmax+1][ntheta]
    nd = 2 * ntheta - 2
    ms = np.arange(-mmax, mmax + 1)
    out = np.zeros((2 * mmax + 1, nd), complex)
    out[:, :ntheta] = F
    sign = (-1.0) ** ((spin + ms) % 2)
    for j in range(1, ntheta - 1):
        out[:, nd - j] = sign * F[:, j]                       # doubling rule (Sect. 3)
    if spin == 0:
        out = out[mmax:]                                       # columns m >= 0
    return out


def rel_l2(a, b):
    return float(np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel()) /
                 max(np.linalg.norm(np.asarray(b).ravel()), 1e-300))


LEG_CASES = [
    # lmax, mmax, spin, ntheta
    (0, 0, 0, 2),
    (1, 1, 1, 3),
    (7, 5, 0, 9),
    (40, 40, 0, 42),
    (40, 33, 2, 43),
    (63, 63, 3, 65),
    (130, 100, 2, 140),
    (200, 200, 0, 203),
    (300, 300, 2, 302),
]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("lmax,mmax,spin,ntheta", LEG_CASES)
def test_legendre_stage_matches_oracle(G, lmax, mmax, spin, ntheta, prec):
    say("legendre stage", lmax, mmax, spin, ntheta, prec)
    rng = np.random.default_rng(lmax * 7 + spin)
    a = wl.gaussian_alm(lmax, mmax, spin, rng, cl=np.ones(lmax + 1))
    ref = doubled_reference(a, lmax, mmax, spin, ntheta)
    cdt = torch.complex128 if prec == "f64" else torch.complex64
    F = G.legendre_rings(dev(a).to(cdt), lmax, mmax, spin, ntheta, prec).cpu().numpy()
    tol = 1e-12 if prec == "f64" else 3e-7
    assert rel_l2(F, ref) < tol, rel_l2(F, ref)


@pytest.mark.parametrize("lmax,mmax,spin,ntheta", LEG_CASES)
def test_legendre_adjoint_stage_matches_oracle(G, lmax, mmax, spin, ntheta):
    say("legendre adjoint stage", lmax, mmax, spin, ntheta)
    rng = np.random.default_rng(100 + lmax + spin)
    nd = 2 * ntheta - 2
    ncol = mmax + 1 if spin == 0 else 2 * mmax + 1
    F = rng.standard_normal((ncol, nd)) + 1j * rng.standard_normal((ncol, nd))
    # undoubling rule (Sect. 3): interior rings add the mirrored row with (-1)^(s+m)
    ms = np.arange(0, mmax + 1) if spin == 0 else np.arange(-mmax, mmax + 1)
    sign = (-1.0) ** ((spin + ms) % 2)
    H = F[:, :ntheta].copy()
    for j in range(1, ntheta - 1):
        H[:, j] += sign * F[:, nd - j]
    Hfull = np.zeros((2 * mmax + 1, ntheta), complex)
    if spin == 0:
        Hfull[mmax:] = H
    else:
        Hfull[:] = H
    ref = oracle.ring_adjoint(Hfull, lmax, mmax, spin, ring_thetas(ntheta))
    got = G.legendre_rings_adjoint(dev(F), lmax, mmax, spin, ntheta, "f64").cpu().numpy()
    assert rel_l2(got, ref) < 1e-12, rel_l2(got, ref)
    # l < spin entries and Im of m = 0 are exactly zero
    if spin > 0:
        for l in range(min(spin, lmax + 1)):
            assert np.all(got[:, oracle.alm_index(l, 0, lmax)] == 0)
    assert np.all(got[:, :lmax + 1].imag == 0)


@pytest.mark.parametrize("syn_r,adj_r,adj_b", [(1, 1, 8), (2, 2, 8), (4, 2, 4), (1, 4, 4),
                                               (2, 3, 8), (4, 4, 8), (2, 3, 4)])
@pytest.mark.parametrize("lmax,mmax,spin,ntheta", [(300, 300, 2, 302), (200, 200, 0, 203),
                                                   (130, 100, 2, 520), (161, 161, 1, 1100)])
def test_legendre_launch_shapes(G, monkeypatch, syn_r, adj_r, adj_b, lmax, mmax, spin, ntheta):
    """Every supported launch shape (ring pairs per lane, degrees per adjoint block)
    of both Legendre kernels against the oracle; ntheta = 520 spans several chunks
    and a ragged last one for every shape, ntheta = 1100 many chunks per column."""
    say("legendre shapes", syn_r, adj_r, adj_b, lmax, mmax, spin, ntheta)
    monkeypatch.setenv("GSHT_SYN_R", str(syn_r))
    monkeypatch.setenv("GSHT_ADJ_R", str(adj_r))
    monkeypatch.setenv("GSHT_ADJ_B", str(adj_b))
    rng = np.random.default_rng(lmax + 13 * spin)
    a = wl.gaussian_alm(lmax, mmax, spin, rng, cl=np.ones(lmax + 1))
    ref = doubled_reference(a, lmax, mmax, spin, ntheta)
    F = G.legendre_rings(dev(a), lmax, mmax, spin, ntheta, "f64").cpu().numpy()
    assert rel_l2(F, ref) < 1e-12, rel_l2(F, ref)
    # adjoint stage on the same doubled field, against the oracle after undoubling
    ahf = G.legendre_rings_adjoint(dev(F), lmax, mmax, spin, ntheta, "f64").cpu().numpy()
    nd = 2 * ntheta - 2
    ms = np.arange(0, mmax + 1) if spin == 0 else np.arange(-mmax, mmax + 1)
    sign = (-1.0) ** ((spin + ms) % 2)
    H = F[:, :ntheta].copy()
    for j in range(1, ntheta - 1):
        H[:, j] += sign * F[:, nd - j]
    Hfull = np.zeros((2 * mmax + 1, ntheta), complex)
    if spin == 0:
        Hfull[mmax:] = H
    else:
        Hfull[:] = H
    ref_a = oracle.ring_adjoint(Hfull, lmax, mmax, spin, ring_thetas(ntheta))
    assert rel_l2(ahf, ref_a) < 1e-12, rel_l2(ahf, ref_a)


def make_case(kind, n, seed):
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        return wl.uniform_sphere(n, rng)
    if kind == "poles":
        th, ph = wl.uniform_sphere(n, rng)
        th[: n // 4] = 0.0
        th[n // 4: n // 2] = np.pi
        th[n // 2: 3 * n // 4] = rng.uniform(0, 1e-6, n // 4)
        return th, ph
    if kind == "wrap":
        th, ph = wl.uniform_sphere(n, rng)
        ph[: n // 3] = 2 * np.pi - rng.uniform(0, 1e-9, n // 3)
        ph[n // 3: 2 * n // 3] = rng.uniform(-20.0, 20.0, n - n // 3 - (n - 2 * n // 3))
        return th, ph
    if kind == "gl":
        nr = max(4, int(math.sqrt(n / 2)))
        th, ph, _ = wl.gl_grid(nr, 2 * nr + 1)
        return deflect_small(th, ph, 48, seed)
    raise ValueError(kind)


E2E = [
    # lmax, mmax, spin, npts, kind, prec, eps
    (127, 127, 0, 20000, "uniform", "f64", 1e-10),
    (127, 127, 0, 20000, "uniform", "f32", 1e-5),
    (64, 50, 2, 5000, "poles", "f64", 1e-10),
    (64, 64, 2, 5000, "wrap", "f64", 1e-12),
    (96, 96, 1, 7000, "gl", "f64", 1e-8),
    (80, 80, 3, 4000, "uniform", "f32", 1e-5),
    (33, 20, 2, 3001, "uniform", "f32", 1e-3),
    (200, 150, 0, 9000, "gl", "f64", 1e-13),
    (5, 5, 0, 1000, "uniform", "f64", 1e-10),
    (2, 2, 2, 700, "poles", "f64", 1e-10),
]


@pytest.mark.parametrize("lmax,mmax,spin,npts,kind,prec,eps", E2E)
def test_synthesis_within_epsilon(G, lmax, mmax, spin, npts, kind, prec, eps):
    say("synth", lmax, mmax, spin, npts, kind, prec, eps)
    th, ph = make_case(kind, npts, 7 + lmax)
    rng = np.random.default_rng(3 + spin)
    a = wl.gaussian_alm(lmax, mmax, spin, rng)
    ref = oracle.synth(a, lmax, mmax, spin, th, ph)
    cdt = torch.complex128 if prec == "f64" else torch.complex64
    got = G.synth_general(dev(a).to(cdt), dev(th), dev(ph), lmax, mmax, spin, eps, prec)
    got = got.cpu().numpy().astype(np.float64)
    err = oracle.eps_eff(got, ref)
    say("  eps_eff", err)
    assert err <= eps, err


@pytest.mark.parametrize("lmax,mmax,spin,npts,kind,prec,eps", E2E)
def test_adjoint_within_epsilon(G, lmax, mmax, spin, npts, kind, prec, eps):
    say("adjoint", lmax, mmax, spin, npts, kind, prec, eps)
    th, ph = make_case(kind, npts, 11 + lmax)
    npts = th.size
    rng = np.random.default_rng(5 + spin)
    y = rng.standard_normal((oracle.ncomp(spin), npts))
    ref = oracle.adjoint(y, lmax, mmax, spin, th, ph)
    rdt = torch.float64 if prec == "f64" else torch.float32
    got = G.adjoint_synth_general(dev(y).to(rdt), dev(th), dev(ph), lmax, mmax, spin, eps, prec)
    got = got.cpu().numpy().astype(np.complex128)
    w = np.sqrt(oracle.alm_weights(lmax, mmax))[None, :]
    err = oracle.eps_eff(got * w, ref * w)
    say("  eps_eff", err)
    assert err <= eps, err
    assert np.all(got[:, :lmax + 1].imag == 0)


@pytest.mark.parametrize("spin", [0, 2])
def test_gpu_pair_is_adjoint(G, spin):
    lmax, mmax, npts = 150, 140, 30000
    rng = np.random.default_rng(50 + spin)
    th, ph = wl.uniform_sphere(npts, rng)
    x = wl.gaussian_alm(lmax, mmax, spin, rng, cl=np.ones(lmax + 1))
    y = rng.standard_normal((oracle.ncomp(spin), npts))
    plan = G.Plan(dev(th), dev(ph), lmax, mmax, spin, 1e-10, "f64")
    ax = plan.synth(dev(x)).cpu().numpy()
    ahy = plan.adjoint(dev(y)).cpu().numpy()
    lhs = float(np.sum(y * ax))
    rhs = oracle.alm_inner(x, ahy, lmax, mmax)
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(y) * np.linalg.norm(ax), (lhs, rhs)


@pytest.mark.parametrize("cells", [True, False])
@pytest.mark.parametrize("kind,npts", [("uniform", 50000), ("gl", 40000), ("poles", 3000),
                                       ("wrap", 20001)])
def test_binsort_bit_exact(G, monkeypatch, kind, npts, cells):
    """Sorted by tile and first kernel cell (the default), or by tile alone."""
    say("binsort", kind, npts, cells)
    if not cells:
        monkeypatch.setenv("GSHT_CELL_SORT", "0")
    th, ph = make_case(kind, npts, 99)
    plan = G.Plan(dev(th), dev(ph), 127, 127, 2, 1e-5, "f32")
    inf = plan.info()
    perm, start = plan.sort()
    assert inf["cell_sort"] == (1 if cells else 0)
    keys = oracle.bin_keys(th, ph, inf["n1"], inf["n2"], inf["w"], inf["a_min"], inf["tile1"],
                           inf["tile2"], inf["ntile2"], cells=cells)
    ntiles = inf["ntile1"] * inf["ntile2"]
    ref_perm, ref_start = oracle.binsort(keys, ntiles, inf["tile1"] * inf["tile2"] if cells else 1)
    assert np.array_equal(perm.cpu().numpy(), ref_perm)
    assert np.array_equal(start.cpu().numpy(), ref_start)


def test_empty_point_set(G):
    th = torch.zeros(0, dtype=torch.float64, device="cuda")
    a = torch.zeros((2, oracle.nalm(16, 16)), dtype=torch.complex128, device="cuda")
    m = G.synth_general(a, th, th.clone(), 16, 16, 2, 1e-10, "f64")
    assert m.shape == (2, 0)
    b = G.adjoint_synth_general(m, th, th.clone(), 16, 16, 2, 1e-10, "f64")
    assert torch.all(b == 0)


def test_invalid_theta_rejected(G):
    th = torch.tensor([0.1, 3.5, 1.0], dtype=torch.float64, device="cuda")
    ph = torch.zeros(3, dtype=torch.float64, device="cuda")
    with pytest.raises(G.GshtError) as ei:
        G.Plan(th, ph, 8, 8, 0, 1e-10, "f64")
    assert ei.value.code == G.GSHT_EINVAL
    ph2 = torch.tensor([0.0, float("nan"), 1.0], dtype=torch.float64, device="cuda")
    th2 = torch.tensor([0.1, 0.2, 1.0], dtype=torch.float64, device="cuda")
    with pytest.raises(G.GshtError):
        G.Plan(th2, ph2, 8, 8, 0, 1e-10, "f64")


def test_plan_reuse_and_repeatability(G):
    """Same plan, several maps: results identical run to run (forward is atomic-free)."""
    lmax, spin = 100, 2
    rng = np.random.default_rng(1)
    th, ph = wl.uniform_sphere(8000, rng)
    plan = G.Plan(dev(th), dev(ph), lmax, lmax, spin, 1e-10, "f64")
    for rep in range(3):
        a = wl.gaussian_alm(lmax, lmax, spin, np.random.default_rng(rep))
        m1 = plan.synth(dev(a))
        m2 = plan.synth(dev(a))
        assert torch.equal(m1, m2)
        ref = oracle.synth(a, lmax, lmax, spin, th[:500], ph[:500])
        assert oracle.eps_eff(m1[:, :500].cpu().numpy(), ref) < 1e-10


@pytest.mark.parametrize("lmax,spin,prec,eps", [(130, 2, "f64", 1e-11), (130, 0, "f32", 1e-5),
                                                (269, 1, "f64", 1e-9), (47, 3, "f32", 1e-4),
                                                (512, 2, "f32", 1e-5), (512, 0, "f64", 1e-10)])
def test_column_stage_modes_agree(G, monkeypatch, lmax, spin, prec, eps):
    """The fused per-column FFT stage (modes 2 and 1) against the separate library
    FFTs (mode 0) and against the oracle, synthesis and adjoint.  lmax = 512 gives
    n1 = 4 lmax, where the split theta transform of mode 2 folds two frequencies
    onto one residue."""
    say("column modes", lmax, spin, prec, eps)
    rng = np.random.default_rng(400 + lmax)
    th, ph = wl.uniform_sphere(6000, rng)
    a = wl.gaussian_alm(lmax, lmax, spin, rng)
    y = rng.standard_normal((oracle.ncomp(spin), th.size))
    cdt = torch.complex128 if prec == "f64" else torch.complex64
    rdt = torch.float64 if prec == "f64" else torch.float32
    ref_m = oracle.synth(a, lmax, lmax, spin, th, ph)
    ref_a = oracle.adjoint(y, lmax, lmax, spin, th, ph)
    w = np.sqrt(oracle.alm_weights(lmax, lmax))[None, :]
    outs = {}
    for mode in (0, 1, 2):
        monkeypatch.setenv("GSHT_COLUMN_MODE", str(mode))
        plan = G.Plan(dev(th), dev(ph), lmax, lmax, spin, eps, prec)
        assert plan.info()["column_mode"] == mode
        m = plan.synth(dev(a).to(cdt)).cpu().numpy().astype(np.float64)
        b = plan.adjoint(dev(y).to(rdt)).cpu().numpy().astype(np.complex128)
        plan.close()
        em, ea = oracle.eps_eff(m, ref_m), oracle.eps_eff(b * w, ref_a * w)
        say("  mode", mode, "synth", em, "adjoint", ea)
        assert em <= eps and ea <= eps, (mode, em, ea)
        outs[mode] = (m, b)
    tol = 1e-12 if prec == "f64" else 2e-6
    for mode in (1, 2):
        assert rel_l2(outs[mode][0], outs[0][0]) <= tol
        assert rel_l2(outs[mode][1] * w, outs[0][1] * w) <= tol


@pytest.mark.parametrize("lmax,mmax,spin,npts,prec,eps,colors", [
    (127, 127, 2, 30000, "f64", 1e-10, 4),   # even number of tile columns
    (40, 23, 2, 20000, "f64", 1e-10, 6),     # n2 = 96: three tile columns (odd)
    (30, 30, 0, 60000, "f64", 1e-9, 4),      # thousands of points per tile: many chunks
    (60, 60, 2, 40000, "f32", 1e-5, 4),
])
def test_spreading_by_tile_colour(G, monkeypatch, lmax, mmax, spin, npts, prec, eps, colors):
    """Adjoint with the colour-ordered, atomic-free spreading flush against the
    per-chunk atomic flush and against the oracle."""
    say("spread colours", lmax, mmax, spin, npts, prec)
    rng = np.random.default_rng(900 + lmax)
    th, ph = wl.uniform_sphere(npts, rng)
    y = rng.standard_normal((oracle.ncomp(spin), npts))
    rdt = torch.float64 if prec == "f64" else torch.float32
    w = np.sqrt(oracle.alm_weights(lmax, mmax))[None, :]
    outs = []
    for env in (None, "0"):
        if env is None:
            monkeypatch.delenv("GSHT_SPREAD_COLORS", raising=False)
        else:
            monkeypatch.setenv("GSHT_SPREAD_COLORS", env)
        plan = G.Plan(dev(th), dev(ph), lmax, mmax, spin, eps, prec)
        assert plan.info()["spread_colors"] == (colors if env is None else 0)
        outs.append(plan.adjoint(dev(y).to(rdt)).cpu().numpy().astype(np.complex128))
        plan.close()
    tol = 1e-12 if prec == "f64" else 2e-6
    assert rel_l2(outs[0] * w, outs[1] * w) <= tol
    ref = oracle.adjoint(y, lmax, mmax, spin, th, ph)
    assert oracle.eps_eff(outs[0] * w, ref * w) <= eps


@pytest.mark.parametrize("spin,eps", [(2, 1e-10), (0, 1e-12)])
def test_spreading_mixed_tile_densities(G, monkeypatch, spin, eps):
    """FP64 colour-ordered spreading on one point set with sparse tiles (at most two
    chunks: spread as a whole with one value bound) and dense ones (a 20000-point cap
    of 0.05 x 0.05 rad near theta = 1, phi = 2, a few tiles of dozens of chunks: chunk
    by chunk), against the per-chunk atomic flush and against the oracle."""
    say("spread mixed densities", spin, eps)
    lmax = 127
    rng = np.random.default_rng(1700 + spin)
    th1, ph1 = wl.uniform_sphere(8000, rng)
    th2 = 1.0 + 0.05 * rng.random(20000)
    ph2 = 2.0 + 0.05 * rng.random(20000)
    th, ph = np.concatenate([th1, th2]), np.concatenate([ph1, ph2])
    y = rng.standard_normal((oracle.ncomp(spin), th.size))
    w = np.sqrt(oracle.alm_weights(lmax, lmax))[None, :]
    outs = []
    for env in (None, "0"):
        if env is None:
            monkeypatch.delenv("GSHT_SPREAD_COLORS", raising=False)
        else:
            monkeypatch.setenv("GSHT_SPREAD_COLORS", env)
        plan = G.Plan(dev(th), dev(ph), lmax, lmax, spin, eps, "f64")
        assert (plan.info()["spread_colors"] > 0) == (env is None)
        outs.append(plan.adjoint(dev(y)).cpu().numpy())
        plan.close()
    d = rel_l2(outs[0] * w, outs[1] * w)
    say("  colour vs atomic: %.2e" % d)
    assert d <= 1e-12
    ref = oracle.adjoint(y, lmax, lmax, spin, th, ph)
    assert oracle.eps_eff(outs[0] * w, ref * w) <= eps


@pytest.mark.parametrize("lmax,mmax,spin,npts,eps", [
    (130, 130, 2, 30000, 1e-10), (200, 150, 0, 20000, 1e-10), (64, 64, 1, 9000, 1e-8)])
def test_fp64_spreading_fast_and_exact_forms(G, monkeypatch, lmax, mmax, spin, npts, eps):
    """FP64 spreading in its two fixed-point forms (step 2^-50 and 2^-63 of a chunk's
    value bound): the adjoints agree far below epsilon and both meet it against the
    oracle."""
    say("spread quantisation", lmax, mmax, spin, npts, eps)
    rng = np.random.default_rng(950 + lmax)
    th, ph = wl.uniform_sphere(npts, rng)
    y = rng.standard_normal((oracle.ncomp(spin), npts))
    w = np.sqrt(oracle.alm_weights(lmax, mmax))[None, :]
    outs = []
    for form in ("exact", "fast"):
        monkeypatch.setenv("GSHT_SPREAD_QUANT", form)
        plan = G.Plan(dev(th), dev(ph), lmax, mmax, spin, eps, "f64")
        outs.append(plan.adjoint(dev(y)).cpu().numpy())
        plan.close()
    d = rel_l2(outs[1] * w, outs[0] * w)
    say("  fast vs exact: %.2e" % d)
    assert d <= 1e-12
    ref = oracle.adjoint(y, lmax, mmax, spin, th, ph)
    for o in outs:
        assert oracle.eps_eff(o * w, ref * w) <= eps


@pytest.mark.parametrize("lmax,mmax,spin,npts,prec,eps", [
    (130, 130, 2, 30000, "f64", 1e-10), (96, 80, 0, 20000, "f64", 1e-12),
    (200, 200, 2, 40000, "f32", 1e-5)])
def test_point_order_within_tiles(G, monkeypatch, lmax, mmax, spin, npts, prec, eps):
    """Points in cell order (FP64 spreading pairs neighbours) and in tile order (few
    pairs) give the same transforms up to rounding, both within epsilon of the oracle,
    on thin Gauss-Legendre rings (dense rows, many couples)."""
    say("point order", lmax, mmax, spin, npts, prec, eps)
    rng = np.random.default_rng(970 + lmax)
    nring = max(8, int(np.sqrt(npts / 2)))
    th, ph = wl.gl_grid(nring, 2 * nring)[:2]
    th, ph = th[:npts], ph[:npts]
    th, ph = deflect_small(th, ph, 24, 5)
    y = rng.standard_normal((oracle.ncomp(spin), th.size))
    a = wl.gaussian_alm(lmax, mmax, spin, rng)
    rdt = torch.float64 if prec == "f64" else torch.float32
    cdt = torch.complex128 if prec == "f64" else torch.complex64
    w = np.sqrt(oracle.alm_weights(lmax, mmax))[None, :]
    outs = []
    for env in (None, "0"):
        if env is None:
            monkeypatch.delenv("GSHT_CELL_SORT", raising=False)
        else:
            monkeypatch.setenv("GSHT_CELL_SORT", env)
        plan = G.Plan(dev(th), dev(ph), lmax, mmax, spin, eps, prec)
        assert plan.info()["cell_sort"] == (1 if env is None else 0)
        outs.append((plan.synth(dev(a).to(cdt)).cpu().numpy().astype(np.float64),
                     plan.adjoint(dev(y).to(rdt)).cpu().numpy().astype(np.complex128)))
        plan.close()
    tol = 1e-12 if prec == "f64" else 2e-6
    assert rel_l2(outs[0][0], outs[1][0]) <= tol
    assert rel_l2(outs[0][1] * w, outs[1][1] * w) <= tol
    ref_a = oracle.adjoint(y, lmax, mmax, spin, th, ph)
    idx = rng.choice(th.size, 500, replace=False)
    ref_s = oracle.synth(a, lmax, mmax, spin, th[idx], ph[idx])
    for s_out, a_out in outs:
        assert oracle.eps_eff(a_out * w, ref_a * w) <= eps
        assert oracle.eps_eff(s_out[:, idx], ref_s) <= eps


@pytest.mark.parametrize("lmax,mmax,spin,prec", [(130, 130, 2, "f64"), (512, 400, 1, "f32"),
                                                 (47, 47, 0, "f32")])
def test_lds_padding_is_bitwise_neutral(G, monkeypatch, lmax, mmax, spin, prec):
    """The padding slots of the in-LDS transforms move values, never the arithmetic:
    every padding (none, one slot per 4, per 32 elements) gives identical bits, for
    the fused column stage."""
    say("lds padding", lmax, mmax, spin, prec)
    rng = np.random.default_rng(600 + lmax)
    th, ph = wl.uniform_sphere(5000, rng)
    a = wl.gaussian_alm(lmax, mmax, spin, rng)
    y = rng.standard_normal((oracle.ncomp(spin), th.size))
    cdt = torch.complex128 if prec == "f64" else torch.complex64
    rdt = torch.float64 if prec == "f64" else torch.float32
    monkeypatch.setenv("GSHT_COLUMN_MODE", "2")
    outs = []
    for pad in ("0", "2", "5"):
        monkeypatch.setenv("GSHT_LDS_PAD", pad)
        plan = G.Plan(dev(th), dev(ph), lmax, mmax, spin, 1e-5 if prec == "f32" else 1e-10, prec)
        outs.append((plan.synth(dev(a).to(cdt)), plan.adjoint(dev(y).to(rdt))))
        plan.close()
    for m, b in outs[1:]:
        assert torch.equal(m, outs[0][0]) and torch.equal(b, outs[0][1])
    monkeypatch.setenv("GSHT_LDS_PAD", "1")
    with pytest.raises(G.GshtError):
        G.Plan(dev(th), dev(ph), lmax, mmax, spin, 1e-5, prec)


@pytest.mark.parametrize("spin,eps", [(2, 1e-10), (0, 1e-5), (1, 1e-13)])
def test_interior_tap_polynomials_match_exact_weights(G, monkeypatch, spin, eps):
    """FP64 interpolation with the host-fitted interior-tap polynomials against the
    exact kernel formula (GSHT_ES_POLY=0): the weights differ by at most ~5e-15, so
    the maps agree far below epsilon; both stay within epsilon of the oracle."""
    say("es poly", spin, eps)
    lmax = 160
    rng = np.random.default_rng(800 + spin)
    th, ph = wl.uniform_sphere(30000, rng)
    a = wl.gaussian_alm(lmax, lmax, spin, rng)
    outs = []
    for flag in ("1", "0"):
        monkeypatch.setenv("GSHT_ES_POLY", flag)
        plan = G.Plan(dev(th), dev(ph), lmax, lmax, spin, eps, "f64")
        outs.append(plan.synth(dev(a)).cpu().numpy())
        plan.close()
    assert rel_l2(outs[0], outs[1]) <= 1e-13
    ref = oracle.synth(a, lmax, lmax, spin, th[:3000], ph[:3000])
    assert oracle.eps_eff(outs[0][:, :3000], ref) <= eps
