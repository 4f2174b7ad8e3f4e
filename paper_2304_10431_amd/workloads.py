"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds no spherical-harmonic, NUFFT or lensing arithmetic: it only
draws random coefficients (signal a_lm and lensing potentials) and builds the
undeflected point sets (uniform, Gauss-Legendre, thinned Gauss-Legendre).  The
GPU path and the oracle receive exactly the arrays produced here; each side
deflects the points with its own code (the library's lensing calls, or the
oracle's direct sums).

Workloads (shapes of the paper's lensing benchmarks, Sect. 4):

* ``tiny_spin0``     -- spin 0, lmax = mmax = 127, 20 000 points uniform on the sphere.
* ``tlens_l2048``    -- spin 0, lmax 2048, Gauss-Legendre 2049 x 4097 points, deflected.
* ``pollens_l4096``  -- spin 2, lmax 4096, Gauss-Legendre 4097 x 8193 points, deflected.
* ``pollens_thin6144`` -- spin 2, lmax 4096, longitude-thinned Gauss-Legendre grid with
  6144 rings (about 4.8e7 points, the "~5e7 pixel" intermediate grid of Sect. 4), deflected.

Deflection model (a stand-in for the paper's simulated lensing potential): a
Gaussian potential phi_LM with C_L proportional to L^-4 above L = 60, flat at
C_60 for 2 <= L <= 60 and zero for L < 2, band-limited at the workload's lmax, and
scaled so that the sphere average of |alpha|^2 with alpha the gradient of the
potential is (2.5 arcmin)^2.  The deflection field is the spin-1 synthesis of
sqrt(L (L + 1)) phi_LM on the undeflected points (eq. deflect) and the points move
along great circles (end of Sect. 3).
"""
from __future__ import annotations

import math

import numpy as np

ARCMIN = math.pi / (180.0 * 60.0)


def seed_for(workload_id: int, replica: int = 0) -> int:
    return 1000 * workload_id + replica


def nalm(lmax: int, mmax: int) -> int:
    return (mmax + 1) * (lmax + 1) - mmax * (mmax + 1) // 2


def gaussian_alm(lmax: int, mmax: int, spin: int, rng: np.random.Generator,
                 cl=None, cl_b_ratio: float = 0.1) -> np.ndarray:
    """Seeded Gaussian a_lm, [ncomp][nalm] complex128, m-major triangular layout.

    m > 0: Re and Im ~ N(0, C_l / 2); m = 0: real ~ N(0, C_l).  Spin 0 uses
    C_l = 1/(l+1)^2 by default.  Spin s > 0 draws G with C_l^E = 1e-2/(l+1)^2 and
    C with C_l^B = cl_b_ratio * C_l^E (a power ratio); degrees l < s are zero.
    """
    ncomp = 1 if spin == 0 else 2
    n = nalm(lmax, mmax)
    ls = np.concatenate([np.arange(m, lmax + 1) for m in range(mmax + 1)])
    ms = np.concatenate([np.full(lmax + 1 - m, m) for m in range(mmax + 1)])
    if cl is None:
        base = (1.0 if spin == 0 else 1e-2) / (ls + 1.0) ** 2
    else:
        base = np.asarray(cl, dtype=np.float64)[ls]
    out = np.zeros((ncomp, n), dtype=np.complex128)
    for c in range(ncomp):
        var = base * (1.0 if c == 0 else cl_b_ratio)
        re = rng.standard_normal(n)
        im = rng.standard_normal(n)
        sd = np.sqrt(np.where(ms == 0, var, var / 2.0))
        out[c] = sd * (re + 1j * np.where(ms == 0, 0.0, im))
        out[c][ls < spin] = 0.0
    return out


def uniform_sphere(npts: int, rng: np.random.Generator):
    """theta = arccos U(-1, 1), phi = U[0, 2 pi)."""
    theta = np.arccos(rng.uniform(-1.0, 1.0, npts))
    phi = rng.uniform(0.0, 2.0 * math.pi, npts)
    return theta, phi


def gl_nodes(nring: int):
    """Gauss-Legendre colatitudes (ascending theta) and weights."""
    from scipy.special import roots_legendre
    x, w = roots_legendre(nring)
    theta = np.arccos(x)[::-1].copy()
    return theta, w[::-1].copy()


def gl_grid(nring: int, nphi: int):
    """Full Gauss-Legendre grid, ring-major; returns theta, phi, quadrature weights
    (GL weight times 2 pi / nphi)."""
    th, w = gl_nodes(nring)
    ph = 2.0 * math.pi * np.arange(nphi) / nphi
    theta = np.repeat(th, nphi)
    phi = np.tile(ph, nring)
    wt = np.repeat(w * 2.0 * math.pi / nphi, nphi)
    return theta, phi, wt


def thinned_gl_grid(nring: int):
    """Longitude-thinned GL grid: ring j carries max(4, ceil(2 nring sin theta_j))
    equispaced points (the paper gives no thinning rule; this one keeps the
    equatorial sampling of the full grid)."""
    th, _ = gl_nodes(nring)
    nphi = np.maximum(4, np.ceil(2 * nring * np.sin(th)).astype(np.int64))
    n = int(nphi.sum())
    theta = np.empty(n)
    phi = np.empty(n)
    o = 0
    for j in range(nring):
        k = int(nphi[j])
        theta[o:o + k] = th[j]
        phi[o:o + k] = np.arange(k) * (2.0 * math.pi / k)
        o += k
    return theta, phi


POTENTIAL_RMS_ARCMIN = 2.5


def potential_cl(lmax: int) -> np.ndarray:
    """Shape of the lensing potential's spectrum: L^-4 above L = 60, flat at its
    L = 60 value for 2 <= L <= 60, zero for L < 2 (the overall scale is set by the
    deflection rms)."""
    ell = np.arange(lmax + 1, dtype=np.float64)
    cl = np.where(ell > 60, (np.maximum(ell, 1.0) / 60.0) ** -4.0, 1.0)
    cl[:2] = 0.0
    return cl


def lensing_potential(lmax: int, seed: int, rms_arcmin: float = POTENTIAL_RMS_ARCMIN) -> np.ndarray:
    """Seeded Gaussian lensing potential phi_LM [nalm] complex128 (mmax = lmax), scaled
    so that the realisation's deflection has the requested rms over the sphere:
    mean |alpha|^2 = (1/4 pi) sum_LM L (L + 1) |phi_LM|^2 over all M (stored M > 0
    counted twice, by the reality of the field)."""
    plm = gaussian_alm(lmax, lmax, 0, np.random.default_rng(seed), cl=potential_cl(lmax))[0]
    ls = np.concatenate([np.arange(m, lmax + 1) for m in range(lmax + 1)]).astype(np.float64)
    ms = np.concatenate([np.full(lmax + 1 - m, m) for m in range(lmax + 1)])
    wm = np.where(ms == 0, 1.0, 2.0)
    ms2 = float(np.sum(wm * ls * (ls + 1.0) * np.abs(plm) ** 2)) / (4.0 * math.pi)
    return plm * (rms_arcmin * ARCMIN / math.sqrt(ms2))


WORKLOADS = {
    "tiny_spin0": dict(id=1, spin=0, lmax=127, mmax=127, points="uniform", npts=20000),
    "tlens_l2048": dict(id=2, spin=0, lmax=2048, mmax=2048, points="gl", nring=2049, nphi=4097),
    "pollens_l4096": dict(id=3, spin=2, lmax=4096, mmax=4096, points="gl", nring=4097, nphi=8193),
    "pollens_thin6144": dict(id=6, spin=2, lmax=4096, mmax=4096, points="thin", nring=6144),
}


def base_points(spec: dict, replica: int = 0):
    """Undeflected point set of a workload (theta, phi) as FP64 numpy arrays
    (uniform workloads are not deflected)."""
    kind = spec["points"]
    if kind == "uniform":
        return uniform_sphere(spec["npts"], np.random.default_rng(seed_for(spec["id"], replica)))
    if kind == "gl":
        th, ph, _ = gl_grid(spec["nring"], spec["nphi"])
    elif kind == "thin":
        th, ph = thinned_gl_grid(spec["nring"])
    else:
        raise ValueError(kind)
    return th, ph


def make_potential(spec: dict, replica: int = 0) -> np.ndarray:
    """The workload's lensing potential (band limit = the workload's lmax)."""
    return lensing_potential(spec["lmax"], seed_for(spec["id"], replica) + 500)


# Sampled accuracy check of the full-size workloads: points near the equator (where
# Sect. 4 evaluates the effective accuracy), within 5 degrees of the poles, and
# uniformly random, drawn without repeats from the undeflected point set.
SAMPLE_SPLIT = (5000, 2500, 2500)
SAMPLE_EQ_BAND = 0.01                   # |theta - pi/2| below this, in radians
SAMPLE_POLE_CAP = 5.0 * math.pi / 180.0


def sample_indices(theta, seed: int, split=SAMPLE_SPLIT) -> np.ndarray:
    """Point indices of the sampled check: the equator group, the polar group and the
    random group, concatenated in that order."""
    th = np.asarray(theta)
    rng = np.random.default_rng(seed)
    eq = np.flatnonzero(np.abs(th - math.pi / 2) < SAMPLE_EQ_BAND)
    pole = np.flatnonzero((th < SAMPLE_POLE_CAP) | (th > math.pi - SAMPLE_POLE_CAP))
    g_eq = rng.choice(eq, split[0], replace=False)
    g_pole = rng.choice(pole, split[1], replace=False)
    taken = np.zeros(th.size, bool)
    taken[g_eq] = True
    taken[g_pole] = True
    g_rand = rng.choice(np.flatnonzero(~taken), split[2], replace=False)
    return np.concatenate([g_eq, g_pole, g_rand]).astype(np.int64)


def adjoint_support(split=SAMPLE_SPLIT) -> np.ndarray:
    """Positions (into the sample) where the adjoint check's input is non-zero: the
    first half of each group."""
    o = np.cumsum((0,) + tuple(split))
    return np.concatenate([np.arange(o[k], o[k] + split[k] // 2) for k in range(3)])


def adjoint_check_input(ncomp: int, n: int, seed: int) -> np.ndarray:
    """Values of the adjoint check's input on its support: N(0, 1), [ncomp][n]."""
    return np.random.default_rng(seed).standard_normal((ncomp, n))


def make_alm(spec: dict, replica: int = 0) -> np.ndarray:
    return gaussian_alm(spec["lmax"], spec["mmax"], spec["spin"],
                        np.random.default_rng(seed_for(spec["id"], replica) + 77))


# Batched uneven workload: independent instances with lmax uniform in [512, 3000],
# spin 0 or 2, 1e6 to 6e6 uniformly random points each, FP32 at epsilon 1e-5; and
# the other reading of "16 maps sharing a geometry": 4 geometries of 16 maps each.
BATCH_ID = 4


def batched_instances(n: int = 64, seed: int = 1000 * BATCH_ID):
    """Specs of the uneven batch: dicts with lmax (= mmax), spin, npts and the seeds of
    the instance's points and coefficients."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        lmax = int(rng.integers(512, 3001))
        out.append(dict(lmax=lmax, mmax=lmax, spin=int(rng.choice([0, 2])),
                        npts=int(rng.integers(1_000_000, 6_000_001)),
                        point_seed=seed + 10 * i + 1, alm_seed=seed + 10 * i + 2))
    return out


def batched_groups(ngroups: int = 4, maps: int = 16, seed: int = 1000 * BATCH_ID + 900):
    """Specs of the geometry groups: dicts with lmax, spin, npts, the point seed and one
    coefficient seed per map."""
    rng = np.random.default_rng(seed)
    out = []
    for g in range(ngroups):
        lmax = int(rng.integers(512, 3001))
        out.append(dict(lmax=lmax, mmax=lmax, spin=int(rng.choice([0, 2])),
                        npts=int(rng.integers(1_000_000, 6_000_001)),
                        point_seed=seed + 100 * g + 1,
                        alm_seeds=[seed + 100 * g + 10 + k for k in range(maps)]))
    return out


def instance_points(spec: dict):
    return uniform_sphere(spec["npts"], np.random.default_rng(spec["point_seed"]))


def instance_alm(spec: dict, seed: int) -> np.ndarray:
    return gaussian_alm(spec["lmax"], spec["mmax"], spec["spin"], np.random.default_rng(seed))
