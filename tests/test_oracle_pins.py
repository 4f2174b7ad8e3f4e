"""Pins of the FP64 oracle against facts fixed outside the oracle itself.

Each test ties one part of the oracle to mathematics or to an independent
routine: closed forms of low-degree harmonics, scipy's spherical harmonics, a
brute-force high-precision Goldberg sum (mpmath), the sum rule
sum_m |sY_lm|^2 = (2l+1)/(4 pi), parity / conjugation / doubling identities, the
theta-derivative ladder identity, exact Gauss-Legendre quadrature (round trip),
and adjointness of the synthesis/adjoint pair.  A dropped term, a wrong sign or
index, or a transposed operand in the oracle breaks at least one of them.
"""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy.special import sph_harm_y

import oracle
from paper_2304_10431_amd import workloads as wl

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def goldberg_mp(l, m, s, th, dps=40):
    """Goldberg et al. (1967) sum at working precision dps, theta part only."""
    with mp.workdps(dps):
        if l < max(abs(m), abs(s)):
            return mp.mpf(0)
        th = mp.mpf(th)
        pre = (-1) ** m * mp.sqrt(mp.factorial(l + m) * mp.factorial(l - m) * (2 * l + 1)
                                  / (4 * mp.pi * mp.factorial(l + s) * mp.factorial(l - s)))
        tot = mp.mpf(0)
        for r in range(0, l - s + 1):
            k = r + s - m
            if k < 0 or k > l + s:
                continue
            tot += (mp.binomial(l - s, r) * mp.binomial(l + s, k) * (-1) ** (l - r - s)
                    * mp.cos(th / 2) ** (2 * r + s - m) * mp.sin(th / 2) ** (2 * l - 2 * r - s + m))
        return pre * tot


THETAS = [0.0, 1e-3, 0.3, 1.2, math.pi / 2, 2.5, math.pi - 1e-3, math.pi]


def test_closed_forms():
    """Low-degree closed forms (theta part of sY_lm, phi = 0)."""
    for th in THETAS:
        c, s = math.cos(th), math.sin(th)
        cases = [
            (0, 0, 0, 0, 1 / math.sqrt(4 * math.pi)),
            (1, 0, 0, 1, math.sqrt(3 / (4 * math.pi)) * c),
            (1, 1, 0, 1, -math.sqrt(3 / (8 * math.pi)) * s),
            (1, 0, 1, 1, math.sqrt(3 / (8 * math.pi)) * s),
            (2, 0, 2, 2, math.sqrt(15 / (32 * math.pi)) * s * s),
            (2, 2, 2, 2, math.sqrt(5 / (64 * math.pi)) * (1 - c) ** 2),
            (2, -2, 2, 2, math.sqrt(5 / (64 * math.pi)) * (1 + c) ** 2),
        ]
        for l, m, spin, lmax, ref in cases:
            got = oracle.slambda(lmax, m, spin, th)[l]
            assert abs(got - ref) < 1e-15, (l, m, spin, th, got, ref)


def test_goldberg_bruteforce_small_l():
    """Brute-force Goldberg sum (40 digits) for l <= 14, |m| <= 8, |s| <= 3."""
    worst = 0.0
    for s in range(-3, 4):
        for m in range(-8, 9):
            for th in (0.0, 0.05, 0.7, 1.9, math.pi - 0.05, math.pi):
                got = oracle.slambda(14, m, s, th)
                ref = np.array([float(goldberg_mp(l, m, s, th)) for l in range(15)])
                worst = max(worst, float(np.max(np.abs(got - ref))))
    assert worst < 2e-14, worst


def test_goldberg_bruteforce_start_value_large_m():
    """The start term at l0 = max(|m|,|s|) for large m against the 60-digit sum
    (checks the factorial ratio and the half-angle powers far outside the
    double range), and a few recurrence steps beyond it."""
    for m, s, th in [(900, 2, 0.4), (900, -2, 2.2), (1500, 0, 1.0), (700, 3, 0.2), (-800, 2, 1.3)]:
        l0 = max(abs(m), abs(s))
        got = oracle.slambda(l0 + 6, m, s, th)[l0:]
        ref = [goldberg_mp(l, m, s, th, dps=60) for l in range(l0, l0 + 7)]
        for g, r in zip(got, ref):
            if abs(r) < mp.mpf(2) ** -1000:
                assert g == 0.0 or abs(g) < 1e-300
            else:
                assert abs(mp.mpf(g) / r - 1) < 1e-12, (m, s, th, g, r)


def test_spin0_matches_scipy():
    """Spin 0 equals scipy.special.sph_harm_y (Condon-Shortley) to 1e-13."""
    rng = np.random.default_rng(3)
    for m in (0, 1, 5, 40, 150):
        for th in rng.uniform(0, math.pi, 4):
            got = oracle.slambda(300, m, 0, th)
            ref = np.array([sph_harm_y(l, m, th, 0.0).real if l >= m else 0.0 for l in range(301)])
            assert np.max(np.abs(got - ref)) < 1e-13


@pytest.mark.parametrize("lmax,spin,tol", [(1024, 0, 2e-11), (4096, 2, 2e-10), (4096, 0, 2e-10)])
def test_sum_rule_large_l(lmax, spin, tol):
    """sum_{m=-l}^{l} |sY_lm(theta)|^2 = (2l+1)/(4 pi) at l = lmax (unitarity of d).

    The FP64 recurrence loses digits close to the poles at high degree (about
    6e-11 at l = 4096, theta = 1e-3; Sect. 4 notes the same loss for the exact
    SHT at this band limit), hence the degree-dependent tolerance."""
    for th in (1e-3, 0.3, math.pi / 2, 2.9):
        tot = 0.0
        for m in range(-lmax, lmax + 1):
            tot += oracle.slambda(lmax, m, spin, th)[lmax] ** 2
        assert abs(tot * 4 * math.pi / (2 * lmax + 1) - 1) < tol, (th, tot)


def test_parity_conjugation_doubling_identities():
    """sY_lm(pi-th) = (-1)^{l+m} (-s)Y_lm(th);  sY_{l,-m} = (-1)^{s+m} (-s)Y_lm (real
    theta parts); analytic continuation sY_lm(2pi-th) = (-1)^{s+m} sY_lm(th) (the
    sign of the doubling step of Sect. 3)."""
    lmax = 2000
    ls = np.arange(lmax + 1)
    for s in (0, 1, 2, 3):
        for m in (0, 1, 2, 7, 300, 1500):
            for th in (0.02, 0.8, 1.7):
                a = oracle.slambda(lmax, m, s, math.pi - th)
                b = oracle.slambda(lmax, m, -s, th) * (-1.0) ** (ls + m)
                assert np.max(np.abs(a - b)) < 1e-11 * max(1.0, np.max(np.abs(b)))
                c = oracle.slambda(lmax, -m, s, th)
                d = oracle.slambda(lmax, m, -s, th) * (-1.0) ** (s + m)
                assert np.max(np.abs(c - d)) < 1e-11 * max(1.0, np.max(np.abs(d)))
                e = oracle.slambda(lmax, m, s, 2 * math.pi - th)
                f = oracle.slambda(lmax, m, s, th) * (-1.0) ** (s + m)
                assert np.max(np.abs(e - f)) < 1e-10 * max(1.0, np.max(np.abs(f)))


def test_doubling_sign_mpmath():
    """The continuation identity of the doubling step at 40 digits (independent
    of the oracle's recurrence)."""
    for (l, m, s) in [(5, 2, 2), (6, 3, 1), (7, -2, 3), (4, 0, 0), (9, 4, -2)]:
        for th in (0.3, 1.1, 2.8):
            with mp.workdps(40):
                th2 = 2 * mp.pi - mp.mpf(th)   # formed at 40 digits, not in float64
            a = goldberg_mp(l, m, s, th2)
            b = goldberg_mp(l, m, s, th)
            with mp.workdps(40):
                assert abs(a - b * (-1) ** (s + m)) < 1e-30


def test_theta_derivative_ladder():
    """d/dth sY_lm = -[sqrt((l-s)(l+s+1)) (s+1)Y_lm - sqrt((l+s)(l-s+1)) (s-1)Y_lm]/2."""
    lmax = 400
    ls = np.arange(lmax + 1, dtype=float)
    h = 1e-5
    for s in (0, 1, 2):
        for m in (0, 3, 50, 250):
            for th in (0.4, 1.3, 2.6):
                fd = (oracle.slambda(lmax, m, s, th + h) - oracle.slambda(lmax, m, s, th - h)) / (2 * h)
                up = np.sqrt(np.maximum((ls - s) * (ls + s + 1), 0)) * oracle.slambda(lmax, m, s + 1, th)
                dn = np.sqrt(np.maximum((ls + s) * (ls - s + 1), 0)) * oracle.slambda(lmax, m, s - 1, th)
                rhs = -(up - dn) / 2
                assert np.max(np.abs(fd - rhs)) < 1e-5 * max(1.0, np.max(np.abs(rhs)))


@pytest.mark.parametrize("spin", [0, 1, 2, 3])
def test_gl_round_trip_exact(spin):
    """adjoint(W * synth(a)) = a on a GL grid with lmax+1 rings and 2 mmax+1
    longitudes: the quadrature is exact for these band-limited products, so
    this pins normalisation, the real-field convention and the G/C split."""
    lmax, mmax = 24, 19
    rng = np.random.default_rng(11 + spin)
    a = wl.gaussian_alm(lmax, mmax, spin, rng, cl=np.ones(lmax + 1))
    th, ph, wt = wl.gl_grid(lmax + 1, 2 * mmax + 1)
    ph = ph + 0.123  # any longitude offset keeps the quadrature exact
    y = oracle.synth(a, lmax, mmax, spin, th, ph)
    b = oracle.adjoint(y * wt[None, :], lmax, mmax, spin, th, ph)
    assert np.max(np.abs(b - a)) < 1e-12


@pytest.mark.parametrize("spin", [0, 1, 2, 5])
def test_adjointness(spin):
    """<y, A x> = <A^H y, x>_w (w_0 = 1, w_{m>0} = 2) to 1e-12 relative."""
    lmax, mmax = 40, 33
    rng = np.random.default_rng(21 + spin)
    x = wl.gaussian_alm(lmax, mmax, spin, rng, cl=np.ones(lmax + 1))
    th, ph = wl.uniform_sphere(700, rng)
    y = rng.standard_normal((oracle.ncomp(spin), th.size))
    ax = oracle.synth(x, lmax, mmax, spin, th, ph)
    ahy = oracle.adjoint(y, lmax, mmax, spin, th, ph)
    lhs = float(np.sum(y * ax))
    rhs = oracle.alm_inner(x, ahy, lmax, mmax)
    assert abs(lhs - rhs) < 1e-12 * np.linalg.norm(y) * np.linalg.norm(ax)


def test_synth_single_coefficients():
    """Single unit coefficients reproduce closed forms through the full synthesis:
    real part of a_11 = 1 gives 2 Re(Y_11 e^{i phi}); spin-2 G_22 = 1 gives
    Q + iU = -(2Y_22 + (-1)^0 (-2)Y_22 (conj phase)) with the real-field term."""
    th = np.array([0.3, 1.1, 2.0, math.pi])
    ph = np.array([0.2, 4.0, 1.5, 0.7])
    lmax = 3
    a = np.zeros((1, oracle.nalm(lmax, lmax)), complex)
    a[0, oracle.alm_index(1, 1, lmax)] = 1.0
    got = oracle.synth(a, lmax, lmax, 0, th, ph)[0]
    ref = 2 * (-math.sqrt(3 / (8 * math.pi)) * np.sin(th) * np.cos(ph))
    assert np.max(np.abs(got - ref)) < 1e-15
    g = np.zeros((2, oracle.nalm(lmax, lmax)), complex)
    g[0, oracle.alm_index(2, 2, lmax)] = 1.0
    got = oracle.synth(g, lmax, lmax, 2, th, ph)
    c = np.cos(th)
    y22 = math.sqrt(5 / (64 * math.pi)) * (1 - c) ** 2 * np.exp(2j * ph)      # 2Y_22
    y2m2 = math.sqrt(5 / (64 * math.pi)) * (1 + c) ** 2 * np.exp(-2j * ph)   # 2Y_{2,-2}
    # G_{2,-2} = (-1)^2 conj(G_22) = 1  ->  P = -(2Y_22 + 2Y_{2,-2})
    p = -(y22 + y2m2)
    assert np.max(np.abs(got[0] - p.real)) < 1e-15
    assert np.max(np.abs(got[1] - p.imag)) < 1e-15


def test_ring_stage_consistent_with_definition():
    """ring_synth summed over m reproduces synth on ring points; ring_adjoint of
    ring sums reproduces adjoint on those points."""
    lmax, mmax, nring, nphi = 30, 25, 9, 64
    for spin in (0, 2):
        rng = np.random.default_rng(5 + spin)
        a = wl.gaussian_alm(lmax, mmax, spin, rng, cl=np.ones(lmax + 1))
        th = np.linspace(0.1, 3.0, nring)
        F = oracle.ring_synth(a, lmax, mmax, spin, th)
        phis = 2 * math.pi * np.arange(nphi) / nphi
        ms = np.arange(-mmax, mmax + 1)
        P = np.einsum("mj,km->jk", F, np.exp(1j * np.outer(phis, ms)))
        T, Ph = np.repeat(th, nphi), np.tile(phis, nring)
        y = oracle.synth(a, lmax, mmax, spin, T, Ph)
        if spin == 0:
            assert np.max(np.abs(P.real.ravel() - y[0])) < 1e-13
        else:
            assert np.max(np.abs(P.real.ravel() - y[0])) < 1e-13
            assert np.max(np.abs(P.imag.ravel() - y[1])) < 1e-13
        z = rng.standard_normal((oracle.ncomp(spin), T.size))
        zc = z[0] + (1j * z[1] if spin else 0)
        H = np.einsum("jk,km->mj", zc.reshape(nring, nphi), np.exp(-1j * np.outer(phis, ms)))
        b1 = oracle.ring_adjoint(H, lmax, mmax, spin, th)
        b2 = oracle.adjoint(z, lmax, mmax, spin, T, Ph)
        assert np.max(np.abs(b1 - b2)) < 1e-12


def test_bin_sort_definition_small():
    """Stable counting sort agrees with a brute-force bucket fill."""
    rng = np.random.default_rng(9)
    keys = rng.integers(0, 37, 5000)
    perm, start = oracle.binsort(keys, 40)
    buckets = [[] for _ in range(40)]
    for i, k in enumerate(keys):
        buckets[k].append(i)
    assert perm.tolist() == [i for b in buckets for i in b]
    assert start.tolist() == list(np.cumsum([0] + [len(b) for b in buckets]))


@pytest.mark.parametrize("spin", [0, 1, 2, 3])
def test_synth_deriv_vs_finite_differences(spin):
    """Oracle derivatives against Richardson-extrapolated central differences of the
    oracle's own synthesis (lmax 12, so that the fifth derivative stays small)."""
    lmax, mmax = 12, 9
    rng = np.random.default_rng(60 + spin)
    nc = oracle.ncomp(spin)
    a = rng.standard_normal((nc, oracle.nalm(lmax, mmax))) + 1j * rng.standard_normal((nc, oracle.nalm(lmax, mmax)))
    th = rng.uniform(0.2, math.pi - 0.2, 40)
    ph = rng.uniform(0, 2 * math.pi, 40)
    dth, dph = oracle.synth_deriv(a, lmax, mmax, spin, th, ph)

    def fd(f, h):
        d1 = (f(h) - f(-h)) / (2 * h)
        d2 = (f(h / 2) - f(-h / 2)) / h
        return (4 * d2 - d1) / 3

    h = 1e-3
    gt = fd(lambda e: oracle.synth(a, lmax, mmax, spin, th + e, ph), h)
    gp = fd(lambda e: oracle.synth(a, lmax, mmax, spin, th, ph + e), h)
    assert np.max(np.abs(dth - gt)) <= 1e-7 * np.max(np.abs(gt))
    assert np.max(np.abs(dph - gp)) <= 1e-7 * np.max(np.abs(gp))


def test_synth_deriv_spin0_is_spin1_synthesis():
    """For spin 0, (d/dtheta + i / sin(theta) d/dphi) f is the spin-1 synthesis with
    G_lm = sqrt(l (l + 1)) a_lm, C = 0, in the sign convention of eq. forwardpol."""
    lmax = mmax = 60
    rng = np.random.default_rng(61)
    a = rng.standard_normal((1, oracle.nalm(lmax, mmax))) + 1j * rng.standard_normal((1, oracle.nalm(lmax, mmax)))
    th = np.arccos(rng.uniform(-0.99, 0.99, 300))
    ph = rng.uniform(0, 2 * math.pi, 300)
    dth, dph = oracle.synth_deriv(a, lmax, mmax, 0, th, ph)
    g = np.zeros((2, oracle.nalm(lmax, mmax)), complex)
    for m in range(mmax + 1):
        i0 = oracle.alm_index(m, m, lmax)
        ls = np.arange(m, lmax + 1)
        g[0, i0:i0 + ls.size] = np.sqrt(ls * (ls + 1.0)) * a[0, i0:i0 + ls.size]
    qu = oracle.synth(g, lmax, mmax, 1, th, ph)
    scale = np.max(np.abs(qu))
    assert np.max(np.abs(qu[0] - dth[0])) <= 1e-12 * scale
    assert np.max(np.abs(qu[1] - dph[0] / np.sin(th))) <= 1e-12 * scale
