"""FP64 CPU oracle for the general spin-weighted SHT pair -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
(``paper_2304_10431_amd``) and never imports it.

What it computes (Reinecke, Belkner & Carron 2023, Sect. 2):

* ``synth``   -- eq. (forward) for spin 0, eq. (forwardpol) with chi = 0 for spin s > 0,
  evaluated as a direct sum over every (l, m), -l <= m <= l.
* ``adjoint`` -- eq. (adjoint) for spin 0; for spin s the two-component adjoint
  followed by the gradient/curl split given right after eq. (forwardpol);
  ``adjoint_cols`` gives the same sums for a chosen set of m only.
* ``ring_synth`` / ``ring_adjoint`` -- the same sums restricted to the
  (theta, m) representation of iso-latitude rings (the "synthesis" step of
  Sect. 3 and its adjoint), used as stage references.
* ``bin_keys`` / ``binsort`` -- definition of the point-to-tile bin sort (no
  paper counterpart; an integer, bit-exact definition).
* ``synth_deriv`` -- derivatives of the synthesis along theta and phi (for the
  gradients with respect to positions that the lensing application of Sect. 2 needs).
* ``eps_eff`` -- the effective relative accuracy of Sect. 4.
* ``nufft_sht`` (submodule) -- a plain FP64 CPU implementation of the FFT/NUFFT
  steps of Sect. 3.

The C part lives in ``gsht_oracle.c`` (plain C + OpenMP) and is compiled with gcc
on first use (or by ``build()``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gsht_oracle.c")
_LIB = os.path.join(_HERE, "libgsht_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c99", "-D_DEFAULT_SOURCE", "-fopenmp", "-fPIC", "-shared",
               "-ffp-contract=off", _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        i, i64 = ctypes.c_int, ctypes.c_int64
        lib.gsht_oracle_slambda.argtypes = [i, i, i, ctypes.c_double, dp]
        lib.gsht_oracle_synth.argtypes = [dp, i, i, i, i64, dp, dp, dp, i]
        lib.gsht_oracle_adjoint.argtypes = [dp, i, i, i, i64, dp, dp, dp, i]
        lib.gsht_oracle_adjoint_cols.argtypes = [dp, i, i, i, i64, dp, dp, dp, i, dp, i]
        lib.gsht_oracle_adjoint_cols.restype = ctypes.c_int
        lib.gsht_oracle_ring_synth.argtypes = [dp, i, i, i, i, dp, dp, i]
        lib.gsht_oracle_ring_adjoint.argtypes = [dp, i, i, i, i, dp, dp, i]
        lib.gsht_oracle_synth_deriv.argtypes = [dp, i, i, i, i64, dp, dp, dp, dp, i]
        lib.gsht_oracle_synth_deriv.restype = ctypes.c_int
        lib.gsht_oracle_nufft_interp.argtypes = [dp, i, i, i, ctypes.c_double, i64, dp, dp, dp, i]
        lib.gsht_oracle_nufft_spread.argtypes = [dp, i, i, i, ctypes.c_double, i64, dp, dp, dp]
        for f in (lib.gsht_oracle_slambda, lib.gsht_oracle_synth, lib.gsht_oracle_adjoint,
                  lib.gsht_oracle_ring_synth, lib.gsht_oracle_ring_adjoint,
                  lib.gsht_oracle_nufft_interp, lib.gsht_oracle_nufft_spread):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError("oracle %s failed with status %d" % (what, rc))


def nalm(lmax: int, mmax: int) -> int:
    """Number of stored coefficients (0 <= m <= mmax, m <= l <= lmax)."""
    return (mmax + 1) * (lmax + 1) - mmax * (mmax + 1) // 2


def alm_index(l, m, lmax: int):
    """m-major triangular index m(2 lmax + 1 - m)/2 + l."""
    return m * (2 * lmax + 1 - m) // 2 + l


def ncomp(spin: int) -> int:
    return 1 if spin == 0 else 2


def slambda(lmax: int, m: int, s: int, theta: float) -> np.ndarray:
    """sY_lm(theta, 0) for l = 0..lmax (any integer m, s); zero below max(|m|, |s|)."""
    out = np.zeros(lmax + 1)
    _check(_load().gsht_oracle_slambda(lmax, m, s, float(theta), _p(out)), "slambda")
    return out


def _as_alm(alm, lmax, mmax, spin):
    a = np.ascontiguousarray(np.asarray(alm, dtype=np.complex128)).reshape(ncomp(spin), nalm(lmax, mmax))
    return a


def synth(alm, lmax: int, mmax: int, spin: int, theta, phi, nthreads: int = 0) -> np.ndarray:
    """Direct-sum synthesis; returns [ncomp][npts] float64 (T, or Q and U)."""
    a = _as_alm(alm, lmax, mmax, spin)
    th = np.ascontiguousarray(theta, dtype=np.float64)
    ph = np.ascontiguousarray(phi, dtype=np.float64)
    out = np.zeros((ncomp(spin), th.size))
    _check(_load().gsht_oracle_synth(_p(a.view(np.float64)), lmax, mmax, spin, th.size,
                                     _p(th), _p(ph), _p(out), nthreads), "synth")
    return out


def adjoint(maps, lmax: int, mmax: int, spin: int, theta, phi, nthreads: int = 0) -> np.ndarray:
    """Direct-sum adjoint; maps [ncomp][npts] float64 -> [ncomp][nalm] complex128."""
    th = np.ascontiguousarray(theta, dtype=np.float64)
    ph = np.ascontiguousarray(phi, dtype=np.float64)
    y = np.ascontiguousarray(np.asarray(maps, dtype=np.float64)).reshape(ncomp(spin), th.size)
    out = np.zeros((ncomp(spin), nalm(lmax, mmax)), dtype=np.complex128)
    _check(_load().gsht_oracle_adjoint(_p(y), lmax, mmax, spin, th.size, _p(th), _p(ph),
                                       _p(out.view(np.float64)), nthreads), "adjoint")
    return out


def adjoint_cols(maps, lmax: int, mmax: int, spin: int, theta, phi, ms,
                 nthreads: int = 0) -> np.ndarray:
    """The direct-sum adjoint restricted to the columns m in ``ms``: [ncomp][nalm]
    complex128 with those columns as ``adjoint`` gives them and zeros elsewhere."""
    th = np.ascontiguousarray(theta, dtype=np.float64)
    ph = np.ascontiguousarray(phi, dtype=np.float64)
    y = np.ascontiguousarray(np.asarray(maps, dtype=np.float64)).reshape(ncomp(spin), th.size)
    ml = np.ascontiguousarray(np.asarray(ms, dtype=np.int32))
    out = np.zeros((ncomp(spin), nalm(lmax, mmax)), dtype=np.complex128)
    _check(_load().gsht_oracle_adjoint_cols(_p(y), lmax, mmax, spin, th.size, _p(th), _p(ph),
                                            _p(ml), ml.size, _p(out.view(np.float64)), nthreads),
           "adjoint_cols")
    return out


def synth_deriv(alm, lmax: int, mmax: int, spin: int, theta, phi, nthreads: int = 0):
    """Derivatives of the direct-sum synthesis along theta and phi at the points:
    (dtheta, dphi), each [ncomp][npts] float64.  d/dphi multiplies each term by i m;
    d/dtheta uses the spin-weighted ladder relation between spins s - 1, s and s + 1."""
    a = _as_alm(alm, lmax, mmax, spin)
    th = np.ascontiguousarray(theta, dtype=np.float64)
    ph = np.ascontiguousarray(phi, dtype=np.float64)
    dth = np.zeros((ncomp(spin), th.size))
    dph = np.zeros((ncomp(spin), th.size))
    _check(_load().gsht_oracle_synth_deriv(_p(a.view(np.float64)), lmax, mmax, spin, th.size,
                                           _p(th), _p(ph), _p(dth), _p(dph), nthreads),
           "synth_deriv")
    return dth, dph


def ring_synth(alm, lmax: int, mmax: int, spin: int, theta, nthreads: int = 0) -> np.ndarray:
    """F_m(theta_j) for m = -mmax..mmax -> [2 mmax + 1][nring] complex (row m + mmax)."""
    a = _as_alm(alm, lmax, mmax, spin)
    th = np.ascontiguousarray(theta, dtype=np.float64)
    out = np.zeros((2 * mmax + 1, th.size), dtype=np.complex128)
    _check(_load().gsht_oracle_ring_synth(_p(a.view(np.float64)), lmax, mmax, spin, th.size,
                                          _p(th), _p(out.view(np.float64)), nthreads), "ring_synth")
    return out


def ring_adjoint(H, lmax: int, mmax: int, spin: int, theta, nthreads: int = 0) -> np.ndarray:
    """Adjoint of the ring synthesis; H [2 mmax + 1][nring] complex -> [ncomp][nalm]."""
    th = np.ascontiguousarray(theta, dtype=np.float64)
    h = np.ascontiguousarray(np.asarray(H, dtype=np.complex128)).reshape(2 * mmax + 1, th.size)
    out = np.zeros((ncomp(spin), nalm(lmax, mmax)), dtype=np.complex128)
    _check(_load().gsht_oracle_ring_adjoint(_p(h.view(np.float64)), lmax, mmax, spin, th.size,
                                            _p(th), _p(out.view(np.float64)), nthreads), "ring_adjoint")
    return out


def eps_eff(est, true) -> float:
    """Effective relative accuracy of Sect. 4: ||est - true||_2 / ||true||_2 over
    all points and components (the formula's reading: an amplitude ratio)."""
    est = np.asarray(est)
    true = np.asarray(true)
    return float(np.linalg.norm((est - true).ravel()) / np.linalg.norm(true.ravel()))


def alm_weights(lmax: int, mmax: int) -> np.ndarray:
    """w_m per stored coefficient: 1 for m = 0, 2 for m > 0 (each stored m > 0
    coefficient stands for the pair +-m of a real field)."""
    w = np.empty(nalm(lmax, mmax))
    for m in range(mmax + 1):
        i0 = alm_index(m, m, lmax)
        w[i0:i0 + lmax + 1 - m] = 1.0 if m == 0 else 2.0
    return w


def alm_inner(x, y, lmax: int, mmax: int) -> float:
    """Real inner product sum_c sum_{l, m>=0} w_m Re(x_lm conj(y_lm)) -- the inner
    product under which the stored-coefficient adjoint is the true adjoint."""
    w = alm_weights(lmax, mmax)
    return float(np.sum(w[None, :] * np.real(np.asarray(x) * np.conj(np.asarray(y)))))


# ---- bin sort definition (integer; no paper counterpart) -------------------

def bin_keys(theta, phi, n1: int, n2: int, w: int, a_min: int, t1: int, t2: int, ntile2: int,
             cells: bool = False):
    """Tile key of each point.

    u = theta * (n1 / (2 pi)) and v = phi * (n2 / (2 pi)) are single-rounded FP64
    products; the first kernel cell is a0 = ceil(u - w/2), b0 = ceil(v - w/2);
    the row offset r0 = a0 - a_min and the column b0 mod n2 give the tile
    (r0 // t1, (b0 mod n2) // t2), flattened row-major with ntile2 tile columns.
    With cells, the key orders a tile's points by that first cell too:
    tile * t1 * t2 + (r0 mod t1) * t2 + ((b0 mod n2) mod t2).
    """
    th = np.asarray(theta, dtype=np.float64)
    ph = np.asarray(phi, dtype=np.float64)
    c1 = np.float64(n1) / (np.float64(2.0) * np.float64(np.pi))
    c2 = np.float64(n2) / (np.float64(2.0) * np.float64(np.pi))
    half = np.float64(w) * np.float64(0.5)
    u = th * c1
    v = ph * c2
    a0 = np.ceil(u - half).astype(np.int64)
    b0 = np.ceil(v - half).astype(np.int64)
    r0 = a0 - a_min
    bm = np.mod(b0, n2)
    tile = (r0 // t1) * ntile2 + bm // t2
    if cells:
        return tile * (t1 * t2) + (r0 % t1) * t2 + bm % t2
    return tile


def binsort(keys, ntiles: int, keys_per_tile: int = 1):
    """Stable sort: (perm, tile_start) with perm = argsort(keys, stable) and
    tile_start[t] = number of points whose tile key // keys_per_tile is < t
    (length ntiles + 1)."""
    k = np.asarray(keys, dtype=np.int64)
    perm = np.argsort(k, kind="stable").astype(np.int32)
    counts = np.bincount(k // keys_per_tile, minlength=ntiles)
    start = np.zeros(ntiles + 1, dtype=np.int64)
    start[1:] = np.cumsum(counts)
    return perm, start.astype(np.int32)
