"""CPU check of the kernel error tables the library chooses its kernel support from.

For each oversampling factor sigma the library stores, per support w, the relative
L2 error of a 2-D type-2 NUFFT with the exponential-of-semicircle kernel (Sect. 3) at
its beta / w, measured on 81 x 81 random Fourier modes at 2000 random points against
the direct sum; a plan takes the smallest w whose entry is at most epsilon / 2.  This
test parses the table from the library source, recomputes every entry with the
oracle's plain FP64 type-2 NUFFT (oracle.nufft_sht.nufft_type2) on the same draw, and
checks that each stored value matches (within a factor 1.5 where the error is above
FP64 rounding) and that every support the plans pick stays within epsilon / 2."""
import os
import re

import numpy as np
import pytest

from oracle import nufft_sht

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2304_10431_amd", "csrc", "capi.cpp")


def stored_tables():
    src = open(SRC).read()
    body = src[src.index("const EsSetting kEs["):]
    body = body[:body.index("};")]
    out = []
    for m in re.finditer(r"\{\s*([0-9.]+)\s*,\s*([0-9.]+)\s*,\s*\{([^}]*)\}\s*\}", body):
        errs = [float(x) for x in m.group(3).replace("\n", " ").split(",")]
        out.append((float(m.group(1)), float(m.group(2)), errs))
    return out


@pytest.fixture(scope="module")
def draw():
    rng = np.random.default_rng(0)
    K, M = 40, 2000
    c = rng.standard_normal((2 * K + 1, 2 * K + 1)) + 1j * rng.standard_normal((2 * K + 1, 2 * K + 1))
    x, y = rng.uniform(0, np.pi, M), rng.uniform(0, 2 * np.pi, M)
    k = np.arange(-K, K + 1)
    exact = np.einsum("ij,pi,pj->p", c, np.exp(1j * np.outer(x, k)), np.exp(1j * np.outer(y, k)))
    return K, c, x, y, exact


def test_table_entries_recomputed(draw):
    K, c, x, y, exact = draw
    tables = stored_tables()
    assert [t[0] for t in tables] == [2.0, 1.5, 1.25]
    for sigma, bw, errs in tables:
        n = int(np.ceil(sigma * (2 * K + 1)))
        n += n % 2
        for w in range(4, 17):
            got = nufft_sht.nufft_type2(c, x, y, n, n, w, bw * w)
            e = float(np.linalg.norm(got - exact) / np.linalg.norm(exact))
            ref = errs[w]
            if ref >= 1e-13:
                assert ref / 1.5 <= e <= ref * 1.5, (sigma, w, e, ref)
            else:
                assert e <= 1e-13, (sigma, w, e)


@pytest.mark.parametrize("eps", [1e-3, 1e-5, 1e-8, 1e-10, 1e-12])
def test_chosen_support_meets_half_eps(draw, eps):
    """The support a plan picks (smallest w with stored error <= eps / 2) reaches
    eps / 2 on the recomputed draw too, and one cell less would not be chosen."""
    K, c, x, y, exact = draw
    for sigma, bw, errs in stored_tables():
        ws = [w for w in range(4, 17) if errs[w] <= 0.5 * eps]
        if not ws:
            continue
        w = ws[0]
        n = int(np.ceil(sigma * (2 * K + 1)))
        n += n % 2
        got = nufft_sht.nufft_type2(c, x, y, n, n, w, bw * w)
        e = float(np.linalg.norm(got - exact) / np.linalg.norm(exact))
        assert e <= 0.5 * eps * 1.5, (sigma, eps, w, e)
        if w > 4:
            assert errs[w - 1] > 0.5 * eps
