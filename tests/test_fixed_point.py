"""The fixed-point rounding the spreading kernels use (host-side check of the
identities, in numpy, with the kernels' constants).

For |x| < 2^51 the double x + M, M = 1.5 * 2^52, has exponent 52, so its bits read
as a 64-bit integer are KM + round(x) (round half to even), KM = bits(M), which is
zero below bit 51.  Sums of such words therefore keep the sum of the rounded values
in their low 51 bits whatever the KM terms add above them, as long as the sum stays
within 2^50 in magnitude (FP64 grids, fast form).  FP32 complex cells pack
Re * 2^32 + Im into one word from bits(Re + M - KMhi) and bits(Im + M)."""
import numpy as np

M = 6755399441055744.0
KM = 0x4338000000000000
KMHI = 0x43380000


def bits(x):
    return np.asarray(x, dtype=np.float64).view(np.uint64)


def test_magic_rounding_is_round_half_even():
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.uniform(-2.0 ** 50, 2.0 ** 50, 20000),
                        rng.uniform(-1e3, 1e3, 20000),
                        np.array([0.5, 1.5, 2.5, -0.5, -1.5, -2.5, 2.0 ** 50 - 0.5, -2.0 ** 50])])
    w = bits(x + M)
    r = (w.astype(np.int64) - np.int64(KM))
    assert np.array_equal(r, np.rint(x).astype(np.int64))
    assert KM & ((1 << 51) - 1) == 0


def test_sum_of_magic_words_keeps_the_sum_in_51_bits():
    rng = np.random.default_rng(4)
    for n in (1, 2, 7, 142, 5000):
        x = rng.uniform(-1.0, 1.0, n) * (2.0 ** 50 / n)
        with np.errstate(over="ignore"):
            t = np.sum(bits(x + M), dtype=np.uint64)  # wraps modulo 2^64, as the LDS adds do
        low = (int(t) << 13) & ((1 << 64) - 1)
        got = low - (1 << 64) if low >> 63 else low
        got >>= 13
        assert got == int(np.sum(np.rint(x).astype(np.int64)))


def test_fp32_packed_word():
    rng = np.random.default_rng(5)
    re = rng.uniform(-2.0 ** 31, 2.0 ** 31, 5000)
    im = rng.uniform(-2.0 ** 31, 2.0 ** 31, 5000)
    br = bits(re + (M - KMHI))
    bi = bits(im + M)
    with np.errstate(over="ignore"):
        word = bi + (br << np.uint64(32))
    want = (np.rint(re).astype(np.int64) * (1 << 32) + np.rint(im).astype(np.int64)).view(np.uint64)
    assert np.array_equal(word, want)
    # decoding as the kernels do: low 32 bits signed, the rest shifted down
    qi = word.astype(np.uint32).view(np.int32).astype(np.int64)
    qr = (word.view(np.int64) - qi) >> 32
    assert np.array_equal(qi, np.rint(im).astype(np.int64))
    assert np.array_equal(qr, np.rint(re).astype(np.int64))
