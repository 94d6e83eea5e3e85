"""Pins of the fixed-accuracy ZFP-method oracle (oracle/zfp.py) against the
published method and hand-worked codes.  CPU only.

  - the integer lifting equals the published transform matrix T on inputs
    divisible by 16, the inverse lifting equals T^-1 on inputs divisible by
    4, and a round trip loses at most 2 units;
  - negabinary digits worked by hand, and the map is a bijection;
  - the bit-plane code of small coefficient sets worked by hand (verbatim
    bits, group tests, the implied last 1);
  - whole streams worked by hand: a block of ones, a zero block, a block
    below the tolerance;
  - the error bound |x' - x| <= tol on noise, smooth fields, images and
    ragged shapes, for tolerances from 1e-1 to 1e-6, and more bits for a
    smaller tolerance;
  - refused inputs: tol below 2^-60, non-finite values, |x| >= 2^100."""
import math

import numpy as np
import pytest

from oracle import zfp

T16 = np.array([[4, 4, 4, 4], [5, 1, -1, -5], [-4, 4, 4, -4], [-2, 6, -6, 2]], dtype=np.int64)  # 16 T
TINV4 = np.array([[4, 6, -4, -1], [4, 2, 4, 5], [4, -2, 4, -5], [4, -6, -4, 1]], dtype=np.int64)  # 4 T^-1


def test_lifting_is_the_published_transform():
    np.testing.assert_array_equal(T16 @ TINV4, 64 * np.eye(4, dtype=np.int64))  # the inverse is right
    rng = np.random.default_rng(0)
    for _ in range(2000):
        v = rng.integers(-2**24, 2**24, 4) * 16
        np.testing.assert_array_equal(zfp.fwd_lift(*map(int, v)), (T16 @ v) // 16)
        c = rng.integers(-2**24, 2**24, 4) * 4
        np.testing.assert_array_equal(zfp.inv_lift(*map(int, c)), (TINV4 @ c) // 4)
    for _ in range(2000):
        v = [int(a) for a in rng.integers(-2**29, 2**29, 4)]
        back = zfp.inv_lift(*zfp.fwd_lift(*v))
        assert max(abs(a - b) for a, b in zip(back, v)) <= 2


def test_negabinary_by_hand():
    # base -2 digits: 3 = 4 - 2 + 1 (0b111), -1 = -2 + 1 (0b11), 2 = 4 - 2 (0b110)
    for q, u in [(0, 0), (1, 1), (-1, 0b11), (2, 0b110), (-2, 0b10), (3, 0b111), (-3, 0b1101)]:
        assert zfp.negabinary(q) == u
        assert zfp.from_negabinary(u) == q
    rng = np.random.default_rng(1)
    for q in rng.integers(-2**31, 2**31, 1000):
        assert zfp.from_negabinary(zfp.negabinary(int(q))) == int(q)
    # value of the digits: sum of (-2)^k over the set bits
    for q in (5, -7, 123456, -2**29):
        u = zfp.negabinary(q)
        assert sum((-2) ** k for k in range(32) if (u >> k) & 1) == q


def test_sequency_order():
    assert sorted(zfp.SEQ) == [(i, j) for i in range(4) for j in range(4)]
    sums = [i + j for i, j in zfp.SEQ]
    assert sums == sorted(sums)


def _bits(words, n):
    return [(words[p >> 5] >> (p & 31)) & 1 for p in range(n)]


def test_plane_code_by_hand():
    # u0 has bit 1, u3 bit 0.  Planes 31..2: a failed group test each (30
    # zeros).  Plane 1: group 1, u0's bit 1 (n = 1), group 0.  Plane 0: u0's
    # bit 0 verbatim, group 1, u1 = 0, u2 = 0, u3 = 1 (n = 4), group 0.
    w = zfp.BitWriter()
    u = [0] * 16
    u[0], u[3] = 0b10, 0b01
    zfp.encode_planes(u, 0, w)
    assert w.bits == [0] * 30 + [1, 1, 0] + [0, 1, 0, 0, 1, 0]
    assert w.words() == [0xC0000000, 0x24]
    # only the last coefficient set: the scan writes 15 zeros and implies its 1
    w = zfp.BitWriter()
    u = [0] * 16
    u[15] = 1
    zfp.encode_planes(u, 0, w)
    assert w.bits == [0] * 31 + [1] + [0] * 15
    assert w.words() == [0x80000000, 0]
    # kmin cuts the planes: only planes 31..30 of a coefficient with bit 30
    w = zfp.BitWriter()
    u = [1 << 30] + [0] * 15
    zfp.encode_planes(u, 30, w)
    assert w.bits == [0, 1, 1, 0]


def test_stream_of_ones_by_hand():
    # 1.0 = 0.5 * 2^1: e = 1, q = 2^29 for every value; the transform leaves
    # only the DC coefficient, 2^29, negabinary 0x60000000 (2^30 - 2^29).
    # tol = 2^-10: minexp = -10, maxprec = 1 + 10 + 6 = 17, planes 31..15.
    # Bits: 1, e + 127 = 128 in 8 bits, plane 31: group 0; plane 30: group 1,
    # DC 1, group 0; plane 29: DC 1, group 0; planes 28..15: DC 0, group 0.
    words = zfp.encode(np.ones((4, 4), np.float32), 2.0 ** -10)
    tol_words = np.frombuffer(np.float64(2.0 ** -10).tobytes(), dtype=np.uint32)
    head = [zfp.MAGIC, 2, 1, 4, 4, 16, int(tol_words[0]), int(tol_words[1])]
    bits = [1] + [0, 0, 0, 0, 0, 0, 0, 1] + [0] + [1, 1, 0] + [1, 0] + [0, 0] * 14
    assert len(bits) == 43
    payload = [sum(b << p for p, b in enumerate(bits[:32])), sum(b << p for p, b in enumerate(bits[32:]))]
    assert list(words) == head + [0, 2] + payload
    assert payload == [0x2D01, 0]
    np.testing.assert_array_equal(zfp.decode(words), np.ones((1, 4, 4), np.float32))


def test_zero_and_negligible_blocks_are_one_bit():
    # two blocks side by side: zeros, then values below tol 2^-6 (maxprec 0)
    a = np.zeros((4, 8), np.float32)
    a[:, 4:] = 2.0 ** -20  # e = -19: -19 - (-6) + 6 < 0
    words = zfp.encode(a, 2.0 ** -6)
    assert list(words[8:]) == [0, 1, 0]  # table [0, 1], payload: two 0 bits
    np.testing.assert_array_equal(zfp.decode(words), np.zeros((1, 4, 8), np.float32))


@pytest.mark.parametrize("tol", [1e-1, 1e-3, 1e-4, 1e-6])
def test_error_bound(tol):
    rng = np.random.default_rng(int(-math.log10(tol)))
    z, x = np.mgrid[0:40, 0:44]
    cases = [
        rng.standard_normal((2, 33, 45)).astype(np.float32),
        (np.sin(z / 7.0) * np.cos(x / 5.0) * 3.0).astype(np.float32),
        (1500.0 + 1000.0 * (z > 20) + rng.standard_normal((40, 44))).astype(np.float32),
        rng.standard_normal((5, 3)).astype(np.float32) * 1e-3,
        np.array([[7.5]], np.float32),
    ]
    for a in cases:
        d = zfp.decode(zfp.encode(a, tol)).reshape(a.shape)
        assert np.abs(d.astype(np.float64) - a).max() <= tol, (a.shape, np.abs(d - a).max())


def test_smaller_tolerance_costs_more_bits():
    a = np.random.default_rng(9).standard_normal((32, 32)).astype(np.float32)
    sizes = [zfp.encode(a, t).size for t in (1e-1, 1e-2, 1e-3, 1e-4)]
    assert sizes == sorted(sizes) and sizes[0] < sizes[-1]


def test_refused_inputs():
    a = np.ones((4, 4), np.float32)
    with pytest.raises(ValueError):
        zfp.encode(a, 2.0 ** -61)
    with pytest.raises(ValueError):
        zfp.encode(a, float("nan"))
    b = a.copy()
    b[1, 1] = np.nan
    with pytest.raises(ValueError):
        zfp.encode(b, 1e-3)
    b[1, 1] = 2.0 ** 100
    with pytest.raises(ValueError):
        zfp.encode(b, 1e-3)


def test_block_floating_point_truncates():
    # e = 1 (largest 1.0), one unit 2^-29: 3 2^-31 scales to 0.75 units,
    # -3 2^-31 to -0.75 and -1.5 2^-29 to -1.5; truncation toward zero gives
    # 0, 0 and -1 (rounding would give 1, -1, -2; flooring 0, -1, -2)
    x = np.zeros((4, 4), np.float32)
    x[0, 0] = 1.0
    x[1, 1] = 3 * 2.0 ** -31
    x[2, 2] = -3 * 2.0 ** -31
    x[3, 3] = -1.5 * 2.0 ** -29
    q = zfp.block_ints(x, 1)
    assert (q[0][0], q[1][1], q[2][2], q[3][3]) == (2**29, 0, 0, -1)


def test_stream_of_a_ramp_by_hand():
    # rows 0, 1/4, 1/2, 3/4: e = 0, q = j 2^28.  Along x each row becomes
    # T (0, 1, 2, 3) 2^28 = (3 2^27, -2^28, 0, 0); columns are constant, so
    # along y only row 0 stays: coefficient (0, 0) = 3 2^27, (0, 1) = -2^28.
    # Negabinary 0x68000000 and 0x30000000.  tol 2^-4: maxprec 10, planes
    # 31..22.  Plane 31: group 0.  30: group 1, c0 1, group 0.  29: c0 1,
    # group 1, c1 1, group 0.  28: c0 0, c1 1, group 0.  27: c0 1, c1 0,
    # group 0.  26..22: 0, 0, 0 each.
    x = np.tile(np.array([0.0, 0.25, 0.5, 0.75], np.float32), (4, 1))
    w = zfp.BitWriter()
    zfp.encode_block(x, zfp.minexp_of(2.0 ** -4), w)
    head = [1] + [1, 1, 1, 1, 1, 1, 1, 0]  # e + 127 = 127
    planes = [0] + [1, 1, 0] + [1, 1, 1, 0] + [0, 1, 0] + [1, 0, 0] + [0, 0, 0] * 5
    assert w.bits == head + planes
    d = zfp.decode_block(zfp.BitReader(w.words()), zfp.minexp_of(2.0 ** -4))
    assert np.abs(d - x).max() <= 2.0 ** -4
