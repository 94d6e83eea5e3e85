"""Pins of the codec oracle (oracle/codec.py) against values derived by hand
and properties the arithmetic fixes.  CPU only.

The codec is this project's definition of the paper's compression stage
(Sec. 3 data-compression paragraph; Sec. 4.2): a fixed-accuracy mode with an
absolute error bound and a lossless mode.  The pins fix each step of the
definition independently of the oracle's own code:
  - the lifting on a linear ramp, worked by hand (transform and orientation);
  - a whole stream worked by hand, word for word (sub-bands, widths, bit
    order, header, chunk table);
  - the error bound and its tightness (the quantiser's step is 2 tol, not tol);
  - bit-exact lossless round trips over special floats and the ordering of
    the lossless key;
  - exact invertibility of the wrapping transform over the full int32 range.
"""
import numpy as np
import pytest

from oracle import codec as zc


def test_ramp_block_by_hand():
    # q[z][x] = x.  Level 1 along x: pairs (2k, 2k+1) give d = -1 and
    # s = (2k+1) + (-1 >> 1) = 2k; along z the rows are equal, so d = 0.
    # Level 2: s values 0,2,4,6 -> pairs (0,2),(4,6): d = -2, s = 1, 5.
    # Level 3: (1,5): d = -4, s = 5 + (-4 >> 1) = 3.
    q = np.tile(np.arange(8, dtype=np.int64), (8, 1))[None]
    want = np.zeros((8, 8), dtype=np.int64)
    want[0, :2] = [3, -4]
    want[:2, 2:4] = -2
    want[:4, 4:] = -1
    got = zc.forward_transform(q)[0]
    np.testing.assert_array_equal(got, want)
    # a ramp along z lands in the transposed positions
    np.testing.assert_array_equal(zc.forward_transform(q.transpose(0, 2, 1).copy())[0], want.T)
    # a constant block keeps only its value in the coarse coefficient
    c = np.full((1, 8, 8), -7, dtype=np.int64)
    want_c = np.zeros((8, 8), dtype=np.int64)
    want_c[0, 0] = -7
    np.testing.assert_array_equal(zc.forward_transform(c)[0], want_c)


def test_ramp_stream_by_hand():
    # x[z][j] = 0.25 j with tol = 0.125: 2 tol = 0.25, so q = j exactly and the
    # coefficients are those of the ramp above.  Zig-zag: 3->6, -4->7, -2->3,
    # -1->1.  Widths: g0 {6,7,0,0} -> 3, g1 {3,3,3,3,0...} -> 2, g2 (all 1) -> 1,
    # g3 = g4 = 0.  Header 3 | 2<<6 | 1<<12 = 4227; 4*3 + 12*2 + 16*1 = 52 bits.
    # Row-major packing: row 0: 6@0-2, 7@3-5, 3@6-7, 3@8-9, 1@10..13;
    # row 1: 0@14-16, 0@17-19, 3@20-21, 3@22-23, 1@24..27; row 2: zeros 28-35,
    # 1@36..39; row 3: zeros 40-47, 1@48..51.  Word 0 has bits 1-13 and 20-27
    # set: 0x0FF03FFE; word 1 bits 4-7 and 16-19: 0x000F00F0.
    x = np.tile(0.25 * np.arange(8, dtype=np.float32), (8, 1))
    words = zc.encode(x, tol=0.125)
    want = [0x315A5452, 0, 1, 8, 8, 256, 0x00000000, 0x3FC00000,  # header, tol = 0.125
            0, 2,                                                  # chunk table
            4227,                                                  # block header
            0x0FF03FFE, 0x000F00F0]                                # payload
    assert [int(w) for w in words] == want
    np.testing.assert_array_equal(zc.decode(words)[0], x)


def test_constant_block_stream_by_hand():
    # 0.5 at tol 0.125 -> q = 2 everywhere -> one coefficient 2 -> zig-zag 4,
    # width 3 in g0, the other three g0 positions hold 0: one payload word = 4.
    x = np.full((8, 8), 0.5, dtype=np.float32)
    assert [int(w) for w in zc.encode(x, tol=0.125)] == [
        0x315A5452, 0, 1, 8, 8, 256, 0, 0x3FC00000, 0, 1, 3, 4]
    # all zeros: a header word of zeros and no payload
    z = zc.encode(np.zeros((8, 8), np.float32), tol=1.0)
    assert [int(w) for w in z[8:]] == [0, 0, 0]


def test_lossless_small_stream_by_hand():
    # +0.0 everywhere except 1.0 at (0, 0): key(1.0) = K = 0x3F800000 = 127 * 2^23,
    # key(+0) = 0.  Each pair step with b = 0 gives d = a, s = a / 2 (K is even
    # enough for every halving), so the non-zero coefficients are
    #   level 1: (0,4) = (4,0) = K/2, (4,4) = K;
    #   level 2: (0,2) = (2,0) = K/8, (2,2) = K/4;
    #   level 3: (0,0) = K/64, (0,1) = (1,0) = K/32, (1,1) = K/16.
    # Zig-zag doubles them; bit lengths (127 * 2^m has m + 7 bits):
    #   g0 max 2K/16 = 127*2^20 -> 27, g1 max 2K/4 -> 29, g2 and g3 2K/2 -> 30,
    #   g4 2K -> 31.  Bits 4*27 + 12*29 + 16*(30+30+31) = 1912 -> 60 words.
    x = np.zeros((8, 8), np.float32)
    x[0, 0] = 1.0
    w = zc.encode(x, mode=zc.MODE_LOSSLESS)
    assert int(w[1]) == zc.MODE_LOSSLESS and int(w[6]) == 0 and int(w[7]) == 0
    assert int(w[10]) == 27 | 29 << 6 | 30 << 12 | 30 << 18 | 31 << 24
    assert [int(v) for v in w[8:10]] == [0, 60] and len(w) == 8 + 2 + 1 + 60
    np.testing.assert_array_equal(zc.decode(w)[0].view(np.uint32), x.view(np.uint32))


@pytest.mark.parametrize("tol", [1e-4, 1e-1, 3.0])
@pytest.mark.parametrize("shape", [(1, 8, 8), (1, 37, 53), (3, 21, 70), (2, 1, 1), (1, 130, 129)])
def test_error_bound_and_tightness(tol, shape):
    rng = np.random.default_rng(7)
    x = (rng.standard_normal(shape) * 50.0).astype(np.float32)
    words = zc.encode(x, tol=tol)
    y = zc.decode(words)
    assert y.shape == x.shape
    err = np.abs(y.astype(np.float64) - x.astype(np.float64))
    assert np.all(err <= zc.error_bound(y, tol))
    if x.size >= 1000 and tol < 1.0:
        # a uniform quantiser of step 2 tol uses most of the bound on random data
        # (a step of tol would stay below tol / 2)
        assert err.max() > 0.9 * tol


def test_edge_replication_and_chunks():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((1, 130, 129)).astype(np.float32)  # 17 x 17 = 289 blocks: 2 chunks
    w = zc.encode(x, tol=1e-3)
    assert zc.parse_header(w)[:5] == (0, 1, 130, 129, 256)
    nblk, nchunks = 289, 2
    table = w[8:8 + nchunks + 1].astype(np.int64)
    headers = w[8 + nchunks + 1: 8 + nchunks + 1 + nblk].astype(np.int64)
    widths = np.stack([(headers >> (6 * g)) & 63 for g in range(5)], axis=1)
    nwords = ((widths * np.array([4, 12, 16, 16, 16])).sum(axis=1) + 31) // 32
    assert table[0] == 0 and table[1] == nwords[:256].sum() and table[2] == nwords.sum()
    assert len(w) == 8 + nchunks + 1 + nblk + nwords.sum()
    # the partial last block column repeats column 128: its coefficients along x
    # within the repeated part are zero, so the stream decodes to the input shape
    assert zc.decode(w).shape == x.shape


def test_lossless_special_values_bit_exact():
    specials = np.array([0.0, -0.0, np.inf, -np.inf, np.nan, 1e-45, -1e-45, 1.17549435e-38,
                         3.4028235e38, -3.4028235e38, 1.0, -1.0], dtype=np.float32)
    payload_nan = np.array([0x7FC12345, 0xFF800001], dtype=np.uint32).view(np.float32)
    rng = np.random.default_rng(11)
    rand_bits = rng.integers(0, 2 ** 32, size=(3, 19, 23), dtype=np.uint64).astype(np.uint32)
    x = rand_bits.view(np.float32).copy()
    flat = x.reshape(-1)
    flat[: len(specials)] = specials
    flat[len(specials): len(specials) + 2] = payload_nan
    y = zc.decode(zc.encode(x, mode=zc.MODE_LOSSLESS))
    np.testing.assert_array_equal(y.view(np.uint32), x.view(np.uint32))


def test_lossless_key_orders_floats():
    rng = np.random.default_rng(5)
    f = np.concatenate([rng.standard_normal(2000).astype(np.float32) * 10.0 ** rng.integers(-30, 30, 2000),
                        np.array([0.0, -0.0, np.inf, -np.inf], np.float32)]).astype(np.float32)
    k = zc.float_key(f)
    order_f = np.argsort(f.astype(np.float64), kind="stable")
    # keys must be non-decreasing along the float order (+0 and -0 compare equal as
    # floats; their keys differ by one)
    assert np.all(np.diff(k[order_f]) >= -1)
    assert np.all(np.diff(np.sort(k)) >= 0)
    np.testing.assert_array_equal(zc.key_float(k).view(np.uint32), f.view(np.uint32))


def test_wrapping_transform_inverts_full_range():
    rng = np.random.default_rng(9)
    q = rng.integers(-2 ** 31, 2 ** 31, size=(500, 8, 8), dtype=np.int64)
    q[0] = 2 ** 31 - 1
    q[1] = -2 ** 31
    q[2, ::2] = 2 ** 31 - 1
    q[2, 1::2] = -2 ** 31
    c = zc.forward_transform(q)
    assert c.min() >= -2 ** 31 and c.max() < 2 ** 31
    np.testing.assert_array_equal(zc.inverse_transform(c), q)
    u = zc.zigzag(c)
    assert u.min() >= 0 and u.max() < 2 ** 32
    np.testing.assert_array_equal(zc.unzigzag(u), c)


def test_zigzag_and_bit_length_by_hand():
    np.testing.assert_array_equal(zc.zigzag([0, -1, 1, -2, 2, 2 ** 31 - 1, -2 ** 31]),
                                  [0, 1, 2, 3, 4, 2 ** 32 - 2, 2 ** 32 - 1])
    np.testing.assert_array_equal(zc.bit_length([0, 1, 2, 3, 4, 255, 256, 2 ** 32 - 1]),
                                  [0, 1, 2, 2, 3, 8, 9, 32])


def test_range_and_finiteness_rejected():
    x = np.zeros((8, 8), np.float32)
    x[3, 3] = np.nan
    with pytest.raises(ValueError):
        zc.encode(x, tol=1e-3)
    y = np.full((8, 8), 5000.0, np.float32)
    with pytest.raises(ValueError):
        zc.encode(y, tol=1e-6)  # 5000 / 2e-6 = 2.5e9 > 2^31 - 1
    zc.encode(y, tol=1e-5)  # 2.5e8 fits


def test_smooth_fields_compress():
    # a smooth field at a coarse tolerance needs far fewer bits than 32 per value;
    # white noise at a tolerance near its spread needs few bits as well
    z, x = np.mgrid[0:64, 0:96].astype(np.float32)
    v = (2000.0 + 3.0 * z + 0.5 * x).astype(np.float32)
    assert zc.stream_bytes(zc.encode(v, tol=0.1)) < 0.25 * v.nbytes
    assert zc.stream_bytes(zc.encode(v, mode=zc.MODE_LOSSLESS)) < v.nbytes
