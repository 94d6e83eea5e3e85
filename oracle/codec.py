"""Block-transform codec for float32 arrays: the definition, in plain NumPy.

TEST INFRASTRUCTURE ONLY: the oracle of the device codec.  Only the tests,
the smoke check and the benchmark's CPU-baseline leg use it; nothing on the
library's path imports it.

The paper passes velocity models, images and seismograms between the stages
of its workflow through an error-bounded lossy coder, and also tries a
lossless setting (Sec. 3, data-compression paragraph; Sec. 4.2, Tables 1 and
2, with absolute error bounds of 1e-4 and 1e-1).  The coder defined here is
this project's own design for the same job, in two modes:

  fixed accuracy (MODE_TOL):  every decoded value x' satisfies
      |x' - x| <= tol (1 + 2^-26) + 2^-24 |x'|
      (the last term is the float32 rounding of the decoded value);
  lossless (MODE_LOSSLESS):   every float32 bit pattern comes back unchanged.

Steps (an integer pipeline; only step 2 differs between the modes):

1. Blocks.  An array of `count` images [rows][cols] is cut into 8 x 8 blocks,
   in order (image, block row, block column).  A block that runs past the
   last row or column repeats that row or column.
2. Integers.  Fixed accuracy: q = rint(x * r) in float64 with r = 1/(2 tol)
   rounded to float64 (ties to even); |q| must not exceed 2^31 - 1 and x
   must be finite.  Lossless: q = the float32 bit pattern read as int32, with
   the low 31 bits flipped when the sign bit is set (an order-preserving
   map that is its own inverse).
3. Transform.  Three levels of a 2-D integer Haar lifting, in int32
   arithmetic that wraps modulo 2^32 (exactly invertible for any input).
   The pair step: d = a - b, s = b + (d >> 1) (arithmetic shift, so
   s = floor((a + b) / 2) when nothing wraps).  At each level on the
   top-left n x n corner (n = 8, 4, 2): pairs of columns (2k, 2k+1) go to
   columns (k, n/2 + k), then pairs of rows (2k, 2k+1) go to rows
   (k, n/2 + k).
4. Sub-bands.  Coefficients are zig-zag mapped to uint32,
   u = (v << 1) ^ (v >> 31), and grouped by position in the 8 x 8 layout:
       g0 rows 0-1, cols 0-1 (4: the coarse average and the last details)
       g1 rows 0-3, cols 0-3 outside g0 (12)
       g2 rows 0-3, cols 4-7 (16)   g3 rows 4-7, cols 0-3 (16)
       g4 rows 4-7, cols 4-7 (16)
   A group's width w_g is the bit length of the largest u in it (0..32).
5. Block code.  One header word w0 | w1<<6 | w2<<12 | w3<<18 | w4<<24, and a
   payload: the 64 coefficients in row-major order of the 8 x 8 layout, each
   in its group's width, concatenated least-significant bit first into
   ceil(bits / 32) 32-bit words (bits = 4 w0 + 12 w1 + 16 (w2 + w3 + w4)).
6. Stream (uint32 words):
       [0] magic 0x315A5452   [1] mode   [2] count   [3] rows   [4] cols
       [5] blocks per chunk (256)         [6..7] tol as float64 (0 if lossless)
       chunk table [nchunks + 1]: payload word offset of each chunk's first
           block, then the total payload words
       block headers [nblocks]
       payload words of every block, in block order.
"""
from __future__ import annotations

import numpy as np

MAGIC = 0x315A5452
MODE_TOL = 0
MODE_LOSSLESS = 1
B = 8
CHUNK = 256
HEADER_WORDS = 8

# group of every position of the 8 x 8 coefficient layout (row-major)
_G = np.full((B, B), 4, dtype=np.int64)
_G[:4, 4:] = 2
_G[4:, :4] = 3
_G[:4, :4] = 1
_G[:2, :2] = 0
GROUP = _G.reshape(-1)
GROUP_SIZE = np.bincount(GROUP)  # [4, 12, 16, 16, 16]


def wrap32(v):
    """Reduce int64 values to int32 two's complement (modulo 2^32)."""
    v = np.asarray(v, dtype=np.int64)
    return ((v + (1 << 31)) & 0xFFFFFFFF) - (1 << 31)


def lift_pair(a, b):
    d = wrap32(a - b)
    return wrap32(b + (d >> 1)), d


def unlift_pair(s, d):
    b = wrap32(s - (d >> 1))
    return wrap32(d + b), b


def forward_transform(blk):
    """[n, 8, 8] int64 (int32 range) -> coefficients in the 8 x 8 layout."""
    x = blk.copy()
    n = B
    while n > 1:
        h = n // 2
        s, d = lift_pair(x[:, :n, 0:n:2], x[:, :n, 1:n:2])
        x[:, :n, :h], x[:, :n, h:n] = s, d
        s, d = lift_pair(x[:, 0:n:2, :n], x[:, 1:n:2, :n])
        x[:, :h, :n], x[:, h:n, :n] = s, d
        n = h
    return x


def inverse_transform(coef):
    x = coef.copy()
    n = 2
    while n <= B:
        h = n // 2
        a, b = unlift_pair(x[:, :h, :n], x[:, h:n, :n])
        x[:, 0:n:2, :n], x[:, 1:n:2, :n] = a, b
        a, b = unlift_pair(x[:, :n, :h], x[:, :n, h:n])
        x[:, :n, 0:n:2], x[:, :n, 1:n:2] = a, b
        n *= 2
    return x


def zigzag(v):
    v = np.asarray(v, dtype=np.int64)
    return ((v << 1) ^ (v >> 63)) & 0xFFFFFFFF  # v is in int32 range


def unzigzag(u):
    u = np.asarray(u, dtype=np.int64)
    return (u >> 1) ^ -(u & 1)


def bit_length(u):
    """Number of significant bits of each value (0 for 0), exact integer arithmetic."""
    u = np.asarray(u, dtype=np.int64)
    n = np.zeros(u.shape, dtype=np.int64)
    for k in range(33):
        n += (u >> k) > 0
    return n


def float_key(x):
    """Lossless step 2: float32 bits -> order-preserving int32."""
    k = np.asarray(x, dtype=np.float32).view(np.int32).astype(np.int64)
    return np.where(k < 0, k ^ 0x7FFFFFFF, k)


def key_float(k):
    k = np.asarray(k, dtype=np.int64)
    k = np.where(k < 0, k ^ 0x7FFFFFFF, k)
    return k.astype(np.int32).view(np.float32)


def block_grid(rows, cols):
    return -(-rows // B), -(-cols // B)


def to_blocks(x):
    """[count][rows][cols] -> [nblocks, 8, 8] with edge replication."""
    count, rows, cols = x.shape
    bz, bx = block_grid(rows, cols)
    zi = np.minimum(np.arange(bz * B), rows - 1)
    xi = np.minimum(np.arange(bx * B), cols - 1)
    p = x[:, zi][:, :, xi]
    return p.reshape(count, bz, B, bx, B).transpose(0, 1, 3, 2, 4).reshape(-1, B, B)


def from_blocks(blk, count, rows, cols):
    bz, bx = block_grid(rows, cols)
    full = blk.reshape(count, bz, bx, B, B).transpose(0, 1, 3, 2, 4).reshape(count, bz * B, bx * B)
    return full[:, :rows, :cols]


def quantise(x, tol):
    r = np.float64(1.0) / (np.float64(2.0) * np.float64(tol))
    q = np.rint(np.asarray(x, dtype=np.float32).astype(np.float64) * r)
    if not np.all(np.abs(q) <= 2147483647.0):  # also false for NaN
        raise ValueError("a value is not finite or exceeds the range of the tolerance")
    return q.astype(np.int64)


def dequantise(q, tol):
    return (np.asarray(q, dtype=np.int64).astype(np.float64) * (np.float64(2.0) * np.float64(tol))).astype(np.float32)


def _as3(x):
    x = np.asarray(x, dtype=np.float32)
    return x[None] if x.ndim == 2 else x


def encode(x, tol=None, mode=MODE_TOL):
    """float32 [rows][cols] or [count][rows][cols] -> uint32 stream words."""
    x = _as3(x)
    count, rows, cols = x.shape
    blk = to_blocks(x)
    if mode == MODE_TOL:
        if not (tol is not None and tol > 0 and np.isfinite(tol)):
            raise ValueError("fixed-accuracy mode needs a finite tolerance > 0")
        q = quantise(blk, tol)
        tol_word = np.float64(tol)
    elif mode == MODE_LOSSLESS:
        q = float_key(blk)
        tol_word = np.float64(0.0)
    else:
        raise ValueError("unknown mode")
    u = zigzag(forward_transform(q)).reshape(-1, B * B)
    nblk = u.shape[0]
    widths = np.zeros((nblk, 5), dtype=np.int64)
    for g in range(5):
        widths[:, g] = bit_length(u[:, GROUP == g].max(axis=1))
    headers = widths[:, 0] | widths[:, 1] << 6 | widths[:, 2] << 12 | widths[:, 3] << 18 | widths[:, 4] << 24
    w = widths[:, GROUP]                                    # width of every coefficient
    bits = (widths * GROUP_SIZE).sum(axis=1)
    nwords = (bits + 31) // 32
    base = np.concatenate([[0], np.cumsum(nwords)])         # payload word offset of each block
    total = int(base[-1])
    # bit position of each coefficient in the payload; scatter its bits into words
    pos = 32 * base[:-1, None] + np.concatenate([np.zeros((nblk, 1), np.int64), np.cumsum(w, axis=1)[:, :-1]], axis=1)
    acc = np.zeros(total + 1, dtype=np.uint64)
    word, shift = (pos // 32).reshape(-1), (pos % 32).reshape(-1)
    val = u.reshape(-1).astype(np.uint64)
    np.add.at(acc, word, (val << shift.astype(np.uint64)) & np.uint64(0xFFFFFFFF))
    spill = (shift + w.reshape(-1)) > 32
    np.add.at(acc, word[spill] + 1, val[spill] >> (32 - shift[spill]).astype(np.uint64))
    payload = acc[:total].astype(np.uint32)
    nchunks = -(-nblk // CHUNK)
    chunk_table = base[np.minimum(np.arange(nchunks + 1) * CHUNK, nblk)]
    head = np.zeros(HEADER_WORDS, dtype=np.uint32)
    head[:6] = [MAGIC, mode, count, rows, cols, CHUNK]
    head[6:8] = np.array([tol_word], dtype=np.float64).view(np.uint32)
    return np.concatenate([head, chunk_table.astype(np.uint32), headers.astype(np.uint32), payload])


def parse_header(words):
    words = np.asarray(words, dtype=np.uint32)
    if len(words) < HEADER_WORDS or int(words[0]) != MAGIC:
        raise ValueError("not a codec stream")
    mode, count, rows, cols, chunk = (int(v) for v in words[1:6])
    tol = float(words[6:8].view(np.float64)[0])
    return mode, count, rows, cols, chunk, tol


def decode(words):
    """uint32 stream words -> float32 [count][rows][cols]."""
    words = np.asarray(words, dtype=np.uint32)
    mode, count, rows, cols, chunk, tol = parse_header(words)
    bz, bx = block_grid(rows, cols)
    nblk = count * bz * bx
    nchunks = -(-nblk // chunk)
    o = HEADER_WORDS + nchunks + 1
    headers = words[o:o + nblk].astype(np.int64)
    payload = words[o + nblk:].astype(np.uint64)
    widths = np.stack([(headers >> (6 * g)) & 63 for g in range(5)], axis=1)
    w = widths[:, GROUP]
    nwords = ((widths * GROUP_SIZE).sum(axis=1) + 31) // 32
    base = np.concatenate([[0], np.cumsum(nwords)])
    pos = 32 * base[:-1, None] + np.concatenate([np.zeros((nblk, 1), np.int64), np.cumsum(w, axis=1)[:, :-1]], axis=1)
    word, shift, wf = (pos // 32).reshape(-1), (pos % 32).reshape(-1), w.reshape(-1)
    padded = np.concatenate([payload, np.zeros(1, np.uint64)])
    both = padded[word] | (padded[np.minimum(word + 1, len(padded) - 1)] << np.uint64(32))
    mask = (np.uint64(1) << wf.astype(np.uint64)) - np.uint64(1)
    u = ((both >> shift.astype(np.uint64)) & mask).astype(np.int64).reshape(nblk, B, B)
    q = inverse_transform(unzigzag(u))
    q = from_blocks(q, count, rows, cols)
    return dequantise(q, tol) if mode == MODE_TOL else key_float(q)


def stream_bytes(words):
    return 4 * len(words)


def error_bound(decoded, tol):
    """Largest |x' - x| the fixed-accuracy mode allows for each decoded value."""
    d = np.abs(np.asarray(decoded, dtype=np.float64))
    return tol * (1.0 + 2.0 ** -26) + d * 2.0 ** -24
