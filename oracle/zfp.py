"""Fixed-accuracy coder of the published ZFP method, in plain NumPy/Python.

TEST INFRASTRUCTURE ONLY: the oracle of the device coder (RTM_CODEC_ZFP).
Only the tests, the smoke check and the benchmark's CPU-baseline leg use it;
nothing on the library's path imports it.

The paper compresses velocity samples, migrated images and seismograms
between its workflow stages with ZFP in fixed-accuracy mode, absolute error
bounds 1e-4 and 1e-1 (Sec. 3, data-compression paragraph; Sec. 4.2, Tables
1 and 2).  This module is the method as Lindstrom published it (Fixed-rate
compressed floating-point arrays, IEEE TVCG 20(12), 2014; fixed-accuracy
mode as in the ZFP documentation), for 2-D float32 arrays, written from its
description; the stream layout around the block codes is this project's.

Steps per 4 x 4 block (a block that runs past the last row or column
repeats that row or column):

1. Block floating point.  e = the exponent of the block's largest |x|
   (largest |x| = f 2^e, f in [1/2, 1)).  Each value becomes the int32
   q = trunc(x 2^(30 - e)) (|q| < 2^30: two guard bits).
2. Decorrelating transform.  The non-orthogonal 4-point transform
       T = 1/16 [[ 4,  4,  4,  4],
                 [ 5,  1, -1, -5],
                 [-4,  4,  4, -4],
                 [-2,  6, -6,  2]]
   applied to every row, then to every column, in integer lifting steps
   (`fwd_lift`; exactly T on inputs divisible by 16, and its inverse lifting
   exactly T^-1 on inputs divisible by 4).
3. Ordering.  The 16 coefficients in order of sequency (i + j), the list
   SEQ below.
4. Negabinary.  u = (q + 0xAAAAAAAA) xor 0xAAAAAAAA (mod 2^32): base -2
   digits, so that truncating bit planes needs no separate sign.
5. Embedded bit-plane code, planes k = 31 down to kmin.  With n the number
   of coefficients already significant (0 at first): the bits of plane k of
   coefficients 0 .. n-1, verbatim; then, while n < 16, a group-test bit
   (does any coefficient from n on have bit k set?); if it is 1, the bits of
   coefficients n, n+1, ... until one that is 1 (each read advances n; when
   only the last coefficient remains its 1 is implied and not written).
6. Fixed accuracy.  minexp = floor(log2 tol); the block keeps
   maxprec = min(32, max(0, e - minexp + 6)) planes (2 (d + 1) = 6 guard
   planes for d = 2), so kmin = 32 - maxprec.  A block of zeros, or with
   maxprec = 0, is coded as one 0 bit; any other block as a 1 bit, e + 127
   in 8 bits, and its planes.

Decoding inverts the steps: planes give u, q = (u xor 0xAAAAAAAA) -
0xAAAAAAAA, the inverse lifting along columns then rows, and x =
float32(q) 2^(e - 30).

Stream (uint32 words; bits are appended least-significant first within a
word, fields least-significant bit first):
    [0] magic 0x465A5452   [1] mode 2   [2] count   [3] rows   [4] cols
    [5] blocks per chunk (16)           [6..7] tol as float64
    chunk table [nchunks + 1]: word offset (from the payload start) of each
        chunk of 16 blocks, then the total payload words
    payload: each chunk's block codes back to back, padded to a word.
Blocks are numbered (array, block row, block column).
"""
from __future__ import annotations

import math

import numpy as np

MAGIC = 0x465A5452
MODE = 2
BS = 4          # block side
CHUNK = 16      # blocks per chunk
HEADER_WORDS = 8
NBMASK = 0xAAAAAAAA

# coefficient order by sequency i + j (i: row frequency, j: column frequency)
SEQ = [(0, 0), (0, 1), (1, 0), (1, 1), (0, 2), (2, 0), (1, 2), (2, 1),
       (0, 3), (3, 0), (2, 2), (1, 3), (3, 1), (2, 3), (3, 2), (3, 3)]


def _i32(v):
    """int -> int32 two's complement value."""
    v &= 0xFFFFFFFF
    return v - (1 << 32) if v >= (1 << 31) else v


def fwd_lift(a0, a1, a2, a3):
    """Forward decorrelating transform of one 4-vector (integer lifting)."""
    a0 += a3; a0 >>= 1; a3 -= a0
    a2 += a1; a2 >>= 1; a1 -= a2
    a0 += a2; a0 >>= 1; a2 -= a0
    a3 += a1; a3 >>= 1; a1 -= a3
    a3 += a1 >> 1; a1 -= a3 >> 1
    return a0, a1, a2, a3


def inv_lift(a0, a1, a2, a3):
    """Inverse of fwd_lift up to the bits its halvings dropped."""
    a1 += a3 >> 1; a3 -= a1 >> 1
    a1 += a3; a3 <<= 1; a3 -= a1
    a2 += a0; a0 <<= 1; a0 -= a2
    a1 += a2; a2 <<= 1; a2 -= a1
    a3 += a0; a0 <<= 1; a0 -= a3
    return a0, a1, a2, a3


def negabinary(q):
    return ((q + NBMASK) ^ NBMASK) & 0xFFFFFFFF


def from_negabinary(u):
    return _i32((u ^ NBMASK) - NBMASK)


def minexp_of(tol):
    """floor(log2 tol) for a positive, finite tol (exact: from frexp)."""
    f, e = math.frexp(tol)
    return e - 1


def exponent(m):
    """e with m = f 2^e, f in [1/2, 1), for m > 0 (exact)."""
    return math.frexp(m)[1]


class BitWriter:
    def __init__(self):
        self.bits = []

    def put(self, value, n):
        for b in range(n):
            self.bits.append((value >> b) & 1)

    def words(self):
        w = [0] * ((len(self.bits) + 31) // 32)
        for p, b in enumerate(self.bits):
            w[p >> 5] |= b << (p & 31)
        return w


class BitReader:
    def __init__(self, words, start_bit=0):
        self.words, self.pos = words, start_bit

    def get(self, n=1):
        v = 0
        for b in range(n):
            p = self.pos
            if (p >> 5) >= len(self.words):
                raise ValueError("read past the end of a chunk")
            v |= ((self.words[p >> 5] >> (p & 31)) & 1) << b
            self.pos += 1
        return v


def block_values(a, bi, bj):
    """The 4 x 4 block (bi, bj) of a 2-D float32 array, edges repeated."""
    rows, cols = a.shape
    r = np.minimum(np.arange(BS) + BS * bi, rows - 1)
    c = np.minimum(np.arange(BS) + BS * bj, cols - 1)
    return a[np.ix_(r, c)].astype(np.float32)


def check_tol(tol):
    """Accepted tolerances: finite, 2^-60 <= tol.  Then every coded block has
    e > minexp - 6 >= -66, so its scale 2^(e - 30) and values are normal."""
    if not (math.isfinite(tol) and tol >= 2.0 ** -60):
        raise ValueError("tol must be finite and at least 2^-60")


MAX_ABS = 2.0 ** 100  # accepted |x| < 2^100 (decoded values cannot overflow)


def block_ints(x, e):
    """Step 1: q = trunc(x 2^(30 - e)) (exact power-of-two scaling, then
    truncation toward zero), as a 4 x 4 list of ints."""
    return [[int(math.ldexp(float(x[i, j]), 30 - e)) for j in range(BS)] for i in range(BS)]


def encode_block(x, minexp, w: BitWriter):
    """Step 1-6 for one 4 x 4 float32 block; appends its code to w."""
    x = np.asarray(x, dtype=np.float32)
    if not np.isfinite(x).all() or float(np.abs(x).max()) >= MAX_ABS:
        raise ValueError("non-finite value or |x| >= 2^100")
    m = float(np.abs(x).max())
    if m == 0.0:
        w.put(0, 1)
        return
    e = exponent(m)
    maxprec = min(32, max(0, e - minexp + 6))
    if maxprec == 0:
        w.put(0, 1)
        return
    w.put(1, 1)
    w.put(e + 127, 8)
    q = block_ints(x, e)
    for i in range(BS):                     # rows (along x)
        q[i] = list(fwd_lift(*q[i]))
    for j in range(BS):                     # columns (along y)
        col = fwd_lift(q[0][j], q[1][j], q[2][j], q[3][j])
        for i in range(BS):
            q[i][j] = col[i]
    u = [negabinary(q[i][j]) for (i, j) in SEQ]
    encode_planes(u, 32 - maxprec, w)


def encode_planes(u, kmin, w: BitWriter):
    """Step 5: embedded bit-plane code of 16 negabinary coefficients, planes
    31 down to kmin."""
    n = 0
    for k in range(31, kmin - 1, -1):
        for c in range(n):                  # coefficients already significant
            w.put((u[c] >> k) & 1, 1)
        while n < 16:                       # group tests for the rest
            anyset = any((u[c] >> k) & 1 for c in range(n, 16))
            w.put(int(anyset), 1)
            if not anyset:
                break
            while True:
                if n == 15:                 # the last one must hold the 1
                    n = 16
                    break
                b = (u[n] >> k) & 1
                w.put(b, 1)
                n += 1
                if b:
                    break


def decode_block(r: BitReader, minexp):
    """Inverse of encode_block: the 4 x 4 float32 block."""
    if r.get(1) == 0:
        return np.zeros((BS, BS), dtype=np.float32)
    e = r.get(8) - 127
    maxprec = min(32, max(0, e - minexp + 6))
    if maxprec == 0:
        raise ValueError("a coded block must keep at least one plane")
    kmin = 32 - maxprec
    u = [0] * 16
    n = 0
    for k in range(31, kmin - 1, -1):
        for c in range(n):
            u[c] |= r.get(1) << k
        while n < 16:
            if r.get(1) == 0:
                break
            while True:
                if n == 15:
                    u[15] |= 1 << k
                    n = 16
                    break
                b = r.get(1)
                u[n] |= b << k
                n += 1
                if b:
                    break
    q = [[0] * BS for _ in range(BS)]
    for c, (i, j) in enumerate(SEQ):
        q[i][j] = from_negabinary(u[c])
    for j in range(BS):                     # columns first (inverse order)
        col = inv_lift(q[0][j], q[1][j], q[2][j], q[3][j])
        for i in range(BS):
            q[i][j] = _i32(col[i])
    for i in range(BS):
        q[i] = [_i32(v) for v in inv_lift(*q[i])]
    # float32(q) then an exact power-of-two scaling (2^(e - 30) is a normal
    # float32 for every e a coded block can have, see check_tol)
    scale = np.float32(math.ldexp(1.0, e - 30))
    return np.array([[np.float32(q[i][j]) * scale for j in range(BS)] for i in range(BS)], dtype=np.float32)


def geometry(count, rows, cols):
    bz, bx = (rows + BS - 1) // BS, (cols + BS - 1) // BS
    nblocks = count * bz * bx
    return bz, bx, nblocks, (nblocks + CHUNK - 1) // CHUNK


def chunk_words(a3, chunk, tol):
    """Payload words of one chunk (its blocks' codes, padded to a word)."""
    count, rows, cols = a3.shape
    bz, bx, nblocks, _ = geometry(count, rows, cols)
    minexp = minexp_of(tol)
    w = BitWriter()
    for b in range(chunk * CHUNK, min(nblocks, (chunk + 1) * CHUNK)):
        img, rem = divmod(b, bz * bx)
        bi, bj = divmod(rem, bx)
        encode_block(block_values(a3[img], bi, bj), minexp, w)
    return w.words()


def encode(x, tol):
    """Stream words (uint32 array) of x [count][rows][cols] (or [rows][cols])."""
    a3 = np.asarray(x, dtype=np.float32)
    if a3.ndim == 2:
        a3 = a3[None]
    check_tol(tol)
    count, rows, cols = a3.shape
    _, _, nblocks, nchunks = geometry(count, rows, cols)
    payload, table = [], [0]
    for c in range(nchunks):
        payload += chunk_words(a3, c, tol)
        table.append(len(payload))
    t = np.frombuffer(np.float64(tol).tobytes(), dtype=np.uint32)
    head = [MAGIC, MODE, count, rows, cols, CHUNK, int(t[0]), int(t[1])]
    return np.array(head + table + payload, dtype=np.uint32)


def decode(words):
    """Array [count][rows][cols] float32 of a stream."""
    w = np.asarray(words, dtype=np.uint32)
    if int(w[0]) != MAGIC or int(w[1]) != MODE or int(w[5]) != CHUNK:
        raise ValueError("not a fixed-accuracy ZFP-method stream")
    count, rows, cols = (int(v) for v in w[2:5])
    tol = float(np.frombuffer(w[6:8].tobytes(), dtype=np.float64)[0])
    minexp = minexp_of(tol)
    bz, bx, nblocks, nchunks = geometry(count, rows, cols)
    table = [int(v) for v in w[HEADER_WORDS:HEADER_WORDS + nchunks + 1]]
    base = HEADER_WORDS + nchunks + 1
    out = np.zeros((count, bz * BS, bx * BS), dtype=np.float32)
    for c in range(nchunks):
        r = BitReader([int(v) for v in w[base + table[c]:base + table[c + 1]]])
        for b in range(c * CHUNK, min(nblocks, (c + 1) * CHUNK)):
            img, rem = divmod(b, bz * bx)
            bi, bj = divmod(rem, bx)
            out[img, BS * bi:BS * bi + BS, BS * bj:BS * bj + BS] = decode_block(r, minexp)
    return out[:, :rows, :cols]
