"""GPU codec (rtm_codec_*) against the codec oracle: byte-identical streams
and bit-identical decoded arrays, error paths, and the full-size banks the
benchmark times (velocity samples, images, seismograms)."""
import numpy as np
import pytest

from oracle import codec as zc
from paper_2001_06444_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def rtm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2001_06444_amd import rtm as _rtm

    return _rtm


@pytest.fixture(scope="module")
def ctx(rtm):
    c = rtm.Context(0, arena_bytes=1 << 28)
    yield c
    c.close()


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


def words_of(stream):
    torch.cuda.synchronize()
    b = stream.cpu().numpy()
    assert len(b) % 4 == 0
    return b.view(np.uint32)


def check_same(ctx, x, tol=None, lossless=False):
    """Encode on the GPU and with the oracle; streams and decodes must match bit for bit."""
    x3 = x[None] if x.ndim == 2 else x
    ref = zc.encode(x3, mode=zc.MODE_LOSSLESS) if lossless else zc.encode(x3, tol=tol)
    s = ctx.codec_encode(dev(x3), tol=tol, lossless=lossless)
    got = words_of(s)
    assert len(got) == len(ref), f"stream length {len(got)} vs oracle {len(ref)}"
    bad = np.nonzero(got != ref)[0]
    assert len(bad) == 0, f"{len(bad)} words differ, first at {bad[:5]}"
    y = ctx.codec_decode(s)
    torch.cuda.synchronize()
    ref_y = zc.decode(ref)
    np.testing.assert_array_equal(y.cpu().numpy().view(np.uint32), ref_y.view(np.uint32))
    return got, y


SHAPES = [(1, 8, 8), (1, 1, 1), (1, 37, 53), (3, 21, 70), (2, 9, 7), (1, 130, 129), (1, 1, 700), (1, 700, 3)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("tol", [1e-4, 1e-1])
def test_fixed_accuracy_matches_oracle(ctx, shape, tol):
    rng = np.random.default_rng(hash((shape, tol)) % 2 ** 32)
    x = (rng.standard_normal(shape) * 20.0).astype(np.float32)
    _, y = check_same(ctx, x, tol=tol)
    err = np.abs(y.cpu().numpy().astype(np.float64) - x)
    assert np.all(err <= zc.error_bound(y.cpu().numpy(), tol))


@pytest.mark.parametrize("shape", SHAPES)
def test_lossless_matches_oracle(ctx, shape):
    rng = np.random.default_rng(sum(shape))
    x = rng.integers(0, 2 ** 32, size=shape, dtype=np.uint64).astype(np.uint32).view(np.float32)
    flat = x.reshape(-1)
    sp = np.array([0.0, -0.0, np.inf, -np.inf, np.nan, 1e-45], np.float32)
    flat[: min(len(sp), flat.size)] = sp[: flat.size]
    _, y = check_same(ctx, x, lossless=True)
    np.testing.assert_array_equal(y.cpu().numpy().view(np.uint32), x.view(np.uint32))


def test_smooth_and_extreme_values(ctx):
    z, x = np.mgrid[0:77, 0:91].astype(np.float32)
    v = (2000.0 + 3.0 * z + 0.5 * x).astype(np.float32)
    check_same(ctx, v, tol=1e-3)
    check_same(ctx, v, lossless=True)
    check_same(ctx, np.zeros((40, 40), np.float32), tol=1.0)
    # values at the edge of the int32 range of the quantiser
    big = np.full((16, 16), 2147483647.0 * 2e-3 * 0.999, np.float32)
    big[::3] *= -1
    check_same(ctx, big, tol=1e-3)


def test_many_chunks_and_repeated_calls(ctx):
    """256 chunks of look-back, then a smaller call reusing the state."""
    rng = np.random.default_rng(21)
    a = (rng.standard_normal((1, 1024, 2048)) * np.linspace(0.1, 100.0, 2048)).astype(np.float32)
    check_same(ctx, a, tol=1e-2)
    b = rng.standard_normal((1, 100, 90)).astype(np.float32)
    check_same(ctx, b, tol=1e-2)
    check_same(ctx, a, lossless=True)


def test_capacity_too_small_writes_nothing_past_it(ctx, rtm):
    rng = np.random.default_rng(4)
    x = dev(rng.standard_normal((1, 200, 300)).astype(np.float32))
    need = len(zc.encode(x.cpu().numpy(), tol=1e-4)) * 4
    buf = torch.full((need + 4096,), 0xAB, dtype=torch.uint8, device="cuda")
    cap = need - 1000
    with pytest.raises(rtm.RTMError) as ei:
        ctx.codec_encode(x, tol=1e-4, out=buf[:cap])
    assert ei.value.code == -3 and str(need) in str(ei.value)
    torch.cuda.synchronize()
    assert bool((buf[cap:] == 0xAB).all())
    # below the index size: rejected before any launch
    with pytest.raises(rtm.RTMError):
        ctx.codec_encode(x, tol=1e-4, out=buf[:64])
    # exactly the length: accepted
    s = ctx.codec_encode(x, tol=1e-4, out=buf[:need])
    assert s.numel() == need


def test_encode_rejects(ctx, rtm):
    x = np.zeros((1, 16, 16), np.float32)
    x[0, 5, 5] = np.nan
    with pytest.raises(rtm.RTMError) as ei:
        ctx.codec_encode(dev(x), tol=1e-3)
    assert ei.value.code == -1
    ctx.codec_encode(dev(x), lossless=True)  # NaN is fine when lossless
    y = np.full((1, 8, 8), 5000.0, np.float32)
    with pytest.raises(rtm.RTMError):
        ctx.codec_encode(dev(y), tol=1e-6)
    for bad_tol in (0.0, -1.0, float("inf"), float("nan")):
        with pytest.raises(rtm.RTMError):
            ctx.codec_encode(dev(y), tol=bad_tol)
    assert ctx.codec_max_bytes(0, 5, 5) == -1
    # the larger of this coder's bound (index + 64 words per 8 x 8 block) and
    # the ZFP-method coder's (index + 585 bits per 4 x 4 block, per chunk)
    assert ctx.codec_max_bytes(1, 8, 8) == max(4 * (8 + 2 + 1 + 64), 4 * (8 + 2 + (4 * 585 + 31) // 32))


def test_decode_rejects_corrupt_streams(ctx, rtm):
    rng = np.random.default_rng(8)
    x = rng.standard_normal((1, 64, 64)).astype(np.float32)
    good = ctx.codec_encode(dev(x), tol=1e-3).clone()
    n = good.numel()
    # truncated payload
    with pytest.raises(rtm.RTMError):
        ctx.codec_decode(good[: n - 8].clone())
    # bad magic
    b = good.clone()
    b[0] = 0
    with pytest.raises(rtm.RTMError):
        ctx.codec_decode(b)
    # a block width above 32
    hw = good.clone().view(torch.int32)
    hdr = 8 + 1 + 1  # 64 blocks: one chunk, so the headers start at word 10
    hw[hdr + 3] = 40
    with pytest.raises(rtm.RTMError):
        ctx.codec_decode(hw.view(torch.uint8))
    # chunk table disagreeing with the block headers
    hw = good.clone().view(torch.int32)
    hw[9] += 1
    with pytest.raises(rtm.RTMError):
        ctx.codec_decode(hw.view(torch.uint8))
    # output too small
    out = torch.empty(64 * 64 - 1, device="cuda")
    with pytest.raises(rtm.RTMError):
        ctx.codec_decode(good, out=out)
    # the untouched stream still decodes
    y = ctx.codec_decode(good)
    torch.cuda.synchronize()
    assert np.all(np.abs(y.cpu().numpy() - x) <= zc.error_bound(y.cpu().numpy(), 1e-3))


# ---- full-size banks, as the benchmark times them -------------------------

def _bank_slices(words, count, rows, cols):
    """Per-array (headers, payload) slices of a bank stream, from its own index."""
    bz, bx = -(-rows // 8), -(-cols // 8)
    per = bz * bx
    nblk = count * per
    nch = -(-nblk // 256)
    hb = 8 + nch + 1
    headers = words[hb: hb + nblk].astype(np.int64)
    widths = np.stack([(headers >> (6 * g)) & 63 for g in range(5)], axis=1)
    nwords = ((widths * np.array([4, 12, 16, 16, 16])).sum(axis=1) + 31) // 32
    base = np.concatenate([[0], np.cumsum(nwords)])
    pay = words[hb + nblk:]
    table = words[8: 8 + nch + 1].astype(np.int64)
    assert np.array_equal(table, base[np.minimum(np.arange(nch + 1) * 256, nblk)])
    assert len(pay) == base[-1]
    return [(headers[a * per:(a + 1) * per], pay[base[a * per]: base[(a + 1) * per]]) for a in range(count)]


@pytest.mark.parametrize("kind", ["velocity", "image", "seismogram"])
def test_full_size_bank_sampled(ctx, rtm, kind):
    """Bank of arrays in one call: every sampled array's block headers and
    payload equal the oracle's stream of that array alone, and the decoded
    bank equals the oracle's decode of those arrays."""
    if kind == "velocity":
        bank = inputs.velocity_bank(6)
        tols = [1e-4, 1e-1]
    elif kind == "image":
        bank = np.stack([inputs.image_like(s) for s in range(6)])
        tols = [1e-4, 1e-1]
    else:
        bank = np.stack([inputs.seismogram_like(s) for s in range(2)])
        tols = [1e-4]
    count, rows, cols = bank.shape
    big = torch.empty(ctx.codec_max_bytes(count, rows, cols), dtype=torch.uint8, device="cuda")
    for tol in tols + [None]:
        s = ctx.codec_encode(dev(bank), tol=tol, lossless=tol is None, out=big)
        w = words_of(s)
        parts = _bank_slices(w, count, rows, cols)
        y = ctx.codec_decode(s).cpu().numpy()
        for a in sorted({0, count // 2, count - 1}):
            ref = zc.encode(bank[a], tol=tol) if tol else zc.encode(bank[a], mode=zc.MODE_LOSSLESS)
            per = len(parts[a][0])
            rh = ref[8 + (-(-per // 256)) + 1:][:per]
            rp = ref[8 + (-(-per // 256)) + 1 + per:]
            assert np.array_equal(parts[a][0], rh), f"{kind} array {a} tol {tol}: headers differ"
            assert np.array_equal(parts[a][1], rp), f"{kind} array {a} tol {tol}: payload differs"
            np.testing.assert_array_equal(y[a].view(np.uint32), zc.decode(ref)[0].view(np.uint32))
        print(f"{kind} tol={tol}: ratio {bank.nbytes / s.numel():.2f}")
