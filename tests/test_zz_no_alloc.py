"""rtm_codec_encode_noalloc, the encoder for callers that cannot allocate:
through the C ABI its streams equal rtm_codec_encode's byte for byte on two
calls in a row (the second on a smaller array, so stale look-back state
from the first would show), in both modes; the context arena is untouched;
an array beyond its scratch limit is rejected before any device work."""
import ctypes

import numpy as np
import pytest

from paper_2001_06444_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def rtm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2001_06444_amd import rtm as _rtm

    return _rtm


def _pair(ctx, x, **kw):
    ref = ctx.codec_encode(x, **kw)
    torch.cuda.synchronize()
    ref = ref.cpu().numpy()
    out = torch.full((ctx.codec_max_bytes(*((1, *x.shape) if x.dim() == 2 else x.shape)),), 0xA5,
                     dtype=torch.uint8, device="cuda")
    used0 = ctx.stats().arena_used
    got = ctx.codec_encode_noalloc(x, out, **kw)
    torch.cuda.synchronize()
    assert ctx.stats().arena_used == used0
    return ref, got.cpu().numpy()


@pytest.mark.parametrize("lossless", [False, True])
def test_noalloc_encoder_equals_the_arena_encoder(rtm, lossless):
    big = torch.as_tensor(inputs.image_bank(3, 351, 1701)).cuda()          # 3 x 44 x 213 blocks: 110 chunks
    small = torch.as_tensor(np.ascontiguousarray(inputs.image_like(7)[:37, :53])).cuda()  # 1 chunk
    kw = dict(lossless=True) if lossless else dict(tol=1e-4)
    with rtm.Context(0, arena_bytes=64 << 20) as ctx:
        for x in (big, small, big):
            ref, got = _pair(ctx, x, **kw)
            assert np.array_equal(ref, got), (x.shape, ref.size, got.size)
            # and it decodes to the same array
            dec = ctx.codec_decode(torch.as_tensor(got).cuda())
            torch.cuda.synchronize()
            ref_dec = ctx.codec_decode(torch.as_tensor(ref).cuda())
            torch.cuda.synchronize()
            assert torch.equal(dec, ref_dec)


def test_noalloc_encoder_rejects_arrays_beyond_its_scratch(rtm):
    with rtm.Context(0, arena_bytes=16 << 20) as ctx:
        x = torch.zeros(8, 8, device="cuda")
        out = torch.zeros(1 << 16, dtype=torch.uint8, device="cuda")
        # 8192 x 4100 blocks = 131200 chunks of 256 > 131040: rejected on the
        # host from the shape alone (x and out are never read or written)
        n = ctypes.c_int64(0)
        lib = rtm.lib()
        rc = lib.rtm_codec_encode_noalloc(ctx.h, x.data_ptr(), 1, 8 * 8192, 8 * 4100, rtm.CODEC_TOL, 1e-3,
                                          out.data_ptr(), out.numel(), ctypes.byref(n))
        assert rc == -1 and b"chunks" in lib.rtm_last_error()
        torch.cuda.synchronize()
        assert not out.any().item()
        # one chunk under the limit passes validation (and then fails on the
        # capacity of the small output buffer, before any device work)
        rc = lib.rtm_codec_encode_noalloc(ctx.h, x.data_ptr(), 1, 8 * 8192, 8 * 4095, rtm.CODEC_TOL, 1e-3,
                                          out.data_ptr(), out.numel(), ctypes.byref(n))
        assert rc == -3 and b"capacity" in lib.rtm_last_error()
