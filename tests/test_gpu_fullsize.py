"""Parity at the full size of the realistic survey (351 x 1701 at 10 m,
nb 50, nt 4000), in the launch configuration the benchmark times: several
shots advancing together in graph-replayed batched launches with the tuned
tile height.  One shot carries data modelled by the FP64 oracle; the other
shots carry zero data, so they do all the work of a shot but add exactly
zero to the stack, which must then equal the oracle's image of that shot.
The shots run in two shot groups (a reduced cache budget) on the two
streams the batched path alternates its groups between, as the
benchmark's shots do.  The oracle migrates with checkpointed source
wavefields (bit-identical to storing them all) and takes about a minute on
the host's cores."""
import numpy as np
import pytest

import oracle
from paper_2001_06444_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def rtm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2001_06444_amd import rtm as _rtm

    return _rtm


def test_faulted_survey_full_size_batched_matches_oracle(rtm, monkeypatch):
    # two backward shot groups of two shots each, one on each stream (60 MiB
    # per group; the benchmark's 100 shots run in 27 backward groups of 3-4
    # under the default cache budget)
    monkeypatch.setenv("RTM_GROUP_STREAMS", "2")
    monkeypatch.setenv("RTM_GROUP_KB", str(120 << 10))
    sv = inputs.faulted_survey(n_shots=100, nt=4000)
    sh = sv.shots[50]
    kw = dict(dz=sv.h, dx=sv.h, dt=sv.dt, nb=sv.nb, nt=sv.nt)
    dtrue = oracle.forward(sv.vel_true, sv.wavelet, sh.src, sh.rec, **kw)["traces"]
    dsm = oracle.forward(sv.vel_mig, sv.wavelet, sh.src, sh.rec, **kw)["traces"]
    data = dtrue - dsm
    ref = oracle.rtm_shot(sv.vel_mig, sv.wavelet, sh.src, sh.rec, data, dz=sv.h, dx=sv.h,
                          dt=sv.dt, nb=sv.nb, s_mode="checkpoint", ckpt=64)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32).cuda()
    grid = rtm.make_grid(sv.nz, sv.nx, sv.nb, sv.nt, sv.h, sv.h, sv.dt)
    zero = torch.zeros(sv.nt, sv.nx, device="cuda")
    shots = []
    for k in (10, 50, 75, 90):
        s = sv.shots[k]
        shots.append((s.src, s.ix0, s.width, s.rec, t(data) if k == 50 else zero))
    with rtm.Context(0, arena_bytes=2 << 30) as ctx:
        # traces of the true model at full size
        tr = torch.empty(sv.nt, len(sh.rec), device="cuda")
        ctx.propagate(grid, t(sv.vel_true), t(sv.wavelet), sh.src, sh.rec, tr)
        torch.cuda.synchronize()
        et = oracle.rel_l2(tr.double().cpu().numpy(), dtrue)
        img = torch.zeros(sv.nz, sv.nx, device="cuda")
        ctx.migrate_batch(grid, t(sv.vel_mig), t(sv.wavelet), shots, rtm.img_opts("reconstruct"), img)
        torch.cuda.synchronize()
        out = img.double().cpu().numpy()
        st = ctx.stats()
    e = oracle.rel_l2(out, ref)
    print(f"full-size traces rel L2 {et:.3e}; batched reconstruct image rel L2 {e:.3e}; "
          f"tile height {st.tile_z}; graph replays {st.graph_replays}")
    assert st.graph_replays > 0
    assert (st.last_groups_fwd, st.last_groups_bwd) == (1, 2), (st.last_groups_fwd, st.last_groups_bwd)
    # Traces: FP32 rounding of the update c L u grows with (v dt / h)^2 and with
    # nt; at 4700 m/s (10x the two-layer model's c at 1500 m/s) and nt = 4000
    # (4x), the two-layer bound of 3e-5 scales to ~1e-4: 2e-4 is the bound here.
    assert et <= 2e-4
    # Images: the stated bound for FP32-stored / reconstructed source wavefields.
    assert e <= 1e-4
