"""GPU Born modelling (the linearised operator migration is the adjoint of),
the Eq. 5 source-normalised image, and the Chan merge of statistics."""
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


@pytest.fixture(scope="module")
def ctx(rtm):
    c = rtm.Context(0, arena_bytes=1 << 30)
    yield c
    c.close()


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def _model(seed=0, nz=40, nx=150):
    rng = np.random.default_rng(seed)
    vel = np.where(np.arange(nz)[:, None] < 17, 1500.0, 2300.0) * np.ones((1, nx))
    return vel * (1 + 0.1 * rng.random((nz, nx)))


def test_born_matches_oracle(rtm, ctx):
    vel = _model()
    nz, nx = vel.shape
    nt, h, dt, nb = 300, 10.0, 1e-3, 10
    w = inputs.ricker(nt, dt, fp=25)
    m = np.random.default_rng(3).standard_normal((nz, nx))
    rec = [(1, i) for i in range(0, nx, 2)]
    ref = oracle.born(vel, w, (3, 70), m, rec, dz=h, dx=h, dt=dt, nb=nb, nt=nt)
    g = rtm.make_grid(nz, nx, nb, nt, h, h, dt)
    dd = torch.empty(nt, len(rec), device="cuda")
    ctx.born(g, dev(vel), dev(w), (3, 70), dev(m), rec, dd)
    e = oracle.rel_l2(host(dd), ref)
    print(f"Born traces rel L2 {e:.3e}")
    assert e <= 5e-5


@pytest.mark.parametrize("tz2", ["16", "24", "32"])
@pytest.mark.parametrize("nt, nb", [(2, 10), (3, 10), (38, 10), (39, 9)])
def test_born_two_step_launches_equal_one_step(rtm, ctx, tz2, nt, nb, monkeypatch):
    """Born modelling two steps per launch (each tile's first step over its
    middle region, the second from LDS) gives the traces of one step per
    launch bit for bit: every forced two-step height; nt = 2 (one step, no
    pair), odd and even step counts (a last single step); nb 9 (a grid whose
    last 24-row tile does not fit takes 16 rows); the source at a tile corner,
    receivers on both sides of two-step tile edges (rows 23-25, columns
    55-57 and 111-113 of the padded grid) and at the grid's corners."""
    vel = _model(7, nz=45, nx=130)
    nz, nx = vel.shape
    h, dt = 10.0, 1e-3
    w = inputs.ricker(nt, dt, fp=25)
    m = np.random.default_rng(8).standard_normal((nz, nx))
    g = rtm.make_grid(nz, nx, nb, nt, h, h, dt)
    rec = sorted({(z - nb, x - nb) for z in (23, 24, 25) for x in (55, 56, 57, 111, 112, 113)
                  if 0 <= z - nb < nz and 0 <= x - nb < nx} | {(0, 0), (nz - 1, nx - 1), (0, nx - 1)})
    src = (24 - nb, 56 - nb)
    out = {}
    for key in ("0", tz2):
        monkeypatch.setenv("RTM_TILE_Z2", key)
        dd = torch.full((nt, len(rec)), float("nan"), device="cuda")
        ctx.born(g, dev(vel), dev(w), src, dev(m), rec, dd)
        out[key] = dd
    torch.cuda.synchronize()
    assert torch.isfinite(out["0"]).all()
    assert torch.equal(out["0"], out[tz2]), (tz2, nt, nb)
    if nt > 3:
        assert float(out[tz2].abs().max()) > 0


@pytest.mark.parametrize("streams", ["1", "2"])
@pytest.mark.parametrize("group_kb", [None, "1", "1000"])
def test_born_batch_equals_born_per_shot(rtm, ctx, group_kb, streams, monkeypatch):
    """Born shots advanced together in shared launches (one c, one copy of the
    perturbation) give each shot's rtm_born traces bit for bit: sources in
    the interior, at the model's edge column and inside the first physical
    row, receiver sets of different sizes, one shot without receivers; and
    the first shot against the oracle.  The cache budget (RTM_GROUP_KB) puts
    the shots in one launch group, one group per shot, or two groups, run on
    one stream or alternating between two (RTM_GROUP_STREAMS)."""
    if group_kb is None:
        monkeypatch.delenv("RTM_GROUP_KB", raising=False)
    else:
        monkeypatch.setenv("RTM_GROUP_KB", group_kb)
    monkeypatch.setenv("RTM_GROUP_STREAMS", streams)
    vel = _model(4)
    nz, nx = vel.shape
    nt, h, dt, nb = 260, 10.0, 1e-3, 10
    w = inputs.ricker(nt, dt, fp=25)
    m = np.random.default_rng(5).standard_normal((nz, nx))
    g = rtm.make_grid(nz, nx, nb, nt, h, h, dt)
    specs = [((3, 70), [(1, i) for i in range(0, nx, 2)]),
             ((0, nx - 1), [(2, i) for i in range(5, 120, 3)]),
             ((20, 0), [(0, 0), (nz - 1, nx - 1), (10, 75)]),
             ((12, 33), [])]
    shots, singles = [], []
    for src, rec in specs:
        out = torch.full((nt, max(len(rec), 1)), float("nan"), device="cuda")
        shots.append((src, rec, out if rec else None))
        one = torch.full((nt, max(len(rec), 1)), float("nan"), device="cuda")
        ctx.born(g, dev(vel), dev(w), src, dev(m), rec, one if rec else None)
        singles.append(one)
    ctx.born_batch(g, dev(vel), dev(w), dev(m), shots)
    torch.cuda.synchronize()
    ngroups = ctx.stats().last_born_groups
    assert ngroups == {None: 1, "1": 4}.get(group_kb, ngroups) and 1 <= ngroups <= 4, ngroups
    for (src, rec, out), one in zip(shots, singles):
        if rec:
            assert torch.equal(out, one), src
            assert torch.isfinite(out).all()
    ref = oracle.born(vel, w, specs[0][0], m, specs[0][1], dz=h, dx=h, dt=dt, nb=nb, nt=nt)
    assert oracle.rel_l2(host(shots[0][2]), ref) <= 5e-5
    with pytest.raises(rtm.RTMError):
        ctx.born_batch(g, dev(vel), dev(w), dev(m), [])


@pytest.mark.parametrize("mode", ["store", "reconstruct"])
def test_gpu_only_dot_product(rtm, ctx, mode):
    """<Born_gpu m, d> = <m, Mig_gpu d> with both operators on the GPU."""
    vel = _model(seed=1)
    nz, nx = vel.shape
    nt, h, dt, nb = 300, 10.0, 1e-3, 10
    w = inputs.ricker(nt, dt, fp=25)
    rng = np.random.default_rng(4)
    m = rng.standard_normal((nz, nx))
    rec = [(1, i) for i in range(nx)]
    d = rng.standard_normal((nt, nx))
    g = rtm.make_grid(nz, nx, nb, nt, h, h, dt)
    dd = torch.empty(nt, nx, device="cuda")
    ctx.born(g, dev(vel), dev(w), (3, 11), dev(m), rec, dd)
    img = torch.zeros(nz, nx, device="cuda")
    ctx.migrate_shot(g, dev(vel), dev(w), (3, 11), rec, dev(d), 0, nx, rtm.img_opts(mode, "fp32", 1), img)
    lhs, rhs = (host(dd) * d).sum(), (m * host(img)).sum()
    assert abs(lhs - rhs) <= 1e-4 * abs(lhs)


def test_source_normalised_image(rtm, ctx):
    vel = _model(seed=2)
    nz, nx = vel.shape
    nt, h, dt, nb = 300, 10.0, 1e-3, 10
    w = inputs.ricker(nt, dt, fp=25)
    rec = [(1, i) for i in range(nx)]
    d = np.random.default_rng(5).standard_normal((nt, nx)) * 1e-3
    ref_i, ref_l = oracle.rtm_shot(vel, w, (3, 70), rec, d, dz=h, dx=h, dt=dt, nb=nb, illum=True)
    g = rtm.make_grid(nz, nx, nb, nt, h, h, dt)
    img = torch.zeros(nz, nx, device="cuda")
    ill = torch.zeros(nz, nx, device="cuda")
    ctx.migrate_shot(g, dev(vel), dev(w), (3, 70), rec, dev(d), 0, nx,
                     rtm.img_opts("reconstruct", illum=True), img, ill)
    assert oracle.rel_l2(host(ill), ref_l) <= 1e-4
    out = torch.empty_like(img)
    ctx.normalize_image(img, ill, out, eps_rel=1e-3)
    ref = ref_i / (ref_l + 1e-3 * ref_l.max())
    assert oracle.rel_l2(host(out), ref) <= 2e-4


def test_chan_merge_equals_two_pass_over_the_union(rtm, ctx):
    rng = np.random.default_rng(6)
    nz, nx = 23, 57
    a = [rng.standard_normal((nz, nx)).astype(np.float32) * 3 + 1 for _ in range(5)]
    b = [rng.standard_normal((nz, nx)).astype(np.float32) - 2 for _ in range(8)]
    sa, sb = ctx.stats_create(nz, nx), ctx.stats_create(nz, nx)
    for im in a:
        ctx.stats_add(sa, dev(im))
    for im in b:
        ctx.stats_add(sb, dev(im[:, :40]), 10, 40)  # b: dense [nz][40] images on columns 10..49
    ctx.stats_merge(sa, sb)
    mean = torch.empty(nz, nx, dtype=torch.float64, device="cuda")
    std = torch.empty_like(mean)
    cnt = torch.empty(nz, nx, dtype=torch.int32, device="cuda")
    ctx.stats_get(sa, mean, std, cnt)
    imgs = a + [im[:, :40] for im in b]
    wins = [(0, nx)] * len(a) + [(10, 40)] * len(b)
    m_ref, s_ref, c_ref = oracle.windowed_stats([i.astype(np.float64) for i in imgs], wins, nz, nx)
    assert np.array_equal(host(cnt), c_ref)
    assert np.abs(host(mean) - m_ref).max() <= 1e-12 * np.abs(m_ref).max()
    assert np.abs(host(std) - s_ref).max() <= 1e-12 * np.abs(s_ref).max()
    ctx.stats_destroy(sa)
    ctx.stats_destroy(sb)
