"""Pins for the FP64 oracle against facts fixed outside the oracle itself.

Each test names the passage it follows and what would break it: a dropped
stencil term, a wrong coefficient, sign or factor, a wrong source scaling,
an off-by-one time pairing, a transposed index.
"""
import math
import pathlib

import numpy as np
import pytest

import oracle
from oracle.green import green_ricker_trace
from paper_2001_06444_amd import inputs

GOLDEN = pathlib.Path(__file__).resolve().parent / "golden"


# ---------------------------------------------------------------------------
# P1: 8th-order spatial operator (Sec. 3: "eighth-order scheme in space")
# ---------------------------------------------------------------------------

def _poly_field(deg_z, deg_x, h, n, rng):
    z = (np.arange(n) - n / 2) * h
    x = (np.arange(n) - n / 2) * h
    pz = rng.standard_normal(deg_z + 1)
    px = rng.standard_normal(deg_x + 1)
    P = np.polynomial.polynomial
    f = P.polyval(z, pz)[:, None] + P.polyval(x, px)[None, :]
    d2 = P.polyval(z, P.polyder(pz, 2))[:, None] + P.polyval(x, P.polyder(px, 2))[None, :]
    return f, d2


@pytest.mark.parametrize("deg", range(0, 10))
def test_laplacian_exact_on_polynomials_up_to_degree_9(deg):
    """A central 8th-order 2nd-derivative stencil differentiates every
    polynomial of degree <= 9 exactly (truncation term ~ h^8 f^(10))."""
    rng = np.random.default_rng(deg)
    h, n = 0.05, 40
    f, d2 = _poly_field(deg, deg, h, n, rng)
    L = oracle.laplacian(f, h, h)
    inner = (slice(4, n - 4), slice(4, n - 4))
    scale = max(np.abs(d2[inner]).max(), np.abs(f[inner]).max() / h**2 * 1e-3)
    assert np.abs(L[inner] - d2[inner]).max() <= 1e-10 * scale


def test_laplacian_truncation_term_at_degree_10():
    """Degree 10 is the first one the stencil misses, by exactly the leading
    truncation term of the order-2m central difference, (-1)^(m+1) 2 (m!)^2 /
    (2m+2)! h^2m f^(2m+2) with m = 4: for f = z^10 that is -2 (4!)^2 h^8."""
    n, h = 40, 0.05
    z = (np.arange(n) - n / 2) * h
    f = np.repeat((z**10)[:, None], n, axis=1)
    d2 = np.repeat((90 * z**8)[:, None], n, axis=1)
    L = oracle.laplacian(f, h, 1.0)
    inner = (slice(4, n - 4), slice(4, n - 4))
    expect = -2.0 * math.factorial(4) ** 2 * h**8
    assert np.allclose(L[inner] - d2[inner], expect, rtol=1e-4, atol=0)


def test_laplacian_converges_at_8th_order():
    """Error on sin(kx) + cos(kz) (periodic box) falls as h^8."""
    errs, hs = [], []
    for n in (10, 12, 16, 20):
        Lx = 2 * math.pi
        h = Lx / n
        z = np.arange(n) * h
        x = np.arange(n) * h
        f = np.sin(x)[None, :] + np.cos(z)[:, None]
        L = oracle.laplacian(f, h, h, periodic=True)
        errs.append(np.abs(L + f).max())
        hs.append(h)
    slope = np.polyfit(np.log(hs), np.log(errs), 1)[0]
    assert abs(slope - 8.0) < 0.3, slope


def test_laplacian_anisotropic_spacing_and_axes():
    """dz and dx enter their own axis only (a transposed index would fail)."""
    n = 32
    dz, dx = 0.1, 0.37
    z = np.arange(n) * dz
    x = np.arange(n) * dx
    f = (z**2)[:, None] + 0.0 * x[None, :]
    L = oracle.laplacian(f, dz, dx)
    assert np.allclose(L[4:-4, 4:-4], 2.0, rtol=0, atol=1e-9)
    g = 0.0 * z[:, None] + (x**3)[None, :]
    L = oracle.laplacian(g, dz, dx)
    assert np.allclose(L[4:-4, 4:-4], (6 * x)[None, 4:-4], rtol=0, atol=1e-8)


# ---------------------------------------------------------------------------
# P2: leapfrog in time (Sec. 3: "second-order finite difference scheme in time")
# ---------------------------------------------------------------------------

def _eigenmode(n, h, jz, jx):
    z = np.arange(n) * h
    x = np.arange(n) * h
    L = n * h
    return np.cos(2 * math.pi * jz * z / L)[:, None] * np.cos(2 * math.pi * jx * x / L)[None, :]


def test_leapfrog_periodic_eigenmode_closed_form():
    """With phi an eigenvector of L (L phi = -lam phi), the damped-free recursion
    started from u^-1 = cos(w) phi, u^0 = phi is exactly u^n = cos(n w) phi,
    cos w = 1 - c lam / 2, c = v^2 dt^2.  lam is measured with the (pinned)
    Laplacian; the check pins the time recursion and the factor c."""
    n, h, v, dt = 32, 10.0, 2000.0, 1.5e-3
    phi = _eigenmode(n, h, 3, 5)
    Lphi = oracle.laplacian(phi, h, h, periodic=True)
    lam = -(Lphi * phi).sum() / (phi * phi).sum()
    assert np.allclose(Lphi, -lam * phi, atol=1e-12 * lam)
    c = v * v * dt * dt
    w = math.acos(1 - 0.5 * c * lam)
    nt = 400
    init = np.stack([math.cos(w) * phi, phi])
    vel = np.full((n, n), v)
    out = oracle.forward(vel, None, None, [], dz=h, dx=h, dt=dt, nb=0, nt=nt, periodic=True,
                         final=True, init=init)
    uN = out["final"][0]  # u^{nt-1}
    expect = math.cos((nt - 1) * w) * phi
    assert np.abs(uN - expect).max() <= 1e-10


def test_propagator_spatial_rate_h8_against_exact_symbol():
    """At fixed dt, the gap between the discrete solution and the same
    recursion with the exact symbol |k|^2 closes as h^8."""
    v, dt, Lbox, nt = 1500.0, 1e-3, 640.0, 300
    errs, hs = [], []
    for n in (12, 16, 20, 24):
        h = Lbox / n
        phi = _eigenmode(n, h, 1, 1)
        k2 = 2 * (2 * math.pi / Lbox) ** 2
        c = v * v * dt * dt
        we = math.acos(1 - 0.5 * c * k2)
        init = np.stack([math.cos(we) * phi, phi])
        out = oracle.forward(np.full((n, n), v), None, None, [], dz=h, dx=h, dt=dt, nb=0, nt=nt,
                             periodic=True, final=True, init=init)
        errs.append(np.abs(out["final"][0] - math.cos((nt - 1) * we) * phi).max())
        hs.append(h)
    slope = np.polyfit(np.log(hs), np.log(errs), 1)[0]
    assert abs(slope - 8.0) < 0.5, (slope, errs)


# ---------------------------------------------------------------------------
# P3: physics and scaling against the analytic 2-D Green's function (Eq. 4)
# ---------------------------------------------------------------------------

def test_forward_matches_analytic_green_ricker_at_config_discretisation():
    """Homogeneous 1500 m/s, h = 10 m, dt = 1 ms, point source: traces at
    200 / 500 / 800 m match the closed form within 1 / 2 / 3 % (relative L2
    over 0..0.75 s; the residual is the 10 m grid's dispersion).  A wrong
    source scaling (dx dz, c, 2 pi) or a one-step time shift fails it."""
    gold = np.loadtxt(GOLDEN / "green_ricker_v1500.txt")
    h, dt, v, nt = 10.0, 1e-3, 1500.0, gold.shape[0]
    n = 301
    src = (150, 150)
    rec = [(150, 170), (150, 200), (150, 230)]
    out = oracle.forward(np.full((n, n), v), inputs.ricker(nt, dt), src, rec, dz=h, dx=h, dt=dt,
                         nb=0, nt=nt)["traces"]
    for j, tol in enumerate((0.01, 0.02, 0.03)):
        an = gold[:, j + 1]
        e = np.linalg.norm(out[:, j] - an) / np.linalg.norm(an)
        assert e < tol, (j, e)


def test_forward_converges_second_order_in_time():
    """h = 5 m (spatial error negligible), r = 250 m, T = 0.6 s: each halving of
    dt cuts the error to a quarter (ratio 4 +- 0.3)."""
    h, v, T, n = 5.0, 1500.0, 0.6, 301
    errs = []
    for dt in (1e-3, 5e-4, 2.5e-4):
        nt = int(round(T / dt)) + 1
        tr = oracle.forward(np.full((n, n), v), inputs.ricker(nt, dt), (150, 150), [(150, 200)],
                            dz=h, dx=h, dt=dt, nb=0, nt=nt)["traces"][:, 0]
        an = green_ricker_trace(250.0, v, np.arange(nt) * dt)
        errs.append(np.linalg.norm(tr - an) / np.linalg.norm(an))
    assert errs[0] < 2e-2
    for a, b in zip(errs, errs[1:]):
        assert abs(a / b - 4.0) < 0.3, errs


# ---------------------------------------------------------------------------
# P4: stability limit (Sec. 3: "each RTM verifies its own CFL condition")
# ---------------------------------------------------------------------------

CFL_2D_EQUAL_SPACING = 0.55463  # v dt / h limit of the 2nd-order-time, 8th-order-space scheme


@pytest.mark.parametrize("factor,stable", [(0.99, True), (1.01, False)])
def test_cfl_limit_brute_force(factor, stable):
    n, h = 32, 10.0
    v = 2000.0
    dt = factor * CFL_2D_EQUAL_SPACING * h / v
    rng = np.random.default_rng(7)
    u0 = rng.standard_normal((n, n))
    out = oracle.forward(np.full((n, n), v), None, None, [], dz=h, dx=h, dt=dt, nb=0, nt=10000,
                         periodic=True, final=True, init=np.stack([u0, u0]))
    growth = np.abs(out["final"][0]).max() / np.abs(u0).max()
    if stable:
        assert np.isfinite(growth) and growth < 1e3
    else:
        assert not np.isfinite(growth) or growth > 1e12


# ---------------------------------------------------------------------------
# P5: reciprocity with sponge and heterogeneity (exact discrete symmetry)
# ---------------------------------------------------------------------------

def _small_model(seed=0, nz=20, nx=24):
    rng = np.random.default_rng(seed)
    vel = np.where(np.arange(nz)[:, None] < 9, 1500.0, 2300.0) * np.ones((1, nx))
    return vel * (1 + 0.1 * rng.random((nz, nx)))


def test_reciprocity_with_sponge():
    vel = _small_model()
    kw = dict(dz=10.0, dx=10.0, dt=1e-3, nb=5, nt=120)
    w = inputs.ricker(120, 1e-3, fp=25)
    s, r = (3, 4), (15, 19)
    a = oracle.forward(vel, w, s, [r], **kw)["traces"][:, 0]
    b = oracle.forward(vel, w, r, [s], **kw)["traces"][:, 0]
    assert np.abs(a).max() > 0
    assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()


def test_sponge_is_not_identity_and_absorbs():
    """The sponge changes the field (the operator is not trivially symmetric)
    and the energy returned from the padded edge is small."""
    n, h, dt, nt = 121, 10.0, 1e-3, 900
    vel = np.full((n, n), 1500.0)
    w = inputs.ricker(nt, dt)
    src, rec = (60, 60), [(60, 60)]
    big = oracle.forward(np.full((n + 400, n + 400), 1500.0), w, (260, 260), [(260, 260)],
                         dz=h, dx=h, dt=dt, nb=0, nt=nt)["traces"][:, 0]
    spg = oracle.forward(vel, w, src, rec, dz=h, dx=h, dt=dt, nb=50, nt=nt)["traces"][:, 0]
    rigid = oracle.forward(vel, w, src, rec, dz=h, dx=h, dt=dt, nb=0, nt=nt)["traces"][:, 0]
    late = slice(700, nt)  # after the first edge return from 600 m (0.8 s round trip)
    ref = np.abs(big).max()
    assert np.abs(rigid[late] - big[late]).max() > 0.05 * ref
    assert np.abs(spg[late] - big[late]).max() < 1e-2 * ref


# ---------------------------------------------------------------------------
# P6: migration is the exact adjoint of Born modelling (Sec. 3, Givoli 2014)
# ---------------------------------------------------------------------------

def test_dot_product_born_vs_migration():
    vel = _small_model(seed=1)
    nz, nx = vel.shape
    nt = 120
    kw = dict(dz=10.0, dx=10.0, dt=1e-3, nb=5)
    w = inputs.ricker(nt, 1e-3, fp=25)
    rng = np.random.default_rng(2)
    m = rng.standard_normal((nz, nx))
    d = rng.standard_normal((nt, nx))
    rec = [(1, i) for i in range(nx)]
    dd = oracle.born(vel, w, (3, 4), m, rec, nt=nt, **kw)
    img = oracle.rtm_shot(vel, w, (3, 4), rec, d, **kw)
    lhs, rhs = (dd * d).sum(), (m * img).sum()
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_same_index_pairing_is_not_adjoint():
    """The S^n R^n pairing differs from S^n R^{n+1} by a percent-level amount,
    so the dot test above would catch a one-step pairing slip."""
    vel = _small_model(seed=1)
    nz, nx = vel.shape
    nt = 120
    kw = dict(dz=10.0, dx=10.0, dt=1e-3, nb=5)
    w = inputs.ricker(nt, 1e-3, fp=25)
    rng = np.random.default_rng(2)
    m = rng.standard_normal((nz, nx))
    d = rng.standard_normal((nt, nx))
    rec = [(1, i) for i in range(nx)]
    dd = oracle.born(vel, w, (3, 4), m, rec, nt=nt, **kw)
    # Same-index pairing == pairing with data delayed by one sample.
    d_shift = np.zeros_like(d)
    d_shift[:-1] = d[1:]
    img = oracle.rtm_shot(vel, w, (3, 4), rec, d_shift, **kw)
    lhs, rhs = (dd * d).sum(), (m * img).sum()
    assert abs(lhs - rhs) > 1e-3 * abs(lhs)


# ---------------------------------------------------------------------------
# P7: source reconstruction by time reversal equals the stored wavefield
# ---------------------------------------------------------------------------

def test_reconstruction_equals_stored_wavefield():
    vel = _small_model(seed=3, nz=24, nx=28)
    nt = 150
    kw = dict(dz=10.0, dx=10.0, dt=1e-3, nb=6)
    w = inputs.ricker(nt, 1e-3, fp=25)
    for src in ((2, 5), (12, 14)):  # on the ring, and in the interior
        fw = oracle.forward(vel, w, src, [], nt=nt, snaps=True, **kw)["snaps"]
        rc = oracle.reconstruct(vel, w, src, nt=nt, **kw)
        assert np.abs(rc - fw).max() <= 1e-10 * np.abs(fw).max()


def test_checkpoint_mode_is_bitwise_store_mode():
    vel = _small_model(seed=4)
    nz, nx = vel.shape
    nt = 97
    kw = dict(dz=10.0, dx=10.0, dt=1e-3, nb=5)
    w = inputs.ricker(nt, 1e-3, fp=25)
    d = np.random.default_rng(5).standard_normal((nt, nx))
    rec = [(1, i) for i in range(nx)]
    a = oracle.rtm_shot(vel, w, (2, 7), rec, d, **kw)
    for ck in (1, 7, 64, 200):
        b = oracle.rtm_shot(vel, w, (2, 7), rec, d, s_mode="checkpoint", ckpt=ck, **kw)
        assert np.array_equal(a, b)


# ---------------------------------------------------------------------------
# P8 / P9: imaging geometry and physics sanity on the two-layer survey
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def two_layer_case():
    sv = inputs.two_layer_shot_survey()
    sh = sv.shots[0]
    kw = dict(dz=sv.h, dx=sv.h, dt=sv.dt, nb=sv.nb, nt=sv.nt)
    dtrue = oracle.forward(sv.vel_true, sv.wavelet, sh.src, sh.rec, **kw)["traces"]
    dsm = oracle.forward(sv.vel_mig, sv.wavelet, sh.src, sh.rec, **kw)["traces"]
    data = dtrue - dsm
    img = oracle.rtm_shot(sv.vel_mig, sv.wavelet, sh.src, sh.rec, data, dz=sv.h, dx=sv.h,
                          dt=sv.dt, nb=sv.nb)
    return sv, data, img


def test_two_layer_image_mirror_symmetry(two_layer_case):
    sv, data, img = two_layer_case
    assert np.abs(img).max() > 0
    assert np.abs(img[:, 100:] - img[:, 100::-1]).max() <= 1e-12 * np.abs(img).max()
    # the data are mirror symmetric too (receivers on every column)
    assert np.abs(data - data[:, ::-1]).max() <= 1e-12 * np.abs(data).max()


def test_two_layer_image_peaks_at_interface(two_layer_case):
    """Away from the source, each column's |I| peaks next to the z = 500 m
    interface (row 50); the image sign is not pinned."""
    _, _, img = two_layer_case
    for c in list(range(25, 96, 5)) + list(range(105, 176, 5)):
        iz = int(np.argmax(np.abs(img[:, c])))
        assert 45 <= iz <= 54, (c, iz)


def test_migration_is_linear_in_data(two_layer_case):
    sv, data, img = two_layer_case
    sh = sv.shots[0]
    kw = dict(dz=sv.h, dx=sv.h, dt=sv.dt, nb=sv.nb)
    rng = np.random.default_rng(9)
    d2 = rng.standard_normal(data.shape) * np.abs(data).max()
    img2 = oracle.rtm_shot(sv.vel_mig, sv.wavelet, sh.src, sh.rec, d2, **kw)
    img3 = oracle.rtm_shot(sv.vel_mig, sv.wavelet, sh.src, sh.rec, 2 * data - 3 * d2, **kw)
    assert np.abs(img3 - (2 * img - 3 * img2)).max() <= 1e-11 * np.abs(img3).max()
    img0 = oracle.rtm_shot(sv.vel_mig, sv.wavelet, sh.src, sh.rec, np.zeros_like(data), **kw)
    assert not np.any(img0)


def test_stride_k_image_is_close_to_stride_1(two_layer_case):
    """Stride-4 imaging (sum over every 4th step times 4) stays within 1e-3 of the
    full sum on the 1 ms two-layer survey, and is not identical to it."""
    sv, data, img = two_layer_case
    sh = sv.shots[0]
    img4 = oracle.rtm_shot(sv.vel_mig, sv.wavelet, sh.src, sh.rec, data, dz=sv.h, dx=sv.h,
                           dt=sv.dt, nb=sv.nb, stride=4)
    e = oracle.rel_l2(img4, img)
    assert 0 < e < 1e-3


# ---------------------------------------------------------------------------
# P12: 16-bit snapshot emulation (round-to-nearest-even, power-of-two scale)
# ---------------------------------------------------------------------------

def _bf16_rne_from_f32_bits(x32):
    """Independent bf16 RNE on float32 bit patterns (finite inputs)."""
    u = x32.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def test_round_fp16_matches_ieee_binary16_cast():
    rng = np.random.default_rng(11)
    x = np.concatenate([
        rng.standard_normal(4000) * 10.0 ** rng.integers(-9, 5, 4000),
        # exact ties between adjacent binary16 values
        (np.arange(1, 2000) + 0.5) * 2.0**-24,
        1.0 + (2 * np.arange(0, 1000) + 1) * 2.0**-11,
    ])
    x = x[np.abs(x) < 60000]
    ours = np.array([oracle.round_fp16(v) for v in x])
    ref = x.astype(np.float16).astype(np.float64)
    assert np.array_equal(ours, ref)


def test_round_bf16_matches_bit_level_rne():
    rng = np.random.default_rng(12)
    x32 = (rng.standard_normal(5000) * 10.0 ** rng.integers(-30, 30, 5000)).astype(np.float32)
    ties = np.array([1.0 + 2.0**-8, 1.0 + 3 * 2.0**-8, -(1.0 + 5 * 2.0**-8)], dtype=np.float32)
    x32 = np.concatenate([x32, ties])
    ours = np.array([oracle.round_bf16(float(v)) for v in x32])
    ref = _bf16_rne_from_f32_bits(x32).astype(np.float64)
    assert np.array_equal(ours, ref)


def test_snapshot_scale_rule():
    rng = np.random.default_rng(13)
    for m in np.concatenate([10.0 ** rng.uniform(-20, 20, 500), [0.5, 1.0, 2.0**-3, 3.0]]):
        s = oracle.snapshot_scale(m)
        assert 2.0**14 <= m * s < 2.0**15
        assert math.frexp(s)[0] == 0.5  # power of two
    assert oracle.snapshot_scale(0.0) == 1.0


def test_quantized_imaging_error_ordering(two_layer_case):
    """16-bit storage perturbs the image at the format's precision: fp16
    (11 significant bits) less than bf16 (8 bits), both far above zero."""
    sv, data, _ = two_layer_case
    sh = sv.shots[0]
    kw = dict(dz=sv.h, dx=sv.h, dt=sv.dt, nb=sv.nb, stride=4)
    ref = oracle.rtm_shot(sv.vel_mig, sv.wavelet, sh.src, sh.rec, data, **kw)
    e16 = oracle.rel_l2(oracle.rtm_shot(sv.vel_mig, sv.wavelet, sh.src, sh.rec, data, quant="fp16",
                                        **kw), ref)
    eb16 = oracle.rel_l2(oracle.rtm_shot(sv.vel_mig, sv.wavelet, sh.src, sh.rec, data, quant="bf16",
                                         **kw), ref)
    assert 1e-7 < e16 < 1e-3
    assert 1e-6 < eb16 < 1e-2
    assert eb16 > 2 * e16


# ---------------------------------------------------------------------------
# Ensemble statistics and stacking (Sec. 2.3; Fig. 2 caption)
# ---------------------------------------------------------------------------

def test_ensemble_stats_closed_form():
    # samples a + b k, k = 0..n-1: mean a + b (n-1)/2, sample var b^2 n (n+1) / 12
    n = 9
    a = np.array([[1.0, -2.0], [0.5, 3.0]])
    b = np.array([[2.0, 0.25], [-1.0, 4.0]])
    x = np.stack([a + b * k for k in range(n)])
    mean, std = oracle.ensemble_stats(x)
    assert np.allclose(mean, a + b * (n - 1) / 2, rtol=1e-14, atol=0)
    assert np.allclose(std, np.abs(b) * math.sqrt(n * (n + 1) / 12), rtol=1e-13, atol=0)


def test_windowed_stats_and_stack_placement():
    nz, nx = 3, 10
    imgs = [np.full((nz, 4), 1.0), np.full((nz, 5), 3.0), np.full((nz, 3), 5.0)]
    wins = [(0, 4), (2, 5), (6, 3)]
    st = oracle.stack(imgs, wins, nx)
    assert np.array_equal(st[0], [1, 1, 4, 4, 3, 3, 8, 5, 5, 0])
    mean, std, cnt = oracle.windowed_stats(imgs, wins, nz, nx)
    assert np.array_equal(cnt[0], [1, 1, 2, 2, 1, 1, 2, 1, 1, 0])
    assert np.allclose(mean[0], [1, 1, 2, 2, 3, 3, 4, 5, 5, 0])
    assert np.allclose(std[0], [0, 0, math.sqrt(2), math.sqrt(2), 0, 0, math.sqrt(2), 0, 0, 0])


# ---------------------------------------------------------------------------
# Stage-3 maps (Sec. 2.3, Eq. 6 and Eq. 7) and the post-stack filter (Sec. 3)
# ---------------------------------------------------------------------------

def test_confidence_index_by_hand():
    """Eq. 6 with extremes over pixels of count >= min_count: std 1, 2, 3 are
    counted (s_min 1, s_max 3) and the std of 10 at count 1 is not, so the map
    is (3 - s) / 2 = 1, 1/2, 0 and 0 at the excluded pixel.  Extremes over all
    pixels would give s_max 10 (1, 8/9, 7/9); a swapped numerator (s - s_min)
    gives 0, 1/2, 1."""
    std = np.array([[1.0, 2.0], [3.0, 10.0]])
    cnt = np.array([[3, 2], [5, 1]])
    np.testing.assert_array_equal(oracle.confidence_index(std, cnt, min_count=2),
                                  [[1.0, 0.5], [0.0, 0.0]])
    # min_count 3 drops the pixel of count 2 as well: extremes 1 and 3 still
    np.testing.assert_array_equal(oracle.confidence_index(std, cnt, min_count=3),
                                  [[1.0, 0.0], [0.0, 0.0]])
    # without counts every pixel takes part: (10 - s) / 9
    np.testing.assert_allclose(oracle.confidence_index(std), [[1.0, 8 / 9], [7 / 9, 0.0]], rtol=1e-15)


def test_confidence_index_degenerate_cases():
    """s_max == s_min gives 0 everywhere (no spread to rank), as does a map
    with no pixel at min_count; the result does not depend on the std of the
    excluded pixels."""
    std = np.full((3, 4), 2.5)
    cnt = np.full((3, 4), 4)
    assert not oracle.confidence_index(std, cnt).any()
    assert not oracle.confidence_index(np.arange(12.0).reshape(3, 4), np.ones((3, 4), int)).any()
    a = np.array([[0.5, 1.5, 9.0]])
    b = np.array([[0.5, 1.5, -7.0]])
    c = np.array([[2, 2, 0]])
    np.testing.assert_array_equal(oracle.confidence_index(a, c), oracle.confidence_index(b, c))
    np.testing.assert_array_equal(oracle.confidence_index(a, c), [[1.0, 0.0, 0.0]])


def test_ratio_map_by_hand():
    """Eq. 7: std / mean, keeping the sign of the mean, and 0 where
    |mean| <= eps (the rule is strict: |mean| == eps gives 0)."""
    std = np.array([1.0, 2.0, 3.0, 4.0, 5.0, 6.0])
    mean = np.array([2.0, -4.0, 1e-4, 0.0, 1e-3, -2e-3])
    np.testing.assert_array_equal(oracle.ratio_map(std, mean, eps=1e-3),
                                  [0.5, -0.5, 0.0, 0.0, 0.0, -3000.0])
    # eps 0: only an exact zero mean is masked
    np.testing.assert_array_equal(oracle.ratio_map(std[:4], mean[:4], eps=0.0),
                                  [0.5, -0.5, 3.0 / 1e-4, 0.0])


def test_laplacian_filter_sign_and_edges():
    """The filter is minus the 8th-order Laplacian: on z^2 (z = i dz) the
    interior value is -2, on z^2 + x^2 it is -4.  Outside the image the field
    is zero, so at a corner of a constant image of 1 only the inner
    neighbours count: L = a0 (1/dz^2 + 1/dx^2) + (a1 + a2 + a3 + a4)(1/dz^2 +
    1/dx^2) = (a0 / 2)(1/dz^2 + 1/dx^2), since a0 + 2 sum a_k = 0, and the
    filter gives +(205 / 144)(1/dz^2 + 1/dx^2)."""
    nz, nx, dz, dx = 20, 23, 10.0, 12.5
    z = np.arange(nz)[:, None] * dz
    x = np.arange(nx)[None, :] * dx
    inner = (slice(4, nz - 4), slice(4, nx - 4))
    f = oracle.laplacian_filter(np.broadcast_to(z * z, (nz, nx)).copy(), dz, dx)
    np.testing.assert_allclose(f[inner], -2.0, rtol=1e-12)
    f = oracle.laplacian_filter(z * z + x * x, dz, dx)
    np.testing.assert_allclose(f[inner], -4.0, rtol=1e-12)
    f = oracle.laplacian_filter(np.ones((nz, nx)), dz, dx)
    corner = 205.0 / 144.0 * (1 / dz**2 + 1 / dx**2)
    for iz, ix in ((0, 0), (0, nx - 1), (nz - 1, 0), (nz - 1, nx - 1)):
        assert f[iz, ix] == pytest.approx(corner, rel=1e-13)
    assert np.abs(f[inner]).max() < 1e-15 * corner
