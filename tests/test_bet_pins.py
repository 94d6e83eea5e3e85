"""Pins of the Stage-1 oracle (oracle/bet.py, bet_oracle.c) against the
definitions it follows, worked values and known properties.  CPU only.

  - splitmix64: the published first outputs for seed 1234567;
  - Godunov upwind Eikonal update: a 3 x 3 grid worked by hand, exactness
    along a single row, first-order convergence to r / v in a homogeneous
    medium, fast marching equal to an independent fixed-point iteration of
    the same discrete equations, single and double precision agreeing;
  - Voronoi model: a small case worked by hand, ties to the lowest index;
  - reversible-jump chains (Sec. 2.1): with a flat likelihood the sampler
    must return the prior (number of cells uniform on [k_min, k_max], nuclei
    uniform in the domain); invalid proposals leave the state unchanged; the
    pooled statistics equal the mean and std of the recorded models.
"""
import math

import numpy as np
import pytest

from oracle import bet


def test_splitmix64_published_outputs():
    # first five outputs of splitmix64 seeded with 1234567 (reference sequence)
    want = [6457827717110365317, 3203168211198807973, 9817491932198370423, 4593380528125082431,
            16408922859458223821]
    assert [bet.sm64_at(1234567, n) for n in range(5)] == want


def test_eikonal_three_by_three_by_hand():
    # h = 1, s = 1, source at the corner (0, 0):
    #   axis neighbours 1, 2;  (1,1): a = b = 1 -> (2 + sqrt 2) / 2
    #   (1,2): a = T(1,1) = 1.70711, b = T(0,2) = 2, d = 0.29289 < 1
    #          -> (a + b + sqrt(2 - d^2)) / 2
    #   (2,2): a = b = T(1,2) -> (2 T(1,2) + sqrt 2) / 2
    T = bet.eikonal(np.ones((3, 3)), 1.0, (0, 0))
    t11 = (2.0 + math.sqrt(2.0)) / 2.0
    d = 2.0 - t11
    t12 = (t11 + 2.0 + math.sqrt(2.0 - d * d)) / 2.0
    t22 = (2.0 * t12 + math.sqrt(2.0)) / 2.0
    want = np.array([[0.0, 1.0, 2.0], [1.0, t11, t12], [2.0, t12, t22]])
    np.testing.assert_allclose(T, want, rtol=0, atol=1e-14)
    # source in the centre: axis neighbours h s, corners (2 + sqrt 2) / 2
    T = bet.eikonal(np.ones((3, 3)), 1.0, (1, 1))
    np.testing.assert_allclose(T, [[t11, 1, t11], [1, 0, 1], [t11, 1, t11]], atol=1e-14)


def test_eikonal_single_row_is_exact():
    # one row: every update is one-sided, T(j+1) = T(j) + h s(j+1)
    rng = np.random.default_rng(1)
    s = rng.uniform(1 / 5000, 1 / 1500, size=(1, 60))
    T = bet.eikonal(s, 25.0, (0, 17))
    want = np.zeros(60)
    for j in range(18, 60):
        want[j] = want[j - 1] + 25.0 * s[0, j]
    for j in range(16, -1, -1):
        want[j] = want[j + 1] + 25.0 * s[0, j]
    np.testing.assert_allclose(T[0], want, rtol=1e-14, atol=0)


def test_eikonal_first_order_convergence():
    # homogeneous 2000 m/s, point source: the error at a fixed point (1 km
    # down, 1.5 km across) shrinks about linearly with h
    errs = []
    for h in (50.0, 25.0, 12.5):
        n = int(round(2000.0 / h)) + 1
        T = bet.eikonal(np.full((n, n), 1 / 2000.0), h, (0, 0))
        i, j = int(round(1000.0 / h)), int(round(1500.0 / h))
        exact = math.hypot(1000.0, 1500.0) / 2000.0
        errs.append(T[i, j] - exact)
    assert all(e > 0 for e in errs)  # the first-order scheme overestimates off the axes
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 1.4 < r1 < 2.5 and 1.4 < r2 < 2.5, (errs, r1, r2)
    assert errs[-1] / (math.hypot(1000.0, 1500.0) / 2000.0) < 0.02


def _fixed_point(s, h, src):
    """Independent solver: Jacobi iteration of the Godunov update over all
    neighbours until nothing changes (same discrete equations, another
    algorithm)."""
    nz, nx = s.shape
    T = np.full((nz, nx), np.inf)
    T[src] = 0.0
    while True:
        P = np.pad(T, 1, constant_values=np.inf)
        a = np.minimum(P[:-2, 1:-1], P[2:, 1:-1])
        b = np.minimum(P[1:-1, :-2], P[1:-1, 2:])
        lo, hi = np.minimum(a, b), np.maximum(a, b)
        sh = s * h
        with np.errstate(invalid="ignore"):
            d = hi - lo
            two = ((lo + hi) + np.sqrt((sh * sh + sh * sh) - d * d)) * 0.5
        new = np.where(~(d < sh), lo + sh, two)
        new[src] = 0.0
        new = np.minimum(T, new)
        if np.array_equal(new, T):
            return T
        T = new


@pytest.mark.parametrize("seed", [0, 1])
def test_fast_marching_equals_fixed_point(seed):
    rng = np.random.default_rng(seed)
    nz, nx, h = 23, 31, 40.0
    # piecewise-constant blocks with strong contrasts (a Voronoi model)
    zs, xs = rng.uniform(0, (nz - 1) * h, 9), rng.uniform(0, (nx - 1) * h, 9)
    vs = rng.uniform(1500, 5000, 9)
    s = 1.0 / vs[bet.voronoi(nz, nx, h, zs, xs)]
    src = (int(rng.integers(nz)), int(rng.integers(nx)))
    T = bet.eikonal(s, h, src)
    np.testing.assert_allclose(T, _fixed_point(s, h, src), rtol=1e-13, atol=0)
    # causality: every node but the source is larger than its smallest neighbour
    P = np.pad(T, 1, constant_values=np.inf)
    nb = np.minimum.reduce([P[:-2, 1:-1], P[2:, 1:-1], P[1:-1, :-2], P[1:-1, 2:]])
    mask = np.ones_like(T, bool)
    mask[src] = False
    assert np.all(T[mask] > nb[mask])


def test_fast_sweeping_single_precision():
    # the FP32 sweeping solver: the hand-worked 3 x 3 values, a single row
    # exactly, and agreement with FP64 fast marching to FP32 rounding on a
    # Voronoi model; a homogeneous grid converges in one pass plus a check
    T, passes = bet.eikonal(np.ones((3, 3), np.float32), 1.0, (0, 0), sweep=True)
    t11 = (2.0 + math.sqrt(2.0)) / 2.0
    assert T[0, 2] == 2.0 and abs(T[1, 1] - t11) < 1e-6 and passes == 1
    rng = np.random.default_rng(1)
    s1 = rng.uniform(1 / 5000, 1 / 1500, size=(1, 40)).astype(np.float32)
    T1, _ = bet.eikonal(s1, 25.0, (0, 7), sweep=True)
    want = np.zeros(40, np.float32)
    for j in range(8, 40):
        want[j] = want[j - 1] + np.float32(s1[0, j] * np.float32(25.0))
    for j in range(6, -1, -1):
        want[j] = want[j + 1] + np.float32(s1[0, j] * np.float32(25.0))
    np.testing.assert_array_equal(T1[0], want)
    nz, nx, h = 36, 171, 100.0
    zs, xs = rng.uniform(0, 3500, 25), rng.uniform(0, 17000, 25)
    vs = rng.uniform(1500, 4700, 25)
    s = 1.0 / vs[bet.voronoi(nz, nx, h, zs, xs)]
    Ts, passes = bet.eikonal(s.astype(np.float32), h, (3, 100), sweep=True)
    np.testing.assert_allclose(Ts, bet.eikonal(s, h, (3, 100)), rtol=2e-6, atol=1e-7)
    assert 2 <= passes < 20


def test_single_precision_variant_agrees():
    rng = np.random.default_rng(4)
    nz, nx, h = 36, 171, 100.0
    zs, xs = rng.uniform(0, 3500, 20), rng.uniform(0, 17000, 20)
    vs = rng.uniform(1500, 4700, 20)
    s = 1.0 / vs[bet.voronoi(nz, nx, h, zs, xs)]
    T64 = bet.eikonal(s, h, (0, 80))
    T32 = bet.eikonal(s.astype(np.float32), h, (0, 80), single=True)
    np.testing.assert_allclose(T32, T64, rtol=2e-6, atol=1e-7)


def test_voronoi_by_hand_and_ties():
    # nuclei at (z, x) = (0, 0) and (0, 30) on a 2 x 4 grid of h = 10: node
    # (0, 1) at x = 10 is 10 from the first and 20 from the second; node (0, 2)
    # at x = 20 is 20 and 10; node (1, 1) at (10, 10): d^2 = 200 and 500
    c = bet.voronoi(2, 4, 10.0, [0.0, 0.0], [0.0, 30.0])
    np.testing.assert_array_equal(c, [[0, 0, 1, 1], [0, 0, 1, 1]])
    # exact tie at x = 10 between nuclei at x = 0 and x = 20: lowest index wins
    c = bet.voronoi(1, 3, 10.0, [0.0, 0.0], [20.0, 0.0])
    np.testing.assert_array_equal(c, [[1, 0, 0]])


def _flat_setup(k_min=2, k_max=8):
    cfg = bet.BetConfig(nz=5, nx=7, h=100.0, chains=8, k_min=k_min, k_max=k_max, k_init=4,
                        sigma=1e9, move_dz=150.0, move_dx=200.0, seed=77, burn_in=200, thin=5)
    srcs, recs = [(0, 0)], [(0, 6), (4, 3)]
    return cfg, srcs, recs, np.zeros((1, 2), np.float32)


def test_flat_likelihood_samples_the_prior():
    cfg, srcs, recs, tt = _flat_setup()
    iters = 6000
    out = bet.run(cfg, srcs, recs, tt, iters, log=True)
    log = out["log"]
    # every valid proposal is accepted when the likelihood is flat
    valid = log >= 0
    assert np.all(log[valid] > 0)
    # number of cells: uniform on [k_min, k_max] under the prior; rebuild the
    # chain's k from the accept log (births +1, deaths -1)
    k = np.full(cfg.chains, cfg.k_init)
    hist = np.zeros(cfg.k_max + 1)
    for t in range(iters):
        k = k + (log[t] == 1) - (log[t] == 2)
        if t >= cfg.burn_in:
            np.add.at(hist, k, 1)
    np.testing.assert_array_equal(k, out["k"])
    p = hist[cfg.k_min:] / hist.sum()
    expect = 1.0 / (cfg.k_max - cfg.k_min + 1)
    assert np.all(np.abs(p - expect) < 0.25 * expect), p
    # nuclei positions uniform over the domain: final positions' means near the centre
    zs = np.concatenate([out["z"][c, :out["k"][c]] for c in range(cfg.chains)])
    xs = np.concatenate([out["x"][c, :out["k"][c]] for c in range(cfg.chains)])
    assert np.all((zs >= 0) & (zs <= 400) & (xs >= 0) & (xs <= 600))


def test_invalid_proposals_leave_the_state():
    cfg, srcs, recs, tt = _flat_setup(k_min=4, k_max=4)
    cfg.p_birth, cfg.p_death = 0.5, 0.5  # births at k_max and deaths at k_min only
    cfg.k_init = 4
    a = bet.run(cfg, srcs, recs, tt, 0)
    b = bet.run(cfg, srcs, recs, tt, 50, log=True)
    assert np.all(b["log"] == -1)
    for key in ("k", "z", "x", "v", "misfit"):
        np.testing.assert_array_equal(a[key], b[key])


def test_pooled_statistics_equal_recorded_models():
    cfg, srcs, recs, tt = _flat_setup()
    cfg.sigma = 0.05
    tt = bet.travel_times(np.full((cfg.nz, cfg.nx), 2500.0), cfg.h, srcs, recs).astype(np.float32)
    iters = 30
    cfg.burn_in, cfg.thin = iters - 1, 1  # exactly one sample: the final state of each chain
    out = bet.run(cfg, srcs, recs, tt, iters)
    models = np.stack([bet.model_velocity(cfg, out["k"][c], out["z"][c], out["x"][c], out["v"][c])
                       for c in range(cfg.chains)])
    assert out["count"] == cfg.chains
    np.testing.assert_allclose(out["mean"], models.mean(axis=0), rtol=1e-13)
    np.testing.assert_allclose(out["std"], models.std(axis=0, ddof=1), rtol=1e-10, atol=1e-9)


def test_informative_data_lowers_the_misfit():
    nz, nx, h = 12, 40, 100.0
    true = np.where(np.arange(nz)[:, None] < 5, 1800.0, 3200.0) * np.ones((1, nx))
    srcs = [(0, j) for j in range(0, nx, 8)]
    recs = [(0, j) for j in range(nx)]
    tt = bet.travel_times(true, h, srcs, recs, single=True).astype(np.float32)
    cfg = bet.BetConfig(nz=nz, nx=nx, h=h, chains=4, k_min=2, k_max=20, k_init=6, sigma=0.01,
                        move_dz=200.0, move_dx=600.0, seed=5, burn_in=10 ** 9)
    first = bet.run(cfg, srcs, recs, tt, 0)["misfit"]
    later = bet.run(cfg, srcs, recs, tt, 400)["misfit"]
    assert np.all(later <= first) and np.median(later) < 0.2 * np.median(first)


def _chain_setup():
    nz, nx, h = 12, 40, 100.0
    true = np.where(np.arange(nz)[:, None] < 5, 1800.0, 3200.0) * np.ones((1, nx))
    srcs = [(0, j) for j in range(0, nx, 8)]
    recs = [(0, j) for j in range(nx)]
    tt = bet.travel_times(true, h, srcs, recs, single=False).astype(np.float32)
    return nz, nx, h, srcs, recs, tt


def _one_chain(single, chain, seed, iters):
    nz, nx, h, srcs, recs, tt = _chain_setup()
    cfg = bet.BetConfig(nz=nz, nx=nx, h=h, chains=1, chain0=chain, k_min=2, k_max=20, k_init=6,
                        sigma=0.004, move_dz=200.0, move_dx=600.0, seed=seed, burn_in=300, thin=4,
                        single=single)
    return bet.run(cfg, srcs, recs, tt, iters, log=True)


def _layer_means(runs):
    """Per-chain pooled mean velocity over the rows above and below the
    interface (rows 0-4 and 6-11), and the per-chain final k."""
    m = np.stack([r["mean"] for r in runs])
    return m[:, :5].mean(axis=(1, 2)), m[:, 6:].mean(axis=(1, 2)), np.array([r["k"][0] for r in runs], float)


def test_fast_sweeping_chains_sample_the_fast_marching_posterior():
    """Sec. 2.1 and Sec. 3 compute first arrivals with fast marching (FaATSO);
    the sampler's accept decisions use single-precision fast sweeping, which
    solves the same discrete Godunov equations.  Chains driven by each
    (common random numbers) must take the same accept decisions, and chains
    of double-precision fast marching with other random numbers must give
    the same posterior means (pooled velocity above and below the interface,
    number of cells) within Monte Carlo error, estimated from the spread of
    independent chains."""
    C, iters = 8, 1200
    fsm = [_one_chain(True, c, 11, iters) for c in range(C)]
    fmm = [_one_chain(False, c, 11, iters) for c in range(C)]
    agree = np.mean([(a["log"] == b["log"]).mean() for a, b in zip(fsm, fmm)])
    assert agree >= 0.99, agree
    other = [_one_chain(False, c, 12, iters) for c in range(C)]
    for a, b in zip(_layer_means(fsm), _layer_means(other)):
        se = np.sqrt(a.var(ddof=1) / C + b.var(ddof=1) / C)
        assert abs(a.mean() - b.mean()) <= 4.0 * se, (a.mean(), b.mean(), se)
    # the data resolve the two layers: the sampled means sit near 1800 / 3200 m/s
    up, lo, _ = _layer_means(fsm)
    assert 1700 < up.mean() < 2200 and 3000 < lo.mean() < 3500
