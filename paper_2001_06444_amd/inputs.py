"""Seeded synthetic inputs: velocity models, wavelet, acquisition geometry.

This module holds no step of the migration itself; it only builds the arrays
a migration consumes.  Both the HIP path's tests/benchmark and the CPU
oracle's tests draw their inputs from here.

The paper's workloads are a two-layer model (Sec. 4.1) and the Marmousi2
benchmark (Sec. 4.2).  Marmousi2 is not available, so a faulted-layer model
of the same 3.5 km x 17 km extent stands in for it; the velocity samples of
the uncertainty study (Sec. 2.1, produced by Bayesian tomography there) are
stood in for by smoothed models times a seeded Gaussian random field.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# ---------------------------------------------------------------------------
# Wavelet
# ---------------------------------------------------------------------------


def ricker(nt: int, dt: float, fp: float = 15.0, t0: float | None = None) -> np.ndarray:
    """Ricker wavelet w(n dt) = (1 - 2 pi^2 fp^2 tau^2) exp(-pi^2 fp^2 tau^2), tau = t - t0.

    Amplitude 1, delay t0 = 1.5 / fp by default (so w(0) is ~1e-8).
    """
    if t0 is None:
        t0 = 1.5 / fp
    t = np.arange(nt, dtype=np.float64) * dt - t0
    a = (math.pi * fp * t) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


# ---------------------------------------------------------------------------
# Velocity models
# ---------------------------------------------------------------------------


def two_layer(nz: int, nx: int, dz: float, v_top: float = 1500.0, v_bot: float = 2500.0,
              z_interface: float = 500.0) -> np.ndarray:
    """Two constant layers; the row at exactly z_interface takes the lower velocity."""
    z = np.arange(nz) * dz
    col = np.where(z < z_interface - 1e-9, v_top, v_bot)
    return np.repeat(col[:, None], nx, axis=1).astype(np.float64)


def smooth_slowness(vel: np.ndarray, sigma_m: float, dz: float, dx: float) -> np.ndarray:
    """Gaussian smoothing of the slowness (1/v), sigma in metres, 4-sigma
    truncation, edge-replicated borders; returns velocity."""
    from scipy.ndimage import gaussian_filter

    s = 1.0 / np.asarray(vel, dtype=np.float64)
    sm = gaussian_filter(s, sigma=(sigma_m / dz, sigma_m / dx), mode="nearest", truncate=4.0)
    return 1.0 / sm


def faulted_layers(nz: int = 351, nx: int = 1701, h: float = 10.0, seed: int = 6444,
                   water_rows: int = 40, n_layers: int = 20, v_first: float = 1600.0,
                   v_last: float = 4700.0, n_faults: int = 3) -> np.ndarray:
    """Layered model with planar normal faults (Marmousi2-sized stand-in).

    Rows [0, water_rows) are 1500 m/s water.  n_layers flat layers of equal
    thickness fill the rest (boundaries at round(water_rows + (nz-water_rows) j
    / n_layers)), velocities linearly spaced from v_first to v_last.  Each fault
    has a surface trace x_f ~ U(0.15, 0.85) * width, dip ~ U(50, 70) degrees,
    dip direction +-1 with equal odds and throw ~ U(50, 200) m; on the hanging
    wall the layer index is looked up at depth z - throw.  Faults act only
    below the water.
    """
    rng = np.random.default_rng(seed)
    width = nx * h
    faults = []
    for _ in range(n_faults):
        xf = rng.uniform(0.15, 0.85) * width
        dip = math.radians(rng.uniform(50.0, 70.0))
        sgn = 1.0 if rng.uniform() < 0.5 else -1.0
        throw = rng.uniform(50.0, 200.0)
        faults.append((xf, dip, sgn, throw))
    bounds = np.round(water_rows + (nz - water_rows) * np.arange(n_layers + 1) / n_layers)
    vels = np.linspace(v_first, v_last, n_layers)
    z = (np.arange(nz) * h)[:, None] * np.ones((1, nx))
    x = (np.arange(nx) * h)[None, :] * np.ones((nz, 1))
    zeff = z.copy()
    for xf, dip, sgn, throw in faults:
        xplane = xf + sgn * z / math.tan(dip)
        hanging = (x - xplane) * sgn > 0
        zeff = np.where(hanging, zeff - throw, zeff)
    row_eff = zeff / h
    idx = np.searchsorted(bounds, row_eff, side="right") - 1
    idx = np.clip(idx, 0, n_layers - 1)
    v = vels[idx]
    v[:water_rows, :] = 1500.0
    return v.astype(np.float64)


def grf(r: int, nz: int = 351, nx: int = 1701, h: float = 10.0, ell: float = 200.0,
        pad_m: float = 600.0) -> np.ndarray:
    """Zero-mean, unit-std Gaussian random field with covariance exp(-d^2 / (2 ell^2)).

    White noise from default_rng(1000 + r) on the grid padded by pad_m on all
    sides, filtered in the Fourier domain by a Gaussian of std ell / sqrt(2),
    cropped, then normalised empirically.
    """
    p = int(round(pad_m / h))
    rng = np.random.default_rng(1000 + r)
    w = rng.standard_normal((nz + 2 * p, nx + 2 * p))
    sig = ell / math.sqrt(2.0)
    kz = np.fft.fftfreq(w.shape[0], d=h)
    kx = np.fft.rfftfreq(w.shape[1], d=h)
    tf = np.exp(-2.0 * math.pi ** 2 * sig ** 2 * (kz[:, None] ** 2 + kx[None, :] ** 2))
    f = np.fft.irfft2(np.fft.rfft2(w) * tf, s=w.shape)[p:p + nz, p:p + nx]
    f = f - f.mean()
    return f / f.std()


def realization(r: int, base: np.ndarray, h: float = 10.0, rel_std: float = 0.05,
                smooth_sigma_m: float = 40.0) -> np.ndarray:
    """Velocity sample r: smooth(base) * (1 + rel_std * grf_r)."""
    nz, nx = base.shape
    return smooth_slowness(base, smooth_sigma_m, h, h) * (1.0 + rel_std * grf(r, nz, nx, h))


# ---------------------------------------------------------------------------
# Geometry
# ---------------------------------------------------------------------------


def window_for(ix_src: int, width: int, nx_model: int) -> int:
    """Left column of an aperture window of `width` centred on the source, clamped."""
    return int(min(max(ix_src - width // 2, 0), nx_model - width))


def surface_receivers(iz: int, ix0: int, width: int) -> np.ndarray:
    """One receiver per column of the window at row iz, model coordinates [n][2]."""
    return np.stack([np.full(width, iz), np.arange(ix0, ix0 + width)], axis=1).astype(np.int32)


# ---------------------------------------------------------------------------
# Workload definitions
# ---------------------------------------------------------------------------


@dataclasses.dataclass
class Shot:
    src: tuple            # (iz, ix) model coordinates
    ix0: int              # aperture window start column
    width: int            # aperture window width (columns)
    rec: np.ndarray       # [nrec][2] model coordinates


@dataclasses.dataclass
class Survey:
    name: str
    nz: int
    nx: int
    h: float
    dt: float
    nt: int
    nb: int
    fp: float
    vel_true: np.ndarray
    vel_mig: np.ndarray
    shots: list
    stride: int = 1

    @property
    def wavelet(self):
        return ricker(self.nt, self.dt, self.fp)


def two_layer_shot_survey(nt: int = 1000) -> Survey:
    """Single-shot two-layer survey: 101 x 201 at 10 m, 1500 over 2500 m/s at
    z = 500 m, 20-cell sponge, Ricker 15 Hz at (z, x) = (10 m, 1000 m),
    201 receivers at z = 10 m, dt = 1 ms."""
    nz, nx, h = 101, 201, 10.0
    v = two_layer(nz, nx, h)
    vs = smooth_slowness(v, 40.0, h, h)
    shot = Shot(src=(1, 100), ix0=0, width=nx, rec=surface_receivers(1, 0, nx))
    return Survey("two_layer_101x201", nz, nx, h, 1e-3, nt, 20, 15.0, v, vs, [shot])


def faulted_survey(n_shots: int = 100, nt: int = 4000, nz: int = 351, nx: int = 1701) -> Survey:
    """Realistic-size survey: faulted-layer model 351 x 1701 at 10 m (seed 6444),
    50-cell sponge, shots every 170 m at ix = 8 + 17k, a receiver on every
    column, dt = 1 ms."""
    h = 10.0
    v = faulted_layers(nz, nx, h)
    vs = smooth_slowness(v, 40.0, h, h)
    shots = []
    for k in range(n_shots):
        ix = 8 + 17 * k
        if ix >= nx:
            break
        shots.append(Shot(src=(1, ix), ix0=0, width=nx, rec=surface_receivers(1, 0, nx)))
    return Survey(f"faulted_{nz}x{nx}", nz, nx, h, 1e-3, nt, 50, 15.0, v, vs, shots)


def ensemble_shots(n_shots: int = 16, nx: int = 1701, seed: int = 3) -> list:
    """Shots at ix = 53 + 106k with aperture widths ~ U{401..1201} drawn once
    per shot index (shared by all realizations)."""
    rng = np.random.default_rng(seed)
    widths = rng.integers(401, 1202, size=n_shots)
    shots = []
    for k in range(n_shots):
        ix = 53 + 106 * k
        w = int(widths[k])
        ix0 = window_for(ix, w, nx)
        shots.append(Shot(src=(1, ix), ix0=ix0, width=w, rec=surface_receivers(1, ix0, w)))
    return shots


def ensemble_base(nz: int = 351, nx: int = 1701, h: float = 10.0) -> np.ndarray:
    """Base law of the ensemble study: 1500 over 2500 m/s at z = 500 m."""
    return two_layer(nz, nx, h)


@dataclasses.dataclass
class StreamJob:
    arrival: float      # seconds since stream start
    realization: int
    src: tuple
    ix0: int
    width: int
    nt: int
    dtype: str          # "fp32" or "bf16"


def poisson_stream(n_jobs: int, rate: float = 20.0, seed: int = 5, n_real: int = 256,
                   nx: int = 1701, h: float = 10.0) -> list:
    """Stream of RTM jobs: exponential inter-arrivals (mean 1/rate), realization
    ~ U{0..n_real-1}, source x ~ U(0, 17 km), width ~ U{301..1701}, nt ~
    U{2000..4000}, snapshot dtype fp32 or bf16 with equal odds."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n_jobs))
    jobs = []
    for j in range(n_jobs):
        r = int(rng.integers(0, n_real))
        xs = rng.uniform(0.0, nx * h)
        ix = int(min(round(xs / h), nx - 1))
        w = int(rng.integers(301, 1702))
        nt = int(rng.integers(2000, 4001))
        dt_ = "bf16" if rng.uniform() < 0.5 else "fp32"
        jobs.append(StreamJob(float(t[j]), r, (1, ix), window_for(ix, w, nx), w, nt, dt_))
    return jobs


# ---------------------------------------------------------------------------
# Arrays for the compression stage (Sec. 4.2 compresses velocity samples,
# migrated images and seismograms of the Marmousi2 study; these stand in)
# ---------------------------------------------------------------------------
def velocity_bank(n: int, nz: int = 351, nx: int = 1701, h: float = 10.0) -> np.ndarray:
    """n velocity samples [n][nz][nx] float32: realizations 0..n-1 of the
    smoothed faulted-layer model times (1 + 0.05 GRF)."""
    base = faulted_layers(nz, nx, h)
    return np.stack([realization(r, base, h) for r in range(n)]).astype(np.float32)


def _image_clean(nz: int, nx: int, h: float, fp: float, v_ref: float) -> np.ndarray:
    v = faulted_layers(nz, nx, h)
    refl = np.zeros((nz, nx))
    refl[1:] = np.diff(np.log(v), axis=0)
    n = int(round(2.0 * v_ref / fp / h))
    zz = (np.arange(-n, n + 1) * h) / v_ref
    a = (math.pi * fp * zz) ** 2
    pulse = (1.0 - 2.0 * a) * np.exp(-a)
    img = np.apply_along_axis(lambda c: np.convolve(c, pulse, mode="same"), 0, refl)
    img /= np.abs(img).max()
    zc, xc = np.mgrid[0:nz, 0:nx]
    return img + 0.1 * np.exp(-((zc - 20.0) ** 2) / (2 * 30.0 ** 2)) * np.cos(2 * math.pi * xc / 400.0)


def image_like(seed: int = 0, nz: int = 351, nx: int = 1701, h: float = 10.0, fp: float = 15.0,
               v_ref: float = 2500.0, noise: float = 0.02) -> np.ndarray:
    """Stand-in for a migrated image [nz][nx] float32, peak amplitude about 1.

    The faulted-layer model's reflectivity (relative contrast of log velocity
    between adjacent rows) convolved along depth with a Ricker pulse whose
    depth wavelength is v_ref / fp, a smooth shallow background like the
    low-frequency artefacts of an unfiltered stack, and white noise
    (default_rng(seed)) of `noise` times the reflectivity peak."""
    img = _image_clean(nz, nx, h, fp, v_ref)
    return (img + noise * np.random.default_rng(seed).standard_normal((nz, nx))).astype(np.float32)


def image_bank(n: int, nz: int = 351, nx: int = 1701, h: float = 10.0) -> np.ndarray:
    """n images [n][nz][nx] float32: image_like(s) for s = 0..n-1."""
    clean = _image_clean(nz, nx, h, 15.0, 2500.0)
    return np.stack([(clean + 0.02 * np.random.default_rng(s).standard_normal((nz, nx)))
                     for s in range(n)]).astype(np.float32)


def seismogram_like(seed: int = 0, nt: int = 4000, nrec: int = 1701, dt: float = 1e-3,
                    h: float = 10.0, fp: float = 15.0, noise: float = 1e-3) -> np.ndarray:
    """Stand-in for a shot record [nt][nrec] float32: a direct arrival and six
    reflection hyperbolas t(x) = sqrt(t0^2 + (x - xs)^2 / v^2) carrying a
    Ricker pulse with 1/sqrt(t) spreading, source position, t0 and v drawn from
    default_rng(seed), plus white noise of `noise` times the peak."""
    rng = np.random.default_rng(seed)
    xs = rng.uniform(0.0, nrec * h)
    x = np.arange(nrec) * h
    t = np.arange(nt)[:, None] * dt
    events = [(0.0, 1500.0, 1.0)]
    for k in range(6):
        events.append((rng.uniform(0.3 + 0.5 * k, 0.6 + 0.5 * k), rng.uniform(1600.0, 3500.0),
                       rng.uniform(0.1, 0.4) * (-1.0 if rng.uniform() < 0.3 else 1.0)))
    rec = np.zeros((nt, nrec))
    t_shift = 1.5 / fp
    for t0, vel, amp in events:
        tt = np.sqrt(t0 ** 2 + ((x - xs) / vel) ** 2)[None, :] + t_shift
        a = (math.pi * fp * (t - tt)) ** 2
        rec += amp * (1.0 - 2.0 * a) * np.exp(-a) / np.sqrt(np.maximum(tt, 0.05))
    rec /= np.abs(rec).max()
    rec += noise * rng.standard_normal((nt, nrec))
    return rec.astype(np.float32)


def seismogram_bank(n: int, nt: int = 4000, nrec: int = 1701) -> np.ndarray:
    """n shot records [n][nt][nrec] float32: seismogram_like(s) for s = 0..n-1."""
    return np.stack([seismogram_like(s, nt, nrec) for s in range(n)])


# ---------------------------------------------------------------------------
# Stage 1: travel-time tomography (Sec. 2.1; Sec. 4.2 uses 34 travel-time
# panels of Marmousi2, stood in for by the faulted-layer model)
# ---------------------------------------------------------------------------
def bet_true_model(nz: int = 36, nx: int = 171, h: float = 100.0) -> np.ndarray:
    """True velocity of the travel-time problem: the faulted-layer model
    (351 x 1701 at 10 m) sampled every (h / 10)-th node, h = 100 m (36 x 171)
    or 50 m (71 x 341), top-left nz x nx."""
    step = {100.0: 10, 50.0: 5}.get(float(h))
    if step is None or nz > 350 // step + 1 or nx > 1700 // step + 1:
        raise ValueError("the coarse model is the 10 m faulted model sampled at 100 m (at most 36 x 171) "
                         "or 50 m (at most 71 x 341)")
    return np.ascontiguousarray(faulted_layers()[::step, ::step][:nz, :nx]).astype(np.float64)


def bet_problem(chains: int = 64, h: float = 100.0) -> dict:
    """Stage-1 benchmark problem on the 3.5 km x 17 km section: 36 x 171
    nodes at 100 m (or 71 x 341 at 50 m), 34 surface sources every 500 m
    (x = 200 m + 500 m k), a receiver at every surface node, and the
    sampler's prior and proposal settings."""
    step = {100.0: 10, 50.0: 5}[float(h)]
    nz, nx = 350 // step + 1, 1700 // step + 1
    return {
        "true": bet_true_model(nz, nx, h), "h": h,
        "srcs": [(0, (200 + 500 * k) // int(h)) for k in range(34)],
        "recs": [(0, j) for j in range(nx)],
        "cfg": dict(nz=nz, nx=nx, h=h, chains=chains, k_min=4, k_max=48, k_init=12, burn_in=20, thin=5,
                    v_min=1400.0, v_max=5000.0, p_birth=0.25, p_death=0.25, move_dz=300.0, move_dx=1500.0,
                    sigma=0.005, seed=2001),
    }
