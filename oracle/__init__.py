"""FP64 CPU oracle of the RTM hot path of arXiv:2001.06444.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  The product path (the HIP library
and its Python binding) never imports this package, and this package imports
nothing from the product.

The arithmetic lives in ``rtm_oracle.c`` (plain C, double precision); this
module marshals NumPy arrays into it and adds the pieces that are plain
array algebra: window placement and stacking over shots, and the two-pass
ensemble statistics.  Each function names the passage of the paper it follows.
"""
from __future__ import annotations

import ctypes
import os
import pathlib

import numpy as np

_HERE = pathlib.Path(__file__).resolve().parent
LIB_PATH = _HERE / "liboracle.so"

QUANT = {None: 0, "fp32": 0, "bf16": 1, "fp16": 2}


class _Grid(ctypes.Structure):
    _fields_ = [
        ("nz", ctypes.c_int32),
        ("nx", ctypes.c_int32),
        ("nb", ctypes.c_int32),
        ("nt", ctypes.c_int32),
        ("dz", ctypes.c_double),
        ("dx", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("sponge_a", ctypes.c_double),
        ("periodic", ctypes.c_int32),
        ("pad_", ctypes.c_int32),
    ]


_lib_handle = None


def build(force: bool = False) -> pathlib.Path:
    """Compile rtm_oracle.c with gcc (FP64, OpenMP, no fast-math)."""
    from . import _build

    return _build.build(force=force)


def _lib():
    global _lib_handle
    if _lib_handle is None:
        if not LIB_PATH.exists():
            build()
        lib = ctypes.CDLL(str(LIB_PATH))
        P = ctypes.POINTER
        d, i = ctypes.c_double, ctypes.c_int
        pd, pi = P(d), P(ctypes.c_int)
        g = P(_Grid)
        lib.orc_laplacian.argtypes = [g, pd, pd]
        lib.orc_forward.argtypes = [g, pd, pd, i, i, i, pi, pi, pd, pd, pd, pd]
        lib.orc_born.argtypes = [g, pd, pd, i, i, pd, i, pi, pi, pd]
        lib.orc_rtm.argtypes = [g, pd, pd, i, i, i, pi, pi, pd, i, i, i, i, pd, pd]
        lib.orc_reconstruct.argtypes = [g, pd, pd, i, i, pd]
        for name in ("orc_round_fp16", "orc_round_bf16", "orc_snapshot_scale"):
            fn = getattr(lib, name)
            fn.argtypes = [d]
            fn.restype = d
        _lib_handle = lib
    return _lib_handle


def _pd(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _pi(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _grid(nz, nx, nb, nt, dz, dx, dt, sponge_a=0.0, periodic=False):
    return _Grid(nz, nx, nb, nt, dz, dx, dt, sponge_a, 1 if periodic else 0, 0)


def _check(rc, name):
    if rc != 0:
        raise ValueError(f"{name} failed with code {rc}")


def _rec_arrays(rec):
    rec = np.asarray(rec, dtype=np.int32).reshape(-1, 2)
    return (np.ascontiguousarray(rec[:, 0], dtype=np.int32),
            np.ascontiguousarray(rec[:, 1], dtype=np.int32))


# ---------------------------------------------------------------------------
# Discrete operators (Sec. 3: 8th order in space, 2nd order in time)
# ---------------------------------------------------------------------------

def laplacian(u, dz, dx, periodic=False):
    """8th-order Laplacian of a 2-D field with zero ghosts or periodic wrap."""
    u = _f64(u)
    nz, nx = u.shape
    out = np.empty_like(u)
    g = _grid(nz, nx, 0, 1, dz, dx, 1.0, periodic=periodic)
    _check(_lib().orc_laplacian(ctypes.byref(g), _pd(u), _pd(out)), "orc_laplacian")
    return out


def forward(vel, wavelet, src, rec, *, dz, dx, dt, nb, nt, sponge_a=0.0, periodic=False,
            snaps=False, final=False, init=None):
    """Forward modelling (Eq. 4 with the wavelet as source term).

    Returns a dict with ``traces`` [nt][nrec] (d[n][r] = u^n(r)), optionally
    ``snaps`` [nt][nz][nx] and ``final`` (u^{nt-1}, u^{nt-2}).
    """
    vel = _f64(vel)
    nz, nx = vel.shape
    w = None if wavelet is None else _f64(wavelet)
    riz, rix = _rec_arrays(rec) if rec is not None and len(rec) else (np.zeros(0, np.int32),) * 2
    nrec = len(riz)
    traces = np.zeros((nt, nrec))
    sn = np.zeros((nt, nz, nx)) if snaps else None
    fin = np.zeros((2, nz, nx)) if final else None
    ini = None if init is None else _f64(init)
    g = _grid(nz, nx, nb, nt, dz, dx, dt, sponge_a, periodic)
    siz, six = (0, 0) if src is None else (int(src[0]), int(src[1]))
    rc = _lib().orc_forward(ctypes.byref(g), _pd(vel), _pd(w), siz, six, nrec, _pi(riz),
                            _pi(rix), _pd(traces), _pd(sn), _pd(fin), _pd(ini))
    _check(rc, "orc_forward")
    out = {"traces": traces}
    if snaps:
        out["snaps"] = sn
    if final:
        out["final"] = fin
    return out


def born(vel, wavelet, src, mpert, rec, *, dz, dx, dt, nb, nt, sponge_a=0.0):
    """Born modelling with perturbation ``mpert`` (adjoint-test partner of rtm)."""
    vel = _f64(vel)
    nz, nx = vel.shape
    mp = _f64(mpert)
    riz, rix = _rec_arrays(rec)
    dd = np.zeros((nt, len(riz)))
    g = _grid(nz, nx, nb, nt, dz, dx, dt, sponge_a)
    rc = _lib().orc_born(ctypes.byref(g), _pd(vel), _pd(_f64(wavelet)), int(src[0]), int(src[1]),
                         _pd(mp), len(riz), _pi(riz), _pi(rix), _pd(dd))
    _check(rc, "orc_born")
    return dd


def rtm_shot(vel, wavelet, src, rec, data, *, dz, dx, dt, nb, stride=1, quant=None,
             s_mode="store", ckpt=64, illum=False, sponge_a=0.0):
    """Reverse time migration of one shot (Sec. 2.2, Eq. 5 numerator).

    ``s_mode`` "store" keeps every S^n; "checkpoint" recomputes segments from
    checkpoints (same S^n bit for bit).  ``quant`` in {None, "bf16", "fp16"}
    applies the per-snapshot power-of-two-scaled 16-bit round trip to S^n.
    Returns image [nz][nx] (and illum if requested).
    """
    vel = _f64(vel)
    nz, nx = vel.shape
    data = _f64(data)
    nt = data.shape[0]
    riz, rix = _rec_arrays(rec)
    if data.shape != (nt, len(riz)):
        raise ValueError("data must be [nt][nrec]")
    img = np.zeros((nz, nx))
    ill = np.zeros((nz, nx)) if illum else None
    g = _grid(nz, nx, nb, nt, dz, dx, dt, sponge_a)
    mode = {"store": 0, "checkpoint": 1}[s_mode]
    rc = _lib().orc_rtm(ctypes.byref(g), _pd(vel), _pd(_f64(wavelet)), int(src[0]), int(src[1]),
                        len(riz), _pi(riz), _pi(rix), _pd(data), int(stride), QUANT[quant], mode,
                        int(ckpt), _pd(img), _pd(ill))
    _check(rc, "orc_rtm")
    return (img, ill) if illum else img


def reconstruct(vel, wavelet, src, *, dz, dx, dt, nb, nt, sponge_a=0.0):
    """Source wavefield rebuilt backward from the saved ring + last two states."""
    vel = _f64(vel)
    nz, nx = vel.shape
    out = np.zeros((nt, nz, nx))
    g = _grid(nz, nx, nb, nt, dz, dx, dt, sponge_a)
    rc = _lib().orc_reconstruct(ctypes.byref(g), _pd(vel), _pd(_f64(wavelet)), int(src[0]),
                                int(src[1]), _pd(out))
    _check(rc, "orc_reconstruct")
    return out


# ---------------------------------------------------------------------------
# 16-bit snapshot emulation (storage-precision stand-in for lossy compression)
# ---------------------------------------------------------------------------

def round_fp16(x: float) -> float:
    return _lib().orc_round_fp16(float(x))


def round_bf16(x: float) -> float:
    return _lib().orc_round_bf16(float(x))


def snapshot_scale(maxabs: float) -> float:
    return _lib().orc_snapshot_scale(float(maxabs))


# ---------------------------------------------------------------------------
# Windows, stacking, ensemble statistics (Fig. 2 caption: stacked sections per
# velocity sample; Sec. 2.3 and Sec. 5: mean and standard-deviation maps)
# ---------------------------------------------------------------------------

def migrate_window(vel_model, ix0, width, wavelet, src, rec, data, **kw):
    """Migrate one shot on the aperture window [ix0, ix0+width) of a model.

    ``src`` and ``rec`` are in model coordinates; the window's own sponge is
    padded around the sliced velocity.  Returns the [nz][width] image.
    """
    v = np.asarray(vel_model)[:, ix0:ix0 + width]
    s = (int(src[0]), int(src[1]) - ix0)
    r = np.asarray(rec, dtype=np.int64).reshape(-1, 2).copy()
    r[:, 1] -= ix0
    return rtm_shot(v, wavelet, s, r, data, **kw)


def stack(images, windows, nx_model):
    """Sum of window-placed shot images, in the given shot order (FP64)."""
    images = list(images)
    nz = images[0].shape[0]
    out = np.zeros((nz, nx_model))
    for img, (ix0, w) in zip(images, windows):
        out[:, ix0:ix0 + w] += img
    return out


def ensemble_stats(samples):
    """Two-pass mean and sample standard deviation (n - 1) over axis 0."""
    x = np.asarray(samples, dtype=np.float64)
    n = x.shape[0]
    mean = x.sum(axis=0) / n
    if n < 2:
        return mean, np.zeros_like(mean)
    dev = x - mean
    var = (dev * dev).sum(axis=0) / (n - 1)
    return mean, np.sqrt(var)


def windowed_stats(images, windows, nz, nx_model):
    """Per-pixel two-pass mean / sample std over windowed images.

    A pixel's samples are the images whose window covers it; count is the
    number of such images.  Returns (mean, std, count), std = 0 where count < 2.
    """
    cnt = np.zeros((nz, nx_model), dtype=np.int64)
    s = np.zeros((nz, nx_model))
    for img, (ix0, w) in zip(images, windows):
        cnt[:, ix0:ix0 + w] += 1
        s[:, ix0:ix0 + w] += img
    mean = np.where(cnt > 0, s / np.maximum(cnt, 1), 0.0)
    ss = np.zeros((nz, nx_model))
    for img, (ix0, w) in zip(images, windows):
        d = img - mean[:, ix0:ix0 + w]
        ss[:, ix0:ix0 + w] += d * d
    std = np.where(cnt > 1, np.sqrt(ss / np.maximum(cnt - 1, 1)), 0.0)
    return mean, std, cnt


def rel_l2(a, ref):
    """Relative L2 error ||a - ref|| / ||ref||, accumulated in FP64."""
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.sqrt((ref * ref).sum())
    return float(np.sqrt(((a - ref) ** 2).sum()) / den) if den > 0 else float(np.abs(a).max())


def nthreads() -> int:
    """OpenMP threads the oracle will use (OMP_NUM_THREADS, else all cores)."""
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        return int(env)
    return os.cpu_count() or 1


# ---------------------------------------------------------------------------
# Stage-3 maps and the post-stack filter (Sec. 2.3, Eq. 6 and Eq. 7; Sec. 3)
# ---------------------------------------------------------------------------

def confidence_index(std, count=None, min_count=2):
    """Eq. 6: c = (s_max - s) / (s_max - s_min), extremes over pixels with
    count >= min_count (all pixels when count is None); 0 elsewhere and when
    s_max == s_min."""
    s = np.asarray(std, dtype=np.float64)
    mask = np.ones(s.shape, bool) if count is None else np.asarray(count) >= min_count
    out = np.zeros_like(s)
    if not mask.any():
        return out
    lo, hi = s[mask].min(), s[mask].max()
    if hi > lo:
        out[mask] = (hi - s[mask]) / (hi - lo)
    return out


def ratio_map(std, mean, eps=0.0):
    """Eq. 7: r = std / mean where |mean| > eps, else 0."""
    s = np.asarray(std, dtype=np.float64)
    m = np.asarray(mean, dtype=np.float64)
    out = np.zeros_like(s)
    ok = np.abs(m) > eps
    out[ok] = s[ok] / m[ok]
    return out


def laplacian_filter(img, dz, dx):
    """Post-stack Laplacian filter: -(8th-order Laplacian), zero outside the image."""
    return -laplacian(img, dz, dx)
