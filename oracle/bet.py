"""Stage 1 oracle (Bayesian Eikonal tomography): marshalling for bet_oracle.c.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg call it; the library's path never imports it.

Sec. 2.1 (Eq. 1-3) defines the pieces: the forward operator F is the Eikonal
equation (first-arrival travel times), the model is a Voronoi tessellation
with a constant velocity per cell, the likelihood is Gaussian in the
travel-time residuals, and reversible-jump chains add, delete and move cell
nuclei.  The arithmetic is in C (``bet_oracle.c``); this module converts
arrays and structs.
"""
from __future__ import annotations

import ctypes
import dataclasses

import numpy as np

from . import LIB_PATH, build

_lib_handle = None


class _Cfg(ctypes.Structure):
    _fields_ = [("nz", ctypes.c_int32), ("nx", ctypes.c_int32), ("h", ctypes.c_double),
                ("nsrc", ctypes.c_int32), ("nrec", ctypes.c_int32),
                ("chains", ctypes.c_int32), ("k_min", ctypes.c_int32), ("k_max", ctypes.c_int32),
                ("k_init", ctypes.c_int32), ("v_min", ctypes.c_double), ("v_max", ctypes.c_double),
                ("p_birth", ctypes.c_double), ("p_death", ctypes.c_double),
                ("move_dz", ctypes.c_double), ("move_dx", ctypes.c_double), ("sigma", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("burn_in", ctypes.c_int32), ("thin", ctypes.c_int32),
                ("single", ctypes.c_int32), ("chain0", ctypes.c_int32)]


class _Info(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("misfit", ctypes.c_double),
                ("proposed", ctypes.c_int64 * 3), ("accepted", ctypes.c_int64 * 3)]


def _lib():
    global _lib_handle
    if _lib_handle is None:
        if not LIB_PATH.exists():
            build()
        L = ctypes.CDLL(str(LIB_PATH))
        P, u64, i32, d = ctypes.POINTER, ctypes.c_uint64, ctypes.c_int, ctypes.c_double
        L.orc_sm64_mix.argtypes, L.orc_sm64_mix.restype = [u64], u64
        L.orc_sm64_at.argtypes, L.orc_sm64_at.restype = [u64, u64], u64
        L.orc_bet_draw.argtypes, L.orc_bet_draw.restype = [u64, i32, i32, i32], u64
        L.orc_voronoi.argtypes = [i32, i32, d, i32, P(d), P(d), P(ctypes.c_int32)]
        L.orc_eikonal_f64.argtypes = [i32, i32, d, P(d), i32, i32, P(d)]
        L.orc_eikonal_f32.argtypes = [i32, i32, ctypes.c_float, P(ctypes.c_float), i32, i32, P(ctypes.c_float)]
        L.orc_eikonal_fsm_f32.argtypes = [i32, i32, ctypes.c_float, P(ctypes.c_float), i32, i32,
                                          P(ctypes.c_float)]
        L.orc_eikonal_table.argtypes = [P(_Cfg), P(d), P(ctypes.c_int32), P(ctypes.c_int32), P(d)]
        L.orc_bet_run.argtypes = [P(_Cfg), P(ctypes.c_int32), P(ctypes.c_int32), P(ctypes.c_float), i32,
                                  P(d), P(d), P(d), P(_Info), P(d), P(d), P(ctypes.c_int64), P(ctypes.c_int8)]
        for f in ("orc_voronoi", "orc_eikonal_f64", "orc_eikonal_f32", "orc_eikonal_fsm_f32", "orc_eikonal_table",
                  "orc_bet_run"):
            getattr(L, f).restype = ctypes.c_int
        _lib_handle = L
    return _lib_handle


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


@dataclasses.dataclass
class BetConfig:
    """Chains, prior and proposal of the Stage-1 sampler (Sec. 2.1)."""
    nz: int
    nx: int
    h: float
    chains: int = 8
    k_min: int = 4
    k_max: int = 48
    k_init: int = 12
    v_min: float = 1400.0
    v_max: float = 5000.0
    p_birth: float = 1.0 / 3.0
    p_death: float = 1.0 / 3.0
    move_dz: float = 300.0
    move_dx: float = 1000.0
    sigma: float = 0.005
    seed: int = 2001
    burn_in: int = 0
    thin: int = 1
    single: bool = True
    chain0: int = 0  # run chains chain0 .. chain0 + chains - 1

    def c(self, nsrc, nrec):
        return _Cfg(self.nz, self.nx, self.h, nsrc, nrec, self.chains, self.k_min, self.k_max, self.k_init,
                    self.v_min, self.v_max, self.p_birth, self.p_death, self.move_dz, self.move_dx,
                    self.sigma, self.seed, self.burn_in, self.thin, int(self.single), self.chain0)


def sm64_at(seed: int, n: int) -> int:
    """Output n of the splitmix64 stream seeded with `seed`."""
    return int(_lib().orc_sm64_at(seed, n))


def draw(seed: int, chain: int, t: int, k: int) -> int:
    return int(_lib().orc_bet_draw(seed, chain, t, k))


def voronoi(nz, nx, h, zs, xs):
    """Index of the nearest nucleus at every node (i h, j h); ties: lowest index."""
    zs = np.ascontiguousarray(zs, dtype=np.float64)
    xs = np.ascontiguousarray(xs, dtype=np.float64)
    out = np.empty((nz, nx), dtype=np.int32)
    _lib().orc_voronoi(nz, nx, h, len(zs), _p(zs, ctypes.c_double), _p(xs, ctypes.c_double),
                       _p(out, ctypes.c_int32))
    return out


def eikonal(slowness, h, src, single=False, sweep=False):
    """First-arrival times on the grid from source node src = (iz, ix): fast
    marching (FP64, or FP32 with single=True), or fast sweeping in FP32
    (sweep=True; returns (T, passes))."""
    if sweep:
        s = np.ascontiguousarray(slowness, dtype=np.float32)
        T = np.empty_like(s)
        passes = _lib().orc_eikonal_fsm_f32(s.shape[0], s.shape[1], np.float32(h), _p(s, ctypes.c_float), src[0],
                                            src[1], _p(T, ctypes.c_float))
        return T, passes
    if single:
        s = np.ascontiguousarray(slowness, dtype=np.float32)
        T = np.empty_like(s)
        _lib().orc_eikonal_f32(s.shape[0], s.shape[1], np.float32(h), _p(s, ctypes.c_float), src[0], src[1],
                               _p(T, ctypes.c_float))
        return T
    s = np.ascontiguousarray(slowness, dtype=np.float64)
    T = np.empty_like(s)
    _lib().orc_eikonal_f64(s.shape[0], s.shape[1], float(h), _p(s, ctypes.c_double), src[0], src[1],
                           _p(T, ctypes.c_double))
    return T


def _pts(pts):
    return np.ascontiguousarray(np.asarray(pts, dtype=np.int32).reshape(-1, 2))


def travel_times(vel, h, srcs, recs, single=False):
    """[nsrc][nrec] first-arrival times of the velocity grid vel (m/s): fast
    marching in FP64, or fast sweeping in FP32 with single=True."""
    vel = np.ascontiguousarray(vel, dtype=np.float64)
    s, r = _pts(srcs), _pts(recs)
    cfg = BetConfig(vel.shape[0], vel.shape[1], h, single=single).c(len(s), len(r))
    tt = np.empty((len(s), len(r)), dtype=np.float64)
    _lib().orc_eikonal_table(ctypes.byref(cfg), _p(vel, ctypes.c_double), _p(s, ctypes.c_int32),
                             _p(r, ctypes.c_int32), _p(tt, ctypes.c_double))
    return tt


def run(cfg: BetConfig, srcs, recs, tt_obs, iters, log=False):
    """Run every chain for `iters` iterations; returns states, counters and the
    pooled post-burn-in velocity statistics (mean, sample std, count)."""
    s, r = _pts(srcs), _pts(recs)
    tt = np.ascontiguousarray(tt_obs, dtype=np.float32)
    C, K, n = cfg.chains, cfg.k_max, cfg.nz * cfg.nx
    z = np.zeros((C, K)); x = np.zeros((C, K)); v = np.zeros((C, K))
    info = (_Info * C)()
    mean = np.zeros(n); m2 = np.zeros(n); cnt = ctypes.c_int64(0)
    alog = np.zeros((iters, C), dtype=np.int8) if log else None
    rc = _lib().orc_bet_run(ctypes.byref(cfg.c(len(s), len(r))), _p(s, ctypes.c_int32), _p(r, ctypes.c_int32),
                            _p(tt, ctypes.c_float), iters, _p(z, ctypes.c_double), _p(x, ctypes.c_double),
                            _p(v, ctypes.c_double), info, _p(mean, ctypes.c_double), _p(m2, ctypes.c_double),
                            ctypes.byref(cnt), _p(alog, ctypes.c_int8) if log else None)
    if rc != 0:
        raise ValueError("bad chain configuration")
    k = np.array([info[c].k for c in range(C)])
    out = {"k": k, "z": z, "x": x, "v": v, "misfit": np.array([info[c].misfit for c in range(C)]),
           "proposed": np.array([list(info[c].proposed) for c in range(C)]),
           "accepted": np.array([list(info[c].accepted) for c in range(C)]),
           "mean": mean.reshape(cfg.nz, cfg.nx), "count": cnt.value,
           "std": np.sqrt(m2 / max(cnt.value - 1, 1)).reshape(cfg.nz, cfg.nx)}
    if log:
        out["log"] = alog
    return out


def model_velocity(cfg: BetConfig, k, zs, xs, vs):
    """Velocity grid of one model (the nearest nucleus's velocity at each node)."""
    cell = voronoi(cfg.nz, cfg.nx, cfg.h, zs[:k], xs[:k])
    return np.asarray(vs)[cell]
