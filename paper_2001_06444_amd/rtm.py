"""Python binding of librtm.so (include/rtm.h): argument marshalling only.

Every computation runs in the HIP library; this module turns torch tensors
into device pointers and Python values into the C structs of the ABI.  If
the built library is missing, loading fails with an error: there is no other
implementation behind these names.
"""
from __future__ import annotations

import ctypes
import pathlib

LIB_PATH = pathlib.Path(__file__).resolve().parent / "librtm.so"

RTM_OK = 0
STATUS = {0: "RTM_OK", -1: "RTM_E_INVAL", -2: "RTM_E_CFL", -3: "RTM_E_NOMEM", -4: "RTM_E_AGAIN",
          -5: "RTM_E_NOTFOUND", -6: "RTM_E_NONFINITE", -7: "RTM_E_DEVICE", -8: "RTM_E_CANCELLED"}
SNAP = {"fp32": 0, "bf16": 1, "fp16": 2}
SRC_STORE, SRC_RECONSTRUCT = 0, 1
IMG_ILLUM = 1
CODEC_TOL, CODEC_LOSSLESS, CODEC_ZFP = 0, 1, 2
JOB_QUEUED, JOB_RUNNING, JOB_DONE, JOB_FAILED, JOB_CANCELLED = range(5)
JOB_ACC_STATS, JOB_ACC_STACK = 1, 2


class RTMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Grid(ctypes.Structure):
    _fields_ = [("nz", ctypes.c_int32), ("nx", ctypes.c_int32), ("nb", ctypes.c_int32),
                ("nt", ctypes.c_int32), ("dz", ctypes.c_float), ("dx", ctypes.c_float),
                ("dt", ctypes.c_float), ("sponge_a", ctypes.c_float)]


class Point(ctypes.Structure):
    _fields_ = [("iz", ctypes.c_int32), ("ix", ctypes.c_int32)]


class ImgOpts(ctypes.Structure):
    _fields_ = [("src_mode", ctypes.c_int32), ("snap_dtype", ctypes.c_int32),
                ("snap_stride", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class ShotDesc(ctypes.Structure):
    _fields_ = [("src", Point), ("ix0", ctypes.c_int32), ("width", ctypes.c_int32),
                ("nrec", ctypes.c_int32), ("rec_host", ctypes.POINTER(Point)),
                ("data_dev", ctypes.c_void_p)]


class BornShot(ctypes.Structure):
    _fields_ = [("src", Point), ("nrec", ctypes.c_int32), ("rec_host", ctypes.POINTER(Point)),
                ("dtraces_dev", ctypes.c_void_p)]


class Job(ctypes.Structure):
    _fields_ = [("realization", ctypes.c_int32), ("src", Point), ("ix0", ctypes.c_int32),
                ("width", ctypes.c_int32), ("rec_iz", ctypes.c_int32), ("nt", ctypes.c_int32),
                ("wavelet_dev", ctypes.c_void_p), ("data_dev", ctypes.c_void_p),
                ("img", ImgOpts), ("flags", ctypes.c_uint32), ("user_tag", ctypes.c_uint64)]


class JobInfo(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("status", ctypes.c_int32),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double), ("grid_updates", ctypes.c_uint64),
                ("alg_bytes", ctypes.c_uint64), ("user_tag", ctypes.c_uint64)]


class CtxStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in (
        "jobs_submitted", "jobs_done", "jobs_failed", "jobs_cancelled", "steps_launched",
        "graph_replays", "grid_updates", "alg_bytes", "arena_bytes", "arena_used", "arena_peak")] + [
        ("tile_z", ctypes.c_int32), ("active_jobs", ctypes.c_int32),
        ("queued_jobs", ctypes.c_int32), ("last_steps_per_launch", ctypes.c_int32),
        ("last_fwd_ms", ctypes.c_float), ("last_bwd_ms", ctypes.c_float),
        ("last_fwd_launches", ctypes.c_int32), ("last_bwd_launches", ctypes.c_int32),
        ("last_fwd_launch_bytes", ctypes.c_uint64), ("last_bwd_launch_bytes", ctypes.c_uint64),
        ("last_codec_ms", ctypes.c_float), ("last_codec_op", ctypes.c_int32),
        ("last_codec_bytes", ctypes.c_uint64),
        ("last_bet_eikonal_ms", ctypes.c_float), ("last_bet_iteration_ms", ctypes.c_float),
        ("last_tile_z2_fwd", ctypes.c_int32), ("last_tile_z2_bwd", ctypes.c_int32),
        ("last_groups_fwd", ctypes.c_int32), ("last_groups_bwd", ctypes.c_int32),
        ("last_born_groups", ctypes.c_int32)]


class BetConfig(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("nz", "nx", "chains", "k_min", "k_max", "k_init", "burn_in",
                                              "thin")] + \
               [(n, ctypes.c_double) for n in ("h", "v_min", "v_max", "p_birth", "p_death", "move_dz",
                                               "move_dx", "sigma")] + [("seed", ctypes.c_uint64)]


class BetChainInfo(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("pad_", ctypes.c_int32), ("misfit", ctypes.c_double),
                ("proposed", ctypes.c_int64 * 3), ("accepted", ctypes.c_int64 * 3),
                ("solves", ctypes.c_int64), ("sweeps", ctypes.c_int64)]


# exported symbols and their C signatures (argtypes, restype)
_P, _V, _I32, _U32, _U64, _F, _D = (ctypes.POINTER, ctypes.c_void_p, ctypes.c_int32,
                                    ctypes.c_uint32, ctypes.c_uint64, ctypes.c_float,
                                    ctypes.c_double)
SIGNATURES = {
    "rtm_status_str": ([ctypes.c_int], ctypes.c_char_p),
    "rtm_last_error": ([], ctypes.c_char_p),
    "rtm_version": ([], ctypes.c_int),
    "rtm_cfl_number": ([_F, _F, _F, _F], _D),
    "rtm_cfl_limit": ([], _D),
    "rtm_ctx_create": ([_P(_V), ctypes.c_int, _V, ctypes.c_size_t, _V, _U32], ctypes.c_int),
    "rtm_ctx_destroy": ([_V], ctypes.c_int),
    "rtm_ctx_synchronize": ([_V], ctypes.c_int),
    "rtm_propagate": ([_V, _P(Grid), _V, _V, Point, _I32, _P(Point), _V, _V], ctypes.c_int),
    "rtm_born": ([_V, _P(Grid), _V, _V, Point, _V, _I32, _P(Point), _V], ctypes.c_int),
    "rtm_born_batch": ([_V, _P(Grid), _V, _V, _V, _I32, _P(BornShot)], ctypes.c_int),
    "rtm_stats_merge": ([_V, _V, _V], ctypes.c_int),
    "rtm_normalize_image": ([_V, _V, _V, _I32, _F, _V], ctypes.c_int),
    "rtm_migrate_shot": ([_V, _P(Grid), _V, _V, Point, _I32, _P(Point), _V, _I32, _I32,
                          _P(ImgOpts), _V, _V], ctypes.c_int),
    "rtm_migrate_batch": ([_V, _P(Grid), _V, _V, _I32, _P(ShotDesc), _P(ImgOpts), _V, _V],
                          ctypes.c_int),
    "rtm_model_register": ([_V, _I32, _V, _I32, _I32, _P(Grid)], ctypes.c_int),
    "rtm_ensemble_submit": ([_V, _P(Job), _P(_U64)], ctypes.c_int),
    "rtm_ensemble_poll": ([_V, _U64, _P(JobInfo), _V, _I32], ctypes.c_int),
    "rtm_ensemble_cancel": ([_V, _U64], ctypes.c_int),
    "rtm_ensemble_drain": ([_V], ctypes.c_int),
    "rtm_ensemble_stats": ([_V, _I32, _V, _V, _V], ctypes.c_int),
    "rtm_ensemble_stack": ([_V, _I32, _V], ctypes.c_int),
    "rtm_stats_create": ([_V, _P(_V), _I32, _I32], ctypes.c_int),
    "rtm_stats_destroy": ([_V, _V], ctypes.c_int),
    "rtm_stats_add": ([_V, _V, _V, _I32, _I32], ctypes.c_int),
    "rtm_stats_get": ([_V, _V, _V, _V, _V], ctypes.c_int),
    "rtm_confidence_map": ([_V, _V, _V, _I32, _I32, _V], ctypes.c_int),
    "rtm_ratio_map": ([_V, _V, _V, _I32, _D, _V], ctypes.c_int),
    "rtm_laplacian_filter": ([_V, _V, _I32, _I32, _F, _F, _V], ctypes.c_int),
    "rtm_codec_max_bytes": ([_I32, _I32, _I32], ctypes.c_int64),
    "rtm_codec_encode": ([_V, _V, _I32, _I32, _I32, _I32, _D, _V, ctypes.c_int64,
                          _P(ctypes.c_int64)], ctypes.c_int),
    "rtm_codec_encode_noalloc": ([_V, _V, _I32, _I32, _I32, _I32, _D, _V, ctypes.c_int64,
                                  _P(ctypes.c_int64)], ctypes.c_int),
    "rtm_codec_info": ([_V, _V, ctypes.c_int64, _P(_I32), _P(_I32), _P(_I32), _P(_I32), _P(_D)],
                       ctypes.c_int),
    "rtm_codec_decode": ([_V, _V, ctypes.c_int64, _V, ctypes.c_int64], ctypes.c_int),
    "rtm_eikonal": ([_V, _V, _I32, _I32, _F, _I32, _P(Point), _I32, _P(Point), _V], ctypes.c_int),
    "rtm_bet_create": ([_V, _P(BetConfig), _I32, _P(Point), _I32, _P(Point), _V, _P(_V)], ctypes.c_int),
    "rtm_bet_run": ([_V, _V, _I32, _V], ctypes.c_int),
    "rtm_bet_chain": ([_V, _V, _I32, _P(BetChainInfo), _V, _V, _V], ctypes.c_int),
    "rtm_bet_stats": ([_V, _V, _V, _V, _V], ctypes.c_int),
    "rtm_bet_model": ([_V, _V, _I32, _I32, _I32, _D, _V], ctypes.c_int),
    "rtm_bet_destroy": ([_V, _V], ctypes.c_int),
    "rtm_sqrt_check": ([_V, ctypes.c_uint32, ctypes.c_uint32, _P(ctypes.c_uint64)], ctypes.c_int),
    "rtm_ctx_stats": ([_V, _P(CtxStats)], ctypes.c_int),
}

_lib = None


def lib():
    """Load librtm.so (built in-tree by the package build step)."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                               "(run __graft_entry__.build())")
        L = ctypes.CDLL(str(LIB_PATH))
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(rc):
    if rc != RTM_OK:
        msg = lib().rtm_last_error().decode(errors="replace")
        raise RTMError(rc, msg)


def cfl_limit() -> float:
    return lib().rtm_cfl_limit()


def cfl_number(vmax, dt, dz, dx) -> float:
    return lib().rtm_cfl_number(vmax, dt, dz, dx)


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return ctypes.c_void_p(t.data_ptr())


def _points(pts):
    pts = [(int(p[0]), int(p[1])) for p in pts]
    arr = (Point * max(len(pts), 1))()
    for i, (z, x) in enumerate(pts):
        arr[i].iz, arr[i].ix = z, x
    return arr, len(pts)


def make_grid(nz, nx, nb, nt, dz, dx, dt, sponge_a=0.0) -> Grid:
    return Grid(nz, nx, nb, nt, dz, dx, dt, sponge_a)


def img_opts(mode="reconstruct", dtype="fp32", stride=1, illum=False) -> ImgOpts:
    m = {"store": SRC_STORE, "reconstruct": SRC_RECONSTRUCT}[mode]
    return ImgOpts(m, SNAP[dtype], int(stride), IMG_ILLUM if illum else 0)


class Context:
    """An rtm_ctx over a torch-owned device arena and a torch stream."""

    def __init__(self, device: int = 0, arena_bytes: int = 1 << 30, stream=None):
        import torch

        self.device = device
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=f"cuda:{device}")
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = ctypes.c_void_p()
        _check(lib().rtm_ctx_create(ctypes.byref(h), device, _ptr(self.arena), int(arena_bytes),
                                    ctypes.c_void_p(stream.cuda_stream), 0))
        self.h = h
        self._keep = []

    def close(self):
        if getattr(self, "h", None):
            _check(lib().rtm_ctx_destroy(self.h))
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def synchronize(self):
        _check(lib().rtm_ctx_synchronize(self.h))

    # ---- plain path ----
    def propagate(self, grid: Grid, vel, wavelet, src, rec, traces, final=None):
        recs, n = _points(rec)
        _check(lib().rtm_propagate(self.h, ctypes.byref(grid), _ptr(vel), _ptr(wavelet),
                                   Point(*src), n, recs, _ptr(traces), _ptr(final)))

    def born(self, grid: Grid, vel, wavelet, src, mpert, rec, dtraces):
        recs, n = _points(rec)
        _check(lib().rtm_born(self.h, ctypes.byref(grid), _ptr(vel), _ptr(wavelet), Point(*src),
                              _ptr(mpert), n, recs, _ptr(dtraces)))

    def born_batch(self, grid: Grid, vel, wavelet, mpert, shots):
        """shots: sequence of (src, rec_points, dtraces_tensor)."""
        descs = (BornShot * len(shots))()
        keep = []
        for i, (src, rec, dtraces) in enumerate(shots):
            recs, n = _points(rec)
            keep.append(recs)
            descs[i].src = Point(*src)
            descs[i].nrec = n
            descs[i].rec_host = ctypes.cast(recs, ctypes.POINTER(Point))
            descs[i].dtraces_dev = _ptr(dtraces)
        _check(lib().rtm_born_batch(self.h, ctypes.byref(grid), _ptr(vel), _ptr(wavelet), _ptr(mpert),
                                    len(shots), descs))

    def migrate_shot(self, grid: Grid, vel, wavelet, src, rec, data, ix0, width, opts: ImgOpts,
                     image, illum=None):
        recs, n = _points(rec)
        _check(lib().rtm_migrate_shot(self.h, ctypes.byref(grid), _ptr(vel), _ptr(wavelet),
                                      Point(*src), n, recs, _ptr(data), int(ix0), int(width),
                                      ctypes.byref(opts), _ptr(image), _ptr(illum)))

    # ---- batched path ----
    def migrate_batch(self, grid: Grid, vel, wavelet, shots, opts: ImgOpts, image, illum=None):
        """shots: sequence of (src, ix0, width, rec_points, data_tensor)."""
        descs = (ShotDesc * len(shots))()
        keep = []
        for i, (src, ix0, width, rec, data) in enumerate(shots):
            recs, n = _points(rec)
            keep.append(recs)
            descs[i].src = Point(*src)
            descs[i].ix0, descs[i].width, descs[i].nrec = int(ix0), int(width), n
            descs[i].rec_host = ctypes.cast(recs, ctypes.POINTER(Point))
            descs[i].data_dev = data.data_ptr()
        _check(lib().rtm_migrate_batch(self.h, ctypes.byref(grid), _ptr(vel), _ptr(wavelet),
                                       len(shots), descs, ctypes.byref(opts), _ptr(image),
                                       _ptr(illum)))

    # ---- ensemble / serving path ----
    def model_register(self, realization, vel, grid: Grid):
        nz, nx = vel.shape
        _check(lib().rtm_model_register(self.h, int(realization), _ptr(vel), nz, nx,
                                        ctypes.byref(grid)))

    def submit(self, realization, src, ix0, width, rec_iz, nt, wavelet, data, opts: ImgOpts,
               flags=0, tag=0) -> int:
        job = Job(int(realization), Point(*src), int(ix0), int(width), int(rec_iz), int(nt),
                  wavelet.data_ptr(), data.data_ptr(), opts, int(flags), int(tag))
        t = ctypes.c_uint64()
        _check(lib().rtm_ensemble_submit(self.h, ctypes.byref(job), ctypes.byref(t)))
        return t.value

    def poll(self, ticket, image=None, release=False) -> JobInfo:
        info = JobInfo()
        _check(lib().rtm_ensemble_poll(self.h, int(ticket), ctypes.byref(info), _ptr(image),
                                       1 if release else 0))
        return info

    def cancel(self, ticket):
        _check(lib().rtm_ensemble_cancel(self.h, int(ticket)))

    def drain(self):
        _check(lib().rtm_ensemble_drain(self.h))

    def ensemble_stats(self, realization, mean=None, std=None, count=None):
        _check(lib().rtm_ensemble_stats(self.h, int(realization), _ptr(mean), _ptr(std),
                                        _ptr(count)))

    def ensemble_stack(self, realization, stack):
        _check(lib().rtm_ensemble_stack(self.h, int(realization), _ptr(stack)))

    # ---- explicit statistics, maps, filter ----
    def stats_create(self, nz, nx):
        h = ctypes.c_void_p()
        _check(lib().rtm_stats_create(self.h, ctypes.byref(h), int(nz), int(nx)))
        return h

    def stats_destroy(self, st):
        _check(lib().rtm_stats_destroy(self.h, st))

    def stats_add(self, st, image, ix0=0, width=None):
        width = image.shape[1] if width is None else width
        _check(lib().rtm_stats_add(self.h, st, _ptr(image), int(ix0), int(width)))

    def stats_get(self, st, mean=None, std=None, count=None):
        _check(lib().rtm_stats_get(self.h, st, _ptr(mean), _ptr(std), _ptr(count)))

    def stats_merge(self, dst, src):
        _check(lib().rtm_stats_merge(self.h, dst, src))

    def normalize_image(self, image, illum, out, eps_rel=1e-6):
        _check(lib().rtm_normalize_image(self.h, _ptr(image), _ptr(illum), image.numel(),
                                         float(eps_rel), _ptr(out)))

    def confidence_map(self, std, count, out, min_count=2):
        _check(lib().rtm_confidence_map(self.h, _ptr(std), _ptr(count), std.numel(),
                                        int(min_count), _ptr(out)))

    def ratio_map(self, std, mean, out, eps=0.0):
        _check(lib().rtm_ratio_map(self.h, _ptr(std), _ptr(mean), std.numel(), float(eps),
                                   _ptr(out)))

    def laplacian_filter(self, img, dz, dx, out):
        nz, nx = img.shape
        _check(lib().rtm_laplacian_filter(self.h, _ptr(img), nz, nx, float(dz), float(dx),
                                          _ptr(out)))

    # ---- codec ----
    def codec_max_bytes(self, count, rows, cols) -> int:
        return int(lib().rtm_codec_max_bytes(int(count), int(rows), int(cols)))

    def codec_encode(self, x, tol=None, lossless=False, out=None, zfp=False):
        """Encode a float32 [rows][cols] or [count][rows][cols] device tensor
        (zfp=True: the fixed-accuracy ZFP-method coder, RTM_CODEC_ZFP).

        Returns the stream as a uint8 device tensor (a view of `out` when given)."""
        import torch
        if x.dtype != torch.float32:
            raise ValueError("float32 tensor expected")
        count, rows, cols = (1, *x.shape) if x.dim() == 2 else tuple(x.shape)
        if out is None:
            cap = self.codec_max_bytes(count, rows, cols)
            if cap < 0:
                raise ValueError("shape outside the codec's limits")
            out = torch.empty(cap, dtype=torch.uint8, device=x.device)
        n = ctypes.c_int64(0)
        mode = CODEC_ZFP if zfp else (CODEC_LOSSLESS if lossless else CODEC_TOL)
        _check(lib().rtm_codec_encode(self.h, _ptr(x), count, rows, cols, mode,
                                      float(tol if tol is not None else 0.0), _ptr(out), out.numel(),
                                      ctypes.byref(n)))
        return out[: n.value]

    def codec_encode_noalloc(self, x, out, tol=None, lossless=False):
        """rtm_codec_encode_noalloc: as codec_encode into the caller's uint8
        device tensor `out`, with nothing allocated by the call."""
        import torch
        if x.dtype != torch.float32 or out.dtype != torch.uint8:
            raise ValueError("float32 input and uint8 output tensors expected")
        count, rows, cols = (1, *x.shape) if x.dim() == 2 else tuple(x.shape)
        n = ctypes.c_int64(0)
        mode = CODEC_LOSSLESS if lossless else CODEC_TOL
        _check(lib().rtm_codec_encode_noalloc(self.h, _ptr(x), count, rows, cols, mode,
                                              float(tol if tol is not None else 0.0), _ptr(out), out.numel(),
                                              ctypes.byref(n)))
        return out[: n.value]

    def codec_info(self, stream):
        m, c, r, k, t = (ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(),
                         ctypes.c_double())
        _check(lib().rtm_codec_info(self.h, _ptr(stream), stream.numel(), ctypes.byref(m),
                                    ctypes.byref(c), ctypes.byref(r), ctypes.byref(k),
                                    ctypes.byref(t)))
        return {"mode": m.value, "count": c.value, "rows": r.value, "cols": k.value, "tol": t.value}

    def codec_decode(self, stream, out=None):
        """Decode a stream (uint8 device tensor) into float32 [count][rows][cols]."""
        import torch
        info = self.codec_info(stream)
        shape = (info["count"], info["rows"], info["cols"])
        if out is None:
            out = torch.empty(shape, dtype=torch.float32, device=stream.device)
        _check(lib().rtm_codec_decode(self.h, _ptr(stream), stream.numel(), _ptr(out), out.numel()))
        return out

    # ---- Stage 1: Bayesian Eikonal tomography ----
    def eikonal(self, vel, h, srcs, recs, out=None):
        """First-arrival times [nsrc][nrec] of the velocity grid `vel` (float32 device tensor)."""
        import torch
        nz, nx = vel.shape
        sp, ns = _points(srcs)
        rp, nr = _points(recs)
        if out is None:
            out = torch.empty(ns, nr, dtype=torch.float32, device=vel.device)
        _check(lib().rtm_eikonal(self.h, _ptr(vel), nz, nx, float(h), ns, sp, nr, rp, _ptr(out)))
        return out

    def bet_create(self, srcs, recs, tt_obs, **cfg):
        """Sampler over the observed travel times tt_obs [nsrc][nrec] (device tensor).
        cfg: nz, nx, h, chains, k_min, k_max, k_init, burn_in, thin, v_min, v_max,
        p_birth, p_death, move_dz, move_dx, sigma, seed."""
        c = BetConfig()
        for k, v in cfg.items():
            setattr(c, k, v)
        sp, ns = _points(srcs)
        rp, nr = _points(recs)
        h = ctypes.c_void_p()
        _check(lib().rtm_bet_create(self.h, ctypes.byref(c), ns, sp, nr, rp, _ptr(tt_obs), ctypes.byref(h)))
        return h

    def bet_run(self, bet, iterations, log=None):
        _check(lib().rtm_bet_run(self.h, bet, int(iterations), _ptr(log)))

    def bet_chain(self, bet, chain, k_max):
        import numpy as np
        info = BetChainInfo()
        z, x, v = (np.zeros(k_max) for _ in range(3))
        _check(lib().rtm_bet_chain(self.h, bet, int(chain), ctypes.byref(info),
                                   z.ctypes.data_as(ctypes.c_void_p), x.ctypes.data_as(ctypes.c_void_p),
                                   v.ctypes.data_as(ctypes.c_void_p)))
        return {"k": info.k, "misfit": info.misfit, "proposed": list(info.proposed),
                "accepted": list(info.accepted), "solves": info.solves, "sweeps": info.sweeps,
                "z": z, "x": x, "v": v}

    def bet_stats(self, bet, mean=None, std=None, count=None):
        _check(lib().rtm_bet_stats(self.h, bet, _ptr(mean), _ptr(std), _ptr(count)))

    def bet_model(self, bet, chain: int, vel_out, h: float):
        """Chain `chain`'s current model sampled on vel_out's [nz][nx] grid at
        spacing h (stream-ordered)."""
        nz, nx = vel_out.shape
        _check(lib().rtm_bet_model(self.h, bet, chain, nz, nx, float(h), _ptr(vel_out)))

    def bet_destroy(self, bet):
        _check(lib().rtm_bet_destroy(self.h, bet))

    def sqrt_check(self, lo_bits: int, hi_bits: int) -> int:
        """Float bit patterns in [lo_bits, hi_bits) where the travel-time
        solves' square root differs from the correctly rounded one."""
        n = ctypes.c_uint64(0)
        _check(lib().rtm_sqrt_check(self.h, lo_bits, hi_bits, ctypes.byref(n)))
        return n.value

    def stats(self) -> CtxStats:
        s = CtxStats()
        _check(lib().rtm_ctx_stats(self.h, ctypes.byref(s)))
        return s
