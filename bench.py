#!/usr/bin/env python3
"""Throughput benchmark of the RTM hot path on one MI355X.

Workload: the realistic-size survey -- faulted-layer velocity model
351 x 1701 at 10 m (a Marmousi2-sized stand-in, seed 6444), 50-cell sponge,
Ricker 15 Hz, dt = 1 ms, nt = 4000, 100 shots every 170 m with a receiver on
every column, source wavefield rebuilt backward from saved boundary rings,
images stacked over shots.  One benchmark step = migrating the whole survey
(forward + backward + imaging of all 100 shots, then the stack), inputs
resident in HBM.  The observed data (true-model minus smooth-model traces)
are modelled on the GPU before timing.

Printed: one JSON line with grid-point updates/s of the batched path (the
value), images/s, the plain one-launch-per-step path for comparison, the
roofline of the dominant kernel (the backward step) and the FP64 CPU oracle
timed on a bounded sample of the same workload; beside them, on the same
GPU, the batched UQ ensemble (64 velocity samples x 16 shots = 1024 RTMs,
nt 3000, all submitted at once to the serving engine: updates/s, images/s,
realization images/s) and the served stream (Poisson 20 jobs/s, 1200 timed
jobs after 100 warm-up: p50/p99 latency and images/s; then all 1300 jobs at
t = 0 for the saturation rate).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import pathlib
import sys
import time

ROOT = pathlib.Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# the step kernels' code; the launch configuration they were counted in (tile
# height, shot groups) is checked against the counter record separately
STEP_SOURCES = ("paper_2001_06444_amd/csrc/rtm_kernels.hip", "paper_2001_06444_amd/csrc/rtm_device.h",
                "paper_2001_06444_amd/csrc/rtm_internal.h")
CODEC_SOURCES = ("paper_2001_06444_amd/csrc/rtm_codec.hip", "paper_2001_06444_amd/csrc/rtm_codec.h")


def group_streams() -> int:
    """Streams the batched path alternates its shot groups over (the library
    reads RTM_GROUP_STREAMS the same way: 1 to 4, default 2)."""
    try:
        v = int(os.environ.get("RTM_GROUP_STREAMS", "2"))
    except ValueError:
        v = 0
    return max(1, min(v, 4))


def kernel_source_hash(sources=STEP_SOURCES) -> str:
    h = hashlib.sha256()
    for p in sources:
        h.update((ROOT / p).read_bytes())
    return h.hexdigest()[:16]


def measured_traffic(record="traffic_backward_step.json", sources=STEP_SOURCES, key=None, launch=None):
    """HBM bytes per launch of a kernel from a committed rocprofv3 counter
    summary, or None if it is missing, was taken on other code or, given
    `launch` (fields the summary must hold with these values: tile height,
    shots per launch), on another launch configuration."""
    f = ROOT / "profiles" / record
    if not f.exists():
        return None
    try:
        rec = json.loads(f.read_text())
    except ValueError:
        return None
    if rec.get("kernel_source_hash") != kernel_source_hash(sources):
        return None
    for k, v in (launch or {}).items():
        if rec.get(k) != v:
            return None
    if key is not None:
        rec = rec.get("kernels", {}).get(key, {})
    return rec.get("hbm_bytes_per_launch")


def copy_rate_gbs(gib: int = 1, reps: int = 5) -> float:
    """Device-to-device copy rate (GB/s of bytes read + written) of a `gib`
    GiB float32 tensor copy, best of `reps` (HIP events): the measured
    denominator of the roofline beside the nominal 8 TB/s."""
    import torch

    n = gib << 28
    src = torch.ones(n, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del src, dst
    torch.cuda.empty_cache()
    return 2 * 4 * n / (best * 1e-3) / 1e9


def cpu_model() -> str:
    """The host CPU's model name from /proc/cpuinfo (first processor)."""
    try:
        for line in pathlib.Path("/proc/cpuinfo").read_text().splitlines():
            if line.lower().startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(sv, nt_sample: int):
    """FP64 oracle on one shot of the same survey, first nt_sample steps."""
    import numpy as np

    import oracle

    oracle.build()
    sh = sv.shots[len(sv.shots) // 2]
    w = sv.wavelet[:nt_sample]
    rng = np.random.default_rng(0)
    data = rng.standard_normal((nt_sample, len(sh.rec))) * 1e-3
    t0 = time.perf_counter()
    oracle.rtm_shot(sv.vel_mig, w, sh.src, sh.rec, data, dz=sv.h, dx=sv.h, dt=sv.dt, nb=sv.nb)
    el = time.perf_counter() - t0
    npad = (sv.nz + 2 * sv.nb) * (sv.nx + 2 * sv.nb)
    updates = ((nt_sample - 1) + nt_sample) * npad
    return {
        "value": updates / el,
        "unit": "grid-pt updates/s",
        "cores": oracle.nthreads(),
        "cpu": cpu_model(),
        "kind": "oracle",
        "sample": (f"1 of {len(sv.shots)} shots (source ix={sh.src[1]}), first {nt_sample} of "
                   f"{sv.nt} time steps, same {sv.nz}x{sv.nx} model, nb={sv.nb}, all receivers; "
                   f"FP64 forward + adjoint + imaging with stored source wavefield; "
                   f"{updates:.3e} updates in {el:.1f} s"),
    }


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["survey", "ensemble", "serve", "small", "born", "codec", "bet", "maps"],
                    default="survey")
    ap.add_argument("--shots", type=int, default=100)
    ap.add_argument("--nt", type=int, default=None, help="default: 4000 survey, 3000 ensemble")
    ap.add_argument("--plain-shots", type=int, default=2)
    ap.add_argument("--cpu-nt", type=int, default=3000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one 1 GiB device-to-device tensor copy (reference dispatch "
                         "for the HBM byte counters)")
    ap.add_argument("--realizations", type=int, default=64, help="ensemble / codec workload")
    ap.add_argument("--seismograms", type=int, default=16, help="codec workload")
    ap.add_argument("--chains", type=int, default=64, help="bet workload")
    ap.add_argument("--bet-iters", type=int, default=20, help="bet workload: iterations per step")
    ap.add_argument("--bet-h", type=float, default=100.0, choices=[100.0, 50.0],
                    help="bet workload: node spacing (100 m: 36 x 171 nodes, 50 m: 71 x 341)")
    ap.add_argument("--serve-jobs", type=int, default=1200, help="serve workload: timed jobs")
    ap.add_argument("--serve-warmup", type=int, default=100)
    ap.add_argument("--rate", type=float, default=20.0, help="serve workload: jobs/s")
    ap.add_argument("--default-serve-jobs", type=int, default=1200,
                    help="survey workload: timed jobs of the served stream reported beside it")
    ap.add_argument("--default-serve-warmup", type=int, default=100,
                    help="survey workload: warm-up jobs of the served stream reported beside it")
    ap.add_argument("--no-serve", action="store_true", help="survey workload: skip the served stream")
    ap.add_argument("--no-ensemble", action="store_true", help="survey workload: skip the velocity ensemble")
    ap.add_argument("--rates", type=str, default="",
                    help="serve workload: extra Poisson rates (jobs/s, comma separated) run after the main one")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); every shot of the "
              "survey is independent, so N GPUs would each migrate a disjoint share of the shots.",
              file=sys.stderr)
        sys.exit(2)
    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.calibrate_copy:
        dev = torch.device("cuda:0")
        src_t = torch.ones(1 << 28, device=dev)
        dst_t = torch.empty_like(src_t)
        dst_t.copy_(src_t)
        torch.cuda.synchronize()
        del src_t, dst_t
        log("[bench] calibration copy: 1 GiB read + 1 GiB written")
    out = {"survey": run_survey, "ensemble": run_ensemble, "serve": run_serve,
           "small": run_small, "born": run_born, "codec": run_codec, "bet": run_bet,
           "maps": run_maps}[args.workload](args)
    print(json.dumps(out), flush=True)


def _base_record(args, value, ms_per_step, config, unit="grid-pt updates/s"):
    return {
        "metric": "RTM grid-pt updates/s + images/s (batched/served vs plain), p99 latency, %HBM roofline",
        "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic", "config": config,
    }


def _plain_rate(ctx, grid_for, jobs):
    """Same jobs through rtm_migrate_shot, one after the other (one launch per step)."""
    import torch

    if not jobs:
        return None
    first = jobs[0]
    img = torch.zeros(*first["image_shape"], device="cuda:0")
    ctx.migrate_shot(grid_for(first), first["vel"], first["wav"], first["src"], first["rec"],
                     first["data"], first["ix0"], first["width"], first["opts"], img)
    torch.cuda.synchronize()
    u0 = ctx.stats().grid_updates
    t0 = time.perf_counter()
    for j in jobs:
        ctx.migrate_shot(grid_for(j), j["vel"], j["wav"], j["src"], j["rec"], j["data"], j["ix0"],
                         j["width"], j["opts"], img)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    return {"updates_per_s": (ctx.stats().grid_updates - u0) / el, "images_per_s": len(jobs) / el,
            "shots": len(jobs), "ms_per_image": el * 1e3 / len(jobs)}


def run_survey(args):
    import numpy as np
    import torch

    from paper_2001_06444_amd import inputs, rtm

    dev = torch.device("cuda:0")
    sv = inputs.faulted_survey(n_shots=args.shots, nt=args.nt or 4000)
    nz, nx, nt, nb, h, dt = sv.nz, sv.nx, sv.nt, sv.nb, sv.h, sv.dt
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device=dev)
    vel_true, vel_mig, wav = t(sv.vel_true), t(sv.vel_mig), t(sv.wavelet)
    grid = rtm.make_grid(nz, nx, nb, nt, h, h, dt)

    # arena: working set of every shot of the batch plus slack
    field = ((nz + 2 * nb + 63) // 64 * 64 + 18) * ((nx + 2 * nb + 4 + 63) // 64 * 64) * 4
    ring = nt * 8 * (nz + nx - 8) * 4
    # four buffers per wavefield and shot; the shots share one c
    per_shot = 8 * field + ring + nz * nx * 4 + nt * 256 + nx * 8 + 8192
    arena = int(len(sv.shots) * per_shot * 1.02) + field + (256 << 20)
    log(f"[bench] survey {sv.name}: {len(sv.shots)} shots, nt={nt}, arena {arena / 2**30:.1f} GiB")
    ctx = rtm.Context(0, arena_bytes=arena)

    # ---- observed data: true-model minus smooth-model traces, modelled on the GPU ----
    t0 = time.perf_counter()
    data = []
    for k, sh in enumerate(sv.shots):
        a = torch.empty(nt, len(sh.rec), device=dev)
        b = torch.empty(nt, len(sh.rec), device=dev)
        ctx.propagate(grid, vel_true, wav, sh.src, sh.rec, a)
        ctx.propagate(grid, vel_mig, wav, sh.src, sh.rec, b)
        a.sub_(b)
        data.append(a)
        del b
    torch.cuda.synchronize()
    log(f"[bench] modelled {len(data)} shot records in {time.perf_counter() - t0:.1f} s")
    shots = [(sh.src, sh.ix0, sh.width, sh.rec, d) for sh, d in zip(sv.shots, data)]
    opts = rtm.img_opts("reconstruct")
    image = torch.zeros(nz, nx, device=dev)

    def step():
        image.zero_()
        ctx.migrate_batch(grid, vel_mig, wav, shots, opts, image)

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"[bench] warmup step {i + 1}/{args.warmup} done")
    s0 = ctx.stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
        log(f"[bench] timed step {i + 1}/{args.steps} enqueued")
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    s1 = ctx.stats()
    updates = s1.grid_updates - s0.grid_updates
    ms_per_step = el * 1e3 / args.steps
    value = updates / el
    images_per_s = len(shots) * args.steps / el
    log(f"[bench] batched: {ms_per_step:.1f} ms/step, {value:.3e} updates/s, "
        f"{images_per_s:.1f} images/s")

    # Phase-level rates of the timed steps: algorithmic bytes of all the
    # phase's launches over its time (HIP events on the work stream).  By
    # default the shot groups alternate between two streams whose launches
    # overlap, so these rates are the figure of the production setting.
    gfw, gbw = max(1, s1.last_groups_fwd), max(1, s1.last_groups_bwd)
    phase = {"streams": group_streams(),
             "shot_groups": {"forward": gfw, "backward": gbw},
             "tile_z2": {"forward": s1.last_tile_z2_fwd, "backward": s1.last_tile_z2_bwd},
             "backward_GBps": s1.last_bwd_launch_bytes * s1.last_bwd_launches / (s1.last_bwd_ms * 1e-3) / 1e9,
             "forward_GBps": s1.last_fwd_launch_bytes * s1.last_fwd_launches / (s1.last_fwd_ms * 1e-3) / 1e9}
    phase["backward_frac"] = phase["backward_GBps"] / HBM_PEAK_GBS
    log(f"[bench] timed steps ({phase['streams']} streams, {gbw} backward / {gfw} forward groups): backward "
        f"phase {phase['backward_GBps']:.0f} GB/s ({phase['backward_frac']:.3f} of peak), forward phase "
        f"{phase['forward_GBps']:.0f} GB/s")

    # Dominant kernel: the backward step, timed in isolation.  One more
    # migration runs its shot groups on one stream (RTM_GROUP_STREAMS=1), so
    # its launches follow one another and a launch's duration is defined (a
    # profiler that serialises kernels sees the same durations).  The library
    # reports per-time-step figures over all shots; a launch advances `spl`
    # steps of one group of shots, so its mean algorithmic bytes are spl x
    # the per-step minimum (16 B per update and the rest, summed over the
    # shots) / groups, and its mean duration the phase time x spl / (steps x
    # groups).
    old_streams = os.environ.get("RTM_GROUP_STREAMS")
    os.environ["RTM_GROUP_STREAMS"] = "1"
    try:
        step()
        torch.cuda.synchronize()
        k1 = ctx.stats()
    finally:
        if old_streams is None:
            os.environ.pop("RTM_GROUP_STREAMS", None)
        else:
            os.environ["RTM_GROUP_STREAMS"] = old_streams
    spl = max(1, k1.last_steps_per_launch)
    kfw, kbw = max(1, k1.last_groups_fwd), max(1, k1.last_groups_bwd)
    bwd_launch_ms = spl * k1.last_bwd_ms / (k1.last_bwd_launches * kbw)
    fwd_launch_ms = spl * k1.last_fwd_ms / (k1.last_fwd_launches * kfw)
    bwd_launch_bytes = spl * k1.last_bwd_launch_bytes / kbw
    fwd_launch_bytes = spl * k1.last_fwd_launch_bytes / kfw
    achieved = bwd_launch_bytes / (bwd_launch_ms * 1e-3) / 1e9
    achieved_fwd = fwd_launch_bytes / (fwd_launch_ms * 1e-3) / 1e9
    log(f"[bench] backward launch ({spl} steps, {len(shots) / kbw:.1f} shots) {bwd_launch_ms * 1e3:.1f} us, "
        f"{achieved:.0f} GB/s; forward launch ({len(shots) / kfw:.1f} shots) {fwd_launch_ms * 1e3:.1f} us, "
        f"{achieved_fwd:.0f} GB/s")

    # ---- plain path: one rtm_migrate_shot per shot, one launch per step ----
    plain = None
    if args.plain_shots > 0:
        pimg = torch.zeros(nz, nx, device=dev)
        sel = shots[: args.plain_shots]
        src, ix0, wd, rec, d = sel[0]
        ctx.migrate_shot(grid, vel_mig, wav, src, rec, d, ix0, wd, opts, pimg)  # warm-up
        torch.cuda.synchronize()
        p0 = ctx.stats().grid_updates
        t1 = time.perf_counter()
        for (src, ix0, wd, rec, d) in sel:
            ctx.migrate_shot(grid, vel_mig, wav, src, rec, d, ix0, wd, opts, pimg)
        torch.cuda.synchronize()
        pel = time.perf_counter() - t1
        pup = ctx.stats().grid_updates - p0
        plain = {"updates_per_s": pup / pel, "images_per_s": len(sel) / pel, "shots": len(sel),
                 "ms_per_image": pel * 1e3 / len(sel)}
        log(f"[bench] plain: {plain['ms_per_image']:.1f} ms/image, {plain['updates_per_s']:.3e} updates/s")

    base = None
    if not args.no_cpu_baseline:
        log(f"[bench] timing the FP64 oracle on {args.cpu_nt} steps of one shot ...")
        base = cpu_baseline(sv, args.cpu_nt)
        log(f"[bench] oracle: {base['value']:.3e} updates/s on {base['cores']} threads")

    copy_gbs = copy_rate_gbs()
    log(f"[bench] device copy of 1 GiB: {copy_gbs:.0f} GB/s (read + written); backward launch "
        f"{achieved / copy_gbs:.2f}x of it")
    ctx.close()
    out = _base_record(args, value, ms_per_step, {
        "workload": f"faulted-layer survey {nz}x{nx} at 10 m, {len(shots)} shots, nt={nt}, "
                    f"nb={nb}, reconstruct mode, stacked",
        "nz": nz, "nx": nx, "nb": nb, "nt": nt, "shots": len(shots), "src_mode": "reconstruct",
        "path": "batched (hipGraph, shot groups sized for the memory-side cache, alternating between "
                f"{phase['streams']} streams)", "tile_z": s1.tile_z,
        "tile_z2": {"forward": s1.last_tile_z2_fwd, "backward": s1.last_tile_z2_bwd},
        "shot_groups": {"forward": gfw, "backward": gbw}})
    out.update({
        "images_per_s": images_per_s,
        "plain": plain,
        "batched_vs_plain": (images_per_s / plain["images_per_s"]) if plain else None,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "copy_GBps": copy_gbs, "frac_of_copy": achieved / copy_gbs,
                     "traffic": measured_traffic(launch={"tile_z2": k1.last_tile_z2_bwd,
                                                         "groups": kbw, "shots": len(shots)}),
                     "kernel": (f"k_step2<{k1.last_tile_z2_bwd},2> backward, two time steps "
                                "per launch" if spl == 2 else "k_step<TZ,2> backward")
                               + " (receiver step + reconstruct + imaging); timed on one stream "
                                 "(launches do not overlap)",
                     "steps_per_launch": spl,
                     "shots_per_launch": len(shots) / kbw,
                     "shot_groups": {"forward": kfw, "backward": kbw},
                     "alg_bytes_per_launch": bwd_launch_bytes,
                     "launch_us": bwd_launch_ms * 1e3,
                     "forward_launch": {"achieved": achieved_fwd, "launch_us": fwd_launch_ms * 1e3,
                                        "alg_bytes_per_launch": fwd_launch_bytes}},
        "cpu_baseline": base,
        "phase_rates": phase,
    })
    del ctx
    torch.cuda.empty_cache()
    if not args.no_ensemble:
        # the batched UQ ensemble on the same GPU: 64 velocity samples x 16
        # shots = 1024 RTMs, all submitted at once to the serving engine
        out["ensemble"] = _ensemble(args, args.realizations, 3000, plain_shots=0)
        torch.cuda.empty_cache()
    if not args.no_serve:
        # the served path on the same GPU: the Poisson stream (percentiles from
        # its timed jobs only), then every job of it again at t = 0
        n_warm, n_timed = args.default_serve_warmup, args.default_serve_jobs
        res = _serve(args, n_warm, n_timed, saturation=True)
        res["workload"] = (f"served stream: Poisson {args.rate} jobs/s, {n_timed} timed jobs after {n_warm} "
                           "warm-up, 256 velocity samples, apertures 301-1701, nt 2000-4000, store mode "
                           "stride 4 fp32/bf16, FP64 per-realization mean/std")
        out["served"] = res
    return out



def _ensemble_setup(nz=351, nx=1701, h=10.0):
    from paper_2001_06444_amd import inputs

    base = inputs.ensemble_base(nz, nx, h)
    smooth = inputs.smooth_slowness(base, 40.0, h, h)
    return base, smooth


def _model_window_data(ctx, grid, vel_true, vel_mig, wav, src, ix0, width, nt):
    """Observed data of one shot on its window columns: true minus smooth model."""
    import torch

    from paper_2001_06444_amd import rtm

    g = rtm.make_grid(grid.nz, grid.nx, grid.nb, nt, grid.dz, grid.dx, grid.dt)
    rec = [(1, x) for x in range(ix0, ix0 + width)]
    a = torch.empty(nt, width, device="cuda:0")
    b = torch.empty(nt, width, device="cuda:0")
    ctx.propagate(g, vel_true, wav, src, rec, a)
    ctx.propagate(g, vel_mig, wav, src, rec, b)
    a.sub_(b)
    return a


def _job_bytes(nz, width, nb, nt, mode="reconstruct", dtype="fp32", stride=1):
    field = ((nz + 2 * nb + 63) // 64 * 64 + 18) * ((width + 2 * nb + 4 + 63) // 64 * 64) * 4
    b = 9 * field + nz * width * 4 + nt * 256 + width * 8 + 16384  # c and four buffers per wavefield
    if mode == "reconstruct":
        b += nt * 8 * (nz + width - 8) * 4
    else:
        b += ((nt - 2) // stride + 1) * nz * width * (4 if dtype == "fp32" else 2)
    return b


def _ensemble(args, R, nt, plain_shots):
    """R velocity samples x 16 shots with uneven apertures, all submitted at
    once to the serving engine (continuous batching, tuned tiles);
    per-realization stacks, then FP64 mean/std over the stacks and the
    Stage-3 confidence map.  Returns the rates and, with plain_shots > 0,
    the same shots through the plain path."""
    import numpy as np
    import torch

    from paper_2001_06444_amd import inputs, rtm

    dev = torch.device("cuda:0")
    nz, nx, h, dt, nb = 351, 1701, 10.0, 1e-3, 50
    base, smooth = _ensemble_setup(nz, nx, h)
    shots = inputs.ensemble_shots(16, nx)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device=dev)
    wav = t(inputs.ricker(nt, dt))
    grid = rtm.make_grid(nz, nx, nb, nt, h, h, dt)
    need = sum(_job_bytes(nz, sh.width, nb, nt) for sh in shots) * R
    free = torch.cuda.mem_get_info()[0]
    arena = int(min(need * 1.05 + (2 << 30), free - (24 << 30)))
    log(f"[bench] ensemble: {R} realizations x {len(shots)} shots, nt={nt}; jobs need "
        f"{need / 2**30:.1f} GiB, arena {arena / 2**30:.1f} GiB")
    ctx = rtm.Context(0, arena_bytes=arena)
    vt, vs = t(base), t(smooth)
    data = [_model_window_data(ctx, grid, vt, vs, wav, sh.src, sh.ix0, sh.width, nt) for sh in shots]
    for r in range(R):
        ctx.model_register(r, t(smooth * (1.0 + 0.05 * inputs.grf(r, nz, nx, h))), grid)
    ctx.model_register(R, vs, grid)  # warm-up model
    torch.cuda.synchronize()
    log("[bench] data modelled, velocity bank registered")
    opts = rtm.img_opts("reconstruct")
    # warm-up (tile tuning, graph capture) on a model outside the ensemble
    for sh, d in zip(shots[:2], data[:2]):
        ctx.submit(R, sh.src, sh.ix0, sh.width, 1, nt, wav, d, opts)
    ctx.drain()
    s0 = ctx.stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tickets = []
    for r in range(R):
        for sh, d in zip(shots, data):
            tickets.append(ctx.submit(r, sh.src, sh.ix0, sh.width, 1, nt, wav, d, opts,
                                      flags=rtm.JOB_ACC_STACK))
    ctx.drain()
    t_rtm = time.perf_counter() - t0
    st = ctx.stats_create(nz, nx)
    buf = torch.empty(nz, nx, device=dev)
    for r in range(R):
        ctx.ensemble_stack(r, buf)
        ctx.stats_add(st, buf)
    mean = torch.empty(nz, nx, dtype=torch.float64, device=dev)
    std = torch.empty_like(mean)
    cnt = torch.empty(nz, nx, dtype=torch.int32, device=dev)
    ctx.stats_get(st, mean, std, cnt)
    conf = torch.empty_like(mean)
    ctx.confidence_map(std, cnt, conf)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    s1 = ctx.stats()
    n_img = R * len(shots)
    failed = sum(1 for tk in tickets if ctx.poll(tk, release=True).state != rtm.JOB_DONE)
    updates = s1.grid_updates - s0.grid_updates
    alg = s1.alg_bytes - s0.alg_bytes  # per-update minimum bytes of the finished jobs
    log(f"[bench] ensemble: {n_img} RTMs in {el:.2f} s ({n_img / el:.1f} images/s, "
        f"{updates / el:.3e} updates/s, {alg / t_rtm / 1e9:.0f} GB/s of algorithmic bytes over the "
        f"served phase), {failed} failed, tile_z {s1.tile_z}")
    plain_jobs = [dict(vel=t(smooth), wav=wav, src=sh.src, rec=[(1, x) for x in range(sh.ix0, sh.ix0 + sh.width)],
                       data=d, ix0=sh.ix0, width=sh.width, opts=opts, image_shape=(nz, nx))
                  for sh, d in list(zip(shots, data))[:plain_shots]]
    plain = _plain_rate(ctx, lambda j: grid, plain_jobs)
    ctx.close()
    return {
        "workload": f"velocity ensemble: {R} realizations x {len(shots)} shots on {nz}x{nx} at 10 m, "
                    f"apertures 401-1201 columns, nt={nt}, nb={nb}, reconstruct mode, "
                    f"FP64 mean/std over realization stacks",
        "rtms": n_img, "seconds": el, "rtm_seconds": t_rtm,
        "updates_per_s": updates / el, "images_per_s": n_img / el, "realization_images_per_s": R / el,
        "failed_jobs": failed, "tile_z": s1.tile_z, "path": "served engine, all jobs at t=0",
        # the jobs' algorithmic bytes (per-update minimum) over the wall time of
        # the served phase, submit to drain: a lower bound on the step kernels'
        # own rate, gaps between launches included
        "served_roofline": {"bound": "hbm", "achieved": alg / t_rtm / 1e9, "peak": HBM_PEAK_GBS,
                            "unit": "GB/s", "frac": alg / t_rtm / 1e9 / HBM_PEAK_GBS,
                            "alg_bytes": alg, "seconds": t_rtm},
        "plain": plain, "batched_vs_plain": (n_img / el) / plain["images_per_s"] if plain else None,
        "std_map": {"max": float(std.max()), "mean": float(std.mean())},
    }


def run_ensemble(args):
    """The velocity ensemble alone (value: its grid-point updates/s)."""
    nt = args.nt or 3000
    res = _ensemble(args, args.realizations, nt, args.plain_shots)
    out = _base_record(args, res["updates_per_s"], res["seconds"] * 1e3, {
        "workload": res["workload"], "realizations": args.realizations, "shots": 16, "nt": nt,
        "path": res["path"], "tile_z": res["tile_z"]})
    out.update({"steps": 1, "warmup": 1, "images_per_s": res["images_per_s"],
                "realization_images_per_s": res["realization_images_per_s"], "rtm_seconds": res["rtm_seconds"],
                "failed_jobs": res["failed_jobs"], "plain": res["plain"],
                "batched_vs_plain": res["batched_vs_plain"], "std_map": res["std_map"]})
    return out


def _serve(args, n_warm, n_timed, saturation, extra_rates=()):
    """Poisson stream of RTM jobs (velocity sample, shot, aperture, nt, snapshot
    dtype) served by continuous batching; latency = completion - arrival,
    including queueing and the upload of the job's data.  Returns the
    latency percentiles and served rate of the timed jobs, and with
    `saturation` also a run with every job arriving at t = 0."""
    import numpy as np
    import torch

    from paper_2001_06444_amd import inputs, rtm

    dev = torch.device("cuda:0")
    nz, nx, h, dt, nb = 351, 1701, 10.0, 1e-3, 50
    base, smooth = _ensemble_setup(nz, nx, h)
    n_all = n_warm + n_timed
    stream = inputs.poisson_stream(n_all, rate=args.rate, seed=5, n_real=256, nx=nx)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device=dev)
    ntmax = max(j.nt for j in stream)
    wav = t(inputs.ricker(ntmax, dt))
    grid = rtm.make_grid(nz, nx, nb, ntmax, h, h, dt)
    free = torch.cuda.mem_get_info()[0]
    arena = int(min(96 << 30, free - (32 << 30)))
    ctx = rtm.Context(0, arena_bytes=arena)
    vt, vs = t(base), t(smooth)
    used = sorted({j.realization for j in stream})
    for r in used:
        ctx.model_register(r, t(smooth * (1.0 + 0.05 * inputs.grf(r, nz, nx, h))), grid)
    log(f"[bench] serve: {n_all} jobs at {args.rate} jobs/s, {len(used)} realizations, "
        f"arena {arena / 2**30:.1f} GiB")
    host = []
    for j in stream:
        d = _model_window_data(ctx, grid, vt, vs, wav, j.src, j.ix0, j.width, j.nt)
        hd = torch.empty(d.shape, dtype=torch.float32, pin_memory=True)
        hd.copy_(d)
        host.append(hd)
        del d
    torch.cuda.synchronize()
    log("[bench] job data modelled and staged in pinned host memory")

    def opts_of(j):
        return rtm.img_opts("store", j.dtype, 4)

    def serve(arrivals):
        pending, done = {}, {}
        t0 = time.monotonic()
        for i, j in enumerate(stream):
            while True:
                now = time.monotonic()
                for tk in [tk for tk in list(pending)]:
                    info = ctx.poll(tk)
                    if info.state >= rtm.JOB_DONE:
                        done[pending[tk][0]] = (info.state, info.t_done)
                        ctx.poll(tk, release=True)
                        del pending[tk]
                if now >= t0 + arrivals[i]:
                    break
                time.sleep(min(0.002, t0 + arrivals[i] - now))
            d = host[i].to(dev)
            tk = ctx.submit(j.realization, j.src, j.ix0, j.width, 1, j.nt, wav, d, opts_of(j),
                            flags=rtm.JOB_ACC_STATS, tag=i)
            pending[tk] = (i, d)
        ctx.drain()
        for tk, (i, d) in pending.items():
            info = ctx.poll(tk, release=True)
            done[i] = (info.state, info.t_done)
        lat = np.array([done[i][1] - (t0 + arrivals[i]) for i in range(len(stream))])
        ok = np.array([done[i][0] == rtm.JOB_DONE for i in range(len(stream))])
        t_end = max(done[i][1] for i in range(len(stream))) - t0
        return lat, ok, t_end

    arrivals = [j.arrival for j in stream]
    lat, ok, t_end = serve(arrivals)
    lt = lat[n_warm:]
    span = t_end - arrivals[n_warm]
    res = {"rate": args.rate, "jobs": n_timed, "warmup_jobs": n_warm,
           "latency_ms": {"p50": float(np.percentile(lt, 50)) * 1e3, "p99": float(np.percentile(lt, 99)) * 1e3,
                          "max": float(lt.max()) * 1e3},
           "images_per_s": n_timed / span, "failed_jobs": int((~ok).sum())}
    log(f"[bench] serve @ {args.rate}/s: p50 {res['latency_ms']['p50']:.0f} ms, "
        f"p99 {res['latency_ms']['p99']:.0f} ms, {res['images_per_s']:.1f} images/s, "
        f"{res['failed_jobs']} failed")
    for rate in extra_rates:  # the same jobs at another rate: arrival times scaled
        lat_r, ok_r, t_end_r = serve([a * args.rate / rate for a in arrivals])
        lr = lat_r[n_warm:]
        span_r = t_end_r - arrivals[n_warm] * args.rate / rate
        res.setdefault("other_rates", []).append(
            {"rate": rate, "latency_ms": {"p50": float(np.percentile(lr, 50)) * 1e3,
                                          "p99": float(np.percentile(lr, 99)) * 1e3, "max": float(lr.max()) * 1e3},
             "images_per_s": n_timed / span_r, "failed_jobs": int((~ok_r).sum())})
        log(f"[bench] serve @ {rate}/s: p50 {np.percentile(lr, 50) * 1e3:.0f} ms, "
            f"p99 {np.percentile(lr, 99) * 1e3:.0f} ms, {n_timed / span_r:.1f} images/s")
    if saturation:  # every job arrives at t = 0
        st0 = ctx.stats()
        u0, a0 = st0.grid_updates, st0.alg_bytes
        lat0, ok0, t_end0 = serve([0.0] * n_all)
        st1 = ctx.stats()
        # the jobs' algorithmic bytes (per-update minimum of every job, each
        # with its own c) over the run's wall time
        alg = st1.alg_bytes - a0
        res["saturation"] = {"jobs": n_all, "seconds": t_end0, "images_per_s": n_all / t_end0,
                             "updates_per_s": (st1.grid_updates - u0) / t_end0,
                             "latency_ms": {"p50": float(np.percentile(lat0, 50)) * 1e3,
                                            "p99": float(np.percentile(lat0, 99)) * 1e3},
                             "failed_jobs": int((~ok0).sum()),
                             "served_roofline": {"bound": "hbm", "achieved": alg / t_end0 / 1e9,
                                                 "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                                 "frac": alg / t_end0 / 1e9 / HBM_PEAK_GBS,
                                                 "alg_bytes": alg, "seconds": t_end0}}
        log(f"[bench] saturation: {n_all} jobs in {t_end0:.2f} s, {n_all / t_end0:.1f} images/s, "
            f"{res['saturation']['updates_per_s']:.3e} updates/s, {alg / t_end0 / 1e9:.0f} GB/s of "
            "algorithmic bytes")
    ctx.close()
    return res


def run_serve(args):
    """The served stream at full length, plus its saturation run."""
    rates = [float(r) for r in args.rates.split(",") if r.strip()]
    res = _serve(args, args.serve_warmup, args.serve_jobs, saturation=True, extra_rates=rates)
    sat = res["saturation"]
    out = _base_record(args, sat["updates_per_s"], sat["seconds"] * 1e3, {
        "workload": f"served stream: Poisson {args.rate} jobs/s, {args.serve_jobs} timed jobs "
                    f"(+{args.serve_warmup} warm-up), 256 velocity samples, apertures 301-1701, "
                    f"nt 2000-4000, store mode stride 4 fp32/bf16, FP64 per-realization mean/std",
        "rate": args.rate, "jobs": args.serve_jobs, "path": "served engine (continuous batching)"})
    out.update({"steps": 1, "warmup": 0,
                "latency_ms": res["latency_ms"],
                "served_images_per_s": res["images_per_s"], "saturation_images_per_s": sat["images_per_s"],
                "failed_jobs": res["failed_jobs"] + sat["failed_jobs"],
                "other_rates": res.get("other_rates", []),
                "value_is": "grid-pt updates/s of the saturation run"})
    return out


def run_small(args):
    """The small two-layer survey (101 x 201, nt 1000), where one shot is ~2000
    tiny launches: many shots batched per launch from graph replays versus
    one rtm_migrate_shot per shot."""
    import numpy as np
    import torch

    from paper_2001_06444_amd import inputs, rtm

    dev = torch.device("cuda:0")
    sv = inputs.two_layer_shot_survey(nt=args.nt or 1000)
    nz, nx, nt, nb, h, dt = sv.nz, sv.nx, sv.nt, sv.nb, sv.h, sv.dt
    n = args.shots if args.shots != 100 else 256
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device=dev)
    vt, vm, wav = t(sv.vel_true), t(sv.vel_mig), t(sv.wavelet)
    grid = rtm.make_grid(nz, nx, nb, nt, h, h, dt)
    ctx = rtm.Context(0, arena_bytes=int(n * _job_bytes(nz, nx, nb, nt) * 1.1) + (256 << 20))
    xs = np.linspace(5, nx - 6, n).round().astype(int)
    rec = [(1, x) for x in range(nx)]
    data = []
    for x in xs:
        a = torch.empty(nt, nx, device=dev)
        b = torch.empty(nt, nx, device=dev)
        ctx.propagate(grid, vt, wav, (1, int(x)), rec, a)
        ctx.propagate(grid, vm, wav, (1, int(x)), rec, b)
        data.append(a.sub_(b))
    shots = [((1, int(x)), 0, nx, rec, d) for x, d in zip(xs, data)]
    opts = rtm.img_opts("reconstruct")
    image = torch.zeros(nz, nx, device=dev)
    for _ in range(args.warmup):
        ctx.migrate_batch(grid, vm, wav, shots, opts, image)
    torch.cuda.synchronize()
    u0 = ctx.stats().grid_updates
    t0 = time.perf_counter()
    for _ in range(args.steps):
        image.zero_()
        ctx.migrate_batch(grid, vm, wav, shots, opts, image)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    upd = ctx.stats().grid_updates - u0
    ips = n * args.steps / el
    plain_jobs = [dict(vel=vm, wav=wav, src=s[0], rec=rec, data=s[4], ix0=0, width=nx, opts=opts,
                       image_shape=(nz, nx)) for s in shots[: max(args.plain_shots, 4)]]
    plain = _plain_rate(ctx, lambda j: grid, plain_jobs)
    log(f"[bench] small: {n} shots batched {ips:.0f} images/s ({upd / el:.3e} updates/s); plain "
        f"{plain['images_per_s']:.0f} images/s ({plain['ms_per_image']:.2f} ms/image)")
    ctx.close()
    out = _base_record(args, upd / el, el * 1e3 / args.steps, {
        "workload": f"two-layer survey {nz}x{nx} at 10 m, nt={nt}, nb={nb}, {n} shots per batch, "
                    f"reconstruct mode", "shots": n, "nt": nt, "path": "batched (hipGraph)"})
    out.update({"images_per_s": ips, "plain": plain, "batched_vs_plain": ips / plain["images_per_s"]})
    return out


def run_born(args):
    """Born modelling of survey shots at full size: the shots one after the
    other through rtm_born (one launch per step and shot), then the same
    shots together through rtm_born_batch (one launch per step advancing
    every shot's background and scattered field)."""
    import numpy as np
    import torch

    from paper_2001_06444_amd import inputs, rtm

    dev = torch.device("cuda:0")
    sv = inputs.faulted_survey(n_shots=100, nt=args.nt or 4000)
    nz, nx, nt, nb, h, dt = sv.nz, sv.nx, sv.nt, sv.nb, sv.h, sv.dt
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device=dev)
    vm, wav = t(sv.vel_mig), t(sv.wavelet)
    mpert = t(sv.vel_true - sv.vel_mig)
    grid = rtm.make_grid(nz, nx, nb, nt, h, h, dt)
    ctx = rtm.Context(0, arena_bytes=4 << 30)
    # 16 shots per launch: a launch's time per shot and step falls from 6.6 us
    # (one shot, 792 workgroups) to 4.7 us at 12 shots and stays there
    nsh = 16
    shots = sv.shots[:: len(sv.shots) // nsh][:nsh]
    dd = [torch.empty(nt, len(sh.rec), device=dev) for sh in shots]
    ctx.born(grid, vm, wav, shots[0].src, mpert, shots[0].rec, dd[0])  # warm-up (tiles tuned)
    ctx.born_batch(grid, vm, wav, mpert, [(sh.src, sh.rec, d) for sh, d in zip(shots, dd)])
    torch.cuda.synchronize()

    def timed(fn):
        u0 = ctx.stats().grid_updates
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1), ctx.stats().grid_updates - u0

    def plain():
        for sh, d in zip(shots, dd):
            ctx.born(grid, vm, wav, sh.src, mpert, sh.rec, d)

    ms_p, upd_p = timed(plain)
    batch = lambda: ctx.born_batch(grid, vm, wav, mpert, [(sh.src, sh.rec, d) for sh, d in zip(shots, dd)])
    ms_b, upd_b = timed(batch)
    ngr_b = max(1, ctx.stats().last_born_groups)
    # the roofline run: the same batch with its shot groups on one stream, so
    # that launches follow one another and a launch's duration is defined
    old_streams = os.environ.get("RTM_GROUP_STREAMS")
    os.environ["RTM_GROUP_STREAMS"] = "1"
    try:
        ms_r, _ = timed(batch)
    finally:
        if old_streams is None:
            os.environ.pop("RTM_GROUP_STREAMS", None)
        else:
            os.environ["RTM_GROUP_STREAMS"] = old_streams
    ngr = max(1, ctx.stats().last_born_groups)  # shot groups: launches cover one group each
    npad, nph = (nz + 2 * nb) * (nx + 2 * nb), nz * nx
    nrec = sum(len(sh.rec) for sh in shots)
    # per step and shot: c 4 B, background 12 B, scattered field 12 B per padded
    # point, m 4 B per physical point, 4 B per receiver sample (the one-step
    # minimum, which a two-step launch undercuts); a batched launch reads c
    # and m once for all the shots of its group
    plain_bytes = npad * 28 + nph * 4 + nrec / nsh * 4
    batch_bytes = (nsh * npad * 24 + ngr * (npad * 4 + nph * 4) + nrec * 4) / ngr
    # launches advance two steps (Born pairs) unless RTM_TILE_Z2=0; the
    # per-launch figures are those of the steps a launch takes
    spl = 1 if os.environ.get("RTM_TILE_Z2") == "0" else 2
    plain_us = spl * ms_p * 1e3 / (nsh * (nt - 1))
    batch_us = spl * ms_r * 1e3 / (ngr * (nt - 1))
    plain_bytes, batch_bytes = spl * plain_bytes, spl * batch_bytes
    gbs_p = plain_bytes / (plain_us * 1e-6) / 1e9
    gbs_b = batch_bytes / (batch_us * 1e-6) / 1e9
    log(f"[bench] born, {nsh} shots one by one: {upd_p / (ms_p * 1e-3):.3e} updates/s, {plain_us:.1f} us/launch "
        f"({spl} steps), {gbs_p:.0f} GB/s")
    log(f"[bench] born, {nsh} shots batched in {ngr_b} shot groups: {upd_b / (ms_b * 1e-3):.3e} updates/s")
    log(f"[bench] born, roofline run ({ngr} shot groups on one stream): {upd_b / (ms_r * 1e-3):.3e} updates/s, "
        f"{batch_us:.1f} us/launch ({spl} steps, {nsh / ngr:.1f} shots), {gbs_b:.0f} GB/s")
    ctx.close()
    out = _base_record(args, upd_b / (ms_b * 1e-3), ms_b, {
        "workload": f"Born modelling, faulted-layer survey {nz}x{nx}, nt={nt}, nb={nb}, {nsh} shots "
                    "in shared launches", "path": "batched (shot groups sized for the memory-side cache, "
                    "each launch advancing every shot of its group; groups alternating between the group streams)",
        "shot_groups": ngr_b})
    out.update({"steps": 1, "warmup": 1,
                "plain": {"updates_per_s": upd_p / (ms_p * 1e-3), "launch_us": plain_us, "GB_per_s": gbs_p,
                          "alg_bytes_per_launch": plain_bytes},
                "batched_vs_plain": ms_p / ms_b,
                "roofline": {"bound": "hbm", "achieved": gbs_b, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": gbs_b / HBM_PEAK_GBS,
                             "traffic": measured_traffic("traffic_born_pair.json",
                                                         launch={"groups": ngr, "shots": nsh}),
                             "kernel": (f"k_step2<TZ2,4> Born pair (two steps per launch)" if spl == 2 else
                                        "k_step<TZ,4> Born step") + f" over {nsh / ngr:.1f} shots (background and "
                                       "scattered field)",
                             "steps_per_launch": spl,
                             "alg_bytes_per_launch": batch_bytes, "launch_us": batch_us, "shot_groups": ngr,
                             "note": "events around the whole call with the shot groups on one stream "
                                     "(launches do not overlap), launch gaps included"}})
    return out

# Algorithmic bytes per pixel of the Stage-3 maps and the filter: every input
# read once, every output written once.
MAPS_BYTES = {"confidence": 8 + 4 + 8, "ratio": 8 + 8 + 8, "laplacian_filter": 4 + 4, "normalize": 4 + 4 + 4}


def run_maps(args):
    """The Stage-3 maps (confidence index, std/mean ratio), the post-stack
    Laplacian filter and the source-normalised image, over one image of the
    paper's size (351 x 1701) and over a bank of 256 such images side by side
    (the size of the serving configuration's Welford state; the filter
    launches one row of workgroups per image row).  Each call
    is timed with HIP events around 20 calls on the library's stream; the
    confidence index and the normalised image take two passes (a reduction,
    then the map), counted in their time but not in their bytes."""
    import torch

    from paper_2001_06444_amd import rtm

    dev = torch.device("cuda:0")
    gen = torch.Generator(device=dev)
    gen.manual_seed(11)
    ctx = rtm.Context(0, arena_bytes=64 << 20)
    K, rows = 20, {}
    for label, (rz, rx) in {"image": (351, 1701), "bank": (351, 256 * 1701)}.items():
        n = rz * rx
        std = torch.rand(n, dtype=torch.float64, device=dev, generator=gen)
        mean = torch.randn(n, dtype=torch.float64, device=dev, generator=gen)
        cnt = torch.randint(0, 8, (n,), dtype=torch.int32, device=dev, generator=gen)
        img = torch.randn(rz, rx, device=dev, generator=gen)
        ill = torch.rand(rz, rx, device=dev, generator=gen)
        o64 = torch.empty(n, dtype=torch.float64, device=dev)
        o32 = torch.empty(rz, rx, device=dev)
        calls = {"confidence": lambda: ctx.confidence_map(std, cnt, o64, min_count=2),
                 "ratio": lambda: ctx.ratio_map(std, mean, o64, eps=1e-3),
                 "laplacian_filter": lambda: ctx.laplacian_filter(img, 10.0, 10.0, o32),
                 "normalize": lambda: ctx.normalize_image(img, ill, o32, eps_rel=1e-3)}
        for name, fn in calls.items():
            for _ in range(3):
                fn()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(K):
                fn()
            e1.record()
            torch.cuda.synchronize()
            us = e0.elapsed_time(e1) * 1e3 / K
            alg = MAPS_BYTES[name] * n
            rows[f"{name} {label}"] = {"pixels": n, "us": us, "alg_bytes": alg, "GB_per_s": alg / (us * 1e-6) / 1e9}
            log(f"[bench] maps: {name:16s} {label:5s} {n:10d} px {us:9.1f} us {rows[f'{name} {label}']['GB_per_s']:7.0f} GB/s")
        del std, mean, cnt, img, ill, o64, o32
    ctx.close()
    bank = {k: v for k, v in rows.items() if k.endswith("bank")}
    tot_b, tot_us = sum(v["alg_bytes"] for v in bank.values()), sum(v["us"] for v in bank.values())
    dom = max(bank, key=lambda k: bank[k]["us"])
    out = _base_record(args, tot_b / (tot_us * 1e-6) / 1e9, tot_us * 1e-3, {
        "workload": "Stage-3 maps + post-stack filter + normalised image over 256 351x1701 images side by side "
                    "(and one image)", "pixels": bank[dom]["pixels"]}, unit="GB/s")
    out.update({"metric": "Stage-3 maps: algorithmic GB/s", "steps": K, "warmup": 3, "dtype": "f64/f32",
                "maps": rows,
                "roofline": {"bound": "hbm", "achieved": bank[dom]["GB_per_s"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": bank[dom]["GB_per_s"] / HBM_PEAK_GBS, "traffic": None,
                             "kernel": dom.split()[0] + " (bank)"}})
    return out


CODEC_SETTINGS = {"velocity": (1e-4, 1e-1, None), "image": (1e-4, 1e-1, None), "seismogram": (1e-4, None)}
# the ZFP-method coder (RTM_CODEC_ZFP) at the paper's two fixed-accuracy bounds
ZFP_SETTINGS = (1e-4, 1e-1)


def _codec_label(kind, tol):
    return f"{kind} {'lossless' if tol is None else f'tol {tol:g}'}"


def codec_cpu_baseline(banks, budget_s=12.0):
    """The codec oracle (NumPy) on the first arrays of each bank, every setting,
    until the time budget is spent."""
    import numpy as np

    from oracle import codec as zc

    done_bytes, el, arrays = 0, 0.0, []
    for i in range(max(len(b) for b in banks.values())):
        for kind, bank in banks.items():
            if i >= len(bank) or el >= budget_s:
                continue
            for tol in CODEC_SETTINGS[kind]:
                t0 = time.perf_counter()
                w = zc.encode(bank[i], tol=tol) if tol else zc.encode(bank[i], mode=zc.MODE_LOSSLESS)
                zc.decode(w)
                el += time.perf_counter() - t0
                done_bytes += 2 * bank[i].nbytes
            arrays.append(f"{kind}[{i}]")
        if el >= budget_s:
            break
    return {"value": done_bytes / el / 1e9, "unit": "GB/s (uncompressed bytes encoded + decoded)",
            "cores": 1, "kind": "oracle",
            "sample": f"{len(arrays)} arrays ({', '.join(arrays[:6])}{', ...' if len(arrays) > 6 else ''}) "
                      f"in every setting of their bank, encode + decode, {el:.1f} s"}


def run_codec(args):
    """Compression stage (Sec. 3 / Sec. 4.2): encode and decode banks of
    velocity samples, migrated images and seismograms at the paper's error
    bounds (1e-4, 1e-1) and losslessly.  One step = every bank in every
    setting, encoded then decoded."""
    import numpy as np
    import torch

    from paper_2001_06444_amd import inputs, rtm

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    banks = {"velocity": inputs.velocity_bank(args.realizations),
             "image": inputs.image_bank(args.realizations),
             "seismogram": inputs.seismogram_bank(args.seismograms)}
    log(f"[bench] codec inputs in {time.perf_counter() - t0:.1f} s: " +
        ", ".join(f"{k} {tuple(v.shape)}" for k, v in banks.items()))
    ctx = rtm.Context(0, arena_bytes=64 << 20)
    xs = {k: torch.as_tensor(v, device=dev) for k, v in banks.items()}
    bufs = {k: torch.empty(ctx.codec_max_bytes(*v.shape), dtype=torch.uint8, device=dev) for k, v in banks.items()}
    outs = {k: torch.empty_like(v) for k, v in xs.items()}
    runs = {}

    def step(keep):
        for kind, x in xs.items():
            for tol in CODEC_SETTINGS[kind]:
                s = ctx.codec_encode(x, tol=tol, lossless=tol is None, out=bufs[kind])
                st = ctx.stats()
                enc = (st.last_codec_ms, st.last_codec_bytes)
                ctx.codec_decode(s, out=outs[kind])
                st = ctx.stats()
                dec = (st.last_codec_ms, st.last_codec_bytes)
                if keep:
                    r = runs.setdefault(_codec_label(kind, tol), {"enc_ms": [], "dec_ms": [], "bytes_in": x.numel() * 4,
                                                                  "stream_bytes": s.numel(), "enc_alg_bytes": enc[1],
                                                                  "dec_alg_bytes": dec[1]})
                    r["enc_ms"].append(enc[0])
                    r["dec_ms"].append(dec[0])

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    step_bytes = sum(2 * x.numel() * 4 * len(CODEC_SETTINGS[k]) for k, x in xs.items())
    # the round trip is exact for lossless and within the bound otherwise
    for kind, x in xs.items():
        y = ctx.codec_decode(ctx.codec_encode(x, tol=1e-4, out=bufs[kind]), out=outs[kind])
        err = (y.double() - x.double()).abs() - (1e-4 * (1 + 2.0 ** -26) + y.double().abs() * 2.0 ** -24)
        assert float(err.max()) <= 0.0, f"{kind}: error bound violated"
    # the ZFP-method coder on the same banks: ratio, kernel times, error
    zfp_table = {}
    for kind, x in xs.items():
        for tol in ZFP_SETTINGS:
            enc_ms, dec_ms = [], []
            for it in range(args.warmup + args.steps):
                s = ctx.codec_encode(x, tol=tol, zfp=True, out=bufs[kind])
                e_st = ctx.stats()
                y = ctx.codec_decode(s, out=outs[kind])
                d_st = ctx.stats()
                if it >= args.warmup:
                    enc_ms.append(e_st.last_codec_ms)
                    dec_ms.append(d_st.last_codec_ms)
            err = float((y.double() - x.double()).abs().max())
            assert err <= tol, f"ZFP-method coder: {kind} tol {tol:g}: error {err:.3e}"
            e_ms, d_ms = float(np.median(enc_ms)), float(np.median(dec_ms))
            row = {"ratio": x.numel() * 4 / s.numel(), "stream_MB": s.numel() / 1e6, "max_error": err,
                   "encode_us": e_ms * 1e3, "decode_us": d_ms * 1e3,
                   "encode_GBps": x.numel() * 4 / (e_ms * 1e-3) / 1e9,
                   "decode_GBps": x.numel() * 4 / (d_ms * 1e-3) / 1e9}
            zfp_table[_codec_label(kind, tol)] = row
            log(f"[bench] zfp {_codec_label(kind, tol):20s} ratio {row['ratio']:6.2f}  max error {err:.2e}  "
                f"encode {row['encode_us']:8.1f} us  decode {row['decode_us']:8.1f} us")
    table, dominant = {}, None
    for label, r in runs.items():
        e_ms, d_ms = float(np.median(r["enc_ms"])), float(np.median(r["dec_ms"]))
        row = {"ratio": r["bytes_in"] / r["stream_bytes"], "stream_MB": r["stream_bytes"] / 1e6,
               "encode_us": e_ms * 1e3, "decode_us": d_ms * 1e3,
               "encode_GBps_alg": r["enc_alg_bytes"] / (e_ms * 1e-3) / 1e9,
               "decode_GBps_alg": r["dec_alg_bytes"] / (d_ms * 1e-3) / 1e9}
        table[label] = row
        for op, ms, ab in (("encode", e_ms, r["enc_alg_bytes"]), ("decode", d_ms, r["dec_alg_bytes"])):
            if dominant is None or ms > dominant[1]:
                dominant = (f"{op} {label}", ms, ab, op, label)
        log(f"[bench] {label:24s} ratio {row['ratio']:6.2f}  encode {row['encode_us']:8.1f} us "
            f"{row['encode_GBps_alg']:7.0f} GB/s  decode {row['decode_us']:8.1f} us {row['decode_GBps_alg']:7.0f} GB/s")
    name, ms, ab, op, label = dominant
    achieved = ab / (ms * 1e-3) / 1e9
    traffic = measured_traffic("traffic_codec.json", CODEC_SOURCES, key=f"{op} {label}")
    cpu = None if args.no_cpu_baseline else codec_cpu_baseline(
        {k: v[: 8] for k, v in banks.items()}, budget_s=15.0)
    ctx.close()
    out = _base_record(args, step_bytes / (el / args.steps) / 1e9, el * 1e3 / args.steps, {
        "workload": f"compression stage: {args.realizations} velocity samples and {args.realizations} images "
                    f"351x1701, {args.seismograms} seismograms 4000x1701; fixed accuracy 1e-4 and 1e-1 (velocity, "
                    f"image), 1e-4 (seismogram), lossless; encode + decode per step",
        "path": "rtm_codec_encode / rtm_codec_decode, one call per bank and setting"},
        unit="GB/s (uncompressed bytes encoded + decoded)")
    out["metric"] = "codec throughput: uncompressed GB/s encoded + decoded; compression ratios"
    out["dtype"] = "f32 in, int32 transform"
    out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": achieved / HBM_PEAK_GBS,
                       "traffic": None if traffic is None else traffic * 1.0,
                       "kernel": f"k_zc_{op} ({label})",
                       "alg_bytes_per_launch": ab,
                       "note": "algorithmic bytes: 4 B per value plus the stream length; HIP events "
                               "around the launch on the library's stream"}
    out["codec"] = table
    out["zfp_method"] = {"settings": zfp_table,
                         "note": "RTM_CODEC_ZFP: the published ZFP method in fixed-accuracy mode (4 x 4 block "
                                 "floating point, decorrelating lifting transform, negabinary, embedded bit-plane "
                                 "coding); GB/s of uncompressed bytes per kernel time"}
    if cpu is not None:
        out["cpu_baseline"] = cpu
    return out


FLOP_PER_NODE_UPDATE = 10  # Godunov update: 3 min, d, compare, q, q + q, d d, difference, sqrt, sum, halving


def bet_cpu_baseline(p, tt_obs, budget_s=12.0):
    """The Stage-1 oracle running chain 0 alone (single thread) for a bounded time."""
    from oracle import bet as obet

    c = p["cfg"]
    cfg = obet.BetConfig(nz=c["nz"], nx=c["nx"], h=c["h"], chains=1, k_min=c["k_min"], k_max=c["k_max"],
                         k_init=c["k_init"], v_min=c["v_min"], v_max=c["v_max"], p_birth=c["p_birth"],
                         p_death=c["p_death"], move_dz=c["move_dz"], move_dx=c["move_dx"], sigma=c["sigma"],
                         seed=c["seed"], burn_in=c["burn_in"], thin=c["thin"], single=True)
    iters, el = 10, 0.0
    while True:
        t0 = time.perf_counter()
        obet.run(cfg, p["srcs"], p["recs"], tt_obs, iters)
        el = time.perf_counter() - t0
        if el >= budget_s / 3 or iters >= 4000:
            break
        iters *= 2
    return {"value": iters / el, "unit": "chain iterations/s", "cores": 1, "kind": "oracle",
            "sample": f"chain 0 alone, {iters} iterations from its initial model (34 FP32 fast-sweeping "
                      f"solves per valid proposal), {el:.1f} s"}


def run_bet(args):
    """Stage 1 (Sec. 2.1): reversible-jump chains over Voronoi velocity models
    with Eikonal travel times.  One step = --bet-iters iterations of every chain."""
    import numpy as np
    import torch

    from paper_2001_06444_amd import inputs, rtm

    p = inputs.bet_problem(args.chains, args.bet_h)
    c = p["cfg"]
    n = c["nz"] * c["nx"]
    ctx = rtm.Context(0, arena_bytes=256 << 20)
    true = torch.as_tensor(p["true"], dtype=torch.float32, device="cuda")
    tt_obs = ctx.eikonal(true, p["h"], p["srcs"], p["recs"])
    b = ctx.bet_create(p["srcs"], p["recs"], tt_obs, **c)

    def work():
        tot = np.zeros(2, dtype=np.int64)
        info = []
        for ch in range(c["chains"]):
            g = ctx.bet_chain(b, ch, c["k_max"])
            tot += (g["solves"], g["sweeps"])
            info.append(g)
        return tot, info

    for _ in range(args.warmup):
        ctx.bet_run(b, args.bet_iters)
    torch.cuda.synchronize()
    w0, _ = work()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.bet_run(b, args.bet_iters)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    w1, info = work()
    st = ctx.stats()
    iters = args.bet_iters * args.steps
    solves, sweeps = (w1 - w0).tolist()
    node_updates = sweeps * n
    per_iter_updates = node_updates / iters
    eik_ms = st.last_bet_eikonal_ms
    # the chain groups' travel-time launches overlap on their streams, so the
    # rate is taken over the whole timed region: every launch's operations /
    # its wall time (which also holds the other, small kernels)
    achieved = node_updates * FLOP_PER_NODE_UPDATE / el / 1e12
    mean = torch.empty(n, dtype=torch.float64, device="cuda")
    std = torch.empty_like(mean)
    ctx.bet_stats(b, mean, std)
    misfits = np.array([g["misfit"] for g in info])
    prop = sum(sum(g["proposed"]) for g in info)
    acc = sum(sum(g["accepted"]) for g in info)
    log(f"[bench] bet: {c['chains']} chains x {iters} iterations in {el:.3f} s; {solves} solves, "
        f"{sweeps / max(solves, 1):.2f} sweeps per solve; {per_iter_updates * FLOP_PER_NODE_UPDATE / 1e9:.3f} GFLOP "
        f"of travel times per iteration; first chain group's travel-time launch {eik_ms:.3f} ms of its "
        f"{st.last_bet_iteration_ms:.3f} ms iteration; acceptance {acc / max(prop, 1):.3f}; "
        f"median misfit per datum {np.median(misfits) / (len(p['srcs']) * len(p['recs'])):.2f}")
    cpu = None if args.no_cpu_baseline else bet_cpu_baseline(p, tt_obs.cpu().numpy())
    ctx.bet_destroy(b)
    ctx.close()
    out = _base_record(args, c["chains"] * iters / el, el * 1e3 / args.steps, {
        "workload": f"Bayesian Eikonal tomography: {c['chains']} reversible-jump chains, Voronoi models "
                    f"(k {c['k_min']}..{c['k_max']}) on {c['nz']}x{c['nx']} nodes at {c['h']:g} m, "
                    f"{len(p['srcs'])} surface sources x {len(p['recs'])} receivers, {args.bet_iters} "
                    f"iterations per step",
        "path": "rtm_bet_run (per chain group and stream: propose, raster, travel times, accept; "
                "pooled statistics at sampling iterations)"},
        unit="chain iterations/s")
    out["metric"] = "Stage-1 chain iterations/s (each: one model, 34 travel-time solves)"
    out["dtype"] = "f32 travel times, f64 misfit and statistics"
    out["solves_per_s"] = solves / el
    out["node_updates_per_s"] = node_updates / el
    out["roofline"] = {"bound": "alu", "achieved": achieved, "peak": 157.3, "unit": "TFLOP/s",
                       "frac": achieved / 157.3, "traffic": None, "kernel": "k_bet_eikonal",
                       "launch_us": eik_ms * 1e3,
                       "note": f"{FLOP_PER_NODE_UPDATE} FP32 operations per node update x node updates (sweeps "
                               "x nodes) of all travel-time launches in the timed region / its wall time: the "
                               "launches of the chain groups overlap on their streams (launch_us: the first "
                               "group's last launch, HIP events); FP32 vector peak 256 CUs x 2.4 GHz x 256; "
                               "the sweeps are bound by the latency of dependent steps"}
    out["acceptance"] = acc / max(prop, 1)
    out["velocity_std_mean"] = float(std.mean())
    if cpu is not None:
        out["cpu_baseline"] = cpu
    return out


if __name__ == "__main__":
    main()
