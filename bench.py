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
timed on a bounded sample of the same workload.
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


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in ("paper_2001_06444_amd/csrc/rtm_kernels.hip", "paper_2001_06444_amd/csrc/rtm_internal.h"):
        h.update((ROOT / p).read_bytes())
    return h.hexdigest()[:16]


def measured_traffic(per_launch_alg_bytes):
    """HBM bytes per dominant-kernel launch from the committed rocprofv3
    counter summary, or None if it is missing or was taken on other code."""
    f = ROOT / "profiles" / "traffic_backward_step.json"
    if not f.exists():
        return None
    try:
        rec = json.loads(f.read_text())
    except ValueError:
        return None
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


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
        "kind": "oracle",
        "sample": (f"1 of {len(sv.shots)} shots (source ix={sh.src[1]}), first {nt_sample} of "
                   f"{sv.nt} time steps, same {sv.nz}x{sv.nx} model, nb={sv.nb}, all receivers; "
                   f"FP64 forward + adjoint + imaging with stored source wavefield; "
                   f"{updates:.3e} updates in {el:.1f} s"),
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--shots", type=int, default=100)
    ap.add_argument("--nt", type=int, default=4000)
    ap.add_argument("--plain-shots", type=int, default=2)
    ap.add_argument("--cpu-nt", type=int, default=2000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one 1 GiB device-to-device tensor copy (reference dispatch "
                         "for the HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); every shot of the "
              "survey is independent, so N GPUs would each migrate a disjoint share of the shots.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2001_06444_amd import inputs, rtm

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        src_t = torch.ones(1 << 28, device=dev)
        dst_t = torch.empty_like(src_t)
        dst_t.copy_(src_t)
        torch.cuda.synchronize()
        del src_t, dst_t
        log("[bench] calibration copy: 1 GiB read + 1 GiB written")
    sv = inputs.faulted_survey(n_shots=args.shots, nt=args.nt)
    nz, nx, nt, nb, h, dt = sv.nz, sv.nx, sv.nt, sv.nb, sv.h, sv.dt
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device=dev)
    vel_true, vel_mig, wav = t(sv.vel_true), t(sv.vel_mig), t(sv.wavelet)
    grid = rtm.make_grid(nz, nx, nb, nt, h, h, dt)

    # arena: working set of every shot of the batch plus slack
    field = ((nz + 2 * nb + 63) // 64 * 64 + 10) * ((nx + 2 * nb + 4 + 63) // 64 * 64) * 4
    ring = nt * 8 * (nz + nx - 8) * 4
    per_shot = 5 * field + ring + nz * nx * 4 + nt * 256 + nx * 8 + 8192
    arena = int(len(sv.shots) * per_shot * 1.02) + (256 << 20)
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

    # dominant kernel: backward step (HIP events around all its launches, work stream)
    bwd_launch_ms = s1.last_bwd_ms / s1.last_bwd_launches
    fwd_launch_ms = s1.last_fwd_ms / s1.last_fwd_launches
    achieved = s1.last_bwd_launch_bytes / (bwd_launch_ms * 1e-3) / 1e9
    achieved_fwd = s1.last_fwd_launch_bytes / (fwd_launch_ms * 1e-3) / 1e9
    log(f"[bench] backward launch {bwd_launch_ms * 1e3:.1f} us, {achieved:.0f} GB/s; "
        f"forward launch {fwd_launch_ms * 1e3:.1f} us, {achieved_fwd:.0f} GB/s")

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

    ctx.close()
    out = {
        "metric": "RTM grid-pt updates/s + images/s (batched/served vs plain), p99 latency, %HBM roofline",
        "value": value,
        "unit": "grid-pt updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"faulted-layer survey {nz}x{nx} at 10 m, {len(shots)} shots, "
                               f"nt={nt}, nb={nb}, reconstruct mode, stacked",
                   "nz": nz, "nx": nx, "nb": nb, "nt": nt, "shots": len(shots),
                   "src_mode": "reconstruct", "path": "batched (hipGraph, all shots per launch)"},
        "images_per_s": images_per_s,
        "plain": plain,
        "batched_vs_plain": (images_per_s / plain["images_per_s"]) if plain else None,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(s1.last_bwd_launch_bytes),
                     "kernel": "k_step<TZ,backward> (receiver step + reconstruct + imaging)",
                     "alg_bytes_per_launch": s1.last_bwd_launch_bytes,
                     "launch_us": bwd_launch_ms * 1e3,
                     "forward_launch": {"achieved": achieved_fwd, "launch_us": fwd_launch_ms * 1e3,
                                        "alg_bytes_per_launch": s1.last_fwd_launch_bytes}},
        "cpu_baseline": base,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
