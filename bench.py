#!/usr/bin/env python3
"""Benchmark of the accelerated FBP (recursive ramp filter + FHT back projection) on one GPU.

Workload: a volume of 512 slices of N = 1024 (30 random ellipsoids with one axis along z, cut
at the slice centres; exact line integrals on the four linogram line classes), reconstructed
with an order-2 recursive ramp pair (fitted on the host to the causal half of the ramp, with
zero response at zero frequency).  One step = one ``fbp_reconstruct`` over the whole batch
(filter fused into the first Hough pass, remaining passes, class sum), inputs resident in HBM.

Printed: one JSON line with slices/s, the dominant kernel's roofline (HIP events recorded by
the library around that kernel's launches, on its own stream), the whole-path bandwidth, the
direct Theta(N^3) GPU FBP comparator at 4N uniform angles on the same GPU, the RMSE of the
method against the direct FBP, and the CPU FP64 oracle timed on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
N_DEFAULT, B_DEFAULT = 1024, 512


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=N_DEFAULT)
    ap.add_argument("--batch", type=int, default=B_DEFAULT)
    ap.add_argument("--order", type=int, default=2)
    ap.add_argument("--no-direct", action="store_true", help="skip the direct-FBP comparator")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-slices", type=int, default=16)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy 5 times (for scaling the "
                         "FETCH_SIZE / WRITE_SIZE counters) and exit")
    return ap.parse_args()


def copy_calibration():
    import torch
    n = 1 << 28                                   # 2^28 floats = 1 GiB each way
    src = torch.ones(n, device="cuda", dtype=torch.float32)
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_each_way": n * 4, "launches": 5}))


def algorithmic_bytes(kind: str, n: int, levels: list[int]) -> float:
    """Compulsory HBM bytes per slice of one launch of each kernel kind (float32).

    first:  reads the 4 linogram classes (16 N^2 B), writes the 4 intermediate classes (16 N^2)
    middle: reads and writes the 4 classes (32 N^2)
    last_v: reads classes 0, 1 (8 N^2), writes the image (4 N^2)
    last_h: reads classes 2, 3 (8 N^2), reads and writes the image (8 N^2)
    """
    n2 = float(n) * n
    return {"first": 32 * n2, "middle": 32 * n2, "last_v": 12 * n2, "last_h": 16 * n2,
            "forward": 20 * n2, "filter": 32 * n2}[kind]


def cpu_baseline(lino_cpu, b, a):
    """The FP64 oracle (as it stands) on a bounded sample of slices, on the host's cores."""
    import torch
    import oracle as O
    cores = torch.get_num_threads()
    x = lino_cpu.to(torch.float64)
    t0 = time.perf_counter()
    ref = O.fbp_fht(x, torch.tensor(b), torch.tensor(a))
    dt = time.perf_counter() - t0
    return ref, {"value": x.shape[0] / dt, "unit": "slices/s", "cores": int(cores),
                 "kind": "oracle", "seconds": dt,
                 "sample": f"{x.shape[0]} slices of N={x.shape[-1]} from the same volume, "
                           f"FP64 oracle fbp_fht batched over torch's {cores} host threads"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); this build has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    import torch
    import fbp_inputs as I
    import paper_2007_06289_amd as F

    N, B = args.n, args.batch
    dev = "cuda"
    torch.cuda.init()
    F.load_library()
    # order-K pair fitted on the host (Sec. 3 objective, zero DC response)
    b, a, fit_err = F.fbp_fit_ramp_iir(args.order, N, dc_zero=args.order > 1)
    print(f"[bench] fit order {args.order}: rel err {fit_err:.4f}", file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    lino, slices = I.volume_linogram(N, B, count=30, seed=3, device=dev, chunk=32)
    torch.cuda.synchronize()
    print(f"[bench] generated {B} x 4 x {N}^2 linogram in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)

    plan = F.fbp_plan(N, B, b, a)
    img = torch.empty((B, N, N), device=dev, dtype=torch.float32)
    for _ in range(args.warmup):
        F.fbp_reconstruct(plan, lino, img)
    torch.cuda.synchronize()
    print("[bench] warmup done", file=sys.stderr, flush=True)

    plan.profile(True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        F.fbp_reconstruct(plan, lino, img)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = plan.profile_read()
    plan.profile(False)
    ms_step = wall * 1e3 / args.steps
    slices_per_s = B * args.steps / wall
    print(f"[bench] {args.steps} steps: {ms_step:.3f} ms/step, {slices_per_s:.0f} slices/s "
          f"(events {ev0.elapsed_time(ev1) / args.steps:.3f} ms/step)", file=sys.stderr,
          flush=True)

    levels = plan.passes()
    kernels = {}
    for kind, (tot, cnt) in prof.items():
        avg = tot / cnt
        byt = algorithmic_bytes(kind, N, levels) * B
        kernels[kind] = {"avg_ms": avg, "launches": cnt, "algorithmic_GB": byt / 1e9,
                         "GB_per_s": byt / (avg * 1e-3) / 1e9}
    dom = max(kernels, key=lambda k: kernels[k]["avg_ms"] * kernels[k]["launches"])
    dk = kernels[dom]
    roofline = {"bound": "hbm", "kernel": f"fht pass ({dom})", "achieved": round(dk["GB_per_s"], 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(dk["GB_per_s"] / HBM_PEAK_GBS, 4),
                "traffic": None}
    path_gbs = 20.0 * N * N * B / (ms_step * 1e-3) / 1e9

    out = {
        "metric": "slices/s at N=1024: FHT-FBP vs direct FBP, same GPU, at stated RMSE; HBM GB/s",
        "value": round(slices_per_s, 1),
        "unit": "slices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"volume of {B} slices, N={N}, 30 random ellipsoids, "
                               f"order-{args.order} recursive ramp pair, fbp_reconstruct",
                   "n": N, "batch": B, "order": args.order, "passes": levels},
        "roofline": roofline,
        "kernels": {k: {kk: round(vv, 4) if isinstance(vv, float) else vv
                        for kk, vv in v.items()} for k, v in kernels.items()},
        "path": {"algorithmic_bytes_per_slice": 20 * N * N,
                 "GB_per_s": round(path_gbs, 1), "frac_of_peak": round(path_gbs / HBM_PEAK_GBS, 4)},
    }

    # ---- the direct Theta(N^3) FBP on the same GPU, 4N uniform angles ---------------------------
    if not args.no_direct:
        nd = 8
        P = 4 * N
        sino = I.parallel_sinogram(I.EllipseSet(slices.params[:nd]), N, P, device=dev,
                                   dtype=torch.float32)
        work = torch.empty_like(sino)
        dimg = torch.empty((nd, N, N), device=dev, dtype=torch.float32)
        F.fbp_direct_parallel(sino, N, dimg, work)
        torch.cuda.synchronize()
        reps = 3
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        t_f = t_b = 0.0
        for _ in range(reps):
            e[0].record()
            F.fbp_direct_filter(sino, work)
            e[1].record()
            F.fbp_direct_backproject(work, N, dimg)
            e[2].record()
            torch.cuda.synchronize()
            t_f += e[0].elapsed_time(e[1]) / reps
            t_b += e[1].elapsed_time(e[2]) / reps
        direct_sps = nd / ((t_f + t_b) * 1e-3)
        mask = I.support_mask(N, device=dev)
        fht = img[:nd].double()
        dref = dimg.double()
        rmse = float(torch.linalg.vector_norm((fht - dref)[:, mask]) /
                     torch.linalg.vector_norm(dref[:, mask]))
        out["direct_fbp"] = {"slices_per_s": round(direct_sps, 2), "angles": P,
                             "filter_ms_per_slice": round(t_f / nd, 3),
                             "backproject_ms_per_slice": round(t_b / nd, 3),
                             "speedup_fht_fbp": round(slices_per_s / direct_sps, 1),
                             "speedup_vs_backprojection_only":
                                 round(slices_per_s / (nd / (t_b * 1e-3)), 1),
                             "rel_rmse_fht_vs_direct": round(rmse, 5)}
        del sino, work, dimg

    # ---- CPU oracle on a bounded sample (also gives the FP32-vs-FP64 RMSE) ---------------------
    if not args.no_cpu:
        idx = torch.linspace(0, B - 1, args.cpu_slices).round().long()
        lino_cpu = lino[idx.to(dev)].cpu()
        ref, cpu = cpu_baseline(lino_cpu, b, a)
        got = img[idx.to(dev)].cpu().double()
        rr = float(torch.linalg.vector_norm(got - ref) / torch.linalg.vector_norm(ref))
        out["cpu_baseline"] = cpu
        out["rel_rmse_fp32_vs_fp64_oracle"] = rr

    plan.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
