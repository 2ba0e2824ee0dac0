"""Accuracy sweeps on seeded phantoms: error against the filter order and against the image size.

    python -m paper_2007_06289_amd.sweeps [--slices 4]

Both follow the paper's accuracy experiments (Sec. 5: relative RMSE against the order of the
recursive filter at N = 512 with P = 512 projections, and against the image size for the
Radon and the Hough back projection), on seeded random-ellipse phantoms instead of the
paper's images, whose values are not available.  Every reconstruction starts from a parallel-
beam sinogram of exact line integrals (P = N angles, D = N + N/2 detectors):

- order sweep (N = 512): FHT-FBP with the recursive pair of order K = 1..8 fitted to the
  ramp (zero DC response), against the phantom, beside the direct FBP (exact ramp, Radon
  back projection) of the same sinogram;
- size sweep (N = 128 .. 2048): the direct FBP (exact ramp, Radon back projection) and
  FHT-FBP (order 4), both against the phantom;
- back-projection sweep (N = 128 .. 2048), the paper's comparison of the Radon and the Hough
  back projection under one filter: the linogram resampled from the sinogram is filtered by
  the exact ramp (the full-length FIR of eq 8, times c_t), then back-projected once along the
  exact lines (``fbp_direct_linogram``) and once along the dyadic patterns (the same filtered
  rows through ``fht_backproject``); both against the phantom, so the difference is the Hough
  back projection's own error.

Errors are relative RMSE over the disc of radius 0.34 N.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import sys

import torch

import fbp_inputs as I

from . import api


def _rel(a: torch.Tensor, b: torch.Tensor, mask: torch.Tensor) -> float:
    d = (a - b)[:, mask].double()
    return float(torch.linalg.vector_norm(d) / torch.linalg.vector_norm(b[:, mask].double()))


def _hough_backprojection(rows: torch.Tensor, n: int) -> torch.Tensor:
    """FHT back projection of filtered rows held in window order (row (q, t) from its window
    start on, as the direct FBP's filter writes them): each row is put back at its cyclic
    shifts, s = (sigma_t + i) mod N with sigma_t = (floor((N - 1 - t) / 2) - N / 2) mod N, then
    back-projected by ``fht_backproject`` (a permutation, then the library's transform)."""
    t = torch.arange(n, device=rows.device)
    sigma = ((n - 1 - t) // 2 - n // 2) % n
    src = (torch.arange(n, device=rows.device)[None, :] - sigma[:, None]) % n     # [t, s]
    lino = torch.gather(rows, -1, src.expand(rows.shape)).contiguous()
    with api.fbp_plan(n, rows.shape[0], [0.125, -0.125], [0.0, 0.0]) as plan:
        return api.fht_backproject(plan, lino)


def _case(n: int, slices: int, seed: int):
    ells = I.random_ellipses(n, 30, seed=seed, batch=slices)
    P, D = n, n + n // 2
    sino = I.parallel_sinogram(ells, n, P, n_det=D, device="cuda", dtype=torch.float32)
    phantom = I.phantom_image(ells, n, supersample=2 if n <= 1024 else 1,
                              device="cuda").to(torch.float32)
    return sino, phantom, P, D


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--slices", type=int, default=4)
    ap.add_argument("--seed", type=int, default=11)
    args = ap.parse_args(argv)
    log = lambda s: print(f"[sweeps] {s}", file=sys.stderr, flush=True)  # noqa: E731
    out = {"phantoms": f"{args.slices} seeded 30-ellipse slices per size, exact line integrals",
           "metric": "relative RMSE against the phantom over the 0.34 N disc"}

    n = 512
    sino, phantom, P, D = _case(n, args.slices, args.seed)
    mask = I.support_mask(n, device="cuda")
    direct = api.fbp_direct_parallel(sino, n)
    e_direct = _rel(direct, phantom, mask)
    orders = {}
    for k in range(1, 9):
        b, a, fit = api.fbp_fit_ramp_iir(k, n, dc_zero=k > 1)
        with api.fbp_plan(n, args.slices, b, a) as plan:
            img = api.fbp_reconstruct_sinogram(plan, sino)
            orders[k] = {"fit_rel_err": round(fit, 5), "rel_rmse": round(_rel(img, phantom, mask), 5)}
        log(f"order {k}: {orders[k]}")
    out["order_sweep"] = {"n": n, "angles": P, "detectors": D,
                          "direct_fbp_rel_rmse": round(e_direct, 5), "fht_fbp": orders}

    sizes = {}
    for n in (128, 256, 512, 1024, 2048):
        sino, phantom, P, D = _case(n, args.slices, args.seed + n)
        mask = I.support_mask(n, device="cuda")
        direct = api.fbp_direct_parallel(sino, n)
        b, a, _ = api.fbp_fit_ramp_iir(4, min(n, 512), dc_zero=True)
        with api.fbp_plan(n, args.slices, b, a) as plan:
            img = api.fbp_reconstruct_sinogram(plan, sino)
        sizes[n] = {"direct_fbp": round(_rel(direct, phantom, mask), 5),
                    "fht_fbp_order4": round(_rel(img, phantom, mask), 5)}
        log(f"N={n}: {sizes[n]}")
        del sino, phantom, direct, img
        torch.cuda.empty_cache()
    out["size_sweep"] = sizes

    bp = {}
    for n in (128, 256, 512, 1024, 2048):
        sino, phantom, P, D = _case(n, args.slices, args.seed + 3 * n)
        mask = I.support_mask(n, device="cuda")
        lino = api.fbp_resample_sinogram(sino, n)
        work = torch.empty((args.slices, 4 * n, n), device="cuda")
        radon = api.fbp_direct_linogram(lino, work=work)
        hough = _hough_backprojection(work.view(args.slices, 4, n, n), n)
        bp[n] = {"radon_backprojection": round(_rel(radon, phantom, mask), 5),
                 "hough_backprojection": round(_rel(hough, phantom, mask), 5)}
        log(f"N={n}: {bp[n]}")
        del sino, phantom, lino, work, radon, hough
        torch.cuda.empty_cache()
    out["backprojection_sweep"] = {"filter": "exact ramp (full-length FIR), row scale c_t",
                                   "by_n": bp}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
