"""Random-ellipse phantoms and their exact line integrals.

Coordinates.  An N x N image covers the square [0, N] x [0, N]; pixel (x, y) (column x, row y)
is the unit cell whose centre is (x + 1/2, y + 1/2).  Phantoms are sums of uniform ellipses
placed inside the disc of radius ``disc * N`` about the centre (N/2, N/2).

Linogram line sets (the four line classes of the (s, t) parameterisation).  Class q, slope
index t in [0, N) and shift s in [0, N) name the line with slope m_t = t / (N - 1):

    q = 0  (mostly vertical, positive shift):   X = s + 1/2 + m_t (Y - 1/2)
    q = 1  (mostly vertical, negative shift):   X = N - s - 1/2 - m_t (Y - 1/2)
    q = 2  (mostly horizontal, positive shift): Y = s + 1/2 + m_t (X - 1/2)
    q = 3  (mostly horizontal, negative shift): Y = N - s - 1/2 - m_t (X - 1/2)

Shifts are cyclic modulo N: the value stored at shift s is the sum of the line integrals at
intercepts s and s - N (the two lines that fold onto index s).  For a phantom inside a disc of
radius below N / (2 sqrt 2) at most one of the two meets the object, so the fold loses nothing.

The values are physical line integrals (integrals with respect to arc length), as a scanner
measures them; the ellipse formula is the textbook closed form for the X-ray transform of a
uniform ellipse.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import torch

F64 = torch.float64


@dataclass
class EllipseSet:
    """A batch of 2-D ellipse phantoms.

    ``params`` has shape [..., E, 6] with columns (cx, cy, semi_a, semi_b, phi, rho): centre,
    semi-axes, rotation of the first axis from +X (radians) and additive density.
    """

    params: torch.Tensor

    @property
    def count(self) -> int:
        return int(self.params.shape[-2])

    def to(self, device=None, dtype=None) -> "EllipseSet":
        return EllipseSet(self.params.to(device=device, dtype=dtype))


def _gen(seed: int) -> torch.Generator:
    g = torch.Generator()
    g.manual_seed(int(seed))
    return g


def random_ellipses(n: int, count: int, seed: int, *, disc: float = 0.34,
                    axes: tuple[float, float] = (0.05, 0.4),
                    density: tuple[float, float] = (-0.5, 1.0),
                    batch: int | None = None) -> EllipseSet:
    """Seeded random ellipses for an N x N slice.

    Full axis lengths are drawn uniformly in ``axes`` * N (semi-axes half of that), rotations
    uniformly in [0, pi), densities uniformly in ``density``; each centre is uniform in the disc
    of radius ``disc * N - semi_major`` about the image centre, so every ellipse lies inside the
    disc of radius ``disc * N``.
    """
    g = _gen(seed)
    shape = (count,) if batch is None else (batch, count)
    u = lambda: torch.rand(shape, generator=g, dtype=F64)  # noqa: E731
    semi_a = 0.5 * n * (axes[0] + (axes[1] - axes[0]) * u())
    semi_b = 0.5 * n * (axes[0] + (axes[1] - axes[0]) * u())
    phi = math.pi * u()
    rho = density[0] + (density[1] - density[0]) * u()
    room = (disc * n - torch.maximum(semi_a, semi_b)).clamp_min(0.0)
    rad = room * torch.sqrt(u())
    ang = 2.0 * math.pi * u()
    cx = 0.5 * n + rad * torch.cos(ang)
    cy = 0.5 * n + rad * torch.sin(ang)
    return EllipseSet(torch.stack([cx, cy, semi_a, semi_b, phi, rho], dim=-1))


def random_ellipsoids(n: int, depth: int, count: int, seed: int, *, disc: float = 0.34,
                      axes: tuple[float, float] = (0.05, 0.4),
                      density: tuple[float, float] = (-0.5, 1.0)) -> torch.Tensor:
    """Seeded random ellipsoids with one axis along z, for a volume of ``depth`` slices.

    Returns [count, 8]: (cx, cy, cz, semi_a, semi_b, semi_z, phi, rho).  The in-plane part
    follows :func:`random_ellipses`; centres cz are uniform in [0.15, 0.85] * depth and the
    z semi-axis uniform in [0.1, 0.5] * depth.
    """
    base = random_ellipses(n, count, seed, disc=disc, axes=axes, density=density).params
    g = _gen(seed + 7919)
    cz = depth * (0.15 + 0.7 * torch.rand(count, generator=g, dtype=F64))
    sz = depth * (0.1 + 0.4 * torch.rand(count, generator=g, dtype=F64))
    cx, cy, sa, sb, phi, rho = base.unbind(-1)
    return torch.stack([cx, cy, cz, sa, sb, sz, phi, rho], dim=-1)


def ellipsoid_slices(ells3d: torch.Tensor, depth: int) -> EllipseSet:
    """Cross-sections z = k + 1/2 (k = 0..depth-1) of an ellipsoid stack as 2-D ellipse sets.

    An ellipsoid cut at height z has its in-plane semi-axes scaled by sqrt(1 - ((z - cz)/sz)^2);
    slices that miss it get density 0 (and a tiny positive size, which keeps formulas finite).
    """
    z = torch.arange(depth, dtype=F64)[:, None] + 0.5
    cx, cy, cz, sa, sb, sz, phi, rho = (c[None, :] for c in ells3d.unbind(-1))
    u = 1.0 - ((z - cz) / sz) ** 2
    inside = u > 0
    scale = torch.sqrt(u.clamp_min(1e-12))
    params = torch.stack([
        cx.expand_as(u), cy.expand_as(u),
        torch.where(inside, sa * scale, torch.full_like(u, 1e-3)),
        torch.where(inside, sb * scale, torch.full_like(u, 1e-3)),
        phi.expand_as(u), torch.where(inside, rho.expand_as(u), torch.zeros_like(u)),
    ], dim=-1)
    return EllipseSet(params)


def phantom_image(ells: EllipseSet, n: int, *, supersample: int = 1, device=None,
                  dtype=F64) -> torch.Tensor:
    """Rasterise the phantom: mean over ``supersample``^2 sub-pixel samples per pixel."""
    p = ells.params.to(device=device, dtype=dtype)
    ss = int(supersample)
    off = (torch.arange(ss, device=device, dtype=dtype) + 0.5) / ss
    ax = (torch.arange(n, device=device, dtype=dtype)[:, None] + off[None, :]).reshape(-1)
    Y = ax[:, None]
    X = ax[None, :]
    img = torch.zeros(p.shape[:-2] + (n * ss, n * ss), device=device, dtype=dtype)
    for e in range(p.shape[-2]):
        cx, cy, a, b, phi, rho = (c[..., None, None] for c in p[..., e, :].unbind(-1))
        dx = X - cx
        dy = Y - cy
        u = dx * torch.cos(phi) + dy * torch.sin(phi)
        v = -dx * torch.sin(phi) + dy * torch.cos(phi)
        img = img + rho * (((u / a) ** 2 + (v / b) ** 2) <= 1.0).to(dtype)
    if ss > 1:
        img = img.reshape(img.shape[:-2] + (n, ss, n, ss)).mean(dim=(-3, -1))
    return img


def _ellipse_line_integrals(p: torch.Tensor, nx: torch.Tensor, ny: torch.Tensor,
                            r: torch.Tensor) -> torch.Tensor:
    """Sum over ellipses of the line integral along {P : P . (nx, ny) = r} (unit normal).

    ``p`` is [..., E, 6]; ``nx, ny, r`` broadcast to the line grid [..., *L].  The batch
    dimensions of ``p`` lead; one extra singleton per line-grid dimension is inserted.
    """
    nl = r.dim()
    out = None
    for e in range(p.shape[-2]):
        col = p[..., e, :]
        cx, cy, a, b, phi, rho = (c.reshape(c.shape + (1,) * nl) for c in col.unbind(-1))
        rr = r - (cx * nx + cy * ny)
        cphi = torch.cos(phi)
        sphi = torch.sin(phi)
        ct = nx * cphi + ny * sphi       # cos(theta - phi)
        st = ny * cphi - nx * sphi       # sin(theta - phi)
        s2 = (a * ct) ** 2 + (b * st) ** 2
        val = 2.0 * rho * a * b * torch.sqrt((s2 - rr * rr).clamp_min(0.0)) / s2
        out = val if out is None else out + val
    return out


def linogram_line_params(n: int, *, device=None, dtype=F64):
    """Unit normals and offsets of all 4 x N x N linogram lines and their s - N folds.

    Returns (nx, ny, r) each of shape [2, 4, N, N]: index 0 of the leading axis is the line at
    intercept s, index 1 the line at intercept s - N.
    """
    t = torch.arange(n, device=device, dtype=dtype)
    m = t / (n - 1) if n > 1 else torch.zeros_like(t)
    k = torch.sqrt(1.0 + m * m)
    s0 = torch.arange(n, device=device, dtype=dtype)
    s = torch.stack([s0, s0 - n])[:, None, None, :]            # [2,1,1,N]
    m_ = m[None, None, :, None]
    k_ = k[None, None, :, None]
    one = torch.ones_like(m_)
    # per class: nx, ny (before /k) and r*k as a function of s
    nx = torch.cat([one, one, -m_, m_], dim=1) / k_               # [1,4,N,1]
    ny = torch.cat([-m_, m_, one, one], dim=1) / k_
    rk = torch.cat([
        s + 0.5 - m_ / 2,
        n - s - 0.5 + m_ / 2,
        s + 0.5 - m_ / 2,
        n - s - 0.5 + m_ / 2,
    ], dim=1)                                                     # [2,4,N,N]
    r = rk / k_
    shape = (2, 4, n, n)
    return nx.expand(shape), ny.expand(shape), r.expand(shape)


def linogram(ells: EllipseSet, n: int, *, device=None, dtype=F64,
             out: torch.Tensor | None = None, chunk: int = 8) -> torch.Tensor:
    """Exact line integrals of the phantom on the four cyclic linogram line sets.

    Returns [..., 4, N, N] (batch dims of ``ells`` lead), index [q, t, s] as in the module
    docstring.  ``chunk`` bounds how many slices are evaluated at once.
    """
    p = ells.params.to(device=device, dtype=dtype)
    batch = p.shape[:-2]
    nx, ny, r = linogram_line_params(n, device=device, dtype=dtype)
    if out is None:
        out = torch.empty(batch + (4, n, n), device=device, dtype=dtype)
    if len(batch) == 0:
        out.copy_(_ellipse_line_integrals(p, nx, ny, r).sum(0))
        return out
    pf = p.reshape(-1, p.shape[-2], 6)
    of = out.view(-1, 4, n, n)
    for i in range(0, pf.shape[0], chunk):
        sl = pf[i:i + chunk]
        of[i:i + chunk].copy_(_ellipse_line_integrals(sl, nx, ny, r).sum(1))
    return out


def parallel_sinogram(ells: EllipseSet, n: int, n_angles: int, *, n_det: int | None = None,
                      device=None, dtype=F64) -> torch.Tensor:
    """Exact line integrals on a uniform parallel-beam geometry.

    Angle i has unit normal (cos th_i, sin th_i), th_i = i * pi / n_angles; detector j sits at
    signed distance r_j = j - n_det/2 + 1/2 from the image centre (N/2, N/2).  Returns
    [..., n_angles, n_det].
    """
    nd = n if n_det is None else int(n_det)
    p = ells.params.to(device=device, dtype=dtype)
    th = torch.arange(n_angles, device=device, dtype=dtype) * (math.pi / n_angles)
    rj = torch.arange(nd, device=device, dtype=dtype) - nd / 2 + 0.5
    nx = torch.cos(th)[:, None].expand(n_angles, nd)
    ny = torch.sin(th)[:, None].expand(n_angles, nd)
    r = rj[None, :] + 0.5 * n * (nx + ny)
    return _ellipse_line_integrals(p, nx, ny, r)


def poisson_noisy(p: torch.Tensor, i0: float, seed: int, *, max_attenuation: float = 2.0,
                  on_device: bool = False):
    """Poisson-noised line integrals at ``i0`` incident photons per ray.

    Line integrals are scaled by mu = max_attenuation / max|p| into attenuations, photon
    counts drawn as Poisson(i0 * exp(-mu p)) (seeded, on the CPU; with ``on_device`` and a
    GPU tensor, on the GPU from a generator of that device seeded the same way, a different
    but equally reproducible draw), floored at 1 count, and converted back by
    -log(counts / i0) / mu.
    """
    if on_device and p.is_cuda:
        g = torch.Generator(device=p.device)
        g.manual_seed(int(seed))
        pc = p.detach().to(torch.float64)
    else:
        g = _gen(seed)
        pc = p.detach().to("cpu", torch.float64)
    mu = max_attenuation / float(pc.abs().max().clamp_min(1e-30))
    lam = i0 * torch.exp(-mu * pc)
    counts = torch.poisson(lam, generator=g).clamp_min(1.0)
    noisy = -torch.log(counts / i0) / mu
    return noisy.to(device=p.device, dtype=p.dtype)


def random_int_array(shape, low: int, high: int, seed: int, *, dtype=F64) -> torch.Tensor:
    """Seeded integers uniform in [low, high] (inclusive), returned in ``dtype``."""
    g = _gen(seed)
    return torch.randint(int(low), int(high) + 1, tuple(shape), generator=g).to(dtype)


def support_mask(n: int, *, disc: float = 0.34, device=None) -> torch.Tensor:
    """Boolean [N, N] mask of pixels whose centres lie in the disc of radius disc * N."""
    c = torch.arange(n, device=device, dtype=F64) + 0.5 - 0.5 * n
    return (c[:, None] ** 2 + c[None, :] ** 2) <= (disc * n) ** 2


def volume_linogram(n: int, depth: int, *, count: int = 30, seed: int = 3, device=None,
                    dtype=torch.float32, chunk: int = 8):
    """Linograms of every z-slice of a seeded ellipsoid volume: [depth, 4, N, N].

    ``count`` ellipsoids (one axis along z, see :func:`random_ellipsoids`) are cut at the slice
    centres and each cross-section's exact line integrals are evaluated on ``device``.
    Returns (linogram, slice ellipse sets).
    """
    e3 = random_ellipsoids(n, depth, count, seed)
    sl = ellipsoid_slices(e3, depth)
    lino = linogram(sl, n, device=device, dtype=dtype, chunk=chunk)
    return lino, sl
