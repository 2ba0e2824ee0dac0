"""FP64 CPU oracle of FHT-FBP: recursive ramp filtering plus Fast-Hough-Transform back projection.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain PyTorch CPU ops in float64, every
step in the paper's order, no blocking or fusion.  Citations name the paper's sections and
equations ("Dolmatova, Chukalina, Nikolaev, Accelerated FBP for computed tomography image
reconstruction", ICIP 2020).

Where the paper is silent or ambiguous this file takes the following readings:

  R1 shift axis: linogram shifts are cyclic modulo N (four N x N images, Sec. 4.1); each
     detector row is filtered over the N-sample window that starts at sigma_t, which keeps
     the projection of an object inside the disc of radius 0.34 N away from the window ends.
  R2 slope scale: class slope m_t = t / (N - 1), t = 0..N-1, so the dyadic pattern of index t
     runs from offset 0 in the first image row to offset t in the last (Sec. 4.1, eq 14).
  R3 angular weights: the four classes tile [0, pi) (Sec. 4.1); inside a class the directions
     theta_t = atan(m_t) are weighted by the trapezoid rule, so the boundary directions, which
     two classes share, get half weight in each.
  R4 signs in eq 18-21: every class contributes with a positive weight; the h classes are
     reconstructed in the transposed image (eq 16), the v classes natively.
  R5 eq 13 feeds each recursion back with its own output (the p-tilde-plus / p-tilde-minus
     sequence), with zero state before the window (causal pass) and after it (anticausal pass).
  R6 eq 8 is the centred FIR with k = -L0..L0; the "exact" ramp filter uses L0 >= row length.
  R7 an order-K recursive filter has M = Q = K (Sec. 5 uses Q = M).
  R8 dyadic patterns: a pattern of height 2h and index t is two patterns of height h and index
     floor(t/2), the upper one displaced by ceil(t/2) (Sec. 4.4, the recursive dyadic FHT).
  R9 eq 15 with N - 1 in place of N (k_t = sqrt(1 + m_t^2)); the input rows are physical line
     integrals, the row scale is c_t = k_t * w_t (band-limited ramp at sample spacing 1/k_t).
  R16 eq 14 in these coordinates: the linogram line (q, t, s) of class q is, in pixel-centre
     coordinates, x = s + m_t y (q = 0), x = N-1-s - m_t y (q = 1), and the same with x and y
     swapped (q = 2, 3); the fold s - N is a second line of the same cell.  A parallel-beam
     sinogram has angle i at theta_i = i pi / P (unit normal (cos, sin)) and detector j at
     signed distance j - D/2 + 1/2 from the image centre.  A line is looked up by its normal
     angle in [0, pi) and signed distance, linearly in both (bilinear), zero outside the
     detector; angle P is angle 0 with the detector mirrored.  Values stay line integrals (no
     k_t factor: R9 puts it in the row scale).

Parity status: every function here is pinned by the CPU tests (closed forms, library routines,
brute force, adjoint identities, analytic phantoms); none is "parity unpinned".  The end-to-end
composition ``fbp_fht`` has no printed value to match (the paper prints none) and is pinned
through its pinned parts and against ``fbp_direct_linogram`` and the analytic phantom.
"""
from __future__ import annotations

import math

import torch

DT = torch.float64

__all__ = [
    "ramp_taps", "ramp_causal", "iir_causal", "iir_anticausal", "iir_pair",
    "iir_impulse_response",
    "slopes", "stretch", "angles", "angle_weights", "row_scale", "window_start",
    "row_groups", "filter_linogram", "filter_linogram_adjoint",
    "dyadic_shift", "fht", "fht_T", "to_frame", "from_frame", "fht_forward",
    "fht_backproject", "fbp_fht",
    "fir_ramp_full", "fbp_direct_linogram", "fbp_direct_parallel",
    "fht_add_count", "relative_rmse", "linogram_lines", "resample_sinogram",
    "residual_cnn",
]


# ---------------------------------------------------------------------------------------------
# Sec. 3: ramp filter and its causal/anticausal recursive approximation
# ---------------------------------------------------------------------------------------------

def ramp_taps(n) -> torch.Tensor:
    """Band-limited discrete ramp impulse response h(n), eq 7 (sample spacing 1, |w| < 1/2):
    1/4 at n = 0, 0 at other even n, -1/(n pi)^2 at odd n."""
    n = torch.as_tensor(n, dtype=torch.int64)
    h = torch.zeros(n.shape, dtype=DT)
    h = torch.where(n == 0, torch.full_like(h, 0.25), h)
    odd = (n % 2) != 0
    nf = n.to(DT)
    h = torch.where(odd, -1.0 / (math.pi * nf) ** 2, h)
    return h


def ramp_causal(length: int) -> torch.Tensor:
    """Causal half h+(n), n = 0..length-1, eq 10: h(0)/2 at n = 0 and h(n) for n > 0."""
    h = ramp_taps(torch.arange(length))
    h[0] = h[0] / 2
    return h


def iir_causal(x: torch.Tensor, b: torch.Tensor, a: torch.Tensor) -> torch.Tensor:
    """Difference equation eq 9 along the last axis, zero state before the first sample.

    y(n) = sum_{k<M} b_k x(n-k) - sum_{k=1..Q} a_k y(n-k).  ``b`` is [..., M] (b_0..b_{M-1}),
    ``a`` is [..., Q] (a_1..a_Q); their leading dims broadcast against x[..., 0].
    """
    M = b.shape[-1]
    Q = a.shape[-1]
    L = x.shape[-1]
    ys = []
    for i in range(L):
        acc = torch.zeros_like(x[..., 0] * b[..., 0])
        for k in range(M):
            if i - k >= 0:
                acc = acc + b[..., k] * x[..., i - k]
        for k in range(1, Q + 1):
            if i - k >= 0:
                acc = acc - a[..., k - 1] * ys[i - k]
        ys.append(acc)
    return torch.stack(ys, dim=-1)


def iir_anticausal(x: torch.Tensor, b: torch.Tensor, a: torch.Tensor) -> torch.Tensor:
    """Anticausal member of eq 13 (lower sign): y(n) = sum b_k x(n+k) - sum a_k y(n+k),
    zero state after the last sample; the same recursion run from the end of the row."""
    return iir_causal(x.flip(-1), b, a).flip(-1)


def iir_pair(x: torch.Tensor, b: torch.Tensor, a: torch.Tensor) -> torch.Tensor:
    """Eq 12: sum of the causal and the anticausal recursions (shared coefficients, Sec. 3)."""
    return iir_causal(x, b, a) + iir_anticausal(x, b, a)


def iir_impulse_response(b: torch.Tensor, a: torch.Tensor, length: int) -> torch.Tensor:
    """Impulse response g(0..length-1) of eq 9."""
    d = torch.zeros(length, dtype=DT)
    d[0] = 1.0
    return iir_causal(d, b.to(DT), a.to(DT))


# ---------------------------------------------------------------------------------------------
# Sec. 4.1-4.2: the (s, t) line classes, their angles and weights
# ---------------------------------------------------------------------------------------------

def slopes(N: int) -> torch.Tensor:
    """m_t = t / (N - 1), t = 0..N-1 (reading R2)."""
    return torch.arange(N, dtype=DT) / (N - 1)


def stretch(N: int) -> torch.Tensor:
    """k_t = sqrt(1 + m_t^2): linogram line length over the sinogram's (eq 15, reading R9)."""
    m = slopes(N)
    return torch.sqrt(1.0 + m * m)


def angles(N: int) -> torch.Tensor:
    """Deviation of line t from its class axis: atan(m_t) in [0, pi/4]."""
    return torch.atan(slopes(N))


def angle_weights(N: int) -> torch.Tensor:
    """Trapezoid weights w_t over the class angles (reading R3); each class sums to pi/4."""
    th = angles(N)
    w = torch.empty(N, dtype=DT)
    w[0] = (th[1] - th[0]) / 2
    w[-1] = (th[-1] - th[-2]) / 2
    w[1:-1] = (th[2:] - th[:-2]) / 2
    return w


def row_scale(N: int, *, input_is_fht: bool = False) -> torch.Tensor:
    """c_t = k_t w_t: ramp at detector spacing 1/k_t times the angular weight (reading R9).

    With ``input_is_fht`` the input rows are sums over image rows (the linogram normalisation of
    Sec. 4.2, which underestimates the line integral by k_t), so one more k_t is applied.
    """
    c = stretch(N) * angle_weights(N)
    if input_is_fht:
        c = c * stretch(N)
    return c


def window_start(N: int) -> torch.Tensor:
    """First shift sigma_t of the filtering window of row t, taken modulo N (reading R1).

    The window is centred on floor((N-1-t)/2), the intercept of the line of slope m_t through
    the image centre.
    """
    t = torch.arange(N)
    return ((N - 1 - t) // 2 - N // 2) % N


def row_groups(N: int, groups: int) -> torch.Tensor:
    """Coefficient group of every linogram row (q, t), as a [4, N] index: the 4N rows in
    (q, t) order are split into ``groups`` equal consecutive ranges (angle groups)."""
    r = torch.arange(4 * N)
    return (r * groups // (4 * N)).reshape(4, N)


def _coeffs_per_row(N: int, coef: torch.Tensor) -> torch.Tensor:
    """Broadcast [K] (one set) or [G, K] (one set per angle group) to [4, N, K]."""
    coef = coef.to(DT)
    if coef.dim() == 1:
        return coef.expand(4, N, coef.shape[0])
    return coef[row_groups(N, coef.shape[0])]


def _window_index(N: int, windowed: bool) -> torch.Tensor:
    sig = window_start(N) if windowed else torch.zeros(N, dtype=torch.int64)
    return (sig[:, None] + torch.arange(N)[None, :]) % N      # [t, i] -> shift s


def filter_linogram(P: torch.Tensor, b: torch.Tensor, a: torch.Tensor, *,
                    scale: bool = True, windowed: bool = True,
                    input_is_fht: bool = False) -> torch.Tensor:
    """Ramp-filter every linogram row with the recursive pair, eq 12-13, then scale by c_t.

    ``P`` is [..., 4, N, N] indexed [q, t, s].  Row (q, t) is read over its window
    s = sigma_t + i (mod N), i = 0..N-1, filtered by eq 12 and written back to the same shifts.
    ``b`` / ``a`` are [K] or [G, K] (per angle group, see ``row_groups``).
    """
    N = P.shape[-1]
    idx = _window_index(N, windowed).expand(P.shape)
    x = torch.gather(P.to(DT), -1, idx)
    y = iir_pair(x, _coeffs_per_row(N, b), _coeffs_per_row(N, a))
    if scale:
        y = y * row_scale(N, input_is_fht=input_is_fht)[:, None]
    return torch.zeros_like(y).scatter(-1, idx, y)


def filter_linogram_adjoint(G: torch.Tensor, b: torch.Tensor, a: torch.Tensor, *,
                            scale: bool = True, windowed: bool = True,
                            input_is_fht: bool = False) -> torch.Tensor:
    """Adjoint of ``filter_linogram`` in its input: the pair is symmetric under reversal of
    the row, so its transpose is itself (causal and anticausal parts exchange roles)."""
    return filter_linogram(G, b, a, scale=scale, windowed=windowed, input_is_fht=input_is_fht)


# ---------------------------------------------------------------------------------------------
# Sec. 4.4-4.5: dyadic patterns, the Fast Hough Transform and its transpose
# ---------------------------------------------------------------------------------------------

def _log2(N: int) -> int:
    n = int(N).bit_length() - 1
    if N < 1 or (1 << n) != N:
        raise ValueError(f"N must be a power of two, got {N}")
    return n


def dyadic_shift(N: int) -> torch.Tensor:
    """Offsets D[t, y] of the dyadic pattern of index t in image row y (reading R8)."""
    _log2(N)
    D = torch.zeros(1, 1, dtype=torch.int64)
    h = 1
    while h < N:
        t = torch.arange(2 * h)
        lower = D[t // 2]                                  # rows y < h
        upper = ((t + 1) // 2)[:, None] + D[t // 2]        # rows y >= h
        D = torch.cat([lower, upper], dim=1)
        h *= 2
    return D


def fht(img: torch.Tensor) -> torch.Tensor:
    """Fast Hough Transform of the mostly-vertical, positive-shift class (Sec. 4.4).

    Returns H[..., t, s] = sum_y img[..., y, (s + D[t, y]) mod N], computed bottom-up: strips of
    height h with h patterns each are merged in pairs, pattern t of the merged strip taking
    pattern floor(t/2) of both halves, the upper half displaced by ceil(t/2).
    """
    N = img.shape[-1]
    _log2(N)
    batch = img.shape[:-2]
    x = torch.arange(N)
    S = img.to(DT).reshape(batch + (N, 1, N))               # [strip, pattern, column]
    h = 1
    while h < N:
        t = torch.arange(2 * h)
        A = S[..., 0::2, :, :][..., t // 2, :]
        B = S[..., 1::2, :, :][..., t // 2, :]
        idx = ((x[None, :] + ((t + 1) // 2)[:, None]) % N).expand(B.shape)
        S = A + torch.gather(B, -1, idx)
        h *= 2
    return S.reshape(batch + (N, N))


def fht_T(P: torch.Tensor) -> torch.Tensor:
    """Transpose of ``fht``: R[..., y, x] = sum_t P[..., t, (x - D[t, y]) mod N].

    This is the back projection of Sec. 4.5 ("inverse FHT"), computed top-down: every merge of
    ``fht`` is undone by sending pattern pair (2t', 2t'+1) to pattern t' of the lower strip
    unshifted and to pattern t' of the upper strip shifted back by t' and t'+1.
    """
    N = P.shape[-1]
    _log2(N)
    batch = P.shape[:-2]
    x = torch.arange(N)
    S = P.to(DT).reshape(batch + (1, N, N))
    h = N
    while h > 1:
        hh = h // 2
        C0 = S[..., :, 0::2, :]
        C1 = S[..., :, 1::2, :]
        tp = torch.arange(hh)
        lower = C0 + C1
        i0 = ((x[None, :] - tp[:, None]) % N).expand(C0.shape)
        i1 = ((x[None, :] - tp[:, None] - 1) % N).expand(C1.shape)
        upper = torch.gather(C0, -1, i0) + torch.gather(C1, -1, i1)
        S = torch.stack([lower, upper], dim=-3)
        S = S.reshape(batch + (S.shape[-4] * 2, hh, N))
        h = hh
    return S.reshape(batch + (N, N))


def to_frame(f: torch.Tensor, q: int) -> torch.Tensor:
    """Image in the frame of class q, where its lines are positive-shift vertical (eq 16):
    q0 identity, q1 mirror in x, q2 transpose, q3 transpose then mirror in x."""
    if q == 0:
        return f
    if q == 1:
        return f.flip(-1)
    if q == 2:
        return f.transpose(-1, -2)
    if q == 3:
        return f.transpose(-1, -2).flip(-1)
    raise ValueError(q)


def from_frame(u: torch.Tensor, q: int) -> torch.Tensor:
    """Inverse of ``to_frame`` (eq 20-21: the h classes come back through a transpose)."""
    if q == 0:
        return u
    if q == 1:
        return u.flip(-1)
    if q == 2:
        return u.transpose(-1, -2)
    if q == 3:
        return u.flip(-1).transpose(-1, -2)
    raise ValueError(q)


def fht_forward(img: torch.Tensor) -> torch.Tensor:
    """Discrete forward projection on the four classes (eq 16-17): [..., N, N] -> [..., 4, N, N].
    Each row is a sum over image rows (the linogram normalisation, no k_t factor)."""
    return torch.stack([fht(to_frame(img.to(DT), q)) for q in range(4)], dim=-3)


def fht_backproject(P: torch.Tensor) -> torch.Tensor:
    """Back projection of the four classes and their sum, eq 21-22: [..., 4, N, N] -> [..., N, N]."""
    P = P.to(DT)
    return sum(from_frame(fht_T(P[..., q, :, :]), q) for q in range(4))


def fbp_fht(P: torch.Tensor, b: torch.Tensor, a: torch.Tensor, *, scale: bool = True,
            windowed: bool = True, input_is_fht: bool = False) -> torch.Tensor:
    """The paper's method: recursive ramp filtering (Sec. 3) then FHT back projection (Sec. 4)."""
    Pf = filter_linogram(P, b, a, scale=scale, windowed=windowed, input_is_fht=input_is_fht)
    return fht_backproject(Pf)


# ---------------------------------------------------------------------------------------------
# Sec. 2-3: direct FBP with the exact (full-length) ramp filter, the method's accuracy yardstick
# ---------------------------------------------------------------------------------------------

def fir_ramp_full(x: torch.Tensor) -> torch.Tensor:
    """Eq 8 with L0 >= row length: out[i] = sum_j x[j] h(i - j) over the whole row."""
    L = x.shape[-1]
    i = torch.arange(L)
    T = ramp_taps(i[:, None] - i[None, :])
    return x.to(DT) @ T.transpose(0, 1)


def _lerp_rows(rows: torch.Tensor, pos: torch.Tensor) -> torch.Tensor:
    """Linear interpolation of rows[..., r, :] at fractional positions pos[r, ...]; zero outside
    [0, L-1].  rows: [..., R, L]; pos: [R, P] -> [..., R, P]."""
    L = rows.shape[-1]
    i0 = torch.floor(pos)
    fr = pos - i0
    i0 = i0.to(torch.int64)
    i1 = i0 + 1
    v0 = torch.gather(rows, -1, i0.clamp(0, L - 1).expand(rows.shape[:-1] + pos.shape[-1:]))
    v1 = torch.gather(rows, -1, i1.clamp(0, L - 1).expand(rows.shape[:-1] + pos.shape[-1:]))
    v0 = torch.where((i0 >= 0) & (i0 < L), v0, torch.zeros_like(v0))
    v1 = torch.where((i1 >= 0) & (i1 < L), v1, torch.zeros_like(v1))
    return v0 * (1 - fr) + v1 * fr


def linogram_lines(N: int):
    """Unit normal (nx, ny) and signed distance rho from the image centre of every linogram
    line, [2, 4, N, N] each (fold, class q, slope index t, shift s); fold 1 is the line at
    s - N (reading R16, Sec. 4.1 and eq 14)."""
    m = slopes(N)[:, None]                                   # [N, 1]
    k = stretch(N)[:, None]
    s = torch.arange(N, dtype=DT)[None, :]                   # [1, N]
    c = (N - 1) / 2.0
    nx, ny, rho = [], [], []
    for fold in (0, 1):
        sf = s - N * fold
        pos = (sf - c * (1 - m)) / k                         # x_c - m y_c = s
        neg = (N - 1 - sf - c * (1 + m)) / k                 # x_c + m y_c = N - 1 - s
        one = torch.ones_like(m) / k
        nx.append(torch.stack([one, one, -m / k, m / k]).expand(4, N, N))
        ny.append(torch.stack([-m / k, m / k, one, one]).expand(4, N, N))
        rho.append(torch.stack([pos.expand(N, N), neg.expand(N, N), pos.expand(N, N),
                                neg.expand(N, N)]))
    return torch.stack(nx), torch.stack(ny), torch.stack(rho)


def resample_sinogram(sino: torch.Tensor, N: int) -> torch.Tensor:
    """Linogram [..., 4, N, N] from a parallel-beam sinogram [..., P, D] by bilinear
    interpolation in (angle, detector) at every linogram line, folds summed (Sec. 4.2, eq 14,
    reading R16)."""
    sino = sino.to(DT)
    Pn, D = sino.shape[-2], sino.shape[-1]
    nx, ny, rho = linogram_lines(N)
    phi = torch.atan2(ny, nx)
    flip = phi < 0
    phi = torch.where(flip, phi + math.pi, phi)
    rho = torch.where(flip, -rho, rho)
    a = phi * (Pn / math.pi)                                 # fractional angle index
    u = rho + D / 2.0 - 0.5                                  # fractional detector index
    a0 = torch.floor(a)
    wa = a - a0
    a0 = a0.to(torch.int64)
    flat = sino.reshape(sino.shape[:-2] + (Pn * D,))
    out = torch.zeros(sino.shape[:-2] + (4, N, N), dtype=DT)
    for da, w in ((0, 1 - wa), (1, wa)):
        i = a0 + da
        wrap = i >= Pn                                       # angle pi = angle 0, mirrored
        i = torch.where(wrap, i - Pn, i)
        uu = torch.where(wrap, (D - 1) - u, u)
        j0 = torch.floor(uu)
        wu = uu - j0
        j0 = j0.to(torch.int64)
        for dj, wj in ((0, 1 - wu), (1, wu)):
            j = j0 + dj
            ok = (j >= 0) & (j < D)
            idx = (i * D + j.clamp(0, D - 1)).reshape(-1)
            v = flat[..., idx].reshape(sino.shape[:-2] + (2, 4, N, N))
            out = out + (torch.where(ok, w * wj, torch.zeros_like(wj)) * v).sum(-4)
    return out


def fbp_direct_linogram(P: torch.Tensor, *, chunk_elems: int = 1 << 24) -> torch.Tensor:
    """Direct Theta(N^3) FBP on the same four-class linogram, with the exact ramp filter.

    Each row is unfolded over its window (reading R1), filtered by the full-length FIR (eq 8),
    scaled by c_t, and back-projected exactly: pixel (x, y) of the class frame takes the
    filtered row at the continuous intercept s* = x - m_t y by linear interpolation (eq 5).
    """
    P = P.to(DT)
    N = P.shape[-1]
    batch = P.shape[:-3]
    m = slopes(N)
    sig_u = (N - 1 - torch.arange(N)) // 2 - N // 2          # unwrapped window start
    idx = _window_index(N, True).expand(P.shape)
    rows = fir_ramp_full(torch.gather(P, -1, idx)) * row_scale(N)[:, None]
    yy = torch.arange(N, dtype=DT)[:, None]
    xx = torch.arange(N, dtype=DT)[None, :]
    out = torch.zeros(batch + (N, N), dtype=DT)
    tc = max(1, chunk_elems // (N * N))
    for q in range(4):
        acc = torch.zeros(batch + (N, N), dtype=DT)
        for t0 in range(0, N, tc):
            ts = torch.arange(t0, min(N, t0 + tc))
            pos = (xx[None] - m[ts][:, None, None] * yy[None]) - sig_u[ts][:, None, None].to(DT)
            vals = _lerp_rows(rows[..., q, ts, :], pos.reshape(len(ts), N * N))
            acc = acc + vals.sum(-2).reshape(batch + (N, N))
        out = out + from_frame(acc, q)
    return out


def fbp_direct_parallel(sino: torch.Tensor, N: int, *, chunk_elems: int = 1 << 24) -> torch.Tensor:
    """Direct Theta(P N^2) FBP of a uniform parallel-beam sinogram (eq 3-5 with eq 7-8).

    ``sino`` is [..., P, Nd] with angle i = i pi / P (unit normal (cos, sin)) and detector j at
    signed distance j - Nd/2 + 1/2 from the image centre.  Rows are filtered by the full FIR
    (eq 8), weighted pi / P and back-projected with linear interpolation on an N x N grid.
    """
    sino = sino.to(DT)
    Pn, Nd = sino.shape[-2], sino.shape[-1]
    batch = sino.shape[:-2]
    rows = fir_ramp_full(sino) * (math.pi / Pn)
    th = torch.arange(Pn, dtype=DT) * (math.pi / Pn)
    c = torch.arange(N, dtype=DT) + 0.5 - N / 2
    X = c[None, :].expand(N, N).reshape(-1)
    Y = c[:, None].expand(N, N).reshape(-1)
    out = torch.zeros(batch + (N * N,), dtype=DT)
    ac = max(1, chunk_elems // (N * N))
    for a0 in range(0, Pn, ac):
        ia = torch.arange(a0, min(Pn, a0 + ac))
        r = torch.cos(th[ia])[:, None] * X[None] + torch.sin(th[ia])[:, None] * Y[None]
        pos = r + Nd / 2 - 0.5
        out = out + _lerp_rows(rows[..., ia, :], pos).sum(-2)
    return out.reshape(batch + (N, N))


# ---------------------------------------------------------------------------------------------
# Accounting and error measures
# ---------------------------------------------------------------------------------------------

def fht_add_count(N: int) -> int:
    """Additions of one FHT (or its transpose) of one class: log2 N levels of N^2 sums."""
    return N * N * _log2(N)


def relative_rmse(a: torch.Tensor, b: torch.Tensor, mask: torch.Tensor | None = None) -> float:
    """||a - b||_2 / ||b||_2, over ``mask`` when given."""
    a = a.to(DT)
    b = b.to(DT)
    if mask is not None:
        a = a[..., mask]
        b = b[..., mask]
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


# ---------------------------------------------------------------------------------------------
# Learned residual correction applied after the reconstruction
# ---------------------------------------------------------------------------------------------

def _round_bf16(x: torch.Tensor) -> torch.Tensor:
    """Round to the nearest bfloat16 value (ties to even), returned in float64."""
    return x.to(torch.float32).to(torch.bfloat16).to(DT)


def residual_cnn(img: torch.Tensor, weights: list[torch.Tensor], biases: list[torch.Tensor], *,
                 bf16_storage: bool = False):
    """out = img + conv3(relu(conv2(relu(conv1(img))))), 3x3 convolutions, zero padding 1.

    ``img`` is [B, N, N]; weights[l] is [C_out, C_in, 3, 3].  Plain conv2d as the library step.
    With ``bf16_storage`` the convolution inputs, the weights and the hidden activations are
    rounded to bfloat16 (the storage format of the matrix-core network); arithmetic stays float64
    and the skip connection uses the unrounded image.
    """
    x = img.to(DT)[:, None]
    h = _round_bf16(x) if bf16_storage else x
    L = len(weights)
    for layer in range(L):
        w = weights[layer].to(DT)
        if bf16_storage:
            w = _round_bf16(w)
        h = torch.nn.functional.conv2d(h, w, biases[layer].to(DT), padding=1)
        if layer < L - 1:
            h = torch.relu(h)
            if bf16_storage:
                h = _round_bf16(h)
    return (x + h)[:, 0]
