"""Learned parts of the reconstruction: recursive-filter coefficients per angle group and a
small residual convolutional network after the back projection.

Both are trained on the GPU with the library's own kernels: the reconstruction
(``fbp_reconstruct``), its adjoint (``fht_forward``), the coefficient gradient
(``fbp_filter_coef_grad``), and the convolutions and their gradients (``fbp_cnn_*``).  The
optimiser, the stable parameterisation of the feedback coefficients and the loss are small
host/torch steps on a few thousand numbers.  With no trained model the plain FHT-FBP (fitted
coefficients, no network) is the fallback.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import api

HIDDEN = 16


# ---- residual network ------------------------------------------------------------------------

def init_cnn(seed: int = 0, scale: float = 1e-2, device="cuda") -> dict:
    """Weights of out = img + conv3(relu(conv2(relu(conv1(img))))).  The last layer starts
    near zero so the untrained network is close to the identity."""
    g = torch.Generator().manual_seed(seed)
    w = {
        "w1": torch.randn(HIDDEN, 1, 3, 3, generator=g) * (1.0 / 3.0),
        "b1": torch.zeros(HIDDEN),
        "w2": torch.randn(HIDDEN, HIDDEN, 3, 3, generator=g) * (1.0 / 12.0),
        "b2": torch.zeros(HIDDEN),
        "w3": torch.randn(1, HIDDEN, 3, 3, generator=g) * scale,
        "b3": torch.zeros(1),
    }
    return {k: v.to(device=device, dtype=torch.float32).contiguous() for k, v in w.items()}


class ResidualCNN(torch.autograd.Function):
    """Forward and backward of the residual network, all in the library's kernels."""

    @staticmethod
    def forward(ctx, x0, w1, b1, w2, b2, w3, b3):
        x0 = x0.contiguous()
        p1, p2, p3 = api.fbp_cnn_pack(w1), api.fbp_cnn_pack(w2), api.fbp_cnn_pack(w3)
        h1 = api.fbp_cnn_conv(1, HIDDEN, x0, p1, bias=b1, relu=True)
        h2 = api.fbp_cnn_conv(HIDDEN, HIDDEN, h1, p2, bias=b2, relu=True)
        out = api.fbp_cnn_conv(HIDDEN, 1, h2, p3, bias=b3, resid=x0)
        ctx.save_for_backward(x0, h1, h2, w1, w2, w3)
        return out

    @staticmethod
    def backward(ctx, dout):
        x0, h1, h2, w1, w2, w3 = ctx.saved_tensors
        dout = dout.contiguous().float()
        g3 = api.fbp_cnn_wgrad(HIDDEN, 1, dout, h2)
        dz2 = api.fbp_cnn_conv(1, HIDDEN, dout, api.fbp_cnn_pack(w3, True), mask=h2)
        g2 = api.fbp_cnn_wgrad(HIDDEN, HIDDEN, dz2, h1)
        dz1 = api.fbp_cnn_conv(HIDDEN, HIDDEN, dz2, api.fbp_cnn_pack(w2, True), mask=h1)
        g1 = api.fbp_cnn_wgrad(1, HIDDEN, dz1, x0)
        dx0 = api.fbp_cnn_conv(HIDDEN, 1, dz1, api.fbp_cnn_pack(w1, True), resid=dout)
        n1, n2, n3 = HIDDEN * 9, HIDDEN * HIDDEN * 9, HIDDEN * 9
        return (dx0, g1[:n1].view(HIDDEN, 1, 3, 3), g1[n1:], g2[:n2].view(HIDDEN, HIDDEN, 3, 3),
                g2[n2:], g3[:n3].view(1, HIDDEN, 3, 3), g3[n3:])


def pack_cnn(w: dict) -> dict:
    """The network's weights packed once for inference (``residual_cnn_packed``)."""
    return {"p1": api.fbp_cnn_pack(w["w1"].detach()), "p2": api.fbp_cnn_pack(w["w2"].detach()),
            "p3": api.fbp_cnn_pack(w["w3"].detach()), "b1": w["b1"].detach(),
            "b2": w["b2"].detach(), "b3": w["b3"].detach()}


def residual_cnn_packed(x0: torch.Tensor, pk: dict, out: torch.Tensor | None = None):
    """The network at inference in one fused launch, on weights packed by ``pack_cnn``; the
    same result as ``residual_cnn`` bit for bit."""
    return api.fbp_cnn_forward(x0.contiguous(), pk["p1"], pk["b1"], pk["p2"], pk["b2"],
                               pk["p3"], pk["b3"], out)


def residual_cnn(x0: torch.Tensor, w: dict) -> torch.Tensor:
    """The network on [B, H, W] images.  When no gradient is needed, one fused launch
    (``fbp_cnn_forward``: hidden activations stay on chip, same result bit for bit); otherwise
    the layer-by-layer form whose activations the backward pass reuses."""
    needs_grad = torch.is_grad_enabled() and (
        x0.requires_grad or any(v.requires_grad for v in w.values()))
    if not needs_grad:
        return api.fbp_cnn_forward(x0.contiguous(), api.fbp_cnn_pack(w["w1"]), w["b1"],
                                   api.fbp_cnn_pack(w["w2"]), w["b2"], api.fbp_cnn_pack(w["w3"]),
                                   w["b3"])
    return ResidualCNN.apply(x0, w["w1"], w["b1"], w["w2"], w["b2"], w["w3"], w["b3"])


# ---- learned recursive-filter coefficients -------------------------------------------------

def step_up(k: torch.Tensor) -> torch.Tensor:
    """Feedback polynomial 1 + a_1 z^-1 + ... from reflection coefficients (stable when |k|<1);
    k is [G, K]; returns a [G, K] (a_1..a_K)."""
    G, K = k.shape
    a = torch.ones(G, 1, dtype=k.dtype)
    for m in range(K):
        ext = torch.cat([a, torch.zeros(G, 1, dtype=k.dtype)], dim=1)
        rev = torch.cat([torch.zeros(G, 1, dtype=k.dtype), a.flip(1)], dim=1)
        a = ext + k[:, m:m + 1] * rev
    return a[:, 1:]


def step_down(a: np.ndarray) -> np.ndarray:
    """Reflection coefficients of a stable feedback polynomial (inverse of step_up)."""
    c = np.concatenate([[1.0], np.asarray(a, dtype=np.float64)])
    K = len(a)
    ks = np.zeros(K)
    for m in range(K, 0, -1):
        km = c[m]
        ks[m - 1] = km
        c = (c[:m] - km * c[m:0:-1]) / (1 - km * km)
    return ks


RMAX = 0.999


class FBPWithCoefficients(torch.autograd.Function):
    """img = fbp_reconstruct(lino) with the plan's coefficients set to (b, a); gradients with
    respect to b and a from ``fbp_filter_coef_grad`` (and to the linogram if asked)."""

    @staticmethod
    def forward(ctx, lino, b, a, plan):
        api.fbp_plan_set_coefficients(plan, b.detach().cpu().numpy(), a.detach().cpu().numpy())
        ctx.plan = plan
        ctx.save_for_backward(lino)
        return api.fbp_reconstruct(plan, lino.contiguous())

    @staticmethod
    def backward(ctx, gimg):
        (lino,) = ctx.saved_tensors
        plan = ctx.plan
        gf = api.fht_forward(plan, gimg.contiguous().float())
        gc = api.fbp_filter_coef_grad(plan, lino, gf).cpu()
        glino = None
        if ctx.needs_input_grad[0]:
            glino = api.fbp_filter(plan, gf)
        return glino, gc[:, 0, :], gc[:, 1, :], None


class LearnedFBP:
    """Per-angle-group order-K coefficients and the residual network.

    a goes through reflection coefficients (always stable).  b is free up to the constraint
    sum(b) = 0 for K > 1: the ramp response vanishes at zero frequency (eq 6), so the recursive
    pair keeps a zero DC gain, which the fit of the plain method also imposes.  Without it the
    DC gain of the learned filter drifts and scales the whole image by a constant offset."""

    def __init__(self, n: int, max_batch: int, order: int = 4, groups: int = 8,
                 cnn: bool = True, seed: int = 0, fit_length: int | None = None):
        b0, a0, _ = api.fbp_fit_ramp_iir(order, fit_length or min(n, 512), dc_zero=order > 1)
        self.n, self.order, self.groups = n, order, groups
        self.b = torch.tensor(np.tile(b0, (groups, 1)), dtype=torch.float64, requires_grad=True)
        th = np.arctanh(np.clip(step_down(a0) / RMAX, -0.999999, 0.999999))
        self.theta = torch.tensor(np.tile(th, (groups, 1)), dtype=torch.float64,
                                  requires_grad=True)
        self.plan = api.fbp_plan(n, max_batch, np.tile(b0, (groups, 1)), np.tile(a0, (groups, 1)))
        self.cnn = init_cnn(seed) if cnn else None
        if self.cnn:
            for v in self.cnn.values():
                v.requires_grad_(True)

    def coefficients(self):
        a = step_up(RMAX * torch.tanh(self.theta))
        b = self.b - self.b.mean(dim=1, keepdim=True) if self.order > 1 else self.b
        return b, a

    def __call__(self, lino: torch.Tensor) -> torch.Tensor:
        b, a = self.coefficients()
        img = FBPWithCoefficients.apply(lino, b, a, self.plan)
        if self.cnn is not None:
            img = residual_cnn(img, self.cnn)
        return img

    def parameters(self):
        ps = [self.b, self.theta]
        if self.cnn is not None:
            ps += list(self.cnn.values())
        return ps

    def state_dict(self):
        b, a = self.coefficients()
        d = {"n": self.n, "order": self.order, "groups": self.groups,
             "b": b.detach().clone(), "a": a.detach().clone(), "theta": self.theta.detach().clone()}
        if self.cnn is not None:
            d["cnn"] = {k: v.detach().cpu().clone() for k, v in self.cnn.items()}
        return d

    def save(self, path: str):
        torch.save(self.state_dict(), path)

    def load_state_dict(self, d: dict):
        with torch.no_grad():
            self.b.copy_(d["b"])
            self.theta.copy_(d["theta"])
            if self.cnn is not None and "cnn" in d:
                for k, v in d["cnn"].items():
                    self.cnn[k].copy_(v.to(self.cnn[k].device))

    def close(self):
        self.plan.close()


def train(model: LearnedFBP, lino: torch.Tensor, target: torch.Tensor, mask: torch.Tensor,
          steps: int = 200, batch: int = 8, lr_coef: float = 1e-3, lr_cnn: float = 1e-3,
          seed: int = 0, log=None):
    """Adam on the coefficients (b, theta) and the network weights, minimising the masked MSE
    to `target` (the direct FBP of the same data) over random mini-batches of slices."""
    g = torch.Generator().manual_seed(seed)
    groups = [{"params": [model.b, model.theta], "lr": lr_coef}]
    if model.cnn is not None:
        groups.append({"params": list(model.cnn.values()), "lr": lr_cnn})
    opt = torch.optim.Adam(groups)
    scale = float((target[:, mask] ** 2).mean())
    # Everything a step needs from the host is ready before the loop, so that the host waits on
    # the device only where the coefficients pass through it (their gradient and the plan's
    # recursion tables): the mini-batches (the same draws as one randperm per step), the mask
    # as a factor and the count of masked pixels, and the losses, read back at the end.
    picks = torch.stack([torch.randperm(lino.shape[0], generator=g)[:batch]
                         for _ in range(steps)]).to(lino.device)
    maskf = mask.to(device=lino.device, dtype=torch.float32)
    per_slice = int(mask.sum())
    hist = []
    for it in range(steps):
        idx = picks[it]
        out = model(lino[idx])
        d = (out - target[idx]) * maskf
        loss = (d * d).sum() / (idx.numel() * per_slice * scale)
        opt.zero_grad()
        loss.backward()
        opt.step()
        hist.append(loss.detach())
        if log and (it % 20 == 0 or it == steps - 1):
            log(f"step {it}: relative MSE {float(hist[-1]):.5f}")
    return torch.stack(hist).tolist() if hist else []


@torch.no_grad()
def relative_rmse(model_or_plan, lino: torch.Tensor, target: torch.Tensor, mask: torch.Tensor,
                  chunk: int = 16) -> float:
    num = den = 0.0
    for i in range(0, lino.shape[0], chunk):
        x = lino[i:i + chunk]
        if isinstance(model_or_plan, LearnedFBP):
            out = model_or_plan(x)
        else:
            out = api.fbp_reconstruct(model_or_plan, x)
        d = (out - target[i:i + chunk])[:, mask].double()
        num += float((d * d).sum())
        den += float((target[i:i + chunk][:, mask].double() ** 2).sum())
    return math.sqrt(num / den)


def load_model(path: str, n: int, max_batch: int) -> LearnedFBP:
    """A LearnedFBP restored from ``save`` output (tensors only, no code is unpickled)."""
    d = torch.load(path, map_location="cpu", weights_only=True)
    if int(d["n"]) != n:
        raise ValueError(f"model at {path} is for N={int(d['n'])}, not {n}")
    m = LearnedFBP(n, max_batch, order=int(d["order"]), groups=int(d["groups"]),
                   cnn="cnn" in d)
    m.load_state_dict(d)
    b, a = m.coefficients()
    api.fbp_plan_set_coefficients(m.plan, b.detach().numpy(), a.detach().numpy())
    return m


def reconstructor(n: int, max_batch: int, path: str | None = None, order: int = 4):
    """lino [B,4,N,N] -> img [B,N,N]: the learned model saved at ``path`` when there is one for
    this N, else the plain FHT-FBP with an order-``order`` pair fitted to the ramp (the
    fallback).  Returns (callable, "learned" | "plain")."""
    import os
    if path and os.path.exists(path):
        try:
            m = load_model(path, n, max_batch)
        except (ValueError, KeyError, RuntimeError):
            m = None
        if m is not None:
            def run(lino):
                with torch.no_grad():
                    return m(lino)
            return run, "learned"
    b, a, _ = api.fbp_fit_ramp_iir(order, min(n, 512), dc_zero=order > 1)
    plan = api.fbp_plan(n, max_batch, b, a)
    return (lambda lino: api.fbp_reconstruct(plan, lino)), "plain"
