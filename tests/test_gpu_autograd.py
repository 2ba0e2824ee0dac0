"""Differentiable reconstruction (64 slices, N = 512): gradients of the HIP backward against
FP64 autograd of the oracle and against central finite differences of the HIP forward."""
import numpy as np
import pytest
import torch

import fbp_inputs as I
import oracle as O

pytestmark = pytest.mark.gpu

B2 = np.array([0.12372452, -0.12372452], dtype=np.float32).astype(np.float64)
A2 = np.array([-0.17164439, -0.13239954], dtype=np.float32).astype(np.float64)


def _rel(a, b):
    a = a.detach().cpu().double()
    b = b.detach().cpu().double()
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


@pytest.fixture(scope="module")
def case(gpu_lib):
    api = gpu_lib
    import paper_2007_06289_amd as F
    N, B = 512, 64
    ells = I.random_ellipses(N, 10, seed=44, batch=B)
    lino = I.linogram(ells, N).to(torch.float32)
    phantom = I.phantom_image(ells, N).to(torch.float32)
    plan = api.fbp_plan(N, B, B2, A2)
    x = lino.cuda().requires_grad_(True)
    img = F.fbp_reconstruct_autograd(plan, x)
    loss = ((img.double() - phantom.cuda().double()) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    yield dict(api=api, F=F, plan=plan, lino=lino, phantom=phantom, grad=x.grad.detach().cpu(),
               loss=float(loss.detach()), N=N, B=B)
    plan.close()


def test_gradient_matches_oracle_fp64_autograd(case):
    lino, phantom, grad = case["lino"], case["phantom"], case["grad"]
    for s in (0, 37):
        p = lino[s].double().requires_grad_(True)
        rec = O.fbp_fht(p, torch.tensor(B2), torch.tensor(A2))
        loss = ((rec - phantom[s].double()) ** 2).sum()
        (g_ref,) = torch.autograd.grad(loss, p)
        assert _rel(grad[s], g_ref) < 1e-4


def test_gradient_matches_central_differences(case):
    """Central differences (step 1e-3) on 32 random linogram entries.  The differences are taken
    on the FP64 forward (the oracle), where a 1e-3 step is far above rounding; the FP32 forward
    would drown them (a perturbed row spreads over ~N^2 pixels)."""
    lino, phantom, grad = case["lino"], case["phantom"], case["grad"]
    g = torch.Generator().manual_seed(123)
    s = 5
    x0 = lino[s].double()
    target = phantom[s].double()
    b, a = torch.tensor(B2), torch.tensor(A2)
    h = 1e-3
    for _ in range(32):
        q, t, u = (int(torch.randint(0, n, (1,), generator=g)) for n in (4, case["N"], case["N"]))
        xp = x0.clone()
        xm = x0.clone()
        xp[q, t, u] += h
        xm[q, t, u] -= h
        lp = ((O.fbp_fht(xp, b, a) - target) ** 2).sum()
        lm = ((O.fbp_fht(xm, b, a) - target) ** 2).sum()
        fd = float(lp - lm) / (2 * h)
        an = float(grad[s, q, t, u])
        assert abs(fd - an) <= 1e-3 * abs(fd) + 1e-6, (q, t, u, fd, an)


def test_backward_is_adjoint_of_forward(case):
    F, plan = case["F"], case["plan"]
    N = case["N"]
    x = torch.randn(2, 4, N, N, device="cuda")
    y = torch.randn(2, N, N, device="cuda")
    xr = x.clone().requires_grad_(True)
    out = F.fbp_reconstruct_autograd(plan, xr)
    (g,) = torch.autograd.grad(out, xr, grad_outputs=y)
    lhs = (out.detach().double() * y.double()).sum()
    rhs = (x.double() * g.double()).sum()
    assert abs(float(lhs - rhs)) < 1e-4 * float(lhs.abs() + rhs.abs())
