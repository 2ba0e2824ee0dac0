"""Learned parts on the GPU: coefficient gradients, the direct FBP that serves as training target,
the BF16 matrix-core residual network (forward and backward), and a short training run that
must lower the error against the FP64 direct FBP below that of the plain method."""
import math

import numpy as np
import pytest
import torch

import fbp_inputs as I
import oracle as O

pytestmark = pytest.mark.gpu


def _rel(a, b):
    a = a.detach().cpu().double()
    b = b.detach().cpu().double()
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


@pytest.mark.parametrize("N,order,groups", [(64, 2, 1), (128, 4, 8), (256, 3, 4)])
def test_coefficient_gradient_matches_oracle(gpu_lib, N, order, groups):
    api = gpu_lib
    B = 2
    gen = torch.Generator().manual_seed(N + order)
    P = I.linogram(I.random_ellipses(N, 8, seed=N, batch=B), N).to(torch.float32)
    Gout = torch.randn(B, 4, N, N, generator=gen, dtype=torch.float64).to(torch.float32)
    rng = np.random.default_rng(order)
    b = np.tile(api.fbp_fit_ramp_iir(order, 128, dc_zero=order > 1)[0], (groups, 1))
    b = b + rng.normal(size=b.shape) * 1e-3
    a = np.tile(api.fbp_fit_ramp_iir(order, 128, dc_zero=order > 1)[1], (groups, 1))
    b = b.astype(np.float32).astype(np.float64)
    a = a.astype(np.float32).astype(np.float64)
    with api.fbp_plan(N, B, b, a) as plan:
        got = api.fbp_filter_coef_grad(plan, P.cuda(), Gout.cuda())
        torch.cuda.synchronize()
    tb = torch.tensor(b, requires_grad=True)
    ta = torch.tensor(a, requires_grad=True)
    y = O.filter_linogram(P.double(), tb, ta)
    gb, ga = torch.autograd.grad((y * Gout.double()).sum(), (tb, ta))
    assert _rel(got[:, 0, :], gb) < 1e-4
    assert _rel(got[:, 1, :], ga) < 1e-4


@pytest.mark.parametrize("N", [64, 128])
def test_direct_linogram_fbp_matches_oracle(gpu_lib, N):
    api = gpu_lib
    P = I.linogram(I.random_ellipses(N, 10, seed=N, batch=2), N).to(torch.float32)
    got = api.fbp_direct_linogram(P.cuda())
    torch.cuda.synchronize()
    ref = O.fbp_direct_linogram(P.double())
    assert _rel(got, ref) < 1e-4


@pytest.mark.parametrize("N", [64, 256])
def test_exact_ramp_rows_through_hough_backprojection_match_oracle(gpu_lib, N):
    """The back-projection sweep's Hough arm: the direct FBP's exact-ramp rows (window order)
    put back at their cyclic shifts and back-projected by the FHT equal the oracle's FHT-FBP
    with the exact ramp as its filter (b = h+ over the whole row, no feedback, eq 10-12)."""
    api = gpu_lib
    from paper_2007_06289_amd import sweeps
    P = I.linogram(I.random_ellipses(N, 10, seed=N + 1, batch=2), N).to(torch.float32)
    work = torch.empty((2, 4 * N, N), device="cuda")
    api.fbp_direct_linogram(P.cuda(), work=work)
    got = sweeps._hough_backprojection(work.view(2, 4, N, N), N)
    torch.cuda.synchronize()
    ref = O.fbp_fht(P.double(), O.ramp_causal(N), torch.zeros(1, dtype=torch.float64))
    assert _rel(got, ref) < 1e-5


def _cnn_weights(seed):
    import paper_2007_06289_amd.learned as L
    w = L.init_cnn(seed, scale=0.2)
    g = torch.Generator().manual_seed(seed + 1)
    w["b1"] = (torch.randn(16, generator=g) * 0.1).cuda()
    w["b2"] = (torch.randn(16, generator=g) * 0.1).cuda()
    w["b3"] = (torch.randn(1, generator=g) * 0.1).cuda()
    return w


def test_cnn_forward_matches_oracle(gpu_lib):
    import paper_2007_06289_amd.learned as L
    N, B = 64, 2
    x0 = I.phantom_image(I.random_ellipses(N, 8, seed=5, batch=B), N, supersample=2).to(torch.float32)
    w = _cnn_weights(3)
    got = L.residual_cnn(x0.cuda(), w)
    torch.cuda.synchronize()
    ref = O.residual_cnn(x0.double(), [w["w1"].cpu(), w["w2"].cpu(), w["w3"].cpu()],
                         [w["b1"].cpu(), w["b2"].cpu(), w["b3"].cpu()], bf16_storage=True)
    # residual part alone (the skip connection would hide errors); the oracle rounds to BF16
    # where the kernels store, so only FP32 accumulation (and a rare BF16 rounding it flips)
    # is left: measured 6e-8 to 8e-8
    assert _rel(got.cpu().double() - x0.double(), ref - x0.double()) < 1e-4


def test_cnn_fused_forward_equals_layer_by_layer(gpu_lib):
    """fbp_cnn_forward (one launch, hidden activations in LDS) against the three fbp_cnn_conv
    launches: the same matrix-core operations on the same operands, so equal bit for bit,
    across tile edges (128 x 96 is 8 x 4 tiles of 16 x 30, the last column of tiles partial)."""
    api = gpu_lib
    import paper_2007_06289_amd.learned as L
    B, H, W = 2, 128, 96
    x0 = (I.phantom_image(I.random_ellipses(128, 8, seed=7, batch=B), 128, supersample=2)
          [:, :, :W].contiguous().to(torch.float32).cuda())
    w = _cnn_weights(5)
    p1, p2, p3 = api.fbp_cnn_pack(w["w1"]), api.fbp_cnn_pack(w["w2"]), api.fbp_cnn_pack(w["w3"])
    fused = api.fbp_cnn_forward(x0, p1, w["b1"], p2, w["b2"], p3, w["b3"])
    h1 = api.fbp_cnn_conv(1, 16, x0, p1, bias=w["b1"], relu=True)
    h2 = api.fbp_cnn_conv(16, 16, h1, p2, bias=w["b2"], relu=True)
    layers = api.fbp_cnn_conv(16, 1, h2, p3, bias=w["b3"], resid=x0)
    torch.cuda.synchronize()
    assert torch.equal(fused, layers)
    with torch.no_grad():
        assert torch.equal(L.residual_cnn(x0, w), fused)
    # inference on weights packed once, into a given output
    out = torch.empty_like(x0)
    assert L.residual_cnn_packed(x0, L.pack_cnn(w), out) is out
    assert torch.equal(out, fused)


@pytest.mark.parametrize("H,W", [(37, 80), (50, 48), (1, 16)])
def test_cnn_layers_equal_fused_at_ragged_sizes(gpu_lib, H, W):
    """The per-layer convolutions where every per-layer kernel has partial tiles (32 x 32 tiles
    for 1 -> 16, 16 x 32 for 16 -> 16, 32 x 30 for 16 -> 1; widths are multiples of 16, as
    fbp_cnn_conv requires) against the fused network, itself checked against the oracle at
    ragged sizes: the same matrix-core operations on the same operands, so equal bit for bit."""
    api = gpu_lib
    B = 2
    g = torch.Generator().manual_seed(H * 1000 + W)
    x0 = torch.randn(B, H, W, generator=g, dtype=torch.float64).to(torch.float32).cuda()
    w = _cnn_weights(8)
    p1, p2, p3 = api.fbp_cnn_pack(w["w1"]), api.fbp_cnn_pack(w["w2"]), api.fbp_cnn_pack(w["w3"])
    fused = api.fbp_cnn_forward(x0, p1, w["b1"], p2, w["b2"], p3, w["b3"])
    h1 = api.fbp_cnn_conv(1, 16, x0, p1, bias=w["b1"], relu=True)
    h2 = api.fbp_cnn_conv(16, 16, h1, p2, bias=w["b2"], relu=True)
    layers = api.fbp_cnn_conv(16, 1, h2, p3, bias=w["b3"], resid=x0)
    torch.cuda.synchronize()
    assert torch.equal(fused, layers)


@pytest.mark.parametrize("H,W", [(100, 72), (17, 33), (1, 5)])
def test_cnn_fused_forward_ragged_sizes_match_oracle(gpu_lib, H, W):
    """Sizes that are not multiples of the 16 x 32 tile (partial tiles, a single row)."""
    api = gpu_lib
    B = 2
    g = torch.Generator().manual_seed(H * W)
    x0 = torch.randn(B, H, W, generator=g, dtype=torch.float64).to(torch.float32)
    w = _cnn_weights(6)
    got = api.fbp_cnn_forward(x0.cuda(), api.fbp_cnn_pack(w["w1"]), w["b1"],
                              api.fbp_cnn_pack(w["w2"]), w["b2"], api.fbp_cnn_pack(w["w3"]),
                              w["b3"])
    torch.cuda.synchronize()
    ref = O.residual_cnn(x0.double(), [w["w1"].cpu(), w["w2"].cpu(), w["w3"].cpu()],
                         [w["b1"].cpu(), w["b2"].cpu(), w["b3"].cpu()], bf16_storage=True)
    assert _rel(got.cpu().double() - x0.double(), ref - x0.double()) < 1e-4


def test_cnn_backward_matches_oracle(gpu_lib):
    import paper_2007_06289_amd.learned as L
    N, B = 64, 2
    x0 = I.phantom_image(I.random_ellipses(N, 8, seed=6, batch=B), N, supersample=2).to(torch.float32)
    R = torch.randn(B, N, N, generator=torch.Generator().manual_seed(9))
    w = _cnn_weights(4)
    params = [w[k].clone().requires_grad_(True) for k in ("w1", "b1", "w2", "b2", "w3", "b3")]
    xg = x0.cuda().requires_grad_(True)
    out = L.ResidualCNN.apply(xg, *params)
    grads = torch.autograd.grad((out * R.cuda()).sum(), [xg] + params)
    torch.cuda.synchronize()
    ps = [p.detach().cpu().double().requires_grad_(True) for p in params]
    xr = x0.double().requires_grad_(True)
    ref_out = O.residual_cnn(xr, [ps[0], ps[2], ps[4]], [ps[1], ps[3], ps[5]], bf16_storage=True)
    refs = torch.autograd.grad((ref_out * R.double()).sum(), [xr] + ps)
    # gradients flow through BF16 storage of the hidden gradients: percent-level agreement
    names = ["x0", "w1", "b1", "w2", "b2", "w3", "b3"]
    for n, g_, r_ in zip(names, grads, refs):
        assert _rel(g_, r_) < 3e-2, n


@pytest.mark.parametrize("H", [40, 37])
@pytest.mark.parametrize("cin,cout", [(16, 16), (16, 1), (1, 16)])
def test_cnn_weight_gradient_matches_fp64(gpu_lib, cin, cout, H):
    """fbp_cnn_wgrad alone: dz and the layer input hold BF16 values, so every product is exact
    in FP32 and only the FP32 sums differ from the FP64 weight gradient (torch's conv2d weight
    gradient on the CPU) and bias gradient.  Heights 40 and 37 leave a partial block of 8 and 5
    rows (for 16 -> 16 a whole and a partial stage of 8 rows), width 128 two column blocks;
    zero padding at every image edge."""
    api = gpu_lib
    B, W = 2, 128
    g = torch.Generator().manual_seed(cin * 17 + cout)

    def bf16(*shape):
        return torch.randn(*shape, generator=g).to(torch.bfloat16)

    dz = bf16(B, H, W, cout)
    x = bf16(B, H, W, cin)
    dz_dev = (dz.view(torch.int16) if cout == 16 else dz[..., 0].float()).contiguous().cuda()
    x_dev = (x.view(torch.int16) if cin == 16 else x[..., 0].float()).contiguous().cuda()
    got = api.fbp_cnn_wgrad(cin, cout, dz_dev, x_dev).cpu().double()
    xd = x.double().permute(0, 3, 1, 2)
    dzd = dz.double().permute(0, 3, 1, 2)
    gw = torch.nn.grad.conv2d_weight(xd, (cout, cin, 3, 3), dzd, padding=1)
    gb = dzd.sum(dim=(0, 2, 3))
    nw = cout * cin * 9
    # each sum adds B H W products of size ~1 in FP32: a few 2^-24 sqrt(B H W) of its scale
    scale = math.sqrt(B * H * W)
    assert float((got[:nw] - gw.reshape(-1)).abs().max()) < 1e-5 * scale
    assert float((got[nw:] - gb).abs().max()) < 1e-5 * scale


def _bf16(t):
    return t.to(torch.float32).to(torch.bfloat16).to(torch.float64)


def _cnn_backward_bf16_reference(x0, w, R):
    """FP64 forward and backward of the residual network with BF16 values exactly where the
    matrix-core network rounds them: the first layer's input, the weights and the stored hidden
    activations in the forward pass; the gradients entering each backward convolution
    (the output gradient as an operand, the stored hidden gradients) in the backward pass.  The
    weight gradients take the FP32 output gradient and image unrounded, as the library's do."""
    F = torch.nn.functional
    x = x0.double()[:, None]
    wb = {k: _bf16(w[k].cpu()) for k in ("w1", "w2", "w3")}
    b = {k: w[k].cpu().double() for k in ("b1", "b2", "b3")}
    h1 = _bf16(torch.relu(F.conv2d(_bf16(x), wb["w1"], b["b1"], padding=1)))
    h2 = _bf16(torch.relu(F.conv2d(h1, wb["w2"], b["b2"], padding=1)))
    dout = R.double()[:, None]
    g3 = torch.nn.grad.conv2d_weight(h2, (1, 16, 3, 3), dout, padding=1)
    dz2 = _bf16((h2 > 0) * F.conv_transpose2d(_bf16(dout), wb["w3"], padding=1))
    g2 = torch.nn.grad.conv2d_weight(h1, (16, 16, 3, 3), dz2, padding=1)
    dz1 = _bf16((h1 > 0) * F.conv_transpose2d(dz2, wb["w2"], padding=1))
    g1 = torch.nn.grad.conv2d_weight(x, (16, 1, 3, 3), dz1, padding=1)
    dx = F.conv_transpose2d(dz1, wb["w1"], padding=1) + dout
    sums = lambda t: t.sum(dim=(0, 2, 3))  # noqa: E731
    return [dx[:, 0], g1, sums(dz1), g2, sums(dz2), g3, sums(dout)]


@pytest.mark.parametrize("H", [64, 37])
def test_cnn_backward_matches_bf16_reference(gpu_lib, H):
    """The network's backward pass against an FP64 reference that rounds to BF16 at the same
    points as the kernels: what is left is FP32 accumulation and the rare BF16 rounding that it
    flips (measured 3e-8 to 1.6e-6 over three seeds), far below the percent-level gap to the
    unrounded FP64 gradient.  Height 37 leaves partial tiles and partial weight-gradient
    blocks."""
    import paper_2007_06289_amd.learned as L
    N, B = 64, 2
    x0 = (I.phantom_image(I.random_ellipses(N, 8, seed=6, batch=B), N, supersample=2)[:, :H]
          .contiguous().to(torch.float32))
    R = torch.randn(B, H, N, generator=torch.Generator().manual_seed(9))
    w = _cnn_weights(4)
    params = [w[k].clone().requires_grad_(True) for k in ("w1", "b1", "w2", "b2", "w3", "b3")]
    xg = x0.cuda().requires_grad_(True)
    out = L.ResidualCNN.apply(xg, *params)
    grads = torch.autograd.grad((out * R.cuda()).sum(), [xg] + params)
    torch.cuda.synchronize()
    refs = _cnn_backward_bf16_reference(x0, w, R)
    names = ["x0", "w1", "b1", "w2", "b2", "w3", "b3"]
    for n, g_, r_ in zip(names, grads, refs):
        assert _rel(g_.reshape(r_.shape), r_) < 1e-4, n


def test_learned_filter_lowers_error_against_direct_fbp(gpu_lib):
    """Order-4 coefficients per 8 angle groups plus the residual network, trained on noisy
    phantom linograms against the direct FBP of the same data; measured against the FP64 direct FBP
    on held-out slices."""
    import paper_2007_06289_amd.learned as L
    api = gpu_lib
    N, n_train, n_test = 128, 48, 4
    ells = I.random_ellipses(N, 30, seed=77, batch=n_train + n_test)
    clean = I.linogram(ells, N)
    noisy = I.poisson_noisy(clean, 1e4, seed=78).to(torch.float32).cuda()
    target = api.fbp_direct_linogram(noisy)
    mask = I.support_mask(N).cuda()
    model = L.LearnedFBP(N, 16, order=4, groups=8, cnn=True, seed=0)
    tr, te = slice(0, n_train), slice(n_train, n_train + n_test)
    b0, a0, _ = api.fbp_fit_ramp_iir(4, 128, dc_zero=True)
    plain = api.fbp_plan(N, n_test, b0, a0)
    before = L.relative_rmse(plain, noisy[te], target[te], mask)
    L.train(model, noisy[tr], target[tr], mask, steps=150, batch=8)
    after = L.relative_rmse(model, noisy[te], target[te], mask)
    # the yardstick: FP64 direct FBP (oracle) on the held-out slices
    ref = O.fbp_direct_linogram(noisy[te].cpu().double())
    with torch.no_grad():
        out_l = model(noisy[te]).cpu().double()
        out_p = api.fbp_reconstruct(plain, noisy[te]).cpu().double()
    m = mask.cpu()
    e_l = float(torch.linalg.vector_norm((out_l - ref)[:, m]) / torch.linalg.vector_norm(ref[:, m]))
    e_p = float(torch.linalg.vector_norm((out_p - ref)[:, m]) / torch.linalg.vector_norm(ref[:, m]))
    print(f"held-out relative RMSE vs direct FBP: plain {before:.4f} learned {after:.4f}; "
          f"FP64 direct FBP: plain {e_p:.4f} learned {e_l:.4f}")
    plain.close()
    model.close()
    assert e_l < 0.8 * e_p


def test_saved_model_round_trip_and_plain_fallback(gpu_lib, tmp_path):
    import paper_2007_06289_amd.learned as L
    api = gpu_lib
    N = 64
    lino = I.linogram(I.random_ellipses(N, 6, seed=12, batch=2), N, device="cuda",
                      dtype=torch.float32)
    model = L.LearnedFBP(N, 2, order=4, groups=8, cnn=True, seed=3)
    with torch.no_grad():
        model.theta.add_(0.05)                     # move away from the fitted start
        model.cnn["b3"].add_(0.01)
        want = model(lino)
    path = str(tmp_path / "model.pt")
    model.save(path)
    run, kind = L.reconstructor(N, 2, path)
    assert kind == "learned"
    assert torch.allclose(run(lino), want, rtol=0, atol=0)
    # no model, or a model for another size: the plain FHT-FBP with fitted coefficients
    run, kind = L.reconstructor(N, 2, str(tmp_path / "missing.pt"))
    b, a, _ = api.fbp_fit_ramp_iir(4, N, dc_zero=True)
    with api.fbp_plan(N, 2, b, a) as plain:
        ref = api.fbp_reconstruct(plain, lino)
        assert kind == "plain" and torch.equal(run(lino), ref)
        run, kind = L.reconstructor(N * 2, 2, path)
        assert kind == "plain"
    torch.cuda.synchronize()
    model.close()
