"""Pins of the oracle's residual network (the learned post-filter of the reconstruction).

The network is out = img + conv3(relu(conv2(relu(conv1(img))))) with 3x3 cross-correlations
and zero padding of one pixel.  The oracle evaluates it with conv2d; these tests hold it to an
explicit sum over taps and channels written out with loops, to exact special cases and to
invariants, so that a wrong padding, a flipped kernel, a misplaced activation or a lost skip
connection fails here.
"""
import itertools

import numpy as np
import pytest
import torch

from oracle import fbp_oracle as O


def _brute_layer(x, w, b):
    """x [C_in, H, W], w [C_out, C_in, 3, 3], b [C_out] -> [C_out, H, W], loops only."""
    cin, H, W = x.shape
    cout = w.shape[0]
    out = np.zeros((cout, H, W))
    for o, y, xx in itertools.product(range(cout), range(H), range(W)):
        acc = b[o]
        for c, dy, dx in itertools.product(range(cin), range(3), range(3)):
            yy, xs = y + dy - 1, xx + dx - 1
            if 0 <= yy < H and 0 <= xs < W:
                acc += w[o, c, dy, dx] * x[c, yy, xs]
        out[o, y, xx] = acc
    return out


def _brute_net(img, ws, bs):
    h = img[None]
    for layer, (w, b) in enumerate(zip(ws, bs)):
        h = _brute_layer(h, w, b)
        if layer < len(ws) - 1:
            h = np.maximum(h, 0.0)
    return img + h[0]


def _rand_net(seed, chans=(1, 3, 2, 1)):
    g = torch.Generator().manual_seed(seed)
    ws = [torch.randn(chans[i + 1], chans[i], 3, 3, generator=g, dtype=torch.float64) * 0.5
          for i in range(len(chans) - 1)]
    bs = [torch.randn(chans[i + 1], generator=g, dtype=torch.float64) * 0.1
          for i in range(len(chans) - 1)]
    return ws, bs


@pytest.mark.parametrize("seed,h,w", [(0, 5, 7), (1, 6, 6), (2, 1, 4)])
def test_matches_explicit_tap_sum(seed, h, w):
    ws, bs = _rand_net(seed)
    img = torch.randn(2, h, w, generator=torch.Generator().manual_seed(seed + 10),
                      dtype=torch.float64)
    got = O.residual_cnn(img, ws, bs)
    for i in range(2):
        ref = _brute_net(img[i].numpy(), [x.numpy() for x in ws], [x.numpy() for x in bs])
        np.testing.assert_allclose(got[i].numpy(), ref, rtol=1e-12, atol=1e-12)


def test_zero_last_layer_is_identity():
    ws, bs = _rand_net(3)
    ws[-1] = torch.zeros_like(ws[-1])
    bs[-1] = torch.zeros_like(bs[-1])
    img = torch.randn(1, 8, 8, dtype=torch.float64)
    assert torch.equal(O.residual_cnn(img, ws, bs), img)


def test_single_tap_chain_is_a_shift():
    """Layers that each copy the pixel to the right (tap dx = 2 reads x + 1) and a nonnegative
    image: the relus pass everything, three layers move the image three pixels left, with the
    zero padding entering from the right edge."""
    w = torch.zeros(1, 1, 3, 3, dtype=torch.float64)
    w[0, 0, 1, 2] = 1.0
    z = torch.zeros(1, dtype=torch.float64)
    img = torch.rand(1, 4, 9, generator=torch.Generator().manual_seed(4), dtype=torch.float64)
    got = O.residual_cnn(img, [w, w, w], [z, z, z])
    shifted = torch.zeros_like(img)
    shifted[:, :, :-3] = img[:, :, 3:]
    assert torch.allclose(got, img + shifted, rtol=0, atol=0)


def test_relu_between_layers_only():
    """Centre taps +1, +1, -1.  A negative image is zeroed by the first relu, so the output is
    the image itself (without that relu it would be img - img = 0).  A positive image passes
    both relus and the last layer cancels it (a relu after the last layer would leave the
    image).  A negative bias on the last layer reaches the output unclipped."""
    c = torch.zeros(1, 1, 3, 3, dtype=torch.float64)
    c[0, 0, 1, 1] = 1.0
    z = torch.zeros(1, dtype=torch.float64)
    img = -torch.rand(1, 5, 5, dtype=torch.float64) - 0.1
    assert torch.equal(O.residual_cnn(img, [c, c, -c], [z, z, z]), img)
    # a positive image passes both relus and the last layer subtracts it
    pos = -img
    assert torch.allclose(O.residual_cnn(pos, [c, c, -c], [z, z, z]),
                          torch.zeros_like(pos), atol=0)
    # the last layer has no relu: a negative last bias reaches the output
    b3 = torch.tensor([-0.25], dtype=torch.float64)
    out = O.residual_cnn(pos, [c, c, c * 0], [z, z, b3])
    assert torch.allclose(out, pos - 0.25, atol=1e-15)


def test_translation_equivariance_away_from_borders():
    ws, bs = _rand_net(5)
    img = torch.zeros(1, 20, 20, dtype=torch.float64)
    img[0, 6:10, 6:11] = torch.rand(4, 5, generator=torch.Generator().manual_seed(6),
                                    dtype=torch.float64)
    a = O.residual_cnn(img, ws, bs)
    b = O.residual_cnn(torch.roll(img, (3, 2), (1, 2)), ws, bs)
    # the receptive field is 7x7: compare where neither evaluation sees the border
    assert torch.allclose(torch.roll(a, (3, 2), (1, 2))[0, 6:14, 6:14], b[0, 6:14, 6:14],
                          atol=1e-13)


def test_bf16_rounding_is_round_to_nearest_even():
    one = 1.0
    ulp = 2.0 ** -7                    # bfloat16 has 8 significant bits: spacing 2^-7 at 1
    x = torch.tensor([one + ulp / 2, one + 1.5 * ulp, one + 0.49 * ulp, -(one + 0.51 * ulp),
                      2.0 ** -130], dtype=torch.float64)
    got = O._round_bf16(x)
    # ties go to the even significand; 2^-130 is a bfloat16 subnormal and stays exact
    exp = torch.tensor([one, one + 2 * ulp, one, -(one + ulp), 2.0 ** -130], dtype=torch.float64)
    assert torch.equal(got, exp)


def test_bf16_storage_matches_rounded_explicit_sum():
    ws, bs = _rand_net(7, chans=(1, 2, 2, 1))
    img = torch.randn(1, 5, 6, generator=torch.Generator().manual_seed(8), dtype=torch.float64)
    got = O.residual_cnn(img, ws, bs, bf16_storage=True)

    def rb(a):
        return torch.from_numpy(np.asarray(a)).to(torch.float32).to(torch.bfloat16).double().numpy()

    h = rb(img[0].numpy())[None]
    for layer, (w, b) in enumerate(zip(ws, bs)):
        h = _brute_layer(h, rb(w.numpy()), b.numpy())
        if layer < 2:
            h = rb(np.maximum(h, 0.0))
    ref = img[0].numpy() + h[0]
    np.testing.assert_allclose(got[0].numpy(), ref, rtol=1e-12, atol=1e-12)
