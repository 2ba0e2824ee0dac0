"""fbp_reconstruct_noalloc, the entry point for callers that cannot allocate device memory,
against fbp_reconstruct through the C ABI: the same kernels with the inter-pass scratch in the
library's fixed array, so the images must be bit-identical.  Two calls in a row on one plan
(the second smaller, so the array holds the first call's values when it starts), then other
sizes: a three-pass schedule (two buffers in the array), a two-pass size checked against the
FP64 oracle too, and the size rejected because one slice needs more than the array."""
import numpy as np
import pytest
import torch

import fbp_inputs as I
import oracle as O

pytestmark = pytest.mark.gpu

B2 = (np.array([0.12372452, -0.12372452]), np.array([-0.17164439, -0.13239954]))


def _lino(N, B, seed):
    ells = I.random_ellipses(N, 10, seed, batch=B)
    return I.linogram(ells, N, device="cuda", dtype=torch.float32)


def _pair(api, N, B, P):
    """fbp_reconstruct on a plan with scratch, fbp_reconstruct_noalloc on one without."""
    with api.fbp_plan(N, B, *B2) as ref_plan:
        ref = api.fbp_reconstruct(ref_plan, P)
        torch.cuda.synchronize()
    return ref


def test_noalloc_equals_reconstruct(gpu_lib):
    api = gpu_lib
    N, B = 1024, 20          # 16 MiB per slice: chunks of 16 and 4 in the 256 MiB array
    P = _lino(N, B, seed=21)
    ref = _pair(api, N, B, P)
    with api.fbp_plan(N, B, *B2, flags=api.FBP_NO_SCRATCH) as plan:
        got = torch.full_like(ref, float("nan"))
        api.fbp_reconstruct_noalloc(plan, P, got)
        torch.cuda.synchronize()
        assert torch.equal(got, ref)
        # second call, smaller: starts with the first call's values in the array
        small = P[5:8].contiguous()
        got2 = torch.full((3, N, N), float("nan"), device="cuda")
        api.fbp_reconstruct_noalloc(plan, small, got2)
        torch.cuda.synchronize()
        assert torch.equal(got2, ref[5:8])
        # the plan holds no scratch of its own: calls that need it are refused
        with pytest.raises(api.FbpError) as e:
            api.fbp_reconstruct(plan, P)
        assert e.value.code == api.FBP_EINVAL


def test_noalloc_three_passes_and_oracle(gpu_lib):
    api = gpu_lib
    N = 2048                 # [2, 4, 5]: two 64 MiB buffers per slice
    P = _lino(N, 1, seed=22)
    ref = _pair(api, N, 1, P)
    with api.fbp_plan(N, 1, *B2, flags=api.FBP_NO_SCRATCH) as plan:
        got = torch.full_like(ref, float("nan"))
        api.fbp_reconstruct_noalloc(plan, P, got)
        torch.cuda.synchronize()
    assert torch.equal(got, ref)
    N = 256
    P = _lino(N, 3, seed=23)
    ref = _pair(api, N, 3, P)
    with api.fbp_plan(N, 3, *B2) as plan:
        got = torch.full_like(ref, float("nan"))
        api.fbp_reconstruct_noalloc(plan, P, got)
        torch.cuda.synchronize()
    assert torch.equal(got, ref)
    oref = O.fbp_fht(P[1].cpu().double(), torch.tensor(B2[0]), torch.tensor(B2[1]))
    err = float(torch.linalg.vector_norm(got[1].cpu().double() - oref) /
                torch.linalg.vector_norm(oref))
    assert err < 1e-5


def test_noalloc_rejects_a_slice_larger_than_the_array(gpu_lib):
    api = gpu_lib
    N = 4096                 # [2, 5, 5]: two 256 MiB buffers per slice
    with api.fbp_plan(N, 1, *B2, flags=api.FBP_NO_SCRATCH) as plan:
        P = torch.zeros(1, 4, N, N, device="cuda")
        img = torch.zeros(1, N, N, device="cuda")
        with pytest.raises(api.FbpError) as e:
            api.fbp_reconstruct_noalloc(plan, P, img)
        assert e.value.code == api.FBP_ERANGE
        assert float(img.abs().max()) == 0.0
