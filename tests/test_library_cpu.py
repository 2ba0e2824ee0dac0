"""The C-ABI library on a machine without a GPU: it loads, exports every declared entry point,
rejects bad arguments before touching the device, and its host-side coefficient fit works."""
import os
import re

import numpy as np
import pytest
import torch

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return names


@pytest.fixture(scope="module")
def lib():
    from paper_2007_06289_amd import api
    return api.load_library()


def test_every_declared_symbol_is_exported(lib):
    names = _declared_functions()
    assert {"fbp_plan", "fbp_filter", "fht_backproject", "fht_forward",
            "fbp_reconstruct"} <= names
    for n in names:
        assert hasattr(lib, n), n


def test_plan_rejects_bad_descriptions_without_a_device():
    from paper_2007_06289_amd import api
    good_b, good_a = [0.125, -0.12], [-0.17, -0.13]
    cases = [
        (dict(n=6), api.FBP_EINVAL),
        (dict(n=2), api.FBP_EINVAL),
        (dict(n=8192), api.FBP_EINVAL),
        (dict(max_batch=0), api.FBP_EINVAL),
        (dict(b=[0.1] * 9, a=[0.0] * 9), api.FBP_EINVAL),
        (dict(a=[0.0, 1.0]), api.FBP_EUNSTABLE),
        (dict(a=[-2.5, 1.2]), api.FBP_EUNSTABLE),
        (dict(b=[float("nan"), 0.1]), api.FBP_EUNSTABLE),
        (dict(flags=64), api.FBP_EINVAL),
    ]
    for kw, code in cases:
        args = dict(n=64, max_batch=1, b=good_b, a=good_a, flags=0)
        args.update(kw)
        with pytest.raises(api.FbpError) as e:
            api.fbp_plan(args["n"], args["max_batch"], args["b"], args["a"], args["flags"])
        assert e.value.code == code, (kw, e.value.code)


def test_entry_points_reject_null_plan(lib):
    assert lib.fbp_filter(None, None, None, 1) == -1
    assert lib.fht_backproject(None, None, None, 1) == -1
    assert lib.fht_forward(None, None, None, 1) == -1
    assert lib.fbp_reconstruct(None, None, None, 1) == -1
    assert lib.fbp_plan_destroy(None) == 0
    assert lib.fbp_direct_parallel(None, None, None, 1, 48, 8, 8, None) == -1
    assert lib.fbp_strerror(-2).decode().startswith("recursive filter")


@pytest.mark.parametrize("order,dc0,bound", [(1, False, 0.32), (2, False, 0.025),
                                             (2, True, 0.033), (3, True, 0.023)])
def test_host_fit_matches_the_ramp_half(order, dc0, bound):
    from paper_2007_06289_amd import api
    L = 256
    b, a, err = api.fbp_fit_ramp_iir(order, L, dc_zero=dc0)
    # independent check of the reported error with the oracle's recursion and ramp
    g = O.iir_impulse_response(torch.tensor(b), torch.tensor(a), L)
    hp = O.ramp_causal(L)
    rel = float(torch.linalg.vector_norm(g - hp) / torch.linalg.vector_norm(hp))
    assert abs(rel - err) < 1e-9
    assert err < bound
    if dc0:
        assert abs(b.sum()) < 1e-12
    # stable: all poles inside the unit circle
    assert np.abs(np.roots(np.concatenate([[1.0], a]))).max() < 1.0


def test_schedule_and_graph_entry_points_reject_bad_arguments(lib):
    assert lib.fbp_plan_set_schedule(None, None, 0, 0) == -1
    assert lib.fbp_plan_schedule_info(None, None, None) == -1
    # an empty mixed batch is a no-op and needs no device
    assert lib.fbp_reconstruct_many(None, None, None, None, 0, None) == 0
    assert lib.fbp_reconstruct_many(None, None, None, None, -1, None) == -1
    assert lib.fbp_reconstruct_many(None, None, None, None, 2, None) == -1
    assert lib.fbp_graph_create(None, None, None, None, 0, None) == -1
    assert lib.fbp_graph_launch(None, None) == -1
    assert lib.fbp_graph_destroy(None) == 0


def test_schedule_candidates_are_all_compositions():
    from math import comb

    from paper_2007_06289_amd.autotune import compositions
    for total in range(1, 13):
        for parts in range(1, 5):
            got = compositions(total, parts, total)
            assert len(got) == len(set(got))
            assert all(sum(c) == total and 1 <= len(c) <= parts for c in got)
            assert len(got) == sum(comb(total - 1, j - 1) for j in range(1, parts + 1))
    assert all(max(c) <= 3 for c in compositions(10, 4, 3))
