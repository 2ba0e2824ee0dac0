"""Pass schedules, mixed-size batches and captured graphs, through the C ABI.

Regrouping the butterfly levels (eq 19-21) into passes changes no addition, so every schedule
must give bit-identical images; a mixed batch must equal its sub-batches run one by one; a
captured graph must equal the eager calls on every replay, with eager work between replays.
One slice per size is held to the FP64 oracle at the usual float32 bar.
"""
import numpy as np
import pytest
import torch

import fbp_inputs as I
import oracle as O

pytestmark = pytest.mark.gpu

B2 = ([0.12372452, -0.12372452], [-0.17164439, -0.13239954])
B4 = ([0.12493199, -0.122976, -0.0727046, 0.07074861],
      [-0.17279862, -0.72164016, 0.07148985, 0.04270461])


def _coef(order=2):
    """Balanced ramp-like sets (sum(b) = 0): the plan filters them in first-difference form."""
    b, a = B2 if order == 2 else B4
    return np.array(b, np.float64), np.array(a, np.float64)


def _lino(N, B, seed):
    ells = I.random_ellipses(N, 10, seed, disc=0.34 if N >= 64 else 0.25, batch=B)
    return I.linogram(ells, N, device="cuda", dtype=torch.float32)


def _rel(got, ref):
    got = got.detach().cpu().double()
    return float(torch.linalg.vector_norm(got - ref) / torch.linalg.vector_norm(ref))


@pytest.mark.parametrize("N,B,order,schedules", [
    (64, 2, 2, [[6], [3, 3], [2, 2, 2], [1, 5], [5, 1]]),
    (256, 2, 2, [[4, 4, 0], [2, 6, 7], [4, 4, 7], [4, 4, 6], [3, 3, 2, 8], [1, 1, 6, 7],
                 [1, 7, 8]]),
    (512, 2, 2, [[2, 7, 8], [1, 1, 7, 8]]),
    (1024, 2, 2, [[5, 5, 7], [5, 5, 9], [4, 6, 7], [3, 3, 4, 8], [2, 4, 4, 8], [5, 1, 4, 8],
                  [3, 7, 8], [1, 2, 7, 8]]),
    (1024, 1, 4, [[4, 6, 7], [3, 3, 4, 8], [5, 1, 4, 8], [3, 7, 8]]),
    (2048, 1, 2, [[4, 4, 3, 8], [3, 5, 3, 8], [4, 3, 4, 9], [2, 3, 3, 3, 8], [4, 7, 8]]),
    (4096, 1, 2, [[3, 4, 5, 8], [1, 6, 5, 8], [3, 5, 4, 8], [2, 5, 5, 9], [3, 2, 7, 8]]),
    (4096, 1, 4, [[3, 4, 5, 8], [1, 6, 5, 8], [3, 5, 4, 8], [3, 2, 7, 8]]),
])
def test_schedules_are_bit_identical(gpu_lib, N, B, order, schedules):
    """Every listed schedule is one the kernels can run (last entry: log2 of the column-tile
    width, 0 = keep; below N = 256 there are no column tiles).  Order 4 at N = 4096 runs pass
    0 of 1, 2 and 3 levels on the two-wave first-pass kernel."""
    api = gpu_lib
    P = _lino(N, B, seed=N)
    with api.fbp_plan(N, B, *_coef(order)) as plan:
        ref = api.fbp_reconstruct(plan, P).clone()
        bp_ref = api.fht_backproject(plan, P).clone()
        fwd_ref = api.fht_forward(plan, ref).clone()
        for sched in schedules:
            levels, w = (sched[:-1], sched[-1]) if N >= 256 else (sched, 0)
            plan.set_schedule(levels, w)
            assert plan.passes() == list(levels)
            got = api.fbp_reconstruct(plan, P)
            assert torch.equal(got, ref), (levels, w)
            assert torch.equal(api.fht_backproject(plan, P), bp_ref), (levels, w)
            assert torch.equal(api.fht_forward(plan, ref), fwd_ref), (levels, w)
        torch.cuda.synchronize()


@pytest.mark.parametrize("N,B,split", [(256, 3, ([3, 1, 4], 8)), (1024, 2, ([5, 1, 4], 8)),
                                        (2048, 1, ([2, 4, 1, 4], 8))])
def test_last_pass_kernels(gpu_lib, N, B, split):
    """A last pass of 5 levels runs as one launch over 128 x 128 image tiles (all four classes);
    a last pass of other depth runs split by class pair (two launches).  Same additions in the
    same order, so the images are bit-identical."""
    api = gpu_lib
    P = _lino(N, B, seed=N + 77)

    def run(plan):
        plan.profile(True)
        img = api.fbp_reconstruct(plan, P).clone()
        kinds = plan.profile_read()
        plan.profile(False)
        return img, kinds

    with api.fbp_plan(N, B, *_coef()) as plan:
        ref, kinds = run(plan)
        assert kinds["last"][1] == 1 and "last_v" not in kinds and "last_h" not in kinds
        plan.set_schedule(*split)
        got, kinds = run(plan)
        assert kinds["last_v"][1] == 1 and kinds["last_h"][1] == 1 and "last" not in kinds
        assert torch.equal(got, ref)


def test_schedule_rejections(gpu_lib):
    api = gpu_lib
    with api.fbp_plan(1024, 1, *_coef()) as plan:
        levels, w, first_max = plan.schedule()
        assert sum(levels) == 10 and first_max >= levels[0]
        cases = [([5, 4], 8, api.FBP_EINVAL),            # levels do not sum to log2 N
                 ([5, 0, 5], 8, api.FBP_EINVAL),         # an empty pass
                 ([first_max + 1, 10 - first_max - 1], 8, api.FBP_ERANGE),
                 ([5, 5], 5, api.FBP_ERANGE),            # column tile too narrow
                 ([5, 5], 11, api.FBP_ERANGE),           # wider than the row
                 ([2, 8], 8, api.FBP_ERANGE),            # 2^8-row column tile overflows LDS
                 ([4, 6], 8, api.FBP_ERANGE)]            # two-class 64 x 320 tile: 169 KB
        for lv, ww, code in cases:
            with pytest.raises(api.FbpError) as e:
                plan.set_schedule(lv, ww)
            assert e.value.code == code, (lv, ww)
        assert plan.schedule()[:2] == (levels, w)       # unchanged after the failures


def _mixed(sizes_counts, seed=0):
    plans, linos, imgs = [], [], []
    for i, (N, count) in enumerate(sizes_counts):
        plans.append(_plan_cache(N, count))
        linos.append(_lino(N, count, seed=seed + 7 * i + N))
        imgs.append(torch.empty((count, N, N), device="cuda"))
    return plans, linos, imgs


_PLANS = {}


def _plan_cache(N, count):
    from paper_2007_06289_amd import api
    key = (N, count)
    if key not in _PLANS:
        _PLANS[key] = api.fbp_plan(N, count, *_coef())
    return _PLANS[key]


MIXED = [(256, 16), (512, 16), (1024, 16), (2048, 16)]   # 64 slices of four sizes


def test_mixed_batch_matches_single_calls_and_oracle(gpu_lib):
    api = gpu_lib
    plans, linos, imgs = _mixed(MIXED)
    api.fbp_reconstruct_many(plans, linos, imgs)
    for p, lino, img in zip(plans, linos, imgs):
        single = api.fbp_reconstruct(p, lino)
        assert torch.equal(single, img), p.n
    torch.cuda.synchronize()
    # one slice of the two smaller sizes against the FP64 oracle
    b, a = _coef()
    for k in (0, 1):
        ref = O.fbp_fht(linos[k][:1].cpu().double(), torch.tensor(b), torch.tensor(a))
        assert _rel(imgs[k][:1], ref) < 1e-5


def test_mixed_batch_argument_errors(gpu_lib):
    api = gpu_lib
    lib = api.load_library()
    plans, linos, imgs = _mixed([(256, 2)])
    with pytest.raises(api.FbpError) as e:
        api.fbp_reconstruct_many(plans, [_lino(256, 3, 1)], [torch.empty(3, 256, 256,
                                                                          device="cuda")])
    assert e.value.code == api.FBP_ERANGE
    with pytest.raises(ValueError):
        api.fbp_reconstruct_many(plans, linos, [])
    assert lib.fbp_reconstruct_many(None, None, None, None, 0, None) == api.FBP_OK
    assert lib.fbp_reconstruct_many(None, None, None, None, -1, None) == api.FBP_EINVAL
    assert lib.fbp_reconstruct_many(None, None, None, None, 1, None) == api.FBP_EINVAL


def test_graph_replays_match_eager(gpu_lib):
    api = gpu_lib
    plans, linos, imgs = _mixed(MIXED, seed=100)
    g = api.fbp_graph_create(plans, linos, imgs)
    eager = [torch.empty_like(x) for x in imgs]
    for rep in range(3):
        # eager work between the replays: change the inputs in place, reconstruct eagerly
        for k, lino in enumerate(linos):
            lino.mul_(1.0 + 0.25 * rep).add_(0.001 * (k + 1))
        api.fbp_reconstruct_many(plans, linos, eager)
        torch.cuda.synchronize()
        for x in imgs:
            x.fill_(float("nan"))
        g.launch()
        torch.cuda.synchronize()
        for k in range(len(imgs)):
            assert torch.equal(imgs[k], eager[k]), (rep, plans[k].n)
    g.close()


def test_graph_sees_new_coefficients_and_refuses_a_new_schedule(gpu_lib):
    api = gpu_lib
    N = 256
    lino = _lino(N, 2, seed=5)
    img = torch.empty((2, N, N), device="cuda")
    with api.fbp_plan(N, 2, *_coef()) as plan:
        g = api.fbp_graph_create([plan], [lino], [img])
        b1 = np.array([[0.11, -0.11]], np.float32).astype(np.float64)
        a1 = np.array([[-0.3, 0.02]], np.float32).astype(np.float64)
        api.fbp_plan_set_coefficients(plan, b1, a1)
        g.launch()
        want = api.fbp_reconstruct(plan, lino)
        torch.cuda.synchronize()
        assert torch.equal(img, want)
        plan.set_schedule([4, 4], 8)                      # not the default ([3, 5])
        with pytest.raises(api.FbpError) as e:
            g.launch()
        assert e.value.code == api.FBP_EINVAL
        g.close()
        g2 = api.fbp_graph_create([plan], [lino], [img])   # recapture with the new schedule
        g2.launch()
        torch.cuda.synchronize()
        assert torch.equal(img, want)
        g2.close()


def test_graph_refuses_a_new_scan_depth(gpu_lib):
    """The scan depth is a kernel argument: coefficients whose chunk transitions decay slowly
    (a double pole at 0.95: every scan level) after fast-decaying ones (the order-2 time-domain
    fit: no level) make a captured graph stale; it refuses to launch, and a recapture gives
    the eager result, which matches the FP64 oracle."""
    api = gpu_lib
    N = 256
    lino = _lino(N, 2, seed=8)
    img = torch.empty((2, N, N), device="cuda")
    with api.fbp_plan(N, 2, *_coef()) as plan:
        assert plan.filter_info()["scan_levels"] == 0
        g = api.fbp_graph_create([plan], [lino], [img])
        g.launch()
        torch.cuda.synchronize()
        b1 = np.array([[0.12, -0.12]])
        a1 = np.array([[-1.9, 0.9025]])
        api.fbp_plan_set_coefficients(plan, b1, a1)
        assert plan.filter_info()["scan_levels"] == 7
        with pytest.raises(api.FbpError) as e:
            g.launch()
        assert e.value.code == api.FBP_EINVAL
        g.close()
        want = api.fbp_reconstruct(plan, lino)
        g2 = api.fbp_graph_create([plan], [lino], [img])
        g2.launch()
        torch.cuda.synchronize()
        assert torch.equal(img, want)
        g2.close()
    ref = O.fbp_fht(lino.cpu().double(), torch.tensor(b1[0]), torch.tensor(a1[0]))
    # 2^-24 times the noise gain of 1/(1 - 0.95 z^-1)^2 (400), twice over
    assert _rel(want, ref) < 2 * 2.0 ** -24 * 400


def test_empty_graph_and_zero_batches(gpu_lib):
    api = gpu_lib
    g = api.fbp_graph_create([], [], [])
    g.launch()
    g.close()
    N = 64
    with api.fbp_plan(N, 2, *_coef()) as plan:
        lino0 = torch.empty((0, 4, N, N), device="cuda")
        img0 = torch.empty((0, N, N), device="cuda")
        lino = _lino(N, 2, seed=9)
        img = torch.empty((2, N, N), device="cuda")
        g = api.fbp_graph_create([plan, plan], [lino0, lino], [img0, img])
        g.launch()
        want = api.fbp_reconstruct(plan, lino)
        torch.cuda.synchronize()
        assert torch.equal(img, want)
        g.close()


def test_autotune_applies_and_caches(gpu_lib, tmp_path):
    api = gpu_lib
    from paper_2007_06289_amd import autotune
    N, B = 256, 4
    lino = _lino(N, B, seed=11)
    cache = str(tmp_path / "sched.json")
    with api.fbp_plan(N, B, *_coef()) as plan:
        ref = api.fbp_reconstruct(plan, lino).clone()
        res = autotune.tune(plan, lino, reps=2, cache_path=cache)
        assert not res["cached"] and res["tried"] >= 2
        assert plan.schedule()[:2] == (res["levels"], res["log2w"])
        assert torch.equal(api.fbp_reconstruct(plan, lino), ref)
    with api.fbp_plan(N, B, *_coef()) as plan2:
        res2 = autotune.tune(plan2, lino, cache_path=cache)
        assert res2["cached"] and plan2.schedule()[:2] == (res["levels"], res["log2w"])
        torch.cuda.synchronize()
