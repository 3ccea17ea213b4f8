"""The batched entry point that allocates no device memory
(wt_plan_run_batch_static): same kernels and launch grids as
wt_plan_run_batch, with every intermediate and the argument table in the
library's fixed workspace, so its outputs equal wt_plan_run_batch's bit for
bit.  Two calls in a row, the second with a smaller batch, each checked
against wt_plan_run_batch and the FP64 oracle; and the host-side refusal of
a batch whose intermediates exceed the workspace."""
import ctypes
import sys

import numpy as np
import pytest

import oracle
import synth
from synth import pipelines as P
from wt_helpers import assert_normwise

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _batch(torch, sizes, seed):
    dev = torch.device("cuda:0")
    host = [[synth.uniform_image(seed + 2 * i, 1, h, w), synth.uniform_image(seed + 2 * i + 1, 1, h, w),
             synth.ramp_mask(h, w)] for i, (w, h) in enumerate(sizes)]
    ins = [[torch.from_numpy(x).to(dev) for x in pair] for pair in host]
    return host, ins


def test_static_batch_equals_run_batch_twice():
    import torch
    import paper_1909_07190_amd as wt
    spec = P.pyramid_blend(3)
    plan = wt.from_spec(spec).plan(300, 200, mode="analytic", any_width=True, batch_images=5)
    _say(f"plan: {plan.describe().strip()}")
    dev = torch.device("cuda:0")
    for call, sizes in enumerate(([(300, 200), (129, 77), (517, 263), (64, 61), (1000, 33)],
                                  [(129, 77), (90, 45), (200, 121)])):
        _say(f"call {call}: {len(sizes)} images {sizes}")
        host, ins = _batch(torch, sizes, 900 + 40 * call)
        ref = [[torch.full((1, h, w), float("nan"), device=dev)] for (w, h) in sizes]
        got = [[torch.full((1, h, w), float("nan"), device=dev)] for (w, h) in sizes]
        plan.run_batch(ins, ref)
        plan.run_batch_static(ins, got)
        torch.cuda.synchronize()
        for i, (r, g) in enumerate(zip(ref, got)):
            assert torch.equal(r[0], g[0]), f"call {call} image {i}: static batch differs from run_batch"
            a, b, m = host[i]
            want = oracle.evaluate(spec, {"A": a, "B": b, "M": m})["R0"]
            assert_normwise(g[0].cpu().numpy(), want, 1e-5, f"call {call} image {i}")


def test_static_batch_refuses_workspace_overflow():
    """Eight 4096 x 4096 pairs need more intermediate storage than the
    fixed workspace holds (every coarser Gaussian level of A, B and M alone
    is 8 x 3 x 16.8 MB): refused on the host (WT_E_NOMEM), no launch."""
    import torch
    import paper_1909_07190_amd as wt
    spec = P.pyramid_blend(3)
    plan = wt.from_spec(spec).plan(512, 512, mode="analytic", any_width=True, batch_images=8)
    dev = torch.device("cuda:0")
    sizes = [(4096, 4096)] * 8
    ins = [[torch.zeros((1, h, w), device=dev) for _ in range(3)] for (w, h) in sizes]
    outs = [[torch.zeros((1, h, w), device=dev)] for (w, h) in sizes]
    with pytest.raises(wt.WtError) as e:
        plan.run_batch_static(ins, outs)
    assert e.value.status == -4  # WT_E_NOMEM
    assert "workspace" in str(e.value)
    torch.cuda.synchronize()


def test_static_batch_histograms_twice():
    """A histogram fused into the blur's group through the allocation-free
    entry point: its counts are cleared by the library's kernel before each
    accumulation, so two calls in a row (the second with fewer images) each
    equal wt_plan_run_batch's counts and the oracle's."""
    import torch
    import paper_1909_07190_amd as wt
    spec = P.blur_histogram(channels=2, bins=64)
    plan = wt.from_spec(spec).plan(400, 300, mode="analytic", any_width=True, batch_images=4)
    assert "hst=3" in plan.describe()
    dev = torch.device("cuda:0")
    for call, sizes in enumerate(([(400, 300), (97, 41), (1000, 513), (64, 64)], [(97, 41), (250, 130)])):
        _say(f"histogram call {call}: {sizes}")
        imgs = [synth.dyadic_image(960 + 10 * call + i, 2, h, w) for i, (w, h) in enumerate(sizes)]
        ins = [[torch.from_numpy(im).to(dev)] for im in imgs]
        ref = [[torch.full((2, 1, 64), 0x5A, dtype=torch.int32, device=dev)] for _ in sizes]
        got = [[torch.full((2, 1, 64), 0x5A, dtype=torch.int32, device=dev)] for _ in sizes]
        plan.run_batch(ins, ref)
        plan.run_batch_static(ins, got)
        torch.cuda.synchronize()
        for i, im in enumerate(imgs):
            assert torch.equal(ref[i][0], got[i][0]), f"call {call} image {i}"
            want = oracle.evaluate(spec, {"img": im})["h"]
            assert np.array_equal(got[i][0].cpu().numpy().astype(np.int64), want), f"call {call} image {i}"
