"""Pre-profiling on the device: stage bodies timed by a one-lane
microbenchmark, VGPRs read from the compiled kernels."""
import pytest

import paper_1909_07190_amd as wt

pytestmark = pytest.mark.gpu


def test_stage_profiles_are_measured_and_ordered():
    print("stage profiles", flush=True)
    spec = {"inputs": [{"name": "img", "channels": 1}],
            "stages": [{"name": "big", "kind": "stencil", "src": "img", "kw": 7, "kh": 7, "ax": 3, "ay": 3,
                        "weights": [1.0 + (i % 5) for i in range(49)], "scale": 0.01},
                       {"name": "small", "kind": "pointwise", "srcs": ["img"], "expr": "abs(s0)", "channels": 1}],
            "outputs": ["big", "small"]}
    pipe = wt.from_spec(spec)
    big = wt.stage_profile(pipe, 1, 512, 512, measure=True)
    small = wt.stage_profile(pipe, 2, 512, 512, measure=True)
    assert big[2] and small[2]
    assert big[0] > 0 and small[0] > 0
    assert big[0] > small[0], (big, small)
    assert big[1] >= 2 and small[1] >= 2
