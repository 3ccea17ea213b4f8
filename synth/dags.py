"""Seeded random pipeline DAGs (plain data, no arithmetic performed here).

Stages: 3x3 / 5x5 stencils (binomial blur, box, Sobel, Laplacian, separable
5-tap blurs), pointwise operations (add, sub, scale, abs, min, max, lerp)
and 2x down/up-sampling, on single-channel inputs.  Every sink is a pipeline
output.  Pointwise operations are continuous (no data-dependent selects), so
FP32 results stay within normwise tolerance of the FP64 oracle.
"""
from __future__ import annotations

from . import SplitMix64

STENCILS = {
    "gauss3": (3, 3, [1, 2, 1, 2, 4, 2, 1, 2, 1], 1 / 16),
    "gauss5": (5, 5, [a * b for a in (1, 4, 6, 4, 1) for b in (1, 4, 6, 4, 1)], 1 / 256),
    "box3": (3, 3, [1] * 9, 1 / 9),
    "sobelx": (3, 3, [-1, 0, 1, -2, 0, 2, -1, 0, 1], 1 / 8),
    "sobely": (3, 3, [-1, -2, -1, 0, 0, 0, 1, 2, 1], 1 / 8),
    "laplace": (3, 3, [0, 1, 0, 1, -4, 1, 0, 1, 0], 1 / 4),
    "blurx5": (5, 1, [1, 4, 6, 4, 1], 1 / 16),
    "blury5": (1, 5, [1, 4, 6, 4, 1], 1 / 16),
}
POINTWISE = {
    "add": (2, "s0 + s1"), "sub": (2, "s0 - s1"), "scale": (1, "0.75 * s0 + 0.125"),
    "abs": (1, "abs(s0)"), "min": (2, "min(s0, s1)"), "max": (2, "max(s0, s1)"),
    "lerp": (2, "s0 + 0.3 * (s1 - s0)"),
}


def random_dag(seed: int, lo: int = 8, hi: int = 24, max_level: int = 2) -> dict:
    rng = SplitMix64(seed)
    n = rng.uniform_int(lo, hi)
    nin = 1 + rng.uniform_int(0, 1)
    inputs = [{"name": f"in{i}", "channels": 1} for i in range(nin)]
    level = {f"in{i}": 0 for i in range(nin)}
    order = list(level)
    stages = []

    def pick(lvl=None):
        cands = [x for x in order if lvl is None or level[x] == lvl]
        recent = cands[-4:]
        return recent[rng.uniform_int(0, len(recent) - 1)]

    while len(stages) < n:
        r = rng.uniform_int(0, 99)
        name = f"s{len(stages)}"
        src = pick()
        if r < 40:
            k = sorted(STENCILS)[rng.uniform_int(0, len(STENCILS) - 1)]
            kw, kh, w, sc = STENCILS[k]
            stages.append({"name": name, "kind": "stencil", "src": src, "kw": kw, "kh": kh,
                           "ax": kw // 2, "ay": kh // 2, "weights": [float(v) for v in w], "scale": sc})
            level[name] = level[src]
        elif r < 75:
            k = sorted(POINTWISE)[rng.uniform_int(0, len(POINTWISE) - 1)]
            ar, expr = POINTWISE[k]
            srcs = [src] + ([pick(level[src])] if ar == 2 else [])
            stages.append({"name": name, "kind": "pointwise", "srcs": srcs, "expr": expr, "channels": 1})
            level[name] = level[src]
        elif r < 87 and level[src] < max_level:
            stages.append({"name": name, "kind": "down2", "src": src})
            level[name] = level[src] + 1
        elif level[src] >= 1:
            stages.append({"name": name, "kind": "up2", "src": src})
            level[name] = level[src] - 1
        else:
            continue
        order.append(name)
    # return to full resolution
    while level[order[-1]] > 0:
        name = f"s{len(stages)}"
        stages.append({"name": name, "kind": "up2", "src": order[-1]})
        level[name] = level[order[-1]] - 1
        order.append(name)
    used = set()
    for st in stages:
        used.update(st.get("srcs", [st.get("src")]))
    outputs = [st["name"] for st in stages if st["name"] not in used]
    return {"inputs": inputs, "stages": stages, "outputs": outputs}
