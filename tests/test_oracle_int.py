"""Pins of the oracle's integer stages (round-half-up division, saturation,
exact integer pointwise arithmetic), by brute force and hand-computed values."""
from fractions import Fraction
import math

import numpy as np
import pytest

import oracle
import synth


def _clamp(v, lo, hi):
    return lo if v < lo else hi if v > hi else v


def _brute_stencil(img, kw, kh, ax, ay, w, d, lo, hi):
    c, h, wd = img.shape
    out = np.zeros_like(img)
    for ch in range(c):
        for y in range(h):
            for x in range(wd):
                acc = 0
                for j in range(kh):
                    for i in range(kw):
                        acc += int(w[j * kw + i]) * int(img[ch, _clamp(y + j - ay, 0, h - 1),
                                                             _clamp(x + i - ax, 0, wd - 1)])
                # round half up: floor(acc/d + 1/2) with exact rationals
                q = math.floor(Fraction(acc, d) + Fraction(1, 2))
                out[ch, y, x] = _clamp(q, lo, hi)
    return out


def test_u8_binomial_is_add_8_shift_4():
    img = synth.integer_image(1, 1, 5, 9, 0, 255)
    got = oracle.stencil_int(img, 5, 1, 2, 0, [1, 4, 6, 4, 1], 16, "u8")
    for y in range(5):
        for x in range(9):
            acc = sum(wv * int(img[0, y, _clamp(x + i - 2, 0, 8)]) for i, wv in enumerate([1, 4, 6, 4, 1]))
            assert got[0, y, x] == (acc + 8) >> 4


def test_round_half_up_on_negative_values():
    v = np.array([[[-3, -1, 1, 3, -5, -6, 6, 0]]], dtype=np.int64)
    # divisor 2: -1.5 -> -1, -0.5 -> 0, 0.5 -> 1, 1.5 -> 2, -2.5 -> -2, -3 -> -3, 3 -> 3
    assert oracle.stencil_int(v, 1, 1, 0, 0, [1], 2, "i16").tolist() == [[[-1, 0, 1, 2, -2, -3, 3, 0]]]
    # divisor 4: -0.75 -> -1, -0.25 -> 0, 0.25 -> 0, 0.75 -> 1, -1.25 -> -1, -1.5 -> -1, 1.5 -> 2
    assert oracle.stencil_int(v, 1, 1, 0, 0, [1], 4, "i16").tolist() == [[[-1, 0, 0, 1, -1, -1, 2, 0]]]


@pytest.mark.parametrize("shape", [(1, 1, 1), (1, 2, 3), (2, 7, 5), (1, 4, 17)])
def test_box_divisor_9_and_sharpen_saturation_by_brute_force(shape):
    img = synth.integer_image(sum(shape), *shape, 0, 255)
    box = [1] * 9
    assert np.array_equal(oracle.stencil_int(img, 3, 3, 1, 1, box, 9, "u8"),
                          _brute_stencil(img, 3, 3, 1, 1, box, 9, 0, 255))
    sharp = [0, -1, 0, -1, 5, -1, 0, -1, 0]
    got = oracle.stencil_int(img, 3, 3, 1, 1, sharp, 1, "u8")
    assert np.array_equal(got, _brute_stencil(img, 3, 3, 1, 1, sharp, 1, 0, 255))
    got16 = oracle.stencil_int(img, 3, 3, 1, 1, sharp, 3, "i16")
    assert np.array_equal(got16, _brute_stencil(img, 3, 3, 1, 1, sharp, 3, -32768, 32767))


def test_saturation_corners():
    full = np.full((1, 4, 4), 255, dtype=np.int64)
    lap = [0, 1, 0, 1, 4, 1, 0, 1, 0]
    assert np.all(oracle.stencil_int(full, 3, 3, 1, 1, lap, 1, "u8") == 255)
    assert np.all(oracle.stencil_int(full, 3, 3, 1, 1, lap, 1, "u16") == 2040)
    assert np.all(oracle.stencil_int(full, 3, 3, 1, 1, lap, 8, "u8") == 255)
    a = np.array([[[3, 10, 200]]], dtype=np.int64)
    b = np.array([[[5, 10, 100]]], dtype=np.int64)
    assert oracle.pointwise("s0 - s1", [a, b], 1, "u8").tolist() == [[[0, 0, 100]]]
    assert oracle.pointwise("s0 - s1", [a, b], 1, "i16").tolist() == [[[-2, 0, 100]]]
    assert oracle.pointwise("s0 * s1", [a, b], 1, "u8").tolist() == [[[15, 100, 255]]]
    assert oracle.pointwise("s0 * s1", [a, b], 1, "i32").tolist() == [[[15, 100, 20000]]]


def test_integer_pointwise_matches_python_loops():
    a = synth.integer_image(5, 1, 3, 7, -300, 300)
    b = synth.integer_image(6, 1, 3, 7, -300, 300)
    got = oracle.pointwise("select(s0 < s1, abs(s0) - 2 * s1, max(s0, s1) - min(s0, -s1) + 7)", [a, b], 1, "i16")
    for y in range(3):
        for x in range(7):
            s0, s1 = int(a[0, y, x]), int(b[0, y, x])
            want = abs(s0) - 2 * s1 if s0 < s1 else max(s0, s1) - min(s0, -s1) + 7
            assert got[0, y, x] == _clamp(want, -32768, 32767)


def test_float_stage_reads_integer_values_exactly():
    spec = {"inputs": [{"name": "img", "channels": 1, "dtype": "u8"}],
            "stages": [{"name": "b", "kind": "stencil", "src": "img", "kw": 3, "kh": 1, "ax": 1, "ay": 0,
                        "weights": [1, 2, 1], "scale": 0.25},
                       {"name": "q", "kind": "down2", "src": "img"}],
            "outputs": ["b", "q"]}
    img = synth.integer_image(9, 1, 4, 6, 0, 255)
    out = oracle.evaluate(spec, {"img": img.astype(np.uint8)})
    assert out["b"].dtype == np.float64 and out["q"].dtype == np.int64
    ref = oracle.stencil(img.astype(np.float64), 3, 1, 1, 0, [1, 2, 1], 0.25)
    assert np.array_equal(out["b"], ref)
    assert np.array_equal(out["q"], img[:, 0::2, 0::2])


def test_integer_rules_are_enforced():
    f = np.zeros((1, 2, 2))
    i = np.zeros((1, 2, 2), dtype=np.int64)
    with pytest.raises(ValueError):
        oracle.stencil_int(f, 1, 1, 0, 0, [1], 1, "u8")
    with pytest.raises(ValueError):
        oracle.stencil_int(i, 1, 1, 0, 0, [0.5], 1, "u8")
    with pytest.raises(ValueError):
        oracle.pointwise("s0 / 2", [i], 1, "i16")
    with pytest.raises(ValueError):
        oracle.pointwise("s0 + 0.5", [i], 1, "i16")
    with pytest.raises(ValueError):
        oracle.pointwise("s0 + 1", [f], 1, "i16")
    spec = {"inputs": [{"name": "img", "channels": 1, "dtype": "u8"}],
            "stages": [{"name": "d", "kind": "down2", "src": "img"},
                       {"name": "u", "kind": "up2", "src": "d"}], "outputs": ["u"]}
    with pytest.raises(ValueError):
        oracle.evaluate(spec, {"img": np.zeros((1, 4, 4), dtype=np.uint8)})
    with pytest.raises(ValueError):
        oracle.evaluate({"inputs": [{"name": "img", "channels": 1, "dtype": "u8"}], "stages": [
            {"name": "b", "kind": "pointwise", "srcs": ["img"], "expr": "s0", "channels": 1}], "outputs": ["b"]},
            {"img": np.full((1, 2, 2), 256)})
