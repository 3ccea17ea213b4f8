"""The learned cost model's device kernels against the FP64 oracle."""
import numpy as np
import pytest

import paper_1909_07190_amd as wt
from oracle import mlp as M

pytestmark = pytest.mark.gpu
DIMS = (40, 128, 128, 128, 1)


def _rel(a, b):
    return float(np.max(np.abs(np.asarray(a, np.float64) - b)) / max(np.max(np.abs(b)), 1e-30))


def test_forward_backward_match_oracle():
    print("mlp forward/backward", flush=True)
    net = wt.Mlp(DIMS, seed=3)
    assert net.num_params == 38401
    p = net.params().astype(np.float64)
    rng = np.random.default_rng(1)
    for batch in (1, 37, 256):
        x = rng.normal(size=(batch, 40)).astype(np.float32)
        t = rng.normal(size=batch).astype(np.float32)
        y = net.forward(x)
        ref = M.forward(p, DIMS, x.astype(np.float64))[-1]
        assert _rel(y, ref) <= 1e-4
        loss, g = net.forward_backward(x, t)
        rl, rg = M.loss_and_grad(p, DIMS, x.astype(np.float64), t.astype(np.float64))
        assert abs(loss - rl) <= 1e-4 * abs(rl)
        assert _rel(g, rg) <= 1e-4, f"batch {batch}: gradient err {_rel(g, rg):.2e}"


def test_adam_step_matches_oracle():
    print("mlp adam", flush=True)
    net = wt.Mlp((8, 16, 1), seed=4)
    p0 = net.params().astype(np.float64)
    rng = np.random.default_rng(2)
    m = np.zeros_like(p0)
    v = np.zeros_like(p0)
    p = p0
    for step in (1, 2, 3):
        g = rng.normal(size=p0.size).astype(np.float32)
        net.adam_step(g, 1e-2)
        p, m, v = M.adam(p, g.astype(np.float64), m, v, step, 1e-2)
        np.testing.assert_allclose(net.params(), p, rtol=1e-5, atol=1e-6)


def test_fits_a_teacher_network():
    """Data from a fixed random teacher network is learnable to small loss."""
    print("mlp teacher fit", flush=True)
    rng = np.random.default_rng(7)
    tdims = [40, 16, 1]
    tn = sum(a * b + b for a, b in zip(tdims[:-1], tdims[1:]))
    tp = rng.normal(size=tn) * 0.3
    x = rng.normal(size=(4096, 40))
    t = M.forward(tp, tdims, x)[-1][:, 0]
    net = wt.Mlp(DIMS, seed=5)
    net.train(x.astype(np.float32), t.astype(np.float32), epochs=60, batch=256, lr=1e-3, seed=1)
    pred = net.predict(x.astype(np.float32))
    mse = float(np.mean((pred - t) ** 2)) / float(np.var(t))
    assert mse < 2e-2, f"relative training MSE {mse:.3e}"


def test_model_train_from_measurement_db(tmp_path):
    """wt_model_train on a measurement database equals training the same
    network on the same rows through wt_mlp_train (same seed, same device
    kernels), and fits the database's timings."""
    import json
    print("model train from a measurement database", flush=True)
    rng = np.random.default_rng(9)
    tdims = [40, 8, 1]
    tp = rng.normal(size=sum(a * b + b for a, b in zip(tdims[:-1], tdims[1:]))) * 0.3
    x = rng.normal(size=(1200, 40)).astype(np.float32)
    logt = M.forward(tp, tdims, x.astype(np.float64))[-1][:, 0]
    db = tmp_path / "db.jsonl"
    with open(db, "w") as f:
        for i in range(len(x)):
            f.write(json.dumps({"pipeline": f"p{i % 7}", "W": 64, "H": 64, "group": "nodes=1",
                                "measured_us": float(np.exp(logt[i])), "pred_us": 1.0, "score": 0.0,
                                "terms": [0.0] * 7, "features": [float(v) for v in x[i]]}) + "\n")
    model = str(tmp_path / "m.txt")
    wt.model_train(str(db), model)
    got = wt.Mlp.load(model)
    t32 = np.log(np.array([float(np.exp(v)) for v in logt], np.float64)).astype(np.float32)
    ref = wt.Mlp(DIMS, seed=1)
    ref.train(x, t32, epochs=200, batch=256, lr=1e-3, seed=1)
    np.testing.assert_array_equal(got.params(), ref.params())
    np.testing.assert_array_equal(got.predict(x), ref.predict(x))
    mse = float(np.mean((got.predict(x) - logt) ** 2)) / float(np.var(logt))
    assert mse < 5e-2, f"relative training MSE {mse:.3e}"
