"""Pins of the fp64 MLP oracle (no GPU): central finite differences, closed
forms of BCE, ReLU layers and Adam's first step, bfloat16 rounding of known
values, and features/labels of hand-made trajectories and oracle runs."""
import numpy as np
import pytest

import oracle
from oracle import mlp


def random_problem(seed, n=12):
    rng = np.random.default_rng(seed)
    params = rng.normal(0, 0.3, mlp.NP)
    X = rng.normal(0, 1, (n, mlp.NI))
    y = (rng.random(n) < 0.5).astype(np.float64)
    return params, X, y


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_backward_matches_finite_differences(seed):
    params, X, y = random_problem(seed)
    _, g = mlp.grad(params, X, y)
    rng = np.random.default_rng(100 + seed)
    # every block of the parameter vector, plus random entries
    idx = [0, 64 * 65 - 1, 64 * 65, 64 * 65 + 63, 4224, 4224 + 4095, 8320, 8383, 8384,
           8447, 8448] + list(rng.integers(0, mlp.NP, 40))
    fd = mlp.finite_difference(params, X, y, idx)
    # ReLU kinks are measure-zero for Gaussian inputs; compare in relative terms
    assert np.allclose(g[idx], fd, rtol=1e-6, atol=1e-9)


def test_bce_closed_forms():
    assert np.isclose(mlp.bce_with_logits(np.array([0.0]), np.array([1.0]))[0], np.log(2))
    z = np.array([-30.0, -2.0, 0.5, 40.0])
    for yv in (0.0, 1.0):
        y = np.full(4, yv)
        p = 1 / (1 + np.exp(-z))
        direct = -(y * np.log(p) + (1 - y) * np.log(1 - p + 1e-300))
        assert np.allclose(mlp.bce_with_logits(z, y)[:3], direct[:3], rtol=1e-12)
    assert np.allclose(mlp.sigmoid(np.array([-800.0, 0.0, 800.0])), [0.0, 0.5, 1.0])


def test_forward_of_a_hand_built_network():
    """W1 copies inputs 0..63 (plus bias), W2 = identity, W3 picks unit 3:
    the logit is max(x_3 + b1_3, 0) + b3."""
    p = {"W1": np.zeros((64, 65)), "b1": np.zeros(64), "W2": np.eye(64), "b2": np.zeros(64),
         "W3": np.zeros(64), "b3": np.array([0.25])}
    p["W1"][:, :64] = np.eye(64)
    p["b1"][3] = -0.5
    p["W3"][3] = 2.0
    params = mlp.pack(p)
    X = np.zeros((3, 65))
    X[:, 3] = [0.1, 0.5, 2.0]
    z, _ = mlp.forward(params, X)
    assert np.allclose(z, [0.25, 0.25, 2.0 * 1.5 + 0.25])


def test_adam_first_step_closed_form():
    """From m = v = 0 the first bias-corrected step is lr * g / (|g| + eps)."""
    g = np.array([0.3, -2e-3, 0.0, 5.0])
    p, m, v = mlp.adam_step(np.zeros(4), np.zeros(4), np.zeros(4), g, 1, lr=1e-3)
    assert np.allclose(-p, 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)


def test_bf16_rounding_known_values():
    # bfloat16 keeps 8 significant bits: 1 + 2^-7 is the successor of 1.
    vals = np.array([1.0, 1 + 2**-8, 1 + 3 * 2**-9, 1 + 2**-7 + 2**-8, 3.140625, -2.5,
                     65504.0, 1e-40], dtype=np.float32)
    want = np.array([1.0, 1.0, 1 + 2**-7, 1 + 2 * 2**-7, 3.140625, -2.5, 65536.0, 0.0],
                    dtype=np.float32)
    got = mlp.to_bf16(vals)
    # 1e-40 is subnormal: its top 16 bits give 9.18e-41 (kept), not zero
    assert np.array_equal(got[:7], want[:7])
    assert abs(got[7]) < 1e-39
    assert np.isinf(mlp.to_bf16(np.array([np.inf], np.float32))[0])


def test_bf16_inference_close_to_fp64():
    params, X, _ = random_problem(5, n=200)
    z64, _ = mlp.forward(params, X)
    zb = mlp.infer_bf16(params, X)
    # 8-bit significands through three layers: a few percent of the scale
    assert np.max(np.abs(zb - z64)) < 0.05 * (1 + np.max(np.abs(z64)))


def test_features_of_hand_made_trajectory():
    steps = 512
    mlr = np.zeros(steps, dtype=np.int64)
    mtb = np.zeros(steps, dtype=np.int64)
    mlr[:8] = 10          # window 0: 80 moves of 100 cars over 8 steps -> 0.1
    mtb[8:16] = 25        # window 1: 200 / 800 -> 0.25
    mlr[-8:] = 100        # last window: everyone moves -> 1.0
    f = mlp.features(mlr, mtb, 100, 0.3125)
    assert f.dtype == np.float32 and f.shape == (65,)
    assert f[0] == np.float32(0.1) and f[1] == np.float32(0.25) and f[63] == 1.0
    assert (f[2:63] == 0).all() and f[64] == np.float32(0.3125)
    assert (mlp.features(mlr, mtb, 0, 0.0)[:64] == 1.0).all()


def test_labels_from_oracle_runs():
    """A frozen lattice is jammed; a lone car always moves (free flow)."""
    g = oracle.init_cells(32, 1, 0.9)
    _, st = oracle.run(g, 300)
    cars = int(st[0, 0] + st[0, 2])
    assert mlp.jam_label(st[:, 1], st[:, 3], cars, last=100) == 1
    lone = np.zeros((32, 32), np.uint8)
    lone[4, 4] = 1
    _, st = oracle.run(lone, 300)
    assert mlp.jam_label(st[:, 1], st[:, 3], 1, last=100) == 0


# --- bfloat16 inference pinned by a hand-built network ------------------------

from tests import bf16_network  # noqa: E402

BF16_SITES = [
    ("input not rounded", "    x = to_bf16(f32(X))", "    x = f32(X)"),
    ("W1 not rounded", '    W1 = to_bf16(f32(p["W1"]))', '    W1 = f32(p["W1"])'),
    ("W2 not rounded", '    W2 = to_bf16(f32(p["W2"]))', '    W2 = f32(p["W2"])'),
    ("W3 not rounded", '    W3 = to_bf16(f32(p["W3"]))', '    W3 = f32(p["W3"])'),
    ("h1 not rounded", "    h1 = to_bf16(np.maximum(x @ W1.T + b1, np.float32(0)))",
     "    h1 = np.maximum(x @ W1.T + b1, np.float32(0))"),
    ("h2 not rounded", "    h2 = to_bf16(np.maximum(h1 @ W2.T + b2, np.float32(0)))",
     "    h2 = np.maximum(h1 @ W2.T + b2, np.float32(0))"),
    ("b1 rounded", '    b1 = f32(p["b1"])', '    b1 = to_bf16(f32(p["b1"]))'),
    ("b2 rounded", '    b2 = f32(p["b2"])', '    b2 = to_bf16(f32(p["b2"]))'),
    ("b3 rounded", '    b3 = f32(p["b3"])', '    b3 = to_bf16(f32(p["b3"]))'),
    ("rounding by truncation", "(u + 0x7fff + ((u >> 16) & 1)) & 0xffff0000",
     "u & 0xffff0000"),
]


def _bf16_logit(infer):
    params, X = bf16_network.network()
    return infer(params, X)


def test_bf16_inference_of_hand_built_network():
    """Every rounding site and every unrounded bias shows in the logit."""
    z = _bf16_logit(mlp.infer_bf16)
    assert z.dtype == np.float32 and z.shape == (1,)
    assert z[0] == np.float32(bf16_network.EXPECTED_LOGIT)
    # the same network in fp64 (no rounding at all) gives another value
    params, X = bf16_network.network()
    z64, _ = mlp.forward(params.astype(np.float64), X.astype(np.float64))
    assert z64[0] != bf16_network.EXPECTED_LOGIT


@pytest.mark.parametrize("name,before,after", BF16_SITES, ids=[s[0] for s in BF16_SITES])
def test_bf16_pin_catches_planted_mistake(name, before, after):
    """A copy of oracle/mlp.py with one rounding site dropped (or a bias
    rounded) gives another logit for the hand-built network."""
    import types
    src = open(mlp.__file__).read()
    assert before in src, "mutation site not found"
    mod = types.ModuleType("mlp_mutant")
    exec(compile(src.replace(before, after, 1), "mlp_mutant", "exec"), mod.__dict__)
    z = _bf16_logit(mod.infer_bf16)
    assert z[0] != np.float32(bf16_network.EXPECTED_LOGIT), name
