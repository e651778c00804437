"""GPU checks of the learned early exit's kernels (through the C ABI)
against the fp64 oracle: features from batch traces (bit-exact), trace
reductions, feature statistics, fp32 gradients, one Adam step, fp32 and
BF16 inference; and a reduced early-exit sweep showing what the trained
network saves over the exact stop rule alone."""
import os
import sys

import numpy as np
import pytest

import oracle
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu
HOST_THREADS = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1804_07981_amd as pkg
    pkg.lib()
    return pkg


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def dev(x, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x))
    return (t if dtype is None else t.to(dtype)).cuda()


def test_features_and_trace_reductions_match_oracle(B):
    import torch
    ns = [64, 96, 128, 256, 64]
    rhos = [0.25, 0.33, 0.4, 0.3, 0.9]
    seeds = [3, 4, 5, 6, 7]
    steps = 600
    outs, stats = oracle.run_many([oracle.init_cells(n, s, r) for n, r, s in zip(ns, rhos, seeds)],
                                  steps, n_threads=HOST_THREADS)
    with B.Batch(ns, rhos, seeds, trace_steps=steps) as bt:
        bt.run(steps)
        bt.synchronize()
        cars = np.array([sum(bt.initial_counts(b)) for b in range(len(ns))], dtype=np.int64)
        X = torch.empty((len(ns), 65), dtype=torch.float32, device="cuda")
        B.bml_features(bt.trace_tensor(), steps, len(ns), dev(cars), dev(np.array(rhos)), 8, X,
                       bt.stream)
        fr = torch.zeros(len(ns), dtype=torch.uint8, device="cuda")
        B.bml_trace_frozen(bt.trace_tensor(), steps, len(ns), 100, 600, fr, bt.stream)
        mv = torch.empty(len(ns), dtype=torch.float64, device="cuda")
        B.bml_trace_mobility(bt.trace_tensor(), steps, len(ns), dev(cars), 400, 600, mv,
                             bt.stream)
        bt.synchronize()
        X = X.cpu().numpy()
        fr = fr.cpu().numpy()
        mv = mv.cpu().numpy()
    for b in range(len(ns)):
        st = stats[b]
        c = int(st[0, 0] + st[0, 2])
        assert c == cars[b]
        want = omlp.features(st[:, 1], st[:, 3], c, rhos[b])
        assert np.array_equal(X[b], want), b
        zero = ((st[100:600, 1] + st[100:600, 3]) == 0).any()
        assert fr[b] == int(zero)
        v = omlp.mobile_fraction(st[400:600, 1], st[400:600, 3], c).mean()
        assert abs(mv[b] - v) <= 1e-12 * max(1.0, v)


def test_feature_stats_and_standardize(B):
    import torch
    rng = np.random.default_rng(2)
    X = rng.normal(3, 2, (1000, 65)).astype(np.float32)
    X[:, 7] = 0.5   # constant column
    Xd = dev(X)
    mean = torch.empty(65, dtype=torch.float32, device="cuda")
    std = torch.empty_like(mean)
    B.bml_feature_stats(Xd, 1000, mean, std)
    B.bml_standardize(Xd, 1000, mean, std)
    torch.cuda.synchronize()
    m = X.astype(np.float64).mean(0)
    s = X.astype(np.float64).std(0)
    assert np.allclose(mean.cpu().numpy(), m, rtol=1e-6, atol=1e-6)
    s[7] = 1.0
    assert np.allclose(std.cpu().numpy(), s, rtol=1e-5)
    want = ((X - m.astype(np.float32)) / s.astype(np.float32))
    assert np.allclose(Xd.cpu().numpy(), want, rtol=1e-5, atol=1e-5)


@pytest.mark.parametrize("n", [1, 37, 256])
def test_gradient_matches_fp64_oracle(B, n):
    import torch
    rng = np.random.default_rng(n)
    params = (rng.normal(0, 0.2, omlp.NP)).astype(np.float32)
    X = rng.normal(0, 1, (n, 65)).astype(np.float32)
    y = (rng.random(n) < 0.4).astype(np.float32)
    scratch = torch.empty(B.bml_mlp_scratch_bytes(), dtype=torch.uint8, device="cuda")
    g = torch.empty(omlp.NP, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    B.bml_mlp_grad(dev(params), dev(X), dev(y), n, scratch, g, loss)
    torch.cuda.synchronize()
    l64, g64 = omlp.grad(params.astype(np.float64), X.astype(np.float64), y.astype(np.float64))
    g32 = g.cpu().numpy().astype(np.float64)
    assert abs(loss.item() - l64) <= 1e-5 * max(1.0, abs(l64))
    assert np.linalg.norm(g32 - g64) <= 1e-4 * np.linalg.norm(g64)
    # entry-wise, for entries that are not tiny
    big = np.abs(g64) > 1e-3 * np.abs(g64).max()
    assert np.allclose(g32[big], g64[big], rtol=1e-3)


def test_adam_step_matches_oracle(B):
    import torch
    rng = np.random.default_rng(9)
    n = 128
    params = rng.normal(0, 0.2, omlp.NP).astype(np.float32)
    X = rng.normal(0, 1, (n, 65)).astype(np.float32)
    y = (rng.random(n) < 0.5).astype(np.float32)
    idx = rng.permutation(n).astype(np.int32)
    P = dev(params)
    m = torch.zeros_like(P)
    v = torch.zeros_like(P)
    g = torch.zeros_like(P)
    scratch = torch.empty(B.bml_mlp_scratch_bytes(), dtype=torch.uint8, device="cuda")
    loss = torch.empty(2, dtype=torch.float32, device="cuda")
    for t in (1, 2):
        B.bml_mlp_train_step(P, m, v, g, t, dev(X), dev(y), dev(idx), n, 1e-3, 0.9, 0.999, 1e-8,
                             scratch, loss.data_ptr() + 4 * (t - 1))
    torch.cuda.synchronize()
    p64 = params.astype(np.float64)
    m64 = np.zeros(omlp.NP)
    v64 = np.zeros(omlp.NP)
    for t in (1, 2):
        _, gg = omlp.grad(p64, X[idx].astype(np.float64), y[idx].astype(np.float64))
        p64, m64, v64 = omlp.adam_step(p64, m64, v64, gg, t)
    step = p64 - params
    got = P.cpu().numpy().astype(np.float64) - params
    # steps are ~1e-3 in size; allow for fp32 gradients of near-zero entries
    assert np.linalg.norm(got - step) <= 2e-2 * np.linalg.norm(step)
    assert np.allclose(m.cpu().numpy(), m64, rtol=1e-3, atol=1e-7)


def test_inference_fp32_and_bf16_match_oracle(B):
    import torch
    rng = np.random.default_rng(4)
    n = 3000
    params = (rng.normal(0, 0.25, omlp.NP)).astype(np.float32)
    X = rng.normal(0, 1, (n, 65)).astype(np.float32)
    z32 = torch.empty(n, dtype=torch.float32, device="cuda")
    zbf = torch.empty(n, dtype=torch.float32, device="cuda")
    B.bml_mlp_forward(dev(params), dev(X), n, z32)
    B.bml_mlp_infer_bf16(dev(params), dev(X), n, zbf)
    torch.cuda.synchronize()
    z64, _ = omlp.forward(params.astype(np.float64), X.astype(np.float64))
    assert np.allclose(z32.cpu().numpy(), z64, rtol=1e-4, atol=1e-4)
    ze = omlp.infer_bf16(params, X)
    zb = zbf.cpu().numpy()
    # Same roundings, different fp32 summation order: a bfloat16 rounding of
    # a hidden value can land one ulp (2^-8 relative) apart.
    assert np.all(np.abs(zb - ze) <= 1e-2 * (1.0 + np.abs(ze)))
    # exit decisions (p > 0.99 / p < 0.01) agree away from the thresholds
    t = np.log(99.0)
    far = np.minimum(np.abs(np.abs(ze) - t), 9) > 0.05
    assert np.array_equal((zb > t)[far], (ze > t)[far])
    assert np.array_equal((zb < -t)[far], (ze < -t)[far])


def test_early_exit_saves_work(B):
    """Reduced sweep (128 x 128, rho 0.20..0.55, 8 seeds each, 3000 steps):
    train on 6 seeds, exit at step 512 when confident.  Lattices that do not
    exit keep their exact labels; the exits cut the simulated cell-steps
    below the exact-stop-rule sweep, with a small label error."""
    from paper_1804_07981_amd import early_exit as ee
    rhos = [0.20 + 0.01 * k for k in range(36)]
    rows = [(128, r, 1000 * k + s, "test" if s >= 6 else "train")
            for k, r in enumerate(rhos) for s in range(8)]
    ns, rh, sd, split = (list(x) for x in zip(*rows))
    rep = ee.experiment(ns, rh, sd, split, full_steps=3000, epochs=150, plain_sample=4,
                        log=say)
    say(rep)
    ex = rep["batch_exact_stop"]
    ml = rep["batch_exact_stop_mlp"]
    assert ex["label_error"] == 0.0                  # the exact rule is exact
    assert rep["batch_full"]["label_error"] == 0.0
    assert ml["mlp_exits"] > 0
    assert ml["cell_steps"] < ex["cell_steps"]
    assert ml["label_error"] <= 0.05
