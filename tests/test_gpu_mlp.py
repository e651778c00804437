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
from tests.hostinfo import HOST_THREADS  # noqa: E402


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
    # Element by element: rtol 1e-4, plus an absolute floor of 1e-6 of the
    # largest entry for entries that are sums of terms cancelling each other
    # (an fp32 sum of n terms of size t carries about sqrt(n) 2^-24 t of
    # rounding, far below the floor for these problem sizes).
    err = np.abs(g32 - g64)
    bound = 1e-4 * np.abs(g64) + 1e-6 * np.abs(g64).max()
    worst = int(np.argmax(err / bound))
    assert (err <= bound).all(), (worst, g32[worst], g64[worst])


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
    gs = []
    for t in (1, 2):
        _, gg = omlp.grad(p64, X[idx].astype(np.float64), y[idx].astype(np.float64))
        p64, m64, v64 = omlp.adam_step(p64, m64, v64, gg, t)
        gs.append(gg)
    step = p64 - params
    got = P.cpu().numpy().astype(np.float64) - params
    # The update lr * mhat / (sqrt(vhat) + eps) is determined to fp32
    # precision wherever the gradient is well above eps = 1e-8 at both steps;
    # there it must agree to 1e-3 of lr entry by entry.  Entries whose
    # gradient is within a few eps of zero flip with any rounding of g and
    # are only bounded.  The bound: mhat_t is sum_i a_i g_i and vhat_t is
    # sum_i c_i g_i^2 with a_i = (1 - b1) b1^(t-i) / (1 - b1^t) and
    # c_i = (1 - b2) b2^(t-i) / (1 - b2^t), so by Cauchy-Schwarz
    # |mhat_t| / sqrt(vhat_t) <= sqrt(sum_i a_i^2 / c_i): exactly 1 at t = 1,
    # slightly above 1 at t = 2 when the two gradients differ.
    firm = np.minimum(np.abs(gs[0]), np.abs(gs[1])) > 1e-5
    assert firm.mean() > 0.5
    assert np.abs(got - step)[firm].max() <= 1e-3 * 1e-3

    def ratio_bound(t, b1=0.9, b2=0.999):
        return np.sqrt(sum(((1 - b1) * b1 ** (t - i) / (1 - b1 ** t)) ** 2
                           / ((1 - b2) * b2 ** (t - i) / (1 - b2 ** t))
                           for i in range(1, t + 1)))
    assert ratio_bound(1) == pytest.approx(1.0)
    lim = 1e-3 * (ratio_bound(1) + ratio_bound(2))
    # plus the two fp32 roundings of the stored parameter (half an ulp each)
    ulp = np.spacing((np.abs(params) + np.float32(lim)).astype(np.float32)).astype(np.float64)
    assert (np.abs(got) <= lim * (1 + 1e-6) + ulp).all()
    assert np.allclose(m.cpu().numpy(), m64, rtol=1e-4, atol=1e-7)


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


def test_bf16_inference_of_hand_built_network(B):
    """The hand-built network whose bfloat16 logit is exact (every value a
    short binary fraction): the GPU kernel must give that logit bit for bit,
    and the fp32 kernel the unrounded one."""
    import torch
    from tests import bf16_network
    params, X = bf16_network.network()
    X = np.repeat(X, 300, axis=0)      # several blocks of samples
    zbf = torch.empty(len(X), dtype=torch.float32, device="cuda")
    z32 = torch.empty(len(X), dtype=torch.float32, device="cuda")
    B.bml_mlp_infer_bf16(dev(params), dev(X), len(X), zbf)
    B.bml_mlp_forward(dev(params), dev(X), len(X), z32)
    torch.cuda.synchronize()
    assert (zbf.cpu().numpy() == np.float32(bf16_network.EXPECTED_LOGIT)).all()
    z64, _ = omlp.forward(params.astype(np.float64), X[:1].astype(np.float64))
    assert (z32.cpu().numpy() == np.float32(z64[0])).all()


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


def test_full_early_exit_sweep(B):
    """The whole learned early-exit workload: 9024 lattices of 512 x 512
    (141 densities x 64 seeds), labels from 20000-step runs, the network
    trained on the GPU, held-out seeds 51..63.  The exact stop rule alone is
    exact; the learned exit keeps the held-out label error within 1 % and
    finishes sooner than the exact rule alone.  The full-run labels of 12
    held-out lattices across the transition are checked against the oracle
    run for the full 20000 steps."""
    from paper_1804_07981_amd import early_exit as ee
    ns, rhos, seeds, split = ee.c4_lattices()
    rep = ee.experiment(ns, rhos, seeds, split, plain_sample=2, log=say, return_labels=True)
    summary = {k: v for k, v in rep.items() if k not in ("labels", "labels_mlp_test",
                                                          "test_index")}
    say(summary)
    assert rep["n_lattices"] == 9024 and rep["n_test"] == 1833
    assert rep["batch_full"]["label_error"] == 0.0
    assert rep["batch_exact_stop"]["label_error"] == 0.0
    ml = rep["batch_exact_stop_mlp"]
    assert ml["mlp_exits"] > 0
    assert ml["label_error"] <= 0.01
    assert rep["gain_vs_exact_stop"] > 1.0
    assert rep["work_saved_vs_exact_stop"] > 0.0
    # oracle labels of held-out lattices around the transition
    te = np.asarray(rep["test_index"])
    mid = [i for i in te if 0.30 <= rhos[i] <= 0.42]
    pick = [mid[j] for j in np.linspace(0, len(mid) - 1, 12).astype(int)]
    say(f"oracle: {len(pick)} lattices of 512^2, 20000 steps, {HOST_THREADS} threads")
    outs, stats = oracle.run_many([oracle.init_cells(ns[i], seeds[i], rhos[i]) for i in pick],
                                  20000, n_threads=HOST_THREADS)
    for i, st in zip(pick, stats):
        cars = int(st[0, 0] + st[0, 2])
        want = omlp.jam_label(st[:, 1], st[:, 3], cars, last=1000, threshold=0.05)
        assert rep["labels"][i] == want, (i, rhos[i], seeds[i])
