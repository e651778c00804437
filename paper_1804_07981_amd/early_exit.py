"""Learned early exit for BML density sweeps, on the GPU.

Physics (Marzolla, arXiv:1804.07981, Sec. 2): a BML lattice settles into
free flow below a critical density and into a global jam above it; near the
critical density either can happen.  A density sweep needs the final phase
of every lattice, normally from a full-length run.  Here:

* every lattice of the sweep runs in one batch (bml_batch_*), chunk by chunk
  through a captured hipGraph;
* exact stop rule: a step in which no car moves leaves the lattice unchanged,
  so from then on it is frozen -- jammed -- and it stops (no learning, no
  error);
* learned exit: after `exit_step` steps a small MLP (bml_mlp_*, trained on
  the GPU by this module) reads the mobile-fraction trajectory and the
  density; lattices it is confident about (p > hi or p < lo) stop with its
  prediction, the rest run to full length as the fallback.

A lattice's label is "jammed" when its mean mobile fraction over the last
`label_window` steps of a full-length run is below `jam_threshold`.

Host code here only orchestrates: every per-cell, per-step and per-sample
computation runs in libbml's kernels.
"""
from __future__ import annotations

import argparse
import json
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib as L
from .batch import Batch
from .lattice import Lattice

WINDOW = 8                 # steps per feature window (64 windows = 512 steps)


def he_uniform_params(seed: int = 0x4D4C50) -> np.ndarray:
    """He-uniform weights (U(-a, a), a = sqrt(6 / fan_in)), zero biases."""
    rng = np.random.default_rng(seed)
    ni, nh = L.BML_MLP_INPUTS, L.BML_MLP_HIDDEN
    parts = [rng.uniform(-1, 1, nh * ni) * np.sqrt(6.0 / ni), np.zeros(nh),
             rng.uniform(-1, 1, nh * nh) * np.sqrt(6.0 / nh), np.zeros(nh),
             rng.uniform(-1, 1, nh) * np.sqrt(6.0 / nh), np.zeros(1)]
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == L.BML_MLP_PARAMS
    return p


class MLP:
    """The 65 -> 64 -> 64 -> 1 classifier; parameters live on the GPU."""

    def __init__(self, device="cuda", seed: int = 0x4D4C50, params: np.ndarray | None = None,
                 stream: torch.cuda.Stream | None = None):
        self.device = torch.device(device)
        self.stream = stream or torch.cuda.current_stream(self.device)
        p = he_uniform_params(seed) if params is None else np.asarray(params, np.float32)
        self.params = torch.from_numpy(p.copy()).to(self.device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.scratch = torch.empty(L.bml_mlp_scratch_bytes(), dtype=torch.uint8,
                                   device=self.device)
        self.t = 0
        self.mean = None
        self.std = None

    def fit_standardizer(self, X: torch.Tensor) -> None:
        self.mean = torch.empty(L.BML_MLP_INPUTS, dtype=torch.float32, device=self.device)
        self.std = torch.empty_like(self.mean)
        L.bml_feature_stats(X, X.shape[0], self.mean, self.std, self.stream)

    def standardize(self, X: torch.Tensor) -> torch.Tensor:
        out = X.clone()
        L.bml_standardize(out, out.shape[0], self.mean, self.std, self.stream)
        return out

    def train(self, X: torch.Tensor, y: torch.Tensor, epochs: int = 200, batch: int = 256,
              lr: float = 1e-3, seed: int = 1, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8) -> np.ndarray:
        """Adam on minibatches of standardized features X (n x 65, float32)
        and labels y (n, float32: 1 = jammed).  Returns the per-epoch mean
        training loss."""
        n = X.shape[0]
        rng = np.random.default_rng(seed)
        steps = -(-n // batch)
        losses = torch.zeros(epochs * steps, dtype=torch.float32, device=self.device)
        for e in range(epochs):
            idx = torch.from_numpy(rng.permutation(n).astype(np.int32)).to(self.device)
            for s in range(steps):
                b = min(batch, n - s * batch)
                self.t += 1
                L.bml_mlp_train_step(self.params, self.m, self.v, self.grad, self.t, X, y,
                                     idx.data_ptr() + 4 * s * batch, b, lr, beta1, beta2, eps,
                                     self.scratch,
                                     losses.data_ptr() + 4 * (e * steps + s), self.stream)
        self.stream.synchronize()
        return losses.view(epochs, steps).mean(dim=1).cpu().numpy()

    def logits(self, X: torch.Tensor, bf16: bool = True) -> torch.Tensor:
        out = torch.empty(X.shape[0], dtype=torch.float32, device=self.device)
        f = L.bml_mlp_infer_bf16 if bf16 else L.bml_mlp_forward
        f(self.params, X, X.shape[0], out, self.stream)
        return out


@dataclass
class SweepResult:
    labels: np.ndarray                 # 1 jammed, 0 free (decided or measured)
    how: np.ndarray                    # 0 full run, 1 frozen (exact), 2 MLP exit
    steps: np.ndarray                  # steps each lattice ran
    wall_s: float
    cell_steps: float
    extra: dict = field(default_factory=dict)


def batch_features(bt: Batch, rhos, stream) -> torch.Tensor:
    """Raw features (count x 65) from the first 512 steps of the trace."""
    dev = bt.device
    cars = torch.tensor([sum(bt.initial_counts(b)) for b in range(bt.count)],
                        dtype=torch.int64, device=dev)
    rho = torch.tensor(np.asarray(rhos, dtype=np.float64), device=dev)
    X = torch.empty((bt.count, L.BML_MLP_INPUTS), dtype=torch.float32, device=dev)
    L.bml_features(bt.trace_tensor(), bt.trace_steps, bt.count, cars, rho, WINDOW, X, stream)
    return X


def run_sweep(ns, rhos, seeds, full_steps: int = 20000, chunk: int = 512,
              stop_frozen: bool = True, mlp: MLP | None = None, exit_step: int = 512,
              lo: float = 0.01, hi: float = 0.99, label_window: int = 1000,
              jam_threshold: float = 0.05, device="cuda", keep_features: bool = False,
              tuning=(0, 0, 0)) -> SweepResult:
    """Batched sweep with the exact stop rule and (optionally) the learned
    exit.  Wall time covers everything from the batch's first step to the
    last label."""
    count = len(ns)
    if mlp is not None and (exit_step <= 0 or exit_step % chunk or exit_step > full_steps):
        raise ValueError(f"exit_step={exit_step} must be a positive multiple of the "
                         f"chunk ({chunk}) within the run ({full_steps} steps)")
    stream = torch.cuda.Stream(torch.device(device))
    bt = Batch(ns, rhos, seeds, layout=L.BML_LAYOUT_BITPLANE, trace_steps=full_steps,
               device=device, stream=stream)
    bt.set_tuning(*tuning)
    dev = bt.device
    cars = torch.tensor([sum(bt.initial_counts(b)) for b in range(count)],
                        dtype=torch.int64, device=dev)
    labels = np.full(count, -1, dtype=np.int64)
    how = np.zeros(count, dtype=np.int64)
    steps = np.zeros(count, dtype=np.int64)
    active = np.ones(count, dtype=np.uint8)
    frozen_d = torch.zeros(count, dtype=torch.uint8, device=dev)
    features = None
    n_cells = np.asarray(ns, dtype=np.float64) ** 2
    cell_steps = 0.0
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    bt.capture(chunk)
    done = 0
    while done < full_steps and active.any():
        k = min(chunk, full_steps - done)
        if k == chunk:
            bt.replay()
        else:
            bt.run(k)
        cell_steps += float(n_cells[active == 1].sum()) * k
        steps[active == 1] += k
        prev, done = done, done + k
        changed = False
        # The exact rule first: a lattice that froze in this chunk is jammed
        # whatever the network would say about it.
        if stop_frozen:
            L.bml_trace_frozen(bt.trace_tensor(), bt.trace_steps, count, prev, done, frozen_d,
                               stream)
            fr = _sync_copy(frozen_d, stream)
            for b in np.nonzero(active & (fr == 1))[0]:
                labels[b] = 1
                how[b] = 1
                active[b] = 0
                changed = True
        if mlp is not None and done == exit_step:
            X = batch_features(bt, rhos, stream)
            stream.synchronize()   # the MLP works on its own stream
            if keep_features:
                features = X.clone()
            Xs = mlp.standardize(X)
            p = _sigmoid(_sync_copy(mlp.logits(Xs), stream))
            for b in np.nonzero(active)[0]:
                if p[b] > hi or p[b] < lo:
                    labels[b] = int(p[b] > hi)
                    how[b] = 2
                    active[b] = 0
                    changed = True
        if changed and active.any():
            bt.set_active(active)
    if keep_features and features is None:
        features = batch_features(bt, rhos, stream)
    rest = np.nonzero(labels < 0)[0]
    if len(rest):
        mean = torch.empty(count, dtype=torch.float64, device=dev)
        L.bml_trace_mobility(bt.trace_tensor(), bt.trace_steps, count, cars,
                             full_steps - label_window, full_steps, mean, stream)
        mv = _sync_copy(mean, stream)
        labels[rest] = (mv[rest] < jam_threshold).astype(np.int64)
    stream.synchronize()
    wall = time.perf_counter() - t0
    bt.check()
    res = SweepResult(labels, how, steps, wall, cell_steps)
    if keep_features:
        res.extra["features"] = features
    bt.close()
    return res


def _sync_copy(t: torch.Tensor, stream) -> np.ndarray:
    stream.synchronize()
    return t.cpu().numpy()


def _sigmoid(z: np.ndarray) -> np.ndarray:
    """Jam probability from logits, for the host's exit decision."""
    z = np.asarray(z, dtype=np.float64)
    return np.where(z >= 0, 1.0 / (1.0 + np.exp(-np.abs(z))),
                    np.exp(-np.abs(z)) / (1.0 + np.exp(-np.abs(z))))


def _rows(X: torch.Tensor, idx: np.ndarray) -> torch.Tensor:
    """Rows idx of a device matrix, selected on the host."""
    return torch.from_numpy(np.ascontiguousarray(X.cpu().numpy()[idx])).to(X.device)


def plain_runs(ns, rhos, seeds, full_steps: int = 20000, label_window: int = 1000,
               jam_threshold: float = 0.05, device="cuda", layout=L.BML_LAYOUT_BITPLANE):
    """The baseline: every lattice run alone (single-lattice API), full
    length, one after the other.  Returns (labels, wall seconds)."""
    labels = np.zeros(len(ns), dtype=np.int64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for b, (n, r, s) in enumerate(zip(ns, rhos, seeds)):
        with Lattice(n, r, s, layout=layout, stats_cap=label_window, device=device) as lat:
            lat.step(full_steps)
            st = lat.stats(full_steps - label_window, label_window)
            cars = int(st["n_lr"][0]) + int(st["n_tb"][0])
            moved = st["moved_lr"].astype(np.float64) + st["moved_tb"]
            v = moved / cars if cars else np.ones(label_window)
            labels[b] = int(v.mean() < jam_threshold)
    torch.cuda.synchronize()
    return labels, time.perf_counter() - t0


def experiment(ns, rhos, seeds, split, full_steps=20000, exit_step=512, epochs=300,
               plain_sample: int | None = None, device="cuda", log=print,
               return_labels: bool = False) -> dict:
    """Full early-exit experiment: labels for every lattice (exact stop rule,
    full length otherwise), train on split == 'train', evaluate on 'test',
    then time on the test lattices (1) plain per-lattice full runs, (2) the
    batch with the exact stop rule, (3) (2) plus the learned exit.  With
    return_labels the report also holds every lattice's full-run label
    ("labels") and the test-set labels of run (3) ("labels_mlp_test")."""
    split = np.asarray(split)
    log(f"labelling {len(ns)} lattices ({full_steps} steps, exact stop rule)")
    lab = run_sweep(ns, rhos, seeds, full_steps, stop_frozen=True, keep_features=True,
                    device=device)
    y = lab.labels.astype(np.float32)
    X = lab.extra["features"]
    tr = np.nonzero(split == "train")[0]
    te = np.nonzero(split == "test")[0]
    va = np.nonzero(split == "val")[0]
    mlp = MLP(device)
    mlp.fit_standardizer(_rows(X, tr))
    Xs = mlp.standardize(X)
    t0 = time.perf_counter()
    losses = mlp.train(_rows(Xs, tr), torch.from_numpy(y[tr]).to(X.device), epochs=epochs)
    train_s = time.perf_counter() - t0
    p = _sigmoid(_sync_copy(mlp.logits(Xs), mlp.stream))
    def split_err(idx):
        dec = (p[idx] > 0.5).astype(int)
        return float((dec != lab.labels[idx]).mean()) if len(idx) else float("nan")
    log(f"trained {epochs} epochs in {train_s:.2f} s; loss {losses[0]:.4f} -> {losses[-1]:.4f}")
    ns_t = [ns[i] for i in te]
    rh_t = [rhos[i] for i in te]
    sd_t = [seeds[i] for i in te]
    full_t = lab.labels[te]
    out = {"n_lattices": len(ns), "n_test": len(te), "full_steps": full_steps,
           "exit_step": exit_step, "jammed_fraction": float(lab.labels.mean()),
           "label_wall_s": lab.wall_s, "train_s": train_s, "epochs": epochs,
           "loss_first": float(losses[0]), "loss_last": float(losses[-1]),
           "argmax_error": {"train": split_err(tr), "val": split_err(va), "test": split_err(te)}}
    # (2) batch + exact stop rule; (3) + learned exit.
    log("timing: batch + exact stop rule")
    r2 = run_sweep(ns_t, rh_t, sd_t, full_steps, stop_frozen=True, device=device)
    log("timing: batch + exact stop rule + learned exit")
    r3 = run_sweep(ns_t, rh_t, sd_t, full_steps, stop_frozen=True, mlp=mlp,
                   exit_step=exit_step, device=device)
    log("timing: batch, full length, no stop rule")
    r1b = run_sweep(ns_t, rh_t, sd_t, full_steps, stop_frozen=False, device=device)
    out["batch_full"] = {"wall_s": r1b.wall_s, "cell_steps": r1b.cell_steps,
                         "label_error": float((r1b.labels != full_t).mean())}
    out["batch_exact_stop"] = {"wall_s": r2.wall_s, "cell_steps": r2.cell_steps,
                               "label_error": float((r2.labels != full_t).mean()),
                               "frozen_stops": int((r2.how == 1).sum())}
    out["batch_exact_stop_mlp"] = {"wall_s": r3.wall_s, "cell_steps": r3.cell_steps,
                                   "label_error": float((r3.labels != full_t).mean()),
                                   "mlp_exits": int((r3.how == 2).sum()),
                                   "frozen_stops": int((r3.how == 1).sum())}
    # (1) plain per-lattice full runs (on a stated sample if requested).
    idx = np.arange(len(te)) if plain_sample is None else np.linspace(
        0, len(te) - 1, plain_sample).astype(int)
    log(f"timing: plain per-lattice full runs ({len(idx)} lattices)")
    pl, pw = plain_runs([ns_t[i] for i in idx], [rh_t[i] for i in idx], [sd_t[i] for i in idx],
                        full_steps, device=device)
    scale = len(te) / len(idx)
    out["plain_per_lattice"] = {"wall_s": pw * scale, "measured_lattices": int(len(idx)),
                                "measured_wall_s": pw,
                                "label_error": float((pl != full_t[idx]).mean())}
    out["gain_vs_plain"] = out["plain_per_lattice"]["wall_s"] / r3.wall_s
    if return_labels:
        out["labels"] = lab.labels.tolist()
        out["labels_mlp_test"] = r3.labels.tolist()
        out["test_index"] = te.tolist()
    out["gain_vs_exact_stop"] = r2.wall_s / r3.wall_s
    out["work_saved_vs_exact_stop"] = 1.0 - r3.cell_steps / r2.cell_steps
    return out


def c4_lattices():
    """The early-exit workload: 512 x 512, rho_k = (80 + k) / 400, k = 0..140,
    64 seeds each (seed = 64 k + s); split by seed index."""
    import workloads
    rows = workloads.early_exit_lattices()
    ns = [lt.n for lt, _, _ in rows]
    rhos = [lt.rho for lt, _, _ in rows]
    seeds = [lt.seed for lt, _, _ in rows]
    split = [workloads.split_of(s) for _, _, s in rows]
    return ns, rhos, seeds, split


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description="learned early-exit density sweep")
    ap.add_argument("--out", default=None, help="write the JSON report here")
    ap.add_argument("--full-steps", type=int, default=20000)
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--plain-sample", type=int, default=None,
                    help="time plain per-lattice runs on this many test lattices and scale")
    ap.add_argument("--subsample", type=int, default=1,
                    help="keep every k-th density of the workload")
    args = ap.parse_args(argv)
    ns, rhos, seeds, split = c4_lattices()
    if args.subsample > 1:
        keep = [i for i in range(len(ns)) if (i // 64) % args.subsample == 0]
        ns, rhos, seeds, split = ([x[i] for i in keep] for x in (ns, rhos, seeds, split))
    rep = experiment(ns, rhos, seeds, split, full_steps=args.full_steps, epochs=args.epochs,
                     plain_sample=args.plain_sample,
                     log=lambda m: print(m, flush=True))
    print(json.dumps(rep), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(rep, f, indent=1)
    return 0


if __name__ == "__main__":
    import sys
    sys.exit(main())
