"""Training of the learned planner.

Corpus: plain-pipeline runs over random synthetic instances (sizes, key
distributions, match rates, selectivities, group counts and correlated
columns all varied). Each run's label is what the plain pipeline reports
(join output rows, groups); each run's input is the GPU sketch. Training runs
on the GPU through librel's own MLP kernels (forward, backward, Adam).

Input and targets are scale-free (the same transform the library's planner
applies before its forward pass, see relative_inputs): size-dependent features
are taken relative to r, the log2 HyperLogLog estimate of the group key, and
the targets are y = (log2(1 + join rows) - log2(1 + N), log2(1 + groups) - r).
Runs of up to 2^17 fact rows then train a model that sizes tables for inputs
hundreds of times larger. Loss: mean squared error. The planner's safety
margin is the 95th percentile of the validation under-prediction of the group
target; a planned group table has twice the expected slots, so a prediction
must be short by about that factor again before the run overflows and falls
back to the plain pipeline.

Usage: python -m paper_2608_13696_amd.planner_train --runs 200000 --out <file.npz>
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import datagen  # noqa: E402

MODEL = os.path.join(os.path.dirname(os.path.abspath(__file__)), "model", "planner_mlp.npz")
N_PARAMS = 6914
SAMPLE_K = 256


def log(msg):
    print(f"[train] {msg}", file=sys.stderr, flush=True)


def run_spec(i: int, seed: int, n_hi: int) -> dict:
    """Parameters of training run i (all from the seeded unit stream)."""
    u = datagen.unit(10, (seed << 24) + i, datagen.S_INST)
    n = int(round(math.exp(math.log(1e3) + u[0] * (math.log(n_hi) - math.log(1e3)))))
    m = max(16, int(round(n / 4 * math.exp(math.log(0.25) + u[1] * (math.log(4.0) - math.log(0.25))))))
    match = 0.05 + 0.95 * u[2]
    zipf = 1.5 * u[3] if u[4] < 0.7 else 0.0
    sel = 0.02 + 0.96 * u[5]
    groups = max(1, int(round(math.exp(u[6] * math.log(m)))))
    corr = int(u[7] * 3)  # 0 none, 1 day follows fk, 2 grp follows pk
    group_by = "dim_grp" if u[8] < 0.8 else "fk"
    return dict(n=n, m=m, domain=max(1, int(round(m / match))), zipf=zipf, day_lt=int(round(sel * datagen.DAY_DOMAIN)),
                groups=groups, corr=corr, group_by=group_by, seed=(seed << 24) + i)


def make_run(s: dict) -> datagen.Tables:
    n, m, seed = s["n"], s["m"], s["seed"]
    T = datagen.make_tables(n, m, seed, day_lt=s["day_lt"], group_by=s["group_by"], fk_zipf=s["zipf"],
                            fk_domain=s["domain"], grp_card=s["groups"])
    if s["corr"] == 1:
        T.day = datagen.correlated(T.fk, 0, s["domain"] - 1, 0, datagen.DAY_DOMAIN - 1, 150, seed, datagen.S_DAY + 50)
    elif s["corr"] == 2:
        T.grp = datagen.correlated(T.pk, 0, m - 1, 0, s["groups"] - 1, 0, seed, datagen.S_GRP + 50)
    return T


def build_corpus(ctx, runs: int, seed: int, n_hi: int, chunk: int = 2048):
    """Features [runs, 40] and labels [runs, 2] (join rows, groups) from plain runs."""
    import torch

    from . import rel

    feats = np.zeros((runs, 40), np.float32)
    labels = np.zeros((runs, 2), np.int64)
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    for c0 in range(0, runs, chunk):
        c1 = min(runs, c0 + chunk)
        insts, tabs = [], []
        for i in range(c0, c1):
            T = make_run(run_spec(i, seed, n_hi))
            d = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(dev)
            fact = {"fk": d(T.fk), "price_cents": d(T.price_cents), "qty": d(T.qty), "day": d(T.day), "flag": d(T.flag)}
            dim = {"pk": d(T.pk), "prio": d(T.prio), "grp": d(T.grp)}
            insts.append((fact, dim, T.day_lt, T.group_by, 0))
            tabs.append(T)
        b = rel.Batch(ctx, insts)  # plain sizing: the labels are what the plain pipeline reports
        b.run()
        st = b.sync()
        fdev = torch.empty((c1 - c0, 40), dtype=torch.float32, device=dev)
        for j, (inst, T) in enumerate(zip(insts, tabs)):
            fact, dim = inst[0], inst[1]
            fs = torch.from_numpy(datagen.sample_index(SAMPLE_K, max(T.n, 1), T.meta["seed"], datagen.S_SAMPLE)).to(dev)
            ds = torch.from_numpy(datagen.sample_index(SAMPLE_K, max(T.m, 1), T.meta["seed"], datagen.S_SAMPLE + 1)).to(dev)
            f, _ = rel.sketch(ctx, fact, dim, T.day_lt, T.group_by, fs, ds)
            fdev[j].copy_(f)
            labels[c0 + j] = (st[j]["join_matches"], st[j]["groups"])
        feats[c0:c1] = fdev.cpu().numpy()
        b.close()
        log(f"corpus {c1}/{runs} runs ({time.perf_counter() - t0:.0f} s)")
    return feats, labels


REL_FEATURES = (0, 1, 12, 13, 16, 17, 37)  # size-dependent: taken relative to r
HLL_REGISTER_FEATURES = slice(19, 37)      # register-level HLL features: left out


def relative_inputs(feats: np.ndarray):
    """The network's input before standardisation, and the reference scale r
    per run (mirrors the library's planner input kernel)."""
    f = np.asarray(feats, np.float64)
    r = np.where(f[:, 4] > 0.5, f[:, 17], np.where(f[:, 5] > 0.5, f[:, 37], np.minimum(f[:, 17], f[:, 1])))
    x = f.copy()
    for i in REL_FEATURES:
        x[:, i] -= r
    x[:, HLL_REGISTER_FEATURES] = 0.0
    return x, r


def targets(feats: np.ndarray, labels: np.ndarray):
    """Scale-free targets (join relative to log2(1 + N), groups relative to r)."""
    _, r = relative_inputs(feats)
    y = np.log2(1.0 + labels.astype(np.float64))
    y[:, 0] -= np.asarray(feats, np.float64)[:, 0]
    y[:, 1] -= r
    return y


def train(ctx, feats: np.ndarray, labels: np.ndarray, seed: int, epochs: int, batch: int = 256, lr: float = 1e-3):
    import torch

    from . import rel

    n = feats.shape[0]
    y = targets(feats, labels).astype(np.float32)
    xin = relative_inputs(feats)[0].astype(np.float32)
    perm = np.argsort(datagen.unit(n, seed, 901))
    n_val = max(1, n // 10)
    val, tr = perm[:n_val], perm[n_val:]
    mean = xin[tr].mean(axis=0).astype(np.float32)
    scale = xin[tr].std(axis=0).astype(np.float32)
    scale[scale < 1e-6] = 1.0
    X = torch.from_numpy((xin - mean) / scale).cuda()
    Y = torch.from_numpy(y).cuda()
    # He-uniform initialisation from seeded unit draws (biases zero)
    u = datagen.unit(N_PARAMS, seed, 902)
    theta = np.zeros(N_PARAMS, np.float32)
    o = 0
    for fan_in, cnt in ((40, 40 * 64), (None, 64), (64, 64 * 64), (None, 64), (64, 64 * 2), (None, 2)):
        if fan_in:
            a = math.sqrt(6.0 / fan_in)
            theta[o:o + cnt] = ((2.0 * u[o:o + cnt] - 1.0) * a).astype(np.float32)
        o += cnt
    P = torch.from_numpy(theta).cuda()
    M = torch.zeros_like(P)
    V = torch.zeros_like(P)
    G = torch.empty_like(P)
    L = torch.empty(1, dtype=torch.float32, device="cuda:0")
    tr_t = torch.from_numpy(tr).cuda()
    step = 0
    hist = []
    for ep in range(epochs):
        order = tr_t[torch.from_numpy(np.argsort(datagen.unit(tr.shape[0], seed, 1000 + ep))).cuda()]
        for b0 in range(0, order.numel() - batch + 1, batch):
            idx = order[b0:b0 + batch]
            xb = X.index_select(0, idx).contiguous()
            yb = Y.index_select(0, idx).contiguous()
            rel.mlp_backward(ctx, P, xb, yb, G, L)
            step += 1
            rel.mlp_adam_step(ctx, P, M, V, G, step, lr=lr)
        yv = rel.mlp_forward(ctx, P, X.index_select(0, torch.from_numpy(val).cuda()).contiguous()).cpu().numpy()
        mse = float(np.mean((yv - y[val]) ** 2))
        hist.append(mse)
        log(f"epoch {ep + 1}/{epochs}: validation MSE {mse:.4f} (log2 units^2)")
    yv = rel.mlp_forward(ctx, P, X.index_select(0, torch.from_numpy(val).cuda()).contiguous()).cpu().numpy()
    under = y[val, 1] - yv[:, 1]  # positive = groups under-predicted
    margin = float(max(0.0, np.quantile(under, 0.95)))
    metrics = {"val_mse": hist[-1], "val_mse_hist": hist, "val_mae_groups_log2": float(np.mean(np.abs(under))),
               "margin_log2": margin, "train_runs": int(tr.shape[0]), "val_runs": int(n_val), "epochs": epochs,
               "batch": batch, "lr": lr}
    return P.cpu().numpy(), mean, scale, margin, metrics


def save_model(path, params, mean, scale, margin, meta: dict):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.savez(path, params=params.astype(np.float32), mean=mean.astype(np.float32), scale=scale.astype(np.float32),
             margin=np.array([margin], np.float32), meta=np.array([json.dumps(meta)]))


def load_model(path: str = MODEL):
    z = np.load(path, allow_pickle=False)
    return z["params"], z["mean"], z["scale"], float(z["margin"][0]), json.loads(str(z["meta"][0]))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--runs", type=int, default=200_000)
    ap.add_argument("--seed", type=int, default=1000)
    ap.add_argument("--n-hi", type=int, default=1 << 17)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--out", default=MODEL)
    ap.add_argument("--corpus", default=None, help="npz to save (or reuse, if present) the features and labels")
    args = ap.parse_args()
    from . import rel

    ctx = rel.Context(0)
    if args.corpus and os.path.exists(args.corpus):
        z = np.load(args.corpus, allow_pickle=False)
        feats, labels = z["feats"], z["labels"]
        log(f"loaded corpus {feats.shape[0]} runs from {args.corpus}")
    else:
        feats, labels = build_corpus(ctx, args.runs, args.seed, args.n_hi)
        if args.corpus:
            np.savez(args.corpus, feats=feats, labels=labels)
    params, mean, scale, margin, metrics = train(ctx, feats, labels, args.seed, args.epochs)
    meta = dict(metrics, runs=int(feats.shape[0]), n_hi=args.n_hi, seed=args.seed,
                inputs="relative to the group key's log2 HLL estimate")
    save_model(args.out, params, mean, scale, margin, meta)
    log(f"saved {args.out}: margin {margin:.3f}, validation MSE {metrics['val_mse']:.4f}")
    print(json.dumps(meta))
    ctx.close()


if __name__ == "__main__":
    main()
