"""Rank predictor of the learned form: training data recorded by the solver
itself, training on the GPU, evaluation.

The solver logs, for every compressed cell, six features (k_T d, k_L d,
level, active DOFs per component, rows of the proxy-plus-near matrix,
-log10 tol) and the cell's four ID ranks (``Factor.rank_log``).  The target
is the largest of the four.  ``mlp_init`` standardises the features and
draws the initial weights, ``mlp_train`` runs minibatch Adam with the
library's own forward / backward / update kernels; the trained float32 blob
is passed to ``Factor(..., predictor=blob)``.

Usage (writes the blob and a JSON summary):
    python -m paper_2411_18026_amd.predictor --geometries 200 --out predictor.npy
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import Factor, mlp_forward, mlp_init, mlp_train


def rank_log_dataset(curves, omega, lam, mu, rho, tol, leaf=64, **kw):
    """(features n x 6, target n) of one factorisation in the adaptive form."""
    F = Factor(curves, omega, lam, mu, rho, tol, leaf=leaf, **kw)
    log = F.rank_log()
    F.close()
    return log["feat"].astype(np.float32), log["rank"].max(axis=1).astype(np.float32)


def collect(geometries, tol=1e-8, leaf=64, lam=2.0, mu=1.0, rho=1.0, progress=None):
    """Rank logs of a list of (curves, k_T) (omega = k_T sqrt(mu / rho))."""
    xs, ys = [], []
    for i, (curves, k_t) in enumerate(geometries):
        omega = k_t * np.sqrt(mu / rho)
        x, y = rank_log_dataset(curves, omega, lam, mu, rho, tol, leaf)
        xs.append(x)
        ys.append(y)
        if progress:
            progress(i, len(y))
    return np.concatenate(xs), np.concatenate(ys)


def train(x, y, steps=3000, batch=512, lr=2e-3, seed=1):
    """A trained predictor blob and its loss history."""
    blob = mlp_init(x, y, seed)
    return mlp_train(blob, x, y, steps, batch, lr, seed + 1)


def evaluate(blob, x, y, oversample=8):
    """Prediction quality as the learned factorisation sees it (bfloat16
    inference): fraction of cells whose rank exceeds ceil(pred) + oversample
    (sketch too small), mean over-allocation, mean absolute error."""
    p = mlp_forward(blob, x, bf16=True).cpu().numpy()
    s = np.ceil(np.maximum(p, 0.0)) + oversample
    return {"cells": int(len(y)), "under": float(np.mean(y >= s)), "mae": float(np.mean(np.abs(p - y))),
            "mean_slack": float(np.mean(s - y))}


def main():
    import synthetic as sy
    ap = argparse.ArgumentParser()
    ap.add_argument("--geometries", type=int, default=200)
    ap.add_argument("--nodes", type=int, default=16384)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--out", default="predictor.npy")
    a = ap.parse_args()
    t0 = time.perf_counter()
    geoms = (sy.training_geometry(i, a.nodes) for i in range(a.geometries))
    x, y = collect(geoms, progress=lambda i, n: print(f"geometry {i}: {n} cells", flush=True))
    t1 = time.perf_counter()
    blob, hist = train(x, y, steps=a.steps)
    t2 = time.perf_counter()
    np.save(a.out, blob)
    summary = {"geometries": a.geometries, "cells": int(len(y)), "collect_s": round(t1 - t0, 2),
               "train_s": round(t2 - t1, 2), "loss_first": float(hist[0]), "loss_last": float(hist[-1]),
               "train_fit": evaluate(blob, x, y)}
    print(json.dumps(summary), flush=True)


if __name__ == "__main__":
    main()
