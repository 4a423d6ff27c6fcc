"""Training driver of the tile-scoring network (VERDICT mode, RD_ORDER_MLP).

Labels come from the library's exact checker (rd_tile_data: every tile of
every eligible pair joined); training runs in the library's forward /
backward / Adam kernels (rd_mlp_train).  Weights are stored as a raw float32
blob (6337 values, the rd_mlp layout) next to a JSON header.

    python -m paper_2604_02106_amd.tile_mlp --out paper_2604_02106_amd/weights/tile_mlp
"""
import argparse
import json
import os

import numpy as np

import paper_2604_02106_amd as hg

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT = os.path.join(HERE, "weights", "tile_mlp")
FEATURE_VERSION = 2  # 32 features incl. per-thread / per-block address steps


def init_weights(seed=0):
    """He-style initial weights in the rd_mlp layout."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w1 = rng.normal(0, np.sqrt(2.0 / 32), (64, 32))
    w2 = rng.normal(0, np.sqrt(2.0 / 64), (64, 64))
    w3 = rng.normal(0, np.sqrt(1.0 / 64), 64)
    return np.concatenate([w1.ravel(), np.zeros(64), w2.ravel(), np.zeros(64),
                           w3, np.zeros(1)]).astype(np.float32)


def training_workloads(seed=4005):
    """Sparse-witness queries with disjoint and with overlapping tiles
    (small grids) plus batched-style models; evaluation uses other seeds."""
    from workloads import configs
    wls = [configs.sparse(seed=seed, n_queries=256, G=32, B=64,
                          queries_per_model=32),
           configs.sparse_overlap(seed=seed, n_queries=256, G=32, B=64,
                                  queries_per_model=32),
           configs.batched(seed=seed + 1, n_models=32, scale=0.02, max_iters=4)]
    return wls


def tile_dataset(ctx, workloads, neg_per_pos=8, seed=0):
    """Balanced (features, labels): every positive tile and up to
    neg_per_pos random negatives per positive (at least 1000)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Xs, Ys = [], []
    for wl in workloads:
        X, Y, _ = hg.rd_tile_data(ctx, wl)
        ok = Y >= 0
        X, Y = X[ok], Y[ok]
        pos = np.nonzero(Y == 1)[0]
        neg = np.nonzero(Y == 0)[0]
        k = min(len(neg), max(1000, neg_per_pos * len(pos)))
        sel = np.concatenate([pos, rng.choice(neg, k, replace=False)]) if k else pos
        Xs.append(X[sel])
        Ys.append(Y[sel])
    return np.concatenate(Xs), np.concatenate(Ys)


def train(ctx, epochs=30, batch=1024, lr=2e-3, seed=0):
    X, Y = tile_dataset(ctx, training_workloads(), seed=seed)
    w0 = init_weights(seed)
    w, losses = hg.rd_mlp_train(ctx, w0, X, Y, epochs=epochs, batch=batch,
                                lr=lr, seed=seed)
    return w, losses, {"rows": int(len(Y)), "positives": int(Y.sum())}


def save(path, w, meta):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.asarray(w, dtype=np.float32).tofile(path + ".bin")
    with open(path + ".json", "w") as f:
        json.dump(dict(meta, n_weights=int(len(w)), dtype="float32",
                       layout="w1[64x32] b1[64] w2[64x64] b2[64] w3[64] b3",
                       feature_version=FEATURE_VERSION), f, indent=1)


def load(path=DEFAULT):
    with open(path + ".json") as f:
        meta = json.load(f)
    assert meta["feature_version"] == FEATURE_VERSION
    w = np.fromfile(path + ".bin", dtype=np.float32)
    assert len(w) == hg.N_MLP
    return w, meta


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--seed", type=int, default=0)
    a = ap.parse_args()
    ctx = hg.Context(0)
    w, losses, info = train(ctx, epochs=a.epochs, seed=a.seed)
    save(a.out, w, dict(info, seed=a.seed, epochs=a.epochs,
                        losses=[float(x) for x in losses]))
    print(json.dumps(dict(info, first_loss=float(losses[0]),
                          last_loss=float(losses[-1]))))


if __name__ == "__main__":
    main()
