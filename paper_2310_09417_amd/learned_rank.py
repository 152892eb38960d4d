"""Learned rank for the batched decomposition.

A small MLP (19 -> 128 -> 128 -> 1, GELU) predicts, from 19 probe features of
a block (``rank_features``), the log2 of the rank the adaptive method reaches
on it at the requested tolerance.  ``rid_lupp_batched`` then sketches about
that many vectors in its first pass (``k_hint``) instead of growing the sketch
b vectors at a time; when the estimate still misses the tolerance the adaptive
loop simply continues from the factorisation it has (the fallback), so the
result always meets the tolerance or reaches the rank cap as without a hint.

Training runs on the GPU through the library's own kernels (forward, backward
of the pinball loss, AdamW).  Labels are the ranks the FP64 batched path
reaches on the same blocks.  This module only drives those calls: batching,
shuffling and bookkeeping.
"""
from __future__ import annotations

import hashlib
import math
from dataclasses import dataclass

import numpy as np

from . import binding as B

HIDDEN = 128


def _torch():
    import torch
    return torch


@dataclass
class RankModel:
    params: "object"   # FP32 device tensor, mlp_param_count() values
    xnorm: "object"    # FP32 device tensor: 19 means, then 19 inverse std devs

    @staticmethod
    def init(seed: int, device, xnorm) -> "RankModel":
        """Uniform(+-1/sqrt(fan_in)) weights and zero biases (numpy RNG)."""
        torch = _torch()
        rng = np.random.default_rng(seed)
        F, H = B.N_FEATURES, HIDDEN
        parts = [rng.uniform(-1, 1, H * F) / math.sqrt(F), np.zeros(H),
                 rng.uniform(-1, 1, H * H) / math.sqrt(H), np.zeros(H),
                 rng.uniform(-1, 1, H) / math.sqrt(H), np.zeros(1)]
        p = np.concatenate(parts).astype(np.float32)
        assert p.size == B.mlp_param_count()
        return RankModel(torch.as_tensor(p).to(device), xnorm)

    def predict_log2(self, F):
        return B.mlp_forward(F, self.params, self.xnorm)

    def hints(self, F, kcap, margin: float = 0.25):
        """int32 device tensor of first-sketch widths (0 = no hint)."""
        return B.rank_hint(self.predict_log2(F), kcap, margin)

    def state(self) -> dict:
        p = self.params.cpu().numpy()
        x = self.xnorm.cpu().numpy()
        h = hashlib.sha256(p.tobytes() + x.tobytes()).hexdigest()
        return {"params": p, "xnorm": x, "sha256": h}

    def save(self, path: str) -> str:
        st = self.state()
        np.savez(path, params=st["params"], xnorm=st["xnorm"], sha256=np.array(st["sha256"]))
        return st["sha256"]

    @staticmethod
    def load(path: str, device) -> "RankModel":
        torch = _torch()
        z = np.load(path, allow_pickle=False)
        p, x = z["params"].astype(np.float32), z["xnorm"].astype(np.float32)
        h = hashlib.sha256(p.tobytes() + x.tobytes()).hexdigest()
        if h != str(z["sha256"]):
            raise ValueError(f"{path}: weights do not match their recorded hash")
        return RankModel(torch.as_tensor(p).to(device), torch.as_tensor(x).to(device))


def feature_norm(F):
    """Per-feature mean and inverse standard deviation (floored) of a
    training set, as the 38-value xnorm tensor."""
    torch = _torch()
    Fd = F.double()
    mu = Fd.mean(dim=0)
    sd = Fd.std(dim=0).clamp_min(1e-3)
    return torch.cat([mu, 1.0 / sd]).float().contiguous()


def labels(blocks, b: int, tol: float, seed: int, kmax=None, relative: bool = True,
           factor=None):
    """Ranks (numpy int32) and statuses the adaptive method reaches on the
    blocks through the batched path (pass FP64 blocks for FP64 labels;
    factor=torch.float64 with FP32 blocks for the FP32-storage form)."""
    plan = B.BatchPlan(blocks, b, tol, kmax=kmax, seed=seed, relative=relative, factor=factor)
    plan.launch()
    out = plan.result()
    return out.k.astype(np.int32), out.status.astype(np.int32)


def training_set(make_chunk, n_chunks: int, forms, b: int, seed: int):
    """Features and labels over n_chunks generated chunks of blocks, keeping
    only those (the blocks of a chunk are dropped before the next one).
    make_chunk(i) -> list of FP64 device blocks; forms: (tol, storage dtype,
    factor) triples, each labelled by the batched path itself with the stream
    of seed + block index within the chunk.  Returns (F: N x 19 device FP32,
    k: numpy int32)."""
    torch = _torch()
    Fs, ks = [], []
    for i in range(n_chunks):
        blocks64 = make_chunk(i)
        for tol, storage, factor in forms:
            blocks = blocks64 if storage == torch.float64 else [a.to(storage) for a in blocks64]
            k, _ = labels(blocks, b, tol, seed, factor=factor)
            Fs.append(B.rank_features(blocks, tol, seed))
            ks.append(k)
            del blocks
        del blocks64
    return torch.cat(Fs), np.concatenate(ks)


def fit(F, k, epochs: int = 60, batch: int = 1024, lr: float = 2e-3, q: float = 0.9,
        wd: float = 1e-4, seed: int = 0, log=None) -> tuple[RankModel, list]:
    """Train on features F (N x 19 device FP32) and ranks k (N, numpy int) to
    predict log2 k under the pinball loss with quantile q.  Minibatch AdamW
    with the library's kernels; returns the model and the per-epoch loss."""
    torch = _torch()
    dev = F.device
    N = int(F.shape[0])
    t = torch.as_tensor(np.log2(np.maximum(np.asarray(k, dtype=np.float64), 1.0)),
                        dtype=torch.float32).to(dev)
    model = RankModel.init(seed, dev, feature_norm(F))
    P = model.params
    m1 = torch.zeros_like(P)
    m2 = torch.zeros_like(P)
    rng = np.random.default_rng(seed + 1)
    work = None
    step = 0
    hist = []
    for ep in range(epochs):
        perm = torch.as_tensor(rng.permutation(N), dtype=torch.int64).to(dev)
        tot = 0.0
        nb = 0
        for s in range(0, N, batch):
            idx = perm[s:s + batch]
            X, tt = F[idx].contiguous(), t[idx].contiguous()
            y, z1, z2 = B.mlp_forward(X, P, model.xnorm, save=True)
            if work is None:
                wb = int(B.library().rid_mlp_workspace_bytes(min(batch, N)))
                work = torch.empty(wb, dtype=torch.uint8, device=dev)
            g, loss = B.mlp_backward(X, z1, z2, y, tt, q, P, model.xnorm, work)
            step += 1
            B.mlp_adamw(P, g, m1, m2, step, lr, wd=wd)
            tot += float(loss.item())
            nb += 1
        hist.append(tot / max(nb, 1))
        if log:
            log(f"[learned] epoch {ep + 1}/{epochs}: pinball loss {hist[-1]:.4f}")
    return model, hist


def learned_launch(plan, model: RankModel, caps, margin: float):
    """The learned batched call on one stream, without host synchronisation
    (capturable in a HIP graph): probe features of the plan's blocks, the
    MLP, the hints written into the plan's k_hint array, then the batched
    launch.  The plan must have been made with a k_hint array."""
    F = plan.features()
    h = B.rank_hint(model.predict_log2(F), caps, margin)
    plan.k_hint.copy_(h)
    plan.launch()


def evaluate(blocks, model: RankModel | None, b: int, tol: float, seed: int, margin=0.25,
             relative: bool = True, factor=None, order=None, graph: bool = False,
             reps: int = 1):
    """Batched runs with and without the model's hints on the same blocks:
    time (the learned time covers the probe features, the MLP and the
    hints as well), passes over each block, ranks, statuses, fallback count.
    graph: time replays of the whole call captured in a HIP graph."""
    torch = _torch()
    res = {}
    dev = blocks[0].device
    caps = torch.tensor([min(int(a.shape[0]), int(a.shape[1])) for a in blocks],
                        dtype=torch.int32, device=dev)
    for name in ("adaptive", "learned"):
        if name == "learned" and model is None:
            continue
        hint0 = np.zeros(len(blocks), dtype=np.int32) if name == "learned" else None
        plan = B.BatchPlan(blocks, b, tol, seed=seed, relative=relative, k_hint=hint0,
                           order=order, factor=factor)
        if name == "learned":
            def call(st=None):
                learned_launch(plan, model, caps, margin)
        else:
            def call(st=None):
                plan.launch()
        call()
        torch.cuda.synchronize()
        run = call
        g = None
        if graph:
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                call()
            g.replay()
            torch.cuda.synchronize()
            run = g.replay
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            run()
        e1.record()
        torch.cuda.synchronize()
        out = plan.result()
        res[name] = {"ms": float(e0.elapsed_time(e1)) / reps, "k": out.k, "status": out.status,
                     "passes": out.passes, "err_est": out.err_est}
        if name == "learned":
            res[name]["hint"] = plan.k_hint.cpu().numpy()
            # the prediction alone (features, MLP, hints), for the split
            e0.record()
            for _ in range(reps):
                F = plan.features()
                plan.k_hint.copy_(B.rank_hint(model.predict_log2(F), caps, margin))
            e1.record()
            torch.cuda.synchronize()
            res[name]["predict_ms"] = float(e0.elapsed_time(e1)) / reps
        del g, plan
    if "learned" in res:
        h = res["learned"]["hint"]
        mn = caps.cpu().numpy()
        # the hinted first passes cover w0 + b vectors (w0 alone at full rank),
        # 64 per pass; any further pass is the adaptive fallback
        first = np.where(h < mn, (h + b + 63) // 64, (h + 63) // 64)
        res["learned"]["fallback"] = int(np.sum(res["learned"]["passes"] > first))
    return res


def choose_margin(blocks, model: RankModel, b: int, tol: float, seed: int,
                  margins=(0.0, 0.1, 0.25, 0.5), **kw):
    """The hint margin with the shortest measured time on a validation set
    (blocks not used for training or for the final comparison)."""
    best, best_ms = margins[0], None
    for mg in margins:
        r = evaluate(blocks, model, b, tol, seed, margin=mg, **kw)["learned"]
        if best_ms is None or r["ms"] < best_ms:
            best, best_ms = mg, r["ms"]
    return best
