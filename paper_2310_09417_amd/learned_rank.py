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


def labels(blocks, b: int, tol: float, seed: int, kmax=None, relative: bool = True):
    """Ranks (numpy int32) and statuses the adaptive method reaches on the
    blocks through the batched path (pass FP64 blocks for FP64 labels)."""
    plan = B.BatchPlan(blocks, b, tol, kmax=kmax, seed=seed, relative=relative)
    plan.launch()
    out = plan.result()
    return out.k.astype(np.int32), out.status.astype(np.int32)


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


def evaluate(blocks, model: RankModel | None, b: int, tol: float, seed: int, margin=0.25,
             relative: bool = True):
    """One batched run with and without the model's hints on the same
    blocks: time, passes over each block, ranks, statuses, fallback count."""
    torch = _torch()
    res = {}
    dev = blocks[0].device
    caps = torch.tensor([min(int(a.shape[0]), int(a.shape[1])) for a in blocks],
                        dtype=torch.int32, device=dev)
    hint = None
    if model is not None:
        F = B.rank_features(blocks, tol, seed, relative)
        hint = model.hints(F, caps, margin)
    for name, h in (("adaptive", None), ("learned", hint)):
        if name == "learned" and h is None:
            continue
        plan = B.BatchPlan(blocks, b, tol, seed=seed, relative=relative,
                           k_hint=h.cpu().numpy() if h is not None else None)
        plan.launch()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        plan.launch()
        e1.record()
        torch.cuda.synchronize()
        out = plan.result()
        res[name] = {"ms": float(e0.elapsed_time(e1)), "k": out.k, "status": out.status,
                     "passes": out.passes, "err_est": out.err_est}
    if hint is not None:
        h = hint.cpu().numpy()
        mn = caps.cpu().numpy()
        # the hinted first passes cover w0 + b vectors (w0 alone at full rank),
        # 64 per pass; any further pass is the adaptive fallback
        first = np.where(h < mn, (h + b + 63) // 64, (h + 63) // 64)
        res["learned"]["fallback"] = int(np.sum(res["learned"]["passes"] > first))
        res["learned"]["hint"] = h
    return res
