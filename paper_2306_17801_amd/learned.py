"""Training and use of the learned polynomial preconditioner.

Marshalling only: the features, the training labels (each system's own
Jacobi-PCG solve), the standardisation, the network's forward and backward
passes, Adam and the flexible solve all run in the library's kernels; this
module allocates the device tensors, orders the calls and keeps uploads alive
until the context has consumed them.
"""
from __future__ import annotations

import numpy as np

from . import (apcg_ctx_synchronize, apcg_ksp_solve_learned, apcg_mlp_loss_grad, apcg_mlp_standardize,
               apcg_mlp_train_step, apcg_pc_features, apcg_pc_label)
from .device import DeviceCSR, DeviceVec
from .problems import MLP_SHAPES, mlp_initial_params

NFEAT = 16
NCOEF = 9
NPARAM = 5833


def _cuda(device):
    return f"cuda:{device}"


def pack_params(params: dict) -> np.ndarray:
    """Flat float32 parameter vector in the library's layout."""
    return np.concatenate([np.asarray(params[k], dtype=np.float64).reshape(-1) for k, _ in MLP_SHAPES]).astype(
        np.float32)


class LearnedPC:
    """A trained network: parameters and the feature standardisation."""

    def __init__(self, params, mean, std):
        self.params = params  # float32[5833] on the device
        self.mean = mean      # float32[16]
        self.std = std        # float32[16]

    def save(self, path: str) -> None:
        np.savez(path, params=self.params.cpu().numpy(), mean=self.mean.cpu().numpy(), std=self.std.cpu().numpy())

    @classmethod
    def load(cls, path: str, device: int = 0) -> "LearnedPC":
        import torch

        z = np.load(path, allow_pickle=False)
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(_cuda(device))
        pc = cls(t(z["params"]), t(z["mean"]), t(z["std"]))
        torch.cuda.synchronize(device)
        return pc


class Dataset:
    """Per-system features X [B, 16], loss forms G [B, 81] and h [B, 9],
    labels [B, 3] = (lmin, a, lmax) and lmax [B] (device tensors)."""

    def __init__(self, X, G, h, label, lmax):
        self.X, self.G, self.h, self.label, self.lmax = X, G, h, label, lmax

    @property
    def size(self) -> int:
        return int(self.X.shape[0])


def collect(ctx, systems, rtol: float = 1e-8, maxit: int = 20000, labels: bool = True,
            device: int = 0, count: int | None = None) -> Dataset:
    """Features (and, with ``labels``, the training labels) of each system.
    ``systems`` holds host systems (uploaded here) or already uploaded
    (DeviceCSR, DeviceVec) pairs, which this call then owns; it may be an
    iterator, with ``count`` giving its length.  One system is resident at a
    time; the context is synchronised before its upload is released."""
    import torch

    B = len(systems) if count is None else int(count)
    dev = _cuda(device)
    X = torch.zeros((B, NFEAT), dtype=torch.float32, device=dev)
    G = torch.zeros((B, NCOEF * NCOEF), dtype=torch.float32, device=dev)
    h = torch.zeros((B, NCOEF), dtype=torch.float32, device=dev)
    lab = torch.zeros((B, 3), dtype=torch.float64, device=dev)
    lmax = torch.zeros(B, dtype=torch.float64, device=dev)
    torch.cuda.synchronize(device)
    for i, s in enumerate(systems):
        if i >= B:
            raise ValueError("more systems than count")
        dA, db = s if isinstance(s, tuple) else (DeviceCSR(s.A, device), DeviceVec(s.b, device))
        apcg_pc_features(ctx, dA.h, db.h, X[i], lmax[i:i + 1])
        if labels:
            apcg_pc_label(ctx, dA.h, db.h, rtol, maxit, G[i], h[i], lab[i])
        apcg_ctx_synchronize(ctx)
        dA.close()
        db.close()
    return Dataset(X, G, h, lab, lmax)


def train(ctx, data: Dataset, epochs: int = 300, batch: int = 128, lr: float = 3e-3, seed: int = 7,
          mu: float = 1.0, eps: float = 0.05, device: int = 0):
    """Adam on the mean loss over contiguous minibatches of the standardised
    features (their order shuffled per epoch on the host).  Returns the
    network and the per-step losses (host array)."""
    import torch

    dev = _cuda(device)
    X = data.X.clone()
    mean = torch.zeros(NFEAT, dtype=torch.float32, device=dev)
    std = torch.zeros(NFEAT, dtype=torch.float32, device=dev)
    params = torch.from_numpy(pack_params(mlp_initial_params(seed))).to(dev)
    m = torch.zeros(NPARAM, dtype=torch.float32, device=dev)
    v = torch.zeros(NPARAM, dtype=torch.float32, device=dev)
    B = data.size
    starts = list(range(0, B, batch))
    losses = torch.zeros(epochs * len(starts), dtype=torch.float32, device=dev)
    torch.cuda.synchronize(device)
    apcg_mlp_standardize(ctx, X, mean, std, True)
    rng = np.random.default_rng(seed)
    t = 0
    for _ in range(epochs):
        for s0 in rng.permutation(starts):
            s1 = min(int(s0) + batch, B)
            apcg_mlp_train_step(ctx, params, m, v, t + 1, lr, X[s0:s1], data.G[s0:s1], data.h[s0:s1],
                                losses[t:t + 1], mu, eps)
            t += 1
    apcg_ctx_synchronize(ctx)
    out = losses.cpu().numpy()
    del X, m, v
    return LearnedPC(params, mean, std), out


def mean_loss(ctx, pc: LearnedPC, data: Dataset, mu: float = 1.0, eps: float = 0.05, device: int = 0) -> float:
    """Mean loss of the network on a dataset (features standardised with the
    network's statistics)."""
    import torch

    dev = _cuda(device)
    X = data.X.clone()
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    grad = torch.zeros(NPARAM, dtype=torch.float32, device=dev)
    torch.cuda.synchronize(device)
    apcg_mlp_standardize(ctx, X, pc.mean, pc.std, False)
    apcg_mlp_loss_grad(ctx, pc.params, X, data.G, data.h, loss, grad, mu, eps)
    apcg_ctx_synchronize(ctx)
    return float(loss.cpu().numpy()[0])


def solve(ctx, pc: LearnedPC, A, b, x, rtol: float, maxit: int, opts=None, fopts=None, info=None,
          info_index: int = 0) -> None:
    """FCG(1) with the network's polynomial for (A, b) (handles)."""
    apcg_ksp_solve_learned(ctx, A, b, x, rtol, maxit, pc.params, pc.mean, pc.std, opts, fopts, info, info_index)
