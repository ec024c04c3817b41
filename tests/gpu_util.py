"""Helpers of the GPU parity tests (comparison in FP64 on the host)."""
import numpy as np
import torch


def gram(B):
    B = B.double().cpu().numpy() if isinstance(B, torch.Tensor) else np.asarray(B, dtype=np.float64)
    return B.T @ B


def rel_fro(X, Y):
    return float(np.linalg.norm(X - Y) / max(np.linalg.norm(Y), 1e-300))


def cov_err_gram(AtA, BtB):
    D = AtA - BtB
    return float(np.max(np.abs(np.linalg.eigvalsh((D + D.T) / 2))))


def note(msg):
    print(msg, flush=True)
