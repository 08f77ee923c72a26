"""Helpers for the GPU parity tests (inputs from the seeded generator, expected
values from the oracle only)."""
import numpy as np
import torch

from synth import he_init_params


def normwise(a, ref) -> float:
    """max |a - ref| / max |ref|: the floating-point parity metric."""
    a = np.asarray(a, np.float64)
    ref = np.asarray(ref, np.float64)
    return float(np.max(np.abs(a - ref)) / max(np.max(np.abs(ref)), 1e-30))


def flat_params(params) -> np.ndarray:
    """Canonical vector: per layer, OIHW weights then bias."""
    return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in params]).astype(np.float32)


def vae_params(C, L, seed, bias_scale=0.1):
    from oracle.vae import layer_shapes
    shapes = [(o, i, k) for (o, i, k, s) in layer_shapes(*C, L)]
    return he_init_params(shapes, seed=seed, bias_scale=bias_scale)


def cuda(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def bits(t: torch.Tensor) -> np.ndarray:
    """int64 census tensor -> uint64 numpy bits."""
    return t.cpu().numpy().view(np.uint64)
