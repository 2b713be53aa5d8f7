"""Finite-width random networks (float32, CPU) whose empirical kernels
converge to the NNGP as width grows: the Monte-Carlo pin for the oracle.

The networks follow App. A: 3x3 SAME convolutions with weights
N(0, sw2 / (9 C_in)) and biases N(0, sb2), ReLU, 2x2 average pools between
stages, global average pool, and a Dense readout with weight variance sw2
(the readout's own randomness is integrated out exactly: its kernel given the
features is sw2 <f, f'> / width + sb2).
"""
import math

import numpy as np
import torch


def myrtle_empirical(x: np.ndarray, depth, sw2: float, sb2: float, width: int, seed: int) -> np.ndarray:
    g = torch.Generator().manual_seed(seed)
    h = torch.tensor(np.asarray(x, dtype=np.float32)).permute(0, 3, 1, 2).contiguous()
    cin = h.shape[1]
    for s, d in enumerate(depth):
        for _ in range(d):
            w = torch.randn(width, cin, 3, 3, generator=g) * math.sqrt(sw2 / (9 * cin))
            b = torch.randn(width, generator=g) * math.sqrt(sb2)
            h = torch.relu(torch.nn.functional.conv2d(h, w, b, padding=1))
            cin = width
        if s + 1 < len(depth):
            h = torch.nn.functional.avg_pool2d(h, 2)
    f = h.mean(dim=(2, 3)).double()
    return (sw2 * f @ f.T / width + sb2).numpy()


def fc_empirical(x: np.ndarray, depth: int, sw2: float, sb2: float, width: int, seed: int) -> np.ndarray:
    g = torch.Generator().manual_seed(seed)
    h = torch.tensor(np.asarray(x, dtype=np.float32).reshape(x.shape[0], -1))
    din = h.shape[1]
    for _ in range(depth):
        w = torch.randn(din, width, generator=g) * math.sqrt(sw2 / din)
        b = torch.randn(width, generator=g) * math.sqrt(sb2)
        h = torch.relu(h @ w + b)
        din = width
    f = h.double()
    return (sw2 * f @ f.T / width + sb2).numpy()
