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


def myrtle_empirical_ntk(x: np.ndarray, depth, sw2: float, sb2: float, width: int, seed: int) -> np.ndarray:
    """Empirical neural tangent kernel of one random finite network in the
    parameterisation where each layer multiplies N(0, 1) weights by
    sqrt(sw2 / fan_in) and N(0, 1) biases by sqrt(sb2) in the forward pass:
    Theta(x, x') = sum over all parameters of df(x)/dp df(x')/dp, for a scalar
    readout f (float64, CPU)."""
    g = torch.Generator().manual_seed(seed)
    params = []
    shapes = []
    cin = x.shape[3]
    for s, d in enumerate(depth):
        for _ in range(d):
            params.append(torch.randn(width, cin, 3, 3, generator=g, dtype=torch.float64).requires_grad_())
            params.append(torch.randn(width, generator=g, dtype=torch.float64).requires_grad_())
            shapes.append(("conv", cin))
            cin = width
    w_out = torch.randn(width, generator=g, dtype=torch.float64).requires_grad_()
    b_out = torch.randn(1, generator=g, dtype=torch.float64).requires_grad_()

    def f(img):
        h = torch.tensor(np.asarray(img, dtype=np.float64)).permute(2, 0, 1).unsqueeze(0)
        k = 0
        for s, d in enumerate(depth):
            for _ in range(d):
                w, b = params[2 * k], params[2 * k + 1]
                fan = shapes[k][1] * 9
                h = torch.relu(torch.nn.functional.conv2d(h, w, None, padding=1) * math.sqrt(sw2 / fan)
                               + b.view(1, -1, 1, 1) * math.sqrt(sb2))
                k += 1
            if s + 1 < len(depth):
                h = torch.nn.functional.avg_pool2d(h, 2)
        feat = h.mean(dim=(2, 3))[0]
        return (feat @ w_out) * math.sqrt(sw2 / width) + b_out[0] * math.sqrt(sb2)

    allp = params + [w_out, b_out]
    grads = []
    for img in x:
        gr = torch.autograd.grad(f(img), allp, allow_unused=True)
        grads.append(torch.cat([(t if t is not None else torch.zeros_like(p)).reshape(-1)
                                for t, p in zip(gr, allp)]))
    G = torch.stack(grads)
    return (G @ G.T).numpy()


def cv_empirical(x: np.ndarray, depth: int, sw2: float, sb2: float, width: int, seed: int) -> np.ndarray:
    """Empirical NNGP of a random CNN-VEC network: ``depth`` SAME 3x3 conv + ReLU
    layers at full resolution (weights N(0, sw2 / (9 C_in)), biases N(0, sb2)),
    Flatten, and a Dense readout whose randomness is integrated out:
    sw2 <f, f'> / (h w width) + sb2."""
    g = torch.Generator().manual_seed(seed)
    h = torch.tensor(np.asarray(x, dtype=np.float32)).permute(0, 3, 1, 2).contiguous()
    cin = h.shape[1]
    for _ in range(depth):
        w = torch.randn(width, cin, 3, 3, generator=g) * math.sqrt(sw2 / (9 * cin))
        b = torch.randn(width, generator=g) * math.sqrt(sb2)
        h = torch.relu(torch.nn.functional.conv2d(h, w, b, padding=1))
        cin = width
    f = h.reshape(h.shape[0], -1).double()
    return (sw2 * f @ f.T / f.shape[1] + sb2).numpy()
