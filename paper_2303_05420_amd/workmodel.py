"""Work model of the Myrtle NNGP: how many covariance entries each pair of
images carries through the network, and the fixed flop count per entry used
to express throughput as a fraction of the FP32 vector peak.

Pure Python; loads no native code.
"""
from __future__ import annotations

from typing import Sequence

# Fixed op model (FMA = 2 flops, sqrt = 1 flop): per entry and conv+ReLU layer,
# 6 flops for the separable 3x3 box sum and 24 for the ReLU arc-cosine map.
FLOPS_PER_ENTRY_LAYER = 30
FLOPS_PER_SEED_ENTRY_PER_CHANNEL = 2
FLOPS_PER_POOLED_ENTRY = 1
# Tangent kernel (NTK), on top of the covariance's 30 per entry-layer: the box
# sum of the tangent (6), the arc-cosine angle from the square root the map
# already takes (counted as a degree-6 polynomial and one product: 13; the
# kernels evaluate shorter fits of the angle) and the tangent
# update, derivative factor times tangent plus covariance (2 FMA: 4).  The
# network's first layer has no tangent input to sum (its tangent is its
# covariance): 17 there.
NTK_EXTRA_FLOPS_PER_ENTRY_LAYER = 23
NTK_EXTRA_FLOPS_FIRST_LAYER = 17
# Adjoint, per entry and layer reversed, for the cotangent of one image of the
# pair: the derivative of the map (the angle as above, 13, and 1 - angle, 1),
# the cotangents of its argument and of the variance tables (rho_bar, v_bar
# and w: 6), one table-adjoint sum (1), the two hyperparameter sums (3) and
# the box of v_bar (6).  The seed's reverse is 2 flops per channel for one
# image, the pool's 1 per entry.  Recomputation is not counted: the model is
# one forward pass plus this.
ADJ_FLOPS_PER_ENTRY_LAYER = 30
ADJ_FLOPS_PER_SEED_ENTRY_PER_CHANNEL = 2
ADJ_FLOPS_PER_POOLED_ENTRY = 1


def stage_sizes(hw: int, n_stages: int):
    return [hw >> s for s in range(n_stages)]


def entry_layers_per_pair(hw: int, depth: Sequence[int]) -> int:
    """Sum over conv+ReLU layers of the (h w)^2 pair-covariance entries."""
    return sum(d * (n ** 4) for n, d in zip(stage_sizes(hw, len(depth)), depth))


def flops_per_pair(hw: int, c: int, depth: Sequence[int]) -> int:
    n = stage_sizes(hw, len(depth))
    f = FLOPS_PER_ENTRY_LAYER * entry_layers_per_pair(hw, depth)
    f += FLOPS_PER_SEED_ENTRY_PER_CHANNEL * c * n[0] ** 4
    # every entry leaving a stage is added once into a pooled (or global) sum
    f += FLOPS_PER_POOLED_ENTRY * sum(k ** 4 for k in n)
    return f


def kernel_storage_bytes(n_examples: int, bytes_per_entry: int = 8) -> float:
    """Upper triangle of an n x n kernel."""
    return n_examples * n_examples / 2 * bytes_per_entry


def upper_triangle_blocks(n_examples: int, block: int) -> float:
    return (n_examples / block) ** 2 / 2


def cv_flops_per_pair(hw: int, c: int, depth: int) -> int:
    """CNN-VEC (flatten readout): the displacement-0 map of h w entries per
    layer, the seed's channel products, and the readout sum."""
    n2 = hw * hw
    return FLOPS_PER_ENTRY_LAYER * depth * n2 + FLOPS_PER_SEED_ENTRY_PER_CHANNEL * c * n2 + FLOPS_PER_POOLED_ENTRY * n2


def ntk_first_stage_flops_per_pair(hw: int, c: int, d: int) -> int:
    """Op-model flops of the tangent kernel's first stage for one pair: seed,
    d conv+ReLU layers of covariance and tangent at hw x hw, and the 2x2 pool
    of both."""
    n4 = hw ** 4
    per_entry = (FLOPS_PER_ENTRY_LAYER * d + NTK_EXTRA_FLOPS_FIRST_LAYER
                 + NTK_EXTRA_FLOPS_PER_ENTRY_LAYER * (d - 1))
    return per_entry * n4 + FLOPS_PER_SEED_ENTRY_PER_CHANNEL * c * n4 + 2 * FLOPS_PER_POOLED_ENTRY * n4


def adjoint_first_stage_flops_per_pair(hw: int, c: int, d: int) -> int:
    """Op-model flops of the first stage's adjoint for one pair: the forward
    values of its d layers once (seed, layers, pool) and their reverse."""
    n4 = hw ** 4
    fwd = FLOPS_PER_ENTRY_LAYER * d + FLOPS_PER_SEED_ENTRY_PER_CHANNEL * c + FLOPS_PER_POOLED_ENTRY
    rev = ADJ_FLOPS_PER_ENTRY_LAYER * d + ADJ_FLOPS_PER_SEED_ENTRY_PER_CHANNEL * c + ADJ_FLOPS_PER_POOLED_ENTRY
    return (fwd + rev) * n4
