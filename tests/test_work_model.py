"""The work model reproduces the size/cost figures the paper states
(tests/golden/paper_scale_figures.txt)."""
import os

from paper_2303_05420_amd import workmodel

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_scale_figures.txt")


def _gold():
    out = {}
    for line in open(GOLD):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        k, v = line.split()[:2]
        out[k] = v
    return out


def test_storage_and_blocks():
    g = _gold()
    n = int(g["largest_kernel_examples"])
    assert abs(workmodel.kernel_storage_bytes(n) / float(g["largest_kernel_bytes"]) - 1) < 0.01
    assert abs(workmodel.upper_triangle_blocks(n, int(g["block_side"])) / float(g["largest_kernel_blocks"]) - 1) < 0.01


def test_pooling_kernel_cost_grows_with_pixels_squared():
    g = _gold()
    # one conv+ReLU layer at full resolution: entries per pair = (h w)^2
    r = workmodel.entry_layers_per_pair(224, [1]) / workmodel.entry_layers_per_pair(32, [1])
    assert r == int(g["pool_kernel_cost_ratio"])


def test_myrtle10_counts():
    g = _gold()
    depth = [int(v) for v in g["myrtle10_conv_per_stage"].split(",")]
    assert workmodel.entry_layers_per_pair(32, depth) == 3 * (32 ** 4 + 16 ** 4 + 8 ** 4) == 3354624
    assert workmodel.entry_layers_per_pair(8, [2, 1, 1]) == 8464


def test_ntk_first_stage_op_model():
    # one layer at 2x2, one channel: 16 entries, 30 + 17 per entry-layer,
    # 2 per seed entry and channel, 1 per pooled entry for each of the two
    # pooled tiles
    assert workmodel.ntk_first_stage_flops_per_pair(2, 1, 1) == 16 * (47 + 2 + 2)
    # each further layer adds 30 + 23 per entry
    d3 = workmodel.ntk_first_stage_flops_per_pair(32, 3, 3)
    d2 = workmodel.ntk_first_stage_flops_per_pair(32, 3, 2)
    assert d3 - d2 == 53 * 32 ** 4


def test_adjoint_first_stage_op_model():
    # forward values (30 per layer, 2 per channel, 1 pooled) plus a reverse
    # of the same size: twice the forward's first-stage count
    for hw, c, d in ((2, 1, 1), (32, 3, 2), (16, 4, 3)):
        fwd = (30 * d + 2 * c + 1) * hw ** 4
        assert workmodel.adjoint_first_stage_flops_per_pair(hw, c, d) == 2 * fwd
