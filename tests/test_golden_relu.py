"""Oracle ReLU map against the closed-form values in tests/golden/relu_map_values.txt."""
import os

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden", "relu_map_values.txt")


def test_relu_map_golden():
    n = 0
    for line in open(GOLD):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        s, q1, q2, f = (float(v) for v in line.split())
        assert abs(oracle.relu_map(s, q1, q2) - f) <= 2e-16 * max(1.0, abs(f))
        n += 1
    assert n == 5
