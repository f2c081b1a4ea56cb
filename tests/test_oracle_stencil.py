"""Pins of the central-difference weights (oracle.stencil) against the
textbook table in tests/golden/fd_weights.txt, and of the window rule."""
import os

import numpy as np
import pytest

from oracle.stencil import fd_weights, fd_weights_exact, window_offsets

GOLD = os.path.join(os.path.dirname(__file__), "golden", "fd_weights.txt")


def _golden():
    rows = []
    for line in open(GOLD):
        if line.strip() and not line.startswith("#"):
            v = [int(x) for x in line.split()]
            rows.append((v[0], tuple(v[1:6]), tuple(v[6:11])))
    return rows


@pytest.mark.parametrize("order,offs,w12", _golden())
def test_weights_match_textbook(order, offs, w12):
    w = fd_weights_exact(offs, order)
    assert tuple(12 * x for x in w) == w12          # exact rationals
    assert np.allclose(np.array(fd_weights(offs, order)) * 12, w12, atol=1e-12)


def test_window_rule():
    n = 9
    assert window_offsets(0, n, False) == (0, 1, 2, 3, 4)
    assert window_offsets(1, n, False) == (-1, 0, 1, 2, 3)
    assert window_offsets(4, n, False) == (-2, -1, 0, 1, 2)
    assert window_offsets(n - 2, n, False) == (-3, -2, -1, 0, 1)
    assert window_offsets(n - 1, n, False) == (-4, -3, -2, -1, 0)
    assert window_offsets(0, n, True) == (-2, -1, 0, 1, 2)
    with pytest.raises(ValueError):
        window_offsets(0, 4, False)


def test_weights_differentiate_sin():
    # Fourth-order accuracy: error of the centred first derivative of sin
    # falls by ~2^4 when the step halves.
    errs = []
    for h in (0.1, 0.05):
        xs = 0.3 + h * np.arange(-2, 3)
        w = np.array(fd_weights((-2, -1, 0, 1, 2), 1))
        errs.append(abs(w @ np.sin(xs) / h - np.cos(0.3)))
    assert 12 < errs[0] / errs[1] < 20
