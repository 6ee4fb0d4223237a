"""Pins of the seeded input generators: Morton keys against hand-derived
interleaved bits (coordinates quantised to 2**21 levels, clamped, bits
interleaved most-significant first in coordinate order), and the stable
order of the sorted points."""
import numpy as np

import synth


def bit(level, c, d):
    """Position of bit `level` of coordinate c in a d-dimensional key."""
    return level * d + (d - 1 - c)


def test_morton_keys_2d_hand_computed():
    # (0.5, 0.25): x quantises to 2**20 (bit 20), y to 2**19 (bit 19)
    # (0, 0): key 0;  (2**-21, 0): x = 1 (bit 0 of x is the key's bit 1)
    pts = np.array([[0.5, 0.25], [0.0, 0.0], [2.0 ** -21, 0.0], [0.0, 2.0 ** -21]])
    k = synth.morton_keys(pts)
    assert int(k[0]) == (1 << bit(20, 0, 2)) | (1 << bit(19, 1, 2)) == (1 << 41) | (1 << 38)
    assert int(k[1]) == 0
    assert int(k[2]) == 2
    assert int(k[3]) == 1


def test_morton_keys_3d_hand_computed():
    # (0.75, 0.5, 0.125): x has bits 20 and 19, y bit 20, z bit 18
    pts = np.array([[0.75, 0.5, 0.125]])
    k = int(synth.morton_keys(pts)[0])
    assert k == (1 << 62) | (1 << 59) | (1 << 61) | (1 << 54)
    assert k == sum(1 << bit(l, c, 3) for l, c in [(20, 0), (19, 0), (20, 1), (18, 2)])


def test_morton_keys_clamp_at_zero_and_one():
    # 1.0 and above clamp to the top level 2**21 - 1 (all 21 bits set);
    # negative coordinates clamp to 0
    pts = np.array([[1.0, 0.0], [1.5, -0.25], [-3.0, 1.0], [1.0, 1.0]])
    k = [int(v) for v in synth.morton_keys(pts)]
    xs = sum(1 << bit(l, 0, 2) for l in range(21))
    ys = sum(1 << bit(l, 1, 2) for l in range(21))
    assert k[0] == xs == 2 * (4 ** 21 - 1) // 3
    assert k[1] == xs
    assert k[2] == ys == (4 ** 21 - 1) // 3
    assert k[3] == (1 << 42) - 1
    # just below 1 is the top level too; just below 2**-21 is level 0
    assert int(synth.morton_keys(np.array([[1.0 - 2.0 ** -30]]))[0]) == (1 << 21) - 1
    assert int(synth.morton_keys(np.array([[2.0 ** -21 - 2.0 ** -40]]))[0]) == 0


def test_morton_keys_tie_and_stable_order():
    """Two points in one quantisation cell share a key; the sort that orders
    the workload's points keeps them in their original order."""
    a = np.array([0.1, 0.2])
    pts = np.array([[0.9, 0.9], a + [1e-9, 0.0], [0.05, 0.05], a])
    k = synth.morton_keys(pts)
    assert k[1] == k[3]
    assert len(set(int(v) for v in k)) == 3
    order = np.argsort(k, kind="stable")
    assert list(order) == [2, 1, 3, 0]
    # the workload generator sorts by the same keys, stably
    x = synth.points(5, synth.STREAM_X, 257, 2)
    kx = synth.morton_keys(x)
    assert np.all(kx[:-1] <= kx[1:])
