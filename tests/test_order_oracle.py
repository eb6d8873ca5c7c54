"""Pins of the spatial-order oracle (oracle/order.py) against values fixed by
its definition, computed by other routes: binary strings for the bit
interleave, hand-worked boxes and cells, brute force over small maps."""
import math

import numpy as np
import pytest

from oracle import order as O


def _string_morton(qx, qy, qz):
    """Morton code by interleaving the characters of 10-digit binary strings
    (most significant first: z, y, x of bit 9, then of bit 8, ...)."""
    sx, sy, sz = (format(int(v), "010b") for v in (qx, qy, qz))
    return int("".join(sz[k] + sy[k] + sx[k] for k in range(10)), 2)


def test_interleave_matches_binary_strings():
    rng = np.random.default_rng(1)
    q = rng.integers(0, 1024, size=(3, 500))
    q[:, 0] = 0
    q[:, 1] = 1023
    q[:, 2] = [1, 0, 0]
    q[:, 3] = [0, 1, 0]
    q[:, 4] = [0, 0, 1]
    got = O.interleave(q)
    want = [_string_morton(*q[:, i]) for i in range(q.shape[1])]
    assert got.tolist() == want
    assert got[1] == (1 << 30) - 1 and got[2:5].tolist() == [1, 2, 4]


def test_cells_on_a_worked_grid():
    """Extent 1023 along x: 1023 = 0.999 * 2^10, so the cell side is
    2^10 / 1024 = 1 and an integer coordinate is its own cell; extent 1024
    (= 0.5 * 2^11) doubles the side."""
    x = np.array([0.0, 1.0, 2.5, 511.0, 1022.9, 1023.0], dtype=np.float32)
    mean = np.stack([x, np.zeros_like(x), np.full_like(x, 7.0)])
    q, fin = O.cells(mean)
    assert fin.all()
    assert q[0].tolist() == [0, 1, 2, 511, 1022, 1023]
    assert q[1].tolist() == [0] * 6 and q[2].tolist() == [0] * 6
    x2 = np.array([-5.0, -4.0, -3.0, 1019.0], dtype=np.float32)  # lo = -5, extent 1024
    mean2 = np.stack([np.zeros_like(x2), x2, np.zeros_like(x2)])
    q2, _ = O.cells(mean2)
    assert q2[1].tolist() == [0, 0, 1, 512]


def test_cells_use_the_largest_extent_for_every_axis():
    """Cubic cells: the side comes from the longest axis (here z, extent 4 =
    0.5 * 2^3, side 8 / 1024), and each axis counts from its own minimum."""
    mean = np.array([[10.0, 10.5, 11.0], [0.0, 0.0, 0.0], [-2.0, 0.0, 2.0]], dtype=np.float32)
    q, _ = O.cells(mean)
    side = 8.0 / 1024
    assert q[0].tolist() == [0, int(0.5 / side), int(1.0 / side)]
    assert q[2].tolist() == [0, int(2.0 / side), int(4.0 / side)]


def test_degenerate_maps():
    one = np.array([[1.0], [2.0], [3.0]], dtype=np.float32)
    assert O.codes(one).tolist() == [0]
    assert O.spatial_order(one, 1).tolist() == [0]
    same = np.ones((3, 9), dtype=np.float32)
    assert O.codes(same).tolist() == [0] * 9
    # equal codes keep index order; B >= n leaves the ranks in place
    assert O.spatial_order(same, 9).tolist() == list(range(9))
    allnan = np.full((3, 4), np.nan, dtype=np.float32)
    assert O.codes(allnan).tolist() == [1 << 30] * 4
    assert O.spatial_order(allnan, 100).tolist() == [0, 1, 2, 3]


def test_nonfinite_go_last_in_index_order():
    rng = np.random.default_rng(2)
    mean = rng.normal(size=(3, 50)).astype(np.float32)
    bad = [3, 17, 40]
    mean[0, 3] = np.nan
    mean[1, 17] = np.inf
    mean[2, 40] = -np.inf
    idx = O.spatial_order(mean, 1000)
    assert idx[-3:].tolist() == bad
    # and they do not move the box
    lo, w = O.box(mean)
    good = np.delete(mean, bad, axis=1).astype(np.float64)
    assert np.array_equal(lo, good.min(axis=1))
    assert w == float(np.max(good.max(axis=1) - good.min(axis=1)))


def test_brick_multiplier_by_hand():
    assert O.brick_multiplier(0) == 1 and O.brick_multiplier(1) == 1
    assert O.brick_multiplier(10) == 7     # 6.68 -> 6, gcd(6, 10) = 2; 7
    assert O.brick_multiplier(13) == 8     # 8.53 -> 8, coprime
    assert O.brick_multiplier(2) == 1      # 1.74 -> 1
    for f in range(2, 300):
        p = O.brick_multiplier(f)
        assert math.gcd(p, f) == 1 and p >= math.floor(0.6180339887498949 * f + 0.5)
        assert sorted((b * p) % f for b in range(f)) == list(range(f))


def _brute_order(mean, brick):
    """Steps 4-6 by Python loops over the oracle's codes (checked above)."""
    n = mean.shape[1]
    code = O.codes(mean).tolist()
    ranked = sorted(range(n), key=lambda i: (code[i], i))
    full = n // brick
    p = O.brick_multiplier(full)
    out = []
    for j in range(full):
        src = (j * p) % full
        out.extend(ranked[src * brick:(src + 1) * brick])
    out.extend(ranked[full * brick:])
    return out


@pytest.mark.parametrize("n,brick", [(1, 1), (7, 3), (100, 1), (100, 7), (1000, 64), (1000, 999), (1000, 1000),
                                     (1001, 1000), (4099, 128)])
def test_order_matches_brute_force(n, brick):
    rng = np.random.default_rng(n + brick)
    mean = (rng.normal(size=(3, n)) * [[3.0], [1.0], [0.2]]).astype(np.float32)
    mean[:, n // 3] = mean[:, 0]  # a duplicate: equal codes, index order
    idx = O.spatial_order(mean, brick)
    assert sorted(idx.tolist()) == list(range(n))
    assert idx.tolist() == _brute_order(mean, brick)


def test_bricks_are_compact_in_space():
    """Within a brick the Gaussians are neighbours: on a uniform cloud the
    mean spread of a 64-Gaussian brick is a fraction of the cloud's,
    while consecutive bricks start far apart."""
    rng = np.random.default_rng(3)
    n, brick = 64 * 400, 64
    mean = rng.uniform(0, 1, size=(3, n)).astype(np.float32)
    idx = O.spatial_order(mean, brick)
    m = mean[:, idx].reshape(3, n // brick, brick)
    spread = np.linalg.norm(m.std(axis=2), axis=0).mean()
    assert spread < 0.3 * np.linalg.norm(mean.std(axis=1))  # 64 random Gaussians: 1.0
    starts = m[:, :, 0]
    jump = np.linalg.norm(np.diff(starts, axis=1), axis=0).mean()
    assert jump > 0.3
