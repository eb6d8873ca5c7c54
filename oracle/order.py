"""Reference definition of the spatial storage order of a Gaussian map.

TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers; the product path never imports it.

The paper fixes no storage order for the map: every quantity of the method is
a sum or a product over Gaussians that does not depend on where a Gaussian is
stored, except the tie-break of equal depths in the depth-ordered sets N(p)
of Eq. (alpha), which goes by index.  The order is therefore a layout choice
of this implementation, defined here in full so that the GPU's permutation can
be checked exactly.  For n Gaussians with float32 means [3][n] and a brick
size B >= 1:

  1. box: lo_a and hi_a, the least and greatest coordinate a over the
     Gaussians whose three coordinates are finite; w = max over a of
     (hi_a - lo_a), in double;
  2. cells: when w > 0, with w = m 2^e and m in [0.5, 1),
     q_a = min(1023, floor((x_a - lo_a) 2^(10 - e))) in double (cubic cells of
     side 2^e / 1024); when w = 0 (or no Gaussian is finite) every q_a = 0;
  3. code: the bits of q_x, q_y, q_z interleaved (bit k of q_x at bit 3k, of
     q_y at 3k + 1, of q_z at 3k + 2), a Morton code below 2^30; a Gaussian
     with a non-finite coordinate takes 2^30;
  4. rank: place in the ascending order of (code, index);
  5. bricks: F = floor(n / B) full bricks of B consecutive ranks.  Position
     j B + k (j < F, k < B) holds the Gaussian of rank ((j P) mod F) B + k,
     with P the least integer >= max(1, floor(0.618... F + 0.5)) such that
     gcd(P, F) = 1 (so j -> j P mod F is a bijection of the bricks, and
     consecutive positions take bricks about 0.618 F apart in the curve's
     order); positions from F B on hold the Gaussian of the same rank;
  6. index[position] = that Gaussian.

Within a brick the Gaussians are neighbours in space; consecutive bricks come
from distant parts of the map.  B >= n gives the plain Morton order.
"""
import math

import numpy as np

GOLDEN = 0.6180339887498949
CELL_BITS = 10
NONFINITE_CODE = 1 << 30


def box(mean):
    """(lo[3], w): the finite Gaussians' least coordinates and the largest
    extent over the three axes (step 1); (None, 0.0) when none is finite."""
    mean = np.asarray(mean, dtype=np.float32)
    fin = np.all(np.isfinite(mean), axis=0)
    if not fin.any():
        return None, 0.0
    m = mean[:, fin].astype(np.float64)
    lo = m.min(axis=1)
    hi = m.max(axis=1)
    return lo, float(np.max(hi - lo))


def cells(mean):
    """Integer cell coordinates q [3][n] (step 2) and the finite mask."""
    mean = np.asarray(mean, dtype=np.float32)
    n = mean.shape[1]
    fin = np.all(np.isfinite(mean), axis=0)
    q = np.zeros((3, n), dtype=np.int64)
    lo, w = box(mean)
    if lo is None or w == 0.0:
        return q, fin
    _, e = math.frexp(w)
    scale = math.ldexp(1.0, CELL_BITS - e)
    for a in range(3):
        x = mean[a, fin].astype(np.float64)
        t = np.floor((x - lo[a]) * scale)
        q[a, fin] = np.minimum((1 << CELL_BITS) - 1, t.astype(np.int64))
    return q, fin


def interleave(q):
    """Morton code of cell coordinates q [3][n] (step 3), bit by bit."""
    q = np.asarray(q, dtype=np.int64)
    code = np.zeros(q.shape[1], dtype=np.int64)
    for k in range(CELL_BITS):
        for a in range(3):
            code |= ((q[a] >> k) & 1) << (3 * k + a)
    return code


def codes(mean):
    q, fin = cells(mean)
    code = interleave(q)
    code[~fin] = NONFINITE_CODE
    return code


def brick_multiplier(full):
    """P of step 5 for F = full bricks."""
    if full <= 1:
        return 1
    p = max(1, int(math.floor(GOLDEN * full + 0.5)))
    while math.gcd(p, full) != 1:
        p += 1
    return p


def spatial_order(mean, brick):
    """index [n] (int64): the Gaussian stored at each position (steps 1-6)."""
    mean = np.asarray(mean, dtype=np.float32)
    n = mean.shape[1]
    if brick < 1:
        raise ValueError("brick must be at least 1")
    code = codes(mean)
    by_rank = np.lexsort((np.arange(n), code))  # step 4: Gaussian of each rank
    full = n // brick
    p = brick_multiplier(full)
    pos = np.arange(n, dtype=np.int64)
    rank = pos.copy()  # step 5: the rank each position takes
    inb = pos < full * brick
    if full > 0:
        rank[inb] = ((pos[inb] // brick) * p % full) * brick + pos[inb] % brick
    return by_rank[rank]
