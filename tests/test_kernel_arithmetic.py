"""Integer arithmetic the kernels rely on, checked exhaustively on the CPU.

The voxel search decodes a tile's brick-box entry e into box coordinates with two divisions
by the box extents, done as a multiply-high by m = floor((2^32 - 1) / d) + 1 (m = 0 and no
division for d = 1). Entries stay below 2,048 and extents at most 2,048, the largest box the
LDS holds; this checks that the quotient is exact over that whole range."""
import numpy as np


def test_multiply_high_division_is_exact_for_box_entries():
    a = np.arange(2048, dtype=np.uint64)
    for d in range(1, 2049):
        if d == 1:
            q = a
        else:
            m = np.uint64((0xFFFFFFFF // d) + 1)
            assert m < 2**32
            q = (a * m) >> np.uint64(32)
        assert np.array_equal(q, a // np.uint64(d)), d
