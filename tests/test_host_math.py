"""Integer identities the kernels rely on, checked exhaustively on the host.

The subfield passes of an image whose state is in LDS take the row of a word
index (below 2^16, rows of WW <= 1024 words) as the high half of
index * (floor((2^32 - 1) / WW) + 1), with WW = 1 handled as the index itself.
"""
import numpy as np


def test_row_of_word_index_by_multiply_high():
    idx = np.arange(1 << 16, dtype=np.uint64)
    for WW in range(1, 1025):
        if WW == 1:
            continue
        m = np.uint64((0xFFFFFFFF // WW + 1) & 0xFFFFFFFF)
        assert np.array_equal((idx * m) >> np.uint64(32), idx // np.uint64(WW)), WW
