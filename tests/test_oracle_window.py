"""The oracle's windowed evolution (used to check large lattices on sampled
blocks) against its full-lattice sweep, including windows across the
periodic seams."""
import numpy as np
import pytest


@pytest.mark.parametrize("L,n", [(64, 3), (128, 2), (48, 1)])
def test_window_inner_sites_are_exact(orc, L, n):
    seed, stream, beta = 13, 2, 0.44
    full = orc.init(L, seed, stream)
    orc.sweeps(full, beta, 1.0, seed, stream, n, 5)
    margin = 2 * n + 1
    for (ci, cj) in [(0, 0), (L - 8, L - 8), (10, L - 3), (L // 2, 7)]:
        blk = 16
        i0, j0 = ci - margin, cj - margin
        win = orc.window_init(L, i0, j0, blk + 2 * margin, blk + 2 * margin, seed, stream)
        rows = (np.arange(blk + 2 * margin) + i0) % L
        cols = (np.arange(blk + 2 * margin) + j0) % L
        assert np.array_equal(win, orc.init(L, seed, stream)[np.ix_(rows, cols)])
        orc.window_sweeps(win, L, i0, j0, beta, 1.0, seed, stream, n, 5)
        inner = win[margin:margin + blk, margin:margin + blk]
        assert np.array_equal(inner, full[np.ix_(rows[margin:margin + blk], cols[margin:margin + blk])])
