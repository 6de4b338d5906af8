"""The matrix-multiply formulation of the neighbour sums (Sec. 3.2: the
bidiagonal kernel matrix K and the four block equations for the sub-lattice
local sums of the black and white blocks), checked in numpy against the
plain four-neighbour stencil sum on a periodic lattice.

This pins the reading the MFMA kernels implement: blocks sigma_ab hold the
sites (2r + a, 2q + b) of a 256 x 256 sub-lattice, K has ones on the
diagonal and the first superdiagonal, and what the local products miss at a
sub-lattice edge is one term from the neighbouring sub-lattice.
"""
import numpy as np
import pytest

import workloads

B = 128  # block edge; a sub-lattice is 2B x 2B


def kernel_matrix(n=B):
    return np.eye(n, dtype=np.int64) + np.eye(n, k=1, dtype=np.int64)


def stencil(s):
    return np.roll(s, 1, 0) + np.roll(s, -1, 0) + np.roll(s, 1, 1) + np.roll(s, -1, 1)


def blocks(s):
    """(S, S, 2, 2, B, B): sub-lattice (I, J), block (a, b), element (r, q)."""
    L = s.shape[0]
    S = L // (2 * B)
    x = s.reshape(S, B, 2, S, B, 2)  # i = (I, r, a), j = (J, q, b)
    return x.transpose(0, 3, 2, 5, 1, 4)


def local_sums(sig):
    """The four block equations of the paper, per sub-lattice, before the
    boundary contributions: returns nn_L[a][b] for every block."""
    K = kernel_matrix()
    s00, s01, s10, s11 = sig[:, :, 0, 0], sig[:, :, 0, 1], sig[:, :, 1, 0], sig[:, :, 1, 1]
    nn = np.zeros_like(sig)
    nn[:, :, 0, 0] = s01 @ K + K.T @ s10      # black
    nn[:, :, 1, 1] = s10 @ K.T + K @ s01      # black
    nn[:, :, 1, 0] = s11 @ K + K @ s00        # white
    nn[:, :, 0, 1] = s00 @ K.T + K.T @ s11    # white
    return nn


def add_boundary(nn, sig):
    """The terms the local products miss: one neighbour from the adjacent
    sub-lattice along the row edge and along the column edge of each block."""
    left = np.roll(sig, 1, axis=1)   # sub-lattice (I, J - 1)
    right = np.roll(sig, -1, axis=1)  # (I, J + 1)
    up = np.roll(sig, 1, axis=0)     # (I - 1, J)
    down = np.roll(sig, -1, axis=0)  # (I + 1, J)
    out = nn.copy()
    for a in (0, 1):
        for b in (0, 1):
            # horizontal neighbours live in block (a, 1 - b)
            if b == 0:
                out[:, :, a, b, :, 0] += left[:, :, a, 1, :, B - 1]
            else:
                out[:, :, a, b, :, B - 1] += right[:, :, a, 0, :, 0]
            # vertical neighbours live in block (1 - a, b)
            if a == 0:
                out[:, :, a, b, 0, :] += up[:, :, 1, b, B - 1, :]
            else:
                out[:, :, a, b, B - 1, :] += down[:, :, 0, b, 0, :]
    return out


@pytest.mark.parametrize("L,seed", [(256, 1), (512, 2), (768, 3)])
def test_block_equations_equal_the_stencil(L, seed):
    s = workloads.random_spins(L, seed).astype(np.int64)
    sig = blocks(s)
    got = add_boundary(local_sums(sig), sig)
    assert np.array_equal(got, blocks(stencil(s)))


def test_local_products_alone_miss_exactly_the_edges():
    """Without the boundary step the sums differ from the stencil only on the
    one edge row and one edge column of each block, by one spin each."""
    L = 512
    s = workloads.random_spins(L, 5).astype(np.int64)
    sig = blocks(s)
    diff = blocks(stencil(s)) - local_sums(sig)
    assert np.all(np.abs(diff) <= 2)
    inner = diff[:, :, :, :, 1:B - 1, 1:B - 1]
    assert not inner.any()


def test_useful_fraction_of_the_products():
    """Every inner product of the 128 x 128 products has two nonzero terms
    (one at the first or last index): 2 / 128 = 1 / 64 of the dense flops."""
    K = kernel_matrix()
    assert K.sum() == 2 * B - 1
    assert np.all(K.sum(axis=0)[1:] == 2) and np.all(K.sum(axis=1)[:-1] == 2)
