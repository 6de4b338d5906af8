"""Test helper: the packed layout of include/ising.h restated in numpy, to
compare the GPU's words with the oracle's int8 lattices.  Colour c holds its
L*L/2 spins in colour-linear order n = i*(L/2) + j//2 (site (i, j) with
(i + j) & 1 == c), bit n & 63 of word n >> 6, bit 1 for spin +1."""
import numpy as np


def colour_sites(L: int, c: int):
    i = np.repeat(np.arange(L), L // 2)
    jc = np.tile(np.arange(L // 2), L)
    j = 2 * jc + ((i + c) & 1)
    return i, j


def pack(spins: np.ndarray) -> np.ndarray:
    """(2, words_per_colour) uint64 words of an L x L +/-1 lattice."""
    L = spins.shape[0]
    M = L * L // 2
    W = (M + 63) // 64
    out = np.zeros((2, W), dtype=np.uint64)
    for c in (0, 1):
        i, j = colour_sites(L, c)
        bits = np.zeros(W * 64, dtype=np.uint8)
        bits[:M] = spins[i, j] > 0
        out[c] = np.packbits(bits, bitorder="little").view(np.uint64)
    return out


def unpack(words: np.ndarray, L: int) -> np.ndarray:
    M = L * L // 2
    s = np.empty((L, L), dtype=np.int8)
    for c in (0, 1):
        bits = np.unpackbits(words[c].view(np.uint8), bitorder="little")[:M]
        i, j = colour_sites(L, c)
        s[i, j] = np.where(bits == 1, 1, -1)
    return s


def pack_rows(spins: np.ndarray) -> np.ndarray:
    """pack() for row-aligned sizes (L % 128 == 0) by strided row slices, without
    index arrays: colour c of row i is spins[i, (i + c) % 2 :: 2]."""
    L = spins.shape[0]
    assert L % 128 == 0
    up = spins > 0
    out = np.empty((2, L * L // 128), dtype=np.uint64)
    for c in (0, 1):
        col = np.empty((L, L // 2), dtype=bool)
        col[0::2] = up[0::2, c::2]
        col[1::2] = up[1::2, (1 - c)::2]
        out[c] = np.packbits(col, axis=1, bitorder="little").view(np.uint64).reshape(-1)
        del col
    return out
