"""Python face of libising: a lattice in device memory and the calls on it.

PyTorch provides the device memory (a flat int64 tensor holding both colours'
bit-packed words) and the stream (torch's current stream); every computation
is a call through the C ABI.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib


def words_per_colour(L: int) -> int:
    w = _lib.load().ising_words_per_colour(int(L))
    if w < 0:
        raise ValueError(f"unsupported lattice size {L}")
    return int(w)


def thresholds(beta: float, J: float) -> np.ndarray:
    T = (ctypes.c_uint64 * 5)()
    _lib.check(_lib.load().ising_thresholds(float(beta), float(J), T))
    return np.array(list(T), dtype=np.uint64)


def set_sweep_kernel(variant: int) -> None:
    """0 = default, 1 = general-geometry kernel, 2 = row kernel without work queue."""
    _lib.check(_lib.load().ising_set_sweep_kernel(int(variant)))


def _stream_handle(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Lattice:
    """An L x L periodic lattice, 1 bit per spin, on a HIP device.

    ``words`` is a torch int64 tensor of 2 * words_per_colour(L) words: colour 0
    (black, (i+j) even) then colour 1, each the colour-linear bit string of its
    spins.
    """

    def __init__(self, L: int, seed: int, stream_id: int = 0, device="cuda", words=None,
                 stream=None):
        self.L = int(L)
        W = words_per_colour(self.L)
        if words is None:
            words = torch.empty(2 * W, dtype=torch.int64, device=device)
        if words.dtype != torch.int64 or words.numel() < 2 * W or not words.is_cuda:
            raise ValueError("words must be a CUDA int64 tensor of at least 2*W elements")
        self.words = words
        self.desc = _lib.LatticeStruct()
        _lib.check(_lib.load().ising_init(ctypes.byref(self.desc), ctypes.c_void_p(words.data_ptr()),
                                          words.numel() * 8, self.L, int(seed), int(stream_id),
                                          _stream_handle(stream)))

    @property
    def seed(self) -> int:
        return int(self.desc.seed)

    @property
    def stream_id(self) -> int:
        return int(self.desc.stream_id)

    def sweep(self, beta: float, J: float = 1.0, nsweeps: int = 1, rng_counter: int = 0,
              stream=None) -> None:
        _lib.check(_lib.load().ising_sweep(ctypes.byref(self.desc), float(beta), float(J),
                                           int(nsweeps), int(rng_counter), _stream_handle(stream)))

    def sweep_traced(self, beta: float, J: float = 1.0, nsweeps: int = 1, rng_counter: int = 0,
                     bond=None, mag=None, stream=None):
        """Sweeps with per-sweep (bond sum, magnetisation) written to device tensors."""
        dev = self.words.device
        if bond is None:
            bond = torch.empty(int(nsweeps), dtype=torch.int64, device=dev)
        if mag is None:
            mag = torch.empty(int(nsweeps), dtype=torch.int64, device=dev)
        _lib.check(_lib.load().ising_sweep_traced(
            ctypes.byref(self.desc), float(beta), float(J), int(nsweeps), int(rng_counter),
            ctypes.c_void_p(bond.data_ptr()), ctypes.c_void_p(mag.data_ptr()),
            _stream_handle(stream)))
        return bond, mag

    def observables_async(self, out=None, stream=None) -> torch.Tensor:
        """Device tensor [bond_sum, M] (energy E = -J * bond_sum)."""
        if out is None:
            out = torch.empty(2, dtype=torch.int64, device=self.words.device)
        p = out.data_ptr()
        _lib.check(_lib.load().ising_observables(ctypes.byref(self.desc), ctypes.c_void_p(p),
                                                 ctypes.c_void_p(p + 8), _stream_handle(stream)))
        return out

    def observables(self, stream=None) -> tuple:
        out = self.observables_async(stream=stream)
        b, m = out.cpu().tolist()
        return int(b), int(m)

    def get_spins(self, stream=None) -> np.ndarray:
        out = np.empty((self.L, self.L), dtype=np.int8)
        _lib.check(_lib.load().ising_get_spins(ctypes.byref(self.desc),
                                               out.ctypes.data_as(ctypes.c_void_p),
                                               _stream_handle(stream)))
        return out

    def set_spins(self, spins: np.ndarray, stream=None) -> None:
        s = np.ascontiguousarray(spins, dtype=np.int8)
        if s.shape != (self.L, self.L):
            raise ValueError("spins must be L x L")
        _lib.check(_lib.load().ising_set_spins(ctypes.byref(self.desc),
                                               s.ctypes.data_as(ctypes.c_void_p),
                                               _stream_handle(stream)))

    def packed(self) -> np.ndarray:
        """Host copy of the packed words as uint64 (2, words_per_colour)."""
        W = words_per_colour(self.L)
        return self.words[: 2 * W].cpu().numpy().view(np.uint64).reshape(2, W)
