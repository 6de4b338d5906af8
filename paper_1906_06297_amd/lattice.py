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
        if words is _VIEW:  # internal: wraps an existing descriptor, see view()
            return
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

    @classmethod
    def view(cls, desc, words):
        """A lattice over an existing descriptor (no initialisation); `words`
        is the tensor that owns the memory."""
        obj = cls(0, 0, words=_VIEW)
        obj.desc = desc
        obj.L = int(desc.L)
        obj.words = words
        obj._base = int(desc.words)
        return obj

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
        off = (getattr(self, "_base", self.words.data_ptr()) - self.words.data_ptr()) // 8
        return self.words[off: off + 2 * W].cpu().numpy().view(np.uint64).reshape(2, W)


_VIEW = object()


def batch_words(Ls) -> int:
    arr = (ctypes.c_int64 * len(Ls))(*[int(x) for x in Ls])
    n = _lib.load().ising_batch_words(len(Ls), arr)
    if n < 0:
        raise ValueError("unsupported lattice size in batch")
    return int(n)


class Batch:
    """Independent lattices advanced together by the persistent batch kernel.

    ``words`` is one torch int64 tensor holding every lattice back to back.
    The batch keeps its own sweep counter on the device; consecutive sweep()
    calls continue every chain.
    """

    def __init__(self, Ls, betas, J: float, seeds, stream_ids, device="cuda"):
        n = len(Ls)
        self.n = n
        self.Ls = [int(x) for x in Ls]
        self.J = float(J)
        self.words = torch.zeros(batch_words(self.Ls), dtype=torch.int64, device=device)
        self._h = ctypes.c_void_p()
        L_arr = (ctypes.c_int64 * n)(*self.Ls)
        b_arr = (ctypes.c_double * n)(*[float(x) for x in betas])
        s_arr = (ctypes.c_uint64 * n)(*[int(x) for x in seeds])
        i_arr = (ctypes.c_uint32 * n)(*[int(x) for x in stream_ids])
        _lib.check(_lib.load().ising_batch_create(
            ctypes.byref(self._h), n, L_arr, b_arr, float(J), s_arr, i_arr,
            ctypes.c_void_p(self.words.data_ptr()), self.words.numel() * 8))

    def close(self) -> None:
        if self._h:
            _lib.load().ising_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init(self, stream=None) -> None:
        _lib.check(_lib.load().ising_batch_init(self._h, _stream_handle(stream)))

    def sweep(self, nsweeps: int, stream=None) -> None:
        _lib.check(_lib.load().ising_batch_sweep(self._h, int(nsweeps), _stream_handle(stream)))

    def set_counter(self, value: int, stream=None) -> None:
        _lib.check(_lib.load().ising_batch_set_counter(self._h, int(value), _stream_handle(stream)))

    def counter(self, stream=None) -> int:
        v = ctypes.c_uint64()
        _lib.check(_lib.load().ising_batch_get_counter(self._h, ctypes.byref(v),
                                                       _stream_handle(stream)))
        return int(v.value)

    def observables_async(self, stream=None):
        """Device tensors (bond[n], M[n]); E_q = -J * bond[q]."""
        out = torch.empty((2, self.n), dtype=torch.int64, device=self.words.device)
        _lib.check(_lib.load().ising_batch_observables(
            self._h, ctypes.c_void_p(out[0].data_ptr()), ctypes.c_void_p(out[1].data_ptr()),
            _stream_handle(stream)))
        return out

    def observables(self, stream=None):
        out = self.observables_async(stream).cpu().numpy()
        return out[0], out[1]

    def lattice(self, q: int) -> "Lattice":
        desc = _lib.LatticeStruct()
        _lib.check(_lib.load().ising_batch_lattice(self._h, int(q), ctypes.byref(desc)))
        return Lattice.view(desc, self.words)

    def tiles(self, L: int) -> tuple:
        """(words per lane group, lanes per word) for lattices of size L."""
        w, l = ctypes.c_uint32(), ctypes.c_uint32()
        _lib.check(_lib.load().ising_batch_get_tiles(self._h, int(L), ctypes.byref(w),
                                                     ctypes.byref(l)))
        return int(w.value), int(l.value)

    def set_tiles(self, L: int, wpt: int, lpw: int = 1) -> None:
        _lib.check(_lib.load().ising_batch_set_tiles(self._h, int(L), int(wpt), int(lpw)))

    def autotune(self, tune_sweeps: int = 20, cache_path=None, stream=None) -> dict:
        path = cache_path.encode() if cache_path else None
        _lib.check(_lib.load().ising_batch_autotune(self._h, int(tune_sweeps), path,
                                                    _stream_handle(stream)))
        return {L: self.tiles(L) for L in sorted(set(self.Ls))}
