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


RULES = {"metropolis": 0, "heatbath": 1}  # ISING_RULE_*


def thresholds(beta: float, J: float, rule: str = "metropolis") -> np.ndarray:
    T = (ctypes.c_uint64 * 5)()
    _lib.check(_lib.load().ising_thresholds_rule(float(beta), float(J), RULES[rule], T))
    return np.array(list(T), dtype=np.uint64)


def set_sweep_kernel(variant: int) -> None:
    """0 = default (by size), 1 = general-geometry kernel, 2 = row kernel without work
    queue, 3, 4, 5 = queued row kernel with 32-, 16-, 8-row bands at every row-aligned
    size."""
    _lib.check(_lib.load().ising_set_sweep_kernel(int(variant)))


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


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
              stream=None, rule: str = "metropolis") -> None:
        """nsweeps checkerboard sweeps under the Metropolis or heat-bath rule."""
        _lib.check(_lib.load().ising_sweep_rule(ctypes.byref(self.desc), float(beta), float(J),
                                                RULES[rule], int(nsweeps), int(rng_counter),
                                                _stream_handle(stream)))

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

    # ------------------------------------------------------ +-J spin glass
    def glass_sweep(self, bonds: "GlassBonds", beta: float, J: float = 1.0, nsweeps: int = 1,
                    rng_counter: int = 0, stream=None) -> None:
        """Metropolis sweeps with the bond signs of `bonds` (L % 128 == 0)."""
        _lib.check(_lib.load().ising_glass_sweep(
            ctypes.byref(self.desc), ctypes.c_void_p(bonds.words.data_ptr()), bonds.nbytes,
            float(beta), float(J), int(nsweeps), int(rng_counter), _stream_handle(stream)))

    def glass_observables(self, bonds: "GlassBonds", stream=None) -> tuple:
        """(bond sum with the bond signs, M)."""
        out = torch.empty(2, dtype=torch.int64, device=self.words.device)
        p = out.data_ptr()
        _lib.check(_lib.load().ising_glass_observables(
            ctypes.byref(self.desc), ctypes.c_void_p(bonds.words.data_ptr()), bonds.nbytes,
            ctypes.c_void_p(p), ctypes.c_void_p(p + 8), _stream_handle(stream)))
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


class MatmulLattice:
    """The matrix-multiply formulation of the sweep (fp16 spins in 256 x 256
    sub-lattices of four 128 x 128 blocks; L % 256 == 0), started from the
    bit-packed lattice `lat` (same L, seed and stream).  `fused` picks the
    one-kernel form; otherwise the products, boundary and update kernels run
    with the sums in HBM."""

    def __init__(self, lat: Lattice, fused: bool = True, stream=None):
        lib = _lib.load()
        self.L, self.seed, self.stream_id = lat.L, lat.seed, lat.stream_id
        nb = lib.ising_mm_lattice_bytes(self.L)
        if nb < 0:
            raise ValueError(f"unsupported lattice size {self.L} (L % 256 == 0 needed)")
        dev = lat.words.device
        self.spins = torch.empty(nb // 2, dtype=torch.int16, device=dev)
        self.fused = bool(fused)
        self.sums = (None if self.fused else
                     torch.empty(lib.ising_mm_sums_bytes(self.L) // 2, dtype=torch.int16, device=dev))
        _lib.check(lib.ising_mm_from_words(ctypes.byref(lat.desc), _ptr(self.spins), nb,
                                           _stream_handle(stream)))

    def sweep(self, beta: float, J: float = 1.0, nsweeps: int = 1, rng_counter: int = 0,
              stream=None) -> None:
        sums = self.sums
        _lib.check(_lib.load().ising_mm_sweep(
            self.L, self.seed, self.stream_id, _ptr(self.spins), self.spins.numel() * 2,
            _ptr(sums) if sums is not None else None, sums.numel() * 2 if sums is not None else 0,
            float(beta), float(J), int(nsweeps), int(rng_counter), int(self.fused),
            _stream_handle(stream)))

    def to_lattice(self, lat: Lattice, stream=None) -> None:
        """Writes the spins into the bit-packed lattice `lat` (same L)."""
        _lib.check(_lib.load().ising_mm_to_words(ctypes.byref(lat.desc), _ptr(self.spins),
                                                 self.spins.numel() * 2, _stream_handle(stream)))


def batch_words(Ls) -> int:
    arr = (ctypes.c_int64 * len(Ls))(*[int(x) for x in Ls])
    n = _lib.load().ising_batch_words(len(Ls), arr)
    if n < 0:
        raise ValueError("unsupported lattice size in batch")
    return int(n)


class GlassBonds:
    """Bond signs of a +-J spin glass on an L x L lattice (device tensor of
    4 * words_per_colour(L) words: right bonds of colour 0, 1, down bonds of
    colour 0, 1, interleaved word by word, word k of array x at 4 k + x; bit
    1 = coupling -J)."""

    def __init__(self, L: int, seed: int = None, stream_id: int = 0, right=None, down=None,
                 stream=None):
        self.L = int(L)
        W = words_per_colour(self.L)
        self.words = torch.zeros(4 * W, dtype=torch.int64, device="cuda")
        self.nbytes = 4 * W * 8
        ptr = ctypes.c_void_p(self.words.data_ptr())
        if right is not None:
            r = np.ascontiguousarray(right, dtype=np.int8)
            d = np.ascontiguousarray(down, dtype=np.int8)
            _lib.check(_lib.load().ising_glass_set_bonds(
                ptr, self.nbytes, self.L, r.ctypes.data_as(ctypes.c_void_p),
                d.ctypes.data_as(ctypes.c_void_p), _stream_handle(stream)))
        else:
            _lib.check(_lib.load().ising_glass_bonds_init(ptr, self.nbytes, self.L, int(seed),
                                                          int(stream_id), _stream_handle(stream)))


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

    def observables_async(self, stream=None, out=None):
        """Device tensors (bond[n], M[n]); E_q = -J * bond[q].  `out`, if
        given, is a contiguous int64 device tensor of shape (2, n) to fill."""
        if out is None:
            out = torch.empty((2, self.n), dtype=torch.int64, device=self.words.device)
        assert out.dtype == torch.int64 and out.is_contiguous() and out.shape == (2, self.n)
        _lib.check(_lib.load().ising_batch_observables(
            self._h, ctypes.c_void_p(out[0].data_ptr()), ctypes.c_void_p(out[1].data_ptr()),
            _stream_handle(stream)))
        return out

    def observables(self, stream=None):
        out = self.observables_async(stream).cpu().numpy()
        return out[0], out[1]

    def spins(self, out=None, stream=None):
        """Every lattice as int8 +1/-1 rasters, concatenated (device tensor)."""
        n = sum(L * L for L in self.Ls)
        if out is None:
            out = torch.empty(n, dtype=torch.int8, device=self.words.device)
        _lib.check(_lib.load().ising_batch_get_spins_dev(self._h, _ptr(out), _stream_handle(stream)))
        return out

    def set_spins(self, spins, stream=None) -> None:
        _lib.check(_lib.load().ising_batch_set_spins_dev(self._h, _ptr(spins),
                                                         _stream_handle(stream)))

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

    def plan(self, L: int) -> tuple:
        """(lattices per workgroup, workgroups) of the lattices of size L."""
        per, n = ctypes.c_uint32(), ctypes.c_uint32()
        _lib.check(_lib.load().ising_batch_get_plan(self._h, int(L), ctypes.byref(per),
                                                    ctypes.byref(n)))
        return int(per.value), int(n.value)

    def mixed(self) -> bool:
        """True if the current plan has bundles that mix lattice sizes."""
        v = ctypes.c_int32()
        _lib.check(_lib.load().ising_batch_get_mixed(self._h, ctypes.byref(v)))
        return bool(v.value)

    def set_bundles(self, bundles) -> None:
        """Explicit plan: a list of lists of lattice indices, one list per
        workgroup load, in launch order (every lattice exactly once)."""
        counts = [len(g) for g in bundles]
        flat = [int(q) for g in bundles for q in g]
        c_arr = (ctypes.c_int32 * len(counts))(*counts)
        l_arr = (ctypes.c_int32 * max(1, len(flat)))(*flat)
        _lib.check(_lib.load().ising_batch_set_bundles(self._h, len(counts), c_arr, l_arr))

    def set_tiles(self, L: int, wpt: int, lpw: int = 1) -> None:
        _lib.check(_lib.load().ising_batch_set_tiles(self._h, int(L), int(wpt), int(lpw)))

    def autotune(self, tune_sweeps: int = 20, cache_path=None, stream=None) -> dict:
        path = cache_path.encode() if cache_path else None
        _lib.check(_lib.load().ising_batch_autotune(self._h, int(tune_sweeps), path,
                                                    _stream_handle(stream)))
        return {L: self.tiles(L) for L in sorted(set(self.Ls))}



def arnet_num_params(channels: int) -> int:
    n = _lib.load().ising_arnet_num_params(int(channels))
    if n < 0:
        raise ValueError("channels must be 32 or 64")
    return int(n)


def batch_sweep_noalloc(Ls, betas, J: float, seeds, stream_ids, words, nsweeps: int,
                        rng_counter: int, stream=None) -> None:
    """Advance the lattices in `words` (laid out as a Batch of the same
    lattices) by nsweeps from sweep counter rng_counter, without any
    allocation by the library (ising_batch_sweep_noalloc)."""
    n = len(Ls)
    assert words.dtype == torch.int64 and words.is_contiguous()
    L_arr = (ctypes.c_int64 * n)(*[int(x) for x in Ls])
    b_arr = (ctypes.c_double * n)(*[float(x) for x in betas])
    s_arr = (ctypes.c_uint64 * n)(*[int(x) for x in seeds])
    i_arr = (ctypes.c_uint32 * n)(*[int(x) for x in stream_ids])
    _lib.check(_lib.load().ising_batch_sweep_noalloc(
        n, L_arr, b_arr, float(J), s_arr, i_arr, ctypes.c_void_p(words.data_ptr()),
        words.numel() * 8, int(nsweeps), int(rng_counter), _stream_handle(stream)))


class ARNet:
    """The learned global proposal: a masked-convolution autoregressive network
    over L x L configurations (int8 +1/-1 device tensors of shape (B, L, L))."""

    def __init__(self, L: int, channels: int, max_batch: int, device="cuda"):
        self.L, self.C, self.max_batch = int(L), int(channels), int(max_batch)
        self.device = torch.device(device)
        self.P = arnet_num_params(self.C)
        self._h = ctypes.c_void_p()
        _lib.check(_lib.load().ising_arnet_create(ctypes.byref(self._h), self.L, self.C,
                                                  self.max_batch))

    def close(self) -> None:
        if self._h:
            _lib.load().ising_arnet_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params, stream=None) -> None:
        t = torch.as_tensor(params, dtype=torch.float32).to(self.device).contiguous()
        assert t.numel() == self.P
        _lib.check(_lib.load().ising_arnet_set_params(self._h, _ptr(t), _stream_handle(stream)))
        self._keep = t  # the copy is stream-ordered; keep the source alive

    def params(self, stream=None):
        out = torch.empty(self.P, dtype=torch.float32, device=self.device)
        _lib.check(_lib.load().ising_arnet_get_params(self._h, _ptr(out), _stream_handle(stream)))
        return out

    def _check_spins(self, spins):
        assert spins.dtype == torch.int8 and spins.is_contiguous()
        assert spins.numel() % (self.L * self.L) == 0
        return spins.numel() // (self.L * self.L)

    EVAL_MODES = {"auto": 0, "layers": 1}  # ISING_ARNET_EVAL_*

    def set_eval_mode(self, mode: str) -> None:
        """'auto': the on-chip evaluator where its LDS fits (the default);
        'layers': one launch per layer always."""
        _lib.check(_lib.load().ising_arnet_set_eval_mode(self._h, self.EVAL_MODES[mode]))

    def log_prob(self, spins, logits=False, stream=None, out=None):
        B = self._check_spins(spins)
        logq = torch.empty(B, dtype=torch.float32, device=self.device) if out is None else out
        assert logq.dtype == torch.float32 and logq.is_contiguous() and logq.numel() == B
        lg = torch.empty((B, self.L, self.L), dtype=torch.float32, device=self.device) if logits else None
        _lib.check(_lib.load().ising_arnet_log_prob(self._h, _ptr(spins), B, _ptr(logq),
                                                    _ptr(lg) if logits else None,
                                                    _stream_handle(stream)))
        return (logq, lg) if logits else logq

    def gradient(self, spins, stream=None):
        B = self._check_spins(spins)
        grad = torch.empty(self.P, dtype=torch.float32, device=self.device)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        _lib.check(_lib.load().ising_arnet_gradient(self._h, _ptr(spins), B, _ptr(grad), _ptr(loss),
                                                    _stream_handle(stream)))
        return loss, grad

    def gradient_at(self, spins, acts, logits, stream=None):
        """(loss, gradient) of the backward pass at given forward values:
        acts a bfloat16 device tensor [5, B, L, L, C] (layers 1..5, post-ReLU),
        logits a float32 device tensor [B, L, L]."""
        B = self._check_spins(spins)
        assert acts.dtype == torch.bfloat16 and acts.is_contiguous()
        assert acts.numel() == 5 * B * self.L * self.L * self.C
        assert logits.dtype == torch.float32 and logits.is_contiguous()
        assert logits.numel() == B * self.L * self.L
        grad = torch.empty(self.P, dtype=torch.float32, device=self.device)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        _lib.check(_lib.load().ising_arnet_gradient_at(self._h, _ptr(spins), B, _ptr(acts),
                                                       _ptr(logits), _ptr(grad), _ptr(loss),
                                                       _stream_handle(stream)))
        return loss, grad

    def train_step(self, spins, lr: float, loss=None, stream=None):
        B = self._check_spins(spins)
        if loss is None:
            loss = torch.empty(1, dtype=torch.float32, device=self.device)
        _lib.check(_lib.load().ising_arnet_train_step(self._h, _ptr(spins), B, float(lr), _ptr(loss),
                                                      _stream_handle(stream)))
        return loss

    def adam(self, grad, lr: float, stream=None) -> None:
        """One Adam step on the master parameters with a caller's gradient
        (device float32 tensor of num_params entries)."""
        assert grad.dtype == torch.float32 and grad.is_contiguous() and grad.numel() == self.P
        _lib.check(_lib.load().ising_arnet_adam(self._h, _ptr(grad), float(lr), _stream_handle(stream)))

    def sample(self, B: int, seed: int, stream_base: int = 0, round: int = 0, out=None,
               logq=None, stream=None):
        if out is None:
            out = torch.empty((B, self.L, self.L), dtype=torch.int8, device=self.device)
        if logq is None:
            logq = torch.empty(B, dtype=torch.float32, device=self.device)
        _lib.check(_lib.load().ising_arnet_sample(self._h, int(B), int(seed), int(stream_base),
                                                  int(round), _ptr(out), _ptr(logq),
                                                  _stream_handle(stream)))
        return out, logq


def spins_minibatch(pool, B: int, seed: int, stream_base: int = 0, round: int = 0, out=None,
                    stream=None):
    """B configurations drawn from `pool` (int8 device tensor (P, L, L)), each
    flipped and translated at random (ising_spins_minibatch)."""
    P, L = int(pool.shape[0]), int(pool.shape[1])
    assert pool.dtype == torch.int8 and pool.is_contiguous()
    if out is None:
        out = torch.empty((B, L, L), dtype=torch.int8, device=pool.device)
    _lib.check(_lib.load().ising_spins_minibatch(_ptr(pool), P, L, int(B), int(seed),
                                                 int(stream_base), int(round), _ptr(out),
                                                 _stream_handle(stream)))
    return out


def spins_observables(spins, L: int, stream=None, bond=None, mag=None):
    """(bond, M) device int64 tensors of int8 configurations of shape (B, L, L)
    (into `bond` and `mag` if given)."""
    B = spins.numel() // (L * L)
    if bond is None:
        bond = torch.empty(B, dtype=torch.int64, device=spins.device)
    if mag is None:
        mag = torch.empty(B, dtype=torch.int64, device=spins.device)
    assert bond.is_contiguous() and mag.is_contiguous() and bond.numel() == mag.numel() == B
    _lib.check(_lib.load().ising_spins_observables(_ptr(spins), B, int(L), _ptr(bond), _ptr(mag),
                                                   _stream_handle(stream)))
    return bond, mag


def mh_independence(state, logq, bond, prop, logq_prop, bond_prop, betaJ, seed: int,
                    stream_base: int, round: int, accepted=None, stream=None):
    """Independence Metropolis-Hastings step on n chains (in place)."""
    n = logq.numel()
    L = int(round_sqrt(state.numel() // n))
    if accepted is None:
        accepted = torch.empty(n, dtype=torch.int32, device=state.device)
    _lib.check(_lib.load().ising_mh_independence(
        n, L, _ptr(state), _ptr(logq), _ptr(bond), _ptr(prop), _ptr(logq_prop), _ptr(bond_prop),
        _ptr(betaJ), int(seed), int(stream_base), int(round), _ptr(accepted),
        _stream_handle(stream)))
    return accepted


def round_sqrt(n: int) -> int:
    r = int(np.sqrt(n) + 0.5)
    assert r * r == n
    return r
