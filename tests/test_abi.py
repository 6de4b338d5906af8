"""The C ABI library: loads without a GPU, exports every symbol that
include/ising.h declares, validates arguments before touching the device,
and builds the same threshold table as the oracle."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "ising.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ising_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1906_06297_amd import _lib

    return _lib.load()


def test_exports_every_declared_symbol(lib):
    names = header_functions()
    assert "ising_sweep" in names and "ising_init" in names and "ising_observables" in names
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_header(lib):
    from paper_1906_06297_amd import _lib

    assert set(header_functions()) <= set(_lib.SIGNATURES)


def test_words_per_colour(lib):
    assert lib.ising_words_per_colour(4) == 1
    assert lib.ising_words_per_colour(24) == 5  # 288 spins per colour
    assert lib.ising_words_per_colour(64) == 32
    assert lib.ising_words_per_colour(65536) == 1 << 25
    for bad in (0, 2, 3, 63, -8, 741456):
        assert lib.ising_words_per_colour(bad) == -1


def test_thresholds_match_oracle(lib, orc):
    from paper_1906_06297_amd import thresholds

    for J in (1.0, -1.0, 0.5, 0.0):
        for beta in [0.0, 0.3, workloads.BETA_CRIT_CONFIG, 0.5, 7.0] + list(np.linspace(0.3, 0.6, 32)):
            assert np.array_equal(thresholds(beta, J), orc.thresholds(beta, J)), (beta, J)


def test_heatbath_thresholds_match_oracle(lib, orc):
    from paper_1906_06297_amd import thresholds

    for J in (1.0, -1.0, 0.5, 0.0):
        for beta in [0.0, 0.3, workloads.BETA_CRIT_CONFIG, 0.5, 7.0, 300.0] + list(np.linspace(0.3, 0.6, 32)):
            assert np.array_equal(thresholds(beta, J, "heatbath"), orc.thresholds(beta, J, "heatbath")), (beta, J)


def test_rule_argument_errors(lib):
    from paper_1906_06297_amd import _lib

    T = (ctypes.c_uint64 * 5)()
    assert lib.ising_thresholds_rule(0.4, 1.0, 2, T) == _lib.ISING_E_BADARG
    assert b"rule" in lib.ising_last_error()
    assert lib.ising_thresholds_rule(-0.1, 1.0, 1, T) == _lib.ISING_E_BADARG
    assert lib.ising_thresholds_rule(0.4, 1.0, 1, None) == _lib.ISING_E_BADARG
    good = _lib.LatticeStruct(words=0x1000, L=8, seed=1, stream_id=0)
    assert lib.ising_sweep_rule(ctypes.byref(good), 0.4, 1.0, 7, 1, 0, None) == _lib.ISING_E_BADARG
    assert lib.ising_sweep_rule(ctypes.byref(good), 0.4, 1.0, 1, -1, 0, None) == _lib.ISING_E_BADARG
    assert lib.ising_thresholds_rule(0.4, 1.0, 1, T) == _lib.ISING_OK


def test_argument_errors_without_device(lib):
    from paper_1906_06297_amd import _lib

    lat = _lib.LatticeStruct()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    assert lib.ising_init(ctypes.byref(lat), fake, 1 << 20, 63, 1, 0, None) == _lib.ISING_E_BADARG
    assert b"even" in lib.ising_last_error()
    assert lib.ising_init(ctypes.byref(lat), fake, 8, 64, 1, 0, None) == _lib.ISING_E_SIZE
    assert lib.ising_init(None, fake, 1 << 20, 64, 1, 0, None) == _lib.ISING_E_BADARG
    assert lib.ising_init(ctypes.byref(lat), fake, 1 << 20, 64, 1, 1 << 24, None) == _lib.ISING_E_BADARG
    good = _lib.LatticeStruct(words=0x1000, L=64, seed=1, stream_id=0)
    for beta, J, n in ((float("nan"), 1.0, 1), (0.4, float("inf"), 1), (-0.1, 1.0, 1), (0.4, 1.0, -1)):
        assert lib.ising_sweep(ctypes.byref(good), beta, J, n, 0, None) == _lib.ISING_E_BADARG
    nowords = _lib.LatticeStruct(words=None, L=64)
    assert lib.ising_sweep(ctypes.byref(nowords), 0.4, 1.0, 1, 0, None) == _lib.ISING_E_BADARG
    odd = _lib.LatticeStruct(words=0x1000, L=65)
    assert lib.ising_sweep(ctypes.byref(odd), 0.4, 1.0, 1, 0, None) == _lib.ISING_E_BADARG
    assert lib.ising_sweep_traced(ctypes.byref(good), 0.4, 1.0, 3, 0, None, None, None) == _lib.ISING_E_BADARG
    assert lib.ising_observables(ctypes.byref(good), None, None, None) == _lib.ISING_E_BADARG
    assert lib.ising_set_sweep_kernel(6) == _lib.ISING_E_BADARG
    assert lib.ising_set_sweep_kernel(-1) == _lib.ISING_E_BADARG
    assert lib.ising_set_sweep_kernel(0) == _lib.ISING_OK
    T = (ctypes.c_uint64 * 5)()
    assert lib.ising_thresholds(float("nan"), 1.0, T) == _lib.ISING_E_BADARG
    assert lib.ising_thresholds(0.4, 1.0, T) == _lib.ISING_OK
    assert lib.ising_last_error() == b""


def test_set_spins_rejects_non_spin_values(lib):
    from paper_1906_06297_amd import _lib

    good = _lib.LatticeStruct(words=0x1000, L=4, seed=1, stream_id=0)
    s = np.ones((4, 4), np.int8)
    s[1, 2] = 0
    assert lib.ising_set_spins(ctypes.byref(good), s.ctypes.data_as(ctypes.c_void_p), None) == _lib.ISING_E_BADARG


def test_layout_helper_roundtrip():
    from layout import pack, unpack

    for L in (4, 6, 10, 24, 64):
        s = workloads.random_spins(L, L)
        w = pack(s)
        assert np.array_equal(unpack(w, L), s)
        # padding bits beyond the last spin stay zero
        M = L * L // 2
        if M % 64:
            assert int(w[0, -1]) >> (M % 64) == 0 and int(w[1, -1]) >> (M % 64) == 0


def test_batch_argument_errors_without_device(lib):
    from paper_1906_06297_amd import _lib

    L = (ctypes.c_int64 * 3)(16, 24, 722)
    assert lib.ising_batch_words(3, L) == 2 * (2 + 5 + 4073)  # 128, 288, 260642 spins per colour
    bad = (ctypes.c_int64 * 2)(16, 724)
    assert lib.ising_batch_words(2, bad) == -1
    odd = (ctypes.c_int64 * 1)(15)
    assert lib.ising_batch_words(1, odd) == -1
    h = ctypes.c_void_p()
    b = (ctypes.c_double * 3)(0.4, 0.4, 0.4)
    s = (ctypes.c_uint64 * 3)(1, 1, 1)
    i = (ctypes.c_uint32 * 3)(0, 1, 2)
    fake = ctypes.c_void_p(0x1000)
    assert lib.ising_batch_create(None, 3, L, b, 1.0, s, i, fake, 1 << 20) == _lib.ISING_E_BADARG
    assert lib.ising_batch_create(ctypes.byref(h), 0, L, b, 1.0, s, i, fake, 1 << 20) == _lib.ISING_E_BADARG
    assert lib.ising_batch_create(ctypes.byref(h), 3, L, b, 1.0, s, i, fake, 64) == _lib.ISING_E_SIZE
    assert lib.ising_batch_create(ctypes.byref(h), 2, bad, b, 1.0, s, i, fake, 1 << 20) == _lib.ISING_E_SIZE
    assert lib.ising_batch_sweep(None, 1, None) == _lib.ISING_E_BADARG
    per, n = ctypes.c_uint32(), ctypes.c_uint32()
    assert lib.ising_batch_get_plan(None, 16, ctypes.byref(per), ctypes.byref(n)) == _lib.ISING_E_BADARG
    assert lib.ising_batch_destroy(None) == _lib.ISING_OK


def test_batch_create_rejects_malformed_batches(lib):
    """Empty and malformed batches are rejected before any device work."""
    from paper_1906_06297_amd import _lib

    out = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first

    def create(Ls, betas, J=1.0, bytes_=1 << 20, n=None):
        n = len(Ls) if n is None else n
        L = (ctypes.c_int64 * max(len(Ls), 1))(*Ls)
        b = (ctypes.c_double * max(len(betas), 1))(*betas)
        s = (ctypes.c_uint64 * max(len(Ls), 1))(*([1] * len(Ls)))
        q = (ctypes.c_uint32 * max(len(Ls), 1))(*range(len(Ls)))
        return lib.ising_batch_create(ctypes.byref(out), n, L, b, J, s, q, fake, bytes_)

    assert create([], [], n=0) == _lib.ISING_E_BADARG
    assert b"empty" in lib.ising_last_error()
    assert create([16], [0.4], n=-1) == _lib.ISING_E_BADARG
    assert create([15], [0.4]) == _lib.ISING_E_SIZE  # odd L
    assert create([2], [0.4]) == _lib.ISING_E_SIZE  # below the minimum
    assert create([724], [0.4]) == _lib.ISING_E_SIZE  # above the LDS-resident maximum
    assert create([16], [-0.1]) == _lib.ISING_E_BADARG
    assert create([16], [float("nan")]) == _lib.ISING_E_BADARG
    assert create([16], [0.4], J=float("inf")) == _lib.ISING_E_BADARG
    assert create([256], [0.4], bytes_=8) == _lib.ISING_E_SIZE  # buffer too small


def test_glass_argument_errors_without_device(lib):
    """Bond arrays: size, alignment and lattice checks come before device work."""
    from paper_1906_06297_amd import _lib

    W = lib.ising_words_per_colour(256)
    need = 4 * W * 8
    fake = ctypes.c_void_p(0x1000)  # 16-byte aligned, never dereferenced
    assert lib.ising_glass_bonds_init(None, need, 256, 1, 0, None) == _lib.ISING_E_BADARG
    assert lib.ising_glass_bonds_init(ctypes.c_void_p(0x1008), need, 256, 1, 0, None) == _lib.ISING_E_BADARG
    assert b"aligned" in lib.ising_last_error()
    assert lib.ising_glass_bonds_init(fake, need - 8, 256, 1, 0, None) == _lib.ISING_E_SIZE
    assert lib.ising_glass_bonds_init(fake, need, 200, 1, 0, None) == _lib.ISING_E_SIZE  # L % 128
    assert lib.ising_glass_bonds_init(fake, need, 256, 1, 1 << 24, None) == _lib.ISING_E_BADARG
    good = _lib.LatticeStruct(words=0x1000, L=256, seed=1, stream_id=0)
    assert lib.ising_glass_sweep(ctypes.byref(good), ctypes.c_void_p(0x1008), need, 0.4, 1.0, 1, 0,
                                 None) == _lib.ISING_E_BADARG
    assert lib.ising_glass_sweep(ctypes.byref(good), fake, need, 0.4, 1.0, -1, 0,
                                 None) == _lib.ISING_E_BADARG
    assert lib.ising_glass_observables(ctypes.byref(good), fake, need, None, None,
                                       None) == _lib.ISING_E_BADARG


def test_matmul_argument_errors_without_device(lib):
    """Matrix-multiply form: size, alignment and buffer checks before device work."""
    from paper_1906_06297_amd import _lib

    assert lib.ising_mm_lattice_bytes(256) == 2 * 256 * 256
    assert lib.ising_mm_lattice_bytes(384) == -1
    assert lib.ising_mm_sums_bytes(768) == 768 * 768
    fake = ctypes.c_void_p(0x1000)
    need = 2 * 256 * 256

    def sweep(L=256, spins=fake, sb=need, sums=fake, nb=256 * 256, fused=0, beta=0.4, n=1):
        return lib.ising_mm_sweep(L, 1, 0, spins, sb, sums, nb, beta, 1.0, n, 0, fused, None)

    assert sweep(L=384) == _lib.ISING_E_SIZE
    assert sweep(spins=None) == _lib.ISING_E_BADARG
    assert sweep(spins=ctypes.c_void_p(0x1002)) == _lib.ISING_E_BADARG
    assert sweep(sb=need - 2) == _lib.ISING_E_SIZE
    assert sweep(sums=None) == _lib.ISING_E_BADARG  # the three-kernel form needs the sums
    assert sweep(nb=100) == _lib.ISING_E_SIZE
    assert sweep(fused=2) == _lib.ISING_E_BADARG
    assert sweep(beta=-1.0) == _lib.ISING_E_BADARG
    assert sweep(n=-1) == _lib.ISING_E_BADARG
    lat = _lib.LatticeStruct(words=0x1000, L=384, seed=1, stream_id=0)
    assert lib.ising_mm_from_words(ctypes.byref(lat), fake, 1 << 20, None) == _lib.ISING_E_SIZE
    lat = _lib.LatticeStruct(words=0x1000, L=256, seed=1, stream_id=0)
    assert lib.ising_mm_to_words(ctypes.byref(lat), fake, need - 1, None) == _lib.ISING_E_SIZE
