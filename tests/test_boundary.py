"""The C interface without a GPU: the library loads, exports every function the
header declares, sizes buffers, and rejects invalid arguments with an error code
(no call here reaches a kernel)."""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import torch
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hsg.h")


@pytest.fixture(scope="module")
def hsg():
    import paper_1006_2566_amd as m
    if not os.path.exists(m.LIB_PATH):
        from paper_1006_2566_amd import build
        build.build()
    m.lib()
    return m


def declared_functions() -> list[str]:
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hsg_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(hsg):
    names = declared_functions()
    assert "hsg_sweep" in names and "hsg_init_lattice" in names
    assert "hsg_energy" in names and "hsg_overlap" in names
    lib = hsg.lib()
    for name in names:
        assert hasattr(lib, name), name


def test_lattice_bytes(hsg):
    s, j, w = hsg.lattice_bytes(8)
    assert s == j == 3 * 512 * 4 and w > 0
    s64, j64, w64 = hsg.lattice_bytes(8, hsg_dtype := __import__("torch").float64)
    assert s64 == j64 == 3 * 512 * 8 and w64 == w
    s, _, _ = hsg.lattice_bytes(1290)
    assert s == 3 * 1290 ** 3 * 4


@pytest.mark.parametrize("L", [0, 1, 3, 7, -2, 1292, 2 ** 20])
def test_lattice_bytes_rejects_bad_L(hsg, L):
    lib = hsg.lib()
    rc = lib.hsg_lattice_bytes(L, 0, None, None, None)
    assert rc == -1
    assert b"L must be even" in lib.hsg_last_error()


def test_lattice_bytes_rejects_bad_dtype(hsg):
    assert hsg.lib().hsg_lattice_bytes(8, 7, None, None, None) == -1


def _desc(hsg, **kw):
    d = hsg._Lattice(8, 0, 1, 0, 0x1000, 0x2000, 0x3000, 0x4000, hsg.lattice_bytes(8)[2])
    for k, v in kw.items():
        setattr(d, k, v)
    return d


def test_null_and_missing_buffers_rejected(hsg):
    lib = hsg.lib()
    assert lib.hsg_init_lattice(None, None) == -1
    assert lib.hsg_sweep(None, None, 1, None) == -1
    d = _desc(hsg, spins=None)
    assert lib.hsg_init_lattice(ctypes.byref(d), None) == -1
    assert b"buffers" in lib.hsg_last_error()
    d = _desc(hsg, work_bytes=16)
    assert lib.hsg_init_lattice(ctypes.byref(d), None) == -1
    assert b"work buffer too small" in lib.hsg_last_error()


@pytest.mark.parametrize("T,k,n_or,R,flags,n", [
    (0.0, 1, 0, 0, 0, 1), (-1.0, 1, 0, 0, 0, 1), (float("nan"), 1, 0, 0, 0, 1),
    (1.0, 0, 0, 0, 0, 1), (1.0, -1, 1, 0, 0, 1), (1.0, 1, -1, 0, 0, 1),
    (1.0, 1, 0, -3, 0, 1), (1.0, 1, 0, 0, 8, 1), (1.0, 1, 0, 0, 0, -1), (1.0, 1, 0, 0, 512, 1),
    (1.0, 70000, 0, 0, 0, 1),
    # HSG_MARCH_PHASE without HSG_FUSED; HSG_FUSED with a pass-by-pass variant
    (1.0, 1, 0, 0, 16, 1), (1.0, 1, 0, 0, 4 | 32, 1), (1.0, 1, 0, 0, 4 | 64, 1),
    (1.0, 1, 0, 0, 4 | 128, 1), (1.0, 1, 0, 0, 4 | 256, 1), (1.0, 1, 0, 0, 1024, 1)])
def test_sweep_rejects_bad_params(hsg, T, k, n_or, R, flags, n):
    lib = hsg.lib()
    d = _desc(hsg)
    p = hsg._SweepParams(T, k, n_or, R, flags)
    assert lib.hsg_sweep(ctypes.byref(d), ctypes.byref(p), n, None) == -1
    assert d.sweep == 0


def test_fused_needs_the_larger_work_buffer(hsg):
    lib = hsg.lib()
    full = hsg.lattice_bytes(256)[2]
    assert full >= 3 * 256 ** 3 * 4
    d = _desc(hsg, L=256, work_bytes=full - 4)
    p = hsg._SweepParams(1.0, 1, 0, 0, hsg.HSG_FUSED)
    assert lib.hsg_sweep(ctypes.byref(d), ctypes.byref(p), 1, None) == -1
    assert b"HSG_FUSED" in lib.hsg_last_error()
    # lattices the fused passes do not cover need no second spin array
    assert hsg.lattice_bytes(96)[2] < 3 * 96 ** 3 * 4


def test_phase_launch_needs_the_larger_work_buffer(hsg):
    lib = hsg.lib()
    full = hsg.lattice_bytes(64)[2]
    d = _desc(hsg, L=64, work_bytes=full - 4)
    p = hsg._SweepParams(1.0, 1, 1, 0, hsg.HSG_PHASE_LAUNCH)
    assert lib.hsg_sweep(ctypes.byref(d), ctypes.byref(p), 1, None) == -1
    assert b"HSG_PHASE_LAUNCH" in lib.hsg_last_error()
    p = hsg._SweepParams(1.0, 1, 1, 0, hsg.HSG_PHASE_MC)
    assert lib.hsg_sweep(ctypes.byref(d), ctypes.byref(p), 2, None) == -1
    assert b"HSG_PHASE_MC" in lib.hsg_last_error()
    assert hsg.phase_supported(64) and not hsg.phase_supported(96)


def test_phase_launch_capped_where_offsets_fit_32_bits(hsg):
    """The phase launch indexes six planes of N/2 from one base with 32-bit offsets
    (up to 3 L^3): it applies up to L = 1024 and is ignored above, which shows in the
    work size (the second spin array is asked for only where a march applies)."""
    assert hsg.phase_supported(1024) and not hsg.phase_supported(1088)
    assert not hsg.phase_supported(1152) and not hsg.phase_supported(1280)
    for L in (1024, 1152, 1280):
        assert 3 * L ** 3 < 2 ** 32 or not hsg.phase_supported(L)
    spin_b, _, work_1024 = hsg.lattice_bytes(1024, torch.float32)
    assert work_1024 >= spin_b  # second spin array for the phase / fused launches
    spin_b, _, work_1152 = hsg.lattice_bytes(1152, torch.float32)
    assert work_1152 < spin_b // 100  # partials only: no march applies at L = 1152


def test_sweep_counter_overflow_rejected(hsg):
    lib = hsg.lib()
    d = _desc(hsg, sweep=2 ** 32 - 1)
    p = hsg._SweepParams(1.0, 1, 0, 0, 0)
    assert lib.hsg_sweep(ctypes.byref(d), ctypes.byref(p), 2, None) == -1
    assert b"2^32" in lib.hsg_last_error()


def test_overlap_requires_matching_lattices(hsg):
    lib = hsg.lib()
    a, b = _desc(hsg), _desc(hsg, L=10, work_bytes=hsg.lattice_bytes(10)[2])
    assert lib.hsg_overlap(ctypes.byref(a), ctypes.byref(b), ctypes.c_void_p(0x5000), None) == -1
    assert b"same L" in lib.hsg_last_error()
    assert lib.hsg_energy(ctypes.byref(a), 1, None, None) == -1
    assert lib.hsg_overlap_fourier(ctypes.byref(a), ctypes.byref(b), ctypes.c_void_p(0x5000),
                                   None) == -1
    assert b"same L" in lib.hsg_last_error()
    c = _desc(hsg)
    assert lib.hsg_overlap_fourier(ctypes.byref(a), ctypes.byref(c), None, None) == -1
    assert b"NULL" in lib.hsg_last_error()


def test_product_path_has_no_fallback(tmp_path, monkeypatch):
    import paper_1006_2566_amd as m
    monkeypatch.setattr(m, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(m, "_lib", None)
    with pytest.raises(ImportError):
        m.lib()


# ------------------------------------------------------------------ batched form
def _table(B, rows):
    import numpy as np
    t = np.zeros(len(rows), dtype=B.CHAIN_DTYPE)
    for i, r in enumerate(rows):
        t[i] = r
    return t


@pytest.mark.parametrize("rows,spin_elems,J_elems,msg", [
    ([(0, 0, 1, 1, 7, 1, 0, 0, 0, 0)], 10 ** 6, 10 ** 6, b"L must be even"),
    ([(0, 0, 1, 1, 258, 1, 0, 0, 0, 0)], 10 ** 9, 10 ** 9, b"L must be even"),
    ([(0, 0, 1, 1, 8, 0, 0, 0, 0, 0)], 10 ** 6, 10 ** 6, b"k_hits"),
    ([(0, 0, 1, 1, 8, 1, 0, 0, 64, 0)], 10 ** 6, 10 ** 6, b"flags"),
    ([(0, 0, 1, 1, 8, 1, 0, 0, 0, 0)], 1000, 10 ** 6, b"spin buffer"),
    ([(0, 10, 1, 1, 8, 1, 0, 0, 0, 0)], 10 ** 6, 1536, b"coupling buffer"),
    ([(0, 0, 1, 1, 8, 1, 0, 0, 0, 0), (1000, 0, 1, 1, 8, 1, 0, 0, 0, 0)], 10 ** 6, 10 ** 6,
     b"overlap"),
])
def test_batch_check_rejects(hsg, rows, spin_elems, J_elems, msg):
    from paper_1006_2566_amd import batch as B
    B._bind()
    t = _table(B, rows)
    lib = hsg.lib()
    assert lib.hsg_batch_check(t.ctypes.data_as(ctypes.c_void_p), len(rows), spin_elems,
                               J_elems) == -1
    assert msg in lib.hsg_last_error()


def test_batch_check_accepts_shared_couplings(hsg):
    from paper_1006_2566_amd import batch as B
    B._bind()
    n = 3 * 8 ** 3
    t = _table(B, [(0, 0, 1, 1, 8, 1, 0, 0, 8, 0), (n, 0, 2, 1, 8, 4, 1, 10, 1, 0)])
    assert hsg.lib().hsg_batch_check(t.ctypes.data_as(ctypes.c_void_p), 2, 2 * n, n) == 0


def test_batch_descriptor_validation(hsg):
    from paper_1006_2566_amd import batch as B
    B._bind()
    lib = hsg.lib()
    d = B._Batch(2, 0, 0x10, 0x20, 0x30, 0x40, 0x50, 0x60, None, 0x70, 96, 0)
    assert lib.hsg_batch_sweep(ctypes.byref(d), 1, None) == -1  # threads not a multiple of 64
    d.threads = 256
    d.reserved = 1
    assert lib.hsg_batch_sweep(ctypes.byref(d), 1, None) == -1
    assert b"reserved" in lib.hsg_last_error()
    d.reserved = 0
    d.order = None
    assert lib.hsg_batch_sweep(ctypes.byref(d), 1, None) == -1
    assert b"order" in lib.hsg_last_error()
    d.order = 0x70
    d.E = None
    assert lib.hsg_batch_init(ctypes.byref(d), None) == -1
    p = B._PT(0, 4, 0x10, 0x20, None, 0x30, 1)
    d.E = 0x50
    assert lib.hsg_pt_exchange(ctypes.byref(p), ctypes.byref(d), None) == -1
    p = B._PT(2, 4, 0x10, 0x20, None, None, 1)
    assert lib.hsg_pt_exchange(ctypes.byref(p), ctypes.byref(d), None) == -1
    assert b"round" in lib.hsg_last_error()


def test_pt_workload_shape():
    from paper_1006_2566_amd import batch as B
    specs, ladders, betas, pairs = B.pt_workload()
    assert len(specs) == 256 * 2 * 24 and ladders.shape == (512, 24) and pairs.shape == (256, 2)
    assert abs(1 / betas[0] - 0.12) < 1e-12 and abs(1 / betas[-1] - 0.5) < 1e-12
    # geometric: constant ratio of successive temperatures
    T = 1 / betas
    assert np.allclose(T[1:] / T[:-1], (0.5 / 0.12) ** (1 / 23))
    Ls = {s.L for s in specs}
    assert Ls <= {16, 24, 32, 48}
    # a sample's 48 chains share one coupling group and one L
    assert len({(s.J_group, s.L) for s in specs}) == 256




def test_default_flags(hsg):
    """Phase launches only where the lattice gives them enough workgroups; in binary32 the
    phase launch also carries the next colour-0 Monte Carlo pass (measured faster), in
    binary64 not (measured slower)."""
    assert hsg.default_flags(256, torch.float32) == hsg.HSG_SNAKE | hsg.HSG_PHASE_MC
    assert hsg.default_flags(512) == hsg.HSG_SNAKE | hsg.HSG_PHASE_MC
    assert hsg.default_flags(256, torch.float64) == hsg.HSG_SNAKE | hsg.HSG_PHASE_LAUNCH
    assert hsg.default_flags(128, torch.float32) == hsg.HSG_SNAKE
    assert hsg.default_flags(320) == hsg.HSG_SNAKE | hsg.HSG_PHASE_MC
    assert hsg.default_flags(288) == hsg.HSG_SNAKE  # not a multiple of 64


def test_sweep_timed_rejects_bad_outputs(hsg):
    """The measurement form validates its output arrays before anything is enqueued,
    and invalid sweep arguments fail as in hsg_sweep."""
    lib = hsg.lib()
    d = _desc(hsg)
    p = hsg._SweepParams(1.0, 1, 0, 0, 0)
    n = ctypes.c_int32(-5)
    assert lib.hsg_sweep_timed(ctypes.byref(d), ctypes.byref(p), 1, None, -1, None, None,
                               ctypes.byref(n)) == -1
    assert lib.hsg_sweep_timed(ctypes.byref(d), ctypes.byref(p), 1, None, 4, None, None,
                               ctypes.byref(n)) == -1
    assert lib.hsg_sweep_timed(ctypes.byref(d), ctypes.byref(p), 1, None, 0, None, None,
                               None) == -1
    bad = hsg._SweepParams(-1.0, 1, 0, 0, 0)
    assert lib.hsg_sweep_timed(ctypes.byref(d), ctypes.byref(bad), 1, None, 0, None, None,
                               ctypes.byref(n)) == -1
    assert b"T must be" in lib.hsg_last_error()
    assert n.value == 0  # nothing was recorded


def test_noalloc_sweep_rejects_what_needs_scratch_it_does_not_have(hsg):
    """hsg_sweep_noalloc checks its limits before anything reaches the device: L beyond
    its scratch, traversals that need a second spin array, and the usual arguments; it
    needs no work buffer."""
    lib = hsg.lib()
    lib.hsg_sweep_noalloc.argtypes = [ctypes.POINTER(hsg._Lattice),
                                      ctypes.POINTER(hsg._SweepParams), ctypes.c_int32,
                                      ctypes.c_void_p]
    p = hsg._SweepParams(1.0, 1, 1, 0, 0)
    big = hsg._Lattice(514, 0, 1, 0, 0x1000, 0x2000, 0x3000, None, 0)
    assert lib.hsg_sweep_noalloc(ctypes.byref(big), ctypes.byref(p), 1, None) == -1
    assert b"HSG_NOALLOC_L_MAX" in lib.hsg_last_error()
    d = hsg._Lattice(64, 0, 1, 0, 0x1000, 0x2000, 0x3000, None, 0)
    for flag in (hsg.HSG_FUSED, hsg.HSG_PHASE_LAUNCH, hsg.HSG_PHASE_MC):
        q = hsg._SweepParams(1.0, 1, 1, 0, flag)
        assert lib.hsg_sweep_noalloc(ctypes.byref(d), ctypes.byref(q), 1, None) == -1
        assert b"second" in lib.hsg_last_error() or b"HSG_FUSED" in lib.hsg_last_error()
    bad = hsg._SweepParams(0.0, 1, 1, 0, 0)
    assert lib.hsg_sweep_noalloc(ctypes.byref(d), ctypes.byref(bad), 1, None) == -1
    nospins = hsg._Lattice(64, 0, 1, 0, None, 0x2000, 0x3000, None, 0)
    assert lib.hsg_sweep_noalloc(ctypes.byref(nospins), ctypes.byref(p), 1, None) == -1
    assert lib.hsg_sweep_noalloc(None, ctypes.byref(p), 1, None) == -1
