"""CPU checks of the C-ABI library: it loads, exports every declared entry
point, and its host-side argument validation behaves as documented.  No
device work is issued."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cube2.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:int|void|const char \*)\s*(cube2_\w+)\(", txt, re.M)))


@pytest.fixture(scope="module")
def L():
    import paper_2512_12629_amd as m
    return m.lib()


def test_header_declares_the_hot_path():
    names = _declared()
    for must in ["cube2_deposit", "cube2_pm_force", "cube2_pp_force", "cube2_kick_drift",
                 "cube2_deposit_backward", "cube2_pm_force_backward",
                 "cube2_pp_force_backward", "cube2_kick_drift_backward"]:
        assert must in names


def test_library_exports_every_declared_symbol(L):
    for name in _declared():
        assert hasattr(L, name), name


def _cfg(**kw):
    import paper_2512_12629_amd as m
    base = dict(n_fine=64, coarse_ratio=0, b_coarse=14.0, b_fine=2.0, b_pp=0.2, m_p=1.0,
                g_newton=1.0, alias_nmax=2, flags=0)
    base.update(kw)
    return m.cube2_config(**base)


def _create(L, cfg):
    h = ctypes.c_void_p()
    code = L.cube2_create(ctypes.byref(cfg), ctypes.byref(h))
    return code, h


def test_create_validates_configuration(L):
    ok, h = _create(L, _cfg())
    assert ok == 0
    L.cube2_destroy(h)
    assert _create(L, _cfg(n_fine=48))[0] == -2        # not a power of two
    assert _create(L, _cfg(n_fine=2048))[0] == -2
    assert _create(L, _cfg(coarse_ratio=3))[0] == -2
    assert _create(L, _cfg(n_fine=32, coarse_ratio=8))[0] == -2   # coarse mesh < 8
    assert _create(L, _cfg(b_pp=2.0))[0] == -1          # b_pp >= b_fine
    assert _create(L, _cfg(b_fine=4.5))[0] == -2        # PP beyond two IOS cells
    assert _create(L, _cfg(b_fine=3.5, b_pp=0.0625))[0] == 0   # two-cell PP reach, K = 112
    assert _create(L, _cfg(b_fine=3.5, b_pp=0.06))[0] == -2    # no K <= 128 aligns 0.03
    assert _create(L, _cfg(coarse_ratio=4, b_coarse=1.0))[0] == -1
    assert _create(L, _cfg(alias_nmax=9))[0] == -2
    # b_pp/2 = 0.03 is on no grid of K <= 128 equal intervals of [0, 2)
    assert _create(L, _cfg(b_pp=0.06))[0] == -2
    assert _create(L, _cfg(b_pp=0.1))[0] == 0           # K = 40


def test_sizes_and_state_errors(L):
    code, h = _create(L, _cfg(n_fine=64, coarse_ratio=4))
    assert code == 0
    tb, wb = ctypes.c_size_t(), ctypes.c_size_t()
    assert L.cube2_sizes(h, 32768, ctypes.byref(tb), ctypes.byref(wb)) == 0
    assert tb.value > 33 ** 3 * 4 and wb.value > 64 ** 3 * 4
    n, p = ctypes.c_int32(), ctypes.c_int32()
    assert L.cube2_level_shape(h, 1, ctypes.byref(n), ctypes.byref(p)) == 0
    assert (n.value, p.value) == (16, 16)
    assert L.cube2_level_shape(h, 2, ctypes.byref(n), ctypes.byref(p)) == -1
    # entry points refuse to run before cube2_init_tables (no device work)
    nul = ctypes.c_void_p()
    assert L.cube2_pm_force(h, nul, nul, 0, nul, 0, nul, 0, nul) == -6
    assert L.cube2_sizes(h, -1, ctypes.byref(tb), ctypes.byref(wb)) == -1
    L.cube2_destroy(h)


def test_strerror(L):
    assert L.cube2_strerror(-4) == b"deposit accumulator overflow guard tripped"


@pytest.mark.parametrize("n_fine,ratio,flags", [
    (16, 0, 0), (32, 0, 0), (64, 0, 0), (256, 0, 0), (1024, 0, 0),
    (32, 2, 0), (64, 4, 0), (64, 8, 0), (512, 4, 0), (1024, 4, 0), (1024, 2, 0), (1024, 8, 0),
    (64, 4, 4), (256, 0, 4)])
def test_self_check_of_index_arithmetic(L, n_fine, ratio, flags):
    """The velocity codec's bulk-cell indices of every tile (one level: cells
    of 4 fine cells; two levels: the coarse cells), its per-tile maxima area,
    the PM adjoint's fixed-point coarse mesh and the concurrent PP staging
    area, checked on the host with the kernels' own index functions, for
    particle counts from 0 to the size of the largest workload."""
    code, h = _create(L, _cfg(n_fine=n_fine, coarse_ratio=ratio, flags=flags))
    assert code == 0
    try:
        for n_max in (0, 1, 4097, (n_fine // 2) ** 3):
            assert L.cube2_self_check(h, n_max) == 0, n_max
        assert L.cube2_self_check(h, -1) == -1
    finally:
        L.cube2_destroy(h)
