"""The HIP C-ABI library builds, loads and exports every entry point declared in include/vstab.h
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vstab.h")
LIB = os.path.join(ROOT, "paper_1701_03572_amd", "libvstab.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(vs_[a-z0-9_]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1701_03572_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_six_operations():
    names = declared_functions()
    for op in ["vs_build_pyramid", "vs_detect_corners", "vs_track_lk", "vs_fit_similarity", "vs_smooth_trajectory",
               "vs_warp_frame"]:
        assert op in names


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_every_declared_symbol():
    from paper_1701_03572_amd import vstab
    assert sorted(vstab.exported_symbols()) == declared_functions()


def test_host_only_calls_without_gpu(lib):
    from paper_1701_03572_amd import vstab
    L = vstab.vs_pyramid_layout(1920, 1080, 1920, 5)
    assert list(L.width)[:5] == [1920, 960, 480, 240, 120]
    assert list(L.height)[:5] == [1080, 540, 270, 135, 68]
    assert all(p % 64 == 0 for p in list(L.pitch)[1:5])
    assert all(o % 256 == 0 for o in list(L.offset)[1:5])
    assert L.bytes >= 960 * 540 + 480 * 270 + 240 * 135 + 120 * 68
    with pytest.raises(vstab.VsError):
        vstab.vs_pyramid_layout(40, 30, 40, 3)          # level 2 would be 10x8
    with pytest.raises(vstab.VsError):
        vstab.vs_pyramid_layout(64, 64, 64, 9)
    assert vstab.vs_detect_workspace(320, 240, 2) >= 2 * 12 * 320 * 240
    assert vstab.vs_fit_workspace(3, 200) > 0
    assert vstab.vs_traj_state_bytes() >= 16 + 8 * 8 + 2 * 256 * 4 * 8
    assert vstab.vs_version() == 1
