"""The C-ABI library loads and exports every entry point that
include/overset.h declares (no compute calls: CPU only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "overset.h")
LIB = os.path.join(ROOT, "paper_1910_09315_amd", "liboverset.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?(?:int|int32_t|int64_t|char|void)\s*\*?\s*(\w+)\s*\(",
                                 text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1910_09315_amd.build import build
        build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_five_step_calls():
    names = declared()
    for n in ("overset_transform", "overset_holecut", "overset_fringe_compact", "overset_donor_search",
              "overset_interp"):
        assert n in names


def test_header_declares_the_matrix_and_frame_calls():
    names = declared()
    for n in ("overset_frame_velocity", "overset_interp_matrix", "overset_interp_apply"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    for n in declared():
        assert hasattr(lib, n), n


def test_binding_covers_every_declared_symbol():
    from paper_1910_09315_amd import binding
    assert sorted(binding.EXPORTS) == declared()


def test_binding_refuses_missing_library(tmp_path):
    from paper_1910_09315_amd import binding
    saved = binding._lib
    binding._lib = None
    try:
        with pytest.raises(binding.OversetError):
            binding.load(str(tmp_path / "missing.so"))
    finally:
        binding._lib = saved
