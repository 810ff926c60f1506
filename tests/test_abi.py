"""The C-ABI library loads and exports every entry point include/sphmap.h
declares (no compute calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

from conftest import ROOT


def header_functions():
    src = open(os.path.join(ROOT, "include", "sphmap.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:int|void|char|double)\s*\*?\s*(\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_lists_the_boundary():
    names = header_functions()
    for n in ["map_particles_to_cells", "map_cells_to_particles", "build_pseudo_particles", "sphmap_create",
              "sphmap_tess_upload"]:
        assert n in names


def test_library_exports_every_symbol():
    from paper_2410_15227_amd import _native
    if not os.path.exists(_native.LIB_PATH):
        pytest.skip("libsphmap.so not built (run __graft_entry__.build())")
    L = ctypes.CDLL(_native.LIB_PATH)
    missing = [n for n in header_functions() if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(_native.EXPORTS) == header_functions()
    assert _native.lib().sphmap_version() >= 100


def test_binding_fails_loudly_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    import paper_2410_15227_amd as pkg
    with pytest.raises(RuntimeError):
        pkg.Context(0)
