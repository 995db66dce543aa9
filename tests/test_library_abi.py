"""The C-ABI library loads and exports every function include/geer.h declares;
host-only entry points (no device work) are checked against the oracle."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "geer.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:geer_status|void|const char\*|int64_t|int32_t)\s+(geer_\w+)\s*\(", src, re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_2505_24053_amd import _lib

    if not os.path.exists(_lib.LIB_PATH):
        import __graft_entry__

        __graft_entry__.build()
    return _lib.load()


def test_exports_every_declared_symbol(lib):
    from paper_2505_24053_amd import _lib

    names = declared_functions()
    assert len(names) >= 12
    assert sorted(_lib.EXPORTS) == names
    for name in names:
        assert hasattr(lib, name), name


def test_default_opts(lib):
    from paper_2505_24053_amd import _lib
    import ctypes as C

    o = _lib.GeerOpts()
    lib.geer_default_opts(C.byref(o))
    assert o.alpha_min == np.float32(1 / 255) and o.alpha_max == np.float32(0.99)
    assert o.t_min == np.float32(1e-4) and o.lambda_fixed == 3.0 and o.lambda_mode == 0


@pytest.mark.parametrize("kind", ["pinhole", "kb190", "kbwide"])
def test_valid_mask_matches_oracle(lib, kind):
    import oracle
    from paper_2505_24053_amd import _lib, synth

    if kind == "pinhole":
        cam = synth.camera_pinhole(64, 48, 60.0)
    elif kind == "kb190":
        cam = synth.camera_kb(128, 96, 190.0, seed=0)
    else:
        cam = synth.camera_kb(128, 96, 190.0, seed=3)
        cam = dict(cam, fov_x=cam["fov_x"] * 1.2, fov_y=cam["fov_y"] * 1.2)
    got = _lib.valid_mask(cam)
    ref = oracle.valid_mask(cam)
    assert (got != ref).sum() <= 2  # only rays landing within rounding of the sensor edge may differ


def test_invalid_view_rejected_on_host(lib):
    from paper_2505_24053_amd import _lib, synth

    cam = synth.camera_pinhole(64, 48, 60.0)
    with pytest.raises(_lib.GeerError):
        _lib.valid_mask(dict(cam, fov_y=4.0))
    with pytest.raises(_lib.GeerError):
        _lib.valid_mask(dict(cam, width=0))
