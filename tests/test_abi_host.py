"""Host-side checks of the C ABI (no GPU needed).

libtmd.so must load and export every function declared in include/tmd.h;
argument validation that happens before any device work is exercised with
null handles.  No kernel is launched here.
"""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tmd.h")
LIB = os.path.join(ROOT, "paper_2310_08439_amd", "libtmd.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tmd_[a-z0-9_]+)\s*\(", text)))


def _ensure_built():
    if not os.path.exists(LIB):
        from paper_2310_08439_amd import build
        build.build()


def test_header_declares_the_boundary_entry_points():
    names = _declared()
    for required in ("tmd_build_neighbors", "tmd_descriptors", "tmd_energy_forces"):
        assert required in names


def test_library_exports_every_declared_symbol():
    _ensure_built()
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(line.split()[-1] for line in out.splitlines() if line.strip())
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing


def test_library_loads_and_binding_covers_header():
    _ensure_built()
    lib = ctypes.CDLL(LIB)
    for n in _declared():
        assert hasattr(lib, n)
    from paper_2310_08439_amd import tmd
    assert set(_declared()) == set(tmd.EXPORTS)


def test_null_argument_validation_without_device():
    _ensure_built()
    from paper_2310_08439_amd import tmd
    L = tmd.load_library()
    assert L.tmd_context_create(0, None, None) == 1
    assert L.tmd_model_set_precision(None, 0) == 1
    assert L.tmd_context_set_stream(None, None) == 1
    assert L.tmd_profile_enable(None, 1) == 1
    assert L.tmd_model_params_per_species(None) == 0
    assert L.tmd_nlist_capacity(None) == 0
    assert L.tmd_last_error(None) == b"null context"
    v = tmd.SystemView()
    assert L.tmd_build_neighbors(None, ctypes.byref(v), 5.0, 0.0, None, None) == 1
    assert L.tmd_train_step(None, None, None, None, None, None) == 1
    assert L.tmd_batch_create(None, None, 1, None, None, None, None, None, None, 0, None) == 1
    assert L.tmd_batch_read(None, None, 0, None) == 1
    assert L.tmd_model_get_params(None, None) == 1
    assert L.tmd_model_tabulate(None, 0.01) == 1
    assert L.tmd_model_tab_spacing(None) == 0.0
    assert L.tmd_serve_create(None, None, None) == 1
    assert L.tmd_serve_submit(None, None, None) == 1
    assert L.tmd_serve_poll(None, 1, None) == 1
    assert L.tmd_serve_wait(None, 1, 0.0, None) == 1
    assert L.tmd_serve_fetch(None, 1, None, None, None, None, None) == 1
    assert L.tmd_serve_release(None, 1) == 1
    assert L.tmd_serve_memory(None, None, None) == 1
    assert L.tmd_serve_last_error(None) == b"null server"


def test_param_layout_matches_library_contract():
    """The generator's per-species block length is the one tmd_model_create documents."""
    from paper_2310_08439_amd import inputs
    for F, hidden in ((32, [64, 64]), (96, [128, 128]), (128, [128, 128, 128])):
        expect = 0
        prev = F
        for h in hidden:
            expect += h * prev + h
            prev = h
        expect += prev + 1
        assert inputs.params_per_species(F, hidden) == expect


def test_default_capacity_covers_mean_count():
    from paper_2310_08439_amd import tmd
    import math
    cap = tmd.default_capacity(1024000, [252.8] * 3, 6.0, 2)
    mean = 1024000 / 252.8 ** 3 * 4 / 3 * math.pi * 6.0 ** 3
    assert cap >= mean / 2 + 8
