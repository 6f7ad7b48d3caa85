"""CPU checks of the C ABI library and the host-side helpers (no GPU calls)."""
import os
import re

import numpy as np

import paper_1309_5050_amd as S
from paper_1309_5050_amd import _native
from paper_1309_5050_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "shssa.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ssa_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for must in ["ssa_ctx_create", "ssa_decompose", "ssa_decompose_multi", "ssa_decompose_batch",
                 "ssa_reconstruct", "ssa_get_sigma", "ssa_get_vectors", "ssa_free"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = S.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_covers_every_symbol():
    assert set(declared_functions()) <= set(_native._SIGS)


def test_error_strings():
    lib = S.lib()
    for code in range(0, -9, -1):
        assert lib.ssa_strerror(code)


def test_ctx_create_fails_cleanly_without_device():
    import ctypes as C
    lib = S.lib()
    h = C.c_void_p()
    rc = lib.ssa_ctx_create(-1, 0, None, C.byref(h))
    assert rc != 0 and not h.value


def test_workloads_are_deterministic():
    a = W.image_2d(n=64, lw=8, seed=3)["x"]
    b = W.image_2d(n=64, lw=8, seed=3)["x"]
    assert np.array_equal(a, b)
    m1 = W.mssa_series(s=5, seed=3)["x"]
    m2 = W.mssa_series(s=5, seed=3)["x"]
    assert all(np.array_equal(x, y) for x, y in zip(m1, m2))
    d = W.shaped_disc(n=160, radius=72.0, lw=8, hole_r=(1, 3))
    nan = np.isnan(d["x"]) & (d["mask"] == 1)
    assert 0.09 <= nan.sum() / d["mask"].sum() <= 0.2


def test_serving_mix_shape():
    reqs = W.serving_mix(n_requests=2000, seed=5)
    kinds = [r["kind"] for r in reqs]
    frac = {k: kinds.count(k) / len(kinds) for k in ("1d", "mssa", "2d")}
    assert abs(frac["1d"] - 0.60) < 0.05 and abs(frac["mssa"] - 0.25) < 0.05 and abs(frac["2d"] - 0.15) < 0.05
