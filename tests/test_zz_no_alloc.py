"""The allocation-free ESPRIT call (ssa_esprit_noalloc, fixed device scratch)
against ssa_esprit: the same kernels on the same inputs, so the roots must
be identical, on consecutive calls whose second one is smaller."""
import numpy as np
import pytest

from paper_1309_5050_amd import workloads as W

pytestmark = pytest.mark.gpu


def _roots(lib, fn, d, grp):
    g = np.ascontiguousarray(grp, dtype=np.int32)
    re, im = np.zeros(len(g)), np.zeros(len(g))
    rc = getattr(lib, fn)(d.handle, g.ctypes.data, len(g), re.ctypes.data, im.ctypes.data)
    return rc, re, im


def test_noalloc_esprit_equals_esprit():
    import paper_1309_5050_amd as S
    from paper_1309_5050_amd import _native
    lib = _native.lib()
    c = S.Context(0)
    try:
        w = W.series_1d()                                            # N = 1000, L = 500, r = 10
        big = c.decompose(w["x"], w["window"], w["r"])
        m = W.mssa_series(s=6, nmin=300, nmax=500, L=100, r=8, seed=3)
        small = c.decompose_multi(m["x"], 100, 8, precision="fp32")
        # two calls in a row through the fixed scratch, the second smaller
        for d, grp in ((big, list(range(10))), (small, [0, 1, 2, 3]), (big, [2, 3])):
            rc0, re0, im0 = _roots(lib, "ssa_esprit", d, grp)
            rc1, re1, im1 = _roots(lib, "ssa_esprit_noalloc", d, grp)
            assert rc0 == 0 and rc1 == 0, (rc0, rc1, lib.ssa_last_error())
            assert np.array_equal(re0, re1) and np.array_equal(im0, im1), grp
        # a group beyond r is refused before the scratch is touched
        rc, _, _ = _roots(lib, "ssa_esprit_noalloc", small, [0, 9])
        assert rc == -1
        assert np.array_equal(small.esprit_noalloc([0, 1]), small.esprit([0, 1]))
    finally:
        c.close()
