"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Tolerances: singular values |s_i - s_i^o| <= tol * s_1 (Weyl), spans of
gap-stable groups |P - P^o|_2 <= C tol s_1 / gap (Wedin), reconstructions
|x_G - x_G^o| / |x| <= C tol s_1 / gap, with tol = 1e-10 for the FP64 path
and 1e-5 for the FP32 path (FP32 products, FP64 Lanczos).  Individual
vectors of clusters closer than 1e-3 s_1 are not unique (only their span
is); such clusters are compared as a whole.
"""
import os

import numpy as np
import pytest

import oracle
from paper_1309_5050_amd import workloads as W

from helpers import TOL, proj_dist, sigma_err, stable_groups

pytestmark = pytest.mark.gpu
C_SUB = 20.0


@pytest.fixture(scope="module")
def ctx():
    import paper_1309_5050_amd as S
    c = S.Context(0)
    yield c
    c.close()


_ORACLE = {}


def oracle_case(name, w):
    if name not in _ORACLE:
        if w["kind"] == "mssa":
            s, U, V = oracle.decompose_mssa(w["x"], w["window"])
            _ORACLE[name] = (None, s, U, V)
        else:
            _ORACLE[name] = oracle.decompose(w["x"], w["mask"], w["wmask"], w["window"])
    return _ORACLE[name]


def gpu_case(ctx, w, prec):
    if w["kind"] == "mssa":
        return ctx.decompose_multi(w["x"], w["window"], w["r"], precision=prec)
    return ctx.decompose(w["x"], w["window"], w["r"], mask=w["mask"], wmask=w["wmask"], precision=prec)


def packed_mssa(w):
    ser = w["x"]
    nmax = max(len(s) for s in ser)
    arr = np.full((nmax, len(ser)), np.nan)
    for p, s in enumerate(ser):
        arr[:len(s), p] = s
    return arr


CASES = {
    "series_1000": lambda: W.series_1d(),
    "image_128": lambda: W.config(2, "small"),
    "mssa_8": lambda: W.config(3, "small"),
    "disc_160": lambda: W.config(4, "small"),
    "small_shaped": lambda: W.small_shaped(),
    "series_ragged": lambda: W.series_1d(n=777, L=301, r=12, seed=9),
    "image_ragged": lambda: dict(W.image_2d(n=97, lw=13, r=14, seed=21), x=W.image_2d(n=97, r=14, seed=21)["x"][:, :83]),
}


def check_case(ctx, name, prec, groups_too=True):
    w = CASES[name]()
    tol = TOL[prec]
    sh, so, Uo, Vo = oracle_case(name, w)
    d = gpu_case(ctx, w, prec)
    r = w["r"]
    s = d.sigma
    err = sigma_err(s, so)
    print(f"{name} {prec}: sigma err {err:.2e} stats {d.stats}")
    assert d.stats["converged"] == 1
    assert err <= tol, (name, prec, err)
    U, V = d.vectors_lex()
    assert U.shape == (Uo.shape[0], r) and V.shape == (Vo.shape[0], r)
    for g, gap in stable_groups(so, r):
        bound = C_SUB * tol * so[0] / gap
        du = proj_dist(U[:, g], Uo[:, g])
        dv = proj_dist(V[:, g], Vo[:, g])
        assert du <= bound and dv <= bound, (name, prec, g, du, dv, bound)
    # orthonormality of both sides
    assert np.allclose(U.T @ U, np.eye(r), atol=max(1e-9, 10 * tol))
    assert np.allclose(V.T @ V, np.eye(r), atol=max(1e-9, 100 * tol))
    if not groups_too:
        return d
    # reconstruction of the gap-stable groups (and of their union)
    sg = [g for g, _ in stable_groups(so, r)]
    gaps = [gap for _, gap in stable_groups(so, r)]
    groups = sg[:4] + [sorted(sum(sg[:4], []))]
    gaps = gaps[:4] + [min(gaps[:4])]
    rec = d.reconstruct(groups)
    if w["kind"] == "mssa":
        lens = [len(x) for x in w["x"]]
        for k, g in enumerate(groups):
            ref = oracle.reconstruct_mssa(lens, w["window"], so, Uo, Vo, g)
            got = [rec[k][:n, p] for p, n in enumerate(lens)]
            assert all(np.all(np.isnan(rec[k][n:, p])) for p, n in enumerate(lens))
            num = np.sqrt(sum(np.sum((a - b) ** 2) for a, b in zip(got, ref)))
            den = np.sqrt(sum(np.sum(x ** 2) for x in w["x"]))
            assert num / den <= C_SUB * tol * so[0] / gaps[k], (name, prec, g, num / den)
    else:
        x = w["x"] if w["x"].ndim == 2 else w["x"][:, None]
        for k, g in enumerate(groups):
            ref = oracle.reconstruct(sh, so, Uo, Vo, g)
            got = rec[k]
            assert np.array_equal(np.isnan(got), np.isnan(ref)), (name, "covered set differs")
            cov = ~np.isnan(ref)
            num = np.linalg.norm(got[cov] - ref[cov])
            den = np.linalg.norm(np.nan_to_num(x[cov]))
            assert num / den <= C_SUB * tol * so[0] / gaps[k], (name, prec, g, num / den)
        assert np.array_equal(d.weights, sh.W)
    return d


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", list(CASES))
def test_parity(ctx, name, prec):
    check_case(ctx, name, prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", ["series_1000", "image_128", "disc_160", "small_shaped", "image_ragged"])
def test_wcor_parity(ctx, name, prec):
    """w-correlations and contributions of the gap-stable groups against the
    oracle's.  A group's reconstruction is within d = 20 tol s_1 / gap of
    the oracle's (relative to |x|), so a correlation moves by at most about
    d (c_a^-1/2 + c_b^-1/2) and a contribution by about 2 d c_a^1/2 (+ d^2),
    c = contribution; the bounds below allow 4x that."""
    w = CASES[name]()
    tol = TOL[prec]
    sh, so, Uo, Vo = oracle_case(name, w)
    d = gpu_case(ctx, w, prec)
    st = stable_groups(so, w["r"])
    groups = [g for g, _ in st][:5]
    gap = min(gp for _, gp in st[:5])
    rho, c = d.wcor(groups)
    rho_o, c_o = oracle.wcor(w["x"], sh, so, Uo, Vo, groups)
    dd = 20 * tol * so[0] / gap
    assert np.allclose(rho, rho.T) and np.allclose(np.diag(rho), 1.0)
    for a in range(len(groups)):
        assert abs(c[a] - c_o[a]) <= 4 * (2 * dd * np.sqrt(c_o[a]) + dd * dd), (name, prec, a, c[a], c_o[a])
        for b in range(len(groups)):
            bound = 4 * dd * (1 / np.sqrt(c_o[a]) + 1 / np.sqrt(c_o[b]))
            assert abs(rho[a, b] - rho_o[a, b]) <= bound, (name, prec, a, b, rho[a, b], rho_o[a, b], bound)


def _rforecast_oracle(name, w, group, h):
    sh, so, Uo, Vo = oracle_case(name, w)
    if w["kind"] == "mssa":
        lens = [len(x) for x in w["x"]]
        recs = oracle.reconstruct_mssa(lens, w["window"], so, Uo, Vo, group)
    else:
        recs = [oracle.reconstruct(sh, so, Uo, Vo, group)[:, 0]]
    return oracle.rforecast_column(recs, Uo, group, h), so


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name,group", [("series_1000", [0, 1, 2, 3, 4, 5]), ("mssa_8", [0, 1, 2, 3])])
def test_rforecast_parity(ctx, name, group, prec):
    """Column recurrent forecast (24 values) from the GPU decomposition and
    reconstruction against the oracle's.  The group is a union of gap-stable
    groups whose span (and reconstruction) is within 20 tol s_1 / gap of the
    oracle's, relative; the bound allows that relative to the largest
    forecast value (the recurrence over 24 steps of these damped signals
    does not amplify it)."""
    w = CASES[name]()
    tol = TOL[prec]
    h = 24
    ref, so = _rforecast_oracle(name, w, group, h)
    d = gpu_case(ctx, w, prec)
    got = d.rforecast(group, h)
    if w["kind"] == "mssa":
        assert got.shape == (len(w["x"]), h)
    gap = so[group[-1]] - so[group[-1] + 1]
    bound = 20 * tol * so[0] / gap * np.max(np.abs(ref))
    err = np.max(np.abs(got - ref))
    print(f"{name} {prec}: forecast error {err:.3e} bound {bound:.3e}")
    assert err <= bound, (name, prec, err, bound)


def test_rforecast_continues_a_cosine(ctx):
    """A pure cosine (rank 2) is continued exactly by its LRR."""
    N, L, h = 300, 120, 40
    t = np.arange(N + h)
    x = 2.0 * np.cos(2 * np.pi * t / 15 + 0.3)
    d = ctx.decompose(x[:N], L, 2)
    f = d.rforecast([0, 1], h)[0]
    assert np.max(np.abs(f - x[N:])) <= 1e-8


def test_rforecast_errors(ctx):
    import paper_1309_5050_amd as S
    x = np.random.default_rng(3).standard_normal((30, 30))
    d = ctx.decompose(x, (5, 5), 3)
    with pytest.raises(S.SsaError):
        d.rforecast([0], 5)            # a 2D window: no recurrent forecast
    y = np.random.default_rng(4).standard_normal(200)
    e = ctx.decompose(y, 50, 3)
    with pytest.raises(S.SsaError):
        e.rforecast([0, 5], 5)         # component beyond r


def test_literal_groups_series(ctx):
    """The 1D workload's own groups {1-2},{3-4},{5} split near-degenerate
    sine pairs; their error is bounded by tol * s_1 / gap of each split."""
    w = W.series_1d()
    sh, so, Uo, Vo = oracle_case("series_1000", w)
    d = gpu_case(ctx, w, "fp64")
    rec = d.reconstruct(w["groups"])
    for k, g in enumerate(w["groups"]):
        ref = oracle.reconstruct(sh, so, Uo, Vo, g)
        gap = min(so[i] - so[i + 1] for i in range(max(g[0] - 1, 0), g[-1] + 1))
        e = np.linalg.norm(rec[k][:, 0] - ref[:, 0]) / np.linalg.norm(w["x"])
        assert e <= C_SUB * 1e-10 * so[0] / gap, (g, e)


def test_window_set_order_and_nan_pattern(ctx):
    w = W.small_shaped()
    sh, so, Uo, Vo = oracle_case("small_shaped", w)
    d = gpu_case(ctx, w, "fp64")
    U, V = d.vectors()
    assert np.array_equal(~np.isnan(U[0]), oracle.grid(sh, np.ones(sh.L), "L") == 1)
    assert np.array_equal(~np.isnan(V[0]), oracle.grid(sh, np.ones(sh.K), "K") == 1)
    assert (d.L, d.K) == (sh.L, sh.K)


def test_column_window_is_transposed_row_case(ctx):
    """An Lx x 1 window on an image (runs through the transposed row family)."""
    g = np.random.default_rng(31)
    x = g.standard_normal((57, 23)) + np.cos(np.arange(57) / 3.0)[:, None]
    x[5, 7] = np.nan
    sh, so, Uo, Vo = oracle.decompose(x, window=(20, 1))
    d = ctx.decompose(x, (20, 1), 6)
    assert sigma_err(d.sigma, so) <= 1e-10
    rec = d.reconstruct([[0], [1, 2]])
    for k, grp in enumerate([[0], [1, 2]]):
        ref = oracle.reconstruct(sh, so, Uo, Vo, grp)
        assert np.array_equal(np.isnan(rec[k]), np.isnan(ref))


def test_row_window_on_image(ctx):
    g = np.random.default_rng(32)
    x = g.standard_normal((19, 64)) + np.cos(np.arange(64) / 4.0)[None, :]
    sh, so, Uo, Vo = oracle.decompose(x, window=(1, 25))
    d = ctx.decompose(x, (1, 25), 5)
    assert sigma_err(d.sigma, so) <= 1e-10


def test_origin_side_basis(ctx):
    """|K| < |L|: the bidiagonalisation keeps its basis on the origin side."""
    w = W.image_2d(n=40, lw=28, r=8, seed=12)
    sh, so, Uo, Vo = oracle.decompose(w["x"], window=(28, 28))
    d = ctx.decompose(w["x"], (28, 28), 8)
    assert d.stats["side"] == 1
    assert sigma_err(d.sigma, so) <= 1e-10
    rec = d.reconstruct([[0, 1, 2, 3]])
    ref = oracle.reconstruct(sh, so, Uo, Vo, [0, 1, 2, 3])
    assert np.allclose(rec[0], ref, atol=1e-8, equal_nan=True)


def test_max_rank_and_tiny(ctx):
    x = np.random.default_rng(5).standard_normal(12)
    sh, so, Uo, Vo = oracle.decompose(x, window=5)
    d = ctx.decompose(x, 5, 4)            # r = min(L, K) - 1
    assert sigma_err(d.sigma, so) <= 1e-10


def test_sine_closed_form_degenerate_pair(ctx):
    """A cos with L w and K w integers: sigma_1 = sigma_2 = A sqrt(LK)/2
    exactly (a degenerate pair), rank 2."""
    n, L, A = 959, 480, 1.7
    t = np.arange(n)
    x = A * np.cos(2 * np.pi * t / 12 + 0.4)
    d = ctx.decompose(x, L, 3)
    K = n - L + 1
    s = d.sigma
    ref = A * np.sqrt(L * K) / 2
    assert abs(s[0] - ref) <= 1e-10 * ref and abs(s[1] - ref) <= 1e-10 * ref
    assert s[2] <= 1e-9 * ref


def test_exponential_rank_one(ctx):
    n, L, a = 60, 25, 0.93
    x = a ** np.arange(1, n + 1)
    d = ctx.decompose(x, L, 2)
    K = n - L + 1
    ref = a * np.sqrt(np.sum(a ** (2 * np.arange(L)))) * np.sqrt(np.sum(a ** (2 * np.arange(K))))
    s = d.sigma
    assert abs(s[0] - ref) <= 1e-12 * ref
    assert s[1] <= 1e-10 * ref


def test_alone_equals_in_batch(ctx):
    """A request gives bit-identical results alone and inside a batch."""
    ws = [W.image_2d(n=100, lw=12, r=8, seed=s) for s in (40, 41, 42)]
    reqs = [dict(x=w["x"], window=w["window"], r=8) for w in ws]
    alone = ctx.decompose_batch(reqs[1:2])[0]
    mix = ctx.decompose_batch(reqs)[1]
    assert np.array_equal(alone.sigma, mix.sigma)
    ua, va = alone.vectors()
    um, vm = mix.vectors()
    assert np.array_equal(ua, um, equal_nan=True) and np.array_equal(va, vm, equal_nan=True)
    ra = alone.reconstruct([[0, 1], [2]])
    rm = mix.reconstruct([[0, 1], [2]])
    assert np.array_equal(ra, rm, equal_nan=True)


def _mixed_requests():
    """Requests of different sizes and shapes in two kernel classes: four
    images (square, oblong, transposed window box, shaped with holes and a
    disc window) with r = 8 and three series of different lengths with
    r = 6."""
    big = W.image_2d(n=128, lw=12, r=8, seed=70)["x"]
    rng = np.random.default_rng(71)
    imgs = [big[:96, :96], big[:100, :112], big[:120, :90], big[5:95, 10:110].copy()]
    imgs[3][rng.random(imgs[3].shape) < 0.02] = np.nan
    wi, wj = np.mgrid[0:13, 0:13]
    disc = ((wi - 6) ** 2 + (wj - 6) ** 2 <= 36).astype(np.uint8)
    reqs = [dict(x=imgs[0], window=(12, 12), r=8), dict(x=imgs[1], window=(12, 12), r=8),
            dict(x=imgs[2], window=(10, 14), r=8), dict(x=imgs[3], window=(13, 13), wmask=disc, r=8)]
    for n in (700, 800, 900):
        reqs.append(dict(x=W.series_1d(n=n, L=n // 3, r=6, seed=n)["x"], window=n // 3, r=6))
    return reqs


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_mixed_sizes_alone_equal_in_batch(ctx, prec):
    """Requests of different sizes share one batch per kernel class; each
    result is bit-identical to the request decomposed alone, and matches the
    oracle."""
    reqs = _mixed_requests()
    mix = ctx.decompose_batch(reqs, precision=prec)
    assert [d.stats["batch"] for d in mix] == [4, 4, 4, 4, 3, 3, 3]
    for q, m in zip(reqs, mix):
        a = ctx.decompose_batch([q], precision=prec)[0]
        assert a.stats["batch"] == 1
        assert np.array_equal(a.sigma, m.sigma)
        ua, va = a.vectors()
        um, vm = m.vectors()
        assert np.array_equal(ua, um, equal_nan=True) and np.array_equal(va, vm, equal_nan=True)
        assert np.array_equal(a.reconstruct([[0, 1], [2]]), m.reconstruct([[0, 1], [2]]), equal_nan=True)
        _, so, _, _ = oracle.decompose(q["x"], None, q.get("wmask"), q["window"])
        assert sigma_err(m.sigma, so) <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_column_configurations_agree(prec, monkeypatch):
    """Every column configuration the tuner can pick (tile width x kernel
    variant) computes the same column transforms: the results match the
    oracle and each other (the variants differ only in where twiddles and
    exchanges live, so only the compiler's choice of fused multiply-adds can
    differ: agreement to rounding, not bit for bit)."""
    import paper_1309_5050_amd as S
    w = W.image_2d(n=128, lw=16, r=6, seed=90)       # column transforms of length 128
    _, so, _, _ = oracle.decompose(w["x"], None, None, (16, 16))
    cfgs = [2, 4, 2 + 256, 4 + 256] if prec == "fp64" else [4, 8, 16, 4 + 256, 8 + 256, 16 + 256]
    ref = None
    for cfg in cfgs:
        monkeypatch.setenv("SHSSA_COL_TILE", str(cfg))
        c = S.Context(0)
        try:
            d = c.decompose(w["x"], (16, 16), 6, precision=prec)
            sig, rec = d.sigma, d.reconstruct([[0, 1]])
            d.free()
        finally:
            c.close()
        assert sigma_err(sig, so) <= TOL[prec], cfg
        if ref is None:
            ref = (sig, rec)
        else:
            assert sigma_err(sig, ref[0]) <= TOL[prec], cfg
            assert np.array_equal(np.isnan(rec), np.isnan(ref[1])), cfg
            scale = np.linalg.norm(np.nan_to_num(w["x"]))
            assert np.linalg.norm(np.nan_to_num(rec - ref[1])) <= 20 * TOL[prec] * scale, cfg


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_replayed_steps_equal_launched_steps(prec, monkeypatch):
    """The captured bidiagonalisation step replayed from a graph (the step
    index read from the device counter) gives the same results, bit for
    bit, as the same steps launched one kernel at a time; with timing
    switched on, sampled steps run outside the graph between replays."""
    import paper_1309_5050_amd as S
    reqs = _mixed_requests()
    out = {}
    for mode in ("0", "1", "timed"):
        monkeypatch.setenv("SHSSA_GRAPHS", "0" if mode == "0" else "1")
        c = S.Context(0)
        try:
            if mode == "timed":
                c.profile("col,row_mid,lz_proj", every=3)
            ds = c.decompose_batch(reqs, precision=prec)
            out[mode] = [(d.sigma, d.reconstruct([[0, 1], [2]])) for d in ds]
            if mode == "timed":
                prof = c.profile_read(["col", "row_mid", "lz_proj"])
                assert all(p["launches"] > 0 for p in prof.values())
            for d in ds:
                d.free()
        finally:
            c.close()
    for mode in ("1", "timed"):
        for (s0, r0), (s1, r1) in zip(out["0"], out[mode]):
            assert np.array_equal(s0, s1) and np.array_equal(r0, r1, equal_nan=True)


def test_errors(ctx):
    import paper_1309_5050_amd as S
    x = np.random.default_rng(1).standard_normal((20, 20))
    with pytest.raises(S.SsaError) as e:
        ctx.decompose(x, (5, 5), 25)                  # r >= min(L, K)
    assert e.value.code == -3
    with pytest.raises(S.SsaError) as e:
        ctx.decompose(x, (21, 2), 2)                  # window beyond the array
    assert e.value.code == -1
    y = x.copy()
    y[::3, :] = np.nan                                # no 5x5 window fits
    with pytest.raises(S.SsaError) as e:
        ctx.decompose(y, (5, 5), 2)
    assert e.value.code == -2
    with pytest.raises(S.SsaError) as e:
        ctx.decompose(np.full((10, 10), np.nan), (3, 3), 1)
    assert e.value.code == -2
    with pytest.raises(S.SsaError) as e:
        ctx.decompose(x, (1, 1), 1)                   # window of one cell
    assert e.value.code == -1
    d = ctx.decompose(x, (5, 5), 3)
    with pytest.raises(S.SsaError) as e:
        d.reconstruct([[0, 25]])                      # beyond min(L, K): no continuation
    assert e.value.code == -3
    import ctypes as C
    from paper_1309_5050_amd import _native
    gp, gi = np.array([0, 2], np.int32), np.array([0, 7], np.int32)
    out = np.zeros((1, 20, 20))
    rc = _native.lib().ssa_reconstruct(d.handle, gp.ctypes.data, gi.ctypes.data, 1, out.ctypes.data)
    assert rc == -1                                   # the C call does not continue by itself


def test_device_inputs_match_host(ctx):
    torch = pytest.importorskip("torch")
    ws = [W.image_2d(n=96, lw=10, r=6, seed=s) for s in (60, 61)]
    xs = [torch.tensor(w["x"], device="cuda:0") for w in ws]
    ctx.set_stream(torch.cuda.current_stream().cuda_stream)
    dev = ctx.decompose_batch_dev(xs, (10, 10), 6)
    host = ctx.decompose_batch([dict(x=w["x"], window=(10, 10), r=6) for w in ws])
    for a, b in zip(dev, host):
        assert np.array_equal(a.sigma, b.sigma)
    outs = [torch.empty((2, 96, 96), dtype=torch.float64, device="cuda:0") for _ in ws]
    ctx.reconstruct_batch_dev(dev, [[0, 1], [2, 3]], outs)
    torch.cuda.synchronize()
    for o, b in zip(outs, host):
        assert np.array_equal(o.cpu().numpy(), b.reconstruct([[0, 1], [2, 3]]), equal_nan=True)


def test_handle_outlives_its_stream():
    """A handle whose work went to the context's own stream stays usable and
    can be freed after set_stream has replaced (and destroyed) that stream:
    a call leaves an event behind its work, not the stream."""
    torch = pytest.importorskip("torch")
    import paper_1309_5050_amd as S
    c = S.Context(0)
    try:
        w = W.image_2d(n=96, lw=12, r=6, seed=77)
        d = c.decompose(w["x"], (12, 12), 6)
        s = torch.cuda.Stream()
        c.set_stream(s.cuda_stream)          # the library's own stream is destroyed here
        sig = d.sigma                        # waits on the handle's event
        assert np.all(np.diff(sig) <= 0)
        rec = d.reconstruct([[0, 1]])
        assert np.isfinite(np.nanmax(rec))
        d.free()
        torch.cuda.synchronize()
    finally:
        c.close()


def _vforecast_oracle(name, w, group, h):
    sh, so, Uo, Vo = oracle_case(name, w)
    lens = [len(x) for x in w["x"]] if w["kind"] == "mssa" else [len(w["x"])]
    return oracle.vforecast_column(lens, w["window"], so, Uo, Vo, group, h), so


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name,group", [("series_1000", [0, 1, 2, 3, 4, 5]), ("mssa_8", [0, 1, 2, 3])])
def test_vforecast_parity(ctx, name, group, prec):
    """Column vector forecast (24 values) from the GPU decomposition against
    the oracle's (its projector definition on the oracle's triplets), with
    the bound of the recurrent forecast: the group's span and coefficients
    are within 20 tol s_1 / gap of the oracle's, relative to the largest
    forecast value."""
    w = CASES[name]()
    tol = TOL[prec]
    h = 24
    ref, so = _vforecast_oracle(name, w, group, h)
    d = gpu_case(ctx, w, prec)
    got = d.vforecast(group, h)
    assert got.shape == ref.shape
    gap = so[group[-1]] - so[group[-1] + 1]
    bound = 20 * tol * so[0] / gap * np.max(np.abs(ref))
    err = np.max(np.abs(got - ref))
    print(f"{name} {prec}: vector forecast error {err:.3e} bound {bound:.3e}")
    assert err <= bound, (name, prec, err, bound)


def test_vforecast_continues_a_cosine(ctx):
    """A pure cosine (rank 2) lies in its signal subspace: the vector
    forecast continues it exactly, as the recurrent one does."""
    N, L, h = 300, 120, 40
    t = np.arange(N + h)
    x = 2.0 * np.cos(2 * np.pi * t / 15 + 0.3)
    d = ctx.decompose(x[:N], L, 2)
    f = d.vforecast([0, 1], h)[0]
    assert np.max(np.abs(f - x[N:])) <= 1e-8
    assert np.max(np.abs(f - d.rforecast([0, 1], h)[0])) <= 1e-8


def test_vforecast_longer_horizon_extends_shorter(ctx):
    w = CASES["mssa_8"]()
    d = gpu_case(ctx, w, "fp64")
    a = d.vforecast([0, 1, 2], 10)
    b = d.vforecast([0, 1, 2], 31)
    assert np.max(np.abs(a - b[:, :10])) <= 1e-12 * np.max(np.abs(b))


def test_vforecast_errors(ctx):
    import paper_1309_5050_amd as S
    x = np.random.default_rng(3).standard_normal((30, 30))
    d = ctx.decompose(x, (5, 5), 3)
    with pytest.raises(S.SsaError):
        d.vforecast([0], 5)            # a 2D window: no vector forecast
    y = np.random.default_rng(4).standard_normal(200)
    e = ctx.decompose(y, 50, 3)
    with pytest.raises(S.SsaError):
        e.vforecast([0, 5], 5)         # component beyond r


def test_vforecast_starts_after_the_last_covered_value(ctx):
    """Values after a gap too short for a window are outside every lagged
    vector: the forecast follows the last covered value, as for the series
    cut there."""
    t = np.arange(200)
    y = 3.0 * np.cos(2 * np.pi * t / 17) + 0.1 * np.random.default_rng(8).standard_normal(200)
    y2 = y.copy()
    y2[197] = np.nan
    a = ctx.decompose(y[:197], 50, 4).vforecast([0, 1], 6)
    b = ctx.decompose(y2, 50, 4).vforecast([0, 1], 6)
    assert np.max(np.abs(a - b)) <= 1e-8 * np.max(np.abs(a))


def _row_forecast_oracle(name, w, group, h, kind):
    sh, so, Uo, Vo = oracle_case(name, w)
    L = w["window"]
    lens = [len(x) for x in w["x"]] if w["kind"] == "mssa" else [len(w["x"])]
    if kind == "vector":
        return oracle.vforecast_row(lens, L, so, Uo, Vo, group, h), so
    recs = oracle.reconstruct_mssa(lens, L, so, Uo, Vo, group)
    return oracle.rforecast_row(recs, L, Vo, group, h), so


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("kind", ["recurrent", "vector"])
@pytest.mark.parametrize("name,group", [("series_1000", [0, 1, 2, 3, 4, 5]), ("mssa_8", [0, 1, 2, 3])])
def test_row_forecast_parity(ctx, name, group, kind, prec):
    """Row forecasts (24 values) from the GPU decomposition against the
    oracle's definitions on its own triplets, with the bound of the column
    forecasts (the group's row space is as close to the oracle's as its
    column space)."""
    w = CASES[name]()
    tol = TOL[prec]
    h = 24
    ref, so = _row_forecast_oracle(name, w, group, h, kind)
    d = gpu_case(ctx, w, prec)
    got = (d.vforecast if kind == "vector" else d.rforecast)(group, h, direction="row")
    assert got.shape == ref.shape
    gap = so[group[-1]] - so[group[-1] + 1]
    bound = 20 * tol * so[0] / gap * np.max(np.abs(ref))
    err = np.max(np.abs(got - ref))
    print(f"{name} {kind} {prec}: row forecast error {err:.3e} bound {bound:.3e}")
    assert err <= bound, (name, kind, prec, err, bound)


def test_row_forecasts_continue_a_cosine_system(ctx):
    L, h = 40, 30
    lens = [150, 190, 230]
    amp, ph = [1.0, 0.5, 2.0], [0.0, 1.0, 2.5]
    full = [a * np.cos(2 * np.pi * np.arange(n + h) / 13 + p) for a, p, n in zip(amp, ph, lens)]
    d = ctx.decompose_multi([f[:n] for f, n in zip(full, lens)], L, 2)
    for f in (d.rforecast([0, 1], h, direction="row"), d.vforecast([0, 1], h, direction="row")):
        for p, n in enumerate(lens):
            assert np.max(np.abs(f[p] - full[p][n:])) <= 1e-8


def test_row_forecast_errors(ctx):
    import paper_1309_5050_amd as S
    x = np.random.default_rng(3).standard_normal((30, 30))
    d = ctx.decompose(x, (5, 5), 3)
    with pytest.raises(S.SsaError):
        d.rforecast([0], 5, direction="row")
    y = np.cos(np.arange(300) / 5.0) + 0.1 * np.random.default_rng(4).standard_normal(300)
    y[150] = np.nan                    # a gap: the trajectory rows are no longer Hankel blocks
    e = ctx.decompose(y, 40, 3)
    with pytest.raises(S.SsaError):
        e.vforecast([0, 1], 5, direction="row")
    with pytest.raises(S.SsaError):
        e.rforecast([0, 1], 5, direction="row")
    e.vforecast([0, 1], 5)             # the column forecasts need no Hankel rows


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name,r0,r1", [("image_128", 4, 10), ("series_1000", 3, 8), ("mssa_8", 2, 6),
                                        ("small_shaped", 3, 7)])
def test_extend_matches_oracle(ctx, name, r0, r1, prec):
    """A decomposition with r0 triplets continued to r1 (thick restart from
    its resident state) against the oracle's first r1 triplets: sigma within
    tol sigma_1, and the reconstruction of every gap-stable prefix group
    within 20 tol sigma_1 / gap."""
    w = dict(CASES[name]())
    tol = TOL[prec]
    sh, so, Uo, Vo = oracle_case(name, w)
    w["r"] = r0
    d = gpu_case(ctx, w, prec)
    d.extend(r1)
    assert d.r == r1
    s = d.sigma
    assert s.shape == (r1,)
    assert sigma_err(s, so) <= tol, (name, prec, sigma_err(s, so))
    st = d.stats
    assert st["converged"]
    for k in range(2, r1 + 1):
        gap = so[k - 1] - so[k]
        if gap < 1e-3 * so[0]:
            continue
        g = list(range(k))
        got = d.reconstruct([g])[0]
        if w["kind"] == "mssa":
            lens = [len(x) for x in w["x"]]
            ref = oracle.reconstruct_mssa(lens, w["window"], so, Uo, Vo, g)
            num = np.sqrt(sum(np.sum((got[:n, p] - ref[p]) ** 2) for p, n in enumerate(lens)))
            den = np.sqrt(sum(np.sum(x ** 2) for x in w["x"]))
        else:
            x = w["x"] if w["x"].ndim == 2 else w["x"][:, None]
            ref = oracle.reconstruct(sh, so, Uo, Vo, g)
            cov = ~np.isnan(ref)
            num = np.linalg.norm(got[cov] - ref[cov])
            den = np.linalg.norm(np.nan_to_num(x[cov]))
        assert num / den <= C_SUB * tol * so[0] / gap, (name, prec, k, num / den)


def test_reconstruct_continues_the_decomposition(ctx):
    """Asking for components beyond r continues the decomposition (the
    result equals that of a decomposition made with enough triplets)."""
    w = W.series_1d()
    a = ctx.decompose(w["x"], w["window"], 3)
    ra = a.reconstruct([[0, 1, 2, 3, 4, 5]])[0]
    assert a.r == 6
    b = ctx.decompose(w["x"], w["window"], 6)
    rb = b.reconstruct([[0, 1, 2, 3, 4, 5]])[0]
    sh, so, Uo, Vo = oracle_case("series_1000", w)
    gap = so[5] - so[6]
    assert np.max(np.abs(ra - rb)) <= 40 * 1e-10 * so[0] / gap * np.max(np.abs(w["x"]))
    np.testing.assert_allclose(a.sigma, b.sigma, rtol=0, atol=2e-10 * so[0])


def test_extend_twice_and_noop(ctx):
    w = W.image_2d(n=96, lw=10, r=4, seed=70)
    d = ctx.decompose(w["x"], w["window"], 2)
    d.extend(2)                                       # no-op
    assert d.r == 2
    d.extend(5)
    d.extend(9)
    e = ctx.decompose(w["x"], w["window"], 9)
    np.testing.assert_allclose(d.sigma, e.sigma, rtol=0, atol=1e-9 * e.sigma[0])


EIGEN_CASES = {
    "small_shaped": lambda: W.small_shaped(),
    "series_400_L100": lambda: W.series_1d(n=400, L=100, r=8),
    "image_64_w8": lambda: W.image_2d(n=64, lw=8, r=6, seed=41),
    "disc_48_w10x12": lambda: dict(W.shaped_disc(n=48, radius=20.0, lw=10, r=6, hole_r=(1, 2)), window=(10, 12)),
}


@pytest.mark.parametrize("name", list(EIGEN_CASES))
def test_eigen_method_matches_oracle(ctx, name):
    """The eigen method (S = X X^T on the matrix cores, eigenpairs by
    Jacobi) against the oracle: sigma within tol sigma_1 wherever sigma_i is
    large enough for the squared matrix to resolve it (sigma_i >= 1e-3
    sigma_1), reconstructions of gap-stable prefix groups within
    20 tol sigma_1 / gap."""
    w = EIGEN_CASES[name]()
    tol = 1e-10
    sh, so, Uo, Vo = oracle.decompose(w["x"], w["mask"], w["wmask"], w["window"])
    r = min(w["r"], sh.L - 1)
    d = ctx.decompose(w["x"], w["window"], r, mask=w["mask"], wmask=w["wmask"], method="eigen")
    s = d.sigma
    big = so[:r] >= 1e-3 * so[0]
    assert np.max(np.abs(s - so[:r])[big]) <= tol * so[0], (name, s, so[:r])
    x = w["x"] if w["x"].ndim == 2 else w["x"][:, None]
    for k in range(1, r):
        gap = so[k - 1] - so[k]
        if gap < 1e-3 * so[0] or not big[k - 1]:
            continue
        g = list(range(k))
        ref = oracle.reconstruct(sh, so, Uo, Vo, g)
        got = d.reconstruct([g])[0]
        assert np.array_equal(np.isnan(got), np.isnan(ref))
        cov = ~np.isnan(ref)
        e = np.linalg.norm(got[cov] - ref[cov]) / np.linalg.norm(np.nan_to_num(x[cov]))
        assert e <= C_SUB * tol * so[0] / gap, (name, k, e)


def test_eigen_method_agrees_with_lanczos_and_extends(ctx):
    w = W.image_2d(n=80, lw=9, r=5, seed=43)
    a = ctx.decompose(w["x"], w["window"], 5, method="eigen")
    b = ctx.decompose(w["x"], w["window"], 5)
    np.testing.assert_allclose(a.sigma, b.sigma, rtol=0, atol=1e-9 * b.sigma[0])
    a.extend(9)
    c = ctx.decompose(w["x"], w["window"], 9, method="eigen")
    assert np.array_equal(a.sigma, c.sigma)          # the same eigenpairs of the same S
    Ua, Va = a.vectors()
    Uc, Vc = c.vectors()
    assert np.allclose(Ua, Uc, atol=1e-12, equal_nan=True)


def test_eigen_method_limits(ctx):
    import paper_1309_5050_amd as S
    x = np.random.default_rng(2).standard_normal((80, 80))
    with pytest.raises(S.SsaError) as e:
        ctx.decompose(x, (65, 65), 3, method="eigen")    # 4225 cells > 4096
    assert e.value.code == -1
    with pytest.raises(ValueError):
        ctx.decompose(x[:40, :40], (5, 5), 3, method="svd")


def _mars_full():
    w = W.mars_like()
    return dict(kind="image", x=np.nan_to_num(w["x"]), mask=None, wmask=None, window=(25, 25), r=50)


# windows beyond the 128 cells of the small-SVD kernel: block Jacobi on S
EIGEN_BIG_CASES = {
    "image_96_w10x20": lambda: W.image_2d(n=96, lw=10, r=12, seed=44) | {"window": (10, 20)},
    "series_300_L250_rankdef": lambda: W.series_1d(n=300, L=250, r=10, seed=45),
    "disc_80_w15x12": lambda: dict(W.shaped_disc(n=80, radius=36.0, lw=15, r=10, hole_r=(1, 2)), window=(15, 12)),
    "mars_like_25x25": _mars_full,
}


@pytest.mark.parametrize("name", list(EIGEN_BIG_CASES))
def test_eigen_method_large_windows_match_oracle(ctx, name):
    """The eigen method for windows of more than 128 cells (the paper's
    25 x 25 window on its 258 x 275 image: S is 625 x 625 beside a 625 x 58734
    trajectory matrix), S's eigenpairs by block Jacobi, against the oracle's
    eigenpairs of S = X X^T: sigma within 1e-10 sigma_1 where sigma_i >= 1e-3
    sigma_1 (a squared matrix resolves no more), spans and reconstructions of
    gap-stable prefix groups within 20 tol sigma_1 / gap; a rank-deficient S
    (L > K) included."""
    w = EIGEN_BIG_CASES[name]()
    tol = 1e-10
    sh, so, Uo, Vo = oracle.decompose(w["x"], w["mask"], w["wmask"], w["window"], method="gram", nvec=12)
    assert sh.L > 128
    r = min(w["r"], sh.L - 1, sh.K - 1)
    d = ctx.decompose(w["x"], w["window"], r, mask=w["mask"], wmask=w["wmask"], method="eigen")
    st = d.stats
    print(f"{name}: L={sh.L} K={sh.K} sweeps {st['svd_sweeps']} converged {st['converged']}")
    assert st["converged"] == 1
    s = d.sigma
    big = so[:r] >= 1e-3 * so[0]
    assert np.max(np.abs(s - so[:r])[big]) <= tol * so[0], (name, np.max(np.abs(s - so[:r])[big]) / so[0])
    U, _ = d.vectors_lex()
    x = w["x"] if w["x"].ndim == 2 else w["x"][:, None]
    for k in range(1, min(r, 12)):
        gap = so[k - 1] - so[k]
        if gap < 1e-3 * so[0] or not big[k - 1]:
            continue
        g = list(range(k))
        assert proj_dist(U[:, g], Uo[:, g]) <= C_SUB * tol * so[0] / gap, (name, k)
        ref = oracle.reconstruct(sh, so, Uo, Vo, g)
        got = d.reconstruct([g])[0]
        assert np.array_equal(np.isnan(got), np.isnan(ref))
        cov = ~np.isnan(ref)
        e = np.linalg.norm(got[cov] - ref[cov]) / np.linalg.norm(np.nan_to_num(x[cov]))
        assert e <= C_SUB * tol * so[0] / gap, (name, k, e)


def test_eigen_method_large_window_extends(ctx):
    """A continuation of a large-window eigen decomposition takes further
    eigenpairs of the resident rotated S: identical to asking for them at
    once."""
    w = W.image_2d(n=96, lw=10, r=6, seed=46)
    a = ctx.decompose(w["x"], (12, 14), 6, method="eigen")
    a.extend(11)
    c = ctx.decompose(w["x"], (12, 14), 11, method="eigen")
    assert np.array_equal(a.sigma, c.sigma)
    Ua, _ = a.vectors()
    Uc, _ = c.vectors()
    assert np.allclose(Ua, Uc, atol=1e-12, equal_nan=True)
    b = ctx.decompose(w["x"], (12, 14), 11)
    np.testing.assert_allclose(a.sigma, b.sigma, rtol=0, atol=1e-9 * b.sigma[0])


def _m2d_case(seed=53):
    g = np.random.default_rng(seed)
    imgs = []
    for nx, ny in [(40, 33), (36, 45), (48, 27)]:
        i, j = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
        imgs.append(2.0 * np.cos(0.5 * i + 0.2 * j) + np.cos(0.9 * j) + 0.3 * g.standard_normal((nx, ny)))
    return imgs


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("hollow", [False, True])
def test_m2d_matches_oracle(ctx, prec, hollow):
    """M-2D-SSA of three images of different sizes: sigma against the SVD of
    the stacked trajectory matrix [T(X_1) : T(X_2) : T(X_3)] (the oracle's
    definition), reconstructions against the oracle's on its own packing."""
    imgs = _m2d_case()
    tol = TOL[prec]
    window = (6, 5)
    wmask = None
    if hollow:
        wmask = np.ones(window, np.uint8)
        wmask[2:4, 1:4] = 0
    r = 6
    X = oracle.trajectory_m2d(imgs, window, wmask)
    so = oracle.svd(X)[0]
    d = ctx.decompose_m2d(imgs, window, r, wmask=wmask, precision=prec)
    assert sigma_err(d.sigma, so) <= tol, (prec, hollow, sigma_err(d.sigma, so))
    packed = oracle.pack_m2d(imgs, window, wmask)
    sh, so2, Uo, Vo = oracle.decompose(packed, None, wmask, window)
    np.testing.assert_allclose(so2[:r], so[:r], rtol=0, atol=1e-12 * so[0])
    for k in range(1, r):
        gap = so2[k - 1] - so2[k]
        if gap < 1e-3 * so2[0]:
            continue
        g = list(range(k))
        ref = oracle.reconstruct(sh, so2, Uo, Vo, g)
        got = d.reconstruct([g])[0]
        assert got.shape == packed.shape
        assert np.array_equal(np.isnan(got), np.isnan(ref))
        cov = ~np.isnan(ref)
        e = np.linalg.norm(got[cov] - ref[cov]) / np.linalg.norm(np.nan_to_num(packed[cov]))
        assert e <= C_SUB * tol * so2[0] / gap, (prec, hollow, k, e)
    parts = d.unpack(d.reconstruct([[0, 1]]))
    assert [p.shape[-2:] for p in parts] == [x.shape for x in imgs]


def _nearest_match(a, b):
    b = list(b)
    worst = 0.0
    for z in a:
        k = int(np.argmin([abs(z - w) for w in b]))
        worst = max(worst, abs(z - b[k]))
        b.pop(k)
    return worst


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name,group", [("series_1000", [0, 1, 2, 3, 4, 5]), ("mssa_8", [0, 1, 2, 3])])
def test_esprit_parity(ctx, name, group, prec):
    """LS-ESPRIT roots from the GPU decomposition against the oracle's roots
    of its own triplets, within the bound on the group's span, 20 tol s_1 /
    gap (the roots of these well-conditioned shift matrices move no more
    than their span)."""
    w = CASES[name]()
    tol = TOL[prec]
    sh, so, Uo, Vo = oracle_case(name, w)
    ref = oracle.esprit(Uo, group)
    d = gpu_case(ctx, w, prec)
    got = d.esprit(group)
    assert got.shape == ref.shape
    gap = so[group[-1]] - so[group[-1] + 1]
    err = _nearest_match(got, ref)
    bound = 20 * tol * so[0] / gap
    print(f"{name} {prec}: ESPRIT root error {err:.3e} bound {bound:.3e}")
    assert err <= bound, (name, prec, err, bound)
    mods = np.abs(got)
    assert np.all(mods[:-1] >= mods[1:] - 1e-15)


def test_esprit_recovers_damped_cosines(ctx):
    N, L = 240, 80
    t = np.arange(N)
    x = 2.0 * 0.99 ** t * np.cos(2 * np.pi * t / 10 + 0.3) + np.cos(2 * np.pi * t / 23) + 0.5 * 1.005 ** t
    d = ctx.decompose(x, L, 5)
    z = d.esprit([0, 1, 2, 3, 4])
    true = [0.99 * np.exp(2j * np.pi / 10), 0.99 * np.exp(-2j * np.pi / 10), np.exp(2j * np.pi / 23),
            np.exp(-2j * np.pi / 23), 1.005]
    assert _nearest_match(z, true) <= 1e-8


def test_esprit_errors(ctx):
    import paper_1309_5050_amd as S
    x = np.random.default_rng(3).standard_normal((30, 30))
    d = ctx.decompose(x, (5, 5), 3)
    y = np.random.default_rng(4).standard_normal(200)
    e = ctx.decompose(y, 50, 3)
    for method in ("ls", "tls"):
        with pytest.raises(S.SsaError):
            d.esprit([0, 1], method)   # a 2D window
        with pytest.raises(S.SsaError):
            e.esprit([0, 7], method)   # component beyond r
    f = ctx.decompose(y, 60, 30)
    with pytest.raises(S.SsaError):
        f.esprit(list(range(25)), "tls")   # beyond the 24 roots TLS solves


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name,group", [("series_1000", [0, 1, 2, 3, 4, 5]), ("mssa_8", [0, 1, 2, 3]),
                                        ("series_1000", [1, 2])])
def test_esprit_tls_parity(ctx, name, group, prec):
    """TLS-ESPRIT roots from the GPU decomposition against the oracle's
    TLS roots of its own triplets, within the same span bound as LS-ESPRIT
    (20 tol s_1 / gap, the gap after the group's last component)."""
    w = CASES[name]()
    tol = TOL[prec]
    sh, so, Uo, Vo = oracle_case(name, w)
    ref = oracle.esprit_tls(Uo, group)
    d = gpu_case(ctx, w, prec)
    got = d.esprit(group, "tls")
    assert got.shape == ref.shape
    gap = min(so[group[-1]] - so[group[-1] + 1], so[group[0] - 1] - so[group[0]] if group[0] > 0 else np.inf)
    err = _nearest_match(got, ref)
    bound = 20 * tol * so[0] / gap
    print(f"{name} {group} {prec}: TLS-ESPRIT root error {err:.3e} bound {bound:.3e}")
    assert err <= bound, (name, prec, err, bound)
    mods = np.abs(got)
    assert np.all(mods[:-1] >= mods[1:] - 1e-15)


def test_esprit_tls_recovers_damped_cosines(ctx):
    """On an exact rank-5 series TLS and LS agree with the true roots."""
    N, L = 240, 80
    t = np.arange(N)
    x = 2.0 * 0.99 ** t * np.cos(2 * np.pi * t / 10 + 0.3) + np.cos(2 * np.pi * t / 23) + 0.5 * 1.005 ** t
    d = ctx.decompose(x, L, 5)
    z = d.esprit([0, 1, 2, 3, 4], "tls")
    true = [0.99 * np.exp(2j * np.pi / 10), 0.99 * np.exp(-2j * np.pi / 10), np.exp(2j * np.pi / 23),
            np.exp(-2j * np.pi / 23), 1.005]
    assert _nearest_match(z, true) <= 1e-8
    assert _nearest_match(z, d.esprit([0, 1, 2, 3, 4])) <= 1e-8


def test_esprit_tls_largest_group(ctx):
    """24 roots (the largest TLS group) from a noisy series against the
    oracle's TLS roots of the GPU's own basis, so that only the small
    eigenproblems are compared."""
    g = np.random.default_rng(11)
    N, L = 600, 150
    t = np.arange(N)
    x = sum(g.uniform(0.5, 2) * np.cos(2 * np.pi * t / g.uniform(2.5, 60) + g.uniform(0, 6)) for _ in range(12))
    x = x + 0.05 * g.standard_normal(N)
    d = ctx.decompose(x, L, 30)
    U, _ = d.vectors_lex()
    grp = list(range(24))
    ref = oracle.esprit_tls(U, grp)
    got = d.esprit(grp, "tls")
    err = _nearest_match(got, ref)
    print(f"24-root TLS-ESPRIT: {err:.3e}")
    assert err <= 1e-9, err


def _pairs_nearest(l1, m1, l2, m2):
    b = list(zip(l2, m2))
    worst = 0.0
    for a in zip(l1, m1):
        d = [max(abs(a[0] - c[0]), abs(a[1] - c[1])) for c in b]
        k = int(np.argmin(d))
        worst = max(worst, d[k])
        b.pop(k)
    return worst


def _planar_waves(noise, seed=2):
    nx, ny = 40, 36
    m, n = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    x = (np.cos(2 * np.pi * (0.11 * m + 0.07 * n) + 0.4)
         + 0.97 ** m * 0.99 ** n * 2 * np.cos(2 * np.pi * (0.04 * m + 0.19 * n)))
    return x + noise * np.random.default_rng(seed).standard_normal((nx, ny))


def _hollow_window():
    wm = np.ones((8, 7), np.uint8)
    wm[3:5, 2:4] = 0
    return wm


@pytest.mark.parametrize("hollow", [False, True])
def test_esprit2d_recovers_planar_waves(ctx, hollow):
    x = _planar_waves(0.0)
    wm = _hollow_window() if hollow else None
    d = ctx.decompose(x, (8, 7), 4, wmask=wm)
    lam, mu = d.esprit2d([0, 1, 2, 3])
    true_l = [np.exp(2j * np.pi * 0.11), np.exp(-2j * np.pi * 0.11), 0.97 * np.exp(2j * np.pi * 0.04),
              0.97 * np.exp(-2j * np.pi * 0.04)]
    true_m = [np.exp(2j * np.pi * 0.07), np.exp(-2j * np.pi * 0.07), 0.99 * np.exp(2j * np.pi * 0.19),
              0.99 * np.exp(-2j * np.pi * 0.19)]
    assert _pairs_nearest(lam, mu, true_l, true_m) <= 1e-8


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("hollow", [False, True])
def test_esprit2d_parity(ctx, prec, hollow):
    """2D-ESPRIT pairs from the GPU decomposition of a noisy image against
    the oracle's pairs of its own triplets, within the bound on the group's
    span, 20 tol s_1 / gap."""
    x = _planar_waves(0.05)
    wm = _hollow_window() if hollow else None
    tol = TOL[prec]
    sh, so, Uo, Vo = oracle.decompose(x, None, wm, (8, 7))
    lam_o, mu_o = oracle.esprit2d(sh, Uo, [0, 1, 2, 3])
    d = ctx.decompose(x, (8, 7), 6, wmask=wm, precision=prec)
    lam, mu = d.esprit2d([0, 1, 2, 3])
    gap = so[3] - so[4]
    err = _pairs_nearest(lam, mu, lam_o, mu_o)
    bound = 20 * tol * so[0] / gap
    print(f"hollow={hollow} {prec}: 2D-ESPRIT pair error {err:.3e} bound {bound:.3e}")
    assert err <= bound, (hollow, prec, err, bound)


def test_esprit2d_errors(ctx):
    import paper_1309_5050_amd as S
    y = np.random.default_rng(4).standard_normal(200)
    e = ctx.decompose(y, 50, 3)
    with pytest.raises(S.SsaError):
        e.esprit2d([0, 1])             # a 1D window
    x = _planar_waves(0.05)
    d = ctx.decompose(x, (8, 7), 4)
    with pytest.raises(S.SsaError):
        d.esprit2d([0, 9])             # component beyond r


@pytest.mark.parametrize("prec,bound", [("fp32", 1e-10), ("fp32_basis32", 1e-6)])
@pytest.mark.parametrize("name", ["image_128", "series_1000", "disc_160"])
def test_fp32_vectors_stay_orthonormal(ctx, name, prec, bound):
    """FP32-product decompositions reorthogonalise in FP64: their
    Lanczos-side vectors are orthonormal to FP64 rounding.  With the FP32
    copy of the basis (SSA_FP32_BASIS32) the copy's rounding bounds the
    orthogonality at about 1e-7, still far inside the 1e-5 tolerance."""
    w = CASES[name]()
    if w["kind"] == "mssa":
        d = ctx.decompose_multi(w["x"], w["window"], w["r"], precision=prec)
    else:
        d = ctx.decompose(w["x"], w["window"], w["r"], mask=w["mask"], wmask=w["wmask"], precision=prec)
    U, V = d.vectors_lex()
    side = d.stats["side"]
    B = U if side == 0 else V
    err = np.max(np.abs(B.T @ B - np.eye(B.shape[1])))
    print(f"{name} {prec}: |B^T B - I| = {err:.2e} (side {side})")
    assert err <= bound, (name, prec, err)


@pytest.mark.parametrize("name", ["image_128", "disc_160", "mssa_8"])
def test_fp32_basis32_parity(ctx, name):
    """The opt-in FP32 basis copy keeps the FP32 tolerance against the oracle."""
    w = CASES[name]()
    sh, so, Uo, Vo = oracle_case(name, w)
    if w["kind"] == "mssa":
        d = ctx.decompose_multi(w["x"], w["window"], w["r"], precision="fp32_basis32")
    else:
        d = ctx.decompose(w["x"], w["window"], w["r"], mask=w["mask"], wmask=w["wmask"], precision="fp32_basis32")
    assert d.stats["converged"] == 1
    assert sigma_err(d.sigma, so) <= TOL["fp32"]
    U, V = d.vectors_lex()
    for g, gap in stable_groups(so, w["r"]):
        bound = C_SUB * TOL["fp32"] * so[0] / gap
        assert proj_dist(U[:, g], Uo[:, g]) <= bound and proj_dist(V[:, g], Vo[:, g]) <= bound


def _mosaic_case(Ls, Ks, seed=61):
    """Series (i, j): a rank-2 mosaic component a_i b_j cos(0.3 n + p_i + q_j),
    a weaker one of frequency 1.1 and noise."""
    g = np.random.default_rng(seed)
    a, p, a2, p2 = (g.uniform(0.5, 2, len(Ls)), g.uniform(0, 6, len(Ls)), g.uniform(0.2, 0.6, len(Ls)),
                    g.uniform(0, 6, len(Ls)))
    b, q = g.uniform(0.5, 2, len(Ks)), g.uniform(0, 6, len(Ks))
    out = []
    for i, L in enumerate(Ls):
        row = []
        for j, K in enumerate(Ks):
            n = np.arange(L + K - 1)
            row.append(a[i] * b[j] * np.cos(0.3 * n + p[i] + q[j]) + a2[i] * np.cos(1.1 * n + p2[i] + q[j])
                       + 0.1 * g.standard_normal(len(n)))
        out.append(row)
    return out


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("Ls,Ks", [([12, 7, 15], [40, 25, 33]), ([30], [60]), ([9], [50, 41, 70]), ([6, 14, 9, 11], [45])])
def test_mosaic_matches_oracle(ctx, prec, Ls, Ks):
    """Mosaic Hankel SSA: sigma against the SVD of the explicit mosaic matrix
    (the oracle's definition), each series' reconstruction against the
    oracle's block-wise anti-diagonal averages of the same group."""
    ser = _mosaic_case(Ls, Ks)
    tol = TOL[prec]
    r = 6
    M = oracle.mosaic_hankel(ser, Ls, Ks)
    so = np.linalg.svd(M, compute_uv=False)
    d = ctx.decompose_mosaic(ser, Ls, Ks, r, precision=prec)
    assert d.L == sum(Ls) and d.K == sum(Ks)
    assert sigma_err(d.sigma, so) <= tol, (prec, Ls, Ks, sigma_err(d.sigma, so))
    xnorm = np.sqrt(sum(np.sum(x ** 2) for row in ser for x in row))
    checked = 0
    for k in range(1, r):
        gap = so[k - 1] - so[k]
        if gap < 1e-3 * so[0]:
            continue
        g = list(range(k))
        ref = oracle.reconstruct_mosaic(ser, Ls, Ks, g)
        got = d.unpack(d.reconstruct([g])[0])
        e = np.sqrt(sum(np.sum((got[i][j] - ref[i][j]) ** 2) for i in range(len(Ls)) for j in range(len(Ks))))
        assert e / xnorm <= C_SUB * tol * so[0] / gap, (prec, Ls, Ks, k, e / xnorm)
        checked += 1
    assert checked > 0


def test_mosaic_errors(ctx):
    import paper_1309_5050_amd as S
    ser = _mosaic_case([5, 6], [9, 8])
    with pytest.raises(ValueError):
        ctx.decompose_mosaic(ser, [5, 6], [9, 7], 2)       # lengths do not match the sizes
    with pytest.raises(ValueError):
        ctx.decompose_mosaic(ser[:1], [5, 6], [9, 8], 2)   # one block row missing
    bad = [[np.zeros(4 + K - 1) for K in (9, 8)], [np.zeros(0 + K - 1) for K in (9, 8)]]
    with pytest.raises(S.SsaError):
        ctx.decompose_mosaic(bad, [4, 0], [9, 8], 2)       # an empty block row


def test_rank_beyond_the_basis_is_refused(ctx):
    """r > 120 leaves a thick restart no room in the 128-vector basis: the
    request is refused before any kernel is queued, also by a continuation."""
    import paper_1309_5050_amd as S
    x = np.random.default_rng(2).standard_normal((200, 200))
    for r in (121, 128, 130):
        with pytest.raises(S.SsaError) as e:
            ctx.decompose(x, (64, 64), r)
        assert e.value.code == -3
    d = ctx.decompose(x, (64, 64), 12)
    with pytest.raises(S.SsaError) as e:
        d.extend(121)
    assert e.value.code == -3
    d.extend(120)                                     # the largest allowed rank still runs
    assert d.r == 120 and d.stats["converged"] == 1


def test_step_limit_returns_enoconv_with_triplets(ctx, monkeypatch):
    """A bidiagonalisation stopped by the step limit returns SSA_ENOCONV with
    its handle: sigma as far as it got, stats.converged = 0."""
    w = W.series_1d()
    sh, so, Uo, Vo = oracle_case("series_1000", w)
    monkeypatch.setenv("SHSSA_MAX_STEPS", "12")
    res = ctx.decompose_batch([{"x": w["x"], "window": w["window"], "r": w["r"]}])
    d = res[0]
    assert getattr(d, "status", None) == -5
    st = d.stats
    assert st["converged"] == 0 and 0 < st["steps"] <= 12 + 128
    s = d.sigma
    assert np.all(np.isfinite(s)) and s[0] > 0
    assert abs(s[0] - so[0]) <= 1e-3 * so[0]          # the leading value is already close
    monkeypatch.delenv("SHSSA_MAX_STEPS")
    d2 = ctx.decompose_batch([{"x": w["x"], "window": w["window"], "r": w["r"]}])[0]
    assert d2.status == 0 and d2.stats["converged"] == 1


def test_tune_cache_persists_choices(tmp_path, capfd, monkeypatch):
    """The column tuner's choice is written to the cache file and read back by
    a new context, which then does not time the configurations again; the
    results are the same."""
    import paper_1309_5050_amd as S
    path = tmp_path / "tune.txt"
    w = W.config(2, "small")
    monkeypatch.setenv("SHSSA_TUNE_LOG", "1")
    out = []
    for k in range(2):
        c = S.Context(0, tune_cache=path)
        try:
            d = c.decompose(w["x"], w["window"], w["r"], precision="fp32")
            out.append(d.sigma)
            del d
        finally:
            c.close()
        err = capfd.readouterr().err
        timed = "column tuner" in err
        assert timed == (k == 0), err
    lines = [l.split() for l in path.read_text().splitlines()]
    assert any(l[0] == "col" and l[1] == "0" for l in lines), lines
    assert np.array_equal(out[0], out[1])


def _cont_requests(kind):
    if kind == "image":
        out = []
        for i in range(10):
            n = 96 + (i % 3) * 7                      # uneven sizes in one kernel class
            w = W.image_2d(n=n, lw=12, r=8, seed=500 + i)
            out.append({"x": w["x"][:, : n - (i % 2) * 5], "window": (12, 12), "r": 8})
        return out
    out = []
    for i in range(9):
        n = 600 + 37 * i
        w = W.series_1d(n=n, L=200, r=6, seed=600 + i)
        out.append({"x": w["x"], "window": 200, "r": 6})
    return out


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("kind", ["image", "series"])
def test_continuous_batching_equals_alone(ctx, kind, prec):
    """Continuous batching: with 4 slots, the requests of a batch call that
    do not fit start as others finish, in the middle of the batch's run.
    Every request's sigma and vectors are bit-identical to the same request
    decomposed alone."""
    import paper_1309_5050_amd as S
    reqs = _cont_requests(kind)
    c = S.Context(0)
    try:
        c.set_slots(4)
        res = c.decompose_batch(reqs, precision=prec)
    finally:
        c.set_slots(0)
    joined = 0
    for q, d in zip(reqs, res):
        assert not isinstance(d, Exception), d
        assert d.status == 0 and d.stats["converged"] == 1
        alone = ctx.decompose(q["x"], q["window"], q["r"], precision=prec)
        assert np.array_equal(d.sigma, alone.sigma)
        U, V = d.vectors_lex()
        Ua, Va = alone.vectors_lex()
        assert np.array_equal(U, Ua) and np.array_equal(V, Va)
        joined += 1
    assert joined == len(reqs)
    c.close()


def test_continuous_batching_fills_freed_slots(ctx):
    """More requests than slots all finish, and the batch's instances report
    the same step counts as alone (their cycles were not stretched by the
    instances that joined)."""
    import paper_1309_5050_amd as S
    reqs = _cont_requests("image")
    c = S.Context(0)
    c.set_slots(3)
    res = c.decompose_batch(reqs, precision="fp32")
    for q, d in zip(reqs, res):
        alone = ctx.decompose(q["x"], q["window"], q["r"], precision="fp32")
        assert d.stats["steps"] == alone.stats["steps"]
        assert d.stats["restarts"] == alone.stats["restarts"]
    with pytest.raises(S.SsaError):
        c.set_slots(-1)
    c.close()


def test_length_tuner_chooses_persists_and_keeps_parity(tmp_path, capfd, monkeypatch):
    """The length tuner (on for contexts created with SHSSA_LEN_TUNE) times a
    class's natural transform length against its power-of-two alternative (a series of 899 values: half-length 450 or
    512; an image of 110 rows: column length 112 or 128), keeps the faster
    one for the process, appends it to the cache file, and the results at
    the chosen length still match the oracle."""
    import paper_1309_5050_amd as S
    monkeypatch.setenv("SHSSA_TUNE_LOG", "1")
    monkeypatch.setenv("SHSSA_LEN_TUNE", "1")          # read when a context is created
    path = tmp_path / "tune.txt"
    ser = W.series_1d(n=899, L=300, r=6, seed=77)
    img = W.image_2d(n=110, lw=10, r=6, seed=78)
    img["x"] = img["x"][:, :100]
    c = S.Context(0, tune_cache=path)
    try:
        d1 = c.decompose(ser["x"], ser["window"], 6)
        d2 = c.decompose(img["x"], img["window"], 6, precision="fp32")
        err = capfd.readouterr().err
        lines = [x.split() for x in path.read_text().splitlines()]
        for w, d, tol in ((ser, d1, 1e-10), (img, d2, 1e-5)):
            sh, so, Uo, Vo = oracle.decompose(w["x"], None, None, w["window"])
            assert sigma_err(d.sigma, so) <= tol
        assert any(l[:3] == ["rowlen", "1", "450"] and l[3] in ("450", "512") for l in lines), lines
        assert any(l[:3] == ["collen", "0", "112"] and l[3] in ("112", "128") for l in lines), lines
        assert "length tuner: row" in err and "length tuner: col" in err
    finally:
        c.close()
    # a second context finds the classes tuned and reproduces the results
    c2 = S.Context(0, tune_cache=path)
    try:
        e1 = c2.decompose(ser["x"], ser["window"], 6)
        assert "length tuner" not in capfd.readouterr().err
        assert np.array_equal(e1.sigma, d1.sigma)
    finally:
        c2.close()


def test_serving_threads_stay_off_by_default(monkeypatch):
    """Without SHSSA_SERVE_ENGINE the server is cooperative: ssa_submit
    starts no thread (the worker threads stay off until a GPU fault seen
    once on them is explained), and the caller's ssa_wait runs the work."""
    import paper_1309_5050_amd as S
    monkeypatch.delenv("SHSSA_SERVE_ENGINE", raising=False)
    c = S.Context(0)
    try:
        x = np.cos(np.arange(400) / 5.0)
        c.decompose(x, 100, r=2).free()                 # the runtime's own threads start here
        before = len(os.listdir("/proc/self/task"))
        t1 = c.submit(x, 100, r=2)
        t2 = c.submit_multi([x, x], 100, r=2)
        assert len(os.listdir("/proc/self/task")) == before
        for t in (t1, t2):
            c.wait(t)
            d, _, _ = c.take(t, shape=(0,), ngroups=0)
            assert d.status == 0
            d.free()
    finally:
        c.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_long_series_in_segments(ctx, prec):
    """A series longer than one transform row (beyond 2 x 10200 values in
    FP64, 2 x 16384 in FP32) runs as the MSSA of overlapping segments whose
    trajectory matrices side by side are the series' own: sigma, the spans
    of U and V, the weights and the reconstructions equal the oracle's on the
    whole series (a missing value sits in the overlap of two segments)."""
    g = np.random.default_rng(41)
    N, L, r = 41000, 48, 5
    t = np.arange(N)
    x = 2.0 * np.sin(2 * np.pi * t / 37) + np.cos(2 * np.pi * t / 11) + 0.2 * g.standard_normal(N)
    x[16340] = np.nan                       # segment 0 ends at 16383, segment 1 starts at 16337 (FP64)
    sh, so, Uo, Vo = oracle.decompose(x, window=(L, 1))
    d = ctx.decompose(x, L, r, precision=prec)
    tol = TOL[prec]
    assert d.shape == (N, 1) and (d.L, d.K) == (sh.L, sh.K)
    assert sigma_err(d.sigma, so) <= tol
    U, V = d.vectors_lex()
    for grp, gap in stable_groups(so, r):
        c = 10 * tol * so[0] / gap
        assert proj_dist(U[:, grp], Uo[:, grp]) <= c
        assert proj_dist(V[:, grp], Vo[:, grp]) <= c
    Ub, Vb = d.vectors()
    assert Vb.shape == (r, N - L + 1, 1)
    assert np.allclose(np.nan_to_num(Vb[:, :, 0][:, sh.ki]), V.T, rtol=0, atol=0)   # box layout = compact order
    assert np.array_equal(d.weights, sh.W)
    groups = [[0, 1], [2, 3]]
    rec = d.reconstruct(groups)
    for k, grp in enumerate(groups):
        ref = oracle.reconstruct(sh, so, Uo, Vo, grp)
        assert np.array_equal(np.isnan(rec[k]), np.isnan(ref))
        ok = ~np.isnan(ref)
        # near-degenerate pairs: the reconstruction error scales with the
        # pair's gap to the rest of the spectrum
        gap = min(so[grp[0] - 1] - so[grp[0]] if grp[0] else np.inf, so[grp[-1]] - so[grp[-1] + 1])
        bound = 10 * tol * (so[0] / gap) * np.sqrt(np.mean(np.nan_to_num(x) ** 2))
        assert np.max(np.abs(rec[k][ok] - ref[ok])) <= bound
    rho, _ = d.wcor([[0, 1], [2, 3], [4]])
    assert np.allclose(np.diag(rho), 1.0)
    assert abs(rho[0, 1]) < 0.05                               # the two sines are w-separable
    with pytest.raises(Exception):
        d.rforecast([0, 1], 10)


def test_memory_budget_refuses_with_enomem():
    """A context's device-memory budget: a decomposition that does not fit
    fails with SSA_ENOMEM, and the blocks it had taken go back (a small
    request still fits afterwards, and repeating the pair changes nothing).
    In a batch call the refused request is reported on its own while the
    others run."""
    import paper_1309_5050_amd as S
    c = S.Context(0, mem_budget=8 << 20)                 # 8 MiB
    try:
        rng = np.random.default_rng(3)
        big = rng.standard_normal((512, 512))
        small = W.series_1d(n=300, L=100, r=4)
        ref = None
        for _ in range(3):
            with pytest.raises(S.SsaError) as e:
                c.decompose(big, (64, 64), 30, precision="fp32")
            assert e.value.code == -4                    # SSA_ENOMEM
            d = c.decompose(small["x"], small["window"], 4)
            s = d.sigma.copy()
            d.free()
            if ref is None:
                ref = s
            assert np.array_equal(s, ref)
        res = c.decompose_batch([{"x": big, "window": (64, 64), "r": 30},
                                 {"x": small["x"], "window": small["window"], "r": 4}], precision="fp64")
        assert isinstance(res[0], S.SsaError) and res[0].code == -4
        assert isinstance(res[1], S.Decomposition)
        assert np.allclose(res[1].sigma, ref, rtol=1e-10, atol=0)
        res[1].free()
    finally:
        c.close()


_MIX_ORACLE = {}


def _mix_request(q):
    """A serving-mix request as a batch-call request: series as they are,
    MSSA series side by side in one array (NaN after each series' end) with
    an L x 1 window."""
    if q["kind"] == "mssa":
        nmax = max(len(x) for x in q["x"])
        arr = np.full((nmax, len(q["x"])), np.nan)
        for p, x in enumerate(q["x"]):
            arr[:len(x), p] = x
        return {"x": arr, "window": (q["window"], 1), "r": q["r"]}
    return {"x": q["x"], "window": q["window"], "r": q["r"]}


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_serving_mix_same_alone_and_in_the_mix(ctx, prec):
    """The serving workload's mix (1D series, MSSA systems, images; r from
    5 to 40) in one batch call with 4 slots per kernel class, so requests
    start as others finish: every result (sigma, both vector sets) is bit for
    bit the one the request gets alone, and the series' and images' sigma
    match the oracle."""
    import paper_1309_5050_amd as S
    mix = W.serving_mix(14, seed=7, max_1d=1500, max_side=128)
    data = [W.materialize(d) for d in mix]
    reqs = [_mix_request(q) for q in data]
    assert {q["kind"] for q in data} == {"1d", "mssa", "2d"}
    c = S.Context(0)
    try:
        c.set_slots(4)
        res = c.decompose_batch(reqs, precision=prec)
        for q, rq, d in zip(data, reqs, res):
            assert not isinstance(d, Exception), d
            assert d.status == 0 and d.stats["converged"] == 1
            alone = ctx.decompose(rq["x"], rq["window"], rq["r"], precision=prec)
            assert np.array_equal(d.sigma, alone.sigma)
            U, V = d.vectors_lex()
            Ua, Va = alone.vectors_lex()
            assert np.array_equal(U, Ua, equal_nan=True) and np.array_equal(V, Va, equal_nan=True)
            if q["kind"] != "mssa":
                key = (q["kind"], len(q["x"]), q["r"])
                if key not in _MIX_ORACLE:
                    _MIX_ORACLE[key] = oracle.decompose(rq["x"], None, None, rq["window"])[1]
                assert sigma_err(d.sigma, _MIX_ORACLE[key]) <= TOL[prec]
            alone.free()
            d.free()
    finally:
        c.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_orthogonality_is_measured_per_result(ctx, prec):
    """ssa_orthogonality: max |U^T U - I| and max |V^T V - I| of a result's
    singular vectors, formed on the device, equal the same quantities formed
    on the host from the returned vectors; the basis side stays orthonormal
    to FP64 rounding in both precisions, the other side to the operator
    precision."""
    cases = [W.series_1d(n=1000, L=500, r=10), W.image_2d(n=128, lw=16, r=12, seed=4), W.small_shaped(),
             W.series_1d(n=41000, L=300, r=6, seed=9)]            # the last in segments
    for w in cases:
        d = ctx.decompose(w["x"], w["window"], w["r"], mask=w["mask"], wmask=w["wmask"], precision=prec)
        ou, ov = d.orthogonality()
        U, V = d.vectors_lex()
        hu = np.max(np.abs(U.T @ U - np.eye(U.shape[1])))
        hv = np.max(np.abs(V.T @ V - np.eye(V.shape[1])))
        assert abs(ou - hu) <= 1e-11 and abs(ov - hv) <= 1e-11, (ou, hu, ov, hv)
        assert min(ou, ov) <= 1e-12
        assert max(ou, ov) <= (1e-9 if prec == "fp64" else 1e-4)
        d.free()
