"""GPU parity at the full workload sizes, against expected values written by
tests/golden/make_golden.py (oracle only: explicit S = X X^T and Jacobi).

Singular values are compared one by one; left subspaces of gap-stable groups
against the stored oracle vectors; reconstructions at sampled cells against
the oracle's explicit averaging evaluated cell by cell, with V_i = X^T U_i /
sigma_i from the oracle's explicit products.
"""
import os

import numpy as np
import pytest

import oracle
from paper_1309_5050_amd import workloads as W

from helpers import TOL, proj_dist, sigma_err, stable_groups

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
C_SUB = 20.0


@pytest.fixture(scope="module")
def ctx():
    import paper_1309_5050_amd as S
    c = S.Context(0)
    yield c
    c.close()


def golden(i):
    return np.load(os.path.join(HERE, "golden", f"config{i}_full.npz"))


def run(ctx, w, prec):
    if w["kind"] == "mssa":
        return ctx.decompose_multi(w["x"], w["window"], w["r"], precision=prec)
    return ctx.decompose(w["x"], w["window"], w["r"], mask=w["mask"], wmask=w["wmask"], precision=prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("cfg", [2, 3, 4])
def test_full_size_sigma_and_subspaces(ctx, cfg, prec):
    w = W.config(cfg)
    g = golden(cfg)
    so, Ug = g["sigma"], g["U"]
    d = run(ctx, w, prec)
    tol = TOL[prec]
    s = d.sigma
    err = sigma_err(s, so)
    print(f"config {cfg} {prec}: sigma err {err:.2e} stats {d.stats}")
    assert d.stats["converged"] == 1
    assert err <= tol
    U, _ = d.vectors_lex()
    nv = Ug.shape[1]
    for grp, gap in stable_groups(so, nv):
        dist = proj_dist(U[:, grp], Ug[:, grp])
        assert dist <= C_SUB * tol * so[0] / gap, (cfg, prec, grp, dist)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_full_size_image_reconstruction_sampled(ctx, prec):
    w = W.config(2)
    g = golden(2)
    so, Ug = g["sigma"], g["U"]
    sh = oracle.shapes(w["x"], window=w["window"])
    nv = Ug.shape[1]
    Vg = np.stack([oracle.rmatvec(w["x"], sh, Ug[:, k]) / so[k] for k in range(nv)], axis=1)
    groups = [[0, 1], [2, 3], [4, 5]]
    d = run(ctx, w, prec)
    rec = d.reconstruct(groups)
    rng = np.random.default_rng(7)
    cells = np.concatenate([rng.integers(0, 512, (1500, 2)),
                            np.array([[0, 0], [0, 511], [511, 0], [511, 511], [63, 63], [448, 448]])])
    gaps = {tuple(gr): gap for gr, gap in stable_groups(so, nv)}
    rms = np.sqrt(np.mean(w["x"] ** 2))
    wc = sh.W[cells[:, 0], cells[:, 1]]
    for k, grp in enumerate(groups):
        ref = oracle.reconstruct_at(sh, so, Ug, Vg, grp, cells)
        got = rec[k][cells[:, 0], cells[:, 1]]
        gap = min(gaps[(i,)] for i in grp)
        bound = C_SUB * TOL[prec] * so[0] / gap
        e = np.sqrt(np.mean((got - ref) ** 2)) / rms
        assert e <= bound, (grp, e)
        ok, worst, lim = elementwise_ok(got, ref, wc, rms, bound)
        assert ok, (prec, grp, worst, lim)


def group_gap(s, grp):
    """Distance of the group's singular values to the rest of the spectrum."""
    lo, hi = min(grp), max(grp)
    a = s[lo - 1] - s[lo] if lo > 0 else np.inf
    b = s[hi] - s[hi + 1] if hi + 1 < len(s) else np.inf
    return min(a, b)


def elementwise_ok(got, ref, w, scale, bound):
    """Per-cell check beside the norm check: a cell averaged over w entries
    of the trajectory matrix may err by bound * scale * sqrt(w_max / w)
    (errors of a mean of w entries shrink like 1/sqrt(w), so cells at hole
    and mask edges, averaged over few entries, get a larger allowance; an
    interior cell gets the allowance of the norm check's RMS)."""
    lim = bound * scale * np.sqrt(w.max() / w)
    err = np.abs(got - ref)
    k = int(np.argmax(err / lim))
    return bool(np.all(err <= lim)), float(err[k]), float(lim[k])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_full_size_mssa_reconstruction(ctx, prec):
    """MSSA workload (50 series of 1000..3000 points, L = 500, r = 20): every
    value of every series for the gap-stable groups {1,2}, {3,4} and
    {1..4}, against the oracle's averaging of sum sigma_i U_i V_i^T with the
    stored U and V_i = X^T U_i / sigma_i from the explicit stacked matrix."""
    w = W.config(3)
    g = golden(3)
    so, Ug = g["sigma"], g["U"]
    L = w["window"]
    X = oracle.trajectory_mssa(w["x"], L)
    nv = Ug.shape[1]
    Vg = (X.T @ Ug) / so[:nv]
    del X
    groups = [[0, 1], [2, 3], [0, 1, 2, 3]]
    d = run(ctx, w, prec)
    assert d.stats["converged"] == 1
    rec = d.reconstruct(groups)
    lens = [len(x) for x in w["x"]]
    xcat = np.concatenate(w["x"])
    rms = np.sqrt(np.mean(xcat ** 2))
    # weights of each series' values: min(t + 1, L, K_p, N_p - t)
    wts = np.concatenate([np.minimum.reduce([np.arange(1, n + 1), np.full(n, L), np.full(n, n - L + 1),
                                             np.arange(n, 0, -1)]) for n in lens]).astype(float)
    for k, grp in enumerate(groups):
        ref = np.concatenate(oracle.reconstruct_mssa(lens, L, so, Ug, Vg, grp))
        got = np.concatenate([rec[k][:n, p] for p, n in enumerate(lens)])
        assert all(np.all(np.isnan(rec[k][n:, p])) for p, n in enumerate(lens))
        bound = C_SUB * TOL[prec] * so[0] / group_gap(so, grp)
        e = np.linalg.norm(got - ref) / np.linalg.norm(xcat)
        assert e <= bound, (prec, grp, e, bound)
        ok, worst, lim = elementwise_ok(got, ref, wts, rms, bound)
        print(f"mssa {prec} {grp}: norm err {e:.2e} (bound {bound:.2e}), worst cell {worst:.2e} (allowed {lim:.2e})")
        assert ok, (prec, grp, worst, lim)


def _edge_cells(covered, nset, rng, n_each=600):
    """Covered cells with a neighbour outside N (hole and disc edges) and
    random covered cells."""
    pad = np.pad(nset, 1, constant_values=False)
    nb_out = ~(pad[:-2, 1:-1] & pad[2:, 1:-1] & pad[1:-1, :-2] & pad[1:-1, 2:])
    edge = np.argwhere(covered & nb_out)
    inner = np.argwhere(covered)
    pick = lambda a: a[rng.choice(len(a), size=min(n_each, len(a)), replace=False)]
    return np.concatenate([pick(edge), pick(inner)])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_full_size_shaped_reconstruction_sampled(ctx, prec):
    """Shaped workload (1024^2 disc with NaN holes, 32x32 window, r = 50):
    the rank-4 texture group {1..4} at covered cells next to the holes and the
    disc edge and at random covered cells, against the oracle's averaging
    evaluated cell by cell (stored U, V_i = X^T U_i / sigma_i by explicit
    sums)."""
    w = W.config(4)
    g = golden(4)
    so, Ug = g["sigma"], g["U"]
    sh = oracle.shapes(w["x"], w["mask"], w["wmask"], w["window"])
    nv = Ug.shape[1]
    Vg = np.stack([oracle.rmatvec(w["x"], sh, Ug[:, k]) / so[k] for k in range(nv)], axis=1)
    grp = [0, 1, 2, 3]
    d = run(ctx, w, prec)
    assert d.stats["converged"] == 1
    rec = d.reconstruct([grp])[0]
    rng = np.random.default_rng(17)
    cells = _edge_cells(sh.covered, sh.nset.astype(bool), rng)
    ref = oracle.reconstruct_at(sh, so, Ug, Vg, grp, cells)
    got = rec[cells[:, 0], cells[:, 1]]
    assert np.all(np.isfinite(got))
    xc = np.nan_to_num(w["x"])[sh.covered]
    rms = np.sqrt(np.mean(xc ** 2))
    bound = C_SUB * TOL[prec] * so[0] / group_gap(so, grp)
    e = np.sqrt(np.mean((got - ref) ** 2)) / rms
    assert e <= bound, (prec, e, bound)
    ok, worst, lim = elementwise_ok(got, ref, sh.W[cells[:, 0], cells[:, 1]], rms, bound)
    print(f"shaped {prec}: rms err {e:.2e} (bound {bound:.2e}), worst cell {worst:.2e} (allowed {lim:.2e})")
    assert ok, (prec, worst, lim)


def test_full_size_shaped_covered_set_and_weights(ctx):
    w = W.config(4)
    d = run(ctx, w, "fp32")
    sh = oracle.shapes(w["x"], w["mask"], w["wmask"], w["window"])
    assert (d.L, d.K) == (sh.L, sh.K)
    assert np.array_equal(d.weights, sh.W)
    rec = d.reconstruct([[0, 1, 2, 3]])
    assert np.array_equal(~np.isnan(rec[0]), sh.covered)


def test_full_size_batched_as_timed(ctx):
    """The timed configuration: a batch of device-resident 512 x 512 images
    (64 x 64 window, r = 30, FP32 products) through decompose_batch_dev and
    reconstruct_batch_dev into device outputs.  The batch's first image is
    the stored oracle case: sigma, stable subspaces and reconstructions at
    sampled cells against the oracle; the others against single-image
    decompositions of the same images (a result must not depend on the
    batch it runs in)."""
    import torch
    dev = torch.device("cuda:0")
    w = W.config(2)
    g = golden(2)
    so, Ug = g["sigma"], g["U"]
    tol = TOL["fp32"]
    imgs = [w["x"]] + [W.image_2d(seed=1000 + i)["x"] for i in range(7)]
    xs = [torch.tensor(x, device=dev) for x in imgs]
    groups = [[0, 1], [2, 3], [4, 5]]
    outs = [torch.empty((len(groups), 512, 512), dtype=torch.float64, device=dev) for _ in imgs]
    ds = ctx.decompose_batch_dev(xs, w["window"], w["r"], precision="fp32")
    assert not any(isinstance(d, Exception) for d in ds)
    type(ctx).reconstruct_batch_dev(ds, groups, outs)
    torch.cuda.synchronize()
    d0 = ds[0]
    assert d0.stats["converged"] == 1
    assert sigma_err(d0.sigma, so) <= tol
    U, _ = d0.vectors_lex()
    nv = Ug.shape[1]
    for grp, gap in stable_groups(so, nv):
        assert proj_dist(U[:, grp], Ug[:, grp]) <= C_SUB * tol * so[0] / gap, grp
    sh = oracle.shapes(w["x"], window=w["window"])
    Vg = np.stack([oracle.rmatvec(w["x"], sh, Ug[:, k]) / so[k] for k in range(nv)], axis=1)
    rng = np.random.default_rng(11)
    cells = rng.integers(0, 512, (800, 2))
    gaps = {tuple(gr): gap for gr, gap in stable_groups(so, nv)}
    rms = np.sqrt(np.mean(w["x"] ** 2))
    rec0 = outs[0].cpu().numpy()
    for k, grp in enumerate(groups):
        ref = oracle.reconstruct_at(sh, so, Ug, Vg, grp, cells)
        e = np.sqrt(np.mean((rec0[k][cells[:, 0], cells[:, 1]] - ref) ** 2)) / rms
        assert e <= C_SUB * tol * so[0] / min(gaps[(i,)] for i in grp), (grp, e)
    for i in range(1, len(imgs)):
        single = ctx.decompose(imgs[i], w["window"], w["r"], precision="fp32")
        s1 = single.sigma
        assert ds[i].stats["converged"] == 1
        assert np.max(np.abs(ds[i].sigma - s1)) <= 2 * tol * s1[0], i
        # its reconstructions in the batch's device outputs against the
        # single-image call's (both within the tolerance of the oracle's)
        r1 = single.reconstruct(groups)
        ri = outs[i].cpu().numpy()
        rmsi = np.sqrt(np.mean(imgs[i] ** 2))
        for k in range(len(groups)):
            e = np.sqrt(np.mean((ri[k] - r1[k]) ** 2)) / rmsi
            assert e <= 2 * C_SUB * tol, (i, k, e)
