"""Serving path (ssa_submit / ssa_poll / ssa_wait / ssa_take) on the GPU.

A request served asynchronously runs the same kernels as the synchronous
call, and results of a request do not depend on the batch it shares, so the
served singular values and reconstructions must equal the synchronous ones
bit for bit.  The synchronous results are themselves pinned to the oracle by
the parity tests.
"""
import numpy as np
import pytest

from paper_1309_5050_amd import workloads as W

pytestmark = [
    pytest.mark.gpu,
    pytest.mark.skip(reason="a full serving benchmark (300 mixed requests, FP32 and FP64 batches on the "
                            "library's worker threads) ended with a GPU memory fault on the build that adds the "
                            "FP32 basis copy; these tests passed in the same run, but the fault's cause is not "
                            "found, so the served path stays off the GPU until it is"),
]


@pytest.fixture(scope="module")
def ctx():
    import os

    import paper_1309_5050_amd as S
    os.environ["SHSSA_SERVE_ENGINE"] = "1"   # the library keeps its serving threads off otherwise
    c = S.Context(0)
    yield c
    c.close()


def _requests():
    reqs = []
    for i in range(3):   # three images of one geometry: one batch
        w = W.image_2d(n=96, lw=12, r=8, seed=300 + i)
        reqs.append(dict(kind="image", x=w["x"], window=w["window"], r=8, groups=[[0, 1], [2, 3]]))
    # images of other sizes and window shapes in the same kernel class: they
    # join the batch of the images above when they wait together
    big = W.image_2d(n=128, lw=12, r=8, seed=310)["x"]
    reqs.append(dict(kind="image", x=big[:100, :112], window=(12, 12), r=8, groups=[[0, 1], [2, 3]]))
    reqs.append(dict(kind="image", x=big[:120, :90], window=(10, 14), r=8, groups=[[0], [1, 2]]))
    for n in (700, 1234):
        w = W.series_1d(n=n, L=n // 2, r=6, seed=n)
        reqs.append(dict(kind="image", x=w["x"], window=w["window"], r=6, groups=[[0, 1]]))
    w = W.mssa_series(s=5, nmin=300, nmax=500, L=100, r=7, seed=11)
    reqs.append(dict(kind="mssa", series=w["x"], L=100, r=7, groups=[[0], [1, 2]]))
    w = W.small_shaped(seed=4)
    reqs.append(dict(kind="image", x=w["x"], window=w["window"], mask=w["mask"], wmask=w["wmask"], r=w["r"],
                     groups=[[0, 1]]))
    return reqs


def _sync(ctx, q, prec):
    if q["kind"] == "mssa":
        d = ctx.decompose_multi(q["series"], q["L"], q["r"], precision=prec)
    else:
        d = ctx.decompose(q["x"], q["window"], q["r"], mask=q.get("mask"), wmask=q.get("wmask"), precision=prec)
    return d, d.reconstruct(q["groups"])


def _submit(ctx, q, prec):
    if q["kind"] == "mssa":
        return ctx.submit_multi(q["series"], q["L"], q["r"], precision=prec, groups=q["groups"])
    return ctx.submit(q["x"], q["window"], q["r"], mask=q.get("mask"), wmask=q.get("wmask"), precision=prec,
                      groups=q["groups"])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_served_equals_synchronous(ctx, prec):
    """Each request decomposed alone (synchronous call) and served inside
    the mix of requests submitted together gives the same results."""
    reqs = _requests()
    ref = [_sync(ctx, q, prec) for q in reqs]
    tickets = [_submit(ctx, q, prec) for q in reqs]
    for q, t, (d0, rec0) in zip(reqs, tickets, ref):
        ctx.wait(t)
        assert ctx.poll(t)
        d, rec, times = ctx.take(t, shape=d0.shape, ngroups=len(q["groups"]))
        assert d.status == 0, d
        assert times["total_ms"] >= times["queue_ms"] >= 0.0
        assert np.array_equal(d.sigma, d0.sigma)
        assert np.array_equal(np.isnan(rec), np.isnan(rec0))
        assert np.array_equal(np.nan_to_num(rec), np.nan_to_num(rec0))


def test_submit_errors(ctx):
    from paper_1309_5050_amd import SsaError
    x = np.random.default_rng(0).standard_normal((20, 20))
    with pytest.raises(SsaError):
        ctx.submit(x, (30, 5), 3)                      # window beyond the array
    with pytest.raises(SsaError):
        ctx.submit(x, (5, 5), 3, groups=[[0, 7]])      # component beyond r
    with pytest.raises(SsaError):
        ctx.poll(123456789)                            # unknown ticket


def test_admission_refuses_oversized_request():
    import paper_1309_5050_amd as S
    c = S.Context(0, mem_budget=1 << 20)               # 1 MiB budget
    try:
        x = np.random.default_rng(1).standard_normal((256, 256))
        with pytest.raises(S.SsaError) as e:
            c.submit(x, (32, 32), 10)
        assert e.value.code == -4                       # SSA_ENOMEM
    finally:
        c.close()


def test_many_requests_and_untaken_cleanup():
    import paper_1309_5050_amd as S
    c = S.Context(0)
    try:
        rng = np.random.default_rng(2)
        tickets = []
        for i in range(12):
            n = int(rng.integers(300, 900))
            w = W.series_1d(n=n, L=n // 3, r=5, seed=i)
            tickets.append(c.submit(w["x"], w["window"], 5, precision="fp32", groups=[[0]]))
        for t in tickets[:8]:
            c.wait(t)
            d, rec, _ = c.take(t, shape=(0,), ngroups=0)
            assert d.status == 0 and np.all(np.diff(d.sigma) <= 0)
        # the remaining four are released by close()
    finally:
        c.close()
