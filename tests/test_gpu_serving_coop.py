"""Cooperative serving (ssa_submit / ssa_poll / ssa_wait / ssa_take without
the worker threads) on the GPU.

Requests queue on submission; each ssa_poll or ssa_wait runs one round on
the context's stream: admissions (set-up and spectrum of the waiting
requests that fit the memory budget), then one restart cycle of every
running kernel class, in which waiting requests take the slots of finished
ones and finished ones leave with their results.  The instances run the
kernels of the continuous batch calls with their own step counters, so a
served request's singular values and reconstructions equal the synchronous
call's bit for bit, whenever it joined; the synchronous results are pinned
to the oracle by the parity tests.
"""
import os

import numpy as np
import pytest

from paper_1309_5050_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1309_5050_amd as S
    assert "SHSSA_SERVE_ENGINE" not in os.environ    # the cooperative server is the default
    c = S.Context(0)
    yield c
    c.close()


def _requests():
    reqs = []
    for i in range(3):   # three images of one geometry: one batch
        w = W.image_2d(n=96, lw=12, r=8, seed=300 + i)
        reqs.append(dict(kind="image", x=w["x"], window=w["window"], r=8, groups=[[0, 1], [2, 3]]))
    # images of other sizes and window shapes in the same kernel class
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


def _check(ctx, q, t, d0, rec0):
    ctx.wait(t)
    assert ctx.poll(t)
    d, rec, times = ctx.take(t, shape=d0.shape, ngroups=len(q["groups"]))
    assert d.status == 0, d
    assert times["total_ms"] >= times["queue_ms"] >= 0.0
    assert np.array_equal(d.sigma, d0.sigma)
    assert np.array_equal(np.isnan(rec), np.isnan(rec0))
    assert np.array_equal(np.nan_to_num(rec), np.nan_to_num(rec0))
    d.free()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_coop_served_equals_synchronous(ctx, prec):
    """Each request of a mix submitted together gives the synchronous
    call's results bit for bit."""
    reqs = _requests()
    ref = [_sync(ctx, q, prec) for q in reqs]
    tickets = [_submit(ctx, q, prec) for q in reqs]
    for q, t, (d0, rec0) in zip(reqs, tickets, ref):
        _check(ctx, q, t, d0, rec0)


def test_coop_requests_join_running_batches():
    """With 2 slots, requests submitted while others run (after some rounds
    of the server) join the running batches as slots free up; every result
    equals the synchronous one."""
    import paper_1309_5050_amd as S
    c = S.Context(0)
    try:
        c.set_slots(2)
        reqs = []
        for i, n in enumerate((1500, 1400, 600, 700, 650, 1300)):
            w = W.series_1d(n=n, L=n // 3, r=6, seed=40 + i)
            reqs.append(dict(kind="image", x=w["x"], window=w["window"], r=6, groups=[[0, 1]]))
        ref = [_sync(c, q, "fp32") for q in reqs]
        first = [_submit(c, q, "fp32") for q in reqs[:2]]
        for _ in range(2):
            c.poll(first[0])                         # rounds of the server
        later = [_submit(c, q, "fp32") for q in reqs[2:]]
        for q, t, (d0, rec0) in zip(reqs, first + later, ref):
            _check(c, q, t, d0, rec0)
    finally:
        c.close()


def test_coop_admission_refuses_oversized_request():
    import paper_1309_5050_amd as S
    c = S.Context(0, mem_budget=1 << 20)               # 1 MiB budget
    try:
        x = np.random.default_rng(1).standard_normal((256, 256))
        with pytest.raises(S.SsaError) as e:
            c.submit(x, (32, 32), 10)
        assert e.value.code == -4                       # SSA_ENOMEM
    finally:
        c.close()


def test_coop_budget_admits_in_turn():
    """A budget that holds one request at a time: the requests are admitted
    one after another as earlier ones finish, and all complete."""
    import paper_1309_5050_amd as S
    w = W.series_1d(n=800, L=300, r=5, seed=3)
    probe = S.Context(0)
    d = probe.decompose(w["x"], w["window"], 5, precision="fp32")
    need = d.stats["device_bytes"]
    d.free()
    probe.close()
    # the smallest budget (in steps of at most 4/3) that admits the request:
    # below twice its estimate, so requests run one after another
    c = None
    for k in (1.0, 1.5, 2, 2.5, 3, 4, 5, 6, 8, 10, 12, 16):
        c = S.Context(0, mem_budget=int(need * k))
        try:
            t0 = c.submit(w["x"], w["window"], 5, precision="fp32", groups=[[0]])
            break
        except S.SsaError as e:
            assert e.code == -4
            c.close()
            c = None
    assert c is not None
    try:
        tickets = [t0] + [c.submit(w["x"], w["window"], 5, precision="fp32", groups=[[0]]) for _ in range(3)]
        sig = []
        for t in tickets:
            c.wait(t)
            d, _, _ = c.take(t, shape=(0,), ngroups=0)
            assert d.status == 0
            sig.append(d.sigma.copy())
            d.free()
        assert all(np.array_equal(s, sig[0]) for s in sig)
    finally:
        c.close()


def test_coop_many_requests_and_untaken_cleanup():
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
            d.free()
        # the remaining four (queued or in a batch) are released by close()
    finally:
        c.close()
