"""Shaped 2D-SSA on MI355X: Python front end of the libshssa C ABI.

Thin marshalling over the C library (include/shssa.h): every step of the
decomposition and reconstruction runs in the library's HIP kernels.  PyTorch
is used only for device buffers and streams in the ``*_dev`` helpers.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _native
from ._native import SSA_FP32, SSA_FP32_BASIS32, SSA_FP64, SsaError, check, lib  # noqa: F401

__all__ = ["Context", "Decomposition", "SSA_FP32", "SSA_FP32_BASIS32", "SSA_FP64", "SsaError"]


def _prec(p) -> int:
    if p in (SSA_FP64, "fp64", "f64", "float64", np.float64):
        return SSA_FP64
    if p in (SSA_FP32, "fp32", "f32", "float32", np.float32):
        return SSA_FP32
    if p in (SSA_FP32_BASIS32, "fp32_basis32"):
        return SSA_FP32_BASIS32
    raise ValueError(f"unknown precision {p!r}")


def _ptr(a):
    return None if a is None else a.ctypes.data


class Decomposition:
    """Handle of one decomposition (sigma, U, V, weights held on the device)."""

    def __init__(self, ctx: "Context", handle: int):
        self.ctx = ctx
        self._h = C.c_void_p(handle)
        lx, ly, kx, ky, r, nx, ny = (C.c_int() for _ in range(7))
        L, K = C.c_long(), C.c_long()
        check(lib().ssa_get_dims(self._h, C.byref(lx), C.byref(ly), C.byref(kx), C.byref(ky), C.byref(L),
                                 C.byref(K), C.byref(r), C.byref(nx), C.byref(ny)), "ssa_get_dims")
        self.window_box = (lx.value, ly.value)
        self.origin_box = (kx.value, ky.value)
        self.L, self.K, self.r = L.value, K.value, r.value
        self.shape = (nx.value, ny.value)

    def __del__(self):
        try:
            self.free()
        except TypeError:   # interpreter shutdown: the module's globals are already gone
            pass

    def free(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ssa_free(self._h)
            self._h = C.c_void_p(0)

    @property
    def handle(self):
        return self._h

    @property
    def sigma(self) -> np.ndarray:
        s = np.zeros(self.r)
        check(lib().ssa_get_sigma(self._h, _ptr(s)), "ssa_get_sigma")
        return s

    def vectors(self):
        """(U, V): r eigenarrays on the window box and r factor arrays on the
        origin box, NaN outside the window shape / origin set."""
        U = np.zeros((self.r,) + self.window_box)
        V = np.zeros((self.r,) + self.origin_box)
        check(lib().ssa_get_vectors(self._h, _ptr(U), _ptr(V)), "ssa_get_vectors")
        return U, V

    def vectors_lex(self):
        """(U, V) as (L, r) and (K, r) columns in the paper's lexicographic order."""
        U = np.zeros(self.r * self.L)
        V = np.zeros(self.r * self.K)
        check(lib().ssa_get_vectors_lex(self._h, _ptr(U), _ptr(V)), "ssa_get_vectors_lex")
        return U.reshape(self.r, self.L).T.copy(), V.reshape(self.r, self.K).T.copy()

    @property
    def weights(self) -> np.ndarray:
        w = np.zeros(self.shape)
        check(lib().ssa_get_weights(self._h, _ptr(w)), "ssa_get_weights")
        return w

    @property
    def stats(self) -> dict:
        st = _native.Stats()
        check(lib().ssa_get_stats(self._h, C.byref(st)), "ssa_get_stats")
        return {k: getattr(st, k) for k, _ in st._fields_}

    def unpack(self, rec):
        """Cut arrays over a packed array (..., nx, ny) into its parts: for
        M-2D-SSA a list of (..., nx_p, ny_p) image views, for a mosaic
        Hankel decomposition the nested list (block rows, block columns) of
        (..., L_i + K_j - 1) series views."""
        if getattr(self, "mosaic_layout", None) is not None:
            return [[rec[..., i, c:c + n] for i, c, n in row] for row in self.mosaic_layout]
        return [rec[..., :a, c:c + b] for a, c, b in self.m2d_layout]

    def extend(self, r: int):
        """Continue the decomposition to r triplets (no-op if r <= self.r)."""
        check(lib().ssa_extend(self._h, int(r)), "ssa_extend")
        self.r = max(self.r, int(r))

    def reconstruct(self, groups) -> np.ndarray:
        """Reconstruct each group (list of 0-based component ids); returns
        (ngroups, nx, ny) with NaN outside the covered cells.  Components
        beyond r continue the decomposition first."""
        need = max((max(g) for g in groups if len(g)), default=-1) + 1
        if need > self.r:
            self.extend(need)
        gp = np.zeros(len(groups) + 1, np.int32)
        gp[1:] = np.cumsum([len(g) for g in groups])
        gi = np.ascontiguousarray(np.concatenate([np.asarray(g, np.int32) for g in groups]))
        out = np.zeros((len(groups),) + self.shape)
        check(lib().ssa_reconstruct(self._h, _ptr(gp), _ptr(gi), len(groups), _ptr(out)), "ssa_reconstruct")
        return out

    def _forecast(self, fn, group, h):
        g = np.ascontiguousarray(group, dtype=np.int32)
        ns = C.c_int()
        f = getattr(lib(), fn)
        check(f(self._h, _ptr(g), len(g), int(h), None, C.byref(ns)), fn)
        out = np.zeros((ns.value, int(h)))
        check(f(self._h, _ptr(g), len(g), int(h), _ptr(out), C.byref(ns)), fn)
        return out

    def rforecast(self, group, h: int, direction: str = "column") -> np.ndarray:
        """Recurrent forecast of h values after each series from the group:
        (series, h).  direction "column" (one LRR from the U_j) or "row"
        (from the V_j; each series' next value uses all series)."""
        fn = {"column": "ssa_rforecast", "row": "ssa_rforecast_row"}[direction]
        return self._forecast(fn, group, h)

    def vforecast(self, group, h: int, direction: str = "column") -> np.ndarray:
        """Vector forecast of h values after each series: (series, h);
        direction "column" (lagged vectors in the span of the U_j) or "row"
        (trajectory rows in the span of the V_j)."""
        fn = {"column": "ssa_vforecast", "row": "ssa_vforecast_row"}[direction]
        return self._forecast(fn, group, h)

    def esprit(self, group, method: str = "ls") -> np.ndarray:
        """ESPRIT roots of the group (complex, by decreasing modulus);
        method "ls" (least squares) or "tls" (total least squares)."""
        fn = {"ls": "ssa_esprit", "tls": "ssa_esprit_tls"}[method]
        g = np.ascontiguousarray(group, dtype=np.int32)
        re, im = np.zeros(len(g)), np.zeros(len(g))
        check(getattr(lib(), fn)(self._h, _ptr(g), len(g), _ptr(re), _ptr(im)), fn)
        return re + 1j * im

    def esprit_noalloc(self, group) -> np.ndarray:
        """LS-ESPRIT roots as ``esprit(group)``, through the call that uses the
        library's fixed device scratch instead of allocating (one call at a
        time per GPU)."""
        g = np.ascontiguousarray(group, dtype=np.int32)
        re, im = np.zeros(len(g)), np.zeros(len(g))
        check(lib().ssa_esprit_noalloc(self._h, _ptr(g), len(g), _ptr(re), _ptr(im)), "ssa_esprit_noalloc")
        return re + 1j * im

    def esprit2d(self, group):
        """2D-ESPRIT pairs of the group: (lambda, mu) complex arrays (x and y roots)."""
        g = np.ascontiguousarray(group, dtype=np.int32)
        a, b, c, e = (np.zeros(len(g)) for _ in range(4))
        check(lib().ssa_esprit2d(self._h, _ptr(g), len(g), _ptr(a), _ptr(b), _ptr(c), _ptr(e)), "ssa_esprit2d")
        return a + 1j * b, c + 1j * e

    def wcor(self, groups):
        """w-correlation matrix (ngroups, ngroups) and contributions
        (ngroups,) of the reconstructed groups."""
        gp = np.zeros(len(groups) + 1, np.int32)
        gp[1:] = np.cumsum([len(g) for g in groups])
        gi = np.ascontiguousarray(np.concatenate([np.asarray(g, np.int32) for g in groups]))
        rho = np.zeros((len(groups), len(groups)))
        contrib = np.zeros(len(groups))
        check(lib().ssa_wcor(self._h, _ptr(gp), _ptr(gi), len(groups), _ptr(rho), _ptr(contrib)), "ssa_wcor")
        return rho, contrib

    def orthogonality(self):
        """(max |U^T U - I|, max |V^T V - I|) of the r singular vectors,
        measured on the device."""
        ou, ov = C.c_double(), C.c_double()
        check(lib().ssa_orthogonality(self._h, C.byref(ou), C.byref(ov)), "ssa_orthogonality")
        return ou.value, ov.value


class Context:
    """A device, a stream and a memory budget for decompositions."""

    def __init__(self, device: int = 0, mem_budget: int = 0, stream=None, tune_cache=None):
        h = C.c_void_p()
        tc = None if tune_cache is None else str(tune_cache).encode()
        check(lib().ssa_ctx_create(device, mem_budget, tc, C.byref(h)), "ssa_ctx_create")
        self._h = h
        if stream is not None:
            self.set_stream(stream)

    def __del__(self):
        try:
            self.close()
        except TypeError:   # interpreter shutdown: the module's globals are already gone
            pass

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ssa_ctx_destroy(self._h)
            self._h = C.c_void_p(0)

    @property
    def handle(self):
        return self._h

    def sync(self):
        check(lib().ssa_ctx_sync(self._h), "ssa_ctx_sync")

    def set_slots(self, slots: int):
        """Continuous batching: at most `slots` decompositions of a batch call
        advance together, the others join as slots free up (0: all at once)."""
        check(lib().ssa_ctx_set_slots(self._h, int(slots)), "ssa_ctx_set_slots")

    def set_stream(self, stream):
        check(lib().ssa_ctx_set_stream(self._h, stream), "ssa_ctx_set_stream")

    def profile(self, kind, every: int = 1):
        """Start (kind = comma-separated kernel classes) or stop (None) event
        timing; with every > 1 only one launch in `every` of each class is
        timed."""
        check(lib().ssa_ctx_profile_every(self._h, int(every)), "ssa_ctx_profile_every")
        check(lib().ssa_ctx_profile(self._h, None if kind is None else kind.encode()), "ssa_ctx_profile")

    def profile_read(self, kinds=None) -> dict:
        """Totals of the recorded launches; with ``kinds`` (a list of kernel
        classes) a dict of per-class totals.  Clears the record."""
        per = None
        if kinds:
            per = {}
            for k in kinds:
                ms, n, b = C.c_double(), C.c_long(), C.c_double()
                check(lib().ssa_ctx_profile_read_kind(self._h, k.encode(), C.byref(ms), C.byref(n), C.byref(b)),
                      "ssa_ctx_profile_read_kind")
                tot = C.c_long()
                check(lib().ssa_ctx_profile_launches(self._h, k.encode(), C.byref(tot)), "ssa_ctx_profile_launches")
                per[k] = {"ms": ms.value, "launches": n.value, "bytes": b.value, "all_launches": tot.value}
        ms, n, b = C.c_double(), C.c_long(), C.c_double()
        check(lib().ssa_ctx_profile_read(self._h, C.byref(ms), C.byref(n), C.byref(b)), "ssa_ctx_profile_read")
        return per if per is not None else {"ms": ms.value, "launches": n.value, "bytes": b.value}

    # ---- decomposition -------------------------------------------------

    @staticmethod
    def _image_args(x, window, mask, wmask):
        x = np.ascontiguousarray(x, dtype=np.float64)
        if x.ndim == 1:
            x = x[:, None]
        if wmask is not None:
            wmask = np.ascontiguousarray(wmask, dtype=np.uint8)
            if wmask.ndim == 1:
                wmask = wmask[:, None]
            lx, ly = wmask.shape
        elif np.isscalar(window):
            lx, ly = int(window), 1
        else:
            lx, ly = int(window[0]), int(window[1])
        if mask is not None:
            mask = np.ascontiguousarray(mask, dtype=np.uint8).reshape(x.shape)
        return x, lx, ly, mask, wmask

    def decompose(self, x, window=None, r: int = 10, mask=None, wmask=None, precision="fp64",
                  method: str = "lanczos") -> Decomposition:
        """Shaped decomposition of an image (or a series given as 1-D).
        method "eigen": S = X X^T and its eigenpairs (windows of at most 4096
        cells, FP64 whatever the precision)."""
        x, lx, ly, mask, wmask = self._image_args(x, window, mask, wmask)
        h = C.c_void_p()
        if method == "eigen":
            check(lib().ssa_decompose_eigen(self._h, _ptr(x), x.shape[0], x.shape[1], _ptr(mask), _ptr(wmask), lx,
                                            ly, r, C.byref(h)), "ssa_decompose_eigen")
            return Decomposition(self, h.value)
        if method != "lanczos":
            raise ValueError("method must be 'lanczos' or 'eigen'")
        check(lib().ssa_decompose(self._h, _ptr(x), x.shape[0], x.shape[1], _ptr(mask), _ptr(wmask), lx, ly, r,
                                  _prec(precision), C.byref(h)), "ssa_decompose")
        return Decomposition(self, h.value)

    def decompose_m2d(self, images, window, r: int, wmask=None, precision="fp64") -> Decomposition:
        """M-2D-SSA of several images with one window (common basis).  The
        handle refers to the packed array; ``unpack(rec)`` of the returned
        handle cuts a reconstruction back into the images."""
        arrs = [np.ascontiguousarray(x, dtype=np.float64) for x in images]
        ptrs = (C.c_void_p * len(arrs))(*[a.ctypes.data for a in arrs])
        nx = np.array([a.shape[0] for a in arrs], np.int32)
        ny = np.array([a.shape[1] for a in arrs], np.int32)
        lx, ly = window
        wm = None if wmask is None else np.ascontiguousarray(wmask, dtype=np.uint8)
        off = np.zeros(len(arrs), np.int32)
        h = C.c_void_p()
        check(lib().ssa_decompose_m2d(self._h, ptrs, _ptr(nx), _ptr(ny), len(arrs), _ptr(wm), lx, ly, r,
                                      _prec(precision), _ptr(off), C.byref(h)), "ssa_decompose_m2d")
        d = Decomposition(self, h.value)
        d.m2d_layout = [(int(a), int(c), int(b)) for a, b, c in zip(nx, ny, off)]   # (rows, col offset, cols)
        return d

    def decompose_mosaic(self, series, Ls, Ks, r: int, precision="fp64") -> Decomposition:
        """Mosaic Hankel SSA: series[i][j] (length Ls[i] + Ks[j] - 1) gives
        block (i, j), the Ls[i] x Ks[j] Hankel matrix.  The handle refers to
        the packed array; ``unpack(rec)`` of the returned handle cuts a
        reconstruction back into the nested list of series."""
        Ls = [int(v) for v in Ls]
        Ks = [int(v) for v in Ks]
        if len(series) != len(Ls) or any(len(row) != len(Ks) for row in series):
            raise ValueError("series must be a len(Ls) x len(Ks) nested list")
        arrs = []
        for i, L in enumerate(Ls):
            for j, K in enumerate(Ks):
                a = np.ascontiguousarray(series[i][j], dtype=np.float64)
                if a.ndim != 1 or len(a) != L + K - 1:
                    raise ValueError("series (%d, %d) needs Ls[i] + Ks[j] - 1 = %d values" % (i, j, L + K - 1))
                arrs.append(a)
        ptrs = (C.c_void_p * len(arrs))(*[a.ctypes.data for a in arrs])
        ls = np.array(Ls, np.int32)
        ks = np.array(Ks, np.int32)
        off = np.zeros(len(Ks), np.int32)
        h = C.c_void_p()
        check(lib().ssa_decompose_mosaic(self._h, ptrs, len(Ls), len(Ks), _ptr(ls), _ptr(ks), r, _prec(precision),
                                         _ptr(off), C.byref(h)), "ssa_decompose_mosaic")
        d = Decomposition(self, h.value)
        d.mosaic_layout = [[(i, int(off[j]), L + K - 1) for j, K in enumerate(Ks)] for i, L in enumerate(Ls)]
        return d

    def decompose_multi(self, series, L: int, r: int, precision="fp64") -> Decomposition:
        """MSSA of uneven series (2D packing: outputs are max N_p x s arrays)."""
        arrs = [np.ascontiguousarray(s, dtype=np.float64) for s in series]
        ptrs = (C.c_void_p * len(arrs))(*[a.ctypes.data for a in arrs])
        lens = np.array([len(a) for a in arrs], np.int32)
        h = C.c_void_p()
        check(lib().ssa_decompose_multi(self._h, ptrs, _ptr(lens), len(arrs), L, r, _prec(precision),
                                        C.byref(h)), "ssa_decompose_multi")
        return Decomposition(self, h.value)

    def decompose_batch(self, requests, precision="fp64", seed: int = 0x5EED):
        """Decompose a list of dicts {x, window, r, mask?, wmask?} in batches
        of equal geometry.  Returns a list of Decomposition (or SsaError)."""
        keep = []
        reqs = (_native.Request * len(requests))()
        for i, rq in enumerate(requests):
            x, lx, ly, mask, wmask = self._image_args(rq["x"], rq.get("window"), rq.get("mask"), rq.get("wmask"))
            keep.append((x, mask, wmask))
            reqs[i] = _native.Request(x.ctypes.data, x.shape[0], x.shape[1], _ptr(mask), _ptr(wmask), lx, ly,
                                      int(rq["r"]), _prec(rq.get("precision", precision)), seed)
        return self._run_batch(reqs, len(requests), dev=False)

    def _run_batch(self, reqs, n, dev):
        out = (C.c_void_p * n)()
        st = (C.c_int * n)()
        fn = lib().ssa_decompose_batch_dev if dev else lib().ssa_decompose_batch
        check(fn(self._h, n, reqs, out, st), "ssa_decompose_batch")
        res = []
        for i in range(n):
            if out[i]:
                d = Decomposition(self, out[i])
                d.status = st[i]
                res.append(d)
            else:
                res.append(SsaError(st[i], f"request {i}"))
        return res

    def decompose_batch_dev(self, xs, window, r: int, precision="fp64", seed: int = 0x5EED, masks=None):
        """Batch of device-resident images: ``xs`` are CUDA float64 tensors
        (nx, ny) on this context's device."""
        n = len(xs)
        reqs = (_native.Request * n)()
        lx, ly = (int(window), 1) if np.isscalar(window) else (int(window[0]), int(window[1]))
        for i, x in enumerate(xs):
            nx, ny = (x.shape[0], 1) if x.dim() == 1 else (x.shape[0], x.shape[1])
            m = None if masks is None else masks[i].data_ptr()
            reqs[i] = _native.Request(x.data_ptr(), nx, ny, m, None, lx, ly, r, _prec(precision), seed)
        return self._run_batch(reqs, n, dev=True)

    @staticmethod
    def reconstruct_batch_dev(decomps, groups, outs):
        """Reconstruct the same groups of several decompositions into CUDA
        float64 tensors outs[i] of shape (ngroups, nx, ny); asynchronous."""
        n = len(decomps)
        gp = np.zeros(len(groups) + 1, np.int32)
        gp[1:] = np.cumsum([len(g) for g in groups])
        gi = np.ascontiguousarray(np.concatenate([np.asarray(g, np.int32) for g in groups]))
        hs = (C.c_void_p * n)(*[d.handle.value for d in decomps])
        ptrs = (C.c_void_p * n)(*[o.data_ptr() for o in outs])
        check(lib().ssa_reconstruct_batch_dev(n, hs, _ptr(gp), _ptr(gi), len(groups), ptrs),
              "ssa_reconstruct_batch_dev")

    # ---- serving -------------------------------------------------------

    @staticmethod
    def _groups(groups):
        if not groups:
            return None, None, 0
        gp = np.zeros(len(groups) + 1, np.int32)
        gp[1:] = np.cumsum([len(g) for g in groups])
        gi = np.ascontiguousarray(np.concatenate([np.asarray(g, np.int32) for g in groups]))
        return gp, gi, len(groups)

    def submit(self, x, window=None, r: int = 10, mask=None, wmask=None, precision="fp64", groups=None) -> int:
        """Queue a decomposition (+ reconstruction of ``groups``); returns a ticket."""
        x, lx, ly, mask, wmask = self._image_args(x, window, mask, wmask)
        gp, gi, ng = self._groups(groups)
        req = _native.Request(x.ctypes.data, x.shape[0], x.shape[1], _ptr(mask), _ptr(wmask), lx, ly, int(r),
                              _prec(precision), 0x5EED)
        t = C.c_uint64()
        check(lib().ssa_submit(self._h, C.byref(req), _ptr(gp), _ptr(gi), ng, C.byref(t)), "ssa_submit")
        return t.value

    def submit_multi(self, series, L: int, r: int, precision="fp64", groups=None) -> int:
        """Queue an MSSA request; returns a ticket."""
        arrs = [np.ascontiguousarray(s, dtype=np.float64) for s in series]
        ptrs = (C.c_void_p * len(arrs))(*[a.ctypes.data for a in arrs])
        lens = np.array([len(a) for a in arrs], np.int32)
        gp, gi, ng = self._groups(groups)
        t = C.c_uint64()
        check(lib().ssa_submit_multi(self._h, ptrs, _ptr(lens), len(arrs), int(L), int(r), _prec(precision),
                                     _ptr(gp), _ptr(gi), ng, C.byref(t)), "ssa_submit_multi")
        return t.value

    def poll(self, ticket: int) -> bool:
        done = C.c_int()
        check(lib().ssa_poll(self._h, ticket, C.byref(done)), "ssa_poll")
        return bool(done.value)

    def wait(self, ticket: int):
        check(lib().ssa_wait(self._h, ticket), "ssa_wait")

    def take(self, ticket: int, shape=None, ngroups: int = 0):
        """Finish a request: (Decomposition or SsaError, reconstruction or
        None, {queue_ms, total_ms}).  ``shape`` (nx, ny) and ``ngroups`` size
        the reconstruction buffer."""
        h = C.c_void_p()
        tm = _native.Times()
        rec = np.zeros((ngroups,) + tuple(shape)) if (ngroups and shape is not None) else None
        rc = lib().ssa_take(self._h, ticket, C.byref(h), _ptr(rec), C.byref(tm))
        times = {"queue_ms": tm.queue_ms, "total_ms": tm.total_ms}
        if rc == _native.SSA_EBUSY:
            raise SsaError(rc, "request not finished")
        if h.value:
            d = Decomposition(self, h.value)
            d.status = rc
            return d, rec, times
        return SsaError(rc, lib().ssa_last_error().decode()), None, times
