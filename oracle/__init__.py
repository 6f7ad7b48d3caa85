"""Reference oracle for Shaped 2D-SSA -- test infrastructure, not product code.

Only the test-suite, the smoke check and the CPU-baseline timing may import
this package.  It computes everything in double precision from the plain
definitions (explicit trajectory matrix, Jacobi SVD, explicit averaging),
in C (``ssa_oracle.c``) driven from here through ctypes.  It shares no code
with the GPU path.

Conventions (0-based): images are (nx, ny) row-major arrays, x = row axis.
Index sets are returned as (row, col) int arrays in column-major
("lexicographic", row index fastest) order.  U is (L, d) and V is (K, d)
with columns = singular vectors, sigma descending, and the sign of each
triplet fixed so that the largest-magnitude entry of U_k is positive.

Parity unpinned: none (each function is pinned in the oracle tests).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ssa_oracle.c")
_LIB = os.path.join(_HERE, "libssa_oracle.so")
_lib = None

_d = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_u8 = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")


def build(force: bool = False) -> str:
    """Compile the oracle library with gcc (OpenMP); returns its path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        L.orc_nset.argtypes = [C.c_int, C.c_int, _d, C.c_void_p, _u8]
        L.orc_window.argtypes = [C.c_int, C.c_int, C.c_void_p, _i, _i, C.POINTER(C.c_int),
                                 C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.orc_window.restype = C.c_int
        L.orc_kset.argtypes = [C.c_int, C.c_int, _u8, C.c_int, _i, _i, C.c_int, C.c_int,
                               _i, _i, C.POINTER(C.c_long)]
        L.orc_weights.argtypes = [C.c_int, C.c_int, C.c_int, _i, _i, C.c_long, _i, _i, _d]
        L.orc_trajectory.argtypes = [C.c_int, C.c_int, _d, C.c_int, _i, _i, C.c_long, _i, _i, _d]
        L.orc_trajectory_mssa.argtypes = [C.c_int, _i, _d, C.c_int, _d]
        L.orc_matvec.argtypes = [C.c_int, C.c_int, _d, C.c_int, _i, _i, C.c_long, _i, _i, _d, _d]
        L.orc_rmatvec.argtypes = L.orc_matvec.argtypes
        L.orc_svd_jacobi.argtypes = [C.c_long, C.c_long, _d, C.c_double, C.c_int, _d, _d, _d]
        L.orc_svd_jacobi.restype = C.c_int
        L.orc_eig_gram.argtypes = [C.c_long, _d, C.c_double, C.c_int, _d, _d]
        L.orc_eig_gram.restype = C.c_int
        L.orc_reconstruct.argtypes = [C.c_int, C.c_int, C.c_int, _i, _i, C.c_long, _i, _i, C.c_int,
                                      _d, _d, _d, C.c_int, _i, _d]
        L.orc_reconstruct_mssa.argtypes = [C.c_int, _i, C.c_int, C.c_int, _d, _d, _d, C.c_int, _i, _d]
        L.orc_reconstruct_at.argtypes = [C.c_int, _i, _i, C.c_int, C.c_int,
                                         np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS"),
                                         C.c_long, C.c_int, _d, _d, _d, C.c_int, _i, C.c_long, _i, _i, _d]
        L.orc_gram_rows.argtypes = [C.c_long, C.c_long, _d, C.c_long, C.c_long, _d]
        L.orc_num_threads.restype = C.c_int
        L.orc_set_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def num_threads() -> int:
    return lib().orc_num_threads()


def set_threads(n: int) -> None:
    """Threads of the oracle's parallel loops (for timing it)."""
    lib().orc_set_threads(int(n))


# --------------------------------------------------------------------------
# shapes
# --------------------------------------------------------------------------

class Shapes:
    """N, L, K, W of one shaped decomposition (all 0-based)."""

    def __init__(self, nx, ny, nset, li, lj, lxt, lyt, ki, kj, W):
        self.nx, self.ny = nx, ny
        self.nset = nset            # (nx, ny) uint8
        self.li, self.lj = li, lj   # window cells, column-major order
        self.lxt, self.lyt = lxt, lyt
        self.ki, self.kj = ki, kj   # origins, column-major order
        self.W = W                  # (nx, ny) float64 weights (counts)

    @property
    def L(self) -> int:
        return len(self.li)

    @property
    def K(self) -> int:
        return len(self.ki)

    @property
    def covered(self) -> np.ndarray:
        return self.W > 0


def shapes(x, mask=None, wmask=None, window=None) -> Shapes:
    """N = mask & ~isnan(x); L = wmask trimmed; K by brute force; W by counting."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    if x.ndim == 1:
        x = x[:, None]
    nx, ny = x.shape
    lib_ = lib()
    nset = np.zeros((nx, ny), np.uint8)
    m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    lib_.orc_nset(nx, ny, x, None if m is None else m.ctypes.data, nset)
    if wmask is not None:
        wm = np.ascontiguousarray(wmask, dtype=np.uint8)
        if wm.ndim == 1:
            wm = wm[:, None]
        lx, ly = wm.shape
        wptr = wm.ctypes.data
    else:
        if np.isscalar(window):
            lx, ly = int(window), 1
        else:
            lx, ly = int(window[0]), int(window[1])
        wm, wptr = None, None
    li = np.zeros(lx * ly, np.int32)
    lj = np.zeros(lx * ly, np.int32)
    nl, lxt, lyt = C.c_int(), C.c_int(), C.c_int()
    if lib_.orc_window(lx, ly, wptr, li, lj, C.byref(nl), C.byref(lxt), C.byref(lyt)) != 0:
        raise ValueError("empty window")
    li, lj = li[:nl.value].copy(), lj[:nl.value].copy()
    kx, ky = nx - lxt.value + 1, ny - lyt.value + 1
    if kx <= 0 or ky <= 0:
        raise ValueError("window larger than the array")
    ki = np.zeros(kx * ky, np.int32)
    kj = np.zeros(kx * ky, np.int32)
    nk = C.c_long()
    lib_.orc_kset(nx, ny, nset, nl.value, li, lj, lxt.value, lyt.value, ki, kj, C.byref(nk))
    ki, kj = ki[:nk.value].copy(), kj[:nk.value].copy()
    W = np.zeros((nx, ny))
    lib_.orc_weights(nx, ny, len(li), li, lj, len(ki), ki, kj, W)
    return Shapes(nx, ny, nset, li, lj, lxt.value, lyt.value, ki, kj, W)


def clean(x, sh: Shapes) -> np.ndarray:
    """x with the cells outside N set to 0 (they never enter X)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    if x.ndim == 1:
        x = x[:, None]
    return np.where(sh.nset.astype(bool), x, 0.0)


def trajectory(x, sh: Shapes) -> np.ndarray:
    """Explicit quasi-Hankel trajectory matrix, (L, K)."""
    xc = clean(x, sh)
    X = np.zeros((sh.L, sh.K))
    lib().orc_trajectory(sh.nx, sh.ny, xc, sh.L, sh.li, sh.lj, sh.K, sh.ki, sh.kj, X)
    return X


def trajectory_mssa(series, L: int) -> np.ndarray:
    """Explicit stacked Hankel matrix [T(x1):...:T(xs)], (L, sum K_p)."""
    lens = np.array([len(s) for s in series], np.int32)
    cat = np.ascontiguousarray(np.concatenate(series), dtype=np.float64)
    K = int(np.sum(lens - L + 1))
    X = np.zeros((L, K))
    lib().orc_trajectory_mssa(len(series), lens, cat, L, X)
    return X


def matvec(x, sh: Shapes, v) -> np.ndarray:
    """u = X v by explicit sums over the trajectory entries."""
    xc = clean(x, sh)
    u = np.zeros(sh.L)
    lib().orc_matvec(sh.nx, sh.ny, xc, sh.L, sh.li, sh.lj, sh.K, sh.ki, sh.kj,
                     np.ascontiguousarray(v, dtype=np.float64), u)
    return u


def rmatvec(x, sh: Shapes, u) -> np.ndarray:
    """v = X^T u by explicit sums over the trajectory entries."""
    xc = clean(x, sh)
    v = np.zeros(sh.K)
    lib().orc_rmatvec(sh.nx, sh.ny, xc, sh.L, sh.li, sh.lj, sh.K, sh.ki, sh.kj,
                      np.ascontiguousarray(u, dtype=np.float64), v)
    return v


# --------------------------------------------------------------------------
# SVD
# --------------------------------------------------------------------------

def svd(X, method: str = "jacobi", tol: float = 1e-14, max_sweeps: int = 100, nvec: int = -1):
    """All min(L, K) triplets of the explicit matrix X (L x K).

    method "jacobi": one-sided Jacobi on the shorter dimension.
    method "gram":   eigenpairs of S = X X^T, V_j = X^T U_j / sigma_j
                     (the paper's statement of the SVD step); with nvec >= 0
                     only the first nvec columns of V are formed (rest zero).
    Returns sigma (d,), U (L, d), V (K, d).
    """
    X = np.ascontiguousarray(X, dtype=np.float64)
    m, n = X.shape
    d = min(m, n)
    if method == "gram":
        if m > n:
            # S = X X^T is the larger Gram; decompose X^T and swap roles
            s, V, U = svd(X.T, "gram", tol, max_sweeps)
            return s, U, _sign_rule(U, V)
        # S = X X^T by a library matrix product, its eigenpairs by cyclic
        # Jacobi, V_j = X^T U_j / sigma_j by a library matrix product
        S = np.ascontiguousarray(X @ X.T)
        S = 0.5 * (S + S.T)
        lam = np.zeros(m)
        Ucm = np.zeros(m * m)
        sweeps = lib().orc_eig_gram(m, S, tol, max_sweeps, lam, Ucm)
        if sweeps < 0:
            raise RuntimeError("Jacobi iteration did not converge")
        U = Ucm.reshape(m, m).T[:, :d].copy()
        sig = np.sqrt(np.maximum(lam[:d], 0.0))
        nv = d if nvec < 0 or nvec > d else nvec
        V = np.zeros((n, d))
        pos = sig[:nv] > 0
        if nv:
            V[:, :nv] = X.T @ U[:, :nv]
            V[:, :nv][:, pos] /= sig[:nv][pos]
            V[:, :nv][:, ~pos] = 0.0
        return sig, U, _sign_rule(U, V)
    sig = np.zeros(d)
    Ucm = np.zeros(m * d)
    Vcm = np.zeros(n * d)
    sweeps = lib().orc_svd_jacobi(m, n, X, tol, max_sweeps, sig, Ucm, Vcm)
    if sweeps < 0:
        raise RuntimeError("Jacobi iteration did not converge")
    U = Ucm.reshape(d, m).T.copy()
    V = Vcm.reshape(d, n).T.copy()
    return sig, U, V


def _sign_rule(U, V):
    """Flips (U_k, V_k) in place so that the entry of largest magnitude of
    U_k is positive (lowest index on ties); returns V."""
    for k in range(U.shape[1]):
        a = int(np.argmax(np.abs(U[:, k])))
        if U[a, k] < 0:
            U[:, k] *= -1
            V[:, k] *= -1
    return V


def gram_rows(X, r0: int, r1: int) -> np.ndarray:
    """Rows r0..r1-1 of S = X X^T by explicit sums (used for timing)."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    m, n = X.shape
    out = np.zeros((r1 - r0, m))
    lib().orc_gram_rows(m, n, X, r0, r1, out)
    return out


def reconstruct(sh: Shapes, sigma, U, V, group) -> np.ndarray:
    """Diagonal averaging of sum_{k in group} sigma_k U_k V_k^T; NaN off N'."""
    out = np.zeros((sh.nx, sh.ny))
    Ucm = np.ascontiguousarray(np.asarray(U, dtype=np.float64).T)
    Vcm = np.ascontiguousarray(np.asarray(V, dtype=np.float64).T)
    g = np.ascontiguousarray(group, dtype=np.int32)
    lib().orc_reconstruct(sh.nx, sh.ny, sh.L, sh.li, sh.lj, sh.K, sh.ki, sh.kj, len(sigma),
                          np.ascontiguousarray(sigma, dtype=np.float64), Ucm, Vcm, len(g), g, out)
    return out


def reconstruct_mssa(series_lens, L, sigma, U, V, group) -> list:
    """MSSA diagonal averaging per series on the stacked Hankel matrix."""
    lens = np.asarray(series_lens, np.int32)
    out = np.zeros(int(lens.sum()))
    Ucm = np.ascontiguousarray(np.asarray(U, dtype=np.float64).T)
    Vcm = np.ascontiguousarray(np.asarray(V, dtype=np.float64).T)
    g = np.ascontiguousarray(group, dtype=np.int32)
    lib().orc_reconstruct_mssa(len(lens), lens, L, len(sigma),
                               np.ascontiguousarray(sigma, dtype=np.float64), Ucm, Vcm, len(g), g, out)
    return np.split(out, np.cumsum(lens)[:-1])


def wcor(x, sh: Shapes, sigma, U, V, groups):
    """w-correlations and contributions of reconstructed groups (general-
    notions subsection, separability and w-correlation paragraphs): the
    weighted inner product (Y, Z)_w =
    sum_k w_k y_k z_k with w_k = |A_k| (the number of trajectory-matrix
    entries holding element k), rho_w(Y, Z) = (Y, Z)_w / (|Y|_w |Z|_w)
    without subtracting means, and the contribution of a component Y,
    |Y|_w^2 / |X|_w^2.  Sums run over the covered cells N' (w > 0).
    Returns (rho, contrib): (ng, ng) and (ng,)."""
    cov = sh.W > 0
    w = sh.W[cov]
    comps = [reconstruct(sh, sigma, U, V, g)[cov] for g in groups]
    xc = clean(x, sh)[cov]
    ng = len(groups)
    G = np.zeros((ng, ng))
    for i in range(ng):
        for j in range(ng):
            G[i, j] = np.sum(w * comps[i] * comps[j])
    d = np.sqrt(np.diag(G))
    rho = G / np.outer(d, d)
    contrib = np.diag(G) / np.sum(w * xc * xc)
    return rho, contrib


def lrr_column(U, group):
    """Coefficients of the column recurrent forecast (MSSA forecasting
    subsection, recurrent column forecast, equation Forec:ContMSSAL; one
    series is the case s = 1): with pi(U_j)
    the last coordinate of U_j and nu^2 = sum_j pi(U_j)^2 over the group,
    R_L = sum_j pi(U_j) U_j[0:L-1] / (1 - nu^2), an LRR of order L-1."""
    U = np.asarray(U, dtype=np.float64)
    pi = U[-1, group]
    nu2 = float(np.sum(pi * pi))
    if not nu2 < 1.0:
        raise ValueError("the last coordinates of the group's U span e_L: no recurrent forecast")
    return (U[:-1, group] @ pi) / (1.0 - nu2)


def rforecast_column(recs, U, group, h: int):
    """Column recurrent forecast of h values for each reconstructed series in
    recs (a list of 1-D arrays, the group's reconstruction of each series):
    x_{N+1} = sum_k R_k x_{N-L+1+k} applied to the last L-1 values, then by
    recurrence on the forecast values.  Returns an (s, h) array."""
    R = lrr_column(U, group)
    out = np.zeros((len(recs), h))
    for p, y in enumerate(recs):
        buf = list(np.asarray(y, dtype=np.float64)[-(len(R)):])
        for k in range(h):
            nxt = float(np.dot(R, buf[-len(R):]))
            buf.append(nxt)
            out[p, k] = nxt
    return out


def vforecast_column(series_lens, L: int, sigma, U, V, group, h: int):
    """Column vector forecast (MSSA forecasting subsection, vector MSSA
    forecasting, column forecast; one series is the case s = 1), from its
    definition.  Series p owns the K_p = N_p - L + 1 columns of the stacked
    trajectory matrix (in series order in V).  Its lagged vectors start as
    the columns of the group's reconstructed matrix, Z_k = sum_j sigma_j U_j
    V_j[k]; each next vector is P(Z_{k-1}), where P maps z to (Pi zbar,
    R_L . zbar) with zbar the last L-1 coordinates of z, Pi the orthogonal
    projector onto the span of the group's U_j without their last coordinate
    and R_L the column LRR (equation Forec:ContMSSAL).  After h + L - 1 new
    vectors, the diagonal average of [Z_1 : ... ] holds the forecast at
    positions N_p .. N_p + h - 1.  Returns an (s, h) array."""
    U = np.asarray(U, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    g = list(group)
    R = lrr_column(U, g)                 # raises when nu^2 >= 1
    Qb, _ = np.linalg.qr(U[:-1, g])      # orthonormal basis of the projected span
    lens = [int(n) for n in series_lens]
    out = np.zeros((len(lens), h))
    off = 0
    for p, n in enumerate(lens):
        K = n - L + 1
        Xh = (U[:, g] * sigma[g]) @ V[off:off + K, g].T      # L x K_p
        off += K
        Z = [Xh[:, k] for k in range(K)]
        for _ in range(h + L - 1):
            zbar = Z[-1][1:]
            Z.append(np.concatenate([Qb @ (Qb.T @ zbar), [float(R @ zbar)]]))
        Zm = np.stack(Z, axis=1)
        ncol = Zm.shape[1]
        acc = np.zeros(L + ncol - 1)
        cnt = np.zeros(L + ncol - 1)
        for i in range(L):
            acc[i:i + ncol] += Zm[i]
            cnt[i:i + ncol] += 1.0
        out[p] = (acc / cnt)[n:n + h]
    return out


def esprit(U, group):
    """LS-ESPRIT roots (the 1D parameter-estimation paragraph; the remark on
    the fast column forecast names its shift matrix): the eigenvalues of
    D = U_low^+ U_high, U_low the group's U without its last row, U_high
    without its first (least squares).  A series term c rho^t cos(omega t +
    phi) contributes the roots rho e^{+-i omega}.  Returns complex roots
    sorted by decreasing modulus, then decreasing imaginary part."""
    Ug = np.asarray(U, dtype=np.float64)[:, list(group)]
    D = np.linalg.lstsq(Ug[:-1], Ug[1:], rcond=None)[0]
    return _sorted_roots(np.linalg.eigvals(D))


def esprit_tls(U, group):
    """TLS-ESPRIT roots (the same paragraph; Roy and Kailath's total least
    squares variant): with Z = [U_low : U_high] ((L-1) x 2r) and its right
    singular vectors V = [[V11, V12], [V21, V22]] (r x r blocks, columns by
    decreasing singular value), the shift matrix is -V12 V22^{-1}; its
    eigenvalues are the roots, sorted as for esprit."""
    Ug = np.asarray(U, dtype=np.float64)[:, list(group)]
    r = Ug.shape[1]
    Z = np.hstack([Ug[:-1], Ug[1:]])
    _, _, Vt = np.linalg.svd(Z, full_matrices=False)
    V = Vt.T
    V12, V22 = V[:r, r:], V[r:, r:]
    return _sorted_roots(np.linalg.eigvals(-V12 @ np.linalg.inv(V22)))


def _sorted_roots(z):
    """Roots by decreasing modulus, then decreasing imaginary part."""
    order = sorted(range(len(z)), key=lambda k: (-abs(z[k]), -z[k].imag))
    return z[order]


ESPRIT2D_GAMMA = 0.6180339887498949   # weight of the y shift in the combination whose eigenvectors pair the roots


def esprit2d(sh: Shapes, U, group, gamma: float = ESPRIT2D_GAMMA):
    """2D-ESPRIT (the parameter-estimation subsection of the 2D-SSA
    examples: a pair of shift matrices for the x and y directions and their
    joint diagonalisation).  For the window cells c whose neighbour one step
    down (x) is also in the window, Phi_x = U_a^+ U_b with U_a the group's U
    on those cells and U_b on their neighbours (least squares); Phi_y the
    same for the neighbour one step right.  The eigenvectors T of
    Phi_x + gamma Phi_y diagonalise both (they commute for a signal of
    finite rank); lambda_k and mu_k are the diagonals of T^-1 Phi_x T and
    T^-1 Phi_y T.  A term rho^m tau^n cos(2 pi (m f + n g) + phi) gives the
    pairs (rho e^{+-2 pi i f}, tau e^{+-2 pi i g}).  Returns (lambda, mu)
    sorted by decreasing |lambda|, then decreasing Im lambda."""
    Ug = np.asarray(U, dtype=np.float64)[:, list(group)]
    pos = {(int(a), int(b)): c for c, (a, b) in enumerate(zip(sh.li, sh.lj))}
    phis = []
    for da, db in ((1, 0), (0, 1)):
        src = [c for (a, b), c in pos.items() if (a + da, b + db) in pos]
        dst = [pos[(int(sh.li[c]) + da, int(sh.lj[c]) + db)] for c in src]
        phis.append(np.linalg.lstsq(Ug[src], Ug[dst], rcond=None)[0])
    px, py = phis
    _, T = np.linalg.eig(px + gamma * py)
    Ti = np.linalg.inv(T)
    lam = np.diag(Ti @ px @ T)
    mu = np.diag(Ti @ py @ T)
    order = sorted(range(len(lam)), key=lambda k: (-abs(lam[k]), -lam[k].imag))
    return lam[order], mu[order]


def _row_blocks(series_lens, L):
    """Start and end (exclusive) of each series' block of K_p = N_p - L + 1
    columns in the stacked trajectory matrix."""
    ks = [int(n) - L + 1 for n in series_lens]
    ends = np.cumsum(ks)
    return [(int(e - k), int(e)) for k, e in zip(ks, ends)]


def lrr_row(series_lens, L, V, group):
    """Coefficients of the recurrent row forecast (MSSA forecasting
    subsection, recurrent row forecast, equation Forec:ContMSSAK):
    R_K = (I_s - S S^T)^{-1} S Vlow^T, an s x (K - s) matrix, where S holds
    the last coordinate of each series' block of the group's V_j (s x ng) and
    Vlow the group's V_j without those coordinates (blocks in series order).
    Row p applied to the stacked last K_q - 1 values of every series q gives
    the next value of series p."""
    V = np.asarray(V, dtype=np.float64)[:, list(group)]
    blocks = _row_blocks(series_lens, L)
    S = np.array([V[e - 1] for _, e in blocks])
    Vlow = np.concatenate([V[b:e - 1] for b, e in blocks])
    Ms = np.eye(len(blocks)) - S @ S.T
    if np.linalg.cond(Ms) > 1e12:
        raise ValueError("I - S S^T is singular: no row forecast")
    return np.linalg.solve(Ms, S @ Vlow.T)


def rforecast_row(recs, L, V, group, h: int):
    """Recurrent row forecast of h values for each reconstructed series in
    recs (the group's reconstruction of each series): the next values of
    all series are R_K times the stacked last K_p - 1 values of every
    series, then by recurrence on the extended series.  Returns (s, h)."""
    lens = [len(y) for y in recs]
    R = lrr_row(lens, L, V, group)
    ext = [list(np.asarray(y, dtype=np.float64)) for y in recs]
    out = np.zeros((len(recs), h))
    for m in range(h):
        Z = np.concatenate([np.asarray(e[len(e) - (n - L):]) for e, n in zip(ext, lens)])
        nxt = R @ Z
        for p in range(len(recs)):
            ext[p].append(float(nxt[p]))
        out[:, m] = nxt
    return out


def vforecast_row(series_lens, L: int, sigma, U, V, group, h: int):
    """Row vector forecast (MSSA forecasting subsection, vector MSSA
    forecasting, row forecast), from its definition.  The rows Y_i of the
    group's reconstructed matrix (K-vectors, i < L) are continued by the map
    that takes the first-dropped part of each block of the previous row
    (all but the first coordinate of each block), projects it onto the span
    of the group's V_j without the last coordinate of each block for the
    new row's leading coordinates, and takes R_K of it for the new row's
    last coordinate of each block.  After h + K* - 1 new rows (K* the
    largest K_p), each series is the diagonal average of its block of
    columns; positions N_p .. N_p + h - 1 are its forecast.  Returns (s, h)."""
    U = np.asarray(U, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    g = list(group)
    lens = [int(n) for n in series_lens]
    blocks = _row_blocks(lens, L)
    R = lrr_row(lens, L, V, g)
    Vg = V[:, g]
    Qb, _ = np.linalg.qr(np.concatenate([Vg[b:e - 1] for b, e in blocks]))
    Xh = (U[:, g] * sigma[g]) @ Vg.T                     # L x K
    rows = [Xh[i] for i in range(L)]
    kstar = max(e - b for b, e in blocks)
    for _ in range(h + kstar - 1):
        prev = rows[-1]
        zf = np.concatenate([prev[b + 1:e] for b, e in blocks])    # each block without its first
        low = Qb @ (Qb.T @ zf)
        last = R @ zf
        new = np.zeros_like(prev)
        o = 0
        for p, (b, e) in enumerate(blocks):
            new[b:e - 1] = low[o:o + (e - 1 - b)]
            new[e - 1] = last[p]
            o += e - 1 - b
        rows.append(new)
    Zm = np.stack(rows)                                  # (L + h + K* - 1) x K
    out = np.zeros((len(lens), h))
    for p, (b, e) in enumerate(blocks):
        blk = Zm[:, b:e]
        nr, kp = blk.shape
        acc = np.zeros(nr + kp - 1)
        cnt = np.zeros(nr + kp - 1)
        for k in range(kp):
            acc[k:k + nr] += blk[:, k]
            cnt[k:k + nr] += 1.0
        out[p] = (acc / cnt)[lens[p]:lens[p] + h]
    return out


# --------------------------------------------------------------------------
# whole decompositions
# --------------------------------------------------------------------------

def decompose(x, mask=None, wmask=None, window=None, method: str = "jacobi", nvec: int = -1):
    """Shaped decomposition: returns (Shapes, sigma, U, V) with all triplets."""
    sh = shapes(x, mask, wmask, window)
    if sh.K == 0:
        raise ValueError("no window position fits")
    X = trajectory(x, sh)
    s, U, V = svd(X, method, nvec=nvec)
    del X
    return sh, s, U, V


def reconstruct_at(sh: Shapes, sigma, U, V, group, cells) -> np.ndarray:
    """The group's diagonal average at the listed cells ((n, 2) int array)."""
    kx, ky = sh.nx - sh.lxt + 1, sh.ny - sh.lyt + 1
    korigin = np.full(kx * ky, -1, np.int64)
    korigin[sh.ki.astype(np.int64) * ky + sh.kj] = np.arange(sh.K)
    cells = np.asarray(cells, np.int32)
    out = np.zeros(len(cells))
    Ucm = np.ascontiguousarray(np.asarray(U, dtype=np.float64).T)
    Vcm = np.ascontiguousarray(np.asarray(V, dtype=np.float64).T)
    g = np.ascontiguousarray(group, dtype=np.int32)
    lib().orc_reconstruct_at(sh.L, sh.li, sh.lj, kx, ky, korigin, sh.K, len(sigma),
                             np.ascontiguousarray(sigma, dtype=np.float64), Ucm, Vcm, len(g), g,
                             len(cells), np.ascontiguousarray(cells[:, 0]),
                             np.ascontiguousarray(cells[:, 1]), out)
    return out


def decompose_mssa(series, L: int, method: str = "jacobi", nvec: int = -1):
    """MSSA decomposition on the stacked Hankel matrix: (sigma, U, V)."""
    X = trajectory_mssa(series, L)
    return svd(X, method, nvec=nvec)


def trajectory_m2d(images, window, wmask=None) -> np.ndarray:
    """M-2D-SSA trajectory matrix (the shaped-variants section, equation
    embedding_m2dssa): the 2D-SSA trajectory matrices of the images side by
    side, [T(X_1) : ... : T(X_s)], each with the same (shaped) window."""
    return np.hstack([trajectory(x, shapes(x, None, wmask, window)) for x in images])


def pack_m2d(images, window, wmask=None) -> np.ndarray:
    """The packing of the same section: the images side by side in one
    array (rows = the tallest image), NaN below shorter images and in the
    separator columns between them, so that no window fits across two
    images.  One separator column, as printed, for a full window; ly - 1
    columns for a shaped window, which may have holes where a separator
    would fall."""
    lx, ly = (window, 1) if np.isscalar(window) else window
    sep = 1 if wmask is None else max(1, ly - 1)
    nx = max(x.shape[0] for x in images)
    ny = sum(x.shape[1] for x in images) + sep * (len(images) - 1)
    out = np.full((nx, ny), np.nan)
    c = 0
    for x in images:
        out[:x.shape[0], c:c + x.shape[1]] = x
        c += x.shape[1] + sep
    return out


def mosaic_hankel(series, Ls, Ks) -> np.ndarray:
    """Mosaic Hankel matrix (the mosaic Hankel subsection): block (i, j) is
    the L_i x K_j Hankel matrix of series[i][j] (length L_i + K_j - 1),
    entry (b, k) = series[i][j][b + k]; block rows of L_i rows, block
    columns of K_j columns."""
    rows = []
    for i, L in enumerate(Ls):
        blocks = []
        for j, K in enumerate(Ks):
            x = np.asarray(series[i][j], dtype=np.float64)
            if len(x) != L + K - 1:
                raise ValueError("series (%d, %d) needs length L_i + K_j - 1" % (i, j))
            H = np.empty((L, K))
            for b in range(L):
                for k in range(K):
                    H[b, k] = x[b + k]
            blocks.append(H)
        rows.append(np.hstack(blocks))
    return np.vstack(rows)


def pack_mosaic(series, Ls, Ks):
    """Shaped packing of a mosaic Hankel matrix (the same subsection: stacked
    shapes with separators): (array, window, wmask).  Row i of an s-row
    array holds series[i][j] from column c_j on; the block columns follow
    each other with one NaN column after the longest series of the block
    (c_{j+1} = c_j + max L + K_j).  The window has s rows, row i its first
    L_i cells; its positions that fit are exactly the K_j origins of each
    block column, so the shaped trajectory matrix is the mosaic matrix."""
    s, t = len(Ls), len(Ks)
    Lm = max(Ls)
    offs = [0]
    for K in Ks[:-1]:
        offs.append(offs[-1] + Lm + K)
    width = offs[-1] + Lm + Ks[-1] - 1
    out = np.full((s, width), np.nan)
    for i, L in enumerate(Ls):
        for j, K in enumerate(Ks):
            out[i, offs[j]:offs[j] + L + K - 1] = series[i][j]
    wmask = np.zeros((s, Lm), np.uint8)
    for i, L in enumerate(Ls):
        wmask[i, :L] = 1
    return out, (s, Lm), wmask


def reconstruct_mosaic(series, Ls, Ks, group):
    """The group's reconstruction of every series of a mosaic Hankel matrix
    (the embedding, grouping and diagonal averaging steps on the mosaic
    matrix): the sum of sigma_k U_k V_k^T over the group, each block averaged
    along its anti-diagonals.  Returns the nested list of series."""
    M = mosaic_hankel(series, Ls, Ks)
    U, s, Vt = np.linalg.svd(M, full_matrices=False)
    g = list(group)
    Mg = (U[:, g] * s[g]) @ Vt[g]
    out = []
    r0 = 0
    for L in Ls:
        row = []
        c0 = 0
        for K in Ks:
            blk = Mg[r0:r0 + L, c0:c0 + K]
            acc = np.zeros(L + K - 1)
            cnt = np.zeros(L + K - 1)
            for b in range(L):
                for k in range(K):
                    acc[b + k] += blk[b, k]
                    cnt[b + k] += 1
            row.append(acc / cnt)
            c0 += K
        out.append(row)
        r0 += L
    return out


def grid(sh: Shapes, vec, which: str) -> np.ndarray:
    """Place a compact vector on its (Lx, Ly) or (Kx, Ky) box, NaN elsewhere."""
    if which == "L":
        out = np.full((sh.lxt, sh.lyt), np.nan)
        out[sh.li, sh.lj] = vec
    else:
        out = np.full((sh.nx - sh.lxt + 1, sh.ny - sh.lyt + 1), np.nan)
        out[sh.ki, sh.kj] = vec
    return out
