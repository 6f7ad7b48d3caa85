"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these tests retypes the oracle's own formula: each compares it with
an independent construction (a LAPACK SVD, scipy's Hankel builder, an FFT
correlation, a dense least-squares solve), a closed form, an invariant, or a
value the paper prints.
"""
import numpy as np
import pytest
import scipy.linalg as sla
from scipy import signal

import oracle
from paper_1309_5050_amd import workloads as W


def _proj(U):
    return U @ U.T


# --------------------------------------------------------------------------
# the SVD step
# --------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(30, 17), (17, 30), (25, 25), (64, 9), (3, 3), (1, 7)])
@pytest.mark.parametrize("method", ["jacobi", "gram"])
def test_svd_matches_lapack(shape, method):
    rng = np.random.default_rng(sum(shape))
    A = rng.standard_normal(shape)
    s, U, V = oracle.svd(A, method)
    s_ref = np.linalg.svd(A, compute_uv=False)
    tol = 1e-13 if method == "jacobi" else 1e-12
    assert np.allclose(s, s_ref, rtol=0, atol=tol * s_ref[0])
    assert np.allclose(U @ np.diag(s) @ V.T, A, atol=1e-12 * s_ref[0])
    d = min(shape)
    assert np.allclose(U.T @ U, np.eye(d), atol=1e-12)
    assert np.allclose(V.T @ V, np.eye(d), atol=1e-10)
    assert np.all(np.diff(s) <= 0)


def test_svd_rank_deficient():
    rng = np.random.default_rng(5)
    A = rng.standard_normal((20, 3)) @ rng.standard_normal((3, 15))
    s, U, V = oracle.svd(A)
    assert np.all(s[3:] < 1e-12 * s[0])
    assert np.allclose(U[:, :3] @ np.diag(s[:3]) @ V[:, :3].T, A, atol=1e-12 * s[0])


def test_svd_sign_rule():
    rng = np.random.default_rng(6)
    A = rng.standard_normal((12, 20))
    s, U, V = oracle.svd(A)
    for k in range(U.shape[1]):
        a = int(np.argmax(np.abs(U[:, k])))
        assert U[a, k] > 0


def test_gram_and_jacobi_agree_on_ssa():
    w = W.series_1d(n=300, L=120)
    sh = oracle.shapes(w["x"], window=w["window"])
    X = oracle.trajectory(w["x"], sh)
    s1, U1, V1 = oracle.svd(X, "jacobi")
    s2, U2, V2 = oracle.svd(X, "gram")
    assert np.allclose(s1, s2, atol=1e-11 * s1[0])
    # gap-stable leading subspace
    assert np.linalg.norm(_proj(U1[:, :1]) - _proj(U2[:, :1]), 2) < 1e-10


# --------------------------------------------------------------------------
# shapes, trajectory matrices and weights
# --------------------------------------------------------------------------

def test_window_trim_and_order():
    wm = np.zeros((4, 5), np.uint8)
    wm[1, 2] = wm[2, 1] = wm[2, 3] = wm[3, 2] = 1     # a plus sign without its centre
    sh = oracle.shapes(np.zeros((10, 10)), wmask=wm)
    assert (sh.lxt, sh.lyt) == (3, 3)
    # column-major: column 0 -> (1,0); column 1 -> (0,1),(2,1); column 2 -> (1,2)
    assert list(zip(sh.li, sh.lj)) == [(1, 0), (0, 1), (2, 1), (1, 2)]


def test_trajectory_sizes_printed_in_paper():
    # 2D-SSA of a 258 x 275 image: 25x25 window -> 625 x 58734,
    # 160x80 window -> 12800 x 19404 (both printed in the 2D-SSA examples).
    x = np.zeros((258, 275))
    sh = oracle.shapes(x, window=(25, 25))
    assert (sh.L, sh.K) == (625, 58734)
    sh = oracle.shapes(x, window=(160, 80))
    assert (sh.L, sh.K) == (12800, 19404)


def test_kset_matches_correlation_count():
    w = W.small_shaped()
    sh = oracle.shapes(w["x"], w["mask"], w["wmask"])
    nset = (w["mask"].astype(bool) & ~np.isnan(w["x"])).astype(float)
    wm = np.asarray(w["wmask"], bool)
    # trim the window box, then count covered cells of every placement
    rows, cols = np.nonzero(wm)
    wm = wm[rows.min():rows.max() + 1, cols.min():cols.max() + 1]
    cnt = signal.correlate2d(nset, wm.astype(float), mode="valid")
    ref = np.argwhere(np.round(cnt) == wm.sum())
    got = set(zip(sh.ki.tolist(), sh.kj.tolist()))
    assert got == set(map(tuple, ref.tolist()))
    # column-major order
    key = sh.kj.astype(np.int64) * 10000 + sh.ki
    assert np.all(np.diff(key) > 0)


def test_kset_brute_force_tiny():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((7, 6))
    x[rng.random((7, 6)) < 0.15] = np.nan
    wm = np.array([[1, 1], [0, 1]], np.uint8)
    sh = oracle.shapes(x, wmask=wm)
    ref = []
    for b in range(6 - 2 + 1):
        for a in range(7 - 2 + 1):
            if all(not np.isnan(x[a + i, b + j]) for i in range(2) for j in range(2) if wm[i, j]):
                ref.append((a, b))
    assert list(zip(sh.ki.tolist(), sh.kj.tolist())) == ref


def test_full_rectangle_is_hankel_block_hankel():
    rng = np.random.default_rng(1)
    nx, ny, lx, ly = 9, 7, 4, 3
    x = rng.standard_normal((nx, ny))
    sh = oracle.shapes(x, window=(lx, ly))
    X = oracle.trajectory(x, sh)
    kx = nx - lx + 1
    H = [sla.hankel(x[:lx, j], x[lx - 1:, j]) for j in range(ny)]   # Lx x Kx blocks
    HbH = np.block([[H[a + b] for b in range(ny - ly + 1)] for a in range(ly)])
    assert HbH.shape == (lx * ly, kx * (ny - ly + 1))
    assert np.array_equal(X, HbH)


def test_series_is_ssa_hankel():
    w = W.series_1d(n=50, L=20)
    sh = oracle.shapes(w["x"], window=20)
    X = oracle.trajectory(w["x"], sh)
    assert np.array_equal(X, sla.hankel(w["x"][:20], w["x"][19:]))


def test_mssa_2d_and_1d_packing():
    w = W.mssa_series(s=4, nmin=30, nmax=50, L=10)
    ser, L = w["x"], w["window"]
    Xs = oracle.trajectory_mssa(ser, L)
    # stacked Hankel from scipy
    ref = np.hstack([sla.hankel(s[:L], s[L - 1:]) for s in ser])
    assert np.array_equal(Xs, ref)
    # 2D packing: max N_p x s array, shape = union of {1..N_p} x {p}, window L x 1
    nmax = max(len(s) for s in ser)
    arr = np.full((nmax, len(ser)), np.nan)
    for p, s in enumerate(ser):
        arr[:len(s), p] = s
    sh = oracle.shapes(arr, window=(L, 1))
    assert np.array_equal(oracle.trajectory(arr, sh), Xs)
    # 1D packing with one-element separators outside the shape
    sep = np.concatenate(sum([[s, [np.nan]] for s in ser], [])[:-1])
    sh1 = oracle.shapes(sep, window=L)
    assert np.array_equal(oracle.trajectory(sep, sh1), Xs)


def test_weights_1d_closed_form():
    n, L = 37, 11
    sh = oracle.shapes(np.zeros(n), window=L)
    K = n - L + 1
    k = np.arange(1, n + 1)
    ref = np.minimum.reduce([k, np.full(n, L), np.full(n, K), n - k + 1])
    assert np.array_equal(sh.W[:, 0], ref)


def test_weights_2d_rectangle_are_separable():
    nx, ny, lx, ly = 12, 9, 5, 3
    sh = oracle.shapes(np.zeros((nx, ny)), window=(lx, ly))

    def w1(n, L):
        k = np.arange(1, n + 1)
        return np.minimum.reduce([k, np.full(n, L), np.full(n, n - L + 1), n - k + 1])
    assert np.array_equal(sh.W, np.outer(w1(nx, lx), w1(ny, ly)))


def test_shaped_covered_set_is_minkowski_sum():
    w = W.small_shaped()
    sh = oracle.shapes(w["x"], w["mask"], w["wmask"])
    cov = np.zeros((sh.nx, sh.ny), bool)
    for a, b in zip(sh.ki, sh.kj):
        cov[a + sh.li, b + sh.lj] = True
    assert np.array_equal(cov, sh.covered)
    assert np.all(sh.nset[cov] == 1)


def test_explicit_products():
    w = W.small_shaped()
    sh = oracle.shapes(w["x"], w["mask"], w["wmask"])
    X = oracle.trajectory(w["x"], sh)
    rng = np.random.default_rng(2)
    v = rng.standard_normal(sh.K)
    u = rng.standard_normal(sh.L)
    assert np.allclose(oracle.matvec(w["x"], sh, v), X @ v, atol=1e-12)
    assert np.allclose(oracle.rmatvec(w["x"], sh, u), X.T @ u, atol=1e-12)


# --------------------------------------------------------------------------
# the lemmas behind the fast products (checked on explicit circulants)
# --------------------------------------------------------------------------

def test_hankel_circulant_lemma():
    # C_H(X) A = F^-1(F X . conj(F A)) for real A (implementation section)
    rng = np.random.default_rng(4)
    n = 11
    x = rng.standard_normal(n)
    a = rng.standard_normal(n)
    CH = np.array([[x[(i + j) % n] for j in range(n)] for i in range(n)])
    lhs = CH @ a
    rhs = np.fft.ifft(np.fft.fft(x) * np.conj(np.fft.fft(a))).real
    assert np.allclose(lhs, rhs, atol=1e-12)


def test_hbh_circulant_lemma():
    rng = np.random.default_rng(8)
    nx, ny = 5, 4
    X = rng.standard_normal((nx, ny))
    A = rng.standard_normal((nx, ny))
    vec = lambda M: M.flatten(order="F")
    # HbH circulant: block (a, b) = C_H(column (a+b) mod ny)
    def ch(col):
        return np.array([[col[(i + j) % nx] for j in range(nx)] for i in range(nx)])
    C = np.block([[ch(X[:, (a + b) % ny]) for b in range(ny)] for a in range(ny)])
    rhs = np.fft.ifft2(np.fft.fft2(X) * np.conj(np.fft.fft2(A))).real
    assert np.allclose(C @ vec(A), vec(rhs), atol=1e-12)


# --------------------------------------------------------------------------
# invariants of the decomposition
# --------------------------------------------------------------------------

def test_frobenius_invariant_shaped():
    w = W.small_shaped()
    sh, s, U, V = oracle.decompose(w["x"], w["mask"], w["wmask"])
    X = oracle.trajectory(w["x"], sh)
    xc = oracle.clean(w["x"], sh)
    fro = np.sum(X ** 2)
    assert np.isclose(np.sum(s ** 2), fro, rtol=1e-13)
    assert np.isclose(np.sum(sh.W * xc ** 2), fro, rtol=1e-13)


def test_elementary_components_sum_to_input():
    w = W.small_shaped()
    sh, s, U, V = oracle.decompose(w["x"], w["mask"], w["wmask"])
    tot = oracle.reconstruct(sh, s, U, V, list(range(len(s))))
    cov = sh.covered
    assert np.allclose(tot[cov], w["x"][cov], atol=1e-11)
    assert np.all(np.isnan(tot[~cov]))
    # reconstructions are linear in the group
    g1 = oracle.reconstruct(sh, s, U, V, [0, 1])
    g2 = oracle.reconstruct(sh, s, U, V, list(range(2, len(s))))
    assert np.allclose(g1[cov] + g2[cov], w["x"][cov], atol=1e-11)


def _reconstruct_at_cases():
    """A shaped case, a holed non-square 2D case with a holed window, and 1D
    series in both orientations: reconstruct_at must equal reconstruct."""
    cases = []
    w = W.small_shaped()
    cases.append((w["x"], w["mask"], w["wmask"], w["window"]))
    g = np.random.default_rng(41)
    x = g.standard_normal((17, 11))
    x[3:5, 6:8] = np.nan
    x[12, 2] = np.nan
    wm = np.ones((5, 3), np.uint8)
    wm[2, 1] = 0
    cases.append((x, None, wm, (5, 3)))
    t = np.arange(1, 61)
    y = np.cos(2 * np.pi * t / 7) + 0.05 * g.standard_normal(60)
    cases.append((y.reshape(60, 1), None, None, (18, 1)))
    cases.append((y.reshape(1, 60), None, None, (1, 18)))
    return cases


@pytest.mark.parametrize("case", range(4))
def test_reconstruct_at_equals_reconstruct_everywhere(case):
    x, mask, wmask, window = _reconstruct_at_cases()[case]
    sh, s, U, V = oracle.decompose(x, mask, wmask, window)
    nx, ny = sh.nx, sh.ny
    cells = np.array([(i, j) for i in range(nx) for j in range(ny)], np.int32)
    for group in ([0], [0, 1, 2], list(range(len(s)))):
        ref = oracle.reconstruct(sh, s, U, V, group)
        got = oracle.reconstruct_at(sh, s, U, V, group, cells).reshape(nx, ny)
        assert np.array_equal(np.isnan(got), np.isnan(ref))
        assert np.array_equal(~np.isnan(ref), sh.covered)
        cov = sh.covered
        assert np.allclose(got[cov], ref[cov], rtol=1e-12, atol=1e-12 * np.nanmax(np.abs(ref)))


def test_hankelization_is_least_squares():
    # The averaging is the Frobenius-optimal structured approximation
    # (Section 2.1, Step 4): solve min_y |T(y) - Y|_F densely.
    rng = np.random.default_rng(9)
    x = rng.standard_normal((5, 4))
    x[0, 3] = np.nan
    wm = np.array([[1, 1], [1, 0]], np.uint8)
    sh = oracle.shapes(x, wmask=wm)
    Y = rng.standard_normal((sh.L, sh.K))
    U, s, Vh = np.linalg.svd(Y, full_matrices=False)
    V = Vh.T
    got = oracle.reconstruct(sh, s, U, V, list(range(len(s))))
    cells = np.argwhere(sh.covered)
    T = np.zeros((sh.L * sh.K, len(cells)))
    index = {tuple(c): t for t, c in enumerate(cells)}
    for i in range(sh.L):
        for j in range(sh.K):
            T[i * sh.K + j, index[(sh.li[i] + sh.ki[j], sh.lj[i] + sh.kj[j])]] = 1.0
    y, *_ = np.linalg.lstsq(T, Y.ravel(), rcond=None)
    assert np.allclose(got[sh.covered], y, atol=1e-12)


# --------------------------------------------------------------------------
# closed forms
# --------------------------------------------------------------------------

def test_sine_has_rank_two_with_closed_form_sigma():
    # A cos(2 pi w t + phi) with L w and K w integers: sigma_1 = sigma_2 =
    # A sqrt(LK)/2 (MSSA theory example with one series).
    n, L, A = 959, 480, 1.7
    t = np.arange(n)
    x = A * np.cos(2 * np.pi * t / 12 + 0.4)
    sh, s, U, V = oracle.decompose(x, window=L)
    K = n - L + 1
    assert np.allclose(s[:2], A * np.sqrt(L * K) / 2, rtol=1e-12)
    assert s[2] < 1e-10 * s[0]


def test_exponential_has_rank_one():
    n, L, a = 60, 25, 0.93
    t = np.arange(1, n + 1)
    x = a ** t
    sh, s, U, V = oracle.decompose(x, window=L)
    K = n - L + 1
    ref = a * np.sqrt(np.sum(a ** (2 * np.arange(L)))) * np.sqrt(np.sum(a ** (2 * np.arange(K))))
    assert np.isclose(s[0], ref, rtol=1e-13)
    assert s[1] < 1e-12 * s[0]


def test_separable_image_sigmas_are_products():
    # f g^T has trajectory matrix T(g) kron T(f) -> sigmas are products.
    rng = np.random.default_rng(12)
    f = rng.standard_normal(14)
    g = rng.standard_normal(11)
    lx, ly = 5, 4
    sh, s, U, V = oracle.decompose(np.outer(f, g), window=(lx, ly))
    sf = np.linalg.svd(sla.hankel(f[:lx], f[lx - 1:]), compute_uv=False)
    sg = np.linalg.svd(sla.hankel(g[:ly], g[ly - 1:]), compute_uv=False)
    ref = np.sort(np.outer(sf, sg).ravel())[::-1]
    assert np.allclose(s, ref[:len(s)], atol=1e-12 * ref[0])


def test_product_of_cosines_has_rank_four():
    m = np.arange(30)[:, None]
    n = np.arange(28)[None, :]
    x = 2 * np.cos(2 * np.pi * m / 7 + 0.3) * np.cos(2 * np.pi * n / 5 + 1.1)
    sh, s, U, V = oracle.decompose(x, window=(10, 9))
    assert s[3] > 1e-3 * s[0]
    assert s[4] < 1e-10 * s[0]


def test_mssa_matched_sines_eigenvalues():
    # lambda_1 = lambda_2 = (A^2 + B^2) L K / 4 when L w, K w are integers.
    n, L, A, B = 120, 60, 2.0, 1.3
    t = np.arange(n)
    ser = [A * np.cos(2 * np.pi * t / 12 + 0.2), B * np.cos(2 * np.pi * t / 12 + 1.4)]
    s, U, V = oracle.decompose_mssa(ser, L)
    K = n - L + 1
    # K = 61 is not a multiple of 12: use the s-series form with K w integer
    n, L = 119, 60
    ser = [A * np.cos(2 * np.pi * np.arange(n) / 12 + 0.2),
           B * np.cos(2 * np.pi * np.arange(n) / 12 + 1.4)]
    s, U, V = oracle.decompose_mssa(ser, L)
    K = 2 * (n - L + 1)        # total columns of the stacked matrix
    Kp = n - L + 1
    lam = (A ** 2 + B ** 2) * L * Kp / 4
    assert np.allclose(s[:2] ** 2, lam, rtol=1e-12)
    assert s[2] < 1e-10 * s[0]
    assert K == 120


def test_table2_signal_ranks():
    # Dimension of the signal trajectory space, Examples A, B, C: SSA 2/2/2,
    # MSSA 2/2/4 (N = 71; L = 24).
    k = np.arange(1, 72)
    ex = {
        "A": (30 * np.cos(2 * np.pi * k / 12), 20 * np.cos(2 * np.pi * k / 12 + np.pi / 4)),
        "B": (30 * np.cos(2 * np.pi * k / 12), 30 * np.cos(2 * np.pi * k / 12 + np.pi / 2)),
        "C": (30 * np.cos(2 * np.pi * k / 12), 20 * np.cos(2 * np.pi * k / 8 + np.pi / 4)),
    }
    mssa_rank = {"A": 2, "B": 2, "C": 4}

    def rank(s):
        return int(np.sum(s > 1e-9 * s[0]))
    for name, (h1, h2) in ex.items():
        s, _, _ = oracle.decompose_mssa([h1, h2], 24)
        assert rank(s) == mssa_rank[name], name
        for h in (h1, h2):
            _, s1, _, _ = oracle.decompose(h, window=24)
            assert rank(s1) == 2


def test_window_symmetry_L_K():
    # SSA(L) and SSA(N-L+1) have transposed trajectory matrices: same sigmas,
    # U and V swap roles.
    w = W.series_1d(n=90, L=30)
    x = w["x"]
    _, s1, U1, V1 = oracle.decompose(x, window=30)
    _, s2, U2, V2 = oracle.decompose(x, window=61)
    assert np.allclose(s1, s2, atol=1e-11 * s1[0])
    assert np.linalg.norm(_proj(U1[:, :1]) - _proj(V2[:, :1]), 2) < 1e-9


# --------------------------------------------------------------------------
# the paper's Monte Carlo table (reconstruction MSE), reduced replication
# --------------------------------------------------------------------------

@pytest.mark.slow
def test_table3_reconstruction_mse():
    """SSA (L=24: 2.00, L=12: 3.22) and MSSA Ex. B (L=24: 1.82), sigma^2 = 25,
    N = 71.  1500 replications; the check allows 5 Monte Carlo standard errors."""
    rng = np.random.default_rng(2024)
    k = np.arange(1, 72)
    h1 = 30 * np.cos(2 * np.pi * k / 12)
    h2 = 30 * np.cos(2 * np.pi * k / 12 + np.pi / 2)
    reps = 1500
    res = {"ssa24": [], "ssa12": [], "mssa24": []}
    for _ in range(reps):
        x1 = h1 + rng.normal(0, 5, 71)
        x2 = h2 + rng.normal(0, 5, 71)
        for L, key in ((24, "ssa24"), (12, "ssa12")):
            m = 0.0
            for x, h in ((x1, h1), (x2, h2)):
                sh, s, U, V = oracle.decompose(x, window=L)
                rec = oracle.reconstruct(sh, s, U, V, [0, 1])[:, 0]
                m += np.mean((rec - h) ** 2)
            res[key].append(m / 2)
        s, U, V = oracle.decompose_mssa([x1, x2], 24)
        r1, r2 = oracle.reconstruct_mssa([71, 71], 24, s, U, V, [0, 1])
        res["mssa24"].append((np.mean((r1 - h1) ** 2) + np.mean((r2 - h2) ** 2)) / 2)
    for key, ref in (("ssa24", 2.00), ("ssa12", 3.22), ("mssa24", 1.82)):
        v = np.array(res[key])
        se = v.std() / np.sqrt(reps)
        assert abs(v.mean() - ref) < 5 * se + 0.005, (key, v.mean(), ref, se)


# --------------------------------------------------------------------------
# w-correlations and contributions
# --------------------------------------------------------------------------

def test_wcor_is_frobenius_correlation_of_trajectory_matrices():
    """rho_w of two reconstructed components equals the normalised Frobenius
    inner product of their trajectory matrices (the paper's definition via
    rho(X~_1, X~_2)), and the contribution equals |T(X~_j)|_F^2 / |X|_F^2."""
    w = W.small_shaped()
    sh, s, U, V = oracle.decompose(w["x"], w["mask"], w["wmask"])
    groups = [[0, 1], [2], [3, 4, 5]]
    rho, contrib = oracle.wcor(w["x"], sh, s, U, V, groups)
    T = [oracle.trajectory(oracle.reconstruct(sh, s, U, V, g), sh) for g in groups]
    X = oracle.trajectory(w["x"], sh)
    for i in range(3):
        assert np.isclose(contrib[i], np.sum(T[i] ** 2) / np.sum(X ** 2), rtol=1e-12)
        for j in range(3):
            ref = np.sum(T[i] * T[j]) / np.sqrt(np.sum(T[i] ** 2) * np.sum(T[j] ** 2))
            assert abs(rho[i, j] - ref) <= 1e-12
    assert np.allclose(rho, rho.T) and np.allclose(np.diag(rho), 1.0)
    assert np.all(np.abs(rho) <= 1 + 1e-12)


def test_wcor_of_a_complete_grouping_recovers_the_norm():
    """The groups of a complete grouping sum to x on N', so the weighted
    inner products of all pairs add up to |X|_w^2: sum_ij rho_ij
    sqrt(c_i c_j) = 1."""
    x = W.series_1d(n=120, L=40, r=6, seed=8)["x"]
    sh, s, U, V = oracle.decompose(x, None, None, 40)
    groups = [[0], [1, 2], [3, 4], list(range(5, len(s)))]
    rho, c = oracle.wcor(x, sh, s, U, V, groups)
    assert abs(np.sum(rho * np.sqrt(np.outer(c, c))) - 1.0) <= 1e-11


def test_wcor_of_exactly_separable_components():
    """x_t = a + b(-1)^t with L and K even: the constant and the alternating
    series have orthogonal row and column trajectory spaces and distinct
    singular values a sqrt(LK) and |b| sqrt(LK), so the two elementary
    reconstructions are exactly a and b(-1)^t.  Their w-correlation and
    contributions then follow from the 1D weights w_k = min(k, L, K, N-k+1)
    and the known signals."""
    N, L, a, b = 31, 10, 1.5, -0.7
    K = N - L + 1
    t = np.arange(N)
    x = a + b * (-1.0) ** t
    # rank 2 (the other singular values vanish): the Gram route of the SVD step
    sh, s, U, V = oracle.decompose(x, None, None, L, method="gram")
    assert np.isclose(s[0], a * np.sqrt(L * K)) and np.isclose(s[1], abs(b) * np.sqrt(L * K))
    rho, c = oracle.wcor(x, sh, s, U, V, [[0], [1]])
    wk = np.minimum.reduce([t + 1, np.full(N, L), np.full(N, K), N - t])
    f1, f2 = np.full(N, a), b * (-1.0) ** t
    ip = lambda p, q: np.sum(wk * p * q)
    assert abs(rho[0, 1] - ip(f1, f2) / np.sqrt(ip(f1, f1) * ip(f2, f2))) <= 1e-12
    assert np.allclose(c, [ip(f1, f1) / ip(x, x), ip(f2, f2) / ip(x, x)], rtol=1e-12)


# --------------------------------------------------------------------------
# recurrent (column) forecast
# --------------------------------------------------------------------------

def _lapack_svd(X):
    # exactly low-rank matrices: LAPACK's SVD (the oracle's Jacobi routes
    # need a numerically full spectrum to meet their convergence test)
    U, s, Vt = np.linalg.svd(X, full_matrices=False)
    return s, U, Vt.T


def _rank_r_forecast(x, L, group, h):
    sh = oracle.shapes(x, None, None, L)
    s, U, V = _lapack_svd(oracle.trajectory(x, sh))
    rec = oracle.reconstruct(sh, s, U, V, group)[:, 0]
    return oracle.rforecast_column([rec], U, group, h)[0]


def test_rforecast_continues_a_sine():
    """A pure cosine has rank 2 and satisfies an LRR: the forecast from the
    group {1,2} continues it exactly."""
    N, L, h = 96, 36, 30
    t = np.arange(N + h)
    x = 1.3 * np.cos(2 * np.pi * t / 12 + 0.4)
    f = _rank_r_forecast(x[:N], L, [0, 1], h)
    assert np.max(np.abs(f - x[N:])) <= 1e-9


def test_rforecast_continues_an_exponential_and_a_line():
    N, L, h = 60, 20, 15
    t = np.arange(N + h)
    x = 0.97 ** t
    assert np.max(np.abs(_rank_r_forecast(x[:N], L, [0], h) - x[N:])) <= 1e-10
    y = 2.0 + 0.1 * t          # a linear trend has rank 2
    assert np.max(np.abs(_rank_r_forecast(y[:N], L, [0, 1], h) - y[N:])) <= 1e-9


def test_rforecast_mssa_uses_one_lrr_for_all_series():
    """MSSA of cosines of one period and different amplitudes and phases: the
    common U gives one LRR that continues every series."""
    L, h = 24, 20
    lens = [80, 95, 110]
    amp, ph = [1.0, 0.5, 2.0], [0.0, 1.0, 2.5]
    full = [a * np.cos(2 * np.pi * np.arange(n + h) / 10 + p) for a, p, n in zip(amp, ph, lens)]
    ser = [f[:n] for f, n in zip(full, lens)]
    s, U, V = _lapack_svd(oracle.trajectory_mssa(ser, L))
    recs = oracle.reconstruct_mssa(lens, L, s, U, V, [0, 1])
    f = oracle.rforecast_column(recs, U, [0, 1], h)
    for p, n in enumerate(lens):
        assert np.max(np.abs(f[p] - full[p][n:])) <= 1e-9


# --------------------------------------------------------------------------
# vector (column) forecast
# --------------------------------------------------------------------------

def _rank_r_vforecast(x, L, group, h):
    sh = oracle.shapes(x, None, None, L)
    s, U, V = _lapack_svd(oracle.trajectory(x, sh))
    return oracle.vforecast_column([len(x)], L, s, U, V, group, h)[0]


def test_vforecast_continues_finite_rank_series():
    """Series of finite rank lie in their signal subspace: every lagged
    vector of the continuation is the true one, so the forecast is exact."""
    N, L, h = 90, 30, 25
    t = np.arange(N + h)
    x = 1.3 * np.cos(2 * np.pi * t / 12 + 0.4)
    assert np.max(np.abs(_rank_r_vforecast(x[:N], L, [0, 1], h) - x[N:])) <= 1e-9
    y = 0.97 ** t
    assert np.max(np.abs(_rank_r_vforecast(y[:N], L, [0], h) - y[N:])) <= 1e-10
    z = 2.0 + 0.1 * t
    assert np.max(np.abs(_rank_r_vforecast(z[:N], L, [0, 1], h) - z[N:])) <= 1e-9


def test_vforecast_mssa_continues_every_series():
    L, h = 24, 20
    lens = [80, 95, 110]
    amp, ph = [1.0, 0.5, 2.0], [0.0, 1.0, 2.5]
    full = [a * np.cos(2 * np.pi * np.arange(n + h) / 10 + p) for a, p, n in zip(amp, ph, lens)]
    ser = [f[:n] for f, n in zip(full, lens)]
    s, U, V = _lapack_svd(oracle.trajectory_mssa(ser, L))
    f = oracle.vforecast_column(lens, L, s, U, V, [0, 1], h)
    for p, n in enumerate(lens):
        assert np.max(np.abs(f[p] - full[p][n:])) <= 1e-9


def _noisy_case():
    g = np.random.default_rng(17)
    N, L = 140, 40
    t = np.arange(N)
    x = np.cos(2 * np.pi * t / 11) + 0.02 * t + 0.3 * g.standard_normal(N)
    sh = oracle.shapes(x, None, None, L)
    s, U, V = _lapack_svd(oracle.trajectory(x, sh))
    return x, L, s, U, V


def test_vforecast_does_not_redraw():
    """A longer horizon extends a shorter one without changing it (the
    number of new lagged vectors grows with the horizon for that reason)."""
    x, L, s, U, V = _noisy_case()
    a = oracle.vforecast_column([len(x)], L, s, U, V, [0, 1, 2], 10)
    b = oracle.vforecast_column([len(x)], L, s, U, V, [0, 1, 2], 17)
    assert np.max(np.abs(a - b[:, :10])) <= 1e-12


def test_vforecast_matches_the_shift_matrix_route():
    """The fast algorithm of the forecast implementation section carries the
    coefficient vectors W_k = D W_{k-1} with D the pseudo-inverse of the
    group's U without its last row times U without its first row; the
    forecast is then an anti-diagonal average of U W.  It must agree with
    the definition on a noisy series whose group is no exact signal."""
    x, L, s, U, V = _noisy_case()
    grp, h = [0, 1, 2], 15
    N = len(x)
    K = N - L + 1
    Ug = U[:, grp]
    D = np.linalg.lstsq(Ug[:-1], Ug[1:], rcond=None)[0]
    w = s[grp] * V[K - 1, grp]
    Ws = []
    for _ in range(h + L - 1):
        w = D @ w
        Ws.append(w)
    Ws = np.array(Ws)                            # row e: column K + e (0-based)
    fast = np.array([np.mean([Ug[i] @ Ws[L - 1 + t - i] for i in range(L)]) for t in range(h)])
    ref = oracle.vforecast_column([N], L, s, U, V, grp, h)[0]
    assert np.max(np.abs(fast - ref)) <= 1e-10 * np.max(np.abs(ref))


def test_vforecast_rejects_a_group_spanning_the_last_axis():
    L = 10
    U = np.eye(L)[:, :2]                     # e_1, e_2: fine
    V = np.eye(20)[:, :2]
    oracle.vforecast_column([L + 19], L, np.ones(2), U, V, [0, 1], 3)
    U2 = np.eye(L)[:, [0, L - 1]]            # e_L in the span: nu^2 = 1
    with pytest.raises(ValueError):
        oracle.vforecast_column([L + 19], L, np.ones(2), U2, V, [0, 1], 3)


# --------------------------------------------------------------------------
# row forecasts (recurrent and vector)
# --------------------------------------------------------------------------

def _noisy_system(lens=(70, 85, 60), L=20, seed=23):
    g = np.random.default_rng(seed)
    ser = [1.5 * np.cos(2 * np.pi * np.arange(n) / 9 + p) + 0.01 * np.arange(n)
           + 0.4 * g.standard_normal(n) for p, n in enumerate(lens)]
    s, U, V = _lapack_svd(oracle.trajectory_mssa(ser, L))
    return ser, list(lens), L, s, U, V


def test_row_forecasts_of_one_series_are_column_forecasts_of_the_transpose():
    """For one series the trajectory matrix with window K is the transpose
    of the one with window L: the row forecasts with window L are the column
    forecasts with window K (U and V swapped, same reconstruction)."""
    g = np.random.default_rng(5)
    N, L, h = 100, 30, 12
    x = np.sin(np.arange(N) / 4.0) + 0.3 * g.standard_normal(N)
    s, U, V = _lapack_svd(oracle.trajectory_mssa([x], L))
    grp = [0, 1, 2]
    rec = oracle.reconstruct_mssa([N], L, s, U, V, grp)
    K = N - L + 1
    a = oracle.rforecast_row(rec, L, V, grp, h)
    b = oracle.rforecast_column(rec, V, grp, h)
    assert np.max(np.abs(a - b)) <= 1e-10 * np.max(np.abs(b))
    c = oracle.vforecast_row([N], L, s, U, V, grp, h)
    d = oracle.vforecast_column([N], K, s, V, U, grp, h)
    assert np.max(np.abs(c - d)) <= 1e-10 * np.max(np.abs(d))


def test_row_forecasts_continue_a_finite_rank_system():
    L, h = 24, 20
    lens = [80, 95, 110]
    amp, ph = [1.0, 0.5, 2.0], [0.0, 1.0, 2.5]
    full = [a * np.cos(2 * np.pi * np.arange(n + h) / 10 + p) for a, p, n in zip(amp, ph, lens)]
    ser = [f[:n] for f, n in zip(full, lens)]
    s, U, V = _lapack_svd(oracle.trajectory_mssa(ser, L))
    recs = oracle.reconstruct_mssa(lens, L, s, U, V, [0, 1])
    fr = oracle.rforecast_row(recs, L, V, [0, 1], h)
    fv = oracle.vforecast_row(lens, L, s, U, V, [0, 1], h)
    for p, n in enumerate(lens):
        assert np.max(np.abs(fr[p] - full[p][n:])) <= 1e-9
        assert np.max(np.abs(fv[p] - full[p][n:])) <= 1e-9


def test_recurrent_row_forecast_is_the_least_squares_completion():
    """The next value of every series completes the next row of the
    trajectory matrix (known: each series' last K_p - 1 values; unknown: one
    value per series) to the vector closest to the group's row space."""
    ser, lens, L, s, U, V = _noisy_system()
    grp = [0, 1, 2, 3]
    recs = oracle.reconstruct_mssa(lens, L, s, U, V, grp)
    got = oracle.rforecast_row(recs, L, V, grp, 1)[:, 0]
    Vg = V[:, grp]
    Pc = np.eye(Vg.shape[0]) - Vg @ Vg.T
    ks = [n - L + 1 for n in lens]
    ends = np.cumsum(ks)
    unknown = ends - 1
    known = np.setdiff1d(np.arange(Vg.shape[0]), unknown)
    z = np.concatenate([r[len(r) - (k - 1):] for r, k in zip(recs, ks)])
    ref = np.linalg.lstsq(Pc[:, unknown], -Pc[:, known] @ z, rcond=None)[0]
    assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(np.abs(ref))


def test_vector_row_forecast_matches_the_shift_matrix_route():
    """Algorithm of the fast row forecast: W_i = D W_{i-1} with D the
    pseudo-inverse of V's blocks without their last coordinate times V's
    blocks without their first; forecast = block-wise anti-diagonal mean."""
    ser, lens, L, s, U, V = _noisy_system()
    grp, h = [0, 1, 2, 3], 9
    Vg = V[:, grp]
    ks = [n - L + 1 for n in lens]
    ends = np.cumsum(ks)
    starts = ends - ks
    lo = np.concatenate([Vg[b:e - 1] for b, e in zip(starts, ends)])
    hi = np.concatenate([Vg[b + 1:e] for b, e in zip(starts, ends)])
    D = np.linalg.lstsq(lo, hi, rcond=None)[0]
    w = s[grp] * U[L - 1, grp]
    Ws = []
    for _ in range(h + max(ks) - 1):
        w = D @ w
        Ws.append(w)
    Ws = np.array(Ws)                       # row e: trajectory row L + e (0-based)
    ref = oracle.vforecast_row(lens, L, s, U, V, grp, h)
    for p, (b, kp) in enumerate(zip(starts, ks)):
        fast = [np.mean([Vg[b + k] @ Ws[kp - 1 + m - k] for k in range(kp)]) for m in range(h)]
        assert np.max(np.abs(np.array(fast) - ref[p])) <= 1e-10 * np.max(np.abs(ref))


def test_vector_row_forecast_does_not_redraw():
    ser, lens, L, s, U, V = _noisy_system()
    a = oracle.vforecast_row(lens, L, s, U, V, [0, 1, 2], 6)
    b = oracle.vforecast_row(lens, L, s, U, V, [0, 1, 2], 11)
    assert np.max(np.abs(a - b[:, :6])) <= 1e-12 * np.max(np.abs(b))


def test_row_forecast_rejects_a_singular_system():
    L = 4
    lens = [L + 2, L + 2]                  # K_1 = K_2 = 3, K = 6
    V = np.zeros((6, 2))
    V[2, 0] = 1.0                          # V_1 = e_3: the last coordinate of block 1
    V[0, 1] = 1.0
    with pytest.raises(ValueError):
        oracle.lrr_row(lens, L, V, [0, 1])


# --------------------------------------------------------------------------
# M-2D-SSA packing
# --------------------------------------------------------------------------

def _m2d_images(seed=29):
    g = np.random.default_rng(seed)
    sizes = [(14, 11), (12, 15), (16, 9)]
    imgs = []
    for nx, ny in sizes:
        i, j = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
        imgs.append(np.cos(0.7 * i + 0.3 * j) + 0.5 * g.standard_normal((nx, ny)))
    return imgs


def test_m2d_packing_gives_the_stacked_trajectory_matrix():
    """The packed array's shaped trajectory matrix has the columns of
    [T(X_1) : ... : T(X_s)] (ordered differently): same Gram X X^T, same
    singular values."""
    imgs = _m2d_images()
    for window, wmask in (((4, 3), None), ((4, 4), np.array([[1, 1, 1, 1], [1, 0, 0, 1], [1, 0, 0, 1], [1, 1, 1, 1]]))):
        Xs = oracle.trajectory_m2d(imgs, window, wmask)
        packed = oracle.pack_m2d(imgs, window, wmask)
        Xp = oracle.trajectory(packed, oracle.shapes(packed, None, wmask, window))
        assert Xp.shape == Xs.shape
        np.testing.assert_allclose(Xp @ Xp.T, Xs @ Xs.T, rtol=0, atol=1e-10 * np.abs(Xs @ Xs.T).max())
        s1 = np.linalg.svd(Xs, compute_uv=False)
        s2 = np.linalg.svd(Xp, compute_uv=False)
        np.testing.assert_allclose(s1, s2, rtol=0, atol=1e-12 * s1[0])


def test_m2d_of_copies_scales_the_singular_values():
    """s copies of one image: X X^T grows s times, so sigma = sqrt(s) times
    the 2D-SSA singular values of the image."""
    img = _m2d_images()[0]
    s1 = np.linalg.svd(oracle.trajectory(img, oracle.shapes(img, None, None, (4, 3))), compute_uv=False)
    s3 = np.linalg.svd(oracle.trajectory_m2d([img, img, img], (4, 3)), compute_uv=False)
    np.testing.assert_allclose(s3[:len(s1)], np.sqrt(3.0) * s1, rtol=0, atol=1e-12 * s3[0])


# --------------------------------------------------------------------------
# LS-ESPRIT roots
# --------------------------------------------------------------------------

def _match_roots(a, b):
    """Largest distance after pairing each root of a with its nearest unused root of b."""
    b = list(b)
    worst = 0.0
    for z in a:
        k = int(np.argmin([abs(z - w) for w in b]))
        worst = max(worst, abs(z - b[k]))
        b.pop(k)
    return worst


def test_esprit_recovers_damped_cosines_and_exponentials():
    """A noiseless sum of a damped cosine, an undamped one and an
    exponential has rank 5; the roots of the five-component group are
    rho e^{+-i omega} of each cosine and the exponential's base."""
    N, L = 120, 40
    t = np.arange(N)
    x = 2.0 * 0.98 ** t * np.cos(2 * np.pi * t / 10 + 0.3) + np.cos(2 * np.pi * t / 23) + 0.5 * 1.01 ** t
    sh = oracle.shapes(x, None, None, L)
    s, U, V = _lapack_svd(oracle.trajectory(x, sh))
    z = oracle.esprit(U, [0, 1, 2, 3, 4])
    true = [0.98 * np.exp(2j * np.pi / 10), 0.98 * np.exp(-2j * np.pi / 10), np.exp(2j * np.pi / 23),
            np.exp(-2j * np.pi / 23), 1.01]
    assert _match_roots(z, true) <= 1e-9
    assert [abs(a) >= abs(b) - 1e-15 for a, b in zip(z, z[1:])] == [True] * 4


def test_esprit_roots_do_not_depend_on_the_basis_of_the_span():
    """The roots are the eigenvalues of the shift operator on the span: any
    other basis of the same span (here a rotation of the group's vectors)
    gives the same roots, a different span does not."""
    g = np.random.default_rng(9)
    N, L = 90, 30
    t = np.arange(N)
    x = np.cos(2 * np.pi * t / 7) + 0.7 * np.cos(2 * np.pi * t / 13 + 1) + 0.05 * g.standard_normal(N)
    sh = oracle.shapes(x, None, None, L)
    s, U, V = _lapack_svd(oracle.trajectory(x, sh))
    Q, _ = np.linalg.qr(g.standard_normal((4, 4)))
    U2 = U.copy()
    U2[:, :4] = U[:, :4] @ Q
    a, b = oracle.esprit(U, [0, 1, 2, 3]), oracle.esprit(U2, [0, 1, 2, 3])
    assert _match_roots(a, b) <= 1e-10
    periods = sorted(2 * np.pi / abs(np.angle(z)) for z in a if z.imag > 0)
    np.testing.assert_allclose(periods, [7.0, 13.0], rtol=2e-2)


def _pairs_match(l1, m1, l2, m2):
    """Largest distance after pairing each (lambda, mu) of one set with its nearest unused pair of the other."""
    b = list(zip(l2, m2))
    worst = 0.0
    for a in zip(l1, m1):
        d = [max(abs(a[0] - c[0]), abs(a[1] - c[1])) for c in b]
        k = int(np.argmin(d))
        worst = max(worst, d[k])
        b.pop(k)
    return worst


def test_esprit2d_recovers_planar_waves():
    """A noiseless sum of two planar cosines, one of them damped in both
    directions, has rank 4; the pairs of the group's joint eigenvalues are
    (rho e^{+-2 pi i f}, tau e^{+-2 pi i g}) of each term, also for a
    window with a hole."""
    nx, ny = 40, 36
    m, n = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    f1, g1, f2, g2 = 0.11, 0.07, 0.04, 0.19
    x = np.cos(2 * np.pi * (f1 * m + g1 * n) + 0.4) + 0.97 ** m * 0.99 ** n * 2 * np.cos(2 * np.pi * (f2 * m + g2 * n))
    true_l = [np.exp(2j * np.pi * f1), np.exp(-2j * np.pi * f1), 0.97 * np.exp(2j * np.pi * f2), 0.97 * np.exp(-2j * np.pi * f2)]
    true_m = [np.exp(2j * np.pi * g1), np.exp(-2j * np.pi * g1), 0.99 * np.exp(2j * np.pi * g2), 0.99 * np.exp(-2j * np.pi * g2)]
    wm = np.ones((8, 7), np.uint8)
    wm[3:5, 2:4] = 0
    for window, wmask in (((8, 7), None), ((8, 7), wm)):
        sh = oracle.shapes(x, None, wmask, window)
        s, U, V = _lapack_svd(oracle.trajectory(x, sh))
        lam, mu = oracle.esprit2d(sh, U, [0, 1, 2, 3])
        assert _pairs_match(lam, mu, true_l, true_m) <= 1e-9


def test_esprit2d_pairs_do_not_depend_on_the_combination_weight():
    """For a signal of finite rank the shift matrices commute, so any
    combination weight gives the same pairs."""
    nx, ny = 30, 30
    m, n = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    x = np.cos(2 * np.pi * (0.13 * m + 0.05 * n)) + 0.5 * np.cos(2 * np.pi * (0.03 * m - 0.21 * n) + 1.0)
    sh = oracle.shapes(x, None, None, (6, 6))
    s, U, V = _lapack_svd(oracle.trajectory(x, sh))
    a = oracle.esprit2d(sh, U, [0, 1, 2, 3])
    b = oracle.esprit2d(sh, U, [0, 1, 2, 3], gamma=2.3)
    assert _pairs_match(a[0], a[1], b[0], b[1]) <= 1e-9


def test_tls_esprit_recovers_damped_cosines_and_agrees_with_ls():
    """Noiseless finite-rank series: TLS-ESPRIT gives the exact roots, like
    LS-ESPRIT; on a noisy one both stay close to the true roots."""
    N, L = 120, 40
    t = np.arange(N)
    x = 2.0 * 0.98 ** t * np.cos(2 * np.pi * t / 10 + 0.3) + np.cos(2 * np.pi * t / 23) + 0.5 * 1.01 ** t
    true = [0.98 * np.exp(2j * np.pi / 10), 0.98 * np.exp(-2j * np.pi / 10), np.exp(2j * np.pi / 23),
            np.exp(-2j * np.pi / 23), 1.01]
    sh = oracle.shapes(x, None, None, L)
    s, U, V = _lapack_svd(oracle.trajectory(x, sh))
    assert _match_roots(oracle.esprit_tls(U, [0, 1, 2, 3, 4]), true) <= 1e-9
    g = np.random.default_rng(12)
    y = x + 0.05 * g.standard_normal(N)
    s, U, V = _lapack_svd(oracle.trajectory(y, oracle.shapes(y, None, None, L)))
    a, b = oracle.esprit_tls(U, [0, 1, 2, 3, 4]), oracle.esprit(U, [0, 1, 2, 3, 4])
    assert _match_roots(a, true) <= 2e-2 and _match_roots(b, true) <= 2e-2
    assert _match_roots(a, b) > 1e-12                  # the two estimators differ on noisy data


def test_tls_esprit_roots_do_not_depend_on_the_basis_of_the_span():
    g = np.random.default_rng(9)
    N, L = 90, 30
    t = np.arange(N)
    x = np.cos(2 * np.pi * t / 7) + 0.7 * np.cos(2 * np.pi * t / 13 + 1) + 0.05 * g.standard_normal(N)
    s, U, V = _lapack_svd(oracle.trajectory(x, oracle.shapes(x, None, None, L)))
    Q, _ = np.linalg.qr(g.standard_normal((4, 4)))
    U2 = U.copy()
    U2[:, :4] = U[:, :4] @ Q
    assert _match_roots(oracle.esprit_tls(U, [0, 1, 2, 3]), oracle.esprit_tls(U2, [0, 1, 2, 3])) <= 1e-10


# --------------------------------------------------------------------------
# Mosaic Hankel matrices
# --------------------------------------------------------------------------

def _mosaic_series(Ls, Ks, seed=7):
    g = np.random.default_rng(seed)
    return [[g.standard_normal(L + K - 1) for K in Ks] for L in Ls]


def test_mosaic_of_one_block_is_the_hankel_matrix():
    from scipy.linalg import hankel
    x = np.random.default_rng(2).standard_normal(20)
    M = oracle.mosaic_hankel([[x]], [6], [15])
    np.testing.assert_array_equal(M, hankel(x[:6], x[5:]))


def test_mosaic_reduces_to_mssa_and_its_transpose():
    """One block row is the MSSA trajectory matrix with window L_1; one
    block column is the transposed MSSA matrix of its series with window
    K_1."""
    row = _mosaic_series([7], [5, 9, 4])
    np.testing.assert_array_equal(oracle.mosaic_hankel(row, [7], [5, 9, 4]),
                                  oracle.trajectory_mssa(row[0], 7))
    col = _mosaic_series([3, 8, 5], [6])
    np.testing.assert_array_equal(oracle.mosaic_hankel(col, [3, 8, 5], [6]),
                                  oracle.trajectory_mssa([c[0] for c in col], 6).T)


@pytest.mark.parametrize("Ls,Ks", [([5, 3, 7], [9, 4]), ([4], [6, 3]), ([2, 6], [7]), ([1, 4], [3, 1, 5])])
def test_mosaic_packing_gives_the_mosaic_matrix(Ls, Ks):
    """The shaped trajectory matrix of the packing is the mosaic matrix,
    its rows in the window's lexicographic cell order (down the window's
    columns) and its columns block after block."""
    ser = _mosaic_series(Ls, Ks)
    M = oracle.mosaic_hankel(ser, Ls, Ks)
    x, window, wmask = oracle.pack_mosaic(ser, Ls, Ks)
    sh = oracle.shapes(x, None, wmask, window)
    X = oracle.trajectory(x, sh)
    r0 = np.concatenate([[0], np.cumsum(Ls)[:-1]])
    rows = r0[sh.li] + sh.lj
    assert sorted(rows) == list(range(sum(Ls)))
    np.testing.assert_array_equal(X, M[rows])


def test_mosaic_reconstruction_is_exact_for_a_rank_two_mosaic_and_complete():
    """Series (i, j) = a_i b_j cos(w n + p_i + q_j): entry (b, k) of block
    (i, j) is the real part of (a_i e^{i(w b + p_i)}) (b_j e^{i(w k + q_j)}),
    so the whole mosaic matrix has rank 2 and the first two components
    reconstruct every series exactly; and the reconstructions of all
    components sum to the input."""
    Ls, Ks = [5, 8, 3], [6, 10]
    g = np.random.default_rng(5)
    a, p = g.uniform(0.5, 2, len(Ls)), g.uniform(0, 6, len(Ls))
    b, q = g.uniform(0.5, 2, len(Ks)), g.uniform(0, 6, len(Ks))
    ser = [[a[i] * b[j] * np.cos(0.7 * np.arange(L + K - 1) + p[i] + q[j]) for j, K in enumerate(Ks)]
           for i, L in enumerate(Ls)]
    assert np.linalg.matrix_rank(oracle.mosaic_hankel(ser, Ls, Ks), tol=1e-9) == 2
    rec = oracle.reconstruct_mosaic(ser, Ls, Ks, [0, 1])
    for i in range(len(Ls)):
        for j in range(len(Ks)):
            np.testing.assert_allclose(rec[i][j], ser[i][j], rtol=0, atol=1e-12)
    noisy = _mosaic_series(Ls, Ks, seed=9)
    n = min(sum(Ls), sum(Ks))
    parts = [oracle.reconstruct_mosaic(noisy, Ls, Ks, [k]) for k in range(n)]
    for i in range(len(Ls)):
        for j in range(len(Ks)):
            np.testing.assert_allclose(sum(p[i][j] for p in parts), noisy[i][j], rtol=0, atol=1e-12)
