"""Shared helpers of the GPU parity tests (comparison rules, not arithmetic
of the method)."""
import numpy as np

TOL = {"fp64": 1e-10, "fp32": 1e-5}


def stable_groups(s_ref, r, rel_gap=1e-3):
    """Clusters of the leading r singular values that are separated from the
    rest of the spectrum by at least rel_gap * sigma_1; returns a list of
    (group indices, gap).  Values closer than that inside a cluster are
    grouped, so only spans that are determined are compared."""
    s = np.asarray(s_ref)
    thr = rel_gap * s[0]
    groups, cur = [], [0]
    for i in range(1, len(s)):
        if s[i - 1] - s[i] < thr:
            cur.append(i)
        else:
            groups.append(cur)
            cur = [i]
    groups.append(cur)
    out = []
    for g in groups:
        if g[-1] >= r:
            break
        lo = s[g[0] - 1] - s[g[0]] if g[0] > 0 else np.inf
        hi = s[g[-1]] - s[g[-1] + 1] if g[-1] + 1 < len(s) else np.inf
        out.append((g, min(lo, hi)))
    return out


def proj_dist(A, B):
    """Spectral norm of the difference of the orthogonal projectors onto the
    column spans of A and B (both with orthonormal columns)."""
    # equal dimensions: ||P - Q||_2 = sine of the largest principal angle
    A = A / np.linalg.norm(A, axis=0)
    B = B / np.linalg.norm(B, axis=0)
    qa, _ = np.linalg.qr(A)
    qb, _ = np.linalg.qr(B)
    # sin of the largest angle = |(I - Qa Qa^T) Qb|_2, accurate for small angles
    R = qb - qa @ (qa.T @ qb)
    return float(np.linalg.norm(R, 2))


def sigma_err(s, s_ref):
    s = np.asarray(s)
    return float(np.max(np.abs(s - s_ref[:len(s)])) / s_ref[0])
