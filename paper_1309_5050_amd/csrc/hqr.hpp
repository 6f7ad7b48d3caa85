// Eigenvalues of a small real non-symmetric matrix: Householder reduction to
// upper Hessenberg form, then the implicit double-shift QR iteration of
// Francis on the active window with deflation at negligible subdiagonal
// entries (the classical algorithm, Golub and Van Loan, Matrix Computations,
// Algorithms 7.4.2 and 7.5.1/7.5.2, written here for eigenvalues only).
// Sequential code for one thread: the matrices it serves (the shift matrix
// of a component group) have at most 64 rows.
#pragma once

#include <cmath>

namespace shssa {

// a: n x n row-major with leading dimension lda, overwritten.  work: n
// values.  wr, wi: the eigenvalues (a complex pair as re +- i im, the one
// with positive imaginary part first).  Returns 0, or -1 if an eigenvalue
// took more than 60 iterations.
template <typename Real>
__host__ __device__ inline int eig_real(Real* a, int n, int lda, Real* work, Real* wr, Real* wi) {
    const auto A = [&](int i, int j) -> Real& { return a[i * lda + j]; };
    // Hessenberg: reflection k zeroes column k below its subdiagonal
    for (int k = 0; k + 2 < n; ++k) {
        Real s2 = 0;
        for (int i = k + 1; i < n; ++i) s2 += A(i, k) * A(i, k);
        if (s2 == 0) continue;
        const Real x0 = A(k + 1, k);
        const Real alpha = -std::copysign(std::sqrt(s2), x0);
        const Real v0 = x0 - alpha;
        const Real vv = s2 - x0 * x0 + v0 * v0;
        if (vv == 0) continue;
        work[k + 1] = v0;
        for (int i = k + 2; i < n; ++i) work[i] = A(i, k);
        for (int j = k; j < n; ++j) {
            Real t = 0;
            for (int i = k + 1; i < n; ++i) t += work[i] * A(i, j);
            t *= 2 / vv;
            for (int i = k + 1; i < n; ++i) A(i, j) -= t * work[i];
        }
        for (int i = 0; i < n; ++i) {
            Real t = 0;
            for (int j = k + 1; j < n; ++j) t += A(i, j) * work[j];
            t *= 2 / vv;
            for (int j = k + 1; j < n; ++j) A(i, j) -= t * work[j];
        }
        A(k + 1, k) = alpha;
        for (int i = k + 2; i < n; ++i) A(i, k) = 0;
    }
    Real anorm = 0;
    for (int i = 0; i < n; ++i)
        for (int j = (i > 0 ? i - 1 : 0); j < n; ++j) anorm += std::fabs(A(i, j));
    const Real eps = sizeof(Real) == 8 ? Real(2.220446049250313e-16) : Real(1.1920929e-7);
    int hi = n - 1, its = 0;
    while (hi >= 0) {
        int l = hi;
        for (; l > 0; --l) {
            Real s = std::fabs(A(l - 1, l - 1)) + std::fabs(A(l, l));
            if (s == 0) s = anorm;
            if (std::fabs(A(l, l - 1)) <= eps * s) {
                A(l, l - 1) = 0;
                break;
            }
        }
        if (l == hi) {   // a 1 x 1 block
            wr[hi] = A(hi, hi);
            wi[hi] = 0;
            --hi;
            its = 0;
            continue;
        }
        if (l == hi - 1) {   // a 2 x 2 block [p q; r s]
            const Real p = A(hi - 1, hi - 1), q = A(hi - 1, hi), r = A(hi, hi - 1), s = A(hi, hi);
            const Real h = Real(0.5) * (p - s), disc = h * h + q * r;
            if (disc >= 0) {
                const Real z = h + std::copysign(std::sqrt(disc), h);
                wr[hi - 1] = s + z;
                wr[hi] = z != 0 ? s - q * r / z : s + z;
                wi[hi - 1] = wi[hi] = 0;
            } else {
                const Real im = std::sqrt(-disc);
                wr[hi - 1] = wr[hi] = s + h;
                wi[hi - 1] = im;
                wi[hi] = -im;
            }
            hi -= 2;
            its = 0;
            continue;
        }
        if (++its > 60) return -1;
        // shifts: the eigenvalues of the trailing 2 x 2 block, through its
        // trace and determinant; every 10th iteration an exceptional shift
        // built from the last subdiagonal entries breaks cycles
        Real tr, dt;
        if (its % 10 == 0) {
            const Real w = std::fabs(A(hi, hi - 1)) + std::fabs(A(hi - 1, hi - 2));
            tr = 2 * A(hi, hi) + Real(1.5) * w;
            dt = A(hi, hi) * A(hi, hi) + Real(1.5) * w * A(hi, hi) + w * w;
        } else {
            tr = A(hi - 1, hi - 1) + A(hi, hi);
            dt = A(hi - 1, hi - 1) * A(hi, hi) - A(hi - 1, hi) * A(hi, hi - 1);
        }
        // first column of H^2 - tr H + dt I
        Real x = A(l, l) * A(l, l) + A(l, l + 1) * A(l + 1, l) - tr * A(l, l) + dt;
        Real y = A(l + 1, l) * (A(l, l) + A(l + 1, l + 1) - tr);
        Real z = A(l + 1, l) * A(l + 2, l + 1);
        for (int k = l; k <= hi - 2; ++k) {
            const Real nrm = std::sqrt(x * x + y * y + z * z);
            if (nrm != 0) {
                const Real alpha = -std::copysign(nrm, x);
                const Real v0 = x - alpha, v1 = y, v2 = z;
                const Real vv = v0 * v0 + v1 * v1 + v2 * v2;
                if (vv != 0) {
                    const Real f = 2 / vv;
                    for (int j = (k - 1 > l ? k - 1 : l); j <= hi; ++j) {
                        const Real t = f * (v0 * A(k, j) + v1 * A(k + 1, j) + v2 * A(k + 2, j));
                        A(k, j) -= t * v0;
                        A(k + 1, j) -= t * v1;
                        A(k + 2, j) -= t * v2;
                    }
                    const int imax = k + 3 < hi ? k + 3 : hi;
                    for (int i = l; i <= imax; ++i) {
                        const Real t = f * (A(i, k) * v0 + A(i, k + 1) * v1 + A(i, k + 2) * v2);
                        A(i, k) -= t * v0;
                        A(i, k + 1) -= t * v1;
                        A(i, k + 2) -= t * v2;
                    }
                }
            }
            x = A(k + 1, k);
            y = A(k + 2, k);
            if (k < hi - 2) z = A(k + 3, k);
        }
        // the last reflection acts on two rows
        const Real nrm = std::sqrt(x * x + y * y);
        if (nrm != 0) {
            const Real alpha = -std::copysign(nrm, x);
            const Real v0 = x - alpha, v1 = y;
            const Real vv = v0 * v0 + v1 * v1;
            if (vv != 0) {
                const Real f = 2 / vv;
                const int k = hi - 1;
                for (int j = (k - 1 > l ? k - 1 : l); j <= hi; ++j) {
                    const Real t = f * (v0 * A(k, j) + v1 * A(k + 1, j));
                    A(k, j) -= t * v0;
                    A(k + 1, j) -= t * v1;
                }
                for (int i = l; i <= hi; ++i) {
                    const Real t = f * (A(i, k) * v0 + A(i, k + 1) * v1);
                    A(i, k) -= t * v0;
                    A(i, k + 1) -= t * v1;
                }
            }
        }
    }
    return 0;
}

// Joint eigenvalues of two real n x n matrices px and py (row-major,
// leading dimension ld) that commute up to noise, as a joint
// diagonalisation: with C = px + gamma py = T diag(z) T^-1, lambda_k =
// (T^-1 px T)_kk and mu_k = (T^-1 py T)_kk.  Column k of T is a right
// eigenvector t_k of C and row k of T^-1 a left eigenvector w_k (C^T w_k =
// z_k w_k) scaled to w_k^T t_k = 1, so lambda_k = w_k^T px t_k / w_k^T t_k.
// Both come from two steps of inverse iteration at each eigenvalue of C
// (complex Gaussian elimination with partial pivoting on C - z I and on
// C^T - z I; the shift is moved off the eigenvalue by a rounding-level
// amount so that the systems stay solvable).  Scratch: c (n * ld), work
// (n), piv (n), lu (2 n n), v, y and t (2 n each).  Returns 0, or -1 if C's
// eigenvalue iteration failed.
template <typename Real>
__host__ __device__ inline int joint_eig(const Real* px, const Real* py, int n, int ld, Real gamma, Real* c,
                                         Real* work, int* piv, Real* lu, Real* v, Real* y, Real* t, Real* wr,
                                         Real* wi, Real* lre, Real* lim, Real* mre, Real* mim) {
    Real cnorm = 0;
    for (int i = 0; i < n; ++i) {
        Real rs = 0;
        for (int j = 0; j < n; ++j) {
            c[i * ld + j] = px[i * ld + j] + gamma * py[i * ld + j];
            rs += std::fabs(c[i * ld + j]);
        }
        cnorm = rs > cnorm ? rs : cnorm;
    }
    if (eig_real(c, n, ld, work, wr, wi) != 0) return -1;
    const Real eps = sizeof(Real) == 8 ? Real(2.220446049250313e-16) : Real(1.1920929e-7);
    const Real tiny = (cnorm > 0 ? cnorm : Real(1)) * eps;
    const auto LR = [&](int i, int j) -> Real& { return lu[2 * (i * n + j)]; };
    const auto LI = [&](int i, int j) -> Real& { return lu[2 * (i * n + j) + 1]; };
    const auto C = [&](int i, int j) -> Real { return px[i * ld + j] + gamma * py[i * ld + j]; };
    // v <- unit vector in the null direction of (C or C^T) - (zr + i zi) I
    const auto inverse_iteration = [&](bool transposed, Real zr, Real zi) {
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                LR(i, j) = (transposed ? C(j, i) : C(i, j)) - (i == j ? zr : Real(0));
                LI(i, j) = i == j ? -zi : Real(0);
            }
        for (int p = 0; p < n; ++p) {
            int best = p;
            Real bm = -1;
            for (int i = p; i < n; ++i) {
                const Real m = std::fabs(LR(i, p)) + std::fabs(LI(i, p));
                if (m > bm) {
                    bm = m;
                    best = i;
                }
            }
            piv[p] = best;
            if (best != p)
                for (int j = 0; j < n; ++j) {
                    const Real tr = LR(p, j), ti = LI(p, j);
                    LR(p, j) = LR(best, j);
                    LI(p, j) = LI(best, j);
                    LR(best, j) = tr;
                    LI(best, j) = ti;
                }
            if (std::fabs(LR(p, p)) + std::fabs(LI(p, p)) == 0) LR(p, p) = tiny;
            const Real dr = LR(p, p), di = LI(p, p), dd = dr * dr + di * di;
            for (int i = p + 1; i < n; ++i) {
                const Real fr = (LR(i, p) * dr + LI(i, p) * di) / dd;
                const Real fi = (LI(i, p) * dr - LR(i, p) * di) / dd;
                LR(i, p) = fr;
                LI(i, p) = fi;
                for (int j = p + 1; j < n; ++j) {
                    LR(i, j) -= fr * LR(p, j) - fi * LI(p, j);
                    LI(i, j) -= fr * LI(p, j) + fi * LR(p, j);
                }
            }
        }
        for (int i = 0; i < n; ++i) {
            v[2 * i] = 1;
            v[2 * i + 1] = 0;
        }
        for (int it = 0; it < 2; ++it) {
            for (int i = 0; i < 2 * n; ++i) y[i] = v[i];
            for (int p = 0; p < n; ++p)
                if (piv[p] != p) {
                    const int q = piv[p];
                    const Real tr = y[2 * p], ti = y[2 * p + 1];
                    y[2 * p] = y[2 * q];
                    y[2 * p + 1] = y[2 * q + 1];
                    y[2 * q] = tr;
                    y[2 * q + 1] = ti;
                }
            for (int i = 1; i < n; ++i)
                for (int j = 0; j < i; ++j) {
                    y[2 * i] -= LR(i, j) * y[2 * j] - LI(i, j) * y[2 * j + 1];
                    y[2 * i + 1] -= LR(i, j) * y[2 * j + 1] + LI(i, j) * y[2 * j];
                }
            for (int i = n - 1; i >= 0; --i) {
                Real sr = y[2 * i], si = y[2 * i + 1];
                for (int j = i + 1; j < n; ++j) {
                    sr -= LR(i, j) * y[2 * j] - LI(i, j) * y[2 * j + 1];
                    si -= LR(i, j) * y[2 * j + 1] + LI(i, j) * y[2 * j];
                }
                const Real dr = LR(i, i), di = LI(i, i), dd = dr * dr + di * di;
                y[2 * i] = (sr * dr + si * di) / dd;
                y[2 * i + 1] = (si * dr - sr * di) / dd;
            }
            Real mx = 0;
            for (int i = 0; i < 2 * n; ++i) mx = std::fabs(y[i]) > mx ? std::fabs(y[i]) : mx;
            if (mx == 0) mx = 1;
            Real nn = 0;
            for (int i = 0; i < 2 * n; ++i) {
                v[i] = y[i] / mx;
                nn += v[i] * v[i];
            }
            nn = std::sqrt(nn);
            for (int i = 0; i < 2 * n; ++i) v[i] /= nn;
        }
    };
    for (int k = 0; k < n; ++k) {
        inverse_iteration(false, wr[k] + tiny, wi[k]);
        for (int i = 0; i < 2 * n; ++i) t[i] = v[i];
        inverse_iteration(true, wr[k] + tiny, wi[k]);   // v = w_k
        // w^T t, w^T px t and w^T py t (no conjugation: rows of T^-1)
        Real sr = 0, si = 0, ar = 0, ai = 0, br = 0, bi = 0;
        for (int i = 0; i < n; ++i) {
            Real xr = 0, xi = 0, qr = 0, qi = 0;
            for (int j = 0; j < n; ++j) {
                xr += px[i * ld + j] * t[2 * j];
                xi += px[i * ld + j] * t[2 * j + 1];
                qr += py[i * ld + j] * t[2 * j];
                qi += py[i * ld + j] * t[2 * j + 1];
            }
            const Real wr_ = v[2 * i], wi_ = v[2 * i + 1];
            sr += wr_ * t[2 * i] - wi_ * t[2 * i + 1];
            si += wr_ * t[2 * i + 1] + wi_ * t[2 * i];
            ar += wr_ * xr - wi_ * xi;
            ai += wr_ * xi + wi_ * xr;
            br += wr_ * qr - wi_ * qi;
            bi += wr_ * qi + wi_ * qr;
        }
        const Real dd = sr * sr + si * si;
        lre[k] = (ar * sr + ai * si) / dd;
        lim[k] = (ai * sr - ar * si) / dd;
        mre[k] = (br * sr + bi * si) / dd;
        mim[k] = (bi * sr - br * si) / dd;
    }
    return 0;
}

// Eigenpairs of a symmetric n x n matrix (row-major, leading dimension lda,
// overwritten) by the cyclic Jacobi method: rotations zero each
// off-diagonal entry in turn until the off-diagonal mass falls below
// rounding.  vec (n x n, leading dimension ldv) receives the eigenvectors as
// columns, w the eigenvalues.  Returns the sweeps used, or -1 if 60 did not
// suffice.
template <typename Real>
__host__ __device__ inline int sym_eig(Real* a, int n, int lda, Real* vec, int ldv, Real* w) {
    const auto A = [&](int i, int j) -> Real& { return a[i * lda + j]; };
    const auto Vv = [&](int i, int j) -> Real& { return vec[i * ldv + j]; };
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Vv(i, j) = i == j ? Real(1) : Real(0);
    const Real eps = sizeof(Real) == 8 ? Real(2.220446049250313e-16) : Real(1.1920929e-7);
    Real nrm = 0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) nrm += A(i, j) * A(i, j);
    int sweep = 0;
    for (; sweep < 60; ++sweep) {
        Real off = 0;
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) off += A(i, j) * A(i, j);
        if (off <= eps * eps * nrm) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                const Real apq = A(p, q);
                if (apq == 0) continue;
                const Real th = (A(q, q) - A(p, p)) / (2 * apq);
                const Real t = std::copysign(Real(1), th) / (std::fabs(th) + std::sqrt(th * th + 1));
                const Real c = 1 / std::sqrt(t * t + 1), sn = t * c;
                for (int k = 0; k < n; ++k) {   // columns p, q
                    const Real akp = A(k, p), akq = A(k, q);
                    A(k, p) = c * akp - sn * akq;
                    A(k, q) = sn * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {   // rows p, q
                    const Real apk = A(p, k), aqk = A(q, k);
                    A(p, k) = c * apk - sn * aqk;
                    A(q, k) = sn * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    const Real vkp = Vv(k, p), vkq = Vv(k, q);
                    Vv(k, p) = c * vkp - sn * vkq;
                    Vv(k, q) = sn * vkp + c * vkq;
                }
            }
    }
    for (int i = 0; i < n; ++i) w[i] = A(i, i);
    return sweep < 60 ? sweep : -1;
}

// TLS-ESPRIT shift matrix of r components from the Gram matrix
// g = Z^T Z (2r x 2r, row-major, leading dimension 2r, overwritten) of
// Z = [U_low : U_high]: with the eigenvectors of g ordered by decreasing
// eigenvalue (the right singular vectors of Z), V = [[V11, V12], [V21, V22]],
// phi = -V12 V22^{-1} (r x r, row-major, leading dimension r).  Scratch:
// vec (4 r^2), w and order (2r each), lu (2 r^2: V22^T and the right-hand
// sides).  Returns 0, or -1 (no convergence) / -2 (V22 singular).
template <typename Real>
__host__ __device__ inline int tls_shift(Real* g, int r, Real* vec, Real* w, int* order, Real* lu, Real* phi) {
    const int n = 2 * r;
    if (sym_eig(g, n, n, vec, n, w) < 0) return -1;
    for (int i = 0; i < n; ++i) order[i] = i;
    for (int i = 1; i < n; ++i) {   // insertion sort by decreasing eigenvalue
        const int o = order[i];
        int k = i - 1;
        while (k >= 0 && w[order[k]] < w[o]) {
            order[k + 1] = order[k];
            --k;
        }
        order[k + 1] = o;
    }
    // solve V22^T X^T = -V12^T by Gauss-Jordan with partial pivoting:
    // M = [V22^T | -V12^T], V12(i, j) = vec(i, order[r + j]), V22(i, j) = vec(r + i, order[r + j])
    Real* m = lu;   // r x 2r
    for (int i = 0; i < r; ++i)
        for (int j = 0; j < r; ++j) {
            m[i * n + j] = vec[(r + j) * n + order[r + i]];   // V22^T(i, j) = V22(j, i)
            m[i * n + r + j] = -vec[j * n + order[r + i]];    // -V12^T(i, j) = -V12(j, i)
        }
    for (int p = 0; p < r; ++p) {
        int best = p;
        for (int i = p + 1; i < r; ++i)
            if (std::fabs(m[i * n + p]) > std::fabs(m[best * n + p])) best = i;
        if (m[best * n + p] == 0) return -2;
        if (best != p)
            for (int j = 0; j < n; ++j) {
                const Real t = m[p * n + j];
                m[p * n + j] = m[best * n + j];
                m[best * n + j] = t;
            }
        const Real piv = m[p * n + p];
        for (int j = 0; j < n; ++j) m[p * n + j] /= piv;
        for (int i = 0; i < r; ++i) {
            if (i == p) continue;
            const Real f = m[i * n + p];
            if (f == 0) continue;
            for (int j = 0; j < n; ++j) m[i * n + j] -= f * m[p * n + j];
        }
    }
    // X^T = right half; phi = X
    for (int i = 0; i < r; ++i)
        for (int j = 0; j < r; ++j) phi[i * r + j] = m[j * n + r + i];
    return 0;
}

}  // namespace shssa
