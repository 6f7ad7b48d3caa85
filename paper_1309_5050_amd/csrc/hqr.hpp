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

}  // namespace shssa
