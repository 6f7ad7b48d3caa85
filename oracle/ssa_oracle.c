/*
 * Reference oracle for Shaped 2D-SSA (test infrastructure only).
 *
 * This file is the plain, slow, obviously correct statement of what the
 * method computes.  It is used by the test-suite, by the smoke check and by
 * the CPU-baseline timing; no product code links or calls it.  It shares no
 * code with the GPU path.
 *
 * Everything is double precision and 0-based.  An image is an nx-by-ny
 * row-major array (x is the row axis, y the column axis, as in the 2D-SSA
 * section of the paper).  An index set is a pair of int arrays (row, col).
 *
 * What follows the paper, step by step:
 *   - the shaped array N = mask AND not-NaN (Shaped 2D-SSA, package section);
 *   - the window shape L and its lexicographic order, which is the order of
 *     the vectorised array, i.e. column-major: row index fastest (Shaped
 *     2D-SSA, construction of the trajectory matrix);
 *   - the origin set K = { k : L (+) {k} subset of N } by brute force
 *     (equation sh_Ks), with (+) the shifted sum, which is a plain sum for
 *     0-based indices;
 *   - the quasi-Hankel trajectory matrix X_ij = x(l_i + k_j) (equation
 *     qh_mat), and the stacked Hankel MSSA matrix (equation mssa_embedding);
 *   - the SVD step (Section 2.1, Step 2), by one-sided Jacobi on the
 *     explicit matrix, or by the eigen-decomposition of S = X X^T with
 *     V_j = X^T U_j / sqrt(lambda_j), which is the paper's own definition;
 *   - reconstruction (Section 2.1, Step 4): the average of the entries of
 *     the grouped matrix over each set A_k, by explicit summation; the
 *     weights w_k = |A_k| are the counts.
 *
 * Parity unpinned: nothing in this file is unpinned; the pins live in the
 * oracle tests.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Shapes                                                                   */
/* ------------------------------------------------------------------------ */

/* N = mask AND not-NaN.  mask may be NULL (all cells). */
void orc_nset(int nx, int ny, const double *x, const uint8_t *mask, uint8_t *nset)
{
    for (long i = 0; i < (long)nx * ny; ++i)
        nset[i] = (uint8_t)((mask == NULL || mask[i] != 0) && !isnan(x[i]));
}

/* Window shape from an lx-by-ly 0/1 mask (NULL = the full box), trimmed to
 * its bounding box and listed in column-major (row-fastest) order.
 * Outputs: li/lj (capacity lx*ly), *nl, and the trimmed box *lxt, *lyt.
 * Returns 0, or -1 if the window is empty. */
int orc_window(int lx, int ly, const uint8_t *wmask, int *li, int *lj, int *nl,
               int *lxt, int *lyt)
{
    int i0 = lx, i1 = -1, j0 = ly, j1 = -1;
    for (int i = 0; i < lx; ++i)
        for (int j = 0; j < ly; ++j)
            if (wmask == NULL || wmask[(long)i * ly + j]) {
                if (i < i0) i0 = i;
                if (i > i1) i1 = i;
                if (j < j0) j0 = j;
                if (j > j1) j1 = j;
            }
    if (i1 < 0) { *nl = 0; return -1; }
    int n = 0;
    for (int j = j0; j <= j1; ++j)          /* column-major: i fastest */
        for (int i = i0; i <= i1; ++i)
            if (wmask == NULL || wmask[(long)i * ly + j]) {
                li[n] = i - i0;
                lj[n] = j - j0;
                ++n;
            }
    *nl = n;
    *lxt = i1 - i0 + 1;
    *lyt = j1 - j0 + 1;
    return 0;
}

/* K = { k : l + k in N for every l in L }, by checking every window cell at
 * every origin of the image.  Column-major order.  Capacity of ki/kj must be
 * (nx-lxt+1)*(ny-lyt+1). */
void orc_kset(int nx, int ny, const uint8_t *nset, int nl, const int *li, const int *lj,
              int lxt, int lyt, int *ki, int *kj, long *nk)
{
    int kx = nx - lxt + 1, ky = ny - lyt + 1;
    long n = 0;
    if (kx <= 0 || ky <= 0) { *nk = 0; return; }
    uint8_t *ok = (uint8_t *)malloc((size_t)kx * ky);
    #pragma omp parallel for schedule(dynamic, 4)
    for (int b = 0; b < ky; ++b)
        for (int a = 0; a < kx; ++a) {
            int good = 1;
            for (int t = 0; t < nl && good; ++t)
                good = nset[(long)(li[t] + a) * ny + (lj[t] + b)] != 0;
            ok[(long)b * kx + a] = (uint8_t)good;
        }
    for (int b = 0; b < ky; ++b)
        for (int a = 0; a < kx; ++a)
            if (ok[(long)b * kx + a]) { ki[n] = a; kj[n] = b; ++n; }
    free(ok);
    *nk = n;
}

/* w_alpha = |A_alpha| = number of trajectory-matrix entries holding x_alpha:
 * count every pair (l_i, k_j). */
void orc_weights(int nx, int ny, int nl, const int *li, const int *lj,
                 long nk, const int *ki, const int *kj, double *w)
{
    memset(w, 0, sizeof(double) * (size_t)nx * ny);
    for (int i = 0; i < nl; ++i)
        for (long j = 0; j < nk; ++j)
            w[(long)(li[i] + ki[j]) * ny + (lj[i] + kj[j])] += 1.0;
}

/* ------------------------------------------------------------------------ */
/* Trajectory matrices                                                       */
/* ------------------------------------------------------------------------ */

/* Quasi-Hankel X (L x K, row-major): X[i][j] = x(l_i + k_j). */
void orc_trajectory(int nx, int ny, const double *x, int nl, const int *li, const int *lj,
                    long nk, const int *ki, const int *kj, double *X)
{
    (void)nx;
    #pragma omp parallel for
    for (int i = 0; i < nl; ++i)
        for (long j = 0; j < nk; ++j)
            X[(long)i * nk + j] = x[(long)(li[i] + ki[j]) * ny + (lj[i] + kj[j])];
}

/* Stacked Hankel MSSA matrix [T(x1) : ... : T(xs)] (L x sum K_p, row-major),
 * T(x)_{ij} = x_{i+j} with K_p = N_p - L + 1.  series is the concatenation
 * of the s series. */
void orc_trajectory_mssa(int s, const int *lens, const double *series, int L, double *X)
{
    long K = 0, off = 0;
    for (int p = 0; p < s; ++p) K += lens[p] - L + 1;
    long col = 0;
    for (int p = 0; p < s; ++p) {
        int Kp = lens[p] - L + 1;
        for (int i = 0; i < L; ++i)
            for (int j = 0; j < Kp; ++j)
                X[(long)i * K + col + j] = series[off + i + j];
        col += Kp;
        off += lens[p];
    }
}

/* Explicit products without forming X:  u = X v,  v = X^T u. */
void orc_matvec(int nx, int ny, const double *x, int nl, const int *li, const int *lj,
                long nk, const int *ki, const int *kj, const double *v, double *u)
{
    (void)nx;
    #pragma omp parallel for
    for (int i = 0; i < nl; ++i) {
        double acc = 0.0;
        for (long j = 0; j < nk; ++j)
            acc += x[(long)(li[i] + ki[j]) * ny + (lj[i] + kj[j])] * v[j];
        u[i] = acc;
    }
}

void orc_rmatvec(int nx, int ny, const double *x, int nl, const int *li, const int *lj,
                 long nk, const int *ki, const int *kj, const double *u, double *v)
{
    (void)nx;
    #pragma omp parallel for
    for (long j = 0; j < nk; ++j) {
        double acc = 0.0;
        for (int i = 0; i < nl; ++i)
            acc += x[(long)(li[i] + ki[j]) * ny + (lj[i] + kj[j])] * u[i];
        v[j] = acc;
    }
}

/* ------------------------------------------------------------------------ */
/* SVD                                                                      */
/* ------------------------------------------------------------------------ */

static double dot(const double *a, const double *b, long n)
{
    double s = 0.0;
    for (long i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* Sort triplets by descending sigma and fix signs so that the entry of
 * largest magnitude of each U column is positive (lowest index on ties).
 * U is m x d column-major (column k at U + k*m), V is n x d column-major. */
static void sort_and_sign(long m, long n, int d, double *sig, double *U, double *V)
{
    int *perm = (int *)malloc(sizeof(int) * d);
    for (int k = 0; k < d; ++k) perm[k] = k;
    for (int a = 1; a < d; ++a) {                 /* insertion sort, stable */
        int p = perm[a], b = a - 1;
        while (b >= 0 && sig[perm[b]] < sig[p]) { perm[b + 1] = perm[b]; --b; }
        perm[b + 1] = p;
    }
    double *s2 = (double *)malloc(sizeof(double) * d);
    double *U2 = (double *)malloc(sizeof(double) * m * d);
    double *V2 = (double *)malloc(sizeof(double) * n * d);
    for (int k = 0; k < d; ++k) {
        int p = perm[k];
        s2[k] = sig[p];
        memcpy(U2 + (long)k * m, U + (long)p * m, sizeof(double) * m);
        memcpy(V2 + (long)k * n, V + (long)p * n, sizeof(double) * n);
        long arg = 0;
        double best = -1.0;
        for (long i = 0; i < m; ++i)
            if (fabs(U2[(long)k * m + i]) > best) { best = fabs(U2[(long)k * m + i]); arg = i; }
        if (U2[(long)k * m + arg] < 0) {
            for (long i = 0; i < m; ++i) U2[(long)k * m + i] = -U2[(long)k * m + i];
            for (long i = 0; i < n; ++i) V2[(long)k * n + i] = -V2[(long)k * n + i];
        }
    }
    memcpy(sig, s2, sizeof(double) * d);
    memcpy(U, U2, sizeof(double) * m * d);
    memcpy(V, V2, sizeof(double) * n * d);
    free(perm); free(s2); free(U2); free(V2);
}

/* Round-robin (tournament) pairing: round r of n-1 (n even) pairs the
 * positions so that every pair (p,q) meets exactly once per sweep. */
static void rr_pair(int n, int r, int t, int *p, int *q)
{
    /* player n-1 is fixed; others rotate */
    int a = (t == 0) ? n - 1 : (r + t) % (n - 1);
    int b = (r - t + (n - 1)) % (n - 1);
    if (t == 0) b = r % (n - 1);
    *p = a < b ? a : b;
    *q = a < b ? b : a;
}

/* One-sided (Hestenes) Jacobi SVD of the explicit m x n row-major matrix A.
 * Orthogonalises the columns of A if n <= m, else of A^T, so that the
 * rotations act on the shorter dimension.  On return (d = min(m, n)):
 * sig[d] descending, U (m x d, column-major), V (n x d, column-major),
 * A = U diag(sig) V^T.  Stops when every pair satisfies
 * |a_p . a_q| <= tol * |a_p| |a_q|.  Returns the number of sweeps, or -1 if
 * max_sweeps was reached. */
int orc_svd_jacobi(long m, long n, const double *A, double tol, int max_sweeps,
                   double *sig, double *U, double *V)
{
    int trans = n > m;                 /* work on columns of A^T */
    long len = trans ? n : m;          /* length of a working column */
    int d = (int)(trans ? m : n);      /* number of working columns  */
    double *G = (double *)malloc(sizeof(double) * len * d);   /* columns */
    double *R = (double *)calloc((size_t)d * d, sizeof(double)); /* rotations */
    for (int k = 0; k < d; ++k) {
        for (long i = 0; i < len; ++i)
            G[(long)k * len + i] = trans ? A[(long)k * n + i] : A[i * n + k];
        R[(long)k * d + k] = 1.0;
    }
    int nn = d + (d & 1);              /* pad to even for the tournament */
    int sweeps = 0, converged = 0;
    while (!converged && sweeps < max_sweeps) {
        converged = 1;
        for (int r = 0; r < nn - 1; ++r) {
            int npairs = nn / 2;
            int conv_round = 1;
            #pragma omp parallel for schedule(dynamic, 1) reduction(&& : conv_round)
            for (int t = 0; t < npairs; ++t) {
                int p, q;
                rr_pair(nn, r, t, &p, &q);
                if (q >= d) continue;              /* dummy player */
                double *ap = G + (long)p * len, *aq = G + (long)q * len;
                double alpha = dot(ap, ap, len), beta = dot(aq, aq, len), gamma = dot(ap, aq, len);
                if (fabs(gamma) <= tol * sqrt(alpha * beta) || gamma == 0.0) continue;
                conv_round = 0;
                double zeta = (beta - alpha) / (2.0 * gamma);
                double tt = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                double c = 1.0 / sqrt(1.0 + tt * tt), s = c * tt;
                for (long i = 0; i < len; ++i) {
                    double x1 = ap[i], x2 = aq[i];
                    ap[i] = c * x1 - s * x2;
                    aq[i] = s * x1 + c * x2;
                }
                double *rp = R + (long)p * d, *rq = R + (long)q * d;
                for (int i = 0; i < d; ++i) {
                    double x1 = rp[i], x2 = rq[i];
                    rp[i] = c * x1 - s * x2;
                    rq[i] = s * x1 + c * x2;
                }
            }
            if (!conv_round) converged = 0;
        }
        ++sweeps;
    }
    /* singular values = column norms; left vectors of the working matrix =
     * normalised columns; right vectors = accumulated rotations. */
    double *Lw = (double *)malloc(sizeof(double) * len * d);
    for (int k = 0; k < d; ++k) {
        double nk = sqrt(dot(G + (long)k * len, G + (long)k * len, len));
        sig[k] = nk;
        for (long i = 0; i < len; ++i)
            Lw[(long)k * len + i] = nk > 0 ? G[(long)k * len + i] / nk : 0.0;
    }
    if (!trans) {          /* A = Lw S R^T : U = Lw (m x d), V = R (n x d) */
        memcpy(U, Lw, sizeof(double) * m * d);
        memcpy(V, R, sizeof(double) * n * d);
    } else {               /* A^T = Lw S R^T  ->  A = R S Lw^T */
        memcpy(U, R, sizeof(double) * m * d);
        memcpy(V, Lw, sizeof(double) * n * d);
    }
    sort_and_sign(m, n, d, sig, U, V);
    free(G); free(R); free(Lw);
    return converged ? sweeps : -1;
}

/* Cyclic two-sided Jacobi eigen-decomposition of the symmetric n x n matrix
 * S (row-major, overwritten).  Outputs eigenvalues lam[n] (unsorted) and
 * eigenvectors as columns of Z (column-major, column k at Z + k*n).
 * Returns sweeps or -1. */
static int jacobi_eig(int n, double *S, double *lam, double *Z, double tol, int max_sweeps)
{
    memset(Z, 0, sizeof(double) * (size_t)n * n);
    for (int i = 0; i < n; ++i) Z[(long)i * n + i] = 1.0;
    int nn = n + (n & 1), sweeps = 0, converged = 0;
    while (!converged && sweeps < max_sweeps) {
        converged = 1;
        for (int r = 0; r < nn - 1; ++r) {
            int npairs = nn / 2;
            int conv_round = 1;
            /* rotation angles for this round: pairs are disjoint, so the
             * similarity transform is applied as one product of rotations:
             * first all row updates, then all column updates. */
            double *cs = (double *)malloc(sizeof(double) * 2 * npairs);
            int *pq = (int *)malloc(sizeof(int) * 2 * npairs);
            for (int t = 0; t < npairs; ++t) {
                int p, q;
                rr_pair(nn, r, t, &p, &q);
                pq[2 * t] = p; pq[2 * t + 1] = q;
                cs[2 * t] = 1.0; cs[2 * t + 1] = 0.0;
                if (q >= n) continue;
                double apq = S[(long)p * n + q], app = S[(long)p * n + p], aqq = S[(long)q * n + q];
                if (fabs(apq) <= tol * sqrt(fabs(app * aqq)) || apq == 0.0) continue;
                conv_round = 0;
                double theta = (aqq - app) / (2.0 * apq);
                double tt = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(1.0 + theta * theta));
                double c = 1.0 / sqrt(1.0 + tt * tt);
                cs[2 * t] = c; cs[2 * t + 1] = c * tt;
            }
            if (!conv_round) converged = 0;
            /* S <- J^T S J with J the product of the disjoint rotations:
             * rows p,q: row_p' = c row_p - s row_q ; row_q' = s row_p + c row_q */
            #pragma omp parallel for schedule(static)
            for (int t = 0; t < npairs; ++t) {
                int p = pq[2 * t], q = pq[2 * t + 1];
                if (q >= n || cs[2 * t + 1] == 0.0) continue;
                double c = cs[2 * t], s = cs[2 * t + 1];
                for (int k = 0; k < n; ++k) {
                    double x1 = S[(long)p * n + k], x2 = S[(long)q * n + k];
                    S[(long)p * n + k] = c * x1 - s * x2;
                    S[(long)q * n + k] = s * x1 + c * x2;
                }
            }
            #pragma omp parallel for schedule(static)
            for (int k = 0; k < n; ++k)
                for (int t = 0; t < npairs; ++t) {
                    int p = pq[2 * t], q = pq[2 * t + 1];
                    if (q >= n || cs[2 * t + 1] == 0.0) continue;
                    double c = cs[2 * t], s = cs[2 * t + 1];
                    double x1 = S[(long)k * n + p], x2 = S[(long)k * n + q];
                    S[(long)k * n + p] = c * x1 - s * x2;
                    S[(long)k * n + q] = s * x1 + c * x2;
                }
            #pragma omp parallel for schedule(static)
            for (int t = 0; t < npairs; ++t) {
                int p = pq[2 * t], q = pq[2 * t + 1];
                if (q >= n || cs[2 * t + 1] == 0.0) continue;
                double c = cs[2 * t], s = cs[2 * t + 1];
                double *zp = Z + (long)p * n, *zq = Z + (long)q * n;
                for (int k = 0; k < n; ++k) {
                    double x1 = zp[k], x2 = zq[k];
                    zp[k] = c * x1 - s * x2;
                    zq[k] = s * x1 + c * x2;
                }
            }
            free(cs); free(pq);
        }
        ++sweeps;
    }
    for (int i = 0; i < n; ++i) lam[i] = S[(long)i * n + i];
    return converged ? sweeps : -1;
}

/* The SVD step exactly as the paper defines it (Section 2.1, Step 2):
 * lambda_j and U_j are the eigenpairs of S = X X^T, and the caller forms
 * V_j = X^T U_j / sqrt(lambda_j).  S (m x m, row-major, overwritten) is
 * formed by the caller with a library matrix product.  Outputs the
 * eigenvalues in decreasing order in lam and the matching eigenvectors as
 * the columns of U (column-major, column k at U + k*m).  Used for the large
 * workloads, where the one-sided iteration over the long columns is too
 * slow.  Returns the sweep count or -1. */
int orc_eig_gram(long m, double *S, double tol, int max_sweeps, double *lam, double *U)
{
    int mm = (int)m;
    double *ev = (double *)malloc(sizeof(double) * m);
    double *Z = (double *)malloc(sizeof(double) * m * m);
    int sw = jacobi_eig(mm, S, ev, Z, tol, max_sweeps);
    int *perm = (int *)malloc(sizeof(int) * m);
    for (int k = 0; k < mm; ++k) perm[k] = k;
    for (int a = 1; a < mm; ++a) {                /* insertion sort, stable */
        int p = perm[a], b = a - 1;
        while (b >= 0 && ev[perm[b]] < ev[p]) { perm[b + 1] = perm[b]; --b; }
        perm[b + 1] = p;
    }
    for (int k = 0; k < mm; ++k) {
        lam[k] = ev[perm[k]];
        memcpy(U + (long)k * m, Z + (long)perm[k] * m, sizeof(double) * m);
    }
    free(ev); free(Z); free(perm);
    return sw;
}

/* ------------------------------------------------------------------------ */
/* Reconstruction                                                           */
/* ------------------------------------------------------------------------ */

/* Shaped reconstruction of one group: Y = sum_{k in G} sig_k U_k V_k^T,
 * then out(alpha) = sum of Y_ij over l_i + k_j = alpha, divided by the
 * number of such (i, j).  Cells no pair reaches get NaN.  U (nl x d) and
 * V (nk x d) are column-major.  Each Y_ij is formed on the fly. */
void orc_reconstruct(int nx, int ny, int nl, const int *li, const int *lj,
                     long nk, const int *ki, const int *kj, int d,
                     const double *sig, const double *U, const double *V,
                     int gsize, const int *group, double *out)
{
    long npix = (long)nx * ny;
    double *acc = (double *)calloc((size_t)npix, sizeof(double));
    double *cnt = (double *)calloc((size_t)npix, sizeof(double));
    for (int i = 0; i < nl; ++i)
        for (long j = 0; j < nk; ++j) {
            double y = 0.0;
            for (int g = 0; g < gsize; ++g) {
                int k = group[g];
                y += sig[k] * U[(long)k * nl + i] * V[(long)k * nk + j];
            }
            long a = (long)(li[i] + ki[j]) * ny + (lj[i] + kj[j]);
            acc[a] += y;
            cnt[a] += 1.0;
        }
    (void)d;
    for (long a = 0; a < npix; ++a) out[a] = cnt[a] > 0 ? acc[a] / cnt[a] : NAN;
    free(acc); free(cnt);
}

/* MSSA reconstruction of one group on the stacked Hankel matrix: for series
 * p, x~_p(t) = average of Y_ij over the block of p with i + j = t.
 * out is the concatenation of the s reconstructed series. */
void orc_reconstruct_mssa(int s, const int *lens, int L, int d, const double *sig,
                          const double *U, const double *V, int gsize, const int *group,
                          double *out)
{
    long K = 0, off = 0, col = 0;
    for (int p = 0; p < s; ++p) K += lens[p] - L + 1;
    (void)d;
    for (int p = 0; p < s; ++p) {
        int Kp = lens[p] - L + 1;
        double *acc = out + off;
        double *cnt = (double *)calloc((size_t)lens[p], sizeof(double));
        for (int t = 0; t < lens[p]; ++t) acc[t] = 0.0;
        for (int i = 0; i < L; ++i)
            for (int j = 0; j < Kp; ++j) {
                double y = 0.0;
                for (int g = 0; g < gsize; ++g) {
                    int k = group[g];
                    y += sig[k] * U[(long)k * L + i] * V[(long)k * K + col + j];
                }
                acc[i + j] += y;
                cnt[i + j] += 1.0;
            }
        for (int t = 0; t < lens[p]; ++t) acc[t] /= cnt[t];
        free(cnt);
        col += Kp;
        off += lens[p];
    }
}

/* The same averaging evaluated only at the listed cells (pi[t], pj[t]):
 * for each cell, visit every window cell l_i, take k = cell - l_i, and add
 * Y_ij if k is an origin.  korigin maps a box position (kx-by-ky, row-major)
 * to its index in the origin list, or -1. */
void orc_reconstruct_at(int nl, const int *li, const int *lj, int kx, int ky,
                        const long *korigin, long nk, int d, const double *sig,
                        const double *U, const double *V, int gsize, const int *group,
                        long npts, const int *pi, const int *pj, double *out)
{
    (void)d;
    #pragma omp parallel for schedule(static)
    for (long t = 0; t < npts; ++t) {
        double acc = 0.0, cnt = 0.0;
        for (int i = 0; i < nl; ++i) {
            int a = pi[t] - li[i], b = pj[t] - lj[i];
            if (a < 0 || b < 0 || a >= kx || b >= ky) continue;
            long j = korigin[(long)a * ky + b];
            if (j < 0) continue;
            double y = 0.0;
            for (int g = 0; g < gsize; ++g) {
                int k = group[g];
                y += sig[k] * U[(long)k * nl + i] * V[(long)k * nk + j];
            }
            acc += y;
            cnt += 1.0;
        }
        out[t] = cnt > 0 ? acc / cnt : NAN;
    }
}

/* Rows [r0, r1) of S = X X^T (all columns), X m x n row-major; S_out is
 * (r1-r0) x m row-major.  Same plain sums as the full Gram formation. */
void orc_gram_rows(long m, long n, const double *X, long r0, long r1, double *S_out)
{
    #pragma omp parallel for schedule(dynamic, 1) collapse(2)
    for (long i = r0; i < r1; ++i)
        for (long j = 0; j < m; ++j)
            S_out[(i - r0) * m + j] = dot(X + i * n, X + j * n, n);
}

/* Threads of the parallel loops (timing of the oracle itself only). */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
