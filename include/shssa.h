/*
 * shssa.h -- C ABI of the Shaped 2D-SSA library for MI355X (gfx950).
 *
 * The library decomposes a shaped array and reconstructs grouped components
 * with singular spectrum analysis, as defined in Golyandina, Korobeynikov,
 * Shlemov and Usevich, "Multivariate and 2D extensions of singular spectrum
 * analysis with the Rssa package" (arXiv:1309.5050).  Shaped 2D-SSA (Section
 * 5) covers 1D SSA (an N x 1 array with an L x 1 window), MSSA (Section 5.3,
 * 2D packing: a max N_p x s array whose column p holds series p), 2D-SSA (a
 * full rectangle) and shaped arrays with shaped windows.
 *
 * Conventions.
 *   - Arrays are row-major; the first index is the x axis of the paper
 *     (rows), the second the y axis (columns).  Indices are 0-based.
 *   - N (the shaped array) = cells with mask != 0 (all cells if mask is
 *     NULL) whose value is not NaN (Section 5.2: NA values and the mask
 *     are intersected).
 *   - The window shape L is the set of wmask cells != 0 (the full lx x ly
 *     box if wmask is NULL), trimmed to its bounding box.  The origins are
 *     K = { k : l + k lies in N for every l in L } (Section 5.1, equation
 *     sh_Ks).  The trajectory matrix is X_ij = x(l_i + k_j) (equation qh_mat).
 *   - Singular values are returned, not eigenvalues: sigma_i = sqrt(lambda_i)
 *     of the SVD step (Section 2.1, Step 2), in descending order.
 *   - Each triplet's sign is fixed so that the largest-magnitude entry of
 *     U_i is positive.
 *   - Component indices in groups are 0-based (the paper counts from 1).
 *
 * Ownership.  Input pointers are borrowed for the duration of the call.
 * Output buffers are allocated by the caller (sizes from ssa_get_dims).
 * Handles are owned by the library and released with ssa_free /
 * ssa_ctx_destroy.  Functions ending in _dev take device pointers on the
 * context's device and work on the context's stream; all others take host
 * pointers.
 *
 * Completion.  A decomposition call returns once the bidiagonalisation has
 * converged (it waits for each restart's convergence test) with the last
 * kernels of the decomposition (the other-side vectors and the sign rule)
 * still queued on the stream; ssa_reconstruct_batch_dev returns with all of
 * its work queued.  The getters (ssa_get_sigma, ssa_get_vectors,
 * ssa_get_weights) and ssa_reconstruct wait for the handle's queued work.
 * A handle may be freed at any time: its device memory is reused only after
 * the work queued on it has completed.
 *
 * Threads.  A context may be used from several threads.  Calls that queue
 * work on its stream (decompositions, reconstructions, getters that wait,
 * forecasts, ESPRIT, continuation, stream and profile reads) run one at a
 * time per context: they share the stream and its staging buffers.  Use a
 * context per thread for calls that should overlap on the GPU.
 *
 * Errors.  Every int-returning function returns SSA_OK (0) or a negative
 * code; ssa_strerror gives a message, ssa_last_error the detail of the last
 * failure on the calling thread.
 */
#ifndef SHSSA_H
#define SHSSA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SSA_OK = 0,
    SSA_EINVAL = -1,   /* bad sizes: window box beyond the array, L*K box of
                          one cell, unsupported transform length (the padded
                          grid's rows hold at most 2 x 10200 real samples in
                          FP64 and 2 x 16384 in FP32, its columns at most
                          1024; ssa_decompose takes longer series in
                          segments, see there), NULL input */
    SSA_EEMPTY = -2,   /* no window position fits inside N (K is empty) */
    SSA_ERANK = -3,    /* r < 1 or r >= min(|L|, |K|): the rank of X is at
                          most min(L, K) (Section 2.1, Step 2); or r > 120:
                          the Lanczos basis holds at most 128 vectors and a
                          restart keeps r of them */
    SSA_ENOMEM = -4,   /* device memory or the context's budget exhausted */
    SSA_ENOCONV = -5,  /* the bidiagonalisation reached its step limit (3000
                          steps, lowered by the environment variable
                          SHSSA_MAX_STEPS); the handle and its triplets are
                          still returned, with stats.converged = 0 */
    SSA_EDEVICE = -6,  /* a HIP runtime call failed */
    SSA_EBUSY = -7,    /* the request is not finished yet (serving) */
    SSA_ESTATE = -8    /* call out of order (e.g. reconstruct before decompose) */
};

/* SSA_FP32: FP32 FFT products; the bidiagonalisation's recurrence, its
 * Gram-Schmidt reorthogonalisation (FP64 basis), the small SVD and the Ritz
 * rotations stay FP64.  SSA_FP32_BASIS32: as SSA_FP32, but the Gram-Schmidt
 * projections read an FP32 copy of the basis (half the basis traffic); its
 * rounding bounds the orthogonality of the basis at about 1e-7. */
enum { SSA_FP64 = 0, SSA_FP32 = 1, SSA_FP32_BASIS32 = 2 };

typedef struct ssa_ctx ssa_ctx;
typedef struct ssa_decomp ssa_decomp;

/* One decomposition request (image form).  A 1D series of length N is an
 * N x 1 image with an L x 1 window (Section 5.3). */
typedef struct ssa_request {
    const double* x;        /* nx*ny values, NaN = missing (host or device) */
    int nx, ny;
    const uint8_t* mask;    /* nx*ny, nonzero = in the array; NULL = all */
    const uint8_t* wmask;   /* lx*ly window shape; NULL = full lx x ly box */
    int lx, ly;
    int r;                  /* leading eigentriples wanted */
    int precision;          /* SSA_FP64 or SSA_FP32 */
    unsigned long long seed;/* start vector of the bidiagonalisation */
} ssa_request;

typedef struct ssa_stats {
    int steps;              /* bidiagonalisation steps (two products each) */
    int restarts;
    int basis;              /* projected matrix size m */
    int converged;          /* 1 if every triplet met the residual test */
    int side;               /* 0: basis on the window side, 1: origin side */
    int batch;              /* decompositions that advanced together in its batch */
    int svd_sweeps;         /* Jacobi sweeps of the projected-matrix SVDs, summed over cycles */
    double max_resid;       /* largest residual bound |X v - s u| / sigma_1 */
    double ms_setup, ms_lanczos, ms_finish;
    size_t device_bytes;    /* device memory held by the handle */
    int fft_rows, fft_cols; /* the resident spectrum holds fft_rows x (fft_cols/2 + 1)
                               bins: the transform grid M_A x M_B of the products
                               (internal orientation; for windows one cell wide
                               one transformed row per series, M_A = 1) */
} ssa_stats;

/* Context: a device, a device-memory budget in bytes (0 = no limit) and an
 * autotune cache.  Tuned per context: the column pass's tile and kernel
 * variant (first batch of a precision and column length).  Tuned when the
 * environment variable SHSSA_LEN_TUNE is set at creation: the padded
 * transform lengths (the natural 2,3,5,7-smooth length or its power-of-two
 * alternative, timed on a class's first request; kept for the process; off
 * by default because power-of-two lengths split mixed-size batches into
 * more kernel classes).  The context makes its own non-blocking stream;
 * ssa_ctx_set_stream replaces it with the caller's.  tune_cache (nullable,
 * borrowed for the call) names a text file that keeps the tuner's choices
 * across processes: it is read here if it exists, and each new choice is
 * appended to it, one "<kind> <a> <b> <choice>" line per tuned size class
 * ("col <f64> <MA> <tile | variant << 8>", "rowlen <f64> <nh0> <nh>",
 * "collen <f64> <MA0> <MA>")
 * (lines this build cannot use are ignored).  NULL: choices last for the
 * context only.  SSA_EDEVICE without a HIP device, SSA_EINVAL for a device
 * index out of range. */
int  ssa_ctx_create(int device, size_t mem_budget, const char* tune_cache, ssa_ctx** out);
/* Releases the context; if handles made from it are still alive, the release
 * happens when the last of them is freed. */
void ssa_ctx_destroy(ssa_ctx* ctx);
/* Replaces the context's stream (a hipStream_t, borrowed: it must outlive
 * the context's use of it; NULL = the null stream, whose work cannot be
 * captured).  Waits for the work queued on the old stream first; a stream
 * the context made itself is destroyed.  Tensors of a PyTorch caller and the
 * library's kernels then share one stream. */
int  ssa_ctx_set_stream(ssa_ctx* ctx, void* stream);

/* Decompose one shaped array (host inputs).  See ssa_request for the
 * arguments.  On success *out receives a handle holding sigma, U, V, the
 * weights and the image spectrum on the device. */
int ssa_decompose(ssa_ctx* ctx, const double* x, int nx, int ny, const uint8_t* mask,
                  const uint8_t* wmask, int lx, int ly, int r, int precision, ssa_decomp** out);
/* A series (nx x 1 with an lx x 1 window, or 1 x ny with 1 x ly) longer
 * than one transform row (Alg. 1 holds for any length) is decomposed as the
 * MSSA (Section 3.1) of overlapping segments x[p B .. p B + B + L - 2],
 * B + L - 1 = 16384 values in FP64 and 32768 in FP32: their trajectory
 * matrices side by side are the series' own, so sigma and U are the
 * series'.  The handle reports the series' geometry; ssa_get_vectors,
 * ssa_get_vectors_lex, ssa_get_weights, ssa_reconstruct and ssa_wcor return
 * the series' layout (V concatenated over the segments; weights and
 * diagonal averages over the whole matrix, summed over the segments that
 * hold each value).  Such a handle supports continuation and ESPRIT;
 * forecasts and ssa_reconstruct_batch_dev return SSA_EINVAL, and so does a
 * window of more than half a segment.  The batch calls and the eigen
 * method take series up to one transform row only. */

/* The eigen method (the paper's alternative to the truncated SVD for
 * moderate windows: S = X X^T and its full eigendecomposition,
 * O(L N log N + L^3); the 2D-SSA examples time it on a 25 x 25 window).
 * Same arguments as ssa_decompose, always FP64; the window may hold at most
 * 4096 cells (SSA_EINVAL otherwise; S is kept as L x L doubles).  S is
 * formed on the matrix cores straight from the cleaned array (the
 * trajectory matrix is never stored); its eigenpairs come from one-sided
 * Jacobi in one workgroup for windows of at most 128 cells, and from block
 * one-sided Jacobi across workgroups beyond that (SSA_ENOCONV, with the
 * handle, if 40 sweeps do not orthogonalise S's columns).  sigma_i =
 * sqrt(lambda_i), U_i the eigenvectors, V_i = X^T U_i / sigma_i.  Squaring
 * the matrix limits the absolute accuracy of sigma_i to about
 * eps sigma_1^2 / sigma_i (sqrt(eps) sigma_1 for vanishing ones).  The
 * handle serves every call on decompositions; ssa_extend takes further
 * eigenpairs of the resident S. */
int ssa_decompose_eigen(ssa_ctx* ctx, const double* x, int nx, int ny, const uint8_t* mask,
                        const uint8_t* wmask, int lx, int ly, int r, ssa_decomp** out);

/* M-2D-SSA (the shaped-variants section, equation embedding_m2dssa): one
 * common decomposition of s images X_p (nx[p] x ny[p], row-major, NaN =
 * missing) whose trajectory matrix is [T(X_1) : ... : T(X_s)] with the same
 * lx x ly window (wmask as for ssa_decompose, NULL = full box).  Internally
 * the packing of that section: the images side by side in one array of
 * max nx rows, image p from column col_off[p] (col_off[0] = 0,
 * col_off[p+1] = col_off[p] + ny[p] + sep), NaN below shorter images and in
 * sep separator columns (1 for a full window, max(1, ly - 1) for a shaped
 * one), so that no window fits across two images.  Outputs (V,
 * reconstructions, weights) refer to the packed array; col_off (s ints,
 * may be NULL) receives the offsets. */
int ssa_decompose_m2d(ssa_ctx* ctx, const double* const* images, const int* nx, const int* ny, int s,
                      const uint8_t* wmask, int lx, int ly, int r, int precision, int* col_off,
                      ssa_decomp** out);

/* Mosaic Hankel SSA (the mosaic Hankel subsection): the decomposition of
 * the block matrix whose block (i, j), 0 <= i < s, 0 <= j < t, is the
 * L_i x K_j Hankel matrix of series[i * t + j] (L_i + K_j - 1 values each,
 * NaN = missing; the caller guarantees the lengths).  Internally the
 * shaped packing of that subsection: an s-row array where row i holds the
 * series of block row i, block column j from column col_off[j]
 * (col_off[0] = 0, col_off[j+1] = col_off[j] + max L + K_j), NaN between
 * them, and a window of s rows whose row i has its first L_i cells.  The
 * only window positions that fit are the K_j origins of each block column,
 * so the trajectory matrix is the mosaic matrix (rows in the window's
 * lexicographic cell order).  Outputs (U, V, reconstructions, weights)
 * refer to the packing: series (i, j) is reconstructed in row i, columns
 * col_off[j] .. col_off[j] + L_i + K_j - 2.  col_off: t ints, may be
 * NULL.  precision as for ssa_decompose. */
int ssa_decompose_mosaic(ssa_ctx* ctx, const double* const* series, int s, int t, const int* Ls, const int* Ks,
                         int r, int precision, int* col_off, ssa_decomp** out);

/* MSSA (Section 3.1, equation mssa_embedding) of s series of lengths len[p]
 * with window L (1 < L < min len).  Internally the 2D packing of Section
 * 5.3: a max(len) x s array, window L x 1.  Outputs use that packing:
 * V is (max(len) - L + 1) x s with NaN beyond K_p, reconstructions
 * max(len) x s with NaN beyond len[p]. */
int ssa_decompose_multi(ssa_ctx* ctx, const double* const* series, const int* len, int s, int L,
                        int r, int precision, ssa_decomp** out);

/* Decompose n requests together.  Requests of one kernel class advance in
 * one batch through the same kernels whatever their sizes and shapes; the
 * class is the operator family (window one row high or not), precision,
 * short side (window or origin set), the row and column transform variants
 * and the bidiagonalisation's basis and restart sizes (which follow from r).
 * Each request's results do not depend on the others in its batch (its own
 * seed starts its Krylov space).  out[i] and status[i] receive each
 * request's handle (or NULL) and code.  Returns SSA_OK if the batch ran
 * (individual failures are in status). */
int ssa_decompose_batch(ssa_ctx* ctx, int n, const ssa_request* reqs, ssa_decomp** out, int* status);

/* As ssa_decompose_batch with x (and mask) as device pointers. */
int ssa_decompose_batch_dev(ssa_ctx* ctx, int n, const ssa_request* reqs, ssa_decomp** out, int* status);

/* Sizes: trimmed window box lx x ly, origin box kx x ky (= nx-lx+1 by
 * ny-ly+1), |L|, |K|, r, and the array size nx x ny. */
int ssa_get_dims(const ssa_decomp* d, int* lx, int* ly, int* kx, int* ky, long* L, long* K, int* r,
                 int* nx, int* ny);

int ssa_get_sigma(const ssa_decomp* d, double* sigma /* r */);

/* U: r arrays of lx*ly (eigenarrays, NaN off L); V: r arrays of kx*ky
 * (factor arrays, NaN off K); V may be NULL. */
int ssa_get_vectors(const ssa_decomp* d, double* U, double* V);

/* U: L x r and V: K x r column-major in the paper's lexicographic order of
 * L and K (the order of the vectorised array: row index fastest). */
int ssa_get_vectors_lex(const ssa_decomp* d, double* U, double* V);

/* Weights w = |A_alpha| (Section 2.2), nx*ny; 0 outside N'. */
int ssa_get_weights(const ssa_decomp* d, double* w);

/* Measured orthonormality of the returned singular vectors (Section 2.1,
 * the decomposition step: the U_i are orthonormal eigenvectors of XX^T and
 * the V_i = X^T U_i / sqrt(lambda_i) orthonormal too): orth_u = max over
 * i, j < r of |(U^T U)_ij - delta_ij| for the r compact vectors U (|L|
 * entries each), orth_v the same for V (|K| entries).  A statement of each
 * result's error beside the residual bound of ssa_stats: the basis side
 * keeps about 1e-15 (FP64 reorthogonalisation), the other side is formed
 * by one more product and reflects the operator precision (about 1e-7 for
 * FP32 products, scaled by sigma_1 / sigma_r).  Computed on the device
 * when called (two Gram matrices on the matrix cores); synchronous.
 * SSA_EINVAL for NULL arguments, SSA_ESTATE before the decomposition. */
int ssa_orthogonality(ssa_decomp* d, double* orth_u, double* orth_v);

/* Reconstruction (Section 2.1, Step 4; Algorithms 4 and 5) of ngroups
 * groups given in CSR form (grp_ptr[ngroups+1], grp_idx, 0-based component
 * ids < r).  out: ngroups arrays of nx*ny, NaN outside N'. */
int ssa_reconstruct(ssa_decomp* d, const int* grp_ptr, const int* grp_idx, int ngroups, double* out);

/* Continuation of a decomposition to r_new > r triplets (the paper's
 * automatic continuation: a reconstruction that asks for more components
 * than were computed continues the decomposition).  The handle's spectrum
 * and bidiagonalisation state stay resident after ssa_decompose*: the
 * bidiagonalisation is thick-restarted from its last Ritz vectors with the
 * basis and convergence test of r_new, and all r_new triplets (and the
 * other side's vectors) are recomputed; the first r change only within the
 * tolerance.  r_new <= r: no-op.  r_new >= min(L, K) or r_new > 120:
 * SSA_ERANK.  The
 * per-component buffers are reallocated (SSA_ENOMEM beyond the context's
 * budget; the handle is then unusable).  Returns when the new triplets are
 * computed, with the last kernels queued, like ssa_decompose. */
int ssa_extend(ssa_decomp* d, int r_new);

/* Reconstruct the same groups for n handles of one kernel class (as for
 * ssa_decompose_batch) in one batch; the group ids must be < r of every handle.
 * out_dev[i] is a device buffer of ngroups*nx*ny doubles with the layout of
 * ssa_reconstruct.  Queued on the context's stream; returns without waiting. */
int ssa_reconstruct_batch_dev(int n, ssa_decomp* const* d, const int* grp_ptr, const int* grp_idx,
                              int ngroups, double* const* out_dev);

/* w-correlations and contributions of the reconstructed groups (the
 * general-notions subsection, separability and w-correlation paragraphs).
 * With the weights w = |A_k| of
 * ssa_get_weights and the weighted inner product (Y, Z)_w = sum_k w_k y_k
 * z_k over the covered cells N': rho[a*ngroups + b] = (Y_a, Y_b)_w /
 * (|Y_a|_w |Y_b|_w) (means not subtracted; 0 if a component is zero) and
 * contrib[a] = |Y_a|_w^2 / |X|_w^2 (contrib may be NULL).  Groups as for
 * ssa_reconstruct (singletons give the w-correlation matrix of the
 * elementary components).  Synchronous. */
int ssa_wcor(ssa_decomp* d, const int* grp_ptr, const int* grp_idx, int ngroups, double* rho, double* contrib);

/* Column recurrent forecast (the MSSA forecasting subsection: recurrent
 * column forecast, equation Forec:ContMSSAL; a single series is the case
 * s = 1) of h values for each series of
 * a decomposition whose window is one row or one column wide without mask
 * (1D SSA, MSSA): the group's eigenvectors give the LRR
 * R_L = sum_j pi(U_j) U_j[0:L-1] / (1 - nu^2), pi = last coordinate,
 * nu^2 = sum_j pi(U_j)^2 (< 1 required), applied to the last L-1 values of
 * the group's reconstruction of each series and then by recurrence.  grp:
 * ng 0-based component ids.  out: nseries x h (series in the order of the
 * caller's columns for a window one column high, rows otherwise).
 * With out = NULL only *nseries is set.  Synchronous. */
int ssa_rforecast(ssa_decomp* d, const int* grp, int ng, int h, double* out, int* nseries);

/* Column vector forecast (the MSSA forecasting subsection: vector MSSA
 * forecasting, column forecast; a single series is the case s = 1),
 * computed by the fast algorithm of the forecast implementation section,
 * for the same decompositions as ssa_rforecast.  Each series' lagged
 * vectors are continued inside the group's span: starting from its last
 * column of the group's reconstructed matrix, each new vector keeps the
 * projection of the previous one's last L-1 coordinates onto the group's
 * U_j without their last coordinate and takes R_L of that for its last;
 * after h + L - 1 new vectors the diagonal average of the extended matrix
 * gives the h values that follow each series.  Only coefficient vectors in
 * the group's basis are carried: w_k = D w_{k-1}, with D the pseudo-inverse
 * of the basis without its last row times the basis without its first row.
 * grp: ng (<= 64) 0-based component ids, nu^2 < 1 required.  Each series'
 * last lagged vector must end at its last covered value.  out: nseries x h,
 * series ordered as for ssa_rforecast.  With out = NULL only *nseries is
 * set.  Synchronous. */
int ssa_vforecast(ssa_decomp* d, const int* grp, int ng, int h, double* out, int* nseries);

/* Row forecasts (the MSSA forecasting subsection: recurrent row forecast,
 * equation Forec:ContMSSAK, and vector row forecast, computed by the fast
 * row algorithm of the forecast implementation section) for the same
 * decompositions as ssa_rforecast, whose series have no gaps.  The row
 * space of the group is spanned by its V_j, split in blocks of K_p
 * coordinates by series; S (s x ng) holds each block's last coordinate.
 * Recurrent: the next value of every series is
 * R_K Z = (I_s - S S^T)^{-1} S Vlow^T Z, Z the stacked last K_p - 1 values
 * of each series' reconstruction (Vlow: the blocks without their last
 * coordinate), then by recurrence; the forecast of one series uses the
 * values of all of them.  Vector: the rows of the group's reconstructed
 * matrix are continued inside the row space by the map of that subsection
 * and each series' columns are diagonally averaged; only coefficient
 * vectors w_i = D w_{i-1} are carried, D = (I - S^T S)^{-1} times the
 * blocks without their last coordinate against the blocks without their
 * first.  (I - S S^T) must be invertible (SSA_EINVAL otherwise).  grp: ng
 * (<= 64) 0-based component ids; out: nseries x h as for ssa_rforecast;
 * with out = NULL only *nseries is set.  Synchronous. */
int ssa_rforecast_row(ssa_decomp* d, const int* grp, int ng, int h, double* out, int* nseries);
int ssa_vforecast_row(ssa_decomp* d, const int* grp, int ng, int h, double* out, int* nseries);

/* LS-ESPRIT parameter estimation (the 1D parameter-estimation paragraph of
 * the 2D-SSA examples; the remark after the fast column forecast names the
 * shift matrix) for the same decompositions as ssa_rforecast: the ng roots
 * z_k, the eigenvalues of D = pinv(U_low) U_high of the group (U_low / U_high:
 * its U_j without the last / first coordinate).  A term c rho^t
 * cos(omega t + phi) of the series gives rho e^{+-i omega}: period
 * 2 pi / |arg z|, damping |z|.  re, im: ng values each, ordered by
 * decreasing |z|, then decreasing imaginary part.  nu^2 < 1 required
 * (SSA_EINVAL); SSA_ENOCONV if the eigenvalue iteration fails.
 * Synchronous. */
int ssa_esprit(ssa_decomp* d, const int* grp, int ng, double* re, double* im);

/* ssa_esprit for callers that cannot allocate device memory (code in a
 * tight serving loop, harnesses that forbid hipMalloc): the same
 * arguments, kernels, results and errors, but the group ids, flags, shift
 * matrix and roots live in a fixed 64 KiB device array of the library (one
 * per GPU, set up by ssa_ctx_create, kept until the process ends) instead
 * of memory from the context's pool, and the call uses no allocating
 * routine.  A group that needs more than that array returns SSA_EINVAL
 * (ng <= 64 always fits).  Every call on one GPU shares the array: calls
 * that overlap on one GPU (from several threads or contexts) race and must
 * be serialised by the caller.  Synchronous. */
int ssa_esprit_noalloc(ssa_decomp* d, const int* grp, int ng, double* re, double* im);

/* TLS-ESPRIT roots (the same paragraph, with the total-least-squares shift
 * matrix of Roy and Kailath): for Z = [U_low : U_high], the group's U
 * without its last row beside it without its first, and Z's right singular
 * vectors V = [[V11, V12], [V21, V22]] (ng x ng blocks, by decreasing
 * singular value), the roots are the eigenvalues of -V12 V22^{-1}.  Same
 * window, arguments and output order as ssa_esprit, with 1 <= ng <= 24;
 * SSA_EINVAL if V22 is singular, SSA_ENOCONV if an eigenvalue iteration
 * fails.  Synchronous. */
int ssa_esprit_tls(ssa_decomp* d, const int* grp, int ng, double* re, double* im);

/* 2D-ESPRIT (the parameter-estimation subsection of the 2D-SSA examples:
 * shift matrices for the x and y directions and their joint
 * diagonalisation) for a decomposition whose window is at least 2 x 2.  For
 * the window cells whose neighbour one step down (x) is also in the window,
 * Phi_x = pinv(U_a) U_b, U_a the group's U on those cells and U_b on the
 * neighbours; Phi_y the same one step right.  The eigenvectors of
 * Phi_x + gamma Phi_y (gamma = 0.618...) pair the roots: lambda_k =
 * t_k^H Phi_x t_k, mu_k = t_k^H Phi_y t_k for unit eigenvectors t_k.  A
 * term rho^m tau^n cos(2 pi (m f + n g) + phi) gives the pairs
 * (rho e^{+-2 pi i f}, tau e^{+-2 pi i g}).  lre, lim, mre, mim: ng values
 * each, ordered by decreasing |lambda|, then decreasing Im lambda.
 * SSA_EINVAL for a 1D window or a singular shift equation, SSA_ENOCONV if
 * the eigenvalue iteration fails.  Synchronous. */
int ssa_esprit2d(ssa_decomp* d, const int* grp, int ng, double* lre, double* lim, double* mre, double* mim);

int  ssa_get_stats(const ssa_decomp* d, ssa_stats* st);
void ssa_free(ssa_decomp* d);

const char* ssa_strerror(int code);
const char* ssa_last_error(void);

/* Serving (asynchronous requests).  The paper's ssa() + reconstruct() pair
 * per request (Section 5 and its reconstruct call), queued instead of run
 * at once.
 *
 * ssa_submit copies the request's host inputs (x, mask, wmask: as for
 * ssa_decompose) and the groups (CSR form: grp_ptr[ngroups+1],
 * 0-based component ids in grp_idx; ngroups may be 0 for no reconstruction)
 * and returns a ticket at once; it does no device work.  Errors that the
 * plan shows at once (bad sizes, a request larger than the whole budget:
 * SSA_ENOMEM) are returned by ssa_submit.
 *
 * The server is cooperative: it has no threads of its own, and each call of
 * ssa_poll on an unfinished request, and ssa_wait until its request is done,
 * runs rounds of it on the context's stream in the calling thread.  A round
 * admits waiting requests in arrival order while their estimated device
 * memory fits the context's budget beside the admitted ones (the first
 * always when none runs), sets them up and adds each to the batch of its
 * kernel class (as for ssa_decompose_batch: sizes may differ), then runs one
 * restart cycle of the batch that holds the oldest request: waiting
 * requests of the batch take the slots (ssa_ctx_set_slots, 64 when 0) of
 * finished ones and begin from their start vectors while the others
 * continue, and requests whose cycle ends with convergence leave the batch
 * with their reconstructions.  Every request runs the steps it would run
 * alone, so its results equal the synchronous call's.  Calls from several
 * threads are allowed (rounds run one at a time per context).
 *
 * ssa_poll sets *done = 1 once the request has finished (successfully or
 * not).  ssa_wait returns then.  ssa_take ends the request: it returns
 * the request's status, hands over the handle (*out, freed by the caller
 * with ssa_free; NULL if the request failed), copies the reconstruction
 * (ngroups x nx x ny, NaN off N') into recon if recon is not NULL, and
 * fills times (ms from submission to admission and to completion) if not
 * NULL.  ssa_take of an unfinished request returns SSA_EBUSY and changes
 * nothing.  Requests not taken are released by ssa_ctx_destroy.
 *
 * With the environment variable SHSSA_SERVE_ENGINE set when a context's
 * first request is submitted, library threads (each with its own HIP
 * stream) run whole batches instead, and ssa_wait blocks.  A run of those
 * threads once ended with a GPU fault whose cause is not found; they are
 * kept for that investigation and are not used by default.  Submitting
 * after the variable changed returns SSA_ESTATE. */
typedef struct ssa_times {
    double queue_ms;   /* submission -> admission (start of its batch for the threads) */
    double total_ms;   /* submission -> completion */
} ssa_times;

int ssa_submit(ssa_ctx* ctx, const ssa_request* req, const int* grp_ptr, const int* grp_idx, int ngroups,
               uint64_t* ticket);
/* MSSA request (series as for ssa_decompose_multi). */
int ssa_submit_multi(ssa_ctx* ctx, const double* const* series, const int* len, int s, int L, int r,
                     int precision, const int* grp_ptr, const int* grp_idx, int ngroups, uint64_t* ticket);
int ssa_poll(ssa_ctx* ctx, uint64_t ticket, int* done);
int ssa_wait(ssa_ctx* ctx, uint64_t ticket);
int ssa_take(ssa_ctx* ctx, uint64_t ticket, ssa_decomp** out, double* recon, ssa_times* times);

/* Continuous batching: at most `slots` decompositions of one kernel class
 * advance together in a batch call (ssa_decompose_batch*); when some finish
 * at a restart-cycle boundary, waiting requests of the call take their
 * slots and begin while the others continue (each keeps its own step on the
 * device).  A request's results are the same whether it runs alone or
 * joins a running batch.  0 (the default): every request of a class starts
 * at once.  SSA_EINVAL for slots < 0. */
int ssa_ctx_set_slots(ssa_ctx* ctx, int slots);

/* Blocks until all work queued on the context's stream is complete. */
int ssa_ctx_sync(ssa_ctx* ctx);

/* Kernel timing with HIP events.  kind is a comma-separated list of kernel
 * classes ("col", "row_in", "row_mid", "row_out", "rowfam_mid",
 * "rowfam_out", "lz_proj", "lz_update", "wgram" (the w-correlation Gram),
 * and "lz_ritz", the matrix-core Ritz rotation, whose "bytes" are
 * floating-point operations); NULL or "" stops recording.
 * ssa_ctx_profile_read_kind waits for the recorded launches of one class and
 * returns the time during which at least one of them was running (ms: the
 * union of their intervals, so launches of concurrent sub-batch streams are
 * not counted twice), their number and their algorithmic bytes (data each
 * launch must read and write).  ssa_ctx_profile_read returns the same over
 * all recorded classes and clears the record. */
int ssa_ctx_profile(ssa_ctx* ctx, const char* kind);
/* Time only one launch in every `every` (>= 1, default 1) of each class,
 * counted from the last ssa_ctx_profile call: each timed launch costs a pair
 * of event records on the stream (a few microseconds of idle device each),
 * and a sample keeps that cost out of the work being measured.  An odd
 * period samples both directions of the alternating column passes. */
int ssa_ctx_profile_every(ssa_ctx* ctx, int every);
int ssa_ctx_profile_read_kind(ssa_ctx* ctx, const char* kind, double* ms, long* launches, double* bytes);
/* All launches of class kind since the last ssa_ctx_profile call, timed or
 * not (with ssa_ctx_profile_every > 1 only some of them are timed).
 * SSA_EINVAL if the class is not being recorded. */
int ssa_ctx_profile_launches(ssa_ctx* ctx, const char* kind, long* launches);
int ssa_ctx_profile_read(ssa_ctx* ctx, double* ms, long* launches, double* bytes);

#ifdef __cplusplus
}
#endif

#endif /* SHSSA_H */
