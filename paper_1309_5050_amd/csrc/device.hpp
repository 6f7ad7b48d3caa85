// Device-visible per-instance descriptors and launch arguments.
#pragma once
#include "common.hpp"

namespace shssa {

// Maximum Lanczos basis (projected matrix held in LDS as m x m doubles).
constexpr int kMaxBasis = 128;
// Largest rank a request may ask for: a thick restart keeps at least r Ritz
// vectors and each cycle must add new ones, so r leaves at least 8 free
// columns of the basis.
constexpr int kMaxRank = kMaxBasis - 8;
// Block width of the block Jacobi eigensolver (eigen method beyond
// kMaxBasis window cells) and the width of a block pair.
constexpr int kBjW = 16;
constexpr int kBjN = 2 * kBjW;
// Largest window (cells) of the eigen method: S = X X^T is held as L x L doubles.
constexpr int kEigMaxL = 4096;
// Rows per Lanczos row block.
constexpr int kLzRows = 256;

// Geometry, spectrum and scratch of one decomposition.
struct OpDesc {
    int A, B;           // grid rows / columns (internal orientation)
    int MA, MB;         // FFT lengths (MA = 1 for the row family)
    int P;              // bins of a row spectrum (MB/2 + 1)
    int ldp;            // row pitch of the row-major spectra (T1, T2, Xh): P rounded up to 16
    int rowfam;         // 1: window one row high
    double spec_scale;  // 1 / (MA MB) (grid family) or 1 / MB (row family): the spectrum's scale
    CellSet S[2];       // S[0] window cells (L), S[1] origins (K)
    FftPlan prow;       // complex transform of length MB/2 (+ real split twiddles)
    FftPlan pcol;       // complex transform of length MA (grid family)
    const void* Xh;     // spectrum, pre-scaled: grid [P][MA], row family [A][P]
    void* T1;           // scratch rows [nrows][P] per component slot
    void* T2;
    void* Us;           // stored spectra of U components (reconstruction)
    long tslot;         // complex elements per component slot in T1/T2
    long uslot;         // complex elements per component in Us
    const double* W;    // weights, A*B
    const double* xc;   // image with cells outside N zeroed, A*B (FP64)
    const uint8_t* nset;// A*B bytes
};

// Golub-Kahan bidiagonalisation state of one decomposition.  The short side
// (window set or origin set, whichever is smaller) keeps a full FP64 basis
// with classical Gram-Schmidt applied twice; the long side keeps only the
// last two (unnormalised) vectors, in the precision of the operator.
struct LzDesc {
    unsigned long long seed;   // start and restart vectors of this decomposition
    const int* step;    // [j, jstart] of the batch's current step (device; see kStepDev)
    int side;           // short side: 0 = window set, 1 = origin set
    int active;
    int r;              // triplets wanted
    double tol;         // stop when beta |q_i[m-1]| <= tol * sigma_1 for i < r
    double eps;         // breakdown threshold relative to the largest alpha / beta seen
    long n;             // short vector length
    long nl;            // long vector length
    double* Q;          // short basis n x (kMaxBasis+1), column-major (ld n)
    float* Q32;         // FP32 copy of Q that the reorthogonalisation reads (instances with
                        // FP32 products: half the basis traffic; nullptr otherwise)
    double* w;          // short work vector
    double* sin;        // modified input vector of the first step after a restart
    double* hp1;        // partial projections, nblk x (kMaxBasis+1)
    double* hp2;
    double* np;         // partial squared norms of w, nblk
    double* np0;        // partial squared norms of w before its first projection, nblk
    void* lbuf[2];      // long vectors (operator precision), ping-pong by step parity
    double* lnp[2];     // partial squared norms of the long vectors, per long-set row
    double* gam;        // [2] gamma_j = beta_{j-1} / alpha_{j-1} of the long update, by step parity
                        // (written by the input pass of step j, read by its long update)
    long lwords;        // 32-bit words of lbuf[0] and lbuf[1] together (contiguous)
    int lrows;          // rows of lnp[0] and of lnp[1] (lnp[1] = lnp[0] + lrows)
    double* Bm;         // projected matrix, kMaxBasis x kMaxBasis column-major (rows: short)
    double* Yl;         // left singular vectors of Bm (kMaxBasis ld)
    double* Yr;         // right singular vectors of Bm
    double* sig;        // singular values of Bm, descending
    int* perm;          // column order of the descending singular values
    double* beta;       // [0] residual norm after the last step, [1] worst residual / sigma_1,
                        // [2], [3] running scale (largest alpha, beta) by step parity
    int* flag;          // [0] converged, [1] sweeps of the last small SVD, [2] breakdown in
                        // this cycle, [3] the cycle started from a fresh random vector
    double* Qtmp;       // n x kMaxBasis (Ritz rotation target)
    int nblk;
};

// Final results of one decomposition (compact FP64 vectors).
struct ResDesc {
    int r;              // triplets of this decomposition
    double* U;          // L x r column-major (ld = L)
    double* V;          // K x r column-major (ld = K)
    double* sigma;      // r
    double* recon;      // ngroups x A x B
    const int* gptr;    // ngroups+1
    const int* gidx;
};

struct Item { int inst; int idx; int comp; int aux; };

// ---- kernel arguments

enum InMode : int {
    IN_LZ_NORM = 0,   // src = w / beta_{j-1}; stores q_j and B[j][j-1] = beta_{j-1}
    IN_LZ_PLAIN = 1,  // src = q_j
    IN_VEC = 2,       // src = result vector (U or V) component `comp`, times scale
    IN_DENSE = 3,     // src = dense image row (spectrum creation)
    IN_LZ_SIN = 4,    // src = modified input of the first step after a restart
    IN_LZ_STEP = 5,   // IN_LZ_SIN on the first step of a restarted cycle, else IN_LZ_NORM
                      // (step from the batch's step counter)
};

// A step index j of kStepDev in launch arguments: the step (and the cycle's
// first step) is read from the batch's step counter in device memory
// (LzDesc::step), so one captured step can be replayed for every j.
constexpr int kStepDev = -1;

// Largest group of a vector forecast (one lane of a wave per coordinate of
// the carried coefficient vectors).
constexpr int kVfMaxGroup = 64;
// TLS-ESPRIT: the 2 ng x 2 ng eigenproblem is solved in one workgroup's LDS.
constexpr int kTlsMaxGroup = 24;

// Weight of the y shift matrix in the combination whose eigenvectors pair
// the x and y roots of 2D-ESPRIT (any weight works when the shift matrices
// commute; an irrational one avoids chance coincidences of the combined
// eigenvalues).
constexpr double kEsprit2dGamma = 0.6180339887498949;

enum RowDest : int {
    DEST_T1 = 0,      // scratch slot `comp` of T1
    DEST_XH = 1,      // spectrum rows (row family), times the spectrum scale
};

struct RowInArgs {
    int mode, set, j, dest;
    double scale;     // IN_VEC: multiply by scale * sigma[comp] if use_sigma; DEST_XH: < 0 = spec_scale
    int use_sigma;
};

enum OutMode : int {
    OUT_NONE = 0,
    OUT_LZ = 1,      // compact values -> Lanczos w
    OUT_VEC = 2,     // compact values -> result vector component `comp`, times scale / sigma
    OUT_IMAGE = 3,   // dense row / W, NaN where W == 0 -> reconstruction `comp`
};

struct RowMidArgs {
    int set;          // mask set applied between the two transforms
    int emit;         // OUT_NONE or OUT_VEC (values of the masked row)
    double scale;     // emitted value = scale * value / sigma[comp] (if div_sigma)
    int div_sigma;
    int fwd;          // 1: transform the masked row forward again into T1
    int gk;           // 1: bidiagonalisation step j: l' = X^T q - gamma l'_{j-1}
    int j, jstart;
};

struct RowOutArgs {
    int mode;         // OUT_LZ, OUT_VEC or OUT_IMAGE
    int set;
    double scale;
    int div_sigma;
    int j;            // OUT_LZ: bidiagonalisation step
    int jstart;       // first step of the current cycle
};

struct RowFamArgs {
    int emit;         // OUT_VEC: emit masked values of X^T u (V side) / sigma
    int full;         // 1: go on to P_a = Xh_a conj(FFT(masked row))
    int gk;           // 1: bidiagonalisation step (long update as in k_row_mid)
    int j, jstart;
};

enum ColMode : int {
    COL_CORR = 0,     // fwd, * conj against Xh, inverse
    COL_SPEC = 1,     // fwd only, * scale, store transposed as the spectrum
    COL_STORE = 2,    // fwd only, store transposed into Us slot comp
    COL_ACCUM = 3,    // for i in group comp: fwd of T1 slot i, * Us_i, summed; inverse
};

// Row counts of the column pass, per instance: a count >= 0, or one of
// ROWS_ALL (A), ROWS_S0 (window box rows), ROWS_S1 (origin box rows).
enum { ROWS_ALL = -1, ROWS_S0 = -2, ROWS_S1 = -3 };

struct ColArgs {
    int mode;
    int nin;          // nonzero input rows (count or ROWS_*)
    int nout;         // output rows written to T2 (count or ROWS_*)
};

__host__ __device__ inline int col_rows(const OpDesc& op, int code) {
    return code >= 0 ? code : code == ROWS_ALL ? op.A : code == ROWS_S0 ? op.S[0].boxA : op.S[1].boxA;
}

// Window rows as runs: run t covers window row ra[t], columns [b0[t], b1[t]).
struct Runs { const int* ra; const int* b0; const int* b1; int nrun; long total; };

}  // namespace shssa
