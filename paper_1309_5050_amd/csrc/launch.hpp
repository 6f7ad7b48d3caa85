// Declarations of the kernel launch wrappers (defined with the kernels).
#pragma once
#include "device.hpp"

namespace shssa {

int row_class(int n, bool f64);
int row_slots(int cls);
// Rows per work item of the row passes: the register row kernels take one
// item per group of rows (instance, first row, component, row count); the
// dense modes and the LDS kernels one item per row.
int row_group(int cls, bool dense);
int col_tile(bool f64);                 // default column configuration (tile width, variant 0)
bool col_tile_ok(bool f64, int MA, int cfg);  // configurations compiled for the precision and length
int col_fast_logn(int MA);              // log2(MA) when the register column kernel applies, else 0

void launch_row_in(bool f64, int cls, int nitems, hipStream_t st, const OpDesc* ops, const LzDesc* lzs,
                   const ResDesc* res, const Item* items, RowInArgs a);
void launch_row_mid(bool f64, int cls, int nitems, hipStream_t st, const OpDesc* ops, const LzDesc* lzs,
                    const ResDesc* res, const Item* items, RowMidArgs a);
void launch_row_out(bool f64, int cls, int nitems, hipStream_t st, const OpDesc* ops, const LzDesc* lzs,
                    const ResDesc* res, const Item* items, RowOutArgs a);
void launch_rowfam_mid(bool f64, int cls, int nitems, hipStream_t st, const OpDesc* ops, const LzDesc* lzs,
                       const ResDesc* res, const Item* items, RowFamArgs a);
void launch_rowfam_out(bool f64, int cls, int nitems, hipStream_t st, const OpDesc* ops, const LzDesc* lzs,
                       const Item* items, RowOutArgs a);
void launch_rowfam_recon(bool f64, int cls, int nitems, hipStream_t st, const OpDesc* ops, const ResDesc* res,
                         const Item* items, double scale);
void launch_copy_uspec(bool f64, int nitems, hipStream_t st, const OpDesc* ops, const Item* items);
// cls: row size class, plus 8 when the row plan has radices 2, 4, 8 only.
void launch_col(bool f64, int nitems, hipStream_t st, const OpDesc* ops, const ResDesc* res, const Item* items,
                ColArgs a, int MA, int cfg);   // cfg: tile | variant << 8
void launch_shape_clean(int nitems, hipStream_t st, const OpDesc* ops, const Item* items, const double* const* x,
                        const uint8_t* const* m, uint8_t* const* nset, double* const* xc, int* const* npref);
// Windows without mask: origin counts by sliding column sums into kpref
// (before launch_shape_origins), weights by sliding column sums (instead of
// launch_shape_weights).  Items: instance x chunk of 256 columns.
void launch_shape_vcount(int nitems, hipStream_t st, const OpDesc* ops, const Item* items, const int* const* npref,
                         int* const* kpref);
void launch_shape_weights_v(int nitems, hipStream_t st, const OpDesc* ops, const Item* items,
                            const int* const* kpref, double* const* W);
void launch_shape_origins(int nitems, hipStream_t st, const OpDesc* ops, const Item* items, const Runs* runs,
                          const int* const* npref, uint8_t* const* kmask, int* const* kpref, int* const* kcount);
void launch_shape_rowoff(int ninst, hipStream_t st, const int* const* kcount, int* const* rowoff, const int* nrows,
                         long* total);
void launch_shape_weights(int nitems, hipStream_t st, const OpDesc* ops, const Item* items, const Runs* runs,
                          const int* const* kpref, double* const* W);
void launch_lz_start(int nitems, hipStream_t st, const LzDesc* lzs, const Item* items, unsigned long long seed);
void launch_lz_proj(int nitems, hipStream_t st, const LzDesc* lzs, const Item* items, int ncols);
void launch_lz_update(int nitems, hipStream_t st, const LzDesc* lzs, const Item* items, int ncols, int pass,
                      int force);
void launch_lz_proj2(int nitems, hipStream_t st, const LzDesc* lzs, const Item* items, int ncols, int force);
void launch_lz_normalize(int nitems, hipStream_t st, const LzDesc* lzs, const Item* items, int m);
void launch_lz_svd(int ninst, hipStream_t st, const LzDesc* lzs, const Item* items, int m, int max_sweeps);
void launch_lz_ritz(int nitems, hipStream_t st, const LzDesc* lzs, const Item* items, int m, int k,
                    double* const* outs);
void launch_lz_restart(int nitems, hipStream_t st, const LzDesc* lzs, const Item* items, int m, int k);
void launch_lz_restart_random(int nitems, hipStream_t st, const LzDesc* lzs, const Item* items, int k,
                              unsigned long long seed);
void launch_lz_sigma(int ninst, hipStream_t st, const LzDesc* lzs, const ResDesc* res, const Item* items);
void launch_sign_fix(int nitems, hipStream_t st, const OpDesc* ops, const ResDesc* res, const Item* items,
                     int with_v);
void launch_gather_flags(int ninst, hipStream_t st, const LzDesc* lzs, int* flags, double* betas);
// Per-instance step counters ([j, jstart] at each listed instance's
// LzDesc::step): set them, or advance j by one.
void launch_step_set(int nitems, hipStream_t st, const LzDesc* lzs, const Item* items, int j, int js);
void launch_step_next_inst(int nitems, hipStream_t st, const LzDesc* lzs, const Item* items);
void launch_step_next(hipStream_t st, int* step);
// Weighted Gram of narr arrays of ncell values over the cells with W > 0:
// 16 x 16 tiles of the upper triangle (wgram_tiles of them), entry
// (16 ib + i, 16 jb + j) of tile t at out[256 t + 16 i + j]; part holds
// tiles*256*nchunk values.
int wgram_tiles(int narr);
// Column recurrent forecast: LRR R (L-1) from the group's U columns (flag[0]
// = 1 if undefined), then h values per row of rec (A x B) into out (A x h);
// buf holds A * (L-1+h) values.
void launch_rforecast(hipStream_t st, const double* U, long L, const int* grp, int ng, double* R, int* flag,
                      const double* rec, const double* W, int A, int B, int h, double* buf, double* out);
// Column vector forecast: shift matrix M (ng x ng) of the group's U columns,
// then h values per row into out (A x h); wbuf holds A * (h+L-1) * ng
// values; flag[0..1] (zeroed by the caller) report rows or a group without
// a forecast.  ng <= kVfMaxGroup.
void launch_vforecast(hipStream_t st, const double* U, long L, const double* V, long K, const double* sigma,
                      const int* grp, int ng, double* M, const int* krow, const uint8_t* kmask, int KB,
                      const double* W, int A, int B, int h, double* wbuf, double* out, int* flag);
// Row forecasts (the group's V blocks by series, A series): structure
// check (flag[0]: an origin row that is not a prefix), Gram terms Mr and
// StS (ng x ng), and D = (I - StS)^{-1} Mr, G = (I - StS)^{-1} (flag[1]:
// singular); T holds 3 ng^2 values.  flag zeroed by the caller.
void launch_rowf_prep(hipStream_t st, const uint8_t* kmask, int KB, const int* krow, int A, const double* V, long K,
                      const int* grp, int ng, double* Mr, double* StS, double* T, double* D, double* G, int* flag);
// Vector row forecast: E coefficient vectors (wbuf, E x ng, E = h + KB - 1)
// then h values per series into out (A x h).
void launch_vrow(hipStream_t st, const double* U, long L, const double* sigma, const int* grp, int ng,
                 const double* D, long E, double* wbuf, const double* V, long K, const int* krow, int A, int h,
                 double* out);
// Recurrent row forecast from the group's reconstruction rec (A x B): yk
// (h x ng) then h values per series into out (A x h).
void launch_rrow(hipStream_t st, const double* V, long K, const int* krow, int A, const int* grp, int ng,
                 const double* G, const double* rec, int B, long L, int h, double* yk, double* out);
// Eigen method: S = X X^T (L x L, L <= kMaxBasis) into Bm from the cleaned
// grid xc and the window-cell and origin offsets; part holds
// ntile * 256 * nchunk values and out ntile * 256, ntile = nb (nb + 1) / 2,
// nb = ceil(L / 16).  Then U and sigma of the r leading eigenpairs from the
// small SVD's output.
void launch_xgram(hipStream_t st, const double* xc, const int* offL, int L, const int* offK, long K, int nchunk,
                  double* part, double* out, double* Bm, long ld);
// One round of the block Jacobi eigensolver on the L x L column-major A:
// npairs disjoint block pairs (block indices, -1 = empty block), their
// rotations in J (npairs x kBjN^2); flag[0] set if a pair was not yet
// orthogonal to tol (entries below floor_abs count as orthogonal), flag[1]
// if an inner iteration ran out of sweeps.
void launch_bj_round(hipStream_t st, double* A, int L, const int2* pairs, int npairs, double* J, int* flag,
                     double tol, double floor_abs);
// lam[c] = |column c of A|.
void launch_bj_norms(hipStream_t st, const double* A, int L, double* lam);
// U (L x r) = columns perm[0..r) of A / lam, sigma = sqrt(lam[perm]).
void launch_bj_take(hipStream_t st, const double* A, int L, const int* perm, const double* lam, double* U,
                    double* sigma, int r);
void launch_eig_take(int nitems, hipStream_t st, const LzDesc* lzs, const ResDesc* res, const Item* items, int L,
                     int r);
// p[0..n) = v on stream st.
void launch_fill_i32(hipStream_t st, int* p, int n, int v);
// LS-ESPRIT roots (ng <= kVfMaxGroup) into re/im; M holds ng^2 values;
// flag[0..1] (zeroed by the caller) as for k_esprit.
void launch_esprit(hipStream_t st, const double* U, long L, const int* grp, int ng, double* M, double* re,
                   double* im, int* flag);
// TLS-ESPRIT roots (ng <= kTlsMaxGroup) into re/im; g holds 4 ng^2 values;
// flag[0] (V22 singular) and flag[1] (no convergence), zeroed by the caller.
void launch_esprit_tls(hipStream_t st, const double* U, long L, const int* grp, int ng, double* g, double* re,
                       double* im, int* flag);
// 2D-ESPRIT: for each axis the Gram terms over the index pairs (pa[2 ax],
// pb[2 ax]: cells and their neighbour; pa/pb[2 ax + 1]: the cells without
// one, with themselves) give phi_ax = (I - S^T S)^{-1} M; then the joint
// eigenvalues into out (lambda re, lambda im, mu re, mu im; ng each).
// gram: 2 ng^2, T: 3 ng^2, phi: 2 ng^2, G: ng^2, scr: 3 ng^2 + 14 ng values;
// flag[1]: singular system, flag[2]: eigenvalue iteration failed.
void launch_esprit2d(hipStream_t st, const double* U, long L, const int* grp, int ng, const int* const* pa,
                     const int* const* pb, const int* np, double* gram, double* T, double* phi, double* G,
                     double gamma, double* scr, double* out, int* flag);
void launch_wgram(hipStream_t st, const double* const* arr, int narr, const double* W, long ncell, int nchunk,
                  double* part, double* out);
void launch_transpose(int nmat, int R, int C, hipStream_t st, const double* in, double* out);
// Device-to-device copies of a batch call's inputs in one launch: job i
// copies bytes from src to dst (device pointers, non-overlapping).  jobs is a
// device array of njobs entries, njobs <= 65535; max_bytes bounds the jobs'
// sizes (it sets the grid).
struct CopyJob {
    const void* src;
    void* dst;
    long bytes;
};
void launch_copy_jobs(hipStream_t st, const CopyJob* jobs, int njobs, long max_bytes);

}  // namespace shssa
