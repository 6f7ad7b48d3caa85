// Device kernels of the Shaped 2D-SSA path (gfx950).
//
// Products with the trajectory matrix follow the implementation section of
// the paper (quasi-Hankel matrix-vector product, Algorithm 3, and its 1D
// special case, Algorithm 1): the input vector is placed on its index set
// inside a zero grid, transformed, multiplied pointwise by the conjugate of
// the input vector's spectrum against the image spectrum, transformed back,
// and read out on the other index set.  X v reads the origin set K and
// writes the window set L; X^T u does the reverse with the same kernels.
//
// Reconstruction follows Algorithms 4 and 5 (quasi-hankelization through
// diagsums): the product of the spectra of U_i (on L) and sigma_i V_i (on K),
// summed over the group in the frequency domain, transformed back once and
// divided by the weights; cells with zero weight are not covered.
//
// Shapes follow Algorithm 6: an origin belongs to K when every window cell
// placed there lands on a cell of N.  The window count is taken by exact
// integer run sums over row prefix counts instead of a rounded FFT product.
#include <type_traits>

#include "common.hpp"
#include "device.hpp"
#include "fft.hpp"
#include "regfft.hpp"
#include "hqr.hpp"

namespace shssa {

// ------------------------------------------------------------------------
// helpers
// ------------------------------------------------------------------------

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// Moves x from another lane of its row by the data-parallel-primitive
// control CTRL (two 32-bit moves for the double's halves).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, x);
    const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, (static_cast<unsigned long long>(static_cast<unsigned>(hi)) << 32) |
                                          static_cast<unsigned>(lo));
}

// Sum over each aligned group of 8 lanes: add lane ^ 1 (quad_perm 1,0,3,2),
// then lane ^ 2 (quad_perm 2,3,0,1), then the mirrored lane 7 - i of the
// half-row.  Each step adds the same two operands in every lane of a group
// (addition commutes exactly), so all 8 lanes end with the same bits.
__device__ __forceinline__ double group8_sum(double v) {
    v += dpp_f64<0xB1>(v);
    v += dpp_f64<0x4E>(v);
    v += dpp_f64<0x141>(v);
    return v;
}


// Visits the cells b = tid + c*G (c < CH, b < len) of set row a, in blocks
// of up to 8 cells per thread: first every compact index of the block (from
// the row offset and the row's prefix counts, no serial scan) and every load
// ld(idx) are issued, then st(b, idx, value) runs for each b < len (idx = -1
// off the set).  Issuing the loads before any store lets them overlap.
template <typename V, int G, int CH, typename LD, typename ST>
__device__ __forceinline__ void row_visit(const CellSet& S, int a, int len, int tid, LD ld, ST st) {
    constexpr int CB = CH < 8 ? CH : 8;
    const bool inrow = a < S.boxA;
    const int base = inrow ? S.rowoff[a] : 0;
    const uint8_t* m = (inrow && S.mask) ? S.mask + (long)a * S.boxB : nullptr;
    const int* pf = (inrow && S.mask) ? S.pref + (long)a * (S.boxB + 1) : nullptr;
    const int lim = inrow ? (len < S.boxB ? len : S.boxB) : 0;
    for (int c0 = 0; c0 < CH; c0 += CB) {
        if (tid + c0 * G >= len) break;
        int idx[CB];
        V val[CB];
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            const int b = tid + (c0 + c) * G;
            int v = -1;
            if (c0 + c < CH && b < lim) {
                if (!m) v = base + b;
                else if (m[b]) v = base + pf[b];
            }
            idx[c] = v;
        }
#pragma unroll
        for (int c = 0; c < CB; ++c) val[c] = idx[c] >= 0 ? ld(idx[c]) : V(0);
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            const int b = tid + (c0 + c) * G;
            if (c0 + c < CH && b < len) st(b, idx[c], val[c]);
        }
    }
}

// Workgroups are dispatched to the 8 XCDs round-robin in launch order, and
// each XCD has its own L2.  xcd_block maps launch index b to a work index so
// that every XCD receives one contiguous range of work items: neighbouring
// items (which share cache lines) then meet in the same L2.  A bijection on
// [0, nb).
__device__ __forceinline__ int xcd_block(int b, int nb) {
    constexpr int kXcd = 8;
    const int x = b % kXcd, k = b / kXcd;
    const int q = nb / kXcd, rem = nb % kXcd;
    return (x < rem ? x * (q + 1) : rem * (q + 1) + (x - rem) * q) + k;
}

template <typename T> __device__ __forceinline__ T to(double v) { return static_cast<T>(v); }

// Sum of v over the G threads of a slot.  G == 64: one wave; otherwise the
// slot is the whole workgroup and the waves combine through LDS.  Every
// thread of the workgroup must call it; all threads get the total.
template <int G>
__device__ __forceinline__ double slot_sum(double v, double* red) {
    v = wave_sum(v);
    if constexpr (G == 64) {
        return v;
    } else {
        const int wv = (threadIdx.x % G) >> 6;
        __syncthreads();
        if (lane_id() == 0) red[wv] = v;
        __syncthreads();
        double t = 0.0;
        for (int q = 0; q < G / 64; ++q) t += red[q];
        return t;
    }
}

// Sum of n partials p[0..n) by one wave: lane l adds p[l], p[l+64], ...,
// then the lanes combine.  Every lane of every wave gets the same total
// (the order is fixed, so the result does not depend on the caller).
// The loads go out eight at a time (clamped addresses, unconditional), then
// are added in the same order, so that a long list costs one memory round
// trip per 512 partials instead of one per 64.
__device__ __forceinline__ double sum_parts(const double* p, int n) {
    const gptr<const double> g = as_global(p);
    const int l = lane_id();
    double s = 0.0;
    for (int q0 = 0; q0 < n; q0 += 512) {
        double v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int q = q0 + l + 64 * k;
            v[k] = gload(g + (q < n ? q : 0));
        }
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (q0 + l + 64 * k < n) s += v[k];
    }
    return wave_sum(s);
}

// sum_parts of three lists at once (a: na partials; b0, b1: nb each), their
// loads issued together: one memory round trip where three calls would take
// three.  Each sum is formed in sum_parts' order (the same value).
struct Sums3 {
    double a, b0, b1;
};
__device__ __forceinline__ Sums3 sum_parts3(const double* pa, int na, const double* pb0, const double* pb1,
                                            int nb) {
    const gptr<const double> ga = as_global(pa), g0 = as_global(pb0), g1 = as_global(pb1);
    const int l = lane_id();
    double sa = 0.0, s0 = 0.0, s1 = 0.0;
    const int n = na > nb ? na : nb;
    for (int q0 = 0; q0 < n; q0 += 512) {
        double va[8], v0[8], v1[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int q = q0 + l + 64 * k;
            va[k] = gload(ga + (q < na ? q : 0));
            v0[k] = gload(g0 + (q < nb ? q : 0));
            v1[k] = gload(g1 + (q < nb ? q : 0));
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int q = q0 + l + 64 * k;
            if (q < na) sa += va[k];
            if (q < nb) {
                s0 += v0[k];
                s1 += v1[k];
            }
        }
    }
    return {wave_sum(sa), wave_sum(s0), wave_sum(s1)};
}

// Twiddle tables of a transform staged in LDS (one copy per workgroup,
// shared by its slots), so the butterflies read them from LDS instead of
// global memory.  Only for the smaller size classes; every thread of the
// workgroup must call this.
template <typename T, int NMAX, bool REAL>
struct TwStage {
    static constexpr bool kOn = kTwStaged<NMAX>;   // the LDS transforms read staged tables as LDS
    static constexpr int kSize = kOn ? (REAL ? 2 * NMAX + 1 : NMAX) : 1;
};

// Twiddle pointers of a plan, staged in LDS when the size class allows.
template <typename T>
struct Tw {
    const cplx<T>* tw;
    const cplx<T>* twr;
};

template <typename T, int NMAX, bool REAL>
__device__ __forceinline__ Tw<T> stage_twiddles(const FftPlan& g, cplx<T>* twl) {
    Tw<T> t{static_cast<const cplx<T>*>(g.tw), static_cast<const cplx<T>*>(g.twr)};
    if constexpr (TwStage<T, NMAX, REAL>::kOn) {
        const int n = g.n;
        for (int i = threadIdx.x; i < n; i += blockDim.x) twl[i] = t.tw[i];
        if constexpr (REAL) {
            for (int i = threadIdx.x; i <= n; i += blockDim.x) twl[NMAX + i] = t.twr[i];
            t.twr = twl + NMAX;
        }
        t.tw = twl;
        __syncthreads();
    }
    return t;
}

// ------------------------------------------------------------------------
// row kernels
// ------------------------------------------------------------------------



// Source of a row-input pass: the compact vector read (src), its scale and
// the basis column that receives the scaled vector (qout, or nullptr).
struct RowInSrc {
    const double* src;
    double sc;
    double* qout;
    float* qout32;   // the FP32 copy of the basis column (or nullptr)
};

__device__ __forceinline__ RowInSrc row_in_source(const OpDesc& op, const LzDesc& lz, const ResDesc* res,
                                                  const Item& item, const RowInArgs& a0, bool leader) {
    RowInSrc r{nullptr, 1.0, nullptr, nullptr};
    RowInArgs args = a0;
    if (args.mode == IN_LZ_NORM || args.mode == IN_LZ_PLAIN || args.mode == IN_LZ_SIN ||
        args.mode == IN_LZ_STEP) {
        // Everything the step may need is loaded first, together, in
        // straight-line code: the descriptor's fields (one scalar round
        // trip), then the step counter, flags, scales and partial sums (one
        // vector round trip).  The choices below depend on the loaded step
        // counter; loads made after them would each wait for the previous
        // one.  Without a batch step counter the counter's loads read the
        // flags instead (always allocated) and are not used.
        const bool stepm = args.mode == IN_LZ_STEP;
        const int* sp = stepm ? lz.step : lz.flag;
        const gptr<const int> fl = as_global(static_cast<const int*>(lz.flag));
        const gptr<const double> bt = as_global(static_cast<const double*>(lz.beta));
        const bool gam_item = (stepm || args.mode == IN_LZ_NORM) && item.idx == 0;
        const int nw = args.mode != IN_LZ_PLAIN ? lz.nblk : 0;
        const int nl = gam_item ? op.S[1 - args.set].boxA : 0;
        const double* np = lz.np;
        const double* lnp0 = lz.lnp[0];
        const double* lnp1 = lz.lnp[1];
        const int s0 = gload(as_global(sp)), s1 = gload(as_global(sp) + 1);
        const int f2 = gload(fl + 2), f3 = gload(fl + 3);
        const double b2 = gload(bt + 2), b3 = gload(bt + 3);
        // |w|^2 for beta_{j-1} and, for gamma_j (below), |l_{j-1}|^2 of both
        // parities (the parity is known only with the step)
        const Sums3 sums = sum_parts3(np, nw, lnp0, lnp1, nl);
        int js = 0;
        if (stepm) {
            args.j = s0;
            js = s1;
        }
        const double beta = sqrt(sums.a);
        const double al0 = sums.b0, al1 = sums.b1;
        if (args.mode == IN_LZ_STEP) args.mode = (args.j == js && js > 0) ? IN_LZ_SIN : IN_LZ_NORM;
        const bool fresh = args.mode == IN_LZ_SIN && f3 != 0;
        if (args.mode == IN_LZ_NORM || fresh) {
            // q_j = w / beta_{j-1}.  A beta at rounding level (the short
            // Krylov space is exhausted) freezes the recurrence for the rest
            // of the cycle: q_j = 0 and B[j][j-1] = 0.  After a fresh random
            // restart w is a random vector orthogonal to the basis and has
            // no coupling to the previous column.
            const double scale = ((args.j - 1) & 1) ? b3 : b2;
            const bool bd = !fresh && (f2 != 0 || (args.j > 0 && beta <= lz.eps * scale));
            r.sc = (!bd && beta > 1e-300) ? 1.0 / beta : 0.0;
            r.src = lz.w;
            r.qout = lz.Q + (long)args.j * lz.n;
            r.qout32 = lz.Q32 ? lz.Q32 + (long)args.j * lz.n : nullptr;
            if (leader) {
                if (args.j > 0 && !fresh) lz.Bm[(long)(args.j - 1) * kMaxBasis + args.j] = bd ? 0.0 : beta;
                if (bd) lz.flag[2] = 1;
            }
            // gamma_j of this step's long update (beta_{j-1} / alpha_{j-1}),
            // formed once here by the work item holding set row 0 instead of
            // by every work item of the long-side pass.  The first step of a
            // cycle has none.
            if (args.mode == IN_LZ_NORM && item.idx == 0 && args.j > 0) {
                const int p = args.j & 1;
                const double alpha = sqrt(p ? al0 : al1);   // lnp[p ^ 1]
                const double gm = (!bd && alpha > 1e-300) ? beta / alpha : 0.0;
                if (leader) lz.gam[p] = gm;
            }
        } else if (args.mode == IN_LZ_SIN) {
            r.src = lz.sin;
        } else {
            r.src = lz.Q + (long)args.j * lz.n;
        }
    } else {
        const ResDesc& rs = res[item.inst];
        const long ld = args.set == 0 ? op.S[0].count : op.S[1].count;
        r.src = (args.set == 0 ? rs.U : rs.V) + (long)item.comp * ld;
        r.sc = args.scale * (args.use_sigma ? rs.sigma[item.comp] : 1.0);
    }
    return r;
}

template <typename T, int NMAX, int G, int SLOTS, bool P2>
__global__ void __launch_bounds__(G * SLOTS)
k_row_in(const OpDesc* __restrict__ ops, const LzDesc* __restrict__ lzs, const ResDesc* __restrict__ res,
         const Item* __restrict__ items, int nitems, RowInArgs args) {
    __shared__ cplx<T> buf[SLOTS][NMAX + 1];
    __shared__ cplx<T> twl[TwStage<T, NMAX, true>::kSize];
    const int slot = threadIdx.x / G, tid = threadIdx.x % G;
    const int it = blockIdx.x * SLOTS + slot;
    const Item item = items[it < nitems ? it : nitems - 1];
    const bool valid = it < nitems && item.aux >= 0;   // aux < 0: padding slot (no writes)
    const OpDesc& op = ops[item.inst];
    const FftPlan& prow = op.prow;
    const Tw<T> tw = stage_twiddles<T, NMAX, true>(prow, twl);
    const LzDesc& lz = lzs[item.inst];
    cplx<T>* s = buf[slot];
    T* sr = reinterpret_cast<T*>(s);
    const int a = item.idx;
    const int MB = op.MB;

    if (args.mode == IN_DENSE) {
        const double* row = op.xc + (long)a * op.B;
        for (int b = tid; b < MB; b += G) sr[b] = b < op.B ? to<T>(row[b]) : T(0);
    } else {
        const CellSet& S = op.S[args.set];
        const RowInSrc rsrc = row_in_source(op, lz, res, item, args, valid && a == 0 && tid == 0);
        const double* src = rsrc.src;
        const double sc = rsrc.sc;
        double* qout = rsrc.qout;
        float* q32 = rsrc.qout32;
        const bool wr = valid && qout != nullptr;
        row_visit<double, G, cdiv(2 * NMAX, G)>(
            S, a, MB, tid, [&](int i) { return src[i] * sc; },
            [&](int b, int i, double v) {
                if (wr && i >= 0) {
                    qout[i] = v;
                    if (q32) q32[i] = static_cast<float>(v);
                }
                sr[b] = to<T>(v);
            });
    }
    __syncthreads();
    rfft_fwd<T, NMAX, G, P2>(s, prow, tw.tw, tw.twr, tid);
    if (!valid) return;
    const int n1 = prow.n + 1;
    cplx<T>* out;
    if (args.dest == DEST_T1) {
        out = static_cast<cplx<T>*>(op.T1) + item.comp * op.tslot + (long)a * op.ldp;
        for (int f = tid; f < n1; f += G) out[f] = s[f];
    } else {
        out = static_cast<cplx<T>*>(const_cast<void*>(op.Xh)) + (long)a * op.ldp;
        const T scl = to<T>(args.scale < 0 ? op.spec_scale : args.scale);
        for (int f = tid; f < n1; f += G) out[f] = {s[f].x * scl, s[f].y * scl};
    }
}



// Long-vector update of step j inside the row pass: gamma = beta_{j-1} /
// alpha_{j-1} (formed by the step's input pass; 0 on the first step of a
// cycle), lcur/lprev by parity.
template <typename T>
struct GkLong {
    T* lcur;
    const T* lprev;
    double* lnp;
    T gamma;
};

template <typename T>
__device__ __forceinline__ GkLong<T> gk_long(const LzDesc& lz, int j, int jstart) {
    // straight-line loads (both parities' gamma with the step counter; the
    // counter's loads read gam when there is no counter and go unused)
    const bool stepm = j == kStepDev;
    const int* sp = stepm ? lz.step : reinterpret_cast<const int*>(lz.gam);
    const gptr<const double> gp = as_global(static_cast<const double*>(lz.gam));
    const int s0 = gload(as_global(sp)), s1 = gload(as_global(sp) + 1);
    const double gm0 = gload(gp), gm1 = gload(gp + 1);
    if (stepm) {
        j = s0;
        jstart = s1;
    }
    GkLong<T> g;
    const int p = j & 1;
    g.lcur = static_cast<T*>(lz.lbuf[p]);
    g.lprev = static_cast<const T*>(lz.lbuf[p ^ 1]);
    g.lnp = lz.lnp[p];
    // gamma_j was formed by this step's input pass (0 on the first step of
    // a cycle and after a breakdown)
    const double gm = j != jstart ? (p ? gm1 : gm0) : 0.0;
    g.gamma = static_cast<T>(gm);
    return g;
}

// C2R of T2 row a, mask to a set row, optional emission, R2C into T1 row a.
template <typename T, int NMAX, int G, int SLOTS, bool P2>
__global__ void __launch_bounds__(G * SLOTS)
k_row_mid(const OpDesc* __restrict__ ops, const LzDesc* __restrict__ lzs, const ResDesc* __restrict__ res,
          const Item* __restrict__ items, int nitems, RowMidArgs args) {
    __shared__ cplx<T> buf[SLOTS][NMAX + 1];
    __shared__ cplx<T> twl[TwStage<T, NMAX, true>::kSize];
    __shared__ double red[16];
    const int slot = threadIdx.x / G, tid = threadIdx.x % G;
    const int it = blockIdx.x * SLOTS + slot;
    const Item item = items[it < nitems ? it : nitems - 1];
    const bool valid = it < nitems && item.aux >= 0;   // aux < 0: padding slot (no writes)
    const OpDesc& op = ops[item.inst];
    const FftPlan& prow = op.prow;
    const Tw<T> tw = stage_twiddles<T, NMAX, true>(prow, twl);
    cplx<T>* s = buf[slot];
    T* sr = reinterpret_cast<T*>(s);
    const int a = item.idx;
    const int n1 = prow.n + 1;
    const cplx<T>* in = static_cast<const cplx<T>*>(op.T2) + item.comp * op.tslot + (long)a * op.ldp;
    for (int f = tid; f < n1; f += G) s[f] = in[f];
    __syncthreads();
    rfft_inv<T, NMAX, G, P2>(s, prow, tw.tw, tw.twr, tid);
    const CellSet& S = op.S[args.set];
    double* vout = nullptr;
    double sc = args.scale;
    if (args.emit == OUT_VEC && valid) {
        const ResDesc& rs = res[item.inst];
        vout = (args.set == 0 ? rs.U : rs.V) + (long)item.comp * S.count;
        if (args.div_sigma) sc = rs.sigma[item.comp] > 0 ? sc / rs.sigma[item.comp] : 0.0;
    }
    if (args.gk) {
        const GkLong<T> g = gk_long<T>(lzs[item.inst], args.j, args.jstart);
        double part = 0.0;
        row_visit<T, G, cdiv(2 * NMAX, G)>(
            S, a, op.MB, tid, [&](int i) { return g.lprev[i]; },
            [&](int b, int i, T p) {
                T v = T(0);
                if (i >= 0) {
                    v = sr[b] - g.gamma * p;
                    if (valid) g.lcur[i] = v;
                    part += static_cast<double>(v) * static_cast<double>(v);
                }
                sr[b] = v;
            });
        part = slot_sum<G>(part, red);
        if (valid && tid == 0) g.lnp[a] = part;
    } else {
        row_visit<T, G, cdiv(2 * NMAX, G)>(
            S, a, op.MB, tid, [&](int) { return T(0); },
            [&](int b, int i, T) {
                T v = sr[b];
                if (i < 0) v = T(0);
                else if (vout) vout[i] = sc * static_cast<double>(v);
                sr[b] = v;
            });
    }
    if (!args.fwd) return;
    __syncthreads();
    rfft_fwd<T, NMAX, G, P2>(s, prow, tw.tw, tw.twr, tid);
    if (!valid) return;
    cplx<T>* out = static_cast<cplx<T>*>(op.T1) + item.comp * op.tslot + (long)a * op.ldp;
    for (int f = tid; f < n1; f += G) out[f] = s[f];
}


// w = (X l'_j) / alpha_j - alpha_j q_j with alpha_j = |l'_j|; B[j][j] = alpha_j.
struct GkShort {
    double inv_alpha, alpha;
    const double* q;
    double* w;
};

// An alpha at rounding level relative to the running scale (the long Krylov
// space is exhausted) freezes the recurrence: alpha = 0 and w = 0.
__device__ __forceinline__ GkShort gk_short(const LzDesc& lz, const CellSet& Slong, int j, int jstart,
                                            bool writer) {
    // straight-line loads: the step counter (read from the flags, unused,
    // when there is none), flag, both parities' scales and the partial sums
    // (both parities of |l|^2 and |w|^2) go out together
    const bool stepm = j == kStepDev;
    const int* sp = stepm ? lz.step : lz.flag;
    const gptr<const int> fl = as_global(static_cast<const int*>(lz.flag));
    const gptr<const double> bt = as_global(static_cast<const double*>(lz.beta));
    const int s0 = gload(as_global(sp)), s1 = gload(as_global(sp) + 1);
    const int f2 = gload(fl + 2);
    const double b2 = gload(bt + 2), b3 = gload(bt + 3);
    const Sums3 sm = sum_parts3(lz.np, lz.nblk, lz.lnp[0], lz.lnp[1], Slong.boxA);
    if (stepm) {
        j = s0;
        jstart = s1;
    }
    GkShort g;
    g.alpha = sqrt((j & 1) ? sm.b1 : sm.b0);
    const double prev = ((j - 1) & 1) ? b3 : b2;
    const double beta_in = (j > jstart) ? sqrt(sm.a) : 0.0;
    double scale = fmax(prev, beta_in);
    const bool bd = f2 != 0 || (j > 0 && g.alpha <= lz.eps * scale);
    if (bd) g.alpha = 0.0;
    g.inv_alpha = (!bd && g.alpha > 1e-300) ? 1.0 / g.alpha : 0.0;
    g.q = lz.Q + (long)j * lz.n;
    g.w = lz.w;
    if (writer) {
        lz.beta[2 + (j & 1)] = fmax(scale, g.alpha);
        lz.Bm[(long)j * kMaxBasis + j] = g.alpha;
        if (bd) lz.flag[2] = 1;
    }
    return g;
}

// C2R of T2 row a, gathered on a set row (compact output) or written dense.
template <typename T, int NMAX, int G, int SLOTS, bool P2>
__global__ void __launch_bounds__(G * SLOTS)
k_row_out(const OpDesc* __restrict__ ops, const LzDesc* __restrict__ lzs, const ResDesc* __restrict__ res,
          const Item* __restrict__ items, int nitems, RowOutArgs args) {
    __shared__ cplx<T> buf[SLOTS][NMAX + 1];
    __shared__ cplx<T> twl[TwStage<T, NMAX, true>::kSize];
    const int slot = threadIdx.x / G, tid = threadIdx.x % G;
    const int it = blockIdx.x * SLOTS + slot;
    const Item item = items[it < nitems ? it : nitems - 1];
    const bool valid = it < nitems && item.aux >= 0;   // aux < 0: padding slot (no writes)
    const OpDesc& op = ops[item.inst];
    const FftPlan& prow = op.prow;
    const Tw<T> tw = stage_twiddles<T, NMAX, true>(prow, twl);
    cplx<T>* s = buf[slot];
    T* sr = reinterpret_cast<T*>(s);
    const int a = item.idx;
    const int n1 = prow.n + 1;
    const cplx<T>* in = static_cast<const cplx<T>*>(op.T2) + item.comp * op.tslot + (long)a * op.ldp;
    for (int f = tid; f < n1; f += G) s[f] = in[f];
    __syncthreads();
    rfft_inv<T, NMAX, G, P2>(s, prow, tw.tw, tw.twr, tid);
    if (args.mode == OUT_IMAGE) {
        if (!valid) return;
        const double sc_img = args.scale < 0 ? op.spec_scale : args.scale;
        const ResDesc& rs = res[item.inst];
        double* out = rs.recon + (long)item.comp * op.A * op.B + (long)a * op.B;
        const double* W = op.W + (long)a * op.B;
        for (int b = tid; b < op.B; b += G) {
            const double w = W[b];
            out[b] = w > 0 ? sc_img * static_cast<double>(sr[b]) / w : __builtin_nan("");
        }
        return;
    }
    const CellSet& S = op.S[args.set];
    if (args.mode == OUT_LZ) {
        const LzDesc& lz = lzs[item.inst];
        const GkShort g = gk_short(lz, op.S[1 - args.set], args.j, args.jstart, valid && a == 0 && tid == 0);
        row_visit<double, G, cdiv(2 * NMAX, G)>(
            S, a, op.MB, tid, [&](int i) { return g.q[i]; },
            [&](int b, int i, double q) {
                if (valid && i >= 0) g.w[i] = static_cast<double>(sr[b]) * g.inv_alpha - g.alpha * q;
            });
        return;
    }
    const ResDesc& rs = res[item.inst];
    double* vout = (args.set == 0 ? rs.U : rs.V) + (long)item.comp * S.count;
    double sc = args.scale;
    if (args.div_sigma) sc /= rs.sigma[item.comp];
    row_visit<double, G, cdiv(2 * NMAX, G)>(
        S, a, op.MB, tid, [&](int) { return 0.0; },
        [&](int b, int i, double) {
            if (valid && i >= 0) vout[i] = sc * static_cast<double>(sr[b]);
        });
}

// ------------------------------------------------------------------------
// register row kernels: half-lengths n = 2^LOGN, 64 <= n <= 512
// ------------------------------------------------------------------------
// A workgroup of 256 threads takes RPW = 256/G consecutive rows of one
// instance (work item: instance, first row, component, row count), G = n/8
// consecutive lanes per row.  Thread t of a row holds the complex pairs
// z_p = (x_{2p}, x_{2p+1}) at positions p = t + G*e (e = 0..7) and, on the
// spectral side, the bins k = t + G*e (thread 0 also the bin n).

template <int LOGN>
struct RowReg {
    static constexpr int N = 1 << LOGN;
    static constexpr int G = N / 8;
    static constexpr int RPW = 256 / G;
    static_assert(LOGN >= 6 && LOGN <= 9, "register row kernels: n = 64..512");
};

// Sum over the G consecutive lanes of a row (G divides 64).  All lanes of
// the row get the same value.
template <int G>
__device__ __forceinline__ double lane_group_sum(double v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Z_k = E'_k + i O'_k for the thread's bins: E'_k = X_k + conj X_{n-k},
// O'_k = (X_k - conj X_{n-k}) conj(W^k), W = exp(-2 pi i/2n); the inverse
// complex transform of Z gives 2n x as pairs.  row: bins 0..n of the row.
// The loads (X_k and X_{n-k} of the thread's bins) are issued by
// row_unsplit_load and consumed by row_unsplit_finish, so that a kernel can
// keep them in flight while it stages its twiddle tables.
template <typename T, int LOGN>
__device__ __forceinline__ void row_unsplit_load(gptr<const cplx<T>> row, int t, cplx<T> (&X)[8], cplx<T> (&Y)[8]) {
    constexpr int N = RowReg<LOGN>::N, G = RowReg<LOGN>::G;
    const gptr<const cplx<T>> lo = row + t, hi = row + (N - t);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        X[e] = gload(lo + G * e);
        Y[e] = gload(hi - G * e);
    }
}

template <typename T, int LOGN, typename WRF>
__device__ __forceinline__ void row_unsplit_finish(const cplx<T> (&X)[8], const cplx<T> (&Y)[8], WRF wr,
                                                   cplx<T> (&v)[8]) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const cplx<T> ep = {X[e].x + Y[e].x, X[e].y - Y[e].y};
        const cplx<T> d = {X[e].x - Y[e].x, X[e].y + Y[e].y};
        const cplx<T> o = cmulc(d, wr(e));
        v[e] = {ep.x - o.y, ep.y + o.x};
    }
}

// From Z = FFT(z) (natural positions in v) to the bins of the real
// transform: X_k = E_k + W^k O_k with E_k = (Z_k + conj Z_{n-k})/2,
// O_k = (Z_k - conj Z_{n-k})/(2i); X_n = E_0 - O_0.  Z_{n-k} comes from the
// partner thread through LDS.  Writes the thread's bins of row.
template <typename T, int LOGN, typename WRF, typename AD>
__device__ __forceinline__ void row_split_store(const cplx<T> (&v)[8], WRF wr, cplx<T>* lds, AD ad, int t,
                                                gptr<cplx<T>> row, bool write) {
    constexpr int N = RowReg<LOGN>::N, G = RowReg<LOGN>::G;
    constexpr int RS = G + G / 8;
    const int pw = rx_pad(t), pn = t ? rx_pad(G - t) : 0;
#pragma unroll
    for (int e = 0; e < 8; ++e) lds[ad(pw + e * RS)] = v[e];
    xsync<XS_WAVE>();
    // partner position (n - k) mod n: G (7 - e) + (G - t), or G ((8 - e) mod 8) for t = 0
    cplx<T> zn[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) zn[e] = lds[ad(t ? pn + (7 - e) * RS : ((8 - e) & 7) * RS)];
    if (!write) return;
    const gptr<cplx<T>> out = row + t;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const cplx<T> zk = v[e];
        const cplx<T> E = {T(0.5) * (zk.x + zn[e].x), T(0.5) * (zk.y - zn[e].y)};
        const cplx<T> O = {T(0.5) * (zk.y + zn[e].y), T(-0.5) * (zk.x - zn[e].x)};
        const cplx<T> wo = cmul(wr(e), O);
        gstore(out + G * e, cadd(E, wo));
        if (e == 0 && t == 0) gstore(row + N, csub(E, O));
    }
}

// Compact indices of the cells 2p + h (slot q = 2e + h, p = t + G*e) of set
// row a; -1 off the set or outside the set's box.  DENSE (no mask): the
// index is the row offset plus the cell, so accesses through it keep one
// per-thread address with immediate offsets.
// All loads are unconditional (clamped to valid addresses, results masked):
// a load under a lane condition becomes a branch with a wait of its own, and
// the loads of a row would no longer overlap.
template <int G, bool DENSE>
__device__ __forceinline__ void pair_idx(const CellSet& S, int a, int t, int (&idx)[16]) {
    const bool inrow = a < S.boxA;
    const int ar = inrow ? a : 0;
    const int base = gload(as_global(S.rowoff) + ar);
    const int lim = inrow ? S.boxB : 0;
    if constexpr (DENSE) {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int b = 2 * (t + G * (q >> 1)) + (q & 1);
            idx[q] = b < lim ? base + b : -1;
        }
    } else {
        // A masked row: cell b's index is the row offset plus the count of
        // set cells before b in the row.  The counts come from the row's
        // mask bytes by a scan across the row's G lanes (lane t holds cells
        // 2 (t + G e) + h: segment e of 2G cells lies in order across the
        // lanes), not from a stored prefix array: one byte per cell read
        // instead of five.
        const gptr<const uint8_t> m = as_global(S.mask) + (long)ar * S.boxB;
        int on[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int b = 2 * (t + G * (q >> 1)) + (q & 1);
            const int bb = b < S.boxB ? b : S.boxB - 1;
            const uint8_t mv = gload(m + bb);
            on[q] = (b < lim && mv) ? 1 : 0;
        }
        // the lane's counts of segments 0..3 and 4..7 in the bytes of two
        // words (at most 2 per lane, 2 G <= 128 per segment: no carry)
        unsigned lo = 0, hi = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            lo |= (unsigned)(on[2 * e] + on[2 * e + 1]) << (8 * e);
            hi |= (unsigned)(on[8 + 2 * e] + on[8 + 2 * e + 1]) << (8 * e);
        }
        unsigned slo = lo, shi = hi;   // inclusive scans over the row's lanes
#pragma unroll
        for (int d = 1; d < G; d <<= 1) {
            const unsigned ulo = __shfl_up(slo, d, G), uhi = __shfl_up(shi, d, G);
            if (t >= d) {
                slo += ulo;
                shi += uhi;
            }
        }
        const unsigned tlo = __shfl(slo, G - 1, G), thi = __shfl(shi, G - 1, G);   // segment totals
        const unsigned xlo = slo - lo, xhi = shi - hi;                            // exclusive
        int before = 0;   // set cells of the earlier segments
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const unsigned xs = e < 4 ? xlo : xhi, ts = e < 4 ? tlo : thi;
            const int sh = 8 * (e & 3);
            const int p0 = base + before + (int)((xs >> sh) & 0xffu);
            idx[2 * e] = on[2 * e] ? p0 : -1;
            idx[2 * e + 1] = on[2 * e + 1] ? p0 + on[2 * e] : -1;
            before += (int)((ts >> sh) & 0xffu);
        }
    }
}

// Unconditional load of p[i] (p[0] when i < 0), zero when i < 0.
template <typename V>
__device__ __forceinline__ V load_or_zero(gptr<const V> p, int i) {
    const V v = gload(p + (i >= 0 ? i : 0));
    return i >= 0 ? v : V(0);
}

// Runs body(std::true_type) for a set without mask, body(std::false_type)
// otherwise (the choice is uniform over the workgroup).
template <typename F>
__device__ __forceinline__ void dense_or_masked(const CellSet& S, F body) {
    if (S.mask == nullptr) body(std::true_type{});
    else body(std::false_type{});
}

template <typename T>
__device__ __forceinline__ T& pair_part(cplx<T>& z, int h) { return h ? z.y : z.x; }

// Twiddles of the register row kernels: the complex transform's (W) and the
// real split's (WR, w^k of length 2n at the thread's bins k = t + G e), both
// tables (2n values) staged once in LDS for the workgroup by stage() (which
// has a barrier).  Reading them from LDS at each use keeps them off the
// registers and off the global-load latency of every transform.
template <typename T, int LOGN>
struct RowTw {
    static constexpr int N = RowReg<LOGN>::N, G = RowReg<LOGN>::G;
    static constexpr int TW = TwTable<T, LOGN>::SIZE;   // complex transform's table
    static constexpr int LDS = TW + N + 1;               // LDS values (the last one a discard slot)
    // Staging runs in two halves: load() issues every global load of both
    // tables at once (the values wait in registers), store() writes them to
    // LDS and synchronises the workgroup (256 threads).  A kernel issues its
    // own first loads between the two, so that they and the table loads are
    // in flight together.
    static constexpr int K1 = (TW + 255) / 256, K2 = (N + 255) / 256;
    cplx<T>* tab;
    int t;
    cplx<T> r1[K1], r2[K2];
    __device__ __forceinline__ RowTw(cplx<T>* table, int tt) : tab(table), t(tt) {}
    __device__ __forceinline__ void load(const FftPlan& prow) {
        const gptr<const cplx<T>> tw = as_global(static_cast<const cplx<T>*>(prow.tw));
        const gptr<const cplx<T>> twr = as_global(static_cast<const cplx<T>*>(prow.twr));
#pragma unroll
        for (int k = 0; k < K1; ++k) {
            const int i = threadIdx.x + 256 * k;
            r1[k] = gload(tw + TwTable<T, LOGN>::src(i < TW ? i : 0));
        }
#pragma unroll
        for (int k = 0; k < K2; ++k) {
            const int i = threadIdx.x + 256 * k;
            r2[k] = gload(twr + (i < N ? i : 0));
        }
    }
    // Threads past a table's end write the discard slot (unconditional
    // stores: a store under a condition lets the compiler sink its load into
    // the branch, after the kernel's other loads).
    __device__ __forceinline__ void store() {
#pragma unroll
        for (int k = 0; k < K1; ++k) {
            const int i = threadIdx.x + 256 * k;
            tab[i < TW ? i : TW + N] = r1[k];
        }
#pragma unroll
        for (int k = 0; k < K2; ++k) {
            const int i = threadIdx.x + 256 * k;
            tab[i < N ? TW + i : TW + N] = r2[k];
        }
        __syncthreads();
    }
    __device__ __forceinline__ auto W() const {
        return [this](int q) -> cplx<T> { return TwTable<T, LOGN>{tab, t}(q); };
    }
    __device__ __forceinline__ auto WR() const {
        return [this](int e) -> cplx<T> { return tab[TW + t + G * e]; };
    }
};

template <typename T>
__device__ __forceinline__ gptr<cplx<T>> spec_row(void* base, long slot, int a, int ldp) {
    return as_global(static_cast<cplx<T>*>(base) + slot + (long)a * ldp);
}

// Row input (all modes but IN_DENSE): gather the compact vector on set row
// a into the pairs, R2C into T1 row a.
template <typename T, int LOGN>
__global__ void __launch_bounds__(256)
k_rowr_in(const OpDesc* __restrict__ ops, const LzDesc* __restrict__ lzs, const ResDesc* __restrict__ res,
          const Item* __restrict__ items, int nitems, RowInArgs args) {
    using RR = RowReg<LOGN>;
    constexpr int G = RR::G;
    constexpr int XB = RR::RPW * RegPlan<LOGN>::LROWS;
    __shared__ cplx<T> lds[XB + RowTw<T, LOGN>::LDS];
    const int c = threadIdx.x / G, t = threadIdx.x % G;
    const Item item = items[blockIdx.x];
    const bool valid = c < item.aux;
    const int a = item.idx + (valid ? c : 0);
    const OpDesc& op = ops[item.inst];
    RowTw<T, LOGN> tw(lds + XB, t);
    tw.load(op.prow);
    const auto ad = [&](int pp) { return rx_addr_row<LOGN>(pp, c); };
    int xe = 0;
    cplx<T> v[8];
    const CellSet& S = op.S[args.set];
    const RowInSrc rs = row_in_source(op, lzs[item.inst], res, item, args, valid && a == 0 && t == 0);
    const gptr<const double> src = as_global(rs.src);
    const gptr<double> qout = as_global(rs.qout);
    const gptr<float> q32 = as_global(rs.qout32);
    const bool wq = valid && rs.qout != nullptr;
    const bool wq32 = wq && rs.qout32 != nullptr;
    dense_or_masked(S, [&](auto dense) {
        int idx[16];
        pair_idx<G, decltype(dense)::value>(S, a, t, idx);
        double val[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) val[q] = load_or_zero(src, idx[q]);
        tw.store();   // the row's loads stay in flight across the barrier
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            val[q] *= rs.sc;
            if (wq && idx[q] >= 0) gstore(qout + idx[q], val[q]);
            if (wq32 && idx[q] >= 0) gstore(q32 + idx[q], static_cast<float>(val[q]));
            pair_part(v[q >> 1], q & 1) = to<T>(val[q]);
        }
    });
    reg_fft_tw<T, LOGN, -1, XS_WAVE>(v, tw.W(), lds, t, ad, xe);
    const gptr<cplx<T>> out = args.dest == DEST_T1 ? spec_row<T>(op.T1, item.comp * op.tslot, a, op.ldp)
                                                   : spec_row<T>(const_cast<void*>(op.Xh), 0, a, op.ldp);
    row_split_store<T, LOGN>(v, tw.WR(), lds, ad, t, out, valid);
}

// C2R of T2 row a, mask to a set row (with the long-vector update or the
// emission of a result vector), optional R2C into T1 row a.
template <typename T, int LOGN>
__global__ void __launch_bounds__(256)
k_rowr_mid(const OpDesc* __restrict__ ops, const LzDesc* __restrict__ lzs, const ResDesc* __restrict__ res,
           const Item* __restrict__ items, int nitems, RowMidArgs args) {
    using RR = RowReg<LOGN>;
    constexpr int G = RR::G;
    constexpr int XB = RR::RPW * RegPlan<LOGN>::LROWS;
    __shared__ cplx<T> lds[XB + RowTw<T, LOGN>::LDS];
    const int c = threadIdx.x / G, t = threadIdx.x % G;
    const Item item = items[blockIdx.x];
    const bool valid = c < item.aux;
    const int a = item.idx + (valid ? c : 0);
    const OpDesc& op = ops[item.inst];
    const auto ad = [&](int pp) { return rx_addr_row<LOGN>(pp, c); };
    int xe = 0;
    cplx<T> v[8];
    RowTw<T, LOGN> tw(lds + XB, t);
    tw.load(op.prow);
    {
        cplx<T> X[8], Y[8];
        row_unsplit_load<T, LOGN>(spec_row<T>(op.T2, item.comp * op.tslot, a, op.ldp), t, X, Y);
        tw.store();
        row_unsplit_finish<T, LOGN>(X, Y, tw.WR(), v);
        reg_fft_tw<T, LOGN, +1, XS_WAVE>(v, tw.W(), lds, t, ad, xe);
    }
    const CellSet& S = op.S[args.set];
    if (args.gk) {
        const GkLong<T> g = gk_long<T>(lzs[item.inst], args.j, args.jstart);
        const gptr<const T> lprev = as_global(g.lprev);
        const gptr<T> lcur = as_global(g.lcur);
        double part = 0.0;
        dense_or_masked(S, [&](auto dense) {
            int idx[16];
            pair_idx<G, decltype(dense)::value>(S, a, t, idx);
            T pv[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) pv[q] = load_or_zero(lprev, idx[q]);
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                T& z = pair_part(v[q >> 1], q & 1);
                T nv = T(0);
                if (idx[q] >= 0) {
                    nv = z - g.gamma * pv[q];
                    if (valid) gstore(lcur + idx[q], nv);
                    part += static_cast<double>(nv) * static_cast<double>(nv);
                }
                z = nv;
            }
        });
        part = lane_group_sum<G>(part);
        if (valid && t == 0) g.lnp[a] = part;
    } else {
        double* vout = nullptr;
        double sc = args.scale;
        if (args.emit == OUT_VEC && valid) {
            const ResDesc& rs = res[item.inst];
            vout = (args.set == 0 ? rs.U : rs.V) + (long)item.comp * S.count;
            if (args.div_sigma) sc = rs.sigma[item.comp] > 0 ? sc / rs.sigma[item.comp] : 0.0;
        }
        const gptr<double> vo = as_global(vout);
        dense_or_masked(S, [&](auto dense) {
            int idx[16];
            pair_idx<G, decltype(dense)::value>(S, a, t, idx);
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                T& z = pair_part(v[q >> 1], q & 1);
                if (idx[q] < 0) z = T(0);
                else if (vout) gstore(vo + idx[q], sc * static_cast<double>(z));
            }
        });
    }
    if (!args.fwd) return;
    reg_fft_tw<T, LOGN, -1, XS_WAVE>(v, tw.W(), lds, t, ad, xe);
    row_split_store<T, LOGN>(v, tw.WR(), lds, ad, t, spec_row<T>(op.T1, item.comp * op.tslot, a, op.ldp), valid);
}

// C2R of T2 row a gathered on a set row: the short-vector update (OUT_LZ)
// or a result vector (OUT_VEC).
template <typename T, int LOGN>
__global__ void __launch_bounds__(256)
k_rowr_out(const OpDesc* __restrict__ ops, const LzDesc* __restrict__ lzs, const ResDesc* __restrict__ res,
           const Item* __restrict__ items, int nitems, RowOutArgs args) {
    using RR = RowReg<LOGN>;
    constexpr int G = RR::G;
    constexpr int XB = RR::RPW * RegPlan<LOGN>::LROWS;
    __shared__ cplx<T> lds[XB + RowTw<T, LOGN>::LDS];
    const int c = threadIdx.x / G, t = threadIdx.x % G;
    const Item item = items[blockIdx.x];
    const bool valid = c < item.aux;
    const int a = item.idx + (valid ? c : 0);
    const OpDesc& op = ops[item.inst];
    const auto ad = [&](int pp) { return rx_addr_row<LOGN>(pp, c); };
    int xe = 0;
    cplx<T> v[8];
    RowTw<T, LOGN> tw(lds + XB, t);
    tw.load(op.prow);
    {
        cplx<T> X[8], Y[8];
        row_unsplit_load<T, LOGN>(spec_row<T>(op.T2, item.comp * op.tslot, a, op.ldp), t, X, Y);
        tw.store();
        row_unsplit_finish<T, LOGN>(X, Y, tw.WR(), v);
    }
    reg_fft_tw<T, LOGN, +1, XS_WAVE>(v, tw.W(), lds, t, ad, xe);
    const CellSet& S = op.S[args.set];
    if (args.mode == OUT_LZ) {
        const GkShort g = gk_short(lzs[item.inst], op.S[1 - args.set], args.j, args.jstart, valid && a == 0 && t == 0);
        const gptr<const double> qv = as_global(g.q);
        const gptr<double> wv = as_global(g.w);
        dense_or_masked(S, [&](auto dense) {
            int idx[16];
            pair_idx<G, decltype(dense)::value>(S, a, t, idx);
            double qq[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) qq[q] = load_or_zero(qv, idx[q]);
            if (!valid) return;
#pragma unroll
            for (int q = 0; q < 16; ++q)
                if (idx[q] >= 0)
                    gstore(wv + idx[q],
                           static_cast<double>(pair_part(v[q >> 1], q & 1)) * g.inv_alpha - g.alpha * qq[q]);
        });
        return;
    }
    if (!valid) return;
    const ResDesc& rs = res[item.inst];
    const gptr<double> vout = as_global((args.set == 0 ? rs.U : rs.V) + (long)item.comp * S.count);
    double sc = args.scale;
    if (args.div_sigma) sc /= rs.sigma[item.comp];
    dense_or_masked(S, [&](auto dense) {
        int idx[16];
        pair_idx<G, decltype(dense)::value>(S, a, t, idx);
#pragma unroll
        for (int q = 0; q < 16; ++q)
            if (idx[q] >= 0) gstore(vout + idx[q], sc * static_cast<double>(pair_part(v[q >> 1], q & 1)));
    });
}

// ------------------------------------------------------------------------
// row family (window one row high): the sum across rows is direct
// ------------------------------------------------------------------------


// Per (instance, row a, component): v = C2R(Xh_a conj(U^)), mask to the
// origin row a, then P_a = Xh_a conj(FFT(v)) into T2 slot comp row a.
// U^ is the spectrum of the window row in T1 slot comp row 0.
template <typename T, int NMAX, int G, int SLOTS, bool P2>
__global__ void __launch_bounds__(G * SLOTS)
k_rowfam_mid(const OpDesc* __restrict__ ops, const LzDesc* __restrict__ lzs, const ResDesc* __restrict__ res,
             const Item* __restrict__ items, int nitems, RowFamArgs args) {
    __shared__ cplx<T> buf[SLOTS][NMAX + 1];
    __shared__ cplx<T> twl[TwStage<T, NMAX, true>::kSize];
    __shared__ double red[16];
    const int slot = threadIdx.x / G, tid = threadIdx.x % G;
    const int it = blockIdx.x * SLOTS + slot;
    const Item item = items[it < nitems ? it : nitems - 1];
    const bool valid = it < nitems && item.aux >= 0;   // aux < 0: padding slot (no writes)
    const OpDesc& op = ops[item.inst];
    const FftPlan& prow = op.prow;
    const Tw<T> tw = stage_twiddles<T, NMAX, true>(prow, twl);
    cplx<T>* s = buf[slot];
    T* sr = reinterpret_cast<T*>(s);
    const int a = item.idx;
    const int n1 = prow.n + 1;
    const cplx<T>* uh = static_cast<const cplx<T>*>(op.T1) + item.comp * op.tslot;
    const cplx<T>* xh = static_cast<const cplx<T>*>(op.Xh) + (long)a * op.ldp;
    for (int f = tid; f < n1; f += G) s[f] = cmulc(xh[f], uh[f]);
    __syncthreads();
    rfft_inv<T, NMAX, G, P2>(s, prow, tw.tw, tw.twr, tid);
    const CellSet& S = op.S[1];
    double* vout = nullptr;
    double sc = 1.0;
    if (args.emit == OUT_VEC && valid) {
        const ResDesc& rs = res[item.inst];
        vout = rs.V + (long)item.comp * S.count;
        sc = rs.sigma[item.comp] > 0 ? 1.0 / rs.sigma[item.comp] : 0.0;
    }
    if (args.gk) {
        const GkLong<T> g = gk_long<T>(lzs[item.inst], args.j, args.jstart);
        double part = 0.0;
        row_visit<T, G, cdiv(2 * NMAX, G)>(
            S, a, op.MB, tid, [&](int i) { return g.lprev[i]; },
            [&](int b, int i, T p) {
                T v = T(0);
                if (i >= 0) {
                    v = sr[b] - g.gamma * p;
                    if (valid) g.lcur[i] = v;
                    part += static_cast<double>(v) * static_cast<double>(v);
                }
                sr[b] = v;
            });
        part = slot_sum<G>(part, red);
        if (valid && tid == 0) g.lnp[a] = part;
    } else {
        row_visit<T, G, cdiv(2 * NMAX, G)>(
            S, a, op.MB, tid, [&](int) { return T(0); },
            [&](int b, int i, T) {
                T v = sr[b];
                if (i < 0) v = T(0);
                else if (vout) vout[i] = sc * static_cast<double>(v);
                sr[b] = v;
            });
    }
    if (!args.full) return;
    __syncthreads();
    rfft_fwd<T, NMAX, G, P2>(s, prow, tw.tw, tw.twr, tid);
    if (!valid) return;
    cplx<T>* out = static_cast<cplx<T>*>(op.T2) + item.comp * op.tslot + (long)a * op.ldp;
    for (int f = tid; f < n1; f += G) out[f] = cmulc(xh[f], s[f]);
}

// Per (instance, component): sum_a P_a in row order, C2R, gather the window
// row into the Lanczos w (OUT_LZ) or a result vector.
template <typename T, int NMAX, int G, int SLOTS, bool P2>
__global__ void __launch_bounds__(G * SLOTS)
k_rowfam_out(const OpDesc* __restrict__ ops, const LzDesc* __restrict__ lzs,
             const Item* __restrict__ items, int nitems, RowOutArgs args) {
    __shared__ cplx<T> buf[SLOTS][NMAX + 1];
    __shared__ cplx<T> twl[TwStage<T, NMAX, true>::kSize];
    const int slot = threadIdx.x / G, tid = threadIdx.x % G;
    const int it = blockIdx.x * SLOTS + slot;
    const Item item = items[it < nitems ? it : nitems - 1];
    const bool valid = it < nitems && item.aux >= 0;   // aux < 0: padding slot (no writes)
    const OpDesc& op = ops[item.inst];
    const FftPlan& prow = op.prow;
    const Tw<T> tw = stage_twiddles<T, NMAX, true>(prow, twl);
    cplx<T>* s = buf[slot];
    T* sr = reinterpret_cast<T*>(s);
    const int n1 = prow.n + 1;
    const gptr<const cplx<T>> pa = as_global(static_cast<const cplx<T>*>(op.T2)) + item.comp * op.tslot;
    for (int f = tid; f < n1; f += G) {
        // eight rows' loads in flight at a time, added in row order
        cplx<T> acc = {T(0), T(0)};
        int a = 0;
        for (; a + 8 <= op.A; a += 8) {
            cplx<T> v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = gload(pa + (long)(a + u) * op.ldp + f);
#pragma unroll
            for (int u = 0; u < 8; ++u) acc = cadd(acc, v[u]);
        }
        for (; a < op.A; ++a) acc = cadd(acc, gload(pa + (long)a * op.ldp + f));
        s[f] = acc;
    }
    __syncthreads();
    rfft_inv<T, NMAX, G, P2>(s, prow, tw.tw, tw.twr, tid);
    const LzDesc& lz = lzs[item.inst];
    const GkShort g = gk_short(lz, op.S[1], args.j, args.jstart, valid && tid == 0);
    row_visit<double, G, cdiv(2 * NMAX, G)>(
        op.S[0], 0, op.MB, tid, [&](int i) { return g.q[i]; },
        [&](int b, int i, double q) {
            if (valid && i >= 0) g.w[i] = static_cast<double>(sr[b]) * g.inv_alpha - g.alpha * q;
        });
}

// Row-family reconstruction of group `comp` on row a: for each i in the
// group, FFT(sigma_i V_i row a) * U^_i summed, one C2R, divided by W.
template <typename T, int NMAX, int G, int SLOTS, bool P2>
__global__ void __launch_bounds__(G * SLOTS)
k_rowfam_recon(const OpDesc* __restrict__ ops, const ResDesc* __restrict__ res,
               const Item* __restrict__ items, int nitems, double scale) {
    __shared__ cplx<T> buf[SLOTS][NMAX + 1];
    __shared__ cplx<T> twl[TwStage<T, NMAX, true>::kSize];
    constexpr int PER = cdiv(NMAX + 1, G);
    const int slot = threadIdx.x / G, tid = threadIdx.x % G;
    const int it = blockIdx.x * SLOTS + slot;
    const Item item = items[it < nitems ? it : nitems - 1];
    const bool valid = it < nitems && item.aux >= 0;   // aux < 0: padding slot (no writes)
    const OpDesc& op = ops[item.inst];
    const FftPlan& prow = op.prow;
    const Tw<T> tw = stage_twiddles<T, NMAX, true>(prow, twl);
    const ResDesc& rs = res[item.inst];
    cplx<T>* s = buf[slot];
    T* sr = reinterpret_cast<T*>(s);
    const int a = item.idx;
    const int n1 = prow.n + 1;
    cplx<T> acc[PER];
#pragma unroll
    for (int p = 0; p < PER; ++p) acc[p] = {T(0), T(0)};
    const int g0 = rs.gptr[item.comp], g1 = rs.gptr[item.comp + 1];
    const CellSet& S = op.S[1];
    for (int g = g0; g < g1; ++g) {
        const int i = rs.gidx[g];
        const double* v = rs.V + (long)i * S.count;
        const double sg = rs.sigma[i];
        row_visit<double, G, cdiv(2 * NMAX, G)>(
            S, a, op.MB, tid, [&](int k) { return v[k]; },
            [&](int b, int k, double val) { sr[b] = k >= 0 ? to<T>(sg * val) : T(0); });
        __syncthreads();
        rfft_fwd<T, NMAX, G, P2>(s, prow, tw.tw, tw.twr, tid);
        const cplx<T>* uh = static_cast<const cplx<T>*>(op.Us) + (long)i * op.uslot;
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int f = tid + p * G;
            if (f < n1) acc[p] = cadd(acc[p], cmul(s[f], uh[f]));
        }
        __syncthreads();
    }
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int f = tid + p * G;
        if (f < n1) s[f] = acc[p];
    }
    __syncthreads();
    rfft_inv<T, NMAX, G, P2>(s, prow, tw.tw, tw.twr, tid);
    if (!valid) return;
    const double sc_img = scale < 0 ? op.spec_scale : scale;
    double* out = rs.recon + (long)item.comp * op.A * op.B + (long)a * op.B;
    const double* W = op.W + (long)a * op.B;
    for (int b = tid; b < op.B; b += G) {
        const double w = W[b];
        out[b] = w > 0 ? sc_img * static_cast<double>(sr[b]) / w : __builtin_nan("");
    }
}

// Copies the first-row spectra of U components (T1 slot i, row 0) into Us.
template <typename T>
__global__ void k_copy_uspec(const OpDesc* __restrict__ ops, const Item* __restrict__ items, int nitems) {
    const Item item = items[blockIdx.x];
    if (item.aux < 0) return;   // padding item
    const OpDesc& op = ops[item.inst];
    const cplx<T>* src = static_cast<const cplx<T>*>(op.T1) + item.comp * op.tslot;
    cplx<T>* dst = static_cast<cplx<T>*>(op.Us) + item.comp * op.uslot;
    for (int f = threadIdx.x; f < op.P; f += blockDim.x) dst[f] = src[f];
}

// ------------------------------------------------------------------------
// column kernel (grid family)
// ------------------------------------------------------------------------



// One workgroup transforms TC adjacent columns f0..f0+TC of a [rows][P]
// array; each column is an independent length-MA transform on G threads.
template <typename T, int NMAX, int G, int TC, bool P2, bool ACC>
__device__ __forceinline__ void
col_body(const OpDesc* __restrict__ ops, const ResDesc* __restrict__ res,
         const Item* __restrict__ items, int nitems, ColArgs args) {
    constexpr int LD = NMAX + 1;
    constexpr int PER = cdiv(NMAX * TC, G * TC);
    __shared__ cplx<T> buf[TC * LD];
    __shared__ cplx<T> twl[TwStage<T, NMAX, false>::kSize];
    const Item item = items[blockIdx.x];
    const OpDesc& op = ops[item.inst];
    const FftPlan& pcol = op.pcol;
    const Tw<T> tw = stage_twiddles<T, NMAX, false>(pcol, twl);
    const int f0 = item.idx * TC;
    const int MA = op.MA, P = op.P;
    const int nthr = G * TC;
    const int c = threadIdx.x / G, tid = threadIdx.x % G;
    cplx<T>* s = buf + c * LD;

    auto load_rows = [&](const cplx<T>* src, int nin) {
        // element e = a * TC + cc : consecutive threads take consecutive columns
        for (int e = threadIdx.x; e < MA * TC; e += nthr) {
            const int a = e / TC, cc = e % TC;
            const int f = f0 + cc;
            cplx<T> v = {T(0), T(0)};
            if (a < nin && f < P) v = src[(long)a * op.ldp + f];
            buf[cc * LD + a] = v;
        }
    };

    if constexpr (ACC) {
        const ResDesc& rs = res[item.inst];
        const int g0 = rs.gptr[item.comp], g1 = rs.gptr[item.comp + 1];
        cplx<T> acc[PER];
#pragma unroll
        for (int p = 0; p < PER; ++p) acc[p] = {T(0), T(0)};
        for (int g = g0; g < g1; ++g) {
            const int i = rs.gidx[g];
            load_rows(static_cast<const cplx<T>*>(op.T1) + i * op.tslot, col_rows(op, args.nin));
            __syncthreads();
            fft_lds<T, NMAX, G, -1, P2>(s, pcol, tw.tw, tid);
            const cplx<T>* uh = static_cast<const cplx<T>*>(op.Us) + (long)i * op.uslot;
#pragma unroll
            for (int p = 0; p < PER; ++p) {
                const int a = tid + p * G;
                const int f = f0 + c;
                if (a < MA && f < P) acc[p] = cadd(acc[p], cmul(s[a], uh[(long)f * MA + a]));
            }
            __syncthreads();
        }
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int a = tid + p * G;
            if (a < MA) s[a] = acc[p];
        }
        __syncthreads();
        fft_lds<T, NMAX, G, +1, P2>(s, pcol, tw.tw, tid);
    } else {
        load_rows(static_cast<const cplx<T>*>(op.T1) + item.comp * op.tslot, col_rows(op, args.nin));
        __syncthreads();
        fft_lds<T, NMAX, G, -1, P2>(s, pcol, tw.tw, tid);
        if (args.mode == COL_SPEC || args.mode == COL_STORE) {
            cplx<T>* dst = args.mode == COL_SPEC ? static_cast<cplx<T>*>(const_cast<void*>(op.Xh))
                                                 : static_cast<cplx<T>*>(op.Us) + (long)item.comp * op.uslot;
            const T scl = to<T>(args.mode == COL_SPEC ? op.spec_scale : 1.0);
            for (int e = threadIdx.x; e < MA * TC; e += nthr) {
                const int cc = e / MA, a = e % MA;
                const int f = f0 + cc;
                if (f < P) {
                    const cplx<T> v = buf[cc * LD + a];
                    dst[(long)f * MA + a] = {v.x * scl, v.y * scl};
                }
            }
            return;
        }
        // COL_CORR
        const cplx<T>* xh = static_cast<const cplx<T>*>(op.Xh);
        for (int e = threadIdx.x; e < MA * TC; e += nthr) {
            const int cc = e / MA, a = e % MA;
            const int f = f0 + cc;
            if (f < P) buf[cc * LD + a] = cmulc(xh[(long)f * MA + a], buf[cc * LD + a]);
        }
        __syncthreads();
        fft_lds<T, NMAX, G, +1, P2>(s, pcol, tw.tw, tid);
    }
    cplx<T>* out = static_cast<cplx<T>*>(op.T2) + item.comp * op.tslot;
    const int nout = col_rows(op, args.nout);
    for (int e = threadIdx.x; e < nout * TC; e += nthr) {
        const int a = e / TC, cc = e % TC;
        const int f = f0 + cc;
        if (f < P) out[(long)a * op.ldp + f] = buf[cc * LD + a];
    }
}

// Column pass for power-of-two column lengths MA = 2^LOGN (64..1024) with
// the transforms held in registers.  A workgroup takes TC adjacent columns
// f0..f0+TC of one instance with G = MA/8 threads per column; thread (c, t)
// is threadIdx.x = c + TC*t, so the lanes of a wave read TC consecutive bins
// of a row.  The spectrum is stored like T1 and T2: [MA rows][P bins].
//   SPEC:  Xh = scale * FFT_col(T1 rows < nin)
//   !SPEC: T2 rows < nout = IFFT_col(Xh * conj(FFT_col(T1 rows < nin)))
// LTW: twiddles from a table in LDS and one exchange buffer (two barriers
// per exchange): fewer registers and less LDS per workgroup, so more
// workgroups per compute unit; otherwise twiddles in registers and two
// exchange buffers used in turn.
template <typename T, int LOGN, int TC, bool SPEC, bool LTW>
__global__ void __launch_bounds__(RegPlan<LOGN>::G * TC, LTW ? 8 : 1)
k_colr(const OpDesc* __restrict__ ops, const Item* __restrict__ items, ColArgs args) {
    using RP = RegPlan<LOGN>;
    constexpr int G = RP::G;
    constexpr int XB = RP::LROWS * TC;
    constexpr int XSM = LTW ? XS_WG : XS_WG2;
    __shared__ cplx<T> lds[(LTW ? 1 : 2) * XB + (LTW ? TwTable<T, LOGN>::SIZE + 1 : 0)];
    const Item item = items[xcd_block(blockIdx.x, gridDim.x)];
    int xe = 0;
    const OpDesc& op = ops[item.inst];
    const int c = threadIdx.x % TC, t = threadIdx.x / TC;
    const int P = op.P;
    const long ld = op.ldp;
    const int f = item.idx * TC + c;
    const bool fok = f < P;
    const int nin = col_rows(op, args.nin), nout = col_rows(op, args.nout);
    cplx<T> w[LTW ? 1 : RP::NTW];
    cplx<T>* tab = lds + XB;
    typename TwTable<T, LOGN>::template Stage<G * TC> stage;
    if constexpr (LTW) {
        // loaded here, written to LDS once the tile's loads are issued; read
        // first after an exchange barrier (the first pass has no twiddles)
        stage.load(as_global(static_cast<const cplx<T>*>(op.pcol.tw)), threadIdx.x);
    } else {
        reg_twiddles<T, LOGN>(static_cast<const cplx<T>*>(op.pcol.tw), t, w);
    }
    const auto W = [&](int q) -> cplx<T> {
        if constexpr (LTW) return TwTable<T, LOGN>{tab, t}(q);
        else return w[q];
    };
    // tile bases (uniform) and the thread's 32-bit offset within a tile
    const long tile = item.comp * op.tslot + (long)item.idx * TC;
    const long estep = (long)G * ld;
    const int lo = t * (int)ld + c;
    gptr<const cplx<T>> src = as_global(static_cast<const cplx<T>*>(op.T1) + tile);
    gptr<cplx<T>> xh = as_global(static_cast<cplx<T>*>(const_cast<void*>(op.Xh)) + (long)item.idx * TC);
    cplx<T> v[8], x[8];
#pragma unroll
    for (int e = 0; e < 8; ++e)
        v[e] = (fok && t + G * e < nin) ? gload(src + e * estep + lo) : cplx<T>{T(0), T(0)};
    if constexpr (!SPEC) {
#pragma unroll
        for (int e = 0; e < 8; ++e) x[e] = fok ? gload(xh + e * estep + lo) : cplx<T>{T(0), T(0)};
    }
    if constexpr (LTW) stage.store(tab, threadIdx.x);
    const auto ad = [&](int pp) { return rx_addr<TC>(pp, c); };
    if (nin <= G) reg_fft_tw<T, LOGN, -1, XSM, true>(v, W, lds, t, ad, xe, XB);
    else reg_fft_tw<T, LOGN, -1, XSM>(v, W, lds, t, ad, xe, XB);
    if constexpr (SPEC) {
        if (!fok) return;
        const T sc = to<T>(op.spec_scale);
#pragma unroll
        for (int e = 0; e < 8; ++e) gstore(xh + e * estep + lo, cplx<T>{v[e].x * sc, v[e].y * sc});
        return;
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = cmulc(x[e], v[e]);
        gptr<cplx<T>> dst = as_global(static_cast<cplx<T>*>(op.T2) + tile);
        if constexpr (RP::REM == 0) {
            if (nout <= G) {
                reg_fft_tw<T, LOGN, +1, XSM, false, true>(v, W, lds, t, ad, xe, XB);
                if (fok && t < nout) gstore(dst + lo, v[0]);
                return;
            }
        }
        reg_fft_tw<T, LOGN, +1, XSM>(v, W, lds, t, ad, xe, XB);
        if (!fok) return;
#pragma unroll
        for (int e = 0; e < 8; ++e)
            if (t + G * e < nout) gstore(dst + e * estep + lo, v[e]);
    }
}

// Column pass without (k_col) and with (k_col_acc) the group accumulation of
// the reconstruction; separate kernels keep the accumulator's registers out
// of the product kernel.
template <typename T, int NMAX, int G, int TC, bool P2>
__global__ void __launch_bounds__(G * TC)
k_col(const OpDesc* __restrict__ ops, const ResDesc* __restrict__ res, const Item* __restrict__ items, int nitems,
      ColArgs args) {
    col_body<T, NMAX, G, TC, P2, false>(ops, res, items, nitems, args);
}

template <typename T, int NMAX, int G, int TC, bool P2>
__global__ void __launch_bounds__(G * TC)
k_col_acc(const OpDesc* __restrict__ ops, const ResDesc* __restrict__ res, const Item* __restrict__ items,
          int nitems, ColArgs args) {
    col_body<T, NMAX, G, TC, P2, true>(ops, res, items, nitems, args);
}

// ------------------------------------------------------------------------
// shape setup (once per decomposition)
// ------------------------------------------------------------------------

// N = mask AND not-NaN, xc = x on N else 0, and row prefix counts of N.
// One workgroup (256 threads) per grid row.
__global__ void __launch_bounds__(256)
k_shape_clean(const OpDesc* __restrict__ ops, const Item* __restrict__ items, const double* const* xin,
              const uint8_t* const* min, uint8_t* const* nset, double* const* xc, int* const* npref) {
    __shared__ int wt[4];
    __shared__ int carry;
    const Item item = items[blockIdx.x];
    const OpDesc& op = ops[item.inst];
    const int a = item.idx, B = op.B;
    const double* x = xin[item.inst] + (long)a * B;
    const uint8_t* m = min[item.inst] ? min[item.inst] + (long)a * B : nullptr;
    uint8_t* ns = nset[item.inst] + (long)a * B;
    double* xo = xc[item.inst] + (long)a * B;
    int* pref = npref[item.inst] + (long)a * (B + 1);
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int c0 = 0; c0 < B; c0 += 256) {
        const int b = c0 + threadIdx.x;
        int in = 0;
        if (b < B) {
            const double v = x[b];
            in = (m == nullptr || m[b] != 0) && !isnan(v);
            ns[b] = (uint8_t)in;
            xo[b] = in ? v : 0.0;
        }
        const unsigned long long bal = __ballot(in);
        const int lane = lane_id(), wv = threadIdx.x >> 6;
        const int r = __popcll(bal & ((1ULL << lane) - 1ULL));
        if (lane == 0) wt[wv] = __popcll(bal);
        __syncthreads();
        int before = carry;
        for (int q = 0; q < wv; ++q) before += wt[q];
        if (b < B) pref[b] = before + r;
        __syncthreads();
        if (threadIdx.x == 0) carry += wt[0] + wt[1] + wt[2] + wt[3];
        __syncthreads();
    }
    if (threadIdx.x == 0) pref[B] = carry;
}


// Origins: count(k) = sum over window runs of N cells under the run; k is in
// K when the count equals |L|.  Also the row prefix of the origin mask and
// the per-row origin counts.  One workgroup per origin-box row.
__global__ void __launch_bounds__(256)
k_shape_origins(const OpDesc* __restrict__ ops, const Item* __restrict__ items, const Runs* __restrict__ runs,
                const int* const* npref, uint8_t* const* kmask, int* const* kpref, int* const* kcount) {
    __shared__ int wt[4];
    __shared__ int carry;
    const Item item = items[blockIdx.x];
    const OpDesc& op = ops[item.inst];
    const Runs& R = runs[item.inst];
    const int a = item.idx;
    const int KB = op.S[1].boxB, B = op.B;
    const int* np = npref[item.inst];
    uint8_t* km = kmask[item.inst] + (long)a * KB;
    int* kp = kpref[item.inst] + (long)a * (KB + 1);
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    // a window without mask: k_shape_vcount has left each origin's count in
    // kp (read here before the prefix overwrites it)
    const bool full = op.S[0].mask == nullptr;
    for (int c0 = 0; c0 < KB; c0 += 256) {
        const int b = c0 + threadIdx.x;
        int in = 0;
        if (b < KB) {
            long cnt = 0;
            if (full) {
                cnt = kp[b];
            } else {
                for (int t = 0; t < R.nrun; ++t) {
                    const int* pr = np + (long)(a + R.ra[t]) * (B + 1);
                    cnt += pr[b + R.b1[t]] - pr[b + R.b0[t]];
                }
            }
            in = cnt == R.total;
            km[b] = (uint8_t)in;
        }
        const unsigned long long bal = __ballot(in);
        const int lane = lane_id(), wv = threadIdx.x >> 6;
        const int r = __popcll(bal & ((1ULL << lane) - 1ULL));
        if (lane == 0) wt[wv] = __popcll(bal);
        __syncthreads();
        int before = carry;
        for (int q = 0; q < wv; ++q) before += wt[q];
        if (b < KB) kp[b] = before + r;
        __syncthreads();
        if (threadIdx.x == 0) carry += wt[0] + wt[1] + wt[2] + wt[3];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        kp[KB] = carry;
        kcount[item.inst][a] = carry;
    }
}

// Origin counts of a window without mask (an LA x LB box): count(ka, b) =
// sum over t < LA of the N cells in row ka + t, columns [b, b + LB), a
// sliding sum down each column of the per-row run counts.  One thread per
// origin-box column (items: instance x chunk of 256 columns), exact integer
// arithmetic; the counts go to kpref rows (row stride KB + 1), which
// k_shape_origins reads before it writes the row prefixes there.
__global__ void __launch_bounds__(256)
k_shape_vcount(const OpDesc* __restrict__ ops, const Item* __restrict__ items, const int* const* npref,
               int* const* kpref) {
    const Item item = items[blockIdx.x];
    const OpDesc& op = ops[item.inst];
    const int b = item.idx * 256 + threadIdx.x;
    const int KA = op.S[1].boxA, KB = op.S[1].boxB, LA = op.S[0].boxA, LB = op.S[0].boxB, B = op.B;
    if (b >= KB) return;
    const int* np = npref[item.inst];
    int* kp = kpref[item.inst];
    const auto rc = [&](int a) { return np[(long)a * (B + 1) + b + LB] - np[(long)a * (B + 1) + b]; };
    long sum = 0;
    for (int t = 0; t < LA; ++t) sum += rc(t);
    kp[b] = (int)sum;
    for (int ka = 1; ka < KA; ++ka) {
        sum += rc(ka + LA - 1) - rc(ka - 1);
        kp[(long)ka * (KB + 1) + b] = (int)sum;
    }
}

// Exclusive scan of per-row origin counts into row offsets (one workgroup
// per instance, sequential over rows in chunks).
__global__ void __launch_bounds__(256)
k_shape_rowoff(int ninst, const int* const* kcount, int* const* rowoff, const int* nrows, long* total) {
    const int inst = blockIdx.x;
    if (inst >= ninst) return;
    __shared__ long wsum[4];
    __shared__ long carry;
    const int n = nrows[inst];
    const int* cnt = kcount[inst];
    int* ro = rowoff[inst];
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int c0 = 0; c0 < n; c0 += 256) {
        const int i = c0 + threadIdx.x;
        long v = i < n ? cnt[i] : 0;
        // inclusive wave scan
        const int lane = lane_id(), wv = threadIdx.x >> 6;
        long x = v;
        for (int o = 1; o < 64; o <<= 1) {
            long y = __shfl_up(x, o);
            if (lane >= o) x += y;
        }
        if (lane == 63) wsum[wv] = x;
        __syncthreads();
        long before = carry;
        for (int q = 0; q < wv; ++q) before += wsum[q];
        if (i < n) ro[i] = (int)(before + x - v);
        __syncthreads();
        if (threadIdx.x == 0) carry += wsum[0] + wsum[1] + wsum[2] + wsum[3];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        ro[n] = (int)carry;
        total[inst] = carry;
    }
}

// Weights W(alpha) = #{ l in L : alpha - l in K }, by run sums over the row
// prefix of the origin mask.  One workgroup per grid row.
__global__ void __launch_bounds__(256)
k_shape_weights(const OpDesc* __restrict__ ops, const Item* __restrict__ items, const Runs* __restrict__ runs,
                const int* const* kpref, double* const* Wout) {
    const Item item = items[blockIdx.x];
    const OpDesc& op = ops[item.inst];
    const Runs& R = runs[item.inst];
    const int a = item.idx, B = op.B;
    const int KA = op.S[1].boxA, KB = op.S[1].boxB;
    const int* kp = kpref[item.inst];
    double* W = Wout[item.inst] + (long)a * B;
    for (int b = threadIdx.x; b < B; b += 256) {
        long cnt = 0;
        for (int t = 0; t < R.nrun; ++t) {
            const int ka = a - R.ra[t];
            if (ka < 0 || ka >= KA) continue;
            // k_b in (b - b1, b - b0]  intersected with [0, KB)
            int lo = b - R.b1[t] + 1, hi = b - R.b0[t] + 1;   // [lo, hi)
            if (lo < 0) lo = 0;
            if (hi > KB) hi = KB;
            if (hi > lo) {
                const int* pr = kp + (long)ka * (KB + 1);
                cnt += pr[hi] - pr[lo];
            }
        }
        W[b] = (double)cnt;
    }
}

// Weights of a window without mask: W(a, b) = sum over ka in (a - LA, a]
// of the origins of row ka in columns (b - LB, b], a sliding sum down each
// column of row-prefix differences of the origin mask.  One thread per grid
// column (items: instance x chunk of 256 columns), exact integer arithmetic.
__global__ void __launch_bounds__(256)
k_shape_weights_v(const OpDesc* __restrict__ ops, const Item* __restrict__ items, const int* const* kpref,
                  double* const* Wout) {
    const Item item = items[blockIdx.x];
    const OpDesc& op = ops[item.inst];
    const int b = item.idx * 256 + threadIdx.x;
    const int A = op.A, B = op.B, KA = op.S[1].boxA, KB = op.S[1].boxB, LA = op.S[0].boxA, LB = op.S[0].boxB;
    if (b >= B) return;
    const int* kp = kpref[item.inst];
    double* W = Wout[item.inst];
    const int lo = b - LB + 1 > 0 ? b - LB + 1 : 0, hi = b + 1 < KB ? b + 1 : KB;
    const auto roww = [&](int ka) { return hi > lo ? kp[(long)ka * (KB + 1) + hi] - kp[(long)ka * (KB + 1) + lo] : 0; };
    long sum = 0;
    for (int a = 0; a < A; ++a) {
        if (a < KA) sum += roww(a);
        if (a - LA >= 0 && a - LA < KA) sum -= roww(a - LA);
        W[(long)a * B + b] = (double)sum;
    }
}

// ------------------------------------------------------------------------
// Lanczos (FP64): classical Gram-Schmidt applied twice against the basis
// ------------------------------------------------------------------------

// Deterministic start vector: hash of (seed, index) mapped to [-1, 1); the
// first step normalises it.
__device__ __forceinline__ double hash_unit(unsigned long long seed, unsigned long long i) {
    unsigned long long z = seed * 0x9E3779B97F4A7C15ULL + i + 0x632BE59BD9B4E019ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z ^= z >> 31;
    return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

__global__ void __launch_bounds__(256)
k_lz_start(const LzDesc* __restrict__ lzs, const Item* __restrict__ items, unsigned long long seed) {
    __shared__ double red[4];
    const Item item = items[blockIdx.x];
    const LzDesc& lz = lzs[item.inst];
    seed ^= lz.seed;   // the decomposition's own seed: a result does not depend on its batch
    const long i = (long)item.idx * kLzRows + threadIdx.x;
    double v = 0.0;
    if (i < lz.n) {
        v = hash_unit(seed, (unsigned long long)i);
        lz.w[i] = v;
    }
    const double p = wave_sum(v * v);
    if (lane_id() == 0) red[threadIdx.x >> 6] = p;
    __syncthreads();
    if (threadIdx.x == 0) lz.np[item.idx] = red[0] + red[1] + red[2] + red[3];
    // clear this block's share of the long vectors and their row norms
    {
        const long wc = (lz.lwords + lz.nblk - 1) / lz.nblk;
        const long w0 = (long)item.idx * wc, w1 = min(lz.lwords, w0 + wc);
        uint32_t* lw = static_cast<uint32_t*>(lz.lbuf[0]);
        for (long e = w0 + threadIdx.x; e < w1; e += 256) lw[e] = 0u;
        const int rc = (2 * lz.lrows + lz.nblk - 1) / lz.nblk;
        const int r0 = item.idx * rc, r1 = min(2 * lz.lrows, r0 + rc);
        for (int e = r0 + threadIdx.x; e < r1; e += 256) lz.lnp[0][e] = 0.0;
    }
    // clear the projected matrix, the breakdown flags and the running scale
    if (item.idx == 0) {
        for (int e = threadIdx.x; e < kMaxBasis * kMaxBasis; e += 256) lz.Bm[e] = 0.0;
        if (threadIdx.x == 0) {
            lz.flag[2] = 0;
            lz.flag[3] = 0;
            lz.beta[2] = 0.0;
            lz.beta[3] = 0.0;
        }
    }
}

// Transposing butterfly over 16 values per lane: each step pairs every lane
// with a partner whose bit O differs, each lane keeps half of its values (the
// lower half when bit O of the lane is clear) and adds the partner's copy of
// that half.  After the steps O = 8, 4, 2, 1 lane l holds value (l & 15)
// summed over its 16-lane row; two more steps sum the four rows of the wave.
// The partners come from DPP moves within the row: lane ^ 8 (rotate by 8),
// 7 - lane within each 8 (mirror: bit 2 differs and the lower bits only
// permute a coset, so every lane of the row still enters each sum once),
// lane ^ 2 and lane ^ 1 (quad permutes).
template <int O>
__device__ __forceinline__ void tr_step(double* v, int l) {
    constexpr int ctrl = O == 8 ? 0x128 : O == 4 ? 0x141 : O == 2 ? 0x4E : 0xB1;
    const bool hi = (l & O) != 0;
#pragma unroll
    for (int k = 0; k < O; ++k) {
        const double send = hi ? v[k] : v[k + O];
        const double keep = hi ? v[k + O] : v[k];
        v[k] = keep + dpp_f64<ctrl>(send);
    }
}

__device__ __forceinline__ double wave_sum16(double (&v)[16]) {
    const int l = lane_id();
    tr_step<8>(v, l);
    tr_step<4>(v, l);
    tr_step<2>(v, l);
    tr_step<1>(v, l);
    double s = v[0];
    s += __shfl_xor(s, 16);
    s += __shfl_xor(s, 32);
    return s;
}

// hp[blk][c] = sum over the block's rows of Q[:, c] * w for c < ncols and,
// when npart is given, npart[blk] = sum over the block's rows of w^2.
// Thread = row; each wave reduces 16 columns at a time with the transposing
// butterfly, the four waves combine through LDS.
// QT: the type of the basis copy read (double, or float for the FP32 copy).
template <typename QT>
__device__ __forceinline__ void lz_project_block_t(const LzDesc& lz, const QT* Qb, int blk, int ncols,
                                                   const double* wp, double* hp, double* npart,
                                                   double (*red)[kMaxBasis + 1]) {
    const long i = (long)blk * kLzRows + threadIdx.x;
    const bool in = i < lz.n;
    const long n = lz.n;
    const gptr<const QT> Q = as_global(Qb) + (in ? i : 0);
    const double wi = in ? gload(as_global(wp) + i) : 0.0;
    const int wv = threadIdx.x >> 6, l = lane_id();
    for (int c0 = 0; c0 < ncols; c0 += 16) {
        double v[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int c = c0 + k;
            const double qv = static_cast<double>(gload(Q + (long)(c < ncols ? c : 0) * n));   // unconditional: loads overlap
            v[k] = c < ncols ? qv * wi : 0.0;
        }
        const double sm = wave_sum16(v);
        if (l < 16 && c0 + l < ncols) red[wv][c0 + l] = sm;
    }
    if (npart) {
        const double p = wave_sum(wi * wi);
        if (l == 0) red[wv][kMaxBasis] = p;
    }
    __syncthreads();
    for (int c = threadIdx.x; c < ncols; c += 256)
        hp[(long)blk * (kMaxBasis + 1) + c] = red[0][c] + red[1][c] + red[2][c] + red[3][c];
    if (npart && threadIdx.x == 0)
        npart[blk] = red[0][kMaxBasis] + red[1][kMaxBasis] + red[2][kMaxBasis] + red[3][kMaxBasis];
}

__device__ __forceinline__ void lz_project_block(const LzDesc& lz, int blk, int ncols, const double* wp,
                                                 double* hp, double* npart, double (*red)[kMaxBasis + 1]) {
    if (lz.Q32) lz_project_block_t<float>(lz, lz.Q32, blk, ncols, wp, hp, npart, red);
    else lz_project_block_t<double>(lz, lz.Q, blk, ncols, wp, hp, npart, red);
}

// Iterated classical Gram-Schmidt of w against Q[:, 0:ncols] with the
// Daniel-Gragg-Kaufman-Stewart test: the second pass runs only when the
// first one shrank |w| below |w_before| / sqrt(2) (or when forced).  Every
// workgroup takes the decision from the same partial norms in the same
// order, so all agree.
__device__ __forceinline__ bool cgs_second_pass(const LzDesc& lz, int force) {
    if (force) return true;
    const double after = sum_parts(lz.np, lz.nblk), before = sum_parts(lz.np0, lz.nblk);
    return after < 0.5 * before;
}

// First projection: hp1 partials of Q^T w, np0 partials of |w|^2.
__global__ void __launch_bounds__(256)
k_lz_proj(const LzDesc* __restrict__ lzs, const Item* __restrict__ items, int ncols) {
    __shared__ double red[4][kMaxBasis + 1];
    const Item item = items[blockIdx.x];
    const LzDesc& lz = lzs[item.inst];
    if (ncols < 0) ncols = lz.step[0] + 1;   // step from the counter
    lz_project_block(lz, item.idx, ncols, lz.w, lz.hp1, lz.np0, red);
}

// Second projection (hp2 partials), only when the second pass runs.
__global__ void __launch_bounds__(256)
k_lz_proj2(const LzDesc* __restrict__ lzs, const Item* __restrict__ items, int ncols, int force) {
    __shared__ double red[4][kMaxBasis + 1];
    const Item item = items[blockIdx.x];
    const LzDesc& lz = lzs[item.inst];
    if (ncols < 0) ncols = lz.step[0] + 1;
    if (!cgs_second_pass(lz, force)) return;
    lz_project_block(lz, item.idx, ncols, lz.w, lz.hp2, nullptr, red);
}

// Update of each pass (one-sided: the coefficients are discarded, they are
// rounding-level terms): h = sum of the pass's partials; w -= Q h;
// np = partial |w|^2.  Pass 2 does nothing unless the second pass runs.
__global__ void __launch_bounds__(256)
k_lz_update(const LzDesc* __restrict__ lzs, const Item* __restrict__ items, int ncols, int pass, int force) {
    __shared__ double h[kMaxBasis + 1];
    __shared__ double red[4];
    const Item item = items[blockIdx.x];
    const LzDesc& lz = lzs[item.inst];
    if (ncols < 0) ncols = lz.step[0] + 1;
    if (pass == 2 && !cgs_second_pass(lz, force)) return;
    const gptr<const double> hp = as_global(static_cast<const double*>(pass == 1 ? lz.hp1 : lz.hp2));
    for (int c = threadIdx.x; c < ncols; c += 256) {
        // four independent partial sums: the block partials load in parallel
        double s4[4] = {0.0, 0.0, 0.0, 0.0};
        int q = 0;
        for (; q + 4 <= lz.nblk; q += 4) {
#pragma unroll
            for (int u = 0; u < 4; ++u) s4[u] += gload(hp + (long)(q + u) * (kMaxBasis + 1) + c);
        }
        for (; q < lz.nblk; ++q) s4[0] += gload(hp + (long)q * (kMaxBasis + 1) + c);
        h[c] = (s4[0] + s4[1]) + (s4[2] + s4[3]);
    }
    __syncthreads();
    const long i = (long)item.idx * kLzRows + threadIdx.x;
    double wi = 0.0;
    if (i < lz.n) {
        const gptr<double> w = as_global(lz.w) + i;
        wi = gload(w);
        double acc = 0.0;
        if (lz.Q32) {
            const gptr<const float> Q = as_global(static_cast<const float*>(lz.Q32)) + i;
#pragma unroll 8
            for (int c = 0; c < ncols; ++c) acc += static_cast<double>(gload(Q + (long)c * lz.n)) * h[c];
        } else {
            const gptr<const double> Q = as_global(static_cast<const double*>(lz.Q)) + i;
#pragma unroll 8
            for (int c = 0; c < ncols; ++c) acc += gload(Q + (long)c * lz.n) * h[c];
        }
        wi -= acc;
        gstore(w, wi);
    }
    const double p = wave_sum(wi * wi);
    if (lane_id() == 0) red[threadIdx.x >> 6] = p;
    __syncthreads();
    if (threadIdx.x == 0) lz.np[item.idx] = red[0] + red[1] + red[2] + red[3];
}

// q_m = w / beta into column m of Q; beta -> lz.beta[0].
__global__ void __launch_bounds__(256)
k_lz_normalize(const LzDesc* __restrict__ lzs, const Item* __restrict__ items, int m) {
    const Item item = items[blockIdx.x];
    const LzDesc& lz = lzs[item.inst];
    const double beta = sqrt(sum_parts(lz.np, lz.nblk));
    const double sc = beta > 1e-300 ? 1.0 / beta : 0.0;
    const long i = (long)item.idx * kLzRows + threadIdx.x;
    if (i < lz.n) {
        const double q = lz.w[i] * sc;
        lz.Q[(long)m * lz.n + i] = q;
        if (lz.Q32) lz.Q32[(long)m * lz.n + i] = static_cast<float>(q);
    }
    if (item.idx == 0 && threadIdx.x == 0) lz.beta[0] = beta;
}

// 1/x (x nonzero, finite) and 1/sqrt(x) (x > 0, finite) from the hardware
// approximations (about 23 correct bits) refined by Newton steps, which
// double the correct bits each: one step for 1/x (used for the rotation
// angle, which only needs to be close), two for 1/sqrt(x) (the cosine, which
// must make c^2 + s^2 = 1 to rounding so that rotations stay orthogonal).
__device__ __forceinline__ double rcp_nr(double x) {
    const double y = __builtin_amdgcn_rcp(x);
    return fma(y, fma(-x, y, 1.0), y);
}
__device__ __forceinline__ double rsqrt_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const double h = 0.5 * x * y;
        y = fma(y, fma(-h, y, 0.5), y);
    }
    return y;
}

// SVD of the m x m projected matrix by one-sided (Hestenes) Jacobi, one
// workgroup of 512 threads per instance.  The columns of B live in LDS,
// zero-padded to 8 PE rows (stride 8 PE: a padded stride measured no
// better); in each round of the
// round-robin ordering every 8-lane group takes one column pair into
// registers (lane g holds rows 2g, 2g + 1 of each 16-row slice, read as
// 16-byte words), forms the three inner products, rotates the pair when it
// is not yet orthogonal and writes it back.  Padding rows stay zero under
// rotations, so loads and stores need no row test.  Only the last row of the
// accumulated right rotations is needed downstream (the residual estimates
// beta * Yr[m-1, i]), so only that row is rotated.  The singular values are
// the final column norms, the left vectors the normalised columns; they are
// ranked (descending) and the residual test beta |Yr[m-1, i]| <= tol * sigma_1
// is evaluated for the r leading ones.
// PE: column entries per lane (even), 8 PE >= m; the launch picks the
// smallest PE that fits (the round time grows with PE: 10 rather than 12 at
// m = 80 took a fifth off).
template <int PE>
__global__ void __launch_bounds__(512)
k_lz_svd(const LzDesc* __restrict__ lzs, const Item* __restrict__ items, int m, int max_sweeps) {
    constexpr int LP = 8;                       // lanes per column pair
    constexpr int R = LP * PE;                  // padded rows per column
    constexpr int CS = R;                       // column stride (doubles)
    static_assert(PE % 2 == 0 && R <= kMaxBasis, "column entries beyond the basis");
    __shared__ __align__(16) double Bs[R * CS];
    __shared__ double yl[kMaxBasis];
    __shared__ double cn[kMaxBasis];
    __shared__ int changed;
    const Item item = items[blockIdx.x];
    const LzDesc& lz = lzs[item.inst];
    const int nt = blockDim.x;
    const int nn = m + (m & 1);
    for (int e = threadIdx.x; e < nn * R; e += nt) {
        const int i = e % R, c = e / R;
        Bs[c * CS + i] = (i < m && c < m) ? lz.Bm[(long)c * kMaxBasis + i] : 0.0;
    }
    for (int c = threadIdx.x; c < m; c += nt) yl[c] = c == m - 1 ? 1.0 : 0.0;
    const int npairs = nn / 2;
    const int t = threadIdx.x / LP, g = threadIdx.x % LP;
    // rotations stop at |a_p . a_q| <= jt |a_p| |a_q| (far below the
    // accuracy the operator precision can support)
    const double jt = lz.eps < 1e-8 ? 1e-15 : 1e-12;
    const double jt2 = jt * jt;
    using d2 = double __attribute__((ext_vector_type(2)));
    int sweep = 0;
    for (; sweep < max_sweeps; ++sweep) {
        if (threadIdx.x == 0) changed = 0;
        __syncthreads();
        // round-robin pairing: round rd pairs (rd + t, rd - t) mod (nn - 1),
        // and nn - 1 with rd for t = 0; both indices advance by one per round
        int a = t == 0 ? nn - 1 : t, b = t == 0 ? 0 : nn - 1 - t;
        for (int rd = 0; rd < nn - 1; ++rd) {
            const int p = a < b ? a : b, q = a < b ? b : a;
            if (t != 0) a = a + 1 == nn - 1 ? 0 : a + 1;
            b = b + 1 == nn - 1 ? 0 : b + 1;
            if (t < npairs && q < m) {
                d2* bp = reinterpret_cast<d2*>(Bs + p * CS) + g;
                d2* bq = reinterpret_cast<d2*>(Bs + q * CS) + g;
                d2 x1[PE / 2], x2[PE / 2];
#pragma unroll
                for (int k = 0; k < PE / 2; ++k) {
                    x1[k] = bp[LP * k];
                    x2[k] = bq[LP * k];
                }
                // two partial sums per product: shorter dependent chains
                double al2[2] = {0.0, 0.0}, be2[2] = {0.0, 0.0}, ga2[2] = {0.0, 0.0};
#pragma unroll
                for (int k = 0; k < PE / 2; ++k) {
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        al2[h] = fma(x1[k][h], x1[k][h], al2[h]);
                        be2[h] = fma(x2[k][h], x2[k][h], be2[h]);
                        ga2[h] = fma(x1[k][h], x2[k][h], ga2[h]);
                    }
                }
                const double al = group8_sum(al2[0] + al2[1]);
                const double be = group8_sum(be2[0] + be2[1]);
                const double ga = group8_sum(ga2[0] + ga2[1]);
                if (ga != 0.0 && ga * ga > jt2 * (al * be)) {
                    const double ze = (be - al) * rcp_nr(2.0 * ga);
                    const double az = fabs(ze);
                    double tt;
                    if (az < 1e100) {
                        const double q1 = 1.0 + ze * ze;
                        tt = copysign(rcp_nr(az + q1 * rsqrt_nr(q1)), ze);
                    } else {
                        tt = 0.5 / ze;   // angle below rounding of 1 + ze^2
                    }
                    const double c = rsqrt_nr(1.0 + tt * tt), sn = c * tt;
#pragma unroll
                    for (int k = 0; k < PE / 2; ++k) {
                        bp[LP * k] = c * x1[k] - sn * x2[k];
                        bq[LP * k] = sn * x1[k] + c * x2[k];
                    }
                    if (g == 0) {
                        const double y1 = yl[p], y2 = yl[q];
                        yl[p] = c * y1 - sn * y2;
                        yl[q] = sn * y1 + c * y2;
                        changed = 1;
                    }
                }
            }
            __syncthreads();
        }
        // read the flag, then let thread 0 reset it only after every thread has
        const int ch = changed;
        __syncthreads();
        if (!ch) break;
    }
    for (int c = threadIdx.x; c < m; c += nt) {
        double s2 = 0.0;
        for (int i = 0; i < m; ++i) s2 += Bs[c * CS + i] * Bs[c * CS + i];
        cn[c] = sqrt(s2);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < m * m; e += nt) {
        const int i = e % m, c = e / m;
        lz.Yl[(long)c * kMaxBasis + i] = cn[c] > 0 ? Bs[c * CS + i] / cn[c] : 0.0;
    }
    for (int c = threadIdx.x; c < m; c += nt) lz.Yr[(long)c * kMaxBasis + (m - 1)] = yl[c];
    for (int i = threadIdx.x; i < m; i += nt) {
        const double ti = cn[i];
        int rank = 0;
        for (int k = 0; k < m; ++k) {
            const double tk = cn[k];
            rank += (tk > ti) || (tk == ti && k < i);
        }
        lz.perm[rank] = i;
        lz.sig[rank] = ti;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int r = lz.r;
        const double beta = lz.beta[0];
        const double s1 = lz.sig[0];
        int ok = 1;
        double worst = 0.0;
        for (int i = 0; i < r; ++i) {
            const int c = lz.perm[i];
            const double resid = fabs(beta * yl[c]);
            if (!(resid <= lz.tol * s1)) ok = 0;
            worst = fmax(worst, s1 > 0 ? resid / s1 : 0.0);
        }
        lz.flag[0] = ok;
        lz.flag[1] = sweep;
        lz.beta[1] = worst;
    }
}

// Ritz rotation out[:, 0:k] = Q[:, 0:m] * Yl[:, perm[0:k]] (FP64) on the
// matrix cores.  Workgroup = 64 rows x up to 32 output columns; each wave
// takes 16 rows and accumulates the transposed
// tiles out^T (16 columns x 16 rows) = Y^T Q^T with v_mfma_f64_16x16x4f64,
// 4 basis vectors per instruction.  Operand lanes: A (16 x 4) element (i, k)
// in lane i + 16 k, B (4 x 16) element (k, j) in lane j + 16 k; the
// accumulator holds element (4 v + lane / 16, lane % 16) in its value v.  So
// the lanes of a wave read 16 consecutive rows of 4 basis vectors
// (coalesced) and write 16 consecutive rows of 4 output columns.  The loads
// of 8 instructions' operands are issued together (memory-level parallelism).
typedef double dvec4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256)
k_lz_ritz(const LzDesc* __restrict__ lzs, const Item* __restrict__ items, int m, int k, double* const* outs) {
    constexpr int CB = 2;   // 16-column blocks per workgroup
    __shared__ double Ys[kMaxBasis][16 * CB];
    const Item item = items[blockIdx.x];
    const LzDesc& lz = lzs[item.inst];
    double* out = outs ? outs[item.inst] : lz.Qtmp;
    if (outs) k = k < lz.r ? k : lz.r;   // final vectors: this decomposition's r
    const int c0 = item.aux * 16 * CB;
    const int m4 = (m + 3) & ~3;
    for (int e = threadIdx.x; e < m4 * 16 * CB; e += 256) {
        const int i = e / (16 * CB), cc = e % (16 * CB);
        const int c = c0 + cc;
        Ys[i][cc] = (i < m && c < k) ? lz.Yl[(long)lz.perm[c] * kMaxBasis + i] : 0.0;
    }
    __syncthreads();
    const int nb = min(CB, (k - c0 + 15) / 16);   // column blocks with output
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lo = lane & 15, hi = lane >> 4;
    const long n = lz.n;
    const long r0 = (long)item.idx * 64 + wave * 16;
    if (r0 >= n || nb <= 0) return;
    const long row = r0 + lo;
    const bool rok = row < n;
    const gptr<const double> Q = as_global(lz.Q) + (rok ? row : 0);
    dvec4 acc[CB];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) acc[cb] = dvec4{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < m4; k0 += 32) {
        double b[8];
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const int col = k0 + 4 * s + hi;
            b[s] = (rok && col < m) ? gload(Q + (long)col * n) : 0.0;
        }
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const int col = k0 + 4 * s + hi;
            if (k0 + 4 * s < m4) {
#pragma unroll
                for (int cb = 0; cb < CB; ++cb)
                    if (cb < nb)
                        acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(Ys[col][16 * cb + lo], b[s], acc[cb], 0, 0, 0);
            }
        }
    }
    if (!rok) return;
    const gptr<double> o = as_global(out) + row;
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int c = c0 + 16 * cb + 4 * v + hi;
            if (cb < nb && c < k) gstore(o + (long)c * n, acc[cb][v]);
        }
}

// Thick restart keeping k Ritz triplets (u_i = Q Yl_i, sigma_i, and the
// implicit right vector v_i = X^T u_i / sigma_i):
//   Q[:, 0:k] = Qtmp, Q[:, k] = q_m,
//   B = diag(sigma_0..k-1) with row k = rho_i = beta * Yr[m-1, i],
//   sin = q_m - sum_i (rho_i / sigma_i) u_i, so that X^T sin equals
//   X^T q_m - sum_i rho_i v_i, the coupling the next step must remove.
__global__ void __launch_bounds__(256)
k_lz_restart(const LzDesc* __restrict__ lzs, const Item* __restrict__ items, int m, int k) {
    __shared__ double coef[kMaxBasis];
    const Item item = items[blockIdx.x];
    const LzDesc& lz = lzs[item.inst];
    const double beta = lz.beta[0];
    const double s1 = lz.sig[0];
    for (int c = threadIdx.x; c < k; c += 256) {
        const double sg = lz.sig[c];
        const double rho = beta * lz.Yr[(long)lz.perm[c] * kMaxBasis + (m - 1)];
        coef[c] = sg > 1e-13 * s1 ? rho / sg : 0.0;
    }
    __syncthreads();
    const long i = (long)item.idx * kLzRows + threadIdx.x;
    if (i < lz.n) {
        const double qm = lz.Q[(long)m * lz.n + i];
        double acc = qm;
        for (int c = 0; c < k; ++c) {
            const double u = lz.Qtmp[(long)c * lz.n + i];
            lz.Q[(long)c * lz.n + i] = u;
            if (lz.Q32) lz.Q32[(long)c * lz.n + i] = static_cast<float>(u);
            acc -= coef[c] * u;
        }
        lz.Q[(long)k * lz.n + i] = qm;
        if (lz.Q32) lz.Q32[(long)k * lz.n + i] = static_cast<float>(qm);
        lz.sin[i] = acc;
    }
    if (item.idx == 0) {
        for (int e = threadIdx.x; e < kMaxBasis * kMaxBasis; e += 256) {
            const int a = e % kMaxBasis, b = e / kMaxBasis;   // row a, column b
            double v = 0.0;
            if (a == b && a < k) v = lz.sig[a];
            else if (a == k && b < k) {
                const double sg = lz.sig[b];
                v = sg > 1e-13 * s1 ? beta * lz.Yr[(long)lz.perm[b] * kMaxBasis + (m - 1)] : 0.0;
            }
            lz.Bm[e] = v;
        }
        if (threadIdx.x == 0) {
            lz.flag[2] = 0;
            lz.flag[3] = 0;
        }
    }
}

// Restart after a breakdown: keep the k Ritz triplets (exact for the
// invariant subspace found), put a fresh random vector in w (to be
// orthogonalised against the kept vectors by the Gram-Schmidt kernels) and
// clear the coupling row, so the next cycle explores the complement.
__global__ void __launch_bounds__(256)
k_lz_restart_random(const LzDesc* __restrict__ lzs, const Item* __restrict__ items, int k,
                    unsigned long long seed) {
    __shared__ double red[4];
    const Item item = items[blockIdx.x];
    const LzDesc& lz = lzs[item.inst];
    seed ^= lz.seed;
    const long i = (long)item.idx * kLzRows + threadIdx.x;
    double v = 0.0;
    if (i < lz.n) {
        for (int c = 0; c < k; ++c) {
            const double u = lz.Qtmp[(long)c * lz.n + i];
            lz.Q[(long)c * lz.n + i] = u;
            if (lz.Q32) lz.Q32[(long)c * lz.n + i] = static_cast<float>(u);
        }
        v = hash_unit(seed, (unsigned long long)i);
        lz.w[i] = v;
    }
    const double p = wave_sum(v * v);
    if (lane_id() == 0) red[threadIdx.x >> 6] = p;
    __syncthreads();
    if (threadIdx.x == 0) lz.np[item.idx] = red[0] + red[1] + red[2] + red[3];
    if (item.idx == 0) {
        for (int e = threadIdx.x; e < kMaxBasis * kMaxBasis; e += 256) {
            const int a = e % kMaxBasis, b = e / kMaxBasis;
            lz.Bm[e] = (a == b && a < k) ? lz.sig[a] : 0.0;
        }
        if (threadIdx.x == 0) {
            lz.flag[2] = 0;
            lz.flag[3] = 1;
        }
    }
}

// sigma_i, i < r.
__global__ void k_lz_sigma(const LzDesc* __restrict__ lzs, const ResDesc* __restrict__ res,
                           const Item* __restrict__ items) {
    const int inst = items[blockIdx.x].inst;
    for (int i = threadIdx.x; i < lzs[inst].r; i += blockDim.x) res[inst].sigma[i] = lzs[inst].sig[i];
}

// Sign rule: flip (U_i, V_i) so that U_i's entry of largest magnitude is
// positive (first such entry in the internal order on ties).  with_v = 0
// flips U_i only: used before V = X^T U / sigma is formed, which then
// inherits the sign.
__global__ void __launch_bounds__(256)
k_sign_fix(const OpDesc* __restrict__ ops, const ResDesc* __restrict__ res, const Item* __restrict__ items,
           int with_v) {
    __shared__ double bv[256];
    __shared__ long bi[256];
    const Item item = items[blockIdx.x];
    const OpDesc& op = ops[item.inst];
    const ResDesc& rs = res[item.inst];
    const long L = op.S[0].count, K = op.S[1].count;
    double* u = rs.U + (long)item.comp * L;
    double* v = rs.V + (long)item.comp * K;
    double best = -1.0;
    long arg = 0;
    for (long i = threadIdx.x; i < L; i += 256) {
        const double a = fabs(u[i]);
        if (a > best) { best = a; arg = i; }
    }
    bv[threadIdx.x] = best;
    bi[threadIdx.x] = arg;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            const double b2 = bv[threadIdx.x + o];
            const long i2 = bi[threadIdx.x + o];
            if (b2 > bv[threadIdx.x] || (b2 == bv[threadIdx.x] && i2 < bi[threadIdx.x])) {
                bv[threadIdx.x] = b2;
                bi[threadIdx.x] = i2;
            }
        }
        __syncthreads();
    }
    const bool flip = u[bi[0]] < 0;
    __syncthreads();
    if (!flip) return;
    for (long i = threadIdx.x; i < L; i += 256) u[i] = -u[i];
    if (with_v)
        for (long i = threadIdx.x; i < K; i += 256) v[i] = -v[i];
}

// out[c][r] = in[r][c] for nmat consecutive R x C matrices (layout change
// between the caller's orientation and the internal one).
__global__ void __launch_bounds__(256) k_transpose(const double* __restrict__ in, double* __restrict__ out,
                                                   int R, int C) {
    __shared__ double tile[32][33];
    const long off = (long)blockIdx.z * R * C;
    const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
    for (int k = threadIdx.y; k < 32; k += 8) {
        const int r = r0 + k, c = c0 + threadIdx.x;
        if (r < R && c < C) tile[k][threadIdx.x] = in[off + (long)r * C + c];
    }
    __syncthreads();
    for (int k = threadIdx.y; k < 32; k += 8) {
        const int c = c0 + k, r = r0 + threadIdx.x;
        if (r < R && c < C) out[off + (long)c * R + r] = tile[threadIdx.x][k];
    }
}

// Batch readbacks: the Lanczos flags and residual figures of every instance
// (4 ints + 2 doubles each), or the r singular values of every instance,
// gathered into one array so the host reads them with a single copy.
// ------------------------------------------------------------------------
// w-correlations: weighted Gram matrix of reconstructed components
// ------------------------------------------------------------------------

// Partial weighted inner products sum_c W[c] y_a[c] y_b[c] over one chunk of
// cells, for a 16 x 16 tile of array pairs (a in block ib, b in block jb,
// ib <= jb; tiles numbered along the rows of the upper triangle), on the
// matrix cores: the Gram R^T diag(W) R is a dense contraction over the
// cells.  Each v_mfma_f64_16x16x4f64 takes 4 cells: A = the 16 arrays of
// block ib (element (i, k) in lane i + 16 k), B = W times the 16 arrays of
// block jb (element (k, j) in lane j + 16 k), so both operands of a lane are
// the same cell of two arrays.  Only cells with W > 0 enter (the
// reconstructions are NaN off the covered set); W = nullptr: unit weights,
// every cell enters (the Gram matrix of the singular vectors).  Grid
// (chunks, tiles), 4 waves per workgroup;
// part[(tile * 256 + 16 i + j) * nchunk + chunk].
__global__ void __launch_bounds__(256)
k_wgram(const double* const* __restrict__ arr, int narr, const double* __restrict__ W, long ncell, int nchunk,
        double* __restrict__ part) {
    __shared__ double red[4][256];
    const int nb = (narr + 15) / 16;
    int k = blockIdx.y, ib = 0;
    while (k >= nb - ib) {
        k -= nb - ib;
        ++ib;
    }
    const int jb = ib + k;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lo = lane & 15, hi = lane >> 4;
    const int ai = ib * 16 + lo, aj = jb * 16 + lo;
    const bool unit = W == nullptr;
    const double* spare = unit ? arr[0] : W;   // unused rows read a finite array
    const gptr<const double> pi = as_global(ai < narr ? arr[ai] : spare);
    const gptr<const double> pj = as_global(aj < narr ? arr[aj] : spare);
    const gptr<const double> pw = as_global(spare);
    constexpr int U = 8;   // 4-cell steps whose operands are loaded together
    const long csz = ((ncell + nchunk - 1) / nchunk + 16 * U - 1) / (16 * U) * (16 * U);
    const long c0 = (long)blockIdx.x * csz;
    const long c1 = min(ncell, c0 + csz);
    dvec4 acc = {0.0, 0.0, 0.0, 0.0};
    // the waves take interleaved 4-cell steps of the chunk, U at a time
    for (long cb = c0 + 4 * wave; cb < c1; cb += 16 * U) {
        double w[U], yi[U], yj[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long c = cb + 16 * u + hi;
            const bool in = c < c1;
            w[u] = in ? (unit ? 1.0 : gload(pw + c)) : 0.0;
            yi[u] = gload(pi + (in ? c : c0));
            yj[u] = gload(pj + (in ? c : c0));
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool on = w[u] > 0;
            const double a = (on && ai < narr) ? yi[u] : 0.0;
            const double b = (on && aj < narr) ? w[u] * yj[u] : 0.0;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
        }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) red[wave][(4 * v + hi) * 16 + lo] = acc[v];
    __syncthreads();
    const int e = threadIdx.x;   // 256 entries of the tile
    part[((long)blockIdx.y * 256 + e) * nchunk + blockIdx.x] = (red[0][e] + red[1][e]) + (red[2][e] + red[3][e]);
}

// ------------------------------------------------------------------------
// eigen method: S = X X^T for a small window, then its eigenpairs
// ------------------------------------------------------------------------

// Partial sums of S = X X^T over one chunk of origins for a 16 x 16 tile of
// window-cell pairs (i in block ib, j in block jb, ib <= jb; tiles numbered
// along the rows of the upper triangle), on the matrix cores.  The
// trajectory matrix is never stored: X[i, k] = xc[offL[i] + offK[k]], the
// cleaned grid (zero off N) at the cell of window cell i seen from origin
// k.  Each v_mfma_f64_16x16x4f64 takes 4 origins: A = X[block ib, 4
// origins] (element (i, k) in lane i + 16 k), B = X[block jb, the same
// origins]^T (element (k, j) in lane j + 16 k).  Grid (chunks, tiles), 4
// waves per workgroup; part[(tile * 256 + 16 i + j) * nchunk + chunk] as
// for the weighted Gram.
__global__ void __launch_bounds__(256)
k_xgram(const double* __restrict__ xc, const int* __restrict__ offL, int L, const int* __restrict__ offK, long K,
        int nchunk, double* __restrict__ part) {
    __shared__ double red[4][256];
    const int nb = (L + 15) / 16;
    int k = blockIdx.y, ib = 0;
    while (k >= nb - ib) {
        k -= nb - ib;
        ++ib;
    }
    const int jb = ib + k;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lo = lane & 15, hi = lane >> 4;
    const int ai = ib * 16 + lo, aj = jb * 16 + lo;
    const long oi = ai < L ? offL[ai] : 0, oj = aj < L ? offL[aj] : 0;   // unused rows read a valid cell
    const gptr<const double> px = as_global(xc);
    const gptr<const int> pk = as_global(offK);
    constexpr int U = 8;   // 4-origin steps whose operands are loaded together
    const long csz = ((K + nchunk - 1) / nchunk + 16 * U - 1) / (16 * U) * (16 * U);
    const long c0 = (long)blockIdx.x * csz;
    const long c1 = min(K, c0 + csz);
    dvec4 acc = {0.0, 0.0, 0.0, 0.0};
    for (long cb = c0 + 4 * wave; cb < c1; cb += 16 * U) {
        int ok[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long c = cb + 16 * u + hi;
            ok[u] = gload(pk + (c < c1 ? c : c0));
        }
        double yi[U], yj[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            yi[u] = gload(px + oi + ok[u]);
            yj[u] = gload(px + oj + ok[u]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool in = cb + 16 * u + hi < c1;
            const double a = (in && ai < L) ? yi[u] : 0.0;
            const double b = (in && aj < L) ? yj[u] : 0.0;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
        }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) red[wave][(4 * v + hi) * 16 + lo] = acc[v];
    __syncthreads();
    const int e = threadIdx.x;
    part[((long)blockIdx.y * 256 + e) * nchunk + blockIdx.x] = (red[0][e] + red[1][e]) + (red[2][e] + red[3][e]);
}

// Places the summed tiles of S (out[tile * 256 + 16 i + j]) into a
// column-major matrix of leading dimension ld (the projected-matrix buffer,
// ld = kMaxBasis, or an L x L array), mirroring the off-diagonal tiles.  One
// workgroup per tile.
__global__ void __launch_bounds__(256)
k_xgram_place(const double* __restrict__ out, int L, long ld, double* __restrict__ Bm) {
    const int nb = (L + 15) / 16;
    int k = blockIdx.x, ib = 0;
    while (k >= nb - ib) {
        k -= nb - ib;
        ++ib;
    }
    const int jb = ib + k;
    const int e = threadIdx.x, i = ib * 16 + e / 16, j = jb * 16 + e % 16;
    if (i >= L || j >= L) return;
    const double v = out[(long)blockIdx.x * 256 + e];
    Bm[(long)j * ld + i] = v;
    if (ib != jb) Bm[(long)i * ld + j] = v;
}

// ------------------------------------------------------------------------
// eigen method for windows beyond the small-SVD kernel: block one-sided
// Jacobi on S (L x L, column-major, symmetric positive semi-definite).  Its
// columns are split into blocks of kBjW; in each round every workgroup
// takes one pair of blocks M (L x 2 kBjW), forms the Gram G = M^T M,
// diagonalises it by cyclic two-sided Jacobi (J^T G J diagonal, J
// orthogonal, accumulated) and replaces M by M J.  The rounds of a sweep
// pair every two blocks once (circle method).  When no pair has a Gram
// entry above tol sqrt(G_kk G_ll), the columns are mutually orthogonal:
// column j is lambda_j u_j, lambda_j = |column j| an eigenvalue of S and
// u_j its eigenvector (S V = U Sigma with U = V for S symmetric PSD).
// ------------------------------------------------------------------------

// Column of S behind position k (0 .. kBjN-1) of the block pair, or -1
// (a block index < 0 is the empty block of an odd count).
__device__ __forceinline__ int bj_col(int2 pr, int k, int L) {
    const int blk = k < kBjW ? pr.x : pr.y;
    const int c = blk * kBjW + (k % kBjW);
    return (blk >= 0 && c < L) ? c : -1;
}

// One workgroup per block pair: Gram, convergence test (flag[0] = 1 if an
// off-diagonal Gram entry exceeds both tol sqrt(G_kk G_ll) and floor_abs,
// an absolute level below which two columns far under the matrix's scale
// are left as they are), rotation J into
// Jout[pair] (row-major kBjN x kBjN); flag[1] = 1 if the inner iteration
// ran out of sweeps.
__global__ void __launch_bounds__(256)
k_bj_pair(const double* __restrict__ A, int L, const int2* __restrict__ pairs, double* __restrict__ Jout,
          int* __restrict__ flag, double tol, double floor_abs) {
    __shared__ double G[kBjN][kBjN + 1];
    __shared__ double J[kBjN][kBjN + 1];
    __shared__ double tile[64][kBjN + 1];
    __shared__ double cs[kBjN / 2][2];
    __shared__ int pq[kBjN / 2][2];
    __shared__ int rot;
    const int2 pr = pairs[blockIdx.x];
    const int t = threadIdx.x;
    constexpr int NE = kBjN * kBjN / 256;   // Gram entries per thread
    double acc[NE];
#pragma unroll
    for (int u = 0; u < NE; ++u) acc[u] = 0.0;
    for (int i0 = 0; i0 < L; i0 += 64) {
        for (int e = t; e < 64 * kBjN; e += 256) {
            const int i = e % 64, k = e / 64;
            const int c = bj_col(pr, k, L);
            tile[i][k] = (c >= 0 && i0 + i < L) ? A[(long)c * L + i0 + i] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < NE; ++u) {
            const int e = t + 256 * u, k = e / kBjN, l = e % kBjN;
            double sum = 0.0;
            for (int i = 0; i < 64; ++i) sum += tile[i][k] * tile[i][l];
            acc[u] += sum;
        }
        __syncthreads();
    }
    if (t == 0) rot = 0;
#pragma unroll
    for (int u = 0; u < NE; ++u) {
        const int e = t + 256 * u, k = e / kBjN, l = e % kBjN;
        G[k][l] = acc[u];
        J[k][l] = k == l ? 1.0 : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NE; ++u) {
        const int e = t + 256 * u, k = e / kBjN, l = e % kBjN;
        if (k != l && fabs(G[k][l]) > tol * sqrt(G[k][k] * G[l][l]) && fabs(G[k][l]) > floor_abs) rot = 1;
    }
    __syncthreads();
    if (rot == 0) {
        // already orthogonal: J = I
        for (int e = t; e < kBjN * kBjN; e += 256) Jout[(long)blockIdx.x * kBjN * kBjN + e] = (e / kBjN == e % kBjN);
        return;
    }
    if (t == 0) flag[0] = 1;
    bool done = false;
    for (int sweep = 0; sweep < 40 && !done; ++sweep) {
        __syncthreads();
        if (t == 0) rot = 0;
        __syncthreads();
        for (int r = 0; r < kBjN - 1; ++r) {
            if (t < kBjN / 2) {
                // circle method: position kBjN-1 fixed, the others rotate
                const int a = t == 0 ? kBjN - 1 : (r + t) % (kBjN - 1);
                const int b = t == 0 ? r : (r - t + kBjN - 1) % (kBjN - 1);
                const int p = min(a, b), q = max(a, b);
                const double gpp = G[p][p], gqq = G[q][q], gpq = G[p][q];
                double c = 1.0, sn = 0.0;
                if (gpq != 0.0 && fabs(gpq) > tol * sqrt(gpp * gqq) && fabs(gpq) > floor_abs) {
                    // J^T G J zeroes (p, q): t = s / c is the smaller root of
                    // t^2 + 2 theta t - 1 = 0, theta = (G_qq - G_pp) / (2 G_pq)
                    const double th = (gqq - gpp) / (2.0 * gpq);
                    const double tt = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1.0 + th * th));
                    c = 1.0 / sqrt(1.0 + tt * tt);
                    sn = tt * c;
                    rot = 1;
                }
                pq[t][0] = p;
                pq[t][1] = q;
                cs[t][0] = c;
                cs[t][1] = sn;
            }
            __syncthreads();
            // G J and J J_r: columns p, q of each pair (pairs are disjoint)
            for (int e = t; e < (kBjN / 2) * kBjN; e += 256) {
                const int pi = e / kBjN, k = e % kBjN;
                const double c = cs[pi][0], sn = cs[pi][1];
                if (sn == 0.0) continue;
                const int p = pq[pi][0], q = pq[pi][1];
                const double gp = G[k][p], gq = G[k][q];
                G[k][p] = c * gp - sn * gq;
                G[k][q] = sn * gp + c * gq;
                const double jp = J[k][p], jq = J[k][q];
                J[k][p] = c * jp - sn * jq;
                J[k][q] = sn * jp + c * jq;
            }
            __syncthreads();
            // J_r^T (G J_r): rows p, q; the rotated pair's entry is zero by
            // construction (set exactly rather than left at rounding level,
            // which the relative test could not pass when G_pp >> G_qq)
            for (int e = t; e < (kBjN / 2) * kBjN; e += 256) {
                const int pi = e / kBjN, k = e % kBjN;
                const double c = cs[pi][0], sn = cs[pi][1];
                if (sn == 0.0) continue;
                const int p = pq[pi][0], q = pq[pi][1];
                const double gp = G[p][k], gq = G[q][k];
                G[p][k] = k == q ? 0.0 : c * gp - sn * gq;
                G[q][k] = k == p ? 0.0 : sn * gp + c * gq;
            }
            __syncthreads();
        }
        done = rot == 0;
    }
    if (!done && t == 0) flag[1] = 1;
    for (int e = t; e < kBjN * kBjN; e += 256) Jout[(long)blockIdx.x * kBjN * kBjN + e] = J[e / kBjN][e % kBjN];
}

// M = M J for the columns of each block pair, rows in chunks of 64: grid
// (row chunks, pairs).  Each workgroup reads its whole chunk before writing
// it back, and the pairs of a round own disjoint columns.
__global__ void __launch_bounds__(256)
k_bj_apply(double* __restrict__ A, int L, const int2* __restrict__ pairs, const double* __restrict__ Jin) {
    __shared__ double M[64][kBjN + 1];
    __shared__ double J[kBjN][kBjN + 1];
    const int2 pr = pairs[blockIdx.y];
    const int i0 = blockIdx.x * 64;
    const int t = threadIdx.x;
    const double* Jp = Jin + (long)blockIdx.y * kBjN * kBjN;
    for (int e = t; e < kBjN * kBjN; e += 256) J[e / kBjN][e % kBjN] = Jp[e];
    for (int e = t; e < 64 * kBjN; e += 256) {
        const int i = e % 64, k = e / 64;
        const int c = bj_col(pr, k, L);
        M[i][k] = (c >= 0 && i0 + i < L) ? A[(long)c * L + i0 + i] : 0.0;
    }
    __syncthreads();
    for (int e = t; e < 64 * kBjN; e += 256) {
        const int i = e % 64, l = e / 64;
        const int c = bj_col(pr, l, L);
        if (c < 0 || i0 + i >= L) continue;
        double sum = 0.0;
        for (int k = 0; k < kBjN; ++k) sum += M[i][k] * J[k][l];
        A[(long)c * L + i0 + i] = sum;
    }
}

// lam[c] = |column c of A| (one wave per column, fixed order).
__global__ void __launch_bounds__(256)
k_bj_norms(const double* __restrict__ A, int L, double* __restrict__ lam) {
    const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (c >= L) return;
    double sum = 0.0;
    for (int i = lane_id(); i < L; i += 64) {
        const double v = A[(long)c * L + i];
        sum += v * v;
    }
    sum = wave_sum(sum);
    if (lane_id() == 0) lam[c] = sqrt(sum);
}

// U_c = column perm[c] of A / lam[perm[c]] (0 for lam = 0), sigma_c =
// sqrt(lam[perm[c]]), c < r.
__global__ void __launch_bounds__(256)
k_bj_take(const double* __restrict__ A, int L, const int* __restrict__ perm, const double* __restrict__ lam,
          double* __restrict__ U, double* __restrict__ sigma, int r) {
    for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < (long)L * r; e += (long)gridDim.x * 256) {
        const int c = (int)(e / L), i = (int)(e % L);
        const int j = perm[c];
        const double l = lam[j];
        U[(long)c * L + i] = l > 0.0 ? A[(long)j * L + i] / l : 0.0;
    }
    if (blockIdx.x == 0)
        for (int c = threadIdx.x; c < r; c += 256) sigma[c] = sqrt(lam[perm[c]]);
}

// After the SVD of the symmetric positive semi-definite S (its left singular
// vectors are eigenvectors, its singular values the eigenvalues):
// U_c = eigenvector of the c-th largest eigenvalue, sigma_c = sqrt(lambda_c)
// (rounding can leave a vanishing eigenvalue slightly negative: 0).
__global__ void __launch_bounds__(256)
k_eig_take(const LzDesc* __restrict__ lzs, const ResDesc* __restrict__ res, const Item* __restrict__ items, int L,
           int r) {
    const int inst = items[blockIdx.x].inst;
    const LzDesc& lz = lzs[inst];
    const ResDesc& rs = res[inst];
    for (int e = threadIdx.x; e < L * r; e += 256) {
        const int c = e / L, i = e % L;
        rs.U[(long)c * L + i] = lz.Yl[(long)lz.perm[c] * kMaxBasis + i];
    }
    for (int c = threadIdx.x; c < r; c += 256) rs.sigma[c] = sqrt(fmax(lz.sig[c], 0.0));
}

// out[e] = sum over the chunks of part[e * nchunk + chunk]: one wave per
// entry, lanes over the chunks, then a fixed-order wave sum.
__global__ void __launch_bounds__(256)
k_wgram_sum(const double* __restrict__ part, int nent, int nchunk, double* __restrict__ out) {
    const int e = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (e >= nent) return;
    double s = 0.0;
    for (int q = lane_id(); q < nchunk; q += 64) s += part[(long)e * nchunk + q];
    s = wave_sum(s);
    if (lane_id() == 0) out[e] = s;
}

// ------------------------------------------------------------------------
// recurrent forecast (column form)
// ------------------------------------------------------------------------

// Sum of v over the 256 threads of the workgroup in a fixed order; every
// thread gets the total.
__device__ __forceinline__ double block_sum256(double v, double* red) {
    v = wave_sum(v);
    __syncthreads();
    if (lane_id() == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}

// LRR coefficients R[k] = sum_j pi_j U_j[k] / (1 - nu^2), k < L - 1, with
// pi_j = U_j[L - 1] the last coordinate of group component j and nu^2 =
// sum_j pi_j^2.  U: L x r column-major.  One workgroup; flag[0] = 1 when
// nu^2 >= 1 (no forecast).
__global__ void __launch_bounds__(256)
k_lrr(const double* __restrict__ U, long L, const int* __restrict__ grp, int ng, double* __restrict__ R,
      int* __restrict__ flag) {
    __shared__ double red[4];
    double p2 = 0.0;
    for (int j = threadIdx.x; j < ng; j += 256) {
        const double pj = U[(long)grp[j] * L + (L - 1)];
        p2 += pj * pj;
    }
    const double nu2 = block_sum256(p2, red);
    if (threadIdx.x == 0) flag[0] = nu2 < 1.0 ? 0 : 1;
    const double sc = nu2 < 1.0 ? 1.0 / (1.0 - nu2) : 0.0;
    for (long k = threadIdx.x; k < L - 1; k += 256) {
        double s = 0.0;
        for (int j = 0; j < ng; ++j) s += U[(long)grp[j] * L + (L - 1)] * U[(long)grp[j] * L + k];
        R[k] = s * sc;
    }
}

// Forecast of h values of series a (internal row a of the reconstruction
// rec, A x B): n_a = the covered cells of the row (a prefix), then x_{n+1} =
// sum_k R_k x_{n-L+1+k} over the last L - 1 values, by recurrence.  One
// workgroup per row; buf (per row, L - 1 + h values) holds the running
// window; out[a * h + k].
__global__ void __launch_bounds__(256)
k_rforecast(const double* __restrict__ rec, const double* __restrict__ W, int B, const double* __restrict__ R,
            long L, int h, double* __restrict__ buf, double* __restrict__ out) {
    __shared__ double red[4];
    __shared__ int nmax[4];
    const int a = blockIdx.x;
    const long L1 = L - 1;
    // covered length of the row: one past its last cell with W > 0
    int last = 0;
    for (int b = threadIdx.x; b < B; b += 256)
        if (W[(long)a * B + b] > 0) last = max(last, b + 1);
    for (int o = 32; o > 0; o >>= 1) last = max(last, __shfl_xor(last, o));
    if (lane_id() == 0) nmax[threadIdx.x >> 6] = last;
    __syncthreads();
    const int n = max(max(nmax[0], nmax[1]), max(nmax[2], nmax[3]));
    double* bw = buf + (long)a * (L1 + h);
    for (long k = threadIdx.x; k < L1; k += 256) bw[k] = n - L1 + k >= 0 ? rec[(long)a * B + n - L1 + k] : 0.0;
    __syncthreads();
    for (int s = 0; s < h; ++s) {
        double p = 0.0;
        for (long k = threadIdx.x; k < L1; k += 256) p += R[k] * bw[s + k];
        const double v = block_sum256(p, red);
        if (threadIdx.x == 0) {
            bw[L1 + s] = v;
            out[(long)a * h + s] = v;
        }
        __syncthreads();
    }
}

// Broadcast of lane j's value to the whole wave (j wave-uniform).
__device__ __forceinline__ double lane_bcast(double v, int j) {
    const long long b = __double_as_longlong(v);
    const unsigned lo = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(b), j));
    const long long hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), j);
    return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

// Vector forecast, shift part: M[i * ng + j] = sum_{l < L-1} U_{g_i}[l]
// U_{g_j}[l + 1], the group's window vectors without their last coordinate
// against the same vectors without their first.  One wave per entry.
__global__ void __launch_bounds__(256)
k_vf_shift(const double* __restrict__ U, long L, const int* __restrict__ grp, int ng, double* __restrict__ M) {
    const int e = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (e >= ng * ng) return;   // whole waves
    const double* ui = U + (long)grp[e / ng] * L;
    const double* uj = U + (long)grp[e % ng] * L + 1;
    double s = 0.0;
    for (long l = lane_id(); l < L - 1; l += 64) s += ui[l] * uj[l];
    s = wave_sum(s);
    if (lane_id() == 0) M[e] = s;
}

// Column vector forecast of series a (internal row a), by the fast
// algorithm of the forecast implementation section: the lagged vectors of
// the continuation stay in the group's span, so only their coefficient
// vectors are carried, w_k = D w_{k-1} with
// D = (I + pi pi^T / (1 - nu^2)) M.  For an orthonormal basis that is the
// pseudo-inverse of the basis without its last row times the basis without
// its first row (pi: the last row, nu^2 = |pi|^2).  w_0 = sigma_j V_j at
// the row's last origin cell; forecast t is the mean over i < L of
// (U w_{L-1+t-i})_i, the anti-diagonal of the extended matrix through
// position n + t.  wbuf: per row (h + L - 1) x ng.  flag[0] = 1: a row
// whose last lagged vector does not end at its covered end; flag[1] = 1:
// nu^2 >= 1.  Such rows get NaN.
__global__ void __launch_bounds__(256)
k_vforecast(const double* __restrict__ U, long L, const double* __restrict__ V, long K,
            const double* __restrict__ sigma, const int* __restrict__ grp, int ng, const double* __restrict__ M,
            const int* __restrict__ krow, const uint8_t* __restrict__ kmask, int KB, const double* __restrict__ W,
            int B, int h, double* __restrict__ wbuf, double* __restrict__ out, int* __restrict__ flag) {
    constexpr int LD = kVfMaxGroup + 1;
    __shared__ double Ds[kVfMaxGroup * LD];
    __shared__ double pis[kVfMaxGroup], cs[kVfMaxGroup];
    __shared__ int ext[2][4];
    const int a = blockIdx.x, tid = threadIdx.x, wv = tid >> 6, lane = lane_id();
    const long E = (long)h + L - 1;
    // covered length n of the row and its last origin column
    int last = 0, klast = -1;
    for (int b = tid; b < B; b += 256)
        if (W[(long)a * B + b] > 0) last = b + 1;
    for (int b = tid; b < KB; b += 256)
        if (kmask[(long)a * KB + b]) klast = b;
    for (int o = 32; o > 0; o >>= 1) {
        last = max(last, __shfl_xor(last, o));
        klast = max(klast, __shfl_xor(klast, o));
    }
    if (lane == 0) {
        ext[0][wv] = last;
        ext[1][wv] = klast;
    }
    if (tid < ng) pis[tid] = U[(long)grp[tid] * L + (L - 1)];
    __syncthreads();
    const int n = max(max(ext[0][0], ext[0][1]), max(ext[0][2], ext[0][3]));
    const int kl = max(max(ext[1][0], ext[1][1]), max(ext[1][2], ext[1][3]));
    double nu2 = 0.0;
    for (int j = 0; j < ng; ++j) nu2 += pis[j] * pis[j];
    const bool row_ok = kl >= 0 && kl + L == n;
    if (!row_ok || !(nu2 < 1.0)) {
        if (tid == 0) flag[row_ok ? 1 : 0] = 1;
        for (int t = tid; t < h; t += 256) out[(long)a * h + t] = __builtin_nan("");
        return;
    }
    if (tid < ng) {
        double c = 0.0;
        for (int i = 0; i < ng; ++i) c += pis[i] * M[i * ng + tid];
        cs[tid] = c;
    }
    __syncthreads();
    const double sc = 1.0 / (1.0 - nu2);
    for (int e = tid; e < ng * ng; e += 256) {
        const int i = e / ng, j = e % ng;
        Ds[i * LD + j] = M[e] + pis[i] * cs[j] * sc;
    }
    __syncthreads();
    double* wb = wbuf + (long)a * E * ng;
    if (wv == 0) {
        // the recursion: lane i holds coordinate i of w
        const long kidx = krow[a + 1] - 1;
        double w = lane < ng ? sigma[grp[lane]] * V[(long)grp[lane] * K + kidx] : 0.0;
        const double* drow = Ds + (lane < ng ? lane : 0) * LD;
        for (long e = 0; e < E; ++e) {
            double s = 0.0;
            for (int j = 0; j < ng; ++j) s += drow[j] * lane_bcast(w, j);
            w = s;
            if (lane < ng) wb[e * ng + lane] = w;
        }
    }
    __syncthreads();
    // forecasts: one wave per value, lanes over the window coordinates
    for (int t = wv; t < h; t += 4) {
        double s = 0.0;
        for (long i = lane; i < L; i += 64) {
            const double* we = wb + (L - 1 + t - i) * ng;
            for (int j = 0; j < ng; ++j) s += U[(long)grp[j] * L + i] * we[j];
        }
        s = wave_sum(s);
        if (lane == 0) out[(long)a * h + t] = s / (double)L;
    }
}

// Roots (wr, wi; n values) into re/im by decreasing modulus, then
// decreasing imaginary part (selection; taken: n values of scratch).
__device__ inline void order_roots(const double* wr, const double* wi, int n, double* taken, double* re,
                                   double* im) {
    for (int k = 0; k < n; ++k) taken[k] = 0.0;
    for (int p = 0; p < n; ++p) {
        int best = -1;
        double bm = 0.0;
        for (int k = 0; k < n; ++k) {
            if (taken[k] != 0.0) continue;
            const double mk = sqrt(wr[k] * wr[k] + wi[k] * wi[k]);
            if (best < 0 || mk > bm || (mk == bm && wi[k] > wi[best])) {
                best = k;
                bm = mk;
            }
        }
        taken[best] = 1.0;
        re[p] = wr[best];
        im[p] = wi[best];
    }
}

// LS-ESPRIT roots of a group: the eigenvalues of its shift matrix
// D = (I + pi pi^T / (1 - nu^2)) M (as for the vector forecast: the
// pseudo-inverse of the group's U without its last row times U without its
// first), sorted by decreasing modulus, then decreasing imaginary part.
// One wave builds D in LDS; its first lane runs the sequential eigenvalue
// iteration (the matrix has at most 64 rows).  flag[0] = 1: nu^2 >= 1;
// flag[1] = 1: the iteration did not converge.
__global__ void __launch_bounds__(64)
k_esprit(const double* __restrict__ U, long L, const int* __restrict__ grp, int ng, const double* __restrict__ M,
         double* __restrict__ re, double* __restrict__ im, int* __restrict__ flag) {
    constexpr int LD = kVfMaxGroup + 1;
    __shared__ double Ds[kVfMaxGroup * LD];
    __shared__ double pis[kVfMaxGroup], cs[kVfMaxGroup], work[kVfMaxGroup], wr[kVfMaxGroup], wi[kVfMaxGroup];
    const int lane = threadIdx.x;
    if (lane < ng) pis[lane] = U[(long)grp[lane] * L + (L - 1)];
    __syncthreads();
    double nu2 = 0.0;
    for (int j = 0; j < ng; ++j) nu2 += pis[j] * pis[j];
    if (!(nu2 < 1.0)) {
        if (lane == 0) flag[0] = 1;
        return;
    }
    if (lane < ng) {
        double c = 0.0;
        for (int i = 0; i < ng; ++i) c += pis[i] * M[i * ng + lane];
        cs[lane] = c;
    }
    __syncthreads();
    const double sc = 1.0 / (1.0 - nu2);
    for (int e = lane; e < ng * ng; e += 64) {
        const int i = e / ng, j = e % ng;
        Ds[i * LD + j] = M[e] + pis[i] * cs[j] * sc;
    }
    __syncthreads();
    if (lane != 0) return;
    if (eig_real<double>(Ds, ng, LD, work, wr, wi) != 0) flag[1] = 1;
    order_roots(wr, wi, ng, work, re, im);
}

// TLS-ESPRIT Gram matrix of Z = [U_low : U_high] (U_low: the group's U
// without its last row, U_high without its first): g (2 ng x 2 ng,
// row-major) = [[U_low^T U_low, U_low^T U_high], [U_high^T U_low,
// U_high^T U_high]], summed explicitly (the blocks are I - pi pi^T, M and
// I - rho rho^T only for an exactly orthonormal U).  One wave per (i, j).
__global__ void __launch_bounds__(256)
k_tls_gram(const double* __restrict__ U, long L, const int* __restrict__ grp, int ng, double* __restrict__ g) {
    const int e = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (e >= ng * ng) return;   // whole waves
    const int i = e / ng, j = e % ng, n = 2 * ng;
    const double* ui = U + (long)grp[i] * L;
    const double* uj = U + (long)grp[j] * L;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (long l = lane_id(); l < L - 1; l += 64) {
        const double a = ui[l], b = ui[l + 1], c = uj[l], d = uj[l + 1];
        s0 += a * c;
        s1 += a * d;
        s2 += b * d;
    }
    s0 = wave_sum(s0);
    s1 = wave_sum(s1);
    s2 = wave_sum(s2);
    if (lane_id() == 0) {
        g[i * n + j] = s0;
        g[i * n + ng + j] = s1;
        g[(ng + j) * n + i] = s1;
        g[(ng + i) * n + ng + j] = s2;
    }
}

// TLS-ESPRIT roots from that Gram matrix: its eigenvectors by decreasing
// eigenvalue are Z's right singular vectors, the shift matrix is
// -V12 V22^{-1}, its eigenvalues the roots, ordered as for k_esprit.  The
// first lane works in LDS (ng <= kTlsMaxGroup).  flag[0] = 1: V22 singular;
// flag[1] = 1: an eigenvalue iteration did not converge.
__global__ void __launch_bounds__(64)
k_esprit_tls(const double* __restrict__ g, int ng, double* __restrict__ re, double* __restrict__ im,
             int* __restrict__ flag) {
    constexpr int NM = 2 * kTlsMaxGroup;
    __shared__ double gs[NM * NM], vec[NM * NM], lu[kTlsMaxGroup * NM], phi[kTlsMaxGroup * kTlsMaxGroup];
    __shared__ double w[NM], work[kTlsMaxGroup], wr[kTlsMaxGroup], wi[kTlsMaxGroup];
    __shared__ int order[NM];
    const int n = 2 * ng;
    for (int e = threadIdx.x; e < n * n; e += 64) gs[e] = g[e];
    __syncthreads();
    if (threadIdx.x != 0) return;
    const int rc = tls_shift<double>(gs, ng, vec, w, order, lu, phi);
    if (rc != 0) {
        flag[rc == -2 ? 0 : 1] = 1;
        return;
    }
    if (eig_real<double>(phi, ng, ng, work, wr, wi) != 0) flag[1] = 1;
    order_roots(wr, wi, ng, work, re, im);
}

// 2D-ESPRIT, Gram terms over index pairs: out[i * ng + j] = sum_p
// U_{g_i}[pa[p]] U_{g_j}[pb[p]] (window cells and their neighbours one step
// along an axis, or the cells without one paired with themselves).  One
// wave per entry.
__global__ void __launch_bounds__(256)
k_pairgram(const double* __restrict__ U, long L, const int* __restrict__ grp, int ng, const int* __restrict__ pa,
           const int* __restrict__ pb, int np, double* __restrict__ out) {
    const int e = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (e >= ng * ng) return;   // whole waves
    const double* ui = U + (long)grp[e / ng] * L;
    const double* uj = U + (long)grp[e % ng] * L;
    double s = 0.0;
    for (int p = lane_id(); p < np; p += 64) s += ui[pa[p]] * uj[pb[p]];
    s = wave_sum(s);
    if (lane_id() == 0) out[e] = s;
}

// 2D-ESPRIT pairing: the joint eigenvalues (lambda_k, mu_k) of the x and y
// shift matrices px, py (ng x ng, leading dimension ng), through the
// eigenvectors of px + gamma py, ordered by decreasing |lambda|, then
// decreasing Im lambda.  One thread (the matrices have at most 64 rows);
// scr: scratch of 3 ng^2 + 14 ng values.  flag[2] = 1: the eigenvalue
// iteration failed.
__global__ void __launch_bounds__(64)
k_esprit2d(const double* __restrict__ px, const double* __restrict__ py, int ng, double gamma,
           double* __restrict__ scr, double* __restrict__ out, int* __restrict__ flag) {
    if (threadIdx.x != 0) return;
    double* c = scr;
    double* lu = c + ng * ng;
    double* work = lu + 2 * ng * ng;
    double* v = work + ng;
    double* y = v + 2 * ng;
    double* t = y + 2 * ng;
    double* wr = t + 2 * ng;
    double* wi = wr + ng;
    double* lre = wi + ng;
    double* lim = lre + ng;
    double* mre = lim + ng;
    double* mim = mre + ng;
    int* piv = reinterpret_cast<int*>(mim + ng);
    if (joint_eig<double>(px, py, ng, ng, gamma, c, work, piv, lu, v, y, t, wr, wi, lre, lim, mre, mim) != 0) {
        flag[2] = 1;
        return;
    }
    for (int k = 0; k < ng; ++k) work[k] = 0.0;
    for (int p = 0; p < ng; ++p) {
        int best = -1;
        double bm = 0.0;
        for (int k = 0; k < ng; ++k) {
            if (work[k] != 0.0) continue;
            const double mk = sqrt(lre[k] * lre[k] + lim[k] * lim[k]);
            if (best < 0 || mk > bm || (mk == bm && lim[k] > lim[best])) {
                best = k;
                bm = mk;
            }
        }
        work[best] = 1.0;
        out[p] = lre[best];
        out[ng + p] = lim[best];
        out[2 * ng + p] = mre[best];
        out[3 * ng + p] = mim[best];
    }
}

// ---- row forecasts (MSSA): V's blocks are the series' origin rows ------

// Row forecasts need every series' origin set to be a prefix [0, K_p) of
// its row (no gaps; then its covered cells are [0, K_p + L - 1)).
// flag[0] = 1 otherwise.  One workgroup per row.
__global__ void __launch_bounds__(256)
k_rowf_check(const uint8_t* __restrict__ kmask, int KB, const int* __restrict__ krow, int* __restrict__ flag) {
    __shared__ int ext[4];
    const int a = blockIdx.x, tid = threadIdx.x;
    int klast = -1;
    for (int b = tid; b < KB; b += 256)
        if (kmask[(long)a * KB + b]) klast = b;
    for (int o = 32; o > 0; o >>= 1) klast = max(klast, __shfl_xor(klast, o));
    if (lane_id() == 0) ext[tid >> 6] = klast;
    __syncthreads();
    const int kl = max(max(ext[0], ext[1]), max(ext[2], ext[3]));
    const int kp = krow[a + 1] - krow[a];
    if (tid == 0 && kl != kp - 1) flag[0] = 1;
}

// Gram terms of the group's row-space basis Q (the V_j, blocks by series):
// e < ng^2:  Mr[i][j] = sum over blocks of sum_{k < K_p - 1} Q_i[k] Q_j[k+1]
//            (blocks without their last coordinate against blocks without
//            their first), as the sum over all adjacent pairs minus the
//            pairs that cross from one block into the next;
// e >= ng^2: StS[i][j] = sum_p Q_i[end_p] Q_j[end_p] over the blocks' last
//            coordinates.  One wave per entry.
__global__ void __launch_bounds__(256)
k_rowf_gram(const double* __restrict__ V, long K, const int* __restrict__ krow, int A, const int* __restrict__ grp,
            int ng, double* __restrict__ Mr, double* __restrict__ StS) {
    const int e = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = lane_id();
    if (e >= 2 * ng * ng) return;   // whole waves
    const int q = e < ng * ng ? e : e - ng * ng;
    const double* vi = V + (long)grp[q / ng] * K;
    const double* vj = V + (long)grp[q % ng] * K;
    double s = 0.0;
    if (e < ng * ng) {
        for (long c = lane; c < K - 1; c += 64) s += vi[c] * vj[c + 1];
        for (int p = lane; p < A; p += 64) {
            const int b = krow[p], en = krow[p + 1];
            if (en > b && en < K) s -= vi[en - 1] * vj[en];
        }
        s = wave_sum(s);
        if (lane == 0) Mr[q] = s;
    } else {
        for (int p = lane; p < A; p += 64) {
            const int b = krow[p], en = krow[p + 1];
            if (en > b) s += vi[en - 1] * vj[en - 1];
        }
        s = wave_sum(s);
        if (lane == 0) StS[q] = s;
    }
}

// Solves (I - StS) [D | G] = [Mr | I] by Gauss-Jordan elimination without
// pivoting (I - StS is symmetric positive definite when the forecast
// exists; a pivot below 1e-12 sets flag[1]).  T: ng x 3ng work array.
// D = (I - S^T S)^{-1} Mr is the row shift matrix (pseudo-inverse of the
// blocks without their last coordinate times the blocks without their
// first, for an orthonormal basis); G = (I - S^T S)^{-1}.  One workgroup.
__global__ void __launch_bounds__(256)
k_rowf_solve(const double* __restrict__ StS, const double* __restrict__ Mr, int ng, double* __restrict__ T,
             double* __restrict__ D, double* __restrict__ G, int* __restrict__ flag) {
    __shared__ double fac[kVfMaxGroup];
    __shared__ int bad;
    const int tid = threadIdx.x, nc = 3 * ng;
    if (tid == 0) bad = 0;
    for (int e = tid; e < ng * nc; e += 256) {
        const int i = e / nc, c = e % nc;
        double v;
        if (c < ng) v = (i == c ? 1.0 : 0.0) - StS[i * ng + c];
        else if (c < 2 * ng) v = Mr[i * ng + (c - ng)];
        else v = (i == c - 2 * ng) ? 1.0 : 0.0;
        T[e] = v;
    }
    __syncthreads();
    for (int kk = 0; kk < ng; ++kk) {
        const double piv = T[kk * nc + kk];
        if (!(piv > 1e-12)) {
            if (tid == 0) bad = 1;
            break;   // uniform: every thread read the same pivot
        }
        if (tid < ng) fac[tid] = T[tid * nc + kk];
        __syncthreads();
        for (int c = tid; c < nc; c += 256) T[kk * nc + c] /= piv;
        __syncthreads();
        for (int e = tid; e < ng * nc; e += 256) {
            const int i = e / nc, c = e % nc;
            if (i != kk) T[e] -= fac[i] * T[kk * nc + c];
        }
        __syncthreads();
    }
    __syncthreads();
    if (bad) {
        if (tid == 0) flag[1] = 1;
        return;
    }
    for (int e = tid; e < ng * ng; e += 256) {
        const int i = e / ng, j = e % ng;
        D[e] = T[i * nc + ng + j];
        G[e] = T[i * nc + 2 * ng + j];
    }
}

// Vector row forecast, the recursion shared by all series: the coefficient
// vectors of the trajectory rows in the group's basis, w_L = D w_{L-1},
// ... from w_{L-1} = sigma_j U_j[L-1] (the last row of the reconstructed
// matrix); wbuf[e * ng + j] holds w_{L+e}, e < E.  One wave.
__global__ void __launch_bounds__(64)
k_vrow_recur(const double* __restrict__ U, long L, const double* __restrict__ sigma, const int* __restrict__ grp,
             int ng, const double* __restrict__ D, long E, double* __restrict__ wbuf) {
    constexpr int LD = kVfMaxGroup + 1;
    __shared__ double Ds[kVfMaxGroup * LD];
    const int lane = threadIdx.x;
    for (int e = lane; e < ng * ng; e += 64) Ds[(e / ng) * LD + e % ng] = D[e];
    __syncthreads();
    double w = lane < ng ? sigma[grp[lane]] * U[(long)grp[lane] * L + (L - 1)] : 0.0;
    const double* drow = Ds + (lane < ng ? lane : 0) * LD;
    for (long e = 0; e < E; ++e) {
        double s = 0.0;
        for (int j = 0; j < ng; ++j) s += drow[j] * lane_bcast(w, j);
        w = s;
        if (lane < ng) wbuf[e * ng + lane] = w;
    }
}

// Vector row forecast of series a: position N_p + m is the mean over the
// block's K_p columns k of (Q^(p) w_{L+K_p-1+m-k})_k, all rows past the
// reconstructed ones.  One workgroup per series, one wave per value.
__global__ void __launch_bounds__(256)
k_vrow_out(const double* __restrict__ V, long K, const int* __restrict__ krow, const int* __restrict__ grp, int ng,
           const double* __restrict__ wbuf, int h, double* __restrict__ out) {
    const int a = blockIdx.x, wv = threadIdx.x >> 6, lane = lane_id();
    const int b0 = krow[a], kp = krow[a + 1] - b0;
    for (int m = wv; m < h; m += 4) {
        double s = 0.0;
        for (int k = lane; k < kp; k += 64) {
            const double* we = wbuf + (long)(kp - 1 + m - k) * ng;
            for (int j = 0; j < ng; ++j) s += V[(long)grp[j] * K + b0 + k] * we[j];
        }
        s = wave_sum(s);
        if (lane == 0) out[(long)a * h + m] = kp > 0 ? s / kp : __builtin_nan("");
    }
}

// Recurrent row forecast, the part from reconstructed values: for step m
// (next values N_p + m) and component j, the sum over series of
// Q_j^(p)[k] x^(p)[L + m + k] over the k < K_p - 1 - m whose value lies in
// the reconstruction rec (A x B).  One wave per (m, j).
__global__ void __launch_bounds__(256)
k_rrow_known(const double* __restrict__ V, long K, const int* __restrict__ krow, int A, const int* __restrict__ grp,
             int ng, const double* __restrict__ rec, int B, long L, int h, double* __restrict__ yk) {
    const int e = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = lane_id();
    if (e >= h * ng) return;   // whole waves
    const int m = e / ng, j = e % ng;
    const double* vj = V + (long)grp[j] * K;
    double s = 0.0;
    for (int p = 0; p < A; ++p) {
        const int b0 = krow[p], kn = krow[p + 1] - b0 - 1 - m;
        for (int k = lane; k < kn; k += 64) s += vj[b0 + k] * rec[(long)p * B + L + m + k];
    }
    s = wave_sum(s);
    if (lane == 0) yk[e] = s;
}

// Recurrent row forecast by recurrence: step m adds to yk[m] the terms whose
// values are earlier forecasts, y = Vlow^T Z; then the next value of every
// series is (S G y)_p with S the blocks' last coordinates.  out (A x h)
// doubles as the store of the forecasts.  One workgroup.
__global__ void __launch_bounds__(256)
k_rrow_recur(const double* __restrict__ V, long K, const int* __restrict__ krow, int A, const int* __restrict__ grp,
             int ng, const double* __restrict__ G, const double* __restrict__ yk, int h, double* __restrict__ out) {
    __shared__ double ys[kVfMaxGroup], gs[kVfMaxGroup];
    const int tid = threadIdx.x, wv = tid >> 6, lane = lane_id();
    for (int m = 0; m < h; ++m) {
        for (int j = wv; j < ng; j += 4) {
            const double* vj = V + (long)grp[j] * K;
            double s = 0.0;
            for (int p = lane; p < A; p += 64) {
                const int b0 = krow[p], kp = krow[p + 1] - b0;
                // forecasts i = 0 .. m-1 sit at block positions k = K_p - 1 - m + i >= 0
                for (int i = max(0, m - kp + 1); i < m; ++i)
                    s += vj[b0 + kp - 1 - m + i] * out[(long)p * h + i];
            }
            s = wave_sum(s);
            if (lane == 0) ys[j] = yk[(long)m * ng + j] + s;
        }
        __syncthreads();
        if (tid < ng) {
            double g = 0.0;
            for (int l = 0; l < ng; ++l) g += G[tid * ng + l] * ys[l];
            gs[tid] = g;
        }
        __syncthreads();
        for (int p = tid; p < A; p += 256) {
            const int kp = krow[p + 1] - krow[p];
            double r = 0.0;
            for (int j = 0; j < ng; ++j) r += V[(long)grp[j] * K + krow[p + 1] - 1] * gs[j];
            out[(long)p * h + m] = kp > 0 ? r : __builtin_nan("");
        }
        __syncthreads();
    }
}

// Advance the batch's step counter (end of a replayed step).
__global__ void k_step_next(int* step) {
    if (threadIdx.x == 0) step[0] += 1;
}

// Per-instance step counters (continuous batching: instances of one launch
// may be at different steps).  Set [j, jstart] of the listed instances, or
// advance their j by one.
__global__ void k_step_set(const LzDesc* __restrict__ lzs, const Item* __restrict__ items, int n, int j, int js) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    int* c = const_cast<int*>(lzs[items[e].inst].step);
    c[0] = j;
    c[1] = js;
}
__global__ void k_step_next_inst(const LzDesc* __restrict__ lzs, const Item* __restrict__ items, int n) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    int* c = const_cast<int*>(lzs[items[e].inst].step);
    c[0] += 1;
}

// p[0..n) = v (clears flags without a memset node, which a caller's graph
// capture would record)
__global__ void k_fill_i32(int* __restrict__ p, int n, int v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_gather_flags(const LzDesc* __restrict__ lzs, int ninst, int* __restrict__ flags,
                               double* __restrict__ betas) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ninst) return;
    const LzDesc& z = lzs[i];
    for (int k = 0; k < 4; ++k) flags[4 * i + k] = z.flag[k];
    for (int k = 0; k < 2; ++k) betas[2 * i + k] = z.beta[k];
}

}  // namespace shssa

#include "launch.inc"
