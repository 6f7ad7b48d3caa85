// Register-resident radix-8 Stockham FFT for power-of-two lengths (device).
//
// A transform of length N = 2^LOGN (64 <= N <= 4096) is spread over
// G = N/8 threads, each holding 8 elements in registers.  On entry and on
// exit thread t holds positions t + G*e in slot e (natural order), so a
// forward transform, a pointwise product and an inverse transform chain
// without any data movement.  Every radix-8 pass works on one butterfly per
// thread; a final radix-2 or radix-4 pass (N not a power of 8) works on 4 or
// 2 butterflies per thread.  Between passes the outputs go through LDS once
// (write, barrier, read in the next pass's order, barrier).
//
// Several transforms share a workgroup: transform c (0 <= c < TC) keeps its
// exchange rows interleaved in LDS as [position][c], so lanes of consecutive
// c touch consecutive words; one empty row per 8 positions keeps the
// stride-8 writes of the first pass off a single bank group.
//
// Twiddles are taken once per thread (all passes) from the plan table
// tw[i] = exp(-2 pi i i/N); the inverse uses their conjugates.
#pragma once
#include "fft.hpp"

namespace shssa {

template <int LOGN>
struct RegPlan {
    static_assert(LOGN >= 6 && LOGN <= 12, "register FFT lengths 64..4096");
    static constexpr int N = 1 << LOGN;
    static constexpr int G = N / 8;
    static constexpr int P8 = LOGN / 3;                 // radix-8 passes
    static constexpr int REM = LOGN % 3;                // 1: final radix-2 pass, 2: final radix-4 pass
    static constexpr int R = REM == 1 ? 2 : (REM == 2 ? 4 : 8);
    static constexpr int NTW = 7 * (P8 - 1) + (REM ? 8 - 8 / R : 0);   // twiddles per thread
    static constexpr int LROWS = N + N / 8;             // padded exchange rows
};

// Exchange slots.  pad(pos) = pos + pos/8 leaves one empty slot per 8
// positions (the stride-8 writes of the first pass then spread over the
// banks).  Every exchange address is pad(base) + r * stride with a
// compile-time stride, so the per-element offsets become instruction
// immediates.  A transform's LDS slot of padded index pp is ad(pp): linear in
// pp, e.g. pp*TC + c for TC interleaved transforms or c*LROWS + pp for
// transforms one after the other.
__device__ __forceinline__ int rx_pad(int pos) { return pos + (pos >> 3); }
template <int TC>
__device__ __forceinline__ int rx_addr(int pp, int c) { return pp * TC + c; }
template <int LOGN>
__device__ __forceinline__ int rx_addr_row(int pp, int c) { return c * RegPlan<LOGN>::LROWS + pp; }

// The thread's twiddles of passes 2..: radix-8 pass p uses
// w^(r k N/(8 Ns)), k = t mod Ns, Ns = 8^p; the final radix-R pass uses
// w^(r j), j = t + q G for its butterflies q.
template <typename T, int LOGN>
__device__ __forceinline__ void reg_twiddles(const cplx<T>* __restrict__ twp, int t,
                                             cplx<T> (&w)[RegPlan<LOGN>::NTW]) {
    using RP = RegPlan<LOGN>;
    const gptr<const cplx<T>> tw = as_global(twp);
    int q = 0;
#pragma unroll
    for (int p = 1; p < RP::P8; ++p) {
        const int Ns = 1 << (3 * p);
        const int k = t & (Ns - 1);
        const int step = k * (RP::N / (8 * Ns));
#pragma unroll
        for (int r = 1; r < 8; ++r) w[q++] = gload(tw + r * step);
    }
    if constexpr (RP::REM != 0) {
        constexpr int B = 8 / RP::R;
#pragma unroll
        for (int b = 0; b < B; ++b)
#pragma unroll
            for (int r = 1; r < RP::R; ++r) w[q++] = gload(tw + r * (t + b * RP::G));
    }
}

// The same twiddles looked up in a table staged in LDS (shared by the
// workgroup), laid out pass by pass so that the lanes of a transform read
// consecutive entries: radix-8 pass p (Ns = 8^p) holds w^(r k N/(8 Ns)) at
// r Ns - 8 + k (r = 1..7, k < Ns); the final radix-R pass holds w^(r j),
// j = t + b G, at 8^P8 - 8 + (b (R-1) + r - 1) G + t.  A table indexed by
// the exponent would put the 8 distinct twiddles of a pass Ns = 8 on
// addresses 8 r words apart (several lanes per bank).  Costs an LDS read per
// use instead of NTW registers.
template <typename T, int LOGN>
struct TwTable {
    using RP = RegPlan<LOGN>;
    static constexpr int OFF_R = (1 << (3 * RP::P8)) - 8;   // start of the final pass's entries
    static constexpr int SIZE = OFF_R + (RP::REM ? (8 / RP::R) * (RP::R - 1) * RP::G : 0);
    const cplx<T>* tab;
    int t;
    __device__ __forceinline__ cplx<T> operator()(int q) const {
        if (q < 7 * (RP::P8 - 1)) {
            const int p = q / 7 + 1, r = q % 7 + 1;
            const int Ns = 1 << (3 * p);
            return tab[r * Ns - 8 + (t & (Ns - 1))];
        }
        const int q2 = q - 7 * (RP::P8 - 1);
        return tab[OFF_R + q2 * RP::G + t];
    }
    // Exponent of entry i (the table holds w^src(i), w = exp(-2 pi i / N)).
    __device__ __forceinline__ static int src(int i) {
        static_assert(RP::P8 <= 4, "segments of the radix-8 passes: Ns = 8, 64, 512");
        if (i < OFF_R) {
            // segment of pass Ns starts at Ns - 8 (selects, not a loop: the
            // address is ready early and its load issues with the others)
            int Ns = 8;
            Ns = i >= 56 ? 64 : Ns;
            Ns = i >= 504 ? 512 : Ns;
            const int j = i - (Ns - 8);
            const int r = j / Ns + 1, k = j % Ns;
            return r * k * (RP::N / (8 * Ns));
        }
        const int j = i - OFF_R;
        const int q2 = j / RP::G, tt = j % RP::G;
        const int b = q2 / (RP::R - 1), r = q2 % (RP::R - 1) + 1;
        return r * (tt + b * RP::G);
    }
    // Filling the table from the N values w^k (global memory) by the NTHR
    // threads of a workgroup, in two halves: load() issues the thread's
    // global loads, store() writes the values to LDS (dst holds SIZE + 1
    // entries; threads past the end write the last, a discard slot, so the
    // stores are unconditional and the compiler keeps the loads where they
    // were issued).  A kernel issues its own loads between the two.
    template <int NTHR>
    struct Stage {
        static constexpr int K = (SIZE + NTHR - 1) / NTHR;
        cplx<T> r[K];
        __device__ __forceinline__ void load(gptr<const cplx<T>> tw, int tid) {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int i = tid + NTHR * k;
                r[k] = gload(tw + src(i < SIZE ? i : 0));
            }
        }
        __device__ __forceinline__ void store(cplx<T>* dst, int tid) const {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int i = tid + NTHR * k;
                dst[i < SIZE ? i : SIZE] = r[k];
            }
        }
    };
};

// Exchange synchronisation.  XS_WG: transforms spread over the waves of a
// workgroup, one LDS buffer (barrier after the writes and after the reads).
// XS_WG2: the same with two buffers used in turn (one barrier per exchange:
// a buffer is rewritten only two exchanges later, after a barrier every
// reader of its previous contents has passed).  XS_WAVE: every transform
// lies inside one wave, whose lanes execute each LDS instruction together;
// a wave-scope fence keeps the compiler from moving LDS accesses across the
// exchange.
enum { XS_WG = 0, XS_WG2 = 1, XS_WAVE = 2 };

template <int XS>
__device__ __forceinline__ void xsync() {
    if constexpr (XS == XS_WAVE) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

template <typename T, int DIR>
__device__ __forceinline__ cplx<T> twiddle(cplx<T> a, cplx<T> w) {
    return DIR < 0 ? cmul(a, w) : cmulc(a, w);
}

// In-place transform of the 8 register values of thread t.  DIR = -1
// forward, +1 inverse (unnormalised).  ad maps a padded position of this
// thread's transform to its LDS slot (transforms of a workgroup use disjoint
// slots); the caller must not touch those slots concurrently.  Every thread
// of the workgroup must call it (it may contain barriers).  XS selects the
// exchange synchronisation; with XS_WG2 exchange number xe (counted by the
// caller across calls) uses buffer lds + (xe & 1) * xbuf.
// SPARSE_IN: only slot 0 of the input is nonzero (the first pass is a
// broadcast).  FIRST_OUT: only slot 0 of the output is used (the last radix-8
// pass computes its first output only); valid when LOGN is a multiple of 3.
// W(q) gives twiddle q of the thread (registers or TwTable).
template <typename T, int LOGN, int DIR, int XS, bool SPARSE_IN = false, bool FIRST_OUT = false, typename TW,
          typename AD>
__device__ __forceinline__ void reg_fft_tw(cplx<T> (&v)[8], TW W, cplx<T>* lds, int t, AD ad, int& xe,
                                           int xbuf = 0) {
    using RP = RegPlan<LOGN>;
    constexpr int G = RP::G;
    constexpr int NPASS = RP::P8 + (RP::REM ? 1 : 0);
    constexpr int RS = G + G / 8;        // padded distance of the read slots
    static_assert(!FIRST_OUT || RP::REM == 0, "FIRST_OUT needs a final radix-8 pass");
    const int prd = rx_pad(t);
#pragma unroll
    for (int p = 0; p < RP::P8; ++p) {
        const int Ns = 1 << (3 * p);
        if (p > 0) {
#pragma unroll
            for (int r = 1; r < 8; ++r) v[r] = twiddle<T, DIR>(v[r], W(7 * (p - 1) + r - 1));
        }
        if (p == NPASS - 1 && FIRST_OUT) {
            cplx<T> s0 = v[0];
#pragma unroll
            for (int r = 1; r < 8; ++r) s0 = cadd(s0, v[r]);
            v[0] = s0;
            return;
        }
        if (p == 0 && SPARSE_IN) {
#pragma unroll
            for (int r = 1; r < 8; ++r) v[r] = v[0];
        } else {
            bf8<T, DIR>(v);
        }
        if (p == NPASS - 1) return;
        cplx<T>* buf = XS == XS_WG2 ? lds + (xe & 1) * xbuf : lds;
        ++xe;
        const int k = t & (Ns - 1);
        const int pb = rx_pad((t - k) * 8 + k);
        const int WS = Ns == 1 ? 1 : Ns + Ns / 8;   // padded distance of the write slots
#pragma unroll
        for (int r = 0; r < 8; ++r) buf[ad(pb + r * WS)] = v[r];
        xsync<XS>();
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = buf[ad(prd + e * RS)];
        if constexpr (XS != XS_WG2) xsync<XS>();
    }
    if constexpr (RP::REM != 0) {
        constexpr int R = RP::R, B = 8 / R;
        constexpr int w0 = 7 * (RP::P8 - 1);
#pragma unroll
        for (int b = 0; b < B; ++b) {
            cplx<T> a[R];
#pragma unroll
            for (int r = 0; r < R; ++r) a[r] = v[b + B * r];
#pragma unroll
            for (int r = 1; r < R; ++r) a[r] = twiddle<T, DIR>(a[r], W(w0 + b * (R - 1) + r - 1));
            if constexpr (R == 2) bf2<T, DIR>(a);
            else bf4<T, DIR>(a);
#pragma unroll
            for (int r = 0; r < R; ++r) v[b + B * r] = a[r];
        }
    }
}

template <typename T, int LOGN, int DIR, int XS, bool SPARSE_IN = false, bool FIRST_OUT = false, typename AD>
__device__ __forceinline__ void reg_fft(cplx<T> (&v)[8], const cplx<T> (&w)[RegPlan<LOGN>::NTW],
                                        cplx<T>* lds, int t, AD ad, int& xe, int xbuf = 0) {
    reg_fft_tw<T, LOGN, DIR, XS, SPARSE_IN, FIRST_OUT>(v, [&](int q) { return w[q]; }, lds, t, ad, xe, xbuf);
}

}  // namespace shssa
