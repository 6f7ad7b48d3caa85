// LDS-resident mixed-radix Stockham FFT for gfx950 (device code).
//
// One transform of length n lives in LDS; G threads of the workgroup work on
// it.  Each radix-R pass reads R strided inputs per butterfly into
// registers, twiddles them, runs the R-point DFT in registers and writes the
// outputs back in autosorted (Stockham) order into the same buffer.  All
// reads of a pass happen before its barrier and all writes after it, so one
// buffer of n values suffices; every butterfly of a thread is held in
// registers between the two halves (at most PMAX butterflies, a compile-time
// bound derived from the largest n of the size class).
//
// Transforms are unnormalised: forward X_k = sum_t x_t exp(-2 pi i k t/n),
// inverse with exp(+...).  Twiddles come from a table of exp(-2 pi i t/n)
// built on the host in double precision.
//
// Real sequences of length 2n are transformed through one complex transform
// of length n (even samples as real parts, odd samples as imaginary parts)
// followed by the usual split into the n+1 non-redundant outputs; the
// inverse does the reverse.
#pragma once
#include "common.hpp"

namespace shssa {

__host__ __device__ constexpr int cdiv(int a, int b) { return (a + b - 1) / b; }

// The transforms below are separate (not inlined) functions, so they take
// generic pointers; they retype them at entry: the data buffer is always in
// LDS, the twiddle tables are in LDS when the size class stages them there
// (largest length NMAX <= 1024) and in global memory otherwise.  Typed
// pointers let the compiler emit LDS and global instructions instead of
// flat ones.
template <int NMAX> inline constexpr bool kTwStaged = NMAX <= 1024;
template <typename T> using lptr = __attribute__((address_space(3))) T*;
template <typename T> using lcptr = const __attribute__((address_space(3))) T*;
template <typename T> using gcptr = const __attribute__((address_space(1))) T*;
template <typename T, bool LDS> struct TwPtr { using type = gcptr<T>; };
template <typename T> struct TwPtr<T, true> { using type = lcptr<T>; };
template <typename T> __device__ __forceinline__ lptr<T> to_lds(T* p) { return (lptr<T>)p; }
template <typename T, bool LDS>
__device__ __forceinline__ typename TwPtr<T, LDS>::type to_tw(const T* p) {
    return (typename TwPtr<T, LDS>::type)p;
}
// element access through those pointers (field by field: no alignment
// beyond the element type's is assumed)
template <typename T, typename P>
__device__ __forceinline__ cplx<T> ldc(P p) { return cplx<T>{p->x, p->y}; }
template <typename T>
__device__ __forceinline__ void stc(lptr<cplx<T>> p, cplx<T> v) {
    p->x = v.x;
    p->y = v.y;
}

// w * v with w = exp(i s) given as (c, s) and DIR folding the sign of s.
template <typename T>
__device__ __forceinline__ cplx<T> mul_i(cplx<T> a) { return {-a.y, a.x}; }   // i * a

// ---- small DFTs in registers: X_k = sum_j a_j w^{jk}, w = exp(DIR 2 pi i / R)

template <typename T, int DIR>
__device__ __forceinline__ void bf2(cplx<T>* a) {
    cplx<T> t = a[0];
    a[0] = cadd(t, a[1]);
    a[1] = csub(t, a[1]);
}

template <typename T, int DIR>
__device__ __forceinline__ void bf4(cplx<T>* a) {
    cplx<T> t0 = cadd(a[0], a[2]), t1 = csub(a[0], a[2]);
    cplx<T> t2 = cadd(a[1], a[3]), t3 = csub(a[1], a[3]);
    // w = exp(DIR i pi/2) = DIR * i
    cplx<T> wt3 = DIR < 0 ? cplx<T>{t3.y, -t3.x} : cplx<T>{-t3.y, t3.x};
    a[0] = cadd(t0, t2);
    a[2] = csub(t0, t2);
    a[1] = cadd(t1, wt3);
    a[3] = csub(t1, wt3);
}

template <typename T, int DIR>
__device__ __forceinline__ void bf8(cplx<T>* a) {
    cplx<T> e[4] = {a[0], a[2], a[4], a[6]};
    cplx<T> o[4] = {a[1], a[3], a[5], a[7]};
    bf4<T, DIR>(e);
    bf4<T, DIR>(o);
    const T h = T(0.7071067811865476);
    // w8^k, k = 0..3, w8 = exp(DIR i pi/4)
    cplx<T> o1 = {h * (o[1].x - DIR * o[1].y), h * (o[1].y + DIR * o[1].x)};
    cplx<T> o2 = DIR < 0 ? cplx<T>{o[2].y, -o[2].x} : cplx<T>{-o[2].y, o[2].x};
    cplx<T> o3 = {h * (-o[3].x - DIR * o[3].y), h * (-o[3].y + DIR * o[3].x)};
    a[0] = cadd(e[0], o[0]);
    a[4] = csub(e[0], o[0]);
    a[1] = cadd(e[1], o1);
    a[5] = csub(e[1], o1);
    a[2] = cadd(e[2], o2);
    a[6] = csub(e[2], o2);
    a[3] = cadd(e[3], o3);
    a[7] = csub(e[3], o3);
}

template <typename T, int DIR>
__device__ __forceinline__ void bf3(cplx<T>* a) {
    const T c = T(-0.5), s = T(DIR) * T(0.8660254037844386);
    cplx<T> t = cadd(a[1], a[2]), d = csub(a[1], a[2]);
    cplx<T> m = {a[0].x + c * t.x, a[0].y + c * t.y};
    cplx<T> isd = {-s * d.y, s * d.x};
    a[0] = cadd(a[0], t);
    a[1] = cadd(m, isd);
    a[2] = csub(m, isd);
}

template <typename T, int DIR>
__device__ __forceinline__ void bf5(cplx<T>* a) {
    const T c1 = T(0.30901699437494745), c2 = T(-0.8090169943749473);
    const T s1 = T(DIR) * T(0.9510565162951535), s2 = T(DIR) * T(0.5877852522924732);
    cplx<T> t1 = cadd(a[1], a[4]), d1 = csub(a[1], a[4]);
    cplx<T> t2 = cadd(a[2], a[3]), d2 = csub(a[2], a[3]);
    cplx<T> m1 = {a[0].x + c1 * t1.x + c2 * t2.x, a[0].y + c1 * t1.y + c2 * t2.y};
    cplx<T> m2 = {a[0].x + c2 * t1.x + c1 * t2.x, a[0].y + c2 * t1.y + c1 * t2.y};
    cplx<T> p1 = {s1 * d1.x + s2 * d2.x, s1 * d1.y + s2 * d2.y};
    cplx<T> p2 = {s2 * d1.x - s1 * d2.x, s2 * d1.y - s1 * d2.y};
    a[0] = cadd(a[0], cadd(t1, t2));
    a[1] = cadd(m1, mul_i(p1));
    a[4] = csub(m1, mul_i(p1));
    a[2] = cadd(m2, mul_i(p2));
    a[3] = csub(m2, mul_i(p2));
}

template <typename T, int DIR>
__device__ __forceinline__ void bf7(cplx<T>* a) {
    // cos / sin of 2 pi m / 7, m = 0..6
    const T C[7] = {T(1.0), T(0.6234898018587336), T(-0.22252093395631434), T(-0.900968867902419),
                    T(-0.9009688679024191), T(-0.2225209339563146), T(0.6234898018587334)};
    const T S[7] = {T(0.0), T(0.7818314824680298), T(0.9749279121818236), T(0.43388373911755823),
                    T(-0.433883739117558), T(-0.9749279121818236), T(-0.7818314824680299)};
    cplx<T> t[4], d[4];
#pragma unroll
    for (int j = 1; j <= 3; ++j) { t[j] = cadd(a[j], a[7 - j]); d[j] = csub(a[j], a[7 - j]); }
    cplx<T> out[7];
    out[0] = cadd(a[0], cadd(t[1], cadd(t[2], t[3])));
#pragma unroll
    for (int k = 1; k <= 3; ++k) {
        cplx<T> m = a[0], p = {T(0), T(0)};
#pragma unroll
        for (int j = 1; j <= 3; ++j) {
            const int q = (j * k) % 7;
            m.x += C[q] * t[j].x; m.y += C[q] * t[j].y;
            p.x += T(DIR) * S[q] * d[j].x; p.y += T(DIR) * S[q] * d[j].y;
        }
        out[k] = cadd(m, mul_i(p));
        out[7 - k] = csub(m, mul_i(p));
    }
#pragma unroll
    for (int k = 0; k < 7; ++k) a[k] = out[k];
}

template <typename T, int R, int DIR>
__device__ __forceinline__ void butterfly(cplx<T>* a) {
    if constexpr (R == 2) bf2<T, DIR>(a);
    else if constexpr (R == 3) bf3<T, DIR>(a);
    else if constexpr (R == 4) bf4<T, DIR>(a);
    else if constexpr (R == 5) bf5<T, DIR>(a);
    else if constexpr (R == 7) bf7<T, DIR>(a);
    else bf8<T, DIR>(a);
}

// One Stockham pass of radix R over s[0..n), sub-transform size Ns so far.
template <typename T, int R, int PMAX, int DIR, typename TWP>
__device__ __forceinline__ void fft_pass(lptr<cplx<T>> s, int n, int Ns, TWP tw, int tid, int G) {
    const int m = n / R;
    const int tstride = n / (Ns * R);
    cplx<T> v[PMAX][R];
#pragma unroll
    for (int p = 0; p < PMAX; ++p) {
        const int j = tid + p * G;
        if (j < m) {
            const int k = j % Ns;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                cplx<T> a = ldc<T>(s + (j + r * m));
                if (r > 0 && k > 0) {
                    cplx<T> w = ldc<T>(tw + r * k * tstride);
                    if (DIR > 0) w.y = -w.y;
                    a = cmul(a, w);
                }
                v[p][r] = a;
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < PMAX; ++p) {
        const int j = tid + p * G;
        if (j < m) {
            butterfly<T, R, DIR>(v[p]);
            const int k = j % Ns;
            const int base = (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) stc<T>(s + (base + r * Ns), v[p][r]);
        }
    }
    __syncthreads();
}

// Complex FFT of length pl.n <= NMAX in LDS, G threads (tid in [0, G)).
// Starts and ends with the buffer synchronised (caller must have issued a
// barrier after filling s).
// P2: the plan has only radices 2, 4 and 8 (the odd-radix passes are not
// compiled in, which keeps the register footprint of the kernel small).
// tw: the plan's twiddle table (global, or a copy staged in LDS).
template <typename T, int NMAX, int G, int DIR, bool P2 = false>
__device__ void fft_lds(cplx<T>* sg, const FftPlan& pl, const cplx<T>* twg, int tid) {
    const lptr<cplx<T>> s = to_lds(sg);
    const auto tw = to_tw<cplx<T>, kTwStaged<NMAX>>(twg);
    int Ns = 1;
    for (int p = 0; p < pl.npass; ++p) {
        if constexpr (P2) {
            switch (pl.radix[p]) {
            case 2: fft_pass<T, 2, cdiv(NMAX, 2 * G), DIR>(s, pl.n, Ns, tw, tid, G); Ns *= 2; break;
            case 4: fft_pass<T, 4, cdiv(NMAX, 4 * G), DIR>(s, pl.n, Ns, tw, tid, G); Ns *= 4; break;
            default: fft_pass<T, 8, cdiv(NMAX, 8 * G), DIR>(s, pl.n, Ns, tw, tid, G); Ns *= 8; break;
            }
            continue;
        }
        switch (pl.radix[p]) {
        case 2: fft_pass<T, 2, cdiv(NMAX, 2 * G), DIR>(s, pl.n, Ns, tw, tid, G); Ns *= 2; break;
        case 3: fft_pass<T, 3, cdiv(NMAX, 3 * G), DIR>(s, pl.n, Ns, tw, tid, G); Ns *= 3; break;
        case 4: fft_pass<T, 4, cdiv(NMAX, 4 * G), DIR>(s, pl.n, Ns, tw, tid, G); Ns *= 4; break;
        case 5: fft_pass<T, 5, cdiv(NMAX, 5 * G), DIR>(s, pl.n, Ns, tw, tid, G); Ns *= 5; break;
        case 7: fft_pass<T, 7, cdiv(NMAX, 7 * G), DIR>(s, pl.n, Ns, tw, tid, G); Ns *= 7; break;
        default: fft_pass<T, 8, cdiv(NMAX, 8 * G), DIR>(s, pl.n, Ns, tw, tid, G); Ns *= 8; break;
        }
    }
}

// Real forward transform of length 2n held in s as n complex pairs.
// On return s[0..n] = X[0..n] (n+1 values).  Ends synchronised.
template <typename T, int NMAX, int G, bool P2 = false>
__device__ void rfft_fwd(cplx<T>* sg, const FftPlan& pl, const cplx<T>* tw, const cplx<T>* twrg, int tid) {
    fft_lds<T, NMAX, G, -1, P2>(sg, pl, tw, tid);
    const lptr<cplx<T>> s = to_lds(sg);
    const auto twr = to_tw<cplx<T>, kTwStaged<NMAX>>(twrg);
    const int n = pl.n;
    for (int k = tid; k <= n / 2; k += G) {
        const int k2 = k == 0 ? 0 : n - k;
        const cplx<T> zk = ldc<T>(s + k), zn = ldc<T>(s + k2);
        // E = (Z_k + conj Z_{n-k}) / 2,  O = (Z_k - conj Z_{n-k}) / (2i)
        const cplx<T> e = {T(0.5) * (zk.x + zn.x), T(0.5) * (zk.y - zn.y)};
        const cplx<T> o = {T(0.5) * (zk.y + zn.y), T(-0.5) * (zk.x - zn.x)};
        const cplx<T> wo = cmul(ldc<T>(twr + k), o);
        stc<T>(s + k, cadd(e, wo));
        const cplx<T> xm = csub(e, wo);
        stc<T>(s + (k == 0 ? n : n - k), cconj(xm));
    }
    __syncthreads();
}

// Inverse of rfft_fwd: from X[0..n] in s, leaves 2n * x (real, as n complex
// pairs) in s[0..n).  Ends synchronised.
template <typename T, int NMAX, int G, bool P2 = false>
__device__ void rfft_inv(cplx<T>* sg, const FftPlan& pl, const cplx<T>* tw, const cplx<T>* twrg, int tid) {
    const lptr<cplx<T>> s = to_lds(sg);
    const auto twr = to_tw<cplx<T>, kTwStaged<NMAX>>(twrg);
    const int n = pl.n;
    for (int k = tid; k <= n / 2; k += G) {
        const int k2 = n - k;
        const cplx<T> xk = ldc<T>(s + k), xn = ldc<T>(s + k2);
        // E' = X_k + conj X_{n-k},  O' = (X_k - conj X_{n-k}) conj(W^k)
        const cplx<T> e = {xk.x + xn.x, xk.y - xn.y};
        const cplx<T> d = {xk.x - xn.x, xk.y + xn.y};
        const cplx<T> o = cmulc(d, ldc<T>(twr + k));
        // Z_k = E' + i O',  Z_{n-k} = conj E' + i conj O'
        stc<T>(s + k, cplx<T>{e.x - o.y, e.y + o.x});
        if (k != 0 && k != k2) stc<T>(s + k2, cplx<T>{e.x + o.y, -e.y + o.x});
    }
    __syncthreads();
    fft_lds<T, NMAX, G, +1, P2>(sg, pl, tw, tid);
}

}  // namespace shssa
