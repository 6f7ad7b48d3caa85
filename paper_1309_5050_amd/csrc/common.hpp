// Shared definitions of the Shaped 2D-SSA GPU library (host and device).
//
// Internal orientation.  Every decomposition is held as a grid of A rows by
// B columns with B the contiguous axis.  The window box is LA x LB and the
// origin box KA x KB (KA = A - LA + 1, KB = B - LB + 1).  Compact vectors on
// a set (window cells or origins) list the set's cells row by row (column
// index fastest); the boundary converts to the caller's layout.
//
// Two operator families:
//   row family  (LA == 1): 1D SSA, MSSA and windows one row high.  The
//                correlation across rows is a plain sum, so only row FFTs
//                of length MB are needed.
//   grid family (LA > 1):  2D and shaped 2D-SSA; row FFTs of length MB and
//                column FFTs of length MA.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace shssa {

template <typename T> struct cplx { T x, y; };

// Pointer to device global memory.  Casting the generic pointers held in the
// descriptors lets the compiler emit global (not flat) loads and stores and
// use the scalar-base + 32-bit-offset addressing form.
template <typename T> using gptr = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gptr<T> as_global(T* p) { return (gptr<T>)p; }
template <typename T>
__device__ __forceinline__ gptr<const T> as_global(const T* p) { return (gptr<const T>)p; }
template <typename T>
__device__ __forceinline__ T gload(gptr<const T> p) { return *p; }
template <typename T>
__device__ __forceinline__ T gload(gptr<T> p) { return *p; }
template <typename T>
__device__ __forceinline__ void gstore(gptr<T> p, T v) { *p = v; }

// Complex values move as one two-element vector (one 8- or 16-byte access).
template <typename T> struct vec2;
template <> struct vec2<float> { typedef float type __attribute__((ext_vector_type(2))); };
template <> struct vec2<double> { typedef double type __attribute__((ext_vector_type(2))); };
template <typename T>
__device__ __forceinline__ cplx<T> gload(gptr<const cplx<T>> p) {
    const typename vec2<T>::type v = *(gptr<const typename vec2<T>::type>)p;
    return cplx<T>{v.x, v.y};
}
template <typename T>
__device__ __forceinline__ cplx<T> gload(gptr<cplx<T>> p) {
    const typename vec2<T>::type v = *(gptr<typename vec2<T>::type>)p;
    return cplx<T>{v.x, v.y};
}
template <typename T>
__device__ __forceinline__ void gstore(gptr<cplx<T>> p, cplx<T> c) {
    typename vec2<T>::type v;
    v.x = c.x;
    v.y = c.y;
    *(gptr<typename vec2<T>::type>)p = v;
}

template <typename T>
__host__ __device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename T>
__host__ __device__ __forceinline__ cplx<T> cmulc(cplx<T> a, cplx<T> b) {
    return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename T>
__host__ __device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__host__ __device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__host__ __device__ __forceinline__ cplx<T> cconj(cplx<T> a) { return {a.x, -a.y}; }

// Maximum number of radix passes of one FFT plan.
constexpr int kMaxPass = 16;

// An FFT of length n = prod(radix[0..npass)).  tw points to n complex values
// exp(-2 pi i t / n), t = 0..n-1, in the precision of the transform.  For a
// real transform of length 2n, twr points to n+1 values exp(-2 pi i t / 2n).
struct FftPlan {
    int n;
    int npass;
    int8_t radix[kMaxPass];
    const void* tw;
    const void* twr;
};

// A set of cells inside a box (window shape or origin set).
struct CellSet {
    int boxA, boxB;          // bounding box rows / columns
    long count;              // number of cells
    const uint8_t* mask;     // boxA*boxB bytes, row-major; nullptr = full box
    const int* rowoff;       // boxA+1 offsets into the compact order
    const int* pref;         // boxA x (boxB+1): cells of the row before column b (with mask)
};

}  // namespace shssa
