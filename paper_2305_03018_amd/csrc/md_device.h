// Device helpers shared by the transform kernels (md_fft.hip) and the
// direct-window kernels (md_direct.hip).  Internal; not part of the public
// interface.
#pragma once

#include "md_internal.h"

namespace md {
namespace {

template <typename R> struct Cx;
template <> struct Cx<float> { using T = float2; };
template <> struct Cx<double> { using T = double2; };

template <typename C>
__device__ __forceinline__ C cadd(C a, C b) { C r; r.x = a.x + b.x; r.y = a.y + b.y; return r; }
template <typename C>
__device__ __forceinline__ C csub(C a, C b) { C r; r.x = a.x - b.x; r.y = a.y - b.y; return r; }
template <typename C>
__device__ __forceinline__ C cmul(C a, C b) {
    C r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}
template <typename C>
__device__ __forceinline__ C czero() { C r; r.x = 0; r.y = 0; return r; }

// Address-space views: tables that every lane of a wavefront reads at the
// same index go through the constant space (scalar loads); per-lane data
// through the global space (no flat addressing).
template <class T>
__device__ __forceinline__ const __attribute__((address_space(4))) T *cst(const T *p) {
    return (const __attribute__((address_space(4))) T *)(p);
}
template <class T>
__device__ __forceinline__ const __attribute__((address_space(1))) T *gld(const T *p) {
    return (const __attribute__((address_space(1))) T *)(p);
}
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T *gst(T *p) {
    return (__attribute__((address_space(1))) T *)(p);
}

// Complex loads/stores through those spaces, as clang vectors (HIP's vector
// structs do not copy out of address-space-qualified storage).
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
template <class C> struct VecOf;
template <> struct VecOf<float2> { using T = f32x2; };
template <> struct VecOf<double2> { using T = f64x2; };

template <class C>
__device__ __forceinline__ C ldg(const C *p, size_t i) {
    using V = typename VecOf<C>::T;
    const V v = ((const __attribute__((address_space(1))) V *)p)[i];
    C r;
    r.x = v.x;
    r.y = v.y;
    return r;
}
template <class C>
__device__ __forceinline__ C ldc(const C *p, size_t i) {
    using V = typename VecOf<C>::T;
    const V v = ((const __attribute__((address_space(4))) V *)p)[i];
    C r;
    r.x = v.x;
    r.y = v.y;
    return r;
}
template <class C>
__device__ __forceinline__ void stg(C *p, size_t i, C v) {
    using V = typename VecOf<C>::T;
    V w;
    w.x = v.x;
    w.y = v.y;
    ((__attribute__((address_space(1))) V *)p)[i] = w;
}

// Segment of a persistent launch that holds work item `it`: the last
// segment whose first item is <= it (segments are in item order).
__device__ __forceinline__ int find_seg(const Seg *__restrict__ segs, int nseg, long long it) {
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (segs[mid].item0 <= it) lo = mid; else hi = mid - 1;
    }
    return lo;
}

}  // namespace
}  // namespace md
