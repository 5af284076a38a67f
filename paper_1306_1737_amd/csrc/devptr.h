// Global-address-space pointers for kernels that read their array pointers
// from a device table (batched replicas).  Such a pointer is otherwise a
// generic one: the compiler could not issue scalar loads through it, and
// atomics through it would use flat addressing.  Typing the pointers as
// address space 1 restores both.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace mxn {

template <class T> using gptr = __attribute__((address_space(1))) T *;
template <class T> using plain = T *;

// Vector loads and stores (component-wise through global pointers; the
// compiler merges them into one 16-byte access).
__device__ inline float4 ld(const float4 *p) { return *p; }
__device__ inline int4 ld(const int4 *p) { return *p; }
__device__ inline nb_jentry ld(const nb_jentry *p) { return *p; }
__device__ inline float4 ld(gptr<const float4> p) {
    const gptr<const float> q = (gptr<const float>)p;
    return make_float4(q[0], q[1], q[2], q[3]);
}
__device__ inline int4 ld(gptr<const int4> p) {
    const gptr<const int> q = (gptr<const int>)p;
    return make_int4(q[0], q[1], q[2], q[3]);
}
__device__ inline nb_jentry ld(gptr<const nb_jentry> p) {
    const int4 t = ld((gptr<const int4>)p);
    return nb_jentry{t.x, t.y, (uint32_t)t.z, (uint32_t)t.w};
}
__device__ inline void st(float4 *p, const float4 &v) { *p = v; }
__device__ inline void st(gptr<float4> p, const float4 &v) {
    const gptr<float> q = (gptr<float>)p;
    q[0] = v.x;
    q[1] = v.y;
    q[2] = v.z;
    q[3] = v.w;
}
__device__ inline void st(nb_jentry *p, const nb_jentry &v) { *p = v; }
__device__ inline void st(gptr<nb_jentry> p, const nb_jentry &v) {
    const gptr<int> q = (gptr<int>)p;
    q[0] = v.cj;
    q[1] = v.shift;
    q[2] = (int)v.mlo;
    q[3] = (int)v.mhi;
}

}  // namespace mxn
