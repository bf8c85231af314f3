// Shared device helpers of the ofks library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define OFKS_WAVE 64

namespace ofks {

// Vector of V consecutive values of T, loaded/stored with one instruction.
template <typename T, int V> struct vec_t;
template <> struct vec_t<double, 1> { using type = double; };
template <> struct vec_t<double, 2> { using type = double2; };
template <> struct vec_t<float, 1> { using type = float; };
template <> struct vec_t<float, 2> { using type = float2; };
template <> struct vec_t<float, 4> { using type = float4; };

template <typename T, int V>
__device__ __forceinline__ void load_vec(const T *__restrict__ p, T (&out)[V]) {
    using VT = typename vec_t<T, V>::type;
    VT v = *reinterpret_cast<const VT *>(p);
    const T *s = reinterpret_cast<const T *>(&v);
#pragma unroll
    for (int i = 0; i < V; ++i) out[i] = s[i];
}

template <typename T, int V>
__device__ __forceinline__ void store_vec(T *__restrict__ p, const T (&in)[V]) {
    using VT = typename vec_t<T, V>::type;
    VT v;
    T *d = reinterpret_cast<T *>(&v);
#pragma unroll
    for (int i = 0; i < V; ++i) d[i] = in[i];
    *reinterpret_cast<VT *>(p) = v;
}

// Layout of a block of p columns over lanes: V columns per lane, LPR lanes
// per row (power of two <= 64), CH column chunks per lane when p > LPR*V.
struct ColMap {
    int p;        // columns
    int v;        // values per lane access
    int lpr_log2; // log2(lanes per row)
    int chunks;   // ceil(p / (lanes*v))
};

}  // namespace ofks
