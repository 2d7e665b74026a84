// engine.hpp -- device building blocks of the Fastfood hot path on gfx950:
// butterflies on register bits, LDS moves between layouts, the Pi gather /
// scatter, HBM loads and stores in the coalesced layout, and the fused
// [cos, sin] feature map.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "layout.hpp"

namespace mck {

typedef float v4f __attribute__((ext_vector_type(4)));

// Orders LDS traffic of one wave: LDS instructions of a wave execute in issue
// order, so only the compiler must be kept from moving accesses across.
__device__ __forceinline__ void wave_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int M>
__device__ __forceinline__ void lds_sync()
{
    if constexpr (Geo<M>::kMulti)
        __syncthreads();
    else
        wave_fence();
}

// index bits owned by lane t in layout ID
template <int M, int ID>
__device__ __forceinline__ uint32_t tpart(uint32_t t)
{
    uint32_t i = 0;
#pragma unroll
    for (int b = 0; b < Geo<M>::T; ++b)
        i |= ((t >> b) & 1u) << thr_bit(M, ID, b);
    return i;
}

// Radix-2 butterflies (a, b) -> (a + b, a - b) on every register bit of
// layout ID whose index bit is in MASK: pairs (i, i + 2^k), bit k of i clear,
// natural (Sylvester) order.
template <int M, int ID, uint32_t MASK>
__device__ __forceinline__ void stages(float (&v)[Geo<M>::EPL])
{
    constexpr int P = Geo<M>::P, EPL = Geo<M>::EPL;
#pragma unroll
    for (int b = 0; b < P; ++b) {
        if (((MASK >> reg_bit(M, ID, b)) & 1u) == 0)
            continue;
#pragma unroll
        for (int r = 0; r < EPL; ++r) {
            if (r & (1 << b))
                continue;
            const float a = v[r], c = v[r | (1 << b)];
            v[r] = a + c;
            v[r | (1 << b)] = a - c;
        }
    }
}

// float4 LDS access is used for the coalesced layout when row regions are
// 16-byte aligned.
template <int M, int ID>
constexpr bool lds_vec() { return ID == 0 && M >= 6; }

template <int M, int ID>
__device__ __forceinline__ void lds_put(float* buf, uint32_t t, const float (&v)[Geo<M>::EPL])
{
    constexpr int EPL = Geo<M>::EPL;
    const uint32_t tb = phys(tpart<M, ID>(t));
    if constexpr (lds_vec<M, ID>()) {
#pragma unroll
        for (int j = 0; j < EPL / 4; ++j) {
            float4 q = make_float4(v[4 * j], v[4 * j + 1], v[4 * j + 2], v[4 * j + 3]);
            *reinterpret_cast<float4*>(buf + (tb ^ phys(rpart(M, ID, 4 * j)))) = q;
        }
    } else {
#pragma unroll
        for (int r = 0; r < EPL; ++r)
            buf[tb ^ phys(rpart(M, ID, r))] = v[r];
    }
}

template <int M, int ID>
__device__ __forceinline__ void lds_get(const float* buf, uint32_t t, float (&v)[Geo<M>::EPL])
{
    constexpr int EPL = Geo<M>::EPL;
    const uint32_t tb = phys(tpart<M, ID>(t));
    if constexpr (lds_vec<M, ID>()) {
#pragma unroll
        for (int j = 0; j < EPL / 4; ++j) {
            const float4 q = *reinterpret_cast<const float4*>(buf + (tb ^ phys(rpart(M, ID, 4 * j))));
            v[4 * j] = q.x;
            v[4 * j + 1] = q.y;
            v[4 * j + 2] = q.z;
            v[4 * j + 3] = q.w;
        }
    } else {
#pragma unroll
        for (int r = 0; r < EPL; ++r)
            v[r] = buf[tb ^ phys(rpart(M, ID, r))];
    }
}

// Move a vector from layout X to layout Y through the row's LDS region.
template <int M, int X, int Y>
__device__ __forceinline__ void relayout(float (&v)[Geo<M>::EPL], float* buf, uint32_t t)
{
    lds_put<M, X>(buf, t, v);
    lds_sync<M>();
    lds_get<M, Y>(buf, t, v);
    lds_sync<M>();
}

// H v, starting in layout 0 and ending in the last chunk layout.
template <int M>
__device__ __forceinline__ void fwht_up(float (&v)[Geo<M>::EPL], float* buf, uint32_t t)
{
    constexpr int K = Geo<M>::K;
    stages<M, 0, fwd1_new_bits(M, 0)>(v);
    if constexpr (K >= 1) {
        relayout<M, 0, 1>(v, buf, t);
        stages<M, 1, fwd1_new_bits(M, 1)>(v);
    }
    if constexpr (K >= 2) {
        relayout<M, 1, 2>(v, buf, t);
        stages<M, 2, fwd1_new_bits(M, 2)>(v);
    }
}

// H v, starting in the last chunk layout and ending in layout 0.
template <int M>
__device__ __forceinline__ void fwht_down(float (&v)[Geo<M>::EPL], float* buf, uint32_t t)
{
    constexpr int K = Geo<M>::K;
    if constexpr (K == 0) {
        stages<M, 0, fwd2_new_bits(M, 0, 0)>(v);
    } else if constexpr (K == 1) {
        stages<M, 1, fwd2_new_bits(M, 1, 1)>(v);
        relayout<M, 1, 0>(v, buf, t);
        stages<M, 0, fwd2_new_bits(M, 1, 0)>(v);
    } else {
        stages<M, 2, fwd2_new_bits(M, 2, 2)>(v);
        relayout<M, 2, 1>(v, buf, t);
        stages<M, 1, fwd2_new_bits(M, 2, 1)>(v);
        relayout<M, 1, 0>(v, buf, t);
        stages<M, 0, fwd2_new_bits(M, 2, 0)>(v);
    }
}

// ------------------------------------------------------------------ HBM access
// Coalesced layout: register r of lane t holds index tpart(t) | rpart(0, r);
// registers 4j..4j+3 are consecutive indices (M >= 2).

template <int M>
__device__ __forceinline__ uint32_t coal_index(uint32_t t, int r)
{
    return tpart<M, 0>(t) | rpart(M, 0, r);
}

// Load one row of length d (zero-padded to n) into the coalesced layout.
template <int M, bool VEC>
__device__ __forceinline__ void load_row(float (&v)[Geo<M>::EPL], const float* __restrict__ src, int d,
                                         uint32_t t, bool valid)
{
    constexpr int EPL = Geo<M>::EPL;
    const uint32_t tb = tpart<M, 0>(t);
    if constexpr (VEC) {
#pragma unroll
        for (int j = 0; j < EPL / 4; ++j) {
            const uint32_t i0 = tb | rpart(M, 0, 4 * j);
            float4 q = make_float4(0.f, 0.f, 0.f, 0.f);
            if (valid && (int)i0 < d)
                q = *reinterpret_cast<const float4*>(src + i0);
            v[4 * j] = q.x;
            v[4 * j + 1] = q.y;
            v[4 * j + 2] = q.z;
            v[4 * j + 3] = q.w;
        }
    } else {
#pragma unroll
        for (int r = 0; r < EPL; ++r) {
            const uint32_t i = tb | rpart(M, 0, r);
            v[r] = (valid && (int)i < d) ? src[i] : 0.f;
        }
    }
}

// Load n parameter values (natural order, n % 4 == 0 when M >= 2) into the
// coalesced layout.
template <int M>
__device__ __forceinline__ void load_param_coal(float (&v)[Geo<M>::EPL], const float* __restrict__ src, uint32_t t)
{
    constexpr int EPL = Geo<M>::EPL;
    const uint32_t tb = tpart<M, 0>(t);
    if constexpr (M >= 2) {
#pragma unroll
        for (int j = 0; j < EPL / 4; ++j) {
            const float4 q = *reinterpret_cast<const float4*>(src + (tb | rpart(M, 0, 4 * j)));
            v[4 * j] = q.x;
            v[4 * j + 1] = q.y;
            v[4 * j + 2] = q.z;
            v[4 * j + 3] = q.w;
        }
    } else {
#pragma unroll
        for (int r = 0; r < EPL; ++r)
            v[r] = src[tb | rpart(M, 0, r)];
    }
}

// Load EPL consecutive values owned by lane t from a lane-major array
// (element r of lane t at src[t * EPL + r]).
template <int M, typename TT>
__device__ __forceinline__ void load_lane_major(TT (&v)[Geo<M>::EPL], const TT* __restrict__ src, uint32_t t)
{
    constexpr int EPL = Geo<M>::EPL;
    const TT* p = src + (size_t)t * EPL;
    if constexpr (EPL % 4 == 0 && sizeof(TT) == 4) {
#pragma unroll
        for (int j = 0; j < EPL / 4; ++j) {
            const uint4 q = *reinterpret_cast<const uint4*>(p + 4 * j);
            v[4 * j] = __builtin_bit_cast(TT, q.x);
            v[4 * j + 1] = __builtin_bit_cast(TT, q.y);
            v[4 * j + 2] = __builtin_bit_cast(TT, q.z);
            v[4 * j + 3] = __builtin_bit_cast(TT, q.w);
        }
    } else {
#pragma unroll
        for (int r = 0; r < EPL; ++r)
            v[r] = p[r];
    }
}

// Store the coalesced layout to dst[i] for all n indices (VEC: float4).
template <int M, bool VEC>
__device__ __forceinline__ void store_coal(float* __restrict__ dst, uint32_t t, const float (&v)[Geo<M>::EPL])
{
    constexpr int EPL = Geo<M>::EPL;
    const uint32_t tb = tpart<M, 0>(t);
    if constexpr (VEC) {
#pragma unroll
        for (int j = 0; j < EPL / 4; ++j) {
            const v4f q = {v[4 * j], v[4 * j + 1], v[4 * j + 2], v[4 * j + 3]};
            __builtin_nontemporal_store(q, reinterpret_cast<v4f*>(dst + (tb | rpart(M, 0, 4 * j))));
        }
    } else {
#pragma unroll
        for (int r = 0; r < EPL; ++r)
            dst[tb | rpart(M, 0, r)] = v[r];
    }
}

// ------------------------------------------------------------------ feature map
// cos and sin of pi*t (t in half turns), both scaled by c = 1/sqrt(nE).
// t = k + f with k = rint(t), |f| <= 1/2; sin(pi f) = f P(f^2), cos(pi f) =
// Q(f^2) with near-minimax polynomials (errors 3e-9 and 5e-8 on [-1/2, 1/2])
// whose coefficients arrive pre-multiplied by c; (-1)^k fixes the sign.
struct FeatCoef {
    float s[5];
    float c[5];
};

__device__ __forceinline__ void cossin_hturn(float t, const FeatCoef& q, float& co, float& si)
{
    const float k = __builtin_rintf(t);
    const float f = t - k;
    const float u = f * f;
    float ps = __builtin_fmaf(q.s[4], u, q.s[3]);
    ps = __builtin_fmaf(ps, u, q.s[2]);
    ps = __builtin_fmaf(ps, u, q.s[1]);
    ps = __builtin_fmaf(ps, u, q.s[0]);
    float pc = __builtin_fmaf(q.c[4], u, q.c[3]);
    pc = __builtin_fmaf(pc, u, q.c[2]);
    pc = __builtin_fmaf(pc, u, q.c[1]);
    pc = __builtin_fmaf(pc, u, q.c[0]);
    const float s = ps * f;
    const uint32_t sg = ((uint32_t)(int)k) << 31;
    co = __uint_as_float(__float_as_uint(pc) ^ sg);
    si = __uint_as_float(__float_as_uint(s) ^ sg);
}

}  // namespace mck
