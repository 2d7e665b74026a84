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

// a lane's register array in a (M, P) geometry
template <typename TT, int M, int P>
using LaneArr = TT[Geo<M, P>::EPL];

// Orders LDS traffic of one wave: LDS instructions of a wave execute in issue
// order, so only the compiler must be kept from moving accesses across.
__device__ __forceinline__ void wave_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The lane index as a value the compiler cannot see through.  LDS
// instructions reach 64 KiB past their address VGPR; in a row buffer larger
// than that, every access further out needs an address VGPR of its own, and
// when those addresses derive from a loop-invariant lane index the compiler
// hoists them out of the kernel's loop, where they stay live and push the
// transform into spills.  Passing the transforms this laundered copy makes
// it compute them where they are used.
__device__ __forceinline__ uint32_t lane_opaque(uint32_t t)
{
    asm volatile("" : "+v"(t));
    return t;
}

// t, laundered when the geometry's row buffer exceeds the 64 KiB offset reach
template <int M, int P>
__device__ __forceinline__ uint32_t lds_lane(uint32_t t)
{
    if constexpr ((int64_t)Geo<M, P>::LDS_FLOATS * 4 > 65536)
        return lane_opaque(t);
    else
        return t;
}

template <int M, int P>
__device__ __forceinline__ void lds_sync()
{
    if constexpr (Geo<M, P>::kMulti)
        __syncthreads();
    else
        wave_fence();
}

// index bits owned by lane t in layout ID
template <int M, int P, int ID>
__device__ __forceinline__ uint32_t tpart(uint32_t t)
{
    uint32_t i = 0;
#pragma unroll
    for (int b = 0; b < Geo<M, P>::T; ++b)
        i |= ((t >> b) & 1u) << thr_bit(M, P, ID, b);
    return i;
}

// Radix-2 butterflies (a, b) -> (a + b, a - b) on every register bit of
// layout ID whose index bit is in MASK: pairs (i, i + 2^k), bit k of i clear,
// natural (Sylvester) order.
template <int M, int P, int ID, uint32_t MASK>
__device__ __forceinline__ void stages(LaneArr<float, M, P>& v)
{
    constexpr int Q = Geo<M, P>::Q, EPL = Geo<M, P>::EPL;
#pragma unroll
    for (int b = 0; b < Q; ++b) {
        if (((MASK >> reg_bit(M, P, ID, b)) & 1u) == 0)
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
template <int M, int P, int ID>
constexpr bool lds_vec() { return (ID == 0 || ID == kSW) && M > P; }

template <int M, int P, int ID>
__device__ __forceinline__ void lds_put(float* buf, uint32_t t, const LaneArr<float, M, P>& v)
{
    constexpr int EPL = Geo<M, P>::EPL;
    float* base = buf + phys<P>(tpart<M, P, ID>(t));
    if constexpr (lds_vec<M, P, ID>()) {
#pragma unroll
        for (int j = 0; j < EPL / 4; ++j) {
            float4 q = make_float4(v[4 * j], v[4 * j + 1], v[4 * j + 2], v[4 * j + 3]);
            *reinterpret_cast<float4*>(base + phys<P>(rpart(M, P, ID, 4 * j))) = q;
        }
    } else {
#pragma unroll
        for (int r = 0; r < EPL; ++r)
            base[phys<P>(rpart(M, P, ID, r))] = v[r];
    }
}

template <int M, int P, int ID>
__device__ __forceinline__ void lds_get(const float* buf, uint32_t t, LaneArr<float, M, P>& v)
{
    constexpr int EPL = Geo<M, P>::EPL;
    const float* base = buf + phys<P>(tpart<M, P, ID>(t));
    if constexpr (lds_vec<M, P, ID>()) {
#pragma unroll
        for (int j = 0; j < EPL / 4; ++j) {
            const float4 q = *reinterpret_cast<const float4*>(base + phys<P>(rpart(M, P, ID, 4 * j)));
            v[4 * j] = q.x;
            v[4 * j + 1] = q.y;
            v[4 * j + 2] = q.z;
            v[4 * j + 3] = q.w;
        }
    } else {
#pragma unroll
        for (int r = 0; r < EPL; ++r)
            v[r] = base[phys<P>(rpart(M, P, ID, r))];
    }
}

// Move a vector from layout X to layout Y through the row's LDS region.
template <int M, int P, int X, int Y>
__device__ __forceinline__ void relayout(LaneArr<float, M, P>& v, float* buf, uint32_t t)
{
    lds_put<M, P, X>(buf, t, v);
    lds_sync<M, P>();
    lds_get<M, P, Y>(buf, t, v);
    lds_sync<M, P>();
}

// Exchange register bits P-2 and P-1 with lane bits 4 and 5 (layout 0 <->
// layout kSW).  v_permlane16_swap(a, b) swaps the odd 16-lane rows of a with
// the even rows of b; applied to the registers (r, r + 2^k) it transposes
// register bit k with lane bit 4, and v_permlane32_swap does the same with
// lane bit 5 (halves of the wave).  Each is its own inverse.
template <int M, int P>
__device__ __forceinline__ void swap_hi(LaneArr<float, M, P>& v)
{
    constexpr int EPL = Geo<M, P>::EPL;
    static_assert(Geo<M, P>::kSwap, "swapped layout needs one vector per 64 lanes");
#pragma unroll
    for (int r = 0; r < EPL; ++r) {
        if (r & (1 << (P - 2)))
            continue;
        const auto q = __builtin_amdgcn_permlane16_swap(__float_as_uint(v[r]), __float_as_uint(v[r | (1 << (P - 2))]),
                                                        false, false);
        v[r] = __uint_as_float(q[0]);
        v[r | (1 << (P - 2))] = __uint_as_float(q[1]);
    }
#pragma unroll
    for (int r = 0; r < EPL; ++r) {
        if (r & (1 << (P - 1)))
            continue;
        const auto q = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[r]), __float_as_uint(v[r | (1 << (P - 1))]),
                                                        false, false);
        v[r] = __uint_as_float(q[0]);
        v[r | (1 << (P - 1))] = __uint_as_float(q[1]);
    }
}

// bits visited by the swapped transform: layout 0, kSW, chunk 1
template <int M, int P>
constexpr bool swap_covers()
{
    return (reg_mask(M, P, 0) | reg_mask(M, P, kSW) | reg_mask(M, P, 1)) == (1u << M) - 1u;
}

// H v, starting in layout 0 and ending in layout GL (the last chunk layout,
// or chunk 1 in the swapped geometry).
template <int M, int P>
__device__ __forceinline__ void fwht_up(LaneArr<float, M, P>& v, float* buf, uint32_t t)
{
    constexpr int K = Geo<M, P>::K;
    if constexpr (Geo<M, P>::kSwap) {
        static_assert(swap_covers<M, P>(), "layouts 0, kSW and 1 must cover every bit");
        constexpr uint32_t m0 = reg_mask(M, P, 0), ms = reg_mask(M, P, kSW);
        stages<M, P, 0, m0>(v);
        swap_hi<M, P>(v);
        stages<M, P, kSW, ms & ~m0>(v);
        relayout<M, P, kSW, 1>(v, buf, t);
        stages<M, P, 1, reg_mask(M, P, 1) & ~(m0 | ms)>(v);
        return;
    }
    stages<M, P, 0, up_new_bits(M, P, 0)>(v);
    if constexpr (K >= 1) {
        relayout<M, P, 0, 1>(v, buf, t);
        stages<M, P, 1, up_new_bits(M, P, 1)>(v);
    }
    if constexpr (K >= 2) {
        relayout<M, P, 1, 2>(v, buf, t);
        stages<M, P, 2, up_new_bits(M, P, 2)>(v);
    }
    if constexpr (K >= 3) {
        relayout<M, P, 2, 3>(v, buf, t);
        stages<M, P, 3, up_new_bits(M, P, 3)>(v);
    }
    static_assert(K <= 3, "at most three chunk layouts");
}

// H v, starting in layout GL and ending in layout 0.
template <int M, int P>
__device__ __forceinline__ void fwht_down(LaneArr<float, M, P>& v, float* buf, uint32_t t)
{
    constexpr int K = Geo<M, P>::K;
    if constexpr (Geo<M, P>::kSwap) {
        constexpr uint32_t m1 = reg_mask(M, P, 1), ms = reg_mask(M, P, kSW);
        stages<M, P, 1, m1>(v);
        relayout<M, P, 1, kSW>(v, buf, t);
        stages<M, P, kSW, ms & ~m1>(v);
        swap_hi<M, P>(v);
        stages<M, P, 0, reg_mask(M, P, 0) & ~(m1 | ms)>(v);
        return;
    }
    if constexpr (K >= 3) {
        stages<M, P, 3, down_new_bits(M, P, K, 3)>(v);
        relayout<M, P, 3, 2>(v, buf, t);
    }
    if constexpr (K >= 2) {
        stages<M, P, 2, down_new_bits(M, P, K, 2)>(v);
        relayout<M, P, 2, 1>(v, buf, t);
    }
    if constexpr (K >= 1) {
        stages<M, P, 1, down_new_bits(M, P, K, 1)>(v);
        relayout<M, P, 1, 0>(v, buf, t);
    }
    stages<M, P, 0, down_new_bits(M, P, K, 0)>(v);
}

// ------------------------------------------------------------------ buffer access
// HBM traffic of the hot kernels goes through buffer instructions: one
// uniform resource (base, byte range) per array lives in SGPRs, each lane
// keeps a 32-bit byte offset that is reused across expansions (the
// expansion's offset rides in the scalar offset), chunk offsets are
// immediates, and offsets past the range read as zero (hardware range
// check), which pads rows to n without branches.  Every array a launch
// touches is kept below 2^31 bytes by the host.
typedef int v4i __attribute__((ext_vector_type(4)));
typedef __amdgpu_buffer_rsrc_t rsrc_t;

constexpr uint32_t kOutOfRange = 0x7ffffff0u;  // any offset >= every range

__device__ __forceinline__ rsrc_t make_rsrc(const void* p, uint32_t bytes)
{
    // word 3 of the descriptor for gfx9-family raw (untyped) buffers
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

// AUX = cache policy bits of the instruction (2: streaming / non-temporal).
template <int AUX = 0>
__device__ __forceinline__ void bload4(float* dst, rsrc_t r, uint32_t voff, uint32_t soff)
{
    const v4i q = __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, AUX);
    dst[0] = __int_as_float(q.x);
    dst[1] = __int_as_float(q.y);
    dst[2] = __int_as_float(q.z);
    dst[3] = __int_as_float(q.w);
}

__device__ __forceinline__ void bload4u(uint32_t* dst, rsrc_t r, uint32_t voff, uint32_t soff)
{
    const v4i q = __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0);
    dst[0] = (uint32_t)q.x;
    dst[1] = (uint32_t)q.y;
    dst[2] = (uint32_t)q.z;
    dst[3] = (uint32_t)q.w;
}

template <int AUX = 0>
__device__ __forceinline__ float bload1(rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __int_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, AUX));
}

// 128-bit stores take the whole byte offset in the VGPR (constant parts go
// to the instruction's immediate field) and a literal zero scalar offset.
// A store wider than 64 bits reads its data VGPRs after issue; the compiler
// separates it from a VALU write of those VGPRs only when the scalar offset
// is not a register, and on gfx950 we observed the overwritten value reach
// memory when it was one.
__device__ __forceinline__ void bstore4_nt(rsrc_t r, uint32_t voff, float a, float b, float c, float d)
{
    const v4i q = {__float_as_int(a), __float_as_int(b), __float_as_int(c), __float_as_int(d)};
    __builtin_amdgcn_raw_buffer_store_b128(q, r, (int)voff, 0, 2);  // streaming (non-temporal)
}

__device__ __forceinline__ void bstore4(rsrc_t r, uint32_t voff, float a, float b, float c, float d)
{
    const v4i q = {__float_as_int(a), __float_as_int(b), __float_as_int(c), __float_as_int(d)};
    __builtin_amdgcn_raw_buffer_store_b128(q, r, (int)voff, 0, 0);
}

__device__ __forceinline__ void bstore1(rsrc_t r, uint32_t voff, uint32_t soff, float a)
{
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_int(a), r, (int)voff, (int)soff, 0);
}

// Row of length d at byte offset rowoff (zero-padded to n) into the
// coalesced layout; invalid rows read as zero.
template <int M, int P, bool VEC, int AUX = 0>
__device__ __forceinline__ void bload_row(LaneArr<float, M, P>& v, rsrc_t r, uint32_t rowoff, int d, uint32_t t,
                                          bool valid)
{
    constexpr int EPL = Geo<M, P>::EPL;
    const uint32_t tb = tpart<M, P, 0>(t);
    if constexpr (VEC) {
#pragma unroll
        for (int j = 0; j < EPL / 4; ++j) {
            const uint32_t i0 = tb | rpart(M, P, 0, 4 * j);
            const uint32_t off = (valid && (int)i0 < d) ? rowoff + 4u * i0 : kOutOfRange;
            bload4<AUX>(&v[4 * j], r, off, 0);
        }
    } else {
#pragma unroll
        for (int k = 0; k < EPL; ++k) {
            const uint32_t i = tb | rpart(M, P, 0, k);
            v[k] = bload1<AUX>(r, (valid && (int)i < d) ? rowoff + 4u * i : kOutOfRange, 0);
        }
    }
}

// n values in natural order at scalar byte offset soff, coalesced layout.
template <int M, int P>
__device__ __forceinline__ void bload_coal(LaneArr<float, M, P>& v, rsrc_t r, uint32_t soff, uint32_t t)
{
    constexpr int EPL = Geo<M, P>::EPL;
    const uint32_t tb = 4u * tpart<M, P, 0>(t);
    if constexpr (M >= 2) {
#pragma unroll
        for (int j = 0; j < EPL / 4; ++j)
            bload4(&v[4 * j], r, tb, soff + 4u * rpart(M, P, 0, 4 * j));
    } else {
#pragma unroll
        for (int k = 0; k < EPL; ++k)
            v[k] = bload1(r, tb, soff + 4u * rpart(M, P, 0, k));
    }
}

// EPL consecutive 32-bit values of lane q (element k at q * EPL + k).
template <int M, int P, typename TT>
__device__ __forceinline__ void bload_lane(LaneArr<TT, M, P>& v, rsrc_t r, uint32_t soff, uint32_t q)
{
    constexpr int EPL = Geo<M, P>::EPL;
    const uint32_t base = 4u * q * EPL;
    if constexpr (EPL % 4 == 0) {
#pragma unroll
        for (int j = 0; j < EPL / 4; ++j) {
            if constexpr (sizeof(TT) == 4 && TT(0.5f) == TT(0))  // integer
                bload4u(reinterpret_cast<uint32_t*>(&v[4 * j]), r, base, soff + 16u * j);
            else
                bload4(reinterpret_cast<float*>(&v[4 * j]), r, base, soff + 16u * j);
        }
    } else {
#pragma unroll
        for (int k = 0; k < EPL; ++k)
            v[k] = __builtin_bit_cast(TT, bload1(r, base, soff + 4u * k));
    }
}

// ------------------------------------------------------------------ storage types
// x and phi may be stored as FP32, bfloat16 or IEEE half; arithmetic stays
// FP32.  16-bit values widen exactly; FP32 results narrow with
// round-to-nearest-even (v_cvt_pk_bf16_f32 / v_cvt_pk_f16_f32 on gfx950).
enum : int { kF32 = 0, kBF16 = 1, kF16 = 2 };

template <int T>
constexpr uint32_t elem_bytes() { return T == kF32 ? 4u : 2u; }

typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2_t __attribute__((ext_vector_type(2)));
typedef unsigned u32x2_t __attribute__((ext_vector_type(2)));

template <int T>
__device__ __forceinline__ uint32_t pack2(float a, float b)
{
    const f32x2_t v = {a, b};
    if constexpr (T == kBF16)
        return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2_t));
    else
        return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, f16x2_t));
}

template <int T>
__device__ __forceinline__ void unpack2(uint32_t w, float& a, float& b)
{
    f32x2_t v;
    if constexpr (T == kBF16)
        v = __builtin_convertvector(__builtin_bit_cast(bf16x2_t, w), f32x2_t);
    else
        v = __builtin_convertvector(__builtin_bit_cast(f16x2_t, w), f32x2_t);
    a = v.x;
    b = v.y;
}

template <int T>
__device__ __forceinline__ float widen1(uint32_t h)
{
    float a, b;
    unpack2<T>(h & 0xffffu, a, b);
    return a;
}

// Row of length d (elements of type T) at byte offset rowoff, zero-padded to
// n, into the coalesced layout; invalid rows read as zero.
template <int M, int P, bool VEC, int T, int AUX = 0>
__device__ __forceinline__ void bload_row_t(LaneArr<float, M, P>& v, rsrc_t r, uint32_t rowoff, int d, uint32_t t,
                                            bool valid)
{
    if constexpr (T == kF32) {
        bload_row<M, P, VEC, AUX>(v, r, rowoff, d, t, valid);
    } else {
        constexpr int EPL = Geo<M, P>::EPL;
        const uint32_t tb = tpart<M, P, 0>(t);
        if constexpr (VEC) {
#pragma unroll
            for (int j = 0; j < EPL / 4; ++j) {
                const uint32_t i0 = tb | rpart(M, P, 0, 4 * j);
                const uint32_t off = (valid && (int)i0 < d) ? rowoff + 2u * i0 : kOutOfRange;
                const u32x2_t q = __builtin_bit_cast(u32x2_t, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, AUX));
                unpack2<T>(q.x, v[4 * j], v[4 * j + 1]);
                unpack2<T>(q.y, v[4 * j + 2], v[4 * j + 3]);
            }
        } else {
#pragma unroll
            for (int k = 0; k < EPL; ++k) {
                const uint32_t i = tb | rpart(M, P, 0, k);
                const uint32_t off = (valid && (int)i < d) ? rowoff + 2u * i : kOutOfRange;
                v[k] = widen1<T>((uint32_t)__builtin_amdgcn_raw_buffer_load_b16(r, (int)off, 0, AUX));
            }
        }
    }
}

// Four consecutive elements (streaming store): 16 bytes in FP32, 8 bytes
// (two packed pairs) in 16-bit types.  The whole offset is in the VGPR.
template <int T>
__device__ __forceinline__ void bstore_quad(rsrc_t r, uint32_t voff, float a, float b, float c, float d)
{
    if constexpr (T == kF32) {
        bstore4_nt(r, voff, a, b, c, d);
    } else {
        const u32x2_t q = {pack2<T>(a, b), pack2<T>(c, d)};
        __builtin_amdgcn_raw_buffer_store_b64(q, r, (int)voff, 0, 2);
    }
}

template <int T>
__device__ __forceinline__ void bstore_elem(rsrc_t r, uint32_t voff, float a)
{
    if constexpr (T == kF32)
        bstore1(r, voff, 0, a);
    else
        __builtin_amdgcn_raw_buffer_store_b16((unsigned short)(pack2<T>(a, 0.f) & 0xffffu), r, (int)voff, 0, 0);
}

// ------------------------------------------------------------------ feature map
// c cos(2 pi t) and c sin(2 pi t) for t in revolutions.  The argument is
// reduced to [0, 1) exactly (fract), then the hardware sine and cosine
// (inputs in revolutions, half rate on gfx950) give an absolute error of
// about 1e-7, well inside the fp32 rounding already present in t.
__device__ __forceinline__ void cossin_rev(float t, float c, float& co, float& si)
{
    const float r = __builtin_amdgcn_fractf(t);
    co = c * __builtin_amdgcn_cosf(r);
    si = c * __builtin_amdgcn_sinf(r);
}

// The same without the scale (callers that fold c into a later product).
__device__ __forceinline__ void cossin_rev1(float t, float& co, float& si)
{
    const float r = __builtin_amdgcn_fractf(t);
    co = __builtin_amdgcn_cosf(r);
    si = __builtin_amdgcn_sinf(r);
}

}  // namespace mck
