// layout.hpp -- how one length-n vector is spread over the lanes of a wave (or
// a workgroup) and over each lane's registers, for the in-register / LDS
// Walsh-Hadamard transform.
//
// n = 2^M.  Each lane holds EPL = 2^Q elements (Q = min(M, P), P = 4 or 5 is
// the kernel's choice) in registers; LPR = 2^(M-Q) lanes share one vector.  A
// "layout" says which Q index bits are register bits (butterflies on them are
// lane-local) and which are lane bits (in increasing order).  Sylvester's H is
// the tensor product of one 2x2 butterfly per index bit (section "Fast Walsh
// Hadamard": H_n c = [H c0 + H c1; H c0 - H c1] splits on the top bit, and
// recursively on every bit), so the stages can be applied bit by bit in any
// order; the transform moves between layouts through LDS so that every bit is
// a register bit once.
//
//   layout 0 ("coalesced"): register bits {0, 1} and the top Q-2 bits.  Lane
//     t holds float4 chunks at 4t + j 2^(M-Q+2), so consecutive lanes touch
//     consecutive 16-byte chunks in HBM.
//   layout k >= 1 ("chunk k"): register bits = the Q consecutive bits ending
//     at min(Qk+1, M-Q+1) (clamped at bit 0); the chunks together cover bits
//     2 .. M-Q+1.
//   layout kSW ("swapped"), only when one vector fills exactly the 64 lanes
//     of a wave (M - Q = 6): layout 0 with its two top register bits
//     exchanged for lane bits 4 and 5 (index bits 6 and 7) by the cross-lane
//     swaps v_permlane16_swap / v_permlane32_swap, which move data between
//     the lanes of a wave without LDS.  A transform then visits layout 0,
//     kSW and chunk 1 with a single LDS round trip.
// For M <= P every bit is a register bit (one lane per vector).
#pragma once

#include <stdint.h>

#if !defined(__HIPCC__) && !defined(__host__)
#define __host__
#define __device__
#endif

namespace mck {

constexpr int cmin(int a, int b) { return a < b ? a : b; }
constexpr int cmax(int a, int b) { return a > b ? a : b; }

constexpr int nreg_bits(int M, int P) { return M < P ? M : P; }

constexpr int kSW = 7;  // id of the swapped layout

// one vector per wave over all 64 lanes: the swapped layout applies
constexpr bool swap_geo(int M, int P) { return M > P && M - P == 6; }

// LDS position of index i: 4 floats of padding after every 2^(P+2).  The
// lanes of one wave-half then hit 32 distinct banks in every layout, float4
// chunks stay contiguous and 16-byte aligned, and the map is additive over
// disjoint bit sets, phys(a | b) = phys(a) + phys(b), so an LDS address is a
// per-lane base plus a compile-time offset per register.
template <int P>
__host__ __device__ constexpr uint32_t phys(uint32_t i)
{
    return i + 4u * (i >> (P + 2));
}

template <int M, int P>
struct Geo {
    static_assert(M >= 1 && M <= 15, "single-pass transform covers 2 <= n <= 2^15");
    static_assert(P == 4 || P == 5, "4 or 5 register bits per layout");
    static constexpr int n = 1 << M;
    static constexpr int Q = nreg_bits(M, P);  // register bits per layout
    static constexpr int EPL = 1 << Q;         // elements per lane
    static constexpr int T = M - Q;            // lane bits per vector
    static constexpr int LPR = 1 << T;         // lanes per vector
    static constexpr bool kMulti = LPR > 64;   // vector spans several waves
    static constexpr int BLOCK = kMulti ? LPR : 64;
    static constexpr int RPB = kMulti ? 1 : 64 / LPR;  // vectors (rows) per wave
    static constexpr int K = M > P ? (M - P + P - 1) / P : 0;  // chunk layouts
    // The forward transform ("up") ends, and the inverse-order one
    // ("down") starts, in layout GL: the layout of the Pi gather/scatter.
    static constexpr bool kSwap = swap_geo(M, P);
    static constexpr int GL = kSwap ? 1 : K;
    // LDS footprint of one vector, and of one row region including padding
    // that spreads the row groups of one wave over banks (and keeps float4
    // alignment where float4 access is used)
    static constexpr int PHYS = (int)phys<P>((uint32_t)n - 1u) + 1;
    static constexpr int PAD = (M <= P) ? 1 : (M <= 9 ? 4 : 0);
    static constexpr int STRIDE = PHYS + PAD;
    static constexpr int LDS_FLOATS = RPB * STRIDE;
};

// index bit held by register bit b in layout `id`
constexpr int reg_bit(int M, int P, int id, int b)
{
    if (M <= P)
        return b;
    if (id == 0)
        return b < 2 ? b : M - P + b;
    if (id == kSW)  // layout 0 with register bits P-2, P-1 <-> lane bits 4, 5 (index bits 6, 7)
        return b < P - 2 ? reg_bit(M, P, 0, b) : 6 + (b - (P - 2));
    int top = cmin(P * id + 1, M - P + 1);
    int lo = cmax(top - P + 1, 0);
    return lo + b;
}

constexpr bool is_reg_bit(int M, int P, int id, int bit)
{
    for (int b = 0; b < nreg_bits(M, P); ++b)
        if (reg_bit(M, P, id, b) == bit)
            return true;
    return false;
}

constexpr uint32_t reg_mask(int M, int P, int id)
{
    uint32_t m = 0;
    for (int b = 0; b < nreg_bits(M, P); ++b)
        m |= 1u << reg_bit(M, P, id, b);
    return m;
}

// index bit held by lane bit b in layout `id` (non-register bits, ascending;
// in the swapped layout lane bits 4 and 5 hold layout 0's two top register
// bits)
constexpr int thr_bit(int M, int P, int id, int b)
{
    if (id == kSW && M > P && b >= 4)
        return b < 6 ? reg_bit(M, P, 0, P - 2 + (b - 4)) : -1;
    int cnt = 0;
    for (int k = 0; k < M; ++k)
        if (!is_reg_bit(M, P, id, k)) {
            if (cnt == b)
                return k;
            ++cnt;
        }
    return -1;
}

// register part of the index of register r in layout `id`
constexpr uint32_t rpart(int M, int P, int id, int r)
{
    uint32_t i = 0;
    for (int b = 0; b < nreg_bits(M, P); ++b)
        i |= (uint32_t)((r >> b) & 1) << reg_bit(M, P, id, b);
    return i;
}

// Index bits processed (butterflies applied) at each step of the two
// transforms.  Transform "up" visits layout 0, then chunks 1..K; transform
// "down" visits chunks K..1, then layout 0.
constexpr uint32_t up_new_bits(int M, int P, int step)  // step 0 = layout 0, step k = chunk k
{
    uint32_t done = 0;
    for (int s = 0; s < step; ++s)
        done |= reg_mask(M, P, s);
    return reg_mask(M, P, step) & ~done;
}

constexpr uint32_t down_new_bits(int M, int P, int K, int id)  // id = K..1 then 0
{
    uint32_t done = 0;
    for (int s = K; s > id && s >= 1; --s)
        done |= reg_mask(M, P, s);
    if (id == 0)
        for (int s = K; s >= 1; --s)
            done |= reg_mask(M, P, s);
    return reg_mask(M, P, id) & ~done;
}

}  // namespace mck
