// layout.hpp -- how one length-n vector is spread over the lanes of a wave (or
// a workgroup) and over each lane's registers, for the in-register / LDS
// Walsh-Hadamard transform.
//
// n = 2^M.  Each lane holds EPL = 2^P elements (P = min(M, 5)) in registers;
// LPR = 2^(M-P) lanes share one vector.  A "layout" says which P index bits
// are register bits (butterflies on them are lane-local) and which are lane
// bits (in increasing order).  Sylvester's H is the tensor product of one 2x2
// butterfly per index bit (section "Fast Walsh Hadamard": H_n c =
// [H c0 + H c1; H c0 - H c1] splits on the top bit, and recursively on every
// bit), so the stages can be applied bit by bit in any order; the transform
// moves between layouts through LDS so that every bit is a register bit once.
//
//   layout 0 ("coalesced"): register bits {0, 1, M-3, M-2, M-1}.  Lane t
//     holds the float4 chunks at 4t + j 2^(M-3), j = 0..7, so consecutive
//     lanes touch consecutive 16-byte chunks in HBM.
//   layout k >= 1 ("chunk k"): register bits = the five consecutive bits
//     ending at min(5k+1, M-4) (clamped at bit 0); the chunks together cover
//     bits 2..M-4.
// For M < 5 every bit is a register bit (one lane per vector).
#pragma once

#include <stdint.h>

#if !defined(__HIPCC__) && !defined(__host__)
#define __host__
#define __device__
#endif

namespace mck {

constexpr int cmin(int a, int b) { return a < b ? a : b; }
constexpr int cmax(int a, int b) { return a > b ? a : b; }

template <int M>
struct Geo {
    static_assert(M >= 1 && M <= 15, "single-pass transform covers 2 <= n <= 2^15");
    static constexpr int n = 1 << M;
    static constexpr int P = M < 5 ? M : 5;       // register bits per layout
    static constexpr int EPL = 1 << P;            // elements per lane
    static constexpr int T = M - P;               // lane bits per vector
    static constexpr int LPR = 1 << T;            // lanes per vector
    static constexpr bool kMulti = LPR > 64;      // vector spans several waves
    static constexpr int BLOCK = kMulti ? LPR : 64;
    static constexpr int RPB = kMulti ? 1 : 64 / LPR;  // vectors (rows) per block
    // LDS row-region padding: spreads the row groups of one wave over banks.
    static constexpr int PAD = (M <= 5) ? 1 : (M <= 9 ? 4 : (M == 10 ? 32 : 0));
    static constexpr int STRIDE = n + PAD;        // floats per row region
    static constexpr int K = M >= 6 ? (M - 5 + 4) / 5 : 0;  // chunk layouts
    static constexpr int LDS_FLOATS = RPB * STRIDE;
};

// index bit held by register bit b in layout `id`
constexpr int reg_bit(int M, int id, int b)
{
    if (M < 5)
        return b;
    if (id == 0)
        return b < 2 ? b : M - 5 + b;
    int top = cmin(5 * id + 1, M - 4);
    int lo = cmax(top - 4, 0);
    return lo + b;
}

constexpr int nreg_bits(int M) { return M < 5 ? M : 5; }

constexpr bool is_reg_bit(int M, int id, int bit)
{
    for (int b = 0; b < nreg_bits(M); ++b)
        if (reg_bit(M, id, b) == bit)
            return true;
    return false;
}

constexpr uint32_t reg_mask(int M, int id)
{
    uint32_t m = 0;
    for (int b = 0; b < nreg_bits(M); ++b)
        m |= 1u << reg_bit(M, id, b);
    return m;
}

// index bit held by lane bit b in layout `id` (non-register bits, ascending)
constexpr int thr_bit(int M, int id, int b)
{
    int cnt = 0;
    for (int k = 0; k < M; ++k)
        if (!is_reg_bit(M, id, k)) {
            if (cnt == b)
                return k;
            ++cnt;
        }
    return -1;
}

// register part of the index of register r in layout `id`
constexpr uint32_t rpart(int M, int id, int r)
{
    uint32_t i = 0;
    for (int b = 0; b < nreg_bits(M); ++b)
        i |= (uint32_t)((r >> b) & 1) << reg_bit(M, id, b);
    return i;
}

// LDS position of index i: bits 7..9 are folded into bits 2..4 so that every
// layout's lanes spread over distinct banks.  XOR-linear: phys(a|b) =
// phys(a) ^ phys(b) for disjoint a, b.  Bits 0,1 are untouched, so float4
// chunks stay contiguous.
__host__ __device__ constexpr uint32_t phys(uint32_t i) { return i ^ (((i >> 7) & 7u) << 2); }

// Index bits processed (butterflies applied) at each step of the two
// transforms.  Transform 1 visits layout 0, then chunks 1..K; transform 2
// visits chunks K..1, then layout 0.
constexpr uint32_t fwd1_new_bits(int M, int step)  // step 0 = layout 0, step k = chunk k
{
    uint32_t done = 0;
    for (int s = 0; s < step; ++s)
        done |= reg_mask(M, s);
    return reg_mask(M, step) & ~done;
}

constexpr uint32_t fwd2_new_bits(int M, int K, int id)  // id = K..1 then 0
{
    uint32_t done = 0;
    for (int s = K; s > id && s >= 1; --s)
        done |= reg_mask(M, s);
    if (id == 0)
        for (int s = K; s >= 1; --s)
            done |= reg_mask(M, s);
    return reg_mask(M, id) & ~done;
}

}  // namespace mck
