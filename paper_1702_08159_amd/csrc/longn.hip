// longn.hip -- the transform and the feature map for n > 2^15 (up to 2^24),
// where one row no longer fits in a workgroup's LDS.
//
// H_n = H_{n/2^15} (x) H_{2^15} (Sylvester's H is the tensor product of one
// 2x2 butterfly per index bit, section "Fast Walsh Hadamard"), so the
// transform splits into two commuting factors
//   a row pass:    H_{2^15} on each contiguous chunk of 2^15 elements
//                  (the register/LDS engine, one chunk per 1024-lane block);
//   column passes: H over the remaining high index bits, at most 5 per pass:
//                  each lane holds the 2^B elements of four adjacent columns
//                  (stride 2^s) in VGPRs, so consecutive lanes read
//                  consecutive 16-byte pieces.
// The feature map per expansion is four passes over two FP32 scratch copies
// u, w of the batch:
//   1. column pass(es) on B o xhat (x read in place, zero padding by range)
//   2. row pass -> u = H B xhat, held in LDS; Pi is applied as an exchange
//      between chunks: each element goes out to w at the place its
//      destination chunk will read it (runs of consecutive positions)
//   3. row pass: each destination chunk reads its contiguous part of w,
//      places the values by dstB in LDS, multiplies by G and transforms -> u
//   4. column pass(es); the last one multiplies by S / (2 pi) and writes
//      c cos, c sin in the storage type of phi.
// A direct gather u[perm[i]] over the whole row would read one 4-byte value
// per 64-byte line from L2; the exchange moves every value twice, in full
// lines.  Row-pass blocks are mapped so that an XCD works on a fixed set of
// chunks, whose plan words then stay in its L2 across rows.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "engine.hpp"
#include "forward.hpp"
#include "launch.hpp"

namespace mck {
namespace {

constexpr int kRowM = 15;        // chunk length 2^15 of the row pass
constexpr int kRowP = 5;         // 32 elements per lane, 1024 lanes per chunk
constexpr int kColThreads = 256;
constexpr int kColMaxB = 5;
constexpr int kMaxChunks = 1 << (24 - kRowM);

using RG = Geo<kRowM, kRowP>;

// Row pass input and output modes.
enum : int { kInRow = 0, kInBucket = 1 };
enum : int { kOutRow = 0, kOutBucket = 1 };

struct RowArgs {
    float* dst;
    const float* src;
    int64_t rows, chunks;
    const float* Gx;         // kInBucket: G of the expansion in exchange order
    const uint32_t* packA;   // kOutBucket
    const int32_t* pdelta;   // kOutBucket
    const uint16_t* dstB;    // kInBucket
};

// Storage slot of exchange position q (0 <= q < 2^15) of a source chunk in
// packA: lane t of the row pass handles the positions q = (4 j + m) 1024 + t
// (j < 8, m < 4), so that the 64 lanes of a wave store 64 consecutive
// exchange positions per instruction, and reads its four positions of j as
// one 16-byte word at slot (j 1024 + t) 4 + m.
__host__ __device__ constexpr uint32_t pack_slot(uint32_t q)
{
    return (((q >> 10) >> 2) * 1024u + (q & 1023u)) * 4u + ((q >> 10) & 3u);
}
static_assert(RG::BLOCK == 1024 && RG::EPL == 32, "pack_slot assumes the 1024-lane, 32-register row pass");

// XCD-aware (row slot, chunk) of a row-pass block: blocks are dealt to the
// 8 XCDs round robin.  With 8 or more chunks, XCD x takes the chunks
// c = x (mod 8) of every row slot, so the plan words of its C / 8 chunks
// (the exchange positions, G, the placement: 320 KB per chunk) are read
// from HBM once and then served by that XCD's L2 for all rows; with fewer
// chunks every XCD's L2 holds them all.
__device__ __forceinline__ void slot_chunk(int64_t chunks, int64_t& slot, int64_t& c)
{
    const int64_t b = blockIdx.x;
    if (chunks >= kXcds) {
        const int64_t xcd = b % kXcds, q = b / kXcds, per = chunks / kXcds;
        c = xcd + kXcds * (q % per);
        slot = q / per;
    } else {
        c = b % chunks;
        slot = b / chunks;
    }
}

// One 2^15 chunk c of RB consecutive rows per block: H_{2^15} of each row's
// chunk input, output to dst (rows of length n = chunks 2^15).
//   kInRow:    the chunk of src (natural order)
//   kInBucket: G o (the elements Pi sends to this chunk), read from the
//              chunk's part of the exchange buffer src and scaled by G in
//              the same order before they are placed in LDS
//   kOutRow:    natural order
//   kOutBucket: every element to its place in the exchange buffer dst
// The chunk's dstB is loaded once per block, and the
// next row's input is loaded into registers while the current row is
// transformed and stored: one block fills a CU's LDS, so this is where its
// HBM latency hides.
template <int IN, int OUT, bool VEC, int RB>
__global__ void __launch_bounds__(RG::BLOCK) k_rows(RowArgs a)
{
    constexpr int M = kRowM, P = kRowP, EPL = RG::EPL, K = RG::K, BLOCK = RG::BLOCK, NQ = EPL / 4;
    constexpr int64_t CH = RG::n;
    __shared__ float lds[RG::LDS_FLOATS];
    int64_t slot, c;
    slot_chunk(a.chunks, slot, c);
    const int64_t r0 = slot * RB;
    if (r0 >= a.rows)
        return;  // uniform per block
    const int nr = a.rows - r0 < RB ? (int)(a.rows - r0) : RB;
    const int64_t n = a.chunks * CH;
    const uint32_t t = threadIdx.x;
    const uint32_t tb = tpart<M, P, 0>(t);

    // the chunk's plan data: dstB stays in VGPRs for all rows; G (in
    // exchange order) and packA are re-read per row (L2) to leave room for
    // the prefetched row
    [[maybe_unused]] const rsrc_t rd = make_rsrc(a.dstB + c * CH, (uint32_t)(CH * 2));
    __shared__ int32_t sdel[OUT == kOutBucket ? kMaxChunks : 1];
    if constexpr (OUT == kOutBucket) {
        const int C = (int)a.chunks;
        for (int i = (int)t; i < C; i += BLOCK)
            sdel[i] = a.pdelta[c * C + i];
    }

    // the row input: layout 0 (kInRow) or exchange order, 4 per float4 (kInBucket)
    float nxt[EPL];
    auto load_input = [&](int64_t r) {
        const rsrc_t rs = make_rsrc(a.src + r * n + c * CH, (uint32_t)(CH * 4));
        if constexpr (IN == kInRow) {
            bload_row<M, P, VEC>(nxt, rs, 0u, (int)CH, t, true);
        } else {
#pragma unroll
            for (int j = 0; j < NQ; ++j)
                bload4(&nxt[4 * j], rs, 16u * (j * BLOCK + t), 0u);
        }
    };
    load_input(r0);

    for (int k = 0; k < nr; ++k) {
        const int64_t r = r0 + k;
        if (k > 0)
            __syncthreads();  // the previous row's last LDS reads are done
        float v[EPL];
        if constexpr (IN == kInBucket) {
            u32x2_t di[NQ];
#pragma unroll
            for (int j = 0; j < NQ; ++j)
                di[j] = __builtin_bit_cast(u32x2_t,
                                           __builtin_amdgcn_raw_buffer_load_b64(rd, (int)(8u * (j * BLOCK + t)), 0, 0));
            {
                const rsrc_t rg = make_rsrc(a.Gx + c * CH, (uint32_t)(CH * 4));
#pragma unroll
                for (int j = 0; j < NQ; ++j) {
                    float gx[4];
                    bload4(gx, rg, 16u * (j * BLOCK + t), 0u);
#pragma unroll
                    for (int m = 0; m < 4; ++m)
                        nxt[4 * j + m] *= gx[m];
                }
            }
#pragma unroll
            for (int j = 0; j < NQ; ++j) {
                lds[phys<P>(di[j].x & 0x7fffu)] = nxt[4 * j];
                lds[phys<P>((di[j].x >> 16) & 0x7fffu)] = nxt[4 * j + 1];
                lds[phys<P>(di[j].y & 0x7fffu)] = nxt[4 * j + 2];
                lds[phys<P>((di[j].y >> 16) & 0x7fffu)] = nxt[4 * j + 3];
            }
            if (k + 1 < nr)
                load_input(r + 1);
            __syncthreads();
            lds_get<M, P, 0>(lds, lds_lane<M, P>(t), v);
            __syncthreads();
        } else {
#pragma unroll
            for (int q = 0; q < EPL; ++q)
                v[q] = nxt[q];
            if (k + 1 < nr)
                load_input(r + 1);
        }
        [[maybe_unused]] uint32_t pk[NQ][4];
        if constexpr (OUT == kOutBucket) {
            const rsrc_t ra = make_rsrc(a.packA + c * CH, (uint32_t)(CH * 4));
#pragma unroll
            for (int j = 0; j < NQ; ++j)
                bload4u(pk[j], ra, 16u * (j * BLOCK + t), 0u);
        }
        fwht_up<M, P>(v, lds, lds_lane<M, P>(t));
        if constexpr (OUT == kOutBucket) {
            lds_put<M, P, RG::GL>(lds, lds_lane<M, P>(t), v);
            __syncthreads();
            const rsrc_t ro = make_rsrc(a.dst + r * n, (uint32_t)(n * 4));
#pragma unroll
            for (int j = 0; j < NQ; ++j)
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const uint32_t q = (uint32_t)((4 * j + m) * BLOCK) + t;  // pk[j][m] is packA at pack_slot(q)
                    const uint32_t w = pk[j][m];
                    const int32_t pos = (int32_t)q + sdel[(w >> kRowM) & (kMaxChunks - 1)];
                    bstore1(ro, 4u * (uint32_t)pos, 0u, lds[phys<P>(w & 0x7fffu)]);
                }
        } else {
            const rsrc_t ro = make_rsrc(a.dst + r * n + c * CH, (uint32_t)(CH * 4));
            relayout<M, P, RG::GL, 0>(v, lds, lds_lane<M, P>(t));
            if constexpr (VEC || IN != kInRow) {
#pragma unroll
                for (int j = 0; j < EPL / 4; ++j)
                    bstore4(ro, 4u * (tb | rpart(M, P, 0, 4 * j)), v[4 * j], v[4 * j + 1], v[4 * j + 2],
                            v[4 * j + 3]);
            } else {
#pragma unroll
                for (int q = 0; q < EPL; ++q)
                    bstore1(ro, 4u * tb, 4u * rpart(M, P, 0, q), v[q]);
            }
        }
    }
}

// ------------------------------------------------------------------ n = 2^16 in one block
// A whole row of n = 2^16 = two 2^15 halves per 1024-lane block: 32 values
// per lane and half in VGPRs (a lane holds the same positions of both
// halves, so everything that pairs element j with j + 2^15 is
// register-local), and each half's relayouts through the one 2^15-float LDS
// buffer in turn.  Pi is split by the outer stage of a Benes network:
//   Pi = S_out (Pi_top (+) Pi_bot) S_in,
// where S_in and S_out exchange, pair by pair, the elements j and j + 2^15
// (register selects), and Pi_top, Pi_bot permute each half within itself
// (a gather through LDS, one half after the other).  The switch settings
// come from a 2-colouring of the source elements computed at plan time
// (k_pair_colour).  Per work item (row, expansion):
//   1. B o xhat (sign words), H_{2^15} on each half, the bit-15 butterfly;
//   2. S_in, Pi_top on the lower half and Pi_bot on the upper half through
//      LDS, S_out, G at the destinations;
//   3. the bit-15 butterfly, H_{2^15} on each half, S / (2 pi), [cos, sin].
// Per item only x is read (from L2 after the first expansion), the plan
// words of the expansion, and phi written: nothing of the row leaves the CU.
//
// Work items: XCD x (blocks b with b % 8 = x, `slots` of them) takes rows
// x, x + 8, x + 16, ... in groups of 8 rows; within a group the items are
// ordered expansion-major, so the group's x rows and one expansion's plan
// words are shared in that XCD's L2.
struct PairArgs {
    const void* x;
    int64_t rows;
    int d;
    int E;
    const uint32_t* Bw;  // sign words [e][h][t]: bit r set where B is -1 at register r of lane t
    const uint32_t* Pw;  // switch words [e][in / out][t]: bit r set where the pair of register r is exchanged
    const uint32_t* Po;  // gather sources [e][h][q][t][4]: 16-bit LDS float indices, two registers per word
    const float* Pg;     // G at the destinations [e][h][q][t][4], register r = 4 q + m
    const float* Sh;
    float cs;
    void* phi;
    const int8_t* xexp;  // nullable per-row exponents of x
    int slots;           // blocks per XCD
};

constexpr int kPairRows = 8;  // rows per group within an XCD
constexpr int64_t kPairN = 2 * RG::n;

template <int XT, int YT, bool VEC>
__global__ void __launch_bounds__(RG::BLOCK, 1) k_forward_pair(PairArgs a)
{
    constexpr int M = kRowM, P = kRowP, EPL = RG::EPL, BLOCK = RG::BLOCK;
    constexpr int64_t CH = RG::n, n = 2 * CH;
    constexpr uint32_t XB = elem_bytes<XT>(), YB = elem_bytes<YT>();
    __shared__ float lds[RG::LDS_FLOATS];
    const int xcd = (int)(blockIdx.x % kXcds), slot = (int)(blockIdx.x / kXcds);
    const int64_t kx = a.rows > xcd ? (a.rows - xcd + kXcds - 1) / kXcds : 0;  // rows of this XCD
    const int64_t jx = (kx + kPairRows - 1) / kPairRows * kPairRows * a.E;
    const int64_t nE = n * a.E;

    // work item j -> (row, e); k >= kx marks the empty tail of a row group
    struct Item {
        int64_t row;
        int e;
        bool live;
    };
    auto item = [&](int64_t j) {
        const int64_t kin = j % kPairRows, q = j / kPairRows;
        const int64_t k = (q / a.E) * kPairRows + kin;
        return Item{xcd + (int64_t)kXcds * k, (int)(q % a.E), k < kx};
    };
    auto next = [&](int64_t j) {
        for (j += a.slots; j < jx; j += a.slots)
            if (item(j).live)
                break;
        return j;
    };
    auto xrsrc = [&](int64_t row) {
        return make_rsrc(static_cast<const char*>(a.x) + row * a.d * XB, (uint32_t)(a.d * XB));
    };
    int64_t j = slot;
    if (j < jx && !item(j).live)
        j = next(j);
    for (; j < jx;) {  // uniform over the block
        // the lane index laundered per item: addresses derived from it are
        // formed where they are used instead of being hoisted out of the
        // item loop, where they would stay live across it
        const uint32_t t = lane_opaque(threadIdx.x);
        const uint32_t tb = tpart<M, P, 0>(t);
        const Item it = item(j);
        const int64_t row = it.row;
        const int e = it.e;
        const int64_t eo = (int64_t)e * n;
        const float xs = a.xexp != nullptr ? __builtin_ldexpf(1.f, (int)a.xexp[row]) : 1.f;

        // 1. H_{2^16} (B o xhat) = the bit-15 butterfly after H_{2^15} on
        //    each half (the two factors commute): the lower half first, then
        //    the upper half, whose x loads overlap the lower transform
        float lo[EPL], hi[EPL];
        bload_row_t<M, P, VEC, XT>(lo, xrsrc(row), 0u, a.d, t, true);
        const uint32_t w0 = a.Bw[(2 * e) * BLOCK + t], w1 = a.Bw[(2 * e + 1) * BLOCK + t];
#pragma unroll
        for (int r = 0; r < EPL; ++r)
            lo[r] = __uint_as_float(__float_as_uint(lo[r] * xs) ^ ((w0 << (31 - r)) & 0x80000000u));
        fwht_up<M, P>(lo, lds, lds_lane<M, P>(t));
        bload_row_t<M, P, VEC, XT>(hi, xrsrc(row), (uint32_t)(CH * XB), a.d - (int)CH, t, true);
#pragma unroll
        for (int r = 0; r < EPL; ++r)
            hi[r] = __uint_as_float(__float_as_uint(hi[r] * xs) ^ ((w1 << (31 - r)) & 0x80000000u));
        fwht_up<M, P>(hi, lds, lds_lane<M, P>(t));
        const uint32_t sw_in = a.Pw[(2 * e) * BLOCK + t];
#pragma unroll
        for (int r = 0; r < EPL; ++r) {
            const float p0 = lo[r], p1 = hi[r];
            lo[r] = p0 + p1;
            hi[r] = p0 - p1;
        }

        // 2. G Pi: S_in; each half's permutation through LDS; S_out; G
        auto exchange = [&](uint32_t w) {
#pragma unroll
            for (int r = 0; r < EPL; ++r) {
                const bool s = ((w >> r) & 1u) != 0u;
                const float p0 = lo[r], p1 = hi[r];
                lo[r] = s ? p1 : p0;
                hi[r] = s ? p0 : p1;
            }
        };
        auto permute_half = [&](float (&v)[EPL], int h) {
            const rsrc_t ro = make_rsrc(a.Po + (int64_t)(2 * e + h) * (EPL / 2) * BLOCK, (uint32_t)(EPL / 2 * BLOCK * 4));
            uint32_t op[EPL / 2];
#pragma unroll
            for (int q = 0; q < EPL / 8; ++q)
                bload4u(&op[4 * q], ro, 16u * (q * BLOCK + t), 0u);
            lds_put<M, P, RG::GL>(lds, lds_lane<M, P>(t), v);
            __syncthreads();
#pragma unroll
            for (int r = 0; r < EPL; ++r)
                v[r] = lds[(op[r >> 1] >> (16 * (r & 1))) & 0xFFFFu];
            __syncthreads();  // LDS free for the next half
        };
        auto scale_g = [&](float (&v)[EPL], int h) {
            const rsrc_t rg = make_rsrc(a.Pg + (int64_t)(2 * e + h) * CH, (uint32_t)(CH * 4));
#pragma unroll
            for (int q = 0; q < EPL / 4; ++q) {
                float g4[4];
                bload4(g4, rg, 16u * (q * BLOCK + t), 0u);
#pragma unroll
                for (int m = 0; m < 4; ++m)
                    v[4 * q + m] *= g4[m];
            }
        };
        exchange(sw_in);
        permute_half(lo, 0);
        permute_half(hi, 1);
        exchange(a.Pw[(2 * e + 1) * BLOCK + t]);
        scale_g(lo, 0);
        scale_g(hi, 1);

        // 3. H_{2^16} G Pi v1: the bit-15 butterfly, H_{2^15} on each half;
        //    z in revolutions (S / 2 pi) for both halves before any store
#pragma unroll
        for (int r = 0; r < EPL; ++r) {
            const float p0 = lo[r], p1 = hi[r];
            lo[r] = p0 + p1;
            hi[r] = p0 - p1;
        }
        fwht_down<M, P>(lo, lds, lds_lane<M, P>(t));
        fwht_down<M, P>(hi, lds, lds_lane<M, P>(t));
        {
            const rsrc_t rs = make_rsrc(a.Sh + eo, (uint32_t)(n * 4));
            float sx[EPL];
            bload_coal<M, P>(sx, rs, 0u, t);
#pragma unroll
            for (int r = 0; r < EPL; ++r)
                lo[r] *= sx[r];
            bload_coal<M, P>(sx, rs, (uint32_t)(CH * 4), t);
#pragma unroll
            for (int r = 0; r < EPL; ++r)
                hi[r] *= sx[r];
        }
        const int64_t jn = next(j);

        // 4. c cos z, c sin z
        const rsrc_t ry = make_rsrc(static_cast<char*>(a.phi) + row * 2 * nE * YB, (uint32_t)(2 * nE * YB));
        auto features = [&](const float (&v)[EPL], int h) {
            const uint32_t yc = YB * (uint32_t)(eo + h * CH + tb), ysn = yc + YB * (uint32_t)nE;
#pragma unroll
            for (int jj = 0; jj < EPL / 4; ++jj) {
                float c4[4], s4[4];
#pragma unroll
                for (int m = 0; m < 4; ++m)
                    cossin_rev(v[4 * jj + m], a.cs, c4[m], s4[m]);
                const uint32_t so = YB * rpart(M, P, 0, 4 * jj);
                bstore_quad<YT>(ry, yc + so, c4[0], c4[1], c4[2], c4[3]);
                bstore_quad<YT>(ry, ysn + so, s4[0], s4[1], s4[2], s4[3]);
            }
        };
        features(lo, 0);
        features(hi, 1);
        j = jn;
    }
}

// ---- plan of k_forward_pair: the outer Benes stage of Pi (gather form,
// v_out[i] = v_in[perm[i]], n = 2N, N = 2^15).  Source element y travels
// through the top subnetwork (colour 0) or the bottom one (colour 1).  The
// input switch of pair j sends j and j + N to different subnetworks, and the
// output switch of pair i takes destinations i and i + N from different ones:
// so y and y ^ N differ in colour, and so do perm[i] and perm[i ^ N].  These
// constraints form disjoint cycles that alternate between the two kinds of
// pair, hence of even length, and colouring a cycle alternately satisfies
// them all (the looping algorithm of Benes network routing).  With
//   link(y) = perm[perm^-1[y ^ N] ^ N]
// (y's input partner, then that element's output partner), the cycle through
// y visits y, y ^ N, link(y), link(y) ^ N, ...: link keeps the colour.

// inv[e][perm[e][i]] = i
__global__ void k_pair_inverse(const int32_t* __restrict__ perm, int64_t E, uint16_t* __restrict__ inv)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= E * kPairN)
        return;
    const int64_t e = i / kPairN;
    inv[e * kPairN + ((uint32_t)perm[i] & (uint32_t)(kPairN - 1))] = (uint16_t)(i % kPairN);
}

__global__ void k_pair_link(const int32_t* __restrict__ perm, const uint16_t* __restrict__ inv, int64_t E,
                            uint16_t* __restrict__ link)
{
    constexpr uint32_t N = RG::n;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= E * kPairN)
        return;
    const int64_t e = i / kPairN;
    const uint32_t y = (uint32_t)(i % kPairN);
    const uint32_t k = (uint32_t)inv[e * kPairN + (y ^ N)] ^ N;
    link[i] = (uint16_t)((uint32_t)perm[e * kPairN + k] & (uint32_t)(kPairN - 1));
}

// One block per expansion: colour[e][j / 32] bit j % 32 = colour of source
// element j < N (that of j + N is the other one).  One lane walks every
// cycle through link, held in LDS; a walk colours the pair {y, y ^ N} per
// step, so a permutation takes N steps in all, and the step budget ends the
// walk even if link were not a bijection.
__global__ void __launch_bounds__(256) k_pair_colour(const uint16_t* __restrict__ link, int64_t E,
                                                     uint32_t* __restrict__ colour)
{
    constexpr uint32_t N = RG::n, W = N / 32;
    __shared__ uint16_t lk[kPairN];
    __shared__ uint32_t seen[W], col[W];
    const int64_t e = blockIdx.x;
    for (uint32_t i = threadIdx.x; i < (uint32_t)kPairN; i += blockDim.x)
        lk[i] = link[e * kPairN + i];
    for (uint32_t i = threadIdx.x; i < W; i += blockDim.x) {
        seen[i] = 0u;
        col[i] = 0u;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t budget = (int32_t)N;
        for (uint32_t w = 0; w < W && budget > 0; ++w) {
            while (seen[w] != 0xFFFFFFFFu && budget > 0) {
                const uint32_t y0 = 32u * w + (uint32_t)__builtin_ctz(~seen[w]);  // colour 0
                uint32_t y = y0;
                do {
                    const uint32_t jj = y & (N - 1u);
                    seen[jj >> 5] |= 1u << (jj & 31u);
                    if (y >= N)
                        col[jj >> 5] |= 1u << (jj & 31u);  // y = jj + N has colour 0
                    y = lk[y];
                } while (y != y0 && --budget > 0);
            }
        }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < W; i += blockDim.x)
        colour[e * W + i] = col[i];
}

// Per expansion e and lane t of k_forward_pair (gather layout GL of the
// 2^15 engine: register r of lane t holds position i(t, r) of each half):
//   Pw[e][0][t] bit r: colour of source i (the input pair travels swapped);
//   Pw[e][1][t] bit r: colour of perm[i] (the output pair arrives swapped);
//   Po[e][h][q][t][m], registers 2(4q+m) and 2(4q+m)+1: LDS float index of
//     the position within the half that Pi_top (h = 0) / Pi_bot (h = 1)
//     gathers for i;
//   Pg[e][h][q][t][m]: G[e][h N + i] for register r = 4q + m.
__global__ void k_pair_plan(const int32_t* __restrict__ perm, const float* __restrict__ G,
                            const uint32_t* __restrict__ colour, int64_t E, uint32_t* __restrict__ Pw,
                            uint32_t* __restrict__ Po, float* __restrict__ Pg)
{
    constexpr int M = kRowM, P = kRowP, EPL = RG::EPL, BLOCK = RG::BLOCK;
    constexpr uint32_t N = RG::n;
    const int64_t gi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gi >= E * BLOCK)
        return;
    const int64_t e = gi / BLOCK;
    const uint32_t t = (uint32_t)(gi % BLOCK);
    const int32_t* pe = perm + e * kPairN;
    const float* ge = G + e * kPairN;
    const uint32_t* ce = colour + e * (N / 32);
    auto colour_of = [&](uint32_t y) {
        const uint32_t jj = y & (N - 1u);
        return ((ce[jj >> 5] >> (jj & 31u)) & 1u) ^ (y >= N ? 1u : 0u);
    };
    uint32_t win = 0, wout = 0, ot[EPL / 2], ob[EPL / 2];
    for (int w = 0; w < EPL / 2; ++w)
        ot[w] = ob[w] = 0u;
    const uint32_t tb = tpart<M, P, RG::GL>(t);
    for (int r = 0; r < EPL; ++r) {
        const uint32_t i = tb | rpart(M, P, RG::GL, r);
        win |= colour_of(i) << r;
        const uint32_t y = (uint32_t)pe[i] & (uint32_t)(kPairN - 1), z = (uint32_t)pe[i + N] & (uint32_t)(kPairN - 1);
        const uint32_t s = colour_of(y);  // 1: perm[i] comes through the bottom subnetwork
        wout |= s << r;
        const uint32_t top = s ? z : y, bot = s ? y : z;
        ot[r >> 1] |= phys<P>(top & (N - 1u)) << (16 * (r & 1));
        ob[r >> 1] |= phys<P>(bot & (N - 1u)) << (16 * (r & 1));
        const int64_t go = ((e * 2) * (EPL / 4) + r / 4) * BLOCK * 4 + t * 4 + r % 4;
        Pg[go] = ge[i];
        Pg[go + (EPL / 4) * BLOCK * 4] = ge[i + N];
    }
    Pw[(e * 2) * BLOCK + t] = win;
    Pw[(e * 2 + 1) * BLOCK + t] = wout;
    for (int w = 0; w < EPL / 2; ++w) {
        const int64_t oo = ((e * 2) * (EPL / 8) + w / 4) * BLOCK * 4 + t * 4 + w % 4;
        Po[oo] = ot[w];
        Po[oo + (EPL / 8) * BLOCK * 4] = ob[w];
    }
}

// Sign words of B for k_forward_pair: word (e, h, t) has bit r set where
// B_e is -1 at element h 2^15 + (the index register r of lane t holds in
// the coalesced layout of the 2^15 engine).
__global__ void k_pair_signs(const float* __restrict__ B, int64_t E, uint32_t* __restrict__ Bw)
{
    constexpr int M = kRowM, P = kRowP, EPL = RG::EPL, BLOCK = RG::BLOCK;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // (e, h, t)
    if (i >= E * 2 * BLOCK)
        return;
    const uint32_t t = (uint32_t)(i % BLOCK);
    const int64_t eh = i / BLOCK;  // 2 e + h
    const float* src = B + (eh / 2) * 2 * RG::n + (eh % 2) * RG::n;
    const uint32_t tb = tpart<M, P, 0>(t);
    uint32_t w = 0;
    for (int r = 0; r < EPL; ++r)
        w |= (src[tb | rpart(M, P, 0, r)] < 0.f ? 1u : 0u) << r;
    Bw[i] = w;
}

// Sh = S / (2 pi) (S in revolutions), from the FP64 S.
__global__ void k_sh(const double* __restrict__ S64, float* __restrict__ Sh, int64_t count)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count)
        Sh[i] = (float)(S64[i] * 0.15915494309189533577);
}

// H over index bits [s, s + B) of every row of length n: lane (row, hi, lo4)
// holds elements hi 2^(s+B) + k 2^s + lo4 + {0..3}, k < 2^B.  With EPI the
// pass is the last one of expansion e: z = v * Sh[i], and c cos z, c sin z
// go to phi (row length 2nE, storage type YT) at e n + i and nE + e n + i.
template <int B, bool EPI, int YT>
__global__ void __launch_bounds__(kColThreads)
    k_cols(float* __restrict__ data, int64_t rows, int64_t n, int s, int64_t blocks_per_row,
           const float* __restrict__ Sh, float cs, int e, int E, void* __restrict__ phi)
{
    constexpr int L = 1 << B;
    const int64_t r = (int64_t)blockIdx.x / blocks_per_row;
    const int64_t q = ((int64_t)blockIdx.x % blocks_per_row) * kColThreads + threadIdx.x;  // float4 column group
    const int64_t lo_groups = (int64_t)1 << (s - 2);
    if (r >= rows || q >= (n >> B) / 4)
        return;
    const int64_t hi = q / lo_groups, lo = (q % lo_groups) * 4;
    const int64_t base = hi * ((int64_t)L << s) + lo;  // element index of k = 0
    float* row = data + r * n;
    const rsrc_t rd = make_rsrc(row, (uint32_t)(n * 4));
    float v[L][4];
#pragma unroll
    for (int k = 0; k < L; ++k)
        bload4(v[k], rd, (uint32_t)((base + ((int64_t)k << s)) * 4), 0u);
#pragma unroll
    for (int h = 1; h < L; h <<= 1)
#pragma unroll
        for (int k = 0; k < L; ++k)
            if ((k & h) == 0)
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const float a = v[k][m], b = v[k | h][m];
                    v[k][m] = a + b;
                    v[k | h][m] = a - b;
                }
    if constexpr (!EPI) {
#pragma unroll
        for (int k = 0; k < L; ++k)
            bstore4(rd, (uint32_t)((base + ((int64_t)k << s)) * 4), v[k][0], v[k][1], v[k][2], v[k][3]);
    } else {
        constexpr uint32_t YB = elem_bytes<YT>();
        const int64_t nE = n * E;
        char* prow = static_cast<char*>(phi) + r * 2 * nE * YB;
        const rsrc_t rp = make_rsrc(prow, (uint32_t)(2 * nE * YB));
        const rsrc_t rh = make_rsrc(Sh, (uint32_t)(n * 4));
#pragma unroll
        for (int k = 0; k < L; ++k) {
            const int64_t i = base + ((int64_t)k << s);
            float sh[4], c4[4], s4[4];
            bload4(sh, rh, (uint32_t)(i * 4), 0u);
#pragma unroll
            for (int m = 0; m < 4; ++m)
                cossin_rev(v[k][m] * sh[m], cs, c4[m], s4[m]);
            const uint32_t oc = (uint32_t)(((int64_t)e * n + i) * YB);
            bstore_quad<YT>(rp, oc, c4[0], c4[1], c4[2], c4[3]);
            bstore_quad<YT>(rp, oc + (uint32_t)(nE * YB), s4[0], s4[1], s4[2], s4[3]);
        }
    }
}

// The first column pass of an expansion: the same butterflies on
// B o xhat, read from x (rows of d elements of type XT; past d reads zero
// through the range check) and written to out (rows of n floats).  xexp
// (nullable): row r of x is the stored row times 2^xexp[r], applied exactly
// to the widened values.
template <int B, int XT, bool VEC>
__global__ void __launch_bounds__(kColThreads)
    k_cols_x(float* __restrict__ out, const void* __restrict__ x, int d, const float* __restrict__ Bv, int64_t rows,
             int64_t n, int s, int64_t blocks_per_row, const int8_t* __restrict__ xexp)
{
    constexpr int L = 1 << B;
    constexpr uint32_t XB = elem_bytes<XT>();
    const int64_t r = (int64_t)blockIdx.x / blocks_per_row;
    const int64_t q = ((int64_t)blockIdx.x % blocks_per_row) * kColThreads + threadIdx.x;
    const int64_t lo_groups = (int64_t)1 << (s - 2);
    if (r >= rows || q >= (n >> B) / 4)
        return;
    const int64_t hi = q / lo_groups, lo = (q % lo_groups) * 4;
    const int64_t base = hi * ((int64_t)L << s) + lo;
    const rsrc_t rx = make_rsrc(static_cast<const char*>(x) + r * d * XB, (uint32_t)d * XB);
    const rsrc_t rb = make_rsrc(Bv, (uint32_t)(n * 4));
    const rsrc_t ro = make_rsrc(out + r * n, (uint32_t)(n * 4));
    const float xs = xexp != nullptr ? __builtin_ldexpf(1.f, (int)xexp[r]) : 1.f;
    float v[L][4];
#pragma unroll
    for (int k = 0; k < L; ++k) {
        const uint32_t i = (uint32_t)(base + ((int64_t)k << s));
        float bq[4];
        bload4(bq, rb, 4u * i, 0u);
#pragma unroll
        for (int m = 0; m < 4; ++m)
            bq[m] *= xs;
        if constexpr (VEC && XT == kF32) {
            bload4<2>(v[k], rx, 4u * i, 0u);
        } else if constexpr (VEC) {
            const u32x2_t h = __builtin_bit_cast(u32x2_t, __builtin_amdgcn_raw_buffer_load_b64(rx, (int)(2u * i), 0, 2));
            unpack2<XT>(h.x, v[k][0], v[k][1]);
            unpack2<XT>(h.y, v[k][2], v[k][3]);
        } else {
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                if constexpr (XT == kF32)
                    v[k][m] = bload1<2>(rx, 4u * (i + m), 0u);
                else
                    v[k][m] = widen1<XT>((uint32_t)__builtin_amdgcn_raw_buffer_load_b16(rx, (int)(2u * (i + m)), 0, 2));
            }
        }
#pragma unroll
        for (int m = 0; m < 4; ++m)
            v[k][m] *= bq[m];
    }
#pragma unroll
    for (int h = 1; h < L; h <<= 1)
#pragma unroll
        for (int k = 0; k < L; ++k)
            if ((k & h) == 0)
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const float a = v[k][m], b = v[k | h][m];
                    v[k][m] = a + b;
                    v[k | h][m] = a - b;
                }
#pragma unroll
    for (int k = 0; k < L; ++k)
        bstore4(ro, (uint32_t)((base + ((int64_t)k << s)) * 4), v[k][0], v[k][1], v[k][2], v[k][3]);
}

template <int XT, bool VEC>
hipError_t col_pass_x(int B, float* out, const void* x, int d, const float* Bv, int64_t rows, int64_t n, int s,
                      const int8_t* xexp, hipStream_t st)
{
    const int64_t groups = (n >> B) / 4;
    const int64_t bpr = (groups + kColThreads - 1) / kColThreads;
    const dim3 grid((unsigned)(rows * bpr)), blk(kColThreads);
#define MCK_COLX_ARGS out, x, d, Bv, rows, n, s, bpr, xexp
    switch (B) {
    case 1: k_cols_x<1, XT, VEC><<<grid, blk, 0, st>>>(MCK_COLX_ARGS); break;
    case 2: k_cols_x<2, XT, VEC><<<grid, blk, 0, st>>>(MCK_COLX_ARGS); break;
    case 3: k_cols_x<3, XT, VEC><<<grid, blk, 0, st>>>(MCK_COLX_ARGS); break;
    case 4: k_cols_x<4, XT, VEC><<<grid, blk, 0, st>>>(MCK_COLX_ARGS); break;
    case 5: k_cols_x<5, XT, VEC><<<grid, blk, 0, st>>>(MCK_COLX_ARGS); break;
    default: return hipErrorInvalidValue;
    }
#undef MCK_COLX_ARGS
    return hipGetLastError();
}

template <bool EPI, int YT>
hipError_t col_pass(int B, float* data, int64_t rows, int64_t n, int s, const float* Sh, float cs, int e, int E,
                    void* phi, hipStream_t st)
{
    const int64_t groups = (n >> B) / 4;
    const int64_t bpr = (groups + kColThreads - 1) / kColThreads;
    const dim3 grid((unsigned)(rows * bpr)), blk(kColThreads);
#define MCK_COL_ARGS data, rows, n, s, bpr, Sh, cs, e, E, phi
    switch (B) {
    case 1: k_cols<1, EPI, YT><<<grid, blk, 0, st>>>(MCK_COL_ARGS); break;
    case 2: k_cols<2, EPI, YT><<<grid, blk, 0, st>>>(MCK_COL_ARGS); break;
    case 3: k_cols<3, EPI, YT><<<grid, blk, 0, st>>>(MCK_COL_ARGS); break;
    case 4: k_cols<4, EPI, YT><<<grid, blk, 0, st>>>(MCK_COL_ARGS); break;
    case 5: k_cols<5, EPI, YT><<<grid, blk, 0, st>>>(MCK_COL_ARGS); break;
    default: return hipErrorInvalidValue;
    }
#undef MCK_COL_ARGS
    return hipGetLastError();
}

// Column passes over bits [15, M): the first takes the bits beyond a
// multiple of 5, each later one 5 bits.  With x the first pass reads B o
// xhat from x; with epi the last one carries the feature epilogue.
template <int XT, bool VEC, int YT>
hipError_t col_passes(int M, float* data, int64_t rows, const void* x, int d, const float* Bv, bool epi,
                      const float* Sh, float cs, int e, int E, void* phi, hipStream_t st,
                      const int8_t* xexp = nullptr)
{
    const int64_t n = int64_t(1) << M;
    int s = kRowM;
    int rem = M - kRowM;
    bool first = true;
    while (rem > 0) {
        const int B = rem % kColMaxB == 0 ? kColMaxB : rem % kColMaxB;
        const bool last = rem == B;
        hipError_t err;
        if (first && x != nullptr)
            err = col_pass_x<XT, VEC>(B, data, x, d, Bv, rows, n, s, xexp, st);
        else if (epi && last)
            err = col_pass<true, YT>(B, data, rows, n, s, Sh, cs, e, E, phi, st);
        else
            err = col_pass<false, kF32>(B, data, rows, n, s, nullptr, 0.f, 0, 0, nullptr, st);
        if (err != hipSuccess)
            return err;
        first = false;
        s += B;
        rem -= B;
    }
    return hipSuccess;
}

// Rows per row-pass block: as many as keep at least 512 blocks (two per CU).
template <int IN, int OUT>
hipError_t row_pass(bool vec, const RowArgs& a, hipStream_t st)
{
    const int rb = a.rows * a.chunks >= 2048 ? 4 : (a.rows * a.chunks >= 1024 ? 2 : 1);
    const int64_t slots = (a.rows + rb - 1) / rb;
    const int64_t blocks = ((slots + kXcds - 1) / kXcds) * kXcds * a.chunks;
    const dim3 grid((unsigned)blocks), blk(RG::BLOCK);
#define MCK_ROWS(RBV)                                                                                              \
    do {                                                                                                          \
        if constexpr (IN != kInRow || OUT != kOutRow)                                                             \
            k_rows<IN, OUT, true, RBV><<<grid, blk, 0, st>>>(a); /* exchange buffers are aligned */               \
        else if (vec)                                                                                             \
            k_rows<IN, OUT, true, RBV><<<grid, blk, 0, st>>>(a);                                                  \
        else                                                                                                      \
            k_rows<IN, OUT, false, RBV><<<grid, blk, 0, st>>>(a);                                                 \
    } while (0)
    if (rb == 4)
        MCK_ROWS(4);
    else if (rb == 2)
        MCK_ROWS(2);
    else
        MCK_ROWS(1);
#undef MCK_ROWS
    return hipGetLastError();
}

template <int XT, int YT>
hipError_t forward_long(int M, bool vec, const void* x, int64_t batch, int d, int64_t E, const float* B,
                        const uint32_t* packA, const uint16_t* dstB, const int32_t* pdelta, const float* Gx,
                        const float* Sh, float cs, void* phi, float* u, float* w, hipStream_t st,
                        const int8_t* xexp)
{
    const int64_t n = int64_t(1) << M, C = n >> kRowM;
    for (int64_t e = 0; e < E; ++e) {
        hipError_t err = vec ? col_passes<XT, true, kF32>(M, u, batch, x, d, B + e * n, false, nullptr, 0.f, 0, 0,
                                                          nullptr, st, xexp)
                             : col_passes<XT, false, kF32>(M, u, batch, x, d, B + e * n, false, nullptr, 0.f, 0, 0,
                                                           nullptr, st, xexp);
        const RowArgs a{w, u, batch, C, nullptr, packA + e * n, pdelta + e * C * C, nullptr};
        if (err == hipSuccess)
            err = row_pass<kInRow, kOutBucket>(true, a, st);
        const RowArgs b{u, w, batch, C, Gx + e * n, nullptr, nullptr, dstB + e * n};
        if (err == hipSuccess)
            err = row_pass<kInBucket, kOutRow>(true, b, st);
        if (err == hipSuccess)
            err = col_passes<kF32, true, YT>(M, u, batch, nullptr, 0, nullptr, true, Sh + e * n, cs, (int)e,
                                             (int)E, phi, st);
        if (err != hipSuccess)
            return err;
    }
    return hipSuccess;
}

// Exchange construction (once per plan).  counts[e][ci][co]: elements that
// destination chunk co takes from source chunk ci.
__global__ void __launch_bounds__(1024)
    k_bucket_count(const int32_t* __restrict__ perm, int64_t n, int C, int32_t* __restrict__ counts)
{
    __shared__ int32_t h[kMaxChunks];
    const int64_t e = blockIdx.x / C;
    const int co = (int)(blockIdx.x % C);
    for (int i = threadIdx.x; i < C; i += blockDim.x)
        h[i] = 0;
    __syncthreads();
    const int32_t* pc = perm + e * n + (int64_t)co * RG::n;
    for (int j = threadIdx.x; j < RG::n; j += blockDim.x)
        atomicAdd(&h[(pc[j] & (int32_t)(n - 1)) >> kRowM], 1);
    __syncthreads();
    for (int ci = threadIdx.x; ci < C; ci += blockDim.x)
        counts[(e * C + ci) * C + co] = h[ci];
}

// seg[e][ci][co]: start of group (ci, co) among the elements leaving source
// chunk ci (one thread per (e, ci)).
__global__ void k_bucket_seg(const int32_t* __restrict__ counts, int64_t E, int C, int32_t* __restrict__ seg)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // e C + ci
    if (g >= E * C)
        return;
    int32_t acc = 0;
    for (int co = 0; co < C; ++co) {
        seg[g * C + co] = acc;
        acc += counts[g * C + co];
    }
}

// pre[e][co][ci]: start of group (ci, co) among the elements destination
// chunk co receives; pdelta from seg and pre (one thread per (e, co)).
__global__ void k_bucket_pre(const int32_t* __restrict__ counts, const int32_t* __restrict__ seg, int64_t E, int C,
                             int32_t* __restrict__ pre, int32_t* __restrict__ pdelta)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // e C + co
    if (g >= E * C)
        return;
    const int64_t e = g / C;
    const int co = (int)(g % C);
    int32_t acc = 0;
    for (int ci = 0; ci < C; ++ci) {
        const int64_t src = e * C + ci;
        pre[g * C + ci] = acc;
        pdelta[src * C + co] = co * RG::n + acc - seg[src * C + co];
        acc += counts[src * C + co];
    }
}

// packA / dstB: thread ci of block (e, co) walks destination chunk co in
// order and appends the elements whose source is in chunk ci to group
// (ci, co) on both sides.
__global__ void __launch_bounds__(512)
    k_bucket_fill(const int32_t* __restrict__ perm, int64_t n, int C, const int32_t* __restrict__ seg,
                  const int32_t* __restrict__ pre, uint32_t* __restrict__ packA, uint16_t* __restrict__ dstB)
{
    constexpr int TILE = 1024;
    __shared__ int32_t tile[TILE];
    const int64_t e = blockIdx.x / C;
    const int co = (int)(blockIdx.x % C);
    const int ci = threadIdx.x;
    const int32_t* pc = perm + e * n + (int64_t)co * RG::n;
    int64_t qa = 0, pb = 0;
    uint32_t q = 0;  // exchange position within source chunk ci
    if (ci < C) {
        qa = e * n + (int64_t)ci * RG::n;
        q = (uint32_t)seg[(e * C + ci) * C + co];
        pb = e * n + (int64_t)co * RG::n + pre[(e * C + co) * C + ci];
    }
    for (int base = 0; base < RG::n; base += TILE) {
        __syncthreads();
        for (int j = threadIdx.x; j < TILE; j += blockDim.x)
            tile[j] = pc[base + j] & (int32_t)(n - 1);
        __syncthreads();
        if (ci < C) {
            for (int j = 0; j < TILE; ++j) {
                const int32_t src = tile[j];
                if ((src >> kRowM) == ci) {
                    packA[qa + pack_slot(q++)] = ((uint32_t)co << kRowM) | (uint32_t)(src & (RG::n - 1));
                    dstB[pb++] = (uint16_t)(base + j);
                }
            }
        }
    }
}

// Gx[e][co 2^15 + p] = G[e][co 2^15 + dstB[e][co 2^15 + p]]: G in the
// order the receiving row pass reads the exchange buffer.
__global__ void k_bucket_gx(const float* __restrict__ G, const uint16_t* __restrict__ dstB, int64_t count,
                            float* __restrict__ Gx)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count)
        Gx[i] = G[(i & ~(int64_t)(RG::n - 1)) + dstB[i]];
}

}  // namespace

hipError_t launch_sh(const double* S64, float* Sh, int64_t count, hipStream_t s)
{
    k_sh<<<dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s>>>(S64, Sh, count);
    return hipGetLastError();
}

hipError_t launch_fwht_long(int M, float* data, int64_t batch, bool vec, hipStream_t s)
{
    if (M <= kRowM || M > 24)
        return hipErrorInvalidValue;
    const int64_t n = int64_t(1) << M;
    const RowArgs a{data, data, batch, n >> kRowM, nullptr, nullptr, nullptr, nullptr};
    hipError_t err = row_pass<kInRow, kOutRow>(vec, a, s);
    if (err != hipSuccess)
        return err;
    return col_passes<kF32, true, kF32>(M, data, batch, nullptr, 0, nullptr, false, nullptr, 0.f, 0, 0, nullptr, s);
}

hipError_t launch_forward_long(int M, bool vec, int xt, int yt, const void* x, int64_t batch, int d, int64_t E,
                               const float* B, const uint32_t* packA, const uint16_t* dstB, const int32_t* pdelta,
                               const float* Gx, const float* Sh, float cs, void* phi, float* u, float* w,
                               hipStream_t s, const int8_t* xexp)
{
    if (M <= kRowM || M > 24)
        return hipErrorInvalidValue;
#define MCK_FL_ARGS M, vec, x, batch, d, E, B, packA, dstB, pdelta, Gx, Sh, cs, phi, u, w, s, xexp
    if (xt == kF32 && yt == kF32)
        return forward_long<kF32, kF32>(MCK_FL_ARGS);
    if (xt == kF32 && yt == kBF16)
        return forward_long<kF32, kBF16>(MCK_FL_ARGS);
    if (xt == kF32 && yt == kF16)
        return forward_long<kF32, kF16>(MCK_FL_ARGS);
    if (xt == kBF16 && yt == kBF16)
        return forward_long<kBF16, kBF16>(MCK_FL_ARGS);
    if (xt == kF16 && yt == kF16)
        return forward_long<kF16, kF16>(MCK_FL_ARGS);
#undef MCK_FL_ARGS
    return hipErrorInvalidValue;
}

hipError_t launch_pair_plan(int64_t E, const int32_t* perm, const float* G, const float* B, uint32_t* Bw,
                            uint32_t* Pw, uint32_t* Po, float* Pg, hipStream_t s)
{
    // the inverse and the links are built in Pg's space, the colours in
    // Bw's; both are overwritten last
    uint16_t* inv = reinterpret_cast<uint16_t*>(Pg);
    uint16_t* link = inv + E * kPairN;
    uint32_t* colour = Bw;
    const unsigned eb = (unsigned)((E * kPairN + 255) / 256);
    k_pair_inverse<<<dim3(eb), dim3(256), 0, s>>>(perm, E, inv);
    k_pair_link<<<dim3(eb), dim3(256), 0, s>>>(perm, inv, E, link);
    k_pair_colour<<<dim3((unsigned)E), dim3(256), 0, s>>>(link, E, colour);
    k_pair_plan<<<dim3((unsigned)((E * RG::BLOCK + 255) / 256)), dim3(256), 0, s>>>(perm, G, colour, E, Pw, Po, Pg);
    const int64_t total = E * 2 * RG::BLOCK;
    k_pair_signs<<<dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s>>>(B, E, Bw);
    return hipGetLastError();
}

int64_t pair_blocks(int64_t rows, int64_t E, int cus)
{
    // one block per CU (the LDS holds one), all XCDs equally; never more
    // slots per XCD than that XCD has work items
    int64_t per_xcd = cus / kXcds;
    per_xcd = per_xcd < 1 ? 1 : per_xcd;
    const int64_t items = (rows + kXcds - 1) / kXcds * E;
    if (items < per_xcd)
        per_xcd = items < 1 ? 1 : items;
    return per_xcd * kXcds;
}

hipError_t launch_forward_pair(bool vec, int xt, int yt, const void* x, int64_t batch, int d, int64_t E,
                               const uint32_t* Bw, const uint32_t* Pw, const uint32_t* Po, const float* Pg,
                               const float* Sh, float cs, void* phi, int64_t blocks, hipStream_t s,
                               const int8_t* xexp)
{
    if (blocks % kXcds != 0 || blocks < kXcds)
        return hipErrorInvalidValue;
    const PairArgs a{x, batch, d, (int)E, Bw, Pw, Po, Pg, Sh, cs, phi, xexp, (int)(blocks / kXcds)};
    const dim3 grid((unsigned)blocks), blk(RG::BLOCK);
#define MCK_PAIR(XT_, YT_)                                                                                      \
    do {                                                                                                       \
        if (vec)                                                                                               \
            k_forward_pair<XT_, YT_, true><<<grid, blk, 0, s>>>(a);                                            \
        else                                                                                                   \
            k_forward_pair<XT_, YT_, false><<<grid, blk, 0, s>>>(a);                                           \
        return hipGetLastError();                                                                              \
    } while (0)
    if (xt == kF32 && yt == kF32)
        MCK_PAIR(kF32, kF32);
    if (xt == kF32 && yt == kBF16)
        MCK_PAIR(kF32, kBF16);
    if (xt == kF32 && yt == kF16)
        MCK_PAIR(kF32, kF16);
    if (xt == kBF16 && yt == kBF16)
        MCK_PAIR(kBF16, kBF16);
    if (xt == kF16 && yt == kF16)
        MCK_PAIR(kF16, kF16);
#undef MCK_PAIR
    return hipErrorInvalidValue;
}

hipError_t launch_buckets(int M, int64_t E, const int32_t* perm, const float* G, uint32_t* packA, uint16_t* dstB,
                          int32_t* pdelta, float* Gx, int32_t* scratch, hipStream_t s)
{
    if (M <= kRowM || M > 24)
        return hipErrorInvalidValue;
    const int64_t n = int64_t(1) << M;
    const int C = (int)(n >> kRowM);
    int32_t* counts = scratch;
    int32_t* seg = counts + E * C * C;
    int32_t* pre = seg + E * C * C;
    const unsigned blocks = (unsigned)(E * C);
    k_bucket_count<<<dim3(blocks), dim3(1024), 0, s>>>(perm, n, C, counts);
    const unsigned tb = (unsigned)((E * C + 255) / 256);
    k_bucket_seg<<<dim3(tb), dim3(256), 0, s>>>(counts, E, C, seg);
    k_bucket_pre<<<dim3(tb), dim3(256), 0, s>>>(counts, seg, E, C, pre, pdelta);
    const int threads = C < 64 ? 64 : C;
    k_bucket_fill<<<dim3(blocks), dim3((unsigned)threads), 0, s>>>(perm, n, C, seg, pre, packA, dstB);
    k_bucket_gx<<<dim3((unsigned)((n * E + 255) / 256)), dim3(256), 0, s>>>(G, dstB, n * E, Gx);
    return hipGetLastError();
}

}  // namespace mck
