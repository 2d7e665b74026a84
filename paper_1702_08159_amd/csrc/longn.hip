// longn.hip -- the transform and the feature map for n > 2^15 (up to 2^24),
// where one row no longer fits in a workgroup's LDS.
//
// H_n = H_{n/2^15} (x) H_{2^15} (Sylvester's H is the tensor product of one
// 2x2 butterfly per index bit, section "Fast Walsh Hadamard"), so the
// transform splits into
//   a row pass:    H_{2^15} on each contiguous chunk of 2^15 elements
//                  (the register/LDS engine, one chunk per 1024-lane block);
//   column passes: H over the remaining high index bits, at most 5 per pass:
//                  each lane holds the 2^B elements of four adjacent columns
//                  (stride 2^s) in VGPRs, so consecutive lanes read
//                  consecutive 16-byte pieces.
// The feature map per expansion is then four passes over an FP32 scratch
// copy of the batch:
//   1. row pass with input B o xhat (x read in place, zero padding by range);
//   2. column pass(es)                           -> u = H B xhat
//   3. row pass with input G_i u[perm[i]]        (gather from L2 / MALL)
//   4. column pass(es); the last one multiplies by S / (2 pi) and writes
//      c cos, c sin in the storage type of phi.
// Row-pass blocks are mapped so that an XCD works on one row at a time,
// which keeps that row's u (4 MB at n = 2^20) in its L2 for the gather.
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

using RG = Geo<kRowM, kRowP>;

// Row pass input modes.
enum : int { kInPlace = 0, kInX = 1, kInGather = 2 };

// XCD-aware (row, chunk) of a row-pass block: blocks are dealt to the 8 XCDs
// round robin; XCD x takes rows x, x + 8, ... one after another, all chunks
// of a row together.
__device__ __forceinline__ void row_chunk(int64_t rows, int64_t chunks, int64_t& r, int64_t& c)
{
    const int64_t b = blockIdx.x;
    const int64_t xcd = b % kXcds, q = b / kXcds;
    r = (q / chunks) * kXcds + xcd;
    c = q % chunks;
}

// One 2^15 chunk per block: load (mode), H_{2^15}, store to dst (FP32,
// natural order).  dst rows have length n = chunks * 2^15.
template <int MODE, bool VEC, int XT>
__global__ void __launch_bounds__(RG::BLOCK)
    k_rows(float* __restrict__ dst, const float* src, int64_t rows, int64_t chunks, const void* __restrict__ x,
           int d, const float* __restrict__ Bv, const int32_t* __restrict__ perm, const float* __restrict__ Gv)
{
    constexpr int M = kRowM, P = kRowP, EPL = RG::EPL, K = RG::K;
    constexpr int64_t CH = RG::n;
    __shared__ float lds[RG::LDS_FLOATS];
    int64_t r, c;
    row_chunk(rows, chunks, r, c);
    if (r >= rows)
        return;  // uniform per block
    const int64_t n = chunks * CH;
    const uint32_t t = threadIdx.x;
    const uint32_t tb = tpart<M, P, 0>(t);
    float* out = dst + r * n + c * CH;
    const rsrc_t ro = make_rsrc(out, (uint32_t)(CH * 4));
    float v[EPL];
    if constexpr (MODE == kInPlace) {
        bload_row<M, P, VEC>(v, ro, 0u, (int)CH, t, true);
    } else if constexpr (MODE == kInX) {
        // xhat o B: the chunk's part of row r of x (elements past d read 0)
        constexpr uint32_t XB = elem_bytes<XT>();
        const int64_t left = (int64_t)d - c * CH;
        const int dl = left <= 0 ? 0 : (left >= CH ? (int)CH : (int)left);
        const char* xb = static_cast<const char*>(x) + (r * d + (dl > 0 ? c * CH : 0)) * XB;
        const rsrc_t rx = make_rsrc(xb, (uint32_t)dl * XB);
        bload_row_t<M, P, VEC, XT>(v, rx, 0u, dl, t, dl > 0);
        float bq[EPL];
        bload_coal<M, P>(bq, make_rsrc(Bv + c * CH, (uint32_t)(CH * 4)), 0u, t);
#pragma unroll
        for (int k = 0; k < EPL; ++k)
            v[k] *= bq[k];
    } else {
        // G_i src[perm[i]] for the chunk's i (gather within row r of src)
        const rsrc_t rs = make_rsrc(src + r * n, (uint32_t)(n * 4));
        const rsrc_t rp = make_rsrc(perm + c * CH, (uint32_t)(CH * 4));
        const rsrc_t rg = make_rsrc(Gv + c * CH, (uint32_t)(CH * 4));
        float gq[EPL];
        uint32_t pq[EPL];
        bload_coal<M, P>(gq, rg, 0u, t);
#pragma unroll
        for (int j = 0; j < EPL / 4; ++j)
            bload4u(&pq[4 * j], rp, 4u * tb, 4u * rpart(M, P, 0, 4 * j));
#pragma unroll
        for (int k = 0; k < EPL; ++k)
            v[k] = gq[k] * bload1(rs, 4u * (pq[k] & (uint32_t)(n - 1)), 0u);
    }
    fwht_up<M, P>(v, lds, t);
    relayout<M, P, K, 0>(v, lds, t);
    if constexpr (VEC || MODE != kInPlace) {
#pragma unroll
        for (int j = 0; j < EPL / 4; ++j)
            bstore4(ro, 4u * (tb | rpart(M, P, 0, 4 * j)), v[4 * j], v[4 * j + 1], v[4 * j + 2], v[4 * j + 3]);
    } else {
#pragma unroll
        for (int k = 0; k < EPL; ++k)
            bstore1(ro, 4u * tb, 4u * rpart(M, P, 0, k), v[k]);
    }
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
// multiple of 5, each later one 5 bits; the last may carry the epilogue.
template <int YT>
hipError_t col_passes(int M, float* data, int64_t rows, bool epi, const float* Sh, float cs, int e, int E,
                      void* phi, hipStream_t st)
{
    const int64_t n = int64_t(1) << M;
    int s = kRowM;
    int rem = M - kRowM;
    while (rem > 0) {
        const int B = rem % kColMaxB == 0 ? kColMaxB : rem % kColMaxB;
        const bool last = rem == B;
        hipError_t err = (epi && last) ? col_pass<true, YT>(B, data, rows, n, s, Sh, cs, e, E, phi, st)
                                       : col_pass<false, kF32>(B, data, rows, n, s, nullptr, 0.f, 0, 0, nullptr, st);
        if (err != hipSuccess)
            return err;
        s += B;
        rem -= B;
    }
    return hipSuccess;
}

template <int MODE, int XT>
hipError_t row_pass(bool vec, float* dst, const float* src, int64_t rows, int64_t chunks, const void* x, int d,
                    const float* Bv, const int32_t* perm, const float* Gv, hipStream_t st)
{
    const int64_t blocks = ((rows + kXcds - 1) / kXcds) * kXcds * chunks;
    const dim3 grid((unsigned)blocks), blk(RG::BLOCK);
    if (vec)
        k_rows<MODE, true, XT><<<grid, blk, 0, st>>>(dst, src, rows, chunks, x, d, Bv, perm, Gv);
    else
        k_rows<MODE, false, XT><<<grid, blk, 0, st>>>(dst, src, rows, chunks, x, d, Bv, perm, Gv);
    return hipGetLastError();
}

template <int XT, int YT>
hipError_t forward_long(int M, bool vec, const void* x, int64_t batch, int d, int64_t E, const float* B,
                        const int32_t* perm, const float* G, const float* Sh, float cs, void* phi, float* u,
                        float* w, hipStream_t st)
{
    const int64_t n = int64_t(1) << M, chunks = n >> kRowM;
    for (int64_t e = 0; e < E; ++e) {
        hipError_t err = row_pass<kInX, XT>(vec, u, nullptr, batch, chunks, x, d, B + e * n, nullptr, nullptr, st);
        if (err == hipSuccess)
            err = col_passes<kF32>(M, u, batch, false, nullptr, 0.f, 0, 0, nullptr, st);
        if (err == hipSuccess)
            err = row_pass<kInGather, kF32>(true, w, u, batch, chunks, nullptr, 0, nullptr, perm + e * n,
                                             G + e * n, st);
        if (err == hipSuccess)
            err = col_passes<YT>(M, w, batch, true, Sh + e * n, cs, (int)e, (int)E, phi, st);
        if (err != hipSuccess)
            return err;
    }
    return hipSuccess;
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
    const int64_t n = int64_t(1) << M, chunks = n >> kRowM;
    hipError_t err = row_pass<kInPlace, kF32>(vec, data, nullptr, batch, chunks, nullptr, 0, nullptr, nullptr,
                                              nullptr, s);
    if (err != hipSuccess)
        return err;
    return col_passes<kF32>(M, data, batch, false, nullptr, 0.f, 0, 0, nullptr, s);
}

hipError_t launch_forward_long(int M, bool vec, int xt, int yt, const void* x, int64_t batch, int d, int64_t E,
                               const float* B, const int32_t* perm, const float* G, const float* Sh, float cs,
                               void* phi, float* u, float* w, hipStream_t s)
{
    if (M <= kRowM || M > 24)
        return hipErrorInvalidValue;
#define MCK_FL_ARGS M, vec, x, batch, d, E, B, perm, G, Sh, cs, phi, u, w, s
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

}  // namespace mck
