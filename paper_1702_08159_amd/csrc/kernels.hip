// kernels.hip -- the Fastfood hot path on gfx950.
//
//   k_fwht      in-place batched H v (section "Fast Walsh Hadamard")
//   k_forward   phi = c [cos z, sin z], z = S H G Pi H B xhat for every
//               expansion (equations mckernel and mcfeatures), fused: one HBM
//               read of x per row and expansion chunk, one HBM write of phi,
//               everything else in registers and LDS
//   k_backward  adjoint of the same chain (H is symmetric, Pi^T a scatter),
//               recomputing the forward instead of storing it
//   k_reduce    fixed-order sum of the backward's per-block partials
//   k_derive    parameter copies in the kernels' register layouts
//
// Vectors are spread over lanes as described in layout.hpp; each lane keeps
// 2^P elements in VGPRs, butterflies on register bits are lane-local, and a
// transform costs P add/sub per element per layout plus one LDS round trip
// per change of layout.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "engine.hpp"
#include "forward.hpp"
#include "launch.hpp"

namespace mck {
namespace {

// ------------------------------------------------------------------ H v
template <int M, bool VEC>
__global__ void __launch_bounds__((Geo<M, kFwhtP>::BLOCK))
    k_fwht(float* __restrict__ data, uint32_t bytes, int64_t batch)
{
    constexpr int P = kFwhtP;
    using g = Geo<M, P>;
    constexpr int K = g::K, EPL = g::EPL;
    __shared__ float lds[g::LDS_FLOATS];
    const uint32_t lane = threadIdx.x;
    const uint32_t grp = g::kMulti ? 0u : lane >> g::T;
    const uint32_t t = g::kMulti ? lane : (lane & (g::LPR - 1));
    const int64_t row = (int64_t)blockIdx.x * g::RPB + grp;
    const bool valid = row < batch;
    float* buf = lds + grp * g::STRIDE;
    const rsrc_t r = make_rsrc(data, bytes);
    const uint32_t rowoff = valid ? (uint32_t)(row * g::n) * 4u : kOutOfRange;
    float v[EPL];
    bload_row<M, P, VEC>(v, r, rowoff, g::n, t, valid);
    fwht_up<M, P>(v, buf, t);
    if constexpr (K >= 1)
        relayout<M, P, g::GL, 0>(v, buf, t);
    const uint32_t tb4 = 4u * tpart<M, P, 0>(t);
    if constexpr (VEC) {
#pragma unroll
        for (int j = 0; j < EPL / 4; ++j)
            bstore4(r, rowoff + tb4 + 4u * rpart(M, P, 0, 4 * j), v[4 * j], v[4 * j + 1], v[4 * j + 2],
                    v[4 * j + 3]);
    } else {
#pragma unroll
        for (int k = 0; k < EPL; ++k)
            bstore1(r, rowoff + tb4, 4u * rpart(M, P, 0, k), v[k]);
    }
}

// ------------------------------------------------------------------ backward
// Block = NW waves, one row per wave and pass (or one multi-wave row for
// large n).  Expansions are the outer loop so that the dS, dG, dB
// contributions of all rows a block owns accumulate in VGPRs; at the end of
// each expansion they are summed across the block in a fixed order and
// written as the block's partial.  dx accumulates over expansions in place
// (every row has one owner, so the read-modify-write is ordered).
constexpr int kBwdWaves = 8;

template <int M>
struct BwdGeo {
    static constexpr int P = bwd_p(M);
    using g = Geo<M, P>;
    static constexpr int NW = g::kMulti ? 1 : kBwdWaves;
    static constexpr int THREADS = g::BLOCK * NW;
    static constexpr int ROWS = NW * g::RPB;  // rows per block per pass
    // Rows of one wave or less: the block's dx rows stay in LDS (dynamic
    // shared memory, rows x d) across the expansion loop and are written
    // once.  Longer rows read-modify-write dx in HBM per expansion.
    static constexpr bool XRES = !g::kMulti;
    static constexpr int STATIC_LDS = (NW * g::LDS_FLOATS + 3) / 4 * 16;
    static constexpr int PARAM_LDS = XRES ? (4 * g::n + g::RPB * g::n) * 4 : 0;
};

constexpr int kLdsBytes = 160 * 1024;

// Sum of the three per-lane accumulators (dS and dB in the coalesced
// layout, dG in the gather layout) over the rows of a block, in slot order
// (wave, row group), written as the block's partial dst[3][n].  Uses the
// first NW * RPB * n floats of the transform scratch; all threads of the
// block must call it.
template <int M>
__device__ __forceinline__ void block_partials(float* lds, const LaneArr<float, M, BwdGeo<M>::P>& aS,
                                               const LaneArr<float, M, BwdGeo<M>::P>& aG,
                                               const LaneArr<float, M, BwdGeo<M>::P>& aB, float* dst,
                                               uint32_t wave, uint32_t grp, uint32_t t, float scaleS)
{
    using bg = BwdGeo<M>;
    constexpr int P = bg::P;
    using g = Geo<M, P>;
    constexpr int EPL = g::EPL, n = g::n, K = g::K, SLOTS = bg::NW * g::RPB;
    float* slot = lds + (wave * g::RPB + grp) * n;
    const uint32_t ct = tpart<M, P, 0>(t), tk = tpart<M, P, g::GL>(t);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        __syncthreads();
        if (a == 1) {
#pragma unroll
            for (int r = 0; r < EPL; ++r)
                slot[tk | rpart(M, P, g::GL, r)] = aG[r];
        } else {
            const float* acc = a == 0 ? aS : aB;
#pragma unroll
            for (int r = 0; r < EPL; ++r)
                slot[ct | rpart(M, P, 0, r)] = acc[r];
        }
        __syncthreads();
        for (int i = threadIdx.x; i < n; i += bg::THREADS) {
            float s = 0.f;
            for (int k = 0; k < SLOTS; ++k)
                s += lds[k * n + i];
            dst[(int64_t)a * n + i] = a == 0 ? s * scaleS : s;
        }
    }
    __syncthreads();
}

template <int M, bool VEC, bool PARAMS>
__global__ void __launch_bounds__(BwdGeo<M>::THREADS)
    k_backward(const float* __restrict__ x, uint32_t x_bytes, const float* __restrict__ dphi, uint32_t dphi_bytes,
               int64_t batch, int d, int E, const float* __restrict__ B, const uint32_t* __restrict__ goff,
               const float* __restrict__ Gk, const float* __restrict__ S32, const float* __restrict__ Sh,
               uint32_t par_bytes, uint32_t goff_bytes, float cs, float* __restrict__ dx,
               float* __restrict__ partial, int passes)
{
    using bg = BwdGeo<M>;
    constexpr int P = bg::P;
    using g = Geo<M, P>;
    constexpr int EPL = g::EPL, n = g::n, K = g::K;
    constexpr uint32_t kGoffE = (uint32_t)g::RPB * n;
    __shared__ __align__(16) float lds[bg::STATIC_LDS / 4];
    const uint32_t wave = g::kMulti ? 0u : threadIdx.x / 64u;
    const uint32_t lane = g::kMulti ? threadIdx.x : threadIdx.x % 64u;
    const uint32_t grp = g::kMulti ? 0u : lane >> g::T;
    const uint32_t t = g::kMulti ? lane : (lane & (g::LPR - 1));
    float* wbuf = lds + wave * g::LDS_FLOATS;
    float* buf = wbuf + grp * g::STRIDE;
    char* lbytes = reinterpret_cast<char*>(wbuf);  // gather offsets include the row region
    const uint32_t nE = (uint32_t)n * (uint32_t)E;
    const uint32_t ct = tpart<M, P, 0>(t);

    const rsrc_t rx = make_rsrc(x, x_bytes), rD = make_rsrc(dphi, dphi_bytes), rB = make_rsrc(B, par_bytes);
    const rsrc_t rG = make_rsrc(Gk, par_bytes), rS = make_rsrc(S32, par_bytes), rH = make_rsrc(Sh, par_bytes);
    const rsrc_t rO = make_rsrc(goff, goff_bytes), rX = make_rsrc(dx, x_bytes);

    for (int e = 0; e < E; ++e) {
        const uint32_t eo4 = 4u * (uint32_t)e * n;
        const uint32_t go4 = 4u * (uint32_t)e * kGoffE;
        float aS[EPL], aG[EPL], aB[EPL];
        if constexpr (PARAMS) {
#pragma unroll
            for (int r = 0; r < EPL; ++r)
                aS[r] = aG[r] = aB[r] = 0.f;
        }
        for (int p = 0; p < passes; ++p) {
            const int64_t row = ((int64_t)blockIdx.x * passes + p) * bg::ROWS + wave * g::RPB + grp;
            const bool valid = row < batch;
            const uint32_t xoff = valid ? (uint32_t)(row * d) * 4u : 0u;
            const uint32_t goffr = valid ? (uint32_t)(row * 2 * (int64_t)nE) * 4u : 0u;

            // forward recompute: v1 = H B xhat, w = Pi v1, v3 = H G w
            float v[EPL];
            {
                float xh[EPL];
                bload_row<M, P, VEC>(xh, rx, xoff, d, t, valid);
                bload_coal<M, P>(v, rB, eo4, t);
#pragma unroll
                for (int r = 0; r < EPL; ++r)
                    v[r] *= xh[r];
            }
            uint32_t off[EPL];
            bload_lane<M, P, uint32_t>(off, rO, go4, lane);
            fwht_up<M, P>(v, buf, lds_lane<M, P>(t));
            lds_put<M, P, g::GL>(buf, lds_lane<M, P>(t), v);
            lds_sync<M, P>();
            float w[EPL];
#pragma unroll
            for (int r = 0; r < EPL; ++r)
                w[r] = *reinterpret_cast<const float*>(lbytes + off[r]);
            lds_sync<M, P>();
            {
                float gk[EPL];
                bload_lane<M, P, float>(gk, rG, eo4, t);
#pragma unroll
                for (int r = 0; r < EPL; ++r)
                    v[r] = w[r] * gk[r];
            }
            fwht_down<M, P>(v, buf, lds_lane<M, P>(t));

            // dz = c (-sin z dphi_cos + cos z dphi_sin); dS += dz v3; g3 = S dz
            {
                float gc[EPL], gsn[EPL];
                bload_row<M, P, VEC, 2>(gc, rD, goffr + eo4, n, t, valid);
                bload_row<M, P, VEC, 2>(gsn, rD, goffr + 4u * nE + eo4, n, t, valid);
                float sh[EPL];
                bload_coal<M, P>(sh, rH, eo4, t);
#pragma unroll
                for (int r = 0; r < EPL; ++r) {
                    float co, si;
                    cossin_rev(v[r] * sh[r], cs, co, si);
                    const float dz = co * gsn[r] - si * gc[r];
                    if constexpr (PARAMS)
                        aS[r] += dz * v[r];
                    v[r] = dz;
                }
                float s32[EPL];
                bload_coal<M, P>(s32, rS, eo4, t);
#pragma unroll
                for (int r = 0; r < EPL; ++r)
                    v[r] *= s32[r];
            }
            // g2 = H g3 (ends in the gather layout); dG += g2 w; Pi^T scatter of G g2
            fwht_up<M, P>(v, buf, lds_lane<M, P>(t));
            {
                float gk[EPL];
                bload_lane<M, P, float>(gk, rG, eo4, t);
#pragma unroll
                for (int r = 0; r < EPL; ++r) {
                    if constexpr (PARAMS)
                        aG[r] += v[r] * w[r];
                    v[r] *= gk[r];
                }
            }
#pragma unroll
            for (int r = 0; r < EPL; ++r)
                *reinterpret_cast<float*>(lbytes + off[r]) = v[r];
            lds_sync<M, P>();
            lds_get<M, P, g::GL>(buf, lds_lane<M, P>(t), v);
            lds_sync<M, P>();
            // g0 = H g1 (ends in the coalesced layout); dB += g0 xhat; dx += B g0
            fwht_down<M, P>(v, buf, lds_lane<M, P>(t));
            {
                float xh[EPL], bb[EPL];
                bload_row<M, P, VEC>(xh, rx, xoff, d, t, valid);
                bload_coal<M, P>(bb, rB, eo4, t);
#pragma unroll
                for (int r = 0; r < EPL; ++r) {
                    if constexpr (PARAMS)
                        aB[r] += v[r] * xh[r];
                    v[r] *= bb[r];
                }
            }
            if (dx != nullptr) {
                // padded coordinates and invalid rows map out of range: dropped
                if (e > 0) {
                    float o[EPL];
                    bload_row<M, P, VEC>(o, rX, xoff, d, t, valid);
#pragma unroll
                    for (int r = 0; r < EPL; ++r)
                        v[r] += o[r];
                }
                if constexpr (VEC) {
#pragma unroll
                    for (int j = 0; j < EPL / 4; ++j) {
                        const uint32_t i0 = ct | rpart(M, P, 0, 4 * j);
                        const uint32_t o = (valid && (int)i0 < d) ? xoff + 4u * i0 : kOutOfRange;
                        bstore4(rX, o, v[4 * j], v[4 * j + 1], v[4 * j + 2], v[4 * j + 3]);
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < EPL; ++k) {
                        const uint32_t i = ct | rpart(M, P, 0, k);
                        bstore1(rX, (valid && (int)i < d) ? xoff + 4u * i : kOutOfRange, 0, v[k]);
                    }
                }
            }
        }

        if constexpr (PARAMS)
            block_partials<M>(lds, aS, aG, aB, partial + (((int64_t)blockIdx.x * E + e) * 3) * n, wave, grp, t, 1.f);
    }
}

// Backward for rows of one wave or less (n <= 1024).  A block of NW waves
// owns passes x ROWS consecutive rows for all expansions:
//  - the block's dx rows accumulate in LDS (dynamic shared memory) and are
//    written to HBM once at the end;
//  - at the start of each expansion the block stages that expansion's B,
//    S, S/(2 pi), G and gather offsets in LDS, so the pass loop issues no
//    parameter loads to L2;
//  - dphi of the next (row, expansion) is loaded into spare VGPRs right
//    after the current dphi is consumed, so its HBM latency hides behind
//    the adjoint half of the current one.  (Loads complete in issue order
//    for the vector-memory counter, which is why the only other load in the
//    loop, x of the row, is issued at the top of the next iteration.)
// Rows owned by no block lane (past the batch) read as zero and are never
// written.
template <int M, bool VEC, bool PARAMS>
__global__ void __launch_bounds__(BwdGeo<M>::THREADS)
    k_backward_rows(const float* __restrict__ x, uint32_t x_bytes, const float* __restrict__ dphi,
                    uint32_t dphi_bytes, int64_t batch, int d, int E, const float* __restrict__ B,
                    const uint32_t* __restrict__ goff, const float* __restrict__ Gk, const float* __restrict__ S32,
                    const float* __restrict__ Sh, float cs, float* __restrict__ dx, float* __restrict__ partial,
                    int passes, int esplit, int64_t rowblocks, int64_t dx_group_stride)
{
    using bg = BwdGeo<M>;
    constexpr int P = bg::P;
    using g = Geo<M, P>;
    static_assert(!g::kMulti, "rows of one wave or less");
    // block = (row block rb, expansion group eg): expansions [e0, e1)
    const int64_t rb = (int64_t)blockIdx.x % rowblocks;
    const int eg = (int)((int64_t)blockIdx.x / rowblocks);
    const int e0 = (int)((int64_t)eg * E / esplit), e1 = (int)((int64_t)(eg + 1) * E / esplit);
    constexpr int EPL = g::EPL, n = g::n, K = g::K, NQ = EPL / 4 > 0 ? EPL / 4 : 1;
    constexpr int GOFF_E = g::RPB * n;  // gather offsets per expansion (all row groups of a wave)
    // parameter stage: B, S, S/(2 pi) in natural order; G and the gather
    // offsets float4-major (chunk j of lane t at (j * lanes + t) * 4) so
    // that a wave's float4 reads hit consecutive LDS addresses
    constexpr int PB = 0, PS = n, PH = 2 * n, PG = 3 * n, PO = 4 * n, PRM = 4 * n + GOFF_E;
    __shared__ __align__(16) float lds[bg::STATIC_LDS / 4];
    __shared__ __align__(16) float prm[PRM];
    extern __shared__ float4 dxl4[];  // passes x ROWS rows of d4 floats
    float* dxl = reinterpret_cast<float*>(dxl4);
    const int d4 = (d + 3) & ~3;

    // the wave index is the same for all lanes of a wave: held in a scalar
    // register, so row indices, bounds and row offsets of one-row-per-wave
    // geometries are scalar work
    const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x / 64u));
    const uint32_t lane = threadIdx.x % 64u;
    const uint32_t grp = lane >> g::T;
    const uint32_t t = lane & (g::LPR - 1);
    float* wbuf = lds + wave * g::LDS_FLOATS;
    float* buf = wbuf + grp * g::STRIDE;
    char* lbytes = reinterpret_cast<char*>(wbuf);
    const uint32_t nE = (uint32_t)n * (uint32_t)E;
    const uint32_t ct = tpart<M, P, 0>(t);
    const rsrc_t rx = make_rsrc(x, x_bytes), rD = make_rsrc(dphi, dphi_bytes);
    const int64_t row_base = rb * passes * bg::ROWS + wave * g::RPB + grp;

    // dphi of the next (row, expansion), prefetched
    float cn[EPL], sn[EPL];
    auto prefetch = [&](int e, int p) {
        const int64_t row = row_base + (int64_t)p * bg::ROWS;
        const bool valid = e < e1 && row < batch;
        const uint32_t doff = valid ? (uint32_t)(row * 2 * (int64_t)nE) * 4u + 4u * (uint32_t)e * n : 0u;
        if constexpr (g::RPB == 1 && VEC && EPL >= 4) {
            // one row per wave: the row is uniform, and its offset goes to the
            // loads' scalar offset beside the lane's fixed part.  A row past
            // the batch reads the last row's dphi instead of zeros: its xhat is
            // zero, so its v3, w and g-products with xhat are zero and it adds
            // nothing to dS, dG, dB for finite dphi (and its dx is not written)
            const int64_t rowc = row < batch ? row : batch - 1;
            const uint32_t dcl = e < e1 ? (uint32_t)(rowc * 2 * (int64_t)nE) * 4u + 4u * (uint32_t)e * n : 0u;
#pragma unroll
            for (int j = 0; j < EPL / 4; ++j) {
                const uint32_t lo = 4u * (ct | rpart(M, P, 0, 4 * j));
                bload4<2>(&cn[4 * j], rD, lo, dcl);
                bload4<2>(&sn[4 * j], rD, lo, dcl + 4u * nE);
            }
        } else {
            bload_row<M, P, VEC, 2>(cn, rD, doff, n, t, valid);
            bload_row<M, P, VEC, 2>(sn, rD, doff + 4u * nE, n, t, valid);
        }
    };
    prefetch(e0, 0);

    auto ld_nat = [&](float (&v)[EPL], int base) {  // natural-order parameter, coalesced layout
        const float* b0 = prm + base + ct;
        if constexpr (M >= 2) {
#pragma unroll
            for (int j = 0; j < EPL / 4; ++j) {
                const float4 q = *reinterpret_cast<const float4*>(b0 + rpart(M, P, 0, 4 * j));
                v[4 * j] = q.x;
                v[4 * j + 1] = q.y;
                v[4 * j + 2] = q.z;
                v[4 * j + 3] = q.w;
            }
        } else {
#pragma unroll
            for (int k = 0; k < EPL; ++k)
                v[k] = b0[rpart(M, P, 0, k)];
        }
    };
    auto ld_lane = [&](float (&v)[EPL], int base, uint32_t q, uint32_t lanes) {  // float4-major, lane q
        if constexpr (EPL >= 4) {
#pragma unroll
            for (int j = 0; j < NQ; ++j) {
                const float4 f = *reinterpret_cast<const float4*>(prm + base + (j * lanes + q) * 4);
                v[4 * j] = f.x;
                v[4 * j + 1] = f.y;
                v[4 * j + 2] = f.z;
                v[4 * j + 3] = f.w;
            }
        } else {
#pragma unroll
            for (int k = 0; k < EPL; ++k)
                v[k] = prm[base + q * EPL + k];
        }
    };

    // the parameter stage of an expansion goes through registers: its loads
    // are issued before the previous expansion's partial sums, which hide
    // their latency, and written to LDS once every wave is done with that
    // expansion
    constexpr int NSP = (n + bg::THREADS - 1) / bg::THREADS, NSO = (GOFF_E + bg::THREADS - 1) / bg::THREADS;
    float sB[NSP], sS[NSP], sH[NSP], sG[NSP];
    uint32_t sO[NSO];
    const rsrc_t rPB = make_rsrc(B, 4u * nE), rPS = make_rsrc(S32, 4u * nE), rPH = make_rsrc(Sh, 4u * nE),
                 rPG = make_rsrc(Gk, 4u * nE), rPO = make_rsrc(goff, 4u * (uint32_t)GOFF_E * (uint32_t)E);
    auto stage_load = [&](int e) {
        const uint32_t se = 4u * (uint32_t)e * n, so = 4u * (uint32_t)e * GOFF_E;
#pragma unroll
        for (int k = 0; k < NSP; ++k) {
            const uint32_t i = threadIdx.x + (uint32_t)(k * bg::THREADS);
            if (n % bg::THREADS == 0 || i < (uint32_t)n) {
                sB[k] = bload1(rPB, 4u * i, se);
                sS[k] = bload1(rPS, 4u * i, se);
                sH[k] = bload1(rPH, 4u * i, se);
                sG[k] = bload1(rPG, 4u * i, se);
            }
        }
#pragma unroll
        for (int k = 0; k < NSO; ++k) {
            const uint32_t i = threadIdx.x + (uint32_t)(k * bg::THREADS);
            if (GOFF_E % bg::THREADS == 0 || i < (uint32_t)GOFF_E)
                sO[k] = __float_as_uint(bload1(rPO, 4u * i, so));
        }
    };
    auto stage_store = [&]() {
#pragma unroll
        for (int k = 0; k < NSP; ++k) {
            const int i = (int)threadIdx.x + k * bg::THREADS;
            if (n % bg::THREADS == 0 || i < n) {
                prm[PB + i] = sB[k];
                prm[PS + i] = cs * sS[k];
                prm[PH + i] = sH[k];
                // lane-major source (t * EPL + r) to float4-major
                const int tq = i / EPL, r = i % EPL;
                prm[PG + ((r / 4) * g::LPR + tq) * 4 + (r % 4)] = sG[k];
            }
        }
#pragma unroll
        for (int k = 0; k < NSO; ++k) {
            const int i = (int)threadIdx.x + k * bg::THREADS;
            if (GOFF_E % bg::THREADS == 0 || i < GOFF_E) {
                const int lq = i / EPL, r = i % EPL;
                prm[PO + ((r / 4) * 64 + lq) * 4 + (r % 4)] = __uint_as_float(sO[k]);
            }
        }
    };
    if (e0 < e1) {
        stage_load(e0);
        stage_store();
        __syncthreads();
    }

    for (int e = e0; e < e1; ++e) {
        float aS[EPL], aG[EPL], aB[EPL];
        if constexpr (PARAMS) {
#pragma unroll
            for (int r = 0; r < EPL; ++r)
                aS[r] = aG[r] = aB[r] = 0.f;
        }
        for (int p = 0; p < passes; ++p) {
            const int64_t row = row_base + (int64_t)p * bg::ROWS;
            const bool valid = row < batch;
            // x of this row (L2-resident after the first expansion); its wait
            // also covers the dphi prefetch issued half an iteration ago
            float xh[EPL];
            bload_row<M, P, VEC>(xh, rx, valid ? (uint32_t)(row * d) * 4u : 0u, d, t, valid);

            // forward recompute: v1 = H B xhat, w = Pi v1, v3 = H G w
            float v[EPL], q[EPL];
            ld_nat(q, PB);
#pragma unroll
            for (int r = 0; r < EPL; ++r)
                v[r] = xh[r] * q[r];
            fwht_up<M, P>(v, buf, t);
            lds_put<M, P, g::GL>(buf, t, v);
            lds_sync<M, P>();
            // the gather positions serve the adjoint's scatter of this pass too
            float w[EPL];
            char* gp[EPL];
            {
                float of[EPL];
                ld_lane(of, PO, lane, 64);
#pragma unroll
                for (int r = 0; r < EPL; ++r) {
                    gp[r] = lbytes + __float_as_uint(of[r]);
                    w[r] = *reinterpret_cast<const float*>(gp[r]);
                }
            }
            lds_sync<M, P>();
            ld_lane(q, PG, t, g::LPR);
#pragma unroll
            for (int r = 0; r < EPL; ++r)
                v[r] = w[r] * q[r];
            fwht_down<M, P>(v, buf, t);

            // dz = c (-sin z dphi_cos + cos z dphi_sin); dS += dz v3; g3 = S dz
            ld_nat(q, PH);
#pragma unroll
            for (int r = 0; r < EPL; ++r) {
                // dz / c: the scale c rides in the staged S (c S) and in
                // the final dS sum
                float co, si;
                cossin_rev1(v[r] * q[r], co, si);
                const float dz = co * sn[r] - si * cn[r];
                if constexpr (PARAMS)
                    aS[r] += dz * v[r];
                v[r] = dz;
            }
            // dphi of the next (row, expansion) while the adjoint runs;
            // the scheduling barrier keeps these loads after the last use of
            // the registers they overwrite
            __builtin_amdgcn_sched_barrier(0);
            if (p + 1 < passes)
                prefetch(e, p + 1);
            else
                prefetch(e + 1, 0);
            __builtin_amdgcn_sched_barrier(0);
            ld_nat(q, PS);
#pragma unroll
            for (int r = 0; r < EPL; ++r)
                v[r] *= q[r];

            // g2 = H g3 (gather layout); dG += g2 w; Pi^T scatter of G g2
            fwht_up<M, P>(v, buf, t);
            ld_lane(q, PG, t, g::LPR);
#pragma unroll
            for (int r = 0; r < EPL; ++r) {
                if constexpr (PARAMS)
                    aG[r] += v[r] * w[r];
                v[r] *= q[r];
            }
#pragma unroll
            for (int r = 0; r < EPL; ++r)
                *reinterpret_cast<float*>(gp[r]) = v[r];
            lds_sync<M, P>();
            lds_get<M, P, g::GL>(buf, t, v);
            lds_sync<M, P>();
            // g0 = H g1 (coalesced layout); dB += g0 xhat; dx += B g0
            fwht_down<M, P>(v, buf, t);
            ld_nat(q, PB);
#pragma unroll
            for (int r = 0; r < EPL; ++r) {
                if constexpr (PARAMS)
                    aB[r] += v[r] * xh[r];
                v[r] *= q[r];
            }
            if (dx != nullptr) {
                float* drow = dxl + (uint32_t)(p * bg::ROWS + (int)(wave * g::RPB + grp)) * (uint32_t)d4;
                if constexpr (VEC && EPL >= 4) {
                    // all reads first (from a clamped, always-valid address),
                    // then the adds and the masked writes: one LDS round trip
                    if (e > e0) {
                        float4 o[NQ];
#pragma unroll
                        for (int j = 0; j < EPL / 4; ++j) {
                            const uint32_t i0 = ct | rpart(M, P, 0, 4 * j);
                            const bool ok = valid && (int)i0 < d;
                            o[j] = *reinterpret_cast<const float4*>(drow + (ok ? i0 : 0u));
                        }
#pragma unroll
                        for (int j = 0; j < EPL / 4; ++j) {
                            v[4 * j] += o[j].x;
                            v[4 * j + 1] += o[j].y;
                            v[4 * j + 2] += o[j].z;
                            v[4 * j + 3] += o[j].w;
                        }
                    }
#pragma unroll
                    for (int j = 0; j < EPL / 4; ++j) {
                        const uint32_t i0 = ct | rpart(M, P, 0, 4 * j);
                        if (valid && (int)i0 < d)
                            *reinterpret_cast<float4*>(drow + i0) =
                                make_float4(v[4 * j], v[4 * j + 1], v[4 * j + 2], v[4 * j + 3]);
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < EPL; ++k) {
                        const uint32_t i = ct | rpart(M, P, 0, k);
                        if (valid && (int)i < d)
                            drow[i] = e > e0 ? drow[i] + v[k] : v[k];
                    }
                }
            }
        }
        if (e + 1 < e1)
            stage_load(e + 1);
        if constexpr (PARAMS)
            block_partials<M>(lds, aS, aG, aB, partial + ((rb * E + e) * 3) * n, wave, grp, t, cs);
        else
            __syncthreads();
        // every wave is done with this expansion's stage (the barrier above)
        if (e + 1 < e1) {
            stage_store();
            __syncthreads();
        }
    }
    if (dx != nullptr) {
        // every wave has added its last expansion: copy the rows out (to
        // the group's slice when the expansions are split)
        __syncthreads();
        const int64_t row0 = rb * passes * bg::ROWS;
        const int64_t left = batch - row0;
        const int nrows = left < (int64_t)passes * bg::ROWS ? (int)left : passes * bg::ROWS;
        float* dxg = dx + eg * dx_group_stride;
        for (int r = 0; r < nrows; ++r)
            for (int i = threadIdx.x; i < d; i += bg::THREADS)
                dxg[(row0 + r) * d + i] = dxl[r * d4 + i];
    }
}

// ------------------------------------------------------------------ reduce
// out[a][e][i] = sum over b of partial[b][e][a][i], in a fixed order: wave w
// of a block sums the blocks b = w, w + 4, w + 8, ... as 8 interleaved
// running sums combined pairwise, then the 4 waves' sums are added in wave
// order.  Each block covers 64 consecutive (a, e, i) outputs, so every load
// instruction reads 256 contiguous bytes.
constexpr int kRedSlices = 4;

__global__ void __launch_bounds__(64 * kRedSlices)
    k_reduce(const float* __restrict__ partial, int64_t blocks, int64_t E, int64_t n, float* __restrict__ dS,
             float* __restrict__ dG, float* __restrict__ dB, float* __restrict__ uS, float* __restrict__ uG,
             float* __restrict__ uB, float alpha, GroupSum gs, int64_t rblocks)
{
    if ((int64_t)blockIdx.x >= rblocks) {
        // the carried group sum, one output per thread
        const int64_t i = ((int64_t)blockIdx.x - rblocks) * (64 * kRedSlices) + threadIdx.x;
        if (i < gs.count) {
            float s = 0.f;
            for (int64_t g = 0; g < gs.groups; ++g)
                s += gs.part[g * gs.count + i];
            gs.out[i] = s;
            if (gs.y != nullptr)
                gs.y[i] += gs.alpha * s;
        }
        return;
    }
    __shared__ float part[kRedSlices][64];
    const int64_t en = E * n;
    const int64_t idx = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
    const int w = (int)(threadIdx.x >> 6);
    const bool live = idx < 3 * en;
    const int64_t a = live ? idx / en : 0;
    const int64_t rem = live ? idx % en : 0;
    const int64_t e = rem / n, i = rem % n;
    const float* src = partial + (e * 3 + a) * n + i;
    const int64_t stride = 3 * en;
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (live) {
        int64_t b = w;
        for (; b + 7 * kRedSlices < blocks; b += 8 * kRedSlices) {
#pragma unroll
            for (int k = 0; k < 8; ++k)
                acc[k] += src[(b + k * kRedSlices) * stride];
        }
#pragma unroll
        for (int k = 0; k < 7; ++k)
            if (b + k * kRedSlices < blocks)
                acc[k] += src[(b + k * kRedSlices) * stride];
    }
    part[w][threadIdx.x & 63] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
    __syncthreads();
    if (w == 0 && live) {
        float s = part[0][threadIdx.x];
        for (int k = 1; k < kRedSlices; ++k)
            s += part[k][threadIdx.x];
        float* out = a == 0 ? dS : (a == 1 ? dG : dB);
        if (out != nullptr)
            out[e * n + i] = s;
        float* upd = a == 0 ? uS : (a == 1 ? uG : uB);
        if (upd != nullptr)
            upd[e * n + i] += alpha * s;
    }
}

// ------------------------------------------------------------------ derive
// For the gather layout of the given P:
//   goff[e][lane][r] = byte offset in the block's LDS of the gather source of
//     register r of lane `lane` (row region included);
//   Gk[e][t][r] = G[e][i] for the element i held there (destination order);
//   Gs[e][q] (forward G): at P = 5, G[e][j] for the destination j whose
//     gather source perm[j] sits at lane-major slot q (G moved to source
//     order, applied before the gather); at P = 4, as Gk (destination order,
//     applied after the gather, where it fuses into the first butterfly);
// and Sh = S / (2 pi) (S in revolutions) in natural order.
template <int M, int P>
__device__ __forceinline__ uint32_t lane_major_slot(uint32_t i)
{
    using g = Geo<M, P>;
    constexpr int L = g::GL;
    uint32_t r = 0, t = 0;
    for (int b = 0; b < g::Q; ++b)
        r |= ((i >> reg_bit(M, P, L, b)) & 1u) << b;
    for (int b = 0; b < g::T; ++b)
        t |= ((i >> thr_bit(M, P, L, b)) & 1u) << b;
    return t * g::EPL + r;
}

// PACK (P = 5, generated B): goff in the packed form of forward.hpp, the
// gather source as a 16-bit LDS float index and the sign words of B after
// the E expansions' indices.
template <int M, int P, bool PACK>
__global__ void k_derive(int64_t E, const int32_t* __restrict__ perm, const float* __restrict__ G,
                         const float* __restrict__ Bsign, const double* __restrict__ S64,
                         const float* __restrict__ S32, uint32_t* __restrict__ goff, float* __restrict__ Gk,
                         float* __restrict__ Gs, float* __restrict__ Sh)
{
    using g = Geo<M, P>;
    constexpr int K = g::K, EPL = g::EPL, n = g::n;
    constexpr int64_t kGoffE = (int64_t)g::RPB * n;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= E * kGoffE)
        return;
    const int64_t e = idx / kGoffE;
    const uint32_t q = (uint32_t)(idx % kGoffE);  // lane * EPL + r
    const uint32_t lane = q / EPL;
    const int r = (int)(q % EPL);
    const uint32_t grp = g::kMulti ? 0u : lane / g::LPR;
    const uint32_t t = g::kMulti ? lane : lane % g::LPR;
    const uint32_t i = tpart<M, P, g::GL>(t) | rpart(M, P, g::GL, r);
    const uint32_t src = (uint32_t)perm[e * n + i] & (uint32_t)(n - 1);
    if constexpr (PACK) {
        static_assert((int64_t)g::RPB * g::STRIDE <= 65536, "16-bit LDS float index");
        reinterpret_cast<uint16_t*>(goff)[idx] = (uint16_t)(grp * (uint32_t)g::STRIDE + phys<P>(src));
        if (q < (uint32_t)g::LPR) {
            // sign word of lane-in-row t = q: bit r set where B is -1 at the
            // element register r holds in the coalesced layout
            uint32_t w = 0;
            const uint32_t tb = tpart<M, P, 0>(q);
            for (int rr = 0; rr < EPL; ++rr)
                w |= (Bsign[e * n + (tb | rpart(M, P, 0, rr))] < 0.f ? 1u : 0u) << rr;
            goff[packed_sign_word0<M, P>(E) + e * g::LPR + q] = w;
        }
    } else {
        goff[idx] = 4u * (grp * (uint32_t)g::STRIDE + phys<P>(src));
    }
    if (q < (uint32_t)n) {
        const uint32_t tq = q / EPL;
        const uint32_t iq = tpart<M, P, g::GL>(tq) | rpart(M, P, g::GL, (int)(q % EPL));
        if (Gk)
            Gk[e * n + q] = G[e * n + iq];
        if (Gs) {
            if constexpr (fwd_g_after_gather(P)) {
                Gs[e * n + q] = G[e * n + iq];
            } else {
                const uint32_t srcq = (uint32_t)perm[e * n + q] & (uint32_t)(n - 1);
                Gs[e * n + lane_major_slot<M, P>(srcq)] = G[e * n + q];
            }
        }
        if (Sh) {
            // S in revolutions for the feature map, from the FP64 value when present
            const double sv = S64 ? S64[e * n + q] : (double)S32[e * n + q];
            Sh[e * n + q] = (float)(sv * 0.15915494309189533577);
        }
    }
}

template <int M>
struct RunFwht {
    static hipError_t run(float* data, int64_t batch, bool vec, hipStream_t s)
    {
        using g = Geo<M, kFwhtP>;
        const int64_t rows_per = kRangeLimit / (4 * g::n);
        for (int64_t r0 = 0; r0 < batch; r0 += rows_per) {
            const int64_t rows = batch - r0 < rows_per ? batch - r0 : rows_per;
            const int64_t blocks = (rows + g::RPB - 1) / g::RPB;
            float* p = data + r0 * g::n;
            const uint32_t bytes = (uint32_t)(4 * rows * g::n);
            if (vec && M >= 2)
                k_fwht<M, true><<<dim3((unsigned)blocks), dim3(g::BLOCK), 0, s>>>(p, bytes, rows);
            else
                k_fwht<M, false><<<dim3((unsigned)blocks), dim3(g::BLOCK), 0, s>>>(p, bytes, rows);
            const hipError_t err = hipGetLastError();
            if (err != hipSuccess)
                return err;
        }
        return hipSuccess;
    }
};

template <int M>
struct RunBackward {
    static hipError_t run(bool vec, const float* x, const float* dphi, int64_t batch, int d, int64_t E,
                          const float* B, const uint32_t* goff, const float* Gk, const float* S32, const float* Sh,
                          float cs, float* dx, float* partial, const BwdGeometry& geo, hipStream_t s)
    {
        using bg = BwdGeo<M>;
        using g = typename bg::g;
        const dim3 grid((unsigned)geo.blocks), blk(bg::THREADS);
        const int Ei = (int)E;
        const size_t dyn = bg::XRES && dx ? (size_t)geo.passes * bg::ROWS * ((d + 3) & ~3) * 4 : 0;
        const uint32_t xb = (uint32_t)(4 * batch * d), db = (uint32_t)(4 * batch * 2 * g::n * E);
        const uint32_t par_bytes = (uint32_t)(4 * g::n * E);
        const uint32_t goff_bytes = (uint32_t)(4 * g::RPB * g::n * E);
        auto launch = [&](auto kern, auto... args) -> hipError_t {
            if (dyn > 0) {
                const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
                if (e != hipSuccess)
                    return e;
            }
            kern<<<grid, blk, dyn, s>>>(args...);
            return hipGetLastError();
        };
#define MCK_BWD_ARGS x, xb, dphi, db, batch, d, Ei, B, goff, Gk, S32, Sh, par_bytes, goff_bytes, cs, dx, partial, \
                     geo.passes
#define MCK_BWDR_ARGS x, xb, dphi, db, batch, d, Ei, B, goff, Gk, S32, Sh, cs, dx, partial, geo.passes, geo.esplit, \
                      geo.rowblocks, (int64_t)batch * d
        hipError_t err;
        if constexpr (bg::XRES) {
            if (vec && M >= 2)
                err = partial ? launch(k_backward_rows<M, true, true>, MCK_BWDR_ARGS)
                              : launch(k_backward_rows<M, true, false>, MCK_BWDR_ARGS);
            else
                err = partial ? launch(k_backward_rows<M, false, true>, MCK_BWDR_ARGS)
                              : launch(k_backward_rows<M, false, false>, MCK_BWDR_ARGS);
        } else {
            if (vec && M >= 2)
                err = partial ? launch(k_backward<M, true, true>, MCK_BWD_ARGS)
                              : launch(k_backward<M, true, false>, MCK_BWD_ARGS);
            else
                err = partial ? launch(k_backward<M, false, true>, MCK_BWD_ARGS)
                              : launch(k_backward<M, false, false>, MCK_BWD_ARGS);
        }
#undef MCK_BWD_ARGS
#undef MCK_BWDR_ARGS
        return err;
    }
};

template <int M>
struct RunGeometry {
    static hipError_t run(int64_t batch, int d, int64_t E, BwdGeometry* out)
    {
        using bg = BwdGeo<M>;
        // Blocks own contiguous runs of rows.  With the dx rows in LDS, one
        // block fills a CU's LDS: aim for one block per CU (256), as many
        // rows per block as the LDS holds; otherwise about 512 blocks.
        const int64_t units = (batch + bg::ROWS - 1) / bg::ROWS;
        const int64_t target = bg::XRES ? 256 : 512;
        int64_t passes = (units + target - 1) / target;
        if (bg::XRES) {
            const int64_t row_bytes = (int64_t)bg::ROWS * ((d + 3) & ~3) * 4;
            int64_t pmax = (kLdsBytes - bg::STATIC_LDS - bg::PARAM_LDS) / row_bytes;
            pmax = pmax < 1 ? 1 : pmax;
            passes = passes > pmax ? pmax : passes;
        }
        if (passes < 1)
            passes = 1;
        out->passes = (int)passes;
        out->blocks = (units + passes - 1) / passes;
        if (out->blocks < 1)
            out->blocks = 1;
        out->rowblocks = out->blocks;
        out->esplit = 1;
        if (bg::XRES && out->blocks < 256 && E > 1) {
            // too few row blocks to fill the CUs: split the expansions over
            // several block groups (each group's dx summed afterwards)
            int64_t es = (256 + out->blocks - 1) / out->blocks;
            es = es > E ? E : (es > 8 ? 8 : es);
            out->esplit = (int)es;
            out->blocks = out->rowblocks * es;
        }
        out->block_threads = bg::THREADS;
        out->rows_per_pass = bg::ROWS;
        return hipSuccess;
    }
};

template <int M>
struct RunPlanElems {
    static hipError_t run(int64_t* fwd_goff, int64_t* bwd_goff)
    {
        int64_t f = (int64_t)Geo<M, fwd_p(M)>::RPB * Geo<M, fwd_p(M)>::n;
        if constexpr (fwd_p_tunable(M)) {
            const int64_t a = (int64_t)Geo<M, fwd_p_alt(M)>::RPB * Geo<M, fwd_p_alt(M)>::n;
            f = a > f ? a : f;
        }
        *fwd_goff = f;
        *bwd_goff = (int64_t)Geo<M, bwd_p(M)>::RPB * Geo<M, bwd_p(M)>::n;
        return hipSuccess;
    }
};

template <int M, int P, bool PACK = false>
hipError_t derive_one(int64_t E, const int32_t* perm, const float* G, const float* Bsign, const double* S64,
                      const float* S32, uint32_t* goff, float* Gk, float* Gs, float* Sh, hipStream_t s)
{
    const int64_t t = E * Geo<M, P>::RPB * Geo<M, P>::n;
    k_derive<M, P, PACK><<<dim3((unsigned)((t + 255) / 256)), dim3(256), 0, s>>>(E, perm, G, Bsign, S64, S32, goff,
                                                                                 Gk, Gs, Sh);
    return hipGetLastError();
}

// forward arrays (and Sh when given) for register split PF; packed at P = 5
// when Bsign (the generated B) is given
template <int M, int PF>
hipError_t derive_fwd_p(int64_t E, const int32_t* perm, const float* G, const float* Bsign, const double* S64,
                        const float* S32, uint32_t* goff_f, float* Gs_f, float* Sh, hipStream_t s)
{
    if constexpr (PF == 5)
        if (Bsign)
            return derive_one<M, PF, true>(E, perm, G, Bsign, S64, S32, goff_f, nullptr, Gs_f, Sh, s);
    return derive_one<M, PF>(E, perm, G, nullptr, S64, S32, goff_f, nullptr, Gs_f, Sh, s);
}

template <int M>
hipError_t derive_fwd(int PF, int64_t E, const int32_t* perm, const float* G, const float* Bsign, const double* S64,
                      const float* S32, uint32_t* goff_f, float* Gs_f, float* Sh, hipStream_t s)
{
    if (PF == fwd_p(M))
        return derive_fwd_p<M, fwd_p(M)>(E, perm, G, Bsign, S64, S32, goff_f, Gs_f, Sh, s);
    if constexpr (fwd_p_tunable(M))
        if (PF == fwd_p_alt(M))
            return derive_fwd_p<M, fwd_p_alt(M)>(E, perm, G, Bsign, S64, S32, goff_f, Gs_f, Sh, s);
    return hipErrorInvalidValue;
}

template <int M>
struct RunDerive {
    static hipError_t run(int PF, int64_t E, const int32_t* perm, const float* G, const float* Bsign,
                          const double* S64, const float* S32, uint32_t* goff_f, float* Gs_f, uint32_t* goff_b,
                          float* Gk_b, float* Sh, hipStream_t s)
    {
        if (goff_b == goff_f) {
            // one unpacked layout serves both directions: one launch
            if (PF != bwd_p(M) || Bsign != nullptr)
                return hipErrorInvalidValue;
            return derive_one<M, bwd_p(M)>(E, perm, G, nullptr, S64, S32, goff_f, Gk_b, Gs_f, Sh, s);
        }
        const hipError_t err = derive_fwd<M>(PF, E, perm, G, Bsign, S64, S32, goff_f, Gs_f, Sh, s);
        if (err != hipSuccess)
            return err;
        return derive_one<M, bwd_p(M)>(E, perm, G, nullptr, S64, S32, goff_b, Gk_b, nullptr, nullptr, s);
    }
};

template <int M>
struct RunDeriveBwd {
    static hipError_t run(int64_t E, const int32_t* perm, const float* G, const float* S32, uint32_t* goff_b,
                          float* Gk_b, float* Sh, hipStream_t s)
    {
        return derive_one<M, bwd_p(M)>(E, perm, G, nullptr, nullptr, S32, goff_b, Gk_b, nullptr, Sh, s);
    }
};

template <int M>
struct RunDeriveFwd {
    static hipError_t run(int PF, int64_t E, const int32_t* perm, const float* G, const float* Bsign,
                          uint32_t* goff_f, float* Gs_f, hipStream_t s)
    {
        return derive_fwd<M>(PF, E, perm, G, Bsign, nullptr, nullptr, goff_f, Gs_f, nullptr, s);
    }
};

template <int M>
struct RunSplit {
    static hipError_t run(int P, bool* ok, int* def)
    {
        *ok = fwd_p_ok(M, P);
        *def = P < 0 ? bwd_p(M) : fwd_p(M);
        return hipSuccess;
    }
};

}  // namespace

hipError_t launch_fwht(int M, float* data, int64_t batch, bool vec, hipStream_t s)
{
    return dispatch_m<RunFwht>(M, data, batch, vec, s);
}

hipError_t launch_forward(int M, int P, int waves, bool packed, bool vec, bool trig, const float* x, int64_t batch,
                          int d, int64_t E, const float* B, const uint32_t* goff, const float* Gs, const float* Sx,
                          float cs, float* out, hipStream_t s, const int8_t* xexp)
{
    return dispatch_m<RunForwardT<kF32, kF32>::Run>(M, P, waves, packed, vec, trig, x, batch, d, E, B, goff, Gs, Sx,
                                                    cs, out, s, xexp);
}

bool fwd_split_ok(int M, int P)
{
    bool ok = false;
    int def = 0;
    return dispatch_m<RunSplit>(M, P, &ok, &def) == hipSuccess && ok;
}

int fwd_split_default(int M)
{
    bool ok = false;
    int def = 0;
    (void)dispatch_m<RunSplit>(M, 0, &ok, &def);
    return def;
}

int bwd_split(int M)
{
    bool ok = false;
    int def = 0;
    (void)dispatch_m<RunSplit>(M, -1, &ok, &def);
    return def;
}

namespace {

template <int M>
struct RunGroup {
    static hipError_t run(int P, int waves, bool vec, const GroupInst* inst, int count, hipStream_t s)
    {
        if (P == fwd_p(M))
            return run_p<fwd_p(M)>(waves, vec, inst, count, s);
        if constexpr (fwd_p_tunable(M))
            if (P == fwd_p_alt(M))
                return run_p<fwd_p_alt(M)>(waves, vec, inst, count, s);
        return hipErrorInvalidValue;
    }

    template <int P>
    static hipError_t run_p(int waves, bool vec, const GroupInst* inst, int count, hipStream_t s)
    {
        using g = Geo<M, P>;
        // split expansions so that the whole group holds >= `waves` waves
        int64_t base_waves = 0;
        for (int i = 0; i < count; ++i)
            base_waves += (inst[i].batch + g::RPB - 1) / g::RPB * (g::BLOCK / 64);
        const int64_t factor = base_waves > 0 ? (waves + base_waves - 1) / base_waves : 1;
        for (int i0 = 0; i0 < count; i0 += kGroupMax) {
            FwdGroup grp;
            grp.count = count - i0 < kGroupMax ? count - i0 : kGroupMax;
            int64_t blocks = 0;
            for (int k = 0; k < grp.count; ++k) {
                const GroupInst& in = inst[i0 + k];
                FwdDesc& q = grp.m[k];
                const int64_t groups = (in.batch + g::RPB - 1) / g::RPB;
                int64_t nchunks = factor > in.E ? in.E : factor;
                const int64_t echunk = (in.E + nchunks - 1) / nchunks;
                nchunks = (in.E + echunk - 1) / echunk;
                q.x = in.x;
                q.out = in.phi;
                q.B = in.B;
                q.goff = in.goff;
                q.Gs = in.Gs;
                q.Sx = in.Sh;
                q.batch = in.batch;
                q.block0 = blocks;
                q.d = in.d;
                q.E = (int)in.E;
                q.echunk = (int)echunk;
                q.nchunks = (int)nchunks;
                q.x_bytes = (uint32_t)(4 * in.batch * in.d);
                q.out_bytes = (uint32_t)(4 * in.batch * 2 * g::n * in.E);
                q.par_bytes = (uint32_t)(4 * g::n * in.E);
                q.goff_bytes = (uint32_t)(4 * g::RPB * g::n * in.E);
                q.cs = in.cs;
                blocks += ((groups + kXcds - 1) / kXcds) * kXcds * nchunks;
            }
            const dim3 grid((unsigned)blocks), blk(g::BLOCK);
            if (vec && M >= 2)
                k_forward_group<M, P, true><<<grid, blk, 0, s>>>(grp);
            else
                k_forward_group<M, P, false><<<grid, blk, 0, s>>>(grp);
            const hipError_t err = hipGetLastError();
            if (err != hipSuccess)
                return err;
        }
        return hipSuccess;
    }
};

}  // namespace

hipError_t launch_forward_group(int M, int P, int waves, bool vec, const GroupInst* inst, int count, hipStream_t s)
{
    return dispatch_m<RunGroup>(M, P, waves, vec, inst, count, s);
}

BwdGeometry backward_geometry(int M, int64_t batch, int d, int64_t E)
{
    BwdGeometry g{1, 1, 64, 1, 1, 1};
    (void)dispatch_m<RunGeometry>(M, batch, d, E, &g);
    return g;
}

hipError_t launch_backward(int M, bool vec, const float* x, const float* dphi, int64_t batch, int d, int64_t E,
                           const float* B, const uint32_t* goff, const float* Gk, const float* S32,
                           const float* Sh, float cs, float* dx, float* partial,
                           const BwdGeometry& geo, hipStream_t s)
{
    return dispatch_m<RunBackward>(M, vec, x, dphi, batch, d, E, B, goff, Gk, S32, Sh, cs, dx, partial, geo, s);
}

hipError_t launch_reduce(const float* partial, int64_t blocks, int64_t E, int64_t n, float* dS, float* dG,
                         float* dB, hipStream_t s, float* uS, float* uG, float* uB, float alpha,
                         const GroupSum* extra)
{
    const int64_t total = 3 * E * n;
    const int64_t rblocks = (total + 63) / 64;
    const GroupSum gs = extra ? *extra : GroupSum{nullptr, 0, 0, nullptr, nullptr, 0.f};
    const int64_t gblocks = (gs.count + 64 * kRedSlices - 1) / (64 * kRedSlices);
    k_reduce<<<dim3((unsigned)(rblocks + gblocks)), dim3(64 * kRedSlices), 0, s>>>(
        partial, blocks, E, n, dS, dG, dB, uS, uG, uB, alpha, gs, rblocks);
    return hipGetLastError();
}

void plan_elems(int M, int64_t* fwd_goff, int64_t* bwd_goff)
{
    *fwd_goff = *bwd_goff = 0;
    (void)dispatch_m<RunPlanElems>(M, fwd_goff, bwd_goff);
}

hipError_t launch_derive(int M, int PF, int64_t E, const int32_t* perm, const float* G, const float* Bsign,
                         const double* S64, const float* S32, uint32_t* goff_f, float* Gs_f, uint32_t* goff_b,
                         float* Gk_b, float* Sh, hipStream_t s)
{
    return dispatch_m<RunDerive>(M, PF, E, perm, G, Bsign, S64, S32, goff_f, Gs_f, goff_b, Gk_b, Sh, s);
}

hipError_t launch_derive_bwd(int M, int64_t E, const int32_t* perm, const float* G, const float* S32,
                             uint32_t* goff_b, float* Gk_b, float* Sh, hipStream_t s)
{
    return dispatch_m<RunDeriveBwd>(M, E, perm, G, S32, goff_b, Gk_b, Sh, s);
}

hipError_t launch_derive_fwd(int M, int PF, int64_t E, const int32_t* perm, const float* G, const float* Bsign,
                             uint32_t* goff_f, float* Gs_f, hipStream_t s)
{
    return dispatch_m<RunDeriveFwd>(M, PF, E, perm, G, Bsign, goff_f, Gs_f, s);
}

}  // namespace mck
