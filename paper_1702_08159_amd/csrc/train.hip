// train.hip -- the training step's feature-map kernels with the classifier
// head fused in (section "Empirical Analysis and Experiments": softmax(W phi
// + b) on the McKernel features, trained by SGD), so that phi never goes to
// HBM:
//   k_forward_logits  phi of 8 rows per block (one wave each) and expansion,
//                     through an LDS tile, straight into the logits W phi:
//                     only the batch x C partial logits leave the block
//   k_head_bwd_fused  phi recomputed the same way for one expansion and a
//                     range of rows: dW partials (dlogits^T phi) accumulate
//                     in VGPRs, and dphi = dlogits W is written for the
//                     adjoint
// For n = 1024 (one row per wave, 16 values per lane: the MNIST-shaped
// configuration) and the explicit-parameter forward layout; the runtime
// takes the unfused kernels elsewhere.  In the tile phase lane L of the
// block owns four consecutive features 4L..4L+3 of the expansion's 2n
// (cos block then sin block), so the contraction over features (logits) or
// over rows (dW) runs with C x 4 weights in VGPRs.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "engine.hpp"
#include "forward.hpp"
#include "launch.hpp"

namespace mck {
namespace {

constexpr int kTM = 10, kTP = 4;  // n = 1024, 16 values per lane
using TG = Geo<kTM, kTP>;
constexpr int kTW = 8;           // rows (waves) per tile
constexpr int kTF = 2 * TG::n;   // features of one row and expansion
static_assert(kTF == 4 * kTW * 64, "four features per lane of the block");
static_assert(!TG::kMulti && TG::RPB == 1, "one row per wave");

struct TileParams {
    rsrc_t rB, rG, rO, rS;  // B (natural), G (destination order), gather offsets, S / 2 pi
};

// One expansion's parameters in a lane's registers (coalesced layout for B
// and S / 2 pi, lane-major for G and the gather offsets).
struct ExpParams {
    float b[16], g[16], s[16];
    uint32_t off[16];
};

__device__ __forceinline__ void load_exp(ExpParams& q, const TileParams& p, int e, uint32_t lane)
{
    constexpr int n = TG::n;
    constexpr uint32_t kGoffE = (uint32_t)TG::RPB * n;
    bload_coal<kTM, kTP>(q.b, p.rB, 4u * (uint32_t)e * n, lane);
    bload_lane<kTM, kTP, float>(q.g, p.rG, 4u * (uint32_t)e * n, lane);
    bload_lane<kTM, kTP, uint32_t>(q.off, p.rO, 4u * (uint32_t)e * kGoffE, lane);
    bload_coal<kTM, kTP>(q.s, p.rS, 4u * (uint32_t)e * n, lane);
}

// z (in revolutions) of one row and expansion, coalesced layout:
// v = B xhat; H; gather v[perm[i]] in LDS; G (destination order); H; S/2pi.
__device__ __forceinline__ void row_z(float (&v)[16], const float (&xh)[16], const ExpParams& q, float* buf,
                                      uint32_t lane)
{
    constexpr int EPL = TG::EPL;
    const char* lbytes = reinterpret_cast<const char*>(buf);
#pragma unroll
    for (int r = 0; r < EPL; ++r)
        v[r] = xh[r] * q.b[r];
    fwht_up<kTM, kTP>(v, buf, lane);
    static_assert(fwd_g_after_gather(kTP), "the forward arrays hold G in destination order");
    lds_put<kTM, kTP, TG::GL>(buf, lane, v);
    wave_fence();
#pragma unroll
    for (int r = 0; r < EPL; ++r)
        v[r] = *reinterpret_cast<const float*>(lbytes + q.off[r]) * q.g[r];
    wave_fence();
    fwht_down<kTM, kTP>(v, buf, lane);
#pragma unroll
    for (int r = 0; r < EPL; ++r)
        v[r] *= q.s[r];
}

// c cos z and c sin z of a row into its tile row: cos at [0, n), sin at
// [n, 2n), natural order.
__device__ __forceinline__ void tile_put(float* trow, const float (&z)[16], float cs, uint32_t lane)
{
    constexpr int EPL = TG::EPL, n = TG::n;
    const uint32_t tb = tpart<kTM, kTP, 0>(lane);
#pragma unroll
    for (int j = 0; j < EPL / 4; ++j) {
        float c4[4], s4[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            cossin_rev(z[4 * j + k], cs, c4[k], s4[k]);
        const uint32_t i0 = tb | rpart(kTM, kTP, 0, 4 * j);
        *reinterpret_cast<float4*>(trow + i0) = make_float4(c4[0], c4[1], c4[2], c4[3]);
        *reinterpret_cast<float4*>(trow + n + i0) = make_float4(s4[0], s4[1], s4[2], s4[3]);
    }
}

// column of phi (row length F = 2nE) of feature f of expansion e
__device__ __forceinline__ int64_t phi_col(int64_t f, int e, int64_t nE)
{
    constexpr int64_t n = TG::n;
    return f < n ? (int64_t)e * n + f : nE + (int64_t)e * n + (f - n);
}

// Block (row group of 8, expansion group eg): rows r0 .. r0 + 7 over the
// expansions [e0, e1); part[eg][row][c] = sum over those expansions of the
// row's features times W[c][.], reduced in a fixed order (lanes by xor
// butterfly within a wave, then waves in order).
template <int C, bool VEC>
__global__ void __launch_bounds__(kTW * 64, 1)
    k_forward_logits(const float* __restrict__ x, uint32_t x_bytes, int64_t batch, int d, int E, int esplit,
                     const float* __restrict__ B, const uint32_t* __restrict__ goff, const float* __restrict__ Gs,
                     const float* __restrict__ Sh, uint32_t par_bytes, uint32_t goff_bytes, float cs,
                     const float* __restrict__ W, int64_t F, float* __restrict__ part)
{
    constexpr int EPL = TG::EPL, n = TG::n;
    __shared__ __align__(16) float tbuf[kTW * TG::LDS_FLOATS];
    __shared__ __align__(16) float tile[kTW * kTF];
    const uint32_t wave = threadIdx.x / 64u, lane = threadIdx.x % 64u, L = threadIdx.x;
    const int64_t groups = (batch + kTW - 1) / kTW;
    const int64_t grp = (int64_t)blockIdx.x % groups;
    const int eg = (int)((int64_t)blockIdx.x / groups);
    const int e0 = (int)((int64_t)eg * E / esplit), e1 = (int)((int64_t)(eg + 1) * E / esplit);
    const int64_t row = grp * kTW + wave;
    const bool valid = row < batch;
    float* buf = tbuf + wave * TG::LDS_FLOATS;
    const TileParams p{make_rsrc(B, par_bytes), make_rsrc(Gs, par_bytes), make_rsrc(goff, goff_bytes),
                       make_rsrc(Sh, par_bytes)};
    const rsrc_t rx = make_rsrc(x, x_bytes), rW = make_rsrc(W, (uint32_t)(C * F * 4));
    const int64_t nE = (int64_t)n * E;
    float xh[EPL];
    bload_row<kTM, kTP, VEC>(xh, rx, valid ? (uint32_t)(row * d) * 4u : 0u, d, lane, valid);
    float acc[kTW][C];
#pragma unroll
    for (int r = 0; r < kTW; ++r)
#pragma unroll
        for (int c = 0; c < C; ++c)
            acc[r][c] = 0.f;
    // the expansion's parameters are loaded one expansion ahead (during the
    // tile phase) and its W columns before its transform, so neither waits
    ExpParams q;
    if (e0 < e1)
        load_exp(q, p, e0, lane);
    for (int e = e0; e < e1; ++e) {
        const int64_t col = phi_col(4 * (int64_t)L, e, nE);
        float w[C][4];
#pragma unroll
        for (int c = 0; c < C; ++c)
            bload4(w[c], rW, (uint32_t)(4 * (c * F + col)), 0u);
        float z[EPL];
        row_z(z, xh, q, buf, lane);
        if (e + 1 < e1)
            load_exp(q, p, e + 1, lane);
        tile_put(tile + wave * kTF, z, cs, lane);
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kTW; ++r) {
            const float4 f = *reinterpret_cast<const float4*>(tile + r * kTF + 4 * L);
#pragma unroll
            for (int c = 0; c < C; ++c)
                acc[r][c] += w[c][0] * f.x + w[c][1] * f.y + w[c][2] * f.z + w[c][3] * f.w;
        }
        __syncthreads();  // the tile is rewritten by the next expansion
    }
#pragma unroll
    for (int r = 0; r < kTW; ++r)
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1)
                acc[r][c] += __shfl_xor(acc[r][c], o);
    float* red = tile;  // [wave][r C + c]
    if (lane == 0) {
#pragma unroll
        for (int r = 0; r < kTW; ++r)
#pragma unroll
            for (int c = 0; c < C; ++c)
                red[wave * kTW * C + r * C + c] = acc[r][c];
    }
    __syncthreads();
    if (L < (uint32_t)(kTW * C)) {
        float s = 0.f;
        for (int w = 0; w < kTW; ++w)
            s += red[w * kTW * C + L];
        const int64_t rr = grp * kTW + L / C;
        if (rr < batch)
            part[((int64_t)eg * batch + rr) * C + L % C] = s;
    }
}

// Block (expansion e, row range rg): the range's rows in tiles of 8; for
// each row r of a tile, dphi[r][cols of the lane's features] = dlogits[r] W
// and acc[c][.] += dlogits[r][c] phi[r][.]; the range's dW partial goes to
// part[rg][c][col].  Rows past the range are computed as zeros and skipped.
template <int C, bool VEC>
__global__ void __launch_bounds__(kTW * 64, 1)
    k_head_bwd_fused(const float* __restrict__ x, uint32_t x_bytes, int64_t batch, int d, int E,
                     int64_t rows_per_range, const float* __restrict__ B, const uint32_t* __restrict__ goff,
                     const float* __restrict__ Gs, const float* __restrict__ Sh, uint32_t par_bytes,
                     uint32_t goff_bytes, float cs, const float* __restrict__ dl, const float* __restrict__ W,
                     int64_t F, float* __restrict__ dphi, float* __restrict__ part)
{
    constexpr int EPL = TG::EPL, n = TG::n;
    __shared__ __align__(16) float tbuf[kTW * TG::LDS_FLOATS];
    __shared__ __align__(16) float tile[kTW * kTF];
    const uint32_t wave = threadIdx.x / 64u, lane = threadIdx.x % 64u, L = threadIdx.x;
    const int e = (int)((int64_t)blockIdx.x % E);
    const int64_t rg = (int64_t)blockIdx.x / E;
    const int64_t rb = rg * rows_per_range;
    const int64_t re = rb + rows_per_range < batch ? rb + rows_per_range : batch;
    float* buf = tbuf + wave * TG::LDS_FLOATS;
    const TileParams p{make_rsrc(B, par_bytes), make_rsrc(Gs, par_bytes), make_rsrc(goff, goff_bytes),
                       make_rsrc(Sh, par_bytes)};
    const rsrc_t rx = make_rsrc(x, x_bytes), rW = make_rsrc(W, (uint32_t)(C * F * 4));
    const int64_t nE = (int64_t)n * E;
    const int64_t col = phi_col(4 * (int64_t)L, e, nE);
    __shared__ float dlt[kTW * C];  // dlogits of the tile's rows
    ExpParams q;  // the block's expansion, for all its rows
    load_exp(q, p, e, lane);
    float w[C][4], acc[C][4];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        bload4(w[c], rW, (uint32_t)(4 * (c * F + col)), 0u);
#pragma unroll
        for (int k = 0; k < 4; ++k)
            acc[c][k] = 0.f;
    }
    for (int64_t r0 = rb; r0 < re; r0 += kTW) {
        const int64_t row = r0 + wave;
        const bool valid = row < re;
        float xh[EPL], z[EPL];
        bload_row<kTM, kTP, VEC>(xh, rx, valid ? (uint32_t)(row * d) * 4u : 0u, d, lane, valid);
        const int nr = re - r0 < kTW ? (int)(re - r0) : kTW;
        if (L < (uint32_t)(nr * C))
            dlt[L] = dl[r0 * C + L];
        row_z(z, xh, q, buf, lane);
        tile_put(tile + wave * kTF, z, cs, lane);
        __syncthreads();
        for (int r = 0; r < nr; ++r) {
            const float4 f = *reinterpret_cast<const float4*>(tile + r * kTF + 4 * L);
            const float* dlr = dlt + r * C;
            float o[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const float g = dlr[c];
                acc[c][0] += g * f.x;
                acc[c][1] += g * f.y;
                acc[c][2] += g * f.z;
                acc[c][3] += g * f.w;
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    o[k] += g * w[c][k];
            }
            bstore4_nt(make_rsrc(dphi + (r0 + r) * F, (uint32_t)(F * 4)), (uint32_t)(4 * col), o[0], o[1], o[2],
                       o[3]);
        }
        __syncthreads();  // the tile is rewritten by the next rows
    }
    const rsrc_t ro = make_rsrc(part + rg * C * F, (uint32_t)(C * F * 4));
#pragma unroll
    for (int c = 0; c < C; ++c)
        bstore4(ro, (uint32_t)(4 * (c * F + col)), acc[c][0], acc[c][1], acc[c][2], acc[c][3]);
}

}  // namespace

bool fused_head_ok(int64_t n, int64_t C) { return n == TG::n && C >= 1 && C <= kFusedHeadMaxC; }

int64_t fused_logits_esplit(int64_t batch, int64_t E)
{
    const int64_t groups = (batch + kTW - 1) / kTW;
    int64_t es = (256 + groups - 1) / groups;
    return es > E ? E : (es < 1 ? 1 : es);
}

void fused_bwd_geometry(int64_t batch, int64_t E, int64_t* ranges, int64_t* rows_per_range)
{
    const int64_t tiles = (batch + kTW - 1) / kTW;
    int64_t rg = (256 + E - 1) / E;
    rg = rg > tiles ? tiles : (rg < 1 ? 1 : rg);
    const int64_t tiles_per = (tiles + rg - 1) / rg;
    *rows_per_range = tiles_per * kTW;
    *ranges = (batch + *rows_per_range - 1) / *rows_per_range;
}

#define MCK_FUSED_C(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10)

hipError_t launch_forward_logits(bool vec, const float* x, int64_t batch, int d, int64_t E, const float* B,
                                 const uint32_t* goff, const float* Gs, const float* Sh, float cs, const float* W,
                                 int C, int64_t esplit, float* part, hipStream_t s)
{
    const int64_t n = TG::n, F = 2 * n * E;
    const int64_t groups = (batch + kTW - 1) / kTW;
    const dim3 grid((unsigned)(groups * esplit)), blk(kTW * 64);
    const uint32_t xb = (uint32_t)(4 * batch * d), pb = (uint32_t)(4 * n * E), ob = (uint32_t)(4 * TG::RPB * n * E);
#define MCK_FL_CASE(K)                                                                                             \
    case K:                                                                                                        \
        if (vec)                                                                                                   \
            k_forward_logits<K, true><<<grid, blk, 0, s>>>(x, xb, batch, d, (int)E, (int)esplit, B, goff, Gs, Sh, \
                                                           pb, ob, cs, W, F, part);                                \
        else                                                                                                       \
            k_forward_logits<K, false><<<grid, blk, 0, s>>>(x, xb, batch, d, (int)E, (int)esplit, B, goff, Gs, Sh, \
                                                            pb, ob, cs, W, F, part);                               \
        break;
    switch (C) {
        MCK_FUSED_C(MCK_FL_CASE)
    default: return hipErrorInvalidValue;
    }
#undef MCK_FL_CASE
    return hipGetLastError();
}

hipError_t launch_head_bwd_fused(bool vec, const float* x, int64_t batch, int d, int64_t E, const float* B,
                                 const uint32_t* goff, const float* Gs, const float* Sh, float cs, const float* dl,
                                 const float* W, int C, int64_t ranges, int64_t rows_per_range, float* dphi,
                                 float* part, hipStream_t s)
{
    const int64_t n = TG::n, F = 2 * n * E;
    const dim3 grid((unsigned)(ranges * E)), blk(kTW * 64);
    const uint32_t xb = (uint32_t)(4 * batch * d), pb = (uint32_t)(4 * n * E), ob = (uint32_t)(4 * TG::RPB * n * E);
#define MCK_FB_CASE(K)                                                                                              \
    case K:                                                                                                         \
        if (vec)                                                                                                    \
            k_head_bwd_fused<K, true><<<grid, blk, 0, s>>>(x, xb, batch, d, (int)E, rows_per_range, B, goff, Gs, Sh, \
                                                           pb, ob, cs, dl, W, F, dphi, part);                       \
        else                                                                                                        \
            k_head_bwd_fused<K, false><<<grid, blk, 0, s>>>(x, xb, batch, d, (int)E, rows_per_range, B, goff, Gs,   \
                                                            Sh, pb, ob, cs, dl, W, F, dphi, part);                  \
        break;
    switch (C) {
        MCK_FUSED_C(MCK_FB_CASE)
    default: return hipErrorInvalidValue;
    }
#undef MCK_FB_CASE
    return hipGetLastError();
}

#undef MCK_FUSED_C

}  // namespace mck
