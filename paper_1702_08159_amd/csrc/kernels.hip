// kernels.hip -- the Fastfood hot path on gfx950.
//
//   k_fwht      in-place batched H v (section "Fast Walsh Hadamard")
//   k_forward   phi = c [cos z, sin z], z = S H G Pi H B xhat for every
//               expansion (equations mckernel and mcfeatures), fused: one HBM
//               read of x per row, one HBM write of phi, everything else in
//               registers and LDS
//   k_backward  adjoint of the same chain (H is symmetric, Pi^T a scatter),
//               recomputing the forward instead of storing it
//   k_reduce    fixed-order sum of the backward's per-block partials
//   k_derive    parameter copies in the kernels' register layout
//
// Vectors are spread over lanes as described in layout.hpp; each lane keeps
// 32 elements in VGPRs and butterflies on register bits are lane-local, so
// the transform costs 5 add/sub per element per layout and one LDS round trip
// per change of layout.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "engine.hpp"
#include "launch.hpp"

namespace mck {
namespace {

// ------------------------------------------------------------------ H v
template <int M, bool VEC>
__global__ void __launch_bounds__(Geo<M>::BLOCK) k_fwht(float* __restrict__ data, int64_t batch)
{
    using g = Geo<M>;
    constexpr int K = g::K;
    __shared__ float lds[g::LDS_FLOATS];
    const uint32_t lane = threadIdx.x;
    const uint32_t grp = g::kMulti ? 0u : lane >> g::T;
    const uint32_t t = g::kMulti ? lane : (lane & (g::LPR - 1));
    const int64_t row = (int64_t)blockIdx.x * g::RPB + grp;
    const bool valid = row < batch;
    float* buf = lds + grp * g::STRIDE;
    float* src = data + (valid ? row : 0) * (int64_t)g::n;
    float v[g::EPL];
    load_row<M, VEC>(v, src, g::n, t, valid);
    fwht_up<M>(v, buf, t);
    if constexpr (K >= 1)
        relayout<M, K, 0>(v, buf, t);
    if (valid)
        store_coal<M, VEC>(src, t, v);
}

// ------------------------------------------------------------------ forward
// One block holds RPB rows (one wave) or one row (n >= 4096, several waves).
// For each expansion e: v = B_e xhat; H; Pi gather through LDS fused with the
// G_e product; H; z = S_e v; phi blocks written with float4 stores.
template <int M, bool VEC, bool TRIG>
__global__ void __launch_bounds__(Geo<M>::BLOCK)
    k_forward(const float* __restrict__ x, int64_t batch, int d, int E, const float* __restrict__ B,
              const uint32_t* __restrict__ goff, const float* __restrict__ Gk, const float* __restrict__ Sx,
              FeatCoef coef, float* __restrict__ out)
{
    using g = Geo<M>;
    constexpr int EPL = g::EPL, n = g::n, K = g::K;
    __shared__ float lds[g::LDS_FLOATS];
    const uint32_t lane = threadIdx.x;
    const uint32_t grp = g::kMulti ? 0u : lane >> g::T;
    const uint32_t t = g::kMulti ? lane : (lane & (g::LPR - 1));
    const int64_t row = (int64_t)blockIdx.x * g::RPB + grp;
    const bool valid = row < batch;
    float* buf = lds + grp * g::STRIDE;
    const char* lbytes = reinterpret_cast<const char*>(buf);

    float xh[EPL];
    load_row<M, VEC>(xh, x + (valid ? row : 0) * (int64_t)d, d, t, valid);
    const int64_t nE = (int64_t)n * E;
    float* orow = out + (valid ? row : 0) * (TRIG ? 2 * nE : nE);

    for (int e = 0; e < E; ++e) {
        const int64_t eo = (int64_t)e * n;
        float v[EPL];
        load_param_coal<M>(v, B + eo, t);
#pragma unroll
        for (int r = 0; r < EPL; ++r)
            v[r] *= xh[r];
        fwht_up<M>(v, buf, t);

        // Pi: v1 to LDS in natural order, then gather v1[perm[i]] * G[i]
        lds_put<M, K>(buf, t, v);
        lds_sync<M>();
        uint32_t off[EPL];
        load_lane_major<M, uint32_t>(off, goff + eo, t);
        float gk[EPL];
        load_lane_major<M, float>(gk, Gk + eo, t);
#pragma unroll
        for (int r = 0; r < EPL; ++r)
            v[r] = *reinterpret_cast<const float*>(lbytes + off[r]) * gk[r];
        lds_sync<M>();

        fwht_down<M>(v, buf, t);

        float sx[EPL];
        load_param_coal<M>(sx, Sx + eo, t);
        if constexpr (TRIG) {
            float co[EPL], si[EPL];
#pragma unroll
            for (int r = 0; r < EPL; ++r)
                cossin_hturn(v[r] * sx[r], coef, co[r], si[r]);
            if (valid) {
                store_coal<M, VEC>(orow + eo, t, co);
                store_coal<M, VEC>(orow + nE + eo, t, si);
            }
        } else {
#pragma unroll
            for (int r = 0; r < EPL; ++r)
                v[r] *= sx[r];
            if (valid)
                store_coal<M, VEC>(orow + eo, t, v);
        }
    }
}

// ------------------------------------------------------------------ backward
// Block = NW waves (or one multi-wave row group for n >= 4096).  The loop runs
// over expansions outermost so that the dS, dG, dB contributions of all rows
// a block owns accumulate in VGPRs; at the end of each expansion they are
// summed across the block in a fixed order and written as the block's
// partial.  dx accumulates over expansions in place (each row has one owner).
constexpr int kBwdWaves = 8;

template <int M>
struct BwdGeo {
    static constexpr int NW = Geo<M>::kMulti ? 1 : kBwdWaves;
    static constexpr int THREADS = Geo<M>::BLOCK * NW;
    static constexpr int ROWS = NW * Geo<M>::RPB;  // rows per block per pass
};

template <int M, bool VEC, bool PARAMS>
__global__ void __launch_bounds__(BwdGeo<M>::THREADS)
    k_backward(const float* __restrict__ x, const float* __restrict__ dphi, int64_t batch, int d, int E,
               const float* __restrict__ B, const uint32_t* __restrict__ goff, const float* __restrict__ Gk,
               const float* __restrict__ S32, const float* __restrict__ Sh, FeatCoef coef, float* __restrict__ dx,
               float* __restrict__ partial, int passes)
{
    using g = Geo<M>;
    using bg = BwdGeo<M>;
    constexpr int EPL = g::EPL, n = g::n, K = g::K;
    __shared__ float lds[bg::NW * g::LDS_FLOATS];
    const uint32_t wave = g::kMulti ? 0u : threadIdx.x / 64u;
    const uint32_t lane = g::kMulti ? threadIdx.x : threadIdx.x % 64u;
    const uint32_t grp = g::kMulti ? 0u : lane >> g::T;
    const uint32_t t = g::kMulti ? lane : (lane & (g::LPR - 1));
    float* buf = lds + wave * g::LDS_FLOATS + grp * g::STRIDE;
    const char* lbytes = reinterpret_cast<const char*>(buf);
    const int64_t nE = (int64_t)n * E;
    const uint32_t ct = tpart<M, 0>(t);

    for (int e = 0; e < E; ++e) {
        const int64_t eo = (int64_t)e * n;
        float aS[EPL], aG[EPL], aB[EPL];
        if constexpr (PARAMS) {
#pragma unroll
            for (int r = 0; r < EPL; ++r)
                aS[r] = aG[r] = aB[r] = 0.f;
        }
        for (int p = 0; p < passes; ++p) {
            const int64_t row = ((int64_t)blockIdx.x * passes + p) * bg::ROWS + wave * g::RPB + grp;
            const bool valid = row < batch;
            const float* xr = x + (valid ? row : 0) * (int64_t)d;
            const float* gr = dphi + (valid ? row : 0) * 2 * nE;

            // forward recompute: v1 = H B xhat, w = Pi v1, v3 = H G w
            float v[EPL];
            {
                float xh[EPL];
                load_row<M, VEC>(xh, xr, d, t, valid);
                load_param_coal<M>(v, B + eo, t);
#pragma unroll
                for (int r = 0; r < EPL; ++r)
                    v[r] *= xh[r];
            }
            fwht_up<M>(v, buf, t);
            lds_put<M, K>(buf, t, v);
            lds_sync<M>();
            uint32_t off[EPL];
            load_lane_major<M, uint32_t>(off, goff + eo, t);
            float w[EPL];
#pragma unroll
            for (int r = 0; r < EPL; ++r)
                w[r] = *reinterpret_cast<const float*>(lbytes + off[r]);
            lds_sync<M>();
            {
                float gk[EPL];
                load_lane_major<M, float>(gk, Gk + eo, t);
#pragma unroll
                for (int r = 0; r < EPL; ++r)
                    v[r] = w[r] * gk[r];
            }
            fwht_down<M>(v, buf, t);

            // dz = c (-sin z dphi_cos + cos z dphi_sin); dS += dz v3; g3 = S dz
            {
                float sh[EPL], s32[EPL], gc[EPL], gs[EPL];
                load_param_coal<M>(sh, Sh + eo, t);
                load_param_coal<M>(s32, S32 + eo, t);
                load_row<M, VEC>(gc, gr + eo, n, t, valid);
                load_row<M, VEC>(gs, gr + nE + eo, n, t, valid);
#pragma unroll
                for (int r = 0; r < EPL; ++r) {
                    float co, si;
                    cossin_hturn(v[r] * sh[r], coef, co, si);
                    const float dz = co * gs[r] - si * gc[r];
                    if constexpr (PARAMS)
                        aS[r] += dz * v[r];
                    v[r] = s32[r] * dz;
                }
            }
            // g2 = H g3 (ends in the gather layout); dG += g2 w; Pi^T scatter of G g2
            fwht_up<M>(v, buf, t);
            {
                float gk[EPL];
                load_lane_major<M, float>(gk, Gk + eo, t);
#pragma unroll
                for (int r = 0; r < EPL; ++r) {
                    if constexpr (PARAMS)
                        aG[r] += v[r] * w[r];
                    v[r] *= gk[r];
                }
            }
#pragma unroll
            for (int r = 0; r < EPL; ++r)
                *reinterpret_cast<float*>(reinterpret_cast<char*>(buf) + off[r]) = v[r];
            lds_sync<M>();
            lds_get<M, K>(buf, t, v);
            lds_sync<M>();
            // g0 = H g1 (ends in the coalesced layout); dB += g0 xhat; dx += B g0
            fwht_down<M>(v, buf, t);
            {
                float xh[EPL], bb[EPL];
                load_row<M, VEC>(xh, xr, d, t, valid);
                load_param_coal<M>(bb, B + eo, t);
#pragma unroll
                for (int r = 0; r < EPL; ++r) {
                    if constexpr (PARAMS)
                        aB[r] += v[r] * xh[r];
                    v[r] *= bb[r];
                }
            }
            if (dx != nullptr && valid) {
                float* dr = dx + row * (int64_t)d;
                if constexpr (VEC) {
#pragma unroll
                    for (int j = 0; j < EPL / 4; ++j) {
                        const uint32_t i0 = ct | rpart(M, 0, 4 * j);
                        if ((int)i0 < d) {
                            float4 q = make_float4(v[4 * j], v[4 * j + 1], v[4 * j + 2], v[4 * j + 3]);
                            if (e > 0) {
                                const float4 o = *reinterpret_cast<const float4*>(dr + i0);
                                q.x += o.x; q.y += o.y; q.z += o.z; q.w += o.w;
                            }
                            *reinterpret_cast<float4*>(dr + i0) = q;
                        }
                    }
                } else {
#pragma unroll
                    for (int r = 0; r < EPL; ++r) {
                        const uint32_t i = ct | rpart(M, 0, r);
                        if ((int)i < d)
                            dr[i] = (e > 0) ? dr[i] + v[r] : v[r];
                    }
                }
            }
        }

        if constexpr (PARAMS) {
            // block sum of the three accumulators in slot order (wave, group)
            constexpr int SLOTS = bg::NW * g::RPB;
            float* slot = lds + (wave * g::RPB + grp) * n;
            float* dst = partial + (((int64_t)blockIdx.x * E + e) * 3) * n;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                __syncthreads();
                if (a == 1) {
                    const uint32_t tk = tpart<M, K>(t);
#pragma unroll
                    for (int r = 0; r < EPL; ++r)
                        slot[tk | rpart(M, K, r)] = aG[r];
                } else {
                    const float* acc = a == 0 ? aS : aB;
#pragma unroll
                    for (int r = 0; r < EPL; ++r)
                        slot[ct | rpart(M, 0, r)] = acc[r];
                }
                __syncthreads();
                for (int i = threadIdx.x; i < n; i += bg::THREADS) {
                    float s = 0.f;
                    for (int k = 0; k < SLOTS; ++k)
                        s += lds[k * n + i];
                    dst[(int64_t)a * n + i] = s;
                }
            }
            __syncthreads();
        }
    }
}

// ------------------------------------------------------------------ reduce
__global__ void k_reduce(const float* __restrict__ partial, int64_t blocks, int64_t E, int64_t n,
                         float* __restrict__ dS, float* __restrict__ dG, float* __restrict__ dB)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= 3 * E * n)
        return;
    const int64_t a = idx / (E * n);
    const int64_t rem = idx % (E * n);
    const int64_t e = rem / n, i = rem % n;
    float* out = a == 0 ? dS : (a == 1 ? dG : dB);
    if (out == nullptr)
        return;
    float s = 0.f;
    for (int64_t b = 0; b < blocks; ++b)
        s += partial[((b * E + e) * 3 + a) * n + i];
    out[e * n + i] = s;
}

// ------------------------------------------------------------------ derive
template <int M>
__global__ void k_derive(int64_t E, const int32_t* __restrict__ perm, const float* __restrict__ G,
                         const double* __restrict__ S64, const float* __restrict__ S32, uint32_t* __restrict__ goff,
                         float* __restrict__ Gk, float* __restrict__ Sh)
{
    using g = Geo<M>;
    constexpr int K = g::K, EPL = g::EPL, n = g::n;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= E * n)
        return;
    const int64_t e = idx / n;
    const uint32_t q = (uint32_t)(idx % n);  // lane-major slot: t * EPL + r
    const uint32_t t = q / EPL;
    const int r = (int)(q % EPL);
    const uint32_t i = tpart<M, K>(t) | rpart(M, K, r);
    const uint32_t src = (uint32_t)perm[e * n + i] & (uint32_t)(n - 1);
    goff[idx] = 4u * phys(src);
    Gk[idx] = G[e * n + i];
    // S in half turns for the feature map, from the FP64 value when present
    const double s = S64 ? S64[idx] : (double)S32[idx];
    Sh[idx] = (float)(s * 0.31830988618379067154);
}

// ------------------------------------------------------------------ dispatch
template <template <int> class F, typename... A>
hipError_t dispatch_m(int M, A&&... args)
{
    switch (M) {
    case 1: return F<1>::run(args...);
    case 2: return F<2>::run(args...);
    case 3: return F<3>::run(args...);
    case 4: return F<4>::run(args...);
    case 5: return F<5>::run(args...);
    case 6: return F<6>::run(args...);
    case 7: return F<7>::run(args...);
    case 8: return F<8>::run(args...);
    case 9: return F<9>::run(args...);
    case 10: return F<10>::run(args...);
    case 11: return F<11>::run(args...);
    case 12: return F<12>::run(args...);
    case 13: return F<13>::run(args...);
    case 14: return F<14>::run(args...);
    case 15: return F<15>::run(args...);
    default: return hipErrorInvalidValue;
    }
}

FeatCoef to_dev(const FeatCoefHost& h)
{
    FeatCoef c;
    for (int i = 0; i < 5; ++i) {
        c.s[i] = h.s[i];
        c.c[i] = h.c[i];
    }
    return c;
}

template <int M>
struct RunFwht {
    static hipError_t run(float* data, int64_t batch, bool vec, hipStream_t s)
    {
        using g = Geo<M>;
        const int64_t blocks = (batch + g::RPB - 1) / g::RPB;
        if (vec && M >= 2)
            k_fwht<M, true><<<dim3((unsigned)blocks), dim3(g::BLOCK), 0, s>>>(data, batch);
        else
            k_fwht<M, false><<<dim3((unsigned)blocks), dim3(g::BLOCK), 0, s>>>(data, batch);
        return hipGetLastError();
    }
};

template <int M>
struct RunForward {
    static hipError_t run(bool vec, bool trig, const float* x, int64_t batch, int d, int64_t E, const float* B,
                          const uint32_t* goff, const float* Gk, const float* Sx, const FeatCoef& coef, float* out,
                          hipStream_t s)
    {
        using g = Geo<M>;
        const int64_t blocks = (batch + g::RPB - 1) / g::RPB;
        const dim3 grid((unsigned)blocks), blk(g::BLOCK);
        const int Ei = (int)E;
        if (vec && M >= 2) {
            if (trig)
                k_forward<M, true, true><<<grid, blk, 0, s>>>(x, batch, d, Ei, B, goff, Gk, Sx, coef, out);
            else
                k_forward<M, true, false><<<grid, blk, 0, s>>>(x, batch, d, Ei, B, goff, Gk, Sx, coef, out);
        } else {
            if (trig)
                k_forward<M, false, true><<<grid, blk, 0, s>>>(x, batch, d, Ei, B, goff, Gk, Sx, coef, out);
            else
                k_forward<M, false, false><<<grid, blk, 0, s>>>(x, batch, d, Ei, B, goff, Gk, Sx, coef, out);
        }
        return hipGetLastError();
    }
};

template <int M>
struct RunBackward {
    static hipError_t run(bool vec, const float* x, const float* dphi, int64_t batch, int d, int64_t E,
                          const float* B, const uint32_t* goff, const float* Gk, const float* S32, const float* Sh,
                          const FeatCoef& coef, float* dx, float* partial, const BwdGeometry& geo, hipStream_t s)
    {
        using bg = BwdGeo<M>;
        const dim3 grid((unsigned)geo.blocks), blk(bg::THREADS);
        const int Ei = (int)E;
        if (vec && M >= 2) {
            if (partial)
                k_backward<M, true, true><<<grid, blk, 0, s>>>(x, dphi, batch, d, Ei, B, goff, Gk, S32, Sh, coef,
                                                                dx, partial, geo.passes);
            else
                k_backward<M, true, false><<<grid, blk, 0, s>>>(x, dphi, batch, d, Ei, B, goff, Gk, S32, Sh, coef,
                                                                 dx, partial, geo.passes);
        } else {
            if (partial)
                k_backward<M, false, true><<<grid, blk, 0, s>>>(x, dphi, batch, d, Ei, B, goff, Gk, S32, Sh, coef,
                                                                 dx, partial, geo.passes);
            else
                k_backward<M, false, false><<<grid, blk, 0, s>>>(x, dphi, batch, d, Ei, B, goff, Gk, S32, Sh, coef,
                                                                  dx, partial, geo.passes);
        }
        return hipGetLastError();
    }
};

template <int M>
struct RunGeometry {
    static hipError_t run(int64_t batch, BwdGeometry* out)
    {
        using bg = BwdGeo<M>;
        // about 256 blocks, each owning a contiguous run of rows
        const int64_t units = (batch + bg::ROWS - 1) / bg::ROWS;
        const int64_t target = 256;
        int64_t passes = (units + target - 1) / target;
        if (passes < 1)
            passes = 1;
        out->passes = (int)passes;
        out->blocks = (units + passes - 1) / passes;
        if (out->blocks < 1)
            out->blocks = 1;
        out->block_threads = bg::THREADS;
        return hipSuccess;
    }
};

template <int M>
struct RunDerive {
    static hipError_t run(int64_t E, const int32_t* perm, const float* G, const double* S64, const float* S32,
                          uint32_t* goff, float* Gk, float* Sh, hipStream_t s)
    {
        const int64_t total = E * Geo<M>::n;
        k_derive<M><<<dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s>>>(E, perm, G, S64, S32, goff, Gk, Sh);
        return hipGetLastError();
    }
};

}  // namespace

hipError_t launch_fwht(int M, float* data, int64_t batch, bool vec, hipStream_t s)
{
    return dispatch_m<RunFwht>(M, data, batch, vec, s);
}

hipError_t launch_forward(int M, bool vec, bool trig, const float* x, int64_t batch, int d, int64_t E,
                          const float* B, const uint32_t* goff, const float* Gk, const float* Sx,
                          const FeatCoefHost& coef, float* out, hipStream_t s)
{
    const FeatCoef c = to_dev(coef);
    return dispatch_m<RunForward>(M, vec, trig, x, batch, d, E, B, goff, Gk, Sx, c, out, s);
}

BwdGeometry backward_geometry(int M, int64_t batch)
{
    BwdGeometry g{1, 1, 64};
    (void)dispatch_m<RunGeometry>(M, batch, &g);
    return g;
}

hipError_t launch_backward(int M, bool vec, const float* x, const float* dphi, int64_t batch, int d, int64_t E,
                           const float* B, const uint32_t* goff, const float* Gk, const float* S32,
                           const float* Sh, const FeatCoefHost& coef, float* dx, float* partial,
                           const BwdGeometry& geo, hipStream_t s)
{
    const FeatCoef c = to_dev(coef);
    return dispatch_m<RunBackward>(M, vec, x, dphi, batch, d, E, B, goff, Gk, S32, Sh, c, dx, partial, geo, s);
}

hipError_t launch_reduce(const float* partial, int64_t blocks, int64_t E, int64_t n, float* dS, float* dG,
                         float* dB, hipStream_t s)
{
    const int64_t total = 3 * E * n;
    k_reduce<<<dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s>>>(partial, blocks, E, n, dS, dG, dB);
    return hipGetLastError();
}

hipError_t launch_derive(int M, int64_t E, const int32_t* perm, const float* G, const double* S64, const float* S32,
                         uint32_t* goff, float* Gk, float* Sh, hipStream_t s)
{
    return dispatch_m<RunDerive>(M, E, perm, G, S64, S32, goff, Gk, Sh, s);
}

}  // namespace mck
