// forward.hpp -- the fused Fastfood forward kernel (x -> phi or z) and its
// host-side launcher, shared by the FP32 and the 16-bit storage builds, plus
// the constants and the size dispatch the kernel translation units share.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "engine.hpp"

namespace mck {
namespace {

constexpr int kXcds = 8;

// Register bits per layout.  The forward keeps four arrays of the next
// expansion in flight while it stores the current one, which fits the
// 128-VGPR budget of 4 waves per SIMD only at 16 elements per lane; the
// transform kernel has no such pipeline and uses 32.  n = 2^15 needs 32 so
// that one row fits in a 1024-thread workgroup.
// register bits per layout: 4 (16 values per lane) up to 2^13; 5 from 2^14,
// where rows span 8 (2^14) or 16 (2^15) waves and fewer relayouts win
constexpr int fwd_p(int M) { return M >= 14 ? 5 : 4; }
constexpr int bwd_p(int M) { return M >= 15 ? 5 : 4; }
constexpr int kFwhtP = 5;

// The forward is also compiled with the other register split for
// 2^9 <= n <= 2^14, where both fit (P = 4 stops at 2^14: a 2^15 row would
// need 2048 lanes); the autotuner picks one per n.
constexpr bool fwd_p_tunable(int M) { return M >= 9 && M <= 14; }
constexpr int fwd_p_alt(int M) { return fwd_p(M) == 4 ? 5 : 4; }
constexpr bool fwd_p_ok(int M, int P) { return P == fwd_p(M) || (fwd_p_tunable(M) && P == fwd_p_alt(M)); }

// Default grid target of the forward: the expansions are split into chunks
// until the grid holds about this many waves.
constexpr int kFwdWaves = 16384;

// Every buffer range a launch uses stays below 2^31 bytes.
constexpr int64_t kRangeLimit = (int64_t(1) << 31) - 4096;


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


// ------------------------------------------------------------------ forward
// A block holds RPB rows (one wave) or one row (several waves) and a chunk of
// `echunk` expansions.  Blocks are numbered so that all chunks of one row
// group land on the same XCD (blocks are dealt to the 8 XCDs round robin),
// which keeps the row's x in that XCD's L2 for the later chunks.
struct ChunkMap {
    int64_t group;  // row group
    int chunk;      // expansion chunk
};

__device__ __forceinline__ ChunkMap chunk_map(int64_t b, int nchunks)
{
    const int64_t q = b / kXcds;
    ChunkMap m;
    m.chunk = (int)(q % nchunks);
    m.group = (q / nchunks) * kXcds + (b % kXcds);
    return m;
}

// Per expansion e: v = B_e xhat; H; scale by G_e in source order and write to
// LDS; gather v[perm[i]]; H; z = S_e v; phi blocks written with float4
// streaming stores.  On gfx9-family GPUs the vector-memory counter counts
// stores as well as loads, so a load issued after an expansion's 2n-float
// feature stores cannot complete (be waited for) before those stores do.
// With PIPE, all loads of expansion e+1 are therefore issued before the
// stores of e; the stores then drain while e+1 computes.
//
// XT, YT: storage types of x and of the output (kF32, kBF16, kF16); the
// arithmetic is FP32 throughout, 16-bit outputs are rounded to nearest even.
// The body is shared by the plain launch (one map) and the grouped launch
// (many maps of the same n, one descriptor each); `blk` is the block's index
// within its map.
template <int M, int P, bool VEC, bool TRIG, int XT, int YT>
__device__ __forceinline__ void forward_body(const void* __restrict__ x, uint32_t x_bytes, int64_t batch, int d,
                                             int E, int echunk, int nchunks, const float* __restrict__ B,
                                             const uint32_t* __restrict__ goff, const float* __restrict__ Gs,
                                             const float* __restrict__ Sx, uint32_t par_bytes, uint32_t goff_bytes,
                                             float cs, void* __restrict__ out, uint32_t out_bytes, int64_t blk,
                                             float* lds)
{
    constexpr uint32_t XB = elem_bytes<XT>(), YB = elem_bytes<YT>();
    using g = Geo<M, P>;
    constexpr int EPL = g::EPL, n = g::n, K = g::K;
    constexpr bool PIPE = (P == 4);
    const ChunkMap cm = chunk_map(blk, nchunks);
    if (cm.group * g::RPB >= batch)
        return;  // whole block past the end (uniform)
    const uint32_t lane = threadIdx.x;
    const uint32_t grp = g::kMulti ? 0u : lane >> g::T;
    const uint32_t t = g::kMulti ? lane : (lane & (g::LPR - 1));
    const int64_t row = cm.group * g::RPB + grp;
    const bool valid = row < batch;
    const int e0 = cm.chunk * echunk;
    const int e1 = e0 + echunk < E ? e0 + echunk : E;
    float* buf = lds + grp * g::STRIDE;
    const char* lbytes = reinterpret_cast<const char*>(lds);  // gather offsets include the row region
    constexpr uint32_t kGoffE = (uint32_t)g::RPB * n;

    const rsrc_t rx = make_rsrc(x, x_bytes), rB = make_rsrc(B, par_bytes), rG = make_rsrc(Gs, par_bytes);
    const rsrc_t rS = make_rsrc(Sx, par_bytes), rO = make_rsrc(goff, goff_bytes), rY = make_rsrc(out, out_bytes);
    const uint32_t nE = (uint32_t)n * (uint32_t)E;
    const uint32_t xoff = valid ? (uint32_t)(row * d) * XB : 0u;
    const uint32_t ooff = valid ? (uint32_t)(row * (TRIG ? 2 * (int64_t)nE : (int64_t)nE)) * YB : kOutOfRange;
    const uint32_t yoff = ooff + YB * tpart<M, P, 0>(t);  // this lane's output base

    // PIPE: x stays in VGPRs; B, G' and the gather offsets of expansion e+1
    // are loaded before the stores of e.  S is loaded after those stores: it
    // is first needed after the second transform, by when they have drained.
    float xh[EPL], bn[EPL], gs[EPL], sx[EPL];
    uint32_t off[EPL];
    if constexpr (PIPE) {
        bload_row_t<M, P, VEC, XT>(xh, rx, xoff, d, t, valid);
        bload_coal<M, P>(bn, rB, 4u * (uint32_t)e0 * n, t);
        bload_lane<M, P, float>(gs, rG, 4u * (uint32_t)e0 * n, t);
        bload_lane<M, P, uint32_t>(off, rO, 4u * (uint32_t)e0 * kGoffE, lane);
    }

    for (int e = e0; e < e1; ++e) {
        const uint32_t eo4 = 4u * (uint32_t)e * n;
        float v[EPL];
        if constexpr (PIPE) {
#pragma unroll
            for (int r = 0; r < EPL; ++r)
                v[r] = xh[r] * bn[r];
            bload_coal<M, P>(sx, rS, eo4, t);
        } else {
            float xn[EPL];
            bload_row_t<M, P, VEC, XT>(xn, rx, xoff, d, t, valid);
            bload_coal<M, P>(v, rB, eo4, t);
            bload_lane<M, P, float>(gs, rG, eo4, t);
#pragma unroll
            for (int r = 0; r < EPL; ++r)
                v[r] *= xn[r];
        }

        fwht_up<M, P>(v, buf, t);
        // without the pipeline (P = 5: 32 values per lane) the gather offsets
        // are loaded only now, which keeps the transform within 128 VGPRs
        // (loaded with the rest they spilled and cost a quarter of the speed)
        if constexpr (!PIPE)
            bload_lane<M, P, uint32_t>(off, rO, 4u * (uint32_t)e * kGoffE, lane);

        // G Pi v1 = Pi (G' v1) with G' = G in source order: scale, write v1 to
        // LDS in natural order, gather v1[perm[i]]
#pragma unroll
        for (int r = 0; r < EPL; ++r)
            v[r] *= gs[r];
        lds_put<M, P, g::GL>(buf, t, v);
        lds_sync<M, P>();
#pragma unroll
        for (int r = 0; r < EPL; ++r)
            v[r] = *reinterpret_cast<const float*>(lbytes + off[r]);
        lds_sync<M, P>();
        if constexpr (!PIPE)
            bload_coal<M, P>(sx, rS, eo4, t);

        fwht_down<M, P>(v, buf, t);
#pragma unroll
        for (int r = 0; r < EPL; ++r)
            v[r] *= sx[r];

        if constexpr (PIPE) {
            if (e + 1 < e1) {
                const uint32_t en4 = eo4 + 4u * n;
                bload_coal<M, P>(bn, rB, en4, t);
                bload_lane<M, P, float>(gs, rG, en4, t);
                bload_lane<M, P, uint32_t>(off, rO, 4u * (uint32_t)(e + 1) * kGoffE, lane);
            }
        }
        if constexpr (TRIG) {
            if constexpr (M >= 2) {
                // four features at a time, straight to HBM (cos block, sin block)
                const uint32_t yc = yoff + YB * (uint32_t)e * n, ys = yc + YB * nE;
#pragma unroll
                for (int j = 0; j < EPL / 4; ++j) {
                    float c4[4], s4[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        cossin_rev(v[4 * j + k], cs, c4[k], s4[k]);
                    const uint32_t so = YB * rpart(M, P, 0, 4 * j);
                    bstore_quad<YT>(rY, yc + so, c4[0], c4[1], c4[2], c4[3]);
                    bstore_quad<YT>(rY, ys + so, s4[0], s4[1], s4[2], s4[3]);
                }
            } else {
#pragma unroll
                for (int k = 0; k < EPL; ++k) {
                    float c1, s1;
                    cossin_rev(v[k], cs, c1, s1);
                    const uint32_t so = YB * ((uint32_t)e * n + rpart(M, P, 0, k));
                    bstore_elem<YT>(rY, yoff + so, c1);
                    bstore_elem<YT>(rY, yoff + YB * nE + so, s1);
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k < EPL; ++k)
                bstore_elem<YT>(rY, yoff + YB * ((uint32_t)e * n + rpart(M, P, 0, k)), v[k]);
        }
    }
}

// Minimum blocks per CU passed to the compiler: 4 for rows of one wave or
// less; 4 for the 512-lane blocks of n = 2^14, which holds that kernel at
// 128 VGPRs (a hint of 2 gave 129 and three waves per SIMD), so two blocks
// share a CU (their LDS fits); otherwise 1.
template <int M, int P>
constexpr int fwd_min_blocks()
{
    return !Geo<M, P>::kMulti ? 4 : (P == 5 && Geo<M, P>::BLOCK < 1024 ? 4 : 1);
}

template <int M, int P, bool VEC, bool TRIG, int XT = kF32, int YT = kF32>
__global__ void __launch_bounds__((Geo<M, P>::BLOCK), (fwd_min_blocks<M, P>()))
    k_forward(const void* __restrict__ x, uint32_t x_bytes, int64_t batch, int d, int E, int echunk, int nchunks,
              const float* __restrict__ B, const uint32_t* __restrict__ goff, const float* __restrict__ Gs,
              const float* __restrict__ Sx, uint32_t par_bytes, uint32_t goff_bytes, float cs,
              void* __restrict__ out, uint32_t out_bytes)
{
    __shared__ float lds[Geo<M, P>::LDS_FLOATS];
    forward_body<M, P, VEC, TRIG, XT, YT>(x, x_bytes, batch, d, E, echunk, nchunks, B, goff, Gs, Sx, par_bytes,
                                          goff_bytes, cs, out, out_bytes, blockIdx.x, lds);
}

// Grouped launch: up to kGroupMax feature maps of the same n (FP32 x and
// phi) in one grid; map i owns blocks [block0, block0 + blocks) and its
// descriptor travels in the kernel arguments.
constexpr int kGroupMax = 32;

struct FwdDesc {
    const void* x;
    void* out;
    const float* B;
    const uint32_t* goff;
    const float* Gs;
    const float* Sx;
    int64_t batch;
    int64_t block0;
    int d, E, echunk, nchunks;
    uint32_t x_bytes, out_bytes, par_bytes, goff_bytes;
    float cs;
};

struct FwdGroup {
    int count;
    FwdDesc m[kGroupMax];
};

template <int M, int P, bool VEC>
__global__ void __launch_bounds__((Geo<M, P>::BLOCK), (fwd_min_blocks<M, P>())) k_forward_group(FwdGroup grp)
{
    __shared__ float lds[Geo<M, P>::LDS_FLOATS];
    const int64_t b = blockIdx.x;
    int i = 0;
    while (i + 1 < grp.count && grp.m[i + 1].block0 <= b)
        ++i;
    const FwdDesc& q = grp.m[i];
    forward_body<M, P, VEC, true, kF32, kF32>(q.x, q.x_bytes, q.batch, q.d, q.E, q.echunk, q.nchunks, q.B, q.goff,
                                              q.Gs, q.Sx, q.par_bytes, q.goff_bytes, q.cs, q.out, q.out_bytes,
                                              b - q.block0, lds);
}


template <int XT, int YT>
struct RunForwardT {
    template <int M>
    struct Run {
    // P: register bits (a compiled split for this n), waves: grid target
    static hipError_t run(int P, int waves, bool vec, bool trig, const void* x, int64_t batch, int d, int64_t E,
                          const float* B, const uint32_t* goff, const float* Gs, const float* Sx, float cs,
                          void* out, hipStream_t s)
    {
        if (P == fwd_p(M))
            return run_p<fwd_p(M)>(waves, vec, trig, x, batch, d, E, B, goff, Gs, Sx, cs, out, s);
        if constexpr (fwd_p_tunable(M))
            if (P == fwd_p_alt(M))
                return run_p<fwd_p_alt(M)>(waves, vec, trig, x, batch, d, E, B, goff, Gs, Sx, cs, out, s);
        return hipErrorInvalidValue;
    }

    template <int P>
    static hipError_t run_p(int waves, bool vec, bool trig, const void* x, int64_t batch, int d, int64_t E,
                            const float* B, const uint32_t* goff, const float* Gs, const float* Sx, float cs,
                            void* out, hipStream_t s)
    {
        constexpr int64_t XB = elem_bytes<XT>(), YB = elem_bytes<YT>();
        using g = Geo<M, P>;
        const int64_t n = g::n;
        const int64_t out_row = (trig ? 2 : 1) * n * E;
        // rows per launch: keep every buffer range of a launch below 2^31 bytes
        int64_t rows_per = kRangeLimit / (YB * out_row > XB * d ? YB * out_row : XB * d);
        rows_per = rows_per < 1 ? 1 : rows_per;
        const uint32_t par_bytes = (uint32_t)(4 * n * E);
        const uint32_t goff_bytes = (uint32_t)(4 * g::RPB * n * E);
        for (int64_t r0 = 0; r0 < batch; r0 += rows_per) {
            const int64_t rows = batch - r0 < rows_per ? batch - r0 : rows_per;
            const int64_t groups = (rows + g::RPB - 1) / g::RPB;
            // split the expansions so that the grid holds >= `waves` waves
            const int64_t waves_per_group = g::BLOCK / 64;
            int64_t nchunks = (waves + groups * waves_per_group - 1) / (groups * waves_per_group);
            nchunks = nchunks > E ? E : (nchunks < 1 ? 1 : nchunks);
            const int64_t echunk = (E + nchunks - 1) / nchunks;
            nchunks = (E + echunk - 1) / echunk;
            const int64_t blocks = ((groups + kXcds - 1) / kXcds) * kXcds * nchunks;
            const dim3 grid((unsigned)blocks), blk(g::BLOCK);
            const void* xs = static_cast<const char*>(x) + r0 * d * XB;
            void* os = static_cast<char*>(out) + r0 * out_row * YB;
            const uint32_t xb = (uint32_t)(XB * rows * d), ob = (uint32_t)(YB * rows * out_row);
            const int Ei = (int)E, ec = (int)echunk, nc = (int)nchunks;
#define MCK_FWD_ARGS xs, xb, rows, d, Ei, ec, nc, B, goff, Gs, Sx, par_bytes, goff_bytes, cs, os, ob
            if constexpr (XT == kF32 && YT == kF32) {
                // z (no feature map) only in FP32
                if (vec && M >= 2) {
                    if (trig)
                        k_forward<M, P, true, true><<<grid, blk, 0, s>>>(MCK_FWD_ARGS);
                    else
                        k_forward<M, P, true, false><<<grid, blk, 0, s>>>(MCK_FWD_ARGS);
                } else {
                    if (trig)
                        k_forward<M, P, false, true><<<grid, blk, 0, s>>>(MCK_FWD_ARGS);
                    else
                        k_forward<M, P, false, false><<<grid, blk, 0, s>>>(MCK_FWD_ARGS);
                }
            } else {
                if (!trig)
                    return hipErrorInvalidValue;
                if (vec && M >= 2)
                    k_forward<M, P, true, true, XT, YT><<<grid, blk, 0, s>>>(MCK_FWD_ARGS);
                else
                    k_forward<M, P, false, true, XT, YT><<<grid, blk, 0, s>>>(MCK_FWD_ARGS);
            }
#undef MCK_FWD_ARGS
            const hipError_t err = hipGetLastError();
            if (err != hipSuccess)
                return err;
        }
        return hipSuccess;
    }
    };
};

}  // namespace
}  // namespace mck
