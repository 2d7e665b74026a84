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
// register bits per layout: 4 (16 values per lane) up to 2^12; 5 from 2^13,
// where rows span 4 to 16 waves, fewer relayouts win and the packed
// parameters below keep the next expansion's loads ahead of the stores
constexpr int fwd_p(int M) { return M >= 13 ? 5 : 4; }
constexpr int bwd_p(int M) { return M >= 15 ? 5 : 4; }
constexpr int kFwhtP = 5;

// The forward is also compiled with the other register split for
// 2^9 <= n <= 2^14, where both fit (P = 4 stops at 2^14: a 2^15 row would
// need 2048 lanes); the autotuner picks one per n (at 2^14, for instance,
// P = 4 is faster for few expansions per map and P = 5 for many).
constexpr bool fwd_p_tunable(int M) { return M >= 9 && M <= 14; }
constexpr int fwd_p_alt(int M) { return fwd_p(M) == 4 ? 5 : 4; }
constexpr bool fwd_p_ok(int M, int P) { return P == fwd_p(M) || (fwd_p_tunable(M) && P == fwd_p_alt(M)); }

// Where the forward applies G.  At P = 4 (the pipelined forward and the
// training step's tile kernels) G multiplies the gathered values in
// destination order, and the compiler fuses that product into the first
// butterfly of the second transform (one multiply and two multiply-adds
// per pair instead of two multiplies and two adds); at P = 5 G multiplies
// the transformed values in source order before the gather.
constexpr bool fwd_g_after_gather(int P) { return P == 4; }

// With P = 5 the parameters of the next expansion fit in VGPRs beside the
// 32 values per lane only in packed form: B as one sign word per lane and
// the gather sources as 16-bit LDS float indices (two per word).  The packed
// arrays exist for the generated B (+-1); caller-given diagonals take the
// unpacked form without the pipeline.
//   packed goff, per expansion e: RPB n 16-bit indices, lane q's EPL of them
//   at [q EPL, (q + 1) EPL); then, after all E expansions, E x LPR sign
//   words: bit r of word (e, t) is set when B_e is -1 at the element that
//   register r of lane t holds in the coalesced layout.
template <int M, int P>
constexpr int64_t packed_sign_word0(int64_t E) { return E * (int64_t)Geo<M, P>::RPB * Geo<M, P>::n / 2; }

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

// phi (TRIG) or z of expansion e from the transformed v, written from the
// coalesced layout: four features at a time for n >= 4.
template <int M, int P, bool TRIG, int YT>
__device__ __forceinline__ void store_features(rsrc_t rY, uint32_t yoff, int e, uint32_t nE, float cs,
                                               const float (&v)[Geo<M, P>::EPL])
{
    constexpr uint32_t YB = elem_bytes<YT>();
    constexpr int EPL = Geo<M, P>::EPL, n = Geo<M, P>::n;
    if constexpr (TRIG) {
        if constexpr (M >= 2) {
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

// The forward with packed parameters (P = 5, generated B).  x stays in
// VGPRs for the whole chunk; the sign word and the 16-bit gather indices of
// expansion e+1 are loaded before the stores of e, so that e+1 starts its
// first transform while those stores drain (the vector-memory counter is
// shared by loads and stores: a load issued after them cannot be waited for
// until they have completed).  G' is loaded at the start of e and first
// needed after that transform; S is loaded after the gather and first
// needed after the second transform.
template <int M, int P, bool VEC, bool TRIG, int XT, int YT>
__device__ __forceinline__ void forward_packed(rsrc_t rx, rsrc_t rG, rsrc_t rS, rsrc_t rO, rsrc_t rY, uint32_t xoff,
                                               uint32_t yoff, int d, int E, int e0, int e1, uint32_t t,
                                               uint32_t lane, bool valid, uint32_t nE, float cs, float xs,
                                               float* buf, const float* lds)
{
    using g = Geo<M, P>;
    constexpr int EPL = g::EPL, n = g::n, NW = EPL / 2;
    constexpr uint32_t kGoffE = (uint32_t)g::RPB * n;
    const uint32_t sign0 = 4u * (uint32_t)packed_sign_word0<M, P>(E);  // byte offset of the sign words
    float xh[EPL], gs[EPL], sx[EPL];
    uint32_t bw = 0, op[NW];
    auto load_params = [&](int e) {
        bw = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(rO, (int)(4u * t),
                                                            (int)(sign0 + 4u * (uint32_t)e * g::LPR), 0);
#pragma unroll
        for (int j = 0; j < NW / 4; ++j)
            bload4u(&op[4 * j], rO, 4u * NW * lane, 2u * (uint32_t)e * kGoffE + 16u * j);
    };
    bload_row_t<M, P, VEC, XT>(xh, rx, xoff, d, t, valid);
#pragma unroll
    for (int r = 0; r < EPL; ++r)
        xh[r] *= xs;
    load_params(e0);
    for (int e = e0; e < e1; ++e) {
        float v[EPL];
#pragma unroll
        for (int r = 0; r < EPL; ++r)
            v[r] = __uint_as_float(__float_as_uint(xh[r]) ^ ((bw << (31 - r)) & 0x80000000u));
        // G' is first needed after the transform, which overlaps the drain
        // of the previous expansion's stores
        bload_lane<M, P, float>(gs, rG, 4u * (uint32_t)e * n, t);
        fwht_up<M, P>(v, buf, lds_lane<M, P>(t));
#pragma unroll
        for (int r = 0; r < EPL; ++r)
            v[r] *= gs[r];
        lds_put<M, P, g::GL>(buf, lds_lane<M, P>(t), v);
        lds_sync<M, P>();
#pragma unroll
        for (int r = 0; r < EPL; ++r)
            v[r] = lds[(op[r >> 1] >> (16 * (r & 1))) & 0xFFFFu];
        lds_sync<M, P>();
        bload_coal<M, P>(sx, rS, 4u * (uint32_t)e * n, t);
        fwht_down<M, P>(v, buf, lds_lane<M, P>(t));
#pragma unroll
        for (int r = 0; r < EPL; ++r)
            v[r] *= sx[r];
        if (e + 1 < e1)
            load_params(e + 1);
        store_features<M, P, TRIG, YT>(rY, yoff, e, nE, cs, v);
    }
}

// Per expansion e: v = B_e xhat; H; write to LDS; gather v[perm[i]] and scale
// by G_e (fwd_g_after_gather); H; z = S_e v; phi blocks written with float4
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
template <int M, int P, bool VEC, bool TRIG, int XT, int YT, bool PACK>
__device__ __forceinline__ void forward_body(const void* __restrict__ x, uint32_t x_bytes, int64_t batch, int d,
                                             int E, int echunk, int nchunks, const float* __restrict__ B,
                                             const uint32_t* __restrict__ goff, const float* __restrict__ Gs,
                                             const float* __restrict__ Sx, uint32_t par_bytes, uint32_t goff_bytes,
                                             float cs, void* __restrict__ out, uint32_t out_bytes, int64_t blk,
                                             float* lds, const int8_t* __restrict__ xexp = nullptr)
{
    constexpr uint32_t XB = elem_bytes<XT>(), YB = elem_bytes<YT>();
    using g = Geo<M, P>;
    constexpr int EPL = g::EPL, n = g::n, K = g::K;
    constexpr bool PIPE = (P == 4);
    static_assert(!PACK || P == 5, "packed parameters are laid out for 32 values per lane");
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
    // per-row power-of-2 scale of a scaled x (x = stored x * 2^xexp[row]): exact
    const float xs = (xexp != nullptr && valid) ? __builtin_ldexpf(1.f, (int)xexp[row]) : 1.f;
    const uint32_t ooff = valid ? (uint32_t)(row * (TRIG ? 2 * (int64_t)nE : (int64_t)nE)) * YB : kOutOfRange;
    const uint32_t yoff = ooff + YB * tpart<M, P, 0>(t);  // this lane's output base

    if constexpr (PACK) {
        forward_packed<M, P, VEC, TRIG, XT, YT>(rx, rG, rS, rO, rY, xoff, yoff, d, E, e0, e1, t, lane, valid, nE,
                                                 cs, xs, buf, lds);
        return;
    }

    // PIPE: x stays in VGPRs; B, G' and the gather offsets of expansion e+1
    // are loaded before the stores of e.  S is loaded after those stores: it
    // is first needed after the second transform, by when they have drained.
    float xh[EPL], bn[EPL], gs[EPL], sx[EPL];
    uint32_t off[EPL];
    if constexpr (PIPE) {
        bload_row_t<M, P, VEC, XT>(xh, rx, xoff, d, t, valid);
#pragma unroll
        for (int r = 0; r < EPL; ++r)
            xh[r] *= xs;
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
                v[r] *= xn[r] * xs;
        }

        fwht_up<M, P>(v, buf, lds_lane<M, P>(t));
        // without the pipeline (P = 5: 32 values per lane) the gather offsets
        // are loaded only now, which keeps the transform within 128 VGPRs
        // (loaded with the rest they spilled and cost a quarter of the speed)
        if constexpr (!PIPE)
            bload_lane<M, P, uint32_t>(off, rO, 4u * (uint32_t)e * kGoffE, lane);

        // G Pi v1: write v1 to LDS in natural order, gather v1[perm[i]]; G
        // in destination order after the gather (P = 4), or moved to source
        // order before it (Pi (G' v1), P = 5)
        if constexpr (!fwd_g_after_gather(P)) {
#pragma unroll
            for (int r = 0; r < EPL; ++r)
                v[r] *= gs[r];
        }
        lds_put<M, P, g::GL>(buf, lds_lane<M, P>(t), v);
        lds_sync<M, P>();
#pragma unroll
        for (int r = 0; r < EPL; ++r)
            v[r] = *reinterpret_cast<const float*>(lbytes + off[r]);
        lds_sync<M, P>();
        if constexpr (fwd_g_after_gather(P)) {
#pragma unroll
            for (int r = 0; r < EPL; ++r)
                v[r] *= gs[r];
        }
        if constexpr (!PIPE)
            bload_coal<M, P>(sx, rS, eo4, t);

        fwht_down<M, P>(v, buf, lds_lane<M, P>(t));
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
        store_features<M, P, TRIG, YT>(rY, yoff, e, nE, cs, v);
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

template <int M, int P, bool VEC, bool TRIG, int XT = kF32, int YT = kF32, bool PACK = false>
__global__ void __launch_bounds__((Geo<M, P>::BLOCK), (fwd_min_blocks<M, P>()))
    k_forward(const void* __restrict__ x, uint32_t x_bytes, int64_t batch, int d, int E, int echunk, int nchunks,
              const float* __restrict__ B, const uint32_t* __restrict__ goff, const float* __restrict__ Gs,
              const float* __restrict__ Sx, uint32_t par_bytes, uint32_t goff_bytes, float cs,
              void* __restrict__ out, uint32_t out_bytes, const int8_t* __restrict__ xexp)
{
    __shared__ float lds[Geo<M, P>::LDS_FLOATS];
    forward_body<M, P, VEC, TRIG, XT, YT, PACK>(x, x_bytes, batch, d, E, echunk, nchunks, B, goff, Gs, Sx,
                                                par_bytes, goff_bytes, cs, out, out_bytes, blockIdx.x, lds, xexp);
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
    // the maps of a group are generated (seed) maps: packed parameters at P = 5
    forward_body<M, P, VEC, true, kF32, kF32, P == 5>(q.x, q.x_bytes, q.batch, q.d, q.E, q.echunk, q.nchunks, q.B,
                                                      q.goff, q.Gs, q.Sx, q.par_bytes, q.goff_bytes, q.cs, q.out,
                                                      q.out_bytes, b - q.block0, lds);
}


template <int XT, int YT>
struct RunForwardT {
    template <int M>
    struct Run {
    // P: register bits (a compiled split for this n), waves: grid target,
    // packed: goff is a generated map's (packed form at P = 5; no meaning
    // at P = 4)
    // xexp: per-row power-of-2 exponents of a scaled x, or null
    static hipError_t run(int P, int waves, bool packed, bool vec, bool trig, const void* x, int64_t batch, int d,
                          int64_t E, const float* B, const uint32_t* goff, const float* Gs, const float* Sx,
                          float cs, void* out, hipStream_t s, const int8_t* xexp)
    {
        if (P == fwd_p(M))
            return run_p<fwd_p(M)>(waves, packed, vec, trig, x, batch, d, E, B, goff, Gs, Sx, cs, out, s, xexp);
        if constexpr (fwd_p_tunable(M))
            if (P == fwd_p_alt(M))
                return run_p<fwd_p_alt(M)>(waves, packed, vec, trig, x, batch, d, E, B, goff, Gs, Sx, cs, out, s,
                                           xexp);
        return hipErrorInvalidValue;
    }

    template <int P>
    static hipError_t run_p(int waves, bool packed, bool vec, bool trig, const void* x, int64_t batch, int d,
                            int64_t E, const float* B, const uint32_t* goff, const float* Gs, const float* Sx,
                            float cs, void* out, hipStream_t s, const int8_t* xexp)
    {
        constexpr bool kPk = (P == 5);
        if (kPk && !packed && !(XT == kF32 && YT == kF32 && trig))
            return hipErrorInvalidValue;  // unpacked P = 5 only for the FP32 feature map
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
            const int8_t* xe = xexp ? xexp + r0 : nullptr;
#define MCK_FWD_ARGS xs, xb, rows, d, Ei, ec, nc, B, goff, Gs, Sx, par_bytes, goff_bytes, cs, os, ob, xe
            if constexpr (XT == kF32 && YT == kF32) {
                // z (no feature map) only in FP32
                if (kPk && !packed) {
                    // caller-given diagonals at P = 5: no pipeline
                    if (vec && M >= 2)
                        k_forward<M, P, true, true><<<grid, blk, 0, s>>>(MCK_FWD_ARGS);
                    else
                        k_forward<M, P, false, true><<<grid, blk, 0, s>>>(MCK_FWD_ARGS);
                } else if (vec && M >= 2) {
                    if (trig)
                        k_forward<M, P, true, true, kF32, kF32, kPk><<<grid, blk, 0, s>>>(MCK_FWD_ARGS);
                    else
                        k_forward<M, P, true, false, kF32, kF32, kPk><<<grid, blk, 0, s>>>(MCK_FWD_ARGS);
                } else {
                    if (trig)
                        k_forward<M, P, false, true, kF32, kF32, kPk><<<grid, blk, 0, s>>>(MCK_FWD_ARGS);
                    else
                        k_forward<M, P, false, false, kF32, kF32, kPk><<<grid, blk, 0, s>>>(MCK_FWD_ARGS);
                }
            } else {
                if (!trig)
                    return hipErrorInvalidValue;
                if (vec && M >= 2)
                    k_forward<M, P, true, true, XT, YT, kPk><<<grid, blk, 0, s>>>(MCK_FWD_ARGS);
                else
                    k_forward<M, P, false, true, XT, YT, kPk><<<grid, blk, 0, s>>>(MCK_FWD_ARGS);
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
