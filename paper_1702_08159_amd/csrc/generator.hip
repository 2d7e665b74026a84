// generator.hip -- the seed -> (B, Pi, G, S) parameter generator on the GPU.
//
// The paper draws the Fastfood diagonals from a hash instead of storing them
// (section "McKernel": B from hash bits, Pi by a Fisher-Yates shuffle driven by
// the hash, G by Box-Muller on hashed uniforms, C = the RBF calibration).  This
// file implements the project's bit-level definition of that generator (hash =
// MurmurHash3_x86_32 of a 16-byte key; FP32 Box-Muller and FP64 chi(n) built
// from + - * / and sqrt only, fixed evaluation order, no fused multiply-add), so
// the values are reproducible bit for bit by any IEEE implementation of the
// same steps.  Compiled with -ffp-contract=off.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "launch.hpp"

#pragma clang fp contract(off)

namespace mck {
namespace {

constexpr uint32_t kTagB = 0, kTagPi = 1, kTagG = 2, kTagS = 3, kTagMX = 4, kTagMU = 5;

__device__ __forceinline__ uint32_t rotl(uint32_t x, int r) { return (x << r) | (x >> (32 - r)); }

__device__ __forceinline__ uint32_t mix_block(uint32_t h, uint32_t k)
{
    k *= 0xcc9e2d51u;
    k = rotl(k, 15);
    k *= 0x1b873593u;
    h ^= k;
    h = rotl(h, 13);
    return h * 5u + 0xe6546b64u;
}

// MurmurHash3_x86_32 of the little-endian 16-byte key (w0, w1, w2, w3).
__device__ __forceinline__ uint32_t hash4(uint32_t seed, uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3)
{
    uint32_t h = seed;
    h = mix_block(h, w0);
    h = mix_block(h, w1);
    h = mix_block(h, w2);
    h = mix_block(h, w3);
    h ^= 16u;
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

// ln of a positive normal float: exponent split, ln m = 2 atanh(f/(2+f)).
__device__ float ln32(float u)
{
    const uint32_t bits = __float_as_uint(u);
    int k = (int)((bits >> 23) & 0xffu) - 127;
    float m = __uint_as_float((bits & 0x7fffffu) | (127u << 23));
    if (m > 0x1.6a09e6p+0f) {
        m = m * 0.5f;
        k = k + 1;
    }
    const float f = m - 1.0f;
    const float den = 2.0f + f;
    const float s = f / den;
    const float z = s * s;
    float p = 0x1.3b13b2p-4f;
    p = p * z; p = p + 0x1.745d18p-4f;
    p = p * z; p = p + 0x1.c71c72p-4f;
    p = p * z; p = p + 0x1.24924ap-3f;
    p = p * z; p = p + 0x1.99999ap-3f;
    p = p * z; p = p + 0x1.555556p-2f;
    p = p * z; p = p + 1.0f;
    const float s2 = s + s;
    const float lnm = s2 * p;
    const float kf = (float)k;
    const float hi = kf * 0x1.62e3p-1f;
    float lo = kf * 0x1.2fefa4p-17f;
    lo = lo + lnm;
    return hi + lo;
}

// (cos, sin) of 2 pi k / 2^24 for k in [0, 2^24): exact quadrant, Taylor
// polynomials on [-pi/4, pi/4).
__device__ void cs32(uint32_t k24, float& co, float& si)
{
    uint32_t q = (k24 >> 22) & 3u;
    int r = (int)(k24 & 0x3fffffu);
    if (r >= 0x200000) {
        r -= 0x400000;
        q = (q + 1u) & 3u;
    }
    const float f = (float)r * 0x1p-22f;
    const float x = f * 0x1.921fb6p+0f;
    const float z = x * x;
    float ps = 0x1.71de3ap-19f;
    ps = ps * z; ps = ps + -0x1.a01a02p-13f;
    ps = ps * z; ps = ps + 0x1.111112p-7f;
    ps = ps * z; ps = ps + -0x1.555556p-3f;
    ps = ps * z; ps = ps + 1.0f;
    const float sn = x * ps;
    float pc = -0x1.27e4fcp-22f;
    pc = pc * z; pc = pc + 0x1.a01a02p-16f;
    pc = pc * z; pc = pc + -0x1.6c16c2p-10f;
    pc = pc * z; pc = pc + 0x1.555556p-5f;
    pc = pc * z; pc = pc + -0.5f;
    pc = pc * z; pc = pc + 1.0f;
    switch (q) {
    case 0: co = pc; si = sn; break;
    case 1: co = -sn; si = pc; break;
    case 2: co = -pc; si = -sn; break;
    default: co = sn; si = -pc; break;
    }
}

__device__ void boxmuller32(uint32_t a, uint32_t b, float& g0, float& g1)
{
    const float u1 = (float)((a >> 8) + 1u) * 0x1p-24f;
    const float L = ln32(u1);
    const float t = -2.0f * L;
    const float r = __builtin_sqrtf(t);
    float c, s;
    cs32(b >> 8, c, s);
    g0 = r * c;
    g1 = r * s;
}

__device__ double ln64(double v)
{
    const uint64_t bits = (uint64_t)__double_as_longlong(v);
    int k = (int)((bits >> 52) & 0x7ffu) - 1023;
    double m = __longlong_as_double((long long)((bits & 0xfffffffffffffull) | (1023ull << 52)));
    if (m > 0x1.6a09e667f3bcdp+0) {
        m = m * 0.5;
        k = k + 1;
    }
    const double f = m - 1.0;
    const double den = 2.0 + f;
    const double s = f / den;
    const double z = s * s;
    // 1/25, 1/23, ..., 1/3 (nearest doubles), Horner from the innermost term
    const double c[12] = {0x1.47ae147ae147bp-5, 0x1.642c8590b2164p-5, 0x1.8618618618618p-5,
                          0x1.af286bca1af28p-5, 0x1.e1e1e1e1e1e1ep-5, 0x1.1111111111111p-4,
                          0x1.3b13b13b13b14p-4, 0x1.745d1745d1746p-4, 0x1.c71c71c71c71cp-4,
                          0x1.2492492492492p-3, 0x1.999999999999ap-3, 0x1.5555555555555p-2};
    double p = c[0];
#pragma unroll
    for (int i = 1; i < 12; ++i) {
        p = p * z;
        p = p + c[i];
    }
    p = p * z;
    p = p + 1.0;
    const double s2 = s + s;
    const double lnm = s2 * p;
    const double kd = (double)k;
    const double hi = kd * 0x1.62e42fee00000p-1;
    double lo = kd * 0x1.a39ef35793c76p-33;
    lo = lo + lnm;
    return hi + lo;
}

__device__ double cos2pi64(uint32_t h)
{
    uint32_t q = h >> 30;
    long long r = (long long)(h & 0x3fffffffu);
    if (r >= 0x20000000ll) {
        r -= 0x40000000ll;
        q = (q + 1u) & 3u;
    }
    const double f = (double)r * 0x1p-30;
    const double x = f * 0x1.921fb54442d18p+0;
    const double z = x * x;
    // (-1)^k/(2k)!, k = 10..0 and (-1)^k/(2k+1)!, k = 9..0
    const double cc[11] = {0x1.e542ba4020225p-62, -0x1.6827863b97d97p-53, 0x1.ae7f3e733b81fp-45,
                           -0x1.93974a8c07c9dp-37, 0x1.1eed8eff8d898p-29, -0x1.27e4fb7789f5cp-22,
                           0x1.a01a01a01a01ap-16, -0x1.6c16c16c16c17p-10, 0x1.5555555555555p-5,
                           -0x1.0000000000000p-1, 0x1.0000000000000p+0};
    const double sc[10] = {-0x1.2f49b46814157p-57, 0x1.952c77030ad4ap-49, -0x1.ae7f3e733b81fp-41,
                           0x1.6124613a86d09p-33, -0x1.ae64567f544e4p-26, 0x1.71de3a556c734p-19,
                           -0x1.a01a01a01a01ap-13, 0x1.1111111111111p-7, -0x1.5555555555555p-3,
                           0x1.0000000000000p+0};
    double pc = cc[0];
#pragma unroll
    for (int i = 1; i < 11; ++i) {
        pc = pc * z;
        pc = pc + cc[i];
    }
    double ps = sc[0];
#pragma unroll
    for (int i = 1; i < 10; ++i) {
        ps = ps * z;
        ps = ps + sc[i];
    }
    const double sn = x * ps;
    switch (q) {
    case 0: return pc;
    case 1: return -sn;
    case 2: return -pc;
    default: return sn;
    }
}

__device__ double normal64(uint32_t ha, uint32_t hb)
{
    const double u1 = (double)((uint64_t)ha + 1u) * 0x1p-32;
    const double L = ln64(u1);
    const double t = -2.0 * L;
    const double r = __builtin_sqrt(t);
    return r * cos2pi64(hb);
}

// chi(n) radius by Marsaglia-Tsang on Gamma(n/2, 1); 64 attempts.
__device__ double chi_radius(uint32_t seed, uint32_t e, uint32_t j, int64_t n)
{
    const double a = (double)n * 0.5;
    const double dd = a - 0x1.5555555555555p-2;
    const double nine_d = 9.0 * dd;
    const double cc = 1.0 / __builtin_sqrt(nine_d);
    double g = dd;
    for (uint32_t t = 0; t < 64u; ++t) {
        const double x = normal64(hash4(seed, kTagS, e, j, 3u * t), hash4(seed, kTagS, e, j, 3u * t + 1u));
        double y = cc * x;
        y = 1.0 + y;
        if (!(y > 0.0))
            continue;
        double v = y * y;
        v = v * y;
        const uint32_t hu = hash4(seed, kTagS, e, j, 3u * t + 2u);
        const double u = (double)((uint64_t)hu + 1u) * 0x1p-32;
        const double x2 = x * x;
        const double x4 = x2 * x2;
        double w = 0.0331 * x4;
        w = 1.0 - w;
        if (u < w) {
            g = dd * v;
            break;
        }
        const double lhs = ln64(u);
        const double a1 = 0.5 * x2;
        double b1 = 1.0 - v;
        b1 = b1 + ln64(v);
        b1 = dd * b1;
        const double rhs = a1 + b1;
        if (lhs < rhs) {
            g = dd * v;
            break;
        }
    }
    const double two_g = 2.0 * g;
    return __builtin_sqrt(two_g);
}

// B and G: one thread per (e, pair p).
__global__ void k_gen_bg(uint32_t seed, int64_t n, int64_t E, float* __restrict__ B, float* __restrict__ G)
{
    const int64_t half = n / 2;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= half * E)
        return;
    const uint32_t e = (uint32_t)(idx / half);
    const uint32_t p = (uint32_t)(idx % half);
    const uint32_t a = hash4(seed, kTagG, e, p, 0u);
    const uint32_t b = hash4(seed, kTagG, e, p, 1u);
    float g0, g1;
    boxmuller32(a, b, g0, g1);
    const int64_t base = (int64_t)e * n;
    G[base + 2 * p] = g0;
    G[base + 2 * p + 1] = g1;
    const uint32_t k0 = 2u * p;
    const uint32_t w = hash4(seed, kTagB, e, k0 >> 5, 0u);
    B[base + k0] = ((w >> (k0 & 31u)) & 1u) ? -1.0f : 1.0f;
    B[base + k0 + 1] = ((w >> ((k0 + 1u) & 31u)) & 1u) ? -1.0f : 1.0f;
}

constexpr int kPermChunk = 256;

// Fisher-Yates shuffle of expansion e = blockIdx.x.  The draws j_i of a chunk
// of 256 positions are hashed in parallel; one lane performs the swaps in
// order i = n-1 .. 1, on a copy held in LDS when it fits.
__global__ void __launch_bounds__(kPermChunk) k_gen_perm(uint32_t seed, int64_t n, int32_t* __restrict__ perm,
                                                        int use_lds)
{
    extern __shared__ int32_t sh_perm[];
    __shared__ uint32_t draws[kPermChunk];
    const uint32_t e = blockIdx.x;
    int32_t* P = use_lds ? sh_perm : perm + (int64_t)e * n;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x)
        P[i] = (int32_t)i;
    __syncthreads();
    for (int64_t top = n - 1; top >= 1; top -= kPermChunk) {
        const int64_t lo = top - kPermChunk + 1 > 1 ? top - kPermChunk + 1 : 1;
        const int64_t i = top - threadIdx.x;
        if (i >= lo) {
            const uint32_t h = hash4(seed, kTagPi, e, (uint32_t)i, 0u);
            draws[threadIdx.x] = (uint32_t)(((uint64_t)h * (uint64_t)(i + 1)) >> 32);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int64_t ii = top; ii >= lo; --ii) {
                const uint32_t j = draws[top - ii];
                const int32_t tmp = P[ii];
                P[ii] = P[j];
                P[j] = tmp;
            }
        }
        __syncthreads();
    }
    if (use_lds)
        for (int64_t i = threadIdx.x; i < n; i += blockDim.x)
            perm[(int64_t)e * n + i] = P[i];
}

constexpr int kNormThreads = 256;
constexpr int kNormLevels = 24 - 8 + 1;  // n <= 2^24 over 256 lanes

// ||G_e||^2 as the canonical pairwise sum of the squares in index order:
// each lane sums an aligned power-of-two chunk with the same tree (binary
// counter), then the lane sums are combined level by level.
__global__ void __launch_bounds__(kNormThreads) k_gen_norm2(int64_t n, const float* __restrict__ G,
                                                           double* __restrict__ norm2)
{
    __shared__ double part[kNormThreads];
    const int64_t lanes = n < kNormThreads ? n : kNormThreads;
    const int64_t chunk = n / lanes;
    const float* g = G + (int64_t)blockIdx.x * n;
    if ((int64_t)threadIdx.x < lanes) {
        // a chunk of 2^L elements needs levels 0..L; L <= 24 - 8 here
        double stack[kNormLevels];
        const float* c = g + threadIdx.x * chunk;
        for (int64_t k = 0; k < chunk; ++k) {
            double cur = (double)c[k] * (double)c[k];
            int l = 0;
            while ((k >> l) & 1) {
                cur = stack[l] + cur;
                ++l;
            }
            stack[l] = cur;
        }
        int top = 0;
        while ((int64_t(1) << top) < chunk)
            ++top;
        part[threadIdx.x] = stack[top];
    }
    __syncthreads();
    for (int64_t len = lanes; len > 1; len /= 2) {
        double s = 0.0;
        if ((int64_t)threadIdx.x < len / 2)
            s = part[2 * threadIdx.x] + part[2 * threadIdx.x + 1];
        __syncthreads();
        if ((int64_t)threadIdx.x < len / 2)
            part[threadIdx.x] = s;
        __syncthreads();
    }
    if (threadIdx.x == 0)
        norm2[blockIdx.x] = part[0];
}

// RBF-Matern radii (section "Customizing McKernel"): C_jj = the norm of the
// sum of t samples uniform in the unit n-ball, sample i of row j being
// U^(1/n) X/||X|| with X_k = normal64(h(4,e,w,2k), h(4,e,w,2k+1)),
// U = (h(5,e,w,0)+1) 2^-32, w = j t + i; U^(1/n) by log2(n) square roots.
// One block per (e, j); thread k owns the contiguous elements
// [k cnt, (k+1) cnt), so a pairwise sum inside each thread followed by a
// pairwise tree over the threads is the canonical pairwise sum of all n.
constexpr int kMaternThreads = 256;
constexpr int kMaternMaxCnt = 8;  // n <= 2048

__device__ double block_pairwise(double* part, const double* y2, int cnt, int lanes)
{
    double loc[kMaternMaxCnt];
    for (int k = 0; k < cnt; ++k)
        loc[k] = y2[k];
    for (int len = cnt; len > 1; len /= 2)
        for (int i = 0; i < len / 2; ++i)
            loc[i] = loc[2 * i] + loc[2 * i + 1];
    if ((int)threadIdx.x < lanes)
        part[threadIdx.x] = loc[0];
    __syncthreads();
    for (int len = lanes; len > 1; len /= 2) {
        double s = 0.0;
        if ((int)threadIdx.x < len / 2)
            s = part[2 * threadIdx.x] + part[2 * threadIdx.x + 1];
        __syncthreads();
        if ((int)threadIdx.x < len / 2)
            part[threadIdx.x] = s;
        __syncthreads();
    }
    const double r = part[0];
    __syncthreads();  // part is reused by the next call
    return r;
}

__global__ void __launch_bounds__(kMaternThreads)
    k_gen_matern(uint32_t seed, int64_t n, int64_t E, int t, double* __restrict__ radius)
{
    __shared__ double part[kMaternThreads];
    const int64_t e = (int64_t)blockIdx.x / n;
    const int64_t j = (int64_t)blockIdx.x % n;
    const int lanes = n < kMaternThreads ? (int)n : kMaternThreads;
    const int cnt = (int)(n / lanes);
    const bool own = (int)threadIdx.x < lanes;
    const int64_t k0 = (int64_t)threadIdx.x * cnt;
    double x[kMaternMaxCnt], acc[kMaternMaxCnt], y2[kMaternMaxCnt];
    for (int k = 0; k < kMaternMaxCnt; ++k)
        acc[k] = 0.0;
    for (int i = 0; i < t; ++i) {
        const uint32_t w = (uint32_t)(j * t + i);
        for (int k = 0; k < cnt; ++k) {
            const uint32_t kk = own ? (uint32_t)(k0 + k) : 0u;
            x[k] = normal64(hash4(seed, kTagMX, (uint32_t)e, w, 2u * kk), hash4(seed, kTagMX, (uint32_t)e, w, 2u * kk + 1u));
            y2[k] = x[k] * x[k];
        }
        const double nx2 = block_pairwise(part, y2, cnt, lanes);
        const double nx = __builtin_sqrt(nx2);
        double r = (double)((uint64_t)hash4(seed, kTagMU, (uint32_t)e, w, 0u) + 1u) * 0x1p-32;
        for (int64_t len = n; len > 1; len /= 2)
            r = __builtin_sqrt(r);
        const double f = r / nx;
        for (int k = 0; k < cnt; ++k) {
            const double z = f * x[k];
            acc[k] = acc[k] + z;
        }
    }
    for (int k = 0; k < cnt; ++k)
        y2[k] = acc[k] * acc[k];
    const double c2 = block_pairwise(part, y2, cnt, lanes);
    if (threadIdx.x == 0)
        radius[blockIdx.x] = __builtin_sqrt(c2);
}

// S'_j = s_j / ((sigma sqrt n) sqrt ||G_e||^2): one thread per (e, j).  s_j is
// the chi(n) radius, or (radius != null) the precomputed calibration radius,
// which may alias S64 (each thread reads its own entry before writing it).
__global__ void k_gen_s(uint32_t seed, int64_t n, int64_t E, double sigma, const double* __restrict__ norm2,
                        const double* radius, double* S64, float* __restrict__ S32)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * E)
        return;
    const uint32_t e = (uint32_t)(idx / n);
    const uint32_t j = (uint32_t)(idx % n);
    const double s = radius ? radius[idx] : chi_radius(seed, e, j, n);
    double d1 = __builtin_sqrt((double)n);
    d1 = sigma * d1;
    const double d2 = __builtin_sqrt(norm2[e]);
    const double den = d1 * d2;
    const double sp = s / den;
    S64[idx] = sp;
    S32[idx] = (float)sp;
}

// Self-check hook: the FP32 Box-Muller pair for given hash words.
__global__ void k_boxmuller(const uint32_t* __restrict__ a, const uint32_t* __restrict__ b, int64_t count,
                            float* __restrict__ g0, float* __restrict__ g1)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= count)
        return;
    float x, y;
    boxmuller32(a[idx], b[idx], x, y);
    g0[idx] = x;
    g1[idx] = y;
}

}  // namespace

hipError_t launch_generate(uint32_t seed, int64_t n, int64_t E, double sigma, int matern_t, float* B, int32_t* perm,
                           float* G, double* S64, float* S32, double* norm2, hipStream_t s)
{
    if (matern_t > 0 && n > kMaternThreads * kMaternMaxCnt)
        return hipErrorInvalidValue;
    if (n > (int64_t(1) << (kNormLevels - 1 + 8)))
        return hipErrorInvalidValue;  // beyond the pairwise stack of k_gen_norm2
    const int64_t pairs = (n / 2) * E;
    k_gen_bg<<<dim3((unsigned)((pairs + 255) / 256)), dim3(256), 0, s>>>(seed, n, E, B, G);
    const int use_lds = n * 4 <= 128 * 1024 ? 1 : 0;
    if (use_lds && n * 4 > 48 * 1024) {
        hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void*>(k_gen_perm),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)(n * 4));
        if (err != hipSuccess)
            return err;
    }
    k_gen_perm<<<dim3((unsigned)E), dim3(kPermChunk), use_lds ? (size_t)n * 4 : 0, s>>>(seed, n, perm, use_lds);
    k_gen_norm2<<<dim3((unsigned)E), dim3(kNormThreads), 0, s>>>(n, G, norm2);
    const int64_t total = n * E;
    const double* radius = nullptr;
    if (matern_t > 0) {
        // radii into S64, rescaled in place by k_gen_s
        k_gen_matern<<<dim3((unsigned)total), dim3(kMaternThreads), 0, s>>>(seed, n, E, matern_t, S64);
        radius = S64;
    }
    k_gen_s<<<dim3((unsigned)((total + 127) / 128)), dim3(128), 0, s>>>(seed, n, E, sigma, norm2, radius, S64,
                                                                       S32);
    return hipGetLastError();
}

hipError_t launch_boxmuller(const uint32_t* a, const uint32_t* b, int64_t count, float* g0, float* g1,
                            hipStream_t s)
{
    if (count <= 0)
        return hipSuccess;
    k_boxmuller<<<dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s>>>(a, b, count, g0, g1);
    return hipGetLastError();
}

}  // namespace mck
