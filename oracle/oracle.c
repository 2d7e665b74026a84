/*
 * oracle.c -- plain, slow, FP64 CPU reference of the Fastfood feature map
 * x -> phi(Z x) used by McKernel (Curto et al., "McKernel: A Library for
 * Approximate Kernel Expansions in Log-linear Time").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The product path
 * (the HIP library) never calls it, and the two share no code: this file has
 * its own hash, its own parameter generator and its own transform.
 *
 * What it computes (paper section "McKernel", equations mckernel and
 * mcfeatures; section "Fast Walsh Hadamard"):
 *   xhat = x zero-padded to n = max(2, next power of two >= d)
 *   for each expansion e:  z_e = S_e . H . G_e . Pi_e . H . B_e . xhat
 *   phi = c * [cos z_0 .. cos z_{E-1}, sin z_0 .. sin z_{E-1}],  c = 1/sqrt(nE)
 * where S_e already carries the 1/(sigma sqrt n) prefactor and the
 * 1/||G_e||_F normalisation (the Fastfood scaling).
 *
 * Arithmetic: FP64 throughout, except the parameter generator, whose
 * precision is part of its definition (B, Pi, G are FP32/integer, S is FP64
 * then rounded to FP32 for the FP32 path).  The generator uses only + - * /,
 * sqrt and integer operations, evaluated in a fixed order with no fused
 * multiply-add, so that any IEEE implementation of the same steps reproduces
 * it bit for bit.  Build with -ffp-contract=off.
 *
 * Pins (tests/): FWHT vs scipy's Sylvester Hadamard and the popcount closed
 * form, H.H = nI; hash vs sklearn's murmurhash3_32; ln/sincos vs libm error
 * bounds; Box-Muller closed cases; distribution tests of B, Pi, G, s;
 * RBF-Matern radii (unit-ball samples: radius law r^n, E||Z||^2 = n/(n+2),
 * t = 1 reduces to U^(1/n), E C^2 = t n/(n+2), kernel against an independent
 * Monte Carlo of the same spectral law);
 * row-norm identity of Z; dense n <= 64 product; ||phi|| = 1 and the
 * cos-difference identity; kernel unbiasedness; adjoint dot-product test and
 * finite differences.  No function here is parity-unpinned.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Hash: MurmurHash3_x86_32 (Appleby), the hash the paper names for    */
/* drawing B, Pi and G from a seed (section McKernel, items B, Pi, G). */
/* ------------------------------------------------------------------ */

static uint32_t rotl32(uint32_t x, int r) { return (x << r) | (x >> (32 - r)); }

uint32_t orc_murmur3_x86_32(const void *key, int64_t len, uint32_t seed)
{
    const uint8_t *p = (const uint8_t *)key;
    const uint32_t c1 = 0xcc9e2d51u, c2 = 0x1b873593u;
    uint32_t h = seed;
    int64_t nblocks = len / 4;
    for (int64_t b = 0; b < nblocks; ++b) {
        uint32_t k = (uint32_t)p[4 * b] | ((uint32_t)p[4 * b + 1] << 8) |
                     ((uint32_t)p[4 * b + 2] << 16) | ((uint32_t)p[4 * b + 3] << 24);
        k *= c1;
        k = rotl32(k, 15);
        k *= c2;
        h ^= k;
        h = rotl32(h, 13);
        h = h * 5u + 0xe6546b64u;
    }
    const uint8_t *tail = p + 4 * nblocks;
    uint32_t k = 0;
    switch (len & 3) {
    case 3: k ^= (uint32_t)tail[2] << 16; /* fall through */
    case 2: k ^= (uint32_t)tail[1] << 8;  /* fall through */
    case 1:
        k ^= (uint32_t)tail[0];
        k *= c1;
        k = rotl32(k, 15);
        k *= c2;
        h ^= k;
    }
    h ^= (uint32_t)len;
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

/* h(w0,w1,w2,w3): the 16-byte little-endian key (w0|w1|w2|w3). */
uint32_t orc_hash4(uint32_t seed, uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3)
{
    uint8_t key[16];
    uint32_t w[4] = {w0, w1, w2, w3};
    for (int i = 0; i < 4; ++i) {
        key[4 * i + 0] = (uint8_t)(w[i]);
        key[4 * i + 1] = (uint8_t)(w[i] >> 8);
        key[4 * i + 2] = (uint8_t)(w[i] >> 16);
        key[4 * i + 3] = (uint8_t)(w[i] >> 24);
    }
    return orc_murmur3_x86_32(key, 16, seed);
}

enum { TAG_B = 0, TAG_PI = 1, TAG_G = 2, TAG_S = 3, TAG_MX = 4, TAG_MU = 5 };

/* ------------------------------------------------------------------ */
/* Elementary functions of the generator, built from + - * / only.     */
/* ------------------------------------------------------------------ */

/* Natural log in FP32 of a positive normal float u.
 * u = m * 2^k with m in (sqrt(1/2), sqrt 2]; ln m = 2 atanh(s), s = f/(2+f),
 * f = m - 1; the odd series is summed to s^13. */
float orc_ln32(float u)
{
    uint32_t bits;
    memcpy(&bits, &u, 4);
    int k = (int)((bits >> 23) & 0xffu) - 127;
    uint32_t mb = (bits & 0x7fffffu) | (127u << 23);
    float m;
    memcpy(&m, &mb, 4);
    if (m > 0x1.6a09e6p+0f) {
        m = m * 0.5f;
        k = k + 1;
    }
    float f = m - 1.0f;
    float den = 2.0f + f;
    float s = f / den;
    float z = s * s;
    float p = 0x1.3b13b2p-4f;           /* 1/13 */
    p = p * z; p = p + 0x1.745d18p-4f;  /* 1/11 */
    p = p * z; p = p + 0x1.c71c72p-4f;  /* 1/9 */
    p = p * z; p = p + 0x1.24924ap-3f;  /* 1/7 */
    p = p * z; p = p + 0x1.99999ap-3f;  /* 1/5 */
    p = p * z; p = p + 0x1.555556p-2f;  /* 1/3 */
    p = p * z; p = p + 1.0f;
    float s2 = s + s;
    float lnm = s2 * p;
    float kf = (float)k;
    float hi = kf * 0x1.62e3p-1f;       /* ln2 high part, exact product */
    float lo = kf * 0x1.2fefa4p-17f;    /* ln2 low part */
    lo = lo + lnm;
    return hi + lo;
}

/* cos and sin of 2*pi*k/2^24 in FP32 for an integer k in [0, 2^24).
 * The quadrant is taken exactly from the top two bits; the remainder is an
 * angle in [-pi/4, pi/4) where Taylor polynomials to x^9 / x^10 are used. */
void orc_sincos2pi32(uint32_t k24, float *c_out, float *s_out)
{
    uint32_t q = (k24 >> 22) & 3u;
    int32_t r = (int32_t)(k24 & 0x3fffffu);
    if (r >= 0x200000) {
        r -= 0x400000;
        q = (q + 1u) & 3u;
    }
    float f = (float)r * 0x1p-22f;
    float x = f * 0x1.921fb6p+0f; /* pi/2 */
    float z = x * x;
    float ps = 0x1.71de3ap-19f;               /* 1/9! */
    ps = ps * z; ps = ps + -0x1.a01a02p-13f;  /* -1/7! */
    ps = ps * z; ps = ps + 0x1.111112p-7f;    /* 1/5! */
    ps = ps * z; ps = ps + -0x1.555556p-3f;   /* -1/3! */
    ps = ps * z; ps = ps + 1.0f;
    float sn = x * ps;
    float pc = -0x1.27e4fcp-22f;              /* -1/10! */
    pc = pc * z; pc = pc + 0x1.a01a02p-16f;   /* 1/8! */
    pc = pc * z; pc = pc + -0x1.6c16c2p-10f;  /* -1/6! */
    pc = pc * z; pc = pc + 0x1.555556p-5f;    /* 1/4! */
    pc = pc * z; pc = pc + -0.5f;
    pc = pc * z; pc = pc + 1.0f;
    float cs = pc;
    float co, si;
    switch (q) {
    case 0: co = cs; si = sn; break;
    case 1: co = -sn; si = cs; break;
    case 2: co = -cs; si = -sn; break;
    default: co = sn; si = -cs; break;
    }
    *c_out = co;
    *s_out = si;
}

/* Box-Muller in FP32 from two hash words (section McKernel, item G):
 * u1 = ((a>>8)+1)/2^24 in (0,1], angle = 2 pi (b>>8)/2^24. */
void orc_boxmuller32(uint32_t a, uint32_t b, float *g0, float *g1)
{
    float u1 = (float)((a >> 8) + 1u) * 0x1p-24f;
    float L = orc_ln32(u1);
    float t = -2.0f * L;
    float r = sqrtf(t);
    float c, s;
    orc_sincos2pi32(b >> 8, &c, &s);
    *g0 = r * c;
    *g1 = r * s;
}

void orc_boxmuller32_many(const uint32_t *a, const uint32_t *b, int64_t count, float *g0, float *g1)
{
    for (int64_t k = 0; k < count; ++k)
        orc_boxmuller32(a[k], b[k], &g0[k], &g1[k]);
}

/* Natural log in FP64 of a positive normal double; series to s^25. */
double orc_ln64(double v)
{
    uint64_t bits;
    memcpy(&bits, &v, 8);
    int k = (int)((bits >> 52) & 0x7ffu) - 1023;
    uint64_t mb = (bits & 0xfffffffffffffull) | (1023ull << 52);
    double m;
    memcpy(&m, &mb, 8);
    if (m > 0x1.6a09e667f3bcdp+0) {
        m = m * 0.5;
        k = k + 1;
    }
    double f = m - 1.0;
    double den = 2.0 + f;
    double s = f / den;
    double z = s * s;
    static const double inv_odd[12] = {
        0x1.5555555555555p-2, 0x1.999999999999ap-3, 0x1.2492492492492p-3,
        0x1.c71c71c71c71cp-4, 0x1.745d1745d1746p-4, 0x1.3b13b13b13b14p-4,
        0x1.1111111111111p-4, 0x1.e1e1e1e1e1e1ep-5, 0x1.af286bca1af28p-5,
        0x1.8618618618618p-5, 0x1.642c8590b2164p-5, 0x1.47ae147ae147bp-5};
    /* inv_odd[i] = 1/(2i+3) */
    double p = inv_odd[11];
    for (int i = 10; i >= 0; --i) {
        p = p * z;
        p = p + inv_odd[i];
    }
    p = p * z;
    p = p + 1.0;
    double s2 = s + s;
    double lnm = s2 * p;
    double kd = (double)k;
    double hi = kd * 0x1.62e42fee00000p-1;
    double lo = kd * 0x1.a39ef35793c76p-33;
    lo = lo + lnm;
    return hi + lo;
}

/* cos(2 pi h / 2^32) in FP64 for a 32-bit integer h; Taylor to x^20. */
double orc_cos2pi64(uint32_t h)
{
    uint32_t q = h >> 30;
    int64_t r = (int64_t)(h & 0x3fffffffu);
    if (r >= 0x20000000) {
        r -= 0x40000000;
        q = (q + 1u) & 3u;
    }
    double f = (double)r * 0x1p-30;
    double x = f * 0x1.921fb54442d18p+0;
    double z = x * x;
    static const double cc[11] = {
        0x1.0000000000000p+0, -0x1.0000000000000p-1, 0x1.5555555555555p-5,
        -0x1.6c16c16c16c17p-10, 0x1.a01a01a01a01ap-16, -0x1.27e4fb7789f5cp-22,
        0x1.1eed8eff8d898p-29, -0x1.93974a8c07c9dp-37, 0x1.ae7f3e733b81fp-45,
        -0x1.6827863b97d97p-53, 0x1.e542ba4020225p-62};
    static const double sc[10] = {
        0x1.0000000000000p+0, -0x1.5555555555555p-3, 0x1.1111111111111p-7,
        -0x1.a01a01a01a01ap-13, 0x1.71de3a556c734p-19, -0x1.ae64567f544e4p-26,
        0x1.6124613a86d09p-33, -0x1.ae7f3e733b81fp-41, 0x1.952c77030ad4ap-49,
        -0x1.2f49b46814157p-57};
    double pc = cc[10];
    for (int i = 9; i >= 0; --i) {
        pc = pc * z;
        pc = pc + cc[i];
    }
    double ps = sc[9];
    for (int i = 8; i >= 0; --i) {
        ps = ps * z;
        ps = ps + sc[i];
    }
    double sn = x * ps;
    switch (q) {
    case 0: return pc;
    case 1: return -sn;
    case 2: return -pc;
    default: return sn;
    }
}

/* Standard normal in FP64 by Box-Muller (cosine branch) from two hash words. */
double orc_normal64(uint32_t ha, uint32_t hb)
{
    double u1 = (double)((uint64_t)ha + 1u) * 0x1p-32;
    double L = orc_ln64(u1);
    double t = -2.0 * L;
    double r = sqrt(t);
    return r * orc_cos2pi64(hb);
}

#define ORC_MT_MAX_TRIES 64

/* s ~ chi(n) for row j of expansion e: s = sqrt(2 g), g ~ Gamma(n/2, 1)
 * drawn by Marsaglia and Tsang's squeeze/rejection method; attempt t uses the
 * hash words h(3,e,j,3t), h(3,e,j,3t+1) for the normal and h(3,e,j,3t+2) for
 * the acceptance uniform.  This is the RBF calibration C (section McKernel,
 * item C): the norm of an n-dimensional standard Gaussian vector. */
double orc_chi(uint32_t seed, int64_t e, int64_t j, int64_t n)
{
    double a = (double)n * 0.5;
    double dd = a - 0x1.5555555555555p-2; /* a - 1/3 */
    double nine_d = 9.0 * dd;
    double cc = 1.0 / sqrt(nine_d);
    double g = dd;
    for (uint32_t t = 0; t < ORC_MT_MAX_TRIES; ++t) {
        double x = orc_normal64(orc_hash4(seed, TAG_S, (uint32_t)e, (uint32_t)j, 3u * t),
                                orc_hash4(seed, TAG_S, (uint32_t)e, (uint32_t)j, 3u * t + 1u));
        double y = cc * x;
        y = 1.0 + y;
        if (!(y > 0.0))
            continue;
        double v = y * y;
        v = v * y;
        uint32_t hu = orc_hash4(seed, TAG_S, (uint32_t)e, (uint32_t)j, 3u * t + 2u);
        double u = (double)((uint64_t)hu + 1u) * 0x1p-32;
        double x2 = x * x;
        double x4 = x2 * x2;
        double w = 0.0331 * x4;
        w = 1.0 - w;
        if (u < w) {
            g = dd * v;
            break;
        }
        double lhs = orc_ln64(u);
        double a1 = 0.5 * x2;
        double b1 = 1.0 - v;
        b1 = b1 + orc_ln64(v);
        b1 = dd * b1;
        double rhs = a1 + b1;
        if (lhs < rhs) {
            g = dd * v;
            break;
        }
    }
    double two_g = 2.0 * g;
    return sqrt(two_g);
}

/* ------------------------------------------------------------------ */
/* Parameters B, Pi, G, S of every expansion (section McKernel).       */
/* ------------------------------------------------------------------ */

int64_t orc_padded_dim(int64_t d)
{
    int64_t n = 2;
    while (n < d)
        n *= 2;
    return n;
}

static int is_pow2(int64_t n) { return n >= 1 && (n & (n - 1)) == 0; }

/* Canonical pairwise (binary tree, index order) sum of squares in FP64. */
static double pairwise_sumsq(const float *g, int64_t n)
{
    double *y = (double *)malloc((size_t)n * sizeof(double));
    for (int64_t k = 0; k < n; ++k)
        y[k] = (double)g[k] * (double)g[k];
    for (int64_t len = n; len > 1; len /= 2)
        for (int64_t i = 0; i < len / 2; ++i)
            y[i] = y[2 * i] + y[2 * i + 1];
    double r = y[0];
    free(y);
    return r;
}

/* Canonical pairwise sum of squares of FP64 values (same tree as above). */
static double pairwise_sumsq64(const double *v, int64_t n)
{
    double *y = (double *)malloc((size_t)n * sizeof(double));
    for (int64_t k = 0; k < n; ++k)
        y[k] = v[k] * v[k];
    for (int64_t len = n; len > 1; len /= 2)
        for (int64_t i = 0; i < len / 2; ++i)
            y[i] = y[2 * i] + y[2 * i + 1];
    double r = y[0];
    free(y);
    return r;
}

/* One sample uniform in the unit n-ball (section "Customizing McKernel"):
 * Z = U^(1/n) X / ||X|| with X ~ N(0, I_n) and U ~ U(0, 1].  Sample `w` of
 * expansion e draws X_k = normal64(h(4,e,w,2k), h(4,e,w,2k+1)) and
 * U = (h(5,e,w,0) + 1) 2^-32; U^(1/n) is taken as log2(n) square roots
 * (n = 2^m), ||X||^2 as the canonical pairwise sum.  Writes Z to z. */
void orc_ball_sample(uint32_t seed, int64_t e, uint32_t w, int64_t n, double *z)
{
    for (int64_t k = 0; k < n; ++k)
        z[k] = orc_normal64(orc_hash4(seed, TAG_MX, (uint32_t)e, w, (uint32_t)(2 * k)),
                            orc_hash4(seed, TAG_MX, (uint32_t)e, w, (uint32_t)(2 * k + 1)));
    double nx2 = pairwise_sumsq64(z, n);
    double nx = sqrt(nx2);
    uint32_t hu = orc_hash4(seed, TAG_MU, (uint32_t)e, w, 0u);
    double r = (double)((uint64_t)hu + 1u) * 0x1p-32;
    for (int64_t len = n; len > 1; len /= 2)
        r = sqrt(r);
    double f = r / nx;
    for (int64_t k = 0; k < n; ++k)
        z[k] = f * z[k];
}

/* RBF-Matern calibration C_jj (section "Customizing McKernel"): the
 * Euclidean norm of the sum of t i.i.d. samples uniform in the unit n-ball;
 * sample i of row j is orc_ball_sample with w = j t + i, summed in order
 * i = 0..t-1, and the norm uses the canonical pairwise sum. */
double orc_matern(uint32_t seed, int64_t e, int64_t j, int64_t n, int64_t t)
{
    double *z = (double *)malloc((size_t)n * sizeof(double));
    double *acc = (double *)calloc((size_t)n, sizeof(double));
    for (int64_t i = 0; i < t; ++i) {
        orc_ball_sample(seed, e, (uint32_t)(j * t + i), n, z);
        for (int64_t k = 0; k < n; ++k)
            acc[k] = acc[k] + z[k];
    }
    double c2 = pairwise_sumsq64(acc, n);
    free(z);
    free(acc);
    return sqrt(c2);
}

/* Every output is E x n, row-major by expansion.  S64 is the FP64 diagonal
 * S'_j = s_j / (sigma sqrt(n) ||G||_F); S32 its round-to-nearest FP32 value.
 * s_j is the calibration radius: chi(n) for the RBF kernel (matern_t = 0),
 * or the RBF-Matern norm of a sum of matern_t unit-ball samples.
 * chi (optional) receives s_j; norm2 (optional, length E) ||G_e||_F^2. */
int orc_params_c(uint32_t seed, int64_t n, int64_t E, double sigma, int64_t matern_t,
                 float *B, int32_t *perm, float *G, double *S64, float *S32,
                 double *chi, double *norm2);

int orc_params(uint32_t seed, int64_t n, int64_t E, double sigma,
               float *B, int32_t *perm, float *G, double *S64, float *S32,
               double *chi, double *norm2)
{
    return orc_params_c(seed, n, E, sigma, 0, B, perm, G, S64, S32, chi, norm2);
}

int orc_params_c(uint32_t seed, int64_t n, int64_t E, double sigma, int64_t matern_t,
                 float *B, int32_t *perm, float *G, double *S64, float *S32,
                 double *chi, double *norm2)
{
    if (!is_pow2(n) || n < 2 || E < 1 || !(sigma > 0.0) || !isfinite(sigma) || matern_t < 0 ||
        matern_t > 255)
        return 1;
    for (int64_t e = 0; e < E; ++e) {
        float *Be = B + e * n;
        int32_t *Pe = perm + e * n;
        float *Ge = G + e * n;
        /* B: one hash word per 32 entries; a set bit means -1. */
        for (int64_t k = 0; k < n; ++k) {
            uint32_t w = orc_hash4(seed, TAG_B, (uint32_t)e, (uint32_t)(k >> 5), 0u);
            Be[k] = ((w >> (k & 31)) & 1u) ? -1.0f : 1.0f;
        }
        /* Pi: Fisher-Yates; position i takes a uniformly chosen element
         * among positions 0..i and the displaced one moves to its place. */
        for (int64_t i = 0; i < n; ++i)
            Pe[i] = (int32_t)i;
        for (int64_t i = n - 1; i >= 1; --i) {
            uint32_t w = orc_hash4(seed, TAG_PI, (uint32_t)e, (uint32_t)i, 0u);
            uint32_t j = (uint32_t)(((uint64_t)w * (uint64_t)(i + 1)) >> 32);
            int32_t tmp = Pe[i];
            Pe[i] = Pe[j];
            Pe[j] = tmp;
        }
        /* G: Box-Muller pairs. */
        for (int64_t p = 0; p < n / 2; ++p) {
            uint32_t a = orc_hash4(seed, TAG_G, (uint32_t)e, (uint32_t)p, 0u);
            uint32_t b = orc_hash4(seed, TAG_G, (uint32_t)e, (uint32_t)p, 1u);
            orc_boxmuller32(a, b, &Ge[2 * p], &Ge[2 * p + 1]);
        }
        /* S: chi(n) radii normalised by ||G||_F and 1/(sigma sqrt n). */
        double nrm2 = pairwise_sumsq(Ge, n);
        if (norm2)
            norm2[e] = nrm2;
        double d1 = sqrt((double)n);
        d1 = sigma * d1;
        double d2 = sqrt(nrm2);
        double den = d1 * d2;
        for (int64_t j = 0; j < n; ++j) {
            double s = matern_t > 0 ? orc_matern(seed, e, j, n, matern_t) : orc_chi(seed, e, j, n);
            if (chi)
                chi[e * n + j] = s;
            double sp = s / den;
            if (S64)
                S64[e * n + j] = sp;
            if (S32)
                S32[e * n + j] = (float)sp;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Walsh-Hadamard transform (section "Fast Walsh Hadamard"):           */
/* H_0 = [1];  H_n c = [H_{n-1} c0 + H_{n-1} c1 ; H_{n-1} c0 - H_{n-1} c1] */
/* computed by the divide-and-conquer recursion, in place.             */
/* ------------------------------------------------------------------ */

static void fwht_rec(double *c, int64_t len)
{
    if (len <= 1)
        return;
    int64_t h = len / 2;
    fwht_rec(c, h);
    fwht_rec(c + h, h);
    for (int64_t i = 0; i < h; ++i) {
        double a = c[i], b = c[i + h];
        c[i] = a + b;
        c[i + h] = a - b;
    }
}

int orc_fwht(double *v, int64_t batch, int64_t n)
{
    if (!is_pow2(n) || batch < 0)
        return 1;
    for (int64_t r = 0; r < batch; ++r)
        fwht_rec(v + r * n, n);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Forward: z = S . H . G . Pi . H . B . xhat for each expansion.      */
/* Explicit FP64 parameters (E x n each); perm is the gather           */
/* (Pi v)_i = v[perm[i]].  z is batch x (E n), expansion-major.        */
/* ------------------------------------------------------------------ */

int orc_project(const double *x, int64_t batch, int64_t d, int64_t n, int64_t E,
                const double *B, const int32_t *perm, const double *G,
                const double *S, double *z)
{
    if (!is_pow2(n) || d < 1 || d > n || E < 1 || batch < 0)
        return 1;
    double *v = (double *)malloc((size_t)n * sizeof(double));
    double *w = (double *)malloc((size_t)n * sizeof(double));
    for (int64_t r = 0; r < batch; ++r) {
        const double *xr = x + r * d;
        for (int64_t e = 0; e < E; ++e) {
            const double *Be = B + e * n, *Ge = G + e * n, *Se = S + e * n;
            const int32_t *Pe = perm + e * n;
            for (int64_t i = 0; i < n; ++i)
                v[i] = (i < d) ? Be[i] * xr[i] : 0.0;
            fwht_rec(v, n);
            for (int64_t i = 0; i < n; ++i)
                w[i] = Ge[i] * v[Pe[i]];
            fwht_rec(w, n);
            double *ze = z + r * n * E + e * n;
            for (int64_t i = 0; i < n; ++i)
                ze[i] = Se[i] * w[i];
        }
    }
    free(v);
    free(w);
    return 0;
}

/* phi = c [cos z, sin z], c = 1/sqrt(nE); layout per row: E cos blocks
 * followed by E sin blocks (equation mcfeatures). */
int orc_features(const double *z, int64_t batch, int64_t n, int64_t E, double *phi)
{
    if (n < 1 || E < 1 || batch < 0)
        return 1;
    double c = 1.0 / sqrt((double)n * (double)E);
    int64_t m = n * E;
    for (int64_t r = 0; r < batch; ++r)
        for (int64_t k = 0; k < m; ++k) {
            double zz = z[r * m + k];
            phi[r * 2 * m + k] = c * cos(zz);
            phi[r * 2 * m + m + k] = c * sin(zz);
        }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Adjoint of phi(Z x) with respect to x and to the diagonals B, G, S. */
/* Each of B, G, S is treated as a free real diagonal.  H is symmetric,*/
/* Pi^T is the scatter g[perm[i]] = v_i.  dB, dG, dS are summed over   */
/* the batch; dx drops the padded coordinates.  Null outputs skipped.  */
/* ------------------------------------------------------------------ */

int orc_backward(const double *x, const double *dphi, int64_t batch, int64_t d,
                 int64_t n, int64_t E, const double *B, const int32_t *perm,
                 const double *G, const double *S, double *dx, double *dB,
                 double *dG, double *dS)
{
    if (!is_pow2(n) || d < 1 || d > n || E < 1 || batch < 0)
        return 1;
    double c = 1.0 / sqrt((double)n * (double)E);
    int64_t m = n * E;
    double *xh = (double *)malloc((size_t)n * sizeof(double));
    double *v1 = (double *)malloc((size_t)n * sizeof(double));
    double *w = (double *)malloc((size_t)n * sizeof(double));
    double *v3 = (double *)malloc((size_t)n * sizeof(double));
    double *g = (double *)malloc((size_t)n * sizeof(double));
    double *g1 = (double *)malloc((size_t)n * sizeof(double));
    double *gx = (double *)malloc((size_t)n * sizeof(double));
    if (dB) memset(dB, 0, (size_t)m * sizeof(double));
    if (dG) memset(dG, 0, (size_t)m * sizeof(double));
    if (dS) memset(dS, 0, (size_t)m * sizeof(double));
    for (int64_t r = 0; r < batch; ++r) {
        const double *xr = x + r * d;
        for (int64_t i = 0; i < n; ++i) {
            xh[i] = (i < d) ? xr[i] : 0.0;
            gx[i] = 0.0;
        }
        for (int64_t e = 0; e < E; ++e) {
            const double *Be = B + e * n, *Ge = G + e * n, *Se = S + e * n;
            const int32_t *Pe = perm + e * n;
            const double *gc = dphi + r * 2 * m + e * n;
            const double *gs = dphi + r * 2 * m + m + e * n;
            /* forward, keeping what the adjoint needs */
            for (int64_t i = 0; i < n; ++i)
                v1[i] = Be[i] * xh[i];
            fwht_rec(v1, n);
            for (int64_t i = 0; i < n; ++i)
                w[i] = v1[Pe[i]];
            for (int64_t i = 0; i < n; ++i)
                v3[i] = Ge[i] * w[i];
            fwht_rec(v3, n);
            /* d phi / d z, then back through S, H, G, Pi, H, B */
            for (int64_t i = 0; i < n; ++i) {
                double zz = Se[i] * v3[i];
                double gz = c * (-sin(zz) * gc[i] + cos(zz) * gs[i]);
                if (dS)
                    dS[e * n + i] += gz * v3[i];
                g[i] = Se[i] * gz;
            }
            fwht_rec(g, n);
            for (int64_t i = 0; i < n; ++i) {
                if (dG)
                    dG[e * n + i] += g[i] * w[i];
                g1[Pe[i]] = Ge[i] * g[i];
            }
            fwht_rec(g1, n);
            for (int64_t i = 0; i < n; ++i) {
                if (dB)
                    dB[e * n + i] += g1[i] * xh[i];
                gx[i] += Be[i] * g1[i];
            }
        }
        if (dx)
            for (int64_t i = 0; i < d; ++i)
                dx[r * d + i] = gx[i];
    }
    free(xh); free(v1); free(w); free(v3); free(g); free(g1); free(gx);
    return 0;
}
