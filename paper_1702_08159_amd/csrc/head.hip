// head.hip -- the linear classifier trained on the McKernel features
// (section "Empirical Analysis and Experiments": softmax(W phi + b) with
// cross-entropy; section "Large-scale Machine Learning": minimised by SGD).
//
//   k_softmax_xent  per row: loss_r = log sum_c exp(l_rc) - l_r,y and the
//                   gradient of the mean loss, (softmax(l_r) - onehot(y)) / batch
//   k_head_sums     fixed-order sums over rows: the mean loss and db
//   k_axpy          y += alpha x (the SGD update with alpha = -learning rate)
//   k_axpy_multi    the same over up to 8 arrays in one launch (W, b, B, G, S)
//   k_fill_i8       fills an int8 array (the per-row exponents of a scaled phi)
//   k_head_logits   logits = phi W^T + b for C <= 16 classes: the W rows of a
//                   column live in VGPRs, phi streams once from HBM
//   k_head_bwd      dphi = dlogits W and per-row-group partials of
//                   dW = dlogits^T phi (one pass over phi)
//   k_sum_groups    the row-group partials summed in a fixed order
// The products are skinny (C rows against 2nE columns), so each is one
// streaming pass over phi rather than a GEMM tiling; every sum has a fixed
// order, so the results are deterministic.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "engine.hpp"
#include "launch.hpp"

namespace mck {
namespace {

constexpr int kHeadThreads = 256;

// One thread per row; C is small (tens of classes).  A label outside
// [0, C) makes that row's loss and gradient NaN.
__global__ void __launch_bounds__(kHeadThreads)
    k_softmax_xent(const float* __restrict__ logits, const int32_t* __restrict__ labels, int64_t batch, int C,
                   float inv_batch, float* __restrict__ row_loss, float* __restrict__ dlogits)
{
    const int64_t r = (int64_t)blockIdx.x * kHeadThreads + threadIdx.x;
    if (r >= batch)
        return;
    const float* l = logits + r * C;
    float* g = dlogits + r * C;
    const int y = labels[r];
    if (y < 0 || y >= C) {
        row_loss[r] = __builtin_nanf("");
        for (int c = 0; c < C; ++c)
            g[c] = __builtin_nanf("");
        return;
    }
    float m = l[0];
    for (int c = 1; c < C; ++c)
        m = fmaxf(m, l[c]);
    float s = 0.f;
    for (int c = 0; c < C; ++c)
        s += expf(l[c] - m);
    const float lse = logf(s) + m;
    row_loss[r] = lse - l[y];
    const float inv_s = 1.f / s;
    for (int c = 0; c < C; ++c) {
        const float p = expf(l[c] - m) * inv_s;
        g[c] = (p - (c == y ? 1.f : 0.f)) * inv_batch;
    }
}

// Block col (C + 1 of them): thread k sums rows k, k + 256, ... of the
// column in order, then a fixed binary tree over the 256 partial sums.
// Column C is the row loss (scaled by 1/batch), columns 0..C-1 are dlogits
// (db).
__global__ void __launch_bounds__(kHeadThreads)
    k_head_sums(const float* __restrict__ row_loss, const float* __restrict__ dlogits, int64_t batch, int C,
                float inv_batch, float* __restrict__ loss, float* __restrict__ db)
{
    __shared__ float part[kHeadThreads];
    const int col = blockIdx.x;
    float s = 0.f;
    for (int64_t r = threadIdx.x; r < batch; r += kHeadThreads)
        s += col == C ? row_loss[r] : dlogits[r * C + col];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = kHeadThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (col == C) {
            if (loss)
                *loss = part[0] * inv_batch;
        } else if (db) {
            db[col] = part[0];
        }
    }
}

__global__ void __launch_bounds__(kHeadThreads)
    k_axpy(float* __restrict__ y, const float* __restrict__ x, int64_t count, float alpha)
{
    const int64_t stride = (int64_t)gridDim.x * kHeadThreads;
    for (int64_t i = (int64_t)blockIdx.x * kHeadThreads + threadIdx.x; i < count; i += stride)
        y[i] += alpha * x[i];
}

// p[i] = value (an exponent array; written by a kernel so that a captured
// graph holds no memset node)
__global__ void __launch_bounds__(kHeadThreads) k_fill_i8(int8_t* __restrict__ p, int64_t count, int8_t value)
{
    const int64_t stride = (int64_t)gridDim.x * kHeadThreads;
    for (int64_t i = (int64_t)blockIdx.x * kHeadThreads + threadIdx.x; i < count; i += stride)
        p[i] = value;
}

// The same update over several arrays in one launch: segment k owns blocks
// [block0[k], block0[k + 1]) and strides over its own count.
__global__ void __launch_bounds__(kHeadThreads) k_axpy_multi(AxpySegs segs, float alpha)
{
    const int64_t b = blockIdx.x;
    int k = 0;
    while (k + 1 < segs.count && segs.block0[k + 1] <= b)
        ++k;
    const int64_t nb = (k + 1 < segs.count ? segs.block0[k + 1] : (int64_t)gridDim.x) - segs.block0[k];
    float* __restrict__ y = segs.y[k];
    const float* __restrict__ x = segs.x[k];
    const int64_t n = segs.n[k];
    const int64_t stride = nb * kHeadThreads;
    for (int64_t i = (b - segs.block0[k]) * kHeadThreads + threadIdx.x; i < n; i += stride)
        y[i] += alpha * x[i];
}

// Block (row group, slab): rows r0 .. r0 + R - 1 against the slab's
// kLogitSlab4 float4 columns; thread t takes float4 columns
// kLogitSlab4 slab + t + 256 i, i < kLogitSlab4 / 256.  Each
// of the R C sums is reduced over the wave (xor butterfly) and the four
// waves (fixed order) into part[slab][r][c].  Rows past the batch read zero
// (empty range) and are not written.
constexpr int kLogitRows = 8;
// float4 columns per slab: at batch 1024, F = 32768, C = 10 a launch took
// 47 us with 1024, 43.5 us with 2048 and 48.6 us with 4096
constexpr int kLogitSlab4 = 2048;

template <int C, int R>
__global__ void __launch_bounds__(kHeadThreads)
    k_head_logits(const float* __restrict__ phi, const float* __restrict__ W, int64_t batch, int64_t F,
                  int64_t slabs, float* __restrict__ part)
{
    const int64_t slab = blockIdx.x % slabs;
    const int64_t r0 = (int64_t)(blockIdx.x / slabs) * R;
    const uint32_t t = threadIdx.x;
    const int64_t F4 = F / 4;
    const rsrc_t rw = make_rsrc(W, (uint32_t)(C * F * 4));
    rsrc_t rp[R];
#pragma unroll
    for (int r = 0; r < R; ++r)
        rp[r] = make_rsrc(phi + (r0 + r) * F, r0 + r < batch ? (uint32_t)(F * 4) : 0u);
    float acc[R][C];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int k = 0; k < C; ++k)
            acc[r][k] = 0.f;
    const int64_t q0 = slab * kLogitSlab4 + t;
#pragma unroll 2
    for (int i = 0; i < kLogitSlab4 / kHeadThreads; ++i) {
        const int64_t q = q0 + i * kHeadThreads;
        if (q >= F4)
            break;
        float p[R][4];
#pragma unroll
        for (int r = 0; r < R; ++r)
            bload4<2>(p[r], rp[r], (uint32_t)(16 * q), 0u);
#pragma unroll
        for (int k = 0; k < C; ++k) {
            float w[4];
            bload4(w, rw, (uint32_t)(16 * (k * F4 + q)), 0u);
#pragma unroll
            for (int r = 0; r < R; ++r)
                acc[r][k] += p[r][0] * w[0] + p[r][1] * w[1] + p[r][2] * w[2] + p[r][3] * w[3];
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int k = 0; k < C; ++k)
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1)
                acc[r][k] += __shfl_xor(acc[r][k], o);
    __shared__ float red[kHeadThreads / 64][R * C];
    const uint32_t wave = t / 64u;
    if (t % 64u == 0) {
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int k = 0; k < C; ++k)
                red[wave][r * C + k] = acc[r][k];
    }
    __syncthreads();
    if (t < (uint32_t)(R * C)) {
        const int r = (int)t / C;
        if (r0 + r < batch)
            part[(slab * batch + r0) * C + t] = (red[0][t] + red[1][t]) + (red[2][t] + red[3][t]);
    }
}

// logits[r][c] = b[c] + sum over slabs of part[slab][r][c], slabs ascending.
__global__ void __launch_bounds__(kHeadThreads)
    k_logits_finish(const float* __restrict__ part, const float* __restrict__ bias, int64_t slabs, int64_t batch,
                    int C, float* __restrict__ logits)
{
    const int64_t i = (int64_t)blockIdx.x * kHeadThreads + threadIdx.x;
    if (i >= batch * C)
        return;
    float s = 0.f;
    for (int64_t sl = 0; sl < slabs; ++sl)
        s += part[sl * batch * C + i];
    logits[i] = (bias ? bias[i % C] : 0.f) + s;
}

// Block (slab, group): thread t owns float4 column q = 256 slab + t and runs
// over the group's rows r: dphi[r][q] = sum_k dl[r][k] W[k][q] and
// acc[k][q] += dl[r][k] phi[r][q]; acc goes to part (group g at g C F).
template <int C>
__global__ void __launch_bounds__(kHeadThreads)
    k_head_bwd(const float* __restrict__ phi, const float* __restrict__ dl, const float* __restrict__ W,
               int64_t batch, int64_t F, int64_t slabs, int64_t rows_per_group, float* __restrict__ dphi,
               float* __restrict__ part)
{
    const int64_t F4 = F / 4;
    const int64_t slab = blockIdx.x % slabs, g = blockIdx.x / slabs;
    const int64_t q = slab * kHeadThreads + threadIdx.x;
    if (q >= F4)
        return;
    const int64_t rb = g * rows_per_group;
    const int64_t re = rb + rows_per_group < batch ? rb + rows_per_group : batch;
    float wq[C][4], acc[C][4];
    const rsrc_t rw = make_rsrc(W, dphi != nullptr ? (uint32_t)(C * F * 4) : 0u);  // W only for dphi
#pragma unroll
    for (int k = 0; k < C; ++k) {
        bload4(wq[k], rw, (uint32_t)(16 * (k * F4 + q)), 0u);
#pragma unroll
        for (int m = 0; m < 4; ++m)
            acc[k][m] = 0.f;
    }
    // eight rows at a time, all loads issued before any store (the compiler
    // does not move buffer loads across buffer stores); rows past the group
    // read zero and are not stored
    constexpr int U = 8;
    for (int64_t r = rb; r < re; r += U) {
        float p[U][4];
        if (part != nullptr) {
#pragma unroll
            for (int u = 0; u < U; ++u)
                bload4<2>(p[u], make_rsrc(phi + (r + u) * F, r + u < re ? (uint32_t)(F * 4) : 0u), (uint32_t)(16 * q),
                          0u);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (r + u >= re)
                break;
            float dlr[C];
#pragma unroll
            for (int k = 0; k < C; ++k)
                dlr[k] = dl[(r + u) * C + k];
            if (part != nullptr) {
#pragma unroll
                for (int k = 0; k < C; ++k)
#pragma unroll
                    for (int m = 0; m < 4; ++m)
                        acc[k][m] += dlr[k] * p[u][m];
            }
            if (dphi != nullptr) {
                float o[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int k = 0; k < C; ++k)
#pragma unroll
                    for (int m = 0; m < 4; ++m)
                        o[m] += dlr[k] * wq[k][m];
                bstore4_nt(make_rsrc(dphi + (r + u) * F, (uint32_t)(F * 4)), (uint32_t)(16 * q), o[0], o[1], o[2],
                           o[3]);
            }
        }
    }
    if (part != nullptr) {
        const rsrc_t ro = make_rsrc(part + g * C * F, (uint32_t)(C * F * 4));
#pragma unroll
        for (int k = 0; k < C; ++k)
            bstore4(ro, (uint32_t)(16 * (k * F4 + q)), acc[k][0], acc[k][1], acc[k][2], acc[k][3]);
    }
}

// out[i] = sum over g of part[g count + i], g ascending (zero for no groups);
// with y, also y[i] += alpha out[i].
__global__ void __launch_bounds__(kHeadThreads)
    k_sum_groups(const float* __restrict__ part, int64_t groups, int64_t count, float* __restrict__ out,
                 float* __restrict__ y, float alpha)
{
    const int64_t i = (int64_t)blockIdx.x * kHeadThreads + threadIdx.x;
    if (i >= count)
        return;
    float s = 0.f;
    for (int64_t g = 0; g < groups; ++g)
        s += part[g * count + i];
    out[i] = s;
    if (y != nullptr)
        y[i] += alpha * s;
}

// One block of 1024 lanes: the logits from the expansion-group partials and
// b, then per row the steps of k_softmax_xent (lane t takes rows t, t + 1024,
// ...); the mean loss and db are summed in a fixed order (each lane's rows in
// order, an xor butterfly within each wave, the 16 waves in order).  b is
// read by every lane before the barrier and updated after it.
constexpr int kTailThreads = 1024;

template <int C>
__global__ void __launch_bounds__(kTailThreads)
    k_head_tail(const float* __restrict__ part, float* __restrict__ b, int64_t esplit, int64_t batch,
                const int32_t* __restrict__ labels, float inv_batch, float* __restrict__ logits,
                float* __restrict__ dlogits, float* __restrict__ loss, float* __restrict__ db, float alpha)
{
    constexpr int NW = kTailThreads / 64;
    __shared__ float red[NW][C + 1];
    const int t = (int)threadIdx.x;
    float bias[C], acc[C + 1];
#pragma unroll
    for (int c = 0; c < C; ++c)
        bias[c] = b ? b[c] : 0.f;
#pragma unroll
    for (int c = 0; c <= C; ++c)
        acc[c] = 0.f;
    for (int64_t r = t; r < batch; r += kTailThreads) {
        float l[C];
#pragma unroll
        for (int c = 0; c < C; ++c)
            l[c] = 0.f;
        for (int64_t sl = 0; sl < esplit; ++sl) {
            const float* p = part + (sl * batch + r) * C;
#pragma unroll
            for (int c = 0; c < C; ++c)
                l[c] += p[c];
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            l[c] += bias[c];
            logits[r * C + c] = l[c];
        }
        const int y = labels[r];
        float* g = dlogits + r * C;
        if (y < 0 || y >= C) {
            acc[C] += __builtin_nanf("");
#pragma unroll
            for (int c = 0; c < C; ++c) {
                g[c] = __builtin_nanf("");
                acc[c] += __builtin_nanf("");
            }
            continue;
        }
        float m = l[0];
#pragma unroll
        for (int c = 1; c < C; ++c)
            m = fmaxf(m, l[c]);
        float s = 0.f;
#pragma unroll
        for (int c = 0; c < C; ++c)
            s += expf(l[c] - m);
        const float lse = logf(s) + m;
        float ly = l[0];
#pragma unroll
        for (int c = 1; c < C; ++c)
            ly = c == y ? l[c] : ly;
        acc[C] += lse - ly;
        const float inv_s = 1.f / s;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const float p = expf(l[c] - m) * inv_s;
            const float gc = (p - (c == y ? 1.f : 0.f)) * inv_batch;
            g[c] = gc;
            acc[c] += gc;
        }
    }
#pragma unroll
    for (int c = 0; c <= C; ++c) {
        float v = acc[c];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1)
            v += __shfl_xor(v, o);
        acc[c] = v;
    }
    if ((t & 63) == 0) {
#pragma unroll
        for (int c = 0; c <= C; ++c)
            red[t >> 6][c] = acc[c];
    }
    __syncthreads();
    if (t <= C) {
        float s = 0.f;
        for (int w = 0; w < NW; ++w)
            s += red[w][t];
        if (t == C) {
            if (loss)
                *loss = s * inv_batch;
        } else {
            if (db)
                db[t] = s;
            if (b && alpha != 0.f)
                b[t] += alpha * s;
        }
    }
}

template <int C>
hipError_t head_logits_c(const float* phi, const float* W, int64_t batch, int64_t F, int64_t slabs, float* part,
                         hipStream_t s)
{
    const int64_t groups = (batch + kLogitRows - 1) / kLogitRows;
    k_head_logits<C, kLogitRows><<<dim3((unsigned)(groups * slabs)), dim3(kHeadThreads), 0, s>>>(phi, W, batch, F,
                                                                                                 slabs, part);
    return hipGetLastError();
}

template <int C>
hipError_t head_bwd_c(const float* phi, const float* dl, const float* W, int64_t batch, int64_t F, int64_t slabs,
                      int64_t groups, int64_t rows_per_group, float* dphi, float* part, hipStream_t s)
{
    k_head_bwd<C><<<dim3((unsigned)(slabs * groups)), dim3(kHeadThreads), 0, s>>>(phi, dl, W, batch, F, slabs,
                                                                                   rows_per_group, dphi, part);
    return hipGetLastError();
}

}  // namespace

int64_t head_logit_slabs(int64_t F) { return (F / 4 + kLogitSlab4 - 1) / kLogitSlab4; }

hipError_t launch_head_logits(const float* phi, const float* W, const float* b, int64_t batch, int64_t F, int C,
                              float* part, float* logits, hipStream_t s)
{
    const int64_t slabs = head_logit_slabs(F);
    hipError_t err;
#define MCK_LOGITS(K) err = head_logits_c<K>(phi, W, batch, F, slabs, part, s); break
    switch (C) {
    case 1: MCK_LOGITS(1);
    case 2: MCK_LOGITS(2);
    case 3: MCK_LOGITS(3);
    case 4: MCK_LOGITS(4);
    case 5: MCK_LOGITS(5);
    case 6: MCK_LOGITS(6);
    case 7: MCK_LOGITS(7);
    case 8: MCK_LOGITS(8);
    case 9: MCK_LOGITS(9);
    case 10: MCK_LOGITS(10);
    case 11: MCK_LOGITS(11);
    case 12: MCK_LOGITS(12);
    case 13: MCK_LOGITS(13);
    case 14: MCK_LOGITS(14);
    case 15: MCK_LOGITS(15);
    case 16: MCK_LOGITS(16);
    default: return hipErrorInvalidValue;
    }
#undef MCK_LOGITS
    if (err != hipSuccess)
        return err;
    const unsigned blocks = (unsigned)((batch * C + kHeadThreads - 1) / kHeadThreads);
    k_logits_finish<<<dim3(blocks), dim3(kHeadThreads), 0, s>>>(part, b, slabs, batch, C, logits);
    return hipGetLastError();
}

hipError_t launch_logits_finish(const float* part, const float* b, int64_t slabs, int64_t batch, int C,
                                float* logits, hipStream_t s)
{
    const unsigned blocks = (unsigned)((batch * C + kHeadThreads - 1) / kHeadThreads);
    k_logits_finish<<<dim3(blocks), dim3(kHeadThreads), 0, s>>>(part, b, slabs, batch, C, logits);
    return hipGetLastError();
}

void head_bwd_geometry(int64_t batch, int64_t F, bool need_dW, int64_t* slabs, int64_t* groups, int64_t* rows_per_group)
{
    const int64_t F4 = F / 4;
    *slabs = (F4 + kHeadThreads - 1) / kHeadThreads;
    // about 512 blocks; with dW each group adds C F floats of partials, so at
    // most 32 groups
    int64_t g = (512 + *slabs - 1) / *slabs;
    if (need_dW && g > 32)
        g = 32;
    if (g > batch)
        g = batch;
    if (g < 1)
        g = 1;
    *rows_per_group = batch > 0 ? (batch + g - 1) / g : 1;
    *groups = batch > 0 ? (batch + *rows_per_group - 1) / *rows_per_group : 0;
}

hipError_t launch_head_bwd(const float* phi, const float* dl, const float* W, int64_t batch, int64_t F, int C,
                           int64_t slabs, int64_t groups, int64_t rows_per_group, float* dphi, float* part,
                           hipStream_t s)
{
    if (groups == 0)
        return hipSuccess;
#define MCK_HBWD(K) head_bwd_c<K>(phi, dl, W, batch, F, slabs, groups, rows_per_group, dphi, part, s)
    switch (C) {
    case 1: return MCK_HBWD(1);
    case 2: return MCK_HBWD(2);
    case 3: return MCK_HBWD(3);
    case 4: return MCK_HBWD(4);
    case 5: return MCK_HBWD(5);
    case 6: return MCK_HBWD(6);
    case 7: return MCK_HBWD(7);
    case 8: return MCK_HBWD(8);
    case 9: return MCK_HBWD(9);
    case 10: return MCK_HBWD(10);
    case 11: return MCK_HBWD(11);
    case 12: return MCK_HBWD(12);
    case 13: return MCK_HBWD(13);
    case 14: return MCK_HBWD(14);
    case 15: return MCK_HBWD(15);
    case 16: return MCK_HBWD(16);
    default: return hipErrorInvalidValue;
    }
#undef MCK_HBWD
}

hipError_t launch_sum_groups(const float* part, int64_t groups, int64_t count, float* out, hipStream_t s, float* y,
                             float alpha)
{
    if (count == 0)
        return hipSuccess;
    const unsigned blocks = (unsigned)((count + kHeadThreads - 1) / kHeadThreads);
    k_sum_groups<<<dim3(blocks), dim3(kHeadThreads), 0, s>>>(part, groups, count, out, y, alpha);
    return hipGetLastError();
}

hipError_t launch_head_tail(const float* part, float* b, int64_t esplit, int64_t batch, int C,
                            const int32_t* labels, float* logits, float* dlogits, float* loss, float* db, float alpha,
                            hipStream_t s)
{
    if (batch < 1 || batch > kHeadTailRows)
        return hipErrorInvalidValue;
    const float inv = 1.f / (float)batch;
#define MCK_TAIL(CC)                                                                                            \
    case CC:                                                                                                   \
        k_head_tail<CC><<<dim3(1), dim3(kTailThreads), 0, s>>>(part, b, esplit, batch, labels, inv, logits,     \
                                                                dlogits, loss, db, alpha);                     \
        return hipGetLastError();
    switch (C) {
        MCK_TAIL(1)
        MCK_TAIL(2)
        MCK_TAIL(3)
        MCK_TAIL(4)
        MCK_TAIL(5)
        MCK_TAIL(6)
        MCK_TAIL(7)
        MCK_TAIL(8)
        MCK_TAIL(9)
        MCK_TAIL(10)
    default: return hipErrorInvalidValue;
    }
#undef MCK_TAIL
}

hipError_t launch_softmax_xent(const float* logits, const int32_t* labels, int64_t batch, int C, float* row_loss,
                               float* dlogits, float* loss, float* db, hipStream_t s)
{
    const float inv = 1.f / (float)batch;
    const unsigned blocks = (unsigned)((batch + kHeadThreads - 1) / kHeadThreads);
    k_softmax_xent<<<dim3(blocks), dim3(kHeadThreads), 0, s>>>(logits, labels, batch, C, inv, row_loss, dlogits);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess)
        return err;
    k_head_sums<<<dim3((unsigned)(C + 1)), dim3(kHeadThreads), 0, s>>>(row_loss, dlogits, batch, C, inv, loss, db);
    return hipGetLastError();
}

hipError_t launch_axpy_multi(float* const* y, const float* const* x, const int64_t* count, int nseg, float alpha,
                             hipStream_t s)
{
    if (nseg < 1 || nseg > kAxpySegs)
        return hipErrorInvalidValue;
    AxpySegs segs;
    segs.count = nseg;
    int64_t blocks = 0;
    for (int k = 0; k < nseg; ++k) {
        segs.y[k] = y[k];
        segs.x[k] = x[k];
        segs.n[k] = count[k];
        segs.block0[k] = blocks;
        int64_t bk = (count[k] + kHeadThreads - 1) / kHeadThreads;
        blocks += bk > 1024 ? 1024 : (bk < 1 ? 1 : bk);
    }
    k_axpy_multi<<<dim3((unsigned)blocks), dim3(kHeadThreads), 0, s>>>(segs, alpha);
    return hipGetLastError();
}

hipError_t launch_fill_i8(int8_t* p, int64_t count, int8_t value, hipStream_t s)
{
    int64_t blocks = (count + kHeadThreads - 1) / kHeadThreads;
    blocks = blocks > 4096 ? 4096 : (blocks < 1 ? 1 : blocks);
    k_fill_i8<<<dim3((unsigned)blocks), dim3(kHeadThreads), 0, s>>>(p, count, value);
    return hipGetLastError();
}

hipError_t launch_axpy(float* y, const float* x, int64_t count, float alpha, hipStream_t s)
{
    int64_t blocks = (count + kHeadThreads - 1) / kHeadThreads;
    blocks = blocks > 4096 ? 4096 : (blocks < 1 ? 1 : blocks);
    k_axpy<<<dim3((unsigned)blocks), dim3(kHeadThreads), 0, s>>>(y, x, count, alpha);
    return hipGetLastError();
}

}  // namespace mck
