// head.hip -- the linear classifier trained on the McKernel features
// (section "Empirical Analysis and Experiments": softmax(W phi + b) with
// cross-entropy; section "Large-scale Machine Learning": minimised by SGD).
//
//   k_softmax_xent  per row: loss_r = log sum_c exp(l_rc) - l_r,y and the
//                   gradient of the mean loss, (softmax(l_r) - onehot(y)) / batch
//   k_head_sums     fixed-order sums over rows: the mean loss and db
//   k_axpy          y += alpha x (the SGD update with alpha = -learning rate)
//
// The logits and the weight gradients are plain GEMMs (phi W^T, dlogits^T
// phi, dlogits W) left to the BLAS library; these kernels hold the rest.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

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

// One block: thread k sums rows k, k + 256, ... of the column in order, then
// a fixed binary tree over the 256 partial sums.  Column C is the row loss
// (scaled by 1/batch), columns 0..C-1 are dlogits (db).
__global__ void __launch_bounds__(kHeadThreads)
    k_head_sums(const float* __restrict__ row_loss, const float* __restrict__ dlogits, int64_t batch, int C,
                float inv_batch, float* __restrict__ loss, float* __restrict__ db)
{
    __shared__ float part[kHeadThreads];
    for (int col = 0; col <= C; ++col) {
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
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kHeadThreads)
    k_axpy(float* __restrict__ y, const float* __restrict__ x, int64_t count, float alpha)
{
    const int64_t stride = (int64_t)gridDim.x * kHeadThreads;
    for (int64_t i = (int64_t)blockIdx.x * kHeadThreads + threadIdx.x; i < count; i += stride)
        y[i] += alpha * x[i];
}

}  // namespace

hipError_t launch_softmax_xent(const float* logits, const int32_t* labels, int64_t batch, int C, float* row_loss,
                               float* dlogits, float* loss, float* db, hipStream_t s)
{
    const float inv = 1.f / (float)batch;
    const unsigned blocks = (unsigned)((batch + kHeadThreads - 1) / kHeadThreads);
    k_softmax_xent<<<dim3(blocks), dim3(kHeadThreads), 0, s>>>(logits, labels, batch, C, inv, row_loss, dlogits);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess)
        return err;
    k_head_sums<<<dim3(1), dim3(kHeadThreads), 0, s>>>(row_loss, dlogits, batch, C, inv, loss, db);
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
