// launch.hpp -- host-side launchers of the device kernels (internal to the
// library; the public interface is include/mckernel.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mck {

// Parameter generator: B, perm, G, S64, S32 (E x n each); norm2 is E doubles
// of scratch.  Six kernels on stream s.
// matern_t = 0: RBF (chi(n) radii); 1..255: RBF-Matern radii from matern_t
// unit-ball samples (n <= 2048).
hipError_t launch_generate(uint32_t seed, int64_t n, int64_t E, double sigma, int matern_t, float* B, int32_t* perm,
                           float* G, double* S64, float* S32, double* norm2, hipStream_t s);

// Box-Muller pairs for given hash words (generator self-check).
hipError_t launch_boxmuller(const uint32_t* a, const uint32_t* b, int64_t count, float* g0, float* g1,
                            hipStream_t s);

// Kernel-layout copies of the parameters, for the forward (F) and the
// backward (B) register layouts: gather offsets (byte offset in the block's
// LDS of the source of each gathered element; plan_elems(M) of them per
// expansion), G by source (Gs_f) and by destination (Gk_b), and S in half
// turns (Sh, natural order).  S64 may be null (then S32 is used).
// fwd_goff is the largest count over the forward's compiled register
// splits, so that one allocation serves whichever split a plan uses.
void plan_elems(int M, int64_t* fwd_goff, int64_t* bwd_goff);
// Bsign: the generated +-1 diagonal B of a seed plan, or null for
// caller-given diagonals; with it the forward arrays of split PF = 5 are
// derived in the packed form of forward.hpp (16-bit gather indices and the
// sign words of B).
hipError_t launch_derive(int M, int PF, int64_t E, const int32_t* perm, const float* G, const float* Bsign,
                         const double* S64, const float* S32, uint32_t* goff_f, float* Gs_f, uint32_t* goff_b,
                         float* Gk_b, float* Sh, hipStream_t s);
// The backward arrays alone (goff_b, Gk_b) and Sh, from FP32 S.
hipError_t launch_derive_bwd(int M, int64_t E, const int32_t* perm, const float* G, const float* S32,
                             uint32_t* goff_b, float* Gk_b, float* Sh, hipStream_t s);
// The forward arrays alone (goff_f, Gs_f) for register split PF.
hipError_t launch_derive_fwd(int M, int PF, int64_t E, const int32_t* perm, const float* G, const float* Bsign,
                             uint32_t* goff_f, float* Gs_f, hipStream_t s);

// Forward register splits (register bits per layout, 4 or 5) compiled for
// n = 2^M, and the default one.
bool fwd_split_ok(int M, int P);
int fwd_split_default(int M);
int bwd_split(int M);  // register split of the backward
constexpr int kFwdWavesDefault = 16384;

// In-place batched Walsh-Hadamard transform, n = 2^M, 1 <= M <= 15.
hipError_t launch_fwht(int M, float* data, int64_t batch, bool vec, hipStream_t s);

// Forward: phi (trig = true) or z = S H G Pi H B xhat (trig = false).  P is
// the register split the arrays goff, Gs were derived for; the expansions
// are split into chunks until the grid holds about `waves` waves.  packed:
// the arrays belong to a seed plan (derived with Bsign); caller-given
// diagonals (packed = false) support only the feature map at P = 5.
// xexp (nullable): per-row power-of-2 exponents of a scaled x, x = stored x * 2^xexp[row].
hipError_t launch_forward(int M, int P, int waves, bool packed, bool vec, bool trig, const float* x, int64_t batch,
                          int d, int64_t E, const float* B, const uint32_t* goff, const float* Gs, const float* Sx,
                          float cs, float* out, hipStream_t s, const int8_t* xexp = nullptr);

// Forward with 16-bit storage (forward16.hip): xt, yt = 0 (FP32), 1 (bf16),
// 2 (half); supported pairs (0,1), (0,2), (1,1), (2,2); the feature map of
// a seed plan only.
hipError_t launch_forward_t(int M, int P, int waves, bool vec, int xt, int yt, const void* x, int64_t batch, int d,
                            int64_t E, const float* B, const uint32_t* goff, const float* Gs, const float* Sx,
                            float cs, void* out, hipStream_t s, const int8_t* xexp = nullptr);

// n = 2^M > 2^15 (longn.hip): in-place H on 16-byte aligned rows, and the
// feature map through FP32 scratch rows u, w (batch x n each).  Sh for such
// plans comes from launch_sh (S / 2 pi from the FP64 S).  xexp (nullable):
// per-row power-of-2 exponents of a scaled x.
hipError_t launch_fwht_long(int M, float* data, int64_t batch, bool vec, hipStream_t s);
hipError_t launch_forward_long(int M, bool vec, int xt, int yt, const void* x, int64_t batch, int d, int64_t E,
                               const float* B, const uint32_t* packA, const uint16_t* dstB, const int32_t* pdelta,
                               const float* Gx, const float* Sh, float cs, void* phi, float* u, float* w,
                               hipStream_t s, const int8_t* xexp = nullptr);
// n = 2^16 (longn.hip): the whole feature map of a row in one 1024-lane
// block per (row, expansion) work item, Pi split by the outer stage of a
// Benes network (register-pair switches around two 2^15 permutations through
// LDS); blocks from pair_blocks (a multiple of 8).  The plan arrays come from
// launch_pair_plan: Bw (sign words of B, E x 2 x 1024), Pw (switch words,
// E x 2 x 1024), Po (gather indices, E n / 2 words), Pg (G, E n floats).
int64_t pair_blocks(int64_t rows, int64_t E, int cus);
hipError_t launch_pair_plan(int64_t E, const int32_t* perm, const float* G, const float* B, uint32_t* Bw,
                            uint32_t* Pw, uint32_t* Po, float* Pg, hipStream_t s);
hipError_t launch_forward_pair(bool vec, int xt, int yt, const void* x, int64_t batch, int d, int64_t E,
                               const uint32_t* Bw, const uint32_t* Pw, const uint32_t* Po, const float* Pg,
                               const float* Sh, float cs, void* phi, int64_t blocks, hipStream_t s,
                               const int8_t* xexp = nullptr);
// Pi (destination i takes source perm[i]) of each expansion as an exchange
// between the C = n / 2^15 chunks of 2^15 elements.  The exchange buffer T
// holds, for each destination chunk co, the elements it receives, grouped
// by source chunk ci (ascending), ascending destination within a group.
// Per expansion (arrays of expansion e start at e n and e C C):
//   packA [ci 2^15 + slot(q)] = co << 15 | s: the q-th element leaving
//       source chunk ci (grouped by co, the same order within a group) is
//       its element s and goes to destination chunk co; slot(q) orders the
//       positions for the row pass's lanes (pack_slot in longn.hip);
//   pdelta [ci C + co]: its position in T is q + pdelta[ci][co];
//   dstB [co 2^15 + p]: T position co 2^15 + p lands at element dstB of
//       destination chunk co;
//   Gx [co 2^15 + p]: G of that element (G in T order).
// scratch: E C (3C + 2) ints.
hipError_t launch_buckets(int M, int64_t E, const int32_t* perm, const float* G, uint32_t* packA, uint16_t* dstB,
                          int32_t* pdelta, float* Gx, int32_t* scratch, hipStream_t s);
hipError_t launch_sh(const double* S64, float* Sh, int64_t count, hipStream_t s);

// Grouped forward (FP32 x and phi, n = 2^M <= 2^15): several feature maps
// of the same n in one launch per kGroupMax maps.  Each map's x and phi
// byte ranges must be below 2^31.
struct GroupInst {
    const float* x;
    int64_t batch;
    int d;
    int64_t E;
    const float* B;
    const uint32_t* goff;
    const float* Gs;
    const float* Sh;
    float cs;
    float* phi;
};
hipError_t launch_forward_group(int M, int P, int waves, bool vec, const GroupInst* inst, int count, hipStream_t s);

// Backward geometry: blocks, passes per block.
// Backward launch shape: rowblocks blocks of passes x rows; for n <= 1024
// with few row blocks the expansions are split over esplit block groups
// (blocks = rowblocks x esplit), and group g writes its share of dx to
// dx + g batch d (the caller sums the esplit slices).
struct BwdGeometry {
    int64_t blocks;
    int passes;
    int block_threads;
    int esplit;
    int64_t rowblocks;
    int rows_per_pass;
};
BwdGeometry backward_geometry(int M, int64_t batch, int d, int64_t E);

// Backward: dx (nullable) and, when partial != null, per-row-block partial
// sums of dS, dG, dB (rowblocks x E x 3 x n) reduced afterwards by
// launch_reduce.
hipError_t launch_backward(int M, bool vec, const float* x, const float* dphi, int64_t batch, int d, int64_t E,
                           const float* B, const uint32_t* goff, const float* Gk, const float* S32,
                           const float* Sh, float cs, float* dx, float* partial,
                           const BwdGeometry& geo, hipStream_t s);

// Fixed-order sum of the partials: out_a[e][i] = sum_b partial[b][e][a][i]
// for a = 0 (S), 1 (G), 2 (B); null outputs skipped.  With uS, uG, uB
// (nullable) each sum also updates u_a[e][i] += alpha out_a[e][i] (the SGD
// step of the training step, after every reader of those arrays).
// A second sum the same launch can carry (the training step's dW from its
// row-range partials): out[i] = sum over g ascending of part[g count + i],
// and with y, y[i] += alpha out[i] -- the same order as launch_sum_groups.
struct GroupSum {
    const float* part;
    int64_t groups;
    int64_t count;
    float* out;
    float* y;
    float alpha;
};
hipError_t launch_reduce(const float* partial, int64_t blocks, int64_t E, int64_t n, float* dS, float* dG,
                         float* dB, hipStream_t s, float* uS = nullptr, float* uG = nullptr, float* uB = nullptr,
                         float alpha = 0.f, const GroupSum* extra = nullptr);

// Classifier head (head.hip): per-row softmax cross-entropy and its
// gradient (dlogits = (softmax - onehot) / batch), then the mean loss and
// db = column sums of dlogits in a fixed order.  row_loss is batch floats of
// scratch.  loss and db may be null.
hipError_t launch_softmax_xent(const float* logits, const int32_t* labels, int64_t batch, int C, float* row_loss,
                               float* dlogits, float* loss, float* db, hipStream_t s);

// y += alpha x over count floats.
// y_k += alpha x_k for up to kAxpySegs arrays in one launch.
constexpr int kAxpySegs = 8;
struct AxpySegs {
    int count;
    float* y[kAxpySegs];
    const float* x[kAxpySegs];
    int64_t n[kAxpySegs];
    int64_t block0[kAxpySegs];
};
hipError_t launch_axpy_multi(float* const* y, const float* const* x, const int64_t* count, int nseg, float alpha,
                             hipStream_t s);
hipError_t launch_axpy(float* y, const float* x, int64_t count, float alpha, hipStream_t s);
hipError_t launch_fill_i8(int8_t* p, int64_t count, int8_t value, hipStream_t s);
// Classifier head products, C in [1, 16] classes, F a multiple of 4, phi,
// W, dphi 16-byte aligned, C F 4 < 2^31.
// part: head_logit_slabs(F) x batch x C floats of scratch.
int64_t head_logit_slabs(int64_t F);
hipError_t launch_head_logits(const float* phi, const float* W, const float* b, int64_t batch, int64_t F, int C,
                              float* part, float* logits, hipStream_t s);
// Launch shape of launch_head_bwd: slabs of 1024 columns x groups of rows;
// dW then needs groups x C x F floats of partials (summed by
// launch_sum_groups) unless groups == 1.
void head_bwd_geometry(int64_t batch, int64_t F, bool need_dW, int64_t* slabs, int64_t* groups,
                       int64_t* rows_per_group);
hipError_t launch_head_bwd(const float* phi, const float* dl, const float* W, int64_t batch, int64_t F, int C,
                           int64_t slabs, int64_t groups, int64_t rows_per_group, float* dphi, float* part,
                           hipStream_t s);
// out[i] = sum over groups of part[g count + i]; with y (nullable) also
// y[i] += alpha out[i].
hipError_t launch_sum_groups(const float* part, int64_t groups, int64_t count, float* out, hipStream_t s,
                             float* y = nullptr, float alpha = 0.f);
// The end of the fused training step's head for batch <= kHeadTailRows and
// C <= kFusedHeadMaxC, in one block: logits = b + the esplit partials, the
// softmax cross-entropy per row (dlogits), the mean loss and db in a fixed
// order, and b += alpha db (alpha may be 0).
constexpr int64_t kHeadTailRows = 4096;
hipError_t launch_head_tail(const float* part, float* b, int64_t esplit, int64_t batch, int C,
                            const int32_t* labels, float* logits, float* dlogits, float* loss, float* db, float alpha,
                            hipStream_t s);
// logits[r][c] = b[c] (b nullable) + sum over slabs of part[slab][r][c].
hipError_t launch_logits_finish(const float* part, const float* b, int64_t slabs, int64_t batch, int C,
                                float* logits, hipStream_t s);

// The training step with the head fused into the feature map (train.hip):
// n = 1024 and C <= kFusedHeadMaxC, the explicit-parameter forward arrays of
// register split 4 (goff, Gs) and Sh.  launch_forward_logits writes
// esplit x batch x C partial logits (summed by launch_logits_finish);
// launch_head_bwd_fused writes dphi (batch x 2nE) and ranges x C x 2nE
// partials of dW (summed by launch_sum_groups).
constexpr int kFusedHeadMaxC = 10;
bool fused_head_ok(int64_t n, int64_t C);
int64_t fused_logits_esplit(int64_t batch, int64_t E);
void fused_bwd_geometry(int64_t batch, int64_t E, int64_t* ranges, int64_t* rows_per_range);
hipError_t launch_forward_logits(bool vec, const float* x, int64_t batch, int d, int64_t E, const float* B,
                                 const uint32_t* goff, const float* Gs, const float* Sh, float cs, const float* W,
                                 int C, int64_t esplit, float* part, hipStream_t s);
hipError_t launch_head_bwd_fused(bool vec, const float* x, int64_t batch, int d, int64_t E, const float* B,
                                 const uint32_t* goff, const float* Gs, const float* Sh, float cs, const float* dl,
                                 const float* W, int C, int64_t ranges, int64_t rows_per_range, float* dphi,
                                 float* part, hipStream_t s);

}  // namespace mck
