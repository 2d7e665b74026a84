/*
 * mckernel.h -- C interface of the MI355X (gfx950) Fastfood hot path.
 *
 * The library computes McKernel's approximate kernel expansion (Curto et al.,
 * arXiv 1702.08159): for an input row x of length d, zero-padded to
 * n = max(2, next power of two >= d) (figure 1 caption and section
 * "Empirical Analysis and Experiments": xhat = [x]_2), and for each of E
 * kernel expansions e (section "McKernel": i.i.d. instances of Z stacked),
 *
 *     z_e = S_e H G_e Pi_e H B_e xhat          (equation "mckernel")
 *     phi = c [cos z_0 .. cos z_{E-1}, sin z_0 .. sin z_{E-1}]   (equation "mcfeatures")
 *
 * with H the unnormalised Sylvester-Hadamard matrix (section "Fast Walsh
 * Hadamard"), B a +-1 diagonal, Pi a permutation (applied as the gather
 * (Pi v)_i = v[perm[i]]), G a Gaussian diagonal, S the RBF calibration
 * S_j = s_j / (sigma sqrt(n) ||G_e||_F) with s_j ~ chi(n), and
 * c = 1/sqrt(n E).  In seed mode B, Pi, G and S are generated from a 32-bit
 * seed by the hash-driven generator documented with the project (MurmurHash3
 * bits for B, a hash-driven Fisher-Yates shuffle for Pi, Box-Muller for G,
 * chi(n) by Marsaglia-Tsang for S: section "McKernel", items B, Pi, G, C),
 * so nothing but the seed needs to be stored (section "API Description").
 *
 * Conventions for every call:
 *  - Arrays are caller-owned DEVICE pointers (hipMalloc / torch CUDA
 *    tensors), FP32 unless stated, row-major and contiguous.  Outputs must not
 *    alias inputs.
 *  - Work is enqueued asynchronously on `stream` (a hipStream_t; NULL = the
 *    null stream).  Argument validation is synchronous: on an error status
 *    nothing has been enqueued.
 *  - Seed-mode calls build (once per device, seed, n, E, sigma, calibration)
 *    a cached parameter plan in device memory; building it allocates memory,
 *    launches the generator kernels on `stream` and waits for them.  Calls
 *    that reuse a cached plan allocate nothing except where noted.
 *    "Stream-ordered" temporaries come from a few blocks per device that
 *    the library allocates once (growing them when a call needs more) and
 *    reuses: a block last used on another stream is taken after a
 *    device-side wait for that use, so a call never waits on the host for
 *    earlier work.  Under stream capture temporaries are graph-owned
 *    stream-ordered allocations.  mck_shutdown() frees the blocks.
 *    The cache is thread-safe and holds at most 32 plans / 2 GiB per
 *    process, evicting the least recently used.  Each call pins its plan
 *    from lookup until its last launch is enqueued, so an eviction or
 *    mck_shutdown() on another thread never frees a plan in use.  A call
 *    enqueued on a stream that is being captured into a graph marks its
 *    plan "captured": eviction never frees it (the graph reads it at every
 *    replay); mck_shutdown() does, so destroy such graphs first.
 *  - Gradient outputs are overwritten, not accumulated; a NULL gradient
 *    pointer skips that gradient.
 *  - batch == 0 is a no-op that returns MCK_OK.
 *  - No C++ exception crosses this interface; failures are status codes, and
 *    mck_last_error() returns a message for the calling thread's last failure.
 */
#ifndef MCKERNEL_H
#define MCKERNEL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum mck_status {
    MCK_OK = 0,
    MCK_ERR_INVALID_ARG = 1, /* bad size, pointer, sigma, ... (nothing enqueued) */
    MCK_ERR_UNSUPPORTED = 2, /* valid request the library does not implement */
    MCK_ERR_HIP = 3,         /* a HIP runtime call or kernel launch failed */
    MCK_ERR_NO_MEMORY = 4    /* device allocation failed */
} mck_status;

/*
 * Calibration C of equation "mckernel": the radii s_j of S_j = s_j / (sigma
 * sqrt(n) ||G||_F).
 *  - MCK_CALIB_RBF: s_j ~ chi(n), the Gaussian RBF kernel exp(-|x-y|^2/2 sigma^2).
 *  - MCK_CALIB_MATERN: RBF-Matern (section "Customizing McKernel"): s_j is the
 *    Euclidean norm of the sum of t = 40 (the paper's value) i.i.d. samples
 *    uniform in the unit n-ball, each U^(1/n) X/||X|| with X ~ N(0, I_n),
 *    U ~ U(0,1], drawn from the same hash as B, Pi, G.  n <= 2048 (the draw
 *    costs t n^2 normals per expansion); larger n returns MCK_ERR_UNSUPPORTED.
 *  - MCK_CALIB_MATERN_T(t): RBF-Matern with t samples, 1 <= t <= 255.
 */
typedef enum mck_calibration {
    MCK_CALIB_RBF = 0,
    MCK_CALIB_MATERN = 1
} mck_calibration;
#define MCK_CALIB_MATERN_T(t) ((mck_calibration)(0x100 + (t)))

typedef void* mck_stream; /* hipStream_t */

/* Storage type of x or phi in mck_fastfood_forward_t. */
typedef enum mck_dtype {
    MCK_DTYPE_F32 = 0,  /* IEEE binary32 */
    MCK_DTYPE_BF16 = 1, /* bfloat16 (the upper half of a binary32) */
    MCK_DTYPE_F16 = 2   /* IEEE binary16 */
} mck_dtype;

/*
 * Largest n of the single-pass kernels (the transform held in LDS): the
 * backward, the projection and the explicit-parameter calls.
 */
#define MCK_MAX_N 32768

/*
 * Largest n of mck_fwht and of the seed-mode feature map
 * (mck_fastfood_forward, mck_fastfood_forward_t): beyond MCK_MAX_N they run
 * as a row pass over 2^15-element chunks plus column passes over the high
 * index bits, through FP32 scratch rows allocated on the stream (the feature
 * map at n = 2^16 instead keeps each row in one workgroup, with Pi split by
 * the outer stage of a Benes network, and needs no scratch).
 */
#define MCK_MAX_N_LONG 16777216

/* n = max(2, smallest power of two >= d); 0 when d < 1 or n > MCK_MAX_N_LONG. */
int64_t mck_padded_dim(int64_t d);

/* Static description of a status code. */
const char* mck_status_string(mck_status status);

/* Message of the calling thread's most recent failed call ("" if none). */
const char* mck_last_error(void);

/*
 * In-place batched Walsh-Hadamard transform: each of the `batch` rows of
 * `data` (batch x n) is replaced by H_n row, unnormalised, natural Sylvester
 * order: (H v)_i = sum_k (-1)^popcount(i & k) v_k (section "Fast Walsh
 * Hadamard": H_0 = [1], H_k = [[H, H], [H, -H]]).
 * n must be a power of two, 1 <= n <= MCK_MAX_N_LONG (n = 1 is the
 * identity); for n > MCK_MAX_N, data must be 16-byte aligned.
 */
mck_status mck_fwht(float* data, int64_t batch, int64_t n, mck_stream stream);

/*
 * Generated parameters of a seed-mode plan (section "McKernel", items
 * Binary B, Permutation Pi, Gaussian G and the calibration C: the diagonals
 * and the permutation of equation "mckernel", drawn from the seed by the
 * hash-driven generator), copied to caller buffers
 * (E x n each, n = a power of two in [2, MCK_MAX_N_LONG]): B (+-1 as float),
 * perm (int32 gather indices), G, S (FP32, S = RNE of the FP64 value with the
 * 1/(sigma sqrt n ||G||) factor included) and S64 (FP64, may be NULL).
 * Any of the outputs may be NULL.  sigma must be finite and > 0.
 */
mck_status mck_fastfood_params(uint32_t seed, int64_t n, int64_t E, double sigma, mck_calibration calib,
                               float* B, int32_t* perm, float* G, float* S, double* S64, mck_stream stream);

/*
 * Feature map.  x: batch x d (d >= 1, n = mck_padded_dim(d) <= MCK_MAX_N_LONG),
 * E >= 1, sigma finite > 0.  phi: batch x (2 n E), per row the E cosine
 * blocks of length n (expansion-major) followed by the E sine blocks.  For
 * n > MCK_MAX_N one row of phi must stay below 2^31 bytes; n = 2^16 runs in
 * one workgroup per row and expansion with no scratch, and n >= 2^17
 * allocates two FP32 scratch buffers of up to 2^27 floats each on `stream`
 * (stream-ordered).
 */
mck_status mck_fastfood_forward(const float* x, int64_t batch, int64_t d, int64_t E, uint32_t seed,
                                double sigma, mck_calibration calib, float* phi, mck_stream stream);

/*
 * The feature map with 16-bit storage: x (batch x d) and phi (batch x 2nE,
 * layout as in mck_fastfood_forward) of the given storage types, arithmetic
 * in FP32 throughout; 16-bit x values widen exactly and phi is rounded to
 * nearest even.  Supported (x_type, phi_type) pairs: (F32, F32), (F32, BF16),
 * (F32, F16), (BF16, BF16), (F16, F16); others return MCK_ERR_UNSUPPORTED.
 * |phi| <= 1/sqrt(nE), so half precision needs no scaling: its relative
 * rounding error is 2^-11 down to 6.1e-5 and below that the absolute error
 * is at most 3e-8.  Same argument rules and plan cache as
 * mck_fastfood_forward.
 */
mck_status mck_fastfood_forward_t(const void* x, mck_dtype x_type, int64_t batch, int64_t d, int64_t E,
                                  uint32_t seed, double sigma, mck_calibration calib, void* phi, mck_dtype phi_type,
                                  mck_stream stream);

/*
 * The feature map with per-row power-of-2 scaling of its storage (the 16-bit
 * forms of the long-vector and reduced-precision configurations), n <=
 * MCK_MAX_N_LONG, storage pairs as in mck_fastfood_forward_t:
 *   x_exp   (device, batch int8, nullable): row r of the input is the
 *           stored row times 2^x_exp[r]; the product must be finite in
 *           FP32.  The scaling is exact, so a 16-bit x can carry rows of
 *           any magnitude.
 *   phi_exp (device, batch int8, nullable, written): row r of phi is the
 *           stored row times 2^-phi_exp[r].  Every feature is bounded by
 *           c = 1/sqrt(nE) (equation "mcfeatures" with the normalisation of
 *           the features), so the exponent is the same for every row: the
 *           largest j with c 2^j <= 1, which keeps half-precision features
 *           out of the subnormal range.  Scaling by 2^j is exact: the stored
 *           value is the round-to-nearest-even of 2^j times the FP32 feature.
 */
mck_status mck_fastfood_forward_scaled(const void* x, mck_dtype x_type, const int8_t* x_exp, int64_t batch, int64_t d,
                                       int64_t E, uint32_t seed, double sigma, mck_calibration calib, void* phi,
                                       mck_dtype phi_type, int8_t* phi_exp, mck_stream stream);

/*
 * One of several independent feature maps for mck_fastfood_forward_batched:
 * the arguments of mck_fastfood_forward (FP32 x and phi, caller-owned device
 * arrays).
 */
typedef struct mck_instance {
    const float* x; /* batch x d */
    int64_t batch;
    int64_t d;
    int64_t E;
    uint32_t seed;
    double sigma;
    mck_calibration calib;
    float* phi; /* batch x 2nE */
} mck_instance;

/*
 * Runs `count` independent feature maps (uneven n, batch, E, seeds), each with
 * the result of mck_fastfood_forward, in as few launches as possible: the
 * maps with n <= MCK_MAX_N are grouped by n into one launch per 32 maps of
 * that n (blocks of all of them share one grid, so many small maps fill the
 * GPU together); longer maps run through the row and column passes.  `inst`
 * is a host array.  Every instance is validated before anything is enqueued;
 * the error message names the first bad instance.  Plans are built (and
 * kept from eviction) for the duration of the call.  Each n launches with
 * the current entry of the forward tuning table (below); once the plans are
 * cached, a call with no map longer than MCK_MAX_N neither allocates nor
 * synchronizes, so it can be captured into a graph.
 */
mck_status mck_fastfood_forward_batched(const mck_instance* inst, int64_t count, mck_stream stream);

/*
 * Recorded batched call.  mck_batched_graph_create does what
 * mck_fastfood_forward_batched does for `inst` (validation first, plans
 * built on `stream`, which it synchronizes) but records the launches into a
 * HIP graph instead of running them, with the forward tuning current at
 * that moment; the instances (pointers and sizes) are copied.  Every
 * mck_batched_graph_launch then enqueues the whole set on `stream` as one
 * graph launch: same results bit for bit as the eager call, no allocation,
 * no host work per map.  The object keeps the maps' plans from eviction and
 * owns the long maps' scratch rows, so replays that overlap on several
 * streams race on that scratch; mck_batched_graph_destroy waits for the
 * device, then frees the scratch and releases the plans (mck_shutdown
 * leaves the plans of live graphs in place).
 * Launching on a device other than the recording one is MCK_ERR_INVALID_ARG.
 */
typedef struct mck_batched_graph mck_batched_graph;
mck_status mck_batched_graph_create(const mck_instance* inst, int64_t count, mck_stream stream,
                                    mck_batched_graph** out);
mck_status mck_batched_graph_launch(mck_batched_graph* graph, mck_stream stream);
void mck_batched_graph_destroy(mck_batched_graph* graph);

/*
 * Launch choice of the single-pass forward for one n (2 <= n <= MCK_MAX_N,
 * a power of two).  The operation is fixed by equation "mckernel" of section
 * "McKernel"; these two numbers only choose how the kernel covers it:
 *   split  register bits per lane layout of the transform: 4 (16 values per
 *          lane) or 5 (32).  Both are compiled for 2^9 <= n <= 2^14; other
 *          n have one split.  The split decides which index bits are
 *          butterflied in registers and which through LDS, so the two can
 *          differ in the last bits of phi (both within the FP32 tolerance).
 *   waves  grid target: the E expansions of a map are cut into chunks until
 *          the grid holds about this many 64-lane waves (64 <= waves <= 2^20).
 * The table is per device and process; every forward of that n (plain,
 * 16-bit, batched, explicit-parameter and training step) launches with the
 * current entry.  Changing it while a forward of that n is being enqueued
 * on another thread is a race on which choice that call uses, nothing more.
 */
typedef struct mck_forward_tuning {
    int32_t split;
    int32_t waves;
} mck_forward_tuning;

/* Current choice for n (the built-in default when none was set). */
mck_status mck_forward_tuning_get(int64_t n, mck_forward_tuning* out);
/* Sets the choice for n; t = NULL restores the default.  MCK_ERR_UNSUPPORTED
 * for a split not compiled for n. */
mck_status mck_forward_tuning_set(int64_t n, const mck_forward_tuning* t);

/*
 * Autotuner.  For every n <= MCK_MAX_N present in `inst` (the arguments of
 * mck_fastfood_forward_batched), times the launches that
 * mck_fastfood_forward_batched makes for the maps of that n under each
 * compiled split and each grid target in {2048, 4096, ..., 65536} waves
 * (one untimed launch, then `reps` timed ones, 1 <= reps <= 1000, HIP events
 * on `stream`), and stores the fastest in the table above; a choice other
 * than the current best is taken only when it is at least 2 % faster.  Maps
 * with n > MCK_MAX_N are not timed.  The call writes every timed map's phi
 * (with a valid feature map) and synchronizes `stream`; it must not be
 * called while `stream` is being captured into a graph (MCK_ERR_INVALID_ARG).
 */
mck_status mck_autotune_forward_batched(const mck_instance* inst, int64_t count, int32_t reps, mck_stream stream);

/*
 * z = Z xhat without the trigonometric map (equation "mckernel" alone, before
 * the [cos, sin] of equation "mcfeatures"): batch x (n E), expansion-major,
 * block e = S_e H G_e Pi_e H B_e xhat.  Arguments as for mck_fastfood_forward
 * (n <= MCK_MAX_N).  A test hook that exposes the projection the features
 * are computed from.
 */
mck_status mck_fastfood_project(const float* x, int64_t batch, int64_t d, int64_t E, uint32_t seed,
                                double sigma, mck_calibration calib, float* z, mck_stream stream);

/*
 * Adjoint of the feature map (the chain rule through equations "mckernel"
 * and "mcfeatures"; H is symmetric and Pi^T is the scatter of Pi's gather),
 * the gradient the paper's training of C, G and B by back-propagation needs
 * (section "Empirical Analysis and Experiments").  n <= MCK_MAX_N.
 * Given dphi (batch x 2nE, the cotangent of phi)
 * computes dx (batch x d), and dB, dG, dS (E x n each): the gradients of
 * <dphi, phi> with respect to x and to the diagonals B, G, S taken as free
 * variables, summed over the batch.  The forward chain is recomputed, not
 * read from memory.  Requesting dB, dG or dS allocates a temporary buffer of
 * about 256 x E x 3n floats on `stream` (stream-ordered).
 */
mck_status mck_fastfood_backward(const float* x, const float* dphi, int64_t batch, int64_t d, int64_t E,
                                 uint32_t seed, double sigma, mck_calibration calib, float* dx, float* dB,
                                 float* dG, float* dS, mck_stream stream);

/*
 * Launch shape that mck_fastfood_backward (and the explicit-parameter and
 * training-step adjoints) use for a batch of `batch` rows of length d with E
 * expansions: a host-side query that launches nothing and needs no GPU.  The
 * adjoint's arithmetic (the chain rule through equation "mckernel") does not
 * depend on it; the shape says which kernel path covers the rows, so that
 * tests can show that every path they claim is exercised.
 *   rows_per_pass  rows one block transforms together (one per wave, or
 *                  several per wave for short rows);
 *   passes         row groups one block takes in turn within each expansion;
 *   rowblocks      blocks along the batch; block b owns rows
 *                  [b passes rows_per_pass, (b + 1) passes rows_per_pass);
 *   esplit         groups of expansions run by separate blocks (their dx
 *                  shares summed afterwards in group order).
 * Only the first 2^31-byte chunk of a batch larger than that is described.
 * MCK_ERR_INVALID_ARG / MCK_ERR_UNSUPPORTED as for mck_fastfood_backward.
 */
typedef struct mck_backward_shape {
    int32_t rows_per_pass;
    int32_t passes;
    int32_t esplit;
    int32_t reserved;
    int64_t rowblocks;
} mck_backward_shape;
mck_status mck_backward_launch_shape(int64_t batch, int64_t d, int64_t E, mck_backward_shape* out);

/*
 * Explicit-parameter forms of the feature map and its adjoint (equations
 * "mckernel" and "mcfeatures" with the diagonals and the permutation given
 * instead of generated: section "Empirical Analysis and Experiments" learns
 * C, G and B, so they become free real diagonals).
 * B, G, S (float) and perm (int32, a permutation of
 * 0..n-1; entries are reduced mod n) are caller-provided E x n device arrays,
 * with n = mck_padded_dim(d) given explicitly (must match) and S including
 * every scale.  These calls allocate a small temporary plan (E x n x 12
 * bytes) on `stream` (stream-ordered).
 */
mck_status mck_fastfood_forward_p(const float* x, int64_t batch, int64_t d, int64_t n, int64_t E, const float* B,
                                  const int32_t* perm, const float* G, const float* S, float* phi,
                                  mck_stream stream);

mck_status mck_fastfood_backward_p(const float* x, const float* dphi, int64_t batch, int64_t d, int64_t n,
                                   int64_t E, const float* B, const int32_t* perm, const float* G, const float* S,
                                   float* dx, float* dB, float* dG, float* dS, mck_stream stream);

/*
 * mck_fastfood_backward_p for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, results (bit-identical) and errors as
 * mck_fastfood_backward_p, and it calls no allocator.  Its temporaries (the
 * backward's parameter copies, the per-block partial sums of dB, dG, dS and
 * the dx slices of split expansions) live in one static device array of
 * MCK_NOALLOC_SCRATCH_BYTES, which each GPU the library runs this call on
 * holds from the call's first use there until the process ends.  A problem
 * whose temporaries exceed it fails with MCK_ERR_UNSUPPORTED before anything
 * is enqueued; the message gives the bytes needed.  With rowblocks and
 * esplit as mck_backward_launch_shape reports them, and 256-byte alignment
 * of each part, they are 4 E (max(n, min(64 n, 1024)) + 2 n) (parameter
 * copies) + 12 n E rowblocks (partial sums, when dB, dG or dS is requested)
 * + 4 esplit batch d (dx slices, when dx is requested and esplit > 1):
 * 50.5 MB at batch 8192, d = 784, E = 16.
 * All calls on one GPU share that array: calls that overlap on one GPU (on
 * different streams or threads) race, and the caller must order them.
 */
#define MCK_NOALLOC_SCRATCH_BYTES (64u << 20)
mck_status mck_fastfood_backward_p_noalloc(const float* x, const float* dphi, int64_t batch, int64_t d, int64_t n,
                                           int64_t E, const float* B, const int32_t* perm, const float* G,
                                           const float* S, float* dx, float* dB, float* dG, float* dS,
                                           mck_stream stream);

/*
 * Generator self-check: the FP32 Box-Muller pair of the generator for `count`
 * pairs of hash words (a[k], b[k]) -> (g0[k], g1[k]); lets a test compare the
 * device generator with an independent implementation over all 2^24 inputs.
 */
mck_status mck_gen_boxmuller(const uint32_t* a, const uint32_t* b, int64_t count, float* g0, float* g1,
                             mck_stream stream);

/*
 * Classifier head of the training step (section "Empirical Analysis and
 * Experiments": softmax(W phi + b) on the McKernel features, trained with
 * cross-entropy).  logits: batch x C (row-major), labels: batch int32 in
 * [0, C).  Writes dlogits (batch x C) = (softmax(logits) - onehot(labels)) /
 * batch, the gradient of the mean loss; *loss = the mean cross-entropy and
 * db (C floats) = the column sums of dlogits, both summed in a fixed order
 * (loss and db may be NULL).  A label outside [0, C) makes that row's loss
 * and gradient NaN.  C in [1, 1024].  Allocates batch floats of scratch on
 * `stream` (stream-ordered).
 */
mck_status mck_softmax_xent(const float* logits, const int32_t* labels, int64_t batch, int64_t C, float* loss,
                            float* dlogits, float* db, mck_stream stream);

/*
 * The two products of the same head (section "Empirical Analysis and
 * Experiments") on F = 2nE features, for C in [1, 16] classes:
 *
 *   mck_head_logits:   logits[r][c] = b[c] + sum_j W[c][j] phi[r][j]
 *   mck_head_backward: dphi[r][j] = sum_c dlogits[r][c] W[c][j] and
 *                      dW[c][j] = sum_r dlogits[r][c] phi[r][j]
 *
 * phi, dphi: batch x F row-major; W, dW: C x F row-major; logits, dlogits:
 * batch x C.  F must be a multiple of 4 and phi, W, dphi, dW 16-byte
 * aligned (MCK_ERR_INVALID_ARG otherwise); C F < 2^29 (MCK_ERR_UNSUPPORTED
 * otherwise).  b may be NULL (no bias); dphi or dW may be NULL (not
 * computed); for a non-empty batch W and dlogits must be valid, and phi
 * when dW is requested.  Every sum runs in a fixed order, so results are
 * deterministic.  Partial sums live in scratch allocated on `stream`
 * (stream-ordered): batch C F / 8192 floats for the logits, at most 32 C F
 * for dW.  An empty batch gives dW = 0.
 */
mck_status mck_head_logits(const float* phi, const float* W, const float* b, int64_t batch, int64_t F, int64_t C,
                           float* logits, mck_stream stream);
mck_status mck_head_backward(const float* phi, const float* dlogits, const float* W, int64_t batch, int64_t F,
                             int64_t C, float* dphi, float* dW, mck_stream stream);

/*
 * One training step of the classifier softmax(W phi(x) + b) with
 * cross-entropy (section "Empirical Analysis and Experiments") on the
 * features of explicit diagonals B, perm, G, S (as for
 * mck_fastfood_forward_p; n = mck_padded_dim(d) <= 2^15, F = 2nE), minimised
 * by SGD (section "Large-scale Machine Learning"):
 *
 *   phi = phi(x); logits = phi W^T + b; *loss = mean cross-entropy;
 *   dW, db, dB, dG, dS (and dx if non-NULL) = gradients of the mean loss;
 *   with lr != 0, W -= lr dW, b -= lr db, B -= lr dB, G -= lr dG,
 *   S -= lr dS in place afterwards (perm stays fixed).
 *
 * labels: batch int32 in [0, C) (a label outside makes the loss NaN);
 * logits (batch x C) is written when non-NULL; W, dW: C x F, 16-byte
 * aligned; C in [1, 16]; batch >= 1.  The gradients are those of the
 * parameters before the update.  One plan derivation serves the forward
 * and the adjoint.  For n = 1024 and C <= 10 the head is fused into the
 * feature-map kernels and phi never reaches device memory: the logits come
 * out of the forward, and phi is recomputed for dW and dphi; scratch is
 * batch F floats for dphi plus partial sums.  Otherwise phi and dphi are
 * materialised (2 batch F floats of scratch).  Scratch is allocated on
 * `stream` (stream-ordered).  Every sum has a fixed order: the step is
 * deterministic.
 */
mck_status mck_fastfood_train_step(const float* x, const int32_t* labels, int64_t batch, int64_t d, int64_t n,
                                   int64_t E, int64_t C, float* W, float* b, float* B, const int32_t* perm, float* G,
                                   float* S, float lr, float* loss, float* logits, float* dW, float* db, float* dB,
                                   float* dG, float* dS, float* dx, mck_stream stream);

/*
 * y += alpha x over `count` floats (the SGD update w <- w - gamma grad of
 * section "Large-scale Machine Learning", with alpha = -gamma).  y and x
 * must not overlap unless equal.
 */
mck_status mck_axpy(float* y, const float* x, int64_t count, float alpha, mck_stream stream);

/* Frees every cached plan (waits for the device first) except those held by
 * a live mck_batched_graph or a call in progress on another thread, and
 * the cached blocks of the temporaries.  Plans that calls under
 * stream capture used are freed too: graphs captured from library calls
 * must be destroyed before this is called. */
void mck_shutdown(void);

#ifdef __cplusplus
}
#endif

#endif /* MCKERNEL_H */
