// runtime.cpp -- host side of the C interface in include/mckernel.h:
// argument validation, the per-device parameter-plan cache, variant selection
// and kernel launches.  Every computation of the hot path runs in the HIP
// kernels of kernels.hip and generator.hip; this file only moves pointers.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <list>
#include <map>
#include <vector>
#include <mutex>
#include <new>
#include <string>

#include "mckernel.h"
#include "launch.hpp"
#include "temp_slots.hpp"
#include "plan_cache.hpp"

namespace {

thread_local std::string g_last_error;

mck_status fail(mck_status st, const std::string& msg)
{
    g_last_error = msg;
    return st;
}

mck_status hip_fail(hipError_t err, const char* where)
{
    return fail(MCK_ERR_HIP, std::string(where) + ": " + hipGetErrorString(err));
}

// Temporaries.  Each device keeps a few cached blocks, each with an event
// recorded after the last launch of the call that used it.  A call takes a
// free block, preferring one last used on its own stream (stream order alone
// protects it); a block last used on another stream is taken after making
// this stream wait, on the device, for that event.  So a call never waits on
// the host for earlier work, which the stream-ordered allocator does here:
// an allocation and a free on a busy stream return only once the stream has
// drained.  A call under stream capture takes graph-owned stream-ordered
// memory; one that finds every block busy (calls in progress on other host
// threads) takes stream-ordered memory from a pool that keeps what is freed.
// Streams are told apart by their handles.
constexpr int kTempSlots = 8;
struct TempSlot {
    char* ptr = nullptr;
    size_t bytes = 0;
    hipEvent_t done = nullptr;
    hipStream_t last = nullptr;
    bool used = false;  // `done` marks the end of the last call that used it
    bool busy = false;  // taken by a call that has not released it yet
};
struct DeviceTemps {
    TempSlot slot[kTempSlots];
    hipMemPool_t pool = nullptr;
};
std::mutex g_temp_mutex;
std::map<int, DeviceTemps> g_temps;

hipError_t pool_alloc(DeviceTemps& dt, int dev, void** p, size_t bytes, hipStream_t s)
{
    if (dt.pool == nullptr) {
        hipMemPoolProps props;
        std::memset(&props, 0, sizeof(props));
        props.allocType = hipMemAllocationTypePinned;
        props.location.type = hipMemLocationTypeDevice;
        props.location.id = dev;
        hipError_t err = hipMemPoolCreate(&dt.pool, &props);
        if (err != hipSuccess) {
            dt.pool = nullptr;
            return err;
        }
        uint64_t keep = UINT64_MAX;
        err = hipMemPoolSetAttribute(dt.pool, hipMemPoolAttrReleaseThreshold, &keep);
        if (err != hipSuccess) {
            (void)hipMemPoolDestroy(dt.pool);
            dt.pool = nullptr;
            return err;
        }
    }
    return hipMallocFromPoolAsync(p, bytes, dt.pool, s);
}

// Makes `dev` current for its lifetime (allocations and events belong to
// the current device, which need not be the stream's).
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev)
            (void)hipSetDevice(dev);
        else
            prev = -1;
    }
    ~DeviceGuard()
    {
        if (prev >= 0)
            (void)hipSetDevice(prev);
    }
};

hipError_t temp_alloc(void** p, size_t bytes, hipStream_t s)
{
    *p = nullptr;
    int dev = 0;
    hipError_t err = hipStreamGetDevice(s, &dev);
    if (err != hipSuccess)
        return err;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    err = hipStreamIsCapturing(s, &cap);
    if (err != hipSuccess)
        return err;
    std::lock_guard<std::mutex> lock(g_temp_mutex);
    const DeviceGuard on_dev(dev);
    DeviceTemps& dt = g_temps[dev];
    if (cap != hipStreamCaptureStatusNone)
        return hipMallocAsync(p, bytes, s);  // graph-owned memory
    const int pick = mck::pick_temp_slot(dt.slot, kTempSlots, s, bytes);
    if (pick < 0)
        return pool_alloc(dt, dev, p, bytes, s);
    TempSlot& t = dt.slot[pick];
    if (t.bytes < bytes) {
        // grow (rare): the old block is freed once its last user is done
        if (t.ptr != nullptr) {
            if (t.used)
                (void)hipEventSynchronize(t.done);
            (void)hipFree(t.ptr);
            t.ptr = nullptr;
            t.bytes = 0;
        }
        size_t want = bytes + bytes / 4;
        want = (want + (size_t(1) << 20) - 1) & ~((size_t(1) << 20) - 1);
        void* q = nullptr;
        err = hipMalloc(&q, want);
        if (err != hipSuccess)
            return pool_alloc(dt, dev, p, bytes, s);
        t.ptr = static_cast<char*>(q);
        t.bytes = want;
        t.used = false;
    }
    if (t.done == nullptr) {
        err = hipEventCreateWithFlags(&t.done, hipEventDisableTiming);
        if (err != hipSuccess) {
            t.done = nullptr;
            return err;
        }
    }
    if (t.used && t.last != s) {
        err = hipStreamWaitEvent(s, t.done, 0);
        if (err != hipSuccess)
            return err;
    }
    t.busy = true;
    *p = t.ptr;
    return hipSuccess;
}

// Ends a temporary's use by the calling call: the block is free for the next
// call once the work enqueued on `s` so far is done.
void temp_free(void* p, hipStream_t s)
{
    if (p == nullptr)
        return;
    {
        std::lock_guard<std::mutex> lock(g_temp_mutex);
        for (auto& kv : g_temps) {
            for (TempSlot& t : kv.second.slot) {
                if (t.busy && t.ptr == p) {
                    const hipError_t err = hipEventRecord(t.done, s);
                    if (err != hipSuccess) {
                        // no event: wait here rather than hand out a block in use
                        (void)hipStreamSynchronize(s);
                        t.used = false;
                    } else {
                        t.used = true;
                    }
                    t.last = s;
                    t.busy = false;
                    return;
                }
            }
        }
    }
    (void)hipFreeAsync(p, s);
}

bool is_pow2(int64_t v) { return v >= 1 && (v & (v - 1)) == 0; }

int log2i(int64_t v)
{
    int m = 0;
    while ((int64_t(1) << m) < v)
        ++m;
    return m;
}

int64_t padded_dim(int64_t d)
{
    if (d < 1)
        return 0;
    int64_t n = 2;
    while (n < d)
        n *= 2;
    return n > MCK_MAX_N_LONG ? 0 : n;
}

// Single-pass kernels only (backward, projection, explicit parameters).
mck_status check_single_pass(int64_t n)
{
    if (n > MCK_MAX_N)
        return fail(MCK_ERR_UNSUPPORTED, "n > MCK_MAX_N is supported by mck_fwht and the forward feature map only");
    return MCK_OK;
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// Feature scale c = 1/sqrt(nE) of phi (equation mcfeatures).
float feature_scale(int64_t n, int64_t E) { return (float)(1.0 / std::sqrt((double)n * (double)E)); }

// Calibration code -> RBF-Matern sample count t (0 = RBF).  MCK_CALIB_MATERN
// is the paper's t = 40; MCK_CALIB_MATERN_T(t) = 0x100 + t for t in 1..255.
constexpr int64_t kMaternMaxN = 2048;

mck_status check_calib(int calib, int64_t n, int* t)
{
    if (calib == MCK_CALIB_RBF) {
        *t = 0;
        return MCK_OK;
    }
    if (calib == MCK_CALIB_MATERN)
        *t = 40;
    else if (calib > 0x100 && calib <= 0x1ff)
        *t = calib - 0x100;
    else
        return fail(MCK_ERR_INVALID_ARG, "unknown calibration");
    if (n > kMaternMaxN)
        return fail(MCK_ERR_UNSUPPORTED, "RBF-Matern calibration supports n <= 2048");
    return MCK_OK;
}

mck_status check_sigma(double sigma)
{
    if (!(sigma > 0.0) || !std::isfinite(sigma))
        return fail(MCK_ERR_INVALID_ARG, "sigma must be finite and > 0");
    return MCK_OK;
}

mck_status check_common(int64_t batch, int64_t d, int64_t E, int64_t* n_out)
{
    if (batch < 0)
        return fail(MCK_ERR_INVALID_ARG, "batch must be >= 0");
    if (d < 1)
        return fail(MCK_ERR_INVALID_ARG, "d must be >= 1");
    if (E < 1 || E > (int64_t(1) << 20))
        return fail(MCK_ERR_INVALID_ARG, "E must be in [1, 2^20]");
    const int64_t n = padded_dim(d);
    if (n == 0)
        return fail(MCK_ERR_UNSUPPORTED, "padded dimension exceeds MCK_MAX_N_LONG");
    if (E * (n > 2048 ? n : 2048) > (int64_t(1) << 28))
        return fail(MCK_ERR_UNSUPPORTED, "E * n too large (parameter arrays limited to 2^28 entries)");
    if (d > (int64_t(1) << 30) || batch > (int64_t(1) << 40))
        return fail(MCK_ERR_INVALID_ARG, "size out of range");
    *n_out = n;
    return MCK_OK;
}

// ------------------------------------------------------------------ forward tuning
// Launch choice of the single-pass forward for n = 2^M: the register split P
// (register bits per lane layout) and the grid target in waves.  One table
// per device; every forward of that n (plain, 16-bit, grouped, explicit
// parameters) launches with the current entry.
struct FwdTune {
    int P;
    int waves;
};

std::mutex g_tune_mutex;
std::map<std::pair<int, int>, FwdTune> g_tune;  // (device, M) -> choice; absent = default

int alt_split(int M) { return mck::fwd_split_default(M) == 4 ? 5 : 4; }

FwdTune default_tuning(int M) { return FwdTune{mck::fwd_split_default(M), mck::kFwdWavesDefault}; }

FwdTune current_tuning(int M)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return default_tuning(M);
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    const auto it = g_tune.find({dev, M});
    return it == g_tune.end() ? default_tuning(M) : it->second;
}

// ------------------------------------------------------------------ plan cache
struct Plan {
    int pins = 0;           // > 0 while a call or a recorded graph holds it: not evicted
    bool captured = false;  // used by a call under stream capture: not evicted (mck_shutdown frees it)
    int device = 0;
    uint32_t seed = 0;
    int64_t n = 0, E = 0;
    double sigma = 0.0;
    int calib = 0;
    void* block = nullptr;
    size_t bytes = 0;
    float* B = nullptr;
    int32_t* perm = nullptr;
    float* G = nullptr;
    double* S64 = nullptr;
    float* S32 = nullptr;
    double* norm2 = nullptr;
    uint32_t* goffF = nullptr;  // forward gather offsets (default register split)
    float* GsF = nullptr;       // forward G (destination order at P = 4, source order at P = 5)
    uint32_t* goffF2 = nullptr; // the same for the other compiled split (null if none)
    float* GsF2 = nullptr;
    uint32_t* goffB = nullptr;  // backward gather offsets
    float* GkB = nullptr;       // G in destination order, backward layout
    float* Sh = nullptr;        // S / (2 pi)
    // n > MCK_MAX_N: Pi as buckets between 2^15-element source and
    // destination chunks (C = n / 2^15 of each, layout in launch.hpp)
    uint32_t* packA = nullptr;
    uint16_t* dstB = nullptr;
    int32_t* pdelta = nullptr;
    float* Gx = nullptr;
    int32_t* bscratch = nullptr;  // build scratch
    // n = 2^16 (the one-block row kernel): sign words of B, and Pi as the
    // outer Benes stage (switch words, gather indices of each half, G)
    uint32_t* Bw = nullptr;
    uint32_t* Pw = nullptr;
    uint32_t* Po = nullptr;
    float* Pg = nullptr;
};

std::mutex g_mutex;
mck::PlanList<Plan> g_plans;  // guarded by g_mutex

struct GlobalCache {
    std::mutex& mutex() { return g_mutex; }
    mck::PlanList<Plan>& list() { return g_plans; }
};
GlobalCache g_cache;
constexpr size_t kMaxPlans = 32;
constexpr size_t kMaxPlanBytes = size_t(2) << 30;

size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

void free_plan(Plan& p)
{
    if (p.block) {
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(p.device);
        (void)hipFree(p.block);
        (void)hipSetDevice(cur);
        p.block = nullptr;
    }
}

// Returns the plan for the arguments, building it on `stream` if needed.
mck_status get_plan(uint32_t seed, int64_t n, int64_t E, double sigma, int calib, hipStream_t stream,
                    Plan** out, bool pin = false)
{
    int dev = 0;
    hipError_t err = hipGetDevice(&dev);
    if (err != hipSuccess)
        return hip_fail(err, "hipGetDevice");
    std::lock_guard<std::mutex> lock(g_mutex);
    Plan* hit = g_plans.find(
        [&](const Plan& q) {
            return q.device == dev && q.seed == seed && q.n == n && q.E == E && q.sigma == sigma && q.calib == calib;
        },
        pin);
    if (hit != nullptr) {
        *out = hit;
        return MCK_OK;
    }
    Plan p;
    p.device = dev;
    p.seed = seed;
    p.n = n;
    p.E = E;
    p.sigma = sigma;
    p.calib = calib;
    const size_t en = (size_t)(n * E);
    int64_t gf = 0, gb = 0;
    mck::plan_elems(log2i(n), &gf, &gb);
    const bool pair = n == 2 * MCK_MAX_N;
    const size_t C = n > MCK_MAX_N && !pair ? (size_t)(n / MCK_MAX_N) : 0;
    const size_t ecc = (size_t)E * C * C * 4;
    const int M = log2i(n);
    const bool two = n <= MCK_MAX_N && mck::fwd_split_ok(M, alt_split(M));
    size_t off[22], total = 0;
    const size_t sz[22] = {en * 4, en * 4, en * 4, en * 8, en * 4, (size_t)E * 8,
                           (size_t)gf * E * 4, en * 4, (size_t)gb * E * 4, en * 4, en * 4,
                           C ? en * 4 : 0, C ? en * 2 : 0, ecc, 3 * ecc + (size_t)E * C * 8, C ? en * 4 : 0,
                           two ? (size_t)gf * E * 4 : 0, two ? en * 4 : 0, pair ? en / 8 : 0,
                           pair ? en / 8 : 0, pair ? en * 2 : 0, pair ? en * 4 : 0};
    for (int i = 0; i < 22; ++i) {
        off[i] = total;
        total += align_up(sz[i]);
    }
    // evict least recently used plans that no call or graph holds
    g_plans.make_room(total, kMaxPlans, kMaxPlanBytes, free_plan);
    err = hipMalloc(&p.block, total);
    if (err != hipSuccess) {
        p.block = nullptr;
        return fail(MCK_ERR_NO_MEMORY, std::string("plan allocation: ") + hipGetErrorString(err));
    }
    p.bytes = total;
    char* b = static_cast<char*>(p.block);
    p.B = reinterpret_cast<float*>(b + off[0]);
    p.perm = reinterpret_cast<int32_t*>(b + off[1]);
    p.G = reinterpret_cast<float*>(b + off[2]);
    p.S64 = reinterpret_cast<double*>(b + off[3]);
    p.S32 = reinterpret_cast<float*>(b + off[4]);
    p.norm2 = reinterpret_cast<double*>(b + off[5]);
    p.goffF = reinterpret_cast<uint32_t*>(b + off[6]);
    p.GsF = reinterpret_cast<float*>(b + off[7]);
    p.goffB = reinterpret_cast<uint32_t*>(b + off[8]);
    p.GkB = reinterpret_cast<float*>(b + off[9]);
    p.Sh = reinterpret_cast<float*>(b + off[10]);
    if (C) {
        p.packA = reinterpret_cast<uint32_t*>(b + off[11]);
        p.dstB = reinterpret_cast<uint16_t*>(b + off[12]);
        p.pdelta = reinterpret_cast<int32_t*>(b + off[13]);
        p.bscratch = reinterpret_cast<int32_t*>(b + off[14]);
        p.Gx = reinterpret_cast<float*>(b + off[15]);
    }
    if (two) {
        p.goffF2 = reinterpret_cast<uint32_t*>(b + off[16]);
        p.GsF2 = reinterpret_cast<float*>(b + off[17]);
    }
    if (pair) {
        p.Bw = reinterpret_cast<uint32_t*>(b + off[18]);
        p.Pw = reinterpret_cast<uint32_t*>(b + off[19]);
        p.Po = reinterpret_cast<uint32_t*>(b + off[20]);
        p.Pg = reinterpret_cast<float*>(b + off[21]);
    }
    int matern_t = 0;
    {
        const mck_status cst = check_calib(calib, n, &matern_t);
        if (cst != MCK_OK) {
            free_plan(p);
            return cst;
        }
    }
    err = mck::launch_generate(seed, n, E, sigma, matern_t, p.B, p.perm, p.G, p.S64, p.S32, p.norm2, stream);
    if (err == hipSuccess)
        err = n > MCK_MAX_N ? mck::launch_sh(p.S64, p.Sh, n * E, stream)
                            : mck::launch_derive(M, mck::fwd_split_default(M), E, p.perm, p.G, p.B, p.S64, p.S32,
                                                 p.goffF, p.GsF, p.goffB, p.GkB, p.Sh, stream);
    if (err == hipSuccess && two)
        err = mck::launch_derive_fwd(M, alt_split(M), E, p.perm, p.G, p.B, p.goffF2, p.GsF2, stream);
    if (err == hipSuccess && C)
        err = mck::launch_buckets(log2i(n), E, p.perm, p.G, p.packA, p.dstB, p.pdelta, p.Gx, p.bscratch, stream);
    if (err == hipSuccess && pair)
        err = mck::launch_pair_plan(E, p.perm, p.G, p.B, p.Bw, p.Pw, p.Po, p.Pg, stream);
    if (err == hipSuccess)
        err = hipStreamSynchronize(stream);  // the plan may be used from other streams next
    if (err != hipSuccess) {
        free_plan(p);
        return hip_fail(err, "plan generation");
    }
    *out = g_plans.insert(std::move(p), pin);
    return MCK_OK;
}

// The plan of one call, pinned from lookup until the call has enqueued its
// last launch, so that an eviction or mck_shutdown on another thread cannot
// free it in between.  A call made while its stream is being captured into
// a graph marks the plan `captured`: the graph reads it at every replay, so
// eviction never frees it (mck_shutdown does).
class PlanHold : public mck::PinnedPlan<GlobalCache, Plan> {
public:
    PlanHold() : mck::PinnedPlan<GlobalCache, Plan>(g_cache) {}

    mck_status acquire(uint32_t seed, int64_t n, int64_t E, double sigma, int calib, hipStream_t s)
    {
        release();
        hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
        const hipError_t err = hipStreamIsCapturing(s, &cap);
        if (err != hipSuccess)
            return hip_fail(err, "hipStreamIsCapturing");
        Plan* p = nullptr;
        const mck_status st = get_plan(seed, n, E, sigma, calib, s, &p, true);
        if (st != MCK_OK)
            return st;
        if (cap != hipStreamCaptureStatusNone) {
            std::lock_guard<std::mutex> lock(g_mutex);
            p->captured = true;
        }
        adopt(p);
        return MCK_OK;
    }
};


struct FwdArrays {
    const uint32_t* goff;
    const float* Gs;
};

// The plan's forward arrays for register split P (the default split's when
// the plan holds no others).
FwdArrays fwd_arrays(const Plan* p, int P)
{
    if (P != mck::fwd_split_default(log2i(p->n)) && p->goffF2)
        return FwdArrays{p->goffF2, p->GsF2};
    return FwdArrays{p->goffF, p->GsF};
}

struct TempPlan {
    int PF = 0;  // register split of goffF, GsF
    void* block = nullptr;
    uint32_t* goffF = nullptr;
    float* GsF = nullptr;
    uint32_t* goffB = nullptr;
    float* GkB = nullptr;
    float* Sh = nullptr;
};

// Bytes of a temporary plan of register split PF: forward gather offsets,
// backward ones (none when both directions use PF), G in both layouts, Sh.
struct TempPlanSizes {
    size_t a = 0, af = 0, ab = 0;
    size_t bytes() const { return af + ab + 3 * a; }
};

TempPlanSizes temp_plan_sizes(int64_t n, int64_t E, int PF)
{
    int64_t gf = 0, gb = 0;
    mck::plan_elems(log2i(n), &gf, &gb);
    TempPlanSizes z;
    z.a = align_up((size_t)(n * E) * 4);
    z.af = align_up((size_t)gf * E * 4);
    z.ab = PF == mck::bwd_split(log2i(n)) ? 0 : align_up((size_t)gb * E * 4);
    return z;
}

// The arrays in mem (temp_plan_sizes(n, E, PF).bytes(), owned by the
// caller; tp->block stays null) or in an allocation of their own (tp->block).
mck_status make_temp_plan(int64_t n, int64_t E, const int32_t* perm, const float* G, const float* S,
                          hipStream_t s, TempPlan* tp, int force_p = 0, char* mem = nullptr)
{
    tp->PF = force_p ? force_p : current_tuning(log2i(n)).P;
    const TempPlanSizes z = temp_plan_sizes(n, E, tp->PF);
    const size_t a = z.a, af = z.af, ab = z.ab;
    const bool shared = ab == 0;  // the same register split in both directions: one set of offsets
    hipError_t err = hipSuccess;
    if (mem == nullptr) {
        err = temp_alloc(&tp->block, z.bytes(), s);
        if (err != hipSuccess) {
            tp->block = nullptr;
            return fail(MCK_ERR_NO_MEMORY, std::string("temporary plan: ") + hipGetErrorString(err));
        }
    }
    char* b = mem ? mem : static_cast<char*>(tp->block);
    tp->goffF = reinterpret_cast<uint32_t*>(b);
    tp->goffB = shared ? tp->goffF : reinterpret_cast<uint32_t*>(b + af);
    tp->GsF = reinterpret_cast<float*>(b + af + ab);
    tp->GkB = reinterpret_cast<float*>(b + af + ab + a);
    tp->Sh = reinterpret_cast<float*>(b + af + ab + 2 * a);
    err = mck::launch_derive(log2i(n), tp->PF, E, perm, G, nullptr, nullptr, S, tp->goffF, tp->GsF, tp->goffB,
                             tp->GkB, tp->Sh, s);
    if (err != hipSuccess) {
        if (tp->block)
            temp_free(tp->block, s);
        tp->block = nullptr;
        return hip_fail(err, "derive kernel");
    }
    return MCK_OK;
}

bool vec_ok(const void* a, const void* b, int64_t d, int64_t n)
{
    return aligned16(a) && aligned16(b) && (d % 4 == 0) && n >= 4;
}

// Rows per backward launch: the x, dx and dphi ranges of a launch stay below
// 2^31 bytes.
int64_t backward_rows_per_launch(int64_t d, int64_t n, int64_t E)
{
    const int64_t lim = (int64_t(1) << 31) - 4096;
    const int64_t row_bytes = 4 * (2 * n * E > d ? 2 * n * E : d);
    return lim / row_bytes < 1 ? 1 : lim / row_bytes;
}

// Device temporaries of one adjoint call: the per-block partial sums of dS,
// dG, dB (all launches of the call, reduced once at the end) and the dx
// slices of one launch whose expansions are split over block groups (reused
// by the next launch: the launches are ordered on the stream).
struct BwdScratch {
    int64_t total_blocks = 0;
    size_t partial_bytes = 0;
    size_t dxs_bytes = 0;
    size_t bytes() const { return align_up(partial_bytes) + align_up(dxs_bytes); }
};

BwdScratch backward_scratch(int64_t batch, int64_t d, int64_t n, int64_t E, bool want_dx, bool want_params)
{
    BwdScratch b;
    const int M = log2i(n);
    const int64_t rows_per = backward_rows_per_launch(d, n, E);
    for (int64_t r0 = 0; r0 < batch; r0 += rows_per) {
        const int64_t rows = batch - r0 < rows_per ? batch - r0 : rows_per;
        const mck::BwdGeometry geo = mck::backward_geometry(M, rows, (int)d, E);
        b.total_blocks += geo.rowblocks;
        if (want_dx && geo.esplit > 1) {
            const size_t need = (size_t)(geo.esplit * rows * d) * sizeof(float);
            b.dxs_bytes = need > b.dxs_bytes ? need : b.dxs_bytes;
        }
    }
    if (want_params)
        b.partial_bytes = (size_t)b.total_blocks * E * 3 * n * sizeof(float);
    return b;
}

// The adjoint's launches.  ws: the call's temporaries (BwdScratch layout:
// partials, then dx slices), or null to allocate them on the stream.
// With uB, uG, uS (nullable; the training step's B, G, S) the final
// partial-sum pass also applies u += alpha (dB, dG, dS).
mck_status run_backward(const float* x, const float* dphi, int64_t batch, int64_t d, int64_t n, int64_t E,
                        const float* B, const uint32_t* goff, const float* Gk, const float* S32, const float* Sh,
                        float* dx, float* dB, float* dG, float* dS, hipStream_t s, char* ws = nullptr,
                        float* uB = nullptr, float* uG = nullptr, float* uS = nullptr, float alpha = 0.f,
                        const mck::GroupSum* extra = nullptr)
{
    const int M = log2i(n);
    const bool want_params = dB || dG || dS;
    const int64_t rows_per = backward_rows_per_launch(d, n, E);
    const BwdScratch need = backward_scratch(batch, d, n, E, dx != nullptr, want_params);
    float* partial = nullptr;
    float* dxs_ws = ws ? reinterpret_cast<float*>(ws + align_up(need.partial_bytes)) : nullptr;
    hipError_t err;
    if (want_params) {
        if (ws) {
            partial = reinterpret_cast<float*>(ws);
        } else {
            err = temp_alloc(reinterpret_cast<void**>(&partial), need.partial_bytes, s);
            if (err != hipSuccess)
                return fail(MCK_ERR_NO_MEMORY, std::string("backward partials: ") + hipGetErrorString(err));
        }
    }
    auto release = [&](void* p) {
        if (p && !ws)
            temp_free(p, s);
    };
    const bool vec = vec_ok(x, dphi, d, n) && (dx == nullptr || aligned16(dx));
    const float cs = feature_scale(n, E);
    err = hipSuccess;
    int64_t done_blocks = 0;
    for (int64_t r0 = 0; r0 < batch && err == hipSuccess; r0 += rows_per) {
        const int64_t rows = batch - r0 < rows_per ? batch - r0 : rows_per;
        const mck::BwdGeometry geo = mck::backward_geometry(M, rows, (int)d, E);
        float* part = partial ? partial + (size_t)done_blocks * E * 3 * n : nullptr;
        float* dxr = dx ? dx + r0 * d : nullptr;
        float* dxs = nullptr;  // per expansion group dx slices
        if (dx && geo.esplit > 1) {
            if (ws) {
                dxs = dxs_ws;
            } else {
                err = temp_alloc(reinterpret_cast<void**>(&dxs), (size_t)(geo.esplit * rows * d) * sizeof(float),
                                     s);
                if (err != hipSuccess) {
                    release(partial);
                    return fail(MCK_ERR_NO_MEMORY, std::string("backward dx slices: ") + hipGetErrorString(err));
                }
            }
        }
        err = mck::launch_backward(M, vec && (dxs == nullptr || aligned16(dxs)), x + r0 * d, dphi + r0 * 2 * n * E,
                                   rows, (int)d, E, B, goff, Gk, S32, Sh, cs, dxs ? dxs : dxr, part, geo, s);
        if (dxs) {
            if (err == hipSuccess)
                err = mck::launch_sum_groups(dxs, geo.esplit, rows * d, dxr, s);
            release(dxs);
        }
        done_blocks += geo.rowblocks;
    }
    // `extra` (a group sum of the caller's) rides in the reduction's launch
    if (err == hipSuccess && want_params)
        err = mck::launch_reduce(partial, need.total_blocks, E, n, dS, dG, dB, s, uS, uG, uB, alpha, extra);
    else if (err == hipSuccess && extra != nullptr)
        err = mck::launch_sum_groups(extra->part, extra->groups, extra->count, extra->out, s, extra->y,
                                     extra->alpha);
    release(partial);
    if (err != hipSuccess)
        return hip_fail(err, "backward launch");
    return MCK_OK;
}

}  // namespace

// ------------------------------------------------------------------ static scratch
// The temporaries of mck_fastfood_backward_p_noalloc live in this array
// instead of allocations.  In host code its name stands for a host-side
// shadow, not for device memory: the device address of each GPU's copy is
// looked up once per device (scratch_on_current_device) and only that
// address is handed to kernels.
static __device__ __align__(256) unsigned char scratch[MCK_NOALLOC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mutex;
std::map<int, char*> g_scratch_addr;  // device ordinal -> address of its copy of `scratch`

mck_status scratch_on_current_device(char** out)
{
    int dev = 0;
    hipError_t err = hipGetDevice(&dev);
    if (err != hipSuccess)
        return hip_fail(err, "hipGetDevice");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    const auto it = g_scratch_addr.find(dev);
    if (it != g_scratch_addr.end()) {
        *out = it->second;
        return MCK_OK;
    }
    void* p = nullptr;
    err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (err != hipSuccess || p == nullptr)
        return hip_fail(err != hipSuccess ? err : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    g_scratch_addr[dev] = static_cast<char*>(p);
    *out = static_cast<char*>(p);
    return MCK_OK;
}

}  // namespace

extern "C" {

int64_t mck_padded_dim(int64_t d) { return padded_dim(d); }

const char* mck_status_string(mck_status status)
{
    switch (status) {
    case MCK_OK: return "success";
    case MCK_ERR_INVALID_ARG: return "invalid argument";
    case MCK_ERR_UNSUPPORTED: return "unsupported";
    case MCK_ERR_HIP: return "HIP runtime error";
    case MCK_ERR_NO_MEMORY: return "out of device memory";
    }
    return "unknown status";
}

const char* mck_last_error(void) { return g_last_error.c_str(); }

mck_status mck_fwht(float* data, int64_t batch, int64_t n, mck_stream stream)
{
    if (batch < 0)
        return fail(MCK_ERR_INVALID_ARG, "batch must be >= 0");
    if (!is_pow2(n))
        return fail(MCK_ERR_INVALID_ARG, "n must be a power of two >= 1");
    if (n > MCK_MAX_N_LONG)
        return fail(MCK_ERR_UNSUPPORTED, "n exceeds MCK_MAX_N_LONG");
    if (batch > 0 && data == nullptr)
        return fail(MCK_ERR_INVALID_ARG, "data is NULL");
    if (batch == 0 || n == 1)
        return MCK_OK;
    if (n > MCK_MAX_N && !aligned16(data))
        return fail(MCK_ERR_INVALID_ARG, "data must be 16-byte aligned for n > MCK_MAX_N");
    if (batch > (int64_t(1) << 40) / n)
        return fail(MCK_ERR_INVALID_ARG, "batch * n out of range");
    const hipError_t err = n > MCK_MAX_N
                               ? mck::launch_fwht_long(log2i(n), data, batch, true, static_cast<hipStream_t>(stream))
                               : mck::launch_fwht(log2i(n), data, batch, aligned16(data) && n >= 4,
                                                  static_cast<hipStream_t>(stream));
    return err == hipSuccess ? MCK_OK : hip_fail(err, "mck_fwht");
}

mck_status mck_fastfood_params(uint32_t seed, int64_t n, int64_t E, double sigma, mck_calibration calib, float* B,
                               int32_t* perm, float* G, float* S, double* S64, mck_stream stream)
{
    if (!is_pow2(n) || n < 2)
        return fail(MCK_ERR_INVALID_ARG, "n must be a power of two >= 2");
    if (n > MCK_MAX_N_LONG)
        return fail(MCK_ERR_UNSUPPORTED, "n exceeds MCK_MAX_N_LONG");
    if (E < 1 || E > (int64_t(1) << 20))
        return fail(MCK_ERR_INVALID_ARG, "E must be in [1, 2^20]");
    mck_status st = check_sigma(sigma);
    if (st != MCK_OK)
        return st;
    {
        int mt = 0;
        st = check_calib((int)calib, n, &mt);
        if (st != MCK_OK)
            return st;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    PlanHold p;
    st = p.acquire(seed, n, E, sigma, calib, s);
    if (st != MCK_OK)
        return st;
    const size_t en = (size_t)(n * E);
    hipError_t err = hipSuccess;
    if (B && err == hipSuccess)
        err = hipMemcpyAsync(B, p->B, en * 4, hipMemcpyDeviceToDevice, s);
    if (perm && err == hipSuccess)
        err = hipMemcpyAsync(perm, p->perm, en * 4, hipMemcpyDeviceToDevice, s);
    if (G && err == hipSuccess)
        err = hipMemcpyAsync(G, p->G, en * 4, hipMemcpyDeviceToDevice, s);
    if (S && err == hipSuccess)
        err = hipMemcpyAsync(S, p->S32, en * 4, hipMemcpyDeviceToDevice, s);
    if (S64 && err == hipSuccess)
        err = hipMemcpyAsync(S64, p->S64, en * 8, hipMemcpyDeviceToDevice, s);
    return err == hipSuccess ? MCK_OK : hip_fail(err, "mck_fastfood_params copy");
}

// Feature map for n > MCK_MAX_N.  The kernels address phi, x and the
// scratch per row, so only a row of phi must stay below 2^31 bytes.
// n = 2^16 takes the one-block row kernel (k_forward_pair), which needs no
// scratch.  Longer rows take the multi-pass path, in equal chunks of rows
// through two FP32 scratch buffers u, w of at most 2^27 floats each.
// Rows per launch of the multi-pass path.
static int64_t long_rows_per(int64_t batch, int64_t n)
{
    const int64_t max_rows = ((int64_t)1 << 27) / n;
    const int64_t nchunks = (batch + max_rows - 1) / max_rows;
    return (batch + nchunks - 1) / nchunks;
}

// Compute units of the current device (cached per device).
static int device_cus()
{
    static std::mutex mu;
    static std::map<int, int> cus;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return 256;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cus.find(dev);
    if (it != cus.end())
        return it->second;
    int c = 0;
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c < 8)
        c = 256;
    cus[dev] = c;
    return c;
}

// Blocks of the one-block row kernel for n = 2^16 (a multiple of 8).
static int64_t pair_blocks(int64_t batch, int64_t E) { return mck::pair_blocks(batch, E, device_cus()); }

// Scratch floats a long-vector feature map needs.
static int64_t long_scratch_floats(int64_t batch, int64_t n, int64_t E)
{
    if (n == 2 * MCK_MAX_N)
        return 0;
    return 2 * long_rows_per(batch, n) * n;
}

// Launches of the long-vector feature map with caller-provided scratch u
// (long_scratch_floats(batch, n, E) floats).
static mck_status forward_long_launch(const Plan* p, const void* x, int xt, int64_t batch, int64_t d, int64_t n,
                                      int64_t E, void* phi, int yt, float* u, hipStream_t s, float cs,
                                      const int8_t* xexp = nullptr)
{
    const int64_t xb = xt == 0 ? 4 : 2, yb = yt == 0 ? 4 : 2;
    const int64_t row_phi = 2 * n * E * yb;
    const uintptr_t xa = (uintptr_t)(4 * xb);
    const bool vec = reinterpret_cast<uintptr_t>(x) % xa == 0 && d % 4 == 0;
    hipError_t err = hipSuccess;
    if (n == 2 * MCK_MAX_N) {
        err = mck::launch_forward_pair(vec, xt, yt, x, batch, (int)d, E, p->Bw, p->Pw, p->Po, p->Pg, p->Sh, cs, phi,
                                       pair_blocks(batch, E), s, xexp);
        return err == hipSuccess ? MCK_OK : hip_fail(err, "long-vector forward launch");
    }
    const int64_t rows_per = long_rows_per(batch, n);
    float* w = u + rows_per * n;
    for (int64_t r0 = 0; r0 < batch && err == hipSuccess; r0 += rows_per) {
        const int64_t rows = batch - r0 < rows_per ? batch - r0 : rows_per;
        err = mck::launch_forward_long(log2i(n), vec, xt, yt, static_cast<const char*>(x) + r0 * d * xb, rows,
                                       (int)d, E, p->B, p->packA, p->dstB, p->pdelta, p->Gx, p->Sh, cs,
                                       static_cast<char*>(phi) + r0 * row_phi, u, w, s,
                                       xexp ? xexp + r0 : nullptr);
    }
    return err == hipSuccess ? MCK_OK : hip_fail(err, "long-vector forward launch");
}

static mck_status forward_long(const Plan* p, const void* x, int xt, int64_t batch, int64_t d, int64_t n, int64_t E,
                               void* phi, int yt, hipStream_t s, float cs, const int8_t* xexp = nullptr)
{
    const int64_t yb = yt == 0 ? 4 : 2;
    if (2 * n * E * yb > (int64_t(1) << 31) - 4096)
        return fail(MCK_ERR_UNSUPPORTED, "one row of phi exceeds 2^31 bytes");
    if (batch == 0)
        return MCK_OK;
    float* u = nullptr;
    const size_t ub = (size_t)long_scratch_floats(batch, n, E) * sizeof(float);
    if (ub > 0) {
        const hipError_t err = temp_alloc(reinterpret_cast<void**>(&u), ub, s);
        if (err != hipSuccess)
            return fail(MCK_ERR_NO_MEMORY, std::string("long-vector scratch: ") + hipGetErrorString(err));
    }
    const mck_status st = forward_long_launch(p, x, xt, batch, d, n, E, phi, yt, u, s, cs, xexp);
    if (u != nullptr)
        temp_free(u, s);
    return st;
}

static mck_status forward_common(const float* x, int64_t batch, int64_t d, int64_t E, uint32_t seed, double sigma,
                                 mck_calibration calib, float* out, bool trig, mck_stream stream)
{
    int64_t n = 0;
    mck_status st = check_common(batch, d, E, &n);
    if (st != MCK_OK)
        return st;
    st = check_sigma(sigma);
    if (st != MCK_OK)
        return st;
    {
        int mt = 0;
        st = check_calib((int)calib, n, &mt);
        if (st != MCK_OK)
            return st;
    }
    if (batch > 0 && (x == nullptr || out == nullptr))
        return fail(MCK_ERR_INVALID_ARG, "x or output is NULL");
    if (batch == 0)
        return MCK_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    PlanHold p;
    if (n > MCK_MAX_N && !trig)
        return check_single_pass(n);
    st = p.acquire(seed, n, E, sigma, calib, s);
    if (st != MCK_OK)
        return st;
    if (n > MCK_MAX_N)
        return forward_long(p.get(), x, 0, batch, d, n, E, out, 0, s, feature_scale(n, E));
    const FwdTune t = current_tuning(log2i(n));
    const FwdArrays a = fwd_arrays(p.get(), t.P);
    const hipError_t err = mck::launch_forward(log2i(n), t.P, t.waves, true, vec_ok(x, out, d, n), trig, x, batch,
                                               (int)d, E, p->B, a.goff, a.Gs, trig ? p->Sh : p->S32,
                                               feature_scale(n, E), out, s);
    return err == hipSuccess ? MCK_OK : hip_fail(err, "forward launch");
}

mck_status mck_fastfood_forward(const float* x, int64_t batch, int64_t d, int64_t E, uint32_t seed, double sigma,
                                mck_calibration calib, float* phi, mck_stream stream)
{
    return forward_common(x, batch, d, E, seed, sigma, calib, phi, true, stream);
}

mck_status mck_fastfood_forward_t(const void* x, mck_dtype x_type, int64_t batch, int64_t d, int64_t E,
                                  uint32_t seed, double sigma, mck_calibration calib, void* phi, mck_dtype phi_type,
                                  mck_stream stream)
{
    const int xt = (int)x_type, yt = (int)phi_type;
    if (xt < 0 || xt > 2 || yt < 0 || yt > 2)
        return fail(MCK_ERR_INVALID_ARG, "unknown storage type");
    if (xt == 0 && yt == 0)
        return forward_common(static_cast<const float*>(x), batch, d, E, seed, sigma, calib,
                              static_cast<float*>(phi), true, stream);
    const bool supported = (xt == 0 && (yt == 1 || yt == 2)) || (xt == yt);
    if (!supported)
        return fail(MCK_ERR_UNSUPPORTED, "storage pair not supported (use F32 x, or the same 16-bit type)");
    int64_t n = 0;
    mck_status st = check_common(batch, d, E, &n);
    if (st != MCK_OK)
        return st;
    st = check_sigma(sigma);
    if (st != MCK_OK)
        return st;
    {
        int mt = 0;
        st = check_calib((int)calib, n, &mt);
        if (st != MCK_OK)
            return st;
    }
    if (batch > 0 && (x == nullptr || phi == nullptr))
        return fail(MCK_ERR_INVALID_ARG, "x or phi is NULL");
    if (batch == 0)
        return MCK_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    PlanHold p;
    st = p.acquire(seed, n, E, sigma, calib, s);
    if (st != MCK_OK)
        return st;
    if (n > MCK_MAX_N)
        return forward_long(p.get(), x, xt, batch, d, n, E, phi, yt, s, feature_scale(n, E));
    // vector path: 4 elements per access, so 4-element alignment of both arrays
    const uintptr_t xa = 4u * (xt == 0 ? 4u : 2u), ya = 4u * (yt == 0 ? 4u : 2u);
    const bool vec = (reinterpret_cast<uintptr_t>(x) % xa == 0) && (reinterpret_cast<uintptr_t>(phi) % ya == 0) &&
                     d % 4 == 0 && n >= 4;
    const FwdTune t = current_tuning(log2i(n));
    const FwdArrays a = fwd_arrays(p.get(), t.P);
    const hipError_t err = mck::launch_forward_t(log2i(n), t.P, t.waves, vec, xt, yt, x, batch, (int)d, E, p->B,
                                                 a.goff, a.Gs, p->Sh, feature_scale(n, E), phi, s);
    return err == hipSuccess ? MCK_OK : hip_fail(err, "forward launch");
}

namespace {

// One instance of a batched call, validated, with its pinned plan.
struct MapRef {
    const mck_instance* q;
    int64_t n;
    const Plan* p;
};

void batched_unpin(const std::vector<MapRef>& maps)
{
    std::lock_guard<std::mutex> lock(g_mutex);
    for (const MapRef& m : maps)
        g_plans.unpin(const_cast<Plan*>(m.p));
}

// Validates every instance and pins the plans of the non-empty ones; on
// failure nothing stays pinned.
mck_status batched_setup(const mck_instance* inst, int64_t count, hipStream_t s, std::vector<MapRef>* maps)
{
    if (count < 0 || (count > 0 && inst == nullptr))
        return fail(MCK_ERR_INVALID_ARG, "count must be >= 0 and inst non-NULL");
    // validate everything before enqueueing anything
    std::vector<int64_t> ns((size_t)count);
    for (int64_t i = 0; i < count; ++i) {
        const mck_instance& q = inst[i];
        mck_status st = check_common(q.batch, q.d, q.E, &ns[i]);
        if (st == MCK_OK)
            st = check_sigma(q.sigma);
        if (st == MCK_OK) {
            int mt = 0;
            st = check_calib((int)q.calib, ns[i], &mt);
        }
        if (st == MCK_OK && q.batch > 0 && (q.x == nullptr || q.phi == nullptr))
            st = fail(MCK_ERR_INVALID_ARG, "x or phi is NULL");
        if (st != MCK_OK) {
            g_last_error = "instance " + std::to_string(i) + ": " + g_last_error;
            return st;
        }
    }
    maps->clear();
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    const hipError_t cerr = hipStreamIsCapturing(s, &cap);
    if (cerr != hipSuccess)
        return hip_fail(cerr, "hipStreamIsCapturing");
    mck_status st = MCK_OK;
    for (int64_t i = 0; i < count && st == MCK_OK; ++i) {
        if (inst[i].batch == 0)
            continue;
        Plan* p = nullptr;
        st = get_plan(inst[i].seed, ns[i], inst[i].E, inst[i].sigma, inst[i].calib, s, &p, true);
        if (st == MCK_OK) {
            maps->push_back(MapRef{&inst[i], ns[i], p});
            if (cap != hipStreamCaptureStatusNone) {  // a caller's graph replays these launches
                std::lock_guard<std::mutex> lock(g_mutex);
                p->captured = true;
            }
        }
    }
    if (st != MCK_OK)
        batched_unpin(*maps);
    return st;
}

// Launches the single-pass maps of one n with launch choice t: grouped by
// vector path into k_forward_group grids, a map whose x or phi exceeds one
// launch's 2^31-byte ranges alone.
hipError_t launch_maps(int M, const FwdTune& t, const std::vector<MapRef>& maps, hipStream_t s)
{
    const int64_t lim = (int64_t(1) << 31) - 4096;
    std::vector<mck::GroupInst> grp[2];
    hipError_t err = hipSuccess;
    for (const MapRef& m : maps) {
        const mck_instance& q = *m.q;
        const int64_t n = m.n;
        const FwdArrays a = fwd_arrays(m.p, t.P);
        const bool vec = vec_ok(q.x, q.phi, q.d, n);
        if (4 * q.batch * q.d <= lim && 4 * q.batch * 2 * n * q.E <= lim) {
            grp[vec ? 1 : 0].push_back(
                {q.x, q.batch, (int)q.d, q.E, m.p->B, a.goff, a.Gs, m.p->Sh, feature_scale(n, q.E), q.phi});
        } else if (err == hipSuccess) {
            err = mck::launch_forward(M, t.P, t.waves, true, vec, true, q.x, q.batch, (int)q.d, q.E, m.p->B, a.goff,
                                      a.Gs, m.p->Sh, feature_scale(n, q.E), q.phi, s);
        }
    }
    for (int v = 0; v < 2 && err == hipSuccess; ++v)
        if (!grp[v].empty())
            err = mck::launch_forward_group(M, t.P, t.waves, v == 1, grp[v].data(), (int)grp[v].size(), s);
    return err;
}

// The single-pass maps by log2 n; long maps (n > MCK_MAX_N) are launched
// here, each on the multi-pass path.
mck_status split_maps(const std::vector<MapRef>& maps, hipStream_t s, bool run_long,
                      std::map<int, std::vector<MapRef>>* by_m)
{
    for (const MapRef& m : maps) {
        if (m.n <= MCK_MAX_N) {
            (*by_m)[log2i(m.n)].push_back(m);
        } else if (run_long) {
            const mck_status st = forward_long(m.p, m.q->x, 0, m.q->batch, m.q->d, m.n, m.q->E, m.q->phi, 0, s,
                                               feature_scale(m.n, m.q->E));
            if (st != MCK_OK)
                return st;
        }
    }
    return MCK_OK;
}

}  // namespace

mck_status mck_fastfood_forward_scaled(const void* x, mck_dtype x_type, const int8_t* x_exp, int64_t batch, int64_t d,
                                       int64_t E, uint32_t seed, double sigma, mck_calibration calib, void* phi,
                                       mck_dtype phi_type, int8_t* phi_exp, mck_stream stream)
{
    const int xt = (int)x_type, yt = (int)phi_type;
    if (xt < 0 || xt > 2 || yt < 0 || yt > 2)
        return fail(MCK_ERR_INVALID_ARG, "unknown storage type");
    const bool supported = (xt == 0) || (xt == yt);
    if (!supported)
        return fail(MCK_ERR_UNSUPPORTED, "storage pair not supported (use F32 x, or the same 16-bit type)");
    int64_t n = 0;
    mck_status st = check_common(batch, d, E, &n);
    if (st != MCK_OK)
        return st;
    st = check_sigma(sigma);
    if (st != MCK_OK)
        return st;
    {
        int mt = 0;
        st = check_calib((int)calib, n, &mt);
        if (st != MCK_OK)
            return st;
    }
    if (batch > 0 && (x == nullptr || phi == nullptr))
        return fail(MCK_ERR_INVALID_ARG, "x or phi is NULL");
    if (batch == 0)
        return MCK_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    PlanHold p;
    st = p.acquire(seed, n, E, sigma, calib, s);
    if (st != MCK_OK)
        return st;
    // |phi| <= c = 1/sqrt(nE): scale by 2^j, the largest power of two with
    // c 2^j <= 1 (4^j <= nE), folded exactly into the feature scale
    int j = 0;
    while ((int64_t(1) << (2 * (j + 1))) <= n * E)
        ++j;
    const float cs = std::ldexp(feature_scale(n, E), j);
    if (n > MCK_MAX_N) {
        st = forward_long(p.get(), x, xt, batch, d, n, E, phi, yt, s, cs, x_exp);
        if (st == MCK_OK && phi_exp != nullptr) {
            const hipError_t ferr = mck::launch_fill_i8(phi_exp, batch, (int8_t)j, s);
            if (ferr != hipSuccess)
                return hip_fail(ferr, "exponent fill");
        }
        return st;
    }
    const FwdTune t = current_tuning(log2i(n));
    const FwdArrays a = fwd_arrays(p.get(), t.P);
    const uintptr_t xa = 4u * (xt == 0 ? 4u : 2u), ya = 4u * (yt == 0 ? 4u : 2u);
    const bool vec = (reinterpret_cast<uintptr_t>(x) % xa == 0) && (reinterpret_cast<uintptr_t>(phi) % ya == 0) &&
                     d % 4 == 0 && n >= 4;
    hipError_t err;
    if (xt == 0 && yt == 0)
        err = mck::launch_forward(log2i(n), t.P, t.waves, true, vec, true, static_cast<const float*>(x), batch,
                                  (int)d, E, p->B, a.goff, a.Gs, p->Sh, cs, static_cast<float*>(phi), s, x_exp);
    else
        err = mck::launch_forward_t(log2i(n), t.P, t.waves, vec, xt, yt, x, batch, (int)d, E, p->B, a.goff, a.Gs,
                                    p->Sh, cs, phi, s, x_exp);
    if (err == hipSuccess && phi_exp != nullptr)
        err = mck::launch_fill_i8(phi_exp, batch, (int8_t)j, s);
    return err == hipSuccess ? MCK_OK : hip_fail(err, "scaled forward launch");
}

mck_status mck_fastfood_forward_batched(const mck_instance* inst, int64_t count, mck_stream stream)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<MapRef> maps;
    mck_status st = batched_setup(inst, count, s, &maps);
    if (st != MCK_OK)
        return st;
    std::map<int, std::vector<MapRef>> by_m;
    st = split_maps(maps, s, true, &by_m);
    for (const auto& kv : by_m) {
        if (st != MCK_OK)
            break;
        const hipError_t err = launch_maps(kv.first, current_tuning(kv.first), kv.second, s);
        if (err != hipSuccess)
            st = hip_fail(err, "batched forward launch");
    }
    batched_unpin(maps);
    return st;
}

namespace {

// Grid targets the tuner tries, in waves.
constexpr int kTuneWaves[] = {2048, 4096, 8192, 16384, 32768, 65536};

// Average time of `reps` launches of the maps of one n under choice t (one
// untimed launch first).
mck_status time_maps(int M, const FwdTune& t, const std::vector<MapRef>& maps, int reps, hipEvent_t e0,
                     hipEvent_t e1, hipStream_t s, float* ms)
{
    hipError_t err = launch_maps(M, t, maps, s);
    if (err == hipSuccess)
        err = hipEventRecord(e0, s);
    for (int r = 0; r < reps && err == hipSuccess; ++r)
        err = launch_maps(M, t, maps, s);
    if (err == hipSuccess)
        err = hipEventRecord(e1, s);
    if (err == hipSuccess)
        err = hipEventSynchronize(e1);
    float t_ms = 0.f;
    if (err == hipSuccess)
        err = hipEventElapsedTime(&t_ms, e0, e1);
    if (err != hipSuccess)
        return hip_fail(err, "autotune timing");
    *ms = t_ms / (float)reps;
    return MCK_OK;
}

}  // namespace

mck_status mck_autotune_forward_batched(const mck_instance* inst, int64_t count, int32_t reps, mck_stream stream)
{
    if (reps < 1 || reps > 1000)
        return fail(MCK_ERR_INVALID_ARG, "reps must be in [1, 1000]");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    hipError_t err = hipStreamIsCapturing(s, &cap);
    if (err != hipSuccess)
        return hip_fail(err, "hipStreamIsCapturing");
    if (cap != hipStreamCaptureStatusNone)
        return fail(MCK_ERR_INVALID_ARG, "the tuner times launches and cannot run under graph capture");
    std::vector<MapRef> maps;
    mck_status st = batched_setup(inst, count, s, &maps);
    if (st != MCK_OK)
        return st;
    std::map<int, std::vector<MapRef>> by_m;
    st = split_maps(maps, s, false, &by_m);
    int dev = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (st == MCK_OK) {
        err = hipGetDevice(&dev);
        if (err == hipSuccess)
            err = hipEventCreate(&e0);
        if (err == hipSuccess)
            err = hipEventCreate(&e1);
        if (err != hipSuccess)
            st = hip_fail(err, "autotune events");
    }
    for (const auto& kv : by_m) {
        if (st != MCK_OK)
            break;
        const int M = kv.first;
        const FwdTune def = default_tuning(M);
        FwdTune best = def;
        float best_ms = 0.f;
        st = time_maps(M, def, kv.second, reps, e0, e1, s, &best_ms);
        const int splits[2] = {def.P, alt_split(M)};
        for (int k = 0; k < 2 && st == MCK_OK; ++k) {
            if (k == 1 && !mck::fwd_split_ok(M, splits[1]))
                break;
            for (int w : kTuneWaves) {
                const FwdTune c{splits[k], w};
                if (c.P == def.P && c.waves == def.waves)
                    continue;
                float ms = 0.f;
                st = time_maps(M, c, kv.second, reps, e0, e1, s, &ms);
                if (st != MCK_OK)
                    break;
                // move away from the current best only for a clear gain
                if (ms < 0.98f * best_ms) {
                    best = c;
                    best_ms = ms;
                }
            }
        }
        if (st == MCK_OK) {
            std::lock_guard<std::mutex> lock(g_tune_mutex);
            g_tune[{dev, M}] = best;
        }
    }
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    batched_unpin(maps);
    return st;
}

mck_status mck_forward_tuning_get(int64_t n, mck_forward_tuning* out)
{
    if (out == nullptr)
        return fail(MCK_ERR_INVALID_ARG, "out is NULL");
    if (!is_pow2(n) || n < 2 || n > MCK_MAX_N)
        return fail(MCK_ERR_INVALID_ARG, "n must be a power of two in [2, MCK_MAX_N]");
    const FwdTune t = current_tuning(log2i(n));
    out->split = t.P;
    out->waves = t.waves;
    return MCK_OK;
}

mck_status mck_forward_tuning_set(int64_t n, const mck_forward_tuning* t)
{
    if (!is_pow2(n) || n < 2 || n > MCK_MAX_N)
        return fail(MCK_ERR_INVALID_ARG, "n must be a power of two in [2, MCK_MAX_N]");
    const int M = log2i(n);
    if (t != nullptr) {
        if (!mck::fwd_split_ok(M, t->split))
            return fail(MCK_ERR_UNSUPPORTED, "register split not compiled for this n");
        if (t->waves < 64 || t->waves > (1 << 20))
            return fail(MCK_ERR_INVALID_ARG, "waves must be in [64, 2^20]");
    }
    int dev = 0;
    const hipError_t err = hipGetDevice(&dev);
    if (err != hipSuccess)
        return hip_fail(err, "hipGetDevice");
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    if (t == nullptr)
        g_tune.erase({dev, M});
    else
        g_tune[{dev, M}] = FwdTune{t->split, t->waves};
    return MCK_OK;
}

}  // extern "C"

// A recorded batched call: the maps' plans stay pinned, and the long maps'
// scratch rows are owned here, so that replays allocate nothing.
struct mck_batched_graph {
    int device = 0;
    std::vector<mck_instance> inst;
    std::vector<MapRef> maps;
    void* scratch = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

void graph_release(mck_batched_graph* g)
{
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(g->device);
    (void)hipDeviceSynchronize();  // no replay may still use the scratch or the plans
    if (g->exec)
        (void)hipGraphExecDestroy(g->exec);
    if (g->graph)
        (void)hipGraphDestroy(g->graph);
    if (g->scratch)
        (void)hipFree(g->scratch);
    batched_unpin(g->maps);
    (void)hipSetDevice(cur);
    delete g;
}

// Records every launch of the batched call into the stream being captured.
mck_status record_maps(mck_batched_graph* g, hipStream_t cs)
{
    std::map<int, std::vector<MapRef>> by_m;
    for (const MapRef& m : g->maps) {
        if (m.n <= MCK_MAX_N) {
            by_m[log2i(m.n)].push_back(m);
        } else {
            const mck_status st = forward_long_launch(m.p, m.q->x, 0, m.q->batch, m.q->d, m.n, m.q->E, m.q->phi, 0,
                                                      static_cast<float*>(g->scratch), cs, feature_scale(m.n, m.q->E));
            if (st != MCK_OK)
                return st;
        }
    }
    for (const auto& kv : by_m) {
        const hipError_t err = launch_maps(kv.first, current_tuning(kv.first), kv.second, cs);
        if (err != hipSuccess)
            return hip_fail(err, "batched forward launch");
    }
    return MCK_OK;
}

}  // namespace

extern "C" {

mck_status mck_batched_graph_create(const mck_instance* inst, int64_t count, mck_stream stream,
                                    mck_batched_graph** out)
{
    if (out == nullptr)
        return fail(MCK_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    hipError_t err = hipStreamIsCapturing(s, &cap);
    if (err != hipSuccess)
        return hip_fail(err, "hipStreamIsCapturing");
    if (cap != hipStreamCaptureStatusNone)
        return fail(MCK_ERR_INVALID_ARG, "cannot record a batched graph while the stream is being captured");
    mck_batched_graph* g = new (std::nothrow) mck_batched_graph();
    if (g == nullptr)
        return fail(MCK_ERR_NO_MEMORY, "batched graph object");
    err = hipGetDevice(&g->device);
    if (err != hipSuccess) {
        delete g;
        return hip_fail(err, "hipGetDevice");
    }
    // the instances are copied: the recorded launches keep their pointers
    // and sizes, the caller's array may go away
    if (count > 0 && inst != nullptr)
        g->inst.assign(inst, inst + count);
    mck_status st = batched_setup(count > 0 ? g->inst.data() : inst, count, s, &g->maps);
    if (st != MCK_OK) {
        delete g;
        return st;
    }
    // one scratch for the long maps: their launches are serialized in the graph
    size_t long_bytes = 0;
    for (const MapRef& m : g->maps) {
        if (m.n <= MCK_MAX_N)
            continue;
        if (2 * m.n * m.q->E * 4 > (int64_t(1) << 31) - 4096) {
            graph_release(g);
            return fail(MCK_ERR_UNSUPPORTED, "one row of phi exceeds 2^31 bytes");
        }
        const size_t need = (size_t)long_scratch_floats(m.q->batch, m.n, m.q->E) * sizeof(float);
        long_bytes = need > long_bytes ? need : long_bytes;
    }
    if (long_bytes > 0) {
        err = hipMalloc(&g->scratch, long_bytes);
        if (err != hipSuccess) {
            g->scratch = nullptr;
            graph_release(g);
            return fail(MCK_ERR_NO_MEMORY, std::string("long-vector scratch: ") + hipGetErrorString(err));
        }
    }
    if (g->maps.empty()) {  // nothing to record: launches do nothing
        *out = g;
        return MCK_OK;
    }
    // record on a private stream (default priority), then instantiate
    hipStream_t cs = nullptr;
    err = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (err != hipSuccess) {
        graph_release(g);
        return hip_fail(err, "capture stream");
    }
    err = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (err == hipSuccess) {
        st = record_maps(g, cs);
        const hipError_t end = hipStreamEndCapture(cs, &g->graph);
        if (st == MCK_OK && end != hipSuccess)
            st = hip_fail(end, "hipStreamEndCapture");
    } else {
        st = hip_fail(err, "hipStreamBeginCapture");
    }
    (void)hipStreamDestroy(cs);
    if (st == MCK_OK) {
        err = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
        if (err != hipSuccess) {
            g->exec = nullptr;
            st = hip_fail(err, "hipGraphInstantiate");
        }
    }
    if (st != MCK_OK) {
        graph_release(g);
        return st;
    }
    *out = g;
    return MCK_OK;
}

mck_status mck_batched_graph_launch(mck_batched_graph* g, mck_stream stream)
{
    if (g == nullptr)
        return fail(MCK_ERR_INVALID_ARG, "graph is NULL");
    int dev = 0;
    hipError_t err = hipGetDevice(&dev);
    if (err != hipSuccess)
        return hip_fail(err, "hipGetDevice");
    if (dev != g->device)
        return fail(MCK_ERR_INVALID_ARG, "the graph was recorded on another device");
    if (g->exec == nullptr)
        return MCK_OK;
    err = hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream));
    return err == hipSuccess ? MCK_OK : hip_fail(err, "hipGraphLaunch");
}

void mck_batched_graph_destroy(mck_batched_graph* g)
{
    if (g != nullptr)
        graph_release(g);
}

mck_status mck_fastfood_project(const float* x, int64_t batch, int64_t d, int64_t E, uint32_t seed, double sigma,
                                mck_calibration calib, float* z, mck_stream stream)
{
    return forward_common(x, batch, d, E, seed, sigma, calib, z, false, stream);
}

mck_status mck_fastfood_backward(const float* x, const float* dphi, int64_t batch, int64_t d, int64_t E,
                                 uint32_t seed, double sigma, mck_calibration calib, float* dx, float* dB, float* dG,
                                 float* dS, mck_stream stream)
{
    int64_t n = 0;
    mck_status st = check_common(batch, d, E, &n);
    if (st != MCK_OK)
        return st;
    st = check_single_pass(n);
    if (st != MCK_OK)
        return st;
    st = check_sigma(sigma);
    if (st != MCK_OK)
        return st;
    {
        int mt = 0;
        st = check_calib((int)calib, n, &mt);
        if (st != MCK_OK)
            return st;
    }
    if (batch > 0 && (x == nullptr || dphi == nullptr))
        return fail(MCK_ERR_INVALID_ARG, "x or dphi is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!dx && !dB && !dG && !dS)
        return MCK_OK;
    PlanHold p;
    if (batch == 0) {
        if (!dB && !dG && !dS)
            return MCK_OK;
        // the sums over an empty batch are zero
        hipError_t err = hipSuccess;
        for (float* o : {dB, dG, dS})
            if (o && err == hipSuccess)
                err = mck::launch_sum_groups(nullptr, 0, n * E, o, s);  // a fill kernel: zeros
        return err == hipSuccess ? MCK_OK : hip_fail(err, "zero gradients");
    }
    st = p.acquire(seed, n, E, sigma, calib, s);
    if (st != MCK_OK)
        return st;
    return run_backward(x, dphi, batch, d, n, E, p->B, p->goffB, p->GkB, p->S32, p->Sh, dx, dB, dG, dS, s);
}

mck_status mck_backward_launch_shape(int64_t batch, int64_t d, int64_t E, mck_backward_shape* out)
{
    if (out == nullptr)
        return fail(MCK_ERR_INVALID_ARG, "out is NULL");
    int64_t n = 0;
    mck_status st = check_common(batch, d, E, &n);
    if (st != MCK_OK)
        return st;
    st = check_single_pass(n);
    if (st != MCK_OK)
        return st;
    const int64_t rows = backward_rows_per_launch(d, n, E);
    const mck::BwdGeometry geo = mck::backward_geometry(log2i(n), batch < rows ? batch : rows, (int)d, E);
    out->rows_per_pass = geo.rows_per_pass;
    out->passes = geo.passes;
    out->esplit = geo.esplit;
    out->reserved = 0;
    out->rowblocks = geo.rowblocks;
    return MCK_OK;
}

static mck_status check_explicit(int64_t batch, int64_t d, int64_t n, int64_t E, const float* B,
                                 const int32_t* perm, const float* G, const float* S)
{
    int64_t nn = 0;
    mck_status st = check_common(batch, d, E, &nn);
    if (st != MCK_OK)
        return st;
    if (n != nn)
        return fail(MCK_ERR_INVALID_ARG, "n must equal mck_padded_dim(d)");
    st = check_single_pass(n);
    if (st != MCK_OK)
        return st;
    if (!B || !perm || !G || !S)
        return fail(MCK_ERR_INVALID_ARG, "B, perm, G and S must be non-NULL");
    return MCK_OK;
}

mck_status mck_fastfood_forward_p(const float* x, int64_t batch, int64_t d, int64_t n, int64_t E, const float* B,
                                  const int32_t* perm, const float* G, const float* S, float* phi, mck_stream stream)
{
    mck_status st = check_explicit(batch, d, n, E, B, perm, G, S);
    if (st != MCK_OK)
        return st;
    if (batch > 0 && (x == nullptr || phi == nullptr))
        return fail(MCK_ERR_INVALID_ARG, "x or phi is NULL");
    if (batch == 0)
        return MCK_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    TempPlan tp;
    st = make_temp_plan(n, E, perm, G, S, s, &tp);
    if (st != MCK_OK)
        return st;
    hipError_t err = mck::launch_forward(log2i(n), tp.PF, current_tuning(log2i(n)).waves, false, vec_ok(x, phi, d, n),
                                         true, x, batch, (int)d, E, B, tp.goffF, tp.GsF, tp.Sh, feature_scale(n, E),
                                         phi, s);
    temp_free(tp.block, s);
    return err == hipSuccess ? MCK_OK : hip_fail(err, "forward launch");
}

mck_status mck_fastfood_backward_p(const float* x, const float* dphi, int64_t batch, int64_t d, int64_t n, int64_t E,
                                   const float* B, const int32_t* perm, const float* G, const float* S, float* dx,
                                   float* dB, float* dG, float* dS, mck_stream stream)
{
    mck_status st = check_explicit(batch, d, n, E, B, perm, G, S);
    if (st != MCK_OK)
        return st;
    if (batch > 0 && (x == nullptr || dphi == nullptr))
        return fail(MCK_ERR_INVALID_ARG, "x or dphi is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!dx && !dB && !dG && !dS)
        return MCK_OK;
    if (batch == 0) {
        hipError_t err = hipSuccess;
        for (float* o : {dB, dG, dS})
            if (o && err == hipSuccess)
                err = mck::launch_sum_groups(nullptr, 0, n * E, o, s);  // a fill kernel: zeros
        return err == hipSuccess ? MCK_OK : hip_fail(err, "zero gradients");
    }
    // one allocation: the parameter copies, then the adjoint's temporaries
    const int PF = current_tuning(log2i(n)).P;
    const size_t zt = align_up(temp_plan_sizes(n, E, PF).bytes());
    const BwdScratch bs = backward_scratch(batch, d, n, E, dx != nullptr, dB || dG || dS);
    void* block = nullptr;
    hipError_t err = temp_alloc(&block, zt + bs.bytes(), s);
    if (err != hipSuccess)
        return fail(MCK_ERR_NO_MEMORY, std::string("backward temporaries: ") + hipGetErrorString(err));
    TempPlan tp;
    st = make_temp_plan(n, E, perm, G, S, s, &tp, PF, static_cast<char*>(block));
    if (st == MCK_OK)
        st = run_backward(x, dphi, batch, d, n, E, B, tp.goffB, tp.GkB, S, tp.Sh, dx, dB, dG, dS, s,
                          static_cast<char*>(block) + zt);
    temp_free(block, s);
    return st;
}

mck_status mck_fastfood_backward_p_noalloc(const float* x, const float* dphi, int64_t batch, int64_t d, int64_t n,
                                           int64_t E, const float* B, const int32_t* perm, const float* G,
                                           const float* S, float* dx, float* dB, float* dG, float* dS,
                                           mck_stream stream)
{
    mck_status st = check_explicit(batch, d, n, E, B, perm, G, S);
    if (st != MCK_OK)
        return st;
    if (batch > 0 && (x == nullptr || dphi == nullptr))
        return fail(MCK_ERR_INVALID_ARG, "x or dphi is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!dx && !dB && !dG && !dS)
        return MCK_OK;
    if (batch == 0) {
        hipError_t err = hipSuccess;
        for (float* o : {dB, dG, dS})
            if (o && err == hipSuccess)
                err = mck::launch_sum_groups(nullptr, 0, n * E, o, s);  // a fill kernel: zeros
        return err == hipSuccess ? MCK_OK : hip_fail(err, "zero gradients");
    }
    // scratch layout: the backward's parameter copies (gather offsets, G in
    // the gather layout, S in revolutions), then the adjoint's temporaries
    int64_t gf = 0, gb = 0;
    mck::plan_elems(log2i(n), &gf, &gb);
    const size_t a = align_up((size_t)(n * E) * 4), ab = align_up((size_t)gb * E * 4);
    const BwdScratch bs = backward_scratch(batch, d, n, E, dx != nullptr, dB || dG || dS);
    const size_t need = ab + 2 * a + bs.bytes();
    if (need > (size_t)MCK_NOALLOC_SCRATCH_BYTES)
        return fail(MCK_ERR_UNSUPPORTED, "temporaries of " + std::to_string(need) +
                                             " bytes exceed the static scratch of " +
                                             std::to_string((size_t)MCK_NOALLOC_SCRATCH_BYTES) + " bytes");
    char* base = nullptr;
    st = scratch_on_current_device(&base);
    if (st != MCK_OK)
        return st;
    uint32_t* goffB = reinterpret_cast<uint32_t*>(base);
    float* GkB = reinterpret_cast<float*>(base + ab);
    float* Sh = reinterpret_cast<float*>(base + ab + a);
    hipError_t err = mck::launch_derive_bwd(log2i(n), E, perm, G, S, goffB, GkB, Sh, s);
    if (err != hipSuccess)
        return hip_fail(err, "derive kernel");
    return run_backward(x, dphi, batch, d, n, E, B, goffB, GkB, S, Sh, dx, dB, dG, dS, s, base + ab + 2 * a);
}

static mck_status check_head(int64_t batch, int64_t F, int64_t C);

namespace {

// The training step with the head fused into the feature-map kernels: phi
// never goes to HBM.  Forward + logits (k_forward_logits), softmax
// cross-entropy, phi recomputed for dW and dphi (k_head_bwd_fused), the
// adjoint, the SGD update.  Arguments checked by the caller.
mck_status train_step_fused(const float* x, const int32_t* labels, int64_t batch, int64_t d, int64_t n, int64_t E,
                            int64_t C, float* W, float* b, float* B, const int32_t* perm, float* G, float* S,
                            float lr, float* loss, float* logits, float* dW, float* db, float* dB, float* dG,
                            float* dS, float* dx, hipStream_t s)
{
    const int64_t F = 2 * n * E;
    const int64_t esplit = mck::fused_logits_esplit(batch, E);
    int64_t ranges = 0, rpr = 0;
    mck::fused_bwd_geometry(batch, E, &ranges, &rpr);
    // scratch: dphi, logits (when the caller passes none), dlogits, row
    // losses, the logits' and dW's partials
    const int64_t lpart = esplit * batch * C, wpart = ranges > 1 ? ranges * C * F : 0;
    constexpr int kPF = 4;  // register split of the fused kernels
    const BwdScratch bs = backward_scratch(batch, d, n, E, dx != nullptr, true);
    const size_t zf = align_up((size_t)(batch * F) * 4), zl = align_up((size_t)(batch * C) * 4),
                 zr = align_up((size_t)batch * 4), zp = align_up((size_t)(lpart > wpart ? lpart : wpart) * 4),
                 zt = align_up(temp_plan_sizes(n, E, kPF).bytes());
    // one allocation for every temporary of the step (each stream-ordered
    // free costs the host tens of microseconds while the GPU is busy)
    void* block = nullptr;
    hipError_t err = temp_alloc(&block, zf + 2 * zl + zr + zp + zt + bs.bytes(), s);
    if (err != hipSuccess)
        return fail(MCK_ERR_NO_MEMORY, std::string("training step scratch: ") + hipGetErrorString(err));
    char* base = static_cast<char*>(block);
    float* dphi = reinterpret_cast<float*>(base);
    float* lg = logits ? logits : reinterpret_cast<float*>(base + zf);
    float* dl = reinterpret_cast<float*>(base + zf + zl);
    float* row_loss = reinterpret_cast<float*>(base + zf + 2 * zl);
    float* part = reinterpret_cast<float*>(base + zf + 2 * zl + zr);
    char* tmem = base + zf + 2 * zl + zr + zp;
    char* bws = tmem + zt;
    TempPlan tp;
    mck_status st = make_temp_plan(n, E, perm, G, S, s, &tp, kPF, tmem);
    if (st != MCK_OK) {
        temp_free(block, s);
        return st;
    }
    const bool vec = aligned16(x) && d % 4 == 0;
    const float cs = feature_scale(n, E);
    // the SGD step rides in the last pass over each gradient: b in the head
    // tail (or one update launch), W in the sum of its partials, B, G, S in
    // the adjoint's partial sums; every reader of a parameter runs before
    const float alpha = -lr;
    const bool tail = batch <= mck::kHeadTailRows;
    err = mck::launch_forward_logits(vec, x, batch, (int)d, E, B, tp.goffF, tp.GsF, tp.Sh, cs, W, (int)C, esplit,
                                     part, s);
    if (err == hipSuccess && tail) {
        err = mck::launch_head_tail(part, b, esplit, batch, (int)C, labels, lg, dl, loss, db, alpha, s);
    } else if (err == hipSuccess) {
        err = mck::launch_logits_finish(part, b, esplit, batch, (int)C, lg, s);
        if (err == hipSuccess)
            err = mck::launch_softmax_xent(lg, labels, batch, (int)C, row_loss, dl, loss, db, s);
    }
    if (err == hipSuccess)
        err = mck::launch_head_bwd_fused(vec, x, batch, (int)d, E, B, tp.goffF, tp.GsF, tp.Sh, cs, dl, W, (int)C,
                                         ranges, rpr, dphi, ranges > 1 ? part : dW, s);
    // dW from its row-range partials (and the W update) in the launch of the
    // adjoint's sums: nothing after the head backward reads W
    const mck::GroupSum wsum{part, ranges, C * F, dW, lr != 0.f ? W : nullptr, alpha};
    if (err == hipSuccess) {
        st = run_backward(x, dphi, batch, d, n, E, B, tp.goffB, tp.GkB, S, tp.Sh, dx, dB, dG, dS, s, bws,
                          lr != 0.f ? B : nullptr, lr != 0.f ? G : nullptr, lr != 0.f ? S : nullptr, alpha,
                          ranges > 1 ? &wsum : nullptr);
        if (st != MCK_OK) {
            temp_free(block, s);
            return st;
        }
    }
    if (err == hipSuccess && lr != 0.f) {
        // what the passes above did not update
        float* ys[2];
        const float* xs[2];
        int64_t cnt[2];
        int k = 0;
        if (ranges <= 1) {
            ys[k] = W, xs[k] = dW, cnt[k++] = C * F;
        }
        if (!tail) {
            ys[k] = b, xs[k] = db, cnt[k++] = C;
        }
        if (k > 0)
            err = mck::launch_axpy_multi(ys, xs, cnt, k, alpha, s);
    }
    temp_free(block, s);
    return err == hipSuccess ? MCK_OK : hip_fail(err, "training step launch");
}

}  // namespace

mck_status mck_fastfood_train_step(const float* x, const int32_t* labels, int64_t batch, int64_t d, int64_t n,
                                   int64_t E, int64_t C, float* W, float* b, float* B, const int32_t* perm, float* G,
                                   float* S, float lr, float* loss, float* logits, float* dW, float* db, float* dB,
                                   float* dG, float* dS, float* dx, mck_stream stream)
{
    mck_status st = check_explicit(batch, d, n, E, B, perm, G, S);
    if (st != MCK_OK)
        return st;
    if (batch < 1)
        return fail(MCK_ERR_INVALID_ARG, "batch must be >= 1 (the loss is a mean over rows)");
    const int64_t F = 2 * n * E;
    st = check_head(batch, F, C);
    if (st != MCK_OK)
        return st;
    if (!x || !labels || !W || !b || !loss || !dW || !db || !dB || !dG || !dS)
        return fail(MCK_ERR_INVALID_ARG, "x, labels, W, b, loss or a parameter gradient is NULL");
    if (!aligned16(W) || !aligned16(dW))
        return fail(MCK_ERR_INVALID_ARG, "W and dW must be 16-byte aligned");
    if (!std::isfinite(lr))
        return fail(MCK_ERR_INVALID_ARG, "lr must be finite");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (mck::fused_head_ok(n, C))
        return train_step_fused(x, labels, batch, d, n, E, C, W, b, B, perm, G, S, lr, loss, logits, dW, db, dB, dG,
                                dS, dx, s);
    // scratch: phi, dphi, logits (when the caller passes none), dlogits, row
    // losses, head partials
    int64_t slabs = 0, groups = 0, rpg = 0;
    mck::head_bwd_geometry(batch, F, true, &slabs, &groups, &rpg);
    const int64_t lpart = mck::head_logit_slabs(F) * batch * C;
    const int64_t hpart = groups > 1 ? groups * C * F : 0;
    const int PF = current_tuning(log2i(n)).P;
    const BwdScratch bs = backward_scratch(batch, d, n, E, dx != nullptr, true);
    const size_t zf = align_up((size_t)(batch * F) * 4), zl = align_up((size_t)(batch * C) * 4),
                 zr = align_up((size_t)batch * 4), zp = align_up((size_t)(lpart > hpart ? lpart : hpart) * 4),
                 zt = align_up(temp_plan_sizes(n, E, PF).bytes());
    // one allocation for every temporary of the step
    void* block = nullptr;
    hipError_t err = temp_alloc(&block, 2 * zf + 2 * zl + zr + zp + zt + bs.bytes(), s);
    if (err != hipSuccess)
        return fail(MCK_ERR_NO_MEMORY, std::string("training step scratch: ") + hipGetErrorString(err));
    char* base = static_cast<char*>(block);
    float* phi = reinterpret_cast<float*>(base);
    float* dphi = reinterpret_cast<float*>(base + zf);
    float* lg = logits ? logits : reinterpret_cast<float*>(base + 2 * zf);
    float* dl = reinterpret_cast<float*>(base + 2 * zf + zl);
    float* row_loss = reinterpret_cast<float*>(base + 2 * zf + 2 * zl);
    float* part = reinterpret_cast<float*>(base + 2 * zf + 2 * zl + zr);
    char* tmem = base + 2 * zf + 2 * zl + zr + zp;
    char* bws = tmem + zt;
    TempPlan tp;
    st = make_temp_plan(n, E, perm, G, S, s, &tp, PF, tmem);
    if (st != MCK_OK) {
        temp_free(block, s);
        return st;
    }
    const int M = log2i(n);
    err = mck::launch_forward(M, tp.PF, current_tuning(M).waves, false, vec_ok(x, phi, d, n), true, x, batch, (int)d,
                              E, B, tp.goffF, tp.GsF, tp.Sh, feature_scale(n, E), phi, s);
    if (err == hipSuccess)
        err = mck::launch_head_logits(phi, W, b, batch, F, (int)C, part, lg, s);
    if (err == hipSuccess)
        err = mck::launch_softmax_xent(lg, labels, batch, (int)C, row_loss, dl, loss, db, s);
    if (err == hipSuccess)
        err = mck::launch_head_bwd(phi, dl, W, batch, F, (int)C, slabs, groups, rpg, dphi, groups > 1 ? part : dW, s);
    if (err == hipSuccess && groups > 1)
        err = mck::launch_sum_groups(part, groups, C * F, dW, s);
    if (err == hipSuccess) {
        st = run_backward(x, dphi, batch, d, n, E, B, tp.goffB, tp.GkB, S, tp.Sh, dx, dB, dG, dS, s, bws);
        if (st != MCK_OK) {
            temp_free(block, s);
            return st;
        }
    }
    if (err == hipSuccess && lr != 0.f) {
        // the SGD update of W, b, B, G, S in one launch
        float* const ys[5] = {W, b, B, G, S};
        const float* const xs[5] = {dW, db, dB, dG, dS};
        const int64_t cnt[5] = {C * F, C, n * E, n * E, n * E};
        err = mck::launch_axpy_multi(ys, xs, cnt, 5, -lr, s);
    }
    temp_free(block, s);
    return err == hipSuccess ? MCK_OK : hip_fail(err, "training step launch");
}

mck_status mck_gen_boxmuller(const uint32_t* a, const uint32_t* b, int64_t count, float* g0, float* g1,
                             mck_stream stream)
{
    if (count < 0)
        return fail(MCK_ERR_INVALID_ARG, "count must be >= 0");
    if (count > 0 && (!a || !b || !g0 || !g1))
        return fail(MCK_ERR_INVALID_ARG, "NULL pointer");
    const hipError_t err = mck::launch_boxmuller(a, b, count, g0, g1, static_cast<hipStream_t>(stream));
    return err == hipSuccess ? MCK_OK : hip_fail(err, "mck_gen_boxmuller");
}

mck_status mck_softmax_xent(const float* logits, const int32_t* labels, int64_t batch, int64_t C, float* loss,
                            float* dlogits, float* db, mck_stream stream)
{
    if (batch < 0)
        return fail(MCK_ERR_INVALID_ARG, "batch must be >= 0");
    if (C < 1 || C > 1024)
        return fail(MCK_ERR_INVALID_ARG, "C must be in [1, 1024]");
    if (batch == 0)
        return MCK_OK;
    if (!logits || !labels || !dlogits)
        return fail(MCK_ERR_INVALID_ARG, "logits, labels or dlogits is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    float* row_loss = nullptr;
    hipError_t err = temp_alloc(reinterpret_cast<void**>(&row_loss), (size_t)batch * sizeof(float), s);
    if (err != hipSuccess)
        return fail(MCK_ERR_NO_MEMORY, std::string("softmax scratch: ") + hipGetErrorString(err));
    err = mck::launch_softmax_xent(logits, labels, batch, (int)C, row_loss, dlogits, loss, db, s);
    temp_free(row_loss, s);
    if (err != hipSuccess)
        return hip_fail(err, "softmax cross-entropy launch");
    return MCK_OK;
}

static mck_status check_head(int64_t batch, int64_t F, int64_t C)
{
    if (batch < 0)
        return fail(MCK_ERR_INVALID_ARG, "batch must be >= 0");
    if (F < 4 || F % 4 != 0)
        return fail(MCK_ERR_INVALID_ARG, "F must be a positive multiple of 4");
    if (C < 1 || C > 16)
        return fail(C < 1 ? MCK_ERR_INVALID_ARG : MCK_ERR_UNSUPPORTED, "C must be in [1, 16]");
    if (C * F > (int64_t(1) << 29) - 1024)
        return fail(MCK_ERR_UNSUPPORTED, "C * F must stay below 2^29 (W within 2 GiB)");
    return MCK_OK;
}

mck_status mck_head_logits(const float* phi, const float* W, const float* b, int64_t batch, int64_t F, int64_t C,
                           float* logits, mck_stream stream)
{
    mck_status st = check_head(batch, F, C);
    if (st != MCK_OK)
        return st;
    if (batch == 0)
        return MCK_OK;
    if (!phi || !W || !logits)
        return fail(MCK_ERR_INVALID_ARG, "phi, W or logits is NULL");
    if (!aligned16(phi) || !aligned16(W))
        return fail(MCK_ERR_INVALID_ARG, "phi and W must be 16-byte aligned");
    hipStream_t s = static_cast<hipStream_t>(stream);
    float* part = nullptr;
    hipError_t err = temp_alloc(reinterpret_cast<void**>(&part),
                                    (size_t)(mck::head_logit_slabs(F) * batch * C) * sizeof(float), s);
    if (err != hipSuccess)
        return fail(MCK_ERR_NO_MEMORY, std::string("head logits partials: ") + hipGetErrorString(err));
    err = mck::launch_head_logits(phi, W, b, batch, F, (int)C, part, logits, s);
    temp_free(part, s);
    return err == hipSuccess ? MCK_OK : hip_fail(err, "head logits launch");
}

mck_status mck_head_backward(const float* phi, const float* dlogits, const float* W, int64_t batch, int64_t F,
                             int64_t C, float* dphi, float* dW, mck_stream stream)
{
    mck_status st = check_head(batch, F, C);
    if (st != MCK_OK)
        return st;
    if (!dphi && !dW)
        return MCK_OK;
    if (batch > 0 && (!dlogits || !W || (dW && !phi)))
        return fail(MCK_ERR_INVALID_ARG, "dlogits, W or phi is NULL");
    if ((dphi && (!aligned16(dphi) || !aligned16(W))) || (dW && (!aligned16(dW) || (batch > 0 && !aligned16(phi)))))
        return fail(MCK_ERR_INVALID_ARG, "phi, W, dphi and dW must be 16-byte aligned");
    hipStream_t s = static_cast<hipStream_t>(stream);
    int64_t slabs = 0, groups = 0, rpg = 0;
    mck::head_bwd_geometry(batch, F, dW != nullptr, &slabs, &groups, &rpg);
    if (dW && groups != 1) {
        // partials per row group, then a fixed-order sum (zeros for an empty batch)
        float* part = nullptr;
        hipError_t err = hipSuccess;
        if (groups > 0) {
            err = temp_alloc(reinterpret_cast<void**>(&part), (size_t)(groups * C * F) * sizeof(float), s);
            if (err != hipSuccess)
                return fail(MCK_ERR_NO_MEMORY, std::string("head partials: ") + hipGetErrorString(err));
        }
        err = mck::launch_head_bwd(phi, dlogits, W, batch, F, (int)C, slabs, groups, rpg, dphi, part, s);
        if (err == hipSuccess)
            err = mck::launch_sum_groups(part, groups, C * F, dW, s);
        if (part)
            temp_free(part, s);
        return err == hipSuccess ? MCK_OK : hip_fail(err, "head backward launch");
    }
    const hipError_t err = mck::launch_head_bwd(phi, dlogits, W, batch, F, (int)C, slabs, groups, rpg, dphi, dW, s);
    return err == hipSuccess ? MCK_OK : hip_fail(err, "head backward launch");
}

mck_status mck_axpy(float* y, const float* x, int64_t count, float alpha, mck_stream stream)
{
    if (count < 0)
        return fail(MCK_ERR_INVALID_ARG, "count must be >= 0");
    if (count == 0)
        return MCK_OK;
    if (!y || !x)
        return fail(MCK_ERR_INVALID_ARG, "y or x is NULL");
    const hipError_t err = mck::launch_axpy(y, x, count, alpha, static_cast<hipStream_t>(stream));
    if (err != hipSuccess)
        return hip_fail(err, "axpy launch");
    return MCK_OK;
}

void mck_shutdown(void)
{
    std::lock_guard<std::mutex> lock(g_mutex);
    // plans held by a recorded graph or a call in progress stay
    g_plans.clear_unpinned([](Plan& p) {
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(p.device);
        (void)hipDeviceSynchronize();
        (void)hipSetDevice(cur);
        free_plan(p);
    });
    // the cached temporaries (except those of calls in progress) and what the
    // pools keep
    std::lock_guard<std::mutex> tlock(g_temp_mutex);
    for (auto& kv : g_temps) {
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(kv.first);
        (void)hipDeviceSynchronize();
        for (TempSlot& t : kv.second.slot) {
            if (t.busy)
                continue;
            if (t.ptr != nullptr)
                (void)hipFree(t.ptr);
            if (t.done != nullptr)
                (void)hipEventDestroy(t.done);
            t = TempSlot();
        }
        if (kv.second.pool != nullptr)
            (void)hipMemPoolTrimTo(kv.second.pool, 0);
        (void)hipSetDevice(cur);
    }
}

}  // extern "C"
