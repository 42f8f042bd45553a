// ot_fmm.hip -- MI355X (gfx950) FP64 fast-multipole cell-to-cell interaction
// kernels behind the C ABI declared in include/ot_fmm.h.
//
// Method (paper Sec. 2.1: Octo-Tiger's gravity solver is an FMM on an octree
// of 8^3 sub-grids; Sec. 2.2.1 / 2.3: a kernel works on one sub-grid plus its
// ghost layers; Sec. 2.2.4: kernels of many sub-grids are aggregated into one
// launch). For each target cell i and |alpha| <= 3:
//   L_alpha(i) = sum_{j in S(i)} sum_{|beta|<=3-|alpha|} s_beta M_beta(j) G_{alpha+beta}(X_i - X_j)
// with G = -1/|r|, s_beta = (-1)^{|beta|}/beta!, S(i) the opening-criterion
// stencil (|j-i| > 4 and |floor(j/2) - floor(i/2)| <= 4) inside the 24^3 halo.
//
// Design (CDNA4):
//  * One work-group per target sub-grid (batched: per work-list entry). The
//    24^3 halo (2.54 MB of FP64 for moments + centres) cannot sit in the
//    160 KB LDS, so it streams through LDS one source z-plane at a time
//    (24 x 24 cells x 23 components = 106 KB), read from HBM with coalesced
//    512-byte rows.
//  * A wavefront = the 64 cells of one target z-plane (lane = x + 8 y). The
//    stencil depends only on the target's parity; the parities differing in
//    x or y are mirror images of each other (the criterion is invariant
//    under j -> 23 - j), so every lane walks the same per-z-parity offset
//    table (a list of (dy, dx-interval) rows per dz) with its own x/y sign.
//    Offsets are wave-uniform: no masking, scalar-unit loop control, and one
//    VALU add per offset for the LDS address. Bank mapping of the 8x8 lane
//    pattern with 24-wide rows is conflict-free for ds_read_b64.
//  * All arithmetic is FP64 VALU: per pair one rsqrt (v_rsq_f64 plus a
//    third-order Newton correction), the derivatives of 1/r from the radial
//    factors D_n = (-1)^{n+1} (2n-1)!! / r^{2n+1}, and the contraction
//    (84 FMAs for the multipole). Source moments are pre-scaled by s_beta
//    when staged, so the inner loop is FMAs only. There is no shared dense
//    operand between pairs, so MFMA does not apply.
//  * Missing neighbours are staged as zero moments at a far, finite centre:
//    their terms are exact zeros, identical to dropping the pairs.
//  * The adjoint is two gather passes with the same skeleton (no atomics):
//    a source-role pass per store sub-grid (sources = the target cells that
//    see it, carrying the weights) and a target-role pass per target.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <utility>
#include <unordered_map>
#include <vector>

#include "ot_common.h"
#include "ot_host.h"
#include "ot_fmm.h"
#include "ot_interact.h"
#include "ot_coarse.h"

namespace {
// wavefronts per work-group of the coarse substitutes: 8, one target per
// work-group (4 and 2, a part of a target each, measured 1.35x and 1.85x
// slower on the 32768-sub-grid workload: their staging is repeated per part)
constexpr int kCoarseWaves = 8;
}  // namespace


// ===========================================================================
// Host side
// ===========================================================================
namespace otfmm {

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_dev_mutex;
int g_dev_state[kMaxDevices];  // 0 unknown, 1 gfx950 ready, -1 unsupported

}  // namespace

int ensure_device()
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(OT_FMM_EUNSUPPORTED, "device index out of range");
    std::lock_guard<std::mutex> lock(g_dev_mutex);
    if (g_dev_state[dev] == 0) {
        hipDeviceProp_t prop;
        e = hipGetDeviceProperties(&prop, dev);
        if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
        const bool ok = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0;
        if (ok && !slot_counts().mirror_ok) {
            g_dev_state[dev] = -1;
            return fail(OT_FMM_EUNSUPPORTED, "stencil mirror check failed");
        }
        g_dev_state[dev] = ok ? 1 : -1;
    }
    if (g_dev_state[dev] < 0) return fail(OT_FMM_EUNSUPPORTED, "current device is not gfx950");
    return OT_FMM_OK;
}

}  // namespace otfmm

namespace {


template <int MODE, int NW, bool SPLIT = false, int NP = 1, bool PERSIST = false>
int launch(const KParams& kp, int nblocks, hipStream_t stream)
{
    if (nblocks <= 0) return OT_FMM_OK;
    hipLaunchKernelGGL((k_interact<MODE, NW, SPLIT, NP, PERSIST>), dim3(nblocks), dim3(NW * 64), 0, stream,
                       kp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return OT_FMM_OK;
}

constexpr int kDefaultSourceSched = OT_FMM_SCHED_W8;

constexpr int kShapeMask = 0x0f;

// a shape (W8, W16, W8P2), optionally with the persistent and local-order
// flags; or AUTO alone
bool valid_fwd_sched(int s)
{
    if (s == OT_FMM_SCHED_AUTO) return true;
    const int shape = s & kShapeMask;
    const int flags = s & ~kShapeMask;
    return s > 0 && (flags & ~(OT_FMM_SCHED_PERSISTENT | OT_FMM_SCHED_LOCAL)) == 0 &&
           shape >= OT_FMM_SCHED_W8 && shape <= OT_FMM_SCHED_W8P2;
}

// target role: any forward schedule; source role: AUTO, W8 or W8P2 (either
// optionally persistent)
bool valid_bwd_sched(int s)
{
    if (s < 0 || (s >> 16) != 0) return false;
    const int t = s & 0xff, r = s >> 8;
    return valid_fwd_sched(t) && valid_fwd_sched(r) && (r & kShapeMask) != OT_FMM_SCHED_W16;
}

// Work counters of persistent launches. Each launch takes a slot of
// kMaxPieces counters that no launch able to run at the same time shares:
//  * eager launches: one slot per stream -- launches on one stream run in
//    order, each preceded on that stream by the kernel that zeroes its slot
//    (kEagerSlots streams per plan);
//  * launches recorded into a graph (the stream is capturing): a slot of
//    their own that no other launch is given, since the graph may be
//    replayed at any time until it is destroyed, which the library cannot
//    see (kCaptureSlots per plan); the slots of the plan's own step graph
//    return to the pool when that graph is replaced.
constexpr int kEagerSlots = 64;
constexpr int kCaptureSlots = 960;
constexpr int kCounterSlots = kEagerSlots + kCaptureSlots;

// default schedule of every full-truncation pass (not autotuned): 8
// wavefronts in two passes, persistent, in the XCD-aware pieces -- measured
// 6% faster than one pass of 8 wavefronts for the forward and the adjoint
constexpr int kFullSched = OT_FMM_SCHED_W8P2 | OT_FMM_SCHED_PERSISTENT | OT_FMM_SCHED_LOCAL;

// default schedule of the forward with saved sums and of the one-pass adjoint
// when the plan has not been tuned (their 40 accumulators rule out 16
// wavefronts, as for the two-pass adjoint's source role)
constexpr int kSaveSched = OT_FMM_SCHED_W8P2 | OT_FMM_SCHED_PERSISTENT | OT_FMM_SCHED_LOCAL;

// kernels timed by the plan's events (ot_fmm_plan_kernel_times)
constexpr int kTimedKernels = OT_FMM_NKERNELS;

int pick_fwd(int sched, int tuned)
{
    if (sched == OT_FMM_SCHED_AUTO) sched = tuned ? tuned : OT_FMM_SCHED_W16;
    return sched;
}

}  // namespace

struct ot_fmm_plan_s {
    int device = 0;
    int32_t S = 0, T = 0;
    bool has_shift = false;
    double period[3] = {0.0, 0.0, 0.0};
    int64_t pairs = 0;
    int4* d_fwd_rel = nullptr;  // [T][27]
    int4* d_rev_rel = nullptr;  // [S][27]
    int* d_tgt = nullptr;       // [T]
    int* d_store_tgt = nullptr; // [S] target index of each store sub-grid, -1 if none
    int* d_fwd_order = nullptr; // [T] longest work first
    int* d_rev_order = nullptr; // [S]
    int* d_fwd_local = nullptr; // [T] XCD-aware (OT_FMM_SCHED_LOCAL)
    int* d_rev_local = nullptr; // [S]
    // the same XCD-aware pieces stored one after the other (persistent
    // launches in the local order: a counter per piece); npieces = 0 when the
    // device has more XCDs than kMaxPieces
    int* d_fwd_piece = nullptr; // [T]
    int* d_rev_piece = nullptr; // [S]
    int npieces = 0;
    int fwd_piece_off[kMaxPieces + 1] = {0};
    int rev_piece_off[kMaxPieces + 1] = {0};
    int tuned_fwd = 0, tuned_bwd = 0;
    int tuned_save = 0, tuned_saved_bwd = 0;  // forward with saved sums, one-pass adjoint
    // persistent launches: kMaxPieces work counters per slot; slots
    // [0, kEagerSlots) belong to streams (eager launches), the others to
    // launches recorded into graphs (see counter_slot)
    int* d_counters = nullptr;  // [kCounterSlots][kMaxPieces]
    std::mutex slot_mutex;
    std::vector<std::pair<hipStream_t, int>> stream_slot;  // eager: stream -> slot
    int next_capture = 0;                  // capture slots handed out so far
    std::vector<int> free_capture;         // capture slots returned by replaced step graphs
    std::vector<int> graph_slots;          // capture slots of the plan's step graph
    std::vector<int>* capture_log = nullptr;  // collects them while it is captured
    hipStream_t capture_stream = nullptr;     // on this stream
    int n_cu = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    // per-kernel timing (forward, adjoint source pass, adjoint target pass,
    // forward with saved sums, one-pass adjoint, forward with the
    // angular-momentum correction)
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pool[kTimedKernels];
    size_t ev_used[kTimedKernels] = {};
    // coarse substitutes for missing neighbours (ot_fmm_plan_set_coarse)
    std::vector<uint32_t> missing;  // [T] bit s: slot s has no fine neighbour
    int32_t Sp_coarse = 0;
    int n_coarse_items = 0;  // work items: targets with substitutes x parts
    int4* d_cf_items = nullptr;     // {target, lane order, first entry, entries}, most work first
    int4* d_cf_entries = nullptr;   // {slot, coarse node, octant, 0}
    int* d_cf_cells = nullptr;      // [orders][512] target cell of each lane
    unsigned long long* d_cf_mask = nullptr;  // [27][512] included coarse cells per target cell
};

namespace {

// Event pair bracketing one launch of kernel `which` on `stream`, or a null
// pair when timing is off. Events come from a per-plan pool.
int timing_begin(ot_fmm_plan plan, int which, hipStream_t stream,
                 std::pair<hipEvent_t, hipEvent_t>* ev)
{
    *ev = {nullptr, nullptr};
    if (!plan->timing || which < 0) return OT_FMM_OK;
    auto& pool = plan->ev_pool[which];
    size_t& used = plan->ev_used[which];
    if (used == pool.size()) {
        hipEvent_t a, b;
        OT_HIP(hipEventCreate(&a));
        OT_HIP(hipEventCreate(&b));
        pool.emplace_back(a, b);
    }
    *ev = pool[used++];
    OT_HIP(hipEventRecord(ev->first, stream));
    return OT_FMM_OK;
}

int timing_end(const std::pair<hipEvent_t, hipEvent_t>& ev, hipStream_t stream)
{
    if (ev.second) OT_HIP(hipEventRecord(ev.second, stream));
    return OT_FMM_OK;
}

// Work-groups of one instantiation resident per CU (LDS and registers), from
// the runtime's occupancy calculator, computed once.
template <int MODE, int NW, int NP>
int resident_per_cu()
{
    static const int n = [] {
        int b = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_interact<MODE, NW, false, NP, true>, NW * 64, 0) !=
                hipSuccess ||
            b < 1)
            b = 1;
        return b;
    }();
    return n;
}

// The counter slot of a persistent launch on `stream` (kEagerSlots /
// kCaptureSlots rules above).
int counter_slot(ot_fmm_plan plan, hipStream_t stream, int** out)
{
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    OT_HIP(hipStreamIsCapturing(stream, &st));
    std::lock_guard<std::mutex> lock(plan->slot_mutex);
    int slot = -1;
    if (st != hipStreamCaptureStatusNone) {
        if (!plan->free_capture.empty()) {
            slot = plan->free_capture.back();
            plan->free_capture.pop_back();
        } else if (plan->next_capture < kCaptureSlots) {
            slot = kEagerSlots + plan->next_capture++;
        } else {
            return fail(OT_FMM_EINVAL, "more persistent launches recorded into graphs than the plan's "
                                       "960 counter slots; use a non-persistent schedule or a new plan");
        }
        if (plan->capture_log && stream == plan->capture_stream) plan->capture_log->push_back(slot);
    } else {
        for (const auto& e : plan->stream_slot)
            if (e.first == stream) {
                slot = e.second;
                break;
            }
        if (slot < 0) {
            if ((int)plan->stream_slot.size() >= kEagerSlots)
                return fail(OT_FMM_EINVAL, "persistent launches of one plan on more than 64 streams; use a "
                                           "non-persistent schedule or another plan");
            slot = (int)plan->stream_slot.size();
            plan->stream_slot.emplace_back(stream, slot);
        }
    }
    *out = plan->d_counters + (size_t)slot * kMaxPieces;
    return OT_FMM_OK;
}

// One launch over `nblocks` work-list entries: a work-group per entry, or
// (persistent) as many work-groups as fit the device at once, each taking
// entries from a counter slot of the plan, zeroed just before on the stream.
template <int MODE, int NW, int NP = 1>
int launch_timed(ot_fmm_plan plan, int which, KParams kp, int nblocks, bool persistent,
                 hipStream_t stream)
{
    int* c = nullptr;
    if (persistent && nblocks > 0) {
        const int rs = counter_slot(plan, stream, &c);
        if (rs) return rs;
    }
    std::pair<hipEvent_t, hipEvent_t> ev;
    int rc = timing_begin(plan, which, stream, &ev);
    if (rc) return rc;
    if (persistent && nblocks > 0) {
        hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(kMaxPieces), 0, stream, c);
        kp.counter = c;
        kp.n_items = nblocks;
        const long resident = (long)plan->n_cu * resident_per_cu<MODE, NW, NP>();
        nblocks = (int)std::min<long>(nblocks, resident);
    }
    rc = persistent ? launch<MODE, NW, false, NP, true>(kp, nblocks, stream)
                    : launch<MODE, NW, false, NP, false>(kp, nblocks, stream);
    if (rc) return rc;
    return timing_end(ev, stream);
}

// The work order of a launch: XCD-aware (OT_FMM_SCHED_LOCAL) or longest work
// first (already in kp.order); a persistent launch in the XCD-aware order
// takes the pieces with a counter each.
void apply_order(KParams& kp, const ot_fmm_plan_s* plan, int sched, bool rev)
{
    if (!(sched & OT_FMM_SCHED_LOCAL)) return;
    if ((sched & OT_FMM_SCHED_PERSISTENT) && plan->npieces > 0) {
        kp.order = rev ? plan->d_rev_piece : plan->d_fwd_piece;
        kp.npieces = plan->npieces;
        const int* off = rev ? plan->rev_piece_off : plan->fwd_piece_off;
        for (int k = 0; k <= plan->npieces; ++k) kp.piece_off[k] = off[k];
    } else {
        kp.order = rev ? plan->d_rev_local : plan->d_fwd_local;
    }
}

int fwd_batched(ot_fmm_plan plan, const double* M, const double* com, double* L, int sched,
                hipStream_t stream)
{
    KParams kp{};
    kp.mom = M;
    kp.pos = com;
    kp.mom_stride = (long)plan->S * kSub3;
    kp.pos_stride = (long)plan->S * kSub3;
    kp.rel = plan->d_fwd_rel;
    kp.own_blk = plan->d_tgt;
    kp.order = plan->d_fwd_order;
    kp.out0 = L;
    kp.out_stride = (long)plan->T * kSub3;
    kp.out_blk = nullptr;
    for (int k = 0; k < 3; ++k) kp.period[k] = plan->period[k];
    sched = pick_fwd(sched, plan->tuned_fwd);
    const bool pers = (sched & OT_FMM_SCHED_PERSISTENT) != 0;
    apply_order(kp, plan, sched, false);
    const int shape = sched & kShapeMask;
    if (shape == OT_FMM_SCHED_W8) return launch_timed<MODE_FWD_STORE, 8>(plan, 0, kp, plan->T, pers, stream);
    if (shape == OT_FMM_SCHED_W16)
        return launch_timed<MODE_FWD_STORE, 16>(plan, 0, kp, plan->T, pers, stream);
    if (shape == OT_FMM_SCHED_W8P2)
        return launch_timed<MODE_FWD_STORE, 8, 2>(plan, 0, kp, plan->T, pers, stream);
    return fail(OT_FMM_EINVAL, "unknown forward schedule");
}

// Forward with the full truncation: the same plan, tables and schedules as
// the forward (not timed by the plan's events); kFullSched by default.
int fwd_full_batched(ot_fmm_plan plan, const double* M, const double* com, double* L, int sched,
                     hipStream_t stream)
{
    KParams kp{};
    kp.mom = M;
    kp.pos = com;
    kp.mom_stride = (long)plan->S * kSub3;
    kp.pos_stride = (long)plan->S * kSub3;
    kp.rel = plan->d_fwd_rel;
    kp.own_blk = plan->d_tgt;
    kp.order = plan->d_fwd_order;
    kp.out0 = L;
    kp.out_stride = (long)plan->T * kSub3;
    kp.out_blk = nullptr;
    for (int k = 0; k < 3; ++k) kp.period[k] = plan->period[k];
    if (sched == OT_FMM_SCHED_AUTO) sched = kFullSched;
    const bool pers = (sched & OT_FMM_SCHED_PERSISTENT) != 0;
    apply_order(kp, plan, sched, false);
    const int shape = sched & kShapeMask;
    if (shape == OT_FMM_SCHED_W8) return launch_timed<MODE_FULL_STORE, 8>(plan, -1, kp, plan->T, pers, stream);
    if (shape == OT_FMM_SCHED_W16)
        return launch_timed<MODE_FULL_STORE, 16>(plan, -1, kp, plan->T, pers, stream);
    if (shape == OT_FMM_SCHED_W8P2)
        return launch_timed<MODE_FULL_STORE, 8, 2>(plan, -1, kp, plan->T, pers, stream);
    return fail(OT_FMM_EINVAL, "unknown forward schedule");
}

// Adjoint of the batched forward (FULL: of the full truncation, with
// derivatives to order 7; kFullSched by default, 16 wavefronts refused -- their
// register budget is far below what the order-7 sums hold -- and not timed
// by the plan's events).
template <bool FULL>
int bwd_any(ot_fmm_plan plan, const double* M, const double* com, const double* gL, double* gM,
            double* gcom, int sched, hipStream_t stream, int passes = 3)
{
    // passes: bit 0 the source-role pass, bit 1 the target-role pass (the
    // autotuner times them one at a time; callers always run both)
    constexpr int kB2 = FULL ? MODE_B2F_STORE : MODE_B2_STORE;
    constexpr int kB1 = FULL ? MODE_B1F_STORE : MODE_B1_STORE;
    const int w2 = FULL ? -1 : 1, w1 = FULL ? -1 : 2;
    // target-role schedule in the low byte, source-role schedule in the next
    int tsched = sched & 0xff, ssched = (sched >> 8) & 0xff;
    if (tsched == OT_FMM_SCHED_AUTO)
        tsched = FULL ? kFullSched
                      : ((plan->tuned_bwd & 0xff) ? (plan->tuned_bwd & 0xff) : OT_FMM_SCHED_W16);
    if (ssched == OT_FMM_SCHED_AUTO)
        ssched = FULL ? kFullSched : ((plan->tuned_bwd >> 8) ? (plan->tuned_bwd >> 8) : kDefaultSourceSched);
    if (!valid_bwd_sched(tsched | (ssched << 8))) return fail(OT_FMM_EINVAL, "unknown backward schedule");
    if (FULL && (tsched & kShapeMask) == OT_FMM_SCHED_W16)
        return fail(OT_FMM_EINVAL, "16 wavefronts are not available for the full truncation's adjoint");
    const long NS = (long)plan->S * kSub3, NT = (long)plan->T * kSub3;
    // source role: owners are store sub-grids, sources the target cells that see them
    KParams b2{};
    b2.mom = gL;
    b2.mom_stride = NT;
    b2.pos = com;
    b2.pos_stride = NS;
    b2.rel = plan->d_rev_rel;
    b2.own_blk = nullptr;
    b2.order = plan->d_rev_order;
    b2.aux = M;
    b2.aux_stride = NS;
    b2.out0 = gM;
    b2.out1 = gcom;
    b2.out_stride = NS;
    b2.out_blk = nullptr;
    for (int k = 0; k < 3; ++k) b2.period[k] = plan->period[k];
    // the source-role pass has 8 wavefronts (its 40 accumulators do not fit
    // the register budget of 16): one pass, or two with split rows
    const bool spers = (ssched & OT_FMM_SCHED_PERSISTENT) != 0;
    apply_order(b2, plan, ssched, true);
    if (passes & 1) {
        const int rc = (ssched & kShapeMask) == OT_FMM_SCHED_W8P2
                           ? launch_timed<kB2, 8, 2>(plan, w2, b2, plan->S, spers, stream)
                           : launch_timed<kB2, 8>(plan, w2, b2, plan->S, spers, stream);
        if (rc) return rc;
    }
    if (!(passes & 2)) return OT_FMM_OK;
    // target role: owners are targets, sources their neighbours' cells
    KParams b1{};
    b1.mom = M;
    b1.mom_stride = NS;
    b1.pos = com;
    b1.pos_stride = NS;
    b1.rel = plan->d_fwd_rel;
    b1.own_blk = plan->d_tgt;
    b1.order = plan->d_fwd_order;
    b1.aux = gL;
    b1.aux_stride = NT;
    b1.out0 = gcom;
    b1.out_stride = NS;
    b1.out_blk = plan->d_tgt;
    for (int k = 0; k < 3; ++k) b1.period[k] = plan->period[k];
    const bool tpers = (tsched & OT_FMM_SCHED_PERSISTENT) != 0;
    apply_order(b1, plan, tsched, false);
    const int tshape = tsched & kShapeMask;
    if constexpr (!FULL)
        if (tshape == OT_FMM_SCHED_W16) return launch_timed<kB1, 16>(plan, w1, b1, plan->T, tpers, stream);
    if (tshape == OT_FMM_SCHED_W8P2) return launch_timed<kB1, 8, 2>(plan, w1, b1, plan->T, tpers, stream);
    return launch_timed<kB1, 8>(plan, w1, b1, plan->T, tpers, stream);
}

int bwd_batched(ot_fmm_plan plan, const double* M, const double* com, const double* gL, double* gM,
                double* gcom, int sched, hipStream_t stream)
{
    return bwd_any<false>(plan, M, com, gL, gM, gcom, sched, stream);
}

// A schedule of the forward with saved sums or of the one-pass adjoint:
// AUTO, or W8 / W8P2 with the persistent and XCD-aware flags.
bool valid_save_sched(int s)
{
    return s == OT_FMM_SCHED_AUTO || (valid_fwd_sched(s) && (s & kShapeMask) != OT_FMM_SCHED_W16);
}

// Forward that also writes the target-role sums of the adjoint,
// C'_g(i) = sum_j sum_{|b| <= 4-|g|} s_b M_b(j) G_{g+b}(X_i - X_j), 1 <= |g| <= 4
// (= dL_a(i)/dX_i,k for g = a + e_k), 24 kept components [24][T*512].
// FULL: the full truncation, C'_g = sum_j sum_{|b| <= 3} s_b M_b(j) G_{g+b}
// (its orders 1..3 are L itself), derivatives to order 7.
template <bool FULL = false>
int fwd_save_batched(ot_fmm_plan plan, const double* M, const double* com, double* L, double* Cs, int sched,
                     hipStream_t stream)
{
    constexpr int kMode = FULL ? MODE_FSF_STORE : MODE_FS_STORE;
    KParams kp{};
    kp.mom = M;
    kp.pos = com;
    kp.mom_stride = (long)plan->S * kSub3;
    kp.pos_stride = (long)plan->S * kSub3;
    kp.rel = plan->d_fwd_rel;
    kp.own_blk = plan->d_tgt;
    kp.order = plan->d_fwd_order;
    kp.out0 = L;
    kp.out1 = Cs;
    kp.out_stride = (long)plan->T * kSub3;
    kp.out_blk = nullptr;
    for (int k = 0; k < 3; ++k) kp.period[k] = plan->period[k];
    if (sched == OT_FMM_SCHED_AUTO) sched = (!FULL && plan->tuned_save) ? plan->tuned_save : kSaveSched;
    const bool pers = (sched & OT_FMM_SCHED_PERSISTENT) != 0;
    apply_order(kp, plan, sched, false);
    const int shape = sched & kShapeMask;
    const int which = FULL ? -1 : 3;
    if (shape == OT_FMM_SCHED_W8) return launch_timed<kMode, 8>(plan, which, kp, plan->T, pers, stream);
    if (shape == OT_FMM_SCHED_W8P2)
        return launch_timed<kMode, 8, 2>(plan, which, kp, plan->T, pers, stream);
    return fail(OT_FMM_EINVAL, "unknown schedule for the forward with saved sums");
}

// Forward with the angular-momentum correction of the force: L, and
// dF_k(i) = -sum_{j in S(i)} sum_{|a|+|b| = 3} (M_a(i)/a!) s_b M_b(j) G_{a+b+e_k}(X_i - X_j),
// [3][T*512]. Same pair loop as the forward with saved sums.
int fwd_amc_batched(ot_fmm_plan plan, const double* M, const double* com, double* L, double* dF, int sched,
                    hipStream_t stream)
{
    KParams kp{};
    kp.mom = M;
    kp.pos = com;
    kp.mom_stride = (long)plan->S * kSub3;
    kp.pos_stride = (long)plan->S * kSub3;
    kp.rel = plan->d_fwd_rel;
    kp.own_blk = plan->d_tgt;
    kp.order = plan->d_fwd_order;
    kp.aux = M;
    kp.aux_stride = (long)plan->S * kSub3;
    kp.out0 = L;
    kp.out1 = dF;
    kp.out_stride = (long)plan->T * kSub3;
    kp.out_blk = nullptr;
    for (int k = 0; k < 3; ++k) kp.period[k] = plan->period[k];
    if (sched == OT_FMM_SCHED_AUTO) sched = plan->tuned_save ? plan->tuned_save : kSaveSched;
    const bool pers = (sched & OT_FMM_SCHED_PERSISTENT) != 0;
    apply_order(kp, plan, sched, false);
    const int shape = sched & kShapeMask;
    if (shape == OT_FMM_SCHED_W8) return launch_timed<MODE_AMC_STORE, 8>(plan, 5, kp, plan->T, pers, stream);
    if (shape == OT_FMM_SCHED_W8P2)
        return launch_timed<MODE_AMC_STORE, 8, 2>(plan, 5, kp, plan->T, pers, stream);
    return fail(OT_FMM_EINVAL, "unknown schedule for the forward with the angular-momentum correction");
}

// One-pass adjoint from the saved sums: the source-role pass over every store
// sub-grid, whose epilogue adds the target role of the sub-grid's own cells
// (when it is a target) from the saved sums and gL. FULL: of the full truncation.
template <bool FULL = false>
int bwd_saved_batched(ot_fmm_plan plan, const double* M, const double* com, const double* gL, const double* Cs,
                      double* gM, double* gcom, int sched, hipStream_t stream)
{
    constexpr int kMode = FULL ? MODE_B2SF_STORE : MODE_B2S_STORE;
    const long NS = (long)plan->S * kSub3, NT = (long)plan->T * kSub3;
    KParams kp{};
    kp.mom = gL;
    kp.mom_stride = NT;
    kp.pos = com;
    kp.pos_stride = NS;
    kp.rel = plan->d_rev_rel;
    kp.own_blk = nullptr;
    kp.order = plan->d_rev_order;
    kp.aux = M;
    kp.aux_stride = NS;
    kp.store_tgt = plan->d_store_tgt;
    kp.aux2 = gL;
    kp.save = Cs;
    kp.aux_stride2 = NT;
    kp.out0 = gM;
    kp.out1 = gcom;
    kp.out_stride = NS;
    kp.out_blk = nullptr;
    for (int k = 0; k < 3; ++k) kp.period[k] = plan->period[k];
    if (sched == OT_FMM_SCHED_AUTO)
        sched = (!FULL && plan->tuned_saved_bwd) ? plan->tuned_saved_bwd : kSaveSched;
    const bool pers = (sched & OT_FMM_SCHED_PERSISTENT) != 0;
    apply_order(kp, plan, sched, true);
    const int shape = sched & kShapeMask;
    const int which = FULL ? -1 : 4;
    if (shape == OT_FMM_SCHED_W8) return launch_timed<kMode, 8>(plan, which, kp, plan->S, pers, stream);
    if (shape == OT_FMM_SCHED_W8P2)
        return launch_timed<kMode, 8, 2>(plan, which, kp, plan->S, pers, stream);
    return fail(OT_FMM_EINVAL, "unknown schedule for the one-pass adjoint");
}

int check_plan(ot_fmm_plan plan)
{
    if (!plan) return fail(OT_FMM_EINVAL, "null plan");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != plan->device) return fail(OT_FMM_EINVAL, "plan belongs to another device");
    return OT_FMM_OK;
}

void free_plan_memory(ot_fmm_plan p)
{
    for (auto& pool : p->ev_pool)
        for (auto& ev : pool) {
            (void)hipEventDestroy(ev.first);
            (void)hipEventDestroy(ev.second);
        }
    if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->graph_exec = nullptr;
    p->graph = nullptr;
    (void)hipFree(p->d_fwd_rel);
    (void)hipFree(p->d_rev_rel);
    (void)hipFree(p->d_tgt);
    (void)hipFree(p->d_store_tgt);
    (void)hipFree(p->d_fwd_order);
    (void)hipFree(p->d_rev_order);
    (void)hipFree(p->d_fwd_local);
    (void)hipFree(p->d_rev_local);
    (void)hipFree(p->d_fwd_piece);
    (void)hipFree(p->d_rev_piece);
    (void)hipFree(p->d_counters);
    (void)hipFree(p->d_cf_items);
    (void)hipFree(p->d_cf_entries);
    (void)hipFree(p->d_cf_cells);
    (void)hipFree(p->d_cf_mask);
    p->d_cf_items = nullptr;
    p->d_cf_entries = nullptr;
    p->d_cf_cells = nullptr;
    p->d_cf_mask = nullptr;
}

// Work order: longest work first (a greedy longest-processing-time list for
// the hardware dispatcher), ties kept in store order for locality.
std::vector<int> lpt_order(const std::vector<int64_t>& work)
{
    std::vector<int> idx(work.size());
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return work[a] > work[b]; });
    return idx;
}

// Spatial position of neighbour slot q relative to the owner.
inline void slot_delta(int q, int* d)
{
    d[0] = q % 3 - 1;
    d[1] = (q / 3) % 3 - 1;
    d[2] = q / 9 - 1;
}

uint64_t spread_bits(uint64_t v)  // 21 bits -> every third bit
{
    v &= 0x1fffff;
    v = (v | v << 32) & 0x1f00000000ffffULL;
    v = (v | v << 16) & 0x1f0000ff0000ffULL;
    v = (v | v << 8) & 0x100f00f00f00f00fULL;
    v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
    v = (v | v << 2) & 0x1249249249249249ULL;
    return v;
}

// XCD-aware work order. A launch's work-groups go to the XCDs round robin
// (work-group b to XCD b % nxcd), and each XCD has its own L2. Lattice
// coordinates are recovered from the neighbour graph (breadth-first, one
// component at a time), the entries are sorted along a Morton curve, the curve
// is cut into nxcd pieces of equal work, and the pieces are interleaved so
// that each XCD walks one spatially compact piece: the neighbour blocks that
// its concurrently resident work-groups stage overlap and are found in its L2.
// adj[v] lists (neighbour entry, slot of the neighbour seen from v).
std::vector<int> locality_order(const std::vector<std::vector<std::pair<int, int>>>& adj,
                                const std::vector<int64_t>& work, int nxcd, std::vector<int>* pieces = nullptr,
                                std::vector<int>* piece_off = nullptr)
{
    const int n = (int)adj.size();
    std::vector<int> comp(n, -1);
    std::vector<std::array<int64_t, 3>> pos(n);
    std::vector<int> queue;
    queue.reserve(n);
    int ncomp = 0;
    for (int seed = 0; seed < n; ++seed) {
        if (comp[seed] >= 0) continue;
        const size_t first = queue.size();
        comp[seed] = ncomp;
        pos[seed] = {0, 0, 0};
        queue.push_back(seed);
        for (size_t h = first; h < queue.size(); ++h) {
            const int v = queue[h];
            for (const auto& e : adj[v]) {
                if (comp[e.first] >= 0) continue;
                int d[3];
                slot_delta(e.second, d);
                comp[e.first] = ncomp;
                pos[e.first] = {pos[v][0] + d[0], pos[v][1] + d[1], pos[v][2] + d[2]};
                queue.push_back(e.first);
            }
        }
        int64_t lo[3] = {INT64_MAX, INT64_MAX, INT64_MAX};
        for (size_t h = first; h < queue.size(); ++h)
            for (int k = 0; k < 3; ++k) lo[k] = std::min(lo[k], pos[queue[h]][k]);
        for (size_t h = first; h < queue.size(); ++h)
            for (int k = 0; k < 3; ++k) pos[queue[h]][k] -= lo[k];
        ++ncomp;
    }
    std::vector<uint64_t> key(n);
    for (int v = 0; v < n; ++v)
        key[v] = spread_bits((uint64_t)pos[v][0]) | spread_bits((uint64_t)pos[v][1]) << 1 |
                 spread_bits((uint64_t)pos[v][2]) << 2;
    std::vector<int> curve(n);
    std::iota(curve.begin(), curve.end(), 0);
    std::stable_sort(curve.begin(), curve.end(), [&](int a, int b) {
        return comp[a] != comp[b] ? comp[a] < comp[b] : key[a] < key[b];
    });
    // pieces of equal work
    int64_t total = 0;
    for (int64_t w : work) total += w;
    std::vector<std::vector<int>> piece(nxcd);
    int64_t run = 0;
    for (int v : curve) {
        const int x = total > 0 ? (int)std::min<int64_t>(nxcd - 1, run * nxcd / total) : 0;
        piece[x].push_back(v);
        run += work[v];
    }
    if (pieces && piece_off) {
        pieces->clear();
        piece_off->assign(1, 0);
        for (int x = 0; x < nxcd; ++x) {
            pieces->insert(pieces->end(), piece[x].begin(), piece[x].end());
            piece_off->push_back((int)pieces->size());
        }
    }
    std::vector<int> order;
    order.reserve(n);
    for (size_t i = 0; order.size() < (size_t)n; ++i)
        for (int x = 0; x < nxcd; ++x)
            if (i < piece[x].size()) order.push_back(piece[x][i]);
    return order;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
namespace {

// Host part of a plan: validation of the descriptor, forward and inverse
// relations, exact pair counts and the work orders (no device call).
struct HostTables {
    std::vector<int4> fwd, rev;
    std::vector<int64_t> fwd_work;
    std::vector<int> tg, fo, ro;
    std::vector<int> fo_local, ro_local;  // XCD-aware orders (filled by make_local_orders)
    std::vector<int> fo_piece, ro_piece, fo_off, ro_off;  // the same, piece after piece
    std::vector<int64_t> rev_work;
    int64_t pairs = 0;
};

// XCD-aware orders of both work lists: targets linked through their
// neighbour slots, store sub-grids through the targets that see them.
void make_local_orders(int32_t S, int32_t T, const int32_t* nbr, HostTables* h, int nxcd)
{
    std::vector<int> tindex(S, -1);
    for (int t = 0; t < T; ++t) tindex[h->tg[t]] = t;
    std::vector<std::vector<std::pair<int, int>>> adj(T), radj(S);
    for (int t = 0; t < T; ++t)
        for (int q = 0; q < 27; ++q) {
            const int32_t b = nbr[(int64_t)t * 27 + q];
            if (q == 13 || b < 0) continue;
            if (tindex[b] >= 0) adj[t].emplace_back(tindex[b], q);
            // store block b sees the target's own block at the opposite slot
            radj[b].emplace_back(h->tg[t], 26 - q);
        }
    h->fo_local = locality_order(adj, h->fwd_work, nxcd, &h->fo_piece, &h->fo_off);
    h->ro_local = locality_order(radj, h->rev_work, nxcd, &h->ro_piece, &h->ro_off);
}

int build_host_tables(int32_t S, int32_t T, const int32_t* tgt, const int32_t* nbr, const int8_t* shift,
                      const double* period, HostTables* h)
{
    if (S <= 0 || T <= 0) return fail(OT_FMM_EINVAL, "S and T must be positive");
    if ((int64_t)S * kSub3 * 20 > ((int64_t)1 << 40) || (int64_t)T * 27 > ((int64_t)1 << 31))
        return fail(OT_FMM_EINVAL, "descriptor too large");
    if (!tgt || !nbr) return fail(OT_FMM_EINVAL, "null tgt or nbr");
    if (shift && !period) return fail(OT_FMM_EINVAL, "shift given without period");
    std::vector<char> seen(S, 0);
    for (int t = 0; t < T; ++t) {
        if (tgt[t] < 0 || tgt[t] >= S) return fail(OT_FMM_EINVAL, "tgt out of range");
        if (seen[tgt[t]]) return fail(OT_FMM_EINVAL, "tgt entries must be distinct");
        seen[tgt[t]] = 1;
        for (int s = 0; s < 27; ++s) {
            const int32_t v = nbr[(int64_t)t * 27 + s];
            if (v < -1 || v >= S) return fail(OT_FMM_EINVAL, "nbr out of range");
        }
        if (nbr[(int64_t)t * 27 + 13] != tgt[t]) return fail(OT_FMM_EINVAL, "nbr[t][13] != tgt[t]");
    }
    if (period)
        for (int k = 0; k < 3; ++k)
            if (!(period[k] == period[k]) || period[k] > 1e15 || period[k] < -1e15)
                return fail(OT_FMM_EINVAL, "period must be finite");
    const SlotCounts& sc = slot_counts();
    std::vector<int4>& fwd = h->fwd;
    std::vector<int4>& rev = h->rev;
    fwd.assign((size_t)T * 27, make_int4(0, 0, 0, 0));
    rev.assign((size_t)S * 27, make_int4(0, 0, 0, 0));
    for (auto& r : rev) r = make_int4(-1, -1, 0, 0);
    std::vector<int64_t> fwd_work(T, 0), rev_work(S, 0);
    int64_t pairs = 0;
    for (int t = 0; t < T; ++t)
        for (int s = 0; s < 27; ++s) {
            const int32_t b = nbr[(int64_t)t * 27 + s];
            int packed = 0, packed_neg = 0;
            if (shift) {
                for (int k = 0; k < 3; ++k) {
                    const int v = shift[((int64_t)t * 27 + s) * 3 + k];
                    packed |= (v & 0xff) << (8 * k);
                    packed_neg |= ((-v) & 0xff) << (8 * k);
                }
            }
            fwd[(size_t)t * 27 + s] = make_int4(b, b, packed, 0);
            if (b < 0) continue;
            if (shift)
                for (int k = 0; k < 3; ++k)
                    if (shift[((int64_t)t * 27 + s) * 3 + k] == -128)
                        return fail(OT_FMM_EINVAL, "shift of -128 cannot be negated");
            const size_t ri = (size_t)b * 27 + (26 - s);
            if (rev[ri].x >= 0)
                return fail(OT_FMM_EINVAL, "two targets claim the same (source, slot) relation");
            rev[ri] = make_int4(t, tgt[t], packed_neg, 0);
            fwd_work[t] += sc.pairs[s];
            rev_work[b] += sc.pairs[s];
            pairs += sc.pairs[s];
        }
    h->tg.assign(tgt, tgt + T);
    h->fo = lpt_order(fwd_work);
    h->ro = lpt_order(rev_work);
    h->pairs = pairs;
    h->fwd_work.swap(fwd_work);
    h->rev_work.swap(rev_work);
    return OT_FMM_OK;
}

}  // namespace

namespace {
// Captures the launches `enqueue(stream)` makes into the plan's step graph
// (replacing any previous one): the counter slots its persistent launches
// take belong to the graph and return to the pool when it is replaced.
template <class F>
int capture_step_graph(ot_fmm_plan plan, F&& enqueue)
{
    hipStream_t cs;
    OT_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(cs);
        return hip_fail(e, "hipStreamBeginCapture");
    }
    const bool timing = plan->timing;
    plan->timing = false;  // no timing events inside the graph
    std::vector<int> slots;  // counter slots the captured launches take
    {
        std::lock_guard<std::mutex> lock(plan->slot_mutex);
        plan->capture_log = &slots;
        plan->capture_stream = cs;
    }
    int rc = enqueue(cs);
    plan->timing = timing;
    {
        std::lock_guard<std::mutex> lock(plan->slot_mutex);
        plan->capture_log = nullptr;
        plan->capture_stream = nullptr;
    }
    // slots of a graph that is never instantiated go back to the pool
    auto give_back = [&](const std::vector<int>& v) {
        std::lock_guard<std::mutex> lock(plan->slot_mutex);
        plan->free_capture.insert(plan->free_capture.end(), v.begin(), v.end());
    };
    e = hipStreamEndCapture(cs, &g);
    (void)hipStreamDestroy(cs);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        give_back(slots);
        return rc;
    }
    if (e != hipSuccess) {
        give_back(slots);
        return hip_fail(e, "hipStreamEndCapture");
    }
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        give_back(slots);
        return hip_fail(e, "hipGraphInstantiate");
    }
    if (plan->graph_exec) {
        // a replay of the graph being replaced may still run: its counter
        // slots are reused only once the device is idle
        e = hipDeviceSynchronize();
        if (e != hipSuccess) {
            (void)hipGraphExecDestroy(ex);
            (void)hipGraphDestroy(g);
            give_back(slots);
            return hip_fail(e, "hipDeviceSynchronize");
        }
        (void)hipGraphExecDestroy(plan->graph_exec);
        give_back(plan->graph_slots);
    }
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    plan->graph = g;
    plan->graph_exec = ex;
    plan->graph_slots.swap(slots);
    return OT_FMM_OK;
}

}  // namespace

extern "C" {

int ot_fmm_version(void) { return OT_FMM_VERSION; }

const char* ot_fmm_strerror(int code)
{
    switch (code) {
    case OT_FMM_OK: return "ok";
    case OT_FMM_EINVAL: return "invalid argument";
    case OT_FMM_EHIP: return "HIP runtime error";
    case OT_FMM_ENOMEM: return "device allocation failed";
    case OT_FMM_EUNSUPPORTED: return "unsupported device";
    case OT_FMM_ETIMEDOUT: return "timed out";
    default: return "unknown error";
    }
}

const char* ot_fmm_last_error(void) { return g_last_error.c_str(); }

int ot_fmm_monopole(const double* mass, const double* com, double* L, void* stream)
{
    g_last_error.clear();
    if (!aligned8(mass) || !aligned8(com) || !aligned8(L))
        return fail(OT_FMM_EINVAL, "null or misaligned (8-byte) pointer");
    if (overlap(L, 20 * kSub3, mass, kHalo3) || overlap(L, 20 * kSub3, com, 3 * kHalo3))
        return fail(OT_FMM_EINVAL, "L overlaps an input");
    int rc = ensure_device();
    if (rc) return rc;
    KParams kp{};
    kp.mom = mass;
    kp.pos = com;
    kp.out0 = L;
    return launch<MODE_MONO_HALO, 8, true>(kp, kSub, (hipStream_t)stream);
}

int ot_fmm_multipole(const double* M, const double* com, double* L, void* stream)
{
    g_last_error.clear();
    if (!aligned8(M) || !aligned8(com) || !aligned8(L))
        return fail(OT_FMM_EINVAL, "null or misaligned (8-byte) pointer");
    if (overlap(L, 20 * kSub3, M, 20 * kHalo3) || overlap(L, 20 * kSub3, com, 3 * kHalo3))
        return fail(OT_FMM_EINVAL, "L overlaps an input");
    int rc = ensure_device();
    if (rc) return rc;
    KParams kp{};
    kp.mom = M;
    kp.pos = com;
    kp.out0 = L;
    return launch<MODE_FWD_HALO, 8, true>(kp, kSub, (hipStream_t)stream);
}

int ot_fmm_plan_create(int32_t S, int32_t T, const int32_t* tgt, const int32_t* nbr,
                       const int8_t* shift, const double* period, ot_fmm_plan* out)
{
    g_last_error.clear();
    if (!out) return fail(OT_FMM_EINVAL, "null output pointer");
    *out = nullptr;
    HostTables ht;
    int rc = build_host_tables(S, T, tgt, nbr, shift, period, &ht);
    if (rc) return rc;
    const std::vector<int4>& fwd = ht.fwd;
    const std::vector<int4>& rev = ht.rev;
    const std::vector<int>& tg = ht.tg;
    const std::vector<int>& fo = ht.fo;
    const std::vector<int>& ro = ht.ro;
    const int64_t pairs = ht.pairs;
    rc = ensure_device();
    if (rc) return rc;

    ot_fmm_plan p = new (std::nothrow) ot_fmm_plan_s();
    if (!p) return fail(OT_FMM_ENOMEM, "host allocation failed");
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
        delete p;
        return hip_fail(e, "hipGetDevice");
    }
    p->S = S;
    p->T = T;
    p->has_shift = shift != nullptr;
    if (period)
        for (int k = 0; k < 3; ++k) p->period[k] = period[k];
    p->pairs = pairs;
    p->missing.assign(T, 0u);
    for (int t = 0; t < T; ++t)
        for (int q = 0; q < 27; ++q)
            if (nbr[(int64_t)t * 27 + q] < 0) p->missing[t] |= 1u << q;
    hipDeviceProp_t prop;
    if ((e = hipGetDeviceProperties(&prop, p->device)) != hipSuccess) {
        delete p;
        return hip_fail(e, "hipGetDeviceProperties");
    }
    p->n_cu = prop.multiProcessorCount;
    int nxcd = 1;
    if (hipDeviceGetAttribute(&nxcd, hipDeviceAttributeNumberOfXccs, p->device) != hipSuccess || nxcd < 1)
        nxcd = 1;
    make_local_orders(S, T, nbr, &ht, nxcd);
    p->npieces = nxcd <= kMaxPieces ? nxcd : 0;
    for (int k = 0; k <= p->npieces; ++k) {
        p->fwd_piece_off[k] = ht.fo_off[k];
        p->rev_piece_off[k] = ht.ro_off[k];
    }
    std::vector<int> store_tgt(S, -1);
    for (int t = 0; t < T; ++t) store_tgt[tg[t]] = t;
    const std::vector<int> zeros((size_t)kCounterSlots * kMaxPieces, 0);
    if ((rc = upload(&p->d_fwd_rel, fwd)) || (rc = upload(&p->d_rev_rel, rev)) ||
        (rc = upload(&p->d_tgt, tg)) || (rc = upload(&p->d_store_tgt, store_tgt)) ||
        (rc = upload(&p->d_fwd_order, fo)) ||
        (rc = upload(&p->d_rev_order, ro)) || (rc = upload(&p->d_counters, zeros)) ||
        (rc = upload(&p->d_fwd_local, ht.fo_local)) || (rc = upload(&p->d_rev_local, ht.ro_local)) ||
        (rc = upload(&p->d_fwd_piece, ht.fo_piece)) || (rc = upload(&p->d_rev_piece, ht.ro_piece))) {
        free_plan_memory(p);
        delete p;
        return rc;
    }
    *out = p;
    return OT_FMM_OK;
}

int ot_fmm_plan_destroy(ot_fmm_plan plan)
{
    g_last_error.clear();
    if (!plan) return OT_FMM_OK;
    free_plan_memory(plan);
    delete plan;
    return OT_FMM_OK;
}

int ot_fmm_count_pairs(int32_t S, int32_t T, const int32_t* tgt, const int32_t* nbr, const int8_t* shift,
                       const double* period, int64_t* pairs, int64_t* work, int32_t* order)
{
    g_last_error.clear();
    if (!pairs) return fail(OT_FMM_EINVAL, "null pairs pointer");
    HostTables ht;
    int rc = build_host_tables(S, T, tgt, nbr, shift, period, &ht);
    if (rc) return rc;
    *pairs = ht.pairs;
    if (work) std::copy(ht.fwd_work.begin(), ht.fwd_work.end(), work);
    if (order) std::copy(ht.fo.begin(), ht.fo.end(), order);
    return OT_FMM_OK;
}

int ot_fmm_work_orders(int32_t S, int32_t T, const int32_t* tgt, const int32_t* nbr, const int8_t* shift,
                       const double* period, int32_t nxcd, int32_t* fwd_local, int32_t* rev_lpt,
                       int32_t* rev_local)
{
    g_last_error.clear();
    if (nxcd < 1 || nxcd > 64) return fail(OT_FMM_EINVAL, "nxcd must be in [1, 64]");
    HostTables ht;
    int rc = build_host_tables(S, T, tgt, nbr, shift, period, &ht);
    if (rc) return rc;
    make_local_orders(S, T, nbr, &ht, nxcd);
    if (fwd_local) std::copy(ht.fo_local.begin(), ht.fo_local.end(), fwd_local);
    if (rev_lpt) std::copy(ht.ro.begin(), ht.ro.end(), rev_lpt);
    if (rev_local) std::copy(ht.ro_local.begin(), ht.ro_local.end(), rev_local);
    return OT_FMM_OK;
}

int ot_fmm_stencil_info(int64_t* slot_pairs, int32_t* offsets_per_target, int32_t* rows_per_parity)
{
    g_last_error.clear();
    if (!slot_pairs || !offsets_per_target || !rows_per_parity) return fail(OT_FMM_EINVAL, "null argument");
    const SlotCounts& sc = slot_counts();
    for (int s = 0; s < 27; ++s) slot_pairs[s] = sc.pairs[s];
    for (int pz = 0; pz < 2; ++pz) {
        offsets_per_target[pz] = kStencilHost.count[pz];
        rows_per_parity[pz] = kStencilHost.range[pz][2 * kReach][2];
    }
    if (!sc.mirror_ok) return fail(OT_FMM_EUNSUPPORTED, "stencil mirror check failed");
    return OT_FMM_OK;
}

int ot_fmm_plan_set_coarse(ot_fmm_plan plan, int32_t Sp, const int32_t* coarse, const int8_t* octant,
                           int64_t* pairs)
{
    g_last_error.clear();
    int rc = check_plan(plan);
    if (rc) return rc;
    if (Sp <= 0 || !coarse || !octant) return fail(OT_FMM_EINVAL, "Sp > 0, coarse and octant required");
    if ((int64_t)Sp * kSub3 * 20 > ((int64_t)1 << 40)) return fail(OT_FMM_EINVAL, "coarse store too large");
    const int T = plan->T;
    for (int t = 0; t < T; ++t)
        for (int q = 0; q < 27; ++q) {
            const int32_t c = coarse[(int64_t)t * 27 + q];
            const int o = octant[(int64_t)t * 27 + q];
            if (c < -1 || c >= Sp) return fail(OT_FMM_EINVAL, "coarse node out of range");
            if (c >= 0 && !((plan->missing[t] >> q) & 1u))
                return fail(OT_FMM_EINVAL, "a substitute is given for a neighbour that is present");
            if (c >= 0 && (o < 0 || o > 7)) return fail(OT_FMM_EINVAL, "octant out of range");
        }
    // per slot (geometry only): the coarse cells included for each target
    // cell, as a 64-bit mask, and their number
    std::vector<unsigned long long> mask((size_t)27 * kSub3, 0ull);
    std::vector<int> cnt((size_t)27 * kSub3, 0);
    int64_t slot_pairs[27] = {0};
    for (int q = 0; q < 27; ++q) {
        const int so[3] = {q % 3, (q / 3) % 3, q / 9};
        for (int c = 0; c < kSub3; ++c) {
            const int hi[3] = {8 + c % 8, 8 + (c / 8) % 8, 8 + c / 64};
            for (int J = 0; J < 64; ++J) {
                const int cj[3] = {J & 3, (J >> 2) & 3, J >> 4};
                bool all_in = true;
                for (int n = 0; n < 8 && all_in; ++n)
                    all_in = criterion(hi[0], hi[1], hi[2], 8 * so[0] + 2 * cj[0] + (n & 1),
                                       8 * so[1] + 2 * cj[1] + ((n >> 1) & 1), 8 * so[2] + 2 * cj[2] + (n >> 2));
                if (all_in) {
                    mask[(size_t)q * kSub3 + c] |= 1ull << J;
                    ++cnt[(size_t)q * kSub3 + c];
                }
            }
            slot_pairs[q] += cnt[(size_t)q * kSub3 + c];
        }
    }
    // per pattern of substituted slots: the target cells in lane order, by
    // decreasing total count, and the loop trips of each block of 64 ranks
    // (its first cell's count); work items are the parts of a target
    constexpr int kParts = CoarseShape<kCoarseWaves>::parts;
    std::unordered_map<uint32_t, int> pattern_id;
    std::vector<int> cells;
    std::vector<std::array<int64_t, 8>> pattern_blocks;
    std::vector<int4> items, entries;
    std::vector<int64_t> item_cost;
    int64_t total = 0;
    for (int t = 0; t < T; ++t) {
        uint32_t pat = 0;
        const int first = (int)entries.size();
        for (int q = 0; q < 27; ++q) {
            const int32_t c = coarse[(int64_t)t * 27 + q];
            if (c < 0) continue;
            pat |= 1u << q;
            entries.push_back(make_int4(q, c, octant[(int64_t)t * 27 + q], 0));
            total += slot_pairs[q];
        }
        if (!pat) continue;
        auto f = pattern_id.find(pat);
        int id;
        if (f == pattern_id.end()) {
            id = (int)pattern_blocks.size();
            pattern_id.emplace(pat, id);
            std::vector<int> tot(kSub3, 0), order(kSub3);
            for (int q = 0; q < 27; ++q)
                if ((pat >> q) & 1u)
                    for (int c = 0; c < kSub3; ++c) tot[c] += cnt[(size_t)q * kSub3 + c];
            for (int c = 0; c < kSub3; ++c) order[c] = c;
            std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return tot[x] > tot[y]; });
            cells.insert(cells.end(), order.begin(), order.end());
            std::array<int64_t, 8> blk{};
            for (int w = 0; w < 8; ++w) blk[w] = tot[order[64 * w]];
            pattern_blocks.push_back(blk);
        } else {
            id = f->second;
        }
        const int n = (int)entries.size() - first;
        for (int part = 0; part < kParts; ++part) {
            int64_t cost = 8 * n;  // staging
            for (int w = part; w < 8; w += kParts) cost += pattern_blocks[id][w];
            items.push_back(make_int4(t, id * 8 + part, first, n));
            item_cost.push_back(cost);
        }
    }
    std::vector<int> idx(items.size());
    for (size_t i = 0; i < idx.size(); ++i) idx[i] = (int)i;
    std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return item_cost[x] > item_cost[y]; });
    std::vector<int4> sorted(items.size());
    for (size_t i = 0; i < idx.size(); ++i) sorted[i] = items[idx[i]];
    if (entries.empty()) entries.push_back(make_int4(0, 0, 0, 0));  // keep every table non-empty
    if (sorted.empty()) sorted.push_back(make_int4(0, 0, 0, 0));
    if (cells.empty()) cells.assign(kSub3, 0);
    int4* d_items = nullptr;
    int4* d_entries = nullptr;
    int* d_cells = nullptr;
    unsigned long long* d_mask = nullptr;
    if ((rc = upload(&d_items, sorted)) || (rc = upload(&d_entries, entries)) || (rc = upload(&d_cells, cells)) ||
        (rc = upload(&d_mask, mask))) {
        (void)hipFree(d_items);
        (void)hipFree(d_entries);
        (void)hipFree(d_cells);
        (void)hipFree(d_mask);
        return rc;
    }
    if (plan->d_cf_items) {
        // earlier tables may still be read by a launch in flight
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) {
            (void)hipFree(d_items);
            (void)hipFree(d_entries);
            (void)hipFree(d_cells);
            (void)hipFree(d_mask);
            return hip_fail(e, "hipDeviceSynchronize");
        }
    }
    (void)hipFree(plan->d_cf_items);
    (void)hipFree(plan->d_cf_entries);
    (void)hipFree(plan->d_cf_cells);
    (void)hipFree(plan->d_cf_mask);
    plan->d_cf_items = d_items;
    plan->d_cf_entries = d_entries;
    plan->d_cf_cells = d_cells;
    plan->d_cf_mask = d_mask;
    plan->Sp_coarse = Sp;
    plan->n_coarse_items = (int)items.size();
    if (pairs) *pairs = total;
    return OT_FMM_OK;
}

static int coarse_fine_any(bool full, ot_fmm_plan plan, const double* com, const double* Mp, const double* comp,
                           double* L, void* stream)
{
    g_last_error.clear();
    int rc = check_plan(plan);
    if (rc) return rc;
    if (plan->Sp_coarse <= 0) return fail(OT_FMM_EINVAL, "no coarse substitutes set (ot_fmm_plan_set_coarse)");
    if (!aligned8(com) || !aligned8(Mp) || !aligned8(comp) || !aligned8(L))
        return fail(OT_FMM_EINVAL, "null or misaligned (8-byte) pointer");
    const int64_t NS = (int64_t)plan->S * kSub3, NT = (int64_t)plan->T * kSub3,
                  NP = (int64_t)plan->Sp_coarse * kSub3;
    if (overlap(L, 20 * NT, com, 3 * NS) || overlap(L, 20 * NT, Mp, 20 * NP) || overlap(L, 20 * NT, comp, 3 * NP))
        return fail(OT_FMM_EINVAL, "L overlaps an input");
    if (plan->n_coarse_items == 0) return OT_FMM_OK;
    CoarseParams cp{};
    cp.pos = com;
    cp.pos_stride = NS;
    cp.mom_c = Mp;
    cp.pos_c = comp;
    cp.c_stride = NP;
    cp.items = plan->d_cf_items;
    cp.entries = plan->d_cf_entries;
    cp.rel = plan->d_fwd_rel;
    cp.own_blk = plan->d_tgt;
    cp.lane_cell = plan->d_cf_cells;
    cp.cell_mask = plan->d_cf_mask;
    cp.out = L;
    cp.out_stride = NT;
    for (int k = 0; k < 3; ++k) cp.period[k] = plan->period[k];
    const dim3 grid((unsigned)plan->n_coarse_items), block(kCoarseWaves * 64);
    if (full)
        hipLaunchKernelGGL((k_coarse_fine<kCoarseWaves, true>), grid, block, 0, (hipStream_t)stream, cp);
    else
        hipLaunchKernelGGL((k_coarse_fine<kCoarseWaves, false>), grid, block, 0, (hipStream_t)stream, cp);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? OT_FMM_OK : hip_fail(e, "kernel launch");
}

int ot_fmm_coarse_fine(ot_fmm_plan plan, const double* com, const double* Mp, const double* comp, double* L,
                       void* stream)
{
    return coarse_fine_any(false, plan, com, Mp, comp, L, stream);
}

int ot_fmm_coarse_fine_full(ot_fmm_plan plan, const double* com, const double* Mp, const double* comp, double* L,
                            void* stream)
{
    return coarse_fine_any(true, plan, com, Mp, comp, L, stream);
}

int ot_fmm_plan_pairs(ot_fmm_plan plan, int64_t* pairs)
{
    g_last_error.clear();
    if (!plan || !pairs) return fail(OT_FMM_EINVAL, "null argument");
    *pairs = plan->pairs;
    return OT_FMM_OK;
}

// Extents rule of the forward and adjoint entry points: outputs overlap no
// input and no other output (the adjoint arrays only when given).
static int check_overlaps(ot_fmm_plan plan, const double* M, const double* com, const double* L,
                          const double* gL, const double* gM, const double* gcom)
{
    const int64_t NS = (int64_t)plan->S * kSub3, NT = (int64_t)plan->T * kSub3;
    if (overlap(L, 20 * NT, M, 20 * NS) || overlap(L, 20 * NT, com, 3 * NS))
        return fail(OT_FMM_EINVAL, "L overlaps an input");
    if (!gM) return OT_FMM_OK;
    const double* in[4] = {M, com, gL, L};
    const int64_t nin[4] = {20 * NS, 3 * NS, 20 * NT, 20 * NT};
    for (int i = 0; i < 4; ++i)
        if (overlap(gM, 20 * NS, in[i], nin[i]) || overlap(gcom, 3 * NS, in[i], nin[i]))
            return fail(OT_FMM_EINVAL, "outputs overlap inputs");
    if (overlap(L, 20 * NT, gL, 20 * NT)) return fail(OT_FMM_EINVAL, "L overlaps gL");
    if (overlap(gM, 20 * NS, gcom, 3 * NS)) return fail(OT_FMM_EINVAL, "gM overlaps gcom");
    return OT_FMM_OK;
}

int ot_fmm_multipole_batched(ot_fmm_plan plan, const double* M, const double* com, double* L,
                             int sched, void* stream)
{
    g_last_error.clear();
    int rc = check_plan(plan);
    if (rc) return rc;
    if (!aligned8(M) || !aligned8(com) || !aligned8(L))
        return fail(OT_FMM_EINVAL, "null or misaligned (8-byte) pointer");
    const int64_t NS = (int64_t)plan->S * kSub3, NT = (int64_t)plan->T * kSub3;
    if (overlap(L, 20 * NT, M, 20 * NS) || overlap(L, 20 * NT, com, 3 * NS))
        return fail(OT_FMM_EINVAL, "L overlaps an input");
    if (!valid_fwd_sched(sched)) return fail(OT_FMM_EINVAL, "unknown schedule");
    return fwd_batched(plan, M, com, L, sched, (hipStream_t)stream);
}

int ot_fmm_multipole_batched_full(ot_fmm_plan plan, const double* M, const double* com, double* L,
                                  int sched, void* stream)
{
    g_last_error.clear();
    int rc = check_plan(plan);
    if (rc) return rc;
    if (!aligned8(M) || !aligned8(com) || !aligned8(L))
        return fail(OT_FMM_EINVAL, "null or misaligned (8-byte) pointer");
    const int64_t NS = (int64_t)plan->S * kSub3, NT = (int64_t)plan->T * kSub3;
    if (overlap(L, 20 * NT, M, 20 * NS) || overlap(L, 20 * NT, com, 3 * NS))
        return fail(OT_FMM_EINVAL, "L overlaps an input");
    if (!valid_fwd_sched(sched)) return fail(OT_FMM_EINVAL, "unknown schedule");
    return fwd_full_batched(plan, M, com, L, sched, (hipStream_t)stream);
}

int ot_fmm_multipole_backward(ot_fmm_plan plan, const double* M, const double* com,
                              const double* gL, double* gM, double* gcom, int sched,
                              void* stream)
{
    g_last_error.clear();
    int rc = check_plan(plan);
    if (rc) return rc;
    if (!aligned8(M) || !aligned8(com) || !aligned8(gL) || !aligned8(gM) || !aligned8(gcom))
        return fail(OT_FMM_EINVAL, "null or misaligned (8-byte) pointer");
    {
        const int64_t NS = (int64_t)plan->S * kSub3, NT = (int64_t)plan->T * kSub3;
        const double* in[3] = {M, com, gL};
        const int64_t nin[3] = {20 * NS, 3 * NS, 20 * NT};
        for (int i = 0; i < 3; ++i)
            if (overlap(gM, 20 * NS, in[i], nin[i]) || overlap(gcom, 3 * NS, in[i], nin[i]))
                return fail(OT_FMM_EINVAL, "outputs overlap inputs");
        if (overlap(gM, 20 * NS, gcom, 3 * NS)) return fail(OT_FMM_EINVAL, "gM overlaps gcom");
    }
    if (!valid_bwd_sched(sched)) return fail(OT_FMM_EINVAL, "unknown backward schedule");
    return bwd_batched(plan, M, com, gL, gM, gcom, sched, (hipStream_t)stream);
}

int ot_fmm_multipole_backward_full(ot_fmm_plan plan, const double* M, const double* com,
                                   const double* gL, double* gM, double* gcom, int sched,
                                   void* stream)
{
    g_last_error.clear();
    int rc = check_plan(plan);
    if (rc) return rc;
    if (!aligned8(M) || !aligned8(com) || !aligned8(gL) || !aligned8(gM) || !aligned8(gcom))
        return fail(OT_FMM_EINVAL, "null or misaligned (8-byte) pointer");
    {
        const int64_t NS = (int64_t)plan->S * kSub3, NT = (int64_t)plan->T * kSub3;
        const double* in[3] = {M, com, gL};
        const int64_t nin[3] = {20 * NS, 3 * NS, 20 * NT};
        for (int i = 0; i < 3; ++i)
            if (overlap(gM, 20 * NS, in[i], nin[i]) || overlap(gcom, 3 * NS, in[i], nin[i]))
                return fail(OT_FMM_EINVAL, "outputs overlap inputs");
        if (overlap(gM, 20 * NS, gcom, 3 * NS)) return fail(OT_FMM_EINVAL, "gM overlaps gcom");
    }
    if (!valid_bwd_sched(sched)) return fail(OT_FMM_EINVAL, "unknown backward schedule");
    return bwd_any<true>(plan, M, com, gL, gM, gcom, sched, (hipStream_t)stream);
}

int ot_fmm_multipole_batched_save(ot_fmm_plan plan, const double* M, const double* com, double* L, double* Cs,
                                  int sched, void* stream)
{
    g_last_error.clear();
    int rc = check_plan(plan);
    if (rc) return rc;
    if (!aligned8(M) || !aligned8(com) || !aligned8(L) || !aligned8(Cs))
        return fail(OT_FMM_EINVAL, "null or misaligned (8-byte) pointer");
    const int64_t NS = (int64_t)plan->S * kSub3, NT = (int64_t)plan->T * kSub3;
    if (overlap(L, 20 * NT, M, 20 * NS) || overlap(L, 20 * NT, com, 3 * NS))
        return fail(OT_FMM_EINVAL, "L overlaps an input");
    if (overlap(Cs, 24 * NT, M, 20 * NS) || overlap(Cs, 24 * NT, com, 3 * NS) || overlap(Cs, 24 * NT, L, 20 * NT))
        return fail(OT_FMM_EINVAL, "the saved sums overlap an input or L");
    if (!valid_save_sched(sched)) return fail(OT_FMM_EINVAL, "unknown schedule (W8 or W8P2, with flags)");
    return fwd_save_batched(plan, M, com, L, Cs, sched, (hipStream_t)stream);
}

int ot_fmm_multipole_batched_amc(ot_fmm_plan plan, const double* M, const double* com, double* L, double* dF,
                                 int sched, void* stream)
{
    g_last_error.clear();
    int rc = check_plan(plan);
    if (rc) return rc;
    if (!aligned8(M) || !aligned8(com) || !aligned8(L) || !aligned8(dF))
        return fail(OT_FMM_EINVAL, "null or misaligned (8-byte) pointer");
    const int64_t NS = (int64_t)plan->S * kSub3, NT = (int64_t)plan->T * kSub3;
    if (overlap(L, 20 * NT, M, 20 * NS) || overlap(L, 20 * NT, com, 3 * NS))
        return fail(OT_FMM_EINVAL, "L overlaps an input");
    if (overlap(dF, 3 * NT, M, 20 * NS) || overlap(dF, 3 * NT, com, 3 * NS) || overlap(dF, 3 * NT, L, 20 * NT))
        return fail(OT_FMM_EINVAL, "dF overlaps an input or L");
    if (!valid_save_sched(sched)) return fail(OT_FMM_EINVAL, "unknown schedule (W8 or W8P2, with flags)");
    return fwd_amc_batched(plan, M, com, L, dF, sched, (hipStream_t)stream);
}

// Extents rule of the one-pass adjoint: gM and gcom overlap no input and not
// each other.
static int check_saved_bwd(ot_fmm_plan plan, const double* M, const double* com, const double* gL,
                           const double* Cs, const double* gM, const double* gcom)
{
    if (!aligned8(M) || !aligned8(com) || !aligned8(gL) || !aligned8(Cs) || !aligned8(gM) ||
        !aligned8(gcom))
        return fail(OT_FMM_EINVAL, "null or misaligned (8-byte) pointer");
    const int64_t NS = (int64_t)plan->S * kSub3, NT = (int64_t)plan->T * kSub3;
    const double* in[4] = {M, com, gL, Cs};
    const int64_t nin[4] = {20 * NS, 3 * NS, 20 * NT, 24 * NT};
    for (int i = 0; i < 4; ++i)
        if (overlap(gM, 20 * NS, in[i], nin[i]) || overlap(gcom, 3 * NS, in[i], nin[i]))
            return fail(OT_FMM_EINVAL, "outputs overlap inputs");
    if (overlap(gM, 20 * NS, gcom, 3 * NS)) return fail(OT_FMM_EINVAL, "gM overlaps gcom");
    return OT_FMM_OK;
}

// Extents rule of a whole step with saved sums: the adjoint's rule, and L
// and the sums overlap no other array.
static int check_saved_step(ot_fmm_plan plan, const double* M, const double* com, const double* L,
                            const double* Cs, const double* gL, const double* gM, const double* gcom)
{
    if (!aligned8(L)) return fail(OT_FMM_EINVAL, "null or misaligned (8-byte) pointer");
    int rc = check_saved_bwd(plan, M, com, gL, Cs, gM, gcom);
    if (rc) return rc;
    const int64_t NS = (int64_t)plan->S * kSub3, NT = (int64_t)plan->T * kSub3;
    if (overlap(L, 20 * NT, M, 20 * NS) || overlap(L, 20 * NT, com, 3 * NS) || overlap(Cs, 24 * NT, M, 20 * NS) ||
        overlap(Cs, 24 * NT, com, 3 * NS) || overlap(Cs, 24 * NT, L, 20 * NT) || overlap(L, 20 * NT, gL, 20 * NT) ||
        overlap(Cs, 24 * NT, gL, 20 * NT) || overlap(gM, 20 * NS, L, 20 * NT) || overlap(gcom, 3 * NS, L, 20 * NT))
        return fail(OT_FMM_EINVAL, "arrays overlap");
    return OT_FMM_OK;
}

int ot_fmm_multipole_backward_saved(ot_fmm_plan plan, const double* M, const double* com, const double* gL,
                                    const double* Cs, double* gM, double* gcom, int sched, void* stream)
{
    g_last_error.clear();
    int rc = check_plan(plan);
    if (rc) return rc;
    if ((rc = check_saved_bwd(plan, M, com, gL, Cs, gM, gcom))) return rc;
    if (!valid_save_sched(sched)) return fail(OT_FMM_EINVAL, "unknown schedule (W8 or W8P2, with flags)");
    return bwd_saved_batched(plan, M, com, gL, Cs, gM, gcom, sched, (hipStream_t)stream);
}

int ot_fmm_multipole_batched_full_save(ot_fmm_plan plan, const double* M, const double* com, double* L,
                                       double* Cs, int sched, void* stream)
{
    g_last_error.clear();
    int rc = check_plan(plan);
    if (rc) return rc;
    if (!aligned8(M) || !aligned8(com) || !aligned8(L) || !aligned8(Cs))
        return fail(OT_FMM_EINVAL, "null or misaligned (8-byte) pointer");
    const int64_t NS = (int64_t)plan->S * kSub3, NT = (int64_t)plan->T * kSub3;
    if (overlap(L, 20 * NT, M, 20 * NS) || overlap(L, 20 * NT, com, 3 * NS))
        return fail(OT_FMM_EINVAL, "L overlaps an input");
    if (overlap(Cs, 24 * NT, M, 20 * NS) || overlap(Cs, 24 * NT, com, 3 * NS) || overlap(Cs, 24 * NT, L, 20 * NT))
        return fail(OT_FMM_EINVAL, "the saved sums overlap an input or L");
    if (!valid_save_sched(sched)) return fail(OT_FMM_EINVAL, "unknown schedule (W8 or W8P2, with flags)");
    return fwd_save_batched<true>(plan, M, com, L, Cs, sched, (hipStream_t)stream);
}

int ot_fmm_multipole_backward_full_saved(ot_fmm_plan plan, const double* M, const double* com, const double* gL,
                                         const double* Cs, double* gM, double* gcom, int sched, void* stream)
{
    g_last_error.clear();
    int rc = check_plan(plan);
    if (rc) return rc;
    if ((rc = check_saved_bwd(plan, M, com, gL, Cs, gM, gcom))) return rc;
    if (!valid_save_sched(sched)) return fail(OT_FMM_EINVAL, "unknown schedule (W8 or W8P2, with flags)");
    return bwd_saved_batched<true>(plan, M, com, gL, Cs, gM, gcom, sched, (hipStream_t)stream);
}

int ot_fmm_autotune_saved(ot_fmm_plan plan, const double* M, const double* com, double* L, double* Cs,
                          const double* gL, double* gM, double* gcom, void* stream, int* fwd_sched,
                          int* bwd_sched)
{
    g_last_error.clear();
    int rc = check_plan(plan);
    if (rc) return rc;
    if ((rc = check_saved_step(plan, M, com, L, Cs, gL, gM, gcom))) return rc;
    hipStream_t s = (hipStream_t)stream;
    struct Events {
        hipEvent_t a = nullptr, b = nullptr;
        ~Events()
        {
            if (a) (void)hipEventDestroy(a);
            if (b) (void)hipEventDestroy(b);
        }
    } ev;
    OT_HIP(hipEventCreate(&ev.a));
    OT_HIP(hipEventCreate(&ev.b));
    auto time_it = [&](auto&& fn, float* ms) -> int {
        int r = fn();  // warm-up
        if (r) return r;
        OT_HIP(hipEventRecord(ev.a, s));
        for (int i = 0; i < 3; ++i)
            if ((r = fn())) return r;
        OT_HIP(hipEventRecord(ev.b, s));
        OT_HIP(hipEventSynchronize(ev.b));
        OT_HIP(hipEventElapsedTime(ms, ev.a, ev.b));
        return OT_FMM_OK;
    };
    const int kFlags[4] = {0, OT_FMM_SCHED_PERSISTENT, OT_FMM_SCHED_LOCAL,
                           OT_FMM_SCHED_PERSISTENT | OT_FMM_SCHED_LOCAL};
    int best_f = kSaveSched, best_b = kSaveSched;
    float best_fms = 3.0e38f, best_bms = 3.0e38f;
    for (int shape : {OT_FMM_SCHED_W8, OT_FMM_SCHED_W8P2})
        for (int f : kFlags) {
            const int cand = shape | f;
            float ms = 0.0f;
            if (!rc) rc = time_it([&] { return fwd_save_batched(plan, M, com, L, Cs, cand, s); }, &ms);
            if (!rc && ms < best_fms) {
                best_fms = ms;
                best_f = cand;
            }
        }
    // the adjoint is timed on the sums of the last forward (any schedule's
    // sums are valid)
    for (int shape : {OT_FMM_SCHED_W8, OT_FMM_SCHED_W8P2})
        for (int f : kFlags) {
            const int cand = shape | f;
            float ms = 0.0f;
            if (!rc) rc = time_it([&] { return bwd_saved_batched(plan, M, com, gL, Cs, gM, gcom, cand, s); }, &ms);
            if (!rc && ms < best_bms) {
                best_bms = ms;
                best_b = cand;
            }
        }
    // leave the results of the chosen schedules in the buffers
    if (!rc) rc = fwd_save_batched(plan, M, com, L, Cs, best_f, s);
    if (!rc) rc = bwd_saved_batched(plan, M, com, gL, Cs, gM, gcom, best_b, s);
    if (!rc) OT_HIP(hipStreamSynchronize(s));
    if (rc) return rc;
    plan->tuned_save = best_f;
    plan->tuned_saved_bwd = best_b;
    if (fwd_sched) *fwd_sched = best_f;
    if (bwd_sched) *bwd_sched = best_b;
    return OT_FMM_OK;
}

int ot_fmm_step_graph_create_saved(ot_fmm_plan plan, const double* M, const double* com, double* L, double* Cs,
                                   const double* gL, double* gM, double* gcom, int fwd_sched, int bwd_sched)
{
    g_last_error.clear();
    int rc = check_plan(plan);
    if (rc) return rc;
    if ((rc = check_saved_step(plan, M, com, L, Cs, gL, gM, gcom))) return rc;
    if (!valid_save_sched(fwd_sched) || !valid_save_sched(bwd_sched))
        return fail(OT_FMM_EINVAL, "unknown schedule (W8 or W8P2, with flags)");
    return capture_step_graph(plan, [&](hipStream_t cs) {
        int r = fwd_save_batched(plan, M, com, L, Cs, fwd_sched, cs);
        if (!r) r = bwd_saved_batched(plan, M, com, gL, Cs, gM, gcom, bwd_sched, cs);
        return r;
    });
}

int ot_fmm_autotune(ot_fmm_plan plan, const double* M, const double* com, double* L,
                    const double* gL, double* gM, double* gcom, void* stream, int* fwd_sched,
                    int* bwd_sched)
{
    g_last_error.clear();
    int rc = check_plan(plan);
    if (rc) return rc;
    if (!aligned8(M) || !aligned8(com) || !aligned8(L))
        return fail(OT_FMM_EINVAL, "null or misaligned (8-byte) pointer");
    const bool with_bwd = gL || gM || gcom;
    if (with_bwd && (!aligned8(gL) || !aligned8(gM) || !aligned8(gcom)))
        return fail(OT_FMM_EINVAL, "null or misaligned backward pointer");
    if ((rc = check_overlaps(plan, M, com, L, gL, with_bwd ? gM : nullptr, gcom))) return rc;
    hipStream_t s = (hipStream_t)stream;
    // the two timing events, destroyed on every return path
    struct Events {
        hipEvent_t a = nullptr, b = nullptr;
        ~Events()
        {
            if (a) (void)hipEventDestroy(a);
            if (b) (void)hipEventDestroy(b);
        }
    } ev;
    OT_HIP(hipEventCreate(&ev.a));
    OT_HIP(hipEventCreate(&ev.b));
    hipEvent_t e0 = ev.a, e1 = ev.b;
    auto time_it = [&](auto&& fn, float* ms) -> int {
        int r = fn();  // warm-up
        if (r) return r;
        OT_HIP(hipEventRecord(e0, s));
        for (int i = 0; i < 3; ++i)
            if ((r = fn())) return r;
        OT_HIP(hipEventRecord(e1, s));
        OT_HIP(hipEventSynchronize(e1));
        OT_HIP(hipEventElapsedTime(ms, e0, e1));
        return OT_FMM_OK;
    };
    // every shape with every combination of the persistent launch and the
    // XCD-aware order, for each pass on its own: the forward, then the
    // source-role pass, then the target-role pass
    const int kFlags[4] = {0, OT_FMM_SCHED_PERSISTENT, OT_FMM_SCHED_LOCAL,
                           OT_FMM_SCHED_PERSISTENT | OT_FMM_SCHED_LOCAL};
    int best_f = OT_FMM_SCHED_W16;
    float best_ms = 3.0e38f;
    auto try_fwd = [&](int cand) -> int {
        float ms = 0.0f;
        int r = time_it([&] { return fwd_batched(plan, M, com, L, cand, s); }, &ms);
        if (!r && ms < best_ms) {
            best_ms = ms;
            best_f = cand;
        }
        return r;
    };
    for (int shape : {OT_FMM_SCHED_W8, OT_FMM_SCHED_W16, OT_FMM_SCHED_W8P2})
        for (int f : kFlags)
            if (!rc) rc = try_fwd(shape | f);
    int best_b = OT_FMM_SCHED_W16 | (kDefaultSourceSched << 8);
    if (!rc && with_bwd) {
        // source role (bits 8..15), timed alone; then the target role
        int best_s = kDefaultSourceSched, best_t = OT_FMM_SCHED_W16;
        auto try_pass = [&](int passes, int sc, int* best) -> int {
            float ms = 0.0f;
            const int full = passes == 1 ? (OT_FMM_SCHED_W16 | (sc << 8)) : (sc | (best_s << 8));
            int r = time_it([&] { return bwd_any<false>(plan, M, com, gL, gM, gcom, full, s, passes); }, &ms);
            if (!r && ms < best_ms) {
                best_ms = ms;
                *best = sc;
            }
            return r;
        };
        best_ms = 3.0e38f;
        for (int shape : {OT_FMM_SCHED_W8, OT_FMM_SCHED_W8P2})
            for (int f : kFlags)
                if (!rc) rc = try_pass(1, shape | f, &best_s);
        best_ms = 3.0e38f;
        for (int shape : {OT_FMM_SCHED_W8, OT_FMM_SCHED_W16, OT_FMM_SCHED_W8P2})
            for (int f : kFlags)
                if (!rc) rc = try_pass(2, shape | f, &best_t);
        best_b = best_t | (best_s << 8);
        // the target-role trials accumulated into gcom: leave valid results
        if (!rc) rc = bwd_batched(plan, M, com, gL, gM, gcom, best_b, s);
        if (!rc) OT_HIP(hipStreamSynchronize(s));
    }
    if (rc) return rc;
    plan->tuned_fwd = best_f;
    plan->tuned_bwd = best_b;
    if (fwd_sched) *fwd_sched = best_f;
    if (bwd_sched) *bwd_sched = best_b;
    return OT_FMM_OK;
}

int ot_fmm_step_graph_create(ot_fmm_plan plan, const double* M, const double* com, double* L,
                             const double* gL, double* gM, double* gcom, int fwd_sched,
                             int bwd_sched)
{
    g_last_error.clear();
    int rc = check_plan(plan);
    if (rc) return rc;
    if (!aligned8(M) || !aligned8(com) || !aligned8(L))
        return fail(OT_FMM_EINVAL, "null or misaligned (8-byte) pointer");
    const bool with_bwd = gL || gM || gcom;
    if (with_bwd && (!aligned8(gL) || !aligned8(gM) || !aligned8(gcom)))
        return fail(OT_FMM_EINVAL, "null or misaligned backward pointer");
    if (!valid_fwd_sched(fwd_sched)) return fail(OT_FMM_EINVAL, "unknown schedule");
    if (with_bwd && !valid_bwd_sched(bwd_sched))
        return fail(OT_FMM_EINVAL, "unknown backward schedule");
    if ((rc = check_overlaps(plan, M, com, L, gL, with_bwd ? gM : nullptr, gcom))) return rc;
    return capture_step_graph(plan, [&](hipStream_t cs) {
        int r = fwd_batched(plan, M, com, L, fwd_sched, cs);
        if (!r && with_bwd) r = bwd_batched(plan, M, com, gL, gM, gcom, bwd_sched, cs);
        return r;
    });
}

int ot_fmm_step_graph_launch(ot_fmm_plan plan, void* stream)
{
    g_last_error.clear();
    int rc = check_plan(plan);
    if (rc) return rc;
    if (!plan->graph_exec) return fail(OT_FMM_EINVAL, "no step graph captured");
    OT_HIP(hipGraphLaunch(plan->graph_exec, (hipStream_t)stream));
    return OT_FMM_OK;
}

int ot_fmm_plan_timing(ot_fmm_plan plan, int enable)
{
    g_last_error.clear();
    int rc = check_plan(plan);
    if (rc) return rc;
    plan->timing = enable != 0;
    return OT_FMM_OK;
}

int ot_fmm_plan_kernel_times(ot_fmm_plan plan, double ms_total[OT_FMM_NKERNELS], int64_t launches[OT_FMM_NKERNELS])
{
    g_last_error.clear();
    int rc = check_plan(plan);
    if (rc) return rc;
    if (!ms_total || !launches) return fail(OT_FMM_EINVAL, "null output");
    for (int w = 0; w < kTimedKernels; ++w) {
        double tot = 0.0;
        for (size_t i = 0; i < plan->ev_used[w]; ++i) {
            const auto& ev = plan->ev_pool[w][i];
            OT_HIP(hipEventSynchronize(ev.second));
            float ms = 0.0f;
            OT_HIP(hipEventElapsedTime(&ms, ev.first, ev.second));
            tot += ms;
        }
        ms_total[w] = tot;
        launches[w] = (int64_t)plan->ev_used[w];
        plan->ev_used[w] = 0;
    }
    return OT_FMM_OK;
}

}  // extern "C"

// ===========================================================================
// Allocation-free batched forward (ot_fmm_multipole_batched_noalloc)
// ===========================================================================
namespace {

constexpr int kNoAllocMaxT = OT_FMM_NOALLOC_MAX_T;
constexpr int kNoAllocDevices = 64;
// Layout of `scratch`, in int4 units: [0, kScrHead) the header -- ints
// 0..15 the work counters of the persistent launch, int 16 the number of
// invalid descriptor entries, int 17 the first of them; then the targets'
// own store blocks (kNoAllocMaxT ints); then the relation table [T][27].
constexpr long kScrHead = 16;
constexpr long kScrOwn = kNoAllocMaxT / 4;
constexpr long kScrInt4 = kScrHead + kScrOwn + 27L * kNoAllocMaxT;
static_assert(kMaxPieces <= 16, "counters fit the header");

// The scratch memory of the allocation-free entry point: one copy per device,
// held until the process ends. Host code passes the address that
// hipGetSymbolAddress returns for it, never this name.
static __device__ __align__(256) int4 scratch[kScrInt4];

std::mutex g_scratch_mutex;
int4* g_scratch_ptr[kNoAllocDevices];  // per device, set once
int g_scratch_ncu[kNoAllocDevices];

// This device's copy of `scratch` and its CU count, looked up on the first
// call on the device (with the device current) and kept.
int scratch_of_current_device(int4** base, int* ncu)
{
    int dev = 0;
    OT_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNoAllocDevices) return fail(OT_FMM_EUNSUPPORTED, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        OT_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr || (reinterpret_cast<uintptr_t>(ptr) & 255u))
            return fail(OT_FMM_EHIP, "scratch array address not 256-byte aligned");
        int n = 0;
        OT_HIP(hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev));
        g_scratch_ncu[dev] = n > 0 ? n : 1;
        g_scratch_ptr[dev] = static_cast<int4*>(ptr);
    }
    *base = g_scratch_ptr[dev];
    *ncu = g_scratch_ncu[dev];
    return OT_FMM_OK;
}

// Clears the header: the work counters and the invalid-entry count start at
// zero, the first invalid entry at INT_MAX (a kernel, so that graph captures
// hold no memset node).
__global__ void k_noalloc_reset(int* head)
{
    const int t = threadIdx.x;
    if (t < 16) head[t] = 0;
    if (t == 16) head[16] = 0;
    if (t == 17) head[17] = 0x7fffffff;
}

// Relation table of the call from the caller's device descriptor, checked
// entry by entry: an entry out of range is dropped (stored as missing, its
// target's own block as 0) and counted.
__global__ void __launch_bounds__(256) k_noalloc_relations(int S, int T, const int* __restrict__ tgt,
                                                           const int* __restrict__ nbr,
                                                           const int8_t* __restrict__ shift, int* own,
                                                           int4* rel, int* status)
{
    const int i = (int)blockIdx.x * 256 + (int)threadIdx.x;
    if (i >= T * 27) return;
    const int t = i / 27, s = i - 27 * t;
    const int ob = tgt[t];
    const bool own_ok = ob >= 0 && ob < S;
    int b = nbr[i];
    const bool ok = own_ok && b >= -1 && b < S && (s != 13 || b == ob);
    int packed = 0;
    if (shift)
        for (int k = 0; k < 3; ++k) packed |= ((int)shift[3 * i + k] & 0xff) << (8 * k);
    if (!ok) {
        atomicAdd(status, 1);
        atomicMin(status + 1, i);
        b = -1;
    }
    rel[i] = make_int4(b, b, packed, 0);
    if (s == 13) own[t] = own_ok ? ob : 0;
}

// After a call with invalid entries every element of L becomes NaN.
__global__ void __launch_bounds__(256) k_noalloc_poison(const int* status, double* L, long n)
{
    if (status[0] == 0) return;
    const double nan = __builtin_nan("");
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) L[i] = nan;
}

// Do the byte ranges [a, a + na) and [b, b + nb) share memory?
bool overlap_bytes(const void* a, size_t na, const void* b, size_t nb)
{
    const uintptr_t a0 = reinterpret_cast<uintptr_t>(a), b0 = reinterpret_cast<uintptr_t>(b);
    return a && b && a0 < b0 + nb && b0 < a0 + na;
}

}  // namespace

extern "C" {

int ot_fmm_multipole_batched_noalloc(int32_t S, int32_t T, const int32_t* tgt, const int32_t* nbr,
                                     const int8_t* shift, const double* period, const double* M,
                                     const double* com, double* L, void* stream)
{
    g_last_error.clear();
    if (S <= 0 || T <= 0) return fail(OT_FMM_EINVAL, "S and T must be positive");
    if (T > kNoAllocMaxT)
        return fail(OT_FMM_EINVAL, "T exceeds the 32768 targets of the allocation-free scratch array "
                                   "(use a plan: ot_fmm_plan_create)");
    if ((int64_t)S * kSub3 * 20 > ((int64_t)1 << 40)) return fail(OT_FMM_EINVAL, "store too large");
    if (!tgt || !nbr || (reinterpret_cast<uintptr_t>(tgt) & 3u) || (reinterpret_cast<uintptr_t>(nbr) & 3u))
        return fail(OT_FMM_EINVAL, "null or misaligned (4-byte) tgt or nbr");
    if (shift && !period) return fail(OT_FMM_EINVAL, "shift given without period");
    double per[3] = {0.0, 0.0, 0.0};
    if (period)
        for (int k = 0; k < 3; ++k) {
            if (!(period[k] == period[k]) || period[k] > 1e15 || period[k] < -1e15)
                return fail(OT_FMM_EINVAL, "period must be finite");
            per[k] = period[k];
        }
    if (!aligned8(M) || !aligned8(com) || !aligned8(L))
        return fail(OT_FMM_EINVAL, "null or misaligned (8-byte) pointer");
    const int64_t NS = (int64_t)S * kSub3, NT = (int64_t)T * kSub3;
    if (overlap(L, 20 * NT, M, 20 * NS) || overlap(L, 20 * NT, com, 3 * NS))
        return fail(OT_FMM_EINVAL, "L overlaps an input");
    const size_t nL = (size_t)(20 * NT) * sizeof(double);
    if (overlap_bytes(L, nL, tgt, (size_t)T * 4) || overlap_bytes(L, nL, nbr, (size_t)T * 27 * 4) ||
        overlap_bytes(L, nL, shift, (size_t)T * 27 * 3))
        return fail(OT_FMM_EINVAL, "L overlaps the descriptor");
    int rc = ensure_device();
    if (rc) return rc;
    int4* base = nullptr;
    int ncu = 1;
    if ((rc = scratch_of_current_device(&base, &ncu))) return rc;
    int* head = reinterpret_cast<int*>(base);
    int* own = reinterpret_cast<int*>(base + kScrHead);
    int4* rel = base + kScrHead + kScrOwn;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_noalloc_reset, dim3(1), dim3(64), 0, s, head);
    hipLaunchKernelGGL(k_noalloc_relations, dim3((unsigned)((T * 27 + 255) / 256)), dim3(256), 0, s, (int)S,
                       (int)T, tgt, nbr, shift, own, rel, head + 16);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    // the forward of ot_fmm_multipole_batched with W16 | PERSISTENT, work
    // entries in target order from the scratch counter
    KParams kp{};
    kp.mom = M;
    kp.pos = com;
    kp.mom_stride = NS;
    kp.pos_stride = NS;
    kp.rel = rel;
    kp.own_blk = own;
    kp.order = nullptr;
    kp.out0 = L;
    kp.out_stride = NT;
    kp.out_blk = nullptr;
    for (int k = 0; k < 3; ++k) kp.period[k] = per[k];
    kp.counter = head;
    kp.n_items = T;
    kp.npieces = 0;
    const long resident = (long)ncu * resident_per_cu<MODE_FWD_STORE, 16, 1>();
    const int nblocks = (int)std::min<long>(T, resident);
    if ((rc = launch<MODE_FWD_STORE, 16, false, 1, true>(kp, nblocks, s))) return rc;
    hipLaunchKernelGGL(k_noalloc_poison, dim3(1024), dim3(256), 0, s, head + 16, L, (long)(20 * NT));
    e = hipGetLastError();
    return e == hipSuccess ? OT_FMM_OK : hip_fail(e, "kernel launch");
}

int ot_fmm_noalloc_status(int32_t* invalid, int32_t* first_invalid)
{
    g_last_error.clear();
    if (!invalid || !first_invalid) return fail(OT_FMM_EINVAL, "null argument");
    int rc = ensure_device();
    if (rc) return rc;
    int4* base = nullptr;
    int ncu = 1;
    if ((rc = scratch_of_current_device(&base, &ncu))) return rc;
    OT_HIP(hipDeviceSynchronize());
    int st[2] = {0, 0};
    OT_HIP(hipMemcpy(st, reinterpret_cast<int*>(base) + 16, sizeof(st), hipMemcpyDeviceToHost));
    *invalid = st[0];
    *first_invalid = st[1];
    return OT_FMM_OK;
}

}  // extern "C"
