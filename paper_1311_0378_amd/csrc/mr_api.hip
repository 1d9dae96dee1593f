// mr_api.hip -- host side of libmrecon: argument checks, workspace layout and
// the launch sequence behind the C ABI declared in include/mr.h.
#include <algorithm>
#include <cstdlib>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "mr_internal.h"

using namespace mr;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(MR_EHIP, "%s: %s", what, hipGetErrorString(e));
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

uint64_t next_pow2(uint64_t v) {
    uint64_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

// The watchdog of the queue phase and the tile queue: microseconds without
// any new ring entry after which a waiting wave gives up (on a working device
// entries come every few microseconds until the queue drains).
constexpr unsigned long long QUEUE_WAIT_US = 2000000ull;



// Where everything lives inside a workspace.
struct Layout {
    int64_t n_tiles = 0;
    uint64_t ring_cap = 0;
    size_t off_desc = 0, off_flags = 0, off_lists = 0, off_qflag = 0, off_bitmap = 0, off_ring = 0, off_plane = 0, total = 0;
    int64_t plane_pitch = 0;
    size_t off_wide = 0; // the queue phase's widened uint8 planes, last (0 bytes when absent)
};

Layout layout_for(int64_t n_tiles, int64_t fill_plane_bytes, int64_t plane_pitch,
                  int64_t n_imgs = 1, size_t wide_bytes = 0) {
    Layout L;
    L.n_tiles = n_tiles;
    L.ring_cap = next_pow2((uint64_t)n_tiles + (uint64_t)RING_SLACK);
    size_t o = align_up(sizeof(Ctrl), 256);
    L.off_desc = o;
    o = align_up(o + sizeof(ImgDesc) * (size_t)n_imgs, 256);
    L.off_flags = o;
    o = align_up(o + (size_t)n_tiles * 4, 256);
    L.off_lists = o;
    o = align_up(o + (size_t)n_tiles * 8, 256);
    L.off_qflag = o;
    o = align_up(o + (size_t)n_tiles * 4, 256);
    L.off_bitmap = o;
    o = align_up(o + (size_t)n_tiles * TS * 8, 256);
    L.off_ring = o;
    o = align_up(o + (size_t)L.ring_cap * 4, 256);
    L.off_plane = o;
    o = align_up(o + (size_t)fill_plane_bytes, 256);
    L.off_wide = o;
    o = align_up(o + wide_bytes, 256);
    L.total = o;
    L.plane_pitch = plane_pitch;
    return L;
}

int64_t tiles_across(int64_t n) { return (n + TI - 1) / TI; }

// uint8 planes whose base and pitch are multiples of 16 bytes: the tile
// loads then move whole aligned 16-byte words (and the rounds may prefetch)
bool staged_planes(int t, const ImgDesc &d) {
    const auto a16 = [](const void *p) { return ((uintptr_t)p & 15) == 0; };
    return t == MR_U8 && a16(d.J) && a16(d.I) && d.pJ % 16 == 0 && d.pI % 16 == 0;
}

bool valid_dtype(int t) { return t == MR_U8 || t == MR_I32; }

int check_tune(const mr_tune *tn) {
    if (!tn) return MR_OK;
    if (tn->sweep_rounds == 0 || tn->sweep_rounds > MAX_ROUNDS)
        return fail(MR_EINVAL, "tune.sweep_rounds must be in 1..%d, or negative", MAX_ROUNDS);
    if (tn->max_sweeps < 1 || tn->max_sweeps > 1024)
        return fail(MR_EINVAL, "tune.max_sweeps must be in 1..1024 (got %d)", tn->max_sweeps);
    if (tn->persistent_blocks < 0)
        return fail(MR_EINVAL, "tune.persistent_blocks must be >= 0");
    if (tn->converge_rounds < 0 || tn->converge_rounds > MAX_ROUNDS)
        return fail(MR_EINVAL, "tune.converge_rounds must be in 0..%d", MAX_ROUNDS);
    if (tn->tail_rounds < 0 || tn->tail_rounds > MAX_ROUNDS)
        return fail(MR_EINVAL, "tune.tail_rounds must be in 0..%d", MAX_ROUNDS);
    if (tn->first_sweeps < 1 || tn->first_sweeps > 1024)
        return fail(MR_EINVAL, "tune.first_sweeps must be in 1..1024 (got %d)", tn->first_sweeps);
    return MR_OK;
}

int check_image(int op, int64_t H, int64_t W, int64_t pitch, int t, int conn) {
    if (op != MR_OP_RECON && op != MR_OP_FILL) return fail(MR_EINVAL, "unknown op %d", op);
    if (H < 1 || W < 1) return fail(MR_EINVAL, "H and W must be >= 1 (got %lld x %lld)",
                                    (long long)H, (long long)W);
    if (pitch != 0 && pitch < W)
        return fail(MR_EINVAL, "pitch %lld is smaller than W %lld", (long long)pitch,
                    (long long)W);
    if (!valid_dtype(t)) return fail(MR_EINVAL, "unknown pixel type %d", t);
    if (conn != 4 && conn != 8) return fail(MR_EINVAL, "conn must be 4 or 8 (got %d)", conn);
    const int64_t nt = tiles_across(H) * tiles_across(W);
    if (nt >= (1ll << 31) - 1) return fail(MR_EINVAL, "image too large (%lld tiles)", (long long)nt);
    // kernels address a plane with 32-bit element offsets
    const int64_t p = pitch ? pitch : W;
    const int64_t pp = (W + 63) / 64 * 64;
    if (H * std::max(p, pp) + 4 >= (1ll << 32))
        return fail(MR_EINVAL, "image plane too large: H * pitch must stay below 2^32 elements");
    return MR_OK;
}

// A schedule whose queue phase follows one or two tile rounds on uint8
// pixels asks for widened planes (one 32-bit key per pixel); a call uses them
// when its workspace holds them, else the queue raises pixels with a
// compare-and-swap on their dword. The planes cost a copy of every tile each
// way, which pays only while the queue does most of the raising: after four
// rounds the compare-and-swap measured faster.
bool wants_wide(int t, const mr_tune *tune) {
    return t == MR_U8 && tune && tune->sweep_rounds > 0 && tune->sweep_rounds <= 2;
}

size_t wide_plane_bytes(int64_t H, int64_t W) { return align_up((size_t)H * (size_t)W * 4, 256); }

Layout single_layout(int op, int64_t H, int64_t W, int t, bool wide = false) {
    const int64_t nt = tiles_across(H) * tiles_across(W);
    int64_t plane = 0, pp = 0;
    if (op == MR_OP_FILL) {
        pp = (int64_t)align_up((size_t)W, 64);
        plane = H * pp * t;
    }
    return layout_for(nt, plane, pp, 1, wide ? wide_plane_bytes(H, W) : 0);
}

mr_tune effective_tune(const mr_tune *tn) {
    mr_tune d;
    mr_default_tune(&d);
    return tn ? *tn : d;
}

// Per-launch timing records of the calling thread (mr_timing_enable).
struct TimedLaunch {
    int32_t kind, round, launches;
    hipEvent_t a, b;
};
struct Timing {
    int on = MR_TIMING_OFF;
    std::vector<TimedLaunch> recs;
    std::vector<hipEvent_t> pool;
    // (thread exit: nobody is left to report a failed destroy to)
    ~Timing() {
        for (auto &r : recs) {
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        for (auto e : pool) (void)hipEventDestroy(e);
    }
    hipEvent_t get() {
        hipEvent_t e = nullptr;
        if (!pool.empty()) {
            e = pool.back();
            pool.pop_back();
        } else if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) {
            e = nullptr;
        }
        return e;
    }
};
thread_local Timing g_timing;

// Brackets one launch with events when timing is on. The events are created
// without the system-scope fence, so recording them writes back and
// invalidates no caches between the launches they time.
struct LaunchTimer {
    hipStream_t s;
    int32_t kind, round;
    hipEvent_t a = nullptr;
    LaunchTimer(hipStream_t s_, int32_t kind_, int32_t round_) : s(s_), kind(kind_), round(round_) {
        // in span mode the tile rounds are timed by a RoundSpan instead
        const bool on = g_timing.on == MR_TIMING_LAUNCHES ||
                        (g_timing.on == MR_TIMING_SPANS && kind != MR_K_TILE_ROUND);
        if (on && (a = g_timing.get()) && hipEventRecord(a, s) != hipSuccess) {
            g_timing.pool.push_back(a);
            a = nullptr;
        }
    }
    ~LaunchTimer() {
        if (!a) return;
        hipEvent_t b = g_timing.get();
        if (!b || hipEventRecord(b, s) != hipSuccess) {
            g_timing.pool.push_back(a);
            if (b) g_timing.pool.push_back(b);
            return;
        }
        g_timing.recs.push_back({kind, round, 1, a, b});
    }
};

// Span mode: one pair of events around consecutive tile rounds. begin()
// before a round's launch (opens a span if none is open), add() after it,
// close() before anything else goes on the stream or the host waits.
struct RoundSpan {
    hipStream_t s;
    hipEvent_t a = nullptr;
    int32_t first = 0, n = 0;
    explicit RoundSpan(hipStream_t s_) : s(s_) {}
    void begin(uint32_t round) {
        if (g_timing.on != MR_TIMING_SPANS || a) return;
        if ((a = g_timing.get()) && hipEventRecord(a, s) != hipSuccess) {
            g_timing.pool.push_back(a);
            a = nullptr;
        }
        first = (int32_t)round;
        n = 0;
    }
    void add() {
        if (a) ++n;
    }
    void close() {
        if (!a) return;
        hipEvent_t b = g_timing.get();
        if (!b || n == 0 || hipEventRecord(b, s) != hipSuccess) {
            g_timing.pool.push_back(a);
            if (b) g_timing.pool.push_back(b);
        } else {
            g_timing.recs.push_back({MR_K_TILE_ROUND, first, n, a, b});
        }
        a = nullptr;
    }
    ~RoundSpan() { close(); }
};

// Pinned words and events the converge mode polls through: two slots of one
// round's band counts, so that one slot is read while the other's copy is in
// flight. A call that stops polling may leave its last copy (of a batch
// enqueued ahead) in flight when it returns; a later call on this thread,
// perhaps on another stream, must not reuse that slot before the copy has
// landed, or the stale count could overwrite the new one. So each call takes
// a set whose recorded events have all completed, and makes a new set only
// when every set is still busy (calls in flight on several streams at once).
struct PollSet {
    uint32_t *words = nullptr;              // [2][NBANDS], pinned
    hipEvent_t ev[2] = {nullptr, nullptr};  // slot copy complete
    bool recorded[2] = {false, false};
};
struct PollSets {
    std::vector<PollSet> sets;
    // (thread exit: nobody is left to report a failed free to)
    ~PollSets() {
        for (auto &p : sets) {
            for (auto e : p.ev)
                if (e) (void)hipEventDestroy(e);
            if (p.words) (void)hipHostFree(p.words);
        }
    }
};
thread_local PollSets g_polls;

PollSet *idle_poll_set() {
    for (auto &p : g_polls.sets) {
        bool busy = false;
        for (int i = 0; i < 2; ++i)
            if (p.recorded[i] && hipEventQuery(p.ev[i]) == hipErrorNotReady) busy = true;
        if (!busy) {
            p.recorded[0] = p.recorded[1] = false;
            return &p;
        }
    }
    PollSet p;
    if (hipHostMalloc((void **)&p.words, sizeof(uint32_t) * 2 * NBANDS, hipHostMallocDefault) !=
        hipSuccess)
        return nullptr;
    for (int i = 0; i < 2; ++i)
        if (hipEventCreateWithFlags(&p.ev[i], hipEventDisableTiming) != hipSuccess) {
            for (auto e : p.ev)
                if (e) (void)hipEventDestroy(e);
            (void)hipHostFree(p.words);
            return nullptr;
        }
    g_polls.sets.push_back(p);
    return &g_polls.sets.back();
}

uint64_t round_total(const Ctrl &h, size_t r) {
    uint64_t n = 0;
    for (int b = 0; b < NBANDS; ++b) n += h.round_tiles[r][b];
    return n;
}

// The whole propagation over the images of one launch.
int run_sequence(int tbytes, int conn, const Imgs &imgs, const Layout &L, void *ws,
                 const mr_tune &tn, hipStream_t s, bool any_fill, int op_all) {
    char *base = (char *)ws;
    Ctrl *ctrl = (Ctrl *)base;
    uint32_t *flags = (uint32_t *)(base + L.off_flags);
    uint32_t *lists = (uint32_t *)(base + L.off_lists);
    uint32_t *qflag = (uint32_t *)(base + L.off_qflag);
    uint64_t *bitmap = (uint64_t *)(base + L.off_bitmap);
    uint32_t *ring = (uint32_t *)(base + L.off_ring);
    const int grid = persistent_grid(); // two 64-thread blocks per SIMD
    hipError_t e;

    // control block, dirty flags, and the queue flags and ring (untouched by
    // the rounds, so the tile queue can start from them as they are)
    if ((e = launch_clear_start(ctrl, L.n_tiles, flags, qflag, ring, (int64_t)L.ring_cap, s)) !=
        hipSuccess)
        return hip_fail(e, "clear");

    uint32_t round = 1;
    RoundSpan span(s); // span-mode timing of consecutive rounds
    span.begin(round);
    {
        // The first round's visits have their own sweep cap: their halos
        // are mostly stale (the neighbours have not been visited yet), and
        // nearly every tile is visited again in the second tile round.
        LaunchTimer lt(s, MR_K_TILE_ROUND, (int32_t)round);
        e = launch_tile_round(tbytes, conn, imgs, L.n_tiles, flags, lists, ctrl, round,
                              tn.first_sweeps, grid, s, op_all);
    }
    if (e != hipSuccess) return hip_fail(e, "tile round");
    span.add();
    // Seed pass and queue phase over the tiles listed for round `seed_round`
    // (the round after the last one run).
    auto queue_phase = [&](uint32_t seed_round) -> int {
        span.close();
        if ((e = launch_clear_u32(qflag, L.n_tiles, 0u, s)) != hipSuccess ||
            (e = launch_clear_u64(bitmap, L.n_tiles * TS, s)) != hipSuccess ||
            (e = launch_clear_u32(ring, (int64_t)L.ring_cap, Q_EMPTY, s)) != hipSuccess)
            return hip_fail(e, "clear");
        {
            LaunchTimer lt(s, MR_K_SEED, 0);
            e = launch_seed(tbytes, conn, imgs, L.n_tiles, lists, seed_round, ctrl, bitmap, qflag,
                            ring, L.ring_cap, grid, s);
        }
        if (e != hipSuccess) return hip_fail(e, "seed");
        int blocks = tn.persistent_blocks;
        const int maxb = queue_max_blocks(tbytes, conn);
        if (maxb <= 0) return fail(MR_EHIP, "cannot size the queue launch");
        if (blocks == 0 || blocks > maxb) blocks = maxb;
        // uint8 images with widened planes: the queue works on 32-bit keys
        if (imgs.wide && (e = launch_widen(imgs, L.n_tiles, true, s)) != hipSuccess)
            return hip_fail(e, "widen");
        {
            LaunchTimer lt(s, MR_K_QUEUE, 0);
            e = launch_queue(tbytes, conn, imgs, ctrl, bitmap, qflag, ring, L.ring_cap, blocks,
                             QUEUE_WAIT_US, s);
        }
        if (e != hipSuccess) return hip_fail(e, "queue");
        if (imgs.wide && (e = launch_widen(imgs, L.n_tiles, false, s)) != hipSuccess)
            return hip_fail(e, "narrow");
        return MR_OK;
    };
    if (tn.sweep_rounds > 0) {
        for (round = 2; round <= (uint32_t)tn.sweep_rounds; ++round) {
            span.begin(round);
            {
                LaunchTimer lt(s, MR_K_TILE_ROUND, (int32_t)round);
                e = launch_tile_round(tbytes, conn, imgs, L.n_tiles, flags, lists, ctrl, round,
                                      tn.max_sweeps, grid, s, op_all);
            }
            if (e != hipSuccess) return hip_fail(e, "tile round");
            span.add();
        }
        span.close();
        if ((e = launch_store_u64(&ctrl->rounds, (unsigned long long)tn.sweep_rounds, s)) !=
            hipSuccess)
            return hip_fail(e, "store");
        const int rc = queue_phase(round);
        if (rc != MR_OK) return rc;
    } else if (tn.tail_rounds > 0) {
        // converge mode with the tile queue: a fixed number of rounds, then
        // the queue takes every tile still listed and runs to the fixed point
        for (round = 2; round <= (uint32_t)tn.tail_rounds; ++round) {
            span.begin(round);
            {
                LaunchTimer lt(s, MR_K_TILE_ROUND, (int32_t)round);
                e = launch_tile_round(tbytes, conn, imgs, L.n_tiles, flags, lists, ctrl, round,
                                      tn.max_sweeps, grid, s, op_all);
            }
            if (e != hipSuccess) return hip_fail(e, "tile round");
            span.add();
        }
        span.close();
        if ((e = launch_store_u64(&ctrl->rounds, (unsigned long long)tn.tail_rounds, s)) !=
            hipSuccess)
            return hip_fail(e, "store");
        {
            LaunchTimer lt(s, MR_K_TILE_QUEUE, 0);
            e = launch_tile_queue(tbytes, conn, imgs, L.n_tiles, lists, (uint32_t)tn.tail_rounds + 1,
                                  ctrl, qflag, ring, L.ring_cap, tn.max_sweeps, grid,
                                  QUEUE_WAIT_US, s, op_all);
        }
        if (e != hipSuccess) return hip_fail(e, "tile queue");
    } else {
        // converge mode: rounds until a round leaves no dirty tile, in
        // batches of 8, each followed by a copy of the next round's list
        // lengths to the host. The host reads a batch's count one batch
        // behind: the next batch is already enqueued while it waits, so the
        // device does not idle on the poll. A batch enqueued after the last
        // dirty round finds empty lists and changes nothing.
        PollSet *ps = idle_poll_set();
        if (!ps) return fail(MR_EHIP, "cannot allocate the pinned poll words or events");
        uint32_t *hw = ps->words;
        hipEvent_t *ev = ps->ev;
        const uint32_t poll = 8;
        const uint32_t cap = tn.converge_rounds > 0 ? (uint32_t)tn.converge_rounds : MAX_ROUNDS;
        bool left = false; // work still listed after `cap` rounds
        auto batch = [&](int slot) -> hipError_t {
            for (uint32_t k = 0; k < poll && round < cap; ++k) {
                ++round;
                span.begin(round);
                {
                    LaunchTimer lt(s, MR_K_TILE_ROUND, (int32_t)round);
                    e = launch_tile_round(tbytes, conn, imgs, L.n_tiles, flags, lists, ctrl,
                                          round, tn.max_sweeps, grid, s, op_all);
                }
                if (e != hipSuccess) return e;
                span.add();
            }
            span.close(); // the host may wait after this batch
            if ((e = hipMemcpyAsync(hw + slot * NBANDS, ctrl->round_tiles[round + 1],
                                    sizeof(uint32_t) * NBANDS, hipMemcpyDeviceToHost, s)) !=
                hipSuccess)
                return e;
            if ((e = hipEventRecord(ev[slot], s)) != hipSuccess) return e;
            ps->recorded[slot] = true;
            return hipSuccess;
        };
        int slot = 0;
        if ((e = batch(slot)) != hipSuccess) return hip_fail(e, "tile round batch");
        while (true) {
            const bool ahead = round < cap; // room for one more batch
            if (ahead && (e = batch(slot ^ 1)) != hipSuccess)
                return hip_fail(e, "tile round batch");
            if ((e = hipEventSynchronize(ev[slot])) != hipSuccess) return hip_fail(e, "poll");
            uint64_t next = 0;
            for (int b = 0; b < NBANDS; ++b) next += hw[slot * NBANDS + b];
            if (next == 0) break; // converged; a batch enqueued ahead is empty
            if (!ahead) {         // this count was taken at the cap
                left = true;
                break;
            }
            slot ^= 1;
        }
        if ((e = launch_store_u64(&ctrl->rounds, (unsigned long long)round, s)) != hipSuccess)
            return hip_fail(e, "store");
        // a propagation path too long for the rounds: the queue finishes it
        if (left) {
            const int rc = queue_phase(round + 1);
            if (rc != MR_OK) return rc;
        }
    }
    if (any_fill && (e = launch_fill_output(tbytes, imgs, L.n_tiles, s)) != hipSuccess)
        return hip_fail(e, "fill output");
    return MR_OK;
}

int run_single(int op, void *J_io, const void *I, int64_t H, int64_t W, int64_t pitch, int t,
               int conn, void *ws, size_t ws_bytes, const mr_tune *tune, void *stream) {
    g_err.clear();
    int rc;
    if ((rc = check_image(op, H, W, pitch, t, conn)) != MR_OK) return rc;
    if ((rc = check_tune(tune)) != MR_OK) return rc;
    if (!J_io || (op == MR_OP_RECON && !I) || !ws)
        return fail(MR_EINVAL, "null image or workspace pointer");
    if ((uintptr_t)ws % 256) return fail(MR_EINVAL, "workspace must be 256-byte aligned");
    if ((uintptr_t)J_io % t || (I && (uintptr_t)I % t))
        return fail(MR_EINVAL, "image pointers must be aligned to the pixel size");
    Layout L = single_layout(op, H, W, t, wants_wide(t, tune));
    if (ws_bytes < L.total) L = single_layout(op, H, W, t); // (no room for the widened plane)
    if (ws_bytes < L.total)
        return fail(MR_ENOMEM, "workspace too small: %zu bytes given, %zu needed", ws_bytes,
                    L.total);
    const bool wide = L.total > L.off_wide;
    if (pitch == 0) pitch = W;
    ImgDesc d{};
    d.H = H;
    d.W = W;
    d.op = op;
    d.ntx = (int32_t)tiles_across(W);
    d.nty = (int32_t)tiles_across(H);
    d.tile_base = 0;
    d.first_round = 1;
    d.done = 0;
    if (op == MR_OP_RECON) {
        d.J = J_io;
        d.I = I;
        d.out = nullptr;
        d.pJ = pitch;
        d.pI = pitch;
    } else {
        d.J = (char *)ws + L.off_plane;
        d.I = J_io;
        d.out = J_io;
        d.pJ = L.plane_pitch;
        d.pI = pitch;
    }
    d.wide = wide ? (uint32_t *)((char *)ws + L.off_wide) : nullptr;
    const mr_tune tn = effective_tune(tune);
    Imgs imgs{};
    imgs.n = 1;
    imgs.owner = nullptr;
    imgs.d = (const ImgDesc *)((char *)ws + L.off_desc);
    imgs.staged = staged_planes(t, d) ? 1 : 0;
    imgs.wide = wide ? 1 : 0;
    hipError_t e = launch_put_desc((ImgDesc *)imgs.d, d, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "descriptor");
    return run_sequence(t, conn, imgs, L, ws, tn, (hipStream_t)stream, op == MR_OP_FILL, op);
}

// ---------------------------------------------------------------- batches

size_t plane_bytes(int64_t H, int64_t W, int t) {
    return align_up((size_t)H * align_up((size_t)W, 64) * (size_t)t, 256);
}

struct BatchPlan {
    Layout L;
    std::vector<ImgDesc> descs;
    bool any_fill = false, any_recon = false;
    size_t data_bytes = 0; // sum of H * W * t (autotune backup)
};

// Checks every image and lays the batch out in a workspace (ws may be null
// when only the size is wanted).
int plan_batch(const mr_tile *tiles, int32_t n, int t, int conn, void *ws, BatchPlan &bp,
               bool wide = false) {
    if (!tiles || n < 1) return fail(MR_EINVAL, "need at least one tile");
    int64_t n_tiles = 0, fill_bytes = 0;
    size_t wide_bytes = 0;
    bp.descs.resize((size_t)n);
    for (int32_t i = 0; i < n; ++i) {
        const mr_tile &tl = tiles[i];
        int rc = check_image(tl.op, tl.H, tl.W, tl.pitch, t, conn);
        if (rc != MR_OK) return fail(rc, "tile %d: %s", i, g_err.c_str());
        if (tl.reserved != 0) return fail(MR_EINVAL, "tile %d: reserved must be 0", i);
        if (!tl.data_inout) return fail(MR_EINVAL, "tile %d: null data pointer", i);
        if (tl.op == MR_OP_RECON && !tl.mask) return fail(MR_EINVAL, "tile %d: null mask", i);
        if ((uintptr_t)tl.data_inout % t || (tl.mask && (uintptr_t)tl.mask % t))
            return fail(MR_EINVAL, "tile %d: pointers must be aligned to the pixel size", i);
        ImgDesc &d = bp.descs[(size_t)i];
        d = ImgDesc{};
        d.H = tl.H;
        d.W = tl.W;
        d.op = tl.op;
        d.ntx = (int32_t)tiles_across(tl.W);
        d.nty = (int32_t)tiles_across(tl.H);
        d.tile_base = n_tiles;
        d.done = 0;
        const int64_t pitch = tl.pitch ? tl.pitch : tl.W;
        if (tl.op == MR_OP_RECON) {
            d.J = tl.data_inout;
            d.I = tl.mask;
            d.pJ = d.pI = pitch;
            bp.any_recon = true;
        } else {
            d.J = (void *)(uintptr_t)fill_bytes; // offset for now, based below
            d.I = tl.data_inout;
            d.out = tl.data_inout;
            d.pJ = (int64_t)align_up((size_t)tl.W, 64);
            d.pI = pitch;
            fill_bytes += (int64_t)plane_bytes(tl.H, tl.W, t);
            bp.any_fill = true;
        }
        d.first_round = 1;
        if (wide) {
            d.wide = (uint32_t *)(uintptr_t)wide_bytes; // offset for now, based below
            wide_bytes += wide_plane_bytes(tl.H, tl.W);
        }
        n_tiles += (int64_t)d.ntx * d.nty;
        bp.data_bytes += align_up((size_t)tl.H * tl.W * t, 256);
        if (n_tiles >= (1ll << 31) - 1) return fail(MR_EINVAL, "batch too large");
    }
    bp.L = layout_for(n_tiles, fill_bytes, 0, n, wide_bytes);
    for (auto &d : bp.descs) {
        if (d.op == MR_OP_FILL)
            d.J = ws ? (void *)((char *)ws + bp.L.off_plane + (uintptr_t)d.J) : nullptr;
        if (wide)
            d.wide = ws ? (uint32_t *)((char *)ws + bp.L.off_wide + (uintptr_t)d.wide) : nullptr;
    }
    return MR_OK;
}

int run_batch(const mr_tile *tiles, int32_t n, int t, int conn, void *ws, size_t ws_bytes,
              const mr_tune *tune, hipStream_t s) {
    int rc;
    if ((rc = check_tune(tune)) != MR_OK) return rc;
    if (!ws) return fail(MR_EINVAL, "null workspace");
    if ((uintptr_t)ws % 256) return fail(MR_EINVAL, "workspace must be 256-byte aligned");
    BatchPlan bp;
    bool wide = wants_wide(t, tune);
    if ((rc = plan_batch(tiles, n, t, conn, ws, bp, wide)) != MR_OK) return rc;
    if (wide && ws_bytes < bp.L.total) { // no room for the widened planes
        wide = false;
        if ((rc = plan_batch(tiles, n, t, conn, ws, bp)) != MR_OK) return rc;
    }
    if (ws_bytes < bp.L.total)
        return fail(MR_ENOMEM, "workspace too small: %zu bytes given, %zu needed", ws_bytes,
                    bp.L.total);
    ImgDesc *dd = (ImgDesc *)((char *)ws + bp.L.off_desc);
    hipError_t e = launch_put_descs(dd, bp.descs.data(), n, s);
    if (e != hipSuccess) return hip_fail(e, "descriptors");
    Imgs imgs{dd, n, nullptr, 1, wide ? 1 : 0};
    for (const auto &d : bp.descs)
        if (!staged_planes(t, d)) imgs.staged = 0;
    const int op_all = bp.any_fill ? (bp.any_recon ? -1 : MR_OP_FILL) : MR_OP_RECON;
    return run_sequence(t, conn, imgs, bp.L, ws, effective_tune(tune), s, bp.any_fill, op_all);
}

} // namespace

// ------------------------------------------------- allocation-free entry

namespace {

// Scratch of mr_recon_dilate_noalloc: one array per GPU, allocated by the
// runtime when the library's code object is loaded on that GPU and held until
// the process ends. In host code `scratch` names a host-side stand-in, not
// the device array: kernels and copies get the device address that
// hipGetSymbolAddress returns for the current device, kept per device.
static __device__ __align__(256) unsigned char scratch[MR_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

// The device address of this device's scratch array, looked up once per
// device with that device current. Null with the error set on failure.
void *scratch_for_current_device() {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        hip_fail(e, "hipGetDevice");
        return nullptr;
    }
    if (dev < 0 || dev >= MAX_DEVICES) {
        fail(MR_EINVAL, "device %d is beyond the %d devices the scratch table holds", dev,
             MAX_DEVICES);
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
            return nullptr;
        }
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

} // namespace

namespace mr {
void clear_error() { g_err.clear(); }
int set_error(int code, const char *msg) {
    g_err = msg;
    return code;
}
} // namespace mr

struct mr_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" {

void mr_default_tune(mr_tune *out) {
    if (!out) return;
    out->sweep_rounds = -1;
    out->max_sweeps = 16;
    out->persistent_blocks = 0;
    out->converge_rounds = 0;
    out->tail_rounds = 8;
    out->first_sweeps = 1;
    // MR_TUNE_<FIELD> environment overrides, each taken only when it is a
    // whole number inside the field's valid range
    auto env = [](const char *name, int32_t lo, int32_t hi, bool nonzero, int32_t &field) {
        const char *v = std::getenv(name);
        if (!v || !*v) return;
        char *end = nullptr;
        const long x = std::strtol(v, &end, 10);
        if (*end || x < lo || x > hi || (nonzero && x == 0)) return;
        field = (int32_t)x;
    };
    env("MR_TUNE_SWEEP_ROUNDS", -1, MAX_ROUNDS, true, out->sweep_rounds);
    env("MR_TUNE_MAX_SWEEPS", 1, 1024, false, out->max_sweeps);
    env("MR_TUNE_PERSISTENT_BLOCKS", 0, 1 << 20, false, out->persistent_blocks);
    env("MR_TUNE_CONVERGE_ROUNDS", 0, MAX_ROUNDS, false, out->converge_rounds);
    env("MR_TUNE_TAIL_ROUNDS", 0, MAX_ROUNDS, false, out->tail_rounds);
    env("MR_TUNE_FIRST_SWEEPS", 1, 1024, false, out->first_sweeps);
}

size_t mr_workspace_bytes(int op, int64_t H, int64_t W, mr_dtype t, int conn, const mr_tune *tune) {
    g_err.clear();
    if (check_image(op, H, W, 0, (int)t, conn) != MR_OK) return 0;
    if (check_tune(tune) != MR_OK) return 0;
    return single_layout(op, H, W, (int)t, wants_wide((int)t, tune)).total;
}

int mr_recon_dilate(void *marker_inout, const void *mask, int64_t H, int64_t W, int64_t pitch,
                    mr_dtype t, int conn, void *ws, size_t ws_bytes, const mr_tune *tune,
                    void *stream) {
    return run_single(MR_OP_RECON, marker_inout, mask, H, W, pitch, (int)t, conn, ws, ws_bytes,
                      tune, stream);
}

int mr_fill_holes(void *img_inout, int64_t H, int64_t W, int64_t pitch, mr_dtype t, int conn,
                  void *ws, size_t ws_bytes, const mr_tune *tune, void *stream) {
    return run_single(MR_OP_FILL, img_inout, nullptr, H, W, pitch, (int)t, conn, ws, ws_bytes,
                      tune, stream);
}

size_t mr_batch_workspace_bytes(const mr_tile *tiles, int32_t n, mr_dtype t, int conn,
                                const mr_tune *tune) {
    g_err.clear();
    if (check_tune(tune) != MR_OK) return 0;
    BatchPlan bp;
    if (plan_batch(tiles, n, (int)t, conn, nullptr, bp, wants_wide((int)t, tune)) != MR_OK)
        return 0;
    return bp.L.total;
}

int mr_batch(const mr_tile *tiles, int32_t n, mr_dtype t, int conn, void *ws, size_t ws_bytes,
             const mr_tune *tune, void *stream) {
    g_err.clear();
    return run_batch(tiles, n, (int)t, conn, ws, ws_bytes, tune, (hipStream_t)stream);
}

int mr_batch_graph_create(const mr_tile *tiles, int32_t n, mr_dtype t, int conn, void *ws,
                          size_t ws_bytes, const mr_tune *tune, mr_graph **out) {
    g_err.clear();
    if (!out) return fail(MR_EINVAL, "null output handle");
    *out = nullptr;
    if (!tune || (tune->sweep_rounds <= 0 && tune->tail_rounds <= 0))
        return fail(MR_EINVAL, "a graph needs tune->sweep_rounds > 0 or tune->tail_rounds > 0 "
                               "(the converge mode without the tile queue waits on the host)");
    if (check_tune(tune) != MR_OK) return MR_EINVAL;
    hipStream_t s = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "stream");
    const int timing = g_timing.on;
    g_timing.on = MR_TIMING_OFF;
    mr_graph *g = new mr_graph();
    int rc = MR_OK;
    if ((e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
        rc = hip_fail(e, "begin capture");
    } else {
        rc = run_batch(tiles, n, (int)t, conn, ws, ws_bytes, tune, s);
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(s, &graph);
        if (rc == MR_OK && e != hipSuccess) rc = hip_fail(e, "end capture");
        g->graph = graph;
        if (rc == MR_OK && (e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0)) !=
                               hipSuccess)
            rc = hip_fail(e, "instantiate");
    }
    g_timing.on = timing;
    // the capture stream never ran work: a failed destroy changes nothing
    (void)hipStreamDestroy(s);
    if (rc != MR_OK) {
        mr_graph_destroy(g);
        return rc;
    }
    *out = g;
    return MR_OK;
}

int mr_graph_launch(mr_graph *g, void *stream) {
    g_err.clear();
    if (!g || !g->exec) return fail(MR_EINVAL, "null graph");
    hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)stream);
    return e == hipSuccess ? MR_OK : hip_fail(e, "graph launch");
}

void mr_graph_destroy(mr_graph *g) {
    if (!g) return;
    // (a void function: a failed destroy can only leak the handle)
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

size_t mr_autotune_workspace_bytes(const mr_tile *tiles, int32_t n, mr_dtype t, int conn) {
    g_err.clear();
    BatchPlan bp;
    if (plan_batch(tiles, n, (int)t, conn, nullptr, bp) != MR_OK) return 0;
    return bp.L.total + bp.data_bytes;
}

int mr_autotune(const mr_tile *tiles, int32_t n, mr_dtype t, int conn, void *ws, size_t ws_bytes,
                void *stream, mr_tune *out) {
    g_err.clear();
    if (!out) return fail(MR_EINVAL, "null output tune");
    if (!ws || (uintptr_t)ws % 256) return fail(MR_EINVAL, "bad workspace");
    const int ti = (int)t;
    BatchPlan bp;
    int rc;
    if ((rc = plan_batch(tiles, n, ti, conn, ws, bp)) != MR_OK) return rc;
    if (ws_bytes < bp.L.total + bp.data_bytes)
        return fail(MR_ENOMEM, "workspace too small for the autotuner: %zu given, %zu needed",
                    ws_bytes, bp.L.total + bp.data_bytes);
    hipStream_t s = (hipStream_t)stream;
    char *backup = (char *)ws + bp.L.total;
    // copy the data aside, and back before every candidate and at the end
    auto copy_all = [&](bool to_backup) -> hipError_t {
        size_t off = 0;
        for (int32_t i = 0; i < n; ++i) {
            const mr_tile &tl = tiles[i];
            const size_t row = (size_t)tl.W * ti, pitch = (size_t)(tl.pitch ? tl.pitch : tl.W) * ti;
            hipError_t e = to_backup
                ? hipMemcpy2DAsync(backup + off, row, tl.data_inout, pitch, row, (size_t)tl.H,
                                   hipMemcpyDeviceToDevice, s)
                : hipMemcpy2DAsync(tl.data_inout, pitch, backup + off, row, row, (size_t)tl.H,
                                   hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) return e;
            off += align_up((size_t)tl.H * tl.W * ti, 256);
        }
        return hipSuccess;
    };
    hipError_t e = copy_all(true);
    if (e != hipSuccess) return hip_fail(e, "backup");
    // {sweep_rounds, max_sweeps, tail_rounds, first_sweeps}
    static const int cand[][4] = {{-1, 16, 0, 1},  {-1, 3, 0, 1},   {-1, 16, 4, 1},  {-1, 16, 6, 1},
                                  {-1, 16, 8, 1},  {-1, 16, 12, 1}, {-1, 16, 4, 16}, {-1, 16, 6, 16},
                                  {-1, 16, 8, 16}, {-1, 16, 12, 16}, {4, 16, 0, 1},  {8, 16, 0, 1},
                                  {12, 16, 0, 1},  {16, 16, 0, 1},  {24, 16, 0, 1},  {32, 16, 0, 1},
                                  {48, 16, 0, 1},  {16, 3, 0, 1},   {-1, 16, 16, 1}, {-1, 16, 20, 1}};
    hipEvent_t a = nullptr, b = nullptr;
    if ((e = hipEventCreate(&a)) != hipSuccess || (e = hipEventCreate(&b)) != hipSuccess) {
        if (a) (void)hipEventDestroy(a);
        return hip_fail(e, "event");
    }
    const int timing = g_timing.on;
    g_timing.on = MR_TIMING_OFF;
    float best = 1e30f;
    mr_tune bt;
    mr_default_tune(&bt);
    for (const auto &c : cand) {
        mr_tune tn;
        mr_default_tune(&tn);
        tn.sweep_rounds = c[0];
        tn.max_sweeps = c[1];
        tn.tail_rounds = c[2];
        tn.first_sweeps = c[3];
        float t_best = 1e30f;
        for (int rep = 0; rep < 2 && rc == MR_OK; ++rep) {
            if ((e = copy_all(false)) != hipSuccess) { rc = hip_fail(e, "restore"); break; }
            if ((e = hipEventRecord(a, s)) != hipSuccess) { rc = hip_fail(e, "event"); break; }
            // (the bytes past bp.L.total hold the backup: the candidate runs
            // in the plain batch layout, without widened planes)
            rc = run_batch(tiles, n, ti, conn, ws, bp.L.total, &tn, s);
            if (rc != MR_OK) break;
            if ((e = hipEventRecord(b, s)) != hipSuccess) { rc = hip_fail(e, "event"); break; }
            if ((e = hipEventSynchronize(b)) != hipSuccess) { rc = hip_fail(e, "sync"); break; }
            float ms = 0.f;
            if ((e = hipEventElapsedTime(&ms, a, b)) != hipSuccess) { rc = hip_fail(e, "event"); break; }
            t_best = std::min(t_best, ms);
        }
        if (rc != MR_OK) break;
        if (t_best < best) {
            best = t_best;
            bt = tn;
        }
    }
    g_timing.on = timing;
    if (rc == MR_OK && (e = copy_all(false)) != hipSuccess) rc = hip_fail(e, "restore");
    if (rc == MR_OK && (e = hipStreamSynchronize(s)) != hipSuccess) rc = hip_fail(e, "sync");
    // the events are no longer recorded anywhere: a failed destroy only leaks them
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (rc == MR_OK) *out = bt;
    return rc;
}

int mr_read_counters(const void *ws, mr_counters *out, void *stream) {
    g_err.clear();
    if (!ws || !out) return fail(MR_EINVAL, "null pointer");
    Ctrl h;
    hipError_t e = hipMemcpyAsync(&h, ws, sizeof h, hipMemcpyDeviceToHost, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "counter copy");
    if ((e = hipStreamSynchronize((hipStream_t)stream)) != hipSuccess)
        return hip_fail(e, "counter sync");
    mr_counters c{};
    c.rounds = h.rounds;
    c.seeds = h.seeds_total.v;
    for (unsigned long long r = 1; r <= h.rounds && r <= (unsigned long long)MAX_ROUNDS; ++r)
        c.tiles += round_total(h, r);
    for (int i = 0; i < NCNT; ++i) {
        c.pops += h.pops[i];
        c.pushes += h.pushes[i];
        c.cas_retries += h.cas[i];
        c.overflows += h.ovf[i];
        c.sweeps += h.iters[i];
        c.tiles += h.tiles[i]; // tile-queue visits
    }
    *out = c;
    if (h.watchdog) return fail(MR_EHIP, "a queue or tile-queue wave saw no progress for its watchdog time");
    return MR_OK;
}

int mr_status(const void *ws, void *stream) {
    g_err.clear();
    if (!ws) return fail(MR_EINVAL, "null workspace");
    unsigned long long w = 0;
    hipError_t e = hipMemcpyAsync(&w, &((const Ctrl *)ws)->watchdog, sizeof w,
                                  hipMemcpyDeviceToHost, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "status copy");
    if ((e = hipStreamSynchronize((hipStream_t)stream)) != hipSuccess)
        return hip_fail(e, "status sync");
    if (w)
        return fail(MR_EHIP, "the last call on this workspace gave up (%llu watchdog or ring "
                             "guard events): its result is incomplete", w);
    return MR_OK;
}

int mr_read_round_tiles(const void *ws, uint32_t *out, int32_t cap, int32_t *n_rounds,
                        void *stream) {
    g_err.clear();
    if (!ws || !n_rounds || (cap > 0 && !out) || cap < 0) return fail(MR_EINVAL, "bad pointer or cap");
    Ctrl h;
    hipError_t e = hipMemcpyAsync(&h, ws, sizeof h, hipMemcpyDeviceToHost, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "copy");
    if ((e = hipStreamSynchronize((hipStream_t)stream)) != hipSuccess) return hip_fail(e, "sync");
    const int n = (int)std::min<unsigned long long>(h.rounds + 1, MAX_ROUNDS);
    *n_rounds = (int32_t)h.rounds;
    for (int i = 0; i < cap && i < n; ++i) out[i] = (uint32_t)round_total(h, i + 1);
    return MR_OK;
}

int mr_timing_enable(int on) {
    g_timing.on = on == MR_TIMING_OFF ? MR_TIMING_OFF
                  : on == MR_TIMING_SPANS ? MR_TIMING_SPANS : MR_TIMING_LAUNCHES;
    return MR_OK;
}

int mr_timing_collect(mr_launch_time *out, int32_t cap, int32_t *n) {
    g_err.clear();
    if (!n || cap < 0 || (cap > 0 && !out)) return fail(MR_EINVAL, "bad pointer or cap");
    *n = (int32_t)g_timing.recs.size();
    int rc = MR_OK;
    for (size_t i = 0; i < g_timing.recs.size(); ++i) {
        TimedLaunch &r = g_timing.recs[i];
        float ms = 0.f;
        hipError_t e = hipEventSynchronize(r.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
        if (e != hipSuccess && rc == MR_OK) rc = hip_fail(e, "event");
        if ((int32_t)i < cap) out[i] = mr_launch_time{r.kind, r.round, r.launches, ms};
        g_timing.pool.push_back(r.a);
        g_timing.pool.push_back(r.b);
    }
    g_timing.recs.clear();
    return rc;
}

int mr_recon_dilate_noalloc(void *marker_inout, const void *mask, int64_t H, int64_t W,
                            int64_t pitch, mr_dtype t, int conn, const mr_tune *tune,
                            void *stream) {
    g_err.clear();
    int rc;
    if ((rc = check_image(MR_OP_RECON, H, W, pitch, (int)t, conn)) != MR_OK) return rc;
    if ((rc = check_tune(tune)) != MR_OK) return rc;
    const mr_tune tn = effective_tune(tune);
    // the converge mode polls the device through pinned host words it
    // allocates; the other schedules never wait for the device
    if (tn.sweep_rounds <= 0 && tn.tail_rounds <= 0)
        return fail(MR_EINVAL, "mr_recon_dilate_noalloc needs tune->sweep_rounds > 0 or "
                               "tune->tail_rounds > 0 (the converge mode allocates its poll words)");
    const size_t need = single_layout(MR_OP_RECON, H, W, (int)t).total;
    if (need > (size_t)MR_NOALLOC_SCRATCH_BYTES)
        return fail(MR_ENOMEM, "a %lld x %lld image needs %zu bytes of scratch; "
                               "mr_recon_dilate_noalloc holds %zu",
                    (long long)H, (long long)W, need, (size_t)MR_NOALLOC_SCRATCH_BYTES);
    void *ws = scratch_for_current_device();
    if (!ws) return MR_EHIP;
    // per-launch timing would create events: off for this call
    const int timing = g_timing.on;
    g_timing.on = MR_TIMING_OFF;
    rc = run_single(MR_OP_RECON, marker_inout, mask, H, W, pitch, (int)t, conn, ws,
                    (size_t)MR_NOALLOC_SCRATCH_BYTES, &tn, stream);
    g_timing.on = timing;
    return rc;
}

const char *mr_last_error(void) { return g_err.c_str(); }

int mr_abi_version(void) { return MR_ABI_VERSION; }

} // extern "C"
