// mr_server.hip -- continuous-batching server of libmrecon (mr_server_* in
// include/mr.h).
//
// The caller's arena is the HBM budget. Its head holds the server's control
// block, descriptors, per-tile arrays (owner, dirty flags, the two halves of
// the band lists) and the round counters; the rest is handed out to jobs.
// Every job owns a range of tile ids and planes in the arena while it is on
// the device. A step runs one tile round over all resident jobs' dirty tiles;
// a job admitted between steps has all its tiles on the next round's list
// with that round as its first, so new requests join work already in flight
// instead of waiting for it to drain. A job is finished when a round leaves
// none of its tiles dirty.
//
// Three streams: rounds (and admissions, which must land between rounds)
// run on the caller's stream; input copies run on an upload stream, and the
// fill-holes epilogue and result copies on a download stream, both the
// server's own, so PCIe traffic overlaps the rounds and runs in both
// directions at once. Ordering between them is by events:
//  - an admission waits for its input copy;
//  - a finished job's epilogue and result copy wait for the round that
//    finished it;
//  - a finished job's arena space, tile ids and slot are handed out again
//    only once the host has seen its result copy complete, so no later
//    upload, admission (which rewrites tile owners and the descriptor) or
//    round can touch them while the download stream still reads them.
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <deque>
#include <map>
#include <string>
#include <vector>

#include "mr_internal.h"

using namespace mr;

namespace {

int sfail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    return set_error(code, buf);
}

size_t up(size_t v, size_t a) { return (v + a - 1) / a * a; }

constexpr int RING = 4; // round counters kept: rounds r and r + 1 in flight

// First-fit allocator over [0, size) in units of `align`.
struct RangeAlloc {
    std::map<size_t, size_t> free_; // offset -> length
    size_t align = 1;
    void init(size_t size, size_t a) {
        align = a;
        free_.clear();
        if (size) free_[0] = size;
    }
    bool alloc(size_t n, size_t &off) {
        n = up(std::max<size_t>(n, 1), align);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            off = it->first;
            const size_t rest = it->second - n;
            free_.erase(it);
            if (rest) free_[off + n] = rest;
            return true;
        }
        return false;
    }
    // First fit inside [lo, hi) only.
    bool alloc_in(size_t n, size_t lo, size_t hi, size_t &off) {
        n = up(std::max<size_t>(n, 1), align);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            const size_t a = up(std::max(it->first, lo), align);
            const size_t e = std::min(it->first + it->second, hi);
            if (a >= e || e - a < n) continue;
            const size_t f = it->first, len = it->second;
            free_.erase(it);
            if (a > f) free_[f] = a - f;
            if (f + len > a + n) free_[a + n] = f + len - (a + n);
            off = a;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t n) {
        n = up(std::max<size_t>(n, 1), align);
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t largest() const {
        size_t m = 0;
        for (auto &kv : free_) m = std::max(m, kv.second);
        return m;
    }
};

struct Job {
    uint64_t id;
    int32_t slot;
    mr_job spec;
    int64_t pitch;     // device plane pitch (elements)
    size_t plane;      // bytes of one plane
    size_t mem_off, mem_len;
    int64_t tile_base, n_tiles;
    int band;
    uint32_t first_round;
    ImgDesc d;
};

struct Returning {
    uint64_t id;
    int32_t slot;
    size_t mem_off, mem_len;
    int64_t tile_base, n_tiles;
    int band;
};

} // namespace

struct mr_server {
    char *arena = nullptr;
    size_t arena_bytes = 0;
    int32_t max_jobs = 0;
    int t = 1, conn = 8, max_sweeps = 16;
    hipStream_t stream = nullptr; // rounds and admissions
    hipStream_t up = nullptr;     // input copies
    hipStream_t down = nullptr;   // fill-holes epilogue, result copies
    int64_t n_tiles = 0;          // tile-id space
    // arena head
    Ctrl *ctrl = nullptr;
    uint32_t *counts = nullptr; // [RING][NBANDS]
    uint32_t *busy = nullptr;   // [max_jobs]
    ImgDesc *descs = nullptr;   // [max_jobs]
    uint32_t *owner = nullptr, *flags = nullptr, *lists = nullptr;
    size_t data_off = 0;
    // host state
    RangeAlloc mem, tiles;
    int64_t band_tiles[NBANDS] = {}; // resident tiles whose ids start in each band
    std::vector<int32_t> free_slots;
    std::map<int32_t, Job> resident;  // slot -> job still working
    std::deque<Returning> returning;  // finished, result copy in flight
    std::deque<uint64_t> done;        // result copy complete, not yet polled
    std::vector<hipEvent_t> ev_in, ev_out; // per slot
    hipEvent_t ev_round[2] = {nullptr, nullptr};
    uint32_t *h_busy = nullptr; // pinned, [2][max_jobs]: busy after the last step of each parity
    uint32_t round = 1;         // the round the next step launches first
    int32_t rounds_per_step = 8;
    uint64_t steps = 0;         // steps that launched rounds
    uint32_t inflight = 0;      // last round of the step launched, not yet retired (0: none)
    int inflight_buf = 0;       // its status buffer and event
    uint64_t next_id = 1;
    uint64_t rounds_run = 0;
};

namespace {

size_t job_bytes(const mr_job &j, int t, int64_t &pitch, size_t &plane) {
    pitch = (int64_t)up((size_t)j.W, 64);
    plane = up((size_t)j.H * pitch * t, 256);
    return 2 * plane; // recon: marker + mask; fill: image + working plane
}

int64_t job_tiles(const mr_job &j) { return ((j.H + TI - 1) / TI) * ((j.W + TI - 1) / TI); }

int check_job(const mr_server *s, const mr_job *j) {
    if (!j) return sfail(MR_EINVAL, "null job");
    if (j->op != MR_OP_RECON && j->op != MR_OP_FILL) return sfail(MR_EINVAL, "unknown op %d", j->op);
    if (j->flags & ~MR_JOB_DEVICE) return sfail(MR_EINVAL, "unknown job flags 0x%x", j->flags);
    if (j->H < 1 || j->W < 1) return sfail(MR_EINVAL, "empty image");
    if ((j->ld != 0 && j->ld < j->W) || (j->ld_result != 0 && j->ld_result < j->W))
        return sfail(MR_EINVAL, "host row pitch below the width");
    if (!j->data || !j->result || (j->op == MR_OP_RECON && !j->mask))
        return sfail(MR_EINVAL, "null host buffer");
    int64_t pitch;
    size_t plane;
    const size_t need = job_bytes(*j, s->t, pitch, plane);
    if (need > s->arena_bytes - s->data_off || job_tiles(*j) > s->n_tiles)
        return sfail(MR_EINVAL, "the job needs %zu arena bytes and %lld tiles; the arena has %zu "
                                "and %lld in all", need, (long long)job_tiles(*j),
                     s->arena_bytes - s->data_off, (long long)s->n_tiles);
    if ((int64_t)j->H * pitch >= (1ll << 32))
        return sfail(MR_EINVAL, "image plane too large");
    return MR_OK;
}

int hip_err(hipError_t e, const char *what) {
    return sfail(MR_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// Moves returning jobs whose result copies have completed to `done`, in
// order (the download stream completes them in order), and gives their
// arena space, tile ids and slots back; with `wait`, all of them.
// The tile rounds split the tile-id space into NBANDS bands (band b: ids
// b * n / NBANDS up to (b + 1) * n / NBANDS) and serve band b with the
// workgroups of one die. A first fit over the whole space would put every
// resident job in the first band or two and leave the other dies' workgroups
// idle, so a job's tiles go into the band with the fewest resident tiles
// that has room, and anywhere only if no band has.
int64_t band_start(int64_t n, int b) { return (int64_t)b * n / NBANDS; }

int band_of_tile(int64_t n, int64_t t) {
    int b = 0;
    while (b + 1 < NBANDS && t >= band_start(n, b + 1)) ++b;
    return b;
}

bool alloc_tiles(mr_server *s, int64_t n, size_t &to) {
    int order[NBANDS];
    for (int b = 0; b < NBANDS; ++b) order[b] = b;
    std::stable_sort(order, order + NBANDS,
                     [&](int a, int b) { return s->band_tiles[a] < s->band_tiles[b]; });
    for (int k = 0; k < NBANDS; ++k) {
        const int b = order[k];
        if (s->tiles.alloc_in((size_t)n, (size_t)band_start(s->n_tiles, b),
                              (size_t)band_start(s->n_tiles, b + 1), to))
            return true;
    }
    return s->tiles.alloc((size_t)n, to);
}

int collect(mr_server *s, bool wait) {
    while (!s->returning.empty()) {
        const Returning r = s->returning.front();
        hipError_t e = wait ? hipEventSynchronize(s->ev_out[r.slot]) : hipEventQuery(s->ev_out[r.slot]);
        if (e == hipErrorNotReady) return MR_OK;
        if (e != hipSuccess) return hip_err(e, "result copy");
        s->done.push_back(r.id);
        s->mem.release(r.mem_off, r.mem_len);
        s->tiles.release((size_t)r.tile_base, (size_t)r.n_tiles);
        s->band_tiles[r.band] -= r.n_tiles;
        s->free_slots.push_back(r.slot);
        s->returning.pop_front();
    }
    return MR_OK;
}

// Frees the server's host-side handles. Called on teardown paths that have
// already waited for the streams (or never used them), where a failed destroy
// can only leak a handle and has nobody to report to.
void destroy_handles(mr_server *s) {
    for (hipEvent_t e : s->ev_in)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : s->ev_out)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : s->ev_round)
        if (e) (void)hipEventDestroy(e);
    if (s->up) (void)hipStreamDestroy(s->up);
    if (s->down) (void)hipStreamDestroy(s->down);
    if (s->h_busy) (void)hipHostFree(s->h_busy);
}

} // namespace

extern "C" {

int mr_server_create(void *arena, size_t arena_bytes, int32_t max_jobs, mr_dtype t, int conn,
                     void *stream, mr_server **out) {
    clear_error();
    if (!out) return sfail(MR_EINVAL, "null output handle");
    *out = nullptr;
    if (!arena || (uintptr_t)arena % 256) return sfail(MR_EINVAL, "arena must be 256-byte aligned");
    if (max_jobs < 1 || max_jobs > (1 << 16)) return sfail(MR_EINVAL, "max_jobs out of range");
    if (t != MR_U8 && t != MR_I32) return sfail(MR_EINVAL, "unknown pixel type");
    if (conn != 4 && conn != 8) return sfail(MR_EINVAL, "conn must be 4 or 8");
    // tile ids: one per 62 x 62 pixels of the data area at 2 planes per job,
    // plus slack for the partial tiles at the right and bottom of every job
    const size_t per_tile = 2 * (size_t)TI * TI * (size_t)t;
    const size_t head_fixed = up(sizeof(Ctrl), 256) + up(sizeof(uint32_t) * RING * NBANDS, 256) +
                              up(sizeof(uint32_t) * max_jobs, 256) +
                              up(sizeof(ImgDesc) * max_jobs, 256);
    if (arena_bytes <= head_fixed + (1 << 20)) return sfail(MR_ENOMEM, "arena too small");
    int64_t nt = (int64_t)((arena_bytes - head_fixed) / per_tile) + 4 * (int64_t)max_jobs + 64;
    nt = std::min<int64_t>(nt, (1ll << 31) - 2);
    mr_server *s = new mr_server();
    s->arena = (char *)arena;
    s->arena_bytes = arena_bytes;
    s->max_jobs = max_jobs;
    s->t = (int)t;
    s->conn = conn;
    s->stream = (hipStream_t)stream;
    size_t o = 0;
    s->ctrl = (Ctrl *)(s->arena + o);
    o += up(sizeof(Ctrl), 256);
    s->counts = (uint32_t *)(s->arena + o);
    o += up(sizeof(uint32_t) * RING * NBANDS, 256);
    s->busy = (uint32_t *)(s->arena + o);
    o += up(sizeof(uint32_t) * max_jobs, 256);
    s->descs = (ImgDesc *)(s->arena + o);
    o += up(sizeof(ImgDesc) * max_jobs, 256);
    s->owner = (uint32_t *)(s->arena + o);
    o += up(sizeof(uint32_t) * nt, 256);
    s->flags = (uint32_t *)(s->arena + o);
    o += up(sizeof(uint32_t) * nt, 256);
    s->lists = (uint32_t *)(s->arena + o);
    o += up(sizeof(uint32_t) * 2 * nt, 256);
    if (o + (1 << 20) > arena_bytes) {
        delete s;
        return sfail(MR_ENOMEM, "arena too small");
    }
    s->data_off = o;
    s->n_tiles = nt;
    s->mem.init(arena_bytes - o, 256);
    s->tiles.init((size_t)nt, 1);
    for (int32_t i = max_jobs - 1; i >= 0; --i) s->free_slots.push_back(i);
    s->ev_in.assign(max_jobs, nullptr);
    s->ev_out.assign(max_jobs, nullptr);
    hipError_t e = hipHostMalloc((void **)&s->h_busy, sizeof(uint32_t) * 2 * max_jobs,
                                 hipHostMallocDefault);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->up, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->down, hipStreamNonBlocking);
    for (int i = 0; i < 2 && e == hipSuccess; ++i)
        e = hipEventCreateWithFlags(&s->ev_round[i], hipEventDisableTiming);
    for (int32_t i = 0; i < max_jobs && e == hipSuccess; ++i) {
        e = hipEventCreateWithFlags(&s->ev_in[i], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s->ev_out[i], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = launch_clear_ctrl(s->ctrl, 0, s->stream);
    if (e == hipSuccess) e = launch_clear_u32(s->counts, RING * NBANDS, 0u, s->stream);
    if (e == hipSuccess) e = launch_clear_u32(s->busy, max_jobs, 0u, s->stream);
    if (e == hipSuccess) e = launch_clear_u32(s->flags, nt, 0u, s->stream);
    if (e != hipSuccess) {
        // the set-up error is what gets reported; the wait only makes sure
        // nothing enqueued above still runs when the handles go
        (void)hipStreamSynchronize(s->stream);
        destroy_handles(s);
        delete s;
        return hip_err(e, "server set-up");
    }
    *out = s;
    return MR_OK;
}

int mr_server_submit(mr_server *s, const mr_job *job, uint64_t *id) {
    clear_error();
    if (!s || !id) return sfail(MR_EINVAL, "null pointer");
    int rc;
    if ((rc = check_job(s, job)) != MR_OK) return rc;
    if ((rc = collect(s, false)) != MR_OK) return rc;
    if (s->free_slots.empty()) return sfail(MR_EAGAIN, "all job slots are busy");
    Job j{};
    j.spec = *job;
    const size_t need = job_bytes(*job, s->t, j.pitch, j.plane);
    j.n_tiles = job_tiles(*job);
    size_t mo = 0, to = 0;
    if (!s->mem.alloc(need, mo)) return sfail(MR_EAGAIN, "no room in the arena now");
    if (!alloc_tiles(s, j.n_tiles, to)) {
        s->mem.release(mo, need);
        return sfail(MR_EAGAIN, "no free tile ids now");
    }
    j.band = band_of_tile(s->n_tiles, (int64_t)to);
    s->band_tiles[j.band] += j.n_tiles;
    j.mem_off = mo;
    j.mem_len = need;
    j.tile_base = (int64_t)to;
    j.slot = s->free_slots.back();
    j.id = s->next_id;
    j.first_round = s->round;

    char *p0 = s->arena + s->data_off + mo, *p1 = p0 + j.plane;
    const size_t row = (size_t)job->W * s->t, dp = (size_t)j.pitch * s->t;
    const size_t hp = (size_t)(job->ld ? job->ld : job->W) * s->t;
    const hipMemcpyKind in_kind =
        (job->flags & MR_JOB_DEVICE) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    hipError_t e = hipMemcpy2DAsync(p0, dp, job->data, hp, row, (size_t)job->H, in_kind, s->up);
    if (e == hipSuccess && job->op == MR_OP_RECON)
        e = hipMemcpy2DAsync(p1, dp, job->mask, hp, row, (size_t)job->H, in_kind, s->up);
    if (e == hipSuccess) e = hipEventRecord(s->ev_in[j.slot], s->up);
    if (e == hipSuccess) e = hipStreamWaitEvent(s->stream, s->ev_in[j.slot], 0);
    ImgDesc &d = j.d;
    d = ImgDesc{};
    d.H = job->H;
    d.W = job->W;
    d.op = job->op;
    d.ntx = (int32_t)((job->W + TI - 1) / TI);
    d.nty = (int32_t)((job->H + TI - 1) / TI);
    d.tile_base = j.tile_base;
    d.first_round = j.first_round;
    d.done = 0;
    d.pJ = d.pI = j.pitch;
    if (job->op == MR_OP_RECON) {
        d.J = p0;
        d.I = p1;
        d.out = nullptr;
    } else {
        d.I = p0;
        d.out = p0;
        d.J = p1;
    }
    const uint32_t r = s->round;
    if (e == hipSuccess)
        e = launch_server_admit(s->descs, j.slot, d, s->owner, s->flags,
                                s->lists + (size_t)(r & 1) * s->n_tiles,
                                s->counts + (r % RING) * NBANDS, s->n_tiles, r, s->stream);
    if (e != hipSuccess) {
        // the slot is not handed out: a failed enqueue leaves the streams in
        // an unknown state, and the error is reported
        s->mem.release(mo, need);
        s->tiles.release(to, (size_t)j.n_tiles);
        s->band_tiles[j.band] -= j.n_tiles;
        return hip_err(e, "admit");
    }
    s->free_slots.pop_back();
    ++s->next_id;
    s->resident[j.slot] = j;
    *id = j.id;
    return MR_OK;
}

int mr_server_step(mr_server *s) {
    clear_error();
    if (!s) return sfail(MR_EINVAL, "null server");
    hipError_t e;
    Imgs imgs{s->descs, s->max_jobs, s->owner};
    // 1. launch the step's rounds over every resident job (including those
    //    admitted since the last step); the host does not wait for them here
    uint32_t launched = 0;
    int buf = 0;
    if (!s->resident.empty()) {
        buf = (int)(s->steps++ & 1);
        uint32_t *cout = nullptr;
        for (int32_t k = 0; k < s->rounds_per_step; ++k) {
            const uint32_t r = s->round;
            uint32_t *cin = s->counts + (r % RING) * NBANDS;
            cout = s->counts + ((r + 1) % RING) * NBANDS;
            if ((e = launch_clear_u32(cout, NBANDS, 0u, s->stream)) != hipSuccess)
                return hip_err(e, "clear");
            if ((e = launch_tile_round_ex(s->t, s->conn, imgs, s->n_tiles, s->flags, s->lists,
                                          cin, cout, 0, s->ctrl, r, s->max_sweeps,
                                          persistent_grid(), s->stream)) != hipSuccess)
                return hip_err(e, "tile round");
            s->round = r + 1;
            ++s->rounds_run;
        }
        const uint32_t last = s->round - 1;
        if ((e = launch_server_status(s->lists + (size_t)((last + 1) & 1) * s->n_tiles, cout,
                                      s->owner, s->busy, s->n_tiles, last + 1, s->stream)) !=
            hipSuccess)
            return hip_err(e, "status");
        if ((e = hipMemcpyAsync(s->h_busy + (size_t)buf * s->max_jobs, s->busy,
                                sizeof(uint32_t) * s->max_jobs, hipMemcpyDeviceToHost,
                                s->stream)) != hipSuccess)
            return hip_err(e, "status copy");
        if ((e = hipEventRecord(s->ev_round[buf], s->stream)) != hipSuccess)
            return hip_err(e, "event");
        launched = last;
    }
    // 2. retire what the previous step finished: jobs that had joined by its
    //    last round p and have no tile on the list p left for the next round
    //    (a job that finished earlier in that step has none on it either)
    const uint32_t p = s->inflight;
    const int pb = s->inflight_buf;
    s->inflight = launched;
    s->inflight_buf = buf;
    if (p) {
        if ((e = hipEventSynchronize(s->ev_round[pb])) != hipSuccess)
            return hip_err(e, "round");
        const uint32_t *hb = s->h_busy + (size_t)pb * s->max_jobs;
        std::vector<int32_t> finished;
        for (auto &kv : s->resident) {
            const Job &j = kv.second;
            if (j.first_round <= p && hb[j.slot] != p + 1) finished.push_back(kv.first);
        }
        if (!finished.empty() &&
            (e = hipStreamWaitEvent(s->down, s->ev_round[pb], 0)) != hipSuccess)
            return hip_err(e, "event wait");
        for (int32_t slot : finished) {
            Job &j = s->resident[slot];
            if (j.spec.op == MR_OP_FILL &&
                (e = launch_fill_output(s->t, imgs, j.n_tiles, s->down, j.tile_base)) !=
                    hipSuccess)
                return hip_err(e, "fill output");
            const char *src = (const char *)(j.spec.op == MR_OP_RECON ? j.d.J : j.d.out);
            const size_t row = (size_t)j.spec.W * s->t, dp = (size_t)j.pitch * s->t;
            const size_t hp = (size_t)(j.spec.ld_result ? j.spec.ld_result : j.spec.W) * s->t;
            const hipMemcpyKind out_kind = (j.spec.flags & MR_JOB_DEVICE)
                                               ? hipMemcpyDeviceToDevice
                                               : hipMemcpyDeviceToHost;
            if ((e = hipMemcpy2DAsync(j.spec.result, hp, src, dp, row, (size_t)j.spec.H,
                                      out_kind, s->down)) != hipSuccess ||
                (e = hipEventRecord(s->ev_out[slot], s->down)) != hipSuccess)
                return hip_err(e, "result copy");
            s->returning.push_back(
                Returning{j.id, slot, j.mem_off, j.mem_len, j.tile_base, j.n_tiles, j.band});
            s->resident.erase(slot);
        }
    }
    return collect(s, false);
}

int mr_server_set_rounds_per_step(mr_server *s, int32_t k) {
    clear_error();
    if (!s) return sfail(MR_EINVAL, "null server");
    if (k < 1 || k > 64) return sfail(MR_EINVAL, "rounds per step must be in 1..64");
    s->rounds_per_step = k;
    return MR_OK;
}

int mr_server_poll(mr_server *s, uint64_t *done_ids, int32_t cap, int32_t *n_done) {
    clear_error();
    if (!s || !n_done || cap < 0 || (cap > 0 && !done_ids)) return sfail(MR_EINVAL, "bad pointer");
    *n_done = 0;
    int rc = collect(s, false);
    if (rc != MR_OK) return rc;
    int32_t n = 0;
    while (n < cap && !s->done.empty()) {
        done_ids[n++] = s->done.front();
        s->done.pop_front();
    }
    *n_done = n;
    return MR_OK;
}

int mr_server_drain(mr_server *s) {
    clear_error();
    if (!s) return sfail(MR_EINVAL, "null server");
    const uint64_t cap = (uint64_t)1 << 24;
    for (uint64_t k = 0; !s->resident.empty() || s->inflight; ++k) {
        int rc = mr_server_step(s);
        if (rc != MR_OK) return rc;
        if (k > cap) return sfail(MR_EHIP, "jobs did not finish");
    }
    return collect(s, true);
}

int mr_server_stats(const mr_server *s, int32_t *resident, uint64_t *rounds, size_t *free_bytes) {
    clear_error();
    if (!s) return sfail(MR_EINVAL, "null server");
    if (resident) *resident = (int32_t)(s->resident.size() + s->returning.size());
    if (rounds) *rounds = s->rounds_run;
    if (free_bytes) *free_bytes = s->mem.largest();
    return MR_OK;
}

void mr_server_destroy(mr_server *s) {
    if (!s) return;
    // A void function: a failed wait (a device fault) is reported again by
    // the caller's next synchronization on the stream, and the handles go
    // either way.
    (void)hipStreamSynchronize(s->stream);
    if (s->up) (void)hipStreamSynchronize(s->up);
    if (s->down) (void)hipStreamSynchronize(s->down);
    destroy_handles(s);
    delete s;
}

} // extern "C"
