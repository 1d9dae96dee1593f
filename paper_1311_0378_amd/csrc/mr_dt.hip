// mr_dt.hip -- distance transform (Table II: IWPP, 8-connected);
// mr_distance_transform in include/mr_ops.h.
//
// D(p) = length in G-steps of the shortest path from p to a background
// pixel. As a wavefront propagation (Algorithm 1): background pixels start at
// 0 and foreground pixels at infinity, and a pixel q takes D(p) + 1 from a
// neighbour p whenever that is smaller (PropagationCondition D(p) + 1 < D(q),
// Update D(q) = D(p) + 1). Every value is at all times an upper bound of the
// true distance, and a state where no pixel can lower a neighbour is the
// true distance (along a shortest path each step can add at most 1), so any
// order of updates that runs to such a state gives the same, unique result.
//
// On the GPU the image is cut into 64 x 64 register tiles (a 62 x 62
// interior and a one-pixel halo) held by one wave each: lane = column,
// register = row. A visit loads the tile (the first round builds it from the
// input image), sweeps down and up the registers (the three upper or lower
// neighbours through DPP lane shifts for 8-connectivity), transposes through
// LDS and sweeps right and left, and repeats until an iteration changes
// nothing; it stores the interior and marks for the next round every
// neighbouring tile whose halo it changed. Rounds run until one marks no
// tile; the host polls a small counter between batches of rounds.
#include <algorithm>
#include <cstdarg>
#include <cstdio>

#include "../../include/mr_ops.h"
#include "mr_internal.h"

using namespace mr;

namespace {

int dfail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    return set_error(code, buf);
}

int dhip(hipError_t e, const char *what) {
    return dfail(MR_EHIP, "%s: %s", what, hipGetErrorString(e));
}

size_t up256(size_t n) { return (n + 255) / 256 * 256; }

constexpr int DS = 64, DI = DS - 2;     // register tile and its interior
constexpr uint32_t INF = 0x7FFFFFFFu;   // "not reached yet"; INF + 1 does not wrap
constexpr int DT_BATCH = 4;             // rounds per host poll
constexpr int64_t DT_MAX_ROUNDS = 1 << 20;

// Per-call control words at the head of the workspace.
struct DtCtrl {
    uint32_t has_bg;     // some pixel of the image is background
    uint32_t pad[63];
    uint32_t marked[2];  // tiles marked for the next round, by round parity
    uint32_t pad2[62];
};

// Lane i gets lane i-1's value (lane 0 keeps its own).
__device__ __forceinline__ uint32_t lane_left(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x138 /* wave_shr:1 */, 0xF,
                                                 0xF, false);
}
// Lane i gets lane i+1's value (lane 63 keeps its own).
__device__ __forceinline__ uint32_t lane_right(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x130 /* wave_shl:1 */, 0xF,
                                                 0xF, false);
}

template <int CONN>
__device__ __forceinline__ uint32_t reach(uint32_t prev_row) {
    // the smallest distance among the neighbours in the adjacent row, + 1
    uint32_t m = prev_row;
    if (CONN == 8) m = min(m, min(lane_left(prev_row), lane_right(prev_row)));
    return m + 1u;
}

// (one wave per block: LDS hand-offs between its lanes need program order
// and a compiler barrier, not a workgroup barrier)
__device__ __forceinline__ void dt_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ void transpose(uint32_t (&A)[DS], uint32_t (*tb)[DS + 1], int lane) {
#pragma unroll
    for (int r = 0; r < DS; ++r) tb[r][lane] = A[r];
    dt_wave_sync();
#pragma unroll
    for (int c = 0; c < DS; ++c) A[c] = tb[lane][c];
    dt_wave_sync();
}

// One visit of tile t by the calling wave (every lane, uniform t). A tile
// raised past `round` before its visit is left to the later round it is
// listed for. `tb` is the wave's transpose buffer.
template <int CONN, bool FIRST>
__device__ __forceinline__ void dt_visit(const uint8_t *__restrict__ img, int64_t ipitch,
                                         int32_t *__restrict__ dist, int64_t dpitch, int64_t H,
                                         int64_t W, int32_t ntx, int32_t nty,
                                         uint32_t *__restrict__ flags, uint32_t round,
                                         DtCtrl *__restrict__ ctrl, uint32_t *__restrict__ lists,
                                         int64_t t, uint32_t (*tb)[DS + 1]) {
    const int lane = threadIdx.x;
    if (!FIRST && flags[t] != round) return;
    const int ty = (int)(t / ntx), tx = (int)(t - (int64_t)ty * ntx);
    const int64_t gy0 = (int64_t)ty * DI - 1, gx = (int64_t)tx * DI - 1 + lane;
    const bool xin = gx >= 0 && gx < W;
    const bool in_lane = lane >= 1 && lane <= DS - 2;

    // the first round builds the tile from the image (background 0, else
    // not reached); later rounds read the distances stored so far. Pixels
    // outside the image are never reached and never lower anything.
    // Every row is loaded from a clamped, in-bounds address and masked
    // afterwards. All 64 loads are issued before any of them is used (the
    // compiler otherwise placed each use, and a wait, right after its load).
    // Rows are addressed from the tile's first in-image row (a uniform base)
    // with 32-bit lane offsets, so a load in flight holds one address
    // register rather than two.
    uint32_t D[DS];
    bool any_bg = false, any_fg = false;
    const int64_t xc = gx < 0 ? 0 : (gx > W - 1 ? W - 1 : gx);
    const int64_t y_first = gy0 < 0 ? 0 : gy0;
    const uint8_t *ib = img + y_first * ipitch;
    const int32_t *db = dist + y_first * dpitch;
    if (gy0 >= 0 && gy0 + DS <= H) {
        // every row inside the image: the row offset lives in a vector
        // register, stepped by one pitch per row, so that the 64 row offsets
        // are not all held (in scalar registers, which spill)
        const uint32_t pitch = (uint32_t)(FIRST ? ipitch : dpitch);
        uint32_t off = (uint32_t)xc;
#pragma unroll
        for (int r = 0; r < DS; ++r) {
            asm volatile("" : "+v"(off));
            D[r] = FIRST ? (uint32_t)ib[off] : (uint32_t)db[off];
            off += pitch;
        }
    } else {
        // the top or bottom tile row: rows outside the image read the
        // nearest row inside it (masked below); the clamp is vector
        // arithmetic for the same reason
        int32_t g0 = (int32_t)(gy0 - y_first), hm = (int32_t)(H - 1 - y_first);
        asm volatile("" : "+v"(g0), "+v"(hm));
        const uint32_t pitch = (uint32_t)(FIRST ? ipitch : dpitch);
#pragma unroll
        for (int r = 0; r < DS; ++r) {
            const int32_t rel = min(max(g0 + r, 0), hm);
            const uint32_t off = (uint32_t)rel * pitch + (uint32_t)xc;
            D[r] = FIRST ? (uint32_t)ib[off] : (uint32_t)db[off];
        }
    }
    asm volatile("" ::: "memory");
#pragma unroll
    for (int r = 0; r < DS; ++r) asm volatile("" : "+v"(D[r]));
    // rows r_lo .. r_hi of the tile lie in the image; compared in vector
    // registers (as 64 scalar conditions they would be held and spilled)
    uint32_t r_lo = (uint32_t)(gy0 < 0 ? -gy0 : 0);
    uint32_t r_hi = (uint32_t)(H - 1 - gy0 < DS - 1 ? H - 1 - gy0 : DS - 1);
    asm volatile("" : "+v"(r_lo), "+v"(r_hi));
    // (0/1 arithmetic rather than comparisons: 64 rows of comparison masks
    // are held in scalar registers and spill)
    const uint32_t xin1 = xin ? 1u : 0u;
    uint32_t bg_seen = 0, fg_seen = 0;
#pragma unroll
    for (int r = 0; r < DS; ++r) {
        // 1 for a row inside the image: neither r - r_lo nor r_hi - r is negative
        const uint32_t ok = xin1 & ~(((uint32_t)r - r_lo) | (r_hi - (uint32_t)r)) >> 31;
        if (FIRST) {
            const uint32_t bg = ok & ((D[r] - 1u) >> 31); // pixel 0 (an 8-bit value)
            bg_seen |= bg;
            fg_seen |= ok & ~bg;
            D[r] = INF & (bg - 1u); // 0 for background, else unreached
        } else {
            D[r] = ok ? D[r] : INF;
        }
    }
    any_bg = bg_seen != 0;
    any_fg = fg_seen != 0;
    if (FIRST) {
        // (one atomic per wave at most, and none once some wave has set it:
        // tens of thousands of them on the one word serialise)
        if (__ballot(any_bg) != 0 && lane == 0 &&
            __hip_atomic_load(&ctrl->has_bg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
            atomicOr(&ctrl->has_bg, 1u);
        // a tile whose pixels (halo included) are all background is final
        if (__ballot(any_fg) == 0) {
            if (in_lane && gx < W) {
                int32_t *drow = dist + (gy0 + 1) * dpitch;
                uint32_t off = (uint32_t)gx;
#pragma unroll
                for (int r = 1; r < DS - 1; ++r) {
                    asm volatile("" : "+v"(off));
                    if ((uint32_t)r <= r_hi) drow[off] = 0;
                    off += (uint32_t)dpitch;
                }
            }
            return;
        }
    }
    // Pixels outside the image start unreached and may be lowered by the
    // sweeps like any other (a path through them is never shorter than one
    // along the image's edge, so they cannot shorten an inside distance), but
    // they are never stored and never count as a change. `valid` holds this
    // lane's interior pixels that lie in the image; rows 1.. are at or below
    // row 0 of the image, so only the bottom can run out.
    const bool col_ok = in_lane && xin;
    const int64_t rows_left = H - gy0 - 1; // interior rows inside the image
    const int last_row = rows_left < DS - 2 ? (int)rows_left : DS - 2;
    // (the bottom tile row compares each row with last_row in vector
    // registers: as scalar conditions the compiler keeps all 62 of them live
    // across the sweep loop, and they spill)
    auto vsum = [&]() {
        uint64_t sm = 0;
        if (last_row == DS - 2) {
#pragma unroll
            for (int r = 1; r < DS - 1; ++r) sm += D[r];
        } else {
            uint32_t lr = (uint32_t)last_row;
            asm volatile("" : "+v"(lr));
#pragma unroll
            for (int r = 1; r < DS - 1; ++r) sm += (uint32_t)r <= lr ? D[r] : 0u;
        }
        return col_ok ? sm : 0ull;
    };
    // border rows as loaded (what the neighbours' halos hold), and each
    // interior column's sum as loaded (distances only fall, so a column
    // changed iff its sum did)
    const uint32_t in_top = D[1], in_bot = D[DS - 2];
    const uint64_t sum_in = vsum();

    // down and up sweeps (the neighbours in the adjacent row: three with
    // 8-connectivity, through lane shifts), then right and left sweeps on
    // the transposed tile (the in-row neighbour), until an iteration changes
    // no interior pixel
    uint64_t sum_prev = sum_in;
    bool changed = false, stable = false;
    for (int it = 0; it < 64; ++it) {
#pragma unroll
        for (int r = 1; r < DS - 1; ++r) D[r] = min(D[r], reach<CONN>(D[r - 1]));
#pragma unroll
        for (int r = DS - 2; r >= 1; --r) D[r] = min(D[r], reach<CONN>(D[r + 1]));
        transpose(D, tb, lane); // lane = row, register = column
#pragma unroll
        for (int c = 1; c < DS - 1; ++c) D[c] = min(D[c], D[c - 1] + 1u);
#pragma unroll
        for (int c = DS - 2; c >= 1; --c) D[c] = min(D[c], D[c + 1] + 1u);
        transpose(D, tb, lane);
        const uint64_t sum = vsum();
        const bool ch = sum != sum_prev;
        sum_prev = sum;
        if (__ballot(ch) == 0) {
            stable = true;
            break;
        }
        changed = true;
    }
    if (changed || FIRST) {
        if (in_lane && gx < W) {
            // rows gy0 + 1 .. are all >= 0; only the bottom may leave the image
            int32_t *drow = dist + (gy0 + 1) * dpitch;
            uint32_t off = (uint32_t)gx;
#pragma unroll
            for (int r = 1; r < DS - 1; ++r) {
                asm volatile("" : "+v"(off));
                if (r <= last_row) drow[off] = (int32_t)D[r];
                off += (uint32_t)dpitch;
            }
        }
    }
    if (!changed && stable) return;
    // mark for the next round this tile if the iteration cap stopped it, and
    // every neighbour whose halo holds a border pixel that changed here:
    // rows 1 and DS-2 (per lane), columns 1 and DS-2 (lanes 1 and DS-2),
    // and the corner pixels for the diagonal neighbours (8-connectivity)
    const uint64_t bt = __ballot(col_ok && D[1] != in_top);
    const uint64_t bb = __ballot(col_ok && last_row == DS - 2 && D[DS - 2] != in_bot);
    const uint64_t bc = __ballot(sum_prev != sum_in);
    const uint32_t nxt = round + 1;
    bool want = false;
    int dy = 0, dx = 0;
    switch (lane) {
    case 0: want = !stable; break;
    case 1: want = bt != 0; dy = -1; break;
    case 2: want = bb != 0; dy = 1; break;
    case 3: want = (bc >> 1) & 1; dx = -1; break;
    case 4: want = (bc >> (DS - 2)) & 1; dx = 1; break;
    case 5: want = CONN == 8 && ((bt >> 1) & 1); dy = -1; dx = -1; break;
    case 6: want = CONN == 8 && ((bt >> (DS - 2)) & 1); dy = -1; dx = 1; break;
    case 7: want = CONN == 8 && ((bb >> 1) & 1); dy = 1; dx = -1; break;
    case 8: want = CONN == 8 && ((bb >> (DS - 2)) & 1); dy = 1; dx = 1; break;
    default: break;
    }
    const int ny = ty + dy, nx = tx + dx;
    if (want && ny >= 0 && ny < nty && nx >= 0 && nx < ntx) {
        const int64_t nb = (int64_t)ny * ntx + nx;
        // the first mark of a tile for round nxt lists it for that round
        if (atomicMax(flags + nb, nxt) < nxt) {
            const int64_t n = (int64_t)ntx * nty;
            const uint32_t slot = atomicAdd(&ctrl->marked[nxt & 1], 1u);
            if ((int64_t)slot < n) lists[(int64_t)(nxt & 1) * n + slot] = (uint32_t)nb;
        }
    }
}

// Round 1 visits every tile, one wave per tile. A later round visits the
// tiles listed for it (each at most once: a tile is listed when its flag
// first reaches the round), a fixed grid of waves walking the list, so that
// a round with few marked tiles does not launch a wave per tile.
template <int CONN, bool FIRST>
__global__ __launch_bounds__(64) void k_dt_round(const uint8_t *__restrict__ img, int64_t ipitch,
                                                 int32_t *__restrict__ dist, int64_t dpitch,
                                                 int64_t H, int64_t W, int32_t ntx, int32_t nty,
                                                 uint32_t *__restrict__ flags, uint32_t round,
                                                 DtCtrl *__restrict__ ctrl,
                                                 uint32_t *__restrict__ lists) {
    __shared__ uint32_t tb[DS][DS + 1];
    if (FIRST) {
        dt_visit<CONN, true>(img, ipitch, dist, dpitch, H, W, ntx, nty, flags, round, ctrl, lists,
                             (int64_t)blockIdx.x, tb);
        return;
    }
    const int64_t n = (int64_t)ntx * nty;
    const int64_t cnt = std::min<int64_t>(ctrl->marked[round & 1], n);
    const uint32_t *list = lists + (int64_t)(round & 1) * n;
    for (int64_t i = blockIdx.x; i < cnt; i += gridDim.x)
        dt_visit<CONN, false>(img, ipitch, dist, dpitch, H, W, ntx, nty, flags, round, ctrl,
                              lists, (int64_t)list[i], tb);
}

__global__ void k_dt_clear(DtCtrl *c, uint32_t *flags, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        c->has_bg = 0;
        c->marked[0] = c->marked[1] = 0;
    }
    for (int64_t k = i; k < n; k += (int64_t)gridDim.x * blockDim.x) flags[k] = 0;
}

__global__ void k_dt_reset_mark(DtCtrl *c, uint32_t parity) { c->marked[parity] = 0; }

__global__ void k_dt_fill(int32_t *dist, int64_t dpitch, int64_t H, int64_t W, int32_t v) {
    const int64_t n = H * W;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t y = i / W;
        dist[y * dpitch + (i - y * W)] = v;
    }
}

struct DtLayout {
    size_t ctrl = 0, flags = 0, lists = 0, total = 0;
    int64_t ntx = 0, nty = 0;
};

DtLayout dt_layout(int64_t H, int64_t W) {
    DtLayout L;
    L.ntx = (W + DI - 1) / DI;
    L.nty = (H + DI - 1) / DI;
    L.ctrl = 0;
    L.flags = up256(sizeof(DtCtrl));
    L.lists = L.flags + up256((size_t)(L.ntx * L.nty) * 4);
    L.total = L.lists + up256((size_t)(L.ntx * L.nty) * 8); // one list per round parity
    return L;
}

hipError_t dt_round(int conn, bool first, const uint8_t *img, int64_t ipitch, int32_t *dist,
                    int64_t dpitch, int64_t H, int64_t W, const DtLayout &L, uint32_t *flags,
                    uint32_t *lists, uint32_t round, DtCtrl *ctrl, hipStream_t s) {
    const unsigned n = (unsigned)(L.ntx * L.nty);
    // later rounds: a fixed grid walks the round's list (the count is on the
    // device); 8192 waves (measured against 2048 to 32768)
    const unsigned g = first ? n : std::min(n, 8192u);
    const int32_t ntx = (int32_t)L.ntx, nty = (int32_t)L.nty;
    if (conn == 8) {
        if (first)
            hipLaunchKernelGGL((k_dt_round<8, true>), dim3(g), dim3(64), 0, s, img, ipitch, dist,
                               dpitch, H, W, ntx, nty, flags, round, ctrl, lists);
        else
            hipLaunchKernelGGL((k_dt_round<8, false>), dim3(g), dim3(64), 0, s, img, ipitch, dist,
                               dpitch, H, W, ntx, nty, flags, round, ctrl, lists);
    } else {
        if (first)
            hipLaunchKernelGGL((k_dt_round<4, true>), dim3(g), dim3(64), 0, s, img, ipitch, dist,
                               dpitch, H, W, ntx, nty, flags, round, ctrl, lists);
        else
            hipLaunchKernelGGL((k_dt_round<4, false>), dim3(g), dim3(64), 0, s, img, ipitch, dist,
                               dpitch, H, W, ntx, nty, flags, round, ctrl, lists);
    }
    return hipGetLastError();
}

} // namespace

extern "C" {

size_t mr_distance_transform_workspace_bytes(int64_t H, int64_t W, int conn) {
    clear_error();
    if (H < 1 || W < 1 || (conn != 4 && conn != 8)) {
        dfail(MR_EINVAL, "bad arguments");
        return 0;
    }
    return dt_layout(H, W).total;
}

int mr_distance_transform(const void *img, void *dist, int64_t H, int64_t W, int64_t pitch,
                          int64_t dist_pitch, int conn, void *ws, size_t ws_bytes,
                          void *stream) {
    clear_error();
    if (pitch == 0) pitch = W;
    if (dist_pitch == 0) dist_pitch = W;
    if (H < 1 || W < 1) return dfail(MR_EINVAL, "H and W must be >= 1");
    if (pitch < W || dist_pitch < W) return dfail(MR_EINVAL, "a pitch is below W");
    if (conn != 4 && conn != 8) return dfail(MR_EINVAL, "conn must be 4 or 8 (got %d)", conn);
    if (!img || !dist || !ws) return dfail(MR_EINVAL, "null pointer");
    if ((uintptr_t)dist % 4) return dfail(MR_EINVAL, "dist must be 4-byte aligned");
    if ((uintptr_t)ws % 256) return dfail(MR_EINVAL, "workspace must be 256-byte aligned");
    const DtLayout L = dt_layout(H, W);
    if (L.ntx * L.nty >= (1ll << 31)) return dfail(MR_EINVAL, "image too large");
    if (ws_bytes < L.total)
        return dfail(MR_ENOMEM, "workspace too small: %zu bytes given, %zu needed", ws_bytes,
                     L.total);
    hipStream_t s = (hipStream_t)stream;
    DtCtrl *ctrl = (DtCtrl *)((char *)ws + L.ctrl);
    uint32_t *flags = (uint32_t *)((char *)ws + L.flags);
    uint32_t *lists = (uint32_t *)((char *)ws + L.lists);
    const uint8_t *im = (const uint8_t *)img;
    int32_t *d = (int32_t *)dist;
    const int64_t n = L.ntx * L.nty;
    hipLaunchKernelGGL(k_dt_clear, dim3((unsigned)std::min<int64_t>((n + 255) / 256 + 1, 4096)),
                       dim3(256), 0, s, ctrl, flags, n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return dhip(e, "clear");
    // round 1 builds every tile from the image; later rounds visit the tiles
    // marked for them, DT_BATCH rounds per host poll of the marks
    uint32_t round = 1;
    if ((e = dt_round(conn, true, im, pitch, d, dist_pitch, H, W, L, flags, lists, round, ctrl, s)) !=
        hipSuccess)
        return dhip(e, "round");
    uint32_t h_marked = 0, h_has_bg = 0;
    while (true) {
        // tiles the last round marked for the next one (counted in the slot
        // of that round's parity)
        if ((e = hipMemcpyAsync(&h_marked, &ctrl->marked[(round + 1) & 1], 4,
                                hipMemcpyDeviceToHost, s)) != hipSuccess ||
            (e = hipMemcpyAsync(&h_has_bg, &ctrl->has_bg, 4, hipMemcpyDeviceToHost, s)) !=
                hipSuccess ||
            (e = hipStreamSynchronize(s)) != hipSuccess)
            return dhip(e, "poll");
        if (h_marked == 0) break;
        if ((int64_t)round > DT_MAX_ROUNDS)
            return dfail(MR_EHIP, "distance transform did not converge");
        // the next DT_BATCH rounds; a round that finds no tile marked for it
        // changes nothing, so a batch that overshoots the end is harmless
        for (int k = 0; k < DT_BATCH; ++k) {
            ++round;
            // the slot that will count this round's marks held round - 1's
            hipLaunchKernelGGL(k_dt_reset_mark, dim3(1), dim3(1), 0, s, ctrl, (round + 1) & 1);
            if ((e = dt_round(conn, false, im, pitch, d, dist_pitch, H, W, L, flags, lists, round,
                              ctrl, s)) != hipSuccess)
                return dhip(e, "round");
        }
    }
    if (!h_has_bg) {
        const int64_t items = H * W;
        hipLaunchKernelGGL(k_dt_fill, dim3((unsigned)std::min<int64_t>((items + 255) / 256, 65536)),
                           dim3(256), 0, s, d, dist_pitch, H, W, -1);
        if ((e = hipGetLastError()) != hipSuccess) return dhip(e, "fill");
    }
    return MR_OK;
}

} // extern "C"
