// mr_ccl.hip -- connected components labeling (union-find) and area threshold
// (map + reduction), Table II; mr_ccl and mr_area_threshold in
// include/mr_ops.h.
//
// Union-find as Sec. II-B describes it: every foreground pixel starts as its
// own tree, trees of adjacent foreground pixels are merged with the smaller
// root becoming the root of the merged tree, and the labels are read from
// the flattened forest. Here a pixel's value in the forest is its linear
// index y * W + x, so every root is the smallest index of its tree and the
// labels (root + 1) do not depend on the order of the merges.
//
// The GPU version follows Sec. III-B's split: each 32 x 64 tile is merged by
// one workgroup in LDS with LDS atomics (k_ccl_local), then the trees that
// cross tile borders are merged in the global forest with device atomics
// (k_ccl_merge), and finally every pixel follows its tree to the root
// (k_ccl_flatten). The global forest holds parent index + 1 per pixel and 0
// for the background, so a root's entry is its label: with unit-pitch label
// rows the label plane itself is the forest, flattened in place (a pixel
// whose entry becomes its root's label still points at that root), and the
// background is written once. A merge links the larger of two roots below the smaller
// with an atomic minimum on the larger's parent; if another merge got there
// first, the atomic returns the new parent and the merge goes on from it.
// Parents only ever decrease and stay below their children, so every walk
// ends at a root.
//
// Area threshold: the map step reads each pixel's label; the reduction counts
// pixels per label with device atomic adds into one counter per possible
// label (the workspace), adding a lane's run of equal labels in one atomic;
// the filter clears every pixel whose label's count is out of range.
#include <algorithm>
#include <cstdarg>
#include <cstdio>

#include "../../include/mr_ops.h"
#include "mr_internal.h"

using namespace mr;

namespace {

int cfail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    return set_error(code, buf);
}

int chip(hipError_t e, const char *what) {
    return cfail(MR_EHIP, "%s: %s", what, hipGetErrorString(e));
}

size_t up256(size_t n) { return (n + 255) / 256 * 256; }

constexpr int CT_H = 32, CT_W = 64;     // tile of the local phase
constexpr int CT_N = CT_H * CT_W;
constexpr int CT_THREADS = 256;         // 8 pixels per lane
constexpr uint32_t NONE = 0xFFFFFFFFu;  // background in the tile's LDS forest

// ------------------------------------------------------------- local phase

__device__ __forceinline__ uint32_t lds_load(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ uint32_t lfind(const uint32_t *P, uint32_t x) {
    uint32_t p = lds_load(P + x);
    while (p != x) {
        x = p;
        p = lds_load(P + x);
    }
    return x;
}

// Merge the trees of a and b in the tile's LDS forest: the larger root goes
// below the smaller one.
__device__ __forceinline__ void lunion(uint32_t *P, uint32_t a, uint32_t b) {
    while (true) {
        a = lfind(P, a);
        b = lfind(P, b);
        if (a == b) return;
        if (a > b) {
            const uint32_t t = a;
            a = b;
            b = t;
        }
        const uint32_t old = atomicMin(P + b, a);
        if (old == b) return; // b was still a root: linked
        b = old;              // b was linked meanwhile: go on from its parent
    }
}

// One wave holds one tile row per step (lane = column), so a ballot is the
// row's foreground mask. A pixel starts pointing at the first pixel of its
// horizontal run, which links every run without an atomic. A run then needs
// one union per run above it that it touches, made at the first of its
// pixels that reaches that run: with 4-connectivity a pixel whose
// above-neighbour is foreground unless its left neighbour (in the same run)
// reached the same above run through the column before; with 8-connectivity
// a run's first pixel takes each run among its three above-neighbours, and
// every later pixel only the column it adds on the right.
template <int CONN>
__global__ __launch_bounds__(CT_THREADS) void k_ccl_local(const uint8_t *__restrict__ img,
                                                          int64_t H, int64_t W, int64_t pitch,
                                                          int64_t tiles_x,
                                                          uint32_t *__restrict__ forest) {
    __shared__ uint32_t P[CT_N];
    __shared__ uint64_t rowfg[CT_H];
    static_assert(CT_W == 64 && CT_THREADS % 64 == 0, "a wave holds one tile row");
    const int64_t ty = blockIdx.x / tiles_x, tx = blockIdx.x - ty * tiles_x;
    const int64_t y0 = ty * CT_H, x0 = tx * CT_W;
    const int lx = threadIdx.x & (CT_W - 1), ly0 = threadIdx.x / CT_W;
    constexpr int RSTEP = CT_THREADS / CT_W; // rows between a lane's pixels
    const uint64_t below = (1ull << lx) - 1; // lanes left of this one
    bool fg[CT_H / RSTEP];
#pragma unroll
    for (int k = 0; k < CT_H / RSTEP; ++k) {
        const int ly = ly0 + k * RSTEP;
        const int64_t y = y0 + ly, x = x0 + lx;
        // (a clamped, unconditional load: loads under a branch are waited
        // for one at a time)
        const uint8_t px = img[(y < H ? y : H - 1) * pitch + (x < W ? x : W - 1)];
        fg[k] = y < H && x < W && px != 0;
        const uint64_t m = __ballot(fg[k]);
        // the run starts after the last background pixel to the left
        const uint64_t z = ~m & below;
        const int start = z ? 64 - __builtin_clzll(z) : 0;
        P[ly * CT_W + lx] = fg[k] ? (uint32_t)(ly * CT_W + start) : NONE;
        if (lx == 0) rowfg[ly] = m;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < CT_H / RSTEP; ++k) {
        const int ly = ly0 + k * RSTEP;
        if (!fg[k] || ly == 0) continue;
        const uint64_t m = rowfg[ly], up = rowfg[ly - 1];
        const uint32_t p = ly * CT_W + lx;
        const bool left = lx > 0 && ((m >> (lx - 1)) & 1);
        const bool aL = lx > 0 && ((up >> (lx - 1)) & 1);
        const bool aC = (up >> lx) & 1;
        const bool aR = lx < CT_W - 1 && ((up >> (lx + 1)) & 1);
        if (CONN == 4) {
            if (aC && !(left && aL)) lunion(P, p, p - CT_W);
        } else {
            if (!left) {
                if (aL) lunion(P, p, p - CT_W - 1);
                if (aC && !aL) lunion(P, p, p - CT_W);
            }
            if (aR && !aC) lunion(P, p, p - CT_W + 1);
        }
    }
    __syncthreads();
    // every run's first pixel takes its root (only first pixels were ever
    // linked, so the other pixels of a run still point at it)
#pragma unroll
    for (int k = 0; k < CT_H / RSTEP; ++k) {
        const int ly = ly0 + k * RSTEP;
        const uint32_t p = ly * CT_W + lx;
        if (fg[k] && (lx == 0 || !((rowfg[ly] >> (lx - 1)) & 1))) {
            const uint32_t r = lfind(P, p);
            if (r != p) __hip_atomic_store(P + p, r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    }
    __syncthreads();
    // each pixel points at its tile-local root, as a global linear index
    // (H * W < 2^31, so linear indices are 32-bit)
    const uint32_t W32 = (uint32_t)W;
    const uint32_t tile0 = (uint32_t)(y0 * W + x0); // the tile's first pixel
#pragma unroll
    for (int k = 0; k < CT_H / RSTEP; ++k) {
        const int ly = ly0 + k * RSTEP;
        const int64_t y = y0 + ly, x = x0 + lx;
        if (y >= H || x >= W) continue;
        uint32_t v = 0;
        if (fg[k]) {
            const uint32_t r = P[P[ly * CT_W + lx]];
            v = tile0 + (r / CT_W) * W32 + r % CT_W + 1u;
        }
        forest[tile0 + (uint32_t)ly * W32 + (uint32_t)lx] = v;
    }
}

// ------------------------------------------------------------- border phase

__device__ __forceinline__ uint32_t gload(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root index of x's tree in the global forest (entries: parent index + 1).
__device__ __forceinline__ uint32_t gfind(const uint32_t *F, uint32_t x) {
    uint32_t p = gload(F + x) - 1u;
    while (p != x) {
        x = p;
        p = gload(F + x) - 1u;
    }
    return x;
}

__device__ __forceinline__ void gunion(uint32_t *F, uint32_t a, uint32_t b) {
    while (true) {
        a = gfind(F, a);
        b = gfind(F, b);
        if (a == b) return;
        if (a > b) {
            const uint32_t t = a;
            a = b;
            b = t;
        }
        const uint32_t old =
            __hip_atomic_fetch_min(F + b, a + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - 1u;
        if (old == b) return;
        b = old;
    }
}

// Pixels of a tile whose backward neighbours lie in another tile: the first
// row (up, and the diagonals), the first column (left, up-left) and, with
// 8-connectivity, the last column (up-right). One workgroup per tile, one
// lane per border pixel.
template <int CONN>
__global__ __launch_bounds__(128) void k_ccl_merge(int64_t H, int64_t W, int64_t tiles_x,
                                                   uint32_t *__restrict__ F) {
    const int64_t ty = blockIdx.x / tiles_x, tx = blockIdx.x - ty * tiles_x;
    const int64_t y0 = ty * CT_H, x0 = tx * CT_W;
    const int i = threadIdx.x;
    int64_t y, x;
    if (i < CT_W) { // first row
        y = y0;
        x = x0 + i;
    } else if (i < CT_W + CT_H) { // first column (its top pixel is in the row)
        y = y0 + (i - CT_W);
        x = x0;
        if (i == CT_W) return;
    } else if (i < CT_W + 2 * CT_H) { // last column, below the first row
        y = y0 + (i - CT_W - CT_H);
        x = x0 + CT_W - 1;
        if (CONN != 8 || i == CT_W + CT_H) return;
    } else {
        return;
    }
    if (y >= H || x >= W) return;
    const uint32_t p = (uint32_t)(y * W + x);
    if (gload(F + p) == 0u) return;
    const bool first_row = y == y0, first_col = x == x0, last_col = x == x0 + CT_W - 1;
    const uint32_t Wu = (uint32_t)W;
    // backward neighbours in another tile
    if (first_col && x > 0 && gload(F + p - 1) != 0u) gunion(F, p, p - 1);
    if (first_row && y > 0) {
        // The row above is the last row of the tiles above, whose adjacent
        // foreground pixels within one tile the local phase connected; a
        // left neighbour in this tile's row is in this pixel's local tree.
        // So, as in the local phase, a run of this row needs one union per
        // run above it that it touches (runs above that straddle a tile
        // border are joined by the column rules of the tiles above).
        const bool aC = gload(F + p - Wu) != 0u;
        const bool aL = x > 0 && gload(F + p - Wu - 1) != 0u;
        const bool aR = x + 1 < W && gload(F + p - Wu + 1) != 0u;
        const bool left = x > x0 && gload(F + p - 1) != 0u;
        if (CONN == 4) {
            if (aC && !(left && aL)) gunion(F, p, p - Wu);
        } else {
            if (!left) {
                if (aL) gunion(F, p, p - Wu - 1);
                if (aC && !aL) gunion(F, p, p - Wu);
            }
            if (aR && !aC) gunion(F, p, p - Wu + 1);
        }
    } else if (CONN == 8 && y > 0) {
        if (first_col && x > 0 && gload(F + p - Wu - 1) != 0u) gunion(F, p, p - Wu - 1);
        if (last_col && x + 1 < W && gload(F + p - Wu + 1) != 0u) gunion(F, p, p - Wu + 1);
    }
}

// ----------------------------------------------------------- flatten, write

// A grid-stride walk over the H x W pixels of a pitched image in linear
// order: (y, x) of this lane's pixel, advanced by the grid's stride without
// a division per pixel (H * W < 2^31).
struct PixelWalk {
    uint32_t i, y, x, dy, dx, n, W;
    __device__ PixelWalk(int64_t H, int64_t Wd, uint32_t first, uint32_t stride) {
        W = (uint32_t)Wd;
        n = (uint32_t)(H * Wd);
        i = first;
        y = first / W;
        x = first - y * W;
        dy = stride / W;
        dx = stride - dy * W;
    }
    __device__ bool ok() const { return i < n; }
    __device__ void next(uint32_t stride) {
        i += stride;
        y += dy;
        x += dx;
        if (x >= W) {
            x -= W;
            ++y;
        }
    }
};

// IN_PLACE: F is the label plane (unit-pitch rows); background entries are
// already 0 and only foreground pixels are rewritten, each to its root's
// entry (its label). Otherwise every pixel's label goes to `labels`.
template <bool IN_PLACE>
__global__ __launch_bounds__(256) void k_ccl_flatten(int64_t H, int64_t W, uint32_t *F,
                                                     int32_t *labels, int64_t lpitch) {
    const uint32_t stride = gridDim.x * 256u;
    for (PixelWalk w(H, W, blockIdx.x * 256u + threadIdx.x, stride); w.ok(); w.next(stride)) {
        const uint32_t v = gload(F + w.i);
        if (IN_PLACE) {
            if (v != 0u)
                __hip_atomic_store(F + w.i, gfind(F, v - 1u) + 1u, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        } else {
            labels[(int64_t)w.y * lpitch + w.x] = v != 0u ? (int32_t)(gfind(F, v - 1u) + 1u) : 0;
        }
    }
}

// In place on a plane of whole 16-byte words (H * W a multiple of 4,
// 16-byte aligned): a lane takes 4 entries, walks each foreground one to its
// root, and writes the word back only if an entry changed. A reader of an
// entry that another lane rewrites finds either its old parent or its root,
// and both lead to the same root.
__global__ __launch_bounds__(256) void k_ccl_flatten4(int64_t n4, uint32_t *F) {
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n4; i += (int64_t)gridDim.x * 256) {
        const uint4 v = ((const uint4 *)F)[i];
        const uint4 o = {v.x ? gfind(F, v.x - 1u) + 1u : 0u, v.y ? gfind(F, v.y - 1u) + 1u : 0u,
                         v.z ? gfind(F, v.z - 1u) + 1u : 0u, v.w ? gfind(F, v.w - 1u) + 1u : 0u};
        if (o.x != v.x || o.y != v.y || o.z != v.z || o.w != v.w) ((uint4 *)F)[i] = o;
    }
}

// --------------------------------------------------------------- area phase

__global__ __launch_bounds__(256) void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * 256)
        p[i] = v;
}

// Count pixels per label: a wave reads 64 consecutive pixels of the image in
// linear order (one per lane, coalesced); a lane whose label differs from
// the previous pixel's (or that starts a row or the wave's chunk) heads a
// run, and adds the run's length, up to the next head, with one atomic.
// Background (0) and out-of-range labels are not counted. A run that spans
// two chunks is added in two parts.
__global__ __launch_bounds__(256) void k_area_count(const int32_t *__restrict__ labels,
                                                    int64_t H, int64_t W, int64_t pitch,
                                                    int32_t *__restrict__ area) {
    const uint32_t N = (uint32_t)(H * W);
    const int lane = threadIdx.x & 63;
    const uint32_t wave = blockIdx.x * 4u + (threadIdx.x >> 6), waves = gridDim.x * 4u;
    const uint32_t stride = waves * 64u;
    // every lane of a wave stays in the loop while its chunk has pixels, so
    // the cross-lane steps below see the whole wave
    for (PixelWalk w(H, W, wave * 64u + lane, stride); w.i - lane < N; w.next(stride)) {
        const bool in = w.ok();
        const int32_t l = in ? labels[(int64_t)w.y * pitch + w.x] : 0;
        const int32_t prev = __shfl_up(l, 1);
        const bool head = in && (lane == 0 || w.x == 0 || l != prev);
        const uint64_t heads = __ballot(head);
        const uint64_t valid = __ballot(in);
        if (head && l > 0 && (uint32_t)l <= N) {
            const uint64_t later = lane == 63 ? 0ull : (heads >> (lane + 1)) << (lane + 1);
            const int end = later ? __builtin_ctzll(later) : 64 - __builtin_clzll(valid);
            atomicAdd(area + l, end - lane);
        }
    }
}

// The same count on rows of whole 16-byte words (W and pitch multiples of 4,
// 16-byte aligned plane): a lane takes 4 labels, a wave's chunk is 64 words.
// Run heads are marked per label; a head's run ends at the next head in its
// lane, else at the first head of the next lane that has one, else at the
// chunk's end.
__global__ __launch_bounds__(256) void k_area_count4(const int32_t *__restrict__ labels,
                                                     int64_t H, int64_t W, int64_t pitch,
                                                     int32_t *__restrict__ area) {
    const uint32_t N = (uint32_t)(H * W), NQ = (uint32_t)(H * (W / 4));
    const int lane = threadIdx.x & 63;
    const uint32_t wave = blockIdx.x * 4u + (threadIdx.x >> 6), waves = gridDim.x * 4u;
    const uint32_t stride = waves * 64u;
    for (PixelWalk w(H, W / 4, wave * 64u + lane, stride); w.i - lane < NQ; w.next(stride)) {
        const bool in = w.ok();
        int4 q = {0, 0, 0, 0};
        if (in) q = *(const int4 *)(labels + (int64_t)w.y * pitch + 4 * (int64_t)w.x);
        const int32_t prev = __shfl_up(q.w, 1);
        uint32_t hm = 0; // bit j: label j of this lane starts a run
        if (in) {
            hm = (lane == 0 || w.x == 0 || q.x != prev) ? 1u : 0u;
            hm |= (q.y != q.x ? 2u : 0u) | (q.z != q.y ? 4u : 0u) | (q.w != q.z ? 8u : 0u);
        }
        const int first = hm ? __builtin_ctz(hm) : 4;
        const uint64_t with_head = __ballot(hm != 0);
        const uint64_t valid = __ballot(in);
        const uint64_t later = lane == 63 ? 0ull : (with_head >> (lane + 1)) << (lane + 1);
        const int ln = later ? __builtin_ctzll(later) : lane;
        const int fn = __shfl(first, ln);
        const int next = later ? 4 * ln + fn : 4 * (64 - __builtin_clzll(valid));
        const int32_t lv[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (!((hm >> j) & 1u)) continue;
            const uint32_t rest = hm >> (j + 1);
            const int end = rest ? 4 * lane + j + 1 + __builtin_ctz(rest) : next;
            if (lv[j] > 0 && (uint32_t)lv[j] <= N) atomicAdd(area + lv[j], end - (4 * lane + j));
        }
    }
}

__global__ __launch_bounds__(256) void k_area_filter(int32_t *__restrict__ labels, int64_t H,
                                                     int64_t W, int64_t pitch,
                                                     const int32_t *__restrict__ area,
                                                     int64_t lo, int64_t hi) {
    const int64_t N = H * W;
    const uint32_t stride = gridDim.x * 256u;
    for (PixelWalk w(H, W, blockIdx.x * 256u + threadIdx.x, stride); w.ok(); w.next(stride)) {
        int32_t *p = labels + (int64_t)w.y * pitch + w.x;
        const int32_t l = *p;
        if (l > 0 && (int64_t)l <= N) {
            const int64_t a = area[l];
            if (a < lo || a > hi) *p = 0;
        }
    }
}

// The same on rows of whole 16-byte words (W and pitch multiples of 4,
// 16-byte aligned plane): a lane takes 4 labels at once, so their 4 counter
// reads are in flight together, and writes the word back only if it cleared
// one of them.
__global__ __launch_bounds__(256) void k_area_filter4(int32_t *__restrict__ labels, int64_t H,
                                                      int64_t W, int64_t pitch,
                                                      const int32_t *__restrict__ area,
                                                      int64_t lo, int64_t hi) {
    const int64_t N = H * W;
    const uint32_t stride = gridDim.x * 256u;
    auto keep = [&](int32_t l) -> int32_t {
        if (l <= 0 || (int64_t)l > N) return l;
        const int64_t a = area[l];
        return a < lo || a > hi ? 0 : l;
    };
    for (PixelWalk w(H, W / 4, blockIdx.x * 256u + threadIdx.x, stride); w.ok(); w.next(stride)) {
        int4 *p = (int4 *)(labels + (int64_t)w.y * pitch + 4 * (int64_t)w.x);
        const int4 l = *p;
        const int4 o = {keep(l.x), keep(l.y), keep(l.z), keep(l.w)};
        if (o.x != l.x || o.y != l.y || o.z != l.z || o.w != l.w) *p = o;
    }
}

unsigned grid_for(int64_t items) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((items + 255) / 256, 1 << 16));
}

int check_labels_dims(int64_t H, int64_t W, int64_t pitch) {
    if (H < 1 || W < 1) return cfail(MR_EINVAL, "H and W must be >= 1");
    if (pitch < W) return cfail(MR_EINVAL, "pitch below W");
    if (H * W >= (1ll << 31) - 1) return cfail(MR_EINVAL, "H * W must be below 2^31 - 1");
    return MR_OK;
}

} // namespace

extern "C" {

size_t mr_ccl_workspace_bytes(int64_t H, int64_t W) {
    clear_error();
    if (check_labels_dims(H, W, W) != MR_OK) return 0;
    return up256((size_t)(H * W) * 4);
}

int mr_ccl(const void *img, void *labels, int64_t H, int64_t W, int64_t pitch,
           int64_t label_pitch, int conn, void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    if (pitch == 0) pitch = W;
    if (label_pitch == 0) label_pitch = W;
    int rc;
    if ((rc = check_labels_dims(H, W, pitch)) != MR_OK) return rc;
    if (label_pitch < W) return cfail(MR_EINVAL, "label_pitch below W");
    if (conn != 4 && conn != 8) return cfail(MR_EINVAL, "conn must be 4 or 8 (got %d)", conn);
    if (!img || !labels || !ws) return cfail(MR_EINVAL, "null pointer");
    if ((uintptr_t)labels % 4) return cfail(MR_EINVAL, "labels must be 4-byte aligned");
    if ((uintptr_t)ws % 256) return cfail(MR_EINVAL, "workspace must be 256-byte aligned");
    const size_t need = up256((size_t)(H * W) * 4);
    if (ws_bytes < need)
        return cfail(MR_ENOMEM, "workspace too small: %zu bytes given, %zu needed", ws_bytes, need);
    hipStream_t s = (hipStream_t)stream;
    // unit-pitch label rows: the label plane is the forest
    const bool in_place = label_pitch == W;
    uint32_t *F = in_place ? (uint32_t *)labels : (uint32_t *)ws;
    const int64_t tx = (W + CT_W - 1) / CT_W, ty = (H + CT_H - 1) / CT_H;
    const unsigned tiles = (unsigned)(tx * ty);
    if (conn == 8) {
        hipLaunchKernelGGL(k_ccl_local<8>, dim3(tiles), dim3(CT_THREADS), 0, s,
                           (const uint8_t *)img, H, W, pitch, tx, F);
        hipLaunchKernelGGL(k_ccl_merge<8>, dim3(tiles), dim3(128), 0, s, H, W, tx, F);
    } else {
        hipLaunchKernelGGL(k_ccl_local<4>, dim3(tiles), dim3(CT_THREADS), 0, s,
                           (const uint8_t *)img, H, W, pitch, tx, F);
        hipLaunchKernelGGL(k_ccl_merge<4>, dim3(tiles), dim3(128), 0, s, H, W, tx, F);
    }
    if (in_place && (H * W) % 4 == 0 && (uintptr_t)labels % 16 == 0)
        hipLaunchKernelGGL(k_ccl_flatten4, dim3(grid_for(H * W / 4)), dim3(256), 0, s,
                           H * W / 4, F);
    else if (in_place)
        hipLaunchKernelGGL(k_ccl_flatten<true>, dim3(grid_for(H * W)), dim3(256), 0, s, H, W, F,
                           (int32_t *)labels, label_pitch);
    else
        hipLaunchKernelGGL(k_ccl_flatten<false>, dim3(grid_for(H * W)), dim3(256), 0, s, H, W, F,
                           (int32_t *)labels, label_pitch);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? MR_OK : chip(e, "ccl");
}

size_t mr_area_threshold_workspace_bytes(int64_t H, int64_t W) {
    clear_error();
    if (check_labels_dims(H, W, W) != MR_OK) return 0;
    return up256((size_t)(H * W + 1) * 4);
}

int mr_area_threshold(void *labels_inout, int64_t H, int64_t W, int64_t pitch, int64_t min_area,
                      int64_t max_area, void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    if (pitch == 0) pitch = W;
    int rc;
    if ((rc = check_labels_dims(H, W, pitch)) != MR_OK) return rc;
    if (!labels_inout || !ws) return cfail(MR_EINVAL, "null pointer");
    if ((uintptr_t)labels_inout % 4) return cfail(MR_EINVAL, "labels must be 4-byte aligned");
    if ((uintptr_t)ws % 256) return cfail(MR_EINVAL, "workspace must be 256-byte aligned");
    const size_t need = up256((size_t)(H * W + 1) * 4);
    if (ws_bytes < need)
        return cfail(MR_ENOMEM, "workspace too small: %zu bytes given, %zu needed", ws_bytes, need);
    hipStream_t s = (hipStream_t)stream;
    int32_t *area = (int32_t *)ws;
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(H * W + 1)), dim3(256), 0, s, area, H * W + 1, 0);
    if (W % 4 == 0 && pitch % 4 == 0 && (uintptr_t)labels_inout % 16 == 0) {
        hipLaunchKernelGGL(k_area_count4, dim3(grid_for(H * W / 4)), dim3(256), 0, s,
                           (const int32_t *)labels_inout, H, W, pitch, area);
        hipLaunchKernelGGL(k_area_filter4, dim3(grid_for(H * W / 4)), dim3(256), 0, s,
                           (int32_t *)labels_inout, H, W, pitch, (const int32_t *)area, min_area,
                           max_area);
    } else {
        hipLaunchKernelGGL(k_area_count, dim3(grid_for(H * W)), dim3(256), 0, s,
                           (const int32_t *)labels_inout, H, W, pitch, area);
        hipLaunchKernelGGL(k_area_filter, dim3(grid_for(H * W)), dim3(256), 0, s,
                           (int32_t *)labels_inout, H, W, pitch, (const int32_t *)area,
                           min_area, max_area);
    }
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? MR_OK : chip(e, "area threshold");
}

} // extern "C"
