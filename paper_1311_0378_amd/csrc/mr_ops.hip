// mr_ops.hip -- the regular operations of Table II and the reconstruction-based
// wrappers (include/mr_ops.h): h-dome, regional maxima, RGB to grayscale and
// opening by a 13 x 13 disk.
//
// All of these are streaming passes over HBM (Sec. V-C.1's regular,
// memory-bound class) except the reconstruction inside the wrappers, which
// runs on the engine of mr.h.
#include <algorithm>
#include <cstdarg>
#include <cstdio>

#include "../../include/mr_ops.h"
#include "mr_internal.h"

using namespace mr;

namespace {

int ofail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    return set_error(code, buf);
}

int ohip(hipError_t e, const char *what) {
    return ofail(MR_EHIP, "%s: %s", what, hipGetErrorString(e));
}

size_t up256(size_t n) { return (n + 255) / 256 * 256; }

int check_dims(int64_t H, int64_t W, int64_t pitch, int64_t elem_bytes) {
    if (H < 1 || W < 1) return ofail(MR_EINVAL, "H and W must be >= 1 (got %lld x %lld)",
                                     (long long)H, (long long)W);
    if (pitch < W) return ofail(MR_EINVAL, "pitch %lld is below W %lld", (long long)pitch,
                                (long long)W);
    if ((double)H * (double)pitch * (double)elem_bytes >= 9.0e18)
        return ofail(MR_EINVAL, "image too large");
    return MR_OK;
}

unsigned grid_for(int64_t items, int per_block) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((items + per_block - 1) / per_block,
                                                            1 << 20));
}

// ------------------------------------------------------ h-dome, regional max

// Pixel keys of the two types (the key order is the pixel order; key 0 is
// the type's minimum).
template <typename T> struct K;
template <> struct K<uint8_t> {
    __device__ static uint32_t key(uint8_t v) { return v; }
    __device__ static uint8_t val(uint32_t k) { return (uint8_t)k; }
};
template <> struct K<int32_t> {
    __device__ static uint32_t key(int32_t v) { return (uint32_t)v ^ 0x80000000u; }
    __device__ static int32_t val(uint32_t k) { return (int32_t)(k ^ 0x80000000u); }
};

// The streaming passes of the wrappers, one kind each:
//  P_MARKER: m = f - h, saturating at the type's minimum (in key space: key -
//            h floored at 0); *above |= 1 if some pixel is above the minimum;
//  P_DOME:   f <- f - r (the h-dome; r <= f everywhere, so 0 <= f - r <= h);
//  P_RMAX:   out = 255 where f > r (a dome of height 1), or everywhere when
//            no pixel is above the minimum (*above == 0); else 0.
// With WORDS every lane takes one 16-byte word of a row (planes whose base
// and pitch are multiples of 16 bytes; the u8 output of P_RMAX likewise, in
// 16 / sizeof(T)-byte pieces), else one pixel. A row's last word may be
// partial and goes pixel by pixel. Grid-stride over a grid of at most
// MAX_STREAM_BLOCKS blocks.
enum { P_MARKER = 0, P_DOME = 1, P_RMAX = 2 };
constexpr int64_t MAX_STREAM_BLOCKS = 4096;

template <typename T> struct alignas(16) Word {
    T e[16 / sizeof(T)];
};

template <typename T, int KIND>
__device__ __forceinline__ void pass_pixel(const T *f, const T *r, T *m, uint8_t *o, uint32_t h,
                                           bool all_min, bool &any, int64_t i, int64_t oi) {
    const uint32_t kf = K<T>::key(f[i]);
    if (KIND == P_MARKER) {
        any |= kf != 0;
        m[i] = K<T>::val(kf > h ? kf - h : 0u);
    } else if (KIND == P_DOME) {
        m[i] = (T)(int32_t)(kf - K<T>::key(r[i])); // m aliases f here
    } else {
        o[oi] = (all_min || kf > K<T>::key(r[i])) ? 255 : 0;
    }
}

// 0xFF in every byte of x that is nonzero, 0 in the others: the low seven
// bits of a byte plus 0x7F carry into its top bit iff they are nonzero, and
// the byte's own top bit covers the rest; no carry leaves a byte.
__device__ __forceinline__ uint32_t bytes_nonzero(uint32_t x) {
    const uint32_t top = (((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x) & 0x80808080u;
    return (top >> 7) * 0xFFu;
}

template <typename T, int KIND, bool WORDS>
__global__ __launch_bounds__(256) void k_stream_pass(const T *f, const T *r, T *m,
                                                     uint8_t *__restrict__ o, int64_t H,
                                                     int64_t W, int64_t pitch, int64_t out_pitch,
                                                     uint32_t h, uint32_t *above) {
    constexpr int EPW = WORDS ? 16 / (int)sizeof(T) : 1;
    const int64_t wpr = (W + EPW - 1) / EPW; // items per row
    const bool all_min = KIND == P_RMAX && *above == 0;
    bool any = false;
    for (int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; it < H * wpr;
         it += (int64_t)gridDim.x * blockDim.x) {
        const int64_t y = it / wpr, x0 = (it - y * wpr) * EPW;
        const int64_t i0 = y * pitch + x0, o0 = y * out_pitch + x0;
        if (WORDS && sizeof(T) == 1 && KIND != P_MARKER && x0 + EPW <= W) {
            // uint8 dome and maxima on whole dwords: r <= f in every byte, so
            // f - r as 32-bit words subtracts byte by byte without borrows
            const uint4 wf = *(const uint4 *)(f + i0), wr = *(const uint4 *)(r + i0);
            uint4 d = {wf.x - wr.x, wf.y - wr.y, wf.z - wr.z, wf.w - wr.w};
            if (KIND == P_DOME) {
                *(uint4 *)(m + i0) = d;
            } else {
                *(uint4 *)(o + o0) = all_min ? uint4{~0u, ~0u, ~0u, ~0u}
                                             : uint4{bytes_nonzero(d.x), bytes_nonzero(d.y),
                                                     bytes_nonzero(d.z), bytes_nonzero(d.w)};
            }
        } else if (WORDS && x0 + EPW <= W) {
            const Word<T> wf = *(const Word<T> *)(f + i0);
            if (KIND == P_MARKER) {
                Word<T> wm;
#pragma unroll
                for (int e = 0; e < EPW; ++e) {
                    const uint32_t kf = K<T>::key(wf.e[e]);
                    any |= kf != 0;
                    wm.e[e] = K<T>::val(kf > h ? kf - h : 0u);
                }
                *(Word<T> *)(m + i0) = wm;
            } else {
                const Word<T> wr = *(const Word<T> *)(r + i0);
                if (KIND == P_DOME) {
                    Word<T> wm;
#pragma unroll
                    for (int e = 0; e < EPW; ++e)
                        wm.e[e] = (T)(int32_t)(K<T>::key(wf.e[e]) - K<T>::key(wr.e[e]));
                    *(Word<T> *)(m + i0) = wm;
                } else {
                    uint8_t ob[EPW];
#pragma unroll
                    for (int e = 0; e < EPW; ++e)
                        ob[e] = (all_min || K<T>::key(wf.e[e]) > K<T>::key(wr.e[e])) ? 255 : 0;
                    if (EPW == 16) {
                        *(Word<uint8_t> *)(o + o0) = *(const Word<uint8_t> *)ob;
                    } else {
                        uint32_t v = 0;
#pragma unroll
                        for (int e = 0; e < EPW; ++e) v |= (uint32_t)ob[e] << (8 * e);
                        *(uint32_t *)(o + o0) = v;
                    }
                }
            }
        } else {
            for (int e = 0; e < EPW && x0 + e < W; ++e)
                pass_pixel<T, KIND>(f, r, m, o, h, all_min, any, i0 + e, o0 + e);
        }
    }
    // one atomic per wave at most, and none once some wave has set the flag
    if (KIND == P_MARKER && __ballot(any) != 0 && (threadIdx.x & 63) == 0 &&
        __hip_atomic_load(above, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
        atomicOr(above, 1u);
}

bool words_ok(const void *p, int64_t pitch_bytes) {
    return ((uintptr_t)p & 15) == 0 && (pitch_bytes & 15) == 0;
}

template <typename T, int KIND>
hipError_t stream_pass(const T *f, const T *r, T *m, uint8_t *o, int64_t H, int64_t W,
                       int64_t pitch, int64_t out_pitch, uint32_t h, uint32_t *above,
                       hipStream_t s) {
    const int64_t pb = pitch * (int64_t)sizeof(T);
    bool words = words_ok(f, pb) && (KIND == P_MARKER || words_ok(r, pb)) &&
                 (KIND == P_RMAX || words_ok(m, pb));
    if (KIND == P_RMAX)
        words = words && ((uintptr_t)o % (16 / sizeof(T))) == 0 &&
                out_pitch % (int64_t)(16 / sizeof(T)) == 0;
    const int64_t epw = words ? 16 / (int64_t)sizeof(T) : 1;
    const int64_t items = H * ((W + epw - 1) / epw);
    const unsigned g =
        (unsigned)std::max<int64_t>(1, std::min<int64_t>((items + 255) / 256, MAX_STREAM_BLOCKS));
    if (words)
        hipLaunchKernelGGL((k_stream_pass<T, KIND, true>), dim3(g), dim3(256), 0, s, f, r, m, o,
                           H, W, pitch, out_pitch, h, above);
    else
        hipLaunchKernelGGL((k_stream_pass<T, KIND, false>), dim3(g), dim3(256), 0, s, f, r, m, o,
                           H, W, pitch, out_pitch, h, above);
    return hipGetLastError();
}

__global__ void k_zero_u32(uint32_t *p) { *p = 0u; }

struct HdomeLayout {
    size_t recon = 0, plane = 0, flag = 0, total = 0;
};

int hdome_layout(int64_t H, int64_t W, int64_t pitch, int t, int conn, const mr_tune *tune,
                 HdomeLayout &L) {
    const size_t r = mr_workspace_bytes(MR_OP_RECON, H, W, (mr_dtype)t, conn, tune);
    if (r == 0) return MR_EINVAL; // the message is set
    L.recon = up256(r);
    L.plane = L.recon;
    L.flag = L.plane + up256((size_t)H * (size_t)pitch * (size_t)t);
    L.total = L.flag + 256;
    return MR_OK;
}

int hdome_common(const void *img, int64_t H, int64_t W, int64_t &pitch, int t, int conn,
                 void *ws, size_t ws_bytes, const mr_tune *tune, HdomeLayout &L) {
    clear_error();
    if (t != MR_U8 && t != MR_I32) return ofail(MR_EINVAL, "unknown pixel type %d", t);
    if (pitch == 0) pitch = W;
    int rc;
    if ((rc = check_dims(H, W, pitch, t)) != MR_OK) return rc;
    if (!img || !ws) return ofail(MR_EINVAL, "null image or workspace");
    if ((uintptr_t)ws % 256) return ofail(MR_EINVAL, "workspace must be 256-byte aligned");
    if ((uintptr_t)img % t) return ofail(MR_EINVAL, "image must be aligned to the pixel size");
    if ((rc = hdome_layout(H, W, pitch, t, conn, tune, L)) != MR_OK) return rc;
    if (ws_bytes < L.total)
        return ofail(MR_ENOMEM, "workspace too small: %zu bytes given, %zu needed", ws_bytes,
                     L.total);
    return MR_OK;
}

template <typename T>
hipError_t hdome_marker(const void *f, void *m, int64_t H, int64_t W, int64_t pitch, uint32_t h,
                        uint32_t *flag, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, s, flag);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return stream_pass<T, P_MARKER>((const T *)f, nullptr, (T *)m, nullptr, H, W, pitch, 0, h,
                                    flag, s);
}

// ------------------------------------------------------------------ RGB2Gray

// BT.601 luma weights in 14-bit fixed point (0.299, 0.587, 0.114; sum 2^14)
constexpr uint32_t WR = 4899u, WG = 9617u, WB = 1868u;

__device__ __forceinline__ uint32_t luma(uint32_t r, uint32_t g, uint32_t b) {
    return (WR * r + WG * g + WB * b + 8192u) >> 14;
}

// 16 pixels per lane from three 16-byte words (48 bytes = 16 RGB triples),
// one 16-byte word out. Rows and both planes are 16-byte aligned; vec = the
// whole 16-pixel groups per row.
__global__ __launch_bounds__(256) void k_rgb2gray16(const uint8_t *__restrict__ rgb,
                                                    int64_t rgb_pitch, uint8_t *__restrict__ gray,
                                                    int64_t gray_pitch, int64_t H, int64_t vec) {
    const int64_t items = H * vec;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < items;
         i += (int64_t)gridDim.x * 256) {
        const int64_t y = i / vec, g = i - y * vec;
        const uint4 *src = (const uint4 *)(rgb + y * rgb_pitch + g * 48);
        const uint4 a = src[0], b = src[1], c = src[2];
        const uint32_t w[12] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c.x, c.y, c.z, c.w};
        uint32_t o[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int p = 0; p < 16; ++p) {
            const int q = 3 * p; // byte index of this pixel's R
            const uint32_t r = (w[q >> 2] >> ((q & 3) * 8)) & 0xFFu;
            const uint32_t gg = (w[(q + 1) >> 2] >> (((q + 1) & 3) * 8)) & 0xFFu;
            const uint32_t bb = (w[(q + 2) >> 2] >> (((q + 2) & 3) * 8)) & 0xFFu;
            o[p >> 2] |= luma(r, gg, bb) << ((p & 3) * 8);
        }
        *(uint4 *)(gray + y * gray_pitch + g * 16) = make_uint4(o[0], o[1], o[2], o[3]);
    }
}

// One pixel per lane, for unaligned planes and the columns past the last
// whole 16-pixel group (x0 = first column handled).
__global__ __launch_bounds__(256) void k_rgb2gray1(const uint8_t *__restrict__ rgb,
                                                   int64_t rgb_pitch, uint8_t *__restrict__ gray,
                                                   int64_t gray_pitch, int64_t H, int64_t x0,
                                                   int64_t W) {
    const int64_t cols = W - x0, items = H * cols;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < items;
         i += (int64_t)gridDim.x * 256) {
        const int64_t y = i / cols, x = x0 + (i - y * cols);
        const uint8_t *p = rgb + y * rgb_pitch + 3 * x;
        gray[y * gray_pitch + x] = (uint8_t)luma(p[0], p[1], p[2]);
    }
}

// -------------------------------------------------------- 13 x 13 disk

// The disk of radius 6 as rows: offset dy has half-width HW[|dy|]
// (dy^2 + dx^2 <= 36: 6, 5, 5, 5, 4, 3, 0).
// One wave per workgroup. A wave's 64 lanes cover a window of 256 adjacent
// columns, 4 per lane, and it produces the 240 columns of lanes 2..61 for
// DK_TH rows: an extremum over 13 columns needs 6 columns on each side, and
// lanes 0, 1, 62 and 63 supply them. Per input row each lane loads the one
// dword of its 4 columns, forms the horizontal extrema of half-widths 1, 3,
// 4, 5 and 6 of its own columns, taking the few values it needs of the
// neighbouring lanes' columns by lane shifts (DPP), and folds them into 13
// running accumulators, one per output row that this input row still
// contributes to (the accumulator of the output row dy above gets the
// extremum of half-width HW[|dy|]). Each output row is complete once its
// last input row is folded in, and is stored. Pixels outside the image read
// as the operation's identity (255 for the erosion, 0 for the dilation),
// which leaves the extrema over the inside offsets.
constexpr int DK_OUT = 240;          // output columns per wave (lanes 2..61)
constexpr int DK_TH = 64;           // output rows per wave
constexpr int DK_ROWS = DK_TH + 12;  // input rows per wave

typedef uint16_t u16x2 __attribute__((ext_vector_type(2)));

template <bool MIN> __device__ __forceinline__ uint32_t ext(uint32_t a, uint32_t b) {
    return MIN ? min(a, b) : max(a, b);
}
template <bool MIN> __device__ __forceinline__ uint32_t ext3(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t r;
    if (MIN)
        asm("v_min3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    else
        asm("v_max3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}
// Lane i gets lane i-1's value; lane i gets lane i+1's value. Lanes 0 and 63
// get 0 from the missing neighbour; only columns of lanes 0, 1, 62 and 63
// depend on those values, and they are not stored.
__device__ __forceinline__ uint32_t from_left(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x138 /* wave_shr:1 */, 0xF, 0xF,
                                                 true);
}
__device__ __forceinline__ uint32_t from_right(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x130 /* wave_shl:1 */, 0xF, 0xF,
                                                 true);
}

template <bool MIN>
__global__ __launch_bounds__(64) void k_disk13(const uint8_t *__restrict__ in,
                                               uint8_t *__restrict__ out, int64_t H, int64_t W,
                                               int64_t pitch, int64_t tiles_x) {
    const uint32_t ident = MIN ? 0xFFu : 0u;
    const uint32_t ident4 = MIN ? 0xFFFFFFFFu : 0u;
    const int lane = threadIdx.x;
    const int64_t tile = blockIdx.x;
    const int64_t ty = tile / tiles_x, tx = tile - ty * tiles_x;
    const int64_t y0 = ty * DK_TH;
    const int64_t gx = tx * DK_OUT - 8 + 4 * lane; // this lane's first column
    const bool whole = gx >= 0 && gx + 3 < W;
    // A strip whose 256 columns all lie inside the image, with dword-aligned
    // rows, takes the fast path: a row is one plain dword load per lane from
    // the row's uniform base plus a 32-bit lane offset, with no per-lane
    // branch, so the 13 loads of a step are in flight together. Strips at the
    // image's left and right edges (and unaligned planes) take the general
    // path below.
    const bool fast =
        ((((uintptr_t)in) | ((uintptr_t)out) | (uintptr_t)pitch) & 3) == 0 &&
        W < (1ll << 31) && __ballot(whole) == ~0ull;
    const uint32_t lx4 = (uint32_t)(fast ? gx : 0);
    // input row r of this wave is image row y0 - 6 + r
    auto load = [&](int r) -> uint32_t {
        const int64_t gy = y0 - 6 + r;
        if (gy < 0 || gy >= H) return ident4;
        const uint8_t *p = in + gy * pitch + gx;
        if (whole && (((uintptr_t)p) & 3) == 0) return *(const uint32_t *)p;
        uint32_t v = 0u;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const uint32_t byte = (gx + b >= 0 && gx + b < W) ? p[b] : ident;
            v |= byte << (8 * b);
        }
        return v;
    };

    // 13 accumulators per column in a ring: output row o (wave-relative)
    // lives in slot o mod 13. Input row r reaches output rows r - 12 .. r
    // (offsets dy = 6 .. -6), which sit in slots (r + 1 + k) mod 13,
    // k = 0..12; the rows are walked 13 at a time so that every slot index is
    // a constant. Two columns per accumulator, one in each 16-bit half (the
    // pixels are 8-bit), folded with packed 16-bit extrema.
    const u16x2 identp = {(uint16_t)ident, (uint16_t)ident};
    u16x2 acc[13][2];
#pragma unroll
    for (int k = 0; k < 13; ++k) acc[k][0] = acc[k][1] = identp;
    constexpr int HWID[7] = {6, 5, 5, 5, 4, 3, 0}; // half-width of the disk row |dy|
    const bool stores = lane >= 2 && lane < 62;
#pragma unroll 1
    for (int r0 = 0; r0 < DK_ROWS; r0 += 13) {
        uint32_t wd[13];
        if (fast) {
#pragma unroll
            for (int rr = 0; rr < 13; ++rr) {
                // rows outside the image (and past the strip's last input
                // row) load a clamped row and take the identity instead
                const int64_t gy = y0 - 6 + r0 + rr;
                const int64_t cy = gy < 0 ? 0 : (gy >= H ? H - 1 : gy);
                const uint32_t v = *(const uint32_t *)(in + cy * pitch + lx4);
                wd[rr] = (gy >= 0 && gy < H && r0 + rr < DK_ROWS) ? v : ident4;
            }
        } else {
#pragma unroll
            for (int rr = 0; rr < 13; ++rr) wd[rr] = r0 + rr < DK_ROWS ? load(r0 + rr) : ident4;
        }
#pragma unroll
        for (int rr = 0; rr < 13; ++rr) {
            const int r = r0 + rr;
            if (r >= DK_ROWS) break;
            // e_w[c]: the extremum over columns c - w .. c + w of this lane's
            // column c (0..3); index c + 1 of the arrays below, so that the
            // left neighbour's last column is index 0 and the right
            // neighbour's first is index 5 where a step needs them
            uint32_t b[4];
            b[0] = wd[rr] & 0xFFu;
#pragma unroll
            for (int c = 1; c < 4; ++c) b[c] = __builtin_amdgcn_ubfe(wd[rr], 8 * c, 8);
            uint32_t e1[4], e3[4], e4[4], e5[4], e6[4];
            {
                const uint32_t l = from_left(b[3]), rt = from_right(b[0]);
                e1[0] = ext3<MIN>(l, b[0], b[1]);
                e1[1] = ext3<MIN>(b[0], b[1], b[2]);
                e1[2] = ext3<MIN>(b[1], b[2], b[3]);
                e1[3] = ext3<MIN>(b[2], b[3], rt);
            }
            {
                const uint32_t l2 = from_left(e1[2]), l3 = from_left(e1[3]);
                const uint32_t r0v = from_right(e1[0]), r1v = from_right(e1[1]);
                e3[0] = ext3<MIN>(l2, e1[0], e1[2]);
                e3[1] = ext3<MIN>(l3, e1[1], e1[3]);
                e3[2] = ext3<MIN>(e1[0], e1[2], r0v);
                e3[3] = ext3<MIN>(e1[1], e1[3], r1v);
            }
            {
                const uint32_t l = from_left(e3[3]), rt = from_right(e3[0]);
                e4[0] = ext<MIN>(l, e3[1]);
                e4[1] = ext<MIN>(e3[0], e3[2]);
                e4[2] = ext<MIN>(e3[1], e3[3]);
                e4[3] = ext<MIN>(e3[2], rt);
            }
            {
                const uint32_t l = from_left(e4[3]), rt = from_right(e4[0]);
                e5[0] = ext<MIN>(l, e4[1]);
                e5[1] = ext<MIN>(e4[0], e4[2]);
                e5[2] = ext<MIN>(e4[1], e4[3]);
                e5[3] = ext<MIN>(e4[2], rt);
            }
            {
                const uint32_t l = from_left(e5[3]), rt = from_right(e5[0]);
                e6[0] = ext<MIN>(l, e5[1]);
                e6[1] = ext<MIN>(e5[0], e5[2]);
                e6[2] = ext<MIN>(e5[1], e5[3]);
                e6[3] = ext<MIN>(e5[2], rt);
            }
            // fold into output row r - 12 + k, which lies dy = 6 - k rows above
            // this input row, with the disk row's half-width at |dy|
#pragma unroll
            for (int k = 0; k < 13; ++k) {
                const int ady = k <= 6 ? 6 - k : k - 6;
                const int hw = HWID[ady];
                const int slot = (rr + 1 + k) % 13;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    auto pick = [&](int c) -> uint32_t {
                        return hw == 6 ? e6[c] : hw == 5 ? e5[c] : hw == 4 ? e4[c]
                             : hw == 3 ? e3[c] : b[c];
                    };
                    const u16x2 v = {(uint16_t)pick(2 * h), (uint16_t)pick(2 * h + 1)};
                    acc[slot][h] = MIN ? __builtin_elementwise_min(acc[slot][h], v)
                                       : __builtin_elementwise_max(acc[slot][h], v);
                }
            }
            // output row r - 12 has all 13 of its input rows: store it, and
            // start the slot over for output row r + 1
            const int done = (rr + 1) % 13;
            const int64_t oy = y0 + r - 12;
            if (fast && r >= 12 && oy < H) {
                if (stores)
                    *(uint32_t *)(out + oy * pitch + lx4) = __builtin_amdgcn_perm(
                        __builtin_bit_cast(uint32_t, acc[done][1]),
                        __builtin_bit_cast(uint32_t, acc[done][0]), 0x06040200u);
            } else if (r >= 12 && oy < H && stores && gx < W) {
                uint8_t *orow = out + oy * pitch;
                // the low bytes of the four 16-bit halves, in column order
                const uint32_t o4 = __builtin_amdgcn_perm(__builtin_bit_cast(uint32_t, acc[done][1]),
                                                          __builtin_bit_cast(uint32_t, acc[done][0]),
                                                          0x06040200u);
                if (gx + 3 < W && (((uintptr_t)(orow + gx)) & 3) == 0) {
                    *(uint32_t *)(orow + gx) = o4;
                } else {
#pragma unroll
                    for (int c = 0; c < 4; ++c)
                        if (gx + c < W) orow[gx + c] = (uint8_t)(o4 >> (8 * c));
                }
            }
            acc[done][0] = acc[done][1] = identp;
        }
    }
}

hipError_t launch_disk13(bool erode, const uint8_t *in, uint8_t *out, int64_t H, int64_t W,
                         int64_t pitch, hipStream_t s) {
    const int64_t tx = (W + DK_OUT - 1) / DK_OUT, ty = (H + DK_TH - 1) / DK_TH;
    const int64_t n = tx * ty;
    if (n >= (1ll << 31)) return hipErrorInvalidValue;
    if (erode)
        hipLaunchKernelGGL(k_disk13<true>, dim3((unsigned)n), dim3(64), 0, s, in, out, H, W, pitch,
                           tx);
    else
        hipLaunchKernelGGL(k_disk13<false>, dim3((unsigned)n), dim3(64), 0, s, in, out, H, W,
                           pitch, tx);
    return hipGetLastError();
}

} // namespace

extern "C" {

size_t mr_hdome_workspace_bytes(int64_t H, int64_t W, int64_t pitch, mr_dtype t, int conn,
                                const mr_tune *tune) {
    clear_error();
    if (pitch == 0) pitch = W;
    if (check_dims(H, W, pitch, (int)t) != MR_OK) return 0;
    HdomeLayout L;
    if (hdome_layout(H, W, pitch, (int)t, conn, tune, L) != MR_OK) return 0;
    return L.total;
}

int mr_hdome(void *img_inout, int64_t H, int64_t W, int64_t pitch, mr_dtype t, int conn,
             int64_t h, void *ws, size_t ws_bytes, const mr_tune *tune, void *stream) {
    HdomeLayout L;
    int rc = hdome_common(img_inout, H, W, pitch, (int)t, conn, ws, ws_bytes, tune, L);
    if (rc != MR_OK) return rc;
    if (h < 0) return ofail(MR_EINVAL, "h must be >= 0 (got %lld)", (long long)h);
    // the dome f - R lies in [0, h]: for int32 pixels h must fit the type
    if ((int)t == MR_I32 && h > 0x7FFFFFFFll)
        return ofail(MR_EINVAL, "h must be at most 2^31 - 1 for int32 pixels");
    const uint32_t hk = h > 0xFFFFFFFFll ? 0xFFFFFFFFu : (uint32_t)h;
    hipStream_t s = (hipStream_t)stream;
    char *w = (char *)ws;
    void *marker = w + L.plane;
    uint32_t *flag = (uint32_t *)(w + L.flag);
    hipError_t e = (int)t == MR_U8
        ? hdome_marker<uint8_t>(img_inout, marker, H, W, pitch, hk, flag, s)
        : hdome_marker<int32_t>(img_inout, marker, H, W, pitch, hk, flag, s);
    if (e != hipSuccess) return ohip(e, "h-dome marker");
    rc = mr_recon_dilate(marker, img_inout, H, W, pitch, t, conn, ws, L.recon, tune, stream);
    if (rc != MR_OK) return rc;
    e = (int)t == MR_U8
        ? stream_pass<uint8_t, P_DOME>((const uint8_t *)img_inout, (const uint8_t *)marker,
                                       (uint8_t *)img_inout, nullptr, H, W, pitch, 0, 0u, flag, s)
        : stream_pass<int32_t, P_DOME>((const int32_t *)img_inout, (const int32_t *)marker,
                                       (int32_t *)img_inout, nullptr, H, W, pitch, 0, 0u, flag, s);
    return e == hipSuccess ? MR_OK : ohip(e, "h-dome output");
}

int mr_regional_maxima(const void *img, void *out_u8, int64_t H, int64_t W, int64_t pitch,
                       int64_t out_pitch, mr_dtype t, int conn, void *ws, size_t ws_bytes,
                       const mr_tune *tune, void *stream) {
    HdomeLayout L;
    int rc = hdome_common(img, H, W, pitch, (int)t, conn, ws, ws_bytes, tune, L);
    if (rc != MR_OK) return rc;
    if (!out_u8) return ofail(MR_EINVAL, "null output");
    if (out_pitch == 0) out_pitch = W;
    if (out_pitch < W) return ofail(MR_EINVAL, "out_pitch below W");
    hipStream_t s = (hipStream_t)stream;
    char *w = (char *)ws;
    void *marker = w + L.plane;
    uint32_t *flag = (uint32_t *)(w + L.flag);
    hipError_t e = (int)t == MR_U8
        ? hdome_marker<uint8_t>(img, marker, H, W, pitch, 1u, flag, s)
        : hdome_marker<int32_t>(img, marker, H, W, pitch, 1u, flag, s);
    if (e != hipSuccess) return ohip(e, "regional maxima marker");
    rc = mr_recon_dilate(marker, img, H, W, pitch, t, conn, ws, L.recon, tune, stream);
    if (rc != MR_OK) return rc;
    e = (int)t == MR_U8
        ? stream_pass<uint8_t, P_RMAX>((const uint8_t *)img, (const uint8_t *)marker, nullptr,
                                       (uint8_t *)out_u8, H, W, pitch, out_pitch, 0u, flag, s)
        : stream_pass<int32_t, P_RMAX>((const int32_t *)img, (const int32_t *)marker, nullptr,
                                       (uint8_t *)out_u8, H, W, pitch, out_pitch, 0u, flag, s);
    return e == hipSuccess ? MR_OK : ohip(e, "regional maxima output");
}

int mr_rgb2gray(const void *rgb, int64_t rgb_pitch, void *gray, int64_t gray_pitch, int64_t H,
                int64_t W, void *stream) {
    clear_error();
    if (!rgb || !gray) return ofail(MR_EINVAL, "null image");
    if (rgb_pitch == 0) rgb_pitch = 3 * W;
    if (gray_pitch == 0) gray_pitch = W;
    int rc;
    if ((rc = check_dims(H, W, gray_pitch, 1)) != MR_OK) return rc;
    if (rgb_pitch < 3 * W) return ofail(MR_EINVAL, "rgb_pitch %lld is below 3 W",
                                        (long long)rgb_pitch);
    hipStream_t s = (hipStream_t)stream;
    const uint8_t *src = (const uint8_t *)rgb;
    uint8_t *dst = (uint8_t *)gray;
    int64_t x0 = 0;
    const bool al = ((uintptr_t)src % 16 == 0) && rgb_pitch % 16 == 0 &&
                    ((uintptr_t)dst % 16 == 0) && gray_pitch % 16 == 0;
    if (al && W >= 16) {
        const int64_t vec = W / 16;
        hipLaunchKernelGGL(k_rgb2gray16, dim3(grid_for(H * vec, 256)), dim3(256), 0, s, src,
                           rgb_pitch, dst, gray_pitch, H, vec);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return ohip(e, "rgb2gray");
        x0 = vec * 16;
    }
    if (x0 < W) {
        hipLaunchKernelGGL(k_rgb2gray1, dim3(grid_for(H * (W - x0), 256)), dim3(256), 0, s, src,
                           rgb_pitch, dst, gray_pitch, H, x0, W);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return ohip(e, "rgb2gray");
    }
    return MR_OK;
}

int mr_disk13(int op, const void *in, void *out, int64_t H, int64_t W, int64_t pitch,
              void *stream) {
    clear_error();
    if (op != MR_DISK_ERODE && op != MR_DISK_DILATE) return ofail(MR_EINVAL, "unknown op %d", op);
    if (!in || !out) return ofail(MR_EINVAL, "null image");
    if (pitch == 0) pitch = W;
    int rc;
    if ((rc = check_dims(H, W, pitch, 1)) != MR_OK) return rc;
    const char *a = (const char *)in, *b = (const char *)out;
    const size_t span = (size_t)((H - 1) * pitch + W);
    if (a < b + span && b < a + span) return ofail(MR_EINVAL, "in and out overlap");
    hipError_t e = launch_disk13(op == MR_DISK_ERODE, (const uint8_t *)in, (uint8_t *)out, H, W,
                                 pitch, (hipStream_t)stream);
    return e == hipSuccess ? MR_OK : ohip(e, "disk13");
}

size_t mr_open_disk13_workspace_bytes(int64_t H, int64_t W, int64_t pitch) {
    clear_error();
    if (pitch == 0) pitch = W;
    if (check_dims(H, W, pitch, 1) != MR_OK) return 0;
    return up256((size_t)H * (size_t)pitch);
}

int mr_open_disk13(const void *in, void *out, int64_t H, int64_t W, int64_t pitch, void *ws,
                   size_t ws_bytes, void *stream) {
    clear_error();
    if (pitch == 0) pitch = W;
    int rc;
    if ((rc = check_dims(H, W, pitch, 1)) != MR_OK) return rc;
    if (!ws) return ofail(MR_EINVAL, "null workspace");
    if ((uintptr_t)ws % 256) return ofail(MR_EINVAL, "workspace must be 256-byte aligned");
    const size_t need = up256((size_t)H * (size_t)pitch);
    if (ws_bytes < need)
        return ofail(MR_ENOMEM, "workspace too small: %zu bytes given, %zu needed", ws_bytes,
                     need);
    if ((rc = mr_disk13(MR_DISK_ERODE, in, ws, H, W, pitch, stream)) != MR_OK) return rc;
    return mr_disk13(MR_DISK_DILATE, ws, out, H, W, pitch, stream);
}

} // extern "C"
