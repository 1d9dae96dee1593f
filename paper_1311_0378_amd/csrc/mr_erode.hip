// mr_erode.hip -- reconstruction by erosion (mr_recon_erode in include/mr.h).
//
// The dual of Table II's reconstruction (after Vincent 1993): E is the
// greatest image at most max(marker, mask) that is stable under
// J(p) <- max(mask(p), min of J over p and its G-neighbours). The bitwise
// complement NOT reverses the order of both pixel types with no overflow (u8:
// 255 - v, i32: -1 - v) and turns min into max, so E = NOT R(NOT marker,
// NOT mask). A call runs three steps on the caller's stream:
//  1. one pass writes NOT mask into a plane at the workspace's tail (same
//     pitch as the images) and complements the marker in place;
//  2. the reconstruction by dilation runs on the two (mr_recon_dilate, with
//     the head of the workspace);
//  3. one pass complements the marker back.
// The passes are plain streaming kernels. Where rows and pointers are
// 16-byte aligned each lane moves 16-byte words; otherwise (and for the
// columns past a row's last whole word) each wave walks 512 consecutive
// pixels of one row, 64 lanes on consecutive pixels per access.
#include <algorithm>
#include <cstdio>

#include "mr_internal.h"

using namespace mr;

namespace {

constexpr int NOT_UNROLL = 8;                 // row segment = 64 * NOT_UNROLL pixels per wave
constexpr int64_t NOT_SEG = 64 * NOT_UNROLL;

// a <- NOT a over the H x W image (row pitch `pitch`); when b is given, also
// b_not <- NOT b at the same offsets.
template <typename T>
__global__ __launch_bounds__(256) void k_not_planes(T *__restrict__ a, const T *__restrict__ b,
                                                    T *__restrict__ b_not, int64_t H, int64_t W,
                                                    int64_t pitch, int64_t segs_per_row) {
    const int lane = threadIdx.x & 63;
    const int64_t items = H * segs_per_row;
    for (int64_t it = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); it < items;
         it += (int64_t)gridDim.x * 4) {
        const int64_t y = it / segs_per_row;
        const int64_t x0 = (it - y * segs_per_row) * NOT_SEG;
        const int64_t row = y * pitch;
        T va[NOT_UNROLL], vb[NOT_UNROLL];
#pragma unroll
        for (int k = 0; k < NOT_UNROLL; ++k) {
            const int64_t x = x0 + k * 64 + lane;
            if (x < W) {
                va[k] = a[row + x];
                if (b) vb[k] = b[row + x];
            }
        }
#pragma unroll
        for (int k = 0; k < NOT_UNROLL; ++k) {
            const int64_t x = x0 + k * 64 + lane;
            if (x < W) {
                a[row + x] = (T)~va[k];
                if (b) b_not[row + x] = (T)~vb[k];
            }
        }
    }
}

// The same on 16-byte words, for rows whose start and pitch are 16-byte
// aligned: bitwise NOT of the raw bits complements u8 and i32 pixels alike.
// vecs = whole 16-byte words per row, vpitch = the pitch in 16-byte words.
__global__ __launch_bounds__(256) void k_not_planes16(uint4 *__restrict__ a,
                                                      const uint4 *__restrict__ b,
                                                      uint4 *__restrict__ b_not, int64_t H,
                                                      int64_t vecs, int64_t vpitch) {
    const int64_t items = H * vecs;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < items;
         i += (int64_t)gridDim.x * 256) {
        const int64_t y = i / vecs;
        const int64_t o = y * vpitch + (i - y * vecs);
        const uint4 va = a[o];
        if (b) {
            const uint4 vb = b[o];
            b_not[o] = make_uint4(~vb.x, ~vb.y, ~vb.z, ~vb.w);
        }
        a[o] = make_uint4(~va.x, ~va.y, ~va.z, ~va.w);
    }
}

template <typename T>
hipError_t launch_not(T *a, const T *b, T *b_not, int64_t H, int64_t W, int64_t pitch,
                      hipStream_t s) {
    const auto al16 = [](const void *p) { return ((uintptr_t)p & 15) == 0; };
    if ((pitch * (int64_t)sizeof(T)) % 16 == 0 && al16(a) && (!b || (al16(b) && al16(b_not)))) {
        const int64_t vecs = W * (int64_t)sizeof(T) / 16;
        if (vecs > 0) {
            const int64_t blocks = std::min<int64_t>((H * vecs + 255) / 256, 1 << 16);
            hipLaunchKernelGGL(k_not_planes16, dim3((unsigned)blocks), dim3(256), 0, s,
                               (uint4 *)a, (const uint4 *)b, (uint4 *)b_not, H, vecs,
                               pitch * (int64_t)sizeof(T) / 16);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        // the columns past the last whole word, element by element
        const int64_t xv = vecs * 16 / (int64_t)sizeof(T);
        if (xv == W) return hipSuccess;
        a += xv;
        if (b) {
            b += xv;
            b_not += xv;
        }
        W -= xv;
    }
    const int64_t segs = (W + NOT_SEG - 1) / NOT_SEG;
    const int64_t blocks = std::min<int64_t>((H * segs + 3) / 4, 1 << 16);
    hipLaunchKernelGGL((k_not_planes<T>), dim3((unsigned)blocks), dim3(256), 0, s, a, b, b_not, H,
                       W, pitch, segs);
    return hipGetLastError();
}

hipError_t not_pass(int t, void *a, const void *b, void *b_not, int64_t H, int64_t W,
                    int64_t pitch, hipStream_t s) {
    if (t == MR_U8)
        return launch_not<uint8_t>((uint8_t *)a, (const uint8_t *)b, (uint8_t *)b_not, H, W,
                                   pitch, s);
    return launch_not<int32_t>((int32_t *)a, (const int32_t *)b, (int32_t *)b_not, H, W, pitch,
                               s);
}

size_t up256(size_t n) { return (n + 255) / 256 * 256; }

int efail(int code, const char *fmt, long long a = 0, long long b = 0) {
    char buf[256];
    snprintf(buf, sizeof buf, fmt, a, b);
    return set_error(code, buf);
}

// Checks what the dilation call would check, plus the plane's pitch, so that
// nothing is enqueued for a call that would be rejected halfway.
int check_erode(int64_t H, int64_t W, int64_t pitch, mr_dtype t, int conn, const mr_tune *tune,
                size_t *recon_ws, size_t *plane) {
    const size_t r = mr_workspace_bytes(MR_OP_RECON, H, W, t, conn, tune);
    if (r == 0) return MR_EINVAL; // message set by mr_workspace_bytes
    clear_error();
    const int64_t p = pitch ? pitch : W;
    if (p < W) return efail(MR_EINVAL, "pitch %lld is smaller than W %lld", p, W);
    const int64_t pp = (W + 63) / 64 * 64;
    if (H * std::max(p, pp) + 4 >= (1ll << 32))
        return efail(MR_EINVAL, "image plane too large: H * pitch must stay below 2^32 elements");
    *recon_ws = up256(r);
    *plane = up256((size_t)(H * p) * (size_t)t);
    return MR_OK;
}

} // namespace

extern "C" size_t mr_recon_erode_workspace_bytes(int64_t H, int64_t W, int64_t pitch, mr_dtype t,
                                                 int conn, const mr_tune *tune) {
    clear_error();
    size_t r = 0, plane = 0;
    if (check_erode(H, W, pitch, t, conn, tune, &r, &plane) != MR_OK) return 0;
    return r + plane;
}

extern "C" int mr_recon_erode(void *marker_inout, const void *mask, int64_t H, int64_t W,
                              int64_t pitch, mr_dtype t, int conn, void *ws, size_t ws_bytes,
                              const mr_tune *tune, void *stream) {
    clear_error();
    size_t r = 0, plane = 0;
    int rc = check_erode(H, W, pitch, t, conn, tune, &r, &plane);
    if (rc != MR_OK) return rc;
    if (!marker_inout || !mask || !ws)
        return set_error(MR_EINVAL, "null image or workspace pointer");
    if ((uintptr_t)ws % 256) return set_error(MR_EINVAL, "workspace must be 256-byte aligned");
    if ((uintptr_t)marker_inout % (int)t || (uintptr_t)mask % (int)t)
        return set_error(MR_EINVAL, "image pointers must be aligned to the pixel size");
    if (ws_bytes < r + plane)
        return efail(MR_ENOMEM, "workspace too small: %lld bytes given, %lld needed",
                     (long long)ws_bytes, (long long)(r + plane));
    const int64_t p = pitch ? pitch : W;
    hipStream_t s = (hipStream_t)stream;
    void *not_mask = (char *)ws + r;
    hipError_t e = not_pass((int)t, marker_inout, mask, not_mask, H, W, p, s);
    if (e != hipSuccess) return set_error(MR_EHIP, hipGetErrorString(e));
    rc = mr_recon_dilate(marker_inout, not_mask, H, W, p, t, conn, ws, r, tune, stream);
    if (rc != MR_OK) return rc;
    e = not_pass((int)t, marker_inout, nullptr, nullptr, H, W, p, s);
    if (e != hipSuccess) return set_error(MR_EHIP, hipGetErrorString(e));
    return MR_OK;
}
