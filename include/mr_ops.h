/*
 * mr_ops.h -- C ABI of the segmentation operations of Table II beside the
 * reconstruction itself, on one AMD Instinct MI355X (gfx950):
 *   - the reconstruction-based h-dome and regional maxima (Table II's
 *     reconstruction after Vincent 1993, run on the engine of mr.h);
 *   - RGB to grayscale and morphological opening with a 13 x 13 disk (the
 *     regular, memory-bound operations of Table II and Sec. V-C.1);
 *   - the distance transform (Table II: an IWPP operation, 8-connected);
 *   - connected components labeling (Table II: union-find, Sec. II-B and
 *     Sec. III-B) and area threshold (Table II: a map and a reduction).
 *
 * Conventions (as in mr.h): every image pointer is a DEVICE pointer owned by
 * the caller; rows are `pitch` elements apart (0 means W); H, W >= 1; the
 * library allocates no device memory, scratch space is the caller's
 * workspace (256-byte aligned, contents on entry irrelevant) whose size the
 * *_workspace_bytes call gives; `stream` is a hipStream_t as void* (NULL =
 * null stream) and calls return without waiting for the device unless
 * stated; arguments are checked on the host before anything is enqueued;
 * errors are the negative MR_* codes of mr.h with a thread-local message in
 * mr_last_error(). Two calls that share a workspace must be ordered on one
 * stream. Device faults surface at the caller's next synchronization.
 */
#ifndef MR_OPS_H
#define MR_OPS_H

#include "mr.h"

#ifdef __cplusplus
extern "C" {
#endif

/* ----------------------------------------------- h-dome, regional maxima */

/* Workspace bytes of mr_hdome and mr_regional_maxima on an H x W image with
 * row pitch `pitch` (0 = W). 0 on invalid arguments. */
size_t mr_hdome_workspace_bytes(int64_t H, int64_t W, int64_t pitch, mr_dtype t, int conn,
                                const mr_tune *tune);

/* h-dome (Vincent 1993, the reconstruction of Table II): in place,
 * f <- f - R(f - h, f), where f - h saturates at the type's minimum and R is
 * the reconstruction by dilation of mr.h. The result lies in [0, h] (for
 * int32 the difference of two int32 values, exact). 0 <= h, and h <= 2^31 - 1
 * for int32 pixels; h = 0 gives 0.
 * The marker is built in the workspace (a plane of H x pitch pixels after
 * the reconstruction's own workspace); f is read as the mask and overwritten
 * at the end. Errors: MR_EINVAL (arguments, h < 0), MR_ENOMEM (ws_bytes
 * below mr_hdome_workspace_bytes), MR_EHIP. */
int mr_hdome(void *img_inout, int64_t H, int64_t W, int64_t pitch, mr_dtype t, int conn,
             int64_t h, void *ws, size_t ws_bytes, const mr_tune *tune, void *stream);

/* Regional maxima: out_u8 (H x W uint8, row pitch out_pitch, 0 = W) gets 255
 * on every pixel of a regional maximum of img -- a G-connected plateau of
 * equal values none of whose G-neighbours is higher -- and 0 elsewhere.
 * Computed as the pixels where the dome of height 1, f - R(f - 1, f), is
 * positive; f - 1 saturates at the type's minimum, so a constant image at
 * the minimum (the one plateau at the minimum with no higher neighbour) is
 * detected separately and is all maximum. img is read only. Workspace as for
 * mr_hdome. Errors as for mr_hdome. */
int mr_regional_maxima(const void *img, void *out_u8, int64_t H, int64_t W, int64_t pitch,
                       int64_t out_pitch, mr_dtype t, int conn, void *ws, size_t ws_bytes,
                       const mr_tune *tune, void *stream);

/* ------------------------------------------------------------ RGB2Gray */

/* RGB to grayscale (Table II): rgb holds H rows of W pixels of three
 * interleaved bytes R, G, B, rows rgb_pitch BYTES apart (0 = 3 W); gray gets
 * H x W uint8 with row pitch gray_pitch (0 = W):
 *   gray = (4899 R + 9617 G + 1868 B + 8192) >> 14,
 * the ITU-R BT.601 luma weights 0.299, 0.587, 0.114 in 14-bit fixed point,
 * rounded half up (within 1 of the real-weighted value; R = G = B = v gives
 * v). No workspace. Errors: MR_EINVAL. */
int mr_rgb2gray(const void *rgb, int64_t rgb_pitch, void *gray, int64_t gray_pitch, int64_t H,
                int64_t W, void *stream);

/* ------------------------------------------------ opening, 13 x 13 disk */

/* Morphological opening of a uint8 image by the flat disk of radius 6 (the
 * offsets (dy, dx) with dy^2 + dx^2 <= 36 in the 13 x 13 box; Table II):
 * out = dilation(erosion(in)). Pixels outside the image are ignored (the
 * erosion takes the minimum, the dilation the maximum, over the offsets that
 * land inside). in and out may not overlap; both have row pitch `pitch`. The
 * erosion goes to a workspace plane of H x pitch bytes. Errors: MR_EINVAL,
 * MR_ENOMEM. */
size_t mr_open_disk13_workspace_bytes(int64_t H, int64_t W, int64_t pitch);
int mr_open_disk13(const void *in, void *out, int64_t H, int64_t W, int64_t pitch, void *ws,
                   size_t ws_bytes, void *stream);

/* One half of the opening: flat erosion (op 0) or dilation (op 1) of in by
 * the same disk into out (no overlap, same pitch). No workspace. */
enum { MR_DISK_ERODE = 0, MR_DISK_DILATE = 1 };
int mr_disk13(int op, const void *in, void *out, int64_t H, int64_t W, int64_t pitch,
              void *stream);

/* ------------------------------------------------- distance transform */

/* Distance transform (Table II: IWPP, 8-connected). img: H x W uint8,
 * nonzero = foreground; dist: H x W int32 (row pitch dist_pitch, 0 = W)
 * receives, for every pixel, the length in steps between G-neighbours of the
 * shortest path to a background (zero) pixel: conn 8 gives the chessboard
 * distance max(|dy|, |dx|), conn 4 the city-block distance |dy| + |dx|;
 * background pixels get 0, and every pixel gets -1 when the image has no
 * background pixel. The result is unique. Computed as wavefront propagation
 * over 64 x 64 tiles, revisiting tiles whose border changed until no tile
 * changes (the host waits on a small counter between batches of rounds).
 * Errors: MR_EINVAL, MR_ENOMEM, MR_EHIP. */
size_t mr_distance_transform_workspace_bytes(int64_t H, int64_t W, int conn);
int mr_distance_transform(const void *img, void *dist, int64_t H, int64_t W, int64_t pitch,
                          int64_t dist_pitch, int conn, void *ws, size_t ws_bytes,
                          void *stream);

/* ------------------------------------- connected components, area threshold */

/* Connected components labeling (Table II: union-find, after Sec. II-B):
 * img H x W uint8 (nonzero = foreground), labels H x W int32 (row pitch
 * label_pitch, 0 = W). Every foreground pixel gets 1 + the smallest linear
 * index y * W + x of its G-connected component, background pixels 0: the
 * root of each union-find tree is its smallest element, so the labels are
 * unique and independent of the order of the merges. H * W < 2^31 - 1.
 * Three launches: union-find inside 32 x 64 tiles in LDS, merges of the
 * trees across tile borders with device atomics, and flattening. Workspace:
 * the forest, 4 bytes per pixel. Errors: MR_EINVAL, MR_ENOMEM, MR_EHIP. */
size_t mr_ccl_workspace_bytes(int64_t H, int64_t W);
int mr_ccl(const void *img, void *labels, int64_t H, int64_t W, int64_t pitch,
           int64_t label_pitch, int conn, void *ws, size_t ws_bytes, void *stream);

/* Area threshold (Table II: map + reduction): labels_inout H x W int32, each
 * value in [0, H * W] (0 = background; mr_ccl's labels qualify). The area of
 * label l is the number of pixels carrying it; every pixel whose label's
 * area lies outside [min_area, max_area] is set to 0 (min_area > max_area
 * removes every object). After the call the workspace starts with the
 * H * W + 1 per-label areas as int32 (entry l = area of label l; entry 0
 * unused), for callers that want them. Labels outside [0, H * W] are neither
 * counted nor changed. Errors: MR_EINVAL, MR_ENOMEM, MR_EHIP. */
size_t mr_area_threshold_workspace_bytes(int64_t H, int64_t W);
int mr_area_threshold(void *labels_inout, int64_t H, int64_t W, int64_t pitch, int64_t min_area,
                      int64_t max_area, void *ws, size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* MR_OPS_H */
