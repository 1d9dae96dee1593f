/* mro_ops.c -- CPU oracle for the segmentation operations of Table II beside
 * reconstruction: RGB to grayscale, morphological opening with a 13x13 disk,
 * distance transform (IWPP), connected components labeling (union-find) and
 * area threshold (reduction).
 *
 * TEST INFRASTRUCTURE. Only tests/, __graft_entry__.smoke() and the CPU
 * baseline of bench.py may load this code. It shares nothing with the GPU
 * path. Every function is a plain sequential loop nest written from the
 * operation's definition (or, for the two pattern-driven operations, from the
 * pattern's steps in the paper's order); no blocking, fusion or reordering.
 * Images are row-major and C-contiguous (pitch = W). Return 0 on success,
 * -1 on a bad argument.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* MRO_PLANT >= 100 builds a copy with one deliberate mistake, for the tests
 * that show the pins catch it (see tests/test_oracle_ops_pins.py). */
#ifndef MRO_PLANT
#define MRO_PLANT 0
#endif

/* ------------------------------------------------------------ RGB2Gray
 * Table II, "Convert RGB to grayscale" (regular, multi-channel local).
 * Reading: ITU-R BT.601 luma weights 0.299, 0.587, 0.114 in 14-bit fixed
 * point (4899, 9617, 1868; they sum to 2^14), rounded half up:
 *   gray = (4899 R + 9617 G + 1868 B + 8192) >> 14.
 * rgb holds H x W pixels of three interleaved bytes R, G, B. */
int mro_rgb2gray(const uint8_t *rgb, uint8_t *gray, int64_t H, int64_t W) {
    if (!rgb || !gray || H < 1 || W < 1) return -1;
    for (int64_t y = 0; y < H; ++y)
        for (int64_t x = 0; x < W; ++x) {
            const uint8_t *p = rgb + (y * W + x) * 3;
#if MRO_PLANT == 101 /* red and blue weights swapped */
            const uint32_t v = 1868u * p[0] + 9617u * p[1] + 4899u * p[2] + 8192u;
#else
            const uint32_t v = 4899u * p[0] + 9617u * p[1] + 1868u * p[2] + 8192u;
#endif
            gray[y * W + x] = (uint8_t)(v >> 14);
        }
    return 0;
}

/* ----------------------------------------------------- morphological open
 * Table II, "Morphological Open" (regular, neighbourhood: 13 x 13 disk).
 * Reading: the flat structuring element is the disk of radius 6, the offsets
 * (dy, dx) with dy^2 + dx^2 <= 36 inside the 13 x 13 box; it is symmetric.
 * Pixels outside the image are ignored (erosion takes the minimum, dilation
 * the maximum, over the offsets that land inside). Opening = dilation of the
 * erosion. */
#if MRO_PLANT == 102 /* the disk's rim left out */
static int in_disk(int dy, int dx) { return dy * dy + dx * dx < 36; }
#else
static int in_disk(int dy, int dx) { return dy * dy + dx * dx <= 36; }
#endif

static void erode_disk_u8(const uint8_t *f, uint8_t *g, int64_t H, int64_t W) {
    for (int64_t y = 0; y < H; ++y)
        for (int64_t x = 0; x < W; ++x) {
            uint8_t m = 255;
            for (int dy = -6; dy <= 6; ++dy)
                for (int dx = -6; dx <= 6; ++dx) {
                    if (!in_disk(dy, dx)) continue;
                    const int64_t yy = y + dy, xx = x + dx;
                    if (yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
                    const uint8_t v = f[yy * W + xx];
                    if (v < m) m = v;
                }
            g[y * W + x] = m;
        }
}

static void dilate_disk_u8(const uint8_t *f, uint8_t *g, int64_t H, int64_t W) {
    for (int64_t y = 0; y < H; ++y)
        for (int64_t x = 0; x < W; ++x) {
            uint8_t m = 0;
            for (int dy = -6; dy <= 6; ++dy)
                for (int dx = -6; dx <= 6; ++dx) {
                    if (!in_disk(dy, dx)) continue;
                    const int64_t yy = y - dy, xx = x - dx;
                    if (yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
                    const uint8_t v = f[yy * W + xx];
                    if (v > m) m = v;
                }
            g[y * W + x] = m;
        }
}

int mro_erode_disk13_u8(const uint8_t *f, uint8_t *out, int64_t H, int64_t W) {
    if (!f || !out || H < 1 || W < 1) return -1;
    erode_disk_u8(f, out, H, W);
    return 0;
}

int mro_dilate_disk13_u8(const uint8_t *f, uint8_t *out, int64_t H, int64_t W) {
    if (!f || !out || H < 1 || W < 1) return -1;
    dilate_disk_u8(f, out, H, W);
    return 0;
}

int mro_open_disk13_u8(const uint8_t *f, uint8_t *out, int64_t H, int64_t W) {
    if (!f || !out || H < 1 || W < 1) return -1;
    uint8_t *t = (uint8_t *)malloc((size_t)(H * W));
    if (!t) return -1;
    erode_disk_u8(f, t, H, W);
    dilate_disk_u8(t, out, H, W);
    free(t);
    return 0;
}

/* --------------------------------------------------------- distance transform
 * Table II, "Distance Transform" (irregular, neighbourhood, 8-connected; IWPP).
 * Reading: the distance of a foreground pixel (nonzero input) to the closest
 * background pixel (zero input) is the length, in steps between G-neighbours,
 * of the shortest path to it: with G = 8 the chessboard distance
 * max(|dy|, |dx|), with G = 4 the city-block distance |dy| + |dx|. Background
 * pixels get 0; if the image has no background pixel every pixel gets -1.
 * Steps of Algorithm 1: the initial active set S is every background pixel,
 * with D = 0 there and D = infinity elsewhere; an element e_i taken from S
 * propagates to a neighbour e_j when D(e_i) + 1 < D(e_j) (the propagation
 * condition), which sets D(e_j) = D(e_i) + 1 (the update) and inserts e_j
 * into S. S is a FIFO queue. */
int mro_distance_transform(const uint8_t *img, int32_t *dist, int64_t H, int64_t W, int conn) {
    if (!img || !dist || H < 1 || W < 1 || (conn != 4 && conn != 8)) return -1;
    const int64_t N = H * W;
    const int32_t INF = INT32_MAX;
    int64_t *fifo = (int64_t *)malloc((size_t)N * sizeof(int64_t));
    if (!fifo) return -1;
    int64_t head = 0, tail = 0;
    for (int64_t p = 0; p < N; ++p) {
        if (img[p] == 0) {
            dist[p] = 0;
            fifo[tail++] = p;
        } else {
            dist[p] = INF;
        }
    }
    static const int DY[8] = {-1, 1, 0, 0, -1, -1, 1, 1};
    static const int DX[8] = {0, 0, -1, 1, -1, 1, -1, 1};
#if MRO_PLANT == 103 /* diagonal neighbours dropped */
    conn = 4;
#endif
    while (head < tail) {
        const int64_t p = fifo[head++];
        const int64_t y = p / W, x = p % W;
        for (int k = 0; k < conn; ++k) {
            const int64_t yy = y + DY[k], xx = x + DX[k];
            if (yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
            const int64_t q = yy * W + xx;
            if (dist[p] + 1 < dist[q]) {
                dist[q] = dist[p] + 1;
                fifo[tail++] = q; /* each pixel enters once: FIFO order is breadth first */
            }
        }
    }
    free(fifo);
    for (int64_t p = 0; p < N; ++p)
        if (dist[p] == INF) dist[p] = -1;
    return 0;
}

/* --------------------------------------------- connected components labeling
 * Table II, "Connected Components Labeling" (irregular, global; union-find),
 * with the union-find pattern of Sec. II-B: MakeSet makes every foreground
 * pixel (nonzero input) its own tree; the image is scanned and each pixel's
 * tree is merged (Union) with the tree of every foreground G-neighbour, the
 * root with the smaller value becoming the root of the merged tree; finally
 * the trees are flattened (Find) and each pixel reads its root's label.
 * Reading: a pixel's value in the forest is its linear index y * W + x, so
 * the root of a component is its smallest index, and the label written is
 * that index + 1; background pixels get 0. Labels are unique per component
 * and independent of any processing order. */
static int64_t uf_find(int64_t *parent, int64_t p) {
    /* path halving: every pixel on the way points to its grandparent, which
     * keeps the trees shallow on large images and changes no root */
    while (parent[p] != p) {
        parent[p] = parent[parent[p]];
        p = parent[p];
    }
    return p;
}

int mro_ccl(const uint8_t *img, int32_t *labels, int64_t H, int64_t W, int conn) {
    if (!img || !labels || H < 1 || W < 1 || (conn != 4 && conn != 8)) return -1;
    const int64_t N = H * W;
    if (N >= INT32_MAX) return -1;
    int64_t *parent = (int64_t *)malloc((size_t)N * sizeof(int64_t));
    if (!parent) return -1;
    for (int64_t p = 0; p < N; ++p) parent[p] = p; /* MakeSet */
    static const int DY[8] = {-1, 1, 0, 0, -1, -1, 1, 1};
    static const int DX[8] = {0, 0, -1, 1, -1, 1, -1, 1};
    for (int64_t p = 0; p < N; ++p) {
        if (!img[p]) continue;
        const int64_t y = p / W, x = p % W;
        for (int k = 0; k < conn; ++k) {
            const int64_t yy = y + DY[k], xx = x + DX[k];
            if (yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
            const int64_t q = yy * W + xx;
            if (!img[q]) continue;
            const int64_t a = uf_find(parent, p), b = uf_find(parent, q); /* Union */
#if MRO_PLANT == 104 /* the larger root wins */
            if (a > b) parent[b] = a;
            else if (b > a) parent[a] = b;
#else
            if (a < b) parent[b] = a;
            else if (b < a) parent[a] = b;
#endif
        }
    }
    for (int64_t p = 0; p < N; ++p)
        labels[p] = img[p] ? (int32_t)(uf_find(parent, p) + 1) : 0; /* flatten */
    free(parent);
    return 0;
}

/* ------------------------------------------------------------ area threshold
 * Table II, "Area Threshold" (reduction): objects whose area is not within
 * [min_area, max_area] are removed. Reading: the objects are the components
 * of a label image as mro_ccl writes it (0 = background, label = smallest
 * linear index + 1); the map step reads each pixel's label, the reduction
 * counts the pixels per label, and the filter writes 0 over every pixel of a
 * component whose count lies outside the closed range. areas (N + 1 entries)
 * receives the per-label counts. */
int mro_area_threshold(int32_t *labels, int64_t H, int64_t W, int64_t min_area,
                       int64_t max_area, int64_t *areas) {
    if (!labels || !areas || H < 1 || W < 1) return -1;
    const int64_t N = H * W;
    memset(areas, 0, (size_t)(N + 1) * sizeof(int64_t));
    for (int64_t p = 0; p < N; ++p) {
        const int32_t l = labels[p];
        if (l < 0 || l > N) return -1;
        if (l) areas[l] += 1;
    }
    for (int64_t p = 0; p < N; ++p) {
        const int32_t l = labels[p];
#if MRO_PLANT == 105 /* the range taken as open at its lower end */
        if (l && (areas[l] <= min_area || areas[l] > max_area)) labels[p] = 0;
#else
        if (l && (areas[l] < min_area || areas[l] > max_area)) labels[p] = 0;
#endif
    }
    return 0;
}
