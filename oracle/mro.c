/*
 * oracle/mro.c -- sequential CPU oracle for grayscale morphological
 * reconstruction by dilation and for fill-holes.
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library. The GPU product path
 * shares no code, header, table or helper with it, and never calls it.
 *
 * What it computes (Table II, "Morphological Reconstruction": flood-fill of a
 * marker image limited by a mask image, 4- or 8-connected, after Vincent 1993;
 * "FillHoles": flood-fill of the background from selected points):
 *
 *   J0 = min(marker, mask) pointwise
 *   delta(J)(p) = min(mask(p), max of J over p and its G-neighbours)
 *   R = delta iterated until nothing changes (the least fixed point >= J0).
 *
 * How (Sec. V-C.2 and Algorithm 1): a regular phase of one raster and one
 * anti-raster scan, after which the remaining work is driven by a FIFO of
 * active pixels -- the wavefront container S of Algorithm 1 -- with
 *   PropagationCondition(p, q):  J(q) < J(p)  and  J(q) != mask(q)
 *   Update(p, q):                J(q) <- min(J(p), mask(q)).
 * The anti-raster scan fills the FIFO with every pixel that can still raise a
 * neighbour that comes after it in anti-raster order.
 *
 * Readings taken where the paper is silent: pixels outside the image do not
 * exist (no wrap-around, no padding value); marker pixels above the mask are
 * clipped to it; the 4-neighbourhood is the edge neighbours and the
 * 8-neighbourhood adds the diagonals; fill-holes seeds the flood from every
 * image-border pixel and runs on the bitwise complement.
 *
 * Work is done on int32 copies of the images (both pixel types fit exactly),
 * so there is one implementation of the arithmetic for both types.
 *
 * Building with -DMRO_PLANT=k plants deliberate mistake number k (used only
 * by the tests that show the pins catch such mistakes).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef MRO_PLANT
#define MRO_PLANT 0
#endif

typedef struct {
    uint64_t passes; /* regular raster/anti-raster scans made (always 2) */
    uint64_t seeds;  /* pixels the anti-raster scan put in the FIFO */
    uint64_t pops;   /* FIFO extractions */
    uint64_t pushes; /* FIFO insertions, seeds included */
} mro_counts;

enum { MRO_OK = 0, MRO_EINVAL = -1, MRO_ENOMEM = -2 };

/* ------------------------------------------------------------------ FIFO */

typedef struct {
    int64_t *buf;
    size_t cap, head, len;
} fifo_t;

static int fifo_push(fifo_t *q, int64_t v) {
    if (q->len == q->cap) {
        size_t ncap = q->cap ? 2 * q->cap : 4096;
        int64_t *nb = (int64_t *)malloc(ncap * sizeof(int64_t));
        if (!nb) return -1;
        for (size_t i = 0; i < q->len; i++) nb[i] = q->buf[(q->head + i) % q->cap];
        free(q->buf);
        q->buf = nb;
        q->cap = ncap;
        q->head = 0;
    }
    q->buf[(q->head + q->len) % q->cap] = v;
    q->len++;
    return 0;
}

static int64_t fifo_pop(fifo_t *q) {
    int64_t v = q->buf[q->head];
    q->head = (q->head + 1) % q->cap;
    q->len--;
    return v;
}

static inline int32_t imax(int32_t a, int32_t b) { return a > b ? a : b; }
static inline int32_t imin(int32_t a, int32_t b) { return a < b ? a : b; }

/* Neighbour offsets (dy, dx). The first `half` entries of each list form the
 * causal half-neighbourhood used by the raster scan (rows above, then the
 * pixel to the left); the anti-raster scan uses their mirror images. */
static const int NB8[8][2] = {{-1, -1}, {-1, 0}, {-1, 1}, {0, -1},
                              {1, 1},   {1, 0},  {1, -1}, {0, 1}};
static const int NB4[4][2] = {{-1, 0}, {0, -1}, {1, 0}, {0, 1}};

static const int (*nbr_list(int conn, int *count))[2] {
    if (conn == 8) { *count = 8; return NB8; }
    *count = 4;
    return NB4;
}

/* Is (y+dy, x+dx) inside the image? */
static inline int inside(int64_t y, int64_t x, int dy, int dx, int64_t H, int64_t W) {
    int64_t yy = y + dy, xx = x + dx;
#if MRO_PLANT == 5
    /* planted: rows wrap around at the right edge (onto the next row; never
     * past the last pixel, so the planted copy stays inside its arrays) */
    return yy >= 0 && yy < H && xx >= 0 && yy * W + xx < H * W;
#else
    return yy >= 0 && yy < H && xx >= 0 && xx < W;
#endif
}

/* Reconstruction on int32 working images. J holds J0 = min(marker, mask) on
 * entry and R on return; I is the mask. */
static int recon_core(int32_t *J, const int32_t *I, int64_t H, int64_t W, int conn,
                      mro_counts *cnt) {
    int nn;
    const int(*nb)[2] = nbr_list(conn, &nn);
    const int half = nn / 2;
    fifo_t q = {0};
    mro_counts c = {0};

    /* Raster scan: each pixel takes the max over itself and its causal
     * half-neighbourhood, limited by the mask. */
    for (int64_t y = 0; y < H; y++) {
        for (int64_t x = 0; x < W; x++) {
            int64_t p = y * W + x;
            int32_t m = J[p];
            for (int k = 0; k < half; k++)
                if (inside(y, x, nb[k][0], nb[k][1], H, W))
                    m = imax(m, J[p + nb[k][0] * W + nb[k][1]]);
            J[p] = imin(m, I[p]);
        }
    }
    /* Anti-raster scan over the mirrored half-neighbourhood, then seed the
     * FIFO with pixels that can still raise one of those neighbours. */
    for (int64_t y = H - 1; y >= 0; y--) {
#if MRO_PLANT == 7
        for (int64_t x = W - 2; x >= 0; x--) { /* planted: last column skipped */
#else
        for (int64_t x = W - 1; x >= 0; x--) {
#endif
            int64_t p = y * W + x;
            int32_t m = J[p];
            for (int k = half; k < nn; k++)
                if (inside(y, x, nb[k][0], nb[k][1], H, W))
                    m = imax(m, J[p + nb[k][0] * W + nb[k][1]]);
            J[p] = imin(m, I[p]);
            for (int k = half; k < nn; k++) {
#if MRO_PLANT == 1
                if (conn == 8 && k == 6) continue; /* planted: seed test skips (y+1, x-1) */
#endif
                if (!inside(y, x, nb[k][0], nb[k][1], H, W)) continue;
                int64_t r = p + nb[k][0] * W + nb[k][1];
                if (J[r] < J[p] && J[r] < I[r]) {
                    if (fifo_push(&q, p)) { free(q.buf); return MRO_ENOMEM; }
                    c.seeds++;
                    c.pushes++;
                    break;
                }
            }
        }
    }
    c.passes = 2;

#if MRO_PLANT != 2 /* planted mistake 2 skips the queue phase */
    /* Queue phase (Algorithm 1's propagation loop). */
    while (q.len) {
        int64_t p = fifo_pop(&q);
        c.pops++;
        int64_t y = p / W, x = p % W;
        for (int k = 0; k < nn; k++) {
            int dy = nb[k][0], dx = nb[k][1];
            if (!inside(y, x, dy, dx, H, W)) continue;
            int64_t r = p + dy * W + dx;
            if (J[r] < J[p] && J[r] != I[r]) {
#if MRO_PLANT == 3
                J[r] = imax(J[p], I[r]); /* planted: wrong operator */
#elif MRO_PLANT == 4
                J[r] = imin(J[p], I[p]); /* planted: mask read at the wrong pixel */
#else
                J[r] = imin(J[p], I[r]);
#endif
                if (fifo_push(&q, r)) { free(q.buf); return MRO_ENOMEM; }
                c.pushes++;
            }
        }
    }
#endif
    free(q.buf);
    if (cnt) *cnt = c;
    return MRO_OK;
}

static int check_args(const void *a, const void *b, int64_t H, int64_t W, int conn) {
    if (!a || !b || H < 1 || W < 1 || (conn != 4 && conn != 8)) return MRO_EINVAL;
    return MRO_OK;
}

/* ----------------------------------------------------- exported functions */

int mro_recon_dilate_u8(uint8_t *marker_inout, const uint8_t *mask, int64_t H, int64_t W,
                        int conn, mro_counts *cnt) {
    if (check_args(marker_inout, mask, H, W, conn)) return MRO_EINVAL;
    size_t n = (size_t)H * (size_t)W;
    int32_t *J = (int32_t *)malloc(n * sizeof(int32_t));
    int32_t *I = (int32_t *)calloc(n, sizeof(int32_t));
    if (!J || !I) { free(J); free(I); return MRO_ENOMEM; }
    for (size_t i = 0; i < n; i++) {
        I[i] = mask[i];
        J[i] = imin(marker_inout[i], mask[i]);
    }
    int rc = recon_core(J, I, H, W, conn, cnt);
    if (rc == MRO_OK)
        for (size_t i = 0; i < n; i++) marker_inout[i] = (uint8_t)J[i];
    free(J);
    free(I);
    return rc;
}

int mro_recon_dilate_i32(int32_t *marker_inout, const int32_t *mask, int64_t H, int64_t W,
                         int conn, mro_counts *cnt) {
    if (check_args(marker_inout, mask, H, W, conn)) return MRO_EINVAL;
    size_t n = (size_t)H * (size_t)W;
    int32_t *I = (int32_t *)malloc(n * sizeof(int32_t));
    if (!I) return MRO_ENOMEM;
    memcpy(I, mask, n * sizeof(int32_t));
    for (size_t i = 0; i < n; i++) marker_inout[i] = imin(marker_inout[i], mask[i]);
    int rc = recon_core(marker_inout, I, H, W, conn, cnt);
    free(I);
    return rc;
}

/* Fill-holes: out = NOT R(Jb, NOT f), where NOT is the bitwise complement (an
 * order-reversing bijection of the pixel type) and Jb equals NOT f on the
 * image border and the type's minimum inside. */
static int fill_core(int32_t *work_f, int64_t H, int64_t W, int conn, int32_t minval,
                     int32_t (*cmpl)(int32_t), mro_counts *cnt) {
    size_t n = (size_t)H * (size_t)W;
    int32_t *I = (int32_t *)malloc(n * sizeof(int32_t));
    if (!I) return MRO_ENOMEM;
    for (int64_t y = 0; y < H; y++) {
        for (int64_t x = 0; x < W; x++) {
            int64_t p = y * W + x;
            I[p] = cmpl(work_f[p]);
#if MRO_PLANT == 6
            int border = (y == 0 || y == H - 1); /* planted: side columns not seeded */
#else
            int border = (y == 0 || y == H - 1 || x == 0 || x == W - 1);
#endif
            work_f[p] = border ? I[p] : minval;
        }
    }
    int rc = recon_core(work_f, I, H, W, conn, cnt);
    if (rc == MRO_OK)
        for (size_t i = 0; i < n; i++) work_f[i] = cmpl(work_f[i]);
    free(I);
    return rc;
}

static int32_t cmpl_u8(int32_t v) { return 255 - v; }
static int32_t cmpl_i32(int32_t v) { return ~v; }

int mro_fill_holes_u8(uint8_t *img_inout, int64_t H, int64_t W, int conn, mro_counts *cnt) {
    if (check_args(img_inout, img_inout, H, W, conn)) return MRO_EINVAL;
    size_t n = (size_t)H * (size_t)W;
    int32_t *w = (int32_t *)malloc(n * sizeof(int32_t));
    if (!w) return MRO_ENOMEM;
    for (size_t i = 0; i < n; i++) w[i] = img_inout[i];
    int rc = fill_core(w, H, W, conn, 0, cmpl_u8, cnt);
    if (rc == MRO_OK)
        for (size_t i = 0; i < n; i++) img_inout[i] = (uint8_t)w[i];
    free(w);
    return rc;
}

int mro_fill_holes_i32(int32_t *img_inout, int64_t H, int64_t W, int conn, mro_counts *cnt) {
    if (check_args(img_inout, img_inout, H, W, conn)) return MRO_EINVAL;
    return fill_core(img_inout, H, W, conn, INT32_MIN, cmpl_i32, cnt);
}

/* Reconstruction by erosion, the dual of Table II's reconstruction (after
 * Vincent 1993): E is the greatest image J <= max(marker, mask) that is stable
 * under J(p) <- max(mask(p), min of J over p and its G-neighbours). NOT, the
 * bitwise complement, reverses the order and maps min to max, so
 * E = NOT R(NOT marker, NOT mask); that identity is the whole computation
 * here, on top of the reconstruction by dilation above. */
static int erode_core(int32_t *J, const int32_t *mask, int64_t H, int64_t W, int conn,
                      int32_t (*cmpl)(int32_t), mro_counts *cnt) {
    size_t n = (size_t)H * (size_t)W;
    int32_t *I = (int32_t *)calloc(n, sizeof(int32_t));
    if (!I) return MRO_ENOMEM;
    for (size_t i = 0; i < n; i++) {
#if MRO_PLANT == 9
        I[i] = mask[i]; /* planted: mask not complemented */
#else
        I[i] = cmpl(mask[i]);
#endif
#if MRO_PLANT == 8
        J[i] = imax(cmpl(J[i]), I[i]); /* planted: clipped with the wrong operator */
#else
        J[i] = imin(cmpl(J[i]), I[i]);
#endif
    }
    int rc = recon_core(J, I, H, W, conn, cnt);
    if (rc == MRO_OK)
        for (size_t i = 0; i < n; i++) J[i] = cmpl(J[i]);
    free(I);
    return rc;
}

int mro_recon_erode_u8(uint8_t *marker_inout, const uint8_t *mask, int64_t H, int64_t W,
                       int conn, mro_counts *cnt) {
    if (check_args(marker_inout, mask, H, W, conn)) return MRO_EINVAL;
    size_t n = (size_t)H * (size_t)W;
    int32_t *J = (int32_t *)malloc(n * sizeof(int32_t));
    int32_t *M = (int32_t *)malloc(n * sizeof(int32_t));
    if (!J || !M) { free(J); free(M); return MRO_ENOMEM; }
    for (size_t i = 0; i < n; i++) {
        J[i] = marker_inout[i];
        M[i] = mask[i];
    }
    int rc = erode_core(J, M, H, W, conn, cmpl_u8, cnt);
    if (rc == MRO_OK)
        for (size_t i = 0; i < n; i++) marker_inout[i] = (uint8_t)J[i];
    free(J);
    free(M);
    return rc;
}

int mro_recon_erode_i32(int32_t *marker_inout, const int32_t *mask, int64_t H, int64_t W,
                        int conn, mro_counts *cnt) {
    if (check_args(marker_inout, mask, H, W, conn)) return MRO_EINVAL;
    return erode_core(marker_inout, mask, H, W, conn, cmpl_i32, cnt);
}
