/* Runs every oracle entry point on seeded random images of many shapes, for a
 * build with AddressSanitizer and UndefinedBehaviorSanitizer
 * (tests/test_oracle_sanitize.py builds it with mro.c and mro_ops.c and runs
 * it). TEST INFRASTRUCTURE: nothing on the GPU path links or runs it.
 *
 * It checks return codes and the bounds every result must keep (marker and
 * mask bracket a reconstruction, labels stay in range); the values themselves
 * are the pin tests' business. The sanitizers report any out-of-bounds access,
 * use of freed memory, leak, signed overflow or bad shift on the way, and
 * abort the run. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    uint64_t passes, seeds, pops, pushes;
} mro_counts;

int mro_recon_dilate_u8(uint8_t *, const uint8_t *, int64_t, int64_t, int, mro_counts *);
int mro_recon_dilate_i32(int32_t *, const int32_t *, int64_t, int64_t, int, mro_counts *);
int mro_recon_erode_u8(uint8_t *, const uint8_t *, int64_t, int64_t, int, mro_counts *);
int mro_recon_erode_i32(int32_t *, const int32_t *, int64_t, int64_t, int, mro_counts *);
int mro_fill_holes_u8(uint8_t *, int64_t, int64_t, int, mro_counts *);
int mro_fill_holes_i32(int32_t *, int64_t, int64_t, int, mro_counts *);
int mro_rgb2gray(const uint8_t *, uint8_t *, int64_t, int64_t);
int mro_erode_disk13_u8(const uint8_t *, uint8_t *, int64_t, int64_t);
int mro_dilate_disk13_u8(const uint8_t *, uint8_t *, int64_t, int64_t);
int mro_open_disk13_u8(const uint8_t *, uint8_t *, int64_t, int64_t);
int mro_distance_transform(const uint8_t *, int32_t *, int64_t, int64_t, int);
int mro_ccl(const uint8_t *, int32_t *, int64_t, int64_t, int);
int mro_area_threshold(int32_t *, int64_t, int64_t, int64_t, int64_t, int64_t *);

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;

static uint32_t rnd(void) { /* xorshift64* */
    rng_state ^= rng_state >> 12;
    rng_state ^= rng_state << 25;
    rng_state ^= rng_state >> 27;
    return (uint32_t)((rng_state * 0x2545F4914F6CDD1Dull) >> 32);
}

static int failures = 0;

static void expect(int ok, const char *what, int64_t H, int64_t W, int conn) {
    if (!ok) {
        fprintf(stderr, "FAILED: %s at %lldx%lld conn%d\n", what, (long long)H, (long long)W,
                conn);
        ++failures;
    }
}

static void run_shape(int64_t H, int64_t W, int conn, int levels) {
    const size_t n = (size_t)H * (size_t)W;
    uint8_t *mask8 = malloc(n), *mark8 = malloc(n), *keep8 = malloc(n), *out8 = malloc(n);
    uint8_t *rgb = malloc(3 * n), *bin = malloc(n);
    int32_t *mask32 = malloc(n * 4), *mark32 = malloc(n * 4), *keep32 = malloc(n * 4);
    int32_t *lab = malloc(n * 4), *dist = malloc(n * 4);
    int64_t *areas = malloc((n + 1) * 8);
    mro_counts c;
    for (size_t i = 0; i < n; ++i) {
        mask8[i] = (uint8_t)(rnd() % (uint32_t)levels);
        mark8[i] = (uint8_t)(rnd() % (uint32_t)levels);
        mask32[i] = (int32_t)rnd();
        mark32[i] = (int32_t)rnd();
        bin[i] = (rnd() & 3) ? 255 : 0;
        rgb[3 * i] = (uint8_t)rnd();
        rgb[3 * i + 1] = (uint8_t)rnd();
        rgb[3 * i + 2] = (uint8_t)rnd();
    }

    memcpy(keep8, mark8, n);
    expect(mro_recon_dilate_u8(keep8, mask8, H, W, conn, &c) == 0, "recon_dilate_u8", H, W, conn);
    for (size_t i = 0; i < n; ++i)
        if (keep8[i] > mask8[i] || keep8[i] < (mark8[i] < mask8[i] ? mark8[i] : mask8[i])) {
            expect(0, "recon_dilate_u8 bounds", H, W, conn);
            break;
        }
    memcpy(keep32, mark32, n * 4);
    expect(mro_recon_dilate_i32(keep32, mask32, H, W, conn, &c) == 0, "recon_dilate_i32", H, W,
           conn);
    for (size_t i = 0; i < n; ++i)
        if (keep32[i] > mask32[i]) {
            expect(0, "recon_dilate_i32 bounds", H, W, conn);
            break;
        }
    memcpy(keep8, mark8, n);
    expect(mro_recon_erode_u8(keep8, mask8, H, W, conn, &c) == 0, "recon_erode_u8", H, W, conn);
    for (size_t i = 0; i < n; ++i)
        if (keep8[i] < mask8[i]) {
            expect(0, "recon_erode_u8 bounds", H, W, conn);
            break;
        }
    memcpy(keep32, mark32, n * 4);
    expect(mro_recon_erode_i32(keep32, mask32, H, W, conn, &c) == 0, "recon_erode_i32", H, W,
           conn);
    memcpy(keep8, bin, n);
    expect(mro_fill_holes_u8(keep8, H, W, conn, &c) == 0, "fill_holes_u8", H, W, conn);
    for (size_t i = 0; i < n; ++i)
        if (keep8[i] < bin[i]) {
            expect(0, "fill_holes_u8 bounds", H, W, conn);
            break;
        }
    memcpy(keep32, mask32, n * 4);
    expect(mro_fill_holes_i32(keep32, H, W, conn, &c) == 0, "fill_holes_i32", H, W, conn);

    expect(mro_rgb2gray(rgb, out8, H, W) == 0, "rgb2gray", H, W, conn);
    expect(mro_erode_disk13_u8(mask8, out8, H, W) == 0, "erode_disk13", H, W, conn);
    expect(mro_dilate_disk13_u8(mask8, out8, H, W) == 0, "dilate_disk13", H, W, conn);
    expect(mro_open_disk13_u8(mask8, out8, H, W) == 0, "open_disk13", H, W, conn);
    expect(mro_distance_transform(bin, dist, H, W, conn) == 0, "distance_transform", H, W, conn);
    expect(mro_ccl(bin, lab, H, W, conn) == 0, "ccl", H, W, conn);
    for (size_t i = 0; i < n; ++i)
        if (lab[i] < 0 || (int64_t)lab[i] > (int64_t)n || (lab[i] != 0) != (bin[i] != 0)) {
            expect(0, "ccl labels", H, W, conn);
            break;
        }
    expect(mro_area_threshold(lab, H, W, 2, 40, areas) == 0, "area_threshold", H, W, conn);

    free(mask8); free(mark8); free(keep8); free(out8); free(rgb); free(bin);
    free(mask32); free(mark32); free(keep32); free(lab); free(dist); free(areas);
}

int main(void) {
    static const int64_t shapes[][2] = {{1, 1}, {1, 2}, {2, 1}, {1, 97}, {97, 1}, {2, 3},
                                        {7, 13}, {13, 7}, {31, 64}, {64, 65}, {100, 37},
                                        {129, 130}, {300, 257}, {3, 700}};
    const int n_shapes = (int)(sizeof shapes / sizeof shapes[0]);
    for (int s = 0; s < n_shapes; ++s)
        for (int conn = 4; conn <= 8; conn += 4)
            for (int levels = 2; levels <= 256; levels *= 16)
                run_shape(shapes[s][0], shapes[s][1], conn, levels);
    /* argument checks: rejected, with no access */
    mro_counts c;
    uint8_t px = 0;
    expect(mro_recon_dilate_u8(&px, &px, 0, 1, 8, &c) != 0, "H = 0 rejected", 0, 1, 8);
    expect(mro_recon_dilate_u8(&px, &px, 1, 1, 6, &c) != 0, "conn 6 rejected", 1, 1, 6);
    if (failures) return 1;
    printf("oracle sanitize check: ok\n");
    return 0;
}
