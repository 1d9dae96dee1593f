// mr_kernels.hip -- gfx950 kernels of libmrecon.
//
// Pixels are handled as 32-bit unsigned keys whose order is the pixel order:
// uint8 v -> v, int32 v -> v ^ 0x80000000. Key 0 is the type's minimum, so it
// is the identity of max and stands for "no pixel" outside the image. The
// bitwise complement used by fill-holes is KMAX - key in key space.
//
// Four kernels carry the propagation (Algorithm 1 split into the regular and
// irregular phases of Sec. V-C.2):
//  * k_tile_round -- the regular phase. One wave owns a 64 x 64 tile of keys
//    held in registers (lane = column, register = row); the outer ring is the
//    halo. Down and up sweeps run along the registers with the diagonal
//    neighbours taken from the adjacent lanes by DPP; the tile is transposed
//    through LDS for the right and left sweeps. Sweeps repeat until the tile
//    is stable, then the interior is stored and the neighbours whose halo the
//    new border can still raise go on the next round's dirty list, which is
//    all that round visits.
//  * k_tile_queue -- the same visits without rounds: waves take tiles from a
//    device ring and mark neighbours straight into it, until none is left.
//  * k_seed -- one relaxation step over each tile still dirty after the last
//    round; every raised pixel is compacted by wave ballot into the tile's row
//    of the frontier bitmap, and the tile into the device frontier ring.
//  * k_queue -- persistent waves pop tiles from the ring, claim the set bits of
//    the tile's bitmap and propagate each claimed pixel to its neighbours with
//    atomic max updates; every raised neighbour is pushed back (bit set, its
//    tile enqueued once). The wave that retires the last entry stops them all.
#include <algorithm>

#include "mr_internal.h"

namespace mr {

template <typename T> struct Pix;
template <> struct Pix<uint8_t> {
    static constexpr uint32_t KMAX = 0xFFu;
    __device__ static __forceinline__ uint32_t key(uint8_t v) { return v; }
    __device__ static __forceinline__ uint8_t val(uint32_t k) { return (uint8_t)k; }
};
template <> struct Pix<int32_t> {
    static constexpr uint32_t KMAX = 0xFFFFFFFFu;
    __device__ static __forceinline__ uint32_t key(int32_t v) { return (uint32_t)v ^ 0x80000000u; }
    __device__ static __forceinline__ int32_t val(uint32_t k) { return (int32_t)(k ^ 0x80000000u); }
};

template <typename T> using gptr = __attribute__((address_space(1))) T *;
template <typename T> using cgptr = const __attribute__((address_space(1))) T *;

// Lane i receives lane i-1's value (lane 0 receives 0).
__device__ __forceinline__ uint32_t from_lower_lane(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x138 /* wave_shr:1 */, 0xF, 0xF, true);
}
// Lane i receives lane i+1's value (lane 63 receives 0).
__device__ __forceinline__ uint32_t from_upper_lane(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x130 /* wave_shl:1 */, 0xF, 0xF, true);
}

// Data that earlier launches wrote and this one only reads (descriptors,
// owner tables, the dirty lists and list lengths of the round being run),
// read through the scalar cache: uniform loads that wait on the scalar
// counter, not on the vector memory counter behind this wave's own loads
// and stores.
template <typename X> using kptr = const __attribute__((address_space(4))) X *;
template <typename X> __device__ __forceinline__ kptr<X> kconst(const X *p) {
    return (kptr<X>)p;
}

// Field-wise copy (the implicit copy constructor does not bind to a
// constant-address-space object).
__device__ __forceinline__ ImgDesc desc_at(kptr<ImgDesc> d, int64_t k) {
    ImgDesc r;
    r.J = d[k].J;
    r.I = d[k].I;
    r.out = d[k].out;
    r.H = d[k].H;
    r.W = d[k].W;
    r.pJ = d[k].pJ;
    r.pI = d[k].pI;
    r.tile_base = d[k].tile_base;
    r.first_round = d[k].first_round;
    r.ntx = d[k].ntx;
    r.nty = d[k].nty;
    r.op = d[k].op;
    r.done = d[k].done;
    r.wide = d[k].wide;
    return r;
}
static_assert(sizeof(ImgDesc) == 96, "desc_at copies every field of ImgDesc");

// Descriptor of the image that owns `tile` (owner table, else binary search
// on tile_base).
__device__ __forceinline__ ImgDesc load_desc(Imgs imgs, int64_t tile) {
    const kptr<ImgDesc> d = kconst(imgs.d);
    if (imgs.owner) return desc_at(d, kconst(imgs.owner)[tile]);
    int lo = 0, hi = imgs.n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (d[mid].tile_base <= tile) lo = mid;
        else hi = mid - 1;
    }
    return desc_at(d, lo);
}

// Coherent (device-scope) access to the working image, used while other
// waves update it with atomics.
template <typename T> struct Atom;
template <> struct Atom<int32_t> {
    __device__ static __forceinline__ uint32_t load_key(const int32_t *base, int64_t off) {
        const int32_t v = __hip_atomic_load(base + off, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return Pix<int32_t>::key(v);
    }
    // Raise the pixel to key k if it is lower; true if this call raised it.
    __device__ static __forceinline__ bool raise(int32_t *base, int64_t off, uint32_t k,
                                                 unsigned long long &retries) {
        (void)retries;
        const int32_t v = Pix<int32_t>::val(k);
        const int32_t old = __hip_atomic_fetch_max(base + off, v, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
        return old < v;
    }
};
template <> struct Atom<uint8_t> {
    __device__ static __forceinline__ uint32_t load_key(const uint8_t *base, int64_t off) {
        const uintptr_t a = (uintptr_t)(base + off);
        const uint32_t *w = (const uint32_t *)(a & ~(uintptr_t)3);
        const uint32_t sh = (uint32_t)(a & 3) * 8u;
        const uint32_t word = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return (word >> sh) & 0xFFu;
    }
    __device__ static __forceinline__ bool raise(uint8_t *base, int64_t off, uint32_t k,
                                                 unsigned long long &retries) {
        const uintptr_t a = (uintptr_t)(base + off);
        uint32_t *w = (uint32_t *)(a & ~(uintptr_t)3);
        const uint32_t sh = (uint32_t)(a & 3) * 8u;
        uint32_t old = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        while (true) {
            if (((old >> sh) & 0xFFu) >= k) return false;
            const uint32_t nw = (old & ~(0xFFu << sh)) | (k << sh);
            uint32_t expect = old;
            if (__hip_atomic_compare_exchange_strong(w, &expect, nw, __ATOMIC_RELAXED,
                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                return true;
            old = expect;
            ++retries;
        }
    }
};

// ------------------------------------------------------------------ tiles

// The tile kernels run one wave per block. LDS that some lanes write and
// others read needs only program order there (a wave's LDS operations are
// performed in the order they issue) and a compiler barrier; a workgroup
// barrier would also wait for every global load and store in flight.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}


// Buffer resource over one uint8 plane of `bytes` bytes, used only when the
// plane base and pitch are multiples of 16, so every 16-byte chunk load is
// aligned and the per-dword range check matches whole memory words. Loads past
// the end, or at the huge offsets used for rows outside the image, return 0.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void *p, uint64_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc((void *)p, (short)0,
                                             (int)(bytes < 0xFFFFFFF0ull ? (uint32_t)bytes : 0xFFFFFFF0u),
                                             0x00020000);
}

__device__ __forceinline__ bool stage_ok(const void *p, int64_t pitch) {
    return ((uintptr_t)p & 15) == 0 && (pitch & 15) == 0;
}

// uint8 staging: row r of a tile (image row gy0 + r) is fetched as five
// 16-byte chunks covering image columns a .. a+79, a = gx0 rounded down to 16,
// and kept in LDS at r * SROW. SROW is an odd number of dwords, so the row
// writes (lane = row) and the column reads (lane = column) are both free of
// bank conflicts.
constexpr int SROW = 84;
// Cache policy of loads that must see other compute units' stores at device
// scope (sc1: not served from a compute unit's or a die's non-coherent cache).
constexpr int CPOL_DEVICE = 16;
constexpr int STAGE_BYTES = TS * SROW;
static_assert(2 * STAGE_BYTES <= TS * (TS + 1) * 4, "the stage must fit in the transpose buffer");

typedef uint32_t v4u __attribute__((ext_vector_type(4)));

// Lane r fetches tile row r, chunk k per load. Staged planes have a pitch of
// at least 16 and H * pitch < 2^32, so rows and offsets fit 32 bits. The lane
// id goes through an empty asm so that nothing derived from it is hoisted out
// of the caller's tile loop: held across the sweeps, such values would be
// spilled, and every reload would wait for all memory operations in flight.
template <int CPOL = 0>
__device__ __forceinline__ void stage_issue(__amdgpu_buffer_rsrc_t rs, int64_t gy0, int64_t H,
                                            uint32_t pitch, int64_t a, int lane, v4u (&v)[5],
                                            bool live = true) {
    uint32_t ln = (uint32_t)lane;
    asm volatile("" : "+v"(ln));
    const int32_t gy = (int32_t)gy0 + (int32_t)ln;
    const bool rowok = live && gy >= 0 && gy < (int32_t)H;
    uint32_t off = (uint32_t)gy * pitch + (uint32_t)(int32_t)a;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        // a + 16 k < 0 only for chunk 0 of a tile at the left image edge;
        // below row 0 it reads the end of the previous row (outside pixels,
        // masked out later), in row 0 it is out of range
        const bool in = rowok && (gy > 0 || a + 16 * k >= 0);
        v[k] = __builtin_amdgcn_raw_buffer_load_b128(rs, in ? off : 0xFFFFFFF0u, 0, CPOL);
        off += 16;
    }
}

// Row `lane` of the stage at st gets the 80 bytes fetched by stage_issue.
__device__ __forceinline__ void stage_commit(const v4u (&v)[5], int lane, uint8_t *st) {
    uint32_t ln = (uint32_t)lane;
    asm volatile("" : "+v"(ln));
    uint32_t *w = (uint32_t *)(st + ln * SROW);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        w[4 * k + 0] = v[k].x;
        w[4 * k + 1] = v[k].y;
        w[4 * k + 2] = v[k].z;
        w[4 * k + 3] = v[k].w;
    }
}

template <int CPOL = 0>
__device__ __forceinline__ void stage_u8(__amdgpu_buffer_rsrc_t rs, int64_t gy0, int64_t H,
                                         uint32_t pitch, int64_t a, int lane, uint8_t *st) {
    v4u v[5];
    stage_issue<CPOL>(rs, gy0, H, pitch, a, lane, v);
    stage_commit(v, lane, st);
}

// A tile's stage rows in flight, held by value (mask words, working-image
// words) so that they stay in registers between the visit that fetches them
// and the one that commits them.
struct StageWords {
    v4u i0, i1, i2, i3, i4, j0, j1, j2, j3, j4;
};

// Issue the stage loads of tile t of image d (uint8, staged planes); with
// live false every load is out of the buffer's range (zeros, no memory
// access), so that the count of loads does not depend on the path.
template <bool NEEDJ>
__device__ __forceinline__ StageWords stage_fetch(const ImgDesc &d, int64_t t, int lane,
                                                  bool live = true) {
    const int64_t lt = t - d.tile_base;
    const int ty = (int)(lt / d.ntx), tx = (int)(lt - (int64_t)ty * d.ntx);
    const int64_t gy0 = (int64_t)ty * TI - 1, gx0 = (int64_t)tx * TI - 1;
    const int64_t a = gx0 & ~(int64_t)15;
    StageWords w;
    v4u v[5];
    stage_issue(plane_rsrc(d.I, (uint64_t)(d.H * d.pI)), gy0, d.H, (uint32_t)d.pI, a, lane, v, live);
    w.i0 = v[0];
    w.i1 = v[1];
    w.i2 = v[2];
    w.i3 = v[3];
    w.i4 = v[4];
    if (NEEDJ) {
        stage_issue(plane_rsrc(d.J, (uint64_t)(d.H * d.pJ)), gy0, d.H, (uint32_t)d.pJ, a, lane, v,
                    live);
        w.j0 = v[0];
        w.j1 = v[1];
        w.j2 = v[2];
        w.j3 = v[3];
        w.j4 = v[4];
    } else {
        w.j0 = w.j1 = w.j2 = w.j3 = w.j4 = v4u{0u, 0u, 0u, 0u};
    }
    return w;
}

template <bool NEEDJ>
__device__ __forceinline__ void stage_commit_words(const StageWords &w, int lane, uint8_t *st) {
    const v4u vi[5] = {w.i0, w.i1, w.i2, w.i3, w.i4};
    stage_commit(vi, lane, st);
    if (NEEDJ) {
        const v4u vj[5] = {w.j0, w.j1, w.j2, w.j3, w.j4};
        stage_commit(vj, lane, st + STAGE_BYTES);
    }
}

// A working-image element; COH reads it device-coherent.
template <typename T, bool COH>
__device__ __forceinline__ T load_j(cgptr<T> p, uint32_t off) {
    if (COH) return __hip_atomic_load((T *)(p + off), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return p[off];
}
template <typename T, bool COH>
__device__ __forceinline__ void store_j(gptr<T> p, uint32_t off, T v) {
    if (COH) __hip_atomic_store((T *)(p + off), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else p[off] = v;
}

// Load one 64 x 64 register tile. INITIAL builds the starting working image
// (reconstruction: min(marker, mask); fill-holes: the complement on the image
// border and the minimum inside) instead of reading it; FILL reads the input
// image and complements it into the mask. Outside pixels become key 0 in
// both, which keeps them at 0.
// The halo is not frozen: a sweep may raise a halo pixel from its in-tile
// neighbours. That is a true geodesic dilation step on real values, so every
// value stays at or below the reconstruction; halo values are never stored,
// and a tile at a fixed point against a raised halo is one against the stored
// halo as well (the dilation step is monotone).
// uint8 tiles whose planes are 16-byte aligned are staged through LDS
// (`stage`, at least 2 * STAGE_BYTES); other uint8 planes and int32 rows (which
// are already 256-byte coalesced loads) go straight to registers from
// clamped, in-bounds addresses. For staged tiles inside the image the
// transposed mask IT (lane = row, register = column) and the loaded halo
// columns JL, JR (lane = row) are read straight from the stage, and `it_done`
// says so.
// From a stage that holds the tile's mask rows (stage) and working-image rows
// (stage + STAGE_BYTES), written and synchronized: the register tile J, I
// (lane = column), and for tiles inside the image the transposed mask IT and
// the halo columns JL, JR (lane = row), with it_done set. Ends with a wave sync:
// the stage's memory is the transpose buffer afterwards.
template <typename T, bool FILL, bool INITIAL>
__device__ __forceinline__ void stage_read(const ImgDesc &d, int64_t gy0, int64_t gx0, int lane,
                                           uint32_t (&J)[TS], uint32_t (&I)[TS],
                                           uint32_t (&IT)[TS], uint32_t &JL, uint32_t &JR,
                                           const uint8_t *stage, bool &it_done) {
    using P = Pix<T>;
    const int64_t H = d.H, W = d.W;
    const int64_t gx = gx0 + lane;
    const bool xin = gx >= 0 && gx < W;
    const bool xedge = gx == 0 || gx == W - 1;
    const bool inside =
        !(FILL && INITIAL) && gy0 >= 0 && gy0 + TS <= H && gx0 >= 0 && gx0 + TS <= W;
    const int64_t a = gx0 & ~(int64_t)15;
    const int sh = (int)(gx0 - a) + lane;
    const uint8_t *stI = stage, *stJ = stage + STAGE_BYTES;
    if (inside) {
#pragma unroll
        for (int r = 0; r < TS; ++r) {
            uint32_t iv = stI[r * SROW + sh];
            if (FILL) iv = P::KMAX - iv;
            uint32_t jv = stJ[r * SROW + sh];
            if (INITIAL) jv = min(jv, iv);
            J[r] = jv;
            I[r] = iv;
        }
        // lane = row: this lane's row of the mask, and the working image's
        // two halo pixels of that row
        const uint8_t *row = stI + lane * SROW + (int)(gx0 - a);
#pragma unroll
        for (int c = 0; c < TS; ++c) {
            uint32_t v = row[c];
            if (FILL) v = P::KMAX - v;
            IT[c] = v;
        }
        const uint8_t *rowJ = stJ + lane * SROW + (int)(gx0 - a);
        JL = rowJ[0];
        JR = rowJ[TS - 1];
        if (INITIAL) {
            JL = min(JL, IT[0]);
            JR = min(JR, IT[TS - 1]);
        }
        it_done = true;
    } else {
#pragma unroll
        for (int r = 0; r < TS; ++r) {
            const int64_t gy = gy0 + r;
            const bool ok = xin && gy >= 0 && gy < H;
            uint32_t iv = stI[r * SROW + sh];
            if (FILL) iv = P::KMAX - iv;
            uint32_t jv;
            if (FILL && INITIAL)
                jv = (xedge || gy == 0 || gy == H - 1) ? iv : 0u;
            else if (INITIAL)
                jv = min((uint32_t)stJ[r * SROW + sh], iv);
            else
                jv = stJ[r * SROW + sh];
            jv = ok ? jv : 0u;
            iv = ok ? iv : 0u;
            J[r] = jv;
            I[r] = iv;
        }
    }
    wave_sync();
}

template <typename T, bool FILL, bool INITIAL, bool COH = false>
__device__ __forceinline__ void load_tile(const ImgDesc &d, int64_t gy0, int64_t gx0, int lane,
                                          uint32_t (&J)[TS], uint32_t (&I)[TS],
                                          uint32_t (&IT)[TS], uint32_t &JL, uint32_t &JR,
                                          uint8_t *stage, bool &it_done) {
    using P = Pix<T>;
    const int64_t H = d.H, W = d.W;
    const int64_t gx = gx0 + lane;
    const bool xin = gx >= 0 && gx < W;
    const bool xedge = gx == 0 || gx == W - 1;
    // The whole tile, halo included, lies inside the image (wave-uniform):
    // no pixel needs the outside rule. A fill-holes image's first visit also
    // needs to know the image border, so it always takes the general path.
    const bool inside =
        !(FILL && INITIAL) && gy0 >= 0 && gy0 + TS <= H && gx0 >= 0 && gx0 + TS <= W;
    if (sizeof(T) == 1 && stage_ok(d.I, d.pI) && stage_ok(d.J, d.pJ)) {
        const int64_t a = gx0 & ~(int64_t)15;
        uint8_t *stI = stage, *stJ = stage + STAGE_BYTES;
        stage_u8(plane_rsrc(d.I, (uint64_t)(H * d.pI)), gy0, H, (uint32_t)d.pI, a, lane, stI);
        const bool needJ = !(FILL && INITIAL);
        if (needJ)
            stage_u8<COH ? CPOL_DEVICE : 0>(plane_rsrc(d.J, (uint64_t)(H * d.pJ)), gy0, H,
                                            (uint32_t)d.pJ, a, lane, stJ);
        wave_sync();
        stage_read<T, FILL, INITIAL>(d, gy0, gx0, lane, J, I, IT, JL, JR, stage, it_done);
        return;
    }
    cgptr<T> Jp = (cgptr<T>)d.J;
    cgptr<T> Ip = (cgptr<T>)d.I;
    if (inside) {
        uint32_t oI = (uint32_t)gy0 * (uint32_t)d.pI + (uint32_t)gx;
        uint32_t oJ = (uint32_t)gy0 * (uint32_t)d.pJ + (uint32_t)gx;
#pragma unroll
        for (int r = 0; r < TS; ++r) {
            uint32_t iv = P::key(Ip[oI]);
            if (FILL) iv = P::KMAX - iv;
            uint32_t jv = P::key(load_j<T, COH>(Jp, oJ));
            if (INITIAL) jv = min(jv, iv);
            J[r] = jv;
            I[r] = iv;
            oI += (uint32_t)d.pI;
            oJ += (uint32_t)d.pJ;
        }
        return;
    }
    const uint32_t xc = (uint32_t)(gx < 0 ? 0 : (gx > W - 1 ? W - 1 : gx));
#pragma unroll
    for (int r = 0; r < TS; ++r) {
        const int64_t gy = gy0 + r;
        const bool ok = xin && gy >= 0 && gy < H;
        const uint32_t yc = (uint32_t)(gy < 0 ? 0 : (gy > H - 1 ? H - 1 : gy));
        uint32_t iv = P::key(Ip[yc * (uint32_t)d.pI + xc]);
        if (FILL) iv = P::KMAX - iv;
        uint32_t jv;
        if (INITIAL) {
            if (FILL)
                jv = (xedge || yc == 0 || yc == (uint32_t)(H - 1)) ? iv : 0u;
            else
                jv = min(P::key(load_j<T, COH>(Jp, yc * (uint32_t)d.pJ + xc)), iv);
        } else {
            jv = P::key(load_j<T, COH>(Jp, yc * (uint32_t)d.pJ + xc));
        }
        jv = ok ? jv : 0u;
        iv = ok ? iv : 0u;
        J[r] = jv;
        I[r] = iv;
    }
}

// Transpose a 64 x 64 register tile through LDS: afterwards lane l holds row
// l and register c holds column c.
__device__ __forceinline__ void transpose(uint32_t (&A)[TS], uint32_t (*tb)[TS + 1], int lane) {
#pragma unroll
    for (int r = 0; r < TS; ++r) tb[r][lane] = A[r];
    wave_sync();
#pragma unroll
    for (int c = 0; c < TS; ++c) A[c] = tb[lane][c];
    wave_sync();
}

// med3(j, n, i) = min(max(j, n), i) whenever j <= i, which holds for every
// key the kernels hold (the working image never exceeds the mask, and the
// frozen halo has i == j): one VALU instead of two.
__device__ __forceinline__ uint32_t med3(uint32_t j, uint32_t n, uint32_t i) {
    uint32_t r;
    asm("v_med3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(j), "v"(n), "v"(i));
    return r;
}

// One 8-connected row step: med3(j, max of u over lanes l-1, l, l+1, i).
// Both lane shifts ride on DPP max instructions. The leading s_nop covers the
// DPP read-after-VALU-write hazard on u, which is written by the previous
// row's step immediately before.
__device__ __forceinline__ uint32_t step3(uint32_t j, uint32_t u, uint32_t i) {
    uint32_t r, t;
    asm("s_nop 1\n\t"
        "v_max_u32_dpp %1, %2, %2 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_max_u32_dpp %1, %2, %1 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_med3_u32 %0, %3, %1, %4"
        : "=v"(r), "=&v"(t)
        : "v"(u), "v"(j), "v"(i));
    return r;
}

// Max over lanes l-1, l, l+1 (0 beyond the wave's ends).
__device__ __forceinline__ uint32_t max3_lanes(uint32_t u) {
    uint32_t t;
    asm("s_nop 1\n\t"
        "v_max_u32_dpp %0, %1, %1 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_max_u32_dpp %0, %1, %0 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1"
        : "=&v"(t)
        : "v"(u));
    return t;
}

// The halo columns 0 and TS-1 of a register tile, lane = row: lanes 0 and
// TS-1 write their registers to LDS and every lane reads its row back.
__device__ __forceinline__ void halo_cols(const uint32_t (&A)[TS], uint32_t (*tb)[TS + 1],
                                          int lane, uint32_t &cl, uint32_t &cr) {
    uint32_t *buf = &tb[0][0];
    if (lane == 0 || lane == TS - 1) {
        uint32_t *dst = buf + (lane == 0 ? 0 : TS);
#pragma unroll
        for (int r = 0; r < TS; ++r) dst[r] = A[r];
    }
    wave_sync();
    cl = buf[lane];
    cr = buf[TS + lane];
    wave_sync();
}

// Sweeps along the registers. With DIAG, A[r] takes the max over the three
// lanes of the previous register (the 3 neighbours in the previous row), else
// only the same lane; the result is limited by B[r]. Values only rise, so
// callers detect change by comparing column sums.
template <bool DIAG>
__device__ __forceinline__ void sweep_fwd(uint32_t (&A)[TS], const uint32_t (&B)[TS]) {
#pragma unroll
    for (int r = 1; r < TS - 1; ++r)
        A[r] = DIAG ? step3(A[r], A[r - 1], B[r]) : med3(A[r], A[r - 1], B[r]);
}

template <bool DIAG>
__device__ __forceinline__ void sweep_bwd(uint32_t (&A)[TS], const uint32_t (&B)[TS]) {
#pragma unroll
    for (int r = TS - 2; r >= 1; --r)
        A[r] = DIAG ? step3(A[r], A[r + 1], B[r]) : med3(A[r], A[r + 1], B[r]);
}

// One relaxation step over the interior rows: every pixel against all its
// neighbours. With 8-connectivity the step reads the values from before it;
// with 4-connectivity the row above is already updated. Both are valid
// steps, and a step that changes nothing means every pixel in rows 1..TS-2 is
// stable against all its neighbours.
template <int CONN>
__device__ __forceinline__ void relax_once(uint32_t (&J)[TS], const uint32_t (&I)[TS]) {
    if (CONN == 8) {
        uint32_t hp = max3_lanes(J[0]), hc = max3_lanes(J[1]);
#pragma unroll
        for (int r = 1; r < TS - 1; ++r) {
            const uint32_t hn = max3_lanes(J[r + 1]);
            J[r] = med3(J[r], max(max(hp, hc), hn), I[r]);
            hp = hc;
            hc = hn;
        }
    } else {
#pragma unroll
        for (int r = 1; r < TS - 1; ++r)
            J[r] = med3(J[r], max(max(J[r - 1], J[r + 1]), max3_lanes(J[r])), I[r]);
    }
}

// Sum of the interior rows of a column. Keys only rise, so the sum rises iff
// some key changed; 62 keys below 2^32 cannot overflow 64 bits, and 62 u8 keys
// cannot overflow 32.
template <typename T>
__device__ __forceinline__ uint64_t col_sum(const uint32_t (&A)[TS]) {
    if (sizeof(T) == 1) {
        uint32_t s = 0;
#pragma unroll
        for (int r = 1; r < TS - 1; ++r) s += A[r];
        return s;
    }
    uint64_t s = 0;
#pragma unroll
    for (int r = 1; r < TS - 1; ++r) s += A[r];
    return s;
}

// Tiles newly made dirty by one wave wait in an LDS batch and go to the next
// round's list with one counter update per batch, not one per tile.
__device__ __forceinline__ int64_t band_lo(int64_t n_tiles, int b) {
    return (int64_t)b * n_tiles / NBANDS;
}

__device__ __forceinline__ int band_of(int64_t n_tiles, int64_t t) {
    int b = (int)(t * NBANDS / n_tiles);
    while (b + 1 < NBANDS && band_lo(n_tiles, b + 1) <= t) ++b;
    while (b > 0 && band_lo(n_tiles, b) > t) --b;
    return b;
}

constexpr int APP_CAP = 64;
struct Appender {
    uint32_t *buf;      // LDS, APP_CAP entries
    uint32_t cnt;       // wave-uniform
    uint32_t *list_out; // next round's dirty lists (band b's at its band start)
    uint32_t *counter;  // their lengths, NBANDS of them
    int64_t n_tiles;
};

// Append the batch: each lane takes one entry, and each band present gets
// one counter update.
__device__ __forceinline__ void app_flush(Appender &a, int lane) {
    if (a.cnt == 0) return;
    asm volatile("" : "+v"(lane)); // (as in visit_tile)
    wave_sync();
    const bool valid = (uint32_t)lane < a.cnt;
    const uint32_t e = valid ? a.buf[lane] : 0u;
    const int be = valid ? band_of(a.n_tiles, e) : -1;
    // lane b < NBANDS reserves band b's share with one atomic; all of them
    // go out together, so the batch costs one round trip
    uint64_t mine = 0, under = 0;
#pragma unroll
    for (int b = 0; b < NBANDS; ++b) {
        const uint64_t m = __ballot(be == b);
        if (lane == b) mine = m;
        if (be == b) under = m & ((1ull << lane) - 1);
    }
    uint32_t base = 0;
    if (lane < NBANDS && mine) base = atomicAdd(a.counter + lane, (uint32_t)__popcll(mine));
    const uint32_t my_base = __shfl(base, be < 0 ? 0 : be);
    if (valid) a.list_out[band_lo(a.n_tiles, be) + my_base + __popcll(under)] = e;
    wave_sync();
    a.cnt = 0;
}

// ------------------------------------------------------------ frontier ring

// The ring holds tile ids; a tile is in it at most once (the seed pass and
// the queue phase: its qflag is 1 from enqueue until a wave finishes with
// it; the tile queue: its state), so it never holds more than the launch's
// tile count, and the capacity exceeds that plus one ticket per wave. The
// pusher has made what the entry stands for visible first: device-scope
// atomics it waited for, device-coherent stores it waited for, or stores of
// an earlier launch.
__device__ __forceinline__ void ring_push(Ctrl *ctrl, uint32_t *ring, uint64_t cap, uint32_t t) {
    __hip_atomic_fetch_add(&ctrl->pending.v, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long pos =
        __hip_atomic_fetch_add(&ctrl->q_tail.v, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint32_t *slot = ring + (pos & (cap - 1));
    // The capacity bound means the slot is already free; the wait is a guard,
    // capped so that a broken bound cannot hang the device. Past the cap the
    // entry is refused rather than written over another: its work is lost,
    // counted as an overflow and raised as the watchdog status, so the call
    // reports an incomplete result instead of returning a wrong one quietly.
    for (uint32_t spin = 0;
         __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != Q_EMPTY; ++spin) {
        if (spin > (1u << 22)) {
            atomicAdd(&ctrl->ovf[t & (NCNT - 1)], 1ull);
            atomicAdd(&ctrl->watchdog, 1ull);
            __hip_atomic_fetch_add(&ctrl->pending.v, (unsigned long long)-1ll, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            return;
        }
        __builtin_amdgcn_s_sleep(2);
    }
    __hip_atomic_store(slot, t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until this wave's memory operations are done (its device-coherent
// stores visible to every compute unit); also a compiler barrier.
__device__ __forceinline__ void wait_vmem() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Ring consumers take a ticket (the next position) and wait for that entry,
// so no two waves contend for one. An entry can legitimately take as long as
// the whole run (a long chain), so the watchdog fires only when no entry at
// all was pushed for wait_us microseconds (100 MHz constant clock): then the
// wave gives up with Q_STOP. One lane per wave calls it.
constexpr uint32_t Q_STOP = 0xFFFFFFFEu;

__device__ __forceinline__ uint32_t ring_take(Ctrl *ctrl, uint32_t *ring, uint64_t cap,
                                              unsigned long long wait_us) {
    const unsigned long long h =
        __hip_atomic_fetch_add(&ctrl->q_head.v, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint32_t *slot = ring + (h & (cap - 1));
    unsigned long long t0 = wall_clock64(), seen = h;
    uint32_t t;
    for (unsigned long long spin = 0;; ++spin) {
        t = __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (t != Q_EMPTY) break;
        if ((spin & 63) == 63 && wall_clock64() - t0 > wait_us * 100ull) {
            const unsigned long long tail =
                __hip_atomic_load(&ctrl->q_tail.v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (tail != seen) { // progress: wait on
                seen = tail;
                t0 = wall_clock64();
                continue;
            }
            atomicAdd(&ctrl->watchdog, 1ull);
            return Q_STOP;
        }
        if (spin < 32)
            __builtin_amdgcn_s_sleep(1);
        else
            __builtin_amdgcn_s_sleep(8);
    }
    if (t != Q_STOP)
        __hip_atomic_store(slot, Q_EMPTY, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return t;
}

// Retire one processed entry; the wave that retires the last one writes a
// stop entry for each of the launch's `waves` waves (each holds at most one
// ticket past the last entry).
__device__ __forceinline__ void ring_retire(Ctrl *ctrl, uint32_t *ring, uint64_t cap,
                                            unsigned waves) {
    const unsigned long long left = __hip_atomic_fetch_add(
        &ctrl->pending.v, (unsigned long long)-1ll, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (left != 1) return;
    const unsigned long long base = __hip_atomic_fetch_add(
        &ctrl->q_tail.v, (unsigned long long)waves, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (unsigned k = 0; k < waves; ++k)
        __hip_atomic_store(ring + ((base + k) & (cap - 1)), Q_STOP, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// Tile queue: a tile's state is 0 (idle), 1 (queued), 2 (a wave visits it)
// or 3 (visited and marked again meanwhile: it goes back on the ring when the
// visit ends). A mark sets bit 0; the one that finds the tile idle enqueues it.
// Tile-queue visits read and write the working image device-coherent and
// wait for their stores before any mark, so a visit that a mark leads to
// sees the marking visit's pixels without cache-wide fences.
struct TailQ {
    uint32_t *state;
    uint32_t *ring;
    uint64_t cap;
    Ctrl *ctrl;
};

__device__ __forceinline__ void tail_mark(const TailQ &q, uint32_t t) {
    const uint32_t prev =
        __hip_atomic_fetch_or(q.state + t, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (prev == 0u) ring_push(q.ctrl, q.ring, q.cap, t);
}

// One visit of one tile: load, sweep to a local fixed point (or the cap),
// store, and mark the neighbours whose halo changed: onto the next round's
// lists, or (TAIL) into the tile queue `tq`.
// Which tile this lane (0..8) asks to visit again: itself if the sweep cap
// stopped it, or the neighbour next to a changed border pixel that can still
// raise one of the neighbour's pixels in this tile's halo (min(mask, max of
// the adjacent border pixels) above the value the halo pixel had when this
// visit loaded it; pixels only rise, so a halo pixel that passes against its
// loaded value passes against its current one too). Rows 0 and TS-1 are
// checked in lanes 0..TS-1 (lane = column), columns 0 and TS-1 in lanes
// 0..TS-1 (lane = row), whose border columns 1 and TS-2 the last transpose
// left in LDS. Returns whether this lane wants tile `nb`.
template <int CONN>
__device__ __forceinline__ bool mark_decide(const ImgDesc &d, int lane, int ty, int tx,
                                            const uint32_t (&J)[TS], const uint32_t (&I)[TS],
                                            const uint32_t (&IT)[TS], uint32_t JT, uint32_t JB,
                                            uint32_t JL, uint32_t JR, uint32_t top_in,
                                            uint32_t bot_in, uint64_t col_in, uint64_t col_out,
                                            bool stable, uint32_t (*tb)[TS + 1], uint32_t &nb) {
    const bool in_lane = lane >= 1 && lane <= TS - 2;
    const uint64_t bt = __ballot(in_lane && J[1] != top_in);
    const uint64_t bb = __ballot(in_lane && J[TS - 2] != bot_in);
    const uint64_t bc = __ballot(col_out != col_in);
    const uint32_t b1 = in_lane ? J[1] : 0u, b2 = in_lane ? J[TS - 2] : 0u;
    const uint32_t c1 = in_lane ? tb[1][lane] : 0u, c2 = in_lane ? tb[TS - 2][lane] : 0u;
    const uint32_t nbT = CONN == 8 ? max3_lanes(b1) : b1, nbB = CONN == 8 ? max3_lanes(b2) : b2;
    const uint32_t nbL = CONN == 8 ? max3_lanes(c1) : c1, nbR = CONN == 8 ? max3_lanes(c2) : c2;
    const uint64_t rt = __ballot(med3(JT, nbT, I[0]) > JT);
    const uint64_t rb = __ballot(med3(JB, nbB, I[TS - 1]) > JB);
    // (after a relaxation step that still changed pixels at the sweep cap,
    // LDS holds the columns from before it: then every halo column counts)
    const uint64_t rl = stable ? __ballot(med3(JL, nbL, IT[0]) > JL) : ~0ull;
    const uint64_t rr = stable ? __ballot(med3(JR, nbR, IT[TS - 1]) > JR) : ~0ull;
    constexpr uint64_t EDGE = ~(1ull | (1ull << (TS - 1))); // lanes 1..TS-2
    bool want = false;
    int dy = 0, dx = 0;
    switch (lane) {
    case 0: want = !stable; break;
    case 1: want = bt != 0 && (rt & EDGE) != 0; dy = -1; break;
    case 2: want = bb != 0 && (rb & EDGE) != 0; dy = 1; break;
    case 3: want = ((bc >> 1) & 1) && (rl & EDGE) != 0; dx = -1; break;
    case 4: want = ((bc >> (TS - 2)) & 1) && (rr & EDGE) != 0; dx = 1; break;
    case 5: want = CONN == 8 && ((bt >> 1) & 1) && (rt & 1); dy = -1; dx = -1; break;
    case 6: want = CONN == 8 && ((bt >> (TS - 2)) & 1) && (rt >> (TS - 1)); dy = -1; dx = 1; break;
    case 7: want = CONN == 8 && ((bb >> 1) & 1) && (rb & 1); dy = 1; dx = -1; break;
    case 8: want = CONN == 8 && ((bb >> (TS - 2)) & 1) && (rb >> (TS - 1)); dy = 1; dx = 1; break;
    default: break;
    }
    const int ny = ty + dy, nx = tx + dx;
    want = want && ny >= 0 && ny < d.nty && nx >= 0 && nx < d.ntx;
    nb = want ? (uint32_t)(d.tile_base + (int64_t)ny * d.ntx + nx) : 0u;
    return want;
}

// The round path's marks: the wanted tiles get the next round in their
// epoch flag; the atomic maximum lets exactly one marker list a tile: the
// one that finds the flag below the next round. Returns the flag's previous
// value (the next round itself where this lane marks nothing), so that
// callers can compare it late and let the wait for the atomic overlap other
// work; the tile's id is in nb.
template <int CONN>
__device__ __forceinline__ uint32_t mark_neighbours(const ImgDesc &d, int lane, int ty, int tx,
                                                const uint32_t (&J)[TS], const uint32_t (&I)[TS],
                                                const uint32_t (&IT)[TS], uint32_t JT, uint32_t JB,
                                                uint32_t JL, uint32_t JR, uint32_t top_in,
                                                uint32_t bot_in, uint64_t col_in,
                                                uint64_t col_out, bool stable,
                                                uint32_t (*tb)[TS + 1], uint32_t *flags,
                                                uint32_t round, uint32_t &nb) {
    const bool want = mark_decide<CONN>(d, lane, ty, tx, J, I, IT, JT, JB, JL, JR, top_in,
                                        bot_in, col_in, col_out, stable, tb, nb);
    const uint32_t nxt = round + 1;
    uint32_t old = nxt;
    if (want) old = atomicMax(flags + nb, nxt);
    return old;
}

// PIPE (the pipelined round kernel; implies a stage the caller has written
// and synchronized): on the round path, after the marking atomics are issued
// and before the stores, the visit issues the stage loads of the next tile
// (*dn, tn) when has_next, and returns them; otherwise it returns zeros.
template <typename T, int CONN, bool FILL, bool INITIAL, bool TAIL = false, bool PIPE = false>
__device__ __forceinline__ StageWords visit_tile(const ImgDesc &d, int64_t t, int lane,
                                                 uint32_t *__restrict__ flags, Appender &app,
                                                 Ctrl *__restrict__ ctrl, uint32_t round,
                                                 int max_iters, uint32_t (*tb)[TS + 1],
                                                 const TailQ *tq = nullptr,
                                                 const ImgDesc *dn = nullptr, int64_t tn = 0,
                                                 bool has_next = false) {
    constexpr bool STAGED = PIPE;
    StageWords pre{};
    using P = Pix<T>;
    // nothing derived from the lane id is hoisted out of the caller's tile
    // loop: held across the sweeps, such values would be spilled, and their
    // reloads would wait behind the stores of the visit
    asm volatile("" : "+v"(lane));
    constexpr bool first = INITIAL;
    const int64_t lt = t - d.tile_base;
    const int ty = (int)(lt / d.ntx), tx = (int)(lt - (int64_t)ty * d.ntx);
    const int64_t gy0 = (int64_t)ty * TI - 1, gx = (int64_t)tx * TI - 1 + lane;

    uint32_t J[TS], I[TS], IT[TS];
    uint32_t JL, JR; // loaded halo columns 0 and TS-1, lane = row
    bool it_done = false;
    if (STAGED) // the caller has written and synchronized the stage
        stage_read<T, FILL, INITIAL>(d, gy0, (int64_t)tx * TI - 1, lane, J, I, IT, JL, JR,
                                     (const uint8_t *)tb, it_done);
    else
        load_tile<T, FILL, INITIAL, TAIL>(d, gy0, (int64_t)tx * TI - 1, lane, J, I, IT, JL, JR,
                                          (uint8_t *)tb, it_done);
    if (!it_done) {
        // (before the mask transpose: fewer registers live)
        halo_cols(J, tb, lane, JL, JR);
#pragma unroll
        for (int r = 0; r < TS; ++r) IT[r] = I[r];
        transpose(IT, tb, lane);
    }
    // loaded halo rows 0 and TS-1 (the sweeps may raise them in registers)
    const uint32_t JT = J[0], JB = J[TS - 1];

    const bool in_lane = lane >= 1 && lane <= TS - 2;
    const uint32_t top_in = J[1], bot_in = J[TS - 2];
    const uint64_t col_in = col_sum<T>(J);
    uint64_t col_prev = col_in;

    bool stable = false, changed = false;
    // Down and up sweeps take the 3 (8-connectivity) or 1 (4-connectivity)
    // neighbours of the adjacent row; on the transposed tile the right and
    // left sweeps take only the in-row neighbour, because the vertical sweeps
    // already test the diagonal ones. A full iteration that changes nothing
    // therefore means every pixel is stable against all its neighbours.
    // A full iteration that changes something mostly leaves the tile at its
    // fixed point; one relaxation step against all neighbours confirms that
    // at a fraction of an iteration's cost (no transposes), and otherwise
    // the iterations go on.
    int it = 0;
    while (it < max_iters) {
        sweep_fwd<CONN == 8>(J, I);
        sweep_bwd<CONN == 8>(J, I);
        transpose(J, tb, lane);
        sweep_fwd<false>(J, IT);
        sweep_bwd<false>(J, IT);
        transpose(J, tb, lane);
        ++it;
        uint64_t col_now = col_sum<T>(J);
        // halo columns may rise too, but only the interior must settle
        bool ch = in_lane && col_now != col_prev;
        col_prev = col_now;
        if (__ballot(ch) == 0) {
            stable = true;
            break;
        }
        changed = true;
        // (int32 visits start checking after the second iteration, which
        // measures faster for them; a first visit at its sweep cap leaves
        // the check out: the tile is left unstable, and so listed again)
        if (sizeof(T) == 4 && it < 2) continue;
        if (INITIAL && it >= max_iters) break;
        relax_once<CONN>(J, I);
        col_now = col_sum<T>(J);
        ch = in_lane && col_now != col_prev;
        col_prev = col_now;
        if (__ballot(ch) == 0) {
            stable = true;
            break;
        }
    }
    if (lane == 0) atomicAdd(&ctrl->iters[t & (NCNT - 1)], (unsigned long long)it);

    if (changed || first) {
        gptr<T> Jw = (gptr<T>)d.J;
        if (in_lane && gx < d.W) {
            // rows gy0+1 .. gy0+62 are all >= 0; only the last tile row may
            // run past the image
            const int64_t left = d.H - gy0 - 1;
            const int rows = left < TS - 2 ? (int)left : TS - 2;
            uint32_t off = (uint32_t)(gy0 + 1) * (uint32_t)d.pJ + (uint32_t)gx;
            if (rows == TS - 2) {
#pragma unroll
                for (int r = 1; r < TS - 1; ++r) {
                    asm volatile("" : "+v"(off));
                    store_j<T, TAIL>(Jw, off, P::val(J[r]));
                    off += (uint32_t)d.pJ;
                }
            } else {
#pragma unroll
                for (int r = 1; r < TS - 1; ++r) {
                    asm volatile("" : "+v"(off));
                    if (r <= rows) store_j<T, TAIL>(Jw, off, P::val(J[r]));
                    off += (uint32_t)d.pJ;
                }
            }
        }
    }
    // PIPE: the next tile's stage loads go out after this tile's stores and
    // mark atomics (on every path, with no loads when there is no next tile),
    // so that waiting for the marks does not wait for them, and they are in
    // flight while the marks are waited for and the list is appended to.
    // Nothing of the next tile may be loaded earlier (its registers would be
    // live across the sweeps).
    auto fetch_next = [&]() {
        if (PIPE) {
            asm volatile("" ::: "memory");
            pre = stage_fetch<!(FILL && INITIAL)>(*dn, tn, lane, has_next);
        }
    };
    if (!changed && stable) {
        fetch_next();
        return pre;
    }
    if (!TAIL) {
        uint32_t nb = 0;
        const uint32_t old =
            mark_neighbours<CONN>(d, lane, ty, tx, J, I, IT, JT, JB, JL, JR, top_in, bot_in,
                                  col_in, col_prev, stable, tb, flags, round, nb);
        fetch_next();
        // (an opaque use: the comparison stays here, behind the loads that
        // fetch_next issued, rather than right after the atomic)
        uint32_t o = old;
        asm volatile("" : "+v"(o));
        const bool fresh = o < round + 1;
        const uint64_t fm = __ballot(fresh);
        if (fresh) app.buf[app.cnt + __popcll(fm & ((1ull << lane) - 1))] = nb;
        app.cnt += (uint32_t)__popcll(fm);
        return pre;
    }
    uint32_t tnb = 0;
    const bool want = mark_decide<CONN>(d, lane, ty, tx, J, I, IT, JT, JB, JL, JR, top_in, bot_in,
                                        col_in, col_prev, stable, tb, tnb);
    // the visits these marks lead to must see this visit's stores
    wait_vmem();
    if (want) tail_mark(*tq, tnb);
    return pre;
}

// The tiles a block of a round visits: band `band`'s list (or, with
// all_tiles, the whole band), entries local, local + per, ... below n, from
// list_in (band start already applied). A round that lists no more tiles
// than the grid has blocks, but more in some band than that band has blocks,
// gives each tile a block of its own: the tail of a flood often sits in one
// or two bands, whose blocks would otherwise visit its tiles one after
// another while the rest of the grid idles. Block g takes entry g of the
// band lists laid end to end. When every band fits its blocks, the bands'
// dealing already gives each tile a block, and keeps neighbouring tiles on
// one die's L2.
struct RoundWork {
    int band;
    int64_t local, per, n, lo;
    const uint32_t *list_in;
    bool fwd;
    // walk the band's tiles in order (static interleave, as in an all-tiles
    // round) and visit those whose epoch flag holds this round, instead of
    // reading the list
    bool walk;
};

// all_tiles: 1 visits every tile (an image's first round), 0 the dirty
// lists, 2 the dirty lists or, for a band that lists at least half its
// tiles, the walk. A list is built in marking order, which scatters the
// tiles visited at one time over the band; the walk visits neighbouring
// tiles together, so they share the cache lines their rows straddle.
// The walk relies on what launch sequences that start at round 1 guarantee:
// a tile is listed for round r exactly when its flag reached r in round
// r - 1. A flag raised again (to r + 1) before the walk reads it means the
// tile is in the next round's list as well, so leaving it to that round
// loses nothing.
__device__ __forceinline__ RoundWork round_work(int64_t n_tiles, const uint32_t *lists,
                                                const uint32_t *counts_in, int all_tiles,
                                                uint32_t round) {
    RoundWork w;
    w.band = blockIdx.x % NBANDS;
    w.local = blockIdx.x / NBANDS;
    w.per = gridDim.x / NBANDS;
    w.walk = false;
    if (all_tiles == 1) {
        w.n = band_lo(n_tiles, w.band + 1) - band_lo(n_tiles, w.band);
    } else {
        uint32_t c[NBANDS], total = 0, cmax = 0;
#pragma unroll
        for (int q = 0; q < NBANDS; ++q) {
            c[q] = kconst(counts_in)[q];
            total += c[q];
            cmax = c[q] > cmax ? c[q] : cmax;
        }
        if (total <= gridDim.x && cmax > (uint32_t)w.per) {
            uint32_t i = blockIdx.x, cb = c[0];
            int b = 0;
#pragma unroll
            for (int q = 0; q < NBANDS - 1; ++q)
                if (b == q && i >= c[q]) {
                    i -= c[q];
                    b = q + 1;
                    cb = c[q + 1];
                }
            w.band = b;
            w.local = i;
            w.per = cb > 0 ? cb : 1; // one iteration: entry i (or n - 1 - i backward)
            w.n = blockIdx.x < total ? cb : 0;
        } else {
            w.n = kconst(counts_in)[w.band];
            const int64_t nb = band_lo(n_tiles, w.band + 1) - band_lo(n_tiles, w.band);
            if (all_tiles == 2 && w.n > 0 && 2 * w.n >= nb) {
                w.walk = true;
                w.n = nb;
            }
        }
    }
    w.lo = band_lo(n_tiles, w.band);
    w.list_in = lists + (round & 1) * n_tiles + w.lo;
    // Odd rounds walk the band forward, even rounds backward: a tile stored
    // early in a round is read by tiles visited later in it, so information
    // travels down the image within odd rounds and up it within even ones,
    // as in a raster / anti-raster pair of scans.
    w.fwd = (round & 1) != 0;
    return w;
}

__device__ __forceinline__ int64_t round_tile(const RoundWork &w, int all_tiles, int64_t i) {
    const int64_t k = w.fwd ? i : w.n - 1 - i;
    return all_tiles == 1 || w.walk ? w.lo + k : (int64_t)kconst(w.list_in)[k];
}

// The block's tiles of a round, in order: band entries local, local + per,
// ... below n. A walk reads the epoch flags of 64 entries at once and keeps
// those that hold the round.
struct TileCursor {
    int64_t i;     // next entry; walk: first entry of the next batch
    int64_t wi;    // walk: first entry of the current batch
    uint64_t mask; // walk: bit j set if entry wi + j * per is to be visited
};

__device__ __forceinline__ TileCursor cursor_start(const RoundWork &w) {
    return TileCursor{w.local, w.local, 0ull};
}

// The next tile, or -1 when the block has none left (wave-uniform).
__device__ __forceinline__ int64_t cursor_next(TileCursor &c, const RoundWork &w, int all_tiles,
                                               const uint32_t *flags, uint32_t round, int lane) {
    if (!w.walk) {
        if (c.i >= w.n) return -1;
        const int64_t t = round_tile(w, all_tiles, c.i);
        c.i += w.per;
        return t;
    }
    while (c.mask == 0) {
        if (c.i >= w.n) return -1;
        uint32_t ln = (uint32_t)lane;
        asm volatile("" : "+v"(ln));
        const int64_t e = c.i + (int64_t)ln * w.per;
        bool take = false;
        if (e < w.n) {
            const int64_t t = w.lo + (w.fwd ? e : w.n - 1 - e);
            take = __hip_atomic_load(flags + t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
                   round;
        }
        c.mask = __ballot(take);
        c.wi = c.i;
        c.i += 64 * w.per;
    }
    const int j = __builtin_ctzll(c.mask);
    c.mask &= c.mask - 1;
    return round_tile(w, all_tiles, c.wi + (int64_t)j * w.per);
}

// One tile round on a persistent grid (two waves per SIMD). Block b serves
// band b % NBANDS and visits either every tile of the band (all_tiles) or the
// band's dirty list (see round_work). Tiles are dealt to the band's blocks by
// static interleave, so no block gets more than one tile above another. A
// tile builds its image's initial working values in the image's first round.
// V selects the visit: -1 dispatches per tile on the image's op and first
// round (mixed batches, the server); otherwise (FILL << 1) | INITIAL for
// launches whose tiles all take the same visit, which keeps the other three
// variants' code, and their registers, out of the kernel.
template <typename T, int CONN, int V>
__global__ __launch_bounds__(64, 2) void k_tile_round(Imgs imgs, int64_t n_tiles,
                                                      uint32_t *__restrict__ flags,
                                                      uint32_t *__restrict__ lists,
                                                      const uint32_t *__restrict__ counts_in,
                                                      uint32_t *__restrict__ counts_out,
                                                      int all_tiles, Ctrl *__restrict__ ctrl,
                                                      uint32_t round, int max_iters) {
    __shared__ uint32_t tb[TS][TS + 1]; // transpose buffer (and load stage)
    __shared__ uint32_t abuf[APP_CAP];
    const int lane = threadIdx.x;
    const RoundWork w = round_work(n_tiles, lists, counts_in, all_tiles, round);
    Appender app{abuf, 0, lists + ((round + 1) & 1) * n_tiles, counts_out, n_tiles};
    TileCursor cur = cursor_start(w);
    for (int64_t t; (t = cursor_next(cur, w, all_tiles, flags, round, lane)) >= 0;) {
        const ImgDesc d = load_desc(imgs, t);
        if (V >= 0) {
            if (!d.done)
                visit_tile<T, CONN, (V >> 1) & 1, V & 1>(d, t, lane, flags, app, ctrl, round,
                                                         max_iters, tb);
        } else if (!d.done) {
            if (d.first_round == (int64_t)round) {
                if (d.op == MR_OP_FILL)
                    visit_tile<T, CONN, true, true>(d, t, lane, flags, app, ctrl, round, max_iters, tb);
                else
                    visit_tile<T, CONN, false, true>(d, t, lane, flags, app, ctrl, round, max_iters, tb);
            } else {
                if (d.op == MR_OP_FILL)
                    visit_tile<T, CONN, true, false>(d, t, lane, flags, app, ctrl, round, max_iters, tb);
                else
                    visit_tile<T, CONN, false, false>(d, t, lane, flags, app, ctrl, round, max_iters, tb);
            }
        }
        if (app.cnt > APP_CAP - 9) app_flush(app, lane);
    }
    app_flush(app, lane);
}

// The same round for launches whose images are all uint8 with 16-byte
// aligned planes and pitches and take one visit kind V, software-pipelined
// over the block's tiles: the stage loads of the next tile are issued during
// the current visit, after its marking atomics and before its stores, so
// that their memory latency (and that of the next list entry and
// descriptor) overlaps the current tile's stores and the wait for its marks
// instead of starting the next visit. The loads land in registers that the
// sweeps no longer need; the next visit writes them to the stage.
template <int CONN, int V>
__global__ __launch_bounds__(64, 2) void k_tile_round_pf(Imgs imgs, int64_t n_tiles,
                                                         uint32_t *__restrict__ flags,
                                                         uint32_t *__restrict__ lists,
                                                         const uint32_t *__restrict__ counts_in,
                                                         uint32_t *__restrict__ counts_out,
                                                         int all_tiles, Ctrl *__restrict__ ctrl,
                                                         uint32_t round, int max_iters) {
    constexpr bool FILL = (V >> 1) & 1, INITIAL = V & 1;
    constexpr bool needJ = !(FILL && INITIAL);
    __shared__ uint32_t tb[TS][TS + 1]; // transpose buffer and load stage
    __shared__ uint32_t abuf[APP_CAP];
    const int lane = threadIdx.x;
    const RoundWork w = round_work(n_tiles, lists, counts_in, all_tiles, round);
    Appender app{abuf, 0, lists + ((round + 1) & 1) * n_tiles, counts_out, n_tiles};
    uint8_t *stage = (uint8_t *)tb;
    TileCursor cur = cursor_start(w);
    int64_t t = cursor_next(cur, w, all_tiles, flags, round, lane);
    if (t >= 0) {
        ImgDesc d = load_desc(imgs, t);
        StageWords pre = stage_fetch<needJ>(d, t, lane);
        while (true) {
            // the fetched rows of tile t go to the stage; the previous visit's
            // last reads of the transpose buffer are behind this sync
            wave_sync();
            stage_commit_words<needJ>(pre, lane, stage);
            wave_sync();
            int64_t tn = cursor_next(cur, w, all_tiles, flags, round, lane);
            const bool has = tn >= 0;
            if (!has) tn = t;
            const ImgDesc dn = has ? load_desc(imgs, tn) : d;
            pre = visit_tile<uint8_t, CONN, FILL, INITIAL, false, true>(
                d, t, lane, flags, app, ctrl, round, max_iters, tb, nullptr, &dn, tn, has);
            if (app.cnt > APP_CAP - 9) app_flush(app, lane);
            if (!has) break;
            t = tn;
            d = dn;
        }
    }
    app_flush(app, lane);
}

// ------------------------------------------------------------- tile queue

// Seeds the tile queue with band b's dirty list of `round` (block b).
__global__ void k_tile_queue_seed(const uint32_t *__restrict__ lists,
                                  const uint32_t *__restrict__ counts, int64_t n_tiles,
                                  uint32_t round, uint32_t *__restrict__ state,
                                  uint32_t *__restrict__ ring, uint64_t cap, Ctrl *ctrl) {
    __shared__ unsigned long long base;
    const int b = blockIdx.x;
    const uint32_t n = counts[b];
    if (n == 0) return;
    const uint32_t *list = lists + (round & 1) * n_tiles + band_lo(n_tiles, b);
    if (threadIdx.x == 0) {
        base = atomicAdd(&ctrl->q_tail.v, (unsigned long long)n);
        atomicAdd(&ctrl->pending.v, (unsigned long long)n);
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
        const uint32_t t = list[i];
        state[t] = 1u;
        ring[(base + i) & (cap - 1)] = t;
    }
}

// The tile queue (the regular phase without rounds): each wave takes a tile
// off the ring, visits it like a tile round does, and marks the neighbours
// straight into the ring, so a chain of dependent tiles costs one visit per
// link instead of one round. A wave takes a ticket (the next ring position)
// and waits for that entry, so no two waves contend for an entry. The wave
// that retires the last queued-or-running tile writes a stop entry for every
// wave. The watchdog (ring_take) turns a stall into an error instead of a hang.

template <typename T, int CONN, int V>
__global__ __launch_bounds__(64, 2) void k_tile_queue(Imgs imgs, Ctrl *__restrict__ ctrl,
                                                      uint32_t *__restrict__ state,
                                                      uint32_t *__restrict__ ring, uint64_t cap,
                                                      int max_iters,
                                                      unsigned long long wait_us) {
    __shared__ uint32_t tb[TS][TS + 1];
    const int lane = threadIdx.x;
    const TailQ tq{state, ring, cap, ctrl};
    Appender app{nullptr, 0, nullptr, nullptr, 0}; // unused: marks go to the ring
    unsigned long long visits = 0;
    // nothing seeded: no wave will ever retire a tile and write the stops
    if (__hip_atomic_load(&ctrl->pending.v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
        return;
    while (true) {
        uint32_t t = Q_EMPTY;
        if (lane == 0) t = ring_take(ctrl, ring, cap, wait_us);
        t = __shfl(t, 0);
        if (t == Q_STOP) break;
        // queued -> visited, performed before any pixel is read: a mark that
        // comes later finds state 2 and gets the tile visited again, one that
        // came earlier had its stores done before it
        if (lane == 0)
            (void)__hip_atomic_exchange(state + t, 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        wait_vmem();
        const ImgDesc d = load_desc(imgs, t);
        if (!d.done) {
            ++visits;
            if (V >= 0) {
                visit_tile<T, CONN, (V >> 1) & 1, false, true>(d, t, lane, nullptr, app, ctrl, 0,
                                                               max_iters, tb, &tq);
            } else if (d.op == MR_OP_FILL) {
                visit_tile<T, CONN, true, false, true>(d, t, lane, nullptr, app, ctrl, 0,
                                                       max_iters, tb, &tq);
            } else {
                visit_tile<T, CONN, false, false, true>(d, t, lane, nullptr, app, ctrl, 0,
                                                        max_iters, tb, &tq);
            }
        }
        wait_vmem();
        if (lane == 0) {
            uint32_t expect = 2u;
            if (!__hip_atomic_compare_exchange_strong(state + t, &expect, 0u, __ATOMIC_RELAXED,
                                                      __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT)) {
                // marked while it was visited (state 3): queue it again
                __hip_atomic_store(state + t, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ring_push(ctrl, ring, cap, t);
            }
            wait_vmem();
            ring_retire(ctrl, ring, cap, gridDim.x);
        }
    }
    if (lane == 0 && visits)
        atomicAdd(&ctrl->tiles[(blockIdx.x) & (NCNT - 1)], visits);
}

// ------------------------------------------------------------------- seeds

// One relaxation step over each tile still dirty for `round`: every interior
// pixel takes min(I, max of J over itself and its neighbours). Raised pixels
// are stored, their bits form the tile's frontier bitmap rows, and the tile
// enters the ring. Tiles that are not dirty only clear their bitmap and flag.
template <typename T, int CONN, bool FILL>
__device__ __forceinline__ void seed_tile(const ImgDesc &d, int64_t t, int lane, Ctrl *ctrl,
                                          uint64_t *bitmap, uint32_t *qflag, uint32_t *ring,
                                          uint64_t cap, uint8_t *stage) {
    using P = Pix<T>;
    const int64_t lt = t - d.tile_base;
    const int ty = (int)(lt / d.ntx), tx = (int)(lt - (int64_t)ty * d.ntx);
    const int64_t gy0 = (int64_t)ty * TI - 1, gx = (int64_t)tx * TI - 1 + lane;
    uint32_t J[TS], I[TS], IT[TS], JL, JR;
    bool it_done = false;
    load_tile<T, FILL, false>(d, gy0, (int64_t)tx * TI - 1, lane, J, I, IT, JL, JR, stage,
                              it_done);
    uint64_t myrow = 0; // lane r ends up holding row r's bits
    uint32_t nseed = 0;
    gptr<T> Jw = (gptr<T>)d.J;
    uint32_t off = (uint32_t)gy0 * (uint32_t)d.pJ + (uint32_t)gx;
#pragma unroll
    for (int r = 1; r < TS - 1; ++r) {
        off += (uint32_t)d.pJ;
        uint32_t n = max(J[r - 1], J[r + 1]);
        n = max(n, max(from_lower_lane(J[r]), from_upper_lane(J[r])));
        if (CONN == 8) {
            n = max(n, max(from_lower_lane(J[r - 1]), from_upper_lane(J[r - 1])));
            n = max(n, max(from_lower_lane(J[r + 1]), from_upper_lane(J[r + 1])));
        }
        const uint32_t v = min(max(J[r], n), I[r]);
        // only this tile's own pixels: the halo columns belong to the
        // neighbours (outside pixels have I == J == 0 and never rise)
        const bool raised = lane >= 1 && lane <= TS - 2 && v > J[r];
        const uint64_t bits = __ballot(raised);
        if (raised) Jw[off] = P::val(v);
        if (lane == r) myrow = bits;
        nseed += (uint32_t)__popcll(bits);
    }
    bitmap[t * TS + lane] = myrow;
    if (lane == 0 && nseed) {
        qflag[t] = 1;
        __hip_atomic_fetch_add(&ctrl->seeds_total.v, (unsigned long long)nseed,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // the queue runs in a later launch, which sees this one's stores
        ring_push(ctrl, ring, cap, (uint32_t)t);
    }
}

// One relaxation step over each tile dirty for `round` (the round after the
// last one run): every interior pixel takes min(I, max of J over itself and
// its neighbours). Raised pixels are stored, their bits form the tile's rows
// of the frontier bitmap (one ballot per row), and the tile enters the
// frontier ring. The bitmap and queue flags start cleared.
template <typename T, int CONN>
__global__ __launch_bounds__(64) void k_seed(Imgs imgs, int64_t n_tiles,
                                             const uint32_t *__restrict__ lists, uint32_t round,
                                             Ctrl *__restrict__ ctrl,
                                             uint64_t *__restrict__ bitmap,
                                             uint32_t *__restrict__ qflag,
                                             uint32_t *__restrict__ ring, uint64_t cap) {
    __shared__ uint8_t stage[2 * STAGE_BYTES];
    const int lane = threadIdx.x;
    const int band = blockIdx.x % NBANDS;
    const int64_t local = blockIdx.x / NBANDS, per = gridDim.x / NBANDS;
    const uint32_t *list_in = lists + (round & 1) * n_tiles + band_lo(n_tiles, band);
    const int64_t n = ctrl->round_tiles[round][band];
    for (int64_t i = local; i < n; i += per) {
        const int64_t t = list_in[i];
        const ImgDesc d = load_desc(imgs, t);
        if (d.done) continue;
        if (d.op == MR_OP_FILL)
            seed_tile<T, CONN, true>(d, t, lane, ctrl, bitmap, qflag, ring, cap, stage);
        else
            seed_tile<T, CONN, false>(d, t, lane, ctrl, bitmap, qflag, ring, cap, stage);
    }
}

// ------------------------------------------------------------------- queue

constexpr int QWAVES = 4;                  // waves per queue workgroup
constexpr int LIST_CAP = TI * TI;          // claimed pixels of one tile

// Process one claimed pixel: propagate its value to every neighbour that it
// can raise (Algorithm 1's PropagationCondition / Update), pushing each
// neighbour actually raised.
template <typename T, int CONN>
__device__ __forceinline__ void relax_pixel(const ImgDesc &d, int64_t y, int64_t x, Ctrl *ctrl,
                                            uint64_t *bitmap, uint32_t *qflag, uint32_t *ring,
                                            uint64_t cap, uint32_t &npush,
                                            unsigned long long &retries) {
    using P = Pix<T>;
    T *Jw = (T *)d.J;
    cgptr<T> Ip = (cgptr<T>)d.I;
    const bool fill = d.op == MR_OP_FILL;
    // uint8 images with a widened plane raise 32-bit keys there
    uint32_t *Wd = sizeof(T) == 1 ? d.wide : nullptr;
    auto load_key = [&](int64_t yy, int64_t xx) -> uint32_t {
        if (Wd)
            return __hip_atomic_load(Wd + yy * d.W + xx, __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT);
        return Atom<T>::load_key(Jw, yy * d.pJ + xx);
    };
    auto raise = [&](int64_t yy, int64_t xx, uint32_t k) -> bool {
        if (Wd)
            return __hip_atomic_fetch_max(Wd + yy * d.W + xx, k, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT) < k;
        return Atom<T>::raise(Jw, yy * d.pJ + xx, k, retries);
    };
    const uint32_t jp = load_key(y, x);
#pragma unroll
    for (int k = 0; k < CONN; ++k) {
        // edge neighbours first, then diagonals
        const int dy = (k == 0) ? -1 : (k == 1) ? 1 : (k < 4) ? 0 : (k < 6 ? -1 : 1);
        const int dx = (k < 2) ? 0 : (k == 2) ? -1 : (k == 3) ? 1 : ((k & 1) ? 1 : -1);
        const int64_t yy = y + dy, xx = x + dx;
        if (yy < 0 || yy >= d.H || xx < 0 || xx >= d.W) continue;
        const uint32_t jq = load_key(yy, xx);
        if (jq >= jp) continue;
        uint32_t iq = P::key(Ip[yy * d.pI + xx]);
        if (fill) iq = P::KMAX - iq;
        if (jq >= iq) continue;
        const uint32_t v = min(jp, iq);
        if (!raise(yy, xx, v)) continue;
        // push: set the pixel's frontier bit, enqueue its tile once
        const int tyq = (int)(yy / TI), txq = (int)(xx / TI);
        const int rq = (int)(yy - (int64_t)tyq * TI) + 1, lq = (int)(xx - (int64_t)txq * TI) + 1;
        const int64_t tq = d.tile_base + (int64_t)tyq * d.ntx + txq;
        const uint64_t bit = 1ull << lq;
        // the raise above returned, so it is done before the bit is set
        const uint64_t old = __hip_atomic_fetch_or(bitmap + tq * TS + rq, bit, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
        ++npush;
        if (old & bit) continue;
        if (__hip_atomic_exchange(qflag + tq, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
            ring_push(ctrl, ring, cap, (uint32_t)tq);
    }
}

template <typename T, int CONN>
__global__ __launch_bounds__(64 * QWAVES) void k_queue(Imgs imgs, Ctrl *__restrict__ ctrl,
                                                       uint64_t *__restrict__ bitmap,
                                                       uint32_t *__restrict__ qflag,
                                                       uint32_t *__restrict__ ring, uint64_t cap,
                                                       unsigned long long wait_us) {
    __shared__ uint16_t list[QWAVES][LIST_CAP];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    uint16_t *mylist = list[w];
    uint32_t npush = 0, npop = 0;
    unsigned long long retries = 0;
    const int cslot = (int)((blockIdx.x * QWAVES + w) & (NCNT - 1));
    // Every access that other waves' work depends on is a device-scope
    // atomic (pixels, bitmap rows, queue flags, ring), each waited for where
    // a later one must see it: no cache-wide fences. Nothing seeded: no wave
    // would ever retire an entry and write the stops.
    if (__hip_atomic_load(&ctrl->pending.v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
        return;

    while (true) {
        uint32_t t = Q_EMPTY;
        if (lane == 0) t = ring_take(ctrl, ring, cap, wait_us);
        t = __shfl(t, 0);
        if (t == Q_STOP) break;
        const ImgDesc d = load_desc(imgs, t);
        const int64_t lt = (int64_t)t - d.tile_base;
        const int ty = (int)(lt / d.ntx), tx = (int)(lt - (int64_t)ty * d.ntx);
        const int64_t gy0 = (int64_t)ty * TI - 1, gx0 = (int64_t)tx * TI - 1;
        uint64_t *rows = bitmap + (int64_t)t * TS;
        bool released = false;
        while (true) {
            uint64_t bits = __hip_atomic_exchange(rows + lane, 0ull, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
            if (__ballot(bits != 0) == 0) {
                if (released) break;
                // let pushes enqueue the tile again, then look once more (the
                // store is done before the rows are read again)
                if (lane == 0)
                    __hip_atomic_store(qflag + t, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                wait_vmem();
                released = true;
                continue;
            }
            // compact the claimed bits into a pixel list (row << 8 | lane)
            const uint32_t c = (uint32_t)__popcll(bits);
            uint32_t off = c; // inclusive scan over lanes
#pragma unroll
            for (int s = 1; s < 64; s <<= 1) {
                const uint32_t o = __shfl_up(off, s);
                if (lane >= s) off += o;
            }
            const uint32_t total = __shfl(off, 63);
            off -= c;
            while (bits) {
                const int l = __ffsll((unsigned long long)bits) - 1;
                bits &= bits - 1;
                mylist[off++] = (uint16_t)((lane << 8) | l);
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
            __builtin_amdgcn_wave_barrier();
            for (uint32_t base = 0; base < total; base += 64) {
                const uint32_t k = base + lane;
                if (k < total) {
                    const uint32_t e = mylist[k];
                    const int64_t y = gy0 + (e >> 8), x = gx0 + (e & 0xFF);
                    relax_pixel<T, CONN>(d, y, x, ctrl, bitmap, qflag, ring, cap, npush, retries);
                }
            }
            npop += total;
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
            __builtin_amdgcn_wave_barrier();
            if (released) {
                // bits arrived after the release; own the tile again if nobody
                // re-enqueued it, else leave the rest to the new entry
                uint32_t prev = 0;
                if (lane == 0)
                    prev = __hip_atomic_exchange(qflag + t, 1u, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
                prev = __shfl(prev, 0);
                if (prev != 0) break;
                released = false;
            }
        }
        // everything this tile produced is pushed; retire the ring entry
        wait_vmem();
        if (lane == 0) ring_retire(ctrl, ring, cap, gridDim.x * QWAVES);
    }
    // fold the per-lane counters
    unsigned long long p = npush, r = retries;
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) {
        p += __shfl_xor(p, s);
        r += __shfl_xor(r, s);
    }
    if (lane == 0) {
        atomicAdd(&ctrl->pushes[cslot], p);
        atomicAdd(&ctrl->pops[cslot], (unsigned long long)npop);
        atomicAdd(&ctrl->cas[cslot], r);
    }
}

// ------------------------------------------------------------ small kernels

__global__ void k_clear_u32(uint32_t *p, int64_t n, uint32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_clear_ctrl(Ctrl *c, int64_t n_tiles) {
    unsigned long long *p = (unsigned long long *)c;
    const int n = (int)(sizeof(Ctrl) / sizeof(unsigned long long));
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
    __syncthreads();
    if (threadIdx.x < NBANDS)
        c->round_tiles[1][threadIdx.x] =
            (uint32_t)(band_lo(n_tiles, threadIdx.x + 1) - band_lo(n_tiles, threadIdx.x));
}

// The start of a launch sequence in one kernel: the control block (block 0;
// round 1 lists every tile of each band), the dirty flags, and the queue
// flags and ring of the tile queue and the queue phase.
__global__ void k_clear_start(Ctrl *c, int64_t n_tiles, uint32_t *flags, uint32_t *qflag,
                              uint32_t *ring, int64_t ring_cap) {
    if (blockIdx.x == 0) {
        unsigned long long *p = (unsigned long long *)c;
        const int n = (int)(sizeof(Ctrl) / sizeof(unsigned long long));
        for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
        __syncthreads();
        if (threadIdx.x < NBANDS)
            c->round_tiles[1][threadIdx.x] =
                (uint32_t)(band_lo(n_tiles, threadIdx.x + 1) - band_lo(n_tiles, threadIdx.x));
    }
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_tiles; i += stride) {
        flags[i] = 0u;
        qflag[i] = 0u;
    }
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < ring_cap; i += stride)
        ring[i] = Q_EMPTY;
}

// The queue phase's widened planes (uint8 images): block t copies tile t's
// interior between J and the image's 32-bit plane, lane = column.
template <bool TO_WIDE>
__global__ __launch_bounds__(64) void k_widen(Imgs imgs, int64_t t0) {
    const int64_t t = t0 + blockIdx.x;
    const ImgDesc d = load_desc(imgs, t);
    if (!d.wide) return;
    const int lane = threadIdx.x;
    const int64_t lt = t - d.tile_base;
    const int64_t ty = lt / d.ntx, tx = lt - ty * d.ntx;
    const int64_t x = tx * TI + lane - 1;
    if (lane < 1 || lane > TI || x >= d.W) return;
    uint8_t *J = (uint8_t *)d.J;
    for (int64_t y = ty * TI, ye = std::min<int64_t>(y + TI, d.H); y < ye; ++y) {
        if (TO_WIDE)
            d.wide[y * d.W + x] = J[y * d.pJ + x];
        else
            J[y * d.pJ + x] = (uint8_t)d.wide[y * d.W + x];
    }
}

// Fill-holes epilogue: out = NOT J over the interior of every tile of the
// launch whose image is a fill-holes image.
template <typename T>
__global__ __launch_bounds__(64) void k_fill_output(Imgs imgs, int64_t t0) {
    using P = Pix<T>;
    const int64_t t = t0 + blockIdx.x;
    const int lane = threadIdx.x;
    const ImgDesc d = load_desc(imgs, t);
    if (d.op != MR_OP_FILL || d.done) return;
    const int64_t lt = t - d.tile_base;
    const int ty = (int)(lt / d.ntx), tx = (int)(lt - (int64_t)ty * d.ntx);
    const int64_t gx = (int64_t)tx * TI - 1 + lane;
    if (lane < 1 || lane > TS - 2 || gx >= d.W) return;
    cgptr<T> Jp = (cgptr<T>)d.J;
    gptr<T> O = (gptr<T>)d.out;
    for (int r = 1; r < TS - 1; ++r) {
        const int64_t gy = (int64_t)ty * TI - 1 + r;
        if (gy >= d.H) break;
        O[gy * d.pI + gx] = P::val(P::KMAX - P::key(Jp[gy * d.pJ + gx]));
    }
}

__global__ void k_store_u64(unsigned long long *p, unsigned long long v) { *p = v; }

__global__ void k_put_desc(ImgDesc *dst, ImgDesc v) { *dst = v; }

struct DescChunk {
    ImgDesc d[DESC_CHUNK];
    int n;
};

__global__ void k_put_descs(ImgDesc *dst, DescChunk c) {
    if ((int)threadIdx.x < c.n) dst[threadIdx.x] = c.d[threadIdx.x];
}

// ------------------------------------------------------------------ server

// Admit one image: its descriptor, owner[t] for its tiles, and every one of
// its tiles on the dirty list of `round` (where it builds its initial
// values). One thread per tile.
__global__ void k_server_admit(ImgDesc *descs, int32_t slot, ImgDesc d, uint32_t *owner,
                               uint32_t *flags, uint32_t *lists_round, uint32_t *counts_round,
                               int64_t n_tiles, uint32_t round) {
    const int64_t nt = (int64_t)d.ntx * d.nty;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i == 0) descs[slot] = d;
    if (i >= nt) return;
    const int64_t t = d.tile_base + i;
    owner[t] = (uint32_t)slot;
    flags[t] = round;
    const int b = band_of(n_tiles, t);
    const uint32_t pos = atomicAdd(counts_round + b, 1u);
    lists_round[band_lo(n_tiles, b) + pos] = (uint32_t)t;
}

// busy[image] = stamp for every image with a tile on the round's lists.
__global__ void k_server_status(const uint32_t *lists_round, const uint32_t *counts_round,
                                const uint32_t *owner, uint32_t *busy, int64_t n_tiles,
                                uint32_t stamp) {
    const int b = blockIdx.x % NBANDS;
    const int64_t per = (gridDim.x / NBANDS) * (int64_t)blockDim.x;
    const int64_t n = counts_round[b];
    const uint32_t *l = lists_round + band_lo(n_tiles, b);
    for (int64_t i = (blockIdx.x / NBANDS) * (int64_t)blockDim.x + threadIdx.x; i < n; i += per)
        busy[owner[l[i]]] = stamp;
}

// ---------------------------------------------------------------- launchers

int persistent_grid() {
    static int g = 0;
    if (!g) {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            cus > 0)
            g = cus * 8;
        else
            g = 2048;
    }
    return g;
}

hipError_t launch_server_admit(ImgDesc *descs, int32_t slot, const ImgDesc &d, uint32_t *owner,
                               uint32_t *flags, uint32_t *lists_round, uint32_t *counts_round,
                               int64_t n_tiles, uint32_t round, hipStream_t s) {
    const int64_t nt = std::max<int64_t>(1, (int64_t)d.ntx * d.nty);
    hipLaunchKernelGGL(k_server_admit, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, descs,
                       slot, d, owner, flags, lists_round, counts_round, n_tiles, round);
    return hipGetLastError();
}

hipError_t launch_server_status(const uint32_t *lists_round, const uint32_t *counts_round,
                                const uint32_t *owner, uint32_t *busy, int64_t n_tiles,
                                uint32_t stamp, hipStream_t s) {
    hipLaunchKernelGGL(k_server_status, dim3(NBANDS * 32), dim3(256), 0, s, lists_round,
                       counts_round, owner, busy, n_tiles, stamp);
    return hipGetLastError();
}

hipError_t launch_clear_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_clear_u32, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_clear_ctrl(Ctrl *c, int64_t n_tiles, hipStream_t s) {
    hipLaunchKernelGGL(k_clear_ctrl, dim3(1), dim3(256), 0, s, c, n_tiles);
    return hipGetLastError();
}
hipError_t launch_clear_start(Ctrl *c, int64_t n_tiles, uint32_t *flags, uint32_t *qflag,
                              uint32_t *ring, int64_t ring_cap, hipStream_t s) {
    const int64_t n = std::max<int64_t>(n_tiles, ring_cap);
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096));
    hipLaunchKernelGGL(k_clear_start, dim3((unsigned)blocks), dim3(256), 0, s, c, n_tiles, flags,
                       qflag, ring, ring_cap);
    return hipGetLastError();
}

template <typename T, int CONN, int V>
static hipError_t tile_round_v(const Imgs &imgs, int64_t n_tiles, uint32_t *flags,
                               uint32_t *lists, const uint32_t *cin, uint32_t *cout, int all,
                               Ctrl *ctrl, uint32_t round, int max_iters, int grid,
                               hipStream_t s) {
    const int64_t want = std::max<int64_t>(NBANDS, (n_tiles + NBANDS - 1) / NBANDS * NBANDS);
    const unsigned g = (unsigned)(std::min<int64_t>(grid, want) / NBANDS * NBANDS);
    if (sizeof(T) == 1 && V >= 0 && imgs.staged)
        hipLaunchKernelGGL((k_tile_round_pf<CONN, (V < 0 ? 0 : V)>), dim3(g), dim3(64), 0, s, imgs,
                           n_tiles, flags, lists, cin, cout, all, ctrl, round, max_iters);
    else
        hipLaunchKernelGGL((k_tile_round<T, CONN, V>), dim3(g), dim3(64), 0, s, imgs, n_tiles,
                           flags, lists, cin, cout, all, ctrl, round, max_iters);
    return hipGetLastError();
}

template <typename T, int CONN>
static hipError_t tile_round_t(const Imgs &imgs, int64_t n_tiles, uint32_t *flags,
                               uint32_t *lists, const uint32_t *cin, uint32_t *cout, int all,
                               Ctrl *ctrl, uint32_t round, int max_iters, int grid,
                               hipStream_t s, int variant) {
    switch (variant) {
    case 0: return tile_round_v<T, CONN, 0>(imgs, n_tiles, flags, lists, cin, cout, all, ctrl, round, max_iters, grid, s);
    case 1: return tile_round_v<T, CONN, 1>(imgs, n_tiles, flags, lists, cin, cout, all, ctrl, round, max_iters, grid, s);
    case 2: return tile_round_v<T, CONN, 2>(imgs, n_tiles, flags, lists, cin, cout, all, ctrl, round, max_iters, grid, s);
    case 3: return tile_round_v<T, CONN, 3>(imgs, n_tiles, flags, lists, cin, cout, all, ctrl, round, max_iters, grid, s);
    default: return tile_round_v<T, CONN, -1>(imgs, n_tiles, flags, lists, cin, cout, all, ctrl, round, max_iters, grid, s);
    }
}

static hipError_t tile_round_any(int tbytes, int conn, const Imgs &imgs, int64_t n_tiles,
                                 uint32_t *flags, uint32_t *lists, const uint32_t *cin,
                                 uint32_t *cout, int all, Ctrl *ctrl, uint32_t round,
                                 int max_iters, int grid, hipStream_t s, int variant) {
    if (!ctrl) return hipErrorInvalidValue;
    if (tbytes == 1)
        return conn == 8 ? tile_round_t<uint8_t, 8>(imgs, n_tiles, flags, lists, cin, cout, all, ctrl, round, max_iters, grid, s, variant)
                         : tile_round_t<uint8_t, 4>(imgs, n_tiles, flags, lists, cin, cout, all, ctrl, round, max_iters, grid, s, variant);
    return conn == 8 ? tile_round_t<int32_t, 8>(imgs, n_tiles, flags, lists, cin, cout, all, ctrl, round, max_iters, grid, s, variant)
                     : tile_round_t<int32_t, 4>(imgs, n_tiles, flags, lists, cin, cout, all, ctrl, round, max_iters, grid, s, variant);
}

hipError_t launch_tile_round_ex(int tbytes, int conn, const Imgs &imgs, int64_t n_tiles,
                                uint32_t *flags, uint32_t *lists, const uint32_t *cin,
                                uint32_t *cout, int all, Ctrl *ctrl, uint32_t round,
                                int max_iters, int grid, hipStream_t s) {
    return tile_round_any(tbytes, conn, imgs, n_tiles, flags, lists, cin, cout, all, ctrl, round,
                          max_iters, grid, s, -1);
}

hipError_t launch_tile_round(int tbytes, int conn, const Imgs &imgs, int64_t n_tiles,
                             uint32_t *flags, uint32_t *lists, Ctrl *ctrl, uint32_t round,
                             int max_iters, int grid, hipStream_t s, int op_all) {
    // every image starts in round 1 here, so with one op for all of them the
    // visit is known for the whole launch
    const int variant = op_all < 0 ? -1 : ((op_all == MR_OP_FILL ? 2 : 0) | (round == 1 ? 1 : 0));
    // Round 1 visits every tile. Later int32 rounds may walk dense bands
    // (the lists of a sequence that starts at round 1 allow it): their
    // visits are bound by memory traffic, which the walk's order lowers.
    // uint8 visits are bound by issue and latency instead; there the walk
    // only adds visits (neighbours visited together see each other's halos
    // stale more often), so uint8 rounds keep the lists.
    return tile_round_any(tbytes, conn, imgs, n_tiles, flags, lists, ctrl->round_tiles[round],
                          ctrl->round_tiles[round + 1], round == 1 ? 1 : (tbytes == 4 ? 2 : 0), ctrl, round,
                          max_iters, grid, s, variant);
}

template <typename T, int CONN, int V>
static hipError_t tile_queue_v(const Imgs &imgs, Ctrl *ctrl, uint32_t *state, uint32_t *ring,
                               uint64_t cap, int max_iters, int grid, unsigned long long wait_us,
                               hipStream_t s) {
    hipLaunchKernelGGL((k_tile_queue<T, CONN, V>), dim3((unsigned)grid), dim3(64), 0, s, imgs,
                       ctrl, state, ring, cap, max_iters, wait_us);
    return hipGetLastError();
}
template <typename T, int CONN>
static hipError_t tile_queue_t(const Imgs &imgs, Ctrl *ctrl, uint32_t *state, uint32_t *ring,
                               uint64_t cap, int max_iters, int grid, unsigned long long wait_us,
                               hipStream_t s, int op_all) {
    if (op_all == MR_OP_RECON)
        return tile_queue_v<T, CONN, 0>(imgs, ctrl, state, ring, cap, max_iters, grid, wait_us, s);
    if (op_all == MR_OP_FILL)
        return tile_queue_v<T, CONN, 2>(imgs, ctrl, state, ring, cap, max_iters, grid, wait_us, s);
    return tile_queue_v<T, CONN, -1>(imgs, ctrl, state, ring, cap, max_iters, grid, wait_us, s);
}
hipError_t launch_tile_queue(int tbytes, int conn, const Imgs &imgs, int64_t n_tiles,
                             const uint32_t *lists, uint32_t round, Ctrl *ctrl, uint32_t *state,
                             uint32_t *ring, uint64_t cap, int max_iters, int grid,
                             unsigned long long wait_us, hipStream_t s, int op_all) {
    if (!ctrl || round > (uint32_t)MAX_ROUNDS + 1 || grid < 1 || n_tiles < 1)
        return hipErrorInvalidValue;
    // no more waves than tiles: a wave visits one tile at a time
    grid = (int)std::min<int64_t>(std::min<int64_t>(grid, RING_SLACK), n_tiles);
    hipLaunchKernelGGL(k_tile_queue_seed, dim3(NBANDS), dim3(256), 0, s, lists,
                       ctrl->round_tiles[round], n_tiles, round, state, ring, cap, ctrl);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (tbytes == 1)
        return conn == 8 ? tile_queue_t<uint8_t, 8>(imgs, ctrl, state, ring, cap, max_iters, grid, wait_us, s, op_all)
                         : tile_queue_t<uint8_t, 4>(imgs, ctrl, state, ring, cap, max_iters, grid, wait_us, s, op_all);
    return conn == 8 ? tile_queue_t<int32_t, 8>(imgs, ctrl, state, ring, cap, max_iters, grid, wait_us, s, op_all)
                     : tile_queue_t<int32_t, 4>(imgs, ctrl, state, ring, cap, max_iters, grid, wait_us, s, op_all);
}

template <typename T, int CONN>
static hipError_t seed_t(const Imgs &imgs, int64_t n_tiles, const uint32_t *lists,
                         uint32_t round, Ctrl *ctrl, uint64_t *bitmap, uint32_t *qflag,
                         uint32_t *ring, uint64_t cap, int grid, hipStream_t s) {
    const int64_t want = std::max<int64_t>(NBANDS, (n_tiles + NBANDS - 1) / NBANDS * NBANDS);
    const unsigned g = (unsigned)(std::min<int64_t>(grid, want) / NBANDS * NBANDS);
    hipLaunchKernelGGL((k_seed<T, CONN>), dim3(g), dim3(64), 0, s, imgs, n_tiles, lists, round,
                       ctrl, bitmap, qflag, ring, cap);
    return hipGetLastError();
}

hipError_t launch_seed(int tbytes, int conn, const Imgs &imgs, int64_t n_tiles,
                       const uint32_t *lists, uint32_t round, Ctrl *ctrl, uint64_t *bitmap,
                       uint32_t *qflag, uint32_t *ring, uint64_t cap, int grid, hipStream_t s) {
    if (tbytes == 1)
        return conn == 8 ? seed_t<uint8_t, 8>(imgs, n_tiles, lists, round, ctrl, bitmap, qflag, ring, cap, grid, s)
                         : seed_t<uint8_t, 4>(imgs, n_tiles, lists, round, ctrl, bitmap, qflag, ring, cap, grid, s);
    return conn == 8 ? seed_t<int32_t, 8>(imgs, n_tiles, lists, round, ctrl, bitmap, qflag, ring, cap, grid, s)
                     : seed_t<int32_t, 4>(imgs, n_tiles, lists, round, ctrl, bitmap, qflag, ring, cap, grid, s);
}

__global__ void k_clear_u64(uint64_t *p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

hipError_t launch_clear_u64(uint64_t *p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_clear_u64, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

template <typename T, int CONN>
static const void *queue_fn() {
    return (const void *)&k_queue<T, CONN>;
}

static const void *queue_kernel(int tbytes, int conn) {
    if (tbytes == 1) return conn == 8 ? queue_fn<uint8_t, 8>() : queue_fn<uint8_t, 4>();
    return conn == 8 ? queue_fn<int32_t, 8>() : queue_fn<int32_t, 4>();
}

int queue_max_blocks(int tbytes, int conn) {
    int per_cu = 0, dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, queue_kernel(tbytes, conn),
                                                     64 * QWAVES, 0) != hipSuccess)
        return 0;
    return per_cu * cus;
}

template <typename T, int CONN>
static hipError_t queue_t(const Imgs &imgs, Ctrl *ctrl, uint64_t *bitmap, uint32_t *qflag,
                          uint32_t *ring, uint64_t cap, int blocks, unsigned long long wait_us,
                          hipStream_t s) {
    hipLaunchKernelGGL((k_queue<T, CONN>), dim3((unsigned)blocks), dim3(64 * QWAVES), 0, s, imgs,
                       ctrl, bitmap, qflag, ring, cap, wait_us);
    return hipGetLastError();
}

hipError_t launch_queue(int tbytes, int conn, const Imgs &imgs, Ctrl *ctrl, uint64_t *bitmap,
                        uint32_t *qflag, uint32_t *ring, uint64_t cap, int blocks,
                        unsigned long long wait_us, hipStream_t s) {
    if (blocks < 1) return hipErrorInvalidValue;
    blocks = (int)std::min<int64_t>(blocks, RING_SLACK / QWAVES);
    if (tbytes == 1)
        return conn == 8 ? queue_t<uint8_t, 8>(imgs, ctrl, bitmap, qflag, ring, cap, blocks, wait_us, s)
                         : queue_t<uint8_t, 4>(imgs, ctrl, bitmap, qflag, ring, cap, blocks, wait_us, s);
    return conn == 8 ? queue_t<int32_t, 8>(imgs, ctrl, bitmap, qflag, ring, cap, blocks, wait_us, s)
                     : queue_t<int32_t, 4>(imgs, ctrl, bitmap, qflag, ring, cap, blocks, wait_us, s);
}

hipError_t launch_widen(const Imgs &imgs, int64_t n_tiles, bool to_wide, hipStream_t s) {
    for (int64_t t0 = 0; t0 < n_tiles; t0 += (int64_t)1 << 30) {
        const unsigned g = (unsigned)std::min<int64_t>(n_tiles - t0, (int64_t)1 << 30);
        if (to_wide)
            hipLaunchKernelGGL(k_widen<true>, dim3(g), dim3(64), 0, s, imgs, t0);
        else
            hipLaunchKernelGGL(k_widen<false>, dim3(g), dim3(64), 0, s, imgs, t0);
    }
    return hipGetLastError();
}

hipError_t launch_fill_output(int tbytes, const Imgs &imgs, int64_t n_tiles, hipStream_t s,
                              int64_t t0) {
    if (n_tiles <= 0) return hipSuccess;
    if (tbytes == 1)
        hipLaunchKernelGGL(k_fill_output<uint8_t>, dim3((unsigned)n_tiles), dim3(64), 0, s, imgs, t0);
    else
        hipLaunchKernelGGL(k_fill_output<int32_t>, dim3((unsigned)n_tiles), dim3(64), 0, s, imgs, t0);
    return hipGetLastError();
}

hipError_t launch_put_desc(ImgDesc *dst, const ImgDesc &v, hipStream_t s) {
    hipLaunchKernelGGL(k_put_desc, dim3(1), dim3(1), 0, s, dst, v);
    return hipGetLastError();
}

hipError_t launch_put_descs(ImgDesc *dst, const ImgDesc *v, int n, hipStream_t s) {
    for (int i = 0; i < n; i += DESC_CHUNK) {
        DescChunk c{};
        c.n = std::min(DESC_CHUNK, n - i);
        for (int k = 0; k < c.n; ++k) c.d[k] = v[i + k];
        hipLaunchKernelGGL(k_put_descs, dim3(1), dim3(DESC_CHUNK), 0, s, dst + i, c);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_store_u64(unsigned long long *p, unsigned long long v, hipStream_t s) {
    hipLaunchKernelGGL(k_store_u64, dim3(1), dim3(1), 0, s, p, v);
    return hipGetLastError();
}

} // namespace mr
