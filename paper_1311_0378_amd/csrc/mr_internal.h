// mr_internal.h -- layouts shared by the device kernels and the host engine of
// libmrecon. Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/mr.h"

namespace mr {

// Register tile: 64 lanes x 64 rows of 32-bit keys, whose outer ring is a
// frozen halo, so each tile owns a 62 x 62 interior. Tile (ty, tx) covers
// image rows ty*62-1 .. ty*62+62 and columns tx*62-1 .. tx*62+62.
constexpr int TS = 64;
constexpr int TI = TS - 2;

// One image of a launch. A single-image call builds one; a batch builds one
// per tile of the batch. The working image J is updated in place: for
// reconstruction it is the caller's marker, for fill-holes a workspace plane.
struct ImgDesc {
    void *J;           // working image, pitch pJ elements
    const void *I;     // reconstruction: the mask; fill-holes: the input image
    void *out;         // fill-holes: where NOT J goes at the end; else null
    int64_t H, W;
    int64_t pJ, pI;    // pitches in elements (out uses pI)
    int64_t tile_base;   // first tile id of this image (its tiles are consecutive)
    int64_t first_round; // the tile round that builds its initial working image
    int32_t ntx, nty;    // tiles across and down
    int32_t op;          // MR_OP_RECON or MR_OP_FILL
    int32_t done;        // serving: 1 once the image needs no more device work
    // uint8 queue phase: the working image widened to one 32-bit key per
    // pixel (row pitch W), so that a raise is one atomic maximum instead of a
    // compare-and-swap on the dword four pixels share; null: no such plane
    uint32_t *wide;
};

// Device control block at the start of every workspace. Contended words sit
// on their own 128-byte lines.
struct alignas(128) Line {
    unsigned long long v;
    unsigned long long pad[15];
};

constexpr int NCNT = 64;      // spread counters, summed on the host
// Tile ids are split into NBANDS contiguous bands, one per XCD of the
// MI355X: band b holds tiles [b * n / NBANDS, (b + 1) * n / NBANDS). A block
// of a persistent tile kernel serves band blockIdx.x % NBANDS, which keeps
// neighbouring tiles (which share cache lines) in one XCD's L2 under the
// round-robin dispatch of workgroups to XCDs.
constexpr int NBANDS = 8;
constexpr int MAX_ROUNDS = 1000; // tile rounds per call (sweep_rounds bound)

struct Ctrl {
    Line q_head;     // frontier ring: next entry to claim
    Line q_tail;     // frontier ring: next free entry
    Line pending;    // entries pushed and not yet fully processed
    Line seeds_total;
    unsigned long long tiles[NCNT];  // tile visits (spread)
    unsigned long long pops[NCNT];   // queue-phase pops (spread)
    unsigned long long pushes[NCNT]; // queue-phase pushes (spread)
    unsigned long long cas[NCNT];    // failed CAS attempts (spread)
    unsigned long long ovf[NCNT];    // ring pushes refused by the guard (spread)
    unsigned long long iters[NCNT];  // sweep iterations over all tile visits (spread)
    unsigned long long rounds;       // written by the host sequence
    unsigned long long watchdog;     // non-zero if a wave gave up waiting or a push was refused
    // round_tiles[r][b]: length of band b's dirty list for round r (round 1:
    // the band's size, written when the block is cleared); round k + 1's lists
    // are what the seed pass starts from after k rounds.
    uint32_t round_tiles[MAX_ROUNDS + 2][NBANDS];
};

// Launch-wide view of the images: a device array of descriptors. Without an
// owner table the descriptors are sorted by tile_base and a tile's image is
// found by binary search; the server keeps owner[t] = descriptor index.
struct Imgs {
    const ImgDesc *d;
    int32_t n;
    const uint32_t *owner;
    // 1 when every image is uint8 with 16-byte aligned planes and pitches
    // (both J and I): the tile rounds may then use the pipelined kernel
    int32_t staged;
    // 1 when the images have widened planes for the queue phase
    int32_t wide;
};

constexpr uint32_t Q_EMPTY = 0xFFFFFFFFu;
// Ring slots beyond the tile count: the ring's consumers (waves of the queue
// phase or the tile queue) hold at most one ticket each past the last entry,
// and their launches are capped to this many waves.
constexpr int64_t RING_SLACK = 8192;

// The calling thread's error message (mr_last_error), shared by all host
// translation units.
void clear_error();
int set_error(int code, const char *msg);

// Host-side launchers (defined in mr_kernels.hip).
hipError_t launch_clear_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s);
hipError_t launch_clear_ctrl(Ctrl *c, int64_t n_tiles, hipStream_t s);
// Clears what a launch sequence starts from in one kernel: the control block,
// flags[n_tiles], qflag[n_tiles] (0) and ring[ring_cap] (Q_EMPTY).
hipError_t launch_clear_start(Ctrl *c, int64_t n_tiles, uint32_t *flags, uint32_t *qflag,
                              uint32_t *ring, int64_t ring_cap, hipStream_t s);
// Round r visits every tile (r == 1) or the dirty lists of round r -- band
// b's at lists[(r & 1) * n_tiles + band start], ctrl->round_tiles[r][b] long
// -- and lists each tile it dirties for round r + 1 in the other half
// (flags[t] = the latest round t is listed for). Every image's first round
// is 1; op_all is the op of all images (MR_OP_RECON / MR_OP_FILL), or -1 if
// they differ.
hipError_t launch_tile_round(int tbytes, int conn, const Imgs &imgs, int64_t n_tiles,
                             uint32_t *flags, uint32_t *lists, Ctrl *ctrl, uint32_t round,
                             int max_iters, int grid, hipStream_t s, int op_all);
// The same round with explicit list-length counters (NBANDS each) for this
// round and the next; all_tiles visits every tile instead of a list.
hipError_t launch_tile_round_ex(int tbytes, int conn, const Imgs &imgs, int64_t n_tiles,
                                uint32_t *flags, uint32_t *lists, const uint32_t *counts_in,
                                uint32_t *counts_out, int all_tiles, Ctrl *ctrl,
                                uint32_t round, int max_iters, int grid, hipStream_t s);
hipError_t launch_seed(int tbytes, int conn, const Imgs &imgs, int64_t n_tiles,
                       const uint32_t *lists, uint32_t round, Ctrl *ctrl, uint64_t *bitmap,
                       uint32_t *qflag, uint32_t *ring, uint64_t cap, int grid, hipStream_t s);
hipError_t launch_clear_u64(uint64_t *p, int64_t n, hipStream_t s);
hipError_t launch_queue(int tbytes, int conn, const Imgs &imgs, Ctrl *ctrl, uint64_t *bitmap,
                        uint32_t *qflag, uint32_t *ring, uint64_t cap, int blocks,
                        unsigned long long wait_us, hipStream_t s);
// Tile queue: seed it with every tile listed for `round` (state[t] = 1, ring
// entries, pending), then visit tiles from it on a persistent grid until none
// is queued or running. state[] and ring[] start cleared (0, Q_EMPTY).
hipError_t launch_tile_queue(int tbytes, int conn, const Imgs &imgs, int64_t n_tiles,
                             const uint32_t *lists, uint32_t round, Ctrl *ctrl, uint32_t *state,
                             uint32_t *ring, uint64_t cap, int max_iters, int grid,
                             unsigned long long wait_us, hipStream_t s, int op_all);
// The queue phase's widened planes: copy every tile interior of J into
// `wide` (to_wide), or back (from wide to J).
hipError_t launch_widen(const Imgs &imgs, int64_t n_tiles, bool to_wide, hipStream_t s);
hipError_t launch_fill_output(int tbytes, const Imgs &imgs, int64_t n_tiles, hipStream_t s,
                              int64_t t0 = 0);
hipError_t launch_store_u64(unsigned long long *p, unsigned long long v, hipStream_t s);
hipError_t launch_put_desc(ImgDesc *dst, const ImgDesc &v, hipStream_t s);
// Writes n descriptors (n <= DESC_CHUNK per launch) through kernel arguments,
// which keeps uploads stream-ordered and capturable.
constexpr int DESC_CHUNK = 16;
hipError_t launch_put_descs(ImgDesc *dst, const ImgDesc *v, int n, hipStream_t s);
int queue_max_blocks(int tbytes, int conn);
int persistent_grid();

// Server support: admit one image (descriptor, owner ids, every tile on the
// dirty list of round `round`), and mark the images that still have tiles on
// a round's lists (busy[owner] = stamp).
hipError_t launch_server_admit(ImgDesc *descs, int32_t slot, const ImgDesc &d, uint32_t *owner,
                               uint32_t *flags, uint32_t *lists_round, uint32_t *counts_round,
                               int64_t n_tiles, uint32_t round, hipStream_t s);
hipError_t launch_server_status(const uint32_t *lists_round, const uint32_t *counts_round,
                                const uint32_t *owner, uint32_t *busy, int64_t n_tiles,
                                uint32_t stamp, hipStream_t s);

} // namespace mr
