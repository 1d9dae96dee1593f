/*
 * mr.h -- C ABI of libmrecon: grayscale morphological reconstruction by
 * dilation and fill-holes on one AMD Instinct MI355X (gfx950), run as an
 * irregular wavefront propagation (IWPP).
 *
 * The operations (Table II of the paper):
 *   Morphological Reconstruction -- flood-fill of a marker image limited by a
 *     mask image, with 4- or 8-connectivity. Here: R = the least image J with
 *     J >= min(marker, mask) that is stable under
 *     J(p) <- min(mask(p), max of J over p and its G-neighbours).
 *   FillHoles -- flood-fill of the background from selected points. Here: the
 *     flood starts from every image-border pixel and runs on the bitwise
 *     complement: out = NOT R(Jb, NOT img), Jb = NOT img on the border and the
 *     type's minimum elsewhere; `conn` is the connectivity of the background
 *     flood. Images of height or width <= 2 are all border: out = img.
 * How (Algorithm 1, Sec. III-B on the GPU queue and atomics, Sec. V-C.2 on the
 * regular-then-irregular hybrid): tile rounds propagate inside 64 x 64
 * register tiles until a local fixed point; tiles whose halo changed are
 * revisited. By default, after `tail_rounds` rounds a persistent tile queue
 * revisits each tile as soon as a neighbour marks it until none is left.
 * With a positive `sweep_rounds`, after that many rounds the pixels that can
 * still raise a neighbour are compacted into a device frontier queue and
 * finished by persistent workgroups with atomic max updates.
 *
 * Conventions for every entry point:
 *  - Images are row-major, element (y, x) at index y * pitch + x; pitch is in
 *    elements, pitch >= W, and 0 means W; H * pitch must be below 2^32.
 *    Pixel types: MR_U8 (uint8) and MR_I32 (int32, full signed range).
 *    Image pointers are aligned to the pixel size. For MR_U8 the working
 *    image is updated with 32-bit compare-and-swap on the aligned words that
 *    hold its pixels, so the allocation must cover those whole words and no
 *    other agent may write bytes that share a word with the image while a
 *    call runs.
 *  - Image, mask and workspace pointers are DEVICE pointers owned by the
 *    caller. The library never allocates device memory: all scratch space is
 *    the caller's workspace, whose size the *_workspace_bytes functions give.
 *    The workspace must be 256-byte aligned.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream). Calls
 *    enqueue work and return without waiting for the device, unless stated.
 *    Faults inside kernels surface at the caller's next synchronization.
 *  - Arguments are checked on the host before anything is enqueued. Errors
 *    are negative return codes; mr_last_error() gives a message for the
 *    calling thread. Nothing is thrown across the ABI.
 *  - Marker pixels above the mask are clipped to the mask (no error).
 *  - Two calls that share a workspace must be ordered on one stream.
 */
#ifndef MR_H
#define MR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MR_ABI_VERSION 4 /* 2: mr_tune.tail_rounds; 3: mr_job.flags; 4: mr_tune.first_sweeps */

typedef enum { MR_U8 = 1, MR_I32 = 4 } mr_dtype; /* value = bytes per pixel */

enum {
    MR_OK = 0,
    MR_EINVAL = -1, /* bad argument */
    MR_ENOMEM = -2, /* workspace or arena too small */
    MR_EHIP = -3,   /* HIP runtime error, or a device-side iteration cap hit */
    MR_EAGAIN = -4  /* serving: the job cannot be admitted now; retry later */
};

enum { MR_OP_RECON = 0, MR_OP_FILL = 1 };

/* Tuning knobs. A NULL mr_tune* means "use the defaults" (mr_default_tune).
 * No knob changes the result, only the time it takes. */
typedef struct {
    int32_t sweep_rounds;      /* tile rounds before the queue phase (1..1000);
                                  a negative value (the default) runs tile
                                  rounds, then the tile queue (tail_rounds),
                                  and skips the queue phase */
    int32_t max_sweeps;        /* cap on sweep iterations per tile visit
                                  (1..1024); a capped tile is revisited */
    int32_t persistent_blocks; /* queue-phase workgroups; 0 = as many as can
                                  be co-resident on the GPU */
    int32_t converge_rounds;   /* with a negative sweep_rounds: tile rounds
                                  after which work still left goes to the seed
                                  pass and the queue phase, which finish any
                                  input (1..1000; 0 = 1000) */
    int32_t tail_rounds;       /* with a negative sweep_rounds: tile rounds
                                  after which the tiles still listed go to
                                  the tile queue, one persistent launch that
                                  revisits a tile as soon as a neighbour marks
                                  it, until none is left; the call then never
                                  waits for the device (0..1000, default 8;
                                  0 = rounds until no tile is dirty, polled
                                  by the host, and converge_rounds applies) */
    int32_t first_sweeps;      /* cap on sweep iterations per tile visit in
                                  the first tile round (1..1024, default 1).
                                  Its halos are mostly stale, and nearly every
                                  tile is visited again; a visit stopped at
                                  this cap lists its tile for the next round
                                  without checking its fixed point */
} mr_tune;

/* Work counters of the last call that used a workspace. */
typedef struct {
    uint64_t rounds;      /* tile rounds launched */
    uint64_t tiles;       /* tile visits (64 x 64 register tiles), in tile
                             rounds and in the tile queue */
    uint64_t seeds;       /* frontier entries made by the seed pass */
    uint64_t pops;        /* frontier entries processed by the queue phase */
    uint64_t pushes;      /* frontier entries produced by the queue phase */
    uint64_t cas_retries; /* failed compare-and-swap attempts (u8 updates) */
    uint64_t overflows;   /* ring pushes refused because their slot was still
                             taken after a capped wait. The ring holds more
                             slots than a launch has tiles plus waves, so this
                             stays 0; a nonzero value means the capacity bound
                             broke, the call's result is incomplete, and
                             mr_status reports MR_EHIP */
    uint64_t sweeps;      /* sweep iterations summed over all tile visits (one
                             iteration = down, up, right and left sweeps) */
} mr_counters;

/* Fills *out with the default knobs. A set environment variable
 * MR_TUNE_SWEEP_ROUNDS, MR_TUNE_MAX_SWEEPS, MR_TUNE_PERSISTENT_BLOCKS,
 * MR_TUNE_CONVERGE_ROUNDS, MR_TUNE_TAIL_ROUNDS or MR_TUNE_FIRST_SWEEPS
 * replaces that field's default when it is a whole number in the field's
 * valid range (it is ignored otherwise). Calls given a NULL mr_tune* use
 * these defaults too. */
void mr_default_tune(mr_tune *out);

/* Workspace bytes needed by one mr_recon_dilate (op = MR_OP_RECON) or
 * mr_fill_holes (op = MR_OP_FILL) call on an H x W image. Returns 0 for
 * invalid arguments (see mr_last_error).
 * For uint8 pixels and a tune with sweep_rounds > 0 (a queue phase) the size
 * includes a plane of H x W 32-bit keys at its end: the queue phase then
 * raises a pixel with one atomic maximum there instead of a compare-and-swap
 * on the dword four pixels share, and the plane is copied in before and out
 * after it. A workspace sized without that plane (by the default tune) is
 * still accepted and takes the compare-and-swap. Same for
 * mr_batch_workspace_bytes, per tile. */
size_t mr_workspace_bytes(int op, int64_t H, int64_t W, mr_dtype t, int conn,
                          const mr_tune *tune);

/* Reconstruction by dilation (Table II, Morphological Reconstruction).
 * marker_inout: device, H x W of type t with the given pitch; on return (in
 *   stream order) it holds R.
 * mask: device, same geometry and pitch, read only.
 * ws / ws_bytes: device workspace of at least mr_workspace_bytes(MR_OP_RECON,
 *   ...) bytes; its contents on entry do not matter.
 * Errors: MR_EINVAL (null pointer, H or W < 1, pitch < W, conn not 4 or 8,
 *   unknown type, misaligned workspace), MR_ENOMEM (ws_bytes too small),
 *   MR_EHIP (launch failure). */
int mr_recon_dilate(void *marker_inout, const void *mask, int64_t H, int64_t W, int64_t pitch,
                    mr_dtype t, int conn, void *ws, size_t ws_bytes, const mr_tune *tune,
                    void *stream);

/* Fill-holes (Table II, FillHoles): img_inout is replaced by its filled
 * version. Arguments and errors as for mr_recon_dilate with op MR_OP_FILL. */
int mr_fill_holes(void *img_inout, int64_t H, int64_t W, int64_t pitch, mr_dtype t, int conn,
                  void *ws, size_t ws_bytes, const mr_tune *tune, void *stream);

/* Reconstruction by dilation without any allocation, for callers that cannot
 * allocate device memory or pass a workspace: code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation. Computes exactly
 * what mr_recon_dilate computes (same kernels), with its workspace in a
 * scratch array the library holds in device memory, MR_NOALLOC_SCRATCH_BYTES
 * per GPU, from the library's load on that GPU until the process ends. The
 * call itself allocates nothing (no device, host or pinned memory, no
 * events).
 * Limits: the image's workspace (mr_workspace_bytes(MR_OP_RECON, ...)) must
 * fit the scratch: at most MR_NOALLOC_SCRATCH_BYTES, which holds images up to
 * 16384 x 16384 and somewhat beyond; larger ones return MR_ENOMEM. The tune
 * must not select the converge mode (sweep_rounds > 0, or a negative
 * sweep_rounds with tail_rounds > 0; the default tune qualifies): else
 * MR_EINVAL.
 * Concurrency: every call on one GPU shares that GPU's scratch, and each call
 * rebuilds what it needs there, so calls on one GPU must be ordered (one
 * stream, or events between streams): calls that overlap race on the scratch
 * and give undefined results. Calls on different GPUs are independent.
 * mr_status, mr_read_counters and mr_read_round_tiles read a caller's
 * workspace, so they do not report on these calls.
 * Other arguments and errors as for mr_recon_dilate; MR_EHIP also when the
 * scratch array's device address cannot be looked up. */
#define MR_NOALLOC_SCRATCH_BYTES (64u << 20)
int mr_recon_dilate_noalloc(void *marker_inout, const void *mask, int64_t H, int64_t W,
                            int64_t pitch, mr_dtype t, int conn, const mr_tune *tune,
                            void *stream);

/* Reconstruction by erosion, the dual of Table II's reconstruction (after
 * Vincent 1993): E = the greatest image J <= max(marker, mask) that is stable
 * under J(p) <- max(mask(p), min of J over p and its G-neighbours). Marker
 * pixels below the mask are raised to it (no error). Computed as
 * NOT R(NOT marker, NOT mask) with the bitwise complement: NOT mask goes into
 * the workspace, the marker is complemented in place, reconstructed by
 * dilation and complemented back.
 * Arguments as for mr_recon_dilate; ws_bytes must be at least
 * mr_recon_erode_workspace_bytes(H, W, pitch, ...), which also covers a
 * plane of H x pitch pixels. mask is read only.
 * Errors: as mr_recon_dilate, checked before anything is enqueued. After
 * MR_EHIP the marker's contents are unspecified. */
size_t mr_recon_erode_workspace_bytes(int64_t H, int64_t W, int64_t pitch, mr_dtype t, int conn,
                                      const mr_tune *tune);
int mr_recon_erode(void *marker_inout, const void *mask, int64_t H, int64_t W, int64_t pitch,
                   mr_dtype t, int conn, void *ws, size_t ws_bytes, const mr_tune *tune,
                   void *stream);

/* ------------------------------------------------------------- batches */

/* One image of a batch (the tiles of a whole-slide image are independent
 * images here: no propagation crosses from one to another). */
typedef struct {
    void *data_inout;  /* device: the marker (MR_OP_RECON) or the image
                          (MR_OP_FILL); replaced by the result */
    const void *mask;  /* device: the mask (MR_OP_RECON, same pitch as the
                          data); NULL for MR_OP_FILL */
    int64_t H, W;
    int64_t pitch;     /* elements, >= W; 0 = W */
    int32_t op;        /* MR_OP_RECON or MR_OP_FILL */
    int32_t reserved;  /* must be 0 */
} mr_tile;

/* Workspace bytes for mr_batch over tiles[0..n). 0 on invalid arguments. */
size_t mr_batch_workspace_bytes(const mr_tile *tiles, int32_t n, mr_dtype t, int conn,
                                const mr_tune *tune);

/* Runs every image of the batch through one launch sequence: the tile
 * rounds, seed pass and queue phase each cover all images at once, so small
 * and large images share the GPU. Pixel type and connectivity are common to
 * the batch; op may differ per image. `tiles` is host memory, read before the
 * call returns. Errors as for mr_recon_dilate, checked for every image. */
int mr_batch(const mr_tile *tiles, int32_t n, mr_dtype t, int conn, void *ws, size_t ws_bytes,
             const mr_tune *tune, void *stream);

/* A batch captured once into a HIP graph, for repeated launches over the same
 * buffers (new data copied into them between launches). Needs a tune whose
 * call never waits for the device: tune->sweep_rounds > 0 (a fixed number of
 * tile rounds, then the queue phase), or a negative sweep_rounds with
 * tail_rounds > 0 (rounds, then the tile queue). */
typedef struct mr_graph mr_graph;
int mr_batch_graph_create(const mr_tile *tiles, int32_t n, mr_dtype t, int conn, void *ws,
                          size_t ws_bytes, const mr_tune *tune, mr_graph **out);
int mr_graph_launch(mr_graph *g, void *stream);
void mr_graph_destroy(mr_graph *g);

/* Autotuner: times candidate tunings (sweep rounds before the queue phase or
 * the tile queue, sweep cap per tile visit) of mr_batch on this batch and
 * writes the fastest to *out. The tiles' data are restored afterwards. ws must hold
 * mr_autotune_workspace_bytes bytes (the batch workspace plus a backup of
 * the data). Waits for `stream`. */
size_t mr_autotune_workspace_bytes(const mr_tile *tiles, int32_t n, mr_dtype t, int conn);
int mr_autotune(const mr_tile *tiles, int32_t n, mr_dtype t, int conn, void *ws, size_t ws_bytes,
                void *stream, mr_tune *out);

/* --------------------------------------------------------------- serving */

/* A request: one image, answered in a buffer of the same kind. Rows of the
 * inputs are `ld` elements apart and rows of the result `ld_result` apart
 * (0 means W), so a job can be a window of a larger image. The buffers must
 * stay valid until the job is reported done.
 * Host jobs (flags 0): data, mask and result are host memory; pinned
 * (page-locked) memory lets the copies run asynchronously, pageable memory
 * works but copies synchronously.
 * Device jobs (flags MR_JOB_DEVICE): data, mask and result are device
 * memory of the server's GPU, for callers whose tiles are already in HBM
 * (an upstream kernel produced them): the copies into and out of the arena
 * are device-to-device, and no PCIe transfer is involved. */
enum { MR_JOB_DEVICE = 1 };
typedef struct {
    const void *data; /* H x W: the marker (MR_OP_RECON) or the image (MR_OP_FILL) */
    const void *mask; /* H x W mask (MR_OP_RECON); NULL otherwise */
    void *result;     /* H x W: receives the result; may alias data */
    int64_t H, W;
    int64_t ld;        /* input row pitch in elements, >= W, or 0 */
    int64_t ld_result; /* result row pitch in elements, >= W, or 0 */
    int32_t op;        /* MR_OP_RECON or MR_OP_FILL */
    int32_t flags;     /* 0 (host buffers) or MR_JOB_DEVICE */
} mr_job;

/* Continuous-batching server over a caller-provided device arena, the HBM
 * budget (256-byte aligned, at least a few MiB). The arena's head holds the
 * server's descriptors, per-tile arrays and counters; the rest is handed out
 * to jobs, two planes each. A job is admitted when a slot, arena space and
 * tile ids are free. Each step launches one tile round over every resident
 * job on `stream`; a job admitted between steps joins the next round,
 * overlapping the jobs already on the device. Dirty-tile lists (the
 * frontiers) stay in the arena between steps. A job is finished when a round
 * leaves none of its tiles dirty; its result is then copied back.
 *
 * Pipelining: input copies and result copies run on two streams that the
 * server creates, so they overlap the rounds and each other (PCIe is full
 * duplex); a step launches round r and then retires what round r-1 finished,
 * so the device always has the next round queued. A finished job's arena
 * space, tile ids and slot are reused only after its result copy has
 * completed. All calls for one server must come from one thread.
 *
 * Errors: MR_EINVAL (bad argument), MR_ENOMEM (arena too small), MR_EHIP. */
typedef struct mr_server mr_server;
int mr_server_create(void *arena, size_t arena_bytes, int32_t max_jobs, mr_dtype t, int conn,
                     void *stream, mr_server **out);
/* Admits a job: starts its input copies and returns its id.
 * MR_EAGAIN: no slot, arena space or tile ids free now -- retry after steps.
 * MR_EINVAL: the job is malformed or could never fit this arena. */
int mr_server_submit(mr_server *s, const mr_job *job, uint64_t *id);
/* Launches the next tile rounds (if any job is still working) and retires
 * the jobs the previous step finished: their result copies are started.
 * Blocks until the previous step's rounds have completed. */
int mr_server_step(mr_server *s);
/* Tile rounds each step launches before its one status read-back (1..64,
 * default 8): more rounds per step mean fewer host round trips, at the cost
 * of noticing a finished job up to that many rounds later. Takes effect at
 * the next step. Errors: MR_EINVAL. */
int mr_server_set_rounds_per_step(mr_server *s, int32_t k);
/* Ids of jobs whose results have fully arrived in their host buffers since
 * the last poll (up to cap), in the order they finished. Does not block. */
int mr_server_poll(mr_server *s, uint64_t *done_ids, int32_t cap, int32_t *n_done);
/* Steps until every job is finished and every result copy has completed;
 * their ids stay available to mr_server_poll. */
int mr_server_drain(mr_server *s);
/* Jobs on the device (admitted and not yet fully returned), tile rounds
 * launched, largest free arena block. */
int mr_server_stats(const mr_server *s, int32_t *resident, uint64_t *rounds,
                    size_t *free_bytes);
/* Waits for the server's work, then frees its host-side state and streams
 * (the arena stays the caller's). */
void mr_server_destroy(mr_server *s);

/* Copies the work counters held in a workspace to *out. Waits for `stream`.
 * Errors: MR_EINVAL (null pointer), MR_EHIP (a copy failed, or a wave of the
 * queue phase or the tile queue saw no new ring entry for 2 s and gave up:
 * the result of that call is then incomplete; *out is still written). */
int mr_read_counters(const void *ws, mr_counters *out, void *stream);

/* Status of the last call that used a workspace (mr_recon_dilate,
 * mr_fill_holes, mr_recon_erode, mr_batch or a graph launch over it). Waits
 * for `stream`, then returns MR_OK if that call ran to its fixed point, or
 * MR_EHIP if a wave of its queue phase or tile queue gave up (no new ring
 * entry for 2 s) or a ring push was refused: the result is then incomplete.
 * The status is kept until the next call on the same workspace clears it, so
 * check it before reusing the workspace. Costs one 8-byte copy.
 * Errors: MR_EINVAL (null ws), MR_EHIP (as above, or a failed copy). */
int mr_status(const void *ws, void *stream);

/* Tile visits per round of the last call that used a workspace: out[i] is
 * the number of 64 x 64 tiles visited in round i + 1, and out[rounds] the
 * number of tiles handed on to the seed pass or the tile queue (0 when the
 * rounds converged).
 * Writes min(cap, rounds + 1) entries, sets *n_rounds. Waits for `stream`.
 * Errors: MR_EINVAL (null pointer, negative cap), MR_EHIP. */
int mr_read_round_tiles(const void *ws, uint32_t *out, int32_t cap, int32_t *n_rounds,
                        void *stream);

/* Per-launch device timing (measurement support). While enabled, every
 * tile-round, seed, queue and tile-queue kernel that a call on this thread
 * enqueues is bracketed by two HIP events recorded on the call's stream; the
 * records accumulate until collected. The events carry no system-scope fence
 * (no cache writeback between launches); each still adds a marker to the
 * stream, a few microseconds of device time per event on MI355X.
 * MR_TIMING_SPANS brackets instead each run of consecutive tile rounds that
 * no host wait interrupts, with one pair of events: the record covers
 * `launches` rounds and the dispatch gaps between them. */
enum { MR_K_TILE_ROUND = 0, MR_K_SEED = 1, MR_K_QUEUE = 2, MR_K_TILE_QUEUE = 3 };
enum { MR_TIMING_OFF = 0, MR_TIMING_LAUNCHES = 1, MR_TIMING_SPANS = 2 };
typedef struct {
    int32_t kind;     /* MR_K_* */
    int32_t round;    /* first tile round covered (MR_K_TILE_ROUND), else 0 */
    int32_t launches; /* launches covered: 1, or the rounds of a span */
    float ms;         /* device time between the two events */
} mr_launch_time;

/* Sets the calling thread's timing mode: MR_TIMING_OFF, MR_TIMING_LAUNCHES
 * (every launch bracketed) or MR_TIMING_SPANS. Any other nonzero value means
 * MR_TIMING_LAUNCHES. Returns MR_OK. */
int mr_timing_enable(int on);

/* Waits for the recorded events, writes up to `cap` records in launch order
 * to `out`, sets *n to the number of records held, and clears them.
 * Errors: MR_EINVAL (null n, or out null with cap > 0), MR_EHIP. */
int mr_timing_collect(mr_launch_time *out, int32_t cap, int32_t *n);

/* Device atomic-rate probe (measurement support; cf. the atomic-throughput
 * measurements of Table IV). Enqueues on `stream` one launch of `waves`
 * 64-lane waves; each lane performs `per_lane` relaxed device-scope atomics
 * on words of `words` (device memory, n_words uint32 values, caller-owned)
 * chosen by a fixed hash of (seed, lane, step):
 *   MR_PROBE_ADD  fetch-add of 1, result unused;
 *   MR_PROBE_CAS  load, then compare-and-swap to the value read + 1, retried
 *                 with the returned value until it lands (the queue phase's
 *                 raise pattern).
 * Either way the sum of the words grows by exactly waves * 64 * per_lane
 * (mod 2^32 per word). Time it with events on the same stream.
 * Errors: MR_EINVAL (words null or not 4-byte aligned; n_words not a power
 * of two in [64, 2^32]; kind unknown; per_lane outside [1, 65536]; waves
 * outside [1, 2^20]), MR_EHIP (launch failure). Nothing is enqueued on
 * error. */
enum { MR_PROBE_ADD = 0, MR_PROBE_CAS = 1 };
int mr_probe_atomics(void *words, size_t n_words, int kind, int32_t per_lane, int32_t waves,
                     uint32_t seed, void *stream);

/* Random-access probe (measurement support; the paper's micro-benchmark for
 * irregular access, Sec. V-A, whose figures Table III gives in MB/s). Enqueues
 * on `stream` one launch of `waves` 64-lane waves that performs n_ops plain
 * (non-atomic) accesses to 32-bit words of `words` (device memory, n_words
 * values, caller-owned), operation i at position indices[i] mod n_words, where
 * `indices` (device memory, n_ops uint32 values, caller-owned, read only) is
 * filled by the caller, as the paper fills its index vector on the host.
 * Lane g of the grid (g < waves * 64) performs the operations g, g + S,
 * g + 2S, ... with S = waves * 64.
 *   MR_RANDOM_READ   lane g writes the 32-bit wrapping sum of the words it
 *                    read to sums[g] (device memory, waves * 64 uint32 values,
 *                    caller-owned); `words` is not written.
 *   MR_RANDOM_WRITE  operation i stores the low 32 bits of i at its position;
 *                    where several operations share a position, which of them
 *                    lands is unspecified. `sums` is ignored.
 * The index vector is read once, in order; the accesses to `words` scatter.
 * Time it with events on the same stream.
 * Errors: MR_EINVAL (words null or not 4-byte aligned; n_words not a power of
 * two in [64, 2^32]; kind unknown; indices null or not 4-byte aligned; n_ops
 * outside [1, 2^34]; waves outside [1, 2^20]; a read with sums null or not
 * 4-byte aligned), MR_EHIP (launch failure). Nothing is enqueued on error. */
enum { MR_RANDOM_READ = 0, MR_RANDOM_WRITE = 1 };
int mr_probe_random(void *words, size_t n_words, const void *indices, size_t n_ops, int kind,
                    int32_t waves, void *sums, void *stream);

/* Message for the last error returned to the calling thread ("" if none). */
const char *mr_last_error(void);

/* ABI version of the loaded library (MR_ABI_VERSION it was built with). */
int mr_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MR_H */
