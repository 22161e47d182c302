/*
 * vsaogm.h -- C ABI of the MI355X (gfx950) VSA-OGM hot path.
 *
 * VSA-OGM (arXiv 2408.09066) builds an occupancy grid map from labelled 2-D
 * points with Spatial Semantic Pointers.  The operations exposed here are:
 *
 *   vsaogm_encode    Sec. III-B "Encoding Point Clouds": every point is
 *                    fractionally bound (2-D encoding equation) and bundled
 *                    (eq. bundling) into the memory of its nearest tile and
 *                    its class (Algorithm 1).
 *   vsaogm_decode    Sec. III-B "Decoding": memory normalisation (eq.
 *                    vector-normalization) and similarity against the
 *                    location vectors of every grid cell (eq. loc-query),
 *                    plus the per-class maximum used by eq. non-linearities.
 *   vsaogm_classify  Sec. III-B: (P/max P)^2 (eq. non-linearities), local
 *                    Shannon entropy over a disk mask (Algorithm 2 and the
 *                    entropy / mask equations), softmax (eq. softmax),
 *                    probabilistic signed difference (eq. psd) and the
 *                    threshold rho (eq. classification).
 *   vsaogm_fuse      Sec. III-B "Multi-Map Fusion" (Algorithm 3).
 *   vsaogm_fuse_many the same for N agents in one pass.
 *   vsaogm_submit /  a request loop that runs whole map updates
 *   vsaogm_poll      (encode + decode + classify) for many maps at once.
 *
 * Representation.  A real D-dimensional SSP is kept as its discrete Fourier
 * spectrum.  The axis vectors have unit-modulus, conjugate-symmetric spectra
 * exp(i*theta_k); the caller passes Theta[k] = theta_k / l (radians per
 * metre, length scale l already applied) for both axes.  Fractional binding
 * of (x, y) is then the spectrum exp(i*(Theta[k][0]*x + Theta[k][1]*y)).
 * Because the spectra are conjugate-symmetric only bins 0..D/2 are stored.
 *
 * Tiles (Sec. III-B "Vector Discretization") split the layout rectangle
 * [x0,x1] x [y0,y1] into tiles_x * tiles_y equal tiles, numbered row-major
 * beta = ty*tiles_x + tx.  Memory 2*beta+psi holds class psi of tile beta
 * (psi = 1 occupied, 0 empty).  A point or a grid cell belongs to the tile
 * whose centre is nearest (double-precision squared distance, lowest index on
 * an exact tie); points outside the rectangle go to the nearest tile.
 *
 * Conventions for every function:
 *   - the return value is a vsaogm_status; no C++ exception crosses the ABI;
 *   - "dev" pointers are HIP device pointers on the map's device, "host"
 *     pointers are ordinary host memory; the caller owns every pointer it
 *     passes, the library owns maps, servers and their internal buffers;
 *   - calls that take a stream only enqueue work on it (they return before the
 *     GPU finishes); the caller must keep inputs alive and outputs untouched
 *     until the stream reaches that point;
 *   - a map is not thread-safe; a server is safe for concurrent submit/poll.
 *
 * Graph capture.  Work buffers and a grid's tables are made on the first call
 * that needs them (vsaogm_encode with more points than before, the first
 * vsaogm_decode of a grid and precision); those calls may allocate and
 * synchronise.  Once a map has run an update of a given point count, grid and
 * precision, vsaogm_map_reset, vsaogm_encode, vsaogm_decode and
 * vsaogm_classify for the same sizes launch kernels only (no allocation, no
 * synchronisation, no memset), so a caller can capture such an update in a HIP
 * graph on its stream and replay it for later scans of that size, copying the
 * new points into the captured input buffers first.
 */
#ifndef VSAOGM_H
#define VSAOGM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    VSAOGM_OK = 0,
    VSAOGM_EINVAL = -1,   /* invalid argument (message in vsaogm_last_error) */
    VSAOGM_ENOMEM = -2,   /* device allocation failed */
    VSAOGM_EDEVICE = -3,  /* a HIP call failed */
    VSAOGM_EAGAIN = -4,   /* vsaogm_poll: request not finished yet */
    VSAOGM_EBUSY = -5,    /* vsaogm_submit: admission refused (queue or memory budget full) */
    VSAOGM_ENOTFOUND = -6 /* unknown ticket or map id */
} vsaogm_status;

/* Arithmetic of the similarity contraction (Sec. III-B eq. loc-query). */
typedef enum {
    VSAOGM_FP32 = 0,    /* fp32 operands, fp32 accumulation (MFMA f32) */
    VSAOGM_BF16 = 1,    /* bf16 operands, fp32 accumulation */
    VSAOGM_FP16 = 2,    /* fp16 operands, fp32 accumulation */
    VSAOGM_BF16X3 = 3   /* bf16 hi+lo split of both operands, 3 products, fp32 accumulation */
} vsaogm_precision;

typedef struct vsaogm_map vsaogm_map;
typedef struct vsaogm_server vsaogm_server;
typedef struct vsaogm_volume vsaogm_volume;
typedef void* vsaogm_stream; /* a hipStream_t; NULL means the device's null stream */

typedef struct {
    int32_t dim;            /* D: even, >= 4 (the paper's vector dimensionality d) */
    const double* theta;    /* host [D][2] Theta in rad/m; Theta[0] = Theta[D/2] = 0 and
                               Theta[D-k] = -Theta[k] exactly, else EINVAL; copied */
    double x0, y0, x1, y1;  /* tile layout rectangle (metres), x1 > x0, y1 > y0 */
    int32_t tiles_x, tiles_y; /* delta per axis, 1..64 each */
    int32_t device;         /* HIP device ordinal */
} vsaogm_map_desc;

/* Query grid: cell (i, j), 0 <= i < nx, 0 <= j < ny, has centre
   (x0 + (i + 0.5) * res, y0 + (j + 0.5) * res).  Maps are [ny][nx] row-major. */
typedef struct {
    double x0, y0, res;
    int32_t nx, ny;
} vsaogm_grid_desc;

/* Library version (major*10000 + minor*100 + patch). */
int32_t vsaogm_version(void);

/* Text of the last error raised on the calling thread ("" if none). */
const char* vsaogm_last_error(void);

/* Create a map with all memories zero.  *out receives the handle. */
int vsaogm_map_create(const vsaogm_map_desc* desc, vsaogm_map** out);

/* Destroy a map (synchronises its device first).  NULL is a no-op. */
int vsaogm_map_destroy(vsaogm_map* map);

/* Number of memories (2 * tiles_x * tiles_y) and the dimension D. */
int vsaogm_map_info(const vsaogm_map* map, int64_t* n_memories, int32_t* dim);

/* Set every memory back to zero (async on stream). */
int vsaogm_map_reset(vsaogm_map* map, vsaogm_stream stream);

/*
 * Algorithm 1: bundle n labelled points into the map's memories.
 *   xy    dev float32 [n][2], world metres
 *   label dev uint8 [n], 1 = occupied, 0 = empty; any other value names no
 *         memory of Algorithm 1 (classes are 0 and 1 only): such a point is not
 *         bundled and is counted, and vsaogm_map_take_rejected reports the count
 *         (the check runs on the device, so the call stays asynchronous)
 * Memories accumulate across calls.  n == 0 is a no-op.  Returns EINVAL for
 * n < 0 or NULL pointers with n > 0.  Work buffers grow on demand (a growth
 * synchronises the stream once).
 */
int vsaogm_encode(vsaogm_map* map, const float* xy, const uint8_t* label, int64_t n,
                  vsaogm_stream stream);

/*
 * Synchronise the stream and return (and clear) the number of points that
 * encode calls rejected for a label outside {0, 1} since the last call.
 */
int vsaogm_map_take_rejected(vsaogm_map* map, vsaogm_stream stream, int64_t* n_rejected);

/*
 * Eqs. vector-normalization and loc-query over a grid:
 *   heat dev float32 [2][ny][nx]; heat[psi][j][i] = normalised memory
 *        2*beta(c)+psi dotted with the location vector of cell c, 0 where
 *        that memory is empty;
 *   hmax dev float32 [2]; hmax[psi] = max over the grid of heat[psi]
 *        (the maximum of eq. non-linearities).
 * precision selects the contraction arithmetic (vsaogm_precision).  The
 * per-grid location tables are built on first use and cached in the map
 * (a new grid synchronises the stream once).  Returns EINVAL for nx, ny < 1,
 * res <= 0, or a grid whose cells cannot be split into per-tile row and
 * column ranges.
 */
int vsaogm_decode(vsaogm_map* map, const vsaogm_grid_desc* grid, int32_t precision,
                  float* heat, float* hmax, vsaogm_stream stream);

/*
 * Localized decoding (Sec. III-A: each tile's cells read only that tile's memories): like
 * vsaogm_decode, but only the cells of tiles whose memories changed since the last
 * incremental decode of this grid, into this same heat buffer at this same precision, are
 * recomputed; the other cells keep their values (heat must be that buffer, unchanged
 * since).  The first call for a grid, or a call with another heat buffer or precision,
 * decodes every cell.  hmax is the maximum over all cells (the map keeps per-tile maxima).
 * A recomputed cell equals vsaogm_decode's value up to the order of the fp32 accumulation
 * (the reduction over frequencies is split among workgroups by the number of tiles decoded).
 * Asynchronous: which memories changed, the tiles to recompute and the split of their work
 * are found by a kernel on the stream (memory versions on the device), so the host never
 * waits; only the first call for a grid synchronises once, as vsaogm_decode does.  Errors as
 * vsaogm_decode.
 */
int vsaogm_decode_incremental(vsaogm_map* map, const vsaogm_grid_desc* grid, int32_t precision,
                              float* heat, float* hmax, vsaogm_stream stream);

/*
 * Post-processing of Sec. III-B on the device:
 *   Q = (heat / hmax)^2 per class (Q = 0 for a class whose hmax <= 0),
 *   H_psi(c) = sum of -Q ln Q over grid cells within Euclidean distance r_psi
 *   (integer cell offsets, inclusive; cells outside the grid are not summed),
 *   ogm = softmax(H)_1 - softmax(H)_0 = tanh((H_1 - H_0) / 2),
 *   label = 1 (occupied) where ogm >= rho, else 0.
 *   heat dev float32 [2][ny][nx] (index 1 = occupied), hmax dev float32 [2],
 *   ogm  dev float32 [ny][nx] or NULL, label dev uint8 [ny][nx].
 * r_occ is the disk radius of class 1, r_emp of class 0; 0 <= r <= 24.
 * Only grid->nx and grid->ny are used.  device selects the HIP device.
 */
int vsaogm_classify(const vsaogm_grid_desc* grid, const float* heat, const float* hmax,
                    int32_t r_occ, int32_t r_emp, float rho, float* ogm, uint8_t* label,
                    int32_t device, vsaogm_stream stream);

/* Activation of the decoding ablation (Sec. IV-B, decoding methodology). */
typedef enum {
    VSAOGM_ACT_ENTROPY = 0,  /* local Shannon entropy over the disks (the decoding of Sec. III-B) */
    VSAOGM_ACT_RELU = 1,     /* max(q, 0) per cell */
    VSAOGM_ACT_TANH = 2,     /* tanh(q) per cell */
    VSAOGM_ACT_SIGMOID = 3   /* 1 / (1 + exp(-q)) per cell */
} vsaogm_activation;

/*
 * vsaogm_classify with the toggles of the decoding ablation of Sec. IV-B: the value fed to
 * the softmax is act(nl(n(P))) with n(P) = P / max P if normalize (0 for a class whose
 * maximum is <= 0), nl(q) = q^2 if square, and act from vsaogm_activation (the entropy term
 * -q ln q is 0 for q <= 0; per-cell activations ignore the radii).  vsaogm_classify is this
 * call with normalize = square = 1 and VSAOGM_ACT_ENTROPY.
 */
int vsaogm_classify_ex(const vsaogm_grid_desc* grid, const float* heat, const float* hmax,
                       int32_t r_occ, int32_t r_emp, float rho, int32_t normalize, int32_t square,
                       int32_t activation, float* ogm, uint8_t* label, int32_t device,
                       vsaogm_stream stream);

/*
 * The bundled memories of eq. bundling as Algorithm 1 leaves them (memory 2*beta+psi holds
 * the sum of the class-psi points of tile beta, 2-D encoding equation), read back in the
 * paper's frame: out dev float32
 * [2R][D/2+1][2] (re, im), out[key][k] = sum over the key's points of
 * exp(i*(Theta[k][0]*x + Theta[k][1]*y)), k = 0..D/2 (the other bins are the
 * complex conjugates, bin D-k = conj(bin k)).
 */
int vsaogm_memories(const vsaogm_map* map, float* out, vsaogm_stream stream);

/*
 * Algorithm 3 for two maps: dst's memories += src's memories, key by key.
 * Both maps must have the same Theta (bitwise), D, layout rectangle, tiling
 * and device (EINVAL otherwise).  Async on stream; src must not be encoded
 * into concurrently.
 */
int vsaogm_fuse(vsaogm_map* dst, const vsaogm_map* src, vsaogm_stream stream);

/*
 * Algorithm 3 for N agents: dst's memories += srcs[0]'s + ... + srcs[n-1]'s, key by key,
 * added in source order in one pass over dst (one launch per 16 sources), so the result is
 * bit-identical to n vsaogm_fuse calls in that order.  srcs: host array of n map handles
 * (n >= 0; n = 0 leaves dst unchanged); every source must satisfy vsaogm_fuse's conditions
 * against dst (EINVAL otherwise, nothing launched); a source may appear more than once, dst
 * not at all.  Async on stream; the sources must not be encoded into concurrently.
 */
int vsaogm_fuse_many(vsaogm_map* dst, const vsaogm_map* const* srcs, int32_t n, vsaogm_stream stream);

/* ---------------------------------------------------------------------------
 * Serving: a request loop for map updates of many maps.
 *
 * A server owns a set of maps (their memories stay resident on the device)
 * and runs whole map updates -- encode the request's points into its map,
 * decode the request's grid, classify it -- for requests that arrive while
 * others are on the GPU.  Requests are admitted as execution slots (one HIP
 * stream each) and device memory budget free up; the updates of different
 * maps overlap on the device, while updates of one map run in submission
 * order (memories are state).  A request's result does not depend on which
 * other requests share the device with it.
 *
 * Memory budget: a request is admitted only if the bytes of the requests in
 * flight (each charged its buffers plus a bound on what its run can add to its
 * map: a new grid's tables, workspace growth), of every map as it stands and of
 * the slots' buffers stay within hbm_budget_bytes.  When nothing runs and the
 * first waiting request still does not fit, the server releases what the maps
 * rebuild on demand (cached grids, workspaces; never memories) and tries again;
 * a request that does not fit even then completes with VSAOGM_ENOMEM.  The
 * accounting is the library's own: the device allocator may round blocks up.
 * ------------------------------------------------------------------------- */

typedef struct {
    int64_t hbm_budget_bytes; /* device bytes the server may hold: its maps (memories,
                                 workspaces, cached grid tables), its slots' buffers and
                                 the requests in flight; <= 0 means a quarter of the free
                                 memory */
    int32_t max_inflight;     /* execution slots (streams), 1..32 */
    int32_t max_queue;        /* pending requests before submit returns EBUSY */
    int32_t device;           /* HIP device ordinal */
    int32_t max_batch;        /* requests of distinct maps run as one batch (one launch per
                                 stage), 1..64; <= 0 means 2 */
} vsaogm_server_desc;

typedef struct {
    int32_t map_id;           /* from vsaogm_server_add_map */
    const float* xy;          /* host [n][2] world metres (copied by submit) */
    const uint8_t* label;     /* host [n] point classes (copied by submit) */
    int64_t n;                /* points, >= 0 */
    vsaogm_grid_desc grid;    /* grid to decode after the update */
    int32_t precision;        /* vsaogm_precision of the similarity contraction */
    int32_t r_occ, r_emp;     /* disk radii (classify) */
    float rho;                /* decision threshold */
    float* ogm;               /* host [ny][nx] signed difference, or NULL */
    uint8_t* label_out;       /* host [ny][nx] occupancy labels, or NULL */
    float* heat;              /* host [2][ny][nx] similarity maps, or NULL */
    int32_t flags;            /* 0, or VSAOGM_REQUEST_LOCAL */
} vsaogm_request;

/* Request flag: decode with vsaogm_decode_incremental into a heat buffer the server keeps
   for the map (one grid per map; a request with another grid or precision decodes in full
   and replaces it).  That buffer (8 bytes per cell) is map state, outside the budget. */
enum { VSAOGM_REQUEST_LOCAL = 1 };

typedef struct {
    int32_t status;           /* VSAOGM_OK, or the error the update hit */
    int32_t slot;             /* execution slot that ran it */
    int64_t t_submit_ns;      /* steady-clock time stamps (ns) */
    int64_t t_start_ns;       /* admitted and launched */
    int64_t t_done_ns;        /* outputs written to the caller's buffers */
    float hmax[2];            /* per-class maxima of the decoded grid */
} vsaogm_result;

/* Create a server on a device.  *out receives the handle. */
int vsaogm_server_create(const vsaogm_server_desc* desc, vsaogm_server** out);

/* Finish every admitted request, then destroy the server and its maps. */
int vsaogm_server_destroy(vsaogm_server* server);

/* Create a map owned by the server (desc->device is ignored: the server's
   device is used).  *map_id receives its id (0, 1, ...).  ENOMEM when the new
   map's own buffers do not fit the memory budget beside what the server holds. */
int vsaogm_server_add_map(vsaogm_server* server, const vsaogm_map_desc* desc, int32_t* map_id);

/* The server-owned map (for vsaogm_memories, vsaogm_decode or vsaogm_fuse after vsaogm_server_drain).
   Not to be encoded into or destroyed by the caller. */
int vsaogm_server_get_map(vsaogm_server* server, int32_t map_id, vsaogm_map** out);

/*
 * Queue one map update.  Inputs are copied before returning; output buffers
 * must stay valid until the ticket completes.  Returns EBUSY when max_queue
 * requests are pending (nothing is queued), ENOTFOUND for an unknown map,
 * EINVAL for invalid arguments (also when the request alone exceeds the
 * memory budget).  Thread-safe.
 */
int vsaogm_submit(vsaogm_server* server, const vsaogm_request* req, uint64_t* ticket);

/*
 * Queue count requests in order, as count calls of vsaogm_submit would, with one lock
 * acquisition.  Stops at the first request that fails; *n_queued receives how many were
 * queued (tickets[0..*n_queued) are valid) and the return value is that request's status
 * (VSAOGM_OK when all were queued).
 */
int vsaogm_submit_many(vsaogm_server* server, const vsaogm_request* reqs, int32_t count,
                       uint64_t* tickets, int32_t* n_queued);

/*
 * Non-blocking: VSAOGM_EAGAIN while the ticket runs; otherwise fills *result,
 * retires the ticket and returns VSAOGM_OK (the update's own status is in
 * result->status).  ENOTFOUND for an unknown or already retired ticket.
 */
int vsaogm_poll(vsaogm_server* server, uint64_t ticket, vsaogm_result* result);

/* Blocking variant of vsaogm_poll. */
int vsaogm_wait(vsaogm_server* server, uint64_t ticket, vsaogm_result* result);

/* Block until every submitted request has completed. */
int vsaogm_server_drain(vsaogm_server* server);

/* Counters: requests completed, peak bytes of the budget in use (maps, slots and
   requests in flight), budget. */
int vsaogm_server_stats(vsaogm_server* server, int64_t* completed, int64_t* peak_bytes,
                        int64_t* budget_bytes);

/* The budget's bytes now: charged to requests in flight, resident in the maps (as last
   reported), held by the slots' buffers; and how many times the server released the maps'
   rebuildable buffers to admit a request.  Any pointer may be NULL. */
int vsaogm_server_memory(vsaogm_server* server, int64_t* in_flight, int64_t* resident, int64_t* fixed,
                         int64_t* reclaims);

/* Device bytes a request holds from admission to completion for its own buffers (admission
   adds a bound on what its run can add to its map, and checks the sum against the budget
   beside the maps' and slots' bytes).  ENOTFOUND for an unknown map. */
int vsaogm_request_bytes(vsaogm_server* server, const vsaogm_request* req, int64_t* bytes);

/*
 * Profiling hook: the given HIP events (hipEvent_t) take the start and end times of
 * every launch of one stage's main kernel(s), recorded by the kernel dispatches
 * themselves (no marker packets are queued between kernels):
 *   stage 0  encode: the sin/cos-and-accumulate kernel,
 *   stage 1  decode: the similarity GEMM and, when the plan splits tiles, its fix-up,
 *   stage 2  classify: the entropy / softmax / threshold kernel(s).
 * Passing NULL events turns the stage's recording off.  Process-wide; not for use
 * while other threads launch the same stage.
 */
int vsaogm_profile_events(int32_t stage, void* begin_event, void* end_event);

/* ---------------------------------------------------------------------------
 * Volumes: the method in three dimensions (Sec. III with a third axis; the 3-D
 * mapping named as future work in Sec. V).  A point's spectrum is
 * exp(i Theta[k].(x, y, z)); tiles are tiles_x x tiles_y x tiles_z boxes numbered
 * beta = (tz * tiles_y + ty) * tiles_x + tx, memory 2*beta + psi; a voxel queries its
 * own nearest tile; the entropy window is the ball of integer voxel offsets
 * dx^2 + dy^2 + dz^2 <= r^2.  Normalisation, maxima, squaring, softmax, signed
 * difference and threshold are those of the plane map.
 * ------------------------------------------------------------------------- */

typedef struct {
    int32_t dim;              /* D: even, >= 4 */
    const double* theta;      /* host [D][3] rad/m, conjugate-symmetric per axis, copied */
    double x0, y0, z0, x1, y1, z1;   /* layout box, m */
    int32_t tiles_x, tiles_y, tiles_z;   /* 1..64 each, at most 4096 tiles */
    int32_t device;
} vsaogm_volume_desc;

typedef struct {
    double x0, y0, z0, res;   /* voxel (i,j,l) centre = (x0+(i+.5)res, y0+(j+.5)res, z0+(l+.5)res) */
    int32_t nx, ny, nz;
} vsaogm_grid3_desc;

/* Create / destroy a volume (memories zero).  EINVAL for invalid descriptors. */
int vsaogm_volume_create(const vsaogm_volume_desc* desc, vsaogm_volume** out);
int vsaogm_volume_destroy(vsaogm_volume* vol);

/* Zero every memory of the volume (a fresh map of the same layout, cached grids kept).
   Asynchronous on the stream; EINVAL for a NULL volume. */
int vsaogm_volume_reset(vsaogm_volume* vol, vsaogm_stream stream);

/* Algorithm 1 in 3-D: bundle n points (device float [n][3] world metres, device uint8 labels
   0/1) into the memories; labels other than 0/1 are counted and skipped.  Asynchronous; work
   buffers grow on demand.  EINVAL for n < 0, NULL pointers with n > 0, or n >= 2^31 - 2048. */
int vsaogm_volume_encode(vsaogm_volume* vol, const float* xyz, const uint8_t* label, int64_t n,
                         vsaogm_stream stream);

/* Labels rejected since the last call (synchronises the stream). */
int vsaogm_volume_take_rejected(vsaogm_volume* vol, vsaogm_stream stream, int64_t* n_rejected);

/* Similarity of every voxel with its tile's normalised memories (eq. loc-query in 3-D):
   heat device float [2][nz][ny][nx] (class 1 = occupied), hmax device float [2] the
   per-class maxima.  precision: VSAOGM_BF16, VSAOGM_FP16 or VSAOGM_BF16X3 (the hi+lo
   split reaches fp32 accuracy); EINVAL for VSAOGM_FP32 and for grids whose voxels do
   not split into per-tile slabs along each axis. */
int vsaogm_volume_decode(vsaogm_volume* vol, const vsaogm_grid3_desc* grid, int32_t precision,
                         float* heat, float* hmax, vsaogm_stream stream);

/* Entropy classification of a volume (Algorithm 2 with a ball mask of radius r_occ for
   class 1 and r_emp for class 0, 0..24): ogm device float [nz][ny][nx] (or NULL), label
   device uint8 [nz][ny][nx].  Asynchronous.  Radii up to 4 run in one kernel; larger radii
   allocate and release a stream-ordered scratch of 2 nx ny nz floats (the entropy terms). */
int vsaogm_classify3(const vsaogm_grid3_desc* grid, const float* heat, const float* hmax,
                     int32_t r_occ, int32_t r_emp, float rho, float* ogm, uint8_t* label,
                     int32_t device, vsaogm_stream stream);

/*
 * vsaogm_classify3 for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same arguments,
 * kernels and results, but the entropy terms of radii above 4 go to a fixed scratch array the
 * library holds on each device it runs on (16 MiB, kept until the process ends) instead of a
 * stream-ordered allocation.  Radii above 4 require nx * ny * nz <= 2097152 voxels (EINVAL
 * otherwise, before any device work); radii up to 4 use no scratch and have no size limit.
 * No call allocates or frees device memory.  All calls on one device share its scratch, and the
 * scratch keeps the last call's contents (every voxel's entropy terms are written before they
 * are read, so nothing needs clearing): calls that overlap on one device, on different streams
 * or threads, race and must be serialised by the caller.  The first call on a device looks up
 * that device's scratch address (no allocation).
 */
int vsaogm_classify3_noalloc(const vsaogm_grid3_desc* grid, const float* heat, const float* hmax,
                             int32_t r_occ, int32_t r_emp, float rho, float* ogm, uint8_t* label,
                             int32_t device, vsaogm_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* VSAOGM_H */
