/*
 * libhasf -- homotopic alternating sequential filter (HASF) on 2D binary
 * images, (8,4) connectivity, for AMD Instinct MI355X (gfx950).
 *
 * The method is the topology-preserving smoother of Mahmoudi & Akil,
 * "Real Time Topological Image Smoothing On Shared Memory Parallel
 * Machines" (arXiv:1603.09337), Sec. 2 and Sec. 4.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - An image is H x W bytes, row-major, row pitch `ld` bytes (ld >= W).
 *    A nonzero byte is an object pixel; outputs are written as 0 or 1, and
 *    only the first W bytes of each row are read or written.
 *  - The plane outside the H x W window is background and never changes.
 *  - Image pointers are DEVICE pointers (e.g. torch tensors' data_ptr()).
 *    The caller owns them; the library never frees them.
 *  - Every call that touches the device is enqueued on the context's stream
 *    (hasf_set_stream) and is asynchronous to the host; hasf_sync() waits
 *    and reports a device error. Arguments are validated on the host before
 *    any device work; a rejected call enqueues nothing.
 *  - Limits: 1 <= H, 1 <= W, H + W <= 65535; 0 <= r <= HASF_R_MAX.
 *  - A context is used by one host thread at a time.
 *  - No C++ exception crosses this interface; every call returns a status.
 *
 * Thinning and thickening follow one deterministic schedule (the order the
 * paper leaves free is fixed so that results are reproducible bit for bit):
 * distance levels in increasing order; inside a level, rounds of four passes
 * over the 2x2 parity subfields (even,even), (even,odd), (odd,even),
 * (odd,odd) of (row, column) relative to the image origin, each pass acting
 * on the state left by the previous one, until a round changes nothing.
 */
#ifndef LIBHASF_H
#define LIBHASF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HASF_OK = 0,
    HASF_EINVAL = -1,     /* bad argument; nothing was enqueued */
    HASF_ENOMEM = -2,     /* device or host allocation failed */
    HASF_EDEVICE = -3,    /* a HIP call failed; see hasf_last_error */
    HASF_EAGAIN = -4,     /* server queue full (non-blocking submit) */
    HASF_ETIMEDOUT = -5,  /* wait timed out */
    HASF_EINTERNAL = -6   /* internal invariant violated */
} hasf_status;

/* Largest radius accepted by hasf_filter / hasf_filter_batch. */
#define HASF_R_MAX 15

typedef struct hasf_ctx hasf_ctx;

/* Defaults of hasf_opts.grid_min_pixels and hasf_opts.batch_grid_min_pixels.
 * A lone image of up to about 512 x 512 is filtered faster by one workgroup
 * than by row tiles; from 768 x 768 on the tiles take less than half the time
 * (measured at r = 2, 5, 8). */
#define HASF_GRID_MIN_PIXELS_DEFAULT ((size_t)1 << 19)
#define HASF_BATCH_GRID_MIN_PIXELS_DEFAULT ((size_t)1 << 23)

/*
 * An image is filtered either by one workgroup (its state in LDS when it fits)
 * or by a grid of workgroups (state in global memory, grid-wide barriers, one
 * launch per image). The grid finishes a large image sooner but spends more
 * device time on it, so it pays for a lone image and not in a busy batch.
 */
typedef struct {
    int device;             /* HIP device ordinal */
    size_t hbm_budget;      /* bytes the server may hold for frames; 0 = 1/4 of device memory */
    unsigned flags;         /* reserved, must be 0 */
    size_t grid_min_pixels; /* hasf_filter (and a batch of one): images with H * W >= this use the
                               grid. 0 = HASF_GRID_MIN_PIXELS_DEFAULT; SIZE_MAX = never */
    size_t batch_grid_min_pixels; /* the same for batches of several images and served frames.
                                     0 = HASF_BATCH_GRID_MIN_PIXELS_DEFAULT; SIZE_MAX = never */
    int tile_rows;          /* large images (hasf_filter, hasf_filter_cd, batches) whose rows fit are filtered
                               by tiles of this many own rows (see tile_cols), each tile's state in LDS with
                               tile_halo rows of its neighbours above and below, exchanged every tile_halo / 4
                               rounds;
                               0 = by image size (HASF_TILE_ROWS_SMALL below HASF_TILE_SMALL_PIXELS,
                               HASF_TILE_ROWS_LARGE from HASF_TILE_LARGE_PIXELS on, HASF_TILE_ROWS_DEFAULT
                               between); an even number >= 4 (raised to tile_halo);
                               -1 = never (the grid of workgroups with the state in global memory) */
    int tile_halo;          /* 0 = by image size (HASF_TILE_HALO_SMALL, HASF_TILE_HALO_DEFAULT or
                               HASF_TILE_HALO_LARGE, as tile_rows); a multiple of 4 from 4 to 32 */
    const char* tune_cache; /* NULL: lone images are routed by the fields above. Otherwise the path of a text
                               file of measured launch choices (created if missing, read at hasf_create):
                               the first lone image (hasf_filter, hasf_filter_cd, a batch of one) of a size
                               class -- H and W rounded up to multiples of 256, and r -- is filtered with each
                               candidate (one workgroup, row tiles of several heights and halos, the grid
                               kernel) on a copy of it, timed, and the fastest is appended to the file and
                               used for that class from then on. Every candidate runs the same schedule, so
                               results do not depend on the choice; the first image of a class costs about
                               2 x (number of candidates) filters more, plus an allocation of H ld bytes. */
    int tile_cols;          /* each band of tile_rows rows is cut into this many column tiles of whole 64-column
                               words (each with one word of its neighbours on each side), so that the tiles of an
                               image fill the CUs; 0 = as many as the CU count allows with at least 8 own words
                               each; more than the image's words or than the CUs allow is lowered */
} hasf_opts;

/* Tile shape by default (measured on MI355X, column tiles filling the CUs):
 * below HASF_TILE_SMALL_PIXELS 32 rows and 12 halo rows (1400x1300 r=6: 2.97 ms,
 * 64 and 16: 3.25 ms); up to HASF_TILE_LARGE_PIXELS 64 and 16 (2048^2 r=8:
 * 6.33 ms, 32 and 12: 6.78 ms); from there on 128 and 24 (4096^2 r=10: 20.5 ms,
 * 128 and 32: 21.0 ms, 64 and 16: 21.5 ms). */
#define HASF_TILE_SMALL_PIXELS ((size_t)1 << 21)
#define HASF_TILE_ROWS_SMALL 32
#define HASF_TILE_HALO_SMALL 12
#define HASF_TILE_ROWS_DEFAULT 64
#define HASF_TILE_HALO_DEFAULT 16
#define HASF_TILE_LARGE_PIXELS ((size_t)1 << 23)
#define HASF_TILE_ROWS_LARGE 128
#define HASF_TILE_HALO_LARGE 24

/* Create a context on opts->device (opts may be NULL: device 0, defaults).
 * The context owns its scratch memory and the default (null) stream. */
hasf_status hasf_create(const hasf_opts* opts, hasf_ctx** out);
void hasf_destroy(hasf_ctx* ctx);

/* Use `hip_stream` (a hipStream_t, e.g. torch.cuda.current_stream().cuda_stream)
 * for every later call on ctx. NULL selects the null stream. The context's
 * calls stay in order across a change: the new stream first waits for the
 * work already queued on the previous one (they share the context's scratch
 * memory). Setting the current stream again does nothing. */
hasf_status hasf_set_stream(hasf_ctx* ctx, void* hip_stream);

/* Wait for ctx's stream; returns HASF_EDEVICE if queued device work failed, and
 * HASF_EINTERNAL if a grid-filtered image since the last hasf_sync could not
 * complete (a grid-wide barrier timed out; that image is undefined). */
hasf_status hasf_sync(hasf_ctx* ctx);

const char* hasf_strerror(int status);
/* Detail of the last failure on ctx (ctx may be NULL: last failure on this thread). */
const char* hasf_last_error(const hasf_ctx* ctx);

/*
 * Schedule counts of the images filtered by a grid of workgroups (hasf_filter,
 * hasf_filter_cd and batches; not served frames), summed over the launches
 * since the context was created or last reset: one launch per image; the
 * rounds of the thinnings and thickenings (a round is the four subfield
 * passes over the whole image; a level that activated candidates takes its
 * rounds up to and including the first that changed nothing; this count is
 * a property of the schedule, not of how it is run); the distance levels
 * that activated candidates; and the grid-wide barriers. Waits for ctx's
 * stream. reset != 0 zeroes the counts after reading them.
 */
typedef struct {
    uint64_t launches;
    uint64_t rounds;
    uint64_t levels;
    uint64_t barriers;
} hasf_grid_counts;
hasf_status hasf_get_grid_counts(hasf_ctx* ctx, hasf_grid_counts* out, int reset);

/*
 * Simple-point table (Sec. 2, topological numbers T and T-bar; a point is
 * simple iff T = 1 and T-bar = 1). Host-only, pure.
 *   n = 8: object 8-adjacency, background 4-adjacency (the filter's pair);
 *   n = 4: object 4-adjacency, background 8-adjacency.
 * bits[m >> 5] bit (m & 31) is set iff neighbourhood code m is simple. Bit k
 * of m is neighbour k in the order E, NE, N, NW, W, SW, S, SE
 * (offsets (0,+1) (-1,+1) (-1,0) (-1,-1) (0,-1) (+1,-1) (+1,0) (+1,+1) in
 * (row, column)). HASF_EINVAL for other n or bits == NULL.
 */
hasf_status hasf_simple_lut(int n, uint32_t bits[8]);

/*
 * Exact squared Euclidean distance transform (Sec. 4.1):
 *   d2[i*ld_out + j] = min over feature pixels q of (i - qi)^2 + (j - qj)^2,
 * where the features are the nonzero bytes of feat (pitch ld) and, when
 * border_is_feature != 0, every pixel outside the window. With no feature at
 * all the result is UINT32_MAX everywhere. d2 is a device array of H rows of
 * ld_out >= W uint32 elements. feat and d2 must not overlap.
 */
hasf_status hasf_edt_sq(hasf_ctx* ctx, const uint8_t* feat, int H, int W, int64_t ld,
                        int border_is_feature, uint32_t* d2, int64_t ld_out);

/*
 * hasf_edt_sq for callers that cannot allocate memory (code being captured
 * into a HIP graph, tight serving loops, harnesses that forbid hipMalloc):
 * the same transform, the same kernels and the same arguments and results,
 * but it calls no hipMalloc, hipFree or other allocating routine. Its
 * scratch (per 32-row segment and column: a feature mask and the nearest
 * feature rows above and below; a list of row strips; marks and counters of
 * the columns that hold a feature; in all at most
 * ceil(H / 32) * W * 12 + 4 H + W / 8 + 6144 bytes) lives in
 * a device array of HASF_NOALLOC_SCRATCH_BYTES that the library holds on
 * each device it runs on until the process ends; 4096 x 4096 needs 6 MiB.
 * HASF_EINVAL (nothing enqueued) for the arguments hasf_edt_sq rejects and
 * for sizes whose scratch exceeds that maximum. Every call on one device
 * shares the array, whichever context makes it: calls that may overlap on
 * one GPU (other streams, other contexts, other threads) race and give
 * undefined results; calls queued in order on one stream do not.
 */
#define HASF_NOALLOC_SCRATCH_BYTES ((size_t)16 << 20)
hasf_status hasf_edt_sq_noalloc(hasf_ctx* ctx, const uint8_t* feat, int H, int W, int64_t ld,
                                int border_is_feature, uint32_t* d2, int64_t ld_out);

/*
 * Constrained homotopic thinning H(X, K) (Sec. 2): repeatedly deletes simple
 * points of X that are not in K, in increasing order of their squared
 * Euclidean distance to the background (outside of the window included),
 * computed once before thinning; ends when no such point is simple (the
 * constrained ultimate skeleton). X is updated in place. K may be NULL (empty)
 * and shares X's pitch.
 */
hasf_status hasf_homotopic_thin(hasf_ctx* ctx, uint8_t* X, const uint8_t* K, int H, int W,
                                int64_t ld);

/*
 * Constrained homotopic thickening *H(Y, V) (Sec. 2): repeatedly adds points
 * of V (inside the window) that are simple for the complement of Y, in
 * increasing order of their squared distance to Y, until stable. Y is updated
 * in place; V shares Y's pitch and must not be NULL.
 */
hasf_status hasf_homotopic_thicken(hasf_ctx* ctx, uint8_t* Y, const uint8_t* V, int H, int W,
                                   int64_t ld);

/*
 * hasf_homotopic_thin / hasf_homotopic_thicken for the connectivity pair
 * chosen by conn (Sec. 2): 8 (or 0) for 8-connected objects and a 4-connected
 * background, 4 for 4-connected objects and an 8-connected background. The
 * priorities do not depend on the pair. HASF_EINVAL for other conn.
 */
hasf_status hasf_homotopic_thin_conn(hasf_ctx* ctx, uint8_t* X, const uint8_t* K, int H, int W,
                                     int64_t ld, int conn);
hasf_status hasf_homotopic_thicken_conn(hasf_ctx* ctx, uint8_t* Y, const uint8_t* V, int H, int W,
                                        int64_t ld, int conn);

/*
 * HASF of order r with constraint set C (Sec. 2):
 *   X <- HF_r o HC_r o ... o HF_1 o HC_1 (X), in place, where for radius i
 *   HC_i(X) = *H(Y, V), Y = H(X, eps_i(X) u C), V = delta_i(Y) n X      (eq. i)
 *   HF_i(X) = H(Z, W),  Z = *H(X, delta_i(X)), W = eps_i(Z) u X          (eq. ii)
 * with Euclidean balls of radius i, thinning priority = squared distance to
 * the background, thickening priority = squared distance to the set being
 * thickened. C may be NULL (empty); C is intersected with X. r = 0 leaves X
 * unchanged (apart from normalising it to 0/1). No background constraint set
 * D is taken (D = empty).
 */
hasf_status hasf_filter(hasf_ctx* ctx, uint8_t* X, const uint8_t* C, int H, int W, int64_t ld,
                        int r);

/*
 * HASF^{C,D} (Sec. 2): as hasf_filter, with a background constraint set D --
 * the filling's thickening never adds a point of D, so D stays background
 * (D is intersected with the complement of X; D may be NULL: empty) -- and
 * the connectivity pair chosen by conn: 8 (or 0) for 8-connected objects and
 * a 4-connected background, 4 for 4-connected objects and an 8-connected
 * background (the simple points of (4,8) are those of (8,4) for the
 * complemented neighbourhood). D shares X's pitch. HASF_EINVAL for other conn.
 */
hasf_status hasf_filter_cd(hasf_ctx* ctx, uint8_t* X, const uint8_t* C, const uint8_t* D, int H, int W,
                           int64_t ld, int r, int conn);

/*
 * "r = infinity" (Tab. 1 reports it; the paper does not define it): the radius
 * loop of hasf_filter_cd, in the given order (as hasf_image.order), run for
 * i = 1, 2, ... and stopped after the first radius whose cutting and filling
 * leave X unchanged, or after radius r_max (r_max = 0: the saturation radius,
 * the least i with i^2 >= (H-1)^2 + (W-1)^2, from which on every radius
 * applies the same operator); *r_used would receive the last radius applied.
 * SWITCHED OFF in this version: after validating its arguments (HASF_EINVAL as
 * hasf_filter_cd, r_used == NULL, r_max < 0, flags other than 0 or
 * HASF_INF_COMPOSED) it returns HASF_EINTERNAL with *r_used = 0 and does no
 * device work.
 */
#define HASF_INF_COMPOSED 1u
hasf_status hasf_filter_inf(hasf_ctx* ctx, uint8_t* X, const uint8_t* C, const uint8_t* D, int H, int W,
                            int64_t ld, int conn, int order, int r_max, unsigned flags, int* r_used);

/*
 * One image of a batch (zero-initialise: D = NULL, conn = 0 and order = 0
 * give hasf_filter). order selects the sequence at every radius: 0 applies
 * HF_i o HC_i (the formula of Sec. 2, cutting first), 1 the dual HC_i o HF_i
 * (filling first); HASF_EINVAL for other values. A batch of one image is
 * hasf_filter on it, so hasf_filter_batch(ctx, &img, 1) filters one image in
 * the dual order.
 */
typedef struct {
    uint8_t* X;        /* device, in/out */
    const uint8_t* C;  /* device or NULL */
    int H, W;
    int64_t ld;
    int r;
    const uint8_t* D;  /* device or NULL: background constraint set, as in hasf_filter_cd */
    int conn;          /* 0 or 8: (8,4); 4: (4,8) */
    int order;         /* 0: cutting first (HF_i o HC_i); 1: filling first (HC_i o HF_i) */
} hasf_image;

/*
 * hasf_filter on n independent images of any sizes and radii, in one
 * persistent launch: each workgroup claims images from a queue ordered by
 * decreasing cost and filters them whole. The descriptor array is a host
 * array; it is copied before the call returns. Images must not overlap.
 * The result of each image equals hasf_filter on that image alone.
 */
hasf_status hasf_filter_batch(hasf_ctx* ctx, const hasf_image* imgs, int n);

/*
 * HASF on 3D binary volumes, 26-connected objects and 6-connected background
 * (Sec. 1: the method smooths 2D and 3D objects; Sec. 4.1: the distance
 * transforms run on 3D images). A volume is D x H x W contiguous bytes,
 * voxel (z, y, x) at (z H + y) W + x, nonzero = object; the outside of the box
 * is background and never changes. For each radius i = 1..r the cutting and
 * then the filling of Sec. 2 (eq. i, eq. ii) with 3D Euclidean balls; a voxel
 * is simple iff T26 = 1 and Tbar6 = 1 (26-components of the object voxels of
 * its 26-neighbourhood; 6-components of the background voxels of its
 * 18-neighbourhood that contain a face neighbour); thinning and thickening run
 * levels of increasing squared distance, and in a level rounds of eight
 * passes over the parity classes (z mod 2, y mod 2, x mod 2) in lexicographic
 * order until a round changes nothing. C (NULL: empty) is intersected with X.
 * Limits: D, H, W >= 1, D H W < 2^31, 0 <= r <= HASF_R_MAX. hasf_filter3_batch
 * filters n volumes in one launch (a workgroup per volume at a time), the
 * descriptor array being a host array copied before the call returns; the
 * library allocates about 9 D H W bytes of scratch per volume.
 */
typedef struct {
    uint8_t* X;        /* device, in/out */
    const uint8_t* C;  /* device or NULL */
    int D, H, W;
    int r;
} hasf_volume;
hasf_status hasf_filter3(hasf_ctx* ctx, uint8_t* X, const uint8_t* C, int D, int H, int W, int r);
hasf_status hasf_filter3_batch(hasf_ctx* ctx, const hasf_volume* vols, int n);

/*
 * The topological watershed's lowering (grey-level W-thinning), in place.
 * Sec. 3.1 places the topological watershed in the class of topology-based
 * operators the filter belongs to, without defining it; the operator is the
 * classical grey-level one on the (8,4) pair of Sec. 2. F is a grey-level
 * image (H rows of ld bytes, levels 0..255); lower sections {p : F(p) < k}
 * are 4-connected and the outside of the window belongs to none. A pixel is
 * W-destructible when it has a lower neighbour and the lower pixels of its
 * 8-neighbourhood 4-adjacent to it lie in one 4-component of them (T-bar = 1);
 * it is then lowered to the largest level of its lower neighbours. Rounds of
 * four passes over the 2x2 parity subfields of (row, column) run until a
 * round lowers nothing: the result is a fixed point, only lowers pixels, and
 * at every level k each 4-component of {F' < k} holds exactly one of {F < k}
 * (no merge of basins, no new minimum). Limits: H, W >= 1, H W < 2^31.
 * hasf_watershed_batch lowers n images in one launch (a workgroup per image at
 * a time; the descriptor array is a host array copied before the call
 * returns).
 */
typedef struct {
    uint8_t* F;   /* device, in/out */
    int H, W;
    int64_t ld;
} hasf_gimage;
hasf_status hasf_watershed(hasf_ctx* ctx, uint8_t* F, int H, int W, int64_t ld);
hasf_status hasf_watershed_batch(hasf_ctx* ctx, const hasf_gimage* imgs, int n);

/*
 * Per-label smoothing of a label (grey-level) image: the binary method of
 * Sec. 2 applied to each label as its own object set (Sec. 3.1 places
 * grey-level topological operators in the same class; the paper smooths
 * binary sets only). For k in [0, n), X_k = {p : L[p] == values[k]}
 * is filtered as hasf_filter(X_k, C = empty, r) -- (8,4), cutting first --
 * and written as 0/1 to plane k of out. The n planes are extracted by one
 * kernel and filtered in one batch (as hasf_filter_batch). The planes are
 * smoothed independently: they may overlap or leave pixels uncovered, and
 * no label image is rebuilt from them.
 *   L       device, H rows of ld bytes (read only)
 *   values  host array of n label values, no value twice; 1 <= n <= 256
 *   out     device; plane k starts at out + k * plane_stride and has H rows
 *           of ld_out bytes (ld_out >= W, plane_stride >= (H - 1) * ld_out + W,
 *           so planes do not overlap); it must not overlap L
 * HASF_EINVAL (before any device work) for NULL pointers, sizes as in
 * hasf_filter, n outside [1, 256], a repeated value, r outside
 * [0, HASF_R_MAX], a short ld_out or plane_stride, or out overlapping L.
 * On a later failure (HASF_ENOMEM, HASF_EDEVICE) the planes are undefined.
 */
hasf_status hasf_filter_labels(hasf_ctx* ctx, const uint8_t* L, int H, int W, int64_t ld,
                               const uint8_t* values, int n, int r, uint8_t* out, int64_t ld_out,
                               int64_t plane_stride);

/*
 * Served stream (continuous batching). hasf_serve starts a server on ctx's
 * device: a host dispatcher thread and a few launch lanes (streams of their
 * own, each with at most one launch of the batched filter kernel in flight).
 * Submitted frames wait in arrival order; whenever a lane is free, the
 * dispatcher admits the waiting frames whose scratch memory (bit planes and
 * level entries, kept on the device) fits in the server's device pool --
 * admission by HBM footprint -- and launches them as one batch. Frames that
 * arrive while others are being filtered go into the next free lane, so their
 * work overlaps on the device with the frames already there. A frame is
 * completed, and its scratch returned to the pool, as soon as the kernel has
 * finished it, not when its launch ends. Each frame's result equals
 * hasf_filter on that frame alone.
 *
 * Frames are device-resident: img->X (and img->C) are DEVICE pointers, filtered
 * in place; the caller keeps them alive and untouched until the frame's
 * hasf_serve_wait has returned. Frames must not overlap one another.
 * hasf_serve_submit_host takes a frame in host memory instead.
 */
#define HASF_SERVE_LANES_MAX 16
/* opts.flags bit: the persistent polling kernel (workgroups that stay resident
 * and claim frames from a host-mapped ring). Switched off: hasf_serve returns
 * HASF_EINTERNAL when it is set. */
#define HASF_SERVE_PERSISTENT 1u

typedef struct {
    size_t pool_bytes;     /* device memory for frame scratch; 0 = the context's hbm_budget */
    int lanes;             /* launches in flight at once, 1..HASF_SERVE_LANES_MAX; 0 = one per hardware
                              queue of the process (GPU_MAX_HW_QUEUES, 4 if unset), at most
                              HASF_SERVE_LANES_MAX. Lanes beyond the hardware queues share them. */
    int max_batch;         /* frames per launch (0 = 1024) */
    int max_pending;       /* submitted but not yet admitted; beyond it submit returns HASF_EAGAIN (0 = 1 << 20) */
    unsigned flags;        /* 0 (HASF_SERVE_PERSISTENT is switched off) */
    int express_lanes;     /* lanes that take only small frames, so that these never wait for a lane held by a
                              large frame; with express lanes no launch mixes small and large frames:
                              -1 = 3/8 of the lanes (at least 1; none with one lane), 0 = none; fewer than lanes */
    int express_max_pixels;/* a frame of at most this many pixels is small (0 = 1 << 19) */
} hasf_serve_opts;

typedef struct hasf_server hasf_server;

typedef struct {
    int status;            /* HASF_OK, or the frame's error */
    uint64_t ticket;
    double submit_s;       /* host steady clock, seconds */
    double done_s;         /* when the dispatcher saw the frame complete */
    double latency_ms;     /* done_s - submit_s */
} hasf_result;

typedef struct {
    uint64_t submitted, completed, rejected;
    uint64_t pending, in_flight;
    double p50_ms, p99_ms, max_ms;   /* latency over completed frames */
    double frames_per_s;             /* completed / (last done - first submit) */
    double mpixel_per_s;
    size_t pool_bytes, pool_peak_bytes;
    uint64_t kernel_launches;
    double frames_per_launch;        /* mean batch size of the launches */
    uint64_t batch_max;              /* largest batch launched */
} hasf_stats;

hasf_status hasf_serve(hasf_ctx* ctx, const hasf_serve_opts* opts, hasf_server** out);
/* Thread-safe. Validates the frame (HASF_EINVAL, nothing queued), then queues
 * it; HASF_EAGAIN when max_pending frames are already waiting. */
hasf_status hasf_serve_submit(hasf_server* s, const hasf_image* img, uint64_t* ticket);
/* The same for a frame in HOST memory: img->X (in/out), img->C and img->D
 * (or NULL) are host pointers (H rows of ld bytes). When the frame is admitted
 * the dispatcher enqueues copies of them into the frame's block of the device
 * pool (which is sized for them too: the scratch plus H W bytes per buffer,
 * each rounded up to 256), filters it there and copies X back; the frame
 * completes when its launch, and that copy, have ended (not on its own
 * completion word), and only then does hasf_serve_wait return. The caller
 * keeps the buffers alive and X untouched until then. The copies are
 * asynchronous only from page-locked memory (hipHostMalloc, pinned tensors);
 * from pageable memory they may hold up the dispatcher while they run.
 * Validation and errors as hasf_serve_submit. */
hasf_status hasf_serve_submit_host(hasf_server* s, const hasf_image* img, uint64_t* ticket);
/* Wait until the frame completes (timeout_ms < 0: forever); HASF_ETIMEDOUT if
 * it has not completed in time (the frame stays queued). A ticket can be
 * waited for once; out may be NULL. */
hasf_status hasf_serve_wait(hasf_server* s, uint64_t ticket, int timeout_ms, hasf_result* out);
hasf_status hasf_serve_stats(hasf_server* s, hasf_stats* out);
/* Finish every submitted frame, stop the kernel and free the server. */
hasf_status hasf_serve_stop(hasf_server* s);

#ifdef __cplusplus
}
#endif

#endif /* LIBHASF_H */
