/*
 * raypc.h -- C ABI of the brushed spherical-shell volume ray caster (gfx950).
 *
 * Method: direct volume ray casting of a multi-variable volume with
 * parallel-coordinates brushing (paper, Section 2 and Section 2.2): every
 * sample is tested against per-variable lower/upper bounds and a sample that
 * fails any of them is discarded and contributes nothing to the ray's colour;
 * samples that pass are classified through an RGBA transfer function on one
 * variable and composited front to back.  The volume carries an octree
 * level-of-detail pyramid with two coarser levels of 1/8 the cells each
 * (Section 2.1) and is rendered in progressive passes (Section 2.2).
 *
 * Conventions shared by every call
 *  - Return value: RAYPC_OK (0) or a RAYPC_ERR_* code.  No exception or
 *    signal crosses the ABI.  raypc_last_error() gives a message for the last
 *    failing call made by the calling thread.
 *  - A failing call leaves the context state unchanged.
 *  - Device pointers are HIP device addresses on the context's device;
 *    "stream" is a hipStream_t (NULL = the default stream).  Calls named
 *    "async" only enqueue work: outputs are valid once the stream is
 *    synchronised.  Host pointers are only read during the call.
 *  - A context is used by one host thread at a time.  State changes
 *    (brush, transfer function, options) apply to renders enqueued after the
 *    call; a render still in flight on another stream when its volume's brush
 *    or skip list is rewritten races with it, so synchronise such streams
 *    first.
 *  - Grid: cubic N^3, cell centred over [-1,1]^3 (x_i = -1 + (i + 1/2) 2/N),
 *    C order [z][y][x].  The shell is r_inner <= |x| <= r_outer; rays are
 *    marched only inside it.
 *  - Images: H x W x 4 float32, row 0 at the top, premultiplied RGBA.
 */
#ifndef RAYPC_H
#define RAYPC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    RAYPC_OK = 0,
    RAYPC_ERR_INVALID = 1,   /* bad argument; state unchanged */
    RAYPC_ERR_NOMEM = 2,     /* device allocation failed / would exceed a budget */
    RAYPC_ERR_DEVICE = 3,    /* a HIP runtime call failed; the context may be unusable */
    RAYPC_ERR_BUSY = 4,      /* resource in use (e.g. unloading a volume with requests in flight) */
    RAYPC_ERR_TIMEOUT = 5,   /* wait deadline passed */
    RAYPC_ERR_CANCELLED = 6, /* request cancelled before it ran */
    RAYPC_ERR_STATE = 7      /* call not valid in the current state (e.g. server not running) */
};

enum {
    RAYPC_STORAGE_F32 = 0,      /* 4 bytes per value */
    RAYPC_STORAGE_F16 = 1,      /* IEEE binary16, round to nearest even, subnormals kept; a brick's
                                 * values are held with copies of the next brick's first x voxels
                                 * (2.25 bytes per voxel) */
    RAYPC_STORAGE_U8_BRICK = 2, /* 8-bit codes with a (scale, offset) pair per 8^3 brick; the codes
                                 * of a brick are held with copies of the next bricks' first x and
                                 * y voxels (1.27 bytes per voxel) */
    /* Flag OR-ed into a storage type: keep only the compact layout.  Without it the library also
     * keeps neighbourhood records: per voxel a 4-byte entry, in brick blocks that also copy the next
     * brick's first x voxels (binary16: the values at (x, y) and (x, y + 1); float32 and 8-bit: the
     * float32 (decoded) value), so that a sample's trilinear fetch takes 2 (binary16) or 4 loads
     * of 8 bytes instead of 8 (float32), 4 (binary16) or 2 code loads and 4 (scale, offset) loads
     * (8-bit).  Records cost 4.5 bytes per voxel and field besides the compact data; both layouts
     * hold the same values and render identically. */
    RAYPC_STORAGE_COMPACT = 0x100
};

#define RAYPC_MAX_FIELDS 8
#define RAYPC_MAX_LODS 3
#define RAYPC_TF_ENTRIES 256
#define RAYPC_TF_SLOTS 8
#define RAYPC_BRICK 8

typedef struct raypc_ctx raypc_ctx;

/* Pinhole camera.  fov_y_deg is the vertical field of view in (0, 180);
 * right = normalize(forward x up), true up = right x forward; pixel (px, py)
 * looks through its centre. */
typedef struct {
    float eye[3];
    float target[3];
    float up[3];
    float fov_y_deg;
} raypc_camera;

/* Create a context on HIP device `device`; *out receives it.  The context owns
 * every device allocation it makes.  Errors: RAYPC_ERR_INVALID (bad device or
 * NULL out), RAYPC_ERR_DEVICE. */
int raypc_create(int device, raypc_ctx **out);

/* Wait for the context's own work, stop its server if running and free
 * everything it owns.  NULL is ignored. */
void raypc_destroy(raypc_ctx *ctx);

/* Message of the last failing call on this thread ("" if none).  Valid until
 * the next call from the same thread. */
const char *raypc_last_error(void);

/* Library version as MAJOR*10000 + MINOR*100 + PATCH. */
int raypc_version(void);

/*
 * Load a multi-variable volume (paper, Section 1: a snapshot holds several
 * output variables; Section 2.1: derived variables are added in
 * preprocessing).
 *   n_fields   1..8 variables; fields[f] points at N^3 float32 values.
 *   n          N, a multiple of 32 in [32, 1024].
 *   on_device  0: fields[] are host pointers (copied);  1: device pointers
 *              (read only, e.g. torch tensors).
 *   storage    RAYPC_STORAGE_*: how every level is kept in device memory
 *              (optionally | RAYPC_STORAGE_COMPACT).
 *   n_lods     1..3 levels: level l+1 is the 2x2x2 mean of level l (float32,
 *              fixed summation order), built from float32 data and only then
 *              encoded (Section 2.1: two coarser levels with 1/8 the cells).
 *   r_inner, r_outer  shell radii, 0 <= r_inner < r_outer <= 1.
 *   stream     work is enqueued here; the call synchronises it before
 *              returning, so inputs may be freed or reused afterwards.
 *   volume_id  receives a handle (> 0).
 * Builds, per level: the encoded brick-ordered field data, the per-brick
 * (min, max) tables of the stored values over each brick's 9^3 window and
 * its eight 4^3 sub-bricks' tables, and (unless compact) the neighbourhood
 * records.  It also keeps, on the host, the values and level-0 sub-brick
 * (min, max) of 2 048 random shell cells (a fixed SplitMix64 stream), from
 * which each brush's field test order is chosen.  The brush starts with no
 * variable restricted.
 * Errors: RAYPC_ERR_INVALID (argument out of range, NULL pointer, or a
 * non-finite input value), RAYPC_ERR_NOMEM, RAYPC_ERR_DEVICE.
 */
int raypc_load_fields(raypc_ctx *ctx, int n_fields, int n, const float *const *fields, int on_device,
                      int storage, int n_lods, float r_inner, float r_outer, void *stream, int *volume_id);

/* Free a volume.  RAYPC_ERR_BUSY while serving requests reference it. */
int raypc_unload(raypc_ctx *ctx, int volume_id);

/* Describe a loaded volume.  Any output pointer may be NULL.  *bytes is the
 * device memory it holds (field data, tables, skip lists). */
int raypc_volume_info(const raypc_ctx *ctx, int volume_id, int *n_fields, int *n, int *n_lods, int *storage,
                      uint64_t *bytes);

/*
 * Set the brush of a volume (paper, Section 2: upper and lower bounds for
 * each variable, set in the parallel-coordinates plot; Section 2.2: the
 * volume data is not modified and nothing is rebuilt).
 *   active[f] != 0 restricts variable f to the inclusive interval
 *   [lo[f], hi[f]]; inactive variables are not tested.  lo > hi selects
 *   nothing; +-INFINITY bounds are allowed; NaN bounds are rejected.
 * Copies the arrays; touches no device memory (the affected skip lists are
 * recomputed by the next render).  Renders test the restricted variables in
 * an order chosen per brush: greedily, the variable that the fewest sampled
 * shell cells still passing the earlier tests pass (cells in sub-bricks the
 * skip rule drops do not count); a sample that fails one test fetches no
 * further variable, and any order gives the same image.
 * Errors: RAYPC_ERR_INVALID.
 */
int raypc_set_brush(raypc_ctx *ctx, int volume_id, int n_fields, const uint8_t *active, const float *lo,
                    const float *hi);

/*
 * Define transfer-function slot `slot` (0..7; slot 0 is the one raypc_render
 * uses).  The colour comes from one variable (paper, Section 3: radial
 * velocity, density anomaly or temperature anomaly colour the volume).
 *   field       variable that is classified.
 *   vmin < vmax value range mapped onto the table; values outside clamp.
 *   rgba        n_entries x 4 straight (not premultiplied) colour and opacity,
 *               each in [0, 1]; entry i sits at normalised value i/255 and the
 *               table is interpolated linearly.
 *   n_entries   must be 256.
 *   ref_step    world-space length the table's opacity refers to (> 0);
 *               a sample of length l gets alpha = 1 - (1 - A)^(l / ref_step).
 * The table is uploaded into a new version of the slot, so renders already
 * enqueued (on any stream) keep the table they were given and renders enqueued
 * after the call returns use the new one.  The upload runs on the context's own
 * stream and the call waits for that copy, not for a device drain (the runtime
 * may map that stream onto a hardware queue it shares with other streams, whose
 * earlier work the copy then waits behind).  A slot keeps 256 versions; a
 * version is rewritten only after the launches that read it have finished (an
 * event per version and stream, recorded by every render), so a definition
 * waits only if renders enqueued 256 definitions earlier are still running.
 * Serving requests copy the table at submission.  Errors: RAYPC_ERR_INVALID,
 * RAYPC_ERR_DEVICE.
 */
int raypc_set_transfer_function(raypc_ctx *ctx, int slot, int field, float vmin, float vmax, const float *rgba,
                                int n_entries, float ref_step);

/* raypc_set_transfer_function ordered on `stream` instead: the table is copied to
 * pinned host memory and its upload enqueued on `stream`, and the call returns
 * without waiting; renders enqueued on `stream` after it use the new table, renders
 * enqueued before it (on any stream) keep theirs, and renders on other streams use
 * it once the caller orders them after `stream` (events).  Same arguments, version
 * rule and errors as raypc_set_transfer_function; the first call allocates the
 * context's pinned staging (8 MiB). */
int raypc_set_transfer_function_async(raypc_ctx *ctx, int slot, int field, float vmin, float vmax,
                                      const float *rgba, int n_entries, float ref_step, void *stream);

/* Coordinate axes of the brush (Section 2.1 derives the altitude from the position; the paper's
 * appendix cuts the volume by Cartesian coordinates on the same plot).  Axes 0, 1, 2 are the world
 * x, y, z of a sample's position (the volume spans [-1, 1]^3), axis 3 is its radius |p|.
 * active[a] enables axis a with the inclusive bounds [lo[a], hi[a]] (world units); a sample whose
 * position falls outside an enabled axis is discarded exactly like a sample failing a field bound
 * (and is not fetched).  The radius test is made on float32 squares: r^2 >= lo^2 when lo > 0,
 * r^2 <= hi^2 when hi >= 0, nothing passes when hi < 0.  For cells (raypc_pc_lines,
 * raypc_export_voxel_mask) the position is the cell centre fl32(fl32(2 i + 1) / N) - 1 per axis.
 * Arrays of 4, copied; NaN bounds: RAYPC_ERR_INVALID with the state unchanged.  Default: no axis
 * enabled. */
int raypc_set_coordinate_brush(raypc_ctx *ctx, int volume_id, const uint8_t *active, const float *lo,
                               const float *hi);

/*
 * Early ray termination threshold (default 0.99; >= 1 disables) and the
 * background (NULL = transparent black, which keeps the output
 * premultiplied).  With a background, out = C + (1 - A) bg_rgb,
 * A_out = A + (1 - A) bg_a.  Errors: RAYPC_ERR_INVALID (threshold <= 0 or NaN,
 * background outside [0, 1]).
 */
int raypc_set_options(raypc_ctx *ctx, float ert_threshold, const float *bg_rgba);

/*
 * Level-of-detail choice (paper, Section 2: a level-of-detail structure is
 * used to raise rendering performance; the rule is this library's): with P
 * the projected diameter of the outer sphere in pixels, the level is
 * clamp(ceil(log2(N / P)), 0, n_lods - 1) when N > P and 0 otherwise, and 0
 * when the eye is inside the outer sphere.  Pure host computation.
 */
int raypc_select_lod(const raypc_ctx *ctx, int volume_id, const raypc_camera *cam, int width, int height,
                     int *lod);

/*
 * Render one view (async).  lod = -1 picks the level with raypc_select_lod.
 * step is the sample spacing in voxels of the rendered level, in [1/64, 64].
 * rgba_out: device buffer of height*width*4 float32, written once per pixel.
 * Uses the volume's brush, transfer-function slot 0 and the options.
 * Errors: RAYPC_ERR_INVALID (width/height outside [1, 16384], bad lod, step,
 * camera with NaN, fov outside (0, 180), up parallel to the view direction,
 * slot 0 undefined or naming a field the volume lacks), RAYPC_ERR_NOMEM,
 * RAYPC_ERR_DEVICE.
 */
int raypc_render(raypc_ctx *ctx, int volume_id, const raypc_camera *cam, int width, int height, int lod,
                 float step, float *rgba_out, void *stream);

/*
 * Progressive passes (paper, Section 2.2: while the camera is stationary
 * additional render passes raise the number of samples per pixel).  Pass k of
 * n_passes (1..8) renders the full image at step * 2^(n_passes - 1 - k) into
 * outs[k]; every pass equals raypc_render at that step (async).
 */
int raypc_render_progressive(raypc_ctx *ctx, int volume_id, const raypc_camera *cam, int width, int height,
                             int lod, float step, int n_passes, float *const *outs, void *stream);

/* Jittered progressive pass (Section 2.2: while the camera does not move, further passes raise the
 * samples per pixel and lower the noise).  Pass `pass` of `n_passes` (1..256) renders like
 * raypc_render with every pixel's sample grid shifted along the ray: the samples of a shell
 * segment [a, b] are the pieces of [a, b] cut at a - s ds + j ds (j integer), each evaluated at
 * its midpoint with its own length in the opacity correction, where
 *   s = min(fl32(fl32(pass + xi) / n_passes), 1 - 2^-24),  xi = (z >> 48) * 2^-16,
 *   z = output number c + 1 of a SplitMix64 generator started at `seed`, for the counter
 *       c = pass * 2^32 + (py * width + px)  (Steele, Lea and Flood, OOPSLA 2014),
 * so each pass draws its offsets from its own stratum [pass, pass + 1) / n_passes.  s = 0 is the
 * partition of raypc_render.  Outputs (device, H x W x 4 float32, any may be NULL but not both
 * images): rgba_out = this pass; mean_inout = running mean of the passes, overwritten with this
 * pass when pass == 0, else updated m <- m + (c - m) / (pass + 1), so after passes 0..k it is
 * their mean.  nominal / composited: per-pixel sample counts as in raypc_render_debug (NULL: not
 * counted).  Uses the volume's brush and transfer slot 0; lod -1 selects the level.  Async on
 * `stream`.  Errors: as raypc_render, plus RAYPC_ERR_INVALID for pass / n_passes out of range. */
int raypc_render_jittered(raypc_ctx *ctx, int volume_id, const raypc_camera *cam, int width, int height, int lod,
                          float step, int pass, int n_passes, uint64_t seed, float *rgba_out, float *mean_inout,
                          uint32_t *nominal, uint32_t *composited, void *stream);

/* Launch shape of single-image renders (raypc_render, _debug, _progressive, _jittered, _depth, _work):
 *   tile_log2w  t in 0..4: each wave marches the 16 rays of a (1 << t) x (16 >> t) pixel tile
 *               (1x16, 2x8, 4x4, 8x2 or 16x1; default 2, 4x4), four lanes per ray;
 *   super_log2  s in 0..3: the tiles are dealt to the 8 XCDs in super-tiles of 2^(s+1) x 2^(s+1)
 *               tiles (default 2: 32x32 pixels with 4x4 tiles), round-robin, so that a super-tile's
 *               rays share one XCD's L2 while every XCD gets tiles from all over the image.
 * The shape changes timing only, never an image (every ray is marched by its own four lanes, the
 * same way whatever tile it is in).  Serving launches keep 4x4 tiles and 32x32-pixel super-tiles.
 * Errors: RAYPC_ERR_INVALID. */
int raypc_set_launch_shape(raypc_ctx *ctx, int super_log2, int tile_log2w);
int raypc_get_launch_shape(raypc_ctx *ctx, int *super_log2, int *tile_log2w);

/* Autotuner of the launch shape: renders the given view (as raypc_render, with the volume's brush
 * and transfer slot 0) once untimed and then `repeats` (1..1000) times back to back for each of the
 * 20 shapes (tile_log2w t = 0..4, super_log2 s = 0..3), timing each run with HIP events on a stream
 * of its own, and makes the fastest the context's launch shape (the default t = 2, s = 2 stays
 * unless another shape is more than 1 % faster, so that runs on one device agree).  times_ms (20
 * floats, index 4 t + s; may be NULL) receives the mean time of one render per shape; best_super and
 * best_tile (may be NULL) the chosen shape.  Synchronous; allocates one image for the duration of
 * the call.  On error the previous launch shape stays.  Errors: as raypc_render, plus
 * RAYPC_ERR_INVALID for repeats out of range and RAYPC_ERR_NOMEM. */
int raypc_autotune_render(raypc_ctx *ctx, int volume_id, const raypc_camera *cam, int width, int height, int lod,
                          float step, int repeats, float *times_ms, int *best_super, int *best_tile);

/* raypc_render plus the depth that image warping reprojects with (Sections 2 and 2.2 warp the last
 * delivered image to fill the frames the renderer has not produced yet; the paper names no depth,
 * so the one taken is this): depth_out (device, H x W float32) receives the mean distance from the
 * eye, along the unit ray, of the composited samples' midpoints, each weighted by its share
 * T_before * alpha of the pixel's opacity (the weights sum to the opacity 1 - T, before any
 * background), and +inf where nothing was composited.  rgba_out is exactly raypc_render's image.
 * depth_out must not be NULL.  Async on `stream`.  Errors: as raypc_render. */
int raypc_render_depth(raypc_ctx *ctx, int volume_id, const raypc_camera *cam, int width, int height, int lod,
                       float step, float *rgba_out, float *depth_out, void *stream);

/* Image warping of a frame to another camera pose (Sections 2 and 2.2: the display hides the
 * renderer's varying frame rate and latency by warping the last image it delivered).  Inputs
 * (device): rgba (src_height x src_width x 4 float32) and depth (src_height x src_width float32,
 * as raypc_render_depth writes it; +inf or NaN: a point at infinity) of a frame rendered with
 * src_cam.  Every source pixel's ray (through its centre, as the render casts it) is followed to
 * its depth and the point projected through dst_cam; it lands on the destination pixel containing
 * the projection unless it lies on or behind dst_cam's image plane or outside its image.  Per
 * destination pixel the point nearest to dst_cam's eye wins (the lowest source index among equal
 * distances).  A pixel nothing landed on takes the winner of its eight neighbours farthest from
 * the eye (the highest source index among equal distances), else stays empty.  The landing
 * pixel and the distance are decided in float32, one correctly rounded operation at a time in the
 * order: sx = (((px + 0.5) (2/W)) - 1) tan(fov/2) W/H, sy = (1 - (py + 0.5) (2/H)) tan(fov/2),
 * e = (fwd + sx right) + sy up, n = e / sqrt((e.x e.x + e.y e.y) + e.z e.z), v = (eye + d n) -
 * dst_eye (v = n at infinity), z = v . fwd' (same summation order), x = (v . right') / (z tan'
 * W'/H'), y = (v . up') / (z tan'), landing pixel (floor((x + 1) (W'/2)), floor((1 - y) (H'/2))),
 * distance sqrt(v . v); the camera frames are those of raypc_render (double, rounded to float32).
 * Outputs (device, dst_height x dst_width): rgba_out = the winner's RGBA unchanged (0 where empty);
 * depth_out (may be NULL) = the winner's distance from dst_cam's eye (+inf where empty);
 * source_out (may be NULL) = the winner's linear source index py * src_width + px (-1 where
 * empty).  Outputs must not overlap the inputs or each other.  The context keeps two 8-byte-per-
 * destination-pixel z-buffers, used in turn (each warp empties the other one's pixels for the next
 * warp) and grown (after a device synchronisation) when a larger image comes; warps in flight on
 * different streams of one context race on them.  Sizes 1..16384 per side.
 * Async on `stream`.  Errors: RAYPC_ERR_INVALID (NULL input or output image, bad camera or size,
 * overlapping buffers), RAYPC_ERR_NOMEM. */
int raypc_warp(raypc_ctx *ctx, const raypc_camera *src_cam, int src_width, int src_height, const float *rgba,
               const float *depth, const raypc_camera *dst_cam, int dst_width, int dst_height, float *rgba_out,
               float *depth_out, int32_t *source_out, void *stream);

/* raypc_warp for callers that cannot allocate device memory (code under HIP graph capture, tight
 * display loops, harnesses that forbid hipMalloc): the same warp, arguments and outputs, bit for
 * bit, with its z-buffer taken from a fixed array in the library's own device memory instead of
 * the context's buffers.  It calls no hipMalloc, hipFree or other allocating routine.  The array
 * holds RAYPC_WARP_NOALLOC_MAX_PIXELS keys (8 bytes each, 32 MiB) on every GPU the library runs
 * on, until the process ends; its address on the context's device is looked up once, at
 * raypc_create.  Every call on one GPU (from any context or thread) shares that GPU's array: each
 * call first fills its dst_width x dst_height leading keys with the empty key (a fill kernel, no
 * memset node), so nothing of an earlier call is seen, but calls that overlap in time on one GPU
 * (on different streams, or from different threads) race on the array and their outputs are then
 * undefined; serialise them (one stream, or events).  Async on `stream`.  Errors: as raypc_warp,
 * and RAYPC_ERR_INVALID when dst_width x dst_height exceeds RAYPC_WARP_NOALLOC_MAX_PIXELS (nothing
 * is launched then); RAYPC_ERR_NOMEM is never returned. */
#define RAYPC_WARP_NOALLOC_MAX_PIXELS (2048 * 2048)
int raypc_warp_noalloc(raypc_ctx *ctx, const raypc_camera *src_cam, int src_width, int src_height,
                       const float *rgba, const float *depth, const raypc_camera *dst_cam, int dst_width,
                       int dst_height, float *rgba_out, float *depth_out, int32_t *source_out, void *stream);

/* The device's measured ceilings, against which the renderer's rates are quoted (the vendor's peak
 * figures are theoretical): *copy_bytes_per_s = bytes moved per second (reads plus writes) by a
 * STREAM-like copy of a 1 GiB float32 array, *fma_lane_ops_per_s = FP32 fused multiply-adds per
 * second of a loop of independent FMA chains in every lane of enough waves to fill every SIMD (one
 * FMA counted as one lane operation; the library is built without packed FP32); each the best of
 * five timed passes after a warm-up.  Allocates and frees 2 GiB of scratch memory; synchronises
 * `stream`.  Errors: RAYPC_ERR_INVALID (NULL argument), RAYPC_ERR_DEVICE. */
int raypc_measure_peaks(raypc_ctx *ctx, double *copy_bytes_per_s, double *fma_lane_ops_per_s, void *stream);

/* ---------------------------------------------------------------- debug exports
 * For parity tests and accounting.  All outputs are device buffers (async). */

/* Stored (decoded) values of one level and field as float32 [z][y][x]. */
int raypc_export_level(raypc_ctx *ctx, int volume_id, int lod, int field, float *out, void *stream);

/* Per-brick (min, max) table of one level and field: nb^3 pairs of float32,
 * bricks in [bz][by][bx] order (nb = N_l / 8). */
int raypc_export_minmax(raypc_ctx *ctx, int volume_id, int lod, int field, float *out, void *stream);

/* Per-sub-brick (min, max) of one level and field (Section 2.2's empty-space
 * skipping at a finer grain): for every brick, its eight 4^3 sub-bricks, each
 * over voxel indices [4s, min(4s+4, N_l-1)] per axis; pair 8 k + sx + 2 sy + 4 sz
 * belongs to brick k, sub-brick (sx, sy, sz).  nb^3 * 16 float32. */
int raypc_export_minmax_sub(raypc_ctx *ctx, int volume_id, int lod, int field, float *out, void *stream);

/* Skip bits of one level for the volume's brush and transfer slot `slot`:
 * ceil(nb^3 / 32) uint32 words; brick k is bit k % 32 of word k / 32. */
int raypc_export_skiplist(raypc_ctx *ctx, int volume_id, int lod, int slot, uint32_t *out, void *stream);

/* Sub-brick skip flags of one level for the volume's brush and transfer slot
 * `slot` (the skip rule applied to each sub-brick's (min, max)): nb^3 bytes,
 * byte k = brick k, bit sx + 2 sy + 4 sz set when that sub-brick is skipped.
 * A skipped brick has all eight bits set.  The renderer skips by these. */
int raypc_export_subskip(raypc_ctx *ctx, int volume_id, int lod, int slot, uint8_t *out, void *stream);

/* The renderer's per-brick flag words for the same brush and slot: nb^3
 * uint16, word k = brick k; bits 0-7 are raypc_export_subskip's byte, bit 8 is
 * set when every brick of brick k's aligned 2x2x2-brick group has all eight
 * sub-bricks skipped, bit 9 the same for its aligned 4x4x4-brick group (a
 * group cut by the grid's upper faces counts the bricks inside the grid), and
 * bit 10 is brick k's bit of raypc_export_skiplist.  A sample in an empty
 * group is stepped past the whole group.  `out` is device
 * memory of nb^3 * 2 bytes, written asynchronously on `stream`; errors as for
 * raypc_export_subskip. */
int raypc_export_skip_words(raypc_ctx *ctx, int volume_id, int lod, int slot, uint16_t *out, void *stream);

/* Voxel brush mask of one level: N_l^3 bytes, 1 where every active variable
 * lies in its [lo, hi]. */
int raypc_export_voxel_mask(raypc_ctx *ctx, int volume_id, int lod, uint8_t *out, void *stream);

/* ---------------------------------------------------------------- parallel coordinates
 * Lines of the parallel-coordinates plot and their linking to the brush (Section 2.1: up to
 * 100 000 randomly chosen cells are stored as the plot's lines; Section 2: the bounds set on the
 * plot's axes select the subset of the data that is shown).  For n_lines cell indices of level
 * `lod` (device uint32, z N_l^2 + y N_l + x, chosen by the caller):
 *   values  device float32 [n_lines][n_fields]: the stored value of every field, i.e. the line's
 *           coordinates on the plot's axes (NULL: not written);
 *   passes  device uint8 [n_lines]: 1 when every active field of the volume's brush lies in its
 *           inclusive [lo, hi], else 0 (NULL: not written);
 *   hist    device uint32 [n_fields][n_bins][2], overwritten: per field, the number of lines per
 *           bin of the axis [axis_lo[f], axis_hi[f]] (host arrays of n_fields floats), all lines in
 *           [.][.][0] and lines that pass in [.][.][1] (NULL: not written).  The bin of value v is
 *           decided in float32: inv = fl32(1 / fl32(hi - lo)), x = fl32(fl32(fl32(v - lo) * inv)
 *           * n_bins), bin = clamp(floor(x), 0, n_bins - 1), so values outside the axis land in
 *           the end bins.
 * A cell index >= N_l^3 gives NaN values, flag 0 and no histogram entry.  n_lines in [0, 2^24],
 * n_bins in [1, 512] (when hist is given), axis ranges finite with hi > lo.  Async on `stream`.
 * Errors: RAYPC_ERR_INVALID (nothing is launched). */
int raypc_pc_lines(raypc_ctx *ctx, int volume_id, int lod, int n_lines, const uint32_t *cells,
                   const float *axis_lo, const float *axis_hi, int n_bins, float *values, uint8_t *passes,
                   uint32_t *hist, void *stream);

/* raypc_render plus per-pixel sample counts: nominal = samples visited up to
 * and including an early-termination stop; composited = samples that passed
 * the brush with non-zero table opacity.  touched_bricks (ceil(nb^3 / 32)
 * words of the rendered level, zeroed by the caller) receives a bit for every
 * brick that holds the base corner of an evaluated (not skipped) sample.
 * flags bit 0 disables empty-space skipping.  nominal / composited /
 * touched_bricks may be NULL. */
int raypc_render_debug(raypc_ctx *ctx, int volume_id, const raypc_camera *cam, int width, int height, int lod,
                       float step, float *rgba_out, uint32_t *nominal, uint32_t *composited,
                       uint32_t *touched_bricks, int flags, void *stream);

/* raypc_render plus the renderer's own work per pixel, for the roofline accounting (Section 2.2:
 * a brush change rebuilds nothing, so the skipped share of the samples is decided per frame):
 * evaluated = samples not skipped (the empty-space skip jumps over the others), fetched = field
 * values interpolated for them (a sample fetches no field after its first failed brush test, and
 * the transfer-function field last); both count up to and including an early-termination stop,
 * like raypc_render_debug's nominal count.  evaluated / fetched: device H x W uint32, either may
 * be NULL.  The image is raypc_render's.  Uses the volume's brush and transfer slot 0; async on
 * `stream`.  Errors: as raypc_render. */
int raypc_render_work(raypc_ctx *ctx, int volume_id, const raypc_camera *cam, int width, int height, int lod,
                      float step, float *rgba_out, uint32_t *evaluated, uint32_t *fetched, void *stream);

/* ---------------------------------------------------------------- serving
 * A request loop that keeps volumes resident and renders many requests at once
 * (continuous batching).  It replaces the paper's asynchronous render thread
 * (Section 2.2: rendering is decoupled from the application's frame rate):
 * a scheduler thread owned by the context admits requests in submission order
 * while a request slot is free and the memory budget allows, and every
 * launch ("step") marches 4x4-pixel tiles of all admitted requests together,
 * oldest request first; requests that arrive while others run join the next
 * step.  Each request carries its own brush and names a transfer-function slot;
 * the brush, the table and the options (termination threshold, background)
 * are captured when it is submitted, so later set_brush /
 * set_transfer_function / set_options calls do not affect it.  A request's image is exactly
 * what raypc_render would produce for the same view, brush and table.
 * submit / poll / wait / cancel / request_times / release / stats may be
 * called from any thread.  The other context calls keep their one-thread rule
 * and must not unload a volume that queued requests name (RAYPC_ERR_BUSY). */

typedef struct {
    uint64_t mem_budget_bytes; /* device memory in-flight requests may hold: each counts its image
                                  (width*height*16 bytes, caller-owned) plus its skip flag words (two bytes per brick);
                                  0 = unlimited */
    int max_inflight;          /* request slots, 1..256 */
    int tiles_per_step;        /* work per step in units of 8x8 pixels, 0 = 32768 (about one 1920x1080 image) */
    int steps_in_flight;       /* steps queued ahead on the device, 1..4 (0 = 2) */
} raypc_server_cfg;

typedef struct {
    int volume_id;
    raypc_camera camera;
    int width, height;                /* 1..16384 */
    int lod;                          /* -1 = raypc_select_lod */
    float step;                       /* voxels of the rendered level, [1/64, 64] */
    uint8_t active[RAYPC_MAX_FIELDS]; /* the request's brush, as in raypc_set_brush; entries beyond */
    float lo[RAYPC_MAX_FIELDS];       /* the volume's field count are ignored */
    float hi[RAYPC_MAX_FIELDS];
    uint8_t coord_active[4];          /* the request's coordinate axes, as in */
    float coord_lo[4], coord_hi[4];   /* raypc_set_coordinate_brush */
    int tf_slot;                      /* defined transfer-function slot */
    float *out;                       /* device, height*width*4 float32, 16-byte aligned, caller-owned,
                                         valid until the request is done */
    double deadline_ms;               /* must be admitted within this many ms of submission; <= 0: none */
} raypc_request;

/* Request states reported by raypc_poll; a negative state is -RAYPC_ERR_* (failed, timed out or
 * cancelled). */
enum { RAYPC_REQ_QUEUED = 0, RAYPC_REQ_RUNNING = 1, RAYPC_REQ_DONE = 2 };

typedef struct {
    uint64_t submitted, completed, timed_out, cancelled, failed;
    uint64_t steps, tiles;
    uint64_t bytes_in_use, peak_bytes_in_use;
    int inflight, queued;
} raypc_server_stats;

/* Start the context's scheduler.  RAYPC_ERR_STATE if one is running; RAYPC_ERR_INVALID for a bad
 * configuration; RAYPC_ERR_NOMEM / RAYPC_ERR_DEVICE if its buffers cannot be created. */
int raypc_server_start(raypc_ctx *ctx, const raypc_server_cfg *cfg);

/* Stop accepting requests, finish every queued and running one, join the scheduler. */
int raypc_server_stop(raypc_ctx *ctx);

/* Queue a copy of *req; *ticket identifies it.  Checks the request as raypc_render does and
 * returns RAYPC_ERR_NOMEM if it alone exceeds the memory budget, RAYPC_ERR_STATE if no server
 * runs.  Never blocks on the device. */
int raypc_submit(raypc_ctx *ctx, const raypc_request *req, uint64_t *ticket);

/* Current state of a ticket (RAYPC_REQ_* or -RAYPC_ERR_*); RAYPC_ERR_INVALID for an unknown one. */
int raypc_poll(raypc_ctx *ctx, uint64_t ticket, int *state);

/* Block until the request is done (RAYPC_OK: its image is complete in device memory), failed
 * (its error code) or timeout_ms passed (RAYPC_ERR_TIMEOUT; < 0 waits without limit). */
int raypc_wait(raypc_ctx *ctx, uint64_t ticket, int timeout_ms);

/* Cancel a request that is still queued (it ends with -RAYPC_ERR_CANCELLED); RAYPC_ERR_BUSY once
 * it has been admitted. */
int raypc_cancel(raypc_ctx *ctx, uint64_t ticket);

/* Host monotonic timestamps in ms: [0] submitted, [1] admitted, [2] first tile launched,
 * [3] completed (0 where not reached). */
int raypc_request_times(raypc_ctx *ctx, uint64_t ticket, double times_ms[4]);

/* Forget a finished ticket (its state and times); queued or running tickets: RAYPC_ERR_BUSY. */
int raypc_release(raypc_ctx *ctx, uint64_t ticket);

int raypc_server_get_stats(raypc_ctx *ctx, raypc_server_stats *stats);

#ifdef __cplusplus
}
#endif
#endif /* RAYPC_H */
