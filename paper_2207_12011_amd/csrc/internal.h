// internal.h -- declarations shared by the library's HIP translation units.
// Not part of the public ABI (that is include/raypc.h).
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/raypc.h"

#include <cstddef>
#include <cstdint>

namespace raypc {

constexpr int kMaxFields = 8;
constexpr int kBrick = 8;           // brick edge in voxels
constexpr int kBrickVoxels = 512;   // 8^3
constexpr int kBlockPix = 4;        // a serving step's wave tiles are 4 x 4 pixels

enum Storage : int { kF32 = 0, kF16 = 1, kU8 = 2 };
// Kernel variants: a storage type, read from the compact layout or from neighbourhood records.
enum Kind : int {
    kKindF32 = 0, kKindF16 = 1, kKindU8 = 2, kKindF32Rec = 3, kKindF16Rec = 4, kKindU8Rec = 5, kKinds = 6
};

// Brick-ordered number of voxel (x, y, z) on a level with nb bricks per axis: bricks in [bz][by][bx]
// order, 512 voxels each.  Inside a brick the voxels form eight 4^3 sub-bricks (x, y, z half-index in
// bits 6, 7, 8), each [z][y][x], so a compact cluster of samples touches few cache lines whatever the
// view direction.  The number is a sum of independent per-axis parts (see axis_x/y/z).  It places the
// float32 compact values; binary16 and 8-bit compact values and the neighbourhood records of every
// storage are held in blocks (block_index9, u8_addr).
__host__ __device__ inline uint32_t axis_x(int x) {
    return (static_cast<uint32_t>(x >> 3) << 9) | (static_cast<uint32_t>((x >> 2) & 1) << 6) |
           static_cast<uint32_t>(x & 3);
}
__host__ __device__ inline uint32_t axis_y(int y, int nb) {
    return ((static_cast<uint32_t>(y >> 3) * nb) << 9) | (static_cast<uint32_t>((y >> 2) & 1) << 7) |
           (static_cast<uint32_t>(y & 3) << 2);
}
__host__ __device__ inline uint32_t axis_z(int z, int nb) {
    return ((static_cast<uint32_t>(z >> 3) * nb * nb) << 9) | (static_cast<uint32_t>((z >> 2) & 1) << 8) |
           (static_cast<uint32_t>(z & 3) << 4);
}
__host__ __device__ inline uint32_t brick_addr(int x, int y, int z, int nb) {
    return axis_x(x) + axis_y(y, nb) + axis_z(z, nb);
}
// Brick-local index (0..511) of the voxel at offsets (x, y, z) in 0..7 within its brick.
__host__ __device__ inline uint32_t brick_local(int x, int y, int z) {
    return (static_cast<uint32_t>(z >> 2) << 8) | (static_cast<uint32_t>(y >> 2) << 7) |
           (static_cast<uint32_t>(x >> 2) << 6) | (static_cast<uint32_t>(z & 3) << 4) |
           (static_cast<uint32_t>(y & 3) << 2) | static_cast<uint32_t>(x & 3);
}

// 8-bit codes use a layout of their own: each 8^3 brick is a 9 x 9 x 8 block of bytes, [z][y][x]
// (648 bytes, bricks in [bz][by][bx] order), holding its 512 codes and, at local x = 8 and y = 8,
// copies of the codes one voxel beyond its upper x and y faces (the next bricks' first voxels; at the
// grid's upper faces the last voxel again, where the interpolation clamps).  The four corners of a
// cell at one z then lie at byte offsets 0, 1, 9 and 10 from its base voxel, within one 12-byte load.
// A copy keeps the code of the voxel it copies: each corner is still decoded with the (scale, offset)
// pair of the brick the voxel belongs to.
constexpr uint32_t kU8BrickBytes = 648;
__host__ __device__ inline uint32_t brick_index(int x, int y, int z, int nb) {
    return static_cast<uint32_t>(x >> 3) + static_cast<uint32_t>(nb) * (static_cast<uint32_t>(y >> 3) +
                                                                        static_cast<uint32_t>(nb) * static_cast<uint32_t>(z >> 3));
}
__host__ __device__ inline uint32_t u8_addr(int x, int y, int z, int nb) {
    return brick_index(x, y, z, nb) * kU8BrickBytes + static_cast<uint32_t>(z & 7) * 81u +
           static_cast<uint32_t>(y & 7) * 9u + static_cast<uint32_t>(x & 7);
}
// Bytes of one field's 8-bit code array on a level with nb bricks per axis: the bricks plus 16 bytes,
// so that the 12-byte load at the last brick's last voxel stays inside the array.
__host__ __device__ inline size_t u8_field_bytes(int nb) {
    return static_cast<size_t>(nb) * nb * nb * kU8BrickBytes + 16;
}

// Blocks of 9 x 8 x 8 entries per 8^3 brick, [z][y][x] (576 entries, bricks in [bz][by][bx] order):
// the brick's 512 voxels and, at local x = 8, a copy of the voxel one beyond its upper x face (the
// next brick's first voxel; at the grid's upper x face the last voxel again, as the interpolation
// clamps), so the two corners of a cell's row (x0 and x0 + 1 at one y and z) are adjacent entries.
// binary16 compact values are 2-byte entries (a row is one 4-byte load); the neighbourhood records are
// 4-byte entries (an x pair, or for binary16 a 2x2 (x, y) quad, is one 8-byte load).
constexpr uint32_t kBlockValues = 576;
constexpr uint32_t kBlockYStride = 9, kBlockZStride = 72;  // entries between neighbours in y and in z
__host__ __device__ inline uint32_t block_index9(int x, int y, int z, int nb) {
    return brick_index(x, y, z, nb) * kBlockValues + static_cast<uint32_t>(z & 7) * kBlockZStride +
           static_cast<uint32_t>(y & 7) * kBlockYStride + static_cast<uint32_t>(x & 7);
}
// Bytes of one field's binary16 array on a level: the bricks plus 16 bytes of padding.
__host__ __device__ inline size_t f16_field_bytes(int nb) {
    return static_cast<size_t>(nb) * nb * nb * kBlockValues * 2 + 16;
}
// Bytes of one field's records (4-byte entries of the same numbering).
__host__ __device__ inline size_t record_bytes(int nb) {
    return static_cast<size_t>(nb) * nb * nb * kBlockValues * 4 + 16;
}

// Coordinate axes of a brush at a position (x, y, z world units): bit a of mask enables axis a
// (x, y, z, radius) with inclusive bounds [clo[a], chi[a]]; the radius is tested on float32
// squares, r^2 = fl32(fl32(fl32(x x) + fl32(y y)) + fl32(z z)) against clo[3] <= r^2 <= chi[3].
__device__ __forceinline__ bool coord_ok(uint32_t mask, const float* clo, const float* chi, float x, float y,
                                         float z) {
    bool ok = true;
    if (mask & 1u) ok = ok && x >= clo[0] && x <= chi[0];
    if (mask & 2u) ok = ok && y >= clo[1] && y <= chi[1];
    if (mask & 4u) ok = ok && z >= clo[2] && z <= chi[2];
    if (mask & 8u) {
        const float r2 = __fadd_rn(__fadd_rn(__fmul_rn(x, x), __fmul_rn(y, y)), __fmul_rn(z, z));
        ok = ok && r2 >= clo[3] && r2 <= chi[3];
    }
    return ok;
}
// World coordinate of the centre of cell i on an N-cell axis: fl32(fl32(2 i + 1) / N) - 1.
__device__ __forceinline__ float cell_coord(int i, int n) {
    return __fsub_rn(__fdiv_rn(static_cast<float>(2 * i + 1), static_cast<float>(n)), 1.0f);
}

// ------------------------------------------------------------------ preprocessing launchers
// Sets *flag on a non-finite value; raises *maxbits to the bits of the largest finite |value|.
hipError_t launch_count_nonfinite(const float* x, size_t count, unsigned int* flag, unsigned int* maxbits,
                                  hipStream_t s);
// binary16 storage scales a field by 2^k, k = max(0, 14 - e) for its largest |value| f 2^e
// (f in [0.5, 1)): scale[0] = 2^k, scale[1] = 2^-k, *exponent = k, from *maxbits on the device.
hipError_t launch_f16_scale(const unsigned int* maxbits, float* scale, int* exponent, hipStream_t s);
hipError_t launch_gather_cells(const float* x, const uint32_t* cells, int k, float* out, hipStream_t s);
hipError_t launch_gather_pairs(const float2* x, const uint32_t* idx, int k, float2* out, hipStream_t s);
// out[N/2]^3 = 2x2x2 mean of in[N]^3 (both linear [z][y][x] float32).
hipError_t launch_lod_build(const float* in, int n, float* out, hipStream_t s);
// Encode a linear float32 level into brick-ordered storage (u8 also writes per-brick (scale, offset);
// binary16 stores the values times f16_scale[0], a power of two, or times 1 when it is null).
hipError_t launch_encode(const float* in, int n, int storage, void* out, float2* u8par, const float* f16_scale,
                         hipStream_t s);
// Per-brick (min, max) of stored values over the 9^3 apron window, and per 4^3 sub-brick over its 5^3
// apron window: out_sub[8 brick + sx + 2 sy + 4 sz].
// (Binary16 codes are taken times f16_scale[1] when it is not null: the tables hold field values.)
hipError_t launch_minmax(const void* data, const float2* u8par, int n, int storage, float2* out, float2* out_sub,
                         const float* f16_scale, hipStream_t s);
// Neighbourhood records: 4-byte entries in the 9 x 8 x 8 blocks (block_index9; entry x = 8 is the next
// brick's first voxel, coordinates clamped to N-1): binary16 keeps the values at (x, y) and (x, y + 1)
// (low and high half), float32 the value, 8-bit storage its decoded float32 value.  A trilinear fetch
// reads 8 bytes (two entries) twice (binary16: the 2x2 corners of the planes z0 and z1) or four times
// (float32, 8-bit: the x pairs of the rows (y0 | y1, z0 | z1)).
hipError_t launch_records(const void* data, const float2* u8par, int n, int storage, void* out, hipStream_t s);
// Decode stored values back to linear [z][y][x] float32.
// (binary16 codes times f16_descale)
hipError_t launch_decode(const void* data, const float2* u8par, int n, int storage, float* out, float f16_descale,
                         hipStream_t s);

struct MaskArgs {
    const void* field[kMaxFields];
    const float2* u8par[kMaxFields];
    float lo[kMaxFields], hi[kMaxFields];
    float descale[kMaxFields];  // binary16: 2^-k of the field's scale (1 otherwise)
    int n_active;  // fields [0, n_active) of the arrays above are the active ones
    uint32_t coord_mask;  // coordinate axes at the cell centre (as RenderArgs)
    float clo[4], chi[4];
    int n, nb, storage;
    uint8_t* out;  // linear [z][y][x]
};
hipError_t launch_voxel_mask(const MaskArgs& a, hipStream_t s);

// Parallel-coordinates lines: per cell index, the stored values, the brush flag and per-field
// histograms of all / passing lines (bins decided in float32, see raypc_pc_lines).
constexpr int kMaxPcBins = 512;
struct PcArgs {
    const void* field[kMaxFields];
    const float2* u8par[kMaxFields];
    uint8_t active[kMaxFields];
    float lo[kMaxFields], hi[kMaxFields];       // the volume's brush
    float axis_lo[kMaxFields], inv[kMaxFields]; // inv = fl32(1 / fl32(axis_hi - axis_lo))
    float descale[kMaxFields];                  // binary16: 2^-k of the field's scale (1 otherwise)
    uint32_t coord_mask;                        // coordinate axes at the cell centre (as RenderArgs)
    float clo[4], chi[4];
    int n_fields, storage, n, nb, n_bins, n_lines;
    const uint32_t* cells;                      // z N^2 + y N + x
    float* values;                              // [n_lines][n_fields] or null
    uint8_t* passes;                            // [n_lines] or null
    uint32_t* hist;                             // [n_fields][n_bins][2] or null
};
hipError_t launch_pc_lines(const PcArgs& a, hipStream_t s);

struct SkipArgs {
    const float2* minmax[kMaxFields];      // active fields' brick (min, max) tables
    const float2* minmax_sub[kMaxFields];  // and their sub-brick tables
    float lo[kMaxFields], hi[kMaxFields];
    int n_active;
    const float2* tf_minmax;               // tables of the transfer-function field
    const float2* tf_minmax_sub;
    float vmin, inv_range;                 // inv_range = fl32(1 / (vmax - vmin))
    int next_nonzero[257];                 // smallest entry index >= i with opacity > 0 (256 if none)
    uint32_t coord_mask;                   // coordinate axes (kernel form, see coord_ok)
    float clo[4], chi[4];
    int n, nb;                             // level size in voxels and bricks per axis
    float h;                               // fl32(2 / n)
    uint32_t n_bricks;
    uint16_t* out_sub;                     // per-brick flag words, see below
};
// Per-brick flag words: bits 0-7 the sub-brick skip flags (bit sx + 2 sy + 4 sz: that 4^3 sub-brick is
// skipped), bit 8 set when every brick of the brick's aligned 2^3-brick group (16^3 voxels) has all
// eight sub-bricks skipped, bit 9 the same for its aligned 4^3-brick group (32^3 voxels; groups cut by
// the grid's upper faces count only the bricks inside it), bit 10 the brick's own skip bit (the skip
// rule on the brick's window).  launch_skip writes them; launch_pack_skip_bits packs the bit-10 skip
// bits 32 to a word (brick k: bit k % 32 of word k / 32).
constexpr uint32_t kBrickSkipBit = 0x400u;
hipError_t launch_skip(const SkipArgs& a, hipStream_t s);
hipError_t launch_pack_skip_bits(const uint16_t* words, uint32_t n_bricks, uint32_t* out, hipStream_t s);

// ------------------------------------------------------------------ ray marcher
struct RenderArgs {
    // fields in "slot" order: slots [0, n_brushed) are brushed, the transfer-function field is
    // slot tf_slot (< n_brushed when it is brushed itself, else == n_brushed)
    const void* field[kMaxFields];
    const float2* u8par[kMaxFields];
    const void* rec[kMaxFields];  // neighbourhood records, in the same slot order (record kinds only)
    float lo[kMaxFields], hi[kMaxFields];
    int n_brushed, tf_slot;
    uint32_t coord_mask;          // coordinate axes in use (bit a = axis a: x, y, z, radius)
    float clo[4], chi[4];         // their bounds; radius as float32 squares (see raypc_set_coordinate_brush)
    int n, nb;
    uint32_t field_bytes;         // bytes of one field of this level (buffer range; f16 and u8 only)
    uint32_t par_bytes;           // bytes of one field's per-brick (scale, offset) table (u8)
    uint32_t rec_bytes;           // bytes of one field's records (buffer range; fields below 4 GiB only)
    float half_n;                 // N / 2: u = (p + 1) N/2 - 1/2
    const uint16_t* skip;         // per-brick flag words of launch_skip (nullptr: no skipping)
    const float4* tf;             // 256 straight-RGBA entries
    float vmin, inv_range;
    float inv_ref;                // 1 / ref_step
    float ert;                    // termination threshold (used only when ert_on)
    int ert_on;
    float bg[4];
    int has_bg;
    float eye[3], fwd[3], right[3], upv[3];
    float sx_scale, sy_scale;     // tan(fov/2) * aspect, tan(fov/2)
    float inv_w2, inv_h2;         // 2 / W, 2 / H
    int width, height;
    float oo;                     // |eye|^2
    float r_in2, r_out2;          // squared radii
    float c_in, c_out;            // |eye|^2 - r^2
    int has_inner;
    float ds, inv_ds;             // sample spacing (world units) and its reciprocal
    float4* out;                  // H x W premultiplied RGBA
    uint32_t* nominal;            // debug counts (only in the counting variant)
    uint32_t* composited;
    uint32_t* touched;            // debug: bit per brick read by an evaluated sample (may be null)
    uint32_t* evaluated;          // debug: per pixel, samples not skipped, up to the termination stop (may be null)
    uint32_t* fetched;            // debug: per pixel, field values interpolated for those samples (may be null)
    int blocks_x, n_blocks;       // wave tiles per row, total
    int tile_log2w;               // a wave tile is (1 << t) x (16 >> t) pixels (serving: t = 2, 4 x 4)
    int super_log2;               // single-image launches: super-tiles of 2^(s+1) x 2^(s+1) wave tiles dealt over the XCDs
    // jittered progressive passes (jittered kernels only): pass `pass` of `n_passes` shifts each
    // pixel's sample grid by s ds, s from a SplitMix64 stream at `seed`; `mean` (may be null)
    // holds the running mean of the passes, updated with weight inv_pass1 = 1 / (pass + 1)
    uint64_t seed;
    uint32_t pass, n_passes;
    float inv_pass1;
    float4* mean;
    float* depth;                 // depth kernels only: H x W opacity-weighted depth (+inf: nothing composited)
};
hipError_t launch_render(const RenderArgs& a, int kind, bool counts, hipStream_t s);
hipError_t launch_render_jittered(const RenderArgs& a, int kind, bool counts, hipStream_t s);
hipError_t launch_render_depth(const RenderArgs& a, int kind, hipStream_t s);
constexpr int kMaxSuperLog2 = 3;  // super-tiles of up to 16 x 16 wave tiles (64 x 64 pixels for 4 x 4 tiles)
constexpr int kMaxTileLog2W = 4;  // wave tiles from 1 x 16 (t = 0) to 16 x 1 (t = 4) pixels
constexpr int kDefaultTileLog2W = 2;  // 4 x 4 pixels

// Image warping: a camera's frame in float32 (the render's frame), and one warp's buffers.
struct WarpCamera {
    float eye[3], fwd[3], right[3], up[3];
    float sx_scale, sy_scale;     // tan(fov/2) * aspect, tan(fov/2)
    float inv_w2, inv_h2;         // 2 / W, 2 / H
    int width, height;
};
struct WarpArgs {
    WarpCamera src, dst;
    const float4* rgba;           // src H x W
    const float* depth;           // src H x W
    uint32_t n_src;               // src H * W
    unsigned long long* keys;     // dst H x W z-buffer (scratch)
    int clear_keys;               // keys not known to be empty: fill them first
    unsigned long long* next_keys;  // the other z-buffer: the resolve empties its dst H x W pixels (may be null)
    float4* out;                  // dst H x W
    float* out_depth;             // may be null
    int32_t* out_src;             // may be null
};
hipError_t launch_warp(const WarpArgs& a, hipStream_t s);
// The allocation-free warp's z-buffer: a fixed array of kWarpScratchPixels keys per GPU (32 MiB),
// shared by every call on that GPU.  warp_scratch returns its address on `device`, which must be
// the current device (looked up once per device, then cached).
constexpr size_t kWarpScratchPixels = RAYPC_WARP_NOALLOC_MAX_PIXELS;
constexpr int kMaxDevices = 64;
hipError_t warp_scratch(int device, unsigned long long** ptr);
// Measured device ceilings (peaks.hip): best of several passes of a 1 GiB device copy (bytes moved
// per second, reads plus writes) and of an FMA loop filling every SIMD (FP32 lane operations per second).
hipError_t measure_peaks(double* copy_bytes_per_s, double* fma_ops_per_s, hipStream_t s);
// Work of one batched launch, passed by value in the kernel arguments: range r covers items
// [end[r-1], end[r]) (end[-1] = 0), which march tiles first[r], first[r] + 1, ... of the request whose
// arguments are descs[slot[r]].  Every descriptor's volume uses the launch's kernel kind.
constexpr int kMaxRanges = 32;
struct BatchRanges {
    int n;
    int end[kMaxRanges];
    int first[kMaxRanges];
    int slot[kMaxRanges];
};
// Requests of one batched launch share the kernel kind, the field-count class (the number of brushed
// fields, or -1, the run-time count variant, when coordinate axes are enabled) and the record offset
// width (batch_wide: record kinds whose record fields reach 4 GiB take 64-bit offsets).
int batch_nb_class(const RenderArgs& a);
bool batch_wide(const RenderArgs& a, int kind);
hipError_t launch_render_batch(const RenderArgs* descs, const BatchRanges& ranges, int kind, int nb_class, bool wide,
                               hipStream_t s);

// Record fields below 4 GiB (every level of grids up to 812^3) can be read at 32-bit byte offsets.
inline bool narrow_records(const RenderArgs& a) {
    return static_cast<uint64_t>(a.n) * a.n * a.n * 8u < 0x100000000ull;
}

}  // namespace raypc
