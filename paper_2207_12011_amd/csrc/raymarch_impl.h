// raymarch_impl.h -- device code of the brushed shell ray march (gfx950), shared by the single-image
// launches (raymarch.hip) and the batched, jittered and depth launches (raymarch_batch.hip).
//
// Paper, Section 2.2: during ray marching every restricted variable is queried
// at every sample; a sample whose values do not satisfy the bounds set in the
// parallel-coordinates plot is discarded and contributes nothing to the ray's
// colour.  Samples that pass are classified through a transfer function on one
// variable and composited front to back.  The cost of the brush therefore
// grows with the number of restricted variables (linear, as the paper notes).
//
// Discrete definition implemented (and mirrored by the FP64 oracle):
//  * pinhole ray through each pixel centre, row 0 at the top;
//  * shell = outer ball minus the open inner ball, t >= 0, at most two
//    segments; the sphere hits use the numerically stable quadratic
//    (Haines et al., "Precision Improvements for Ray/Sphere Intersection",
//    Ray Tracing Gems, 2019): disc = r^2 - |o - (o.d) d|^2, q = -b - sign(b) sqrt(disc),
//    t = c / q and t = q;
//  * per segment [a, b]: n = ceil((b - a) / ds) samples, sample j covers
//    [a + j ds, min(a + (j+1) ds, b)] and is taken at its midpoint;
//  * trilinear fetch at u = (p + 1) N/2 - 1/2 with corners clamped to [0, N-1];
//  * brush: every active variable inside its inclusive [lo, hi];
//  * 256-entry straight-RGBA table, linear between entries, opacity corrected
//    to the sample length: alpha = 1 - (1 - A)^(len / ref_step);
//  * front-to-back "over", stop once the accumulated opacity reaches the
//    termination threshold.
//
// Mapping to CDNA4.  Four lanes share a ray and evaluate four consecutive
// samples of it at once (binary16 records: two such groups per step, each lane
// taking samples j and j + 4, their loads issued together); a wave64 covers a
// 4 x 4 pixel tile, so the samples it fetches per step form a compact cluster
// of a few voxels on a side, which the brick-ordered layouts serve from a
// handful of cache lines.  Each group of four
// is merged in order with DPP quad broadcasts: every lane replays the four sequential
// front-to-back updates, stopping at the first sample whose accumulated
// opacity reaches the threshold, so the result is bit for bit the sequential
// sum whatever the grouping.  Every lane of a quad holds identical copies of
// the ray state.  A wave
// leaves its loop when all 16 of its rays have terminated or left the shell.
// 4^3 sub-bricks flagged as skipped are stepped over without fetching (the whole
// 8^3 brick when all eight of its sub-bricks are flagged): every sample whose
// base corner lies in such a box would be discarded or fully transparent, so
// skipping changes no value.  Blocks of one wave (4 x 4 pixels) are dealt to the
// XCDs by super-tiles (32 x 32 pixels unless the launch shape says otherwise); the transfer function
// sits in LDS.
#pragma once
#include <hip/hip_fp16.h>

#include "internal.h"

// 24-bit unsigned multiply (the LLVM intrinsic, full rate; HIP's __umul24 may be selected as a
// quarter-rate 64-bit multiply-add).
__device__ uint32_t raypc_mul_u24(uint32_t a, uint32_t b) __asm("llvm.amdgcn.mul.u24.i32");

namespace raypc {
namespace {

constexpr float kSkipShrink = 2e-3f;  // voxels: shrink of a skipped box before computing its exit
constexpr float kSkipMargin = 0.01f;  // samples: margin on the first sample after a skipped box
constexpr int kQuad = 4;              // lanes (consecutive samples) per ray
constexpr int kWaveRays = 16;         // a wave marches 16 rays, on a tile of (1 << t) x (16 >> t) pixels

// Global-memory view of a pointer.  Pointers read from memory (the batched launch takes its
// arguments from a device array) would otherwise be accessed with generic flat loads.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* global_ptr(const void* p) {
    return reinterpret_cast<const __attribute__((address_space(1))) T*>(reinterpret_cast<uintptr_t>(p));
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// log2 of the bytes per stored value.
template <int S>
constexpr int kLogBytes = S == kF32 ? 2 : (S == kF16 ? 1 : 0);

// Where one field's stored values come from.  binary16 and 8-bit fields are read with buffer loads
// (a uniform 128-bit resource plus a 32-bit per-lane byte offset, range-checked by the hardware
// against the field size); float32 fields (up to 4 GiB per field) with global loads.
template <int S>
struct Source;
template <>
struct Source<kF32> {
    const float* base;
};
template <>
struct Source<kF16> {
    __amdgpu_buffer_rsrc_t rsrc;
};
template <>
struct Source<kU8> {
    __amdgpu_buffer_rsrc_t rsrc, par;
};

constexpr int kRawBufferFlags = 0x00020000;  // raw (untyped) buffer, 32-bit data format

template <int S>
__device__ __forceinline__ Source<S> source(const RenderArgs& A, int k) {
    Source<S> src;
    if constexpr (S == kF32) {
        src.base = static_cast<const float*>(A.field[k]);
    } else {
        src.rsrc = __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(A.field[k]), 0, static_cast<int>(A.field_bytes),
                                                     kRawBufferFlags);
        if constexpr (S == kU8)
            src.par = __builtin_amdgcn_make_buffer_rsrc(const_cast<float2*>(A.u8par[k]), 0,
                                                        static_cast<int>(A.par_bytes), kRawBufferFlags);
    }
    return src;
}

// Stored float32 value at byte offset `ob` (the other storages are read by rows, see fetch).
template <int S>
__device__ __forceinline__ float corner(const Source<S>& src, uint32_t ob) {
    static_assert(S == kF32, "binary16 and 8-bit values are read by rows (fetch)");
    return global_ptr<float>(reinterpret_cast<const char*>(src.base) + ob)[0];
}

// Trilinear interpolation written as a weighted sum of the eight corners (index bit 0 = x, bit 1 = y,
// bit 2 = z).  The weights depend only on the sample position, so one sample computes them once for
// all its fields; each field then costs eight multiply-adds, which take binary16 corners as operands
// directly (mixed-precision FMA) instead of converting them first.
struct Tri {
    float w[8];
};
__device__ __forceinline__ Tri tri_weights(float wx, float wy, float wz) {
    const float ax = 1.0f - wx, ay = 1.0f - wy, az = 1.0f - wz;
    const float q0 = ay * az, q1 = wy * az, q2 = ay * wz, q3 = wy * wz;  // (y, z) = (0,0) (1,0) (0,1) (1,1)
    Tri t;
    t.w[0] = ax * q0, t.w[1] = wx * q0, t.w[2] = ax * q1, t.w[3] = wx * q1;
    t.w[4] = ax * q2, t.w[5] = wx * q2, t.w[6] = ax * q3, t.w[7] = wx * q3;
    return t;
}
__device__ __forceinline__ float blend(const Tri& t, float c0, float c1, float c2, float c3, float c4, float c5,
                                       float c6, float c7) {
    float v = fmaf(t.w[0], c0, 0.0f);
    v = fmaf(t.w[1], c1, v);
    v = fmaf(t.w[2], c2, v);
    v = fmaf(t.w[3], c3, v);
    v = fmaf(t.w[4], c4, v);
    v = fmaf(t.w[5], c5, v);
    v = fmaf(t.w[6], c6, v);
    return fmaf(t.w[7], c7, v);
}

// Trilinear value from the 8 stored corners.  float32: o[] holds the corners' byte offsets.
// binary16 (the 9 x 8 x 8 blocks of block_index9): o[0..3] are the byte offsets of the corners (x0, y, z)
// of the rows (y, z) = (y0, z0), (y1, z0), (y0, z1), (y1, z1), each the start of one 4-byte load of the
// row's two values (eight 2-byte loads took 1.24 ms for the headline frame, four row loads 0.85 ms).
// 8-bit codes (the 9 x 9 x 8 brick blocks of u8_addr): o[0] and o[1] are the byte offsets of
// the cell's base voxel (x0, y0) in the z0 and z1 planes, each the start of one 12-byte load whose bytes
// 0, 1, 9 and 10 are the plane's four corners; o[2..5] the bricks of the corners (x0, y, z) of the rows
// (y, z) = (y0, z0), (y1, z0), (y0, z1), (y1, z1); o[6] is nonzero where x1 lies in the next brick.
// Each corner is decoded with the (scale, offset) pair of its own brick: one 16-byte load per row
// brings the pairs of the row's brick and of the next brick in x, stored side by side, and the row's
// x1 corner takes the second pair where it lies in that brick.  Without a branch, a field costs two
// code loads and four pair loads (one byte and one pair load per corner, with a pair load per
// straddling corner in a branch each, took 2.16 ms for the headline frame; rows of pairs with byte
// loads 1.80 ms).  The second pair of the last brick lies beyond the pair array: a zero pair is
// stored there, and no corner takes it (the upper corner clamps onto the grid's last voxel).
template <int S>
__device__ __forceinline__ float fetch(const Source<S>& src, const uint32_t (&o)[8], const Tri& t) {
    if constexpr (S == kU8) {
        typedef unsigned int u32x3 __attribute__((ext_vector_type(3)));
        const u32x3 p0 = __builtin_amdgcn_raw_buffer_load_b96(src.rsrc, static_cast<int>(o[0]), 0, 0);
        const u32x3 p1 = __builtin_amdgcn_raw_buffer_load_b96(src.rsrc, static_cast<int>(o[1]), 0, 0);
        // codes of the corners (bit 0 = x, bit 1 = y, bit 2 = z): bytes 0 and 1 of the first word, 1 and
        // 2 of the third (plane bytes 9 and 10)
        const uint32_t code[8] = {p0.x, p0.x >> 8, p0.z >> 8, p0.z >> 16, p1.x, p1.x >> 8, p1.z >> 8, p1.z >> 16};
        const bool next = o[6] != 0;
        float c[8];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const u32x4 pr = __builtin_amdgcn_raw_buffer_load_b128(src.par, static_cast<int>(o[2 + r] * 8u), 0, 0);
            const float q0 = static_cast<float>(code[2 * r] & 0xFFu);
            const float q1 = static_cast<float>(code[2 * r + 1] & 0xFFu);
            c[2 * r] = __fadd_rn(__fmul_rn(__uint_as_float(pr.x), q0), __uint_as_float(pr.y));
            c[2 * r + 1] =
                __fadd_rn(__fmul_rn(__uint_as_float(next ? pr.z : pr.x), q1), __uint_as_float(next ? pr.w : pr.y));
        }
        return blend(t, c[0], c[1], c[2], c[3], c[4], c[5], c[6], c[7]);
    } else if constexpr (S == kF16) {
        float c[8];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const uint32_t w = __builtin_amdgcn_raw_buffer_load_b32(src.rsrc, static_cast<int>(o[r]), 0, 0);
            c[2 * r] = __half2float(__ushort_as_half(static_cast<unsigned short>(w & 0xFFFFu)));
            c[2 * r + 1] = __half2float(__ushort_as_half(static_cast<unsigned short>(w >> 16)));
        }
        return blend(t, c[0], c[1], c[2], c[3], c[4], c[5], c[6], c[7]);
    } else {
        return blend(t, corner<S>(src, o[0]), corner<S>(src, o[1]), corner<S>(src, o[2]), corner<S>(src, o[3]),
                     corner<S>(src, o[4]), corner<S>(src, o[5]), corner<S>(src, o[6]), corner<S>(src, o[7]));
    }
}

// Trilinear value from neighbourhood records: 4-byte entries in 9 x 8 x 8 brick blocks (the block_index9
// numbering, x = 8 a copy of the next brick's first voxel), so that the 8 bytes at the base voxel's
// entry are the cell's two x-neighbouring entries.  binary16: entry (x, y, z) holds the values at
// (x, y) and (x, y + 1), and those 8 bytes are the cell's 2x2 (x, y) corners in the plane: one load for
// z0 and one for z1.  float32 (and decoded 8-bit values): entry (x, y, z) holds the value at (x, y),
// and the 8 bytes are an x pair: loads for the rows (y0, z0), (y1, z0), (y0, z1), (y1, z1).  r00 / r10 /
// r01 / r11 are the entry numbers of the base voxel's row at (y0, z0), (y1, z0), (y0, z1), (y1, z1).  The arithmetic is that of fetch(), so both layouts give identical
// values.  WIDE: global loads at 64-bit byte offsets (fields of 4 GiB and more); else buffer loads at
// 32-bit byte offsets, whose base the load adds itself (`bytes`: the field's size).
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
template <int S>
constexpr uint32_t kRecShift = 2;  // log2 of the bytes per entry
template <int S, bool WIDE>
__device__ __forceinline__ u32x2 load_record(const void* base, uint32_t bytes, uint32_t r) {
    if constexpr (WIDE) {
        return global_ptr<u32x2>(static_cast<const char*>(base) + (static_cast<size_t>(r) << kRecShift<S>))[0];
    } else {
        const __amdgpu_buffer_rsrc_t rsrc =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, static_cast<int>(bytes), kRawBufferFlags);
        return __builtin_amdgcn_raw_buffer_load_b64(rsrc, static_cast<int>(r << kRecShift<S>), 0, 0);
    }
}
template <int S, bool WIDE>
__device__ __forceinline__ float fetch_rec(const void* __restrict__ base, uint32_t bytes, uint32_t r00, uint32_t r10,
                                           uint32_t r01, uint32_t r11, const Tri& t) {
    if constexpr (S == kF16) {
        // entries (x0, y) and (x1, y): the halves are (x0, y0), (x0, y1), (x1, y0), (x1, y1)
        const u32x2 p = load_record<S, WIDE>(base, bytes, r00);
        const u32x2 q = load_record<S, WIDE>(base, bytes, r01);
        auto lo = [](unsigned int u) { return __half2float(__ushort_as_half(static_cast<unsigned short>(u & 0xFFFFu))); };
        auto hi = [](unsigned int u) { return __half2float(__ushort_as_half(static_cast<unsigned short>(u >> 16))); };
        return blend(t, lo(p.x), lo(p.y), hi(p.x), hi(p.y), lo(q.x), lo(q.y), hi(q.x), hi(q.y));
    } else {
        const u32x2 p0 = load_record<S, WIDE>(base, bytes, r00);
        const u32x2 p1 = load_record<S, WIDE>(base, bytes, r10);
        const u32x2 p2 = load_record<S, WIDE>(base, bytes, r01);
        const u32x2 p3 = load_record<S, WIDE>(base, bytes, r11);
        return blend(t, __uint_as_float(p0.x), __uint_as_float(p0.y), __uint_as_float(p1.x), __uint_as_float(p1.y),
                     __uint_as_float(p2.x), __uint_as_float(p2.y), __uint_as_float(p3.x), __uint_as_float(p3.y));
    }
}

// fetch_rec for a lane that may not need the value (the value is then meaningless).  At 32-bit offsets
// the loads of a lane whose `use` is clear go to an offset beyond the field, which reads no memory and
// returns zero: issued this way the loads need no branch, so those of several samples are in flight
// together.  kNoLoad lies beyond every field and flag array (record fields of the 32-bit offset kinds
// stay below 0xFF4E0000 bytes).  At 64-bit offsets (global loads) the loads are predicated.
constexpr uint32_t kNoLoad = 0xFFFFFFF0u;
template <int S, bool WIDE>
__device__ __forceinline__ float fetch_rec_guarded(const void* __restrict__ base, uint32_t bytes, bool use, uint32_t r00,
                                                   uint32_t r10, uint32_t r01, uint32_t r11, const Tri& t) {
    auto ld = [&](uint32_t r) -> u32x2 {
        if constexpr (WIDE) {
            u32x2 v = {0u, 0u};
            if (use) v = global_ptr<u32x2>(static_cast<const char*>(base) + (static_cast<size_t>(r) << kRecShift<S>))[0];
            return v;
        } else {
            const __amdgpu_buffer_rsrc_t rsrc =
                __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, static_cast<int>(bytes), kRawBufferFlags);
            return __builtin_amdgcn_raw_buffer_load_b64(rsrc, static_cast<int>(use ? r << kRecShift<S> : kNoLoad), 0, 0);
        }
    };
    if constexpr (S == kF16) {
        const u32x2 p = ld(r00);
        const u32x2 q = ld(r01);
        auto lo = [](unsigned int u) { return __half2float(__ushort_as_half(static_cast<unsigned short>(u & 0xFFFFu))); };
        auto hi = [](unsigned int u) { return __half2float(__ushort_as_half(static_cast<unsigned short>(u >> 16))); };
        return blend(t, lo(p.x), lo(p.y), hi(p.x), hi(p.y), lo(q.x), lo(q.y), hi(q.x), hi(q.y));
    } else {
        const u32x2 p0 = ld(r00);
        const u32x2 p1 = ld(r10);
        const u32x2 p2 = ld(r01);
        const u32x2 p3 = ld(r11);
        return blend(t, __uint_as_float(p0.x), __uint_as_float(p0.y), __uint_as_float(p1.x), __uint_as_float(p1.y),
                     __uint_as_float(p2.x), __uint_as_float(p2.y), __uint_as_float(p3.x), __uint_as_float(p3.y));
    }
}

// Kernel kinds: storage type and layout.
constexpr int storage_of(int K) {
    return K == kKindF32Rec ? kF32 : (K == kKindF16Rec ? kF16 : (K == kKindU8Rec ? kU8 : K));
}
constexpr bool records_of(int K) { return K >= kKindF32Rec; }
// Value type held by a kind's records: binary16 pairs in y, or float32 values (also for decoded 8-bit codes).
constexpr int record_type_of(int K) { return K == kKindF16Rec ? kF16 : kF32; }

// Ray parameter where u(t) = uo + du t leaves the box [c, c + e) along one axis (voxel units, forward
// only): the crossing of the face the ray moves towards, moved kSkipShrink into the box against
// rounding, or +inf when that face is a face of the grid (clamping maps every position beyond it into
// the boundary box).  Per ray: up = -1 when the component's sign bit is clear (moving up; +0 too), else
// 0; uos = uo + kSkipShrink when moving up, uo - kSkipShrink when moving down; inv_du = 1 / du.  For
// du = 0 the result is +inf or a conservative (earlier) exit.  Written without a per-ray select, so
// no per-lane condition stays live across the march.
__device__ __forceinline__ float box_exit(int c, int e, int up, float uos, float inv_du, int n) {
    const int face = c + (e & up);
    const float t = (static_cast<float>(face) - uos) * inv_du;
    return static_cast<uint32_t>(face - 1) >= static_cast<uint32_t>(n - 1) ? INFINITY : t;
}

// Stable ray/sphere hit for |d| = 1.  Returns false when the ray misses or touches.
__device__ __forceinline__ bool sphere_hit(float b, float px, float py, float pz, float r2, float c, float& t0,
                                           float& t1) {
    const float disc = r2 - (px * px + py * py + pz * pz);
    if (!(disc > 0.0f)) return false;
    const float q = -b - copysignf(sqrtf(disc), b);
    const float ta = c / q, tb = q;
    t0 = fminf(ta, tb);
    t1 = fmaxf(ta, tb);
    return true;
}

// Value of `v` held by lane SRC (0..3) of the calling lane's quad (one DPP quad_perm move).
template <int SRC>
__device__ __forceinline__ float quad_bcast(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), SRC * 0x55, 0xF, 0xF, true));
}
template <int SRC>
__device__ __forceinline__ int quad_bcast(int v) {
    return __builtin_amdgcn_mov_dpp(v, SRC * 0x55, 0xF, 0xF, true);
}

// Tiles are grouped in super-tiles and super-tiles are dealt round-robin over the 8 XCDs (block i runs
// on XCD i % 8).  The tiles of a super-tile run together on one XCD (their rays share voxels in its
// L2), and every XCD gets super-tiles from all over the image, so the work of the shell's disc is
// spread evenly; 32 x 32 pixels balances the two (larger super-tiles leave some XCDs with more of the
// disc's costly centre, smaller ones share less).  Super-tiles go in row-major order: dealing the
// costly middle first (centre-out) was 5 % slower, as consecutive super-tiles of an XCD no longer
// shared voxels.  Batched launches use super-tiles of kSuper x kSuper 4 x 4 pixel tiles.
constexpr int kSuper = 8;
constexpr int kSuperTiles = kSuper * kSuper;

// Batched launches number a request's tiles super-tile by super-tile in row-major order, tiles
// row-major inside each (narrower at the right and bottom edges), so consecutive tile indices
// cover a compact patch of the image.  A bijection of [0, bx_count * by_count).
__device__ __forceinline__ void tile_coords(int i, int bx_count, int by_count, int& bx, int& by) {
    const int sr = i / (bx_count * kSuper);
    const int rem = i - sr * bx_count * kSuper;
    const int rows = min(kSuper, by_count - sr * kSuper);
    const int full_cols = bx_count / kSuper;
    const int sc = rem / (kSuper * rows);
    if (sc < full_cols) {
        const int r2 = rem - sc * kSuper * rows;
        bx = sc * kSuper + r2 % kSuper;
        by = sr * kSuper + r2 / kSuper;
    } else {
        const int wl = bx_count - full_cols * kSuper;
        const int r3 = rem - full_cols * kSuper * rows;
        bx = full_cols * kSuper + r3 % wl;
        by = sr * kSuper + r3 / wl;
    }
}

// Single-image launches deal super-tiles of 2^s x 2^s blocks (2^(A.super_log2 + 1) wave tiles on a
// side for the launch-shape parameter A.super_log2, see launch_tiles: 8 << A.super_log2 pixels square
// with 4 x 4 tiles; the serving path keeps 32 pixels): the j-th
// block an XCD receives is tile j % 4^s of super-tile (j / 4^s) * 8 + xcd (super-tiles row-major over
// the image).  The grid is padded to whole rounds of 8 super-tiles; blocks outside the image return
// at once.
__host__ __device__ inline int super_cols(int blocks_x, int s) { return (blocks_x + (1 << s) - 1) >> s; }
__host__ __device__ inline int padded_blocks(int blocks_x, int blocks_y, int s) {
    const int supers = super_cols(blocks_x, s) * ((blocks_y + (1 << s) - 1) >> s);
    return (supers + 7) / 8 * 8 << (2 * s);
}
__device__ __forceinline__ void interleaved_tile(int bid, int blocks_x, int s, int& bx, int& by) {
    const int xcd = bid & 7, p = bid >> 3;
    const int st = (p >> (2 * s)) * 8 + xcd;
    const int w = p & ((1 << (2 * s)) - 1);
    const int sc = super_cols(blocks_x, s);
    bx = ((st % sc) << s) + (w & ((1 << s) - 1));
    by = ((st / sc) << s) + (w >> s);
}

// Waves per block of the single-image kernels: record fields of 4 GiB and more (the WIDE record kinds,
// level 0 of a 1024^3 grid) keep four waves on 8 x 8 pixels, whose rays share a CU's L1 (faster on such
// volumes); every other kernel runs one wave on 4 x 4 pixels, whose CU slot frees as soon as its 16
// rays end (a block of several waves holds its slot until the slowest of them ends).
constexpr int block_waves(int K, bool WIDE) { return records_of(K) && WIDE ? 4 : 1; }

// The 256-entry transfer-function table into LDS by a block of BW waves.
template <int BW>
__device__ __forceinline__ void load_tf(const float4* tf, float4* s_tf) {
#pragma unroll
    for (int i = 0; i < 4 / BW; ++i) {
        const f32x4 e = global_ptr<f32x4>(tf)[threadIdx.x + 64 * BW * i];
        s_tf[threadIdx.x + 64 * BW * i] = make_float4(e.x, e.y, e.z, e.w);
    }
    __syncthreads();
}

// Number of brushed fields known only at run time, tested per field in the loop (coordinate axes take
// this variant, which carries their test).
constexpr int kRuntimeNB = -1;

// Sample-grid offset s in [0, 1) of pixel p in a jittered pass: output number c + 1 of a SplitMix64
// stream started at the seed (Steele, Lea and Flood, OOPSLA 2014: gamma 0x9E3779B97F4A7C15 and the
// 30 / 27 / 31 xor-shift, multiply mix), for the counter c = pass 2^32 + p; its top 16 bits give
// xi, and s = min(fl32(fl32(pass + xi) / n_passes), 1 - 2^-24) (stratified per pass).
__device__ __forceinline__ float jitter_offset(const RenderArgs& A, uint32_t p) {
    const uint64_t c = (static_cast<uint64_t>(A.pass) << 32) | p;
    uint64_t z = A.seed + (c + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    const float xi = static_cast<float>(static_cast<uint32_t>(z >> 48)) * 0x1p-16f;
    const float s = __fdiv_rn(__fadd_rn(static_cast<float>(A.pass), xi), static_cast<float>(A.n_passes));
    return fminf(s, 0x1.fffffep-1f);
}

// Samples a lane evaluates per step.  binary16 records take two, j0 + sub and j0 + 4 + sub: the
// loads of both samples are issued together (see fetch_rec_guarded), so a wave has twice the loads
// in flight while each ray advances eight samples per step (headline frame 0.876 -> 0.740 ms; the
// 1024^3 4K passes at 64-bit offsets 17-21 % faster).  The other kinds take one: with two, float32-pair
// records (float32 and decoded 8-bit values) need 80 registers, which leaves 6 waves per SIMD (two
// frames in flight 0.840 -> 0.878 ms per step); the compact binary16 layout 87 (7 % slower) and the 8-bit code
// blocks 116, 4 waves per SIMD (1.55 -> 1.70 ms).  The counting variant takes one.
constexpr int samples_per_lane(int K, bool COUNTS) { return !COUNTS && K == kKindF16Rec ? 2 : 1; }

// One 4 x 4 pixel tile (bx, by) of the image described by A, marched by the calling one-wave block.  NB is the number of brushed fields, or kRuntimeNB to read it from A.
// JIT: a jittered progressive pass (the sample grid of every segment starts s ds before it, so the
// first and last samples of a segment are partial).  DEPTH: also write the opacity-weighted depth, the
// mean distance of the composited samples, each weighted by its share w of the pixel's opacity (the
// depth that image warping reprojects with; +inf where nothing was composited).  WIDE: 64-bit record
// offsets (needed for record fields of 4 GiB and more).  L points to the same arguments as A; the
// pixel's outputs are written through it (see late_args).
//
// A step of the march takes, for each ray, the next P groups of four consecutive samples (P =
// samples_per_lane): lane `sub` of the ray's quad evaluates samples j0 + 4 q + sub, q < P.  The
// groups are composited in sample order; a skipped box of the last group's fourth sample moves the
// next step past that box.  A sample of group q > 0 that lies inside a box the previous group's
// fourth sample would have jumped over is itself in that skipped box, so it is skipped and adds
// nothing, and the image does not depend on P.
template <int K, int NB, bool COUNTS, bool JIT = false, bool DEPTH = false, bool WIDE = true, int BW = 1,
          typename LP>
__device__ __forceinline__ void march_tile(const RenderArgs& A, LP L, int bx, int by, float4* s_tf) {
    constexpr int S = storage_of(K);
    constexpr bool R = records_of(K);
    constexpr int RT = record_type_of(K);
    constexpr int P = samples_per_lane(K, COUNTS);
    static_assert(P == 1 || !COUNTS, "the counting variant takes one sample per lane");
    // the wave tile: tw x th pixels, tw = 2^t (A.tile_log2w), th = 16 / tw; a block of four waves
    // takes 2 x 2 wave tiles
    const int tl = A.tile_log2w, tw = 1 << tl, th = kWaveRays >> tl;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int ray = lane >> 2, sub = lane & 3, quad_base = lane & ~3;
    const int px = (BW == 4 ? 2 * bx + (wave & 1) : bx) * tw + (ray & (tw - 1));
    const int py = (BW == 4 ? 2 * by + (wave >> 1) : by) * th + (ray >> tl);
    const bool inside = px < A.width && py < A.height;

    // ---- ray through the pixel centre (identical in the four lanes of the quad)
    const float sx = fmaf(static_cast<float>(px) + 0.5f, A.inv_w2, -1.0f) * A.sx_scale;
    const float sy = fmaf(-(static_cast<float>(py) + 0.5f), A.inv_h2, 1.0f) * A.sy_scale;
    float dx = fmaf(sy, A.upv[0], fmaf(sx, A.right[0], A.fwd[0]));
    float dy = fmaf(sy, A.upv[1], fmaf(sx, A.right[1], A.fwd[1]));
    float dz = fmaf(sy, A.upv[2], fmaf(sx, A.right[2], A.fwd[2]));
    const float inv_len = 1.0f / sqrtf(fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
    dx *= inv_len;
    dy *= inv_len;
    dz *= inv_len;
    const float ox = A.eye[0], oy = A.eye[1], oz = A.eye[2];

    // ---- shell segments
    const float b = fmaf(ox, dx, fmaf(oy, dy, oz * dz));
    const float fx = fmaf(-b, dx, ox), fy = fmaf(-b, dy, oy), fz = fmaf(-b, dz, oz);
    // the non-empty segments in ray order, (sa0, sb0) then (sa1, sb1) (scalars: an array indexed by
    // the segment count would live in scratch memory)
    float sa0 = 0.0f, sb0 = 0.0f, sa1 = 0.0f, sb1 = 0.0f;
    int nseg = 0;
    float t0, t1;
    if (inside && sphere_hit(b, fx, fy, fz, A.r_out2, A.c_out, t0, t1)) {
        float s0, s1;
        const bool inner = A.has_inner && sphere_hit(b, fx, fy, fz, A.r_in2, A.c_in, s0, s1);
        float ca0 = t0, cb0 = t1, ca1 = 0.0f, cb1 = 0.0f;
        if (inner) {
            cb0 = fminf(t1, s0);
            ca1 = fmaxf(t0, s1);
            cb1 = t1;
        }
        ca0 = fmaxf(ca0, 0.0f);
        ca1 = fmaxf(ca1, 0.0f);
        const bool near = cb0 > ca0, far = inner && cb1 > ca1;
        nseg = static_cast<int>(near) + static_cast<int>(far);
        sa0 = near ? ca0 : ca1;
        sb0 = near ? cb0 : cb1;
        sa1 = ca1;
        sb1 = cb1;
    }

    // the transfer-function table into LDS; a one-wave block loads it only if one of its rays passes
    // through the shell (most waves of a frame see background alone)
    if (BW > 1 || __ballot(nseg > 0) != 0ull) load_tf<BW>(A.tf, s_tf);

    const int n = A.n, nb = A.nb;
    const uint32_t nbu = static_cast<uint32_t>(nb);
    // the flag words as a buffer (no flags: an empty range, so every load returns zero)
    const __amdgpu_buffer_rsrc_t flag_rsrc = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<void*>(A.skip != nullptr ? static_cast<const void*>(A.skip) : static_cast<const void*>(A.tf)), 0,
        A.skip != nullptr ? static_cast<int>(nbu * nbu * nbu * 2u) : 0, kRawBufferFlags);
    // block entry steps (records and binary16 values) from a row at local y = 7 (z = 7) to the row at
    // local 0 of the next brick
    const uint32_t block_y_step = nbu * kBlockValues - 7u * kBlockYStride;
    const uint32_t block_z_step = nbu * nbu * kBlockValues - 7u * kBlockZStride;
    const float top = static_cast<float>(n - 1);  // largest voxel index
    const float hn = A.half_n;
    const float uox = fmaf(ox, hn, hn - 0.5f), uoy = fmaf(oy, hn, hn - 0.5f), uoz = fmaf(oz, hn, hn - 0.5f);
    const float dux = dx * hn, duy = dy * hn, duz = dz * hn;
    const float inv_dux = 1.0f / dux, inv_duy = 1.0f / duy, inv_duz = 1.0f / duz;
    // skipped-box exits (box_exit): direction of each axis as a bit mask, origin moved by the shrink
    const int upx = static_cast<int>(__float_as_uint(dux) >> 31) - 1;
    const int upy = static_cast<int>(__float_as_uint(duy) >> 31) - 1;
    const int upz = static_cast<int>(__float_as_uint(duz) >> 31) - 1;
    const float uosx = uox - copysignf(kSkipShrink, -dux), uosy = uoy - copysignf(kSkipShrink, -duy);
    const float uosz = uoz - copysignf(kSkipShrink, -duz);
    const float ds = A.ds, inv_ds = A.inv_ds;
    const float r_full = ds * A.inv_ref;

    float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
    float D = 0.0f;  // DEPTH: sum of w tm over the composited samples
    uint32_t cnt_nom = 0, cnt_comp = 0;
    uint32_t cnt_eval = 0, cnt_fetch = 0;  // COUNTS: this lane's evaluated samples and field fetches
    uint32_t last_brick = 0xFFFFFFFFu;
    int seg = 0, j0 = 0;  // j0: first sample of the quad's current step
    float sa = sa0, sb = sb0;
    // grid origin of the current segment: sample j covers [max(sa, g + j ds), min(g + (j+1) ds, sb)]
    float s_jit = 0.0f;
    if constexpr (JIT) s_jit = jitter_offset(A, static_cast<uint32_t>(py) * A.width + px);
    float g = JIT ? fmaf(-s_jit, ds, sa) : sa;
    int ns = nseg > 0 ? max(static_cast<int>(ceilf((sb - g) / ds)), 1) : 0;
    bool alive = nseg > 0;
    // The segment's partial samples, computed once per segment: the last (and, in a jittered pass, the
    // first) sample covers only part of its step; it is taken at the midpoint of what it covers and its
    // opacity corrected to that length (r = length / ref_step).  Every other sample j sits at
    // g + (j + 1/2) ds with r = ds / ref_step.
    float tm_first = 0.0f, r_first = 0.0f, tm_last = 0.0f, r_last = 0.0f;
    auto partial_samples = [&]() {
        if constexpr (JIT) {
            const float thi0 = ns == 1 ? sb : fmaf(1.0f, ds, g);
            tm_first = 0.5f * (sa + thi0);
            r_first = fmaxf(thi0 - sa, 0.0f) * A.inv_ref;
        }
        const float tlo = fmaf(static_cast<float>(ns - 1), ds, g);
        tm_last = 0.5f * (tlo + sb);
        r_last = fmaxf(sb - tlo, 0.0f) * A.inv_ref;
    };
    partial_samples();

    while (alive) {
        // ---- sample positions and their bricks' flag words (the loads of all P samples together)
        bool valid[P], skipped[P], pass[P];
        float tv[P], tm[P], rs[P], ux[P], uy[P], uz[P], flx[P], fly[P], flz[P];
        int x0[P], y0[P], z0[P];
        uint32_t brick[P], sbi[P], flags[P];
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const int j = j0 + kQuad * q + sub;
            valid[q] = j < ns;
            const bool last = j == ns - 1;
            skipped[q] = false;
            pass[q] = false;
            tv[q] = 0.0f;
            tm[q] = last ? tm_last : fmaf(static_cast<float>(j) + 0.5f, ds, g);
            rs[q] = last ? r_last : r_full;
            if constexpr (JIT) {
                if (j == 0) {
                    tm[q] = tm_first;
                    rs[q] = r_first;
                }
            }
            // a position below the grid (u < 0 on an axis, where both corners clamp to index 0) is taken
            // on its lower face, u = 0: the upper corner's weight is then zero, which gives the clamped
            // value exactly (and lets a record of the base voxel serve)
            ux[q] = fmaxf(fmaf(dux, tm[q], uox), 0.0f), uy[q] = fmaxf(fmaf(duy, tm[q], uoy), 0.0f);
            uz[q] = fmaxf(fmaf(duz, tm[q], uoz), 0.0f);
            flx[q] = floorf(ux[q]), fly[q] = floorf(uy[q]), flz[q] = floorf(uz[q]);
            // corner indices clamped onto the grid (the clamp taken on the integer-valued floors)
            x0[q] = static_cast<int>(__builtin_amdgcn_fmed3f(flx[q], 0.0f, top));
            y0[q] = static_cast<int>(__builtin_amdgcn_fmed3f(fly[q], 0.0f, top));
            z0[q] = static_cast<int>(__builtin_amdgcn_fmed3f(flz[q], 0.0f, top));
            const int bxi = x0[q] >> 3, byi = y0[q] >> 3, bzi = z0[q] >> 3;
            // brick rows and slabs below 2^7, bricks per row below 2^8: 24-bit products are exact
            brick[q] = raypc_mul_u24(raypc_mul_u24(static_cast<uint32_t>(bzi), nbu) + byi, nbu) + bxi;
            sbi[q] = ((x0[q] >> 2) & 1) | (((y0[q] >> 2) & 1) << 1) | (((z0[q] >> 2) & 1) << 2);  // sub-brick
            flags[q] = __builtin_amdgcn_raw_buffer_load_b16(flag_rsrc, static_cast<int>(valid[q] ? brick[q] * 2u : kNoLoad),
                                                            0, 0);
        }
        bool any_fetch = false;
#pragma unroll
        for (int q = 0; q < P; ++q) {
            skipped[q] = valid[q] && ((flags[q] >> sbi[q]) & 1u);
            any_fetch = any_fetch || (valid[q] && !skipped[q]);
        }
        // ---- every sample whose base corner lies in a flagged sub-brick (in this brick, or its empty
        // brick group, when flagged so) is discarded or transparent.  The quad's fourth lane finds, for
        // its last sample, the first sample that may lie beyond the box (shrunk by a margin against
        // rounding; open at the grid's faces, where clamping maps every outside position to the
        // boundary box): the next step starts there.
        int jn = 0;
        if (skipped[P - 1] && sub == kQuad - 1) {
            constexpr int q = P - 1;
            const int j = j0 + kQuad * q + sub;
            const uint32_t fl = flags[q];
            // the largest empty box holding the sample's base corner: its aligned 4^3- or 2^3-brick
            // group, the brick, or the sub-brick (corner x0 & m, edge -m voxels)
            const int m = (fl & 0x200u) ? -32 : ((fl & 0x100u) ? -16 : ((fl & 0xFFu) == 0xFFu ? -8 : -4));
            const float t_exit = fminf(box_exit(x0[q] & m, -m, upx, uosx, inv_dux, n),
                                       fminf(box_exit(y0[q] & m, -m, upy, uosy, inv_duy, n),
                                             box_exit(z0[q] & m, -m, upz, uosz, inv_duz, n)));
            float jc = (t_exit - g) * inv_ds - 0.5f - kSkipMargin;
            jc = fminf(fmaxf(jc, 0.0f), static_cast<float>(ns));
            jn = max(j + 1, static_cast<int>(ceilf(jc)));
        }
        uint32_t it_eval = 0, it_fetch = 0;  // COUNTS: this step's sample evaluated, fields fetched
        if (any_fetch) {
            Tri tri[P];
            uint32_t o[P][8];
            uint32_t r00[P], r10[P], r01[P], r11[P];
#pragma unroll
            for (int q = 0; q < P; ++q) {
                if constexpr (COUNTS) {
                    if (A.touched != nullptr && valid[q] && !skipped[q] && brick[q] != last_brick) {
                        atomicOr(&A.touched[brick[q] >> 5], 1u << (brick[q] & 31));
                        last_brick = brick[q];
                    }
                }
                const float wx = ux[q] - flx[q], wy = uy[q] - fly[q], wz = uz[q] - flz[q];
                tri[q] = tri_weights(wx, wy, wz);
                r00[q] = r10[q] = r01[q] = r11[q] = 0;
                if constexpr (R) {
                    // entry number of the base voxel in the record blocks (the block_index9 numbering): its
                    // brick's block, then z, y, x.  The row one up in y (z) is 9 (72) entries on inside a
                    // brick, in the next brick beyond its face, and the same row where the upper corner
                    // clamps onto the base voxel (at the grid's upper face).  binary16 entries hold y and
                    // y + 1, so they need no row in y.
                    r00[q] = raypc_mul_u24(brick[q], kBlockValues) + static_cast<uint32_t>(z0[q] & 7) * kBlockZStride +
                             static_cast<uint32_t>(y0[q] & 7) * kBlockYStride + static_cast<uint32_t>(x0[q] & 7);
                    const uint32_t dz = (z0[q] & 7) != 7 ? kBlockZStride : block_z_step;
                    r01[q] = r00[q] + (flz[q] < top ? dz : 0u);
                    if constexpr (RT == kF32) {
                        const uint32_t dy = (y0[q] & 7) != 7 ? kBlockYStride : block_y_step;
                        const uint32_t dyv = fly[q] < top ? dy : 0u;
                        r10[q] = r00[q] + dyv;
                        r11[q] = r01[q] + dyv;
                    }
                } else if constexpr (S == kF16) {
                    // the slots of fetch() for binary16 values: byte offsets of the four rows at x0.  The
                    // row one up in y (z) is 9 (72) values on inside a brick, in the next brick beyond
                    // its face, and the same row where the upper corner clamps onto the grid's face.
                    const int iy = static_cast<int>(fly[q]), iz = static_cast<int>(flz[q]);
                    const int y1 = min(iy + 1, n - 1), z1 = min(iz + 1, n - 1);
                    const uint32_t dyv = y1 == y0[q] ? 0u : ((y0[q] & 7) != 7 ? kBlockYStride : block_y_step);
                    const uint32_t dzv = z1 == z0[q] ? 0u : ((z0[q] & 7) != 7 ? kBlockZStride : block_z_step);
                    const uint32_t base = raypc_mul_u24(brick[q], kBlockValues) +
                                          static_cast<uint32_t>(z0[q] & 7) * kBlockZStride +
                                          static_cast<uint32_t>(y0[q] & 7) * kBlockYStride + static_cast<uint32_t>(x0[q] & 7);
                    o[q][0] = base * 2u;
                    o[q][1] = (base + dyv) * 2u;
                    o[q][2] = (base + dzv) * 2u;
                    o[q][3] = (base + dyv + dzv) * 2u;
                    o[q][4] = o[q][5] = o[q][6] = o[q][7] = 0;
                } else if constexpr (S == kU8) {
                    // the slots of fetch() for 8-bit codes
                    const int ix = static_cast<int>(flx[q]), iy = static_cast<int>(fly[q]), iz = static_cast<int>(flz[q]);
                    const int x1 = min(ix + 1, n - 1), y1 = min(iy + 1, n - 1), z1 = min(iz + 1, n - 1);
                    const uint32_t dyb = (y1 >> 3) != (y0[q] >> 3) ? nbu : 0u;
                    const uint32_t dzb = (z1 >> 3) != (z0[q] >> 3) ? nbu * nbu : 0u;
                    const uint32_t in_xy = static_cast<uint32_t>(y0[q] & 7) * 9u + static_cast<uint32_t>(x0[q] & 7);
                    o[q][0] = raypc_mul_u24(brick[q], kU8BrickBytes) + static_cast<uint32_t>(z0[q] & 7) * 81u + in_xy;
                    o[q][1] = raypc_mul_u24(brick[q] + dzb, kU8BrickBytes) + static_cast<uint32_t>(z1 & 7) * 81u + in_xy;
                    o[q][2] = brick[q];
                    o[q][3] = brick[q] + dyb;
                    o[q][4] = brick[q] + dzb;
                    o[q][5] = brick[q] + dyb + dzb;
                    o[q][6] = (x1 >> 3) != (x0[q] >> 3) ? 1u : 0u;
                    o[q][7] = 0;
                } else {
                    constexpr int LB = kLogBytes<S>;
                    const int ix = static_cast<int>(flx[q]), iy = static_cast<int>(fly[q]), iz = static_cast<int>(flz[q]);
                    const int x1 = min(ix + 1, n - 1), y1 = min(iy + 1, n - 1), z1 = min(iz + 1, n - 1);
                    const uint32_t X0 = axis_x(x0[q]) << LB, X1 = axis_x(x1) << LB;
                    const uint32_t Y0 = axis_y(y0[q], nb) << LB, Y1 = axis_y(y1, nb) << LB;
                    const uint32_t Z0 = axis_z(z0[q], nb) << LB, Z1 = axis_z(z1, nb) << LB;
                    const uint32_t zy00 = Z0 + Y0, zy01 = Z0 + Y1, zy10 = Z1 + Y0, zy11 = Z1 + Y1;
                    o[q][0] = zy00 + X0, o[q][1] = zy00 + X1, o[q][2] = zy01 + X0, o[q][3] = zy01 + X1;
                    o[q][4] = zy10 + X0, o[q][5] = zy10 + X1, o[q][6] = zy11 + X0, o[q][7] = zy11 + X1;
                }
                // coordinate axes first: a sample outside them fetches no field (the kernels with a
                // fixed field count carry no coordinate axes; renders that use them take the
                // run-time variant)
                pass[q] = valid[q] && !skipped[q];
                if constexpr (NB < 0) {
                    if (A.coord_mask)
                        pass[q] = pass[q] && coord_ok(A.coord_mask, A.clo, A.chi, fmaf(dx, tm[q], ox),
                                                      fmaf(dy, tm[q], oy), fmaf(dz, tm[q], oz));
                }
            }
            if constexpr (COUNTS) it_eval = valid[0] && !skipped[0] ? 1u : 0u;
            // field k's value at every sample of the lane that still passes (with two samples per
            // lane, both loads are issued, a sample that no longer passes loading nothing)
            auto field_values = [&](int k, float (&v)[P]) {
#pragma unroll
                for (int q = 0; q < P; ++q) {
                    if constexpr (R) {
                        if constexpr (P > 1)
                            v[q] = fetch_rec_guarded<RT, WIDE>(A.rec[k], A.rec_bytes, pass[q], r00[q], r10[q], r01[q],
                                                               r11[q], tri[q]);
                        else
                            v[q] = fetch_rec<RT, WIDE>(A.rec[k], A.rec_bytes, r00[q], r10[q], r01[q], r11[q], tri[q]);
                    } else {
                        v[q] = fetch<S>(source<S>(A, k), o[q], tri[q]);
                    }
                }
            };
            auto any_pass = [&]() {
                bool a = false;
#pragma unroll
                for (int q = 0; q < P; ++q) a = a || pass[q];
                return a;
            };
            constexpr int kUnroll = NB >= 0 ? NB : kMaxFields;
            const int nbr = NB >= 0 ? NB : A.n_brushed;
            // The slot comparisons below are made afresh in every step: hoisted out of the loop,
            // each would hold a 64-bit lane mask for the whole march.
            int tfs = A.tf_slot;
            asm volatile("" : "+s"(tfs));
#pragma unroll
            for (int k = 0; k < kUnroll; ++k) {
                if ((NB >= 0 || k < nbr) && any_pass()) {
                    float v[P];
                    field_values(k, v);
                    if constexpr (COUNTS) ++it_fetch;
#pragma unroll
                    for (int q = 0; q < P; ++q) {
                        pass[q] = pass[q] && (v[q] >= A.lo[k]) && (v[q] <= A.hi[k]);
                        if (k == tfs) tv[q] = v[q];
                    }
                }
            }
            if (any_pass()) {
                int tk = -1;
                if constexpr (NB >= 0 && NB < kMaxFields) {
                    if (tfs == NB) tk = NB;
                } else if constexpr (NB < 0) {
                    if (tfs == nbr && nbr < kMaxFields) tk = nbr;
                }
                if (tk >= 0) {
                    float v[P];
                    field_values(tk, v);
                    if constexpr (COUNTS) ++it_fetch;
#pragma unroll
                    for (int q = 0; q < P; ++q) tv[q] = v[q];
                }
            }
        }
        // ---- advance past a skipped box of the quad's last sample
        const int last_skipped = quad_bcast<3>(static_cast<int>(skipped[P - 1]));
        const int jn3 = quad_bcast<3>(jn);
        bool stopped = false;
        int stop_at = kQuad - 1;  // COUNTS: the quad's last sample that counts
#pragma unroll
        for (int q = 0; q < P; ++q) {
            // nothing to classify or composite when no sample of the group passed the brush
            if (__ballot(pass[q] && !stopped) == 0ull) continue;
            const float xt = fminf(fmaxf((tv[q] - A.vmin) * A.inv_range, 0.0f), 1.0f) * 255.0f;
            const int it = min(static_cast<int>(xt), 254);
            const float wt = xt - static_cast<float>(it);
            const float4 e0 = s_tf[it], e1 = s_tf[it + 1];
            const float al = fmaf(wt, e1.w - e0.w, e0.w);
            const bool contributes = pass[q] && al > 0.0f;
            const float kcq = al >= 1.0f ? 0.0f : __builtin_amdgcn_exp2f(rs[q] * __log2f(1.0f - al));
            // a ray that stopped in an earlier group composites nothing more
            const bool con = contributes && !stopped;
            if (__ballot(con) == 0ull) continue;  // else nothing to composite anywhere in the wave
            const float crq = fmaf(wt, e1.x - e0.x, e0.x);
            const float cgq = fmaf(wt, e1.y - e0.y, e0.y);
            const float cbq = fmaf(wt, e1.z - e0.z, e0.z);
            const float keep = con ? kcq : 1.0f;
            const float qr = con ? crq : 0.0f, qg = con ? cgq : 0.0f, qb = con ? cbq : 0.0f;
            // ---- merge the quad's four samples in sample order.  Every lane replays the same
            // sequential updates (T <- T k, then C <- C + w rgb) on broadcast values, so the ray
            // state is identical in the four lanes and independent of how samples were grouped
            // (a skipped or discarded sample has k = 1 and w = 0, both exact).
            const float k0 = quad_bcast<0>(keep), k1 = quad_bcast<1>(keep);
            const float k2 = quad_bcast<2>(keep), k3 = quad_bcast<3>(keep);
            const float t1 = T * k0, t2 = t1 * k1, t3 = t2 * k2, t4 = t3 * k3;  // T after each sample
            const float t_before = sub == 0 ? T : (sub == 1 ? t1 : (sub == 2 ? t2 : t3));
            const float w = t_before * (1.0f - keep);
            const float tmq = tm[q];
            // each lane forms its own sample's contribution w rgb (zero past the first stop: those
            // samples are not composited), and the four are added to the ray's sums in sample order,
            // each addition taking its operand from the lane that holds it
            auto merge = [&](float wq) {
                const float pr = wq * qr, pg = wq * qg, pb = wq * qb;
                C0 = C0 + quad_bcast<0>(pr);
                C1 = C1 + quad_bcast<0>(pg);
                C2 = C2 + quad_bcast<0>(pb);
                C0 = C0 + quad_bcast<1>(pr);
                C1 = C1 + quad_bcast<1>(pg);
                C2 = C2 + quad_bcast<1>(pb);
                C0 = C0 + quad_bcast<2>(pr);
                C1 = C1 + quad_bcast<2>(pg);
                C2 = C2 + quad_bcast<2>(pb);
                C0 = C0 + quad_bcast<3>(pr);
                C1 = C1 + quad_bcast<3>(pg);
                C2 = C2 + quad_bcast<3>(pb);
                if constexpr (DEPTH) {
                    // samples that were not composited add w tm = 0
                    const float pd = wq * tmq;
                    D = D + quad_bcast<0>(pd);
                    D = D + quad_bcast<1>(pd);
                    D = D + quad_bcast<2>(pd);
                    D = D + quad_bcast<3>(pd);
                }
            };
            int first_stop = kQuad - 1;  // last sample that counts
            // A sample can end its ray only if it contributes and its quad's transmittance after all
            // four samples, t4 (<= the transmittance after any of them: every factor is at most 1),
            // is at or past the threshold.  When no lane of the wave has such a sample (the usual
            // case) every sample counts and T becomes t4: the stop search below would find nothing
            // and give the same values.
            if (__ballot(con && A.ert_on && (1.0f - t4 >= A.ert)) == 0ull) {
                merge(w);
                T = t4;
            } else {
                const float t_after = sub == 0 ? t1 : (sub == 1 ? t2 : (sub == 2 ? t3 : t4));
                const bool stop_here = con && (1.0f - t_after >= A.ert);
                const unsigned long long stop_mask = __ballot(stop_here);
                const int stop_bits = static_cast<int>((stop_mask >> quad_base) & 0xFull);
                if (stop_bits) first_stop = __ffs(stop_bits) - 1;
                merge(sub <= first_stop ? w : 0.0f);
                // T after the last sample that counts: t4 without a stop (selected on the stop bits,
                // not on first_stop, which would become a branch and part the additions above from
                // their lane moves)
                T = (stop_bits & 1) ? t1 : ((stop_bits & 2) ? t2 : ((stop_bits & 4) ? t3 : t4));
                // (a ray that stopped in an earlier group has no stop bits here and stays stopped)
                stopped = stopped || stop_bits != 0;
                cnt_nom += stop_bits ? static_cast<uint32_t>(kQuad * q + first_stop + 1) : 0u;
            }
            if constexpr (COUNTS) {
                const unsigned long long comp_mask = __ballot(con);
                const int comp_bits = static_cast<int>((comp_mask >> quad_base) & 0xFull);
                cnt_comp += __popc(comp_bits & ((2 << first_stop) - 1));
                stop_at = first_stop;
            }
        }
        if constexpr (COUNTS) {
            // samples after the termination stop were evaluated by their lanes but are not the method's
            const bool counted = !stopped || sub <= stop_at;
            cnt_eval += counted ? it_eval : 0u;
            cnt_fetch += counted ? it_fetch : 0u;
        }
        if (stopped) {
            alive = false;
        } else {
            // next step: after the P groups, or past the skipped box of the last group's fourth sample
            const int next = last_skipped ? max(j0 + kQuad * P, jn3) : j0 + kQuad * P;
            cnt_nom += static_cast<uint32_t>(min(next, ns) - j0);
            j0 = next;
            if (j0 >= ns) {
                if (seg + 1 < nseg) {
                    seg = 1;
                    sa = sa1;
                    sb = sb1;
                    g = JIT ? fmaf(-s_jit, ds, sa) : sa;
                    ns = max(static_cast<int>(ceilf((sb - g) / ds)), 1);
                    partial_samples();
                    j0 = 0;
                } else {
                    alive = false;
                }
            }
        }
    }

    if constexpr (COUNTS) {
        // the pixel's totals over its quad (every lane takes part in the moves)
        const int e = static_cast<int>(cnt_eval), f = static_cast<int>(cnt_fetch);
        cnt_eval = static_cast<uint32_t>(quad_bcast<0>(e) + quad_bcast<1>(e) + quad_bcast<2>(e) + quad_bcast<3>(e));
        cnt_fetch = static_cast<uint32_t>(quad_bcast<0>(f) + quad_bcast<1>(f) + quad_bcast<2>(f) + quad_bcast<3>(f));
    }
    if (!inside || sub != 0) return;
    const float acc = 1.0f - T;
    float4 res = make_float4(C0, C1, C2, acc);
    if (L->has_bg) {
        res.x = fmaf(T, L->bg[0], res.x);
        res.y = fmaf(T, L->bg[1], res.y);
        res.z = fmaf(T, L->bg[2], res.z);
        res.w = fmaf(T, L->bg[3], res.w);
    }
    const size_t pix = static_cast<size_t>(py) * L->width + px;
    f32x4 o4;
    o4.x = res.x, o4.y = res.y, o4.z = res.z, o4.w = res.w;
    if (!JIT || L->out != nullptr)
        reinterpret_cast<__attribute__((address_space(1))) f32x4*>(reinterpret_cast<uintptr_t>(L->out))[pix] = o4;
    if constexpr (JIT) {
        if (L->mean != nullptr) {
            // running mean over the passes: m <- m + (c - m) / (pass + 1), exactly c on pass 0
            auto* m = reinterpret_cast<__attribute__((address_space(1))) f32x4*>(reinterpret_cast<uintptr_t>(L->mean));
            f32x4 prev = L->pass == 0 ? o4 : m[pix];
            f32x4 nm;
            nm.x = fmaf(o4.x - prev.x, L->inv_pass1, prev.x);
            nm.y = fmaf(o4.y - prev.y, L->inv_pass1, prev.y);
            nm.z = fmaf(o4.z - prev.z, L->inv_pass1, prev.z);
            nm.w = fmaf(o4.w - prev.w, L->inv_pass1, prev.w);
            m[pix] = nm;
        }
    }
    if constexpr (COUNTS) {
        if (L->nominal) L->nominal[pix] = cnt_nom;
        if (L->composited) L->composited[pix] = cnt_comp;
        if (L->evaluated) L->evaluated[pix] = cnt_eval;
        if (L->fetched) L->fetched[pix] = cnt_fetch;
    }
    if constexpr (DEPTH) {
        // the weights sum to the opacity 1 - T (before the background, which has no depth)
        L->depth[pix] = acc > 0.0f ? D / acc : INFINITY;
    }
}

// The kernel's arguments read through a pointer to the argument segment that the compiler cannot see
// through: the loads of the arguments used only after the march (outputs, background, running mean)
// then stay there instead of holding scalar registers throughout it.
typedef const __attribute__((address_space(4))) RenderArgs* KernelArgsPtr;
__device__ __forceinline__ KernelArgsPtr late_args() {
    KernelArgsPtr p = (KernelArgsPtr)__builtin_amdgcn_kernarg_segment_ptr();
    asm volatile("" : "+s"(p));
    return p;
}

// Tiles of a single-image launch: the host counts wave tiles (blocks_x per row); blocks of four waves
// take 2 x 2 of them, and super-tiles hold 2^(s+1) x 2^(s+1) wave tiles (s = super_log2) either way.
struct LaunchTiles {
    int cols, rows, s;
};
template <int BW>
__host__ __device__ inline LaunchTiles launch_tiles(int blocks_x, int n_blocks, int super_log2) {
    const int rows4 = n_blocks / blocks_x;
    if (BW == 4) return {(blocks_x + 1) / 2, (rows4 + 1) / 2, super_log2};
    return {blocks_x, rows4, super_log2 + 1};
}

template <int K, int NB, bool COUNTS, bool JIT = false, bool DEPTH = false, bool WIDE = true>
__global__ __launch_bounds__(64 * block_waves(K, WIDE)) void raymarch_kernel(RenderArgs A) {
    constexpr int BW = block_waves(K, WIDE), BS = BW == 4 ? 2 : 1;  // wave tiles per block side
    const LaunchTiles lt = launch_tiles<BW>(A.blocks_x, A.n_blocks, A.super_log2);
    int bx, by;
    interleaved_tile(blockIdx.x, lt.cols, lt.s, bx, by);
    if (by * BS * (kWaveRays >> A.tile_log2w) >= A.height || bx * BS * (1 << A.tile_log2w) >= A.width)
        return;  // padding block
    __shared__ float4 s_tf[256];
    march_tile<K, NB, COUNTS, JIT, DEPTH, WIDE, BW>(A, late_args(), bx, by, s_tf);
}

// Single-image launch of the kernel with the request's field count as a template argument (the field
// loop unrolled, no per-field guard); coordinate axes take the run-time count variant, which carries
// their test.
template <int K, bool COUNTS, bool JIT, bool DEPTH, bool WIDE = true>
hipError_t launch_fixed(const RenderArgs& a, hipStream_t s) {
    constexpr int BW = block_waves(K, WIDE);
    const LaunchTiles lt = launch_tiles<BW>(a.blocks_x, a.n_blocks, a.super_log2);
    const dim3 grid(padded_blocks(lt.cols, lt.rows, lt.s)), block(64 * BW);
    if (a.coord_mask) {
        hipLaunchKernelGGL((raymarch_kernel<K, kRuntimeNB, COUNTS, JIT, DEPTH, WIDE>), grid, block, 0, s, a);
        return hipGetLastError();
    }
    switch (a.n_brushed) {
        case 0: hipLaunchKernelGGL((raymarch_kernel<K, 0, COUNTS, JIT, DEPTH, WIDE>), grid, block, 0, s, a); break;
        case 1: hipLaunchKernelGGL((raymarch_kernel<K, 1, COUNTS, JIT, DEPTH, WIDE>), grid, block, 0, s, a); break;
        case 2: hipLaunchKernelGGL((raymarch_kernel<K, 2, COUNTS, JIT, DEPTH, WIDE>), grid, block, 0, s, a); break;
        case 3: hipLaunchKernelGGL((raymarch_kernel<K, 3, COUNTS, JIT, DEPTH, WIDE>), grid, block, 0, s, a); break;
        case 4: hipLaunchKernelGGL((raymarch_kernel<K, 4, COUNTS, JIT, DEPTH, WIDE>), grid, block, 0, s, a); break;
        case 5: hipLaunchKernelGGL((raymarch_kernel<K, 5, COUNTS, JIT, DEPTH, WIDE>), grid, block, 0, s, a); break;
        case 6: hipLaunchKernelGGL((raymarch_kernel<K, 6, COUNTS, JIT, DEPTH, WIDE>), grid, block, 0, s, a); break;
        case 7: hipLaunchKernelGGL((raymarch_kernel<K, 7, COUNTS, JIT, DEPTH, WIDE>), grid, block, 0, s, a); break;
        default: hipLaunchKernelGGL((raymarch_kernel<K, 8, COUNTS, JIT, DEPTH, WIDE>), grid, block, 0, s, a); break;
    }
    return hipGetLastError();
}

// The same for every kernel kind; record kinds with record fields below 4 GiB take the 32-bit offset
// variant (except the counting variant, a debugging aid).
template <bool COUNTS, bool JIT, bool DEPTH>
hipError_t launch_fixed_kind(const RenderArgs& a, int kind, hipStream_t s) {
    if constexpr (!COUNTS) {
        if (narrow_records(a)) {
            switch (kind) {
                case kKindF32Rec: return launch_fixed<kKindF32Rec, false, JIT, DEPTH, false>(a, s);
                case kKindF16Rec: return launch_fixed<kKindF16Rec, false, JIT, DEPTH, false>(a, s);
                case kKindU8Rec: return launch_fixed<kKindU8Rec, false, JIT, DEPTH, false>(a, s);
                default: break;
            }
        }
    }
    switch (kind) {
        case kKindF32: return launch_fixed<kKindF32, COUNTS, JIT, DEPTH>(a, s);
        case kKindF16: return launch_fixed<kKindF16, COUNTS, JIT, DEPTH>(a, s);
        case kKindU8: return launch_fixed<kKindU8, COUNTS, JIT, DEPTH>(a, s);
        case kKindF32Rec: return launch_fixed<kKindF32Rec, COUNTS, JIT, DEPTH>(a, s);
        case kKindF16Rec: return launch_fixed<kKindF16Rec, COUNTS, JIT, DEPTH>(a, s);
        default: return launch_fixed<kKindU8Rec, COUNTS, JIT, DEPTH>(a, s);
    }
}

}  // namespace
}  // namespace raypc
