// preprocess.hip -- one-off volume preparation and brush-time tables (gfx950).
//
//  * level build: the octree level-of-detail pyramid of the paper's
//    preprocessing (Section 2.1, two coarser levels with 1/8 the cells):
//    parent = fl32(fl32(fl32((a+b)+(c+d)) + fl32((e+f)+(g+h))) * 0.125),
//    children in (z, y, x) lexicographic order, no contraction;
//  * encode: float32 -> brick-ordered float32 / binary16 (nearest even) /
//    8-bit codes with a per-8^3-brick (scale, offset): offset = brick min,
//    scale = fl32((max - min) / 255), q = clamp(rint(fl32(fl32(v - offset) / scale)), 0, 255),
//    decoded as fl32(fl32(scale * q) + offset);
//  * brick (min, max) of decoded values over voxel indices [8b, min(8b+8, N-1)]
//    per axis -- every voxel a sample whose clamped floor index lies in brick b
//    can read -- and the same over [4s, min(4s+4, N-1)] for each 4^3 sub-brick s;
//  * skip bits (Section 2.2: brush changes rebuild nothing, so only this
//    bit-per-brick table is recomputed): a brick is skipped when an active
//    variable's brick range misses [lo, hi] (or lo > hi), or when the table
//    opacity is zero over every entry the transfer-function variable's brick
//    range can address; the same rule per 4^3 sub-brick gives one byte of
//    sub-brick flags per brick (bit sx + 2 sy + 4 sz), which the ray marcher
//    reads: a brick's window contains its sub-bricks' windows, so a skipped
//    brick has all eight flags set and the bytes alone drive the skipping;
//  * voxel brush masks and decoded exports for parity checks.
// Everything here is streaming work over HBM; none of it is on the per-frame path
// except the skip bits, which touch only the small min/max tables.
#include <hip/hip_fp16.h>

#include "internal.h"

namespace raypc {
namespace {

// Stored value of voxel (x, y, z) on a level with nb bricks per axis: binary16 codes are held scaled
// by the field's power of two 2^k (see f16_scale_kernel) and `descale` = 2^-k gives the value back
// exactly; an 8-bit code is decoded with its brick's (scale, offset) pair.
template <int S>
__device__ __forceinline__ float stored(const void* base, const float2* par, int x, int y, int z, int nb,
                                        float descale = 1.0f) {
    if constexpr (S == kF32) {
        return static_cast<const float*>(base)[brick_addr(x, y, z, nb)];
    } else if constexpr (S == kF16) {
        return __half2float(static_cast<const __half*>(base)[block_index9(x, y, z, nb)]) * descale;
    } else {
        const float q = static_cast<float>(static_cast<const uint8_t*>(base)[u8_addr(x, y, z, nb)]);
        const float2 p = par[brick_index(x, y, z, nb)];
        return __fadd_rn(__fmul_rn(p.x, q), p.y);
    }
}

__device__ __forceinline__ float wave_max(float v);

// Sets *flag when the field holds a non-finite value; raises *maxbits to the bit pattern of the
// largest finite |value| (non-negative floats order as their bit patterns).
__global__ void count_nonfinite_kernel(const float* __restrict__ x, size_t count, unsigned int* flag,
                                       unsigned int* maxbits) {
    size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
    bool bad = false;
    float m = 0.0f;
    for (; i < count; i += stride) {
        const float v = x[i];
        const bool fin = isfinite(v);
        bad |= !fin;
        m = fin ? fmaxf(m, fabsf(v)) : m;
    }
    if (__any(bad) && bad) atomicOr(flag, 1u);
    m = wave_max(m);
    if ((threadIdx.x & 63) == 0) atomicMax(maxbits, __float_as_uint(m));
}

// The power of two that binary16 storage scales a field by: with the field's largest |value| m =
// f 2^e (f in [0.5, 1)), k = max(0, 14 - e), so the scaled values stay below 2^14 and a field of
// small values (one that would otherwise fall in binary16's subnormal range) keeps binary16's
// normal-range precision; k = 0 for an all-zero field.  scale[0] = 2^k, scale[1] = 2^-k.
__global__ void f16_scale_kernel(const unsigned int* maxbits, float* scale, int* exponent) {
    const float m = __uint_as_float(*maxbits);
    int k = 0;
    if (m > 0.0f) {
        int e = 0;
        (void)frexpf(m, &e);
        k = max(0, 14 - e);
    }
    scale[0] = ldexpf(1.0f, k);
    scale[1] = ldexpf(1.0f, -k);
    *exponent = k;
}

// Values of one float32 field at k linear voxel indices (the cells that estimate brush selectivity).
__global__ void gather_cells_kernel(const float* __restrict__ x, const uint32_t* __restrict__ cells, int k,
                                    float* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < k) out[i] = x[cells[i]];
}

// (min, max) pairs of one field's sub-brick table at k indices.
__global__ void gather_pairs_kernel(const float2* __restrict__ x, const uint32_t* __restrict__ idx, int k,
                                    float2* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < k) out[i] = x[idx[i]];
}

__global__ void lod_build_kernel(const float* __restrict__ in, int n, float* __restrict__ out) {
    const int m = n >> 1;
    const uint32_t o = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t total = static_cast<uint32_t>(m) * m * m;
    if (o >= total) return;
    const int x = o % m, y = (o / m) % m, z = o / (static_cast<uint32_t>(m) * m);
    const size_t nn = static_cast<size_t>(n);
    const size_t base = ((2 * static_cast<size_t>(z)) * nn + 2 * y) * nn + 2 * x;
    const size_t dy = nn, dz = nn * nn;
    const float a = in[base], b = in[base + 1];
    const float c = in[base + dy], d = in[base + dy + 1];
    const float e = in[base + dz], f = in[base + dz + 1];
    const float g = in[base + dz + dy], h = in[base + dz + dy + 1];
    const float s0 = __fadd_rn(__fadd_rn(a, b), __fadd_rn(c, d));
    const float s1 = __fadd_rn(__fadd_rn(e, f), __fadd_rn(g, h));
    out[o] = __fmul_rn(__fadd_rn(s0, s1), 0.125f);
}

__device__ __forceinline__ float wave_min(float v) {
    for (int off = 32; off > 0; off >>= 1) v = fminf(v, __shfl_xor(v, off));
    return v;
}
__device__ __forceinline__ float wave_max(float v) {
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
    return v;
}

// One 512-thread block per brick; thread t is the brick-local voxel t.
template <int S>
__global__ __launch_bounds__(512) void encode_kernel(const float* __restrict__ in, int n, void* __restrict__ out,
                                                     float2* __restrict__ u8par, const float* __restrict__ f16_scale) {
    const int nb = n >> 3;
    const uint32_t brick = blockIdx.x;
    const int bx = brick % nb, by = (brick / nb) % nb, bz = brick / (nb * nb);
    const int t = threadIdx.x;
    const int x = bx * 8 + (t & 7), y = by * 8 + ((t >> 3) & 7), z = bz * 8 + (t >> 6);
    const size_t nn = static_cast<size_t>(n);
    const float v = in[(static_cast<size_t>(z) * nn + y) * nn + x];
    if constexpr (S == kF32) {
        const uint32_t a = (brick << 9) | brick_local(t & 7, (t >> 3) & 7, t >> 6);
        static_cast<float*>(out)[a] = v;
    } else if constexpr (S == kF16) {
        const uint32_t a = brick * kBlockValues + (t >> 6) * kBlockZStride + ((t >> 3) & 7) * kBlockYStride + (t & 7);
        // scaling by a power of two is exact: only the binary16 rounding remains
        static_cast<__half*>(out)[a] = __float2half_rn(v * (f16_scale ? f16_scale[0] : 1.0f));
    } else {
        __shared__ float smin[8], smax[8];
        float mn = wave_min(v), mx = wave_max(v);
        const int w = t >> 6;
        if ((t & 63) == 0) {
            smin[w] = mn;
            smax[w] = mx;
        }
        __syncthreads();
        mn = smin[0];
        mx = smax[0];
        for (int k = 1; k < 8; ++k) {
            mn = fminf(mn, smin[k]);
            mx = fmaxf(mx, smax[k]);
        }
        const float scale = __fdiv_rn(__fsub_rn(mx, mn), 255.0f);
        float q = 0.0f;
        if (scale > 0.0f) q = fminf(fmaxf(rintf(__fdiv_rn(__fsub_rn(v, mn), scale)), 0.0f), 255.0f);
        static_cast<uint8_t*>(out)[brick * kU8BrickBytes + (t >> 6) * 81u + ((t >> 3) & 7) * 9u + (t & 7)] =
            static_cast<uint8_t>(q);
        if (t == 0) u8par[brick] = make_float2(scale, mn);
    }
}

// binary16 values: the copies at local x = 8 of every brick (64 per brick), taken from the voxels
// they copy once every brick is encoded.
__global__ __launch_bounds__(64) void f16_apron_kernel(uint16_t* __restrict__ values, int n) {
    const int nb = n >> 3;
    const uint32_t brick = blockIdx.x;
    const int k = threadIdx.x;
    const int bx = brick % nb, by = (brick / nb) % nb, bz = brick / (nb * nb);
    const int ly = k & 7, lz = k >> 3;
    const int x = min(bx * 8 + 8, n - 1), y = by * 8 + ly, z = bz * 8 + lz;
    values[brick * kBlockValues + lz * kBlockZStride + ly * kBlockYStride + 8u] = values[block_index9(x, y, z, nb)];
}

// 8-bit codes: the copies at local x = 8 and y = 8 of every brick (136 per brick: 9 at y = 8 and 8 at
// x = 8 in each of the 8 z planes), taken from the voxels they copy once every brick is encoded.
__global__ __launch_bounds__(192) void u8_apron_kernel(uint8_t* __restrict__ codes, int n) {
    const int nb = n >> 3;
    const uint32_t brick = blockIdx.x;
    const int k = threadIdx.x;
    if (k >= 136) return;
    const int bx = brick % nb, by = (brick / nb) % nb, bz = brick / (nb * nb);
    const int lz = k / 17, r = k % 17;
    const int lx = r < 9 ? r : 8, ly = r < 9 ? 8 : r - 9;
    const int x = min(bx * 8 + lx, n - 1), y = min(by * 8 + ly, n - 1), z = bz * 8 + lz;
    codes[brick * kU8BrickBytes + lz * 81u + ly * 9u + lx] = codes[u8_addr(x, y, z, nb)];
}

// One wave per brick: min / max over the 9^3 apron window of stored values, and over the 5^3 apron
// window of each 4^3 sub-brick (local offsets [4 s, 4 s + 4] per axis, s = 0, 1; offset 4 belongs
// to both halves).  The brick window is the union of the sub-brick windows.
template <int S>
__global__ __launch_bounds__(64) void minmax_kernel(const void* __restrict__ data, const float2* __restrict__ par,
                                                    int n, float2* __restrict__ out, float2* __restrict__ out_sub,
                                                    const float* __restrict__ f16_scale) {
    const float descale = f16_scale ? f16_scale[1] : 1.0f;
    const int nb = n >> 3;
    const uint32_t brick = blockIdx.x;
    const int bx = brick % nb, by = (brick / nb) % nb, bz = brick / (nb * nb);
    float mn[8], mx[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        mn[i] = INFINITY;
        mx[i] = -INFINITY;
    }
    for (int k = threadIdx.x; k < 729; k += 64) {
        const int lx = k % 9, ly = (k / 9) % 9, lz = k / 81;
        const int x = min(bx * 8 + lx, n - 1);
        const int y = min(by * 8 + ly, n - 1);
        const int z = min(bz * 8 + lz, n - 1);
        const float v = stored<S>(data, par, x, y, z, nb, descale);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const bool in = ((i & 1) ? lx >= 4 : lx <= 4) && ((i & 2) ? ly >= 4 : ly <= 4) &&
                            ((i & 4) ? lz >= 4 : lz <= 4);
            if (in) {
                mn[i] = fminf(mn[i], v);
                mx[i] = fmaxf(mx[i], v);
            }
        }
    }
    float bmn = INFINITY, bmx = -INFINITY;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        mn[i] = wave_min(mn[i]);
        mx[i] = wave_max(mx[i]);
        bmn = fminf(bmn, mn[i]);
        bmx = fmaxf(bmx, mx[i]);
    }
    if (threadIdx.x < 8) {
        float a = mn[0], b = mx[0];
#pragma unroll
        for (int i = 1; i < 8; ++i)
            if (static_cast<int>(threadIdx.x) == i) a = mn[i], b = mx[i];
        out_sub[static_cast<size_t>(brick) * 8 + threadIdx.x] = make_float2(a, b);
    }
    if (threadIdx.x == 0) out[brick] = make_float2(bmn, bmx);
}

template <int S>
__global__ void decode_kernel(const void* __restrict__ data, const float2* __restrict__ par, int n,
                              float* __restrict__ out, float descale) {
    const uint32_t o = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t total = static_cast<uint32_t>(n) * n * n;
    if (o >= total) return;
    const int x = o % n, y = (o / n) % n, z = o / (static_cast<uint32_t>(n) * n);
    out[o] = stored<S>(data, par, x, y, z, n >> 3, descale);
}

// Records, one thread per entry of the 9 x 8 x 8 blocks (block_index9 numbering): entry (x, y, z)
// is the voxel at (min(x, N-1), y, z), x = 8 being the next brick's first voxel.  float32: its value
// (bit pattern copied from the float32 array); 8-bit: its value decoded exactly as the compact path
// decodes it; binary16: the pair of values at (x, y) and (x, min(y + 1, N-1)) from the binary16 blocks.
template <int S>
__global__ __launch_bounds__(256) void records_kernel(const void* __restrict__ data, const float2* __restrict__ par,
                                                      int n, uint32_t* __restrict__ out) {
    const int nb = n >> 3;
    const uint32_t total = static_cast<uint32_t>(nb) * nb * nb * kBlockValues;
    const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    const uint32_t brick = e / kBlockValues, rem = e % kBlockValues;
    const int lz = (rem / kBlockZStride) % 8, ly = (rem / kBlockYStride) % 8, lx = rem % 9;
    const int bx = brick % nb, by = (brick / nb) % nb, bz = brick / (nb * nb);
    const int x = min(bx * 8 + lx, n - 1), y = by * 8 + ly, z = bz * 8 + lz;
    if constexpr (S == kF32) {
        out[e] = static_cast<const uint32_t*>(data)[brick_addr(x, y, z, nb)];
    } else if constexpr (S == kU8) {
        out[e] = __float_as_uint(stored<kU8>(data, par, x, y, z, nb));
    } else {
        const uint16_t* v = static_cast<const uint16_t*>(data);
        const int y1 = min(y + 1, n - 1);
        out[e] = static_cast<uint32_t>(v[block_index9(x, y, z, nb)]) |
                 (static_cast<uint32_t>(v[block_index9(x, y1, z, nb)]) << 16);
    }
}

template <int S>
__global__ void voxel_mask_kernel(MaskArgs a) {
    const uint32_t o = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t total = static_cast<uint32_t>(a.n) * a.n * a.n;
    if (o >= total) return;
    const int x = o % a.n, y = (o / a.n) % a.n, z = o / (static_cast<uint32_t>(a.n) * a.n);
    bool keep = true;
    for (int f = 0; f < a.n_active; ++f) {
        const float v = stored<S>(a.field[f], a.u8par[f], x, y, z, a.nb, a.descale[f]);
        keep = keep && (v >= a.lo[f]) && (v <= a.hi[f]);
    }
    if (a.coord_mask)
        keep = keep && coord_ok(a.coord_mask, a.clo, a.chi, cell_coord(x, a.n), cell_coord(y, a.n), cell_coord(z, a.n));
    a.out[o] = keep ? 1 : 0;
}

// Parallel-coordinates lines: one thread per line; histograms gather in LDS and are added to the
// (zeroed) output once per block.  A cell index outside the grid gives NaN values, flag 0 and no
// histogram entry.
template <int S>
__global__ __launch_bounds__(256) void pc_lines_kernel(PcArgs a) {
    __shared__ uint32_t s_hist[kMaxFields * kMaxPcBins * 2];
    const int hist_len = a.n_fields * a.n_bins * 2;
    if (a.hist != nullptr)
        for (int i = threadIdx.x; i < hist_len; i += blockDim.x) s_hist[i] = 0;
    __syncthreads();
    const uint32_t total = static_cast<uint32_t>(a.n) * a.n * a.n;
    for (int line = blockIdx.x * blockDim.x + threadIdx.x; line < a.n_lines; line += gridDim.x * blockDim.x) {
        const uint32_t c = a.cells[line];
        const bool valid = c < total;
        const int x = static_cast<int>(c % a.n), y = static_cast<int>((c / a.n) % a.n);
        const int z = static_cast<int>(c / (static_cast<uint32_t>(a.n) * a.n));
        bool pass = valid;
        if (valid && a.coord_mask)
            pass = coord_ok(a.coord_mask, a.clo, a.chi, cell_coord(x, a.n), cell_coord(y, a.n), cell_coord(z, a.n));
        for (int f = 0; f < a.n_fields; ++f) {
            const float v = valid ? stored<S>(a.field[f], a.u8par[f], x, y, z, a.nb, a.descale[f]) : NAN;
            if (a.values != nullptr) a.values[static_cast<size_t>(line) * a.n_fields + f] = v;
            if (a.active[f]) pass = pass && (v >= a.lo[f]) && (v <= a.hi[f]);
        }
        if (a.passes != nullptr) a.passes[line] = pass ? 1 : 0;
        if (a.hist != nullptr && valid) {
            for (int f = 0; f < a.n_fields; ++f) {
                const float v = stored<S>(a.field[f], a.u8par[f], x, y, z, a.nb, a.descale[f]);
                const float t = __fmul_rn(__fsub_rn(v, a.axis_lo[f]), a.inv[f]);
                const float xb = fminf(fmaxf(__fmul_rn(t, static_cast<float>(a.n_bins)), 0.0f),
                                       static_cast<float>(a.n_bins - 1));
                const int b = static_cast<int>(floorf(xb));
                atomicAdd(&s_hist[(f * a.n_bins + b) * 2], 1u);
                if (pass) atomicAdd(&s_hist[(f * a.n_bins + b) * 2 + 1], 1u);
            }
        }
    }
    if (a.hist == nullptr) return;
    __syncthreads();
    for (int i = threadIdx.x; i < hist_len; i += blockDim.x)
        if (s_hist[i]) atomicAdd(&a.hist[i], s_hist[i]);
}

__global__ void zero_u32_kernel(uint32_t* p, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0;
}

// The skip rule for one (min, max) window: some active field misses its [lo, hi] (or lo > hi), or
// the table opacity is zero over every entry the transfer-function field's range can address.
__device__ __forceinline__ bool tf_range_empty(const SkipArgs& a, float2 tm) {
    const float t0 = fminf(fmaxf(__fmul_rn(__fsub_rn(tm.x, a.vmin), a.inv_range), 0.0f), 1.0f);
    const float t1 = fminf(fmaxf(__fmul_rn(__fsub_rn(tm.y, a.vmin), a.inv_range), 0.0f), 1.0f);
    const int i0 = static_cast<int>(floorf(__fmul_rn(t0, 255.0f)));
    const int i1 = min(static_cast<int>(ceilf(__fmul_rn(t1, 255.0f))), 255);
    return a.next_nonzero[i0] > i1;
}

// Sub-brick flags (bit i) of the eight (min, max) pairs at p (one brick's 64-byte block) against one
// field's [lo, hi], read as four 16-byte loads.
__device__ __forceinline__ uint32_t sub_range_misses(const float2* p, float lo, float hi) {
    const float4* q = reinterpret_cast<const float4*>(p);
    uint32_t m = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float4 v = q[k];
        m |= static_cast<uint32_t>((v.y < lo) | (v.x > hi)) << (2 * k);
        m |= static_cast<uint32_t>((v.w < lo) | (v.z > hi)) << (2 * k + 1);
    }
    return m;
}

// Coordinate axes against a box of box^3 voxels starting at voxel (x0, y0, z0): true when no sample
// position whose clamped floor index lies in the box can pass them.  Those positions lie inside
// [fl32(fl32(i0 h) - 1), fl32(fl32((i1 + 2) h) - 1)] per axis (half a voxel of margin each side,
// open at the grid faces); the radius axis compares the box's float32 squared-radius range.
__device__ bool coord_box_miss(const SkipArgs& a, int x0, int y0, int z0, int box) {
    const int i0[3] = {x0, y0, z0};
    float bmin[3], bmax[3];
    for (int ax = 0; ax < 3; ++ax) {
        const int i1 = i0[ax] + box - 1;
        bmin[ax] = i0[ax] == 0 ? -INFINITY : __fsub_rn(__fmul_rn(static_cast<float>(i0[ax]), a.h), 1.0f);
        bmax[ax] = i1 == a.n - 1 ? INFINITY : __fsub_rn(__fmul_rn(static_cast<float>(i1 + 2), a.h), 1.0f);
    }
    bool miss = false;
    for (int ax = 0; ax < 3; ++ax)
        if (a.coord_mask & (1u << ax)) miss = miss || bmax[ax] < a.clo[ax] || bmin[ax] > a.chi[ax];
    if (a.coord_mask & 8u) {
        float d2[3], m2[3];
        for (int ax = 0; ax < 3; ++ax) {
            const float d = fmaxf(fmaxf(0.0f, bmin[ax]), -bmax[ax]);
            d2[ax] = __fmul_rn(d, d);
            m2[ax] = fmaxf(__fmul_rn(bmin[ax], bmin[ax]), __fmul_rn(bmax[ax], bmax[ax]));
        }
        const float rmin2 = __fadd_rn(__fadd_rn(d2[0], d2[1]), d2[2]);
        const float rmax2 = __fadd_rn(__fadd_rn(m2[0], m2[1]), m2[2]);
        miss = miss || rmin2 > a.chi[3] || rmax2 < a.clo[3];
    }
    return miss;
}

// One brick's flag word without the group bits: the brick rule's skip bit (kBrickSkipBit) and the
// sub-brick flags (bits 0-7).  A skipped brick's sub-bricks are all skipped (their windows lie inside
// its window and the table index map is monotone), so only the other bricks read sub-brick tables.
__device__ uint32_t brick_word(const SkipArgs& a, uint32_t b, int bx, int by, int bz) {
    bool skip = false;
    for (int f = 0; f < a.n_active; ++f) {
        const float2 mm = a.minmax[f][b];
        skip |= (mm.y < a.lo[f]) | (mm.x > a.hi[f]) | (a.lo[f] > a.hi[f]);
    }
    skip |= tf_range_empty(a, a.tf_minmax[b]);
    if (a.coord_mask) skip = skip || coord_box_miss(a, bx * 8, by * 8, bz * 8, 8);
    if (skip) return 0xFFu | kBrickSkipBit;
    uint32_t sub = 0;
    for (int f = 0; f < a.n_active; ++f) sub |= sub_range_misses(a.minmax_sub[f] + static_cast<size_t>(b) * 8, a.lo[f], a.hi[f]);
    const float4* q = reinterpret_cast<const float4*>(a.tf_minmax_sub + static_cast<size_t>(b) * 8);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float4 v = q[k];
        sub |= static_cast<uint32_t>(tf_range_empty(a, make_float2(v.x, v.y))) << (2 * k);
        sub |= static_cast<uint32_t>(tf_range_empty(a, make_float2(v.z, v.w))) << (2 * k + 1);
    }
    if (a.coord_mask)
        for (int i = 0; i < 8; ++i)
            if (coord_box_miss(a, bx * 8 + (i & 1) * 4, by * 8 + ((i >> 1) & 1) * 4, bz * 8 + (i >> 2) * 4, 4))
                sub |= 1u << i;
    return sub;
}

// The skip pass: one wave per aligned 4^3-brick group (four groups per block), lane t on the brick at
// offset (x, y, z) with t = x0 + 2 y0 + 4 z0 + 8 (x1 + 2 y1 + 4 z1) (bit 0 and bit 1 of each offset), so
// that each 2^3-brick subgroup is one run of 8 lanes; a wave ballot gives the empty-group bits.
// Bricks outside the grid count as empty.
__global__ __launch_bounds__(256) void skip_kernel(SkipArgs a) {
    const int gpa = (a.nb + 3) / 4;  // groups per axis
    const int g = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (g >= gpa * gpa * gpa) return;  // the whole wave
    const int gx = g % gpa, gy = (g / gpa) % gpa, gz = g / (gpa * gpa);
    const int t = threadIdx.x & 63;
    const int x = gx * 4 + ((t & 1) | ((t >> 2) & 2));
    const int y = gy * 4 + (((t >> 1) & 1) | ((t >> 3) & 2));
    const int z = gz * 4 + (((t >> 2) & 1) | ((t >> 4) & 2));
    const bool inside = x < a.nb && y < a.nb && z < a.nb;
    const uint32_t b = (static_cast<uint32_t>(z) * a.nb + y) * a.nb + x;
    const uint32_t w = inside ? brick_word(a, b, x, y, z) : 0xFFu;
    const unsigned long long full = __ballot((w & 0xFFu) == 0xFFu);
    const bool group16 = ((full >> (t & ~7)) & 0xFFull) == 0xFFull;
    const bool group32 = full == ~0ull;
    if (inside) a.out_sub[b] = static_cast<uint16_t>(w | (group16 ? 0x100u : 0u) | (group32 ? 0x200u : 0u));
}

// Brick skip bits of the flag words packed 32 to a word (brick k: bit k % 32 of word k / 32).
__global__ __launch_bounds__(256) void pack_skip_bits_kernel(const uint16_t* __restrict__ words, uint32_t n_bricks,
                                                             uint32_t* __restrict__ out) {
    const uint32_t wd = blockIdx.x * blockDim.x + threadIdx.x;
    if (wd >= (n_bricks + 31) / 32) return;
    uint32_t m = 0;
    for (uint32_t i = 0; i < 32; ++i) {
        const uint32_t b = wd * 32 + i;
        if (b < n_bricks && (words[b] & kBrickSkipBit)) m |= 1u << i;
    }
    out[wd] = m;
}

inline unsigned blocks_for(size_t count, unsigned threads) {
    return static_cast<unsigned>((count + threads - 1) / threads);
}

}  // namespace

hipError_t launch_count_nonfinite(const float* x, size_t count, unsigned int* flag, unsigned int* maxbits,
                                  hipStream_t s) {
    const unsigned blocks = static_cast<unsigned>(std::min<size_t>(blocks_for(count, 256), 8192));
    hipLaunchKernelGGL(count_nonfinite_kernel, dim3(std::max(blocks, 1u)), dim3(256), 0, s, x, count, flag, maxbits);
    return hipGetLastError();
}

hipError_t launch_f16_scale(const unsigned int* maxbits, float* scale, int* exponent, hipStream_t s) {
    hipLaunchKernelGGL(f16_scale_kernel, dim3(1), dim3(1), 0, s, maxbits, scale, exponent);
    return hipGetLastError();
}

hipError_t launch_gather_cells(const float* x, const uint32_t* cells, int k, float* out, hipStream_t s) {
    if (k <= 0) return hipSuccess;
    hipLaunchKernelGGL(gather_cells_kernel, dim3(blocks_for(static_cast<size_t>(k), 256)), dim3(256), 0, s, x, cells,
                       k, out);
    return hipGetLastError();
}

hipError_t launch_gather_pairs(const float2* x, const uint32_t* idx, int k, float2* out, hipStream_t s) {
    if (k <= 0) return hipSuccess;
    hipLaunchKernelGGL(gather_pairs_kernel, dim3(blocks_for(static_cast<size_t>(k), 256)), dim3(256), 0, s, x, idx,
                       k, out);
    return hipGetLastError();
}

hipError_t launch_lod_build(const float* in, int n, float* out, hipStream_t s) {
    const size_t m = static_cast<size_t>(n / 2);
    hipLaunchKernelGGL(lod_build_kernel, dim3(blocks_for(m * m * m, 256)), dim3(256), 0, s, in, n, out);
    return hipGetLastError();
}

hipError_t launch_encode(const float* in, int n, int storage, void* out, float2* u8par, const float* f16_scale,
                         hipStream_t s) {
    const unsigned nbr = static_cast<unsigned>((n / 8) * (n / 8) * (n / 8));
    switch (storage) {
        case kF32: hipLaunchKernelGGL(encode_kernel<kF32>, dim3(nbr), dim3(512), 0, s, in, n, out, u8par, nullptr); break;
        case kF16:
            hipLaunchKernelGGL(encode_kernel<kF16>, dim3(nbr), dim3(512), 0, s, in, n, out, u8par, f16_scale);
            hipLaunchKernelGGL(f16_apron_kernel, dim3(nbr), dim3(64), 0, s, static_cast<uint16_t*>(out), n);
            break;
        default:
            hipLaunchKernelGGL(encode_kernel<kU8>, dim3(nbr), dim3(512), 0, s, in, n, out, u8par, nullptr);
            hipLaunchKernelGGL(u8_apron_kernel, dim3(nbr), dim3(192), 0, s, static_cast<uint8_t*>(out), n);
            break;
    }
    return hipGetLastError();
}

hipError_t launch_minmax(const void* data, const float2* u8par, int n, int storage, float2* out, float2* out_sub,
                         const float* f16_scale, hipStream_t s) {
    const unsigned nbr = static_cast<unsigned>((n / 8) * (n / 8) * (n / 8));
    switch (storage) {
        case kF32:
            hipLaunchKernelGGL(minmax_kernel<kF32>, dim3(nbr), dim3(64), 0, s, data, u8par, n, out, out_sub, nullptr);
            break;
        case kF16:
            hipLaunchKernelGGL(minmax_kernel<kF16>, dim3(nbr), dim3(64), 0, s, data, u8par, n, out, out_sub, f16_scale);
            break;
        default:
            hipLaunchKernelGGL(minmax_kernel<kU8>, dim3(nbr), dim3(64), 0, s, data, u8par, n, out, out_sub, nullptr);
            break;
    }
    return hipGetLastError();
}

hipError_t launch_decode(const void* data, const float2* u8par, int n, int storage, float* out, float f16_descale,
                         hipStream_t s) {
    const size_t total = static_cast<size_t>(n) * n * n;
    const dim3 g(blocks_for(total, 256));
    switch (storage) {
        case kF32: hipLaunchKernelGGL(decode_kernel<kF32>, g, dim3(256), 0, s, data, u8par, n, out, 1.0f); break;
        case kF16: hipLaunchKernelGGL(decode_kernel<kF16>, g, dim3(256), 0, s, data, u8par, n, out, f16_descale); break;
        default: hipLaunchKernelGGL(decode_kernel<kU8>, g, dim3(256), 0, s, data, u8par, n, out, 1.0f); break;
    }
    return hipGetLastError();
}

hipError_t launch_records(const void* data, const float2* u8par, int n, int storage, void* out, hipStream_t s) {
    const size_t entries = static_cast<size_t>(n >> 3) * (n >> 3) * (n >> 3) * kBlockValues;
    const dim3 g(blocks_for(entries, 256));
    uint32_t* o = static_cast<uint32_t*>(out);
    switch (storage) {
        case kF32: hipLaunchKernelGGL(records_kernel<kF32>, g, dim3(256), 0, s, data, u8par, n, o); break;
        case kF16: hipLaunchKernelGGL(records_kernel<kF16>, g, dim3(256), 0, s, data, u8par, n, o); break;
        default: hipLaunchKernelGGL(records_kernel<kU8>, g, dim3(256), 0, s, data, u8par, n, o); break;
    }
    return hipGetLastError();
}

hipError_t launch_voxel_mask(const MaskArgs& a, hipStream_t s) {
    const size_t total = static_cast<size_t>(a.n) * a.n * a.n;
    const dim3 g(blocks_for(total, 256));
    switch (a.storage) {
        case kF32: hipLaunchKernelGGL(voxel_mask_kernel<kF32>, g, dim3(256), 0, s, a); break;
        case kF16: hipLaunchKernelGGL(voxel_mask_kernel<kF16>, g, dim3(256), 0, s, a); break;
        default: hipLaunchKernelGGL(voxel_mask_kernel<kU8>, g, dim3(256), 0, s, a); break;
    }
    return hipGetLastError();
}

hipError_t launch_pc_lines(const PcArgs& a, hipStream_t s) {
    if (a.hist != nullptr) {
        const int count = a.n_fields * a.n_bins * 2;
        hipLaunchKernelGGL(zero_u32_kernel, dim3(blocks_for(count, 256)), dim3(256), 0, s, a.hist, count);
    }
    if (a.n_lines <= 0) return hipGetLastError();
    const unsigned blocks = std::min(blocks_for(static_cast<size_t>(a.n_lines), 256), 1024u);
    switch (a.storage) {
        case kF32: hipLaunchKernelGGL(pc_lines_kernel<kF32>, dim3(blocks), dim3(256), 0, s, a); break;
        case kF16: hipLaunchKernelGGL(pc_lines_kernel<kF16>, dim3(blocks), dim3(256), 0, s, a); break;
        default: hipLaunchKernelGGL(pc_lines_kernel<kU8>, dim3(blocks), dim3(256), 0, s, a); break;
    }
    return hipGetLastError();
}

hipError_t launch_skip(const SkipArgs& a, hipStream_t s) {
    const unsigned gpa = static_cast<unsigned>((a.nb + 3) / 4);
    const unsigned groups = gpa * gpa * gpa;
    hipLaunchKernelGGL(skip_kernel, dim3(std::max((groups + 3) / 4, 1u)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_pack_skip_bits(const uint16_t* words, uint32_t n_bricks, uint32_t* out, hipStream_t s) {
    const unsigned blocks = blocks_for((n_bricks + 31) / 32, 256);
    hipLaunchKernelGGL(pack_skip_bits_kernel, dim3(std::max(blocks, 1u)), dim3(256), 0, s, words, n_bricks, out);
    return hipGetLastError();
}

}  // namespace raypc
