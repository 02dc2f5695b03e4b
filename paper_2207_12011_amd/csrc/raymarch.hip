// raymarch.hip -- brushed direct volume ray casting of a spherical shell (gfx950).
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
// Mapping to CDNA4: one ray per lane, one wave64 per 8 x 8 pixel tile, four
// waves per 256-thread block (16 x 16 pixels).  The lane loop runs while any
// lane of the wave is alive, so a tile leaves as soon as all of its rays have
// terminated or left the shell.  Blocks are remapped so that each XCD (blocks
// are dealt round-robin over the 8 XCDs) works on one contiguous band of the
// image and its L2 sees neighbouring rays.  The transfer function sits in LDS.
// Field data is brick ordered (8^3 bricks), so the 8 corners of a sample
// usually fall into one 512-voxel brick.  Bricks whose skip bit is set are
// stepped over without fetching: every sample inside such a brick would be
// discarded or fully transparent, so skipping changes no value.
#include <hip/hip_fp16.h>

#include "internal.h"

namespace raypc {
namespace {

constexpr float kSkipShrink = 2e-3f;    // voxels: shrink of a skipped brick before computing its exit
constexpr float kSkipMargin = 0.01f;    // samples: margin on the first sample after a skipped brick

template <int S>
__device__ __forceinline__ float corner(const void* __restrict__ base, const float2* __restrict__ par, uint32_t a) {
    if constexpr (S == kF32) {
        return static_cast<const float*>(base)[a];
    } else if constexpr (S == kF16) {
        return __half2float(static_cast<const __half*>(base)[a]);
    } else {
        const float q = static_cast<float>(static_cast<const uint8_t*>(base)[a]);
        const float2 p = par[a >> 9];
        return __fadd_rn(__fmul_rn(p.x, q), p.y);
    }
}

// Corner addresses are indexed by bit 0 = x, bit 1 = y, bit 2 = z.
template <int S>
__device__ __forceinline__ float fetch(const void* __restrict__ base, const float2* __restrict__ par,
                                       const uint32_t (&o)[8], float wx, float wy, float wz) {
    const float c0 = corner<S>(base, par, o[0]), c1 = corner<S>(base, par, o[1]);
    const float c2 = corner<S>(base, par, o[2]), c3 = corner<S>(base, par, o[3]);
    const float c4 = corner<S>(base, par, o[4]), c5 = corner<S>(base, par, o[5]);
    const float c6 = corner<S>(base, par, o[6]), c7 = corner<S>(base, par, o[7]);
    const float x00 = fmaf(wx, c1 - c0, c0);
    const float x10 = fmaf(wx, c3 - c2, c2);
    const float x01 = fmaf(wx, c5 - c4, c4);
    const float x11 = fmaf(wx, c7 - c6, c6);
    const float y0 = fmaf(wy, x10 - x00, x00);
    const float y1 = fmaf(wy, x11 - x01, x01);
    return fmaf(wz, y1 - y0, y0);
}

// Ray parameter where u(t) = uo + du t leaves [lo, hi] along one axis (forward only).
__device__ __forceinline__ float axis_exit(float uo, float du, float lo, float hi) {
    if (du > 0.0f) return (hi - uo) / du;
    if (du < 0.0f) return (lo - uo) / du;
    return INFINITY;
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

template <int S, int NB, bool COUNTS>
__global__ __launch_bounds__(256) void raymarch_kernel(RenderArgs A) {
    __shared__ float4 s_tf[256];
    s_tf[threadIdx.x] = A.tf[threadIdx.x];
    __syncthreads();

    // XCD-aware block order: block i runs on XCD i % 8; give each XCD a contiguous range.
    const int nbk = A.n_blocks;
    const int bid = blockIdx.x;
    const int q8 = nbk >> 3, r8 = nbk & 7;
    const int xcd = bid & 7, pos = bid >> 3;
    const int blk = xcd < r8 ? xcd * (q8 + 1) + pos : r8 * (q8 + 1) + (xcd - r8) * q8 + pos;
    const int bx = blk % A.blocks_x, by = blk / A.blocks_x;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int px = bx * kBlockPix + (wave & 1) * kTileW + (lane & 7);
    const int py = by * kBlockPix + (wave >> 1) * kTileW + (lane >> 3);
    const bool inside = px < A.width && py < A.height;

    // ---- ray through the pixel centre
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
    float seg_a[2] = {0.0f, 0.0f}, seg_b[2] = {0.0f, 0.0f};
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
        if (cb0 > ca0) {
            seg_a[nseg] = ca0;
            seg_b[nseg] = cb0;
            ++nseg;
        }
        if (inner) {
            ca1 = fmaxf(ca1, 0.0f);
            if (cb1 > ca1) {
                seg_a[nseg] = ca1;
                seg_b[nseg] = cb1;
                ++nseg;
            }
        }
    }

    const int n = A.n, nb = A.nb;
    const float hn = A.half_n;
    const float uox = fmaf(ox, hn, hn - 0.5f), uoy = fmaf(oy, hn, hn - 0.5f), uoz = fmaf(oz, hn, hn - 0.5f);
    const float dux = dx * hn, duy = dy * hn, duz = dz * hn;
    const float ds = A.ds, inv_ds = A.inv_ds;
    const float r_full = ds * A.inv_ref;

    float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
    uint32_t cnt_nom = 0, cnt_comp = 0;
    uint32_t last_brick = 0xFFFFFFFFu;
    int seg = 0, j = 0;
    float sa = seg_a[0], sb = seg_b[0];
    int ns = nseg > 0 ? static_cast<int>(ceilf((sb - sa) / ds)) : 0;
    bool alive = nseg > 0;

    while (alive) {
        const float tlo = fmaf(static_cast<float>(j), ds, sa);
        const bool last = j == ns - 1;
        const float tm = last ? 0.5f * (tlo + sb) : fmaf(static_cast<float>(j) + 0.5f, ds, sa);
        const float ux = fmaf(dux, tm, uox), uy = fmaf(duy, tm, uoy), uz = fmaf(duz, tm, uoz);
        const float flx = floorf(ux), fly = floorf(uy), flz = floorf(uz);
        const int ix = static_cast<int>(flx), iy = static_cast<int>(fly), iz = static_cast<int>(flz);
        const int x0 = min(max(ix, 0), n - 1), x1 = min(max(ix + 1, 0), n - 1);
        const int y0 = min(max(iy, 0), n - 1), y1 = min(max(iy + 1, 0), n - 1);
        const int z0 = min(max(iz, 0), n - 1), z1 = min(max(iz + 1, 0), n - 1);

        bool skipped = false;
        const int bxi = x0 >> 3, byi = y0 >> 3, bzi = z0 >> 3;
        const uint32_t brick = (static_cast<uint32_t>(bzi) * nb + byi) * nb + bxi;
        if (A.skip != nullptr) {
            if ((A.skip[brick >> 5] >> (brick & 31)) & 1u) {
                skipped = true;
                const float lx = bxi == 0 ? -INFINITY : bxi * 8.0f + kSkipShrink;
                const float hx = bxi == nb - 1 ? INFINITY : bxi * 8.0f + 8.0f - kSkipShrink;
                const float ly = byi == 0 ? -INFINITY : byi * 8.0f + kSkipShrink;
                const float hy = byi == nb - 1 ? INFINITY : byi * 8.0f + 8.0f - kSkipShrink;
                const float lz = bzi == 0 ? -INFINITY : bzi * 8.0f + kSkipShrink;
                const float hz = bzi == nb - 1 ? INFINITY : bzi * 8.0f + 8.0f - kSkipShrink;
                const float t_exit = fminf(axis_exit(uox, dux, lx, hx),
                                           fminf(axis_exit(uoy, duy, ly, hy), axis_exit(uoz, duz, lz, hz)));
                // first sample whose midpoint may lie beyond the exit
                float jc = (t_exit - sa) * inv_ds - 0.5f - kSkipMargin;
                jc = fminf(fmaxf(jc, 0.0f), static_cast<float>(ns));
                const int jn = max(j + 1, static_cast<int>(ceilf(jc)));
                cnt_nom += static_cast<uint32_t>(jn - j);
                j = jn;
            }
        }

        if (!skipped) {
            cnt_nom += 1;
            if constexpr (COUNTS) {
                if (A.touched != nullptr && brick != last_brick) {
                    atomicOr(&A.touched[brick >> 5], 1u << (brick & 31));
                    last_brick = brick;
                }
            }
            const float wx = ux - flx, wy = uy - fly, wz = uz - flz;
            const uint32_t X0 = (static_cast<uint32_t>(x0 >> 3) << 9) | (x0 & 7);
            const uint32_t X1 = (static_cast<uint32_t>(x1 >> 3) << 9) | (x1 & 7);
            const uint32_t Y0 = ((static_cast<uint32_t>(y0 >> 3) * nb) << 9) | ((y0 & 7) << 3);
            const uint32_t Y1 = ((static_cast<uint32_t>(y1 >> 3) * nb) << 9) | ((y1 & 7) << 3);
            const uint32_t Z0 = ((static_cast<uint32_t>(z0 >> 3) * nb * nb) << 9) | ((z0 & 7) << 6);
            const uint32_t Z1 = ((static_cast<uint32_t>(z1 >> 3) * nb * nb) << 9) | ((z1 & 7) << 6);
            const uint32_t zy00 = Z0 + Y0, zy01 = Z0 + Y1, zy10 = Z1 + Y0, zy11 = Z1 + Y1;
            const uint32_t o[8] = {zy00 + X0, zy00 + X1, zy01 + X0, zy01 + X1,
                                   zy10 + X0, zy10 + X1, zy11 + X0, zy11 + X1};

            bool pass = true;
            float tv = 0.0f;
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                if (pass) {
                    const float v = fetch<S>(A.field[k], A.u8par[k], o, wx, wy, wz);
                    pass = (v >= A.lo[k]) && (v <= A.hi[k]);
                    if (k == A.tf_slot) tv = v;
                }
            }
            if (pass) {
                if constexpr (NB < kMaxFields) {
                    if (A.tf_slot == NB) tv = fetch<S>(A.field[NB], A.u8par[NB], o, wx, wy, wz);
                }
                const float xt = fminf(fmaxf((tv - A.vmin) * A.inv_range, 0.0f), 1.0f) * 255.0f;
                const int it = min(static_cast<int>(xt), 254);
                const float wt = xt - static_cast<float>(it);
                const float4 e0 = s_tf[it], e1 = s_tf[it + 1];
                const float al = fmaf(wt, e1.w - e0.w, e0.w);
                if (al > 0.0f) {
                    if constexpr (COUNTS) cnt_comp += 1;
                    const float r = last ? fmaxf(sb - tlo, 0.0f) * A.inv_ref : r_full;
                    const float keep = al >= 1.0f ? 0.0f : exp2f(r * __log2f(1.0f - al));
                    const float w = T * (1.0f - keep);
                    C0 = fmaf(w, fmaf(wt, e1.x - e0.x, e0.x), C0);
                    C1 = fmaf(w, fmaf(wt, e1.y - e0.y, e0.y), C1);
                    C2 = fmaf(w, fmaf(wt, e1.z - e0.z, e0.z), C2);
                    T *= keep;
                    if (A.ert_on && 1.0f - T >= A.ert) alive = false;
                }
            }
            j += 1;
        }

        if (alive && j >= ns) {
            if (seg == 0 && nseg == 2) {
                seg = 1;
                sa = seg_a[1];
                sb = seg_b[1];
                ns = static_cast<int>(ceilf((sb - sa) / ds));
                j = 0;
            } else {
                alive = false;
            }
        }
    }

    if (!inside) return;
    float4 res = make_float4(C0, C1, C2, 1.0f - T);
    if (A.has_bg) {
        res.x = fmaf(T, A.bg[0], res.x);
        res.y = fmaf(T, A.bg[1], res.y);
        res.z = fmaf(T, A.bg[2], res.z);
        res.w = fmaf(T, A.bg[3], res.w);
    }
    const size_t pix = static_cast<size_t>(py) * A.width + px;
    A.out[pix] = res;
    if constexpr (COUNTS) {
        if (A.nominal) A.nominal[pix] = cnt_nom;
        if (A.composited) A.composited[pix] = cnt_comp;
    }
}

template <int S, bool COUNTS>
hipError_t launch_nb(const RenderArgs& a, hipStream_t s) {
    const dim3 grid(a.n_blocks), block(256);
    switch (a.n_brushed) {
        case 0: hipLaunchKernelGGL((raymarch_kernel<S, 0, COUNTS>), grid, block, 0, s, a); break;
        case 1: hipLaunchKernelGGL((raymarch_kernel<S, 1, COUNTS>), grid, block, 0, s, a); break;
        case 2: hipLaunchKernelGGL((raymarch_kernel<S, 2, COUNTS>), grid, block, 0, s, a); break;
        case 3: hipLaunchKernelGGL((raymarch_kernel<S, 3, COUNTS>), grid, block, 0, s, a); break;
        case 4: hipLaunchKernelGGL((raymarch_kernel<S, 4, COUNTS>), grid, block, 0, s, a); break;
        case 5: hipLaunchKernelGGL((raymarch_kernel<S, 5, COUNTS>), grid, block, 0, s, a); break;
        case 6: hipLaunchKernelGGL((raymarch_kernel<S, 6, COUNTS>), grid, block, 0, s, a); break;
        case 7: hipLaunchKernelGGL((raymarch_kernel<S, 7, COUNTS>), grid, block, 0, s, a); break;
        default: hipLaunchKernelGGL((raymarch_kernel<S, 8, COUNTS>), grid, block, 0, s, a); break;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_render(const RenderArgs& a, int storage, bool counts, hipStream_t s) {
    if (counts) {
        switch (storage) {
            case kF32: return launch_nb<kF32, true>(a, s);
            case kF16: return launch_nb<kF16, true>(a, s);
            default: return launch_nb<kU8, true>(a, s);
        }
    }
    switch (storage) {
        case kF32: return launch_nb<kF32, false>(a, s);
        case kF16: return launch_nb<kF16, false>(a, s);
        default: return launch_nb<kU8, false>(a, s);
    }
}

}  // namespace raypc
