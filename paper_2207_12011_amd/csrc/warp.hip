// warp.hip -- forward image warping of a rendered frame to another camera pose (gfx950).
//
// Paper, Sections 2 and 2.2: the display runs decoupled from the ray caster and fills the frames the
// caster has not delivered yet by warping the last image it did deliver.  The warp implemented here
// reprojects every pixel of that image with its opacity-weighted depth:
//  * the pixel's ray (through its centre, as the render casts it) is followed to its depth, giving a
//    world point; a pixel whose depth is not finite is a point at infinity along its ray;
//  * the point is projected through the destination camera and lands on the pixel containing the
//    projection (points on or behind the destination's image plane, or outside its image, are
//    dropped);
//  * a z-buffer on (distance from the destination eye, source index) picks one winner per pixel:
//    the nearest point, the lowest source index among equal distances;
//  * a pixel that nothing landed on takes the winner of its eight neighbours with the greatest key
//    (the farthest: the cracks of forward warping open where a nearer surface uncovers a farther
//    one), else stays empty (RGBA 0, depth +inf, source -1);
//  * the winner's RGBA is copied unchanged and its distance from the destination eye becomes the
//    new depth.
// Which pixel a point lands on is a floating-point decision that selects an integer, so it is taken
// in float32 one correctly rounded operation at a time (the library is compiled without contraction;
// float32 division and square root compile to correctly rounded sequences), in a fixed order.
//
// Mapping to CDNA4.  Two passes over the source and destination images, both bound by memory: a
// splat (one lane per source pixel: 20 bytes in, one 64-bit atomic minimum on the key of its landing
// pixel) and a resolve (one lane per destination pixel: its key, for empty pixels the eight neighbour
// keys, a 16-byte gather of the winner's RGBA and the outputs).  Two z-buffers are used in turn: the
// resolve empties its pixels in the other one, so the next warp of no larger size needs no fill pass
// (a fill kernel runs only when a buffer is not known to be empty).
// The splat's waves each cover 64 pixels of one row: points of neighbouring pixels land on neighbouring
// keys, and the atomics of a wave are sent as one request per 64-byte segment of keys they touch (a
// device-scope atomic is performed beyond the XCDs' L2 caches, so the request count sets the splat's
// time); a 64 x 1 wave touches about 9 segments after a small move where a 16 x 4 wave touched 12.
// The resolve's blocks cover 16 x 16 pixel tiles so that its neighbour reads stay within a few cache
// lines of keys.
#include <algorithm>
#include <mutex>

#include "internal.h"

namespace raypc {
namespace {

constexpr unsigned long long kEmpty = ~0ull;

// The z-buffer of the allocation-free warp (raypc_warp_noalloc): one per GPU, in the code object's
// own device memory, so that a caller that cannot allocate can still warp.  Host code never uses
// this name as an address (it names the host-side stand-in): warp_scratch() asks the runtime for
// each device's address once and hands that out.
static __device__ __align__(256) unsigned long long scratch[kWarpScratchPixels];
constexpr int kTile = 16;
constexpr int kSplatRow = 64, kSplatRows = 4;  // splat blocks: 64 x 4 pixels, one row per wave

typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float dot3(float a0, float a1, float a2, const float* b) {
    return (a0 * b[0] + a1 * b[1]) + a2 * b[2];
}

__global__ __launch_bounds__(256) void warp_clear_kernel(unsigned long long* __restrict__ keys, size_t n) {
    for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<size_t>(gridDim.x) * blockDim.x)
        keys[i] = kEmpty;
}

__global__ __launch_bounds__(256) void warp_splat_kernel(WarpArgs A) {
    const int px = blockIdx.x * kSplatRow + (threadIdx.x & (kSplatRow - 1));
    const int py = blockIdx.y * kSplatRows + (threadIdx.x / kSplatRow);
    const WarpCamera& S = A.src;
    const WarpCamera& Dc = A.dst;
    if (px >= S.width || py >= S.height) return;
    const uint32_t p = static_cast<uint32_t>(py) * static_cast<uint32_t>(S.width) + static_cast<uint32_t>(px);
    const float d = A.depth[p];

    // the source pixel's ray, as the render casts it (unit direction)
    const float sx = ((static_cast<float>(px) + 0.5f) * S.inv_w2 - 1.0f) * S.sx_scale;
    const float sy = (1.0f - (static_cast<float>(py) + 0.5f) * S.inv_h2) * S.sy_scale;
    const float e0 = (S.fwd[0] + sx * S.right[0]) + sy * S.up[0];
    const float e1 = (S.fwd[1] + sx * S.right[1]) + sy * S.up[1];
    const float e2 = (S.fwd[2] + sx * S.right[2]) + sy * S.up[2];
    const float len = sqrtf((e0 * e0 + e1 * e1) + e2 * e2);
    const float n0 = e0 / len, n1 = e1 / len, n2 = e2 / len;

    // the point relative to the destination eye (a direction for a point at infinity)
    const bool finite = d < INFINITY;
    const float v0 = finite ? (S.eye[0] + d * n0) - Dc.eye[0] : n0;
    const float v1 = finite ? (S.eye[1] + d * n1) - Dc.eye[1] : n1;
    const float v2 = finite ? (S.eye[2] + d * n2) - Dc.eye[2] : n2;
    const float z = dot3(v0, v1, v2, Dc.fwd);
    const float xr = dot3(v0, v1, v2, Dc.right);
    const float yu = dot3(v0, v1, v2, Dc.up);
    const float xn = xr / (z * Dc.sx_scale);
    const float yn = yu / (z * Dc.sy_scale);
    const float fx = (xn + 1.0f) * (0.5f * static_cast<float>(Dc.width));
    const float fy = (1.0f - yn) * (0.5f * static_cast<float>(Dc.height));
    if (!(z > 0.0f && fx >= 0.0f && fx < static_cast<float>(Dc.width) && fy >= 0.0f &&
          fy < static_cast<float>(Dc.height)))
        return;
    const uint32_t tx = static_cast<uint32_t>(floorf(fx)), ty = static_cast<uint32_t>(floorf(fy));
    const float q = finite ? sqrtf((v0 * v0 + v1 * v1) + v2 * v2) : INFINITY;
    // distances are >= 0, so their bit patterns order as the distances do
    const unsigned long long key = (static_cast<unsigned long long>(__float_as_uint(q)) << 32) | p;
    atomicMin(&A.keys[static_cast<size_t>(ty) * Dc.width + tx], key);
}

__global__ __launch_bounds__(256) void warp_resolve_kernel(WarpArgs A) {
    const int tx = blockIdx.x * kTile + (threadIdx.x & (kTile - 1));
    const int ty = blockIdx.y * kTile + (threadIdx.x >> 4);
    const int W = A.dst.width, H = A.dst.height;
    if (tx >= W || ty >= H) return;
    const size_t t = static_cast<size_t>(ty) * W + tx;
    unsigned long long key = A.keys[t];
    if (key == kEmpty) {
        // the farthest landed neighbour: keys + 1 so that 0 means none (keys are below 2^63)
        unsigned long long best = 0;
        for (int dy = -1; dy <= 1; ++dy) {
            const int y = ty + dy;
            if (y < 0 || y >= H) continue;
            for (int dx = -1; dx <= 1; ++dx) {
                const int x = tx + dx;
                if ((dx == 0 && dy == 0) || x < 0 || x >= W) continue;
                const unsigned long long k = A.keys[static_cast<size_t>(y) * W + x];
                if (k != kEmpty) best = max(best, k + 1);
            }
        }
        key = best ? best - 1 : kEmpty;
    }
    f32x4 c = {0.0f, 0.0f, 0.0f, 0.0f};
    float dep = INFINITY;
    int32_t src = -1;
    // a key always names a pixel of this warp's source image, unless another warp raced on the buffer
    if (key != kEmpty && (key & 0xFFFFFFFFull) < A.n_src) {
        src = static_cast<int32_t>(key & 0xFFFFFFFFull);
        const float4 s = A.rgba[src];
        c.x = s.x, c.y = s.y, c.z = s.z, c.w = s.w;
        dep = __uint_as_float(static_cast<uint32_t>(key >> 32));
    }
    reinterpret_cast<f32x4*>(A.out)[t] = c;
    if (A.out_depth) A.out_depth[t] = dep;
    if (A.out_src) A.out_src[t] = src;
    if (A.next_keys) A.next_keys[t] = kEmpty;  // ready for the next warp, which uses the other buffer
}

}  // namespace

hipError_t warp_scratch(int device, unsigned long long** ptr) {
    static std::mutex mu;
    static unsigned long long* addr[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;  // the caller makes `device` current
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[device] = static_cast<unsigned long long*>(p);
    }
    *ptr = addr[device];
    return hipSuccess;
}

hipError_t launch_warp(const WarpArgs& a, hipStream_t s) {
    const size_t n_dst = static_cast<size_t>(a.dst.width) * a.dst.height;
    if (a.clear_keys) {
        const unsigned clear_blocks = static_cast<unsigned>(std::min<size_t>((n_dst + 255) / 256, 8192));
        hipLaunchKernelGGL(warp_clear_kernel, dim3(clear_blocks), dim3(256), 0, s, a.keys, n_dst);
    }
    const dim3 src_grid((a.src.width + kSplatRow - 1) / kSplatRow, (a.src.height + kSplatRows - 1) / kSplatRows);
    hipLaunchKernelGGL(warp_splat_kernel, src_grid, dim3(256), 0, s, a);
    const dim3 dst_grid((a.dst.width + kTile - 1) / kTile, (a.dst.height + kTile - 1) / kTile);
    hipLaunchKernelGGL(warp_resolve_kernel, dst_grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace raypc
