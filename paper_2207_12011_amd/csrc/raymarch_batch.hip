// raymarch_batch.hip -- ray-march launches besides the plain single-image render: batched serving
// steps (tiles of many requests in one launch), jittered progressive passes and depth renders.  Every
// launch runs the kernel whose brushed-field count is a template argument (the scheduler groups a
// step's tiles by kernel kind and field count), except with coordinate axes, whose run-time count
// variant carries their test.
#include "raymarch_impl.h"

namespace raypc {
namespace {

// Batched launch: item j marches one tile of one request, as the ranges in the kernel arguments
// say.  Tiles of many requests (different images, brushes, levels and transfer functions, one
// kernel kind and field count) share a launch; each tile runs exactly the code path of a
// single-request render.  Chunks of 64 consecutive items (one super-tile of a request, as the
// scheduler lists them) are dealt round-robin over the 8 XCDs; the grid is padded to whole rounds of
// 8 chunks.  Blocks are single waves (4 x 4 pixels).  WIDE: 64-bit record offsets (record fields of 4 GiB and more).
template <int K, int NB, bool WIDE>
__global__ __launch_bounds__(64) void raymarch_batch_kernel(
    const RenderArgs* __restrict__ descs, BatchRanges R) {
    __shared__ float4 s_tf[256];
    const int xcd = blockIdx.x & 7, p = blockIdx.x >> 3;
    const int j = ((p / kSuperTiles) * 8 + xcd) * kSuperTiles + p % kSuperTiles;
    if (j >= R.end[R.n - 1]) return;  // padding block
    int r = 0;
    while (j >= R.end[r]) ++r;
    const int tile = R.first[r] + j - (r ? R.end[r - 1] : 0);
    const RenderArgs& A = descs[R.slot[r]];
    int bx, by;
    tile_coords(tile, A.blocks_x, A.n_blocks / A.blocks_x, bx, by);
    march_tile<K, NB, false, false, false, WIDE, 1>(A, &A, bx, by, s_tf);
}

template <int K, bool WIDE>
hipError_t launch_batch_nb(const RenderArgs* descs, const BatchRanges& R, int nb_class, dim3 grid, hipStream_t s) {
    const dim3 block(64);
    switch (nb_class) {
        case kRuntimeNB: hipLaunchKernelGGL((raymarch_batch_kernel<K, kRuntimeNB, WIDE>), grid, block, 0, s, descs, R); break;
        case 0: hipLaunchKernelGGL((raymarch_batch_kernel<K, 0, WIDE>), grid, block, 0, s, descs, R); break;
        case 1: hipLaunchKernelGGL((raymarch_batch_kernel<K, 1, WIDE>), grid, block, 0, s, descs, R); break;
        case 2: hipLaunchKernelGGL((raymarch_batch_kernel<K, 2, WIDE>), grid, block, 0, s, descs, R); break;
        case 3: hipLaunchKernelGGL((raymarch_batch_kernel<K, 3, WIDE>), grid, block, 0, s, descs, R); break;
        case 4: hipLaunchKernelGGL((raymarch_batch_kernel<K, 4, WIDE>), grid, block, 0, s, descs, R); break;
        case 5: hipLaunchKernelGGL((raymarch_batch_kernel<K, 5, WIDE>), grid, block, 0, s, descs, R); break;
        case 6: hipLaunchKernelGGL((raymarch_batch_kernel<K, 6, WIDE>), grid, block, 0, s, descs, R); break;
        case 7: hipLaunchKernelGGL((raymarch_batch_kernel<K, 7, WIDE>), grid, block, 0, s, descs, R); break;
        default: hipLaunchKernelGGL((raymarch_batch_kernel<K, 8, WIDE>), grid, block, 0, s, descs, R); break;
    }
    return hipGetLastError();
}

}  // namespace

int batch_nb_class(const RenderArgs& a) { return a.coord_mask ? kRuntimeNB : a.n_brushed; }

bool batch_wide(const RenderArgs& a, int kind) { return records_of(kind) && !narrow_records(a); }

hipError_t launch_render_batch(const RenderArgs* descs, const BatchRanges& R, int kind, int nb_class, bool wide,
                               hipStream_t s) {
    if (R.n <= 0 || R.n > kMaxRanges || R.end[R.n - 1] <= 0) return hipSuccess;
    constexpr int kRound = 8 * kSuperTiles;
    const dim3 grid((R.end[R.n - 1] + kRound - 1) / kRound * kRound);
    switch (kind) {
        case kKindF32: return launch_batch_nb<kKindF32, true>(descs, R, nb_class, grid, s);
        case kKindF16: return launch_batch_nb<kKindF16, true>(descs, R, nb_class, grid, s);
        case kKindU8: return launch_batch_nb<kKindU8, true>(descs, R, nb_class, grid, s);
        case kKindF32Rec:
            return wide ? launch_batch_nb<kKindF32Rec, true>(descs, R, nb_class, grid, s)
                        : launch_batch_nb<kKindF32Rec, false>(descs, R, nb_class, grid, s);
        case kKindF16Rec:
            return wide ? launch_batch_nb<kKindF16Rec, true>(descs, R, nb_class, grid, s)
                        : launch_batch_nb<kKindF16Rec, false>(descs, R, nb_class, grid, s);
        default:
            return wide ? launch_batch_nb<kKindU8Rec, true>(descs, R, nb_class, grid, s)
                        : launch_batch_nb<kKindU8Rec, false>(descs, R, nb_class, grid, s);
    }
}

hipError_t launch_render_jittered(const RenderArgs& a, int kind, bool counts, hipStream_t s) {
    return counts ? launch_fixed_kind<true, true, false>(a, kind, s) : launch_fixed_kind<false, true, false>(a, kind, s);
}

hipError_t launch_render_depth(const RenderArgs& a, int kind, hipStream_t s) {
    return launch_fixed_kind<false, false, true>(a, kind, s);
}

}  // namespace raypc
