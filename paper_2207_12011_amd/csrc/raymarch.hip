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
// Mapping to CDNA4.  Four lanes share a ray and evaluate four consecutive
// samples of it at once (binary16 records: two such groups per step, each lane
// taking samples j and j + 4, their loads issued together); a wave64 covers a
// 4 x 4 pixel tile, so the samples it fetches per step form a compact cluster
// of a few voxels on a side, which the brick layout (4^3 sub-bricks per cache
// line for binary16) serves from a handful of cache lines.  Each group of four
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
// sits in LDS.  This file holds the single-image launches, whose field count is a template argument;
// raymarch_batch.hip holds those that read it at run time.
#include "raymarch_impl.h"

namespace raypc {

hipError_t launch_render(const RenderArgs& a, int kind, bool counts, hipStream_t s) {
    return counts ? launch_fixed_kind<true, false, false>(a, kind, s) : launch_fixed_kind<false, false, false>(a, kind, s);
}

}  // namespace raypc

