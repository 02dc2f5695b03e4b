// raymarch.hip -- the single-image ray-march launches (plain and counting), whose field count is a
// template argument.  The kernel and the method it implements are in raymarch_impl.h; the batched,
// jittered and depth launches are in raymarch_batch.hip (two translation units, compiled in parallel).
#include "raymarch_impl.h"

namespace raypc {

hipError_t launch_render(const RenderArgs& a, int kind, bool counts, hipStream_t s) {
    return counts ? launch_fixed_kind<true, false, false>(a, kind, s) : launch_fixed_kind<false, false, false>(a, kind, s);
}

}  // namespace raypc

