// Octree refinement (Sec. 3.2): placeholder until the device implementation lands.
#include <hip/hip_runtime.h>

#include "dot_internal.h"

namespace dot {

int refine_tree(dot_tree&, const float*, const dot_refine_params&, dot_refine_stats*, hipStream_t) {
    return fail(DOT_EUNSUPPORTED, "dot_refine: not implemented yet");
}

}  // namespace dot
