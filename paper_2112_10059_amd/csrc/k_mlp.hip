// Learned leaf selector (placeholder until the network kernels land).
#include <hip/hip_runtime.h>

#include "ph_internal.h"

namespace ph {

void selector_apply(Plan &, hipStream_t) { throw Error{PH_EUNSUPPORTED, "learned selector not built yet"}; }
void launch_mlp_forward(const float *, const float *, int64_t, float *, int, hipStream_t)
{
    throw Error{PH_EUNSUPPORTED, "mlp forward not built yet"};
}
void launch_mlp_backward(const float *, const float *, const float *, float, int64_t, float *, float *, hipStream_t)
{
    throw Error{PH_EUNSUPPORTED, "mlp backward not built yet"};
}
void launch_adam(float *, float *, float *, const float *, int64_t, float, float, float, float, int64_t, hipStream_t)
{
    throw Error{PH_EUNSUPPORTED, "adam not built yet"};
}

}  // namespace ph

extern "C" ph_status ph_selector_features(ph_plan *, float *, int64_t, int64_t *, void *)
{
    ph::set_last_error("selector features not built yet");
    return PH_EUNSUPPORTED;
}
