// axf_batch.hip -- batched launches (placeholder entry points).
#include "axf_internal.hpp"

using namespace axf;

struct axf_batch {
    int dummy;
};

extern "C" {

axf_status axf_batch_create(const axf_params *, int32_t, const axf_problem *, void *, axf_batch **out)
{
    if (out) *out = nullptr;
    set_error("batched launches are not available in this build");
    return AXF_ERR_UNSUPPORTED;
}
axf_status axf_batch_launch(axf_batch *, void *)
{
    set_error("batched launches are not available in this build");
    return AXF_ERR_UNSUPPORTED;
}
axf_status axf_batch_launch_plain(axf_batch *, void *)
{
    set_error("batched launches are not available in this build");
    return AXF_ERR_UNSUPPORTED;
}
axf_status axf_batch_problem_depth(const axf_batch *, int32_t, int32_t *)
{
    set_error("batched launches are not available in this build");
    return AXF_ERR_UNSUPPORTED;
}
void axf_batch_destroy(axf_batch *b) { delete b; }
}
