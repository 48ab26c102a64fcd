// placeholder, replaced below
#include "launch.h"
extern "C" {
int sof_query_workspace_size(int64_t, const sof_camera*, int32_t, const sof_options*, int64_t, int64_t, size_t*, size_t*, size_t*) { return SOF_E_UNSUPPORTED; }
int sof_opacity_query(const sof_gaussians*, const sof_camera*, const sof_camera*, int32_t, const sof_options*, const float*, int64_t, int64_t, float*, void*, size_t, void*, size_t, void*, size_t, hipStream_t) { return SOF_E_UNSUPPORTED; }
}
