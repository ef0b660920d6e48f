// 3D query kernels (placeholder until the 3D path lands).
#include <hip/hip_runtime.h>

#include "gwn_internal.h"

namespace gwn {

struct LaunchTable;
gwn_status launch_query3d(const LaunchTable &, const double *, const int32_t *, double *, uint8_t *, int32_t *,
                          int32_t *, long long *, bool, hipStream_t, std::string &err)
{
    err = "3D queries are not implemented yet";
    return GWN_EUNSUPPORTED;
}

}  // namespace gwn
