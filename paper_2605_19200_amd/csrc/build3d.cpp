// Host preprocessing of a 3D model (placeholder until the 3D path lands).
#include "gwn_internal.h"

namespace gwn {

gwn_status build3d_host(const gwn_patches3d *, const gwn_params *, Model &, std::string &err)
{
    err = "3D models are not implemented yet";
    return GWN_EUNSUPPORTED;
}

void pack3d(const Model &, std::vector<Node3> &, std::vector<Prim3> &) {}

}  // namespace gwn
