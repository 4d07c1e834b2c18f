// Host-side construction of the rasteriser's mesh layout (see mesh.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "b3d_device.hpp"

namespace b3d {

struct MeshLayout {
  std::vector<ClusterDev> clusters;  // [0, n_visible) always drawn; the rest only near the near plane
  std::vector<float4> cverts;        // cluster-local vertex copies
  std::vector<uint2> ctris;          // (local indices a | b << 8 | c << 16, caller's triangle id)
  int n_visible = 0;
  int n_drawn = 0, n_hidden = 0, n_dropped = 0;
};

MeshLayout build_mesh_layout(const float* verts, int V, const int* tris, int T);

}  // namespace b3d
