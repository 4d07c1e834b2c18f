// Host-side construction of the rasteriser's mesh layout (see mesh.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "b3d_device.hpp"

namespace b3d {

struct MeshLayout {
  std::vector<ClusterDev> clusters;  // [0, n_visible) always drawn; the rest only near the near plane
  std::vector<float4> pverts;        // 4 object-frame corners (a, b, c, d) per primitive
  std::vector<uint2> pids;           // (id of triangle (a, b, c), id of triangle (a, c, d) or kNoTri)
  int n_visible = 0;
  int n_drawn = 0, n_hidden = 0, n_dropped = 0, n_quads = 0;
};

MeshLayout build_mesh_layout(const float* verts, int V, const int* tris, int T);

}  // namespace b3d
