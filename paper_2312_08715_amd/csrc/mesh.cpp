// Host-side device layout of a triangle mesh for the rasteriser.
//
// The rasteriser walks a mesh cluster by cluster: each cluster holds up to
// kClusterTris triangles of one orientation class that are close in space,
// with its own copy of the (deduplicated) vertices they use, a bounding
// sphere and a cone bounding its face normals.  Per hypothesis a cluster is
// skipped as a whole when its cone and sphere show that every triangle in it
// faces away from the camera, or when its sphere misses the pixels being
// drawn.  Two sets of triangles that can never be the nearest surface for a
// camera outside the object are moved to trailing clusters drawn only when
// the object reaches the near plane:
//   * pairs of triangles with the same three vertex positions and opposite
//     winding that lie on two different closed components (the touching
//     faces of adjacent voxels): a ray that crosses such a face is already
//     inside one of the two solids, so it entered that solid through a nearer
//     camera-facing face;
// and triangles with a repeated vertex position (zero area, never drawn) are
// dropped.  Triangle ids stay the caller's row indices.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <unordered_map>
#include <vector>

#include "b3d_mesh_layout.hpp"

namespace b3d {

namespace {

struct PosKey {
  uint32_t x, y, z;
  bool operator==(const PosKey& o) const { return x == o.x && y == o.y && z == o.z; }
};
struct PosHash {
  size_t operator()(const PosKey& k) const {
    uint64_t h = k.x * 0x9E3779B97F4A7C15ull;
    h ^= (k.y + 0x632BE59BD9B4E019ull) + (h << 6) + (h >> 2);
    h ^= (k.z + 0xD6E8FEB86659FD93ull) + (h << 6) + (h >> 2);
    return (size_t)h;
  }
};

uint32_t bits(float f) {
  if (f == 0.0f) f = 0.0f;  // one key for +0 and -0
  uint32_t u;
  std::memcpy(&u, &f, 4);
  return u;
}

struct Tri3Key {
  int a, b, c;  // sorted position ids
  bool operator==(const Tri3Key& o) const { return a == o.a && b == o.b && c == o.c; }
};
struct Tri3Hash {
  size_t operator()(const Tri3Key& k) const {
    uint64_t h = (uint64_t)(uint32_t)k.a * 0x9E3779B97F4A7C15ull;
    h ^= (uint64_t)(uint32_t)k.b * 0xC2B2AE3D27D4EB4Full + (h << 6) + (h >> 2);
    h ^= (uint64_t)(uint32_t)k.c * 0x165667B19E3779F9ull + (h << 6) + (h >> 2);
    return (size_t)h;
  }
};

int find(std::vector<int>& p, int x) {
  while (p[x] != x) {
    p[x] = p[p[x]];
    x = p[x];
  }
  return x;
}

uint32_t spread10(uint32_t v) {
  v &= 1023u;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

}  // namespace

MeshLayout build_mesh_layout(const float* verts, int V, const int* tris, int T) {
  MeshLayout L;
  // 1. positions: deduplicate exactly equal coordinates
  std::unordered_map<PosKey, int, PosHash> pos_of;
  std::vector<int> pid((size_t)V);
  std::vector<int> pos_first;  // original vertex index of each position
  for (int i = 0; i < V; ++i) {
    PosKey k{bits(verts[3 * i]), bits(verts[3 * i + 1]), bits(verts[3 * i + 2])};
    auto it = pos_of.find(k);
    if (it == pos_of.end()) {
      pid[i] = (int)pos_first.size();
      pos_of.emplace(k, pid[i]);
      pos_first.push_back(i);
    } else {
      pid[i] = it->second;
    }
  }
  // 2. closed components over the caller's vertex indices
  std::vector<int> parent((size_t)V);
  std::iota(parent.begin(), parent.end(), 0);
  for (int t = 0; t < T; ++t) {
    const int a = find(parent, tris[3 * t]), b = find(parent, tris[3 * t + 1]), c = find(parent, tris[3 * t + 2]);
    parent[b] = a;
    parent[find(parent, c)] = a;
  }
  std::unordered_map<uint64_t, int> edge_count;  // directed edge i->j
  edge_count.reserve((size_t)T * 3);
  for (int t = 0; t < T; ++t)
    for (int k = 0; k < 3; ++k) {
      const uint32_t i = (uint32_t)tris[3 * t + k], j = (uint32_t)tris[3 * t + (k + 1) % 3];
      edge_count[((uint64_t)i << 32) | j] += 1;
    }
  std::unordered_map<int, bool> comp_closed;
  for (int t = 0; t < T; ++t) {
    const int root = find(parent, tris[3 * t]);
    bool ok = true;
    for (int k = 0; k < 3; ++k) {
      const uint32_t i = (uint32_t)tris[3 * t + k], j = (uint32_t)tris[3 * t + (k + 1) % 3];
      auto f = edge_count.find(((uint64_t)i << 32) | j);
      auto r = edge_count.find(((uint64_t)j << 32) | i);
      ok = ok && f != edge_count.end() && f->second == 1 && r != edge_count.end() && r->second == 1;
    }
    auto it = comp_closed.find(root);
    if (it == comp_closed.end())
      comp_closed.emplace(root, ok);
    else
      it->second = it->second && ok;
  }
  // 3. classify triangles: dropped (repeated position), hidden pair, drawn
  std::vector<int8_t> cls((size_t)T, 0);  // 0 drawn, 1 hidden pair, 2 dropped
  std::unordered_map<Tri3Key, std::vector<int>, Tri3Hash> by_key;
  for (int t = 0; t < T; ++t) {
    const int a = pid[tris[3 * t]], b = pid[tris[3 * t + 1]], c = pid[tris[3 * t + 2]];
    if (a == b || b == c || a == c) {
      cls[t] = 2;
      continue;
    }
    int s[3] = {a, b, c};
    std::sort(s, s + 3);
    by_key[Tri3Key{s[0], s[1], s[2]}].push_back(t);
  }
  for (auto& kv : by_key) {
    std::vector<int>& ts = kv.second;
    if (ts.size() < 2) continue;
    std::sort(ts.begin(), ts.end());
    // orientation: the cyclic order of the position ids, rotated to start at the smallest
    auto orient = [&](int t) {
      int a = pid[tris[3 * t]], b = pid[tris[3 * t + 1]], c = pid[tris[3 * t + 2]];
      while (a > b || a > c) {
        const int x = a;
        a = b;
        b = c;
        c = x;
      }
      return b < c ? 0 : 1;
    };
    std::vector<int> even, odd;
    for (int t : ts) (orient(t) == 0 ? even : odd).push_back(t);
    std::vector<bool> used_odd(odd.size(), false);
    for (int te : even) {
      const int ce = find(parent, tris[3 * te]);
      if (!comp_closed[ce]) continue;
      for (size_t j = 0; j < odd.size(); ++j) {
        if (used_odd[j]) continue;
        const int co = find(parent, tris[3 * odd[j]]);
        if (co == ce || !comp_closed[co]) continue;
        used_odd[j] = true;
        cls[te] = 1;
        cls[odd[j]] = 1;
        break;
      }
    }
  }
  // 4. orientation class (nearest of 26 directions) and Morton code of the centroid
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int i = 0; i < V; ++i)
    for (int k = 0; k < 3; ++k) {
      lo[k] = std::min(lo[k], (double)verts[3 * i + k]);
      hi[k] = std::max(hi[k], (double)verts[3 * i + k]);
    }
  std::vector<double> unit((size_t)T * 3, 0.0);
  std::vector<uint64_t> order_key((size_t)T);
  double dirs[26][3];
  int nd = 0;
  for (int x = -1; x <= 1; ++x)
    for (int y = -1; y <= 1; ++y)
      for (int z = -1; z <= 1; ++z) {
        if (!x && !y && !z) continue;
        const double n = std::sqrt((double)(x * x + y * y + z * z));
        dirs[nd][0] = x / n;
        dirs[nd][1] = y / n;
        dirs[nd][2] = z / n;
        ++nd;
      }
  for (int t = 0; t < T; ++t) {
    const float* v0 = verts + 3 * tris[3 * t];
    const float* v1 = verts + 3 * tris[3 * t + 1];
    const float* v2 = verts + 3 * tris[3 * t + 2];
    const double e1[3] = {(double)v1[0] - v0[0], (double)v1[1] - v0[1], (double)v1[2] - v0[2]};
    const double e2[3] = {(double)v2[0] - v0[0], (double)v2[1] - v0[1], (double)v2[2] - v0[2]};
    double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    const double len = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    int best = 0;
    if (len > 0) {
      double bd = -2.0;
      for (int k = 0; k < 3; ++k) unit[3 * t + k] = n[k] / len;
      for (int d = 0; d < nd; ++d) {
        const double dd = unit[3 * t] * dirs[d][0] + unit[3 * t + 1] * dirs[d][1] + unit[3 * t + 2] * dirs[d][2];
        if (dd > bd) {
          bd = dd;
          best = d;
        }
      }
    }
    uint32_t q[3];
    for (int k = 0; k < 3; ++k) {
      const double cen = ((double)v0[k] + v1[k] + v2[k]) / 3.0;
      const double span = hi[k] - lo[k];
      q[k] = span > 0 ? (uint32_t)std::min(1023.0, std::max(0.0, (cen - lo[k]) / span * 1023.0)) : 0u;
    }
    const uint64_t morton = spread10(q[0]) | (spread10(q[1]) << 1) | (spread10(q[2]) << 2);
    order_key[t] = ((uint64_t)best << 32) | morton;
  }
  // 5. clusters: drawn triangles first, then hidden pairs
  auto emit = [&](std::vector<int>& ids) {
    std::stable_sort(ids.begin(), ids.end(), [&](int a, int b) { return order_key[a] < order_key[b]; });
    size_t i = 0;
    std::vector<int> stamp_local;
    std::unordered_map<int, int> local;
    while (i < ids.size()) {
      ClusterDev c{};
      c.vfirst = (int)L.cverts.size();
      c.tfirst = (int)L.ctris.size();
      local.clear();
      const uint64_t cls_dir = order_key[ids[i]] >> 32;
      double axis[3] = {0, 0, 0};
      double blo[3] = {1e300, 1e300, 1e300}, bhi[3] = {-1e300, -1e300, -1e300};
      size_t j = i;
      for (; j < ids.size(); ++j) {
        const int t = ids[j];
        if ((order_key[t] >> 32) != cls_dir || c.nt == kClusterTris) break;
        int fresh = 0;
        for (int k = 0; k < 3; ++k) {
          const int p = pid[tris[3 * t + k]];
          bool seen = local.count(p) > 0;
          for (int m = 0; m < k; ++m) seen = seen || pid[tris[3 * t + m]] == p;
          fresh += seen ? 0 : 1;
        }
        if (c.nv + fresh > kClusterVerts) break;
        uint32_t packed = 0;
        for (int k = 0; k < 3; ++k) {
          const int p = pid[tris[3 * t + k]];
          auto it = local.find(p);
          int li;
          if (it == local.end()) {
            li = c.nv++;
            local.emplace(p, li);
            const float* pv = verts + 3 * pos_first[p];
            L.cverts.push_back(make_float4(pv[0], pv[1], pv[2], 0.0f));
            for (int a = 0; a < 3; ++a) {
              blo[a] = std::min(blo[a], (double)pv[a]);
              bhi[a] = std::max(bhi[a], (double)pv[a]);
            }
          } else {
            li = it->second;
          }
          packed |= (uint32_t)li << (8 * k);
        }
        L.ctris.push_back(make_uint2(packed, (uint32_t)t));
        for (int a = 0; a < 3; ++a) axis[a] += unit[3 * t + a];
        ++c.nt;
      }
      double ctr[3], rad = 0.0;
      for (int a = 0; a < 3; ++a) ctr[a] = 0.5 * (blo[a] + bhi[a]);
      for (int v = 0; v < c.nv; ++v) {
        const float4 p = L.cverts[(size_t)c.vfirst + v];
        const double d2 = (p.x - ctr[0]) * (p.x - ctr[0]) + (p.y - ctr[1]) * (p.y - ctr[1]) +
                          (p.z - ctr[2]) * (p.z - ctr[2]);
        rad = std::max(rad, std::sqrt(d2));
      }
      c.sphere = make_float4((float)ctr[0], (float)ctr[1], (float)ctr[2], (float)(rad * (1.0 + 1e-5) + 1e-6));
      const double al = std::sqrt(axis[0] * axis[0] + axis[1] * axis[1] + axis[2] * axis[2]);
      double cos_a = 1.0;
      bool ok = al > 0;
      for (size_t k = i; k < j && ok; ++k) {
        const int t = ids[k];
        const double d = (unit[3 * t] * axis[0] + unit[3 * t + 1] * axis[1] + unit[3 * t + 2] * axis[2]) / al;
        if (unit[3 * t] == 0 && unit[3 * t + 1] == 0 && unit[3 * t + 2] == 0) ok = false;
        cos_a = std::min(cos_a, d);
      }
      // half-angle of the normal cone, widened slightly; > pi/2 disables culling
      const double alpha = ok ? std::acos(std::max(-1.0, std::min(1.0, cos_a))) + 1e-4 : 4.0;
      c.cone = ok ? make_float4((float)(axis[0] / al), (float)(axis[1] / al), (float)(axis[2] / al), (float)alpha)
                  : make_float4(0.0f, 0.0f, 1.0f, 4.0f);
      L.clusters.push_back(c);
      i = j;
    }
  };
  std::vector<int> drawn, hidden;
  for (int t = 0; t < T; ++t) {
    if (cls[t] == 0) drawn.push_back(t);
    if (cls[t] == 1) hidden.push_back(t);
  }
  emit(drawn);
  L.n_visible = (int)L.clusters.size();
  emit(hidden);
  L.n_drawn = (int)drawn.size();
  L.n_hidden = (int)hidden.size();
  L.n_dropped = T - L.n_drawn - L.n_hidden;
  return L;
}

}  // namespace b3d
