// Host-side device layout of a triangle mesh for the rasteriser.
//
// The rasteriser walks a mesh cluster by cluster: each cluster holds up to
// kClusterPrims primitives of one orientation class that are close in space,
// a bounding sphere and a cone bounding its face normals.  A primitive is one
// triangle or a quad: two triangles (a, b, c) and (a, c, d) that share the
// edge a-c with opposite directions (consistent winding), lie in one plane
// and form a convex quadrilateral -- the two halves of a voxel face.  One lane
// walks the quad's pixel box once for both triangles; each triangle is still
// tested against its own three edges, and keeps its own id.  Per hypothesis a cluster is
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
  // 5. primitives: pair triangles into convex planar quads (within the drawn
  //    set and within the hidden set), the rest stay single
  auto pos = [&](int p, int k) { return (double)verts[3 * pos_first[p] + k]; };
  std::unordered_map<uint64_t, std::vector<int>> by_edge;  // directed position edge -> triangles
  for (int t = 0; t < T; ++t) {
    if (cls[t] == 2) continue;
    for (int k = 0; k < 3; ++k) {
      const uint32_t i = (uint32_t)pid[tris[3 * t + k]], j = (uint32_t)pid[tris[3 * t + (k + 1) % 3]];
      by_edge[((uint64_t)i << 32) | j].push_back(t);
    }
  }
  struct Prim {
    int p[4];       // position ids a, b, c, d (d = c for a single triangle)
    int id1, id2;   // caller's triangle ids (id2 = -1: single)
    uint64_t key;
  };
  std::vector<int> mate((size_t)T, -1);
  std::vector<Prim> prims[2];  // 0 drawn, 1 hidden
  auto convex_quad = [&](int a, int b, int c, int d, const double* n) {
    // planar convex iff b and d lie on opposite sides of a-c and a and c on opposite sides of b-d
    auto side = [&](int o, int e, int q) {
      const double u[3] = {pos(e, 0) - pos(o, 0), pos(e, 1) - pos(o, 1), pos(e, 2) - pos(o, 2)};
      const double w[3] = {pos(q, 0) - pos(o, 0), pos(q, 1) - pos(o, 1), pos(q, 2) - pos(o, 2)};
      const double x[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]};
      return x[0] * n[0] + x[1] * n[1] + x[2] * n[2];
    };
    return side(a, c, b) * side(a, c, d) < 0.0 && side(b, d, a) * side(b, d, c) < 0.0;
  };
  for (int t = 0; t < T; ++t) {
    if (cls[t] == 2 || mate[t] >= 0) continue;
    const int pt[3] = {pid[tris[3 * t]], pid[tris[3 * t + 1]], pid[tris[3 * t + 2]]};
    int found = -1, fk = 0;
    // longest edge first: a voxel face's two halves share its diagonal
    int ord[3] = {0, 1, 2};
    double len2[3];
    for (int k = 0; k < 3; ++k) {
      len2[k] = 0.0;
      for (int a2 = 0; a2 < 3; ++a2) {
        const double d = pos(pt[(k + 1) % 3], a2) - pos(pt[k], a2);
        len2[k] += d * d;
      }
    }
    std::stable_sort(ord, ord + 3, [&](int x, int y) { return len2[x] > len2[y]; });
    for (int oi = 0; oi < 3 && found < 0; ++oi) {
      const int k = ord[oi];
      // the partner holds the edge p_{k+1} -> p_k
      const uint64_t rev = ((uint64_t)(uint32_t)pt[(k + 1) % 3] << 32) | (uint32_t)pt[k];
      auto it = by_edge.find(rev);
      if (it == by_edge.end()) continue;
      for (int u : it->second) {
        if (u == t || mate[u] >= 0 || cls[u] != cls[t] || (order_key[u] >> 32) != (order_key[t] >> 32)) continue;
        const double dn = unit[3 * t] * unit[3 * u] + unit[3 * t + 1] * unit[3 * u + 1] + unit[3 * t + 2] * unit[3 * u + 2];
        if (!(dn > 1.0 - 1e-9)) continue;
        int far = -1;
        for (int m2 = 0; m2 < 3; ++m2) {
          const int q = pid[tris[3 * u + m2]];
          if (q != pt[k] && q != pt[(k + 1) % 3]) far = q;
        }
        // t = (a, b, c) with the shared edge c -> a: a = p_{k+1}, b = p_{k+2}, c = p_k
        const int qa = pt[(k + 1) % 3], qb = pt[(k + 2) % 3], qc = pt[k];
        if (far < 0 || !convex_quad(qa, qb, qc, far, &unit[3 * t])) continue;
        found = u;
        fk = k;
        break;
      }
    }
    Prim pr;
    if (found >= 0) {
      mate[t] = found;
      mate[found] = t;
      pr.p[0] = pt[(fk + 1) % 3];
      pr.p[1] = pt[(fk + 2) % 3];
      pr.p[2] = pt[fk];
      for (int m2 = 0; m2 < 3; ++m2) {
        const int q = pid[tris[3 * found + m2]];
        if (q != pr.p[0] && q != pr.p[2]) pr.p[3] = q;
      }
      pr.id1 = t;
      pr.id2 = found;
      ++L.n_quads;
    } else {
      pr.p[0] = pt[0];
      pr.p[1] = pt[1];
      pr.p[2] = pt[2];
      pr.p[3] = pt[2];
      pr.id1 = t;
      pr.id2 = -1;
    }
    pr.key = order_key[t];
    prims[cls[t]].push_back(pr);
  }
  // 6. clusters: drawn primitives first, then hidden ones
  auto emit = [&](std::vector<Prim>& ps) {
    std::stable_sort(ps.begin(), ps.end(), [](const Prim& x, const Prim& y) { return x.key < y.key; });
    size_t i = 0;
    while (i < ps.size()) {
      ClusterDev c{};
      c.pfirst = (int)L.pids.size();
      const uint64_t cls_dir = ps[i].key >> 32;
      double axis[3] = {0, 0, 0};
      double blo[3] = {1e300, 1e300, 1e300}, bhi[3] = {-1e300, -1e300, -1e300};
      size_t j = i;
      for (; j < ps.size() && c.np < kClusterPrims && (ps[j].key >> 32) == cls_dir; ++j) {
        const Prim& pr = ps[j];
        for (int k = 0; k < 4; ++k) {
          L.pverts.push_back(make_float4((float)pos(pr.p[k], 0), (float)pos(pr.p[k], 1), (float)pos(pr.p[k], 2), 0.0f));
          for (int a2 = 0; a2 < 3; ++a2) {
            blo[a2] = std::min(blo[a2], pos(pr.p[k], a2));
            bhi[a2] = std::max(bhi[a2], pos(pr.p[k], a2));
          }
        }
        L.pids.push_back(make_uint2((uint32_t)pr.id1, pr.id2 < 0 ? kNoTri : (uint32_t)pr.id2));
        for (int a2 = 0; a2 < 3; ++a2) axis[a2] += unit[3 * pr.id1 + a2] + (pr.id2 >= 0 ? unit[3 * pr.id2 + a2] : 0.0);
        ++c.np;
      }
      double ctr[3], rad = 0.0;
      for (int a2 = 0; a2 < 3; ++a2) ctr[a2] = 0.5 * (blo[a2] + bhi[a2]);
      for (int v = 0; v < 4 * c.np; ++v) {
        const float4 q = L.pverts[4 * (size_t)c.pfirst + v];
        const double d2 = (q.x - ctr[0]) * (q.x - ctr[0]) + (q.y - ctr[1]) * (q.y - ctr[1]) +
                          (q.z - ctr[2]) * (q.z - ctr[2]);
        rad = std::max(rad, std::sqrt(d2));
      }
      c.sphere = make_float4((float)ctr[0], (float)ctr[1], (float)ctr[2], (float)(rad * (1.0 + 1e-5) + 1e-6));
      const double al = std::sqrt(axis[0] * axis[0] + axis[1] * axis[1] + axis[2] * axis[2]);
      double cos_a = 1.0;
      bool ok = al > 0;
      for (size_t k = i; k < j && ok; ++k) {
        for (int h2 = 0; h2 < 2; ++h2) {
          const int t = h2 == 0 ? ps[k].id1 : ps[k].id2;
          if (t < 0) continue;
          if (unit[3 * t] == 0 && unit[3 * t + 1] == 0 && unit[3 * t + 2] == 0) ok = false;
          const double d = (unit[3 * t] * axis[0] + unit[3 * t + 1] * axis[1] + unit[3 * t + 2] * axis[2]) / al;
          cos_a = std::min(cos_a, d);
        }
      }
      // half-angle of the normal cone, widened slightly; > pi/2 disables culling
      const double alpha = ok ? std::acos(std::max(-1.0, std::min(1.0, cos_a))) + 1e-4 : 4.0;
      c.cone = ok ? make_float4((float)(axis[0] / al), (float)(axis[1] / al), (float)(axis[2] / al), (float)alpha)
                  : make_float4(0.0f, 0.0f, 1.0f, 4.0f);
      L.clusters.push_back(c);
      i = j;
    }
  };
  emit(prims[0]);
  L.n_visible = (int)L.clusters.size();
  emit(prims[1]);
  for (int t = 0; t < T; ++t) {
    if (cls[t] == 0) ++L.n_drawn;
    if (cls[t] == 1) ++L.n_hidden;
  }
  L.n_dropped = T - L.n_drawn - L.n_hidden;
  return L;
}

}  // namespace b3d
