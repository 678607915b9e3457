// The obstacle of the rectangle (Sec. 2.3 on the faces of solid cells): the
// host builds, from the problem's solid mask, the list of obstacle faces and
// a neighbour map; the kernels of the two-dimensional step and of the
// full-tensor step read them through Obs2.
//
// Faces of the rectangle are numbered b = [x_lo: ny][x_hi: ny][y_lo: nx]
// [y_hi: nx]; obstacle faces follow, b = nface + i, i in the order of gas
// cells (index ascending) and, within a cell, of the solid neighbour's
// direction -x, +x, -y, +y (k = 0..3, the face's outward normal from the gas
// side, the same numbering as the rectangle's faces).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "internal.hpp"

namespace blr {

struct Obs2 {
  const int* face;          // 2 per obstacle face: gas cell p, direction k
  const int* nbmap;         // 4 per cell: obstacle face index b, or -1
  const uint8_t* solid;     // nx ny bytes; null: no obstacle
  const double* f;          // the obstacle walls' Maxwellian shape
  int nface;                // faces of the rectangle, 2 (nx + ny)
  int nob;                  // obstacle faces
  __device__ __forceinline__ bool is_solid(long p) const { return solid && solid[p]; }
  // obstacle face of gas cell p towards direction dir (0 -x, 1 +x, 2 -y, 3 +y), or -1
  __device__ __forceinline__ int towards(long p, int dir) const {
    return nbmap ? nbmap[p * 4 + dir] : -1;
  }
};

struct ObstacleHost {
  std::vector<int> face;       // 2 per face
  std::vector<int> nbmap;      // 4 per cell
  std::vector<uint8_t> solid;  // nx ny
  int nob = 0;
  bool any = false;
  uint64_t hash = 0;           // FNV-1a of the mask (graph keys)
};

inline ObstacleHost obstacle_host(const blr_problem* pb) {
  ObstacleHost o;
  if (pb->ny < 2 || !pb->solid) return o;
  const int nx = pb->nx, ny = pb->ny, nface = 2 * (nx + ny);
  const long nc = (long)nx * ny;
  o.solid.assign(pb->solid, pb->solid + nc);
  uint64_t h = 1469598103934665603ull;
  for (long p = 0; p < nc; ++p) {
    o.solid[p] = o.solid[p] ? 1 : 0;
    h = (h ^ o.solid[p]) * 1099511628211ull;
    o.any = o.any || o.solid[p];
  }
  o.hash = h;
  if (!o.any) return o;
  o.nbmap.assign((size_t)nc * 4, -1);
  for (long p = 0; p < nc; ++p) {
    if (o.solid[p]) continue;
    const int ix = (int)(p / ny), iy = (int)(p % ny);
    const int jx[4] = {ix - 1, ix + 1, ix, ix};
    const int jy[4] = {iy, iy, iy - 1, iy + 1};
    for (int k = 0; k < 4; ++k) {
      if (jx[k] < 0 || jx[k] >= nx || jy[k] < 0 || jy[k] >= ny) continue;
      if (!o.solid[(long)jx[k] * ny + jy[k]]) continue;
      o.nbmap[p * 4 + k] = nface + o.nob;
      o.face.push_back((int)p);
      o.face.push_back(k);
      ++o.nob;
    }
  }
  return o;
}

}  // namespace blr
