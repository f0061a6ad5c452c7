// occlusion.hpp -- exact (FP64) test of a straight leg against the scene's
// triangles through the FP32 BVH, shared by the image-method path rebuild and
// the edge-diffraction paths.
#pragma once

#include "sbr_device.hpp"
#include "sbr_internal.hpp"

namespace sbr {

// Any triangle outside face groups ga, gb crossing the open leg a -> b at
// s in (1e-9, 1 - 1e-9), with inclusive barycentric margins of 1e-9 (the same
// margin as the face tests, so that a leg along a crack between two triangles
// of one blocker is still blocked).  SP: any parameter block with the scene
// fields used below (BVH nodes and root box in a frame centred on (cx, cy,
// cz), FP32 leaves with their original ids and groups, FP64 triangles, and
// the oversized triangles kept out of the tree).  stk: STACK entries with a
// stride of one wave (the caller's LDS slice for this lane).
template <int STACK, class SP>
__device__ bool leg_blocked(const SP& P, int32_t* stk, d3 a, d3 b, int ga, int gb) {
  if (!P.has_bvh && P.n_big == 0) return false;
  const d3 D = b - a;
  const d3 ac = a - mk3(P.cx, P.cy, P.cz);
  auto inv1 = [](double v) { return 1.0 / (fabs(v) > 1e-300 ? v : copysign(1e-300, v)); };
  const d3 inv = mk3(inv1(D.x), inv1(D.y), inv1(D.z));
  auto box_hit = [&](double lx, double ly, double lz, double hx, double hy, double hz) {
    const double t0x = (lx - ac.x) * inv.x, t1x = (hx - ac.x) * inv.x;
    const double t0y = (ly - ac.y) * inv.y, t1y = (hy - ac.y) * inv.y;
    const double t0z = (lz - ac.z) * inv.z, t1z = (hz - ac.z) * inv.z;
    const double tmin = fmax(fmax(fmin(t0x, t1x), fmin(t0y, t1y)), fmax(fmin(t0z, t1z), 0.0));
    const double tmx = fmin(fmin(fmax(t0x, t1x), fmax(t0y, t1y)), fmin(fmax(t0z, t1z), 1.0));
    return tmin <= tmx * (1.0 + 1e-12) + 1e-300;
  };
  auto tri_block = [&](int32_t leaf) -> bool {
    const int grp = __float_as_int(P.tri32[kTriVecs * leaf + 2].w);
    if (grp == ga || grp == gb) return false;
    const int orig = __float_as_int(P.tri32[kTriVecs * leaf].w);
    const double* t = P.tri64 + 9 * (int64_t)orig;
    const d3 v0 = ld3(t), e1 = ld3(t + 3) - v0, e2 = ld3(t + 6) - v0;
    const d3 pv = cross(D, e2);
    const double det = dot(e1, pv);
    if (det == 0.0) return false;
    const double inv_det = 1.0 / det;
    const d3 tv = a - v0;
    const double u = dot(tv, pv) * inv_det;
    if (u < -1e-9 || u > 1.0 + 1e-9) return false;
    const d3 qv = cross(tv, e1);
    const double v = dot(D, qv) * inv_det;
    if (v < -1e-9 || u + v > 1.0 + 1e-9) return false;  // crack-free margin, as for the faces
    const double s = dot(e2, qv) * inv_det;
    return s > 1e-9 && s < 1.0 - 1e-9;
  };
  for (int q = 0; q < P.n_big; ++q)
    if (tri_block(P.big_off + q)) return true;
  if (!P.has_bvh) return false;
  if (!box_hit(P.root[0], P.root[1], P.root[2], P.root[3], P.root[4], P.root[5])) return false;
  int sp = 0;
  int32_t node = 0;
  while (true) {
    const float4 n0 = P.nodes[4 * node], n1 = P.nodes[4 * node + 1], n2 = P.nodes[4 * node + 2],
                 n3 = P.nodes[4 * node + 3];
    bool hl = box_hit(n0.x, n0.y, n0.z, n0.w, n1.x, n1.y);
    bool hr = box_hit(n1.z, n1.w, n2.x, n2.y, n2.z, n2.w);
    const int32_t cl = __float_as_int(n3.x), cr = __float_as_int(n3.y);
    if (hl && cl < 0) {
      if (tri_block(~cl)) return true;
      hl = false;
    }
    if (hr && cr < 0) {
      if (cr != cl && tri_block(~cr)) return true;
      hr = false;
    }
    if (hl && hr) {
      stk[kWave * sp] = cr;
      ++sp;
      node = cl;
    } else if (hl) {
      node = cl;
    } else if (hr) {
      node = cr;
    } else {
      if (sp == 0) return false;
      --sp;
      node = stk[kWave * sp];
    }
  }
}

}  // namespace sbr
