// Analytic closest-point functions on the device (App. A: analytic cp where
// it exists).  Every decision of the band builder (band membership, Omega(C),
// check region, stencil base, crossing tests) depends on these values, so the
// formulas use only +, -, *, / and sqrt, which are correctly rounded in IEEE
// FP64, in a fixed order; the file that includes this header is compiled with
// -ffp-contract=off so no product is fused into an FMA.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/cpm.h"

namespace cpm {

struct V3 {
  double x, y, z;
};

__device__ __forceinline__ V3 node_pos(int kx, int ky, int kz, int N) {
  const double dn = (double)N;
  return V3{(double)kx / dn, (double)ky / dn, (double)kz / dn};
}

// ((a.x b.x + a.y b.y) + a.z b.z); 2-D callers keep z = 0 and skip the term.
template <int DIM>
__device__ __forceinline__ double dot3(const V3& a, const V3& b) {
  double s = a.x * b.x + a.y * b.y;
  if (DIM == 3) s = s + a.z * b.z;
  return s;
}

template <int DIM>
__device__ __forceinline__ double dist(const V3& a, const V3& b) {
  V3 d{a.x - b.x, a.y - b.y, a.z - b.z};
  return sqrt(dot3<DIM>(d, d));
}

// cp_S: circle / sphere  c + (x - c) R / |x - c|;
// torus: nearest core-circle point q, then q + (x - q) rho / |x - q|.
template <int DIM>
__device__ __forceinline__ V3 cp_surface(const cpm_surface& S, const V3& p) {
  const double cx = S.center[0], cy = S.center[1], cz = S.center[2];
  const double dx = p.x - cx, dy = p.y - cy;
  if (DIM == 2) {
    const double rho = sqrt(dx * dx + dy * dy);
    const double s = S.R / rho;
    return V3{cx + dx * s, cy + dy * s, 0.0};
  }
  const double dz = p.z - cz;
  if (S.kind == CPM_SURF_SPHERE) {
    const double rho = sqrt((dx * dx + dy * dy) + dz * dz);
    const double s = S.R / rho;
    return V3{cx + dx * s, cy + dy * s, cz + dz * s};
  }
  // torus
  const double qr = sqrt(dx * dx + dy * dy);
  const double s = S.R / qr;
  const double qx = dx * s, qy = dy * s;
  const double ex = dx - qx, ey = dy - qy;
  const double e = sqrt((ex * ex + ey * ey) + dz * dz);
  const double t = S.rho / e;
  return V3{cx + (qx + ex * t), cy + (qy + ey * t), cz + dz * t};
}

// Open latitude arc: does the horizontal direction of p lie in the arc
// (counter-clockwise from a to b)?  Sign tests of cross products only.
__device__ __forceinline__ bool arc_inside(const cpm_surface& S, const cpm_ibc& C, const V3& p) {
  const double dx = p.x - S.center[0], dy = p.y - S.center[1];
  const double a0 = C.arc[0], a1 = C.arc[1], b0 = C.arc[2], b1 = C.arc[3];
  const double ca = a0 * dy - a1 * dx;
  const double cb = dx * b1 - dy * b0;
  if (a0 * b1 - a1 * b0 >= 0.0) return ca >= 0.0 && cb >= 0.0;
  return ca >= 0.0 || cb >= 0.0;
}

// Is cp_C(p) an endpoint of an open curve (Omega(dC), eq. IBC_boundary_set)?
__device__ __forceinline__ bool curve_at_end(const cpm_surface& S, const cpm_ibc& C,
                                             const V3& p) {
  return C.kind == CPM_IBC_LATITUDE_ARC && !arc_inside(S, C, p);
}

// cp_C for a point, a latitude circle or arc of a sphere, a meridian of a
// torus.  For an arc outside its angular range: the nearer endpoint (squared
// distances, ties to the start).
template <int DIM>
__device__ __forceinline__ V3 cp_curve(const cpm_surface& S, const cpm_ibc& C,
                                       const V3& p) {
  if (C.kind == CPM_IBC_POINT) return V3{C.p[0], C.p[1], DIM == 3 ? C.p[2] : 0.0};
  const double cx = S.center[0], cy = S.center[1], cz = S.center[2];
  if (C.kind == CPM_IBC_LATITUDE || C.kind == CPM_IBC_LATITUDE_ARC) {
    const double rho0 = sqrt(S.R * S.R - C.z0 * C.z0);
    if (C.kind == CPM_IBC_LATITUDE_ARC && !arc_inside(S, C, p)) {
      const double z = cz + C.z0;
      const V3 e0{cx + rho0 * C.arc[0], cy + rho0 * C.arc[1], z};
      const V3 e1{cx + rho0 * C.arc[2], cy + rho0 * C.arc[3], z};
      const double d0x = p.x - e0.x, d0y = p.y - e0.y, d0z = p.z - e0.z;
      const double d1x = p.x - e1.x, d1y = p.y - e1.y, d1z = p.z - e1.z;
      const double d0 = (d0x * d0x + d0y * d0y) + d0z * d0z;
      const double d1 = (d1x * d1x + d1y * d1y) + d1z * d1z;
      return d1 < d0 ? e1 : e0;
    }
    const double dx = p.x - cx, dy = p.y - cy;
    const double q = sqrt(dx * dx + dy * dy);
    const double s = rho0 / q;
    return V3{cx + dx * s, cy + dy * s, cz + C.z0};
  }
  // meridian
  const double ex = C.dir[0], ey = C.dir[1];
  const double c0x = cx + S.R * ex, c0y = cy + S.R * ey;
  const double dx = p.x - c0x, dy = p.y - c0y, dz = p.z - cz;
  const double a = dx * ex + dy * ey;
  const double nrm = sqrt(a * a + dz * dz);
  const double s = S.rho / nrm;
  const double as = a * s;
  return V3{c0x + as * ex, c0y + as * ey, cz + dz * s};
}

// o_C at a point of C: the side an on-C closest point is assigned to.
template <int DIM>
__device__ __forceinline__ V3 orient_curve(const cpm_surface& S,
                                           const cpm_ibc& C, const V3& cpc) {
  if (C.kind == CPM_IBC_POINT) return V3{C.orient[0], C.orient[1], DIM == 3 ? C.orient[2] : 0.0};
  if (C.kind == CPM_IBC_LATITUDE || C.kind == CPM_IBC_LATITUDE_ARC) {
    const double rho0 = sqrt(S.R * S.R - C.z0 * C.z0);
    const double ux = (cpc.x - S.center[0]) / rho0;
    const double uy = (cpc.y - S.center[1]) / rho0;
    return V3{(-C.z0 * ux) / S.R, (-C.z0 * uy) / S.R, rho0 / S.R};
  }
  return V3{-C.dir[1], C.dir[0], 0.0};
}

}  // namespace cpm
