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

// cp_C for a point, a latitude circle of a sphere, a meridian of a torus.
template <int DIM>
__device__ __forceinline__ V3 cp_curve(const cpm_surface& S, const cpm_ibc& C,
                                       const V3& p) {
  if (C.kind == CPM_IBC_POINT) return V3{C.p[0], C.p[1], DIM == 3 ? C.p[2] : 0.0};
  const double cx = S.center[0], cy = S.center[1], cz = S.center[2];
  if (C.kind == CPM_IBC_LATITUDE) {
    const double rho0 = sqrt(S.R * S.R - C.z0 * C.z0);
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
  if (C.kind == CPM_IBC_LATITUDE) {
    const double rho0 = sqrt(S.R * S.R - C.z0 * C.z0);
    const double ux = (cpc.x - S.center[0]) / rho0;
    const double uy = (cpc.y - S.center[1]) / rho0;
    return V3{(-C.z0 * ux) / S.R, (-C.z0 * uy) / S.R, rho0 / S.R};
  }
  return V3{-C.dir[1], C.dir[0], 0.0};
}

}  // namespace cpm
