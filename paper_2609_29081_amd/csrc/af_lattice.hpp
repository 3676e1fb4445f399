// af_lattice.hpp -- addressing of the 2D half lattice in a state buffer and
// the boundary images of ghost sites, shared by the 2D stage and the
// learned-blend kernels.
#pragma once

#include "af_device.hpp"
#include "af_internal.hpp"

namespace afd {

using G2 = afi::StageGeo;

// offset of interior lattice site (X, Y) in a state (its first component;
// centre sites hold the cell average, the periodic seam is folded) and the
// distance between its component planes.  Plane indices fit 32 bits (the
// grid size is bounded at init).  The grid is the same for the whole wave:
// its sizes are taken as wave-uniform values, so that the per-site choice
// among them is a register select, never a per-lane load of a size.
__device__ __forceinline__ void site_ofs(const G2& g, int X, int Y, long& o, int& st) {
  const int n1 = __builtin_amdgcn_readfirstlane(g.n1), n1x = __builtin_amdgcn_readfirstlane(g.n1x);
  const int n2 = __builtin_amdgcn_readfirstlane(g.n2), n2y = __builtin_amdgcn_readfirstlane(g.n2y);
  if (X == 2 * n1 && n1x == n1) X = 0;
  if (Y == 2 * n2 && n2y == n2) Y = 0;
  const bool xo = X & 1, yo = Y & 1;
  const int ncol = xo ? n1 : n1x;
  const long base = xo ? (yo ? 0L : g.off_ye) : (yo ? g.off_xe : g.off_co);
  st = ncol * (yo ? n2 : n2y);
  o = base + (long)((Y >> 1) * ncol + (X >> 1));
}

// FP64 value of lattice site (X, Y), X in [-4, 2n1+4], read from the state:
// ghosts are images of interior sites (centre sites hold the average)
__device__ __forceinline__ void raw_value(const G2& g, const double* __restrict__ U, int X, int Y,
                                          double* V) {
  int kx, ky;
  const int Xi = axis_image(X, 2 * g.n1, g.bc0, g.bc1, kx);
  const int Yi = axis_image(Y, 2 * g.n2, g.bc2, g.bc3, ky);
  const Signs sg = image_signs(kx, ky);
  long o;
  int st;
  site_ofs(g, Xi, Yi, o, st);
#pragma unroll
  for (int k = 0; k < 4; ++k) V[k] = U[o + (long)k * st];
  V[1] *= sg.sx;
  V[2] *= sg.sy;
}

}  // namespace afd
