// af_device.hpp -- device-side building blocks of the AF stage kernels for
// gfx950: physical fluxes, closures, one-line lattice operators and the Theta
// scaling rule.  Everything is FP64 and inlined into the stage kernels.
//
// Notation follows the paper: U = (rho, rho u, rho v, E), W = (rho,u,v,p),
// Z = (0,u,v,T), T = p/rho, kappa = gamma mu/((gamma-1) Pr); the half lattice
// has spacing dx/2, even coordinates on cell faces, odd ones on cell centres.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace afd {

constexpr int kMargin = 4;            // ghost lattice lines kept per side
constexpr double kPPEps = 1.0e-13;    // positivity epsilon (Sec. 3.3)
constexpr double kDucros = 1.0e-13;   // Ducros-sensor regularisation (Sec. 3.2)

enum : int { BC_PERIODIC = 0, BC_OUTFLOW = 1, BC_NOSLIP = 2, BC_SYMMETRY = 3 };
enum : int { LIM_SMOOTH = 1, LIM_PP = 2, LIM_POINT = 4, LIM_CENTRE = 8, LIM_LOWONLY = 16 };
enum : unsigned { FLAG_CELL_LOW = 1u, FLAG_POINT_LOW = 2u, FLAG_NONFINITE = 4u };

struct Phys {
  double gam, gm1, mu, kap, Cs;
  int lim;
};

// NaN-propagating max/min: an inadmissible state anywhere in a stencil must
// make the stage non-finite (and raise the flag), never be skipped
__device__ __forceinline__ double mx(double a, double b) {
  return (a != a || b != b) ? a + b : (a > b ? a : b);
}
__device__ __forceinline__ double mn(double a, double b) {
  return (a != a || b != b) ? a + b : (a < b ? a : b);
}

// ---------------------------------------------------------------------------
// lattice images of ghost coordinates along one axis of 2n half cells.
// kind receives the wall kind crossed (-1 if none).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int axis_image(int X, int twon, int lo, int hi, int& kind) {
  kind = -1;
  if (lo == BC_PERIODIC) {
    int r = X % twon;
    return r < 0 ? r + twon : r;
  }
  if (X < 0) {
    if (lo == BC_OUTFLOW) return (X & 1) ? 1 : 0;
    kind = lo;
    return -X;
  }
  if (X > twon) {
    if (hi == BC_OUTFLOW) return ((X - twon) & 1) ? twon - 1 : twon;
    kind = hi;
    return 2 * twon - X;
  }
  return X;
}

// momentum signs (sx, sy) of the image of a site reached across the wall
// kinds kx (normal x) and ky (normal y), -1 when none was crossed: a no-slip
// wall flips both momenta, a symmetry line the normal one.  Plain integer
// parity, so the result stays in registers.
struct Signs {
  double sx, sy;
};
__device__ __forceinline__ Signs image_signs(int kx, int ky) {
  const int fx = (kx == BC_NOSLIP || kx == BC_SYMMETRY) ^ (ky == BC_NOSLIP);
  const int fy = (kx == BC_NOSLIP) ^ (ky == BC_NOSLIP || ky == BC_SYMMETRY);
  return Signs{fx ? -1.0 : 1.0, fy ? -1.0 : 1.0};
}

// ---------------------------------------------------------------------------
// Theta of the linear scaling rule (Sec. 3.3): largest blend keeping
// (1-t) zL + t zH >= eps, for zL >= eps.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double theta_lin(double zL, double zH, double eps) {
  // the division only where the limiter acts (a branch, not a select)
  if (zH < eps) return (zL - eps) / (zL - zH);
  return 1.0;
}

__device__ __forceinline__ double pressure2(double r, double mx, double my, double E, double gm1) {
  return gm1 * (E - (mx * mx + my * my) / (2.0 * r));
}
__device__ __forceinline__ double pressure1(double r, double m, double E, double gm1) {
  return gm1 * (E - m * m / (2.0 * r));
}

// Density-then-pressure blend from UL toward UH (2D, 4 components).  Returns
// theta^rho theta^p; sets bad if UL is not admissible (rho<=0 gives 0).
__device__ __forceinline__ double theta_pair2(const double* UL, const double* UH, double gm1,
                                              bool& bad) {
  if (!(UL[0] > 0.0)) {
    bad = true;
    return 0.0;
  }
  const double pL = pressure2(UL[0], UL[1], UL[2], UL[3], gm1);
  if (!(pL > 0.0)) bad = true;
  const double tr = theta_lin(UL[0], UH[0], mn(kPPEps, UL[0]));
  const double t0 = UL[0] + tr * (UH[0] - UL[0]);
  const double t1 = UL[1] + tr * (UH[1] - UL[1]);
  const double t2 = UL[2] + tr * (UH[2] - UL[2]);
  const double t3 = UL[3] + tr * (UH[3] - UL[3]);
  const double tp = theta_lin(pL, pressure2(t0, t1, t2, t3, gm1), mn(kPPEps, pL));
  return tr * tp;
}

__device__ __forceinline__ double theta_pair1(const double* UL, const double* UH, double gm1,
                                              bool& bad) {
  if (!(UL[0] > 0.0)) {
    bad = true;
    return 0.0;
  }
  const double pL = pressure1(UL[0], UL[1], UL[2], gm1);
  if (!(pL > 0.0)) bad = true;
  const double tr = theta_lin(UL[0], UH[0], mn(kPPEps, UL[0]));
  const double t0 = UL[0] + tr * (UH[0] - UL[0]);
  const double t1 = UL[1] + tr * (UH[1] - UL[1]);
  const double t2 = UL[2] + tr * (UH[2] - UL[2]);
  const double tp = theta_lin(pL, pressure1(t0, t1, t2, gm1), mn(kPPEps, pL));
  return tr * tp;
}

// ---------------------------------------------------------------------------
// one-line operators, offsets -2..2 (Sec. 2.1).  The point update uses the
// identity D+(F+) + D-(F-) = D_c(F) + alpha/(6h) (1,-4,6,-4,1).U, which
// follows from the biased stencils and the splitting F+- = (F +- alpha U)/2.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double dc5(double zm2, double zm1, double zp1, double zp2, double inv6h) {
  return ((zm2 - zp2) + 8.0 * (zp1 - zm1)) * inv6h;
}
__device__ __forceinline__ double d4(double a, double b, double c, double d, double e) {
  return (a + e) - 4.0 * (b + d) + 6.0 * c;
}

// compact second-derivative matrix B = [0 0; 0 M] - [M 0; 0 0] (rows: K site
// m, columns: Z site n, both ordered -2..2) and its column sums
__device__ __forceinline__ double bmat(int m, int n) {
  constexpr double B[5][5] = {
      {-1.0 / 8.0, 1.0 / 6.0, -1.0 / 24.0, 0.0, 0.0},
      {1.0 / 6.0, 1.0 / 2.0, -5.0 / 6.0, 1.0 / 6.0, 0.0},
      {-1.0 / 8.0, 1.0 / 2.0, -3.0 / 4.0, 1.0 / 2.0, -1.0 / 8.0},
      {0.0, 1.0 / 6.0, -5.0 / 6.0, 1.0 / 2.0, 1.0 / 6.0},
      {0.0, 0.0, -1.0 / 24.0, 1.0 / 6.0, -1.0 / 8.0}};
  return B[m][n];
}

// sum_m sum_n b_mn a_m z_n  (quadratic/bilinear form of B)
__device__ __forceinline__ double bform(const double* a, const double* z) {
  double s = 0.0;
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    double t = 0.0;
#pragma unroll
    for (int n = 0; n < 5; ++n) t += bmat(m, n) * z[n];
    s += a[m] * t;
  }
  return s;
}

// sum_n (sum_m b_mn) z_n with column sums (-1/12, 4/3, -5/2, 4/3, -1/12)
__device__ __forceinline__ double bcol(const double* z) {
  return (-1.0 / 12.0) * (z[0] + z[4]) + (4.0 / 3.0) * (z[1] + z[3]) - 2.5 * z[2];
}

// viscous flux in direction d from the velocity/temperature gradients
// (Newtonian stress, Fourier heat flux):
//   Fv_x = (0, txx, txy, u txx + v txy + kappa Tx), Fv_y likewise.
__device__ __forceinline__ void visc_flux2(int d, double u, double v, double ux, double vx,
                                           double Tx, double uy, double vy, double Ty,
                                           const Phys& ph, double* F) {
  const double txx = ph.mu * ((4.0 / 3.0) * ux - (2.0 / 3.0) * vy);
  const double tyy = ph.mu * ((4.0 / 3.0) * vy - (2.0 / 3.0) * ux);
  const double txy = ph.mu * (uy + vx);
  F[0] = 0.0;
  if (d == 0) {
    F[1] = txx;
    F[2] = txy;
    F[3] = u * txx + v * txy + ph.kap * Tx;
  } else {
    F[1] = txy;
    F[2] = tyy;
    F[3] = u * txy + v * tyy + ph.kap * Ty;
  }
}

// b_l of the viscous splitting lemma (Sec. 3.1): with rho e = p/(gamma-1),
//   b = (sqrt(q^2 + 2 e |tau_l|^2) + |q|) / (2 rho e)
// both b_x and b_y with shared terms: e = T/(gamma-1), 1/(2 rho e) =
// (gamma-1)/(2 p); one division for the pair
__device__ __forceinline__ void bvisc2_xy(double p, double T, double ux, double vx, double Tx,
                                          double uy, double vy, double Ty, const Phys& ph,
                                          double& bx, double& by) {
  const double txx = ph.mu * ((4.0 / 3.0) * ux - (2.0 / 3.0) * vy);
  const double tyy = ph.mu * ((4.0 / 3.0) * vy - (2.0 / 3.0) * ux);
  const double txy = ph.mu * (uy + vx);
  const double qx = ph.kap * Tx, qy = ph.kap * Ty;
  const double e2 = 2.0 * T / ph.gm1;
  const double inv = 0.5 * ph.gm1 / p;
  bx = (sqrt(qx * qx + e2 * (txx * txx + txy * txy)) + fabs(qx)) * inv;
  by = (sqrt(qy * qy + e2 * (txy * txy + tyy * tyy)) + fabs(qy)) * inv;
}

// b_d alone, in the same form
__device__ __forceinline__ double bvisc2_dir(int d, double p, double T, double ux, double vx,
                                             double Tx, double uy, double vy, double Ty,
                                             const Phys& ph) {
  const double txx = ph.mu * ((4.0 / 3.0) * ux - (2.0 / 3.0) * vy);
  const double tyy = ph.mu * ((4.0 / 3.0) * vy - (2.0 / 3.0) * ux);
  const double txy = ph.mu * (uy + vx);
  const double q = ph.kap * (d == 0 ? Tx : Ty);
  const double t2 = d == 0 ? txx * txx + txy * txy : txy * txy + tyy * tyy;
  const double e2 = 2.0 * T / ph.gm1;
  return (sqrt(q * q + e2 * t2) + fabs(q)) * (0.5 * ph.gm1 / p);
}

__device__ __forceinline__ double bvisc1(double rho, double p, double ux, double Tx,
                                         const Phys& ph) {
  const double tau = ph.mu * (4.0 / 3.0) * ux;
  const double q = ph.kap * Tx;
  const double re = p / ph.gm1;
  const double e = re / rho;
  return (sqrt(q * q + 2.0 * e * tau * tau) + fabs(q)) / (2.0 * re);
}

// sticky flag word
__device__ __forceinline__ void raise_flag(unsigned* flags, unsigned f) {
  atomicOr(flags, f);
}

// current value of the flag word, as other workgroups of a running kernel
// may have raised it (device-coherent load)
__device__ __forceinline__ unsigned peek_flags(unsigned* flags) {
  return __hip_atomic_load(flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace afd
