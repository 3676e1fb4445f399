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

enum : int { BC_PERIODIC = 0, BC_OUTFLOW = 1, BC_NOSLIP = 2, BC_SYMMETRY = 3, BC_DIRICHLET = 4 };
enum : int {
  LIM_SMOOTH = 1, LIM_PP = 2, LIM_POINT = 4, LIM_CENTRE = 8, LIM_LOWONLY = 16, LIM_LEARNED = 32,
  LIM_PEXACT = 64
};
enum : unsigned { FLAG_CELL_LOW = 1u, FLAG_POINT_LOW = 2u, FLAG_NONFINITE = 4u };

// gas and limiter constants in the arithmetic type R of a kernel (FP64, or
// FP32 for the stencils of the mixed-precision stage)
template <typename R>
struct PhysT {
  R gam, gm1, mu, kap, Cs;
  R igm1;  // 1/(gamma-1)
  int lim;
};
using Phys = PhysT<double>;

template <typename R>
__host__ __device__ __forceinline__ PhysT<R> phys_as(const Phys& p) {
  return PhysT<R>{R(p.gam), R(p.gm1), R(p.mu), R(p.kap), R(p.Cs), R(p.igm1), p.lim};
}

// 1/x.  FP64: the hardware reciprocal refined by two Newton steps, which is
// as accurate as the division for the positive normal values it is used on
// (densities, pressures) and much shorter; x = 0 or a non-finite x gives NaN,
// which the stage flags as a non-finite result
template <typename R>
__device__ __forceinline__ R rcp(R x) { return R(1.0) / x; }
template <>
__device__ __forceinline__ double rcp<double>(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(fma(-x, r, 1.0), r, r);
  return fma(fma(-x, r, 1.0), r, r);
}

// NaN-propagating max/min: an inadmissible state anywhere in a stencil must
// make the stage non-finite (and raise the flag), never be skipped.  The
// hardware max/min returns the other operand for a NaN one; 0 * (a + b) is 0
// for finite operands and NaN otherwise, and adding it leaves the exact
// max/min of finite operands unchanged (three instructions, against six for
// the compares and selects of the plain rule)
template <typename R>
__device__ __forceinline__ R mx(R a, R b) {
  return fma(R(0.0), a + b, fmax(a, b));
}
template <typename R>
__device__ __forceinline__ R mn(R a, R b) {
  return fma(R(0.0), a + b, fmin(a, b));
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
// the same as bits: bit 0 negates the x momentum, bit 1 the y momentum
__device__ __forceinline__ int image_flips(int kx, int ky) {
  const int fx = (kx == BC_NOSLIP || kx == BC_SYMMETRY) ^ (ky == BC_NOSLIP);
  const int fy = (kx == BC_NOSLIP) ^ (ky == BC_NOSLIP || ky == BC_SYMMETRY);
  return fx | (fy << 1);
}
__device__ __forceinline__ Signs image_signs(int kx, int ky) {
  const int f = image_flips(kx, ky);
  return Signs{(f & 1) ? -1.0 : 1.0, (f & 2) ? -1.0 : 1.0};
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
  return gm1 * (E - (mx * mx + my * my) * (0.5 * rcp(r)));
}
__device__ __forceinline__ double pressure1(double r, double m, double E, double gm1) {
  return gm1 * (E - m * m / (2.0 * r));
}

// ---------------------------------------------------------------------------
// theta^p solved exactly (the pressure quadratic; switch LIM_PEXACT): the
// largest t in [0, 1] keeping p >= eps on the whole segment from
// UL = (rL, m1L, m2L, EL), of pressure pL, to UT = (rT, m1T, m2T, ET), of
// pressure below eps.  With positive density on the segment (theta^rho
// sees to it), p(s) - eps has the sign of the quadratic
// q(s) = rho(s) (E(s) - eps/(gamma-1)) - |m(s)|^2 / 2, which is positive at
// UL and negative at UT, so it has one root in (0, 1).  The root is taken
// in its cancellation-free form about UL, and again about UT when it lies
// nearer that end: near UT the value of q is a small difference of the
// large terms of the expansion about UL, and p = q (gamma-1) / rho
// magnifies that by 1/rho, so a dense-to-near-vacuum segment needs the
// expansion about UT, whose terms are its own small ones.  Where pL is at
// the 1e-13 floor (eps = pL) the blend is 0, as under the linear rule.
// 1D passes m2 = 0 at both ends.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double theta_p_root(double rL, double m1L, double m2L, double EL,
                                               double rT, double m1T, double m2T, double ET,
                                               double pL, double eps, double gm1) {
  if (!(pL > eps)) return 0.0;
  const double e1 = eps / gm1;
  const double dr = rT - rL, d1 = m1T - m1L, d2 = m2T - m2L, dE = ET - EL;
  const double a = dr * dE - 0.5 * (d1 * d1 + d2 * d2);
  // about UL: q(s) = a s^2 + b s + c, c > 0
  const double c = rL * (EL - e1) - 0.5 * (m1L * m1L + m2L * m2L);
  const double b = dr * (EL - e1) + rL * dE - (m1L * d1 + m2L * d2);
  const double sq = sqrt(fmax(b * b - 4.0 * a * c, 0.0));
  double t = b <= 0.0 ? 2.0 * c / (-b + sq) : (-b - sq) / (2.0 * a);
  if (t > 0.5) {
    // about UT, toward UL: q = a u^2 + bT u + cT in u = 1 - s, cT < 0
    const double cT = rT * (ET - e1) - 0.5 * (m1T * m1T + m2T * m2T);
    const double bT = -(dr * (ET - e1) + rT * dE - (m1T * d1 + m2T * d2));
    const double sqT = sqrt(fmax(bT * bT - 4.0 * a * cT, 0.0));
    const double u = bT >= 0.0 ? 2.0 * cT / (-bT - sqT) : (-bT + sqT) / (2.0 * a);
    t = 1.0 - u;
  }
  return t > 0.0 ? (t < 1.0 ? t : 1.0) : 0.0;
}

// theta^p from UL (pressure pL) toward UT under the linear rule of Sec. 3.3,
// or solved exactly; 1 where p(UT) >= eps
__device__ __forceinline__ double theta_p2(const double* UL, double pL, const double* UT,
                                           double eps, double gm1, bool exact) {
  const double pT = pressure2(UT[0], UT[1], UT[2], UT[3], gm1);
  if (exact && pT < eps)
    return theta_p_root(UL[0], UL[1], UL[2], UL[3], UT[0], UT[1], UT[2], UT[3], pL, eps, gm1);
  return theta_lin(pL, pT, eps);
}
__device__ __forceinline__ double theta_p1(const double* UL, double pL, const double* UT,
                                           double eps, double gm1, bool exact) {
  const double pT = pressure1(UT[0], UT[1], UT[2], gm1);
  if (exact && pT < eps)
    return theta_p_root(UL[0], UL[1], 0.0, UL[2], UT[0], UT[1], 0.0, UT[2], pL, eps, gm1);
  return theta_lin(pL, pT, eps);
}

// Density-then-pressure blend from UL toward UH (2D, 4 components).  Returns
// theta^rho theta^p; sets bad if UL is not admissible (rho<=0 gives 0).
__device__ __forceinline__ double theta_pair2(const double* UL, const double* UH, double gm1,
                                              bool& bad, bool exact) {
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
  const double Ut[4] = {t0, t1, t2, t3};
  const double tp = theta_p2(UL, pL, Ut, mn(kPPEps, pL), gm1, exact);
  return tr * tp;
}

__device__ __forceinline__ double theta_pair1(const double* UL, const double* UH, double gm1,
                                              bool& bad, bool exact) {
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
  const double Ut[3] = {t0, t1, t2};
  const double tp = theta_p1(UL, pL, Ut, mn(kPPEps, pL), gm1, exact);
  return tr * tp;
}

// ---------------------------------------------------------------------------
// one-line operators, offsets -2..2 (Sec. 2.1).  The point update uses the
// identity D+(F+) + D-(F-) = D_c(F) + alpha/(6h) (1,-4,6,-4,1).U, which
// follows from the biased stencils and the splitting F+- = (F +- alpha U)/2.
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ R dc5(R zm2, R zm1, R zp1, R zp2, R inv6h) {
  return ((zm2 - zp2) + R(8.0) * (zp1 - zm1)) * inv6h;
}
template <typename R>
__device__ __forceinline__ R d4(R a, R b, R c, R d, R e) {
  return (a + e) - R(4.0) * (b + d) + R(6.0) * c;
}

// compact second-derivative matrix B = [0 0; 0 M] - [M 0; 0 0] (rows: K site
// m, columns: Z site n, both ordered -2..2) and its column sums
template <typename R>
__device__ __forceinline__ R bmat(int m, int n) {
  constexpr double B[5][5] = {
      {-1.0 / 8.0, 1.0 / 6.0, -1.0 / 24.0, 0.0, 0.0},
      {1.0 / 6.0, 1.0 / 2.0, -5.0 / 6.0, 1.0 / 6.0, 0.0},
      {-1.0 / 8.0, 1.0 / 2.0, -3.0 / 4.0, 1.0 / 2.0, -1.0 / 8.0},
      {0.0, 1.0 / 6.0, -5.0 / 6.0, 1.0 / 2.0, 1.0 / 6.0},
      {0.0, 0.0, -1.0 / 24.0, 1.0 / 6.0, -1.0 / 8.0}};
  return R(B[m][n]);
}

// sum_m sum_n b_mn a_m z_n  (quadratic/bilinear form of B)
template <typename R>
__device__ __forceinline__ R bform(const R* a, const R* z) {
  R s = R(0.0);
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    R t = R(0.0);
#pragma unroll
    for (int n = 0; n < 5; ++n) t += bmat<R>(m, n) * z[n];
    s += a[m] * t;
  }
  return s;
}

// the quadratic form sum_m sum_n b_mn z_m z_n, from the symmetric part of B:
// its twelve nonzero terms, grouped by the lower site index
template <typename R>
__device__ __forceinline__ R bquad(const R* z) {
  const R t0 = R(-1.0 / 8.0) * z[0] + R(1.0 / 3.0) * z[1] - R(1.0 / 6.0) * z[2];
  const R t1 = R(1.0 / 2.0) * z[1] - R(1.0 / 3.0) * z[2] + R(1.0 / 3.0) * z[3];
  const R t2 = R(-3.0 / 4.0) * z[2] - R(1.0 / 3.0) * z[3] - R(1.0 / 6.0) * z[4];
  const R t3 = R(1.0 / 2.0) * z[3] + R(1.0 / 3.0) * z[4];
  const R t4 = R(-1.0 / 8.0) * z[4];
  return z[0] * t0 + z[1] * t1 + z[2] * t2 + z[3] * t3 + z[4] * t4;
}

// sum_n (sum_m b_mn) z_n with column sums (-1/12, 4/3, -5/2, 4/3, -1/12)
template <typename R>
__device__ __forceinline__ R bcol(const R* z) {
  return R(-1.0 / 12.0) * (z[0] + z[4]) + R(4.0 / 3.0) * (z[1] + z[3]) - R(2.5) * z[2];
}

// viscous flux in direction d from the velocity/temperature gradients
// (Newtonian stress, Fourier heat flux):
//   Fv_x = (0, txx, txy, u txx + v txy + kappa Tx), Fv_y likewise.
template <typename R>
__device__ __forceinline__ void visc_flux2(int d, R u, R v, R ux, R vx, R Tx, R uy, R vy, R Ty,
                                           const PhysT<R>& ph, R* F) {
  const R txx = ph.mu * (R(4.0 / 3.0) * ux - R(2.0 / 3.0) * vy);
  const R tyy = ph.mu * (R(4.0 / 3.0) * vy - R(2.0 / 3.0) * ux);
  const R txy = ph.mu * (uy + vx);
  F[0] = R(0.0);
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
template <typename R>
__device__ __forceinline__ void bvisc2_xy(R p, R T, R ux, R vx, R Tx, R uy, R vy, R Ty,
                                          const PhysT<R>& ph, R& bx, R& by) {
  const R txx = ph.mu * (R(4.0 / 3.0) * ux - R(2.0 / 3.0) * vy);
  const R tyy = ph.mu * (R(4.0 / 3.0) * vy - R(2.0 / 3.0) * ux);
  const R txy = ph.mu * (uy + vx);
  const R qx = ph.kap * Tx, qy = ph.kap * Ty;
  const R e2 = R(2.0) * T * ph.igm1;
  const R inv = R(0.5) * ph.gm1 * rcp(p);
  bx = (sqrt(qx * qx + e2 * (txx * txx + txy * txy)) + fabs(qx)) * inv;
  by = (sqrt(qy * qy + e2 * (txy * txy + tyy * tyy)) + fabs(qy)) * inv;
}

// b_d alone, in the same form
template <typename R>
__device__ __forceinline__ R bvisc2_dir(int d, R p, R T, R ux, R vx, R Tx, R uy, R vy, R Ty,
                                        const PhysT<R>& ph) {
  const R txx = ph.mu * (R(4.0 / 3.0) * ux - R(2.0 / 3.0) * vy);
  const R tyy = ph.mu * (R(4.0 / 3.0) * vy - R(2.0 / 3.0) * ux);
  const R txy = ph.mu * (uy + vx);
  const R q = ph.kap * (d == 0 ? Tx : Ty);
  const R t2 = d == 0 ? txx * txx + txy * txy : txy * txy + tyy * tyy;
  const R e2 = R(2.0) * T * ph.igm1;
  return (sqrt(q * q + e2 * t2) + fabs(q)) * (R(0.5) * ph.gm1 * rcp(p));
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
