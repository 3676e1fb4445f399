// af_kern2d.hip -- one SSP-RK3 stage of the 2D compact AF method on gfx950.
//
// Pipeline per stage (all FP64, SoA arrays with x fastest):
//   lattice : conservative value + (u,v,p,T,c) at every half-lattice site,
//             ghosts as boundary images, Simpson centres scaled toward the
//             cell average (Sec. 2.2; Remark after the pressure blend, Sec. 3.3)
//   grad    : D_c gradients of (u,v,T) along both lattice directions
//   cellpre : per cell (with a one-cell ring): low-order gradient S, total
//             flux F_l, |u_l|+c, b_l, smoothness sensors phi1, phi2 (Sec. 3.1-3.2)
//   face    : Simpson high-order face flux, LLF low-order flux, theta^s,
//             theta^rho theta^p from the intermediate states (Sec. 3.3)
//   cells   : conservative update of the averages + RK combination
//   points  : AF point residual (biased inviscid operators with the downwind
//             point, compact D^2, mixed terms; Sec. 2.2), point LLF and
//             scaling limiter (Sec. 3.4), wall projection, RK combination
#include "af_device.hpp"
#include "af_internal.hpp"

using namespace afd;

namespace {

constexpr int kBlock = 256;

struct G2 {
  int n1, n2, n1x, n2y, LX, LY;
  long ns, off_xe, off_ye, off_co;
  int bc0, bc1, bc2, bc3;
  double dx, dy;
};

G2 make_g2(const afi::Geo& g) {
  G2 r;
  r.n1 = g.n1;
  r.n2 = g.n2;
  r.n1x = g.n1x;
  r.n2y = g.n2y;
  r.LX = g.LX;
  r.LY = g.LY;
  r.ns = g.ns;
  r.off_xe = g.off_xe;
  r.off_ye = g.off_ye;
  r.off_co = g.off_co;
  r.bc0 = g.bc[0];
  r.bc1 = g.bc[1];
  r.bc2 = g.bc[2];
  r.bc3 = g.bc[3];
  r.dx = g.dx;
  r.dy = g.dy;
  return r;
}

__device__ __forceinline__ long lidx(const G2& g, int X, int Y) {
  return (long)(Y + kMargin) * g.LX + (X + kMargin);
}

// interior point DOF (X,Y not both odd), periodic seam folded
__device__ __forceinline__ double dof(const G2& g, const double* __restrict__ U, int X, int Y,
                                      int k) {
  if (X == 2 * g.n1 && g.n1x == g.n1) X = 0;
  if (Y == 2 * g.n2 && g.n2y == g.n2) Y = 0;
  if (Y & 1) return U[g.off_xe + ((long)k * g.n2 + (Y >> 1)) * g.n1x + (X >> 1)];
  if (X & 1) return U[g.off_ye + ((long)k * g.n2y + (Y >> 1)) * g.n1 + (X >> 1)];
  return U[g.off_co + ((long)k * g.n2y + (Y >> 1)) * g.n1x + (X >> 1)];
}

__device__ __forceinline__ double avg(const G2& g, const double* __restrict__ U, int i, int j,
                                      int k) {
  return U[((long)k * g.n2 + j) * g.n1 + i];
}

// cell average of a (possibly ghost) cell via its lattice image
__device__ __forceinline__ void cell_image(const G2& g, const double* __restrict__ U, int i, int j,
                                           double* V) {
  int kx, ky;
  const int Xi = axis_image(2 * i + 1, 2 * g.n1, g.bc0, g.bc1, kx);
  const int Yi = axis_image(2 * j + 1, 2 * g.n2, g.bc2, g.bc3, ky);
  double sx = 1.0, sy = 1.0;
  mirror_signs(kx, 0, sx, sy);
  mirror_signs(ky, 1, sx, sy);
  const int ii = Xi >> 1, jj = Yi >> 1;
  V[0] = avg(g, U, ii, jj, 0);
  V[1] = sx * avg(g, U, ii, jj, 1);
  V[2] = sy * avg(g, U, ii, jj, 2);
  V[3] = avg(g, U, ii, jj, 3);
}

// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_lattice(G2 g, Phys ph, const double* __restrict__ U,
                                                    double* __restrict__ LU,
                                                    double* __restrict__ LA) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.ns) return;
  const int X = (int)(t % g.LX) - kMargin;
  const int Y = (int)(t / g.LX) - kMargin;
  int kx, ky;
  const int Xi = axis_image(X, 2 * g.n1, g.bc0, g.bc1, kx);
  const int Yi = axis_image(Y, 2 * g.n2, g.bc2, g.bc3, ky);
  double sx = 1.0, sy = 1.0;
  mirror_signs(kx, 0, sx, sy);
  mirror_signs(ky, 1, sx, sy);
  double V[4];
  if ((Xi & 1) && (Yi & 1)) {
    const int i = Xi >> 1, j = Yi >> 1;
    double Ub[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      Ub[k] = avg(g, U, i, j, k);
      const double e = dof(g, U, Xi - 1, Yi, k) + dof(g, U, Xi + 1, Yi, k) +
                       dof(g, U, Xi, Yi - 1, k) + dof(g, U, Xi, Yi + 1, k);
      const double c = dof(g, U, Xi - 1, Yi - 1, k) + dof(g, U, Xi + 1, Yi - 1, k) +
                       dof(g, U, Xi - 1, Yi + 1, k) + dof(g, U, Xi + 1, Yi + 1, k);
      V[k] = (36.0 * Ub[k] - 4.0 * e - c) / 16.0;
    }
    if (ph.lim & LIM_CENTRE) {
      if (!(Ub[0] > 0.0)) {
#pragma unroll
        for (int k = 0; k < 4; ++k) V[k] = Ub[k];
      } else {
        bool bad = false;
        const double th = theta_pair2(Ub, V, ph.gm1, bad);
        if (th < 1.0) {
#pragma unroll
          for (int k = 0; k < 4; ++k) V[k] = Ub[k] + th * (V[k] - Ub[k]);
        }
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k) V[k] = dof(g, U, Xi, Yi, k);
  }
  V[1] *= sx;
  V[2] *= sy;
  const double u = V[1] / V[0], v = V[2] / V[0];
  const double p = pressure2(V[0], V[1], V[2], V[3], ph.gm1);
  const double T = p / V[0];
  const double c = sqrt(ph.gam * p / V[0]);
#pragma unroll
  for (int k = 0; k < 4; ++k) LU[k * g.ns + t] = V[k];
  LA[0 * g.ns + t] = u;
  LA[1 * g.ns + t] = v;
  LA[2 * g.ns + t] = p;
  LA[3 * g.ns + t] = T;
  LA[4 * g.ns + t] = c;
}

// gradients D_c^{(1)}, D_c^{(2)} of (u, v, T) on sites [-2, 2n+2]^2
__global__ void __launch_bounds__(kBlock) k_grad(G2 g, const double* __restrict__ LA,
                                                 double* __restrict__ LG) {
  const int W = 2 * g.n1 + 5, H = 2 * g.n2 + 5;
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)W * H) return;
  const int X = (int)(t % W) - 2, Y = (int)(t / W) - 2;
  const long q = lidx(g, X, Y);
  const double ihx = 1.0 / (6.0 * g.dx), ihy = 1.0 / (6.0 * g.dy);
  const long sy = g.LX;
  const int src[3] = {0, 1, 3};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double* z = LA + src[a] * g.ns;
    LG[a * g.ns + q] = dc5(z[q - 2], z[q - 1], z[q + 1], z[q + 2], ihx);
    LG[(3 + a) * g.ns + q] = dc5(z[q - 2 * sy], z[q - sy], z[q + sy], z[q + 2 * sy], ihy);
  }
}

// per-cell low-order data on cells [-1, n1] x [-1, n2]
// CP layout: 0-3 F_x, 4-7 F_y, 8 rs_x, 9 rs_y, 10 b_x, 11 b_y, 12 phi1,
//            13 phi2, 14-17 cell average

__global__ void __launch_bounds__(kBlock) k_cellpre(G2 g, Phys ph, const double* __restrict__ U,
                                                    double* __restrict__ CP) {
  const int W = g.n1 + 2, H = g.n2 + 2;
  const long nc = (long)W * H;
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nc) return;
  const int i = (int)(t % W) - 1, j = (int)(t / W) - 1;
  double C0[4], Cxm[4], Cxp[4], Cym[4], Cyp[4];
  cell_image(g, U, i, j, C0);
  cell_image(g, U, i - 1, j, Cxm);
  cell_image(g, U, i + 1, j, Cxp);
  cell_image(g, U, i, j - 1, Cym);
  cell_image(g, U, i, j + 1, Cyp);
  auto pr = [&](const double* V) { return pressure2(V[0], V[1], V[2], V[3], ph.gm1); };
  const double p0 = pr(C0), pxm = pr(Cxm), pxp = pr(Cxp), pym = pr(Cym), pyp = pr(Cyp);
  const double u0 = C0[1] / C0[0], v0 = C0[2] / C0[0];
  const double uxm = Cxm[1] / Cxm[0], uxp = Cxp[1] / Cxp[0], uym = Cym[1] / Cym[0],
               uyp = Cyp[1] / Cyp[0];
  const double vxm = Cxm[2] / Cxm[0], vxp = Cxp[2] / Cxp[0], vym = Cym[2] / Cym[0],
               vyp = Cyp[2] / Cyp[0];
  const double i2x = 1.0 / (2.0 * g.dx), i2y = 1.0 / (2.0 * g.dy);
  // low-order gradient S: central differences of Z(average)
  const double ux = (uxp - uxm) * i2x, vx = (vxp - vxm) * i2x;
  const double Tx = (pxp / Cxp[0] - pxm / Cxm[0]) * i2x;
  const double uy = (uyp - uym) * i2y, vy = (vyp - vym) * i2y;
  const double Ty = (pyp / Cyp[0] - pym / Cym[0]) * i2y;
  const double c0 = sqrt(ph.gam * p0 / C0[0]);
  double Fv[4];
  const long ncp = nc;
  // F_x = F^c_x - F^v_x
  visc_flux2(0, u0, v0, ux, vx, Tx, uy, vy, Ty, ph, Fv);
  CP[0 * ncp + t] = C0[1] - Fv[0];
  CP[1 * ncp + t] = C0[1] * u0 + p0 - Fv[1];
  CP[2 * ncp + t] = C0[2] * u0 - Fv[2];
  CP[3 * ncp + t] = (C0[3] + p0) * u0 - Fv[3];
  visc_flux2(1, u0, v0, ux, vx, Tx, uy, vy, Ty, ph, Fv);
  CP[4 * ncp + t] = C0[2] - Fv[0];
  CP[5 * ncp + t] = C0[1] * v0 - Fv[1];
  CP[6 * ncp + t] = C0[2] * v0 + p0 - Fv[2];
  CP[7 * ncp + t] = (C0[3] + p0) * v0 - Fv[3];
  CP[8 * ncp + t] = fabs(u0) + c0;
  CP[9 * ncp + t] = fabs(v0) + c0;
  CP[10 * ncp + t] = bvisc2(0, C0[0], p0, ux, vx, Tx, uy, vy, Ty, ph);
  CP[11 * ncp + t] = bvisc2(1, C0[0], p0, ux, vx, Tx, uy, vy, Ty, ph);
  // smoothness sensors (Jameson pressure sensor, modified Ducros sensor)
  const double jx = fabs(pxp - 2.0 * p0 + pxm) / fabs(pxp + 2.0 * p0 + pxm);
  const double jy = fabs(pyp - 2.0 * p0 + pym) / fabs(pyp + 2.0 * p0 + pym);
  CP[12 * ncp + t] = mx(jx, jy);
  const double div = ux + vy, curl = vx - uy;
  CP[13 * ncp + t] = mx(-div / sqrt(div * div + curl * curl + kDucros), 0.0);
#pragma unroll
  for (int k = 0; k < 4; ++k) CP[(14 + k) * ncp + t] = C0[k];
}

// total flux F_d (= F^c_d - F^v_d) at a lattice site from the lattice arrays
__device__ __forceinline__ void site_flux(const G2& g, const Phys& ph, const double* __restrict__ LU,
                                          const double* __restrict__ LA,
                                          const double* __restrict__ LG, long q, int d,
                                          double* F) {
  const double r = LU[q], mx = LU[g.ns + q], my = LU[2 * g.ns + q], E = LU[3 * g.ns + q];
  const double u = LA[q], v = LA[g.ns + q], p = LA[2 * g.ns + q];
  double Fv[4];
  visc_flux2(d, u, v, LG[q], LG[g.ns + q], LG[2 * g.ns + q], LG[3 * g.ns + q],
             LG[4 * g.ns + q], LG[5 * g.ns + q], ph, Fv);
  const double ud = d == 0 ? u : v;
  F[0] = (d == 0 ? mx : my) - Fv[0];
  F[1] = mx * ud + (d == 0 ? p : 0.0) - Fv[1];
  F[2] = my * ud + (d == 1 ? p : 0.0) - Fv[2];
  F[3] = (E + p) * ud - Fv[3];
  (void)r;
}

template <int D>
__global__ void __launch_bounds__(kBlock) k_face(G2 g, Phys ph, const double* __restrict__ LU,
                                                 const double* __restrict__ LA,
                                                 const double* __restrict__ LG,
                                                 const double* __restrict__ CP,
                                                 double* __restrict__ FO, const double* dt_dev,
                                                 double dt_host, unsigned* flags) {
  const int ni = D == 0 ? g.n1 + 1 : g.n1;
  const int nj = D == 0 ? g.n2 : g.n2 + 1;
  const long nf = (long)ni * nj;
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nf) return;
  const int i = (int)(t % ni), j = (int)(t / ni);
  const double dt = dt_dev ? *dt_dev : dt_host;
  // lattice face-centre point and its Simpson neighbours along the face
  const int X = D == 0 ? 2 * i : 2 * i + 1;
  const int Y = D == 0 ? 2 * j + 1 : 2 * j;
  const long q = lidx(g, X, Y);
  const long st = D == 0 ? (long)g.LX : 1;
  double Fa[4], Fm[4], Fb[4], FH[4];
  site_flux(g, ph, LU, LA, LG, q - st, D, Fa);
  site_flux(g, ph, LU, LA, LG, q, D, Fm);
  site_flux(g, ph, LU, LA, LG, q + st, D, Fb);
#pragma unroll
  for (int k = 0; k < 4; ++k) FH[k] = (Fa[k] + 4.0 * Fm[k] + Fb[k]) / 6.0;
  double F[4];
  const int limc = ph.lim & (LIM_SMOOTH | LIM_PP | 16);
  if (!limc) {
#pragma unroll
    for (int k = 0; k < 4; ++k) F[k] = FH[k];
  } else {
    const int W = g.n1 + 2;
    const long ncp = (long)W * (g.n2 + 2);
    // cells a (minus side) and b (plus side), indices in the ringed cell grid
    const long cb = (long)(j + 1) * W + (i + 1);
    const long ca = D == 0 ? cb - 1 : cb - W;
    const double lam = mx(CP[(8 + D) * ncp + ca], CP[(8 + D) * ncp + cb]) +
                       mx(CP[(10 + D) * ncp + ca], CP[(10 + D) * ncp + cb]);
    double FL[4], Ua[4], Ub[4], Fca[4], Fcb[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      Ua[k] = CP[(14 + k) * ncp + ca];
      Ub[k] = CP[(14 + k) * ncp + cb];
      Fca[k] = CP[(4 * D + k) * ncp + ca];
      Fcb[k] = CP[(4 * D + k) * ncp + cb];
      FL[k] = 0.5 * (Fca[k] + Fcb[k]) - 0.5 * lam * (Ub[k] - Ua[k]);
    }
    double ts = 1.0, tpp = 1.0;
    if (ph.lim & 16) {
      ts = 0.0;
      tpp = 0.0;
    } else {
      if (ph.lim & LIM_SMOOTH)
        ts = exp(-ph.Cs * mx(CP[12 * ncp + ca], CP[12 * ncp + cb]) *
                 mx(CP[13 * ncp + ca], CP[13 * ncp + cb]));
      if (ph.lim & LIM_PP) {
        const double m4 = 4.0 * dt / (D == 0 ? g.dx : g.dy);
        double ULp[4], UHp[4], ULm[4], UHm[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const double Fs = FL[k] + ts * (FH[k] - FL[k]);
          ULp[k] = Ua[k] - m4 * (FL[k] - Fca[k]);
          UHp[k] = Ua[k] - m4 * (Fs - Fca[k]);
          ULm[k] = Ub[k] - m4 * (Fcb[k] - FL[k]);
          UHm[k] = Ub[k] - m4 * (Fcb[k] - Fs);
        }
        tpp = 0.0;
        bool bad = false;
        if (!(ULp[0] > 0.0) || !(ULm[0] > 0.0)) {
          bad = true;
        } else {
          const double pLp = pressure2(ULp[0], ULp[1], ULp[2], ULp[3], ph.gm1);
          const double pLm = pressure2(ULm[0], ULm[1], ULm[2], ULm[3], ph.gm1);
          if (!(pLp > 0.0) || !(pLm > 0.0)) bad = true;
          const double tr = mn(theta_lin(ULp[0], UHp[0], mn(kPPEps, ULp[0])),
                                 theta_lin(ULm[0], UHm[0], mn(kPPEps, ULm[0])));
          double Tp[4], Tm[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            Tp[k] = ULp[k] + tr * (UHp[k] - ULp[k]);
            Tm[k] = ULm[k] + tr * (UHm[k] - ULm[k]);
          }
          const double tp =
              mn(theta_lin(pLp, pressure2(Tp[0], Tp[1], Tp[2], Tp[3], ph.gm1), mn(kPPEps, pLp)),
                   theta_lin(pLm, pressure2(Tm[0], Tm[1], Tm[2], Tm[3], ph.gm1), mn(kPPEps, pLm)));
          tpp = tr * tp;
        }
        if (bad) raise_flag(flags, FLAG_CELL_LOW);
      }
    }
    const double th = ts * tpp;
#pragma unroll
    for (int k = 0; k < 4; ++k) F[k] = FL[k] + th * (FH[k] - FL[k]);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) FO[k * nf + t] = F[k];
}

__global__ void __launch_bounds__(kBlock) k_cells(G2 g, const double* __restrict__ Un,
                                                  const double* __restrict__ Uk,
                                                  double* __restrict__ Uout,
                                                  const double* __restrict__ FX,
                                                  const double* __restrict__ FY,
                                                  const double* dt_dev, double dt_host, double ca,
                                                  double cb, int first, unsigned* flags) {
  const long nc = (long)g.n1 * g.n2;
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nc) return;
  const int i = (int)(t % g.n1), j = (int)(t / g.n1);
  const double dt = dt_dev ? *dt_dev : dt_host;
  const double mx = dt / g.dx, my = dt / g.dy;
  const long nfx = (long)g.n2 * (g.n1 + 1), nfy = (long)(g.n2 + 1) * g.n1;
  bool bad = false;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double dfx = FX[k * nfx + (long)j * (g.n1 + 1) + i + 1] - FX[k * nfx + (long)j * (g.n1 + 1) + i];
    const double dfy = FY[k * nfy + (long)(j + 1) * g.n1 + i] - FY[k * nfy + (long)j * g.n1 + i];
    const double fe = Uk[k * nc + t] - mx * dfx - my * dfy;
    const double o = first ? fe : ca * Un[k * nc + t] + cb * fe;
    if (!isfinite(o)) bad = true;
    Uout[k * nc + t] = o;
  }
  if (bad) raise_flag(flags, FLAG_NONFINITE);
}

// wall projection of a point value (no-slip: zero momentum; symmetry: zero
// normal momentum; density and internal energy kept)
__device__ __forceinline__ void project(int kind, int ax, double* V) {
  if (kind == BC_NOSLIP) {
    V[3] -= (V[1] * V[1] + V[2] * V[2]) / (2.0 * V[0]);
    V[1] = 0.0;
    V[2] = 0.0;
  } else if (kind == BC_SYMMETRY) {
    V[3] -= V[1 + ax] * V[1 + ax] / (2.0 * V[0]);
    V[1 + ax] = 0.0;
  }
}

__device__ __forceinline__ int wall_of(int bc) {
  return (bc == BC_NOSLIP || bc == BC_SYMMETRY) ? bc : -1;
}

// low-order LLF flux between lattice sites qa (minus) and qb (plus) along d
__device__ __forceinline__ void llf_pair(const G2& g, const Phys& ph, const double* __restrict__ LU,
                                         const double* __restrict__ LA,
                                         const double* __restrict__ LG, long qa, long qb, int d,
                                         double* F) {
  double Fa[4], Fb[4];
  site_flux(g, ph, LU, LA, LG, qa, d, Fa);
  site_flux(g, ph, LU, LA, LG, qb, d, Fb);
  const double ra = fabs(LA[d * g.ns + qa]) + LA[4 * g.ns + qa];
  const double rb = fabs(LA[d * g.ns + qb]) + LA[4 * g.ns + qb];
  const double ba = bvisc2(d, LU[qa], LA[2 * g.ns + qa], LG[qa], LG[g.ns + qa], LG[2 * g.ns + qa],
                           LG[3 * g.ns + qa], LG[4 * g.ns + qa], LG[5 * g.ns + qa], ph);
  const double bb = bvisc2(d, LU[qb], LA[2 * g.ns + qb], LG[qb], LG[g.ns + qb], LG[2 * g.ns + qb],
                           LG[3 * g.ns + qb], LG[4 * g.ns + qb], LG[5 * g.ns + qb], ph);
  const double lam = mx(ra, rb) + mx(ba, bb);
#pragma unroll
  for (int k = 0; k < 4; ++k) F[k] = 0.5 * (Fa[k] + Fb[k]) - 0.5 * lam * (LU[k * g.ns + qb] - LU[k * g.ns + qa]);
}

// point residual R at lattice site q (Sec. 2.2 point update)
__device__ __forceinline__ void point_residual(const G2& g, const Phys& ph,
                                               const double* __restrict__ LU,
                                               const double* __restrict__ LA,
                                               const double* __restrict__ LG, long q,
                                               double* R) {
#pragma unroll
  for (int k = 0; k < 4; ++k) R[k] = 0.0;
#pragma unroll
  for (int d = 0; d < 2; ++d) {
    const long st = d == 0 ? 1 : (long)g.LX;
    const double h = d == 0 ? g.dx : g.dy;
    const double i6h = 1.0 / (6.0 * h);
    double Us[5][4], u[5], v[5], p[5], T[5];
    double alpha = 0.0;
#pragma unroll
    for (int o = 0; o < 5; ++o) {
      const long s = q + (o - 2) * st;
#pragma unroll
      for (int k = 0; k < 4; ++k) Us[o][k] = LU[k * g.ns + s];
      u[o] = LA[s];
      v[o] = LA[g.ns + s];
      p[o] = LA[2 * g.ns + s];
      T[o] = LA[3 * g.ns + s];
      alpha = mx(alpha, fabs(d == 0 ? u[o] : v[o]) + LA[4 * g.ns + s]);
    }
    // inviscid part: D_c(F^c_d) + alpha/(6h) * fourth difference of U
    double Fc[5][4];
#pragma unroll
    for (int o = 0; o < 5; ++o) {
      const double ud = d == 0 ? u[o] : v[o];
      Fc[o][0] = Us[o][1 + d];
      Fc[o][1] = Us[o][1] * ud + (d == 0 ? p[o] : 0.0);
      Fc[o][2] = Us[o][2] * ud + (d == 1 ? p[o] : 0.0);
      Fc[o][3] = (Us[o][3] + p[o]) * ud;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double dF = dc5(Fc[0][k], Fc[1][k], Fc[3][k], Fc[4][k], i6h);
      const double dU = d4(Us[0][k], Us[1][k], Us[2][k], Us[3][k], Us[4][k]);
      R[k] -= dF + alpha * i6h * dU;
    }
    // compact D^{(d),2}(K_dd, Z)
    const double s4 = 4.0 / (h * h);
    const double mu = ph.mu, m43 = (4.0 / 3.0) * ph.mu;
    const double cu = bcol(u), cv = bcol(v), cT = bcol(T);
    const double fu = bform(u, u), fv = bform(v, v);
    if (d == 0) {
      R[1] += s4 * m43 * cu;
      R[2] += s4 * mu * cv;
      R[3] += s4 * (m43 * fu + mu * fv + ph.kap * cT);
    } else {
      R[1] += s4 * mu * cu;
      R[2] += s4 * m43 * cv;
      R[3] += s4 * (mu * fu + m43 * fv + ph.kap * cT);
    }
    // mixed term D_c^{(d)} (K_{d,o} D_c^{(o)} Z), o the other direction
    double m1[5], m2[5], m3[5];
#pragma unroll
    for (int o = 0; o < 5; ++o) {
      if (o == 2) {
        m1[o] = m2[o] = m3[o] = 0.0;
        continue;
      }
      const long s = q + (o - 2) * st;
      if (d == 0) {  // K_12 dZ/dy
        const double uy = LG[3 * g.ns + s], vy = LG[4 * g.ns + s];
        m1[o] = -(2.0 / 3.0) * mu * vy;
        m2[o] = mu * uy;
        m3[o] = mu * (v[o] * uy - (2.0 / 3.0) * u[o] * vy);
      } else {  // K_21 dZ/dx
        const double ux = LG[s], vx = LG[g.ns + s];
        m1[o] = mu * vx;
        m2[o] = -(2.0 / 3.0) * mu * ux;
        m3[o] = mu * (u[o] * vx - (2.0 / 3.0) * v[o] * ux);
      }
    }
    R[1] += dc5(m1[0], m1[1], m1[3], m1[4], i6h);
    R[2] += dc5(m2[0], m2[1], m2[3], m2[4], i6h);
    R[3] += dc5(m3[0], m3[1], m3[3], m3[4], i6h);
  }
}

__global__ void __launch_bounds__(kBlock) k_points(G2 g, Phys ph, const double* __restrict__ LU,
                                                   const double* __restrict__ LA,
                                                   const double* __restrict__ LG,
                                                   const double* __restrict__ Un,
                                                   double* __restrict__ Uout, const double* dt_dev,
                                                   double dt_host, double ca, double cb, int first,
                                                   unsigned* flags) {
  const int type = blockIdx.y;  // 0 xe, 1 ye, 2 co
  const int ni = type == 1 ? g.n1 : g.n1x;
  const int nj = type == 0 ? g.n2 : g.n2y;
  const long np = (long)ni * nj;
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= np) return;
  const int i = (int)(t % ni), j = (int)(t / ni);
  const int X = type == 1 ? 2 * i + 1 : 2 * i;
  const int Y = type == 0 ? 2 * j + 1 : 2 * j;
  const long q = lidx(g, X, Y);
  const double dt = dt_dev ? *dt_dev : dt_host;
  double R[4];
  point_residual(g, ph, LU, LA, LG, q, R);
  double U0[4], UH[4], out[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    U0[k] = LU[k * g.ns + q];
    UH[k] = U0[k] + dt * R[k];
  }
  bool bad = false;
  if (ph.lim & LIM_POINT) {
    double Fxp[4], Fxm[4], Fyp[4], Fym[4], UL[4];
    const long sx = 1, sy = g.LX;
    llf_pair(g, ph, LU, LA, LG, q, q + sx, 0, Fxp);
    llf_pair(g, ph, LU, LA, LG, q - sx, q, 0, Fxm);
    llf_pair(g, ph, LU, LA, LG, q, q + sy, 1, Fyp);
    llf_pair(g, ph, LU, LA, LG, q - sy, q, 1, Fym);
    const double cx = 2.0 * dt / g.dx, cy = 2.0 * dt / g.dy;
#pragma unroll
    for (int k = 0; k < 4; ++k) UL[k] = U0[k] - cx * (Fxp[k] - Fxm[k]) - cy * (Fyp[k] - Fym[k]);
    bool lbad = false;
    const double th = theta_pair2(UL, UH, ph.gm1, lbad);
    if (lbad) raise_flag(flags, FLAG_POINT_LOW);
#pragma unroll
    for (int k = 0; k < 4; ++k) out[k] = (th == 1.0) ? UH[k] : UL[k] + th * (UH[k] - UL[k]);
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k) out[k] = UH[k];
  }
  if (X == 0) project(wall_of(g.bc0), 0, out);
  if (X == 2 * g.n1) project(wall_of(g.bc1), 0, out);
  if (Y == 0) project(wall_of(g.bc2), 1, out);
  if (Y == 2 * g.n2) project(wall_of(g.bc3), 1, out);
  const long off = type == 0 ? g.off_xe : (type == 1 ? g.off_ye : g.off_co);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const long a = off + k * np + t;
    const double o = first ? out[k] : ca * Un[a] + cb * out[k];
    if (!isfinite(o)) bad = true;
    Uout[a] = o;
  }
  if (bad) raise_flag(flags, FLAG_NONFINITE);
}

inline unsigned nblk(long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

namespace afi {

hipError_t stage2d(const Geo& geo, const Phys& ph, const Work& w, const double* Un,
                   const double* Uk, double* Uout, const double* dt_dev, double dt_host,
                   StageCoef sc, hipStream_t s, Timer* tm) {
  const G2 g = make_g2(geo);
  AFI_TIMED(tm, 0, s,
            hipLaunchKernelGGL(k_lattice, dim3(nblk(g.ns)), dim3(kBlock), 0, s, g, ph, Uk, w.LU,
                               w.LA));
  const long ng = (long)(2 * g.n1 + 5) * (2 * g.n2 + 5);
  AFI_TIMED(tm, 1, s,
            hipLaunchKernelGGL(k_grad, dim3(nblk(ng)), dim3(kBlock), 0, s, g,
                               (const double*)w.LA, w.LG));
  const long ncp = (long)(g.n1 + 2) * (g.n2 + 2);
  AFI_TIMED(tm, 2, s,
            hipLaunchKernelGGL(k_cellpre, dim3(nblk(ncp)), dim3(kBlock), 0, s, g, ph, Uk, w.CP));
  const long nfx = (long)(g.n1 + 1) * g.n2, nfy = (long)g.n1 * (g.n2 + 1);
  AFI_TIMED(tm, 3, s,
            hipLaunchKernelGGL(k_face<0>, dim3(nblk(nfx)), dim3(kBlock), 0, s, g, ph,
                               (const double*)w.LU, (const double*)w.LA, (const double*)w.LG,
                               (const double*)w.CP, w.FX, dt_dev, dt_host, w.flags));
  AFI_TIMED(tm, 3, s,
            hipLaunchKernelGGL(k_face<1>, dim3(nblk(nfy)), dim3(kBlock), 0, s, g, ph,
                               (const double*)w.LU, (const double*)w.LA, (const double*)w.LG,
                               (const double*)w.CP, w.FY, dt_dev, dt_host, w.flags));
  const long nc = (long)g.n1 * g.n2;
  AFI_TIMED(tm, 4, s,
            hipLaunchKernelGGL(k_cells, dim3(nblk(nc)), dim3(kBlock), 0, s, g, Un, Uk, Uout,
                               (const double*)w.FX, (const double*)w.FY, dt_dev, dt_host, sc.a,
                               sc.b, sc.first, w.flags));
  const long npmax = (long)(g.n1 + 1) * (g.n2 + 1);
  AFI_TIMED(tm, 5, s,
            hipLaunchKernelGGL(k_points, dim3(nblk(npmax), 3), dim3(kBlock), 0, s, g, ph,
                               (const double*)w.LU, (const double*)w.LA, (const double*)w.LG, Un,
                               Uout, dt_dev, dt_host, sc.a, sc.b, sc.first, w.flags));
  return hipGetLastError();
}

}  // namespace afi
