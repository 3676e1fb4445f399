// af_kern1d.hip -- one SSP-RK3 stage of the 1D compact AF method (Sec. 2.1)
// on gfx950, FP64.  Same pipeline as the 2D stage (lattice, gradients,
// per-cell low-order data, limited face fluxes, cell update, point update),
// with U = (rho, rho u, E), W = (rho, u, p), Z = (0, u, T) and
//   K(W) = [[0,0,0],[0,4mu/3,0],[0,4mu u/3,kappa]].
#include "af_device.hpp"
#include "af_internal.hpp"

using namespace afd;

namespace {

constexpr int kBlock = 256;

struct G1 {
  int n, np, LX;
  long off_pts;
  int bc0, bc1;
  double dx;
  double dl[3], dr[3];  // states of Dirichlet sides (x-low, x-high)
  // inside a step attempt: stop once the attempt's flag word is set (it is
  // rejected and the stage output is never read)
  int skip_flagged;
  unsigned* fl;
};

__device__ __forceinline__ bool rejected(const G1& g) {
  return g.skip_flagged && peek_flags(g.fl) != 0u;
}

__device__ __forceinline__ double pt(const G1& g, const double* __restrict__ U, int X, int k) {
  if (X == 2 * g.n && g.np == g.n) X = 0;
  return U[g.off_pts + (long)k * g.np + (X >> 1)];
}

__device__ __forceinline__ void cell_image1(const G1& g, const double* __restrict__ U, int i,
                                            double* V) {
  // beyond a Dirichlet side, its state
  if ((i < 0 && g.bc0 == BC_DIRICHLET) || (i >= g.n && g.bc1 == BC_DIRICHLET)) {
    const double* d = i < 0 ? g.dl : g.dr;
#pragma unroll
    for (int k = 0; k < 3; ++k) V[k] = d[k];
    return;
  }
  int kind;
  const int Xi = axis_image(2 * i + 1, 2 * g.n, g.bc0, g.bc1, kind);
  const double s = (kind == BC_NOSLIP || kind == BC_SYMMETRY) ? -1.0 : 1.0;
  const int ii = Xi >> 1;
  V[0] = U[ii];
  V[1] = s * U[g.n + ii];
  V[2] = U[2 * g.n + ii];
}

__global__ void __launch_bounds__(kBlock) k_lattice1(G1 g, Phys ph, const double* __restrict__ U,
                                                     double* __restrict__ LU,
                                                     double* __restrict__ LA) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.LX || rejected(g)) return;
  const int X = t - kMargin;
  int kind;
  const int Xi = axis_image(X, 2 * g.n, g.bc0, g.bc1, kind);
  const double s = (kind == BC_NOSLIP || kind == BC_SYMMETRY) ? -1.0 : 1.0;
  double V[3];
  if (Xi & 1) {
    const int i = Xi >> 1;
    double Ub[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      Ub[k] = U[k * g.n + i];
      V[k] = (6.0 * Ub[k] - (pt(g, U, Xi - 1, k) + pt(g, U, Xi + 1, k))) / 4.0;
    }
    if (ph.lim & LIM_CENTRE) {
      if (!(Ub[0] > 0.0)) {
#pragma unroll
        for (int k = 0; k < 3; ++k) V[k] = Ub[k];
      } else {
        bool bad = false;
        const double th = theta_pair1(Ub, V, ph.gm1, bad, ph.lim & LIM_PEXACT);
        if (th < 1.0) {
#pragma unroll
          for (int k = 0; k < 3; ++k) V[k] = Ub[k] + th * (V[k] - Ub[k]);
        }
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < 3; ++k) V[k] = pt(g, U, Xi, k);
  }
  V[1] *= s;
  if ((X < 0 && g.bc0 == BC_DIRICHLET) || (X > 2 * g.n && g.bc1 == BC_DIRICHLET)) {
    const double* d = X < 0 ? g.dl : g.dr;
#pragma unroll
    for (int k = 0; k < 3; ++k) V[k] = d[k];
  }
  const double u = V[1] / V[0];
  const double p = pressure1(V[0], V[1], V[2], ph.gm1);
#pragma unroll
  for (int k = 0; k < 3; ++k) LU[k * g.LX + t] = V[k];
  LA[0 * g.LX + t] = u;
  LA[1 * g.LX + t] = p;
  LA[2 * g.LX + t] = p / V[0];
  LA[3 * g.LX + t] = sqrt(ph.gam * p / V[0]);
}

__global__ void __launch_bounds__(kBlock) k_grad1(G1 g, const double* __restrict__ LA,
                                                  double* __restrict__ LG) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * g.n + 5 || rejected(g)) return;
  const int q = t - 2 + kMargin;
  const double i6 = 1.0 / (6.0 * g.dx);
  const double* u = LA;
  const double* T = LA + 2 * g.LX;
  LG[q] = dc5(u[q - 2], u[q - 1], u[q + 1], u[q + 2], i6);
  LG[g.LX + q] = dc5(T[q - 2], T[q - 1], T[q + 1], T[q + 2], i6);
}

// CP layout (cells -1..n): 0-2 F, 3 rs, 4 b, 5 phi1, 6 phi2, 7-9 average

__global__ void __launch_bounds__(kBlock) k_cellpre1(G1 g, Phys ph, const double* __restrict__ U,
                                                     double* __restrict__ CP) {
  const int nc = g.n + 2;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nc || rejected(g)) return;
  const int i = t - 1;
  double C0[3], Cm[3], Cp[3];
  cell_image1(g, U, i, C0);
  cell_image1(g, U, i - 1, Cm);
  cell_image1(g, U, i + 1, Cp);
  const double p0 = pressure1(C0[0], C0[1], C0[2], ph.gm1);
  const double pm = pressure1(Cm[0], Cm[1], Cm[2], ph.gm1);
  const double pp = pressure1(Cp[0], Cp[1], Cp[2], ph.gm1);
  const double u0 = C0[1] / C0[0], um = Cm[1] / Cm[0], up = Cp[1] / Cp[0];
  const double i2 = 1.0 / (2.0 * g.dx);
  const double ux = (up - um) * i2;
  const double Tx = (pp / Cp[0] - pm / Cm[0]) * i2;
  const double tau = (4.0 / 3.0) * ph.mu * ux;
  CP[0 * nc + t] = C0[1];
  CP[1 * nc + t] = C0[1] * u0 + p0 - tau;
  CP[2 * nc + t] = (C0[2] + p0) * u0 - (u0 * tau + ph.kap * Tx);
  CP[3 * nc + t] = fabs(u0) + sqrt(ph.gam * p0 / C0[0]);
  CP[4 * nc + t] = bvisc1(C0[0], p0, ux, Tx, ph);
  CP[5 * nc + t] = fabs(pp - 2.0 * p0 + pm) / fabs(pp + 2.0 * p0 + pm);
  CP[6 * nc + t] = mx(-ux / sqrt(ux * ux + kDucros), 0.0);
#pragma unroll
  for (int k = 0; k < 3; ++k) CP[(7 + k) * nc + t] = C0[k];
}

__device__ __forceinline__ void site_flux1(const G1& g, const Phys& ph, const double* __restrict__ LU,
                                           const double* __restrict__ LA,
                                           const double* __restrict__ LG, int q, double* F) {
  const double m = LU[g.LX + q], E = LU[2 * g.LX + q];
  const double u = LA[q], p = LA[g.LX + q];
  const double tau = (4.0 / 3.0) * ph.mu * LG[q];
  F[0] = m;
  F[1] = m * u + p - tau;
  F[2] = (E + p) * u - (u * tau + ph.kap * LG[g.LX + q]);
}

__global__ void __launch_bounds__(kBlock) k_face1(G1 g, Phys ph, const double* __restrict__ LU,
                                                  const double* __restrict__ LA,
                                                  const double* __restrict__ LG,
                                                  const double* __restrict__ CP,
                                                  double* __restrict__ FO, const double* dt_dev,
                                                  double dt_host, unsigned* flags) {
  const int nf = g.n + 1;
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf || rejected(g)) return;
  const double dt = dt_dev ? *dt_dev : dt_host;
  double FH[3], F[3];
  site_flux1(g, ph, LU, LA, LG, 2 * f + kMargin, FH);
  const int limc = ph.lim & (LIM_SMOOTH | LIM_PP | LIM_LOWONLY);
  if (!limc) {
#pragma unroll
    for (int k = 0; k < 3; ++k) F[k] = FH[k];
  } else {
    const int nc = g.n + 2;
    const int a = f, b = f + 1;  // cells f-1 and f in the ringed grid
    const double lam = mx(CP[3 * nc + a], CP[3 * nc + b]) + mx(CP[4 * nc + a], CP[4 * nc + b]);
    double FL[3], Ua[3], Ub[3], Fa[3], Fb[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      Ua[k] = CP[(7 + k) * nc + a];
      Ub[k] = CP[(7 + k) * nc + b];
      Fa[k] = CP[k * nc + a];
      Fb[k] = CP[k * nc + b];
      FL[k] = 0.5 * (Fa[k] + Fb[k]) - 0.5 * lam * (Ub[k] - Ua[k]);
    }
    double ts = 1.0, tpp = 1.0;
    if (ph.lim & LIM_LOWONLY) {
      ts = 0.0;
      tpp = 0.0;
    } else {
      if (ph.lim & LIM_SMOOTH)
        ts = exp(-ph.Cs * mx(CP[5 * nc + a], CP[5 * nc + b]) * mx(CP[6 * nc + a], CP[6 * nc + b]));
      if (ph.lim & LIM_PP) {
        const double m2 = 2.0 * dt / g.dx;
        double ULp[3], UHp[3], ULm[3], UHm[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const double Fs = FL[k] + ts * (FH[k] - FL[k]);
          ULp[k] = Ua[k] - m2 * (FL[k] - Fa[k]);
          UHp[k] = Ua[k] - m2 * (Fs - Fa[k]);
          ULm[k] = Ub[k] - m2 * (Fb[k] - FL[k]);
          UHm[k] = Ub[k] - m2 * (Fb[k] - Fs);
        }
        tpp = 0.0;
        bool bad = false;
        if (!(ULp[0] > 0.0) || !(ULm[0] > 0.0)) {
          bad = true;
        } else {
          const double pLp = pressure1(ULp[0], ULp[1], ULp[2], ph.gm1);
          const double pLm = pressure1(ULm[0], ULm[1], ULm[2], ph.gm1);
          if (!(pLp > 0.0) || !(pLm > 0.0)) bad = true;
          const double tr = mn(theta_lin(ULp[0], UHp[0], mn(kPPEps, ULp[0])),
                                 theta_lin(ULm[0], UHm[0], mn(kPPEps, ULm[0])));
          double Tp[3], Tm[3];
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            Tp[k] = ULp[k] + tr * (UHp[k] - ULp[k]);
            Tm[k] = ULm[k] + tr * (UHm[k] - ULm[k]);
          }
          const bool ex = ph.lim & LIM_PEXACT;
          const double tp = mn(theta_p1(ULp, pLp, Tp, mn(kPPEps, pLp), ph.gm1, ex),
                               theta_p1(ULm, pLm, Tm, mn(kPPEps, pLm), ph.gm1, ex));
          tpp = tr * tp;
        }
        if (bad) raise_flag(flags, FLAG_CELL_LOW);
      }
    }
    const double th = ts * tpp;
#pragma unroll
    for (int k = 0; k < 3; ++k) F[k] = FL[k] + th * (FH[k] - FL[k]);
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) FO[k * nf + f] = F[k];
}

__global__ void __launch_bounds__(kBlock) k_cells1(G1 g, const double* __restrict__ Un,
                                                   const double* __restrict__ Uk,
                                                   double* __restrict__ Uout,
                                                   const double* __restrict__ FX,
                                                   const double* dt_dev, double dt_host, double ca,
                                                   double cb, int first, unsigned* flags) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.n || rejected(g)) return;
  const double dt = dt_dev ? *dt_dev : dt_host;
  const double m = dt / g.dx;
  const int nf = g.n + 1;
  bool bad = false;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double fe = Uk[k * g.n + i] - m * (FX[k * nf + i + 1] - FX[k * nf + i]);
    const double o = first ? fe : ca * Un[k * g.n + i] + cb * fe;
    if (!isfinite(o)) bad = true;
    Uout[k * g.n + i] = o;
  }
  if (bad) raise_flag(flags, FLAG_NONFINITE);
}

// low-order data of site o (1..3) of the five-site low-order point lattice
// V[0..4] (point, average, point, average, point): total flux with the
// central-difference gradient over its neighbours, |u|+c and b
__device__ __forceinline__ void lo_site1(const Phys& ph, const double (&V)[5][3],
                                         const double* u, const double* p, const double* T,
                                         const double* c, int o, double ih, double* F,
                                         double& r, double& b) {
  const double ux = (u[o + 1] - u[o - 1]) * ih, Tx = (T[o + 1] - T[o - 1]) * ih;
  const double tau = (4.0 / 3.0) * ph.mu * ux;
  F[0] = V[o][1];
  F[1] = V[o][1] * u[o] + p[o] - tau;
  F[2] = (V[o][2] + p[o]) * u[o] - (u[o] * tau + ph.kap * Tx);
  r = fabs(u[o]) + c[o];
  b = bvisc1(V[o][0], p[o], ux, Tx, ph);
}

__global__ void __launch_bounds__(kBlock) k_points1(G1 g, Phys ph, const double* __restrict__ LU,
                                                    const double* __restrict__ LA,
                                                    const double* __restrict__ CP,
                                                    const double* __restrict__ Un,
                                                    double* __restrict__ Uout, const double* dt_dev,
                                                    double dt_host, double ca, double cb, int first,
                                                    unsigned* flags) {
  const int k0 = blockIdx.x * blockDim.x + threadIdx.x;
  if (k0 >= g.np || rejected(g)) return;
  const int X = 2 * k0;
  const int q = X + kMargin;
  const double dt = dt_dev ? *dt_dev : dt_host;
  const double i6h = 1.0 / (6.0 * g.dx);
  double Us[5][3], u[5], p[5], T[5];
  double alpha = 0.0;
#pragma unroll
  for (int o = 0; o < 5; ++o) {
    const int s = q + o - 2;
#pragma unroll
    for (int k = 0; k < 3; ++k) Us[o][k] = LU[k * g.LX + s];
    u[o] = LA[s];
    p[o] = LA[g.LX + s];
    T[o] = LA[2 * g.LX + s];
    alpha = mx(alpha, fabs(u[o]) + LA[3 * g.LX + s]);
  }
  double Fc[5][3];
#pragma unroll
  for (int o = 0; o < 5; ++o) {
    Fc[o][0] = Us[o][1];
    Fc[o][1] = Us[o][1] * u[o] + p[o];
    Fc[o][2] = (Us[o][2] + p[o]) * u[o];
  }
  double R[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double dF = dc5(Fc[0][k], Fc[1][k], Fc[3][k], Fc[4][k], i6h);
    const double dU = d4(Us[0][k], Us[1][k], Us[2][k], Us[3][k], Us[4][k]);
    R[k] = -(dF + alpha * i6h * dU);
  }
  const double s4 = 4.0 / (g.dx * g.dx);
  const double m43 = (4.0 / 3.0) * ph.mu;
  R[1] += s4 * m43 * bcol(u);
  R[2] += s4 * (m43 * bform(u, u) + ph.kap * bcol(T));
  double U0[3], UH[3], out[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    U0[k] = Us[2][k];
    UH[k] = U0[k] + dt * R[k];
  }
  if (ph.lim & LIM_POINT) {
    // low-order LLF scheme on the lattice of point values (X-2, X, X+2) and
    // cell averages (X-1, X+1: ring cells k0 and k0+1), Sec. 3.4
    const int nc = g.n + 2;
    double V[5][3], lu[5], lp[5], lT[5], lc[5];
#pragma unroll
    for (int o = 0; o < 5; o += 2) {
#pragma unroll
      for (int k = 0; k < 3; ++k) V[o][k] = Us[o][k];
      lu[o] = u[o];
      lp[o] = p[o];
      lT[o] = T[o];
      lc[o] = LA[3 * g.LX + q + o - 2];
    }
#pragma unroll
    for (int o = 1; o < 5; o += 2) {
#pragma unroll
      for (int k = 0; k < 3; ++k) V[o][k] = CP[(7 + k) * nc + k0 + (o >> 1)];
      const double ir = 1.0 / V[o][0];
      lu[o] = V[o][1] * ir;
      lp[o] = pressure1(V[o][0], V[o][1], V[o][2], ph.gm1);
      lT[o] = lp[o] * ir;
      lc[o] = sqrt(ph.gam * lT[o]);
    }
    const double ih = 1.0 / g.dx;
    double F1[3], F2[3], F3[3], r1, r2, r3, b1, b2, b3;
    lo_site1(ph, V, lu, lp, lT, lc, 1, ih, F1, r1, b1);
    lo_site1(ph, V, lu, lp, lT, lc, 2, ih, F2, r2, b2);
    lo_site1(ph, V, lu, lp, lT, lc, 3, ih, F3, r3, b3);
    const double lp23 = mx(r2, r3) + mx(b2, b3), lm12 = mx(r1, r2) + mx(b1, b2);
    double Fp[3], Fm[3], UL[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      Fp[k] = 0.5 * (F2[k] + F3[k]) - 0.5 * lp23 * (V[3][k] - V[2][k]);
      Fm[k] = 0.5 * (F1[k] + F2[k]) - 0.5 * lm12 * (V[2][k] - V[1][k]);
    }
    const double c2 = 2.0 * dt / g.dx;
#pragma unroll
    for (int k = 0; k < 3; ++k) UL[k] = U0[k] - c2 * (Fp[k] - Fm[k]);
    bool lbad = false;
    double th = theta_pair1(UL, UH, ph.gm1, lbad, ph.lim & LIM_PEXACT);
    if (ph.lim & LIM_LOWONLY) th = 0.0;
    if (lbad) raise_flag(flags, FLAG_POINT_LOW);
#pragma unroll
    for (int k = 0; k < 3; ++k) out[k] = (th == 1.0) ? UH[k] : UL[k] + th * (UH[k] - UL[k]);
  } else {
#pragma unroll
    for (int k = 0; k < 3; ++k) out[k] = UH[k];
  }
  const int wl = (g.bc0 == BC_NOSLIP || g.bc0 == BC_SYMMETRY);
  const int wr = (g.bc1 == BC_NOSLIP || g.bc1 == BC_SYMMETRY);
  if ((X == 0 && wl) || (X == 2 * g.n && wr)) {
    out[2] -= out[1] * out[1] / (2.0 * out[0]);
    out[1] = 0.0;
  }
  // a point on a Dirichlet side keeps the prescribed state
  if ((X == 0 && g.bc0 == BC_DIRICHLET) || (X == 2 * g.n && g.bc1 == BC_DIRICHLET)) {
    const double* d = X == 0 ? g.dl : g.dr;
#pragma unroll
    for (int k = 0; k < 3; ++k) out[k] = d[k];
  }
  bool bad = false;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const long a = g.off_pts + (long)k * g.np + k0;
    const double o = first ? out[k] : ca * Un[a] + cb * out[k];
    if (!isfinite(o)) bad = true;
    Uout[a] = o;
  }
  if (bad) raise_flag(flags, FLAG_NONFINITE);
}

inline unsigned nblk(long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

namespace afi {

hipError_t stage1d(const Geo& geo, const Phys& ph, const Work& w, const double* Un,
                   const double* Uk, double* Uout, const double* dt_dev, double dt_host,
                   StageCoef sc, hipStream_t s, Timer* tm) {
  G1 g;
  g.n = geo.n1;
  g.np = geo.n1x;
  g.LX = geo.LX;
  g.off_pts = geo.off_pts;
  g.bc0 = geo.bc[0];
  g.bc1 = geo.bc[1];
  g.dx = geo.dx;
  for (int k = 0; k < 3; ++k) {
    g.dl[k] = geo.bcstate[0][k];
    g.dr[k] = geo.bcstate[1][k];
  }
  g.skip_flagged = sc.skip_flagged;
  g.fl = w.flags;
  AFI_TIMED(tm, 0, s,
            hipLaunchKernelGGL(k_lattice1, dim3(nblk(g.LX)), dim3(kBlock), 0, s, g, ph, Uk, w.LU,
                               w.LA));
  AFI_TIMED(tm, 1, s,
            hipLaunchKernelGGL(k_grad1, dim3(nblk(2 * g.n + 5)), dim3(kBlock), 0, s, g,
                               (const double*)w.LA, w.LG));
  AFI_TIMED(tm, 2, s,
            hipLaunchKernelGGL(k_cellpre1, dim3(nblk(g.n + 2)), dim3(kBlock), 0, s, g, ph, Uk,
                               w.CP));
  AFI_TIMED(tm, 3, s,
            hipLaunchKernelGGL(k_face1, dim3(nblk(g.n + 1)), dim3(kBlock), 0, s, g, ph,
                               (const double*)w.LU, (const double*)w.LA, (const double*)w.LG,
                               (const double*)w.CP, w.FX, dt_dev, dt_host, w.flags));
  AFI_TIMED(tm, 4, s,
            hipLaunchKernelGGL(k_cells1, dim3(nblk(g.n)), dim3(kBlock), 0, s, g, Un, Uk, Uout,
                               (const double*)w.FX, dt_dev, dt_host, sc.a, sc.b, sc.first,
                               w.flags));
  AFI_TIMED(tm, 5, s,
            hipLaunchKernelGGL(k_points1, dim3(nblk(g.np)), dim3(kBlock), 0, s, g, ph,
                               (const double*)w.LU, (const double*)w.LA, (const double*)w.CP, Un,
                               Uout, dt_dev, dt_host, sc.a, sc.b, sc.first, w.flags));
  return hipGetLastError();
}

}  // namespace afi
