/*
 * af_oracle.c -- plain FP64 CPU oracle of the compact fourth-order
 * positivity-preserving Active Flux method for compressible Navier-Stokes
 * (Duan, Barsukow, Klingenberg: "A compact high-order and positivity-
 * preserving active flux method for compressible Navier-Stokes equations on
 * Cartesian meshes").
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark; never by the product path.  It shares no
 * code with the HIP library.
 *
 * The code follows the paper's formulas one site at a time, in the paper's
 * order, with no blocking, fusion or algebraic restructuring.  Where the paper
 * is silent the following readings are taken (numbered as in the design
 * notes):
 *   R-centre : the Simpson centre value is scaled toward the cell average
 *              with the same density-then-pressure Theta rule as the fluxes
 *              (Remark after the pressure limiting, Sec. 3.3).
 *   R-alpha  : in 2D the FVS coefficient alpha of a point and direction is the
 *              max of |u_l|+c over the five lattice sites of that direction
 *              (Sec. 2.1 definition of alpha, applied per direction, Sec. 2.2).
 *   R-tang   : the tangential gradient at face points is D_c along the face
 *              line (Sec. 2.2 only gives the normal one).
 *   R-S      : the low-order gradient S_i of a cell is the two-point central
 *              difference of Z(average) in every direction (Sec. 3.1).
 *   R-point  : the low-order point scheme is the LLF scheme (eq. of the low
 *              face fluxes, Sec. 3.1) on the half-spaced lattice around the
 *              point: U^L = U - sum_l (2 dt/dx_l) (F^L(z,z+) - F^L(z-,z)).
 *              Its states are point values and, at centre sites, cell
 *              averages: the states the positivity theorem (end of Sec. 3.4)
 *              assumes admissible.  Its gradients S are central differences
 *              of Z over the neighbouring sites of that lattice, as the cell
 *              scheme's S is of Z(average).  Blend by Theta on density then
 *              pressure (Sec. 3.4).
 *   R-bc     : ghost lattice sites are images of interior sites: mirror about
 *              the wall line (walls; no-slip flips both momenta, symmetry the
 *              normal one), zero-order copy (outflow: even ghost lines copy the
 *              boundary point line, odd ones the first cell line), wrap
 *              (periodic).  Point values on walls are projected after each
 *              stage (no-slip: momentum 0; symmetry: normal momentum 0;
 *              internal energy kept).
 *   R-eps    : eps = min(1e-13, z(U^L)) per state; a state with rho<=0 is
 *              flagged and its blend parameter set to 0.
 *   R-pquad  : (optional, ORC_LIM_PEXACT) theta^p is the largest blend
 *              keeping the pressure >= eps on the whole segment (where
 *              p(blend) = eps, a quadratic once multiplied by the blended
 *              density), in place of the linear bound that the concavity of
 *              p gives (Sec. 3.3); 0 where p(U^L) is at the 1e-13 floor, as
 *              under the linear rule.  It is never below the linear one.
 *   R-blend  : final cell flux F^L + theta^s theta^rho theta^p (F^H - F^L);
 *              with every cell limiter switched off the flux is F^H itself;
 *              a point whose blend parameter is 1 keeps U^H itself.
 */
#include "af_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PP_EPS 1.0e-13      /* positivity epsilon, Sec. 3.3 */
#define DUCROS_EPS 1.0e-13  /* modified Ducros regularisation, Sec. 3.2 */
#define GM 4                /* ghost margin of the half lattice */

/* max/min that return NaN if either argument is NaN, so that an inadmissible
 * state anywhere in a stencil makes the stage non-finite (and flagged) */
static double dmax(double a, double b) { return (a != a || b != b) ? a + b : (a > b ? a : b); }
static double dmin(double a, double b) { return (a != a || b != b) ? a + b : (a < b ? a : b); }

int orc_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* finite-difference operators on one lattice line, offsets -2..2 -> z[0..4] */
/* (Sec. 2.1: biased D+, D-, central D_c, compact D^2)                       */
/* ------------------------------------------------------------------------ */

double orc_op_dplus(const double* z, double dx) {
  return (z[0] - 6.0 * z[1] + 3.0 * z[2] + 2.0 * z[3]) / (3.0 * dx);
}

double orc_op_dminus(const double* z, double dx) {
  return (-2.0 * z[1] - 3.0 * z[2] + 6.0 * z[3] - z[4]) / (3.0 * dx);
}

double orc_op_dc(const double* z, double dx) {
  return (z[0] - 8.0 * z[1] + 8.0 * z[3] - z[4]) / (6.0 * dx);
}

/* B = [0 0; 0 M] - [M 0; 0 0], rows/cols ordered -2..2 (eq. of the compact
 * second-derivative coefficients, Sec. 2.1) */
static const double Mmat[4][4] = {
    {1.0 / 8.0, -1.0 / 6.0, 1.0 / 24.0, 0.0},
    {-1.0 / 6.0, -3.0 / 8.0, 2.0 / 3.0, -1.0 / 8.0},
    {1.0 / 8.0, -2.0 / 3.0, 3.0 / 8.0, 1.0 / 6.0},
    {0.0, -1.0 / 24.0, 1.0 / 6.0, -1.0 / 8.0}};

static void build_B(double B[5][5]) {
  for (int r = 0; r < 5; ++r)
    for (int c = 0; c < 5; ++c) B[r][c] = 0.0;
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) {
      B[r + 1][c + 1] += Mmat[r][c];
      B[r][c] -= Mmat[r][c];
    }
}

double orc_op_d2(const double* k, const double* z, double dx) {
  double B[5][5];
  build_B(B);
  double s = 0.0;
  for (int m = 0; m < 5; ++m)
    for (int n = 0; n < 5; ++n) s += B[m][n] * k[m] * z[n];
  return 4.0 / (dx * dx) * s;
}

/* Theta of the linear scaling rule (Sec. 3.3), defined for zL >= eps */
double orc_Theta(double zL, double zH, double eps) {
  if (zH < eps) return (zL - eps) / (zL - zH);
  return 1.0;
}

/* ------------------------------------------------------------------------ */
/* physics: fluxes, closures, admissible set (Sec. 1, Sec. 2, Sec. 3.1)      */
/* ------------------------------------------------------------------------ */

static int ncomp(const orc_cfg* c) { return c->dim == 1 ? 3 : 4; }
static double kappa_of(const orc_cfg* c) {
  return c->gamma * c->mu / ((c->gamma - 1.0) * c->Pr);
}

double orc_pressure(const orc_cfg* c, const double* U) {
  if (c->dim == 1) return (c->gamma - 1.0) * (U[2] - U[1] * U[1] / (2.0 * U[0]));
  return (c->gamma - 1.0) * (U[3] - (U[1] * U[1] + U[2] * U[2]) / (2.0 * U[0]));
}

/* primitive W: 1D (rho,u,p), 2D (rho,u,v,p) */
static void prim(const orc_cfg* c, const double* U, double* W) {
  if (c->dim == 1) {
    W[0] = U[0];
    W[1] = U[1] / U[0];
    W[2] = orc_pressure(c, U);
  } else {
    W[0] = U[0];
    W[1] = U[1] / U[0];
    W[2] = U[2] / U[0];
    W[3] = orc_pressure(c, U);
  }
}

/* Z = (0,u,T) or (0,u,v,T), T = p/rho */
static void zvar(const orc_cfg* c, const double* W, double* Z) {
  if (c->dim == 1) {
    Z[0] = 0.0;
    Z[1] = W[1];
    Z[2] = W[2] / W[0];
  } else {
    Z[0] = 0.0;
    Z[1] = W[1];
    Z[2] = W[2];
    Z[3] = W[3] / W[0];
  }
}

/* spectral radius |u_l| + c, c = sqrt(gamma p / rho) (Lemma on the inviscid split) */
static double rho_spec(const orc_cfg* c, int dir, const double* W) {
  double p = c->dim == 1 ? W[2] : W[3];
  return fabs(W[1 + dir]) + sqrt(c->gamma * p / W[0]);
}

/* inviscid flux F^c_l (eq. of the directional fluxes) */
void orc_flux_c(const orc_cfg* c, int dir, const double* U, double* F) {
  double p = orc_pressure(c, U);
  if (c->dim == 1) {
    double u = U[1] / U[0];
    F[0] = U[0] * u;
    F[1] = U[1] * u + p;
    F[2] = (U[2] + p) * u;
    return;
  }
  double ul = U[1 + dir] / U[0];
  F[0] = U[0] * ul;
  F[1] = U[1] * ul + (dir == 0 ? p : 0.0);
  F[2] = U[2] * ul + (dir == 1 ? p : 0.0);
  F[3] = (U[3] + p) * ul;
}

/* diffusion matrices.  1D: K(W) (Sec. 2.1).  2D: K_lm(W) (Sec. 2.2). */
static void kmat1(const orc_cfg* c, const double* W, double K[3][3]) {
  double mu = c->mu, ka = kappa_of(c);
  memset(K, 0, sizeof(double) * 9);
  K[1][1] = 4.0 / 3.0 * mu;
  K[2][1] = 4.0 / 3.0 * mu * W[1];
  K[2][2] = ka;
}

static void kmat2(const orc_cfg* c, int l, int m, const double* W, double K[4][4]) {
  double mu = c->mu, ka = kappa_of(c), u = W[1], v = W[2];
  memset(K, 0, sizeof(double) * 16);
  if (l == 0 && m == 0) {
    K[1][1] = 4.0 / 3.0 * mu;
    K[2][2] = mu;
    K[3][1] = 4.0 / 3.0 * mu * u;
    K[3][2] = mu * v;
    K[3][3] = ka;
  } else if (l == 1 && m == 1) {
    K[1][1] = mu;
    K[2][2] = 4.0 / 3.0 * mu;
    K[3][1] = mu * u;
    K[3][2] = 4.0 / 3.0 * mu * v;
    K[3][3] = ka;
  } else if (l == 0 && m == 1) {
    K[1][2] = -2.0 / 3.0 * mu;
    K[2][1] = mu;
    K[3][1] = mu * v;
    K[3][2] = -2.0 / 3.0 * mu * u;
  } else {
    K[1][2] = mu;
    K[2][1] = -2.0 / 3.0 * mu;
    K[3][1] = -2.0 / 3.0 * mu * v;
    K[3][2] = mu * u;
  }
}

static void matvec3(double K[3][3], const double* z, double* y) {
  for (int r = 0; r < 3; ++r) y[r] = K[r][0] * z[0] + K[r][1] * z[1] + K[r][2] * z[2];
}
static void matvec4(double K[4][4], const double* z, double* y) {
  for (int r = 0; r < 4; ++r)
    y[r] = K[r][0] * z[0] + K[r][1] * z[1] + K[r][2] * z[2] + K[r][3] * z[3];
}

/* viscous flux F^v_l(U,S): 1D K(W) S; 2D K_l1 S_x + K_l2 S_y (S = [Sx(4),Sy(4)]) */
void orc_flux_v(const orc_cfg* c, int dir, const double* U, const double* S, double* F) {
  double W[4];
  prim(c, U, W);
  if (c->dim == 1) {
    double K[3][3];
    kmat1(c, W, K);
    matvec3(K, S, F);
    return;
  }
  double K[4][4], a[4], b[4];
  kmat2(c, dir, 0, W, K);
  matvec4(K, S, a);
  kmat2(c, dir, 1, W, K);
  matvec4(K, S + 4, b);
  for (int r = 0; r < 4; ++r) F[r] = a[r] + b[r];
}

/* b_l of the viscous LF splitting lemma, from the stress tensor and heat flux
 * definitions (Newton/Fourier closure, Sec. 1) */
double orc_bvisc(const orc_cfg* c, int dir, const double* U, const double* S) {
  double W[4];
  prim(c, U, W);
  double mu = c->mu, ka = kappa_of(c);
  double rho = W[0];
  double p = c->dim == 1 ? W[2] : W[3];
  double e = p / ((c->gamma - 1.0) * rho);
  double ql, tau2;
  if (c->dim == 1) {
    double ux = S[1], Tx = S[2];
    double tau = mu * (2.0 * ux - 2.0 / 3.0 * ux);
    ql = -ka * Tx;
    tau2 = tau * tau;
  } else {
    double ux = S[1], vx = S[2], Tx = S[3];
    double uy = S[5], vy = S[6], Ty = S[7];
    double div = ux + vy;
    double txx = mu * (2.0 * ux - 2.0 / 3.0 * div);
    double tyy = mu * (2.0 * vy - 2.0 / 3.0 * div);
    double txy = mu * (uy + vx);
    if (dir == 0) {
      ql = -ka * Tx;
      tau2 = txx * txx + txy * txy;
    } else {
      ql = -ka * Ty;
      tau2 = txy * txy + tyy * tyy;
    }
  }
  double r2 = rho * rho;
  return (sqrt(r2 * ql * ql + 2.0 * r2 * e * tau2) + rho * fabs(ql)) / (2.0 * r2 * e);
}

/* total flux F_l = F^c_l - F^v_l (lemma on the total flux) */
static void flux_tot(const orc_cfg* c, int dir, const double* U, const double* S, double* F) {
  double Fc[4], Fv[4];
  orc_flux_c(c, dir, U, Fc);
  orc_flux_v(c, dir, U, S, Fv);
  for (int r = 0; r < ncomp(c); ++r) F[r] = Fc[r] - Fv[r];
}

/* theta^p by the exact rule (reading R-pquad): the largest t in [0, 1] such
 * that p(UL + s (UT - UL)) >= eps for every s in [0, t].  With positive
 * density along the segment (theta^rho has made it so) p is concave on it,
 * so the s with p >= eps form an interval that holds 0, and its end is found
 * by bisection on the pressure of the state as formed (the iteration stops
 * when the bracket no longer shrinks).  t = 1 if p(UT) >= eps.  Where p(UL)
 * is itself at the floor (eps = p(UL), at most 1e-13) the blend is 0, as
 * under the linear rule: the crossing would leave the state at that floor,
 * below the rounding of E - |m|^2 / (2 rho). */
double orc_theta_p_root(const orc_cfg* c, const double* UL, const double* UT, double eps) {
  int nc = ncomp(c);
  /* not below eps (a non-finite pressure included, as in orc_Theta) */
  if (!(orc_pressure(c, UT) < eps)) return 1.0;
  if (!(orc_pressure(c, UL) > eps)) return 0.0;
  double lo = 0.0, hi = 1.0, W[4];
  for (int it = 0; it < 1100; ++it) {
    double mid = 0.5 * (lo + hi);
    if (!(mid > lo && mid < hi)) break;
    for (int r = 0; r < nc; ++r) W[r] = UL[r] + mid * (UT[r] - UL[r]);
    if (orc_pressure(c, W) >= eps)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

/* theta^p from UL (pressure pL) toward UT under the configured rule */
static double theta_p(const orc_cfg* c, const double* UL, double pL, const double* UT,
                      double eps) {
  if (c->limiter & ORC_LIM_PEXACT) return orc_theta_p_root(c, UL, UT, eps);
  return orc_Theta(pL, orc_pressure(c, UT), eps);
}

/* two-step Theta blend (density, then pressure through concavity), Sec. 3.3.
 * Returns theta^rho theta^p for moving from UL toward UH; *bad set if UL is not
 * admissible. */
static double theta_pair(const orc_cfg* c, const double* UL, const double* UH, int* bad) {
  int nc = ncomp(c);
  if (!(UL[0] > 0.0)) {
    *bad = 1;
    return 0.0;
  }
  double pL = orc_pressure(c, UL);
  if (!(pL > 0.0)) *bad = 1;
  double er = dmin(PP_EPS, UL[0]);
  double tr = orc_Theta(UL[0], UH[0], er);
  double Ut[4];
  for (int r = 0; r < nc; ++r) Ut[r] = UL[r] + tr * (UH[r] - UL[r]);
  double ep = dmin(PP_EPS, pL);
  double tp = theta_p(c, UL, pL, Ut, ep);
  return tr * tp;
}

/* ------------------------------------------------------------------------ */
/* lattice images (reading R-bc)                                             */
/* ------------------------------------------------------------------------ */

/* image of lattice coordinate X on an axis with 2n half cells; *kind receives
 * the wall kind crossed (or -1) */
static int axis_image(int X, int n, int lo, int hi, int* kind) {
  int M = 2 * n;
  *kind = -1;
  if (lo == ORC_PERIODIC) {
    X %= M;
    if (X < 0) X += M;
    return X;
  }
  if (X < 0) {
    if (lo == ORC_OUTFLOW) return (X % 2 == 0) ? 0 : 1;
    *kind = lo;
    return -X;
  }
  if (X > M) {
    if (hi == ORC_OUTFLOW) return ((X - M) % 2 == 0) ? M : M - 1;
    *kind = hi;
    return 2 * M - X;
  }
  return X;
}

/* sign changes of a mirror across a wall normal to axis `ax` */
static void wall_signs(const orc_cfg* c, int ax, int kind, double* sg) {
  if (kind == ORC_NOSLIP) {
    sg[1] = -sg[1];
    if (c->dim == 2) sg[2] = -sg[2];
  } else if (kind == ORC_SYMMETRY) {
    sg[1 + ax] = -sg[1 + ax];
  }
}

/* ======================================================================== */
/* 1D                                                                        */
/* ======================================================================== */

typedef struct {
  const orc_cfg* c;
  int n, np, LX;
  double dx;
  const double* avg;
  const double* pts;
  double* LU; /* [3][LX] conservative point values, X in [-GM, 2n+GM] */
  double* LW; /* [3][LX] primitives */
  double* LZ; /* [3][LX] Z */
  double* GZ; /* [3][LX] D_c Z, valid on [-2, 2n+2] */
  double* CA; /* [3][n+4] cell averages, cells -2..n+1 */
} lat1;

#define L1(a, k, X) ((a)[(k) * L->LX + (X) + GM])
#define C1(k, i) (L->CA[(k) * (L->n + 4) + (i) + 2])

static double dof1(const lat1* L, int X, int k) {
  if (X == 2 * L->n && L->np == L->n) X = 0;
  return L->pts[k * L->np + X / 2];
}

/* Simpson centre value (Sec. 2.1) */
static void centre1(const lat1* L, int X, double* Uc) {
  int i = (X - 1) / 2;
  for (int k = 0; k < 3; ++k)
    Uc[k] = (6.0 * L->avg[k * L->n + i] - (dof1(L, X - 1, k) + dof1(L, X + 1, k))) / 4.0;
}

/* scaling of a centre value toward its cell average (reading R-centre) */
static void limit_centre(const orc_cfg* c, const double* Ub, double* Uc) {
  int nc = ncomp(c);
  if (!(Ub[0] > 0.0)) {
    for (int r = 0; r < nc; ++r) Uc[r] = Ub[r];
    return;
  }
  int bad = 0;
  double th = theta_pair(c, Ub, Uc, &bad);
  if (th < 1.0)
    for (int r = 0; r < nc; ++r) Uc[r] = Ub[r] + th * (Uc[r] - Ub[r]);
}

static void build1(lat1* L) {
  const orc_cfg* c = L->c;
  int n = L->n;
  /* interior sites */
  for (int X = 0; X <= 2 * n; ++X) {
    double U[4];
    if (X % 2 == 1) {
      centre1(L, X, U);
      if (c->limiter & ORC_LIM_CENTRE) {
        double Ub[4];
        for (int k = 0; k < 3; ++k) Ub[k] = L->avg[k * n + (X - 1) / 2];
        limit_centre(c, Ub, U);
      }
    } else {
      for (int k = 0; k < 3; ++k) U[k] = dof1(L, X, k);
    }
    for (int k = 0; k < 3; ++k) L1(L->LU, k, X) = U[k];
  }
  /* ghost sites as images; beyond a Dirichlet side, its state (the paper
     prescribes boundary values there, Sec. 4) */
  for (int X = -GM; X <= 2 * n + GM; ++X) {
    if (X >= 0 && X <= 2 * n) continue;
    const int side = X < 0 ? 0 : 1;
    if (c->bc[side] == ORC_DIRICHLET) {
      for (int k = 0; k < 3; ++k) L1(L->LU, k, X) = c->bcstate[side][k];
      continue;
    }
    int kind;
    int Xi = axis_image(X, n, c->bc[0], c->bc[1], &kind);
    double sg[4] = {1.0, 1.0, 1.0};
    wall_signs(c, 0, kind, sg);
    for (int k = 0; k < 3; ++k) L1(L->LU, k, X) = sg[k] * L1(L->LU, k, Xi);
  }
  /* periodic: the site X=2n duplicates X=0 */
  for (int X = -GM; X <= 2 * n + GM; ++X) {
    double U[4], W[4], Z[4];
    for (int k = 0; k < 3; ++k) U[k] = L1(L->LU, k, X);
    prim(c, U, W);
    zvar(c, W, Z);
    for (int k = 0; k < 3; ++k) {
      L1(L->LW, k, X) = W[k];
      L1(L->LZ, k, X) = Z[k];
    }
  }
  for (int X = -2; X <= 2 * n + 2; ++X)
    for (int k = 0; k < 3; ++k) {
      double z[5];
      for (int o = 0; o < 5; ++o) z[o] = L1(L->LZ, k, X - 2 + o);
      L1(L->GZ, k, X) = orc_op_dc(z, L->dx);
    }
  /* cell averages with two ghost cells */
  for (int i = -2; i <= n + 1; ++i) {
    const int side = i < 0 ? 0 : 1;
    if ((i < 0 || i >= n) && c->bc[side] == ORC_DIRICHLET) {
      for (int k = 0; k < 3; ++k) C1(k, i) = c->bcstate[side][k];
      continue;
    }
    int kind;
    int Xi = axis_image(2 * i + 1, n, c->bc[0], c->bc[1], &kind);
    double sg[4] = {1.0, 1.0, 1.0};
    wall_signs(c, 0, kind, sg);
    int ii = (Xi - 1) / 2;
    for (int k = 0; k < 3; ++k) C1(k, i) = sg[k] * L->avg[k * n + ii];
  }
}

/* point residual R (eq. of the 1D point update): -D+ F^{c,+} - D- F^{c,-} + D^2(K,Z) */
static void resid1(const lat1* L, int X, double* R) {
  const orc_cfg* c = L->c;
  double dx = L->dx;
  double U[5][4], W[5][4], Z[5][4], F[5][4];
  double alpha = 0.0;
  for (int o = 0; o < 5; ++o) {
    for (int k = 0; k < 3; ++k) {
      U[o][k] = L1(L->LU, k, X - 2 + o);
      W[o][k] = L1(L->LW, k, X - 2 + o);
      Z[o][k] = L1(L->LZ, k, X - 2 + o);
    }
    orc_flux_c(c, 0, U[o], F[o]);
    alpha = dmax(alpha, rho_spec(c, 0, W[o]));
  }
  double B[5][5];
  build_B(B);
  double visc[4] = {0.0, 0.0, 0.0};
  for (int m = 0; m < 5; ++m) {
    double K[3][3];
    kmat1(c, W[m], K);
    for (int nn = 0; nn < 5; ++nn) {
      double y[4];
      matvec3(K, Z[nn], y);
      for (int k = 0; k < 3; ++k) visc[k] += B[m][nn] * y[k];
    }
  }
  for (int k = 0; k < 3; ++k) {
    double fp[5], fm[5];
    for (int o = 0; o < 5; ++o) {
      fp[o] = 0.5 * (F[o][k] + alpha * U[o][k]);
      fm[o] = 0.5 * (F[o][k] - alpha * U[o][k]);
    }
    double inv = orc_op_dplus(fp, dx) + orc_op_dminus(fm, dx);
    R[k] = -inv + 4.0 / (dx * dx) * visc[k];
  }
}

/* high-order face flux at face X (even): F^c - K(W) D_c Z */
static void fluxH1(const lat1* L, int X, double* F) {
  const orc_cfg* c = L->c;
  double U[4], S[4];
  for (int k = 0; k < 3; ++k) {
    U[k] = L1(L->LU, k, X);
    S[k] = L1(L->GZ, k, X);
  }
  flux_tot(c, 0, U, S, F);
}

/* state of a site of the low-order point lattice (reading R-point): a point
   site holds its point value, a centre site the cell average */
static void lo_site1(const lat1* L, int X, double* U) {
  for (int k = 0; k < 3; ++k) U[k] = (X & 1) ? C1(k, (X - 1) / 2) : L1(L->LU, k, X);
}

/* low-order gradient at a site of that lattice: central difference of Z
   over its two neighbours, dx/2 away on either side */
static void lo_grad1(const lat1* L, int X, double* S) {
  double Um[4], Up[4], Wm[4], Wp[4], Zm[4], Zp[4];
  lo_site1(L, X - 1, Um);
  lo_site1(L, X + 1, Up);
  prim(L->c, Um, Wm);
  prim(L->c, Up, Wp);
  zvar(L->c, Wm, Zm);
  zvar(L->c, Wp, Zp);
  for (int k = 0; k < 3; ++k) S[k] = (Zp[k] - Zm[k]) / L->dx;
}

/* low-order LLF flux between two neighbouring sites of the low-order point
   lattice (reading R-point) */
static void llf_sites1(const lat1* L, int Xa, int Xb, double* F) {
  const orc_cfg* c = L->c;
  double Ua[4], Ub[4], Sa[4], Sb[4], Wa[4], Wb[4], Fa[4], Fb[4];
  lo_site1(L, Xa, Ua);
  lo_site1(L, Xb, Ub);
  lo_grad1(L, Xa, Sa);
  lo_grad1(L, Xb, Sb);
  prim(c, Ua, Wa);
  prim(c, Ub, Wb);
  flux_tot(c, 0, Ua, Sa, Fa);
  flux_tot(c, 0, Ub, Sb, Fb);
  double lam = dmax(rho_spec(c, 0, Wa), rho_spec(c, 0, Wb)) +
               dmax(orc_bvisc(c, 0, Ua, Sa), orc_bvisc(c, 0, Ub, Sb));
  for (int k = 0; k < 3; ++k) F[k] = 0.5 * (Fa[k] + Fb[k]) - 0.5 * lam * (Ub[k] - Ua[k]);
}

static void project_wall(const orc_cfg* c, int ax, int kind, double* U) {
  if (kind == ORC_NOSLIP) {
    double m2 = U[1] * U[1] + (c->dim == 2 ? U[2] * U[2] : 0.0);
    int e = c->dim == 1 ? 2 : 3;
    U[e] -= m2 / (2.0 * U[0]);
    U[1] = 0.0;
    if (c->dim == 2) U[2] = 0.0;
  } else if (kind == ORC_SYMMETRY) {
    int e = c->dim == 1 ? 2 : 3;
    U[e] -= U[1 + ax] * U[1 + ax] / (2.0 * U[0]);
    U[1 + ax] = 0.0;
  }
}

static int wall_kind(int bc) { return (bc == ORC_NOSLIP || bc == ORC_SYMMETRY) ? bc : -1; }

static int fe1(const orc_cfg* c, const double* U, double dt, double* Ufe, double* ths,
               double* thpp) {
  lat1 Ls, *L = &Ls;
  int n = c->n1;
  L->c = c;
  L->n = n;
  L->np = (c->bc[0] == ORC_PERIODIC) ? n : n + 1;
  L->LX = 2 * n + 1 + 2 * GM;
  L->dx = (c->x1 - c->x0) / n;
  L->avg = U;
  L->pts = U + 3 * n;
  L->LU = calloc(3 * L->LX, sizeof(double));
  L->LW = calloc(3 * L->LX, sizeof(double));
  L->LZ = calloc(3 * L->LX, sizeof(double));
  L->GZ = calloc(3 * L->LX, sizeof(double));
  L->CA = calloc(3 * (n + 4), sizeof(double));
  build1(L);
  double dx = L->dx, mu_x = dt / dx;
  int flags = 0;
  int lim_cell = c->limiter & (ORC_LIM_SMOOTH | ORC_LIM_PP | ORC_LIM_LOWONLY);

  /* ---- point values ---- */
  double* Pfe = Ufe + 3 * n;
  for (int k = 0; k < L->np; ++k) {
    int X = 2 * k;
    double R[4], UH[4], U0[4], out[4];
    resid1(L, X, R);
    for (int r = 0; r < 3; ++r) {
      U0[r] = L1(L->LU, r, X);
      UH[r] = U0[r] + dt * R[r];
    }
    if (c->limiter & ORC_LIM_POINT) {
      double Fp[4], Fm[4], UL[4];
      llf_sites1(L, X, X + 1, Fp);
      llf_sites1(L, X - 1, X, Fm);
      for (int r = 0; r < 3; ++r) UL[r] = U0[r] - 2.0 * dt / dx * (Fp[r] - Fm[r]);
      int bad = 0;
      double th = theta_pair(c, UL, UH, &bad);
      if (c->limiter & ORC_LIM_LOWONLY) th = 0.0; /* low-order point values */
      if (bad) flags |= ORC_FLAG_POINT_LOW;
      for (int r = 0; r < 3; ++r) out[r] = (th == 1.0) ? UH[r] : UL[r] + th * (UH[r] - UL[r]);
    } else {
      for (int r = 0; r < 3; ++r) out[r] = UH[r];
    }
    if (k == 0) project_wall(c, 0, wall_kind(c->bc[0]), out);
    if (k == n) project_wall(c, 0, wall_kind(c->bc[1]), out);
    /* a point on a Dirichlet side keeps the prescribed state */
    if (k == 0 && c->bc[0] == ORC_DIRICHLET)
      for (int q = 0; q < 3; ++q) out[q] = c->bcstate[0][q];
    if (k == n && c->bc[1] == ORC_DIRICHLET)
      for (int q = 0; q < 3; ++q) out[q] = c->bcstate[1][q];
    for (int r = 0; r < 3; ++r) Pfe[r * L->np + k] = out[r];
  }

  /* ---- cell averages ---- */
  int nce = n + 2; /* cells -1..n */
  double* Wb = calloc(3 * (n + 4), sizeof(double));
  double* Zb = calloc(3 * (n + 4), sizeof(double));
  double* Fc_ = calloc(3 * nce, sizeof(double));
  double* rs = calloc(nce, sizeof(double));
  double* bv = calloc(nce, sizeof(double));
  double* ph1 = calloc(nce, sizeof(double));
  double* ph2 = calloc(nce, sizeof(double));
  for (int i = -2; i <= n + 1; ++i) {
    double Ub[4], W[4], Z[4];
    for (int k = 0; k < 3; ++k) Ub[k] = C1(k, i);
    prim(c, Ub, W);
    zvar(c, W, Z);
    for (int k = 0; k < 3; ++k) {
      Wb[k * (n + 4) + i + 2] = W[k];
      Zb[k * (n + 4) + i + 2] = Z[k];
    }
  }
#define WB(k, i) Wb[(k) * (n + 4) + (i) + 2]
#define ZB(k, i) Zb[(k) * (n + 4) + (i) + 2]
  for (int i = -1; i <= n; ++i) {
    int q = i + 1;
    double Ub[4], S[4], F[4], W[4];
    for (int k = 0; k < 3; ++k) {
      Ub[k] = C1(k, i);
      S[k] = (ZB(k, i + 1) - ZB(k, i - 1)) / (2.0 * dx);
      W[k] = WB(k, i);
    }
    flux_tot(c, 0, Ub, S, F);
    for (int k = 0; k < 3; ++k) Fc_[k * nce + q] = F[k];
    rs[q] = rho_spec(c, 0, W);
    bv[q] = orc_bvisc(c, 0, Ub, S);
    double pp = WB(2, i + 1), p0 = WB(2, i), pm = WB(2, i - 1);
    ph1[q] = fabs(pp - 2.0 * p0 + pm) / fabs(pp + 2.0 * p0 + pm);
    double div = (WB(1, i + 1) - WB(1, i - 1)) / (2.0 * dx);
    ph2[q] = dmax(-div / sqrt(div * div + DUCROS_EPS), 0.0);
  }
  double* Fh = calloc(3 * (n + 1), sizeof(double));
  for (int f = 0; f <= n; ++f) {
    int X = 2 * f;
    int a = f, b = f + 1; /* indices into pre arrays (cell i = f-1 -> a) */
    double FH[4], F[4];
    fluxH1(L, X, FH);
    double ts = 1.0, tpp = 1.0;
    if (!lim_cell) {
      for (int k = 0; k < 3; ++k) F[k] = FH[k];
    } else {
      double lam = dmax(rs[a], rs[b]) + dmax(bv[a], bv[b]);
      double FL[4];
      for (int k = 0; k < 3; ++k)
        FL[k] = 0.5 * (Fc_[k * nce + a] + Fc_[k * nce + b]) - 0.5 * lam * (C1(k, f) - C1(k, f - 1));
      if (c->limiter & ORC_LIM_LOWONLY) {
        ts = 0.0;
        tpp = 0.0;
      } else {
        if (c->limiter & ORC_LIM_SMOOTH)
          ts = exp(-c->Cs * dmax(ph1[a], ph1[b]) * dmax(ph2[a], ph2[b]));
        if (c->limiter & ORC_LIM_PP) {
          double Fs[4], ULp[4], UHp[4], ULm[4], UHm[4];
          for (int k = 0; k < 3; ++k) {
            Fs[k] = FL[k] + ts * (FH[k] - FL[k]);
            ULp[k] = C1(k, f - 1) - 2.0 * mu_x * (FL[k] - Fc_[k * nce + a]);
            UHp[k] = C1(k, f - 1) - 2.0 * mu_x * (Fs[k] - Fc_[k * nce + a]);
            ULm[k] = C1(k, f) - 2.0 * mu_x * (Fc_[k * nce + b] - FL[k]);
            UHm[k] = C1(k, f) - 2.0 * mu_x * (Fc_[k * nce + b] - Fs[k]);
          }
          tpp = 0.0;
          int bad = 0;
          if (!(ULp[0] > 0.0) || !(ULm[0] > 0.0)) {
            bad = 1;
          } else {
            double pLp = orc_pressure(c, ULp), pLm = orc_pressure(c, ULm);
            if (!(pLp > 0.0) || !(pLm > 0.0)) bad = 1;
            double tr = dmin(orc_Theta(ULp[0], UHp[0], dmin(PP_EPS, ULp[0])),
                             orc_Theta(ULm[0], UHm[0], dmin(PP_EPS, ULm[0])));
            double Tp[4], Tm[4];
            for (int k = 0; k < 3; ++k) {
              Tp[k] = ULp[k] + tr * (UHp[k] - ULp[k]);
              Tm[k] = ULm[k] + tr * (UHm[k] - ULm[k]);
            }
            double tp = dmin(theta_p(c, ULp, pLp, Tp, dmin(PP_EPS, pLp)),
                             theta_p(c, ULm, pLm, Tm, dmin(PP_EPS, pLm)));
            tpp = tr * tp;
          }
          if (bad) flags |= ORC_FLAG_CELL_LOW;
        }
      }
      double th = ts * tpp;
      for (int k = 0; k < 3; ++k) F[k] = FL[k] + th * (FH[k] - FL[k]);
    }
    if (ths) ths[f] = ts;
    if (thpp) thpp[f] = tpp;
    for (int k = 0; k < 3; ++k) Fh[k * (n + 1) + f] = F[k];
  }
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < 3; ++k)
      Ufe[k * n + i] = L->avg[k * n + i] - mu_x * (Fh[k * (n + 1) + i + 1] - Fh[k * (n + 1) + i]);
#undef WB
#undef ZB
  long len = orc_state_len(c);
  for (long q = 0; q < len; ++q)
    if (!isfinite(Ufe[q])) {
      flags |= ORC_FLAG_NONFINITE;
      break;
    }
  free(Wb);
  free(Zb);
  free(Fc_);
  free(rs);
  free(bv);
  free(ph1);
  free(ph2);
  free(Fh);
  free(L->LU);
  free(L->LW);
  free(L->LZ);
  free(L->GZ);
  free(L->CA);
  return flags;
}

/* unlimited semi-discrete right-hand side (1D) */
static void rhs1(const orc_cfg* c, const double* U, double* dU) {
  lat1 Ls, *L = &Ls;
  int n = c->n1;
  L->c = c;
  L->n = n;
  L->np = (c->bc[0] == ORC_PERIODIC) ? n : n + 1;
  L->LX = 2 * n + 1 + 2 * GM;
  L->dx = (c->x1 - c->x0) / n;
  L->avg = U;
  L->pts = U + 3 * n;
  L->LU = calloc(3 * L->LX, sizeof(double));
  L->LW = calloc(3 * L->LX, sizeof(double));
  L->LZ = calloc(3 * L->LX, sizeof(double));
  L->GZ = calloc(3 * L->LX, sizeof(double));
  L->CA = calloc(3 * (n + 4), sizeof(double));
  build1(L);
  for (int k = 0; k < L->np; ++k) {
    double R[4];
    resid1(L, 2 * k, R);
    for (int r = 0; r < 3; ++r) dU[3 * n + r * L->np + k] = R[r];
  }
  for (int i = 0; i < n; ++i) {
    double Fl[4], Fr[4];
    fluxH1(L, 2 * i, Fl);
    fluxH1(L, 2 * i + 2, Fr);
    for (int r = 0; r < 3; ++r) dU[r * n + i] = -(Fr[r] - Fl[r]) / L->dx;
  }
  free(L->LU);
  free(L->LW);
  free(L->LZ);
  free(L->GZ);
  free(L->CA);
}

/* ======================================================================== */
/* 2D                                                                        */
/* ======================================================================== */

typedef struct {
  const orc_cfg* c;
  int n1, n2, n1x, n2y, LX, LY;
  double dx, dy;
  const double *avg, *xe, *ye, *co;
  double* LU; /* [4][LY][LX] */
  double* LW;
  double* LZ;
  double* GZ; /* [2][4][LY][LX]: D_c^{(1)} Z, D_c^{(2)} Z */
  double* CA; /* [4][n2+4][n1+4] */
} lat2;

#define L2(a, k, X, Y) ((a)[((long)(k) * L->LY + (Y) + GM) * L->LX + (X) + GM])
#define G2(d, k, X, Y) (L->GZ[(((long)(d) * 4 + (k)) * L->LY + (Y) + GM) * L->LX + (X) + GM])
#define C2(k, i, j) (L->CA[((long)(k) * (L->n2 + 4) + (j) + 2) * (L->n1 + 4) + (i) + 2])
#define AVG(k, i, j) (L->avg[((long)(k) * L->n2 + (j)) * L->n1 + (i)])

static double dof2(const lat2* L, int X, int Y, int k) {
  if (X == 2 * L->n1 && L->n1x == L->n1) X = 0;
  if (Y == 2 * L->n2 && L->n2y == L->n2) Y = 0;
  if (X % 2 == 0 && Y % 2 == 1) return L->xe[((long)k * L->n2 + (Y - 1) / 2) * L->n1x + X / 2];
  if (X % 2 == 1 && Y % 2 == 0) return L->ye[((long)k * L->n2y + Y / 2) * L->n1 + (X - 1) / 2];
  return L->co[((long)k * L->n2y + Y / 2) * L->n1x + X / 2];
}

/* 2D centre value from the average, four edge and four corner points (Sec. 2.2) */
static void centre2(const lat2* L, int X, int Y, double* Uc) {
  int i = (X - 1) / 2, j = (Y - 1) / 2;
  for (int k = 0; k < 4; ++k) {
    double edges = dof2(L, X - 1, Y, k) + dof2(L, X + 1, Y, k) + dof2(L, X, Y - 1, k) +
                   dof2(L, X, Y + 1, k);
    double corners = dof2(L, X - 1, Y - 1, k) + dof2(L, X + 1, Y - 1, k) +
                     dof2(L, X - 1, Y + 1, k) + dof2(L, X + 1, Y + 1, k);
    Uc[k] = (36.0 * AVG(k, i, j) - 4.0 * edges - corners) / 16.0;
  }
}

static void image2(const lat2* L, int X, int Y, int* Xi, int* Yi, double* sg) {
  const orc_cfg* c = L->c;
  int kx, ky;
  *Xi = axis_image(X, L->n1, c->bc[0], c->bc[1], &kx);
  *Yi = axis_image(Y, L->n2, c->bc[2], c->bc[3], &ky);
  sg[0] = sg[1] = sg[2] = sg[3] = 1.0;
  wall_signs(c, 0, kx, sg);
  wall_signs(c, 1, ky, sg);
}

static void build2(lat2* L) {
  const orc_cfg* c = L->c;
  int n1 = L->n1, n2 = L->n2;
#pragma omp parallel for schedule(static)
  for (int Y = 0; Y <= 2 * n2; ++Y)
    for (int X = 0; X <= 2 * n1; ++X) {
      double U[4];
      if (X % 2 == 1 && Y % 2 == 1) {
        centre2(L, X, Y, U);
        if (c->limiter & ORC_LIM_CENTRE) {
          double Ub[4];
          for (int k = 0; k < 4; ++k) Ub[k] = AVG(k, (X - 1) / 2, (Y - 1) / 2);
          limit_centre(c, Ub, U);
        }
      } else {
        for (int k = 0; k < 4; ++k) U[k] = dof2(L, X, Y, k);
      }
      for (int k = 0; k < 4; ++k) L2(L->LU, k, X, Y) = U[k];
    }
#pragma omp parallel for schedule(static)
  for (int Y = -GM; Y <= 2 * n2 + GM; ++Y)
    for (int X = -GM; X <= 2 * n1 + GM; ++X) {
      if (X >= 0 && X <= 2 * n1 && Y >= 0 && Y <= 2 * n2) continue;
      int Xi, Yi;
      double sg[4];
      image2(L, X, Y, &Xi, &Yi, sg);
      for (int k = 0; k < 4; ++k) L2(L->LU, k, X, Y) = sg[k] * L2(L->LU, k, Xi, Yi);
    }
#pragma omp parallel for schedule(static)
  for (int Y = -GM; Y <= 2 * n2 + GM; ++Y)
    for (int X = -GM; X <= 2 * n1 + GM; ++X) {
      double U[4], W[4], Z[4];
      for (int k = 0; k < 4; ++k) U[k] = L2(L->LU, k, X, Y);
      prim(c, U, W);
      zvar(c, W, Z);
      for (int k = 0; k < 4; ++k) {
        L2(L->LW, k, X, Y) = W[k];
        L2(L->LZ, k, X, Y) = Z[k];
      }
    }
#pragma omp parallel for schedule(static)
  for (int Y = -2; Y <= 2 * n2 + 2; ++Y)
    for (int X = -2; X <= 2 * n1 + 2; ++X)
      for (int k = 0; k < 4; ++k) {
        double zx[5], zy[5];
        for (int o = 0; o < 5; ++o) {
          zx[o] = L2(L->LZ, k, X - 2 + o, Y);
          zy[o] = L2(L->LZ, k, X, Y - 2 + o);
        }
        G2(0, k, X, Y) = orc_op_dc(zx, L->dx);
        G2(1, k, X, Y) = orc_op_dc(zy, L->dy);
      }
  for (int j = -2; j <= n2 + 1; ++j)
    for (int i = -2; i <= n1 + 1; ++i) {
      int Xi, Yi;
      double sg[4];
      image2(L, 2 * i + 1, 2 * j + 1, &Xi, &Yi, sg);
      for (int k = 0; k < 4; ++k) C2(k, i, j) = sg[k] * AVG(k, (Xi - 1) / 2, (Yi - 1) / 2);
    }
}

static void site2(const lat2* L, int X, int Y, double* U, double* W, double* Z) {
  for (int k = 0; k < 4; ++k) {
    if (U) U[k] = L2(L->LU, k, X, Y);
    if (W) W[k] = L2(L->LW, k, X, Y);
    if (Z) Z[k] = L2(L->LZ, k, X, Y);
  }
}

/* point residual (eq. of the 2D semi-discrete AF point update) */
static void resid2(const lat2* L, int X, int Y, double* R) {
  const orc_cfg* c = L->c;
  double B[5][5];
  build_B(B);
  for (int k = 0; k < 4; ++k) R[k] = 0.0;
  for (int d = 0; d < 2; ++d) {
    int ex = (d == 0), ey = (d == 1);
    double h = d == 0 ? L->dx : L->dy;
    double U[5][4], W[5][4], Z[5][4], F[5][4];
    double alpha = 0.0;
    for (int o = 0; o < 5; ++o) {
      site2(L, X + (o - 2) * ex, Y + (o - 2) * ey, U[o], W[o], Z[o]);
      orc_flux_c(c, d, U[o], F[o]);
      alpha = dmax(alpha, rho_spec(c, d, W[o]));
    }
    /* inviscid: D+ F^{c,+} + D- F^{c,-} */
    for (int k = 0; k < 4; ++k) {
      double fp[5], fm[5];
      for (int o = 0; o < 5; ++o) {
        fp[o] = 0.5 * (F[o][k] + alpha * U[o][k]);
        fm[o] = 0.5 * (F[o][k] - alpha * U[o][k]);
      }
      R[k] -= orc_op_dplus(fp, h) + orc_op_dminus(fm, h);
    }
    /* compact D^{(d),2}(K_dd, Z) */
    double visc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int m = 0; m < 5; ++m) {
      double K[4][4];
      kmat2(c, d, d, W[m], K);
      for (int nn = 0; nn < 5; ++nn) {
        double y[4];
        matvec4(K, Z[nn], y);
        for (int k = 0; k < 4; ++k) visc[k] += B[m][nn] * y[k];
      }
    }
    for (int k = 0; k < 4; ++k) R[k] += 4.0 / (h * h) * visc[k];
    /* mixed: D_c^{(d)} (K_{d,o} D_c^{(o)} Z) */
    int od = 1 - d;
    double g[5][4];
    for (int o = 0; o < 5; ++o) {
      if (o == 2) {
        for (int k = 0; k < 4; ++k) g[o][k] = 0.0;
        continue;
      }
      int Xs = X + (o - 2) * ex, Ys = Y + (o - 2) * ey;
      double K[4][4], gz[4];
      kmat2(c, d, od, W[o], K);
      for (int k = 0; k < 4; ++k) gz[k] = G2(od, k, Xs, Ys);
      matvec4(K, gz, g[o]);
    }
    for (int k = 0; k < 4; ++k) {
      double z[5];
      for (int o = 0; o < 5; ++o) z[o] = g[o][k];
      R[k] += orc_op_dc(z, h);
    }
  }
}

/* total flux F_d at a lattice site using the D_c lattice gradients */
static void fluxsite2(const lat2* L, int d, int X, int Y, double* F) {
  double U[4], S[8];
  site2(L, X, Y, U, NULL, NULL);
  for (int k = 0; k < 4; ++k) {
    S[k] = G2(0, k, X, Y);
    S[4 + k] = G2(1, k, X, Y);
  }
  flux_tot(L->c, d, U, S, F);
}

/* state of a site of the low-order point lattice (reading R-point): point
   sites hold their point values, centre sites the cell averages */
static void lo_site2(const lat2* L, int X, int Y, double* U) {
  const int centre = (X & 1) && (Y & 1);
  for (int k = 0; k < 4; ++k)
    U[k] = centre ? C2(k, (X - 1) / 2, (Y - 1) / 2) : L2(L->LU, k, X, Y);
}

/* low-order gradient (x then y derivatives of Z) at a site of that lattice:
   central differences over the neighbouring sites, half a cell away */
static void lo_grad2(const lat2* L, int X, int Y, double* S) {
  const orc_cfg* c = L->c;
  double U[4][4], W[4], Z[4][4];
  lo_site2(L, X - 1, Y, U[0]);
  lo_site2(L, X + 1, Y, U[1]);
  lo_site2(L, X, Y - 1, U[2]);
  lo_site2(L, X, Y + 1, U[3]);
  for (int m = 0; m < 4; ++m) {
    prim(c, U[m], W);
    zvar(c, W, Z[m]);
  }
  for (int k = 0; k < 4; ++k) {
    S[k] = (Z[1][k] - Z[0][k]) / L->dx;
    S[4 + k] = (Z[3][k] - Z[2][k]) / L->dy;
  }
}

/* high-order face flux: Simpson average along the face (Sec. 2.2) */
static void fluxH2(const lat2* L, int d, int X, int Y, double* F) {
  double Fa[4], Fb[4], Fm[4];
  if (d == 0) {
    fluxsite2(L, 0, X, Y - 1, Fa);
    fluxsite2(L, 0, X, Y, Fm);
    fluxsite2(L, 0, X, Y + 1, Fb);
  } else {
    fluxsite2(L, 1, X - 1, Y, Fa);
    fluxsite2(L, 1, X, Y, Fm);
    fluxsite2(L, 1, X + 1, Y, Fb);
  }
  for (int k = 0; k < 4; ++k) F[k] = (Fa[k] + 4.0 * Fm[k] + Fb[k]) / 6.0;
}

static void llf_sites2(const lat2* L, int d, int Xa, int Ya, int Xb, int Yb, double* F) {
  const orc_cfg* c = L->c;
  double Ua[4], Ub[4], Wa[4], Wb[4], Sa[8], Sb[8], Fa[4], Fb[4];
  lo_site2(L, Xa, Ya, Ua);
  lo_site2(L, Xb, Yb, Ub);
  prim(c, Ua, Wa);
  prim(c, Ub, Wb);
  lo_grad2(L, Xa, Ya, Sa);
  lo_grad2(L, Xb, Yb, Sb);
  flux_tot(c, d, Ua, Sa, Fa);
  flux_tot(c, d, Ub, Sb, Fb);
  double lam = dmax(rho_spec(c, d, Wa), rho_spec(c, d, Wb)) +
               dmax(orc_bvisc(c, d, Ua, Sa), orc_bvisc(c, d, Ub, Sb));
  for (int k = 0; k < 4; ++k) F[k] = 0.5 * (Fa[k] + Fb[k]) - 0.5 * lam * (Ub[k] - Ua[k]);
}

static void setup2(lat2* L, const orc_cfg* c, const double* U) {
  L->c = c;
  L->n1 = c->n1;
  L->n2 = c->n2;
  L->n1x = (c->bc[0] == ORC_PERIODIC) ? c->n1 : c->n1 + 1;
  L->n2y = (c->bc[2] == ORC_PERIODIC) ? c->n2 : c->n2 + 1;
  L->LX = 2 * c->n1 + 1 + 2 * GM;
  L->LY = 2 * c->n2 + 1 + 2 * GM;
  L->dx = (c->x1 - c->x0) / c->n1;
  L->dy = (c->y1 - c->y0) / c->n2;
  L->avg = U;
  L->xe = L->avg + 4L * c->n1 * c->n2;
  L->ye = L->xe + 4L * L->n2 * L->n1x;
  L->co = L->ye + 4L * L->n2y * L->n1;
  long ns = (long)L->LX * L->LY;
  L->LU = calloc(4 * ns, sizeof(double));
  L->LW = calloc(4 * ns, sizeof(double));
  L->LZ = calloc(4 * ns, sizeof(double));
  L->GZ = calloc(8 * ns, sizeof(double));
  L->CA = calloc(4L * (c->n1 + 4) * (c->n2 + 4), sizeof(double));
  build2(L);
}

static void free2(lat2* L) {
  free(L->LU);
  free(L->LW);
  free(L->LZ);
  free(L->GZ);
  free(L->CA);
}

/* point DOF enumeration: type 0 xe, 1 ye, 2 co */
static void point_xy(int type, int i, int j, int* X, int* Y) {
  if (type == 0) {
    *X = 2 * i;
    *Y = 2 * j + 1;
  } else if (type == 1) {
    *X = 2 * i + 1;
    *Y = 2 * j;
  } else {
    *X = 2 * i;
    *Y = 2 * j;
  }
}

/* thnn: NULL, or a blend coefficient per face (x-faces, then y-faces) that
 * takes the place of theta^s: the density/pressure limiter of Sec. 3.3 then
 * acts on the candidate F^L + thnn (F^H - F^L), so the face flux is
 * F^L + thnn theta^rho theta^p (F^H - F^L) */
static int fe2(const orc_cfg* c, const double* U, double dt, double* Ufe, double* ths,
               double* thpp, const double* thnn) {
  lat2 Ls, *L = &Ls;
  setup2(L, c, U);
  int n1 = L->n1, n2 = L->n2;
  double dx = L->dx, dy = L->dy;
  int flags = 0;
  int lim_cell = (c->limiter & (ORC_LIM_SMOOTH | ORC_LIM_PP | ORC_LIM_LOWONLY)) || thnn;

  /* ---- point values ---- */
  double* outp[3];
  outp[0] = Ufe + 4L * n1 * n2;
  outp[1] = outp[0] + 4L * n2 * L->n1x;
  outp[2] = outp[1] + 4L * L->n2y * n1;
  int ext_i[3] = {L->n1x, n1, L->n1x};
  int ext_j[3] = {n2, L->n2y, L->n2y};
  for (int t = 0; t < 3; ++t) {
    int fl = 0;
#pragma omp parallel for schedule(static) reduction(| : fl)
    for (int j = 0; j < ext_j[t]; ++j)
      for (int i = 0; i < ext_i[t]; ++i) {
        int X, Y;
        point_xy(t, i, j, &X, &Y);
        double R[4], U0[4], UH[4], out[4];
        resid2(L, X, Y, R);
        site2(L, X, Y, U0, NULL, NULL);
        for (int k = 0; k < 4; ++k) UH[k] = U0[k] + dt * R[k];
        if (c->limiter & ORC_LIM_POINT) {
          double Fxp[4], Fxm[4], Fyp[4], Fym[4], UL[4];
          llf_sites2(L, 0, X, Y, X + 1, Y, Fxp);
          llf_sites2(L, 0, X - 1, Y, X, Y, Fxm);
          llf_sites2(L, 1, X, Y, X, Y + 1, Fyp);
          llf_sites2(L, 1, X, Y - 1, X, Y, Fym);
          for (int k = 0; k < 4; ++k)
            UL[k] = U0[k] - 2.0 * dt / dx * (Fxp[k] - Fxm[k]) - 2.0 * dt / dy * (Fyp[k] - Fym[k]);
          int bad = 0;
          double th = theta_pair(c, UL, UH, &bad);
          if (c->limiter & ORC_LIM_LOWONLY) th = 0.0; /* low-order point values */
          if (bad) fl |= ORC_FLAG_POINT_LOW;
          for (int k = 0; k < 4; ++k) out[k] = (th == 1.0) ? UH[k] : UL[k] + th * (UH[k] - UL[k]);
        } else {
          for (int k = 0; k < 4; ++k) out[k] = UH[k];
        }
        if (X == 0) project_wall(c, 0, wall_kind(c->bc[0]), out);
        if (X == 2 * n1) project_wall(c, 0, wall_kind(c->bc[1]), out);
        if (Y == 0) project_wall(c, 1, wall_kind(c->bc[2]), out);
        if (Y == 2 * n2) project_wall(c, 1, wall_kind(c->bc[3]), out);
        for (int k = 0; k < 4; ++k) outp[t][((long)k * ext_j[t] + j) * ext_i[t] + i] = out[k];
      }
    flags |= fl;
  }

  /* ---- cell averages ---- */
  int W1 = n1 + 4, W2 = n2 + 4;
  long nc4 = (long)W1 * W2;
  double* Wb = calloc(4 * nc4, sizeof(double));
  double* Zb = calloc(4 * nc4, sizeof(double));
  double* Fd = calloc(2 * 4 * nc4, sizeof(double)); /* total fluxes F_l,i */
  double* rs = calloc(2 * nc4, sizeof(double));
  double* bv = calloc(2 * nc4, sizeof(double));
  double* ph1 = calloc(nc4, sizeof(double));
  double* ph2 = calloc(nc4, sizeof(double));
#define CI(i, j) (((long)(j) + 2) * W1 + (i) + 2)
  for (int j = -2; j <= n2 + 1; ++j)
    for (int i = -2; i <= n1 + 1; ++i) {
      double Ub[4], W[4], Z[4];
      for (int k = 0; k < 4; ++k) Ub[k] = C2(k, i, j);
      prim(c, Ub, W);
      zvar(c, W, Z);
      for (int k = 0; k < 4; ++k) {
        Wb[k * nc4 + CI(i, j)] = W[k];
        Zb[k * nc4 + CI(i, j)] = Z[k];
      }
    }
#pragma omp parallel for schedule(static)
  for (int j = -1; j <= n2; ++j)
    for (int i = -1; i <= n1; ++i) {
      long q = CI(i, j);
      double Ub[4], S[8], W[4];
      for (int k = 0; k < 4; ++k) {
        Ub[k] = C2(k, i, j);
        W[k] = Wb[k * nc4 + q];
        S[k] = (Zb[k * nc4 + CI(i + 1, j)] - Zb[k * nc4 + CI(i - 1, j)]) / (2.0 * dx);
        S[4 + k] = (Zb[k * nc4 + CI(i, j + 1)] - Zb[k * nc4 + CI(i, j - 1)]) / (2.0 * dy);
      }
      for (int d = 0; d < 2; ++d) {
        double F[4];
        flux_tot(c, d, Ub, S, F);
        for (int k = 0; k < 4; ++k) Fd[(d * 4 + k) * nc4 + q] = F[k];
        rs[d * nc4 + q] = rho_spec(c, d, W);
        bv[d * nc4 + q] = orc_bvisc(c, d, Ub, S);
      }
      double p0 = Wb[3 * nc4 + q];
      double pxp = Wb[3 * nc4 + CI(i + 1, j)], pxm = Wb[3 * nc4 + CI(i - 1, j)];
      double pyp = Wb[3 * nc4 + CI(i, j + 1)], pym = Wb[3 * nc4 + CI(i, j - 1)];
      ph1[q] = dmax(fabs(pxp - 2.0 * p0 + pxm) / fabs(pxp + 2.0 * p0 + pxm),
                    fabs(pyp - 2.0 * p0 + pym) / fabs(pyp + 2.0 * p0 + pym));
      double ux = (Wb[1 * nc4 + CI(i + 1, j)] - Wb[1 * nc4 + CI(i - 1, j)]) / (2.0 * dx);
      double vy = (Wb[2 * nc4 + CI(i, j + 1)] - Wb[2 * nc4 + CI(i, j - 1)]) / (2.0 * dy);
      double vx = (Wb[2 * nc4 + CI(i + 1, j)] - Wb[2 * nc4 + CI(i - 1, j)]) / (2.0 * dx);
      double uy = (Wb[1 * nc4 + CI(i, j + 1)] - Wb[1 * nc4 + CI(i, j - 1)]) / (2.0 * dy);
      double div = ux + vy, curl = vx - uy;
      ph2[q] = dmax(-div / sqrt(div * div + curl * curl + DUCROS_EPS), 0.0);
    }
  /* faces: x-faces [n2][n1+1], then y-faces [n2+1][n1] */
  long nfx = (long)n2 * (n1 + 1), nfy = (long)(n2 + 1) * n1;
  double* Fx = calloc(4 * nfx, sizeof(double));
  double* Fy = calloc(4 * nfy, sizeof(double));
  for (int d = 0; d < 2; ++d) {
    int ni = d == 0 ? n1 + 1 : n1, nj = d == 0 ? n2 : n2 + 1;
    double mu_d = dt / (d == 0 ? dx : dy);
    double* Fo = d == 0 ? Fx : Fy;
    long nf = d == 0 ? nfx : nfy;
    int fl = 0;
#pragma omp parallel for schedule(static) reduction(| : fl)
    for (int j = 0; j < nj; ++j)
      for (int i = 0; i < ni; ++i) {
        /* cells a (minus side) and b (plus side) */
        int ia = d == 0 ? i - 1 : i, ja = d == 0 ? j : j - 1;
        long qa = CI(ia, ja), qb = CI(i, j);
        int X = d == 0 ? 2 * i : 2 * i + 1, Y = d == 0 ? 2 * j + 1 : 2 * j;
        double FH[4], F[4], ts = 1.0, tpp = 1.0;
        fluxH2(L, d, X, Y, FH);
        if (!lim_cell) {
          for (int k = 0; k < 4; ++k) F[k] = FH[k];
        } else {
          double lam = dmax(rs[d * nc4 + qa], rs[d * nc4 + qb]) + dmax(bv[d * nc4 + qa], bv[d * nc4 + qb]);
          double FL[4], Ua[4], Ub[4], Fa[4], Fb[4];
          for (int k = 0; k < 4; ++k) {
            Ua[k] = C2(k, ia, ja);
            Ub[k] = C2(k, i, j);
            Fa[k] = Fd[(d * 4 + k) * nc4 + qa];
            Fb[k] = Fd[(d * 4 + k) * nc4 + qb];
            FL[k] = 0.5 * (Fa[k] + Fb[k]) - 0.5 * lam * (Ub[k] - Ua[k]);
          }
          if (c->limiter & ORC_LIM_LOWONLY) {
            ts = 0.0;
            tpp = 0.0;
          } else {
            if (thnn) {
              /* on a periodic axis the last face is the first one again */
              int fi = (d == 0 && i == n1 && c->bc[0] == ORC_PERIODIC) ? 0 : i;
              int fj = (d == 1 && j == n2 && c->bc[2] == ORC_PERIODIC) ? 0 : j;
              ts = thnn[(d == 0 ? 0 : nfx) + (long)fj * ni + fi];
            } else if (c->limiter & ORC_LIM_SMOOTH) {
              ts = exp(-c->Cs * dmax(ph1[qa], ph1[qb]) * dmax(ph2[qa], ph2[qb]));
            }
            if (c->limiter & ORC_LIM_PP) {
              double Fs[4], ULp[4], UHp[4], ULm[4], UHm[4];
              for (int k = 0; k < 4; ++k) {
                Fs[k] = FL[k] + ts * (FH[k] - FL[k]);
                ULp[k] = Ua[k] - 4.0 * mu_d * (FL[k] - Fa[k]);
                UHp[k] = Ua[k] - 4.0 * mu_d * (Fs[k] - Fa[k]);
                ULm[k] = Ub[k] - 4.0 * mu_d * (Fb[k] - FL[k]);
                UHm[k] = Ub[k] - 4.0 * mu_d * (Fb[k] - Fs[k]);
              }
              tpp = 0.0;
              int bad = 0;
              if (!(ULp[0] > 0.0) || !(ULm[0] > 0.0)) {
                bad = 1;
              } else {
                double pLp = orc_pressure(c, ULp), pLm = orc_pressure(c, ULm);
                if (!(pLp > 0.0) || !(pLm > 0.0)) bad = 1;
                double tr = dmin(orc_Theta(ULp[0], UHp[0], dmin(PP_EPS, ULp[0])),
                                 orc_Theta(ULm[0], UHm[0], dmin(PP_EPS, ULm[0])));
                double Tp[4], Tm[4];
                for (int k = 0; k < 4; ++k) {
                  Tp[k] = ULp[k] + tr * (UHp[k] - ULp[k]);
                  Tm[k] = ULm[k] + tr * (UHm[k] - ULm[k]);
                }
                double tp = dmin(theta_p(c, ULp, pLp, Tp, dmin(PP_EPS, pLp)),
                                 theta_p(c, ULm, pLm, Tm, dmin(PP_EPS, pLm)));
                tpp = tr * tp;
              }
              if (bad) fl |= ORC_FLAG_CELL_LOW;
            }
          }
          double th = ts * tpp;
          for (int k = 0; k < 4; ++k) F[k] = FL[k] + th * (FH[k] - FL[k]);
        }
        long fidx = (long)j * ni + i;
        if (ths) ths[(d == 0 ? 0 : nfx) + fidx] = ts;
        if (thpp) thpp[(d == 0 ? 0 : nfx) + fidx] = tpp;
        for (int k = 0; k < 4; ++k) Fo[k * nf + fidx] = F[k];
      }
    flags |= fl;
  }
  double mx = dt / dx, my = dt / dy;
  for (int k = 0; k < 4; ++k)
    for (int j = 0; j < n2; ++j)
      for (int i = 0; i < n1; ++i) {
        double dfx = Fx[k * nfx + (long)j * (n1 + 1) + i + 1] - Fx[k * nfx + (long)j * (n1 + 1) + i];
        double dfy = Fy[k * nfy + (long)(j + 1) * n1 + i] - Fy[k * nfy + (long)j * n1 + i];
        Ufe[((long)k * n2 + j) * n1 + i] = AVG(k, i, j) - mx * dfx - my * dfy;
      }
#undef CI
  long len = orc_state_len(c);
  for (long q = 0; q < len; ++q)
    if (!isfinite(Ufe[q])) {
      flags |= ORC_FLAG_NONFINITE;
      break;
    }
  free(Wb);
  free(Zb);
  free(Fd);
  free(rs);
  free(bv);
  free(ph1);
  free(ph2);
  free(Fx);
  free(Fy);
  free2(L);
  return flags;
}

static void rhs2(const orc_cfg* c, const double* U, double* dU) {
  lat2 Ls, *L = &Ls;
  setup2(L, c, U);
  int n1 = L->n1, n2 = L->n2;
  double* outp[3];
  outp[0] = dU + 4L * n1 * n2;
  outp[1] = outp[0] + 4L * n2 * L->n1x;
  outp[2] = outp[1] + 4L * L->n2y * n1;
  int ext_i[3] = {L->n1x, n1, L->n1x};
  int ext_j[3] = {n2, L->n2y, L->n2y};
  for (int t = 0; t < 3; ++t)
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ext_j[t]; ++j)
      for (int i = 0; i < ext_i[t]; ++i) {
        int X, Y;
        point_xy(t, i, j, &X, &Y);
        double R[4];
        resid2(L, X, Y, R);
        for (int k = 0; k < 4; ++k) outp[t][((long)k * ext_j[t] + j) * ext_i[t] + i] = R[k];
      }
#pragma omp parallel for schedule(static)
  for (int j = 0; j < n2; ++j)
    for (int i = 0; i < n1; ++i) {
      double Fl[4], Fr[4], Fb[4], Ft[4];
      fluxH2(L, 0, 2 * i, 2 * j + 1, Fl);
      fluxH2(L, 0, 2 * i + 2, 2 * j + 1, Fr);
      fluxH2(L, 1, 2 * i + 1, 2 * j, Fb);
      fluxH2(L, 1, 2 * i + 1, 2 * j + 2, Ft);
      for (int k = 0; k < 4; ++k)
        dU[((long)k * n2 + j) * n1 + i] = -(Fr[k] - Fl[k]) / L->dx - (Ft[k] - Fb[k]) / L->dy;
    }
  free2(L);
}

/* ======================================================================== */
/* common driver: sizes, CFL dt, SSP-RK3 step with halving, run              */
/* ======================================================================== */

long orc_state_len(const orc_cfg* c) {
  if (c->dim == 1) {
    long np = (c->bc[0] == ORC_PERIODIC) ? c->n1 : c->n1 + 1;
    return 3L * (c->n1 + np);
  }
  long n1 = c->n1, n2 = c->n2;
  long n1x = (c->bc[0] == ORC_PERIODIC) ? n1 : n1 + 1;
  long n2y = (c->bc[2] == ORC_PERIODIC) ? n2 : n2 + 1;
  return 4L * (n1 * n2 + n2 * n1x + n2y * n1 + n2y * n1x);
}

int orc_fe(const orc_cfg* c, const double* U, double dt, double* Ufe, double* ths,
           double* thpp) {
  return c->dim == 1 ? fe1(c, U, dt, Ufe, ths, thpp) : fe2(c, U, dt, Ufe, ths, thpp, NULL);
}

int orc_fe_blend(const orc_cfg* c, const double* U, double dt, const double* theta_nn,
                 double* Ufe, double* ths, double* thpp) {
  if (c->dim != 2 || !theta_nn) return -1;
  return fe2(c, U, dt, Ufe, ths, thpp, theta_nn);
}

long orc_nfaces(const orc_cfg* c) {
  return c->dim == 1 ? c->n1 + 1 : (long)c->n2 * (c->n1 + 1) + (long)(c->n2 + 1) * c->n1;
}

/* Features of the learned blend coefficient of one face (a reading of the
 * paper's limiter as a function of local data; the paper has no learned
 * part).  The face lies between cells a and b; in its frame (normal n along
 * the face's axis, tangent t along the other axis) the stencil is the 4 x 3
 * block of cell averages at normal offsets -2, -1 (a), +1 (b), +2 and
 * tangential offsets -1, 0, +1, ghost cells being the boundary images used by
 * the stage.  With face values rho_f = (rho_a + rho_b)/2, p_f likewise,
 * u_nf, u_tf likewise and c_f = sqrt(gamma p_f / rho_f), the 40 features are:
 * for tangential offset s = -1, 0, +1 and normal offset m = -2, -1, +1, +2,
 * [ln(p / p_f), (u_n - u_nf) / c_f, (u_t - u_tf) / c_f] (36 values), then
 * ln(rho / rho_f) for m = -2, -1, +1, +2 at s = 0.  The smoothness blend of
 * Sec. 3.2 is a function of the same block, through pressure ratios and
 * velocity gradients relative to a velocity scale. */
static double pos_or_tiny(double v) { return v > 1e-300 ? v : 1e-300; }

int orc_blend_features(const orc_cfg* c, const double* U, double* feat) {
  if (c->dim != 2) return -1;
  lat2 Ls, *L = &Ls;
  setup2(L, c, U);
  int n1 = c->n1, n2 = c->n2;
  long nfx = (long)n2 * (n1 + 1);
  for (int d = 0; d < 2; ++d) {
    int ni = d == 0 ? n1 + 1 : n1, nj = d == 0 ? n2 : n2 + 1;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < nj; ++j)
      for (int i = 0; i < ni; ++i) {
        /* primitives (rho, u_n, u_t, p) of the cell at normal offset m and
           tangential offset s; cell a is m = -1, cell b is m = +1 */
        double P[3][4][4];
        const int moff[4] = {-2, -1, 1, 2};
        for (int s = 0; s < 3; ++s)
          for (int q = 0; q < 4; ++q) {
            int m = moff[q];
            int nidx = (d == 0 ? i : j) + (m < 0 ? m : m - 1);
            int ci = d == 0 ? nidx : i + (s - 1);
            int cj = d == 0 ? j + (s - 1) : nidx;
            double Uc[4], W[4];
            for (int k = 0; k < 4; ++k) Uc[k] = C2(k, ci, cj);
            prim(c, Uc, W);
            P[s][q][0] = Uc[0];
            P[s][q][1] = d == 0 ? W[1] : W[2];
            P[s][q][2] = d == 0 ? W[2] : W[1];
            P[s][q][3] = W[3];
          }
        double rf = 0.5 * (P[1][1][0] + P[1][2][0]);
        double pf = 0.5 * (P[1][1][3] + P[1][2][3]);
        double unf = 0.5 * (P[1][1][1] + P[1][2][1]);
        double utf = 0.5 * (P[1][1][2] + P[1][2][2]);
        double cf = sqrt(c->gamma * pos_or_tiny(pf) / pos_or_tiny(rf));
        long f = (d == 0 ? 0 : nfx) + (long)j * ni + i;
        double* o = feat + 40 * f;
        int n = 0;
        for (int s = 0; s < 3; ++s)
          for (int q = 0; q < 4; ++q) {
            o[n++] = log(pos_or_tiny(P[s][q][3]) / pos_or_tiny(pf));
            o[n++] = (P[s][q][1] - unf) / cf;
            o[n++] = (P[s][q][2] - utf) / cf;
          }
        for (int q = 0; q < 4; ++q) o[n++] = log(pos_or_tiny(P[1][q][0]) / pos_or_tiny(rf));
      }
  }
  free2(L);
  return 0;
}

void orc_rhs(const orc_cfg* c, const double* U, double* dUdt) {
  if (c->dim == 1)
    rhs1(c, U, dUdt);
  else
    rhs2(c, U, dUdt);
}

/* CFL condition (eq. cfl) over the cell averages */
double orc_dt(const orc_cfg* c, const double* U) {
  int nc = ncomp(c);
  long ncell = c->dim == 1 ? c->n1 : (long)c->n1 * c->n2;
  double h[2];
  h[0] = (c->x1 - c->x0) / c->n1;
  h[1] = c->dim == 2 ? (c->y1 - c->y0) / c->n2 : 1.0;
  double a = 0.0, v = 0.0;
  for (long q = 0; q < ncell; ++q) {
    double Ub[4], W[4];
    for (int k = 0; k < nc; ++k) Ub[k] = U[k * ncell + q];
    prim(c, Ub, W);
    double rt = dmax(4.0 * c->mu / (3.0 * W[0]), c->gamma * c->mu / (c->Pr * W[0]));
    for (int d = 0; d < c->dim; ++d) {
      a = dmax(a, rho_spec(c, d, W) / (c->cfl_c * h[d]));
      v = dmax(v, rt / (c->cfl_v * h[d] * h[d]));
    }
  }
  return 1.0 / (a + v);
}

/* Time-step bound of the positivity theorem at the end of Sec. 3.4.  The
 * theorem asks dt to satisfy the sufficient condition of the
 * proposition on the intermediate states of the LLF scheme (Sec. 3.1),
 * dt <= dx_l / (2 d max lambda_l), both for the cell averages and for the
 * low-order point scheme, whose lattice has spacing dx_l / 2.  lambda of a
 * face or lattice link is max varrho_l + max b_l over its two ends (eq. of
 * the low face fluxes); here it is bounded above by the largest varrho_l
 * plus the largest b_l over all ends in direction l, so the bound returned
 * is sufficient for every face and link.  Only the low-order schemes that a
 * limiter switch uses count: the cell one under ORC_LIM_PP, the point one
 * under ORC_LIM_POINT (neither: +infinity).
 *   cell ends: the cells on either side of every face, ghost cells being
 *     boundary images; S by central differences of Z(average) (R-S);
 *   point ends: every site a point DOF links to in direction l (points,
 *     cell averages at centres, ghost images), with the gradients of R-point.
 */
static double dt_bound(double h, int dim, double a, double b) {
  double lam = a + b;
  return lam > 0.0 ? h / (2.0 * dim * lam) : HUGE_VAL;
}

static double dt_pp1(const orc_cfg* c, const double* U) {
  lat1 Ls, *L = &Ls;
  int n = c->n1;
  L->c = c;
  L->n = n;
  L->np = (c->bc[0] == ORC_PERIODIC) ? n : n + 1;
  L->LX = 2 * n + 1 + 2 * GM;
  L->dx = (c->x1 - c->x0) / n;
  L->avg = U;
  L->pts = U + 3 * n;
  L->LU = calloc(3 * L->LX, sizeof(double));
  L->LW = calloc(3 * L->LX, sizeof(double));
  L->LZ = calloc(3 * L->LX, sizeof(double));
  L->GZ = calloc(3 * L->LX, sizeof(double));
  L->CA = calloc(3 * (n + 4), sizeof(double));
  build1(L);
  double dt = HUGE_VAL;
  if (c->limiter & ORC_LIM_PP) {
    double a = 0.0, b = 0.0;
    for (int i = -1; i <= n; ++i) {
      double Ub[4], W[4], Wm[4], Wp[4], Z[4], Zm[4], Zp[4], Um[4], Up[4], S[4];
      for (int k = 0; k < 3; ++k) {
        Ub[k] = C1(k, i);
        Um[k] = C1(k, i - 1);
        Up[k] = C1(k, i + 1);
      }
      prim(c, Ub, W);
      prim(c, Um, Wm);
      prim(c, Up, Wp);
      zvar(c, W, Z);
      zvar(c, Wm, Zm);
      zvar(c, Wp, Zp);
      for (int k = 0; k < 3; ++k) S[k] = (Zp[k] - Zm[k]) / (2.0 * L->dx);
      a = dmax(a, rho_spec(c, 0, W));
      b = dmax(b, orc_bvisc(c, 0, Ub, S));
    }
    dt = dmin(dt, dt_bound(L->dx, 1, a, b));
  }
  if (c->limiter & ORC_LIM_POINT) {
    double a = 0.0, b = 0.0;
    for (int X = -1; X <= 2 * n + 1; ++X) {
      double Us[4], W[4], S[4];
      lo_site1(L, X, Us);
      prim(c, Us, W);
      lo_grad1(L, X, S);
      a = dmax(a, rho_spec(c, 0, W));
      b = dmax(b, orc_bvisc(c, 0, Us, S));
    }
    dt = dmin(dt, dt_bound(0.5 * L->dx, 1, a, b));
  }
  free(L->LU);
  free(L->LW);
  free(L->LZ);
  free(L->GZ);
  free(L->CA);
  return dt;
}

static double dt_pp2(const orc_cfg* c, const double* U) {
  lat2 Ls, *L = &Ls;
  setup2(L, c, U);
  int n1 = L->n1, n2 = L->n2;
  double h[2] = {L->dx, L->dy};
  double dt = HUGE_VAL;
  if (c->limiter & ORC_LIM_PP) {
    for (int d = 0; d < 2; ++d) {
      /* cells beside the faces normal to d: one ghost layer along d */
      int ilo = d == 0 ? -1 : 0, ihi = d == 0 ? n1 : n1 - 1;
      int jlo = d == 1 ? -1 : 0, jhi = d == 1 ? n2 : n2 - 1;
      double a = 0.0, b = 0.0;
      for (int j = jlo; j <= jhi; ++j)
        for (int i = ilo; i <= ihi; ++i) {
          double Ub[4], W[4], S[8], Zn[4][4];
          const int ni[4] = {i - 1, i + 1, i, i}, nj[4] = {j, j, j - 1, j + 1};
          for (int m = 0; m < 4; ++m) {
            double Un[4], Wn[4];
            for (int k = 0; k < 4; ++k) Un[k] = C2(k, ni[m], nj[m]);
            prim(c, Un, Wn);
            zvar(c, Wn, Zn[m]);
          }
          for (int k = 0; k < 4; ++k) {
            Ub[k] = C2(k, i, j);
            S[k] = (Zn[1][k] - Zn[0][k]) / (2.0 * L->dx);
            S[4 + k] = (Zn[3][k] - Zn[2][k]) / (2.0 * L->dy);
          }
          prim(c, Ub, W);
          a = dmax(a, rho_spec(c, d, W));
          b = dmax(b, orc_bvisc(c, d, Ub, S));
        }
      dt = dmin(dt, dt_bound(h[d], 2, a, b));
    }
  }
  if (c->limiter & ORC_LIM_POINT) {
    for (int d = 0; d < 2; ++d) {
      /* ends of the links along d of every point: one ghost line along d */
      int Xlo = d == 0 ? -1 : 0, Xhi = d == 0 ? 2 * n1 + 1 : 2 * n1;
      int Ylo = d == 1 ? -1 : 0, Yhi = d == 1 ? 2 * n2 + 1 : 2 * n2;
      double a = 0.0, b = 0.0;
      for (int Y = Ylo; Y <= Yhi; ++Y)
        for (int X = Xlo; X <= Xhi; ++X) {
          double Us[4], W[4], S[8];
          lo_site2(L, X, Y, Us);
          prim(c, Us, W);
          lo_grad2(L, X, Y, S);
          a = dmax(a, rho_spec(c, d, W));
          b = dmax(b, orc_bvisc(c, d, Us, S));
        }
      dt = dmin(dt, dt_bound(0.5 * h[d], 2, a, b));
    }
  }
  free2(L);
  return dt;
}

double orc_dt_pp(const orc_cfg* c, const double* U) {
  return c->dim == 1 ? dt_pp1(c, U) : dt_pp2(c, U);
}

/* SSP-RK54 (Sec. 2.3 names the five-stage, fourth-order SSP Runge-Kutta
 * method; coefficients of Spiteri and Ruuth's SSPRK(5,4) in Shu-Osher form).
 * In forward-Euler steps E_k = FE(u_k, c_k dt):
 *   u1 = E0
 *   u2 = a20 u0 + a21 E1,   u3 = a30 u0 + a32 E2,   u4 = a40 u0 + a43 E3
 *   u5 = a52 u2 + a53 E3 + a54 E4
 * with c_0 = b10, c_1 = b21/a21, c_2 = b32/a32, c_3 = b43/a43 = b53/a53
 * (the two agree to the 15 digits of the coefficients: E3 is one
 * evaluation) and c_4 = b54/a54. */
static const double RK54_A20 = 0.444370493651235, RK54_A21 = 0.555629506348765;
static const double RK54_A30 = 0.620101851488403, RK54_A32 = 0.379898148511597;
static const double RK54_A40 = 0.178079954393132, RK54_A43 = 0.821920045606868;
static const double RK54_A52 = 0.517231671970585, RK54_A53 = 0.096059710526147;
static const double RK54_A54 = 0.386708617503269;
static const double RK54_B10 = 0.391752226571890, RK54_B21 = 0.368410593050371;
static const double RK54_B32 = 0.251891774271694, RK54_B43 = 0.544974750228521;
static const double RK54_B54 = 0.226007483236906;

/* one attempt of SSP-RK54 from U (untouched) into out; returns the flags */
static int rk54_attempt(const orc_cfg* c, const double* U, double dt, double* out) {
  long len = orc_state_len(c);
  double* u1 = malloc(len * sizeof(double));
  double* u2 = malloc(len * sizeof(double));
  double* u3 = malloc(len * sizeof(double));
  double* e = malloc(len * sizeof(double));
  double* e3 = malloc(len * sizeof(double));
  int fl = 0;
  fl |= orc_fe(c, U, RK54_B10 * dt, u1, NULL, NULL);
  fl |= orc_fe(c, u1, RK54_B21 / RK54_A21 * dt, e, NULL, NULL);
  for (long q = 0; q < len; ++q) u2[q] = RK54_A20 * U[q] + RK54_A21 * e[q];
  fl |= orc_fe(c, u2, RK54_B32 / RK54_A32 * dt, e, NULL, NULL);
  for (long q = 0; q < len; ++q) u3[q] = RK54_A30 * U[q] + RK54_A32 * e[q];
  fl |= orc_fe(c, u3, RK54_B43 / RK54_A43 * dt, e3, NULL, NULL);
  double* u4 = u1; /* u1 is no longer needed */
  for (long q = 0; q < len; ++q) u4[q] = RK54_A40 * U[q] + RK54_A43 * e3[q];
  fl |= orc_fe(c, u4, RK54_B54 / RK54_A54 * dt, e, NULL, NULL);
  for (long q = 0; q < len; ++q)
    out[q] = RK54_A52 * u2[q] + RK54_A53 * e3[q] + RK54_A54 * e[q];
  free(u1);
  free(u2);
  free(u3);
  free(e);
  free(e3);
  return fl;
}

int orc_step(const orc_cfg* c, double* U, double dt, double t, double t_final, double* dt_used,
             int* halvings, int* flags_out) {
  long len = orc_state_len(c);
  if (dt <= 0.0) dt = orc_dt(c, U);
  if (t + dt > t_final) dt = t_final - t;
  double* U1 = malloc(len * sizeof(double));
  double* U2 = malloc(len * sizeof(double));
  double* Fe = malloc(len * sizeof(double));
  int status = 1, h;
  int fl_all = 0;
  for (h = 0; h <= c->max_halvings; ++h) {
    int fl = 0;
    if (c->rk == 54) {
      fl = rk54_attempt(c, U, dt, Fe);
      fl_all = fl;
      if (fl == 0) {
        for (long q = 0; q < len; ++q) U[q] = Fe[q];
        status = 0;
        break;
      }
      dt *= 0.5;
      continue;
    }
    fl |= orc_fe(c, U, dt, U1, NULL, NULL);
    fl |= orc_fe(c, U1, dt, Fe, NULL, NULL);
    for (long q = 0; q < len; ++q) U2[q] = 0.75 * U[q] + 0.25 * Fe[q];
    fl |= orc_fe(c, U2, dt, Fe, NULL, NULL);
    fl_all = fl;
    if (fl == 0) {
      for (long q = 0; q < len; ++q) U[q] = (1.0 / 3.0) * U[q] + (2.0 / 3.0) * Fe[q];
      status = 0;
      break;
    }
    dt *= 0.5;
  }
  if (dt_used) *dt_used = dt;
  if (halvings) *halvings = h;
  if (flags_out) *flags_out = fl_all;
  free(U1);
  free(U2);
  free(Fe);
  return status;
}

int orc_run(const orc_cfg* c, double* U, double t0, double t_final, long max_steps, long* nsteps,
            double* t_out) {
  double t = t0;
  long s = 0;
  int st = 0;
  while (t < t_final && s < max_steps) {
    double dtu;
    int h, fl;
    st = orc_step(c, U, 0.0, t, t_final, &dtu, &h, &fl);
    if (st) break;
    t += dtu;
    ++s;
  }
  if (nsteps) *nsteps = s;
  if (t_out) *t_out = t;
  return st;
}
