// af_stage2d.hip -- one SSP-RK3 stage of the 2D compact AF method on gfx950
// as a single fused, LDS-tiled kernel.
//
// A workgroup owns a tile of TX x TY cells, i.e. the half-lattice block
// [X0, X0+2TX) x [Y0, Y0+2TY): the cell averages, x-edge, y-edge and corner
// point values inside it.  It stages everything the stage needs for that
// block in LDS and writes only the stage output:
//   phase 0  lattice values on the block +- 4 half cells: ghosts as boundary
//            images, Simpson centres scaled toward the cell average (Sec. 2.2;
//            Remark after the pressure blend, Sec. 3.3), and (u, v, p, T, c)
//   phase 1  D_c gradients of (u, v, T) on the block +- 2 (Sec. 2.2 central
//            operator)
//   phase 2  low-order data of the cells of the tile +- 1: S, F_l, |u_l|+c,
//            b_l, the two smoothness sensors, (u, v, p, T, c) of the average
//            (Sec. 3.1, Sec. 3.2)
//   phase 3  limited face fluxes of the tile's cells: Simpson high-order
//            flux, LLF low-order flux, theta^s, theta^rho theta^p (Sec. 3.3)
//   phase 4  cell-average update and RK combination
//   phase 5a total flux and b of every lattice site the point LLF of Sec.
//            3.4 reads, once per site and direction (beside phase 4)
//   phase 5  point residual (biased inviscid operators with the downwind
//            point, compact D^2, mixed terms; Sec. 2.2), point LLF on the
//            lattice of point values and cell averages and the scaling limiter
//            (Sec. 3.4), wall projection, RK combination; two lanes per
//            point, one per direction
//
// The kernel is a template over the arithmetic type R of the stencils, fluxes
// and residuals (LDS included).  R = double is the FP64 stage.  R = float is
// the mixed-precision stage: stencils and fluxes in FP32, while the density
// and pressure blends (the Theta rule of Sec. 3.3 and 3.4), the cell-average
// update, the point-value update and the low-order point value stay FP64 on
// FP64 data read from the state, and the point sites' (u, v, p, T, c) are
// taken from their FP64 values; the state itself is FP64 in both.
#include <type_traits>

#include "af_device.hpp"
#include "af_internal.hpp"
#include "af_lattice.hpp"

using namespace afd;

namespace {

// One object file holds one instance: its arithmetic type and tile height
// are set when it is compiled (the FP64 stage with 16 x 7 tiles, the mixed
// stage with 16 x 14 tiles, which its FP32 LDS arrays leave room for), and
// its entry point is afi::AF_STAGE_ENTRY.
#ifndef AF_STAGE_REAL
#define AF_STAGE_REAL double
#endif
#ifndef AF_STAGE_TY
#define AF_STAGE_TY 7
#endif
#ifndef AF_STAGE_ENTRY
#define AF_STAGE_ENTRY stage2d_fp64
#endif
#define AF_CAT2(a, b) a##b
#define AF_CAT(a, b) AF_CAT2(a, b)
#define AF_STAGE_TILES AF_CAT(AF_STAGE_ENTRY, _tiles)
#define AF_STAGE_BATCH AF_CAT(AF_STAGE_ENTRY, _batch)

// tile shape: 16 x TY cells, 512 threads (eight wave64s, two per SIMD)
constexpr int TX = 16, TY = AF_STAGE_TY, NT = 512;
// lattice region [X0-4, X0+2TX+4] x [Y0-4, Y0+2TY+4]: both edges are face
// lines, so every centre inside has its eight neighbours inside
constexpr int WA = 2 * TX + 9, HA = 2 * TY + 9, NA = WA * HA;
constexpr int WG = 2 * TX + 4, HG = 2 * TY + 4, NG = WG * HG;  // block +- 2
constexpr int WC = TX + 2, HC = TY + 2, NC = WC * HC;          // tile cells +- 1
constexpr int NFX = TY * (TX + 1), NFY = (TY + 1) * TX;
constexpr int NCEN = (TX + 4) * (TY + 4);  // centre sites of the lattice region
constexpr int NPT = 3 * TX * TY;           // point DOF sites of a tile
// sites of the low-order point scheme: [X0-1, X0+2TX] x [Y0-1, Y0+2TY], the
// tile's point sites and their lattice neighbours; x-direction data on its
// rows Y0..Y0+2TY-1, y-direction data on its columns X0..X0+2TX-1
constexpr int SW = 2 * TX + 2, SH = 2 * TY + 2, NSR = SW * SH;
constexpr int NSX = SW * 2 * TY, NSY = 2 * TX * SH;

template <typename R>
constexpr bool kFP64 = std::is_same<R, double>::value;

// (u, v, p, T, c) of state V, given 1/rho
template <typename R>
__device__ __forceinline__ void aux_of(const PhysT<R>& ph, const R* V, R ir, R* w) {
  const R p = ph.gm1 * (V[3] - R(0.5) * (V[1] * V[1] + V[2] * V[2]) * ir);
  w[0] = V[1] * ir;
  w[1] = V[2] * ir;
  w[2] = p;
  w[3] = p * ir;
  w[4] = sqrt(ph.gam * w[3]);
}

// Simpson centre value from the cell average, the sum of the four edge
// points and the sum of the four corners (Sec. 2.2), scaled toward the
// average with the density-then-pressure rule when the centre limiter is on,
// and its (u, v, p, T, c).  A centre whose density and pressure are already
// at least eps keeps its value: the rule's parameter is 1 there (the rule is
// continuous at that threshold, so only round-off separates the two
// evaluations of the test).  The rule itself runs in FP64.
template <typename R>
__device__ __forceinline__ void centre_value(const PhysT<R>& ph, const Phys& phd, const R* Ub,
                                             const R* e, const R* c, R* V, R* w) {
#pragma unroll
  for (int k = 0; k < 4; ++k) V[k] = (R(36.0) * Ub[k] - R(4.0) * e[k] - c[k]) / R(16.0);
  R ir = rcp(V[0]);
  const R p = ph.gm1 * (V[3] - R(0.5) * (V[1] * V[1] + V[2] * V[2]) * ir);
  if ((ph.lim & LIM_CENTRE) && !(Ub[0] > R(0.0) && V[0] >= R(kPPEps) && p >= R(kPPEps))) {
    if (!(Ub[0] > R(0.0))) {
#pragma unroll
      for (int k = 0; k < 4; ++k) V[k] = Ub[k];
    } else {
      double Ud[4], Vd[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        Ud[k] = Ub[k];
        Vd[k] = V[k];
      }
      bool bad = false;
      const double th = theta_pair2(Ud, Vd, phd.gm1, bad, ph.lim & LIM_PEXACT);
      if (th < 1.0) {
        double Wd[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          Wd[k] = Ud[k] + th * (Vd[k] - Ud[k]);
          V[k] = R(Wd[k]);
        }
        if constexpr (!std::is_same<R, double>::value) {
          // FP32 stencils: the scaled centre's pressure may sit at eps, far
          // below the rounding of E - |m|^2 / (2 rho) in FP32, so its
          // (u, v, p, T, c) are taken from the FP64 value
          const double ird = rcp(Wd[0]);
          const double pd = phd.gm1 * (Wd[3] - 0.5 * (Wd[1] * Wd[1] + Wd[2] * Wd[2]) * ird);
          w[0] = R(Wd[1] * ird);
          w[1] = R(Wd[2] * ird);
          w[2] = R(pd);
          w[3] = R(pd * ird);
          w[4] = R(sqrt(phd.gam * (pd * ird)));
          return;
        }
      }
    }
    ir = rcp(V[0]);
  }
  aux_of(ph, V, ir, w);
}

// whether the centre site (X, Y) of the lattice is a ghost beyond a wall or
// outflow side (not a periodic one)
__device__ __forceinline__ bool ghost_centre(const G2& g, int X, int Y) {
  return ((X < 0 || X > 2 * g.n1) && g.bc0 != BC_PERIODIC) ||
         ((Y < 0 || Y > 2 * g.n2) && g.bc2 != BC_PERIODIC);
}

// per-cell low-order data (Sec. 3.1-3.2):
//   o[0..3] F_x, o[4..7] F_y (total fluxes with S = central differences of
//   Z(average)), o[8] |u|+c, o[9] |v|+c, o[10] b_x, o[11] b_y, o[12] phi1,
//   o[13] phi2, o[14..17] the cell average, o[18..22] its (u, v, p, T, c);
//   from the averages of the cell and of its four neighbours (ghost cells as
//   boundary images)
template <typename R>
__device__ __forceinline__ void cell_low(const G2& g, const PhysT<R>& ph, const R* C0,
                                         const R* Cxm, const R* Cxp, const R* Cym, const R* Cyp,
                                         R* o) {
  // one reciprocal density per cell
  const R r0 = rcp(C0[0]), rxm = rcp(Cxm[0]), rxp = rcp(Cxp[0]),
          rym = rcp(Cym[0]), ryp = rcp(Cyp[0]);
  auto pr = [&](const R* V, R ir) {
    return ph.gm1 * (V[3] - R(0.5) * (V[1] * V[1] + V[2] * V[2]) * ir);
  };
  const R p0 = pr(C0, r0), pxm = pr(Cxm, rxm), pxp = pr(Cxp, rxp), pym = pr(Cym, rym),
          pyp = pr(Cyp, ryp);
  const R u0 = C0[1] * r0, v0 = C0[2] * r0;
  const R i2x = R(1.0 / (2.0 * g.dx)), i2y = R(1.0 / (2.0 * g.dy));
  const R ux = (Cxp[1] * rxp - Cxm[1] * rxm) * i2x;
  const R vx = (Cxp[2] * rxp - Cxm[2] * rxm) * i2x;
  const R Tx = (pxp * rxp - pxm * rxm) * i2x;
  const R uy = (Cyp[1] * ryp - Cym[1] * rym) * i2y;
  const R vy = (Cyp[2] * ryp - Cym[2] * rym) * i2y;
  const R Ty = (pyp * ryp - pym * rym) * i2y;
  const R c0 = sqrt(ph.gam * p0 * r0);
  R Fv[4];
  visc_flux2(0, u0, v0, ux, vx, Tx, uy, vy, Ty, ph, Fv);
  o[0] = C0[1] - Fv[0];
  o[1] = C0[1] * u0 + p0 - Fv[1];
  o[2] = C0[2] * u0 - Fv[2];
  o[3] = (C0[3] + p0) * u0 - Fv[3];
  visc_flux2(1, u0, v0, ux, vx, Tx, uy, vy, Ty, ph, Fv);
  o[4] = C0[2] - Fv[0];
  o[5] = C0[1] * v0 - Fv[1];
  o[6] = C0[2] * v0 + p0 - Fv[2];
  o[7] = (C0[3] + p0) * v0 - Fv[3];
  o[8] = fabs(u0) + c0;
  o[9] = fabs(v0) + c0;
  o[18] = u0;
  o[19] = v0;
  o[20] = p0;
  o[21] = p0 * r0;
  o[22] = c0;
  bvisc2_xy(p0, p0 * r0, ux, vx, Tx, uy, vy, Ty, ph, o[10], o[11]);
  const R jx = fabs(pxp - R(2.0) * p0 + pxm) / fabs(pxp + R(2.0) * p0 + pxm);
  const R jy = fabs(pyp - R(2.0) * p0 + pym) / fabs(pyp + R(2.0) * p0 + pym);
  o[12] = mx(jx, jy);
  const R div = ux + vy, curl = vx - uy;
  o[13] = mx(-div / sqrt(div * div + curl * curl + R(kDucros)), R(0.0));
#pragma unroll
  for (int k = 0; k < 4; ++k) o[14 + k] = C0[k];
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

// LDS-resident tile data
template <typename R>
struct Tile {
  R U[4][NA];   // conservative values, block +- 4
  R A[5][NA];   // u, v, p, T, c
  R G[6][NG];   // du/dx dv/dx dT/dx du/dy dv/dy dT/dy, block +- 2
  union {
    R C[23][NC];  // cell low-order data, tile +- 1
    // phase 5: y-direction flux (components 1-3) and b_y of the low-order
    // point scheme's sites, over rows 0-13 of C, which only phase 3 reads
    R SY[4][NSY];
  };
  union {
    // FP32 stencils, phase 2: centre values and their (u, v, p, T, c),
    // staged while the cells read the averages in the centre slots
    R STG[kFP64<R> ? 1 : 9 * NCEN];
    R SX[4][NSX];  // phase 5: x-direction flux (components 1-3) and b_x
  };
  R FX[4][NFX];  // limited x-face fluxes of the tile's cells
  R FY[4][NFY];  // limited y-face fluxes
  // FP64 cell averages of the tile +- 1 for the mixed-precision stage (the
  // FP64 stage reads them from C)
  double AV[4][kFP64<R> ? 1 : NC];
  // mixed-precision stage: the low part V - float(V) of the FP64 value V of
  // each of the tile's point DOFs, so that phase 5 has V to 48 bits from
  // U (the high part) without reading the state again
  float PL[4][kFP64<R> ? 1 : NPT];
  // FP64 stage: the cell averages at the centre sites of the lattice region
  // (the centre slots of U take the Simpson centres in phase 2)
  R AVG[4][kFP64<R> ? NCEN : 1];
};
static_assert(4 * NSY <= 14 * NC, "the y-direction site data fit in rows 0-13 of C");

// auxiliaries (u, v, p, T, c) of LDS lattice site s from its FP64 value V:
// the pressure of a state whose internal energy is a small part of its
// total is a difference of nearly equal numbers, so it is taken in FP64
// before the FP32 stencils see it
template <typename R>
__device__ __forceinline__ void store_aux(Tile<R>& T, const PhysT<double>& pd, int s,
                                          const double* V) {
  const double ir = rcp(V[0]);
  const double p = pd.gm1 * (V[3] - 0.5 * (V[1] * V[1] + V[2] * V[2]) * ir);
  const double Tt = p * ir;
  T.A[0][s] = R(V[1] * ir);
  T.A[1][s] = R(V[2] * ir);
  T.A[2][s] = R(p);
  T.A[3][s] = R(Tt);
  T.A[4][s] = R(sqrt(pd.gam * Tt));
}

// total flux F_d = F^c_d - F^v_d at an LDS site (a: block+-4 index, q: block+-2 index)
template <typename R>
__device__ __forceinline__ void site_flux(const Tile<R>& T, const PhysT<R>& ph, int a, int q,
                                          int d, R* F) {
  const R m1 = T.U[1][a], m2 = T.U[2][a], E = T.U[3][a];
  const R u = T.A[0][a], v = T.A[1][a], p = T.A[2][a];
  R Fv[4];
  visc_flux2(d, u, v, T.G[0][q], T.G[1][q], T.G[2][q], T.G[3][q], T.G[4][q], T.G[5][q], ph, Fv);
  const R ud = d == 0 ? u : v;
  F[0] = (d == 0 ? m1 : m2) - Fv[0];
  F[1] = m1 * ud + (d == 0 ? p : R(0.0)) - Fv[1];
  F[2] = m2 * ud + (d == 1 ? p : R(0.0)) - Fv[2];
  F[3] = (E + p) * ud - Fv[3];
}

// total flux F_d = F^c_d - F^v_d of state (m1, m2, E) with velocity (u, v),
// pressure p and gradients gr = (u_x, v_x, T_x, u_y, v_y, T_y)
template <typename R>
__device__ __forceinline__ void tot_flux(int d, const R* U, R u, R v, R p, const R* gr,
                                         const PhysT<R>& ph, R* F) {
  R Fv[4];
  visc_flux2(d, u, v, gr[0], gr[1], gr[2], gr[3], gr[4], gr[5], ph, Fv);
  const R ud = d == 0 ? u : v;
  F[0] = U[1 + d] - Fv[0];
  F[1] = U[1] * ud + (d == 0 ? p : R(0.0)) - Fv[1];
  F[2] = U[2] * ud + (d == 1 ? p : R(0.0)) - Fv[2];
  F[3] = (U[3] + p) * ud - Fv[3];
}

// The low-order point scheme works on the half lattice whose point sites hold
// the point values and whose centre sites hold the cell averages (Sec. 3.4
// with the LLF flux of Sec. 3.1).  Sites are addressed by their coordinates
// (lx, ly) in the LDS lattice region; a centre site (both odd) reads the cell
// data of phase 2.
__device__ __forceinline__ int lo_cell(int lx, int ly) {
  return ((ly - 3) >> 1) * WC + ((lx - 3) >> 1);
}
template <typename R>
__device__ __forceinline__ void lo_z(const Tile<R>& T, int lx, int ly, R& u, R& v, R& t) {
  if (lx & ly & 1) {
    const int c = lo_cell(lx, ly);
    u = T.C[18][c];
    v = T.C[19][c];
    t = T.C[21][c];
  } else {
    const int a = ly * WA + lx;
    u = T.A[0][a];
    v = T.A[1][a];
    t = T.A[3][a];
  }
}
// state and (u, v, p, T, c) of a site
template <typename R>
__device__ __forceinline__ void lo_state(const Tile<R>& T, int lx, int ly, R* U, R* w) {
  if (lx & ly & 1) {
    const int c = lo_cell(lx, ly);
#pragma unroll
    for (int k = 0; k < 4; ++k) U[k] = T.C[14 + k][c];
#pragma unroll
    for (int k = 0; k < 5; ++k) w[k] = T.C[18 + k][c];
  } else {
    const int a = ly * WA + lx;
#pragma unroll
    for (int k = 0; k < 4; ++k) U[k] = T.U[k][a];
#pragma unroll
    for (int k = 0; k < 5; ++k) w[k] = T.A[k][a];
  }
}
// low-order gradient at a site: central differences of Z = (u, v, T) over the
// four neighbouring sites, half a cell away
template <typename R>
__device__ __forceinline__ void lo_grad(const Tile<R>& T, int lx, int ly, R ihx, R ihy, R* gr) {
  R um, vm, tm, up, vp, tp;
  lo_z(T, lx - 1, ly, um, vm, tm);
  lo_z(T, lx + 1, ly, up, vp, tp);
  gr[0] = (up - um) * ihx;
  gr[1] = (vp - vm) * ihx;
  gr[2] = (tp - tm) * ihx;
  lo_z(T, lx, ly - 1, um, vm, tm);
  lo_z(T, lx, ly + 1, up, vp, tp);
  gr[3] = (up - um) * ihy;
  gr[4] = (vp - vm) * ihy;
  gr[5] = (tp - tm) * ihy;
}

// x- or y-direction data of the low-order point scheme at a site: the total
// flux F_d (its density component is the momentum, not stored) and b_d, as
// SX/SY entry o
template <typename R>
__device__ __forceinline__ void lo_site(Tile<R>& T, const PhysT<R>& ph, int lx, int ly, R ihx,
                                        R ihy, bool need_x, bool need_y, int ox, int oy) {
  R U[4], w[5], gr[6];
  lo_state(T, lx, ly, U, w);
  lo_grad(T, lx, ly, ihx, ihy, gr);
#pragma unroll
  for (int d = 0; d < 2; ++d) {
    if (!(d == 0 ? need_x : need_y)) continue;
    R F[4];
    tot_flux(d, U, w[0], w[1], w[2], gr, ph, F);
    const R b = bvisc2_dir(d, w[2], w[3], gr[0], gr[1], gr[2], gr[3], gr[4], gr[5], ph);
    R* S = d == 0 ? &T.SX[0][0] : &T.SY[0][0];
    const int n = d == 0 ? NSX : NSY, o = d == 0 ? ox : oy;
    S[o] = F[1];
    S[n + o] = F[2];
    S[2 * n + o] = F[3];
    S[3 * n + o] = b;
  }
}

// direction-d part of the low-order point update of Sec. 3.4: the point at
// (lx, ly) moves by U^L - U = -sum_d L_d with
// L_d = (2 dt/h_d) (F^L(z, z+e_d) - F^L(z-e_d, z)) and the LLF flux
// F^L(a, b) = (F_a + F_b)/2 - (max(|u_d|+c) + max(b_d))/2 (U_b - U_a),
// from the site data of lo_site.  d is a lane value (lanes of one wave take
// either direction)
template <typename R>
__device__ __forceinline__ void lo_point_dir(const Tile<R>& T, int lx, int ly, int d, double h,
                                             double dt, R* L) {
  R U0[4], w0[5];
  lo_state(T, lx, ly, U0, w0);
  const int sx = lx - 3, sy = ly - 3;
  const R* S = d ? &T.SY[0][0] : &T.SX[0][0];
  const int n = d ? NSY : NSX;
  const int o0 = d ? sy * (2 * TX) + sx - 1 : (sy - 1) * SW + sx;
  const int st = d ? 2 * TX : 1;
  const R F0[4] = {d ? U0[2] : U0[1], S[o0], S[n + o0], S[2 * n + o0]};
  const R b0 = S[3 * n + o0];
  const R r0 = fabs(d ? w0[1] : w0[0]) + w0[4];
  R Fp[4];
#pragma unroll
  for (int sg = 1; sg >= -1; sg -= 2) {
    const int nx = lx + (d ? 0 : sg), ny = ly + (d ? sg : 0);
    const int on = o0 + sg * st;
    R Un[4], wn[5];
    lo_state(T, nx, ny, Un, wn);
    const R Fn[4] = {d ? Un[2] : Un[1], S[on], S[n + on], S[2 * n + on]};
    const R bn = S[3 * n + on];
    const R lam = mx(r0, fabs(d ? wn[1] : wn[0]) + wn[4]) + mx(b0, bn);
    if (sg == 1) {
#pragma unroll
      for (int k = 0; k < 4; ++k)
        Fp[k] = R(0.5) * (F0[k] + Fn[k]) - R(0.5) * lam * (Un[k] - U0[k]);
    } else {
      const R c = R(2.0 * dt / h);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const R Fm = R(0.5) * (Fn[k] + F0[k]) - R(0.5) * lam * (U0[k] - Un[k]);
        L[k] = c * (Fp[k] - Fm);
      }
    }
  }
}

// value of x in the other lane of this lane's pair (lanes 2m and 2m+1), by
// a quad permutation (1, 0, 3, 2)
__device__ __forceinline__ float pair_swap(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0xB1, 0xF, 0xF, false));
}
__device__ __forceinline__ double pair_swap(double x) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(v >> 32), 0xB1, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// direction-d terms of the residual of the point at LDS site a (block +- 2
// index q), in components (rho, m_x, m_y, E): the biased inviscid operators
// with the downwind point, written as D+(F+) + D-(F-) = D_c(F) + alpha/(6h)
// times the fourth difference with alpha the max of |u_d| + c over the five
// sites of the line; the compact D^{(d),2}(K_dd, Z); the mixed term
// D_c^{(d)}(K_{d,o} D_c^{(o)} Z) with o the other direction (Sec. 2.2).  It
// is computed in components (rho, m_d, m_o, E), m_d the momentum along d and
// m_o the other, with a the velocity along d and b the other, so that both
// directions run the same instructions (d may differ between the lanes of a
// wave)
template <typename R>
__device__ __forceinline__ void point_resid_dir(const Tile<R>& T, const PhysT<R>& ph, int a, int q,
                                                int d, double h, R* Rd) {
  const int sa = d ? WA : 1, sq = d ? WG : 1;
  const R i6h = R(1.0 / (6.0 * h));
  const R* Md = T.U[1 + d];
  const R* Mo = T.U[2 - d];
  const R* Va = T.A[d];
  const R* Vb = T.A[1 - d];
  // derivatives across d of the velocity along d and of the other one
  const R* Ga = T.G[d ? 1 : 3];
  const R* Gb = T.G[d ? 0 : 4];
  R alpha = R(0.0);
#pragma unroll
  for (int o = 0; o < 5; ++o) {
    const int b = a + (o - 2) * sa;
    alpha = mx(alpha, fabs(Va[b]) + T.A[4][b]);
  }
  R Rr[4];
  // inviscid, one component at a time (short live ranges)
  const R ai = alpha * i6h;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    R f[5], w[5];
#pragma unroll
    for (int o = 0; o < 5; ++o) {
      const int b = a + (o - 2) * sa;
      const R ud = Va[b], pb = T.A[2][b];
      w[o] = k == 0 ? T.U[0][b] : (k == 1 ? Md[b] : (k == 2 ? Mo[b] : T.U[3][b]));
      f[o] = k == 0 ? Md[b] : (k == 1 ? w[o] * ud + pb : (k == 2 ? w[o] * ud : (w[o] + pb) * ud));
    }
    Rr[k] = -(dc5(f[0], f[1], f[3], f[4], i6h) + ai * d4(w[0], w[1], w[2], w[3], w[4]));
  }
  R va[5], vb[5], Tt[5];
#pragma unroll
  for (int o = 0; o < 5; ++o) {
    const int b = a + (o - 2) * sa;
    va[o] = Va[b];
    vb[o] = Vb[b];
    Tt[o] = T.A[3][b];
  }
  // compact D^{(d),2}(K_dd, Z)
  const R s4 = R(4.0 / (h * h));
  const R mu = ph.mu, m43 = R(4.0 / 3.0) * ph.mu;
  Rr[1] += s4 * m43 * bcol(va);
  Rr[2] += s4 * mu * bcol(vb);
  Rr[3] += s4 * (m43 * bquad(va) + mu * bquad(vb) + ph.kap * bcol(Tt));
  // mixed
  R m1[5], m2[5], m3[5];
#pragma unroll
  for (int o = 0; o < 5; ++o) {
    if (o == 2) {
      m1[o] = m2[o] = m3[o] = R(0.0);
      continue;
    }
    const int qq = q + (o - 2) * sq;
    const R ga = Ga[qq], gb = Gb[qq];
    m1[o] = -R(2.0 / 3.0) * mu * gb;
    m2[o] = mu * ga;
    m3[o] = mu * (vb[o] * ga - R(2.0 / 3.0) * va[o] * gb);
  }
  Rr[1] += dc5(m1[0], m1[1], m1[3], m1[4], i6h);
  Rr[2] += dc5(m2[0], m2[1], m2[3], m2[4], i6h);
  Rr[3] += dc5(m3[0], m3[1], m3[3], m3[4], i6h);
  // back to (rho, m_x, m_y, E)
  Rd[0] = Rr[0];
  Rd[1] = d ? Rr[2] : Rr[1];
  Rd[2] = d ? Rr[1] : Rr[2];
  Rd[3] = Rr[3];
}

// raw values of the lattice region of the tile at (X0, Y0): point sites hold
// their DOF, centre sites the cell average, ghosts as boundary images.  Each
// thread gathers the sites tid, tid+NT, tid+2NT into registers, with the
// image's momentum sign flips as bits: the loads are only issued here, and
// nothing waits for them before the values are stored to LDS.
constexpr int kRawPerThread = (NA + NT - 1) / NT;

__device__ __forceinline__ void load_raw(const G2& g, const double* __restrict__ Uk, int X0, int Y0,
                                         int tid, double (&pre)[kRawPerThread][4],
                                         int (&flip)[kRawPerThread]) {
  const int Xlim = 2 * __builtin_amdgcn_readfirstlane(g.n1);
  const int Ylim = 2 * __builtin_amdgcn_readfirstlane(g.n2);
  // a region inside the grid on both axes (no ghost site, no periodic seam):
  // every site is read where it is, with no image map
  if (X0 >= 4 && X0 - 4 + WA <= Xlim && Y0 >= 4 && Y0 - 4 + HA <= Ylim) {
#pragma unroll
    for (int r = 0; r < kRawPerThread; ++r) {
      const int s = tid + r * NT;
      if (s >= NA) continue;
      flip[r] = 0;
      long o;
      int st;
      site_ofs(g, X0 - 4 + s % WA, Y0 - 4 + s / WA, o, st);
      const double* src = Uk + o;
#pragma unroll
      for (int k = 0; k < 4; ++k) pre[r][k] = src[(long)k * st];
    }
    return;
  }
#pragma unroll
  for (int r = 0; r < kRawPerThread; ++r) {
    const int s = tid + r * NT;
    const int X = X0 - 4 + s % WA, Y = Y0 - 4 + s / WA;
    if (s >= NA || X > Xlim + kMargin || Y > Ylim + kMargin) continue;
    int kx, ky;
    const int Xi = axis_image(X, Xlim, g.bc0, g.bc1, kx);
    const int Yi = axis_image(Y, Ylim, g.bc2, g.bc3, ky);
    flip[r] = image_flips(kx, ky);
    long o;
    int st;
    site_ofs(g, Xi, Yi, o, st);
    const double* src = Uk + o;
#pragma unroll
    for (int k = 0; k < 4; ++k) pre[r][k] = src[(long)k * st];
  }
}

// Tiles are visited by persistent workgroups.  Workgroups are dispatched to
// the eight XCDs round-robin by index, so the tiles are cut into eight
// contiguous bands, one per XCD: neighbouring tiles (whose lattice regions
// overlap) are then read through the same L2.
struct TileIter {
  int cur, end, step;
  __device__ TileIter(int ntiles, int wg, int nwg) {
    if (nwg >= 8 && nwg % 8 == 0) {
      const int xcd = wg % 8, local = wg / 8;
      cur = (int)((long)xcd * ntiles / 8) + local;
      end = (int)((long)(xcd + 1) * ntiles / 8);
      step = nwg / 8;
    } else {
      cur = wg;
      end = ntiles;
      step = nwg;
    }
  }
  __device__ int get() const { return cur < end ? cur : -1; }
  __device__ int advance() {
    cur += step;
    return get();
  }
};

// launch arguments of a stage: one instance, or a batch of 2D instances
constexpr int kMaxBatch = 512;
struct StageArgs {
  // one instance
  G2 g;
  Phys ph;
  const double* Uk;
  const double* Un;
  double* Uout;
  const double* dt_dev;
  double dt_host;
  unsigned* flags;
  int ntx;
  // learned blend (one instance): a blend coefficient per face replacing
  // theta^s, or NULL; and where to write theta^s per face, or NULL
  const float* blend;
  float* ts_out;
  // a batch: its instances (stage k reads and writes their rotating buffers)
  afi::BatchInst* inst;
  int ninst, k;
  const int* n_active;
  // one instance whose step machinery lives on the device (a single
  // descriptor; stage k of its current attempt, nothing once it is
  // inactive), or NULL: then Uk, Un, Uout, dt and flags above are used.
  // Its last stage leaves the CFL maxima of the new state in cfl_partial
  // (a at [wg], v at [kSingleCflBlocks + wg]), for the next step's dt
  afi::BatchInst* dinst;
  double* cfl_partial;
  // both
  double ca, cb;
  int first, skip_flagged, ntiles;
};

// what one tile of a stage works on.  Geometry and physics are referenced,
// not copied: a copy would hold some thirty uniform values live across the
// whole tile (register pressure of a kernel that is at its VGPR limit), while
// a reference to the kernel arguments or to the batch descriptor in global
// memory is re-read where needed.
struct TileArgs {
  const G2* g;
  const Phys* phd;
  const double* Uk;
  const double* Un;
  double* Uout;
  double dt;
  unsigned* flags;
  int ntx, lt;  // tiles along x of its grid, the tile's index in its grid
};

// position of tile t in a batch's list of n active instances whose first
// tiles are t0[0] = 0 < t0[1] < ...
__device__ __forceinline__ int batch_slot_of(const int* t0, int n, int t) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (t0[mid] <= t)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// tile t of the active tiles of a batch: active instance j is instance
// id[j] and owns tiles [t0[j], t0[j + 1])
__device__ __forceinline__ TileArgs batch_tile(const StageArgs& sa, const int* t0, const int* id,
                                               int nact, int t) {
  // the instance is the same for the whole workgroup
  const int j = __builtin_amdgcn_readfirstlane(batch_slot_of(t0, nact, t));
  const int in = __builtin_amdgcn_readfirstlane(id[j]);
  const afi::BatchInst& I = sa.inst[in];
  TileArgs A;
  A.g = &I.g;
  A.phd = &I.ph;
  A.ntx = I.ntx;
  A.lt = t - t0[j];
  A.dt = I.dt;
  A.flags = &sa.inst[in].flags;
  // the three RK3 stages from buf[cur], through the other two buffers
  const int c = I.cur, a = (c + 1) % 3, b = (c + 2) % 3;
  A.Un = I.buf[c];
  A.Uk = sa.k == 0 ? I.buf[c] : (sa.k == 1 ? I.buf[a] : I.buf[b]);
  A.Uout = sa.k == 1 ? I.buf[b] : I.buf[a];
  return A;
}

// BLEND: the single-instance kernel with per-face blend input/output arrays
// (its own instance, so that the plain stage carries none of that code)
// DEV: the single-instance kernel of a device-resident step loop, whose
// buffers, dt and flag word come from the descriptor sa.dinst
template <typename R, bool BATCH, bool BLEND = false, bool DEV = false>
__global__ void __launch_bounds__(NT) k_stage(StageArgs sa) {
  __shared__ Tile<R> T;
  __shared__ unsigned stop;  // workgroup-uniform copy of the flag word
  const int tid = threadIdx.x;
  const double ca = sa.ca, cb = sa.cb;
  const int first = sa.first, skip_flagged = sa.skip_flagged;
  bool nonfinite = false;
  // DEV, last stage: CFL rate maxima of the cells this thread writes
  double cfl_a = 0.0, cfl_v = 0.0;
  // a batch: only the tiles of its active instances are numbered, so that
  // every XCD band holds an equal share of the work whichever instances are
  // active (instances finish their steps after different numbers of
  // attempts).  Active instance j is instance bid[j] and owns tiles
  // [bt0[j], bt0[j] + its ntiles); the numbering comes from two inclusive
  // scans over the instances (one per thread), done in place in bt0 / bid.
  __shared__ int bt0[BATCH ? kMaxBatch : 1], bid[BATCH ? kMaxBatch : 1];
  int ntiles = sa.ntiles, nact = 0;
  if constexpr (BATCH) {
    static_assert(kMaxBatch == NT, "one instance per thread in the scans");
    if (*sa.n_active == 0) return;  // every instance has finished its step
  }
  if (BATCH && sa.ninst == 1) {
    // one instance, active (n_active is not 0): its tiles are all the tiles
    if (tid == 0) {
      bid[0] = 0;
      bt0[0] = 0;
    }
    nact = 1;
    ntiles = sa.inst[0].ntiles;
    __syncthreads();
  } else if constexpr (BATCH) {
    const bool act = tid < sa.ninst && sa.inst[tid].active;
    const int own = act ? sa.inst[tid].ntiles : 0;
    bid[tid] = act ? 1 : 0;
    bt0[tid] = own;
    __syncthreads();
    for (int off = 1; off < NT; off <<= 1) {
      const int c = tid >= off ? bid[tid - off] : 0;
      const int t = tid >= off ? bt0[tid - off] : 0;
      __syncthreads();
      bid[tid] += c;
      bt0[tid] += t;
      __syncthreads();
    }
    const int pos = bid[tid] - 1, first_tile = bt0[tid] - own;
    nact = bid[NT - 1];
    ntiles = bt0[NT - 1];
    __syncthreads();
    if (act) {
      bid[pos] = tid;
      bt0[pos] = first_tile;
    }
    __syncthreads();
  }
  // the one instance's buffers, dt and flag word, read once (a per-tile read
  // of dt costs ~3% of the stage)
  double dt1 = 0.0;
  const double* Uk1 = nullptr;
  const double* Un1 = nullptr;
  double* Uout1 = nullptr;
  unsigned* flags1 = nullptr;
  if constexpr (!BATCH) {
    if constexpr (DEV) {
      const afi::BatchInst& I = *sa.dinst;
      if (!I.active) return;  // its step is done; the round has nothing to do
      // the three RK3 stages from buf[cur], through the other two buffers
      const int c = I.cur, a = (c + 1) % 3, b = (c + 2) % 3;
      Un1 = I.buf[c];
      Uk1 = sa.k == 0 ? I.buf[c] : (sa.k == 1 ? I.buf[a] : I.buf[b]);
      Uout1 = sa.k == 1 ? I.buf[b] : I.buf[a];
      dt1 = I.dt;
      flags1 = &sa.dinst->flags;
    } else {
      dt1 = sa.dt_dev ? *sa.dt_dev : sa.dt_host;
    }
  }
  // what tile t works on (built where used, from the kernel arguments or the
  // batch descriptors, so that nothing of it stays live across tiles)
  auto args = [&](int t) {
    if constexpr (BATCH) {
      return batch_tile(sa, bt0, bid, nact, t);
    } else {
      TileArgs A;
      A.g = &sa.g;
      A.phd = &sa.ph;
      A.Uk = DEV ? Uk1 : sa.Uk;
      A.Un = DEV ? Un1 : sa.Un;
      A.Uout = DEV ? Uout1 : sa.Uout;
      A.dt = dt1;
      A.flags = DEV ? flags1 : sa.flags;
      A.ntx = sa.ntx;
      A.lt = t;
      return A;
    }
  };
  TileIter it(ntiles, blockIdx.x, gridDim.x);
  int tile = it.get();
  double pre[kRawPerThread][4];
  int flip[kRawPerThread] = {};
  // a batch: whether pre holds the current tile's raw values (tiles of an
  // instance whose attempt is rejected are passed over without loading them)
  bool have_pre = true;
  if (tile >= 0) {
    const TileArgs A = args(tile);
    load_raw(*A.g, A.Uk, 2 * TX * (A.lt % A.ntx), 2 * TY * (A.lt / A.ntx), tid, pre, flip);
  }
  while (tile >= 0) {
  const TileArgs A = args(tile);
  const G2& g = *A.g;
  const Phys& phd = *A.phd;
  const PhysT<R> ph = phys_as<R>(phd);
  const PhysT<double> phd64 = phys_as<double>(phd);
  const double* __restrict__ Uk = A.Uk;
  const double* __restrict__ Un = A.Un;
  double* __restrict__ Uout = A.Uout;
  const double dt = A.dt;
  unsigned* flags = A.flags;
  const int Xlim = 2 * g.n1, Ylim = 2 * g.n2;
  const int i0 = (A.lt % A.ntx) * TX, j0 = (A.lt / A.ntx) * TY;
  const int X0 = 2 * i0, Y0 = 2 * j0;
  // inside a step attempt, stop once any workgroup has flagged the attempt:
  // it is rejected and this output is never read (a batch skips the tiles of
  // that instance only)
  if (tid == 0) stop = skip_flagged ? peek_flags(flags) : 0u;
  __syncthreads();  // the previous tile is done with the LDS; stop is visible
  if (stop) {
    if constexpr (BATCH) {
      // with one active instance every later tile is that instance's too
      if (nact == 1) break;
      // every wave has read `stop` before thread 0 writes it for the next
      // tile, which is loaded only once it is known not to be skipped too
      __syncthreads();
      tile = it.advance();
      have_pre = false;
      continue;
    } else {
      break;
    }
  }
  if constexpr (BATCH) {
    if (!have_pre) {
      load_raw(g, Uk, X0, Y0, tid, pre, flip);
      have_pre = true;
    }
  }

  // ---- phase 0a: raw values of the lattice region (prefetched) ----
#pragma unroll
  for (int r = 0; r < kRawPerThread; ++r) {
    const int s = tid + r * NT;
    const int X = X0 - 4 + s % WA, Y = Y0 - 4 + s / WA;
    if (s >= NA || X > Xlim + kMargin || Y > Ylim + kMargin) continue;
    double V[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const bool neg = (k == 1 && (flip[r] & 1)) || (k == 2 && (flip[r] & 2));
      V[k] = neg ? -pre[r][k] : pre[r][k];
    }
    if constexpr (kFP64<R>) {
      // FP64: averages to AVG, point values to U
      if ((X & 1) && (Y & 1)) {
        const int ci = ((s / WA - 1) >> 1) * (TX + 4) + ((s % WA - 1) >> 1);
#pragma unroll
        for (int k = 0; k < 4; ++k) T.AVG[k][ci] = V[k];
      } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) T.U[k][s] = V[k];
      }
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) T.U[k][s] = R(V[k]);
    }
    // FP32 stencils: the point sites' (u, v, p, T, c) from the FP64 values
    // (centre sites get the Simpson centre's); the FP64 stage takes them in
    // phase 2, where they cost fewer live registers.  The FP64 averages of
    // the tile's cells +- 1 go to AV, and the low parts of the FP64 values
    // of the tile's own points to PL, for the FP64 updates
    if constexpr (!kFP64<R>) {
      const int lx = X - X0, ly = Y - Y0;
      if ((X & 1) && (Y & 1)) {
        const int ci = (lx + 1) >> 1, cj = (ly + 1) >> 1;  // cell offset + 1
        if (lx >= -1 && ly >= -1 && ci <= TX + 1 && cj <= TY + 1) {
#pragma unroll
          for (int k = 0; k < 4; ++k) T.AV[k][cj * WC + ci] = V[k];
        }
      } else {
        store_aux(T, phd64, s, V);
        if (lx >= 0 && ly >= 0 && lx < 2 * TX && ly < 2 * TY) {
          // point type 0 x-edge (X even, Y odd), 1 y-edge, 2 corner
          const int pt = (X & 1) ? 1 : ((Y & 1) ? 0 : 2);
          const int pi = pt * (TX * TY) + (ly >> 1) * TX + (lx >> 1);
#pragma unroll
          for (int k = 0; k < 4; ++k) T.PL[k][pi] = float(V[k] - double(float(V[k])));
        }
      }
    }
  }
  __syncthreads();

  // ---- phase 2: centre values (Simpson + scaling; waves 4-7, compact
  //      mapping, staged until the cells have read the averages in the centre
  //      slots), cell low-order data of the tile +- 1 (waves 0-2),
  //      auxiliaries of the point sites (all; FP64 stage only, the FP32
  //      stencils took theirs in phase 0a) ----
  // lattice slot of centre cidx of the region, or -1 beyond the grid's ghosts
  auto centre_slot = [&](int cidx) {
    const int X = X0 - 3 + 2 * (cidx % (TX + 4)), Y = Y0 - 3 + 2 * (cidx / (TX + 4));
    return (X <= Xlim + kMargin && Y <= Ylim + kMargin) ? (Y - Y0 + 4) * WA + (X - X0 + 4) : -1;
  };
  for (int cidx = tid - NT / 2; cidx >= 0 && cidx < NCEN; cidx += NT / 2) {
    const int cs = centre_slot(cidx);
    const int X = X0 - 3 + 2 * (cidx % (TX + 4)), Y = Y0 - 3 + 2 * (cidx / (TX + 4));
    // a centre beyond a wall or outflow side is taken from its image below;
    // periodic ghosts are computed here, from the wrapped values
    if (cs >= 0 && !ghost_centre(g, X, Y)) {
      R Ub[4], e[4], cc[4], cV[4], cw[5];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const R* z = T.U[k];
        Ub[k] = kFP64<R> ? T.AVG[k][cidx] : z[cs];
        e[k] = z[cs - 1] + z[cs + 1] + z[cs - WA] + z[cs + WA];
        cc[k] = z[cs - WA - 1] + z[cs - WA + 1] + z[cs + WA - 1] + z[cs + WA + 1];
      }
      centre_value(ph, phd, Ub, e, cc, cV, cw);
      if constexpr (kFP64<R>) {
        // the cells read the averages from AVG: the centre goes in place
#pragma unroll
        for (int k = 0; k < 4; ++k) T.U[k][cs] = cV[k];
#pragma unroll
        for (int k = 0; k < 5; ++k) T.A[k][cs] = cw[k];
      } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) T.STG[k * NCEN + cidx] = cV[k];
#pragma unroll
        for (int k = 0; k < 5; ++k) T.STG[(4 + k) * NCEN + cidx] = cw[k];
      }
    }
  }
  // cells: the first NT/2 on waves 0-3, the rest from the top thread down
  // (waves 7, 6, ...), away from the waves 4 and 5 that take the centres'
  // second round when there is one
  static_assert(NC <= NT, "one cell per thread");
  {
    const int s = tid < NT / 2 ? tid : NT / 2 + (NT - 1 - tid);
    const int i = i0 - 1 + s % WC, j = j0 - 1 + s / WC;
    if (s < NC && i <= g.n1 && j <= g.n2) {
    R C0[4], Cxm[4], Cxp[4], Cym[4], Cyp[4], o[23];
    if constexpr (kFP64<R>) {
      // the cell's index among the centres of the region
      const int c = (s / WC + 1) * (TX + 4) + s % WC + 1;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        C0[k] = T.AVG[k][c];
        Cxm[k] = T.AVG[k][c - 1];
        Cxp[k] = T.AVG[k][c + 1];
        Cym[k] = T.AVG[k][c - (TX + 4)];
        Cyp[k] = T.AVG[k][c + (TX + 4)];
      }
    } else {
      const int a = (2 * j + 1 - Y0 + 4) * WA + (2 * i + 1 - X0 + 4);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        C0[k] = T.U[k][a];
        Cxm[k] = T.U[k][a - 2];
        Cxp[k] = T.U[k][a + 2];
        Cym[k] = T.U[k][a - 2 * WA];
        Cyp[k] = T.U[k][a + 2 * WA];
      }
    }
    cell_low(g, ph, C0, Cxm, Cxp, Cym, Cyp, o);
#pragma unroll
    for (int k = 0; k < 23; ++k) T.C[k][s] = o[k];
    }
  }
  if constexpr (kFP64<R>) {
    // the point sites of the lattice region, numbered p: each pair of rows
    // (an even one, all 41 sites points; an odd one, its 21 even sites)
    // holds 62 of them, so no lane falls on a centre
    constexpr int PPR = WA + (WA + 1) / 2;  // points per pair of rows
    constexpr int NPS = (HA + 1) / 2 * WA + HA / 2 * ((WA + 1) / 2);
    auto aux_point = [&](int p) {
      const int r2 = p / PPR, m = p % PPR;
      const int ly = m < WA ? 2 * r2 : 2 * r2 + 1, lx = m < WA ? m : 2 * (m - WA);
      const int s = ly * WA + lx;
      const int X = X0 - 4 + lx, Y = Y0 - 4 + ly;
      if (X > Xlim + kMargin || Y > Ylim + kMargin) return;
      const double V[4] = {T.U[0][s], T.U[1][s], T.U[2][s], T.U[3][s]};
      store_aux(T, phd64, s, V);
    };
    // one site per thread, then the rest on waves 3 and 7: the SIMD they
    // share (waves go to the SIMDs round-robin) updates no cells
    if (tid < NPS) aux_point(tid);
    const int wv = tid >> 6;
    if (wv == 3 || wv == 7) {
      for (int p = NT + (tid & 63) + (wv == 7 ? 64 : 0); p < NPS; p += 128) aux_point(p);
    }
  }
  __syncthreads();
  if constexpr (!kFP64<R>) {
    for (int cidx = tid - NT / 2; cidx >= 0 && cidx < NCEN; cidx += NT / 2) {
      const int cs = centre_slot(cidx);
      if (cs < 0) continue;
#pragma unroll
      for (int k = 0; k < 4; ++k) T.U[k][cs] = T.STG[k * NCEN + cidx];
#pragma unroll
      for (int k = 0; k < 5; ++k) T.A[k][cs] = T.STG[(4 + k) * NCEN + cidx];
    }
    __syncthreads();
  }
  // ghost centres: the value and (u, v, p, T, c) of the image centre, with
  // the image's momentum and velocity signs.  Ghosts reach at most four
  // lattice lines past a side, so the image (a mirror or the first interior
  // centre; along a periodic axis the unwrapped ghost itself) lies in this
  // tile's region, and phase 2 computed it from the same values in the same
  // order as the image's own Simpson value: the copy is that value exactly
  if (!(X0 >= 4 && X0 - 4 + WA <= Xlim && Y0 >= 4 && Y0 - 4 + HA <= Ylim)) {
    for (int cidx = tid; cidx < NCEN; cidx += NT) {
      const int cs = centre_slot(cidx);
      const int X = X0 - 3 + 2 * (cidx % (TX + 4)), Y = Y0 - 3 + 2 * (cidx / (TX + 4));
      if (cs < 0 || !ghost_centre(g, X, Y)) continue;
      int kx = -1, ky = -1;
      const int Xi = g.bc0 == BC_PERIODIC ? X : axis_image(X, Xlim, g.bc0, g.bc1, kx);
      const int Yi = g.bc2 == BC_PERIODIC ? Y : axis_image(Y, Ylim, g.bc2, g.bc3, ky);
      const int f = image_flips(kx, ky);
      const int si = (Yi - Y0 + 4) * WA + (Xi - X0 + 4);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const R v = T.U[k][si];
        T.U[k][cs] = ((k == 1 && (f & 1)) || (k == 2 && (f & 2))) ? -v : v;
      }
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        const R v = T.A[k][si];
        T.A[k][cs] = ((k == 0 && (f & 1)) || (k == 1 && (f & 2))) ? -v : v;
      }
    }
    __syncthreads();
  }

  // prefetch the next tile's raw values; the loads complete while this tile
  // computes
  const int next = it.advance();
  if (next >= 0) {
    const TileArgs An = args(next);
    load_raw(*An.g, An.Uk, 2 * TX * (An.lt % An.ntx), 2 * TY * (An.lt / An.ntx), tid, pre, flip);
  }

  // ---- phase 1: gradients on the block +- 2 ----
  {
    const R ihx = R(1.0 / (6.0 * g.dx)), ihy = R(1.0 / (6.0 * g.dy));
    for (int s = tid; s < NG; s += NT) {
      const int lx = s % WG, ly = s / WG;
      const int X = X0 - 2 + lx, Y = Y0 - 2 + ly;
      if (X > Xlim + 2 || Y > Ylim + 2) continue;
      const int a = (ly + 2) * WA + (lx + 2);
      R gr[6];
      const int src[3] = {0, 1, 3};
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const R* z = T.A[src[c]];
        gr[c] = dc5(z[a - 2], z[a - 1], z[a + 1], z[a + 2], ihx);
        gr[3 + c] = dc5(z[a - 2 * WA], z[a - WA], z[a + WA], z[a + 2 * WA], ihy);
      }
#pragma unroll
      for (int c = 0; c < 6; ++c) T.G[c][s] = gr[c];
    }
  }
  __syncthreads();

  // ---- phase 3: limited face fluxes of the tile's cells ----
  const float* blend = nullptr;
  float* ts_out = nullptr;
  if constexpr (BLEND && !BATCH) {
    blend = sa.blend;
    ts_out = sa.ts_out;
  }
  const int limc = (ph.lim & (LIM_SMOOTH | LIM_PP | LIM_LOWONLY)) | (blend ? 1 : 0);
  // FP64: the faces take waves 0-3 only; waves 4-7 compute the
  // x-direction site data of the low-order point scheme meanwhile (phase 5a
  // keeps the y-direction data, which overlay cell data the faces read)
  if constexpr (kFP64<R>) {
    static_assert(!kFP64<R> || NFX + NFY <= NT / 2, "the faces on waves 0-3");
    if ((ph.lim & LIM_POINT) && tid >= NT / 2) {
      const R ihx = R(1.0 / g.dx), ihy = R(1.0 / g.dy);
      for (int s = tid - NT / 2; s < NSX; s += NT / 2) {
        const int sx = s % SW, sy = 1 + s / SW;
        lo_site(T, ph, sx + 3, sy + 3, ihx, ihy, true, false, (sy - 1) * SW + sx, 0);
      }
    }
  }
  for (int s = tid; s < NFX + NFY; s += NT) {
    const int d = s < NFX ? 0 : 1;
    int ff, jj, i, j, X, Y;  // face (i,j) between cells a (minus) and b (plus)
    if (d == 0) {
      ff = s % (TX + 1);
      jj = s / (TX + 1);
      i = i0 + ff;
      j = j0 + jj;
      if (i > g.n1 || j >= g.n2) continue;
      X = 2 * i;
      Y = 2 * j + 1;
    } else {
      const int r = s - NFX;
      ff = r % TX;
      jj = r / TX;
      i = i0 + ff;
      j = j0 + jj;
      if (i >= g.n1 || j > g.n2) continue;
      X = 2 * i + 1;
      Y = 2 * j;
    }
    const int a = (Y - Y0 + 4) * WA + (X - X0 + 4);
    const int q = (Y - Y0 + 2) * WG + (X - X0 + 2);
    const int sa = d == 0 ? WA : 1, sq = d == 0 ? WG : 1;  // along the face
    R Fa[4], Fm[4], Fb[4], FH[4], F[4];
    site_flux(T, ph, a - sa, q - sq, d, Fa);
    site_flux(T, ph, a, q, d, Fm);
    site_flux(T, ph, a + sa, q + sq, d, Fb);
#pragma unroll
    for (int k = 0; k < 4; ++k) FH[k] = (Fa[k] + R(4.0) * Fm[k] + Fb[k]) * R(1.0 / 6.0);
    if (!limc) {
#pragma unroll
      for (int k = 0; k < 4; ++k) F[k] = FH[k];
    } else {
      const int cbx = (j - j0 + 1) * WC + (i - i0 + 1);
      const int cax = d == 0 ? cbx - 1 : cbx - WC;
      const R lam = mx(T.C[8 + d][cax], T.C[8 + d][cbx]) + mx(T.C[10 + d][cax], T.C[10 + d][cbx]);
      R FL[4], Fca[4], Fcb[4];
      double Ua[4], Ub[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if constexpr (kFP64<R>) {
          Ua[k] = T.C[14 + k][cax];
          Ub[k] = T.C[14 + k][cbx];
        } else {
          Ua[k] = T.AV[k][cax];
          Ub[k] = T.AV[k][cbx];
        }
        Fca[k] = T.C[4 * d + k][cax];
        Fcb[k] = T.C[4 * d + k][cbx];
        FL[k] = R(0.5) * (Fca[k] + Fcb[k]) - R(0.5) * lam * (T.C[14 + k][cbx] - T.C[14 + k][cax]);
      }
      R ts = R(1.0);
      double tpp = 1.0;
      // the face's entries in per-face arrays: x-faces [n2][n1+1], then
      // y-faces [n2+1][n1]; a periodic axis's last face is its first again
      const bool use_blend = blend != nullptr;
      if (ph.lim & LIM_LOWONLY) {
        ts = R(0.0);
        tpp = 0.0;
      } else {
        if (use_blend) {
          // the given coefficient takes the place of theta^s
          const long nfx = (long)g.n2 * (g.n1 + 1);
          const int fi = (d == 0 && i == g.n1 && g.n1x == g.n1) ? 0 : i;
          const int fj = (d == 1 && j == g.n2 && g.n2y == g.n2) ? 0 : j;
          ts = R(blend[d == 0 ? (long)fj * (g.n1 + 1) + fi : nfx + (long)fj * g.n1 + fi]);
        } else if (ph.lim & LIM_SMOOTH) {
          ts = exp(-ph.Cs * mx(T.C[12][cax], T.C[12][cbx]) * mx(T.C[13][cax], T.C[13][cbx]));
        }
        if (ph.lim & LIM_PP) {
          // the density and pressure blend in FP64 (Sec. 3.3)
          const double m4 = 4.0 * dt / (d == 0 ? g.dx : g.dy);
          double ULp[4], UHp[4], ULm[4], UHm[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const double fl = FL[k], fh = FH[k], fca = Fca[k], fcb = Fcb[k];
            const double Fs = fl + double(ts) * (fh - fl);
            ULp[k] = Ua[k] - m4 * (fl - fca);
            UHp[k] = Ua[k] - m4 * (Fs - fca);
            ULm[k] = Ub[k] - m4 * (fcb - fl);
            UHm[k] = Ub[k] - m4 * (fcb - Fs);
          }
          tpp = 0.0;
          bool bad = false;
          if (!(ULp[0] > 0.0) || !(ULm[0] > 0.0)) {
            bad = true;
          } else {
            const double pLp = pressure2(ULp[0], ULp[1], ULp[2], ULp[3], phd.gm1);
            const double pLm = pressure2(ULm[0], ULm[1], ULm[2], ULm[3], phd.gm1);
            if (!(pLp > 0.0) || !(pLm > 0.0)) bad = true;
            const double tr = mn(theta_lin(ULp[0], UHp[0], mn(kPPEps, ULp[0])),
                                 theta_lin(ULm[0], UHm[0], mn(kPPEps, ULm[0])));
            double Tp[4], Tm[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              Tp[k] = ULp[k] + tr * (UHp[k] - ULp[k]);
              Tm[k] = ULm[k] + tr * (UHm[k] - ULm[k]);
            }
            const bool ex = ph.lim & LIM_PEXACT;
            const double tp = mn(theta_p2(ULp, pLp, Tp, mn(kPPEps, pLp), phd.gm1, ex),
                                 theta_p2(ULm, pLm, Tm, mn(kPPEps, pLm), phd.gm1, ex));
            tpp = tr * tp;
          }
          if (bad) raise_flag(flags, FLAG_CELL_LOW);
        }
      }
      const double th = double(ts) * tpp;
      if (ts_out) {
        const long nfx = (long)g.n2 * (g.n1 + 1);
        ts_out[d == 0 ? (long)j * (g.n1 + 1) + i : nfx + (long)j * g.n1 + i] = float(ts);
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double fl = FL[k], fh = FH[k];
        F[k] = R(fl + th * (fh - fl));
      }
    }
    if (d == 0) {
#pragma unroll
      for (int k = 0; k < 4; ++k) T.FX[k][jj * (TX + 1) + ff] = F[k];
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) T.FY[k][jj * TX + ff] = F[k];
    }
  }
  __syncthreads();

  // ---- phase 4: cell averages (FP64 accumulation) ----
  {
    const double mxd = dt / g.dx, myd = dt / g.dy;
    const long nc = (long)g.n1 * g.n2;
    for (int s = tid; s < TX * TY; s += NT) {
      const int ii = s % TX, jj = s / TX;
      const int i = i0 + ii, j = j0 + jj;
      if (i >= g.n1 || j >= g.n2) continue;
      const int c = (jj + 1) * WC + ii + 1;
      const long gi = (long)j * g.n1 + i;
      // U^n of the cell, all four loads in flight together
      double un[4] = {0.0, 0.0, 0.0, 0.0};
      if (!first) {
#pragma unroll
        for (int k = 0; k < 4; ++k) un[k] = Un[k * nc + gi];
      }
      double o4[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double dfx = double(T.FX[k][jj * (TX + 1) + ii + 1]) - double(T.FX[k][jj * (TX + 1) + ii]);
        const double dfy = double(T.FY[k][(jj + 1) * TX + ii]) - double(T.FY[k][jj * TX + ii]);
        double av;
        if constexpr (kFP64<R>)
          av = T.C[14 + k][c];
        else
          av = T.AV[k][c];
        const double fe = av - mxd * dfx - myd * dfy;
        const double o = first ? fe : ca * un[k] + cb * fe;
        if (!isfinite(o)) nonfinite = true;
        Uout[k * nc + gi] = o;
        o4[k] = o;
      }
      if constexpr (DEV) {
        // the last stage of a device-resident step: the CFL rates (eq. cfl)
        // of the new average, as the CFL kernel takes them, for the next step
        if (sa.k == 2) {
          const double p = pressure2(o4[0], o4[1], o4[2], o4[3], phd.gm1);
          const double cs = sqrt(phd.gam * p / o4[0]);
          cfl_a = mx(cfl_a, (fabs(o4[1] / o4[0]) + cs) * sa.dinst->icx);
          cfl_a = mx(cfl_a, (fabs(o4[2] / o4[0]) + cs) * sa.dinst->icy);
          cfl_v = mx(cfl_v, sa.dinst->vcoef / o4[0]);
        }
      }
    }
  }

  // ---- phase 5a: site data of the low-order point scheme (Sec. 3.4); it
  //      shares no LDS with phase 4, and starts on the threads phase 4 leaves
  //      idle ----
  if (ph.lim & LIM_POINT) {
    const R ihx = R(1.0 / g.dx), ihy = R(1.0 / g.dy);
    auto site = [&](int s) {
      const int sx = s % SW, sy = s / SW;
      const bool need_x = !kFP64<R> && sy >= 1 && sy <= 2 * TY, need_y = sx >= 1 && sx <= 2 * TX;
      if (need_x || need_y)
        lo_site(T, ph, sx + 3, sy + 3, ihx, ihy, need_x, need_y, (sy - 1) * SW + sx,
                sy * (2 * TX) + sx - 1);
    };
    if constexpr (kFP64<R>) {
      // the y-direction data (the x-direction data came during phase 3)
      const int s = (tid + NT - TX * TY) % NT;
      if (s < NSY) {
        const int sx = 1 + s % (2 * TX), sy = s / (2 * TX);
        lo_site(T, ph, sx + 3, sy + 3, ihx, ihy, false, true, 0, sy * (2 * TX) + sx - 1);
      }
      static_assert(!kFP64<R> || NSY <= NT, "one site per thread");
    } else {
      // the first NT sites from the first thread phase 4 leaves idle on; the
      // rest from wave 3 on, away from the waves that also update cells
      const int s1 = (tid + NT - TX * TY) % NT;
      if (s1 < NSR) site(s1);
      for (int s = NT + (tid + NT - 192) % NT; s < NSR; s += NT) site(s);
    }
    __syncthreads();
  }

  // ---- phase 5: point values (0 x-edge, 1 y-edge, 2 corner points).  The
  //      FP64 stage gives each point two lanes: lane d of a pair takes the
  //      direction-d terms of the residual and of the low-order point
  //      update, the pair swaps them, and each lane finishes the point and
  //      writes two of its four components (672 half-points spread over all
  //      eight waves, where 336 whole points left two SIMDs with two waves
  //      and two with one).  The FP32-stencil stage, whose tiles hold twice
  //      the points, keeps one lane per point ----
  constexpr int LPP = kFP64<R> ? 2 : 1;  // lanes per point
  constexpr int NW = 4 / LPP;            // components a lane writes
  for (int s2 = tid; s2 < LPP * NPT; s2 += NT) {
    const int s = s2 / LPP, d = LPP == 2 ? (s2 & 1) : 0;
    const int t = s / (TX * TY), r = s % (TX * TY);
    const int ni = t == 1 ? g.n1 : g.n1x;
    const int nj = t == 0 ? g.n2 : g.n2y;
    const long np = (long)ni * nj;
    const long off = t == 0 ? g.off_xe : (t == 1 ? g.off_ye : g.off_co);
    {
      const int i = i0 + r % TX, j = j0 + r / TX;
      // both lanes of a pair take this branch together
      if (i >= ni || j >= nj) continue;
      const int X = t == 1 ? 2 * i + 1 : 2 * i;
      const int Y = t == 0 ? 2 * j + 1 : 2 * j;
      const int a = (Y - Y0 + 4) * WA + (X - X0 + 4);
      const int q = (Y - Y0 + 2) * WG + (X - X0 + 2);
      const long gi = (long)j * ni + i;
      // U^n of the components this lane writes (NW * d onwards), loaded
      // while the residual is computed
      double un[NW];
#pragma unroll
      for (int c = 0; c < NW; ++c) un[c] = first ? 0.0 : Un[off + (NW * d + c) * np + gi];
      // the residual; the two directions' terms are added in the same order
      // in both lanes of a pair
      R Rs[4];
      if constexpr (LPP == 2) {
        R Rd[4];
        point_resid_dir(T, ph, a, q, d, d ? g.dy : g.dx, Rd);
#pragma unroll
        for (int k = 0; k < 4; ++k) Rs[k] = Rd[k] + pair_swap(Rd[k]);
      } else {
        R Rx[4], Ry[4];
        point_resid_dir(T, ph, a, q, 0, g.dx, Rx);
        point_resid_dir(T, ph, a, q, 1, g.dy, Ry);
#pragma unroll
        for (int k = 0; k < 4; ++k) Rs[k] = Rx[k] + Ry[k];
      }
      // the point update and its blend in FP64, from the FP64 point value
      double U0[4], UH[4], out[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if constexpr (kFP64<R>)
          U0[k] = T.U[k][a];
        else
          U0[k] = double(T.U[k][a]) + double(T.PL[k][s]);
        UH[k] = U0[k] + dt * double(Rs[k]);
      }
      if (ph.lim & LIM_POINT) {
        double Ls[4];
        if constexpr (LPP == 2) {
          R Ld[4];
          lo_point_dir(T, X - X0 + 4, Y - Y0 + 4, d, d ? g.dy : g.dx, dt, Ld);
#pragma unroll
          for (int k = 0; k < 4; ++k) Ls[k] = double(Ld[k]) + double(pair_swap(Ld[k]));
        } else {
          R Lx[4], Ly[4];
          lo_point_dir(T, X - X0 + 4, Y - Y0 + 4, 0, g.dx, dt, Lx);
          lo_point_dir(T, X - X0 + 4, Y - Y0 + 4, 1, g.dy, dt, Ly);
#pragma unroll
          for (int k = 0; k < 4; ++k) Ls[k] = double(Lx[k]) + double(Ly[k]);
        }
        double UL[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) UL[k] = U0[k] - Ls[k];
        bool lbad = false;
        double th = theta_pair2(UL, UH, phd.gm1, lbad, ph.lim & LIM_PEXACT);
        if (ph.lim & LIM_LOWONLY) th = 0.0;
        if (lbad && d == 0) raise_flag(flags, FLAG_POINT_LOW);
#pragma unroll
        for (int k = 0; k < 4; ++k) out[k] = (th == 1.0) ? UH[k] : UL[k] + th * (UH[k] - UL[k]);
      } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) out[k] = UH[k];
      }
      if (X == 0) project(wall_of(g.bc0), 0, out);
      if (X == Xlim) project(wall_of(g.bc1), 0, out);
      if (Y == 0) project(wall_of(g.bc2), 1, out);
      if (Y == Ylim) project(wall_of(g.bc3), 1, out);
      // this lane's components (selected by value: an index computed from d
      // would put out in scratch memory)
      double v[NW];
      if constexpr (LPP == 2) {
        v[0] = d ? out[2] : out[0];
        v[1] = d ? out[3] : out[1];
      } else {
#pragma unroll
        for (int c = 0; c < NW; ++c) v[c] = out[c];
      }
#pragma unroll
      for (int c = 0; c < NW; ++c) {
        const double o = first ? v[c] : ca * un[c] + cb * v[c];
        if (!isfinite(o)) nonfinite = true;
        Uout[off + (NW * d + c) * np + gi] = o;
      }
    }
  }
  if constexpr (BATCH) {
    if (nonfinite) raise_flag(flags, FLAG_NONFINITE);
    nonfinite = false;
  }
  tile = next;
  }  // tiles
  if constexpr (!BATCH) {
    if (nonfinite) raise_flag(DEV ? flags1 : sa.flags, FLAG_NONFINITE);
  }
  if constexpr (DEV) {
    // the workgroup's CFL maxima of the new state, one pair per workgroup
    // (rates of cells this workgroup did not write are 0, neutral for max)
    if (sa.k == 2) {
      __shared__ double cfl_w[2][NT / 64];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        cfl_a = mx(cfl_a, __shfl_xor(cfl_a, o, 64));
        cfl_v = mx(cfl_v, __shfl_xor(cfl_v, o, 64));
      }
      __syncthreads();
      if ((tid & 63) == 0) {
        cfl_w[0][tid >> 6] = cfl_a;
        cfl_w[1][tid >> 6] = cfl_v;
      }
      __syncthreads();
      if (tid == 0) {
        double a = 0.0, v = 0.0;
        for (int w = 0; w < NT / 64; ++w) {
          a = mx(a, cfl_w[0][w]);
          v = mx(v, cfl_w[1][w]);
        }
        sa.cfl_partial[blockIdx.x] = a;
        sa.cfl_partial[afi::kSingleCflBlocks + blockIdx.x] = v;
      }
    }
  }
}

// persistent workgroups of a stage kernel instance: as many as fit on the
// device at once (the tile's LDS footprint decides), cached per device
template <typename R>
int resident_workgroups() {
  static int cache[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cache[dev] == 0) {
    int cus = 0, per = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
      cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_stage<R, false>, NT, 0) != hipSuccess ||
        per <= 0)
      per = 1;
    cache[dev] = cus * per;
  }
  return cache[dev];
}

template <typename R>
hipError_t launch(const G2& g, const Phys& ph, const afi::Work& w, const double* Un,
                  const double* Uk, double* Uout, const double* dt_dev, double dt_host,
                  afi::StageCoef sc, hipStream_t s, afi::Timer* tm) {
  // tiles cover cells [0, n1) and the point columns up to index n1
  const int ntx = g.n1 / TX + 1, nty = g.n2 / TY + 1;
  const int ntiles = ntx * nty;
  int nwg = resident_workgroups<R>();
  if (nwg > ntiles) nwg = ntiles;
  if (nwg >= 8) nwg -= nwg % 8;
  StageArgs sa{};
  sa.g = g;
  sa.ph = ph;
  sa.Uk = Uk;
  sa.Un = Un;
  sa.Uout = Uout;
  sa.dt_dev = dt_dev;
  sa.dt_host = dt_host;
  sa.flags = w.flags;
  sa.ntx = ntx;
  sa.ca = sc.a;
  sa.cb = sc.b;
  sa.first = sc.first;
  sa.skip_flagged = sc.skip_flagged;
  sa.blend = sc.blend;
  sa.ts_out = sc.ts_out;
  sa.ntiles = ntiles;
  if (sa.blend || sa.ts_out) {
    AFI_TIMED(tm, 7, s,
              hipLaunchKernelGGL((k_stage<R, false, true>), dim3((unsigned)nwg), dim3(NT), 0, s,
                                 sa));
  } else {
    AFI_TIMED(tm, 7, s,
              hipLaunchKernelGGL((k_stage<R, false>), dim3((unsigned)nwg), dim3(NT), 0, s, sa));
  }
  return hipGetLastError();
}

// stage k of the current attempt of the one instance whose descriptor is
// dinst (the device-resident step loop of af_run_graph): the single-instance
// kernel, with its buffers, dt and flags read from the descriptor
template <typename R>
hipError_t launch_dev(const G2& g, const Phys& ph, afi::BatchInst* dinst, double* cfl_partial,
                      int k, hipStream_t s) {
  const int ntx = g.n1 / TX + 1, nty = g.n2 / TY + 1;
  const int ntiles = ntx * nty;
  int nwg = resident_workgroups<R>();
  if (nwg > ntiles) nwg = ntiles;
  if (nwg >= 8) nwg -= nwg % 8;
  StageArgs sa{};
  sa.g = g;
  sa.ph = ph;
  sa.dinst = dinst;
  sa.cfl_partial = cfl_partial;
  sa.k = k;
  sa.ntx = ntx;
  sa.ca = k == 0 ? 0.0 : (k == 1 ? 0.75 : 1.0 / 3.0);
  sa.cb = k == 0 ? 1.0 : (k == 1 ? 0.25 : 2.0 / 3.0);
  sa.first = k == 0;
  sa.skip_flagged = 1;
  sa.ntiles = ntiles;
  hipLaunchKernelGGL((k_stage<R, false, false, true>), dim3((unsigned)nwg), dim3(NT), 0, s, sa);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_batch(afi::BatchInst* inst, int ninst, int total_tiles, const int* n_active,
                        int k, hipStream_t s, afi::Timer* tm) {
  if (ninst > kMaxBatch) return hipErrorInvalidValue;
  StageArgs sa{};
  sa.inst = inst;
  sa.ninst = ninst;
  sa.k = k;
  sa.n_active = n_active;
  sa.ca = k == 0 ? 0.0 : (k == 1 ? 0.75 : 1.0 / 3.0);
  sa.cb = k == 0 ? 1.0 : (k == 1 ? 0.25 : 2.0 / 3.0);
  sa.first = k == 0;
  sa.skip_flagged = 1;
  sa.ntiles = total_tiles;
  int nwg = resident_workgroups<R>();
  if (nwg > total_tiles) nwg = total_tiles;
  if (nwg >= 8) nwg -= nwg % 8;
  AFI_TIMED(tm, 7, s,
            hipLaunchKernelGGL((k_stage<R, true>), dim3((unsigned)nwg), dim3(NT), 0, s, sa));
  return hipGetLastError();
}

}  // namespace

namespace afi {

hipError_t AF_STAGE_ENTRY(const Geo& geo, const Phys& ph, const Work& w, const double* Un,
                          const double* Uk, double* Uout, const double* dt_dev, double dt_host,
                          StageCoef sc, hipStream_t s, Timer* tm) {
  return launch<AF_STAGE_REAL>(afi::stage_geo(geo), ph, w, Un, Uk, Uout, dt_dev, dt_host, sc, s, tm);
}

// tiles of one 2D grid for this instance's tile shape
int AF_STAGE_TILES(const Geo& geo) { return (geo.n1 / TX + 1) * (geo.n2 / TY + 1); }

// stage k of the current attempt of the single instance described at dinst
hipError_t AF_CAT(AF_STAGE_ENTRY, _dev)(const Geo& geo, const Phys& ph, BatchInst* dinst,
                                        double* cfl_partial, int k, hipStream_t s) {
  return launch_dev<AF_STAGE_REAL>(afi::stage_geo(geo), ph, dinst, cfl_partial, k, s);
}

// workgroups of a single-instance stage launch of grid geo
int AF_CAT(AF_STAGE_ENTRY, _nwg)(const Geo& geo) {
  const int ntiles = AF_STAGE_TILES(geo);
  int nwg = resident_workgroups<AF_STAGE_REAL>();
  if (nwg > ntiles) nwg = ntiles;
  if (nwg >= 8) nwg -= nwg % 8;
  return nwg;
}

// stage k of a step attempt of every active instance of a batch, one launch
hipError_t AF_STAGE_BATCH(BatchInst* inst, int ninst, int total_tiles, const int* n_active, int k,
                          hipStream_t s, Timer* tm) {
  return launch_batch<AF_STAGE_REAL>(inst, ninst, total_tiles, n_active, k, s, tm);
}

}  // namespace afi
