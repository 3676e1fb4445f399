// af_internal.hpp -- host-side structures shared by the C ABI and the kernel
// launchers (not part of the public interface).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include "af_device.hpp"

namespace afi {

// geometry of a 2D (or 1D: n2 = 1 unused) grid and its half lattice
struct Geo {
  int dim;
  int n1, n2;        // cells
  int n1x, n2y;      // point extents along x / y (n or n+1)
  int LX, LY;        // lattice extents incl. ghost margin: 2n+1+2*margin
  long ns;           // LX*LY (lattice sites)
  long off_xe, off_ye, off_co;  // 2D: offsets of the point arrays in a state
  long off_pts;                 // 1D: offset of the point array
  long state_len;    // doubles per state
  int bc[4];
  double dx, dy;
  int mixed;  // 2D: stencils in FP32, blends and updates in FP64
};

// device workspace carve-up (all device pointers)
struct Work {
  double* scal;      // [0] dt  [1] t  [2] steps taken  [3] spare
  unsigned* flags;   // sticky flag word
  unsigned long long* count;  // result of the admissibility count
  double* partial;   // CFL partial maxima [2][nb_cfl]
  int nb_cfl;
  double* LU;        // lattice conservative values  [ncomp][ns]
  double* LA;        // lattice auxiliaries          [naux][ns]
  double* LG;        // lattice gradients            [ngrad][ns]
  double* CP;        // per-cell low-order data      [ncp][ncells incl. ring]
  double* FX;        // limited x-face fluxes
  double* FY;        // limited y-face fluxes (2D)
  double* S1;        // stage buffers and checkpoint (one state each)
  double* S2;
  double* SAVE;
  size_t bytes;      // total
};

// stage coefficients of the Shu-Osher SSP-RK3 form
struct StageCoef {
  double a, b;
  int first;  // 1: Uout = FE(Uk)
  // 1: the stage belongs to a step attempt and stops as soon as the attempt's
  // flag word is set (the attempt is rejected, so its output is never used)
  int skip_flagged;
};

size_t workspace_layout(const Geo& g, Work* w, char* base);

// optional per-launch timing: begin/end bracket one kernel launch on stream s
struct Timer {
  virtual void begin(int kind, hipStream_t s) = 0;
  virtual void end(hipStream_t s) = 0;
  virtual ~Timer() {}
};

#define AFI_TIMED(tm, kind, s, launch) \
  do {                                 \
    if (tm) (tm)->begin((kind), (s));  \
    launch;                            \
    if (tm) (tm)->end(s);              \
  } while (0)

// launchers (enqueue on stream; return the first HIP error)
hipError_t stage2d_fp64(const Geo& g, const afd::Phys& ph, const Work& w, const double* Un,
                        const double* Uk, double* Uout, const double* dt_dev, double dt_host,
                        StageCoef sc, hipStream_t s, Timer* tm);
hipError_t stage2d_mixed(const Geo& g, const afd::Phys& ph, const Work& w, const double* Un,
                         const double* Uk, double* Uout, const double* dt_dev, double dt_host,
                         StageCoef sc, hipStream_t s, Timer* tm);
inline hipError_t stage2d(const Geo& g, const afd::Phys& ph, const Work& w, const double* Un,
                          const double* Uk, double* Uout, const double* dt_dev, double dt_host,
                          StageCoef sc, hipStream_t s, Timer* tm) {
  return g.mixed ? stage2d_mixed(g, ph, w, Un, Uk, Uout, dt_dev, dt_host, sc, s, tm)
                 : stage2d_fp64(g, ph, w, Un, Uk, Uout, dt_dev, dt_host, sc, s, tm);
}
hipError_t stage1d(const Geo& g, const afd::Phys& ph, const Work& w, const double* Un,
                   const double* Uk, double* Uout, const double* dt_dev, double dt_host,
                   StageCoef sc, hipStream_t s, Timer* tm);
hipError_t cfl_dt(const Geo& g, const afd::Phys& ph, double cfl_c, double cfl_v, double visc_a,
                  double visc_b, const Work& w, const double* U, double t_host,
                  const double* t_dev, double t_final, double* dt_out, hipStream_t s,
                  Timer* tm);
hipError_t advance_time(const Work& w, hipStream_t s);
hipError_t clear_flags(const Work& w, hipStream_t s);
hipError_t copy_state(double* dst, const double* src, long n, hipStream_t s);
hipError_t set_scalar(double* dst, double v, hipStream_t s);
hipError_t scale_scalar(double* dst, double f, hipStream_t s);
// number of DOF sites of state U whose density or pressure is not positive
// (NaN included), into *w.count (asynchronous)
hipError_t count_inadmissible(const Geo& g, double gm1, const Work& w, const double* U,
                              hipStream_t s);

}  // namespace afi
