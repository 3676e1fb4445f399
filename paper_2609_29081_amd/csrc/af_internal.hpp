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
  double bcstate[2][3];  // 1D Dirichlet states of the x-low and x-high sides
};

// geometry of a 2D grid as the stage kernels read it
struct StageGeo {
  int n1, n2, n1x, n2y;
  long off_xe, off_ye, off_co;
  int bc0, bc1, bc2, bc3;
  double dx, dy;
};

inline StageGeo stage_geo(const Geo& g) {
  StageGeo r;
  r.n1 = g.n1;
  r.n2 = g.n2;
  r.n1x = g.n1x;
  r.n2y = g.n2y;
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

// One 2D instance of a batch, in device memory.  The host fills the static
// part; the batch kernels update the rest.  A step of an instance is a
// sequence of attempts: the CFL kernel opens it (active = 1, fresh dt), each
// attempt runs the three stages from buf[cur], and the decide kernel either
// accepts it (cur advances, t += dt) or halves dt for the next attempt.
struct BatchInst {
  StageGeo g;
  afd::Phys ph;
  double* buf[3];        // rotating states; buf[cur] is the current one
  int ntx, ntiles;       // stage tiles along x and in all
  long ncell;            // CFL: cells, 1/(C^c dx), 1/(C^c dy), viscous rate factor
  double icx, icy, vcoef;
  double t_final;
  long max_steps;
  int max_halvings;
  // a single instance whose last stage leaves the CFL maxima of the new
  // state (af_run_graph): the number of its stage workgroups, else 0
  int stage_nwg;
  // updated on the device
  double dt, t;
  long steps;
  int cur, active, halvings, status;
  unsigned flags;
  long attempts;  // RK3 attempts so far (accepted and rejected)
  // partial CFL maxima the next step opens from: 0 for the CFL kernel's own
  // count, else the number written by the last accepted stage
  int cfl_nb;
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
  double* S3;        // fourth stage buffer of SSP-RK54
  double* SAVE;
  // 2D learned blend: one coefficient per face, and the network's weights as
  // the inference kernel reads them (bfloat16 W1, W2, w3; FP32 biases)
  float* blend;
  void* mlp;
  // 2D: one batch descriptor, its CFL partial maxima and active count, for
  // the single instance's device-resident step loop (af_run_graph)
  struct BatchInst* binst;
  double* bpartial;
  int* bnact;
  // host-side: the context's learned-blend network (device parameters), or NULL
  const float* net;
  size_t bytes;      // total
};

// stage coefficients of the Shu-Osher SSP-RK3 form
struct StageCoef {
  double a, b;
  int first;  // 1: Uout = FE(Uk)
  // 1: the stage belongs to a step attempt and stops as soon as the attempt's
  // flag word is set (the attempt is rejected, so its output is never used)
  int skip_flagged;
  // 2D only: a blend coefficient per face that takes the place of theta^s
  // (the density/pressure limiter then clamps it as it clamps theta^s), or
  // NULL; and an array that receives the coefficient used in theta^s's
  // place per face, or NULL
  const float* blend;
  float* ts_out;
  // the forward-Euler step is dt_mul * dt (the stages of SSP-RK54)
  double dt_mul = 1.0;
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

// the learned blend (af_learn.hip)
constexpr int kMlpIn = 40, kMlpHidden = 64;
constexpr long kMlpParams = (long)kMlpHidden * kMlpIn + kMlpHidden + (long)kMlpHidden * kMlpHidden +
                            kMlpHidden + kMlpHidden + 1;
constexpr size_t kMlpPackedBytes = 14336;
hipError_t blend_features(const Geo& g, const afd::Phys& ph, const double* U, float* feat,
                          hipStream_t s);
hipError_t mlp_pack(const float* params, void* packed, hipStream_t s);
hipError_t blend_infer(const Geo& g, const afd::Phys& ph, const double* U, const void* packed,
                       float* theta, hipStream_t s, Timer* tm);
size_t mlp_grad_workspace(long n);
hipError_t mlp_grad(const float* X, const float* y, long n, const float* params, float* grad,
                    float* loss, void* ws, hipStream_t s);
hipError_t mlp_adam(float* params, const float* grad, float* m, float* v, long step, float lr,
                    hipStream_t s);

// launchers (enqueue on stream; return the first HIP error)
// the 2D stage of one instance, with its precision's default variant
hipError_t stage2d(const Geo& g, const afd::Phys& ph, const Work& w, const double* Un,
                   const double* Uk, double* Uout, const double* dt_dev, double dt_host,
                   StageCoef sc, hipStream_t s, Timer* tm);
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
// out = a x + b y over n values (out may be x or y)
hipError_t lincomb(double* out, double a, const double* x, double b, const double* y, long n,
                   hipStream_t s);
// *dst = f * *src (device scalars)
hipError_t scaled_scalar(double* dst, const double* src, double f, hipStream_t s);
hipError_t set_scalar(double* dst, double v, hipStream_t s);
hipError_t scale_scalar(double* dst, double f, hipStream_t s);
// number of DOF sites of state U whose density or pressure is not positive
// (NaN included), into *w.count (asynchronous)
hipError_t count_inadmissible(const Geo& g, double gm1, const Work& w, const double* U,
                              hipStream_t s);

// batch kernels (af_common.hip): CFL partial maxima of every instance that
// may open a step (B blocks each); opening of steps (fresh CFL dt, active);
// the decision after an attempt.  Both of the latter recount the active
// instances into *n_active.
// nb CFL blocks per instance: kBatchCflBlocks in a batch, kSingleCflBlocks
// for the single instance of af_run_graph
constexpr int kBatchCflBlocks = 32;
constexpr int kSingleCflBlocks = 1024;
hipError_t batch_cfl(BatchInst* inst, int n, double* partial, int nb, hipStream_t s);
hipError_t batch_open(BatchInst* inst, int n, const double* partial, int nb, int* n_active,
                      hipStream_t s);
hipError_t batch_decide(BatchInst* inst, int n, int* n_active, hipStream_t s);
// Compiled variants of the 2D stage (af_stage2d.hip, one object each): the
// single-instance stage, the batch stage and the tile count of a grid.
struct StageVariant {
  const char* name;
  int mixed;  // 1: FP32 stencils
  int ty;     // tile height (cells)
  hipError_t (*single)(const Geo&, const afd::Phys&, const Work&, const double*, const double*,
                       double*, const double*, double, StageCoef, hipStream_t, Timer*);
  hipError_t (*batch)(BatchInst*, int, int, const int*, int, hipStream_t, Timer*);
  int (*tiles)(const Geo&);
  // stage k of the current attempt of one instance whose step machinery is on
  // the device (descriptor dinst): the single-instance kernel; its last stage
  // writes the CFL maxima of the new state per workgroup into cfl_partial
  // (stride kSingleCflBlocks); dev_nwg: its number of workgroups
  hipError_t (*dev)(const Geo&, const afd::Phys&, BatchInst*, double* cfl_partial, int,
                    hipStream_t);
  int (*dev_nwg)(const Geo&);
};
// all variants; the first of each precision is its default
extern const StageVariant kStageVariants[];
extern const int kNumStageVariants;
const StageVariant* default_variant(int mixed);

}  // namespace afi
