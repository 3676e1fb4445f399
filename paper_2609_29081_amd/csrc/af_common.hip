// af_common.hip -- CFL time-step reduction (eq. cfl), device-side time
// bookkeeping, flag handling and the workspace layout.
#include "af_device.hpp"
#include "af_internal.hpp"

using namespace afd;

namespace {

constexpr int kBlock = 256;
constexpr int kMaxCflBlocks = 1024;

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = mx(v, __shfl_xor(v, o, 64));
  return v;
}

// block max of two values; the result is valid in thread 0
__device__ __forceinline__ void block_max2(double& a, double& b) {
  __shared__ double sa[kBlock / 64], sb[kBlock / 64];
  a = wave_max(a);
  b = wave_max(b);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    sa[wid] = a;
    sb[wid] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < kBlock / 64; ++k) {
      a = mx(a, sa[k]);
      b = mx(b, sb[k]);
    }
  }
}

// per-cell inviscid and viscous rates (eq. cfl): max_l (|u_l|+c)/(C^c dx_l)
// and rho~/(C^v min_l dx_l^2), rho~ = max(4mu/3, gamma mu/Pr)/rho
__global__ void __launch_bounds__(kBlock) k_cfl(int dim, long ncell, double gm1, double gam,
                                                double icx, double icy, double vcoef,
                                                const double* __restrict__ U,
                                                double* __restrict__ partial) {
  double a = 0.0, v = 0.0;
  for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < ncell;
       c += (long)gridDim.x * blockDim.x) {
    const double r = U[c];
    if (dim == 1) {
      const double m = U[ncell + c], E = U[2 * ncell + c];
      const double p = pressure1(r, m, E, gm1);
      const double cs = sqrt(gam * p / r);
      a = mx(a, (fabs(m / r) + cs) * icx);
    } else {
      const double m1 = U[ncell + c], m2 = U[2 * ncell + c], E = U[3 * ncell + c];
      const double p = pressure2(r, m1, m2, E, gm1);
      const double cs = sqrt(gam * p / r);
      a = mx(a, (fabs(m1 / r) + cs) * icx);
      a = mx(a, (fabs(m2 / r) + cs) * icy);
    }
    v = mx(v, vcoef / r);
  }
  block_max2(a, v);
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = a;
    partial[gridDim.x + blockIdx.x] = v;
  }
}

// final reduction: dt = 1/(a+v), clipped to t_final - t
__global__ void __launch_bounds__(kBlock) k_cfl_finish(const double* __restrict__ partial, int nb,
                                                       double t_host, const double* t_dev,
                                                       double t_final, double* dt_out) {
  double a = 0.0, v = 0.0;
  for (int k = threadIdx.x; k < nb; k += blockDim.x) {
    a = mx(a, partial[k]);
    v = mx(v, partial[nb + k]);
  }
  block_max2(a, v);
  if (threadIdx.x == 0) {
    const double t = t_dev ? *t_dev : t_host;
    double dt = 1.0 / (a + v);
    if (t + dt > t_final) dt = t_final - t;
    if (!(dt > 0.0)) dt = 0.0;
    *dt_out = dt;
  }
}

// t += dt and count the step if dt > 0 (scal[0] dt, scal[1] t, scal[2] steps)
__global__ void k_advance(double* scal) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const double dt = scal[0];
    if (dt > 0.0) {
      scal[1] = scal[1] + dt;
      scal[2] = scal[2] + 1.0;
    }
  }
}

// sites of one DOF array (len sites, component planes len apart, nc
// components) whose density or pressure is not positive
__global__ void __launch_bounds__(kBlock) k_inadmissible(int nc, const double* __restrict__ U,
                                                         long len, double gm1,
                                                         unsigned long long* count) {
  __shared__ unsigned long long part[kBlock / 64];
  unsigned long long c = 0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < len;
       i += (long)gridDim.x * blockDim.x) {
    const double r = U[i];
    double kin = 0.0;
    for (int k = 1; k < nc - 1; ++k) {
      const double m = U[k * len + i];
      kin += m * m;
    }
    const double p = gm1 * (U[(nc - 1) * len + i] - 0.5 * kin / r);
    if (!(r > 0.0) || !(p > 0.0)) ++c;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int k = 0; k < kBlock / 64; ++k) t += part[k];
    if (t) atomicAdd(count, t);
  }
}

__global__ void k_zero_count(unsigned long long* count) {
  if (threadIdx.x == 0 && blockIdx.x == 0) count[0] = 0ull;
}

__global__ void k_clear_flags(unsigned* flags) {
  if (threadIdx.x == 0 && blockIdx.x == 0) flags[0] = 0u;
}

__global__ void k_set(double* p, double v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) p[0] = v;
}

__global__ void __launch_bounds__(kBlock) k_lincomb(double* out, double a, const double* x,
                                                   double b, const double* y, long n) {
  for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < n; q += (long)gridDim.x * blockDim.x)
    out[q] = a * x[q] + b * y[q];
}

__global__ void k_scaled(double* dst, const double* src, double f) {
  if (threadIdx.x == 0 && blockIdx.x == 0) dst[0] = f * src[0];
}

__global__ void k_scale(double* p, double f) {
  if (threadIdx.x == 0 && blockIdx.x == 0) p[0] = p[0] * f;
}

__global__ void __launch_bounds__(kBlock) k_copy(double* __restrict__ d, const double* __restrict__ s,
                                                 long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    d[i] = s[i];
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// an instance may open a new step: idle, healthy, steps and time left
__device__ __forceinline__ bool may_open(const afi::BatchInst& I) {
  return !I.active && I.status == 0 && I.steps < I.max_steps && I.t < I.t_final;
}

// CFL partial maxima of instance blockIdx.y over its cell averages
__global__ void __launch_bounds__(kBlock) k_batch_cfl(afi::BatchInst* inst, double* partial) {
  const afi::BatchInst& I = inst[blockIdx.y];
  if (!may_open(I)) return;
  const double* U = I.buf[I.cur];
  const long nc = I.ncell;
  const double gm1 = I.ph.gm1, gam = I.ph.gam;
  double a = 0.0, v = 0.0;
  for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < nc;
       c += (long)gridDim.x * blockDim.x) {
    const double r = U[c];
    const double m1 = U[nc + c], m2 = U[2 * nc + c], E = U[3 * nc + c];
    const double p = pressure2(r, m1, m2, E, gm1);
    const double cs = sqrt(gam * p / r);
    a = mx(a, (fabs(m1 / r) + cs) * I.icx);
    a = mx(a, (fabs(m2 / r) + cs) * I.icy);
    v = mx(v, I.vcoef / r);
  }
  block_max2(a, v);
  if (threadIdx.x == 0) {
    double* q = partial + 2L * gridDim.x * blockIdx.y;
    q[blockIdx.x] = a;
    q[gridDim.x + blockIdx.x] = v;
  }
}

// number of active instances, into *n_active (one block)
__device__ void count_active(afi::BatchInst* inst, int n, int* n_active) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  int c = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) c += inst[i].active;
  if (c) atomicAdd(&cnt, c);
  __syncthreads();
  if (threadIdx.x == 0) n_active[0] = cnt;
}

// open a step for instance i if it may: dt = 1/(a + v) (eq. cfl) from its
// nb pairs of partial maxima, clipped to t_final - t (one thread)
__device__ void open_one(afi::BatchInst& I, double a, double v) {
  double dt = 1.0 / (a + v);
  if (I.t + dt > I.t_final) dt = I.t_final - I.t;
  if (!(dt > 0.0)) {
    I.status = 4;  // AF_E_NONFINITE: no finite time step from this state
    return;
  }
  I.dt = dt;
  I.halvings = 0;
  I.flags = 0u;
  I.active = 1;
}

// open a step for every instance that may.  Many instances: one thread per
// instance over its nb partials; one instance: the whole block reduces its
// partials (a single instance takes many CFL blocks)
__global__ void __launch_bounds__(kBlock) k_batch_open(afi::BatchInst* inst, int n,
                                                       const double* partial, int nb,
                                                       int* n_active) {
  if (n == 1) {
    afi::BatchInst& I = inst[0];
    if (may_open(I)) {
      double a = 0.0, v = 0.0;
      const int nr = I.cfl_nb > 0 ? I.cfl_nb : nb;  // maxima from the last stage, or all
      for (int k = threadIdx.x; k < nr; k += blockDim.x) {
        a = mx(a, partial[k]);
        v = mx(v, partial[nb + k]);
      }
      block_max2(a, v);
      if (threadIdx.x == 0) open_one(I, a, v);
    }
  } else {
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      afi::BatchInst& I = inst[i];
      if (!may_open(I)) continue;
      const double* q = partial + 2L * nb * i;
      double a = 0.0, v = 0.0;
      for (int k = 0; k < nb; ++k) {
        a = mx(a, q[k]);
        v = mx(v, q[nb + k]);
      }
      open_one(I, a, v);
    }
  }
  __syncthreads();
  count_active(inst, n, n_active);
}

// after an attempt: accept it (the output becomes the current state) or
// redo it with dt/2, up to max_halvings times (then the instance stops with
// its status set and its state left at the start of the step)
__global__ void __launch_bounds__(kBlock) k_batch_decide(afi::BatchInst* inst, int n,
                                                         int* n_active) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    afi::BatchInst& I = inst[i];
    if (!I.active) continue;
    I.attempts += 1;
    const unsigned f = I.flags;
    if (f == 0u) {
      I.t += I.dt;
      I.steps += 1;
      I.cur = (I.cur + 1) % 3;
      I.active = 0;
      // the accepted last stage left the new state's CFL maxima
      if (I.stage_nwg > 0) I.cfl_nb = I.stage_nwg;
    } else if (I.halvings < I.max_halvings) {
      I.dt *= 0.5;
      I.halvings += 1;
      I.flags = 0u;
    } else {
      I.status = (f & FLAG_NONFINITE) ? 4 : 3;  // AF_E_NONFINITE : AF_E_PP
      I.active = 0;
    }
  }
  __syncthreads();
  count_active(inst, n, n_active);
}

}  // namespace

namespace afi {

// carve the workspace; with base == nullptr only the size is computed
size_t workspace_layout(const Geo& g, Work* w, char* base) {
  const int nc = g.dim == 1 ? 3 : 4;
  const int naux = g.dim == 1 ? 4 : 5;
  const int ngrad = g.dim == 1 ? 2 : 6;
  const int ncp = g.dim == 1 ? 10 : 18;
  const long ncells_ring = g.dim == 1 ? (long)(g.n1 + 2) : (long)(g.n1 + 2) * (g.n2 + 2);
  const long nfx = g.dim == 1 ? (long)(g.n1 + 1) : (long)(g.n1 + 1) * g.n2;
  const long nfy = g.dim == 1 ? 0 : (long)g.n1 * (g.n2 + 1);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align256(bytes);
    return base ? base + o : nullptr;
  };
  Work r{};
  r.scal = (double*)take(4 * sizeof(double));
  r.flags = (unsigned*)take(sizeof(unsigned) * 4);
  r.count = (unsigned long long*)take(sizeof(unsigned long long));
  r.nb_cfl = kMaxCflBlocks;
  r.partial = (double*)take(2 * sizeof(double) * kMaxCflBlocks);
  if (g.dim == 1) {
    // the 1D stage passes its lattice, gradient, cell and face data through
    // device memory; the 2D stage keeps them in LDS
    r.LU = (double*)take(sizeof(double) * nc * g.ns);
    r.LA = (double*)take(sizeof(double) * naux * g.ns);
    r.LG = (double*)take(sizeof(double) * ngrad * g.ns);
    r.CP = (double*)take(sizeof(double) * ncp * ncells_ring);
    r.FX = (double*)take(sizeof(double) * nc * nfx);
    r.FY = (double*)take(sizeof(double) * nc * (nfy > 0 ? nfy : 1));
  }
  r.S1 = (double*)take(sizeof(double) * g.state_len);
  r.S2 = (double*)take(sizeof(double) * g.state_len);
  r.S3 = (double*)take(sizeof(double) * g.state_len);
  r.SAVE = (double*)take(sizeof(double) * g.state_len);
  if (g.dim == 2) {
    r.blend = (float*)take(sizeof(float) * (nfx + nfy));
    r.mlp = (void*)take(kMlpPackedBytes);
    r.binst = (BatchInst*)take(sizeof(BatchInst));
    r.bpartial = (double*)take(2 * sizeof(double) * kSingleCflBlocks);
    r.bnact = (int*)take(sizeof(int));
  }
  r.bytes = off;
  if (w) *w = r;
  return off;
}

hipError_t cfl_dt(const Geo& g, const Phys& ph, double cfl_c, double cfl_v, double visc_a,
                  double visc_b, const Work& w, const double* U, double t_host,
                  const double* t_dev, double t_final, double* dt_out, hipStream_t s,
                  Timer* tm) {
  const long ncell = g.dim == 1 ? (long)g.n1 : (long)g.n1 * g.n2;
  long nb = (ncell + kBlock - 1) / kBlock;
  if (nb > w.nb_cfl) nb = w.nb_cfl;
  if (nb < 1) nb = 1;
  const double hmin = g.dim == 1 ? g.dx : fmin(g.dx, g.dy);
  const double vcoef = fmax(visc_a, visc_b) / (cfl_v * hmin * hmin);
  const double icx = 1.0 / (cfl_c * g.dx);
  const double icy = g.dim == 1 ? 0.0 : 1.0 / (cfl_c * g.dy);
  AFI_TIMED(tm, 6, s,
            hipLaunchKernelGGL(k_cfl, dim3((unsigned)nb), dim3(kBlock), 0, s, g.dim, ncell, ph.gm1,
                               ph.gam, icx, icy, vcoef, U, w.partial));
  AFI_TIMED(tm, 6, s,
            hipLaunchKernelGGL(k_cfl_finish, dim3(1), dim3(kBlock), 0, s,
                               (const double*)w.partial, (int)nb, t_host, t_dev, t_final, dt_out));
  return hipGetLastError();
}

hipError_t advance_time(const Work& w, hipStream_t s) {
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, s, w.scal);
  return hipGetLastError();
}

hipError_t clear_flags(const Work& w, hipStream_t s) {
  hipLaunchKernelGGL(k_clear_flags, dim3(1), dim3(64), 0, s, w.flags);
  return hipGetLastError();
}

hipError_t set_scalar(double* dst, double v, hipStream_t s) {
  hipLaunchKernelGGL(k_set, dim3(1), dim3(64), 0, s, dst, v);
  return hipGetLastError();
}

hipError_t scale_scalar(double* dst, double f, hipStream_t s) {
  hipLaunchKernelGGL(k_scale, dim3(1), dim3(64), 0, s, dst, f);
  return hipGetLastError();
}

hipError_t count_inadmissible(const Geo& g, double gm1, const Work& w, const double* U,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_zero_count, dim3(1), dim3(64), 0, s, w.count);
  const int nc = g.dim == 1 ? 3 : 4;
  long off[4], len[4];
  int na;
  if (g.dim == 1) {
    na = 2;
    off[0] = 0;
    len[0] = g.n1;
    off[1] = g.off_pts;
    len[1] = g.n1x;
  } else {
    na = 4;
    off[0] = 0;
    len[0] = (long)g.n1 * g.n2;
    off[1] = g.off_xe;
    len[1] = (long)g.n2 * g.n1x;
    off[2] = g.off_ye;
    len[2] = (long)g.n2y * g.n1;
    off[3] = g.off_co;
    len[3] = (long)g.n2y * g.n1x;
  }
  for (int a = 0; a < na; ++a) {
    long nb = (len[a] + kBlock - 1) / kBlock;
    if (nb > 2048) nb = 2048;
    hipLaunchKernelGGL(k_inadmissible, dim3((unsigned)nb), dim3(kBlock), 0, s, nc, U + off[a],
                       len[a], gm1, w.count);
  }
  return hipGetLastError();
}

hipError_t batch_cfl(BatchInst* inst, int n, double* partial, int nb, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_cfl, dim3((unsigned)nb, (unsigned)n), dim3(kBlock), 0, s, inst,
                     partial);
  return hipGetLastError();
}

hipError_t batch_open(BatchInst* inst, int n, const double* partial, int nb, int* n_active,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_batch_open, dim3(1), dim3(kBlock), 0, s, inst, n, partial, nb, n_active);
  return hipGetLastError();
}

hipError_t batch_decide(BatchInst* inst, int n, int* n_active, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_decide, dim3(1), dim3(kBlock), 0, s, inst, n, n_active);
  return hipGetLastError();
}

hipError_t lincomb(double* out, double a, const double* x, double b, const double* y, long n,
                   hipStream_t s) {
  long nb = (n + kBlock - 1) / kBlock;
  if (nb > 4096) nb = 4096;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(k_lincomb, dim3((unsigned)nb), dim3(kBlock), 0, s, out, a, x, b, y, n);
  return hipGetLastError();
}

hipError_t scaled_scalar(double* dst, const double* src, double f, hipStream_t s) {
  hipLaunchKernelGGL(k_scaled, dim3(1), dim3(64), 0, s, dst, src, f);
  return hipGetLastError();
}

hipError_t copy_state(double* dst, const double* src, long n, hipStream_t s) {
  long nb = (n + kBlock - 1) / kBlock;
  if (nb > 4096) nb = 4096;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)nb), dim3(kBlock), 0, s, dst, src, n);
  return hipGetLastError();
}

}  // namespace afi
