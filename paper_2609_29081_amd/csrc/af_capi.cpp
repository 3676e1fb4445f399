// af_capi.cpp -- the C ABI declared in include/af.h: parameter validation,
// grid/lattice geometry, workspace carve-up, SSP-RK3 stage sequencing, the
// CFL step, step halving (Remark on the time step, Sec. 3.4) and the
// device-resident run loop.
#include "../../include/af.h"

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include <string.h>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "af_device.hpp"
#include "af_internal.hpp"

// workspace of af_step_noalloc: one copy per GPU, resident for the life of
// the process.  Host code never uses this name as an address (on the host it
// is only a stand-in for the device symbol): the device address comes from
// hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[AF_NOALLOC_SCRATCH_BYTES];

namespace {

// per-launch HIP event pairs, reduced to per-kind sums on read
struct EventTimer : afi::Timer {
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
  std::vector<int> kinds;  // kind of pool entry i (for the first n entries)
  size_t n = 0;
  int open_kind = -1;
  hipError_t err = hipSuccess;

  void begin(int kind, hipStream_t s) override {
    if (n == pool.size()) {
      hipEvent_t a, b;
      if ((err = hipEventCreate(&a)) != hipSuccess) return;
      if ((err = hipEventCreate(&b)) != hipSuccess) return;
      pool.emplace_back(a, b);
      kinds.push_back(kind);
    }
    kinds[n] = kind;
    open_kind = kind;
    hipError_t e = hipEventRecord(pool[n].first, s);
    if (e != hipSuccess) err = e;
  }
  void end(hipStream_t s) override {
    if (open_kind < 0 || n >= pool.size()) return;
    hipError_t e = hipEventRecord(pool[n].second, s);
    if (e != hipSuccess) err = e;
    ++n;
    open_kind = -1;
  }
  ~EventTimer() override {
    for (auto& pr : pool) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
  }
};

}  // namespace

struct af_ctx {
  af_params p;
  int bc[4];
  EventTimer* timer = nullptr;
  // af_run_graph's executable graph, reused while its workspace and slot
  // length stay the same (the stages read everything else from the device
  // descriptor)
  hipGraphExec_t run_exec = nullptr;
  const void* run_ws = nullptr;
  int run_slot = 0, run_dev = -1;
  const float* net = nullptr;  // learned-blend network parameters (device), or NULL
  double bcstate[2][3] = {{1.0, 0.0, 1.0}, {1.0, 0.0, 1.0}};  // 1D Dirichlet states
};

struct af_batch {
  std::vector<af_ctx*> ctx;
  std::vector<afi::Geo> geo;
  int mixed = 0;
  const afi::StageVariant* var = nullptr;  // stage variant (tile shape) of the batch
  // workspace: descriptors, CFL partials, active count, then two stage
  // buffers per instance
  size_t off_partial = 0, off_nact = 0, bytes = 0;
  std::vector<size_t> off_bufs;
};

namespace {

thread_local std::string g_err;

af_status fail(af_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

af_status hip_fail(hipError_t e, const char* where) {
  return fail(AF_E_HIP, "%s: %s", where, hipGetErrorString(e));
}

#define AF_HIP(call)                                   \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return hip_fail(e_, #call);  \
  } while (0)

bool geometry(const af_ctx* c, afi::Geo* g);

// a context under AF_LIM_LEARNED needs its network
bool net_ready(const af_ctx* c) {
  if ((c->p.limiter & AF_LIM_LEARNED) && !c->net) {
    fail(AF_E_ARG, "AF_LIM_LEARNED: no network set (af_set_blend_net)");
    return false;
  }
  return true;
}

// the workspace carve-up of a context, with its network pointer
afi::Work work_of(const af_ctx* c, const afi::Geo& g, const void* ws) {
  afi::Work w;
  afi::workspace_layout(g, &w, (char*)const_cast<void*>(ws));
  w.net = c->net;
  return w;
}

bool geometry(const af_ctx* c, afi::Geo* g) {
  const af_params& p = c->p;
  if ((c->bc[0] == AF_PERIODIC) != (c->bc[1] == AF_PERIODIC)) {
    fail(AF_E_ARG, "x axis: periodic must be set on both sides");
    return false;
  }
  if (p.dim == 2 && (c->bc[2] == AF_PERIODIC) != (c->bc[3] == AF_PERIODIC)) {
    fail(AF_E_ARG, "y axis: periodic must be set on both sides");
    return false;
  }
  afi::Geo r{};
  r.dim = p.dim;
  r.n1 = p.n1;
  r.n2 = p.dim == 2 ? p.n2 : 1;
  r.n1x = c->bc[0] == AF_PERIODIC ? p.n1 : p.n1 + 1;
  r.n2y = p.dim == 2 ? (c->bc[2] == AF_PERIODIC ? p.n2 : p.n2 + 1) : 1;
  r.LX = 2 * p.n1 + 1 + 2 * afd::kMargin;
  r.LY = p.dim == 2 ? 2 * p.n2 + 1 + 2 * afd::kMargin : 1;
  r.ns = (long)r.LX * r.LY;
  for (int k = 0; k < 4; ++k) r.bc[k] = c->bc[k];
  r.dx = (p.x1 - p.x0) / p.n1;
  r.dy = p.dim == 2 ? (p.y1 - p.y0) / p.n2 : 1.0;
  r.mixed = p.precision == AF_PREC_MIXED;
  for (int s = 0; s < 2; ++s)
    for (int k = 0; k < 3; ++k) r.bcstate[s][k] = c->bcstate[s][k];
  if (p.dim == 1) {
    r.off_pts = 3L * p.n1;
    r.state_len = 3L * (p.n1 + r.n1x);
  } else {
    const long n1 = p.n1, n2 = p.n2;
    r.off_xe = 4 * n1 * n2;
    r.off_ye = r.off_xe + 4 * n2 * r.n1x;
    r.off_co = r.off_ye + 4L * r.n2y * n1;
    r.state_len = r.off_co + 4L * r.n2y * r.n1x;
  }
  *g = r;
  return true;
}

afd::Phys physics(const af_params& p) {
  afd::Phys ph;
  ph.gam = p.gamma;
  ph.gm1 = p.gamma - 1.0;
  ph.mu = p.mu;
  ph.kap = p.gamma * p.mu / ((p.gamma - 1.0) * p.Pr);
  ph.Cs = p.Cs;
  ph.igm1 = 1.0 / (p.gamma - 1.0);
  ph.lim = p.limiter;
  return ph;
}

const afi::StageCoef kCoef[3] = {{0.0, 1.0, 1, 0}, {0.75, 0.25, 0, 0}, {1.0 / 3.0, 2.0 / 3.0, 0, 0}};

// in_step: the stage is part of a step attempt (af_step, af_run), whose
// output is discarded once a flag is raised, so it may stop early
// one stage with coefficients sc: Uout = sc.a Un + sc.b FE(Uk, sc.dt_mul dt)
hipError_t launch_coef(const afi::Geo& g, const afd::Phys& ph, const afi::Work& w,
                       afi::StageCoef sc, const double* Un, const double* Uk, double* Uout,
                       const double* dt_dev, double dt_host, hipStream_t s, afi::Timer* tm) {
  if (!Un) Un = Uk;
  if (sc.dt_mul != 1.0) {
    // the stage's step as its own device scalar (the spare workspace slot)
    if (dt_dev) {
      hipError_t e = afi::scaled_scalar(w.scal + 3, dt_dev, sc.dt_mul, s);
      if (e != hipSuccess) return e;
      dt_dev = w.scal + 3;
    } else {
      dt_host *= sc.dt_mul;
    }
  }
  if (g.dim == 2 && (ph.lim & afd::LIM_LEARNED)) {
    // the network's blend from this stage's input, then the stage
    if (!w.net) return hipErrorInvalidValue;
    hipError_t e;
    if ((e = afi::mlp_pack(w.net, w.mlp, s)) != hipSuccess) return e;
    if ((e = afi::blend_infer(g, ph, Uk, w.mlp, w.blend, s, tm)) != hipSuccess) return e;
    sc.blend = w.blend;
  }
  return g.dim == 1 ? afi::stage1d(g, ph, w, Un, Uk, Uout, dt_dev, dt_host, sc, s, tm)
                    : afi::stage2d(g, ph, w, Un, Uk, Uout, dt_dev, dt_host, sc, s, tm);
}

hipError_t launch_stage(const afi::Geo& g, const afd::Phys& ph, const afi::Work& w, int k,
                        const double* Un, const double* Uk, double* Uout, const double* dt_dev,
                        double dt_host, hipStream_t s, afi::Timer* tm, bool in_step = true) {
  afi::StageCoef sc = kCoef[k];
  sc.skip_flagged = in_step ? 1 : 0;
  return launch_coef(g, ph, w, sc, Un, Uk, Uout, dt_dev, dt_host, s, tm);
}

// a stage output plus its share of a source term: out += f S (S may be NULL)
hipError_t add_source(const afi::Geo& g, double* out, double f, const double* S, hipStream_t s) {
  return S ? afi::lincomb(out, 1.0, out, f, S, g.state_len, s) : hipSuccess;
}

// SSP-RK54 (Sec. 2.3 names the five-stage, fourth-order SSP method; these
// are Spiteri and Ruuth's SSPRK(5,4) coefficients in Shu-Osher form).  With
// E_k = FE(u_k, c_k dt): u1 = E0, u2 = a20 u0 + a21 E1, u3 = a30 u0 + a32 E2,
// u4 = a40 u0 + a43 E3, u5 = a52 u2 + a53 E3 + a54 E4, where c_3 = b43/a43
// = b53/a53 makes E3 one evaluation shared by u4 and u5.
constexpr double kA20 = 0.444370493651235, kA21 = 0.555629506348765;
constexpr double kA30 = 0.620101851488403, kA32 = 0.379898148511597;
constexpr double kA40 = 0.178079954393132, kA43 = 0.821920045606868;
constexpr double kA52 = 0.517231671970585, kA53 = 0.096059710526147;
constexpr double kA54 = 0.386708617503269;
constexpr double kB10 = 0.391752226571890, kB21 = 0.368410593050371;
constexpr double kB32 = 0.251891774271694, kB43 = 0.544974750228521;
constexpr double kB54 = 0.226007483236906;

// one SSP-RK54 attempt from u0 (kept) through buffers A, B into X; src as
// for rk3 (five stage inputs)
hipError_t rk54(const afi::Geo& g, const afd::Phys& ph, const afi::Work& w, const double* u0,
                double* A, double* B, double* X, const double* dt_dev, double dt, hipStream_t s,
                afi::Timer* tm, const double* const* src = nullptr) {
  auto coef = [](double a, double b, double mul) {
    afi::StageCoef c{};
    c.a = a;
    c.b = b;
    c.first = a == 0.0 ? 1 : 0;
    c.skip_flagged = 1;
    c.dt_mul = mul;
    return c;
  };
  const long n = g.state_len;
  hipError_t e;
  auto S = [&](int k) { return src ? src[k] : nullptr; };
  if ((e = launch_coef(g, ph, w, coef(0.0, 1.0, kB10), u0, u0, A, dt_dev, dt, s, tm)) != hipSuccess)
    return e;  // A = u1
  if ((e = add_source(g, A, kB10 * dt, S(0), s)) != hipSuccess) return e;
  if ((e = launch_coef(g, ph, w, coef(kA20, kA21, kB21 / kA21), u0, A, B, dt_dev, dt, s, tm)) !=
      hipSuccess)
    return e;  // B = u2
  if ((e = add_source(g, B, kB21 * dt, S(1), s)) != hipSuccess) return e;
  if ((e = launch_coef(g, ph, w, coef(kA30, kA32, kB32 / kA32), u0, B, A, dt_dev, dt, s, tm)) !=
      hipSuccess)
    return e;  // A = u3
  if ((e = add_source(g, A, kB32 * dt, S(2), s)) != hipSuccess) return e;
  if ((e = launch_coef(g, ph, w, coef(0.0, 1.0, kB43 / kA43), u0, A, X, dt_dev, dt, s, tm)) !=
      hipSuccess)
    return e;  // X = E3
  if ((e = add_source(g, X, kB43 / kA43 * dt, S(3), s)) != hipSuccess) return e;
  if ((e = afi::lincomb(A, kA40, u0, kA43, X, n, s)) != hipSuccess) return e;   // A = u4
  if ((e = afi::lincomb(B, kA52, B, kA53, X, n, s)) != hipSuccess) return e;    // B = a52 u2 + a53 E3
  if ((e = launch_coef(g, ph, w, coef(1.0, kA54, kB54 / kA54), B, A, X, dt_dev, dt, s, tm)) !=
      hipSuccess)
    return e;
  return add_source(g, X, kB54 * dt, S(4), s);
}

hipError_t launch_cfl(const af_ctx* c, const afi::Geo& g, const afi::Work& w, const double* U,
                      double t_host, const double* t_dev, double t_final, double* dt_out,
                      hipStream_t s) {
  const af_params& p = c->p;
  return afi::cfl_dt(g, physics(p), p.cfl_c, p.cfl_v, 4.0 * p.mu / 3.0, p.gamma * p.mu / p.Pr, w,
                     U, t_host, t_dev, t_final, dt_out, s, c->timer);
}

af_status read_flags(const afi::Work& w, hipStream_t s, unsigned* out) {
  AF_HIP(hipMemcpyAsync(out, w.flags, sizeof(unsigned), hipMemcpyDeviceToHost, s));
  AF_HIP(hipStreamSynchronize(s));
  return AF_OK;
}

// device address of the scratch array on the current device, looked up once
// per device (each GPU holds its own copy at its own address)
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

af_status scratch_on_current_device(void** out) {
  int dev = 0;
  AF_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(AF_E_ARG, "device %d: too many devices", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    AF_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(AF_E_HIP, "hipGetSymbolAddress: NULL address of the scratch array");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return AF_OK;
}

// three stages with a host-given dt; cur -> out through S1, S2.  src, if not
// NULL, holds a source term at each stage input's time (host dt only): each
// forward Euler step then adds tau S_k after its limited update
hipError_t rk3(const afi::Geo& g, const afd::Phys& ph, const afi::Work& w, const double* cur,
               double* out, const double* dt_dev, double dt, hipStream_t s, afi::Timer* tm,
               const double* const* src = nullptr) {
  hipError_t e;
  if ((e = launch_stage(g, ph, w, 0, cur, cur, w.S1, dt_dev, dt, s, tm)) != hipSuccess) return e;
  if (src && (e = add_source(g, w.S1, dt, src[0], s)) != hipSuccess) return e;
  if ((e = launch_stage(g, ph, w, 1, cur, w.S1, w.S2, dt_dev, dt, s, tm)) != hipSuccess) return e;
  if (src && (e = add_source(g, w.S2, 0.25 * dt, src[1], s)) != hipSuccess) return e;
  if ((e = launch_stage(g, ph, w, 2, cur, w.S2, out, dt_dev, dt, s, tm)) != hipSuccess) return e;
  if (src && (e = add_source(g, out, 2.0 / 3.0 * dt, src[2], s)) != hipSuccess) return e;
  return hipSuccess;
}

// the static part of one instance's batch descriptor: context c with grid
// g, stage variant v, rotating state buffers b0 (the caller's state), b1,
// b2, times t0..t_final and at most max_steps steps
afi::BatchInst instance_of(const af_ctx* c, const afi::Geo& g, const afi::StageVariant* v,
                           double* b0, double* b1, double* b2, double t0, double t_final,
                           long max_steps) {
  const af_params& p = c->p;
  afi::BatchInst I;
  memset(&I, 0, sizeof(I));
  I.g = afi::stage_geo(g);
  I.ph = physics(p);
  I.buf[0] = b0;
  I.buf[1] = b1;
  I.buf[2] = b2;
  I.ntx = g.n1 / 16 + 1;
  I.ntiles = v->tiles(g);
  I.ncell = (long)g.n1 * g.n2;
  I.icx = 1.0 / (p.cfl_c * g.dx);
  I.icy = 1.0 / (p.cfl_c * g.dy);
  const double hmin = fmin(g.dx, g.dy);
  I.vcoef = fmax(4.0 * p.mu / 3.0, p.gamma * p.mu / p.Pr) / (p.cfl_v * hmin * hmin);
  I.t_final = t_final;
  I.max_steps = max_steps;
  I.max_halvings = p.max_halvings;
  I.t = t0;
  return I;
}

// host copies of the batch descriptors for states U, times t0..t_final and
// the tile shape of stage variant v; *total_tiles receives the tiles of all
// instances (a stage launch has at most that many)
af_status batch_descriptors(const af_batch* b, const afi::StageVariant* v, double* const* U,
                            char* base, double t0, double t_final, long max_steps,
                            std::vector<afi::BatchInst>& h, int* total_tiles) {
  const int n = (int)b->ctx.size();
  h.assign(n, afi::BatchInst{});
  int total = 0;
  for (int i = 0; i < n; ++i) {
    if (!U[i]) return fail(AF_E_ARG, "batch: state %d is NULL", i);
    h[i] = instance_of(b->ctx[i], b->geo[i], v, U[i], (double*)(base + b->off_bufs[2 * i]),
                       (double*)(base + b->off_bufs[2 * i + 1]), t0, t_final, max_steps);
    total += h[i].ntiles;
  }
  *total_tiles = total;
  return AF_OK;
}

// one slot of a batch: `rounds` rounds, each of which opens a step (fresh
// CFL dt) for every instance that is between steps and then runs one RK3
// attempt of every instance inside a step (three stage launches of variant
// v, then the accept/halve decision).  An instance that accepts a step opens
// the next one in the following round, while others redo theirs with dt/2.
hipError_t batch_slot(const afi::StageVariant* v, afi::BatchInst* dinst, int n, int total_tiles,
                      double* partial, int* nact, int rounds, hipStream_t q) {
  hipError_t e;
  const int nb = n == 1 ? afi::kSingleCflBlocks : afi::kBatchCflBlocks;
  for (int a = 0; a < rounds; ++a) {
    if ((e = afi::batch_cfl(dinst, n, partial, nb, q)) != hipSuccess) return e;
    if ((e = afi::batch_open(dinst, n, partial, nb, nact, q)) != hipSuccess) return e;
    for (int k = 0; k < 3; ++k)
      if ((e = v->batch(dinst, n, total_tiles, nact, k, q, nullptr)) != hipSuccess) return e;
    if ((e = afi::batch_decide(dinst, n, nact, q)) != hipSuccess) return e;
  }
  return hipSuccess;
}

// Enqueue step slots (slot(stream) enqueues one) for the n instances whose
// descriptors (host copies h, already on the device at dinst) are set, on
// stream s: captured once in a HIP graph (use_graph) or launched directly,
// in chunks of `chunk` slots with a read-back of the descriptors after each; stops
// once no instance is active or may open a step.  h receives the final
// descriptors.
// keep (cache != NULL): the instantiated graph is taken from *cache if set
// there, else built and left in *cache for the caller to reuse and destroy.
template <typename Slot>
af_status run_slots(Slot slot, afi::BatchInst* dinst, int n, int use_graph, hipStream_t s,
                    long max_steps, double t_final, std::vector<afi::BatchInst>& h,
                    const char* who, hipGraphExec_t* cache = nullptr, long chunk = 8) {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = cache ? *cache : nullptr;
  if (use_graph && !exec) {
    // the slot is captured on a private stream (the caller's may be the null
    // stream, which cannot be captured) and replayed on the caller's
    hipStream_t cs = nullptr;
    AF_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
    if (e == hipSuccess) e = slot(cs);
    hipGraph_t gcap = nullptr;
    const hipError_t e2 = hipStreamEndCapture(cs, &gcap);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (gcap) (void)hipGraphDestroy(gcap);
      return fail(AF_E_HIP, "%s: graph capture: %s", who,
                  hipGetErrorString(e != hipSuccess ? e : e2));
    }
    graph = gcap;
    if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return fail(AF_E_HIP, "%s: graph instantiation failed", who);
    }
    (void)hipGraphDestroy(graph);  // the executable graph keeps what it needs
    graph = nullptr;
    if (cache) *cache = exec;
  }
  af_status st = AF_OK;
  long progress = -1;  // sum of steps and attempts: it grows while any instance works
  for (;;) {
    for (long c = 0; c < chunk; ++c) {
      const hipError_t e = exec ? hipGraphLaunch(exec, s) : slot(s);
      if (e != hipSuccess) {
        st = fail(AF_E_HIP, "%s: launch: %s", who, hipGetErrorString(e));
        break;
      }
    }
    if (st != AF_OK) break;
    if (hipMemcpyAsync(h.data(), dinst, sizeof(afi::BatchInst) * n, hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      st = fail(AF_E_HIP, "%s: read-back failed", who);
      break;
    }
    bool busy = false;
    long prog = 0;
    for (int i = 0; i < n; ++i) {
      const afi::BatchInst& I = h[i];
      if (I.active || (I.status == 0 && I.steps < max_steps && I.t < t_final)) busy = true;
      prog += I.steps + I.attempts;
    }
    if (!busy) break;
    if (prog == progress) {
      st = fail(AF_E_HIP, "%s: no instance made progress", who);
      break;
    }
    progress = prog;
  }
  if (exec && !cache) (void)hipGraphExecDestroy(exec);
  return st;
}

}  // namespace

extern "C" {

af_status af_default_params(af_params* p) {
  if (!p) return fail(AF_E_ARG, "af_default_params: NULL");
  p->dim = 2;
  p->n1 = 64;
  p->n2 = 64;
  p->x0 = 0.0;
  p->x1 = 1.0;
  p->y0 = 0.0;
  p->y1 = 1.0;
  p->gamma = 1.4;
  p->mu = 1e-3;
  p->Pr = 0.72;
  p->cfl_c = 0.2;
  p->cfl_v = 0.05;
  p->Cs = 1.0;
  p->limiter = AF_LIM_ALL;
  p->max_halvings = 40;
  p->precision = AF_PREC_FP64;
  p->rk = 3;
  return AF_OK;
}

af_status af_init_grid(const af_params* p, af_ctx** out) {
  if (!p || !out) return fail(AF_E_ARG, "af_init_grid: NULL argument");
  *out = nullptr;
  if (p->dim != 1 && p->dim != 2) return fail(AF_E_ARG, "dim must be 1 or 2 (got %d)", p->dim);
  if (p->n1 < 4) return fail(AF_E_ARG, "n1 must be >= 4 (got %d)", p->n1);
  if (p->dim == 2 && p->n2 < 4) return fail(AF_E_ARG, "n2 must be >= 4 (got %d)", p->n2);
  if ((long)p->n1 * (p->dim == 2 ? p->n2 : 1) > (1L << 28))
    return fail(AF_E_ARG, "grid too large");
  if (!(p->x1 > p->x0) || (p->dim == 2 && !(p->y1 > p->y0)))
    return fail(AF_E_ARG, "degenerate box");
  if (!(p->gamma > 1.0)) return fail(AF_E_ARG, "gamma must be > 1");
  if (!(p->mu >= 0.0)) return fail(AF_E_ARG, "mu must be >= 0");
  if (!(p->Pr > 0.0)) return fail(AF_E_ARG, "Pr must be > 0");
  if (!(p->cfl_c > 0.0) || !(p->cfl_v > 0.0)) return fail(AF_E_ARG, "CFL numbers must be > 0");
  if (!(p->Cs >= 0.0)) return fail(AF_E_ARG, "Cs must be >= 0");
  if (p->limiter < 0 || p->limiter > 127) return fail(AF_E_ARG, "bad limiter bits");
  if ((p->limiter & AF_LIM_LEARNED) && p->dim != 2)
    return fail(AF_E_ARG, "the learned blend exists for 2D only");
  if (p->max_halvings < 0) return fail(AF_E_ARG, "max_halvings must be >= 0");
  if (p->precision != AF_PREC_FP64 && p->precision != AF_PREC_MIXED)
    return fail(AF_E_ARG, "precision must be AF_PREC_FP64 or AF_PREC_MIXED");
  if (p->rk != 3 && p->rk != 54) return fail(AF_E_ARG, "rk must be 3 or 54 (got %d)", p->rk);
  if (p->precision == AF_PREC_MIXED && p->dim != 2)
    return fail(AF_E_ARG, "the mixed-precision stage exists for 2D only");
  af_ctx* c = new (std::nothrow) af_ctx;
  if (!c) return fail(AF_E_ARG, "out of host memory");
  c->p = *p;
  for (int k = 0; k < 4; ++k) c->bc[k] = AF_OUTFLOW;
  *out = c;
  return AF_OK;
}

void af_destroy(af_ctx* c) {
  if (!c) return;
  if (c->run_exec) (void)hipGraphExecDestroy(c->run_exec);
  delete c->timer;
  delete c;
}

af_status af_timing(af_ctx* c, int enable) {
  if (!c) return fail(AF_E_ARG, "af_timing: NULL context");
  if (enable && !c->timer) c->timer = new (std::nothrow) EventTimer;
  if (enable && !c->timer) return fail(AF_E_ARG, "out of host memory");
  if (!enable) {
    delete c->timer;
    c->timer = nullptr;
  }
  return AF_OK;
}

af_status af_timing_read(af_ctx* c, long* launches, double* ms) {
  if (!c || !launches || !ms) return fail(AF_E_ARG, "af_timing_read: NULL argument");
  for (int k = 0; k < AF_K_COUNT; ++k) {
    launches[k] = 0;
    ms[k] = 0.0;
  }
  EventTimer* t = c->timer;
  if (!t) return fail(AF_E_ARG, "timing is not enabled");
  if (t->err != hipSuccess) {
    hipError_t e = t->err;
    t->err = hipSuccess;
    t->n = 0;
    return hip_fail(e, "kernel timing events");
  }
  for (size_t i = 0; i < t->n; ++i) {
    AF_HIP(hipEventSynchronize(t->pool[i].second));
    float dms = 0.0f;
    AF_HIP(hipEventElapsedTime(&dms, t->pool[i].first, t->pool[i].second));
    const int k = t->kinds[i];
    if (k >= 0 && k < AF_K_COUNT) {
      launches[k] += 1;
      ms[k] += dms;
    }
  }
  t->n = 0;
  return AF_OK;
}

af_status af_set_bc(af_ctx* c, int side, int kind) {
  if (!c) return fail(AF_E_ARG, "af_set_bc: NULL context");
  if (side < 0 || side > 3) return fail(AF_E_ARG, "bad side %d", side);
  if (c->p.dim == 1 && side > 1) return fail(AF_E_ARG, "1D grid has no y sides");
  if (kind < AF_PERIODIC || kind > AF_DIRICHLET) return fail(AF_E_ARG, "bad boundary kind %d", kind);
  if (kind == AF_DIRICHLET && c->p.dim != 1)
    return fail(AF_E_ARG, "Dirichlet sides exist in 1D only");
  c->bc[side] = kind;
  return AF_OK;
}

af_status af_set_bc_state(af_ctx* c, int side, const double* state) {
  if (!c || !state) return fail(AF_E_ARG, "af_set_bc_state: NULL argument");
  if (c->p.dim != 1 || side < 0 || side > 1)
    return fail(AF_E_ARG, "Dirichlet states exist for the two sides of a 1D grid");
  if (!(state[0] > 0.0)) return fail(AF_E_ARG, "Dirichlet density must be > 0");
  for (int k = 0; k < 3; ++k) c->bcstate[side][k] = state[k];
  return AF_OK;
}

size_t af_state_len(const af_ctx* c) {
  afi::Geo g;
  if (!c || !geometry(c, &g)) return 0;
  return (size_t)g.state_len;
}

size_t af_state_bytes(const af_ctx* c) { return af_state_len(c) * sizeof(double); }

af_status af_set_state(af_ctx* c, double* U_dev, const double* U_host, void* stream) {
  if (!c || !U_dev || !U_host) return fail(AF_E_ARG, "af_set_state: NULL argument");
  const hipStream_t s = (hipStream_t)stream;
  AF_HIP(hipMemcpyAsync(U_dev, U_host, af_state_bytes(c), hipMemcpyHostToDevice, s));
  AF_HIP(hipStreamSynchronize(s));
  return AF_OK;
}

af_status af_get_state(af_ctx* c, const double* U_dev, double* U_host, void* stream) {
  if (!c || !U_dev || !U_host) return fail(AF_E_ARG, "af_get_state: NULL argument");
  const hipStream_t s = (hipStream_t)stream;
  AF_HIP(hipMemcpyAsync(U_host, U_dev, af_state_bytes(c), hipMemcpyDeviceToHost, s));
  AF_HIP(hipStreamSynchronize(s));
  return AF_OK;
}

af_status af_check_admissible(af_ctx* c, const double* U, void* ws, void* stream, long* count) {
  if (!c || !U || !ws || !count) return fail(AF_E_ARG, "af_check_admissible: NULL argument");
  afi::Geo g;
  if (!geometry(c, &g)) return AF_E_ARG;
  const afi::Work w = work_of(c, g, ws);
  const hipStream_t s = (hipStream_t)stream;
  AF_HIP(afi::count_inadmissible(g, c->p.gamma - 1.0, w, U, s));
  unsigned long long n = 0;
  AF_HIP(hipMemcpyAsync(&n, w.count, sizeof(n), hipMemcpyDeviceToHost, s));
  AF_HIP(hipStreamSynchronize(s));
  *count = (long)n;
  return AF_OK;
}

size_t af_workspace_bytes(const af_ctx* c) {
  afi::Geo g;
  if (!c || !geometry(c, &g)) return 0;
  return afi::workspace_layout(g, nullptr, nullptr);
}

af_status af_rk_stage(af_ctx* c, int k, const double* dt_dev, double dt_host, const double* Un,
                      const double* Uk, double* Uout, void* ws, void* stream) {
  if (!c || !Uk || !Uout || !ws) return fail(AF_E_ARG, "af_rk_stage: NULL argument");
  if (!net_ready(c)) return AF_E_ARG;
  if (k < 0 || k > 2) return fail(AF_E_ARG, "stage index must be 0..2 (got %d)", k);
  if (k > 0 && !Un) return fail(AF_E_ARG, "stage %d needs Un", k);
  if (Uout == Uk || (Un && Uout == Un)) return fail(AF_E_ARG, "Uout aliases an input");
  if (!dt_dev && !(dt_host >= 0.0)) return fail(AF_E_ARG, "dt must be >= 0");
  afi::Geo g;
  if (!geometry(c, &g)) return AF_E_ARG;
  const afi::Work w = work_of(c, g, ws);
  hipError_t e = launch_stage(g, physics(c->p), w, k, Un, Uk, Uout, dt_dev, dt_host,
                              (hipStream_t)stream, c->timer, false);
  if (e != hipSuccess) return hip_fail(e, "af_rk_stage launch");
  return AF_OK;
}

af_status af_cfl_dt(af_ctx* c, const double* U, double t, double t_final, double* dt_dev,
                    void* ws, void* stream) {
  if (!c || !U || !ws || !dt_dev) return fail(AF_E_ARG, "af_cfl_dt: NULL argument");
  afi::Geo g;
  if (!geometry(c, &g)) return AF_E_ARG;
  const afi::Work w = work_of(c, g, ws);
  hipError_t e = launch_cfl(c, g, w, U, t, nullptr, t_final, dt_dev, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "af_cfl_dt launch");
  return AF_OK;
}

af_status af_read_flags(af_ctx* c, const void* ws, int* flags, void* stream) {
  if (!c || !ws || !flags) return fail(AF_E_ARG, "af_read_flags: NULL argument");
  afi::Geo g;
  if (!geometry(c, &g)) return AF_E_ARG;
  const afi::Work w = work_of(c, g, ws);
  unsigned f = 0;
  af_status st = read_flags(w, (hipStream_t)stream, &f);
  *flags = (int)f;
  return st;
}

af_status af_reset_flags(af_ctx* c, void* ws, void* stream) {
  if (!c || !ws) return fail(AF_E_ARG, "af_reset_flags: NULL argument");
  afi::Geo g;
  if (!geometry(c, &g)) return AF_E_ARG;
  const afi::Work w = work_of(c, g, ws);
  AF_HIP(afi::clear_flags(w, (hipStream_t)stream));
  return AF_OK;
}

af_status af_step(af_ctx* c, double* U, void* ws, void* stream, double dt, double t,
                  double t_final, double* dt_used, int* halvings) {
  if (!c || !U || !ws) return fail(AF_E_ARG, "af_step: NULL argument");
  if (!net_ready(c)) return AF_E_ARG;
  if (!(t_final >= t)) return fail(AF_E_ARG, "t_final < t");
  afi::Geo g;
  if (!geometry(c, &g)) return AF_E_ARG;
  const afi::Work w = work_of(c, g, ws);
  const hipStream_t s = (hipStream_t)stream;
  const afd::Phys ph = physics(c->p);
  AF_HIP(afi::copy_state(w.SAVE, U, g.state_len, s));
  if (dt <= 0.0) {
    AF_HIP(launch_cfl(c, g, w, U, t, nullptr, t_final, w.scal, s));
    AF_HIP(hipMemcpyAsync(&dt, w.scal, sizeof(double), hipMemcpyDeviceToHost, s));
    AF_HIP(hipStreamSynchronize(s));
  } else if (t + dt > t_final) {
    dt = t_final - t;
  }
  unsigned fl = 0;
  int h;
  for (h = 0; h <= c->p.max_halvings; ++h) {
    AF_HIP(afi::clear_flags(w, s));
    if (c->p.rk == 54)
      AF_HIP(rk54(g, ph, w, w.SAVE, w.S1, w.S2, U, nullptr, dt, s, c->timer));
    else
      AF_HIP(rk3(g, ph, w, w.SAVE, U, nullptr, dt, s, c->timer));
    af_status st = read_flags(w, s, &fl);
    if (st != AF_OK) return st;
    if (fl == 0) break;
    dt *= 0.5;
  }
  if (dt_used) *dt_used = dt;
  if (halvings) *halvings = h;
  if (fl != 0) {
    AF_HIP(afi::copy_state(U, w.SAVE, g.state_len, s));
    AF_HIP(hipStreamSynchronize(s));
    if (fl & AF_FLAG_NONFINITE) return fail(AF_E_NONFINITE, "non-finite values after %d halvings", h - 1);
    return fail(AF_E_PP, "low-order states inadmissible after %d halvings (flags %u)", h - 1, fl);
  }
  return AF_OK;
}

af_status af_step_noalloc(af_ctx* c, double* U, void* stream, double dt, double t,
                          double t_final, double* dt_used, int* halvings) {
  if (!c || !U) return fail(AF_E_ARG, "af_step_noalloc: NULL argument");
  afi::Geo g;
  if (!geometry(c, &g)) return AF_E_ARG;
  const size_t need = afi::workspace_layout(g, nullptr, nullptr);
  if (need > (size_t)AF_NOALLOC_SCRATCH_BYTES)
    return fail(AF_E_ARG,
                "af_step_noalloc: this grid needs %zu workspace bytes, more than the %zu of "
                "the library's scratch array",
                need, (size_t)AF_NOALLOC_SCRATCH_BYTES);
  void* ws = nullptr;
  const af_status st = scratch_on_current_device(&ws);
  if (st != AF_OK) return st;
  return af_step(c, U, ws, stream, dt, t, t_final, dt_used, halvings);
}

af_status af_run(af_ctx* c, double* U, void* ws, void* stream, double t0, double t_final,
                 long max_steps, int check_every, long* nsteps_out, double* t_out) {
  if (!c || !U || !ws) return fail(AF_E_ARG, "af_run: NULL argument");
  if (!net_ready(c)) return AF_E_ARG;
  if (check_every < 1) return fail(AF_E_ARG, "check_every must be >= 1");
  if (max_steps < 0) return fail(AF_E_ARG, "max_steps must be >= 0");
  afi::Geo g;
  if (!geometry(c, &g)) return AF_E_ARG;
  const afi::Work w = work_of(c, g, ws);
  const hipStream_t s = (hipStream_t)stream;
  const afd::Phys ph = physics(c->p);
  // the current state rotates through U, S1, S2 (and S3 for SSP-RK54): a
  // step reads `cur` and writes its stages to the others, so `cur`
  // survives a rejected step
  const bool rk54s = c->p.rk == 54;
  double* bufs[4] = {U, w.S1, w.S2, w.S3};
  auto next = [&](int from) { return rk54s ? (from + 3) % 4 : (from + 1) % 3; };
  int cur = 0;
  double t = t0;
  long done = 0;
  af_status status = AF_OK;
  double sc[4];
  unsigned fl = 0;
  auto read_back = [&]() -> af_status {
    AF_HIP(hipMemcpyAsync(sc, w.scal, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
    AF_HIP(hipMemcpyAsync(&fl, w.flags, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    AF_HIP(hipStreamSynchronize(s));
    return AF_OK;
  };
  auto three_stages = [&](int from) -> hipError_t {
    if (rk54s)
      return rk54(g, ph, w, bufs[from], bufs[(from + 1) % 4], bufs[(from + 2) % 4],
                  bufs[(from + 3) % 4], w.scal, 0.0, s, c->timer);
    const int a = (from + 1) % 3, b = (from + 2) % 3;
    hipError_t e;
    if ((e = launch_stage(g, ph, w, 0, bufs[from], bufs[from], bufs[a], w.scal, 0.0, s,
                          c->timer)) != hipSuccess)
      return e;
    if ((e = launch_stage(g, ph, w, 1, bufs[from], bufs[a], bufs[b], w.scal, 0.0, s,
                          c->timer)) != hipSuccess)
      return e;
    return launch_stage(g, ph, w, 2, bufs[from], bufs[b], bufs[a], w.scal, 0.0, s, c->timer);
  };
  AF_HIP(afi::set_scalar(w.scal + 1, t, s));
  while (done < max_steps && t < t_final) {
    const long K = (max_steps - done) < check_every ? (max_steps - done) : check_every;
    if (K > 1) {
      // optimistic block of K steps with one synchronisation at its end
      AF_HIP(afi::copy_state(w.SAVE, bufs[cur], g.state_len, s));
      AF_HIP(afi::set_scalar(w.scal + 2, 0.0, s));
      AF_HIP(afi::clear_flags(w, s));
      int c2 = cur;
      for (long k = 0; k < K; ++k) {
        AF_HIP(launch_cfl(c, g, w, bufs[c2], 0.0, w.scal + 1, t_final, w.scal, s));
        AF_HIP(three_stages(c2));
        AF_HIP(afi::advance_time(w, s));
        c2 = next(c2);
      }
      if ((status = read_back()) != AF_OK) break;
      if (fl == 0) {
        cur = c2;
        t = sc[1];
        done += (long)sc[2];
        if ((long)sc[2] < K) break;  // t_final reached inside the block
        continue;
      }
      // a step of the block was rejected: restore its start, step singly
      AF_HIP(afi::copy_state(bufs[cur], w.SAVE, g.state_len, s));
      AF_HIP(afi::set_scalar(w.scal + 1, t, s));
    }
    for (long k = 0; k < K && t < t_final; ++k) {
      AF_HIP(launch_cfl(c, g, w, bufs[cur], 0.0, w.scal + 1, t_final, w.scal, s));
      int h;
      for (h = 0; h <= c->p.max_halvings; ++h) {
        AF_HIP(afi::clear_flags(w, s));
        AF_HIP(three_stages(cur));
        if ((status = read_back()) != AF_OK) break;
        if (fl == 0) break;
        AF_HIP(afi::scale_scalar(w.scal, 0.5, s));  // redo with dt/2
      }
      if (status != AF_OK) break;
      if (fl != 0) {
        status = (fl & AF_FLAG_NONFINITE)
                     ? fail(AF_E_NONFINITE, "non-finite values at t=%g after %d halvings", t, h - 1)
                     : fail(AF_E_PP, "low-order states inadmissible at t=%g after %d halvings", t,
                            h - 1);
        break;
      }
      AF_HIP(afi::set_scalar(w.scal + 2, 0.0, s));
      AF_HIP(afi::advance_time(w, s));
      t = sc[1] + sc[0];
      cur = next(cur);
      ++done;
    }
    if (status != AF_OK) break;
  }
  if (cur != 0) {
    AF_HIP(afi::copy_state(U, bufs[cur], g.state_len, s));
  }
  AF_HIP(hipStreamSynchronize(s));
  if (nsteps_out) *nsteps_out = done;
  if (t_out) *t_out = t;
  return status;
}

af_status af_batch_create(af_ctx* const* ctxs, int n, af_batch** out) {
  if (!ctxs || !out || n < 1) return fail(AF_E_ARG, "af_batch_create: NULL argument or n < 1");
  *out = nullptr;
  if (n > 512) return fail(AF_E_ARG, "af_batch_create: at most 512 instances");
  std::unique_ptr<af_batch> b(new (std::nothrow) af_batch);
  if (!b) return fail(AF_E_ARG, "out of host memory");
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) & ~(size_t)255;
    return o;
  };
  take(sizeof(afi::BatchInst) * n);
  b->off_partial = take(sizeof(double) * 2 *
                        (n == 1 ? afi::kSingleCflBlocks : afi::kBatchCflBlocks * n));
  b->off_nact = take(sizeof(int));
  for (int i = 0; i < n; ++i) {
    af_ctx* c = ctxs[i];
    if (!c) return fail(AF_E_ARG, "af_batch_create: context %d is NULL", i);
    if (c->p.dim != 2) return fail(AF_E_ARG, "af_batch_create: context %d is not 2D", i);
    if (i == 0) b->mixed = c->p.precision == AF_PREC_MIXED;
    if ((c->p.precision == AF_PREC_MIXED) != (b->mixed != 0))
      return fail(AF_E_ARG, "af_batch_create: the contexts must share one precision");
    afi::Geo g;
    if (!geometry(c, &g)) return AF_E_ARG;
    b->ctx.push_back(c);
    b->geo.push_back(g);
    b->off_bufs.push_back(take(sizeof(double) * g.state_len));
    b->off_bufs.push_back(take(sizeof(double) * g.state_len));
  }
  b->bytes = off;
  b->var = afi::default_variant(b->mixed);
  *out = b.release();
  return AF_OK;
}

void af_batch_destroy(af_batch* b) { delete b; }

size_t af_batch_workspace_bytes(const af_batch* b) { return b ? b->bytes : 0; }

af_status af_batch_run(af_batch* b, double* const* U, void* ws, void* stream, double t0,
                       double t_final, long max_steps, int attempts_per_slot, int use_graph,
                       long* steps, double* t_out, int* status, long* attempts) {
  if (!b || !U || !ws) return fail(AF_E_ARG, "af_batch_run: NULL argument");
  if (attempts_per_slot < 1) return fail(AF_E_ARG, "attempts_per_slot must be >= 1");
  if (max_steps < 0 || !(t_final >= t0)) return fail(AF_E_ARG, "af_batch_run: bad steps or times");
  const int n = (int)b->ctx.size();
  const hipStream_t s = (hipStream_t)stream;
  char* base = (char*)ws;
  afi::BatchInst* dinst = (afi::BatchInst*)base;
  double* partial = (double*)(base + b->off_partial);
  int* nact = (int*)(base + b->off_nact);
  std::vector<afi::BatchInst> h;
  int total_tiles = 0;
  const af_status sd =
      batch_descriptors(b, b->var, U, base, t0, t_final, max_steps, h, &total_tiles);
  if (sd != AF_OK) return sd;
  AF_HIP(hipMemcpyAsync(dinst, h.data(), sizeof(afi::BatchInst) * n, hipMemcpyHostToDevice, s));
  auto slot = [&](hipStream_t q) {
    return batch_slot(b->var, dinst, n, total_tiles, partial, nact, attempts_per_slot, q);
  };
  const af_status st =
      run_slots(slot, dinst, n, use_graph, s, max_steps, t_final, h, "af_batch_run");
  if (st != AF_OK) return st;
  // the current state of every instance back into its U
  for (int i = 0; i < n; ++i)
    if (h[i].cur != 0) AF_HIP(afi::copy_state(U[i], h[i].buf[h[i].cur], b->geo[i].state_len, s));
  AF_HIP(hipStreamSynchronize(s));
  for (int i = 0; i < n; ++i) {
    if (steps) steps[i] = h[i].steps;
    if (t_out) t_out[i] = h[i].t;
    if (status) status[i] = h[i].status;
    if (attempts) attempts[i] = h[i].attempts;
  }
  return AF_OK;
}

af_status af_run_graph(af_ctx* c, double* U, void* ws, void* stream, double t0, double t_final,
                       long max_steps, int attempts_per_slot, long* nsteps_out, double* t_out,
                       long* attempts_out) {
  if (!c || !U || !ws) return fail(AF_E_ARG, "af_run_graph: NULL argument");
  if (c->p.dim != 2 || c->p.rk != 3 || (c->p.limiter & AF_LIM_LEARNED))
    return fail(AF_E_ARG, "af_run_graph: 2D, SSP-RK3, plain limiters only");
  if (attempts_per_slot < 1) return fail(AF_E_ARG, "attempts_per_slot must be >= 1");
  if (max_steps < 0 || !(t_final >= t0)) return fail(AF_E_ARG, "af_run_graph: bad steps or times");
  afi::Geo g;
  if (!geometry(c, &g)) return AF_E_ARG;
  const afi::Work w = work_of(c, g, ws);
  const hipStream_t s = (hipStream_t)stream;
  const afi::StageVariant* v = afi::default_variant(g.mixed);
  std::vector<afi::BatchInst> h(1);
  h[0] = instance_of(c, g, v, U, w.S1, w.S2, t0, t_final, max_steps);
  h[0].stage_nwg = v->dev_nwg(g);
  AF_HIP(hipMemcpyAsync(w.binst, h.data(), sizeof(afi::BatchInst), hipMemcpyHostToDevice, s));
  // the first step's CFL maxima; every later step opens from those its
  // predecessor's last stage left (the dt reduction fused into that stage)
  AF_HIP(afi::batch_cfl(w.binst, 1, w.bpartial, afi::kSingleCflBlocks, s));
  int dev = 0;
  AF_HIP(hipGetDevice(&dev));
  if (c->run_exec && (c->run_ws != ws || c->run_slot != attempts_per_slot || c->run_dev != dev)) {
    (void)hipGraphExecDestroy(c->run_exec);
    c->run_exec = nullptr;
  }
  c->run_ws = ws;
  c->run_slot = attempts_per_slot;
  c->run_dev = dev;
  const afd::Phys ph = physics(c->p);
  // a round: open a step if the last one was accepted (CFL dt from the
  // maxima its last stage left), one RK3 attempt with the single-instance
  // stage kernel, accept or halve
  auto slot = [&](hipStream_t q) {
    hipError_t e;
    for (int a = 0; a < attempts_per_slot; ++a) {
      if ((e = afi::batch_open(w.binst, 1, w.bpartial, afi::kSingleCflBlocks, w.bnact, q)) !=
          hipSuccess)
        return e;
      for (int k = 0; k < 3; ++k)
        if ((e = v->dev(g, ph, w.binst, w.bpartial, k, q)) != hipSuccess) return e;
      if ((e = afi::batch_decide(w.binst, 1, w.bnact, q)) != hipSuccess) return e;
    }
    return hipSuccess;
  };
  const af_status st = run_slots(slot, w.binst, 1, 1, s, max_steps, t_final, h, "af_run_graph",
                                 &c->run_exec, 4);
  if (st != AF_OK) return st;
  if (h[0].cur != 0) AF_HIP(afi::copy_state(U, h[0].buf[h[0].cur], g.state_len, s));
  AF_HIP(hipStreamSynchronize(s));
  if (nsteps_out) *nsteps_out = h[0].steps;
  if (t_out) *t_out = h[0].t;
  if (attempts_out) *attempts_out = h[0].attempts;
  if (h[0].status == AF_E_NONFINITE)
    return fail(AF_E_NONFINITE, "non-finite values at t=%g", h[0].t);
  if (h[0].status == AF_E_PP)
    return fail(AF_E_PP, "low-order states inadmissible at t=%g after %d halvings", h[0].t,
                c->p.max_halvings);
  return AF_OK;
}

long af_face_count(const af_ctx* c) {
  if (!c) return 0;
  const long n1 = c->p.n1, n2 = c->p.dim == 2 ? c->p.n2 : 0;
  return c->p.dim == 1 ? n1 + 1 : n2 * (n1 + 1) + (n2 + 1) * n1;
}

size_t af_mlp_param_count(void) { return (size_t)afi::kMlpParams; }

af_status af_blend_features(af_ctx* c, const double* U, float* feat, void* stream) {
  if (!c || !U || !feat) return fail(AF_E_ARG, "af_blend_features: NULL argument");
  if (c->p.dim != 2) return fail(AF_E_ARG, "af_blend_features: 2D only");
  afi::Geo g;
  if (!geometry(c, &g)) return AF_E_ARG;
  AF_HIP(afi::blend_features(g, physics(c->p), U, feat, (hipStream_t)stream));
  return AF_OK;
}

af_status af_set_blend_net(af_ctx* c, const float* params) {
  if (!c) return fail(AF_E_ARG, "af_set_blend_net: NULL context");
  if (c->p.dim != 2 && params) return fail(AF_E_ARG, "af_set_blend_net: 2D only");
  c->net = params;
  return AF_OK;
}

af_status af_blend_infer(af_ctx* c, const double* U, float* theta, void* ws, void* stream) {
  if (!c || !U || !theta || !ws) return fail(AF_E_ARG, "af_blend_infer: NULL argument");
  if (c->p.dim != 2) return fail(AF_E_ARG, "af_blend_infer: 2D only");
  if (!c->net) return fail(AF_E_ARG, "af_blend_infer: no network set (af_set_blend_net)");
  afi::Geo g;
  if (!geometry(c, &g)) return AF_E_ARG;
  const afi::Work w = work_of(c, g, ws);
  const hipStream_t s = (hipStream_t)stream;
  AF_HIP(afi::mlp_pack(c->net, w.mlp, s));
  AF_HIP(afi::blend_infer(g, physics(c->p), U, w.mlp, theta, s, c->timer));
  return AF_OK;
}

af_status af_rk_stage_blend(af_ctx* c, int k, const double* dt_dev, double dt_host,
                            const double* Un, const double* Uk, double* Uout, const float* theta,
                            float* theta_s_out, void* ws, void* stream) {
  if (!c || !Uk || !Uout || !ws) return fail(AF_E_ARG, "af_rk_stage_blend: NULL argument");
  if (c->p.dim != 2) return fail(AF_E_ARG, "af_rk_stage_blend: 2D only");
  if (k < 0 || k > 2) return fail(AF_E_ARG, "stage index must be 0..2 (got %d)", k);
  if (k > 0 && !Un) return fail(AF_E_ARG, "stage %d needs Un", k);
  if (Uout == Uk || (Un && Uout == Un)) return fail(AF_E_ARG, "Uout aliases an input");
  if (!dt_dev && !(dt_host >= 0.0)) return fail(AF_E_ARG, "dt must be >= 0");
  if (!theta && !net_ready(c)) return AF_E_ARG;
  afi::Geo g;
  if (!geometry(c, &g)) return AF_E_ARG;
  const afi::Work w = work_of(c, g, ws);
  afd::Phys ph = physics(c->p);
  if (theta) ph.lim &= ~afd::LIM_LEARNED;  // the given blend, no inference
  if (!Un) Un = Uk;
  afi::StageCoef sc = kCoef[k];
  sc.skip_flagged = 0;
  sc.ts_out = theta_s_out;
  const hipStream_t s = (hipStream_t)stream;
  if (theta) {
    sc.blend = theta;
  } else if (ph.lim & afd::LIM_LEARNED) {
    AF_HIP(afi::mlp_pack(c->net, w.mlp, s));
    AF_HIP(afi::blend_infer(g, ph, Uk, w.mlp, w.blend, s, c->timer));
    sc.blend = w.blend;
  }
  AF_HIP(afi::stage2d(g, ph, w, Un, Uk, Uout, dt_dev, dt_host, sc, s, c->timer));
  return AF_OK;
}

size_t af_mlp_grad_workspace_bytes(long n) { return afi::mlp_grad_workspace(n); }

af_status af_mlp_grad(const float* X, const float* y, long n, const float* params, float* grad,
                      float* loss, void* gws, void* stream) {
  if (!X || !y || !params || !grad || !gws) return fail(AF_E_ARG, "af_mlp_grad: NULL argument");
  if (n < 1) return fail(AF_E_ARG, "af_mlp_grad: n must be >= 1");
  AF_HIP(afi::mlp_grad(X, y, n, params, grad, loss, gws, (hipStream_t)stream));
  return AF_OK;
}

af_status af_mlp_adam(float* params, const float* grad, float* m, float* v, long step, float lr,
                      void* stream) {
  if (!params || !grad || !m || !v) return fail(AF_E_ARG, "af_mlp_adam: NULL argument");
  if (step < 1) return fail(AF_E_ARG, "af_mlp_adam: step counts from 1");
  AF_HIP(afi::mlp_adam(params, grad, m, v, step, lr, (hipStream_t)stream));
  return AF_OK;
}

af_status af_mlp_train(const float* X, const float* y, long n, float* params, float* grad,
                       float* m, float* v, long step0, int steps, int batch, float lr,
                       float* loss_out, void* gws, void* stream) {
  if (!X || !y || !params || !grad || !m || !v || !gws)
    return fail(AF_E_ARG, "af_mlp_train: NULL argument");
  if (n < 1 || steps < 0 || batch < 1 || step0 < 0)
    return fail(AF_E_ARG, "af_mlp_train: bad sizes");
  const hipStream_t s = (hipStream_t)stream;
  long row = 0;
  for (int k = 0; k < steps; ++k) {
    // the next minibatch in order; a batch that would cross the end starts
    // over from the first row
    long nb = batch < n ? batch : n;
    if (row + nb > n) row = 0;
    AF_HIP(afi::mlp_grad(X + row * afi::kMlpIn, y + row, nb, params, grad, loss_out, gws, s));
    AF_HIP(afi::mlp_adam(params, grad, m, v, step0 + k + 1, lr, s));
    row += nb;
  }
  return AF_OK;
}

int af_stage_times(int rk, double* c) {
  if (!c) return -1;
  if (rk == 3) {
    c[0] = 0.0;
    c[1] = 1.0;
    c[2] = 0.5;
    return 3;
  }
  if (rk != 54) return -1;
  c[0] = 0.0;
  c[1] = kB10;
  c[2] = kA21 * c[1] + kB21;
  c[3] = kA32 * c[2] + kB32;
  c[4] = kA43 * c[3] + kB43;
  return 5;
}

af_status af_step_source(af_ctx* c, double* U, void* ws, void* stream, double dt,
                         const double* const* src, int nsrc) {
  if (!c || !U || !ws || !src) return fail(AF_E_ARG, "af_step_source: NULL argument");
  if (!(dt > 0.0)) return fail(AF_E_ARG, "af_step_source: dt must be > 0");
  if (!net_ready(c)) return AF_E_ARG;
  const int need = c->p.rk == 54 ? 5 : 3;
  if (nsrc != need) return fail(AF_E_ARG, "af_step_source: %d source states needed", need);
  for (int k = 0; k < need; ++k)
    if (!src[k]) return fail(AF_E_ARG, "af_step_source: source %d is NULL", k);
  afi::Geo g;
  if (!geometry(c, &g)) return AF_E_ARG;
  const afi::Work w = work_of(c, g, ws);
  const hipStream_t s = (hipStream_t)stream;
  const afd::Phys ph = physics(c->p);
  AF_HIP(afi::copy_state(w.SAVE, U, g.state_len, s));
  AF_HIP(afi::clear_flags(w, s));
  if (c->p.rk == 54)
    AF_HIP(rk54(g, ph, w, w.SAVE, w.S1, w.S2, U, nullptr, dt, s, c->timer, src));
  else
    AF_HIP(rk3(g, ph, w, w.SAVE, U, nullptr, dt, s, c->timer, src));
  unsigned fl = 0;
  af_status st = read_flags(w, s, &fl);
  if (st != AF_OK) return st;
  if (fl != 0) {
    AF_HIP(afi::copy_state(U, w.SAVE, g.state_len, s));
    AF_HIP(hipStreamSynchronize(s));
    if (fl & AF_FLAG_NONFINITE) return fail(AF_E_NONFINITE, "non-finite values (flags %u)", fl);
    return fail(AF_E_PP, "low-order states inadmissible (flags %u)", fl);
  }
  return AF_OK;
}

int af_stage_variant_count(void) { return afi::kNumStageVariants; }

af_status af_stage_variant_info(int i, const char** name, int* precision, int* tile_height) {
  if (i < 0 || i >= afi::kNumStageVariants)
    return fail(AF_E_ARG, "af_stage_variant_info: no variant %d", i);
  const afi::StageVariant& v = afi::kStageVariants[i];
  if (name) *name = v.name;
  if (precision) *precision = v.mixed ? AF_PREC_MIXED : AF_PREC_FP64;
  if (tile_height) *tile_height = v.ty;
  return AF_OK;
}

int af_batch_variant(const af_batch* b) {
  return b ? (int)(b->var - afi::kStageVariants) : -1;
}

af_status af_batch_set_variant(af_batch* b, int i) {
  if (!b) return fail(AF_E_ARG, "af_batch_set_variant: NULL batch");
  if (i < 0 || i >= afi::kNumStageVariants)
    return fail(AF_E_ARG, "af_batch_set_variant: no variant %d", i);
  if (afi::kStageVariants[i].mixed != b->mixed)
    return fail(AF_E_ARG, "af_batch_set_variant: variant %s has another precision",
                afi::kStageVariants[i].name);
  b->var = &afi::kStageVariants[i];
  return AF_OK;
}

af_status af_batch_tune(af_batch* b, double* const* U, void* ws, void* stream, double t0,
                        double t_final, int reps, double* us_per_slot) {
  if (!b || !U || !ws) return fail(AF_E_ARG, "af_batch_tune: NULL argument");
  if (reps < 1) return fail(AF_E_ARG, "af_batch_tune: reps must be >= 1");
  if (!(t_final > t0)) return fail(AF_E_ARG, "af_batch_tune: t_final must exceed t0");
  const int n = (int)b->ctx.size();
  const hipStream_t s = (hipStream_t)stream;
  char* base = (char*)ws;
  afi::BatchInst* dinst = (afi::BatchInst*)base;
  double* partial = (double*)(base + b->off_partial);
  int* nact = (int*)(base + b->off_nact);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  AF_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(AF_E_HIP, "af_batch_tune: event creation failed");
  }
  af_status st = AF_OK;
  const afi::StageVariant* best = b->var;
  double best_us = -1.0;
  std::vector<afi::BatchInst> h;
  for (int i = 0; i < afi::kNumStageVariants && st == AF_OK; ++i) {
    const afi::StageVariant* v = &afi::kStageVariants[i];
    if (us_per_slot) us_per_slot[i] = -1.0;
    if (v->mixed != b->mixed) continue;
    int total = 0;
    st = batch_descriptors(b, v, U, base, t0, t_final, 1, h, &total);
    if (st != AF_OK) break;
    // one untimed slot, then the fastest of reps; every slot starts from the
    // same descriptors (current buffer U, so U is never written)
    double best_v = -1.0;
    for (int r = 0; r <= reps; ++r) {
      hipError_t e = hipMemcpyAsync(dinst, h.data(), sizeof(afi::BatchInst) * n,
                                    hipMemcpyHostToDevice, s);
      if (e == hipSuccess) e = hipEventRecord(e0, s);
      if (e == hipSuccess) e = batch_slot(v, dinst, n, total, partial, nact, 1, s);
      if (e == hipSuccess) e = hipEventRecord(e1, s);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) {
        st = hip_fail(e, "af_batch_tune");
        break;
      }
      if (r > 0 && (best_v < 0.0 || ms * 1e3 < best_v)) best_v = ms * 1e3;
    }
    if (st != AF_OK) break;
    if (us_per_slot) us_per_slot[i] = best_v;
    if (best_us < 0.0 || best_v < best_us) {
      best_us = best_v;
      best = v;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st == AF_OK) b->var = best;
  return st;
}

const char* af_last_error(void) { return g_err.c_str(); }

}  // extern "C"
