// pn_api.hip -- host side of libpn: the extern "C" entry points declared in
// include/pn.h, argument validation, per-device scratch, launch shapes and
// the HIP graph that replays one Runge-Kutta step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "pn.h"
#include "pn_kernels.h"

namespace {

using namespace pn;

// ------------------------------------------------------------------ errors
char g_err[512] = "no error";
std::mutex g_mu;  // serialises every entry point (scratch and graphs are shared)

int fail_hip(hipError_t e, const char* what, int line) {
  snprintf(g_err, sizeof g_err, "%s failed at pn_api.hip:%d: %s", what, line, hipGetErrorString(e));
  return (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? PN_ENOMEM : PN_EDEVICE;
}
#define HIPCK(x)                                                   \
  do {                                                             \
    hipError_t e_ = (x);                                           \
    if (e_ != hipSuccess) return fail_hip(e_, #x, __LINE__);       \
  } while (0)

// ------------------------------------------------------------------ launch shapes
struct Shape {
  int ipt = 1;     // i-bodies per lane
  int ws = 4;      // wavefronts sharing one i-range (1 or 4)
  int nsplit = 1;  // j splits (gridDim.y)
  int jchunk = 1;  // j per split
  int iblocks = 1; // gridDim.x
};

// Tuned shapes installed with pn_set_shape (searched by the autotuner).
struct TunedShape {
  int precision;
  int64_t n_min, n_max;
  int ipt, ws, nsplit;
};
std::vector<TunedShape> g_tuned;

// Shape: a tuned entry if one covers (precision, N), else the default: four
// wavefronts per i-range, one i per lane, and 16 j-splits (measured best for
// the whole evaluation at N = 16k-64k on MI355X: enough workgroups in flight
// without making the epilogue's split reduction dominate), at least 32 j per
// wavefront.  PN_SHAPE="ipt,ws,nsplit" overrides everything (tuning runs).
Shape pick_shape(int Ns, int precision) {
  Shape s;
  s.ipt = 1;
  s.ws = 4;
  int want_nsplit = 0;
  for (const TunedShape& t : g_tuned) {
    if (t.precision == precision && Ns + 1 >= t.n_min && Ns + 1 <= t.n_max) {
      s.ipt = t.ipt;
      s.ws = t.ws;
      want_nsplit = t.nsplit;
      break;
    }
  }
  if (const char* env = getenv("PN_SHAPE")) {
    int a = 0, b = 0, c = 0;
    if (sscanf(env, "%d,%d,%d", &a, &b, &c) == 3 && (a == 1 || a == 2) && (b == 1 || b == 4) &&
        c >= 0) {
      s.ipt = a;
      s.ws = b;
      want_nsplit = c;
    }
  }
  const int ib = kBlock / s.ws * s.ipt;  // i-bodies per workgroup
  s.iblocks = (Ns + ib - 1) / ib;
  if (want_nsplit <= 0) {
    want_nsplit = std::max(16, (4096 + s.iblocks - 1) / s.iblocks);
    want_nsplit = std::min(want_nsplit, std::max(1, Ns / (32 * s.ws)));
  }
  want_nsplit = std::max(1, std::min(want_nsplit, Ns));
  s.jchunk = (Ns + want_nsplit - 1) / want_nsplit;
  s.nsplit = (Ns + s.jchunk - 1) / s.jchunk;
  return s;
}

// ------------------------------------------------------------------ scratch
size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
  size_t pk, ub, bpart, part, bhpart, status, xs, vs, kx, kv, dpart, out8, total;
};

Layout layout_for(int64_t N, const Shape& s, bool rk4) {
  const size_t Ns = (size_t)(N - 1);
  const size_t nb = (Ns + kBlock - 1) / kBlock;
  Layout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += align256(bytes);
    return at;
  };
  L.pk = take(Ns * sizeof(PkF64));
  L.ub = take(Ns * 4 * sizeof(double));
  L.bpart = take(nb * 8 * sizeof(double));
  L.part = take((size_t)s.nsplit * std::max(kNF, kND) * Ns * sizeof(double));
  L.bhpart = take(((Ns + kEpiStars - 1) / kEpiStars) * 4 * sizeof(double));
  L.status = take(sizeof(int));
  L.dpart = take(nb * 10 * sizeof(double));
  L.out8 = take(8 * sizeof(double));
  const size_t n3 = 3 * (size_t)N * sizeof(double);
  L.xs = take(rk4 ? n3 : 0);
  L.vs = take(rk4 ? n3 : 0);
  L.kx = take(rk4 ? n3 : 0);
  L.kv = take(rk4 ? n3 : 0);
  L.total = o;
  return L;
}

struct GraphKey {
  const void *pos = nullptr, *vel = nullptr, *mass = nullptr;
  int64_t N = 0;
  double G = 0, c = 0, eps = 0, dt = 0;
  int precision = -1, ipt = 0, ws = 0, nsplit = 0;
  char* base = nullptr;
  bool operator==(const GraphKey& o) const {
    return pos == o.pos && vel == o.vel && mass == o.mass && N == o.N && G == o.G &&
           (c == o.c || (std::isinf(c) && std::isinf(o.c))) && eps == o.eps && dt == o.dt &&
           precision == o.precision && ipt == o.ipt && ws == o.ws && nsplit == o.nsplit &&
           base == o.base;
  }
};

struct DevState {
  bool init = false;
  hipStream_t own = nullptr;
  char* base = nullptr;
  size_t cap = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  GraphKey key;
  std::vector<hipEvent_t> ev;
};
std::vector<DevState> g_dev;

double g_timing[3] = {0, 0, 0};

int dev_state(DevState** out) {
  int dev = 0;
  HIPCK(hipGetDevice(&dev));
  if ((int)g_dev.size() <= dev) g_dev.resize(dev + 1);
  DevState& d = g_dev[dev];
  if (!d.init) {
    HIPCK(hipStreamCreateWithFlags(&d.own, hipStreamDefault));
    d.init = true;
  }
  *out = &d;
  return PN_OK;
}

void drop_graph(DevState& d) {
  if (d.gexec) hipGraphExecDestroy(d.gexec);
  if (d.graph) hipGraphDestroy(d.graph);
  d.gexec = nullptr;
  d.graph = nullptr;
  d.key = GraphKey();
}

int ensure_scratch(DevState& d, size_t bytes) {
  if (bytes <= d.cap) return PN_OK;
  HIPCK(hipDeviceSynchronize());
  drop_graph(d);  // graphs hold the old addresses
  if (d.base) HIPCK(hipFree(d.base));
  d.base = nullptr;
  d.cap = 0;
  size_t want = std::max(bytes, (size_t)1 << 20);
  hipError_t e = hipMalloc(&d.base, want);
  if (e != hipSuccess) return fail_hip(e, "hipMalloc(scratch)", __LINE__);
  d.cap = want;
  return PN_OK;
}

// ------------------------------------------------------------------ validation
bool dptr_ok(const void* p) { return p != nullptr && ((uintptr_t)p & 7u) == 0; }

int check_system(const void* pos, const void* mass, int64_t N, double G, double c, double eps) {
  if (!dptr_ok(pos) || !dptr_ok(mass)) return PN_EINVAL;
  if (N < 2 || N > ((int64_t)1 << 28)) return PN_EINVAL;
  if (!(G > 0.0) || !std::isfinite(G)) return PN_EINVAL;
  if (std::isnan(c) || !(c > 0.0)) return PN_EINVAL;
  if (!(eps >= 0.0) || !std::isfinite(eps)) return PN_EINVAL;
  return PN_OK;
}

double lambda_of(double c) { return std::isinf(c) ? 0.0 : 1.0 / (c * c); }

// ------------------------------------------------------------------ enqueue helpers
struct Sys {
  const double* pos;
  const double* vel;
  const double* mass;
  int64_t N;
  double G, c, eps;
};

struct Ptrs {
  char* base;
  Layout L;
  template <typename T>
  T* at(size_t off) const { return reinterpret_cast<T*>(base + off); }
};

int launch_prologue(const Sys& s, const Ptrs& P, int precision, hipStream_t st) {
  const int Ns = (int)(s.N - 1);
  ProArgs a;
  a.pos = s.pos;
  a.vel = s.vel;
  a.mass = s.mass;
  a.Ns = Ns;
  a.G = s.G;
  a.eps2 = s.eps * s.eps;
  a.pk = P.at<void>(P.L.pk);
  a.ub = P.at<double>(P.L.ub);
  a.bpart = P.at<double>(P.L.bpart);
  a.status = P.at<int>(P.L.status);
  const int nb = (Ns + kBlock - 1) / kBlock;
  if (precision == PN_MIXED)
    hipLaunchKernelGGL(k_prologue<float>, dim3(nb), dim3(kBlock), 0, st, a);
  else
    hipLaunchKernelGGL(k_prologue<double>, dim3(nb), dim3(kBlock), 0, st, a);
  HIPCK(hipGetLastError());
  return PN_OK;
}

template <typename T, int MODE>
void launch_pair_t(const PairArgs& a, const Shape& sh, hipStream_t st) {
  dim3 grid(sh.iblocks, sh.nsplit);
  if (sh.ws == 4) {
    if (sh.ipt == 2)
      hipLaunchKernelGGL((k_pair<T, MODE, 2, 4>), grid, dim3(kBlock), 0, st, a);
    else
      hipLaunchKernelGGL((k_pair<T, MODE, 1, 4>), grid, dim3(kBlock), 0, st, a);
  } else {
    if (sh.ipt == 2)
      hipLaunchKernelGGL((k_pair<T, MODE, 2, 1>), grid, dim3(kBlock), 0, st, a);
    else
      hipLaunchKernelGGL((k_pair<T, MODE, 1, 1>), grid, dim3(kBlock), 0, st, a);
  }
}

int launch_pair(const Sys& s, const Ptrs& P, const Shape& sh, int precision, int mode,
                hipStream_t st) {
  PairArgs a;
  a.pk = P.at<void>(P.L.pk);
  a.Ns = (int)(s.N - 1);
  a.jchunk = sh.jchunk;
  a.eps2 = s.eps * s.eps;
  a.part = P.at<double>(P.L.part);
  if (precision == PN_MIXED) {
    if (mode == MODE_FUSED) launch_pair_t<float, MODE_FUSED>(a, sh, st);
    else if (mode == MODE_P1) launch_pair_t<float, MODE_P1>(a, sh, st);
    else launch_pair_t<float, MODE_P2>(a, sh, st);
  } else {
    if (mode == MODE_FUSED) launch_pair_t<double, MODE_FUSED>(a, sh, st);
    else if (mode == MODE_P1) launch_pair_t<double, MODE_P1>(a, sh, st);
    else launch_pair_t<double, MODE_P2>(a, sh, st);
  }
  HIPCK(hipGetLastError());
  return PN_OK;
}

struct Outs {
  double* acc_newton = nullptr;
  double* phi = nullptr;
  double* acc_1pn = nullptr;
  const double* phi_in = nullptr;
  const double* accN_in = nullptr;
  bool newton_only = false;
  int stage = -1;
  double dt = 0.0;
  double *X = nullptr, *V = nullptr, *Xs = nullptr, *Vs = nullptr, *KX = nullptr, *KV = nullptr;
};

int launch_epilogue(const Sys& s, const Ptrs& P, const Shape& sh, const Outs& o, hipStream_t st) {
  const int Ns = (int)(s.N - 1);
  const int nb = (Ns + kBlock - 1) / kBlock;            // prologue workgroups
  const int ne = (Ns + kEpiStars - 1) / kEpiStars;      // epilogue workgroups
  EpiArgs a;
  a.pos = s.pos;
  a.vel = s.vel;
  a.mass = s.mass;
  a.Ns = Ns;
  a.G = s.G;
  a.lam = lambda_of(s.c);
  a.eps2 = s.eps * s.eps;
  a.ub = P.at<double>(P.L.ub);
  a.bpart = P.at<double>(P.L.bpart);
  a.nbpro = nb;
  a.part = P.at<double>(P.L.part);
  a.nsplit = sh.nsplit;
  a.newton_only = o.newton_only ? 1 : 0;
  a.phi_in = o.phi_in;
  a.accN_in = o.accN_in;
  a.acc_newton = o.acc_newton;
  a.phi = o.phi;
  a.acc_1pn = o.acc_1pn;
  a.bhpart = P.at<double>(P.L.bhpart);
  a.nbepi = ne;
  a.status = P.at<int>(P.L.status);
  a.stage = o.stage;
  a.dt = o.dt;
  a.X = o.X;
  a.V = o.V;
  a.Xs = o.Xs;
  a.Vs = o.Vs;
  a.KX = o.KX;
  a.KV = o.KV;
  hipLaunchKernelGGL(k_epilogue, dim3(ne), dim3(kBlock), 0, st, a);
  HIPCK(hipGetLastError());
  hipLaunchKernelGGL(k_bh_final, dim3(1), dim3(kBlock), 0, st, a);
  HIPCK(hipGetLastError());
  return PN_OK;
}

// Optional per-launch timing of the pair kernel (PN_TIMING).
struct Timer {
  DevState* d = nullptr;
  bool on = false;
  size_t used = 0;
  int begin(hipStream_t st) {
    if (!on) return PN_OK;
    while (d->ev.size() < used + 2) {
      hipEvent_t e;
      HIPCK(hipEventCreate(&e));
      d->ev.push_back(e);
    }
    HIPCK(hipEventRecord(d->ev[used], st));
    return PN_OK;
  }
  int end(hipStream_t st) {
    if (!on) return PN_OK;
    HIPCK(hipEventRecord(d->ev[used + 1], st));
    used += 2;
    return PN_OK;
  }
  int collect(double pairs) {
    if (!on) return PN_OK;
    double total = 0.0;
    for (size_t k = 0; k < used; k += 2) {
      float ms = 0.f;
      HIPCK(hipEventSynchronize(d->ev[k + 1]));
      HIPCK(hipEventElapsedTime(&ms, d->ev[k], d->ev[k + 1]));
      total += ms;
    }
    g_timing[0] = (double)(used / 2);
    g_timing[1] = total;
    g_timing[2] = pairs;
    return PN_OK;
  }
};

// One force evaluation (+ optional RK4 stage update).
int enqueue_eval(const Sys& s, const Ptrs& P, const Shape& sh, int precision, const Outs& o,
                 hipStream_t st, Timer* tm) {
  int rc;
  if ((rc = launch_prologue(s, P, precision, st))) return rc;
  if (tm && (rc = tm->begin(st))) return rc;
  if ((rc = launch_pair(s, P, sh, precision, MODE_FUSED, st))) return rc;
  if (tm && (rc = tm->end(st))) return rc;
  return launch_epilogue(s, P, sh, o, st);
}

int enqueue_rk4_step(const Sys& s, const Ptrs& P, const Shape& sh, int precision, double dt,
                     double* X, double* V, hipStream_t st, Timer* tm) {
  double* Xs = P.at<double>(P.L.xs);
  double* Vs = P.at<double>(P.L.vs);
  for (int stage = 0; stage < 4; ++stage) {
    Sys e = s;
    e.pos = stage == 0 ? X : Xs;
    e.vel = stage == 0 ? V : Vs;
    Outs o;
    o.stage = stage;
    o.dt = dt;
    o.X = X;
    o.V = V;
    o.Xs = Xs;
    o.Vs = Vs;
    o.KX = P.at<double>(P.L.kx);
    o.KV = P.at<double>(P.L.kv);
    int rc = enqueue_eval(e, P, sh, precision, o, st, tm);
    if (rc) return rc;
  }
  return PN_OK;
}

int finish(DevState& d, const Ptrs& P, hipStream_t st, int flags) {
  (void)d;
  if (flags & PN_ASYNC) return PN_OK;
  int status = 0;
  HIPCK(hipMemcpyAsync(&status, P.at<int>(P.L.status), sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCK(hipStreamSynchronize(st));
  if (status & 2) {
    snprintf(g_err, sizeof g_err, "mass[0] must be positive and finite");
    return PN_EINVAL;
  }
  if (status & 1) return PN_ENONFINITE;
  return PN_OK;
}

int reset_status(const Ptrs& P, hipStream_t st) {
  hipLaunchKernelGGL(k_reset_status, dim3(1), dim3(64), 0, st, P.at<int>(P.L.status));
  HIPCK(hipGetLastError());
  return PN_OK;
}

hipStream_t pick_stream(DevState& d, void* stream) {
  return stream ? reinterpret_cast<hipStream_t>(stream) : d.own;
}

}  // namespace

// ====================================================================== ABI
extern "C" {

int pn_potential_accel(const double* pos, const double* vel, const double* mass, int64_t N,
                       double G, double c, double eps, double* acc_newton, double* phi,
                       void* stream, int flags) {
  (void)vel;
  int rc = check_system(pos, mass, N, G, c, eps);
  if (rc) return rc;
  if (!dptr_ok(acc_newton) || !dptr_ok(phi)) return PN_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  DevState* d;
  if ((rc = dev_state(&d))) return rc;
  const Shape sh = pick_shape((int)(N - 1), PN_FP64);
  const Layout L = layout_for(N, sh, false);
  if ((rc = ensure_scratch(*d, L.total))) return rc;
  Ptrs P{d->base, L};
  hipStream_t st = pick_stream(*d, stream);
  Sys s{pos, nullptr, mass, N, G, c, eps};
  if ((rc = reset_status(P, st))) return rc;
  if ((rc = launch_prologue(s, P, PN_FP64, st))) return rc;
  if ((rc = launch_pair(s, P, sh, PN_FP64, MODE_P1, st))) return rc;
  Outs o;
  o.acc_newton = acc_newton;
  o.phi = phi;
  o.newton_only = true;
  if ((rc = launch_epilogue(s, P, sh, o, st))) return rc;
  return finish(*d, P, st, flags);
}

int pn_correction(const double* pos, const double* vel, const double* mass, int64_t N, double G,
                  double c, double eps, const double* phi, const double* acc_newton,
                  double* acc_1pn, void* stream, int flags) {
  int rc = check_system(pos, mass, N, G, c, eps);
  if (rc) return rc;
  if (!dptr_ok(vel) || !dptr_ok(phi) || !dptr_ok(acc_newton) || !dptr_ok(acc_1pn)) return PN_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  DevState* d;
  if ((rc = dev_state(&d))) return rc;
  const Shape sh = pick_shape((int)(N - 1), PN_FP64);
  const Layout L = layout_for(N, sh, false);
  if ((rc = ensure_scratch(*d, L.total))) return rc;
  Ptrs P{d->base, L};
  hipStream_t st = pick_stream(*d, stream);
  Sys s{pos, vel, mass, N, G, c, eps};
  if ((rc = reset_status(P, st))) return rc;
  if ((rc = launch_prologue(s, P, PN_FP64, st))) return rc;
  if ((rc = launch_pair(s, P, sh, PN_FP64, MODE_P2, st))) return rc;
  Outs o;
  o.acc_1pn = acc_1pn;
  o.phi_in = phi;
  o.accN_in = acc_newton;
  if ((rc = launch_epilogue(s, P, sh, o, st))) return rc;
  return finish(*d, P, st, flags);
}

int pn_accel(const double* pos, const double* vel, const double* mass, int64_t N, double G,
             double c, double eps, int precision, double* acc_newton, double* phi,
             double* acc_1pn, void* stream, int flags) {
  int rc = check_system(pos, mass, N, G, c, eps);
  if (rc) return rc;
  if (!dptr_ok(vel)) return PN_EINVAL;
  if (precision != PN_FP64 && precision != PN_MIXED) return PN_EINVAL;
  if ((acc_newton && !dptr_ok(acc_newton)) || (phi && !dptr_ok(phi)) ||
      (acc_1pn && !dptr_ok(acc_1pn)))
    return PN_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  DevState* d;
  if ((rc = dev_state(&d))) return rc;
  const Shape sh = pick_shape((int)(N - 1), precision);
  const Layout L = layout_for(N, sh, false);
  if ((rc = ensure_scratch(*d, L.total))) return rc;
  Ptrs P{d->base, L};
  hipStream_t st = pick_stream(*d, stream);
  Sys s{pos, vel, mass, N, G, c, eps};
  Timer tm;
  tm.d = d;
  tm.on = (flags & PN_TIMING) != 0;
  if ((rc = reset_status(P, st))) return rc;
  Outs o;
  o.acc_newton = acc_newton;
  o.phi = phi;
  o.acc_1pn = acc_1pn;
  if ((rc = enqueue_eval(s, P, sh, precision, o, st, &tm))) return rc;
  if ((rc = tm.collect((double)(N - 1) * (double)(N - 2)))) return rc;
  return finish(*d, P, st, flags & ~PN_TIMING);
}

int pn_step(double* pos, double* vel, const double* mass, int64_t N, double G, double c,
            double eps, double dt, int64_t nsteps, int precision, void* stream, int flags) {
  int rc = check_system(pos, mass, N, G, c, eps);
  if (rc) return rc;
  if (!dptr_ok(vel) || !std::isfinite(dt) || nsteps < 0) return PN_EINVAL;
  if (precision != PN_FP64 && precision != PN_MIXED) return PN_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  DevState* d;
  if ((rc = dev_state(&d))) return rc;
  const Shape sh = pick_shape((int)(N - 1), precision);
  const Layout L = layout_for(N, sh, true);
  if ((rc = ensure_scratch(*d, L.total))) return rc;
  Ptrs P{d->base, L};
  hipStream_t st = pick_stream(*d, stream);
  Sys s{pos, vel, mass, N, G, c, eps};
  if ((rc = reset_status(P, st))) return rc;
  const bool timing = (flags & PN_TIMING) != 0;
  const bool graph = !(flags & (PN_NOGRAPH | PN_TIMING));
  if (nsteps > 0) {
    if (!graph) {
      Timer tm;
      tm.d = d;
      tm.on = timing;
      for (int64_t k = 0; k < nsteps; ++k)
        if ((rc = enqueue_rk4_step(s, P, sh, precision, dt, pos, vel, st, &tm))) return rc;
      if ((rc = tm.collect((double)(N - 1) * (double)(N - 2)))) return rc;
    } else {
      GraphKey key;
      key.pos = pos;
      key.vel = vel;
      key.mass = mass;
      key.N = N;
      key.G = G;
      key.c = c;
      key.eps = eps;
      key.dt = dt;
      key.precision = precision;
      key.ipt = sh.ipt;
      key.ws = sh.ws;
      key.nsplit = sh.nsplit;
      key.base = d->base;
      if (!d->gexec || !(key == d->key)) {
        drop_graph(*d);
        // capture on the library's own stream; the graph is launched on `st`
        HIPCK(hipStreamSynchronize(d->own));
        HIPCK(hipStreamBeginCapture(d->own, hipStreamCaptureModeThreadLocal));
        rc = enqueue_rk4_step(s, P, sh, precision, dt, pos, vel, d->own, nullptr);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(d->own, &g);
        if (rc) {
          if (g) hipGraphDestroy(g);
          return rc;
        }
        if (e != hipSuccess) return fail_hip(e, "hipStreamEndCapture", __LINE__);
        d->graph = g;
        HIPCK(hipGraphInstantiate(&d->gexec, d->graph, nullptr, nullptr, 0));
        d->key = key;
      }
      for (int64_t k = 0; k < nsteps; ++k) HIPCK(hipGraphLaunch(d->gexec, st));
    }
  }
  return finish(*d, P, st, flags & ~PN_TIMING);
}

int pn_diagnostics(const double* pos, const double* vel, const double* mass, int64_t N, double G,
                   double c, double eps, double* out8, void* stream, int flags) {
  (void)flags;
  int rc = check_system(pos, mass, N, G, c, eps);
  if (rc) return rc;
  if (!dptr_ok(vel) || out8 == nullptr) return PN_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  DevState* d;
  if ((rc = dev_state(&d))) return rc;
  const Shape sh = pick_shape((int)(N - 1), PN_FP64);
  const Layout L = layout_for(N, sh, false);
  if ((rc = ensure_scratch(*d, L.total))) return rc;
  Ptrs P{d->base, L};
  hipStream_t st = pick_stream(*d, stream);
  Sys s{pos, vel, mass, N, G, c, eps};
  if ((rc = reset_status(P, st))) return rc;
  if ((rc = launch_prologue(s, P, PN_FP64, st))) return rc;
  const int Ns = (int)(N - 1);
  const int nb = (Ns + kBlock - 1) / kBlock;
  DiagPairArgs dp;
  dp.pk = P.at<PkF64>(L.pk);
  dp.Ns = Ns;
  dp.jchunk = sh.jchunk;
  dp.eps2 = eps * eps;
  dp.part = P.at<double>(L.part);
  hipLaunchKernelGGL(k_diag_pair, dim3(nb, sh.nsplit), dim3(kBlock), 0, st, dp);
  HIPCK(hipGetLastError());
  DiagEpiArgs de;
  de.pos = pos;
  de.vel = vel;
  de.mass = mass;
  de.Ns = Ns;
  de.G = G;
  de.lam = lambda_of(c);
  de.eps2 = eps * eps;
  de.ub = P.at<double>(L.ub);
  de.part = P.at<double>(L.part);
  de.nsplit = sh.nsplit;
  de.dpart = P.at<double>(L.dpart);
  de.ndpart = nb;
  de.out8 = P.at<double>(L.out8);
  hipLaunchKernelGGL(k_diag_epi, dim3(nb), dim3(kBlock), 0, st, de);
  HIPCK(hipGetLastError());
  hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(kBlock), 0, st, de);
  HIPCK(hipGetLastError());
  HIPCK(hipMemcpyAsync(out8, P.at<double>(L.out8), 8 * sizeof(double), hipMemcpyDeviceToHost, st));
  return finish(*d, P, st, 0);
}

int pn_step_batched(int32_t n_sys, const int64_t* offsets, const double* G, const double* c,
                    const double* eps, double* pos, double* vel, const double* mass, double dt,
                    int64_t nsteps, int precision, void* stream, int flags) {
  if (n_sys < 1 || !offsets || !G || !c || !eps) return PN_EINVAL;
  if (offsets[0] != 0) return PN_EINVAL;
  for (int b = 0; b < n_sys; ++b) {
    if (offsets[b + 1] - offsets[b] < 2) return PN_EINVAL;
    int rc = check_system(pos, mass, offsets[b + 1] - offsets[b], G[b], c[b], eps[b]);
    if (rc) return rc;
  }
  for (int b = 0; b < n_sys; ++b) {
    const int64_t o = offsets[b];
    int rc = pn_step(pos + 3 * o, vel + 3 * o, mass + o, offsets[b + 1] - o, G[b], c[b], eps[b],
                     dt, nsteps, precision, stream, flags | PN_ASYNC | PN_NOGRAPH);
    if (rc) return rc;
  }
  if (flags & PN_ASYNC) return PN_OK;
  std::lock_guard<std::mutex> lk(g_mu);
  DevState* d;
  int rc = dev_state(&d);
  if (rc) return rc;
  HIPCK(hipStreamSynchronize(pick_stream(*d, stream)));
  return PN_OK;
}

int pn_set_shape(int precision, int64_t n_min, int64_t n_max, int ipt, int ws, int nsplit) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (precision < 0) {
    g_tuned.clear();
    return PN_OK;
  }
  if ((precision != PN_FP64 && precision != PN_MIXED) || n_min < 2 || n_max < n_min ||
      (ipt != 1 && ipt != 2) || (ws != 1 && ws != 4) || nsplit < 0 || nsplit > 65535)
    return PN_EINVAL;
  g_tuned.push_back(TunedShape{precision, n_min, n_max, ipt, ws, nsplit});
  return PN_OK;
}

const char* pn_strerror(int code) {
  switch (code) {
    case PN_OK: return "ok";
    case PN_EINVAL: return "invalid argument";
    case PN_ENONFINITE: return "non-finite acceleration produced";
    case PN_EDEVICE: return g_err;
    case PN_ENOMEM: return "device allocation failed";
    default: return "unknown error code";
  }
}

int pn_last_timing(double* out) {
  if (!out) return PN_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  out[0] = g_timing[0];
  out[1] = g_timing[1];
  out[2] = g_timing[2];
  return PN_OK;
}

int pn_release(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess) {
    g_dev.clear();
    return PN_OK;
  }
  for (size_t dev = 0; dev < g_dev.size(); ++dev) {
    DevState& d = g_dev[dev];
    if (!d.init) continue;
    (void)hipSetDevice((int)dev);
    (void)hipDeviceSynchronize();
    drop_graph(d);
    for (hipEvent_t e : d.ev) (void)hipEventDestroy(e);
    d.ev.clear();
    if (d.base) (void)hipFree(d.base);
    d.base = nullptr;
    d.cap = 0;
    if (d.own) (void)hipStreamDestroy(d.own);
    d.own = nullptr;
    d.init = false;
  }
  (void)hipSetDevice(cur);
  return PN_OK;
}

}  // extern "C"
