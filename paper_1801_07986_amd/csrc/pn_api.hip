// pn_api.hip -- host side of libpn: the extern "C" entry points declared in
// include/pn.h, argument validation, per-device scratch, launch shapes and
// the HIP graphs that replay time steps.
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
// detail of this thread's last PN_EINVAL that has one ("" if none); per
// thread because argument checks run before the library lock is taken
thread_local char g_inval[256] = "";
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

int fail_inval(const char* what) {
  snprintf(g_inval, sizeof g_inval, "%s", what);
  return PN_EINVAL;
}

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
    if (sscanf(env, "%d,%d,%d", &a, &b, &c) == 3 && (a == 1 || a == 2) &&
        (b == 1 || b == 4 || b == 8) && c >= 0) {
      s.ipt = a;
      s.ws = b;
      want_nsplit = c;
    }
  }
  const int ib = (s.ws == 1 ? kBlock : 64) * s.ipt;  // i-bodies per workgroup
  s.iblocks = (Ns + ib - 1) / ib;
  if (want_nsplit <= 0) {
    // default: about 4096 sweep workgroups, but at least 16 j per wavefront
    want_nsplit = std::max(16, (4096 + s.iblocks - 1) / s.iblocks);
    want_nsplit = std::min(want_nsplit, std::max(1, Ns / (16 * s.ws)));
  }
  want_nsplit = std::max(1, std::min(want_nsplit, Ns));
  s.jchunk = (Ns + want_nsplit - 1) / want_nsplit;
  s.nsplit = (Ns + s.jchunk - 1) / s.jchunk;
  return s;
}

// The same shape with (at most) `want` j-splits.
Shape with_splits(Shape s, int Ns, int want) {
  want = std::max(1, std::min(want, Ns));
  s.jchunk = (Ns + want - 1) / want;
  s.nsplit = (Ns + s.jchunk - 1) / s.jchunk;
  return s;
}

// One-launch Runge-Kutta stages (k_stage) for small systems: entries
// (precision, n_min <= N <= n_max, stars per workgroup) installed with
// pn_set_stage_kernel (the autotuner's table); no matching entry: the chained
// two-kernel stages.  PN_STAGE_NS=ns overrides it for every size (tuning
// runs; 0 turns it off).
struct StageSel {
  int precision;
  int64_t n_min, n_max;
  int ns;
};
std::vector<StageSel> g_stage;
bool stage_ns_ok(int ns) { return ns == 2 || ns == 4 || ns == 8 || ns == 16; }
int pick_stage_ns(int64_t N, int precision) {
  if (const char* env = getenv("PN_STAGE_NS")) {
    const int v = atoi(env);
    return stage_ns_ok(v) ? v : 0;
  }
  for (const StageSel& t : g_stage)
    if (t.precision == precision && N >= t.n_min && N <= t.n_max) return t.ns;
  return 0;
}

// ------------------------------------------------------------------ scratch
size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
  size_t pk, ub, bpart, ub2, bpart2, bhpart2, part, bhpart, status, xs, vs, kx, kv, dpart, out8, ha, hj, xp, vp, ap,
      pk2, bpart3, bpart4, bhs, total;
};

// What a call needs beyond one force evaluation: the RK4 stage arrays, or the
// jerk sweep's wider packets and partials (dual numbers), or those and the
// Hermite state.
enum class Need { EVAL, RK4, JERK, HERMITE };

// stage_ns > 0 (RK4 only): the one-launch stages' extra buffers (k_stage:
// a second packet buffer, four block-row buffers of a row per stage_ns stars,
// two massive-object row buffers and two copies of its state).
Layout layout_for(int64_t N, const Shape& s, Need need, int stage_ns = 0) {
  const bool rk4 = need == Need::RK4;
  const bool dual = need == Need::JERK || need == Need::HERMITE;
  const bool herm = need == Need::HERMITE;
  const size_t W = dual ? 2 : 1;
  const size_t Ns = (size_t)(N - 1);
  const size_t nb = (Ns + kBlock - 1) / kBlock;
  Layout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += align256(bytes);
    return at;
  };
  // massive-object block rows: one per 64 stars (kProRows per prologue
  // workgroup, one per epilogue workgroup).  Runge-Kutta steps chain their
  // evaluations: each stage's epilogue writes the next stage's u/b rows and
  // block rows into the other of two buffers; a jerk evaluation's FP64
  // epilogue writes the jerk sweep's (dual) rows into the second buffers.
  const bool fused = rk4 && stage_ns > 0;
  const size_t nbf = fused ? (Ns + stage_ns - 1) / stage_ns : 0;  // k_stage workgroups = rows
  const size_t nrows = std::max(nb * kProRows, nbf);
  const size_t nepi = std::max((Ns + kEpiStars - 1) / kEpiStars, nbf);
  L.pk = take(Ns * (dual ? sizeof(PkDual) : sizeof(PkF64)));
  L.ub = take(Ns * 4 * W * sizeof(double));
  L.bpart = take(nrows * 8 * W * sizeof(double));
  L.ub2 = take(rk4 || dual ? Ns * 4 * W * sizeof(double) : 0);
  L.bpart2 = take(rk4 || dual ? nrows * 8 * W * sizeof(double) : 0);
  L.part = take((size_t)s.nsplit * std::max<size_t>(kNF * W, kND) * Ns * sizeof(double));
  L.bhpart = take(nepi * 4 * W * sizeof(double));
  L.bhpart2 = take(dual || fused ? nepi * 4 * W * sizeof(double) : 0);
  L.pk2 = take(fused ? Ns * sizeof(PkF64) : 0);
  L.bpart3 = take(fused ? nbf * 8 * sizeof(double) : 0);
  L.bpart4 = take(fused ? nbf * 8 * sizeof(double) : 0);
  L.bhs = take(fused ? 36 * sizeof(double) : 0);
  L.status = take(sizeof(int));
  L.dpart = take(nb * 10 * sizeof(double));
  L.out8 = take(8 * sizeof(double));
  const size_t n3 = 3 * (size_t)N * sizeof(double);
  L.xs = take(rk4 ? n3 : 0);
  L.vs = take(rk4 ? n3 : 0);
  L.kx = take(rk4 ? n3 : 0);
  L.kv = take(rk4 ? n3 : 0);
  L.ha = take(herm ? n3 : 0);
  L.hj = take(herm ? n3 : 0);
  L.xp = take(herm ? n3 : 0);
  L.vp = take(herm ? n3 : 0);
  L.ap = take(herm ? n3 : 0);
  L.total = o;
  return L;
}

// Scratch of pn_accel_noalloc: a file-scope device array, which the code
// object loader places on every device the library runs on (held until the
// process ends).  On the host the array's name is only a stand-in and is never
// handed to a kernel or a copy: host code uses the device address that
// hipGetSymbolAddress returns for the current device (DevState::fixed), looked
// up once when the library first sets up that device.
constexpr size_t kFixedScratchBytes = (size_t)64 << 20;
__device__ __align__(256) char scratch[kFixedScratchBytes];

struct GraphKey {
  const void *pos = nullptr, *vel = nullptr, *mass = nullptr;
  int64_t N = 0;
  double G = 0, c = 0, eps = 0, dt = 0;
  int precision = -1, ipt = 0, ws = 0, nsplit = 0;
  int stage_ns = 0;  // one-launch stages (k_stage): stars per workgroup
  int scheme = 0;  // 0: Runge-Kutta step, 1: Hermite step
  char* base = nullptr;
  bool operator==(const GraphKey& o) const {
    return scheme == o.scheme && pos == o.pos && vel == o.vel && mass == o.mass && N == o.N && G == o.G &&
           (c == o.c || (std::isinf(c) && std::isinf(o.c))) && eps == o.eps && dt == o.dt &&
           precision == o.precision && ipt == o.ipt && ws == o.ws && nsplit == o.nsplit &&
           stage_ns == o.stage_ns && base == o.base;
  }
};

struct BatchKey {
  std::vector<int64_t> offsets;
  std::vector<double> G, c, eps;
  const void *pos = nullptr, *vel = nullptr, *mass = nullptr;
  double dt = 0;
  int precision = -1;
  int ipt = 0, splits = 0;  // the plan's shape: i per lane, common split count
  char* base = nullptr;
  bool operator==(const BatchKey& o) const {
    return offsets == o.offsets && G == o.G && c == o.c && eps == o.eps && pos == o.pos &&
           vel == o.vel && mass == o.mass && dt == o.dt && precision == o.precision &&
           ipt == o.ipt && splits == o.splits && base == o.base;
  }
};

struct DevState {
  bool init = false;
  hipStream_t own = nullptr;
  char* base = nullptr;
  size_t cap = 0;
  char* fixed = nullptr;  // this device's copy of `scratch` (pn_accel_noalloc)
  hipGraph_t graph = nullptr;      // one time step
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph_k = nullptr;    // kStepsPerGraph time steps
  hipGraphExec_t gexec_k = nullptr;
  GraphKey key;  // the system both graphs were captured for
  std::vector<hipEvent_t> ev;
  // batched ensembles: own scratch and step graph
  char* bbase = nullptr;
  size_t bcap = 0;
  hipGraph_t bgraph = nullptr;
  hipGraphExec_t bgexec = nullptr;
  BatchKey bkey;   // ensemble the cached graph was captured for
  BatchKey bdesc;  // ensemble whose descriptors are in the batched scratch now
  bool bdesc_valid = false;
  // every call's device work shares the scratch above: a call on another
  // stream than the previous one waits for it (last_ev recorded on last_st)
  hipEvent_t last_ev = nullptr;
  hipStream_t last_st = nullptr;
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
    void* fixed = nullptr;
    HIPCK(hipGetSymbolAddress(&fixed, HIP_SYMBOL(scratch)));
    d.fixed = static_cast<char*>(fixed);
    d.init = true;
  }
  *out = &d;
  return PN_OK;
}

void drop_graph(DevState& d) {
  if (d.gexec) (void)hipGraphExecDestroy(d.gexec);
  if (d.graph) (void)hipGraphDestroy(d.graph);
  if (d.gexec_k) (void)hipGraphExecDestroy(d.gexec_k);
  if (d.graph_k) (void)hipGraphDestroy(d.graph_k);
  d.gexec = nullptr;
  d.graph = nullptr;
  d.gexec_k = nullptr;
  d.graph_k = nullptr;
  d.key = GraphKey();
}

void drop_batch_graph(DevState& d) {
  if (d.bgexec) (void)hipGraphExecDestroy(d.bgexec);
  if (d.bgraph) (void)hipGraphDestroy(d.bgraph);
  d.bgexec = nullptr;
  d.bgraph = nullptr;
  d.bkey = BatchKey();
}

int ensure_batch_scratch(DevState& d, size_t bytes) {
  if (bytes <= d.bcap) return PN_OK;
  HIPCK(hipDeviceSynchronize());
  drop_batch_graph(d);
  d.bdesc_valid = false;
  if (d.bbase) HIPCK(hipFree(d.bbase));
  d.bbase = nullptr;
  d.bcap = 0;
  hipError_t e = hipMalloc(&d.bbase, bytes);
  if (e != hipSuccess) return fail_hip(e, "hipMalloc(batched scratch)", __LINE__);
  d.bcap = bytes;
  return PN_OK;
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
  g_inval[0] = '\0';
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

// precision PN_FP64 / PN_MIXED; dual: the jerk sweep's packets, with the
// derivatives pos_d (velocities) and vel_d (accelerations).
int launch_prologue(const Sys& s, const Ptrs& P, int precision, hipStream_t st,
                    bool dual = false, const double* pos_d = nullptr,
                    const double* vel_d = nullptr) {
  const int Ns = (int)(s.N - 1);
  ProArgs a;
  a.pos_d = pos_d;
  a.vel_d = vel_d;
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
  if (dual)
    hipLaunchKernelGGL(k_prologue<Dual>, dim3(nb), dim3(kBlock), 0, st, a);
  else if (precision == PN_MIXED)
    hipLaunchKernelGGL(k_prologue<float>, dim3(nb), dim3(kBlock), 0, st, a);
  else
    hipLaunchKernelGGL(k_prologue<double>, dim3(nb), dim3(kBlock), 0, st, a);
  HIPCK(hipGetLastError());
  return PN_OK;
}

template <typename T, int MODE>
void launch_pair_t(const PairArgs& a, const Shape& sh, hipStream_t st) {
  dim3 grid(sh.iblocks, sh.nsplit);
  if (sh.ws == 8) {
    if (sh.ipt == 2)
      hipLaunchKernelGGL((k_pair<T, MODE, 2, 8>), grid, dim3(2 * kBlock), 0, st, a);
    else
      hipLaunchKernelGGL((k_pair<T, MODE, 1, 8>), grid, dim3(2 * kBlock), 0, st, a);
  } else if (sh.ws == 4) {
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

// The jerk sweep: FP64 dual numbers, one i per lane, four wavefronts per
// i-range, the j-splits of the evaluation's shape.
int launch_pair_dual(const Sys& s, const Ptrs& P, const Shape& sh, hipStream_t st) {
  PairArgs a;
  a.pk = P.at<void>(P.L.pk);
  a.Ns = (int)(s.N - 1);
  a.jchunk = sh.jchunk;
  a.eps2 = s.eps * s.eps;
  a.part = P.at<double>(P.L.part);
  const int iblocks = (a.Ns + 63) / 64;
  hipLaunchKernelGGL((k_pair<Dual, MODE_FUSED, 1, 4>), dim3(iblocks, sh.nsplit), dim3(kBlock), 0,
                     st, a);
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
  double* acc_tot = nullptr;
  // jerk evaluation (dual): derivatives of the state, jerk output, Hermite update
  bool dual = false;
  const double* pos_d = nullptr;
  const double* vel_d = nullptr;
  double* jerk = nullptr;
  int herm = -1;
  double *HA = nullptr, *HJ = nullptr, *XP = nullptr, *VP = nullptr;
  // chained Runge-Kutta stage: reads u/b and block rows from buffer `chain`
  // (0 or 1), writes the next stage's packets (of `precision`) and rows into
  // the other; -1: not chained
  int chain = -1;
  int precision = PN_FP64;
  // jerk evaluation: the FP64 epilogue writes the jerk sweep's packets and
  // (dual) rows into the second buffers (jerk_next), which the dual epilogue
  // then reads, writing its own massive-object rows there too (second_rows);
  // fp64_bh: the FP64 pass's massive-object update, run by the dual epilogue
  bool jerk_next = false;
  bool second_rows = false;
  const EpiArgs* fp64_bh = nullptr;
};

EpiArgs epi_args(const Sys& s, const Ptrs& P, const Shape& sh, const Outs& o) {
  const int Ns = (int)(s.N - 1);
  const int ne = (Ns + kEpiStars - 1) / kEpiStars;  // epilogue workgroups = prologue rows
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
  a.nbpro = ne;
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
  a.acc_tot = o.acc_tot;
  a.pos_d = o.pos_d;
  a.vel_d = o.vel_d;
  a.jerk = o.jerk;
  a.herm = o.herm;
  a.HA = o.HA;
  a.HJ = o.HJ;
  a.XP = o.XP;
  a.VP = o.VP;
  if (o.chain >= 0) {
    double* ubs[2] = {P.at<double>(P.L.ub), P.at<double>(P.L.ub2)};
    double* bps[2] = {P.at<double>(P.L.bpart), P.at<double>(P.L.bpart2)};
    a.ub = ubs[o.chain];
    a.bpart = bps[o.chain];
    a.pk_next = P.at<void>(P.L.pk);
    a.ub_next = ubs[1 - o.chain];
    a.bpart_next = bps[1 - o.chain];
  }
  if (o.jerk_next) {
    a.pk_next = P.at<void>(P.L.pk);
    a.ub_next = P.at<double>(P.L.ub2);
    a.bpart_next = P.at<double>(P.L.bpart2);
  }
  if (o.second_rows) {
    a.ub = P.at<double>(P.L.ub2);
    a.bpart = P.at<double>(P.L.bpart2);
    a.bhpart = P.at<double>(P.L.bhpart2);
  }
  return a;
}

// Epilogue and massive-object update of one evaluation.  A chained stage
// (o.chain >= 0) or a jerk evaluation's FP64 pass (o.jerk_next) launches the
// epilogue only: its massive-object update rides on the next sweep
// (launch_pair_bh, launch_pair_dual) or follows alone (launch_bh_final).
int launch_epilogue(const Sys& s, const Ptrs& P, const Shape& sh, const Outs& o, hipStream_t st) {
  const int Ns = (int)(s.N - 1);
  const int ne = (Ns + kEpiStars - 1) / kEpiStars;
  const EpiArgs a = epi_args(s, P, sh, o);
  if (o.jerk_next) {
    hipLaunchKernelGGL(k_epilogue_chain<Dual>, dim3(ne), dim3(kBlock), 0, st, a);
  } else if (o.chain >= 0) {
    if (o.precision == PN_MIXED)
      hipLaunchKernelGGL(k_epilogue_chain<float>, dim3(ne), dim3(kBlock), 0, st, a);
    else
      hipLaunchKernelGGL(k_epilogue_chain<double>, dim3(ne), dim3(kBlock), 0, st, a);
  } else if (o.dual && o.fp64_bh) {
    hipLaunchKernelGGL(k_epilogue_dual_bh, dim3(ne + 1), dim3(kBlock), 0, st, a, *o.fp64_bh);
    HIPCK(hipGetLastError());
    hipLaunchKernelGGL(k_bh_final<Dual>, dim3(1), dim3(kBlock), 0, st, a);
  } else if (o.dual) {
    hipLaunchKernelGGL(k_epilogue<Dual>, dim3(ne), dim3(kBlock), 0, st, a);
    HIPCK(hipGetLastError());
    hipLaunchKernelGGL(k_bh_final<Dual>, dim3(1), dim3(kBlock), 0, st, a);
  } else {
    hipLaunchKernelGGL(k_epilogue<double>, dim3(ne), dim3(kBlock), 0, st, a);
    HIPCK(hipGetLastError());
    hipLaunchKernelGGL(k_bh_final<double>, dim3(1), dim3(kBlock), 0, st, a);
  }
  HIPCK(hipGetLastError());
  return PN_OK;
}

int launch_bh_final(const EpiArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_bh_final<double>, dim3(1), dim3(kBlock), 0, st, a);
  HIPCK(hipGetLastError());
  return PN_OK;
}

template <typename T>
void launch_pair_bh_t(const PairArgs& a, const EpiArgs& e, const Shape& sh, hipStream_t st) {
  dim3 grid(sh.iblocks + 1, sh.nsplit);
  if (sh.ws == 8) {
    if (sh.ipt == 2)
      hipLaunchKernelGGL((k_pair_bh<T, MODE_FUSED, 2, 8>), grid, dim3(2 * kBlock), 0, st, a, e);
    else
      hipLaunchKernelGGL((k_pair_bh<T, MODE_FUSED, 1, 8>), grid, dim3(2 * kBlock), 0, st, a, e);
  } else if (sh.ws == 4) {
    if (sh.ipt == 2)
      hipLaunchKernelGGL((k_pair_bh<T, MODE_FUSED, 2, 4>), grid, dim3(kBlock), 0, st, a, e);
    else
      hipLaunchKernelGGL((k_pair_bh<T, MODE_FUSED, 1, 4>), grid, dim3(kBlock), 0, st, a, e);
  } else {
    if (sh.ipt == 2)
      hipLaunchKernelGGL((k_pair_bh<T, MODE_FUSED, 2, 1>), grid, dim3(kBlock), 0, st, a, e);
    else
      hipLaunchKernelGGL((k_pair_bh<T, MODE_FUSED, 1, 1>), grid, dim3(kBlock), 0, st, a, e);
  }
}

// The fused sweep of the state s with, in one extra workgroup, the
// massive-object update e of the previous chained stage.
int launch_pair_bh(const Sys& s, const Ptrs& P, const Shape& sh, int precision, const EpiArgs& e,
                   hipStream_t st) {
  PairArgs a;
  a.pk = P.at<void>(P.L.pk);
  a.Ns = (int)(s.N - 1);
  a.jchunk = sh.jchunk;
  a.eps2 = s.eps * s.eps;
  a.part = P.at<double>(P.L.part);
  if (precision == PN_MIXED) launch_pair_bh_t<float>(a, e, sh, st);
  else launch_pair_bh_t<double>(a, e, sh, st);
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

// Chained RK4 steps.  Stage k of a step evaluates at (X, V) (k = 0) or
// (Xs, Vs); its epilogue (k_epilogue_chain) reads the u/b and block rows of
// buffer k % 2 and writes the next stage's packets and rows (stage 3: the next
// step's stage 0, buffer 0 again) into the other; its massive-object update
// runs in an extra workgroup of the next stage's sweep (k_pair_bh).  So a run
// of steps is: prologue at (X, V), the first sweep (enqueue_rk4_head), then
// per step enqueue_rk4_body, whose last update rides on the next step's first
// sweep (more) or runs alone after the last step.
void rk4_stage(const Sys& s, const Ptrs& P, int precision, double dt, double* X, double* V,
               int stage, Sys& e, Outs& o) {
  double* Xs = P.at<double>(P.L.xs);
  double* Vs = P.at<double>(P.L.vs);
  e = s;
  e.pos = stage == 0 ? X : Xs;
  e.vel = stage == 0 ? V : Vs;
  o = Outs();
  o.stage = stage;
  o.dt = dt;
  o.X = X;
  o.V = V;
  o.Xs = Xs;
  o.Vs = Vs;
  o.KX = P.at<double>(P.L.kx);
  o.KV = P.at<double>(P.L.kv);
  o.chain = stage & 1;
  o.precision = precision;
}

int enqueue_rk4_head(const Sys& s, const Ptrs& P, const Shape& sh, int precision, double dt,
                     double* X, double* V, hipStream_t st, Timer* tm) {
  Sys e;
  Outs o;
  rk4_stage(s, P, precision, dt, X, V, 0, e, o);
  int rc;
  if (tm && (rc = tm->begin(st))) return rc;
  if ((rc = launch_pair(e, P, sh, precision, MODE_FUSED, st))) return rc;
  if (tm && (rc = tm->end(st))) return rc;
  return PN_OK;
}

int enqueue_rk4_body(const Sys& s, const Ptrs& P, const Shape& sh, int precision, double dt,
                     double* X, double* V, bool more, hipStream_t st, Timer* tm) {
  for (int stage = 0; stage < 4; ++stage) {
    Sys e, en;
    Outs o, on;
    rk4_stage(s, P, precision, dt, X, V, stage, e, o);
    int rc;
    if ((rc = launch_epilogue(e, P, sh, o, st))) return rc;
    const EpiArgs a = epi_args(e, P, sh, o);
    if (stage < 3 || more) {
      rk4_stage(s, P, precision, dt, X, V, (stage + 1) & 3, en, on);
      if (tm && (rc = tm->begin(st))) return rc;
      if ((rc = launch_pair_bh(en, P, sh, precision, a, st))) return rc;
      if (tm && (rc = tm->end(st))) return rc;
    } else if ((rc = launch_bh_final(a, st))) {
      return rc;
    }
  }
  return PN_OK;
}

// One-launch Runge-Kutta stages (k_stage, small systems).  Buffers of stage k:
// packets and u/b rows k % 2, block rows k % 4, massive-object 1PN rows
// k % 2, massive-object state read from copy k % 2 and written to the other.
struct StageBufs {
  void* pk[2];
  double* ub[2];
  double* bpart[4];
  double* bhpart[2];
  double* bhs[2];
  int nb;  // workgroups = rows per row buffer
};
StageBufs stage_bufs(const Ptrs& P, int64_t N, int ns) {
  StageBufs b;
  b.pk[0] = P.at<void>(P.L.pk);
  b.pk[1] = P.at<void>(P.L.pk2);
  b.ub[0] = P.at<double>(P.L.ub);
  b.ub[1] = P.at<double>(P.L.ub2);
  b.bpart[0] = P.at<double>(P.L.bpart);
  b.bpart[1] = P.at<double>(P.L.bpart2);
  b.bpart[2] = P.at<double>(P.L.bpart3);
  b.bpart[3] = P.at<double>(P.L.bpart4);
  b.bhpart[0] = P.at<double>(P.L.bhpart);
  b.bhpart[1] = P.at<double>(P.L.bhpart2);
  b.bhs[0] = P.at<double>(P.L.bhs);
  b.bhs[1] = b.bhs[0] + 18;
  b.nb = (int)((N - 1 + ns - 1) / ns);
  return b;
}

template <typename T, int NS>
void launch_stage_t(const StageArgs& sa, int grid, hipStream_t st) {
  hipLaunchKernelGGL((k_stage<T, NS>), dim3(grid), dim3(kBlock), 0, st, sa);
}
template <typename T>
int launch_stage_ns(const StageArgs& sa, int grid, int ns, hipStream_t st) {
  switch (ns) {
    case 2: launch_stage_t<T, 2>(sa, grid, st); break;
    case 4: launch_stage_t<T, 4>(sa, grid, st); break;
    case 8: launch_stage_t<T, 8>(sa, grid, st); break;
    case 16: launch_stage_t<T, 16>(sa, grid, st); break;
    default: return fail_inval("stars per workgroup of the stage kernel: 2, 4, 8 or 16");
  }
  HIPCK(hipGetLastError());
  return PN_OK;
}

// Stage `stage` of a step (mode kStageFirst / kStageFull), or the last
// pending update (kStageFinal, with stage 0: it reads what stage 0 would).
int launch_stage(const Sys& s, const Ptrs& P, const Shape& sh, int precision, double dt,
                 double* X, double* V, int stage, int mode, int ns, hipStream_t st) {
  Sys e;
  Outs o;
  rk4_stage(s, P, precision, dt, X, V, stage, e, o);
  EpiArgs a = epi_args(e, P, sh, o);
  const StageBufs b = stage_bufs(P, s.N, ns);
  a.ub = b.ub[stage & 1];
  a.bpart = b.bpart[stage];
  a.nbpro = b.nb;
  a.bhpart = b.bhpart[stage & 1];
  a.nbepi = b.nb;
  a.pk_next = b.pk[(stage + 1) & 1];
  a.ub_next = b.ub[(stage + 1) & 1];
  a.bpart_next = b.bpart[(stage + 1) & 3];
  StageArgs sa;
  sa.e = a;
  sa.pk = b.pk[stage & 1];
  sa.mode = mode;
  sa.pstage = (stage + 3) & 3;
  sa.prow = b.bpart[(stage + 3) & 3];
  sa.phrow = b.bhpart[((stage + 3) & 3) & 1];
  sa.bhs_in = b.bhs[stage & 1];
  sa.bhs_out = b.bhs[(stage + 1) & 1];
  const int grid = mode == kStageFinal ? 1 : b.nb;
  return precision == PN_MIXED ? launch_stage_ns<float>(sa, grid, ns, st)
                               : launch_stage_ns<double>(sa, grid, ns, st);
}

// A call's first packets and rows in the stage kernel's layout.
template <typename T>
int launch_stage_head_t(const EpiArgs& a, int grid, int ns, hipStream_t st) {
  switch (ns) {
    case 2: hipLaunchKernelGGL((k_stage_head<T, 2>), dim3(grid), dim3(kBlock), 0, st, a); break;
    case 4: hipLaunchKernelGGL((k_stage_head<T, 4>), dim3(grid), dim3(kBlock), 0, st, a); break;
    case 8: hipLaunchKernelGGL((k_stage_head<T, 8>), dim3(grid), dim3(kBlock), 0, st, a); break;
    case 16: hipLaunchKernelGGL((k_stage_head<T, 16>), dim3(grid), dim3(kBlock), 0, st, a); break;
    default: return fail_inval("stars per workgroup of the stage kernel: 2, 4, 8 or 16");
  }
  HIPCK(hipGetLastError());
  return PN_OK;
}
int launch_stage_head(const Sys& s, const Ptrs& P, const Shape& sh, int precision, int ns,
                      hipStream_t st) {
  Outs o;
  EpiArgs a = epi_args(s, P, sh, o);
  const StageBufs b = stage_bufs(P, s.N, ns);
  a.pk_next = b.pk[0];
  a.ub_next = b.ub[0];
  a.bpart_next = b.bpart[0];
  return precision == PN_MIXED ? launch_stage_head_t<float>(a, b.nb, ns, st)
                               : launch_stage_head_t<double>(a, b.nb, ns, st);
}

// The four stages of one step; the first step of a call starts without a
// pending update.
int enqueue_stage_step(const Sys& s, const Ptrs& P, const Shape& sh, int precision, double dt,
                       double* X, double* V, int ns, bool first, hipStream_t st, Timer* tm) {
  for (int stage = 0; stage < 4; ++stage) {
    int rc;
    if (tm && (rc = tm->begin(st))) return rc;
    rc = launch_stage(s, P, sh, precision, dt, X, V, stage,
                      first && stage == 0 ? kStageFirst : kStageFull, ns, st);
    if (rc) return rc;
    if (tm && (rc = tm->end(st))) return rc;
  }
  return PN_OK;
}

// Acceleration and jerk at the state s: an FP64 evaluation writes the total
// acceleration to acc, then the dual sweep differentiates the force along
// (dx/dt, dv/dt) = (v, acc).  o carries the dual pass's outputs.
// Six kernels: prologue, FP64 sweep, FP64 epilogue that also writes the jerk
// sweep's packets and rows (second buffers), the jerk sweep, the dual
// epilogue carrying the FP64 massive-object update, the dual massive-object
// update.
int enqueue_jerk(const Sys& s, const Ptrs& P, const Shape& sh, double* acc, Outs o,
                 hipStream_t st) {
  Outs e;
  e.acc_tot = acc;
  e.jerk_next = true;
  int rc;
  if ((rc = launch_prologue(s, P, PN_FP64, st))) return rc;
  if ((rc = launch_pair(s, P, sh, PN_FP64, MODE_FUSED, st))) return rc;
  if ((rc = launch_epilogue(s, P, sh, e, st))) return rc;
  if ((rc = launch_pair_dual(s, P, sh, st))) return rc;
  const EpiArgs fp64 = epi_args(s, P, sh, e);
  o.dual = true;
  o.pos_d = s.vel;
  o.vel_d = acc;
  o.second_rows = true;
  o.fp64_bh = &fp64;
  return launch_epilogue(s, P, sh, o, st);
}

Outs hermite_outs(const Ptrs& P, double dt, double* X, double* V, int herm) {
  Outs o;
  o.herm = herm;
  o.dt = dt;
  o.X = X;
  o.V = V;
  o.HA = P.at<double>(P.L.ha);
  o.HJ = P.at<double>(P.L.hj);
  o.XP = P.at<double>(P.L.xp);
  o.VP = P.at<double>(P.L.vp);
  return o;
}

// First Hermite evaluation: acceleration and jerk at (X, V), first prediction.
int enqueue_hermite_start(const Sys& s, const Ptrs& P, const Shape& sh, double dt, double* X,
                          double* V, hipStream_t st) {
  Sys e = s;
  e.pos = X;
  e.vel = V;
  return enqueue_jerk(e, P, sh, P.at<double>(P.L.ap), hermite_outs(P, dt, X, V, 0), st);
}

// One Hermite step: evaluate at the prediction (XP, VP), correct (X, V) and
// predict the next state.
int enqueue_hermite_step(const Sys& s, const Ptrs& P, const Shape& sh, double dt, double* X,
                         double* V, hipStream_t st) {
  Sys e = s;
  e.pos = P.at<double>(P.L.xp);
  e.vel = P.at<double>(P.L.vp);
  return enqueue_jerk(e, P, sh, P.at<double>(P.L.ap), hermite_outs(P, dt, X, V, 1), st);
}

// Calls share the per-device scratch, so device work of a call must not
// overlap the previous call's.  On one stream that is stream order; on a
// different stream the new call first waits for the previous call's event.
int order_after_previous(DevState& d, hipStream_t st) {
  if (d.last_ev && d.last_st != st) HIPCK(hipStreamWaitEvent(st, d.last_ev, 0));
  return PN_OK;
}

int mark_call_end(DevState& d, hipStream_t st) {
  if (!d.last_ev) HIPCK(hipEventCreateWithFlags(&d.last_ev, hipEventDisableTiming));
  HIPCK(hipEventRecord(d.last_ev, st));
  d.last_st = st;
  return PN_OK;
}

// Waits for st and reports the device status word of the call.
int read_status(const Ptrs& P, hipStream_t st) {
  int status = 0;
  HIPCK(hipMemcpyAsync(&status, P.at<int>(P.L.status), sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCK(hipStreamSynchronize(st));
  if (status & 2) return fail_inval("mass[0] must be positive and finite");
  if (status & 1) return PN_ENONFINITE;
  return PN_OK;
}

int finish(DevState& d, const Ptrs& P, hipStream_t st, int flags) {
  int rc = mark_call_end(d, st);
  if (rc) return rc;
  if (flags & PN_ASYNC) return PN_OK;
  return read_status(P, st);
}

int reset_status(const Ptrs& P, hipStream_t st) {
  hipLaunchKernelGGL(k_reset_status, dim3(1), dim3(64), 0, st, P.at<int>(P.L.status));
  HIPCK(hipGetLastError());
  return PN_OK;
}

hipStream_t pick_stream(DevState& d, void* stream) {
  return stream ? reinterpret_cast<hipStream_t>(stream) : d.own;
}


// Time steps per replay of the long graph.  Consecutive graph launches are
// separated by several microseconds more than kernels within one graph (at
// N = 1024 about 6.5 against 1.1-1.7 us, against a step of about 60 us), so
// long runs replay kStepsPerGraph steps per launch.
constexpr int kStepsPerGraph = 16;

// Captures `steps` time steps (on the library's own stream) into *graph/*exec.
template <typename Enqueue>
int capture_steps(DevState& d, int steps, Enqueue& enqueue_step, hipGraph_t* graph,
                  hipGraphExec_t* exec) {
  HIPCK(hipStreamSynchronize(d.own));
  HIPCK(hipStreamBeginCapture(d.own, hipStreamCaptureModeThreadLocal));
  int rc = PN_OK;
  for (int k = 0; k < steps && rc == PN_OK; ++k) rc = enqueue_step(d.own);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(d.own, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail_hip(e, "hipStreamEndCapture", __LINE__);
  hipGraphExec_t x = nullptr;
  e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return fail_hip(e, "hipGraphInstantiate", __LINE__);
  }
  *graph = g;
  *exec = x;
  return PN_OK;
}

// Replays the captured time step nsteps times on `st`: kStepsPerGraph steps
// per launch of the long graph, the rest one per launch.  Both graphs are
// captured on the first call for a key (a new key drops both), so that a
// short warm-up call leaves a long run nothing to capture.  The steps and
// their order are those of direct launches, so are the results.
template <typename Enqueue>
int replay_step(DevState& d, const GraphKey& key, int64_t nsteps, hipStream_t st,
                Enqueue enqueue_step) {
  if (!(key == d.key)) drop_graph(d);
  const int64_t nlong = nsteps / kStepsPerGraph, nshort = nsteps % kStepsPerGraph;
  int rc;
  if (!d.gexec_k) {
    if ((rc = capture_steps(d, kStepsPerGraph, enqueue_step, &d.graph_k, &d.gexec_k))) return rc;
  }
  if (!d.gexec) {
    if ((rc = capture_steps(d, 1, enqueue_step, &d.graph, &d.gexec))) return rc;
  }
  d.key = key;
  for (int64_t k = 0; k < nlong; ++k) HIPCK(hipGraphLaunch(d.gexec_k, st));
  for (int64_t k = 0; k < nshort; ++k) HIPCK(hipGraphLaunch(d.gexec, st));
  return PN_OK;
}

// ------------------------------------------------------------------ batched ensembles
// Batched sweep shape per precision (pn_set_batch_shape, from the
// autotuner's table): i-bodies per lane of every system, and the common
// j-split count (0: the rule in plan_batch).
struct BatchShape {
  int ipt = 1, nsplit = 0;
};
BatchShape g_batch_shape[2];

struct BatchPlan {
  std::vector<SysDev> sys;
  std::vector<int> order, pre_pro, pre_pair, pre_epi;
  int ipt = 1;     // i-bodies per lane (1 or 2), every system
  int splits = 1;  // common j-split count (before the per-system cap)
  size_t o_sys, o_order, o_pre_pro, o_pre_pair, o_pre_epi, o_pk, o_ub, o_bpart, o_part, o_bhpart,
      o_status, o_xs, o_vs, o_kx, o_kv, total;
  int64_t n_bodies = 0;
};

// Shapes, partial-sum slots and launch prefixes of an ensemble.  Every
// system uses one sweep shape: IPT i-bodies per lane (the installed batched
// shape of the precision, default 1), 4 wavefronts per i-range; the number of
// j-splits is common, by default chosen so the whole ensemble has ~16k sweep
// workgroups, and capped per system so each wavefront keeps at least 32 j.
// PN_BATCH_SHAPE="ipt,nsplit" overrides the shape (tuning runs).
// (G, c, eps may be null when only the shape is wanted)
BatchPlan plan_batch(int n_sys, const int64_t* off, int precision, const double* G = nullptr,
                     const double* c = nullptr, const double* eps = nullptr) {
  BatchPlan P;
  P.sys.resize(n_sys);
  BatchShape bs = g_batch_shape[precision == PN_MIXED ? 1 : 0];
  if (const char* env = getenv("PN_BATCH_SHAPE")) {
    int a = 0, b = -1;
    if (sscanf(env, "%d,%d", &a, &b) == 2 && (a == 1 || a == 2) && b >= 0 && b <= 64) {
      bs.ipt = a;
      bs.nsplit = b;
    }
  }
  P.ipt = bs.ipt;
  const int ib = 64 * P.ipt;  // i-bodies per sweep workgroup
  int64_t tot_iblocks = 0;
  for (int b = 0; b < n_sys; ++b) tot_iblocks += (off[b + 1] - off[b] - 1 + ib - 1) / ib;
  int ns_common =
      (int)std::max<int64_t>(1, std::min<int64_t>(16, (16384 + tot_iblocks - 1) / tot_iblocks));
  if (bs.nsplit > 0) ns_common = bs.nsplit;
  P.splits = ns_common;
  int64_t star0 = 0, part0 = 0;
  int pro0 = 0, epi0 = 0;
  for (int b = 0; b < n_sys; ++b) {
    SysDev& S = P.sys[b];
    const int Ns = (int)(off[b + 1] - off[b] - 1);
    S.body0 = off[b];
    S.star0 = star0;
    S.part0 = part0;
    S.Ns = Ns;
    S.iblocks = (Ns + ib - 1) / ib;
    int ns = std::max(1, std::min(ns_common, Ns / 128));
    S.jchunk = (Ns + ns - 1) / ns;
    S.nsplit = (Ns + S.jchunk - 1) / S.jchunk;
    S.npro = (Ns + kBlock - 1) / kBlock;
    S.nepi = (Ns + kEpiStars - 1) / kEpiStars;
    S.pro0 = pro0;
    S.epi0 = epi0;
    if (G && c && eps) {
      S.G = G[b];
      S.lam = lambda_of(c[b]);
      S.eps2 = eps[b] * eps[b];
    }
    star0 += Ns;
    part0 += (int64_t)S.nsplit * kNF * Ns;
    pro0 += S.npro;
    epi0 += S.nepi;
  }
  P.n_bodies = off[n_sys];
  P.order.resize(n_sys);
  for (int b = 0; b < n_sys; ++b) P.order[b] = b;
  std::stable_sort(P.order.begin(), P.order.end(),
                   [&](int x, int y) { return P.sys[x].Ns > P.sys[y].Ns; });
  P.pre_pro.assign(n_sys + 1, 0);
  P.pre_pair.assign(n_sys + 1, 0);
  P.pre_epi.assign(n_sys + 1, 0);
  for (int r = 0; r < n_sys; ++r) {
    const SysDev& S = P.sys[P.order[r]];
    P.pre_pro[r + 1] = P.pre_pro[r] + S.npro;
    P.pre_pair[r + 1] = P.pre_pair[r] + S.iblocks * S.nsplit;
    P.pre_epi[r + 1] = P.pre_epi[r] + S.nepi;
  }
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += align256(bytes);
    return at;
  };
  P.o_sys = take(n_sys * sizeof(SysDev));
  P.o_order = take(n_sys * sizeof(int));
  P.o_pre_pro = take((n_sys + 1) * sizeof(int));
  P.o_pre_pair = take((n_sys + 1) * sizeof(int));
  P.o_pre_epi = take((n_sys + 1) * sizeof(int));
  P.o_pk = take((size_t)star0 * sizeof(PkF64));
  P.o_ub = take((size_t)star0 * 4 * sizeof(double));
  P.o_bpart = take((size_t)pro0 * kProRows * 8 * sizeof(double));
  P.o_part = take((size_t)part0 * sizeof(double));
  P.o_bhpart = take((size_t)epi0 * 4 * sizeof(double));
  P.o_status = take(sizeof(int));
  const size_t n3 = 3 * (size_t)P.n_bodies * sizeof(double);
  P.o_xs = take(n3);
  P.o_vs = take(n3);
  P.o_kx = take(n3);
  P.o_kv = take(n3);
  P.total = o;
  return P;
}

int enqueue_batched_step(const BatchPlan& P, char* base, const double* mass, double* X, double* V,
                         double dt, int precision, hipStream_t st) {
  const int n_sys = (int)P.sys.size();
  BatchArgs b;
  b.sys = reinterpret_cast<const SysDev*>(base + P.o_sys);
  b.order = reinterpret_cast<const int*>(base + P.o_order);
  b.n_sys = n_sys;
  b.mass = mass;
  b.pk = base + P.o_pk;
  b.ub = reinterpret_cast<double*>(base + P.o_ub);
  b.bpart = reinterpret_cast<double*>(base + P.o_bpart);
  b.part = reinterpret_cast<double*>(base + P.o_part);
  b.bhpart = reinterpret_cast<double*>(base + P.o_bhpart);
  b.status = reinterpret_cast<int*>(base + P.o_status);
  b.dt = dt;
  b.X = X;
  b.V = V;
  b.Xs = reinterpret_cast<double*>(base + P.o_xs);
  b.Vs = reinterpret_cast<double*>(base + P.o_vs);
  b.KX = reinterpret_cast<double*>(base + P.o_kx);
  b.KV = reinterpret_cast<double*>(base + P.o_kv);
  const int* pre_pro = reinterpret_cast<const int*>(base + P.o_pre_pro);
  const int* pre_pair = reinterpret_cast<const int*>(base + P.o_pre_pair);
  const int* pre_epi = reinterpret_cast<const int*>(base + P.o_pre_epi);
  for (int stage = 0; stage < 4; ++stage) {
    b.stage = stage;
    b.pos = stage == 0 ? X : b.Xs;
    b.vel = stage == 0 ? V : b.Vs;
    b.pre = pre_pro;
    if (precision == PN_MIXED)
      hipLaunchKernelGGL(k_prologue_batched<float>, dim3(P.pre_pro[n_sys]), dim3(kBlock), 0, st, b);
    else
      hipLaunchKernelGGL(k_prologue_batched<double>, dim3(P.pre_pro[n_sys]), dim3(kBlock), 0, st, b);
    HIPCK(hipGetLastError());
    b.pre = pre_pair;
    const dim3 gp(P.pre_pair[n_sys]);
    if (precision == PN_MIXED) {
      if (P.ipt == 2) hipLaunchKernelGGL((k_pair_batched<float, 2>), gp, dim3(kBlock), 0, st, b);
      else hipLaunchKernelGGL((k_pair_batched<float, 1>), gp, dim3(kBlock), 0, st, b);
    } else {
      if (P.ipt == 2) hipLaunchKernelGGL((k_pair_batched<double, 2>), gp, dim3(kBlock), 0, st, b);
      else hipLaunchKernelGGL((k_pair_batched<double, 1>), gp, dim3(kBlock), 0, st, b);
    }
    HIPCK(hipGetLastError());
    b.pre = pre_epi;
    hipLaunchKernelGGL(k_epilogue_batched, dim3(P.pre_epi[n_sys]), dim3(kBlock), 0, st, b);
    HIPCK(hipGetLastError());
    hipLaunchKernelGGL(k_bh_final_batched, dim3(n_sys), dim3(kBlock), 0, st, b);
    HIPCK(hipGetLastError());
  }
  return PN_OK;
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
  const Layout L = layout_for(N, sh, Need::EVAL);
  if ((rc = ensure_scratch(*d, L.total))) return rc;
  Ptrs P{d->base, L};
  hipStream_t st = pick_stream(*d, stream);
  if ((rc = order_after_previous(*d, st))) return rc;
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
  const Layout L = layout_for(N, sh, Need::EVAL);
  if ((rc = ensure_scratch(*d, L.total))) return rc;
  Ptrs P{d->base, L};
  hipStream_t st = pick_stream(*d, stream);
  if ((rc = order_after_previous(*d, st))) return rc;
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
  const Layout L = layout_for(N, sh, Need::EVAL);
  if ((rc = ensure_scratch(*d, L.total))) return rc;
  Ptrs P{d->base, L};
  hipStream_t st = pick_stream(*d, stream);
  if ((rc = order_after_previous(*d, st))) return rc;
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

int pn_accel_noalloc(const double* pos, const double* vel, const double* mass, int64_t N,
                     double G, double c, double eps, int precision, double* acc_newton,
                     double* phi, double* acc_1pn, void* stream, int flags) {
  int rc = check_system(pos, mass, N, G, c, eps);
  if (rc) return rc;
  if (!dptr_ok(vel)) return PN_EINVAL;
  if (precision != PN_FP64 && precision != PN_MIXED) return PN_EINVAL;
  if ((acc_newton && !dptr_ok(acc_newton)) || (phi && !dptr_ok(phi)) ||
      (acc_1pn && !dptr_ok(acc_1pn)))
    return PN_EINVAL;
  if (flags & PN_TIMING) return fail_inval("pn_accel_noalloc does not take PN_TIMING");
  std::lock_guard<std::mutex> lk(g_mu);
  // pn_accel's shape, with fewer j-splits where its partial sums would not
  // fit the fixed scratch; sizes that do not fit even with one split are
  // rejected before any device work
  const int Ns = (int)(N - 1);
  const Shape tuned = pick_shape(Ns, precision);
  Shape sh = tuned;
  Layout L = layout_for(N, sh, Need::EVAL);
  for (int want = tuned.nsplit - 1; L.total > kFixedScratchBytes && want >= 1; --want) {
    sh = with_splits(tuned, Ns, want);
    L = layout_for(N, sh, Need::EVAL);
  }
  if (L.total > kFixedScratchBytes) {
    char msg[192];
    snprintf(msg, sizeof msg,
             "pn_accel_noalloc: N = %lld needs %zu bytes of scratch, more than its fixed %zu",
             (long long)N, L.total, kFixedScratchBytes);
    return fail_inval(msg);
  }
  DevState* d;
  if ((rc = dev_state(&d))) return rc;
  Ptrs P{d->fixed, L};
  hipStream_t st = pick_stream(*d, stream);
  Sys s{pos, vel, mass, N, G, c, eps};
  if ((rc = reset_status(P, st))) return rc;
  Outs o;
  o.acc_newton = acc_newton;
  o.phi = phi;
  o.acc_1pn = acc_1pn;
  if ((rc = enqueue_eval(s, P, sh, precision, o, st, nullptr))) return rc;
  if (flags & PN_ASYNC) return PN_OK;
  return read_status(P, st);
}

int pn_accel_eih(const double* pos, const double* vel, const double* mass, int64_t N, double G,
                 double c, double eps, int precision, double* acc_newton, double* phi,
                 double* acc_1pn, void* stream, int flags) {
  int rc = check_system(pos, mass, N, G, c, eps);
  if (rc) return rc;
  if (!dptr_ok(vel)) return PN_EINVAL;
  if (precision != PN_FP64 && precision != PN_MIXED) return PN_EINVAL;
  if ((acc_newton && !dptr_ok(acc_newton)) || (phi && !dptr_ok(phi)) ||
      (acc_1pn && !dptr_ok(acc_1pn)))
    return PN_EINVAL;
  if (N >= ((int64_t)1 << 28)) return PN_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  DevState* d;
  if ((rc = dev_state(&d))) return rc;
  // both sweeps run over all N bodies: shapes and scratch sized for N "stars"
  const Shape sh = pick_shape((int)N, precision);
  const Layout L = layout_for(N + 1, sh, Need::EVAL);
  if ((rc = ensure_scratch(*d, L.total))) return rc;
  Ptrs P{d->base, L};
  hipStream_t st = pick_stream(*d, stream);
  if ((rc = order_after_previous(*d, st))) return rc;
  if ((rc = reset_status(P, st))) return rc;
  EihArgs e;
  e.pos = pos;
  e.vel = vel;
  e.mass = mass;
  e.N = (int)N;
  e.G = G;
  e.lam = lambda_of(c);
  e.pk = P.at<void>(L.pk);
  e.va = P.at<double>(L.ub);
  e.part = P.at<double>(L.part);
  e.nsplit = sh.nsplit;
  e.acc_newton = acc_newton;
  e.phi = phi;
  e.acc_1pn = acc_1pn;
  e.status = P.at<int>(L.status);
  const int nb = (int)((N + kBlock - 1) / kBlock);
  Sys all{pos, vel, mass, N + 1, G, c, eps};  // launch_pair sweeps Ns = N bodies
  const bool mixed = precision == PN_MIXED;
  if (mixed) hipLaunchKernelGGL(k_eih_packets<float>, dim3(nb), dim3(kBlock), 0, st, e);
  else hipLaunchKernelGGL(k_eih_packets<double>, dim3(nb), dim3(kBlock), 0, st, e);
  HIPCK(hipGetLastError());
  if ((rc = launch_pair(all, P, sh, precision, MODE_P1, st))) return rc;
  if (mixed) hipLaunchKernelGGL(k_eih_mid<float>, dim3(nb), dim3(kBlock), 0, st, e);
  else hipLaunchKernelGGL(k_eih_mid<double>, dim3(nb), dim3(kBlock), 0, st, e);
  HIPCK(hipGetLastError());
  if ((rc = launch_pair(all, P, sh, precision, MODE_P2, st))) return rc;
  hipLaunchKernelGGL(k_eih_final, dim3(nb), dim3(kBlock), 0, st, e);
  HIPCK(hipGetLastError());
  return finish(*d, P, st, flags);
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
  const int ns = pick_stage_ns(N, precision);
  const Layout L = layout_for(N, sh, Need::RK4, ns);
  if ((rc = ensure_scratch(*d, L.total))) return rc;
  Ptrs P{d->base, L};
  hipStream_t st = pick_stream(*d, stream);
  if ((rc = order_after_previous(*d, st))) return rc;
  Sys s{pos, vel, mass, N, G, c, eps};
  if ((rc = reset_status(P, st))) return rc;
  const bool timing = (flags & PN_TIMING) != 0;
  const bool graph = !(flags & (PN_NOGRAPH | PN_TIMING));
  if (nsteps > 0 && ns > 0) {
    // one launch per stage: the head, the first step, nsteps - 1 further
    // steps (replayed from a graph), the last pending update
    Timer tm;
    tm.d = d;
    tm.on = timing;
    if ((rc = launch_stage_head(s, P, sh, precision, ns, st))) return rc;
    if ((rc = enqueue_stage_step(s, P, sh, precision, dt, pos, vel, ns, true, st, &tm))) return rc;
    if (nsteps > 1) {
      if (!graph) {
        for (int64_t k = 1; k < nsteps; ++k)
          if ((rc = enqueue_stage_step(s, P, sh, precision, dt, pos, vel, ns, false, st, &tm)))
            return rc;
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
        key.stage_ns = ns;
        key.base = d->base;
        rc = replay_step(*d, key, nsteps - 1, st, [&](hipStream_t cs) {
          return enqueue_stage_step(s, P, sh, precision, dt, pos, vel, ns, false, cs, nullptr);
        });
        if (rc) return rc;
      }
    }
    if ((rc = launch_stage(s, P, sh, precision, dt, pos, vel, 0, kStageFinal, ns, st))) return rc;
    if ((rc = tm.collect((double)(N - 1) * (double)(N - 2)))) return rc;
  } else if (nsteps > 0) {
    if ((rc = launch_prologue(s, P, precision, st))) return rc;  // stage 0's packets, buffer 0
    if (!graph) {
      Timer tm;
      tm.d = d;
      tm.on = timing;
      if ((rc = enqueue_rk4_head(s, P, sh, precision, dt, pos, vel, st, &tm))) return rc;
      for (int64_t k = 0; k < nsteps; ++k)
        if ((rc = enqueue_rk4_body(s, P, sh, precision, dt, pos, vel, k + 1 < nsteps, st, &tm)))
          return rc;
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
      // the first sweep, nsteps - 1 replayed steps (each ending in the next
      // step's first sweep), and the last step launched directly
      if ((rc = enqueue_rk4_head(s, P, sh, precision, dt, pos, vel, st, nullptr))) return rc;
      if (nsteps > 1) {
        rc = replay_step(*d, key, nsteps - 1, st, [&](hipStream_t cs) {
          return enqueue_rk4_body(s, P, sh, precision, dt, pos, vel, true, cs, nullptr);
        });
        if (rc) return rc;
      }
      if ((rc = enqueue_rk4_body(s, P, sh, precision, dt, pos, vel, false, st, nullptr)))
        return rc;
    }
  }
  return finish(*d, P, st, flags & ~PN_TIMING);
}

int pn_jerk(const double* pos, const double* vel, const double* mass, int64_t N, double G,
            double c, double eps, double* acc, double* jerk, void* stream, int flags) {
  int rc = check_system(pos, mass, N, G, c, eps);
  if (rc) return rc;
  if (!dptr_ok(vel) || !dptr_ok(acc) || !dptr_ok(jerk)) return PN_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  DevState* d;
  if ((rc = dev_state(&d))) return rc;
  const Shape sh = pick_shape((int)(N - 1), PN_FP64);
  const Layout L = layout_for(N, sh, Need::JERK);
  if ((rc = ensure_scratch(*d, L.total))) return rc;
  Ptrs P{d->base, L};
  hipStream_t st = pick_stream(*d, stream);
  if ((rc = order_after_previous(*d, st))) return rc;
  Sys s{pos, vel, mass, N, G, c, eps};
  if ((rc = reset_status(P, st))) return rc;
  Outs o;
  o.jerk = jerk;
  if ((rc = enqueue_jerk(s, P, sh, acc, o, st))) return rc;
  return finish(*d, P, st, flags & ~PN_TIMING);
}

int pn_step_hermite(double* pos, double* vel, const double* mass, int64_t N, double G, double c,
                    double eps, double dt, int64_t nsteps, void* stream, int flags) {
  int rc = check_system(pos, mass, N, G, c, eps);
  if (rc) return rc;
  if (!dptr_ok(vel) || !std::isfinite(dt) || !(dt > 0.0) || nsteps < 0) return PN_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  DevState* d;
  if ((rc = dev_state(&d))) return rc;
  const Shape sh = pick_shape((int)(N - 1), PN_FP64);
  const Layout L = layout_for(N, sh, Need::HERMITE);
  if ((rc = ensure_scratch(*d, L.total))) return rc;
  Ptrs P{d->base, L};
  hipStream_t st = pick_stream(*d, stream);
  if ((rc = order_after_previous(*d, st))) return rc;
  Sys s{pos, vel, mass, N, G, c, eps};
  if ((rc = reset_status(P, st))) return rc;
  if (nsteps > 0) {
    if ((rc = enqueue_hermite_start(s, P, sh, dt, pos, vel, st))) return rc;
    if (flags & (PN_NOGRAPH | PN_TIMING)) {
      for (int64_t k = 0; k < nsteps; ++k)
        if ((rc = enqueue_hermite_step(s, P, sh, dt, pos, vel, st))) return rc;
    } else {
      GraphKey key;
      key.scheme = 1;
      key.pos = pos;
      key.vel = vel;
      key.mass = mass;
      key.N = N;
      key.G = G;
      key.c = c;
      key.eps = eps;
      key.dt = dt;
      key.precision = PN_FP64;
      key.ipt = sh.ipt;
      key.ws = sh.ws;
      key.nsplit = sh.nsplit;
      key.base = d->base;
      rc = replay_step(*d, key, nsteps, st, [&](hipStream_t cs) {
        return enqueue_hermite_step(s, P, sh, dt, pos, vel, cs);
      });
      if (rc) return rc;
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
  const Layout L = layout_for(N, sh, Need::EVAL);
  if ((rc = ensure_scratch(*d, L.total))) return rc;
  Ptrs P{d->base, L};
  hipStream_t st = pick_stream(*d, stream);
  if ((rc = order_after_previous(*d, st))) return rc;
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

int pn_encounters(const double* pos, const double* vel, const double* mass, int64_t N, double G,
                  double c, double r_close, double* out8, void* stream, int flags) {
  (void)flags;
  if (!dptr_ok(pos) || !dptr_ok(vel) || !dptr_ok(mass) || N < 3 || N > ((int64_t)1 << 28) ||
      !out8)
    return PN_EINVAL;
  if (!(G > 0.0) || !std::isfinite(G) || std::isnan(c) || !(c > 0.0)) return PN_EINVAL;
  if (!(r_close >= 0.0) || std::isnan(r_close)) return PN_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  DevState* d;
  int rc = dev_state(&d);
  if (rc) return rc;
  const int Ns = (int)(N - 1);
  const int nb = (Ns + kBlock - 1) / kBlock;
  Shape sh = pick_shape(Ns, PN_FP64);
  const int nsplit = std::max(1, std::min(sh.nsplit * 4, std::max(1, Ns / 64)));
  const int jchunk = (Ns + nsplit - 1) / nsplit;
  const int ns = (Ns + jchunk - 1) / jchunk;
  Shape s2 = sh;
  s2.nsplit = std::max(sh.nsplit, ns);  // scratch for the larger split count
  Layout L = layout_for(N, s2, Need::EVAL);
  const size_t extra = align256((size_t)nb * 2 * sizeof(long long));
  if ((rc = ensure_scratch(*d, L.total + extra))) return rc;
  Ptrs P{d->base, L};
  hipStream_t st = pick_stream(*d, stream);
  if ((rc = order_after_previous(*d, st))) return rc;
  Sys sys{pos, nullptr, mass, N, 1.0, 1.0, 0.0};
  if ((rc = reset_status(P, st))) return rc;
  if ((rc = launch_prologue(sys, P, PN_FP64, st))) return rc;  // packets hold the positions
  EncArgs e;
  e.pos = pos;
  e.vel = vel;
  e.mass = mass;
  e.G = G;
  e.lam = lambda_of(c);
  e.pk = P.at<PkF64>(L.pk);
  e.Ns = Ns;
  e.jchunk = jchunk;
  e.r_close2 = r_close * r_close;
  e.part = P.at<double>(L.part);
  e.nsplit = ns;
  e.bpart = P.at<double>(L.dpart);
  e.bpair = reinterpret_cast<long long*>(d->base + L.total);
  e.nb = nb;
  e.out = P.at<double>(L.out8);
  hipLaunchKernelGGL(k_enc_pair, dim3(nb, ns), dim3(kBlock), 0, st, e);
  HIPCK(hipGetLastError());
  hipLaunchKernelGGL(k_enc_star, dim3(nb), dim3(kBlock), 0, st, e);
  HIPCK(hipGetLastError());
  hipLaunchKernelGGL(k_enc_final, dim3(1), dim3(64), 0, st, e);
  HIPCK(hipGetLastError());
  HIPCK(hipMemcpyAsync(out8, P.at<double>(L.out8), 8 * sizeof(double), hipMemcpyDeviceToHost, st));
  if ((rc = mark_call_end(*d, st))) return rc;
  HIPCK(hipStreamSynchronize(st));
  return PN_OK;
}

int pn_step_batched(int32_t n_sys, const int64_t* offsets, const double* G, const double* c,
                    const double* eps, double* pos, double* vel, const double* mass, double dt,
                    int64_t nsteps, int precision, void* stream, int flags) {
  if (n_sys < 1 || !offsets || !G || !c || !eps) return PN_EINVAL;
  if (offsets[0] != 0) return PN_EINVAL;
  if (!dptr_ok(vel) || !std::isfinite(dt) || nsteps < 0) return PN_EINVAL;
  if (precision != PN_FP64 && precision != PN_MIXED) return PN_EINVAL;
  for (int b = 0; b < n_sys; ++b) {
    if (offsets[b + 1] - offsets[b] < 2) return PN_EINVAL;
    int rc = check_system(pos, mass, offsets[b + 1] - offsets[b], G[b], c[b], eps[b]);
    if (rc) return rc;
  }
  if (offsets[n_sys] > ((int64_t)1 << 28)) return PN_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  DevState* d;
  int rc = dev_state(&d);
  if (rc) return rc;
  hipStream_t st = pick_stream(*d, stream);
  if ((rc = order_after_previous(*d, st))) return rc;
  const BatchPlan P = plan_batch(n_sys, offsets, precision, G, c, eps);
  if ((rc = ensure_batch_scratch(*d, P.total))) return rc;
  char* base = d->bbase;
  int* status = reinterpret_cast<int*>(base + P.o_status);
  BatchKey key;
  key.offsets.assign(offsets, offsets + n_sys + 1);
  key.G.assign(G, G + n_sys);
  key.c.assign(c, c + n_sys);
  key.eps.assign(eps, eps + n_sys);
  key.pos = pos;
  key.vel = vel;
  key.mass = mass;
  key.dt = dt;
  key.precision = precision;
  key.ipt = P.ipt;
  key.splits = P.splits;
  key.base = base;
  const bool graph = !(flags & PN_NOGRAPH);
  // The descriptors in scratch are tracked apart from the cached graph: a
  // direct-launch call for another ensemble overwrites them while the graph
  // (captured for the first ensemble) stays cached.
  if (!(d->bdesc_valid && key == d->bdesc)) {
    // system descriptors, launch order and prefixes (host -> device, once per ensemble)
    HIPCK(hipMemcpyAsync(base + P.o_sys, P.sys.data(), n_sys * sizeof(SysDev),
                         hipMemcpyHostToDevice, st));
    HIPCK(hipMemcpyAsync(base + P.o_order, P.order.data(), n_sys * sizeof(int),
                         hipMemcpyHostToDevice, st));
    HIPCK(hipMemcpyAsync(base + P.o_pre_pro, P.pre_pro.data(), (n_sys + 1) * sizeof(int),
                         hipMemcpyHostToDevice, st));
    HIPCK(hipMemcpyAsync(base + P.o_pre_pair, P.pre_pair.data(), (n_sys + 1) * sizeof(int),
                         hipMemcpyHostToDevice, st));
    HIPCK(hipMemcpyAsync(base + P.o_pre_epi, P.pre_epi.data(), (n_sys + 1) * sizeof(int),
                         hipMemcpyHostToDevice, st));
    HIPCK(hipStreamSynchronize(st));
    d->bdesc = key;
    d->bdesc_valid = true;
  }
  hipLaunchKernelGGL(k_reset_status, dim3(1), dim3(64), 0, st, status);
  HIPCK(hipGetLastError());
  if (nsteps > 0) {
    if (!graph) {
      for (int64_t k = 0; k < nsteps; ++k)
        if ((rc = enqueue_batched_step(P, base, mass, pos, vel, dt, precision, st))) return rc;
    } else {
      if (!(d->bgexec && key == d->bkey)) {
        drop_batch_graph(*d);
        HIPCK(hipStreamSynchronize(d->own));
        HIPCK(hipStreamBeginCapture(d->own, hipStreamCaptureModeThreadLocal));
        rc = enqueue_batched_step(P, base, mass, pos, vel, dt, precision, d->own);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(d->own, &g);
        if (rc) {
          if (g) (void)hipGraphDestroy(g);
          return rc;
        }
        if (e != hipSuccess) return fail_hip(e, "hipStreamEndCapture", __LINE__);
        d->bgraph = g;
        HIPCK(hipGraphInstantiate(&d->bgexec, d->bgraph, nullptr, nullptr, 0));
        d->bkey = key;
      }
      for (int64_t k = 0; k < nsteps; ++k) HIPCK(hipGraphLaunch(d->bgexec, st));
    }
  }
  if ((rc = mark_call_end(*d, st))) return rc;
  if (flags & PN_ASYNC) return PN_OK;
  int hstatus = 0;
  HIPCK(hipMemcpyAsync(&hstatus, status, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCK(hipStreamSynchronize(st));
  if (hstatus & 2) return fail_inval("mass of a massive object must be positive and finite");
  if (hstatus & 1) return PN_ENONFINITE;
  return PN_OK;
}

int pn_set_shape(int precision, int64_t n_min, int64_t n_max, int ipt, int ws, int nsplit) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (precision < 0) {
    g_tuned.clear();
    return PN_OK;
  }
  if ((precision != PN_FP64 && precision != PN_MIXED) || n_min < 2 || n_max < n_min ||
      (ipt != 1 && ipt != 2) || (ws != 1 && ws != 4 && ws != 8) || nsplit < 0 || nsplit > 65535)
    return PN_EINVAL;
  g_tuned.push_back(TunedShape{precision, n_min, n_max, ipt, ws, nsplit});
  return PN_OK;
}

int pn_query_shape(int precision, int64_t N, int* out4) {
  if (!out4 || N < 2 || N > ((int64_t)1 << 28)) return PN_EINVAL;
  if (precision != PN_FP64 && precision != PN_MIXED) return PN_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  const Shape sh = pick_shape((int)(N - 1), precision);
  out4[0] = sh.ipt;
  out4[1] = sh.ws;
  out4[2] = sh.nsplit;
  out4[3] = sh.iblocks;
  return PN_OK;
}

int pn_set_stage_kernel(int precision, int64_t n_min, int64_t n_max, int ns) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (precision < 0) {
    g_stage.clear();
    return PN_OK;
  }
  if ((precision != PN_FP64 && precision != PN_MIXED) || n_min < 2 || n_max < n_min ||
      !stage_ns_ok(ns))
    return PN_EINVAL;
  g_stage.push_back(StageSel{precision, n_min, n_max, ns});
  return PN_OK;
}

int pn_query_stage_kernel(int precision, int64_t N) {
  if (N < 2 || N > ((int64_t)1 << 28)) return PN_EINVAL;
  if (precision != PN_FP64 && precision != PN_MIXED) return PN_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  return pick_stage_ns(N, precision);
}

int pn_set_batch_shape(int precision, int ipt, int nsplit) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (precision < 0) {
    g_batch_shape[0] = g_batch_shape[1] = BatchShape();
    return PN_OK;
  }
  if ((precision != PN_FP64 && precision != PN_MIXED) || (ipt != 1 && ipt != 2) || nsplit < 0 ||
      nsplit > 64)
    return PN_EINVAL;
  g_batch_shape[precision] = BatchShape{ipt, nsplit};
  return PN_OK;
}

int pn_query_batch_shape(int precision, int32_t n_sys, const int64_t* offsets, int* out) {
  if (n_sys < 1 || !offsets || !out || offsets[0] != 0) return PN_EINVAL;
  if (precision != PN_FP64 && precision != PN_MIXED) return PN_EINVAL;
  for (int b = 0; b < n_sys; ++b)
    if (offsets[b + 1] - offsets[b] < 2) return PN_EINVAL;
  if (offsets[n_sys] > ((int64_t)1 << 28)) return PN_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  const BatchPlan P = plan_batch(n_sys, offsets, precision);
  out[0] = P.ipt;
  for (int b = 0; b < n_sys; ++b) out[1 + b] = P.sys[b].nsplit;
  return PN_OK;
}

const char* pn_strerror(int code) {
  switch (code) {
    case PN_OK: return "ok";
    case PN_EINVAL: return g_inval[0] ? g_inval : "invalid argument";
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
    drop_batch_graph(d);
    if (d.bbase) (void)hipFree(d.bbase);
    d.bbase = nullptr;
    d.bcap = 0;
    d.bdesc_valid = false;
    for (hipEvent_t e : d.ev) (void)hipEventDestroy(e);
    d.ev.clear();
    if (d.last_ev) (void)hipEventDestroy(d.last_ev);
    d.last_ev = nullptr;
    d.last_st = nullptr;
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
