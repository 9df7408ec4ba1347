// C ABI of libhrlb (declared in include/hrlb.h): argument checking, buffer carve-up,
// table upload and the launch sequence of the RK3 step.  Host code only; all device work
// is enqueued on the caller's stream.
#include "hrlb.h"

#include <hip/hip_runtime_api.h>

#include <dlfcn.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "hrlb_internal.h"

using namespace hrlb;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(HRLB_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr, what)            \
  do {                                 \
    hipError_t _e = (expr);            \
    if (_e != hipSuccess) return hip_fail(_e, what); \
  } while (0)

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

namespace hrlb {
int set_error(int code, const char* msg) { return fail(code, msg); }
}  // namespace hrlb

struct hrlb_quad {
  QuadTables t;
};

struct hrlb_sim {
  Shape sh;
  DevPtrs d;
  WorkLayout lay;
  hipStream_t stream;
  int cells, waves;
  int part_nvb;      // nvb of the launch that produced the current moment partials
  int resid_nres;    // residual partial count of the last stage-3 launch (0: none yet)
  bool timing;
  bool graph_on;
  hipGraphExec_t gexec;   // one captured RK3 step (valid when gexec != nullptr)
  hipGraphExec_t gexec_k; // GRAPH_BLOCK captured steps (nullptr until a long enough run)
  hipStream_t cap_stream; // private stream the steps are captured on
  int g_cells, g_waves;   // launch shape the graphs were captured with
  std::vector<hipEvent_t> ev;  // pairs (start, stop), kind in ev_kind
  std::vector<int> ev_kind;
  double ms[4];          // device time of stage 1, 2, 3 launches and of closure launches
  long long launches[4];
};

struct hrlb_batch {
  std::vector<hrlb_sim*> sims;
  std::vector<int> inst_offset;   // first concatenated instance index of each sim
  int cells, waves;
  hipStream_t stream;
  GroupDesc* d_groups;
  int* d_tiles;      // int4 per tile
  int* d_ntiles;
  int* d_items;      // int2 per closure item
  int* d_nitems;
  int max_tiles, max_items, ntiles, nitems;
  int nb;            // nodes per closure block (all groups)
  int grid_stage, grid_closure;
  size_t lds_stage, lds_closure;
  std::vector<int> active;
  hipGraphExec_t gexec;    // one captured batched step
  hipGraphExec_t gexec_k;  // GRAPH_BLOCK captured batched steps
  hipStream_t cap_stream;
};

namespace hrlb {

WorkLayout work_layout(const Shape& sh) {
  WorkLayout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align256(bytes);
    return o;
  };
  const size_t dsz = sizeof(double);
  L.nvb_max = (sh.V + 63) / 64;
  L.nres_max = L.nvb_max * sh.S;
  L.px = take(2 * sh.Qx * dsz);
  L.py = take(sh.Qy * dsz);
  L.pz = take(sh.Qz * dsz);
  L.phix = take((size_t)sh.Qx * (sh.Nx + 1) * dsz);
  L.cx = take((size_t)(sh.Nx + 1) * (sh.Nx + 1) * dsz);
  L.phiy = take((size_t)sh.Qy * (sh.Ny + 1) * dsz);
  L.phiz = take((size_t)sh.Qz * (sh.Nz + 1) * dsz);
  L.ptab = take((size_t)ptab_blocks(sh.V) * 1024 * dsz);
  L.inst = take((size_t)sh.B * sizeof(InstDev));
  L.inv_dx = take((size_t)sh.B * sh.S * dsz);
  L.g_rest = take((size_t)sh.B * sh.V * dsz);
  L.g_wall = take((size_t)sh.B * sh.V * dsz);
  L.partials = take((size_t)sh.B * part_groups(sh.S) * L.nvb_max * PART_GROUP * dsz);
  L.rec = take((size_t)sh.B * sh.S * sh.rec_len * dsz);
  L.nw = take((size_t)sh.B * dsz);
  L.resid_part = take((size_t)sh.B * L.nres_max * 2 * dsz);
  L.resid = take((size_t)sh.B * dsz);
  L.flags = take((size_t)sh.B * sizeof(int));
  L.junk = take(256 * dsz);
  L.total = off;
  return L;
}

}  // namespace hrlb

static Shape make_shape(const QuadTables& t, int S, int B, int scheme) {
  Shape sh;
  sh.Qx = t.Qx;
  sh.Nx = t.Nx;
  sh.Qy = t.Qy;
  sh.Ny = t.Ny;
  sh.Qz = t.Qz;
  sh.Nz = t.Nz;
  sh.QyQz = t.Qy * t.Qz;
  sh.V = 2 * t.Qx * sh.QyQz;
  sh.S = S;
  sh.B = B;
  sh.scheme = scheme;
  sh.reduced = t.reduced;
  sh.pad = 0;
  // whole 128-byte lines per node record
  int rl = REC_HEAD + 2 * t.Qx + sh.QyQz;
  sh.rec_len = (rl + 15) & ~15;
  return sh;
}

// The stage kernel addresses one instance's populations and closure records with 32-bit
// byte offsets.
static bool instance_fits(const Shape& sh) {
  const size_t lim = (size_t)1 << 32;
  return (size_t)sh.S * sh.V * sizeof(double) < lim && (size_t)sh.S * sh.rec_len * sizeof(double) < lim;
}

// Node positions of App. A.2 (Eqs. stretch, etas), 1-based fractional index s.
static double node_x(double s, int S, double A) {
  if (A == 0.0) return (s - 0.5) / (2.0 * S);
  const double eta = (s - 0.5) * std::atanh(A) / S;
  return std::tanh(eta) / (2.0 * A);
}

static int default_cells(const Shape& sh) {
  // long marches amortise the halo re-reads and per-block setup; short ones fill the
  // device when there are few instances
  const long long pairs = (long long)sh.B * sh.S * sh.V;
  if (pairs >= (1LL << 24)) return 32;
  if (pairs >= (1LL << 21)) return 16;
  return 4;
}

static int default_waves(const Shape& sh) {
  const int wv = (sh.V + 63) / 64;
  // waves per block in 1..MAX_WAVES with the fewest idle lanes, larger on ties
  int best = 1, best_waste = 1 << 30;
  for (int w = 1; w <= MAX_WAVES; ++w) {
    const int waste = ((wv + w - 1) / w) * w - wv;
    if (waste <= best_waste) {
      best = w;
      best_waste = waste;
    }
  }
  return best;
}

// Optional roctx ranges around the library's calls (HRLB_TRACE=1 in the environment when the
// library is first used): they name the host-side interval of each call, the enqueue of a
// step and of each stage, in a rocprofv3 --marker-trace timeline beside the kernels those
// calls launch.  The roctx library is opened at run time, so without the variable, or
// without the library, nothing changes and nothing is linked.
namespace {
struct Trace {
  int (*push)(const char*) = nullptr;
  int (*pop)() = nullptr;
  bool on = false;
  Trace() {
    const char* e = std::getenv("HRLB_TRACE");
    if (!e || !*e || std::strcmp(e, "0") == 0) return;
    void* h = dlopen("librocprofiler-sdk-roctx.so.1", RTLD_NOW | RTLD_LOCAL);
    if (!h) h = dlopen("librocprofiler-sdk-roctx.so", RTLD_NOW | RTLD_LOCAL);
    if (!h) return;
    push = reinterpret_cast<int (*)(const char*)>(dlsym(h, "roctxRangePushA"));
    pop = reinterpret_cast<int (*)()>(dlsym(h, "roctxRangePop"));
    on = push && pop;
  }
};
Trace& trace() {
  static Trace t;
  return t;
}
// one range for the lifetime of the object (pushed and popped on the calling thread)
struct Range {
  bool on;
  explicit Range(const char* name) : on(trace().on) {
    if (on) trace().push(name);
  }
  ~Range() {
    if (on) trace().pop();
  }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};
const char* const STAGE_RANGE[3] = {"RK3 stage 1", "RK3 stage 2", "RK3 stage 3"};
}  // namespace

extern "C" {

const char* hrlb_last_error(void) { return g_err.c_str(); }

int hrlb_trace_status(int* enabled) {
  if (!enabled) return fail(HRLB_EINVAL, "trace_status: enabled is NULL");
  *enabled = trace().on ? 1 : 0;
  return HRLB_OK;
}

int hrlb_init_quadrature(int Qx, int Nx, int Qy, int Ny, int Qz, int Nz, hrlb_quad** out) {
  if (!out) return fail(HRLB_EINVAL, "init_quadrature: out is NULL");
  *out = nullptr;
  if (Qx < 1 || Qx > QX_MAX) return fail(HRLB_EINVAL, "init_quadrature: Qx must be in 1..128");
  if (Nx < 0 || Nx > std::min(Qx - 1, NX_MAX)) return fail(HRLB_EINVAL, "init_quadrature: need 0 <= Nx <= min(Qx-1, 8)");
  if (Qy < 1 || Qy > QYZ_MAX || Qz < 1 || Qz > QYZ_MAX) return fail(HRLB_EINVAL, "init_quadrature: Qy, Qz must be in 1..16");
  if (Ny < 0 || Ny > Qy - 1 || Nz < 0 || Nz > Qz - 1)
    return fail(HRLB_EINVAL, "init_quadrature: need 0 <= Ny <= Qy-1 and 0 <= Nz <= Qz-1");
  hrlb_quad* q = new hrlb_quad;
  build_quadrature(Qx, Nx, Qy, Ny, Qz, Nz, q->t);
  *out = q;
  return HRLB_OK;
}

int hrlb_init_quadrature_reduced(int Qx, int Nx, int Qy, int Ny, hrlb_quad** out) {
  if (!out) return fail(HRLB_EINVAL, "init_quadrature_reduced: out is NULL");
  *out = nullptr;
  if (Qx < 1 || Qx > QX_MAX) return fail(HRLB_EINVAL, "init_quadrature_reduced: Qx must be in 1..128");
  if (Nx < 0 || Nx > std::min(Qx - 1, NX_MAX))
    return fail(HRLB_EINVAL, "init_quadrature_reduced: need 0 <= Nx <= min(Qx-1, 8)");
  if (Qy < 1 || Qy > QYZ_MAX) return fail(HRLB_EINVAL, "init_quadrature_reduced: Qy must be in 1..16");
  if (Ny < 0 || Ny > Qy - 1) return fail(HRLB_EINVAL, "init_quadrature_reduced: need 0 <= Ny <= Qy-1");
  hrlb_quad* q = new hrlb_quad;
  build_quadrature(Qx, Nx, Qy, Ny, 1, 0, q->t);
  // the z axis becomes the pair of reduced distributions (phi, chi): no p_z, and a z factor
  // of the equilibrium of 1 for phi and T for chi, which the kernels form themselves
  q->t.Qz = 2;
  q->t.Nz = 0;
  q->t.pz.assign(2, 0.0);
  q->t.wz.assign(2, 1.0);
  q->t.phiz.assign(2, 1.0);
  q->t.reduced = 1;
  *out = q;
  return HRLB_OK;
}

void hrlb_quad_free(hrlb_quad* q) { delete q; }

int hrlb_quad_size(const hrlb_quad* q, int* V) {
  if (!q || !V) return fail(HRLB_EINVAL, "quad_size: NULL argument");
  *V = 2 * q->t.Qx * q->t.Qy * q->t.Qz;
  return HRLB_OK;
}

int hrlb_quad_nodes(const hrlb_quad* q, int axis, double* nodes, double* weights) {
  if (!q || !nodes || !weights) return fail(HRLB_EINVAL, "quad_nodes: NULL argument");
  const std::vector<double>*p, *w;
  if (axis == 0) {
    p = &q->t.px;
    w = &q->t.wx;
  } else if (axis == 1) {
    p = &q->t.py;
    w = &q->t.wy;
  } else if (axis == 2) {
    if (q->t.reduced) return fail(HRLB_EINVAL, "quad_nodes: the reduced (phi, chi) model has no p_z axis");
    p = &q->t.pz;
    w = &q->t.wz;
  } else {
    return fail(HRLB_EINVAL, "quad_nodes: axis must be 0, 1 or 2");
  }
  std::memcpy(nodes, p->data(), p->size() * sizeof(double));
  std::memcpy(weights, w->data(), w->size() * sizeof(double));
  return HRLB_OK;
}

int hrlb_state_bytes(const hrlb_quad* q, int S, int batch, size_t* state_bytes, size_t* work_bytes) {
  if (!q || !state_bytes || !work_bytes) return fail(HRLB_EINVAL, "state_bytes: NULL argument");
  if (S < 3 || batch < 1) return fail(HRLB_EINVAL, "state_bytes: need S >= 3 and batch >= 1");
  const Shape sh = make_shape(q->t, S, batch, 0);
  if (!instance_fits(sh)) return fail(HRLB_EINVAL, "state_bytes: one instance's populations (S * V * 8 bytes) must stay below 4 GiB");
  *state_bytes = 3 * align256((size_t)batch * S * sh.V * sizeof(double));
  *work_bytes = work_layout(sh).total;
  return HRLB_OK;
}

// Parameter checks shared by init_state and step_noalloc (before any device use).
static int check_instances(const char* fn, int S, int scheme, const hrlb_params* params, int batch) {
  const std::string f(fn);
  if (S < 3) return fail(HRLB_EINVAL, f + ": S must be >= 3 (three ghost layers mirror nodes 1..3)");
  if (batch < 1) return fail(HRLB_EINVAL, f + ": batch must be >= 1");
  if (scheme != HRLB_SCHEME_UPWIND2 && scheme != HRLB_SCHEME_WENO5 && scheme != HRLB_SCHEME_LINEAR5)
    return fail(HRLB_EINVAL, f + ": unknown scheme");
  for (int b = 0; b < batch; ++b) {
    const hrlb_params& p = params[b];
    const std::string at = " (instance " + std::to_string(b) + ")";
    if (!(p.dt > 0) || !std::isfinite(p.dt)) return fail(HRLB_EINVAL, f + ": dt must be > 0" + at);
    if (!(p.kn > 0) || !std::isfinite(p.kn)) return fail(HRLB_EINVAL, f + ": kn must be > 0" + at);
    if (!(p.T_w > 0)) return fail(HRLB_EINVAL, f + ": T_w must be > 0" + at);
    if (!(p.n0 > 0)) return fail(HRLB_EINVAL, f + ": n0 must be > 0" + at);
    if (!(p.pr > 0)) return fail(HRLB_EINVAL, f + ": pr must be > 0" + at);
    if (!(p.A >= 0 && p.A < 1)) return fail(HRLB_EINVAL, f + ": A must be in [0, 1)" + at);
    if (p.law != HRLB_LAW_POWER && p.law != HRLB_LAW_SUTHERLAND && p.law != HRLB_LAW_LOWMACH)
      return fail(HRLB_EINVAL, f + ": unknown law" + at);
    if (p.law == HRLB_LAW_SUTHERLAND && !(p.suth_S >= 0)) return fail(HRLB_EINVAL, f + ": suth_S must be >= 0" + at);
    if (!std::isfinite(p.u_w) || !std::isfinite(p.omega)) return fail(HRLB_EINVAL, f + ": non-finite u_w/omega" + at);
  }
  return HRLB_OK;
}

// RK3 (Eq. rk3) stability limits of the linear schemes, from the amplification factor
// 1 + z + z^2/2 + z^3/6 over the Fourier symbols of the advection operators: Courant number
// max|p_x| dt / dx up to 0.628 for second-order upwind and 1.434 for the fifth-order
// candidates with the ideal weights; dt / tau up to 2.512 on the negative real axis for the
// relaxation.  WENO-5 is not linear: its weights leave the ideal ones wherever the data are
// not smooth, and the paper itself runs it at a Courant number of 1.65 at the outermost
// node of HHLB(6;100) on 16 stretched nodes (Table III), which stays bounded; for it the
// check is a guard against gross violations at 2.
constexpr double CFL_UPWIND2 = 0.628, CFL_LINEAR5 = 1.434, CFL_WENO5_GUARD = 2.0, RELAX_RK3 = 2.512;

// A time step beyond these limits cannot give a bounded solution: reject it before any
// device use.  The relaxation limit is checked at the initial state (n0, T_w); a state that
// later grows stiffer shows up as a numerical fault in the step.
static int check_stability(const char* fn, const QuadTables& t, int S, int scheme, const hrlb_params* params,
                           int batch) {
  double pmax = 0.0;
  for (double p : t.px) pmax = std::max(pmax, std::fabs(p));
  const double lim = scheme == HRLB_SCHEME_UPWIND2 ? CFL_UPWIND2 : scheme == HRLB_SCHEME_LINEAR5 ? CFL_LINEAR5 : CFL_WENO5_GUARD;
  for (int b = 0; b < batch; ++b) {
    const hrlb_params& p = params[b];
    double dxmin = 1e300;
    for (int c = 0; c < S; ++c) dxmin = std::min(dxmin, node_x(c + 1.5, S, p.A) - node_x(c + 0.5, S, p.A));
    const double courant = pmax * p.dt / dxmin;
    const std::string at = " (instance " + std::to_string(b) + ")";
    if (courant > lim)
      return fail(HRLB_ENUMERIC, std::string(fn) + ": time step beyond the RK3 stability limit of the advection: Courant number " +
                                     std::to_string(courant) + " > " + std::to_string(lim) + at);
    if (!p.collisionless) {
      const double T = p.T_w, n = p.n0;
      const double tau = p.law == HRLB_LAW_POWER        ? p.kn * std::pow(T, p.omega - 1.0) / n
                         : p.law == HRLB_LAW_SUTHERLAND ? p.kn * (1.0 + p.suth_S) / (n * std::sqrt(T) * (1.0 + p.suth_S / T))
                                                        : p.kn / std::sqrt(2.0);
      if (p.dt / tau > RELAX_RK3)
        return fail(HRLB_ENUMERIC, std::string(fn) + ": time step beyond the RK3 stability limit of the relaxation: dt / tau = " +
                                       std::to_string(p.dt / tau) + " > " + std::to_string(RELAX_RK3) + at);
    }
  }
  return HRLB_OK;
}

// Device pointers of a work region laid out by L and of the three population arrays.
static DevPtrs carve(const WorkLayout& L, char* w, char* state, size_t arr) {
  DevPtrs d;
  d.px = (const double*)(w + L.px);
  d.py = (const double*)(w + L.py);
  d.pz = (const double*)(w + L.pz);
  d.phix = (const double*)(w + L.phix);
  d.cx = (const double*)(w + L.cx);
  d.phiy = (const double*)(w + L.phiy);
  d.phiz = (const double*)(w + L.phiz);
  d.ptab = (double*)(w + L.ptab);
  d.inst = (InstDev*)(w + L.inst);
  d.inv_dx = (double*)(w + L.inv_dx);
  d.g_rest = (double*)(w + L.g_rest);
  d.g_wall = (double*)(w + L.g_wall);
  d.partials = (double*)(w + L.partials);
  d.rec = (double*)(w + L.rec);
  d.nw = (double*)(w + L.nw);
  d.resid_part = (double*)(w + L.resid_part);
  d.resid = (double*)(w + L.resid);
  d.flags = (int*)(w + L.flags);
  d.junk = (double*)(w + L.junk);
  for (int k = 0; k < 3; ++k) d.F[k] = (double*)(state + k * arr);
  return d;
}

// Upload the velocity-set tables and the per-instance constants (collision parameters,
// Lagrange weights of the wall extrapolation, 1/dx of every node) on st, clear the fault
// flags and residuals with a fill kernel, and synchronise st (the host staging vectors die
// on return).  Then fill the equilibrium tables on the device.
static hipError_t upload_tables(const QuadTables& t, const Shape& sh, const hrlb_params* params, const DevPtrs& d,
                                hipStream_t st) {
  const int batch = sh.B, S = sh.S;
  std::vector<InstDev> inst(batch);
  std::vector<double> invdx((size_t)batch * S);
  for (int b = 0; b < batch; ++b) {
    const hrlb_params& p = params[b];
    InstDev& I = inst[b];
    std::memset(&I, 0, sizeof(I));
    I.dt = p.dt;
    I.kn = p.kn;
    I.omega = p.omega;
    I.suth = p.suth_S;
    I.pr = p.pr;
    I.n0 = p.n0;
    I.T_w = p.T_w;
    I.u_w = p.u_w;
    I.law = p.law;
    I.collisionless = p.collisionless ? 1.0 : 0.0;
    // Lagrange weights of App. A.4: node S+1 from S, S-1, S-2 and node S+2 from S+1, S, S-1 (1-based)
    for (int g = 0; g < 2; ++g) {
      const double xs = node_x(S + 1 + g, S, p.A);
      const double x1 = node_x(S + g, S, p.A), x2 = node_x(S - 1 + g, S, p.A), x3 = node_x(S - 2 + g, S, p.A);
      I.ex[3 * g + 0] = (xs - x2) * (xs - x3) / ((x1 - x2) * (x1 - x3));
      I.ex[3 * g + 1] = (xs - x1) * (xs - x3) / ((x2 - x1) * (x2 - x3));
      I.ex[3 * g + 2] = (xs - x1) * (xs - x2) / ((x3 - x1) * (x3 - x2));
    }
    for (int c = 0; c < S; ++c) {
      const double dx = node_x(c + 1.5, S, p.A) - node_x(c + 0.5, S, p.A);
      invdx[(size_t)b * S + c] = 1.0 / dx;
    }
  }
  auto up = [&](const void* dst, const void* src, size_t bytes) {
    return hipMemcpyAsync((void*)dst, src, bytes, hipMemcpyHostToDevice, st);
  };
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = up(d.px, t.px.data(), t.px.size() * sizeof(double));
  if (e == hipSuccess) e = up(d.py, t.py.data(), t.py.size() * sizeof(double));
  if (e == hipSuccess) e = up(d.pz, t.pz.data(), t.pz.size() * sizeof(double));
  if (e == hipSuccess) e = up(d.phix, t.phix.data(), t.phix.size() * sizeof(double));
  if (e == hipSuccess) e = up(d.cx, t.cx.data(), t.cx.size() * sizeof(double));
  if (e == hipSuccess) e = up(d.phiy, t.phiy.data(), t.phiy.size() * sizeof(double));
  if (e == hipSuccess) e = up(d.phiz, t.phiz.data(), t.phiz.size() * sizeof(double));
  if (e == hipSuccess) e = up(d.inst, inst.data(), inst.size() * sizeof(InstDev));
  if (e == hipSuccess) e = up(d.inv_dx, invdx.data(), invdx.size() * sizeof(double));
  if (e == hipSuccess) e = (hipError_t)launch_clear_flags(sh, d, st);
  // the host vectors above must stay alive until the copies complete
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e == hipSuccess) e = (hipError_t)launch_setup_tables(sh, d, st);
  return e;
}

int hrlb_init_state(const hrlb_quad* q, int S, int scheme, const hrlb_params* params, int batch, void* d_state,
                    size_t state_bytes, void* d_work, size_t work_bytes, void* stream, const double* d_perturb,
                    double eps, hrlb_sim** out) {
  if (!out) return fail(HRLB_EINVAL, "init_state: out is NULL");
  *out = nullptr;
  Range r_call("hrlb_init_state");
  if (!q || !params || !d_state || !d_work) return fail(HRLB_EINVAL, "init_state: NULL argument");
  int rc = check_instances("init_state", S, scheme, params, batch);
  if (rc != HRLB_OK) return rc;
  if (((uintptr_t)d_state & 255) || ((uintptr_t)d_work & 255))
    return fail(HRLB_EINVAL, "init_state: buffers must be 256-byte aligned");
  const Shape sh = make_shape(q->t, S, batch, scheme);
  if (!instance_fits(sh)) return fail(HRLB_EINVAL, "init_state: one instance's populations (S * V * 8 bytes) must stay below 4 GiB");
  if ((rc = check_stability("init_state", q->t, S, scheme, params, batch)) != HRLB_OK) return rc;
  const WorkLayout L = work_layout(sh);
  const size_t arr = align256((size_t)batch * S * sh.V * sizeof(double));
  if (state_bytes < 3 * arr) return fail(HRLB_ENOMEM, "init_state: state buffer smaller than hrlb_state_bytes");
  if (work_bytes < L.total) return fail(HRLB_ENOMEM, "init_state: work buffer smaller than hrlb_state_bytes");

  hrlb_sim* s = new hrlb_sim;
  s->sh = sh;
  s->lay = L;
  s->stream = (hipStream_t)stream;
  s->cells = default_cells(sh);
  s->waves = default_waves(sh);
  s->part_nvb = 0;
  s->resid_nres = 0;
  s->timing = false;
  s->graph_on = false;
  s->gexec = s->gexec_k = nullptr;
  s->cap_stream = nullptr;
  s->g_cells = s->g_waves = 0;
  for (int k = 0; k < 4; ++k) {
    s->ms[k] = 0;
    s->launches[k] = 0;
  }
  s->d = carve(L, (char*)d_work, (char*)d_state, arr);
  const DevPtrs& d = s->d;
  hipStream_t st = s->stream;
  hipError_t e = upload_tables(q->t, sh, params, d, st);
  if (e != hipSuccess) {
    delete s;
    return hip_fail(e, "init_state: table upload");
  }
  if ((e = (hipError_t)launch_init_state(sh, d, d_perturb, eps, st)) != hipSuccess ||
      (e = (hipError_t)launch_partials(sh, d, d.F[0], s->cells, s->waves, st)) != hipSuccess) {
    delete s;
    return hip_fail(e, "init_state: launch");
  }
  s->part_nvb = (sh.V + 64 * s->waves - 1) / (64 * s->waves);
  *out = s;
  return HRLB_OK;
}

int hrlb_step_noalloc(const hrlb_quad* q, int S, int scheme, const hrlb_params* params, int batch, void* d_state,
                      size_t state_bytes, int nsteps, double* d_moments, void* stream) {
  if (!q || !params || !d_state) return fail(HRLB_EINVAL, "step_noalloc: NULL argument");
  if (nsteps < 0) return fail(HRLB_EINVAL, "step_noalloc: nsteps must be >= 0");
  Range r_call("hrlb_step_noalloc");
  int rc = check_instances("step_noalloc", S, scheme, params, batch);
  if (rc != HRLB_OK) return rc;
  if ((uintptr_t)d_state & 255) return fail(HRLB_EINVAL, "step_noalloc: state buffer must be 256-byte aligned");
  const Shape sh = make_shape(q->t, S, batch, scheme);
  if (!instance_fits(sh))
    return fail(HRLB_EINVAL, "step_noalloc: one instance's populations (S * V * 8 bytes) must stay below 4 GiB");
  if ((rc = check_stability("step_noalloc", q->t, S, scheme, params, batch)) != HRLB_OK) return rc;
  const WorkLayout L = work_layout(sh);
  if (L.total > SCRATCH_BYTES)
    return fail(HRLB_ENOMEM, "step_noalloc: this batch needs " + std::to_string(L.total) +
                                 " bytes of work memory, more than the fixed array's " + std::to_string(SCRATCH_BYTES) +
                                 " (HRLB_SCRATCH_BYTES); use hrlb_init_state with a work buffer, or fewer instances");
  const size_t arr = align256((size_t)batch * S * sh.V * sizeof(double));
  if (state_bytes < 3 * arr) return fail(HRLB_ENOMEM, "step_noalloc: state buffer smaller than hrlb_state_bytes");
  void* work = nullptr;
  hipError_t e = (hipError_t)scratch_pointer(&work);
  if (e != hipSuccess) return hip_fail(e, "step_noalloc: address of the fixed work array");
  const DevPtrs d = carve(L, (char*)work, (char*)d_state, arr);
  hipStream_t st = (hipStream_t)stream;
  e = upload_tables(q->t, sh, params, d, st);
  if (e != hipSuccess) return hip_fail(e, "step_noalloc: table upload");
  // the launch sequence of hrlb_init_state (partials of the current state) and of the eager
  // hrlb_step with the default launch shape, so the results equal that path's
  const int cells = default_cells(sh), waves = default_waves(sh);
  const int nvb = (sh.V + 64 * waves - 1) / (64 * waves);
  e = (hipError_t)launch_partials(sh, d, d.F[0], cells, waves, st);
  for (int n = 0; n < nsteps && e == hipSuccess; ++n)
    for (int stage = 1; stage <= 3 && e == hipSuccess; ++stage) {
      const double* Fin = d.F[stage - 1];
      double* Fout = d.F[stage % 3];
      e = (hipError_t)launch_closure(sh, d, Fin, nvb, nullptr, st);
      if (e == hipSuccess) e = (hipError_t)launch_stage(sh, d, stage, Fin, d.F[0], Fout, cells, waves, st);
    }
  if (e == hipSuccess && d_moments) {
    e = (hipError_t)launch_partials(sh, d, d.F[0], cells, waves, st);
    if (e == hipSuccess) e = (hipError_t)launch_closure(sh, d, d.F[0], nvb, d_moments, st);
  }
  if (e != hipSuccess) return hip_fail(e, "step_noalloc: launch");
  return HRLB_OK;
}

void hrlb_sim_free(hrlb_sim* s) {
  if (!s) return;
  for (hipEvent_t e : s->ev) (void)hipEventDestroy(e);
  if (s->gexec) (void)hipGraphExecDestroy(s->gexec);
  if (s->gexec_k) (void)hipGraphExecDestroy(s->gexec_k);
  if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
  delete s;
}

static hipError_t ev_begin(hrlb_sim* s, hipEvent_t* e0) {
  if (!s->timing) return hipSuccess;
  hipError_t e = hipEventCreate(e0);
  if (e == hipSuccess) e = hipEventRecord(*e0, s->stream);
  return e;
}

static hipError_t ev_end(hrlb_sim* s, hipEvent_t e0, int kind) {
  if (!s->timing) return hipSuccess;
  hipEvent_t e1;
  hipError_t e = hipEventCreate(&e1);
  if (e == hipSuccess) e = hipEventRecord(e1, s->stream);
  if (e == hipSuccess) {
    s->ev.push_back(e0);
    s->ev.push_back(e1);
    s->ev_kind.push_back(kind);
  }
  return e;
}

// enqueue the six launches of one RK3 step on `st` (no timing events)
static hipError_t enqueue_step(hrlb_sim* s, hipStream_t st, int part_nvb) {
  const Shape& sh = s->sh;
  DevPtrs& d = s->d;
  const int nvb = (sh.V + 64 * s->waves - 1) / (64 * s->waves);
  hipError_t e = hipSuccess;
  for (int stage = 1; stage <= 3 && e == hipSuccess; ++stage) {
    const double* Fin = d.F[stage - 1];
    double* Fout = d.F[stage % 3];  // stage 1 -> F[1], 2 -> F[2], 3 -> F[0] (in place over F_l)
    e = (hipError_t)launch_closure(sh, d, Fin, stage == 1 ? part_nvb : nvb, nullptr, st);
    if (e == hipSuccess) e = (hipError_t)launch_stage(sh, d, stage, Fin, d.F[0], Fout, s->cells, s->waves, st);
  }
  return e;
}

// Steps captured in the long graph.  Each graph launch costs the GPU an idle gap at the
// launch boundary (8.5 us measured between replays of a one-step graph, none between the
// kernels inside a graph), so runs of many steps replay GRAPH_BLOCK steps per launch.
constexpr int GRAPH_BLOCK = 8;

// capture `nsteps` RK3 steps of the sim's current launch shape into *out (replaced)
static hipError_t capture_steps(hrlb_sim* s, int nsteps, hipGraphExec_t* out) {
  hipError_t e = hipSuccess;
  if (*out) {
    (void)hipGraphExecDestroy(*out);
    *out = nullptr;
  }
  if (!s->cap_stream) e = hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking);
  if (e != hipSuccess) return e;
  const int nvb = (s->sh.V + 64 * s->waves - 1) / (64 * s->waves);
  hipGraph_t g = nullptr;
  e = hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  hipError_t el = hipSuccess;
  for (int k = 0; k < nsteps && el == hipSuccess; ++k) el = enqueue_step(s, s->cap_stream, nvb);
  e = hipStreamEndCapture(s->cap_stream, &g);
  if (el != hipSuccess) e = el;
  if (e == hipSuccess) e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  return e;
}

int hrlb_step(hrlb_sim* s, int nsteps) {
  if (!s) return fail(HRLB_EINVAL, "step: sim is NULL");
  if (nsteps < 0) return fail(HRLB_EINVAL, "step: nsteps must be >= 0");
  Range r_call("hrlb_step");
  const Shape& sh = s->sh;
  DevPtrs& d = s->d;
  const int nvb = (sh.V + 64 * s->waves - 1) / (64 * s->waves);
  const int nch = (sh.S + s->cells - 1) / s->cells;
  int n = 0;
  if (s->graph_on && !s->timing) {
    // the captured step expects partials laid out by its own launch shape; one eager step
    // re-lays them out after an init, set_state, moments or shape change
    if (s->part_nvb != nvb && nsteps > 0) {
      hipError_t e = enqueue_step(s, s->stream, s->part_nvb);
      if (e != hipSuccess) return hip_fail(e, "step: launch");
      s->part_nvb = nvb;
      s->resid_nres = nvb * nch;
      n = 1;
    }
    if (n < nsteps && (s->g_cells != s->cells || s->g_waves != s->waves)) {
      // a new launch shape: both graphs are captured again when next needed
      for (hipGraphExec_t* x : {&s->gexec, &s->gexec_k})
        if (*x) {
          (void)hipGraphExecDestroy(*x);
          *x = nullptr;
        }
      s->g_cells = s->cells;
      s->g_waves = s->waves;
    }
    if (nsteps - n >= GRAPH_BLOCK && !s->gexec_k) {
      hipError_t e = capture_steps(s, GRAPH_BLOCK, &s->gexec_k);
      if (e != hipSuccess) return hip_fail(e, "step: graph capture");
    }
    for (; nsteps - n >= GRAPH_BLOCK; n += GRAPH_BLOCK) {
      Range r_step("RK3 steps (graph launch)");
      hipError_t e = hipGraphLaunch(s->gexec_k, s->stream);
      if (e != hipSuccess) return hip_fail(e, "step: graph launch");
      s->resid_nres = nvb * nch;
    }
    if (n < nsteps && !s->gexec) {
      hipError_t e = capture_steps(s, 1, &s->gexec);
      if (e != hipSuccess) return hip_fail(e, "step: graph capture");
    }
    for (; n < nsteps; ++n) {
      Range r_step("RK3 step (graph launch)");
      hipError_t e = hipGraphLaunch(s->gexec, s->stream);
      if (e != hipSuccess) return hip_fail(e, "step: graph launch");
      s->resid_nres = nvb * nch;
    }
    return HRLB_OK;
  }
  for (; n < nsteps; ++n) {
    for (int stage = 1; stage <= 3; ++stage) {
      const double* Fin = d.F[stage - 1];
      double* Fout = d.F[stage % 3];  // stage 1 -> F[1], 2 -> F[2], 3 -> F[0] (in place over F_l)
      hipEvent_t e0 = nullptr;
      hipError_t e = ev_begin(s, &e0);
      {
        Range r_cl("closure");
        if (e == hipSuccess) e = (hipError_t)launch_closure(sh, d, Fin, s->part_nvb, nullptr, s->stream);
      }
      if (e == hipSuccess) e = ev_end(s, e0, 3);
      if (e == hipSuccess) e = ev_begin(s, &e0);
      {
        Range r_st(STAGE_RANGE[stage - 1]);
        if (e == hipSuccess)
          e = (hipError_t)launch_stage(sh, d, stage, Fin, d.F[0], Fout, s->cells, s->waves, s->stream);
      }
      if (e == hipSuccess) e = ev_end(s, e0, stage - 1);
      if (e != hipSuccess) return hip_fail(e, "step: launch");
      s->part_nvb = nvb;
    }
    s->resid_nres = nvb * nch;
  }
  return HRLB_OK;
}

static std::string tune_key(const Shape& sh) {
  std::ostringstream k;
  k << "Qx" << sh.Qx << "_Qy" << sh.Qy << "_Qz" << sh.Qz << "_S" << sh.S << "_B" << sh.B << "_scheme" << sh.scheme;
  return k.str();
}

// cache file: one JSON object per line, {"key": "...", "cells": c, "waves": w, "ms": t}
static bool tune_lookup(const char* path, const std::string& key, int* cells, int* waves) {
  if (!path) return false;
  std::ifstream f(path);
  std::string line;
  bool found = false;
  while (std::getline(f, line)) {
    const std::string tag = "\"key\": \"" + key + "\"";
    if (line.find(tag) == std::string::npos) continue;
    int c = 0, w = 0;
    const size_t pc = line.find("\"cells\":"), pw = line.find("\"waves\":");
    if (pc == std::string::npos || pw == std::string::npos) continue;
    if (std::sscanf(line.c_str() + pc + 8, "%d", &c) == 1 && std::sscanf(line.c_str() + pw + 8, "%d", &w) == 1 &&
        c >= 1 && w >= 1 && w <= MAX_WAVES) {
      *cells = c;
      *waves = w;
      found = true;  // the last entry for a key wins
    }
  }
  return found;
}

int hrlb_autotune(hrlb_sim* s, int probe_steps, const char* cache_path, int* best_cells, int* best_waves,
                  double* best_ms) {
  if (!s || !best_cells || !best_waves || !best_ms) return fail(HRLB_EINVAL, "autotune: NULL argument");
  if (probe_steps < 1) return fail(HRLB_EINVAL, "autotune: probe_steps must be >= 1");
  Range r_call("hrlb_autotune");
  const std::string key = tune_key(s->sh);
  int c = 0, w = 0;
  if (tune_lookup(cache_path, key, &c, &w)) {
    s->cells = c;
    s->waves = w;
    *best_cells = c;
    *best_waves = w;
    *best_ms = -1.0;
    return HRLB_OK;
  }
  const bool graph = s->graph_on, timing = s->timing;
  s->timing = false;
  s->graph_on = true;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0), "autotune: event");
  HIP_TRY(hipEventCreate(&e1), "autotune: event");
  const int cells_c[] = {2, 4, 8, 16, 32, 48, 64, 96, 128};
  // time one shape: two untimed steps (they re-lay the partials and capture this shape's
  // graph), then probe_steps timed graph replays
  auto time_shape = [&](int ci, int wv, double* per) -> int {
    s->cells = ci;
    s->waves = wv;
    int r = hrlb_step(s, 2);
    if (r != HRLB_OK) return r;
    hipError_t e = hipEventRecord(e0, s->stream);
    if (e == hipSuccess) {
      r = hrlb_step(s, probe_steps);
      if (r != HRLB_OK) return r;
      e = hipEventRecord(e1, s->stream);
    }
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) return hip_fail(e, "autotune: timing");
    *per = ms / probe_steps;
    return HRLB_OK;
  };
  struct Cand {
    double per;
    int cells, waves;
  };
  std::vector<Cand> cand;
  int rc = HRLB_OK;
  for (int wv = 1; wv <= MAX_WAVES && rc == HRLB_OK; ++wv)
    for (int ci : cells_c) {
      if (ci > 2 * s->sh.S) continue;
      double per = 0;
      rc = time_shape(ci, wv, &per);
      if (rc != HRLB_OK) break;
      cand.push_back({per, ci, wv});
    }
  // a second timing of the three fastest, each keeping its better time, so one noisy probe
  // does not decide
  if (rc == HRLB_OK) {
    std::sort(cand.begin(), cand.end(), [](const Cand& a, const Cand& b) { return a.per < b.per; });
    for (size_t k = 0; k < cand.size() && k < 3 && rc == HRLB_OK; ++k) {
      double per = 0;
      rc = time_shape(cand[k].cells, cand[k].waves, &per);
      cand[k].per = std::min(cand[k].per, per);
    }
  }
  double best = 1e300;
  int bc = s->cells, bw = s->waves;
  for (const Cand& c2 : cand)
    if (c2.per < best) {
      best = c2.per;
      bc = c2.cells;
      bw = c2.waves;
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  s->cells = bc;
  s->waves = bw;
  s->graph_on = graph;
  s->timing = timing;
  if (rc != HRLB_OK) return rc;
  *best_cells = bc;
  *best_waves = bw;
  *best_ms = best;
  if (cache_path) {
    std::ofstream f(cache_path, std::ios::app);
    f << "{\"key\": \"" << key << "\", \"cells\": " << bc << ", \"waves\": " << bw << ", \"ms\": " << best << "}\n";
  }
  return HRLB_OK;
}

// ---- batches of sims (ragged sweeps) ---------------------------------------------------

static int device_cus() {
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    ncu = 256;
  return ncu;
}

// Nodes per closure block of a batch, one count for all its groups: the smallest of
// 4, 8, 16 for which every closure item of the batch (the node blocks of each group plus
// one wall item per instance) is resident at once, so the closure launch runs in a single
// round (its time is then one block's critical path, and fewer nodes per block shorten that
// path); 16 when none is.  Larger blocks would keep a big batch in one round, but measured
// on single groups of 65 536 and 262 144 nodes, 16-node blocks in several rounds beat
// 32- and 64-node blocks, whose LDS leaves fewer blocks per CU.
static int batch_closure_nodes(hrlb_sim* const* sims, int nsims) {
  const long long ncu = device_cus();
  for (int nb = 4;; nb *= 2) {
    long long items = 0;
    size_t lds = 0;
    for (int k = 0; k < nsims; ++k) {
      const Shape& sh = sims[k]->sh;
      items += ((long long)sh.B * sh.S + nb - 1) / nb + sh.B;
      lds = std::max(lds, closure_lds_bytes_for(sh, nb));
    }
    if (nb == CL_NODES || items <= ncu * batch_closure_blocks_per_cu(lds)) return nb;
  }
}

static void batch_sizes(hrlb_sim* const* sims, int nsims, int cells, int waves, int nb, int* max_tiles,
                        int* max_items) {
  long long t = 0, it = 0;
  for (int k = 0; k < nsims; ++k) {
    const Shape& sh = sims[k]->sh;
    const int nvb = (sh.V + 64 * waves - 1) / (64 * waves), nch = (sh.S + cells - 1) / cells;
    t += (long long)sh.B * nvb * nch;
    const int total = sh.B * sh.S;
    it += (total + nb - 1) / nb + sh.B;
  }
  *max_tiles = (int)t;
  *max_items = (int)it;
}

static size_t batch_bytes_of(int nsims, int max_tiles, int max_items) {
  return align256(nsims * sizeof(GroupDesc)) + align256((size_t)max_tiles * 4 * sizeof(int)) + 256 +
         align256((size_t)max_items * 2 * sizeof(int)) + 256;
}

static int batch_check(hrlb_sim* const* sims, int nsims, int cells, int waves) {
  if (!sims || nsims < 1) return fail(HRLB_EINVAL, "batch: need at least one sim");
  for (int k = 0; k < nsims; ++k)
    if (!sims[k]) return fail(HRLB_EINVAL, "batch: NULL sim");
  if (cells < 1 || cells > 4096) return fail(HRLB_EINVAL, "batch: cells must be in 1..4096");
  if (waves < 1 || waves > MAX_WAVES) return fail(HRLB_EINVAL, "batch: waves must be in 1..4");
  return HRLB_OK;
}

int hrlb_batch_bytes(hrlb_sim* const* sims, int nsims, int cells, int waves, size_t* bytes) {
  if (!bytes) return fail(HRLB_EINVAL, "batch_bytes: NULL argument");
  int rc = batch_check(sims, nsims, cells, waves);
  if (rc != HRLB_OK) return rc;
  int mt, mi;
  batch_sizes(sims, nsims, cells, waves, batch_closure_nodes(sims, nsims), &mt, &mi);
  *bytes = batch_bytes_of(nsims, mt, mi);
  return HRLB_OK;
}

// rewrite the tile and closure-item tables from the active flags (stream-ordered upload,
// then synchronise so the host staging vectors may be released).  A retired instance keeps
// no stage tile and no wall item; a closure node block stays while any instance it covers
// is active.
static int batch_upload_tables(hrlb_batch* bt) {
  std::vector<int> items;
  items.reserve((size_t)bt->max_items * 2);
  for (size_t k = 0; k < bt->sims.size(); ++k) {
    const Shape& sh = bt->sims[k]->sh;
    const int* act = bt->active.data() + bt->inst_offset[k];
    const long long total = (long long)sh.B * sh.S;
    const int node_blocks = (int)((total + bt->nb - 1) / bt->nb);
    for (int blk = 0; blk < node_blocks; ++blk) {
      const long long g0 = (long long)blk * bt->nb, g1 = std::min(total, g0 + bt->nb) - 1;
      bool any = false;
      for (long long b = g0 / sh.S; b <= g1 / sh.S && !any; ++b) any = act[b] != 0;
      if (!any) continue;
      items.push_back((int)k);
      items.push_back(blk);
    }
    for (int b = 0; b < sh.B; ++b) {
      if (!act[b]) continue;
      items.push_back((int)k);
      items.push_back(node_blocks + b);
    }
  }
  bt->nitems = (int)(items.size() / 2);
  if (!items.empty())
    HIP_TRY(hipMemcpyAsync(bt->d_items, items.data(), items.size() * sizeof(int), hipMemcpyHostToDevice, bt->stream),
            "batch: item upload");
  HIP_TRY(hipMemcpyAsync(bt->d_nitems, &bt->nitems, sizeof(int), hipMemcpyHostToDevice, bt->stream), "batch: item upload");
  std::vector<int> tiles;
  tiles.reserve((size_t)bt->max_tiles * 4);
  for (size_t k = 0; k < bt->sims.size(); ++k) {
    const Shape& sh = bt->sims[k]->sh;
    const int nvb = (sh.V + 64 * bt->waves - 1) / (64 * bt->waves), nch = (sh.S + bt->cells - 1) / bt->cells;
    for (int b = 0; b < sh.B; ++b) {
      if (!bt->active[bt->inst_offset[k] + b]) continue;
      for (int vb = 0; vb < nvb; ++vb)
        for (int ch = 0; ch < nch; ++ch) {
          tiles.push_back((int)k);
          tiles.push_back(b);
          tiles.push_back(vb);
          tiles.push_back(ch);
        }
    }
  }
  bt->ntiles = (int)(tiles.size() / 4);
  if (!tiles.empty())
    HIP_TRY(hipMemcpyAsync(bt->d_tiles, tiles.data(), tiles.size() * sizeof(int), hipMemcpyHostToDevice, bt->stream),
            "batch: tile upload");
  HIP_TRY(hipMemcpyAsync(bt->d_ntiles, &bt->ntiles, sizeof(int), hipMemcpyHostToDevice, bt->stream), "batch: tile upload");
  HIP_TRY(hipStreamSynchronize(bt->stream), "batch: tile upload");
  return HRLB_OK;
}

int hrlb_batch_create(hrlb_sim* const* sims, int nsims, int cells, int waves, void* d_work, size_t work_bytes,
                      void* stream, hrlb_batch** out) {
  if (!out) return fail(HRLB_EINVAL, "batch_create: out is NULL");
  *out = nullptr;
  int rc = batch_check(sims, nsims, cells, waves);
  if (rc != HRLB_OK) return rc;
  if (!d_work || ((uintptr_t)d_work & 255)) return fail(HRLB_EINVAL, "batch_create: work buffer NULL or misaligned");
  int mt, mi;
  const int nb = batch_closure_nodes(sims, nsims);
  batch_sizes(sims, nsims, cells, waves, nb, &mt, &mi);
  if (work_bytes < batch_bytes_of(nsims, mt, mi)) return fail(HRLB_ENOMEM, "batch_create: work buffer too small");
  for (int a = 0; a < nsims; ++a)
    for (int b = a + 1; b < nsims; ++b)
      if (sims[a] == sims[b]) return fail(HRLB_EINVAL, "batch_create: a sim appears twice");
  hrlb_batch* bt = new hrlb_batch;
  bt->sims.assign(sims, sims + nsims);
  bt->cells = cells;
  bt->waves = waves;
  bt->stream = (hipStream_t)stream;
  bt->max_tiles = mt;
  bt->max_items = mi;
  bt->nb = nb;
  bt->gexec = bt->gexec_k = nullptr;
  bt->cap_stream = nullptr;
  char* w = (char*)d_work;
  bt->d_groups = (GroupDesc*)w;
  w += align256(nsims * sizeof(GroupDesc));
  bt->d_tiles = (int*)w;
  w += align256((size_t)mt * 4 * sizeof(int));
  bt->d_ntiles = (int*)w;
  w += 256;
  bt->d_items = (int*)w;
  w += align256((size_t)mi * 2 * sizeof(int));
  bt->d_nitems = (int*)w;
  std::vector<GroupDesc> groups(nsims);
  int total_inst = 0;
  bt->lds_closure = 0;
  for (int k = 0; k < nsims; ++k) {
    hrlb_sim* sm = sims[k];
    // every instance of the group advances with the batch's launch shape; re-lay the
    // moment partials of the current state accordingly (on the batch's stream)
    hipError_t e = (hipError_t)launch_partials(sm->sh, sm->d, sm->d.F[0], cells, waves, bt->stream);
    if (e != hipSuccess) {
      delete bt;
      return hip_fail(e, "batch_create: partials");
    }
    sm->cells = cells;
    sm->waves = waves;
    GroupDesc& g = groups[k];
    std::memset(&g, 0, sizeof(g));
    g.sh = sm->sh;
    g.d = sm->d;
    g.nvb = (sm->sh.V + 64 * waves - 1) / (64 * waves);
    g.nch = (sm->sh.S + cells - 1) / cells;
    g.cs = cells;
    const int total = sm->sh.B * sm->sh.S;
    g.nb = nb;
    g.node_blocks = (total + g.nb - 1) / g.nb;
    sm->part_nvb = g.nvb;
    bt->lds_closure = std::max(bt->lds_closure, closure_lds_bytes_for(sm->sh, g.nb));
    bt->inst_offset.push_back(total_inst);
    total_inst += sm->sh.B;
  }
  bt->active.assign(total_inst, 1);
  bt->lds_stage = stage_lds_bytes_for(waves);
  hipError_t e = hipMemcpyAsync(bt->d_groups, groups.data(), nsims * sizeof(GroupDesc), hipMemcpyHostToDevice, bt->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(bt->stream);
  if (e != hipSuccess) {
    delete bt;
    return hip_fail(e, "batch_create: upload");
  }
  if ((rc = batch_upload_tables(bt)) != HRLB_OK) {
    delete bt;
    return rc;
  }
  // one block per tile and per closure item (blocks past the live counts return)
  bt->grid_stage = std::max(1, mt);
  bt->grid_closure = std::max(1, mi);
  *out = bt;
  return HRLB_OK;
}

static hipError_t batch_enqueue_step(hrlb_batch* bt, hipStream_t st) {
  hipError_t e = hipSuccess;
  for (int stage = 1; stage <= 3 && e == hipSuccess; ++stage) {
    e = (hipError_t)launch_batch_closure(stage, bt->d_groups, bt->d_items, bt->d_nitems, bt->grid_closure,
                                         bt->lds_closure, st);
    if (e == hipSuccess)
      e = (hipError_t)launch_batch_stage(stage, bt->d_groups, bt->d_tiles, bt->d_ntiles, bt->grid_stage, bt->waves,
                                         bt->lds_stage, st);
  }
  return e;
}

int hrlb_batch_step(hrlb_batch* bt, int nsteps) {
  if (!bt) return fail(HRLB_EINVAL, "batch_step: batch is NULL");
  if (nsteps < 0) return fail(HRLB_EINVAL, "batch_step: nsteps must be >= 0");
  if (nsteps == 0) return HRLB_OK;
  Range r_call("hrlb_batch_step");
  // one captured step, and GRAPH_BLOCK steps per launch for long runs (as hrlb_step)
  auto capture = [&](int k, hipGraphExec_t* out) -> hipError_t {
    hipError_t e = hipSuccess;
    if (!bt->cap_stream) e = hipStreamCreateWithFlags(&bt->cap_stream, hipStreamNonBlocking);
    hipGraph_t g = nullptr;
    if (e == hipSuccess) e = hipStreamBeginCapture(bt->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      hipError_t el = hipSuccess;
      for (int i = 0; i < k && el == hipSuccess; ++i) el = batch_enqueue_step(bt, bt->cap_stream);
      e = hipStreamEndCapture(bt->cap_stream, &g);
      if (el != hipSuccess) e = el;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    return e;
  };
  if (nsteps % GRAPH_BLOCK && !bt->gexec) {
    hipError_t e = capture(1, &bt->gexec);
    if (e != hipSuccess) return hip_fail(e, "batch_step: graph capture");
  }
  if (nsteps >= GRAPH_BLOCK && !bt->gexec_k) {
    hipError_t e = capture(GRAPH_BLOCK, &bt->gexec_k);
    if (e != hipSuccess) return hip_fail(e, "batch_step: graph capture");
  }
  // a sim stepped on its own or by another batch since may hold moment partials laid out
  // for another wave count: re-lay them from the current state first
  for (hrlb_sim* sm : bt->sims) {
    const int nvb = (sm->sh.V + 64 * bt->waves - 1) / (64 * bt->waves);
    if (sm->part_nvb != nvb)
      HIP_TRY((hipError_t)launch_partials(sm->sh, sm->d, sm->d.F[0], bt->cells, bt->waves, bt->stream),
              "batch_step: partials");
  }
  int n = 0;
  for (; nsteps - n >= GRAPH_BLOCK; n += GRAPH_BLOCK) {
    Range r_step("batched RK3 steps (graph launch)");
    HIP_TRY(hipGraphLaunch(bt->gexec_k, bt->stream), "batch_step: graph launch");
  }
  for (; n < nsteps; ++n) {
    Range r_step("batched RK3 step (graph launch)");
    HIP_TRY(hipGraphLaunch(bt->gexec, bt->stream), "batch_step: graph launch");
  }
  for (hrlb_sim* sm : bt->sims) {
    const int nvb = (sm->sh.V + 64 * bt->waves - 1) / (64 * bt->waves), nch = (sm->sh.S + bt->cells - 1) / bt->cells;
    sm->part_nvb = nvb;
    sm->resid_nres = nvb * nch;
  }
  return HRLB_OK;
}

int hrlb_batch_residual(hrlb_batch* bt, double* h_out) {
  if (!bt || !h_out) return fail(HRLB_EINVAL, "batch_residual: NULL argument");
  Range r_call("hrlb_batch_residual");
  std::vector<int> flags(bt->active.size());
  for (size_t k = 0; k < bt->sims.size(); ++k) {
    hrlb_sim* sm = bt->sims[k];
    if (sm->resid_nres > 0) {
      hipError_t e = (hipError_t)launch_residual(sm->sh, sm->d, sm->resid_nres, bt->stream);
      if (e != hipSuccess) return hip_fail(e, "batch_residual: launch");
    }
    const int o = bt->inst_offset[k];
    HIP_TRY(hipMemcpyAsync(h_out + o, sm->d.resid, sm->sh.B * sizeof(double), hipMemcpyDeviceToHost, bt->stream),
            "batch_residual: copy");
    HIP_TRY(hipMemcpyAsync(flags.data() + o, sm->d.flags, sm->sh.B * sizeof(int), hipMemcpyDeviceToHost, bt->stream),
            "batch_residual: copy");
  }
  HIP_TRY(hipStreamSynchronize(bt->stream), "batch_residual: synchronize");
  for (size_t i = 0; i < flags.size(); ++i)
    if (flags[i]) return fail(HRLB_ENUMERIC, "batch_residual: instance " + std::to_string(i) + " met n <= 0, T <= 0 or a non-finite moment");
  return HRLB_OK;
}

int hrlb_batch_set_active(hrlb_batch* bt, const int* active) {
  if (!bt || !active) return fail(HRLB_EINVAL, "batch_set_active: NULL argument");
  for (size_t i = 0; i < bt->active.size(); ++i) bt->active[i] = active[i] ? 1 : 0;
  return batch_upload_tables(bt);
}

int hrlb_batch_info(const hrlb_batch* bt, int* ntiles, int* nitems, int* grid_stage, int* grid_closure) {
  if (!bt || !ntiles || !nitems || !grid_stage || !grid_closure) return fail(HRLB_EINVAL, "batch_info: NULL argument");
  *ntiles = bt->ntiles;
  *nitems = bt->nitems;
  *grid_stage = bt->grid_stage;
  *grid_closure = bt->grid_closure;
  return HRLB_OK;
}

void hrlb_batch_free(hrlb_batch* bt) {
  if (!bt) return;
  if (bt->gexec) (void)hipGraphExecDestroy(bt->gexec);
  if (bt->gexec_k) (void)hipGraphExecDestroy(bt->gexec_k);
  if (bt->cap_stream) (void)hipStreamDestroy(bt->cap_stream);
  delete bt;
}

int hrlb_set_graph(hrlb_sim* s, int on) {
  if (!s) return fail(HRLB_EINVAL, "set_graph: sim is NULL");
  s->graph_on = on != 0;
  return HRLB_OK;
}

int hrlb_moments(hrlb_sim* s, double* d_out) {
  if (!s || !d_out) return fail(HRLB_EINVAL, "moments: NULL argument");
  Range r_call("hrlb_moments");
  hipError_t e = (hipError_t)launch_partials(s->sh, s->d, s->d.F[0], s->cells, s->waves, s->stream);
  if (e == hipSuccess) {
    s->part_nvb = (s->sh.V + 64 * s->waves - 1) / (64 * s->waves);
    e = (hipError_t)launch_closure(s->sh, s->d, s->d.F[0], s->part_nvb, d_out, s->stream);
  }
  if (e != hipSuccess) return hip_fail(e, "moments: launch");
  return HRLB_OK;
}

int hrlb_residual(hrlb_sim* s, double* h_out) {
  if (!s || !h_out) return fail(HRLB_EINVAL, "residual: NULL argument");
  Range r_call("hrlb_residual");
  const int B = s->sh.B;
  if (s->resid_nres > 0) {
    hipError_t e = (hipError_t)launch_residual(s->sh, s->d, s->resid_nres, s->stream);
    if (e != hipSuccess) return hip_fail(e, "residual: launch");
  }
  std::vector<int> flags(B);
  HIP_TRY(hipMemcpyAsync(h_out, s->d.resid, B * sizeof(double), hipMemcpyDeviceToHost, s->stream), "residual: copy");
  HIP_TRY(hipMemcpyAsync(flags.data(), s->d.flags, B * sizeof(int), hipMemcpyDeviceToHost, s->stream), "residual: copy");
  HIP_TRY(hipStreamSynchronize(s->stream), "residual: synchronize");
  for (int b = 0; b < B; ++b)
    if (flags[b]) return fail(HRLB_ENUMERIC, "residual: instance " + std::to_string(b) + " met n <= 0, T <= 0 or a non-finite moment");
  return HRLB_OK;
}

int hrlb_get_state(hrlb_sim* s, double* d_out) {
  if (!s || !d_out) return fail(HRLB_EINVAL, "get_state: NULL argument");
  const size_t bytes = (size_t)s->sh.B * s->sh.S * s->sh.V * sizeof(double);
  HIP_TRY(hipMemcpyAsync(d_out, s->d.F[0], bytes, hipMemcpyDeviceToDevice, s->stream), "get_state: copy");
  return HRLB_OK;
}

int hrlb_set_state(hrlb_sim* s, const double* d_in) {
  if (!s || !d_in) return fail(HRLB_EINVAL, "set_state: NULL argument");
  Range r_call("hrlb_set_state");
  const size_t bytes = (size_t)s->sh.B * s->sh.S * s->sh.V * sizeof(double);
  HIP_TRY(hipMemcpyAsync(s->d.F[0], d_in, bytes, hipMemcpyDeviceToDevice, s->stream), "set_state: copy");
  hipError_t e = (hipError_t)launch_partials(s->sh, s->d, s->d.F[0], s->cells, s->waves, s->stream);
  if (e != hipSuccess) return hip_fail(e, "set_state: launch");
  s->part_nvb = (s->sh.V + 64 * s->waves - 1) / (64 * s->waves);
  s->resid_nres = 0;
  return HRLB_OK;
}

int hrlb_free_molecular_state(hrlb_sim* s) {
  if (!s) return fail(HRLB_EINVAL, "free_molecular_state: sim is NULL");
  hipError_t e = (hipError_t)launch_fm_state(s->sh, s->d, s->stream);
  if (e == hipSuccess) e = (hipError_t)launch_clear_flags(s->sh, s->d, s->stream);
  if (e == hipSuccess) e = (hipError_t)launch_partials(s->sh, s->d, s->d.F[0], s->cells, s->waves, s->stream);
  if (e != hipSuccess) return hip_fail(e, "free_molecular_state: launch");
  s->part_nvb = (s->sh.V + 64 * s->waves - 1) / (64 * s->waves);
  s->resid_nres = 0;
  return HRLB_OK;
}

int hrlb_seed_state(hrlb_sim* s, const double* d_table, int preserve_mass, int* h_fallback) {
  if (!s || !d_table) return fail(HRLB_EINVAL, "seed_state: NULL argument");
  if (s->sh.reduced) return fail(HRLB_EINVAL, "seed_state: not available for the reduced (phi, chi) model");
  Range r_call("hrlb_seed_state");
  hipError_t e = (hipError_t)launch_seed(s->sh, s->d, d_table, preserve_mass ? 1 : 0, s->stream);
  if (e != hipSuccess) return hip_fail(e, "seed_state: launch");
  if (h_fallback)
    HIP_TRY(hipMemcpyAsync(h_fallback, s->d.flags, s->sh.B * sizeof(int), hipMemcpyDeviceToHost, s->stream),
            "seed_state: copy");
  e = (hipError_t)launch_clear_flags(s->sh, s->d, s->stream);
  if (e == hipSuccess) e = (hipError_t)launch_partials(s->sh, s->d, s->d.F[0], s->cells, s->waves, s->stream);
  if (e != hipSuccess) return hip_fail(e, "seed_state: launch");
  HIP_TRY(hipStreamSynchronize(s->stream), "seed_state: synchronize");
  s->part_nvb = (s->sh.V + 64 * s->waves - 1) / (64 * s->waves);
  s->resid_nres = 0;
  return HRLB_OK;
}

int hrlb_set_launch(hrlb_sim* s, int cells, int waves) {
  if (!s) return fail(HRLB_EINVAL, "set_launch: sim is NULL");
  if (cells == 0) cells = default_cells(s->sh);
  if (waves == 0) waves = default_waves(s->sh);
  if (cells < 1 || cells > 4096) return fail(HRLB_EINVAL, "set_launch: cells must be in 1..4096");
  if (waves < 1 || waves > MAX_WAVES) return fail(HRLB_EINVAL, "set_launch: waves must be in 1..4");
  // the partials in flight keep their own block count (part_nvb)
  s->cells = cells;
  s->waves = waves;
  return HRLB_OK;
}

int hrlb_get_launch(const hrlb_sim* s, int* cells, int* waves) {
  if (!s || !cells || !waves) return fail(HRLB_EINVAL, "get_launch: NULL argument");
  *cells = s->cells;
  *waves = s->waves;
  return HRLB_OK;
}

int hrlb_set_timing(hrlb_sim* s, int on) {
  if (!s) return fail(HRLB_EINVAL, "set_timing: sim is NULL");
  HIP_TRY(hipStreamSynchronize(s->stream), "set_timing: synchronize");
  for (hipEvent_t e : s->ev) (void)hipEventDestroy(e);
  s->ev.clear();
  s->ev_kind.clear();
  for (int k = 0; k < 4; ++k) {
    s->ms[k] = 0;
    s->launches[k] = 0;
  }
  s->timing = on != 0;
  return HRLB_OK;
}

static int collect_timing(hrlb_sim* s) {
  HIP_TRY(hipStreamSynchronize(s->stream), "get_timing: synchronize");
  for (size_t k = 0; k < s->ev_kind.size(); ++k) {
    float t = 0;
    HIP_TRY(hipEventElapsedTime(&t, s->ev[2 * k], s->ev[2 * k + 1]), "get_timing: elapsed");
    s->ms[s->ev_kind[k]] += t;
    s->launches[s->ev_kind[k]] += 1;
    (void)hipEventDestroy(s->ev[2 * k]);
    (void)hipEventDestroy(s->ev[2 * k + 1]);
  }
  s->ev.clear();
  s->ev_kind.clear();
  return HRLB_OK;
}

int hrlb_get_timing(hrlb_sim* s, double* ms, long long* launches) {
  if (!s || !ms || !launches) return fail(HRLB_EINVAL, "get_timing: NULL argument");
  int rc = collect_timing(s);
  if (rc != HRLB_OK) return rc;
  ms[0] = s->ms[0] + s->ms[1] + s->ms[2];
  ms[1] = s->ms[3];
  launches[0] = s->launches[0] + s->launches[1] + s->launches[2];
  launches[1] = s->launches[3];
  return HRLB_OK;
}

int hrlb_get_stage_timing(hrlb_sim* s, double* ms, long long* launches) {
  if (!s || !ms || !launches) return fail(HRLB_EINVAL, "get_stage_timing: NULL argument");
  int rc = collect_timing(s);
  if (rc != HRLB_OK) return rc;
  for (int k = 0; k < 4; ++k) {
    ms[k] = s->ms[k];
    launches[k] = s->launches[k];
  }
  return HRLB_OK;
}

}  // extern "C"
