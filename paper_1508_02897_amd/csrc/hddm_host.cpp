// Host side of the C ABI declared in include/hddm.h: geometry and stretch
// tables, buffer planning, state machine and the FGMRES driver.  Every
// arithmetic step on vectors runs in the gfx950 kernels of hddm_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/hddm.h"
#include "hddm_internal.h"
#include "hddm_nd_plan.h"

using hddm::AxisCover;
using hddm::BoxDesc;
using cd = std::complex<double>;

namespace {

thread_local std::string g_err;

hddm_status fail(hddm_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

enum State { kSetup = 0, kBound = 1, kFactored = 2 };

}  // namespace

struct hddm_ctx {
  hddm_problem p{};
  int device = 0;
  int ngx = 0, ngy = 0, nbx = 1, nby = 1, nboxes = 1, max_m = 0;
  std::vector<BoxDesc> desc;
  std::vector<cd> ltab;     // per-box stretch tables
  std::vector<cd> gtab;     // global: ax[ngx], ihx[ngx+1], ay[ngy], ihy[ngy+1]
  std::vector<cd> gstretch; // global stretch values (nodes, flux points) for introspection
  std::vector<double> k2;
  std::vector<AxisCover> cx, cy;
  std::vector<int2> ownx, owny;  // per column: (tile, column in its box); per row: (tile, row in the tile)
  // smoothing weights beta along each axis for the covering boxes of cx / cy
  // (x: box0's weight, y: box1's), used by the gathers when smooth is set
  std::vector<double2> wx, wy;
  bool smooth = false;
  std::vector<int32_t> geom;  // 8 per box
  int64_t factor_entries = 0, x_entries = 0;
  // complex64 symmetric-packed factor format (16x16 tiles on and above the
  // diagonal); the factor kernels then work in per-workgroup dense slots
  bool packed = false;
  int factor_slots = 0;
  int64_t fws_stride = 0;  // entries per slot
  size_t elem = 16;           // bytes per factor/workspace entry
  // bytes per factor entry: the nested-dissection fronts are complex128
  size_t felem() const { return nd ? 16 : elem; }
  int sweep_threads = 0;
  // complex64 sweep kernel choice: the wave-structured kernel holds one
  // workgroup per CU and prefetches the next block, which wins while the boxes
  // fit one per CU; with more boxes than CUs the one-row-per-thread kernel
  // keeps several workgroups (boxes) in flight per CU and wins.  Decided at
  // bind from the device's CU count; HDDM_SWEEP_GENERIC=0/1 overrides.
  bool sweep_generic = false;
  int sweep_variant = 0;   // hddm_tune: 0 auto, 1 wave, 2 one row per thread
  int factor_variant = 0;  // hddm_tune: 0 auto (MFMA for complex64), 1 vector, 2 MFMA, memory
                           // working matrix, 3 MFMA, registers, 4 as 3 with symmetric elimination
  int cus = 0;             // compute units of the bound device
  // block form (several right-hand sides per sweep): kernel width in tile
  // blocks (0: unavailable), workspace row width, workspace entries
  int blk_nt = 0, blk_xw = 0, max_tile_rows = 0;
  int blk_variant = 0;  // hddm_tune_block: 0 auto, 1 3M + LDS transpose, 2 4M, 3 3M
  int64_t blk_entries = 0;    // solution planes X (complex64 entries)
  int64_t blk_s_entries = 0;  // source planes S
  size_t blk_bytes() const { return align256((size_t)blk_entries * 8) + (size_t)blk_s_entries * 8; }
  float2* blk_S(void* work_blk) const {
    return reinterpret_cast<float2*>(static_cast<char*>(work_blk) + align256((size_t)blk_entries * 8));
  }
  // bound device memory
  char* factor = nullptr;
  size_t factor_bytes = 0;
  char* work = nullptr;
  size_t work_bytes = 0;
  size_t off_ox = 0, off_oy = 0, off_wx = 0, off_wy = 0;
  size_t off_desc = 0, off_ltab = 0, off_gtab = 0, off_k2 = 0, off_cx = 0, off_cy = 0, off_x = 0,
         off_fws = 0, off_piv = 0, work_need = 0;
  int state = kSetup;
  bool state_shared = false;  // factored through hddm_share_factor (pivots live in the source)
  // event timing (hddm_profile)
  struct Pending {
    hipEvent_t a, b;
    int k;
  };
  bool prof_on = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<Pending> pending;
  int64_t prof_launches[HDDM_K_COUNT] = {};
  double prof_ms[HDDM_K_COUNT] = {};
  hipStream_t prof_stream = nullptr;
  // residual estimates after each Arnoldi step of the last completed solve,
  // one list per right-hand side (hddm_solve_history)
  std::vector<std::vector<double>> hist;
  bool has_hist = false;
  // graphs of fixed launch sequences (hddm_use_graphs), each replayed with
  // the arguments of the current launch
  struct Graph {
    hipGraph_t g = nullptr;
    hipGraphExec_t ex = nullptr;
    std::vector<hipGraphNode_t> kn, en;  // kernel nodes; event nodes (2 per kernel) when timed
    std::vector<const void*> funcs;
    std::vector<unsigned> shape;  // grid, block and LDS bytes of every kernel
    bool timed = false;
  };
  bool use_graphs = true;
  std::vector<Graph> graphs;
  // nested-dissection local solver (factor_format 2): symbolic tables, the
  // class of every box, and where tables, working matrices and update
  // matrices sit in the work buffer; the update vectors follow the box
  // solutions in the block workspace
  bool nd = false;
  hddm::NDPlan ndp;
  std::vector<int32_t> nd_bcls;
  size_t off_nd_fr = 0, off_nd_nodes = 0, off_nd_asm = 0, off_nd_cmap = 0, off_nd_dlist = 0,
         off_nd_doff = 0, off_nd_dcnt = 0, off_nd_bcls = 0, off_nd_w = 0, off_nd_u = 0,
         off_nd_blk = 0;  // block workspace of the single-form entry points
  int nd_slots = 0;
  int64_t nd_v_entries = 0;  // entries of X before the update vectors in the block workspace
  hddm::NDDev nd_dev() const {
    hddm::NDDev d{};
    d.fr = reinterpret_cast<const hddm::NDFront*>(work + off_nd_fr);
    d.nodes = reinterpret_cast<const int32_t*>(work + off_nd_nodes);
    d.asmp = reinterpret_cast<const int32_t*>(work + off_nd_asm);
    d.cmap = reinterpret_cast<const int32_t*>(work + off_nd_cmap);
    d.dlist = reinterpret_cast<const int32_t*>(work + off_nd_dlist);
    d.doff = reinterpret_cast<const int32_t*>(work + off_nd_doff);
    d.dcnt = reinterpret_cast<const int32_t*>(work + off_nd_dcnt);
    d.bcls = reinterpret_cast<const int32_t*>(work + off_nd_bcls);
    d.depths = ndp.depths;
    d.ustride = ndp.ustride;
    d.vstride = ndp.vstride;
    return d;
  }

  bool mixed() const { return p.precision == HDDM_MIXED_C64; }
  int64_t n() const { return (int64_t)ngx * ngy; }
  const BoxDesc* d_desc() const { return reinterpret_cast<const BoxDesc*>(work + off_desc); }
  const double2* d_ltab() const { return reinterpret_cast<const double2*>(work + off_ltab); }
  const double2* d_gtab() const { return reinterpret_cast<const double2*>(work + off_gtab); }
  const double* d_k2() const { return reinterpret_cast<const double*>(work + off_k2); }
  const AxisCover* d_cx() const { return reinterpret_cast<const AxisCover*>(work + off_cx); }
  const AxisCover* d_cy() const { return reinterpret_cast<const AxisCover*>(work + off_cy); }
  const int2* d_ownx() const { return reinterpret_cast<const int2*>(work + off_ox); }
  const int2* d_owny() const { return reinterpret_cast<const int2*>(work + off_oy); }
  // the gathers' weights: null when the smoothing function is off
  const double2* d_wx() const {
    return smooth ? reinterpret_cast<const double2*>(work + off_wx) : nullptr;
  }
  const double2* d_wy() const {
    return smooth ? reinterpret_cast<const double2*>(work + off_wy) : nullptr;
  }
  void* d_x() const { return work + off_x; }
  // per box (smallest, largest) pivot magnitude of the line factor
  float2* d_piv() const { return reinterpret_cast<float2*>(work + off_piv); }
};

namespace {

// Stretch a(t) = 1 + i s0 (d/L)^power on a node grid measured in units of h:
// t = g - P + 1/2 at node g, t = g - P at flux point g - 1/2; the physical
// interval is [lo, hi] (also in units of h) and L = P.
cd stretch_units(double t, double lo, double hi, int P, double s0, int power) {
  const double d = std::max(0.0, std::max(lo - t, t - hi));
  return cd(1.0, s0 * std::pow(d / P, power));
}

// One axis of one box (or of the whole grid): nodes g0..g0+m-1.
void axis_tables(int g0, int m, int P, double h, double lo, double hi, double s0, int power,
                 std::vector<cd>& a, std::vector<cd>& ih, std::vector<cd>* raw_half = nullptr) {
  a.resize(m);
  ih.resize(m + 1);
  const double inv_h2 = 1.0 / (h * h);
  for (int i = 0; i < m; ++i) a[i] = stretch_units(g0 + i - P + 0.5, lo, hi, P, s0, power);
  if (raw_half) raw_half->resize(m + 1);
  for (int i = 0; i <= m; ++i) {
    const cd ah = stretch_units(g0 + i - P, lo, hi, P, s0, power);
    ih[i] = inv_h2 / ah;
    if (raw_half) (*raw_half)[i] = ah;
  }
}

// Tile and box ranges along one axis (global node indices, half-open) and the
// box's physical interval in units of h (Sec. 2, overlapping subdomains; the
// first/last tile takes the adjacent global layer strip).
void axis_ranges(int i, int nb, int n, int n_ol, int P, int& t0, int& t1, int& b0, int& b1,
                 double& lo, double& hi) {
  const int N = nb * n;
  t0 = (i == 0) ? 0 : P + i * n;
  t1 = (i == nb - 1) ? N + 2 * P : P + (i + 1) * n;
  b0 = (i == 0) ? 0 : i * n - n_ol;
  b1 = (i == nb - 1) ? N + 2 * P : (i + 1) * n + n_ol + 2 * P;
  lo = (i == 0) ? 0.0 : double(i * n - n_ol);
  hi = (i == nb - 1) ? double(N) : double((i + 1) * n + n_ol);
}

#define HIPCHK(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(HDDM_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));   \
  } while (0)

hipEvent_t take_event(hddm_ctx* c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Brackets one launch with events when profiling is on.
struct Timed {
  hddm_ctx* c;
  hipEvent_t a = nullptr;
  int k;
  hipStream_t s;
  Timed(hddm_ctx* c_, int k_, hipStream_t s_) : c(c_), k(k_), s(s_) {
    if (c->prof_on) {
      a = take_event(c);
      if (a) (void)hipEventRecord(a, s);
    }
  }
  ~Timed() {
    if (!a) return;
    hipEvent_t b = take_event(c);
    if (!b) return;
    (void)hipEventRecord(b, s);
    c->pending.push_back({a, b, k});
    c->prof_stream = s;
  }
};

void graph_free(hddm_ctx::Graph& g) {
  if (g.ex) (void)hipGraphExecDestroy(g.ex);
  if (g.g) (void)hipGraphDestroy(g.g);
  g = hddm_ctx::Graph{};
}

// Runs ks[0..n) in order on s, launch i timed under class cls[i] when
// profiling is on: one launch after another, or (use_graphs) as one graph
// launch.  A graph is built once per sequence of kernels and launch shapes
// (kernel nodes in a chain, with event-record nodes around each kernel when
// timed) and replayed with this call's arguments and events.
hddm_status run_launches(hddm_ctx* c, hddm::KLaunch* ks, const int* cls, int n, hipStream_t s) {
  if (!c->use_graphs) {
    for (int i = 0; i < n; ++i) {
      Timed tm(c, cls[i], s);
      HIPCHK(ks[i].launch(s));
    }
    return HDDM_OK;
  }
  const bool timed = c->prof_on;
  std::vector<const void*> funcs(n);
  std::vector<unsigned> shape;
  for (int i = 0; i < n; ++i) {
    const hddm::KLaunch& k = ks[i];
    funcs[i] = k.func;
    shape.insert(shape.end(), {k.grid.x, k.grid.y, k.grid.z, k.block.x, k.block.y, k.block.z,
                               k.shmem});
  }
  hddm_ctx::Graph* g = nullptr;
  for (auto& x : c->graphs)
    if (x.timed == timed && x.funcs == funcs && x.shape == shape) g = &x;
  if (!g) {
    if (c->graphs.size() >= 8) {
      graph_free(c->graphs.front());
      c->graphs.erase(c->graphs.begin());
    }
    c->graphs.emplace_back();
    g = &c->graphs.back();
    g->funcs = funcs;
    g->shape = shape;
    g->timed = timed;
    HIPCHK(hipGraphCreate(&g->g, 0));
    hipGraphNode_t prev = nullptr;
    auto add_event = [&]() -> hddm_status {
      hipEvent_t e = take_event(c);  // a placeholder: replaced before every launch
      if (!e) return fail(HDDM_EDEVICE, "hipEventCreate failed");
      hipGraphNode_t node;
      HIPCHK(hipGraphAddEventRecordNode(&node, g->g, prev ? &prev : nullptr, prev ? 1 : 0, e));
      c->ev_pool.push_back(e);
      g->en.push_back(node);
      prev = node;
      return HDDM_OK;
    };
    for (int i = 0; i < n; ++i) {
      hddm_status st;
      if (timed && (st = add_event())) return st;
      hipGraphNode_t node;
      hipKernelNodeParams p = ks[i].params();
      HIPCHK(hipGraphAddKernelNode(&node, g->g, prev ? &prev : nullptr, prev ? 1 : 0, &p));
      g->kn.push_back(node);
      prev = node;
      if (timed && (st = add_event())) return st;
    }
    HIPCHK(hipGraphInstantiate(&g->ex, g->g, nullptr, nullptr, 0));
  }
  for (int i = 0; i < n; ++i) {
    hipKernelNodeParams p = ks[i].params();
    HIPCHK(hipGraphExecKernelNodeSetParams(g->ex, g->kn[i], &p));
  }
  if (timed) {
    for (int i = 0; i < n; ++i) {
      hipEvent_t a = take_event(c), b = take_event(c);
      if (!a || !b) return fail(HDDM_EDEVICE, "hipEventCreate failed");
      HIPCHK(hipGraphExecEventRecordNodeSetEvent(g->ex, g->en[2 * i], a));
      HIPCHK(hipGraphExecEventRecordNodeSetEvent(g->ex, g->en[2 * i + 1], b));
      c->pending.push_back({a, b, cls[i]});
    }
    c->prof_stream = s;
  }
  HIPCHK(hipGraphLaunch(g->ex, s));
  return HDDM_OK;
}

void prof_resolve(hddm_ctx* c) {
  for (auto& p : c->pending) {
    float ms = 0.f;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      c->prof_ms[p.k] += ms;
      c->prof_launches[p.k] += 1;
    }
    c->ev_pool.push_back(p.a);
    c->ev_pool.push_back(p.b);
  }
  c->pending.clear();
}

int pick_sweep_threads(int max_m, int requested) {
  int t = requested;
  if (t <= 0) {
    // as many column groups as fit in 1024 threads: more loads in flight per
    // box (measured best for 168/176-wide boxes: 77% of HBM peak at 4096^2)
    const int rp = std::max(1, max_m / 2);
    t = rp * std::max(1, 1024 / rp);
  }
  t = ((t + 63) / 64) * 64;
  t = std::max(t, ((max_m + 63) / 64) * 64);
  return std::min(t, 1024);
}

hddm_status check_ctx(const hddm_ctx* c, int need) {
  if (!c) return fail(HDDM_EINVAL, "null context");
  if (c->state < need)
    return fail(HDDM_ESTATE, need == kFactored ? "call hddm_factor first"
                                               : "call hddm_bind first");
  return HDDM_OK;
}

}  // namespace

namespace {
template <typename CO>
hddm_status block_sweep_gather(hddm_ctx* c, const hddm::GatherList<CO>& gl, int nz, float2* Xb,
                               const float2* Sb, hipStream_t s,
                               const hddm::KLaunch* first = nullptr, int first_cls = 0);
}  // namespace

extern "C" {

const char* hddm_last_error(void) { return g_err.c_str(); }

hddm_status hddm_setup(const hddm_problem* prob, const double* velocity, int32_t device,
                       hddm_ctx** out) {
  if (!prob || !velocity || !out) return fail(HDDM_EINVAL, "null argument");
  *out = nullptr;
  const hddm_problem& p = *prob;
  if (p.nx <= 0 || p.ny <= 0 || p.npml < 1 || p.tile <= 0 || p.n_ol < 0)
    return fail(HDDM_EINVAL, "sizes must be positive (npml >= 1, n_ol >= 0)");
  if (p.nx % p.tile || p.ny % p.tile) return fail(HDDM_EINVAL, "nx and ny must be multiples of tile");
  if (p.tile % 2 || p.n_ol % 2) return fail(HDDM_EINVAL, "tile and n_ol must be even");
  if (!(p.h > 0) || !(p.omega > 0) || !(p.k_ref > 0) || !(p.sigma0_over_kref >= 0) ||
      p.pml_power < 0)
    return fail(HDDM_EINVAL, "h, omega, k_ref must be positive; sigma0/k_ref, power >= 0");
  if (p.precision != HDDM_PLAIN_C128 && p.precision != HDDM_MIXED_C64)
    return fail(HDDM_EINVAL, "unknown precision");
  if (p.factor_format < 0 || p.factor_format > 2) return fail(HDDM_EINVAL, "unknown factor format");
  if (p.factor_format == 2 && p.precision != HDDM_MIXED_C64)
    return fail(HDDM_EINVAL, "the nested-dissection factor needs precision HDDM_MIXED_C64");
  const int nbx = p.nx / p.tile, nby = p.ny / p.tile;
  if ((nbx > 1 || nby > 1) && p.tile < 2 * (p.n_ol + p.npml))
    return fail(HDDM_EINVAL, "tile must be >= 2*(n_ol + npml) so a node lies in <= 2 boxes per axis");
  if ((nbx > 1 || nby > 1) && p.tile <= p.n_ol)
    return fail(HDDM_EINVAL, "overlap must be smaller than the tile");
  auto* c = new hddm_ctx();
  c->p = p;
  c->device = device;
  c->ngx = p.nx + 2 * p.npml;
  c->ngy = p.ny + 2 * p.npml;
  c->nbx = nbx;
  c->nby = nby;
  c->nboxes = nbx * nby;
  c->elem = c->mixed() ? 8 : 16;
  const int P = p.npml;
  const int64_t n = c->n();
  c->k2.resize(n);
  for (int64_t i = 0; i < n; ++i) {
    const double v = velocity[i];
    if (!(v > 0) || !std::isfinite(v)) {
      delete c;
      return fail(HDDM_EINVAL, "velocity must be positive and finite");
    }
    c->k2[i] = (p.omega / v) * (p.omega / v);
  }
  // global stretch tables: physical region [0, nx] x [0, ny] in units of h
  {
    std::vector<cd> ax, ihx, ay, ihy, hxr, hyr;
    axis_tables(0, c->ngx, P, p.h, 0.0, p.nx, p.sigma0_over_kref, p.pml_power, ax, ihx, &hxr);
    axis_tables(0, c->ngy, P, p.h, 0.0, p.ny, p.sigma0_over_kref, p.pml_power, ay, ihy, &hyr);
    c->gtab.insert(c->gtab.end(), ax.begin(), ax.end());
    c->gtab.insert(c->gtab.end(), ihx.begin(), ihx.end());
    c->gtab.insert(c->gtab.end(), ay.begin(), ay.end());
    c->gtab.insert(c->gtab.end(), ihy.begin(), ihy.end());
    c->gstretch.insert(c->gstretch.end(), ax.begin(), ax.end());
    c->gstretch.insert(c->gstretch.end(), hxr.begin(), hxr.end());
    c->gstretch.insert(c->gstretch.end(), ay.begin(), ay.end());
    c->gstretch.insert(c->gstretch.end(), hyr.begin(), hyr.end());
  }
  // boxes, lexicographic with y outer
  c->cx.assign(c->ngx, AxisCover{-1, -1, -1, -1});
  c->cy.assign(c->ngy, AxisCover{-1, -1, -1, -1});
  auto add_cover = [](AxisCover& a, int box, int loc) {
    if (a.box0 < 0) {
      a.box0 = box;
      a.loc0 = loc;
    } else {
      a.box1 = box;
      a.loc1 = loc;
    }
  };
  c->ownx.assign(c->ngx, int2{-1, -1});
  c->owny.assign(c->ngy, int2{-1, -1});
  // beta along one axis for a box with tile [t0, t1) inside [b0, b1): 1 on the
  // tile; across each side strip of L nodes, 1 - S(s) at s = (d + 1/2) / L for
  // the node d nodes past the tile edge, S(s) = s^3 (10 - 15 s + 6 s^2), the
  // quintic with vanishing first and second derivatives at s = 0 and 1 (a C^2
  // function equal to 1 on the tile and 0 outside the box, as the Remark
  // after eq. pc asks)
  auto beta = [](int g, int t0, int t1, int b0, int b1) {
    double sv;
    if (g < t0)
      sv = (t0 - g - 0.5) / (double)(t0 - b0);
    else if (g >= t1)
      sv = (g - t1 + 0.5) / (double)(b1 - t1);
    else
      return 1.0;
    return 1.0 - sv * sv * sv * (10.0 - 15.0 * sv + 6.0 * sv * sv);
  };
  c->wx.assign(c->ngx, double2{0.0, 0.0});
  c->wy.assign(c->ngy, double2{0.0, 0.0});
  auto add_weight = [](double2& w, const AxisCover& a, int box, double v) {
    if (a.box0 == box)
      w.x = v;
    else
      w.y = v;
  };
  for (int i = 0; i < nbx; ++i) {
    int t0, t1, b0, b1;
    double lo, hi;
    axis_ranges(i, nbx, p.tile, p.n_ol, P, t0, t1, b0, b1, lo, hi);
    for (int g = b0; g < b1; ++g) {
      add_cover(c->cx[g], i, g - b0);
      add_weight(c->wx[g], c->cx[g], i, beta(g, t0, t1, b0, b1));
    }
    for (int g = t0; g < t1; ++g) c->ownx[g] = int2{i, g - b0};
  }
  for (int i = 0; i < nby; ++i) {
    int t0, t1, b0, b1;
    double lo, hi;
    axis_ranges(i, nby, p.tile, p.n_ol, P, t0, t1, b0, b1, lo, hi);
    for (int g = b0; g < b1; ++g) {
      add_cover(c->cy[g], i, g - b0);
      add_weight(c->wy[g], c->cy[g], i, beta(g, t0, t1, b0, b1));
    }
    for (int g = t0; g < t1; ++g) c->owny[g] = int2{i, g - t0};
  }
  // widest box decides whether the packed format applies (16x16 tiles, <= 256)
  {
    int mm = 0;
    for (int i = 0; i < nbx; ++i) {
      int t0, t1, b0, b1;
      double lo, hi;
      axis_ranges(i, nbx, p.tile, p.n_ol, P, t0, t1, b0, b1, lo, hi);
      mm = std::max(mm, b1 - b0);
    }
    for (int i = 0; i < nby; ++i) {
      int t0, t1, b0, b1;
      double lo, hi;
      axis_ranges(i, nby, p.tile, p.n_ol, P, t0, t1, b0, b1, lo, hi);
      mm = std::max(mm, b1 - b0);
    }
    c->packed = c->mixed() && p.factor_format == 0 && mm <= 256;
    c->nd = p.factor_format == 2;
  }
  if (c->nd) {
    std::vector<std::pair<int, int>> shapes;
    for (int iy = 0; iy < nby; ++iy)
      for (int ix = 0; ix < nbx; ++ix) {
        int t0, t1, x0, x1, y0, y1;
        double lo, hi;
        axis_ranges(ix, nbx, p.tile, p.n_ol, P, t0, t1, x0, x1, lo, hi);
        axis_ranges(iy, nby, p.tile, p.n_ol, P, t0, t1, y0, y1, lo, hi);
        const std::pair<int, int> sh{x1 - x0, y1 - y0};
        auto it = std::find(shapes.begin(), shapes.end(), sh);
        c->nd_bcls.push_back((int32_t)(it - shapes.begin()));
        if (it == shapes.end()) shapes.push_back(sh);
      }
    std::string err;
    if (!hddm::nd_build(shapes, hddm::ND_LEAF, c->ndp, err)) {
      delete c;
      return fail(HDDM_EINVAL, "nested dissection: " + err);
    }
  }
  int64_t goff = 0, xoff = 0;
  for (int iy = 0; iy < nby; ++iy) {
    int ty0, ty1, by0, by1;
    double ylo, yhi;
    axis_ranges(iy, nby, p.tile, p.n_ol, P, ty0, ty1, by0, by1, ylo, yhi);
    for (int ix = 0; ix < nbx; ++ix) {
      int tx0, tx1, bx0, bx1;
      double xlo, xhi;
      axis_ranges(ix, nbx, p.tile, p.n_ol, P, tx0, tx1, bx0, bx1, xlo, xhi);
      BoxDesc d{};
      d.mx = bx1 - bx0;
      d.my = by1 - by0;
      d.bx0 = bx0;
      d.by0 = by0;
      d.tx0 = tx0 - bx0;
      d.tx1 = tx1 - bx0;
      d.ty0 = ty0 - by0;
      d.ty1 = ty1 - by0;
      d.g_off = goff;
      d.x_off = xoff;
      d.tab_off = (int32_t)c->ltab.size();
      std::vector<cd> ax, ihx, ay, ihy;
      axis_tables(bx0, d.mx, P, p.h, xlo, xhi, p.sigma0_over_kref, p.pml_power, ax, ihx);
      axis_tables(by0, d.my, P, p.h, ylo, yhi, p.sigma0_over_kref, p.pml_power, ay, ihy);
      c->ltab.insert(c->ltab.end(), ax.begin(), ax.end());
      c->ltab.insert(c->ltab.end(), ihx.begin(), ihx.end());
      c->ltab.insert(c->ltab.end(), ay.begin(), ay.end());
      c->ltab.insert(c->ltab.end(), ihy.begin(), ihy.end());
      if (c->nd) {
        goff += c->ndp.class_entries[c->nd_bcls[c->desc.size()]];
      } else if (c->packed) {
        const int64_t nt = (d.mx + 15) / 16;
        goff += nt * (nt + 1) / 2 * 256 * d.my;
      } else {
        goff += (int64_t)d.mx * d.mx * d.my;
      }
      // keep every box's factor and workspace start 256-byte aligned
      goff = (goff + 31) & ~int64_t(31);
      xoff += (int64_t)d.mx * d.my;
      xoff = (xoff + 31) & ~int64_t(31);
      c->max_m = std::max(c->max_m, std::max(d.mx, d.my));
      c->desc.push_back(d);
      const int32_t g8[8] = {bx0, bx1, by0, by1, tx0, tx1, ty0, ty1};
      c->geom.insert(c->geom.end(), g8, g8 + 8);
    }
  }
  c->factor_entries = goff;
  c->x_entries = xoff;
  {
    int max_mx = 0;
    for (const BoxDesc& d : c->desc) {
      max_mx = std::max(max_mx, d.mx);
      c->max_tile_rows = std::max(c->max_tile_rows, d.ty1 - d.ty0);
    }
    c->blk_nt = c->packed ? hddm::block_nt((max_mx + 15) / 16) : 0;
    if (c->nd) {
      // sources as planes (written by the Krylov kernels), box solutions
      // node-major, then the update vectors of the two depth parities
      c->blk_xw = 16 * ((max_mx + 15) / 16);
      int64_t xb = 0;
      for (BoxDesc& d : c->desc) {
        d.xb_off = xb;
        xb += (int64_t)d.mx * d.my * HDDM_BLOCK_MAX;
        xb = (xb + 31) & ~int64_t(31);
      }
      c->nd_v_entries = xb;
      c->blk_entries = xb + 2 * (int64_t)c->nboxes * c->ndp.vstride;
      c->blk_s_entries = (int64_t)c->nboxes * HDDM_BLOCK_MAX * c->max_tile_rows * c->blk_xw;
    } else if (c->blk_nt > 0) {
      c->blk_xw = 16 * c->blk_nt;
      int64_t xb = 0;
      for (BoxDesc& d : c->desc) {
        d.xb_off = xb;
        xb += (int64_t)d.my * c->blk_xw * HDDM_BLOCK_MAX;
        xb = (xb + 31) & ~int64_t(31);
      }
      c->blk_entries = xb;
      c->blk_s_entries = (int64_t)c->nboxes * HDDM_BLOCK_MAX * c->max_tile_rows * c->blk_xw;
    }
  }
  const int ld_limit = c->mixed() ? 416 : 208;  // factor LDS panels: (256 + 48 ld) entries
  if (c->max_m > ld_limit) {
    const int mm = c->max_m;
    delete c;
    return fail(HDDM_EINVAL, "box side " + std::to_string(mm) + " exceeds " +
                                 std::to_string(ld_limit) + " for this precision");
  }
  c->sweep_threads = pick_sweep_threads(c->max_m, 0);
  // work buffer plan
  size_t off = 0;
  c->off_desc = off;
  off = align256(off + c->desc.size() * sizeof(BoxDesc));
  c->off_ltab = off;
  off = align256(off + c->ltab.size() * 16);
  c->off_gtab = off;
  off = align256(off + c->gtab.size() * 16);
  c->off_k2 = off;
  off = align256(off + c->k2.size() * 8);
  c->off_cx = off;
  off = align256(off + c->cx.size() * sizeof(AxisCover));
  c->off_cy = off;
  off = align256(off + c->cy.size() * sizeof(AxisCover));
  c->off_ox = off;
  off = align256(off + c->ownx.size() * sizeof(int2));
  c->off_oy = off;
  off = align256(off + c->owny.size() * sizeof(int2));
  c->off_wx = off;
  off = align256(off + c->wx.size() * sizeof(double2));
  c->off_wy = off;
  off = align256(off + c->wy.size() * sizeof(double2));
  c->off_piv = off;
  off = align256(off + (size_t)c->nboxes * sizeof(float2));
  c->off_x = off;
  // the single form's box solutions (the nested-dissection factor keeps its
  // own block workspace instead)
  off = align256(off + (c->nd ? 0 : (size_t)c->x_entries * c->elem));
  c->off_fws = off;
  if (c->nd) {
    const hddm::NDPlan& pl = c->ndp;
    c->off_nd_fr = off;
    off = align256(off + pl.fronts.size() * sizeof(hddm::NDFront));
    c->off_nd_nodes = off;
    off = align256(off + pl.nodes.size() * 4);
    c->off_nd_asm = off;
    off = align256(off + pl.asmp.size() * 4);
    c->off_nd_cmap = off;
    off = align256(off + pl.cmap.size() * 4);
    c->off_nd_dlist = off;
    off = align256(off + pl.dlist.size() * 4);
    c->off_nd_doff = off;
    off = align256(off + pl.doff.size() * 4);
    c->off_nd_dcnt = off;
    off = align256(off + pl.dcnt.size() * 4);
    c->off_nd_bcls = off;
    off = align256(off + c->nd_bcls.size() * 4);
    // factor working matrices: one per workgroup of the factor launches (which
    // grid-stride over the (box, front) items of a depth).  About 512 of its
    // 256-thread workgroups are resident on a 256-CU device at once, so 1024
    // slots keep it full; fewer when no depth has that many items.
    int64_t items = 1;
    for (int d = 0; d < pl.depths; ++d) items = std::max(items, (int64_t)c->nboxes * pl.maxcnt[d]);
    c->nd_slots = (int)std::min<int64_t>(1024, items);
    c->off_nd_w = off;
    off = align256(off + (size_t)c->nd_slots * pl.wstride * 16);
    c->off_nd_u = off;
    off = align256(off + 2 * (size_t)c->nboxes * pl.ustride * 16);
    c->off_nd_blk = off;
    off = align256(off + c->blk_bytes());
  }
  if (c->packed) {
    c->factor_slots = std::min(c->nboxes, 512);
    c->fws_stride = ((int64_t)c->max_m * c->max_m + 31) & ~int64_t(31);
    off = align256(off + (size_t)c->factor_slots * c->fws_stride * 8);
  }
  c->work_need = off;
  *out = c;
  return HDDM_OK;
}

// Per right-hand side: V[(m+1)][n] c128 | Z[m][n] (c64 mixed / c128 plain) |
// partial[2(m+1)][nblk] c128 | npart[nblk] f64 | summary | Gram[(m+1)^2] c128.
// The summary (summary_len entries) holds what the host reads or writes per
// Arnoldi step: h1[2(m+1)] | h2[m+1] | y[m] | (|w|, |r|) | nu[m+1] (f64, the
// norms of the unscaled basis vectors of the block solve).
static int summary_len(int m) { return 4 * m + 4 + (m + 2) / 2; }
static size_t krylov_need(const hddm_ctx* c, int m, size_t* offs) {
  const int64_t n = c->n();
  const int nblk = hddm::krylov_partials(c->ngx, c->ngy);
  const size_t zel = c->mixed() ? 8 : 16;
  size_t off = 0;
  offs[0] = off;
  off = align256(off + (size_t)(m + 1) * n * 16);
  offs[1] = off;
  off = align256(off + (size_t)m * n * zel);
  offs[2] = off;
  off = align256(off + 2 * (size_t)(m + 1) * nblk * 16);
  offs[3] = off;
  off = align256(off + (size_t)nblk * 8);
  offs[4] = off;
  off = align256(off + (size_t)summary_len(m) * 16);
  offs[5] = off;
  off = align256(off + (size_t)(m + 1) * (m + 1) * 16);
  return off;
}

hddm_status hddm_query_bytes(const hddm_ctx* c, int32_t restart, size_t* factor_bytes,
                             size_t* work_bytes, size_t* krylov_bytes) {
  if (!c) return fail(HDDM_EINVAL, "null context");
  if (restart < 1) return fail(HDDM_EINVAL, "restart must be >= 1");
  size_t offs[6];
  if (factor_bytes) *factor_bytes = (size_t)c->factor_entries * c->felem();
  if (work_bytes) *work_bytes = c->work_need;
  if (krylov_bytes) *krylov_bytes = krylov_need(c, restart, offs);
  return HDDM_OK;
}

hddm_status hddm_bind(hddm_ctx* c, void* factor_buf, size_t factor_bytes, void* work_buf,
                      size_t work_bytes, void* stream) {
  if (!c) return fail(HDDM_EINVAL, "null context");
  if (!factor_buf || !work_buf) return fail(HDDM_EINVAL, "null buffer");
  if (((uintptr_t)factor_buf | (uintptr_t)work_buf) & 255)
    return fail(HDDM_EINVAL, "buffers must be 256-byte aligned");
  if (factor_bytes < (size_t)c->factor_entries * c->felem())
    return fail(HDDM_ENOMEM, "factor buffer too small");
  if (work_bytes < c->work_need) return fail(HDDM_ENOMEM, "work buffer too small");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  HIPCHK(hipSetDevice(c->device));
  HIPCHK(hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, c->device));
  c->factor = static_cast<char*>(factor_buf);
  c->factor_bytes = factor_bytes;
  c->work = static_cast<char*>(work_buf);
  c->work_bytes = work_bytes;
  HIPCHK(hipMemcpyAsync(c->work + c->off_desc, c->desc.data(), c->desc.size() * sizeof(BoxDesc),
                        hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(c->work + c->off_ltab, c->ltab.data(), c->ltab.size() * 16,
                        hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(c->work + c->off_gtab, c->gtab.data(), c->gtab.size() * 16,
                        hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(c->work + c->off_k2, c->k2.data(), c->k2.size() * 8, hipMemcpyHostToDevice,
                        s));
  HIPCHK(hipMemcpyAsync(c->work + c->off_cx, c->cx.data(), c->cx.size() * sizeof(AxisCover),
                        hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(c->work + c->off_cy, c->cy.data(), c->cy.size() * sizeof(AxisCover),
                        hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(c->work + c->off_ox, c->ownx.data(), c->ownx.size() * sizeof(int2),
                        hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(c->work + c->off_oy, c->owny.data(), c->owny.size() * sizeof(int2),
                        hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(c->work + c->off_wx, c->wx.data(), c->wx.size() * sizeof(double2),
                        hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(c->work + c->off_wy, c->wy.data(), c->wy.size() * sizeof(double2),
                        hipMemcpyHostToDevice, s));
  if (c->nd) {
    const hddm::NDPlan& pl = c->ndp;
    HIPCHK(hipMemcpyAsync(c->work + c->off_nd_fr, pl.fronts.data(),
                          pl.fronts.size() * sizeof(hddm::NDFront), hipMemcpyHostToDevice, s));
    const std::pair<size_t, const std::vector<int32_t>*> tabs[] = {
        {c->off_nd_nodes, &pl.nodes}, {c->off_nd_asm, &pl.asmp},   {c->off_nd_cmap, &pl.cmap},
        {c->off_nd_dlist, &pl.dlist}, {c->off_nd_doff, &pl.doff},  {c->off_nd_dcnt, &pl.dcnt},
        {c->off_nd_bcls, &c->nd_bcls}};
    for (const auto& t : tabs)
      if (!t.second->empty())
        HIPCHK(hipMemcpyAsync(c->work + t.first, t.second->data(), t.second->size() * 4,
                              hipMemcpyHostToDevice, s));
  }
  HIPCHK(hipStreamSynchronize(s));
  c->state = kBound;
  return HDDM_OK;
}

hddm_status hddm_factor(hddm_ctx* c, void* stream) {
  hddm_status st = check_ctx(c, kBound);
  if (st) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  HIPCHK(hipSetDevice(c->device));
  Timed tm(c, HDDM_K_FACTOR, s);
  if (c->nd) {
    // depth by depth from the leaves: a front needs its children's update matrices
    const hddm::NDPlan& pl = c->ndp;
    for (int d = pl.depths - 1; d >= 0; --d)
      HIPCHK(hddm::launch_nd_factor(c->nd_dev(), d, pl.maxcnt[d], c->nboxes, pl.maxn[d],
                                    c->d_desc(), c->d_ltab(), c->d_k2(), c->ngx,
                                    reinterpret_cast<double2*>(c->factor),
                                    reinterpret_cast<double2*>(c->work + c->off_nd_w), pl.wstride,
                                    c->nd_slots, reinterpret_cast<double2*>(c->work + c->off_nd_u),
                                    s));
  } else if (c->mixed()) {
    float2* G = reinterpret_cast<float2*>(c->factor);
    float2* ws = reinterpret_cast<float2*>(c->work + c->off_fws);
    const bool mfma = c->factor_variant != 1 && c->max_m <= 256;
    // the register-resident MFMA kernel with symmetric elimination where the
    // boxes fit it (factor_variant 0), else the MFMA kernel with a memory
    // working matrix
    float2* pv = c->d_piv();
    if ((c->factor_variant == 0 || c->factor_variant == 4) && c->max_m <= 192)
      HIPCHK(hddm::launch_factor_c64_sym_regs(c->d_desc(), c->d_ltab(), c->d_k2(), c->ngx, G,
                                              c->nboxes, c->max_m, c->packed, pv, s));
    else if (c->factor_variant == 3 && c->max_m <= 192)
      HIPCHK(hddm::launch_factor_c64_mfma_regs(c->d_desc(), c->d_ltab(), c->d_k2(), c->ngx, G,
                                               c->nboxes, c->max_m, c->packed, pv, s));
    else if (c->packed && mfma)
      HIPCHK(hddm::launch_factor_c64_mfma(c->d_desc(), c->d_ltab(), c->d_k2(), c->ngx, G,
                                          c->nboxes, c->max_m, ws, c->fws_stride,
                                          c->factor_slots, pv, s));
    else if (c->packed)
      HIPCHK(hddm::launch_factor_c64_packed(c->d_desc(), c->d_ltab(), c->d_k2(), c->ngx, G,
                                            c->nboxes, c->max_m, ws, c->fws_stride,
                                            c->factor_slots, pv, s));
    else if (mfma)
      HIPCHK(hddm::launch_factor_c64_mfma(c->d_desc(), c->d_ltab(), c->d_k2(), c->ngx, G,
                                          c->nboxes, c->max_m, nullptr, 0, 0, pv, s));
    else
      HIPCHK(hddm::launch_factor_c64(c->d_desc(), c->d_ltab(), c->d_k2(), c->ngx, G, c->nboxes,
                                     c->max_m, pv, s));
  } else {
    HIPCHK(hddm::launch_factor_c128(c->d_desc(), c->d_ltab(), c->d_k2(), c->ngx,
                                    reinterpret_cast<double2*>(c->factor), c->nboxes, c->max_m,
                                    c->d_piv(), s));
  }
  c->state = kFactored;
  c->state_shared = false;
  return HDDM_OK;
}

hddm_status hddm_factor_pivots(hddm_ctx* c, float* out, void* stream) {
  hddm_status st = check_ctx(c, kFactored);
  if (st) return st;
  if (!out) return fail(HDDM_EINVAL, "null output");
  if (c->nd) return fail(HDDM_EINVAL, "pivots are reported for the line factor only");
  if (c->state_shared) return fail(HDDM_ESTATE, "factorisation shared from another context");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  HIPCHK(hipSetDevice(c->device));
  HIPCHK(hipMemcpyAsync(out, c->d_piv(), (size_t)c->nboxes * sizeof(float2), hipMemcpyDeviceToHost,
                        s));
  HIPCHK(hipStreamSynchronize(s));
  return HDDM_OK;
}

hddm_status hddm_share_factor(hddm_ctx* dst, const hddm_ctx* src) {
  if (!dst || !src) return fail(HDDM_EINVAL, "null context");
  if (src->state < kFactored) return fail(HDDM_ESTATE, "source context is not factored");
  if (dst->state < kBound) return fail(HDDM_ESTATE, "call hddm_bind on the destination first");
  const hddm_problem &a = dst->p, &b = src->p;
  const bool same = a.nx == b.nx && a.ny == b.ny && a.npml == b.npml && a.tile == b.tile &&
                    a.n_ol == b.n_ol && a.pml_power == b.pml_power && a.precision == b.precision &&
                    a.factor_format == b.factor_format &&
                    a.h == b.h && a.omega == b.omega && a.k_ref == b.k_ref &&
                    a.sigma0_over_kref == b.sigma0_over_kref && dst->k2 == src->k2;
  if (!same) return fail(HDDM_EINVAL, "contexts describe different problems");
  if (dst->factor != src->factor) return fail(HDDM_EINVAL, "destination is bound to another factor buffer");
  dst->factor_variant = src->factor_variant;
  dst->state = kFactored;
  dst->state_shared = true;
  return HDDM_OK;
}

// Sweeps of every box on r (c128), leaving the box solutions in the workspace.
// The single form's sweep over all boxes (restricting r itself).
// X: the box-solution workspace (x_entries entries of elem bytes).
static hddm_status describe_sweeps(hddm_ctx* c, const double2* r, void* X, hddm::KLaunch& k) {
  c->sweep_generic = c->sweep_variant == 2 || (c->sweep_variant == 0 && c->nboxes > c->cus);
  if (c->packed) {
    HIPCHK(hddm::describe_sweep_c64_packed(k, c->d_desc(), c->d_ltab(),
                                           reinterpret_cast<const float2*>(c->factor),
                                           static_cast<float2*>(X), r, c->ngx,
                                           c->nboxes, c->max_m, c->sweep_variant == 1));
  } else if (c->mixed()) {
    HIPCHK(hddm::describe_sweep_c64(k, c->d_desc(), c->d_ltab(),
                                    reinterpret_cast<const float2*>(c->factor),
                                    static_cast<float2*>(X), r, c->ngx, c->nboxes,
                                    c->sweep_threads, c->max_m, c->sweep_generic));
  } else {
    HIPCHK(hddm::describe_sweep_c128(k, c->d_desc(), c->d_ltab(),
                                     reinterpret_cast<const double2*>(c->factor),
                                     static_cast<double2*>(X), r, c->ngx, c->nboxes,
                                     c->sweep_threads, c->max_m));
  }
  return HDDM_OK;
}

// The line-factor single form's sweep + gather for z = P^-1 r (z complex64 if
// z_c64, else complex128) with the box solutions in X.
static hddm_status describe_single(hddm_ctx* c, const double2* r, void* z, bool z_c64, void* X,
                                   hddm::KLaunch* ks) {
  hddm_status st = describe_sweeps(c, r, X, ks[0]);
  if (st) return st;
  if (!c->mixed())
    HIPCHK(hddm::describe_gather_c128_to_c128(ks[1], c->d_desc(), c->d_cx(), c->d_cy(),
                                              static_cast<const double2*>(X),
                                              static_cast<double2*>(z), c->ngx, c->ngy, c->nbx,
                                              c->d_wx(), c->d_wy()));
  else if (z_c64)
    HIPCHK(hddm::describe_gather_c64_to_c64(ks[1], c->d_desc(), c->d_cx(), c->d_cy(),
                                            static_cast<const float2*>(X),
                                            static_cast<float2*>(z), c->ngx, c->ngy, c->nbx,
                                            c->d_wx(), c->d_wy()));
  else
    HIPCHK(hddm::describe_gather_c64_to_c128(ks[1], c->d_desc(), c->d_cx(), c->d_cy(),
                                             static_cast<const float2*>(X),
                                             static_cast<double2*>(z), c->ngx, c->ngy, c->nbx,
                                             c->d_wx(), c->d_wy()));
  return HDDM_OK;
}

// One single-form application z = P^-1 r: sweep + gather (to complex64 if
// z_c64, else complex128), one graph launch.
static hddm_status single_apply(hddm_ctx* c, const double2* r, void* z, bool z_c64,
                                hipStream_t s) {
  if (c->nd) {
    // through the block kernels with one column, in the work buffer's own
    // block workspace: restriction (the other 15 source planes zero), the
    // nested-dissection sweeps, gather of plane 0
    float2* Xb = reinterpret_cast<float2*>(c->work + c->off_nd_blk);
    float2* Sb = c->blk_S(Xb);
    hddm::VecList rl{};
    for (int k = 0; k < hddm::BLOCK_RHS; ++k) rl.p[k] = r;
    hddm::KLaunch rk;
    HIPCHK(hddm::describe_restrict_block(rk, c->d_desc(), c->nboxes, c->max_tile_rows, rl, 1, Sb,
                                         c->ngx, c->blk_xw));
    if (z_c64) {
      hddm::GatherList<float2> gl{};
      for (int k = 0; k < hddm::BLOCK_RHS; ++k) gl.z[k] = static_cast<float2*>(z);
      return block_sweep_gather<float2>(c, gl, 1, Xb, Sb, s, &rk, HDDM_K_RESTRICT);
    }
    hddm::GatherList<double2> gl{};
    for (int k = 0; k < hddm::BLOCK_RHS; ++k) gl.z[k] = static_cast<double2*>(z);
    return block_sweep_gather<double2>(c, gl, 1, Xb, Sb, s, &rk, HDDM_K_RESTRICT);
  }
  hddm::KLaunch ks[2];
  const int cls[2] = {HDDM_K_SWEEP, HDDM_K_GATHER};
  hddm_status st = describe_single(c, r, z, z_c64, c->d_x(), ks);
  if (st) return st;
  return run_launches(c, ks, cls, 2, s);
}

hddm_status hddm_apply_precond(hddm_ctx* c, const void* r, void* z, void* stream) {
  hddm_status st = check_ctx(c, kFactored);
  if (st) return st;
  if (!r || !z) return fail(HDDM_EINVAL, "null vector");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  HIPCHK(hipSetDevice(c->device));
  return single_apply(c, static_cast<const double2*>(r), z, false, s);
}

hddm_status hddm_matvec(hddm_ctx* c, const void* x, void* y, void* stream) {
  hddm_status st = check_ctx(c, kBound);
  if (st) return st;
  if (!x || !y) return fail(HDDM_EINVAL, "null vector");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  HIPCHK(hipSetDevice(c->device));
  Timed tm(c, HDDM_K_MATVEC, s);
  HIPCHK(hddm::launch_matvec_c128(c->d_gtab(), c->d_k2(), static_cast<const double2*>(x), nullptr,
                                  static_cast<double2*>(y), c->ngx, c->ngy, s));
  return HDDM_OK;
}

}  // extern "C"

namespace {

// Restarted FGMRES of one right-hand side (Sec. 3: GMRES preconditioned from
// the right by the one-step method; flexible form x = x0 + Z y with
// Z = P^-1 V kept, so the complex64 preconditioner may vary slightly between
// applications).  Device pointers live in the RHS's Krylov region; `sum` is
// its summary (h1 | h2 | y | norms), mirrored on the host in `hs`.
struct Fg {
  double2* V = nullptr;
  char* Z = nullptr;
  double2* part = nullptr;
  double* npart = nullptr;
  double2* gram = nullptr;
  double2* sum = nullptr;
  cd* hs = nullptr;
  const double2* b = nullptr;
  double2* x = nullptr;
  std::vector<cd> H, gamma, sn, hcol;
  std::vector<double> cs;
  int j = 0, iters = 0;
  double bnorm = 0.0;
  bool running = false;
  int slot = 0;  // plane of the block workspace (block solve)
  hddm_solve_info inf{};
  std::vector<double> hist;  // |gamma_{j+1}| / |b| after every Arnoldi step
};

// The FGMRES iterations of the right-hand sides of one context that share a
// summary array on the device (read back with one copy per round) and, in the
// block form, a block workspace.  The steps below advance every running
// right-hand side of one or several groups by one round: each round applies
// the preconditioner to every running RHS's current Arnoldi vector
// (Z_j = P^-1 V_j), runs their Arnoldi steps, reads the summaries back and
// updates the Givens rotations on the host; a right-hand side whose cycle
// ended gets x += Z y and its true residual in the same round.  Right-hand
// sides converge, restart and stop independently.
// lazy: the basis vectors stay unscaled (their norms kept on the device and
// folded into every product by the kernels), so no scaling pass runs; sm:
// where the Arnoldi and residual kernels also write the next block sources.
struct FgGroup {
  hddm_ctx* c = nullptr;
  std::vector<Fg>* st = nullptr;
  hddm_solve_opts o{};
  double2* sums = nullptr;
  std::vector<cd>* hsum = nullptr;
  bool lazy = false;
  hddm::SrcMap sm{};
  float2* Xb = nullptr;  // block workspace (block form)
  float2* Sb = nullptr;
  std::vector<Fg*> run, ended, going;  // this round's lists
};

hddm::KSet kset_of(const std::vector<Fg*>& v, bool lazy) {
  hddm::KSet ks{};
  ks.n = (int)v.size();
  ks.lazy = lazy ? 1 : 0;
  for (int y = 0; y < ks.n; ++y) {
    Fg& f = *v[y];
    ks.j[y] = f.j;
    ks.slot[y] = f.slot;
    ks.V[y] = f.V;
    ks.part[y] = f.part;
    ks.npart[y] = f.npart;
    ks.sum[y] = f.sum;
    ks.gram[y] = f.gram;
    ks.Z[y] = f.Z;
    ks.x[y] = f.x;
    ks.b[y] = f.b;
  }
  return ks;
}

// Copies the summaries of every group in `gs` to the host, then waits once.
hddm_status fg_read(const std::vector<FgGroup*>& gs, hipStream_t s) {
  for (FgGroup* g : gs)
    HIPCHK(hipMemcpyAsync(g->hsum->data(), g->sums, g->hsum->size() * sizeof(cd),
                          hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (FgGroup* g : gs)
    if (g->c->prof_on) prof_resolve(g->c);
  return HDDM_OK;
}

double fg_hn(const Fg& f, int m) { return f.hs[4 * m + 3].real(); }
double fg_rn(const Fg& f, int m) { return f.hs[4 * m + 3].imag(); }

// x = 0, V_0 = b - M 0 = b and |b| (and the first sources).
hddm_status fg_launch_init(FgGroup& g, hipStream_t s) {
  const int m = g.o.restart;
  std::vector<Fg*> all;
  for (Fg& f : *g.st) {
    f.H.assign((size_t)(m + 1) * m, cd(0));
    f.gamma.assign(m + 1, cd(0));
    f.sn.assign(m, cd(0));
    f.hcol.assign(m + 1, cd(0));
    f.cs.assign(m, 0.0);
    f.inf = hddm_solve_info{};
    f.inf.status = HDDM_OK;
    f.inf.relres_est = f.inf.relres_true = 1.0;
    f.iters = 0;
    f.running = false;
    f.hist.clear();
    HIPCHK(hddm::launch_zero(f.x, (size_t)g.c->n() * 16, s));
    all.push_back(&f);
  }
  HIPCHK(hddm::launch_residual(kset_of(all, g.lazy), m, g.c->d_gtab(), g.c->d_k2(), g.c->ngx,
                               g.c->ngy, g.sm, s));
  return HDDM_OK;
}

hddm_status fg_after_init(FgGroup& g, hipStream_t s) {
  const int m = g.o.restart;
  std::vector<Fg*> start;
  for (Fg& f : *g.st) {
    f.bnorm = fg_rn(f, m);
    if (!std::isfinite(f.bnorm)) {
      f.inf.status = HDDM_EBREAKDOWN;
      continue;
    }
    if (f.bnorm == 0) {
      f.inf.relres_est = f.inf.relres_true = 0.0;
      continue;
    }
    f.gamma[0] = f.bnorm;
    f.j = 0;
    f.inf.restarts = 1;
    f.running = true;
    start.push_back(&f);
  }
  if (!g.lazy && !start.empty())
    HIPCHK(hddm::launch_arnoldi_scale(kset_of(start, false), m, g.c->n(), 1, s));  // V_0 = b / |b|
  return HDDM_OK;
}

// The group's running right-hand sides into g.run; false when none.
bool fg_collect(FgGroup& g) {
  g.run.clear();
  for (Fg& f : *g.st)
    if (f.running) g.run.push_back(&f);
  return !g.run.empty();
}

// One Arnoldi step of every running right-hand side (w = M z_j formed inside).
hddm_status fg_launch_arnoldi(FgGroup& g, hipStream_t s) {
  hddm_ctx* c = g.c;
  hddm::KSet ks = kset_of(g.run, g.lazy);
  const hddm::Op op{c->d_gtab(), c->d_k2(), c->ngx, c->ngy, c->mixed()};
  Timed tm(c, HDDM_K_KRYLOV, s);
  if (g.o.ortho == 1)
    HIPCHK(hddm::launch_arnoldi_gram(ks, g.o.restart, op, g.sm, s));
  else
    HIPCHK(hddm::launch_arnoldi_cgs2(ks, g.o.restart, op, g.sm, s));
  return HDDM_OK;
}

// Givens update of every running right-hand side from the summaries just
// read; sorts them into g.ended (cycle over) and g.going (next Arnoldi index).
hddm_status fg_after_arnoldi(FgGroup& g, hipStream_t s) {
  const int m = g.o.restart;
  const bool gram_cgs = g.o.ortho == 1;
  g.ended.clear();
  g.going.clear();
  for (Fg* fp : g.run) {
    Fg& f = *fp;
    const int j = f.j;
    ++f.iters;
    const double hn = fg_hn(f, m);
    bool finite = std::isfinite(hn);
    for (int i = 0; i <= j; ++i) {
      f.hcol[i] = gram_cgs ? f.hs[2 * (m + 1) + i] : f.hs[i] + f.hs[2 * (m + 1) + i];
      finite = finite && std::isfinite(f.hcol[i].real()) && std::isfinite(f.hcol[i].imag());
    }
    if (!finite) {
      f.inf.status = HDDM_EBREAKDOWN;
      f.running = false;
      continue;
    }
    f.hcol[j + 1] = hn;
    for (int i = 0; i < j; ++i) {  // previous rotations
      const cd t = f.cs[i] * f.hcol[i] + f.sn[i] * f.hcol[i + 1];
      f.hcol[i + 1] = -std::conj(f.sn[i]) * f.hcol[i] + f.cs[i] * f.hcol[i + 1];
      f.hcol[i] = t;
    }
    // new rotation zeroing hcol[j+1] below hcol[j]
    const cd a = f.hcol[j], bb = f.hcol[j + 1];
    double cc;
    cd ss;
    if (std::abs(a) == 0.0) {
      cc = 0.0;
      ss = 1.0;
    } else {
      const double rho = std::sqrt(std::norm(a) + std::norm(bb));
      cc = std::abs(a) / rho;
      ss = (a / std::abs(a)) * std::conj(bb) / rho;
    }
    f.cs[j] = cc;
    f.sn[j] = ss;
    f.hcol[j] = cc * a + ss * bb;
    f.hcol[j + 1] = 0.0;
    for (int i = 0; i <= j; ++i) f.H[(size_t)i * m + j] = f.hcol[i];
    f.gamma[j + 1] = -std::conj(ss) * f.gamma[j];
    f.gamma[j] = cc * f.gamma[j];
    f.inf.relres_est = std::abs(f.gamma[j + 1]) / f.bnorm;
    f.hist.push_back(f.inf.relres_est);
    if (f.inf.relres_est <= g.o.tol || hn == 0.0 || f.iters >= g.o.maxit || j + 1 == m)
      g.ended.push_back(&f);
    else
      g.going.push_back(&f);
  }
  if (!g.going.empty()) {  // V_{j+1} = w / |w|
    if (!g.lazy) {
      Timed tm(g.c, HDDM_K_KRYLOV, s);
      HIPCHK(hddm::launch_arnoldi_scale(kset_of(g.going, false), m, g.c->n(), 0, s));
    }
    for (Fg* fp : g.going) fp->j += 1;
  }
  return HDDM_OK;
}

// End of a cycle for g.ended: y = R^-1 gamma (back substitution, host),
// x += Z y, true residual r = b - M x into V_0 and its norm.
hddm_status fg_launch_cycle_end(FgGroup& g, hipStream_t s) {
  const int m = g.o.restart;
  for (Fg* fp : g.ended) {
    Fg& f = *fp;
    const int kdone = f.j + 1;
    cd* y = f.hs + 3 * (m + 1);
    for (int i = kdone - 1; i >= 0; --i) {
      cd acc = f.gamma[i];
      for (int k = i + 1; k < kdone; ++k) acc -= f.H[(size_t)i * m + k] * y[k];
      y[i] = acc / f.H[(size_t)i * m + i];
    }
  }
  HIPCHK(hipMemcpyAsync(g.sums, g.hsum->data(), g.hsum->size() * sizeof(cd), hipMemcpyHostToDevice,
                        s));
  hddm::KSet ks = kset_of(g.ended, g.lazy);
  Timed tm(g.c, HDDM_K_KRYLOV, s);
  HIPCHK(hddm::launch_combine(ks, m, g.c->n(), g.c->mixed(), s));
  HIPCHK(hddm::launch_residual(ks, m, g.c->d_gtab(), g.c->d_k2(), g.c->ngx, g.c->ngy, g.sm, s));
  return HDDM_OK;
}

hddm_status fg_after_cycle_end(FgGroup& g, hipStream_t s) {
  const int m = g.o.restart;
  std::vector<Fg*> again;
  for (Fg* fp : g.ended) {
    Fg& f = *fp;
    const double rn = fg_rn(f, m);
    f.inf.relres_true = rn / f.bnorm;
    if (!std::isfinite(rn)) {
      f.inf.status = HDDM_EBREAKDOWN;
      f.running = false;
    } else if (f.inf.relres_true <= g.o.tol) {
      f.running = false;
    } else if (f.iters >= g.o.maxit) {
      f.inf.status = HDDM_ENOCONV;
      f.running = false;
    } else {
      std::fill(f.gamma.begin(), f.gamma.end(), cd(0));
      f.gamma[0] = rn;
      f.j = 0;
      f.inf.restarts++;
      again.push_back(&f);
    }
  }
  if (!again.empty() && !g.lazy) {  // V_0 = r / |r|
    Timed tm(g.c, HDDM_K_KRYLOV, s);
    HIPCHK(hddm::launch_arnoldi_scale(kset_of(again, false), m, g.c->n(), 1, s));
  }
  for (Fg& f : *g.st) f.inf.iters = f.iters;
  return HDDM_OK;
}

// One round for the groups gs (each with running right-hand sides collected
// in its run list), after `apply` has put every Z_j: Arnoldi, read, Givens,
// cycle ends.
hddm_status fg_round(std::vector<FgGroup*>& gs, hipStream_t s) {
  hddm_status e;
  for (FgGroup* g : gs)
    if ((e = fg_launch_arnoldi(*g, s))) return e;
  if ((e = fg_read(gs, s))) return e;
  std::vector<FgGroup*> cyc;
  for (FgGroup* g : gs) {
    if ((e = fg_after_arnoldi(*g, s))) return e;
    if (!g->ended.empty()) cyc.push_back(g);
  }
  if (cyc.empty()) return HDDM_OK;
  for (FgGroup* g : cyc)
    if ((e = fg_launch_cycle_end(*g, s))) return e;
  if ((e = fg_read(cyc, s))) return e;
  for (FgGroup* g : cyc)
    if ((e = fg_after_cycle_end(*g, s))) return e;
  return HDDM_OK;
}

// FGMRES of the right-hand sides `st` of one context to the end; `apply`
// serves each round's preconditioner applications (Z_j = P^-1 V_j for the
// running right-hand sides it is given).
template <typename Apply>
hddm_status fgmres(hddm_ctx* c, std::vector<Fg>& st, const hddm_solve_opts& o, double2* sums,
                   std::vector<cd>& hsum, Apply apply, bool lazy,
                   const hddm::SrcMap& sm, hipStream_t s) {
  FgGroup g;
  g.c = c;
  g.st = &st;
  g.o = o;
  g.sums = sums;
  g.hsum = &hsum;
  g.lazy = lazy;
  g.sm = sm;
  std::vector<FgGroup*> gs{&g};
  hddm_status e;
  if ((e = fg_launch_init(g, s)) || (e = fg_read(gs, s)) || (e = fg_after_init(g, s))) return e;
  while (fg_collect(g)) {
    if ((e = apply(g.run))) return e;
    if ((e = fg_round(gs, s))) return e;
  }
  for (Fg& f : st) f.inf.iters = f.iters;
  return HDDM_OK;
}

// Points the state of each right-hand side at its Krylov region; summaries
// either inside the regions (sums == nullptr) or packed at `sums`.
void carve(std::vector<Fg>& st, const hddm_ctx* c, int m, char* kb, size_t region, double2* sums,
           std::vector<cd>& hsum) {
  size_t offs[6];
  krylov_need(c, m, offs);
  for (size_t k = 0; k < st.size(); ++k) {
    char* base = kb + k * region;
    Fg& f = st[k];
    f.V = reinterpret_cast<double2*>(base + offs[0]);
    f.Z = base + offs[1];
    f.part = reinterpret_cast<double2*>(base + offs[2]);
    f.npart = reinterpret_cast<double*>(base + offs[3]);
    f.sum = sums ? sums + k * summary_len(m) : reinterpret_cast<double2*>(base + offs[4]);
    f.gram = reinterpret_cast<double2*>(base + offs[5]);
    f.hs = hsum.data() + k * summary_len(m);
  }
}

hddm_status check_opts(const hddm_solve_opts* o) {
  const int m = o->restart;
  if (m < 1 || o->maxit < 1 || !(o->tol > 0) || o->ortho < 0 || o->ortho > 1)
    return fail(HDDM_EINVAL, "bad solve options");
  if (o->ortho == 1 && m + 1 > 1024) return fail(HDDM_EINVAL, "restart too long for ortho = 1");
  return HDDM_OK;
}

hddm_status report(hddm_ctx* c, const std::vector<Fg>& st, hddm_solve_info* info) {
  c->hist.clear();
  for (const Fg& f : st) c->hist.push_back(f.hist);
  c->has_hist = true;
  hddm_status worst = HDDM_OK;
  for (size_t k = 0; k < st.size(); ++k) {
    if (info) info[k] = st[k].inf;
    if (st[k].inf.status == HDDM_EBREAKDOWN) worst = HDDM_EBREAKDOWN;
    else if (st[k].inf.status == HDDM_ENOCONV && worst == HDDM_OK) worst = HDDM_ENOCONV;
  }
  if (worst == HDDM_ENOCONV) return fail(HDDM_ENOCONV, "maxit reached before tol");
  if (worst == HDDM_EBREAKDOWN) return fail(HDDM_EBREAKDOWN, "non-finite value in the iteration");
  return HDDM_OK;
}

bool block_ok(const hddm_ctx* c) { return c->nd || (c->packed && c->blk_nt > 0); }

// Appends context c (line factor, block form) to the boxes of a block sweep
// launch: entry b.n - 1, its workgroups following those of the entries
// before it.
void add_to_batch(hddm::BlockBatch& b, const hddm_ctx* c, float2* Xb, const float2* Sb) {
  const int i = b.n - 1;
  b.desc[i] = c->d_desc();
  b.ltab[i] = c->d_ltab();
  b.G[i] = reinterpret_cast<const float2*>(c->factor);
  b.X[i] = Xb;
  b.S[i] = Sb;
  b.tr[i] = c->max_tile_rows;
  b.start[i + 1] = b.start[i] + c->nboxes;
}

size_t block_sums_bytes(int m, int nrhs) { return align256((size_t)nrhs * summary_len(m) * 16); }

// Block form of the preconditioner: the sweeps of all boxes on the sources
// already in the source planes Sb (0..15), solutions into Xb, then output
// k <- plane slot[k] summed over boxes (times 1/nu[k][0] if given).
template <typename CO>
hddm_status block_sweep_gather(hddm_ctx* c, const hddm::GatherList<CO>& gl, int nz, float2* Xb,
                               const float2* Sb, hipStream_t s, const hddm::KLaunch* first,
                               int first_cls) {
  // [first (the restriction of a stand-alone apply)] -> sweep (nested
  // dissection: forward launches from the deepest level, backward launches
  // from the root) -> gather, one graph launch
  const int nmax = 2 + (c->nd ? 2 * c->ndp.depths : 1);
  std::vector<hddm::KLaunch> ks(nmax);
  std::vector<int> cls(nmax);
  int n = 0;
  if (first) {
    ks[n] = *first;
    cls[n++] = first_cls;
  }
  if (c->nd) {
    const hddm::NDPlan& pl = c->ndp;
    const hddm::NDDev nd = c->nd_dev();
    const double2* G = reinterpret_cast<const double2*>(c->factor);
    float2* V = Xb + c->nd_v_entries;
    for (int d = pl.depths - 1; d >= 0; --d) {
      HIPCHK(hddm::describe_nd_forward(ks[n], nd, d, pl.maxcnt[d], c->nboxes, pl.maxw[d],
                                       c->d_desc(), G, Sb, c->max_tile_rows, c->blk_xw, Xb, V));
      cls[n++] = HDDM_K_SWEEP;
    }
    for (int d = 0; d < pl.depths; ++d) {
      HIPCHK(hddm::describe_nd_backward(ks[n], nd, d, pl.maxcnt[d], c->nboxes, pl.maxw[d],
                                        c->d_desc(), G, Xb));
      cls[n++] = HDDM_K_SWEEP;
    }
  } else {
    hddm::BlockBatch b{};
    b.n = 1;
    add_to_batch(b, c, Xb, Sb);
    HIPCHK(hddm::describe_sweep_block(ks[n], b, c->blk_nt, c->blk_variant));
    cls[n++] = HDDM_K_SWEEP;
  }
  if constexpr (std::is_same<CO, float2>::value)
    HIPCHK(hddm::describe_gather_block_c64(ks[n], c->d_desc(), c->d_cx(), c->d_cy(), Xb, gl, nz,
                                           c->ngx, c->ngy, c->nbx, c->blk_xw, c->d_wx(),
                                           c->d_wy(), c->nd));
  else
    HIPCHK(hddm::describe_gather_block_c128(ks[n], c->d_desc(), c->d_cx(), c->d_cy(), Xb, gl, nz,
                                            c->ngx, c->ngy, c->nbx, c->blk_xw, c->d_wx(),
                                            c->d_wy(), c->nd));
  cls[n++] = HDDM_K_GATHER;
  return run_launches(c, ks.data(), cls.data(), n, s);
}

hddm::SrcMap block_srcmap(const hddm_ctx* c, float2* S) {
  hddm::SrcMap sm{};
  sm.S = S;
  sm.own_x = c->d_ownx();
  sm.own_y = c->d_owny();
  sm.nbx = c->nbx;
  sm.tr = c->max_tile_rows;
  sm.xw = c->blk_xw;
  return sm;
}

}  // namespace

extern "C" {

hddm_status hddm_solve(hddm_ctx* c, const void* rhs, void* xout, const hddm_solve_opts* opts,
                       hddm_solve_info* info, void* krylov_buf, size_t krylov_bytes,
                       void* stream) {
  hddm_status st = check_ctx(c, kFactored);
  if (st) return st;
  if (!rhs || !xout || !opts || !krylov_buf) return fail(HDDM_EINVAL, "null argument");
  if ((st = check_opts(opts))) return st;
  const int m = opts->restart;
  size_t offs[6];
  const size_t need = krylov_need(c, m, offs);
  if (krylov_bytes < need) return fail(HDDM_ENOMEM, "krylov buffer too small for this restart");
  if ((uintptr_t)krylov_buf & 255) return fail(HDDM_EINVAL, "krylov buffer must be 256-byte aligned");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  HIPCHK(hipSetDevice(c->device));
  std::vector<Fg> fs(1);
  std::vector<cd> hsum(summary_len(m));
  carve(fs, c, m, static_cast<char*>(krylov_buf), need, nullptr, hsum);
  fs[0].b = static_cast<const double2*>(rhs);
  fs[0].x = static_cast<double2*>(xout);
  auto apply = [&](std::vector<Fg*>& run) -> hddm_status {
    Fg& f = *run[0];
    const size_t zel = c->mixed() ? 8 : 16;
    return single_apply(c, f.V + (size_t)f.j * c->n(), f.Z + (size_t)f.j * c->n() * zel,
                        c->mixed(), s);
  };
  st = fgmres(c, fs, *opts, fs[0].sum, hsum, apply, false, hddm::SrcMap{}, s);
  if (st) return st;
  return report(c, fs, info);
}

hddm_status hddm_query_block_bytes(const hddm_ctx* c, int32_t nrhs, int32_t restart,
                                   size_t* block_work_bytes, size_t* krylov_bytes) {
  if (!c) return fail(HDDM_EINVAL, "null context");
  if (!block_ok(c))
    return fail(HDDM_EINVAL, "the block form needs complex64 symmetric-packed factors and boxes "
                             "at most 192 nodes wide");
  if (nrhs < 1 || nrhs > HDDM_BLOCK_MAX) return fail(HDDM_EINVAL, "nrhs must be in 1..16");
  if (restart < 1) return fail(HDDM_EINVAL, "restart must be >= 1");
  size_t offs[6];
  if (block_work_bytes) *block_work_bytes = c->blk_bytes();
  if (krylov_bytes)
    *krylov_bytes = (size_t)nrhs * krylov_need(c, restart, offs) + block_sums_bytes(restart, nrhs);
  return HDDM_OK;
}

hddm_status hddm_apply_precond_block(hddm_ctx* c, const void* r, int64_t ldr, void* z,
                                     int64_t ldz, int32_t nrhs, void* block_work,
                                     size_t block_work_bytes, void* stream) {
  hddm_status st = check_ctx(c, kFactored);
  if (st) return st;
  if (!block_ok(c))
    return fail(HDDM_EINVAL, "the block form needs complex64 symmetric-packed factors and boxes "
                             "at most 192 nodes wide");
  if (!r || !z || !block_work) return fail(HDDM_EINVAL, "null argument");
  if (nrhs < 1 || nrhs > HDDM_BLOCK_MAX) return fail(HDDM_EINVAL, "nrhs must be in 1..16");
  if ((nrhs > 1 && (ldr < c->n() || ldz < c->n())))
    return fail(HDDM_EINVAL, "vector strides must be at least the grid size");
  if (block_work_bytes < c->blk_bytes()) return fail(HDDM_ENOMEM, "block workspace too small");
  if ((uintptr_t)block_work & 255) return fail(HDDM_EINVAL, "block workspace must be 256-byte aligned");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  HIPCHK(hipSetDevice(c->device));
  hddm::VecList rl{};
  hddm::GatherList<double2> gl{};
  for (int k = 0; k < hddm::BLOCK_RHS; ++k) {  // unused slots repeat the first vector
    const int kk = k < nrhs ? k : 0;
    rl.p[k] = static_cast<const double2*>(r) + (size_t)kk * ldr;
    gl.slot[k] = kk;
    gl.z[k] = static_cast<double2*>(z) + (size_t)kk * ldz;
    gl.nu[k] = nullptr;
  }
  float2* Xb = static_cast<float2*>(block_work);
  float2* Sb = c->blk_S(block_work);
  hddm::KLaunch rk;
  HIPCHK(hddm::describe_restrict_block(rk, c->d_desc(), c->nboxes, c->max_tile_rows, rl, nrhs, Sb,
                                       c->ngx, c->blk_xw));
  return block_sweep_gather<double2>(c, gl, nrhs, Xb, Sb, s, &rk, HDDM_K_RESTRICT);
}

hddm_status hddm_solve_block(hddm_ctx* c, const void* rhs, int64_t ldb, void* xout, int64_t ldx,
                             int32_t nrhs, const hddm_solve_opts* opts, hddm_solve_info* info,
                             void* block_work, size_t block_work_bytes, void* krylov_buf,
                             size_t krylov_bytes, void* stream) {
  hddm_status st = check_ctx(c, kFactored);
  if (st) return st;
  if (!block_ok(c))
    return fail(HDDM_EINVAL, "the block form needs complex64 symmetric-packed factors and boxes "
                             "at most 192 nodes wide");
  if (!rhs || !xout || !opts || !block_work || !krylov_buf) return fail(HDDM_EINVAL, "null argument");
  if (nrhs < 1 || nrhs > HDDM_BLOCK_MAX) return fail(HDDM_EINVAL, "nrhs must be in 1..16");
  if (nrhs > 1 && (ldb < c->n() || ldx < c->n()))
    return fail(HDDM_EINVAL, "vector strides must be at least the grid size");
  if ((st = check_opts(opts))) return st;
  const int m = opts->restart;
  size_t offs[6];
  const size_t region = krylov_need(c, m, offs);
  if (krylov_bytes < (size_t)nrhs * region + block_sums_bytes(m, nrhs))
    return fail(HDDM_ENOMEM, "krylov buffer too small for this restart and nrhs");
  if (block_work_bytes < c->blk_bytes()) return fail(HDDM_ENOMEM, "block workspace too small");
  if (((uintptr_t)krylov_buf | (uintptr_t)block_work) & 255)
    return fail(HDDM_EINVAL, "buffers must be 256-byte aligned");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  HIPCHK(hipSetDevice(c->device));
  char* kb = static_cast<char*>(krylov_buf);
  double2* sums = reinterpret_cast<double2*>(kb + (size_t)nrhs * region);
  std::vector<Fg> fs(nrhs);
  std::vector<cd> hsum((size_t)nrhs * summary_len(m));
  carve(fs, c, m, kb, region, sums, hsum);
  for (int k = 0; k < nrhs; ++k) {
    fs[k].b = static_cast<const double2*>(rhs) + (size_t)k * ldb;
    fs[k].x = static_cast<double2*>(xout) + (size_t)k * ldx;
  }
  float2* Xb = static_cast<float2*>(block_work);
  float2* Sb = c->blk_S(block_work);
  const int64_t n = c->n();
  for (int k = 0; k < nrhs; ++k) fs[k].slot = k;
  // sources: the Krylov kernels write only tile nodes, so the rest stays zero;
  // planes of right-hand sides that are not (or no longer) solved hold zeros
  // or an earlier source: their columns are computed and never read
  HIPCHK(hddm::launch_zero(Sb, (size_t)c->blk_s_entries * 8, s));
  auto apply = [&](std::vector<Fg*>& run) -> hddm_status {
    hddm::GatherList<float2> gl{};
    const int nr = (int)run.size();
    for (int k = 0; k < hddm::BLOCK_RHS; ++k) {
      const Fg& f = *run[k < nr ? k : 0];
      gl.slot[k] = f.slot;
      gl.z[k] = reinterpret_cast<float2*>(f.Z) + (size_t)f.j * n;
      gl.nu[k] = reinterpret_cast<const double*>(f.sum + 4 * m + 4) + f.j;  // nu_j
    }
    return block_sweep_gather<float2>(c, gl, nr, Xb, Sb, s);
  };
  st = fgmres(c, fs, *opts, sums, hsum, apply, true, block_srcmap(c, Sb), s);
  if (st) return st;
  return report(c, fs, info);
}

hddm_status hddm_solve_history(const hddm_ctx* c, int32_t rhs, double* out, int32_t cap,
                               int32_t* n) {
  if (!c || !n) return fail(HDDM_EINVAL, "null argument");
  if (!c->has_hist) return fail(HDDM_ESTATE, "no solve has completed on this context");
  if (rhs < 0 || rhs >= (int32_t)c->hist.size())
    return fail(HDDM_EINVAL, "rhs outside the last solve's right-hand sides");
  if (cap < 0 || (cap > 0 && !out)) return fail(HDDM_EINVAL, "bad output buffer");
  const std::vector<double>& h = c->hist[(size_t)rhs];
  *n = (int32_t)h.size();
  const size_t k = std::min((size_t)cap, h.size());
  std::copy(h.begin(), h.begin() + (long)k, out);
  return HDDM_OK;
}

}  // extern "C"

// ---- Preconditioner applications of several contexts in one launch
// sequence: their restrictions, one block sweep over the union of their
// boxes, their gathers.

namespace {

// Checks shared by the batched entry points: context i takes part in a fused
// block sweep (line factor, block form, the kernel width of the others).
hddm_status batch_ok(hddm_ctx* const* ctxs, int32_t n) {
  if (!ctxs || n < 1 || n > hddm::BATCH_MAX) return fail(HDDM_EINVAL, "1..8 contexts per batch");
  for (int i = 0; i < n; ++i) {
    hddm_ctx* c = ctxs[i];
    hddm_status st = check_ctx(c, kFactored);
    if (st) return st;
    if (c->nd || !c->packed || c->blk_nt <= 0)
      return fail(HDDM_EINVAL, "batched applications need the block form of the line factor "
                               "(complex64 symmetric-packed, boxes at most 192 wide)");
    if (c->blk_nt != ctxs[0]->blk_nt || c->device != ctxs[0]->device)
      return fail(HDDM_EINVAL, "contexts of a batch need boxes of the same tile-block width "
                               "on the same device");
    for (int k = 0; k < i; ++k)
      if (ctxs[k] == c) return fail(HDDM_EINVAL, "a context appears twice in the batch");
  }
  return HDDM_OK;
}

}  // namespace

extern "C" {

hddm_status hddm_apply_precond_batch(hddm_ctx* const* ctxs, int32_t n, const void* const* r,
                                     const int64_t* ldr, void* const* z, const int64_t* ldz,
                                     const int32_t* nrhs, void* const* block_work,
                                     const size_t* block_work_bytes, void* stream) {
  hddm_status st = batch_ok(ctxs, n);
  if (st) return st;
  if (!r || !ldr || !z || !ldz || !nrhs || !block_work || !block_work_bytes)
    return fail(HDDM_EINVAL, "null argument");
  for (int i = 0; i < n; ++i) {
    const hddm_ctx* c = ctxs[i];
    if (!r[i] || !z[i] || !block_work[i]) return fail(HDDM_EINVAL, "null vector or workspace");
    if (nrhs[i] < 1 || nrhs[i] > HDDM_BLOCK_MAX) return fail(HDDM_EINVAL, "nrhs must be in 1..16");
    if (nrhs[i] > 1 && (ldr[i] < c->n() || ldz[i] < c->n()))
      return fail(HDDM_EINVAL, "vector strides must be at least the grid size");
    if (block_work_bytes[i] < c->blk_bytes()) return fail(HDDM_ENOMEM, "block workspace too small");
    if ((uintptr_t)block_work[i] & 255)
      return fail(HDDM_EINVAL, "block workspaces must be 256-byte aligned");
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  HIPCHK(hipSetDevice(ctxs[0]->device));
  std::vector<hddm::KLaunch> ks(2 * n + 1);
  std::vector<int> cls(2 * n + 1);
  hddm::BlockBatch b{};
  for (int i = 0; i < n; ++i) {
    hddm_ctx* c = ctxs[i];
    float2* Xb = static_cast<float2*>(block_work[i]);
    float2* Sb = c->blk_S(block_work[i]);
    hddm::VecList rl{};
    hddm::GatherList<double2> gl{};
    for (int k = 0; k < hddm::BLOCK_RHS; ++k) {  // unused slots repeat the first vector
      const int kk = k < nrhs[i] ? k : 0;
      rl.p[k] = static_cast<const double2*>(r[i]) + (size_t)kk * ldr[i];
      gl.slot[k] = kk;
      gl.z[k] = static_cast<double2*>(z[i]) + (size_t)kk * ldz[i];
      gl.nu[k] = nullptr;
    }
    HIPCHK(hddm::describe_restrict_block(ks[i], c->d_desc(), c->nboxes, c->max_tile_rows, rl,
                                         nrhs[i], Sb, c->ngx, c->blk_xw));
    cls[i] = HDDM_K_RESTRICT;
    b.n = i + 1;
    add_to_batch(b, c, Xb, Sb);
    HIPCHK(hddm::describe_gather_block_c128(ks[n + 1 + i], c->d_desc(), c->d_cx(), c->d_cy(), Xb,
                                            gl, nrhs[i], c->ngx, c->ngy, c->nbx, c->blk_xw,
                                            c->d_wx(), c->d_wy(), false));
    cls[n + 1 + i] = HDDM_K_GATHER;
  }
  HIPCHK(hddm::describe_sweep_block(ks[n], b, ctxs[0]->blk_nt, ctxs[0]->blk_variant));
  cls[n] = HDDM_K_SWEEP;
  return run_launches(ctxs[0], ks.data(), cls.data(), 2 * n + 1, s);
}

}  // extern "C"

// ---- Solver session: block FGMRES problems of several contexts advanced
// together, one round at a time, every round's preconditioner applications
// served by one fused launch sequence.
struct hddm_session {
  struct Prob {
    int32_t id = 0;
    hddm_ctx* c = nullptr;
    std::vector<Fg> st;
    std::vector<cd> hsum;
    FgGroup g;
    bool inited = false;
    bool finished = false;
  };
  std::vector<std::unique_ptr<Prob>> probs;
  int32_t next_id = 1;
  int device = -1;
  int blk_nt = 0;
  // holder of the graphs of the fused launches (kernel choice: 3M + LDS)
  hddm_ctx launcher;
};

extern "C" {

hddm_status hddm_session_create(hddm_session** out) {
  if (!out) return fail(HDDM_EINVAL, "null argument");
  *out = new hddm_session();
  return HDDM_OK;
}

hddm_status hddm_session_add(hddm_session* ss, hddm_ctx* c, const void* rhs, int64_t ldb,
                             void* xout, int64_t ldx, int32_t nrhs, const hddm_solve_opts* opts,
                             void* block_work, size_t block_work_bytes, void* krylov_buf,
                             size_t krylov_bytes, int32_t* id) {
  if (!ss || !id) return fail(HDDM_EINVAL, "null argument");
  hddm_status st = batch_ok(&c, 1);
  if (st) return st;
  if (!rhs || !xout || !opts || !block_work || !krylov_buf) return fail(HDDM_EINVAL, "null argument");
  if (nrhs < 1 || nrhs > HDDM_BLOCK_MAX) return fail(HDDM_EINVAL, "nrhs must be in 1..16");
  if (nrhs > 1 && (ldb < c->n() || ldx < c->n()))
    return fail(HDDM_EINVAL, "vector strides must be at least the grid size");
  if ((st = check_opts(opts))) return st;
  int active = 0;
  for (auto& p : ss->probs) {
    if (p->c == c) return fail(HDDM_EINVAL, "the context already has a problem in the session");
    active += 1;
  }
  if (active >= hddm::BATCH_MAX) return fail(HDDM_EINVAL, "the session holds 8 problems");
  if (active > 0 && (c->blk_nt != ss->blk_nt || c->device != ss->device))
    return fail(HDDM_EINVAL, "problems of a session need boxes of the same tile-block width on "
                             "the same device");
  const int m = opts->restart;
  size_t offs[6];
  const size_t region = krylov_need(c, m, offs);
  if (krylov_bytes < (size_t)nrhs * region + block_sums_bytes(m, nrhs))
    return fail(HDDM_ENOMEM, "krylov buffer too small for this restart and nrhs");
  if (block_work_bytes < c->blk_bytes()) return fail(HDDM_ENOMEM, "block workspace too small");
  if (((uintptr_t)krylov_buf | (uintptr_t)block_work) & 255)
    return fail(HDDM_EINVAL, "buffers must be 256-byte aligned");
  auto p = std::make_unique<hddm_session::Prob>();
  p->id = ss->next_id++;
  p->c = c;
  p->st.resize(nrhs);
  p->hsum.assign((size_t)nrhs * summary_len(m), cd(0));
  char* kb = static_cast<char*>(krylov_buf);
  double2* sums = reinterpret_cast<double2*>(kb + (size_t)nrhs * region);
  carve(p->st, c, m, kb, region, sums, p->hsum);
  for (int k = 0; k < nrhs; ++k) {
    p->st[k].b = static_cast<const double2*>(rhs) + (size_t)k * ldb;
    p->st[k].x = static_cast<double2*>(xout) + (size_t)k * ldx;
    p->st[k].slot = k;
  }
  FgGroup& g = p->g;
  g.c = c;
  g.st = &p->st;
  g.o = *opts;
  g.sums = sums;
  g.hsum = &p->hsum;
  g.lazy = true;
  g.Xb = static_cast<float2*>(block_work);
  g.Sb = c->blk_S(block_work);
  g.sm = block_srcmap(c, g.Sb);
  ss->device = c->device;
  ss->blk_nt = c->blk_nt;
  *id = p->id;
  ss->probs.push_back(std::move(p));
  return HDDM_OK;
}

hddm_status hddm_session_step(hddm_session* ss, void* stream, int32_t* finished, int32_t* nfinished) {
  if (!ss || !finished || !nfinished) return fail(HDDM_EINVAL, "null argument");
  *nfinished = 0;
  if (ss->probs.empty()) return HDDM_OK;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  HIPCHK(hipSetDevice(ss->device));
  hddm_status e;
  // problems added since the last round: x = 0, first residuals and sources
  std::vector<FgGroup*> fresh;
  for (auto& p : ss->probs)
    if (!p->inited) {
      HIPCHK(hddm::launch_zero(p->g.Sb, (size_t)p->c->blk_s_entries * 8, s));
      if ((e = fg_launch_init(p->g, s))) return e;
      fresh.push_back(&p->g);
    }
  if (!fresh.empty()) {
    if ((e = fg_read(fresh, s))) return e;
    for (auto& p : ss->probs)
      if (!p->inited) {
        if ((e = fg_after_init(p->g, s))) return e;
        p->inited = true;
      }
  }
  // one round for every problem still iterating
  std::vector<FgGroup*> act;
  for (auto& p : ss->probs)
    if (!p->finished && fg_collect(p->g)) act.push_back(&p->g);
  if (!act.empty()) {
    const int na = (int)act.size();
    std::vector<hddm::KLaunch> ks(na + 1);
    std::vector<int> cls(na + 1);
    hddm::BlockBatch b{};
    for (int i = 0; i < na; ++i) {
      FgGroup& g = *act[i];
      hddm_ctx* c = g.c;
      const int m = g.o.restart, nr = (int)g.run.size();
      hddm::GatherList<float2> gl{};
      for (int k = 0; k < hddm::BLOCK_RHS; ++k) {
        const Fg& f = *g.run[k < nr ? k : 0];
        gl.slot[k] = f.slot;
        gl.z[k] = reinterpret_cast<float2*>(f.Z) + (size_t)f.j * c->n();
        gl.nu[k] = reinterpret_cast<const double*>(f.sum + 4 * m + 4) + f.j;  // nu_j
      }
      b.n = i + 1;
      add_to_batch(b, c, g.Xb, g.Sb);
      HIPCHK(hddm::describe_gather_block_c64(ks[1 + i], c->d_desc(), c->d_cx(), c->d_cy(), g.Xb,
                                             gl, nr, c->ngx, c->ngy, c->nbx, c->blk_xw, c->d_wx(),
                                             c->d_wy(), false));
      cls[1 + i] = HDDM_K_GATHER;
    }
    HIPCHK(hddm::describe_sweep_block(ks[0], b, ss->blk_nt, 1));
    cls[0] = HDDM_K_SWEEP;
    if ((e = run_launches(&ss->launcher, ks.data(), cls.data(), na + 1, s))) return e;
    if ((e = fg_round(act, s))) return e;
  }
  for (auto& p : ss->probs) {
    if (p->finished || !p->inited) continue;
    bool any = false;
    for (const Fg& f : p->st) any = any || f.running;
    if (!any) {
      p->finished = true;
      for (Fg& f : p->st) f.inf.iters = f.iters;
      finished[(*nfinished)++] = p->id;
    }
  }
  return HDDM_OK;
}

hddm_status hddm_session_result(hddm_session* ss, int32_t id, hddm_solve_info* info) {
  if (!ss) return fail(HDDM_EINVAL, "null session");
  for (size_t i = 0; i < ss->probs.size(); ++i) {
    hddm_session::Prob& p = *ss->probs[i];
    if (p.id != id) continue;
    if (!p.finished) return fail(HDDM_ESTATE, "the problem is still iterating");
    hddm_status st = report(p.c, p.st, info);
    ss->probs.erase(ss->probs.begin() + (long)i);
    return st;
  }
  return fail(HDDM_EINVAL, "no problem with this id in the session");
}

hddm_status hddm_session_destroy(hddm_session* ss) {
  if (ss) {
    for (auto& g : ss->launcher.graphs) graph_free(g);
    for (hipEvent_t e : ss->launcher.ev_pool) (void)hipEventDestroy(e);
  }
  delete ss;
  return HDDM_OK;
}

hddm_status hddm_destroy(hddm_ctx* c) {
  if (c) {
    prof_resolve(c);
    for (auto& g : c->graphs) graph_free(g);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  }
  delete c;
  return HDDM_OK;
}

hddm_status hddm_tune(hddm_ctx* c, int32_t sweep_variant, int32_t sweep_threads,
                      int32_t factor_variant) {
  if (!c) return fail(HDDM_EINVAL, "null context");
  if (sweep_variant < 0 || sweep_variant > 2 || factor_variant < 0 || factor_variant > 4 ||
      sweep_threads < 0 || sweep_threads > 1024)
    return fail(HDDM_EINVAL, "unknown kernel variant or thread count");
  c->sweep_variant = sweep_variant;
  c->factor_variant = factor_variant;
  c->sweep_threads = pick_sweep_threads(c->max_m, sweep_threads);
  return HDDM_OK;
}

// Work of hddm_ddm_solve: residuals r (two, c128), the step's sum z (c64 or
// c128 by precision), norm partials and the norm.
static size_t ddm_need(const hddm_ctx* c, size_t* offs) {
  const int64_t n = c->n();
  size_t off = 0;
  offs[0] = off;
  off = align256(off + (size_t)n * 16);
  offs[1] = off;
  off = align256(off + (size_t)n * 16);
  offs[2] = off;
  off = align256(off + (size_t)n * (c->mixed() ? 8 : 16));
  offs[3] = off;
  off = align256(off + (size_t)hddm::krylov_blocks(n) * 8);
  offs[4] = off;
  off = align256(off + 8);
  return off;
}

hddm_status hddm_ddm_query_bytes(const hddm_ctx* c, size_t* work_bytes) {
  if (!c || !work_bytes) return fail(HDDM_EINVAL, "null argument");
  size_t offs[5];
  *work_bytes = ddm_need(c, offs);
  return HDDM_OK;
}

hddm_status hddm_ddm_solve(hddm_ctx* c, const void* rhs, void* xout, int32_t max_steps,
                           double tol, hddm_solve_info* info, void* work, size_t work_bytes,
                           void* stream) {
  hddm_status st = check_ctx(c, kFactored);
  if (st) return st;
  if (!rhs || !xout || !work) return fail(HDDM_EINVAL, "null argument");
  if (max_steps < 1 || !(tol >= 0)) return fail(HDDM_EINVAL, "max_steps >= 1 and tol >= 0");
  size_t offs[5];
  if (work_bytes < ddm_need(c, offs)) return fail(HDDM_ENOMEM, "work buffer too small");
  if ((uintptr_t)work & 255) return fail(HDDM_EINVAL, "work buffer must be 256-byte aligned");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  HIPCHK(hipSetDevice(c->device));
  char* w = static_cast<char*>(work);
  double2* r[2] = {reinterpret_cast<double2*>(w + offs[0]), reinterpret_cast<double2*>(w + offs[1])};
  void* z = w + offs[2];
  double* partial = reinterpret_cast<double*>(w + offs[3]);
  double* nrm = reinterpret_cast<double*>(w + offs[4]);
  const double2* b = static_cast<const double2*>(rhs);
  double2* x = static_cast<double2*>(xout);
  const int64_t n = c->n();
  auto norm = [&](const double2* v, double& out) -> hddm_status {
    {
      Timed tm(c, HDDM_K_KRYLOV, s);
      HIPCHK(hddm::launch_norm(v, n, partial, nrm, s));
    }
    HIPCHK(hipMemcpyAsync(&out, nrm, 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (c->prof_on) prof_resolve(c);
    return HDDM_OK;
  };
  hddm_solve_info inf{};
  HIPCHK(hddm::launch_zero(x, (size_t)n * 16, s));
  HIPCHK(hipMemcpyAsync(r[0], b, (size_t)n * 16, hipMemcpyDeviceToDevice, s));
  double bn = 0.0, rn = 0.0;
  if ((st = norm(b, bn))) return st;
  inf.relres_est = inf.relres_true = bn > 0 ? 1.0 : 0.0;
  int cur = 0;
  while (bn > 0 && inf.iters < max_steps && !(inf.relres_est <= tol)) {
    // sum of this step's local solutions, each box solved with its tile of r
    if ((st = single_apply(c, r[cur], z, c->mixed(), s))) return st;
    {
      Timed tm(c, HDDM_K_KRYLOV, s);
      if (c->mixed())
        HIPCHK(hddm::launch_add_c64(static_cast<const float2*>(z), x, n, s));
      else
        HIPCHK(hddm::launch_add_c128(static_cast<const double2*>(z), x, n, s));
    }
    {
      // next sources: r - M z (summed over the tiles, the neighbours' residuals)
      Timed tm(c, HDDM_K_MATVEC, s);
      if (c->mixed())
        HIPCHK(hddm::launch_matvec_c64in(c->d_gtab(), c->d_k2(), static_cast<const float2*>(z),
                                         r[cur], r[cur ^ 1], c->ngx, c->ngy, s));
      else
        HIPCHK(hddm::launch_matvec_c128(c->d_gtab(), c->d_k2(), static_cast<const double2*>(z),
                                        r[cur], r[cur ^ 1], c->ngx, c->ngy, s));
    }
    cur ^= 1;
    ++inf.iters;
    if ((st = norm(r[cur], rn))) return st;
    inf.relres_est = rn / bn;
    if (!std::isfinite(rn)) break;
  }
  // true residual b - M x
  {
    Timed tm(c, HDDM_K_MATVEC, s);
    HIPCHK(hddm::launch_matvec_c128(c->d_gtab(), c->d_k2(), x, b, r[cur ^ 1], c->ngx, c->ngy, s));
  }
  if ((st = norm(r[cur ^ 1], rn))) return st;
  inf.relres_true = bn > 0 ? rn / bn : 0.0;
  inf.status = !std::isfinite(rn)          ? HDDM_EBREAKDOWN
               : inf.relres_est <= tol || bn == 0 ? HDDM_OK
                                          : HDDM_ENOCONV;
  if (info) *info = inf;
  if (inf.status == HDDM_EBREAKDOWN) return fail(HDDM_EBREAKDOWN, "non-finite residual");
  if (inf.status == HDDM_ENOCONV) return fail(HDDM_ENOCONV, "max_steps reached before tol");
  return HDDM_OK;
}

hddm_status hddm_set_smoothing(hddm_ctx* c, int32_t enable) {
  if (!c) return fail(HDDM_EINVAL, "null context");
  c->smooth = enable != 0;
  return HDDM_OK;
}

hddm_status hddm_use_graphs(hddm_ctx* c, int32_t enable) {
  if (!c) return fail(HDDM_EINVAL, "null context");
  c->use_graphs = enable != 0;
  return HDDM_OK;
}

hddm_status hddm_tune_block(hddm_ctx* c, int32_t variant) {
  if (!c) return fail(HDDM_EINVAL, "null context");
  if (variant < 0 || variant > 3) return fail(HDDM_EINVAL, "unknown block kernel variant");
  c->blk_variant = variant;
  return HDDM_OK;
}

hddm_status hddm_profile(hddm_ctx* c, int32_t enable) {
  if (!c) return fail(HDDM_EINVAL, "null context");
  prof_resolve(c);
  c->prof_on = enable != 0;
  for (int k = 0; k < HDDM_K_COUNT; ++k) {
    c->prof_launches[k] = 0;
    c->prof_ms[k] = 0.0;
  }
  return HDDM_OK;
}

hddm_status hddm_profile_read(hddm_ctx* c, int32_t kernel, int64_t* launches, double* total_ms) {
  if (!c) return fail(HDDM_EINVAL, "null context");
  if (kernel < 0 || kernel >= HDDM_K_COUNT) return fail(HDDM_EINVAL, "unknown kernel class");
  prof_resolve(c);
  if (launches) *launches = c->prof_launches[kernel];
  if (total_ms) *total_ms = c->prof_ms[kernel];
  return HDDM_OK;
}

hddm_status hddm_geometry(const hddm_ctx* c, int32_t* nbx, int32_t* nby, int32_t* boxes) {
  if (!c) return fail(HDDM_EINVAL, "null context");
  if (nbx) *nbx = c->nbx;
  if (nby) *nby = c->nby;
  if (boxes) std::memcpy(boxes, c->geom.data(), c->geom.size() * sizeof(int32_t));
  return HDDM_OK;
}

hddm_status hddm_stretch_tables(const hddm_ctx* c, double* out) {
  if (!c || !out) return fail(HDDM_EINVAL, "null argument");
  std::memcpy(out, c->gstretch.data(), c->gstretch.size() * sizeof(cd));
  return HDDM_OK;
}

}  // extern "C"

namespace hddm {

hddm_status set_error(hddm_status st, const char* msg) { return fail(st, msg); }

int ctx_device(const hddm_ctx* c) { return c->device; }

size_t single_x_bytes(const hddm_ctx* c) { return (size_t)c->x_entries * c->elem; }

hddm_status apply_precond_ws(hddm_ctx* c, const void* r, void* z, void* X, size_t x_bytes,
                             hipStream_t s) {
  hddm_status st = check_ctx(c, kFactored);
  if (st) return st;
  if (c->nd) return fail(HDDM_EINVAL, "needs the line factor (factor_format 0 or 1)");
  if (!r || !z || !X) return fail(HDDM_EINVAL, "null vector");
  if (x_bytes < single_x_bytes(c)) return fail(HDDM_ENOMEM, "box workspace too small");
  HIPCHK(hipSetDevice(c->device));
  hddm::KLaunch ks[2];
  if ((st = describe_single(c, static_cast<const double2*>(r), z, false, X, ks))) return st;
  for (hddm::KLaunch& k : ks) HIPCHK(k.launch(s));
  return HDDM_OK;
}

}  // namespace hddm
