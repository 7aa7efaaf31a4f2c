// Host-only exercise of the C ABI for the address and undefined-behaviour
// sanitizers: setup over several layouts (corner-only, uneven edge boxes,
// nested-dissection plans, one box), buffer queries, geometry and stretch
// introspection, the setup validation paths, the state machine before bind,
// and destroy.  Nothing here reaches a GPU: the kernel launch wrappers are
// never called (the link leaves them unresolved), and the three host helpers
// of the kernel files that setup and the queries use are given below with
// the same results for the shapes used.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/hddm.h"

namespace hddm {
int block_nt(int nt) { return nt <= 4 ? 4 : nt <= 6 ? 6 : nt <= 8 ? 8 : nt <= 10 ? 10 : nt <= 12 ? nt : 0; }
int krylov_blocks(long n) { return (int)((n + 4095) / 4096); }
int krylov_partials(int ngx, int ngy) { return krylov_blocks((long)ngx * ngy) + ngy; }
}  // namespace hddm

static int failures = 0;
#define CHECK(c)                                                    \
  do {                                                              \
    if (!(c)) {                                                     \
      std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
      ++failures;                                                   \
    }                                                               \
  } while (0)

static hddm_problem make(int n, int P, int tile, int n_ol, int prec, int fmt) {
  hddm_problem p{};
  p.nx = p.ny = n;
  p.npml = P;
  p.tile = tile;
  p.n_ol = n_ol;
  p.pml_power = 2;
  p.precision = prec;
  p.factor_format = fmt;
  p.h = 1.0 / n;
  p.omega = 2 * M_PI * 0.8 * n / 10.0;
  p.k_ref = p.omega;
  p.sigma0_over_kref = 20.0;
  return p;
}

int main() {
  struct Case { int n, P, tile, n_ol, prec, fmt; };
  const Case cases[] = {{128, 16, 64, 8, 0, 0},  {96, 8, 32, 4, 1, 0},   {384, 16, 128, 8, 1, 0},
                        {384, 16, 128, 8, 1, 1}, {96, 8, 32, 4, 1, 2},   {320, 30, 160, 50, 1, 2},
                        {64, 8, 64, 0, 0, 0},    {360, 8, 120, 8, 1, 0}};
  for (const Case& k : cases) {
    hddm_problem p = make(k.n, k.P, k.tile, k.n_ol, k.prec, k.fmt);
    const int ng = k.n + 2 * k.P;
    std::vector<double> vel((size_t)ng * ng);
    for (size_t i = 0; i < vel.size(); ++i) vel[i] = 1.0 + 0.3 * std::sin(0.01 * (double)i);
    hddm_ctx* c = nullptr;
    CHECK(hddm_setup(&p, vel.data(), 0, &c) == HDDM_OK);
    if (!c) continue;
    size_t fb = 0, wb = 0, kb = 0, bw = 0, bk = 0;
    CHECK(hddm_query_bytes(c, 30, &fb, &wb, &kb) == HDDM_OK && fb > 0 && wb > 0 && kb > 0);
    CHECK(hddm_query_bytes(c, 3, nullptr, nullptr, nullptr) == HDDM_OK);
    const hddm_status sb = hddm_query_block_bytes(c, 16, 3, &bw, &bk);
    CHECK(sb == HDDM_OK || sb == HDDM_EINVAL);
    CHECK(hddm_query_block_bytes(c, 17, 3, &bw, &bk) == HDDM_EINVAL);
    int32_t nbx = 0, nby = 0;
    CHECK(hddm_geometry(c, &nbx, &nby, nullptr) == HDDM_OK && nbx == k.n / k.tile);
    std::vector<int32_t> g(8 * (size_t)nbx * nby);
    CHECK(hddm_geometry(c, &nbx, &nby, g.data()) == HDDM_OK);
    for (size_t b = 0; b < g.size(); b += 8) CHECK(g[b] < g[b + 1] && g[b + 4] >= g[b]);
    std::vector<double> st(2 * (2 * ng + 1 + 2 * ng + 1));
    CHECK(hddm_stretch_tables(c, st.data()) == HDDM_OK);
    CHECK(st[0] == 1.0);  // real part of the stretch at node 0
    // state machine: nothing runs before bind / factor
    CHECK(hddm_factor(c, nullptr) == HDDM_ESTATE);
    CHECK(hddm_apply_precond(c, nullptr, nullptr, nullptr) == HDDM_ESTATE);
    CHECK(hddm_matvec(c, nullptr, nullptr, nullptr) == HDDM_ESTATE);
    {
      int32_t nh = -1;
      double hbuf[4];
      CHECK(hddm_solve_history(c, 0, hbuf, 4, &nh) == HDDM_ESTATE);
      CHECK(hddm_solve_history(c, 0, nullptr, 0, nullptr) == HDDM_EINVAL);
    }
    CHECK(hddm_tune(c, 9, 0, 0) == HDDM_EINVAL);
    CHECK(hddm_tune_block(c, 7) == HDDM_EINVAL);
    CHECK(hddm_set_smoothing(c, 1) == HDDM_OK);
    CHECK(hddm_use_graphs(c, 0) == HDDM_OK);
    CHECK(hddm_destroy(c) == HDDM_OK);
  }
  // validation paths
  std::vector<double> vel(160 * 160, 1.0);
  hddm_ctx* c = nullptr;
  hddm_problem bad = make(100, 16, 64, 8, 0, 0);
  CHECK(hddm_setup(&bad, vel.data(), 0, &c) == HDDM_EINVAL && c == nullptr);
  CHECK(std::strlen(hddm_last_error()) > 0);
  bad = make(128, 16, 64, 8, 5, 0);
  CHECK(hddm_setup(&bad, vel.data(), 0, &c) == HDDM_EINVAL);
  bad = make(128, 16, 64, 8, 0, 2);  // nested dissection needs complex64
  CHECK(hddm_setup(&bad, vel.data(), 0, &c) == HDDM_EINVAL);
  hddm_problem ok = make(128, 16, 64, 8, 0, 0);
  vel[777] = -1.0;
  CHECK(hddm_setup(&ok, vel.data(), 0, &c) == HDDM_EINVAL);
  vel[777] = NAN;
  CHECK(hddm_setup(&ok, vel.data(), 0, &c) == HDDM_EINVAL);
  CHECK(hddm_setup(nullptr, vel.data(), 0, &c) == HDDM_EINVAL);
  CHECK(hddm_query_bytes(nullptr, 3, nullptr, nullptr, nullptr) == HDDM_EINVAL);
  CHECK(hddm_destroy(nullptr) == HDDM_OK);
  std::printf("host ABI checks: %d failures\n", failures);
  return failures ? 1 : 0;
}
