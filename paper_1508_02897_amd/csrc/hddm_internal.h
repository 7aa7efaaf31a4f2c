// Internal declarations shared by the host library and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hddm {

// One overlapping box (Sec. 2: tile widened by the overlap on interior sides
// and by its own layer on every side).  Indices are box-local unless noted.
struct BoxDesc {
  int32_t mx, my;        // box nodes along x / y
  int32_t bx0, by0;      // global index of the box's first node
  int32_t tx0, tx1;      // tile columns inside the box, half-open
  int32_t ty0, ty1;      // tile rows inside the box, half-open
  int64_t g_off;         // entry offset of G_0 in the factor buffer; G_j follows at j*mx*mx
  int64_t x_off;         // entry offset of the box solution (my*mx, row-major) in the workspace
  int32_t tab_off;       // offset (complex entries) of the box's stretch tables:
                         //   ax[mx], ihx[mx+1], ay[my], ihy[my+1]
                         // with ihx = 1 / (h^2 a(x_{i-1/2})) at flux points
  int32_t pad;
  int64_t xb_off;        // entry offset of the box in the block workspace (my rows of
                         // xw * BLOCK_RHS entries), 0 when the block form is unavailable
};

// Block form: right-hand sides per block (the N dimension of the MFMA tiles).
constexpr int BLOCK_RHS = 16;
struct VecList {
  const double2* p[BLOCK_RHS];
};
template <typename T>
struct OutList {
  T* p[BLOCK_RHS];
};

// Gather table entry along one axis: the at most two boxes covering a node.
struct AxisCover {
  int32_t box0, loc0;    // box index along the axis and local index, -1 if none
  int32_t box1, loc1;
};

// Launch wrappers (kernels in hddm_kernels.hip).  All asynchronous on `s`.
hipError_t launch_factor_c128(const BoxDesc* d, const double2* ltab, const double* k2, int ngx,
                              double2* G, int nboxes, int max_m, hipStream_t s);
hipError_t launch_factor_c64(const BoxDesc* d, const double2* ltab, const double* k2, int ngx,
                             float2* G, int nboxes, int max_m, hipStream_t s);
// Complex64 factors.  ws == nullptr: dense column-major G_j in place; else the
// symmetric-packed tile format, `slots` workgroups each using ws_stride
// entries of ws as its working matrix.
hipError_t launch_factor_c64_mfma(const BoxDesc* d, const double2* ltab, const double* k2,
                                  int ngx, float2* G, int nboxes, int max_m, float2* ws,
                                  int64_t ws_stride, int slots, hipStream_t s);
hipError_t launch_factor_c64_packed(const BoxDesc* d, const double2* ltab, const double* k2,
                                    int ngx, float2* G, int nboxes, int max_m, float2* ws,
                                    int64_t ws_stride, int slots, hipStream_t s);
hipError_t launch_sweep_c64_packed(const BoxDesc* d, const double2* ltab, const float2* G,
                                   float2* X, const double2* r, int ngx, int nboxes, int max_m,
                                   bool two_per_cu, hipStream_t s);

hipError_t launch_sweep_c128(const BoxDesc* d, const double2* ltab, const double2* G,
                             double2* X, const double2* r, int ngx, int nboxes, int threads,
                             int max_m, hipStream_t s);
// generic = true selects the one-row-per-thread kernel also for narrow boxes.
hipError_t launch_sweep_c64(const BoxDesc* d, const double2* ltab, const float2* G, float2* X,
                            const double2* r, int ngx, int nboxes, int threads, int max_m,
                            bool generic, hipStream_t s);

hipError_t launch_gather_c128_to_c128(const BoxDesc* d, const AxisCover* cx, const AxisCover* cy,
                                      const double2* X, double2* z, int ngx, int ngy, int nbx,
                                      hipStream_t s);
hipError_t launch_gather_c64_to_c128(const BoxDesc* d, const AxisCover* cx, const AxisCover* cy,
                                     const float2* X, double2* z, int ngx, int ngy, int nbx,
                                     hipStream_t s);
hipError_t launch_gather_c64_to_c64(const BoxDesc* d, const AxisCover* cx, const AxisCover* cy,
                                    const float2* X, float2* z, int ngx, int ngy, int nbx,
                                    hipStream_t s);

// y = M x  (sub_from == nullptr) or  y = sub_from - M x.
hipError_t launch_matvec_c128(const double2* gtab, const double* k2, const double2* x,
                              const double2* sub_from, double2* y, int ngx, int ngy,
                              hipStream_t s);
hipError_t launch_matvec_c64in(const double2* gtab, const double* k2, const float2* x,
                               const double2* sub_from, double2* y, int ngx, int ngy,
                               hipStream_t s);

// Block form (hddm_block.hip).  block_nt: tile blocks per row of the kernel
// instantiation used for boxes of nt tile blocks (0: too wide).  The block
// workspace rows are xw = 16 * block_nt entries wide.
int block_nt(int nt);
hipError_t launch_restrict_block(const BoxDesc* d, int nboxes, int max_tile_rows, VecList r,
                                 int nrhs, float2* X, int ngx, int xw, hipStream_t s);
hipError_t launch_sweep_block(const BoxDesc* d, const double2* ltab, const float2* G, float2* X,
                              int nboxes, int nt_block, hipStream_t s);
hipError_t launch_gather_block_c64(const BoxDesc* d, const AxisCover* cx, const AxisCover* cy,
                                   const float2* X, OutList<float2> z, int nrhs, int ngx, int ngy,
                                   int nbx, int xw, hipStream_t s);
hipError_t launch_gather_block_c128(const BoxDesc* d, const AxisCover* cx, const AxisCover* cy,
                                    const float2* X, OutList<double2> z, int nrhs, int ngx,
                                    int ngy, int nbx, int xw, hipStream_t s);

// Krylov helpers on c128 vectors of length n.  Block partials are reduced in
// a fixed order by a second kernel, so results are deterministic.
int krylov_blocks(int64_t n);
hipError_t launch_mdot(const double2* V, int64_t ldv, int nk, const double2* w, int64_t n,
                       double2* partial, double2* out, hipStream_t s);
// Two right-hand vectors in one pass: out[0..nk) = V^H w0, out[nk..2nk) = V^H w1.
hipError_t launch_mdot2(const double2* V, int64_t ldv, int nk, const double2* w0,
                        const double2* w1, int64_t n, double2* partial, double2* out,
                        hipStream_t s);
// Gram column j <- pq[nk..2nk); c = 2 pq[0..nk) - Gm pq[0..nk)  (nk = j + 1).
hipError_t launch_gram_coef(double2* Gm, int ld, int j, const double2* pq, double2* c,
                            hipStream_t s);
hipError_t launch_mupdate(const double2* V, int64_t ldv, int nk, const double2* coef,
                          double2* w, int64_t n, double* norm_partial, double* norm_out,
                          hipStream_t s);
hipError_t launch_norm(const double2* w, int64_t n, double* partial, double* out, hipStream_t s);
hipError_t launch_scale(double2* w, int64_t n, const double* norm, hipStream_t s);
hipError_t launch_combine_c128(const double2* Z, int64_t ldz, int nk, const double2* y,
                               double2* x, int64_t n, hipStream_t s);
hipError_t launch_combine_c64(const float2* Z, int64_t ldz, int nk, const double2* y, double2* x,
                              int64_t n, hipStream_t s);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);

}  // namespace hddm
