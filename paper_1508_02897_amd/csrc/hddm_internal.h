// Internal declarations shared by the host library and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

namespace hddm {

// A kernel launch held as data (function, shape, argument values), so that it
// can be launched at once or become a node of a graph whose arguments are
// updated before each replay.
struct KLaunch {
  const void* func = nullptr;
  dim3 grid, block;
  unsigned shmem = 0;
  int nargs = 0;
  unsigned used = 0;
  unsigned off[12] = {};
  void* args[12] = {};
  alignas(16) unsigned char store[768];
  template <typename T>
  void push(const T& v) {
    used = (used + alignof(T) - 1) / alignof(T) * alignof(T);
    memcpy(store + used, &v, sizeof(T));
    off[nargs++] = used;
    used += sizeof(T);
  }
  // argument pointers into this object's own storage
  void** argv() {
    for (int i = 0; i < nargs; ++i) args[i] = store + off[i];
    return args;
  }
  hipKernelNodeParams params() {
    hipKernelNodeParams p{};
    p.func = const_cast<void*>(func);
    p.gridDim = grid;
    p.blockDim = block;
    p.sharedMemBytes = shmem;
    p.kernelParams = argv();
    p.extra = nullptr;
    return p;
  }
  hipError_t launch(hipStream_t s) {
    return hipLaunchKernel(func, grid, block, argv(), shmem, s);
  }
};

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

// Symmetric-packed factor format: the 16x16 tiles on and above the diagonal
// of each G_j, tile (I, J), I <= J, in slot J(J+1)/2 + I of 256 entries,
// row-major inside an off-diagonal tile.  A diagonal tile is itself
// symmetric: its slot holds the entries on and above its diagonal row by row
// (136 entries, (r, c) with r <= c), then zeros in the remaining 120 places,
// so that readers fetch only the first 1088 bytes.
__host__ __device__ constexpr int diag_pos(int r, int c) {
  return r <= c ? r * 16 - r * (r - 1) / 2 + (c - r) : 136 + r * (r - 1) / 2 + c;
}
// where entry (r, c) of a diagonal tile is read from (its stored twin)
__host__ __device__ constexpr int diag_read_pos(int r, int c) {
  return r <= c ? diag_pos(r, c) : diag_pos(c, r);
}
struct VecList {
  const double2* p[BLOCK_RHS];
};
// Block gather targets: output k reads workspace plane slot[k] and writes
// z[k], scaled by 1 / nu[k][0] when nu[k] is given.
template <typename T>
struct GatherList {
  int slot[BLOCK_RHS];
  T* z[BLOCK_RHS];
  const double* nu[BLOCK_RHS];
};

// Gather table entry along one axis: the at most two boxes covering a node.
struct AxisCover {
  int32_t box0, loc0;    // box index along the axis and local index, -1 if none
  int32_t box1, loc1;
};

// Launch wrappers (kernels in hddm_kernels.hip).  All asynchronous on `s`.
// pivstat (may be null): per box, the smallest and largest magnitude of the
// scalar pivots of all its line inversions (the unpivoted Gauss-Jordan's).
hipError_t launch_factor_c128(const BoxDesc* d, const double2* ltab, const double* k2, int ngx,
                              double2* G, int nboxes, int max_m, float2* pivstat, hipStream_t s);
hipError_t launch_factor_c64(const BoxDesc* d, const double2* ltab, const double* k2, int ngx,
                             float2* G, int nboxes, int max_m, float2* pivstat, hipStream_t s);
// Complex64 factors.  ws == nullptr: dense column-major G_j in place; else the
// symmetric-packed tile format, `slots` workgroups each using ws_stride
// entries of ws as its working matrix.
hipError_t launch_factor_c64_mfma(const BoxDesc* d, const double2* ltab, const double* k2,
                                  int ngx, float2* G, int nboxes, int max_m, float2* ws,
                                  int64_t ws_stride, int slots, float2* pivstat, hipStream_t s);
// Register-resident MFMA factor (boxes up to 192 wide), packed or dense G.
hipError_t launch_factor_c64_mfma_regs(const BoxDesc* d, const double2* ltab, const double* k2,
                                       int ngx, float2* G, int nboxes, int max_m, bool packed,
                                       float2* pivstat, hipStream_t s);
// The same inverse by symmetric elimination on the upper tiles only (boxes up
// to 192 wide), packed or dense G.
hipError_t launch_factor_c64_sym_regs(const BoxDesc* d, const double2* ltab, const double* k2,
                                      int ngx, float2* G, int nboxes, int max_m, bool packed,
                                      float2* pivstat, hipStream_t s);
hipError_t launch_factor_c64_packed(const BoxDesc* d, const double2* ltab, const double* k2,
                                    int ngx, float2* G, int nboxes, int max_m, float2* ws,
                                    int64_t ws_stride, int slots, float2* pivstat, hipStream_t s);
// Single-form applications, described for direct or graph launch
// (KLaunch): the sweeps restrict r (FP64) to every box themselves.
hipError_t describe_sweep_c64_packed(KLaunch& k, const BoxDesc* d, const double2* ltab,
                                     const float2* G, float2* X, const double2* r, int ngx,
                                     int nboxes, int max_m, bool two_per_cu);
hipError_t describe_sweep_c128(KLaunch& k, const BoxDesc* d, const double2* ltab,
                               const double2* G, double2* X, const double2* r, int ngx,
                               int nboxes, int threads, int max_m);
// generic = true selects the one-row-per-thread kernel also for narrow boxes.
hipError_t describe_sweep_c64(KLaunch& k, const BoxDesc* d, const double2* ltab, const float2* G,
                              float2* X, const double2* r, int ngx, int nboxes, int threads,
                              int max_m, bool generic);
// wx / wy (null: plain sum): smoothing weights of the covering boxes along
// each axis, (box0, box1) per column / row; box (a, b) adds wy[a] wx[b] x_box.
hipError_t describe_gather_c128_to_c128(KLaunch& k, const BoxDesc* d, const AxisCover* cx,
                                        const AxisCover* cy, const double2* X, double2* z,
                                        int ngx, int ngy, int nbx, const double2* wx,
                                        const double2* wy);
hipError_t describe_gather_c64_to_c128(KLaunch& k, const BoxDesc* d, const AxisCover* cx,
                                       const AxisCover* cy, const float2* X, double2* z, int ngx,
                                       int ngy, int nbx, const double2* wx, const double2* wy);
hipError_t describe_gather_c64_to_c64(KLaunch& k, const BoxDesc* d, const AxisCover* cx,
                                      const AxisCover* cy, const float2* X, float2* z, int ngx,
                                      int ngy, int nbx, const double2* wx, const double2* wy);

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
// The block-form launches are described into a KLaunch (launched directly or
// replayed from a graph); each returns hipErrorInvalidValue for shapes it
// does not support.
// Sources (block workspace S, tr tile rows per plane) of r_0..r_{nrhs-1}.
hipError_t describe_restrict_block(KLaunch& k, const BoxDesc* d, int nboxes, int tr, VecList r,
                                   int nrhs, float2* S, int ngx, int xw);
// The boxes of one block sweep launch: those of up to BATCH_MAX contexts (the
// preconditioner applications of several problems fused into one launch),
// context c owning workgroups start[c] .. start[c+1]-1, each with its own
// descriptors, stretch tables, factor, solution and source planes and tile
// rows per plane.
constexpr int BATCH_MAX = 8;
struct BlockBatch {
  int n;
  int start[BATCH_MAX + 1];
  int tr[BATCH_MAX];
  const BoxDesc* desc[BATCH_MAX];
  const double2* ltab[BATCH_MAX];
  const float2* G[BATCH_MAX];
  float2* X[BATCH_MAX];
  const float2* S[BATCH_MAX];
};
// variant (as hddm_tune_block): 0/1 three real MFMAs per complex product with
// the transposed operand staged in LDS, 2 four real MFMAs, 3 three real MFMAs
// with the transposed operand loaded from memory.  All contexts of the batch
// must use the same nt_block (the kernel's row width).
hipError_t describe_sweep_block(KLaunch& k, const BlockBatch& b, int nt_block, int variant);
hipError_t describe_gather_block_c64(KLaunch& k, const BoxDesc* d, const AxisCover* cx,
                                     const AxisCover* cy, const float2* X,
                                     const GatherList<float2>& z, int nz, int ngx, int ngy,
                                     int nbx, int xw, const double2* wx, const double2* wy,
                                     bool node_major = false);
hipError_t describe_gather_block_c128(KLaunch& k, const BoxDesc* d, const AxisCover* cx,
                                      const AxisCover* cy, const float2* X,
                                      const GatherList<double2>& z, int nz, int ngx, int ngy,
                                      int nbx, int xw, const double2* wx, const double2* wy,
                                     bool node_major = false);

// Arnoldi steps of several right-hand sides in one launch.  Per right-hand side y: basis V (vector k at V + k*n),
// block partials, norm partials, summary (h1[2(m+1)] | h2[m+1] | y[m] |
// norms[2]) and Gram matrix ((m+1) x (m+1)); j is its current Arnoldi index,
// so it has j+1 basis vectors and w = V_{j+1}.
// At the end of a cycle the same descriptor carries Z (P^-1 V, complex64 or
// complex128 by precision), the solution x and the right-hand side b.
// lazy != 0: basis vectors are stored unscaled, V_k = W_k / nu_k, with the
// norms nu_0..nu_m in the summary after the two norms; the kernels fold
// 1/nu_k into every product and coefficient, so no scaling pass is needed.
// slot: the right-hand side's plane in the block workspace.
struct KSet {
  int n;
  int lazy;
  int j[BLOCK_RHS];
  int slot[BLOCK_RHS];
  double2* V[BLOCK_RHS];
  double2* part[BLOCK_RHS];
  double* npart[BLOCK_RHS];
  double2* sum[BLOCK_RHS];
  double2* gram[BLOCK_RHS];
  const void* Z[BLOCK_RHS];
  double2* x[BLOCK_RHS];
  const double2* b[BLOCK_RHS];
};
// Where the block form's next sources go: the source planes S (tr tile rows
// of xw entries per plane, 16 planes per box), plane `slot` of the box whose
// tile owns each node (tiles partition the grid).  S == nullptr: none.
struct SrcMap {
  float2* S;
  const int2* own_x;  // per grid column: (tile index along x, column in its box)
  const int2* own_y;  // per grid row: (tile index along y, row within the tile)
  int nbx, tr, xw;
};
// One Arnoldi step of each right-hand side, w = M z_j formed inside the
// kernels that use it (z_j = Z_j, complex64 if z_c64) and written once, as
// the new basis vector V_{j+1}.  The grid tables gtab / k2 are those of the
// global operator (ngx x ngy nodes).
struct Op {
  const double2* gtab;
  const double* k2;
  int ngx, ngy;
  bool z_c64;
};
// Classical Gram-Schmidt, twice, with the second projection from the Gram
// matrix: h1 <- [V^H w ; V^H v_j], h2 <- 2p - G p, V_{j+1} = w - V h2,
// norms[0] = |V_{j+1}| (lazy: also nu_{j+1}); sm.S: the new vector's
// complex64 source planes are written too.
hipError_t launch_arnoldi_gram(const KSet& ks, int m, const Op& op, const SrcMap& sm,
                               hipStream_t s);
// Classical Gram-Schmidt, twice, with two passes of inner products:
// h1 <- V^H w, w -= V h1, h2 <- V^H w, w -= V h2, norms[0] = |w|.
hipError_t launch_arnoldi_cgs2(const KSet& ks, int m, const Op& op, const SrcMap& sm,
                               hipStream_t s);
// restart == 0: w = V_{j+1} <- w / norms[0]; restart == 1: V_0 <- V_0 / norms[1].
hipError_t launch_arnoldi_scale(const KSet& ks, int m, int64_t n, int restart, hipStream_t s);
// x += Z y (y = summary + 3(m+1), j+1 terms).  z_c64: Z holds complex64 vectors.
hipError_t launch_combine(const KSet& ks, int m, int64_t n, bool z_c64, hipStream_t s);
// V_0 = b - M x, norms[1] = |V_0| (lazy: also nu_0); sm.S: its source planes.
hipError_t launch_residual(const KSet& ks, int m, const double2* gtab, const double* k2,
                           int ngx, int ngy, const SrcMap& sm, hipStream_t s);

// Krylov helpers on c128 vectors of length n.  Block partials are reduced in
// a fixed order by a second kernel, so results are deterministic.
int krylov_blocks(int64_t n);
// Partial sums per right-hand side that the Krylov kernels may write: at
// least krylov_blocks(ngx * ngy) and the number of stencil tiles.
int krylov_partials(int ngx, int ngy);
hipError_t launch_norm(const double2* w, int64_t n, double* partial, double* out, hipStream_t s);
// x += z (z complex64 or complex128, x complex128), n entries.
hipError_t launch_add_c64(const float2* z, double2* x, int64_t n, hipStream_t s);
hipError_t launch_add_c128(const double2* z, double2* x, int64_t n, hipStream_t s);
hipError_t launch_scale(double2* w, int64_t n, const double* norm, hipStream_t s);
hipError_t launch_combine_c128(const double2* Z, int64_t ldz, int nk, const double2* y,
                               double2* x, int64_t n, hipStream_t s);
hipError_t launch_combine_c64(const float2* Z, int64_t ldz, int nk, const double2* y, double2* x,
                              int64_t n, hipStream_t s);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);

// ------------------------------------------------ nested-dissection local solver
// A second local solver for the block form (complex64): each box is ordered by
// nested dissection (a separator line halves the longer side of a rectangle,
// recursively, down to rectangles of at most ND_LEAF nodes) and factorised by
// the multifrontal method with explicit front inverses.  Front F eliminates
// its separator nodes s(F) against the ring b(F) of nodes just outside its
// rectangle (all on ancestor separators).  With the front matrix
// [[A_ss, A_sb], [A_bs, A_bb]] assembled from the local matrix and the
// children's update matrices, the factor keeps G = A_ss^-1 and L = -A_bs G
// (also transposed), complex128, and passes U = A_bb - A_bs G A_sb to the
// parent.  The
// solve: forward, bottom-up, w_s = f_s + (children's update vectors), and the
// parent receives w_b + L w_s; backward, top-down, x_s = G w_s + L^T x_b.
constexpr int ND_LEAF = 16;       // largest leaf rectangle (nodes)
constexpr int ND_MAX_N = 512;     // largest padded front (sp + bp)
constexpr int ND_MAX_W = 448;     // largest front (s + b): its 16 vectors fit 64 KB of LDS

struct NDFront {
  int32_t s, b, sp, bp;   // separator / ring sizes, and both rounded up to 16
  int32_t node_off;       // s separator then b ring nodes (box-local j * mx + x)
  int32_t asm_off;        // per separator node 4 front positions (W, E, S, N neighbour) or -1
  int32_t c0, c1;         // children (indices into the front array) or -1
  int32_t cmap0, cmap1;   // front positions of each child's ring nodes
  int32_t g_off;          // factor entries from the box base: G (s*s), L (b*s), L^T (s*b)
  int32_t u_off;          // update matrix (b*b) in the box's region of this depth's parity
  int32_t v_off;          // update vectors (b*16) likewise
  int32_t depth, pad0, pad1;
};

// Device view of the symbolic tables (all box classes concatenated).
struct NDDev {
  const NDFront* fr;
  const int32_t* nodes;
  const int32_t* asmp;
  const int32_t* cmap;
  const int32_t* dlist;     // front indices, per class and depth
  const int32_t* doff;      // [class * depths + d]: offset into dlist
  const int32_t* dcnt;      // [class * depths + d]: count
  const int32_t* bcls;      // class of every box
  int32_t depths;
  int32_t pad;
  int64_t ustride, vstride; // entries per box and parity
};

hipError_t launch_nd_factor(const NDDev& nd, int d, int maxcnt, int nboxes, int maxn,
                            const BoxDesc* desc, const double2* ltab, const double* k2, int ngx,
                            double2* G, double2* W, int64_t wstride, int nslots, double2* U,
                            hipStream_t s);
hipError_t describe_nd_forward(KLaunch& k, const NDDev& nd, int d, int maxcnt, int nboxes,
                               int maxw, const BoxDesc* desc, const double2* G, const float2* S,
                               int tr, int xw, float2* X, float2* V);
hipError_t describe_nd_backward(KLaunch& k, const NDDev& nd, int d, int maxcnt, int nboxes,
                                int maxw, const BoxDesc* desc, const double2* G, float2* X);

}  // namespace hddm

// Host helpers of the allocation-free entry point (hddm_noalloc.hip), defined
// in hddm_host.cpp.
#include "../../include/hddm.h"
namespace hddm {
hddm_status set_error(hddm_status st, const char* msg);
int ctx_device(const hddm_ctx* c);
// bytes of the line-factor single form's box-solution workspace
size_t single_x_bytes(const hddm_ctx* c);
// hddm_apply_precond with the box solutions in X (x_bytes long) instead of
// the work buffer, each kernel launched directly on s (no graph)
hddm_status apply_precond_ws(hddm_ctx* c, const void* r, void* z, void* X, size_t x_bytes,
                             hipStream_t s);
}  // namespace hddm
