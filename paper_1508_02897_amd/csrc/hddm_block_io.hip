// gfx950 kernels that move data into and out of the block workspace of the
// one-step preconditioner (Leng & Ju, Sec. 2 eq. pc; the layout of the
// workspace, X and S, is described in hddm_block.hip):
//  * restrict_block: the sources of every box from up to 16 residuals
//                    (FP64 -> complex64), for a stand-alone application; in
//                    the solve they are written by the Krylov kernels.
//  * gather_block:   z_k(g) = sum of the (at most four) box solutions
//                    covering g, in the fixed order of the single form,
//                    times 1/nu_k for an unscaled Arnoldi vector.
#include <hip/hip_runtime.h>

#include "hddm_internal.h"

namespace hddm {
namespace {

constexpr int NB = BLOCK_RHS;

__device__ __forceinline__ float2 f2(double2 v) { return make_float2((float)v.x, (float)v.y); }

// --------------------------------------------------------------- restrict
// Sources of every box from r_0..r_{nrhs-1}: plane n, tile row t, entry
// (n, t, x) = r_n at the global node of (ty0 + t, x) for x inside the tile's
// columns, zero elsewhere (and in the planes n >= nrhs).  One block per (box,
// tile row); consecutive threads take consecutive columns of one plane, so
// reads and writes are contiguous.
__global__ __launch_bounds__(256) void restrict_block_kernel(const BoxDesc* __restrict__ desc,
                                                             VecList r, int nrhs,
                                                             float2* __restrict__ S, int tr,
                                                             int ngx, int xw) {
  const BoxDesc bd = desc[blockIdx.x];
  const int t = blockIdx.y, j = bd.ty0 + t;
  if (j >= bd.ty1) return;
  const int64_t grow = (int64_t)(bd.by0 + j) * ngx + bd.bx0;
  float2* __restrict__ Sb = S + (int64_t)blockIdx.x * NB * tr * xw;
  for (int u = threadIdx.x; u < NB * xw; u += blockDim.x) {
    const int n = u / xw, x = u - n * xw;
    float2 v = make_float2(0.f, 0.f);
    if (n < nrhs && x >= bd.tx0 && x < bd.tx1) v = f2(r.p[n][grow + x]);
    Sb[((int64_t)n * tr + t) * xw + x] = v;
  }
}

// ----------------------------------------------------------------- gather
template <typename CO>
__device__ __forceinline__ CO out_of(double re, double im);
template <>
__device__ __forceinline__ float2 out_of<float2>(double re, double im) {
  return make_float2((float)re, (float)im);
}
template <>
__device__ __forceinline__ double2 out_of<double2>(double re, double im) {
  return make_double2(re, im);
}

// z_k(g) = sum over the (at most four) boxes covering g, in the fixed order of
// the single form, of plane slot[k] of their workspace, times 1/nu[k][0] if
// nu[k] is given, for k < nz.  One thread per node (consecutive threads,
// consecutive nodes of a grid row: contiguous reads within a box row and
// contiguous writes); all planes of a box are loaded before any store.
// NM: the workspace is node-major (the nested-dissection solver's layout,
// entry (n, j, x) at xb_off + (j * mx + x) * 16 + n) instead of planes.
template <typename CO, bool SMOOTH, bool NM>
__global__ __launch_bounds__(256) void gather_block_kernel(const BoxDesc* __restrict__ desc,
                                                           const AxisCover* __restrict__ cx,
                                                           const AxisCover* __restrict__ cy,
                                                           const float2* __restrict__ X,
                                                           GatherList<CO> z, int nz, int ngx,
                                                           int ngy, int nbx, int xw,
                                                           const double2* __restrict__ wx,
                                                           const double2* __restrict__ wy) {
  const int gx = blockIdx.x * blockDim.x + threadIdx.x;
  const int gy = blockIdx.y;
  if (gx >= ngx) return;
  const AxisCover ax = cx[gx], ay = cy[gy];
  const int bys[2] = {ay.box0, ay.box1}, lys[2] = {ay.loc0, ay.loc1};
  const int bxs[2] = {ax.box0, ax.box1}, lxs[2] = {ax.loc0, ax.loc1};
  // SMOOTH: box (a, b) weighted by beta = wy[a] * wx[b]
  double wxs[2] = {1.0, 1.0}, wys[2] = {1.0, 1.0};
  if (SMOOTH) {
    const double2 u = wx[gx], w = wy[gy];
    wxs[0] = u.x;
    wxs[1] = u.y;
    wys[0] = w.x;
    wys[1] = w.y;
  }
  double sr[NB], si[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) sr[k] = si[k] = 0.0;
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    if (bys[a] < 0) continue;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      if (bxs[b] < 0) continue;
      const BoxDesc& bd = desc[bys[a] * nbx + bxs[b]];
      const float2* __restrict__ p =
          NM ? X + bd.xb_off + ((int64_t)lys[a] * bd.mx + lxs[b]) * NB
             : X + bd.xb_off + (int64_t)lys[a] * xw + lxs[b];
      const int64_t plane = NM ? 1 : (int64_t)bd.my * xw;
      float2 u[NB];
#pragma unroll
      for (int k = 0; k < NB; ++k) u[k] = p[z.slot[k] * plane];  // unused slots repeat one
      if (SMOOTH) {
        const double wt = wys[a] * wxs[b];
#pragma unroll
        for (int k = 0; k < NB; ++k) {
          sr[k] += wt * u[k].x;
          si[k] += wt * u[k].y;
        }
      } else {
#pragma unroll
        for (int k = 0; k < NB; ++k) {
          sr[k] += u[k].x;
          si[k] += u[k].y;
        }
      }
    }
  }
  const int64_t gi = (int64_t)gy * ngx + gx;
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    if (k >= nz) break;
    const double inv = z.nu[k] ? 1.0 / z.nu[k][0] : 1.0;
    z.z[k][gi] = out_of<CO>(sr[k] * inv, si[k] * inv);
  }
}

}  // namespace

hipError_t describe_restrict_block(KLaunch& k, const BoxDesc* d, int nboxes, int tr, VecList r,
                                   int nrhs, float2* S, int ngx, int xw) {
  if (nrhs < 1 || nrhs > NB) return hipErrorInvalidValue;
  k = KLaunch{};
  k.func = reinterpret_cast<const void*>(&restrict_block_kernel);
  k.grid = dim3(nboxes, tr);
  k.block = dim3(256);
  k.push(d);
  k.push(r);
  k.push(nrhs);
  k.push(S);
  k.push(tr);
  k.push(ngx);
  k.push(xw);
  return hipSuccess;
}

template <typename CO>
static hipError_t describe_gather(KLaunch& k, const BoxDesc* d, const AxisCover* cx,
                                  const AxisCover* cy, const float2* X, const GatherList<CO>& z,
                                  int nz, int ngx, int ngy, int nbx, int xw, const double2* wx,
                                  const double2* wy, bool nm) {
  if (nz < 1 || nz > NB) return hipErrorInvalidValue;
  k = KLaunch{};
  if (nm)
    k.func = wx ? reinterpret_cast<const void*>(&gather_block_kernel<CO, true, true>)
                : reinterpret_cast<const void*>(&gather_block_kernel<CO, false, true>);
  else
    k.func = wx ? reinterpret_cast<const void*>(&gather_block_kernel<CO, true, false>)
                : reinterpret_cast<const void*>(&gather_block_kernel<CO, false, false>);
  k.grid = dim3((ngx + 255) / 256, ngy);
  k.block = dim3(256);
  k.push(d);
  k.push(cx);
  k.push(cy);
  k.push(X);
  k.push(z);
  k.push(nz);
  k.push(ngx);
  k.push(ngy);
  k.push(nbx);
  k.push(xw);
  k.push(wx);
  k.push(wy);
  return hipSuccess;
}
hipError_t describe_gather_block_c64(KLaunch& k, const BoxDesc* d, const AxisCover* cx,
                                     const AxisCover* cy, const float2* X,
                                     const GatherList<float2>& z, int nz, int ngx, int ngy,
                                     int nbx, int xw, const double2* wx, const double2* wy,
                                     bool node_major) {
  return describe_gather(k, d, cx, cy, X, z, nz, ngx, ngy, nbx, xw, wx, wy, node_major);
}
hipError_t describe_gather_block_c128(KLaunch& k, const BoxDesc* d, const AxisCover* cx,
                                      const AxisCover* cy, const float2* X,
                                      const GatherList<double2>& z, int nz, int ngx, int ngy,
                                      int nbx, int xw, const double2* wx, const double2* wy,
                                     bool node_major) {
  return describe_gather(k, d, cx, cy, X, z, nz, ngx, ngy, nbx, xw, wx, wy, node_major);
}

}  // namespace hddm
