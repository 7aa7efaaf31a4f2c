// gfx950 kernels of the nested-dissection local solver (the low-fill
// alternative to the line-by-line factorisation of the local problems of the
// one-step preconditioner, Leng & Ju Sec. 2 eq. pc and Sec. 3), block form:
// 16 right-hand sides.  One launch per depth of the separator tree, each over
// (front of that depth) x (box); the symbolic tables come from the host
// (hddm_nd_plan.cpp).
//
// Precision: the fronts are factorised and stored in complex FP64.  The
// rectangles eliminated first lie inside the box, away from its absorbing
// layer, and their Dirichlet problems can be close to resonance, so rounding
// the front inverses to complex64 can lose most digits of a local solution
// (the line-by-line factor instead eliminates half-boxes that end in the
// layer, which damps them).  The right-hand-side vectors are complex64, the
// products accumulate in FP64.
//
// Front positions: separator node k at k (k < s), padding s..sp-1, ring node p
// at sp + p.  Factor of one front (box base + g_off, complex128): G = A_ss^-1
// (s x s), L = -A_bs G (b x s) and L^T (s x b), all column-major.  Update
// matrices (b x b, column-major, complex128) and update vectors (b x 16,
// node-major, complex64) of depth d live in the box's region of parity d & 1,
// so depth d reads depth d + 1's while writing its own.  Box solutions are
// node-major: entry (n, node) at xb_off + node * 16 + n.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "hddm_device.h"
#include "hddm_internal.h"

namespace hddm {
namespace {

constexpr int NB = BLOCK_RHS;

__device__ __forceinline__ const NDFront& nd_front(const NDDev& nd, int cls, int d, int fi) {
  return nd.fr[nd.dlist[nd.doff[cls * nd.depths + d] + fi]];
}

// ------------------------------------------------------------------ factor
// One workgroup per (box, front) item, grid-strided.  The front matrix is
// assembled in this workgroup's slot of W (column-major n x n, n = sp + bp,
// followed by the three 16 x n Gauss-Jordan panels) and swept by blocked
// Gauss-Jordan over its separator pivots only, which leaves G in the
// separator block, -A_bs G below it and the update matrix in the ring block.
__global__ __launch_bounds__(256) void nd_factor_kernel(
    NDDev nd, int d, int maxcnt, int nboxes, const BoxDesc* __restrict__ desc,
    const double2* __restrict__ ltab, const double* __restrict__ k2, int ngx,
    double2* __restrict__ G, double2* __restrict__ W, int64_t wstride, double2* __restrict__ U) {
  __shared__ double2 Dl[FB * FB];
  const int tid = threadIdx.x;
  double2* Wk = W + (int64_t)blockIdx.x * wstride;
  const int64_t items = (int64_t)nboxes * maxcnt;
  for (int64_t it = blockIdx.x; it < items; it += gridDim.x) {
    const int box = (int)(it / maxcnt), fi = (int)(it - (int64_t)box * maxcnt);
    const int cls = nd.bcls[box];
    if (fi >= nd.dcnt[cls * nd.depths + d]) continue;  // uniform over the workgroup
    const NDFront F = nd_front(nd, cls, d, fi);
    const BoxDesc bd = desc[box];
    const int s = F.s, b = F.b, sp = F.sp, n = F.sp + F.bp;
    double2* Cp = Wk + (int64_t)n * n;
    double2* Rr = Cp + FB * n;
    double2* Rp = Rr + FB * n;
    // zero, with identity on the separator padding
    for (int e = tid; e < n * n; e += blockDim.x) {
      const int col = e / n, row = e - col * n;
      Wk[e] = make_double2(row == col && row >= s && row < sp ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    // entries of the local matrix in rows of separator nodes (their columns
    // in the separator or the ring; neighbours below were assembled there)
    {
      const BoxTabs t = box_tabs(ltab, bd);
      const int32_t* nodes = nd.nodes + F.node_off;
      const int32_t* ap = nd.asmp + F.asm_off;
      for (int k = tid; k < s; k += blockDim.x) {
        const int g = nodes[k], j = g / bd.mx, a = g - j * bd.mx;
        const double kk = k2[(int64_t)(bd.by0 + j) * ngx + bd.bx0 + a];
        Wk[(int64_t)k * n + k] = line_block_entry(t, a, a, j, kk);
        // couplings to the W, E, S, N neighbours
        const double2 cpl[4] = {dmul(t.ay[j], t.ihx[a]), dmul(t.ay[j], t.ihx[a + 1]),
                                dmul(t.ax[a], t.ihy[j]), dmul(t.ax[a], t.ihy[j + 1])};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int p = ap[4 * k + q];
          if (p < 0) continue;
          Wk[(int64_t)p * n + k] = cpl[q];
          if (p >= sp) Wk[(int64_t)k * n + p] = cpl[q];
        }
      }
    }
    __syncthreads();
    // extend-add of the children's update matrices, one child at a time
    for (int q = 0; q < 2; ++q) {
      const int c = q ? F.c1 : F.c0;
      if (c < 0) continue;
      const NDFront& C = nd.fr[c];
      const int cb = C.b;
      const int32_t* cm = nd.cmap + (q ? F.cmap1 : F.cmap0);
      const double2* Uc = U + ((int64_t)((d + 1) & 1) * nboxes + box) * nd.ustride + C.u_off;
      for (int e = tid; e < cb * cb; e += blockDim.x) {
        const int qq = e / cb, pp = e - qq * cb;
        double2& dst = Wk[(int64_t)cm[qq] * n + cm[pp]];
        const double2 u = Uc[e];
        dst = make_double2(dst.x + u.x, dst.y + u.y);
      }
      __syncthreads();
    }
    float pmin = 0.f, pmax = 0.f;  // pivot magnitudes: not reported for the fronts
    gj_sweep(Wk, n, sp, Dl, Cp, Rr, Rp, n, static_cast<const float*>(nullptr), pmin, pmax);
    // G, L, L^T to the factor; the update matrix to this depth's region
    double2* Gf = G + bd.g_off + F.g_off;
    for (int e = tid; e < s * s; e += blockDim.x) {
      const int col = e / s, row = e - col * s;
      Gf[e] = Wk[(int64_t)col * n + row];
    }
    double2* Lf = Gf + (int64_t)s * s;
    for (int e = tid; e < b * s; e += blockDim.x) {
      const int k = e / b, i = e - k * b;
      Lf[e] = Wk[(int64_t)k * n + sp + i];
    }
    double2* LT = Lf + (int64_t)b * s;
    for (int e = tid; e < s * b; e += blockDim.x) {
      const int i = e / s, k = e - i * s;
      LT[e] = Wk[(int64_t)k * n + sp + i];
    }
    double2* Uo = U + ((int64_t)(d & 1) * nboxes + box) * nd.ustride + F.u_off;
    for (int e = tid; e < b * b; e += blockDim.x) {
      const int qq = e / b, pp = e - qq * b;
      Uo[e] = Wk[(int64_t)(sp + qq) * n + sp + pp];
    }
    __syncthreads();
  }
}

// Right-hand sides per thread in the solve: four threads share a row (one
// quarter of the 16 columns each), so a level's rows fill the workgroup.
constexpr int RPT = 4;
constexpr int QPR = NB / RPT;  // threads per row

// acc[r] += m * w[r] for this thread's RPT right-hand sides (complex, FP64
// accumulation of the complex64 vector entries in LDS)
__device__ __forceinline__ void row_mac(double2 m, const float2* __restrict__ w, double* ar,
                                        double* ai) {
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const float2 x = w[r];
    ar[r] = fma(m.x, (double)x.x, fma(-m.y, (double)x.y, ar[r]));
    ai[r] = fma(m.x, (double)x.y, fma(m.y, (double)x.x, ai[r]));
  }
}

// ----------------------------------------------------------------- forward
// One workgroup per (front, box): w = [f_s; 0] plus the children's update
// vectors, in LDS as (s + b) x 16; w_s is stored to the box solution (the
// backward sweep reads it back), and w_b + L w_s (four threads per ring row,
// consecutive rows on consecutive thread quads, so a column of L is read
// contiguously) becomes this front's update vector.
__global__ __launch_bounds__(256) void nd_forward_kernel(NDDev nd, int d, int nboxes,
                                                         const BoxDesc* __restrict__ desc,
                                                         const double2* __restrict__ G,
                                                         const float2* __restrict__ S, int tr,
                                                         int xw, float2* __restrict__ X,
                                                         float2* __restrict__ V) {
  extern __shared__ float2 w[];
  const int box = blockIdx.y, fi = blockIdx.x;
  const int cls = nd.bcls[box];
  if (fi >= nd.dcnt[cls * nd.depths + d]) return;
  const NDFront F = nd_front(nd, cls, d, fi);
  const BoxDesc bd = desc[box];
  const int s = F.s, b = F.b, sp = F.sp;
  const int tid = threadIdx.x;
  const int32_t* nodes = nd.nodes + F.node_off;
  // sources of the separator nodes (zero outside the tile); ring rows zero
  const float2* Sb = S + (int64_t)box * NB * tr * xw;
  for (int e = tid; e < (s + b) * NB; e += blockDim.x) {
    const int k = e >> 4, r = e & 15;
    float2 v = make_float2(0.f, 0.f);
    if (k < s) {
      const int g = nodes[k], j = g / bd.mx, a = g - j * bd.mx;
      if (j >= bd.ty0 && j < bd.ty1 && a >= bd.tx0 && a < bd.tx1)
        v = Sb[((int64_t)r * tr + (j - bd.ty0)) * xw + a];
    }
    w[e] = v;
  }
  __syncthreads();
  for (int q = 0; q < 2; ++q) {
    const int c = q ? F.c1 : F.c0;
    if (c < 0) continue;
    const NDFront& C = nd.fr[c];
    const int32_t* cm = nd.cmap + (q ? F.cmap1 : F.cmap0);
    const float2* Vc = V + ((int64_t)((d + 1) & 1) * nboxes + box) * nd.vstride + C.v_off;
    for (int e = tid; e < C.b * NB; e += blockDim.x) {
      const int p = e >> 4, r = e & 15;
      const int pos = cm[p];
      const int row = pos < sp ? pos : pos - sp + s;
      const float2 u = Vc[e];
      w[row * NB + r] = make_float2(w[row * NB + r].x + u.x, w[row * NB + r].y + u.y);
    }
    __syncthreads();
  }
  float2* Xb = X + bd.xb_off;
  for (int e = tid; e < s * NB; e += blockDim.x) Xb[(int64_t)nodes[e >> 4] * NB + (e & 15)] = w[e];
  const double2* L = G + bd.g_off + F.g_off + (int64_t)s * s;
  float2* Vo = V + ((int64_t)(d & 1) * nboxes + box) * nd.vstride + F.v_off;
  for (int e = tid; e < b * QPR; e += blockDim.x) {
    const int i = e / QPR, r0 = (e - i * QPR) * RPT;
    double ar[RPT], ai[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) ar[r] = ai[r] = 0.0;
    for (int k = 0; k < s; ++k) row_mac(L[(int64_t)k * b + i], w + k * NB + r0, ar, ai);
    const float2* wb = w + (s + i) * NB + r0;
#pragma unroll
    for (int r = 0; r < RPT; ++r)
      Vo[i * NB + r0 + r] = make_float2((float)(ar[r] + wb[r].x), (float)(ai[r] + wb[r].y));
  }
}

// ---------------------------------------------------------------- backward
// One workgroup per (front, box): x_s = G w_s + L^T x_b with w_s (stored by
// the forward sweep) and x_b (final: ring nodes lie on ancestor separators)
// staged in LDS, four threads per separator row.
__global__ __launch_bounds__(256) void nd_backward_kernel(NDDev nd, int d,
                                                          const BoxDesc* __restrict__ desc,
                                                          const double2* __restrict__ G,
                                                          float2* __restrict__ X) {
  extern __shared__ float2 w[];
  const int box = blockIdx.y, fi = blockIdx.x;
  const int cls = nd.bcls[box];
  if (fi >= nd.dcnt[cls * nd.depths + d]) return;
  const NDFront F = nd_front(nd, cls, d, fi);
  const BoxDesc bd = desc[box];
  const int s = F.s, b = F.b;
  const int tid = threadIdx.x;
  const int32_t* nodes = nd.nodes + F.node_off;
  float2* Xb = X + bd.xb_off;
  for (int e = tid; e < (s + b) * NB; e += blockDim.x)
    w[e] = Xb[(int64_t)nodes[e >> 4] * NB + (e & 15)];
  __syncthreads();
  const double2* Gm = G + bd.g_off + F.g_off;
  const double2* LT = Gm + (int64_t)s * s + (int64_t)b * s;
  for (int e = tid; e < s * QPR; e += blockDim.x) {
    const int i = e / QPR, r0 = (e - i * QPR) * RPT;
    double ar[RPT], ai[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) ar[r] = ai[r] = 0.0;
    for (int k = 0; k < s; ++k) row_mac(Gm[(int64_t)k * s + i], w + k * NB + r0, ar, ai);
    for (int p = 0; p < b; ++p) row_mac(LT[(int64_t)p * s + i], w + (s + p) * NB + r0, ar, ai);
    float2* xo = Xb + (int64_t)nodes[i] * NB + r0;
#pragma unroll
    for (int r = 0; r < RPT; ++r) xo[r] = make_float2((float)ar[r], (float)ai[r]);
  }
}

// Threads of a solve workgroup: a level whose fronts have at most 16 (32)
// nodes gets one (two) waves, and more fronts run at once.
int nd_threads(int maxw) { return maxw <= 16 ? 64 : maxw <= 32 ? 128 : 256; }

}  // namespace

hipError_t launch_nd_factor(const NDDev& nd, int d, int maxcnt, int nboxes, int maxn,
                            const BoxDesc* desc, const double2* ltab, const double* k2, int ngx,
                            double2* G, double2* W, int64_t wstride, int nslots, double2* U,
                            hipStream_t s) {
  if (maxcnt <= 0) return hipSuccess;
  if (maxn <= 0 || maxn > ND_MAX_N || maxn % 16 ||
      wstride < (int64_t)maxn * maxn + 3 * 16 * (int64_t)maxn)
    return hipErrorInvalidValue;
  const int64_t items = (int64_t)nboxes * maxcnt;
  const int grid = (int)std::min<int64_t>(items, nslots);
  hipLaunchKernelGGL(nd_factor_kernel, dim3(grid), dim3(256), 0, s, nd, d, maxcnt, nboxes, desc,
                     ltab, k2, ngx, G, W, wstride, U);
  return hipGetLastError();
}

hipError_t describe_nd_forward(KLaunch& k, const NDDev& nd, int d, int maxcnt, int nboxes,
                               int maxw, const BoxDesc* desc, const double2* G, const float2* S,
                               int tr, int xw, float2* X, float2* V) {
  if (maxcnt <= 0 || maxw <= 0 || maxw > ND_MAX_W) return hipErrorInvalidValue;
  k = KLaunch{};
  k.func = reinterpret_cast<const void*>(&nd_forward_kernel);
  k.grid = dim3(maxcnt, nboxes);
  k.block = dim3(nd_threads(maxw));
  k.shmem = (unsigned)(maxw * NB * sizeof(float2));
  k.push(nd);
  k.push(d);
  k.push(nboxes);
  k.push(desc);
  k.push(G);
  k.push(S);
  k.push(tr);
  k.push(xw);
  k.push(X);
  k.push(V);
  return hipSuccess;
}

hipError_t describe_nd_backward(KLaunch& k, const NDDev& nd, int d, int maxcnt, int nboxes,
                                int maxw, const BoxDesc* desc, const double2* G, float2* X) {
  if (maxcnt <= 0 || maxw <= 0 || maxw > ND_MAX_W) return hipErrorInvalidValue;
  k = KLaunch{};
  k.func = reinterpret_cast<const void*>(&nd_backward_kernel);
  k.grid = dim3(maxcnt, nboxes);
  k.block = dim3(nd_threads(maxw));
  k.shmem = (unsigned)(maxw * NB * sizeof(float2));
  k.push(nd);
  k.push(d);
  k.push(desc);
  k.push(G);
  k.push(X);
  return hipSuccess;
}

}  // namespace hddm
