// Device helpers shared by the gfx950 kernel files: complex arithmetic on
// float2/double2, the per-box stretch tables and the entries of the local
// 5-point matrix (Leng & Ju, Sec. 2 eq. pmlij), and the 16x16 complex MFMA
// tile primitives of the blocked Gauss-Jordan factorisations.
#pragma once
#include <hip/hip_runtime.h>

#include "hddm_internal.h"

namespace hddm {
namespace {

// ---------------------------------------------------------------- complex
template <typename C> struct RealOf;
template <> struct RealOf<float2> { using T = float; };
template <> struct RealOf<double2> { using T = double; };

template <typename C>
__device__ __forceinline__ C mk(double re, double im) {
  C c;
  c.x = static_cast<typename RealOf<C>::T>(re);
  c.y = static_cast<typename RealOf<C>::T>(im);
  return c;
}
template <typename C>
__device__ __forceinline__ C czero() {
  C c;
  c.x = 0;
  c.y = 0;
  return c;
}
template <typename C>
__device__ __forceinline__ C cadd(C a, C b) {
  C c;
  c.x = a.x + b.x;
  c.y = a.y + b.y;
  return c;
}
template <typename C>
__device__ __forceinline__ C csub(C a, C b) {
  C c;
  c.x = a.x - b.x;
  c.y = a.y - b.y;
  return c;
}
template <typename C>
__device__ __forceinline__ C cmul(C a, C b) {
  C c;
  c.x = a.x * b.x - a.y * b.y;
  c.y = a.x * b.y + a.y * b.x;
  return c;
}
// acc + a*b
template <typename C>
__device__ __forceinline__ C cfma(C a, C b, C acc) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
  return acc;
}
template <typename C>
__device__ __forceinline__ C cdiv(C a, C b) {
  typename RealOf<C>::T d = b.x * b.x + b.y * b.y;
  C c;
  c.x = (a.x * b.x + a.y * b.y) / d;
  c.y = (a.y * b.x - a.x * b.y) / d;
  return c;
}
template <typename C>
__device__ __forceinline__ C cneg(C a) {
  a.x = -a.x;
  a.y = -a.y;
  return a;
}
template <typename C>
__device__ __forceinline__ C from_d(double2 v) {
  return mk<C>(v.x, v.y);
}
__device__ __forceinline__ double2 to_d(float2 v) { return make_double2(v.x, v.y); }
__device__ __forceinline__ double2 to_d(double2 v) { return v; }

template <typename C>
__device__ __forceinline__ C shfl_c(C v, int lane) {
  C r;
  r.x = __shfl(v.x, lane, 64);
  r.y = __shfl(v.y, lane, 64);
  return r;
}

// Box stretch tables: ax[mx], ihx[mx+1], ay[my], ihy[my+1] (complex FP64).
struct BoxTabs {
  const double2 *ax, *ihx, *ay, *ihy;
};
__device__ __forceinline__ BoxTabs box_tabs(const double2* ltab, const BoxDesc& bd) {
  BoxTabs t;
  t.ax = ltab + bd.tab_off;
  t.ihx = t.ax + bd.mx;
  t.ay = t.ihx + bd.mx + 1;
  t.ihy = t.ay + bd.my;
  return t;
}

__device__ __forceinline__ double2 dmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Entry (a, b) of the tridiagonal x-line block T_j of a box:
// diagonal -(cW + cE + cS + cN) + k^2 ax ay, off-diagonal cE(a) = ay ihx[a+1].
__device__ __forceinline__ double2 line_block_entry(const BoxTabs& t, int a, int b, int j,
                                                    double kk) {
  if (a == b) {
    const double2 axa = t.ax[a], ayj = t.ay[j];
    const double2 cw = dmul(ayj, t.ihx[a]), ce = dmul(ayj, t.ihx[a + 1]);
    const double2 cs = dmul(axa, t.ihy[j]), cn = dmul(axa, t.ihy[j + 1]);
    const double2 jac = dmul(axa, ayj);
    return make_double2(-(cw.x + ce.x + cs.x + cn.x) + kk * jac.x,
                        -(cw.y + ce.y + cs.y + cn.y) + kk * jac.y);
  }
  if (a == b + 1 || b == a + 1) return dmul(t.ay[j], t.ihx[max(a, b)]);
  return make_double2(0.0, 0.0);
}

// ------------------------------------------------- blocked Gauss-Jordan
constexpr int FB = 16;  // Gauss-Jordan block width

// Invert the kb x kb diagonal block D (rows/cols k0.. of the row panel Rr,
// D[q][p] = Rr[q*ld + k0 + p]) into Dl (row-major, stride FB) with one wave.
// Lane c holds column c; pivots travel by cross-lane shuffles.  Padded
// columns/rows (kb < FB) are identity and drop out of the top-left block.
// pmin / pmax: running smallest and largest relative pivot |p_k| / sd[k]
// (|p_k| if sd is null) over the kb real pivots, the same in every lane.
template <typename C>
__device__ void invert_block_wave(const C* Rr, int ld, int k0, int kb, C* Dl, const float* sd,
                                  float& pmin, float& pmax) {
  const int c = threadIdx.x & 63;
  C col[FB];
#pragma unroll
  for (int r = 0; r < FB; ++r) {
    if (c < kb && r < kb)
      col[r] = Rr[r * ld + k0 + c];
    else
      col[r] = (r == c) ? mk<C>(1.0, 0.0) : czero<C>();
  }
#pragma unroll
  for (int p = 0; p < FB; ++p) {
    C piv = shfl_c(col[p], p);
    if (p < kb) {
      float mag = (float)sqrt((double)piv.x * piv.x + (double)piv.y * piv.y);
      if (sd) mag /= sd[k0 + p];
      pmin = fminf(pmin, mag);
      pmax = fmaxf(pmax, mag);
    }
    C ip = cdiv(mk<C>(1.0, 0.0), piv);
    C colp[FB];
#pragma unroll
    for (int r = 0; r < FB; ++r) colp[r] = shfl_c(col[r], p);
    if (c == p) {
#pragma unroll
      for (int r = 0; r < FB; ++r) col[r] = (r == p) ? ip : cneg(cmul(colp[r], ip));
    } else {
      C rowp = cmul(col[p], ip);  // new D[p][c]
#pragma unroll
      for (int r = 0; r < FB; ++r) col[r] = (r == p) ? rowp : csub(col[r], cmul(colp[r], rowp));
    }
  }
  if (c < FB) {
#pragma unroll
    for (int r = 0; r < FB; ++r) Dl[r * FB + c] = col[r];
  }
}

// Blocked Gauss-Jordan on the n x n column-major matrix S (entry (i, j) at
// j*n+i) over its first npiv pivots: per 16-wide block K with D = S[K,K],
// S[K,K] <- D^-1, S[K,J] <- D^-1 S[K,J], S[I,K] <- -S[I,K] D^-1,
// S[I,J] <- S[I,J] - S[I,K] D^-1 S[K,J].  With npiv = n this is the in-place
// inverse; with npiv < n it leaves [[A^-1, A^-1 B], [-C A^-1, D - C A^-1 B]]
// for S = [[A, B], [C, D]].  Whole workgroup; panels Cp, Rr, Rp (16 x ld) and
// Dl (16 x 16) in LDS or memory.  pmin / pmax (meaningful in the first wave):
// running smallest and largest pivot magnitude, relative to sd[k] (the
// magnitude of the matrix's own diagonal entry) when sd is given.
template <typename C>
__device__ void gj_sweep(C* __restrict__ S, int n, int npiv, C* Dl, C* Cp, C* Rr, C* Rp, int ld,
                         const float* sd, float& pmin, float& pmax) {
  const int nt = (npiv + FB - 1) / FB;
  const int tid = threadIdx.x, nth = blockDim.x;
  for (int K = 0; K < nt; ++K) {
    const int k0 = K * FB, kb = min(FB, npiv - k0);
    for (int e = tid; e < kb * n; e += nth) {  // column panel, Cp[q][i] = S[i][k0+q]
      const int q = e / n, i = e - q * n;
      Cp[q * ld + i] = S[(int64_t)(k0 + q) * n + i];
    }
    for (int e = tid; e < kb * n; e += nth) {  // row panel, Rr[q][j] = S[k0+q][j]
      const int j = e / kb, q = e - j * kb;
      Rr[q * ld + j] = S[(int64_t)j * n + k0 + q];
    }
    __syncthreads();
    if (tid < 64) invert_block_wave(Rr, ld, k0, kb, Dl, sd, pmin, pmax);
    __syncthreads();
    for (int e = tid; e < kb * n; e += nth) {  // Rp = D^-1 Rr
      const int q = e / n, j = e - q * n;
      C acc = czero<C>();
      for (int p = 0; p < kb; ++p) acc = cfma(Dl[q * FB + p], Rr[p * ld + j], acc);
      Rp[q * ld + j] = acc;
    }
    __syncthreads();
    for (int e = tid; e < n * n; e += nth) {
      const int j = e / n, i = e - j * n;
      const bool ik = (i >= k0) && (i < k0 + kb);
      const bool jk = (j >= k0) && (j < k0 + kb);
      C val;
      if (ik && jk) {
        val = Dl[(i - k0) * FB + (j - k0)];
      } else if (ik) {
        val = Rp[(i - k0) * ld + j];
      } else if (jk) {
        C acc = czero<C>();
        for (int p = 0; p < kb; ++p) acc = cfma(Cp[p * ld + i], Dl[p * FB + (j - k0)], acc);
        val = cneg(acc);
      } else {
        C acc = S[e];
        for (int p = 0; p < kb; ++p) acc = cfma(cneg(Cp[p * ld + i]), Rp[p * ld + j], acc);
        val = acc;
      }
      S[e] = val;
    }
    __syncthreads();
  }
}

// In-place inverse of the n x n column-major matrix S.
template <typename C>
__device__ void gj_invert(C* __restrict__ S, int n, C* Dl, C* Cp, C* Rr, C* Rp, int ld,
                          const float* sd, float& pmin, float& pmax) {
  gj_sweep(S, n, n, Dl, Cp, Rr, Rp, ld, sd, pmin, pmax);
}

// ----------------------------------------------------- 16x16 MFMA tiles
// Tile layout in a wave: lane l, register v holds entry
// (16I + 4(l>>4) + v, 16J + (l & 15)) -- the MFMA output layout (A operand:
// lane l gives A[l&15][l>>4]; B operand: lane l gives B[l>>4][l&15]).
typedef float mf4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ mf4 mfma4(float a, float b, mf4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// (cre, cim) += (A_re + i A_im)(B_re + i B_im) over one 16x16x16 block; the
// operands are read from LDS arrays laid out [k][16] (16 floats per k).
__device__ __forceinline__ void cmfma16(const float* Ar, const float* Ai, const float* Br,
                                        const float* Bi, int lane, mf4& cre, mf4& cim) {
#pragma unroll
  for (int kc = 0; kc < 4; ++kc) {
    const int o = (kc * 4 + (lane >> 4)) * 16 + (lane & 15);
    const float ar = Ar[o], ai = Ai[o], br = Br[o], bi = Bi[o];
    cre = mfma4(ar, br, cre);
    cre = mfma4(-ai, bi, cre);
    cim = mfma4(ar, bi, cim);
    cim = mfma4(ai, br, cim);
  }
}

// Tile (I, J) of the column-major mx x mx matrix S to/from accumulators.
__device__ __forceinline__ void tile_load(const float2* S, int mx, int I, int J, int lane, mf4& re,
                                          mf4& im) {
  const int b = 16 * J + (lane & 15), a = 16 * I + 4 * (lane >> 4);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    float2 x;
    if (a + v < mx && b < mx)
      x = S[(int64_t)b * mx + a + v];
    else
      x = make_float2(a + v == b ? 1.f : 0.f, 0.f);
    re[v] = x.x;
    im[v] = x.y;
  }
}
__device__ __forceinline__ void tile_store(float2* S, int mx, int I, int J, int lane, const mf4& re,
                                           const mf4& im) {
  const int b = 16 * J + (lane & 15), a = 16 * I + 4 * (lane >> 4);
  if (b >= mx) return;
#pragma unroll
  for (int v = 0; v < 4; ++v)
    if (a + v < mx) S[(int64_t)b * mx + a + v] = make_float2(re[v], im[v]);
}

// D^-1 for the 16x16 diagonal block D[r][c] = (Dre + i Dim)[r*16 + c], by
// Gauss-Jordan with one wave: lane l holds rows 4(l>>4) .. 4(l>>4)+3 of
// column l & 15; the pivot comes by a lane read, the pivot row and column
// entries each lane needs by lane permutes.  Result into DR (row-major
// [r][c]) and DT (transposed [c][r]).  pmin / pmax: running smallest and
// largest of |p| / sd[k] over the first nvalid pivots (the rest are padding),
// sd[k] the magnitude of the diagonal entry the k-th pivot started from.
__device__ __forceinline__ void invert_d16(const float* Dre, const float* Dim, int lane,
                                           float* DRre, float* DRim, float* DTre, float* DTim,
                                           int nvalid, const float* sd, float& pmin,
                                           float& pmax) {
  const int c = lane & 15, q = lane >> 4;
  float2 d[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) d[v] = make_float2(Dre[(4 * q + v) * 16 + c], Dim[(4 * q + v) * 16 + c]);
  auto bcast = [](float2 x, int src) {  // src is a constant once unrolled
    return make_float2(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(x.x), src)),
                       __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x.y), src)));
  };
#pragma unroll
  for (int pv = 0; pv < 16; ++pv) {
    const int qp = pv >> 2, vp = pv & 3;
    const float2 piv = bcast(d[vp], 16 * qp + pv);
    if (pv < nvalid) {
      const float rp = sqrtf(piv.x * piv.x + piv.y * piv.y) / sd[pv];
      pmin = fminf(pmin, rp);
      pmax = fmaxf(pmax, rp);
    }
    const float2 ip = cdiv(make_float2(1.f, 0.f), piv);
    const float2 rowp = cmul(shfl_c(d[vp], 16 * qp + c), ip);  // new D[pv][c] (c != pv)
    float2 cp[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) cp[v] = shfl_c(d[v], 16 * q + pv);  // old D[4q+v][pv]
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 4 * q + v;
      if (c == pv)
        d[v] = (r == pv) ? ip : cneg(cmul(cp[v], ip));
      else
        d[v] = (r == pv) ? rowp : csub(d[v], cmul(cp[v], rowp));
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = 4 * q + v;
    DRre[r * 16 + c] = d[v].x;
    DRim[r * 16 + c] = d[v].y;
    DTre[c * 16 + r] = d[v].x;
    DTim[c * 16 + r] = d[v].y;
  }
}

}  // namespace
}  // namespace hddm
