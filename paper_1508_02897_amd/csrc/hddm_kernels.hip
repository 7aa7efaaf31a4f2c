// gfx950 kernels of the one-step overlapping DDM preconditioner (Leng & Ju,
// Sec. 2 eq. ddm0 / eq. pc) and of the FGMRES loop around it (Sec. 3).
//
//  * factor_gj:  per box, block Schur recursion over x-lines
//                S_0 = T_0, S_j = T_j - B_{j-1} G_{j-1} B_{j-1}, G_j = S_j^-1,
//                each inverse by in-place blocked Gauss-Jordan (16-wide blocks,
//                no pivoting: the layer-damped Schur complements are well
//                conditioned and diagonally dominated), vector FMA, any
//                precision.  G_j is stored column-major: entry (a, b) at b*mx + a.
//  * sweep:      restriction of r to the tile, forward sweep
//                y_j = G_j (b_j - B_{j-1} y_{j-1}) and backward sweep
//                x_j = y_j - G_j (B_j x_{j+1}), one workgroup per box; each
//                step is a dense complex GEMV streamed from HBM.
//  * gather:     z(g) = sum of the (at most four) box solutions covering g,
//                layers included, in a fixed order (no atomics).
//  * matvec:     the global 5-point PML operator in FP64.
//  * krylov:     multi-dot, multi-axpy, norms, scaling for CGS2 Arnoldi.
#include <hip/hip_runtime.h>

#include "hddm_internal.h"
#include "hddm_device.h"

namespace hddm {
namespace {

// ------------------------------------------- symmetric-packed tile format
// G_j is complex symmetric (the local matrix is, and so are its Schur
// complements and their inverses).  The packed format keeps the 16x16 tiles on
// and above the diagonal, column-block by column-block: tile (I, J), I <= J,
// is number J(J+1)/2 + I, and holds entry (16I + r, 16J + c) at r*16 + c
// (row-major inside the tile, complex64); a diagonal tile holds its upper
// triangle only, row by row (diag_pos in hddm_internal.h).  Entries past mx
// are zero.
__device__ __forceinline__ int packed_tiles(int nt) { return nt * (nt + 1) / 2; }

// Packed upper tiles of the full column-major mx x mx matrix S into out
// (whole workgroup).  Entry (16I + r, 16J + c) is read as S(16J + c, 16I + r)
// -- the same value by symmetry -- so both sides are read and written
// contiguously.
__device__ void store_packed(const float2* __restrict__ S, int mx, float2* __restrict__ out) {
  const int nt = (mx + 15) >> 4, tot = packed_tiles(nt) * 256;
  for (int e = threadIdx.x; e < tot; e += blockDim.x) {
    const int t = e >> 8, rc = e & 255, r = rc >> 4, c = rc & 15;
    int J = 0;
    while ((J + 1) * (J + 2) / 2 <= t) ++J;
    const int I = t - J * (J + 1) / 2;
    const int a = 16 * J + c, b = 16 * I + r;  // column-major entry (a, b) of S
    // a diagonal tile keeps its upper triangle only (diag_pos), zeros after it
    const bool keep = a < mx && b < mx && (I != J || r <= c);
    out[(int64_t)t * 256 + (I == J ? diag_pos(r, c) : rc)] =
        keep ? S[(int64_t)b * mx + a] : make_float2(0.f, 0.f);
  }
}

// ---------------------------------------------------------------- factor
template <typename C>
__global__ __launch_bounds__(512) void factor_gj_kernel(const BoxDesc* __restrict__ desc,
                                                        const double2* __restrict__ ltab,
                                                        const double* __restrict__ k2, int ngx,
                                                        C* __restrict__ G, int nboxes, int ld,
                                                        C* __restrict__ ws, int64_t ws_stride,
                                                        int packed, float2* __restrict__ pivstat) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* Dl = reinterpret_cast<C*>(smem_raw);
  C* Cp = Dl + FB * FB;
  C* Rr = Cp + FB * ld;
  C* Rp = Rr + FB * ld;
  __shared__ float Sd[FB * 26];  // |S_j(a, a)| (boxes up to 416 wide)
  for (int box = blockIdx.x; box < nboxes; box += gridDim.x) {
    const BoxDesc bd = desc[box];
    const int mx = bd.mx, my = bd.my;
    const BoxTabs t = box_tabs(ltab, bd);
    C* Gb = G + bd.g_off;
    const int n2 = mx * mx;
    C* Wk = ws + (int64_t)blockIdx.x * ws_stride;
    float pmin = __builtin_inff(), pmax = 0.f;  // pivot magnitudes of this box (first wave)
    for (int j = 0; j < my; ++j) {
      C* S = packed ? Wk : Gb + (int64_t)j * n2;
      const C* Gprev = packed ? Wk : S - n2;  // G_{j-1}, read before overwrite
      const double* krow = k2 + (int64_t)(bd.by0 + j) * ngx + bd.bx0;
      const double2 ihyj = t.ihy[j];
      for (int e = threadIdx.x; e < n2; e += blockDim.x) {
        const int b = e / mx, a = e - b * mx;
        const double kk = (a == b) ? krow[a] : 0.0;
        C val = from_d<C>(line_block_entry(t, a, b, j, kk));
        if (j > 0) {  // - B_{j-1}[a] G_{j-1}(a, b) B_{j-1}[b], B_{j-1}[i] = ax[i] ihy[j]
          const C ba = from_d<C>(dmul(t.ax[a], ihyj));
          const C bb = from_d<C>(dmul(t.ax[b], ihyj));
          val = csub(val, cmul(cmul(ba, Gprev[e]), bb));
        }
        S[e] = val;
        if (a == b) Sd[a] = (float)sqrt((double)val.x * val.x + (double)val.y * val.y);
      }
      __syncthreads();
      gj_invert(S, mx, Dl, Cp, Rr, Rp, ld, Sd, pmin, pmax);
      if constexpr (sizeof(C) == sizeof(float2)) {
        if (packed) {
          store_packed(reinterpret_cast<const float2*>(S), mx,
                       reinterpret_cast<float2*>(Gb) + (int64_t)j * packed_tiles((mx + 15) >> 4) * 256);
          __syncthreads();
        }
      }
    }
    if (pivstat && threadIdx.x == 0) pivstat[box] = make_float2(pmin, pmax);
  }
}

// ------------------------------------------------ complex64 factor, MFMA
// One workgroup (MF_WAVES waves) per box.  The working matrix of x-line j is
// built in G_j's own slot of the factor buffer (column-major, entry (a, b) at
// b*mx + a), where it stays cache-resident while it is inverted in place by
// blocked Gauss-Jordan with 16-wide blocks:
//   * the diagonal block D and the row/column panels of block K are staged in
//     LDS in MFMA operand order; wave 0 inverts D (shuffles, FP32);
//   * the row panel becomes D^-1 S[K,J], the column panel -S[I,K] D^-1, and
//     every other 16x16 tile the rank-16 update S[I,J] - S[I,K] D^-1 S[K,J],
//     each tile loaded into MFMA accumulators by one wave, updated with
//     v_mfma_f32_16x16x4f32 (complex products as four real MFMAs:
//     re*re - im*im, re*im + im*re) and stored back.
// Tile layout in a wave: lane l, register v holds entry
// (16I + 4(l>>4) + v, 16J + (l & 15)) -- the MFMA output layout (A operand:
// lane l gives A[l&15][l>>4]; B operand: lane l gives B[l>>4][l&15]).
// Entries past mx (ragged last block) act as identity and are never stored.
constexpr int MF_NT = 16;     // tiles per side (boxes up to 256 wide)
constexpr int MF_WAVES = 8;

// packed != 0: the working matrix lives in this workgroup's slot of `ws`
// (ws_stride entries) and each G_j is written in the symmetric-packed format;
// otherwise it is built in G_j's own (dense) slot.
__global__ __launch_bounds__(64 * MF_WAVES) void factor_mfma_kernel(
    const BoxDesc* __restrict__ desc, const double2* __restrict__ ltab,
    const double* __restrict__ k2, int ngx, float2* __restrict__ G, int nboxes,
    float2* __restrict__ ws, int64_t ws_stride, int packed, float2* __restrict__ pivstat) {
  __shared__ float Cre[MF_NT * 256], Cim[MF_NT * 256];  // -S[I,K] as [k][i] per I
  __shared__ float Rre[MF_NT * 256], Rim[MF_NT * 256];  // S[K,J] then D^-1 S[K,J], [k][j]
  __shared__ float DRre[256], DRim[256];                // D^-1 row-major [k][j]
  __shared__ float DTre[256], DTim[256];                // D^-1 transposed [k][i]
  __shared__ float Sd[MF_NT * 16];                      // |S_j(a, a)|
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int box = blockIdx.x; box < nboxes; box += gridDim.x) {
    const BoxDesc bd = desc[box];
    const int mx = bd.mx, my = bd.my;
    const int nt = (mx + 15) >> 4;
    const BoxTabs t = box_tabs(ltab, bd);
    float2* Gb = G + bd.g_off;
    const int n2 = mx * mx;
    const int64_t pk = (int64_t)packed_tiles(nt) * 256;  // entries of one packed G_j
    float2* Wk = ws + (int64_t)blockIdx.x * ws_stride;
    float pmin = __builtin_inff(), pmax = 0.f;  // pivot magnitudes of this box (wave 0)
    for (int j = 0; j < my; ++j) {
      float2* S = packed ? Wk : Gb + (int64_t)j * n2;
      const float2* Gprev = packed ? Wk : S - n2;  // G_{j-1}, read before overwrite
      // S_j = T_j - B_{j-1} G_{j-1} B_{j-1}
      {
        const double* krow = k2 + (int64_t)(bd.by0 + j) * ngx + bd.bx0;
        const double2 ihyj = t.ihy[j];
        for (int e = tid; e < n2; e += blockDim.x) {
          const int bcol = e / mx, arow = e - bcol * mx;
          const double kk = (arow == bcol) ? krow[arow] : 0.0;
          float2 val = from_d<float2>(line_block_entry(t, arow, bcol, j, kk));
          if (j > 0) {
            const float2 ba = from_d<float2>(dmul(t.ax[arow], ihyj));
            const float2 bb = from_d<float2>(dmul(t.ax[bcol], ihyj));
            val = csub(val, cmul(cmul(ba, Gprev[e]), bb));
          }
          S[e] = val;
          if (arow == bcol) Sd[arow] = sqrtf(val.x * val.x + val.y * val.y);
        }
      }
      __syncthreads();
      for (int K = 0; K < nt; ++K) {
        // stage the panels of block K (identity past mx): column panel
        // negated as [k][i], row panel as [k][j]
        for (int e = tid; e < nt * 256; e += blockDim.x) {
          const int blk = e >> 8, k = (e >> 4) & 15, i = e & 15;
          const int a = 16 * blk + i, c = 16 * K + k;
          float2 x = (a < mx && c < mx) ? S[(int64_t)c * mx + a] : make_float2(a == c ? 1.f : 0.f, 0.f);
          Cre[e] = -x.x;
          Cim[e] = -x.y;
          // row panel entry (16K + k, 16 blk + i)
          const int rr = 16 * K + k, cc = 16 * blk + i;
          x = (rr < mx && cc < mx) ? S[(int64_t)cc * mx + rr] : make_float2(rr == cc ? 1.f : 0.f, 0.f);
          Rre[e] = x.x;
          Rim[e] = x.y;
        }
        __syncthreads();
        if (wave == 0)
          invert_d16(Rre + K * 256, Rim + K * 256, lane, DRre, DRim, DTre, DTim, mx - 16 * K,
                     Sd + 16 * K, pmin, pmax);
        __syncthreads();
        // row panel: D^-1 S[K,J] (to LDS and to S)
        for (int J = wave; J < nt; J += MF_WAVES) {
          if (J == K) continue;
          mf4 cr = mf4{0.f, 0.f, 0.f, 0.f}, ci = mf4{0.f, 0.f, 0.f, 0.f};
          cmfma16(DTre, DTim, Rre + J * 256, Rim + J * 256, lane, cr, ci);
          const int lr = 4 * (lane >> 4), lc = lane & 15;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            Rre[J * 256 + (lr + v) * 16 + lc] = cr[v];
            Rim[J * 256 + (lr + v) * 16 + lc] = ci[v];
          }
          tile_store(S, mx, K, J, lane, cr, ci);
        }
        __syncthreads();
        // pivot block, column panel, rank-16 update of every other tile
        for (int tt = wave; tt < nt * nt; tt += MF_WAVES) {
          const int I = tt / nt, J = tt - (tt / nt) * nt;
          if (I == K && J != K) continue;
          mf4 cr, ci;
          if (I == K) {  // J == K
            const int lr = 4 * (lane >> 4), lc = lane & 15;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              cr[v] = DRre[(lr + v) * 16 + lc];
              ci[v] = DRim[(lr + v) * 16 + lc];
            }
          } else if (J == K) {
            cr = mf4{0.f, 0.f, 0.f, 0.f};
            ci = mf4{0.f, 0.f, 0.f, 0.f};
            cmfma16(Cre + I * 256, Cim + I * 256, DRre, DRim, lane, cr, ci);
          } else {
            tile_load(S, mx, I, J, lane, cr, ci);
            cmfma16(Cre + I * 256, Cim + I * 256, Rre + J * 256, Rim + J * 256, lane, cr, ci);
          }
          tile_store(S, mx, I, J, lane, cr, ci);
        }
        __syncthreads();
      }
      if (packed) {
        store_packed(S, mx, Gb + (int64_t)j * pk);
        __syncthreads();
      }
    }
    if (pivstat && tid == 0) pivstat[box] = make_float2(pmin, pmax);
  }
}

// ------------------------------- complex64 factor, MFMA, register-resident
// The same blocked Gauss-Jordan as factor_mfma_kernel (identical arithmetic in
// identical order, so the factors are bitwise equal), for boxes up to
// 16 * RF_NT wide, with the working matrix held in registers instead of
// memory: 8 waves per box, tile t = I * nt + J owned by wave t % 8 in its
// slot t / 8 (MFMA output layout, as above).  Only the panels of block K
// pass through LDS; S_j = T_j - B_{j-1} G_{j-1} B_{j-1} is formed in the same
// registers from G_{j-1}, so the only traffic to memory is the output G_j.
// Entries past mx are kept as identity after every update, as the
// workspace kernel's loads present them.
constexpr int RF_NT = 12;
constexpr int RF_WAVES = 8;
constexpr int RF_SLOTS = (RF_NT * RF_NT + RF_WAVES - 1) / RF_WAVES;

__global__ __launch_bounds__(64 * RF_WAVES) void factor_mfma_regs_kernel(
    const BoxDesc* __restrict__ desc, const double2* __restrict__ ltab,
    const double* __restrict__ k2, int ngx, float2* __restrict__ G, int packed,
    float2* __restrict__ pivstat) {
  __shared__ float Cre[RF_NT * 256], Cim[RF_NT * 256];  // -S[I,K] as [k][i] per I
  __shared__ float Rre[RF_NT * 256], Rim[RF_NT * 256];  // S[K,J] then D^-1 S[K,J], [k][j]
  __shared__ float DRre[256], DRim[256];                // D^-1 row-major [k][j]
  __shared__ float DTre[256], DTim[256];                // D^-1 transposed [k][i]
  // x-line j: diagonal and first off-diagonal of T_j, and the coupling
  // factors B_{j-1}(a) = ax(a) ihy(j), rounded to complex64 as used
  __shared__ float2 Tdg[16 * RF_NT], Tof[16 * RF_NT], Bf[16 * RF_NT];
  __shared__ float Sd[16 * RF_NT];  // |S_j(a, a)|
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave0 = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform: tile choices are scalar
  const int lr = 4 * (lane >> 4), lc = lane & 15;
  const BoxDesc bd = desc[blockIdx.x];
  const int mx = bd.mx, my = bd.my;
  const int nt = (mx + 15) >> 4;
  const BoxTabs t = box_tabs(ltab, bd);
  float2* Gb = G + bd.g_off;
  const int64_t pk = (int64_t)packed_tiles(nt) * 256;  // entries of one packed G_j
  mf4 tre[RF_SLOTS], tim[RF_SLOTS];
  float pmin = __builtin_inff(), pmax = 0.f;  // pivot magnitudes of this box (wave 0)
  // entries past mx: identity (selects, no branches)
  auto pad = [&](int I, int J, mf4& re, mf4& im) {
    const int b = 16 * J + lc;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int a = 16 * I + lr + v;
      const bool out = a >= mx || b >= mx;
      re[v] = out ? (a == b ? 1.f : 0.f) : re[v];
      im[v] = out ? 0.f : im[v];
    }
  };
  for (int j = 0; j < my; ++j) {
    // the wave index is made opaque in every loop iteration, so the per-slot
    // index arithmetic is recomputed rather than hoisted and kept live for all
    // slots (which would not fit the registers next to the tiles)
    int wave = wave0;
    asm volatile("" : "+s"(wave));
    // S_j = T_j - B_{j-1} G_{j-1} B_{j-1}, G_{j-1} being this lane's registers
    {
      const double* krow = k2 + (int64_t)(bd.by0 + j) * ngx + bd.bx0;
      const double2 ihyj = t.ihy[j];
      for (int a = tid; a < mx; a += blockDim.x) {
        Tdg[a] = from_d<float2>(line_block_entry(t, a, a, j, krow[a]));
        Tof[a] = a + 1 < mx ? from_d<float2>(line_block_entry(t, a + 1, a, j, 0.0))
                            : make_float2(0.f, 0.f);
        Bf[a] = from_d<float2>(dmul(t.ax[a], ihyj));
      }
      __syncthreads();
#pragma unroll
      for (int s = 0; s < RF_SLOTS; ++s) {
        const int tt = wave + RF_WAVES * s;
        if (tt >= nt * nt) continue;
        const int I = tt / nt, J = tt - I * nt;
        const int b = 16 * J + lc, bc = min(b, mx - 1);
        const float2 bb = Bf[bc], tdb = Tdg[bc], tob = Tof[bc];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int a = 16 * I + lr + v, ac = min(a, mx - 1);
          const float2 ba = Bf[ac], toa = Tof[ac];
          float2 val = a == b       ? tdb
                       : a == b + 1 ? tob
                       : b == a + 1 ? toa
                                    : make_float2(0.f, 0.f);
          if (j > 0) val = csub(val, cmul(cmul(ba, make_float2(tre[s][v], tim[s][v])), bb));
          tre[s][v] = val.x;
          tim[s][v] = val.y;
          if (a == b && a < mx) Sd[a] = sqrtf(val.x * val.x + val.y * val.y);
        }
        pad(I, J, tre[s], tim[s]);
      }
    }
    for (int K = 0; K < nt; ++K) {
      wave = wave0;
      asm volatile("" : "+s"(wave));
      // panels of block K from their owners: column panel negated as [k][i],
      // row panel as [k][j]
#pragma unroll
      for (int s = 0; s < RF_SLOTS; ++s) {
        const int tt = wave + RF_WAVES * s;
        if (tt >= nt * nt) continue;
        const int I = tt / nt, J = tt - I * nt;
        if (J == K) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            Cre[I * 256 + lc * 16 + lr + v] = -tre[s][v];
            Cim[I * 256 + lc * 16 + lr + v] = -tim[s][v];
          }
        }
        if (I == K) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            Rre[J * 256 + (lr + v) * 16 + lc] = tre[s][v];
            Rim[J * 256 + (lr + v) * 16 + lc] = tim[s][v];
          }
        }
      }
      __syncthreads();
      if (wave0 == 0)
        invert_d16(Rre + K * 256, Rim + K * 256, lane, DRre, DRim, DTre, DTim, mx - 16 * K,
                   Sd + 16 * K, pmin, pmax);
      __syncthreads();
      // row panel: D^-1 S[K,J], by the owner of (K, J), to LDS and registers
#pragma unroll
      for (int s = 0; s < RF_SLOTS; ++s) {
        const int tt = wave + RF_WAVES * s;
        if (tt >= nt * nt) continue;
        const int I = tt / nt, J = tt - I * nt;
        if (I != K || J == K) continue;
        mf4 cr = mf4{0.f, 0.f, 0.f, 0.f}, ci = mf4{0.f, 0.f, 0.f, 0.f};
        cmfma16(DTre, DTim, Rre + J * 256, Rim + J * 256, lane, cr, ci);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          Rre[J * 256 + (lr + v) * 16 + lc] = cr[v];
          Rim[J * 256 + (lr + v) * 16 + lc] = ci[v];
        }
        pad(I, J, cr, ci);
        tre[s] = cr;
        tim[s] = ci;
      }
      __syncthreads();
      // pivot block, column panel, rank-16 update of every other tile
#pragma unroll
      for (int s = 0; s < RF_SLOTS; ++s) {
        const int tt = wave + RF_WAVES * s;
        if (tt >= nt * nt) continue;
        const int I = tt / nt, J = tt - I * nt;
        if (I == K && J != K) continue;
        mf4 cr, ci;
        if (I == K) {  // J == K
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            cr[v] = DRre[(lr + v) * 16 + lc];
            ci[v] = DRim[(lr + v) * 16 + lc];
          }
        } else if (J == K) {
          cr = mf4{0.f, 0.f, 0.f, 0.f};
          ci = mf4{0.f, 0.f, 0.f, 0.f};
          cmfma16(Cre + I * 256, Cim + I * 256, DRre, DRim, lane, cr, ci);
        } else {
          cr = tre[s];
          ci = tim[s];
          cmfma16(Cre + I * 256, Cim + I * 256, Rre + J * 256, Rim + J * 256, lane, cr, ci);
        }
        pad(I, J, cr, ci);
        tre[s] = cr;
        tim[s] = ci;
      }
      __syncthreads();
    }
    wave = wave0;
    asm volatile("" : "+s"(wave));
    // G_j out.  Packed: tile (I, J), I <= J, entry (r, c) = G(16J + c, 16I + r),
    // i.e. register tile (J, I) read across (a diagonal tile's upper triangle
    // at diag_pos); dense: column-major, all entries.
#pragma unroll
    for (int s = 0; s < RF_SLOTS; ++s) {
      const int tt = wave + RF_WAVES * s;
      if (tt >= nt * nt) continue;
      const int P = tt / nt, Q = tt - P * nt;  // rows block P, columns block Q
      const int b = 16 * Q + lc;
      float2 o[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int a = 16 * P + lr + v;
        o[v] = (a < mx && b < mx) ? make_float2(tre[s][v], tim[s][v]) : make_float2(0.f, 0.f);
      }
      if (packed) {
        if (P < Q) continue;
        if (P == Q) {  // diagonal tile: entry (lc, lr + v), upper triangle only
          float2* dt = Gb + (int64_t)j * pk + (int64_t)(P * (P + 1) / 2 + Q) * 256;
#pragma unroll
          for (int v = 0; v < 4; ++v)
            dt[diag_pos(lc, lr + v)] = lc <= lr + v ? o[v] : make_float2(0.f, 0.f);
          continue;
        }
        float4* dst = reinterpret_cast<float4*>(Gb + (int64_t)j * pk +
                                                (int64_t)(P * (P + 1) / 2 + Q) * 256 + lc * 16 + lr);
        dst[0] = make_float4(o[0].x, o[0].y, o[1].x, o[1].y);
        dst[1] = make_float4(o[2].x, o[2].y, o[3].x, o[3].y);
      } else if (b < mx) {
        float2* col = Gb + (int64_t)j * mx * mx + (int64_t)b * mx;
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (16 * P + lr + v < mx) col[16 * P + lr + v] = o[v];
      }
    }
  }
  if (pivstat && tid == 0) pivstat[blockIdx.x] = make_float2(pmin, pmax);
}

// ----------------- complex64 factor, MFMA, registers, symmetric elimination
// S_j is complex symmetric, so its inverse can be formed on the tiles on and
// above the diagonal only, by the symmetric form of Gauss-Jordan (the sweep
// operator): eliminating on the diagonal block D = A[K,K] maps
//     A[K,K] -> -D^-1,      A[K,J] -> D^-1 A[K,J],      A[I,K] -> A[I,K] D^-1,
//     A[I,J] -> A[I,J] - A[I,K] D^-1 A[K,J]       (I, J != K),
// which keeps A symmetric; after every block has been eliminated A holds
// -S_j^-1.  With P_J = A[K,J] (the old block row) and Q_J = D^-1 P_J, the
// upper tiles update as A[I,J] -= P_I^T Q_J, the new block row is Q_J (tile
// (K, J), J > K) or Q_J^T (tile (J, K), J < K).  The pivot blocks and hence
// the pivots are those of the full elimination (same Schur complements);
// about half the matrix-core work and half the registers of
// factor_mfma_regs_kernel, so two boxes share a compute unit.
// Tile u of the upper triangle (row by row: (0,0), (0,1), ..., (1,1), ...) is
// held by wave u % 8 in its slot u / 8, in MFMA output layout.  Registers
// hold A = -G between x-lines: S_{j+1} = T_{j+1} + B_j A B_j.
constexpr int SF_NT = 12;
constexpr int SF_WAVES = 8;
constexpr int SF_SLOTS = (SF_NT * (SF_NT + 1) / 2 + SF_WAVES - 1) / SF_WAVES;

// (I, J) of upper-triangle tile u (wave-uniform)
__device__ __forceinline__ void tri_tile(int u, int nt, int& I, int& J) {
  I = 0;
  while (u >= nt - I) {
    u -= nt - I;
    ++I;
  }
  J = I + u;
}

// (cre, cim) += (-A)^T B over one 16x16x16 block, the operands laid out
// [k][16] in LDS as for cmfma16
__device__ __forceinline__ void cmfma16_neg(const float* Ar, const float* Ai, const float* Br,
                                            const float* Bi, int lane, mf4& cre, mf4& cim) {
#pragma unroll
  for (int kc = 0; kc < 4; ++kc) {
    const int o = (kc * 4 + (lane >> 4)) * 16 + (lane & 15);
    const float ar = Ar[o], ai = Ai[o], br = Br[o], bi = Bi[o];
    cre = mfma4(-ar, br, cre);
    cre = mfma4(ai, bi, cre);
    cim = mfma4(-ar, bi, cim);
    cim = mfma4(-ai, br, cim);
  }
}

__global__ __launch_bounds__(64 * SF_WAVES) __attribute__((amdgpu_waves_per_eu(4, 4))) void
factor_sym_regs_kernel(const BoxDesc* __restrict__ desc, const double2* __restrict__ ltab,
                       const double* __restrict__ k2, int ngx, float2* __restrict__ G, int packed,
                       float2* __restrict__ pivstat) {
  __shared__ float Pre[SF_NT * 256], Pim[SF_NT * 256];  // P_J = A[K,J] as [k][j] per J
  __shared__ float Qre[SF_NT * 256], Qim[SF_NT * 256];  // Q_J = D^-1 P_J as [k][j] per J
  __shared__ float DRre[256], DRim[256];                // D^-1 row-major [k][j]
  __shared__ float DTre[256], DTim[256];                // D^-1 transposed [j][k]
  __shared__ float2 Tdg[16 * SF_NT], Tof[16 * SF_NT], Bf[16 * SF_NT];
  __shared__ float Sd[16 * SF_NT];  // |S_j(a, a)|
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave0 = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lr = 4 * (lane >> 4), lc = lane & 15;
  const BoxDesc bd = desc[blockIdx.x];
  const int mx = bd.mx, my = bd.my;
  const int nt = (mx + 15) >> 4, ntri = nt * (nt + 1) / 2;
  const BoxTabs t = box_tabs(ltab, bd);
  float2* Gb = G + bd.g_off;
  const int64_t pk = (int64_t)packed_tiles(nt) * 256;
  mf4 tre[SF_SLOTS], tim[SF_SLOTS];
  float pmin = __builtin_inff(), pmax = 0.f;
  auto pad = [&](int I, int J, mf4& re, mf4& im) {
    const int b = 16 * J + lc;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int a = 16 * I + lr + v;
      const bool out = a >= mx || b >= mx;
      re[v] = out ? (a == b ? 1.f : 0.f) : re[v];
      im[v] = out ? 0.f : im[v];
    }
  };
  for (int j = 0; j < my; ++j) {
    int wave = wave0;
    asm volatile("" : "+s"(wave));
    {
      const double* krow = k2 + (int64_t)(bd.by0 + j) * ngx + bd.bx0;
      const double2 ihyj = t.ihy[j];
      for (int a = tid; a < mx; a += blockDim.x) {
        Tdg[a] = from_d<float2>(line_block_entry(t, a, a, j, krow[a]));
        Tof[a] = a + 1 < mx ? from_d<float2>(line_block_entry(t, a + 1, a, j, 0.0))
                            : make_float2(0.f, 0.f);
        Bf[a] = from_d<float2>(dmul(t.ax[a], ihyj));
      }
      __syncthreads();
#pragma unroll
      for (int s = 0; s < SF_SLOTS; ++s) {
        const int u = wave + SF_WAVES * s;
        if (u >= ntri) continue;
        int I, J;
        tri_tile(u, nt, I, J);
        const int b = 16 * J + lc, bc = min(b, mx - 1);
        const float2 bb = Bf[bc], tdb = Tdg[bc], tob = Tof[bc];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int a = 16 * I + lr + v, ac = min(a, mx - 1);
          const float2 ba = Bf[ac], toa = Tof[ac];
          float2 val = a == b       ? tdb
                       : a == b + 1 ? tob
                       : b == a + 1 ? toa
                                    : make_float2(0.f, 0.f);
          // - B G_{j-1} B with the registers holding -G_{j-1}
          if (j > 0) val = cadd(val, cmul(cmul(ba, make_float2(tre[s][v], tim[s][v])), bb));
          tre[s][v] = val.x;
          tim[s][v] = val.y;
          if (a == b && a < mx) Sd[a] = sqrtf(val.x * val.x + val.y * val.y);
        }
        pad(I, J, tre[s], tim[s]);
      }
    }
    for (int K = 0; K < nt; ++K) {
      wave = wave0;
      asm volatile("" : "+s"(wave));
      // old block row P_J = A[K,J]: from tile (K, J), J >= K, or, read
      // across, from tile (J, K), J < K
#pragma unroll
      for (int s = 0; s < SF_SLOTS; ++s) {
        const int u = wave + SF_WAVES * s;
        if (u >= ntri) continue;
        int I, J;
        tri_tile(u, nt, I, J);
        if (I == K) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            Pre[J * 256 + (lr + v) * 16 + lc] = tre[s][v];
            Pim[J * 256 + (lr + v) * 16 + lc] = tim[s][v];
          }
        } else if (J == K) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            Pre[I * 256 + lc * 16 + lr + v] = tre[s][v];
            Pim[I * 256 + lc * 16 + lr + v] = tim[s][v];
          }
        }
      }
      __syncthreads();
      if (wave0 == 0)
        invert_d16(Pre + K * 256, Pim + K * 256, lane, DRre, DRim, DTre, DTim, mx - 16 * K,
                   Sd + 16 * K, pmin, pmax);
      __syncthreads();
      // new block row: Q_J = D^-1 P_J into tile (K, J), Q_J^T = P_J^T D^-T
      // into tile (J, K); Q_J to LDS as [k][j] either way; -D^-1 on the diagonal
#pragma unroll
      for (int s = 0; s < SF_SLOTS; ++s) {
        const int u = wave + SF_WAVES * s;
        if (u >= ntri) continue;
        int I, J;
        tri_tile(u, nt, I, J);
        if (I != K && J != K) continue;
        mf4 cr = mf4{0.f, 0.f, 0.f, 0.f}, ci = mf4{0.f, 0.f, 0.f, 0.f};
        if (I == K && J == K) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            cr[v] = -DRre[(lr + v) * 16 + lc];
            ci[v] = -DRim[(lr + v) * 16 + lc];
          }
        } else if (I == K) {
          cmfma16(DTre, DTim, Pre + J * 256, Pim + J * 256, lane, cr, ci);
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            Qre[J * 256 + (lr + v) * 16 + lc] = cr[v];
            Qim[J * 256 + (lr + v) * 16 + lc] = ci[v];
          }
        } else {
          cmfma16(Pre + I * 256, Pim + I * 256, DTre, DTim, lane, cr, ci);
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            Qre[I * 256 + lc * 16 + lr + v] = cr[v];
            Qim[I * 256 + lc * 16 + lr + v] = ci[v];
          }
        }
        tre[s] = cr;
        tim[s] = ci;
      }
      __syncthreads();
      // A[I,J] -= P_I^T Q_J on every other upper tile
#pragma unroll
      for (int s = 0; s < SF_SLOTS; ++s) {
        const int u = wave + SF_WAVES * s;
        if (u >= ntri) continue;
        int I, J;
        tri_tile(u, nt, I, J);
        if (I == K || J == K) continue;
        cmfma16_neg(Pre + I * 256, Pim + I * 256, Qre + J * 256, Qim + J * 256, lane, tre[s],
                    tim[s]);
      }
      __syncthreads();
    }
    wave = wave0;
    asm volatile("" : "+s"(wave));
    // G_j = -A.  Packed: tile (I, J), I <= J, entry (r, c) = G(16I + r, 16J + c)
    // = this lane's register tile directly (a diagonal tile's upper triangle
    // at diag_pos); dense: column-major, both triangles.
#pragma unroll
    for (int s = 0; s < SF_SLOTS; ++s) {
      const int u = wave + SF_WAVES * s;
      if (u >= ntri) continue;
      int I, J;
      tri_tile(u, nt, I, J);
      const int b = 16 * J + lc;
      float2 o[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int a = 16 * I + lr + v;
        o[v] = (a < mx && b < mx) ? make_float2(-tre[s][v], -tim[s][v]) : make_float2(0.f, 0.f);
      }
      if (packed) {
        float2* dst = Gb + (int64_t)j * pk + (int64_t)(J * (J + 1) / 2 + I) * 256;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          if (I == J)  // diagonal tile: upper triangle only, zeros after it
            dst[diag_pos(lr + v, lc)] = lr + v <= lc ? o[v] : make_float2(0.f, 0.f);
          else
            dst[(lr + v) * 16 + lc] = o[v];
        }
      } else {
        float2* Gj = Gb + (int64_t)j * mx * mx;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int a = 16 * I + lr + v;
          if (a < mx && b < mx) {
            Gj[(int64_t)b * mx + a] = o[v];
            if (I != J) Gj[(int64_t)a * mx + b] = o[v];
          }
        }
      }
    }
  }
  if (pivstat && tid == 0) pivstat[blockIdx.x] = make_float2(pmin, pmax);
}

// ---------------------------------------------------------------- sweeps
// Vector loads of two consecutive complex entries (rows 2p, 2p+1 of a column).
__device__ __forceinline__ void load_pair(const float2* p, float2& a, float2& b) {
  const float4 v = *reinterpret_cast<const float4*>(p);
  a = make_float2(v.x, v.y);
  b = make_float2(v.z, v.w);
}
__device__ __forceinline__ void load_pair(const double2* p, double2& a, double2& b) {
  a = p[0];
  b = p[1];
}

// One workgroup per box (grid-stride over boxes).  Thread t = k*RP + rp owns
// rows 2rp, 2rp+1 of every GEMV and columns b = k, k+K, ...; partial sums of
// the K column groups meet in LDS and are added in a fixed order.
template <typename C>
__global__ __launch_bounds__(1024) void sweep_kernel(const BoxDesc* __restrict__ desc,
                                                     const double2* __restrict__ ltab,
                                                     const C* __restrict__ G, C* __restrict__ X,
                                                     const double2* __restrict__ r, int ngx,
                                                     int nboxes, int max_m) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* vbuf = reinterpret_cast<C*>(smem_raw);  // [2][max_m]
  C* pbuf = vbuf + 2 * max_m;                // [K][mx] partials, <= 2*blockDim entries
  const int tid = threadIdx.x;
  for (int box = blockIdx.x; box < nboxes; box += gridDim.x) {
    const BoxDesc bd = desc[box];
    const int mx = bd.mx, my = bd.my;
    const int RP = mx >> 1;
    const int K = blockDim.x / RP;
    const int k = tid / RP, rp = tid - (tid / RP) * RP;
    const bool active = k < K;
    const BoxTabs t = box_tabs(ltab, bd);
    const C* Gb = G + bd.g_off;
    C* Xb = X + bd.x_off;
    const int64_t n2 = (int64_t)mx * mx;
    // source row j restricted to the tile (Sec. 2 eq. ddm0)
    auto src = [&](int j, int i) -> C {
      if (j >= bd.ty0 && j < bd.ty1 && i >= bd.tx0 && i < bd.tx1)
        return from_d<C>(r[(int64_t)(bd.by0 + j) * ngx + bd.bx0 + i]);
      return czero<C>();
    };
    // ---- forward sweep: rows below the tile have zero source, so y = 0 there
    const int j0 = bd.ty0;
    for (int e = tid; e < j0 * mx; e += blockDim.x) Xb[e] = czero<C>();
    if (tid < mx) vbuf[tid] = src(j0, tid);
    __syncthreads();
    int cur = 0;
    for (int j = j0; j < my; ++j) {
      const C* Gj = Gb + (int64_t)j * n2;
      C acc0 = czero<C>(), acc1 = czero<C>();
      if (active) {
        for (int b = k; b < mx; b += K) {
          C g0, g1;
          load_pair(Gj + (int64_t)b * mx + 2 * rp, g0, g1);
          const C vb = vbuf[cur * max_m + b];
          acc0 = cfma(g0, vb, acc0);
          acc1 = cfma(g1, vb, acc1);
        }
        pbuf[k * mx + 2 * rp] = acc0;
        pbuf[k * mx + 2 * rp + 1] = acc1;
      }
      __syncthreads();
      if (tid < mx) {
        C y = czero<C>();
        for (int q = 0; q < K; ++q) y = cadd(y, pbuf[q * mx + tid]);
        Xb[(int64_t)j * mx + tid] = y;
        if (j + 1 < my) {
          const C bj = from_d<C>(dmul(t.ax[tid], t.ihy[j + 1]));  // B_j coupling to line j+1
          vbuf[(cur ^ 1) * max_m + tid] = csub(src(j + 1, tid), cmul(bj, y));
        }
      }
      cur ^= 1;
      __syncthreads();
    }
    // ---- backward sweep: x_{my-1} = y_{my-1}; x_j = y_j - G_j (B_j x_{j+1})
    if (tid < mx && my > 1) {
      const C bj = from_d<C>(dmul(t.ax[tid], t.ihy[my - 1]));  // B_{my-2}
      vbuf[tid] = cmul(bj, Xb[(int64_t)(my - 1) * mx + tid]);
    }
    cur = 0;
    __syncthreads();
    for (int j = my - 2; j >= 0; --j) {
      const C* Gj = Gb + (int64_t)j * n2;
      C acc0 = czero<C>(), acc1 = czero<C>();
      if (active) {
        for (int b = k; b < mx; b += K) {
          C g0, g1;
          load_pair(Gj + (int64_t)b * mx + 2 * rp, g0, g1);
          const C vb = vbuf[cur * max_m + b];
          acc0 = cfma(g0, vb, acc0);
          acc1 = cfma(g1, vb, acc1);
        }
        pbuf[k * mx + 2 * rp] = acc0;
        pbuf[k * mx + 2 * rp + 1] = acc1;
      }
      __syncthreads();
      if (tid < mx) {
        C s = czero<C>();
        for (int q = 0; q < K; ++q) s = cadd(s, pbuf[q * mx + tid]);
        const C x = csub(Xb[(int64_t)j * mx + tid], s);
        Xb[(int64_t)j * mx + tid] = x;
        if (j > 0) {
          const C bj = from_d<C>(dmul(t.ax[tid], t.ihy[j]));  // B_{j-1}
          vbuf[(cur ^ 1) * max_m + tid] = cmul(bj, x);
        }
      }
      cur ^= 1;
      __syncthreads();
    }
  }
}

// ------------------------------------------------------- complex64 sweeps
// Workgroup barrier that orders LDS only: global loads issued before it (the
// next block's prefetch) stay in flight across the barrier.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

typedef float nf4 __attribute__((ext_vector_type(4)));
typedef unsigned int nu4 __attribute__((ext_vector_type(4)));
typedef unsigned int nu2 __attribute__((ext_vector_type(2)));

// Streaming 16-byte load that bypasses cache retention (each G entry is used
// once per sweep).
__device__ __forceinline__ float4 stream_load(const float2* p) {
  const nf4 v = __builtin_nontemporal_load(reinterpret_cast<const nf4*>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}

// Values the whole wave shares, moved to scalar registers explicitly.
__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
template <typename T>
__device__ __forceinline__ T* wave_uniform_ptr(T* p) {
  const uint64_t a = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
  return reinterpret_cast<T*>(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ float2 f2fma(float2 a, float2 b, float2 acc) {
  acc.x = fmaf(a.x, b.x, acc.x);
  acc.x = fmaf(-a.y, b.y, acc.x);
  acc.y = fmaf(a.x, b.y, acc.y);
  acc.y = fmaf(a.y, b.x, acc.y);
  return acc;
}

// One workgroup per box, ceil(mx/16) waves.  Lane l of wave w owns rows
// 2p, 2p+1 with p = 8w + (l & 7) and the column group k = l >> 3 (columns
// c = k, k+8, ...).  Each step of the two sweeps is one GEMV with G_j: every
// lane streams its <= LMAX column pairs (16 bytes each; 8 lanes of a group
// read 128 contiguous bytes), the 8 column groups are summed by cross-lane
// shuffles, and lanes with k = 0 form the next right-hand side in LDS.  The
// loads of the next block are issued before the step's reduction and barrier
// so HBM streaming never waits on the sequential dependence.
template <int LMAX>
__global__ __launch_bounds__(64 * LMAX / 2) void sweep64_kernel(const BoxDesc* __restrict__ desc,
                                                       const double2* __restrict__ ltab,
                                                       const float2* __restrict__ G,
                                                       float2* __restrict__ X,
                                                       const double2* __restrict__ r, int ngx,
                                                       int nboxes, int max_m) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  float2* vbuf = reinterpret_cast<float2*>(smem_raw);  // [2][max_m]
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int k = lane >> 3;
  for (int box = blockIdx.x; box < nboxes; box += gridDim.x) {
    const BoxDesc bd = desc[box];
    const int mx = wave_uniform(bd.mx), my = wave_uniform(bd.my);
    const int p = wave * 8 + (lane & 7);
    const bool active = p < (mx >> 1);
    const bool lead = active && k == 0;
    const int r0 = 2 * p;
    const BoxTabs t = box_tabs(ltab, bd);
    const float2* __restrict__ Gbox = wave_uniform_ptr(G + bd.g_off);
    const int64_t n2 = (int64_t)mx * mx;
    const int j0 = wave_uniform(bd.ty0), nf = my - j0, T = nf + (my - 1);
    // stretch factors of this lane's two rows (the coupling B_j = ax ihy is
    // formed in FP32, the precision of the whole complex64 sweep)
    float2 ax0 = make_float2(0.f, 0.f), ax1 = make_float2(0.f, 0.f);
    if (lead) {
      const double2 a0d = t.ax[r0], a1d = t.ax[r0 + 1];
      ax0 = make_float2((float)a0d.x, (float)a0d.y);
      ax1 = make_float2((float)a1d.x, (float)a1d.y);
    }
    const bool col0_in = r0 >= bd.tx0 && r0 < bd.tx1, col1_in = r0 + 1 >= bd.tx0 && r0 + 1 < bd.tx1;
    // All loads in the step loop are unconditional on in-bounds addresses;
    // masks are applied when the value is used one step later, so no load is
    // ever waited on early and the compiler's wait counters stay exact.
    const int rs = active ? r0 : 0;  // idle lanes read row pair 0
    const double2* __restrict__ rbase = r + (int64_t)bd.by0 * ngx + bd.bx0 + rs;
    float2* __restrict__ Xs = X + bd.x_off + rs;
    auto row_of = [&](int st) { return st < nf ? j0 + st : my - 2 - (st - nf); };
    float4 g[LMAX];
    // G_j is read through a buffer resource covering exactly that block: one
    // 32-bit lane offset plus a uniform per-column offset, and offsets past the
    // block (columns >= mx, idle lanes) return zeros without touching memory.
    const int voff = active ? (k * mx + r0) * 8 : 0x40000000;
    const int col_step = 64 * mx;  // 8 columns of mx complex64 entries
    const int blk_bytes = (int)(n2 * 8);
    auto block_rsrc = [&](int jr, int bytes) {
      return __builtin_amdgcn_make_buffer_rsrc(
          const_cast<float2*>(wave_uniform_ptr(Gbox + (int64_t)jr * n2)), 0, wave_uniform(bytes),
          0x00020000);
    };
    auto load_col = [&](__amdgpu_buffer_rsrc_t rsrc, int s) {
      const nu4 v = __builtin_amdgcn_raw_buffer_load_b128(rsrc, voff, s * col_step, 2 /*nt*/);
      g[s] = make_float4(__uint_as_float(v.x), __uint_as_float(v.y), __uint_as_float(v.z),
                         __uint_as_float(v.w));
    };
    // entries past this box's width stay zero for the whole box
    for (int e = threadIdx.x; e < 2 * max_m; e += blockDim.x)
      if (e % max_m >= mx) vbuf[e] = make_float2(0.f, 0.f);
    // prologue: right-hand side of the first step (tile source of row j0),
    // the prefetched inputs of step 0's reduction, the first block
    if (lead) {
      const bool row_in = j0 >= bd.ty0 && j0 < bd.ty1;
      const double2* rr = rbase + (int64_t)j0 * ngx;
      const double2 s0 = (row_in && col0_in) ? rr[0] : make_double2(0.0, 0.0);
      const double2 s1 = (row_in && col1_in) ? rr[1] : make_double2(0.0, 0.0);
      vbuf[r0] = make_float2((float)s0.x, (float)s0.y);
      vbuf[r0 + 1] = make_float2((float)s1.x, (float)s1.y);
    }
    // prefetched state for the reduction of the coming step
    float4 py = make_float4(0.f, 0.f, 0.f, 0.f);  // y of its row (backward)
    bool py_use = false;
    double2 ps0, ps1;                              // source of the row after it
    bool ps_row = false;
    double2 pih;                                   // coupling factor ihy[.]
    {
      const int jr = min(j0 + 1, my - 1);
      const double2* rr = rbase + (int64_t)jr * ngx;
      ps0 = rr[0];
      ps1 = rr[1];
      ps_row = (j0 + 1 >= bd.ty0) && (j0 + 1 < bd.ty1);
      pih = t.ihy[nf > 1 ? j0 + 1 : j0];
      const __amdgpu_buffer_rsrc_t r0src = block_rsrc(j0, blk_bytes);
#pragma unroll
      for (int s = 0; s < LMAX; ++s) load_col(r0src, s);
    }
    lds_barrier();
    int cur = 0;
#pragma unroll 1
    for (int st = 0; st < T; ++st) {
      const bool fwd = st < nf;
      const int j = __builtin_amdgcn_readfirstlane(row_of(st));
      const bool more = st + 1 < T;
      const int jn = __builtin_amdgcn_readfirstlane(row_of(more ? st + 1 : st));
      // partial GEMV over this lane's columns in chunks of 8 (only 8
      // right-hand-side values live at once).  No masking: entries of vbuf
      // past mx are zero, and G entries of idle lanes and of columns past mx
      // arrive as zeros from the range check.
      float2 a0 = make_float2(0.f, 0.f), a1 = make_float2(0.f, 0.f);
      const float2* vb = vbuf + cur * max_m;
#pragma unroll
      for (int s0 = 0; s0 < LMAX; s0 += 8) {
#pragma unroll
        for (int s = s0; s < (s0 + 8 < LMAX ? s0 + 8 : LMAX); ++s) {
          const float2 v = vb[min(k + 8 * s, max_m - 1)];
          a0 = f2fma(make_float2(g[s].x, g[s].y), v, a0);
          a1 = f2fma(make_float2(g[s].z, g[s].w), v, a1);
        }
        __builtin_amdgcn_sched_barrier(0);
      }
      // inputs of this step's reduction, loaded during the previous step
      const float4 cy = py_use ? py : make_float4(0.f, 0.f, 0.f, 0.f);
      const double2 cs0 = (ps_row && col0_in) ? ps0 : make_double2(0.0, 0.0);
      const double2 cs1 = (ps_row && col1_in) ? ps1 : make_double2(0.0, 0.0);
      const double2 ih = pih;
      // sum the 8 column groups (lanes l, l^8, l^16, l^32 share rows)
#pragma unroll
      for (int o = 8; o < 64; o <<= 1) {
        a0.x += __shfl_xor(a0.x, o, 64);
        a0.y += __shfl_xor(a0.y, o, 64);
        a1.x += __shfl_xor(a1.x, o, 64);
        a1.y += __shfl_xor(a1.y, o, 64);
      }
      if (lead) {
        float2 x0, x1;
        if (fwd) {
          x0 = a0;
          x1 = a1;
        } else {  // x_j = y_j - G_j (B_j x_{j+1});  y_j = 0 below the tile
          x0 = make_float2(cy.x - a0.x, cy.y - a0.y);
          x1 = make_float2(cy.z - a1.x, cy.w - a1.y);
        }
        *reinterpret_cast<float4*>(Xs + (int64_t)j * mx) = make_float4(x0.x, x0.y, x1.x, x1.y);
        if (more) {
          float2* vn = vbuf + (cur ^ 1) * max_m;
          const float2 ihf = make_float2((float)ih.x, (float)ih.y);
          const float2 b0 = cmul(ax0, ihf), b1 = cmul(ax1, ihf);
          const float2 c0 = cmul(b0, x0), c1 = cmul(b1, x1);
          // forward next (row j+1): b_{j+1} - B_j y_j with B_j = ax ihy[j+1];
          // backward next (row j-1): B_{j-1} x_j with B_{j-1} = ax ihy[j]
          const float sg = (st + 1 < nf) ? -1.f : 1.f;
          vn[r0] = make_float2((float)cs0.x + sg * c0.x, (float)cs0.y + sg * c0.y);
          vn[r0 + 1] = make_float2((float)cs1.x + sg * c1.x, (float)cs1.y + sg * c1.y);
        }
      }
      // prefetch for the next step, after this step's reduction so that the
      // block's registers are free: its y (backward), the source of the row
      // after it, its coupling factor, then its block (an empty resource
      // after the last step: zeros, no traffic).  These loads stay in flight
      // across the LDS-only barrier.
      __builtin_amdgcn_sched_barrier(0);
      {
        py = *reinterpret_cast<const float4*>(Xs + (int64_t)jn * mx);
        py_use = more && st + 1 >= nf && jn >= j0;
        const bool nn_fwd = st + 2 < nf;  // is the step after next forward?
        const int jr = min(jn + 1, my - 1);
        const double2* rr = rbase + (int64_t)jr * ngx;
        ps0 = rr[0];
        ps1 = rr[1];
        ps_row = nn_fwd && (jn + 1 >= bd.ty0) && (jn + 1 < bd.ty1);
        pih = t.ihy[nn_fwd ? jn + 1 : jn];
        const __amdgpu_buffer_rsrc_t nsrc = block_rsrc(jn, more ? blk_bytes : 0);
#pragma unroll
        for (int s = 0; s < LMAX; ++s) load_col(nsrc, s);
      }
      cur ^= 1;
      lds_barrier();
    }
  }
}

// ------------------------------------ complex64 sweeps, symmetric-packed G
// One workgroup per box with ceil(nt/2) waves.  Wave w owns the column blocks
// J0 = w and J1 = nt-1-w of the packed upper tiles (nt+1 tiles per wave, or
// (nt+1)/2 for the middle block of an odd nt), so every stored entry is read
// once per step and used twice:
//   row part    y_I += T_IJ v_J   for every owned tile (I <= J), and
//   column part y_J += T_IJ^T v_I for the strictly upper ones (I < J).
// Lane l holds row r = l & 15 and columns 4q..4q+3 (q = l >> 4) of a tile (32
// contiguous bytes).  Row parts are summed over q by shuffles and passed
// through LDS per (J, I); column parts accumulate in registers over the wave's
// tiles and are summed over r by shuffles once per step.  Thread a < mx then
// forms y_a (row parts of all J >= I plus the column part of block I), the
// box-solution row and the next right-hand side.  Loads of the next block go
// through a buffer resource (unused tile slots and idle lanes read zeros with
// no traffic) and are issued before the step's barriers.
template <int TMAX, int OCC>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(OCC))) void sweep64_sym_kernel(const BoxDesc* __restrict__ desc,
                                                          const double2* __restrict__ ltab,
                                                          const float2* __restrict__ G,
                                                          float2* __restrict__ X,
                                                          const double2* __restrict__ r, int ngx,
                                                          int nboxes) {
  constexpr int NTM = 16;
  __shared__ float2 vbuf[2][NTM * 16];
  __shared__ float2 rowpart[NTM][NTM][16];  // [J][I][r]
  __shared__ float2 colpart[NTM][16];       // [J][c]
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // scalar: tile lists are per wave
  const int lr = lane & 15, lq = lane >> 4;
  for (int box = blockIdx.x; box < nboxes; box += gridDim.x) {
    const BoxDesc bd = desc[box];
    const int mx = wave_uniform(bd.mx), my = wave_uniform(bd.my);
    const int nt = (mx + 15) >> 4, npk = packed_tiles(nt);
    const int nw = (nt + 1) >> 1;
    const bool wactive = wave < nw;
    const int J0 = wave, J1 = nt - 1 - wave;
    const int n0 = J0 + 1;                                  // tiles in column block J0
    const int ntw = !wactive ? 0 : (J1 != J0 ? n0 + J1 + 1 : n0);
    const BoxTabs t = box_tabs(ltab, bd);
    const float2* __restrict__ Gbox = wave_uniform_ptr(G + bd.g_off);
    const int64_t blk = (int64_t)npk * 256;  // entries of one packed G_j
    const int j0 = wave_uniform(bd.ty0), nf = my - j0, T = nf + (my - 1);
    // reducer thread a = tid < mx
    const bool red = tid < mx;
    const int ra = red ? tid : 0;
    const bool col_in = ra >= bd.tx0 && ra < bd.tx1;
    float2 axa = make_float2(0.f, 0.f);
    if (red) {
      const double2 ad = t.ax[ra];
      axa = make_float2((float)ad.x, (float)ad.y);
    }
    const double2* __restrict__ rbase = r + (int64_t)bd.by0 * ngx + bd.bx0 + ra;
    float2* __restrict__ Xa = X + bd.x_off + ra;
    auto row_of = [&](int st) { return st < nf ? j0 + st : my - 2 - (st - nf); };
    auto tile_IJ = [&](int sidx, int& I, int& J) {
      if (sidx < n0) {
        I = sidx;
        J = J0;
      } else {
        I = sidx - n0;
        J = J1;
      }
    };
    // packed tiles of this wave, 2 x 16 bytes per lane each
    float4 g0[TMAX], g1[TMAX];
    const int voff = (lr * 16 + 4 * lq) * 8;
    const int voff_d[4] = {diag_read_pos(lr, 4 * lq) * 8, diag_read_pos(lr, 4 * lq + 1) * 8,
                           diag_read_pos(lr, 4 * lq + 2) * 8, diag_read_pos(lr, 4 * lq + 3) * 8};
    auto block_rsrc = [&](int jr, bool valid) {
      return __builtin_amdgcn_make_buffer_rsrc(
          const_cast<float2*>(wave_uniform_ptr(Gbox + (int64_t)jr * blk)), 0,
          wave_uniform(valid ? npk * 2048 : 0), 0x00020000);
    };
    auto load_tile = [&](__amdgpu_buffer_rsrc_t rsrc, int sidx) {
      int I, J;
      tile_IJ(sidx, I, J);
      const int tno = sidx < ntw ? J * (J + 1) / 2 + I : npk;  // past the block: zeros
      if (sidx < ntw && I == J) {
        // diagonal tile: its upper triangle only; each entry from its stored twin
        const nu2 d0 = __builtin_amdgcn_raw_buffer_load_b64(rsrc, voff_d[0], tno * 2048, 2);
        const nu2 d1 = __builtin_amdgcn_raw_buffer_load_b64(rsrc, voff_d[1], tno * 2048, 2);
        const nu2 d2 = __builtin_amdgcn_raw_buffer_load_b64(rsrc, voff_d[2], tno * 2048, 2);
        const nu2 d3 = __builtin_amdgcn_raw_buffer_load_b64(rsrc, voff_d[3], tno * 2048, 2);
        g0[sidx] = make_float4(__uint_as_float(d0.x), __uint_as_float(d0.y), __uint_as_float(d1.x),
                               __uint_as_float(d1.y));
        g1[sidx] = make_float4(__uint_as_float(d2.x), __uint_as_float(d2.y), __uint_as_float(d3.x),
                               __uint_as_float(d3.y));
        return;
      }
      const nu4 u0 = __builtin_amdgcn_raw_buffer_load_b128(rsrc, voff, tno * 2048, 2 /*nt*/);
      const nu4 u1 = __builtin_amdgcn_raw_buffer_load_b128(rsrc, voff + 16, tno * 2048, 2);
      g0[sidx] = make_float4(__uint_as_float(u0.x), __uint_as_float(u0.y), __uint_as_float(u0.z),
                             __uint_as_float(u0.w));
      g1[sidx] = make_float4(__uint_as_float(u1.x), __uint_as_float(u1.y), __uint_as_float(u1.z),
                             __uint_as_float(u1.w));
    };
    // right-hand-side buffers: zero past mx for the whole box
    for (int e = tid; e < 2 * NTM * 16; e += blockDim.x) (&vbuf[0][0])[e] = make_float2(0.f, 0.f);
    __syncthreads();
    if (red) {  // tile source of row j0
      const bool row_in = j0 >= bd.ty0 && j0 < bd.ty1;
      const double2 s0 = (row_in && col_in) ? rbase[(int64_t)j0 * ngx] : make_double2(0.0, 0.0);
      vbuf[0][ra] = make_float2((float)s0.x, (float)s0.y);
    }
    // prefetched inputs of the coming step's reduction
    float2 py = make_float2(0.f, 0.f);
    bool py_use = false;
    double2 ps = rbase[(int64_t)min(j0 + 1, my - 1) * ngx];
    bool ps_row = (j0 + 1 >= bd.ty0) && (j0 + 1 < bd.ty1);
    double2 pih = t.ihy[nf > 1 ? j0 + 1 : j0];
    {
      const __amdgpu_buffer_rsrc_t r0s = block_rsrc(j0, true);
#pragma unroll
      for (int sidx = 0; sidx < TMAX; ++sidx) load_tile(r0s, sidx);
    }
    __syncthreads();
    int cur = 0;
#pragma unroll 1
    for (int st = 0; st < T; ++st) {
      const bool fwd = st < nf;
      const int j = __builtin_amdgcn_readfirstlane(row_of(st));
      const bool more = st + 1 < T;
      const int jn = __builtin_amdgcn_readfirstlane(row_of(more ? st + 1 : st));
      const float2* vb = vbuf[cur];
      // the next block streams in tile by tile behind this step's FMAs: each
      // tile slot is reloaded as soon as its values have been used
      const __amdgpu_buffer_rsrc_t nsrc = block_rsrc(jn, more);
      float2 ca0[4], ca1[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        ca0[c] = make_float2(0.f, 0.f);
        ca1[c] = make_float2(0.f, 0.f);
      }
#pragma unroll
      for (int sidx = 0; sidx < TMAX; ++sidx) {
        int I, J;
        tile_IJ(sidx, I, J);
        const bool valid = sidx < ntw;
        const int Ic = valid ? I : 0, Jc = valid ? J : 0;
        const float2 t0 = make_float2(g0[sidx].x, g0[sidx].y), t1 = make_float2(g0[sidx].z, g0[sidx].w);
        const float2 t2 = make_float2(g1[sidx].x, g1[sidx].y), t3 = make_float2(g1[sidx].z, g1[sidx].w);
        const float2* vJ = vb + 16 * Jc + 4 * lq;
        float2 rp = make_float2(0.f, 0.f);
        rp = f2fma(t0, vJ[0], rp);
        rp = f2fma(t1, vJ[1], rp);
        rp = f2fma(t2, vJ[2], rp);
        rp = f2fma(t3, vJ[3], rp);
        rp.x += __shfl_xor(rp.x, 16, 64);
        rp.y += __shfl_xor(rp.y, 16, 64);
        rp.x += __shfl_xor(rp.x, 32, 64);
        rp.y += __shfl_xor(rp.y, 32, 64);
        if (valid && lq == 0) rowpart[Jc][Ic][lr] = rp;
        if (valid && I < J) {  // column part T^T v_I into block J (J0 or J1)
          const float2 vI = vb[16 * Ic + lr];
          if (sidx < n0) {
            ca0[0] = f2fma(t0, vI, ca0[0]);
            ca0[1] = f2fma(t1, vI, ca0[1]);
            ca0[2] = f2fma(t2, vI, ca0[2]);
            ca0[3] = f2fma(t3, vI, ca0[3]);
          } else {
            ca1[0] = f2fma(t0, vI, ca1[0]);
            ca1[1] = f2fma(t1, vI, ca1[1]);
            ca1[2] = f2fma(t2, vI, ca1[2]);
            ca1[3] = f2fma(t3, vI, ca1[3]);
          }
        }
        __builtin_amdgcn_sched_barrier(0);
        load_tile(nsrc, sidx);
        __builtin_amdgcn_sched_barrier(0);
      }
      // column parts: sum over the 16 rows (lanes with equal q)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) {
          ca0[c].x += __shfl_xor(ca0[c].x, o, 64);
          ca0[c].y += __shfl_xor(ca0[c].y, o, 64);
          ca1[c].x += __shfl_xor(ca1[c].x, o, 64);
          ca1[c].y += __shfl_xor(ca1[c].y, o, 64);
        }
      }
      if (wactive && lr == 0) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          colpart[J0][4 * lq + c] = ca0[c];
          if (J1 != J0) colpart[J1][4 * lq + c] = ca1[c];
        }
      }
      // inputs of this step's reduction (loaded one step earlier)
      const float2 cy = py_use ? py : make_float2(0.f, 0.f);
      const double2 cs = (ps_row && col_in) ? ps : make_double2(0.0, 0.0);
      const double2 ih = pih;
      // small inputs of the next step's reduction
      __builtin_amdgcn_sched_barrier(0);
      {
        py = Xa[(int64_t)jn * mx];
        py_use = more && st + 1 >= nf && jn >= j0;
        const bool nn_fwd = st + 2 < nf;
        ps = rbase[(int64_t)min(jn + 1, my - 1) * ngx];
        ps_row = nn_fwd && (jn + 1 >= bd.ty0) && (jn + 1 < bd.ty1);
        pih = t.ihy[nn_fwd ? jn + 1 : jn];
      }
      lds_barrier();
      if (red) {
        const int I = ra >> 4, rr = ra & 15;
        float2 y = colpart[I][rr];  // zero for block 0 (no tiles above it)
        for (int J = I; J < nt; ++J) {
          const float2 v = rowpart[J][I][rr];
          y.x += v.x;
          y.y += v.y;
        }
        const float2 x = fwd ? y : make_float2(cy.x - y.x, cy.y - y.y);
        Xa[(int64_t)j * mx] = x;
        if (more) {
          const float2 ihf = make_float2((float)ih.x, (float)ih.y);
          const float2 c0 = cmul(cmul(axa, ihf), x);
          const float sg = (st + 1 < nf) ? -1.f : 1.f;
          vbuf[cur ^ 1][ra] = make_float2((float)cs.x + sg * c0.x, (float)cs.y + sg * c0.y);
        }
      }
      cur ^= 1;
      lds_barrier();
    }
  }
}

// ---------------------------------------------------------------- gather
template <typename CI, typename CO, bool SMOOTH>
__global__ __launch_bounds__(256) void gather_kernel(const BoxDesc* __restrict__ desc,
                                                     const AxisCover* __restrict__ cx,
                                                     const AxisCover* __restrict__ cy,
                                                     const CI* __restrict__ X, CO* __restrict__ z,
                                                     int ngx, int ngy, int nbx,
                                                     const double2* __restrict__ wx,
                                                     const double2* __restrict__ wy) {
  const int gx = blockIdx.x * blockDim.x + threadIdx.x;
  const int gy = blockIdx.y;
  if (gx >= ngx || gy >= ngy) return;
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
  double sr = 0.0, si = 0.0;
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    if (bys[a] < 0) continue;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      if (bxs[b] < 0) continue;
      const BoxDesc& bd = desc[bys[a] * nbx + bxs[b]];
      const double2 v = to_d(X[bd.x_off + (int64_t)lys[a] * bd.mx + lxs[b]]);
      if (SMOOTH) {
        const double w = wys[a] * wxs[b];
        sr += w * v.x;
        si += w * v.y;
      } else {
        sr += v.x;
        si += v.y;
      }
    }
  }
  z[(int64_t)gy * ngx + gx] = mk<CO>(sr, si);
}

// ---------------------------------------------------------------- matvec
// gtab: ax[ngx], ihx[ngx+1], ay[ngy], ihy[ngy+1]; ghost neighbours are zero.
// Coefficients of the symmetric 5-point row of node (gx, gy).
struct Stencil {
  double2 cw, ce, cs, cn, kj;  // kj = k^2 ax ay
};
__device__ __forceinline__ Stencil stencil_at(const double2* __restrict__ gtab,
                                              const double* __restrict__ k2, int gx, int gy,
                                              int ngx, int ngy) {
  const double2* ax = gtab;
  const double2* ihx = ax + ngx;
  const double2* ay = ihx + ngx + 1;
  const double2* ihy = ay + ngy;
  const double2 a1 = ax[gx], a2 = ay[gy];
  Stencil c;
  c.cw = dmul(a2, ihx[gx]);
  c.ce = dmul(a2, ihx[gx + 1]);
  c.cs = dmul(a1, ihy[gy]);
  c.cn = dmul(a1, ihy[gy + 1]);
  const double2 jac = dmul(a1, a2);
  const double kk = k2[(int64_t)gy * ngx + gx];
  c.kj = make_double2(kk * jac.x, kk * jac.y);
  return c;
}
// (M u)(node) from the node's value u and its west/east/south/north
// neighbours (zero outside the grid).
__device__ __forceinline__ double2 stencil_sum(const Stencil& c, double2 u, double2 uw, double2 ue,
                                               double2 us, double2 un) {
  double2 s = dmul(c.ce, make_double2(ue.x - u.x, ue.y - u.y));
  double2 t2 = dmul(c.cw, make_double2(uw.x - u.x, uw.y - u.y));
  s.x += t2.x; s.y += t2.y;
  t2 = dmul(c.cn, make_double2(un.x - u.x, un.y - u.y));
  s.x += t2.x; s.y += t2.y;
  t2 = dmul(c.cs, make_double2(us.x - u.x, us.y - u.y));
  s.x += t2.x; s.y += t2.y;
  t2 = dmul(c.kj, u);
  s.x += t2.x; s.y += t2.y;
  return s;
}
template <typename CI>
__device__ __forceinline__ double2 stencil_apply(const Stencil& c, const CI* __restrict__ x,
                                                 int64_t idx, int gx, int gy, int ngx, int ngy) {
  const double2 u = to_d(x[idx]);
  const double2 uw = gx > 0 ? to_d(x[idx - 1]) : make_double2(0.0, 0.0);
  const double2 ue = gx + 1 < ngx ? to_d(x[idx + 1]) : make_double2(0.0, 0.0);
  const double2 us = gy > 0 ? to_d(x[idx - ngx]) : make_double2(0.0, 0.0);
  const double2 un = gy + 1 < ngy ? to_d(x[idx + ngx]) : make_double2(0.0, 0.0);
  return stencil_sum(c, u, uw, ue, us, un);
}

template <typename CI>
__global__ __launch_bounds__(256) void matvec_kernel(const double2* __restrict__ gtab,
                                                     const double* __restrict__ k2,
                                                     const CI* __restrict__ x,
                                                     const double2* __restrict__ sub_from,
                                                     double2* __restrict__ y, int ngx, int ngy) {
  const int gx = blockIdx.x * blockDim.x + threadIdx.x;
  const int gy = blockIdx.y;
  if (gx >= ngx) return;
  const int64_t idx = (int64_t)gy * ngx + gx;
  const Stencil c = stencil_at(gtab, k2, gx, gy, ngx, ngy);
  double2 s = stencil_apply(c, x, idx, gx, gy, ngx, ngy);
  if (sub_from) {
    const double2 b = sub_from[idx];
    s = make_double2(b.x - s.x, b.y - s.y);
  }
  y[idx] = s;
}

// ---------------------------------------------------------------- krylov
constexpr int KT = 256;  // threads per Krylov block
constexpr int KE = 8;    // elements per thread
constexpr int KCHUNK = KT * KE;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
// Block sum in a fixed order; result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
  return s;
}

// Stencil tiles.  Krylov kernels that form w = M z themselves cover the grid
// with tiles of SC columns x R rows, one thread per column and R rows per
// thread, so each z row is read once per tile (plus one halo row above and
// below) and the x-neighbours come from the same cache lines.  A launch runs
// every (tile, right-hand side) pair; logical block L = (tile, rhs) with the
// right-hand side fastest.  Workgroups are handed to the 8 XCDs in turn, so
// xcd_order() gives each XCD a contiguous range of logical blocks: the
// right-hand sides of one tile (which share its coefficient rows) and
// vertically adjacent tiles meet in one L2.
constexpr int SC = KT, NXCD = 8;
constexpr int SR = 8;   // rows per thread of the lighter tile kernels
constexpr int SR4 = 4;  // rows per thread where more vectors stay in registers
__device__ __forceinline__ int xcd_order(int b, int nb) {
  const int per = nb / NXCD;
  if (b >= per * NXCD) return b;
  return (b % NXCD) * per + b / NXCD;
}
struct TileAt {
  int y, t;     // right-hand side, tile
  int gx, gy0;  // this thread's column, the tile's first row
};
template <int R>
__device__ __forceinline__ TileAt tile_at(int nrhs, int ntx) {
  const int L = xcd_order(blockIdx.x, gridDim.x);
  TileAt a;
  a.y = L % nrhs;
  a.t = L / nrhs;
  a.gx = (a.t % ntx) * SC + threadIdx.x;
  a.gy0 = (a.t / ntx) * R;
  return a;
}
// w[r] = (M z)(gx, gy0 + r) for r < R, zero where the node is outside the
// grid; idx[r] = a valid index for loads at that node (clamped to the grid).
// The arithmetic is stencil_apply's, so results equal the plain matvec's.
template <int R, typename CZ>
__device__ __forceinline__ void stencil_tile(const double2* __restrict__ gtab,
                                             const double* __restrict__ k2,
                                             const CZ* __restrict__ z, int gx, int gy0, int ngx,
                                             int ngy, double2 (&w)[R], int64_t (&idx)[R],
                                             bool (&ok)[R]) {
  const double2* ax = gtab;
  const double2* ihx = ax + ngx;
  const double2* ay = ihx + ngx + 1;
  const double2* ihy = ay + ngy;
  const double2 zero = make_double2(0.0, 0.0);
  const int gxc = min(gx, ngx - 1);
  const double2 a1 = ax[gxc], hw = ihx[gxc], he = ihx[gxc + 1];
  const bool okw = gx > 0, oke = gx + 1 < ngx;
  double2 zc[R + 2];  // rows gy0-1 .. gy0+R of column gx
#pragma unroll
  for (int r = 0; r < R + 2; ++r) {
    const int gy = gy0 - 1 + r;
    const int gyc = min(max(gy, 0), ngy - 1);
    const double2 v = to_d(z[(int64_t)gyc * ngx + gxc]);
    zc[r] = (gy >= 0 && gy < ngy) ? v : zero;
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int gy = gy0 + r, gyc = min(gy, ngy - 1);
    const int64_t row = (int64_t)gyc * ngx;
    idx[r] = row + gxc;
    ok[r] = gx < ngx && gy < ngy;
    const double2 uw0 = to_d(z[row + max(gxc - 1, 0)]);
    const double2 ue0 = to_d(z[row + min(gxc + 1, ngx - 1)]);
    const double2 a2 = ay[gyc];
    Stencil c;
    c.cw = dmul(a2, hw);
    c.ce = dmul(a2, he);
    c.cs = dmul(a1, ihy[gyc]);
    c.cn = dmul(a1, ihy[gyc + 1]);
    const double2 jac = dmul(a1, a2);
    const double kk = k2[row + gxc];
    c.kj = make_double2(kk * jac.x, kk * jac.y);
    const double2 v = stencil_sum(c, zc[r + 1], okw ? uw0 : zero, oke ? ue0 : zero, zc[r],
                                  zc[r + 2]);
    w[r] = ok[r] ? v : zero;
  }
}

__global__ __launch_bounds__(KT) void reduce_r_kernel(const double* __restrict__ partial, int nblk,
                                                      double* __restrict__ out) {
  __shared__ double red[KT / 64];
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += KT) s += partial[b];
  const double t = block_sum(s, red);
  if (threadIdx.x == 0) out[0] = sqrt(t);
}

__global__ __launch_bounds__(KT) void norm_partial_kernel(const double2* __restrict__ w, int64_t n,
                                                          double* __restrict__ partial) {
  __shared__ double red[KT / 64];
  const int64_t base = (int64_t)blockIdx.x * KCHUNK + threadIdx.x;
  double s = 0.0;
#pragma unroll
  for (int e = 0; e < KE; ++e) {
    const int64_t i = base + (int64_t)e * KT;
    if (i < n) {
      const double2 a = w[i];
      s = fma(a.x, a.x, s);
      s = fma(a.y, a.y, s);
    }
  }
  const double t = block_sum(s, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

__global__ __launch_bounds__(KT) void scale_kernel(double2* __restrict__ w, int64_t n,
                                                   const double* __restrict__ norm) {
  const double inv = 1.0 / norm[0];
  for (int64_t i = (int64_t)blockIdx.x * KT + threadIdx.x; i < n; i += (int64_t)gridDim.x * KT) {
    double2 a = w[i];
    a.x *= inv;
    a.y *= inv;
    w[i] = a;
  }
}

// x += sum_k Z_k y_k
template <typename CZ>
__global__ __launch_bounds__(KT) void combine_kernel(const CZ* __restrict__ Z, int64_t ldz, int nk,
                                                     const double2* __restrict__ y,
                                                     double2* __restrict__ x, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * KT + threadIdx.x; i < n; i += (int64_t)gridDim.x * KT) {
    double2 acc = x[i];
    for (int k = 0; k < nk; ++k) {
      const double2 a = to_d(Z[(int64_t)k * ldz + i]);
      const double2 c = y[k];
      acc.x = fma(a.x, c.x, acc.x);
      acc.x = fma(-a.y, c.y, acc.x);
      acc.y = fma(a.x, c.y, acc.y);
      acc.y = fma(a.y, c.x, acc.y);
    }
    x[i] = acc;
  }
}

// ------------------------------------------------- batched Arnoldi steps
// Summary slots of a right-hand side (restart m): h1 at 0, h2 at 2(m+1),
// norms at 4m+3 (|w|, |r|), the basis norms nu_0..nu_m (lazy form) after them.
__device__ __forceinline__ double2* ks_h2(double2* sum, int m) { return sum + 2 * (m + 1); }
__device__ __forceinline__ double* ks_norm(double2* sum, int m) {
  return reinterpret_cast<double*>(sum + 4 * m + 3);
}
__device__ __forceinline__ const double* ks_nu(const double2* sum, int m) {
  return reinterpret_cast<const double*>(sum + 4 * m + 4);
}

// Complex64 copy of v at node (gx, gy) into plane `slot` of the owning box's
// source planes.
__device__ __forceinline__ void put_source(const SrcMap& sm, int slot, int gx, int gy, double2 v) {
  const int2 ox = sm.own_x[gx], oy = sm.own_y[gy];
  const int64_t box = (int64_t)oy.x * sm.nbx + ox.x;
  sm.S[(box * BLOCK_RHS + slot) * sm.tr * sm.xw + (int64_t)oy.y * sm.xw + ox.y] =
      make_float2((float)v.x, (float)v.y);
}

// Partial inner products of one chunk: partial[(q*nk + k)*nblk + blk] =
// sum over the chunk of conj(V_k) u_q, with u_0 = w = V_{j+1} and (NR = 2)
// u_1 = v_j, whose own product with V_j reuses the registers instead of a
// second read.
template <int NR>
__global__ __launch_bounds__(KT) void ks_dots_kernel(KSet ks, int64_t n) {
  extern __shared__ double red[];  // [nk][2*NR][KT/64]
  constexpr int NW = KT / 64;
  const int y = blockIdx.y;
  const int j = ks.j[y], nk = j + 1;
  const double2* __restrict__ V = ks.V[y];
  const double2* __restrict__ w0 = V + (int64_t)(j + 1) * n;
  const double2* __restrict__ w1 = V + (int64_t)j * n;
  double2* __restrict__ partial = ks.part[y];
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
  const int64_t base = (int64_t)blockIdx.x * KCHUNK + threadIdx.x;
  double2 wl[NR][KE];
#pragma unroll
  for (int e = 0; e < KE; ++e) {
    const int64_t i = base + (int64_t)e * KT;
    wl[0][e] = i < n ? w0[i] : make_double2(0.0, 0.0);
    if (NR > 1) wl[NR - 1][e] = i < n ? w1[i] : make_double2(0.0, 0.0);
  }
  for (int k = 0; k < nk; ++k) {
    const double2* __restrict__ v = V + (int64_t)k * n;
    const bool last = NR > 1 && k == j;  // V_j is already in registers
    double sr[NR], si[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) sr[q] = si[q] = 0.0;
#pragma unroll
    for (int e = 0; e < KE; ++e) {
      const int64_t i = base + (int64_t)e * KT;
      if (i < n) {
        const double2 a = last ? wl[NR - 1][e] : v[i];
#pragma unroll
        for (int q = 0; q < NR; ++q) {
          sr[q] = fma(a.x, wl[q][e].x, sr[q]);
          sr[q] = fma(a.y, wl[q][e].y, sr[q]);
          si[q] = fma(a.x, wl[q][e].y, si[q]);
          si[q] = fma(-a.y, wl[q][e].x, si[q]);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      const double tr = wave_sum(sr[q]), ti = wave_sum(si[q]);
      if (ln == 0) {
        red[((k * NR + q) * 2 + 0) * NW + wv] = tr;
        red[((k * NR + q) * 2 + 1) * NW + wv] = ti;
      }
    }
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < nk * NR; idx += KT) {
    const int k = idx / NR, q = idx - (idx / NR) * NR;
    double tr = 0.0, ti = 0.0;
    for (int w = 0; w < NW; ++w) {
      tr += red[((k * NR + q) * 2 + 0) * NW + w];
      ti += red[((k * NR + q) * 2 + 1) * NW + w];
    }
    partial[((int64_t)q * nk + k) * gridDim.x + blockIdx.x] = make_double2(tr, ti);
  }
}

// out[k] = sum over blocks of partial[k*nblk + b] for k < NR*(j+1), one block
// per (k, right-hand side); out = summary + out_off.  Lazy form: products
// with W_kk are divided by nu_kk (and those with W_j by nu_j as well).
__global__ __launch_bounds__(KT) void ks_reduce_kernel(KSet ks, int nr, int nblk, int out_off,
                                                       int m) {
  __shared__ double red[KT / 64];
  const int y = blockIdx.y, k = blockIdx.x;
  const int nk = ks.j[y] + 1;
  if (k >= nr * nk) return;
  const double2* __restrict__ partial = ks.part[y];
  double sr = 0.0, si = 0.0;
  for (int b = threadIdx.x; b < nblk; b += KT) {
    const double2 p = partial[(int64_t)k * nblk + b];
    sr += p.x;
    si += p.y;
  }
  const double tr = block_sum(sr, red);
  const double ti = block_sum(si, red);
  if (threadIdx.x == 0) {
    double sc = 1.0;
    if (ks.lazy) {
      const double* nu = ks_nu(ks.sum[y], m);
      const int q = k / nk, kk = k - q * nk;
      sc = 1.0 / nu[kk];
      if (q == 1) sc /= nu[nk - 1];
    }
    ks.sum[y][out_off + k] = make_double2(tr * sc, ti * sc);
  }
}

// Gram coefficients (one block per right-hand side): column j of the Gram
// matrix <- q = h1[nk..2nk), then h2 = 2p - G p with p = h1[0..nk).
__global__ __launch_bounds__(KT) void ks_gram_kernel(KSet ks, int m) {
  const int y = blockIdx.x;
  const int j = ks.j[y], nk = j + 1, ld = m + 1;
  double2* __restrict__ Gm = ks.gram[y];
  const double2* p = ks.sum[y];
  const double2* q = p + nk;
  double2* __restrict__ c = ks_h2(ks.sum[y], m);
  for (int i = threadIdx.x; i < nk; i += KT) Gm[(int64_t)j * ld + i] = q[i];
  __syncthreads();
  for (int i = threadIdx.x; i < nk; i += KT) {
    double2 acc = make_double2(2.0 * p[i].x, 2.0 * p[i].y);
    for (int k = 0; k < nk; ++k) {
      // Gm(i, k): stored in column max(i,k); conjugate when i > k
      double2 g = (i <= k) ? Gm[(int64_t)k * ld + i] : Gm[(int64_t)i * ld + k];
      if (i > k) g.y = -g.y;
      const double2 pk = p[k];
      acc.x -= g.x * pk.x - g.y * pk.y;
      acc.y -= g.x * pk.y + g.y * pk.x;
    }
    c[i] = acc;
  }
}

// w -= sum_k V_k coef_k (coef = summary + coef_off; lazy: W_k coef_k / nu_k);
// with_norm: block partial sums of |w|^2, and w's source planes if sm.S
// (ngx: grid row length, to place node i).
__global__ __launch_bounds__(KT) void ks_update_kernel(KSet ks, int64_t n, int coef_off,
                                                       int with_norm, int m, SrcMap sm, int ngx) {
  __shared__ double red[KT / 64];
  const int y = blockIdx.y;
  const int j = ks.j[y], nk = j + 1;
  const double2* __restrict__ V = ks.V[y];
  double2* __restrict__ w = ks.V[y] + (int64_t)(j + 1) * n;
  const double2* coef = ks.sum[y] + coef_off;
  const double* nu = ks_nu(ks.sum[y], m);
  const int64_t base = (int64_t)blockIdx.x * KCHUNK + threadIdx.x;
  double2 wl[KE];
#pragma unroll
  for (int e = 0; e < KE; ++e) {
    const int64_t i = base + (int64_t)e * KT;
    wl[e] = i < n ? w[i] : make_double2(0.0, 0.0);
  }
  for (int k = 0; k < nk; ++k) {
    double2 c = coef[k];
    if (ks.lazy) {
      const double inv = 1.0 / nu[k];
      c = make_double2(c.x * inv, c.y * inv);
    }
    const double2* __restrict__ v = V + (int64_t)k * n;
#pragma unroll
    for (int e = 0; e < KE; ++e) {
      const int64_t i = base + (int64_t)e * KT;
      if (i < n) {
        const double2 a = v[i];
        wl[e].x = fma(-a.x, c.x, wl[e].x);
        wl[e].x = fma(a.y, c.y, wl[e].x);
        wl[e].y = fma(-a.x, c.y, wl[e].y);
        wl[e].y = fma(-a.y, c.x, wl[e].y);
      }
    }
  }
  double s = 0.0;
  const bool src = with_norm && sm.S != nullptr;
#pragma unroll
  for (int e = 0; e < KE; ++e) {
    const int64_t i = base + (int64_t)e * KT;
    if (i < n) {
      w[i] = wl[e];
      s = fma(wl[e].x, wl[e].x, s);
      s = fma(wl[e].y, wl[e].y, s);
      if (src) {
        const int ii = (int)i;  // grids have < 2^31 nodes
        const int gy = ii / ngx;
        put_source(sm, ks.slot[y], ii - gy * ngx, gy, wl[e]);
      }
    }
  }
  if (with_norm) {
    const double t = block_sum(s, red);
    if (threadIdx.x == 0) ks.npart[y][blockIdx.x] = t;
  }
}

// ks_dots_kernel with w = M z_j formed on the fly over stencil tiles instead
// of read: partial[(q*nk + k)*ntiles + tile].
template <int NR, int R, typename CZ>
__global__ __launch_bounds__(KT) void ks_mvdots_kernel(const double2* __restrict__ gtab,
                                                       const double* __restrict__ k2, KSet ks,
                                                       int ngx, int ngy, int ntx, int ntiles) {
  extern __shared__ double red[];  // [nk][2*NR][KT/64]
  constexpr int NW = KT / 64;
  const TileAt at = tile_at<R>(ks.n, ntx);
  const int y = at.y;
  const int j = ks.j[y], nk = j + 1;
  const int64_t n = (int64_t)ngx * ngy;
  const double2* __restrict__ V = ks.V[y];
  const CZ* __restrict__ z = reinterpret_cast<const CZ*>(ks.Z[y]) + (int64_t)j * n;
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
  double2 wl[NR][R];
  int64_t idx[R];
  bool ok[R];
  stencil_tile(gtab, k2, z, at.gx, at.gy0, ngx, ngy, wl[0], idx, ok);
  if (NR > 1) {
    const double2* __restrict__ vj = V + (int64_t)j * n;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const double2 a = vj[idx[r]];
      wl[NR - 1][r] = ok[r] ? a : make_double2(0.0, 0.0);
    }
  }
  for (int k = 0; k < nk; ++k) {
    const double2* __restrict__ v = V + (int64_t)k * n;
    const bool last = NR > 1 && k == j;  // V_j is already in registers
    double sr[NR], si[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) sr[q] = si[q] = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const double2 a = last ? wl[NR - 1][r] : v[idx[r]];
#pragma unroll
      for (int q = 0; q < NR; ++q) {
        sr[q] = fma(a.x, wl[q][r].x, sr[q]);
        sr[q] = fma(a.y, wl[q][r].y, sr[q]);
        si[q] = fma(a.x, wl[q][r].y, si[q]);
        si[q] = fma(-a.y, wl[q][r].x, si[q]);
      }
    }
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      const double tr = wave_sum(sr[q]), ti = wave_sum(si[q]);
      if (ln == 0) {
        red[((k * NR + q) * 2 + 0) * NW + wv] = tr;
        red[((k * NR + q) * 2 + 1) * NW + wv] = ti;
      }
    }
  }
  __syncthreads();
  double2* __restrict__ partial = ks.part[y];
  for (int i = threadIdx.x; i < nk * NR; i += KT) {
    const int k = i / NR, q = i - (i / NR) * NR;
    double tr = 0.0, ti = 0.0;
    for (int w = 0; w < NW; ++w) {
      tr += red[((k * NR + q) * 2 + 0) * NW + w];
      ti += red[((k * NR + q) * 2 + 1) * NW + w];
    }
    partial[((int64_t)q * nk + k) * ntiles + at.t] = make_double2(tr, ti);
  }
}

// ks_update_kernel with w = M z_j formed on the fly: V_{j+1} = w - sum_k
// coef[k] V_k (lazy: coef[k] / nu_k), with_norm: norm partials per tile (and
// the sources if sm.S).
template <int R, typename CZ>
__global__ __launch_bounds__(KT) void ks_mvupdate_kernel(const double2* __restrict__ gtab,
                                                         const double* __restrict__ k2, KSet ks,
                                                         int coef_off, int with_norm, int m,
                                                         SrcMap sm, int ngx, int ngy, int ntx) {
  __shared__ double red[KT / 64];
  const TileAt at = tile_at<R>(ks.n, ntx);
  const int y = at.y;
  const int j = ks.j[y], nk = j + 1;
  const int64_t n = (int64_t)ngx * ngy;
  const double2* __restrict__ V = ks.V[y];
  double2* __restrict__ w = ks.V[y] + (int64_t)(j + 1) * n;
  const CZ* __restrict__ z = reinterpret_cast<const CZ*>(ks.Z[y]) + (int64_t)j * n;
  const double2* coef = ks.sum[y] + coef_off;
  const double* nu = ks_nu(ks.sum[y], m);
  double2 wl[R];
  int64_t idx[R];
  bool ok[R];
  stencil_tile(gtab, k2, z, at.gx, at.gy0, ngx, ngy, wl, idx, ok);
  for (int k = 0; k < nk; ++k) {
    double2 c = coef[k];
    if (ks.lazy) {
      const double inv = 1.0 / nu[k];
      c = make_double2(c.x * inv, c.y * inv);
    }
    const double2* __restrict__ v = V + (int64_t)k * n;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const double2 a = v[idx[r]];
      wl[r].x = fma(-a.x, c.x, wl[r].x);
      wl[r].x = fma(a.y, c.y, wl[r].x);
      wl[r].y = fma(-a.x, c.y, wl[r].y);
      wl[r].y = fma(-a.y, c.x, wl[r].y);
    }
  }
  double s = 0.0;
  // the last Arnoldi step of a cycle (j + 1 == m, final update): V_m is never
  // read -- the cycle ends with x += Z y and a fresh residual in V_0 -- so
  // only its norm is formed, and neither it nor its sources are stored
  const bool store = !with_norm || j + 1 < m;
  const bool src = with_norm && sm.S != nullptr && store;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (ok[r]) {
      if (store) w[idx[r]] = wl[r];
      s = fma(wl[r].x, wl[r].x, s);
      s = fma(wl[r].y, wl[r].y, s);
      if (src) put_source(sm, ks.slot[y], at.gx, at.gy0 + r, wl[r]);
    }
  }
  if (with_norm) {
    const double t = block_sum(s, red);
    if (threadIdx.x == 0) ks.npart[y][at.t] = t;
  }
}

// norms[slot] = sqrt(sum of the norm partials), one block per right-hand side;
// lazy form: also nu_{j+1} (slot 0, the new Arnoldi vector) or nu_0 (slot 1).
__global__ __launch_bounds__(KT) void ks_norm_kernel(KSet ks, int m, int nblk, int slot) {
  __shared__ double red[KT / 64];
  const int y = blockIdx.x;
  const double* __restrict__ partial = ks.npart[y];
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += KT) s += partial[b];
  const double t = block_sum(s, red);
  if (threadIdx.x == 0) {
    const double nrm = sqrt(t);
    ks_norm(ks.sum[y], m)[slot] = nrm;
    if (ks.lazy) const_cast<double*>(ks_nu(ks.sum[y], m))[slot == 0 ? ks.j[y] + 1 : 0] = nrm;
  }
}

// x += sum_{k <= j} Z_k y_k with y = summary + 3(m+1).
template <typename CZ>
__global__ __launch_bounds__(KT) void ks_combine_kernel(KSet ks, int m, int64_t n) {
  const int y = blockIdx.y;
  const int nk = ks.j[y] + 1;
  const CZ* __restrict__ Z = static_cast<const CZ*>(ks.Z[y]);
  const double2* coef = ks.sum[y] + 3 * (m + 1);
  double2* __restrict__ x = ks.x[y];
  for (int64_t i = (int64_t)blockIdx.x * KT + threadIdx.x; i < n; i += (int64_t)gridDim.x * KT) {
    double2 acc = x[i];
    for (int k = 0; k < nk; ++k) {
      const double2 a = to_d(Z[(int64_t)k * n + i]);
      const double2 c = coef[k];
      acc.x = fma(a.x, c.x, acc.x);
      acc.x = fma(-a.y, c.y, acc.x);
      acc.y = fma(a.x, c.y, acc.y);
      acc.y = fma(a.y, c.x, acc.y);
    }
    x[i] = acc;
  }
}

// V_0 = b - M x (and its source planes if sm.S) over stencil tiles, with the
// norm partials of V_0 per tile.
__global__ __launch_bounds__(KT) void ks_residual_kernel(const double2* __restrict__ gtab,
                                                          const double* __restrict__ k2, KSet ks,
                                                          int ngx, int ngy, int ntx, SrcMap sm) {
  __shared__ double red[KT / 64];
  const TileAt at = tile_at<SR4>(ks.n, ntx);
  const int y = at.y;
  const double2* __restrict__ b = ks.b[y];
  double2* __restrict__ v0 = ks.V[y];
  double2 wl[SR4];
  int64_t idx[SR4];
  bool ok[SR4];
  stencil_tile(gtab, k2, static_cast<const double2*>(ks.x[y]), at.gx, at.gy0, ngx, ngy, wl, idx,
               ok);
  double s = 0.0;
#pragma unroll
  for (int r = 0; r < SR4; ++r) {
    const double2 bb = b[idx[r]];
    if (ok[r]) {
      const double2 rr = make_double2(bb.x - wl[r].x, bb.y - wl[r].y);
      v0[idx[r]] = rr;
      s = fma(rr.x, rr.x, s);
      s = fma(rr.y, rr.y, s);
      if (sm.S) put_source(sm, ks.slot[y], at.gx, at.gy0 + r, rr);
    }
  }
  const double t = block_sum(s, red);
  if (threadIdx.x == 0) ks.npart[y][at.t] = t;
}

__global__ __launch_bounds__(KT) void ks_scale_kernel(KSet ks, int m, int64_t n, int restart) {
  const int y = blockIdx.y;
  double2* __restrict__ w = ks.V[y] + (restart ? 0 : (int64_t)(ks.j[y] + 1) * n);
  const double inv = 1.0 / ks_norm(ks.sum[y], m)[restart ? 1 : 0];
  for (int64_t i = (int64_t)blockIdx.x * KT + threadIdx.x; i < n; i += (int64_t)gridDim.x * KT) {
    double2 a = w[i];
    a.x *= inv;
    a.y *= inv;
    w[i] = a;
  }
}

__global__ __launch_bounds__(256) void zero_kernel(uint4* __restrict__ p, size_t n16) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += (size_t)gridDim.x * 256)
    p[i] = make_uint4(0, 0, 0, 0);
}

inline int grid_for(int64_t n, int per_block) {
  int64_t g = (n + per_block - 1) / per_block;
  if (g > 65535 * 16) g = 65535 * 16;
  return (int)(g < 1 ? 1 : g);
}

}  // namespace

// ---------------------------------------------------------------- wrappers
template <typename C>
static hipError_t factor_launch(const BoxDesc* d, const double2* ltab, const double* k2, int ngx,
                                C* G, int nboxes, int max_m, float2* pivstat, hipStream_t s) {
  const size_t lds = sizeof(C) * (FB * FB + 3 * (size_t)FB * max_m);
  hipLaunchKernelGGL(factor_gj_kernel<C>, dim3(nboxes), dim3(512), lds, s, d, ltab, k2, ngx, G,
                     nboxes, max_m, static_cast<C*>(nullptr), (int64_t)0, 0, pivstat);
  return hipGetLastError();
}
hipError_t launch_factor_c128(const BoxDesc* d, const double2* ltab, const double* k2, int ngx,
                              double2* G, int nboxes, int max_m, float2* pivstat, hipStream_t s) {
  return factor_launch<double2>(d, ltab, k2, ngx, G, nboxes, max_m, pivstat, s);
}
hipError_t launch_factor_c64(const BoxDesc* d, const double2* ltab, const double* k2, int ngx,
                             float2* G, int nboxes, int max_m, float2* pivstat, hipStream_t s) {
  return factor_launch<float2>(d, ltab, k2, ngx, G, nboxes, max_m, pivstat, s);
}
// MFMA path for boxes up to 16 * MF_NT wide.  ws == nullptr: dense format,
// in place; otherwise symmetric-packed output with `slots` workgroups, each
// owning ws_stride entries of ws as its working matrix.
hipError_t launch_factor_c64_mfma(const BoxDesc* d, const double2* ltab, const double* k2,
                                  int ngx, float2* G, int nboxes, int max_m, float2* ws,
                                  int64_t ws_stride, int slots, float2* pivstat, hipStream_t s) {
  if (max_m > 16 * MF_NT) return hipErrorInvalidValue;
  const int grid = ws ? min(nboxes, slots) : nboxes;
  hipLaunchKernelGGL(factor_mfma_kernel, dim3(grid), dim3(64 * MF_WAVES), 0, s, d, ltab, k2, ngx,
                     G, nboxes, ws, ws_stride, ws ? 1 : 0, pivstat);
  return hipGetLastError();
}
// Register-resident MFMA factor for boxes up to 16 * RF_NT wide (packed or
// dense output, one workgroup per box).
hipError_t launch_factor_c64_mfma_regs(const BoxDesc* d, const double2* ltab, const double* k2,
                                       int ngx, float2* G, int nboxes, int max_m, bool packed,
                                       float2* pivstat, hipStream_t s) {
  if (max_m > 16 * RF_NT) return hipErrorInvalidValue;
  hipLaunchKernelGGL(factor_mfma_regs_kernel, dim3(nboxes), dim3(64 * RF_WAVES), 0, s, d, ltab,
                     k2, ngx, G, packed ? 1 : 0, pivstat);
  return hipGetLastError();
}
// Symmetric-elimination register-resident MFMA factor for boxes up to
// 16 * SF_NT wide (packed or dense output, one workgroup per box).
hipError_t launch_factor_c64_sym_regs(const BoxDesc* d, const double2* ltab, const double* k2,
                                      int ngx, float2* G, int nboxes, int max_m, bool packed,
                                      float2* pivstat, hipStream_t s) {
  if (max_m > 16 * SF_NT) return hipErrorInvalidValue;
  hipLaunchKernelGGL(factor_sym_regs_kernel, dim3(nboxes), dim3(64 * SF_WAVES), 0, s, d, ltab,
                     k2, ngx, G, packed ? 1 : 0, pivstat);
  return hipGetLastError();
}
hipError_t launch_factor_c64_packed(const BoxDesc* d, const double2* ltab, const double* k2,
                                    int ngx, float2* G, int nboxes, int max_m, float2* ws,
                                    int64_t ws_stride, int slots, float2* pivstat, hipStream_t s) {
  const size_t lds = sizeof(float2) * (FB * FB + 3 * (size_t)FB * max_m);
  hipLaunchKernelGGL(factor_gj_kernel<float2>, dim3(min(nboxes, slots)), dim3(512), lds, s, d, ltab,
                     k2, ngx, G, nboxes, max_m, ws, ws_stride, 1, pivstat);
  return hipGetLastError();
}
// Symmetric-packed complex64 sweep; boxes up to 256 wide.  two_per_cu: build
// with a register cap that lets two workgroups (boxes) share a CU.
hipError_t describe_sweep_c64_packed(KLaunch& k, const BoxDesc* d, const double2* ltab,
                                     const float2* G, float2* X, const double2* r, int ngx,
                                     int nboxes, int max_m, bool two_per_cu) {
  const int nt = (max_m + 15) / 16;
  if (nt > 16) return hipErrorInvalidValue;
  k = KLaunch{};
  if (nt <= 7)
    k.func = two_per_cu ? reinterpret_cast<const void*>(&sweep64_sym_kernel<8, 3>)
                        : reinterpret_cast<const void*>(&sweep64_sym_kernel<8, 1>);
  else if (nt <= 11)
    k.func = two_per_cu ? reinterpret_cast<const void*>(&sweep64_sym_kernel<12, 3>)
                        : reinterpret_cast<const void*>(&sweep64_sym_kernel<12, 1>);
  else
    k.func = reinterpret_cast<const void*>(&sweep64_sym_kernel<17, 1>);
  k.grid = dim3(nboxes);
  k.block = dim3(64 * ((nt + 1) / 2));
  k.push(d);
  k.push(ltab);
  k.push(G);
  k.push(X);
  k.push(r);
  k.push(ngx);
  k.push(nboxes);
  return hipSuccess;
}

template <typename C>
static void sweep_generic(KLaunch& k, const BoxDesc* d, const double2* ltab, const C* G, C* X,
                          const double2* r, int ngx, int nboxes, int threads, int max_m) {
  k = KLaunch{};
  k.func = reinterpret_cast<const void*>(&sweep_kernel<C>);
  k.grid = dim3(nboxes);
  k.block = dim3(threads);
  k.shmem = (unsigned)(sizeof(C) * (2 * (size_t)max_m + 2 * (size_t)threads));
  k.push(d);
  k.push(ltab);
  k.push(G);
  k.push(X);
  k.push(r);
  k.push(ngx);
  k.push(nboxes);
  k.push(max_m);
}
// threads >= max_m (every row has a reducing thread).
hipError_t describe_sweep_c128(KLaunch& k, const BoxDesc* d, const double2* ltab,
                               const double2* G, double2* X, const double2* r, int ngx,
                               int nboxes, int threads, int max_m) {
  sweep_generic<double2>(k, d, ltab, G, X, r, ngx, nboxes, threads, max_m);
  return hipSuccess;
}
// complex64: wave-structured kernel for boxes up to 192 nodes wide (16 rows per
// wave, <= 12 waves, LMAX = 8 * waves / 4 column pairs per lane); wider boxes
// use the generic kernel.
hipError_t describe_sweep_c64(KLaunch& k, const BoxDesc* d, const double2* ltab, const float2* G,
                              float2* X, const double2* r, int ngx, int nboxes, int threads,
                              int max_m, bool generic) {
  if (max_m > 192 || generic) {
    sweep_generic<float2>(k, d, ltab, G, X, r, ngx, nboxes, threads, max_m);
    return hipSuccess;
  }
  // waves = LMAX / 2 of the chosen variant (16 rows per wave, 8 columns groups)
  const int lmax = max_m <= 96 ? 12 : max_m <= 128 ? 16 : max_m <= 176 ? 22 : 24;
  k = KLaunch{};
  k.func = lmax == 12   ? reinterpret_cast<const void*>(&sweep64_kernel<12>)
           : lmax == 16 ? reinterpret_cast<const void*>(&sweep64_kernel<16>)
           : lmax == 22 ? reinterpret_cast<const void*>(&sweep64_kernel<22>)
                        : reinterpret_cast<const void*>(&sweep64_kernel<24>);
  k.grid = dim3(nboxes);
  k.block = dim3(64 * (lmax / 2));
  k.shmem = (unsigned)(sizeof(float2) * 2 * (size_t)max_m);
  k.push(d);
  k.push(ltab);
  k.push(G);
  k.push(X);
  k.push(r);
  k.push(ngx);
  k.push(nboxes);
  k.push(max_m);
  return hipSuccess;
}

template <typename CI, typename CO>
static hipError_t gather_describe(KLaunch& k, const BoxDesc* d, const AxisCover* cx,
                                  const AxisCover* cy, const CI* X, CO* z, int ngx, int ngy,
                                  int nbx, const double2* wx, const double2* wy) {
  k = KLaunch{};
  k.func = wx ? reinterpret_cast<const void*>(&gather_kernel<CI, CO, true>)
              : reinterpret_cast<const void*>(&gather_kernel<CI, CO, false>);
  k.grid = dim3((ngx + 255) / 256, ngy);
  k.block = dim3(256);
  k.push(d);
  k.push(cx);
  k.push(cy);
  k.push(X);
  k.push(z);
  k.push(ngx);
  k.push(ngy);
  k.push(nbx);
  k.push(wx);
  k.push(wy);
  return hipSuccess;
}
hipError_t describe_gather_c128_to_c128(KLaunch& k, const BoxDesc* d, const AxisCover* cx,
                                        const AxisCover* cy, const double2* X, double2* z,
                                        int ngx, int ngy, int nbx, const double2* wx,
                                        const double2* wy) {
  return gather_describe(k, d, cx, cy, X, z, ngx, ngy, nbx, wx, wy);
}
hipError_t describe_gather_c64_to_c128(KLaunch& k, const BoxDesc* d, const AxisCover* cx,
                                       const AxisCover* cy, const float2* X, double2* z, int ngx,
                                       int ngy, int nbx, const double2* wx, const double2* wy) {
  return gather_describe(k, d, cx, cy, X, z, ngx, ngy, nbx, wx, wy);
}
hipError_t describe_gather_c64_to_c64(KLaunch& k, const BoxDesc* d, const AxisCover* cx,
                                      const AxisCover* cy, const float2* X, float2* z, int ngx,
                                      int ngy, int nbx, const double2* wx, const double2* wy) {
  return gather_describe(k, d, cx, cy, X, z, ngx, ngy, nbx, wx, wy);
}

template <typename CI>
static hipError_t matvec_launch(const double2* gtab, const double* k2, const CI* x,
                                const double2* sub_from, double2* y, int ngx, int ngy,
                                hipStream_t s) {
  dim3 grid((ngx + 255) / 256, ngy);
  hipLaunchKernelGGL(matvec_kernel<CI>, grid, dim3(256), 0, s, gtab, k2, x, sub_from, y, ngx, ngy);
  return hipGetLastError();
}
hipError_t launch_matvec_c128(const double2* gtab, const double* k2, const double2* x,
                              const double2* sub_from, double2* y, int ngx, int ngy,
                              hipStream_t s) {
  return matvec_launch(gtab, k2, x, sub_from, y, ngx, ngy, s);
}
hipError_t launch_matvec_c64in(const double2* gtab, const double* k2, const float2* x,
                               const double2* sub_from, double2* y, int ngx, int ngy,
                               hipStream_t s) {
  return matvec_launch(gtab, k2, x, sub_from, y, ngx, ngy, s);
}

int krylov_blocks(int64_t n) { return (int)((n + KCHUNK - 1) / KCHUNK); }

template <typename CZ>
__global__ __launch_bounds__(KT) void add_to_kernel(const CZ* __restrict__ z,
                                                    double2* __restrict__ x, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * KT + threadIdx.x; i < n; i += (int64_t)gridDim.x * KT) {
    const double2 a = to_d(z[i]);
    double2 b = x[i];
    b.x += a.x;
    b.y += a.y;
    x[i] = b;
  }
}
hipError_t launch_add_c64(const float2* z, double2* x, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(add_to_kernel<float2>, dim3(grid_for(n, KT * 4)), dim3(KT), 0, s, z, x, n);
  return hipGetLastError();
}
hipError_t launch_add_c128(const double2* z, double2* x, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(add_to_kernel<double2>, dim3(grid_for(n, KT * 4)), dim3(KT), 0, s, z, x, n);
  return hipGetLastError();
}
hipError_t launch_norm(const double2* w, int64_t n, double* partial, double* out, hipStream_t s) {
  const int nblk = krylov_blocks(n);
  hipLaunchKernelGGL(norm_partial_kernel, dim3(nblk), dim3(KT), 0, s, w, n, partial);
  hipLaunchKernelGGL(reduce_r_kernel, dim3(1), dim3(KT), 0, s, partial, nblk, out);
  return hipGetLastError();
}
hipError_t launch_scale(double2* w, int64_t n, const double* norm, hipStream_t s) {
  hipLaunchKernelGGL(scale_kernel, dim3(grid_for(n, KT * 4)), dim3(KT), 0, s, w, n, norm);
  return hipGetLastError();
}
hipError_t launch_combine_c128(const double2* Z, int64_t ldz, int nk, const double2* y,
                               double2* x, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(combine_kernel<double2>, dim3(grid_for(n, KT * 4)), dim3(KT), 0, s, Z, ldz,
                     nk, y, x, n);
  return hipGetLastError();
}
hipError_t launch_combine_c64(const float2* Z, int64_t ldz, int nk, const double2* y, double2* x,
                              int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(combine_kernel<float2>, dim3(grid_for(n, KT * 4)), dim3(KT), 0, s, Z, ldz,
                     nk, y, x, n);
  return hipGetLastError();
}
static int ks_max_nk(const KSet& ks) {
  int nk = 1;
  for (int y = 0; y < ks.n; ++y) nk = max(nk, ks.j[y] + 1);
  return nk;
}
static int tiles_x(int ngx) { return (ngx + SC - 1) / SC; }
static int stencil_tiles(int ngx, int ngy, int rows) {
  return tiles_x(ngx) * ((ngy + rows - 1) / rows);
}
int krylov_partials(int ngx, int ngy) {
  return max(krylov_blocks((int64_t)ngx * ngy), stencil_tiles(ngx, ngy, SR4));
}
// Rows per thread of the dot-product kernel: 4 when w and v_j both stay in
// registers (NR = 2), else 8.
template <int NR>
constexpr int dots_rows() { return NR > 1 ? SR4 : SR; }
template <int NR>
static int mvdots(const KSet& ks, const Op& op, size_t lds, hipStream_t s) {
  constexpr int R = dots_rows<NR>();
  const int ntx = tiles_x(op.ngx), nt = stencil_tiles(op.ngx, op.ngy, R);
  const dim3 g(nt * ks.n);
  if (op.z_c64)
    hipLaunchKernelGGL((ks_mvdots_kernel<NR, R, float2>), g, dim3(KT), lds, s, op.gtab, op.k2,
                       ks, op.ngx, op.ngy, ntx, nt);
  else
    hipLaunchKernelGGL((ks_mvdots_kernel<NR, R, double2>), g, dim3(KT), lds, s, op.gtab, op.k2,
                       ks, op.ngx, op.ngy, ntx, nt);
  return nt;
}
static int mvupdate(const KSet& ks, const Op& op, int coef_off, int with_norm, int m,
                    const SrcMap& sm, hipStream_t s) {
  constexpr int UR = SR;
  const int ntx = tiles_x(op.ngx), nt = stencil_tiles(op.ngx, op.ngy, UR);
  const dim3 g(nt * ks.n);
  if (op.z_c64)
    hipLaunchKernelGGL((ks_mvupdate_kernel<UR, float2>), g, dim3(KT), 0, s, op.gtab, op.k2, ks,
                       coef_off, with_norm, m, sm, op.ngx, op.ngy, ntx);
  else
    hipLaunchKernelGGL((ks_mvupdate_kernel<UR, double2>), g, dim3(KT), 0, s, op.gtab, op.k2, ks,
                       coef_off, with_norm, m, sm, op.ngx, op.ngy, ntx);
  return nt;
}
hipError_t launch_arnoldi_gram(const KSet& ks, int m, const Op& op, const SrcMap& sm,
                               hipStream_t s) {
  if (ks.n < 1 || ks.n > BLOCK_RHS) return hipErrorInvalidValue;
  const int nk = ks_max_nk(ks);
  const size_t lds = sizeof(double) * 4 * (size_t)nk * (KT / 64);
  const int nd = mvdots<2>(ks, op, lds, s);
  hipLaunchKernelGGL(ks_reduce_kernel, dim3(2 * nk, ks.n), dim3(KT), 0, s, ks, 2, nd, 0, m);
  hipLaunchKernelGGL(ks_gram_kernel, dim3(ks.n), dim3(KT), 0, s, ks, m);
  const int nu = mvupdate(ks, op, 2 * (m + 1), 1, m, sm, s);
  hipLaunchKernelGGL(ks_norm_kernel, dim3(ks.n), dim3(KT), 0, s, ks, m, nu, 0);
  return hipGetLastError();
}
hipError_t launch_arnoldi_cgs2(const KSet& ks, int m, const Op& op, const SrcMap& sm,
                               hipStream_t s) {
  if (ks.n < 1 || ks.n > BLOCK_RHS) return hipErrorInvalidValue;
  const int64_t n = (int64_t)op.ngx * op.ngy;
  const int nblk = krylov_blocks(n), nk = ks_max_nk(ks);
  const size_t lds = sizeof(double) * 2 * (size_t)nk * (KT / 64);
  const int h2 = 2 * (m + 1);
  // first pass from M z_j (V_{j+1} = w - V h1), second pass on the stored V_{j+1}
  const int nd = mvdots<1>(ks, op, lds, s);
  hipLaunchKernelGGL(ks_reduce_kernel, dim3(nk, ks.n), dim3(KT), 0, s, ks, 1, nd, 0, m);
  mvupdate(ks, op, 0, 0, m, sm, s);
  hipLaunchKernelGGL(ks_dots_kernel<1>, dim3(nblk, ks.n), dim3(KT), lds, s, ks, n);
  hipLaunchKernelGGL(ks_reduce_kernel, dim3(nk, ks.n), dim3(KT), 0, s, ks, 1, nblk, h2, m);
  hipLaunchKernelGGL(ks_update_kernel, dim3(nblk, ks.n), dim3(KT), 0, s, ks, n, h2, 1, m, sm,
                     op.ngx);
  hipLaunchKernelGGL(ks_norm_kernel, dim3(ks.n), dim3(KT), 0, s, ks, m, nblk, 0);
  return hipGetLastError();
}
hipError_t launch_arnoldi_scale(const KSet& ks, int m, int64_t n, int restart, hipStream_t s) {
  if (ks.n < 1 || ks.n > BLOCK_RHS) return hipErrorInvalidValue;
  hipLaunchKernelGGL(ks_scale_kernel, dim3(grid_for(n, KT * 4), ks.n), dim3(KT), 0, s, ks, m, n,
                     restart);
  return hipGetLastError();
}
hipError_t launch_combine(const KSet& ks, int m, int64_t n, bool z_c64, hipStream_t s) {
  if (ks.n < 1 || ks.n > BLOCK_RHS) return hipErrorInvalidValue;
  const dim3 g(grid_for(n, KT * 4), ks.n);
  if (z_c64)
    hipLaunchKernelGGL(ks_combine_kernel<float2>, g, dim3(KT), 0, s, ks, m, n);
  else
    hipLaunchKernelGGL(ks_combine_kernel<double2>, g, dim3(KT), 0, s, ks, m, n);
  return hipGetLastError();
}
hipError_t launch_residual(const KSet& ks, int m, const double2* gtab, const double* k2,
                           int ngx, int ngy, const SrcMap& sm, hipStream_t s) {
  if (ks.n < 1 || ks.n > BLOCK_RHS) return hipErrorInvalidValue;
  const int nt = stencil_tiles(ngx, ngy, SR4);
  hipLaunchKernelGGL(ks_residual_kernel, dim3(nt * ks.n), dim3(KT), 0, s, gtab, k2, ks, ngx, ngy,
                     tiles_x(ngx), sm);
  hipLaunchKernelGGL(ks_norm_kernel, dim3(ks.n), dim3(KT), 0, s, ks, m, nt, 1);
  return hipGetLastError();
}
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
  const size_t n16 = bytes / 16;
  if (n16 == 0) return hipSuccess;
  hipLaunchKernelGGL(zero_kernel, dim3(grid_for((int64_t)n16, 256 * 4)), dim3(256), 0, s,
                     reinterpret_cast<uint4*>(p), n16);
  return hipGetLastError();
}

}  // namespace hddm
