// gfx950 kernels of the block form of the one-step preconditioner (Leng & Ju,
// Sec. 2 eq. pc): up to 16 right-hand sides share every read of the local
// factors, so each step of the two sweeps is a complex GEMM
// G_j [mx x mx] x V_j [mx x 16] on the matrix cores instead of 16 GEMVs.
//
// Block workspace (complex64), per box, 16 planes (one per right-hand-side
// slot n), rows XW = 16 * NT entries wide (NT tile blocks of the widest box):
//  * X, the box solutions: my rows per plane, (n, j, x) at
//    xb_off + (n * my + j) * XW + x;
//  * S, the sources: TR rows per plane (TR = most tile rows of any box), row t
//    = box row ty0 + t, (n, t, x) at box * 16 * TR * XW + (n * TR + t) * XW + x.
//    Only the tile's columns are ever written, the rest stays zero.
//
// sweep_block: one wave per box; forward sweep from the first tile row and
// backward sweep, in place in the block workspace.  The restriction into S
// and the gather out of X are in hddm_block_io.hip.
#include <hip/hip_runtime.h>

#include "hddm_internal.h"

namespace hddm {
namespace {

constexpr int NB = BLOCK_RHS;  // right-hand sides per block (the MFMA N dimension)

typedef float bf4 __attribute__((ext_vector_type(4)));
typedef unsigned int bu4 __attribute__((ext_vector_type(4)));
typedef unsigned int bu2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ bf4 mfma(float a, float b, bf4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
template <typename T>
__device__ __forceinline__ T* uni_ptr(T* p) {
  const uint64_t a = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
  return reinterpret_cast<T*>(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ float2 f2(double2 v) { return make_float2((float)v.x, (float)v.y); }
__device__ __forceinline__ float2 c32mul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Largest ring depth <= dmax that divides the tile count of one step, so
// every tile keeps its ring slot from one step to the next.
constexpr int ring_depth(int npk, int dmax) {
  for (int d = dmax; d > 1; --d)
    if (npk % d == 0) return d;
  return 1;
}

// Tiles of the upper triangle visited row by row: tile s is (tri_row, tri_col).
constexpr int tri_row(int s, int nt) {
  int I = 0;
  while (s >= nt - I) {
    s -= nt - I;
    ++I;
  }
  return I;
}
constexpr int tri_col(int s, int nt) { return tri_row(s, nt) + s - (tri_row(s, nt) * (2 * nt - tri_row(s, nt) + 1)) / 2; }

// Buffer resource over [base, base + bytes): loads past the end return zero
// and move no data.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void* base, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(uni_ptr(base)), 0, uni(bytes),
                                           0x00020000);
}

// ------------------------------------------------------------------ sweep
// One wave per box.  Lane l = 16q + r.  Row block I of a 16-column panel of
// the box is held in MFMA output layout: lane l, register v holds row
// 16I + 4q + v for right-hand side r.  That is also the B-operand layout of
// v_mfma_f32_16x16x4f32 when chunk kc of the reduction index carries rows
// 4q + kc, so the next step's right-hand side V_{j+1} (an elementwise function
// of this step's result) never leaves the lane.
//
// G_j is stored symmetric-packed (16x16 tiles on and above the diagonal,
// row-major inside an off-diagonal tile, a diagonal tile as its upper
// triangle, zero past mx).  Tiles are visited row by row of the
// upper triangle; tile U = G(I, J), I <= J, contributes
//     Y[I] += U V[J]        (A operand: lane gives U[r][4q + kc], 32 contiguous bytes)
//     Y[J] += U^T V[I]      (I < J; A operand: lane gives U[4q + kc][r])
// so after the last tile of row I both Y[I] is complete and V[I] is dead:
// block I is finished (stored, next V[I] formed) right there, with its
// workspace row loaded a few rows earlier.  The tiles stream through a ring
// of D register slots, D tiles ahead, across step boundaries.
//
// M3 = false: complex products as four real MFMAs (Re += Ur Vr - Ui Vi,
// Im += Ur Vi + Ui Vr); M3 = true: three (P1 += Ur Vr, P2 += Ui Vi,
// P3 += (Ur + Ui)(Vr + Vi); Re = P1 - P2, Im = P3 - P1 - P2).
// LDS_T = false: the transposed operand is a second, strided load of the
// tile (it hits the cache lines the first one brought in); LDS_T = true: it
// is staged through this wave's LDS (row-major write, column read) while the
// previous tile computes.
template <int NT, bool M3, bool LDS_T>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 1))) void
sweep_block_kernel(BlockBatch A) {
  constexpr int NPK = NT * (NT + 1) / 2;
  constexpr int D = ring_depth(NPK, LDS_T ? 11 : 6);  // transposes from memory take ring registers
  constexpr int XW = 16 * NT;
  constexpr int LA = 2;  // workspace rows of block I are loaded at the start of row I - LA
  constexpr int NACC = M3 ? 3 : 2;
  constexpr int TROW = 18;  // float2 per LDS tile row (16 + 2 of padding, 16-byte aligned)
  __shared__ float2 axs[XW];
  __shared__ float2 tstage[LDS_T ? 2 : 1][16 * TROW];
  const int lane = threadIdx.x, lr = lane & 15, lq = lane >> 4;
  // the context of this workgroup's box: scalar selects over the small table
  // (constant indices once unrolled, so nothing is indexed dynamically)
  const int wg = blockIdx.x;
  int cix = 0;
#pragma unroll
  for (int k = 1; k < BATCH_MAX; ++k) cix = (k < A.n && wg >= A.start[k]) ? k : cix;
  const BoxDesc* desc = A.desc[0];
  const double2* ltab = A.ltab[0];
  const float2* G = A.G[0];
  float2* X = A.X[0];
  const float2* S = A.S[0];
  int TR = A.tr[0], first = A.start[0];
#pragma unroll
  for (int k = 1; k < BATCH_MAX; ++k) {
    if (k == cix) {
      desc = A.desc[k];
      ltab = A.ltab[k];
      G = A.G[k];
      X = A.X[k];
      S = A.S[k];
      TR = A.tr[k];
      first = A.start[k];
    }
  }
  const int box = wg - first;
  const BoxDesc bd = desc[box];
  const int mx = uni(bd.mx), my = uni(bd.my);
  const int nt = (mx + 15) >> 4, npk = nt * (nt + 1) / 2;
  const double2* __restrict__ ax = ltab + bd.tab_off;
  const double2* __restrict__ ihy = ax + mx + (mx + 1) + my;
  for (int x = lane; x < XW; x += 64) axs[x] = x < mx ? f2(ax[x]) : make_float2(0.f, 0.f);
  __syncthreads();
  float2* __restrict__ Xb = uni_ptr(X + bd.xb_off);
  const float2* __restrict__ Gbox = uni_ptr(G + bd.g_off);
  const int64_t blk = (int64_t)npk * 256;
  const int j0 = uni(bd.ty0), j1 = uni(bd.ty1);
  const int nf = my - j0, T = nf + my - 1;
  auto row_of = [&](int st) { return st < nf ? j0 + st : my - 2 - (st - nf); };
  auto g_rsrc = [&](int j, bool valid) {
    return rsrc(Gbox + (int64_t)j * blk, valid ? npk * 2048 : 0);
  };
  // the box's solutions / sources as resources (empty when not needed: loads
  // give zeros without traffic)
  const int tr = uni(TR);
  const float2* __restrict__ Sb = uni_ptr(S + (int64_t)box * NB * tr * XW);
  auto x_rsrc = [&](bool valid) { return rsrc(Xb, valid ? NB * my * XW * 8 : 0); };
  auto s_rsrc = [&](bool valid) { return rsrc(Sb, valid ? NB * tr * XW * 8 : 0); };
  const int voff_a = (lr * 16 + 4 * lq) * 8;  // U[r][4q .. 4q+3]
  // the same entries of a diagonal tile (upper triangle stored only)
  const int voff_d[4] = {diag_read_pos(lr, 4 * lq) * 8, diag_read_pos(lr, 4 * lq + 1) * 8,
                         diag_read_pos(lr, 4 * lq + 2) * 8, diag_read_pos(lr, 4 * lq + 3) * 8};
  const int voff_t = (4 * lq * 16 + lr) * 8;  // U[4q + kc][r] at + kc * 128
  // plane n = r, columns x = 4q .. 4q+3 (+ 16I, + row * XW)
  const int voff_x = (lr * my * XW + 4 * lq) * 8;
  const int voff_s = (lr * tr * XW + 4 * lq) * 8;

  bf4 acc[NT][NACC], Vr[NT], Vi[NT];
  bf4 Vs[M3 ? NT : 1];  // M3: Vr + Vi, formed once per block and step
  bu4 ga0[D], ga1[D];
  bu2 gt[LDS_T ? 2 : D][4];  // transposed operand: staged copies (LDS_T) or ring slots
  float2 fin[NT][4];

  auto load_tile = [&](int slot, __amdgpu_buffer_rsrc_t rs, int I, int J) {
    const int so = (J * (J + 1) / 2 + I) * 2048;
    if (I == J) {
      // diagonal tile: its upper triangle only (1088 bytes); U[r][4q + kc]
      // from the stored twin of each entry
      const bu2 d0 = __builtin_amdgcn_raw_buffer_load_b64(rs, voff_d[0], so, 0);
      const bu2 d1 = __builtin_amdgcn_raw_buffer_load_b64(rs, voff_d[1], so, 0);
      const bu2 d2 = __builtin_amdgcn_raw_buffer_load_b64(rs, voff_d[2], so, 0);
      const bu2 d3 = __builtin_amdgcn_raw_buffer_load_b64(rs, voff_d[3], so, 0);
      ga0[slot] = bu4{d0.x, d0.y, d1.x, d1.y};
      ga1[slot] = bu4{d2.x, d2.y, d3.x, d3.y};
      return;
    }
    ga0[slot] = __builtin_amdgcn_raw_buffer_load_b128(rs, voff_a, so, 0);
    ga1[slot] = __builtin_amdgcn_raw_buffer_load_b128(rs, voff_a + 16, so, 0);
    if (!LDS_T && I != J) {
#pragma unroll
      for (int kc = 0; kc < 4; ++kc)
        gt[slot][kc] = __builtin_amdgcn_raw_buffer_load_b64(rs, voff_t + kc * 128, so, 0);
    }
  };
  // LDS_T: tile in ring slot `slot` -> LDS buffer b (row-major) -> gt[b] (column reads)
  auto stage_t = [&](int slot, int b) {
    float2* t = tstage[b];
    *reinterpret_cast<bu4*>(t + lr * TROW + 4 * lq) = ga0[slot];
    *reinterpret_cast<bu4*>(t + lr * TROW + 4 * lq + 2) = ga1[slot];
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) gt[b][kc] = *reinterpret_cast<const bu2*>(t + (4 * lq + kc) * TROW + lr);
  };
  // row `row`, block I of this lane's plane (lane offset voff): 4 consecutive
  // columns, 32 bytes
  auto load_fin = [&](__amdgpu_buffer_rsrc_t rs, int voff, int row, int I) {
    const bu4 u0 = __builtin_amdgcn_raw_buffer_load_b128(rs, voff + I * 128, row * XW * 8, 0);
    const bu4 u1 = __builtin_amdgcn_raw_buffer_load_b128(rs, voff + I * 128 + 16, row * XW * 8, 0);
    fin[I][0] = make_float2(__uint_as_float(u0.x), __uint_as_float(u0.y));
    fin[I][1] = make_float2(__uint_as_float(u0.z), __uint_as_float(u0.w));
    fin[I][2] = make_float2(__uint_as_float(u1.x), __uint_as_float(u1.y));
    fin[I][3] = make_float2(__uint_as_float(u1.z), __uint_as_float(u1.w));
  };

  // V = source of the first tile row; ring = first D tiles of G_{j0}
  {
    const __amdgpu_buffer_rsrc_t ss = s_rsrc(true);
#pragma unroll
    for (int I = 0; I < NT; ++I) {
      load_fin(ss, voff_s, 0, I);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        Vr[I][v] = fin[I][v].x;
        Vi[I][v] = fin[I][v].y;
      }
      if (M3) Vs[I] = Vr[I] + Vi[I];
#pragma unroll
      for (int a = 0; a < NACC; ++a) acc[I][a] = bf4{0.f, 0.f, 0.f, 0.f};
    }
    const __amdgpu_buffer_rsrc_t g0 = g_rsrc(j0, true);
    int pI = 0, pJ = 0;
#pragma unroll
    for (int s = 0; s < D; ++s) {
      load_tile(s, g0, pI, pJ);
      if (++pJ == NT) pJ = ++pI;
    }
  }

#pragma unroll 1
  for (int st = 0; st < T; ++st) {
    const bool fwd = st < nf;
    const bool fwd_next = st + 1 < nf;
    const bool more = st + 1 < T;
    const int j = uni(row_of(st));
    const int jn = uni(row_of(more ? st + 1 : st));
    const __amdgpu_buffer_rsrc_t gcur = g_rsrc(j, true);
    const __amdgpu_buffer_rsrc_t gnext = g_rsrc(jn, more);
    // finishing input of every block: forward -> source row j+1 (inside the
    // tile rows), backward -> y_j from the forward sweep (rows >= j0); an
    // empty resource (zeros, no traffic) otherwise
    // forward: source row j+1 - j0 of S (an empty resource past the tile
    // rows); backward: y_j from X (empty below the first tile row); the two
    // are selected by scalar values, so the loads stay branch-free
    const bool need = fwd ? (fwd_next && j + 1 < j1) : (j >= j0);
    const __amdgpu_buffer_rsrc_t xr = fwd ? s_rsrc(need) : x_rsrc(need);
    const int voff_r = fwd ? voff_s : voff_x;
    const int rr = fwd ? min(j + 1 - j0, tr - 1) : j;
    const float2 ih = f2(ihy[fwd_next ? j + 1 : j]);
    const __amdgpu_buffer_rsrc_t xw = x_rsrc(true);  // this step's row (stores)
#pragma unroll
    for (int I = 0; I <= LA && I < NT; ++I) load_fin(xr, voff_r, rr, I);
    // (pI, pJ): the tile D positions ahead, advanced with the loop counters so
    // that every index folds to a constant once the loops are unrolled
    constexpr int kI0 = tri_row(D % NPK, NT), kJ0 = tri_col(D % NPK, NT);
    int pI = kI0, pJ = kJ0;
    int s = 0;
#pragma unroll
    for (int I = 0; I < NT; ++I) {
      if (I > 0 && I + LA < NT) load_fin(xr, voff_r, rr, I + LA);
#pragma unroll
      for (int J = I; J < NT; ++J, ++s) {
        const int slot = s % D;
        // LDS_T: stage the transposed operand of the next tile of this step
        // (tile 0 of a step is diagonal, so every off-diagonal tile is staged here)
        if (LDS_T) {
          const int In = J + 1 < NT ? I : I + 1, Jn = J + 1 < NT ? J + 1 : I + 1;
          if (In < NT && In != Jn) stage_t((s + 1) % D, (s + 1) & 1);
        }
        float ur[4], ui[4], tr[4], ti[4];
        ur[0] = __uint_as_float(ga0[slot].x);
        ui[0] = __uint_as_float(ga0[slot].y);
        ur[1] = __uint_as_float(ga0[slot].z);
        ui[1] = __uint_as_float(ga0[slot].w);
        ur[2] = __uint_as_float(ga1[slot].x);
        ui[2] = __uint_as_float(ga1[slot].y);
        ur[3] = __uint_as_float(ga1[slot].z);
        ui[3] = __uint_as_float(ga1[slot].w);
        if (I != J) {
          const int ts = LDS_T ? (s & 1) : slot;
#pragma unroll
          for (int kc = 0; kc < 4; ++kc) {
            tr[kc] = __uint_as_float(gt[ts][kc].x);
            ti[kc] = __uint_as_float(gt[ts][kc].y);
          }
        }
        // the slot is free again: tile s + D of this block or the next one
        // (scheduling barriers keep the loads D tiles ahead of their use)
        __builtin_amdgcn_sched_barrier(0);
        load_tile(slot, s + D < NPK ? gcur : gnext, pI, pJ);
        __builtin_amdgcn_sched_barrier(0);
        if (++pJ == NT) {
          pJ = ++pI;
          if (pI == NT) pI = pJ = 0;
        }
        if (M3) {
#pragma unroll
          for (int kc = 0; kc < 4; ++kc) {
            acc[I][0] = mfma(ur[kc], Vr[J][kc], acc[I][0]);
            acc[I][1] = mfma(ui[kc], Vi[J][kc], acc[I][1]);
            acc[I][NACC - 1] = mfma(ur[kc] + ui[kc], Vs[M3 ? J : 0][kc], acc[I][NACC - 1]);
            if (I != J) {
              acc[J][0] = mfma(tr[kc], Vr[I][kc], acc[J][0]);
              acc[J][1] = mfma(ti[kc], Vi[I][kc], acc[J][1]);
              acc[J][NACC - 1] = mfma(tr[kc] + ti[kc], Vs[M3 ? I : 0][kc], acc[J][NACC - 1]);
            }
          }
        } else {
#pragma unroll
          for (int kc = 0; kc < 4; ++kc) {
            acc[I][0] = mfma(ur[kc], Vr[J][kc], acc[I][0]);
            acc[I][1] = mfma(ur[kc], Vi[J][kc], acc[I][1]);
            if (I != J) {
              acc[J][0] = mfma(tr[kc], Vr[I][kc], acc[J][0]);
              acc[J][1] = mfma(tr[kc], Vi[I][kc], acc[J][1]);
            }
            acc[I][0] = mfma(-ui[kc], Vi[J][kc], acc[I][0]);
            acc[I][1] = mfma(ui[kc], Vr[J][kc], acc[I][1]);
            if (I != J) {
              acc[J][0] = mfma(-ti[kc], Vi[I][kc], acc[J][0]);
              acc[J][1] = mfma(ti[kc], Vr[I][kc], acc[J][1]);
            }
          }
        }
      }
      // row I done: Y[I] complete, V[I] no longer read this step
      float2 xo[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        float xr_, xi_;
        if (M3) {
          xr_ = acc[I][0][v] - acc[I][1][v];
          xi_ = acc[I][NACC - 1][v] - acc[I][0][v] - acc[I][1][v];
        } else {
          xr_ = acc[I][0][v];
          xi_ = acc[I][1][v];
        }
        if (!fwd) {
          xr_ = fin[I][v].x - xr_;
          xi_ = fin[I][v].y - xi_;
        }
        const int x = 16 * I + 4 * lq + v;
        xo[v] = make_float2(xr_, xi_);
        const float2 cy = c32mul(c32mul(axs[x], ih), make_float2(xr_, xi_));
        if (fwd_next) {
          Vr[I][v] = fin[I][v].x - cy.x;
          Vi[I][v] = fin[I][v].y - cy.y;
        } else {
          Vr[I][v] = cy.x;
          Vi[I][v] = cy.y;
        }
      }
      __builtin_amdgcn_raw_buffer_store_b128(
          bu4{__float_as_uint(xo[0].x), __float_as_uint(xo[0].y), __float_as_uint(xo[1].x),
              __float_as_uint(xo[1].y)},
          xw, voff_x + I * 128, j * XW * 8, 0);
      __builtin_amdgcn_raw_buffer_store_b128(
          bu4{__float_as_uint(xo[2].x), __float_as_uint(xo[2].y), __float_as_uint(xo[3].x),
              __float_as_uint(xo[3].y)},
          xw, voff_x + I * 128 + 16, j * XW * 8, 0);
      if (M3) Vs[I] = Vr[I] + Vi[I];
#pragma unroll
      for (int a = 0; a < NACC; ++a) acc[I][a] = bf4{0.f, 0.f, 0.f, 0.f};
    }
  }
}

}  // namespace

int block_nt(int nt) {
  if (nt <= 4) return 4;
  if (nt <= 6) return 6;
  if (nt <= 8) return 8;
  if (nt <= 10) return 10;
  if (nt <= 12) return nt;
  return 0;
}

hipError_t describe_sweep_block(KLaunch& k, const BlockBatch& b, int nt_block, int variant) {
  if (b.n < 1 || b.n > BATCH_MAX || b.start[0] != 0 || b.start[b.n] <= 0) return hipErrorInvalidValue;
  k = KLaunch{};
#define HDDM_BLK(NTV)                                                                          \
  case NTV:                                                                                    \
    k.func = variant == 2   ? reinterpret_cast<const void*>(&sweep_block_kernel<NTV, false, false>) \
             : variant == 3 ? reinterpret_cast<const void*>(&sweep_block_kernel<NTV, true, false>)  \
                            : reinterpret_cast<const void*>(&sweep_block_kernel<NTV, true, true>);  \
    break;
  switch (nt_block) {
    HDDM_BLK(4)
    HDDM_BLK(6)
    HDDM_BLK(8)
    HDDM_BLK(10)
    HDDM_BLK(11)
    HDDM_BLK(12)
    default: return hipErrorInvalidValue;
  }
#undef HDDM_BLK
  k.grid = dim3(b.start[b.n]);
  k.block = dim3(64);
  k.push(b);
  return hipSuccess;
}

}  // namespace hddm
