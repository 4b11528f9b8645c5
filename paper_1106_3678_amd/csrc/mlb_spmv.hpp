// Sparse matrix-vector products of the iteration (gfx950): w = A g with the
// shadow inner products of the step fused into the epilogue, z = A u with the
// two sums of the minimisation step, r = b - A x, and plain products.  CSR rows
// of up to 8 entries use a wave-local kernel (k_spmv_csrw), 3x3-block (BSR3)
// rows of up to 8 blocks another (k_spmv_bsrw); longer rows use an LDS-tiled
// kernel (k_spmv).  Every product is one pass over A and the vectors, with the
// sums reduced into per-workgroup partials like the vector passes.
#pragma once

#include "mlb_kernels.hpp"

namespace mlb {

// Sum over aligned groups of G = 4 or 8 lanes with DPP moves (VALU only):
// quad permutes for lane ^ 1 and lane ^ 2, then the half-row mirror (lane i
// of an 8-lane half-row takes lane 7 - i, which lies in the other quad).
// Every lane of the group ends with the group's sum, added in a fixed order.
template <int CTRL>
__device__ inline float dpp_(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ inline double dpp_(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}
template <int CTRL, class R>
__device__ inline cplx<R> dpp_(cplx<R> v) {
  return {dpp_<CTRL>(v.re), dpp_<CTRL>(v.im)};
}
constexpr int DPP_XOR1 = 0xB1;       // quad_perm [1, 0, 3, 2]
constexpr int DPP_XOR2 = 0x4E;       // quad_perm [2, 3, 0, 1]
constexpr int DPP_HALF_MIRROR = 0x141;

template <int G, class T>
__device__ inline T group_sum(T v) {
  static_assert(G == 4 || G == 8, "DPP group sums cover 4 or 8 lanes");
  add_(v, dpp_<DPP_XOR1>(v));
  add_(v, dpp_<DPP_XOR2>(v));
  if constexpr (G == 8) add_(v, dpp_<DPP_HALF_MIRROR>(v));
  return v;
}

// The CSR kernels read the column indices and values of A once per pass,
// coalesced: they are loaded non-temporally, which leaves the caches (L2,
// Infinity Cache) to the vectors the next passes read again.  (Row pointers,
// shared by adjacent rows, and the 3x3 blocks of BSR3, read in 72-byte pieces
// per lane, keep ordinary loads: they rely on cache-line reuse.)
__device__ inline int ld_stream(const int* p) { return __builtin_nontemporal_load(p); }
__device__ inline double ld_stream(const double* p) { return __builtin_nontemporal_load(p); }
__device__ inline float ld_stream(const float* p) { return __builtin_nontemporal_load(p); }
template <class R>
__device__ inline cplx<R> ld_stream(const cplx<R>* p) {
  return {ld_stream(&p->re), ld_stream(&p->im)};
}

// ---------------------------------------------------------------- SpMV tiles
// A workgroup computes y = A x for a tile of rows into LDS: each wave takes
// 64 (block) rows, LPR lanes per row, so the column/value streams of one row
// are read by adjacent lanes (coalesced) and the row sums are reduced with
// butterfly shuffles.  The epilogue then runs one lane per row.

template <class V, int LPR>
__device__ inline void csr_tile(const int* __restrict__ rp, const int* __restrict__ ci, const V* __restrict__ val,
                                const V* __restrict__ xin, int nrows, int row0, V* ylds) {
  const int lane = threadIdx.x % WAVE;
  const int wbase = (threadIdx.x / WAVE) * WAVE;
  constexpr int RPP = WAVE / LPR;
  const int sub = lane % LPR, grp = lane / LPR;
  if constexpr (LPR <= 8) {
    // All LPR passes at once: row bounds, then one entry per lane and pass,
    // then the gathers, so every load of a stage is in flight together.
    int beg[LPR], end[LPR];
#pragma unroll
    for (int p = 0; p < LPR; ++p) {
      const int row = row0 + wbase + p * RPP + grp;
      beg[p] = row < nrows ? rp[row] : 0;
      end[p] = row < nrows ? rp[row + 1] : 0;
    }
    V acc[LPR];
    int col[LPR];
    V v[LPR];
#pragma unroll
    for (int p = 0; p < LPR; ++p) {
      const int q = beg[p] + sub;
      const bool on = q < end[p];
      col[p] = on ? ld_stream(ci + q) : 0;
      v[p] = on ? ld_stream(val + q) : zero<V>();
    }
#pragma unroll
    for (int p = 0; p < LPR; ++p) acc[p] = axpy(zero<V>(), v[p], xin[col[p]]);
    // rows longer than LPR entries
#pragma unroll
    for (int p = 0; p < LPR; ++p)
      for (int q = beg[p] + sub + LPR; q < end[p]; q += LPR)
        acc[p] = axpy(acc[p], ld_stream(val + q), xin[ld_stream(ci + q)]);
#pragma unroll
    for (int p = 0; p < LPR; ++p) {
#pragma unroll
      for (int m = LPR / 2; m > 0; m >>= 1) add_(acc[p], shfl_xor_(acc[p], m));
      if (sub == 0) ylds[wbase + p * RPP + grp] = acc[p];
    }
  } else {
#pragma unroll 2
    for (int p = 0; p < LPR; ++p) {
      const int lr = wbase + p * RPP + grp;
      const int row = row0 + lr;
      V acc = zero<V>();
      if (row < nrows) {
        const int beg = rp[row], end = rp[row + 1];
        for (int q = beg + sub; q < end; q += LPR) acc = axpy(acc, ld_stream(val + q), xin[ld_stream(ci + q)]);
      }
#pragma unroll
      for (int m = LPR / 2; m > 0; m >>= 1) add_(acc, shfl_xor_(acc, m));
      if (sub == 0) ylds[lr] = acc;
    }
  }
}

// The block-row bounds of the wave's 64 block rows come from one row-pointer
// load per lane (rows past the end read rp[nbrows]: empty rows) and lane
// shuffles, so the passes start with their block loads.
template <class V, int LPR>
__device__ inline void bsr3_tile(const int* __restrict__ rp, const int* __restrict__ ci, const V* __restrict__ val,
                                 const V* __restrict__ xin, int nbrows, int brow0, V* ylds) {
  const int lane = threadIdx.x % WAVE;
  const int wbase = (threadIdx.x / WAVE) * WAVE;
  constexpr int RPP = WAVE / LPR;
  const int sub = lane % LPR, grp = lane / LPR;
  const int rpl = rp[min(brow0 + wbase + lane, nbrows)];
  const int rpn = rp[min(brow0 + wbase + WAVE, nbrows)];
#pragma unroll 2
  for (int p = 0; p < LPR; ++p) {
    const int lb = wbase + p * RPP + grp;
    const int idx = p * RPP + grp;   // block row - first block row of the wave
    const int beg = __shfl(rpl, idx, WAVE);
    const int e1 = __shfl(rpl, (idx + 1) & (WAVE - 1), WAVE);
    const int end = idx == WAVE - 1 ? rpn : e1;
    V a0 = zero<V>(), a1 = zero<V>(), a2 = zero<V>();
    {
      for (int q = beg + sub; q < end; q += LPR) {
        const V* blk = val + (size_t)9 * q;
        const int c3 = 3 * ci[q];
        const V x0 = xin[c3], x1 = xin[c3 + 1], x2 = xin[c3 + 2];
        a0 = axpy(axpy(axpy(a0, blk[0], x0), blk[1], x1), blk[2], x2);
        a1 = axpy(axpy(axpy(a1, blk[3], x0), blk[4], x1), blk[5], x2);
        a2 = axpy(axpy(axpy(a2, blk[6], x0), blk[7], x1), blk[8], x2);
      }
    }
#pragma unroll
    for (int m = LPR / 2; m > 0; m >>= 1) {
      add_(a0, shfl_xor_(a0, m));
      add_(a1, shfl_xor_(a1, m));
      add_(a2, shfl_xor_(a2, m));
    }
    if (sub == 0) {
      ylds[3 * lb] = a0;
      ylds[3 * lb + 1] = a1;
      ylds[3 * lb + 2] = a2;
    }
  }
}

// SpMV epilogue modes
enum SpmvMode : int {
  SM_PLAIN = 0,   // out1 = A x
  SM_RESID = 1,   // out1 = b - A x ; sums: ||out1||^2, ||b||^2, q_1^H out1
  SM_STEP = 2,    // out1 = A x ; out2 = xown (if given) ; sums: q_s^H out1, s in [d0, d0+nd)
  SM_OMEGA = 3    // out1 = A x ; sums: out1^H out1, out1^H xown
};

template <class V>
struct SpmvArgs {
  int format;                 // 0 CSR, 1 BSR3
  int nrows;                  // scalar rows
  int nbrows;                 // block rows (BSR3) or rows (CSR)
  const int* rp;
  const int* ci;
  const V* val;
  const V* xin;               // the vector multiplied (gathered)
  const V* xown;              // the vector the epilogue reads row by row: xin, or with a
                              // preconditioner the vector xin = M^{-1} xown was made from
  V* out1;
  V* out2;
  const V* b;                 // SM_RESID
  const V* Q;                 // dots against Q columns [d0, d0+nd)
  long long ldq;
  int d0, nd;
};

template <class V, class Sc, int ND, int LPR, int FMT, int MODE>
__global__ __launch_bounds__(BLOCK) void k_spmv(State<Sc>* st, Sc* partial, SpmvArgs<V> a, int phase, int i, int j,
                                                int n, int flags) {
  if (!(flags & F_IGNORE_DONE) && st->done) return;
  constexpr int TROWS = FMT == 0 ? BLOCK : 3 * BLOCK;   // scalar rows per tile
  constexpr int NA = ND > 3 ? ND : 3;
  __shared__ V ylds[TROWS];
  V acc[NA];
#pragma unroll
  for (int d = 0; d < NA; ++d) acc[d] = zero<V>();
  const int ntiles = (a.nbrows + BLOCK - 1) / BLOCK;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    if constexpr (FMT == 0) csr_tile<V, LPR>(a.rp, a.ci, a.val, a.xin, a.nbrows, tile * BLOCK, ylds);
    else bsr3_tile<V, LPR>(a.rp, a.ci, a.val, a.xin, a.nbrows, tile * BLOCK, ylds);
    __syncthreads();
    const int rbase = tile * TROWS;
    for (int e = threadIdx.x; e < TROWS; e += BLOCK) {
      const int row = rbase + e;
      if (row >= a.nrows) break;
      V y = ylds[e];
      if constexpr (MODE == SM_PLAIN) {
        a.out1[row] = y;
      } else if constexpr (MODE == SM_RESID) {
        V bv = a.b[row];
        V rv = bv - y;
        a.out1[row] = rv;
        cdot_acc(acc[0], rv, rv);
        cdot_acc(acc[1], bv, bv);
        if (a.nd > 0) cdot_acc(acc[2], a.Q[row], rv);
      } else if constexpr (MODE == SM_STEP) {
        a.out1[row] = y;
        if (a.out2) a.out2[row] = a.xown[row];
        if constexpr (ND >= 8) {
          // columns in groups of 4, the loads of a group issued together (a group's columns
          // past nd repeat column d0 and feed sums that are never reduced)
#pragma unroll
          for (int d4 = 0; d4 < ND; d4 += 4) {
            if (d4 < a.nd) {
              V qv[4];
#pragma unroll
              for (int u = 0; u < 4; ++u) qv[u] = a.Q[row + (long long)(a.d0 + (d4 + u < a.nd ? d4 + u : 0)) * a.ldq];
#pragma unroll
              for (int u = 0; u < 4; ++u) cdot_acc(acc[d4 + u], qv[u], y);
            }
          }
        } else {
#pragma unroll
          for (int d = 0; d < ND; ++d)
            if (d < a.nd) cdot_acc(acc[d], a.Q[row + (long long)(a.d0 + d) * a.ldq], y);
        }
      } else {  // SM_OMEGA
        a.out1[row] = y;
        cdot_acc(acc[0], y, y);
        cdot_acc(acc[1], y, a.xown[row]);
      }
    }
    __syncthreads();
  }
  if (MODE == SM_PLAIN || (flags & F_SKIP_SCALAR)) return;
  const int nsum = MODE == SM_RESID ? 3 : (MODE == SM_OMEGA ? 2 : a.nd);
  block_partials<NA>(acc, nsum, partial);
}

// BSR3 SpMV with LPR <= 8 lanes per block row, wave-local: each wave computes
// 64 consecutive block rows (LPR passes of 64/LPR block rows; lane `sub` of a
// row's group takes blocks sub, sub + LPR, ...), reduces each block row's three
// sums within its lane group, puts them in the wave's LDS slice in row order
// and runs the epilogue on the tile's 192 scalar rows, three rounds of one row
// per lane (coalesced).  The block-row bounds come from one row-pointer load
// per lane and lane shuffles, the next tile's pointers loaded while the current
// tile is processed.  No workgroup barrier, so waves stream independently.
template <class V, class Sc, int ND, int LPR, int MODE>
__global__ __launch_bounds__(BLOCK) void k_spmv_bsrw(State<Sc>* st, Sc* partial, SpmvArgs<V> a, int flags) {
  const int done = st->done;   // tested once the first row pointers are in flight
  constexpr int NA = ND > 3 ? ND : 3;
  constexpr int RPP = WAVE / LPR;
  V acc[NA];
#pragma unroll
  for (int d = 0; d < NA; ++d) acc[d] = zero<V>();
  const int lane = threadIdx.x % WAVE;
  const int sub = lane % LPR, grp = lane / LPR;
  const int nwt = (a.nbrows + WAVE - 1) / WAVE;                 // wave tiles of 64 block rows
  __shared__ V tr[3 * BLOCK];                                   // 192 scalar row sums per wave
  const int wslot = (threadIdx.x / WAVE) * (3 * WAVE);
  const int wglobal = blockIdx.x * (BLOCK / WAVE) + threadIdx.x / WAVE;
  const int wstride = gridDim.x * (BLOCK / WAVE);
  auto rp_at = [&](int t, int off) { return a.rp[min((long long)t * WAVE + off, (long long)a.nbrows)]; };
  int rpl = 0, rpn = 0;
  if (wglobal < nwt) {
    rpl = rp_at(wglobal, lane);
    rpn = rp_at(wglobal, WAVE);
  }
  if (!(flags & F_IGNORE_DONE) && done) return;
  for (int wt = wglobal; wt < nwt; wt += wstride) {
    const int brow0 = wt * WAVE;
    int beg[LPR], end[LPR];
#pragma unroll
    for (int p = 0; p < LPR; ++p) {
      const int idx = p * RPP + grp;   // block row - brow0
      beg[p] = __shfl(rpl, idx, WAVE);
      const int e = __shfl(rpl, (idx + 1) & (WAVE - 1), WAVE);
      end[p] = idx == WAVE - 1 ? rpn : e;
    }
    if (wt + wstride < nwt) {
      rpl = rp_at(wt + wstride, lane);
      rpn = rp_at(wt + wstride, WAVE);
    }
    // One pass of 64/LPR block rows at a time: with two passes unrolled the
    // kernel measured 4% slower on a reservoir matrix of 7 blocks per row
    // (probably twice the block lines held in L1 between the nine strided
    // loads of each block).
#pragma unroll 1
    for (int p = 0; p < LPR; ++p) {
      V a0 = zero<V>(), a1 = zero<V>(), a2 = zero<V>();
      for (int q = beg[p] + sub; q < end[p]; q += LPR) {
        const V* blk = a.val + (size_t)9 * q;
        const int c3 = 3 * a.ci[q];
        const V x0 = a.xin[c3], x1 = a.xin[c3 + 1], x2 = a.xin[c3 + 2];
        a0 = axpy(axpy(axpy(a0, blk[0], x0), blk[1], x1), blk[2], x2);
        a1 = axpy(axpy(axpy(a1, blk[3], x0), blk[4], x1), blk[5], x2);
        a2 = axpy(axpy(axpy(a2, blk[6], x0), blk[7], x1), blk[8], x2);
      }
      a0 = group_sum<LPR>(a0);
      a1 = group_sum<LPR>(a1);
      a2 = group_sum<LPR>(a2);
      if (sub == 0) {
        const int lb = p * RPP + grp;
        tr[wslot + 3 * lb] = a0;
        tr[wslot + 3 * lb + 1] = a1;
        tr[wslot + 3 * lb + 2] = a2;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    V ys[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) ys[c] = tr[wslot + c * WAVE + lane];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int row = 3 * brow0 + c * WAVE + lane;
      if (row >= a.nrows) break;
      const V y = ys[c];
      if constexpr (MODE == SM_PLAIN) {
        a.out1[row] = y;
      } else if constexpr (MODE == SM_RESID) {
        V bv = a.b[row];
        V rv = bv - y;
        a.out1[row] = rv;
        cdot_acc(acc[0], rv, rv);
        cdot_acc(acc[1], bv, bv);
        if (a.nd > 0) cdot_acc(acc[2], a.Q[row], rv);
      } else if constexpr (MODE == SM_STEP) {
        a.out1[row] = y;
        if (a.out2) a.out2[row] = a.xown[row];
        if constexpr (ND >= 8) {
          // columns in groups of 4, the loads of a group issued together (a group's columns
          // past nd repeat column d0 and feed sums that are never reduced)
#pragma unroll
          for (int d4 = 0; d4 < ND; d4 += 4) {
            if (d4 < a.nd) {
              V qv[4];
#pragma unroll
              for (int u = 0; u < 4; ++u) qv[u] = a.Q[row + (long long)(a.d0 + (d4 + u < a.nd ? d4 + u : 0)) * a.ldq];
#pragma unroll
              for (int u = 0; u < 4; ++u) cdot_acc(acc[d4 + u], qv[u], y);
            }
          }
        } else {
#pragma unroll
          for (int d = 0; d < ND; ++d)
            if (d < a.nd) cdot_acc(acc[d], a.Q[row + (long long)(a.d0 + d) * a.ldq], y);
        }
      } else {  // SM_OMEGA
        a.out1[row] = y;
        cdot_acc(acc[0], y, y);
        cdot_acc(acc[1], y, a.xown[row]);
      }
    }
  }
  if (MODE == SM_PLAIN || (flags & F_SKIP_SCALAR)) return;
  const int nsum = MODE == SM_RESID ? 3 : (MODE == SM_OMEGA ? 2 : a.nd);
  block_partials<NA>(acc, nsum, partial);
}

// CSR SpMV with LPR <= 8 lanes per row, wave-local: each wave computes 64
// consecutive rows (LPR passes of 64/LPR rows, all loads of a stage issued
// together), moves each row sum to lane "row - first row" with shuffles and
// runs the epilogue one lane per row.  No LDS tile and no workgroup barrier
// inside the row loop, so waves stream independently.
template <class V, class Sc, int ND, int LPR, int MODE>
__global__ __launch_bounds__(BLOCK) void k_spmv_csrw(State<Sc>* st, Sc* partial, SpmvArgs<V> a, int flags) {
  if (!(flags & F_IGNORE_DONE) && st->done) return;
  constexpr int NA = ND > 3 ? ND : 3;
  constexpr int RPP = WAVE / LPR;
  V acc[NA];
#pragma unroll
  for (int d = 0; d < NA; ++d) acc[d] = zero<V>();
  const int lane = threadIdx.x % WAVE;
  const int sub = lane % LPR, grp = lane / LPR;
  const int nwt = (a.nrows + WAVE - 1) / WAVE;                 // wave tiles
  __shared__ V tr[BLOCK];                                       // 64 row sums per wave
  const int wslot = (threadIdx.x / WAVE) * WAVE;
  const int wglobal = blockIdx.x * (BLOCK / WAVE) + threadIdx.x / WAVE;
  const int wstride = gridDim.x * (BLOCK / WAVE);
  // Real values: lane L loads rp[row0 + L] and every lane loads rp[row0 + 64]
  // (rows past the end read rp[nrows]: empty rows); the bounds of each lane's
  // rows then come by lane shuffles, and the next tile's pointers are loaded
  // while the current tile is processed.  Complex values keep one pointer
  // pair per row and lane: their registers would cut the occupancy.
  constexpr bool SHUF = sizeof(V) <= 8;
  auto rp_at = [&](int t, int off) { return a.rp[min((long long)t * WAVE + off, (long long)a.nrows)]; };
  int rpl = 0, rpn = 0;
  if (SHUF && wglobal < nwt) {
    rpl = rp_at(wglobal, lane);
    rpn = rp_at(wglobal, WAVE);
  }
  for (int wt = wglobal; wt < nwt; wt += wstride) {
    const int row0 = wt * WAVE;
    int beg[LPR], end[LPR];
#pragma unroll
    for (int p = 0; p < LPR; ++p) {
      const int idx = p * RPP + grp;   // row - row0
      if constexpr (SHUF) {
        beg[p] = __shfl(rpl, idx, WAVE);
        const int e = __shfl(rpl, (idx + 1) & (WAVE - 1), WAVE);
        end[p] = idx == WAVE - 1 ? rpn : e;
      } else {
        const int row = row0 + idx;
        beg[p] = row < a.nrows ? a.rp[row] : 0;
        end[p] = row < a.nrows ? a.rp[row + 1] : 0;
      }
    }
    int col[LPR];
    V v[LPR];
#pragma unroll
    for (int p = 0; p < LPR; ++p) {
      const int q = beg[p] + sub;
      const bool on = q < end[p];
      col[p] = on ? ld_stream(a.ci + q) : 0;
      v[p] = on ? ld_stream(a.val + q) : zero<V>();
    }
    if (SHUF && wt + wstride < nwt) {
      rpl = rp_at(wt + wstride, lane);
      rpn = rp_at(wt + wstride, WAVE);
    }
    V ys[LPR];
#pragma unroll
    for (int p = 0; p < LPR; ++p) ys[p] = axpy(zero<V>(), v[p], a.xin[col[p]]);
#pragma unroll
    for (int p = 0; p < LPR; ++p)
      for (int q = beg[p] + sub + LPR; q < end[p]; q += LPR)
        ys[p] = axpy(ys[p], ld_stream(a.val + q), a.xin[ld_stream(a.ci + q)]);
    // row sums within each group of LPR lanes (DPP), then the group leaders put
    // them in the wave's LDS slice in row order and lane L reads row row0 + L
#pragma unroll
    for (int p = 0; p < LPR; ++p) {
      ys[p] = group_sum<LPR>(ys[p]);
      if (sub == 0) tr[wslot + p * RPP + grp] = ys[p];
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    V y = tr[wslot + lane];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const int row = row0 + lane;
    if (row < a.nrows) {
      if constexpr (MODE == SM_PLAIN) {
        a.out1[row] = y;
      } else if constexpr (MODE == SM_RESID) {
        V bv = a.b[row];
        V rv = bv - y;
        a.out1[row] = rv;
        cdot_acc(acc[0], rv, rv);
        cdot_acc(acc[1], bv, bv);
        if (a.nd > 0) cdot_acc(acc[2], a.Q[row], rv);
      } else if constexpr (MODE == SM_STEP) {
        a.out1[row] = y;
        if (a.out2) a.out2[row] = a.xown[row];
        if constexpr (ND >= 8) {
          // columns in groups of 4, the loads of a group issued together (a group's columns
          // past nd repeat column d0 and feed sums that are never reduced)
#pragma unroll
          for (int d4 = 0; d4 < ND; d4 += 4) {
            if (d4 < a.nd) {
              V qv[4];
#pragma unroll
              for (int u = 0; u < 4; ++u) qv[u] = a.Q[row + (long long)(a.d0 + (d4 + u < a.nd ? d4 + u : 0)) * a.ldq];
#pragma unroll
              for (int u = 0; u < 4; ++u) cdot_acc(acc[d4 + u], qv[u], y);
            }
          }
        } else {
#pragma unroll
          for (int d = 0; d < ND; ++d)
            if (d < a.nd) cdot_acc(acc[d], a.Q[row + (long long)(a.d0 + d) * a.ldq], y);
        }
      } else {  // SM_OMEGA
        a.out1[row] = y;
        cdot_acc(acc[0], y, y);
        cdot_acc(acc[1], y, a.xown[row]);
      }
    }
  }
  if (MODE == SM_PLAIN || (flags & F_SKIP_SCALAR)) return;
  const int nsum = MODE == SM_RESID ? 3 : (MODE == SM_OMEGA ? 2 : a.nd);
  block_partials<NA>(acc, nsum, partial);
}

}  // namespace mlb
