// Device code of the ML(n)BiCGStabt iteration (Algorithm 4.1 / Algorithm 7.1
// with M = I) for gfx950.
//
// The iteration is carried out as a fixed sequence of fused passes over the
// N-vectors.  Each pass streams its vectors once, coalesced (column-major
// N x n blocks, one row per lane), and reduces the inner products the next
// scalar step needs into per-workgroup partials; a one-workgroup launch
// (k_scalar) then sums the partials in a fixed order and runs the
// coefficient recurrence on one lane.  Scalars never leave the device, and a
// device "done" flag makes every later pass return at once.
//
// The sequential beta~ and beta recurrences of the algorithm (each
// coefficient uses the vector the previous one updated) are evaluated from
// small Gram matrices, which is the same arithmetic in exact arithmetic:
//   beta~ at step i (columns s = i..n-1 of the previous cycle):
//     t_s = -(q_s^H r + sum_{i<=u<s} t_u S[s][u]) / c_s
//   beta (columns s = 0..i-1 of this cycle):
//     b_s = -(f_s^H g + sum_{u<s} b_u S[s][u]) / c_s
// where S[s][u] = q_s^H w_u is produced by the SpMV pass that made w_u (its
// diagonal is c_u), and f_s^H g_u = q_s^H A g_u = q_s^H w_u (f_s = A^H q_s).
// Then one pass forms g = r + sum t_s w_s - (1/omega) sum t_s g_s, a second
// forms g_k = g + sum b_s g_s, and the SpMV pass forms w_k = A g_k from the
// stored g_k (a fresh product: recombining old w columns instead would save
// the pass but lets w_k drift from A g_k and costs attainable accuracy).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "mlb_types.hpp"

namespace mlb {

constexpr int NMAX = 32;        // largest n
constexpr int MAX_PARTIAL_ROWS = 2048;   // most workgroups of a reducing pass
constexpr int BLOCK = 256;      // threads per workgroup (4 waves of 64)
constexpr int WAVE = 64;

// Kernel flags
constexpr int F_IGNORE_DONE = 1;   // run even if the solve has finished (timing)
constexpr int F_SKIP_SCALAR = 2;   // no last-workgroup reduction / recurrence (timing)

// Phases of the scalar program run by the last workgroup
enum Phase : int {
  PH_NONE = 0,        // only store the sums in st->aux
  PH_SETUP = 1,       // r_0 = b - A x_0: ||b||, ||r_0||, e_0 = q_1^H r_0
  PH_INNER = 2,       // after x, r update of step i: err, e, beta~ coefficients
  PH_HALF = 3,        // after x, u update ending a cycle: err on u
  PH_COMBINE = 4,     // after g = r + sum t w - sum t/omega g: beta coefficients
  PH_SPMV_STEP = 5,   // after w = A g + ...: S column, c, next alpha
  PH_SPMV_OMEGA = 6,  // after z = A u: omega (eq. (5.1))
  PH_OMEGA_UPD = 7    // after x += omega u, r = u - omega z: err, e, beta~ of the cycle close
};

// Everything the recurrences need, resident in device memory.  Written only
// by k_scalar (one lane) and read by every later pass.
template <class Sc>
struct State {
  int done;             // 1 once the solve has ended
  int flag;             // 0 converged, 1 maxit, -1 breakdown
  long long iter;       // k
  long long maxit;
  double tol, kappa;
  double bnrm2, err, uu;
  Sc e, alpha, omega;
  Sc c[NMAX];
  Sc S[NMAX * NMAX];    // S[s * NMAX + u] = q_s^H w_u  (s >= u)
  Sc t[NMAX];           // pending beta~ coefficients (of the w columns)
  Sc tg[NMAX];          // -t / omega (of the g columns)
  Sc beta[NMAX];        // pending beta coefficients
  Sc aux[8];            // PH_NONE results
  double best_err;      // smallest err seen so far (stagnation guard)
  long long best_k;     // iteration at which best_err last halved
  long long stag_window;  // > 0: stop with flag 2 after this many iterations without halving
  int* host_done;       // host-mapped copy of `done` (may be null)
};

// ---------------------------------------------------------------- reductions

__device__ inline double shfl_xor_(double v, int m) { return __shfl_xor(v, m, WAVE); }
__device__ inline float shfl_xor_(float v, int m) { return __shfl_xor(v, m, WAVE); }
template <class R>
__device__ inline cplx<R> shfl_xor_(cplx<R> v, int m) {
  return {__shfl_xor(v.re, m, WAVE), __shfl_xor(v.im, m, WAVE)};
}
__device__ inline double shfl_(double v, int src) { return __shfl(v, src, WAVE); }
__device__ inline float shfl_(float v, int src) { return __shfl(v, src, WAVE); }
template <class R>
__device__ inline cplx<R> shfl_(cplx<R> v, int src) {
  return {__shfl(v.re, src, WAVE), __shfl(v.im, src, WAVE)};
}
__device__ inline void add_(double& a, double b) { a += b; }
__device__ inline void add_(float& a, float b) { a += b; }
template <class R>
__device__ inline void add_(cplx<R>& a, cplx<R> b) { a.re += b.re; a.im += b.im; }

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

template <class T>
__device__ inline T wave_sum(T v) {
#pragma unroll
  for (int m = WAVE / 2; m > 0; m >>= 1) add_(v, shfl_xor_(v, m));
  return v;
}

// Reduce acc[0..nd) over the workgroup and store the workgroup's partial sums
// (as fp64 Sc) in partial[blockIdx.x * ND + d].  The coefficient recurrence
// that needs the totals runs in the next launch (k_scalar), so the kernel
// boundary orders these stores before their use.
template <int ND, class V, class Sc>
__device__ void block_partials(V (&acc)[ND], int nd, Sc* __restrict__ partial) {
  __shared__ V red[BLOCK / WAVE][ND > 0 ? ND : 1];
  const int lane = threadIdx.x % WAVE, wid = threadIdx.x / WAVE;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    if (d < nd) {
      V v = wave_sum(acc[d]);
      if (lane == 0) red[wid][d] = v;
    }
  }
  __syncthreads();
  if (threadIdx.x < nd) {
    V v = red[0][threadIdx.x];
    for (int w = 1; w < BLOCK / WAVE; ++w) add_(v, red[w][threadIdx.x]);
    partial[(size_t)blockIdx.x * ND + threadIdx.x] = convert<Sc>(v);
  }
}

// ---------------------------------------------------------------- scalar program
// Runs on one lane of the last workgroup.  Names follow Algorithm 7.1.

template <class Sc>
__device__ inline void finish(State<Sc>* st, int flag) {
  st->flag = flag;
  st->done = 1;
  if (st->host_done) *(volatile int*)st->host_done = 1;
}

template <class Sc>
__device__ inline Sc sc_div(Sc a, Sc b) { return a / b; }
template <>
__device__ inline double sc_div<double>(double a, double b) { return a / b; }

// beta~ coefficients of step i (columns i..n-1) from d_s = q_s^H r (s = i..n-1):
// t_s = -(d_s + sum_{u=i}^{s-1} t_u S[s][u]) / c_s ; tg_s = -t_s / omega.
template <class Sc>
__device__ inline void beta_tilde(State<Sc>* st, const Sc* d, int i, int n) {
  const Sc om = st->omega;
  for (int s = i; s < n; ++s) {
    Sc acc = d[s - i];
    for (int u = i; u < s; ++u) acc = acc + st->t[u] * st->S[s * NMAX + u];
    Sc ts = zero<Sc>() - sc_div(acc, st->c[s]);
    st->t[s] = ts;
    st->tg[s] = zero<Sc>() - sc_div(ts, om);
  }
}

// Stagnation guard of the fp32 inner iteration (an addition of this library):
// flag 2 once the residual has not halved for stag_window iterations.
template <class Sc>
__device__ inline bool stagnated(State<Sc>* st, double err, long long k) {
  if (st->stag_window <= 0) return false;
  if (err < 0.5 * st->best_err) {
    st->best_err = err;
    st->best_k = k;
    return false;
  }
  return k - st->best_k >= st->stag_window;
}

template <class Sc>
__device__ void scalar_program(State<Sc>* st, const Sc* sums, int phase, int i, int j, int n) {
  switch (phase) {
    case PH_NONE:   // residual sums: ||r||^2, ||b||^2, q^H r
      for (int d = 0; d < 3; ++d) st->aux[d] = sums[d];
      break;
    case PH_SETUP: {
      double bn = sqrt(re(sums[1]));
      if (bn == 0.0) bn = 1.0;
      st->bnrm2 = bn;
      double err = sqrt(re(sums[0])) / bn;
      st->err = err;
      st->best_err = err;
      st->best_k = 0;
      st->iter = 0;
      st->e = sums[2];
      if (!finite(err)) finish(st, -1);
      else if (err < st->tol) finish(st, 0);
      break;
    }
    case PH_INNER: {
      long long k = ++st->iter;
      double err = sqrt(re(sums[0])) / st->bnrm2;
      st->err = err;
      if (!finite(err)) { finish(st, -1); break; }
      if (err < st->tol) { finish(st, 0); break; }
      if (k >= st->maxit) { finish(st, 1); break; }
      if (stagnated(st, err, k)) { finish(st, 2); break; }
      st->e = sums[1];                       // e = q_{i+1}^H r
      if (j >= 1) beta_tilde(st, sums + 1, i, n);
      break;
    }
    case PH_HALF: {
      double uu = re(sums[0]);
      double err = sqrt(uu) / st->bnrm2;
      st->uu = uu;
      st->err = err;
      if (!finite(err)) { finish(st, -1); break; }
      if (err < st->tol) { st->iter += 1; finish(st, 0); }
      break;
    }
    case PH_COMBINE: {
      // beta recurrence against this cycle's columns 0..i-1
      for (int s = 0; s < i; ++s) {
        Sc acc = sums[s];
        for (int u = 0; u < s; ++u) acc = acc + st->beta[u] * st->S[s * NMAX + u];
        st->beta[s] = zero<Sc>() - sc_div(acc, st->c[s]);
      }
      break;
    }
    case PH_SPMV_STEP: {
      for (int s = i; s < n; ++s) st->S[s * NMAX + i] = sums[s - i];
      Sc ci = sums[0];
      st->c[i] = ci;
      if (is_zero(ci) || !finite(ci)) { finish(st, -1); break; }
      st->alpha = sc_div(st->e, ci);
      break;
    }
    case PH_SPMV_OMEGA: {
      double zz = re(sums[0]);
      if (zz == 0.0 || !finite(zz)) { finish(st, -1); break; }
      Sc rho = sums[1];
      Sc om = rho / zz;
      if (st->kappa > 0) {
        Sc rn = rho / (sqrt(zz) * sqrt(st->uu));
        double a = sqrt(abs2(rn));
        if (a < st->kappa && a != 0.0) om = (st->kappa / a) * om;
      }
      if (is_zero(om) || !finite(om)) { finish(st, -1); break; }
      st->omega = om;
      break;
    }
    case PH_OMEGA_UPD: {
      long long k = ++st->iter;
      double err = sqrt(re(sums[0])) / st->bnrm2;
      st->err = err;
      if (!finite(err)) { finish(st, -1); break; }
      if (err < st->tol) { finish(st, 0); break; }
      if (k >= st->maxit) { finish(st, 1); break; }
      if (stagnated(st, err, k)) { finish(st, 2); break; }
      st->e = sums[1];                       // e = q_1^H r
      beta_tilde(st, sums + 1, 0, n);
      break;
    }
  }
}

// One workgroup: sum the partials of the previous pass in a fixed order
// (lane-strided over workgroups, then a tree; the order depends only on the
// producer's grid size) and run the coefficient recurrence on one lane.
// STRIDE is the producer's partial row length; all loads are issued before
// any reduction.
template <class Sc, int STRIDE>
__global__ __launch_bounds__(BLOCK) void k_scalar(State<Sc>* st, const Sc* __restrict__ partial, int nblocks,
                                                  int nsum, int phase, int i, int j, int n) {
  if (st->done) return;
  __shared__ Sc red2[BLOCK / WAVE][STRIDE];
  __shared__ Sc sums[STRIDE];
  const int lane = threadIdx.x % WAVE, wid = threadIdx.x / WAVE;
  Sc acc[STRIDE];
#pragma unroll
  for (int d = 0; d < STRIDE; ++d) acc[d] = zero<Sc>();
  // up to MAX_PARTIAL_ROWS producer workgroups: a fixed trip count lets every
  // load of a lane be in flight at once (the order of the sums stays fixed)
  constexpr int KR = MAX_PARTIAL_ROWS / BLOCK;                  // rows per lane
  // rows loaded together: as many as fit in a budget of 64 eight-byte registers per lane
  constexpr int WORDS = (int)(STRIDE * sizeof(Sc) / 8);
  constexpr int KC = WORDS <= 8 ? KR : WORDS <= 16 ? 4 : 2;
  if constexpr (WORDS > 32) {
    // long rows (complex, large n): the accumulators alone take half the
    // register file, so each row is summed as it arrives
    for (int b = threadIdx.x; b < nblocks; b += BLOCK) {
      const Sc* row = partial + (size_t)b * STRIDE;
#pragma unroll
      for (int d = 0; d < STRIDE; ++d)
        if (d < nsum) add_(acc[d], row[d]);
    }
  } else {
#pragma unroll
  for (int k0 = 0; k0 < KR; k0 += KC) {
    Sc v[KC][STRIDE];
#pragma unroll
    for (int k = 0; k < KC; ++k) {
      const int b = threadIdx.x + (k0 + k) * BLOCK;
      // rows past nblocks re-read row 0 and entries past nsum are read unused:
      // the buffer holds STRIDE entries for every producer workgroup
      const Sc* row = partial + (size_t)(b < nblocks ? b : 0) * STRIDE;
#pragma unroll
      for (int d = 0; d < STRIDE; ++d) v[k][d] = row[d];
    }
#pragma unroll
    for (int k = 0; k < KC; ++k) {
      const bool on = threadIdx.x + (k0 + k) * BLOCK < nblocks;
#pragma unroll
      for (int d = 0; d < STRIDE; ++d)
        if (on && d < nsum) add_(acc[d], v[k][d]);
    }
  }
  }
#pragma unroll
  for (int d = 0; d < STRIDE; ++d) {
    if (d < nsum) {
      Sc v = wave_sum(acc[d]);
      if (lane == 0) red2[wid][d] = v;
    }
  }
  __syncthreads();   // every wave's red2 row is written before any lane sums across waves
  if (threadIdx.x < nsum) {
    Sc v = red2[0][threadIdx.x];
    for (int w = 1; w < BLOCK / WAVE; ++w) add_(v, red2[w][threadIdx.x]);
    sums[threadIdx.x] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) scalar_program(st, sums, phase, i, j, n);
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
      col[p] = on ? ci[q] : 0;
      v[p] = on ? val[q] : zero<V>();
    }
#pragma unroll
    for (int p = 0; p < LPR; ++p) acc[p] = axpy(zero<V>(), v[p], xin[col[p]]);
    // rows longer than LPR entries
#pragma unroll
    for (int p = 0; p < LPR; ++p)
      for (int q = beg[p] + sub + LPR; q < end[p]; q += LPR) acc[p] = axpy(acc[p], val[q], xin[ci[q]]);
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
        for (int q = beg + sub; q < end; q += LPR) acc = axpy(acc, val[q], xin[ci[q]]);
      }
#pragma unroll
      for (int m = LPR / 2; m > 0; m >>= 1) add_(acc, shfl_xor_(acc, m));
      if (sub == 0) ylds[lr] = acc;
    }
  }
}

template <class V, int LPR>
__device__ inline void bsr3_tile(const int* __restrict__ rp, const int* __restrict__ ci, const V* __restrict__ val,
                                 const V* __restrict__ xin, int nbrows, int brow0, V* ylds) {
  const int lane = threadIdx.x % WAVE;
  const int wbase = (threadIdx.x / WAVE) * WAVE;
  constexpr int RPP = WAVE / LPR;
  const int sub = lane % LPR, grp = lane / LPR;
#pragma unroll 2
  for (int p = 0; p < LPR; ++p) {
    const int lb = wbase + p * RPP + grp;
    const int brow = brow0 + lb;
    V a0 = zero<V>(), a1 = zero<V>(), a2 = zero<V>();
    if (brow < nbrows) {
      const int beg = rp[brow], end = rp[brow + 1];
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
  SM_STEP = 2,    // out1 = A x ; out2 = x (if given) ; sums: q_s^H out1, s in [d0, d0+nd)
  SM_OMEGA = 3    // out1 = A x ; sums: out1^H out1, out1^H x
};

template <class V>
struct SpmvArgs {
  int format;                 // 0 CSR, 1 BSR3
  int nrows;                  // scalar rows
  int nbrows;                 // block rows (BSR3) or rows (CSR)
  const int* rp;
  const int* ci;
  const V* val;
  const V* xin;
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
        if (a.out2) a.out2[row] = a.xin[row];
#pragma unroll
        for (int d = 0; d < ND; ++d)
          if (d < a.nd) cdot_acc(acc[d], a.Q[row + (long long)(a.d0 + d) * a.ldq], y);
      } else {  // SM_OMEGA
        a.out1[row] = y;
        cdot_acc(acc[0], y, y);
        cdot_acc(acc[1], y, a.xin[row]);
      }
    }
    __syncthreads();
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
  for (int wt = wglobal; wt < nwt; wt += wstride) {
    const int row0 = wt * WAVE;
    int beg[LPR], end[LPR];
#pragma unroll
    for (int p = 0; p < LPR; ++p) {
      const int row = row0 + p * RPP + grp;
      beg[p] = row < a.nrows ? a.rp[row] : 0;
      end[p] = row < a.nrows ? a.rp[row + 1] : 0;
    }
    int col[LPR];
    V v[LPR];
#pragma unroll
    for (int p = 0; p < LPR; ++p) {
      const int q = beg[p] + sub;
      const bool on = q < end[p];
      col[p] = on ? a.ci[q] : 0;
      v[p] = on ? a.val[q] : zero<V>();
    }
    V ys[LPR];
#pragma unroll
    for (int p = 0; p < LPR; ++p) ys[p] = axpy(zero<V>(), v[p], a.xin[col[p]]);
#pragma unroll
    for (int p = 0; p < LPR; ++p)
      for (int q = beg[p] + sub + LPR; q < end[p]; q += LPR) ys[p] = axpy(ys[p], a.val[q], a.xin[a.ci[q]]);
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
        if (a.out2) a.out2[row] = a.xin[row];
#pragma unroll
        for (int d = 0; d < ND; ++d)
          if (d < a.nd) cdot_acc(acc[d], a.Q[row + (long long)(a.d0 + d) * a.ldq], y);
      } else {  // SM_OMEGA
        a.out1[row] = y;
        cdot_acc(acc[0], y, y);
        cdot_acc(acc[1], y, a.xin[row]);
      }
    }
  }
  if (MODE == SM_PLAIN || (flags & F_SKIP_SCALAR)) return;
  const int nsum = MODE == SM_RESID ? 3 : (MODE == SM_OMEGA ? 2 : a.nd);
  block_partials<NA>(acc, nsum, partial);
}

// ---------------------------------------------------------------- vector passes

// x += alpha gh ; r -= alpha w ; sums: ||r||^2, q_s^H r for s in [d0, d0+nd).
// With xrec, x_k is also stored in column k-1 of the iterate record.
template <class V, class Sc, int ND>
__global__ __launch_bounds__(BLOCK) void k_alpha(State<Sc>* st, Sc* partial, int N, V* __restrict__ x,
                                                 const V* __restrict__ gh, V* __restrict__ r, const V* __restrict__ w,
                                                 const V* __restrict__ Q, long long ldq, int d0, int nd,
                                                 V* __restrict__ xrec, long long K, int phase, int i, int j, int n,
                                                 int flags) {
  if (!(flags & F_IGNORE_DONE) && st->done) return;
  V acc[ND + 1];
#pragma unroll
  for (int d = 0; d <= ND; ++d) acc[d] = zero<V>();
  const V al = convert<V>(st->alpha);
  const V mal = convert<V>(zero<Sc>() - st->alpha);
  const long long k = st->iter + 1;
  V* rec = (xrec && k <= K) ? xrec + (k - 1) * (long long)N : nullptr;
  for (int row = blockIdx.x * BLOCK + threadIdx.x; row < N; row += gridDim.x * BLOCK) {
    V xv = axpy(x[row], al, gh[row]);
    x[row] = xv;
    if (rec) rec[row] = xv;
    V rv = axpy(r[row], mal, w[row]);
    r[row] = rv;
    cdot_acc(acc[0], rv, rv);
#pragma unroll
    for (int d = 0; d < ND; ++d)
      if (d < nd) cdot_acc(acc[1 + d], Q[row + (long long)(d0 + d) * ldq], rv);
  }
  if (flags & F_SKIP_SCALAR) return;
  block_partials<ND + 1>(acc, nd + 1, partial);
}

// g = r + sum_{s in [t0, n)} (t_s W_s + tg_s G_s) -> gout ; sums: f_s^H g, s < nf.
template <class V, class Sc, int ND>
__global__ __launch_bounds__(BLOCK) void k_combine(State<Sc>* st, Sc* partial, int N, const V* __restrict__ r,
                                                   const V* __restrict__ Wb, const V* __restrict__ Gb, long long ldw,
                                                   int t0, int t1, V* __restrict__ gout, const V* __restrict__ F,
                                                   long long ldf, int nf, int phase, int i, int j, int n, int flags) {
  if (!(flags & F_IGNORE_DONE) && st->done) return;
  V acc[ND > 0 ? ND : 1];
#pragma unroll
  for (int d = 0; d < (ND > 0 ? ND : 1); ++d) acc[d] = zero<V>();
  // beta~ coefficients of the w and g columns, staged in LDS
  __shared__ V tw[NMAX], tgv[NMAX];
  if (threadIdx.x >= t0 && threadIdx.x < t1) {
    tw[threadIdx.x] = convert<V>(st->t[threadIdx.x]);
    tgv[threadIdx.x] = convert<V>(st->tg[threadIdx.x]);
  }
  __syncthreads();
  for (int row = blockIdx.x * BLOCK + threadIdx.x; row < N; row += gridDim.x * BLOCK) {
    V g = r[row];
    for (int s = t0; s < t1; ++s) {
      g = axpy(g, tw[s], Wb[row + s * ldw]);
      g = axpy(g, tgv[s], Gb[row + s * ldw]);
    }
    gout[row] = g;
#pragma unroll
    for (int d = 0; d < ND; ++d)
      if (d < nf) cdot_acc(acc[d], F[row + (long long)d * ldf], g);
  }
  if ((flags & F_SKIP_SCALAR) || nf == 0) return;   // nf == 0: the beta list is empty
  block_partials<(ND > 0 ? ND : 1)>(acc, nf, partial);
}

// g_k = g + sum_{s<nb} beta_s G_s  -> gout (column k of G); beta staged in LDS.
template <class V, class Sc>
__global__ __launch_bounds__(BLOCK) void k_gcomb(const State<Sc>* st, int N, const V* __restrict__ g,
                                                 const V* __restrict__ Gb, long long ldg, int nb, V* __restrict__ gout,
                                                 int flags) {
  if (!(flags & F_IGNORE_DONE) && st->done) return;
  __shared__ V bco[NMAX];
  if (threadIdx.x < nb) bco[threadIdx.x] = convert<V>(st->beta[threadIdx.x]);
  __syncthreads();
  for (int row = blockIdx.x * BLOCK + threadIdx.x; row < N; row += gridDim.x * BLOCK) {
    V v = g[row];
    for (int s = 0; s < nb; ++s) v = axpy(v, bco[s], Gb[row + s * ldg]);
    gout[row] = v;
  }
}

// x += omega u ; r = u - omega z (u held in r) ; sums: ||r||^2, q_s^H r, s < nd.
template <class V, class Sc, int ND>
__global__ __launch_bounds__(BLOCK) void k_omega(State<Sc>* st, Sc* partial, int N, V* __restrict__ x,
                                                 V* __restrict__ r, const V* __restrict__ z, const V* __restrict__ Q,
                                                 long long ldq, int nd, V* __restrict__ xrec, long long K, int phase,
                                                 int n, int flags) {
  if (!(flags & F_IGNORE_DONE) && st->done) return;
  V acc[ND + 1];
#pragma unroll
  for (int d = 0; d <= ND; ++d) acc[d] = zero<V>();
  const V om = convert<V>(st->omega);
  const V mom = convert<V>(zero<Sc>() - st->omega);
  const long long k = st->iter + 1;
  V* rec = (xrec && k <= K) ? xrec + (k - 1) * (long long)N : nullptr;
  for (int row = blockIdx.x * BLOCK + threadIdx.x; row < N; row += gridDim.x * BLOCK) {
    const V u = r[row];
    V xv = axpy(x[row], om, u);
    x[row] = xv;
    if (rec) rec[row] = xv;
    V rv = axpy(u, mom, z[row]);
    r[row] = rv;
    cdot_acc(acc[0], rv, rv);
#pragma unroll
    for (int d = 0; d < ND; ++d)
      if (d < nd) cdot_acc(acc[1 + d], Q[row + (long long)d * ldq], rv);
  }
  if (flags & F_SKIP_SCALAR) return;
  block_partials<ND + 1>(acc, nd + 1, partial);
}

// ---------------------------------------------------------------- small helpers

template <class V>
__global__ void k_fill(V* __restrict__ y, long long N, V v) {
  for (long long i = blockIdx.x * (long long)BLOCK + threadIdx.x; i < N; i += (long long)gridDim.x * BLOCK) y[i] = v;
}

// out (To) = s * in (From), s = 1 / sqrt(re(st->aux[0])) when scale_by_aux, else 1
template <class To, class From, class Sc>
__global__ void k_cast(To* __restrict__ out, const From* __restrict__ in, long long N, const State<Sc>* st,
                       int scale_by_aux) {
  double s = 1.0;
  if (scale_by_aux) s = 1.0 / sqrt(re(st->aux[0]));
  for (long long i = blockIdx.x * (long long)BLOCK + threadIdx.x; i < N; i += (long long)gridDim.x * BLOCK) {
    auto w = convert<typename traits<From>::wide>(in[i]);
    out[i] = convert<To>(s * w);
  }
}

// x (wide) += sqrt(re(st->aux[0])) * Minv d (narrow), Minv block diagonal (BS = 1 or 3);
// without Minv: x += sqrt(re(st->aux[0])) * d.
template <class Vw, class Vn, class Sc, int BS>
__global__ void k_axpy_wide_minv(Vw* __restrict__ x, const Vn* __restrict__ d, const Vw* __restrict__ Minv,
                                 int nbrows, const State<Sc>* st) {
  const Vw s = from_real<Vw>(sqrt(re(st->aux[0])));
  for (int row = blockIdx.x * BLOCK + threadIdx.x; row < nbrows; row += gridDim.x * BLOCK) {
    Vw dv[BS];
    for (int k = 0; k < BS; ++k) dv[k] = convert<Vw>(d[(long long)BS * row + k]);
    for (int r = 0; r < BS; ++r) {
      Vw t = dv[r];
      if (Minv) {
        t = zero<Vw>();
        for (int k = 0; k < BS; ++k) t = axpy(t, Minv[(size_t)BS * BS * row + BS * r + k], dv[k]);
      }
      x[(long long)BS * row + r] = axpy(x[(long long)BS * row + r], s, t);
    }
  }
}

// x (wide) += sqrt(re(st->aux[0])) * d (narrow)
template <class Vw, class Vn, class Sc>
__global__ void k_axpy_wide(Vw* __restrict__ x, const Vn* __restrict__ d, long long N, const State<Sc>* st) {
  const double s = sqrt(re(st->aux[0]));
  for (long long i = blockIdx.x * (long long)BLOCK + threadIdx.x; i < N; i += (long long)gridDim.x * BLOCK) {
    Vw dv = convert<Vw>(d[i]);
    x[i] = axpy(x[i], from_real<Vw>(s), dv);
  }
}

}  // namespace mlb
