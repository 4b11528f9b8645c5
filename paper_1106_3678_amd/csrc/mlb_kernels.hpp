// Device code of the ML(n)BiCGStabt iteration (Algorithm 4.1 / Algorithm 7.1
// with M = I) for gfx950.
//
// The iteration is carried out as a fixed sequence of fused passes over the
// N-vectors.  Each pass streams its vectors once, coalesced (column-major
// N x n blocks, one row per lane), and reduces the inner products the next
// scalar step needs into per-workgroup partials; a one-workgroup launch
// (k_scalar) then sums the partials in a fixed order and runs the
// coefficient recurrence on one wave.  Scalars never leave the device, and a
// device "done" flag makes every later pass return at once.
//
// The sequential beta~ and beta recurrences of the algorithm (each
// coefficient uses the vector the previous one updated) are evaluated from
// small Gram matrices, which is the same arithmetic in exact arithmetic:
//   beta~ at step i (columns s = i..n-1 of the previous cycle):
//     t_s = -(q_s^H r + sum_{i<=u<s} t_u S[s][u]) / c_s
//   beta (columns s = 0..i-1 of this cycle):
//     b_s = -(f_s^H g + sum_{u<s} b_u S[s][u]) / c_s
// where S[s][u] = q_s^H w_u and f_s^H g_u = q_s^H A g_u = q_s^H w_u
// (f_s = A^H q_s).  The diagonal c_u comes from the SpMV pass that made w_u
// (the next alpha needs it); the entries below it (s > u) from the next alpha
// pass, which reads w_u and the same columns q_s (for q_s^H r) anyway, so the
// SpMV pass reads one column of Q instead of n - u.  Every S[s][u] is first
// used by a recurrence after that alpha pass: beta~ at step i reads columns
// u >= i of the previous cycle, beta at step i columns u <= i - 2.
// Then one pass forms g = r + sum t_s w_s - (1/omega) sum t_s g_s, a second
// forms g_k = g + sum b_s g_s, and the SpMV pass forms w_k = A g_k from the
// stored g_k (a fresh product: recombining old w columns instead would save
// the pass but lets w_k drift from A g_k and costs attainable accuracy).
//
// Transpose-free variant: f_s^H g = q_s^H (A g), so the SpMV pass forms
// v = A g before the beta recurrence and reduces q_s^H v (s < i) for it; one
// pass (k_gwcomb) then forms g_k = g + sum b_s g_s and w_k = v + sum b_s w_s
// (the recombination, the price of having no A^H) and reduces q_s^H w_k,
// s >= i, the S column and c of step i.
//
// Literal order: the two recurrences can also run as written, one coefficient
// per pass and reduction (k_lit_tilde, k_lit_beta, PH_LIT_T / PH_LIT_B), each
// from the inner product of the vector the previous coefficient updated.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "mlb_types.hpp"

namespace mlb {

constexpr int NMAX = 32;        // largest n
constexpr int MAX_PARTIAL_ROWS = 2048;   // most workgroups of a reducing pass
constexpr int PSUM_GRID = 64;            // first-stage workgroups for long partial rows
constexpr int BLOCK = 256;      // threads per workgroup (4 waves of 64)
// Complex partial rows longer than 64 bytes are summed in two stages (k_psum
// first): the one-workgroup stage does not keep enough of their 16-byte loads
// in flight.
template <class Sc, int STRIDE>
constexpr bool wide_rows() { return sizeof(Sc) > 8 && STRIDE * sizeof(Sc) > 64; }
// Threads of the one-workgroup recurrence kernel (k_scalar) for partial rows of
// STRIDE entries: 1024 for the longer real rows, which keeps more of a long
// table's loads in flight.
template <class Sc, int STRIDE>
constexpr int sblock() { return STRIDE <= 5 || wide_rows<Sc, STRIDE>() ? 256 : 1024; }
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
  PH_OMEGA_UPD = 7,   // after x += omega u, r = u - omega z: err, e, beta~ of the cycle close
  // the sequential (literal) order of the recurrences: one coefficient per reduction
  PH_LIT_T = 8,       // after a beta~ pass: t_i = -(q_i^H z_w) / c_i (i = the coefficient's index)
  PH_LIT_B = 9,       // after a beta pass: beta_i = -(f_i^H g) / c_i
  PH_OMEGA_LIT = 10,  // as PH_OMEGA_UPD, without the beta~ list (computed pass by pass)
  PH_INNER_S = 11,    // as PH_INNER, and the S column of w_{i-1} below its diagonal
  PH_SPMV_C = 12      // as PH_SPMV_STEP with only c (the rest of the S column: next PH_INNER_S)
};

// The shadow-vector count a pass is compiled for (the bucket of n): the
// number of dot columns of its accumulators.
__host__ __device__ constexpr int bucket_of(int n) { return n <= 4 ? 4 : n <= 8 ? 8 : n <= 16 ? 16 : 32; }

// Everything the recurrences need, resident in device memory.  Written only
// by k_scalar and read by every later pass.
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
  Sc cinv[NMAX];        // 1 / c
  Sc t[NMAX];           // pending beta~ coefficients (of the w columns)
  Sc tg[NMAX];          // -t / omega (of the g columns)
  Sc beta[NMAX];        // pending beta coefficients
  Sc aux[8];            // PH_NONE results
  double best_err;      // smallest err seen so far (stagnation guard)
  long long best_k;     // iteration at which best_err last halved
  long long stag_window;  // > 0: stop with flag 2 after this many iterations without halving
  int* host_done;       // host-mapped copy of `done` (may be null)
  // Deferred x updates (solves that record no iterates): alph[t] is the alpha that
  // multiplies g in column t of G this cycle (set with it by the SpMV step of
  // column t); npend of them are pending: x_k = x + sum_{t < npend} alph[t] G_t.
  Sc alph[NMAX];
  int npend;
  int npad_;
  Sc S[NMAX * NMAX];    // S[s * NMAX + u] = q_s^H w_u  (s >= u); last, so rows s >= n can be left out of copies
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
// Runs on the 64 lanes of one wave of k_scalar, over the state staged in LDS.
// Every lane evaluates the scalar bookkeeping (the same arithmetic on the same
// values, so all lanes take the same branches) and lane 0 stores it; the two
// triangular recurrences run across the lanes.  Names follow Algorithm 7.1.

template <class Sc>
__device__ inline void finish(State<Sc>* st, int flag) {
  if (threadIdx.x % WAVE != 0) return;
  st->flag = flag;
  st->done = 1;
  if (st->host_done) *(volatile int*)st->host_done = 1;
}

template <class Sc>
__device__ inline Sc sc_div(Sc a, Sc b) { return a / b; }
template <>
__device__ inline double sc_div<double>(double a, double b) { return a / b; }

// value of lane `src` (wave-uniform) in every lane
__device__ inline double bcast_(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}
template <class R>
__device__ inline cplx<R> bcast_(cplx<R> v, int src) {
  return {bcast_(v.re, src), bcast_(v.im, src)};
}

// Forward substitution x_s = -(d_s + sum_{lo<=u<s} x_u S[s][u]) / c_s for
// s = lo..hi-1 (hi - lo <= 32), by columns: lane s - lo keeps the running sum
// of row s, and at step u the lane of row u finishes x_u = -sum * (1/c_u),
// which is broadcast to the rows below.  Each row adds its terms in the order
// u = lo, lo+1, ..., as the sequential recurrence does.  Returns x_s in lane
// s - lo (zero in the other lanes).
template <class Sc>
__device__ inline Sc forward_subst(const State<Sc>* st, const Sc* d, int lo, int hi) {
  const int lane = threadIdx.x % WAVE;
  const int s = lo + lane;
  const bool mine = s < hi;
  Sc acc = mine ? d[lane] : zero<Sc>();
  Sc xs = zero<Sc>();
  for (int u = lo; u < hi; ++u) {
    const Sc xu = bcast_(zero<Sc>() - acc * st->cinv[u], u - lo);
    if (s == u) xs = xu;
    if (mine && s > u) acc = acc + xu * st->S[s * NMAX + u];
  }
  return xs;
}

// beta~ coefficients of step i (columns i..n-1) from d_s = q_s^H r (s = i..n-1):
// t_s = -(d_s + sum_{u=i}^{s-1} t_u S[s][u]) / c_s ; tg_s = -t_s / omega.
template <class Sc>
__device__ inline void beta_tilde(State<Sc>* st, const Sc* d, int i, int n) {
  const Sc ts = forward_subst(st, d, i, n);
  const int s = i + threadIdx.x % WAVE;
  if (s < n) {
    st->t[s] = ts;
    st->tg[s] = zero<Sc>() - sc_div(ts, st->omega);
  }
}

// Stagnation guard of the fp32 inner iteration (an addition of this library):
// flag 2 once the residual has not halved for stag_window iterations.
template <class Sc>
__device__ inline bool stagnated(State<Sc>* st, double err, long long k) {
  if (st->stag_window <= 0) return false;
  if (err < 0.5 * st->best_err) {
    if (threadIdx.x % WAVE == 0) {
      st->best_err = err;
      st->best_k = k;
    }
    return false;
  }
  return k - st->best_k >= st->stag_window;
}

template <class Sc>
__device__ void scalar_program(State<Sc>* st, const Sc* sums, int phase, int i, int j, int n) {
  const bool w0 = threadIdx.x % WAVE == 0;   // the lane that stores scalars
  switch (phase) {
    case PH_NONE:   // residual sums: ||r||^2, ||b||^2, q^H r
      if (w0)
        for (int d = 0; d < 3; ++d) st->aux[d] = sums[d];
      break;
    case PH_SETUP: {
      double bn = sqrt(re(sums[1]));
      if (bn == 0.0) bn = 1.0;
      double err = sqrt(re(sums[0])) / bn;
      if (w0) {
        st->bnrm2 = bn;
        st->err = err;
        st->best_err = err;
        st->best_k = 0;
        st->iter = 0;
        st->e = sums[2];
        st->npend = 0;
      }
      if (!finite(err)) finish(st, -1);
      else if (err < st->tol) finish(st, 0);
      break;
    }
    case PH_INNER_S:
    case PH_INNER: {
      if (phase == PH_INNER_S) {
        // sums[1 + bucket + l] = q_{i+l}^H w_{i-1}, l = 0..n-i-1 (k_alpha with SW)
        const int l = threadIdx.x % WAVE;
        if (l < n - i) st->S[(i + l) * NMAX + (i - 1)] = sums[1 + bucket_of(n) + l];
      }
      const long long k = st->iter + 1;
      double err = sqrt(re(sums[0])) / st->bnrm2;
      if (w0) {
        st->iter = k;
        st->err = err;
        st->npend = i;                       // x_{jn+i} = x + sum_{t < i} alph[t] G_t
      }
      if (!finite(err)) { finish(st, -1); break; }
      if (err < st->tol) { finish(st, 0); break; }
      if (k >= st->maxit) { finish(st, 1); break; }
      if (stagnated(st, err, k)) { finish(st, 2); break; }
      if (w0) st->e = sums[1];               // e = q_{i+1}^H r
      if (j >= 1) beta_tilde(st, sums + 1, i, n);
      break;
    }
    case PH_HALF: {
      double uu = re(sums[0]);
      double err = sqrt(uu) / st->bnrm2;
      if (w0) {
        st->uu = uu;
        st->err = err;
        st->npend = n;                       // the half-step x: all n alpha steps of the cycle
      }
      if (!finite(err)) { finish(st, -1); break; }
      if (err < st->tol) {
        if (w0) st->iter += 1;
        finish(st, 0);
      }
      break;
    }
    case PH_COMBINE: {
      // beta recurrence against this cycle's columns 0..i-1
      const Sc b = forward_subst(st, sums, 0, i);
      const int s = threadIdx.x % WAVE;
      if (s < i) st->beta[s] = b;
      break;
    }
    case PH_SPMV_C:
    case PH_SPMV_STEP: {
      const int l = threadIdx.x % WAVE;
      if (i + l < n && (l == 0 || phase == PH_SPMV_STEP)) st->S[(i + l) * NMAX + i] = sums[l];
      Sc ci = sums[0];
      if (w0) st->c[i] = ci;
      if (is_zero(ci) || !finite(ci)) { finish(st, -1); break; }
      if (w0) {
        st->cinv[i] = sc_div(from_real<Sc>(1.0), ci);
        st->alpha = sc_div(st->e, ci);
        st->alph[i] = st->alpha;             // multiplies G_i in the next alpha step
      }
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
      if (w0) st->omega = om;
      break;
    }
    case PH_LIT_T:
      if (w0) st->t[i] = zero<Sc>() - sums[0] * st->cinv[i];
      break;
    case PH_LIT_B:
      if (w0) st->beta[i] = zero<Sc>() - sums[0] * st->cinv[i];
      break;
    case PH_OMEGA_LIT:
    case PH_OMEGA_UPD: {
      const long long k = st->iter + 1;
      double err = sqrt(re(sums[0])) / st->bnrm2;
      if (w0) {
        st->iter = k;
        st->err = err;
        st->npend = 0;                       // k_omega applied the cycle's alpha steps
      }
      if (!finite(err)) { finish(st, -1); break; }
      if (err < st->tol) { finish(st, 0); break; }
      if (k >= st->maxit) { finish(st, 1); break; }
      if (stagnated(st, err, k)) { finish(st, 2); break; }
      if (w0) st->e = sums[1];               // e = q_1^H r
      if (phase == PH_OMEGA_UPD) beta_tilde(st, sums + 1, 0, n);
      break;
    }
  }
}

// Sums rows [r0, r1) of a pass's partials (row length STRIDE) into
// sums[0..nsum) in LDS, in a fixed order, with NT threads.  Thread (g, d)
// (d = t % STRIDE, g = t / STRIDE, G = NT / STRIDE groups) adds entry d of
// rows g, g + G, g + 2G, ... in that order; the rows are loaded in batches of
// SUM_BATCH, all loads of a batch issued before its adds (adjacent threads read
// adjacent words).  The G group sums of each entry are then added in group
// order; beyond 64 groups in a fixed two-level order instead (32 runs of
// consecutive groups, then the run sums), which keeps the dependent chain
// short.  Ends with a barrier; every thread must call it.
constexpr int SUM_BATCH = 16;
template <class Sc, int STRIDE, int NT>
__device__ void sum_rows(const Sc* __restrict__ partial, int r0, int r1, int nsum, Sc* sums) {
  constexpr int G = NT / STRIDE;
  __shared__ Sc red[G][STRIDE];
  const int t = threadIdx.x, d = t % STRIDE, g = t / STRIDE;
  const int nrows = r1 - r0;
  if (g < G && d < nsum) {
    const Sc* base = partial + (size_t)r0 * STRIDE + d;
    Sc acc = zero<Sc>();
    for (int k0 = g; k0 < nrows; k0 += SUM_BATCH * G) {
      Sc v[SUM_BATCH];
#pragma unroll
      for (int u = 0; u < SUM_BATCH; ++u) {
        const int r = k0 + u * G;
        v[u] = base[(size_t)(r < nrows ? r : 0) * STRIDE];   // row 0 of the range re-read, unused
      }
#pragma unroll
      for (int u = 0; u < SUM_BATCH; ++u)
        if (k0 + u * G < nrows) add_(acc, v[u]);
    }
    red[g][d] = acc;
  }
  __syncthreads();
  if constexpr (G <= 64) {
    if (t < nsum) {
      Sc v = red[0][t];
      for (int q = 1; q < G; ++q) add_(v, red[q][t]);
      sums[t] = v;
    }
  } else {
    constexpr int H = 32;
    __shared__ Sc red2[H][STRIDE];
    if (g < H && d < nsum) {
      const int q0 = g * G / H, q1 = (g + 1) * G / H;
      Sc v = red[q0][d];
      for (int q = q0 + 1; q < q1; ++q) add_(v, red[q][d]);
      red2[g][d] = v;
    }
    __syncthreads();
    if (t < nsum) {
      Sc v = red2[0][t];
      for (int q = 1; q < H; ++q) add_(v, red2[q][t]);
      sums[t] = v;
    }
  }
  __syncthreads();
}

// Partial tables that would take the one-workgroup stage more than three load
// batches per thread (long rows: many shadow vectors), and wide complex rows,
// are summed in two stages, PSUM_GRID workgroups first (the extra launch costs
// more than a third batch).
template <class Sc, int STRIDE>
constexpr bool two_stage() {
  constexpr int G = sblock<Sc, STRIDE>() / STRIDE;
  return wide_rows<Sc, STRIDE>() || (MAX_PARTIAL_ROWS + G - 1) / G > 3 * SUM_BATCH;
}

// First stage: workgroup g sums the g-th contiguous share of the rows into row
// g of `out`, so that the one-workgroup stage reads PSUM_GRID rows.  It does not
// test the done flag: after the end it sums stale partials into `out`, which
// k_scalar then ignores, and it saves the flag's round trip before the loads.
template <class Sc, int STRIDE>
__global__ __launch_bounds__(BLOCK) void k_psum(const Sc* __restrict__ partial, int nblocks, int nsum,
                                                Sc* __restrict__ out) {
  __shared__ Sc sums[STRIDE];
  const int r0 = (int)((long long)nblocks * blockIdx.x / gridDim.x);
  const int r1 = (int)((long long)nblocks * (blockIdx.x + 1) / gridDim.x);
  sum_rows<Sc, STRIDE, BLOCK>(partial, r0, r1, nsum, sums);
  if (threadIdx.x < nsum) out[(size_t)blockIdx.x * STRIDE + threadIdx.x] = sums[threadIdx.x];
}

// One workgroup of sblock<Sc, STRIDE>() threads: sum the partials of the previous pass (or of
// k_psum) in a fixed order and run the coefficient recurrence on one wave.  The state is
// staged in LDS for the recurrence (its loops read the n x n Gram matrix and
// the coefficient lists entry by entry) and written back afterwards; rows
// s >= n of the Gram matrix are never touched and stay out of both copies.
// The state words (the done flag among them) and the partials are loaded in
// one round trip: the flag is tested once both have arrived (after the end,
// the partials read are stale and ignored; the buffer always holds nblocks
// rows, so the reads stay in bounds).
template <class Sc, int STRIDE>
__global__ __launch_bounds__((sblock<Sc, STRIDE>())) void k_scalar(State<Sc>* st, const Sc* __restrict__ partial, int nblocks,
                                                  int nsum, int phase, int i, int j, int n) {
  static_assert(sizeof(State<Sc>) % 8 == 0 && offsetof(State<Sc>, S) % 8 == 0, "state is copied in 8-byte words");
  constexpr int SB = sblock<Sc, STRIDE>();
  constexpr int CW = (int)((sizeof(State<Sc>) / 8 + SB - 1) / SB);   // state words per thread, at most
  __shared__ State<Sc> ss;
  __shared__ Sc sums[STRIDE];
  const int nwords = (int)((offsetof(State<Sc>, S) + sizeof(Sc) * (size_t)n * NMAX) / 8);
  unsigned long long* gw = reinterpret_cast<unsigned long long*>(st);
  unsigned long long* lw = reinterpret_cast<unsigned long long*>(&ss);
  unsigned long long sw[CW];
#pragma unroll
  for (int c = 0; c < CW; ++c) {
    const int w = threadIdx.x + c * SB;
    sw[c] = w < nwords ? gw[w] : 0ull;
  }
  sum_rows<Sc, STRIDE, SB>(partial, 0, nblocks, nsum, sums);
#pragma unroll
  for (int c = 0; c < CW; ++c) {
    const int w = threadIdx.x + c * SB;
    if (w < nwords) lw[w] = sw[c];
  }
  __syncthreads();
  if (ss.done) return;   // the same LDS word for every thread
  if (threadIdx.x < WAVE) scalar_program(&ss, sums, phase, i, j, n);
  __syncthreads();
  for (int w = threadIdx.x; w < nwords; w += SB) gw[w] = lw[w];
}

// ---------------------------------------------------------------- vector passes

// x += alpha gh ; r -= alpha w ; sums: ||r||^2, q_s^H r for s in [d0, d0+nd).
// SW: also q_s^H w for the same s (the S column of w below its diagonal), at
// sums[1 + ND + d]; the partial rows are then 2 ND + 1 long.
// With xrec, x_k is also stored in column k-1 of the iterate record.
// XD: x is not touched (neither x nor gh is read): the update is deferred to
// k_omega, or to k_xflush when the solve ends within the cycle.
// All ND column loads of a row are issued together, before any is used: the
// columns past nd repeat column d0 (cache hits) and feed sums that no
// recurrence reads.  Loads under a per-column test are issued one at a time,
// each waited for (2-4% slower solves at n = 8, 16).  k_omega does the same.
template <class V, class Sc, int ND, bool SW, bool XD>
__global__ __launch_bounds__(BLOCK) void k_alpha(State<Sc>* st, Sc* partial, int N, V* __restrict__ x,
                                                 const V* __restrict__ gh, V* __restrict__ r, const V* __restrict__ w,
                                                 const V* __restrict__ Q, long long ldq, int d0, int nd,
                                                 V* __restrict__ xrec, long long K, int phase, int i, int j, int n,
                                                 int flags) {
  if (!(flags & F_IGNORE_DONE) && st->done) return;
  constexpr int NACC = SW ? 2 * ND + 1 : ND + 1;
  V acc[NACC];
#pragma unroll
  for (int d = 0; d < NACC; ++d) acc[d] = zero<V>();
  const V al = convert<V>(st->alpha);
  const V mal = convert<V>(zero<Sc>() - st->alpha);
  const long long k = st->iter + 1;
  V* rec = (xrec && k <= K) ? xrec + (k - 1) * (long long)N : nullptr;
  for (int row = blockIdx.x * BLOCK + threadIdx.x; row < N; row += gridDim.x * BLOCK) {
    const V wv = w[row], r0 = r[row];
    V gv = zero<V>(), x0 = zero<V>();
    if constexpr (!XD) {
      gv = gh[row];
      x0 = x[row];
    }
    V qv[ND];
    if (nd > 0) {
#pragma unroll
      for (int d = 0; d < ND; ++d) qv[d] = Q[row + (long long)(d0 + (d < nd ? d : 0)) * ldq];
    }
    if constexpr (!XD) {
      V xv = axpy(x0, al, gv);
      x[row] = xv;
      if (rec) rec[row] = xv;
    }
    V rv = axpy(r0, mal, wv);
    r[row] = rv;
    cdot_acc(acc[0], rv, rv);
    if (nd > 0) {
#pragma unroll
      for (int d = 0; d < ND; ++d) {
        cdot_acc(acc[1 + d], qv[d], rv);
        if constexpr (SW) cdot_acc(acc[1 + ND + d], qv[d], wv);
      }
    }
  }
  if (flags & F_SKIP_SCALAR) return;
  block_partials<NACC>(acc, SW ? 1 + ND + nd : nd + 1, partial);
}

// g = r + sum_{s in [t0, n)} (t_s W_s + tg_s G_s) -> gout ; sums: f_s^H g, s < nf.
// gout may be one of the G columns read (the cycle close writes g_{jn+n} over
// column 0): every row is read before the same thread writes it.
template <class V, class Sc, int ND>
__global__ __launch_bounds__(BLOCK) void k_combine(State<Sc>* st, Sc* partial, int N, const V* __restrict__ r,
                                                   const V* __restrict__ Wb, const V* Gb, long long ldw,
                                                   int t0, int t1, V* gout, const V* __restrict__ F,
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
    // columns in groups of 4, all loads of a group issued before its updates
    // (the order of the updates is unchanged)
    int s = t0;
    for (; s + 4 <= t1; s += 4) {
      V wv[4], gv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        wv[u] = Wb[row + (s + u) * ldw];
        gv[u] = Gb[row + (s + u) * ldw];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        g = axpy(g, tw[s + u], wv[u]);
        g = axpy(g, tgv[s + u], gv[u]);
      }
    }
    for (; s < t1; ++s) {
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
    int s = 0;
    for (; s + 4 <= nb; s += 4) {   // loads of 4 columns issued together, same order of updates
      V gv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) gv[u] = Gb[row + (s + u) * ldg];
#pragma unroll
      for (int u = 0; u < 4; ++u) v = axpy(v, bco[s + u], gv[u]);
    }
    for (; s < nb; ++s) v = axpy(v, bco[s], Gb[row + s * ldg]);
    gout[row] = v;
  }
}

// Transpose-free step i: g_k = g + sum_{s<i} beta_s G_s -> G_i and
// w_k = v + sum_{s<i} beta_s W_s -> W_i, where v = A g was stored in W_i by the
// SpMV pass; sums: q_s^H w_k, s in [i, n) (the S column of step i).  beta is
// staged in LDS; every row of W_i is read before the same thread writes it.
template <class V, class Sc, int ND>
__global__ __launch_bounds__(BLOCK) void k_gwcomb(State<Sc>* st, Sc* partial, int N, const V* __restrict__ g,
                                                  V* G, V* W, long long ld, int i, const V* __restrict__ Q,
                                                  long long ldq, int n, int flags) {
  if (!(flags & F_IGNORE_DONE) && st->done) return;
  __shared__ V bco[NMAX];
  if (threadIdx.x < i) bco[threadIdx.x] = convert<V>(st->beta[threadIdx.x]);
  __syncthreads();
  V acc[ND];
#pragma unroll
  for (int d = 0; d < ND; ++d) acc[d] = zero<V>();
  const int nd = n - i;
  V* Gi = G + i * ld;
  V* Wi = W + i * ld;
  for (int row = blockIdx.x * BLOCK + threadIdx.x; row < N; row += gridDim.x * BLOCK) {
    V gv = g[row];
    V wv = Wi[row];
    int s = 0;
    for (; s + 4 <= i; s += 4) {   // loads of 4 column pairs issued together, same order of updates
      V ga[4], wa[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        ga[u] = G[row + (s + u) * ld];
        wa[u] = W[row + (s + u) * ld];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        gv = axpy(gv, bco[s + u], ga[u]);
        wv = axpy(wv, bco[s + u], wa[u]);
      }
    }
    for (; s < i; ++s) {
      gv = axpy(gv, bco[s], G[row + s * ld]);
      wv = axpy(wv, bco[s], W[row + s * ld]);
    }
    Gi[row] = gv;
    Wi[row] = wv;
#pragma unroll
    for (int d = 0; d < ND; ++d)
      if (d < nd) cdot_acc(acc[d], Q[row + (long long)(i + d) * ldq], wv);
  }
  if (flags & F_SKIP_SCALAR) return;
  block_partials<ND>(acc, nd, partial);
}

// Literal order, one pass of the beta~ recurrence (coefficient s, paired with
// q_s, w_s, g_s, c_s): z_w += t_s W_s and gs += t_s G_s, where the first pass
// starts from z_w = r, gs = 0 with t_s = -e / c_s.  The sum is the next
// coefficient's q_{s+1}^H z_w; the last pass instead forms g = z_w - gs / omega
// into gout, with f_0^H g when nf = 1 (inner steps).  z_w and gs live in zw and
// gsum; gout may be zw (each row read before the same thread writes it) or a G
// column read by the pass (n = 1 at the cycle close).
template <class V, class Sc>
__global__ __launch_bounds__(BLOCK) void k_lit_tilde(State<Sc>* st, Sc* partial, int N, int s, int first, int last,
                                                     const V* __restrict__ r, const V* __restrict__ Ws, const V* Gs,
                                                     V* zw, V* __restrict__ gsum, V* gout, const V* __restrict__ qf,
                                                     int nf, int flags) {
  const int done = st->done;
  const Sc t = first ? zero<Sc>() - st->e * st->cinv[s] : st->t[s];
  const Sc mw = zero<Sc>() - sc_div(from_real<Sc>(1.0), st->omega);
  if (!(flags & F_IGNORE_DONE) && done) return;
  const V tv = convert<V>(t), mwv = convert<V>(mw);
  V acc[4] = {zero<V>(), zero<V>(), zero<V>(), zero<V>()};
  for (int row = blockIdx.x * BLOCK + threadIdx.x; row < N; row += gridDim.x * BLOCK) {
    const V z = axpy(first ? r[row] : zw[row], tv, Ws[row]);
    const V g = axpy(first ? zero<V>() : gsum[row], tv, Gs[row]);
    if (last) {
      const V gv = axpy(z, mwv, g);
      gout[row] = gv;
      if (nf) cdot_acc(acc[0], qf[row], gv);
    } else {
      zw[row] = z;
      gsum[row] = g;
      cdot_acc(acc[0], qf[row], z);
    }
  }
  if ((flags & F_SKIP_SCALAR) || (last && !nf)) return;
  block_partials<4>(acc, 1, partial);
}

// Literal order, one pass of the beta recurrence (coefficient s, paired with
// f_s, g_s, c_s): g += beta_s G_s in place; the sum is the next coefficient's
// f_{s+1}^H g.  The last pass writes g_k into gout (its G column) instead.
template <class V, class Sc>
__global__ __launch_bounds__(BLOCK) void k_lit_beta(State<Sc>* st, Sc* partial, int N, int s, int last, V* g,
                                                    const V* __restrict__ Gs, V* __restrict__ gout,
                                                    const V* __restrict__ fnext, int flags) {
  const int done = st->done;
  const Sc b = st->beta[s];
  if (!(flags & F_IGNORE_DONE) && done) return;
  const V bv = convert<V>(b);
  V acc[4] = {zero<V>(), zero<V>(), zero<V>(), zero<V>()};
  for (int row = blockIdx.x * BLOCK + threadIdx.x; row < N; row += gridDim.x * BLOCK) {
    const V v = axpy(g[row], bv, Gs[row]);
    if (last) {
      gout[row] = v;
    } else {
      g[row] = v;
      cdot_acc(acc[0], fnext[row], v);
    }
  }
  if ((flags & F_SKIP_SCALAR) || last) return;
  block_partials<4>(acc, 1, partial);
}

// x += omega u ; r = u - omega z (u held in r) ; sums: ||r||^2, q_s^H r, s < nd.
// XD: first the cycle's deferred alpha steps, x += alph[t] G_t for t < npend in
// order (the same fused multiply-adds, in the same order, as the alpha passes
// would have made), then the omega step.
template <class V, class Sc, int ND, bool XD>
__global__ __launch_bounds__(BLOCK) void k_omega(State<Sc>* st, Sc* partial, int N, V* __restrict__ x,
                                                 V* __restrict__ r, const V* __restrict__ z, const V* __restrict__ Q,
                                                 long long ldq, int nd, V* __restrict__ xrec, long long K, int phase,
                                                 int n, int flags, const V* __restrict__ G, long long ldg) {
  if (!(flags & F_IGNORE_DONE) && st->done) return;
  V acc[ND + 1];
#pragma unroll
  for (int d = 0; d <= ND; ++d) acc[d] = zero<V>();
  const V om = convert<V>(st->omega);
  const V mom = convert<V>(zero<Sc>() - st->omega);
  const long long k = st->iter + 1;
  V* rec = (xrec && k <= K) ? xrec + (k - 1) * (long long)N : nullptr;
  __shared__ V ca[NMAX];
  int np = 0;
  if constexpr (XD) {
    np = st->npend;
    if (threadIdx.x < np) ca[threadIdx.x] = convert<V>(st->alph[threadIdx.x]);
    __syncthreads();
  }
  for (int row = blockIdx.x * BLOCK + threadIdx.x; row < N; row += gridDim.x * BLOCK) {
    const V u = r[row], x0 = x[row], zv = z[row];
    V qv[ND];
#pragma unroll
    for (int d = 0; d < ND; ++d) qv[d] = Q[row + (long long)(d < nd ? d : 0) * ldq];
    V xa = x0;
    if constexpr (XD) {
      for (int t4 = 0; t4 < np; t4 += 4) {   // columns in groups of 4, loads issued together
        V gv[4];
#pragma unroll
        for (int u4 = 0; u4 < 4; ++u4) gv[u4] = G[row + (long long)(t4 + u4 < np ? t4 + u4 : np - 1) * ldg];
#pragma unroll
        for (int u4 = 0; u4 < 4; ++u4)
          if (t4 + u4 < np) xa = axpy(xa, ca[t4 + u4], gv[u4]);
      }
    }
    V xv = axpy(xa, om, u);
    x[row] = xv;
    if (rec) rec[row] = xv;
    V rv = axpy(u, mom, zv);
    r[row] = rv;
    cdot_acc(acc[0], rv, rv);
#pragma unroll
    for (int d = 0; d < ND; ++d) cdot_acc(acc[1 + d], qv[d], rv);
  }
  if (flags & F_SKIP_SCALAR) return;
  block_partials<ND + 1>(acc, nd + 1, partial);
}

// The deferred alpha steps of a solve that ended within a cycle:
// x += alph[t] G_t for t < npend, in order (nothing when npend is 0).  Runs
// after the done flag is set, so it does not test it.
template <class V, class Sc>
__global__ __launch_bounds__(BLOCK) void k_xflush(const State<Sc>* st, int N, V* __restrict__ x,
                                                  const V* __restrict__ G, long long ldg) {
  const int np = st->npend;
  if (np == 0) return;
  __shared__ V ca[NMAX];
  if (threadIdx.x < np) ca[threadIdx.x] = convert<V>(st->alph[threadIdx.x]);
  __syncthreads();
  for (int row = blockIdx.x * BLOCK + threadIdx.x; row < N; row += gridDim.x * BLOCK) {
    V xa = x[row];
    for (int t = 0; t < np; ++t) xa = axpy(xa, ca[t], G[row + (long long)t * ldg]);
    x[row] = xa;
  }
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
