// One-workgroup solves of small systems, many systems per launch.
//
// For small N the multi-launch iteration is bound by launch latency (seven
// launches per step, each a few microseconds whatever N is).  Here workgroup b
// of a launch runs the whole of Algorithm 7.1 (M = I) for system b: the same
// passes, coefficient recurrences and exits as the multi-launch path, with
// workgroup barriers in place of kernel boundaries, the sums reduced in LDS
// and the scalar state kept in LDS.  Systems are independent, so a result
// does not depend on which other systems share the launch.  The vectors of a
// system stay in the L2 / Infinity Cache at the sizes this path is used for.
// Every workgroup ends after at most maxit / n + 2 cycles.  A system may also
// run the transpose-free steps (no A^H and no F; the same passes as the
// multi-launch engine's spmv_h and k_gwcomb).
#pragma once

#include "mlb_kernels.hpp"

namespace mlb {

constexpr int SB = 512;   // threads of a small-solve workgroup (8 waves)

template <class V, class Sc>
struct SmallJob {
  int N = 0, n = 0;
  const int* rp = nullptr;    // A, CSR
  const int* ci = nullptr;
  const V* val = nullptr;
  const int* rpT = nullptr;   // A^H, CSR
  const int* ciT = nullptr;
  const V* valT = nullptr;
  const V* b = nullptr;
  V* x = nullptr;
  const V* Q = nullptr;
  long long ldq = 0;
  V *G = nullptr, *W = nullptr, *F = nullptr;   // N x n, N x n, N x (n-1); ld = N
  V *r = nullptr, *gt = nullptr, *z = nullptr;
  State<Sc>* st = nullptr;    // receives the final state
  V* xrec = nullptr;          // iterate record: x_k in column k-1, k <= K (or null)
  long long K = 0;
  double tol = 0, kappa = 0;
  long long maxit = 0;
  int* host_done = nullptr;   // host-mapped done flag, or null
  int tf = 0;                 // transpose-free inner steps (rpT, ciT, valT and F unused)
};

// Workgroup sums of acc[0..nd) into sums[0..nd) (LDS), fixed order: a tree
// over each wave, then the waves in order.  Ends with a barrier.
template <int ND, class V, class Sc>
__device__ inline void wg_sums(V (&acc)[ND], int nd, Sc* sums) {
  __shared__ V red[SB / WAVE][ND];
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
    for (int w = 1; w < SB / WAVE; ++w) add_(v, red[w][threadIdx.x]);
    sums[threadIdx.x] = convert<Sc>(v);
  }
  __syncthreads();
}

// The iteration of one system by the calling workgroup (state in ss).
template <class V, class Sc, int NB>
__device__ __forceinline__ void small_solve(const SmallJob<V, Sc>& J, State<Sc>& ss, Sc* sums) {
  constexpr int NA = NB + 1;
  const int tid = threadIdx.x, N = J.N, n = J.n;
  const long long ldq = J.ldq;
  V acc[NA];
  auto clear = [&] {
#pragma unroll
    for (int d = 0; d < NA; ++d) acc[d] = zero<V>();
  };
  // the recurrence of `phase` on wave 0; true once the solve has ended
  auto program = [&](int nsum, int phase, int i, int j) {
    wg_sums<NA>(acc, nsum, sums);
    if (tid < WAVE) scalar_program(&ss, sums, phase, i, j, n);
    __syncthreads();
    return ss.done != 0;
  };
  // Every pass takes UR rows per thread at a time (rows r0 + u * SB) and issues
  // all loads of those rows before any store, so that each wave keeps UR rows
  // of loads in flight (the stores of one row could alias the loads of the
  // next, which keeps the compiler from overlapping them by itself).
  constexpr int UR = sizeof(V) * NB <= 64 ? (sizeof(V) > 8 ? 2 : 4) : (sizeof(V) * NB <= 128 ? 2 : 1);
  // y = A xin (CSR, one row per lane) with the epilogue of `mode`.  The first
  // RB entries of a row are loaded in one batch (then their inputs in one
  // batch): a row of up to RB entries costs three dependent loads.
  auto spmv = [&](const int* rp, const int* ci, const V* val, const V* xin, V* out1, V* out2, int mode, int d0,
                  int nd) {
    constexpr int RB = 8, US = UR > 1 ? 2 : 1;
    clear();
    for (int r0 = tid; r0 < N; r0 += SB * US) {
      int beg[US], end[US];
#pragma unroll
      for (int u = 0; u < US; ++u) {
        const int row = r0 + u * SB;
        beg[u] = row < N ? rp[row] : 0;
        end[u] = row < N ? rp[row + 1] : 0;
      }
      int c[US][RB];
      V v[US][RB];
#pragma unroll
      for (int u = 0; u < US; ++u)
#pragma unroll
        for (int k = 0; k < RB; ++k) {
          const bool on = beg[u] + k < end[u];
          c[u][k] = on ? ci[beg[u] + k] : 0;
          v[u][k] = on ? val[beg[u] + k] : zero<V>();
        }
      V y[US];
#pragma unroll
      for (int u = 0; u < US; ++u) {
        V xs[RB];
#pragma unroll
        for (int k = 0; k < RB; ++k) xs[k] = xin[c[u][k]];
        y[u] = zero<V>();
#pragma unroll
        for (int k = 0; k < RB; ++k)
          if (beg[u] + k < end[u]) y[u] = axpy(y[u], v[u][k], xs[k]);
        for (int q = beg[u] + RB; q < end[u]; ++q) y[u] = axpy(y[u], val[q], xin[ci[q]]);
      }
#pragma unroll
      for (int u = 0; u < US; ++u) {
        const int row = r0 + u * SB;
        if (row >= N) break;
        if (mode == SM_RESID) {
          const V bv = J.b[row];
          const V rv = bv - y[u];
          out1[row] = rv;
          cdot_acc(acc[0], rv, rv);
          cdot_acc(acc[1], bv, bv);
          cdot_acc(acc[2], J.Q[row], rv);
        } else if (mode == SM_STEP) {
          out1[row] = y[u];
          if (out2) out2[row] = xin[row];
#pragma unroll
          for (int d = 0; d < NB; ++d)
            if (d < nd) cdot_acc(acc[d], J.Q[row + (long long)(d0 + d) * ldq], y[u]);
        } else if (mode == SM_OMEGA) {
          out1[row] = y[u];
          cdot_acc(acc[0], y[u], y[u]);
          cdot_acc(acc[1], y[u], xin[row]);
        } else {
          out1[row] = y[u];
        }
      }
    }
    __syncthreads();
  };
  // x += alpha g_prev ; r -= alpha w_prev ; ||r||^2, q_s^H r (s in [d0, d0+nd))
  auto alpha = [&](int iprev, int d0, int nd, int phase, int i, int j) {
    clear();
    const V al = convert<V>(ss.alpha), mal = convert<V>(zero<Sc>() - ss.alpha);
    const V* gh = J.G + (size_t)iprev * N;
    const V* w = J.W + (size_t)iprev * N;
    const long long k = ss.iter + 1;
    V* rec = (J.xrec && k <= J.K) ? J.xrec + (k - 1) * (long long)N : nullptr;
    for (int r0 = tid; r0 < N; r0 += SB * UR) {
      V xv[UR], gv[UR], rv[UR], wv[UR];
#pragma unroll
      for (int u = 0; u < UR; ++u) {
        const int row = min(r0 + u * SB, N - 1);   // rows past N re-read row N - 1, unused
        xv[u] = J.x[row];
        gv[u] = gh[row];
        rv[u] = J.r[row];
        wv[u] = w[row];
      }
#pragma unroll
      for (int u = 0; u < UR; ++u) {
        const int row = r0 + u * SB;
        if (row >= N) break;
        const V xn = axpy(xv[u], al, gv[u]);
        J.x[row] = xn;
        if (rec) rec[row] = xn;
        const V rn = axpy(rv[u], mal, wv[u]);
        J.r[row] = rn;
        cdot_acc(acc[0], rn, rn);
#pragma unroll
        for (int d = 0; d < NB; ++d)
          if (d < nd) cdot_acc(acc[1 + d], J.Q[row + (long long)(d0 + d) * ldq], rn);
      }
    }
    __syncthreads();
    return program(nd + 1, phase, i, j);
  };
  // gt = r + sum_{s in [t0, t1)} (t_s W_s + tg_s G_s) ; f_s^H gt (s < nf)
  auto combine = [&](int t0, int t1, int nf, int i, int j) {
    clear();
    for (int r0 = tid; r0 < N; r0 += SB * UR) {
      V g[UR];
      int rows[UR];
#pragma unroll
      for (int u = 0; u < UR; ++u) {
        rows[u] = min(r0 + u * SB, N - 1);
        g[u] = J.r[rows[u]];
      }
      for (int s = t0; s < t1; ++s) {
        const V ts = convert<V>(ss.t[s]), tgs = convert<V>(ss.tg[s]);
        V wv[UR], gv[UR];
#pragma unroll
        for (int u = 0; u < UR; ++u) {
          wv[u] = J.W[rows[u] + (size_t)s * N];
          gv[u] = J.G[rows[u] + (size_t)s * N];
        }
#pragma unroll
        for (int u = 0; u < UR; ++u) {
          g[u] = axpy(g[u], ts, wv[u]);
          g[u] = axpy(g[u], tgs, gv[u]);
        }
      }
#pragma unroll
      for (int u = 0; u < UR; ++u) {
        const int row = r0 + u * SB;
        if (row >= N) break;
        J.gt[row] = g[u];
#pragma unroll
        for (int d = 0; d < NB; ++d)
          if (d < nf) cdot_acc(acc[d], J.F[row + (size_t)d * N], g[u]);
      }
    }
    __syncthreads();
    return nf > 0 ? program(nf, PH_COMBINE, i, j) : false;
  };
  // G_i = g0 + sum_{s<i} beta_s G_s.  Transpose-free (wi): v = A g was stored in W_i, and
  // also W_i = v + sum_{s<i} beta_s W_s with its S column, c_i and alpha (returns true
  // once the solve has ended); otherwise returns false.
  auto gcomb = [&](const V* g0, int i, bool wi) {
    clear();
    for (int r0 = tid; r0 < N; r0 += SB * UR) {
      V v[UR], wv[UR];
      int rows[UR];
#pragma unroll
      for (int u = 0; u < UR; ++u) {
        rows[u] = min(r0 + u * SB, N - 1);   // rows past N re-read row N - 1, unused
        v[u] = g0[rows[u]];
        wv[u] = wi ? J.W[rows[u] + (size_t)i * N] : zero<V>();
      }
      for (int s = 0; s < i; ++s) {
        const V bs = convert<V>(ss.beta[s]);
        V gv[UR];
#pragma unroll
        for (int u = 0; u < UR; ++u) gv[u] = J.G[rows[u] + (size_t)s * N];
        if (wi) {
          V wa[UR];
#pragma unroll
          for (int u = 0; u < UR; ++u) wa[u] = J.W[rows[u] + (size_t)s * N];
#pragma unroll
          for (int u = 0; u < UR; ++u) wv[u] = axpy(wv[u], bs, wa[u]);
        }
#pragma unroll
        for (int u = 0; u < UR; ++u) v[u] = axpy(v[u], bs, gv[u]);
      }
#pragma unroll
      for (int u = 0; u < UR; ++u) {
        const int row = r0 + u * SB;
        if (row >= N) break;
        J.G[row + (size_t)i * N] = v[u];
        if (wi) {
          J.W[row + (size_t)i * N] = wv[u];
#pragma unroll
          for (int d = 0; d < NB; ++d)
            if (d < n - i) cdot_acc(acc[d], J.Q[row + (long long)(i + d) * ldq], wv[u]);
        }
      }
    }
    __syncthreads();
    return wi ? program(n - i, PH_SPMV_STEP, i, 0) : false;
  };
  // W_i = A gin (G_i = gin when gin is another vector) ; S column i, c_i, alpha
  auto step = [&](const V* gin, int i) {
    V* Gi = J.G + (size_t)i * N;
    spmv(J.rp, J.ci, J.val, gin, J.W + (size_t)i * N, gin == Gi ? nullptr : Gi, SM_STEP, i, n - i);
    return program(n - i, PH_SPMV_STEP, i, 0);
  };

  // set-up: r_0 = b - A x_0, ||b||, e_0 ; F = A^H Q(:, 0:n-1) ; w_0 = A r_0
  spmv(J.rp, J.ci, J.val, J.x, J.r, nullptr, SM_RESID, 0, 0);
  if (program(3, PH_SETUP, 0, 0)) return;
  if (!J.tf)
    for (int c = 0; c + 1 < n; ++c)
      spmv(J.rpT, J.ciT, J.valT, J.Q + (size_t)c * ldq, J.F + (size_t)c * N, nullptr, SM_PLAIN, 0, 0);
  if (step(J.r, 0)) return;
  const long long max_cycles = J.maxit / n + 2;
  for (long long jj = 0; jj <= max_cycles; ++jj) {
    const int j = jj >= 1 ? 1 : 0;
    for (int i = 1; i < n; ++i) {
      if (alpha(i - 1, i, j >= 1 ? n - i : 1, PH_INNER, i, j)) return;
      if (J.tf) {
        // g = z_w - g/omega (j >= 1) or r (j = 0); v = A g -> W_i with q_s^H v (s < i), beta;
        // then g_{jn+i}, w_{jn+i} recombined with the S column
        const V* g0 = J.r;
        if (j >= 1) {
          combine(i, n, 0, i, j);
          g0 = J.gt;
        }
        spmv(J.rp, J.ci, J.val, g0, J.W + (size_t)i * N, nullptr, SM_STEP, 0, i);
        if (program(i, PH_COMBINE, i, j)) return;
        if (gcomb(g0, i, true)) return;
        continue;
      }
      if (combine(i, j >= 1 ? n : i, i, i, j)) return;
      gcomb(J.gt, i, false);
      if (step(J.G + (size_t)i * N, i)) return;
    }
    // k = jn + n: half step, minimisation step, cycle close
    if (alpha(n - 1, 0, 0, PH_HALF, n, j)) return;
    spmv(J.rp, J.ci, J.val, J.r, J.z, nullptr, SM_OMEGA, 0, 0);
    if (program(2, PH_SPMV_OMEGA, 0, 0)) return;
    {
      clear();
      const V om = convert<V>(ss.omega), mom = convert<V>(zero<Sc>() - ss.omega);
      const long long k = ss.iter + 1;
      V* rec = (J.xrec && k <= J.K) ? J.xrec + (k - 1) * (long long)N : nullptr;
      for (int r0 = tid; r0 < N; r0 += SB * UR) {
        V uv[UR], xv[UR], zv[UR];
#pragma unroll
        for (int u = 0; u < UR; ++u) {
          const int row = min(r0 + u * SB, N - 1);
          uv[u] = J.r[row];
          xv[u] = J.x[row];
          zv[u] = J.z[row];
        }
#pragma unroll
        for (int u = 0; u < UR; ++u) {
          const int row = r0 + u * SB;
          if (row >= N) break;
          const V xn = axpy(xv[u], om, uv[u]);
          J.x[row] = xn;
          if (rec) rec[row] = xn;
          const V rn = axpy(uv[u], mom, zv[u]);
          J.r[row] = rn;
          cdot_acc(acc[0], rn, rn);
#pragma unroll
          for (int d = 0; d < NB; ++d)
            if (d < n) cdot_acc(acc[1 + d], J.Q[row + (long long)d * ldq], rn);
        }
      }
      __syncthreads();
      if (program(n + 1, PH_OMEGA_UPD, 0, 1)) return;
    }
    combine(0, n, 0, 0, j);
    if (step(J.gt, 0)) return;
  }
}

template <class V, class Sc, int NB>
__global__ __launch_bounds__(SB) void k_small(const SmallJob<V, Sc>* __restrict__ jobs) {
  static_assert(sizeof(State<Sc>) % 8 == 0, "state is copied in 8-byte words");
  const SmallJob<V, Sc> J = jobs[blockIdx.x];
  __shared__ State<Sc> ss;
  __shared__ Sc sums[NMAX + 1];
  // the state a solve starts from
  {
    unsigned long long* lw = reinterpret_cast<unsigned long long*>(&ss);
    for (int w = threadIdx.x; w < (int)(sizeof(State<Sc>) / 8); w += SB) lw[w] = 0ull;
    __syncthreads();
    if (threadIdx.x == 0) {
      ss.flag = 1;
      ss.maxit = J.maxit;
      ss.tol = J.tol;
      ss.kappa = J.kappa;
      ss.bnrm2 = 1.0;
      ss.omega = from_real<Sc>(1.0);
      ss.host_done = J.host_done;
    }
    __syncthreads();
  }
  small_solve<V, Sc, NB>(J, ss, sums);
  __syncthreads();
  unsigned long long* gw = reinterpret_cast<unsigned long long*>(J.st);
  const unsigned long long* lw = reinterpret_cast<const unsigned long long*>(&ss);
  for (int w = threadIdx.x; w < (int)(sizeof(State<Sc>) / 8); w += SB) gw[w] = lw[w];
}

}  // namespace mlb
