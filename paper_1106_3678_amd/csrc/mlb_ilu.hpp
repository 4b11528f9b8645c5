// ILU(0) right preconditioning for Algorithm 7.1 (Section 7), the
// preconditioner of the paper's experiments (Section 5).
//
// M = L U with L unit lower and U upper triangular (3x3 blocks for BSR3: L with
// identity diagonal blocks, U with full ones), both on A's pattern, and
// (L U)_ij = a_ij wherever A is stored.  The factors live in one matrix with
// A's pattern, each row sorted by column: the entries left of the diagonal are
// L, the rest U.  The factorisation eliminates row by row: for every stored
// k < i of row i, in increasing k, l_ik = a_ik u_kk^{-1}, then a_ij -= l_ik u_kj
// for every stored j > k of row i that row k also stores.  A row only reads
// rows k < i of its own pattern, so all the rows of one level (rows whose
// longest chain of such dependencies has the same length) are factored
// together, one launch per level.  The triangular solves of M^{-1} v = U^{-1}
// (L^{-1} v) take the rows in the same level order (forward for L, backward
// for U), one launch per solve (k_ilu_solve_sweep), and M^{-H} v = L^{-H}
// (U^{-H} v) runs on the conjugate transpose of the factor matrix, whose lower
// part is U^H and whose upper part is L^H.
//
// The engine iterates on A M^{-1} y = b: every product with A is preceded by
// M^{-1} applied to its input, F = M^{-H} A^H Q(:, 1:n-1), y_0 = M x_0 and
// x = M^{-1} y at the end.
#pragma once

#include <hip/hip_runtime.h>

#include "mlb_precond.hpp"
#include "mlb_types.hpp"

namespace mlb {

// Position of the diagonal entry of every (block) row of a row-sorted matrix,
// and a check of its pattern.  bad |= 1: no stored diagonal; bad |= 4: a column
// stored twice in one row.
__global__ void k_ilu_diag_pos(const int* __restrict__ rp, const int* __restrict__ ci, int nbrows,
                               int* __restrict__ dpos, int* __restrict__ bad) {
  for (int row = blockIdx.x * blockDim.x + threadIdx.x; row < nbrows; row += gridDim.x * blockDim.x) {
    int qd = -1;
    for (int q = rp[row]; q < rp[row + 1]; ++q) {
      if (q > rp[row] && ci[q] == ci[q - 1]) atomicOr(bad, 4);
      if (ci[q] == row) qd = q;
    }
    if (qd < 0) atomicOr(bad, 1);
    dpos[row] = qd < 0 ? rp[row] : qd;
  }
}

// o = a b for 3x3 row-major blocks (BS = 3) or scalars (BS = 1).
template <class V, int BS>
__device__ inline void blk_mul(const V* a, const V* b, V* o) {
#pragma unroll
  for (int r = 0; r < BS; ++r)
#pragma unroll
    for (int c = 0; c < BS; ++c) {
      V acc = zero<V>();
#pragma unroll
      for (int k = 0; k < BS; ++k) acc = axpy(acc, a[BS * r + k], b[BS * k + c]);
      o[BS * r + c] = acc;
    }
}

// Factor the rows of one level in place (val holds A's values on entry, the
// factors on exit) and store the inverse of each row's diagonal (block) in
// dinv.  bad |= 2: a zero or singular pivot.
template <class V, int BS>
__global__ void k_ilu_factor_level(const int* __restrict__ rp, const int* __restrict__ ci, V* __restrict__ val,
                                   const int* __restrict__ dpos, V* __restrict__ dinv, const int* __restrict__ rows,
                                   int count, int* __restrict__ bad) {
  constexpr int B2 = BS * BS;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < count; t += gridDim.x * blockDim.x) {
    const int i = rows[t];
    const int beg = rp[i], end = rp[i + 1], qd = dpos[i];
    for (int q = beg; q < qd; ++q) {   // stored k < i, increasing
      const int k = ci[q];
      V l[B2];
      if constexpr (BS == 1) {
        l[0] = val[q] / val[dpos[k]];   // l_ik = a_ik / u_kk
      } else {
        blk_mul<V, 3>(val + (size_t)B2 * q, dinv + (size_t)B2 * k, l);   // l_ik = a_ik u_kk^{-1}
      }
#pragma unroll
      for (int e = 0; e < B2; ++e) val[(size_t)B2 * q + e] = l[e];
      // a_ij -= l_ik u_kj for stored j > k of row i that row k stores (both rows sorted)
      int p = dpos[k] + 1;
      const int pend = rp[k + 1];
      for (int q2 = q + 1; q2 < end && p < pend; ++q2) {
        const int j = ci[q2];
        while (p < pend && ci[p] < j) ++p;
        if (p < pend && ci[p] == j) {
          V prod[B2];
          blk_mul<V, BS>(l, val + (size_t)B2 * p, prod);
#pragma unroll
          for (int e = 0; e < B2; ++e) val[(size_t)B2 * q2 + e] = val[(size_t)B2 * q2 + e] - prod[e];
        }
      }
    }
    const V* d = val + (size_t)B2 * qd;
    V* di = dinv + (size_t)B2 * i;
    if constexpr (BS == 1) {
      if (is_zero(d[0]) || !finite(d[0])) {
        atomicOr(bad, 2);
        di[0] = from_real<V>(1.0);
      } else {
        di[0] = from_real<V>(1.0) / d[0];
      }
    } else {
      if (!inv3(d, di)) {
        atomicOr(bad, 2);
        for (int e = 0; e < 9; ++e) di[e] = from_real<V>((e % 4) == 0 ? 1.0 : 0.0);
      }
    }
  }
}

// Inverse of every diagonal (block) of a matrix (for the conjugate-transposed
// factor, whose diagonal blocks are U_ii^H).
template <class V, int BS>
__global__ void k_ilu_inv_diag(const V* __restrict__ val, const int* __restrict__ dpos, int nbrows,
                               V* __restrict__ dinv, int* __restrict__ bad) {
  constexpr int B2 = BS * BS;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nbrows; i += gridDim.x * blockDim.x) {
    const V* d = val + (size_t)B2 * dpos[i];
    V* di = dinv + (size_t)B2 * i;
    if constexpr (BS == 1) {
      if (is_zero(d[0]) || !finite(d[0])) { atomicOr(bad, 2); di[0] = from_real<V>(1.0); }
      else di[0] = from_real<V>(1.0) / d[0];
    } else {
      if (!inv3(d, di)) {
        atomicOr(bad, 2);
        for (int e = 0; e < 9; ++e) di[e] = from_real<V>((e % 4) == 0 ? 1.0 : 0.0);
      }
    }
  }
}

// ---- one launch per triangular solve ---------------------------------------
//
// The rows of a whole solve go through one launch, in level order: each wave
// claims the next 64 positions from a counter, so every position below a
// claimed one is claimed too, by a wave that is running.  A row waits for the
// solved values it reads (rows of earlier levels, so at lower positions) to
// arrive.  The output is first filled with a pending mark, and every solved
// value is its own completion flag: its 64-bit words are stored and read with
// agent-scope relaxed atomics, which keeps them coherent across the XCDs'
// L2 caches without a release of a whole cache.  The lowest position still
// waiting reads only finished rows, so the solve always moves on; a wave
// whose lanes wait on each other (a level boundary inside its 64 positions)
// retries its pending lanes together, so a finished lane stores before the
// others test again.

// The pending mark: a signalling-NaN bit pattern.  Arithmetic never returns
// one (it quiets NaNs); a value that would be stored with this pattern (only a
// row copied through without arithmetic, from an input that holds it) is
// stored as the canonical quiet NaN instead.
constexpr unsigned long long ILU_PENDING = 0x7FF00000000000A5ull;
constexpr unsigned long long ILU_QNAN = 0x7FF8000000000000ull;
// Wall-clock ticks (s_memrealtime, 100 MHz) one row may wait before its wait
// counts as lost, far beyond any legitimate wait (a whole solve takes a few
// ms): the row is then stored as a quiet NaN and err set, and every row still
// waiting gives up within 256 further tries, so the launch always ends.
constexpr long long ILU_WAIT_TICKS = 200000000;

__device__ inline unsigned long long ilu_ld(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void ilu_st(unsigned long long* p, unsigned long long v) {
  __hip_atomic_store(p, v == ILU_PENDING ? ILU_QNAN : v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One group of (at most) 4 entries of a row: loads the solved values they
// reference (entries at u >= cnt repeat the last one, unused) and, when none
// is pending, subtracts a_u x_u from s in entry order.  Returns false, leaving
// s as it was, while one is pending; *waitw then holds the address of a
// pending word.
template <class V, int BS>
__device__ inline bool ilu_group(const V (&a)[4][BS * BS], const int (&c)[4], int cnt, unsigned long long* ow,
                                 V (&s)[BS], unsigned long long** waitw) {
  constexpr int W = sizeof(V) / 8;
  using U = unsigned long long;
  U xw[4][BS * W];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int k = 0; k < BS * W; ++k) xw[u][k] = ilu_ld(ow + (size_t)BS * W * c[u] + k);
  bool ready = true;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int k = 0; k < BS * W; ++k)
      if (xw[u][k] == ILU_PENDING) {
        ready = false;
        *waitw = ow + (size_t)BS * W * c[u] + k;
      }
  if (!ready) return false;
#pragma unroll
  for (int u = 0; u < 4; ++u)
    if (u < cnt) {
      V xv[BS];
#pragma unroll
      for (int e = 0; e < BS; ++e) __builtin_memcpy(&xv[e], &xw[u][W * e], sizeof(V));
#pragma unroll
      for (int r = 0; r < BS; ++r) {
        V acc = zero<V>();
#pragma unroll
        for (int k = 0; k < BS; ++k) acc = axpy(acc, a[u][BS * r + k], xv[k]);
        s[r] = s[r] - acc;
      }
    }
  return true;
}

// Marks nw 64-bit words of a solve's output pending and resets the two claim
// counters (ctl[0] and ctl[1]) of the solves that follow.
__global__ void k_ilu_pending(unsigned long long* __restrict__ w, long long nw, unsigned* __restrict__ ctl,
                              const int* done) {
  if (done && *(volatile const int*)done) return;
  if (blockIdx.x == 0 && threadIdx.x < 2) ctl[threadIdx.x] = 0;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < nw; k += (long long)gridDim.x * blockDim.x)
    w[k] = ILU_PENDING;
}

// One triangular solve with a factor matrix, the same arithmetic as one
// launch per level (the same entries in the same order): LOWER: out_i = in_i -
// sum_{stored j < i} a_ij out_j, else with the stored j > i; UNIT: that value is
// out_i, else out_i = a_ii^{-1} (value) (a division for scalars, the stored
// inverse block dinv for 3x3 blocks).  lv: all m rows in level order, {i, q0,
// q1, 0} with [q0, q1) the entries left (LOWER) or right of the diagonal.  out
// must hold the pending mark (k_ilu_pending) and may not overlap in.  next: the
// output of the solve that follows, or null: row i of it is marked pending
// once in_i is read (so next may be in).  tick: this solve's claim counter, 0
// at launch; err: set to 1 when a wait ran past its bound; max_tries: tries of
// one row before it gives up regardless of time (~0u: no such limit; a small
// value forces the give-up path in tests).  done: the solve's done flag (the
// launch returns at once when it is set), or null.
template <class V, int BS, bool LOWER, bool UNIT>
__global__ __launch_bounds__(WAVE) void k_ilu_solve_sweep(const int* __restrict__ ci, const V* __restrict__ val,
                                                          const V* __restrict__ dinv, const int4* __restrict__ lv,
                                                          int m, const V* in, V* out, V* next, unsigned* tick,
                                                          unsigned* err, unsigned max_tries, const int* done) {
  constexpr int B2 = BS * BS;
  constexpr int W = sizeof(V) / 8;   // 64-bit words per value (1 real, 2 complex)
  using U = unsigned long long;
  static_assert(sizeof(V) == 8 * W, "fp64 values only");
  if (done && *(volatile const int*)done) return;
  const int lane = threadIdx.x & (WAVE - 1);
  U* ow = reinterpret_cast<U*>(out);
  for (;;) {
    unsigned base = 0;
    if (lane == 0) base = atomicAdd(tick, (unsigned)WAVE);
    base = __shfl(base, 0, WAVE);
    if (base >= (unsigned)m) return;
    const int t = (int)base + lane;
    bool pending = t < m;
    int4 rw = make_int4(0, 0, 0, 0);
    if (pending) rw = lv[t];
    const int i = rw.x, q0 = rw.y, q1 = rw.z;
    V s0[BS];
#pragma unroll
    for (int e = 0; e < BS; ++e) s0[e] = pending ? in[(size_t)BS * i + e] : zero<V>();
    if (pending && next) {
      U* nw = reinterpret_cast<U*>(next) + (size_t)BS * W * i;
#pragma unroll
      for (int k = 0; k < BS * W; ++k) nw[k] = ILU_PENDING;
    }
    // the first (at most) 4 entries, held in registers across the tries: most rows
    // have no more, and a try then reloads only the solved values they reference
    int c0[4];
    V a0[4][B2];
    const bool has0 = pending && q0 < q1;
    if (has0) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int q = q0 + u < q1 ? q0 + u : q1 - 1;
        c0[u] = ci[q];
#pragma unroll
        for (int e = 0; e < B2; ++e) a0[u][e] = val[(size_t)B2 * q + e];
      }
    }
    // the diagonal (block) inverse's operand, off the waiting path
    V dg[UNIT ? 1 : (BS == 1 ? 1 : B2)];
    if constexpr (!UNIT) {
      if (pending) {
        if constexpr (BS == 1) {
          dg[0] = val[LOWER ? q1 : q0 - 1];
        } else {
#pragma unroll
          for (int e = 0; e < B2; ++e) dg[e] = dinv[(size_t)B2 * i + e];
        }
      }
    }
    const long long t_start = wall_clock64();
    unsigned tries = 0;
    U* waitw = nullptr;   // a word the last try found pending: polled alone first
    while (__any(pending)) {
      if (pending) {
        V s[BS];
#pragma unroll
        for (int e = 0; e < BS; ++e) s[e] = s0[e];
        bool ready = !waitw || ilu_ld(waitw) != ILU_PENDING;
        if (ready) waitw = nullptr;
        if (ready && has0) ready = ilu_group<V, BS>(a0, c0, q1 - q0, ow, s, &waitw);
        // further entries in groups of 4, loaded again on every try
        for (int q4 = q0 + 4; q4 < q1 && ready; q4 += 4) {
          int c[4];
          V a[4][B2];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int q = q4 + u < q1 ? q4 + u : q1 - 1;
            c[u] = ci[q];
#pragma unroll
            for (int e = 0; e < B2; ++e) a[u][e] = val[(size_t)B2 * q + e];
          }
          ready = ilu_group<V, BS>(a, c, q1 - q4, ow, s, &waitw);
        }
        // give up on this row after ILU_WAIT_TICKS, or once another row has (err), both
        // read every 256 tries, or after max_tries tries
        bool lost = false;
        if (!ready) {
          ++tries;
          lost = tries >= max_tries ||
                 ((tries & 255u) == 0 && (wall_clock64() - t_start > ILU_WAIT_TICKS ||
                                          __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0));
          if (lost) atomicOr(err, 1u);
        }
        if (ready || lost) {
          U ww[BS * W];
          if (lost) {
#pragma unroll
            for (int k = 0; k < BS * W; ++k) ww[k] = ILU_QNAN;
          } else {
            V o[BS];
            if constexpr (UNIT) {
#pragma unroll
              for (int e = 0; e < BS; ++e) o[e] = s[e];
            } else if constexpr (BS == 1) {
              o[0] = s[0] / dg[0];
            } else {
#pragma unroll
              for (int r = 0; r < BS; ++r) {
                V acc = zero<V>();
#pragma unroll
                for (int k = 0; k < BS; ++k) acc = axpy(acc, dg[BS * r + k], s[k]);
                o[r] = acc;
              }
            }
            __builtin_memcpy(ww, o, sizeof(o));
          }
#pragma unroll
          for (int k = 0; k < BS * W; ++k) ilu_st(ow + (size_t)BS * W * i + k, ww[k]);
          pending = false;
        }
      }
      if (__any(pending)) __builtin_amdgcn_s_sleep(8);
    }
  }
}

// y = U x (the diagonal (block) and right of it) or y = L x (unit diagonal and
// left of it) of the factor matrix, every (block) row independently: the
// forward map y_0 = M x_0 = L (U x_0).
template <class V, int BS, bool LOWER>
__global__ void k_ilu_tri_matvec(const int* __restrict__ rp, const int* __restrict__ ci, const V* __restrict__ val,
                                 const int* __restrict__ dpos, int nbrows, const V* __restrict__ x,
                                 V* __restrict__ y) {
  constexpr int B2 = BS * BS;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nbrows; i += gridDim.x * blockDim.x) {
    const int qd = dpos[i];
    const int q0 = LOWER ? rp[i] : qd;
    const int q1 = LOWER ? qd : rp[i + 1];
    V s[BS];
#pragma unroll
    for (int e = 0; e < BS; ++e) s[e] = LOWER ? x[(size_t)BS * i + e] : zero<V>();
    for (int q = q0; q < q1; ++q) {
      const V* a = val + (size_t)B2 * q;
      const V* xc = x + (size_t)BS * ci[q];
#pragma unroll
      for (int r = 0; r < BS; ++r)
#pragma unroll
        for (int k = 0; k < BS; ++k) s[r] = axpy(s[r], a[BS * r + k], xc[k]);
    }
#pragma unroll
    for (int e = 0; e < BS; ++e) y[(size_t)BS * i + e] = s[e];
  }
}

}  // namespace mlb
