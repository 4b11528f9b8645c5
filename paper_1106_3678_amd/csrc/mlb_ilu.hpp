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
// (L^{-1} v) use the same level sets (forward for L, backward for U), and
// M^{-H} v = L^{-H} (U^{-H} v) runs on the conjugate transpose of the factor
// matrix, whose lower part is U^H and whose upper part is L^H.
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

// One level of a triangular solve with a factor matrix (rows sorted).  LOWER:
// out_i = in_i - sum_{stored j < i} a_ij out_j; else out_i = in_i -
// sum_{stored j > i} a_ij out_j.  UNIT: that value is out_i; else out_i =
// a_ii^{-1} (value): a division for scalars, the stored inverse block (dinv)
// for 3x3 blocks.  The rows of a level only read out_j of earlier levels.  in
// and out are BS-vectors per (block) row; they may not overlap.  lv: the
// level's rows in solve order, {i, q0, q1, 0} with [q0, q1) the stored entries
// left (LOWER) or right of row i's diagonal, so one load gives a row and its
// range (the diagonal entry is q1, or q0 - 1).  done: the solve's done flag
// (the launch returns at once when it is set), or null outside an iteration.
template <class V, int BS, bool LOWER, bool UNIT>
__global__ void k_ilu_solve_level(const int* __restrict__ ci, const V* __restrict__ val,
                                  const V* __restrict__ dinv, const int4* __restrict__ lv, int count,
                                  const V* __restrict__ in, V* __restrict__ out, const int* done) {
  constexpr int B2 = BS * BS;
  const int t0 = blockIdx.x * blockDim.x + threadIdx.x, stride = gridDim.x * blockDim.x;
  int4 rnext = t0 < count ? lv[t0] : make_int4(0, 0, 0, 0);   // issued before the flag test
  if (done && *(volatile const int*)done) return;
  for (int t = t0; t < count; t += stride) {
    const int4 rw = rnext;
    if (t + stride < count) rnext = lv[t + stride];
    const int i = rw.x, q0 = rw.y, q1 = rw.z;
    const int qd = LOWER ? q1 : q0 - 1;
    V s[BS];
#pragma unroll
    for (int e = 0; e < BS; ++e) s[e] = in[(size_t)BS * i + e];
    // entries in groups of 4: their indices and values loaded together, then the solved
    // values they reference, then the updates in entry order (past q1: entry q1 - 1 again,
    // unused)
    for (int q4 = q0; q4 < q1; q4 += 4) {
      int c[4];
      V a[4][B2], xv[4][BS];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int q = q4 + u < q1 ? q4 + u : q1 - 1;
        c[u] = ci[q];
#pragma unroll
        for (int e = 0; e < B2; ++e) a[u][e] = val[(size_t)B2 * q + e];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int e = 0; e < BS; ++e) xv[u][e] = out[(size_t)BS * c[u] + e];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (q4 + u < q1) {
#pragma unroll
          for (int r = 0; r < BS; ++r) {
            V acc = zero<V>();
#pragma unroll
            for (int k = 0; k < BS; ++k) acc = axpy(acc, a[u][BS * r + k], xv[u][k]);
            s[r] = s[r] - acc;
          }
        }
    }
    if constexpr (UNIT) {
#pragma unroll
      for (int e = 0; e < BS; ++e) out[(size_t)BS * i + e] = s[e];
    } else if constexpr (BS == 1) {
      out[i] = s[0] / val[qd];
    } else {
      const V* di = dinv + (size_t)B2 * i;
#pragma unroll
      for (int r = 0; r < BS; ++r) {
        V acc = zero<V>();
#pragma unroll
        for (int k = 0; k < BS; ++k) acc = axpy(acc, di[BS * r + k], s[k]);
        out[(size_t)BS * i + r] = acc;
      }
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
