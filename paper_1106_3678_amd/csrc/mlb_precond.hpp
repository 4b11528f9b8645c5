// Block-Jacobi right preconditioning for Algorithm 7.1 (Section 7).
//
// With M = the block diagonal of A (3x3 blocks for BSR3, the diagonal for
// CSR), Algorithm 7.1 is Algorithm 4.1 applied to A M^{-1} y = b followed by
// x = M^{-1} y.  The library forms A M^{-1} once (every stored block times the
// inverse diagonal block of its column), runs the unpreconditioned iteration on
// it with y_0 = M x_0, and maps the result back with x = M^{-1} y.  The
// residual of the scaled system equals b - A x, so the stopping test is the
// paper's.  f_s = M^{-H} A^H q_s is (A M^{-1})^H q_s, i.e. the conjugate
// transpose of the scaled matrix applied to q_s.
#pragma once

#include <hip/hip_runtime.h>

#include "mlb_types.hpp"

namespace mlb {

// 3x3 inverse by cofactors; returns false for a zero or non-finite determinant.
template <class V>
__device__ inline bool inv3(const V* a, V* o) {
  const V c00 = a[4] * a[8] - a[5] * a[7];
  const V c01 = a[5] * a[6] - a[3] * a[8];
  const V c02 = a[3] * a[7] - a[4] * a[6];
  const V det = a[0] * c00 + a[1] * c01 + a[2] * c02;
  if (is_zero(det) || !finite(det)) return false;
  const V one = from_real<V>(1.0);
  const V r = one / det;
  o[0] = c00 * r;
  o[1] = (a[2] * a[7] - a[1] * a[8]) * r;
  o[2] = (a[1] * a[5] - a[2] * a[4]) * r;
  o[3] = c01 * r;
  o[4] = (a[0] * a[8] - a[2] * a[6]) * r;
  o[5] = (a[2] * a[3] - a[0] * a[5]) * r;
  o[6] = c02 * r;
  o[7] = (a[1] * a[6] - a[0] * a[7]) * r;
  o[8] = (a[0] * a[4] - a[1] * a[3]) * r;
  return true;
}

// Diagonal (block) of every (block) row and its inverse.  bad |= 1: no stored
// diagonal entry; bad |= 2: singular (or non-finite) diagonal (block).
template <class V, int BS>
__global__ void k_diag_inverse(const int* __restrict__ rp, const int* __restrict__ ci, const V* __restrict__ val,
                               int nbrows, V* __restrict__ Mblk, V* __restrict__ Minv, int* __restrict__ bad) {
  constexpr int B2 = BS * BS;
  for (int row = blockIdx.x * blockDim.x + threadIdx.x; row < nbrows; row += gridDim.x * blockDim.x) {
    int qd = -1;
    for (int q = rp[row]; q < rp[row + 1]; ++q)
      if (ci[q] == row) { qd = q; break; }
    V* mb = Mblk + (size_t)B2 * row;
    V* mi = Minv + (size_t)B2 * row;
    if (qd < 0) {
      atomicOr(bad, 1);
      for (int e = 0; e < B2; ++e) mb[e] = mi[e] = from_real<V>((e % (BS + 1)) == 0 ? 1.0 : 0.0);
      continue;
    }
    const V* d = val + (size_t)B2 * qd;
    for (int e = 0; e < B2; ++e) mb[e] = d[e];
    if constexpr (BS == 1) {
      if (is_zero(d[0]) || !finite(d[0])) { atomicOr(bad, 2); mi[0] = from_real<V>(1.0); }
      else mi[0] = from_real<V>(1.0) / d[0];
    } else {
      if (!inv3(d, mi)) {
        atomicOr(bad, 2);
        for (int e = 0; e < 9; ++e) mi[e] = from_real<V>((e % 4) == 0 ? 1.0 : 0.0);
      }
    }
  }
}

// out = A M^{-1}: entry (row, c) times the inverse diagonal (block) of column c.
template <class V, int BS>
__global__ void k_right_scale(const int* __restrict__ rp, const int* __restrict__ ci, const V* __restrict__ val,
                              int nbrows, const V* __restrict__ Minv, V* __restrict__ out) {
  constexpr int B2 = BS * BS;
  for (int row = blockIdx.x * blockDim.x + threadIdx.x; row < nbrows; row += gridDim.x * blockDim.x) {
    for (int q = rp[row]; q < rp[row + 1]; ++q) {
      const V* a = val + (size_t)B2 * q;
      const V* m = Minv + (size_t)B2 * ci[q];
      V* o = out + (size_t)B2 * q;
      for (int r = 0; r < BS; ++r)
        for (int c = 0; c < BS; ++c) {
          V acc = zero<V>();
          for (int k = 0; k < BS; ++k) acc = axpy(acc, a[BS * r + k], m[BS * k + c]);
          o[BS * r + c] = acc;
        }
    }
  }
}

// X <- blockdiag(blk) X for ncols columns of length nbrows * BS (leading dimension ld), in place.
template <class V, int BS>
__global__ void k_block_apply(const V* __restrict__ blk, V* __restrict__ X, int nbrows, int ncols, long long ld) {
  constexpr int B2 = BS * BS;
  const long long total = (long long)nbrows * ncols;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total; t += (long long)gridDim.x * blockDim.x) {
    const int row = (int)(t % nbrows);
    const long long col = t / nbrows;
    V* x = X + col * ld + (long long)BS * row;
    const V* m = blk + (size_t)B2 * row;
    V in[BS];
    for (int k = 0; k < BS; ++k) in[k] = x[k];
    for (int r = 0; r < BS; ++r) {
      V acc = zero<V>();
      for (int k = 0; k < BS; ++k) acc = axpy(acc, m[BS * r + k], in[k]);
      x[r] = acc;
    }
  }
}

}  // namespace mlb
