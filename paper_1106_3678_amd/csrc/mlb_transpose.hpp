// Explicit conjugate transpose A^H on the device (CSR and 3x3-block BSR).
//
// Algorithm 4.1 forms f_s = A^H q_s once, before the iteration; the library
// keeps A^H as its own CSR/BSR3 copy so that this product is a row-parallel
// SpMV like every other.  The construction is a counting sort by column:
// count entries per column (integer atomics), exclusive scan into the row
// pointer of A^H, scatter with per-column atomic slots, then sort every row
// of A^H by its column index.  The final sort makes the result independent
// of the order the atomics happened to run in, so A^H (and everything
// computed from it) is bitwise reproducible.
#pragma once

#include <hip/hip_runtime.h>

#include "mlb_types.hpp"

namespace mlb {

__global__ void k_col_count(const int* __restrict__ ci, long long nnz, int* __restrict__ cnt) {
  for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < nnz; q += (long long)gridDim.x * blockDim.x)
    atomicAdd(&cnt[ci[q]], 1);
}

// Exclusive scan of cnt[0..m) into out[0..m], out[m] = total, in three passes:
// per-tile sums (tiles of SCAN_TILE entries, one workgroup each), one
// workgroup scanning the tile sums, then every tile rescanned from its offset.
constexpr int SCAN_T = 1024, SCAN_ITEMS = 8, SCAN_TILE = SCAN_T * SCAN_ITEMS;

// Inclusive scan of one value per thread across the workgroup (Hillis-Steele in
// LDS); returns this thread's inclusive prefix, and the total in *total.
__device__ inline int block_scan_incl(int v, int* part, int* total) {
  part[threadIdx.x] = v;
  __syncthreads();
  for (int off = 1; off < SCAN_T; off <<= 1) {
    const int add = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += add;
    __syncthreads();
  }
  const int r = part[threadIdx.x];
  *total = part[SCAN_T - 1];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_tiles(const int* __restrict__ cnt, long long m, int* __restrict__ tsum) {
  __shared__ int part[SCAN_T];
  const long long my = (long long)blockIdx.x * SCAN_TILE + (long long)threadIdx.x * SCAN_ITEMS;
  int sum = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) sum += my + k < m ? cnt[my + k] : 0;
  int total;
  block_scan_incl(sum, part, &total);
  if (threadIdx.x == 0) tsum[blockIdx.x] = total;
}

// Exclusive scan of the ntiles tile sums in place (one workgroup), total in tsum[ntiles].
__global__ __launch_bounds__(SCAN_T) void k_scan_sums(int* __restrict__ tsum, int ntiles) {
  __shared__ int part[SCAN_T];
  __shared__ int carry_s;
  if (threadIdx.x == 0) carry_s = 0;
  __syncthreads();
  for (int base = 0; base < ntiles; base += SCAN_T) {
    const int i = base + threadIdx.x;
    const int v = i < ntiles ? tsum[i] : 0;
    int total;
    const int incl = block_scan_incl(v, part, &total);
    const int carry = carry_s;
    if (i < ntiles) tsum[i] = carry + incl - v;
    __syncthreads();
    if (threadIdx.x == 0) carry_s = carry + total;
    __syncthreads();
  }
  if (threadIdx.x == 0) tsum[ntiles] = carry_s;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_apply(const int* __restrict__ cnt, long long m,
                                                       const int* __restrict__ toff, int ntiles, int* __restrict__ out) {
  __shared__ int part[SCAN_T];
  const long long my = (long long)blockIdx.x * SCAN_TILE + (long long)threadIdx.x * SCAN_ITEMS;
  int v[SCAN_ITEMS];
  int sum = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    v[k] = my + k < m ? cnt[my + k] : 0;
    sum += v[k];
  }
  int total;
  int run = toff[blockIdx.x] + block_scan_incl(sum, part, &total) - sum;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    if (my + k < m) out[my + k] = run;
    run += v[k];
  }
  if (blockIdx.x == ntiles - 1 && threadIdx.x == 0) out[m] = toff[ntiles];
}

// Scatter entry (row, c) of A to row c of A^H as conj(value) (CSR), or the
// conjugate-transposed 3x3 block (BSR3).
template <class V, int BS>
__global__ void k_scatter(const int* __restrict__ rp, const int* __restrict__ ci, const V* __restrict__ val, int nrows,
                          const int* __restrict__ rpT, int* __restrict__ fill, int* __restrict__ ciT,
                          V* __restrict__ valT) {
  for (int row = blockIdx.x * blockDim.x + threadIdx.x; row < nrows; row += gridDim.x * blockDim.x) {
    for (int q = rp[row]; q < rp[row + 1]; ++q) {
      const int c = ci[q];
      const int pos = rpT[c] + atomicAdd(&fill[c], 1);
      ciT[pos] = row;
      if (BS == 1) {
        valT[pos] = conj(val[q]);
      } else {
        const V* b = val + (size_t)9 * q;
        V* o = valT + (size_t)9 * pos;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int e = 0; e < 3; ++e) o[3 * a + e] = conj(b[3 * e + a]);
      }
    }
  }
}

// Sort every row of A^H by column (insertion sort; rows are short).
template <class V, int BS>
__global__ void k_sort_rows(const int* __restrict__ rpT, int nrows, int* __restrict__ ciT, V* __restrict__ valT) {
  for (int row = blockIdx.x * blockDim.x + threadIdx.x; row < nrows; row += gridDim.x * blockDim.x) {
    const int beg = rpT[row], end = rpT[row + 1];
    for (int a = beg + 1; a < end; ++a) {
      const int key = ciT[a];
      V tmp[BS];
#pragma unroll
      for (int e = 0; e < BS; ++e) tmp[e] = valT[(size_t)BS * a + e];
      int b = a - 1;
      while (b >= beg && ciT[b] > key) {
        ciT[b + 1] = ciT[b];
#pragma unroll
        for (int e = 0; e < BS; ++e) valT[(size_t)BS * (b + 1) + e] = valT[(size_t)BS * b + e];
        --b;
      }
      ciT[b + 1] = key;
#pragma unroll
      for (int e = 0; e < BS; ++e) valT[(size_t)BS * (b + 1) + e] = tmp[e];
    }
  }
}

// Narrowing copy of matrix values (fp64 -> fp32) for the fp32 inner iteration.
template <class To, class From>
__global__ void k_narrow(To* __restrict__ out, const From* __restrict__ in, long long m) {
  for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < m; q += (long long)gridDim.x * blockDim.x)
    out[q] = convert<To>(in[q]);
}

}  // namespace mlb
