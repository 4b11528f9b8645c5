// Host side of the ML(n)BiCGStab library: the C ABI of include/mlbicgstab.h,
// the per-cycle launch schedule of Algorithm 7.1 (M = I; the block-Jacobi M is
// folded into A M^{-1}), in the fused order, the literal order or the
// transpose-free form, the construction of A^H, the fp32-inner /
// fp64-refinement driver, batched one-workgroup solves, sequences of systems
// with the choice of n of Section 5.2, and the serving loop.
//
// One Engine<V> owns the Krylov workspace for one value type V (fp64 or fp32,
// real or complex).  Every step of the iteration is a kernel from
// mlb_kernels.hpp; the host only enqueues them, cycle by cycle, and watches a
// host-mapped "done" flag the device raises when the solve ends.  The host
// stays at most two cycles ahead of the device, so the iteration never waits
// for the host and the kernels of at most one cycle run after the end (they
// return at once because the device flag is set).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/mlbicgstab.h"
#include "mlb_kernels.hpp"
#include "mlb_spmv.hpp"
#include "mlb_small.hpp"
#include "mlb_precond.hpp"
#include "mlb_ilu.hpp"
#include "mlb_transpose.hpp"

namespace mlb {

static thread_local std::string g_last_error;

struct Error {
  int code;
  std::string msg;
};

#define HIP_TRY(call)                                                                            \
  do {                                                                                           \
    hipError_t e_ = (call);                                                                      \
    if (e_ != hipSuccess) throw Error{MLB_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)}; \
  } while (0)

// Device allocations owned by one solver, freed together.  Stream-ordered mode
// (hipMallocAsync / hipFreeAsync on one stream) is used by the serving path, so
// that admitting or retiring a request never synchronises the whole device.
// Arena mode (arena != nullptr) allocates nothing: every request is carved,
// 256-byte aligned, from [arena, arena + cap), a region the caller owns (the
// static scratch of mlbicgstab_solve_noalloc), and nothing is freed.
constexpr size_t ARENA_ALIGN = 256;
struct Allocs {
  std::vector<void*> ptrs;
  hipStream_t stream = nullptr;
  bool ordered = false;
  char* arena = nullptr;
  size_t cap = 0, used = 0;
  Allocs() = default;
  Allocs(hipStream_t s, bool ord) : stream(s), ordered(ord) {}
  Allocs(const Allocs&) = delete;
  Allocs& operator=(const Allocs&) = delete;
  template <class T>
  T* get(size_t count) {
    void* p = nullptr;
    if (count == 0) count = 1;
    if (arena) {
      const size_t off = (used + ARENA_ALIGN - 1) & ~(ARENA_ALIGN - 1);
      if (off > cap || count > (cap - off) / sizeof(T))
        throw Error{MLB_EUNSUPPORTED, "the static scratch of " + std::to_string(cap) + " bytes is too small"};
      used = off + count * sizeof(T);
      return (T*)(arena + off);
    }
    const hipError_t e = ordered ? hipMallocAsync(&p, count * sizeof(T), stream) : hipMalloc(&p, count * sizeof(T));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw Error{MLB_ENOMEM, "device allocation of " + std::to_string(count * sizeof(T)) + " bytes failed"};
    }
    ptrs.push_back(p);
    return (T*)p;
  }
  ~Allocs() {
    for (void* p : ptrs) (void)(ordered ? hipFreeAsync(p, stream) : hipFree(p));
  }
};

// Bytes an arena needs for `count` objects of T (alignment padding included).
template <class T>
static size_t arena_bytes(size_t count) {
  return (std::max<size_t>(count, 1) * sizeof(T) + ARENA_ALIGN - 1) & ~(ARENA_ALIGN - 1);
}

static int grid_for(long long work, int cap) {
  long long g = (work + BLOCK - 1) / BLOCK;
  if (g < 1) g = 1;
  return (int)std::min<long long>(g, cap);
}

// Upper bound on the workgroups of a streaming pass (8 per CU on a 256-CU
// MI355X).  MLB_MAX_GRID in the environment lowers or raises it (a tuning knob;
// read once).
static int max_grid() {
  static const int g = [] {
    const char* v = getenv("MLB_MAX_GRID");
    const int x = v ? atoi(v) : 0;
    return x >= 64 && x <= MAX_PARTIAL_ROWS ? x : MAX_PARTIAL_ROWS;
  }();
  return g;
}
#define MAX_GRID max_grid()

// ------------------------------------------------------------------ matrices

template <class V>
struct Mat {
  int format = MLB_CSR;
  int nrows = 0;       // scalar rows
  int nbrows = 0;      // rows of the index structure (block rows for BSR3)
  long long nnz = 0;   // entries / blocks
  const int* rp = nullptr;
  const int* ci = nullptr;
  const V* val = nullptr;
  int lpr = 8;         // lanes per (block) row in the SpMV tile
};

static int pick_lpr(long long nnz, int nbrows) {
  double mean = nbrows > 0 ? (double)nnz / nbrows : 1.0;
  if (mean <= 4.0) return 4;
  if (mean <= 8.0) return 8;
  if (mean <= 16.0) return 16;
  return 32;
}

// Checks row_ptr / col_idx of a user matrix on the device (so that no kernel
// ever indexes outside the arrays the descriptor declares).
__global__ void k_validate(const int* __restrict__ rp, const int* __restrict__ ci, int nbrows, long long nnz,
                           int ncols, int* __restrict__ bad) {
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t <= nbrows; t += (long long)gridDim.x * blockDim.x) {
    const int v = rp[t];
    if (t == 0 && v != 0) atomicOr(bad, 1);
    if (t == nbrows && (long long)v != nnz) atomicOr(bad, 2);
    if (t < nbrows && rp[t + 1] < v) atomicOr(bad, 4);
  }
  for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < nnz; q += (long long)gridDim.x * blockDim.x) {
    const int c = ci[q];
    if (c < 0 || c >= ncols) atomicOr(bad, 8);
  }
}

template <class V>
static Mat<V> build_transpose(const Mat<V>& A, Allocs& al, hipStream_t s) {
  Mat<V> T;
  T.format = A.format;
  T.nrows = A.nrows;
  T.nbrows = A.nbrows;
  T.nnz = A.nnz;
  const int m = A.nbrows;
  const int bs = A.format == MLB_BSR3 ? 9 : 1;
  int* rpT = al.get<int>(m + 1);
  int* ciT = al.get<int>(A.nnz);
  V* valT = al.get<V>((size_t)A.nnz * bs);
  Allocs tmp_own(al.stream, al.ordered);
  Allocs& tmp = al.arena ? al : tmp_own;   // arena mode: temporaries stay in the arena
  int* cnt = tmp.get<int>(m);
  int* fill = tmp.get<int>(m);
  if (al.arena) {
    k_fill<int><<<grid_for(m, 4096), BLOCK, 0, s>>>(cnt, m, 0);
    k_fill<int><<<grid_for(m, 4096), BLOCK, 0, s>>>(fill, m, 0);
  } else {
    HIP_TRY(hipMemsetAsync(cnt, 0, sizeof(int) * m, s));
    HIP_TRY(hipMemsetAsync(fill, 0, sizeof(int) * m, s));
  }
  if (A.nnz > 0) k_col_count<<<grid_for(A.nnz, 4096), BLOCK, 0, s>>>(A.ci, A.nnz, cnt);
  {
    const int ntiles = (int)((m + SCAN_TILE - 1) / SCAN_TILE);
    int* tsum = tmp.get<int>((size_t)ntiles + 1);
    k_scan_tiles<<<ntiles, SCAN_T, 0, s>>>(cnt, m, tsum);
    k_scan_sums<<<1, SCAN_T, 0, s>>>(tsum, ntiles);
    k_scan_apply<<<ntiles, SCAN_T, 0, s>>>(cnt, m, tsum, ntiles, rpT);
  }
  if (bs == 1) {
    k_scatter<V, 1><<<grid_for(m, 4096), BLOCK, 0, s>>>(A.rp, A.ci, A.val, m, rpT, fill, ciT, valT);
    k_sort_rows<V, 1><<<grid_for(m, 4096), BLOCK, 0, s>>>(rpT, m, ciT, valT);
  } else {
    k_scatter<V, 9><<<grid_for(m, 4096), BLOCK, 0, s>>>(A.rp, A.ci, A.val, m, rpT, fill, ciT, valT);
    k_sort_rows<V, 9><<<grid_for(m, 4096), BLOCK, 0, s>>>(rpT, m, ciT, valT);
  }
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));   // tmp_own is freed on return
  T.rp = rpT;
  T.ci = ciT;
  T.val = valT;
  T.lpr = pick_lpr(T.nnz, T.nbrows);
  return T;
}

// ------------------------------------------------------------------ ILU(0)

// Level sets of the dependencies of a row-sorted pattern: lower = rows j < i of
// row i (forward substitution), else rows j > i (backward).  The row order is
// grouped by level (rows in increasing order inside a level); ptr[l] .. ptr[l+1]
// are the rows of level l.  Integer set-up work on the host over a copy of the
// index arrays.
static void level_sets(const std::vector<int>& rp, const std::vector<int>& ci, bool lower, std::vector<int>& order,
                       std::vector<int>& ptr) {
  const int m = (int)rp.size() - 1;
  std::vector<int> lev((size_t)m, 0);
  int nlev = 0;
  for (int t = 0; t < m; ++t) {
    const int i = lower ? t : m - 1 - t;
    int l = 0;
    for (int q = rp[i]; q < rp[i + 1]; ++q) {
      const int j = ci[q];
      if (lower ? j < i : j > i) l = std::max(l, lev[j] + 1);
    }
    lev[i] = l;
    nlev = std::max(nlev, l + 1);
  }
  ptr.assign((size_t)nlev + 1, 0);
  for (int i = 0; i < m; ++i) ptr[lev[i] + 1]++;
  for (int l = 0; l < nlev; ++l) ptr[l + 1] += ptr[l];
  order.assign((size_t)m, 0);
  std::vector<int> fill(ptr.begin(), ptr.end() - 1);
  for (int i = 0; i < m; ++i) order[fill[lev[i]]++] = i;
}

// Compute units of the current device (256 if the query fails).
static int device_cus() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                               hipSuccess || cus <= 0) {
    (void)hipGetLastError();
    cus = 256;
  }
  return cus;
}

// The ILU(0) factor of A, its conjugate transpose and the rows of the four
// triangular solves in level order (L, U of the factor; U^H, L^H of its
// transpose).
template <class V>
struct IluFactor {
  int bs = 1, nbrows = 0;
  Mat<V> F, FH;                       // factor (A's sorted pattern) and its conjugate transpose
  int* dpos = nullptr;                // diagonal positions in F and FH
  int* dposH = nullptr;
  V* dinv = nullptr;                  // inverse diagonal (blocks) of F (U_ii^{-1}) and FH ((U_ii^H)^{-1})
  V* dinvH = nullptr;
  int* ordL = nullptr;                                                         // rows by level of L (device)
  int4 *lvL = nullptr, *lvU = nullptr, *lvHf = nullptr, *lvHb = nullptr;       // the solves' rows and ranges
  std::vector<int> ptrL;                                                       // level pointers of L (host)
  V* tmid = nullptr;                  // intermediate vector of the two solves
  unsigned* ctl = nullptr;            // one-launch solves: claim counters [0] and [1], lost-wait flag [2]
  int sweep_grid = 1;                 // their workgroups (persistent: each wave claims until none are left)
  unsigned max_tries = ~0u;           // tries of a row before it gives up (MLB_ILU_MAX_TRIES, for tests)
};

// Waves of a one-launch triangular solve, as a multiple of the waves one
// average level fills (capped at two per CU), one wave per workgroup so that
// they spread over the CUs.
static constexpr double ILU_SWEEP_LEVEL_MULT = 3.0;

static int level_grid(int count) { return std::max(1, std::min((count + BLOCK - 1) / BLOCK, 4096)); }

// The rows of a sweep in solve order with their entry ranges (host): {i, q0, q1, 0},
// [q0, q1) the stored entries left (lower) or right of row i's diagonal.  Every row
// has a stored diagonal (checked before).
static std::vector<int4> level_rows(const std::vector<int>& rp, const std::vector<int>& ci, const std::vector<int>& ord,
                                    bool lower) {
  std::vector<int4> out(ord.size());
  for (size_t t = 0; t < ord.size(); ++t) {
    const int i = ord[t];
    int qd = rp[i];
    for (int q = rp[i]; q < rp[i + 1]; ++q)
      if (ci[q] == i) {
        qd = q;
        break;
      }
    out[t] = make_int4(i, lower ? rp[i] : qd + 1, lower ? qd : rp[i + 1], 0);
  }
  return out;
}

// One triangular solve in one launch (k_ilu_solve_sweep); `which` picks its claim counter.
template <class V, int BS, bool LOWER, bool UNIT>
static void ilu_sweep1(const IluFactor<V>& f, const Mat<V>& M, const V* dinv, const int4* lv, const V* in, V* out,
                       V* next, int which, hipStream_t s, const int* done) {
  k_ilu_solve_sweep<V, BS, LOWER, UNIT><<<f.sweep_grid, WAVE, 0, s>>>(M.ci, M.val, dinv, lv, f.nbrows, in, out,
                                                                       next, f.ctl + which, f.ctl + 2, f.max_tries,
                                                                       done);
}

// Marks f.tmid pending and resets both claim counters: the start of a pair of one-launch solves.
template <class V>
static void ilu_pending(const IluFactor<V>& f, hipStream_t s, const int* done) {
  const long long nw = (long long)f.nbrows * f.bs * (long long)(sizeof(V) / 8);
  k_ilu_pending<<<grid_for(nw, 4096), BLOCK, 0, s>>>(reinterpret_cast<unsigned long long*>(f.tmid), nw, f.ctl, done);
}

// out = M^{-1} in = U^{-1} (L^{-1} in) through f.tmid (out may be in).
template <class V>
static void ilu_apply(const IluFactor<V>& f, const V* in, V* out, hipStream_t s, const int* done) {
  if constexpr (!std::is_same<typename traits<V>::real, double>::value) {
    throw Error{MLB_EUNSUPPORTED, "ILU(0) runs on fp64 values only"};
  } else {
    ilu_pending(f, s, done);
    if (f.bs == 1) {
      ilu_sweep1<V, 1, true, true>(f, f.F, f.dinv, f.lvL, in, f.tmid, out, 0, s, done);
      ilu_sweep1<V, 1, false, false>(f, f.F, f.dinv, f.lvU, f.tmid, out, nullptr, 1, s, done);
    } else {
      ilu_sweep1<V, 3, true, true>(f, f.F, f.dinv, f.lvL, in, f.tmid, out, 0, s, done);
      ilu_sweep1<V, 3, false, false>(f, f.F, f.dinv, f.lvU, f.tmid, out, nullptr, 1, s, done);
    }
  }
}

// v = M^{-H} v = L^{-H} (U^{-H} v), in place through f.tmid.
template <class V>
static void ilu_apply_h(const IluFactor<V>& f, V* v, hipStream_t s, const int* done) {
  if constexpr (!std::is_same<typename traits<V>::real, double>::value) {
    throw Error{MLB_EUNSUPPORTED, "ILU(0) runs on fp64 values only"};
  } else {
    ilu_pending(f, s, done);
    if (f.bs == 1) {
      ilu_sweep1<V, 1, true, false>(f, f.FH, f.dinvH, f.lvHf, v, f.tmid, v, 0, s, done);
      ilu_sweep1<V, 1, false, true>(f, f.FH, f.dinvH, f.lvHb, f.tmid, v, nullptr, 1, s, done);
    } else {
      ilu_sweep1<V, 3, true, false>(f, f.FH, f.dinvH, f.lvHf, v, f.tmid, v, 0, s, done);
      ilu_sweep1<V, 3, false, true>(f, f.FH, f.dinvH, f.lvHb, f.tmid, v, nullptr, 1, s, done);
    }
  }
}

// x <- M x = L (U x) in place through f.tmid (the map y_0 = M x_0).
template <class V>
static void ilu_forward_map(const IluFactor<V>& f, V* x, hipStream_t s) {
  const int g = grid_for(f.nbrows, 4096);
  if (f.bs == 1) {
    k_ilu_tri_matvec<V, 1, false><<<g, BLOCK, 0, s>>>(f.F.rp, f.F.ci, f.F.val, f.dpos, f.nbrows, x, f.tmid);
    k_ilu_tri_matvec<V, 1, true><<<g, BLOCK, 0, s>>>(f.F.rp, f.F.ci, f.F.val, f.dpos, f.nbrows, f.tmid, x);
  } else {
    k_ilu_tri_matvec<V, 3, false><<<g, BLOCK, 0, s>>>(f.F.rp, f.F.ci, f.F.val, f.dpos, f.nbrows, x, f.tmid);
    k_ilu_tri_matvec<V, 3, true><<<g, BLOCK, 0, s>>>(f.F.rp, f.F.ci, f.F.val, f.dpos, f.nbrows, f.tmid, x);
  }
}

static std::vector<int> to_host(const int* d, size_t count, hipStream_t s) {
  std::vector<int> h(count);
  if (count) HIP_TRY(hipMemcpyAsync(h.data(), d, count * sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return h;
}

// Builds the ILU(0) factor of A on the device: a row-sorted copy of A, the
// pattern checks, the level sets, the factorisation level by level, the
// conjugate transpose with its diagonal inverses.  Throws MLB_EINVAL for a
// missing diagonal, a repeated column in a row or a zero / singular pivot.
template <class V>
static void build_ilu(const Mat<V>& A, IluFactor<V>& f, Allocs& al, hipStream_t s) {
  const int m = A.nbrows;
  const int bs = A.format == MLB_BSR3 ? 3 : 1;
  const int b2 = bs * bs;
  f.bs = bs;
  f.nbrows = m;
  f.F = A;
  int* ci = al.get<int>((size_t)A.nnz);
  V* val = al.get<V>((size_t)A.nnz * b2);
  if (A.nnz > 0) {
    HIP_TRY(hipMemcpyAsync(ci, A.ci, sizeof(int) * A.nnz, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(val, A.val, sizeof(V) * A.nnz * b2, hipMemcpyDeviceToDevice, s));
  }
  if (bs == 1) k_sort_rows<V, 1><<<grid_for(m, 4096), BLOCK, 0, s>>>(A.rp, m, ci, val);
  else k_sort_rows<V, 9><<<grid_for(m, 4096), BLOCK, 0, s>>>(A.rp, m, ci, val);
  f.F.ci = ci;
  f.F.val = val;
  f.dpos = al.get<int>(m);
  f.dinv = al.get<V>((size_t)m * b2);
  f.tmid = al.get<V>((size_t)m * bs);
  f.ctl = al.get<unsigned>(4);
  k_fill<unsigned><<<1, BLOCK, 0, s>>>(f.ctl, 4, 0u);
  // a test hook: a positive MLB_ILU_MAX_TRIES makes every row that waits that many tries give up
  // (its solve then fails with MLB_EHIP), so the give-up path can be exercised from the host
  if (const char* e = std::getenv("MLB_ILU_MAX_TRIES")) {
    const long v = std::strtol(e, nullptr, 10);
    if (v > 0) f.max_tries = (unsigned)std::min<long>(v, 0x7fffffffL);
  }
  Allocs tmp_own(al.stream, al.ordered);
  int* bad = tmp_own.get<int>(1);
  k_fill<int><<<1, BLOCK, 0, s>>>(bad, 1, 0);
  k_ilu_diag_pos<<<grid_for(m, 4096), BLOCK, 0, s>>>(A.rp, ci, m, f.dpos, bad);
  HIP_TRY(hipGetLastError());
  int hb = 0;
  HIP_TRY(hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (hb & 1) throw Error{MLB_EINVAL, "ILU(0): a (block) row has no stored diagonal entry"};
  if (hb & 4) throw Error{MLB_EINVAL, "ILU(0): a column is stored twice in one (block) row"};
  // level sets of the factor's solves (and of the factorisation, the same as L's)
  const std::vector<int> hrp = to_host(A.rp, (size_t)m + 1, s);
  const std::vector<int> hci = to_host(ci, (size_t)A.nnz, s);
  std::vector<int> ord;
  level_sets(hrp, hci, true, ord, f.ptrL);
  f.ordL = al.get<int>(m);
  HIP_TRY(hipMemcpyAsync(f.ordL, ord.data(), sizeof(int) * m, hipMemcpyHostToDevice, s));
  std::vector<int> ordU, ptrU;
  level_sets(hrp, hci, false, ordU, ptrU);
  {
    const double level_waves = (double)m / (double)std::max<size_t>(1, f.ptrL.size() - 1) / WAVE;
    f.sweep_grid = (int)std::min<double>(2.0 * device_cus(), std::max(1.0, ILU_SWEEP_LEVEL_MULT * level_waves));
  }
  const std::vector<int4> lvL = level_rows(hrp, hci, ord, true), lvU = level_rows(hrp, hci, ordU, false);
  f.lvL = al.get<int4>(m);
  f.lvU = al.get<int4>(m);
  HIP_TRY(hipMemcpyAsync(f.lvL, lvL.data(), sizeof(int4) * m, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(f.lvU, lvU.data(), sizeof(int4) * m, hipMemcpyHostToDevice, s));
  // factorisation, one launch per level of L
  for (size_t l = 0; l + 1 < f.ptrL.size(); ++l) {
    const int c = f.ptrL[l + 1] - f.ptrL[l];
    if (bs == 1)
      k_ilu_factor_level<V, 1><<<level_grid(c), BLOCK, 0, s>>>(A.rp, ci, val, f.dpos, f.dinv, f.ordL + f.ptrL[l], c, bad);
    else
      k_ilu_factor_level<V, 3><<<level_grid(c), BLOCK, 0, s>>>(A.rp, ci, val, f.dpos, f.dinv, f.ordL + f.ptrL[l], c, bad);
  }
  HIP_TRY(hipGetLastError());
  // conjugate transpose of the factor (rows sorted) and its diagonal inverses
  f.FH = build_transpose(f.F, al, s);
  f.dposH = al.get<int>(m);
  f.dinvH = al.get<V>((size_t)m * b2);
  k_ilu_diag_pos<<<grid_for(m, 4096), BLOCK, 0, s>>>(f.FH.rp, f.FH.ci, m, f.dposH, bad);
  if (bs == 1) k_ilu_inv_diag<V, 1><<<grid_for(m, 4096), BLOCK, 0, s>>>(f.FH.val, f.dposH, m, f.dinvH, bad);
  else k_ilu_inv_diag<V, 3><<<grid_for(m, 4096), BLOCK, 0, s>>>(f.FH.val, f.dposH, m, f.dinvH, bad);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (hb & 2) throw Error{MLB_EINVAL, "ILU(0): a zero or singular pivot"};
  const std::vector<int> hrpH = to_host(f.FH.rp, (size_t)m + 1, s);
  const std::vector<int> hciH = to_host(f.FH.ci, (size_t)A.nnz, s);
  std::vector<int> ordHf, ordHb, ptrHf, ptrHb;
  level_sets(hrpH, hciH, true, ordHf, ptrHf);
  level_sets(hrpH, hciH, false, ordHb, ptrHb);
  const std::vector<int4> lvHf = level_rows(hrpH, hciH, ordHf, true), lvHb = level_rows(hrpH, hciH, ordHb, false);
  f.lvHf = al.get<int4>(m);
  f.lvHb = al.get<int4>(m);
  HIP_TRY(hipMemcpyAsync(f.lvHf, lvHf.data(), sizeof(int4) * m, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(f.lvHb, lvHb.data(), sizeof(int4) * m, hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));   // the host vectors above are copied before they go
}

// Device bytes build_ilu allocates (beside the transpose's own temporaries).
static size_t ilu_bytes(long long nnz, int m, int bs, size_t sv) {
  const size_t b2 = (size_t)bs * bs;
  return (size_t)nnz * 4 * 2 + (size_t)nnz * b2 * sv * 2 + (size_t)(m + 1) * 4 + (size_t)m * 4 * 3 +
         (size_t)m * sizeof(int4) * 4 + (size_t)m * b2 * sv * 2 + (size_t)m * bs * sv + 16;
}

// ------------------------------------------------------------------ launch dispatch

// Kernel timing hook: a pair of HIP events attached to one launch.  With
// hipExtLaunchKernel the events take the kernel's own start and end times
// (no separate marker packets on the stream).
struct Timed {
  hipEvent_t start = nullptr, stop = nullptr;
};
#define MLB_LAUNCH(kernel, grid, stream, tm, ...)                                                       \
  do {                                                                                                 \
    if ((tm).start)                                                                                    \
      hipExtLaunchKernelGGL(kernel, dim3(grid), dim3(BLOCK), 0, stream, (tm).start, (tm).stop, 0, __VA_ARGS__); \
    else                                                                                               \
      kernel<<<grid, BLOCK, 0, stream>>>(__VA_ARGS__);                                                 \
  } while (0)

static int bucket(int n) { return bucket_of(n); }

// Launches the SpMV kernel for A's format and lanes-per-row with epilogue MODE.
// With grid == 0 nothing is launched and the kernel's occupancy (workgroups per
// CU) is returned instead.
template <class K>
static int occupancy_of(K kernel) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, BLOCK, 0) != hipSuccess) {
    (void)hipGetLastError();
    per_cu = 4;
  }
  return std::max(per_cu, 1);
}

template <class V, class Sc, int MODE, int ND>
static int launch_spmv_nd(const Mat<V>& A, int grid, hipStream_t s, State<Sc>* st, Sc* part, const SpmvArgs<V>& a,
                          int phase, int i, int j, int n, int flags, Timed tm = {}) {
#define MLB_SPMV_CASE(L)                                                                                     \
  if (A.format == MLB_CSR) {                                                                                 \
    if (!grid) return occupancy_of(k_spmv<V, Sc, ND, L, 0, MODE>);                                          \
    MLB_LAUNCH((k_spmv<V, Sc, ND, L, 0, MODE>), grid, s, tm, st, part, a, phase, i, j, n, flags);            \
  } else {                                                                                                   \
    if (!grid) return occupancy_of(k_spmv<V, Sc, ND, L, 1, MODE>);                                          \
    MLB_LAUNCH((k_spmv<V, Sc, ND, L, 1, MODE>), grid, s, tm, st, part, a, phase, i, j, n, flags);            \
  }
#define MLB_SPMV_WCASE(L)                                                                                    \
  if (A.format == MLB_CSR) {                                                                                 \
    if (!grid) return occupancy_of(k_spmv_csrw<V, Sc, ND, L, MODE>);                                        \
    MLB_LAUNCH((k_spmv_csrw<V, Sc, ND, L, MODE>), grid, s, tm, st, part, a, flags);                         \
  } else {                                                                                                   \
    if (!grid) return occupancy_of(k_spmv_bsrw<V, Sc, ND, L, MODE>);                                        \
    MLB_LAUNCH((k_spmv_bsrw<V, Sc, ND, L, MODE>), grid, s, tm, st, part, a, flags);                         \
  }
  switch (A.lpr) {
    case 4: MLB_SPMV_WCASE(4) break;
    case 8: MLB_SPMV_WCASE(8) break;
    case 16: MLB_SPMV_CASE(16) break;
    default: MLB_SPMV_CASE(32) break;
  }
#undef MLB_SPMV_CASE
#undef MLB_SPMV_WCASE
  return 0;
}

// Resets the device scalars before a solve.
template <class Sc>
__global__ void k_init_state(State<Sc>* st, double tol, long long maxit, double kappa, int* host_done,
                             long long stag_window) {
  st->done = 0;
  st->flag = 1;
  st->iter = 0;
  st->maxit = maxit;
  st->tol = tol;
  st->kappa = kappa;
  st->bnrm2 = 1.0;
  st->err = 0.0;
  st->uu = 0.0;
  st->e = st->alpha = zero<Sc>();
  st->omega = from_real<Sc>(1.0);
  for (int q = 0; q < NMAX; ++q) st->c[q] = st->cinv[q] = st->t[q] = st->tg[q] = st->beta[q] = zero<Sc>();
  for (int q = 0; q < NMAX * NMAX; ++q) st->S[q] = zero<Sc>();
  for (int q = 0; q < 8; ++q) st->aux[q] = zero<Sc>();
  for (int q = 0; q < NMAX; ++q) st->alph[q] = zero<Sc>();
  st->npend = 0;
  st->host_done = host_done;
  st->best_err = 0.0;
  st->best_k = 0;
  st->stag_window = stag_window;
}


// ------------------------------------------------------------------ engine

template <class V>
struct Engine {
  using Sc = typename traits<V>::wide;
  int N = 0, n = 0, nb = 4;
  Mat<V> A, AH;
  V *G = nullptr, *W = nullptr, *F = nullptr, *r = nullptr, *gt = nullptr, *z = nullptr;
  State<Sc>* st = nullptr;
  Sc* part = nullptr;    // per-workgroup partial sums of the last reducing pass
  Sc* part2 = nullptr;   // their first-stage sums (long rows)
  int grid_vec = 1, grid_spmv = 1, grid_sw = 1;
  hipStream_t s = nullptr;
  int* host_done = nullptr;       // pinned, mapped
  int* host_done_dev = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  // per solve
  const V* Q = nullptr;
  long long ldq = 0;

  bool own_flag = true;
  // Poll mode (set before init): no host-mapped done flag and no HIP events; the
  // host reads the device flag every POLL_CYCLES cycles (allocation-free solves).
  bool poll = false;
  static constexpr int POLL_CYCLES = 4;
  bool tf = false;   // transpose-free inner steps: no A^H, no F (set before init)
  // ILU(0) from the right (set before init): every product with A is preceded by
  // M^{-1} applied to its input (into tpre), and f_s = M^{-H} (A^H q_s).
  const IluFactor<V>* ilu = nullptr;
  V* tpre = nullptr;
  bool literal = false;   // beta~ and beta recurrences in the sequential order, one reduction per coefficient
  // The S column of w_i below its diagonal from the next alpha pass (PH_INNER_S)
  // instead of the SpMV step, which then reduces c_i alone (PH_SPMV_C).  It saves
  // the SpMV epilogue n - i - 1 columns of Q (the alpha pass reads them anyway)
  // but doubles the sums the alpha pass reduces per workgroup.  Set by set_n for
  // the Gram-form steps with A^H where that measured faster: a bucket of 8 or 16
  // whose 2 nb + 1 alpha accumulators stay within 288 bytes (real n <= 16,
  // complex n <= 8).  At n <= 4 the column is at most 3 entries long and the
  // wider reduction costs more than the saved reads; complex n = 16 would need
  // 154 VGPRs in the alpha pass.
  bool s_alpha = false;

  // ext_flag: a pinned, host-mapped int the caller owns (serving workers reuse one
  // per worker); NULL = allocate one.
  // n_alloc: the largest n this engine will run (its workspace); the active n is
  // set by set_n and may change between solves.
  void init(const Mat<V>& A_, const Mat<V>& AH_, int n_alloc, hipStream_t s_, Allocs& al, int* ext_flag = nullptr) {
    A = A_;
    AH = AH_;
    N = A.nrows;
    s = s_;
    const size_t Nn = (size_t)N * n_alloc;
    G = al.get<V>(Nn);
    W = al.get<V>(Nn);
    F = tf ? nullptr : al.get<V>((size_t)N * std::max(n_alloc - 1, 1));
    r = al.get<V>(N);
    gt = al.get<V>(N);
    z = al.get<V>(N);
    if (ilu) tpre = al.get<V>(N);
    st = al.get<State<Sc>>(1);
    part = al.get<Sc>((size_t)MAX_PARTIAL_ROWS * (NMAX + 1));
    part2 = al.get<Sc>((size_t)PSUM_GRID * (NMAX + 1));
    set_n(n_alloc);
    if (poll) return;   // no host-mapped flag, no events
    if (ext_flag) {
      host_done = ext_flag;
      own_flag = false;
    } else {
      HIP_TRY(hipHostMalloc((void**)&host_done, sizeof(int), hipHostMallocMapped));
    }
    *host_done = 0;
    HIP_TRY(hipHostGetDevicePointer((void**)&host_done_dev, host_done, 0));
    for (auto& e : ev) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  // Workspace init() carves for N rows and n shadow vectors (arena mode).
  static size_t arena_need(int N, int n, bool tf) {
    const size_t Nn = (size_t)N * n;
    return 2 * arena_bytes<V>(Nn) + (tf ? 0 : arena_bytes<V>((size_t)N * std::max(n - 1, 1))) +
           3 * arena_bytes<V>(N) + arena_bytes<State<Sc>>(1) + arena_bytes<Sc>((size_t)MAX_PARTIAL_ROWS * (NMAX + 1)) +
           arena_bytes<Sc>((size_t)PSUM_GRID * (NMAX + 1));
  }
  // Active number of shadow vectors (<= the n the workspace was sized for).  The
  // grids: one resident round of workgroups, CUs x the SpMV-step kernel's
  // occupancy for the SpMV passes (no partly filled second round), 4 or 6 per
  // CU for the streaming vector passes; MLB_MAX_GRID caps both.
  void set_n(int n_) {
    n = n_;
    nb = bucket(n);
    s_alpha = !literal && !tf && nb >= 8 && nb <= 16 && (2 * nb + 1) * (int)sizeof(V) <= 288;
    const int cus = device_cus();
    SpmvArgs<V> probe{};
    int occ = 4;
    switch (nb) {
      case 4: occ = launch_spmv_nd<V, Sc, SM_STEP, 4>(A, 0, s, st, nullptr, probe, 0, 0, 0, n, 0); break;
      case 8: occ = launch_spmv_nd<V, Sc, SM_STEP, 8>(A, 0, s, st, nullptr, probe, 0, 0, 0, n, 0); break;
      case 16: occ = launch_spmv_nd<V, Sc, SM_STEP, 16>(A, 0, s, st, nullptr, probe, 0, 0, 0, n, 0); break;
      default: occ = launch_spmv_nd<V, Sc, SM_STEP, 32>(A, 0, s, st, nullptr, probe, 0, 0, 0, n, 0); break;
    }
    // Complex values and 16 or more shadow vectors: 4 workgroups per CU (4-5%
    // faster solves than 8 on 128^3 real n = 16 and 96^3 complex n = 4, 8, 16);
    // real values with n <= 8: 6 (2-3% faster than 8 on 128^3 n = 4, 8 and the
    // reservoir system, where 4 is 1.4-2.6% slower than 8).
    const int vec_per_cu = traits<V>::is_complex || nb >= 16 ? 4 : 6;
    grid_vec = grid_for(N, std::min(MAX_GRID, vec_per_cu * cus));
    // The alpha pass that also reduces the S column (2 nb + 1 sums per workgroup):
    // 2 workgroups per CU, which halves the partial rows its recurrence launch
    // sums (0.5-1% faster solves at n = 8, 16 and on the reservoir system than 6).
    grid_sw = grid_for(N, std::min(MAX_GRID, 2 * cus));
    grid_spmv = grid_for(A.nbrows, std::min(MAX_GRID, occ * cus));
    // The LDS-tile SpMV (rows of more than 8 entries or blocks) takes 256-row
    // tiles in rounds of the grid: the smallest grid with the same number of
    // rounds gives every workgroup the same number of tiles, instead of a last
    // round that is only partly filled while the rest waits.  The wave-local
    // kernels and the vector passes keep the full grid: for them the lower
    // occupancy costs more than the imbalance.
    if (A.lpr > 8) {
      const long long tiles = (A.nbrows + BLOCK - 1) / BLOCK;
      const long long rounds = (tiles + grid_spmv - 1) / grid_spmv;
      grid_spmv = (int)std::max(1LL, (tiles + rounds - 1) / rounds);
    }
  }

  void release() {
    if (host_done && own_flag) (void)hipHostFree(host_done);
    host_done = nullptr;
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
  }

  static size_t bytes(int N, int n, bool tf) {
    return sizeof(V) * ((size_t)N * (2 * n + (tf ? 0 : std::max(n - 1, 1)) + 3)) + sizeof(State<Sc>) +
           sizeof(Sc) * (size_t)(MAX_PARTIAL_ROWS + PSUM_GRID) * (NMAX + 1);
  }

  // ---- single launches --------------------------------------------------

  bool launch_scalars = true;   // false while timing kernels (same kernel work, no recurrence)
  int force_flags = 0;          // OR-ed into every pass's flags (timing: F_IGNORE_DONE)
  // Timing hook: every launch of kernel class ev_kernel gets a start/stop event
  // pair attached to the launch itself; the pairs are collected in ev_list.
  int ev_kernel = -1;
  std::vector<hipEvent_t>* ev_list = nullptr;
  Timed timed(int kind) {
    Timed tm;
    if (ev_kernel != kind || !ev_list) return tm;
    if (hipEventCreate(&tm.start) != hipSuccess) return Timed{};
    if (hipEventCreate(&tm.stop) != hipSuccess) {
      (void)hipEventDestroy(tm.start);
      return Timed{};
    }
    ev_list->push_back(tm.start);
    ev_list->push_back(tm.stop);
    return tm;
  }

  // Sum the partials of the pass just launched and run the recurrence of `phase`.
  // Rows longer than 64 bytes are first summed in PSUM_GRID contiguous shares
  // (k_psum), so that the one-workgroup stage reads few rows.
  template <int STRIDE>
  void scalar_t(int nblocks, int nsum, int phase, int i, int j) {
    if (two_stage<Sc, STRIDE>() && nblocks > PSUM_GRID) {
      k_psum<Sc, STRIDE><<<PSUM_GRID, BLOCK, 0, s>>>(part, nblocks, nsum, part2);
      k_scalar<Sc, STRIDE><<<1, sblock<Sc, STRIDE>(), 0, s>>>(st, part2, PSUM_GRID, nsum, phase, i, j, n);
    } else {
      k_scalar<Sc, STRIDE><<<1, sblock<Sc, STRIDE>(), 0, s>>>(st, part, nblocks, nsum, phase, i, j, n);
    }
  }
  void scalar(int nblocks, int stride, int nsum, int phase, int i, int j) {
    if (!launch_scalars) return;
    switch (stride) {
      case 4: scalar_t<4>(nblocks, nsum, phase, i, j); break;
      case 5: scalar_t<5>(nblocks, nsum, phase, i, j); break;
      case 8: scalar_t<8>(nblocks, nsum, phase, i, j); break;
      case 9: scalar_t<9>(nblocks, nsum, phase, i, j); break;
      case 16: scalar_t<16>(nblocks, nsum, phase, i, j); break;
      case 17: scalar_t<17>(nblocks, nsum, phase, i, j); break;
      case 32: scalar_t<32>(nblocks, nsum, phase, i, j); break;
      default: scalar_t<33>(nblocks, nsum, phase, i, j); break;
    }
  }

  void spmv_resid(const Mat<V>& M, const V* xin, const V* b, V* out, const V* Qc, int phase, int flags = 0) {
    SpmvArgs<V> a{};
    a.format = M.format; a.nrows = M.nrows; a.nbrows = M.nbrows; a.rp = M.rp; a.ci = M.ci; a.val = M.val;
    a.xin = xin; a.xown = xin; a.out1 = out; a.b = b; a.Q = Qc; a.nd = Qc ? 1 : 0;
    launch_spmv_nd<V, Sc, SM_RESID, 4>(M, grid_spmv, s, st, part, a, phase, 0, 0, n, flags);
    if (!(flags & F_SKIP_SCALAR)) scalar(grid_spmv, 4, 3, phase, 0, 0);
  }
  void spmv_plain(const Mat<V>& M, const V* xin, V* out, int flags = 0) {
    SpmvArgs<V> a{};
    a.format = M.format; a.nrows = M.nrows; a.nbrows = M.nbrows; a.rp = M.rp; a.ci = M.ci; a.val = M.val;
    a.xin = xin; a.xown = xin; a.out1 = out;
    launch_spmv_nd<V, Sc, SM_PLAIN, 4>(M, grid_spmv, s, st, part, a, PH_NONE, 0, 0, n, flags);
  }
  // The vector a product with A M^{-1} multiplies: v itself, or M^{-1} v in tpre.
  const V* pre(const V* v) {
    if (!ilu) return v;
    ilu_apply(*ilu, v, tpre, s, (force_flags & F_IGNORE_DONE) ? nullptr : &st->done);
    return tpre;
  }
  void spmv_omega(const V* u, V* zout) {
    SpmvArgs<V> a{};
    a.format = A.format; a.nrows = A.nrows; a.nbrows = A.nbrows; a.rp = A.rp; a.ci = A.ci; a.val = A.val;
    a.xin = pre(u); a.xown = u; a.out1 = zout;
    launch_spmv_nd<V, Sc, SM_OMEGA, 4>(A, grid_spmv, s, st, part, a, PH_SPMV_OMEGA, 0, 0, n, force_flags);
    scalar(grid_spmv, 4, 2, PH_SPMV_OMEGA, 0, 0);
  }
  // G_i = g + sum_{s<i} beta_s G_s (beta from the last PH_COMBINE)
  void gcomb(const V* gin, int i, int flags = 0) {
    flags |= force_flags;
    const Timed tm = timed(MLB_KERNEL_RECOMBINE);
    MLB_LAUNCH((k_gcomb<V, Sc>), grid_vec, s, tm, st, N, gin, (const V*)G, (long long)N, i, G + (size_t)i * N, flags);
  }
  // Transpose-free step i: v = A g -> W_i with q_s^H v, s < i, and the beta
  // recurrence (f_s^H g = q_s^H v).
  void spmv_h(const V* gin, int i, int j) {
    SpmvArgs<V> a{};
    a.format = A.format; a.nrows = A.nrows; a.nbrows = A.nbrows; a.rp = A.rp; a.ci = A.ci; a.val = A.val;
    a.xin = pre(gin); a.xown = gin; a.out1 = W + (size_t)i * N; a.out2 = nullptr;
    a.Q = Q; a.ldq = ldq; a.d0 = 0; a.nd = i;
    const int flags = force_flags;
    const Timed tm = timed(MLB_KERNEL_SPMV_STEP);
    switch (nb) {
      case 4: launch_spmv_nd<V, Sc, SM_STEP, 4>(A, grid_spmv, s, st, part, a, PH_COMBINE, i, j, n, flags, tm); break;
      case 8: launch_spmv_nd<V, Sc, SM_STEP, 8>(A, grid_spmv, s, st, part, a, PH_COMBINE, i, j, n, flags, tm); break;
      case 16: launch_spmv_nd<V, Sc, SM_STEP, 16>(A, grid_spmv, s, st, part, a, PH_COMBINE, i, j, n, flags, tm); break;
      default: launch_spmv_nd<V, Sc, SM_STEP, 32>(A, grid_spmv, s, st, part, a, PH_COMBINE, i, j, n, flags, tm); break;
    }
    scalar(grid_spmv, nb, i, PH_COMBINE, i, j);
  }
  // Transpose-free step i: g_k -> G_i, w_k = v + sum beta_s W_s -> W_i, S column i,
  // c_i and the next alpha.
  void gwcomb(const V* gin, int i) {
    const int flags = force_flags;
    const Timed tm = timed(MLB_KERNEL_RECOMBINE);
#define MLB_GW(B) \
  MLB_LAUNCH((k_gwcomb<V, Sc, B>), grid_vec, s, tm, st, part, N, gin, G, W, (long long)N, i, Q, ldq, n, flags)
    switch (nb) {
      case 4: MLB_GW(4); break;
      case 8: MLB_GW(8); break;
      case 16: MLB_GW(16); break;
      default: MLB_GW(32); break;
    }
#undef MLB_GW
    scalar(grid_vec, nb, n - i, PH_SPMV_STEP, i, 0);
  }
  // w_i = A G_i ; S[s][i] = q_s^H w_i, s = i..n-1 (s = i only with s_alpha: the
  // rest comes from the next alpha pass).  With gin != G_i the input is
  // also copied to G_i (cycle close and set-up, where g_k = g).
  // The literal order needs only c_i = q_i^H w_i (nd = 1).
  void spmv_step(const V* gin, int i, int flags = 0) {
    SpmvArgs<V> a{};
    a.format = A.format; a.nrows = A.nrows; a.nbrows = A.nbrows; a.rp = A.rp; a.ci = A.ci; a.val = A.val;
    V* Gi = G + (size_t)i * N;
    a.xin = pre(gin); a.xown = gin; a.out1 = W + (size_t)i * N; a.out2 = gin == Gi ? nullptr : Gi;
    a.Q = Q; a.ldq = ldq; a.d0 = i; a.nd = literal || s_alpha ? 1 : n - i;
    flags |= force_flags;
    const Timed tm = timed(MLB_KERNEL_SPMV_STEP);
    const int nbs = s_alpha ? 4 : nb;   // one dot column: the smallest accumulator set
    switch (nbs) {
      case 4: launch_spmv_nd<V, Sc, SM_STEP, 4>(A, grid_spmv, s, st, part, a, PH_SPMV_STEP, i, 0, n, flags, tm); break;
      case 8: launch_spmv_nd<V, Sc, SM_STEP, 8>(A, grid_spmv, s, st, part, a, PH_SPMV_STEP, i, 0, n, flags, tm); break;
      case 16: launch_spmv_nd<V, Sc, SM_STEP, 16>(A, grid_spmv, s, st, part, a, PH_SPMV_STEP, i, 0, n, flags, tm); break;
      default: launch_spmv_nd<V, Sc, SM_STEP, 32>(A, grid_spmv, s, st, part, a, PH_SPMV_STEP, i, 0, n, flags, tm); break;
    }
    if (!(flags & F_SKIP_SCALAR)) scalar(grid_spmv, std::max(nbs, 3), a.nd, s_alpha ? PH_SPMV_C : PH_SPMV_STEP, i, 0);
  }
  void alpha(V* x, int i_prev, int d0, int nd, int phase, int i, int j, V* xrec, long long K, int flags = 0) {
    const V* gh = G + (size_t)i_prev * N;
    const V* w = W + (size_t)i_prev * N;
    flags |= force_flags;
    const Timed tm = timed(MLB_KERNEL_ALPHA_STEP);
    // inner steps of the Gram form: also the S column of w = w_{i-1} (PH_INNER_S)
    const bool sw = s_alpha && phase == PH_INNER;
    // without an iterate record the x update is deferred to k_omega / k_xflush
#define MLB_ALPHA2(B, SW, XD)                                                                                   \
  MLB_LAUNCH((k_alpha<V, Sc, B, SW, XD>), SW ? grid_sw : grid_vec, s, tm, st, part, N, x, gh, r, w, Q, ldq, d0, nd, xrec, \
             K, phase, i, j, n, flags)
#define MLB_ALPHA(B, SW)              \
  do {                                \
    if (xrec) MLB_ALPHA2(B, SW, false); \
    else MLB_ALPHA2(B, SW, true);       \
  } while (0)
    if (sw) {
      switch (nb) {
        case 4: MLB_ALPHA(4, true); break;
        case 8: MLB_ALPHA(8, true); break;
        default: MLB_ALPHA(16, true); break;
      }
    } else {
      switch (nb) {
        case 4: MLB_ALPHA(4, false); break;
        case 8: MLB_ALPHA(8, false); break;
        case 16: MLB_ALPHA(16, false); break;
        default: MLB_ALPHA(32, false); break;
      }
    }
#undef MLB_ALPHA
#undef MLB_ALPHA2
    if (!(flags & F_SKIP_SCALAR)) {
      if (sw) scalar(grid_sw, 2 * nb + 1, 1 + nb + nd, PH_INNER_S, i, j);
      else scalar(grid_vec, nb + 1, nd + 1, phase, i, j);
    }
  }
  // out: gt (inner steps) or G_0 (cycle close)
  // phase / pi: the recurrence run on the f_s^H g sums (the literal order takes
  // beta_0 from f_0^H r with PH_LIT_B)
  void combine(int t0, int t1, int nf, int i, int j, V* out, int flags = 0, int phase = PH_COMBINE, int pi = -1) {
    flags |= force_flags;
    const Timed tm = timed(MLB_KERNEL_COMBINE);
#define MLB_COMB(B)                                                                                            \
  MLB_LAUNCH((k_combine<V, Sc, B>), grid_vec, s, tm, st, part, N, (const V*)r, (const V*)W, (const V*)G, (long long)N, \
             t0, t1, out, (const V*)F, (long long)N, nf, (int)PH_COMBINE, i, j, n, flags)
    switch (nb) {
      case 4: MLB_COMB(4); break;
      case 8: MLB_COMB(8); break;
      case 16: MLB_COMB(16); break;
      default: MLB_COMB(32); break;
    }
#undef MLB_COMB
    if (!(flags & F_SKIP_SCALAR) && nf > 0) scalar(grid_vec, nb, nf, phase, pi >= 0 ? pi : i, j);
  }
  // Literal order: the beta~ passes of step i (coefficients i..n-1; z_w in gt,
  // the g sum in z), the last writing g into gout with f_0^H g (i >= 1), each
  // followed by the one-coefficient recurrence.
  void lit_tilde(int i, V* gout) {
    const int flags = force_flags;
    for (int sidx = i; sidx < n; ++sidx) {
      const int first = sidx == i, last = sidx == n - 1;
      const V* qf = last ? (i >= 1 ? (const V*)F : nullptr) : Q + (size_t)(sidx + 1) * ldq;
      const int nf = last ? (i >= 1 ? 1 : 0) : 1;
      const Timed tm = timed(MLB_KERNEL_COMBINE);
      MLB_LAUNCH((k_lit_tilde<V, Sc>), grid_vec, s, tm, st, part, N, sidx, first, last, (const V*)r,
                 (const V*)(W + (size_t)sidx * N), (const V*)(G + (size_t)sidx * N), gt, z, gout, qf, nf, flags);
      if (!last) scalar(grid_vec, 4, 1, PH_LIT_T, sidx + 1, 0);
      else if (nf) scalar(grid_vec, 4, 1, PH_LIT_B, 0, 0);
    }
  }
  // Literal order: the beta passes of step i (coefficients 0..i-1) on g in gt;
  // the last writes g_{jn+i} into G_i.
  void lit_beta(int i) {
    const int flags = force_flags;
    for (int sidx = 0; sidx < i; ++sidx) {
      const int last = sidx == i - 1;
      const Timed tm = timed(MLB_KERNEL_RECOMBINE);
      MLB_LAUNCH((k_lit_beta<V, Sc>), grid_vec, s, tm, st, part, N, sidx, last, gt, (const V*)(G + (size_t)sidx * N),
                 G + (size_t)i * N, last ? (const V*)nullptr : (const V*)(F + (size_t)(sidx + 1) * N), flags);
      if (!last) scalar(grid_vec, 4, 1, PH_LIT_B, sidx + 1, 0);
    }
  }
  void omega_update(V* x, V* xrec, long long K) {
    const int nq = literal ? 1 : n;   // the literal order needs only e = q_1^H r here
#define MLB_OM(B)                                                                                              \
  do {                                                                                                        \
    if (xrec)                                                                                                 \
      k_omega<V, Sc, B, false><<<grid_vec, BLOCK, 0, s>>>(st, part, N, x, r, z, Q, ldq, nq, xrec, K, PH_OMEGA_UPD, n, \
                                                          force_flags, (const V*)G, (long long)N);            \
    else                                                                                                      \
      k_omega<V, Sc, B, true><<<grid_vec, BLOCK, 0, s>>>(st, part, N, x, r, z, Q, ldq, nq, xrec, K, PH_OMEGA_UPD, n, \
                                                         force_flags, (const V*)G, (long long)N);             \
  } while (0)
    switch (nb) {
      case 4: MLB_OM(4); break;
      case 8: MLB_OM(8); break;
      case 16: MLB_OM(16); break;
      default: MLB_OM(32); break;
    }
#undef MLB_OM
    scalar(grid_vec, nb + 1, nq + 1, literal ? PH_OMEGA_LIT : PH_OMEGA_UPD, 0, 1);
  }

  // ---- the iteration ----------------------------------------------------

  // Steps k = jn+1 .. jn+n of cycle j in the literal order of Algorithm 7.1: each
  // coefficient of the beta~ and beta recurrences from its own reduction, on the
  // vector the previous coefficient updated.
  void cycle_literal(int j, V* x, V* xrec, long long K) {
    for (int i = 1; i < n; ++i) {
      // x, r update; e = q_{i+1}^H r (no beta~ list: j = 0 for the recurrence)
      alpha(x, i - 1, i, 1, PH_INNER, i, 0, xrec, K);
      if (j >= 1) lit_tilde(i, gt);                         // g = z_w - g/omega, f_0^H g
      else combine(i, i, 1, i, 0, gt, 0, PH_LIT_B, 0);      // g = r, f_0^H r
      lit_beta(i);                                          // g_{jn+i} -> G_i
      spmv_step(G + (size_t)i * N, i);                      // w, c_i, alpha
    }
    alpha(x, n - 1, 0, 0, PH_HALF, n, j, xrec, K);
    spmv_omega(r, z);
    omega_update(x, xrec, K);
    lit_tilde(0, G);   // g_{jn+n} straight into G_0
    spmv_step(G, 0);
  }

  // Steps k = jn+1 .. jn+n of cycle j (Algorithm 7.1, i/j form).
  void cycle(int j, V* x, V* xrec, long long K) {
    if (literal) {
      cycle_literal(j, x, xrec, K);
      return;
    }
    for (int i = 1; i < n; ++i) {
      // x_{jn+i} = x + alpha g ; r_{jn+i} = r - alpha w ; e = q_{i+1}^H r (and q_s^H r, s > i, when j >= 1;
      // with s_alpha also q_s^H w_{jn+i-1}, s >= i, at every j)
      alpha(x, i - 1, i, j >= 1 || s_alpha ? n - i : 1, PH_INNER, i, j, xrec, K);
      if (tf) {
        // g = z_w - g/omega (j >= 1) or r (j = 0); v = A g and the beta recurrence from
        // q_s^H v; g_{jn+i}, w_{jn+i} = v + sum beta_s w_s, c and S column i
        const V* g0 = r;
        if (j >= 1) {
          combine(i, n, 0, i, j, gt);
          g0 = gt;
        }
        spmv_h(g0, i, j);
        gwcomb(g0, i);
        continue;
      }
      // g = z_w - g/omega from the previous cycle's columns (j >= 1), or g = r (j = 0); f_s^H g, s < i
      if (j >= 1) combine(i, n, i, i, j, gt);
      else combine(i, i, i, i, j, gt);
      // g_{jn+i} = g + sum beta_s g_s ; w_{jn+i} = A g_{jn+i} ; c (and S column i without s_alpha)
      gcomb(gt, i);
      spmv_step(G + (size_t)i * N, i);
    }
    // k = jn + n: half step to u, minimisation step, cycle close
    alpha(x, n - 1, 0, 0, PH_HALF, n, j, xrec, K);
    spmv_omega(r, z);
    omega_update(x, xrec, K);
    combine(0, n, 0, 0, j, G);   // g_{jn+n} straight into G_0 (no copy in the SpMV)
    spmv_step(G, 0);
  }

  struct Out {
    int flag;
    long long iter;
    double err;
    float setup_ms;
  };

  // Algorithm 7.1 with M = I from x (in: x_0, out: solution).
  Out solve(const V* b, V* x, const V* Q_, long long ldq_, double tol, long long maxit, double kappa, V* xrec,
            long long K, long long stag_window = 0) {
    if (poll) return solve_polled(b, x, Q_, ldq_, tol, maxit, kappa, xrec, K, stag_window);
    Q = Q_;
    ldq = ldq_;
    *(volatile int*)host_done = 0;
    hipEvent_t t0, t1;
    HIP_TRY(hipEventCreate(&t0));
    HIP_TRY(hipEventCreate(&t1));
    HIP_TRY(hipEventRecord(t0, s));
    k_init_state<Sc><<<1, 1, 0, s>>>(st, tol, maxit, kappa, host_done_dev, stag_window);
    // r_0 = b - A x_0, ||b||, e_0 = q_1^H r_0, early exit
    spmv_resid(A, pre(x), b, r, Q, PH_SETUP);
    // f_s = M^{-H} A^H q_s, s = 1..n-1 (not used by the transpose-free steps)
    if (!tf)
      for (int c = 0; c + 1 < n; ++c) {
        spmv_plain(AH, Q + (size_t)c * ldq, F + (size_t)c * N);
        if (ilu) ilu_apply_h(*ilu, F + (size_t)c * N, s, &st->done);
      }
    // g_0 = r_0, w_0 = A g_0, c_0 (and S column 0), alpha_1 = e_0 / c_0
    spmv_step(r, 0);
    HIP_TRY(hipEventRecord(t1, s));
    HIP_TRY(hipGetLastError());
    const long long max_cycles = maxit / n + 2;
    for (long long j = 0; j <= max_cycles; ++j) {
      cycle((int)std::min<long long>(j, 1), x, xrec, K);
      HIP_TRY(hipEventRecord(ev[j & 1], s));
      if (j >= 1) {
        HIP_TRY(hipEventSynchronize(ev[(j - 1) & 1]));
        if (*(volatile int*)host_done) break;
      }
    }
    // the alpha steps still pending when the solve ended within a cycle
    if (!xrec) k_xflush<V, Sc><<<grid_vec, BLOCK, 0, s>>>(st, N, x, (const V*)G, (long long)N);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    Out o{};
    State<Sc> h;
    HIP_TRY(hipMemcpy(&h, st, sizeof(State<Sc>), hipMemcpyDeviceToHost));
    o.flag = h.done ? h.flag : 1;
    o.iter = h.iter;
    o.err = h.err;
    HIP_TRY(hipEventElapsedTime(&o.setup_ms, t0, t1));
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    return o;
  }

  // The same solve without a host-mapped flag or events: the cycles are enqueued
  // POLL_CYCLES at a time, each batch followed by a copy of the device done flag
  // into a host word and a wait for it.  Set-up time is not measured (0).
  Out solve_polled(const V* b, V* x, const V* Q_, long long ldq_, double tol, long long maxit, double kappa,
                   V* xrec, long long K, long long stag_window) {
    Q = Q_;
    ldq = ldq_;
    k_init_state<Sc><<<1, 1, 0, s>>>(st, tol, maxit, kappa, nullptr, stag_window);
    spmv_resid(A, pre(x), b, r, Q, PH_SETUP);
    if (!tf)
      for (int c = 0; c + 1 < n; ++c) {
        spmv_plain(AH, Q + (size_t)c * ldq, F + (size_t)c * N);
        if (ilu) ilu_apply_h(*ilu, F + (size_t)c * N, s, &st->done);
      }
    spmv_step(r, 0);
    HIP_TRY(hipGetLastError());
    const long long max_cycles = maxit / n + 2;
    for (long long j = 0; j <= max_cycles; ++j) {
      cycle((int)std::min<long long>(j, 1), x, xrec, K);
      if ((j + 1) % POLL_CYCLES == 0 || j == max_cycles) {
        int d = 0;
        HIP_TRY(hipMemcpyAsync(&d, &st->done, sizeof(int), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (d) break;
      }
    }
    // the alpha steps still pending when the solve ended within a cycle
    if (!xrec) k_xflush<V, Sc><<<grid_vec, BLOCK, 0, s>>>(st, N, x, (const V*)G, (long long)N);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    State<Sc> h;
    HIP_TRY(hipMemcpyAsync(&h, st, sizeof(State<Sc>), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    Out o{};
    o.flag = h.done ? h.flag : 1;
    o.iter = h.iter;
    o.err = h.err;
    o.setup_ms = 0.f;
    return o;
  }

  // ||b - M x|| and ||b|| in this engine's precision (sums left in st->aux).
  void resid_sums(const Mat<V>& M, const V* b, const V* x, V* out) {
    k_init_state<Sc><<<1, 1, 0, s>>>(st, 1.0, 1, 0.0, nullptr, 0);
    spmv_resid(M, x, b, out, nullptr, PH_NONE);
  }
  void read_aux(double* rr, double* bb) {
    State<Sc> h;
    HIP_TRY(hipMemcpyAsync(&h, st, sizeof(State<Sc>), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *rr = re(h.aux[0]);
    *bb = re(h.aux[1]);
  }
};

// ------------------------------------------------------------------ solver object

template <class V64, class V32>
struct Impl {
  Engine<V64> e64;
  Engine<V32> e32;
  bool has32 = false;
  V32* b32 = nullptr;   // scaled residual (inner right-hand side)
  V32* x32 = nullptr;   // inner solution
  V32* Q32 = nullptr;   // fp32 shadow block (ld = N)
  V64* r64 = nullptr;   // fp64 residual b - A x
  Mat<V64> A0;          // the caller's A (true residuals); the engines iterate on A M^{-1}
  int bs = 1;           // 1 (CSR) or 3 (BSR3): size of the diagonal blocks of M
  V64* Mblk = nullptr;  // diagonal (blocks) of A, when preconditioned
  V64* Minv = nullptr;  // their inverses
  IluFactor<V64> ilu;   // ILU(0) factor, when has_ilu
  bool has_ilu = false;
  void release() {
    e64.release();
    if (has32) e32.release();
  }
};

}  // namespace mlb

using namespace mlb;

struct mlb_solver {
  int dtype = MLB_R64, format = MLB_CSR;
  int N = 0;
  mlb_options opt{};
  hipStream_t s = nullptr;
  bool own_stream = false;
  bool solved = false;
  int* ext_flags = nullptr;   // two pinned host-mapped ints owned by a serving worker, or NULL
  bool noalloc = false;       // everything in the caller's arena, no host-mapped flags or events
  int n_active = 0;           // shadow vectors of the next solve (<= opt.n, the workspace's)
  Allocs al;
  std::unique_ptr<Impl<double, float>> real;
  std::unique_ptr<Impl<cplx<double>, cplx<float>>> cpx;
  ~mlb_solver() {
    if (real) real->release();
    if (cpx) cpx->release();
    if (own_stream && s) (void)hipStreamDestroy(s);
  }
};

namespace mlb {

static void check_options(const mlb_options* opt) {
  if (!opt) throw Error{MLB_EINVAL, "options pointer is NULL"};
  if (opt->n < 1) throw Error{MLB_EINVAL, "n must be >= 1"};
  if (opt->n > MLB_MAX_N) throw Error{MLB_EUNSUPPORTED, "n > MLB_MAX_N (32) is not supported"};
  if (!(opt->tol > 0.0) || !std::isfinite(opt->tol)) throw Error{MLB_EINVAL, "tol must be a finite positive number"};
  if (opt->maxit < 1) throw Error{MLB_EINVAL, "maxit must be >= 1"};
  if (!(opt->kappa >= 0.0) || !std::isfinite(opt->kappa)) throw Error{MLB_EINVAL, "kappa must be finite and >= 0"};
  if (opt->precision != MLB_PREC_FP64 && opt->precision != MLB_PREC_FP32_IR)
    throw Error{MLB_EINVAL, "precision must be MLB_PREC_FP64 or MLB_PREC_FP32_IR"};
  if (opt->precond != MLB_PRECOND_NONE && opt->precond != MLB_PRECOND_JACOBI && opt->precond != MLB_PRECOND_ILU0)
    throw Error{MLB_EINVAL, "precond must be MLB_PRECOND_NONE, MLB_PRECOND_JACOBI or MLB_PRECOND_ILU0"};
  if (opt->precond == MLB_PRECOND_ILU0 && opt->precision != MLB_PREC_FP64)
    throw Error{MLB_EUNSUPPORTED, "ILU(0) runs with the fp64 iteration only"};
  if (opt->transpose_free != 0 && opt->transpose_free != 1) throw Error{MLB_EINVAL, "transpose_free must be 0 or 1"};
  if (opt->order != MLB_ORDER_FUSED && opt->order != MLB_ORDER_LITERAL)
    throw Error{MLB_EINVAL, "order must be MLB_ORDER_FUSED or MLB_ORDER_LITERAL"};
  if (opt->order == MLB_ORDER_LITERAL && opt->transpose_free)
    throw Error{MLB_EUNSUPPORTED, "the literal order is not combined with transpose_free"};
  if (opt->max_restarts < 0 || opt->max_restarts > 100) throw Error{MLB_EINVAL, "max_restarts must be in [0, 100]"};
  if (opt->max_restarts > 0 && opt->precision != MLB_PREC_FP64)
    throw Error{MLB_EUNSUPPORTED, "max_restarts applies to the fp64 iteration"};
  if (opt->record_iterates < 0) throw Error{MLB_EINVAL, "record_iterates must be >= 0"};
  if (opt->record_iterates > 0) {
    if (!opt->iterates) throw Error{MLB_EINVAL, "record_iterates > 0 needs an iterates buffer"};
    if (opt->precision != MLB_PREC_FP64) throw Error{MLB_EINVAL, "iterates are recorded by the fp64 iteration only"};
    if (opt->record_iterates > opt->maxit) throw Error{MLB_EINVAL, "record_iterates must be <= maxit"};
  }
}

static void check_matrix(const mlb_matrix* A) {
  if (!A) throw Error{MLB_EINVAL, "matrix pointer is NULL"};
  if (A->format != MLB_CSR && A->format != MLB_BSR3) throw Error{MLB_EINVAL, "format must be MLB_CSR or MLB_BSR3"};
  if (A->dtype != MLB_R64 && A->dtype != MLB_C128) throw Error{MLB_EINVAL, "dtype must be MLB_R64 or MLB_C128"};
  // 32-bit row and entry indices advance by grid strides of up to 4096 * BLOCK
  static_assert(4096LL * BLOCK + MLB_MAX_INDEX <= 0x7fffffffLL + 1, "index headroom below 2^31");
  if (A->nrows < 1 || A->nrows > MLB_MAX_INDEX) throw Error{MLB_EINVAL, "nrows must be in [1, 2^31 - 2^20]"};
  if (A->format == MLB_BSR3 && A->nrows % 3 != 0) throw Error{MLB_EINVAL, "BSR3 needs nrows divisible by 3"};
  if (A->nnz < 0 || A->nnz > MLB_MAX_INDEX) throw Error{MLB_EINVAL, "nnz must be in [0, 2^31 - 2^20]"};
  if (!A->row_ptr || (A->nnz > 0 && (!A->col_idx || !A->values)))
    throw Error{MLB_EINVAL, "row_ptr, col_idx and values must be device pointers"};
}

template <class V>
static Mat<V> user_matrix(const mlb_matrix* A) {
  Mat<V> M;
  M.format = A->format;
  M.nrows = (int)A->nrows;
  M.nbrows = A->format == MLB_BSR3 ? (int)(A->nrows / 3) : (int)A->nrows;
  M.nnz = A->nnz;
  M.rp = A->row_ptr;
  M.ci = A->col_idx;
  M.val = (const V*)A->values;
  M.lpr = pick_lpr(M.nnz, M.nbrows);
  return M;
}

template <class V64, class V32>
static void create_impl(mlb_solver* h, const mlb_matrix* Adesc, Impl<V64, V32>& im) {
  Mat<V64> A = user_matrix<V64>(Adesc);
  if (A.nnz == 0) {
    // no entries: the caller may pass NULL index / value arrays; give the kernels
    // valid (never read) ones instead
    const int bs = A.format == MLB_BSR3 ? 9 : 1;
    int* ci = h->al.get<int>(1);
    V64* val = h->al.get<V64>(bs);
    k_fill<int><<<1, BLOCK, 0, h->s>>>(ci, 1, 0);
    k_fill<V64><<<1, BLOCK, 0, h->s>>>(val, bs, zero<V64>());
    A.ci = ci;
    A.val = val;
  }
  im.A0 = A;
  im.bs = A.format == MLB_BSR3 ? 3 : 1;
  if (h->opt.precond == MLB_PRECOND_JACOBI) {
    // M = block diagonal of A; iterate on A M^{-1} (formed once)
    const int b2 = im.bs * im.bs;
    im.Mblk = h->al.get<V64>((size_t)A.nbrows * b2);
    im.Minv = h->al.get<V64>((size_t)A.nbrows * b2);
    V64* scaled = h->al.get<V64>((size_t)A.nnz * b2);
    Allocs tmp(h->al.stream, h->al.ordered);
    int* bad = tmp.get<int>(1);
    HIP_TRY(hipMemsetAsync(bad, 0, sizeof(int), h->s));
    const int g = grid_for(A.nbrows, 4096);
    if (im.bs == 1) {
      k_diag_inverse<V64, 1><<<g, BLOCK, 0, h->s>>>(A.rp, A.ci, A.val, A.nbrows, im.Mblk, im.Minv, bad);
      k_right_scale<V64, 1><<<g, BLOCK, 0, h->s>>>(A.rp, A.ci, A.val, A.nbrows, im.Minv, scaled);
    } else {
      k_diag_inverse<V64, 3><<<g, BLOCK, 0, h->s>>>(A.rp, A.ci, A.val, A.nbrows, im.Mblk, im.Minv, bad);
      k_right_scale<V64, 3><<<g, BLOCK, 0, h->s>>>(A.rp, A.ci, A.val, A.nbrows, im.Minv, scaled);
    }
    HIP_TRY(hipGetLastError());
    int hb = 0;
    HIP_TRY(hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, h->s));
    HIP_TRY(hipStreamSynchronize(h->s));
    if (hb & 1) throw Error{MLB_EINVAL, "Jacobi preconditioner: a (block) row has no stored diagonal entry"};
    if (hb & 2) throw Error{MLB_EINVAL, "Jacobi preconditioner: a diagonal (block) is singular"};
    A.val = scaled;
  }
  if (h->opt.precond == MLB_PRECOND_ILU0) {
    // M = ILU(0) of A; the iteration multiplies by A after M^{-1}
    build_ilu(A, im.ilu, h->al, h->s);
    im.has_ilu = true;
    im.e64.ilu = &im.ilu;
  }
  const bool tf = h->opt.transpose_free != 0;
  const Mat<V64> AH = tf ? Mat<V64>{} : build_transpose(A, h->al, h->s);
  im.e64.tf = tf;
  im.e64.literal = h->opt.order == MLB_ORDER_LITERAL;
  im.e64.poll = h->noalloc;
  im.e64.init(A, AH, h->opt.n, h->s, h->al, h->ext_flags);
  im.r64 = h->al.get<V64>(h->N);
  if (h->opt.precision == MLB_PREC_FP32_IR) {
    const int bs = A.format == MLB_BSR3 ? 9 : 1;
    Mat<V32> A32, AH32;
    A32.format = AH32.format = A.format;
    A32.nrows = AH32.nrows = A.nrows;
    A32.nbrows = AH32.nbrows = A.nbrows;
    A32.nnz = AH32.nnz = A.nnz;
    A32.rp = A.rp;
    A32.ci = A.ci;
    AH32.rp = AH.rp;
    AH32.ci = AH.ci;
    V32* v = h->al.get<V32>((size_t)A.nnz * bs);
    V32* vt = tf ? nullptr : h->al.get<V32>((size_t)A.nnz * bs);
    const long long m = (long long)A.nnz * bs;
    if (m > 0) {
      k_narrow<V32, V64><<<grid_for(m, 4096), BLOCK, 0, h->s>>>(v, A.val, m);
      if (!tf) k_narrow<V32, V64><<<grid_for(m, 4096), BLOCK, 0, h->s>>>(vt, AH.val, m);
    }
    A32.val = v;
    AH32.val = vt;
    A32.lpr = A.lpr;
    AH32.lpr = AH.lpr;
    im.e32.tf = tf;
    im.e32.literal = h->opt.order == MLB_ORDER_LITERAL;
    im.e32.init(A32, AH32, h->opt.n, h->s, h->al, h->ext_flags ? h->ext_flags + 1 : nullptr);
    im.has32 = true;
    im.b32 = h->al.get<V32>(h->N);
    im.x32 = h->al.get<V32>(h->N);
    im.Q32 = h->al.get<V32>((size_t)h->N * h->opt.n);
  }
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(h->s));
}

// Stream time of a whole solve: a HIP event pair, or (host_only, allocation-free
// solves) the host clock around the work, which ends with a stream synchronisation.
struct SolveClock {
  hipStream_t s;
  bool host_only;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  std::chrono::steady_clock::time_point h0;
  SolveClock(hipStream_t s_, bool host_only_) : s(s_), host_only(host_only_) {
    if (host_only) {
      HIP_TRY(hipStreamSynchronize(s));
      h0 = std::chrono::steady_clock::now();
      return;
    }
    HIP_TRY(hipEventCreate(&t0));
    HIP_TRY(hipEventCreate(&t1));
    HIP_TRY(hipEventRecord(t0, s));
  }
  double stop_ms() {
    if (host_only) {
      HIP_TRY(hipStreamSynchronize(s));
      return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - h0).count();
    }
    HIP_TRY(hipEventRecord(t1, s));
    HIP_TRY(hipEventSynchronize(t1));
    float ms = 0;
    HIP_TRY(hipEventElapsedTime(&ms, t0, t1));
    return ms;
  }
  ~SolveClock() {
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
  }
};

// MLB_DEBUG=1 in the environment prints one line per refinement step on stderr.
static bool debug_enabled() {
  static const bool on = [] {
    const char* v = getenv("MLB_DEBUG");
    return v && *v && *v != '0';
  }();
  return on;
}

// Throws when a one-launch triangular solve gave up a wait since the last check
// (the flag is cleared before the error is raised, so the factor stays usable).
template <class V>
static void ilu_check(const IluFactor<V>& f, hipStream_t s) {
  unsigned e = 0;
  HIP_TRY(hipMemcpyAsync(&e, f.ctl + 2, sizeof(unsigned), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (e) {
    k_fill<unsigned><<<1, BLOCK, 0, s>>>(f.ctl + 2, 1, 0u);
    HIP_TRY(hipStreamSynchronize(s));
    throw Error{MLB_EHIP, "ILU(0): a triangular solve gave up waiting for a solved value"};
  }
}

// x <- M x (forward) or x <- M^{-1} x (back) for `cols` columns; no-op without a preconditioner.
template <class V64, class V32>
static void precond_map(mlb_solver* h, Impl<V64, V32>& im, V64* x, int cols, long long ld, bool back) {
  if (im.has_ilu) {
    for (int c = 0; c < cols; ++c) {
      V64* xc = x + (size_t)c * ld;
      if (back) ilu_apply(im.ilu, xc, xc, h->s, nullptr);
      else ilu_forward_map(im.ilu, xc, h->s);
    }
    return;
  }
  if (!im.Minv || cols <= 0) return;
  const V64* blk = back ? im.Minv : im.Mblk;
  const int nbr = im.A0.nbrows;
  const int g = grid_for((long long)nbr * cols, 4096);
  if (im.bs == 1) k_block_apply<V64, 1><<<g, BLOCK, 0, h->s>>>(blk, x, nbr, cols, ld);
  else k_block_apply<V64, 3><<<g, BLOCK, 0, h->s>>>(blk, x, nbr, cols, ld);
}

// The fp64 iteration (Algorithm 7.1) from the current x; with a preconditioner it
// runs on A M^{-1} y = b with y_0 = M x and maps back x = M^{-1} y (also the
// recorded iterates).
template <class V64, class V32>
static typename Engine<V64>::Out fp64_iteration(mlb_solver* h, Impl<V64, V32>& im, const V64* b, V64* x,
                                                const V64* Q, long long ldq, long long maxit, V64* xrec, long long K) {
  const mlb_options& o = h->opt;
  precond_map(h, im, x, 1, h->N, false);
  auto out = im.e64.solve(b, x, Q, ldq, o.tol, maxit, o.kappa, xrec, K);
  precond_map(h, im, x, 1, h->N, true);
  if (xrec) precond_map(h, im, xrec, (int)std::min<long long>(K, std::max<long long>(out.iter, 0)), h->N, true);
  if (im.has_ilu) ilu_check(im.ilu, h->s);
  return out;
}

template <class V64, class V32>
static int solve_impl(mlb_solver* h, Impl<V64, V32>& im, const V64* b, V64* x, const V64* Q, long long ldq,
                      mlb_result* res) {
  const mlb_options& o = h->opt;
  const int N = h->N;
  SolveClock clock(h->s, h->noalloc);
  mlb_result R{};
  int flag = 1;
  if (o.precision == MLB_PREC_FP64) {
    auto out = fp64_iteration(h, im, b, x, Q, ldq, o.maxit, (V64*)o.iterates, o.record_iterates);
    flag = out.flag;
    R.iter = out.iter;
    R.fp64_iters = out.iter;
    R.err_recursive = out.err;
    R.setup_ms = out.setup_ms;
    // restarts from the x reached while a converged run leaves the true residual above tol
    int restarts = 0;
    while (flag == 0 && restarts < o.max_restarts && R.iter < o.maxit) {
      im.e64.resid_sums(im.A0, b, x, im.r64);
      double rr, bb;
      im.e64.read_aux(&rr, &bb);
      const double et = std::sqrt(rr) / (bb > 0 ? std::sqrt(bb) : 1.0);
      if (!(et >= o.tol)) break;
      ++restarts;
      auto more = fp64_iteration(h, im, b, x, Q, ldq, o.maxit - R.iter, (V64*)nullptr, 0);
      flag = more.flag;
      R.iter += more.iter;
      R.fp64_iters += more.iter;
      R.err_recursive = more.err;
    }
    R.outer_iters = restarts;
  } else {
    // fp32 inner iteration inside fp64 iterative refinement (an addition of this library)
    auto& e32 = im.e32;
    for (int c = 0; c < h->n_active; ++c)
      k_cast<V32, V64, typename traits<V64>::wide><<<grid_for(N, 4096), BLOCK, 0, h->s>>>(
          im.Q32 + (size_t)c * N, Q + (size_t)c * ldq, N, im.e64.st, 0);
    const double inner_tol = o.inner_tol > 0 ? o.inner_tol : 1e-6;
    const int max_outer = o.max_outer > 0 ? o.max_outer : 30;
    const long long window = std::max(300, 20 * h->n_active);   // stagnation window of the inner iteration
    long long used = 0;
    double prev = INFINITY;
    bool fallback = false;
    int outer = 0;
    flag = 1;
    while (true) {
      im.e64.resid_sums(im.A0, b, x, im.r64);
      double rr, bb;
      im.e64.read_aux(&rr, &bb);
      const double bn = bb > 0 ? std::sqrt(bb) : 1.0;
      const double et = std::sqrt(rr) / bn;
      R.err_true = et;
      if (!std::isfinite(et)) { flag = -1; break; }
      if (et < o.tol) { flag = 0; break; }
      if (outer >= max_outer || used >= o.maxit) { flag = 1; break; }
      if (outer >= 1 && et > 0.1 * prev) { fallback = true; break; }
      prev = et;
      ++outer;
      // right-hand side r / ||r|| in fp32, zero initial guess
      k_cast<V32, V64, typename traits<V64>::wide><<<grid_for(N, 4096), BLOCK, 0, h->s>>>(im.b32, im.r64, N,
                                                                                          im.e64.st, 1);
      k_fill<V32><<<grid_for(N, 4096), BLOCK, 0, h->s>>>(im.x32, N, zero<V32>());
      // the last refinement step only needs to bring ||r|| from et down to tol: do not over-solve it
      const double step_tol = std::max(inner_tol, 0.25 * o.tol / et);
      auto io = e32.solve(im.b32, im.x32, im.Q32, N, step_tol, o.maxit - used, o.kappa, nullptr, 0, window);
      used += io.iter;
      if (outer == 1) R.setup_ms = io.setup_ms;
      if (debug_enabled())
        fprintf(stderr, "[mlbicgstab] refinement step %d: true err before %.3e, inner flag %d, inner iters %lld, "
                "inner recursive err %.3e\n", outer, et, io.flag, (long long)io.iter, io.err);
      // an inner solve that broke down, or stagnated without halving the residual, ends the refinement
      if (io.flag == -1 || !(io.err < 0.5)) { fallback = true; break; }
      // x += ||r|| M^{-1} d  (d solves the scaled system in fp32)
      const V64* minv = im.Minv;
      if (im.bs == 1 || !minv)
        k_axpy_wide_minv<V64, V32, typename traits<V64>::wide, 1><<<grid_for(N, 4096), BLOCK, 0, h->s>>>(
            x, im.x32, minv, N, im.e64.st);
      else
        k_axpy_wide_minv<V64, V32, typename traits<V64>::wide, 3><<<grid_for(N / 3, 4096), BLOCK, 0, h->s>>>(
            x, im.x32, minv, N / 3, im.e64.st);
      HIP_TRY(hipGetLastError());
    }
    R.outer_iters = outer;
    R.iter = used;
    if (fallback) {
      long long left = std::max<long long>(1, o.maxit - used);
      auto out = fp64_iteration(h, im, b, x, Q, ldq, left, (V64*)nullptr, 0);
      flag = out.flag;
      R.fp64_iters = out.iter;
      R.iter = used + out.iter;
      R.err_recursive = out.err;
    }
  }
  // true residual ||b - A x|| / ||b|| in fp64 with the caller's A
  im.e64.resid_sums(im.A0, b, x, im.r64);
  double rr, bb;
  im.e64.read_aux(&rr, &bb);
  R.err_true = std::sqrt(rr) / (bb > 0 ? std::sqrt(bb) : 1.0);
  if (o.precision == MLB_PREC_FP32_IR && R.fp64_iters == 0) R.err_recursive = R.err_true;
  R.solve_ms = clock.stop_ms();
  R.flag = flag;
  if (res) *res = R;
  return flag;
}

// Mean duration of one kernel class as it runs inside the iteration: whole cycles
// are replayed (same kernels, same predecessors, same cache context; the one-
// workgroup recurrences are left out and the done flag is ignored) and only the
// requested kernel's launches carry a HIP start/stop event pair.
template <class V>
static double time_kernel_impl(Engine<V>& e, int kernel, int reps) {
  Allocs tmp(e.s, false);
  V* xs = tmp.get<V>(e.N);   // scratch iterate (the caller's x is not touched)
  HIP_TRY(hipMemsetAsync(xs, 0, sizeof(V) * e.N, e.s));
  std::vector<hipEvent_t> evs;
  struct Restore {
    Engine<V>& e;
    std::vector<hipEvent_t>& evs;
    ~Restore() {
      e.launch_scalars = true;
      e.force_flags = 0;
      e.ev_kernel = -1;
      e.ev_list = nullptr;
      for (auto ev : evs) (void)hipEventDestroy(ev);
    }
  } restore{e, evs};
  e.launch_scalars = false;
  e.force_flags = F_IGNORE_DONE;
  e.cycle(1, xs, nullptr, 0);   // warm-up, not recorded
  e.ev_kernel = kernel;
  e.ev_list = &evs;
  for (int r = 0; r < reps; ++r) e.cycle(1, xs, nullptr, 0);
  HIP_TRY(hipStreamSynchronize(e.s));
  HIP_TRY(hipGetLastError());
  double total = 0;
  const size_t pairs = evs.size() / 2;
  for (size_t k = 0; k < pairs; ++k) {
    float ms = 0;
    HIP_TRY(hipEventElapsedTime(&ms, evs[2 * k], evs[2 * k + 1]));
    total += ms;
  }
  return pairs ? total / pairs : 0.0;
}

// y = A x with the caller's A, or y = A^H x with the solver's conjugate transpose,
// on the solver's stream (whatever the done flag of the last solve says).
template <class V64, class V32>
static void matvec_impl(mlb_solver* h, Impl<V64, V32>& im, int op, const V64* x, V64* y) {
  if (op == MLB_OP_MINV) {
    ilu_apply(im.ilu, x, y, h->s, nullptr);
  } else if (op == MLB_OP_MINVH) {
    HIP_TRY(hipMemcpyAsync(y, x, sizeof(V64) * (size_t)h->N, hipMemcpyDeviceToDevice, h->s));
    ilu_apply_h(im.ilu, y, h->s, nullptr);
  } else {
    im.e64.spmv_plain(op == MLB_OP_A ? im.A0 : im.e64.AH, x, y, F_IGNORE_DONE);
  }
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(h->s));
  if (op == MLB_OP_MINV || op == MLB_OP_MINVH) ilu_check(im.ilu, h->s);
}

template <class F>
static int guarded(F&& f) {
  try {
    g_last_error.clear();
    return f();
  } catch (const Error& e) {
    g_last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return MLB_ENOMEM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return MLB_EHIP;
  }
}

// Validates A and opt, builds A^H (and the preconditioned / fp32 copies) and the
// workspace.  ordered: stream-ordered allocations on `stream` (serving);
// flags: two pinned host-mapped ints for the engines' done flags, or NULL.
// arena / arena_cap: allocation-free mode, every device buffer carved from the
// caller's region (see Allocs).
static std::unique_ptr<mlb_solver> create_solver(const mlb_matrix* A, const mlb_options* opt, hipStream_t stream,
                                                 bool ordered, int* flags, char* arena = nullptr,
                                                 size_t arena_cap = 0) {
  check_matrix(A);
  check_options(opt);
  auto h = std::make_unique<mlb_solver>();
  h->dtype = A->dtype;
  h->format = A->format;
  h->N = (int)A->nrows;
  h->opt = *opt;
  // NULL is the legacy default stream: work stays ordered with everything else
  // the caller enqueued there (e.g. the fill that zeroes x before a solve).
  h->s = stream;
  h->al.stream = stream;
  h->al.ordered = ordered;
  h->ext_flags = flags;
  h->n_active = opt->n;
  h->al.arena = arena;
  h->al.cap = arena_cap;
  h->noalloc = arena != nullptr;
  // validate the index arrays on the device before any kernel relies on them
  {
    Allocs tmp_own(stream, ordered);
    Allocs& tmp = h->noalloc ? h->al : tmp_own;
    int* bad = tmp.get<int>(1);
    k_fill<int><<<1, BLOCK, 0, h->s>>>(bad, 1, 0);
    const int nbr = A->format == MLB_BSR3 ? (int)(A->nrows / 3) : (int)A->nrows;
    k_validate<<<grid_for(std::max<long long>(nbr + 1, A->nnz), 4096), BLOCK, 0, h->s>>>(A->row_ptr, A->col_idx, nbr,
                                                                                         A->nnz, nbr, bad);
    HIP_TRY(hipGetLastError());
    int hb = 0;
    HIP_TRY(hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, h->s));
    HIP_TRY(hipStreamSynchronize(h->s));
    if (hb) {
      std::string why;
      if (hb & 1) why += " row_ptr[0] != 0;";
      if (hb & 2) why += " row_ptr[last] != nnz;";
      if (hb & 4) why += " row_ptr decreases;";
      if (hb & 8) why += " col_idx out of range;";
      throw Error{MLB_EINVAL, "invalid matrix:" + why};
    }
  }
  if (A->dtype == MLB_R64) {
    h->real = std::make_unique<Impl<double, float>>();
    create_impl(h.get(), A, *h->real);
  } else {
    h->cpx = std::make_unique<Impl<cplx<double>, cplx<float>>>();
    create_impl(h.get(), A, *h->cpx);
  }
  return h;
}

// Number of shadow vectors of the following solves (1 <= n <= the n of create).
static void set_active_n(mlb_solver* h, int n) {
  if (n < 1 || n > h->opt.n) throw Error{MLB_EINVAL, "n must be in [1, the n the solver was created with]"};
  if (n == h->n_active) return;
  h->n_active = n;
  if (h->real) {
    h->real->e64.set_n(n);
    if (h->real->has32) h->real->e32.set_n(n);
  } else {
    h->cpx->e64.set_n(n);
    if (h->cpx->has32) h->cpx->e32.set_n(n);
  }
}

// Moves a solver's work (and the stream-ordered frees of its buffers) to stream
// s; the caller has synchronised the old stream.  Serving sequences run their
// solver on whichever worker takes the next request.
static void set_stream(mlb_solver* h, hipStream_t s) {
  h->s = s;
  h->al.stream = s;
  if (h->real) {
    h->real->e64.s = s;
    if (h->real->has32) h->real->e32.s = s;
  } else {
    h->cpx->e64.s = s;
    if (h->cpx->has32) h->cpx->e32.s = s;
  }
}

static int solve_solver(mlb_solver* h, const void* b, void* x, const void* Q, int64_t ldq, mlb_result* res) {
  if (!b || !x || !Q) throw Error{MLB_EINVAL, "b, x and Q must be device pointers"};
  if (ldq < h->N) throw Error{MLB_EINVAL, "ldq must be >= N"};
  int rc;
  if (h->real)
    rc = solve_impl(h, *h->real, (const double*)b, (double*)x, (const double*)Q, ldq, res);
  else
    rc = solve_impl(h, *h->cpx, (const cplx<double>*)b, (cplx<double>*)x, (const cplx<double>*)Q, ldq, res);
  h->solved = true;
  return rc;
}

// ------------------------------------------------------------------ batched small solves

// Which prepared solvers the one-workgroup batch kernel takes.
static void check_batchable(const mlb_solver* h) {
  if (h->format != MLB_CSR) throw Error{MLB_EUNSUPPORTED, "batched solves take CSR matrices"};
  if (h->opt.precision != MLB_PREC_FP64) throw Error{MLB_EUNSUPPORTED, "batched solves run in fp64"};
  if (h->opt.precond != MLB_PRECOND_NONE) throw Error{MLB_EUNSUPPORTED, "batched solves take no preconditioner"};
  if (h->opt.order != MLB_ORDER_FUSED) throw Error{MLB_EUNSUPPORTED, "batched solves run the fused order"};
  if (h->opt.max_restarts != 0) throw Error{MLB_EUNSUPPORTED, "batched solves take no restarts"};
  if (h->N > MLB_BATCH_MAX_N) throw Error{MLB_EUNSUPPORTED, "batched solves take at most MLB_BATCH_MAX_N rows"};
}

template <class V64, int NB>
static void launch_small(const SmallJob<V64, typename traits<V64>::wide>* dj, int count, hipStream_t s) {
  k_small<V64, typename traits<V64>::wide, NB><<<count, SB, 0, s>>>(dj);
}

// Runs the systems of hs (same dtype, same stream) in one launch of k_small and
// fills res[k] as mlbicgstab_solve would.
// job_buf: a device buffer for at least `count` job descriptors, or NULL to
// allocate one for the call (the serving batchers keep one each).
template <class V64, class V32>
static void batch_impl(mlb_solver* const* hs, int count, const void* const* b, void* const* x,
                       const void* const* Q, const int64_t* ldq, mlb_result* res,
                       Impl<V64, V32>* (*impl_of)(mlb_solver*), void* job_buf) {
  using Sc = typename traits<V64>::wide;
  hipStream_t s = hs[0]->s;
  std::vector<SmallJob<V64, Sc>> jobs((size_t)count);
  int nb = 4;
  for (int k = 0; k < count; ++k) {
    Engine<V64>& e = impl_of(hs[k])->e64;
    SmallJob<V64, Sc>& J = jobs[(size_t)k];
    J.N = e.N;
    J.n = e.n;
    J.rp = e.A.rp;
    J.ci = e.A.ci;
    J.val = e.A.val;
    J.rpT = e.AH.rp;
    J.ciT = e.AH.ci;
    J.valT = e.AH.val;
    J.b = (const V64*)b[k];
    J.x = (V64*)x[k];
    J.Q = (const V64*)Q[k];
    J.ldq = ldq[k];
    J.G = e.G;
    J.W = e.W;
    J.F = e.F;
    J.r = e.r;
    J.gt = e.gt;
    J.z = e.z;
    J.st = e.st;
    J.tol = hs[k]->opt.tol;
    J.kappa = hs[k]->opt.kappa;
    J.maxit = hs[k]->opt.maxit;
    J.host_done = e.host_done_dev;
    J.tf = e.tf ? 1 : 0;
    J.xrec = (V64*)hs[k]->opt.iterates;
    J.K = hs[k]->opt.record_iterates > 0 ? std::min<long long>(hs[k]->opt.record_iterates, hs[k]->opt.maxit) : 0;
    *(volatile int*)e.host_done = 0;
    nb = std::max(nb, bucket(e.n));
  }
  Allocs tmp(s, false);
  auto* dj = job_buf ? (SmallJob<V64, Sc>*)job_buf : tmp.get<SmallJob<V64, Sc>>((size_t)count);
  HIP_TRY(hipMemcpyAsync(dj, jobs.data(), sizeof(SmallJob<V64, Sc>) * count, hipMemcpyHostToDevice, s));
  hipEvent_t t0, t1;
  HIP_TRY(hipEventCreate(&t0));
  HIP_TRY(hipEventCreate(&t1));
  HIP_TRY(hipEventRecord(t0, s));
  switch (nb) {
    case 4: launch_small<V64, 4>(dj, count, s); break;
    case 8: launch_small<V64, 8>(dj, count, s); break;
    case 16: launch_small<V64, 16>(dj, count, s); break;
    default: launch_small<V64, 32>(dj, count, s); break;
  }
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipEventRecord(t1, s));
  HIP_TRY(hipEventSynchronize(t1));
  float ms = 0;
  HIP_TRY(hipEventElapsedTime(&ms, t0, t1));
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  for (int k = 0; k < count; ++k) {
    Impl<V64, V32>& im = *impl_of(hs[k]);
    State<Sc> st;
    HIP_TRY(hipMemcpyAsync(&st, im.e64.st, sizeof(State<Sc>), hipMemcpyDeviceToHost, s));
    im.e64.resid_sums(im.A0, (const V64*)b[k], (const V64*)x[k], im.r64);
    double rr, bb;
    im.e64.read_aux(&rr, &bb);   // synchronises the stream (st is then valid too)
    mlb_result R{};
    R.flag = st.done ? st.flag : 1;
    R.iter = st.iter;
    R.fp64_iters = st.iter;
    R.err_recursive = st.err;
    R.err_true = std::sqrt(rr) / (bb > 0 ? std::sqrt(bb) : 1.0);
    R.solve_ms = ms;
    if (res) res[k] = R;
    hs[k]->solved = true;
  }
}

static Impl<double, float>* real_impl(mlb_solver* h) { return h->real.get(); }
static Impl<cplx<double>, cplx<float>>* cplx_impl(mlb_solver* h) { return h->cpx.get(); }

static int solve_batch(mlb_solver* const* hs, int count, const void* const* b, void* const* x, const void* const* Q,
                       const int64_t* ldq, mlb_result* res, void* job_buf = nullptr) {
  if (!hs || !b || !x || !Q || !ldq) throw Error{MLB_EINVAL, "handles, b, x, Q and ldq must be non-NULL"};
  if (count < 1 || count > MLB_BATCH_MAX) throw Error{MLB_EINVAL, "count must be in [1, MLB_BATCH_MAX]"};
  for (int k = 0; k < count; ++k) {
    if (!hs[k]) throw Error{MLB_EINVAL, "a handle is NULL"};
    if (!b[k] || !x[k] || !Q[k]) throw Error{MLB_EINVAL, "b, x and Q must be device pointers"};
    if (ldq[k] < hs[k]->N) throw Error{MLB_EINVAL, "ldq must be >= N"};
    if (hs[k]->s != hs[0]->s) throw Error{MLB_EINVAL, "batched solvers must share one stream"};
    if (hs[k]->dtype != hs[0]->dtype) throw Error{MLB_EINVAL, "batched solvers must share one value type"};
    check_batchable(hs[k]);
  }
  if (hs[0]->real)
    batch_impl(hs, count, b, x, Q, ldq, res, real_impl, job_buf);
  else
    batch_impl(hs, count, b, x, Q, ldq, res, cplx_impl, job_buf);
  return 0;
}

}  // namespace mlb

// ------------------------------------------------------------------ C ABI

extern "C" {

int mlbicgstab_workspace_size(const mlb_matrix* A, const mlb_options* opt, size_t* bytes) {
  return guarded([&]() -> int {
    check_matrix(A);
    check_options(opt);
    if (!bytes) throw Error{MLB_EINVAL, "bytes pointer is NULL"};
    const int N = (int)A->nrows;
    const int nbr = A->format == MLB_BSR3 ? N / 3 : N;
    const int bs = A->format == MLB_BSR3 ? 9 : 1;
    const bool c = A->dtype == MLB_C128;
    const size_t sv = c ? 16 : 8;
    const bool tf = opt->transpose_free != 0;
    size_t t = tf ? 0 : (size_t)(nbr + 1) * 4 + (size_t)A->nnz * 4 + (size_t)A->nnz * bs * sv;   // A^H
    t += c ? Engine<cplx<double>>::bytes(N, opt->n, tf) : Engine<double>::bytes(N, opt->n, tf);
    t += (size_t)N * sv;                                                                   // r64
    if (opt->precond == MLB_PRECOND_JACOBI)                                                // M, M^{-1}, A M^{-1}
      t += (size_t)nbr * bs * 2 * sv + (size_t)A->nnz * bs * sv;
    if (opt->precond == MLB_PRECOND_ILU0)                                                  // factor, its transpose, M^{-1} v
      t += ilu_bytes(A->nnz, nbr, A->format == MLB_BSR3 ? 3 : 1, sv) + (size_t)N * sv;
    if (opt->precision == MLB_PREC_FP32_IR) {
      t += (size_t)A->nnz * bs * (tf ? sv / 2 : sv);                                       // fp32 A (and A^H) values
      t += c ? Engine<cplx<float>>::bytes(N, opt->n, tf) : Engine<float>::bytes(N, opt->n, tf);
      t += (size_t)N * (2 + opt->n) * (sv / 2);
    }
    *bytes = t;
    return 0;
  });
}

int mlbicgstab_create(const mlb_matrix* A, const mlb_options* opt, void* hip_stream, mlb_handle* out) {
  if (out) *out = nullptr;
  return guarded([&]() -> int {
    if (!out) throw Error{MLB_EINVAL, "out pointer is NULL"};
    *out = create_solver(A, opt, (hipStream_t)hip_stream, false, nullptr).release();
    return 0;
  });
}

int mlbicgstab_solve(mlb_handle h, const void* b, void* x, const void* Q, int64_t ldq, mlb_result* res) {
  return guarded([&]() -> int {
    if (!h) throw Error{MLB_EINVAL, "handle is NULL"};
    return solve_solver(h, b, x, Q, ldq, res);
  });
}

int mlbicgstab_destroy(mlb_handle h) {
  return guarded([&]() -> int {
    if (!h) return 0;
    (void)hipStreamSynchronize(h->s);
    delete h;
    return 0;
  });
}

int mlbicgstab_solve_batch(const mlb_handle* h, int32_t count, const void* const* b, void* const* x,
                           const void* const* Q, const int64_t* ldq, mlb_result* res) {
  return guarded([&]() -> int { return solve_batch(h, count, b, x, Q, ldq, res); });
}

const char* mlbicgstab_last_error(void) { return g_last_error.c_str(); }

// ---- sequences of systems with the automatic choice of n (Section 5.2)

int32_t mlb_sequence_next_n(int32_t n, double t_prev_ms, double t_cur_ms, int32_t step, int32_t n_min,
                            int32_t n_max) {
  if (step < 0 || n_min < 1 || n_max < n_min || n_max > MLB_MAX_N || n < n_min || n > n_max) return MLB_EINVAL;
  if (!(t_prev_ms >= 0.0) || !(t_cur_ms >= 0.0)) return n;   // no previous system yet
  const int32_t m = t_prev_ms > t_cur_ms ? n + step : n - step;
  return std::min(std::max(m, n_min), n_max);
}

}  // extern "C"

struct mlb_sequence {
  std::unique_ptr<mlb_solver> h;
  int32_t n_min = 1, n_max = 1, step = 1;
  double t_prev = -1.0;   // solve time of the previous system (ms), < 0 before the first
};

extern "C" {

int mlb_sequence_create(const mlb_matrix* A, const mlb_options* opt, int32_t n_min, int32_t n_max, int32_t step,
                        void* hip_stream, mlb_sequence_handle* out) {
  if (out) *out = nullptr;
  return guarded([&]() -> int {
    if (!A || !opt || !out) throw Error{MLB_EINVAL, "A, opt and out must be non-NULL"};
    check_options(opt);
    if (n_max > MLB_MAX_N) throw Error{MLB_EUNSUPPORTED, "n_max > MLB_MAX_N (32) is not supported"};
    if (step < 0 || n_min < 1 || n_max < n_min || opt->n < n_min || opt->n > n_max)
      throw Error{MLB_EINVAL, "need step >= 0 and 1 <= n_min <= opt->n <= n_max"};
    if (opt->record_iterates > 0) throw Error{MLB_EINVAL, "a sequence records no iterates"};
    mlb_options o = *opt;
    o.n = n_max;   // workspace for the largest n
    auto q = std::make_unique<mlb_sequence>();
    q->h = create_solver(A, &o, (hipStream_t)hip_stream, false, nullptr);
    set_active_n(q->h.get(), opt->n);
    q->n_min = n_min;
    q->n_max = n_max;
    q->step = step;
    *out = q.release();
    return 0;
  });
}

int mlb_sequence_solve(mlb_sequence_handle q, const void* b, void* x, const void* Q, int64_t ldq, mlb_result* res,
                       int32_t* n_used) {
  return guarded([&]() -> int {
    if (!q) throw Error{MLB_EINVAL, "sequence is NULL"};
    mlb_result R{};
    const int32_t n = q->h->n_active;
    const int rc = solve_solver(q->h.get(), b, x, Q, ldq, &R);
    if (res) *res = R;
    if (n_used) *n_used = n;
    const double t = R.solve_ms;
    set_active_n(q->h.get(), mlb_sequence_next_n(n, q->t_prev, t, q->step, q->n_min, q->n_max));
    q->t_prev = t;
    return rc;
  });
}

int mlb_sequence_destroy(mlb_sequence_handle q) {
  return guarded([&]() -> int {
    if (!q) return 0;
    (void)hipStreamSynchronize(q->h->s);
    delete q;
    return 0;
  });
}

int mlbicgstab_matvec(mlb_handle h, int32_t op, const void* x, void* y) {
  return guarded([&]() -> int {
    if (!h || !x || !y) throw Error{MLB_EINVAL, "handle, x and y must be non-NULL"};
    if (op < MLB_OP_A || op > MLB_OP_MINVH) throw Error{MLB_EINVAL, "op must be MLB_OP_A, _AH, _MINV or _MINVH"};
    if (op == MLB_OP_AH && (h->opt.transpose_free || h->opt.precond != MLB_PRECOND_NONE))
      throw Error{MLB_EUNSUPPORTED, "A^H is held only without transpose_free and without a preconditioner"};
    if ((op == MLB_OP_MINV || op == MLB_OP_MINVH) && h->opt.precond != MLB_PRECOND_ILU0)
      throw Error{MLB_EUNSUPPORTED, "M^{-1} and M^{-H} are applied for an ILU(0) preconditioner only"};
    if (h->real)
      matvec_impl(h, *h->real, op, (const double*)x, (double*)y);
    else
      matvec_impl(h, *h->cpx, op, (const cplx<double>*)x, (cplx<double>*)y);
    return 0;
  });
}

int mlbicgstab_time_kernel(mlb_handle h, int32_t kernel, int32_t reps, double* ms_per_launch) {
  return guarded([&]() -> int {
    if (!h || !ms_per_launch) throw Error{MLB_EINVAL, "handle and ms_per_launch must be non-NULL"};
    if (!h->solved) throw Error{MLB_EINVAL, "time_kernel needs a prior solve"};
    if (kernel < MLB_KERNEL_SPMV_STEP || kernel > MLB_KERNEL_RECOMBINE) throw Error{MLB_EINVAL, "unknown kernel"};
    if (reps < 1) throw Error{MLB_EINVAL, "reps must be >= 1"};
    const bool ir = h->opt.precision == MLB_PREC_FP32_IR;
    if (h->real)
      *ms_per_launch = ir ? time_kernel_impl(h->real->e32, kernel, reps) : time_kernel_impl(h->real->e64, kernel, reps);
    else
      *ms_per_launch = ir ? time_kernel_impl(h->cpx->e32, kernel, reps) : time_kernel_impl(h->cpx->e64, kernel, reps);
    return 0;
  });
}

}  // extern "C"

// ------------------------------------------------------------------ allocation-free solves
//
// mlbicgstab_solve_noalloc carves every device buffer of one create + solve
// (index check flag, A^H and its transpose temporaries, the Krylov workspace,
// partial sums, the scalar state) from one static device array per GPU.  In
// host code the array's name is only a stand-in: its device address on the
// current GPU comes from hipGetSymbolAddress, taken once per device and kept.
// The library's lock serialises these calls within a process, so two of them
// never share the array at once; each call re-initialises what it reads.

static __device__ __align__(256) unsigned char scratch[MLB_NOALLOC_SCRATCH_BYTES];

namespace mlb {

constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;                          // guards the table and the arrays
static char* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};    // device address of `scratch` per device

// Device address of the static scratch on the current device (looked up once).
static char* scratch_on_current_device() {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) throw Error{MLB_EUNSUPPORTED, "device ordinal beyond 63"};
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw Error{MLB_EHIP, "hipGetSymbolAddress returned no address for the scratch array"};
    g_scratch_ptr[dev] = (char*)p;
  }
  return g_scratch_ptr[dev];
}

// Scratch bytes an allocation-free solve of A with opt carves, in the order
// create_solver carves them (each piece padded to the arena alignment).
template <class V>
static size_t noalloc_bytes_t(const mlb_matrix* A, const mlb_options* opt) {
  const bool bsr = A->format == MLB_BSR3;
  const size_t N = (size_t)A->nrows;
  const size_t m = bsr ? N / 3 : N;
  const size_t bs = bsr ? 9 : 1;
  const size_t nnz = (size_t)A->nnz;
  const bool tf = opt->transpose_free != 0;
  size_t t = arena_bytes<int>(1);                                   // index check flag
  if (nnz == 0) t += arena_bytes<int>(1) + arena_bytes<V>(bs);       // stand-in index / value arrays
  if (!tf) {
    t += arena_bytes<int>(m + 1) + arena_bytes<int>(nnz) + arena_bytes<V>(nnz * bs);   // A^H
    t += 2 * arena_bytes<int>(m) + arena_bytes<int>((m + SCAN_TILE - 1) / SCAN_TILE + 1);   // its temporaries
  }
  t += Engine<V>::arena_need((int)N, opt->n, tf);
  t += arena_bytes<V>(N);                                           // fp64 residual
  return t;
}

static size_t noalloc_bytes(const mlb_matrix* A, const mlb_options* opt) {
  return A->dtype == MLB_C128 ? noalloc_bytes_t<cplx<double>>(A, opt) : noalloc_bytes_t<double>(A, opt);
}

}  // namespace mlb

extern "C" {

int mlbicgstab_solve_noalloc(const mlb_matrix* A, const mlb_options* opt, void* hip_stream, const void* b, void* x,
                             const void* Q, int64_t ldq, mlb_result* res) {
  return guarded([&]() -> int {
    check_matrix(A);
    check_options(opt);
    if (opt->precision != MLB_PREC_FP64)
      throw Error{MLB_EUNSUPPORTED, "the allocation-free solve runs the fp64 iteration only"};
    if (opt->precond != MLB_PRECOND_NONE)
      throw Error{MLB_EUNSUPPORTED, "the allocation-free solve takes no preconditioner"};
    if (!b || !x || !Q) throw Error{MLB_EINVAL, "b, x and Q must be device pointers"};
    if (ldq < A->nrows) throw Error{MLB_EINVAL, "ldq must be >= N"};
    const size_t need = noalloc_bytes(A, opt);
    if (need > (size_t)MLB_NOALLOC_SCRATCH_BYTES)
      throw Error{MLB_EUNSUPPORTED, "the allocation-free solve needs " + std::to_string(need) +
                                        " bytes of scratch for this A and n; the static scratch holds " +
                                        std::to_string((size_t)MLB_NOALLOC_SCRATCH_BYTES)};
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    char* base = scratch_on_current_device();
    auto h = create_solver(A, opt, (hipStream_t)hip_stream, false, nullptr, base, (size_t)MLB_NOALLOC_SCRATCH_BYTES);
    const int rc = solve_solver(h.get(), b, x, Q, ldq, res);
    HIP_TRY(hipStreamSynchronize(h->s));   // the scratch is free again when the lock is released
    return rc;
  });
}

}  // extern "C"

// ------------------------------------------------------------------ serving
//
// Continuous batching of whole solves.  Requests wait in a FIFO queue; each of
// max_inflight workers owns a HIP stream (non-blocking, default priority) and a
// pinned done-flag pair.  A worker takes the head request as soon as it is free
// and the request's device footprint (mlbicgstab_workspace_size) fits the
// unused part of the HBM budget, then runs create -> solve -> destroy on its
// stream with stream-ordered allocations.  Requests that arrive while others
// run are admitted as slots and memory free up; their kernels overlap on the
// device.  Every solve uses the same grids and reduction order as it would
// alone, so its result does not depend on what else is running.

namespace mlb {

static double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct SeqEntry;

struct Request {
  int64_t ticket = 0;
  mlb_matrix A{};
  mlb_options opt{};
  const void* b = nullptr;
  void* x = nullptr;
  const void* Q = nullptr;
  int64_t ldq = 0;
  size_t footprint = 0;
  double t_submit = 0, t_start = 0, t_done = 0;
  mlb_result res{};
  int rc = 0;
  std::string err;
  bool done = false;
  bool small = false;   // solved by a batcher (one workgroup per system)
  std::shared_ptr<SeqEntry> seq;   // the sequence it belongs to, or null
  int32_t n_used = 0;              // shadow vectors it ran with
};

// A sequence of systems with one A inside the server (Section 5.2): one solver
// (A^H, workspace for n_max) serves every request of the sequence, one request
// at a time in submission order, and n follows the rule of mlb_sequence_next_n
// from one request to the next.  Its footprint is admitted with its first
// request and held until the sequence ends.
struct SeqEntry {
  uint64_t key = 0;
  mlb_matrix A{};
  mlb_options opt{};
  int32_t n_min = 1, n_max = 1, step = 0, n_next = 1;
  double t_prev = -1.0;
  std::unique_ptr<mlb_solver> h;
  size_t footprint = 0;
  bool admitted = false;   // footprint counted in the server's used bytes
  bool busy = false;       // a worker is running one of its requests
  bool ending = false;     // mlb_server_end_sequence was called
  std::deque<std::shared_ptr<Request>> pending;   // taken while busy, in order
};

struct Server {
  size_t budget = 0, used = 0, peak = 0;
  int max_inflight = 1;
  int device = 0;
  int running = 0, peak_running = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Request>> queue;        // requests for the workers
  std::deque<std::shared_ptr<Request>> small_queue;  // requests for the batchers
  int small_n_max = 0;                                // largest N a batcher takes (0: none)
  int order = MLB_SERVE_FIFO;                         // the workers' pick order
  double max_wait_s = 1.0;                            // MLB_SERVE_SMALLEST: age that goes first
  std::unordered_map<int64_t, std::shared_ptr<Request>> table;
  std::unordered_map<uint64_t, std::shared_ptr<SeqEntry>> seqs;   // live sequences by key
  int64_t next_ticket = 1;
  int64_t completed = 0;
  bool stopping = false;
  std::vector<std::thread> workers, batchers;
  std::string init_error;
};

static void run_request(Request& r, hipStream_t st, int* flags) {
  try {
    auto h = create_solver(&r.A, &r.opt, st, true, flags);
    r.rc = solve_solver(h.get(), r.b, r.x, r.Q, r.ldq, &r.res);
    HIP_TRY(hipStreamSynchronize(st));
    h.reset();
    HIP_TRY(hipStreamSynchronize(st));
  } catch (const Error& e) {
    r.rc = e.code;
    r.err = e.msg;
  } catch (const std::exception& e) {
    r.rc = MLB_EHIP;
    r.err = e.what();
  }
}

// One request of a sequence on this worker's stream: the sequence's solver is
// created with its first request (own done flag, workspace for n_max) and moved
// to the stream of whichever worker runs the next one.
static void run_seq_request(SeqEntry& q, Request& r, hipStream_t st) {
  try {
    if (!q.h) {
      mlb_options o = q.opt;
      o.n = q.n_max;
      q.h = create_solver(&q.A, &o, st, true, nullptr);
    }
    set_stream(q.h.get(), st);
    set_active_n(q.h.get(), q.n_next);
    r.n_used = q.n_next;
    r.rc = solve_solver(q.h.get(), r.b, r.x, r.Q, r.ldq, &r.res);
    HIP_TRY(hipStreamSynchronize(st));
    const double t = r.res.solve_ms;
    q.n_next = mlb_sequence_next_n(r.n_used, q.t_prev, t, q.step, q.n_min, q.n_max);
    q.t_prev = t;
    set_stream(q.h.get(), nullptr);   // idle: frees, if any, go to the legacy stream
  } catch (const Error& e) {
    r.rc = e.code;
    r.err = e.msg;
  } catch (const std::exception& e) {
    r.rc = MLB_EHIP;
    r.err = e.what();
  }
}

// Whether a request of the worker queue may start now (its footprint fits; a
// sequence's is admitted once, with its first request).
static bool fits(const Server* S, const Request& r) {
  if (r.seq) return r.seq->busy || r.seq->admitted || S->used + r.seq->footprint <= S->budget;
  return S->used + r.footprint <= S->budget;
}

// The request a free worker takes next, or queue.end() if none may start now.
// FIFO: the head, once it fits.  SMALLEST: the oldest request that has waited
// max_wait_s (it holds the queue until it fits), else the smallest footprint
// that fits, the oldest among equal ones.
static std::deque<std::shared_ptr<Request>>::iterator pick(Server* S) {
  auto& q = S->queue;
  if (q.empty()) return q.end();
  if (S->order == MLB_SERVE_FIFO) return fits(S, *q.front()) ? q.begin() : q.end();
  if (now_s() - q.front()->t_submit >= S->max_wait_s) return fits(S, *q.front()) ? q.begin() : q.end();
  auto best = q.end();
  size_t best_fp = 0;
  for (auto it = q.begin(); it != q.end(); ++it) {
    const Request& r = **it;
    const size_t fp = r.seq ? r.seq->footprint : r.footprint;
    if ((best == q.end() || fp < best_fp) && fits(S, r)) {
      best = it;
      best_fp = fp;
    }
  }
  return best;
}

// Whether a request of sequence q still waits in the worker queue.
static bool seq_queued(const Server* S, const std::shared_ptr<SeqEntry>& q) {
  for (auto& r : S->queue)
    if (r->seq == q) return true;
  return false;
}

// Frees a finished sequence's solver (called without the server lock).
static void drop_sequence(std::shared_ptr<SeqEntry>& q) {
  if (!q || !q->h) return;
  (void)hipStreamSynchronize(q->h->s);
  q->h.reset();
}

static void worker_main(Server* S) {
  hipStream_t st = nullptr;
  int* flags = nullptr;
  bool ok = hipSetDevice(S->device) == hipSuccess && hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess &&
            hipHostMalloc((void**)&flags, 2 * sizeof(int), hipHostMallocMapped) == hipSuccess;
  while (true) {
    std::shared_ptr<Request> r;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      while (true) {
        // (age alone never makes a request startable: when none fits, only a
        // completion or a submission changes that, and both notify)
        auto it = S->queue.end();
        S->cv_work.wait(lk, [&] {
          if (S->stopping && S->queue.empty()) return true;
          it = pick(S);
          return it != S->queue.end();
        });
        if (S->queue.empty()) break;   // stopping and drained
        r = *it;
        S->queue.erase(it);
        if (r->seq && r->seq->busy) {   // its sequence runs on another worker, which takes it next
          r->seq->pending.push_back(r);
          r.reset();
          continue;
        }
        break;
      }
      if (!r) break;
      if (r->seq) {
        r->seq->busy = true;
        if (!r->seq->admitted) {
          S->used += r->seq->footprint;
          r->seq->admitted = true;
        }
      } else {
        S->used += r->footprint;
      }
      S->peak = std::max(S->peak, S->used);
      S->running++;
      S->peak_running = std::max(S->peak_running, S->running);
      r->t_start = now_s();
    }
    S->cv_work.notify_all();   // the next head may fit too
    while (r) {
      std::shared_ptr<SeqEntry> q = r->seq, finished;
      if (!ok) {
        r->rc = MLB_EHIP;
        r->err = "serving worker could not create its stream or pinned flags";
      } else if (q) {
        run_seq_request(*q, *r, st);
      } else {
        run_request(*r, st, flags);
      }
      std::shared_ptr<Request> next;
      {
        std::lock_guard<std::mutex> lk(S->mu);
        r->t_done = now_s();
        r->done = true;
        if (!q) S->used -= r->footprint;
        S->running--;
        S->completed++;
        if (q && !q->pending.empty()) {   // the sequence's next request, on this worker
          next = q->pending.front();
          q->pending.pop_front();
          S->running++;
          next->t_start = now_s();
        } else if (q) {
          q->busy = false;
          if (q->ending && !seq_queued(S, q)) {
            S->used -= q->footprint;
            S->seqs.erase(q->key);
            finished = q;
          }
        }
      }
      S->cv_work.notify_all();
      S->cv_done.notify_all();
      drop_sequence(finished);
      r = next;
    }
  }
  if (flags) (void)hipHostFree(flags);
  if (st) (void)hipStreamDestroy(st);
}

// A batcher takes every waiting small request that fits the budget (FIFO, at
// most BATCH_CAP), prepares each on its stream (validation, A^H, workspace),
// solves them all in one launch of the one-workgroup kernel and completes them
// together.  Requests that arrive meanwhile wait for the next batch of the
// next free batcher.
constexpr int BATCH_CAP = 256;
constexpr int N_BATCHERS = 2;

static void batcher_main(Server* S) {
  hipStream_t st = nullptr;
  int* flags = nullptr;
  void* jobs = nullptr;   // job descriptors of one batch, kept for the batcher's life
  const size_t job_bytes = BATCH_CAP * std::max(sizeof(SmallJob<double, double>),
                                                sizeof(SmallJob<cplx<double>, cplx<double>>));
  bool ok = hipSetDevice(S->device) == hipSuccess && hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess &&
            hipHostMalloc((void**)&flags, 2 * BATCH_CAP * sizeof(int), hipHostMallocMapped) == hipSuccess &&
            hipMalloc(&jobs, job_bytes) == hipSuccess;
  while (true) {
    std::vector<std::shared_ptr<Request>> batch;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_work.wait(lk, [&] {
        return (S->stopping && S->small_queue.empty()) ||
               (!S->small_queue.empty() && S->used + S->small_queue.front()->footprint <= S->budget);
      });
      if (S->small_queue.empty()) break;   // stopping and drained
      const double t = now_s();
      while (!S->small_queue.empty() && (int)batch.size() < BATCH_CAP &&
             S->used + S->small_queue.front()->footprint <= S->budget) {
        auto r = S->small_queue.front();
        S->small_queue.pop_front();
        S->used += r->footprint;
        r->t_start = t;
        batch.push_back(r);
      }
      S->peak = std::max(S->peak, S->used);
      S->running += (int)batch.size();
      S->peak_running = std::max(S->peak_running, S->running);
    }
    S->cv_work.notify_all();
    if (!ok) {
      for (auto& r : batch) {
        r->rc = MLB_EHIP;
        r->err = "serving batcher could not create its stream or pinned flags";
      }
    } else {
      std::vector<std::unique_ptr<mlb_solver>> hs(batch.size());
      std::vector<mlb_solver*> run;
      std::vector<const void*> bs, Qs;
      std::vector<void*> xs;
      std::vector<int64_t> lds;
      std::vector<size_t> idx;
      for (size_t k = 0; k < batch.size(); ++k) {
        Request& r = *batch[k];
        try {
          mlb_options ob = r.opt;   // the batched run itself takes no restarts (see below)
          ob.max_restarts = 0;
          hs[k] = create_solver(&r.A, &ob, st, true, flags + 2 * k);
          run.push_back(hs[k].get());
          bs.push_back(r.b);
          xs.push_back(r.x);
          Qs.push_back(r.Q);
          lds.push_back(r.ldq);
          idx.push_back(k);
        } catch (const Error& e) {
          r.rc = e.code;
          r.err = e.msg;
        } catch (const std::exception& e) {
          r.rc = MLB_EHIP;
          r.err = e.what();
        }
      }
      // one batch per value type (the kernel is instantiated per type)
      for (int pass = 0; pass < 2 && !run.empty(); ++pass) {
        std::vector<mlb_solver*> part;
        std::vector<const void*> pb, pq;
        std::vector<void*> px;
        std::vector<int64_t> pl;
        std::vector<size_t> pi;
        for (size_t q = 0; q < run.size(); ++q)
          if ((run[q]->dtype == MLB_C128) == (pass == 1)) {
            part.push_back(run[q]);
            pb.push_back(bs[q]);
            px.push_back(xs[q]);
            pq.push_back(Qs[q]);
            pl.push_back(lds[q]);
            pi.push_back(idx[q]);
          }
        if (part.empty()) continue;
        std::vector<mlb_result> res(part.size());
        try {
          solve_batch(part.data(), (int)part.size(), pb.data(), px.data(), pq.data(), pl.data(), res.data(), jobs);
          for (size_t q = 0; q < part.size(); ++q) {
            batch[pi[q]]->res = res[q];
            batch[pi[q]]->rc = res[q].flag;
          }
        } catch (const Error& e) {
          for (size_t q = 0; q < part.size(); ++q) {
            batch[pi[q]]->rc = e.code;
            batch[pi[q]]->err = e.msg;
          }
        } catch (const std::exception& e) {
          for (size_t q = 0; q < part.size(); ++q) {
            batch[pi[q]]->rc = MLB_EHIP;
            batch[pi[q]]->err = e.what();
          }
        }
      }
      for (auto& h : hs) h.reset();
      (void)hipStreamSynchronize(st);
      // a request with restarts whose batched run converged with its true residual not below
      // tol goes on from its x on the multi-launch iteration, within its admitted footprint
      for (size_t k = 0; k < batch.size(); ++k) {
        Request& r = *batch[k];
        if (r.rc != 0 || r.opt.max_restarts <= 0 || !(r.res.err_true >= r.opt.tol) || r.res.iter >= r.opt.maxit)
          continue;
        try {
          mlb_options o2 = r.opt;
          o2.max_restarts = r.opt.max_restarts - 1;
          o2.maxit = r.opt.maxit - r.res.iter;
          auto h2 = create_solver(&r.A, &o2, st, true, flags + 2 * k);
          mlb_result r2{};
          const int rc2 = solve_solver(h2.get(), r.b, r.x, r.Q, r.ldq, &r2);
          h2.reset();
          (void)hipStreamSynchronize(st);
          r.res.iter += r2.iter;
          r.res.fp64_iters += r2.fp64_iters;
          r.res.outer_iters = 1 + r2.outer_iters;
          r.res.err_true = r2.err_true;
          r.res.err_recursive = r2.err_recursive;
          r.res.solve_ms += r2.solve_ms;
          r.res.flag = rc2;
          r.rc = rc2;
        } catch (const Error& e) {
          r.rc = e.code;
          r.err = e.msg;
        } catch (const std::exception& e) {
          r.rc = MLB_EHIP;
          r.err = e.what();
        }
      }
    }
    {
      std::lock_guard<std::mutex> lk(S->mu);
      const double t = now_s();
      for (auto& r : batch) {
        r->t_done = t;
        r->done = true;
        S->used -= r->footprint;
        S->running--;
        S->completed++;
      }
    }
    S->cv_work.notify_all();
    S->cv_done.notify_all();
  }
  if (jobs) (void)hipFree(jobs);
  if (flags) (void)hipHostFree(flags);
  if (st) (void)hipStreamDestroy(st);
}

static void fill_timing(const Request& r, mlb_request_timing* t) {
  if (!t) return;
  t->queued_ms = 1e3 * (r.t_start - r.t_submit);
  t->run_ms = 1e3 * (r.t_done - r.t_start);
  t->latency_ms = 1e3 * (r.t_done - r.t_submit);
  t->footprint_bytes = r.seq ? r.seq->footprint : r.footprint;
  t->n_used = r.n_used ? r.n_used : r.opt.n;
}

}  // namespace mlb

struct mlb_server : mlb::Server {};

extern "C" {

int mlb_server_create(const mlb_server_options* o, mlb_server_handle* out) {
  if (out) *out = nullptr;
  return guarded([&]() -> int {
    if (!o || !out) throw Error{MLB_EINVAL, "options and out must be non-NULL"};
    if (o->budget_bytes == 0) throw Error{MLB_EINVAL, "budget_bytes must be > 0"};
    if (o->max_inflight < 1 || o->max_inflight > 64) throw Error{MLB_EINVAL, "max_inflight must be in [1, 64]"};
    if (o->small_n_max < -1 || o->small_n_max > MLB_BATCH_MAX_N)
      throw Error{MLB_EINVAL, "small_n_max must be -1, 0 or at most MLB_BATCH_MAX_N"};
    if (o->order != MLB_SERVE_FIFO && o->order != MLB_SERVE_SMALLEST)
      throw Error{MLB_EINVAL, "order must be MLB_SERVE_FIFO or MLB_SERVE_SMALLEST"};
    if (!(o->max_wait_ms >= 0.0) || !(o->max_wait_ms < 1e12)) throw Error{MLB_EINVAL, "max_wait_ms must be in [0, 1e12)"};
    auto S = std::make_unique<mlb_server>();
    S->budget = o->budget_bytes;
    S->max_inflight = o->max_inflight;
    S->small_n_max = o->small_n_max == 0 ? MLB_SERVER_SMALL_N : std::max(o->small_n_max, 0);
    S->order = o->order;
    S->max_wait_s = (o->max_wait_ms > 0.0 ? o->max_wait_ms : MLB_SERVER_MAX_WAIT_MS) * 1e-3;
    HIP_TRY(hipGetDevice(&S->device));
    // keep freed stream-ordered memory cached in the pool between requests
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, S->device) == hipSuccess) {
      uint64_t thr = UINT64_MAX;
      (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
    (void)hipGetLastError();
    for (int w = 0; w < o->max_inflight; ++w) S->workers.emplace_back(worker_main, S.get());
    if (S->small_n_max > 0)
      for (int w = 0; w < N_BATCHERS; ++w) S->batchers.emplace_back(batcher_main, S.get());
    *out = S.release();
    return 0;
  });
}

int mlb_server_submit(mlb_server_handle S, const mlb_matrix* A, const mlb_options* opt, const void* b, void* x,
                      const void* Q, int64_t ldq, int64_t* ticket) {
  return guarded([&]() -> int {
    if (!S || !ticket) throw Error{MLB_EINVAL, "server and ticket must be non-NULL"};
    check_matrix(A);
    check_options(opt);
    if (!b || !x || !Q) throw Error{MLB_EINVAL, "b, x and Q must be device pointers"};
    if (ldq < A->nrows) throw Error{MLB_EINVAL, "ldq must be >= N"};
    auto r = std::make_shared<Request>();
    r->A = *A;
    r->opt = *opt;
    r->b = b;
    r->x = x;
    r->Q = Q;
    r->ldq = ldq;
    size_t fp = 0;
    int rc = mlbicgstab_workspace_size(A, opt, &fp);
    if (rc != 0) throw Error{rc, g_last_error};
    r->footprint = fp;
    if (fp > S->budget) throw Error{MLB_ENOMEM, "request footprint exceeds the server's HBM budget"};
    {
      std::lock_guard<std::mutex> lk(S->mu);
      if (S->stopping) throw Error{MLB_EINVAL, "server is shutting down"};
      r->ticket = S->next_ticket++;
      r->t_submit = now_s();
      S->table[r->ticket] = r;
      r->small = A->format == MLB_CSR && opt->precision == MLB_PREC_FP64 && opt->precond == MLB_PRECOND_NONE &&
                 opt->record_iterates == 0 && opt->order == MLB_ORDER_FUSED && A->nrows <= S->small_n_max;
      (r->small ? S->small_queue : S->queue).push_back(r);
      *ticket = r->ticket;
    }
    S->cv_work.notify_all();
    return 0;
  });
}

static bool same_matrix(const mlb_matrix& a, const mlb_matrix& b) {
  return a.format == b.format && a.dtype == b.dtype && a.nrows == b.nrows && a.nnz == b.nnz && a.row_ptr == b.row_ptr &&
         a.col_idx == b.col_idx && a.values == b.values;
}

static bool same_options_but_n(const mlb_options& a, const mlb_options& b) {
  return a.tol == b.tol && a.maxit == b.maxit && a.kappa == b.kappa && a.precision == b.precision &&
         a.inner_tol == b.inner_tol && a.max_outer == b.max_outer && a.precond == b.precond &&
         a.transpose_free == b.transpose_free && a.order == b.order && a.max_restarts == b.max_restarts;
}

int mlb_server_submit_sequence(mlb_server_handle S, uint64_t key, const mlb_matrix* A, const mlb_options* opt,
                               int32_t n_min, int32_t n_max, int32_t step, const void* b, void* x, const void* Q,
                               int64_t ldq, int64_t* ticket) {
  return guarded([&]() -> int {
    if (!S || !ticket) throw Error{MLB_EINVAL, "server and ticket must be non-NULL"};
    if (key == 0) throw Error{MLB_EINVAL, "the sequence key must be nonzero"};
    check_matrix(A);
    check_options(opt);
    if (opt->record_iterates > 0) throw Error{MLB_EINVAL, "a sequence records no iterates"};
    if (n_max > MLB_MAX_N) throw Error{MLB_EUNSUPPORTED, "n_max > MLB_MAX_N (32) is not supported"};
    if (step < 0 || n_min < 1 || n_max < n_min || opt->n < n_min || opt->n > n_max)
      throw Error{MLB_EINVAL, "need step >= 0 and 1 <= n_min <= opt->n <= n_max"};
    if (!b || !x || !Q) throw Error{MLB_EINVAL, "b, x and Q must be device pointers"};
    if (ldq < A->nrows) throw Error{MLB_EINVAL, "ldq must be >= N"};
    mlb_options o = *opt;
    o.n = n_max;
    size_t fp = 0;
    int rc = mlbicgstab_workspace_size(A, &o, &fp);
    if (rc != 0) throw Error{rc, g_last_error};
    if (fp > S->budget) throw Error{MLB_ENOMEM, "the sequence's footprint exceeds the server's HBM budget"};
    auto r = std::make_shared<Request>();
    r->A = *A;
    r->opt = *opt;
    r->b = b;
    r->x = x;
    r->Q = Q;
    r->ldq = ldq;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      if (S->stopping) throw Error{MLB_EINVAL, "server is shutting down"};
      auto it = S->seqs.find(key);
      std::shared_ptr<SeqEntry> q;
      if (it == S->seqs.end()) {
        q = std::make_shared<SeqEntry>();
        q->key = key;
        q->A = *A;
        q->opt = *opt;
        q->n_min = n_min;
        q->n_max = n_max;
        q->step = step;
        q->n_next = opt->n;
        q->footprint = fp;
        S->seqs[key] = q;
      } else {
        q = it->second;
        if (q->ending) throw Error{MLB_EINVAL, "the sequence has been ended"};
        if (!same_matrix(q->A, *A)) throw Error{MLB_EINVAL, "a sequence keeps one A (the same device arrays)"};
        if (!same_options_but_n(q->opt, *opt) || q->n_min != n_min || q->n_max != n_max || q->step != step)
          throw Error{MLB_EINVAL, "a sequence keeps its options and its rule for n"};
      }
      r->seq = q;
      r->ticket = S->next_ticket++;
      r->t_submit = now_s();
      S->table[r->ticket] = r;
      S->queue.push_back(r);
      *ticket = r->ticket;
    }
    S->cv_work.notify_all();
    return 0;
  });
}

int mlb_server_end_sequence(mlb_server_handle S, uint64_t key) {
  return guarded([&]() -> int {
    if (!S) throw Error{MLB_EINVAL, "server is NULL"};
    std::shared_ptr<SeqEntry> finished;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      auto it = S->seqs.find(key);
      if (it == S->seqs.end()) throw Error{MLB_EINVAL, "no live sequence with this key"};
      auto q = it->second;
      q->ending = true;
      // requests of the sequence still queued keep it alive; the worker that
      // finishes the last one releases it
      if (!q->busy && q->pending.empty() && !seq_queued(S, q)) {
        if (q->admitted) S->used -= q->footprint;
        S->seqs.erase(it);
        finished = q;
      }
    }
    drop_sequence(finished);
    S->cv_work.notify_all();
    return 0;
  });
}

static int collect(mlb_server_handle S, int64_t ticket, mlb_result* res, mlb_request_timing* t, bool block) {
  std::shared_ptr<Request> r;
  {
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->table.find(ticket);
    if (it == S->table.end()) throw Error{MLB_EINVAL, "unknown or already collected ticket"};
    r = it->second;
    if (!r->done) {
      if (!block) return 0;
      S->cv_done.wait(lk, [&] { return r->done; });
    }
    S->table.erase(ticket);
  }
  if (res) *res = r->res;
  fill_timing(*r, t);
  if (r->rc <= -2) throw Error{r->rc, r->err};
  return 1;
}

int mlb_server_poll(mlb_server_handle S, int64_t ticket, mlb_result* res, mlb_request_timing* t) {
  return guarded([&]() -> int {
    if (!S) throw Error{MLB_EINVAL, "server is NULL"};
    return collect(S, ticket, res, t, false);
  });
}

int mlb_server_wait(mlb_server_handle S, int64_t ticket, mlb_result* res, mlb_request_timing* t) {
  return guarded([&]() -> int {
    if (!S) throw Error{MLB_EINVAL, "server is NULL"};
    return collect(S, ticket, res, t, true);
  });
}

int mlb_server_stats(mlb_server_handle S, mlb_server_stats_t* st) {
  return guarded([&]() -> int {
    if (!S || !st) throw Error{MLB_EINVAL, "server and stats must be non-NULL"};
    std::lock_guard<std::mutex> lk(S->mu);
    st->budget_bytes = S->budget;
    st->used_bytes = S->used;
    st->peak_used_bytes = S->peak;
    st->queued = (int64_t)(S->queue.size() + S->small_queue.size());
    st->running = S->running;
    st->peak_running = S->peak_running;
    st->completed = S->completed;
    return 0;
  });
}

int mlb_server_destroy(mlb_server_handle S) {
  return guarded([&]() -> int {
    if (!S) return 0;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->stopping = true;
    }
    S->cv_work.notify_all();
    for (auto& w : S->workers) w.join();
    for (auto& w : S->batchers) w.join();
    for (auto& kv : S->seqs) drop_sequence(kv.second);   // sequences never ended
    S->seqs.clear();
    delete S;
    return 0;
  });
}

}  // extern "C"
