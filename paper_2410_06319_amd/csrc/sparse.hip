// Sparse sign embedding (Section 2): Y = Omega [A b] where column i of Omega
// has zeta nonzeros +-1/sqrt(zeta) at distinct rows chosen uniformly at
// random.  Omega only adds and subtracts rows of [A b], so the sketch is an
// HBM-bound gather with binary64 accumulation, no MFMA.
//
// Steps (all deterministic; Y is the same bit for bit on every run):
//   1. one thread per row i of [A b] draws its zeta rows and signs from the
//      words of the Philox4x32-10 blocks with counter (i, t, prob, 1),
//      t = 0, 1, ...: word w proposes row floor(w s / 2^32), negative when w
//      is odd; a proposal equal to an earlier row of the column is skipped;
//      (destination row, 2 i + sign bit) pairs are written in (i, draw) order;
//   2. a stable counting sort of the pairs by destination row, so that each
//      row of Y lists its sources in increasing i: per tile of kTileRows
//      source rows an LDS histogram of destinations, a scan over (tile,
//      destination) giving every tile its first slot per destination, then
//      one wave per tile places its pairs in source order (a pair's rank
//      among equal destinations of its round of 64 rows by comparison in LDS);
//   3. [A b] is copied to row-major order (one pass), so that a source row is
//      one contiguous read;
//   4. one block per row of Y adds its source rows, with their signs, in that
//      order in binary64, then multiplies by 1/sqrt(zeta).
#include "common.h"
#include "kernels.h"

namespace ls {
namespace {
constexpr int kZetaMax = 32;          // nonzeros per column of Omega
constexpr int kSparseMaxWords = 256;  // Philox words a column may use before the draw fails
constexpr int kDrawThreads = 256;
constexpr int kGatherThreads = 256;
constexpr int kGatherCols = 4;        // columns of Y per thread in one sweep over the sources

__global__ __launch_bounds__(kDrawThreads) void k_ss_draw(int64_t m, int64_t s, int zeta, uint32_t key0,
                                                          uint32_t key1, uint32_t prob, uint32_t* __restrict__ keys,
                                                          uint32_t* __restrict__ vals, int* __restrict__ fail) {
  __shared__ uint32_t picks[kDrawThreads][kZetaMax + 1];
  const int64_t i = (int64_t)blockIdx.x * kDrawThreads + threadIdx.x;
  if (i >= m) return;
  uint32_t* mine = picks[threadIdx.x];
  int cnt = 0;
  for (uint32_t t = 0; cnt < zeta; ++t) {
    if (4 * (int)t >= kSparseMaxWords) {
      // draw failed: the remaining entries go past the last row of Y
      // (never gathered) and the call reports the failure
      *fail = 1;
      for (int k = cnt; k < zeta; ++k) {
        keys[i * zeta + k] = (uint32_t)s;
        vals[i * zeta + k] = 0u;
      }
      return;
    }
    uint32_t w0 = (uint32_t)i, w1 = t, w2 = prob, w3 = 1u;
    ls_philox4x32_10(w0, w1, w2, w3, key0, key1);
    const uint32_t w[4] = {w0, w1, w2, w3};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (cnt < zeta) {
        const uint32_t h = (uint32_t)(((uint64_t)w[q] * (uint64_t)s) >> 32);
        bool dup = false;
        for (int k = 0; k < cnt; ++k) dup |= (mine[k] == h);
        if (!dup) {
          mine[cnt] = h;
          keys[i * zeta + cnt] = h;
          vals[i * zeta + cnt] = ((uint32_t)i << 1) | (w[q] & 1u);
          ++cnt;
        }
      }
    }
  }
}

// ------------------------------------------------------------------ counting sort
constexpr int kTileRows = 256;     // source rows per tile of the counting sort
constexpr int kScanGroup = 32;     // tiles per group of the offset scan
constexpr int kSortBuckets = 8192; // destinations (rows of Y) the LDS histogram holds

// cnt[t s + r] = pairs of tile t with destination r (tile-major, so that the
// writes are coalesced).  Integer LDS atomics: the counts do not depend on
// their order.
__global__ __launch_bounds__(256) void k_ss_count(int64_t m, int64_t s, int zeta, const uint32_t* __restrict__ keys,
                                                  uint32_t* __restrict__ cnt) {
  __shared__ uint32_t h[kSortBuckets];
  const int64_t t = blockIdx.x;
  for (int64_t r = threadIdx.x; r < s; r += 256) h[r] = 0u;
  __syncthreads();
  const int64_t i = t * kTileRows + threadIdx.x;
  if (i < m)
    for (int k = 0; k < zeta; ++k) {
      const uint32_t d = keys[i * zeta + k];
      if (d < (uint32_t)s) atomicAdd(&h[d], 1u);
    }
  __syncthreads();
  for (int64_t r = threadIdx.x; r < s; r += 256) cnt[t * s + r] = h[r];
}

// Exclusive prefix over the tiles of each group (in place) and the group
// totals gsum[g s + r]; thread per destination, the group's tiles in order.
__global__ __launch_bounds__(256) void k_ss_scan_tiles(int64_t s, int64_t ntile, uint32_t* __restrict__ cnt,
                                                       uint32_t* __restrict__ gsum) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t g = blockIdx.y;
  if (r >= s) return;
  uint32_t acc = 0u;
  const int64_t t1 = (g + 1) * kScanGroup < ntile ? (g + 1) * kScanGroup : ntile;
  for (int64_t t = g * kScanGroup; t < t1; ++t) {
    const uint32_t c = cnt[t * s + r];
    cnt[t * s + r] = acc;
    acc += c;
  }
  gsum[g * s + r] = acc;
}

// Exclusive prefix over the groups of each destination (in place) and the
// destination totals; then (one block) the exclusive scan of the totals gives
// start[r], the first slot of destination r (start[s] = all pairs).
__global__ __launch_bounds__(256) void k_ss_scan_groups(int64_t s, int64_t ngroup, uint32_t* __restrict__ gsum,
                                                        uint32_t* __restrict__ total) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= s) return;
  uint32_t acc = 0u;
  for (int64_t g = 0; g < ngroup; ++g) {
    const uint32_t c = gsum[g * s + r];
    gsum[g * s + r] = acc;
    acc += c;
  }
  total[r] = acc;
}

__global__ __launch_bounds__(1024) void k_ss_scan_starts(int64_t s, const uint32_t* __restrict__ total,
                                                         int64_t* __restrict__ start) {
  __shared__ int64_t part[1024];
  // each thread a contiguous run of destinations, then a scan of the run sums
  const int64_t per = ls_cdiv(s, 1024);
  const int64_t r0 = (int64_t)threadIdx.x * per;
  int64_t sum = 0;
  for (int64_t r = r0; r < r0 + per && r < s; ++r) sum += total[r];
  part[threadIdx.x] = sum;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int64_t v = (threadIdx.x >= (unsigned)off) ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  int64_t acc = (threadIdx.x > 0) ? part[threadIdx.x - 1] : 0;
  for (int64_t r = r0; r < r0 + per && r < s; ++r) {
    start[r] = acc;
    acc += total[r];
  }
  if (threadIdx.x == 1023) start[s] = part[1023];
}

// One wave per tile: its pairs go to start[r] + (group offset) + (tile
// offset) + (rank among the tile's earlier pairs with destination r), in
// source order.  Rounds of 64 source rows (lane = row); a pair's rank within
// its round counts the pairs of lower lanes with the same destination (the
// pairs of one row have distinct destinations), read from LDS.
__global__ __launch_bounds__(64) void k_ss_scatter(int64_t m, int64_t s, int zeta, const uint32_t* __restrict__ keys,
                                                   const uint32_t* __restrict__ vals,
                                                   const uint32_t* __restrict__ cnt,
                                                   const uint32_t* __restrict__ gsum,
                                                   const int64_t* __restrict__ start,
                                                   uint32_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out) {
  __shared__ uint32_t base[kSortBuckets];
  __shared__ uint32_t rk[64 * kZetaMax];
  const int lane = threadIdx.x;
  const int64_t t = blockIdx.x;
  const int64_t g = t / kScanGroup;
  for (int64_t r = lane; r < s; r += 64) base[r] = (uint32_t)start[r] + gsum[g * s + r] + cnt[t * s + r];
  __syncthreads();
  for (int rd = 0; rd < kTileRows / 64; ++rd) {
    const int64_t i = t * kTileRows + rd * 64 + lane;
    const bool live = i < m;
    uint32_t mk[kZetaMax], mv[kZetaMax];
    for (int k = 0; k < zeta; ++k) {
      mk[k] = live ? keys[i * zeta + k] : 0xffffffffu;
      mv[k] = live ? vals[i * zeta + k] : 0u;
      rk[lane * zeta + k] = mk[k];
    }
    __syncthreads();
    for (int k = 0; k < zeta; ++k) {
      const uint32_t d = mk[k];
      if (!live || d >= (uint32_t)s) continue;   // failed draws point past the last row
      uint32_t rank = 0;
      for (int l = 0; l < lane; ++l)
        for (int k2 = 0; k2 < zeta; ++k2) rank += (rk[l * zeta + k2] == d) ? 1u : 0u;
      const uint32_t pos = base[d] + rank;
      keys_out[pos] = d;
      vals_out[pos] = mv[k];
    }
    __syncthreads();
    for (int k = 0; k < zeta; ++k)
      if (live && mk[k] < (uint32_t)s) atomicAdd(&base[mk[k]], 1u);
    __syncthreads();
  }
}

// T (m x (n+1), row-major) = [A b]; 32 x 32 tiles through LDS.
template <typename TA>
__global__ __launch_bounds__(256) void k_ss_transpose(const TA* __restrict__ A, int64_t lda, const TA* __restrict__ b,
                                                      int64_t m, int64_t n, TA* __restrict__ T) {
  __shared__ TA tile[32][33];
  const int64_t i0 = (int64_t)blockIdx.x * 32, j0 = (int64_t)blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t i = i0 + tx, j = j0 + ty + 8 * k;
    TA v = 0;
    if (i < m && j <= n) v = (j < n) ? A[i + j * lda] : b[i];
    tile[ty + 8 * k][tx] = v;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t i = i0 + ty + 8 * k, j = j0 + tx;
    if (i < m && j <= n) T[i * (n + 1) + j] = tile[tx][ty + 8 * k];
  }
}

// Row r of Y (one block): sum over its sources e (increasing i) of
// sign_e T[i_e, :], times scale; columns in sweeps of kGatherCols per thread.
template <typename TA>
__global__ __launch_bounds__(kGatherThreads) void k_ss_gather(const TA* __restrict__ T, int64_t n1,
                                                              const int64_t* __restrict__ start,
                                                              const uint32_t* __restrict__ vals, double scale,
                                                              double* __restrict__ Y, int64_t ldy) {
  const int64_t r = blockIdx.x;
  const int64_t lo = start[r], hi = start[r + 1];
  for (int64_t jc = 0; jc < n1; jc += (int64_t)kGatherThreads * kGatherCols) {
    double acc[kGatherCols];
#pragma unroll
    for (int q = 0; q < kGatherCols; ++q) acc[q] = 0.0;
    int64_t e = lo;
    for (; e + 4 <= hi; e += 4) {
      uint32_t v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = vals[e + u];
      TA x[4][kGatherCols];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const TA* row = T + (int64_t)(v[u] >> 1) * n1;
#pragma unroll
        for (int q = 0; q < kGatherCols; ++q) {
          const int64_t j = jc + threadIdx.x + (int64_t)kGatherThreads * q;
          x[u][q] = (j < n1) ? row[j] : TA(0);
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int q = 0; q < kGatherCols; ++q) {
          const double xv = (double)x[u][q];
          acc[q] += (v[u] & 1u) ? -xv : xv;
        }
    }
    for (; e < hi; ++e) {
      const uint32_t v = vals[e];
      const TA* row = T + (int64_t)(v >> 1) * n1;
#pragma unroll
      for (int q = 0; q < kGatherCols; ++q) {
        const int64_t j = jc + threadIdx.x + (int64_t)kGatherThreads * q;
        const double xv = (j < n1) ? (double)row[j] : 0.0;
        acc[q] += (v & 1u) ? -xv : xv;
      }
    }
#pragma unroll
    for (int q = 0; q < kGatherCols; ++q) {
      const int64_t j = jc + threadIdx.x + (int64_t)kGatherThreads * q;
      if (j < n1) Y[r + j * ldy] = acc[q] * scale;
    }
  }
}

struct SparseCarve {
  uint32_t *keys_in, *vals_in, *keys_out, *vals_out;
  int* fail;
  int64_t* start;
  uint32_t *cnt, *gsum, *total;
  char* T;
  size_t bytes;
};

SparseCarve sparse_carve(char* ws, int64_t m, int64_t n, int zeta, int64_t s, size_t ta_bytes) {
  SparseCarve c{};
  const int64_t N = m * zeta;
  const int64_t ntile = ls_cdiv(m, kTileRows), ngroup = ls_cdiv(ntile, kScanGroup);
  size_t off = 0;
  auto take = [&](size_t b) {
    char* q = ws ? ws + off : nullptr;
    off += ls_align256(b);
    return q;
  };
  c.keys_in = reinterpret_cast<uint32_t*>(take(4 * (size_t)N));
  c.vals_in = reinterpret_cast<uint32_t*>(take(4 * (size_t)N));
  c.keys_out = reinterpret_cast<uint32_t*>(take(4 * (size_t)N));
  c.vals_out = reinterpret_cast<uint32_t*>(take(4 * (size_t)N));
  c.fail = reinterpret_cast<int*>(take(sizeof(int)));
  c.start = reinterpret_cast<int64_t*>(take(8 * (size_t)(s + 1)));
  c.cnt = reinterpret_cast<uint32_t*>(take(4 * (size_t)ntile * s));
  c.gsum = reinterpret_cast<uint32_t*>(take(4 * (size_t)ngroup * s));
  c.total = reinterpret_cast<uint32_t*>(take(4 * (size_t)s));
  c.T = take(ta_bytes * (size_t)m * (size_t)(n + 1));
  c.bytes = off;
  return c;
}

template <typename TA>
int sparse_typed(const ls_problem_t* P, const ls_sketch_opts_t* so, int64_t s, double* Y, int64_t ldy, char* ws,
                 hipStream_t st) {
  const int64_t m = P->m, n = P->n, n1 = n + 1;
  const int zeta = so->zeta;
  const int64_t N = m * zeta;
  SparseCarve c = sparse_carve(ws, m, n, zeta, s, sizeof(TA));
  const uint32_t key0 = (uint32_t)(so->seed & 0xffffffffu), key1 = (uint32_t)(so->seed >> 32);
  LS_HIP_TRY(hipMemsetAsync(c.fail, 0, sizeof(int), st));
  hipLaunchKernelGGL(k_ss_draw, dim3((unsigned)ls_cdiv(m, kDrawThreads)), dim3(kDrawThreads), 0, st, m, s, zeta, key0,
                     key1, so->prob_id, c.keys_in, c.vals_in, c.fail);
  const int64_t ntile = ls_cdiv(m, kTileRows), ngroup = ls_cdiv(ntile, kScanGroup);
  hipLaunchKernelGGL(k_ss_count, dim3((unsigned)ntile), dim3(256), 0, st, m, s, zeta, c.keys_in, c.cnt);
  hipLaunchKernelGGL(k_ss_scan_tiles, dim3((unsigned)ls_cdiv(s, 256), (unsigned)ngroup), dim3(256), 0, st, s, ntile,
                     c.cnt, c.gsum);
  hipLaunchKernelGGL(k_ss_scan_groups, dim3((unsigned)ls_cdiv(s, 256)), dim3(256), 0, st, s, ngroup, c.gsum,
                     c.total);
  hipLaunchKernelGGL(k_ss_scan_starts, dim3(1), dim3(1024), 0, st, s, c.total, c.start);
  hipLaunchKernelGGL(k_ss_scatter, dim3((unsigned)ntile), dim3(64), 0, st, m, s, zeta, c.keys_in, c.vals_in, c.cnt,
                     c.gsum, c.start, c.keys_out, c.vals_out);
  const dim3 gt((unsigned)ls_cdiv(m, 32), (unsigned)ls_cdiv(n1, 32));
  hipLaunchKernelGGL((k_ss_transpose<TA>), gt, dim3(256), 0, st, static_cast<const TA*>(P->A), P->lda,
                     static_cast<const TA*>(P->b), m, n, reinterpret_cast<TA*>(c.T));
  const double scale = 1.0 / std::sqrt((double)zeta);
  const ProfEv ev = prof_events(kProfSparse);
  hipExtLaunchKernelGGL((k_ss_gather<TA>), dim3((unsigned)s), dim3(kGatherThreads), 0, st, ev.a, ev.b, 0,
                        reinterpret_cast<const TA*>(c.T), n1, c.start, c.vals_out, scale, Y, ldy);
  // [A b] once (as the transposed copy) and Y written
  prof_commit(kProfSparse, (double)m * n1 * sizeof(TA) + 8.0 * (double)s * n1);
  LS_HIP_TRY(hipGetLastError());
  int fail = 0;
  LS_HIP_TRY(hipMemcpyAsync(&fail, c.fail, sizeof(int), hipMemcpyDeviceToHost, st));
  LS_HIP_TRY(hipStreamSynchronize(st));
  return fail ? LS_E_UNSUPPORTED : LS_OK;
}
}  // namespace

size_t sparse_workspace(int64_t m, int64_t n, int zeta, int64_t s, size_t ta_bytes) {
  return sparse_carve(nullptr, m, n, zeta, s, ta_bytes).bytes;
}

int sparse_check(int64_t m, int zeta, int64_t s) {
  if (zeta < 2 || zeta > kZetaMax || 4 * (int64_t)zeta > s) return LS_E_ARG;
  if (s > kSortBuckets) return LS_E_UNSUPPORTED;
  if (m * (int64_t)zeta >= ((int64_t)1 << 31) || m >= ((int64_t)1 << 31)) return LS_E_UNSUPPORTED;
  return LS_OK;
}

int sparse_run(const ls_problem_t* P, const ls_sketch_opts_t* so, int64_t s, double* Y, int64_t ldy, char* ws,
               hipStream_t st) {
  if (P->store == LS_FP32) return sparse_typed<float>(P, so, s, Y, ldy, ws, st);
  if (P->store == LS_FP64) return sparse_typed<double>(P, so, s, Y, ldy, ws, st);
  return LS_E_UNSUPPORTED;
}

}  // namespace ls
