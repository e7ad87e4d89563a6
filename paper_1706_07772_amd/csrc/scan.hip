// Exclusive prefix sums over per-atom counts (the offsets of every CSR list).
// Three passes: per-tile sums, a scan of the tile sums (recursive), and the
// per-tile scan with the tile's offset added.  Tiles are 1024 elements
// (256 threads x 4).
#include "internal.h"

namespace rx {

constexpr int SCAN_BS = 256;
constexpr int SCAN_IPT = 4;
constexpr int SCAN_TILE = SCAN_BS * SCAN_IPT;

template <class TI>
__global__ __launch_bounds__(SCAN_BS) void k_tile_sums(const TI* __restrict__ in, int64_t n,
                                                       int64_t* __restrict__ sums) {
  __shared__ int64_t sh[SCAN_BS / 64];
  const int64_t base = blockIdx.x * (int64_t)SCAN_TILE;
  int64_t v = 0;
  for (int k = 0; k < SCAN_IPT; ++k) {
    const int64_t idx = base + threadIdx.x * SCAN_IPT + k;
    if (idx < n) v += (int64_t)in[idx];
  }
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t s = 0;
    for (int w = 0; w < SCAN_BS / 64; ++w) s += sh[w];
    sums[blockIdx.x] = s;
  }
}

// block-wide exclusive scan of one value per thread
__device__ __forceinline__ int64_t block_excl_scan(int64_t v, int64_t* total) {
  __shared__ int64_t wsum[SCAN_BS / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int64_t x = v;
  for (int off = 1; off < 64; off <<= 1) {
    const int64_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  int64_t pre = 0, tot = 0;
  for (int k = 0; k < SCAN_BS / 64; ++k) {
    if (k < w) pre += wsum[k];
    tot += wsum[k];
  }
  __syncthreads();
  *total = tot;
  return pre + x - v;
}

template <class TI, class TO>
__global__ __launch_bounds__(SCAN_BS) void k_tile_scan(const TI* __restrict__ in, int64_t n,
                                                       const int64_t* __restrict__ offs,
                                                       TO* __restrict__ out) {
  const int64_t base = blockIdx.x * (int64_t)SCAN_TILE;
  int64_t loc[SCAN_IPT];
  int64_t s = 0;
  for (int k = 0; k < SCAN_IPT; ++k) {
    const int64_t idx = base + threadIdx.x * SCAN_IPT + k;
    loc[k] = idx < n ? (int64_t)in[idx] : 0;
    s += loc[k];
  }
  int64_t tot;
  int64_t pre = block_excl_scan(s, &tot) + (offs ? offs[blockIdx.x] : 0);
  for (int k = 0; k < SCAN_IPT; ++k) {
    const int64_t idx = base + threadIdx.x * SCAN_IPT + k;
    if (idx < n) out[idx] = (TO)pre;
    pre += loc[k];
  }
}

static int64_t tiles_of(int64_t n) { return (n + SCAN_TILE - 1) / SCAN_TILE; }

// exclusive scan of int64 sums in place, using tmp beyond it for deeper levels
static void scan_sums(int64_t* sums, int64_t m, int64_t* tmp, hipStream_t st) {
  if (m <= 1) {
    if (m == 1) hipMemsetAsync(sums, 0, sizeof(int64_t), st);
    return;
  }
  if (m <= SCAN_TILE) {
    hipLaunchKernelGGL((k_tile_scan<int64_t, int64_t>), dim3(1), dim3(SCAN_BS), 0, st, sums, m,
                       (const int64_t*)nullptr, sums);
    return;
  }
  const int64_t t = tiles_of(m);
  int64_t* sub = tmp;
  hipLaunchKernelGGL((k_tile_sums<int64_t>), dim3((unsigned)t), dim3(SCAN_BS), 0, st, sums, m, sub);
  scan_sums(sub, t, tmp + t, st);
  hipLaunchKernelGGL((k_tile_scan<int64_t, int64_t>), dim3((unsigned)t), dim3(SCAN_BS), 0, st,
                     sums, m, sub, sums);
}

static int ensure_tmp(Scratch& sc, int64_t n) {
  int64_t need = 16;
  for (int64_t m = tiles_of(n); m > 1; m = tiles_of(m)) need += m + 16;
  if (need <= sc.scan_cap) return 0;
  if (sc.scan_tmp) hipFree(sc.scan_tmp);
  sc.scan_tmp = nullptr;
  sc.scan_cap = 0;
  if (hipMalloc(&sc.scan_tmp, sizeof(int64_t) * need) != hipSuccess) return -1;
  sc.scan_cap = need;
  return 0;
}

template <class TI, class TO>
static int scan_any(const TI* in, TO* out, int64_t n, Scratch& sc, hipStream_t st) {
  if (n <= 0) return 0;
  if (ensure_tmp(sc, n)) return -1;
  const int64_t t = tiles_of(n);
  int64_t* sums = sc.scan_tmp;
  if (t == 1) {
    hipLaunchKernelGGL((k_tile_scan<TI, TO>), dim3(1), dim3(SCAN_BS), 0, st, in, n,
                       (const int64_t*)nullptr, out);
  } else {
    hipLaunchKernelGGL((k_tile_sums<TI>), dim3((unsigned)t), dim3(SCAN_BS), 0, st, in, n, sums);
    scan_sums(sums, t, sums + t, st);
    hipLaunchKernelGGL((k_tile_scan<TI, TO>), dim3((unsigned)t), dim3(SCAN_BS), 0, st, in, n, sums,
                       out);
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int scan_i32(const int32_t* in, int32_t* out, int64_t n, Scratch& sc, hipStream_t st) {
  return scan_any<int32_t, int32_t>(in, out, n, sc, st);
}
int scan_i32_to_i64(const int32_t* in, int64_t* out, int64_t n, Scratch& sc, hipStream_t st) {
  return scan_any<int32_t, int64_t>(in, out, n, sc, st);
}

}  // namespace rx
