// In-situ molecular species analysis (Section 3.4) over the corrected bond
// orders of the last force evaluation:
//   * atoms joined by a bond order above the threshold share a molecule whose
//     ID is the smallest global ID (the caller's atom index) among its atoms;
//   * molecule IDs are renumbered 1..M in increasing order;
//   * a species is a count of atoms per element; the summary lists each
//     distinct count vector with its number of molecules.
// The paper assigns the smaller ID of each bonded pair repeatedly until
// nothing changes, one sweep per step of the longest chain.  Here the
// components come from a lock-free union-find over caller indices in which a
// root is only ever hooked under a smaller root (one compare-and-swap), so
// every parent index is smaller than its child's, no cycle can form, and the
// root of each finished tree is its smallest member: the molecule ID itself,
// in one pass over the bonds however long the molecules are.  Finds halve
// their paths as they go.  Renumbering is a prefix sum over the roots; the
// species table comes from four stable radix sorts of the molecules by their
// element counts (least significant element first), so it is in increasing
// lexicographic order of (C, H, N, O) counts.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <string>

#include "internal.h"

namespace rx {

constexpr int SB = 256;

__device__ __forceinline__ int ld_rel(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rel(int32_t* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// root of v's tree; on the way, each visited node is pointed at its
// grandparent (still an ancestor with a smaller index)
__device__ __forceinline__ int uf_root(int32_t* p, int v) {
  int cur = v, par = ld_rel(p + v);
  while (par != cur) {
    const int gp = ld_rel(p + par);
    if (gp != par) st_rel(p + cur, gp);
    cur = par;
    par = gp;
  }
  return cur;
}

__device__ __forceinline__ void uf_union(int32_t* p, int a, int b) {
  for (;;) {
    a = uf_root(p, a);
    b = uf_root(p, b);
    if (a == b) return;
    if (a < b) {
      const int t = a;
      a = b;
      b = t;
    }
    // a > b: hook a under b if a is still a root
    if (atomicCAS(p + a, a, b) == a) return;
  }
}

__global__ __launch_bounds__(SB) void k_sp_init(int64_t n, int32_t* __restrict__ parent) {
  const int64_t g = blockIdx.x * (int64_t)SB + threadIdx.x;
  if (g < n) parent[g] = (int32_t)g;
}

// one thread per directed bond entry; each bond once (from its lower sorted atom)
__global__ __launch_bounds__(SB) void k_sp_union(Lists L, Work W, double thr, int32_t* parent) {
  const int64_t e = blockIdx.x * (int64_t)SB + threadIdx.x;
  if (e >= L.nbond) return;
  const int i = L.bond_i[e], j = L.bond_j[e];
  if (i < j && W.bo[e].x > thr) uf_union(parent, L.perm[i], L.perm[j]);
}

// roots flagged for the renumbering prefix sum
__global__ __launch_bounds__(SB) void k_sp_roots(int64_t n, int32_t* __restrict__ parent,
                                                 int32_t* __restrict__ isroot) {
  const int64_t g = blockIdx.x * (int64_t)SB + threadIdx.x;
  if (g < n) {
    const int r = uf_root(parent, (int)g);
    isroot[g] = r == (int)g ? 1 : 0;
  }
}

// molecule number of every atom and per-molecule element counts
__global__ __launch_bounds__(SB) void k_sp_number(Lists L, int32_t* __restrict__ parent,
                                                  const int32_t* __restrict__ rank, int32_t* __restrict__ mol,
                                                  int32_t* __restrict__ counts) {
  const int64_t i = blockIdx.x * (int64_t)SB + threadIdx.x;
  if (i >= L.n) return;
  const int g = L.perm[i];
  const int m = rank[uf_root(parent, g)];
  mol[g] = m + 1;
  atomicAdd(counts + 4 * (int64_t)m + L.type_s[i], 1);
}

__global__ __launch_bounds__(SB) void k_sp_iota(int64_t m, int32_t* __restrict__ v) {
  const int64_t k = blockIdx.x * (int64_t)SB + threadIdx.x;
  if (k < m) v[k] = (int32_t)k;
}

// key of molecule order[k] for the sort by element e
__global__ __launch_bounds__(SB) void k_sp_key(int64_t m, const int32_t* __restrict__ counts,
                                               const int32_t* __restrict__ order, int e,
                                               uint32_t* __restrict__ key) {
  const int64_t k = blockIdx.x * (int64_t)SB + threadIdx.x;
  if (k < m) key[k] = (uint32_t)counts[4 * (int64_t)order[k] + e];
}

__device__ __forceinline__ bool same_counts(const int32_t* c, int a, int b) {
  const int4 x = *reinterpret_cast<const int4*>(c + 4 * (int64_t)a);
  const int4 y = *reinterpret_cast<const int4*>(c + 4 * (int64_t)b);
  return x.x == y.x && x.y == y.y && x.z == y.z && x.w == y.w;
}

// 1 where a new species starts in the sorted molecule order
__global__ __launch_bounds__(SB) void k_sp_bounds(int64_t m, const int32_t* __restrict__ counts,
                                                  const int32_t* __restrict__ order, int32_t* __restrict__ flag) {
  const int64_t k = blockIdx.x * (int64_t)SB + threadIdx.x;
  if (k < m) flag[k] = (k == 0 || !same_counts(counts, order[k], order[k - 1])) ? 1 : 0;
}

// first sorted position of each species (start[S] = m)
__global__ __launch_bounds__(SB) void k_sp_starts(int64_t m, const int32_t* __restrict__ flag,
                                                  const int32_t* __restrict__ sid, int32_t* __restrict__ start) {
  const int64_t k = blockIdx.x * (int64_t)SB + threadIdx.x;
  if (k < m && flag[k]) start[sid[k]] = (int32_t)k;
  if (k == m) start[sid[m]] = (int32_t)m;
}

// species table rows (C, H, N, O counts, number of molecules)
__global__ __launch_bounds__(SB) void k_sp_table(int64_t ns, const int32_t* __restrict__ counts,
                                                 const int32_t* __restrict__ order, const int32_t* __restrict__ start,
                                                 int32_t* __restrict__ table) {
  const int64_t s = blockIdx.x * (int64_t)SB + threadIdx.x;
  if (s >= ns) return;
  const int32_t* c = counts + 4 * (int64_t)order[start[s]];
  int32_t* row = table + 5 * s;
  row[0] = c[0];
  row[1] = c[1];
  row[2] = c[2];
  row[3] = c[3];
  row[4] = start[s + 1] - start[s];
}

}  // namespace rx

using namespace rx;

namespace {

int sfail(reaxff_ctx* c, int code, const std::string& msg) {
  c->err = msg;
  return code;
}

#define SHIP(ctx, expr)                                                                  \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return sfail(ctx, REAXFF_ERR_HIP, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

inline unsigned nb(int64_t n) { return (unsigned)std::max<int64_t>((n + SB - 1) / SB, 1); }

}  // namespace

extern "C" {

int reaxff_species(reaxff_ctx* c, double bo_threshold, int32_t* mol, int32_t* mol_counts, int32_t* table,
                   int64_t* nmol, int64_t* nspecies, hipStream_t st) {
  if (!c) return REAXFF_ERR_ARG;
  if (!c->built || !c->forces_done) return sfail(c, REAXFF_ERR_STATE, "reaxff_species: no force evaluation yet");
  const int64_t n = c->L.n;
  if ((n > 0 && !mol) || !nmol || !nspecies || !std::isfinite(bo_threshold))
    return sfail(c, REAXFF_ERR_ARG, "reaxff_species: null pointer or non-finite threshold");
  SHIP(c, hipSetDevice(c->device));
  *nmol = 0;
  *nspecies = 0;
  if (n == 0) return REAXFF_OK;
  Species& S = c->species;
  if (n + 1 > S.cap) {
    for (int32_t** p : {&S.parent, &S.flag, &S.rank, &S.counts, &S.order, &S.order2, &S.sid})
      if (*p) (void)hipFree(*p);
    for (uint32_t** p : {&S.key, &S.key2})
      if (*p) (void)hipFree(*p);
    if (S.tmp) (void)hipFree(S.tmp);
    S = Species{};
    const int64_t cap = n + n / 8 + 64;
    SHIP(c, hipMalloc(&S.parent, sizeof(int32_t) * cap));
    SHIP(c, hipMalloc(&S.flag, sizeof(int32_t) * cap));
    SHIP(c, hipMalloc(&S.rank, sizeof(int32_t) * cap));
    SHIP(c, hipMalloc(&S.counts, sizeof(int32_t) * 4 * cap));
    SHIP(c, hipMalloc(&S.order, sizeof(int32_t) * cap));
    SHIP(c, hipMalloc(&S.order2, sizeof(int32_t) * cap));
    SHIP(c, hipMalloc(&S.sid, sizeof(int32_t) * cap));
    SHIP(c, hipMalloc(&S.key, sizeof(uint32_t) * cap));
    SHIP(c, hipMalloc(&S.key2, sizeof(uint32_t) * cap));
    S.cap = cap;
  }
  const Lists& L = c->L;
  hipLaunchKernelGGL(k_sp_init, dim3(nb(n)), dim3(SB), 0, st, n, S.parent);
  if (L.nbond > 0)
    hipLaunchKernelGGL(k_sp_union, dim3(nb(L.nbond)), dim3(SB), 0, st, L, c->W, bo_threshold, S.parent);
  hipLaunchKernelGGL(k_sp_roots, dim3(nb(n)), dim3(SB), 0, st, n, S.parent, S.flag);
  SHIP(c, hipMemsetAsync(S.flag + n, 0, sizeof(int32_t), st));
  if (scan_i32(S.flag, S.rank, n + 1, c->sc, st)) return sfail(c, REAXFF_ERR_HIP, "reaxff_species: scan");
  int32_t M = 0;
  SHIP(c, hipMemcpyAsync(&M, S.rank + n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  SHIP(c, hipStreamSynchronize(st));
  SHIP(c, hipMemsetAsync(S.counts, 0, sizeof(int32_t) * 4 * (int64_t)M, st));
  hipLaunchKernelGGL(k_sp_number, dim3(nb(n)), dim3(SB), 0, st, L, S.parent, S.rank, mol, S.counts);
  if (mol_counts)
    SHIP(c, hipMemcpyAsync(mol_counts, S.counts, sizeof(int32_t) * 4 * (int64_t)M, hipMemcpyDeviceToDevice, st));
  if (M == 0) {   // unreachable for n > 0 (every atom is in a molecule)
    SHIP(c, hipStreamSynchronize(st));
    return REAXFF_OK;
  }
  // species: stable sorts of the molecules by O, N, H, then C counts
  hipLaunchKernelGGL(k_sp_iota, dim3(nb(M)), dim3(SB), 0, st, (int64_t)M, S.order);
  size_t need = 0;
  SHIP(c, hipcub::DeviceRadixSort::SortPairs(nullptr, need, S.key, S.key2, S.order, S.order2, (int)M, 0, 32, st));
  if (need > S.tmp_bytes) {
    if (S.tmp) (void)hipFree(S.tmp);
    S.tmp = nullptr;
    S.tmp_bytes = 0;
    SHIP(c, hipMalloc(&S.tmp, need));
    S.tmp_bytes = need;
  }
  for (int e = 3; e >= 0; --e) {
    hipLaunchKernelGGL(k_sp_key, dim3(nb(M)), dim3(SB), 0, st, (int64_t)M, S.counts, S.order, e, S.key);
    size_t bytes = S.tmp_bytes;
    SHIP(c, hipcub::DeviceRadixSort::SortPairs(S.tmp, bytes, S.key, S.key2, S.order, S.order2, (int)M, 0, 32,
                                               st));
    std::swap(S.order, S.order2);
  }
  hipLaunchKernelGGL(k_sp_bounds, dim3(nb(M)), dim3(SB), 0, st, (int64_t)M, S.counts, S.order, S.flag);
  SHIP(c, hipMemsetAsync(S.flag + M, 0, sizeof(int32_t), st));
  if (scan_i32(S.flag, S.sid, (int64_t)M + 1, c->sc, st)) return sfail(c, REAXFF_ERR_HIP, "reaxff_species: scan");
  int32_t NS = 0;
  SHIP(c, hipMemcpyAsync(&NS, S.sid + M, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  SHIP(c, hipStreamSynchronize(st));
  if (table) {
    int32_t* start = S.rank;   // the renumbering ranks are no longer needed
    hipLaunchKernelGGL(k_sp_starts, dim3(nb((int64_t)M + 1)), dim3(SB), 0, st, (int64_t)M, S.flag, S.sid, start);
    hipLaunchKernelGGL(k_sp_table, dim3(nb(NS)), dim3(SB), 0, st, (int64_t)NS, S.counts, S.order, start, table);
    SHIP(c, hipStreamSynchronize(st));
  }
  SHIP(c, hipGetLastError());
  *nmol = M;
  *nspecies = NS;
  return REAXFF_OK;
}

}  // extern "C"
