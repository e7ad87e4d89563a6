// Batched ReaxFF: thousands of small non-periodic clusters in one persistent
// launch replayed from a HIP graph.
//
// One workgroup evaluates one cluster at a time, stage by stage, with a
// workgroup barrier between stages: the same stages and the same arithmetic
// (terms.h) as the one-launch-per-stage path, with
//   * the cluster's atoms (x, y, z, q), types, bond-row offsets and the
//     nonbonded/H-bond force accumulators in LDS;
//   * the bond list built as the paper builds its lists (Section 3.3): each
//     pair tested once, rows counted, prefix-summed and filled, here inside
//     the workgroup;
//   * far-neighbour and H-bond relations tested in place over all pairs of
//     the cluster (same predicates as the stored lists of the large path);
//   * the per-entry and per-atom work arrays in a private slice of device
//     scratch per persistent workgroup (L2-resident while it works).
// Clusters come from a per-workgroup list (static or longest-processing-
// time-first) or from an atomic queue, chosen by the autotuner.
#include <algorithm>
#include <climits>
#include <cmath>
#include <mutex>
#include <numeric>
#include <queue>

#include "internal.h"
#include "terms.h"

using namespace rx;

namespace rx {

constexpr int BNMAX = REAXFF_BATCH_MAX_ATOMS;
constexpr int NCOUNT = 5;   // angles, torsions, hbonds, far pairs, bonds

// status bits of a cluster: bond entries beyond the scratch slice, an atom
// type outside 0..3, offsets that do not describe a cluster of at most the
// slice's atom count (only the device-offset entry point can pass those)
constexpr int ST_CAPACITY = 1, ST_TYPE = 2, ST_SIZE = 4;

// byte offsets of the arrays inside one workgroup's scratch slice
struct BatchLayout {
  int64_t ast, dp, gS, gSig, gRso, gSBO, gStot, gDp;    // per atom (nmax)
  int64_t bj, bi, bm;                             // per entry (ecap), int32
  int64_t bd, bop, dbop, bo, gbo, gvec, gup;      // per entry, double4
  int64_t stride;
};

static BatchLayout make_layout(int nmax, int ecap) {
  BatchLayout y{};
  int64_t o = 0;
  auto take = [&](int64_t bytes) {
    const int64_t at = o;
    o += (bytes + 255) & ~int64_t(255);
    return at;
  };
  y.ast = take(sizeof(AtomState) * (int64_t)nmax);
  y.dp = take(sizeof(double2) * (int64_t)nmax);
  y.gS = take(sizeof(double) * (int64_t)nmax);
  y.gSig = take(sizeof(double) * (int64_t)nmax);
  y.gRso = take(sizeof(double) * (int64_t)nmax);
  y.gSBO = take(sizeof(double) * (int64_t)nmax);
  y.gStot = take(sizeof(double) * (int64_t)nmax);
  y.gDp = take(sizeof(double) * (int64_t)nmax);
  y.bj = take(sizeof(int32_t) * (int64_t)ecap);
  y.bi = take(sizeof(int32_t) * (int64_t)ecap);
  y.bm = take(sizeof(int32_t) * (int64_t)ecap);
  y.bd = take(sizeof(double4) * (int64_t)ecap);
  y.bop = take(sizeof(double4) * (int64_t)ecap);
  y.dbop = take(sizeof(double4) * (int64_t)ecap);
  y.bo = take(sizeof(double4) * (int64_t)ecap);
  y.gbo = take(sizeof(double4) * (int64_t)ecap);
  y.gvec = take(sizeof(double4) * (int64_t)ecap);
  y.gup = take(sizeof(double4) * (int64_t)ecap);
  y.stride = o;
  return y;
}

struct BatchArgs {
  const DevParams* P;
  int32_t ncl;
  int32_t dynamic;           // 1: clusters from the queue, in `order`
  const int64_t* off;        // [ncl + 1] atom offsets
  const int32_t* order;      // cluster order (grouped per workgroup for static schedules);
                             // null: the queue hands out clusters in index order
  const int32_t* wg_first;   // [G + 1] static schedules: workgroup b takes order[wg_first[b] ..)
  int32_t* queue;            // [1] next position in `order` (dynamic)
  const double* pos;
  const int32_t* type;
  const double* q;
  double* forces;
  double* energies;          // [ncl][NTERMS]
  long long* counts;         // [ncl][NCOUNT], or null
  int32_t* status;           // [ncl], or null
  int32_t* err;              // [0] OR of statuses, [1] largest entry count, [2] lowest bad cluster
  char* scratch;
  BatchLayout lay;
  int32_t ecap;
  int32_t nmax;              // atoms per cluster the slice holds
};

__global__ void k_batch_reset(int32_t* queue, int32_t* err) {
  if (threadIdx.x == 0) {
    queue[0] = 0;
    err[0] = 0;
    err[1] = 0;
    err[2] = INT_MAX;
  }
}

// inclusive prefix sum of v[1..n] in place (v[0] = 0), by the first wavefront
__device__ __forceinline__ void wave_scan_inplace(int32_t* v, int n) {
  if (threadIdx.x >= 64) return;
  const int lane = threadIdx.x;
  int carry = 0;
  for (int base = 1; base <= n; base += 64) {
    const int k = base + lane;
    int x = k <= n ? v[k] : 0;
    for (int d = 1; d < 64; d <<= 1) {
      const int y = __shfl_up(x, d, 64);
      if (lane >= d) x += y;
    }
    x += carry;
    if (k <= n) v[k] = x;
    carry = __shfl(x, 63, 64);
  }
}

// wavefront sum of v added to an LDS accumulator (one LDS atomic per wave)
__device__ __forceinline__ void wave_acc(double v, double* acc) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((threadIdx.x & 63) == 0 && v != 0.0) atomicAdd(acc, v);
}

// LDS of the workgroup's current cluster
constexpr int NRED = NTERMS + NCOUNT;
__shared__ double4 b_x[BNMAX];        // x, y, z, q
__shared__ int32_t b_ty[BNMAX];
__shared__ int32_t b_off[BNMAX + 1];  // bond rows
__shared__ double4 b_f[BNMAX];        // nonbonded + H-bond forces
__shared__ NbP b_nb[NT * NT];
__shared__ HbP b_hb[NT * NT * NT];
__shared__ double b_reach2[NT * NT];  // min(bond reach, r_bond)^2 of each type pair
__shared__ int32_t b_alist[BNMAX];    // the cluster's acceptors, in index order
__shared__ int32_t b_aoff[BNMAX + 1]; // angle counts per centre, then their offsets
__shared__ int32_t b_nacc;
__shared__ double b_acc[NRED];        // per-cluster energies and counts
__shared__ int32_t b_next;

// The kernel's argument block, copied to LDS once per workgroup.  A stage
// function reads it back with readfirstlane, so its fields and every pointer
// derived from them are wave-uniform (scalar registers) inside the stage.
__shared__ BatchArgs b_args;

template <class T>
__device__ __forceinline__ T uni_copy(const T& src) {
  static_assert(sizeof(T) % 4 == 0, "copied as 32-bit words");
  T out;
  const int* s = reinterpret_cast<const int*>(&src);
  int* d = reinterpret_cast<int*>(&out);
#pragma unroll
  for (int k = 0; k < (int)(sizeof(T) / 4); ++k) d[k] = __builtin_amdgcn_readfirstlane(s[k]);
  return out;
}

// values the caller holds uniformly across the wavefront, made scalar again
// after the call boundary (arguments of called functions arrive in vector
// registers)
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni64(int64_t v) {
  const int lo = __builtin_amdgcn_readfirstlane((int)v);
  const int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
  return ((int64_t)hi << 32) | (uint32_t)lo;
}

// views of this workgroup's scratch slice, with atoms and forces in LDS
__device__ __forceinline__ void views(const BatchArgs& A, Lists& L, Work& W) {
  char* base = A.scratch + (int64_t)blockIdx.x * A.lay.stride;
  L = Lists{};
  W = Work{};
  L.xs = b_x;
  L.type_s = b_ty;
  L.bond_off = b_off;
  L.bond_j = reinterpret_cast<int32_t*>(base + A.lay.bj);
  L.bond_i = reinterpret_cast<int32_t*>(base + A.lay.bi);
  L.bond_mir = reinterpret_cast<int32_t*>(base + A.lay.bm);
  W.ast = reinterpret_cast<AtomState*>(base + A.lay.ast);
  W.dp = reinterpret_cast<double2*>(base + A.lay.dp);
  W.gS = reinterpret_cast<double*>(base + A.lay.gS);
  W.gSig = reinterpret_cast<double*>(base + A.lay.gSig);
  W.gRso = reinterpret_cast<double*>(base + A.lay.gRso);
  W.gSBO = reinterpret_cast<double*>(base + A.lay.gSBO);
  W.gStot = reinterpret_cast<double*>(base + A.lay.gStot);
  W.gDp = reinterpret_cast<double*>(base + A.lay.gDp);
  W.bd = reinterpret_cast<double4*>(base + A.lay.bd);
  W.bop = reinterpret_cast<double4*>(base + A.lay.bop);
  W.dbop = reinterpret_cast<double4*>(base + A.lay.dbop);
  W.bo = reinterpret_cast<double4*>(base + A.lay.bo);
  W.gbo = reinterpret_cast<double4*>(base + A.lay.gbo);
  W.gvec = reinterpret_cast<double4*>(base + A.lay.gvec);
  W.gup = reinterpret_cast<double4*>(base + A.lay.gup);
  W.fnb = b_f;
}

// Each stage is a separate (not inlined) function so that it gets its own
// register allocation: the kernel's register count is the largest stage's,
// not the union over all stages.

// load the cluster; returns nonzero on a bad type
template <int BSZ>
__device__ __noinline__ int st_load(int64_t a0, int n) {
  const BatchArgs A = uni_copy(b_args);
  a0 = uni64(a0);
  n = uni(n);
  Lists L;
  Work W;
  views(A, L, W);
  const int tid = threadIdx.x;
  if (tid < NRED) b_acc[tid] = 0.0;
  int bad = 0;
  for (int i = tid; i < n; i += BSZ) {
    int t = A.type[a0 + i];
    if (t < 0 || t >= NT) {
      bad = 1;
      t = 0;
    }
    b_x[i] = make_double4(A.pos[3 * (a0 + i)], A.pos[3 * (a0 + i) + 1], A.pos[3 * (a0 + i) + 2], A.q[a0 + i]);
    b_ty[i] = t;
    b_f[i] = make_double4(0.0, 0.0, 0.0, 0.0);
    b_off[i + 1] = 0;
    W.gSBO[i] = 0.0;
  }
  if (tid == 0) b_off[0] = 0;
  return bad;
}

// a failed cluster: NaN outputs and its status
template <int BSZ>
__device__ __noinline__ void st_fail(int c, int64_t a0, int n, int code, int nent) {
  const BatchArgs A = uni_copy(b_args);
  c = uni(c);
  a0 = uni64(a0);
  n = uni(n);
  code = uni(code);
  nent = uni(nent);
  const int tid = threadIdx.x;
  const double nan = __longlong_as_double(0x7ff8000000000000LL);
  for (int i = tid; i < 3 * n; i += BSZ) A.forces[3 * a0 + i] = nan;
  if (tid < NTERMS) A.energies[(int64_t)c * NTERMS + tid] = nan;
  if (tid == 0) {
    if (A.status) A.status[c] = code;
    atomicOr(&A.err[0], code);
    if (code == ST_CAPACITY) atomicMax(&A.err[1], nent);
    atomicMin(&A.err[2], c);
  }
}

// bond rows: count per atom (and far pairs, for the counts)
template <int BSZ>
__device__ __noinline__ void st_count(int n, int far) {
  const BatchArgs A = uni_copy(b_args);
  n = uni(n);
  far = uni(far);
  const DevParams* __restrict__ P = A.P;
  const double rn2 = P->rn2, rb2 = P->r_bond * P->r_bond, bo_cut = P->bo_cut;
  const int tid = threadIdx.x;
  double nfar = 0.0;
  for (int i = tid; i < n; i += BSZ) {
    const double4 xi = b_x[i];
    const int ti = b_ty[i];
    int nb = 0;
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      const double4 xj = b_x[j];
      const double r2 = r2_of(xj.x - xi.x, xj.y - xi.y, xj.z - xi.z);
      if (j > i && r2 <= rn2) nfar += 1.0;
      const PairP& p = P->pair[ti * NT + b_ty[j]];
      if (r2 <= fmin(p.reach2, rb2) && bo_raw(p, sqrt(r2), bo_cut) >= bo_cut) ++nb;
    }
    b_off[i + 1] = nb;
  }
  if (tid == 0) b_off[0] = 0;
  if (far) wave_acc(nfar, &b_acc[NTERMS + 3]);
}

// bond rows: fill (same predicate, same order) and clear the entry adjoints
template <int BSZ>
__device__ __noinline__ void st_fill(int n) {
  const BatchArgs A = uni_copy(b_args);
  n = uni(n);
  Lists L;
  Work W;
  views(A, L, W);
  const DevParams* __restrict__ P = A.P;
  const double rb2 = P->r_bond * P->r_bond, bo_cut = P->bo_cut;
  for (int i = threadIdx.x; i < n; i += BSZ) {
    const double4 xi = b_x[i];
    const int ti = b_ty[i];
    int e = b_off[i];
    const int e1 = b_off[i + 1];
    for (int j = 0; j < n && e < e1; ++j) {
      if (j == i) continue;
      const double4 xj = b_x[j];
      const double r2 = r2_of(xj.x - xi.x, xj.y - xi.y, xj.z - xi.z);
      const PairP& p = P->pair[ti * NT + b_ty[j]];
      if (r2 <= fmin(p.reach2, rb2) && bo_raw(p, sqrt(r2), bo_cut) >= bo_cut) {
        L.bond_j[e] = j;
        L.bond_i[e] = i;
        W.gbo[e] = make_double4(0.0, 0.0, 0.0, 0.0);
        W.gvec[e] = make_double4(0.0, 0.0, 0.0, 0.0);
        ++e;
      }
    }
  }
}

// the cluster's acceptors listed in index order, by the first wavefront
template <int BSZ>
__device__ __noinline__ void st_acceptors(int n) {
  const BatchArgs A = uni_copy(b_args);
  n = uni(n);
  if (threadIdx.x >= 64) return;
  const int lane = threadIdx.x;
  int na = 0;
  for (int b = 0; b < n; b += 64) {
    const int i = b + lane;
    const bool a = i < n && A.P->atom[b_ty[i]].hbond == 2;
    const unsigned long long m = ballot(a);
    if (a) b_alist[na + __popcll(m & ((1ull << lane) - 1ull))] = i;
    na += __popcll(m);
  }
  if (lane == 0) b_nacc = na;
}

// Bond rows with each pair tested once: one wavefront per atom i, one
// partner j > i per lane.  Pairs within the bond reach of their types are
// queued in LDS (per wavefront) and their raw bond orders evaluated 64 at a
// time, so the bond-order test runs on full wavefronts.  A bond goes to both
// atoms' staging rows (BSTAGE entries per atom, in the storage of the
// entries' bond-order derivatives, which is written only later) at places
// taken with LDS atomics on the row counts b_off[1..n]; far pairs are
// counted.  A count above BSTAGE means the staging row overflowed (the caller
// then builds the rows by the two full sweeps st_count and st_fill).
constexpr int BSTAGE = 32;

struct PairQ {
  int32_t i, j;
  double r2;
};

template <int BSZ>
__device__ __noinline__ void st_pairs(int n) {
  __shared__ PairQ cq[BSZ / 64][128];
  const BatchArgs A = uni_copy(b_args);
  n = uni(n);
  int32_t* __restrict__ stage =
      reinterpret_cast<int32_t*>(A.scratch + (int64_t)blockIdx.x * A.lay.stride + A.lay.dbop);
  const DevParams* __restrict__ P = A.P;
  const double rn2 = P->rn2, bo_cut = P->bo_cut;
  constexpr int NW = BSZ / 64;
  const int lane = threadIdx.x & 63;
  const unsigned long long below = (1ull << lane) - 1ull;
  PairQ* __restrict__ q = cq[threadIdx.x >> 6];
  auto sync_wave = [] {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };
  // the first cnt queued pairs, one per lane
  auto test = [&](int cnt) {
    if (lane < cnt) {
      const PairQ e = q[lane];
      const int ti = b_ty[e.i], tj = b_ty[e.j];
      if (bo_raw(P->pair[ti * NT + tj], sqrt(e.r2), bo_cut) >= bo_cut) {
        const int ki = atomicAdd(&b_off[e.i + 1], 1), kj = atomicAdd(&b_off[e.j + 1], 1);
        if (ki < BSTAGE) stage[e.i * BSTAGE + ki] = e.j;
        if (kj < BSTAGE) stage[e.j * BSTAGE + kj] = e.i;
      }
    }
  };
  int qn = 0;   // queued pairs (uniform)
  double nfar = 0.0;
  for (int i = threadIdx.x >> 6; i < n; i += NW) {
    const double4 xi = b_x[i];
    const int ti = b_ty[i];
    for (int j0 = i + 1; j0 < n; j0 += 64) {
      const int j = j0 + lane;
      bool cand = false;
      double r2 = 0.0;
      if (j < n) {
        const double4 xj = b_x[j];
        r2 = r2_of(xj.x - xi.x, xj.y - xi.y, xj.z - xi.z);
        if (r2 <= rn2) nfar += 1.0;
        cand = r2 <= b_reach2[ti * NT + b_ty[j]];
      }
      const unsigned long long m = ballot(cand);
      if (cand) q[qn + __popcll(m & below)] = PairQ{i, j, r2};
      qn += __popcll(m);
      if (qn >= 64) {
        sync_wave();
        test(64);
        sync_wave();
        if (lane < qn - 64) q[lane] = q[64 + lane];
        sync_wave();
        qn -= 64;
      }
    }
  }
  sync_wave();
  test(qn);
  wave_acc(nfar, &b_acc[NTERMS + 3]);
}

// staged bond rows -> the rows at their offsets, in increasing partner order
// (insertion sort: rows hold a few bonds); entry adjoints cleared
template <int BSZ>
__device__ __noinline__ void st_rows(int n) {
  const BatchArgs A = uni_copy(b_args);
  n = uni(n);
  Lists L;
  Work W;
  views(A, L, W);
  const int32_t* __restrict__ stage =
      reinterpret_cast<const int32_t*>(A.scratch + (int64_t)blockIdx.x * A.lay.stride + A.lay.dbop);
  for (int i = threadIdx.x; i < n; i += BSZ) {
    const int e0 = b_off[i], m = b_off[i + 1] - e0;
    for (int k = 0; k < m; ++k) {
      const int v = stage[i * BSTAGE + k];
      int t = k - 1;
      while (t >= 0 && L.bond_j[e0 + t] > v) {
        L.bond_j[e0 + t + 1] = L.bond_j[e0 + t];
        --t;
      }
      L.bond_j[e0 + t + 1] = v;
      L.bond_i[e0 + k] = i;
      W.gbo[e0 + k] = make_double4(0.0, 0.0, 0.0, 0.0);
      W.gvec[e0 + k] = make_double4(0.0, 0.0, 0.0, 0.0);
    }
  }
}

// mirror entries and uncorrected bond orders
template <int BSZ>
__device__ __noinline__ void st_bo_prime(int n) {
  const BatchArgs A = uni_copy(b_args);
  n = uni(n);
  Lists L;
  Work W;
  views(A, L, W);
  Grid g{};
  g.periodic = 0;
  // one bond entry per thread: an atom's entries are independent here
  const int ne = b_off[n];
  for (int e = threadIdx.x; e < ne; e += BSZ) {
    const int i = L.bond_i[e], j = L.bond_j[e];
    int m = e;
    for (int f = b_off[j]; f < b_off[j + 1]; ++f)
      if (L.bond_j[f] == i) m = f;
    L.bond_mir[e] = m;
    bo_prime_entry(A.P, g, L, W, i, e);
  }
}

template <int BSZ>
__device__ __noinline__ void st_delta_prime(int n) {
  const BatchArgs A = uni_copy(b_args);
  n = uni(n);
  Lists L;
  Work W;
  views(A, L, W);
  for (int i = threadIdx.x; i < n; i += BSZ) delta_prime_atom(A.P, L, W, i);
}

template <int BSZ>
__device__ __noinline__ void st_bo_corr(int n) {
  const BatchArgs A = uni_copy(b_args);
  n = uni(n);
  Lists L;
  Work W;
  views(A, L, W);
  const int ne = b_off[n];
  for (int e = threadIdx.x; e < ne; e += BSZ) bo_corr_entry(A.P, L, W, L.bond_i[e], e);
}

template <int BSZ>
__device__ __noinline__ void st_atom_state(int n) {
  const BatchArgs A = uni_copy(b_args);
  n = uni(n);
  Lists L;
  Work W;
  views(A, L, W);
  for (int i = threadIdx.x; i < n; i += BSZ) atom_state_atom(A.P, L, W, i);
}

// per atom: bond, lone-pair, over- and under-coordination energies
template <int BSZ>
__device__ __noinline__ void st_atom_energy(int n) {
  const BatchArgs A = uni_copy(b_args);
  n = uni(n);
  Lists L;
  Work W;
  views(A, L, W);
  double e4[4] = {0.0, 0.0, 0.0, 0.0};
  for (int j = threadIdx.x; j < n; j += BSZ) atom_energy_atom(A.P, L, W, j, e4);
  for (int k = 0; k < 4; ++k) wave_acc(e4[k], &b_acc[E_BOND + k]);
}

// valence angles centred on each atom (one thread owns all of the centre's
// entries, so no atomics)
template <int BSZ>
__device__ __noinline__ void st_angles(int n) {
  const BatchArgs A = uni_copy(b_args);
  n = uni(n);
  Lists L;
  Work W;
  views(A, L, W);
  const DevParams* __restrict__ P = A.P;
  const double thb = P->thb_cut, thb2 = P->thb_cutsq;
  double ev = 0.0, ep = 0.0, ec = 0.0, nang = 0.0;
  for (int j = threadIdx.x; j < n; j += BSZ) {
    const int e0 = b_off[j], e1 = b_off[j + 1];
    double gS = 0.0, gSBO2 = 0.0;
    for (int u = e0; u < e1; ++u) {
      const double bu = W.bo[u].x;
      if (!(bu - thb > 0.0)) continue;
      for (int v = u + 1; v < e1; ++v) {
        const double bv = W.bo[v].x;
        if (!(bv - thb > 0.0 && bu * bv > thb2)) continue;
        const AngOut o = angle_eval(P, L, W, u, v);
        ev += o.ev;
        ep += o.ep;
        ec += o.ec;
        nang += 1.0;
        double4 gu = W.gvec[u], gv = W.gvec[v];
        gu.x += o.gu[0]; gu.y += o.gu[1]; gu.z += o.gu[2];
        gv.x += o.gv[0]; gv.y += o.gv[1]; gv.z += o.gv[2];
        W.gvec[u] = gu;
        W.gvec[v] = gv;
        W.gbo[u].x += o.gu[3];
        W.gbo[u].w += o.gu[4];
        W.gbo[v].x += o.gv[3];
        W.gbo[v].w += o.gv[4];
        gS += o.gS;
        gSBO2 += o.gSBO2;
      }
    }
    W.gS[j] += gS;
    W.gSBO[j] = gSBO2;
  }
  wave_acc(ev, &b_acc[E_VAL]);
  wave_acc(ep, &b_acc[E_PEN]);
  wave_acc(ec, &b_acc[E_COA]);
  wave_acc(nang, &b_acc[NTERMS + 0]);
}

// Valence angles in three passes, when the cluster's angles fit in the
// storage of the entries' correction adjoints (written only later, by the
// backward pass): count each centre's angles (b_aoff), evaluate them 64 at a
// time (every lane walks its centre's pairs one per step, all lanes together,
// and the passing pairs are queued), each angle's adjoints stored at its
// centre's offset, then one thread per centre adds its angles' adjoints to
// its own entries in the order st_angles would, so no atomics are needed and
// the sums are deterministic.
constexpr int ANG_STAGE = 3;   // double4 records per staged angle

template <int BSZ>
__device__ __noinline__ void st_angle_count(int n) {
  const BatchArgs A = uni_copy(b_args);
  n = uni(n);
  Lists L;
  Work W;
  views(A, L, W);
  const double thb = A.P->thb_cut, thb2 = A.P->thb_cutsq;
  for (int j = threadIdx.x; j < n; j += BSZ) {
    const int e0 = b_off[j], e1 = b_off[j + 1];
    int cnt = 0;
    for (int u = e0; u < e1; ++u) {
      const double bu = W.bo[u].x;
      if (!(bu - thb > 0.0)) continue;
      for (int v = u + 1; v < e1; ++v) {
        const double bv = W.bo[v].x;
        cnt += (bv - thb > 0.0 && bu * bv > thb2) ? 1 : 0;
      }
    }
    b_aoff[j + 1] = cnt;
  }
  if (threadIdx.x == 0) b_aoff[0] = 0;
}

struct AngQ {
  int32_t u, v, slot, pad;
};

template <int BSZ>
__device__ __noinline__ void st_angle_eval(int n) {
  __shared__ AngQ aq[BSZ / 64][128];
  const BatchArgs A = uni_copy(b_args);
  n = uni(n);
  Lists L;
  Work W;
  views(A, L, W);
  const DevParams* __restrict__ P = A.P;
  const double thb = P->thb_cut, thb2 = P->thb_cutsq;
  double4* __restrict__ stage = W.gup;
  const int lane = threadIdx.x & 63;
  const unsigned long long below = (1ull << lane) - 1ull;
  AngQ* __restrict__ q = aq[threadIdx.x >> 6];
  auto sync_wave = [] {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };
  double ev = 0.0, ep = 0.0, ec = 0.0, nang = 0.0;
  auto evaluate = [&](int m) {   // the first m queued angles, one per lane
    if (lane < m) {
      const AngQ e = q[lane];
      const AngOut o = angle_eval(P, L, W, e.u, e.v);
      ev += o.ev;
      ep += o.ep;
      ec += o.ec;
      nang += 1.0;
      double4* __restrict__ r = stage + (int64_t)e.slot * ANG_STAGE;
      r[0] = make_double4(o.gu[0], o.gu[1], o.gu[2], o.gu[3]);
      r[1] = make_double4(o.gu[4], o.gv[0], o.gv[1], o.gv[2]);
      r[2] = make_double4(o.gv[3], o.gv[4], o.gS, o.gSBO2);
    }
  };
  int qn = 0;   // queued angles (uniform)
  for (int jb = threadIdx.x - lane; jb < n; jb += BSZ) {
    const int j = jb + lane;
    const int e0 = j < n ? b_off[j] : 0, e1 = j < n ? b_off[j + 1] : 0;
    int slot = j < n ? b_aoff[j] : 0;
    // the next pair is (u, v); v = e1 makes the first step look for the first u
    int u = e0 - 1, v = e1;
    double bu = 0.0;
    bool on = j < n && e1 - e0 > 1;
    while (ballot(on)) {
      bool cand = false;
      if (on) {
        ++v;
        if (v >= e1) {   // next u with BO - thb > 0
          ++u;
          while (u < e1 && !(W.bo[u].x - thb > 0.0)) ++u;
          if (u + 1 < e1) {
            bu = W.bo[u].x;
            v = u + 1;
          } else {
            on = false;
          }
        }
        if (on) {
          const double bv = W.bo[v].x;
          cand = bv - thb > 0.0 && bu * bv > thb2;
        }
      }
      const unsigned long long m = ballot(cand);
      if (cand) q[qn + __popcll(m & below)] = AngQ{u, v, slot, 0};
      slot += cand ? 1 : 0;
      qn += __popcll(m);
      if (qn >= 64) {
        sync_wave();
        evaluate(64);
        sync_wave();
        if (lane < qn - 64) q[lane] = q[64 + lane];
        sync_wave();
        qn -= 64;
      }
    }
  }
  sync_wave();
  evaluate(qn);
  wave_acc(ev, &b_acc[E_VAL]);
  wave_acc(ep, &b_acc[E_PEN]);
  wave_acc(ec, &b_acc[E_COA]);
  wave_acc(nang, &b_acc[NTERMS + 0]);
}

template <int BSZ>
__device__ __noinline__ void st_angle_gather(int n) {
  const BatchArgs A = uni_copy(b_args);
  n = uni(n);
  Lists L;
  Work W;
  views(A, L, W);
  const double thb = A.P->thb_cut, thb2 = A.P->thb_cutsq;
  const double4* __restrict__ stage = W.gup;
  for (int j = threadIdx.x; j < n; j += BSZ) {
    const int e0 = b_off[j], e1 = b_off[j + 1];
    int slot = b_aoff[j];
    double gS = 0.0, gSBO2 = 0.0;
    for (int u = e0; u < e1; ++u) {
      const double bu = W.bo[u].x;
      if (!(bu - thb > 0.0)) continue;
      for (int v = u + 1; v < e1; ++v) {
        const double bv = W.bo[v].x;
        if (!(bv - thb > 0.0 && bu * bv > thb2)) continue;
        const double4* __restrict__ r = stage + (int64_t)slot * ANG_STAGE;
        ++slot;
        const double4 r0 = r[0], r1 = r[1], r2 = r[2];
        double4 gu = W.gvec[u], gv = W.gvec[v];
        gu.x += r0.x; gu.y += r0.y; gu.z += r0.z;
        gv.x += r1.y; gv.y += r1.z; gv.z += r1.w;
        W.gvec[u] = gu;
        W.gvec[v] = gv;
        W.gbo[u].x += r0.w;
        W.gbo[u].w += r1.x;
        W.gbo[v].x += r2.x;
        W.gbo[v].w += r2.y;
        gS += r2.z;
        gSBO2 += r2.w;
      }
    }
    W.gS[j] += gS;
    W.gSBO[j] = gSBO2;
  }
}

// nonbonded: one wavefront per atom i, one partner j > i per lane, so every
// unordered pair is evaluated once; the partner's force goes to the LDS force
// array with atomic adds, the atom's own sum is reduced over the wavefront
template <int BSZ>
__device__ __noinline__ void st_nonbonded(int n) {
  const BatchArgs A = uni_copy(b_args);
  n = uni(n);
  const DevParams* __restrict__ P = A.P;
  const double rn2 = P->rn2, iR = P->inv_r_nonb, pv = P->p_vdW1, ipv = P->inv_p_vdW1;
  constexpr int NW = BSZ / 64;
  const int lane = threadIdx.x & 63;
  double ev = 0.0, eq = 0.0;
  for (int i = threadIdx.x >> 6; i < n; i += NW) {
    const double4 xi = b_x[i];
    const double qi = xi.w * C_ELE;
    const NbP* __restrict__ spi = b_nb + b_ty[i] * NT;
    double fx = 0.0, fy = 0.0, fz = 0.0;
    for (int j = i + 1 + lane; j < n; j += 64) {
      const double4 xj = b_x[j];
      const double dx = xj.x - xi.x, dy = xj.y - xi.y, dz = xj.z - xi.z;
      const double r2 = r2_of(dx, dy, dz);
      if (!(r2 <= rn2)) continue;
      const NbOut o = nb_pair(spi[b_ty[j]], iR, pv, ipv, qi * xj.w, r2);
      ev += o.ev;
      eq += o.eq;
      fx += o.f * dx;
      fy += o.f * dy;
      fz += o.f * dz;
      atomic_add3(&b_f[j], -o.f * dx, -o.f * dy, -o.f * dz);
    }
    for (int off = 32; off > 0; off >>= 1) {
      fx += __shfl_down(fx, off, 64);
      fy += __shfl_down(fy, off, 64);
      fz += __shfl_down(fz, off, 64);
    }
    if (lane == 0) atomic_add3(&b_f[i], fx, fy, fz);
  }
  wave_acc(ev, &b_acc[E_VDW]);
  wave_acc(eq, &b_acc[E_COUL]);
}

// torsions about the bonds each atom owns (lower index), with atomic adds.
// Each lane walks the candidates (j-k, j-i, k-l) of its atom j one per step
// (the central bond, then j's other bonds, then k's), all lanes stepping
// together; the candidates that pass the thresholds are queued in LDS and
// evaluated 64 at a time, so the torsion term runs on full wavefronts.
struct TorQ {
  int32_t u, a, b, pad;
};

template <int BSZ>
__device__ __noinline__ void st_torsions(int n) {
  __shared__ TorQ tq[BSZ / 64][128];
  const BatchArgs A = uni_copy(b_args);
  n = uni(n);
  Lists L;
  Work W;
  views(A, L, W);
  const DevParams* __restrict__ P = A.P;
  const double thb = P->thb_cut;
  const int lane = threadIdx.x & 63;
  const unsigned long long below = (1ull << lane) - 1ull;
  TorQ* __restrict__ q = tq[threadIdx.x >> 6];
  auto sync_wave = [] {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };
  double etor = 0.0, econj = 0.0, ntor = 0.0;
  auto evaluate = [&](int m) {   // the first m queued torsions, one per lane
    if (lane < m) {
      const TorQ e = q[lane];
      torsion_eval(P, L, W, e.u, e.a, e.b, etor, econj);
      ntor += 1.0;
    }
  };
  int qn = 0;   // queued torsions (uniform)
  for (int jb = threadIdx.x - lane; jb < n; jb += BSZ) {
    const int j = jb + lane;
    const int e0 = j < n ? b_off[j] : 0, e1 = j < n ? b_off[j + 1] : 0;
    // the next candidate is (u, a, b); a = e1 makes the first step look for
    // the first central bond
    int u = e0 - 1, a = e1, bb = 0, f0 = 0, f1 = 0;
    double bu = 0.0;
    bool on = j < n && e0 < e1;
    while (ballot(on)) {
      bool cand = false;
      if (on) {
        ++bb;
        if (bb >= f1) {
          ++a;
          bb = f0;
        }
        if (a >= e1) {   // next central bond j-k with k > j and BO > thb
          ++u;
          while (u < e1 && !(L.bond_j[u] > j && W.bo[u].x > thb)) ++u;
          if (u < e1) {
            const int k = L.bond_j[u];
            bu = W.bo[u].x;
            f0 = b_off[k];
            f1 = b_off[k + 1];
            a = e0;
            bb = f0;
          } else {
            on = false;
          }
        }
        if (on && a != u) {
          const double ba = W.bo[a].x;
          const int i = L.bond_j[a];
          const int l = L.bond_j[bb];
          const double bl = W.bo[bb].x;
          cand = ba > thb && l != j && l != i && bl > thb && ba * bu * bl > thb;
        }
      }
      const unsigned long long m = ballot(cand);
      if (cand) q[qn + __popcll(m & below)] = TorQ{u, a, bb, 0};
      qn += __popcll(m);
      if (qn >= 64) {
        sync_wave();
        evaluate(64);
        sync_wave();
        if (lane < qn - 64) q[lane] = q[64 + lane];
        sync_wave();
        qn -= 64;
      }
    }
  }
  sync_wave();
  evaluate(qn);
  wave_acc(etor, &b_acc[E_TOR]);
  wave_acc(econj, &b_acc[E_CONJ]);
  wave_acc(ntor, &b_acc[NTERMS + 1]);
}

// hydrogen bonds: one wavefront per H atom and donor bond, one acceptor of
// the cluster's list per lane (those within r_hb); acceptor forces with LDS
// atomic adds, the donor entry's adjoints and the force on H summed over the
// wavefront
template <int BSZ>
__device__ __noinline__ void st_hbonds(int n) {
  const BatchArgs A = uni_copy(b_args);
  n = uni(n);
  Lists L;
  Work W;
  views(A, L, W);
  const DevParams* __restrict__ P = A.P;
  const double rh2 = P->rh2, hb_bo_cut = P->hb_bo_cut;
  constexpr int NW = BSZ / 64;
  const int lane = threadIdx.x & 63;
  const int nacc = b_nacc;
  double ehb = 0.0, nhb = 0.0;
  for (int h = threadIdx.x >> 6; h < n; h += NW) {
    const int th = b_ty[h];
    if (P->atom[th].hbond != 1) continue;
    const double4 xh = b_x[h];
    double3 fh = make_double3(0.0, 0.0, 0.0);
    for (int u = b_off[h]; u < b_off[h + 1]; ++u) {
      const int X = L.bond_j[u];
      const int tx = b_ty[X];
      const double bo = W.bo[u].x;
      if (P->atom[tx].hbond != 2 || !(bo >= hb_bo_cut)) continue;
      const double4 rx = W.bd[u];
      double gbo = 0.0;
      double3 gx = make_double3(0.0, 0.0, 0.0);
      for (int k = lane; k < nacc; k += 64) {
        const int Z = b_alist[k];
        if (Z == X) continue;
        const double4 xz = b_x[Z];
        const double dx = xz.x - xh.x, dy = xz.y - xh.y, dz = xz.z - xh.z;
        if (!(r2_of(dx, dy, dz) <= rh2)) continue;
        const HbTerm o = hb_term(b_hb[(tx * NT + th) * NT + b_ty[Z]], bo, rx, dx, dy, dz);
        ehb += o.E;
        gbo += o.dE_dbo;
        gx = add3(gx, o.g_rx);
        fh = add3(fh, o.g_rz);
        atomic_add3(&b_f[Z], -o.g_rz.x, -o.g_rz.y, -o.g_rz.z);
        nhb += 1.0;
      }
      for (int off = 32; off > 0; off >>= 1) {
        gbo += __shfl_down(gbo, off, 64);
        gx.x += __shfl_down(gx.x, off, 64);
        gx.y += __shfl_down(gx.y, off, 64);
        gx.z += __shfl_down(gx.z, off, 64);
      }
      if (lane == 0) {
        atomic_add3(&W.gvec[u], gx);
        atomicAdd(&W.gbo[u].x, gbo);
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      fh.x += __shfl_down(fh.x, off, 64);
      fh.y += __shfl_down(fh.y, off, 64);
      fh.z += __shfl_down(fh.z, off, 64);
    }
    if (lane == 0) atomic_add3(&b_f[h], fh);
  }
  wave_acc(ehb, &b_acc[E_HB]);
  wave_acc(nhb, &b_acc[NTERMS + 2]);
}

template <int BSZ>
__device__ __noinline__ void st_back_s(int n) {
  const BatchArgs A = uni_copy(b_args);
  n = uni(n);
  Lists L;
  Work W;
  views(A, L, W);
  for (int i = threadIdx.x; i < n; i += BSZ) back_s_atom(L, W, i);
}

template <int BSZ>
__device__ __noinline__ void st_back_corr(int n) {
  const BatchArgs A = uni_copy(b_args);
  n = uni(n);
  Lists L;
  Work W;
  views(A, L, W);
  const int ne = b_off[n];
  for (int e = threadIdx.x; e < ne; e += BSZ) back_corr_entry(A.P, L, W, L.bond_i[e], e);
}

template <int BSZ>
__device__ __noinline__ void st_back_dp(int n) {
  const BatchArgs A = uni_copy(b_args);
  n = uni(n);
  Lists L;
  Work W;
  views(A, L, W);
  for (int i = threadIdx.x; i < n; i += BSZ) back_dp_atom(L, W, i);
}

// forces, energies and counts of the cluster
template <int BSZ>
__device__ __noinline__ void st_out(int c, int64_t a0, int n) {
  const BatchArgs A = uni_copy(b_args);
  c = uni(c);
  a0 = uni64(a0);
  n = uni(n);
  Lists L;
  Work W;
  views(A, L, W);
  for (int i = threadIdx.x; i < n; i += BSZ) {
    const double3 f = force_atom(L, W, i);
    A.forces[3 * (a0 + i)] = f.x;
    A.forces[3 * (a0 + i) + 1] = f.y;
    A.forces[3 * (a0 + i) + 2] = f.z;
  }
}

template <int BSZ>
// 2 waves per SIMD: the largest stages (torsions, angles) fit in 256 VGPRs without spills
__global__ __launch_bounds__(BSZ) __attribute__((amdgpu_waves_per_eu(2))) void k_batch(BatchArgs A) {
  const int tid = threadIdx.x;
  if (tid == 0) b_args = A;
  for (int k = tid; k < NT * NT; k += BSZ) {
    b_nb[k] = nb_params(A.P->pair[k]);
    b_reach2[k] = fmin(A.P->pair[k].reach2, A.P->r_bond * A.P->r_bond);
  }
  for (int k = tid; k < NT * NT * NT; k += BSZ) b_hb[k] = A.P->hb[k];
  int pos_in_order = A.dynamic ? 0 : A.wg_first[blockIdx.x];
  const int pos_end = A.dynamic ? 0 : A.wg_first[blockIdx.x + 1];
  for (;;) {
    if (tid == 0) {
      int idx;
      if (A.dynamic) idx = atomicAdd(A.queue, 1);
      else idx = pos_in_order < pos_end ? pos_in_order : A.ncl;
      b_next = idx < A.ncl ? (A.order ? A.order[idx] : idx) : -1;
    }
    ++pos_in_order;
    __syncthreads();
    const int c = b_next;
    if (c < 0) break;
    const int64_t a0 = A.off[c];
    const int64_t len = A.off[c + 1] - a0;
    if (len < 0 || len > A.nmax || a0 < 0 || a0 + len > A.off[A.ncl]) {
      st_fail<BSZ>(c, a0, 0, ST_SIZE, 0);   // no atom range to write: energies and status only
      __syncthreads();
      continue;
    }
    const int n = (int)len;
    if (__syncthreads_or(st_load<BSZ>(a0, n))) {
      st_fail<BSZ>(c, a0, n, ST_TYPE, 0);
      __syncthreads();
      continue;
    }
    st_acceptors<BSZ>(n);
    // staging rows of BSTAGE entries per atom need BSTAGE n of the 8 ecap
    // words of the entries' derivative storage
    const bool staged = BSTAGE * n <= 8 * A.ecap;
    bool over = !staged;
    if (staged) {
      st_pairs<BSZ>(n);
      __syncthreads();
      for (int i = tid; i < n; i += BSZ) over = over || b_off[i + 1] > BSTAGE;
      over = __syncthreads_or(over);
    }
    if (over) {   // no staging, or a row overflowed: both sweeps over all pairs
      st_count<BSZ>(n, staged ? 0 : 1);
      __syncthreads();
    }
    wave_scan_inplace(b_off, n);
    __syncthreads();
    const int nent = b_off[n];
    if (nent > A.ecap) {
      st_fail<BSZ>(c, a0, n, ST_CAPACITY, nent);
      __syncthreads();
      continue;
    }
    if (over) st_fill<BSZ>(n);
    else st_rows<BSZ>(n);
    __syncthreads();
    st_bo_prime<BSZ>(n);
    __syncthreads();
    st_delta_prime<BSZ>(n);
    __syncthreads();
    st_bo_corr<BSZ>(n);
    __syncthreads();
    st_atom_state<BSZ>(n);
    __syncthreads();
    st_atom_energy<BSZ>(n);
    st_nonbonded<BSZ>(n);
    __syncthreads();
    st_angle_count<BSZ>(n);
    __syncthreads();
    wave_scan_inplace(b_aoff, n);
    __syncthreads();
    if ((int64_t)b_aoff[n] * ANG_STAGE <= A.ecap) {   // staged in the correction adjoints' storage
      st_angle_eval<BSZ>(n);
      __syncthreads();
      st_angle_gather<BSZ>(n);
    } else {
      st_angles<BSZ>(n);
    }
    __syncthreads();
    st_torsions<BSZ>(n);
    st_hbonds<BSZ>(n);
    __syncthreads();
    st_back_s<BSZ>(n);
    __syncthreads();
    st_back_corr<BSZ>(n);
    __syncthreads();
    st_back_dp<BSZ>(n);
    __syncthreads();
    st_out<BSZ>(c, a0, n);
    __syncthreads();
    if (tid < NTERMS) A.energies[(int64_t)c * NTERMS + tid] = b_acc[tid];
    else if (A.counts && tid < NTERMS + 4) A.counts[(int64_t)c * NCOUNT + (tid - NTERMS)] = (long long)b_acc[tid];
    else if (A.counts && tid == NTERMS + 4) A.counts[(int64_t)c * NCOUNT + 4] = nent / 2;
    if (tid == 0 && A.status) A.status[c] = 0;
    __syncthreads();
  }
}

}  // namespace rx

// ---------------------------------------------------------------------------
// Scratch of reaxff_compute_forces_batched, the batched evaluation that
// allocates nothing: one fixed array per device (every device the library
// runs on holds its own copy until the process ends).  Bytes [0, 256) hold the
// work queue and the internal status words; persistent workgroup slices
// follow.  In host code `scratch` names a host-side stand-in, never a device
// address: the host takes the array's address on each device once, with
// hipGetSymbolAddress, and only ever passes that address to kernels.
// ---------------------------------------------------------------------------
static __device__ __align__(256) char scratch[REAXFF_BATCHED_SCRATCH_BYTES];

namespace rx {
namespace {
constexpr int MAXDEV = 64;
constexpr int64_t SCRATCH_HEAD = 256;
std::mutex g_scratch_mu;
char* g_scratch_dev[MAXDEV] = {};   // device address of `scratch`, per device
int g_scratch_cus[MAXDEV] = {};     // compute units of that device
}  // namespace

// Look up the address of `scratch` on `device`, which must be current; once per
// device (reaxff_create calls this).  Returns a HIP error code.
int batched_scratch_init(int device) {
  if (device < 0 || device >= MAXDEV) return (int)hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_dev[device]) return (int)hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || ptr == nullptr) return (int)(e != hipSuccess ? e : hipErrorInvalidSymbol);
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus <= 0)
    cus = 256;
  g_scratch_cus[device] = cus;
  g_scratch_dev[device] = static_cast<char*>(ptr);
  return (int)hipSuccess;
}
}  // namespace rx

// ---------------------------------------------------------------------------
// host side: plan, schedule, graph, autotuner
// ---------------------------------------------------------------------------
struct reaxff_batch {
  reaxff_ctx* ctx = nullptr;
  int32_t ncl = 0;
  std::vector<int64_t> off;
  int nmax = 0;
  int cus = 0;
  uint64_t sig = 0;
  reaxff_batch_config cfg{256, REAXFF_SCHED_LPT, 4};
  // device
  int64_t* d_off = nullptr;
  int32_t* d_order = nullptr;
  int32_t* d_wg_first = nullptr;
  int32_t* d_queue = nullptr;
  int32_t* d_err = nullptr;
  int32_t* d_status = nullptr;
  long long* d_counts = nullptr;
  char* d_scratch = nullptr;
  int64_t scratch_bytes = 0;
  int ecap = 0;
  int ecap_need = 0;
  int grid = 0;
  bool sched_valid = false;
  // graph
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const void* key[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  reaxff_batch_config key_cfg{0, 0, 0};
  hipStream_t last_stream = nullptr;
};

namespace {

int bfail(reaxff_batch* b, int code, const std::string& msg) {
  if (b && b->ctx) b->ctx->err = msg;
  return code;
}

#define BHIP(b, expr)                                                                \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess)                                                            \
      return bfail(b, REAXFF_ERR_HIP, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

bool valid_cfg(const reaxff_batch_config& c) {
  return (c.block == 64 || c.block == 128 || c.block == 256 || c.block == 512) &&
         (c.schedule >= REAXFF_SCHED_STATIC && c.schedule <= REAXFF_SCHED_DYNAMIC) &&
         c.wg_per_cu >= 1 && c.wg_per_cu <= 16;
}

// order-independent signature of the multiset of cluster sizes
uint64_t size_signature(const std::vector<int64_t>& off) {
  std::vector<int64_t> s(off.size() - 1);
  for (size_t c = 0; c + 1 < off.size(); ++c) s[c] = off[c + 1] - off[c];
  std::sort(s.begin(), s.end());
  uint64_t h = 1469598103934665603ull;
  for (int64_t v : s) {
    h ^= (uint64_t)v + 0x9e3779b97f4a7c15ull;
    h *= 1099511628211ull;
  }
  return h ^ (uint64_t)s.size();
}

void drop_graph(reaxff_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

// per-workgroup cluster lists for the configuration's schedule
int make_schedule(reaxff_batch* b) {
  const int C = b->ncl;
  const int G = std::max(1, std::min(b->cfg.wg_per_cu * b->cus, std::max(C, 1)));
  std::vector<int64_t> cost(C);
  for (int c = 0; c < C; ++c) {
    const int64_t n = b->off[c + 1] - b->off[c];
    cost[c] = n * n + 64;
  }
  std::vector<int32_t> order;
  std::vector<int32_t> first(G + 1, 0);
  if (b->cfg.schedule == REAXFF_SCHED_DYNAMIC) {
    order.resize(C);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return cost[a] > cost[c]; });
  } else {
    std::vector<std::vector<int32_t>> per(G);
    if (b->cfg.schedule == REAXFF_SCHED_STATIC) {
      for (int c = 0; c < C; ++c) per[c % G].push_back(c);
    } else {
      std::vector<int32_t> idx(C);
      std::iota(idx.begin(), idx.end(), 0);
      std::stable_sort(idx.begin(), idx.end(), [&](int a, int c) { return cost[a] > cost[c]; });
      using Load = std::pair<int64_t, int>;
      std::priority_queue<Load, std::vector<Load>, std::greater<Load>> heap;
      for (int w = 0; w < G; ++w) heap.push({0, w});
      for (int c : idx) {
        Load l = heap.top();
        heap.pop();
        per[l.second].push_back(c);
        l.first += cost[c];
        heap.push(l);
      }
    }
    for (int w = 0; w < G; ++w) {
      first[w] = (int32_t)order.size();
      order.insert(order.end(), per[w].begin(), per[w].end());
    }
    first[G] = (int32_t)order.size();
  }
  b->grid = G;
  if (b->d_order) (void)hipFree(b->d_order);
  if (b->d_wg_first) (void)hipFree(b->d_wg_first);
  b->d_order = nullptr;
  b->d_wg_first = nullptr;
  BHIP(b, hipMalloc(&b->d_order, sizeof(int32_t) * std::max<size_t>(order.size(), 1)));
  BHIP(b, hipMalloc(&b->d_wg_first, sizeof(int32_t) * first.size()));
  if (!order.empty())
    BHIP(b, hipMemcpy(b->d_order, order.data(), sizeof(int32_t) * order.size(), hipMemcpyHostToDevice));
  BHIP(b, hipMemcpy(b->d_wg_first, first.data(), sizeof(int32_t) * first.size(), hipMemcpyHostToDevice));
  // scratch: one slice per workgroup
  const BatchLayout lay = make_layout(std::max(b->nmax, 1), b->ecap);
  const int64_t need = lay.stride * (int64_t)G;
  if (need > b->scratch_bytes) {
    if (b->d_scratch) (void)hipFree(b->d_scratch);
    b->d_scratch = nullptr;
    b->scratch_bytes = 0;
    BHIP(b, hipMalloc(&b->d_scratch, need));
    b->scratch_bytes = need;
  }
  b->sched_valid = true;
  drop_graph(b);
  return 0;
}

template <int BSZ>
void launch_batch(const BatchArgs& a, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_batch<BSZ>, dim3(grid), dim3(BSZ), 0, st, a);
}

int capture(reaxff_batch* b, const double* pos, const int32_t* type, const double* q, double* forces,
            double* energies) {
  drop_graph(b);
  reaxff_ctx* c = b->ctx;
  BatchArgs a{};
  a.P = c->dp;
  a.ncl = b->ncl;
  a.dynamic = b->cfg.schedule == REAXFF_SCHED_DYNAMIC;
  a.off = b->d_off;
  a.order = b->d_order;
  a.wg_first = b->d_wg_first;
  a.queue = b->d_queue;
  a.pos = pos;
  a.type = type;
  a.q = q;
  a.forces = forces;
  a.energies = energies;
  a.counts = b->d_counts;
  a.status = b->d_status;
  a.err = b->d_err;
  a.scratch = b->d_scratch;
  a.lay = make_layout(std::max(b->nmax, 1), b->ecap);
  a.ecap = b->ecap;
  a.nmax = std::max(b->nmax, 1);
  BHIP(b, hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
  hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, b->cap_stream, b->d_queue, b->d_err);
  if (b->ncl > 0) {
    switch (b->cfg.block) {
      case 64: launch_batch<64>(a, b->grid, b->cap_stream); break;
      case 128: launch_batch<128>(a, b->grid, b->cap_stream); break;
      case 256: launch_batch<256>(a, b->grid, b->cap_stream); break;
      default: launch_batch<512>(a, b->grid, b->cap_stream); break;
    }
  }
  const hipError_t le = hipGetLastError();
  hipGraph_t gph = nullptr;
  const hipError_t ee = hipStreamEndCapture(b->cap_stream, &gph);
  if (le != hipSuccess) {
    if (gph) (void)hipGraphDestroy(gph);
    return bfail(b, REAXFF_ERR_HIP, std::string("batch launch: ") + hipGetErrorString(le));
  }
  if (ee != hipSuccess) return bfail(b, REAXFF_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ee));
  b->graph = gph;
  BHIP(b, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  b->key[0] = pos;
  b->key[1] = type;
  b->key[2] = q;
  b->key[3] = forces;
  b->key[4] = energies;
  b->key_cfg = b->cfg;
  return 0;
}

}  // namespace

extern "C" {

int reaxff_batch_create(reaxff_ctx* ctx, int32_t nclusters, const int64_t* offsets,
                        const reaxff_batch_config* cfg, reaxff_batch** out) {
  if (!ctx || !out || nclusters < 0 || (!offsets && nclusters > 0)) {
    if (ctx) ctx->err = "reaxff_batch_create: null argument or negative cluster count";
    return REAXFF_ERR_ARG;
  }
  *out = nullptr;
  std::vector<int64_t> off(offsets, offsets + nclusters + 1);
  if (nclusters == 0) off.assign(1, 0);
  if (off[0] != 0) {
    ctx->err = "reaxff_batch_create: offsets[0] must be 0";
    return REAXFF_ERR_ARG;
  }
  int nmax = 0;
  for (int c = 0; c < nclusters; ++c) {
    const int64_t n = off[c + 1] - off[c];
    if (n < 0 || n > REAXFF_BATCH_MAX_ATOMS) {
      ctx->err = "reaxff_batch_create: cluster " + std::to_string(c) + " has " + std::to_string(n) +
                 " atoms (allowed 0.." + std::to_string(REAXFF_BATCH_MAX_ATOMS) + ")";
      return REAXFF_ERR_ARG;
    }
    nmax = std::max<int>(nmax, (int)n);
  }
  if (cfg && !valid_cfg(*cfg)) {
    ctx->err = "reaxff_batch_create: invalid configuration";
    return REAXFF_ERR_ARG;
  }
  if (hipSetDevice(ctx->device) != hipSuccess) {
    ctx->err = "hipSetDevice failed";
    return REAXFF_ERR_HIP;
  }
  reaxff_batch* b = new reaxff_batch();
  b->ctx = ctx;
  b->ncl = nclusters;
  b->off = off;
  b->nmax = nmax;
  b->sig = size_signature(off);
  // directed bond entries per atom: dense molecular matter stays far below 8
  // on average; a cluster beyond it is reported and the slices grow
  b->ecap = std::max(64, 8 * nmax);
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess || cus <= 0)
    cus = 256;
  b->cus = cus;
  if (cfg) {
    b->cfg = *cfg;
  } else {
    auto it = ctx->tuned.find(b->sig);
    if (it != ctx->tuned.end()) b->cfg = it->second;
  }
  auto cleanup = [&](int code) {
    reaxff_batch_destroy(b);
    return code;
  };
  if (hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess)
    return cleanup(bfail(b, REAXFF_ERR_HIP, "hipStreamCreate failed"));
  const size_t C = (size_t)std::max(nclusters, 1);
  if (hipMalloc(&b->d_off, sizeof(int64_t) * off.size()) != hipSuccess ||
      hipMalloc(&b->d_queue, sizeof(int32_t)) != hipSuccess ||
      hipMalloc(&b->d_err, sizeof(int32_t) * 4) != hipSuccess ||
      hipMalloc(&b->d_status, sizeof(int32_t) * C) != hipSuccess ||
      hipMalloc(&b->d_counts, sizeof(long long) * C * rx::NCOUNT) != hipSuccess)
    return cleanup(bfail(b, REAXFF_ERR_HIP, "hipMalloc failed (batch plan)"));
  if (hipMemcpy(b->d_off, off.data(), sizeof(int64_t) * off.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(b->d_err, 0, sizeof(int32_t) * 4) != hipSuccess ||
      hipMemset(b->d_status, 0, sizeof(int32_t) * C) != hipSuccess ||
      hipMemset(b->d_counts, 0, sizeof(long long) * C * rx::NCOUNT) != hipSuccess)
    return cleanup(bfail(b, REAXFF_ERR_HIP, "hipMemcpy failed (batch plan)"));
  const int r = make_schedule(b);
  if (r) return cleanup(r);
  *out = b;
  return REAXFF_OK;
}

void reaxff_batch_destroy(reaxff_batch* b) {
  if (!b) return;
  if (b->ctx) (void)hipSetDevice(b->ctx->device);
  if (b->cap_stream) (void)hipStreamSynchronize(b->cap_stream);
  if (b->last_stream) (void)hipStreamSynchronize(b->last_stream);
  drop_graph(b);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  for (void* p : {(void*)b->d_off, (void*)b->d_order, (void*)b->d_wg_first, (void*)b->d_queue, (void*)b->d_err,
                  (void*)b->d_status, (void*)b->d_counts, (void*)b->d_scratch})
    if (p) (void)hipFree(p);
  delete b;
}

int reaxff_batch_set_config(reaxff_batch* b, const reaxff_batch_config* cfg) {
  if (!b || !cfg) return REAXFF_ERR_ARG;
  if (!valid_cfg(*cfg)) return bfail(b, REAXFF_ERR_ARG, "reaxff_batch_set_config: invalid configuration");
  if (b->last_stream) (void)hipStreamSynchronize(b->last_stream);
  b->cfg = *cfg;
  return make_schedule(b);
}

int reaxff_batch_get_config(const reaxff_batch* b, reaxff_batch_config* cfg) {
  if (!b || !cfg) return REAXFF_ERR_ARG;
  *cfg = b->cfg;
  return REAXFF_OK;
}

int reaxff_batch_compute(reaxff_batch* b, const double* pos, const int32_t* type, const double* q,
                         double* forces, double* energies, hipStream_t stream) {
  if (!b) return REAXFF_ERR_ARG;
  const bool any = b->off.back() > 0;
  if (any && (!pos || !type || !q || !forces)) return bfail(b, REAXFF_ERR_ARG, "reaxff_batch_compute: null pointer");
  if (b->ncl > 0 && !energies) return bfail(b, REAXFF_ERR_ARG, "reaxff_batch_compute: null energies");
  BHIP(b, hipSetDevice(b->ctx->device));
  if (b->ecap_need > b->ecap) {
    if (b->last_stream) (void)hipStreamSynchronize(b->last_stream);
    b->ecap = b->ecap_need + b->ecap_need / 4 + 16;
    b->ecap_need = 0;
    const int r = make_schedule(b);
    if (r) return r;
  }
  const bool same = b->exec && b->key[0] == pos && b->key[1] == type && b->key[2] == q &&
                    b->key[3] == forces && b->key[4] == energies && b->key_cfg.block == b->cfg.block &&
                    b->key_cfg.schedule == b->cfg.schedule && b->key_cfg.wg_per_cu == b->cfg.wg_per_cu;
  if (!same) {
    const int r = capture(b, pos, type, q, forces, energies);
    if (r) return r;
  }
  rx::Prof& pf = b->ctx->prof;
  pf.begin(rx::KID_BATCH, stream);
  BHIP(b, hipGraphLaunch(b->exec, stream));
  pf.end(stream);
  b->last_stream = stream;
  return REAXFF_OK;
}

int reaxff_batch_status(reaxff_batch* b, int32_t* first_bad) {
  if (!b) return REAXFF_ERR_ARG;
  BHIP(b, hipSetDevice(b->ctx->device));
  int32_t e[4] = {0, 0, INT_MAX, 0};
  BHIP(b, hipStreamSynchronize(b->last_stream));
  BHIP(b, hipMemcpy(e, b->d_err, sizeof(e), hipMemcpyDeviceToHost));
  if (first_bad) *first_bad = e[0] ? e[2] : -1;
  if (e[0] & rx::ST_TYPE)
    return bfail(b, REAXFF_ERR_ARG, "batch: atom type outside 0..3 in cluster " + std::to_string(e[2]));
  if (e[0] & rx::ST_CAPACITY) {
    b->ecap_need = std::max(b->ecap_need, (int)e[1]);
    return bfail(b, REAXFF_ERR_CAPACITY,
                 "batch: " + std::to_string(e[1]) + " bond entries in one cluster exceed the scratch slice (" +
                     std::to_string(b->ecap) + "); the next compute grows it");
  }
  return REAXFF_OK;
}

int reaxff_batch_counts(reaxff_batch* b, int64_t* counts) {
  if (!b || (!counts && b->ncl > 0)) return REAXFF_ERR_ARG;
  BHIP(b, hipSetDevice(b->ctx->device));
  BHIP(b, hipStreamSynchronize(b->last_stream));
  if (b->ncl > 0)
    BHIP(b, hipMemcpy(counts, b->d_counts, sizeof(long long) * (size_t)b->ncl * rx::NCOUNT,
                      hipMemcpyDeviceToHost));
  return REAXFF_OK;
}

int reaxff_batch_tune(reaxff_batch* b, const double* pos, const int32_t* type, const double* q,
                      double* forces, double* energies, hipStream_t stream, int32_t reps,
                      int32_t max_trials, reaxff_batch_config* trials, double* trial_ms,
                      int32_t* ntrials) {
  if (!b) return REAXFF_ERR_ARG;
  if (reps < 1) reps = 1;
  static const int blocks[4] = {64, 128, 256, 512};
  static const int scheds[3] = {REAXFF_SCHED_STATIC, REAXFF_SCHED_LPT, REAXFF_SCHED_DYNAMIC};
  static const int wgs[4] = {1, 2, 4, 8};
  std::vector<reaxff_batch_config> all;
  for (int bl : blocks)
    for (int s : scheds)
      for (int w : wgs) all.push_back(reaxff_batch_config{bl, s, w});
  if (max_trials > 0 && (size_t)max_trials < all.size()) all.resize(max_trials);
  hipEvent_t e0, e1;
  BHIP(b, hipSetDevice(b->ctx->device));
  BHIP(b, hipEventCreate(&e0));
  BHIP(b, hipEventCreate(&e1));
  double best = 1e300;
  reaxff_batch_config bestc = b->cfg;
  int k = 0;
  int rc = REAXFF_OK;
  for (const auto& cf : all) {
    if ((rc = reaxff_batch_set_config(b, &cf))) break;
    if ((rc = reaxff_batch_compute(b, pos, type, q, forces, energies, stream))) break;   // untimed
    (void)hipEventRecord(e0, stream);
    for (int r = 0; r < reps && !rc; ++r) rc = reaxff_batch_compute(b, pos, type, q, forces, energies, stream);
    (void)hipEventRecord(e1, stream);
    if (rc) break;
    if (hipEventSynchronize(e1) != hipSuccess) {
      rc = bfail(b, REAXFF_ERR_HIP, "batch tune: event synchronise failed");
      break;
    }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    const double per = (double)ms / reps;
    if (trials) trials[k] = cf;
    if (trial_ms) trial_ms[k] = per;
    ++k;
    if (per < best) {
      best = per;
      bestc = cf;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (ntrials) *ntrials = k;
  if (rc) return rc;
  b->ctx->tuned[b->sig] = bestc;
  rc = reaxff_batch_set_config(b, &bestc);
  if (rc) return rc;
  return reaxff_batch_compute(b, pos, type, q, forces, energies, stream);
}

int reaxff_compute_forces_batched(reaxff_ctx* ctx, int32_t nsys, const int64_t* sys_off, int32_t max_atoms,
                                  const double* pos, const int32_t* type, const double* q, double* forces,
                                  double* energies, int32_t* status, hipStream_t stream) {
  using namespace rx;
  if (!ctx) return REAXFF_ERR_ARG;
  if (nsys < 0) {
    ctx->err = "reaxff_compute_forces_batched: nsys < 0";
    return REAXFF_ERR_ARG;
  }
  if (nsys > 0 && (!sys_off || !pos || !type || !q || !forces || !energies)) {
    ctx->err = "reaxff_compute_forces_batched: null pointer";
    return REAXFF_ERR_ARG;
  }
  if (nsys > 0 && (max_atoms < 1 || max_atoms > REAXFF_BATCH_MAX_ATOMS)) {
    ctx->err = "reaxff_compute_forces_batched: max_atoms " + std::to_string(max_atoms) + " outside 1.." +
               std::to_string(REAXFF_BATCH_MAX_ATOMS);
    return REAXFF_ERR_ARG;
  }
  const int dev = ctx->device;
  char* base = (dev >= 0 && dev < MAXDEV) ? g_scratch_dev[dev] : nullptr;
  if (!base) {
    ctx->err = "reaxff_compute_forces_batched: scratch address of this device not set up";
    return REAXFF_ERR_STATE;
  }
  const hipError_t se = hipSetDevice(dev);
  if (se != hipSuccess) {
    ctx->err = std::string("hipSetDevice: ") + hipGetErrorString(se);
    return REAXFF_ERR_HIP;
  }
  const int nmax = std::max(max_atoms, 1);
  const int ecap = REAXFF_BATCHED_ENTRIES_PER_ATOM * nmax;
  const BatchLayout lay = make_layout(nmax, ecap);
  const int64_t slices = (REAXFF_BATCHED_SCRATCH_BYTES - SCRATCH_HEAD) / lay.stride;
  if (slices < 1) {
    ctx->err = "reaxff_compute_forces_batched: one workgroup slice exceeds the scratch array";
    return REAXFF_ERR_CAPACITY;
  }
  constexpr int BSZ = 256, WG_PER_CU = 4;
  const int grid = (int)std::min<int64_t>(std::min<int64_t>(slices, (int64_t)g_scratch_cus[dev] * WG_PER_CU),
                                          std::max(nsys, 1));
  int32_t* queue = reinterpret_cast<int32_t*>(base);
  int32_t* err = status ? status : reinterpret_cast<int32_t*>(base + 64);
  // the array keeps the previous call's contents: the queue and status words
  // start again from zero (a kernel, not a memset, so that the call can be
  // captured into a graph)
  hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, stream, queue, err);
  if (nsys > 0) {
    BatchArgs a{};
    a.P = ctx->dp;
    a.ncl = nsys;
    a.dynamic = 1;
    a.off = sys_off;
    a.order = nullptr;
    a.wg_first = nullptr;
    a.queue = queue;
    a.pos = pos;
    a.type = type;
    a.q = q;
    a.forces = forces;
    a.energies = energies;
    a.counts = nullptr;
    a.status = nullptr;
    a.err = err;
    a.scratch = base + SCRATCH_HEAD;
    a.lay = lay;
    a.ecap = ecap;
    a.nmax = nmax;
    hipLaunchKernelGGL(k_batch<BSZ>, dim3(grid), dim3(BSZ), 0, stream, a);
  }
  const hipError_t le = hipGetLastError();
  if (le != hipSuccess) {
    ctx->err = std::string("reaxff_compute_forces_batched launch: ") + hipGetErrorString(le);
    return REAXFF_ERR_HIP;
  }
  return REAXFF_OK;
}

}  // extern "C"
