// Charge equilibration (Section 3.3, QEq): the charges that minimise
//   E(q) = sum_i (chi_i q_i + J_i q_i^2 / 2) + sum_{i<j} H_ij q_i q_j,
//   H_ij = Tap(r_ij) C_ele / (r_ij^3 + gamma_ij^-3)^(1/3)  (r_ij <= r_nonb),
// under sum_i q_i = 0, from the two systems H s = -chi and H t = -1 with the
// common matrix H (diagonal J): q = s - (sum s / sum t) t.
//
// As in the paper: the matrix is computed once per call from the neighbours
// within r_nonb and stored; the two systems are solved together by
// conjugate gradients with a diagonal preconditioner, one product of H with
// both search directions per iteration; the start is extrapolated from
// earlier solutions.  On this GPU:
//   * H rows: one wavefront per atom walks its cell stencil (contiguous
//     ranges of cell-sorted atoms, coalesced) and appends the neighbours
//     within r_nonb, with H_ij, to a fixed-width row (ballot + popcount
//     numbering, stencil order, so the row order is deterministic).  Each row
//     holds both halves of the symmetric matrix: a product then gathers and
//     never scatters, so no partial result vectors and no atomics are needed
//     (the paper keeps unique entries and pays for thread-private result
//     arrays, Section 4's QEq discussion).
//   * the product is HBM-bound: one wavefront per row reads the row's
//     (index, value) entries once and gathers the two search directions as
//     one 16-byte record per neighbour (L2-resident: neighbours are near in
//     the cell-sorted order).
//   * the scalar recurrences stay on the device: each kernel folds the
//     64 partial-sum slots of the previous stage itself; the host reads only
//     the residual norms, once per iteration, to stop.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "internal.h"
#include "terms.h"

namespace rx {

constexpr int QB = 256, QWAVES = QB / 64;
// fields of one partial-sum slot: p.Ap (s, t), r.z (s, t), r.r (s, t), b.b (s, t)
constexpr int QF = 8;

struct QeqPar {
  double chi[NT], J[NT], Jinv[NT];
};

__device__ __forceinline__ unsigned long long lanes_below() {
  const int lane = threadIdx.x & 63;
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// sum of a slot field over the ESLOT slots (every thread of the block may call)
__device__ __forceinline__ double fold(const double* __restrict__ set, int f) {
  double s = 0.0;
  for (int k = 0; k < ESLOT; ++k) s += set[k * QF + f];
  return s;
}

// add per-block sums of NF fields to this block's slot
template <int NF>
__device__ __forceinline__ void slot_add(double* __restrict__ set, const int* fields, const double* v) {
  __shared__ double red[NF][QWAVES];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double x[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    x[f] = v[f];
    for (int off = 32; off > 0; off >>= 1) x[f] += __shfl_down(x[f], off, 64);
  }
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int f = 0; f < NF; ++f) red[f][w] = x[f];
  __syncthreads();
  if (threadIdx.x < NF) {
    double s = 0.0;
    for (int k = 0; k < QWAVES; ++k) s += red[threadIdx.x][k];
    if (s != 0.0) atomicAdd(&set[(blockIdx.x & (ESLOT - 1)) * QF + fields[threadIdx.x]], s);
  }
}

// H rows, one wavefront per cell: every j != i of the cell's stencil with
// r_ij^2 <= r_nonb^2 (minimum image, the far list's predicate; the chunk's
// image shift when it is the minimum image of every listed pair), for each
// atom i of the cell.  As in the list sweep, the stencil's chunks are laid
// end to end and walked in batches of 64 candidates, one per lane, each
// batch tested against the cell's atoms in turn; accepted neighbours are
// numbered with the ballot and their indices stored in stencil order.
// Their (row, place, type pair, r^2) are queued in LDS and the matrix
// elements computed 64 at a time, so the taper and the shielded Coulomb run
// on full wavefronts.
constexpr int QRMAXQ = 64;   // chunks of a stencil: 2 (2 reach + 1)^2 <= 50

struct QRowQ {
  int32_t i, k, p, pad;
  double r2;
};

__global__ __launch_bounds__(QB) void k_qeq_rows(const DevParams* __restrict__ P, Grid g, Lists L, int ncell,
                                                 int32_t* __restrict__ hj, double* __restrict__ hv,
                                                 int32_t* __restrict__ hcnt, int32_t w,
                                                 int32_t* __restrict__ need) {
  __shared__ QRowQ rq[QWAVES][128];
  __shared__ int q_s0[QWAVES][QRMAXQ], q_base[QWAVES][QRMAXQ + 1];
  __shared__ double q_sh[QWAVES][QRMAXQ][3];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int c = (int)(xcd_block() * QWAVES + wv);
  if (c >= ncell) return;   // uniform over the wavefront
  const int a0 = L.cell_start[c], m = L.cell_start[c + 1] - a0;
  if (m == 0) return;
  QRowQ* __restrict__ q = rq[wv];
  int* __restrict__ qs0 = q_s0[wv];
  int* __restrict__ qb = q_base[wv];
  const unsigned long long below = lanes_below();
  auto sync_wave = [] {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };
  const bool minimg = g.periodic && !g.shift_ok;
  const int nq = stencil_chunks(g);
  {
    int len = 0;
    if (lane < nq) {
      int s0, s1;
      double sx, sy, sz;
      stencil_chunk(g, L.cell_start, c, lane, s0, s1, sx, sy, sz);
      qs0[lane] = s0;
      len = s1 - s0;
      q_sh[wv][lane][0] = sx;
      q_sh[wv][lane][1] = sy;
      q_sh[wv][lane][2] = sz;
    }
    const int v = wave_incl_scan(len);
    if (lane < nq) qb[lane + 1] = v;
    if (lane == 0) qb[0] = 0;
  }
  sync_wave();
  const int nst = __builtin_amdgcn_readfirstlane(qb[nq]);
  const double rn2 = P->rn2, iR = P->inv_r_nonb;
  auto evaluate = [&](int mq) {   // the first mq queued elements, one per lane
    if (lane < mq) {
      const QRowQ e = q[lane];
      if (e.k < w) {
        const double r = sqrt(e.r2);
        const double u = r * iR;
        const double u4 = (u * u) * (u * u);
        const double tap = fma(u4, fma(u, fma(u, fma(u, 20.0, -70.0), 84.0), -35.0), 1.0);
        hv[(int64_t)e.i * w + e.k] = tap * C_ELE * rcbrt_f(fma(e.r2, r, P->pair[e.p].g3));
      }
    }
  };
  int qn = 0;   // queued elements (uniform)
  for (int ig = 0; ig < m; ig += 64) {   // the cell's atoms, 64 at a time, one per lane
    const int mi = m - ig < 64 ? m - ig : 64;
    int tmine = 0;
    if (lane < mi) tmine = (int)L.xs[a0 + ig + lane].w;
    int kc = 0;   // lane l: row length of the cell's atom ig + l
    int cq = 0;   // this lane's chunk
    for (int b0 = 0; b0 < nst; b0 += 64) {
      const int slot = b0 + lane;
      const bool valid = slot < nst;
      int sj = 0;
      double sx = 0.0, sy = 0.0, sz = 0.0;
      if (valid) {
        while (qb[cq + 1] <= slot) ++cq;
        sj = qs0[cq] + (slot - qb[cq]);
        sx = q_sh[wv][cq][0];
        sy = q_sh[wv][cq][1];
        sz = q_sh[wv][cq][2];
      }
      // lanes past the stencil's end hold NaN, so every distance test fails there
      double4 xj = make_double4(__builtin_nan(""), 0.0, 0.0, 0.0);
      if (valid) xj = L.xs[sj];
      const int tj = (int)xj.w;
      for (int l = 0; l < mi; ++l) {
        const int i = a0 + ig + l;
        const double4 xi = L.xs[i];   // uniform: a scalar load
        double dx = xj.x - xi.x, dy = xj.y - xi.y, dz = xj.z - xi.z;
        if (minimg) {
          dx = min_image(dx, g.L[0], g.invL[0]);
          dy = min_image(dy, g.L[1], g.invL[1]);
          dz = min_image(dz, g.L[2], g.invL[2]);
        } else {
          dx -= sx;
          dy -= sy;
          dz -= sz;
        }
        const double r2 = r2_of(dx, dy, dz);
        const bool ok = r2 <= rn2 && sj != i;
        const int pij = readlane_i(tmine, l) * NT + tj;
        const unsigned long long mk = ballot(ok);
        if (mk) {
          const int k0 = readlane_i(kc, l);
          if (ok) {
            const int pos = __popcll(mk & below);
            const int k = k0 + pos;
            if (k < w) hj[(int64_t)i * w + k] = sj;
            q[qn + pos] = QRowQ{i, k, pij, 0, r2};
          }
          kc = writelane_i(k0 + __popcll(mk), l, kc);
          qn += __popcll(mk);
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
    }
    if (lane < mi) {
      hcnt[a0 + ig + lane] = kc;
      if (kc > w) atomicMax(need, kc);
    }
  }
  sync_wave();
  evaluate(qn);
}

// y = H x for the pair of vectors (s, t), one wavefront per row; with `set`,
// the block's sums of x_i . y_i per system go to the slot fields 0 and 1
__global__ __launch_bounds__(QB) void k_qeq_spmv(Lists L, const int32_t* __restrict__ hj,
                                                 const double* __restrict__ hv,
                                                 const int32_t* __restrict__ hcnt, int32_t w, QeqPar qp,
                                                 const double2* __restrict__ x, double2* __restrict__ y,
                                                 double* __restrict__ set) {
  const int lane = threadIdx.x & 63;
  const int64_t i = xcd_block() * QWAVES + (threadIdx.x >> 6);
  double ds = 0.0, dt = 0.0;
  if (i < L.n) {
    const int cnt = min(hcnt[i], w);
    const int32_t* __restrict__ rj = hj + i * (int64_t)w;
    const double* __restrict__ rv = hv + i * (int64_t)w;
    double as = 0.0, at = 0.0;
    // eight entries per lane at a time: their index and value loads, then
    // their gathers, are in flight together
    for (int k0 = lane; k0 < cnt; k0 += 8 * 64) {
      int jj[8];
      double hh[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int k = k0 + u * 64;
        jj[u] = k < cnt ? rj[k] : (int)i;
        hh[u] = k < cnt ? rv[k] : 0.0;
      }
      double2 xj[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) xj[u] = x[jj[u]];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        as = fma(hh[u], xj[u].x, as);
        at = fma(hh[u], xj[u].y, at);
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      as += __shfl_down(as, off, 64);
      at += __shfl_down(at, off, 64);
    }
    if (lane == 0) {
      const double2 xi = x[i];
      const double Ji = qp.J[L.type_s[i]];
      const double2 yi = make_double2(fma(Ji, xi.x, as), fma(Ji, xi.y, at));
      y[i] = yi;
      ds = xi.x * yi.x;
      dt = xi.y * yi.y;
    }
  }
  if (set) {
    const int f[2] = {0, 1};
    const double v[2] = {ds, dt};
    slot_add<2>(set, f, v);
  }
}

// start: r = b - y (y = H x0, or x0 = 0 when y is null), p = M^-1 r; slot
// fields 2..7 of the start set: r.z, r.r, b.b per system
__global__ __launch_bounds__(QB) void k_qeq_start(Lists L, QeqPar qp, const double2* __restrict__ y,
                                                  double2* __restrict__ x, double2* __restrict__ r,
                                                  double2* __restrict__ p, double* __restrict__ set) {
  const int64_t i = xcd_block() * QB + threadIdx.x;
  double v[6] = {0, 0, 0, 0, 0, 0};
  if (i < L.n) {
    const int t = L.type_s[i];
    const double2 b = make_double2(-qp.chi[t], -1.0);
    double2 ri = b;
    if (y) {
      const double2 yi = y[i];
      ri = make_double2(b.x - yi.x, b.y - yi.y);
    } else {
      x[i] = make_double2(0.0, 0.0);
    }
    const double mi = qp.Jinv[t];
    const double2 zi = make_double2(mi * ri.x, mi * ri.y);
    r[i] = ri;
    p[i] = zi;
    v[0] = ri.x * zi.x;
    v[1] = ri.y * zi.y;
    v[2] = ri.x * ri.x;
    v[3] = ri.y * ri.y;
    v[4] = b.x * b.x;
    v[5] = b.y * b.y;
  }
  const int f[6] = {2, 3, 4, 5, 6, 7};
  slot_add<6>(set, f, v);
}

// step lengths alpha = (r.z)_old / (p.Ap) per system (zero once a system's
// residual or curvature is exactly zero); x += alpha p, r -= alpha Ap; slot
// fields 2..5 of this iteration's set: new r.z and r.r
__global__ __launch_bounds__(QB) void k_qeq_update(Lists L, QeqPar qp, const double* __restrict__ prev,
                                                   double* __restrict__ cur, double2* __restrict__ x,
                                                   double2* __restrict__ r, const double2* __restrict__ p,
                                                   const double2* __restrict__ ap) {
  __shared__ double alpha[2];
  if (threadIdx.x < 2) {
    const double pap = fold(cur, threadIdx.x), rz = fold(prev, 2 + threadIdx.x);
    alpha[threadIdx.x] = (pap > 0.0 && rz > 0.0) ? rz / pap : 0.0;
  }
  __syncthreads();
  const double as = alpha[0], at = alpha[1];
  const int64_t i = xcd_block() * QB + threadIdx.x;
  double v[4] = {0, 0, 0, 0};
  if (i < L.n) {
    const double2 pi = p[i], api = ap[i];
    double2 xi = x[i], ri = r[i];
    xi.x = fma(as, pi.x, xi.x);
    xi.y = fma(at, pi.y, xi.y);
    ri.x = fma(-as, api.x, ri.x);
    ri.y = fma(-at, api.y, ri.y);
    x[i] = xi;
    r[i] = ri;
    const double mi = qp.Jinv[L.type_s[i]];
    v[0] = mi * ri.x * ri.x;
    v[1] = mi * ri.y * ri.y;
    v[2] = ri.x * ri.x;
    v[3] = ri.y * ri.y;
  }
  const int f[4] = {2, 3, 4, 5};
  slot_add<4>(cur, f, v);
}

// p = M^-1 r + beta p, beta = (r.z)_new / (r.z)_old per system
__global__ __launch_bounds__(QB) void k_qeq_direction(Lists L, QeqPar qp, const double* __restrict__ prev,
                                                      const double* __restrict__ cur,
                                                      const double2* __restrict__ r, double2* __restrict__ p) {
  __shared__ double beta[2];
  if (threadIdx.x < 2) {
    const double rzo = fold(prev, 2 + threadIdx.x), rzn = fold(cur, 2 + threadIdx.x);
    beta[threadIdx.x] = rzo > 0.0 ? rzn / rzo : 0.0;
  }
  __syncthreads();
  const int64_t i = xcd_block() * QB + threadIdx.x;
  if (i < L.n) {
    const double mi = qp.Jinv[L.type_s[i]];
    const double2 ri = r[i], pi = p[i];
    p[i] = make_double2(fma(beta[0], pi.x, mi * ri.x), fma(beta[1], pi.y, mi * ri.y));
  }
}

// sums of s and t (slot fields 0, 1 of the final set)
__global__ __launch_bounds__(QB) void k_qeq_sums(Lists L, const double2* __restrict__ x, double* __restrict__ set) {
  const int64_t i = xcd_block() * QB + threadIdx.x;
  double v[2] = {0, 0};
  if (i < L.n) {
    const double2 xi = x[i];
    v[0] = xi.x;
    v[1] = xi.y;
  }
  const int f[2] = {0, 1};
  slot_add<2>(set, f, v);
}

// q = s - (sum s / sum t) t, written in the caller's order with s and t
// (history ring slot `hist`, optional outputs)
__global__ __launch_bounds__(QB) void k_qeq_charges(Lists L, const double2* __restrict__ x,
                                                    const double* __restrict__ set, double* __restrict__ q,
                                                    double2* __restrict__ hist, double* __restrict__ s_out,
                                                    double* __restrict__ t_out) {
  __shared__ double ratio;
  if (threadIdx.x == 0) ratio = fold(set, 0) / fold(set, 1);
  __syncthreads();
  const int64_t i = xcd_block() * QB + threadIdx.x;
  if (i < L.n) {
    const double2 xi = x[i];
    const int o = L.perm[i];
    q[o] = fma(-ratio, xi.y, xi.x);
    hist[o] = xi;
    if (s_out) s_out[o] = xi.x;
    if (t_out) t_out[o] = xi.y;
  }
}

// ---------------------------------------------------------------------------
// Matrix-free product over the half far list.  When the last build left the
// far rows in the half, run-window form (those the nonbonded term walks: each
// pair within r_nonb once, as a slot in the window of the centre's run), H x
// needs no stored matrix: the workgroup of a run stages its upper window
// (positions and both search directions) in LDS, evaluates H_ij of each of
// its pairs once, adds H_ij x_j to the centre (sums over the 8 lanes of a
// unit) and H_ij x_i to the partner (an LDS accumulator), and stores the
// accumulators to the run's partial array; k_qeq_hreduce then sums, for each
// atom, the partial arrays of the runs whose upper window holds it and adds
// J_i x_i and the dot products of the CG step.  H_ij is k_qeq_rows's element
// (the same taper and shielded Coulomb), and each pair is taken once, as in
// the paper's storage of unique entries.  Against the stored rows: no 12-byte
// entries for both halves of the matrix (5.2 GB at 1.04M atoms) and no row
// build, for ~15% more time per product.
// ---------------------------------------------------------------------------
constexpr int QH_BS = 1024, QH_WAVES = QH_BS / 64;
constexpr int QH_MG = 128;   // centre atoms of a run per pass (two per lane of one wavefront)

__global__ __launch_bounds__(QH_BS) void k_qeq_half(const DevParams* __restrict__ P, Grid g, Lists L, int nrun,
                                                    int per_xcd, const double2* __restrict__ x,
                                                    double* __restrict__ part, int32_t* __restrict__ tab) {
  __shared__ double sg3[NT * NT];
  __shared__ double sxx[NB_HALF_CAP], sxy[NB_HALF_CAP], sxz[NB_HALF_CAP], sxs[NB_HALF_CAP], sxt[NB_HALF_CAP];
  __shared__ double fas[NB_HALF_CAP], fat[NB_HALF_CAP];
  __shared__ unsigned char sty[NB_HALF_CAP];
  __shared__ int q_s0[NB_QMAX], q_base[NB_QMAX + 1];
  __shared__ double q_sh[NB_QMAX][3];
  __shared__ int upre[QH_MG + 1];
  __shared__ double ixx[QH_MG], ixy[QH_MG], ixz[QH_MG], ixs[QH_MG], ixt[QH_MG];
  __shared__ int ity[QH_MG], icnt[QH_MG], ilo[QH_MG];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int r = (int)(blockIdx.x & 7) * per_xcd + (int)(blockIdx.x >> 3);
  if (r >= nrun) return;
  int c, nk;
  run_cells(g, r, c, nk);
  const int a0 = L.cell_start[c], m = L.cell_start[c + nk] - a0;
  const int nq = stencil_chunks(g);
  if (m == 0) {   // no pairs: chunk offsets that send the reduce past every slot
    if (tid < nq) tab[(int64_t)r * NB_QMAX + tid] = -0x40000000;
    return;
  }
  if (tid < NT * NT) sg3[tid] = P->pair[tid].g3;
  const bool shifted = g.periodic && g.shift_ok;
  const bool minimg = g.periodic && !g.shift_ok;
  if (tid < nq) {
    int s0, s1;
    double sx, sy, sz;
    window_chunk(g, L.cell_start, c, tid, s0, s1, sx, sy, sz);
    q_s0[tid] = s0;
    q_base[tid + 1] = s1 - s0;
    q_sh[tid][0] = shifted ? sx : 0.0;
    q_sh[tid][1] = shifted ? sy : 0.0;
    q_sh[tid][2] = shifted ? sz : 0.0;
  }
  __syncthreads();
  if (wv == 0) {
    const int v = wave_incl_scan(lane < nq ? q_base[lane + 1] : 0);
    if (lane < nq) q_base[lane + 1] = v;
    if (lane == 0) q_base[0] = 0;
  }
  __syncthreads();
  const int nst = q_base[nq];
  // the run's own chunk: its column is the middle one, and its unwrapped z
  // range comes second when the window wraps below the run
  const int z0 = c % g.nc[2];
  const int col_own = g.reach * g.span[1] + g.reach;
  const bool wrap_first = g.periodic && z0 - g.reach < 0;
  const int q_own = 2 * col_own + (wrap_first ? 1 : 0);
  const int S0 = q_base[q_own] + (a0 - q_s0[q_own]);
  const int nup = nst - S0;                            // <= NB_HALF_CAP (checked by the sweep)
  // for the reduce: atom j of chunk q has staged index tab[q] + j
  if (tid < nq) tab[(int64_t)r * NB_QMAX + tid] = q_base[tid] - S0 - q_s0[tid];
  // staging: wavefront w copies the upper-window parts of chunks w, w + 16,
  // ...; its lanes stride a chunk's atoms, which are contiguous in memory
  for (int q = q_own + wv; q < nq; q += QH_WAVES) {
    const int b = q_base[q], e = q_base[q + 1];
    const int sb = b > S0 ? b : S0, src = q_s0[q] - b;
    const double hx = q_sh[q][0], hy = q_sh[q][1], hz = q_sh[q][2];
    for (int s0 = sb; s0 < e; s0 += 128) {
      double4 v[2];
      double2 xv[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int s = s0 + 64 * u + lane;
        if (s < e) {
          v[u] = L.xs[src + s];
          xv[u] = x[src + s];
        }
      }
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int s = s0 + 64 * u + lane;
        if (s < e) {
          const int t = s - S0;
          sxx[t] = v[u].x - hx;
          sxy[t] = v[u].y - hy;
          sxz[t] = v[u].z - hz;
          sty[t] = (unsigned char)(int)v[u].w;
          sxs[t] = xv[u].x;
          sxt[t] = xv[u].y;
          fas[t] = fat[t] = 0.0;
        }
      }
    }
  }
  const double iR = P->inv_r_nonb, rn2c = P->rn2;
  for (int g0 = 0; g0 < m; g0 += QH_MG) {
    const int mg = m - g0 < QH_MG ? m - g0 : QH_MG;
    if (g0 > 0) __syncthreads();   // the previous pass's units done
    if (wv == 0) {   // the pass's centres, two per lane: 2 lane and 2 lane + 1
      int nu[2] = {0, 0};
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int k = 2 * lane + h;
        if (k < mg) {
          const int i = a0 + g0 + k;
          const int cnt = L.far_cnt[i], lo = L.far_lo[i];
          const double4 xi = L.xs[i];
          const double2 vi = x[i];
          ixx[k] = xi.x;
          ixy[k] = xi.y;
          ixz[k] = xi.z;
          ixs[k] = vi.x;
          ixt[k] = vi.y;
          ity[k] = (int)xi.w;
          icnt[k] = cnt;
          ilo[k] = lo;
          nu[h] = (cnt - lo + 7) >> 3;   // units of 8 entries
        }
      }
      const int v = wave_incl_scan(nu[0] + nu[1]);
      upre[2 * lane + 1] = v - nu[1];
      upre[2 * lane + 2] = v;
      if (lane == 0) upre[0] = 0;
    }
    __syncthreads();   // staging and the pass's centres in place
    // units of 8 row entries, a contiguous share per wavefront, one unit per
    // group of 8 lanes at a time (the centre is uniform over a group); the
    // row entry of the unit after next and the staged data of the next one
    // are loaded during each pair
    const int U = __builtin_amdgcn_readfirstlane(upre[mg]);
    const int wu = __builtin_amdgcn_readfirstlane(wv);
    const int u0 = U * wu / QH_WAVES, u1 = U * (wu + 1) / QH_WAVES;
    if (u0 < u1) {
      const int hh = lane >> 3, sl = lane & 7;
      int a = 0, ua = 0, un = 0, lo = 0, cn = 0;
      const int32_t* __restrict__ rowp = L.far_j;
      auto enter = [&](int na) {
        a = na;
        ua = upre[a];
        un = upre[a + 1];
        lo = ilo[a];
        cn = icnt[a];
        rowp = L.far_j + (int64_t)(a0 + g0 + a) * L.far_w;
      };
      auto fetch = [&](int u, bool& ok) {
        ok = false;
        if (u >= u1) return 0;
        if (un <= u) {
          int na = a + 1;
          while (upre[na + 1] <= u) ++na;
          enter(na);
        }
        const int k = lo + ((u - ua) << 3) + sl;
        ok = k < cn;
        return ok ? rowp[k] : 0;
      };
      auto staged = [&](int raw, bool ok) {
        const int t = raw - S0;
        return ok && (unsigned)t < (unsigned)nup ? t : -1;
      };
      const int uh = u0 + hh;
      enter(last_le(upre, mg, uh < u1 ? uh : u1 - 1));
      bool ok0, ok1;
      const int r0 = fetch(uh, ok0);
      const int acur0 = a;
      int r1 = fetch(uh + 8, ok1);
      int anext = a;
      int tnow = staged(r0, ok0), anow = acur0;
      double jx, jy, jz, js, jt;
      int jty;
      {
        const int t = tnow >= 0 ? tnow : 0;
        jx = sxx[t];
        jy = sxy[t];
        jz = sxz[t];
        js = sxs[t];
        jt = sxt[t];
        jty = sty[t];
      }
      int cur = anow;
      double xix = ixx[cur], xiy = ixy[cur], xiz = ixz[cur], vs = ixs[cur], vt = ixt[cur];
      const double* __restrict__ g3i = sg3 + ity[cur] * NT;
      double ys = 0.0, yt = 0.0;
      auto flush = [&]() {   // over the 8 lanes, into the last
        ys = oct_sum_last(ys);
        yt = oct_sum_last(yt);
        if (sl == 7) {
          const int t = g0 + cur;   // the centre's staged index: slot - S0 = i - a0
          atomicAdd(&fas[t], ys);
          atomicAdd(&fat[t], yt);
        }
        ys = yt = 0.0;
      };
      for (int ub = u0; ub < u1; ub += 8) {
        bool ok2;
        const int r2n = fetch(ub + 16 + hh, ok2);
        const int aafter = a;
        const int tnext = staged(r1, ok1);
        double nx, ny, nz, ns, nt;
        int nty;
        {
          const int t = tnext >= 0 ? tnext : 0;
          nx = sxx[t];
          ny = sxy[t];
          nz = sxz[t];
          ns = sxs[t];
          nt = sxt[t];
          nty = sty[t];
        }
        if (anow != cur) {
          flush();
          cur = anow;
          xix = ixx[cur];
          xiy = ixy[cur];
          xiz = ixz[cur];
          vs = ixs[cur];
          vt = ixt[cur];
          g3i = sg3 + ity[cur] * NT;
        }
        if (tnow >= 0) {
          double dx = jx - xix, dy = jy - xiy, dz = jz - xiz;
          if (minimg) {
            dx = min_image(dx, g.L[0], g.invL[0]);
            dy = min_image(dy, g.L[1], g.invL[1]);
            dz = min_image(dz, g.L[2], g.invL[2]);
          }
          const double rr = dx * dx + dy * dy + dz * dz;
          if (!(L.cut_check && rr > rn2c)) {   // else a skin entry beyond r_nonb
            const double rv = rr * rsq_f(rr);
            const double u = rv * iR;
            const double u4 = (u * u) * (u * u);
            const double tap = fma(u4, fma(u, fma(u, fma(u, 20.0, -70.0), 84.0), -35.0), 1.0);
            const double h = tap * C_ELE * rcbrt_f(fma(rr, rv, g3i[jty]));
            ys = fma(h, js, ys);
            yt = fma(h, jt, yt);
            atomicAdd(&fas[tnow], h * vs);
            atomicAdd(&fat[tnow], h * vt);
          }
        }
        tnow = tnext;
        anow = anext;
        jx = nx;
        jy = ny;
        jz = nz;
        js = ns;
        jt = nt;
        jty = nty;
        r1 = r2n;
        ok1 = ok2;
        anext = aafter;
      }
      flush();
    }
  }
  __syncthreads();
  double* __restrict__ pr = part + (int64_t)r * 2 * NB_HALF_CAP;
  for (int t = tid; t < nup; t += QH_BS) {
    pr[2 * t] = fas[t];
    pr[2 * t + 1] = fat[t];
  }
}

// y = H x from the partial arrays of k_qeq_half: for each atom j, the sum
// over the runs whose upper window holds it (for_upper_windows), plus
// J_j x_j; with `set`, the block's sums of x . y per system go to the slot
// fields 0 and 1.  R: the stencil reach.
template <int R>
__global__ __launch_bounds__(QB) void k_qeq_hreduce(Grid g, Lists L, const int32_t* __restrict__ tab,
                                                    const double* __restrict__ part, QeqPar qp,
                                                    const double2* __restrict__ x, double2* __restrict__ y,
                                                    double* __restrict__ set) {
  const int64_t j = xcd_block() * QB + threadIdx.x;
  double ds = 0.0, dt = 0.0;
  if (j < L.n) {
    double as = 0.0, at = 0.0;
    for_upper_windows<R>(g, L.cell_of[j], tab, (int)j, [&](int64_t r, int t) {
      const double2 pv = *(const double2*)(part + r * 2 * NB_HALF_CAP + 2 * t);
      as += pv.x;
      at += pv.y;
    });
    const double2 xj = x[j];
    const double Jj = qp.J[L.type_s[j]];
    const double2 yj = make_double2(fma(Jj, xj.x, as), fma(Jj, xj.y, at));
    y[j] = yj;
    ds = xj.x * yj.x;
    dt = xj.y * yj.y;
  }
  if (set) {
    const int f[2] = {0, 1};
    const double v[2] = {ds, dt};
    slot_add<2>(set, f, v);
  }
}

// initial guess from the history ring (caller order, newest first):
// x_i = sum_k c_k hist_k[perm i]
__global__ __launch_bounds__(QB) void k_qeq_guess(Lists L, const double2* __restrict__ h0,
                                                  const double2* __restrict__ h1, const double2* __restrict__ h2,
                                                  const double2* __restrict__ h3, double4 c, double2* __restrict__ x) {
  const int64_t i = xcd_block() * QB + threadIdx.x;
  if (i >= L.n) return;
  const int o = L.perm[i];
  double2 v = h0[o];
  v.x *= c.x;
  v.y *= c.x;
  if (h1) {
    const double2 a = h1[o];
    v.x = fma(c.y, a.x, v.x);
    v.y = fma(c.y, a.y, v.y);
  }
  if (h2) {
    const double2 a = h2[o];
    v.x = fma(c.z, a.x, v.x);
    v.y = fma(c.z, a.y, v.y);
  }
  if (h3) {
    const double2 a = h3[o];
    v.x = fma(c.w, a.x, v.x);
    v.y = fma(c.w, a.y, v.y);
  }
  x[i] = v;
}

}  // namespace rx

using namespace rx;

namespace {

int qfail(reaxff_ctx* c, int code, const std::string& msg) {
  c->err = msg;
  return code;
}

#define QHIP(ctx, expr)                                                                  \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return qfail(ctx, REAXFF_ERR_HIP, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

template <class T>
int qgrow(reaxff_ctx* c, T*& p, int64_t& cap, int64_t need) {
  if (need <= cap && p) return 0;
  if (p) (void)hipFree(p);
  p = nullptr;
  const int64_t n = std::max<int64_t>(need + need / 8 + 64, 64);
  const hipError_t e = hipMalloc(&p, sizeof(T) * n);
  if (e != hipSuccess) {
    cap = 0;
    return qfail(c, REAXFF_ERR_HIP, std::string("hipMalloc (QEq): ") + hipGetErrorString(e));
  }
  cap = n;
  return 0;
}

}  // namespace

extern "C" {

int reaxff_set_qeq_product(reaxff_ctx* c, int32_t mode) {
  if (!c) return REAXFF_ERR_ARG;
  if (mode != REAXFF_QEQ_AUTO && mode != REAXFF_QEQ_STORED)
    return qfail(c, REAXFF_ERR_ARG, "reaxff_set_qeq_product: mode must be REAXFF_QEQ_AUTO or REAXFF_QEQ_STORED");
  c->qeq.mode = mode;
  return REAXFF_OK;
}

int reaxff_qeq(reaxff_ctx* c, int64_t n, const reaxff_qeq_params* qpar, double tol, int32_t maxit,
               int32_t guess, double* q, double* s_out, double* t_out, int32_t* iters, double* resid,
               hipStream_t st) {
  if (!c) return REAXFF_ERR_ARG;
  if (!qpar || (n > 0 && !q)) return qfail(c, REAXFF_ERR_ARG, "reaxff_qeq: null pointer");
  if (!(tol > 0.0) || maxit < 0 || maxit > REAXFF_QEQ_MAXIT)
    return qfail(c, REAXFF_ERR_ARG, "reaxff_qeq: tol must be > 0 and maxit within 0..REAXFF_QEQ_MAXIT");
  for (int t = 0; t < NT; ++t)
    if (!(qpar->J[t] > 0.0) || !std::isfinite(qpar->J[t]) || !std::isfinite(qpar->chi[t]))
      return qfail(c, REAXFF_ERR_ARG, "reaxff_qeq: J must be positive and finite, chi finite");
  if (!c->built || n != c->L.n) return qfail(c, REAXFF_ERR_STATE, "reaxff_qeq: lists not built for this n");
  QHIP(c, hipSetDevice(c->device));
  if (iters) *iters = 0;
  if (resid) resid[0] = resid[1] = 0.0;
  if (n == 0) return REAXFF_OK;
  Qeq& Q = c->qeq;
  QeqPar qp{};
  for (int t = 0; t < NT; ++t) {
    qp.chi[t] = qpar->chi[t];
    qp.J[t] = qpar->J[t];
    qp.Jinv[t] = 1.0 / qpar->J[t];
  }
  // per-atom vectors, reduction sets (one per iteration, plus start and final)
  if (qgrow(c, Q.x, Q.cap_n, n)) return REAXFF_ERR_HIP;
  if (n > Q.cap_vec) {
    for (double2** v : {&Q.r, &Q.p, &Q.ap}) {
      if (*v) (void)hipFree(*v);
      *v = nullptr;
      QHIP(c, hipMalloc(v, sizeof(double2) * Q.cap_n));
    }
    for (int k = 0; k < 4; ++k) {
      if (Q.hist[k]) (void)hipFree(Q.hist[k]);
      Q.hist[k] = nullptr;
      QHIP(c, hipMalloc(&Q.hist[k], sizeof(double2) * Q.cap_n));
    }
    Q.cap_vec = Q.cap_n;
    Q.nhist = 0;
  }
  const int64_t nsets = (int64_t)maxit + 2;
  if (qgrow(c, Q.red, Q.cap_red, nsets * ESLOT * QF)) return REAXFF_ERR_HIP;
  if (!Q.red_host) QHIP(c, hipHostMalloc(&Q.red_host, sizeof(double) * ESLOT * QF, hipHostMallocDefault));
  if (!Q.need) QHIP(c, hipMalloc(&Q.need, sizeof(int32_t)));
  // stored rows: width from the density estimate
  const Lists& L = c->L;
  const Grid& g = c->grid;
  if (Q.w == 0) {
    double vol = 1.0;
    for (int k = 0; k < 3; ++k) vol *= g.periodic ? g.L[k] : std::max(g.nc[k] / g.invw[k], 1.0);
    const double rho = (double)n / vol;
    const double r = c->cut.r_nonb;
    Q.w = (int32_t)std::min<double>((double)std::max<int64_t>(n, 1), 1.3 * rho * 4.18879 * r * r * r + 64.0);
  }
  const unsigned gw = xcd_grid((n + QWAVES - 1) / QWAVES), ga = xcd_grid((n + QB - 1) / QB);
  const int64_t ncell = (int64_t)g.nc[0] * g.nc[1] * g.nc[2];
  if (stencil_chunks(g) > QRMAXQ) return qfail(c, REAXFF_ERR_STATE, "reaxff_qeq: stencil beyond the chunk table");
  const unsigned gc = xcd_grid((unsigned)((ncell + QWAVES - 1) / QWAVES));
  // the product: matrix-free over the half far rows when the build left them
  // (and the stored rows are not asked for), else the stored rows
  const bool half = Q.mode == REAXFF_QEQ_AUTO && L.nb_half != 0 && g.reach <= 2;
  const int nrun = g.nc[0] * g.nc[1] * run_rows(g), per_run_xcd = (nrun + 7) / 8;
  if (half) {
    if (qgrow(c, Q.part, Q.cap_part, (int64_t)nrun * 2 * NB_HALF_CAP)) return REAXFF_ERR_HIP;
    if (qgrow(c, Q.tab, Q.cap_tab, (int64_t)nrun * NB_QMAX)) return REAXFF_ERR_HIP;
  }
  auto product = [&](const double2* xin, double2* yout, double* set) {
    if (half) {
      c->prof.begin(KID_QEQ_HALF, st);
      hipLaunchKernelGGL(k_qeq_half, dim3(8u * (unsigned)per_run_xcd), dim3(QH_BS), 0, st, c->dp, g, L, nrun,
                         per_run_xcd, xin, Q.part, Q.tab);
      c->prof.end(st);
      c->prof.begin(KID_QEQ_HREDUCE, st);
      if (g.reach == 1)
        hipLaunchKernelGGL(k_qeq_hreduce<1>, dim3(ga), dim3(QB), 0, st, g, L, Q.tab, Q.part, qp, xin, yout, set);
      else
        hipLaunchKernelGGL(k_qeq_hreduce<2>, dim3(ga), dim3(QB), 0, st, g, L, Q.tab, Q.part, qp, xin, yout, set);
      c->prof.end(st);
    } else {
      c->prof.begin(KID_QEQ_SPMV, st);
      hipLaunchKernelGGL(k_qeq_spmv, dim3(gw), dim3(QB), 0, st, L, Q.hj, Q.hv, Q.hcnt, Q.w, qp, xin, yout, set);
      c->prof.end(st);
    }
  };
  // the stored rows, the width grown if a row overflows
  for (int attempt = 0; !half; ++attempt) {
    if (qgrow(c, Q.hj, Q.cap_rows, n * (int64_t)Q.w)) return REAXFF_ERR_HIP;
    int64_t capv = Q.cap_rowsv;
    if (qgrow(c, Q.hv, capv, n * (int64_t)Q.w)) return REAXFF_ERR_HIP;
    Q.cap_rowsv = capv;
    if (!Q.hcnt || Q.cap_cnt < n) {
      if (qgrow(c, Q.hcnt, Q.cap_cnt, n)) return REAXFF_ERR_HIP;
    }
    QHIP(c, hipMemsetAsync(Q.need, 0, sizeof(int32_t), st));
    c->prof.begin(KID_QEQ_ROWS, st);
    hipLaunchKernelGGL(k_qeq_rows, dim3(gc), dim3(QB), 0, st, c->dp, g, L, (int)ncell, Q.hj, Q.hv, Q.hcnt, Q.w,
                       Q.need);
    c->prof.end(st);
    int32_t need = 0;
    QHIP(c, hipMemcpyAsync(&need, Q.need, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    QHIP(c, hipStreamSynchronize(st));
    if (need <= Q.w) break;
    if (attempt >= 2) return qfail(c, REAXFF_ERR_CAPACITY, "reaxff_qeq: row width did not converge");
    Q.w = need + need / 8 + 16;
  }
  QHIP(c, hipMemsetAsync(Q.red, 0, sizeof(double) * nsets * ESLOT * QF, st));
  double* const start = Q.red;                       // set -1
  auto set_of = [&](int k) { return Q.red + (int64_t)(k + 1) * ESLOT * QF; };
  // initial guess
  const bool use_guess = guess != 0 && Q.nhist > 0 && Q.hist_n == n;
  if (!use_guess) Q.nhist = 0;
  if (use_guess) {
    static const double coef[4][4] = {{1, 0, 0, 0}, {2, -1, 0, 0}, {3, -3, 1, 0}, {4, -6, 4, -1}};
    const int k = std::min(Q.nhist, 4);
    const double* cf = coef[k - 1];
    auto h = [&](int a) -> const double2* { return a < k ? Q.hist[(Q.head - a + 4) % 4] : nullptr; };
    hipLaunchKernelGGL(k_qeq_guess, dim3(ga), dim3(QB), 0, st, L, h(0), h(1), h(2), h(3),
                       make_double4(cf[0], cf[1], cf[2], cf[3]), Q.x);
    product(Q.x, Q.ap, nullptr);
    hipLaunchKernelGGL(k_qeq_start, dim3(ga), dim3(QB), 0, st, L, qp, Q.ap, Q.x, Q.r, Q.p, start);
  } else {
    hipLaunchKernelGGL(k_qeq_start, dim3(ga), dim3(QB), 0, st, L, qp, (const double2*)nullptr, Q.x, Q.r, Q.p,
                       start);
  }
  // relative residuals of a set, read on the host
  double bb[2] = {0, 0};
  auto residuals = [&](const double* set, double out[2], bool first) -> int {
    QHIP(c, hipMemcpyAsync(Q.red_host, set, sizeof(double) * ESLOT * QF, hipMemcpyDeviceToHost, st));
    QHIP(c, hipStreamSynchronize(st));
    double rr[2] = {0, 0};
    for (int k = 0; k < ESLOT; ++k) {
      rr[0] += Q.red_host[k * QF + 4];
      rr[1] += Q.red_host[k * QF + 5];
      if (first) {
        bb[0] += Q.red_host[k * QF + 6];
        bb[1] += Q.red_host[k * QF + 7];
      }
    }
    for (int s = 0; s < 2; ++s) out[s] = bb[s] > 0.0 ? std::sqrt(rr[s] / bb[s]) : std::sqrt(rr[s]);
    return 0;
  };
  double res[2];
  if (residuals(start, res, true)) return REAXFF_ERR_HIP;
  int it = 0;
  const double* last = start;
  while ((res[0] > tol || res[1] > tol) && it < maxit) {
    double* cur = set_of(it);
    product(Q.p, Q.ap, cur);
    c->prof.begin(KID_QEQ_VEC, st);
    hipLaunchKernelGGL(k_qeq_update, dim3(ga), dim3(QB), 0, st, L, qp, last, cur, Q.x, Q.r, Q.p, Q.ap);
    c->prof.end(st);
    ++it;
    if (residuals(cur, res, false)) return REAXFF_ERR_HIP;
    if (res[0] > tol || res[1] > tol) {
      c->prof.begin(KID_QEQ_VEC, st);
      hipLaunchKernelGGL(k_qeq_direction, dim3(ga), dim3(QB), 0, st, L, qp, last, cur, Q.r, Q.p);
      c->prof.end(st);
    }
    last = cur;
  }
  // charges, and the solutions into the history ring
  double* fin = set_of(maxit);
  QHIP(c, hipMemsetAsync(fin, 0, sizeof(double) * ESLOT * QF, st));
  hipLaunchKernelGGL(k_qeq_sums, dim3(ga), dim3(QB), 0, st, L, Q.x, fin);
  Q.head = (Q.head + 1) % 4;
  hipLaunchKernelGGL(k_qeq_charges, dim3(ga), dim3(QB), 0, st, L, Q.x, fin, q, Q.hist[Q.head], s_out, t_out);
  Q.nhist = std::min(Q.nhist + 1, 4);
  Q.hist_n = n;
  QHIP(c, hipGetLastError());
  if (iters) *iters = it;
  if (resid) {
    resid[0] = res[0];
    resid[1] = res[1];
  }
  if (res[0] > tol || res[1] > tol)
    return qfail(c, REAXFF_ERR_CONVERGENCE, "reaxff_qeq: not converged within maxit iterations");
  return REAXFF_OK;
}

}  // extern "C"
