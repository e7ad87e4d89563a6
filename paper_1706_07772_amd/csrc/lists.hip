// List construction on the GPU: cell-sorted layout, far-neighbour half list,
// full bond list with mirror index, and hydrogen-bond list.
//
// The paper builds the bond and H-bond lists in one pass over the half
// neighbour list and serialises only the slot reservation (Section 3.3); the
// 3-body list is counted, prefix-summed and then filled (Section 3.3,
// "Three-body Interactions").  Here every list is built the latter way:
// one thread per atom counts its entries of all three lists in one sweep over
// its cell stencil, the counts are prefix-summed, and a second sweep writes
// each entry at its atom's offset.  No slot is ever contended, the order of
// entries is deterministic, and the only host synchronisation is the readback
// of the three totals that size the buffers.
#include "reaxff_dev.h"
#include "internal.h"

namespace rx {

// ---------------------------------------------------------------------------
// cell assignment and counting sort
// ---------------------------------------------------------------------------
__device__ __forceinline__ int cell_coord(double x, int k, const Grid& g) {
  double v = x - g.lo[k];
  if (g.periodic) v -= g.L[k] * floor(v * g.invL[k]);
  int c = (int)floor(v * g.invw[k]);
  c = c < 0 ? 0 : c;
  c = c >= g.nc[k] ? g.nc[k] - 1 : c;
  return c;
}

// bounding box and finiteness check: per-block partial min/max
// and type check (flag bit 0)
__global__ void k_bbox(const double* __restrict__ pos, const int32_t* __restrict__ type, int64_t n,
                       double* __restrict__ part, int32_t* __restrict__ flag) {
  __shared__ double sh[6][256];
  double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
  bool bad = false, badt = false;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int t = type[i];
    if (t < 0 || t >= NT) badt = true;
    for (int k = 0; k < 3; ++k) {
      const double v = pos[3 * i + k];
      if (!isfinite(v)) bad = true;
      mn[k] = fmin(mn[k], v);
      mx[k] = fmax(mx[k], v);
    }
  }
  if (badt) atomicOr(flag, 1);
  for (int k = 0; k < 3; ++k) {
    sh[k][threadIdx.x] = bad ? -1e308 : mn[k];   // a non-finite value poisons the min
    sh[3 + k][threadIdx.x] = mx[k];
  }
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int k = 0; k < 3; ++k) {
        sh[k][threadIdx.x] = fmin(sh[k][threadIdx.x], sh[k][threadIdx.x + s]);
        sh[3 + k][threadIdx.x] = fmax(sh[3 + k][threadIdx.x], sh[3 + k][threadIdx.x + s]);
      }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < 6; ++k) part[6 * blockIdx.x + k] = sh[k][0];
}

__global__ void k_cell_hist(const double* __restrict__ pos, const int32_t* __restrict__ type,
                            int64_t n, Grid g, int32_t* __restrict__ cid,
                            int32_t* __restrict__ count, int32_t* __restrict__ flag) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c0 = cell_coord(pos[3 * i], 0, g), c1 = cell_coord(pos[3 * i + 1], 1, g),
            c2 = cell_coord(pos[3 * i + 2], 2, g);
  const int c = (c0 * g.nc[1] + c1) * g.nc[2] + c2;
  cid[i] = c;
  atomicAdd(&count[c], 1);
}

__global__ void k_cell_scatter(const int32_t* __restrict__ cid, int64_t n,
                               const int32_t* __restrict__ start, int32_t* __restrict__ cursor,
                               int32_t* __restrict__ perm) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c = cid[i];
  const int slot = start[c] + atomicAdd(&cursor[c], 1);
  perm[slot] = (int32_t)i;
}

// order the atoms of each cell by caller index: a deterministic layout
__global__ void k_cell_sort(const int32_t* __restrict__ start, int ncell, int32_t* __restrict__ perm) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncell) return;
  const int a = start[c], b = start[c + 1];
  for (int s = a + 1; s < b; ++s) {
    const int v = perm[s];
    int t = s - 1;
    while (t >= a && perm[t] > v) {
      perm[t + 1] = perm[t];
      --t;
    }
    perm[t + 1] = v;
  }
}

__global__ void k_gather_sorted(const double* __restrict__ pos, const int32_t* __restrict__ type,
                                const int32_t* __restrict__ perm, const int32_t* __restrict__ cid,
                                int64_t n, double4* __restrict__ xs, int32_t* __restrict__ type_s,
                                int32_t* __restrict__ cell_s) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int i = perm[s];
  xs[s] = make_double4(pos[3 * i], pos[3 * i + 1], pos[3 * i + 2], (double)type[i]);
  type_s[s] = type[i];
  cell_s[s] = cid[i];
}

// ---------------------------------------------------------------------------
// raw uncorrected bond order of a pair (sigma scaled by 1 + bo_cut)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double bo_raw(const PairP& p, double r, double bo_cut) {
  double s = 0.0, pi = 0.0, pp = 0.0;
  if (p.r_s > 0.0) s = (1.0 + bo_cut) * exp(p.p_bo1 * pow(r / p.r_s, p.p_bo2));
  if (p.r_p > 0.0) pi = exp(p.p_bo3 * pow(r / p.r_p, p.p_bo4));
  if (p.r_pp > 0.0) pp = exp(p.p_bo5 * pow(r / p.r_pp, p.p_bo6));
  return s + pi + pp;
}

// visit every atom slot in the cell stencil of cell (c0,c1,c2).  Cells are
// numbered with z fastest, so the 5 cells of a stencil column (x, y, z-2..z+2)
// are one contiguous range of sorted atoms (two when the column wraps).
template <class F>
__device__ __forceinline__ void for_stencil(const Grid& g, const int32_t* __restrict__ cstart,
                                            int c0, int c1, int c2, F&& f) {
  // z ranges of the column, as offsets within a row of cells
  int za0, za1, zb0 = 0, zb1 = 0;   // [za0, za1) and [zb0, zb1) in cell units
  if (g.full[2]) {
    za0 = 0; za1 = g.nc[2];
  } else if (g.periodic) {
    if (c2 - 2 < 0) { za0 = 0; za1 = c2 + 3; zb0 = g.nc[2] + c2 - 2; zb1 = g.nc[2]; }
    else if (c2 + 2 >= g.nc[2]) { za0 = c2 - 2; za1 = g.nc[2]; zb0 = 0; zb1 = c2 + 3 - g.nc[2]; }
    else { za0 = c2 - 2; za1 = c2 + 3; }
  } else {
    za0 = c2 - 2 < 0 ? 0 : c2 - 2;
    za1 = c2 + 3 > g.nc[2] ? g.nc[2] : c2 + 3;
  }
  for (int a = 0; a < g.span[0]; ++a) {
    int x = g.full[0] ? a : c0 + a - 2;
    if (g.periodic) x = x < 0 ? x + g.nc[0] : (x >= g.nc[0] ? x - g.nc[0] : x);
    else if (x < 0 || x >= g.nc[0]) continue;
    for (int b = 0; b < g.span[1]; ++b) {
      int y = g.full[1] ? b : c1 + b - 2;
      if (g.periodic) y = y < 0 ? y + g.nc[1] : (y >= g.nc[1] ? y - g.nc[1] : y);
      else if (y < 0 || y >= g.nc[1]) continue;
      const int row = (x * g.nc[1] + y) * g.nc[2];
      const int s0 = cstart[row + za0], s1 = cstart[row + za1];
      for (int s = s0; s < s1; ++s) f(s);
      if (zb1 > zb0) {
        const int t0 = cstart[row + zb0], t1 = cstart[row + zb1];
        for (int s = t0; s < t1; ++s) f(s);
      }
    }
  }
}

// One thread per sorted atom, one sweep over its cell stencil.  The sweep
// writes the far list directly (fixed-width blocked layout) and stages bond
// candidates (pairs inside the per-type bond reach) and H-list entries; the
// bond-order test of the candidates then runs as a dense loop per atom, so
// the transcendental work is not paid by every lane of a wavefront whenever
// one lane meets a candidate.  Counts beyond a width are still counted, and
// the largest count of each list is reported so the host can grow the
// buffers and sweep again.
__global__ __launch_bounds__(256) void k_sweep(
    const DevParams* __restrict__ P, Grid g, int64_t n, const double4* __restrict__ xs,
    const int32_t* __restrict__ cell_s, const int32_t* __restrict__ cstart,
    int32_t* __restrict__ far_cnt, int32_t* __restrict__ far_j, int far_w,
    int32_t* __restrict__ cnt_cand, int32_t* __restrict__ cand_j, int cand_w,
    int32_t* __restrict__ cnt_bond, int32_t* __restrict__ bond_t, int bond_w,
    int32_t* __restrict__ cnt_hb, int32_t* __restrict__ hb_t, int hb_w,
    int32_t* __restrict__ need, unsigned long long* __restrict__ far_total) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int nf = 0;
  if (i < n) {
    const double4 xi = xs[i];
    const int ti = (int)xi.w;
    const int c = cell_s[i];
    const int c2 = c % g.nc[2], c1 = (c / g.nc[2]) % g.nc[1], c0 = c / (g.nc[1] * g.nc[2]);
    const double rn2 = P->rn2, rh2 = P->rh2, bo_cut = P->bo_cut;
    const double rb2 = P->r_bond * P->r_bond;
    // bond prefilter of this atom's type against each partner type
    const double q0 = fmin(P->pair[ti * NT + 0].reach2, rb2), q1 = fmin(P->pair[ti * NT + 1].reach2, rb2),
                 q2 = fmin(P->pair[ti * NT + 2].reach2, rb2), q3 = fmin(P->pair[ti * NT + 3].reach2, rb2);
    const double qmax = fmax(fmax(q0, q1), fmax(q2, q3));
    int accmask = 0;
    for (int t = 0; t < NT; ++t) accmask |= (P->atom[t].hbond == 2) << t;
    const bool donor = P->atom[ti].hbond == 1;
    int nc = 0, nh = 0;
    for_stencil(g, cstart, c0, c1, c2, [&](int s) {
      const double4 xj = xs[s];
      double dx = xj.x - xi.x, dy = xj.y - xi.y, dz = xj.z - xi.z;
      if (g.periodic) {
        dx = min_image(dx, g.L[0], g.invL[0]);
        dy = min_image(dy, g.L[1], g.invL[1]);
        dz = min_image(dz, g.L[2], g.invL[2]);
      }
      const double r2 = r2_of(dx, dy, dz);
      if (r2 <= rn2 && s != (int)i) {
        if (nf < far_w) far_j[blk_index(i, nf, far_w)] = s;
        ++nf;
        const int tj = (int)xj.w;
        if (r2 <= qmax) {
          const double qt = tj == 0 ? q0 : (tj == 1 ? q1 : (tj == 2 ? q2 : q3));
          if (r2 <= qt) {
            if (nc < cand_w) cand_j[blk_index(i, nc, cand_w)] = s;
            ++nc;
          }
        }
        if (donor && r2 <= rh2 && ((accmask >> tj) & 1)) {
          if (nh < hb_w) hb_t[blk_index(i, nh, hb_w)] = s;
          ++nh;
        }
      }
    });
    // bond-order test of the staged candidates (kept in stencil order)
    int nb = 0;
    const int ncand = nc < cand_w ? nc : cand_w;
    for (int k = 0; k < ncand; ++k) {
      const int s = cand_j[blk_index(i, k, cand_w)];
      const double4 xj = xs[s];
      double dx = xj.x - xi.x, dy = xj.y - xi.y, dz = xj.z - xi.z;
      if (g.periodic) {
        dx = min_image(dx, g.L[0], g.invL[0]);
        dy = min_image(dy, g.L[1], g.invL[1]);
        dz = min_image(dz, g.L[2], g.invL[2]);
      }
      const double r2 = r2_of(dx, dy, dz);
      if (bo_raw(P->pair[ti * NT + (int)xj.w], sqrt(r2), bo_cut) >= bo_cut) {
        if (nb < bond_w) bond_t[blk_index(i, nb, bond_w)] = s;
        ++nb;
      }
    }
    far_cnt[i] = nf;
    cnt_cand[i] = nc;
    cnt_bond[i] = nb;
    cnt_hb[i] = nh;
    if (nf > far_w) atomicMax(&need[0], nf);
    if (nc > cand_w) atomicMax(&need[1], nc);
    if (nb > bond_w) atomicMax(&need[2], nb);
    if (nh > hb_w) atomicMax(&need[3], nh);
  }
  // total far entries: wave sums, one atomic per wavefront
  unsigned long long v = (unsigned long long)nf;
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((threadIdx.x & 63) == 0 && v) atomicAdd(far_total, v);
}

// staged (blocked) bond and H-list entries -> compressed rows
__global__ void k_compact(int64_t n, const int32_t* __restrict__ cnt_bond,
                          const int32_t* __restrict__ bond_t, int bond_w,
                          const int32_t* __restrict__ bond_off, int32_t* __restrict__ bond_j,
                          const int32_t* __restrict__ cnt_hb, const int32_t* __restrict__ hb_t,
                          int hb_w, const int32_t* __restrict__ hb_off, int32_t* __restrict__ hb_j) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int ob = bond_off[i], nb = cnt_bond[i];
  for (int k = 0; k < nb; ++k) bond_j[ob + k] = bond_t[blk_index(i, k, bond_w)];
  const int oh = hb_off[i], nh = cnt_hb[i];
  for (int k = 0; k < nh; ++k) hb_j[oh + k] = hb_t[blk_index(i, k, hb_w)];
}

// mirror entry: position of i in the bond list of j
__global__ void k_mirror(int64_t n, const int32_t* __restrict__ off, const int32_t* __restrict__ bj,
                         int32_t* __restrict__ mir, int32_t* __restrict__ flag) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int e = off[i]; e < off[i + 1]; ++e) {
    const int j = bj[e];
    int m = -1;
    for (int f = off[j]; f < off[j + 1]; ++f)
      if (bj[f] == (int)i) { m = f; break; }
    // the bond predicate is symmetric, so the partner entry exists; should it
    // not, point at the entry itself and raise the flag rather than index -1
    if (m < 0) {
      atomicOr(flag, 2);
      m = e;
    }
    mir[e] = m;
  }
}

// export helpers: lists in caller indices
// half far list from the full list: the entries with j > i, at per-atom
// offsets hoff (exclusive scan of the per-atom half counts)
template <bool WRITE>
__global__ void k_export_far(int64_t n, const int32_t* __restrict__ cnt, const int32_t* __restrict__ fj,
                             int far_w, const int32_t* __restrict__ perm, int32_t* __restrict__ hcnt,
                             const int64_t* __restrict__ hoff, int32_t* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t o = WRITE ? hoff[i] : 0;
  int h = 0;
  const int pi = WRITE ? perm[i] : 0;
  for (int k = 0; k < cnt[i]; ++k) {
    const int j = fj[blk_index(i, k, far_w)];
    if (j > (int)i) {
      if (WRITE) {
        const int pj = perm[j];
        out[2 * o] = pi < pj ? pi : pj;
        out[2 * o + 1] = pi < pj ? pj : pi;
        ++o;
      }
      ++h;
    }
  }
  if (!WRITE) hcnt[i] = h;
}

__global__ void k_export_csr(int64_t n, const int32_t* __restrict__ off, const int32_t* __restrict__ bj,
                             const int32_t* __restrict__ perm, int32_t* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int pi = perm[i];
  for (int e = off[i]; e < off[i + 1]; ++e) {
    out[2 * (int64_t)e] = pi;
    out[2 * (int64_t)e + 1] = perm[bj[e]];
  }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
static inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

int launch_bbox(const double* pos, const int32_t* type, int64_t n, double* part, int nparts,
                int32_t* flag, Prof& pf, hipStream_t st) {
  pf.begin(KID_BBOX, st);
  hipLaunchKernelGGL(k_bbox, dim3(nparts), dim3(256), 0, st, pos, type, n, part, flag);
  pf.end(st);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_cell_sort(const double* pos, const int32_t* type, int64_t n, const Grid& g, int ncell,
                     Scratch& sc, Lists& L, Prof& pf, hipStream_t st) {
  pf.begin(KID_ZERO, st);
  (void)hipMemsetAsync(sc.cell_count, 0, sizeof(int32_t) * (ncell + 1), st);
  (void)hipMemsetAsync(sc.cell_cursor, 0, sizeof(int32_t) * (ncell + 1), st);
  pf.end(st);
  pf.begin(KID_CELL_HIST, st);
  hipLaunchKernelGGL(k_cell_hist, dim3(nblk(n, 256)), dim3(256), 0, st, pos, type, n, g, sc.cid,
                     sc.cell_count, sc.flag);
  pf.end(st);
  pf.begin(KID_SCAN, st);
  scan_i32(sc.cell_count, L.cell_start, ncell + 1, sc, st);
  pf.end(st);
  pf.begin(KID_CELL_SCATTER, st);
  hipLaunchKernelGGL(k_cell_scatter, dim3(nblk(n, 256)), dim3(256), 0, st, sc.cid, n,
                     L.cell_start, sc.cell_cursor, L.perm);
  pf.end(st);
  pf.begin(KID_CELL_SORT, st);
  hipLaunchKernelGGL(k_cell_sort, dim3(nblk(ncell, 256)), dim3(256), 0, st, L.cell_start, ncell,
                     L.perm);
  pf.end(st);
  pf.begin(KID_GATHER, st);
  hipLaunchKernelGGL(k_gather_sorted, dim3(nblk(n, 256)), dim3(256), 0, st, pos, type, L.perm,
                     sc.cid, n, L.xs, L.type_s, sc.cell_s);
  pf.end(st);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_sweep(const DevParams* P, const Grid& g, int64_t n, Scratch& sc, Lists& L, Prof& pf,
                 hipStream_t st) {
  (void)hipMemsetAsync(sc.need, 0, sizeof(int32_t) * 4, st);
  (void)hipMemsetAsync(sc.totals, 0, sizeof(int64_t) * 4, st);
  pf.begin(KID_LIST_SWEEP, st);
  hipLaunchKernelGGL(k_sweep, dim3(nblk(n, 256)), dim3(256), 0, st, P, g, n, L.xs, sc.cell_s,
                     L.cell_start, L.far_cnt, L.far_j, L.far_w, sc.cnt_cand, sc.cand_j, sc.cand_w,
                     sc.cnt_bond, sc.bond_t, sc.bond_w, sc.cnt_hb, sc.hb_t, sc.hb_w, sc.need,
                     reinterpret_cast<unsigned long long*>(sc.totals));
  pf.end(st);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_compact(int64_t n, Scratch& sc, Lists& L, Prof& pf, hipStream_t st) {
  pf.begin(KID_COMPACT, st);
  hipLaunchKernelGGL(k_compact, dim3(nblk(n, 256)), dim3(256), 0, st, n, sc.cnt_bond, sc.bond_t,
                     sc.bond_w, L.bond_off, L.bond_j, sc.cnt_hb, sc.hb_t, sc.hb_w, L.hb_off, L.hb_j);
  pf.end(st);
  pf.begin(KID_MIRROR, st);
  hipLaunchKernelGGL(k_mirror, dim3(nblk(n, 256)), dim3(256), 0, st, n, L.bond_off, L.bond_j,
                     L.bond_mir, sc.flag);
  pf.end(st);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_export(const Lists& L, int32_t* far, int32_t* bonds, int32_t* hb, Scratch& sc,
                  hipStream_t st) {
  const int64_t n = L.n;
  if (far) {
    int32_t* hcnt = nullptr;
    int64_t* hoff = nullptr;
    if (hipMalloc(&hcnt, sizeof(int32_t) * (n + 1)) != hipSuccess) return -1;
    if (hipMalloc(&hoff, sizeof(int64_t) * (n + 1)) != hipSuccess) return -1;
    (void)hipMemsetAsync(hcnt + n, 0, sizeof(int32_t), st);
    hipLaunchKernelGGL(k_export_far<false>, dim3(nblk(n, 256)), dim3(256), 0, st, n, L.far_cnt,
                       L.far_j, L.far_w, L.perm, hcnt, nullptr, nullptr);
    scan_i32_to_i64(hcnt, hoff, n + 1, sc, st);
    hipLaunchKernelGGL(k_export_far<true>, dim3(nblk(n, 256)), dim3(256), 0, st, n, L.far_cnt,
                       L.far_j, L.far_w, L.perm, nullptr, hoff, far);
    (void)hipStreamSynchronize(st);
    (void)hipFree(hcnt);
    (void)hipFree(hoff);
  }
  if (bonds) hipLaunchKernelGGL(k_export_csr, dim3(nblk(n, 256)), dim3(256), 0, st, n, L.bond_off, L.bond_j, L.perm, bonds);
  if (hb) hipLaunchKernelGGL(k_export_csr, dim3(nblk(n, 256)), dim3(256), 0, st, n, L.hb_off, L.hb_j, L.perm, hb);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace rx
