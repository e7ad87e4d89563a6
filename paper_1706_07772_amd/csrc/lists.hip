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
  xs[s] = make_double4(pos[3 * i], pos[3 * i + 1], pos[3 * i + 2], 0.0);
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

// visit every atom slot in the cell stencil of cell (c0,c1,c2)
template <class F>
__device__ __forceinline__ void for_stencil(const Grid& g, const int32_t* __restrict__ cstart,
                                            int c0, int c1, int c2, F&& f) {
  for (int a = 0; a < g.span[0]; ++a) {
    int x = g.full[0] ? a : c0 + a - 2;
    if (g.periodic) x = x < 0 ? x + g.nc[0] : (x >= g.nc[0] ? x - g.nc[0] : x);
    else if (x < 0 || x >= g.nc[0]) continue;
    for (int b = 0; b < g.span[1]; ++b) {
      int y = g.full[1] ? b : c1 + b - 2;
      if (g.periodic) y = y < 0 ? y + g.nc[1] : (y >= g.nc[1] ? y - g.nc[1] : y);
      else if (y < 0 || y >= g.nc[1]) continue;
      const int row = (x * g.nc[1] + y) * g.nc[2];
      if (g.full[2]) {
        const int s0 = cstart[row], s1 = cstart[row + g.nc[2]];
        for (int s = s0; s < s1; ++s) f(s);
      } else {
        for (int c = 0; c < 5; ++c) {
          int z = c2 + c - 2;
          if (g.periodic) z = z < 0 ? z + g.nc[2] : (z >= g.nc[2] ? z - g.nc[2] : z);
          else if (z < 0 || z >= g.nc[2]) continue;
          const int s0 = cstart[row + z], s1 = cstart[row + z + 1];
          for (int s = s0; s < s1; ++s) f(s);
        }
      }
    }
  }
}

template <bool FILL>
__global__ __launch_bounds__(256) void k_lists(
    const DevParams* __restrict__ P, Grid g, int64_t n, const double4* __restrict__ xs,
    const int32_t* __restrict__ type_s, const int32_t* __restrict__ cell_s,
    const int32_t* __restrict__ cstart, int32_t* __restrict__ cnt_far,
    int32_t* __restrict__ cnt_bond, int32_t* __restrict__ cnt_hb,
    const int64_t* __restrict__ far_off, int32_t* __restrict__ far_j,
    const int32_t* __restrict__ bond_off, int32_t* __restrict__ bond_j,
    const int32_t* __restrict__ hb_off, int32_t* __restrict__ hb_j) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double4 xi = xs[i];
  const int ti = type_s[i];
  const int c = cell_s[i];
  const int c2 = c % g.nc[2], c1 = (c / g.nc[2]) % g.nc[1], c0 = c / (g.nc[1] * g.nc[2]);
  const double rn2 = P->rn2, rh2 = P->rh2, rb2 = P->r_bond * P->r_bond, bo_cut = P->bo_cut;
  const bool donor = P->atom[ti].hbond == 1;
  int64_t pf = FILL ? far_off[i] : 0;
  int pb = FILL ? bond_off[i] : 0, ph = FILL ? hb_off[i] : 0;
  int nf = 0, nb = 0, nh = 0;
  for_stencil(g, cstart, c0, c1, c2, [&](int s) {
    if (s == i) return;
    const double4 xj = xs[s];
    double dx = xj.x - xi.x, dy = xj.y - xi.y, dz = xj.z - xi.z;
    if (g.periodic) {
      dx = min_image(dx, g.L[0], g.invL[0]);
      dy = min_image(dy, g.L[1], g.invL[1]);
      dz = min_image(dz, g.L[2], g.invL[2]);
    }
    const double r2 = r2_of(dx, dy, dz);
    if (s > i && r2 <= rn2) {
      if (FILL) far_j[pf++] = s;
      else ++nf;
    }
    const int tj = type_s[s];
    const PairP& pp = P->pair[ti * NT + tj];
    if (r2 <= rb2 && r2 <= pp.reach2) {
      if (bo_raw(pp, sqrt(r2), bo_cut) >= bo_cut) {
        if (FILL) bond_j[pb++] = s;
        else ++nb;
      }
    }
    if (donor && r2 <= rh2 && P->atom[tj].hbond == 2) {
      if (FILL) hb_j[ph++] = s;
      else ++nh;
    }
  });
  if (!FILL) {
    cnt_far[i] = nf;
    cnt_bond[i] = nb;
    cnt_hb[i] = nh;
  }
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
__global__ void k_export_far(int64_t n, const int64_t* __restrict__ off, const int32_t* __restrict__ fj,
                             const int32_t* __restrict__ perm, int32_t* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int pi = perm[i];
  for (int64_t e = off[i]; e < off[i + 1]; ++e) {
    const int pj = perm[fj[e]];
    out[2 * e] = pi < pj ? pi : pj;
    out[2 * e + 1] = pi < pj ? pj : pi;
  }
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
                int32_t* flag, hipStream_t st) {
  hipLaunchKernelGGL(k_bbox, dim3(nparts), dim3(256), 0, st, pos, type, n, part, flag);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_cell_sort(const double* pos, const int32_t* type, int64_t n, const Grid& g, int ncell,
                     Scratch& sc, Lists& L, hipStream_t st) {
  hipMemsetAsync(sc.cell_count, 0, sizeof(int32_t) * (ncell + 1), st);
  hipMemsetAsync(sc.cell_cursor, 0, sizeof(int32_t) * (ncell + 1), st);
  hipLaunchKernelGGL(k_cell_hist, dim3(nblk(n, 256)), dim3(256), 0, st, pos, type, n, g, sc.cid,
                     sc.cell_count, sc.flag);
  scan_i32(sc.cell_count, L.cell_start, ncell + 1, sc, st);
  hipLaunchKernelGGL(k_cell_scatter, dim3(nblk(n, 256)), dim3(256), 0, st, sc.cid, n,
                     L.cell_start, sc.cell_cursor, L.perm);
  hipLaunchKernelGGL(k_cell_sort, dim3(nblk(ncell, 256)), dim3(256), 0, st, L.cell_start, ncell,
                     L.perm);
  hipLaunchKernelGGL(k_gather_sorted, dim3(nblk(n, 256)), dim3(256), 0, st, pos, type, L.perm,
                     sc.cid, n, L.xs, L.type_s, sc.cell_s);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_count(const DevParams* P, const Grid& g, int64_t n, Scratch& sc, Lists& L, hipStream_t st) {
  hipLaunchKernelGGL(k_lists<false>, dim3(nblk(n, 256)), dim3(256), 0, st, P, g, n, L.xs, L.type_s,
                     sc.cell_s, L.cell_start, sc.cnt_far, sc.cnt_bond, sc.cnt_hb, nullptr, nullptr,
                     nullptr, nullptr, nullptr, nullptr);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_fill(const DevParams* P, const Grid& g, int64_t n, Scratch& sc, Lists& L, hipStream_t st) {
  hipLaunchKernelGGL(k_lists<true>, dim3(nblk(n, 256)), dim3(256), 0, st, P, g, n, L.xs, L.type_s,
                     sc.cell_s, L.cell_start, nullptr, nullptr, nullptr, L.far_off, L.far_j,
                     L.bond_off, L.bond_j, L.hb_off, L.hb_j);
  hipLaunchKernelGGL(k_mirror, dim3(nblk(n, 256)), dim3(256), 0, st, n, L.bond_off, L.bond_j,
                     L.bond_mir, sc.flag);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_export(const Lists& L, int32_t* far, int32_t* bonds, int32_t* hb, hipStream_t st) {
  const int64_t n = L.n;
  if (far) hipLaunchKernelGGL(k_export_far, dim3(nblk(n, 256)), dim3(256), 0, st, n, L.far_off, L.far_j, L.perm, far);
  if (bonds) hipLaunchKernelGGL(k_export_csr, dim3(nblk(n, 256)), dim3(256), 0, st, n, L.bond_off, L.bond_j, L.perm, bonds);
  if (hb) hipLaunchKernelGGL(k_export_csr, dim3(nblk(n, 256)), dim3(256), 0, st, n, L.hb_off, L.hb_j, L.perm, hb);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace rx
