// Exact plain forces on a marked subset of the atoms, at a cost that follows
// the subset rather than the whole system.
//
// The force on atom f, -dE/dx_f, collects every term whose inputs include
// x_f.  A pair term reaches r_nonb.  Every bonded term reads positions at
// most three bond hops from its centre: its corrected bond orders read the
// uncorrected orders of their atoms' own bonds (one hop on), and the
// over/under-coordination and coalition terms read a neighbour's total bond
// order, whose corrections reach one hop further.  So a bonded term that
// moves f has its centre within three hops of f and its inputs within six.
// A hydrogen bond X-H...Z reads its donor bond's order (two hops from H)
// and Z within r_hb of H.  With b the largest distance at which an
// uncorrected bond order still reaches bo_cut (a hop is never longer), every
// input of every term that moves a marked atom lies within
//     R = max(r_nonb, 6 b, r_hb + 2 b)
// of it.  The plain evaluation of the atoms within R of the marked ones (in
// the same periodic box, so every distance is the same) therefore computes
// every such term exactly as the whole system would; the marked atoms'
// forces are taken from it and the rest of it is discarded.
//
// The subsystem is found on a grid of cells at least R / 3 wide: cells
// holding a marked atom are marked, the marks dilated by three cells along
// each axis in turn (wrapping in a periodic box), and the atoms of marked
// cells (a superset of the balls of radius R) gathered in caller order.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "internal.h"

namespace rx {

constexpr int MB = 256;
constexpr int MK = 3;   // dilation in cells; cells are at least R / MK wide

struct MGrid {
  int nc[3];
  int periodic;
  double lo[3], invw[3];
};

__device__ __forceinline__ int mcell(double x, int k, const MGrid& g) {
  int c = (int)floor((x - g.lo[k]) * g.invw[k]);
  if (g.periodic) {
    c %= g.nc[k];
    if (c < 0) c += g.nc[k];
  } else {
    c = c < 0 ? 0 : (c >= g.nc[k] ? g.nc[k] - 1 : c);
  }
  return c;
}

__global__ __launch_bounds__(MB) void k_mask_cells(int64_t n, const double* __restrict__ pos,
                                                   const uint8_t* __restrict__ mask, MGrid g,
                                                   int32_t* __restrict__ cid, uint8_t* __restrict__ mark) {
  const int64_t i = blockIdx.x * (int64_t)MB + threadIdx.x;
  if (i >= n) return;
  const int c = (mcell(pos[3 * i], 0, g) * g.nc[1] + mcell(pos[3 * i + 1], 1, g)) * g.nc[2] +
                mcell(pos[3 * i + 2], 2, g);
  cid[i] = c;
  if (mask[i]) mark[c] = 1;   // the same value from every writer
}

// out[c] = OR of in over MK cells either side along axis `ax`
__global__ __launch_bounds__(MB) void k_dilate(int ncell, MGrid g, int ax, const uint8_t* __restrict__ in,
                                               uint8_t* __restrict__ out) {
  const int c = blockIdx.x * MB + threadIdx.x;
  if (c >= ncell) return;
  int x[3];
  x[2] = c % g.nc[2];
  x[1] = (c / g.nc[2]) % g.nc[1];
  x[0] = c / (g.nc[1] * g.nc[2]);
  const int stride = ax == 2 ? 1 : (ax == 1 ? g.nc[2] : g.nc[1] * g.nc[2]);
  const int nax = g.nc[ax];
  uint8_t v = 0;
  if (g.periodic && nax <= 2 * MK + 1) {
    for (int k = 0; k < nax && !v; ++k) v = in[c + (k - x[ax]) * stride];
  } else {
    for (int d = -MK; d <= MK && !v; ++d) {
      int y = x[ax] + d;
      if (g.periodic) y = (y % nax + nax) % nax;
      else if (y < 0 || y >= nax) continue;
      v = in[c + (y - x[ax]) * stride];
    }
  }
  out[c] = v;
}

__global__ __launch_bounds__(MB) void k_mask_select(int64_t n, const int32_t* __restrict__ cid,
                                                    const uint8_t* __restrict__ mark, int32_t* __restrict__ sel) {
  const int64_t i = blockIdx.x * (int64_t)MB + threadIdx.x;
  if (i < n) sel[i] = mark[cid[i]] ? 1 : 0;
}

__global__ __launch_bounds__(MB) void k_mask_gather(int64_t n, const int32_t* __restrict__ sel,
                                                    const int32_t* __restrict__ idx, const double* __restrict__ pos,
                                                    const int32_t* __restrict__ type, const double* __restrict__ q,
                                                    double* __restrict__ spos, int32_t* __restrict__ stype,
                                                    double* __restrict__ sq) {
  const int64_t i = blockIdx.x * (int64_t)MB + threadIdx.x;
  if (i >= n || !sel[i]) return;
  const int64_t k = idx[i];
  spos[3 * k] = pos[3 * i];
  spos[3 * k + 1] = pos[3 * i + 1];
  spos[3 * k + 2] = pos[3 * i + 2];
  stype[k] = type[i];
  sq[k] = q[i];
}

__global__ __launch_bounds__(MB) void k_mask_scatter(int64_t n, const uint8_t* __restrict__ mask,
                                                     const int32_t* __restrict__ idx,
                                                     const double* __restrict__ sf, double* __restrict__ forces) {
  const int64_t i = blockIdx.x * (int64_t)MB + threadIdx.x;
  if (i >= n || !mask[i]) return;
  const int64_t k = idx[i];
  forces[3 * i] = sf[3 * k];
  forces[3 * i + 1] = sf[3 * k + 1];
  forces[3 * i + 2] = sf[3 * k + 2];
}

}  // namespace rx

using namespace rx;

namespace {

int mfail(reaxff_ctx* c, int code, const std::string& msg) {
  c->err = msg;
  return code;
}

#define MHIP(ctx, expr)                                                                  \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return mfail(ctx, REAXFF_ERR_HIP, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

template <class T>
int mgrow(reaxff_ctx* c, T*& p, int64_t& cap, int64_t need) {
  if (need <= cap && p) return 0;
  if (p) (void)hipFree(p);
  p = nullptr;
  const int64_t k = std::max<int64_t>(need + need / 8 + 64, 64);
  const hipError_t e = hipMalloc(&p, sizeof(T) * k);
  if (e != hipSuccess) {
    cap = 0;
    return mfail(c, REAXFF_ERR_HIP, std::string("hipMalloc (masked forces): ") + hipGetErrorString(e));
  }
  cap = k;
  return 0;
}

inline unsigned mb(int64_t n) { return (unsigned)std::max<int64_t>((n + MB - 1) / MB, 1); }

}  // namespace

extern "C" {

double reaxff_dependency_radius(const reaxff_ctx* c) {
  if (!c) return 0.0;
  double b = 0.0;
  for (int t = 0; t < NT * NT; ++t) b = std::max(b, std::sqrt(c->hd.pair[t].reach2));
  return std::max(c->cut.r_nonb, std::max(6.0 * b, c->cut.r_hb + 2.0 * b));
}

int reaxff_forces_masked(reaxff_ctx* c, int64_t n, const double* pos, const int32_t* type, const double* q,
                         const double* box, const uint8_t* mask, double* forces, int64_t* nsub, hipStream_t st) {
  if (!c) return REAXFF_ERR_ARG;
  if (n < 0 || (n > 0 && (!pos || !type || !q || !mask || !forces)))
    return mfail(c, REAXFF_ERR_ARG, "reaxff_forces_masked: bad n or null pointer");
  if (nsub) *nsub = 0;
  if (n == 0) return REAXFF_OK;
  MHIP(c, hipSetDevice(c->device));
  Masked& M = c->masked;
  const double R = reaxff_dependency_radius(c);
  // the grid: the box, or the bounding box of a non-periodic system
  MGrid g{};
  double ext[3];
  if (box) {
    g.periodic = 1;
    for (int k = 0; k < 3; ++k) {
      if (!(std::isfinite(box[k]) && box[k] > 0.0)) return mfail(c, REAXFF_ERR_BOX, "bad box");
      g.lo[k] = 0.0;
      ext[k] = box[k];
    }
  } else {
    const int nparts = (int)std::min<int64_t>(std::max<int64_t>((n + 255) / 256, 1), 1024);
    if (mgrow(c, M.part, M.cap_part, 6 * nparts)) return REAXFF_ERR_HIP;
    if (mgrow(c, M.flag, M.cap_flag, 4)) return REAXFF_ERR_HIP;
    MHIP(c, hipMemsetAsync(M.flag, 0, sizeof(int32_t) * 4, st));
    if (launch_bbox(pos, type, n, M.part, nparts, M.flag, c->prof, st))
      return mfail(c, REAXFF_ERR_HIP, "bounding box launch failed");
    std::vector<double> part(6 * nparts);
    MHIP(c, hipMemcpyAsync(part.data(), M.part, sizeof(double) * 6 * nparts, hipMemcpyDeviceToHost, st));
    MHIP(c, hipStreamSynchronize(st));
    for (int k = 0; k < 3; ++k) {
      double lo = 1e300, hi = -1e300;
      for (int b = 0; b < nparts; ++b) {
        lo = std::min(lo, part[6 * b + k]);
        hi = std::max(hi, part[6 * b + 3 + k]);
      }
      if (!std::isfinite(lo) || !std::isfinite(hi)) return mfail(c, REAXFF_ERR_NONFINITE, "non-finite position");
      g.lo[k] = lo;
      ext[k] = std::max(hi - lo, 1e-9);
    }
  }
  int64_t ncell = 1;
  for (int k = 0; k < 3; ++k) {
    int nc = (int)std::floor(ext[k] / (R / MK));
    nc = std::max(1, std::min(nc, 512));
    g.nc[k] = nc;
    g.invw[k] = nc / ext[k];
    ncell *= nc;
  }
  if (mgrow(c, M.cid, M.cap_cid, n)) return REAXFF_ERR_HIP;
  if (mgrow(c, M.sel, M.cap_sel, n + 1)) return REAXFF_ERR_HIP;
  if (mgrow(c, M.idx, M.cap_idx, n + 1)) return REAXFF_ERR_HIP;
  if (mgrow(c, M.mark, M.cap_mark, ncell)) return REAXFF_ERR_HIP;
  if (mgrow(c, M.mark2, M.cap_mark2, ncell)) return REAXFF_ERR_HIP;
  MHIP(c, hipMemsetAsync(M.mark, 0, ncell, st));
  hipLaunchKernelGGL(k_mask_cells, dim3(mb(n)), dim3(MB), 0, st, n, pos, mask, g, M.cid, M.mark);
  for (int ax = 0; ax < 3; ++ax) {
    hipLaunchKernelGGL(k_dilate, dim3(mb(ncell)), dim3(MB), 0, st, (int)ncell, g, ax, M.mark, M.mark2);
    std::swap(M.mark, M.mark2);
  }
  hipLaunchKernelGGL(k_mask_select, dim3(mb(n)), dim3(MB), 0, st, n, M.cid, M.mark, M.sel);
  MHIP(c, hipMemsetAsync(M.sel + n, 0, sizeof(int32_t), st));
  if (scan_i32(M.sel, M.idx, n + 1, c->sc, st)) return mfail(c, REAXFF_ERR_HIP, "scan failed");
  int32_t ns = 0;
  MHIP(c, hipMemcpyAsync(&ns, M.idx + n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  MHIP(c, hipStreamSynchronize(st));
  if (nsub) *nsub = ns;
  if (ns == 0) return REAXFF_OK;
  if (mgrow(c, M.spos, M.cap_spos, 3 * (int64_t)ns)) return REAXFF_ERR_HIP;
  if (mgrow(c, M.sforce, M.cap_sforce, 3 * (int64_t)ns)) return REAXFF_ERR_HIP;
  if (mgrow(c, M.sq, M.cap_sq, (int64_t)ns)) return REAXFF_ERR_HIP;
  if (mgrow(c, M.stype, M.cap_stype, (int64_t)ns)) return REAXFF_ERR_HIP;
  if (!M.senergy) MHIP(c, hipMalloc(&M.senergy, sizeof(double) * NTERMS));
  hipLaunchKernelGGL(k_mask_gather, dim3(mb(n)), dim3(MB), 0, st, n, M.sel, M.idx, pos, type, q, M.spos, M.stype,
                     M.sq);
  int rc = reaxff_build_lists(c, ns, M.spos, M.stype, box, st);
  if (rc) return rc;
  rc = reaxff_compute_forces(c, ns, M.spos, M.stype, M.sq, box, M.sforce, M.senergy, st);
  if (rc) return rc;
  hipLaunchKernelGGL(k_mask_scatter, dim3(mb(n)), dim3(MB), 0, st, n, mask, M.idx, M.sforce, forces);
  MHIP(c, hipGetLastError());
  return REAXFF_OK;
}

}  // extern "C"
