// List construction on the GPU: cell-sorted layout, far-neighbour list,
// full bond list with mirror index, and hydrogen-bond lists.
//
// The paper builds the bond and H-bond lists in one pass over the half
// neighbour list (Section 3.3).  Here one sweep over each cell's stencil
// writes all of them: a wavefront per cell loads the stencil's candidates 64
// at a time, one per lane, and tests them against each of the cell's atoms
// in turn, numbering the accepted ones with a ballot, so every row is filled
// in slot order with no contended counter.  When no dimension is covered
// whole, far and bond-candidate rows take each pair once (from the atom that
// sees the other after its own slot), which halves those tests; H rows keep
// both halves (the slots before a group's own are tested for H pairs only,
// by its donor H and acceptor atoms).  Rows have fixed widths; an overflow
// is counted and reported, and the host widens the rows and sweeps again.
// Bond candidates are then tested on their raw bond order, each bond found
// once is given to its partner's row as well, and the bond rows are
// compacted in increasing partner order with their mirror index.  The only
// host synchronisation is the readback of the totals that size the buffers.
#include <climits>
#include <type_traits>
#include "reaxff_dev.h"
#include "internal.h"
#include "terms.h"

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

// One wavefront per cell.  Every atom of a cell has the same (2R+1)^3 cell
// stencil.  The wavefront lays the stencil's chunks (stencil_chunk) end to end
// and walks the resulting slot sequence in full batches of 64 candidates, one
// per lane (each lane advances through a table of the chunks' first atoms,
// first slots and image shifts in LDS), loading each batch once and testing
// it against each atom of its cell in turn: the cell's atoms live in the
// lanes and are broadcast one at a time.  Accepted candidates of atom i are
// numbered with a ballot and written contiguously to i's rows (far list, bond
// candidates inside the per-type bond reach, H lists), in slot order.  Entries
// beyond a row's width are counted but not written; the largest count of each
// list is reported so the host can widen the rows and sweep again.  Far
// entries are slots when slots is set (positions in the window of the cell's
// run, window_chunk), sorted atom indices otherwise.  With far_lo set and no
// dimension covered whole, far_lo[i] counts the far entries before i's own
// slot (the pairs the partner's run owns) and need[5] reports the largest
// upper window (the run's first atom to the window's end).
// MINIMG: periodic box without stencil image shifts (minimum image per pair);
// otherwise each chunk carries its image shift (zero in open boundaries).
constexpr int SWEEP_WAVES = 4;
constexpr int SWEEP_MAXQ = 64;   // chunks of a stencil: 2 (2 reach + 1)^2 <= 50

// UPPER: far rows keep only the entries after the centre's own slot.
// HALF (with UPPER): far and bond-candidate rows take each pair once, from
// the atom that sees the other after its own slot, so their tests cover half
// the stencil; batches wholly before a group's own slots are only tested for
// H pairs, by the donor H and acceptor centres.  The bonds' other halves are
// added after the bond test (k_transpose, k_merge_bonds).
template <bool MINIMG, bool UPPER, bool HALF>
__global__ __launch_bounds__(64 * SWEEP_WAVES) void k_sweep(
    const DevParams* __restrict__ P, Grid g, int ncell, const double4* __restrict__ xs,
    const int32_t* __restrict__ cstart, int32_t* __restrict__ far_cnt, int32_t* __restrict__ far_j,
    int far_w, int32_t* __restrict__ cnt_cand, int32_t* __restrict__ cand_j, int cand_w,
    int32_t* __restrict__ hb_cnt, int32_t* __restrict__ hb_j, int hb_w,
    int32_t* __restrict__ ha_cnt, int32_t* __restrict__ ha_j, int ha_w, int slots,
    int32_t* __restrict__ far_lo, int32_t* __restrict__ need, unsigned long long* __restrict__ tslot,
    int32_t* __restrict__ nslot) {
  static_assert(!HALF || UPPER, "each pair once needs the upper rows");
  __shared__ unsigned long long red[SWEEP_WAVES][2];
  __shared__ int q_s0[SWEEP_WAVES][SWEEP_MAXQ], q_base[SWEEP_WAVES][SWEEP_MAXQ + 1];
  __shared__ double q_sh[SWEEP_WAVES][SWEEP_MAXQ][3];
  __shared__ int q_wd[SWEEP_WAVES][SWEEP_MAXQ];
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int c = blockIdx.x * SWEEP_WAVES + wv;
  const unsigned long long below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  unsigned long long tf = 0, th = 0;
  int a0 = 0, m = 0;
  if (c < ncell) {
    a0 = cstart[c];
    m = cstart[c + 1] - a0;
  }
  const double rn2 = P->rn2, rh2 = P->rh2;
  const double rb2 = P->r_bond * P->r_bond;
  int accmask = 0, donmask = 0;
  for (int t = 0; t < NT; ++t) {
    accmask |= (P->atom[t].hbond == 2) << t;
    donmask |= (P->atom[t].hbond == 1) << t;
  }
  // the stencil's chunk table: first atom, first slot and image shift
  int* __restrict__ qs0 = q_s0[wv];
  int* __restrict__ qb = q_base[wv];
  const int nq = stencil_chunks(g);
  {
    int len = 0;
    if (m > 0 && lane < nq) {
      int s0, s1;
      double sx, sy, sz;
      stencil_chunk(g, cstart, c, lane, s0, s1, sx, sy, sz);
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
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  const int nst = m > 0 ? __builtin_amdgcn_readfirstlane(qb[nq]) : 0;
  // slot of the cell's first atom: in the centre column's unwrapped z range,
  // which comes second when the column wraps below the cell
  const bool halfable = far_lo != nullptr && !g.full[0] && !g.full[1] && !g.full[2];
  int own0 = 0;
  if (halfable && m > 0) {
    const int c2 = c % g.nc[2];
    const int q_own = 2 * (g.reach * g.span[1] + g.reach) + (g.periodic && c2 - g.reach < 0 ? 1 : 0);
    own0 = __builtin_amdgcn_readfirstlane(qb[q_own] + (a0 - qs0[q_own]));
    if (g.run <= 1 && lane == 0) atomicMax(&nslot[(blockIdx.x * SWEEP_WAVES + wv) & (ESLOT - 1)], nst - own0);
  }
  // far entries number the window of the cell's run: the slot of a candidate
  // in chunk q is its slot here plus wd[q] (the window chunk of the same
  // column and side, which holds this chunk, laid end to end with the others);
  // need[5] then reports the largest upper window (the run's first atom to
  // the window's end)
  int* __restrict__ wd = q_wd[wv];
  if (g.run > 1 && m > 0) {
    int w0 = 0, w1 = 0;
    if (lane < nq) {
      double sx, sy, sz;
      window_chunk(g, cstart, c, lane, w0, w1, sx, sy, sz);
    }
    const int wl = w1 - w0;
    const int wb = wave_incl_scan(wl) - wl;   // the window chunk's first slot
    const int pair0 = lane & ~1;
    const int a_0 = __shfl(w0, pair0), l_0 = __shfl(wl, pair0), b_0 = __shfl(wb, pair0);
    const int a_1 = __shfl(w0, pair0 + 1), b_1 = __shfl(wb, pair0 + 1);
    if (lane < nq) {
      const int cs0 = qs0[lane];
      const bool in0 = cs0 >= a_0 && cs0 < a_0 + l_0;
      wd[lane] = (in0 ? b_0 + (cs0 - a_0) : b_1 + (cs0 - a_1)) - qb[lane];
    }
    if (halfable) {
      const int c2 = c % g.nc[2], z0 = c2 / g.run * g.run;
      const int q_own = 2 * (g.reach * g.span[1] + g.reach) + (g.periodic && z0 - g.reach < 0 ? 1 : 0);
      const int wend = readlane_i(wb + wl, nq - 1);
      const int w_own = readlane_i(wb, q_own) + (cstart[c - (c2 - z0)] - readlane_i(w0, q_own));
      if (lane == 0) atomicMax(&nslot[(blockIdx.x * SWEEP_WAVES + wv) & (ESLOT - 1)], wend - w_own);
    }
  } else if (lane < nq) {
    wd[lane] = 0;
  }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  for (int ig = 0; ig < m; ig += 64) {       // the cell's atoms, 64 at a time, one per lane
    const int mi = m - ig < 64 ? m - ig : 64;
    double4 xmine = make_double4(0.0, 0.0, 0.0, 0.0);
    if (lane < mi) xmine = xs[a0 + ig + lane];
    const int tmine = (int)xmine.w;
    // bit l: the group's centre l is a donor H / an acceptor
    const unsigned long long donc = ballot(lane < mi && ((donmask >> tmine) & 1));
    const unsigned long long accc = ballot(lane < mi && ((accmask >> tmine) & 1));
    int kf = 0, kc = 0, kh = 0, ka = 0;       // lane l: counts of the cell's atom l
    int klo = 0;                              // lane l: far entries before atom l's own slot
    int q = 0;                                // this lane's chunk
    for (int b0 = 0; b0 < nst; b0 += 64) {
      const int slot = b0 + lane;
      const bool valid = slot < nst;
      int s = 0, wdq = 0;
      double sx = 0.0, sy = 0.0, sz = 0.0;
      if (valid) {
        while (qb[q + 1] <= slot) ++q;
        s = qs0[q] + (slot - qb[q]);
        wdq = wd[q];
        if constexpr (!MINIMG) {
          sx = q_sh[wv][q][0];
          sy = q_sh[wv][q][1];
          sz = q_sh[wv][q][2];
        }
      }
      // HALF: lanes past the stencil's end hold NaN, so every distance
      // test fails there and no mask of valid lanes enters the predicates
      double4 xj = make_double4(HALF ? __builtin_nan("") : 0.0, 0.0, 0.0, 0.0);
      if (valid) xj = xs[s];
      const int tj = (int)xj.w;
      // bond reach of this candidate's type against each centre type
      const double q0 = fmin(P->pair[0 * NT + tj].reach2, rb2), q1 = fmin(P->pair[1 * NT + tj].reach2, rb2),
                   q2 = fmin(P->pair[2 * NT + tj].reach2, rb2), q3 = fmin(P->pair[3 * NT + tj].reach2, rb2);
      const double qmx = fmax(fmax(q0, q1), fmax(q2, q3));   // the largest, whatever the centre's type
      const bool acc = (accmask >> tj) & 1, don = (donmask >> tj) & 1;
      // lane masks of the batch: the count masks below are ANDs of plain
      // compares with these, so no predicate is rebuilt for its ballot
      const unsigned long long vmask = ballot(valid), accl = ballot(valid && acc), donl = ballot(valid && don);
      // the distance of candidate lanes from a centre (uniform position)
      auto dist2 = [&](double4 xi4) {
        double dx = xj.x - xi4.x, dy = xj.y - xi4.y, dz = xj.z - xi4.z;
        if constexpr (MINIMG) {
          dx = min_image(dx, g.L[0], g.invL[0]);
          dy = min_image(dy, g.L[1], g.invL[1]);
          dz = min_image(dz, g.L[2], g.invL[2]);
        } else {
          dx -= sx;
          dy -= sy;
          dz -= sz;
        }
        return r2_of(dx, dy, dz);
      };
      // a centre's H entries of this batch (its hb row for a donor H, its
      // ha row for an acceptor), numbered with the ballot in slot order
      auto hrow = [&](int l, int i, double r2) {
        if ((donc >> l) & 1) {
          const bool h = acc && r2 <= rh2;
          const unsigned long long mh = ballot(h);
          if (mh) {
            const int k2 = readlane_i(kh, l);
            if (h) {
              const int k = k2 + __popcll(mh & below);
              if (k < hb_w) __builtin_nontemporal_store(s, &hb_j[(int64_t)i * hb_w + k]);
            }
            kh = writelane_i(k2 + __popcll(mh), l, kh);
          }
        } else {
          const bool h = don && r2 <= rh2;
          const unsigned long long ma = ballot(h);
          if (ma) {
            const int k3 = readlane_i(ka, l);
            if (h) {
              const int k = k3 + __popcll(ma & below);
              if (k < ha_w) __builtin_nontemporal_store(s, &ha_j[(int64_t)i * ha_w + k]);
            }
            ka = writelane_i(k3 + __popcll(ma), l, ka);
          }
        }
      };
      if constexpr (HALF) {
        // H rows keep both halves (their pairs are few, and rows in slot
        // order need no merging); far and bond-candidate rows only the pairs
        // after each centre's own slot.  A batch wholly before the group's
        // own slots holds H pairs only: the donor H and acceptor centres
        // that have a partner class in it test it.
        if (b0 + 64 <= own0 + ig) {
          unsigned long long hm = (accl ? donc : 0ull) | (donl ? accc : 0ull);
          while (hm) {
            const int l = __builtin_ctzll(hm);
            hm &= hm - 1;
            const int i = a0 + ig + l;
            hrow(l, i, dist2(xs[i]));
          }
          continue;
        }
        const double4* __restrict__ xcen = xs + (a0 + ig);
        int32_t* __restrict__ frow = far_j + (int64_t)(a0 + ig) * far_w;
        for (int l = 0; l < mi; ++l, ++xcen, frow += far_w) {
          const int i = a0 + ig + l;
          const double r2 = dist2(*xcen);
          const int dl = own0 + ig + l - b0;   // the centre's own lane (uniform)
          const bool f = r2 <= rn2 && lane > dl;
          const unsigned long long mf = ballot(f);
          if (mf) {
            const int k0 = readlane_i(kf, l);
            if (f) {
              const int k = k0 + __popcll(mf & below);
              if (k < far_w) __builtin_nontemporal_store(slot + wdq, &frow[k]);
            }
            kf = writelane_i(k0 + __popcll(mf), l, kf);
            if (mf & ballot(r2 <= qmx)) {
              const int ti = readlane_i(tmine, l);
              const double qa = (ti & 1) ? q1 : q0, qbr = (ti & 1) ? q3 : q2;
              const double qt = (ti & 2) ? qbr : qa;
              const bool b = f && r2 <= qt;
              const unsigned long long mb = ballot(b);
              if (mb) {
                const int k1 = readlane_i(kc, l);
                if (b) {
                  const int k = k1 + __popcll(mb & below);
                  if (k < cand_w) __builtin_nontemporal_store(s, &cand_j[(int64_t)i * cand_w + k]);
                }
                kc = writelane_i(k1 + __popcll(mb), l, kc);
              }
            }
          }
          if (((donc | accc) >> l) & 1) hrow(l, i, r2);
        }
        continue;
      }
      // batches holding some centre's own slot set that centre's count of
      // entries before it; the others run the loop without that code
      const bool hasown = !UPPER && halfable && b0 < own0 + ig + mi && b0 + 64 > own0 + ig;
      auto centres = [&](auto own_t) {
        constexpr bool OWN = decltype(own_t)::value;
        // the centre's position and far row, advanced with the centre
        const double4* __restrict__ xcen = xs + (a0 + ig);
        int32_t* __restrict__ frow = far_j + (int64_t)(a0 + ig) * far_w;
        for (int l = 0; l < mi; ++l, ++xcen, frow += far_w) {
          const int i = a0 + ig + l;
          const double4 xi4 = *xcen;   // uniform: a scalar load
          const double xix = xi4.x, xiy = xi4.y, xiz = xi4.z;
          double dx = xj.x - xix, dy = xj.y - xiy, dz = xj.z - xiz;
          if constexpr (MINIMG) {
            dx = min_image(dx, g.L[0], g.invL[0]);
            dy = min_image(dy, g.L[1], g.invL[1]);
            dz = min_image(dz, g.L[2], g.invL[2]);
          } else {
            dx -= sx;
            dy -= sy;
            dz -= sz;
          }
          const double r2 = r2_of(dx, dy, dz);
          const bool f = valid && r2 <= rn2 && s != i;
          const unsigned long long mf = ballot(r2 <= rn2) & ballot(s != i) & vmask;
          if constexpr (OWN) {
            // far entries before the centre's own slot: every entry of the
            // batches below it, plus the lanes below it in the batch holding
            // it (rows fill in slot order), so the count is set once
            const int ol = own0 + ig + l - b0;   // the own slot's lane (uniform)
            if ((unsigned)ol < 64u) {
              const unsigned long long low = ol == 0 ? 0ull : (~0ull >> (64 - ol));
              klo = writelane_i(readlane_i(kf, l) + __popcll(mf & low), l, klo);
            }
          }
          if (mf) {
            // far entries: all, or (UPPER) those after the own slot, whose
            // lane in this batch is d
            unsigned long long mfu = mf;
            const int d = own0 + ig + l - b0;
            if constexpr (UPPER) mfu = d < 0 ? mf : (d >= 63 ? 0ull : (mf & (~0ull << (d + 1))));
            if (mfu) {
              const int k0 = readlane_i(kf, l);
              if (f && (!UPPER || lane > d)) {
                const int k = k0 + __popcll(mfu & below);
                // list rows are streamed out (non-temporal), keeping the
                // stencil's positions in L2
                if (k < far_w) __builtin_nontemporal_store(slots ? slot + wdq : s, &frow[k]);
              }
              kf = writelane_i(k0 + __popcll(mfu), l, kf);
            }
            // bond candidates: the pair reach (by the centre's type) is only
            // selected when some lane lies within its largest one
            if (mf & ballot(r2 <= qmx)) {
              const int ti = readlane_i(tmine, l);
              const double qa = (ti & 1) ? q1 : q0, qbr = (ti & 1) ? q3 : q2;
              const double qt = (ti & 2) ? qbr : qa;
              const unsigned long long mb = mf & ballot(r2 <= qt);
              if (mb) {
                const int k1 = readlane_i(kc, l);
                if (f && r2 <= qt) {
                  const int k = k1 + __popcll(mb & below);
                  if (k < cand_w) __builtin_nontemporal_store(s, &cand_j[(int64_t)i * cand_w + k]);
                }
                kc = writelane_i(k1 + __popcll(mb), l, kc);
              }
            }
            // H-bond rows: only for a donor H or an acceptor centre
            const bool hdon = (donc >> l) & 1, hacc = (accc >> l) & 1;
            if (hdon || hacc) {
              const bool hr = f && r2 <= rh2;
              const unsigned long long mhr = mf & ballot(r2 <= rh2);
              if (hdon) {
                const unsigned long long mh = mhr & accl;
                if (mh) {
                  const int k2 = readlane_i(kh, l);
                  if (hr && acc) {
                    const int k = k2 + __popcll(mh & below);
                    if (k < hb_w) __builtin_nontemporal_store(s, &hb_j[(int64_t)i * hb_w + k]);
                  }
                  kh = writelane_i(k2 + __popcll(mh), l, kh);
                }
              }
              if (hacc) {
                const unsigned long long ma = mhr & donl;
                if (ma) {
                  const int k3 = readlane_i(ka, l);
                  if (hr && don) {
                    const int k = k3 + __popcll(ma & below);
                    if (k < ha_w) __builtin_nontemporal_store(s, &ha_j[(int64_t)i * ha_w + k]);
                  }
                  ka = writelane_i(k3 + __popcll(ma), l, ka);
                }
              }
            }
          }
        }
      };
      if (hasown) centres(std::true_type{});
      else centres(std::false_type{});
    }
    if (lane < mi) {
      const int i = a0 + ig + lane;
      far_cnt[i] = kf;
      if (far_lo) far_lo[i] = klo;
      cnt_cand[i] = kc;
      hb_cnt[i] = kh;
      ha_cnt[i] = ka;
      if (ka > ha_w) atomicMax(&need[4], ka);
      if (kf > far_w) atomicMax(&need[0], kf);
      if (kc > cand_w) atomicMax(&need[1], kc);
      if (kh > hb_w) atomicMax(&need[3], kh);
      tf += (unsigned long long)kf;
      th += (unsigned long long)kh;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    tf += __shfl_down(tf, off, 64);
    th += __shfl_down(th, off, 64);
  }
  if (lane == 0) {
    red[wv][0] = tf;
    red[wv][1] = th;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    unsigned long long v = 0;
    for (int w = 0; w < SWEEP_WAVES; ++w) v += red[w][threadIdx.x];
    if (v) atomicAdd(&tslot[(blockIdx.x & (ESLOT - 1)) * 8 + (threadIdx.x == 0 ? 0 : 4)], v);
  }
}

// bond-order test of each atom's staged candidates, 16 lanes per atom, one
// candidate per lane: a candidate is a bond iff its raw uncorrected bond order
// reaches bo_cut.  Accepted candidates keep their candidate order (numbered
// with the group's ballot).  Workgroups stride over tiles of 16 atoms and
// add their task-list bounds to the three totals once per workgroup.  The
// pair parameters the test reads sit in LDS, and the next tile's atoms,
// counts and first 16 candidates are loaded while this tile is tested, so a
// tile waits on one global load (the candidates' positions) instead of four
// dependent ones.
constexpr int BT_GROUP = 16, BT_BS = 256, BT_TILE = BT_BS / BT_GROUP;

struct BondTestP {
  double r_s, r_p, r_pp, p_bo1, p_bo2, p_bo3, p_bo4, p_bo5, p_bo6, ln_r_s, ln_r_p, ln_r_pp;
};

__global__ __launch_bounds__(BT_BS) void k_bondtest(
    const DevParams* __restrict__ P, Grid g, int64_t n, const double4* __restrict__ xs,
    const int32_t* __restrict__ cnt_cand, const int32_t* __restrict__ cand_j, int cand_w,
    int32_t* __restrict__ cnt_bond, int32_t* __restrict__ bond_t, int bond_w,
    int32_t* __restrict__ need, unsigned long long* __restrict__ tslot, double rb2, int acct) {
  __shared__ unsigned long long red[BT_BS / 64][3];
  __shared__ BondTestP bp[NT * NT];
  for (int t = threadIdx.x; t < NT * NT; t += BT_BS) {
    const PairP& q = P->pair[t];
    bp[t] = BondTestP{q.r_s, q.r_p, q.r_pp, q.p_bo1, q.p_bo2, q.p_bo3, q.p_bo4, q.p_bo5, q.p_bo6,
                      q.ln_r_s, q.ln_r_p, q.ln_r_pp};
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, sub = lane & (BT_GROUP - 1), gsh = lane & ~(BT_GROUP - 1);
  const double bo_cut = P->bo_cut;
  unsigned long long ba = 0, bt = 0, bd = 0;
  const int64_t ntile = (n + BT_TILE - 1) / BT_TILE;
  if (n <= 0) return;
  // the loads of a tile that do not depend on its candidates, made for every
  // lane (atoms past the end read the last atom; rows are cand_w wide, so
  // the first entries exist whatever the count) so that no wait follows them
  double4 xi_n;
  int cnt_n;
  int32_t s_n;
  auto fetch = [&](int64_t tile) {
    int64_t i = tile * BT_TILE + threadIdx.x / BT_GROUP;
    i = i < n ? i : n - 1;
    xi_n = xs[i];
    cnt_n = cnt_cand[i];
    s_n = cand_j[i * (int64_t)cand_w + (sub < cand_w ? sub : 0)];
  };
  int64_t tile = xcd_block();
  fetch(tile);
  for (; tile < ntile; tile += gridDim.x) {
    const int64_t i = tile * BT_TILE + threadIdx.x / BT_GROUP;
    const bool live = i < n;
    const double4 xi = xi_n;
    const int ti = (int)xi.w;
    const int nc = live ? (cnt_n < cand_w ? cnt_n : cand_w) : 0;
    const int32_t s_first = s_n;
    const int32_t* crow = cand_j + (live ? i : 0) * (int64_t)cand_w;
    int32_t* brow = bond_t + (live ? i : 0) * (int64_t)bond_w;
    // the longest candidate row of the wavefront bounds its (uniform) loop
    int ncmax = nc;
    for (int off = BT_GROUP; off < 64; off <<= 1) ncmax = max(ncmax, __shfl_xor(ncmax, off, 64));
    int nb = 0;
    for (int k0 = 0; k0 < ncmax; k0 += BT_GROUP) {
      const int k = k0 + sub;
      const bool in = k < nc;
      const int s = in ? (k0 == 0 ? s_first : crow[k]) : 0;
      const double4 xj = xs[s];
      if (k0 == 0) fetch(tile + gridDim.x);
      bool ok = false;
      if (in) {
        double dx = xj.x - xi.x, dy = xj.y - xi.y, dz = xj.z - xi.z;
        if (g.periodic) {
          dx = min_image(dx, g.L[0], g.invL[0]);
          dy = min_image(dy, g.L[1], g.invL[1]);
          dz = min_image(dz, g.L[2], g.invL[2]);
        }
        const double r2 = r2_of(dx, dy, dz);
        // within r_bond (candidates found with a skin may lie beyond it), and
        // the raw order at the threshold
        ok = r2 <= rb2 && bo_raw(bp[ti * NT + (int)xj.w], sqrt(r2), bo_cut) >= bo_cut;
      }
      const unsigned mask = (unsigned)(ballot(ok) >> gsh) & ((1u << BT_GROUP) - 1u);
      if (ok) {
        const int pos = nb + __popc(mask & ((1u << sub) - 1u));
        if (pos < bond_w) brow[pos] = s;
      }
      nb += __popc(mask);
    }
    if (ncmax == 0) fetch(tile + gridDim.x);
    if (live && sub == 0) {
      cnt_bond[i] = nb;
      if (nb > bond_w) atomicMax(&need[2], nb);
      // bounds of the interaction task lists built from this bond list:
      // angles at i <= C(d,2); torsions about i's bonds <= ceil(d (d-1)^2 / 2)
      // (the sum over bonds of (d_j-1)(d_k-1) is at most half the sum of
      // squares); donor bonds <= d for an H atom
      if (acct) {
        const unsigned long long d = (unsigned long long)nb;
        ba += d * (d > 0 ? d - 1 : 0) / 2;
        bt += (d * (d > 0 ? (d - 1) * (d - 1) : 0) + 1) / 2;
        bd += P->atom[ti].hbond == 1 ? d : 0;
      }
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    ba += __shfl_down(ba, off, 64);
    bt += __shfl_down(bt, off, 64);
    bd += __shfl_down(bd, off, 64);
  }
  if (lane == 0) {
    red[threadIdx.x >> 6][0] = ba;
    red[threadIdx.x >> 6][1] = bt;
    red[threadIdx.x >> 6][2] = bd;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    unsigned long long v = 0;
    for (int w = 0; w < BT_BS / 64; ++w) v += red[w][threadIdx.x];
    if (v) atomicAdd(&tslot[(blockIdx.x & (ESLOT - 1)) * 8 + threadIdx.x + 1], v);
  }
}

// staged bond rows -> compressed rows in increasing partner order, with the
// owner of each entry
__global__ void k_compact(int64_t n, const int32_t* __restrict__ cnt_bond,
                          const int32_t* __restrict__ bond_t, int bond_w,
                          const int32_t* __restrict__ bond_off, int32_t* __restrict__ bond_j,
                          int32_t* __restrict__ bond_i) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int ob = bond_off[i], nb = cnt_bond[i];
  const int32_t* row = bond_t + i * (int64_t)bond_w;
  for (int k = 0; k < nb; ++k) {
    const int v = row[k];
    int t = k - 1;   // insertion into the sorted prefix (rows hold a few bonds)
    while (t >= 0 && bond_j[ob + t] > v) {
      bond_j[ob + t + 1] = bond_j[ob + t];
      --t;
    }
    bond_j[ob + t + 1] = v;
    bond_i[ob + k] = (int32_t)i;
  }
}

// ---------------------------------------------------------------------------
// the partners' halves of the rows of an each-pair-once sweep
// ---------------------------------------------------------------------------
// For each atom i and each of the first cnt[i] entries j of its row in src,
// i is written into j's row of dst from the row's end (lo[j] counts them; an
// entry beyond the width is counted and not written).  GROUP lanes per atom,
// each taking up to four entries at a time so that their atomics are in
// flight together.
template <int GROUP>
__global__ __launch_bounds__(256) void k_transpose(int64_t n, const int32_t* __restrict__ cnt,
                                                   const int32_t* __restrict__ src, int sw,
                                                   int32_t* __restrict__ lo, int32_t* __restrict__ dst, int dw) {
  const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / GROUP;
  const int sub = threadIdx.x & (GROUP - 1);
  if (i >= n) return;
  const int c = min(cnt[i], sw);
  const int32_t* __restrict__ row = src + i * (int64_t)sw;
  for (int k0 = 0; k0 < c; k0 += 4 * GROUP) {
    int j[4], kl[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = k0 + u * GROUP + sub;
      j[u] = k < c ? row[k] : -1;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) kl[u] = j[u] >= 0 ? atomicAdd(&lo[j[u]], 1) : dw;
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (kl[u] < dw) dst[(int64_t)j[u] * dw + (dw - 1 - kl[u])] = (int32_t)i;
  }
}

// Bond rows of an each-pair-once sweep: the partners' entries (written from
// the row's end) moved next to the atom's own, one thread per row (the order
// is fixed when the rows are compacted); the interaction task bounds are
// taken from the full rows (as the bond test does for full sweeps).
__global__ __launch_bounds__(256) void k_merge_bonds(const DevParams* __restrict__ P, int64_t n,
                                                     const double4* __restrict__ xs, int32_t* __restrict__ cnt_bond,
                                                     const int32_t* __restrict__ lo, int32_t* __restrict__ bond_t,
                                                     int bond_w, int32_t* __restrict__ need,
                                                     unsigned long long* __restrict__ tslot) {
  __shared__ unsigned long long red[4][3];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long ba = 0, bt = 0, bd = 0;
  if (i < n) {
    const int cu = cnt_bond[i], cl = lo[i], tot = cu + cl;
    if (tot > bond_w) {
      atomicMax(&need[2], tot);
    } else if (cl > 0) {
      // the entries at [w - cl, w) that lie outside [cu, cu + cl) fill its gap
      int32_t* __restrict__ row = bond_t + i * (int64_t)bond_w;
      const int m = min(cl, bond_w - cl - cu), src0 = max(cu + cl, bond_w - cl);
      for (int k = 0; k < m; ++k) row[cu + k] = row[src0 + k];
    }
    cnt_bond[i] = tot;
    const unsigned long long d = (unsigned long long)tot;
    ba = d * (d > 0 ? d - 1 : 0) / 2;
    bt = (d * (d > 0 ? (d - 1) * (d - 1) : 0) + 1) / 2;
    bd = P->atom[(int)xs[i].w].hbond == 1 ? d : 0;
  }
  for (int off = 32; off > 0; off >>= 1) {
    ba += __shfl_down(ba, off, 64);
    bt += __shfl_down(bt, off, 64);
    bd += __shfl_down(bd, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6][0] = ba;
    red[threadIdx.x >> 6][1] = bt;
    red[threadIdx.x >> 6][2] = bd;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    unsigned long long v = 0;
    for (int w = 0; w < 4; ++w) v += red[w][threadIdx.x];
    if (v) atomicAdd(&tslot[(blockIdx.x & (ESLOT - 1)) * 8 + threadIdx.x + 1], v);
  }
}

// mirror entry: position of i in the bond list of j (one thread per entry)
__global__ void k_mirror(int64_t nbond, const int32_t* __restrict__ off, const int32_t* __restrict__ bj,
                         const int32_t* __restrict__ bi, int32_t* __restrict__ mir, int32_t* __restrict__ flag) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= nbond) return;
  const int i = bi[e], j = bj[e];
  int m = -1;
  for (int f = off[j]; f < off[j + 1]; ++f)
    if (bj[f] == i) { m = f; break; }
  // the bond predicate is symmetric, so the partner entry exists; should it
  // not, point at the entry itself and raise the flag rather than index -1
  if (m < 0) {
    atomicOr(flag, 2);
    m = (int)e;
  }
  mir[e] = m;
}

// export helpers: lists in caller indices
// half far list from the full rows: the entries with j > i, at per-atom
// offsets hoff (exclusive scan of the per-atom half counts).  Slot entries are
// mapped back to sorted indices by walking the chunk sequence of the window of
// the atom's run along the (increasing) row.
template <bool WRITE>
__global__ void k_export_far(int64_t n, Grid g, const int32_t* __restrict__ cstart,
                             const int32_t* __restrict__ cell_s, const int32_t* __restrict__ cnt,
                             const int32_t* __restrict__ fj, int far_w, int slots, int upper,
                             const int32_t* __restrict__ perm, int32_t* __restrict__ hcnt,
                             const int64_t* __restrict__ hoff, int32_t* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t o = WRITE ? hoff[i] : 0;
  int h = 0;
  const int pi = WRITE ? perm[i] : 0;
  const int32_t* row = fj + i * (int64_t)far_w;
  const int c = slots ? cell_s[i] : 0, nq = stencil_chunks(g);
  int q = 0, s0 = 0, s1 = 0, base = 0;
  double sx, sy, sz;
  if (slots) window_chunk(g, cstart, c, 0, s0, s1, sx, sy, sz);
  for (int k = 0; k < cnt[i]; ++k) {
    int j = row[k];
    if (slots) {
      while (j >= base + (s1 - s0) && q + 1 < nq) {
        base += s1 - s0;
        window_chunk(g, cstart, c, ++q, s0, s1, sx, sy, sz);
      }
      j = s0 + (j - base);
    }
    if (upper || j > (int)i) {   // upper rows hold each pair once
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

// H rows -> (h, z) pairs at offsets hoff
__global__ void k_export_rows(int64_t n, const int32_t* __restrict__ cnt, const int32_t* __restrict__ rows,
                              int w, const int64_t* __restrict__ off, const int32_t* __restrict__ perm,
                              int32_t* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int pi = perm[i];
  int64_t o = off[i];
  for (int k = 0; k < cnt[i]; ++k) {
    out[2 * o] = pi;
    out[2 * o + 1] = perm[rows[i * (int64_t)w + k]];
    ++o;
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

// the sweep's and bond test's partial totals and need[5] maxima, folded
__global__ void k_fold_totals(const unsigned long long* __restrict__ tslot, const int32_t* __restrict__ nslot,
                              unsigned long long* __restrict__ totals, int32_t* __restrict__ need) {
  const int t = threadIdx.x;
  if (t < 8) {
    unsigned long long v = 0;
    for (int k = 0; k < ESLOT; ++k) v += tslot[k * 8 + t];
    totals[t] += v;
  } else if (t == 8) {
    int m = need[5];
    for (int k = 0; k < ESLOT; ++k) m = nslot[k] > m ? nslot[k] : m;
    need[5] = m;
  }
}

int launch_sweep(const DevParams* P, const Grid& g, int64_t n, int ncell, double rb2, bool half, Scratch& sc,
                 Lists& L, Prof& pf, hipStream_t st) {
  if (stencil_chunks(g) > SWEEP_MAXQ) return -1;   // the sweep's chunk table
  // each pair once: upper rows of stencil slots, no dimension covered whole
  half = half && L.far_upper && L.far_slots && !g.full[0] && !g.full[1] && !g.full[2];
  (void)hipMemsetAsync(sc.need, 0, sizeof(int32_t) * 8, st);
  (void)hipMemsetAsync(sc.totals, 0, sizeof(int64_t) * 8, st);
  (void)hipMemsetAsync(sc.tslot, 0, sizeof(int64_t) * 8 * ESLOT, st);
  (void)hipMemsetAsync(sc.nslot, 0, sizeof(int32_t) * ESLOT, st);
  sc.half = half;
  pf.begin(KID_LIST_SWEEP, st);
  auto sweep = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3(nblk(ncell, SWEEP_WAVES)), dim3(64 * SWEEP_WAVES), 0, st, P, g, ncell, L.xs,
                       L.cell_start, L.far_cnt, L.far_j, L.far_w, sc.cnt_cand, sc.cand_j, sc.cand_w, L.hb_cnt,
                       L.hb_j, L.hb_w, L.ha_cnt, L.ha_j, L.ha_w, L.far_slots,
                       L.far_slots ? L.far_lo : nullptr, sc.need,
                       reinterpret_cast<unsigned long long*>(sc.tslot), sc.nslot);
  };
  const bool minimg = g.periodic && !g.shift_ok;
  if (minimg) {
    if (half) sweep(k_sweep<true, true, true>);
    else if (L.far_upper) sweep(k_sweep<true, true, false>);
    else sweep(k_sweep<true, false, false>);
  } else {
    if (half) sweep(k_sweep<false, true, true>);
    else if (L.far_upper) sweep(k_sweep<false, true, false>);
    else sweep(k_sweep<false, false, false>);
  }
  pf.end(st);
  return launch_bondtest(P, g, n, rb2, sc, L, pf, st);
}

int launch_bondtest(const DevParams* P, const Grid& g, int64_t n, double rb2, Scratch& sc, Lists& L, Prof& pf,
                    hipStream_t st) {
  pf.begin(KID_BONDTEST, st);
  hipLaunchKernelGGL(k_bondtest, dim3(xcd_grid(std::min<int64_t>(nblk(n, BT_TILE), 4096))), dim3(BT_BS), 0, st,
                     P, g, n, L.xs, sc.cnt_cand,
                     sc.cand_j, sc.cand_w, sc.cnt_bond, sc.bond_t, sc.bond_w, sc.need,
                     reinterpret_cast<unsigned long long*>(sc.tslot), rb2, sc.half ? 0 : 1);
  pf.end(st);
  if (sc.half) {
    pf.begin(KID_BOND_MERGE, st);
    // candidates were each pair once, so are the bonds: each atom's bonds
    // go to its partners' rows too
    (void)hipMemsetAsync(sc.cnt_lo, 0, sizeof(int32_t) * n, st);
    constexpr int BG = 2;
    hipLaunchKernelGGL(k_transpose<BG>, dim3(nblk(n * BG, 256)), dim3(256), 0, st, n, sc.cnt_bond, sc.bond_t,
                       sc.bond_w, sc.cnt_lo, sc.bond_t, sc.bond_w);
    hipLaunchKernelGGL(k_merge_bonds, dim3(nblk(n, 256)), dim3(256), 0, st, P, n, L.xs, sc.cnt_bond, sc.cnt_lo,
                       sc.bond_t, sc.bond_w, sc.need, reinterpret_cast<unsigned long long*>(sc.tslot));
    pf.end(st);
  }
  hipLaunchKernelGGL(k_fold_totals, dim3(1), dim3(64), 0, st, reinterpret_cast<const unsigned long long*>(sc.tslot), sc.nslot,
                     reinterpret_cast<unsigned long long*>(sc.totals), sc.need);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// positions of the sorted layout from the caller's (the order fixed at the
// last build), and the largest squared displacement since then (as the
// order-preserving bits of a non-negative double)
__global__ void k_refresh_gather(const double* __restrict__ pos, const int32_t* __restrict__ perm, int64_t n,
                                 const double4* __restrict__ xref, double4* __restrict__ xs,
                                 unsigned long long* __restrict__ dmax) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  double d2 = 0.0;
  if (s < n) {
    const int i = perm[s];
    const double4 r = xref[s];
    const double x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
    xs[s] = make_double4(x, y, z, r.w);
    d2 = (x - r.x) * (x - r.x) + (y - r.y) * (y - r.y) + (z - r.z) * (z - r.z);
    if (!(d2 <= 1e300)) d2 = 1e300;   // non-finite: forces a rebuild, which reports it
  }
  for (int off = 32; off > 0; off >>= 1) d2 = fmax(d2, __shfl_down(d2, off, 64));
  if ((threadIdx.x & 63) == 0 && d2 > 0.0) atomicMax(dmax, (unsigned long long)__double_as_longlong(d2));
}

int launch_refresh_gather(const double* pos, int64_t n, const double4* xref, Lists& L, unsigned long long* dmax,
                          Prof& pf, hipStream_t st) {
  pf.begin(KID_GATHER, st);
  if (n > 0)
    hipLaunchKernelGGL(k_refresh_gather, dim3(nblk(n, 256)), dim3(256), 0, st, pos, L.perm, n, xref, L.xs, dmax);
  pf.end(st);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_compact(int64_t n, Scratch& sc, Lists& L, Prof& pf, hipStream_t st) {
  pf.begin(KID_COMPACT, st);
  hipLaunchKernelGGL(k_compact, dim3(nblk(n, 256)), dim3(256), 0, st, n, sc.cnt_bond, sc.bond_t,
                     sc.bond_w, L.bond_off, L.bond_j, L.bond_i);
  pf.end(st);
  pf.begin(KID_MIRROR, st);
  hipLaunchKernelGGL(k_mirror, dim3(nblk(std::max<int64_t>(L.nbond, 1), 256)), dim3(256), 0, st, L.nbond,
                     L.bond_off, L.bond_j, L.bond_i, L.bond_mir, sc.flag);
  pf.end(st);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_export(const Grid& g, const Lists& L, int32_t* far, int32_t* bonds, int32_t* hb, Scratch& sc,
                  hipStream_t st) {
  const int64_t n = L.n;
  int32_t* hcnt = nullptr;
  int64_t* hoff = nullptr;
  if (hipMalloc(&hcnt, sizeof(int32_t) * (n + 1)) != hipSuccess) return -1;
  if (hipMalloc(&hoff, sizeof(int64_t) * (n + 1)) != hipSuccess) return -1;
  if (far) {
    (void)hipMemsetAsync(hcnt + n, 0, sizeof(int32_t), st);
    hipLaunchKernelGGL(k_export_far<false>, dim3(nblk(n, 256)), dim3(256), 0, st, n, g, L.cell_start,
                       sc.cell_s, L.far_cnt, L.far_j, L.far_w, L.far_slots, L.far_upper, L.perm, hcnt, nullptr,
                       nullptr);
    scan_i32_to_i64(hcnt, hoff, n + 1, sc, st);
    hipLaunchKernelGGL(k_export_far<true>, dim3(nblk(n, 256)), dim3(256), 0, st, n, g, L.cell_start,
                       sc.cell_s, L.far_cnt, L.far_j, L.far_w, L.far_slots, L.far_upper, L.perm, nullptr, hoff, far);
  }
  if (bonds)
    hipLaunchKernelGGL(k_export_csr, dim3(nblk(n, 256)), dim3(256), 0, st, n, L.bond_off, L.bond_j,
                       L.perm, bonds);
  if (hb) {
    (void)hipStreamSynchronize(st);
    (void)hipMemcpyAsync(hcnt, L.hb_cnt, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, st);
    (void)hipMemsetAsync(hcnt + n, 0, sizeof(int32_t), st);
    scan_i32_to_i64(hcnt, hoff, n + 1, sc, st);
    hipLaunchKernelGGL(k_export_rows, dim3(nblk(n, 256)), dim3(256), 0, st, n, L.hb_cnt, L.hb_j,
                       L.hb_w, hoff, L.perm, hb);
  }
  (void)hipStreamSynchronize(st);
  (void)hipFree(hcnt);
  (void)hipFree(hoff);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace rx
