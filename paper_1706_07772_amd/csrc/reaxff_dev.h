// Device-side data layout and helpers of the gfx950 ReaxFF library.
//
// Everything runs in "sorted" atom order: atoms are counting-sorted by cell
// so that spatial neighbours are neighbours in memory (the spatially reordered
// atom list the paper relies on in Section 3.2, made explicit).  The caller's
// order is restored only when forces are written out.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/reaxff.h"

namespace rx {

constexpr int NT = REAXFF_NTYPES;
constexpr int NTERMS = REAXFF_NTERMS;
enum Term { E_BOND, E_LP, E_OVER, E_UNDER, E_VAL, E_PEN, E_COA, E_TOR, E_CONJ, E_HB, E_VDW, E_COUL };

constexpr double C_ELE = 332.06371;      // kcal A / (mol e^2)
constexpr double ACC_CONV = 4.184e-4;    // (kcal/mol/A) / (g/mol) -> A/fs^2
constexpr double PI = 3.14159265358979323846;

// per element pair, with derived constants the kernels need
struct PairP {
  double r_s, r_p, r_pp;            // mixed bond radii (<= 0: component off)
  double p_bo1, p_bo2, p_bo3, p_bo4, p_bo5, p_bo6;
  double D_s, D_p, D_pp, p_be1, p_be2, p_ovun1;
  double p_boc3, p_boc4, p_boc5;
  double D_vdw, alpha, inv_r_vdw, gw_pow;  // gw_pow = gamma_w^(-p_vdW1)
  double g3;                                // gamma^(-3)
  double e_core, a_core, inv_r_core;
  double reach2;                            // bond prefilter: raw BO' < bo_cut beyond it
  double ln_r_s, ln_r_p, ln_r_pp;           // logs of the bond radii (0 when off)
  double pad[2];
};

struct AtomP {
  double val, val_e, val_boc, val_ang, mass, p_lp2, p_ovun2, p_ovun5, p_val3, p_val5;
  double nlp_opt;
  int32_t hbond;  // 0 none, 1 donor H, 2 acceptor
  int32_t pad;
};

struct AngleP { double theta00_rad, p_val1, p_val2, p_val4, p_val7, p_pen1, p_coa1, pad; };
struct TorsP { double V1, V2, V3, p_tor1, p_cot1, pad0, pad1, pad2; };
struct HbP { double r0hb, p_hb1, p_hb2, p_hb3; };

struct DevParams {
  double p_boc1, p_boc2, p_coa2, p_coa3, p_coa4, p_ovun3, p_ovun4, p_ovun6, p_ovun7, p_ovun8,
      p_val6, p_val8, p_val9, p_val10, p_pen2, p_pen3, p_pen4, p_tor2, p_tor3, p_tor4, p_cot2,
      p_vdW1, p_lp1, inv_p_vdW1;
  double r_nonb, r_bond, r_hb, bo_cut, thb_cut, thb_cutsq, hb_bo_cut;
  double rn2, rh2, inv_r_nonb;
  AtomP atom[NT];
  PairP pair[NT * NT];
  AngleP angle[NT * NT * NT];
  TorsP tors[NT * NT * NT * NT];
  HbP hb[NT * NT * NT];
};

// geometry of the cell grid (sorted layout)
struct Grid {
  int periodic;
  int nc[3];        // cells per dimension
  int reach;        // stencil half-width in cells (1 or 2)
  int span[3];      // distinct stencil offsets per dimension (2 reach + 1, or nc when fewer)
  int full[3];      // 1: iterate every cell in this dimension
  double lo[3];     // origin (0 for periodic)
  double L[3], invL[3];
  double invw[3];   // 1 / cell width
  // 1 when every position lies in [0, L) and every dimension has at least
  // 2 reach + 3 cells: then any pair within r_nonb of a stencil column has the column's
  // image shift as its minimum image, and d - shift is bit-identical to
  // d - L rint(d / L)
  int shift_ok;
  // cells per run: the cells of a column are grouped into runs of `run`
  // consecutive z cells, and far-row slots number the window of the centre's
  // run (its stencil columns over the run's z cells and reach on either side)
  // instead of the centre cell's own stencil; 1: the cell's own stencil.
  // Greater than 1 only with no dimension covered whole and, in a periodic
  // box, run + 2 reach <= nc[2].
  int run;
};

// --- lists and work arrays (device pointers, owned by the context) -------
struct Lists {
  int64_t n;
  // sorted layout
  int32_t* perm;        // sorted slot -> caller index
  int32_t* type_s;      // sorted types
  double4* xs;          // sorted positions, w = type (as a double)
  int32_t* cell_start;  // [ncell + 1]
  // far-neighbour list, full (both directions of every pair), one row of
  // width far_w per atom: entry k of atom i is far_j[i * far_w + k], in
  // increasing order.  With far_slots set an entry is the neighbour's slot:
  // its position in the chunk sequence of the window of i's run
  // (window_chunk; with Grid::run = 1 the stencil of i's cell), which is also
  // its place in the staged copy of that window; otherwise it is the
  // neighbour's sorted index.
  int32_t* far_cnt;     // [n]
  int32_t* far_j;
  int32_t far_w;
  int32_t far_slots;
  // half evaluation of the nonbonded term (slot form, no dimension covered
  // whole, every run's upper window within NB_HALF_CAP atoms): far_lo[i]
  // entries of row i precede i's own slot; the pairs of the rest of the row
  // are evaluated by i's run, the others by the partner's run
  int32_t* far_lo;      // [n]
  // far_upper: rows hold only the entries after the centre's own slot, so
  // each pair appears once, in the row of the atom whose run evaluates it
  // (far_lo is then 0).  Set when the half evaluation is expected; a build
  // that finds it impossible sweeps again with full rows.
  int32_t far_upper;
  int32_t nb_half;
  int32_t* cell_of;     // [n] cell of each sorted atom
  // full bond list
  int32_t* bond_off;    // [n + 1]
  int32_t* bond_j;
  int32_t* bond_i;      // owner atom of each entry
  int32_t* bond_mir;
  // H list, one row of width hb_w per atom (rows of non-H atoms are empty)
  int32_t* hb_cnt;      // [n]
  int32_t* hb_j;
  int32_t hb_w;
  // the same relation seen from the acceptor: donors H within r_hb of each
  // acceptor (rows of non-acceptors are empty)
  int32_t* ha_cnt;      // [n]
  int32_t* ha_j;
  int32_t ha_w;
  // the far and H lists are supersets built with a skin (Verlet lists kept
  // over several steps): the force kernels apply the exact cutoffs themselves
  int32_t cut_check;
  int64_t nfar;         // unordered pairs (half the entries)
  int64_t nbond, nhb;
  // upper bounds on the interaction task lists (from the bond degrees)
  int64_t bound_ang, bound_tor, bound_don;
};

// per-atom state of the bond-order stage
struct AtomState {
  double S, Delta, Dang, Dlp;   // total bond order, deviations, lone-pair deficit
  double dnlp;                  // d nlp / d S
  double SBO2, dSBO2;           // SBO2 and dSBO2/dSBO
  double prod, W, dW;           // prod_e exp(-BO^8), W = -Dang - p_val8 vlpadj, dW/dS
  // angle-centre factors: 1 - e^{-p_val10 (2 - SBO2)} and its SBO2 derivative,
  // e^{p_val6 Dang}, penalty f9 and d f9/d Delta, coalition 1/(1+e^{p_coa2 Dang})
  // and its Dang derivative
  double th0f, dth0f, e6, f9, df9, fc, dfc;
  double pad[3];
};

// a donor bond h->X as the acceptor side of the hydrogen-bond term reads it
struct DonRec {
  double4 bd;        // x_X - x_h and its length
  double bo;         // corrected bond order
  int32_t X, tX;     // donor atom and its type
};

// atoms of a run's upper window (the centre column from the run's first atom
// on, and every later chunk) that the half nonbonded kernel holds in LDS
constexpr int NB_HALF_CAP = 2560;
// chunk-table entries per run: 2 (2 reach + 1)^2 <= 50 chunks and the total
constexpr int NB_QMAX = 64;

struct Work {
  // per directed bond entry
  double4* bd;     // (dx, dy, dz, r): x_j - x_i
  double4* bop;    // uncorrected (sigma shifted, pi, pipi, total)
  double4* dbop;   // d/dr of sigma, pi, pipi
  double4* bo;     // corrected (BO, BOpi, BOpipi, BOsigma)
  double4* gbo;    // adjoints (BO, BOpi, BOpipi, S of the outer atom of an angle)
  double4* gvec;   // vector adjoint dE/d(x_j - x_i)
  double4* gup;    // adjoints of uncorrected (total, pi, pipi) and Delta' part of own atom
  // per atom
  double2* dp;     // (Delta', Delta'boc)
  AtomState* ast;
  double* gS;      // dE/dS (direct terms)
  double* gSig;    // dE/dSigma_pi of the over/under term
  double* gRso;    // R so of the over-coordination term (its bond-order factor)
  double* gSBO;    // dE/dSBO
  double* gStot;   // dE/dS including gathered cross-atom terms
  double* gDp;     // dE/dDelta' (sum over own bonds)
  double4* fnb;    // nonbonded forces
  double4* fhb;    // hydrogen-bond forces on H (atomics) and on acceptors
  double4* xq;     // sorted positions with charge in w
  unsigned long long* counters;  // [0] angles [1] torsions [2] hbonds
  // interaction task lists: per-owner counts, exclusive sums, flat tasks
  // per bond entry u (owner j = bond_i[u]); an atom's tasks start at the
  // offset of its first entry, off[bond_off[j]]
  int32_t* cnt_ang;  // [nbond + 1] valence angles (u, v > u) centred on j
  int32_t* cnt_tor;  // [nbond + 1] torsions about the central bond u = j->k, k > j
  int32_t* cnt_don;  // [nbond + 1] donor bond u = H->X (0 or 1)
  int32_t* off_ang;
  int32_t* off_tor;
  int32_t* off_don;
  int2* ang;         // (entry j->i, entry j->k)
  int4* tor;         // (entry j->k, entry j->i, entry k->l, unused)
  int32_t* don;      // entry h->X
  DonRec* donrec;    // per donor task: what the acceptor side reads of h->X
  int2* don_rng;     // [n] each atom's donor tasks [x, y)
  // [ESLOT][NTERMS] energy partial sums: each workgroup adds its per-term
  // sums to slot (block mod ESLOT), so no single address takes one atomic
  // per workgroup of a large grid; folded into the energies at the end
  double* epart;
  // [nbond] corrected total bond order BO alone (the .x of bo), for the
  // kernels that only test or scale by it; null: read bo[e].x
  double* bo1;
  // [n] what other atoms' terms read of atom j, in one 32-byte record:
  // (S, Delta - Dlp, Dang, prod W); null: read from ast
  double4* nv;
  int64_t cap_ang, cap_tor, cap_don;
  // half nonbonded evaluation: per-run partial forces on the upper window
  // ([run][NB_HALF_CAP][3]) and per-run chunk bases relative to the run's
  // first atom ([run][NB_QMAX])
  double* nbpart;
  int32_t* nbtab;
  int64_t cap_nbpart, cap_nbtab;
  // per-run nonbonded energies (van der Waals, Coulomb), summed by a small
  // reduction instead of one pair of same-address atomics per run
  double2* nbe;
  int64_t cap_nbe;
};

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ double sqr(double x) { return x * x; }

// minimum-image displacement x_j - x_i, rounded exactly as the plain
// definition spells it: d = xj - xi; d -= L * rint(d * invL)
__device__ __forceinline__ double min_image(double d, double L, double invL) {
#pragma clang fp contract(off)
  const double s = L * rint(d * invL);
  return d - s;
}

// broadcast lane l's value to the whole wavefront (l uniform)
__device__ __forceinline__ double readlane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ int readlane_i(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

// lanes of the wavefront whose predicate holds (taken straight from the
// compare's lane mask)
__device__ __forceinline__ unsigned long long ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// DPP move of a double (both 32-bit halves): lanes whose source lies outside
// the row, and rows outside ROWMASK, read 0
template <int CTRL, int ROWMASK = 0xF>
__device__ __forceinline__ double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROWMASK, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWMASK, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over each aligned group of four lanes, in every lane of the group
// (quad permutations [1,0,3,2] and [2,3,0,1]); all four lanes must be active.
__device__ __forceinline__ double quad_sum(double v) {
  v += dpp_d<0xB1>(v);
  v += dpp_d<0x4E>(v);
  return v;
}

// Sum over each group of 8 lanes, left in the group's last lane (7, 15, ...):
// row shifts by 1, 2, 4 (lanes shifted in from before a 16-lane row read 0);
// every lane of a group must be active.
__device__ __forceinline__ double oct_sum_last(double v) {
  v += dpp_d<0x111>(v);          // row_shr:1
  v += dpp_d<0x112>(v);          // row_shr:2
  v += dpp_d<0x114>(v);          // row_shr:4
  return v;
}

// Sum over each 16-lane row, left in the row's last lane (15, 31, 47, 63);
// every lane of a row must be active.
__device__ __forceinline__ double row_sum_last(double v) {
  v += dpp_d<0x111>(v);          // row_shr:1
  v += dpp_d<0x112>(v);          // row_shr:2
  v += dpp_d<0x114>(v);          // row_shr:4
  v += dpp_d<0x118>(v);          // row_shr:8
  return v;
}

// lane l takes the (uniform) value v, the other lanes keep old
__device__ __forceinline__ int writelane_i(int v, int l, int old) {
  asm("v_writelane_b32 %0, %1, m0" : "+v"(old) : "s"(v), "{m0}"(l));
  return old;
}

// Work-group order for kernels over cell-sorted data.  The hardware deals
// work-groups to the 8 XCDs round-robin; giving work-group b the logical index
// (b mod 8) * (grid / 8) + b / 8, on a grid padded to a multiple of 8, lets
// each XCD walk one contiguous range of atoms (a slab of the box), so the
// neighbour data its work-groups gather stays in that XCD's L2.
constexpr int NXCD = 8;
__host__ __device__ __forceinline__ unsigned xcd_grid(int64_t nblocks) {
  const int64_t b = nblocks < 1 ? 1 : nblocks;
  return (unsigned)(NXCD * ((b + NXCD - 1) / NXCD));
}
__device__ __forceinline__ int64_t xcd_block() {
  return (int64_t)(blockIdx.x % NXCD) * (gridDim.x / NXCD) + blockIdx.x / NXCD;
}

// Blocks over work whose size A is known only on the device, on a grid sized
// by an upper bound (a multiple of NXCD blocks, at least A): XCD k takes the
// contiguous active blocks [k ceil(A/NXCD), (k+1) ceil(A/NXCD)), so each
// XCD's L2 sees one region of the cell-sorted data and every XCD gets an
// equal share.  -1: no work for this block.
__device__ __forceinline__ int64_t xcd_active_block(int64_t A) {
  const int64_t per = (A + NXCD - 1) / NXCD;
  const int64_t j = blockIdx.x / NXCD;
  const int64_t a = (int64_t)(blockIdx.x % NXCD) * per + j;
  return j < per && a < A ? a : -1;
}

__device__ __forceinline__ double r2_of(double dx, double dy, double dz) {
  return fma(dz, dz, fma(dy, dy, dx * dx));
}

// z ranges of a stencil column around cell z = c2, in cell units within a
// row: [za0, za1) and [zb0, zb1).  Cells are numbered with z fastest, so the
// 2R+1 cells of a column (x, y, c2-R..c2+R, R = g.reach) are one contiguous
// range of sorted atoms, or two when the column wraps around a periodic edge.
__device__ __forceinline__ void column_ranges(const Grid& g, int c2, int& za0, int& za1, int& zb0,
                                              int& zb1) {
  const int R = g.reach;
  zb0 = zb1 = 0;
  if (g.full[2]) {
    za0 = 0; za1 = g.nc[2];
  } else if (g.periodic) {
    if (c2 - R < 0) { za0 = 0; za1 = c2 + R + 1; zb0 = g.nc[2] + c2 - R; zb1 = g.nc[2]; }
    else if (c2 + R >= g.nc[2]) { za0 = c2 - R; za1 = g.nc[2]; zb0 = 0; zb1 = c2 + R + 1 - g.nc[2]; }
    else { za0 = c2 - R; za1 = c2 + R + 1; }
  } else {
    za0 = c2 - R < 0 ? 0 : c2 - R;
    za1 = c2 + R + 1 > g.nc[2] ? g.nc[2] : c2 + R + 1;
  }
}

// The same z ranges for the window of the run holding cell z = c2: the run's
// cells [z0, z1) and reach cells on either side.
__device__ __forceinline__ void window_ranges(const Grid& g, int c2, int& za0, int& za1, int& zb0,
                                              int& zb1) {
  if (g.run <= 1 || g.full[2]) {
    column_ranges(g, c2, za0, za1, zb0, zb1);
    return;
  }
  const int R = g.reach, nz = g.nc[2];
  const int z0 = c2 / g.run * g.run, z1 = z0 + g.run < nz ? z0 + g.run : nz;
  zb0 = zb1 = 0;
  if (g.periodic) {
    if (z0 - R < 0) { za0 = 0; za1 = z1 + R; zb0 = nz + z0 - R; zb1 = nz; }
    else if (z1 + R > nz) { za0 = z0 - R; za1 = nz; zb0 = 0; zb1 = z1 + R - nz; }
    else { za0 = z0 - R; za1 = z1 + R; }
  } else {
    za0 = z0 - R < 0 ? 0 : z0 - R;
    za1 = z1 + R > nz ? nz : z1 + R;
  }
}

// The stencil of cell c as a fixed sequence of chunks of contiguous sorted
// atoms: chunk q (0 <= q < stencil_chunks) is column (a, b) = ((q/2) / span1,
// (q/2) % span1) of the (x, y) stencil; within a column the z range at
// negative offsets comes first: the wrapped range, then the unwrapped one,
// when the column wraps below the cell (c2 < reach), otherwise the unwrapped
// range, then the wrapped one.  A chunk is empty when its column lies
// outside a non-periodic grid or has no wrapped part.  (sx, sy, sz) is the
// chunk's image shift.  Far-list entries number a neighbour by its position
// in this sequence, so the order is part of the list format.  When no
// dimension is covered whole, the sequence runs through the stencil in
// increasing (x, y, z) offset order except inside z ranges, so a neighbour
// at a lexicographically positive offset, or in the centre's own cell after
// it, has a larger slot than the centre itself.
__host__ __device__ __forceinline__ int stencil_chunks(const Grid& g) { return 2 * g.span[0] * g.span[1]; }

template <bool WIN>
__device__ __forceinline__ void chunk_range(const Grid& g, const int32_t* __restrict__ cstart, int c, int q,
                                            int& s0, int& s1, double& sx, double& sy, double& sz) {
  const int c2 = c % g.nc[2], c1 = (c / g.nc[2]) % g.nc[1], c0 = c / (g.nc[1] * g.nc[2]);
  const int col = q >> 1, a = col / g.span[1], bb = col % g.span[1];
  s0 = s1 = 0;
  sx = sy = sz = 0.0;
  int x = g.full[0] ? a : c0 + a - g.reach;
  if (g.periodic) {
    if (x < 0) { x += g.nc[0]; sx = g.L[0]; }
    else if (x >= g.nc[0]) { x -= g.nc[0]; sx = -g.L[0]; }
  } else if (x < 0 || x >= g.nc[0]) return;
  int y = g.full[1] ? bb : c1 + bb - g.reach;
  if (g.periodic) {
    if (y < 0) { y += g.nc[1]; sy = g.L[1]; }
    else if (y >= g.nc[1]) { y -= g.nc[1]; sy = -g.L[1]; }
  } else if (y < 0 || y >= g.nc[1]) return;
  int za0, za1, zb0, zb1;
  if constexpr (WIN) window_ranges(g, c2, za0, za1, zb0, zb1);
  else column_ranges(g, c2, za0, za1, zb0, zb1);
  // the cell whose reach decides which side wraps: the run's first for a window
  const int zc = WIN && g.run > 1 ? c2 / g.run * g.run : c2;
  const int row = (x * g.nc[1] + y) * g.nc[2];
  const bool wrap_first = zb1 > zb0 && zc - g.reach < 0;
  if (((q & 1) == 0) != wrap_first) {
    s0 = cstart[row + za0];
    s1 = cstart[row + za1];
  } else if (zb1 > zb0) {
    s0 = cstart[row + zb0];
    s1 = cstart[row + zb1];
    sz = zc - g.reach < 0 ? g.L[2] : -g.L[2];
  }
}
// chunk q of cell c's own stencil (the candidates of its atoms)
__device__ __forceinline__ void stencil_chunk(const Grid& g, const int32_t* __restrict__ cstart, int c, int q,
                                              int& s0, int& s1, double& sx, double& sy, double& sz) {
  chunk_range<false>(g, cstart, c, q, s0, s1, sx, sy, sz);
}
// runs of the grid (Grid::run consecutive z cells of one column; the last
// run of a column may be shorter) and the cells of run r: first cell, count
__host__ __device__ __forceinline__ int run_rows(const Grid& g) { return (g.nc[2] + g.run - 1) / g.run; }
__device__ __forceinline__ void run_cells(const Grid& g, int r, int& cfirst, int& nk) {
  const int nrz = run_rows(g), rz = r % nrz, col = r / nrz;
  cfirst = col * g.nc[2] + rz * g.run;
  nk = g.nc[2] - rz * g.run < g.run ? g.nc[2] - rz * g.run : g.run;
}

// chunk q of the window of c's run (the numbering of far-row slots): the same
// columns and order over the run's z ranges; every chunk of a cell's stencil
// lies inside the window's chunk of the same column and side, so slots keep
// their order
__device__ __forceinline__ void window_chunk(const Grid& g, const int32_t* __restrict__ cstart, int c, int q,
                                             int& s0, int& s1, double& sx, double& sy, double& sz) {
  chunk_range<true>(g, cstart, c, q, s0, s1, sx, sy, sz);
}

// The runs whose upper window (the half evaluation's LDS copy: the centre
// column from the run's first atom on, and every later chunk) holds atom j of
// cell cj, and j's staged index t there: visit(r, t) for each.  Those are the
// runs of the cells z - oz of the columns at offsets (ox, oy) = column(j) -
// column(run) with (ox, oy) lexicographically positive (oz in [-R, R]), or
// ox = oy = 0 (oz in [0, R]: the window's upper part starts at the run's
// first cell).  In the run's chunk sequence j lies in column (ox, oy) and in
// that column's unwrapped or wrapped z range, chunk q; its staged index is
// tab[r NB_QMAX + q] + j (an empty run's offsets put every atom out of range).
// R: the stencil reach.
template <int R, class F>
__device__ __forceinline__ void for_upper_windows(const Grid& g, int cj, const int32_t* __restrict__ tab, int j,
                                                  F&& visit) {
  const int nrz = run_rows(g);
  const int jz = cj % g.nc[2], jy = (cj / g.nc[2]) % g.nc[1], jx = cj / (g.nc[1] * g.nc[2]);
  // the runs of the cells jz - oz, oz in [-R, R] (the same in every column):
  // their z index, the side of their window holding j (chunk 2 col + side)
  // and whether one of those cells has oz >= 0 (the centre column's upper part)
  int nr = 0, rzs[2 * R + 1], side[2 * R + 1];
  bool up[2 * R + 1];
  {
    int last = -1;
#pragma unroll
    for (int oz = -R; oz <= R; ++oz) {
      int cz = jz - oz;
      if (cz < 0 || cz >= g.nc[2]) {
        if (!g.periodic) continue;
        cz += cz < 0 ? g.nc[2] : -g.nc[2];
      }
      const int rz = cz / g.run;
      if (rz == last) {   // cells of one run follow each other
        up[nr - 1] = up[nr - 1] || oz >= 0;
        continue;
      }
      last = rz;
      const int z0 = rz * g.run;
      int za0, za1, zb0, zb1;
      window_ranges(g, z0, za0, za1, zb0, zb1);
      const bool in_a = jz >= za0 && jz < za1;
      const bool wrap_first = zb1 > zb0 && z0 - R < 0;
      rzs[nr] = rz;
      side[nr] = (in_a != wrap_first) ? 0 : 1;
      up[nr] = oz >= 0;
      ++nr;
    }
  }
  for (int ox = 0; ox <= R; ++ox) {
    int cx = jx - ox;
    if (cx < 0) {
      if (!g.periodic) continue;
      cx += g.nc[0];
    }
    for (int oy = ox == 0 ? 0 : -R; oy <= R; ++oy) {
      int cy = jy - oy;
      if (cy < 0 || cy >= g.nc[1]) {
        if (!g.periodic) continue;
        cy += cy < 0 ? g.nc[1] : -g.nc[1];
      }
      const int col = (ox + R) * g.span[1] + (oy + R);
      const int64_t rcol = (int64_t)(cx * g.nc[1] + cy) * nrz;
      const bool own = ox == 0 && oy == 0;
#pragma unroll
      for (int k = 0; k < 2 * R + 1; ++k) {
        if (k >= nr || (own && !up[k])) continue;
        const int64_t r = rcol + rzs[k];
        const int t = tab[r * NB_QMAX + 2 * col + side[k]] + j;
        if ((unsigned)t >= (unsigned)NB_HALF_CAP) continue;   // an empty run
        visit(r, t);
      }
    }
  }
}

// largest k in [0, n) with b[k] <= t, for non-decreasing b with b[0] <= t
__device__ __forceinline__ int last_le(const int* b, int n, int t) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (b[mid] <= t) lo = mid;
    else hi = mid;
  }
  return lo;
}

// inclusive prefix sum over the 64 lanes
__device__ __forceinline__ int wave_incl_scan(int v) {
  const int lane = threadIdx.x & 63;
  for (int off = 1; off < 64; off <<= 1) {
    const int t = __shfl_up(v, off, 64);
    if (lane >= off) v += t;
  }
  return v;
}

// wave64 + block reduction of one double into *dst (one atomic per block)
constexpr int ESLOT = 64;   // energy partial-sum slots

// this workgroup's row of the energy partial sums
__device__ __forceinline__ double* eslot(double* epart) {
  return epart + (int64_t)(blockIdx.x & (ESLOT - 1)) * NTERMS;
}

template <int BS>
__device__ __forceinline__ void block_add(double v, double* dst) {
  __shared__ double red[BS / 64];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int k = 0; k < BS / 64; ++k) s += red[k];
    if (s != 0.0) atomicAdd(dst, s);
  }
}

// wave64 + block reduction of one double; the sum is valid in thread 0
template <int BS>
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double red[BS / 64];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < BS / 64; ++k) s += red[k];
  return s;
}

}  // namespace rx
