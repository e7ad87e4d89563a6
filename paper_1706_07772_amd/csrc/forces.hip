// One ReaxFF force evaluation on gfx950, FP64.
//
// Forward: uncorrected bond orders and their radial derivatives per bond
// entry; Delta' per atom; corrected bond orders per entry; atom state
// (S, Delta, lone pairs, SBO).  Energy terms then run as interaction
// kernels that also emit adjoints: scalar adjoints of the corrected bond
// orders (gbo), vector adjoints of bond vectors (gvec), adjoints of atom
// sums (gS, gSig, gSBO).  Backward ("aggregate forces", Table 2's last force
// row): gather cross-atom adjoints, push them through the bond-order
// correction to the uncorrected orders and Delta', then through dBO'/dr to
// forces, and gather each atom's force from its own bond entries
// F_i = sum_j [dE/dr_ij rhat_ij + g_ij - g_ji] plus nonbonded terms.
//
// Race freedom (the paper's Section 3.1 concern): a kernel with one thread
// per atom writes only that atom's entries; cross-atom quantities are stored
// per entry and gathered through the mirror index.  Only the torsion terms
// (which touch entries of both central atoms) and the hydrogen-bond acceptor
// use atomic adds; the nonbonded pairs are evaluated from both sides instead.
#include <type_traits>
#include <algorithm>

#include "internal.h"
#include "terms.h"

namespace rx {

constexpr int BS = 256;

static inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// ---------------------------------------------------------------------------
// stage kernels: one thread per atom, or per bond entry where the entries
// of an atom are independent (no serial loop over the entries)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BS) void k_bo_prime(const DevParams* __restrict__ P, Grid g, Lists L,
                                                 Work W) {
  const int64_t e = xcd_block() * blockDim.x + threadIdx.x;
  if (e < L.nbond) bo_prime_entry(P, g, L, W, L.bond_i[e], (int)e);
}

__global__ __launch_bounds__(BS) void k_delta_prime(const DevParams* __restrict__ P, Lists L, Work W) {
  const int64_t t = xcd_block() * blockDim.x + threadIdx.x;
  const int64_t i = t >> 2;   // four lanes per atom
  if (i < L.n) delta_prime_atom<4>(P, L, W, (int)i, (int)(t & 3));
}

__global__ __launch_bounds__(BS) void k_bo_corr(const DevParams* __restrict__ P, Lists L, Work W) {
  const int64_t e = xcd_block() * blockDim.x + threadIdx.x;
  if (e < L.nbond) bo_corr_entry(P, L, W, L.bond_i[e], (int)e);
}

__global__ __launch_bounds__(BS) void k_atom_state(const DevParams* __restrict__ P, Lists L, Work W) {
  const int64_t i = xcd_block() * blockDim.x + threadIdx.x;
  if (i < L.n) atom_state_atom(P, L, W, (int)i);
}

// ---------------------------------------------------------------------------
// interaction task lists, built as the paper builds its 3-body list
// (Section 3.3): count the interactions each atom owns, prefix-sum the
// counts, then store each interaction at its owner's offset.  Owners: the
// centre atom of a valence angle; the lower-index atom of a torsion's central
// bond; the H atom of a donor bond H-X.
// ---------------------------------------------------------------------------
template <bool FILL>
__global__ __launch_bounds__(BS) void k_tasks(const DevParams* __restrict__ P, Lists L, Work W) {
  // one thread per bond entry u = j->k; the entries of an atom are
  // consecutive, so the tasks come out in the order of the atom-major
  // enumeration: angles (u, v > u) centred on j, torsions about u when k > j,
  // and the donor bond u when j is a hydrogen.  The first TK_C entries of j
  // and of k (bond order, partner) are read into registers in one batch of
  // loads, since the angle and torsion loops both walk them; entries past
  // TK_C are read from memory.
  constexpr int TK_C = 8;
  const int64_t u = xcd_block() * blockDim.x + threadIdx.x;
  if (FILL && u < L.n) W.don_rng[u] = make_int2(W.off_don[L.bond_off[u]], W.off_don[L.bond_off[u + 1]]);
  if (u >= L.nbond) return;
  const double thb = P->thb_cut, thb2 = P->thb_cutsq;
  // H-bond roles of the types as bit masks (uniform loads)
  unsigned hmask = 0, amask = 0;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    hmask |= (P->atom[t].hbond == 1 ? 1u : 0u) << t;
    amask |= (P->atom[t].hbond == 2 ? 1u : 0u) << t;
  }
  const int j = L.bond_i[u];
  const int k = L.bond_j[u];
  const double bu = W.bo1[u];
  const int e0 = L.bond_off[j], e1 = L.bond_off[j + 1];
  const int f0 = L.bond_off[k], f1 = L.bond_off[k + 1];
  const int dj = e1 - e0, dk = f1 - f0, qu = (int)u - e0;
  double boj[TK_C], bok[TK_C];
  int nj[TK_C], nk[TK_C];
#pragma unroll
  for (int q = 0; q < TK_C; ++q) {
    boj[q] = q < dj ? W.bo1[e0 + q] : 0.0;
    nj[q] = q < dj ? L.bond_j[e0 + q] : -1;
    bok[q] = q < dk ? W.bo1[f0 + q] : 0.0;
    nk[q] = q < dk ? L.bond_j[f0 + q] : -1;
  }
  int na = 0, nt = 0, nd = 0;
  const int oa = FILL ? W.off_ang[u] : 0, ot = FILL ? W.off_tor[u] : 0, od = FILL ? W.off_don[u] : 0;
  // the fill pass knows the counts: it skips empty kinds
  const int ca = FILL ? W.cnt_ang[u] : 0, ct = FILL ? W.cnt_tor[u] : 0, cd = FILL ? W.cnt_don[u] : 0;
  // angles (u, v), u < v
  if (FILL ? ca > 0 : bu - thb > 0.0) {
    auto ang = [&](int v, double bv) {
      if (bv - thb > 0.0 && bu * bv > thb2) {
        if (FILL) W.ang[oa + na] = make_int2((int)u, v);
        ++na;
      }
    };
#pragma unroll
    for (int q = 0; q < TK_C; ++q)
      if (q > qu && q < dj) ang(e0 + q, boj[q]);
    for (int v = e0 + (qu + 1 > TK_C ? qu + 1 : TK_C); v < e1; ++v) ang(v, W.bo1[v]);
  }
  // torsions about the central bond u = j->k, k > j: entries a of j (a != u)
  // and b of k, in that nesting
  if (FILL ? ct > 0 : (k > j && bu > thb)) {
    auto tor = [&](int a, double ba, int i) {
      if (a == (int)u || !(ba > thb)) return;
      auto one = [&](int b, double bb, int l) {
        if (l == j || l == i || !(bb > thb) || !(ba * bu * bb > thb)) return;
        if (FILL) W.tor[ot + nt] = make_int4((int)u, a, b, 0);
        ++nt;
      };
#pragma unroll
      for (int r = 0; r < TK_C; ++r)
        if (r < dk) one(f0 + r, bok[r], nk[r]);
      for (int b = f0 + TK_C; b < f1; ++b) one(b, W.bo1[b], L.bond_j[b]);
    };
#pragma unroll
    for (int q = 0; q < TK_C; ++q)
      if (q < dj) tor(e0 + q, boj[q], nj[q]);
    for (int a = e0 + TK_C; a < e1; ++a) tor(a, W.bo1[a], L.bond_j[a]);
  }
  // donor bond
  if (FILL ? cd > 0
           : (((hmask >> L.type_s[j]) & 1u) && ((amask >> L.type_s[k]) & 1u) && bu >= P->hb_bo_cut &&
              L.hb_cnt[j] > 0)) {
    if (FILL) {
      W.don[od] = (int)u;
      W.donrec[od] = DonRec{W.bd[u], bu, k, L.type_s[k]};
    }
    nd = 1;
  }
  if (!FILL) {
    W.cnt_ang[u] = na;
    W.cnt_tor[u] = nt;
    W.cnt_don[u] = nd;
  }
}

// (5) bond energy, lone pair, over- and under-coordination (per atom; the
//     atom's own terms are arithmetic-heavy, so one lane per atom)
__global__ __launch_bounds__(BS) void k_atom_energy(const DevParams* __restrict__ P, Lists L, Work W,
                                                    double* __restrict__ energies) {
  const int64_t i = xcd_block() * blockDim.x + threadIdx.x;
  double e[4] = {0.0, 0.0, 0.0, 0.0};
  if (i < L.n) atom_energy_atom(P, L, W, (int)i, e);
  block_add<BS>(e[0], eslot(W.epart) + E_BOND);
  block_add<BS>(e[1], eslot(W.epart) + E_LP);
  block_add<BS>(e[2], eslot(W.epart) + E_OVER);
  block_add<BS>(e[3], eslot(W.epart) + E_UNDER);
}

// ---------------------------------------------------------------------------
// (6) valence angle, penalty, coalition: one thread per angle task
// ---------------------------------------------------------------------------

// The tasks are ordered by centre atom and a centre's bond entries are
// contiguous, so the 256 tasks of a block touch one contiguous range of
// entries and centres.  Their adjoints are summed in LDS (FP64 LDS atomics),
// then written once: plain stores for centres whose tasks all lie in this
// block, global atomics for the first and last centre, which may share tasks
// with the neighbouring blocks.  Entries or centres beyond the LDS capacity
// go straight to global atomics.
constexpr int ANG_CAPE = 512;   // bond entries per block held in LDS
constexpr int ANG_CAPC = 256;   // centres per block held in LDS

__global__ __launch_bounds__(BS) void k_angles(const DevParams* __restrict__ P, Lists L, Work W,
                                               double* __restrict__ energies) {
  __shared__ double se[ANG_CAPE][5];   // gvec x, y, z, gbo.x, gbo.w per entry
  __shared__ double sc[ANG_CAPC][2];   // gS, dE/dSBO2 per centre
  __shared__ int range[4];
  const int64_t ntask = W.off_ang[L.nbond];
  const int64_t ab = xcd_active_block((ntask + BS - 1) / BS);
  if (ab < 0) return;                               // uniform over the block
  const int64_t T0 = ab * BS;
  const int64_t T1 = T0 + BS < ntask ? T0 + BS : ntask;
  if (threadIdx.x == 0) {
    const int jf = L.bond_i[W.ang[T0].x], jl = L.bond_i[W.ang[T1 - 1].x];
    range[0] = jf;
    range[1] = jl;
    range[2] = L.bond_off[jf];
    range[3] = L.bond_off[jl + 1];
  }
  for (int k = threadIdx.x; k < ANG_CAPE; k += BS)
    for (int c = 0; c < 5; ++c) se[k][c] = 0.0;
  for (int k = threadIdx.x; k < ANG_CAPC; k += BS) sc[k][0] = sc[k][1] = 0.0;
  __syncthreads();
  const int jf = range[0], jl = range[1], E0 = range[2], E1 = range[3];
  double eval = 0.0, epen = 0.0, ecoa = 0.0;
  const int64_t t = T0 + threadIdx.x;
  if (t < T1) {
    const int2 uv = W.ang[t];
    const int u = uv.x, v = uv.y;
    const int j = L.bond_i[u];
    const AngOut o = angle_eval(P, L, W, u, v);
    eval = o.ev;
    epen = o.ep;
    ecoa = o.ec;
    const double* gu = o.gu;
    const double* gv = o.gv;
    const double gS = o.gS, gSBO2 = o.gSBO2;
    const int lu = u - E0, lv = v - E0, lj = j - jf;
    if (lu < ANG_CAPE) {
      for (int q = 0; q < 5; ++q) atomicAdd(&se[lu][q], gu[q]);
    } else {
      atomic_add3(&W.gvec[u], gu[0], gu[1], gu[2]);
      atomicAdd(&W.gbo[u].x, gu[3]);
      atomicAdd(&W.gbo[u].w, gu[4]);
    }
    if (lv < ANG_CAPE) {
      for (int q = 0; q < 5; ++q) atomicAdd(&se[lv][q], gv[q]);
    } else {
      atomic_add3(&W.gvec[v], gv[0], gv[1], gv[2]);
      atomicAdd(&W.gbo[v].x, gv[3]);
      atomicAdd(&W.gbo[v].w, gv[4]);
    }
    if (lj < ANG_CAPC) {
      atomicAdd(&sc[lj][0], gS);
      atomicAdd(&sc[lj][1], gSBO2);
    } else {
      atomicAdd(&W.gS[j], gS);
      atomicAdd(&W.gSBO[j], gSBO2);
    }
  }
  __syncthreads();
  // flush: entries of boundary centres with atomics, the rest with stores
  const int Eb0 = L.bond_off[jf + 1];   // entries of jf end here
  const int Eb1 = L.bond_off[jl];       // entries of jl start here
  const int ne = E1 - E0 < ANG_CAPE ? E1 - E0 : ANG_CAPE;
  for (int k = threadIdx.x; k < ne; k += BS) {
    const int e = E0 + k;
    const bool boundary = e < Eb0 || e >= Eb1;
    double4* gv = &W.gvec[e];
    if (boundary) {
      if (se[k][0] != 0.0 || se[k][1] != 0.0 || se[k][2] != 0.0) atomic_add3(gv, se[k][0], se[k][1], se[k][2]);
      if (se[k][3] != 0.0) atomicAdd(&W.gbo[e].x, se[k][3]);
      if (se[k][4] != 0.0) atomicAdd(&W.gbo[e].w, se[k][4]);
    } else {
      // this block holds all of the entry's angle terms; the arrays were zeroed
      *gv = make_double4(se[k][0], se[k][1], se[k][2], 0.0);
      W.gbo[e].x += se[k][3];
      W.gbo[e].w = se[k][4];
    }
  }
  const int nc = jl - jf + 1 < ANG_CAPC ? jl - jf + 1 : ANG_CAPC;
  for (int k = threadIdx.x; k < nc; k += BS) {
    const int j = jf + k;
    if (j == jf || j == jl) {
      if (sc[k][0] != 0.0) atomicAdd(&W.gS[j], sc[k][0]);
      if (sc[k][1] != 0.0) atomicAdd(&W.gSBO[j], sc[k][1]);
    } else {
      W.gS[j] += sc[k][0];
      W.gSBO[j] = sc[k][1];
    }
  }
  block_add<BS>(eval, eslot(W.epart) + E_VAL);
  block_add<BS>(epen, eslot(W.epart) + E_PEN);
  block_add<BS>(ecoa, eslot(W.epart) + E_COA);
}

// ---------------------------------------------------------------------------
// (7) torsion and 4-body conjugation: one thread per torsion task
// ---------------------------------------------------------------------------
// The tasks are ordered by the central bond's lower atom j, so the BS tasks
// of a block touch one contiguous range of j's entries (j->i and j->k) and
// of j atoms.  Those adjoints are summed in LDS and added to memory once per
// block, with atomics (other blocks reach the same entries as the far atom k
// of their central bond); the k side (entry k->l, Delta_k) goes straight to
// global atomics.  Blocks run in plain order, so the global atomics of
// blocks running together fall on separate parts of the system.
constexpr int TOR_CAPE = 1024;   // j-side entries per block held in LDS
constexpr int TOR_CAPC = 512;    // j atoms per block held in LDS

__global__ __launch_bounds__(BS) void k_torsions(const DevParams* __restrict__ P, Lists L, Work W,
                                                 double* __restrict__ energies) {
  __shared__ double se[TOR_CAPE][5];   // gvec x, y, z, gbo.x, gbo.y per entry
  __shared__ double sj[TOR_CAPC];      // gS per j atom
  __shared__ int range[3];
  const int64_t ntask = W.off_tor[L.nbond];
  double etor = 0.0, econj = 0.0;
  for (int64_t T0 = (int64_t)blockIdx.x * BS; T0 < ntask; T0 += (int64_t)gridDim.x * BS) {
    const int64_t T1 = T0 + BS < ntask ? T0 + BS : ntask;
    __syncthreads();   // the previous pass's flush is done
    if (threadIdx.x == 0) {
      const int jf = L.bond_i[W.tor[T0].x], jl = L.bond_i[W.tor[T1 - 1].x];
      range[0] = jf;
      range[1] = L.bond_off[jf];
      range[2] = L.bond_off[jl + 1];
    }
    for (int k = threadIdx.x; k < TOR_CAPE; k += BS)
      for (int c = 0; c < 5; ++c) se[k][c] = 0.0;
    for (int k = threadIdx.x; k < TOR_CAPC; k += BS) sj[k] = 0.0;
    __syncthreads();
    const int jf = range[0], E0 = range[1], E1 = range[2];
    const int64_t t = T0 + threadIdx.x;
    if (t < T1) {
      const int4 q = W.tor[t];
      const int ejk = q.x, eji = q.y, ekl = q.z;
      const TorOut o = torsion_terms(P, L, W, ejk, eji, ekl, etor, econj);
      const int j = L.bond_i[ejk], k = L.bond_j[ejk];
      const int lji = eji - E0, ljk = ejk - E0, lj = j - jf;
      if (lji < TOR_CAPE) {
        atomicAdd(&se[lji][0], o.gji.x);
        atomicAdd(&se[lji][1], o.gji.y);
        atomicAdd(&se[lji][2], o.gji.z);
        atomicAdd(&se[lji][3], o.gBij);
      } else {
        atomic_add3(&W.gvec[eji], o.gji);
        atomicAdd(&W.gbo[eji].x, o.gBij);
      }
      if (ljk < TOR_CAPE) {
        atomicAdd(&se[ljk][0], o.gjk.x);
        atomicAdd(&se[ljk][1], o.gjk.y);
        atomicAdd(&se[ljk][2], o.gjk.z);
        atomicAdd(&se[ljk][3], o.gBjk);
        atomicAdd(&se[ljk][4], o.gPjk);
      } else {
        atomic_add3(&W.gvec[ejk], o.gjk);
        atomicAdd(&W.gbo[ejk].x, o.gBjk);
        atomicAdd(&W.gbo[ejk].y, o.gPjk);
      }
      if (lj < TOR_CAPC) atomicAdd(&sj[lj], o.gD);
      else atomicAdd(&W.gS[j], o.gD);
      atomic_add3(&W.gvec[ekl], o.gkl);
      atomicAdd(&W.gbo[ekl].x, o.gBkl);
      atomicAdd(&W.gS[k], o.gD);
    }
    __syncthreads();
    const int ne = E1 - E0 < TOR_CAPE ? E1 - E0 : TOR_CAPE;
    for (int k = threadIdx.x; k < ne; k += BS) {
      const int e = E0 + k;
      if (se[k][0] != 0.0 || se[k][1] != 0.0 || se[k][2] != 0.0)
        atomic_add3(&W.gvec[e], se[k][0], se[k][1], se[k][2]);
      if (se[k][3] != 0.0) atomicAdd(&W.gbo[e].x, se[k][3]);
      if (se[k][4] != 0.0) atomicAdd(&W.gbo[e].y, se[k][4]);
    }
    const int jl = L.bond_i[W.tor[T1 - 1].x];
    const int nc = jl - jf + 1 < TOR_CAPC ? jl - jf + 1 : TOR_CAPC;
    for (int k = threadIdx.x; k < nc; k += BS)
      if (sj[k] != 0.0) atomicAdd(&W.gS[jf + k], sj[k]);
  }
  block_add<BS>(etor, eslot(W.epart) + E_TOR);
  block_add<BS>(econj, eslot(W.epart) + E_CONJ);
}

constexpr int HB_DROW = 16;   // lanes per donor task

// ---------------------------------------------------------------------------
// (8) hydrogen bonds.  Each term X-H...Z moves three atoms.  The donor side
//     (16 lanes per donor bond H-X, striding over H's acceptor row) sums the energy,
//     the adjoints of the H-X bond entry and the force on H.  The acceptor
//     side (16 lanes per acceptor Z, over Z's acceptor row: the donors H
//     within r_hb, found by the sweep with the H list's own predicate)
//     recomputes the term's gradient with respect to Z and reduces it over
//     the lanes, so no force is scattered to acceptors.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(BS) void k_hbonds(const DevParams* __restrict__ P, Grid g, Lists L, Work W,
                                               double* __restrict__ energies) {
  // the H-bond parameters in LDS: a neighbour's record is then one LDS read
  // after its position arrives
  __shared__ HbP hbt[NT * NT * NT];
  for (int q = threadIdx.x; q < NT * NT * NT; q += BS) hbt[q] = P->hb[q];
  __syncthreads();
  const int64_t ntask = W.off_don[L.nbond];
  double ehb = 0.0;
  unsigned long long nhb = 0;
  // one 16-lane row per task, the lanes striding over H's row of acceptor
  // candidates; XCD k takes the k-th eighth of the blocks with work
  constexpr int TPB = BS / HB_DROW;
  const int sub = threadIdx.x & (HB_DROW - 1);
  const int64_t ab = xcd_active_block((ntask + TPB - 1) / TPB);
  const int64_t t = ab * TPB + threadIdx.x / HB_DROW;
  const bool live = ab >= 0 && t < ntask;
  double gbo = 0.0;
  double3 gx = make_double3(0.0, 0.0, 0.0), fh = make_double3(0.0, 0.0, 0.0);
  int ex = 0, h = 0;
  if (live) {
    ex = W.don[t];
    h = L.bond_i[ex];
    const int X = L.bond_j[ex];
    const int th = L.type_s[h], tx = L.type_s[X];
    const double4 xh = L.xs[h];
    const double bo = W.bo1[ex];
    const double4 rx = W.bd[ex];     // x_X - x_h
    const int nz = L.hb_cnt[h];
    const int32_t* __restrict__ zrow = L.hb_j + (int64_t)h * L.hb_w;
    for (int s = sub; s < nz; s += HB_DROW) {
      const int Z = zrow[s];
      if (Z == X) continue;
      const double4 xz = L.xs[Z];   // position and type
      const HbP& hp = hbt[(tx * NT + th) * NT + (int)xz.w];
      double dx = xz.x - xh.x, dy = xz.y - xh.y, dz = xz.z - xh.z;
      if (g.periodic) {
        dx = min_image(dx, g.L[0], g.invL[0]);
        dy = min_image(dy, g.L[1], g.invL[1]);
        dz = min_image(dz, g.L[2], g.invL[2]);
      }
      // a skin entry beyond r_hb (the list's own predicate, same rounding)
      if (L.cut_check && r2_of(dx, dy, dz) > P->rh2) continue;
      ++nhb;
      const HbTerm o = hb_term(hp, bo, rx, dx, dy, dz);
      ehb += o.E;
      gbo += o.dE_dbo;
      gx = add3(gx, o.g_rx);
      fh = add3(fh, o.g_rz);            // r_hZ = x_Z - x_h: F_h = +dE/dr_hZ
    }
  }
  // row sums (every lane takes part), written by the row's last lane: the
  // entry h->X belongs to this task alone
  gbo = row_sum_last(gbo);
  gx.x = row_sum_last(gx.x);
  gx.y = row_sum_last(gx.y);
  gx.z = row_sum_last(gx.z);
  fh.x = row_sum_last(fh.x);
  fh.y = row_sum_last(fh.y);
  fh.z = row_sum_last(fh.z);
  if (live && sub == HB_DROW - 1) {
    double4 gv = W.gvec[ex];
    gv.x += gx.x;
    gv.y += gx.y;
    gv.z += gx.z;
    W.gvec[ex] = gv;
    W.gbo[ex].x += gbo;
    atomic_add3(&W.fhb[h], fh);
  }
  block_add<BS>(ehb, eslot(W.epart) + E_HB);
  {
    __shared__ unsigned long long rn[BS / 64];
    for (int off = 32; off > 0; off >>= 1) nhb += __shfl_down(nhb, off, 64);
    if ((threadIdx.x & 63) == 0) rn[threadIdx.x >> 6] = nhb;
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned long long t = 0;
      for (int w = 0; w < BS / 64; ++w) t += rn[w];
      if (t) atomicAdd(&W.counters[2], t);
    }
  }
}

// Acceptor side: F_Z = -dE/dx_Z = -sum dE/d(x_Z - x_h) over the donors H of
// Z's acceptor row.  Four acceptors per wavefront, one 16-lane row each.  The
// row's lanes first list the (H, donor task) pairs of Z's acceptor row in LDS
// (most H atoms have no donor bond), then share the list evenly, so the
// lanes evaluate terms instead of idling; a list longer than the LDS slot is
// walked directly.  Each donor bond H-X is read from its packed record; the
// row sums are written once per acceptor (no atomics).
constexpr int HB_GROUP = 16;
constexpr int HB_PACK = 128;   // listed (H, task) pairs per acceptor

__global__ __launch_bounds__(BS) void k_hb_acceptors(const DevParams* __restrict__ P, Grid g, Lists L,
                                                     Work W) {
  __shared__ int2 pk[BS / HB_GROUP][HB_PACK];
  __shared__ HbP hbt[NT * NT * NT];
  for (int q = threadIdx.x; q < NT * NT * NT; q += BS) hbt[q] = P->hb[q];
  __syncthreads();
  const int lane = threadIdx.x & 63, sub = lane & (HB_GROUP - 1);
  int2* __restrict__ mylist = pk[threadIdx.x / HB_GROUP];
  const int64_t z = (xcd_block() * BS + threadIdx.x) / HB_GROUP;
  const int cnt = z < L.n ? L.ha_cnt[z] : 0;   // uniform over the row
  double3 fz = make_double3(0.0, 0.0, 0.0);
  const int32_t* __restrict__ row = L.ha_j + z * (int64_t)L.ha_w;
  // this lane's pairs, and their offset in the row's list; the first
  // HB_KMAX row entries of the lane are read in one go and kept
  constexpr int HB_KMAX = 8;
  int hh[HB_KMAX];
  int2 rr[HB_KMAX];
  int mine = 0;
#pragma unroll
  for (int j = 0; j < HB_KMAX; ++j) {
    const int k = sub + j * HB_GROUP;
    hh[j] = k < cnt ? row[k] : 0;
  }
#pragma unroll
  for (int j = 0; j < HB_KMAX; ++j) {
    const int k = sub + j * HB_GROUP;
    rr[j] = k < cnt ? W.don_rng[hh[j]] : make_int2(0, 0);
    mine += rr[j].y - rr[j].x;
  }
  for (int k = sub + HB_KMAX * HB_GROUP; k < cnt; k += HB_GROUP) {
    const int2 tr = W.don_rng[row[k]];
    mine += tr.y - tr.x;
  }
  int incl = mine;
  for (int off = 1; off < HB_GROUP; off <<= 1) {
    const int v = __shfl_up(incl, off, HB_GROUP);
    if (sub >= off) incl += v;
  }
  const int total = __shfl(incl, HB_GROUP - 1, HB_GROUP);
  auto term = [&](int h, int t, double4 xz, int tz) {
    const DonRec d = W.donrec[t];
    if (d.X == (int)z) return;
    const double4 xh = L.xs[h];   // position and type
    const int th = (int)xh.w;
    double dx = xz.x - xh.x, dy = xz.y - xh.y, dz = xz.z - xh.z;   // x_Z - x_h
    if (g.periodic) {
      dx = min_image(dx, g.L[0], g.invL[0]);
      dy = min_image(dy, g.L[1], g.invL[1]);
      dz = min_image(dz, g.L[2], g.invL[2]);
    }
    if (L.cut_check && r2_of(dx, dy, dz) > P->rh2) return;   // a skin entry beyond r_hb
    const HbP& hp = hbt[(d.tX * NT + th) * NT + tz];
    const HbTerm o = hb_term(hp, d.bo, d.bd, dx, dy, dz);
    fz.x -= o.g_rz.x;
    fz.y -= o.g_rz.y;
    fz.z -= o.g_rz.z;
  };
  if (total > 0) {
    const int tz = L.type_s[z];
    const double4 xz = L.xs[z];
    if (total <= HB_PACK) {
      int pos = incl - mine;
#pragma unroll
      for (int j = 0; j < HB_KMAX; ++j)
        for (int t = rr[j].x; t < rr[j].y; ++t) mylist[pos++] = make_int2(hh[j], t);
      for (int k = sub + HB_KMAX * HB_GROUP; k < cnt; k += HB_GROUP) {
        const int h = row[k];
        const int2 tr = W.don_rng[h];
        for (int t = tr.x; t < tr.y; ++t) mylist[pos++] = make_int2(h, t);
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      for (int q = sub; q < total; q += HB_GROUP) {
        const int2 ht = mylist[q];
        term(ht.x, ht.y, xz, tz);
      }
    } else {
      for (int k = sub; k < cnt; k += HB_GROUP) {
        const int h = row[k];
        const int2 tr = W.don_rng[h];
        for (int t = tr.x; t < tr.y; ++t) term(h, t, xz, tz);
      }
    }
  }
  fz.x = row_sum_last(fz.x);
  fz.y = row_sum_last(fz.y);
  fz.z = row_sum_last(fz.z);
  if (sub == HB_GROUP - 1 && total > 0) {
    double4 f = W.fhb[z];
    f.x += fz.x;
    f.y += fz.y;
    f.z += fz.z;
    W.fhb[z] = f;
  }
}

// ---------------------------------------------------------------------------
// (9) van der Waals and Coulomb.  One workgroup per cell.  All atoms of a
//     cell share one stencil, so the workgroup first copies the stencil's
//     atoms (position, charge, type) into LDS with coalesced loads; far rows
//     hold stencil slots, so each neighbour is then read from LDS rather than
//     gathered from memory.  The cell's rows are cut into units of 64
//     entries that never cross a row, and the units are split evenly over
//     the workgroup's wavefronts, one entry per lane: the centre atom is the
//     same for the whole wavefront, and its force is reduced across the
//     wavefront and added to the atom's LDS accumulator whenever the
//     wavefront moves on to the next atom.  Every pair is evaluated from both
//     sides and no force is scattered (the redundant-computation choice for
//     pairwise terms, Section 3.1); energies weigh each visit by 1/2.  A
//     stencil too large for the LDS copy reads its neighbours from memory
//     through the chunk table instead.  Cells go to the XCDs in contiguous
//     ranges, so the cells running together on an XCD share stencils in its L2.
// ---------------------------------------------------------------------------
constexpr int NBC_BS = 512, NBC_WAVES = NBC_BS / 64;
constexpr int NBC_CAP = 2048;  // stencil atoms held in LDS
constexpr int NBC_MG = 64;     // atoms of a cell per pass
constexpr int NBC_MAXQ = 64;   // chunks of a stencil: 2 (2 reach + 1)^2 <= 50

__global__ __launch_bounds__(NBC_BS) void k_nonbonded(const DevParams* __restrict__ P, Grid g, Lists L,
                                                      Work W, int ncell, int per_xcd,
                                                      double* __restrict__ energies) {
  __shared__ NbP sp[NT * NT];
  __shared__ double sxx[NBC_CAP], sxy[NBC_CAP], sxz[NBC_CAP], sxq[NBC_CAP];
  __shared__ unsigned char sty[NBC_CAP];
  __shared__ int q_s0[NBC_MAXQ], q_base[NBC_MAXQ + 1];
  __shared__ int upre[NBC_MG + 1];
  __shared__ double facc[3][NBC_MG];
  // the pass's centre atoms: position, charge times the Coulomb constant,
  // type and row length
  __shared__ double ixx[NBC_MG], ixy[NBC_MG], ixz[NBC_MG], iqq[NBC_MG];
  __shared__ int ity[NBC_MG], icnt[NBC_MG];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int c = (int)(blockIdx.x & 7) * per_xcd + (int)(blockIdx.x >> 3);
  if (c >= ncell) return;
  const int a0 = L.cell_start[c], m = L.cell_start[c + 1] - a0;
  if (m == 0) {
    if (tid == 0) W.nbe[c] = make_double2(0.0, 0.0);
    return;
  }
  if (tid < NT * NT) sp[tid] = nb_params(P->pair[tid]);
  // chunk table of the stencil: start atom and first slot of each chunk
  const int nq = stencil_chunks(g);
  if (tid < nq) {
    int s0, s1;
    double sx, sy, sz;
    stencil_chunk(g, L.cell_start, c, tid, s0, s1, sx, sy, sz);
    q_s0[tid] = s0;
    q_base[tid + 1] = s1 - s0;
  }
  __syncthreads();
  if (wv == 0) {
    const int v = wave_incl_scan(lane < nq ? q_base[lane + 1] : 0);
    if (lane < nq) q_base[lane + 1] = v;
    if (lane == 0) q_base[0] = 0;
  }
  __syncthreads();
  const int nst = q_base[nq];
  const bool staged = nst <= NBC_CAP;
  if (staged) {
    for (int t0 = 0; t0 < nst; t0 += 4 * NBC_BS) {
      int idx[4];
      double4 v[4];
      int ty[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int t = t0 + u * NBC_BS + tid;
        idx[u] = -1;
        if (t < nst) {
          const int q = last_le(q_base, nq, t);
          idx[u] = q_s0[q] + (t - q_base[q]);
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (idx[u] >= 0) {
          v[u] = W.xq[idx[u]];
          ty[u] = L.type_s[idx[u]];
        }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (idx[u] >= 0) {
          const int t = t0 + u * NBC_BS + tid;
          sxx[t] = v[u].x;
          sxy[t] = v[u].y;
          sxz[t] = v[u].z;
          sxq[t] = v[u].w;
          sty[t] = (unsigned char)ty[u];
        }
    }
  }
  const double iR = P->inv_r_nonb, pv = P->p_vdW1, ipv = P->inv_p_vdW1;
  double evdw = 0.0, ecoul = 0.0;
  for (int g0 = 0; g0 < m; g0 += NBC_MG) {
    const int mg = m - g0 < NBC_MG ? m - g0 : NBC_MG;
    // units of 64 row entries per atom, prefix-summed
    if (wv == 0) {
      int cnt = 0;
      if (lane < mg) {
        const int i = a0 + g0 + lane;
        cnt = L.far_cnt[i];
        const double4 xi = W.xq[i];
        ixx[lane] = xi.x;
        ixy[lane] = xi.y;
        ixz[lane] = xi.z;
        iqq[lane] = xi.w * C_ELE;
        ity[lane] = L.type_s[i];
        icnt[lane] = cnt;
      }
      const int v = wave_incl_scan((cnt + 63) >> 6);
      if (lane < mg) upre[lane + 1] = v;
      if (lane == 0) upre[0] = 0;
    }
    for (int t = tid; t < 3 * NBC_MG; t += NBC_BS) facc[t / NBC_MG][t % NBC_MG] = 0.0;
    __syncthreads();
    const int U = __builtin_amdgcn_readfirstlane(upre[mg]);
    const int wu = __builtin_amdgcn_readfirstlane(wv);
    const int u0 = U * wu / NBC_WAVES, u1 = U * (wu + 1) / NBC_WAVES;
    // one copy of the unit loop per neighbour source, so that each keeps its
    // own address space (LDS reads, or global reads through the chunk table)
    auto units = [&](auto from_lds) {
      constexpr bool LDS = decltype(from_lds)::value;
      // the row entry of unit u + 1 is loaded while unit u is computed
      auto locate = [&](int u, int& a) {
        while (__builtin_amdgcn_readfirstlane(upre[a + 1]) <= u) ++a;
      };
      auto fetch = [&](int u, int a) {
        const int k = ((u - __builtin_amdgcn_readfirstlane(upre[a])) << 6) + lane;
        const int32_t* __restrict__ row = L.far_j + (int64_t)(a0 + g0 + a) * L.far_w;
        return k < __builtin_amdgcn_readfirstlane(icnt[a]) ? row[k] : -1;
      };
      int a = __builtin_amdgcn_readfirstlane(last_le(upre, mg, u0));
      locate(u0, a);
      int slot = fetch(u0, a);
      int cur = a;
      double xix = ixx[cur], xiy = ixy[cur], xiz = ixz[cur], qi = iqq[cur];
      const NbP* __restrict__ spi = sp + ity[cur] * NT;
      double fx = 0.0, fy = 0.0, fz = 0.0;
      auto flush = [&]() {
        for (int off = 32; off > 0; off >>= 1) {
          fx += __shfl_down(fx, off, 64);
          fy += __shfl_down(fy, off, 64);
          fz += __shfl_down(fz, off, 64);
        }
        if (lane == 0) {
          atomicAdd(&facc[0][cur], fx);
          atomicAdd(&facc[1][cur], fy);
          atomicAdd(&facc[2][cur], fz);
        }
        fx = fy = fz = 0.0;
      };
      for (int u = u0; u < u1; ++u) {
        const int snow = slot, anow = a;
        if (u + 1 < u1) {
          locate(u + 1, a);
          slot = fetch(u + 1, a);
        }
        if (anow != cur) {
          flush();
          cur = anow;
          xix = ixx[cur];
          xiy = ixy[cur];
          xiz = ixz[cur];
          qi = iqq[cur];
          spi = sp + ity[cur] * NT;
        }
        if (snow >= 0) {
          double xjx, xjy, xjz, qj;
          int tj;
          if constexpr (LDS) {
            xjx = sxx[snow];
            xjy = sxy[snow];
            xjz = sxz[snow];
            qj = sxq[snow];
            tj = sty[snow];
          } else {
            const int q = last_le(q_base, nq, snow);
            const int j = q_s0[q] + (snow - q_base[q]);
            const double4 xj = W.xq[j];
            xjx = xj.x;
            xjy = xj.y;
            xjz = xj.z;
            qj = xj.w;
            tj = L.type_s[j];
          }
          double dx = xjx - xix, dy = xjy - xiy, dz = xjz - xiz;
          if (g.periodic) {
            dx = min_image(dx, g.L[0], g.invL[0]);
            dy = min_image(dy, g.L[1], g.invL[1]);
            dz = min_image(dz, g.L[2], g.invL[2]);
          }
          const double r2 = dx * dx + dy * dy + dz * dz;
          if (L.cut_check && r2 > P->rn2) continue;   // a skin entry beyond the cutoff
          const NbOut o = nb_pair(spi[tj], iR, pv, ipv, qi * qj, r2);
          evdw += o.ev;
          ecoul += o.eq;
          fx += o.f * dx;
          fy += o.f * dy;
          fz += o.f * dz;
        }
      }
      flush();
    };
    if (u0 < u1) {
      if (staged) units(std::true_type{});
      else units(std::false_type{});
    }
    __syncthreads();
    if (tid < mg) W.fnb[a0 + g0 + tid] = make_double4(facc[0][tid], facc[1][tid], facc[2][tid], 0.0);
    __syncthreads();
  }
  const double sv = block_sum<NBC_BS>(0.5 * evdw), sq = block_sum<NBC_BS>(0.5 * ecoul);
  if (tid == 0) W.nbe[c] = make_double2(sv, sq);
}

// ---------------------------------------------------------------------------
// (9) half evaluation.  With the chunk order of stencil_chunk and no
//     dimension covered whole, the neighbours of atom i at a larger slot than
//     i's own are exactly those at a lexicographically positive cell offset
//     (or after i in its own cell); of every pair, exactly one atom sees the
//     other there.  Slots number the window of i's run (window_chunk, the
//     stencils of the run's Grid::run cells of one column laid together), so
//     the workgroup of a run stages the run's upper window once (from the
//     run's first atom on) and evaluates each such pair once, for the row
//     suffix [far_lo[i], cnt_i) of each atom of the run's cells.  Both atoms'
//     forces are added to LDS accumulators on the staged slots (the centre's
//     through sums over the 8 lanes of a unit when they move on, the partner's per
//     pair); the accumulators are stored, not added, to the run's partial
//     array (x, y, z of a slot contiguous), and k_nb_reduce sums, for each
//     atom, the partial arrays of the runs whose upper window holds it.
//     Energies take each pair once.  In a periodic box whose chunk shifts are
//     the minimum images, the staged positions carry their chunk's shift, so
//     a displacement is a plain difference; the row sums use DPP moves.
// ---------------------------------------------------------------------------
constexpr int NBH_BS = 1024, NBH_WAVES = NBH_BS / 64;
constexpr int NBH_MG = 128;   // centre atoms of a run per pass (two per lane of one wavefront)

__global__ __launch_bounds__(NBH_BS) __attribute__((amdgpu_waves_per_eu(4))) void k_nonbonded_half(
    const DevParams* __restrict__ P, Grid g, Lists L, Work W, int nrun, int per_xcd,
    double* __restrict__ energies) {
  __shared__ NbP sp[NT * NT];
  __shared__ double sxx[NB_HALF_CAP], sxy[NB_HALF_CAP], sxz[NB_HALF_CAP], sxq[NB_HALF_CAP];
  __shared__ double fax[NB_HALF_CAP], fay[NB_HALF_CAP], faz[NB_HALF_CAP];
  __shared__ unsigned char sty[NB_HALF_CAP];
  __shared__ int q_s0[NBC_MAXQ], q_base[NBC_MAXQ + 1];
  __shared__ double q_sh[NBC_MAXQ][3];
  __shared__ int upre[NBH_MG + 1];
  __shared__ double ixx[NBH_MG], ixy[NBH_MG], ixz[NBH_MG], iqq[NBH_MG];
  __shared__ int ity[NBH_MG], icnt[NBH_MG], ilo[NBH_MG];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int r = (int)(blockIdx.x & 7) * per_xcd + (int)(blockIdx.x >> 3);
  if (r >= nrun) return;
  int c, nk;
  run_cells(g, r, c, nk);
  const int a0 = L.cell_start[c], m = L.cell_start[c + nk] - a0;
  if (m == 0) {   // no pairs: chunk offsets that send the reduce past every slot
    if (tid == 0) W.nbe[r] = make_double2(0.0, 0.0);
    if (tid < stencil_chunks(g)) W.nbtab[(int64_t)r * NB_QMAX + tid] = -0x40000000;
    return;
  }
  if (tid < NT * NT) sp[tid] = nb_params(P->pair[tid]);
  const int nq = stencil_chunks(g);
  // staged positions carry their chunk's image shift when it is the minimum
  // image of every listed pair; otherwise each pair takes the minimum image
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
  const int S0 = q_base[q_own] + (a0 - q_s0[q_own]);   // slot of the run's first atom
  const int nup = nst - S0;                            // <= NB_HALF_CAP (checked by the sweep)
  // for the reduce: atom j of chunk q has staged index nbtab[q] + j
  if (tid < nq) W.nbtab[(int64_t)r * NB_QMAX + tid] = q_base[tid] - S0 - q_s0[tid];
  // staging: wavefront w copies the upper-window parts of chunks w, w + 16,
  // ...; its lanes stride a chunk's atoms, which are contiguous in memory
  for (int q = q_own + wv; q < nq; q += NBH_WAVES) {
    const int b = q_base[q], e = q_base[q + 1];
    const int sb = b > S0 ? b : S0, src = q_s0[q] - b;
    const double hx = q_sh[q][0], hy = q_sh[q][1], hz = q_sh[q][2];
    for (int s0 = sb; s0 < e; s0 += 128) {
      double4 v[2];
      int ty[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int s = s0 + 64 * u + lane;
        if (s < e) {
          v[u] = W.xq[src + s];
          ty[u] = L.type_s[src + s];
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
          sxq[t] = v[u].w;
          sty[t] = (unsigned char)ty[u];
          fax[t] = fay[t] = faz[t] = 0.0;
        }
      }
    }
  }
  const double iR = P->inv_r_nonb, pv = P->p_vdW1, ipv = P->inv_p_vdW1, rn2c = P->rn2;
  double evdw = 0.0, ecoul = 0.0;
  for (int g0 = 0; g0 < m; g0 += NBH_MG) {
    const int mg = m - g0 < NBH_MG ? m - g0 : NBH_MG;
    if (g0 > 0) __syncthreads();   // the previous pass's units done
    if (wv == 0) {   // the pass's centres, two per lane: 2 lane and 2 lane + 1
      int nu[2] = {0, 0};
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int k = 2 * lane + h;
        if (k < mg) {
          const int i = a0 + g0 + k;
          const int cnt = L.far_cnt[i], lo = L.far_lo[i];
          const double4 xi = W.xq[i];
          ixx[k] = xi.x;
          ixy[k] = xi.y;
          ixz[k] = xi.z;
          iqq[k] = xi.w * C_ELE;
          ity[k] = L.type_s[i];
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
    // units of 8 row entries: each wavefront takes a contiguous share of the
    // units and works on eight at a time, one per group of 8 lanes, so a far
    // row's last unit idles at most 7 lanes; the centre atom is uniform over
    // each group
    const int U = __builtin_amdgcn_readfirstlane(upre[mg]);
    const int wu = __builtin_amdgcn_readfirstlane(wv);
    const int u0 = U * wu / NBH_WAVES, u1 = U * (wu + 1) / NBH_WAVES;
    if (u0 < u1) {
      const int hh = lane >> 3, sl = lane & 7;
      // the far row of centre a (uniform over the 8 lanes) kept in registers: units
      // [ua, un) are its, starting at entry lo, cn entries in all
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
      // the raw row entry of this lane in unit u (0 when u is past the end or
      // the entry past the row); ok says whether it is an entry
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
      auto staged = [&](int raw, bool ok) {   // always in range for a consistent list
        const int t = raw - S0;
        return ok && (unsigned)t < (unsigned)nup ? t : -1;
      };
      // three units in flight per 8 lanes: this iteration's (its partner's
      // staged data loaded), the next one's (row entry loaded) and the one
      // after, whose row entry is fetched during this iteration's pair
      const int uh = u0 + hh;
      enter(last_le(upre, mg, uh < u1 ? uh : u1 - 1));
      bool ok0, ok1;
      const int r0 = fetch(uh, ok0);
      const int acur0 = a;
      int r1 = fetch(uh + 8, ok1);
      int anext = a;
      int tnow = staged(r0, ok0), anow = acur0;
      double jx, jy, jz, jq;
      int jt;
      {
        const int t = tnow >= 0 ? tnow : 0;
        jx = sxx[t];
        jy = sxy[t];
        jz = sxz[t];
        jq = sxq[t];
        jt = sty[t];
      }
      int cur = anow;
      double xix = ixx[cur], xiy = ixy[cur], xiz = ixz[cur], qi = iqq[cur];
      const NbP* __restrict__ spi = sp + ity[cur] * NT;
      double fx = 0.0, fy = 0.0, fz = 0.0;
      auto flush = [&]() {   // over the 8 lanes, into the last
        fx = oct_sum_last(fx);
        fy = oct_sum_last(fy);
        fz = oct_sum_last(fz);
        if (sl == 7) {
          const int t = g0 + cur;   // the centre's staged index: slot - S0 = i - a0
          atomicAdd(&fax[t], fx);
          atomicAdd(&fay[t], fy);
          atomicAdd(&faz[t], fz);
        }
        fx = fy = fz = 0.0;
      };
      for (int ub = u0; ub < u1; ub += 8) {
        // the unit after next: its row entry is loaded during this pair
        bool ok2;
        const int r2n = fetch(ub + 16 + hh, ok2);
        const int aafter = a;
        // the next unit: its partner's staged data is loaded during this pair
        const int tnext = staged(r1, ok1);
        double nx, ny, nz, nq;
        int nt;
        {
          const int t = tnext >= 0 ? tnext : 0;
          nx = sxx[t];
          ny = sxy[t];
          nz = sxz[t];
          nq = sxq[t];
          nt = sty[t];
        }
        if (anow != cur) {
          flush();
          cur = anow;
          xix = ixx[cur];
          xiy = ixy[cur];
          xiz = ixz[cur];
          qi = iqq[cur];
          spi = sp + ity[cur] * NT;
        }
        if (tnow >= 0) {
          double dx = jx - xix, dy = jy - xiy, dz = jz - xiz;
          if (minimg) {
            dx = min_image(dx, g.L[0], g.invL[0]);
            dy = min_image(dy, g.L[1], g.invL[1]);
            dz = min_image(dz, g.L[2], g.invL[2]);
          }
          const double rr = dx * dx + dy * dy + dz * dz;
          if (!(L.cut_check && rr > rn2c)) {   // else a skin entry beyond the cutoff
            const NbOut o = nb_pair(spi[jt], iR, pv, ipv, qi * jq, rr);
            evdw += o.ev;
            ecoul += o.eq;
            const double px = o.f * dx, py = o.f * dy, pz = o.f * dz;
            fx += px;
            fy += py;
            fz += pz;
            atomicAdd(&fax[tnow], -px);
            atomicAdd(&fay[tnow], -py);
            atomicAdd(&faz[tnow], -pz);
          }
        }
        tnow = tnext;
        anow = anext;
        jx = nx;
        jy = ny;
        jz = nz;
        jq = nq;
        jt = nt;
        r1 = r2n;
        ok1 = ok2;
        anext = aafter;
      }
      flush();
    }
  }
  __syncthreads();
  double* __restrict__ part = W.nbpart + (int64_t)r * 3 * NB_HALF_CAP;
  for (int t = tid; t < nup; t += NBH_BS) {
    part[3 * t] = fax[t];
    part[3 * t + 1] = fay[t];
    part[3 * t + 2] = faz[t];
  }
  const double sv = block_sum<NBH_BS>(evdw), sq = block_sum<NBH_BS>(ecoul);
  if (tid == 0) W.nbe[r] = make_double2(sv, sq);
}

// the cells' nonbonded energies, summed into the two energy terms
__global__ __launch_bounds__(BS) void k_nb_energy(int ncell, const double2* __restrict__ nbe,
                                                  double* __restrict__ energies) {
  double ev = 0.0, eq = 0.0;
  for (int c = blockIdx.x * BS + threadIdx.x; c < ncell; c += gridDim.x * BS) {
    const double2 e = nbe[c];
    ev += e.x;
    eq += e.y;
  }
  block_add<BS>(ev, energies + E_VDW);
  block_add<BS>(eq, energies + E_COUL);
}

// Nonbonded force of each atom j from the partial arrays of the runs whose
// upper window holds it (for_upper_windows).  Writes the per-atom
// accumulator the hydrogen-bond kernels then add to.  R: the stencil reach.
template <int R>
__global__ __launch_bounds__(BS) void k_nb_reduce(Grid g, Lists L, Work W) {
  const int64_t j = xcd_block() * blockDim.x + threadIdx.x;
  if (j >= L.n) return;
  double fx = 0.0, fy = 0.0, fz = 0.0;
  for_upper_windows<R>(g, L.cell_of[j], W.nbtab, (int)j, [&](int64_t r, int t) {
    const double* __restrict__ part = W.nbpart + r * 3 * NB_HALF_CAP + 3 * t;
    fx += part[0];
    fy += part[1];
    fz += part[2];
  });
  W.fnb[j] = make_double4(fx, fy, fz, 0.0);
}

// ---------------------------------------------------------------------------
// backward
// ---------------------------------------------------------------------------
// (10)-(13) backward, one thread per atom
__global__ __launch_bounds__(BS) void k_back_s(Lists L, Work W) {
  const int64_t t = xcd_block() * blockDim.x + threadIdx.x;
  const int64_t i = t >> 2;
  if (i < L.n) back_s_atom<4>(L, W, (int)i, (int)(t & 3));
}

__global__ __launch_bounds__(BS) void k_back_corr(const DevParams* __restrict__ P, Lists L, Work W) {
  const int64_t e = xcd_block() * blockDim.x + threadIdx.x;
  if (e < L.nbond) back_corr_entry(P, L, W, L.bond_i[e], (int)e);
}

__global__ __launch_bounds__(BS) void k_back_dp(Lists L, Work W) {
  const int64_t t = xcd_block() * blockDim.x + threadIdx.x;
  const int64_t i = t >> 2;   // four lanes per atom
  if (i < L.n) back_dp_atom<4>(L, W, (int)i, (int)(t & 3));
}

// per-atom force gather, four lanes per atom over its entries, written in
// the caller's order
__global__ __launch_bounds__(BS) void k_forces(Lists L, Work W, double* __restrict__ forces) {
  const int64_t t = xcd_block() * blockDim.x + threadIdx.x;
  const int64_t i = t >> 2;
  const int sub = (int)(t & 3);
  if (i >= L.n) return;   // uniform over the four lanes of an atom
  double3 f = force_atom(L, W, (int)i, sub, 4);
  f.x = quad_sum(f.x);
  f.y = quad_sum(f.y);
  f.z = quad_sum(f.z);
  if (sub == 0) {
    const double4 h = W.fhb[i];
    const int o = L.perm[i];
    forces[3 * (int64_t)o] = f.x + h.x;
    forces[3 * (int64_t)o + 1] = f.y + h.y;
    forces[3 * (int64_t)o + 2] = f.z + h.z;
  }
}

__global__ void k_gather_q(const double* __restrict__ q, const int32_t* __restrict__ perm,
                           const double4* __restrict__ xs, int64_t n, double4* __restrict__ xq) {
  const int64_t s = xcd_block() * blockDim.x + threadIdx.x;
  if (s < n) {
    const double4 x = xs[s];
    xq[s] = make_double4(x.x, x.y, x.z, q[perm[s]]);
  }
}

// the energy partial-sum slots, summed into the energies
__global__ void k_energy_fold(const double* __restrict__ epart, double* __restrict__ energies) {
  const int t = threadIdx.x;
  if (t >= NTERMS) return;
  double v = 0.0;
  for (int k = 0; k < ESLOT; ++k) v += epart[k * NTERMS + t];
  if (v != 0.0) atomicAdd(&energies[t], v);
}

const char* const kKernelNames[KID_COUNT] = {
    "bbox", "cell_hist", "cell_scatter", "cell_sort", "gather_sorted", "list_sweep", "bond_merge", "scan",
    "bondtest", "compact", "mirror", "zero", "gather_q", "bo_prime", "delta_prime", "bo_corr", "atom_state",
    "atom_energy", "tasks", "angles", "torsions", "hbonds", "hb_acceptors", "nonbonded", "back_s", "back_corr",
    "back_dp", "forces", "batch", "nb_reduce", "nb_energy", "energy_fold", "qeq_rows", "qeq_spmv", "qeq_vec", "sur_desc", "sur_net", "sur_pairw",
    "sur_gather", "sur_mirror", "qeq_half", "qeq_hreduce"};

int launch_forces(const DevParams* P, const Grid& g, const Lists& L, Work& W, const double* q,
                  hipStream_t side, hipEvent_t ev_fork, hipEvent_t ev_join, double* forces,
                  double* energies, Scratch& sc, Prof& pf, hipStream_t st) {
  const int64_t n = L.n, nb = L.nbond;
  pf.begin(KID_ZERO, st);
  (void)hipMemsetAsync(energies, 0, sizeof(double) * NTERMS, st);
  (void)hipMemsetAsync(W.epart, 0, sizeof(double) * ESLOT * NTERMS, st);
  (void)hipMemsetAsync(W.counters, 0, sizeof(unsigned long long) * 4, st);
  if (nb > 0) {
    (void)hipMemsetAsync(W.gbo, 0, sizeof(double4) * nb, st);
    (void)hipMemsetAsync(W.gvec, 0, sizeof(double4) * nb, st);
  }
  if (n > 0) (void)hipMemsetAsync(W.gSBO, 0, sizeof(double) * n, st);
  if (n > 0) (void)hipMemsetAsync(W.fhb, 0, sizeof(double4) * n, st);
  pf.end(st);
  if (n == 0) return hipGetLastError() == hipSuccess ? 0 : -1;
  const dim3 grid(xcd_grid(nblk(n, BS))), blk(BS);
#define LAUNCH(id, ...)                                  \
  do {                                                   \
    pf.begin(id, st);                                    \
    hipLaunchKernelGGL(__VA_ARGS__);                     \
    pf.end(st);                                          \
  } while (0)
  // the nonbonded kernels read neighbours by slot through a chunk table; the
  // per-cell kernel stages a cell's own stencil, so its slots must number it
  if (!L.far_slots || stencil_chunks(g) > NBC_MAXQ || (!L.nb_half && g.run != 1)) return -1;
  LAUNCH(KID_GATHER_Q, k_gather_q, grid, blk, 0, st, q, L.perm, L.xs, n, W.xq);
  // fork: the nonbonded term (writing fnb) runs on the side stream while the
  // bonded terms run on the caller's stream; they share only the energy
  // accumulators (atomic adds) until the join before the force gather.  With
  // side == st everything runs in order on the caller's stream.
  const bool fork = side != st;
  if (fork) {
    (void)hipEventRecord(ev_fork, st);
    (void)hipStreamWaitEvent(side, ev_fork, 0);
  }
  {
    const int ncell = g.nc[0] * g.nc[1] * g.nc[2], per_xcd = (ncell + 7) / 8;
#define LAUNCH_SIDE(id, ...)                             \
  do {                                                   \
    pf.begin(id, side);                                  \
    hipLaunchKernelGGL(__VA_ARGS__);                     \
    pf.end(side);                                        \
  } while (0)
    // one energy pair per run of the half evaluation, per cell otherwise
    const int nrun = g.nc[0] * g.nc[1] * run_rows(g), per_run_xcd = (nrun + 7) / 8;
    if (L.nb_half) {
      LAUNCH_SIDE(KID_NONBONDED, k_nonbonded_half, dim3(8u * (unsigned)per_run_xcd), dim3(NBH_BS), 0, side, P,
                  g, L, W, nrun, per_run_xcd, energies);
      if (g.reach == 1) LAUNCH_SIDE(KID_NB_REDUCE, k_nb_reduce<1>, grid, blk, 0, side, g, L, W);
      else LAUNCH_SIDE(KID_NB_REDUCE, k_nb_reduce<2>, grid, blk, 0, side, g, L, W);
    } else {
      LAUNCH_SIDE(KID_NONBONDED, k_nonbonded, dim3(8u * (unsigned)per_xcd), dim3(NBC_BS), 0, side, P, g, L,
                  W, ncell, per_xcd, energies);
    }
    const int nnbe = L.nb_half ? nrun : ncell;
    LAUNCH_SIDE(KID_NB_ENERGY, k_nb_energy, dim3((unsigned)std::min<int64_t>(nblk(nnbe, BS), 64)), blk, 0, side,
                nnbe, W.nbe, energies);
#undef LAUNCH_SIDE
  }
  if (fork) (void)hipEventRecord(ev_join, side);
  const dim3 grid_e(xcd_grid(nblk(std::max<int64_t>(nb, 1), BS)));   // one thread per bond entry
  LAUNCH(KID_BO_PRIME, k_bo_prime, grid_e, blk, 0, st, P, g, L, W);
  LAUNCH(KID_DELTA_PRIME, k_delta_prime, dim3(xcd_grid(nblk(4 * n, BS))), blk, 0, st, P, L, W);
  LAUNCH(KID_BO_CORR, k_bo_corr, grid_e, blk, 0, st, P, L, W);
  LAUNCH(KID_ATOM_STATE, k_atom_state, grid, blk, 0, st, P, L, W);
  LAUNCH(KID_ATOM_ENERGY, k_atom_energy, grid, blk, 0, st, P, L, W, energies);
  // task lists: count, prefix sums, fill
  const dim3 gridb(xcd_grid(nblk(std::max<int64_t>(std::max(nb, n), 1), BS)));
  LAUNCH(KID_TASKS, k_tasks<false>, gridb, blk, 0, st, P, L, W);
  (void)hipMemsetAsync(W.cnt_ang + nb, 0, sizeof(int32_t), st);
  (void)hipMemsetAsync(W.cnt_tor + nb, 0, sizeof(int32_t), st);
  (void)hipMemsetAsync(W.cnt_don + nb, 0, sizeof(int32_t), st);
  pf.begin(KID_SCAN, st);
  scan_i32(W.cnt_ang, W.off_ang, nb + 1, sc, st);
  scan_i32(W.cnt_tor, W.off_tor, nb + 1, sc, st);
  scan_i32(W.cnt_don, W.off_don, nb + 1, sc, st);
  pf.end(st);
  LAUNCH(KID_TASKS, k_tasks<true>, gridb, blk, 0, st, P, L, W);
  const int64_t bt = (L.bound_tor + BS - 1) / BS;
  const dim3 gt((unsigned)(bt < 1 ? 1 : (bt > 8192 ? 8192 : bt)));
  LAUNCH(KID_ANGLES, k_angles, dim3(xcd_grid((L.bound_ang + BS - 1) / BS)), blk, 0,
         st, P, L, W, energies);
  LAUNCH(KID_TORSIONS, k_torsions, gt, blk, 0, st, P, L, W, energies);
  LAUNCH(KID_HBONDS, k_hbonds, dim3(xcd_grid((L.bound_don + BS / HB_DROW - 1) / (BS / HB_DROW))), blk, 0, st, P, g,
         L, W, energies);
  LAUNCH(KID_HB_ACC, k_hb_acceptors, dim3(xcd_grid(nblk(n, BS / HB_GROUP))), blk, 0, st, P, g, L, W);
  (void)hipMemcpyAsync(W.counters, W.off_ang + nb, sizeof(int32_t), hipMemcpyDeviceToDevice, st);
  (void)hipMemcpyAsync(W.counters + 1, W.off_tor + nb, sizeof(int32_t), hipMemcpyDeviceToDevice, st);
  LAUNCH(KID_BACK_S, k_back_s, dim3(xcd_grid(nblk(4 * n, BS))), blk, 0, st, L, W);
  LAUNCH(KID_BACK_CORR, k_back_corr, grid_e, blk, 0, st, P, L, W);
  LAUNCH(KID_BACK_DP, k_back_dp, dim3(xcd_grid(nblk(4 * n, BS))), blk, 0, st, L, W);
  // join: the force gather reads the nonbonded forces
  if (fork) (void)hipStreamWaitEvent(st, ev_join, 0);
  LAUNCH(KID_FORCES, k_forces, dim3(xcd_grid(nblk(4 * n, BS))), blk, 0, st, L, W, forces);
  LAUNCH(KID_ENERGY_FOLD, k_energy_fold, dim3(1), dim3(64), 0, st, W.epart, energies);
#undef LAUNCH
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// ---------------------------------------------------------------------------
// velocity Verlet pieces (caller order)
// ---------------------------------------------------------------------------
__global__ void k_kick(int64_t n, double* __restrict__ vel, const double* __restrict__ f,
                       const int32_t* __restrict__ type, const DevParams* __restrict__ P, double hdt) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double s = hdt * ACC_CONV / P->atom[type[i]].mass;
  for (int k = 0; k < 3; ++k) vel[3 * i + k] += s * f[3 * i + k];
}

// positions advance by dt v; with wrap, every coordinate is put back into
// [0, L) of a periodic box (lists kept over several steps need continuous
// positions between their rebuilds, and wrap only then)
__global__ void k_drift(int64_t n, double* __restrict__ pos, const double* __restrict__ vel, double dt,
                        Grid g, int wrap) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int k = 0; k < 3; ++k) {
    double x = pos[3 * i + k] + dt * vel[3 * i + k];
    if (g.periodic && wrap) x -= g.L[k] * floor(x * g.invL[k]);
    pos[3 * i + k] = x;
  }
}

__global__ void k_wrap(int64_t n, double* __restrict__ pos, Grid g) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int k = 0; k < 3; ++k) {
    const double x = pos[3 * i + k];
    pos[3 * i + k] = x - g.L[k] * floor(x * g.invL[k]);
  }
}

__global__ void k_kinetic(int64_t n, const double* __restrict__ vel, const int32_t* __restrict__ type,
                          const DevParams* __restrict__ P, double* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  double ke = 0.0;
  if (i < n) {
    const double m = P->atom[type[i]].mass;
    ke = 0.5 * m * (vel[3 * i] * vel[3 * i] + vel[3 * i + 1] * vel[3 * i + 1] + vel[3 * i + 2] * vel[3 * i + 2]) /
         ACC_CONV;
  }
  block_add<BS>(ke, out);
}

int launch_kick(int64_t n, double* vel, const double* forces, const int32_t* type, const DevParams* P,
                double half_dt, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_kick, dim3(nblk(n, BS)), dim3(BS), 0, st, n, vel, forces, type, P, half_dt);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}
int launch_drift(int64_t n, double* pos, const double* vel, double dt, const Grid& g, bool wrap, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_drift, dim3(nblk(n, BS)), dim3(BS), 0, st, n, pos, vel, dt, g, wrap ? 1 : 0);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}
int launch_wrap(int64_t n, double* pos, const Grid& g, hipStream_t st) {
  if (n > 0 && g.periodic) hipLaunchKernelGGL(k_wrap, dim3(nblk(n, BS)), dim3(BS), 0, st, n, pos, g);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}
int launch_kinetic(int64_t n, const double* vel, const int32_t* type, const DevParams* P, double* out,
                   hipStream_t st) {
  (void)hipMemsetAsync(out, 0, sizeof(double), st);
  if (n > 0) hipLaunchKernelGGL(k_kinetic, dim3(nblk(n, BS)), dim3(BS), 0, st, n, vel, type, P, out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace rx
