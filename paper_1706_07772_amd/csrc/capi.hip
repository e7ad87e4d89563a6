// C ABI of the library: context, parameter upload, buffer management and
// the three calls of the hot path (build lists, compute forces, MD step).
#include <cmath>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <string>
#include <vector>

#include "internal.h"

using namespace rx;


namespace {

int fail(reaxff_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define HIPCHK(ctx, expr)                                                            \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess)                                                            \
      return fail(ctx, REAXFF_ERR_HIP, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

template <class T>
int grow(reaxff_ctx* c, T*& p, int64_t& cap, int64_t need, double slack = 1.2) {
  if (need <= cap && p) return 0;
  if (p) (void)hipFree(p);
  p = nullptr;
  const int64_t n = std::max<int64_t>((int64_t)(need * slack) + 64, 64);
  hipError_t e = hipMalloc(&p, sizeof(T) * n);
  if (e != hipSuccess) {
    cap = 0;
    return fail(c, REAXFF_ERR_HIP, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  cap = n;
  return 0;
}

// largest r with raw uncorrected bond order >= bo_cut for a pair (decreasing in r)
double bond_reach(const PairP& p, double bo_cut, double rmax) {
  auto raw = [&](double r) {
    double s = 0, pi = 0, pp = 0;
    if (p.r_s > 0) s = (1.0 + bo_cut) * std::exp(p.p_bo1 * std::pow(r / p.r_s, p.p_bo2));
    if (p.r_p > 0) pi = std::exp(p.p_bo3 * std::pow(r / p.r_p, p.p_bo4));
    if (p.r_pp > 0) pp = std::exp(p.p_bo5 * std::pow(r / p.r_pp, p.p_bo6));
    return s + pi + pp;
  };
  const bool mono = (p.r_s <= 0 || (p.p_bo1 < 0 && p.p_bo2 > 0)) &&
                    (p.r_p <= 0 || (p.p_bo3 < 0 && p.p_bo4 > 0)) &&
                    (p.r_pp <= 0 || (p.p_bo5 < 0 && p.p_bo6 > 0));
  if (!mono) return rmax;
  if (raw(rmax) >= bo_cut) return rmax;
  double lo = 1e-6, hi = rmax;
  if (raw(lo) < bo_cut) return 0.0;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (raw(mid) >= bo_cut) lo = mid;
    else hi = mid;
  }
  // generous margin: the exact test is applied after this prefilter
  return std::min(rmax, hi * (1.0 + 1e-3) + 1e-3);
}

void fill_dev_params(const reaxff_params& p, const reaxff_cutoffs& c, DevParams& d) {
  std::memset(&d, 0, sizeof(d));
  d.p_boc1 = p.p_boc1; d.p_boc2 = p.p_boc2; d.p_coa2 = p.p_coa2; d.p_coa3 = p.p_coa3;
  d.p_coa4 = p.p_coa4; d.p_ovun3 = p.p_ovun3; d.p_ovun4 = p.p_ovun4; d.p_ovun6 = p.p_ovun6;
  d.p_ovun7 = p.p_ovun7; d.p_ovun8 = p.p_ovun8; d.p_val6 = p.p_val6; d.p_val8 = p.p_val8;
  d.p_val9 = p.p_val9; d.p_val10 = p.p_val10; d.p_pen2 = p.p_pen2; d.p_pen3 = p.p_pen3;
  d.p_pen4 = p.p_pen4; d.p_tor2 = p.p_tor2; d.p_tor3 = p.p_tor3; d.p_tor4 = p.p_tor4;
  d.p_cot2 = p.p_cot2; d.p_vdW1 = p.p_vdW1; d.p_lp1 = p.p_lp1; d.inv_p_vdW1 = 1.0 / p.p_vdW1;
  d.r_nonb = c.r_nonb; d.r_bond = c.r_bond; d.r_hb = c.r_hb; d.bo_cut = c.bo_cut;
  d.thb_cut = c.thb_cut; d.thb_cutsq = c.thb_cutsq; d.hb_bo_cut = c.hb_bo_cut;
  d.rn2 = c.r_nonb * c.r_nonb; d.rh2 = c.r_hb * c.r_hb; d.inv_r_nonb = 1.0 / c.r_nonb;
  for (int t = 0; t < NT; ++t) {
    AtomP& a = d.atom[t];
    a.val = p.val[t]; a.val_e = p.val_e[t]; a.val_boc = p.val_boc[t]; a.val_ang = p.val_ang[t];
    a.mass = p.mass[t]; a.p_lp2 = p.p_lp2[t]; a.p_ovun2 = p.p_ovun2[t]; a.p_ovun5 = p.p_ovun5[t];
    a.p_val3 = p.p_val3[t]; a.p_val5 = p.p_val5[t];
    a.nlp_opt = 0.5 * (p.val_e[t] - p.val[t]);
    a.hbond = (int32_t)std::lround(p.p_hbond[t]);
  }
  for (int i = 0; i < NT; ++i)
    for (int j = 0; j < NT; ++j) {
      PairP& q = d.pair[i * NT + j];
      q.r_s = p.r_s[i][j]; q.r_p = p.r_p[i][j]; q.r_pp = p.r_pp[i][j];
      q.ln_r_s = q.r_s > 0 ? std::log(q.r_s) : 0.0;
      q.ln_r_p = q.r_p > 0 ? std::log(q.r_p) : 0.0;
      q.ln_r_pp = q.r_pp > 0 ? std::log(q.r_pp) : 0.0;
      q.p_bo1 = p.p_bo1[i][j]; q.p_bo2 = p.p_bo2[i][j]; q.p_bo3 = p.p_bo3[i][j];
      q.p_bo4 = p.p_bo4[i][j]; q.p_bo5 = p.p_bo5[i][j]; q.p_bo6 = p.p_bo6[i][j];
      q.D_s = p.D_s[i][j]; q.D_p = p.D_p[i][j]; q.D_pp = p.D_pp[i][j];
      q.p_be1 = p.p_be1[i][j]; q.p_be2 = p.p_be2[i][j]; q.p_ovun1 = p.p_ovun1[i][j];
      q.p_boc3 = p.p_boc3[i][j]; q.p_boc4 = p.p_boc4[i][j]; q.p_boc5 = p.p_boc5[i][j];
      q.D_vdw = p.D_vdw[i][j]; q.alpha = p.alpha[i][j]; q.inv_r_vdw = 1.0 / p.r_vdw[i][j];
      q.gw_pow = std::pow(p.gamma_w[i][j], -p.p_vdW1);
      q.g3 = std::pow(p.gamma[i][j], -3.0);
      q.e_core = p.e_core[i][j]; q.a_core = p.a_core[i][j]; q.inv_r_core = 1.0 / p.r_core[i][j];
      const double reach = bond_reach(q, c.bo_cut, c.r_bond);
      q.reach2 = reach * reach;
    }
  for (int i = 0; i < NT; ++i)
    for (int j = 0; j < NT; ++j)
      for (int k = 0; k < NT; ++k) {
        AngleP& a = d.angle[(i * NT + j) * NT + k];
        a.theta00_rad = p.theta00[i][j][k] * (PI / 180.0);
        a.p_val1 = p.p_val1[i][j][k]; a.p_val2 = p.p_val2[i][j][k]; a.p_val4 = p.p_val4[i][j][k];
        a.p_val7 = p.p_val7[i][j][k]; a.p_pen1 = p.p_pen1[i][j][k]; a.p_coa1 = p.p_coa1[i][j][k];
        HbP& h = d.hb[(i * NT + j) * NT + k];
        h.r0hb = p.r0hb[i][j][k]; h.p_hb1 = p.p_hb1[i][j][k]; h.p_hb2 = p.p_hb2[i][j][k];
        h.p_hb3 = p.p_hb3[i][j][k];
        for (int l = 0; l < NT; ++l) {
          TorsP& t = d.tors[((i * NT + j) * NT + k) * NT + l];
          t.V1 = p.V1[i][j][k][l]; t.V2 = p.V2[i][j][k][l]; t.V3 = p.V3[i][j][k][l];
          t.p_tor1 = p.p_tor1[i][j][k][l]; t.p_cot1 = p.p_cot1[i][j][k][l];
        }
      }
}

// grid: cells at least r_nonb/2 wide, +-2 cell stencil
// cells at least r_nonb / reach wide, so every pair within r_nonb lies within
// +-reach cells in each dimension
void make_grid(Grid& g, bool periodic, const double* box, const double lo[3], const double hi[3],
               double r_nonb, int reach) {
  g.periodic = periodic ? 1 : 0;
  g.reach = reach;
  const double wmin = r_nonb / reach;
  for (int k = 0; k < 3; ++k) {
    double ext;
    if (periodic) {
      g.lo[k] = 0.0;
      ext = box[k];
      g.L[k] = box[k];
      g.invL[k] = 1.0 / box[k];
    } else {
      g.lo[k] = lo[k];
      ext = std::max(hi[k] - lo[k], 1e-9);
      g.L[k] = 0.0;
      g.invL[k] = 0.0;
    }
    int nc = (int)std::floor(ext / wmin);
    if (nc < 1) nc = 1;
    g.nc[k] = nc;
    g.invw[k] = nc / ext;
    g.full[k] = nc < 2 * reach + 1 ? 1 : 0;
    g.span[k] = nc < 2 * reach + 1 ? nc : 2 * reach + 1;
  }
  g.run = 1;
}

int alloc_atoms(reaxff_ctx* c, int64_t n) {
  if (n + 1 <= c->cap_n && c->L.perm) return 0;
  int64_t cap = 0;
  const int64_t need = n + 1;
  int64_t tmp;
#define G(ptr) do { tmp = c->cap_n; if (grow(c, ptr, tmp, need)) return REAXFF_ERR_HIP; cap = tmp; } while (0)
  G(c->L.perm); G(c->L.type_s); G(c->L.xs); G(c->L.far_cnt); G(c->L.far_lo); G(c->L.bond_off); G(c->L.hb_cnt);
  G(c->L.ha_cnt);
  G(c->sc.cid); G(c->sc.cell_s); G(c->sc.cnt_cand); G(c->sc.cnt_bond); G(c->sc.cnt_lo);
  G(c->W.dp); G(c->W.ast); G(c->W.gS); G(c->W.gSig); G(c->W.gSBO); G(c->W.gStot); G(c->W.gDp);
  G(c->W.gRso);
  G(c->W.fnb); G(c->W.fhb); G(c->W.xq); G(c->W.don_rng); G(c->W.nv);
#undef G

  c->cap_n = cap;
  return 0;
}

// per-entry work arrays for nb bond entries; the entries themselves (bond_j,
// bond_mir) in the context's storage, or in the caller's (ext)
int alloc_bonds(reaxff_ctx* c, int64_t nb, const reaxff_lists* ext) {
  if (!(nb + 1 <= c->cap_bond && c->W.bd)) {
    int64_t cap = 0, tmp;
#define G(ptr) do { tmp = c->cap_bond; if (grow(c, ptr, tmp, nb + 1)) return REAXFF_ERR_HIP; cap = tmp; } while (0)
    G(c->L.bond_i); G(c->W.bd); G(c->W.bop); G(c->W.dbop); G(c->W.bo);
    G(c->W.gbo); G(c->W.gvec); G(c->W.gup);
    G(c->W.cnt_ang); G(c->W.cnt_tor); G(c->W.cnt_don); G(c->W.off_ang); G(c->W.off_tor); G(c->W.off_don);
    G(c->W.bo1);
#undef G
    c->cap_bond = cap;
  }
  if (ext) {
    c->L.bond_j = ext->bond_j;
    c->L.bond_mir = ext->bond_mir;
  } else {
    if (!(nb + 1 <= c->cap_own_bj && c->own_bj)) {
      int64_t t = c->cap_own_bj;
      if (grow(c, c->own_bj, t, nb + 1)) return REAXFF_ERR_HIP;
      int64_t t2 = c->cap_own_bj;
      if (grow(c, c->own_mir, t2, nb + 1)) return REAXFF_ERR_HIP;
      c->cap_own_bj = t;
    }
    c->L.bond_j = c->own_bj;
    c->L.bond_mir = c->own_mir;
  }
  return 0;
}

int set_task_bounds(reaxff_ctx* c, const int64_t* th) {
  c->L.bound_ang = th[1];
  c->L.bound_tor = th[2];
  c->L.bound_don = th[3];
  int64_t t = c->W.cap_ang;
  if (grow(c, c->W.ang, t, std::max<int64_t>(c->L.bound_ang, 1))) return REAXFF_ERR_HIP;
  c->W.cap_ang = t;
  t = c->W.cap_tor;
  if (grow(c, c->W.tor, t, std::max<int64_t>(c->L.bound_tor, 1))) return REAXFF_ERR_HIP;
  c->W.cap_tor = t;
  t = c->W.cap_don;
  if (grow(c, c->W.don, t, std::max<int64_t>(c->L.bound_don, 1))) return REAXFF_ERR_HIP;
  int64_t t2 = c->W.cap_don;
  if (grow(c, c->W.donrec, t2, std::max<int64_t>(c->L.bound_don, 1))) return REAXFF_ERR_HIP;
  c->W.cap_don = t;
  return 0;
}

// Lists for the current positions with the sorted order, cells, far and H
// rows of the last build kept: when skin lists are on, the build is recent
// enough (fewer than `every` refreshes) and no atom has moved more than
// skin / 2 since it, only the sorted positions and the bond list (bond test
// over the stored candidates, compressed rows, mirror index, task bounds) are
// made again.  Otherwise a full build, after wrapping pos_mut into a
// periodic box when it is given.  *rebuilt tells which happened.
int build_lists_impl(reaxff_ctx* c, int64_t n, const double* pos, const int32_t* type, const double* box,
                     reaxff_lists* ext, hipStream_t st);

int refresh_lists(reaxff_ctx* c, int64_t n, const double* pos, double* pos_mut, const int32_t* type,
                  const double* box, int32_t* rebuilt, hipStream_t st) {
  if (c->ext_on && c->built)
    return fail(c, REAXFF_ERR_STATE, "lists in caller buffers are built again with reaxff_build_lists_into");
  bool full = !(c->skin > 0.0) || !c->built || n != c->L.n || n == 0 || (box != nullptr) != c->periodic ||
              c->since + 1 >= c->every;
  if (!full && box)
    for (int k = 0; k < 3; ++k) full = full || box[k] != c->box[k];
  if (!full) {
    HIPCHK(c, hipSetDevice(c->device));
    c->built = false;
    c->forces_done = false;
    Scratch& sc = c->sc;
    HIPCHK(c, hipMemsetAsync(c->dmax, 0, sizeof(unsigned long long), st));
    if (launch_refresh_gather(pos, n, c->xref, c->L, c->dmax, c->prof, st))
      return fail(c, REAXFF_ERR_HIP, "refresh gather failed");
    int32_t need[8];
    int32_t nb = 0;
    unsigned long long dm = 0;
    int64_t* th = sc.totals_host;
    for (int attempt = 0;; ++attempt) {
      HIPCHK(c, hipMemsetAsync(sc.need, 0, sizeof(int32_t) * 8, st));
      HIPCHK(c, hipMemsetAsync(sc.totals, 0, sizeof(int64_t) * 8, st));
      HIPCHK(c, hipMemsetAsync(sc.tslot, 0, sizeof(int64_t) * 8 * ESLOT, st));
      HIPCHK(c, hipMemsetAsync(sc.nslot, 0, sizeof(int32_t) * ESLOT, st));
      if (launch_bondtest(c->dp, c->grid, n, c->cut.r_bond * c->cut.r_bond, sc, c->L, c->prof, st))
        return fail(c, REAXFF_ERR_HIP, "bond test launch failed");
      HIPCHK(c, hipMemsetAsync(sc.cnt_bond + n, 0, sizeof(int32_t), st));
      c->prof.begin(KID_SCAN, st);
      const int src = scan_i32(sc.cnt_bond, c->L.bond_off, n + 1, sc, st);
      c->prof.end(st);
      if (src) return fail(c, REAXFF_ERR_HIP, "scan failed");
      HIPCHK(c, hipMemcpyAsync(th, sc.totals, sizeof(int64_t) * 8, hipMemcpyDeviceToHost, st));
      HIPCHK(c, hipMemcpyAsync(&nb, c->L.bond_off + n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
      HIPCHK(c, hipMemcpyAsync(need, sc.need, sizeof(need), hipMemcpyDeviceToHost, st));
      HIPCHK(c, hipMemcpyAsync(&dm, c->dmax, sizeof(dm), hipMemcpyDeviceToHost, st));
      HIPCHK(c, hipStreamSynchronize(st));
      double d2;
      std::memcpy(&d2, &dm, sizeof(d2));
      if (!(std::sqrt(d2) <= 0.5 * c->skin)) {   // moved too far (or non-finite): build again
        full = true;
        break;
      }
      if (need[2] <= sc.bond_w) break;
      if (attempt >= 3) return fail(c, REAXFF_ERR_CAPACITY, "bond staging width did not converge");
      sc.bond_w = (int32_t)(need[2] * 1.15) + 16;
      int64_t t = sc.cap_bondt;
      if (grow(c, sc.bond_t, t, n * (int64_t)sc.bond_w, 1.0)) return REAXFF_ERR_HIP;
      sc.cap_bondt = t;
    }
    if (!full) {
      c->L.nbond = nb;
      if (set_task_bounds(c, th)) return REAXFF_ERR_HIP;
      if (alloc_bonds(c, std::max<int64_t>(c->L.nbond, 1), nullptr)) return REAXFF_ERR_HIP;
      if (launch_compact(n, sc, c->L, c->prof, st)) return fail(c, REAXFF_ERR_HIP, "compact launch failed");
      ++c->since;
      ++c->nrefresh;
      c->built = true;
      if (rebuilt) *rebuilt = 0;
      return REAXFF_OK;
    }
  }
  if (pos_mut && box) {
    // wrap into the box before building (the grid of the last build is only
    // used for its box edges here)
    Grid g{};
    g.periodic = 1;
    for (int k = 0; k < 3; ++k) {
      g.L[k] = box[k];
      g.invL[k] = 1.0 / box[k];
    }
    if (launch_wrap(n, pos_mut, g, st)) return fail(c, REAXFF_ERR_HIP, "wrap launch failed");
  }
  if (rebuilt) *rebuilt = 1;
  return build_lists_impl(c, n, pos, type, box, nullptr, st);
}

}  // namespace

extern "C" {

int64_t reaxff_params_size(void) { return (int64_t)sizeof(reaxff_params); }

const char* reaxff_strerror(int code) {
  switch (code) {
    case REAXFF_OK: return "ok";
    case REAXFF_ERR_ARG: return "invalid argument";
    case REAXFF_ERR_CAPACITY: return "buffer capacity exceeded";
    case REAXFF_ERR_BOX: return "periodic box edge below 2 r_nonb";
    case REAXFF_ERR_HIP: return "HIP runtime error";
    case REAXFF_ERR_NONFINITE: return "non-finite input";
    case REAXFF_ERR_STATE: return "call out of order";
    case REAXFF_ERR_CONVERGENCE: return "iterative solver did not converge";
    default: return "unknown error";
  }
}

const char* reaxff_last_error(const reaxff_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

// the symmetries reaxff_params states: pair tables [i][j] = [j][i], angle
// tables [i][j][k] = [k][j][i], torsion tables [i][j][k][l] = [l][k][j][i]
// (a bond found from one atom must be found from the other, and each
// interaction has one parameter set whichever end it is read from)
static bool params_symmetric(const reaxff_params& p) {
  const double* pair = &p.r_s[0][0];
  const int npair = (int)((&p.a_core[3][3] - pair) + 1) / 16;
  for (int t = 0; t < npair; ++t)
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j)
        if (!(pair[16 * t + 4 * i + j] == pair[16 * t + 4 * j + i])) return false;
  const double* ang = &p.theta00[0][0][0];
  const int nang = (int)((&p.p_coa1[3][3][3] - ang) + 1) / 64;
  for (int t = 0; t < nang; ++t)
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j)
        for (int k = 0; k < 4; ++k)
          if (!(ang[64 * t + 16 * i + 4 * j + k] == ang[64 * t + 16 * k + 4 * j + i])) return false;
  const double* tor = &p.V1[0][0][0][0];
  const int ntor = (int)((&p.p_cot1[3][3][3][3] - tor) + 1) / 256;
  for (int t = 0; t < ntor; ++t)
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j)
        for (int k = 0; k < 4; ++k)
          for (int l = 0; l < 4; ++l)
            if (!(tor[256 * t + 64 * i + 16 * j + 4 * k + l] == tor[256 * t + 64 * l + 16 * k + 4 * j + i]))
              return false;
  return true;
}

int reaxff_create(const reaxff_params* params, const reaxff_cutoffs* cutoffs, int device,
                  reaxff_ctx** out) {
  if (!params || !out) return REAXFF_ERR_ARG;
  *out = nullptr;
  if (!params_symmetric(*params)) return REAXFF_ERR_ARG;
  auto* c = new reaxff_ctx();
  c->device = device;
  c->hp = *params;
  if (cutoffs) c->cut = *cutoffs;
  else c->cut = reaxff_cutoffs{10.0, 5.0, 7.5, 0.01, 0.001, 1e-5, 0.01};
  c->L.far_slots = 1;
  const reaxff_cutoffs& cc = c->cut;
  if (!(cc.r_nonb > 0 && cc.r_bond > 0 && cc.r_hb > 0 && cc.r_bond <= cc.r_nonb &&
        cc.r_hb <= cc.r_nonb && cc.bo_cut >= 0)) {
    delete c;
    return REAXFF_ERR_ARG;
  }
  if (hipSetDevice(device) != hipSuccess) {
    delete c;
    return REAXFF_ERR_HIP;
  }
  fill_dev_params(c->hp, c->cut, c->hd);
  if (batched_scratch_init(device) != (int)hipSuccess) {
    delete c;
    return REAXFF_ERR_HIP;
  }
  if (hipMalloc(&c->dp, sizeof(DevParams)) != hipSuccess ||
      hipMemcpy(c->dp, &c->hd, sizeof(DevParams), hipMemcpyHostToDevice) != hipSuccess ||
      hipMalloc(&c->sc.flag, sizeof(int32_t) * 4) != hipSuccess ||
      hipMalloc(&c->sc.totals, sizeof(int64_t) * 8) != hipSuccess ||
      hipMalloc(&c->sc.tslot, sizeof(int64_t) * 8 * ESLOT) != hipSuccess ||
      hipMalloc(&c->sc.nslot, sizeof(int32_t) * ESLOT) != hipSuccess ||
      hipMalloc(&c->sc.need, sizeof(int32_t) * 8) != hipSuccess ||
      hipHostMalloc(&c->sc.totals_host, sizeof(int64_t) * 8, hipHostMallocDefault) != hipSuccess ||
      hipMalloc(&c->W.counters, sizeof(unsigned long long) * 4) != hipSuccess ||
      hipMalloc(&c->dmax, sizeof(unsigned long long)) != hipSuccess ||
      hipMalloc(&c->W.epart, sizeof(double) * ESLOT * NTERMS) != hipSuccess ||
      hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess) {
    reaxff_destroy(c);
    return REAXFF_ERR_HIP;
  }
  *out = c;
  return REAXFF_OK;
}

void reaxff_destroy(reaxff_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  void* ptrs[] = {c->dp, c->L.perm, c->L.type_s, c->L.xs, c->L.cell_start, c->L.far_cnt,
                  c->own_far, c->L.bond_off, c->own_bj, c->own_mir, c->L.hb_cnt, c->own_hb,
                  c->L.ha_cnt, c->L.ha_j,
                  c->W.bd, c->W.bop, c->W.dbop, c->W.bo, c->W.gbo, c->W.gvec, c->W.gup, c->W.dp,
                  c->W.ast, c->W.gS, c->W.gSig, c->W.gRso, c->W.gSBO, c->W.gStot, c->W.gDp, c->W.fnb, c->W.fhb, c->W.don_rng, c->W.nv, c->W.bo1,
                  c->W.xq, c->W.counters, c->W.epart, c->W.cnt_ang, c->W.cnt_tor, c->W.cnt_don,
                  c->W.off_ang, c->W.off_tor, c->W.off_don, c->W.ang, c->W.tor, c->W.don, c->W.donrec, c->L.far_lo, c->W.nbpart, c->W.nbtab, c->W.nbe,
                  c->L.bond_i, c->sc.cid, c->sc.cell_s, c->sc.cell_count,
                  c->sc.cell_cursor, c->sc.flag, c->sc.cnt_cand, c->sc.cnt_lo, c->sc.cnt_bond,
                  c->sc.cand_j, c->sc.bond_t, c->sc.need, c->sc.tslot, c->sc.nslot,
                  c->sc.part, c->sc.totals, c->sc.scan_tmp};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (c->sc.totals_host) (void)hipHostFree(c->sc.totals_host);
  for (void* p : {(void*)c->dp_list, (void*)c->xref, (void*)c->dmax})
    if (p) (void)hipFree(p);
  {
    rx::Qeq& Q = c->qeq;
    void* qp[] = {Q.hj, Q.hv, Q.hcnt, Q.part, Q.tab, Q.x, Q.r, Q.p, Q.ap, Q.red, Q.need, Q.hist[0], Q.hist[1], Q.hist[2], Q.hist[3]};
    for (void* p : qp)
      if (p) (void)hipFree(p);
    if (Q.red_host) (void)hipHostFree(Q.red_host);
    rx::Masked& Mk = c->masked;
    void* mp[] = {Mk.cid, Mk.sel, Mk.idx, Mk.stype, Mk.flag, Mk.mark, Mk.mark2, Mk.spos, Mk.sq, Mk.sforce,
                  Mk.senergy, Mk.part};
    for (void* p : mp)
      if (p) (void)hipFree(p);
    rx::Species& S = c->species;
    void* sp[] = {S.parent, S.flag, S.rank, S.counts, S.order, S.order2, S.sid, S.key, S.key2, S.tmp};
    for (void* p : sp)
      if (p) (void)hipFree(p);
  }
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  if (c->ev_join) (void)hipEventDestroy(c->ev_join);
  if (c->side) (void)hipStreamDestroy(c->side);
  delete c;
}

int reaxff_build_lists(reaxff_ctx* c, int64_t n, const double* pos, const int32_t* type,
                       const double* box, hipStream_t st) {
  if (!c) return REAXFF_ERR_ARG;
  return build_lists_impl(c, n, pos, type, box, nullptr, st);
}

int reaxff_build_lists_into(reaxff_ctx* c, int64_t n, const double* pos, const int32_t* type,
                            const double* box, reaxff_lists* lists, hipStream_t st) {
  if (!c) return REAXFF_ERR_ARG;
  if (!lists || lists->far_cap < 0 || lists->bond_cap < 0 || lists->hb_cap < 0 ||
      (lists->far_cap > 0 && !lists->far_j) || (lists->hb_cap > 0 && !lists->hb_j) ||
      (lists->bond_cap > 0 && (!lists->bond_j || !lists->bond_mir)))
    return fail(c, REAXFF_ERR_ARG, "reaxff_build_lists_into: bad list descriptor");
  return build_lists_impl(c, n, pos, type, box, lists, st);
}

int reaxff_compute_forces_from(reaxff_ctx* c, int64_t n, const double* pos, const int32_t* type, const double* q,
                               const double* box, const reaxff_lists* lists, double* forces, double* energies,
                               hipStream_t st) {
  if (!c) return REAXFF_ERR_ARG;
  if (!lists) return fail(c, REAXFF_ERR_ARG, "null list descriptor");
  if (!c->built || !c->ext_on || lists->far_j != c->L.far_j || lists->hb_j != c->L.hb_j ||
      lists->bond_j != c->L.bond_j || lists->bond_mir != c->L.bond_mir)
    return fail(c, REAXFF_ERR_STATE, "lists were not built into these buffers by the last build");
  return reaxff_compute_forces(c, n, pos, type, q, box, forces, energies, st);
}

}  // extern "C"

namespace {

int build_lists_impl(reaxff_ctx* c, int64_t n, const double* pos, const int32_t* type, const double* box,
                     reaxff_lists* ext, hipStream_t st) {
  if (n < 0 || (n > 0 && (!pos || !type))) return fail(c, REAXFF_ERR_ARG, "bad n or null pointer");
  if (n >= (int64_t)INT32_MAX / 2) return fail(c, REAXFF_ERR_ARG, "n too large for 32-bit indices");
  HIPCHK(c, hipSetDevice(c->device));
  c->built = false;
  c->forces_done = false;
  c->periodic = box != nullptr;
  // list cutoff: r_nonb, plus the skin when lists are kept over several steps
  const double r_list = c->cut.r_nonb + c->skin;
  if (box) {
    for (int k = 0; k < 3; ++k) {
      if (!(std::isfinite(box[k]) && box[k] >= 2.0 * r_list))
        return fail(c, REAXFF_ERR_BOX, "periodic box edge below 2 (r_nonb + skin)");
      c->box[k] = box[k];
    }
  }
  if (alloc_atoms(c, n)) return REAXFF_ERR_HIP;
  c->L.n = n;
  // bounding box + finiteness
  const int nparts = (int)std::min<int64_t>(std::max<int64_t>((n + 255) / 256, 1), 1024);
  if (grow(c, c->sc.part, c->cap_part, 6 * nparts)) return REAXFF_ERR_HIP;
  double lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1};
  if (n > 0) {
    HIPCHK(c, hipMemsetAsync(c->sc.flag, 0, sizeof(int32_t) * 4, st));
    launch_bbox(pos, type, n, c->sc.part, nparts, c->sc.flag, c->prof, st);
    std::vector<double> part(6 * nparts);
    int32_t flag = 0;
    HIPCHK(c, hipMemcpyAsync(part.data(), c->sc.part, sizeof(double) * 6 * nparts,
                             hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipMemcpyAsync(&flag, c->sc.flag, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    if (flag & 1) return fail(c, REAXFF_ERR_ARG, "atom type out of range 0..3");
    for (int k = 0; k < 3; ++k) { lo[k] = 1e300; hi[k] = -1e300; }
    for (int b = 0; b < nparts; ++b)
      for (int k = 0; k < 3; ++k) {
        lo[k] = std::min(lo[k], part[6 * b + k]);
        hi[k] = std::max(hi[k], part[6 * b + 3 + k]);
      }
    for (int k = 0; k < 3; ++k)
      if (!(lo[k] > -1e307) || !std::isfinite(hi[k]) || !std::isfinite(lo[k]))
        return fail(c, REAXFF_ERR_NONFINITE, "non-finite position");
  }
  // stencil reach: +-2 cells of r_nonb/2 unless such cells would hold fewer than
  // about 4 atoms (short cutoffs), then +-1 cell of r_nonb (fuller wavefronts)
  int reach = 2;
  {
    double vol = 1.0;
    for (int k = 0; k < 3; ++k) vol *= c->periodic ? c->box[k] : std::max(hi[k] - lo[k], 1.0);
    const double per_cell = (double)n / vol * std::pow(0.5 * r_list, 3.0);
    if (per_cell < 4.0) reach = 1;
  }
  make_grid(c->grid, c->periodic, c->box, lo, hi, r_list, reach);
  c->grid.shift_ok = 0;
  if (c->periodic && n > 0) {
    bool ok = true;
    for (int k = 0; k < 3; ++k)
      ok = ok && lo[k] >= 0.0 && hi[k] < c->box[k] && c->grid.nc[k] >= 2 * reach + 3;
    c->grid.shift_ok = ok ? 1 : 0;
  }
  const int64_t ncell = (int64_t)c->grid.nc[0] * c->grid.nc[1] * c->grid.nc[2];
  if (ncell > (int64_t)INT32_MAX / 4) return fail(c, REAXFF_ERR_ARG, "cell grid too large");
  {
    int64_t cap = c->cap_cell, t = cap;
    if (grow(c, c->L.cell_start, t, ncell + 1)) return REAXFF_ERR_HIP;
    t = cap; if (grow(c, c->sc.cell_count, t, ncell + 1)) return REAXFF_ERR_HIP;
    t = cap; if (grow(c, c->sc.cell_cursor, t, ncell + 1)) return REAXFF_ERR_HIP;
    c->cap_cell = t;
  }
  if (n > 0) {
    if (launch_cell_sort(pos, type, n, c->grid, (int)ncell, c->sc, c->L, c->prof, st))
      return fail(c, REAXFF_ERR_HIP, "cell sort launch failed");
  }
  // staging widths: first estimates from the density, grown on overflow
  const int64_t nblock = (n + 63) / 64;
  {
    double vol = 1.0;
    for (int k = 0; k < 3; ++k) vol *= c->periodic ? c->box[k] : std::max(hi[k] - lo[k], 1.0);
    const double rho = n / vol;
    auto est = [&](double r) {
      const double m = rho * 4.18879 * r * r * r;
      return (int32_t)std::min<double>((double)std::max<int64_t>(n, 1), 1.3 * m + 32.0);
    };
    c->L.far_upper = c->L.far_slots && !c->upper_off && !c->grid.full[0] && !c->grid.full[1] &&
                     !c->grid.full[2];
    // runs of cells for the half evaluation: the longest (up to 8 cells)
    // whose upper window, at the mean density, fills at most 80% of the
    // kernel's LDS copy; a run needs run + 2 reach <= nc[2] in a periodic box
    if (c->L.far_upper && n > 0) {
      const int R = reach, C = 2 * R * R + 2 * R;   // upper columns besides the centre's
      const double per_cell = (double)n / (double)ncell;
      const double room = 0.8 * NB_HALF_CAP / std::max(per_cell, 1e-3) - 2.0 * R * C - R;
      int K = (int)std::floor(room / (C + 1));
      K = std::min(K, c->nb_run_max);
      K = std::min(K, c->periodic ? c->grid.nc[2] - 2 * R : c->grid.nc[2]);
      c->grid.run = std::max(K, 1);
    }
    if (c->L.far_w == 0) c->L.far_w = c->L.far_upper ? est(r_list) / 2 + 32 : est(r_list);
    if (c->L.hb_w == 0) c->L.hb_w = est(c->cut.r_hb + c->skin);
    if (c->L.ha_w == 0) c->L.ha_w = est(c->cut.r_hb + c->skin);
    if (c->sc.cand_w == 0) c->sc.cand_w = 32;
    if (c->sc.bond_w == 0) c->sc.bond_w = 16;
  }
  int64_t* th = c->sc.totals_host;
  int32_t need[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int32_t t32[2] = {0, 0};
  for (int attempt = 0;; ++attempt) {
    const int64_t rows = std::max<int64_t>(n, 1);
    {
      int64_t t;
      if (ext) {
        // the caller's row storage must hold n rows of the current widths
        const int64_t nf = rows * c->L.far_w, nh = rows * c->L.hb_w;
        if (ext->far_cap < nf || ext->hb_cap < nh) {
          ext->required[0] = nf;
          ext->required[1] = std::max<int64_t>(ext->required[1], 8 * rows);   // bonds: estimate until swept
          ext->required[2] = nh;
          return fail(c, REAXFF_ERR_CAPACITY, "caller list buffers too small; required[] holds the sizes");
        }
        c->L.far_j = ext->far_j;
        c->L.hb_j = ext->hb_j;
      } else {
        t = c->cap_far;
        if (grow(c, c->own_far, t, rows * c->L.far_w, 1.0)) return REAXFF_ERR_HIP;
        c->cap_far = t;
        t = c->cap_hb;
        if (grow(c, c->own_hb, t, rows * c->L.hb_w, 1.0)) return REAXFF_ERR_HIP;
        c->cap_hb = t;
        c->L.far_j = c->own_far;
        c->L.hb_j = c->own_hb;
      }
      t = c->sc.cap_cand;
      if (grow(c, c->sc.cand_j, t, rows * c->sc.cand_w, 1.0)) return REAXFF_ERR_HIP;
      c->sc.cap_cand = t;
      t = c->sc.cap_bondt;
      if (grow(c, c->sc.bond_t, t, rows * c->sc.bond_w, 1.0)) return REAXFF_ERR_HIP;
      c->sc.cap_bondt = t;
      t = c->cap_ha;
      if (grow(c, c->L.ha_j, t, rows * c->L.ha_w, 1.0)) return REAXFF_ERR_HIP;
      c->cap_ha = t;
    }
    if (n > 0 && launch_sweep(c->skin > 0.0 ? c->dp_list : c->dp, c->grid, n, (int)ncell,
                              c->cut.r_bond * c->cut.r_bond, true, c->sc, c->L,
                              c->prof, st))
      return fail(c, REAXFF_ERR_HIP, "sweep launch failed");
    if (n == 0) HIPCHK(c, hipMemsetAsync(c->sc.totals, 0, sizeof(int64_t) * 8, st));
    // bond offsets: counts with a trailing zero, exclusive scan, last element = total
    HIPCHK(c, hipMemsetAsync(c->sc.cnt_bond + n, 0, sizeof(int32_t), st));
    c->prof.begin(KID_SCAN, st);
    const int src = scan_i32(c->sc.cnt_bond, c->L.bond_off, n + 1, c->sc, st);
    c->prof.end(st);
    if (src) return fail(c, REAXFF_ERR_HIP, "scan failed");
    // the one host synchronisation: list totals and overflow report
    HIPCHK(c, hipMemcpyAsync(th, c->sc.totals, sizeof(int64_t) * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipMemcpyAsync(&t32[0], c->L.bond_off + n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    if (n > 0)
      HIPCHK(c, hipMemcpyAsync(need, c->sc.need, sizeof(need), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    bool again = false;
    auto widen = [&](int32_t& w, int32_t nd) {
      if (nd > w) {
        w = (int32_t)(nd * 1.15) + 16;
        again = true;
      }
    };
    widen(c->L.far_w, need[0]);
    widen(c->sc.cand_w, need[1]);
    widen(c->sc.bond_w, need[2]);
    widen(c->L.hb_w, need[3]);
    widen(c->L.ha_w, need[4]);
    // an upper window beyond the LDS copy: shorter runs; upper-only rows
    // serve the half evaluation alone, so without it (one cell per run does
    // not fit either) sweep again with full rows and keep them for later
    // builds
    if (c->L.far_upper && n > 0 && !(need[5] > 0 && need[5] <= NB_HALF_CAP)) {
      if (c->grid.run > 1) {
        c->grid.run /= 2;
      } else {
        c->upper_off = true;
        c->L.far_upper = 0;
      }
      again = true;
    }
    if (!again) break;
    if (attempt >= 8) return fail(c, REAXFF_ERR_CAPACITY, "list widths did not converge");
  }
  c->L.nfar = c->L.far_upper ? th[0] : th[0] / 2;
  // half nonbonded evaluation when every cell's upper stencil fits in LDS
  // (need[5], reported by the sweep; zero when a dimension is covered whole)
  c->L.cell_of = c->sc.cell_s;
  {
    int64_t t = c->W.cap_nbe;
    if (grow(c, c->W.nbe, t, std::max<int64_t>(ncell, 1))) return REAXFF_ERR_HIP;
    c->W.cap_nbe = t;
  }
  c->L.nb_half = c->L.far_slots && n > 0 && need[5] > 0 && need[5] <= NB_HALF_CAP;
  if (c->L.nb_half) {
    const int64_t nrun = (int64_t)c->grid.nc[0] * c->grid.nc[1] * ((c->grid.nc[2] + c->grid.run - 1) / c->grid.run);
    int64_t t = c->W.cap_nbpart;
    if (grow(c, c->W.nbpart, t, nrun * 3 * (int64_t)NB_HALF_CAP, 1.0)) return REAXFF_ERR_HIP;
    c->W.cap_nbpart = t;
    t = c->W.cap_nbtab;
    if (grow(c, c->W.nbtab, t, nrun * (int64_t)NB_QMAX, 1.0)) return REAXFF_ERR_HIP;
    c->W.cap_nbtab = t;
  }
  c->L.nbond = t32[0];
  c->L.nhb = th[4];
  if (ext) {
    const int64_t rows = std::max<int64_t>(n, 1);
    ext->required[0] = rows * c->L.far_w;
    ext->required[1] = c->L.nbond;
    ext->required[2] = rows * c->L.hb_w;
    if (ext->bond_cap < c->L.nbond)
      return fail(c, REAXFF_ERR_CAPACITY, "caller bond buffers too small; required[] holds the sizes");
  }
  if (set_task_bounds(c, th)) return REAXFF_ERR_HIP;
  if (alloc_bonds(c, std::max<int64_t>(c->L.nbond, 1), ext)) return REAXFF_ERR_HIP;
  if (n > 0 && launch_compact(n, c->sc, c->L, c->prof, st))
    return fail(c, REAXFF_ERR_HIP, "compact launch failed");
  c->L.cut_check = c->skin > 0.0 ? 1 : 0;
  if (c->skin > 0.0 && n > 0) {
    // reference positions for the displacement check of later refreshes
    if (grow(c, c->xref, c->cap_xref, n)) return REAXFF_ERR_HIP;
    HIPCHK(c, hipMemcpyAsync(c->xref, c->L.xs, sizeof(double4) * n, hipMemcpyDeviceToDevice, st));
  }
  c->since = 0;
  ++c->nrebuild;
  c->ext_on = ext != nullptr;
  c->built = true;
  return REAXFF_OK;
}

}  // namespace

extern "C" {

int reaxff_compute_forces(reaxff_ctx* c, int64_t n, const double* pos, const int32_t* type,
                          const double* q, const double* box, double* forces, double* energies,
                          hipStream_t st) {
  if (!c) return REAXFF_ERR_ARG;
  if (!c->built || n != c->L.n) return fail(c, REAXFF_ERR_STATE, "lists not built for this n");
  if ((box != nullptr) != c->periodic) return fail(c, REAXFF_ERR_STATE, "box differs from build");
  if (box)
    for (int k = 0; k < 3; ++k)
      if (box[k] != c->box[k]) return fail(c, REAXFF_ERR_STATE, "box differs from build");
  if (!energies || (n > 0 && (!pos || !type || !q || !forces)))
    return fail(c, REAXFF_ERR_ARG, "null pointer");
  (void)pos; (void)type;   // the sorted copies made by the list build are used
  HIPCHK(c, hipSetDevice(c->device));
  if (launch_forces(c->dp, c->grid, c->L, c->W, q, c->overlap ? c->side : st, c->ev_fork, c->ev_join, forces,
                    energies, c->sc, c->prof, st))
    return fail(c, REAXFF_ERR_HIP, "force launch failed");
  c->forces_done = true;
  return REAXFF_OK;
}

int reaxff_step(reaxff_ctx* c, int64_t n, double* pos, double* vel, const int32_t* type,
                const double* q, const double* box, double dt, int32_t nsteps, double* forces,
                double* energies, hipStream_t st) {
  if (!c) return REAXFF_ERR_ARG;
  if (n < 0 || nsteps < 0 || !energies || (n > 0 && (!pos || !vel || !type || !q || !forces)))
    return fail(c, REAXFF_ERR_ARG, "bad argument");
  if (!(std::isfinite(dt))) return fail(c, REAXFF_ERR_ARG, "bad time step");
  HIPCHK(c, hipSetDevice(c->device));
  const int64_t row = REAXFF_NTERMS + 1;
  int rc;
  if ((rc = reaxff_build_lists(c, n, pos, type, box, st))) return rc;
  if ((rc = reaxff_compute_forces(c, n, pos, type, q, box, forces, energies, st))) return rc;
  launch_kinetic(n, vel, type, c->dp, energies + REAXFF_NTERMS, st);
  // with skin lists, positions stay continuous between rebuilds (wrapped
  // into the box only when the lists are built again)
  const bool keep = c->skin > 0.0;
  for (int s = 1; s <= nsteps; ++s) {
    launch_kick(n, vel, forces, type, c->dp, 0.5 * dt, st);
    launch_drift(n, pos, vel, dt, c->grid, !keep, st);
    if ((rc = refresh_lists(c, n, pos, pos, type, box, nullptr, st))) return rc;
    if ((rc = reaxff_compute_forces(c, n, pos, type, q, box, forces, energies + s * row, st)))
      return rc;
    launch_kick(n, vel, forces, type, c->dp, 0.5 * dt, st);
    launch_kinetic(n, vel, type, c->dp, energies + s * row + REAXFF_NTERMS, st);
  }
  HIPCHK(c, hipGetLastError());
  return REAXFF_OK;
}

int reaxff_list_sizes(const reaxff_ctx* c, int64_t sizes[3]) {
  if (!c || !sizes) return REAXFF_ERR_ARG;
  if (!c->built) return REAXFF_ERR_STATE;
  sizes[0] = c->L.nfar;
  sizes[1] = c->L.nbond;
  sizes[2] = c->L.nhb;
  return REAXFF_OK;
}

int reaxff_export_lists(reaxff_ctx* c, int32_t* far, int32_t* bonds, int32_t* hb) {
  if (!c) return REAXFF_ERR_ARG;
  if (!c->built) return fail(c, REAXFF_ERR_STATE, "lists not built");
  HIPCHK(c, hipSetDevice(c->device));
  int32_t *df = nullptr, *db = nullptr, *dh = nullptr;
  if (far && c->L.nfar) HIPCHK(c, hipMalloc(&df, sizeof(int32_t) * 2 * c->L.nfar));
  if (bonds && c->L.nbond) HIPCHK(c, hipMalloc(&db, sizeof(int32_t) * 2 * c->L.nbond));
  if (hb && c->L.nhb) HIPCHK(c, hipMalloc(&dh, sizeof(int32_t) * 2 * c->L.nhb));
  if (launch_export(c->grid, c->L, df, db, dh, c->sc, 0)) return fail(c, REAXFF_ERR_HIP, "export failed");
  HIPCHK(c, hipDeviceSynchronize());
  if (df) HIPCHK(c, hipMemcpy(far, df, sizeof(int32_t) * 2 * c->L.nfar, hipMemcpyDeviceToHost));
  if (db) HIPCHK(c, hipMemcpy(bonds, db, sizeof(int32_t) * 2 * c->L.nbond, hipMemcpyDeviceToHost));
  if (dh) HIPCHK(c, hipMemcpy(hb, dh, sizeof(int32_t) * 2 * c->L.nhb, hipMemcpyDeviceToHost));
  if (df) (void)hipFree(df);
  if (db) (void)hipFree(db);
  if (dh) (void)hipFree(dh);
  return REAXFF_OK;
}

int reaxff_set_overlap(reaxff_ctx* c, int32_t enable) {
  if (!c) return REAXFF_ERR_ARG;
  c->overlap = enable != 0;
  return REAXFF_OK;
}

int reaxff_set_nb_run(reaxff_ctx* c, int32_t run_max) {
  if (!c) return REAXFF_ERR_ARG;
  if (run_max < 1 || run_max > 16) return fail(c, REAXFF_ERR_ARG, "reaxff_set_nb_run: run_max must lie in 1..16");
  c->nb_run_max = run_max;
  return REAXFF_OK;
}

int reaxff_set_skin(reaxff_ctx* c, double skin, int32_t every) {
  if (!c) return REAXFF_ERR_ARG;
  if (!(skin >= 0.0 && skin <= c->cut.r_nonb) || every < 1)
    return fail(c, REAXFF_ERR_ARG, "reaxff_set_skin: skin must lie in [0, r_nonb] and every >= 1");
  HIPCHK(c, hipSetDevice(c->device));
  c->skin = skin;
  c->every = every;
  c->built = false;
  c->forces_done = false;
  c->L.far_w = 0;   // widths re-estimated for the new cutoffs
  c->L.hb_w = 0;
  c->L.ha_w = 0;
  if (skin > 0.0) {
    DevParams d = c->hd;
    const double rl = c->cut.r_nonb + skin, rh = c->cut.r_hb + skin;
    d.rn2 = rl * rl;
    d.rh2 = rh * rh;
    d.r_bond = c->cut.r_bond + skin;
    for (int t = 0; t < NT * NT; ++t) {
      const double r = std::sqrt(c->hd.pair[t].reach2) + skin;
      d.pair[t].reach2 = r * r;
    }
    if (!c->dp_list) HIPCHK(c, hipMalloc(&c->dp_list, sizeof(DevParams)));
    HIPCHK(c, hipMemcpy(c->dp_list, &d, sizeof(DevParams), hipMemcpyHostToDevice));
  }
  return REAXFF_OK;
}

int reaxff_refresh_lists(reaxff_ctx* c, int64_t n, const double* pos, const int32_t* type, const double* box,
                         int32_t* rebuilt, hipStream_t st) {
  if (!c) return REAXFF_ERR_ARG;
  if (n < 0 || (n > 0 && (!pos || !type))) return fail(c, REAXFF_ERR_ARG, "bad n or null pointer");
  return refresh_lists(c, n, pos, nullptr, type, box, rebuilt, st);
}

int reaxff_list_stats(const reaxff_ctx* c, int64_t stats[2]) {
  if (!c || !stats) return REAXFF_ERR_ARG;
  stats[0] = c->nrebuild;
  stats[1] = c->nrefresh;
  return REAXFF_OK;
}

int reaxff_profile(reaxff_ctx* c, int32_t enable) {
  if (!c) return REAXFF_ERR_ARG;
  c->prof.reset();
  c->prof.on = enable != 0;
  return REAXFF_OK;
}

int reaxff_profile_read(reaxff_ctx* c, int32_t max, double* ms, int64_t* launches,
                        const char** names) {
  if (!c) return REAXFF_ERR_ARG;
  c->prof.collect();
  const int k = std::min<int>(max, KID_COUNT);
  for (int i = 0; i < k; ++i) {
    if (ms) ms[i] = c->prof.ms[i];
    if (launches) launches[i] = c->prof.calls[i];
    if (names) names[i] = kKernelNames[i];
  }
  return k;
}

int reaxff_interaction_counts(reaxff_ctx* c, int64_t counts[5]) {
  if (!c || !counts) return REAXFF_ERR_ARG;
  HIPCHK(c, hipSetDevice(c->device));
  unsigned long long h[4] = {0, 0, 0, 0};
  HIPCHK(c, hipDeviceSynchronize());
  HIPCHK(c, hipMemcpy(h, c->W.counters, sizeof(h), hipMemcpyDeviceToHost));
  counts[0] = (int64_t)h[0];
  counts[1] = (int64_t)h[1];
  counts[2] = (int64_t)h[2];
  counts[3] = c->L.nfar;
  counts[4] = c->L.nbond / 2;
  return REAXFF_OK;
}

}  // extern "C"
