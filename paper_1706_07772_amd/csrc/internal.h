// Host-side internals shared by the library's translation units.
#pragma once

#include <map>
#include <string>
#include <vector>

#include "reaxff_dev.h"

namespace rx {

// kernels timed by the optional event profiler (reaxff_profile)
enum KernelId {
  KID_BBOX, KID_CELL_HIST, KID_CELL_SCATTER, KID_CELL_SORT, KID_GATHER, KID_LIST_SWEEP, KID_BOND_MERGE, KID_SCAN,
  KID_BONDTEST, KID_COMPACT, KID_MIRROR, KID_ZERO, KID_GATHER_Q, KID_BO_PRIME, KID_DELTA_PRIME, KID_BO_CORR,
  KID_ATOM_STATE, KID_ATOM_ENERGY, KID_TASKS, KID_ANGLES, KID_TORSIONS, KID_HBONDS, KID_HB_ACC, KID_NONBONDED,
  KID_BACK_S, KID_BACK_CORR, KID_BACK_DP, KID_FORCES, KID_BATCH, KID_NB_REDUCE, KID_NB_ENERGY, KID_ENERGY_FOLD,
  KID_QEQ_ROWS, KID_QEQ_SPMV, KID_QEQ_VEC, KID_SUR_DESC, KID_SUR_NET, KID_SUR_PAIRW, KID_SUR_GATHER,
  KID_SUR_MIRROR, KID_QEQ_HALF, KID_QEQ_HREDUCE, KID_COUNT
};
extern const char* const kKernelNames[KID_COUNT];

// pairs of HIP events recorded around kernel launches on the launch stream
struct Prof {
  bool on = false;
  struct Pending { int id; hipEvent_t a, b; };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  double ms[KID_COUNT] = {};
  int64_t calls[KID_COUNT] = {};
  hipEvent_t get() {
    if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
    hipEvent_t e;
    (void)hipEventCreate(&e);
    return e;
  }
  void begin(int id, hipStream_t st) {
    if (!on) return;
    Pending p{id, get(), get()};
    (void)hipEventRecord(p.a, st);
    pending.push_back(p);
  }
  void end(hipStream_t st) {
    if (!on || pending.empty()) return;
    (void)hipEventRecord(pending.back().b, st);
  }
  void collect() {
    for (auto& p : pending) {
      (void)hipEventSynchronize(p.b);
      float t = 0.f;
      (void)hipEventElapsedTime(&t, p.a, p.b);
      ms[p.id] += t;
      calls[p.id] += 1;
      pool.push_back(p.a);
      pool.push_back(p.b);
    }
    pending.clear();
  }
  void reset() {
    collect();
    for (int k = 0; k < KID_COUNT; ++k) { ms[k] = 0; calls[k] = 0; }
  }
  ~Prof() {
    for (auto& p : pending) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

// scratch owned by the context (device pointers)
struct Scratch {
  int32_t* cid = nullptr;         // [n] cell of each caller-order atom
  int32_t* cell_s = nullptr;      // [n] cell of each sorted atom
  int32_t* cell_count = nullptr;  // [ncell + 1]
  int32_t* cell_cursor = nullptr; // [ncell + 1]
  int32_t* flag = nullptr;        // error flags written by kernels
  int32_t* cnt_bond = nullptr;    // [n + 1]
  int32_t* cnt_cand = nullptr;    // [n] bond candidates
  int32_t* cnt_lo = nullptr;      // [n] bonds written by partners (each-pair-once sweep)
  bool half = false;              // the last sweep took each pair once
  // fixed-width rows (one per atom) staging the sweep's bond candidates and bonds
  int32_t* cand_j = nullptr;      // width cand_w
  int32_t* bond_t = nullptr;      // width bond_w
  int32_t cand_w = 0, bond_w = 0;
  int64_t cap_cand = 0, cap_bondt = 0;
  int32_t* need = nullptr;        // device [4]: largest counts seen (far, cand, bond, hb)
  double* part = nullptr;         // bbox partials
  int64_t* totals = nullptr;      // device [8]
  // device [ESLOT][8] partial totals and [ESLOT] partial need[5] maxima of
  // the sweep and bond test (workgroup mod ESLOT), folded into totals, need
  int64_t* tslot = nullptr;
  int32_t* nslot = nullptr;
  int64_t* totals_host = nullptr; // pinned host [8]
  // scan temporaries
  int64_t* scan_tmp = nullptr;
  int64_t scan_cap = 0;
};

// charge-equilibration state (device pointers): the rows of H, the CG
// vectors of the two systems as (s, t) pairs in sorted order, per-iteration
// partial-sum sets, and a ring of the last four solutions in caller order
struct Qeq {
  int32_t* hj = nullptr;     // [n][w] sorted neighbour index
  double* hv = nullptr;      // [n][w] H_ij
  int32_t* hcnt = nullptr;   // [n] row lengths
  int32_t w = 0;
  int64_t cap_rows = 0, cap_rowsv = 0, cap_cnt = 0;
  double2 *x = nullptr, *r = nullptr, *p = nullptr, *ap = nullptr;
  int64_t cap_n = 0, cap_vec = 0;
  double* red = nullptr;     // [maxit + 2][ESLOT][8]
  int64_t cap_red = 0;
  double* red_host = nullptr;  // pinned [ESLOT][8]
  int32_t* need = nullptr;   // device: longest row beyond w
  double2* hist[4] = {nullptr, nullptr, nullptr, nullptr};
  int head = 0, nhist = 0;
  int64_t hist_n = -1;
  double* part = nullptr;    // matrix-free product: per-run partial arrays [nrun][NB_HALF_CAP][2]
  int32_t* tab = nullptr;    // and per-run chunk offsets [nrun][NB_QMAX]
  int64_t cap_part = 0, cap_tab = 0;
  int32_t mode = 0;          // REAXFF_QEQ_AUTO or REAXFF_QEQ_STORED
};

// species-analysis work arrays (device): union-find parents over caller
// indices, root flags and ranks, per-molecule element counts, sort buffers
struct Species {
  int32_t *parent = nullptr, *flag = nullptr, *rank = nullptr, *counts = nullptr;
  int32_t *order = nullptr, *order2 = nullptr, *sid = nullptr;
  uint32_t *key = nullptr, *key2 = nullptr;
  void* tmp = nullptr;
  size_t tmp_bytes = 0;
  int64_t cap = 0;
};

// work arrays of reaxff_forces_masked (device): cell of each atom, cell marks
// (two, for the dilation passes), selection flags and their prefix sums, the
// gathered subsystem and its forces and energies
struct Masked {
  int32_t *cid = nullptr, *sel = nullptr, *idx = nullptr, *stype = nullptr, *flag = nullptr;
  uint8_t *mark = nullptr, *mark2 = nullptr;
  double *spos = nullptr, *sq = nullptr, *sforce = nullptr, *senergy = nullptr, *part = nullptr;
  int64_t cap_cid = 0, cap_sel = 0, cap_idx = 0, cap_stype = 0, cap_flag = 0, cap_mark = 0, cap_mark2 = 0;
  int64_t cap_spos = 0, cap_sq = 0, cap_sforce = 0, cap_part = 0;
};

// exclusive prefix sums; out[n-1] holds the total when in[n-1] == 0
int scan_i32(const int32_t* in, int32_t* out, int64_t n, Scratch& sc, hipStream_t st);
int scan_i32_to_i64(const int32_t* in, int64_t* out, int64_t n, Scratch& sc, hipStream_t st);

int launch_bbox(const double* pos, const int32_t* type, int64_t n, double* part, int nparts,
                int32_t* flag, Prof& pf, hipStream_t st);
int launch_cell_sort(const double* pos, const int32_t* type, int64_t n, const Grid& g, int ncell,
                     Scratch& sc, Lists& L, Prof& pf, hipStream_t st);
int launch_sweep(const DevParams* P, const Grid& g, int64_t n, int ncell, double rb2, bool half, Scratch& sc,
                 Lists& L, Prof& pf, hipStream_t st);
int launch_bondtest(const DevParams* P, const Grid& g, int64_t n, double rb2, Scratch& sc, Lists& L, Prof& pf,
                    hipStream_t st);
int launch_refresh_gather(const double* pos, int64_t n, const double4* xref, Lists& L, unsigned long long* dmax,
                          Prof& pf, hipStream_t st);
int launch_compact(int64_t n, Scratch& sc, Lists& L, Prof& pf, hipStream_t st);
int launch_export(const Grid& g, const Lists& L, int32_t* far, int32_t* bonds, int32_t* hb, Scratch& sc,
                  hipStream_t st);

int launch_forces(const DevParams* P, const Grid& g, const Lists& L, Work& W, const double* q,
                  hipStream_t side, hipEvent_t ev_fork, hipEvent_t ev_join,
                  double* forces, double* energies, Scratch& sc, Prof& pf, hipStream_t st);
int launch_kick(int64_t n, double* vel, const double* forces, const int32_t* type,
                const DevParams* P, double half_dt, hipStream_t st);
int launch_drift(int64_t n, double* pos, const double* vel, double dt, const Grid& g, bool wrap, hipStream_t st);
int launch_wrap(int64_t n, double* pos, const Grid& g, hipStream_t st);
int launch_kinetic(int64_t n, const double* vel, const int32_t* type, const DevParams* P,
                   double* out, hipStream_t st);

// address of the fixed scratch array of reaxff_compute_forces_batched on a
// device (which must be current), looked up once per device; a HIP error code
int batched_scratch_init(int device);

}  // namespace rx

// the library context (opaque to callers)
struct reaxff_ctx {
  int device = 0;
  reaxff_params hp;
  reaxff_cutoffs cut;
  rx::DevParams* dp = nullptr;    // device copy
  rx::DevParams hd;               // host copy
  rx::Grid grid{};
  rx::Lists L{};
  rx::Work W{};
  rx::Scratch sc{};
  rx::Prof prof;
  rx::Qeq qeq;
  rx::Species species;
  rx::Masked masked;
  // the nonbonded term runs on a stream of its own, concurrent with the
  // bonded terms, between a fork and a join event on the caller's stream
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  bool overlap = true;
  int nb_run_max = 8;       // longest run of cells of the half nonbonded evaluation
  bool upper_off = false;   // a build found the half evaluation impossible: full far rows from then on
  // Verlet-skin lists: far, H and bond-candidate lists built with the cutoffs
  // plus `skin` and kept while no atom has moved more than skin / 2 since the
  // build, for at most `every` refreshes; dp_list holds the enlarged cutoffs
  double skin = 0.0;
  int32_t every = 1;
  int32_t since = 0;
  rx::DevParams* dp_list = nullptr;
  double4* xref = nullptr;          // sorted positions at the last build
  int64_t cap_xref = 0;
  unsigned long long* dmax = nullptr;
  int64_t nrebuild = 0, nrefresh = 0;
  bool built = false;
  bool forces_done = false;  // bond orders of the current lists are computed
  double box[3] = {0, 0, 0};
  bool periodic = false;
  int64_t cap_n = 0, cap_cell = 0, cap_far = 0, cap_bond = 0, cap_hb = 0, cap_ha = 0, cap_part = 0;
  // list storage the context owns; the lists (L) point here, or into the
  // caller's buffers after reaxff_build_lists_into (ext_on)
  int32_t *own_far = nullptr, *own_hb = nullptr, *own_bj = nullptr, *own_mir = nullptr;
  int64_t cap_own_bj = 0;
  bool ext_on = false;
  std::string err;
  // autotuned batch configurations, keyed by a signature of the cluster sizes
  std::map<uint64_t, reaxff_batch_config> tuned;
};
