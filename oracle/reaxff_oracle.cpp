// CPU oracle for one ReaxFF force evaluation -- TEST INFRASTRUCTURE ONLY.
//
// Plain, slow, single-threaded FP64.  Only tests, the build check and the
// CPU-baseline leg of the benchmark may call it; the GPU library never does.
//
// What it computes: the ReaxFF potential energy E(x; q, params) of the model
// the paper works with (Section 2.1: bond orders, bond, lone pair, over- and
// under-coordination, valence angle, torsion, hydrogen bond, van der Waals and
// Coulomb, summed per term; forces per atom), for given charges, and the force
// F = -dE/dx.  The paper prints no formula; the functional forms follow the
// ReaxFF papers it cites for the model ([6,7] and [11,12]), with each point
// they leave open fixed by a stated reading.  The lists are the ones the paper
// describes in Section 3.3: a half far-neighbour list, a full bond list with
// both directions, and a hydrogen-bond list per H atom.
//
// Structure:
//   * lists: brute force O(N^2) over all pairs, or a cell list producing the
//     identical sets from the identical pair predicate;
//   * energy<T>(): the energy written once, as a template over the scalar;
//     T = double (energies), T = ad::Var (reverse-mode differentiation, which
//     gives F = -grad E mechanically), T = std::complex<double> (complex-step
//     derivatives, used to check the differentiation);
//   * a velocity-Verlet NVE driver.
//
// Build: g++ -O2 -fno-fast-math -ffp-contract=off (oracle/build.py).

#include "oracle_api.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

namespace oracle {

// ---------------------------------------------------------------------------
// parameter layout (name-major blocks; orders mirrored by oracle/__init__.py)
// ---------------------------------------------------------------------------
enum General {
  p_boc1, p_boc2, p_coa2, p_coa3, p_coa4, p_ovun3, p_ovun4, p_ovun6, p_ovun7,
  p_ovun8, p_val6, p_val8, p_val9, p_val10, p_pen2, p_pen3, p_pen4, p_tor2,
  p_tor3, p_tor4, p_cot2, p_vdW1, p_lp1, NG
};
enum Atom { a_val, a_val_e, a_val_boc, a_val_ang, a_mass, a_p_hbond, a_p_lp2,
            a_p_ovun2, a_p_ovun5, a_p_val3, a_p_val5, NA };
enum Pair { r_s, r_p, r_pp, D_s, D_p, D_pp, p_be1, p_be2, p_bo1, p_bo2, p_bo3,
            p_bo4, p_bo5, p_bo6, p_ovun1, p_boc3, p_boc4, p_boc5, D_vdw, r_vdw,
            alpha, gamma_w, gamma_c, r_core, e_core, a_core, NP };
enum Angle { theta00, p_val1, p_val2, p_val4, p_val7, p_pen1, p_coa1, NANG };
enum Tors { V1, V2, V3, p_tor1, p_cot1, NT };
enum HBond { r0hb, p_hb1, p_hb2, p_hb3, NH };

enum Term { E_BOND, E_LP, E_OVER, E_UNDER, E_VAL, E_PEN, E_COA, E_TOR, E_CONJ,
            E_HB, E_VDW, E_COUL, NTERMS };
static_assert(NTERMS == ORACLE_NTERMS, "term count");

constexpr double C_ELE = 332.06371;        // kcal A / (mol e^2)
constexpr double ACC_CONV = 4.184e-4;      // (kcal/mol/A)/(g/mol) -> A/fs^2
constexpr double PI = 3.14159265358979323846;

struct Params {
  double g[NG];
  double a[NA][4];
  double p[NP][4][4];
  double ang[NANG][4][4][4];
  double tor[NT][4][4][4][4];
  double hb[NH][4][4][4];
};

struct Cutoffs { double r_nonb, r_bond, r_hb, bo_cut, thb_cut, thb_cutsq, hb_bo_cut; };

static thread_local std::string g_err;

// ---------------------------------------------------------------------------
// reverse-mode differentiation: a tape of nodes with up to two parents
// ---------------------------------------------------------------------------
namespace ad {
struct Node { int32_t a, b; double da, db; };
struct Tape {
  std::vector<Node> nodes;
  std::vector<double> adj;
  int32_t push(int32_t a, double da, int32_t b, double db) {
    nodes.push_back(Node{a, b, da, db});
    adj.push_back(0.0);
    return (int32_t)nodes.size() - 1;
  }
  // propagate adjoints of nodes [mark, size) to their parents, then drop them
  void sweep_to(size_t mark) {
    for (size_t k = nodes.size(); k-- > mark;) {
      const double w = adj[k];
      if (w == 0.0) continue;
      const Node& nd = nodes[k];
      if (nd.a >= 0) adj[nd.a] += w * nd.da;
      if (nd.b >= 0) adj[nd.b] += w * nd.db;
    }
    nodes.resize(mark);
    adj.resize(mark);
  }
};
static thread_local Tape* tape = nullptr;

struct Var {
  double v;
  int32_t id;
  Var() : v(0.0), id(-1) {}
  Var(double x) : v(x), id(-1) {}  // constants carry no node
  Var(double x, int32_t i) : v(x), id(i) {}
};
inline Var leaf(double v) { return Var(v, tape->push(-1, 0.0, -1, 0.0)); }
inline Var un(double v, const Var& x, double dx) {
  if (x.id < 0) return Var(v);
  return Var(v, tape->push(x.id, dx, -1, 0.0));
}
inline Var bin(double v, const Var& x, double dx, const Var& y, double dy) {
  if (x.id < 0 && y.id < 0) return Var(v);
  if (x.id < 0) return Var(v, tape->push(y.id, dy, -1, 0.0));
  if (y.id < 0) return Var(v, tape->push(x.id, dx, -1, 0.0));
  return Var(v, tape->push(x.id, dx, y.id, dy));
}
inline Var operator+(const Var& x, const Var& y) { return bin(x.v + y.v, x, 1.0, y, 1.0); }
inline Var operator-(const Var& x, const Var& y) { return bin(x.v - y.v, x, 1.0, y, -1.0); }
inline Var operator*(const Var& x, const Var& y) { return bin(x.v * y.v, x, y.v, y, x.v); }
inline Var operator/(const Var& x, const Var& y) {
  const double v = x.v / y.v;
  return bin(v, x, 1.0 / y.v, y, -v / y.v);
}
inline Var operator-(const Var& x) { return un(-x.v, x, -1.0); }
inline Var& operator+=(Var& x, const Var& y) { x = x + y; return x; }
inline Var& operator-=(Var& x, const Var& y) { x = x - y; return x; }
inline Var& operator*=(Var& x, const Var& y) { x = x * y; return x; }
inline Var exp(const Var& x) { const double v = std::exp(x.v); return un(v, x, v); }
inline Var log(const Var& x) { return un(std::log(x.v), x, 1.0 / x.v); }
inline Var sqrt(const Var& x) { const double v = std::sqrt(x.v); return un(v, x, 0.5 / v); }
inline Var pow(const Var& x, double p) {
  return un(std::pow(x.v, p), x, p * std::pow(x.v, p - 1.0));
}
inline Var atan(const Var& x) { return un(std::atan(x.v), x, 1.0 / (1.0 + x.v * x.v)); }
}  // namespace ad

using ad::Var;
using cplx = std::complex<double>;

inline double re(double x) { return x; }
inline double re(const Var& x) { return x.v; }
inline double re(const cplx& x) { return x.real(); }

// ---------------------------------------------------------------------------
// system, geometry and lists
// ---------------------------------------------------------------------------
struct Sys {
  int n = 0;
  std::vector<double> x;       // positions [n][3]
  std::vector<int> type;
  std::vector<double> q;
  bool periodic = false;
  double L[3] = {0, 0, 0}, invL[3] = {0, 0, 0};
  Params P;
  Cutoffs c;
  bool brute = false;
  // lists (atom indices as given)
  std::vector<std::pair<int, int>> far;            // unordered, i < j
  std::vector<std::vector<int>> hbl;               // acceptors of each H atom, ascending
  std::vector<int> bi, bj;                         // undirected bonds, bi < bj
  std::vector<std::vector<std::pair<int, int>>> adj;  // (neighbour, bond id), ascending
};

// displacement x_j - x_i, minimum image: d -= L * rint(d * (1/L)) per axis
template <class T>
inline void dvec(const Sys& s, const T* x, int i, int j, T d[3]) {
  for (int k = 0; k < 3; ++k) {
    T dk = x[3 * j + k] - x[3 * i + k];
    if (s.periodic) {
      const double shift = s.L[k] * std::rint(re(dk) * s.invL[k]);
      dk = dk - shift;
    }
    d[k] = dk;
  }
}

// squared distance used for every list decision: fma(dz,dz, fma(dy,dy, dx*dx))
inline double r2_list(const double d[3]) {
  return std::fma(d[2], d[2], std::fma(d[1], d[1], d[0] * d[0]));
}

// uncorrected bond-order components of a pair at distance r (sigma scaled by
// 1 + bo_cut; a component is absent when its mixed radius is not positive)
template <class T>
inline void bo_prime(const Params& P, const Cutoffs& c, int ti, int tj, const T& r,
                     T& s, T& p, T& pp) {
  using std::exp; using std::pow;
  const double rs = P.p[r_s][ti][tj], rp = P.p[r_p][ti][tj], rpp = P.p[r_pp][ti][tj];
  s = rs > 0.0 ? (1.0 + c.bo_cut) * exp(P.p[p_bo1][ti][tj] * pow(r / rs, P.p[p_bo2][ti][tj])) : T(0.0);
  p = rp > 0.0 ? exp(P.p[p_bo3][ti][tj] * pow(r / rp, P.p[p_bo4][ti][tj])) : T(0.0);
  pp = rpp > 0.0 ? exp(P.p[p_bo5][ti][tj] * pow(r / rpp, P.p[p_bo6][ti][tj])) : T(0.0);
}

inline double bo_raw_at(const Sys& s, int i, int j) {
  double d[3];
  dvec(s, s.x.data(), i, j, d);
  const double r = std::sqrt(r2_list(d));
  double a, b, e;
  bo_prime<double>(s.P, s.c, s.type[i], s.type[j], r, a, b, e);
  return a + b + e;
}

// classify one unordered pair i<j into the three lists
static void visit_pair(Sys& s, int i, int j, std::vector<std::vector<int>>& bnd) {
  double d[3];
  dvec(s, s.x.data(), i, j, d);
  const double r2 = r2_list(d);
  const double rn2 = s.c.r_nonb * s.c.r_nonb, rb2 = s.c.r_bond * s.c.r_bond,
               rh2 = s.c.r_hb * s.c.r_hb;
  if (r2 <= rn2) s.far.emplace_back(i, j);
  if (r2 <= rb2) {
    const double r = std::sqrt(r2);
    double a, b, e;
    bo_prime<double>(s.P, s.c, s.type[i], s.type[j], r, a, b, e);
    if (a + b + e >= s.c.bo_cut) {
      bnd[i].push_back(j);
      bnd[j].push_back(i);
    }
  }
  if (r2 <= rh2) {
    const int ti = s.type[i], tj = s.type[j];
    if (s.P.a[a_p_hbond][ti] == 1.0 && s.P.a[a_p_hbond][tj] == 2.0) s.hbl[i].push_back(j);
    if (s.P.a[a_p_hbond][tj] == 1.0 && s.P.a[a_p_hbond][ti] == 2.0) s.hbl[j].push_back(i);
  }
}

static void build_lists(Sys& s) {
  const int n = s.n;
  s.far.clear();
  s.hbl.assign(n, {});
  std::vector<std::vector<int>> bnd(n);
  if (s.brute) {
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) visit_pair(s, i, j, bnd);
  } else {
    // cells at least r_nonb wide; the candidate set is every atom of the
    // distinct neighbouring cells, the decision is the same predicate
    double lo[3], ext[3];
    for (int k = 0; k < 3; ++k) {
      if (s.periodic) {
        lo[k] = 0.0;
        ext[k] = s.L[k];
      } else {
        double mn = 1e300, mx = -1e300;
        for (int i = 0; i < n; ++i) {
          mn = std::min(mn, s.x[3 * i + k]);
          mx = std::max(mx, s.x[3 * i + k]);
        }
        lo[k] = mn;
        ext[k] = std::max(mx - mn, 1e-9);
      }
    }
    int nc[3];
    double w[3];
    for (int k = 0; k < 3; ++k) {
      nc[k] = std::max(1, (int)std::floor(ext[k] / s.c.r_nonb));
      w[k] = ext[k] / nc[k];
    }
    auto cell_of = [&](int i, int k) {
      double v = s.x[3 * i + k] - lo[k];
      if (s.periodic) v -= s.L[k] * std::floor(v * s.invL[k]);
      int ci = (int)std::floor(v / w[k]);
      return std::min(std::max(ci, 0), nc[k] - 1);
    };
    const int ncell = nc[0] * nc[1] * nc[2];
    std::vector<std::vector<int>> cells(ncell);
    std::vector<int> cid(n);
    for (int i = 0; i < n; ++i) {
      const int c0 = cell_of(i, 0), c1 = cell_of(i, 1), c2 = cell_of(i, 2);
      cid[i] = (c0 * nc[1] + c1) * nc[2] + c2;
      cells[cid[i]].push_back(i);
    }
    for (int i = 0; i < n; ++i) {
      const int c0 = cid[i] / (nc[1] * nc[2]), c1 = (cid[i] / nc[2]) % nc[1], c2 = cid[i] % nc[2];
      std::vector<int> ncells;
      for (int d0 = -1; d0 <= 1; ++d0)
        for (int d1 = -1; d1 <= 1; ++d1)
          for (int d2 = -1; d2 <= 1; ++d2) {
            int e[3] = {c0 + d0, c1 + d1, c2 + d2};
            bool ok = true;
            for (int k = 0; k < 3; ++k) {
              if (s.periodic) e[k] = ((e[k] % nc[k]) + nc[k]) % nc[k];
              else if (e[k] < 0 || e[k] >= nc[k]) ok = false;
            }
            if (ok) ncells.push_back((e[0] * nc[1] + e[1]) * nc[2] + e[2]);
          }
      std::sort(ncells.begin(), ncells.end());
      ncells.erase(std::unique(ncells.begin(), ncells.end()), ncells.end());
      for (int cc : ncells)
        for (int j : cells[cc])
          if (j > i) visit_pair(s, i, j, bnd);
    }
  }
  std::sort(s.far.begin(), s.far.end());
  for (auto& v : s.hbl) std::sort(v.begin(), v.end());
  s.bi.clear();
  s.bj.clear();
  s.adj.assign(n, {});
  for (int i = 0; i < n; ++i) std::sort(bnd[i].begin(), bnd[i].end());
  for (int i = 0; i < n; ++i)
    for (int j : bnd[i])
      if (j > i) {
        const int b = (int)s.bi.size();
        s.bi.push_back(i);
        s.bj.push_back(j);
        s.adj[i].emplace_back(j, b);
        s.adj[j].emplace_back(i, b);
      }
  for (auto& v : s.adj) std::sort(v.begin(), v.end());
}

// ---------------------------------------------------------------------------
// energy sinks
// ---------------------------------------------------------------------------
struct Neumaier {
  double s = 0.0, c = 0.0;
  void add(double v) {
    const double t = s + v;
    if (std::fabs(s) >= std::fabs(v)) c += (s - t) + v;
    else c += (v - t) + s;
    s = t;
  }
  double value() const { return s + c; }
};

struct DoubleSink {
  Neumaier E[NTERMS];
  Neumaier A[NTERMS];   // sum of |interaction energy|: the conditioning of each term
  size_t begin() { return 0; }
  void add(int t, double e) { E[t].add(e); A[t].add(std::fabs(e)); }
  void end(size_t) {}
};

struct ComplexSink {
  cplx E[NTERMS];
  size_t begin() { return 0; }
  void add(int t, const cplx& e) { E[t] += e; }
  void end(size_t) {}
};

// each interaction is differentiated on its own: its nodes are swept back to
// the interaction's first node, which deposits adjoints on the shared
// intermediates (bond orders, atom sums, positions), and are then discarded
struct AdSink {
  Neumaier E[NTERMS];
  std::vector<int32_t> pending;
  size_t begin() { return ad::tape->nodes.size(); }
  void add(int t, const Var& e) {
    E[t].add(e.v);
    if (e.id >= 0) pending.push_back(e.id);
  }
  void end(size_t mark) {
    for (int32_t id : pending) ad::tape->adj[id] += 1.0;
    pending.clear();
    ad::tape->sweep_to(mark);
  }
};

// ---------------------------------------------------------------------------
// the energy, written once
// ---------------------------------------------------------------------------
template <class T>
inline T sq(const T& v) { return v * v; }

template <class T>
inline T dot3(const T a[3], const T b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// The angle in [0, pi] between two vectors a, b from y = |a x b| and x = a . b:
// twice the angle whose tangent is y / (|a||b| + x), or its supplement when
// x < 0, so that neither a straight nor a folded angle loses digits (the
// arccosine of the cosine does, and so does its derivative).
template <class T>
inline T angle_of(const T& y, const T& x) {
  using std::atan; using std::sqrt;
  const T r = sqrt(x * x + y * y);
  if (re(x) >= 0.0) return 2.0 * atan(y / (r + x));
  return PI - 2.0 * atan(y / (r - x));
}

template <class T>
inline void cross3(const T a[3], const T b[3], T out[3]) {
  out[0] = a[1] * b[2] - a[2] * b[1];
  out[1] = a[2] * b[0] - a[0] * b[2];
  out[2] = a[0] * b[1] - a[1] * b[0];
}

template <class T>
struct BondStage {
  // per undirected bond
  std::vector<T> BOs, BOpi, BOpi2, BOt;     // uncorrected (after the threshold shift)
  std::vector<T> BO, BOp, BOpp, BOsig;      // corrected
  // per atom
  std::vector<T> Dp, Dboc, S, Delta, Dang, nlp, vlpex, Dlp, SBO, SBO2;
};

template <class T>
void bond_stage(const Sys& s, const T* x, BondStage<T>& B) {
  using std::exp; using std::log; using std::pow; using std::sqrt;
  const Params& P = s.P;
  const Cutoffs& c = s.c;
  const int n = s.n, nb = (int)s.bi.size();
  B.BOs.resize(nb); B.BOpi.resize(nb); B.BOpi2.resize(nb); B.BOt.resize(nb);
  B.BO.resize(nb); B.BOp.resize(nb); B.BOpp.resize(nb); B.BOsig.resize(nb);
  // (1) uncorrected bond orders
  for (int b = 0; b < nb; ++b) {
    const int i = s.bi[b], j = s.bj[b];
    T d[3];
    dvec(s, x, i, j, d);
    const T r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    T sg, pi, pp;
    bo_prime<T>(P, c, s.type[i], s.type[j], r, sg, pi, pp);
    const T raw = sg + pi + pp;
    B.BOs[b] = sg - c.bo_cut;
    B.BOpi[b] = pi;
    B.BOpi2[b] = pp;
    B.BOt[b] = raw - c.bo_cut;
  }
  // Delta'_i = sum_j BO'_ij - Val_i ; Delta'boc_i = sum_j BO'_ij - Val_boc_i
  B.Dp.resize(n); B.Dboc.resize(n);
  for (int i = 0; i < n; ++i) {
    T sum = T(0.0);
    for (auto& nb_ : s.adj[i]) sum = sum + B.BOt[nb_.second];
    B.Dp[i] = sum - P.a[a_val][s.type[i]];
    B.Dboc[i] = sum - P.a[a_val_boc][s.type[i]];
  }
  // (2) corrected bond orders
  const double pb1 = P.g[p_boc1], pb2 = P.g[p_boc2];
  for (int b = 0; b < nb; ++b) {
    const int i = s.bi[b], j = s.bj[b];
    const int ti = s.type[i], tj = s.type[j];
    const double vi = P.a[a_val][ti], vj = P.a[a_val][tj];
    const T f2 = exp(-pb1 * B.Dp[i]) + exp(-pb1 * B.Dp[j]);
    const T f3 = -(1.0 / pb2) * log(0.5 * (exp(-pb2 * B.Dp[i]) + exp(-pb2 * B.Dp[j])));
    const T f1 = 0.5 * ((vi + f2) / (vi + f2 + f3) + (vj + f2) / (vj + f2 + f3));
    const double b3 = P.p[p_boc3][ti][tj], b4 = P.p[p_boc4][ti][tj], b5 = P.p[p_boc5][ti][tj];
    const T bo2 = B.BOt[b] * B.BOt[b];
    const T f4 = 1.0 / (1.0 + exp(-b3 * (b4 * bo2 - B.Dboc[i]) + b5));
    const T f5 = 1.0 / (1.0 + exp(-b3 * (b4 * bo2 - B.Dboc[j]) + b5));
    B.BO[b] = B.BOt[b] * f1 * f4 * f5;
    B.BOp[b] = B.BOpi[b] * f1 * f1 * f4 * f5;
    B.BOpp[b] = B.BOpi2[b] * f1 * f1 * f4 * f5;
    B.BOsig[b] = B.BO[b] - B.BOp[b] - B.BOpp[b];
  }
  // (3) atom quantities
  B.S.resize(n); B.Delta.resize(n); B.Dang.resize(n); B.nlp.resize(n);
  B.vlpex.resize(n); B.Dlp.resize(n); B.SBO.resize(n); B.SBO2.resize(n);
  const double plp1 = P.g[p_lp1], pv8 = P.g[p_val8], pv9 = P.g[p_val9];
  for (int i = 0; i < n; ++i) {
    const int ti = s.type[i];
    T sum = T(0.0);
    for (auto& nb_ : s.adj[i]) sum = sum + B.BO[nb_.second];
    B.S[i] = sum;
    B.Delta[i] = sum - P.a[a_val][ti];
    const T De = sum - P.a[a_val_e][ti];
    B.Dang[i] = sum - P.a[a_val_ang][ti];
    const double nlp_opt = 0.5 * (P.a[a_val_e][ti] - P.a[a_val][ti]);
    const double tr = std::trunc(re(De) / 2.0);   // integer part, zero derivative
    B.vlpex[i] = De - 2.0 * tr;
    B.nlp[i] = exp(-plp1 * sq(2.0 + B.vlpex[i])) - tr;
    B.Dlp[i] = nlp_opt - B.nlp[i];
    // SBO: pi bond orders of the centre plus a lone-pair / valence term
    T sumpi = T(0.0), prod = T(1.0);
    for (auto& nb_ : s.adj[i]) {
      const int b = nb_.second;
      sumpi = sumpi + (B.BOp[b] + B.BOpp[b]);
      const T b2 = B.BO[b] * B.BO[b];
      const T b4 = b2 * b2;
      prod = prod * exp(-(b4 * b4));
    }
    const T vlpadj = re(B.vlpex[i]) < 0.0 ? B.nlp[i] : T(0.0);
    B.SBO[i] = sumpi + (1.0 - prod) * (-B.Dang[i] - pv8 * vlpadj);
    const double sv = re(B.SBO[i]);
    if (sv <= 0.0) B.SBO2[i] = T(0.0);
    else if (sv <= 1.0) B.SBO2[i] = pow(B.SBO[i], pv9);
    else if (sv < 2.0) B.SBO2[i] = 2.0 - pow(2.0 - B.SBO[i], pv9);
    else B.SBO2[i] = T(2.0);
  }
}

template <class T, class Sink>
void energy(const Sys& s, const T* x, BondStage<T>& B, Sink& sink) {
  using std::exp; using std::log; using std::pow; using std::sqrt;
  const Params& P = s.P;
  const Cutoffs& c = s.c;
  const int n = s.n, nb = (int)s.bi.size();
  bond_stage(s, x, B);

  // (4) bond energy, per undirected bond
  for (int b = 0; b < nb; ++b) {
    const int ti = s.type[s.bi[b]], tj = s.type[s.bj[b]];
    const size_t mark = sink.begin();
    // the sigma power is taken only for a positive sigma bond order (reading
    // for BOsig <= 0: the power is zero, which keeps E continuous and smooth)
    const T pw = re(B.BOsig[b]) > 0.0 ? pow(B.BOsig[b], P.p[p_be2][ti][tj]) : T(0.0);
    const T e = -P.p[D_s][ti][tj] * B.BOsig[b] * exp(P.p[p_be1][ti][tj] * (1.0 - pw)) -
                P.p[D_p][ti][tj] * B.BOp[b] - P.p[D_pp][ti][tj] * B.BOpp[b];
    sink.add(E_BOND, e);
    sink.end(mark);
  }

  // (5) lone pair, over- and under-coordination, per atom
  const double po3 = P.g[p_ovun3], po4 = P.g[p_ovun4], po6 = P.g[p_ovun6],
               po7 = P.g[p_ovun7], po8 = P.g[p_ovun8];
  for (int i = 0; i < n; ++i) {
    const int ti = s.type[i];
    const size_t mark = sink.begin();
    const T elp = P.a[a_p_lp2][ti] * B.Dlp[i] / (1.0 + exp(-75.0 * B.Dlp[i]));
    T sumpi = T(0.0), sumov = T(0.0);
    for (auto& nb_ : s.adj[i]) {
      const int j = nb_.first, b = nb_.second, tj = s.type[j];
      sumpi = sumpi + (B.Delta[j] - B.Dlp[j]) * (B.BOp[b] + B.BOpp[b]);
      sumov = sumov + P.p[p_ovun1][ti][tj] * P.p[D_s][ti][tj] * B.BO[b];
    }
    const T Dlpc = B.Delta[i] - B.Dlp[i] / (1.0 + po3 * exp(po4 * sumpi));
    const double po2 = P.a[a_p_ovun2][ti];
    const T eover = sumov * (Dlpc / (Dlpc + P.a[a_val][ti] + 1e-8)) * (1.0 / (1.0 + exp(po2 * Dlpc)));
    const T eunder = -P.a[a_p_ovun5][ti] * (1.0 - exp(po6 * Dlpc)) / (1.0 + exp(-po2 * Dlpc)) *
                     (1.0 / (1.0 + po7 * exp(po8 * sumpi)));
    sink.add(E_LP, elp);
    sink.add(E_OVER, eover);
    sink.add(E_UNDER, eunder);
    sink.end(mark);
  }

  // (6) valence angle, penalty and coalition: centre j, unordered pairs of bonds
  const double pv6 = P.g[p_val6], pv10 = P.g[p_val10], pp2 = P.g[p_pen2],
               pp3 = P.g[p_pen3], pp4 = P.g[p_pen4], pc2 = P.g[p_coa2],
               pc3 = P.g[p_coa3], pc4 = P.g[p_coa4];
  for (int j = 0; j < n; ++j) {
    const int tj = s.type[j];
    const auto& aj = s.adj[j];
    for (size_t u = 0; u < aj.size(); ++u) {
      for (size_t v = u + 1; v < aj.size(); ++v) {
        const int i = aj[u].first, bij = aj[u].second;
        const int k = aj[v].first, bjk = aj[v].second;
        const double bo_ij = re(B.BO[bij]), bo_jk = re(B.BO[bjk]);
        if (!(bo_ij - c.thb_cut > 0.0 && bo_jk - c.thb_cut > 0.0 && bo_ij * bo_jk > c.thb_cutsq)) continue;
        const int ti = s.type[i], tk = s.type[k];
        const size_t mark = sink.begin();
        const T BOA_ij = B.BO[bij] - c.thb_cut, BOA_jk = B.BO[bjk] - c.thb_cut;
        T rji[3], rjk[3];
        dvec(s, x, j, i, rji);
        dvec(s, x, j, k, rjk);
        T cr[3];
        cross3(rji, rjk, cr);
        const T theta = angle_of(sqrt(dot3(cr, cr)), dot3(rji, rjk));
        const T theta0 = PI - (PI / 180.0) * P.ang[theta00][ti][tj][tk] *
                                  (1.0 - exp(-pv10 * (2.0 - B.SBO2[j])));
        const double pv3 = P.a[a_p_val3][tj], pv4 = P.ang[p_val4][ti][tj][tk];
        const T f7ij = 1.0 - exp(-pv3 * pow(BOA_ij, pv4));
        const T f7jk = 1.0 - exp(-pv3 * pow(BOA_jk, pv4));
        const double pv5 = P.a[a_p_val5][tj], pv7 = P.ang[p_val7][ti][tj][tk];
        const T e6 = exp(pv6 * B.Dang[j]), e7 = exp(-pv7 * B.Dang[j]);
        const T f8 = pv5 - (pv5 - 1.0) * (2.0 + e6) / (1.0 + e6 + e7);
        const T eval = f7ij * f7jk * f8 * P.ang[p_val1][ti][tj][tk] *
                       (1.0 - exp(-P.ang[p_val2][ti][tj][tk] * sq(theta0 - theta)));
        const T ep3 = exp(-pp3 * B.Delta[j]), ep4 = exp(pp4 * B.Delta[j]);
        const T f9 = (2.0 + ep3) / (1.0 + ep3 + ep4);
        const T epen = P.ang[p_pen1][ti][tj][tk] * f9 * exp(-pp2 * sq(BOA_ij - 2.0)) *
                       exp(-pp2 * sq(BOA_jk - 2.0));
        const T ecoa = P.ang[p_coa1][ti][tj][tk] / (1.0 + exp(pc2 * B.Dang[j])) *
                       exp(-pc3 * sq(B.S[i] - BOA_ij)) * exp(-pc3 * sq(B.S[k] - BOA_jk)) *
                       exp(-pc4 * sq(BOA_ij - 1.5)) * exp(-pc4 * sq(BOA_jk - 1.5));
        sink.add(E_VAL, eval);
        sink.add(E_PEN, epen);
        sink.add(E_COA, ecoa);
        sink.end(mark);
      }
    }
  }

  // (7) torsion and 4-body conjugation: each central bond j-k once
  const double pt2 = P.g[p_tor2], pt3 = P.g[p_tor3], pt4 = P.g[p_tor4], pcot2 = P.g[p_cot2];
  for (int b = 0; b < nb; ++b) {
    const int j = s.bi[b], k = s.bj[b];
    const double bo_jk = re(B.BO[b]);
    if (!(bo_jk > c.thb_cut)) continue;
    for (auto& ni : s.adj[j]) {
      const int i = ni.first, bij = ni.second;
      if (i == k) continue;
      const double bo_ij = re(B.BO[bij]);
      if (!(bo_ij > c.thb_cut)) continue;
      for (auto& nl : s.adj[k]) {
        const int l = nl.first, bkl = nl.second;
        if (l == j || l == i) continue;
        const double bo_kl = re(B.BO[bkl]);
        if (!(bo_kl > c.thb_cut)) continue;
        if (!(bo_ij * bo_jk * bo_kl > c.thb_cut)) continue;
        const int ti = s.type[i], tj = s.type[j], tk = s.type[k], tl = s.type[l];
        const size_t mark = sink.begin();
        T b1[3], b2[3], b3[3];
        dvec(s, x, i, j, b1);   // x_j - x_i
        dvec(s, x, j, k, b2);   // x_k - x_j
        dvec(s, x, k, l, b3);   // x_l - x_k
        T c1[3], c2[3];
        cross3(b1, b2, c1);
        cross3(b2, b3, c2);
        T n1 = sqrt(dot3(c1, c1)), n2 = sqrt(dot3(c2, c2));
        if (re(n1) < 1e-20) n1 = T(1e-20);
        if (re(n2) < 1e-20) n2 = T(1e-20);
        const T cw = dot3(c1, c2) / (n1 * n2);
        const T l1 = sqrt(dot3(b1, b1)), l2 = sqrt(dot3(b2, b2)), l3 = sqrt(dot3(b3, b3));
        // angle i-j-k between r_ji = -b1 and r_jk = b2; angle j-k-l between r_kj = -b2 and r_kl = b3
        // their sines from the cross products (|r_ji x r_jk| = |b1 x b2|)
        const T sin_ijk = n1 / (l1 * l2), sin_jkl = n2 / (l2 * l3);
        const T BOA_ij = B.BO[bij] - c.thb_cut, BOA_jk = B.BO[b] - c.thb_cut,
                BOA_kl = B.BO[bkl] - c.thb_cut;
        const T f10 = (1.0 - exp(-pt2 * BOA_ij)) * (1.0 - exp(-pt2 * BOA_jk)) *
                      (1.0 - exp(-pt2 * BOA_kl));
        const T D = B.Dang[j] + B.Dang[k];
        const T et3 = exp(-pt3 * D), et4 = exp(pt4 * D);
        const T f11 = (2.0 + et3) / (1.0 + et3 + et4);
        const T cos2w = 2.0 * cw * cw - 1.0;
        const T cos3w = 4.0 * cw * cw * cw - 3.0 * cw;
        const T etor = f10 * sin_ijk * sin_jkl * 0.5 *
                       (P.tor[V1][ti][tj][tk][tl] * (1.0 + cw) +
                        P.tor[V2][ti][tj][tk][tl] *
                            exp(P.tor[p_tor1][ti][tj][tk][tl] * sq(2.0 - B.BOp[b] - f11)) *
                            (1.0 - cos2w) +
                        P.tor[V3][ti][tj][tk][tl] * (1.0 + cos3w));
        const T econj = P.tor[p_cot1][ti][tj][tk][tl] * exp(-pcot2 * sq(BOA_ij - 1.5)) *
                        exp(-pcot2 * sq(BOA_jk - 1.5)) * exp(-pcot2 * sq(BOA_kl - 1.5)) *
                        (1.0 + (cw * cw - 1.0) * sin_ijk * sin_jkl);
        sink.add(E_TOR, etor);
        sink.add(E_CONJ, econj);
        sink.end(mark);
      }
    }
  }

  // (8) hydrogen bonds: H atom h, bonded acceptor-type X, listed acceptor Z != X
  for (int h = 0; h < n; ++h) {
    const int th = s.type[h];
    if (P.a[a_p_hbond][th] != 1.0) continue;
    for (auto& nx : s.adj[h]) {
      const int X = nx.first, bhx = nx.second, tx = s.type[X];
      if (P.a[a_p_hbond][tx] != 2.0) continue;
      if (!(re(B.BO[bhx]) >= c.hb_bo_cut)) continue;
      for (int Z : s.hbl[h]) {
        if (Z == X) continue;
        const int tz = s.type[Z];
        const size_t mark = sink.begin();
        T rx[3], rz[3];
        dvec(s, x, h, X, rx);
        dvec(s, x, h, Z, rz);
        const T lx = sqrt(dot3(rx, rx)), lz = sqrt(dot3(rz, rz));
        const T cth = dot3(rx, rz) / (lx * lz);
        const T s4 = sq((1.0 - cth) / 2.0);
        const double r0 = P.hb[r0hb][tx][th][tz];
        const T e = P.hb[p_hb1][tx][th][tz] * (1.0 - exp(-P.hb[p_hb2][tx][th][tz] * B.BO[bhx])) *
                    exp(-P.hb[p_hb3][tx][th][tz] * (r0 / lz + lz / r0 - 2.0)) * s4;
        sink.add(E_HB, e);
        sink.end(mark);
      }
    }
  }

  // (9) van der Waals and Coulomb over every far pair (no bonded exclusions)
  const double R = c.r_nonb, pw1 = P.g[p_vdW1];
  for (const auto& pr : s.far) {
    const int i = pr.first, j = pr.second, ti = s.type[i], tj = s.type[j];
    const size_t mark = sink.begin();
    T d[3];
    dvec(s, x, i, j, d);
    const T r = sqrt(dot3(d, d));
    const T u = r / R;
    const T u2 = u * u, u4 = u2 * u2;
    const T tap = 20.0 * u4 * u2 * u - 70.0 * u4 * u2 + 84.0 * u4 * u - 35.0 * u4 + 1.0;
    const T f13 = pow(pow(r, pw1) + std::pow(P.p[gamma_w][ti][tj], -pw1), 1.0 / pw1);
    const double a = P.p[alpha][ti][tj], rv = P.p[r_vdw][ti][tj];
    const T ev = P.p[D_vdw][ti][tj] * (exp(a * (1.0 - f13 / rv)) - 2.0 * exp(0.5 * a * (1.0 - f13 / rv))) +
                 P.p[e_core][ti][tj] * exp(P.p[a_core][ti][tj] * (1.0 - r / P.p[r_core][ti][tj]));
    const T ec = C_ELE * s.q[i] * s.q[j] /
                 pow(r * r * r + std::pow(P.p[gamma_c][ti][tj], -3.0), 1.0 / 3.0);
    sink.add(E_VDW, tap * ev);
    sink.add(E_COUL, tap * ec);
    sink.end(mark);
  }
}

// ---------------------------------------------------------------------------
// drivers
// ---------------------------------------------------------------------------
static void energies_double(const Sys& s, double* E, double* Eabs = nullptr) {
  DoubleSink sink;
  BondStage<double> B;
  energy<double>(s, s.x.data(), B, sink);
  for (int t = 0; t < NTERMS; ++t) E[t] = sink.E[t].value();
  if (Eabs)
    for (int t = 0; t < NTERMS; ++t) Eabs[t] = sink.A[t].value();
}

static void energies_forces(const Sys& s, double* E, double* F) {
  ad::Tape tape;
  ad::tape = &tape;
  std::vector<Var> xv(3 * s.n);
  for (int k = 0; k < 3 * s.n; ++k) xv[k] = ad::leaf(s.x[k]);
  AdSink sink;
  {
    BondStage<Var> B;
    energy<Var>(s, xv.data(), B, sink);
  }
  tape.sweep_to(3 * s.n);   // the shared stage, down to the position leaves
  for (int k = 0; k < 3 * s.n; ++k) F[k] = -tape.adj[k];
  for (int t = 0; t < NTERMS; ++t) E[t] = sink.E[t].value();
  ad::tape = nullptr;
}

}  // namespace oracle

using namespace oracle;

extern "C" {

int oracle_param_counts(int32_t out[6]) {
  out[0] = NG; out[1] = NA; out[2] = NP; out[3] = NANG; out[4] = NT; out[5] = NH;
  return 0;
}

const char* oracle_error(void) { return g_err.c_str(); }

void* oracle_new(int32_t n, const double* pos, const int32_t* type, const double* q,
                 const double* box, const double* general, const double* atom,
                 const double* pair, const double* angle, const double* tors,
                 const double* hb, const double* cutoffs, int32_t brute) {
  if (n < 0 || (n > 0 && (!pos || !type || !q))) { g_err = "bad arguments"; return nullptr; }
  auto s = std::make_unique<Sys>();
  s->n = n;
  s->x.assign(pos, pos + 3 * (size_t)n);
  s->type.assign(type, type + n);
  s->q.assign(q, q + n);
  for (int i = 0; i < n; ++i)
    if (s->type[i] < 0 || s->type[i] > 3) { g_err = "type index out of range"; return nullptr; }
  std::memcpy(s->P.g, general, sizeof(s->P.g));
  std::memcpy(s->P.a, atom, sizeof(s->P.a));
  std::memcpy(s->P.p, pair, sizeof(s->P.p));
  std::memcpy(s->P.ang, angle, sizeof(s->P.ang));
  std::memcpy(s->P.tor, tors, sizeof(s->P.tor));
  std::memcpy(s->P.hb, hb, sizeof(s->P.hb));
  s->c = Cutoffs{cutoffs[0], cutoffs[1], cutoffs[2], cutoffs[3], cutoffs[4], cutoffs[5], cutoffs[6]};
  s->brute = brute != 0;
  if (box) {
    s->periodic = true;
    for (int k = 0; k < 3; ++k) {
      s->L[k] = box[k];
      s->invL[k] = 1.0 / box[k];
      if (box[k] < 2.0 * s->c.r_nonb) { g_err = "periodic box edge below 2 r_nonb"; return nullptr; }
    }
  }
  build_lists(*s);
  return s.release();
}

void oracle_free(void* h) { delete static_cast<Sys*>(h); }

int oracle_set_positions(void* h, const double* pos) {
  Sys& s = *static_cast<Sys*>(h);
  s.x.assign(pos, pos + 3 * (size_t)s.n);
  build_lists(s);
  return 0;
}

void oracle_list_sizes(void* h, int64_t sizes[3]) {
  const Sys& s = *static_cast<Sys*>(h);
  sizes[0] = (int64_t)s.far.size();
  sizes[1] = 2 * (int64_t)s.bi.size();
  int64_t k = 0;
  for (auto& v : s.hbl) k += (int64_t)v.size();
  sizes[2] = k;
}

void oracle_get_lists(void* h, int32_t* far, int32_t* bonds, int32_t* hb) {
  const Sys& s = *static_cast<Sys*>(h);
  size_t k = 0;
  for (auto& p : s.far) { far[2 * k] = p.first; far[2 * k + 1] = p.second; ++k; }
  k = 0;
  for (int i = 0; i < s.n; ++i)
    for (auto& nb : s.adj[i]) { bonds[2 * k] = i; bonds[2 * k + 1] = nb.first; ++k; }
  k = 0;
  for (int i = 0; i < s.n; ++i)
    for (int z : s.hbl[i]) { hb[2 * k] = i; hb[2 * k + 1] = z; ++k; }
}

double oracle_bo_raw(void* h, int32_t i, int32_t j) {
  return bo_raw_at(*static_cast<Sys*>(h), i, j);
}

int oracle_energy(void* h, double* E) {
  energies_double(*static_cast<Sys*>(h), E);
  return 0;
}

int oracle_energy_abs(void* h, double* E, double* Eabs) {
  energies_double(*static_cast<Sys*>(h), E, Eabs);
  return 0;
}

int oracle_forces(void* h, double* E, double* F) {
  energies_forces(*static_cast<Sys*>(h), E, F);
  return 0;
}

int oracle_energy_cs(void* h, int32_t atom, int32_t comp, double hstep, double* Ere, double* Eim) {
  const Sys& s = *static_cast<Sys*>(h);
  if (atom < 0 || atom >= s.n || comp < 0 || comp > 2) { g_err = "bad coordinate"; return -1; }
  std::vector<cplx> xc(3 * s.n);
  for (int k = 0; k < 3 * s.n; ++k) xc[k] = cplx(s.x[k], 0.0);
  xc[3 * atom + comp] += cplx(0.0, hstep);
  ComplexSink sink;
  BondStage<cplx> B;
  energy<cplx>(s, xc.data(), B, sink);
  for (int t = 0; t < NTERMS; ++t) { Ere[t] = sink.E[t].real(); Eim[t] = sink.E[t].imag(); }
  return 0;
}

int oracle_atom_terms(void* h, double* out) {
  const Sys& s = *static_cast<Sys*>(h);
  BondStage<double> B;
  bond_stage<double>(s, s.x.data(), B);
  for (int i = 0; i < s.n; ++i) {
    double* o = out + 8 * (size_t)i;
    o[0] = B.Dp[i]; o[1] = B.Dboc[i]; o[2] = B.S[i]; o[3] = B.Delta[i];
    o[4] = B.nlp[i]; o[5] = B.Dlp[i]; o[6] = B.SBO[i]; o[7] = B.SBO2[i];
  }
  return 0;
}

int oracle_bond_terms(void* h, double* out) {
  const Sys& s = *static_cast<Sys*>(h);
  BondStage<double> B;
  bond_stage<double>(s, s.x.data(), B);
  size_t k = 0;
  for (int i = 0; i < s.n; ++i)
    for (auto& nb : s.adj[i]) {
      const int b = nb.second;
      double* o = out + 7 * k;
      o[0] = B.BO[b]; o[1] = B.BOp[b]; o[2] = B.BOpp[b]; o[3] = B.BOt[b];
      o[4] = B.BOs[b]; o[5] = B.BOpi[b]; o[6] = B.BOpi2[b];
      ++k;
    }
  return 0;
}

int oracle_md(void* h, double* pos, double* vel, double dt, int32_t nsteps, double* energies) {
  Sys& s = *static_cast<Sys*>(h);
  const int n = s.n;
  s.x.assign(pos, pos + 3 * (size_t)n);
  build_lists(s);
  std::vector<double> F(3 * n), E(NTERMS);
  auto kinetic = [&]() {
    Neumaier ke;
    for (int i = 0; i < n; ++i) {
      const double m = s.P.a[a_mass][s.type[i]];
      for (int k = 0; k < 3; ++k) ke.add(0.5 * m * vel[3 * i + k] * vel[3 * i + k] / ACC_CONV);
    }
    return ke.value();
  };
  auto record = [&](int step) {
    for (int t = 0; t < NTERMS; ++t) energies[(size_t)step * (NTERMS + 1) + t] = E[t];
    energies[(size_t)step * (NTERMS + 1) + NTERMS] = kinetic();
  };
  energies_forces(s, E.data(), F.data());
  record(0);
  for (int st = 1; st <= nsteps; ++st) {
    for (int i = 0; i < n; ++i) {
      const double m = s.P.a[a_mass][s.type[i]];
      for (int k = 0; k < 3; ++k) {
        vel[3 * i + k] += 0.5 * dt * ACC_CONV * F[3 * i + k] / m;
        double xk = s.x[3 * i + k] + dt * vel[3 * i + k];
        if (s.periodic) xk -= s.L[k] * std::floor(xk * s.invL[k]);
        s.x[3 * i + k] = xk;
      }
    }
    build_lists(s);
    energies_forces(s, E.data(), F.data());
    for (int i = 0; i < n; ++i) {
      const double m = s.P.a[a_mass][s.type[i]];
      for (int k = 0; k < 3; ++k) vel[3 * i + k] += 0.5 * dt * ACC_CONV * F[3 * i + k] / m;
    }
    record(st);
  }
  std::memcpy(pos, s.x.data(), sizeof(double) * 3 * (size_t)n);
  return 0;
}

}  // extern "C"
