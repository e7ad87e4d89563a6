// Per-atom and per-interaction ReaxFF arithmetic, shared by the kernels of
// the large-system path (one launch per stage, forces.hip) and the batched
// cluster kernel (all stages inside one workgroup, batch.hip).  Each function
// works on the Lists/Work views of reaxff_dev.h; the batched kernel points
// some of those views at LDS.
#pragma once

#include "reaxff_dev.h"

namespace rx {

// ---------------------------------------------------------------------------
// FP64 elementary functions written for the arguments of the force terms
// (exp_f, log_f for finite positive x; exp_c and pow_c for any argument):
//   exp_f:   Cody-Waite reduction x = k ln2 + r, |r| <= ln2/2, with ln 2
//            split into a head of 29 significant bits (k * head exact for
//            |k| < 2^24) and a tail; exp(r) from a degree-11 polynomial,
//            scaled by 2^k.  The polynomial is the Taylor series to degree 13
//            economized by Chebyshev polynomials on |r| <= 0.3466 (Lanczos:
//            the r^13 and r^12 terms replaced through T_13 and T_12), which
//            adds at most 3.1e-18 to the series' 4.1e-18 truncation.
//   log_f:   x = 2^e m with m in [1/sqrt2, sqrt2); log m = 2 atanh(s) with
//            s = (m - 1)/(m + 1), |s| < 0.172, log m = 2s + 2s z p(z),
//            z = s^2, where p(z) = sum_k z^k / (2k + 3) to k = 8 (truncation
//            below 1e-17) economized to degree 6 by shifted Chebyshev
//            polynomials on z in [0, 0.02944]: |p error| < 1.6e-16, so the
//            relative error it adds to log m is below z * 1.6e-16 < 5e-18.
//   rcbrt_f: x^(-1/3) from a single-precision seed y = 2^(-log2(x)/3)
//            (relative error about 1e-7) and one step of the series
//            (1 - e)^(-1/3) = 1 + e/3 + 2e^2/9 + ..., e = 1 - x y^3, taken to
//            second order: y <- y (1 + e (1/3 + 2e/9)); the error left is
//            about e^3 / 6, far below rounding.
//   rcp_f:   1/x from the hardware reciprocal estimate and two Newton steps
//            y <- y (2 - x y).
//   rsq_f:   x^(-1/2) for finite x > 0 from the hardware estimate y and one
//            third-order step y + y e (1/2 + 3/8 e), e = 1 - x y^2.
//   exp_c:   exp_f after clamping the argument to [-1000, 1000] (exp is 0 or
//            infinity beyond; the reduction then stays exact); NaN passes.
//   pow_c:   x^y = exp_c(y log x) for x > 0, with 0^y spelled out.
// Each is within a few units in the last place, far inside the 1e-9
// relative agreement asked of energies and forces.  poly_coeffs.py beside
// this file derives the exp and log coefficients (exact rationals rounded to
// double).
// ---------------------------------------------------------------------------
constexpr double LN2_HEAD = 0x1.62e42ff000000p-1;
constexpr double LN2_TAIL = -0x1.718432a1b0e26p-35;
constexpr double LOG2_E = 1.4426950408889634;

__device__ __forceinline__ double exp_f(double x) {
  const double k = rint(x * LOG2_E);
  double r = fma(-k, LN2_HEAD, x);
  r = fma(-k, LN2_TAIL, r);
  double p = 0x1.af781738d6a07p-26;
  p = fma(p, r, 0x1.28b3cc02abb37p-22);
  p = fma(p, r, 0x1.71dde78463672p-19);
  p = fma(p, r, 0x1.a01991d2b4315p-16);
  p = fma(p, r, 0x1.a01a01b7fa994p-13);
  p = fma(p, r, 0x1.6c16c187f21d0p-10);
  p = fma(p, r, 0x1.111111110db86p-7);
  p = fma(p, r, 0x1.555555554f0f0p-5);
  p = fma(p, r, 0x1.5555555555562p-3);
  p = fma(p, r, 0x1.0000000000011p-1);
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
  return ldexp(p, (int)k);
}

__device__ __forceinline__ double rcp_f(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = y * fma(-x, y, 2.0);
  y = y * fma(-x, y, 2.0);
  return y;
}

__device__ __forceinline__ double rsq_f(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = fma(-x * y, y, 1.0);
  return fma(y * e, fma(0.375, e, 0.5), y);
}

__device__ __forceinline__ double log_f(double x) {
  int e;
  double m = frexp(x, &e);
  if (m < 0.7071067811865476) {
    m *= 2.0;
    e -= 1;
  }
  const double f = m - 1.0;
  const double s = f * rcp_f(2.0 + f);
  const double z = s * s;
  double p = 0x1.2b4b69e452555p-4;
  p = fma(p, z, 0x1.39ff0e0e536dep-4);
  p = fma(p, z, 0x1.7462b13e69a0bp-4);
  p = fma(p, z, 0x1.c71c62ecdd1abp-4);
  p = fma(p, z, 0x1.2492492dee8abp-3);
  p = fma(p, z, 0x1.99999999952e2p-3);
  p = fma(p, z, 0x1.5555555555558p-2);
  const double lm = fma(2.0 * s * z, p, 2.0 * s);
  const double de = (double)e;
  return fma(de, LN2_HEAD, fma(de, LN2_TAIL, lm));
}

__device__ __forceinline__ double rcbrt_f(double x) {
  const float xf = (float)x;
  const double y = (double)__builtin_amdgcn_exp2f(__builtin_amdgcn_logf(xf) * (-1.0f / 3.0f));
  const double e = fma(-x, y * y * y, 1.0);
  return fma(y, e * fma(e, 2.0 / 9.0, 1.0 / 3.0), y);
}

// exp_r, log_r: exp_f and log_f with the same reductions and polynomials,
// but the integer steps done on the bit pattern, with no conversion, frexp or
// ldexp instruction.  exp_r rounds x log2(e) to an integer k with the
// 1.5 * 2^52 shifter (k is then the low word of the sum) and multiplies by
// 2^k by adding k to the exponent field of the polynomial's value (in
// [0.70, 1.42]), so it needs |x| < 700.  log_r reads the exponent and the
// mantissa of a positive normal x from its bits (the mantissa is halved when
// its top 20 bits reach those of sqrt 2) and forms the exponent as a double
// by the 2^52 + 2^31 offset.  The pair term calls them: its arguments stay
// far inside these ranges.
__device__ __forceinline__ double exp_r(double x) {
  constexpr double SH = 0x1.8p52;
  const double ks = fma(x, LOG2_E, SH);
  const int k = __double2loint(ks);
  const double kd = ks - SH;
  double r = fma(-kd, LN2_HEAD, x);
  r = fma(-kd, LN2_TAIL, r);
  double p = 0x1.af781738d6a07p-26;
  p = fma(p, r, 0x1.28b3cc02abb37p-22);
  p = fma(p, r, 0x1.71dde78463672p-19);
  p = fma(p, r, 0x1.a01991d2b4315p-16);
  p = fma(p, r, 0x1.a01a01b7fa994p-13);
  p = fma(p, r, 0x1.6c16c187f21d0p-10);
  p = fma(p, r, 0x1.111111110db86p-7);
  p = fma(p, r, 0x1.555555554f0f0p-5);
  p = fma(p, r, 0x1.5555555555562p-3);
  p = fma(p, r, 0x1.0000000000011p-1);
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
  return __hiloint2double(__double2hiint(p) + (k << 20), __double2loint(p));
}

__device__ __forceinline__ double log_r(double x) {
  const int hi = __double2hiint(x);
  const int mb = hi & 0x000fffff;
  const int up = mb >= 0x6a09e ? 1 : 0;   // mantissa at or above sqrt 2: halve it
  const int e = (hi >> 20) - 1023 + up;
  const double m = __hiloint2double(mb | ((1023 - up) << 20), __double2loint(x));
  const double f = m - 1.0;
  const double s = f * rcp_f(2.0 + f);
  const double z = s * s;
  double p = 0x1.2b4b69e452555p-4;
  p = fma(p, z, 0x1.39ff0e0e536dep-4);
  p = fma(p, z, 0x1.7462b13e69a0bp-4);
  p = fma(p, z, 0x1.c71c62ecdd1abp-4);
  p = fma(p, z, 0x1.2492492dee8abp-3);
  p = fma(p, z, 0x1.99999999952e2p-3);
  p = fma(p, z, 0x1.5555555555558p-2);
  const double lm = fma(2.0 * s * z, p, 2.0 * s);
  const double de = __hiloint2double(0x43300000, e ^ (int)0x80000000) - 0x1.00000800p52;
  return fma(de, LN2_HEAD, fma(de, LN2_TAIL, lm));
}

__device__ __forceinline__ double exp_c(double x) {
  x = x < -1000.0 ? -1000.0 : (x > 1000.0 ? 1000.0 : x);
  return exp_f(x);
}

__device__ __forceinline__ double pow_c(double x, double y) {
  if (x > 0.0) return exp_c(y * log_f(x));
  if (x == 0.0) return y > 0.0 ? 0.0 : (y == 0.0 ? 1.0 : __builtin_inf());
  return __builtin_nan("");
}


__device__ __forceinline__ void atomic_add3(double4* p, double x, double y, double z) {
  double* d = reinterpret_cast<double*>(p);
  atomicAdd(d + 0, x);
  atomicAdd(d + 1, y);
  atomicAdd(d + 2, z);
}
__device__ __forceinline__ double3 cross(double3 a, double3 b) {
  return make_double3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double dot(double3 a, double3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ double3 d3(double4 v) { return make_double3(v.x, v.y, v.z); }
__device__ __forceinline__ double3 axpy(double a, double3 x, double3 y) {
  return make_double3(a * x.x + y.x, a * x.y + y.y, a * x.z + y.z);
}
__device__ __forceinline__ double3 scale(double a, double3 x) { return make_double3(a * x.x, a * x.y, a * x.z); }
__device__ __forceinline__ double3 add3(double3 a, double3 b) { return make_double3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ void atomic_add3(double4* p, double3 v) { atomic_add3(p, v.x, v.y, v.z); }

// raw uncorrected bond order sum of sigma, pi and pi-pi (the bond-list test)
// ((r / r_x)^p as exp(p (log r - log r_x)): one log for the three terms)
// (PP: PairP, or any record with the same bond-order members, such as a
// workgroup's LDS copy of them)
template <class PP>
__device__ __forceinline__ double bo_raw(const PP& p, double r, double bo_cut) {
  double s = 0.0, pi = 0.0, pp = 0.0;
  const double lr = log_f(r);
  if (p.r_s > 0.0) s = (1.0 + bo_cut) * exp_c(p.p_bo1 * exp_c(p.p_bo2 * (lr - p.ln_r_s)));
  if (p.r_p > 0.0) pi = exp_c(p.p_bo3 * exp_c(p.p_bo4 * (lr - p.ln_r_p)));
  if (p.r_pp > 0.0) pp = exp_c(p.p_bo5 * exp_c(p.p_bo6 * (lr - p.ln_r_pp)));
  return s + pi + pp;
}

// ---------------------------------------------------------------------------
// (1) uncorrected bond orders of atom i's entries, computed in a canonical
//     orientation (lower index first) so both entries of a bond hold
//     identical bits
// ---------------------------------------------------------------------------
__device__ __forceinline__ void bo_prime_entry(const DevParams* __restrict__ P, const Grid& g,
                                               const Lists& L, const Work& W, int i, int e) {
  const double4 xi = L.xs[i];
  const int ti = L.type_s[i];
  const double bo_cut = P->bo_cut;
  {
    const int j = L.bond_j[e];
    const double4 xj = L.xs[j];
    const bool lo = i < j;
    // d = x_b - x_a with a the lower index
    double dx = lo ? xj.x - xi.x : xi.x - xj.x;
    double dy = lo ? xj.y - xi.y : xi.y - xj.y;
    double dz = lo ? xj.z - xi.z : xi.z - xj.z;
    if (g.periodic) {
      dx = min_image(dx, g.L[0], g.invL[0]);
      dy = min_image(dy, g.L[1], g.invL[1]);
      dz = min_image(dz, g.L[2], g.invL[2]);
    }
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    W.bd[e] = lo ? make_double4(dx, dy, dz, r) : make_double4(-dx, -dy, -dz, r);
    const PairP& p = P->pair[ti * NT + L.type_s[j]];
    double s = 0.0, ds = 0.0, pi = 0.0, dpi = 0.0, pp = 0.0, dpp = 0.0;
    const double ir = rcp_f(r);
    const double lr = log_f(r);   // (r / r_x)^p = exp(p (log r - log r_x))
    if (p.r_s > 0.0) {
      const double x = exp_c(p.p_bo2 * (lr - p.ln_r_s));
      s = (1.0 + bo_cut) * exp_c(p.p_bo1 * x);
      ds = s * p.p_bo1 * p.p_bo2 * x * ir;
    }
    if (p.r_p > 0.0) {
      const double x = exp_c(p.p_bo4 * (lr - p.ln_r_p));
      pi = exp_c(p.p_bo3 * x);
      dpi = pi * p.p_bo3 * p.p_bo4 * x * ir;
    }
    if (p.r_pp > 0.0) {
      const double x = exp_c(p.p_bo6 * (lr - p.ln_r_pp));
      pp = exp_c(p.p_bo5 * x);
      dpp = pp * p.p_bo5 * p.p_bo6 * x * ir;
    }
    const double raw = s + pi + pp;
    W.bop[e] = make_double4(s - bo_cut, pi, pp, raw - bo_cut);
    W.dbop[e] = make_double4(ds, dpi, dpp, 0.0);
  }
}
__device__ __forceinline__ void bo_prime_atom(const DevParams* __restrict__ P, const Grid& g,
                                              const Lists& L, const Work& W, int i) {
  for (int e = L.bond_off[i]; e < L.bond_off[i + 1]; ++e) bo_prime_entry(P, g, L, W, i, e);
}

// (2) Delta'_i = sum BO' - Val_i,  Delta'boc_i = sum BO' - Val_boc_i
//     (G = 4: a quad of lanes per atom, lane sub over entries sub, sub + 4, ...)
template <int G = 1>
__device__ __forceinline__ void delta_prime_atom(const DevParams* __restrict__ P, const Lists& L,
                                                 const Work& W, int i, int sub = 0) {
  double s = 0.0;
  for (int e = L.bond_off[i] + sub; e < L.bond_off[i + 1]; e += G) s += W.bop[e].w;
  if constexpr (G == 4) s = quad_sum(s);
  if (sub != 0) return;
  const AtomP& a = P->atom[L.type_s[i]];
  W.dp[i] = make_double2(s - a.val, s - a.val_boc);
}

// bond-order correction of one bond, canonical orientation (a lower index)
struct Corr {
  double f1, f4, f5;
  double df1_da, df1_db;     // d f1 / d Delta'_a, d Delta'_b
  double df4_dbo, df5_dbo;   // d f4 / d BO', d f5 / d BO'
  double df4_da, df5_db;     // d f4 / d Delta'boc_a, d f5 / d Delta'boc_b
};

__device__ __forceinline__ Corr correction(const DevParams* __restrict__ P, double bop, double va,
                                           double vb, double2 da, double2 db, const PairP& p) {
  Corr c;
  const double ea1 = exp_c(-P->p_boc1 * da.x), eb1 = exp_c(-P->p_boc1 * db.x);
  const double ea2 = exp_c(-P->p_boc2 * da.x), eb2 = exp_c(-P->p_boc2 * db.x);
  const double f2 = ea1 + eb1;
  const double u = 0.5 * (ea2 + eb2);
  const double f3 = -(1.0 / P->p_boc2) * log_f(u);
  const double A = va + f2, Ad = va + f2 + f3;
  const double B = vb + f2, Bd = vb + f2 + f3;
  c.f1 = 0.5 * (A / Ad + B / Bd);
  const double df1_df2 = 0.5 * (f3 / (Ad * Ad) + f3 / (Bd * Bd));
  const double df1_df3 = -0.5 * (A / (Ad * Ad) + B / (Bd * Bd));
  const double w2 = 1.0 / (ea2 + eb2);
  c.df1_da = df1_df2 * (-P->p_boc1 * ea1) + df1_df3 * (ea2 * w2);
  c.df1_db = df1_df2 * (-P->p_boc1 * eb1) + df1_df3 * (eb2 * w2);
  const double bo2 = bop * bop;
  const double e4 = exp_c(-p.p_boc3 * (p.p_boc4 * bo2 - da.y) + p.p_boc5);
  const double e5 = exp_c(-p.p_boc3 * (p.p_boc4 * bo2 - db.y) + p.p_boc5);
  c.f4 = 1.0 / (1.0 + e4);
  c.f5 = 1.0 / (1.0 + e5);
  const double s4 = c.f4 * (1.0 - c.f4), s5 = c.f5 * (1.0 - c.f5);
  c.df4_dbo = s4 * 2.0 * p.p_boc3 * p.p_boc4 * bop;
  c.df5_dbo = s5 * 2.0 * p.p_boc3 * p.p_boc4 * bop;
  c.df4_da = -s4 * p.p_boc3;
  c.df5_db = -s5 * p.p_boc3;
  return c;
}

// (3) corrected bond orders of atom i's entries
__device__ __forceinline__ void bo_corr_entry(const DevParams* __restrict__ P, const Lists& L,
                                              const Work& W, int i, int e) {
  const int ti = L.type_s[i];
  {
    const int j = L.bond_j[e];
    const int tj = L.type_s[j];
    const bool lo = i < j;
    const int a = lo ? i : j, b = lo ? j : i;
    const int ta = lo ? ti : tj, tb = lo ? tj : ti;
    const double4 bp = W.bop[e];
    const Corr c = correction(P, bp.w, P->atom[ta].val, P->atom[tb].val, W.dp[a], W.dp[b],
                              P->pair[ti * NT + tj]);
    const double F = c.f1 * c.f4 * c.f5;
    const double G = c.f1 * c.f1 * c.f4 * c.f5;
    const double BO = bp.w * F, BOp = bp.y * G, BOpp = bp.z * G;
    W.bo[e] = make_double4(BO, BOp, BOpp, BO - BOp - BOpp);
    if (W.bo1) W.bo1[e] = BO;
  }
}
__device__ __forceinline__ void bo_corr_atom(const DevParams* __restrict__ P, const Lists& L,
                                             const Work& W, int i) {
  for (int e = L.bond_off[i]; e < L.bond_off[i + 1]; ++e) bo_corr_entry(P, L, W, i, e);
}

// (4) atom state
__device__ __forceinline__ void atom_state_atom(const DevParams* __restrict__ P, const Lists& L,
                                                const Work& W, int i) {
  const AtomP& a = P->atom[L.type_s[i]];
  double S = 0.0, sumpi = 0.0, sum8 = 0.0;
  for (int e = L.bond_off[i]; e < L.bond_off[i + 1]; ++e) {
    const double4 b = W.bo[e];
    S += b.x;
    sumpi += b.y + b.z;
    const double b2 = b.x * b.x, b4 = b2 * b2;
    sum8 += b4 * b4;
  }
  AtomState st;
  st.S = S;
  st.Delta = S - a.val;
  st.Dang = S - a.val_ang;
  const double De = S - a.val_e;
  const double tr = trunc(De * 0.5);
  const double vlpex = De - 2.0 * tr;
  const double enlp = exp_c(-P->p_lp1 * sqr(2.0 + vlpex));
  const double nlp = enlp - tr;
  st.Dlp = a.nlp_opt - nlp;
  st.dnlp = enlp * (-2.0 * P->p_lp1 * (2.0 + vlpex));
  st.prod = exp_c(-sum8);
  const bool neg = vlpex < 0.0;
  st.W = -st.Dang - P->p_val8 * (neg ? nlp : 0.0);
  st.dW = -1.0 - P->p_val8 * (neg ? st.dnlp : 0.0);
  const double SBO = sumpi + (1.0 - st.prod) * st.W;
  const double p9 = P->p_val9;
  if (SBO <= 0.0) {
    st.SBO2 = 0.0; st.dSBO2 = 0.0;
  } else if (SBO <= 1.0) {
    const double t = pow_c(SBO, p9);
    st.SBO2 = t; st.dSBO2 = p9 * t / SBO;
  } else if (SBO < 2.0) {
    const double t = pow_c(2.0 - SBO, p9);
    st.SBO2 = 2.0 - t; st.dSBO2 = p9 * t / (2.0 - SBO);
  } else {
    st.SBO2 = 2.0; st.dSBO2 = 0.0;
  }
  // centre factors of the valence-angle family
  const double ex10 = exp_c(-P->p_val10 * (2.0 - st.SBO2));
  st.th0f = 1.0 - ex10;
  st.dth0f = -ex10 * P->p_val10;                 // d th0f / d SBO2
  st.e6 = exp_c(P->p_val6 * st.Dang);
  const double ep3 = exp_c(-P->p_pen3 * st.Delta), ep4 = exp_c(P->p_pen4 * st.Delta);
  const double f9d = 1.0 + ep3 + ep4;
  st.f9 = (2.0 + ep3) / f9d;
  st.df9 = (-P->p_pen3 * ep3 * f9d - (2.0 + ep3) * (-P->p_pen3 * ep3 + P->p_pen4 * ep4)) / (f9d * f9d);
  const double ec = exp_c(P->p_coa2 * st.Dang);
  st.fc = 1.0 / (1.0 + ec);
  st.dfc = -P->p_coa2 * ec * st.fc * st.fc;
  W.ast[i] = st;
  if (W.nv) W.nv[i] = make_double4(st.S, st.Delta - st.Dlp, st.Dang, st.prod * st.W);
}

// corrected total bond order of entry e (the compact copy when there is one)
__device__ __forceinline__ double bo_tot(const Work& W, int e) { return W.bo1 ? W.bo1[e] : W.bo[e].x; }

// what a term centred elsewhere reads of atom j (S, Delta - Dlp, Dang,
// prod W): the compact record when there is one
__device__ __forceinline__ double4 nview(const Work& W, int j) {
  if (W.nv) return W.nv[j];
  const AtomState& s = W.ast[j];
  return make_double4(s.S, s.Delta - s.Dlp, s.Dang, s.prod * s.W);
}

// (5) bond energy (once per bond, from its lower-index entry), lone pair,
//     over- and under-coordination of atom i; adds the scalar adjoints to i's
//     own entries and sets gS[i], gSig[i].  e[0..3] += bond, lp, over, under.
//     G = 4: the four lanes of an aligned group share atom i, lane sub taking
//     entries sub, sub + 4, ...; the sums are combined across the group and
//     the atom's own terms are added by lane 0 only.
template <int G = 1>
__device__ __forceinline__ void atom_energy_atom(const DevParams* __restrict__ P, const Lists& L,
                                                 const Work& W, int i, double e[4], int sub = 0) {
  static_assert(G == 1 || G == 4, "one lane or a quad per atom");
  const int ti = L.type_s[i];
  const AtomP& a = P->atom[ti];
  const AtomState st = W.ast[i];
  double sumpi = 0.0, sumov = 0.0, ebond = 0.0;
#pragma unroll 4
  for (int e = L.bond_off[i] + sub; e < L.bond_off[i + 1]; e += G) {
    const int j = L.bond_j[e];
    const int tj = L.type_s[j];
    const PairP& p = P->pair[ti * NT + tj];
    const double4 b = W.bo[e];
    sumpi += nview(W, j).y * (b.y + b.z);
    sumov += p.p_ovun1 * p.D_s * b.x;
    if (i < j) {
      const double sig = b.w;
      const double pw = sig > 0.0 ? pow_c(sig, p.p_be2) : 0.0;
      const double ex = exp_c(p.p_be1 * (1.0 - pw));
      ebond += -p.D_s * sig * ex - p.D_p * b.y - p.D_pp * b.z;
      const double dsig = -p.D_s * ex * (1.0 - p.p_be1 * p.p_be2 * pw);
      double4 gb = W.gbo[e];
      gb.x += dsig;
      gb.y += -p.D_p - dsig;
      gb.z += -p.D_pp - dsig;
      W.gbo[e] = gb;
    }
  }
  if constexpr (G == 4) {
    sumpi = quad_sum(sumpi);
    sumov = quad_sum(sumov);
  }
  // lone pair
  const double e75 = exp_c(-75.0 * st.Dlp);
  const double den75 = 1.0 / (1.0 + e75);
  const double elp = a.p_lp2 * st.Dlp * den75;
  const double dElp_dDlp = a.p_lp2 * (den75 + st.Dlp * 75.0 * e75 * den75 * den75);
  // over / under
  const double ep4 = exp_c(P->p_ovun4 * sumpi);
  const double DD = 1.0 + P->p_ovun3 * ep4;
  const double Dlpc = st.Delta - st.Dlp / DD;
  const double Vp = a.val + 1e-8;
  const double R = Dlpc / (Dlpc + Vp);
  const double dR = Vp / sqr(Dlpc + Vp);
  const double so = 1.0 / (1.0 + exp_c(a.p_ovun2 * Dlpc));
  const double dso = -a.p_ovun2 * so * (1.0 - so);
  const double eover = sumov * R * so;
  const double e6 = exp_c(P->p_ovun6 * Dlpc);
  const double su = 1.0 / (1.0 + exp_c(-a.p_ovun2 * Dlpc));
  const double dsu = a.p_ovun2 * su * (1.0 - su);
  const double ep8 = exp_c(P->p_ovun8 * sumpi);
  const double t8 = 1.0 / (1.0 + P->p_ovun7 * ep8);
  const double eunder = -a.p_ovun5 * (1.0 - e6) * su * t8;
  const double gL = sumov * (dR * so + R * dso) +
                    (-a.p_ovun5 * t8) * (-P->p_ovun6 * e6 * su + (1.0 - e6) * dsu);
  const double dt8 = -P->p_ovun7 * P->p_ovun8 * ep8 * t8 * t8;
  const double dDlpc_dsig = st.Dlp * P->p_ovun3 * P->p_ovun4 * ep4 / (DD * DD);
  const double gSig = -a.p_ovun5 * (1.0 - e6) * su * dt8 + gL * dDlpc_dsig;
  // the over/under terms' adjoints of i's entries, p_ovun1 D_s R so on BO
  // and gSig (Delta_j - Dlp_j) on BOpi and BOpipi, are added where the
  // entries' adjoints are read (back_corr_entry), from gRso and gSig
  e[0] += ebond;
  if (sub != 0) return;
  W.gS[i] = dElp_dDlp * (-st.dnlp) + gL * (1.0 + st.dnlp / DD);
  W.gSig[i] = gSig;
  W.gRso[i] = R * so;
  e[1] += elp;
  e[2] += eover;
  e[3] += eunder;
}

// ---------------------------------------------------------------------------
// (6) one valence angle i-j-k given by the centre's entries u = j->i and
//     v = j->k: energies and the adjoints to deposit
// ---------------------------------------------------------------------------
struct AngOut {
  double gu[5], gv[5];   // gvec (x, y, z), gbo.x, gbo.w of entries u and v
  double gS, gSBO2;      // centre adjoints: dE/dS (via Dang, Delta), dE/dSBO2
  double ev, ep, ec;     // valence, penalty, coalition energies
};

__device__ __forceinline__ AngOut angle_eval(const DevParams* __restrict__ P, const Lists& L,
                                             const Work& W, int u, int v) {
  AngOut o;
  const double thb = P->thb_cut;
  const int j = L.bond_i[u], i = L.bond_j[u], k = L.bond_j[v];
  const int ti = L.type_s[i], tj = L.type_s[j], tk = L.type_s[k];
  const AtomP& aj = P->atom[tj];
  const AngleP& ap = P->angle[(ti * NT + tj) * NT + tk];
  const AtomState& st = W.ast[j];
  const double4 ru = W.bd[u], rv = W.bd[v];
  const double B1 = bo_tot(W, u) - thb, B2 = bo_tot(W, v) - thb;
  const double Si = nview(W, i).x, Sk = nview(W, k).x;
  // angle between a = r_ji (= bd[u]) and b = r_jk (= bd[v]), from |a x b| and
  // a . b (no digits lost next to a straight angle, unlike the arccosine)
  const double il1 = 1.0 / ru.w, il2 = 1.0 / rv.w;
  const double3 av = d3(ru), bv = d3(rv);
  const double3 cr = cross(av, bv);
  const double ncr = sqrt(dot(cr, cr));
  const double th = atan2(ncr, dot(av, bv));
  const double th0 = PI - ap.theta00_rad * st.th0f;
  const double dth0 = -ap.theta00_rad * st.dth0f;     // d th0 / d SBO2
  // f7
  const double x1 = pow_c(B1, ap.p_val4), x2 = pow_c(B2, ap.p_val4);
  const double g1 = exp_c(-aj.p_val3 * x1), g2 = exp_c(-aj.p_val3 * x2);
  const double f7a = 1.0 - g1, f7b = 1.0 - g2;
  const double df7a = aj.p_val3 * ap.p_val4 * x1 / B1 * g1;
  const double df7b = aj.p_val3 * ap.p_val4 * x2 / B2 * g2;
  // f8
  const double e6 = st.e6;
  const double e7 = exp_c(-ap.p_val7 * st.Dang);
  const double f8d = 1.0 + e6 + e7;
  const double f8 = aj.p_val5 - (aj.p_val5 - 1.0) * (2.0 + e6) / f8d;
  const double df8 = -(aj.p_val5 - 1.0) *
                     (P->p_val6 * e6 * f8d - (2.0 + e6) * (P->p_val6 * e6 - ap.p_val7 * e7)) /
                     (f8d * f8d);
  const double dt = th0 - th;
  const double ev = exp_c(-ap.p_val2 * dt * dt);
  const double Ea = f7a * f7b * f8 * ap.p_val1;
  const double Ev = Ea * (1.0 - ev);
  const double gdt = Ea * ev * 2.0 * ap.p_val2 * dt;   // dE/d(th0 - th)
  double gB1 = df7a * f7b * f8 * ap.p_val1 * (1.0 - ev);
  double gB2 = f7a * df7b * f8 * ap.p_val1 * (1.0 - ev);
  double gS = f7a * f7b * df8 * ap.p_val1 * (1.0 - ev);      // via Dang
  o.gSBO2 = gdt * dth0;
  // penalty
  const double pe1 = exp_c(-P->p_pen2 * sqr(B1 - 2.0)), pe2 = exp_c(-P->p_pen2 * sqr(B2 - 2.0));
  const double Ep = ap.p_pen1 * st.f9 * pe1 * pe2;
  gB1 += Ep * (-2.0 * P->p_pen2 * (B1 - 2.0));
  gB2 += Ep * (-2.0 * P->p_pen2 * (B2 - 2.0));
  gS += ap.p_pen1 * st.df9 * pe1 * pe2;                       // via Delta
  // coalition
  const double ci = exp_c(-P->p_coa3 * sqr(Si - B1)), ck = exp_c(-P->p_coa3 * sqr(Sk - B2));
  const double cb1 = exp_c(-P->p_coa4 * sqr(B1 - 1.5)), cb2 = exp_c(-P->p_coa4 * sqr(B2 - 1.5));
  const double Ec = ap.p_coa1 * st.fc * ci * ck * cb1 * cb2;
  gS += ap.p_coa1 * st.dfc * ci * ck * cb1 * cb2;            // via Dang
  const double gSi = Ec * (-2.0 * P->p_coa3 * (Si - B1));
  const double gSk = Ec * (-2.0 * P->p_coa3 * (Sk - B2));
  gB1 += Ec * (2.0 * P->p_coa3 * (Si - B1) - 2.0 * P->p_coa4 * (B1 - 1.5));
  gB2 += Ec * (2.0 * P->p_coa3 * (Sk - B2) - 2.0 * P->p_coa4 * (B2 - 1.5));
  o.ev = Ev;
  o.ep = Ep;
  o.ec = Ec;
  o.gS = gS;
  // geometry: d theta / d a = -(c x a) / (|a|^2 |c|) and d theta / d b =
  // -(b x c) / (|b|^2 |c|), c = a x b: the in-plane directions away from the
  // other bond, with no sine formed from the cosine; dE/dtheta = -gdt.  (At an
  // exactly straight angle the direction is undefined and the term is left
  // without a geometric gradient.)
  const double inc = ncr > 0.0 ? 1.0 / ncr : 0.0;
  const double3 ta = cross(cr, av), tb = cross(bv, cr);
  const double ga = gdt * inc * il1 * il1, gb = gdt * inc * il2 * il2;
  o.gu[0] = ga * ta.x;
  o.gu[1] = ga * ta.y;
  o.gu[2] = ga * ta.z;
  o.gu[3] = gB1;
  o.gu[4] = gSi;
  o.gv[0] = gb * tb.x;
  o.gv[1] = gb * tb.y;
  o.gv[2] = gb * tb.z;
  o.gv[3] = gB2;
  o.gv[4] = gSk;
  return o;
}

// ---------------------------------------------------------------------------
// (7) one torsion i-j-k-l (entries ejk = j->k, eji = j->i, ekl = k->l):
//     energies into etor/econj, adjoints deposited with atomic adds
// ---------------------------------------------------------------------------
// adjoints of one torsion term: gradients of the three entries' vectors
// (entry j->i, j->k, k->l), of their bond orders, and of Delta_j, Delta_k
struct TorOut {
  double3 gji, gjk, gkl;
  double gBij, gBjk, gPjk, gBkl, gD;
};

__device__ __forceinline__ TorOut torsion_terms(const DevParams* __restrict__ P, const Lists& L,
                                                const Work& W, int ejk, int eji, int ekl, double& etor,
                                                double& econj) {
  const double thb = P->thb_cut, pt2 = P->p_tor2, pc2 = P->p_cot2;
  const int j = L.bond_i[ejk], k = L.bond_j[ejk], i = L.bond_j[eji], l = L.bond_j[ekl];
  const int ti = L.type_s[i], tj = L.type_s[j], tk = L.type_s[k], tl = L.type_s[l];
  const TorsP& tp = P->tors[((ti * NT + tj) * NT + tk) * NT + tl];
  const double4 bjk = W.bo[ejk];
  const double bij = bo_tot(W, eji), bkl = bo_tot(W, ekl);
  // f11 of the central bond
  const double Dsum = nview(W, j).z + nview(W, k).z;
  const double et3 = exp_c(-P->p_tor3 * Dsum), et4 = exp_c(P->p_tor4 * Dsum);
  const double f11d = 1.0 + et3 + et4;
  const double f11 = (2.0 + et3) / f11d;
  const double df11 = (-P->p_tor3 * et3 * f11d - (2.0 + et3) * (-P->p_tor3 * et3 + P->p_tor4 * et4)) /
                      (f11d * f11d);
  const double Bij = bij - thb, Bjk = bjk.x - thb, Bkl = bkl - thb;
  const double xij = exp_c(-pt2 * Bij), xjk = exp_c(-pt2 * Bjk), xkl = exp_c(-pt2 * Bkl);
  const double hij = 1.0 - xij, hjk = 1.0 - xjk, hkl = 1.0 - xkl;
  const double dhij = pt2 * xij, dhjk = pt2 * xjk, dhkl = pt2 * xkl;
  const double cij = exp_c(-pc2 * sqr(Bij - 1.5)), cjk = exp_c(-pc2 * sqr(Bjk - 1.5)),
               ckl = exp_c(-pc2 * sqr(Bkl - 1.5));
  const double pi2 = 2.0 - bjk.y - f11;
  // geometry: b1 = x_j - x_i = -r_ji, b2 = x_k - x_j, b3 = x_l - x_k
  const double4 r1v = W.bd[eji], r2v = W.bd[ejk], r3v = W.bd[ekl];
  const double3 b1 = make_double3(-r1v.x, -r1v.y, -r1v.z), b2 = d3(r2v), b3 = d3(r3v);
  const double l1 = r1v.w, l2 = r2v.w, l3 = r3v.w;
  const double3 m = cross(b1, b2), nv = cross(b2, b3);
  const double nm = fmax(sqrt(dot(m, m)), 1e-20), nn = fmax(sqrt(dot(nv, nv)), 1e-20);
  // sines of the angles i-j-k and j-k-l from the cross products
  // (|r_ji x r_jk| = |b1 x b2|, |r_kj x r_kl| = |b2 x b3|)
  const double s1 = nm / (l1 * l2), s2 = nn / (l2 * l3);
  const double cw = dot(m, nv) / (nm * nn);
  const double ss = s1 * s2;
  const double f10 = hij * hjk * hkl;
  const double exv = exp_c(tp.p_tor1 * pi2 * pi2);
  const double c2w = 2.0 * cw * cw - 1.0;
  const double c3w = 4.0 * cw * cw * cw - 3.0 * cw;
  const double Vt = 0.5 * (tp.V1 * (1.0 + cw) + tp.V2 * exv * (1.0 - c2w) + tp.V3 * (1.0 + c3w));
  const double Et = f10 * ss * Vt;
  const double f12 = cij * cjk * ckl;
  const double Ec = tp.p_cot1 * f12 * (1.0 + (cw * cw - 1.0) * ss);
  etor += Et;
  econj += Ec;
  // scalar adjoints
  const double dVt_dcw = 0.5 * (tp.V1 - 4.0 * tp.V2 * exv * cw + tp.V3 * (12.0 * cw * cw - 3.0));
  // d exv / d BOpi_jk = d exv / d f11 = -2 p_tor1 pi2 exv
  const double dex = 0.5 * tp.V2 * (1.0 - c2w) * exv * tp.p_tor1 * 2.0 * pi2 * (-1.0);
  const double gPjk = f10 * ss * dex;
  const double gD = f10 * ss * dex * df11;
  const double gss = f10 * Vt + tp.p_cot1 * f12 * (cw * cw - 1.0);
  const double gcw = f10 * ss * dVt_dcw + tp.p_cot1 * f12 * 2.0 * cw * ss;
  const double gBij = dhij * hjk * hkl * ss * Vt + Ec * (-2.0 * pc2 * (Bij - 1.5));
  const double gBjk = hij * dhjk * hkl * ss * Vt + Ec * (-2.0 * pc2 * (Bjk - 1.5));
  const double gBkl = hij * hjk * dhkl * ss * Vt + Ec * (-2.0 * pc2 * (Bkl - 1.5));
  // cos w gradients
  const double inm = 1.0 / (nm * nn);
  const double3 Gm = axpy(-cw / (nm * nm), m, scale(inm, nv));
  const double3 Gn = axpy(-cw / (nn * nn), nv, scale(inm, m));
  const double3 dcw_b1 = cross(b2, Gm);
  const double3 dcw_b2 = add3(cross(Gm, b1), cross(b3, Gn));
  const double3 dcw_b3 = cross(Gn, b2);
  // s1 = |m| / (l1 l2) with d|m| = (b2 x mh) . db1 + (mh x b1) . db2, mh = m / |m|
  // (likewise s2 with n = b2 x b3)
  const double gs1 = gss * s2, gs2 = gss * s1;
  const double i12 = 1.0 / (l1 * l2), i23 = 1.0 / (l2 * l3);
  const double3 mh = scale(1.0 / nm, m), nh = scale(1.0 / nn, nv);
  const double3 ds1_b1 = axpy(-s1 / (l1 * l1), b1, scale(i12, cross(b2, mh)));
  const double3 ds1_b2 = axpy(-s1 / (l2 * l2), b2, scale(i12, cross(mh, b1)));
  const double3 ds2_b2 = axpy(-s2 / (l2 * l2), b2, scale(i23, cross(b3, nh)));
  const double3 ds2_b3 = axpy(-s2 / (l3 * l3), b3, scale(i23, cross(nh, b2)));
  const double3 gb1 = axpy(gs1, ds1_b1, scale(gcw, dcw_b1));
  const double3 gb2 = axpy(gs2, ds2_b2, axpy(gs1, ds1_b2, scale(gcw, dcw_b2)));
  const double3 gb3 = axpy(gs2, ds2_b3, scale(gcw, dcw_b3));
  // entry j->i holds r_ji = -b1; j->k holds b2; k->l holds b3
  TorOut o;
  o.gji = make_double3(-gb1.x, -gb1.y, -gb1.z);
  o.gjk = gb2;
  o.gkl = gb3;
  o.gBij = gBij;
  o.gBjk = gBjk;
  o.gPjk = gPjk;
  o.gBkl = gBkl;
  o.gD = gD;
  return o;
}

// one torsion, its adjoints added with global atomics
__device__ __forceinline__ void torsion_eval(const DevParams* __restrict__ P, const Lists& L,
                                             const Work& W, int ejk, int eji, int ekl, double& etor,
                                             double& econj) {
  const TorOut o = torsion_terms(P, L, W, ejk, eji, ekl, etor, econj);
  const int j = L.bond_i[ejk], k = L.bond_j[ejk];
  atomic_add3(&W.gvec[eji], o.gji);
  atomic_add3(&W.gvec[ejk], o.gjk);
  atomic_add3(&W.gvec[ekl], o.gkl);
  atomicAdd(&W.gbo[eji].x, o.gBij);
  atomicAdd(&W.gbo[ejk].x, o.gBjk);
  atomicAdd(&W.gbo[ejk].y, o.gPjk);
  atomicAdd(&W.gbo[ekl].x, o.gBkl);
  atomicAdd(&W.gS[j], o.gD);
  atomicAdd(&W.gS[k], o.gD);
}

// ---------------------------------------------------------------------------
// (8) one hydrogen-bond term X-H...Z from the H-X bond order, r_hX (with its
//     length in w) and r_hZ = (dx, dy, dz)
// ---------------------------------------------------------------------------
struct HbTerm {
  double E, dE_dbo;
  double3 g_rx, g_rz;   // dE/d(x_X - x_h), dE/d(x_Z - x_h)
};

__device__ __forceinline__ HbTerm hb_term(const HbP& hp, double bo, double4 rx, double dx, double dy,
                                          double dz) {
  HbTerm o;
  // reciprocals and the length from rcp_f / rsqrt (a few ulp), not IEEE
  // division and square root
  const double ilx = rcp_f(rx.w);
  const double ilz = rsq_f(dx * dx + dy * dy + dz * dz);
  const double rz = (dx * dx + dy * dy + dz * dz) * ilz;
  const double ir0 = rcp_f(hp.r0hb);
  const double c = (rx.x * dx + rx.y * dy + rx.z * dz) * ilx * ilz;
  const double hc = 0.5 * (1.0 - c);
  const double s4 = hc * hc;
  const double ds4 = -hc;                 // d s4 / d c
  const double eb = exp_c(-hp.p_hb2 * bo);
  const double fbo = 1.0 - eb, dfbo = hp.p_hb2 * eb;
  const double fr = exp_c(-hp.p_hb3 * (hp.r0hb * ilz + rz * ir0 - 2.0));
  const double dfr = fr * (-hp.p_hb3) * (-hp.r0hb * ilz * ilz + ir0);
  o.E = hp.p_hb1 * fbo * fr * s4;
  o.dE_dbo = hp.p_hb1 * dfbo * fr * s4;
  const double gc = hp.p_hb1 * fbo * fr * ds4;
  const double grz = hp.p_hb1 * fbo * dfr * s4;
  o.g_rx = make_double3(gc * (dx * ilx * ilz - c * rx.x * ilx * ilx), gc * (dy * ilx * ilz - c * rx.y * ilx * ilx),
                        gc * (dz * ilx * ilz - c * rx.z * ilx * ilx));
  o.g_rz = make_double3(gc * (rx.x * ilx * ilz - c * dx * ilz * ilz) + grz * dx * ilz,
                        gc * (rx.y * ilx * ilz - c * dy * ilz * ilz) + grz * dy * ilz,
                        gc * (rx.z * ilx * ilz - c * dz * ilz * ilz) + grz * dz * ilz);
  return o;
}


// ---------------------------------------------------------------------------
// (9) one van der Waals + Coulomb pair at squared distance r2: tapered
//     shielded Morse with inner wall, tapered shielded Coulomb.  qq = q_i q_j
//     C_ele.  Returns the two energies and f = (dE/dr) / r.
// ---------------------------------------------------------------------------
// (halpha = alpha / 2; Dar = D alpha / r_vdw; acr = a_core / r_core)
struct NbP { double D, halpha, inv_rv, gw_pow, g3, e_core, a_core, acr, Dar; };

struct NbOut { double ev, eq, f; };

__device__ __forceinline__ NbOut nb_pair(const NbP& p, double iR, double pv, double ipv, double qq,
                                         double r2) {
  const double ir = rsq_f(r2);
  const double r = r2 * ir;
  // taper 1 - 35u^4 + 84u^5 - 70u^6 + 20u^7 in Horner form, and its
  // derivative 140 u^3 (u - 1)^3 / R
  const double u = r * iR, u2 = u * u, u4 = u2 * u2;
  const double tap = fma(u4, fma(u, fma(u, fma(20.0, u, -70.0), 84.0), -35.0), 1.0);
  const double um = u - 1.0;
  const double dtap = (140.0 * iR) * (u2 * u) * (um * um * um);
  // shielded Morse with inner wall
  const double pw = exp_r(pv * log_r(r));
  const double sum = pw + p.gw_pow;
  const double isum = rcp_f(sum);
  const double f13 = exp_r(ipv * log_r(sum));
  const double df13 = f13 * isum * pw * ir;
  const double t = 1.0 - f13 * p.inv_rv;
  const double e2 = exp_r(p.halpha * t);
  const double e1 = e2 * e2;
  const double ev = p.D * (e1 - 2.0 * e2);
  const double dev = -p.Dar * (e1 - e2) * df13;
  const double ecr = p.e_core * exp_r(fma(-p.acr, r, p.a_core));   // a_core (1 - r / r_core)
  const double decr = -ecr * p.acr;
  // shielded Coulomb: den = (r^3 + gamma^-3)^(1/3), 1/s3 = (1/den)^3
  const double s3 = r2 * r + p.g3;
  const double iden = rcbrt_f(s3);
  const double eq = qq * iden;
  const double deq = -eq * r2 * (iden * iden * iden);
  const double Ev = ev + ecr;
  NbOut o;
  o.ev = tap * Ev;
  o.eq = tap * eq;
  o.f = (dtap * (Ev + eq) + tap * (dev + decr + deq)) * ir;
  return o;
}

__device__ __forceinline__ NbP nb_params(const PairP& p) {
  return NbP{p.D_vdw, 0.5 * p.alpha, p.inv_r_vdw, p.gw_pow, p.g3, p.e_core, p.a_core, p.a_core * p.inv_r_core,
             p.D_vdw * p.alpha * p.inv_r_vdw};
}

// ---------------------------------------------------------------------------
// backward
// ---------------------------------------------------------------------------
// (10) total dE/dS of atom i: own terms, coalition terms of angles centred on
//      neighbours (stored in the neighbour's entry), the Sigma_pi term of the
//      neighbours' over/under-coordination, and SBO's valence term
//      (G = 4: a quad of lanes per atom, as in atom_energy_atom)
template <int G = 1>
__device__ __forceinline__ void back_s_atom(const Lists& L, const Work& W, int i, int sub = 0) {
  static_assert(G == 1 || G == 4, "one lane or a quad per atom");
  double g = 0.0;
  double gsig = 0.0;
  for (int e = L.bond_off[i] + sub; e < L.bond_off[i + 1]; e += G) {
    const int m = L.bond_mir[e];
    const int j = L.bond_j[e];
    g += W.gbo[m].w;
    const double4 b = W.bo[e];
    gsig += W.gSig[j] * (b.y + b.z);
  }
  if constexpr (G == 4) {
    g = quad_sum(g);
    gsig = quad_sum(gsig);
  }
  if (sub != 0) return;
  const AtomState st = W.ast[i];
  g += W.gS[i];
  g += (1.0 + st.dnlp) * gsig;
  // the angle terms accumulated dE/dSBO2; convert to dE/dSBO for the next stage
  const double gsbo = W.gSBO[i] * st.dSBO2;
  W.gSBO[i] = gsbo;
  g += gsbo * (1.0 - st.prod) * st.dW;
  W.gStot[i] = g;
}

// (11) through the correction to the uncorrected orders and Delta'
__device__ __forceinline__ void back_corr_entry(const DevParams* __restrict__ P, const Lists& L,
                                                const Work& W, int i, int e) {
  const int ti = L.type_s[i];
  {
    const int j = L.bond_j[e];
    const int m = L.bond_mir[e];
    const int tj = L.type_s[j];
    const bool lo = i < j;
    const int a = lo ? i : j, b = lo ? j : i;
    const int ea = lo ? e : m, eb = lo ? m : e;
    const int ta = lo ? ti : tj, tb = lo ? tj : ti;
    const double4 bp = W.bop[e];
    const double4 bo = W.bo[e];
    const double4 na = nview(W, a), nb = nview(W, b);
    const double pwa = na.w, pwb = nb.w;   // prod W of a and b
    double4 ga = W.gbo[ea], gb = W.gbo[eb];
    {
      // over/under-coordination adjoints of the two entries (atom_energy_atom)
      const PairP& pa = P->pair[ta * NT + tb];
      const PairP& pb = P->pair[tb * NT + ta];
      ga.x += pa.p_ovun1 * pa.D_s * W.gRso[a];
      gb.x += pb.p_ovun1 * pb.D_s * W.gRso[b];
      const double wa = W.gSig[a] * nb.y, wb = W.gSig[b] * na.y;
      ga.y += wa;
      ga.z += wa;
      gb.y += wb;
      gb.z += wb;
    }
    const double gsa = W.gSBO[a], gsb = W.gSBO[b];
    const double b2 = bo.x * bo.x, b7 = b2 * b2 * b2 * bo.x;
    const double gBO = ga.x + gb.x + W.gStot[a] + W.gStot[b] + 8.0 * b7 * (gsa * pwa + gsb * pwb);
    const double gBOp = ga.y + gb.y + gsa + gsb;
    const double gBOpp = ga.z + gb.z + gsa + gsb;
    const Corr c = correction(P, bp.w, P->atom[ta].val, P->atom[tb].val, W.dp[a], W.dp[b],
                              P->pair[ti * NT + tj]);
    const double F = c.f1 * c.f4 * c.f5, G = c.f1 * c.f1 * c.f4 * c.f5;
    const double gF = gBO * bp.w;
    const double gG = gBOp * bp.y + gBOpp * bp.z;
    const double gf1 = gF * c.f4 * c.f5 + gG * 2.0 * c.f1 * c.f4 * c.f5;
    const double gf4 = gF * c.f1 * c.f5 + gG * c.f1 * c.f1 * c.f5;
    const double gf5 = gF * c.f1 * c.f4 + gG * c.f1 * c.f1 * c.f4;
    const double gBOt = gBO * F + gf4 * c.df4_dbo + gf5 * c.df5_dbo;   // uncorrected total
    const double gPi = gBOp * G, gPp = gBOpp * G;                       // uncorrected pi parts
    const double own = lo ? gf1 * c.df1_da + gf4 * c.df4_da : gf1 * c.df1_db + gf5 * c.df5_db;
    W.gup[e] = make_double4(gBOt, gPi, gPp, own);
  }
}
__device__ __forceinline__ void back_corr_atom(const DevParams* __restrict__ P, const Lists& L,
                                               const Work& W, int i) {
  for (int e = L.bond_off[i]; e < L.bond_off[i + 1]; ++e) back_corr_entry(P, L, W, i, e);
}

// (12) dE/dDelta' of atom i (Delta' and Delta'boc both are sums of BO')
template <int G = 1>
__device__ __forceinline__ void back_dp_atom(const Lists& L, const Work& W, int i, int sub = 0) {
  double g = 0.0;
  for (int e = L.bond_off[i] + sub; e < L.bond_off[i + 1]; e += G) g += W.gup[e].w;
  if constexpr (G == 4) g = quad_sum(g);
  if (sub == 0) W.gDp[i] = g;
}

// (13) force on atom i: nonbonded/H-bond part plus its bond entries
// (entries first + sub, first + sub + stride, ...; sub = 0 adds the
// nonbonded part)
__device__ __forceinline__ double3 force_atom(const Lists& L, const Work& W, int i, int sub = 0,
                                             int stride = 1) {
  double fx = 0.0, fy = 0.0, fz = 0.0;
  if (sub == 0) {
    const double4 f0 = W.fnb[i];
    fx = f0.x;
    fy = f0.y;
    fz = f0.z;
  }
  const double gi = W.gDp[i];
  for (int e = L.bond_off[i] + sub; e < L.bond_off[i + 1]; e += stride) {
    const int j = L.bond_j[e];
    const int m = L.bond_mir[e];
    const double gj = W.gDp[j];
    const double gsum = i < j ? gi + gj : gj + gi;
    const double4 gu = W.gup[e];
    const double4 db = W.dbop[e];
    const double dEdr = (gu.x + gsum) * (db.x + db.y + db.z) + gu.y * db.y + gu.z * db.z;
    const double4 d = W.bd[e];
    const double s = dEdr / d.w;
    const double4 ge = W.gvec[e], gm = W.gvec[m];
    fx += s * d.x + ge.x - gm.x;
    fy += s * d.y + ge.y - gm.y;
    fz += s * d.z + ge.z - gm.z;
  }
  return make_double3(fx, fy, fz);
}

}  // namespace rx
