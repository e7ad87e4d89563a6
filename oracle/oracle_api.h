/*
 * CPU oracle for one ReaxFF force evaluation -- test infrastructure only.
 *
 * A plain, slow, single-threaded FP64 implementation of what the GPU path
 * computes, written from the definition of the ReaxFF energy (the model the
 * paper names in Section 2.1 and evaluates per MD step, Algorithms 1-2).
 * Forces are F = -dE/dx, obtained by mechanical reverse-mode differentiation
 * of the energy expression; no force formula is written by hand.  It shares
 * no code with the HIP library and is used only by tests, the build check
 * and the CPU-baseline timing of bench.py.
 *
 * Units: Angstrom, kcal/mol, elementary charge, fs, g/mol.
 *
 * Parameter arrays are name-major: general[NG]; atom[NA][4]; pair[NP][4][4];
 * angle[NANG][4][4][4] (indexed i, centre j, k); tors[NT][4][4][4][4];
 * hb[NH][4][4][4] (indexed X, H, Z).  The name orders are the ones listed in
 * reaxff_oracle.cpp (enum blocks) and mirrored by oracle/__init__.py.
 * cutoffs[7] = r_nonb, r_bond, r_hb, bo_cut, thb_cut, thb_cutsq, hb_bo_cut.
 */
#ifndef REAXFF_ORACLE_API_H
#define REAXFF_ORACLE_API_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORACLE_NTERMS 12

/* counts of the parameter blocks, checked by the Python wrapper */
int oracle_param_counts(int32_t out[6]);

/* Create a system and build its lists (brute != 0: O(N^2) all pairs, else cells).
 * box == NULL: non-periodic.  Returns NULL on bad input (message via oracle_error). */
void* oracle_new(int32_t n, const double* pos, const int32_t* type, const double* q,
                 const double* box, const double* general, const double* atom,
                 const double* pair, const double* angle, const double* tors,
                 const double* hb, const double* cutoffs, int32_t brute);
void oracle_free(void* h);
const char* oracle_error(void);

/* Replace positions and rebuild lists. */
int oracle_set_positions(void* h, const double* pos);

/* sizes[0] = far pairs (unordered), sizes[1] = bonds (directed entries),
 * sizes[2] = H-list entries */
void oracle_list_sizes(void* h, int64_t sizes[3]);
/* far[2*M] pairs (i<j); bonds[2*B] directed (i,j); hb[2*K] (h,z) */
void oracle_get_lists(void* h, int32_t* far, int32_t* bonds, int32_t* hb);
/* uncorrected raw bond order (sigma+pi+pipi, before the threshold shift) of a pair */
double oracle_bo_raw(void* h, int32_t i, int32_t j);

/* energies only (E[ORACLE_NTERMS]) */
int oracle_energy(void* h, double* E);
/* energies and, per term, the sum of |interaction energy| (E, Eabs [ORACLE_NTERMS]) */
int oracle_energy_abs(void* h, double* E, double* Eabs);
/* energies and forces F[3n] (reverse-mode differentiation) */
int oracle_forces(void* h, double* E, double* F);
/* complex-step: energies evaluated at x + i*hstep*e_(atom,comp);
 * Ere = real parts, Eim = imaginary parts (dE/dx = Eim/hstep) */
int oracle_energy_cs(void* h, int32_t atom, int32_t comp, double hstep, double* Ere, double* Eim);
/* per-atom intermediates of the bond-order stage (for pins):
 * out[n][8] = Delta'_i, Delta'boc_i, S_i, Delta_i, nlp_i, Delta_lp_i, SBO_i, SBO2_i */
int oracle_atom_terms(void* h, double* out);
/* per-bond orders for directed bonds in the order of oracle_get_lists:
 * out[B][7] = BO, BOpi, BOpipi (corrected), BO' (uncorrected total after the
 * threshold shift), BO'sigma (shifted), BO'pi, BO'pipi */
int oracle_bond_terms(void* h, double* out);
/* velocity-Verlet NVE, lists rebuilt every step; positions wrapped into the box.
 * energies[(nsteps+1)][ORACLE_NTERMS+1]: potential terms and kinetic energy. */
int oracle_md(void* h, double* pos, double* vel, double dt, int32_t nsteps, double* energies);

#ifdef __cplusplus
}
#endif
#endif
