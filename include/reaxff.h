/*
 * reaxff.h -- C ABI of the MI355X (gfx950) ReaxFF force-evaluation library.
 *
 * One ReaxFF force evaluation per MD step, for given atomic charges: the
 * problem of the paper's Algorithms 1 and 2 (input: atom list and positions;
 * output: potential energy and per-atom forces), with the lists of its
 * Section 3.3 (half far-neighbour list in compressed-row form, full bond list
 * holding both directions, hydrogen-bond list around H atoms) and the
 * interactions named in Section 2.1 (bond orders; bond, lone pair, over- and
 * under-coordination, valence angle, torsion and hydrogen-bond terms;
 * tapered van der Waals and shielded Coulomb).  Charge equilibration is not
 * part of this library: charges are an input.
 *
 * Conventions
 *   Units: Angstrom, fs, g/mol, e, kcal/mol; forces in kcal/(mol A).
 *   Atom types: 0..3 = C, H, N, O.  Any other value -> REAXFF_ERR_ARG.
 *   Pointers marked [dev] are device memory of the context's GPU, owned by
 *   the caller (the library never frees or reallocates them); [host] pointers
 *   are host memory.  Positions are [n][3] row-major doubles, forces likewise.
 *   Outputs are in the caller's atom order.
 *   box: [host] three edge lengths of a periodic orthorhombic box with its
 *   corner at the origin (minimum image convention; every edge must be at
 *   least 2 r_nonb, else REAXFF_ERR_BOX), or NULL for a non-periodic system.
 *   Streams: all device work of a call is enqueued on `stream`.
 *   Thread safety: one context is used by one host thread at a time.
 *
 * Errors: every int-returning call returns 0 (REAXFF_OK) or a negative code;
 *   reaxff_last_error() gives the message of the context's last failure.
 */
#ifndef REAXFF_H
#define REAXFF_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define REAXFF_NTYPES 4
/* energies[] order: bond, lone pair, over-coordination, under-coordination,
 * valence angle, penalty, coalition, torsion, 4-body conjugation,
 * hydrogen bond, van der Waals (incl. inner wall), Coulomb */
#define REAXFF_NTERMS 12

enum {
  REAXFF_OK = 0,
  REAXFF_ERR_ARG = -1,       /* bad argument (null pointer, n < 0, bad type index) */
  REAXFF_ERR_CAPACITY = -2,  /* a fixed-capacity buffer is too small (batched call) */
  REAXFF_ERR_BOX = -3,       /* periodic box edge below 2 r_nonb */
  REAXFF_ERR_HIP = -4,       /* HIP runtime failure (allocation, launch) */
  REAXFF_ERR_NONFINITE = -5, /* non-finite position */
  REAXFF_ERR_STATE = -6,     /* call out of order (forces before lists, n changed) */
  REAXFF_ERR_CONVERGENCE = -7 /* an iterative solver stopped at its iteration limit */
};

/* Force-field parameters, flattened per element (C,H,N,O).  Pair tables are
 * symmetric; angle tables are indexed [i][j=centre][k] and symmetric in i,k;
 * torsion tables [i][j][k][l] are symmetric under reversal; hydrogen-bond
 * tables are indexed [X][H][Z].  A non-positive bond radius switches the
 * corresponding bond-order component off for that pair. */
typedef struct reaxff_params {
  /* general */
  double p_boc1, p_boc2, p_coa2, p_coa3, p_coa4, p_ovun3, p_ovun4, p_ovun6,
      p_ovun7, p_ovun8, p_val6, p_val8, p_val9, p_val10, p_pen2, p_pen3,
      p_pen4, p_tor2, p_tor3, p_tor4, p_cot2, p_vdW1, p_lp1;
  /* per element */
  double val[4], val_e[4], val_boc[4], val_ang[4], mass[4], p_hbond[4],
      p_lp2[4], p_ovun2[4], p_ovun5[4], p_val3[4], p_val5[4];
  /* per element pair */
  double r_s[4][4], r_p[4][4], r_pp[4][4], D_s[4][4], D_p[4][4], D_pp[4][4],
      p_be1[4][4], p_be2[4][4], p_bo1[4][4], p_bo2[4][4], p_bo3[4][4],
      p_bo4[4][4], p_bo5[4][4], p_bo6[4][4], p_ovun1[4][4], p_boc3[4][4],
      p_boc4[4][4], p_boc5[4][4], D_vdw[4][4], r_vdw[4][4], alpha[4][4],
      gamma_w[4][4], gamma[4][4], r_core[4][4], e_core[4][4], a_core[4][4];
  /* valence angle [i][j][k] */
  double theta00[4][4][4], p_val1[4][4][4], p_val2[4][4][4], p_val4[4][4][4],
      p_val7[4][4][4], p_pen1[4][4][4], p_coa1[4][4][4];
  /* torsion [i][j][k][l] */
  double V1[4][4][4][4], V2[4][4][4][4], V3[4][4][4][4], p_tor1[4][4][4][4],
      p_cot1[4][4][4][4];
  /* hydrogen bond [X][H][Z] */
  double r0hb[4][4][4], p_hb1[4][4][4], p_hb2[4][4][4], p_hb3[4][4][4];
} reaxff_params;

/* Cutoffs (A) and bond-order thresholds.  Defaults: 10, 5, 7.5, 0.01, 0.001,
 * 1e-5, 0.01. */
typedef struct reaxff_cutoffs {
  double r_nonb;    /* nonbonded cutoff; the 7th-order taper vanishes here */
  double r_bond;    /* bond-candidate distance */
  double r_hb;      /* donor H to acceptor distance */
  double bo_cut;    /* uncorrected bond-order threshold of the bond list */
  double thb_cut;   /* bond-order threshold inside angles and torsions */
  double thb_cutsq; /* bond-order product threshold of angles */
  double hb_bo_cut; /* donor bond-order threshold of hydrogen bonds */
} reaxff_cutoffs;

typedef struct reaxff_ctx reaxff_ctx;

/* Size in bytes of reaxff_params as compiled into the library (layout check). */
int64_t reaxff_params_size(void);

/* Create a context on HIP device `device` for the force field whose terms
 * Section 2.1 names (the parameter tables of those terms) with the distance
 * and bond-order cutoffs of the lists of Section 3.3 (NULL = defaults):
 * uploads the parameters.  *out receives the context; REAXFF_ERR_ARG for
 * null pointers, inconsistent cutoffs or parameter tables without the
 * symmetries reaxff_params states, REAXFF_ERR_HIP when the device
 * cannot be set up.  Device scratch (cell arrays, lists, per-bond and
 * per-atom work arrays) is owned by the context and grows inside
 * reaxff_build_lists; reaxff_destroy releases it. */
int reaxff_create(const reaxff_params* params, const reaxff_cutoffs* cutoffs,
                  int device, reaxff_ctx** out);
void reaxff_destroy(reaxff_ctx* ctx);

/* Build the three lists for n atoms (Section 3.3): cell-sort the atoms,
 * then count, prefix-sum and fill the half far-neighbour list (pairs with
 * r <= r_nonb), the full bond list (r <= r_bond and raw uncorrected bond
 * order >= bo_cut, both directions, with mirror index) and the H-bond list
 * (H donors, N/O acceptors, r <= r_hb).  pos [dev] (n,3), type [dev] (n).
 * Performs the library's only host synchronisation: one readback of the
 * list totals to size the list buffers. */
int reaxff_build_lists(reaxff_ctx* ctx, int64_t n, const double* pos,
                       const int32_t* type, const double* box, hipStream_t stream);

/* The three lists of reaxff_build_lists in device buffers the caller owns
 * (Section 3.3's far-neighbour, bond and H-bond lists; the library never
 * allocates, frees or keeps them beyond the next build).  Capacities are in
 * entries.  far_j and hb_j hold one row per atom of a width the build chooses
 * from the density (far rows: stencil slots of the neighbours, see
 * reaxff_export_lists for the atom pairs; H rows: acceptors of each H atom),
 * so they need n x width entries; bond_j and bond_mir hold the directed bond
 * entries (partner and the position of the reverse entry), bond_cap of each. */
typedef struct reaxff_lists {
  int64_t far_cap;    /* entries of far_j */
  int32_t* far_j;     /* [dev] far-list rows */
  int64_t bond_cap;   /* entries of bond_j and of bond_mir */
  int32_t* bond_j;    /* [dev] bond partners, rows per atom in the cell-sorted order */
  int32_t* bond_mir;  /* [dev] reverse entry of each bond entry */
  int64_t hb_cap;     /* entries of hb_j */
  int32_t* hb_j;      /* [dev] H-bond rows */
  int64_t required[3];/* [host] out: entries needed (far, bond, hb) */
} reaxff_lists;

/* reaxff_build_lists into the caller's buffers.  When a buffer is too small
 * the call returns REAXFF_ERR_CAPACITY with required[] set (a list whose size
 * is not known yet at that point reports an estimate), leaves the context
 * without built lists and the buffers' contents unspecified; the caller
 * grows the buffers to at least required[] and calls again (sizes can grow
 * once more as the rows fill).  On success required[] holds the sizes used.
 * Lists kept over several steps (reaxff_refresh_lists) stay in the
 * context's own storage: after this call they are built again with it. */
int reaxff_build_lists_into(reaxff_ctx* ctx, int64_t n, const double* pos, const int32_t* type,
                            const double* box, reaxff_lists* lists, hipStream_t stream);

/* reaxff_compute_forces over lists built by reaxff_build_lists_into into
 * exactly these buffers (else REAXFF_ERR_STATE). */
int reaxff_compute_forces_from(reaxff_ctx* ctx, int64_t n, const double* pos, const int32_t* type,
                               const double* q, const double* box, const reaxff_lists* lists,
                               double* forces, double* energies, hipStream_t stream);

/* One force evaluation, the problem of Algorithms 1 and 2 (input: the atom
 * list and positions; output: the potential energy and the forces), over
 * the lists of the last reaxff_build_lists call, which must have been made
 * with the same n, pos and type (else REAXFF_ERR_STATE).  q [dev] (n)
 * charges (given; QEq is reaxff_qeq).  forces [dev] (n,3) = -dE/dx and
 * energies [dev] (REAXFF_NTERMS, the terms of Section 2.1 in the order
 * above) are overwritten.  Asynchronous on `stream`. */
int reaxff_compute_forces(reaxff_ctx* ctx, int64_t n, const double* pos,
                          const int32_t* type, const double* q, const double* box,
                          double* forces, double* energies, hipStream_t stream);

/* nsteps steps of velocity-Verlet NVE (dt in fs, Section 4's MD step): lists
 * and forces at the initial positions, then per step half kick, drift
 * (positions wrapped into a periodic box), lists, forces, half kick.  Lists
 * are built every step, or with skin lists (reaxff_set_skin) refreshed as
 * reaxff_refresh_lists does, positions then being wrapped only when the
 * lists are built again.  pos, vel [dev] (n,3) in/out; forces [dev] (n,3) out:
 * the forces at the final positions.  energies [dev]
 * ((nsteps+1), REAXFF_NTERMS+1): potential terms and kinetic energy at every
 * step, step 0 first.  One host synchronisation per step (list sizes). */
int reaxff_step(reaxff_ctx* ctx, int64_t n, double* pos, double* vel,
                const int32_t* type, const double* q, const double* box,
                double dt, int32_t nsteps, double* forces, double* energies,
                hipStream_t stream);

/* Verlet-skin lists (the paper's runs check the neighbour lists every 10
 * steps, Section 4): with skin > 0 the far list, the H-bond list and the bond
 * candidates are built with every distance cutoff enlarged by `skin` (A), and
 * kept by reaxff_refresh_lists while no atom has moved more than skin / 2
 * since the build, for at most `every` (>= 1) calls; each call still remakes
 * the bond list (bond orders change every step) and the force kernels apply
 * the exact cutoffs to the kept far and H lists, so energies and forces are
 * those of exact lists.  Periodic box edges must then be at least
 * 2 (r_nonb + skin).  skin = 0 (the default): exact lists, built by every
 * call.  Takes effect at the next build; 0 <= skin <= r_nonb, else
 * REAXFF_ERR_ARG. */
int reaxff_set_skin(reaxff_ctx* ctx, double skin, int32_t every);

/* Lists for new positions of the same atoms (same n, types and box): a full
 * reaxff_build_lists when skin lists are off, when the kept lists are `every`
 * calls old, when some atom moved more than skin / 2 since the build (pos
 * compared without wrapping: positions must move continuously between
 * builds), or when n or the box changed; otherwise the kept far and H lists
 * with the current positions and a new bond list.  *rebuilt [host] (may be
 * NULL): 1 for a full build, 0 otherwise.  One host synchronisation. */
int reaxff_refresh_lists(reaxff_ctx* ctx, int64_t n, const double* pos, const int32_t* type,
                         const double* box, int32_t* rebuilt, hipStream_t stream);

/* stats[0] full list builds, stats[1] refreshes that kept the lists, since
 * the context was created [host]. */
int reaxff_list_stats(const reaxff_ctx* ctx, int64_t stats[2]);

/* Sizes of the last built lists: sizes[0] far pairs (unordered),
 * sizes[1] bond-list entries (directed), sizes[2] H-list entries. [host] */
int reaxff_list_sizes(const reaxff_ctx* ctx, int64_t sizes[3]);

/* Copy the last built lists of Section 3.3 to host memory in the caller's
 * atom order (for inspection and checking):
 * far[2*sizes[0]] as (i,j) pairs, bonds[2*sizes[1]] as directed (i,j),
 * hb[2*sizes[2]] as (h,z).  Order within each array is unspecified.
 * Any pointer may be NULL to skip that list.  Synchronises the device. */
int reaxff_export_lists(reaxff_ctx* ctx, int32_t* far, int32_t* bonds, int32_t* hb);

/* Interaction counts of the last reaxff_compute_forces [host]:
 * counts[0] valence angles, [1] torsions, [2] hydrogen bonds evaluated,
 * [3] far pairs, [4] bonds (undirected).  Synchronises the device. */
int reaxff_interaction_counts(reaxff_ctx* ctx, int64_t counts[5]);

/* Optional per-kernel timing for measurement: when enabled, every kernel
 * launch of the context is bracketed by two HIP events recorded on the
 * launch's stream.  reaxff_profile() resets the accumulators and switches
 * timing on (enable != 0) or off.  reaxff_profile_read() waits for the
 * recorded events and writes, for up to `max` kernels, the accumulated
 * milliseconds, launch counts and static kernel names (any output may be
 * NULL); it returns the number of kernels reported. */
int reaxff_profile(reaxff_ctx* ctx, int32_t enable);
int reaxff_profile_read(reaxff_ctx* ctx, int32_t max, double* ms, int64_t* launches,
                        const char** names);

/* Concurrent terms [host]: with enable != 0 (the default) the nonbonded term
 * of reaxff_compute_forces runs on a stream of the context's own,
 * concurrently with the bonded terms, joined back to the caller's stream
 * before the per-atom force gather (Section 3.2 schedules the paper's terms
 * one after another; they are independent until forces are summed).  With
 * enable == 0 every kernel runs on the caller's stream in order, so that
 * per-kernel timings measure each kernel alone.  Results are the same up to
 * the order of floating-point additions.  Returns REAXFF_OK or
 * REAXFF_ERR_ARG for a null context. */
int reaxff_set_overlap(reaxff_ctx* ctx, int32_t enable);

/* Runs of the half nonbonded evaluation [host]: Algorithm 2 visits each
 * far-list pair once (Section 3.1); the library evaluates the pairs of up to
 * run_max consecutive cells of a grid column in one workgroup, which holds the
 * neighbourhood common to those cells in its local memory once, and shortens
 * the runs when the atoms are too dense for that copy (the build then sweeps
 * again).  1 <= run_max <= 16; default 8.  Takes effect at the next build;
 * results are the same up to the order of floating-point additions.  Returns
 * REAXFF_OK, or REAXFF_ERR_ARG for a null context or run_max out of range. */
int reaxff_set_nb_run(reaxff_ctx* ctx, int32_t run_max);

/* ---- Elementary functions ----------------------------------------------------
 *
 * The force terms of Section 2.1 evaluate exponentials, logarithms, powers,
 * x^(-1/3), reciprocals and x^(-1/2) in FP64 with the library's own
 * functions (range reduction plus economized polynomials, or a hardware
 * estimate plus Newton or series steps).  reaxff_math_eval applies function
 * fn to n arguments x [dev] (and exponents y [dev] for REAXFF_MATH_POW,
 * x^y; y may be NULL otherwise), writing out [dev] (n), asynchronously on
 * `stream`; it needs no context.  Domains: EXP, LOG, POW any finite x > 0
 * (POW also x = 0) with results in the normal range; EXP_R |x| < 700; LOG_R
 * positive normal x; EXP_C any x (clamped to [-1000, 1000], NaN passes);
 * RCBRT, RSQRT finite x > 0; RCP finite nonzero x.  Returns REAXFF_OK, or
 * REAXFF_ERR_ARG for an unknown fn, n < 0 or a null array, REAXFF_ERR_HIP
 * for a failed launch. */
enum {
  REAXFF_MATH_EXP = 0,    /* exp, Cody-Waite reduction and a degree-11 polynomial */
  REAXFF_MATH_EXP_R = 1,  /* the same exp with the integer steps done on the bits */
  REAXFF_MATH_EXP_C = 2,  /* exp of the argument clamped to [-1000, 1000] */
  REAXFF_MATH_LOG = 3,    /* log, 2 atanh((m - 1)/(m + 1)) */
  REAXFF_MATH_LOG_R = 4,  /* the same log with the exponent and mantissa read from the bits */
  REAXFF_MATH_POW = 5,    /* x^y = exp(y log x) */
  REAXFF_MATH_RCBRT = 6,  /* x^(-1/3) */
  REAXFF_MATH_RCP = 7,    /* 1/x */
  REAXFF_MATH_RSQRT = 8   /* x^(-1/2) */
};
int reaxff_math_eval(int32_t fn, int64_t n, const double* x, const double* y, double* out,
                     hipStream_t stream);

/* ---- Charge equilibration (Section 3.3, QEq) ------------------------------
 *
 * The charges that minimise the electrostatic energy
 *   E(q) = sum_i (chi_i q_i + J_i q_i^2 / 2) + sum_{i<j} H_ij q_i q_j
 * subject to sum_i q_i = 0, where H_ij is the force field's tapered shielded
 * Coulomb coupling Tap(r) C_ele / (r^3 + gamma_ij^-3)^(1/3) over the pairs
 * within r_nonb (minimum image in a periodic box) and H_ii = J_i.  As the
 * paper describes, the minimum follows from two linear systems with the
 * common matrix H, H s = -chi and H t = -1, as q = s - (sum s / sum t) t; H
 * is computed once per call from the neighbours and stored, and both
 * systems are solved together by diagonally preconditioned conjugate
 * gradients (one product of H with both search directions per iteration),
 * from a start extrapolated from earlier calls.  The paper's benchmarks stop
 * at a relative residual of 1e-6 (Section 4). */
typedef struct reaxff_qeq_params {
  double chi[REAXFF_NTYPES];  /* electronegativity per element, kcal/(mol e) */
  double J[REAXFF_NTYPES];    /* self-Coulomb (twice the hardness) per element,
                                 kcal/(mol e^2); must be > 0, and H positive
                                 definite for the iteration to converge */
} reaxff_qeq_params;
#define REAXFF_QEQ_MAXIT 10000

/* Charges for the atoms of the last reaxff_build_lists call (same n; its
 * positions, types and box).  qp [host].  Stops when both relative residuals
 * |b - H x| / |b| are at most tol (> 0), or after maxit (0..REAXFF_QEQ_MAXIT)
 * iterations, then returns REAXFF_ERR_CONVERGENCE with the charges of the
 * last iterate.  guess != 0: start from the polynomial extrapolation through
 * the solutions of up to four earlier calls for the same n (cubic with four:
 * 4x1 - 6x2 + 4x3 - x4, newest first), else from zero (and forget them).
 * q [dev] (n) the charges, s_out/t_out [dev] (n) or NULL the two solutions,
 * all in the caller's order; iters [host] or NULL the iterations taken;
 * resid [host] (2) or NULL the final relative residuals.  The product with
 * H is chosen by reaxff_set_qeq_product.  The context owns the solver vectors
 * and, for stored rows, H (n x row width entries of 12 bytes).  One host
 * synchronisation per iteration (the residual norms). */
int reaxff_qeq(reaxff_ctx* ctx, int64_t n, const reaxff_qeq_params* qp, double tol,
               int32_t maxit, int32_t guess, double* q, double* s_out, double* t_out,
               int32_t* iters, double* resid, hipStream_t stream);

/* How reaxff_qeq multiplies by H [host].  REAXFF_QEQ_STORED: the paper's way
 * (Section 3.3): the matrix elements within r_nonb are computed once per call
 * into rows (both halves of the symmetric matrix, so a product only gathers)
 * and each CG iteration reads them.  REAXFF_QEQ_AUTO (the default): when the
 * last build left the far list in its half form (each pair once; grids of at
 * least 2 reach + 1 cells per edge, the nonbonded term's half evaluation), no
 * matrix is stored: each product evaluates H_ij of every far pair within
 * r_nonb once and adds it to both atoms; otherwise the stored rows.  The
 * matrix-free product skips the row build (about three products' time) and
 * the rows' memory for ~15% more time per product, so it is the faster choice
 * below ~20 iterations, as with an extrapolated start along a trajectory.
 * Charges agree to the order of floating-point additions.  Returns REAXFF_OK,
 * or REAXFF_ERR_ARG for a null context or another mode. */
#define REAXFF_QEQ_AUTO 0
#define REAXFF_QEQ_STORED 1
int reaxff_set_qeq_product(reaxff_ctx* ctx, int32_t mode);

/* ---- Exact forces on a subset of the atoms ---------------------------------
 *
 * The force on an atom collects the terms whose inputs include its position
 * (Section 2.1's terms): pair terms reach r_nonb; a bonded term reads
 * positions up to three bond hops from its centre (corrected bond orders read
 * the orders of their atoms' bonds; over/under-coordination and coalition
 * read neighbours' total orders), so it moves atoms within three hops and
 * reads atoms within six hops of them; a hydrogen bond reads its donor
 * bond's order (two hops from H) and acceptors within r_hb of H.  Every input
 * of every term that moves atom f thus lies within
 *   R = max(r_nonb, 6 b, r_hb + 2 b)
 * of f, b being the largest distance at which an uncorrected bond order
 * reaches bo_cut (reaxff_dependency_radius returns R).  reaxff_forces_masked
 * evaluates the atoms within R of the atoms with mask [dev] (n) != 0 (a
 * superset from a grid of cells at least R/3 wide) as one system in the same
 * box and writes their exact forces into forces [dev] (n,3) at the masked
 * atoms only; other rows are left as they were.  *nsub [host] (may be NULL)
 * the atoms evaluated.  The context's lists are those of the subsystem
 * afterwards.  Synchronises two to three times. */
double reaxff_dependency_radius(const reaxff_ctx* ctx);
int reaxff_forces_masked(reaxff_ctx* ctx, int64_t n, const double* pos, const int32_t* type,
                         const double* q, const double* box, const uint8_t* mask, double* forces,
                         int64_t* nsub, hipStream_t stream);

/* ---- In-situ molecular species analysis (Section 3.4) ---------------------
 *
 * Over the corrected bond orders of the last reaxff_compute_forces: two atoms
 * are bonded when their bond order is larger than bo_threshold (the paper's
 * default is 0.3); bonded atoms share a molecule whose ID is the smallest
 * caller index among its atoms; the IDs are renumbered 1..M in increasing
 * order; a species is a molecule's count of atoms per element, molecules
 * with equal counts being the same species (isomers are not told apart).
 * mol [dev] (n) int32: each atom's molecule number 1..M (caller order).
 * mol_counts [dev] (n, 4) int32 or NULL: rows 0..M-1 hold molecule m+1's C,
 * H, N, O counts.  table [dev] (n, 5) int32 or NULL: rows 0..S-1 hold each
 * species' C, H, N, O counts and its number of molecules, in increasing
 * lexicographic order of the counts.  *nmol = M, *nspecies = S [host].
 * REAXFF_ERR_STATE before any force evaluation on the current lists.
 * Synchronises the device twice. */
int reaxff_species(reaxff_ctx* ctx, double bo_threshold, int32_t* mol, int32_t* mol_counts,
                   int32_t* table, int64_t* nmol, int64_t* nspecies, hipStream_t stream);

/* ---- Batched evaluation of many small non-periodic systems ---------------
 *
 * Force-field fitting and cluster screening evaluate thousands of small,
 * independent, unevenly sized systems: the small-system regime that the
 * paper's closing discussion leaves to a serial code.  A batch plan fixes the
 * cluster sizes; each compute call then evaluates every cluster in ONE
 * persistent kernel launch replayed from a HIP graph.  Every workgroup takes
 * whole clusters, one at a time, and runs the complete force evaluation of a
 * cluster (bond list, bond orders, every energy term of reaxff_compute_forces,
 * forces) with the cluster's atoms and nonbonded/H-bond forces in LDS and its
 * bond-entry arrays in a private slice of device scratch.  Clusters are
 * non-periodic; the far-neighbour and H-bond relations are tested in place
 * (all pairs within the cluster, same predicates as the lists of
 * reaxff_build_lists) instead of being stored.
 */
#define REAXFF_BATCH_MAX_ATOMS 384   /* atoms per cluster (LDS-resident) */

enum {
  REAXFF_SCHED_STATIC = 0,   /* clusters dealt round-robin in the given order */
  REAXFF_SCHED_LPT = 1,      /* longest-processing-time-first greedy assignment
                                (cost model: n^2 per cluster) */
  REAXFF_SCHED_DYNAMIC = 2   /* atomic work queue over clusters sorted by
                                decreasing size */
};

typedef struct reaxff_batch_config {
  int32_t block;      /* threads per workgroup: 64, 128, 256 or 512 */
  int32_t schedule;   /* REAXFF_SCHED_* */
  int32_t wg_per_cu;  /* persistent workgroups per compute unit, 1..16 */
} reaxff_batch_config;

typedef struct reaxff_batch reaxff_batch;

/* Plan a batch of `nclusters` clusters; cluster c holds atoms
 * offsets[c] .. offsets[c+1]-1 of the concatenated arrays.  offsets [host]
 * (nclusters+1), offsets[0] = 0, non-decreasing, every cluster at most
 * REAXFF_BATCH_MAX_ATOMS atoms (else REAXFF_ERR_ARG).  cfg NULL: the
 * configuration autotuned earlier in this context for the same multiset of
 * cluster sizes, else {256, LPT, 4}.  The plan allocates its device scratch
 * here (one slice per persistent workgroup) and uses the context's
 * parameters and cutoffs.  The context must outlive the plan. */
int reaxff_batch_create(reaxff_ctx* ctx, int32_t nclusters, const int64_t* offsets,
                        const reaxff_batch_config* cfg, reaxff_batch** out);
void reaxff_batch_destroy(reaxff_batch* b);
int reaxff_batch_set_config(reaxff_batch* b, const reaxff_batch_config* cfg);
int reaxff_batch_get_config(const reaxff_batch* b, reaxff_batch_config* cfg);

/* Evaluate every cluster: pos [dev] (N,3), type [dev] (N), q [dev] (N) over
 * the N = offsets[nclusters] concatenated atoms; forces [dev] (N,3) and
 * energies [dev] (nclusters, REAXFF_NTERMS) are overwritten.  One graph
 * launch on `stream`, no host synchronisation; the graph is captured again
 * only when a pointer or the configuration changes.  A cluster that fails
 * (type outside 0..3, more bond entries than its scratch slice holds) gets
 * NaN energies and forces; reaxff_batch_status reports it. */
int reaxff_batch_compute(reaxff_batch* b, const double* pos, const int32_t* type,
                         const double* q, double* forces, double* energies,
                         hipStream_t stream);

/* Wait for the last compute and report: REAXFF_OK, REAXFF_ERR_ARG (a bad
 * type) or REAXFF_ERR_CAPACITY (bond entries beyond the scratch slice; the
 * next compute grows the slices to fit and recaptures).  *first_bad (may be
 * NULL) receives the lowest failing cluster index or -1. */
int reaxff_batch_status(reaxff_batch* b, int32_t* first_bad);

/* Per-cluster interaction counts of the last compute [host]
 * (nclusters, 5): valence angles, torsions, hydrogen bonds, far pairs
 * (unordered, r <= r_nonb), bonds (undirected).  Synchronises. */
int reaxff_batch_counts(reaxff_batch* b, int64_t* counts);

/* Autotuner: times every configuration of block {64,128,256,512} x
 * schedule {STATIC, LPT, DYNAMIC} x wg_per_cu {1,2,4,8} (at most max_trials
 * of them, in that order; max_trials <= 0: all 48) by `reps` graph replays
 * each on `stream` (events around the replays, one untimed replay first),
 * selects the fastest, makes it the plan's configuration and caches it in
 * the context for reaxff_batch_create.  trials/trial_ms [host] (may be
 * NULL) receive each configuration and its mean milliseconds per launch;
 * *ntrials their number.  The buffers' contents after tuning are those of
 * the last replay. */
int reaxff_batch_tune(reaxff_batch* b, const double* pos, const int32_t* type,
                      const double* q, double* forces, double* energies,
                      hipStream_t stream, int32_t reps, int32_t max_trials,
                      reaxff_batch_config* trials, double* trial_ms, int32_t* ntrials);

/* ---- Batched evaluation that allocates nothing -----------------------------
 *
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * per-cluster evaluation as reaxff_batch_compute (one persistent launch,
 * every cluster in one workgroup), without a plan: cluster offsets stay on
 * the device, clusters are taken from a work queue in index order, and all
 * scratch (queue, status words, one slice per persistent workgroup) lives in
 * one fixed device array of REAXFF_BATCHED_SCRATCH_BYTES that each GPU the
 * library runs on holds until the process ends.  The call allocates nothing,
 * synchronises nothing and may be captured into a graph.
 *
 * nsys clusters; sys_off [dev] (nsys+1) int64 atom offsets (sys_off[0] = 0,
 * non-decreasing); max_atoms [host] an upper bound on the atoms of any
 * cluster, 1..REAXFF_BATCH_MAX_ATOMS (else REAXFF_ERR_ARG; it sizes the
 * workgroup slices, and the number of workgroups is what fits in the array).
 * pos [dev] (N,3), type [dev] (N), q [dev] (N) over N = sys_off[nsys] atoms;
 * forces [dev] (N,3) and energies [dev] (nsys, REAXFF_NTERMS) overwritten.
 * status [dev] (3) int32 or NULL: [0] the OR of the failures (1: bond entries
 * beyond REAXFF_BATCHED_ENTRIES_PER_ATOM * max_atoms, 2: a type outside 0..3,
 * 4: a cluster longer than max_atoms or offsets out of order), [1] the largest
 * entry count of a failing cluster, [2] the lowest failing cluster (INT32_MAX
 * if none); a failing cluster gets NaN energies (and NaN forces when its
 * atom range is valid).  Calls that overlap on one GPU share the array and
 * race: serialise them (one stream, or events). */
#define REAXFF_BATCHED_SCRATCH_BYTES (256ll << 20)
#define REAXFF_BATCHED_ENTRIES_PER_ATOM 6
int reaxff_compute_forces_batched(reaxff_ctx* ctx, int32_t nsys, const int64_t* sys_off,
                                  int32_t max_atoms, const double* pos, const int32_t* type,
                                  const double* q, double* forces, double* energies,
                                  int32_t* status, hipStream_t stream);

/* ---- Learned surrogate with the plain evaluation as fallback -------------
 *
 * An ensemble of per-element neural networks predicts per-atom energies
 * from atom-centred descriptors of the neighbours within 5 A (Behler-
 * Parrinello radial functions: 16 per neighbour element; angular power
 * spectrum: 16 per unordered neighbour-element pair; 224 features), and
 * forces as the exact negative gradient of that energy.  Each network maps
 * x = (G - shift) * scale through 224 -> 128 -> 128 -> 1 with SiLU
 * activations; products run on BF16 matrix cores with FP32 accumulation.
 * Parameters are FP32, per member and element network, flattened as
 * W1[224][128], b1[128], W2[128][128], b2[128], w3[128], b3
 * (reaxff_surrogate_param_count() floats per network; networks ordered
 * [member][element]).  The plain FP64 force evaluation of this library is
 * the fallback wherever the members disagree (reaxff_surrogate_gated_forces).
 * Energies in kcal/mol, forces in kcal/(mol A), as elsewhere.
 */
typedef struct reaxff_surrogate reaxff_surrogate;

/* Floats per element network. */
int64_t reaxff_surrogate_param_count(void);

/* An ensemble of `members` (1..16) on the device of ctx; the neighbour lists
 * come from an internal context with ctx's parameters and a 5 A cutoff.
 * Parameters start at zero, shift at 0 and scale at 1. */
int reaxff_surrogate_create(reaxff_ctx* ctx, int32_t members, reaxff_surrogate** out);
void reaxff_surrogate_destroy(reaxff_surrogate* s);
const char* reaxff_surrogate_last_error(const reaxff_surrogate* s);

/* [host] theta (members*4*param_count), shift and scale (224 each); any may be
 * NULL to leave it unchanged.  Setting theta resets the Adam state. */
int reaxff_surrogate_set_params(reaxff_surrogate* s, const float* theta, const float* shift,
                                const float* scale);
int reaxff_surrogate_get_params(reaxff_surrogate* s, float* theta, float* shift, float* scale);

/* Descriptors G [dev] (n, 224) FP32, caller order.  pos/type/box as in
 * reaxff_build_lists.  Synchronises once (list sizes). */
int reaxff_surrogate_descriptors(reaxff_surrogate* s, int64_t n, const double* pos,
                                 const int32_t* type, const double* box, float* G,
                                 hipStream_t stream);

/* Every member on one configuration: energies [dev] (members) FP64 totals;
 * optional [dev] outputs (NULL to skip): eatom (members, n) per-atom energies,
 * forces (members, n, 3), fmean (n, 3) FP64 ensemble mean force, sigma (n)
 * ensemble spread sqrt(mean_m |F_i^m - Fbar_i|^2).  Caller order. */
int reaxff_surrogate_evaluate(reaxff_surrogate* s, int64_t n, const double* pos,
                              const int32_t* type, const double* box, double* energies,
                              float* eatom, float* forces, double* fmean, float* sigma,
                              hipStream_t stream);

/* One training step of every member on one reference frame (eref total
 * energy, fref [dev] (n, 3) forces, caller order): loss [dev] (members)
 * = wE ((E - eref)/n)^2 + wF/(3n) sum_i |F_i - fref_i|^2 before the step,
 * its parameter gradient by forward-over-reverse differentiation, then one
 * Adam step of size lr (none if lr <= 0; the gradient stays readable). */
int reaxff_surrogate_train_step(reaxff_surrogate* s, int64_t n, const double* pos,
                                const int32_t* type, const double* box, double eref,
                                const double* fref, double wE, double wF, double lr,
                                double* loss, hipStream_t stream);
/* Input normalisation of the networks: over `rows` descriptor rows G [dev]
 * (rows, 224) FP32 (e.g. the descriptors of several frames, concatenated),
 * shift [host] (224) = the mean of each feature and scale [host] (224) =
 * 1 / max(standard deviation, std_floor) (population deviation, FP64 sums).
 * Synchronises once. */
int reaxff_surrogate_normaliser(reaxff_surrogate* s, int64_t rows, const float* G, double std_floor,
                                float* shift, float* scale, hipStream_t stream);

/* The surrogate's own context (its 5 A neighbour lists), for reaxff_profile
 * and reaxff_profile_read over the surrogate's kernels; owned by s. */
reaxff_ctx* reaxff_surrogate_context(reaxff_surrogate* s);

/* [host] (members*4*param_count) gradient of the last train_step. */
int reaxff_surrogate_get_grad(reaxff_surrogate* s, float* grad);

/* Gated forces: the ensemble mean force, except on atoms whose spread
 * exceeds `threshold` (kcal/(mol A)), which take the exact plain FP64 ReaxFF
 * force computed by `plain` (a context of this library, charges q [dev])
 * through reaxff_forces_masked, so the fallback costs what the flagged atoms'
 * neighbourhoods cost.  forces [dev] (n,3) FP64, mask [dev] (n) 1 = fallback,
 * energies [dev] (members) surrogate totals, *nflagged [host] number of
 * flagged atoms, *nsub [host] (may be NULL) atoms of the plain evaluation
 * (0 when none is flagged).  Synchronises two to three times. */
int reaxff_surrogate_gated_forces(reaxff_surrogate* s, reaxff_ctx* plain, int64_t n,
                                  const double* pos, const int32_t* type, const double* q,
                                  const double* box, double threshold, double* forces,
                                  uint8_t* mask, double* energies, int64_t* nflagged,
                                  int64_t* nsub, hipStream_t stream);

const char* reaxff_strerror(int code);
const char* reaxff_last_error(const reaxff_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* REAXFF_H */
