/*
 * tk.h -- C-ABI of the MI355X real-space AMOEBA pair engine (libtk.so).
 *
 * What it computes (arXiv 1906.01211, section "Hotspots", Table of the Rel
 * profile): the routines that dominate a polarizable AMOEBA step on the
 * paper's CPUs -- the cell-list neighbour builders, the permanent-multipole
 * real-space energy and forces, the permanent field (the right-hand side of
 * the polarization equations), the induced-dipole field mat-vec used at every
 * iteration of the polarization solver, the Halgren buffered 14-7 vdW term,
 * and, for the non-polarizable path, point charges and Lennard-Jones 12-6.
 * The paper names these terms (section "Polarizable AMOEBA force field") but
 * does not write their formulas; the definitions implemented are the textbook
 * Ewald real-space / Thole / Halgren ones and are stated at each entry point.
 *
 * Conventions shared by every call:
 *  - Units: Angstrom, elementary charge e, e*A (dipoles), e*A^2 (quadrupoles),
 *    A^3 (polarizabilities), kcal/mol, kcal/mol/A.  Dipole tolerances in Debye
 *    (1 e*A = 4.80320 D).  Coulomb constant C = 332.0637 kcal*A/(mol*e^2).
 *  - Periodic cubic box of edge `box`; pair vectors use the minimum image;
 *    every cutoff must satisfy cutoff <= box/2 (else TK_E_CUTOFF).
 *  - Pair vector r = r_j - r_i; forces are F = -dE/dx, written (not
 *    accumulated) as [n][3]; virials W_ab = sum over pairs r_a dE/dr_b, [3][3].
 *  - Array arguments are DEVICE pointers owned by the caller (unless a
 *    parameter says "host"); nothing is retained after the call returns.
 *    `stream` is a hipStream_t (NULL = default stream).  Calls are ordered on
 *    that stream.  Entry points that return results through host memory
 *    (tk_nblist_build, tk_polarize_pcg, tk_batch_step) synchronise the
 *    stream to produce them; device outputs are always written in stream
 *    order.  The stream-ordered forms (tk_nblist_build_async,
 *    tk_polarize_pcg_queued, tk_empole_polarize_queued) return their sizes,
 *    statuses and outcomes in device memory and never wait for the device
 *    (except to grow a buffer, once).
 *  - Errors: every call returns a tk_status; argument errors are detected on
 *    the host before any work is queued; no exception crosses the ABI.
 *  - Precision: prec = TK_FP64 (all pair arithmetic in FP64) or TK_MIXED (pair
 *    geometry, screening, damping and contractions in FP32; energies, virial,
 *    forces, fields and all solver reductions accumulated in FP64).
 *  - A tk_ctx owns scratch device memory (grown on demand, never shrunk, never
 *    freed between calls) and up to TK_MAX_PLANS neighbour-list plans.  A
 *    context is not thread safe; use one per host thread.  Work of one context
 *    queued on different streams may run concurrently where it touches
 *    different memory: the pair terms keep their scratch per stream and the
 *    builds of one tk_nblist_build_multi call have their own; the solver
 *    (tk_polarize_pcg and its other forms) has one scratch set per context,
 *    so two solves of a context must be ordered, and a plan slot must not be rebuilt while work
 *    that reads it is still queued on another stream.
 */
#ifndef TK_H
#define TK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tk_ctx tk_ctx;
typedef int32_t tk_status;

enum {
  TK_OK = 0,
  TK_E_ARG = -1,       /* invalid argument (null pointer, n < 0, NaN, bad enum) */
  TK_E_CUTOFF = -2,    /* cutoff > box/2 */
  TK_E_CAPACITY = -3,  /* output capacity too small; the required size is reported */
  TK_E_NOCONV = -4,    /* PCG did not reach the tolerance within maxiter */
  TK_E_BREAKDOWN = -5, /* PCG found p.Ap <= 0 (operator not positive definite) */
  TK_E_NOMEM = -6,     /* device allocation failed */
  TK_E_HIP = -7,       /* a HIP runtime call failed */
  TK_E_BUSY = -8,      /* serving: result not ready yet */
  TK_E_PLAN = -9,      /* the list's plan slot is empty or was built for another system */
  TK_E_TOOBIG = -10    /* allocation-free call: the system needs more than its fixed scratch */
};

enum { TK_FP64 = 0, TK_MIXED = 1 };
enum { TK_VDW_HAL = 0, TK_VDW_LJ = 1 };
#define TK_MAX_PLANS 8

/* Atoms of one periodic system.  xyz: device [n][3] (A, any real values:
 * they are wrapped), molid: device [n] molecule id (pairs with equal molid are
 * "excluded": see each entry point). */
typedef struct {
  int32_t n;
  const double* xyz;
  double box;
  const int32_t* molid;
} tk_system;

/* A neighbour list as returned by tk_nblist_build.
 * row_ptr: device [n+1]; col: device [npairs]; row i holds every j > i with
 * |r_ij| <= cutoff (integer test below), ascending.  `plan` names the context
 * slot that holds the same pair set in the cell-pair order the kernels use.
 * A list from tk_nblist_build_async has npairs = -1 (its count is on the
 * device). */
typedef struct {
  const int32_t* row_ptr;
  const int32_t* col;
  int64_t npairs;
  double cutoff;
  int32_t plan;
} tk_nblist;

/* Outcome of a polarization solve (host memory). */
typedef struct {
  int32_t status;      /* TK_OK, TK_E_NOCONV, TK_E_BREAKDOWN, or TK_E_CAPACITY (the
                          list's stream-ordered build failed: nothing solved) */
  int32_t iters;       /* PCG updates performed (mat-vecs after the initial residual) */
  int32_t refinements; /* FP64 refinement rounds (TK_MIXED only) */
  int32_t converged;   /* 1 if the stopping rule was met (TK_MIXED: the FP64 check) */
  double rms_debye;      /* RMS preconditioned residual at exit (solver recurrence) */
  double rms_true_debye; /* same, from a fresh FP64 residual b - A mu */
  double epol;           /* -1/2 C sum_i mu_i . E_perm_i, kcal/mol */
} tk_pcg_info;

/* Context on HIP device `device`. */
tk_status tk_create(int device, tk_ctx** out);
void tk_destroy(tk_ctx* ctx);
const char* tk_strerror(tk_status s);

/*
 * Neighbour list (the cell-list builders of the Rel profile; neighbour
 * selection by cutoff, section "General Structure"; the selection mask and
 * compress loop, section "Typical selection loop").
 * Exact integer definition: u = floor(frac(x/box) * 2^32) per coordinate
 * (x/box rounded as an IEEE division; a fraction that rounds to 1 wraps to 0),
 * d = (int32)(u_j - u_i), and (i, j) is listed iff dx^2+dy^2+dz^2 <= rq^2 in
 * exact 64-bit arithmetic with rq = floor((cutoff/box) * 2^32).  The list is
 * purely geometric (same-molecule pairs are included).
 * Writes the canonical half list (row_ptr [n+1], col [cap]) and fills plan
 * slot `plan_slot` of the context.  *npairs (host) receives the number of
 * pairs; if it exceeds `cap`, returns TK_E_CAPACITY, col is not written and
 * the plan is left empty.  row_ptr/col may be NULL (with cap = 0) to build the
 * plan only.  Synchronises `stream`.  Errors: TK_E_ARG (n < 0, NULL xyz,
 * non-finite coordinate, plan_slot out of range), TK_E_CUTOFF.
 */
tk_status tk_nblist_build(tk_ctx* ctx, void* stream, const tk_system* sys, double cutoff,
                          int32_t plan_slot, int32_t* row_ptr, int32_t* col, int64_t cap,
                          int64_t* npairs);

/* Sizes a neighbour-list build depends on, as bounds for
 * tk_nblist_build_async (and as the sizes a build measured). */
typedef struct {
  int32_t max_occ;  /* atoms in the fullest cell */
  int32_t max_row;  /* longest row of the half list */
  int32_t max_nbhd; /* atoms in the fullest cell with its neighbour cells */
  int32_t reserved; /* 0 */
  int64_t windows;  /* candidate pairs: sum over cell pairs of |H| |K| */
  int64_t npairs;   /* listed pairs */
} tk_nblist_bounds;

/*
 * Bounds for later builds of plan slot `plan_slot`, from the sizes its last
 * synchronous build (tk_nblist_build, tk_nblist_build_multi) measured: each
 * scaled by 1 + headroom and rounded up (max_occ at most 512, the largest
 * cell a build accepts).  Host call, no GPU work.  Errors: TK_E_ARG (NULL ctx or out,
 * slot out of range, headroom < 0 or not finite), TK_E_PLAN (the slot holds
 * no list from a synchronous build).
 */
tk_status tk_nblist_bounds_get(tk_ctx* ctx, int32_t plan_slot, double headroom,
                               tk_nblist_bounds* out);

/*
 * The list of tk_nblist_build, queued on `stream` with no host
 * synchronisation (the stream-ordered form of the list boundary: the list
 * builders of the Rel profile, section "Hotspots").  Every buffer is sized
 * from `bounds` (host memory; windows and max_occ size the enumeration,
 * max_occ, max_row and max_nbhd the LDS of the kernels that use the list)
 * and from `cap` (entries of col, and of the plan's pair array).
 * Device outputs, written in stream order before the list's first user runs:
 *   *npairs_dev (int64) the listed pairs; *status_dev (int32) TK_OK, or
 *   TK_E_CAPACITY when a measured size exceeds its bound or npairs > cap
 *   (then col and the plan hold no list: every kernel that uses the plan
 *   skips its work, and a solve on it returns TK_E_CAPACITY), or the error
 *   a synchronous build would return (TK_E_CAPACITY for a cell above 512
 *   atoms);
 *   report_dev (nullable, device tk_nblist_bounds): the sizes measured
 *   (windows, max_occ and max_nbhd always; npairs and max_row only when the
 *   enumeration fitted, else -1), for the caller's next bounds.
 * row_ptr/col may be NULL (with cap >= 0 still bounding the plan's pairs).
 * A later call taking this list (tk_nblist with npairs = -1 and this
 * plan_slot) reads its status on the device.  Host-side argument errors as
 * tk_nblist_build (bounds: TK_E_ARG if windows, max_occ, max_row or max_nbhd
 * is < 1 or npairs < 0; max_occ above 512 acts as 512; TK_E_CAPACITY if
 * max_row is above 1024 and the row sort's LDS for it exceeds the GPU's).  One system; the first build of a new cell grid also
 * uploads that grid's cell tables (a synchronous copy, once per grid), and
 * a buffer that must grow is reallocated after a device synchronisation.
 * Builds of different plan slots may run concurrently on different streams;
 * builds of one slot, and the calls that use it, must be ordered by the
 * caller.
 */
tk_status tk_nblist_build_async(tk_ctx* ctx, void* stream, const tk_system* sys, double cutoff,
                                int32_t plan_slot, const tk_nblist_bounds* bounds,
                                int32_t* row_ptr, int32_t* col, int64_t cap,
                                int64_t* npairs_dev, int32_t* status_dev,
                                tk_nblist_bounds* report_dev);

/*
 * Several neighbour lists of the same atoms (e.g. the Ewald and the vdW list
 * of a step, section "Hotspots": both list builders are on the profile),
 * 1 <= nlists <= 4.  List k is exactly what tk_nblist_build(ctx, streams[k],
 * sys, cutoffs[k], plan_slots[k], row_ptrs[k], cols[k], caps[k], &npairs[k])
 * gives; the builds share one host synchronisation per distinct stream, and
 * builds on different streams run concurrently.  All arrays are host arrays of
 * nlists entries; streams may be NULL (all lists on the default stream) and
 * entries may repeat; row_ptrs/cols/caps may be NULL (plans only) or hold NULL
 * entries.  The plan slots must be distinct.  On return each list's results
 * (CSR and plan) are queued on its stream: work that uses list k on another
 * stream must wait for streams[k].  Errors as tk_nblist_build; on an error the
 * lists after the failing one are left empty.
 */
tk_status tk_nblist_build_multi(tk_ctx* ctx, int32_t nlists, void* const* streams,
                                const tk_system* sys, const double* cutoffs,
                                const int32_t* plan_slots, int32_t* const* row_ptrs,
                                int32_t* const* cols, const int64_t* caps, int64_t* npairs);

/*
 * Real-space Ewald permanent-multipole energy, forces and virial (the
 * multipolar permanent electrostatic routine of section "Hotspots").
 * mpole: device [n][10] = q, mu_x, mu_y, mu_z, Theta_xx, Theta_xy, Theta_xz,
 * Theta_yy, Theta_yz, Theta_zz with Theta traceless and the site potential
 * [q - mu.grad + Theta:grad grad] 1/r.  For each listed pair with r <= cutoff
 * the energy is C sum_n c_n g_n (n = 0..4; c_n the usual charge/dipole/
 * quadrupole invariants), g_n = B_n (Ewald-screened radial functions,
 * B_0 = erfc(beta r)/r) for pairs of different molecules and g_n = B_n - R_n
 * (removal of the screened part, R_n bare) within a molecule.  No
 * self or reciprocal-space term.  energy: device [3] = total, sum over
 * non-excluded pairs, sum of intramolecular corrections.  force: [n][3];
 * virial: [3][3].  A charge-only input (mu = Theta = 0) is accepted; see also
 * tk_echarge_real.
 */
tk_status tk_empole_real(tk_ctx* ctx, void* stream, const tk_system* sys, const tk_nblist* list,
                         const double* mpole, double ewald_beta, double cutoff, int prec,
                         double* energy, double* force, double* virial);

/*
 * Point-charge Ewald real space (the charge-charge routine of the CHARMM
 * profile): e = C q_i q_j g_0 with the same molecule rule as tk_empole_real.
 * q: device [n].  energy: device [3] as above.
 */
tk_status tk_echarge_real(tk_ctx* ctx, void* stream, const tk_system* sys, const tk_nblist* list,
                          const double* q, double ewald_beta, double cutoff, int prec,
                          double* energy, double* force, double* virial);

/*
 * Permanent field at every site (the right-hand side of the polarization
 * equations; efld0_direct in the Rel profile).  For each listed pair with
 * r <= cutoff: E_i += q_j T1 + T2 mu_j + T3:Theta_j and
 * E_j += -q_i T1 + T2 mu_i - T3:Theta_i, with T1 = -r g1, T2 = r r g2 - I g1,
 * (T3:Theta)_a = -r_a (r.Theta.r) g3 + 2 (Theta r)_a g2,
 * g_n = B_n - (1 - s l_(2n+1)) R_n, s = 0 within a molecule else 1, and the
 * Thole factors l3 = 1 - e^-x, l5 = 1 - (1+x) e^-x, l7 = 1 - (1+x+0.6x^2) e^-x,
 * x = min(a_i, a_j) r^3 / sqrt(alpha_i alpha_j) (l = 1 when alpha_i alpha_j = 0);
 * plus the Ewald self field c mu_i, c = 4 beta^3 / (3 sqrt(pi)).
 * polarity: device [n] (A^3, >= 0); thole: device [n]; field: device [n][3]
 * in e/A^2 (no Coulomb constant).
 */
tk_status tk_efield_direct(tk_ctx* ctx, void* stream, const tk_system* sys, const tk_nblist* list,
                           const double* mpole, const double* polarity, const double* thole,
                           double ewald_beta, double cutoff, int prec, double* field);

/*
 * Induced-dipole field mat-vec (tmatxb in the Rel profile, the largest
 * hotspot).  For every listed pair with r <= cutoff (same molecule included):
 * out_i += T2 mu_j, out_j += T2 mu_i with g1 = B1 - (1 - l3) R1,
 * g2 = B2 - (1 - l5) R2, plus the self field c mu_i.  include_diag = 0 returns
 * this field (T + cI) mu; include_diag = 1 returns A mu = mu_i/alpha_i - field_i
 * (rows of atoms with alpha = 0 are zero).  mu, out: device [n][3].
 */
tk_status tk_tmatvec(tk_ctx* ctx, void* stream, const tk_system* sys, const tk_nblist* list,
                     const double* polarity, const double* thole, double ewald_beta,
                     double cutoff, int include_diag, int prec, const double* mu, double* out);

/*
 * tk_tmatvec for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).  Same
 * arguments, result and errors as tk_tmatvec (bitwise the same result), but no
 * device allocation at all: its scratch is one fixed 32 MiB array in the
 * library, one copy per device, held until the process ends.  The list's plan
 * must already exist (tk_nblist_build allocates; this call does not).  Limit:
 * n <= tk_tmatvec_noalloc_max_atoms() (46,592 atoms), else TK_E_TOOBIG with
 * nothing launched.  Every call on a device shares that device's array, so
 * calls that overlap on one device (other streams, other contexts) race and
 * must be ordered by the caller.
 */
tk_status tk_tmatvec_noalloc(tk_ctx* ctx, void* stream, const tk_system* sys,
                             const tk_nblist* list, const double* polarity, const double* thole,
                             double ewald_beta, double cutoff, int include_diag, int prec,
                             const double* mu, double* out);
/* The largest atom count tk_tmatvec_noalloc accepts. */
int32_t tk_tmatvec_noalloc_max_atoms(void);

/*
 * Induced dipoles: solve A mu = E_perm (A as in tk_tmatvec, E_perm as in
 * tk_efield_direct) by preconditioned conjugate gradient, the polarization
 * solver that calls the mat-vec up to 12 times per step (section
 * "Hotspots").  Preconditioner diag(alpha); initial guess mu_guess (device
 * [n][3], may be NULL: then alpha * E_perm).  Stopping rule, checked before
 * each mat-vec: 4.80320 * sqrt(sum |alpha_i r_i|^2 / n_pol) <= tol_debye.
 * After the loop a fresh FP64 residual is formed (info->rms_true_debye);
 * with TK_MIXED, up to 3 FP64-residual refinement rounds are added while it
 * exceeds the tolerance, and the outcome is that FP64 check: converged = 1
 * and TK_OK only if rms_true_debye <= tol_debye at the end, else TK_E_NOCONV
 * (also when the FP32 recurrence met its own test).  mu_out: device [n][3], written in stream order
 * (later work on `stream` sees it).  info: HOST memory, complete on return.
 * Returns info->status.  Synchronises `stream` while solving.
 */
tk_status tk_polarize_pcg(tk_ctx* ctx, void* stream, const tk_system* sys, const tk_nblist* list,
                          const double* mpole, const double* polarity, const double* thole,
                          double ewald_beta, double cutoff, double tol_debye, int32_t maxiter,
                          int prec, const double* mu_guess, double* mu_out, tk_pcg_info* info);

/*
 * tk_polarize_pcg with no host synchronisation: the same solve (operator,
 * preconditioner, guess, stopping rule, FP64 true residual) queued on
 * `stream` as `iterations` PCG steps, 1 <= iterations <= 10000, that stop
 * early on convergence (the steps queued after it return at once).  For
 * callers that keep the host off the critical path and know how many steps
 * their systems need (e.g. the previous solve's count, read later from
 * info_dev).  The outcome goes to info_dev, DEVICE memory (one tk_pcg_info),
 * written in stream order: status TK_OK with converged = 1 when the test was
 * met, TK_E_NOCONV when `iterations` ran out, TK_E_BREAKDOWN, or TK_E_CAPACITY
 * when the list came from a stream-ordered build that failed (nothing is
 * solved then and mu_out is not written).  With TK_MIXED there is no FP64
 * refinement: converged = 1 only if rms_true_debye <= tol_debye.  With
 * iterations >= the count tk_polarize_pcg takes, mu_out and every info field
 * equal its result bitwise (TK_MIXED: when it needed no refinement).  An
 * empty system writes converged = 1.  Returns TK_OK once queued, or an
 * argument/launch error with nothing written.  Shares the solver scratch of
 * tk_polarize_pcg: two solves of one context must be ordered.
 */
tk_status tk_polarize_pcg_queued(tk_ctx* ctx, void* stream, const tk_system* sys,
                                 const tk_nblist* list, const double* mpole,
                                 const double* polarity, const double* thole, double ewald_beta,
                                 double cutoff, double tol_debye, int32_t iterations, int prec,
                                 const double* mu_guess, double* mu_out, tk_pcg_info* info_dev);

/*
 * tk_empole_real and tk_polarize_pcg in one call: the permanent multipoles'
 * energy, forces and virial (as tk_empole_real, same cutoff and Ewald
 * parameter) and the induced dipoles (as tk_polarize_pcg).  The multipole
 * terms and the right-hand side E_perm come from one pass over the list,
 * since both walk the same pairs with the same screened radial functions
 * (empole1 and efld0_direct2 of section "Hotspots").  energy: device [3]
 * {total, non-excluded, exclusion correction}; force: device [n][3];
 * virial: device [9]; written in stream order.  Other arguments, outputs,
 * errors and synchronisation as tk_polarize_pcg; returns info->status.
 */
tk_status tk_empole_polarize(tk_ctx* ctx, void* stream, const tk_system* sys,
                             const tk_nblist* list, const double* mpole, const double* polarity,
                             const double* thole, double ewald_beta, double cutoff,
                             double tol_debye, int32_t maxiter, int prec, const double* mu_guess,
                             double* mu_out, tk_pcg_info* info, double* energy, double* force,
                             double* virial);

/*
 * tk_empole_polarize with the solve of tk_polarize_pcg_queued: the multipole
 * energy, forces and virial (as tk_empole_polarize) and the induced dipoles
 * from `iterations` queued PCG steps, with no host synchronisation; the
 * outcome in info_dev (device memory), with the rules of
 * tk_polarize_pcg_queued.  Every output is written in stream order.  With
 * iterations >= the count tk_empole_polarize takes, all outputs and info
 * fields equal its results bitwise (TK_MIXED: when it needed no refinement).
 * After a failed stream-ordered list build (TK_E_CAPACITY in info_dev) the
 * energy, forces and virial are not valid either.  Errors as
 * tk_polarize_pcg_queued, plus TK_E_ARG for NULL energy, force or virial.
 */
tk_status tk_empole_polarize_queued(tk_ctx* ctx, void* stream, const tk_system* sys,
                                    const tk_nblist* list, const double* mpole,
                                    const double* polarity, const double* thole,
                                    double ewald_beta, double cutoff, double tol_debye,
                                    int32_t iterations, int prec, const double* mu_guess,
                                    double* mu_out, tk_pcg_info* info_dev, double* energy,
                                    double* force, double* virial);

/*
 * Induced dipoles with the full Ewald operator: tk_polarize_pcg with the
 * reciprocal space included (the reciprocal polarization routine named in
 * section "Hotspots").  The operator is A = diag(1/alpha) - T - cI - R, R mu
 * the smooth-PME field of the dipoles themselves (as tk_pme_mpole's field with
 * mu as the only multipoles, each site's own contribution included), and the
 * right-hand side is E_perm = tk_efield_direct's field + the PME field of the
 * permanent multipoles.  Rows of atoms with alpha = 0 stay zero.  Same
 * stopping rule, guess, outputs and synchronisation as tk_polarize_pcg;
 * info->epol = -1/2 C mu.E_perm with the full field.  FP64 only; grid and
 * order as tk_pme_mpole; ewald_beta > 0.
 */
tk_status tk_polarize_pcg_ewald(tk_ctx* ctx, void* stream, const tk_system* sys,
                                const tk_nblist* list, const double* mpole,
                                const double* polarity, const double* thole, double ewald_beta,
                                double cutoff, int32_t grid, int32_t order, double tol_debye,
                                int32_t maxiter, const double* mu_guess, double* mu_out,
                                tk_pcg_info* info);

/*
 * Two dipole sets on one operator: the induced dipoles of the AMOEBA model
 * (section "Polarizable AMOEBA force field") come from two permanent fields,
 * solved together by the solver of section "Hotspots" (batched solves of the
 * solver work in section "Perspectives on Tinker-HP 1.2 performance").
 * mu_d solves A mu = E_d, the field of tk_efield_direct (no same-molecule
 * pairs); mu_p solves A mu = E_p, the same field with the damped part of
 * same-molecule pairs scaled by pscale in [0, 1] (pscale = 0: E_p = E_d).
 * Each has its own PCG recurrence, guess rule and stopping test as in
 * tk_polarize_pcg; every mat-vec applies A to both, reading each pair's data
 * once.  mu_guess: device [2][n][3] (mu_d's block first) or NULL; mu_out:
 * device [2][n][3], written in stream order.  info: HOST [2], info[0] for
 * mu_d with epol = -1/2 C mu_d.E_p, info[1] for mu_p with
 * epol = -1/2 C mu_p.E_d (equal up to the residuals, A being symmetric).
 * FP64, real space (tk_polarize_pcg2_ewald adds the reciprocal part).
 * Returns info[0].status if not TK_OK, else info[1].status.  Synchronises `stream` while solving.
 */
tk_status tk_polarize_pcg2(tk_ctx* ctx, void* stream, const tk_system* sys, const tk_nblist* list,
                           const double* mpole, const double* polarity, const double* thole,
                           double ewald_beta, double cutoff, double pscale, double tol_debye,
                           int32_t maxiter, const double* mu_guess, double* mu_out,
                           tk_pcg_info* info);

/*
 * Polarization forces at fixed induced dipoles with the full Ewald operator
 * (the polarization gradient routine of section "Hotspots" with the
 * reciprocal part of the same section): tk_epolar_real's pair terms plus
 * the reciprocal part, which at fixed mu is E_pme(M + mu) - E_pme(M) (the
 * cross term with the permanent multipoles and the dipoles' own
 * interaction).  The two PME evaluations share one pass over the mesh.  At
 * the dipoles of tk_polarize_pcg_ewald the force is the gradient of its
 * E_pol.  energy: device [3] = {total, real-space pair energy (as
 * tk_epolar_real's [0]), reciprocal part}; force: device [n][3].  grid and
 * order as tk_pme_mpole; ewald_beta > 0; FP64; no virial.
 */
tk_status tk_epolar_ewald(tk_ctx* ctx, void* stream, const tk_system* sys,
                          const tk_nblist* list, const double* mpole, const double* polarity,
                          const double* thole, const double* mu, double ewald_beta, double cutoff,
                          int32_t grid, int32_t order, double* energy, double* force);

/*
 * Both dipole sets with the full Ewald operator: tk_polarize_pcg2 with the
 * reciprocal space of tk_polarize_pcg_ewald.  The operator gains the PME
 * field of the dipoles, and both right-hand sides gain the PME field of the
 * permanent multipoles; the same-molecule scaling stays in real space.
 * Arguments, outputs and errors as tk_polarize_pcg2; grid and order as
 * tk_pme_mpole; ewald_beta > 0; FP64.
 */
tk_status tk_polarize_pcg2_ewald(tk_ctx* ctx, void* stream, const tk_system* sys,
                                 const tk_nblist* list, const double* mpole,
                                 const double* polarity, const double* thole, double ewald_beta,
                                 double cutoff, int32_t grid, int32_t order, double pscale,
                                 double tol_debye, int32_t maxiter, const double* mu_guess,
                                 double* mu_out, tk_pcg_info* info);

/*
 * Polarization forces with both dipole sets of tk_polarize_pcg2 (the
 * polarization gradient routine of section "Hotspots" for the two-set model
 * of section "Polarizable AMOEBA force field").  E_pol = -1/2 C E_d.A^-1 E_p
 * is the stationary value of L = 1/2 C [x.A y - x.E_p - y.E_d] at x = mu_d,
 * y = mu_p; the force is -dL/dx at fixed sets (at the solved sets, the
 * gradient of E_pol).  Pair energies:
 *   e_ip = 1/2 [U(mu_d,i, M_j) + U(M_i, mu_d,j)] in the field family of E_p
 *        + 1/2 [U(mu_p,i, M_j) + U(M_i, mu_p,j)] in the field family of E_d,
 *   e_ii = 1/2 [U(mu_d,i, mu_p,j) + U(mu_p,i, mu_d,j)] in the mutual family,
 * the families as tk_epolar_real's, E_p's taking pscale on same-molecule
 * pairs.  mu2: device [2][n][3], mu_d first.  energy: device [3] (total,
 * sum of e_ip, sum of e_ii); force: device [n][3]; virial: device [3][3].
 * FP64.  With mu_d = mu_p and pscale = 0 this is tk_epolar_real.
 */
tk_status tk_epolar2_real(tk_ctx* ctx, void* stream, const tk_system* sys, const tk_nblist* list,
                          const double* mpole, const double* polarity, const double* thole,
                          const double* mu2, double ewald_beta, double cutoff, double pscale,
                          double* energy, double* force, double* virial);

/*
 * Local-frame multipoles (the rotation step that section "Hotspots" lists
 * beside the multipole routines).  frame_type: device [n] int32 (TK_FRAME_*);
 * frame_atoms: device [n][3] int32, the z-, x- and y-atom of each site.  A
 * type reads only the atoms it takes (z: types 1-5, x: 1, 2, 4, 5, y: 4, 5);
 * those are in [0, n), not the site, and distinct.  With d_k = r_katom - r_i
 * (minimum image) and u_k = unit(d_k), each type takes z and a vector a:
 *   1 Z-then-X:   z = u_z,                   a = d_x;
 *   2 bisector:   z = unit(u_z + u_x),       a = u_x;
 *   3 Z-only:     z = u_z,                   a = the global x axis, or the
 *                 global y axis when |z_x| > 0.866;
 *   4 Z-bisector: z = u_z,                   a = u_x + u_y;
 *   5 3-fold:     z = unit(u_z + u_x + u_y), a = u_x;
 * then x = unit(a - (a.z) z), y = z x x.  With R = [x y z]: q = q_loc,
 * mu = R mu_loc, Theta = R Theta_loc R^T.  mpole_local, mpole_global: device
 * [n][10] in the layout of tk_empole_real.  An invalid frame copies the
 * site's local multipoles unchanged.
 */
#define TK_FRAME_NONE 0
#define TK_FRAME_Z_THEN_X 1
#define TK_FRAME_BISECTOR 2
#define TK_FRAME_Z_ONLY 3
#define TK_FRAME_Z_BISECTOR 4
#define TK_FRAME_3FOLD 5
tk_status tk_rotate_mpole(tk_ctx* ctx, void* stream, const tk_system* sys,
                          const int32_t* frame_type, const int32_t* frame_atoms,
                          const double* mpole_local, double* mpole_global);

/*
 * Real-space permanent-multipole energy and forces with local-frame
 * multipoles (the multipole routine with its torque step): the energy of
 * tk_empole_real at the rotated multipoles M(x), and its full gradient, the
 * direct pair forces plus the frame part -sum_c dE/dM_i,c dM_i,c/dx for the
 * site and its frame atoms.  FP64.  energy: device [3] as
 * tk_empole_real (all three NaN if a frame is invalid); force: device [n][3];
 * virial: device [3][3] or NULL, W_ab = sum over the relative vectors v the
 * energy depends on (pair vectors and each site's frame vectors d_k) of
 * v_a dE/dv_b: tk_empole_real's pair virial at M plus the frame part
 * sum_k d_k,a dE/dd_k,b (NaN if a frame is invalid); mpole_global: device
 * [n][10] receiving the rotated multipoles, or NULL.  The frame forces are
 * added with atomics: reproducible to rounding, not bitwise; the virial's
 * sums run in a fixed order.
 */
tk_status tk_empole_frames(tk_ctx* ctx, void* stream, const tk_system* sys,
                           const tk_nblist* list, const int32_t* frame_type,
                           const int32_t* frame_atoms, const double* mpole_local,
                           double ewald_beta, double cutoff, double* energy, double* force,
                           double* virial, double* mpole_global);

/*
 * Polarization forces at fixed induced dipoles with local-frame multipoles:
 * the pair energies of tk_epolar_real at the rotated multipoles M(x), and
 * their full gradient, the pair forces plus the frame part of the
 * induced-permanent energy (its dE/dM through the rotation, as in
 * tk_empole_frames).  Arguments as tk_empole_frames and tk_epolar_real; FP64;
 * energy: device [3] (NaN if a frame is invalid); virial: device [3][3] or
 * NULL, tk_epolar_real's pair virial at M plus the frame part, as in
 * tk_empole_frames.
 */
tk_status tk_epolar_frames(tk_ctx* ctx, void* stream, const tk_system* sys,
                           const tk_nblist* list, const int32_t* frame_type,
                           const int32_t* frame_atoms, const double* mpole_local,
                           const double* polarity, const double* thole, const double* mu,
                           double ewald_beta, double cutoff, double* energy, double* force,
                           double* virial);

/*
 * vdW hydrogen reduction (AMOEBA's Halgren term puts a hydrogen's vdW site on
 * its bond).  tk_vdw_sites: site i at r_p + red_i (r_i - r_p), minimum image,
 * for parent[i] = p >= 0, else at r_i; an invalid parent (>= n or i) gives a
 * NaN site.  parent: device [n] int32 (-1: none); red: device [n];
 * sites: device [n][3].  The caller lists and evaluates the sites with
 * tk_nblist_build and tk_evdw on a tk_system holding them, then
 * tk_vdw_site_forces maps the site forces to atoms by the chain rule: atom i
 * receives red_i f_i, its parent (1 - red_i) f_i (added with atomics:
 * reproducible to rounding).  site_force, atom_force: device [n][3],
 * distinct.  The site virial of tk_evdw is not mapped.
 */
tk_status tk_vdw_sites(tk_ctx* ctx, void* stream, const tk_system* sys, const int32_t* parent,
                       const double* red, double* sites);
tk_status tk_vdw_site_forces(tk_ctx* ctx, void* stream, int32_t n, const int32_t* parent,
                             const double* red, const double* site_force, double* atom_force);

/*
 * One-step truncated conjugate gradient (TCG1), a fixed-cost polarization
 * solve with the exact derivative of its energy (the fixed-cost solvers of
 * the paper's later versions).  With A, E_perm as in tk_polarize_pcg,
 * diagonal preconditioner alpha, direct guess and no "peek" step:
 *   mu0 = alpha E,  r0 = E - A mu0,  p0 = alpha r0,  a = (r0.p0)/(p0.A p0),
 *   mu1 = mu0 + a p0,  U = -1/2 C mu1.E.
 * mu_out: device [n][3] (mu1); epol: device [1] (U); force: device [n][3]
 * or NULL, the total derivative -dU/dx through every step (U is not
 * variational, so this is not tk_epolar_real at mu1).  FP64; no host
 * synchronisation.
 */
tk_status tk_polarize_tcg1(tk_ctx* ctx, void* stream, const tk_system* sys, const tk_nblist* list,
                           const double* mpole, const double* polarity, const double* thole,
                           double ewald_beta, double cutoff, double* mu_out, double* epol,
                           double* force);

/*
 * Real-space polarization forces (epolar1 in the Rel profile, the second
 * AMOEBA hotspot of section "Hotspots").  The polarization energy is the
 * minimum over mu of C [1/2 mu.A mu - mu.E_perm] (A, E_perm as above),
 * -1/2 C mu.E_perm at the solution.  This call returns -d/dx of that
 * expression at the given, fixed mu: at converged dipoles, the gradient of
 * the polarization energy itself.  For each listed pair with r <= cutoff,
 * with an induced dipole written as the multipole (0, mu, 0) and U the pair
 * energy of tk_empole_real:
 *   e_ip = U(mu_i, M_j; gp) + U(M_i, mu_j; gp) = -C (mu_i.E_i<-j + mu_j.E_j<-i),
 *   e_ii = U(mu_i, mu_j; gm) = -C mu_i.T2 mu_j,
 * gp_n = B_n - (1 - s l_(2n+1)) R_n (s = 0 within a molecule, else 1),
 * gm_n = B_n - (1 - l_(2n+1)) R_n, Thole factors as in tk_efield_direct plus
 * l9 = 1 - (1 + x + 18/35 x^2 + 9/35 x^3) e^-x for the quadrupole term.
 * mu: device [n][3] (e A), e.g. tk_polarize_pcg's mu_out.  energy: device
 * [3] = e_ip + e_ii, sum of e_ip, sum of e_ii (the self and 1/2 mu.mu/alpha
 * terms do not depend on positions and are not included; at the solution
 * -1/2 C mu.E_perm is tk_pcg_info.epol).  force: device [n][3];
 * virial: device [3][3], W_ab = sum over pairs r_a de/dr_b.
 */
tk_status tk_epolar_real(tk_ctx* ctx, void* stream, const tk_system* sys, const tk_nblist* list,
                         const double* mpole, const double* polarity, const double* thole,
                         const double* mu, double ewald_beta, double cutoff, int prec,
                         double* energy, double* force, double* virial);

/*
 * Reciprocal-space multipole energy, forces and field by smooth particle-mesh
 * Ewald (the reciprocal multipole routine that section "Hotspots" names beside
 * the real-space one; the paper leaves it unvectorized).  It approximates the
 * Ewald sum (C/2V) sum_{k != 0} (4 pi/k^2) exp(-k^2/(4 beta^2)) |S(k)|^2,
 * S(k) = sum_j (q_j + i mu_j.k - Theta_j:kk) exp(i k.r_j) (tin-foil boundary),
 * on a grid x grid x grid mesh with cardinal B-splines of the given order:
 * sites are spread as q M + mu.grad M + Theta:grad grad M, the mesh is
 * convolved with (4 pi/k^2) exp(-k^2/(4 beta^2)) / (V |b(m)|^-2) by FFTs
 * (|b(m)|^-2 the spline modulus, at a zero replaced by the mean of its
 * neighbours), and the potential and its derivatives up to third order are
 * interpolated back at each site.  mpole: device [n][10] as tk_empole_real;
 * the coordinates of sys, any values (wrapped into the box).  grid: 16, 32,
 * 64 or 128; order: 5..8 with grid >= 2 order.  energy: device [1] (NaN if a
 * site's spread contribution reaches 2^17 e/A^k, outside the fixed-point
 * range of the deterministic grid); force: device [n][3], -dE/dx; field:
 * device [n][3] or NULL, -grad phi in e/A^2 (no Coulomb constant), including
 * each site's own contribution (the real-space self field removes it).  No
 * real-space, self or virial term.  sys->molid is not used.
 */
tk_status tk_pme_mpole(tk_ctx* ctx, void* stream, const tk_system* sys, const double* mpole,
                       double ewald_beta, int32_t grid, int32_t order, double* energy,
                       double* force, double* field);

/*
 * van der Waals (ehal / elj in the Rel profile).  form = TK_VDW_HAL: Halgren
 * buffered 14-7, e = eps_ij [(1+d) R_ij/(r + d R_ij)]^7
 * [(1+g) R_ij^7/(r^7 + g R_ij^7) - 2], R_ij = (R_i^3+R_j^3)/(R_i^2+R_j^2),
 * eps_ij = 4 e_i e_j/(sqrt(e_i)+sqrt(e_j))^2, d = hal_delta, g = hal_gamma.
 * form = TK_VDW_LJ: e = 4 eps_ij [(s/r)^12 - (s/r)^6], s = (s_i+s_j)/2,
 * eps_ij = sqrt(e_i e_j).  Same-molecule pairs are skipped; for
 * r > taper_on_frac * cutoff the energy is multiplied by
 * S(x) = 1 - 10x^3 + 15x^4 - 6x^5, x = (r - r_on)/(cutoff - r_on).
 * radius_or_sigma, eps: device [n].  energy: device [1].
 */
tk_status tk_evdw(tk_ctx* ctx, void* stream, const tk_system* sys, const tk_nblist* list,
                  int form, const double* radius_or_sigma, const double* eps, double cutoff,
                  double taper_on_frac, double hal_delta, double hal_gamma, int prec,
                  double* energy, double* force, double* virial);

/* ------------------------------------------------------------------------
 * Batches of independent systems (the serving form; the paper has no serving
 * path, so this is an engine feature around the terms of section "Hotspots").
 *
 * A batch holds nsys systems, each with its own periodic cubic box; every
 * launch of a batch step covers all of them (multi-system kernels: each cell
 * and each unit knows its system), and each system's results are bitwise
 * identical to those of the same system stepped alone.
 */
typedef struct {
  int32_t nsys;              /* number of systems, >= 1 */
  const int32_t* atom_off;   /* host [nsys+1]: system k owns atoms atom_off[k] .. atom_off[k+1]-1,
                                atom_off[0] = 0, non-decreasing */
  const double* box;         /* host [nsys]: cubic edge of each system (A) */
  const double* xyz;         /* device [atom_off[nsys]][3], each system in its own frame */
  const int32_t* molid;      /* device [atom_off[nsys]]: molecule ids (compared within a system) */
} tk_batch;

typedef struct {             /* host; one AMOEBA step for every system of a batch */
  double rc_ewald;           /* real-space Ewald cutoff (A); rc_ewald + skin <= box/2 is required */
  double rc_vdw;             /* vdW cutoff; per system clamped to box/2 - skin (small boxes) */
  double skin;               /* list skin added to both cutoffs (>= 0) */
  double ewald_beta;         /* Ewald screening parameter (1/A) */
  double tol_debye;          /* PCG tolerance, RMS of the preconditioned residual (D) */
  double taper_on_frac;      /* vdW taper start as a fraction of the vdW cutoff */
  double hal_delta, hal_gamma;
  int32_t maxiter;           /* PCG iteration limit */
  int32_t prec;              /* TK_FP64 or TK_MIXED */
} tk_step_params;

typedef struct {             /* host; per system */
  double e_mpole[3];         /* permanent multipoles: total, non-excluded, exclusion correction */
  double w_mpole[9];
  double e_vdw;              /* Halgren 14-7 */
  double w_vdw[9];
  double rc_vdw;             /* the vdW cutoff used for this system */
  tk_pcg_info pcg;           /* the induced-dipole solve (epol = -C/2 mu.E_perm) */
} tk_step_result;

/*
 * One step for every system of the batch: neighbour lists at rc_ewald + skin
 * and rc_vdw(k) + skin, tk_empole_real, tk_polarize_pcg and tk_evdw (HAL)
 * with the definitions stated at those entry points.
 * mpole [n][10], polarity, thole, vdw_rad, vdw_eps [n]: device, caller order.
 * mu_guess: device [n][3] or NULL; use_guess: host [nsys] or NULL.  System k
 * starts its dipole solve from mu_guess when mu_guess is given and
 * (use_guess is NULL or use_guess[k] != 0), else from alpha * E_perm.
 * Outputs (device, [n][3], overwritten): force_mpole, mu, force_vdw.
 * results: host [nsys].
 * Synchronises the stream.  Returns TK_OK even when some system's solve did
 * not converge (see results[k].pcg.status); TK_E_CUTOFF when rc_ewald + skin
 * exceeds some box/2; TK_E_CAPACITY when a cell holds more atoms than the
 * kernels stage.  Uses two context plan slots of its own (not the caller's).
 */
tk_status tk_batch_step(tk_ctx* ctx, void* stream, const tk_batch* batch,
                        const tk_step_params* params, const double* mpole,
                        const double* polarity, const double* thole, const double* vdw_rad,
                        const double* vdw_eps, const double* mu_guess,
                        const int32_t* use_guess, double* force_mpole, double* mu,
                        double* force_vdw, tk_step_result* results);

/*
 * Serving runtime: continuous batching of step requests.  A server runs
 * three lanes on `device`, each a host thread with its own context, HIP
 * stream and pinned staging.  Requests are queued by tk_server_submit (host
 * arrays, copied at once).  An idle lane takes the requests queued at that
 * moment, in arrival order (at most max_batch), into a batch and runs one
 * tk_batch_step on its stream; a request arriving while batches are on the
 * GPU is taken by the next idle lane at once, and its work overlaps theirs.
 * Admission is by measured device memory: a batch joins a lane while the
 * lane's projected holdings (the measured bytes per atom of earlier
 * batches; tk_server_footprint before the first) plus the other lanes'
 * holdings stay within hbm_budget, and the lane's context is bounded by the
 * same limit (a batch that would overrun it runs its first request alone
 * and returns the rest to the queue).  The lanes' device bytes never exceed
 * the budget.  A system's results are the same whatever batch it runs in.
 * A request that alone exceeds the budget is rejected (TK_E_CAPACITY).  A
 * lane that cannot make a new device context stops; when no lane is left,
 * queued requests complete with TK_E_NOMEM and tk_server_submit returns it.
 * Sessions: a request with a nonzero session id starts its dipole solve from
 * the dipoles of the previous completed request of the same session when
 * the atom count matches (resident guesses; otherwise from alpha * E_perm).
 * The server's functions may be called from any host thread.
 */
typedef struct tk_server tk_server;

typedef struct {             /* host arrays, copied by tk_server_submit */
  int32_t n;
  double box;
  const double* xyz;         /* [n][3] */
  const int32_t* molid;      /* [n] */
  const double* mpole;       /* [n][10] */
  const double* polarity;    /* [n] */
  const double* thole;       /* [n] */
  const double* vdw_rad;     /* [n] */
  const double* vdw_eps;     /* [n] */
  uint64_t session;          /* 0: none */
} tk_request;

typedef struct {             /* host timestamps (ns, monotonic clock) and the batch it ran in */
  int64_t t_submit, t_start, t_done;
  int32_t batch_size;        /* systems in that batch */
  int32_t batch_index;       /* sequence number of the batch */
  int32_t lane;              /* the lane that ran it */
} tk_timing;

typedef struct {
  int32_t lanes, batches;      /* concurrent lanes; batches run so far */
  size_t budget;               /* hbm_budget */
  size_t peak_device_bytes;    /* largest measured sum of the lanes' device holdings */
  size_t device_bytes;         /* their sum now */
  double bytes_per_atom;       /* measured admission rate (0 before the first batch) */
} tk_server_usage;

tk_status tk_server_create(int device, const tk_step_params* params, size_t hbm_budget,
                           int32_t max_batch, tk_server** out);
/* As tk_server_create with `lanes` lanes (1 to 3; TK_E_ARG otherwise).  One
 * lane with max_batch 1 serves one request at a time. */
tk_status tk_server_create_lanes(int device, const tk_step_params* params, size_t hbm_budget,
                                 int32_t max_batch, int32_t lanes, tk_server** out);
/* Estimated device bytes of one request of n atoms (the admission measure
 * before the server has measured a batch). */
size_t tk_server_footprint(int32_t n);
tk_status tk_server_submit(tk_server* srv, const tk_request* req, uint64_t* id);
/*
 * TK_E_BUSY while request `id` is queued or running; then copies its results
 * (any output pointer may be NULL: host [n][3] arrays force_mpole, mu,
 * force_vdw) and returns the step status (TK_OK, or the batch's error).
 * A request's results can be polled until tk_server_release(id).
 */
tk_status tk_server_poll(tk_server* srv, uint64_t id, tk_step_result* result, tk_timing* timing,
                         double* force_mpole, double* mu, double* force_vdw);
tk_status tk_server_release(tk_server* srv, uint64_t id);
/* Lanes, batches and measured device memory of the server (host struct). */
tk_status tk_server_stats(tk_server* srv, tk_server_usage* out);
/* Waits for every submitted request, then stops the lanes and frees all. */
void tk_server_destroy(tk_server* srv);

/*
 * Device-memory budget of a context: the sum of the device buffers the
 * context keeps (plans, solver and pair-term scratch; all grow-only) may not
 * exceed `bytes` (0: no bound, the default).  A call that would need more
 * returns TK_E_NOMEM before launching anything that uses the missing buffer;
 * the buffers the context already holds stay valid, so the caller may raise
 * the budget and call again.  tk_arena_bytes returns what the context holds.
 */
tk_status tk_set_arena_budget(tk_ctx* ctx, size_t bytes);
size_t tk_arena_bytes(const tk_ctx* ctx);

/*
 * Kernel timing (tracing aid).  When enabled, the library brackets its kernel
 * launches with HIP events on the launch stream; `only` (host string, may be
 * NULL) restricts timing to the kernel of that name.  tk_profile_read returns
 * the idx-th timed kernel (names like "units_tmat_fp64", "nblist_rows_fill"):
 * name (host buffer of name_len bytes), number of timed launches and total
 * milliseconds; it waits for the timed work to finish.  TK_E_ARG when idx is
 * past the last kernel.  tk_profile_enable(ctx, 0, NULL) stops timing;
 * tk_profile_reset clears the counters.
 */
tk_status tk_profile_enable(tk_ctx* ctx, int on, const char* only);
tk_status tk_profile_read(tk_ctx* ctx, int32_t idx, char* name, int32_t name_len,
                          int64_t* launches, double* total_ms);
tk_status tk_profile_reset(tk_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* TK_H */
