/*
 * dem.h -- C ABI of the MI355X DEM + fluid-coupling library.
 *
 * The library advances the coarse-grained CFD-DEM particle phase of
 * Kazidenov, Khamitov & Amanbek, "Coarse-graining of CFD-DEM for simulation
 * of sand production in the modified cohesive contact model"
 * (arXiv:2211.06142):
 *   - Newton-Euler motion of spheres (section 2.1, eq 1-2), velocity Verlet;
 *   - modified JKR cohesive normal law: bonds break at the pull-off point C
 *     and never re-form, new contacts are Hertz (section 2.3, eq 12-13,
 *     Table 1, Fig. 2); damping from the restitution coefficient (eq 32-33);
 *   - tangential spring-dashpot with Coulomb cap and contact torque
 *     (section 2.1, eq 4-5, eq 35), optional rolling resistance;
 *   - fluid-particle coupling of unresolved CFD-DEM "model A": porosity of
 *     each fluid cell, Di Felice drag on each particle, drag source of each
 *     cell (section 2.2, eq 6-11), buoyancy and pressure-gradient force;
 *   - the fine-to-coarse scaling of section 2.4 (eq 14-35, Table 3) applied
 *     by the coarse-grain factor k: only the surface energy changes
 *     (gamma_g = k gamma_p), drag on a grain is k^3 times the drag on a fine
 *     particle of diameter d/k.
 *
 * Conventions (all calls)
 *   - SI units; 3-vectors interleaved (x0,y0,z0,x1,...), FP64 unless stated.
 *   - Every call returns dem_status; no exception or longjmp crosses the ABI.
 *   - A context is single-stream and not thread-safe.  All device work is
 *     ordered on the HIP stream given to dem_init; calls return after the work
 *     they queue has completed unless stated otherwise.
 *   - Pointers marked "host or device" are inspected with
 *     hipPointerGetAttributes; both kinds are accepted.
 *   - Device faults found during stepping (pair capacity overflow, non-finite
 *     force, a particle moving more than half the skin in one step) are latched
 *     in a device status word and returned by the call that observes them;
 *     the context then refuses further steps (DEM_E_STATE) until destroyed.
 *   - Batches: a context may hold several independent samples (systems that
 *     never interact), each with its own dem_params; particles of sample s are
 *     the contiguous range [offsets[s], offsets[s+1]) of every per-particle
 *     array and its fluid cells follow those of sample s-1.
 */
#ifndef DEM_H
#define DEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DEM_OK = 0,
  DEM_E_INVAL = -1,     /* invalid argument; no state was changed              */
  DEM_E_NOMEM = -2,     /* device allocation failed                            */
  DEM_E_CAPACITY = -3,  /* pair capacity exceeded and DEM_FLAG_AUTO_REGROW off  */
  DEM_E_NONFINITE = -4, /* a force or torque became NaN or infinite            */
  DEM_E_DEVICE = -5,    /* a HIP runtime call failed                           */
  DEM_E_STATE = -6      /* call not valid in this state (see dem_status_str)   */
} dem_status;

#define DEM_MAX_WALLS 8

enum { DEM_WALL_PLANE = 0, DEM_WALL_CYL_IN = 1, DEM_WALL_CYL_OUT = 2, DEM_WALL_PLANE_HOLE = 3 };
/* Normal laws.  JKR_MOD: the modified JKR model of section 2.3 (Fig. 2), bonds
 * set at init (bond_at_init or the given history) break at point C and never
 * re-form, other contacts are Hertz.  HERTZ: no cohesion.  LINEAR: eq 3, a test
 * law.  JKR_ORIG: the original JKR cycle of section 2.3 (Fig. 1), the paper's
 * generation stage: a contact forms whenever two particles touch (point A,
 * where the force drops to -8/9 F_C), follows eq 12-13 through C and separates
 * at point S, the smallest overlap of eq 13, (-delta_S)^3 = (27/16) pi^2 gamma^2
 * R* / E*^2 (separations count in broken_bonds), and forms again on the next
 * touch. */
enum { DEM_NORMAL_JKR_MOD = 0, DEM_NORMAL_HERTZ = 1, DEM_NORMAL_LINEAR = 2, DEM_NORMAL_JKR_ORIG = 3 };
enum { DEM_VOID_CIC = 0, DEM_VOID_CENTROID = 1 };
/* Outlets (section 3.3 eq 40: a particle that leaves is produced sand).  CAVITY:
 * a centre inside the vertical cylinder outlet[0..1] axis, outlet[2] radius
 * leaves (the workloads' cavity).  ABOVE: a centre above the level z =
 * outlet[3] leaves (the paper's outlet on the top face of its box, with a
 * PLANE_HOLE wall as the top plate: the only way up is through the hole). */
enum { DEM_OUTLET_NONE = 0, DEM_OUTLET_CAVITY = 1, DEM_OUTLET_ABOVE = 2 };
enum { DEM_PREC_FP64 = 0, DEM_PREC_MIXED = 1 };
enum { DEM_CG_SSW = 0, DEM_CG_SSP = 1 };
enum { DEM_FLAG_AUTO_REGROW = 1u };
#define DEM_MAX_SIZE_CLASSES 16

/* A wall.  PLANE: p[0..2] unit normal pointing into the particle side, p[3]
 * offset (signed distance of a point x is n.x - p[3]).  CYL_IN: particles
 * inside a z-axis cylinder, p[0], p[1] axis position, p[2] radius.  CYL_OUT:
 * particles outside such a cylinder.  PLANE_HOLE: the horizontal plane
 * z = p[2] with particles on the side p[3] (+1 above, -1 below) and a circular
 * hole of radius p[4] about the vertical axis through (p[0], p[1]): a particle
 * whose centre lies within the hole radius of that axis does not touch the
 * plane (the outlet in the top face of the paper's box, section 3.1).  Walls
 * are rigid, static, of the particles' material; contact with them is Hertz
 * with tangential history (the particle-wall law of section 3.1). */
typedef struct {
  int32_t kind;
  int32_t reserved;
  double p[6];
} dem_wall;

/* Cell-centred fluid grid: n[0]*n[1]*n[2] cells of equal size covering
 * [lo, hi]; cell (ix, iy, iz) has linear index (iz*n[1] + iy)*n[0] + ix.
 * At most 2^30 cells per sample (DEM_E_INVAL otherwise). */
typedef struct {
  double lo[3], hi[3];
  int32_t n[3];
  int32_t reserved;
} dem_grid;

/* Parameters of one sample.  Material values are FINE-scale (the layout of
 * Table 3); the library applies the coarse-graining of section 2.4 with the
 * factor k: gamma_g = k gamma, everything else unchanged, drag rule k^3 f(d/k).
 * Particle radii given to dem_init are the grains' own radii (SSW: fine
 * diameters times k; SSP: one diameter, see dem_cg_diameters). */
typedef struct {
  double rho, E, nu, e, mu, mu_roll, gamma;  /* density, Young, Poisson, restitution,
                                                friction, rolling friction, surface energy */
  double k;                 /* coarse-grain factor (eq 14), >= 1; 1 = no scaling    */
  int32_t cg_scheme;        /* DEM_CG_SSW or DEM_CG_SSP (bookkeeping only)          */
  int32_t normal_model;     /* DEM_NORMAL_*; LINEAR (eq 3) is a test law            */
  double k_lin;             /* spring constant of the LINEAR law, N/m               */
  int32_t fluid_on;         /* 1: drag/porosity coupling active                     */
  int32_t voidfrac;         /* DEM_VOID_CIC (trilinear) or DEM_VOID_CENTROID         */
  int32_t u_superficial;    /* 1: fluid velocity passed to dem_map_fluid is n*u     */
  int32_t couple_every;     /* DEM steps between coupling evaluations (>= 1)        */
  double rho_f, mu_f;       /* fluid density and viscosity (Table 4)                */
  double n_min;             /* lower clamp of the cell porosity                     */
  dem_grid grid;            /* fluid grid of this sample                            */
  double g[3];              /* gravity                                              */
  double dt;                /* DEM time step (same for all samples)                 */
  double skin;              /* neighbour-list skin; <= 0: 0.2 x smallest diameter   */
  double dt_rayleigh_max_frac; /* > 0: reject dt above this fraction of eq 37       */
  int32_t outlet_kind;      /* DEM_OUTLET_*                                         */
  int32_t n_walls;          /* <= DEM_MAX_WALLS                                     */
  double outlet[4];         /* CAVITY: axis x, axis y, radius; ABOVE: [3] the level */
  dem_wall walls[DEM_MAX_WALLS];
  int32_t precision;        /* DEM_PREC_FP64 or DEM_PREC_MIXED (same for all samples) */
  int32_t bond_at_init;     /* 1: every touching pair starts bonded (JKR_MOD, ORIG) */
  int64_t pair_capacity;    /* half-pair capacity; <= 0: automatic (grows at every
                               rebuild as needed).  > 0 without DEM_FLAG_AUTO_REGROW
                               (sample 0's value): fixed -- a rebuild that needs
                               more half pairs, row entries (2x) or wall entries
                               (n/4 + 256) latches fault bit 1 and the step call
                               returns DEM_E_CAPACITY; with the flag: initial size */
  uint32_t flags;           /* DEM_FLAG_*                                           */
  int32_t reserved;
} dem_params;

/* Particle state.  Owned by the caller; on input to dem_init every pointer
 * may be host or device, on output of dem_read_state every pointer may be
 * host or device or NULL (not wanted).  Order of particles is the caller's
 * original order throughout.  Everything one step depends on is here: the
 * state read from one context and given to dem_init continues the run (to
 * the rounding of the force sums, whose order follows the new context's
 * binning), and the oracle can be seeded from it. */
typedef struct {
  int64_t n;                /* number of particles (all samples)                    */
  double* x;                /* 3n positions                                         */
  double* v;                /* 3n velocities                                        */
  double* omega;            /* 3n angular velocities                                */
  double* force;            /* 3n total force of the last evaluation (NULL: zero)   */
  double* torque;           /* 3n total torque of the last evaluation (NULL: zero)  */
  double* radius;           /* n radii (input only)                                 */
  uint8_t* alive;           /* n; 0 = removed through the outlet (NULL: all alive)  */
  /* contact history; dem_init: optional input (n_pairs > 0 replaces
   * bond_at_init); dem_read_state: see dem_read_pairs */
  int64_t n_pairs;
  int64_t* pair_idx;        /* 2 n_pairs particle indices (a, b), a < b             */
  double* pair_dt;          /* 3 n_pairs tangential elongation, orientation a -> b  */
  uint8_t* pair_bonded;     /* n_pairs                                              */
  /* scalars filled by dem_read_state */
  double produced_mass;     /* mass removed through the outlet (eq 40 integrand)    */
  double time;              /* simulated time                                       */
  double coordination;      /* 2 x active contacts / alive particles                */
  double kinetic;           /* translational + rotational kinetic energy            */
  int64_t step;             /* steps taken                                          */
  int64_t broken_bonds;     /* bonds broken at point C since init                   */
  int64_t n_alive;
  int64_t n_contacts;       /* active particle-particle contacts                    */
  /* held state (input to dem_init and output of dem_read_state; NULL: zero /
   * not wanted) */
  double* fluid_force;      /* 3n fluid force on each particle (drag of eq 8 plus
                               buoyancy and pressure gradient) held since the
                               latest coupling evaluation                          */
  double* wall_dt;          /* 3 n DEM_MAX_WALLS tangential elongation of every
                               particle-wall contact, [particle][wall][xyz], wall =
                               index into its sample's walls                       */
} dem_state;

typedef struct dem_ctx dem_ctx;

/* Create a context on `device` using HIP stream `hip_stream` (NULL: the
 * default stream).  params: n_samples entries; sample_offsets: n_samples+1
 * increasing particle offsets (NULL allowed when n_samples == 1).  The
 * initial state is copied; the caller keeps ownership.  init->step (>= 0) is
 * the step count the run resumes at (it decides the coupling schedule, step
 * modulo couple_every; 0 for a new run); the produced-mass, broken-bond and
 * size-class counters start at zero.  Validation failures
 * (dt <= 0 or differing between samples, nu outside (-1, 0.5), e outside
 * (0, 1], k < 1, a radius <= 0, a non-finite input, an empty fluid grid while
 * fluid_on, dt above dt_rayleigh_max_frac of the Rayleigh step of eq 37-38
 * for the smallest radius) return DEM_E_INVAL and leave *out NULL. */
dem_status dem_init(dem_ctx** out, const dem_params* params, int32_t n_samples,
                    const int64_t* sample_offsets, const dem_state* init, int32_t device,
                    void* hip_stream);

/* Advance every sample by nsteps DEM steps (stream-ordered).  One step
 * (section 2.1 eq 1-2 integrated by velocity Verlet): first half kick and
 * drift; outlet removal (section 3.3 eq 40: a centre inside the cavity leaves
 * as produced sand, its contacts are deleted); the coupling evaluation of
 * section 2.2 eq 6-11 every couple_every steps (porosity by deposition, Di
 * Felice drag with the coarse-grained rule, buoyancy and pressure gradient,
 * the eq 7 cell source); the contact forces of every pair (modified JKR /
 * Hertz normal law of section 2.3 eq 12-13, damping eq 32-33, tangential
 * spring with Coulomb cap eq 4 and 35, torque eq 5) and of every wall
 * contact; gravity; second half kick.  nsteps < 0: DEM_E_INVAL; a latched
 * fault (see the conventions above) is returned by the call that finds it.
 * Returns after the steps have completed. */
dem_status dem_step(dem_ctx* ctx, int64_t nsteps);

/* Coupling exchange with the fluid solver (section 2.2, eq 6-7).
 * u_cell, gradp_cell: 3*ncell fluid velocity (superficial n*u when
 * u_superficial) and dynamic pressure gradient per cell, host or device,
 * FP64; they replace the fields used by later coupling evaluations.
 * eps_solid_out (ncell) and fdrag_out (3*ncell), host, device or NULL,
 * receive the solid volume fraction and the eq 7 drag source (sum over the
 * particles of the drag ON them, weighted into the cell, per cell volume;
 * the fluid receives its negative) of the latest coupling evaluation, and
 * zeros before the first one.  ncell is the total over all samples. */
dem_status dem_map_fluid(dem_ctx* ctx, const double* u_cell, const double* gradp_cell,
                         double* eps_solid_out, double* fdrag_out);

/* The fluid side of the coupling (section 2.2, eq 6, model A) in its
 * drag-dominated limit: with the unsteady, advective and viscous terms small
 * against the pressure gradient and the particle-fluid force (the packed bed
 * at low particle Reynolds number), eq 6 reduces to n grad(p) = -beta u and,
 * with the bed at rest relative to the fluid, div(n u) = 0 to the pressure
 * equation div(K grad p) = 0 with K = n^2 / beta.  beta per cell is the drag
 * coefficient of the latest coupling evaluation (|eq 7 drag source| /
 * |interstitial velocity|) plus 12 mu_f / h_min^2, the viscous resistance of
 * flow between plates one cell apart (particle-free cells); n is that
 * evaluation's porosity.  Cell-centred finite volumes on each sample's grid
 * (face coefficient: harmonic mean of K), solved by conjugate gradients with
 * the diagonal as preconditioner to |r| <= rel_tol |b| or max_iter iterations,
 * warm-started from the previous solution.  cell_kind (int8, ncell):
 * DEM_CELL_OPEN unknown pressure, DEM_CELL_PRESSURE pressure p_fixed (the
 * outlets and inlets), DEM_CELL_SOLID no flow (walls); the outer boundary of
 * the grid carries no flow.  Each connected set of open cells must reach a
 * fixed-pressure cell.  Outputs (host, device or NULL): p_out (ncell, dynamic
 * pressure), u_out (3 ncell, superficial velocity n u: the mean of each axis's
 * two face fluxes) and gradp_out (3 ncell, mean one-sided differences): the
 * fields dem_map_fluid takes for the next evaluations (with u_superficial 1),
 * which closes the two-way coupling.  iters, rel_residual: host (may be NULL).
 * DEM_E_INVAL for a missing input, a kind outside 0..2, max_iter < 0 or
 * rel_tol <= 0; DEM_E_STATE without fluid cells.  Synchronises. */
enum { DEM_CELL_OPEN = 0, DEM_CELL_PRESSURE = 1, DEM_CELL_SOLID = 2 };
dem_status dem_fluid_solve(dem_ctx* ctx, const int8_t* cell_kind, const double* p_fixed, int32_t max_iter,
                           double rel_tol, double* p_out, double* u_out, double* gradp_out, int32_t* iters,
                           double* rel_residual);

/* Copy the state out in the caller's particle order (see dem_state): the
 * Newton-Euler state of eq 1-2 (x, v, omega), the forces and torques of the
 * latest evaluation, the alive flags, the held fluid force and wall history,
 * and the section 3.3-3.4 observables (produced mass of eq 40, coordination,
 * broken bonds, kinetic energy).  The pair arrays are not written; use
 * dem_read_pairs.  Synchronises.  A latched fault is returned after the copy
 * (DEM_E_NONFINITE or DEM_E_STATE), so the state that raised it can be read. */
dem_status dem_read_state(dem_ctx* ctx, dem_state* out);

/* Active contact history: pairs with a bond or touching at the last force
 * evaluation, as particle indices a < b in the caller's order.  cap is the
 * capacity of the output arrays (host or device); *n_out receives the count
 * (which may exceed cap; then only cap entries are written).  touching_only:
 * 0 active pairs, 1 only pairs with d < r_a + r_b, 2 every candidate pair of
 * the neighbour list (d < r_a + r_b + cutoff margin). */
dem_status dem_read_pairs(dem_ctx* ctx, int32_t which, int64_t cap, int64_t* pair_idx,
                          double* pair_dt, uint8_t* pair_bonded, int64_t* n_out);

/* Per-sample aggregates (section 3.3-3.4 observables): produced mass,
 * coordination number, broken bonds, alive count.  Arrays of n_samples, host. */
dem_status dem_read_aggregates(dem_ctx* ctx, double* produced_mass, double* coordination,
                               int64_t* broken_bonds, int64_t* n_alive);

/* Produced sand by size class (section 3.3, Fig. 11: produced mass per
 * diameter group).  dem_set_size_classes: n_edges increasing diameters
 * (2 <= n_edges <= DEM_MAX_SIZE_CLASSES + 1, host) bound n_edges - 1 classes
 * [e0, e1), [e1, e2), ... of the fine-scale diameter d/k of the removed
 * grain (SSW grains count in the class of the fine particles they stand for);
 * the end classes also take diameters beyond the outer edges.  It zeroes the
 * per-class counters; later removals are counted (NULL or n_edges 0: off).
 * dem_read_produced_classes: mass[s * n_classes + c] (kg) of sample s and
 * class c, host or device array of n_samples x n_classes; DEM_E_STATE if no
 * classes are set.  Every removal adds its mass exactly (fixed point), so the
 * counts do not depend on the order of removals. */
dem_status dem_set_size_classes(dem_ctx* ctx, int32_t n_edges, const double* edges);
dem_status dem_read_produced_classes(dem_ctx* ctx, double* mass);

/* Walls in motion (section 3.1: the top plate compresses the sample to its
 * overburden stress before perforation).  dem_read_wall_forces: force[(s *
 * DEM_MAX_WALLS + w) * 3 + c] (N, host or device, n_samples x DEM_MAX_WALLS x 3)
 * is the total force the particles of sample s exert on its wall w at the last
 * force evaluation (the negative of the wall's Hertz contact forces on them,
 * summed in a fixed order); zero for walls a sample does not have.
 * Synchronises.  dem_set_walls: replace the n_walls walls of `sample` (n_walls
 * must equal its current count; the same validation as dem_init), from the
 * next step on.  A wall moves only between calls, and its velocity does not
 * enter the contact law (a quasi-static move, as a servo-controlled plate
 * makes); the neighbour and wall lists are rebuilt at the next step.
 * DEM_E_INVAL for a bad sample, count or wall. */
dem_status dem_read_wall_forces(dem_ctx* ctx, double* force);
dem_status dem_set_walls(dem_ctx* ctx, int32_t sample, int32_t n_walls, const dem_wall* walls);

/* Query: total fluid cells, pair-list size and capacity, rebuild count, and
 * the candidate margin (skin plus the largest pull-off separation) used by
 * the neighbour list of sample 0. */
dem_status dem_info(dem_ctx* ctx, int64_t* ncell, int64_t* n_pairs, int64_t* pair_capacity,
                    int64_t* rebuilds, double* cutoff_margin);

/* Force a neighbour-list rebuild at the start of the next step. */
dem_status dem_request_rebuild(dem_ctx* ctx);

/* Step windows as recorded HIP graphs (enable 1) or direct launches (0, the
 * default).  A window that does not contain the last step of a dem_step call
 * is recorded once per (state buffer, step modulo the coupling interval,
 * length) and replayed; the kernels read the context's state through a device
 * copy refreshed at every call and rebuild, so a recording survives list
 * rebuilds.  Results are identical either way.  Recording is skipped while
 * kernel timing (dem_profile) is on, and abandoned for the context if the
 * runtime refuses it. */
dem_status dem_set_graphs(dem_ctx* ctx, int32_t enable);

/* Lanes of the step kernel that share one particle's neighbour row: 1, 2, 4,
 * 8 or 16; anything else is DEM_E_INVAL.  Until it is called, the pair mode
 * picks it: 2 for DEM_PAIRS_HALF (the row gather), 4 for DEM_PAIRS_FULL_ROWS (the
 * row evaluation).  A tuning knob: forces are summed in a fixed tree within the
 * group, so results differ between settings by rounding only, and are
 * reproducible for each. */
dem_status dem_set_lanes(dem_ctx* ctx, int32_t lanes);

/* How the step evaluates the contact law of a pair (a tuning knob; results
 * are identical bit for bit).  DEM_PAIRS_FULL_ROWS: each particle walks its
 * full neighbour row and evaluates every contact itself, in the pair's
 * canonical orientation, so each pair is evaluated twice and no force record
 * is written (one launch per step).  DEM_PAIRS_HALF: a first launch evaluates
 * every half pair once and writes the force record of each pair in contact
 * (force, n x F_t and rolling torque on the owner); a second adds the records
 * of each particle's row in the same order (two launches per step; the
 * default, faster at 200 000 spheres).  With the same lanes the two modes give
 * bit-identical results.  Anything else is DEM_E_INVAL. */
enum { DEM_PAIRS_FULL_ROWS = 0, DEM_PAIRS_HALF = 1 };
dem_status dem_set_pair_mode(dem_ctx* ctx, int32_t mode);

/* Kernel-class timing with HIP events recorded on the context's stream
 * around every launch of each class (for roofline reporting).  enable = 1
 * starts (and zeroes) the accumulators, 0 stops.  dem_read_profile fills
 * DEM_PROF_N entries: total milliseconds and number of launches of each
 * class since the last enable (host arrays). */
enum { DEM_PROF_PROLOGUE = 0, DEM_PROF_REBUILD = 1, DEM_PROF_FLUID = 2, DEM_PROF_STEP = 3,
       DEM_PROF_N = 4 };
dem_status dem_profile(dem_ctx* ctx, int32_t enable);
dem_status dem_read_profile(dem_ctx* ctx, double* total_ms, int64_t* launches);

/* Latched device fault bits (0: none): 1 pair capacity, 2 non-finite force,
 * 4 a particle moved half the skin or more in one step, 8 a bonded pair was
 * missing from a rebuilt neighbour list, 16 inconsistent rebuild request. */
dem_status dem_read_fault(dem_ctx* ctx, int32_t* bits);

void dem_destroy(dem_ctx* ctx);
const char* dem_status_str(dem_status s);

/* ---- learned closure (an extension of the method; not in the paper) ----
 * A network 6 -> 64 -> 64 -> 64 -> 2 (GELU, erf form) maps per-particle
 * features x = [porosity at the particle, slip speed |u - v|, Re of eq 11,
 * k, mean delta/R* over the pairs of the last force evaluation, their count],
 * normalised as (x - mean) / sd, to y; the factors c = exp(clip(y, -ln 2,
 * ln 2)) in [0.5, 2] multiply the particle's drag force (eq 8: c_drag = c[0])
 * and scale the surface energy of a pair as gamma sqrt(c_i c_j) (c_coh = c[1]).
 * Matrix products run on the matrix cores in BF16 with FP32 accumulation.
 *
 * Parameters: DEM_MLP_NPARAMS FP32 values, W1 6x64 | b1 64 | W2 64x64 | b2 64 |
 * W3 64x64 | b3 64 | W4 64x2 | b4 2, each W[k][m] row-major with k the input.
 * A dem_mlp holds FP32 master parameters, a BF16 copy used by every product,
 * and Adam moments (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected).  It is
 * used on the stream given at creation; not thread-safe.
 *
 * dem_mlp_set_params / get_params: host or device pointer (8898 FP32); set
 *   also zeroes the Adam moments and step count.
 * dem_mlp_forward: x = batch x 6 normalised features (FP32, device), y =
 *   batch x 2 raw outputs (FP32, device).  Asynchronous.
 * dem_mlp_grad: loss L = mean over the batch and both outputs of (y - t)^2
 *   for targets t (batch x 2, FP32, device); writes dL/dparams (8898 FP32, host
 *   or device) and the loss (host, may be NULL).  Synchronises.
 * dem_mlp_train_step: the same gradient, then one Adam step with learning rate
 *   lr > 0 on the master parameters.  Synchronises when loss is not NULL.
 * Errors: DEM_E_INVAL for NULL handles or buffers, batch < 0 or lr <= 0;
 *   DEM_E_NOMEM when the batch buffers cannot grow.
 *
 * dem_set_closure: mlp NULL switches the closure off (factors 1).  Otherwise
 *   the context takes a snapshot of the network's current parameters and
 *   norm = mean[6], sd[6] (host, sd > 0); from the next coupling evaluation on,
 *   every evaluation recomputes the features and factors of every particle
 *   before the drag.  Until then the factors are 1.
 * dem_read_closure: features (n x 6), c_drag, c_coh (n) of the latest
 *   evaluation, in caller order, into host arrays (any may be NULL);
 *   DEM_E_STATE if the closure is off.  Synchronises. */
#define DEM_MLP_NPARAMS 8898
typedef struct dem_mlp dem_mlp;
dem_status dem_mlp_create(dem_mlp** out, int32_t device, void* hip_stream);
void dem_mlp_destroy(dem_mlp* mlp);
dem_status dem_mlp_set_params(dem_mlp* mlp, const float* params);
dem_status dem_mlp_get_params(dem_mlp* mlp, float* params);
dem_status dem_mlp_forward(dem_mlp* mlp, const float* x, float* y, int64_t batch);
dem_status dem_mlp_grad(dem_mlp* mlp, const float* x, const float* t, int64_t batch, float* grad, float* loss);
dem_status dem_mlp_train_step(dem_mlp* mlp, const float* x, const float* t, int64_t batch, float lr, float* loss);
/* dem_mlp_train_step_noalloc: for callers that cannot allocate device memory
 * (code under HIP graph capture, tight training loops, harnesses that forbid
 * hipMalloc).  The same step as dem_mlp_train_step, bit for bit, but its batch
 * buffers (activations, backward signals, chunk partial gradients) live in one
 * static device array of the library, about 6.6 MB per GPU, held by each GPU
 * the library runs on until the process ends; the call itself allocates
 * nothing.  batch must be 1 .. DEM_MLP_NOALLOC_MAX_BATCH, else DEM_E_INVAL
 * (nothing is launched).  Every call on one GPU shares that array: calls that
 * overlap on one GPU (several streams, several networks) race, so callers order
 * them on one stream.  Nothing in the array needs clearing: each call writes
 * every location it reads.  DEM_E_DEVICE if the array's address could not be
 * looked up when the network was created. */
#define DEM_MLP_NOALLOC_MAX_BATCH 4096
dem_status dem_mlp_train_step_noalloc(dem_mlp* mlp, const float* x, const float* t, int64_t batch, float lr,
                                      float* loss);
dem_status dem_set_closure(dem_ctx* ctx, const dem_mlp* mlp, const double* norm);
dem_status dem_read_closure(dem_ctx* ctx, double* features, double* c_drag, double* c_coh);

/* ---- coarse-graining helpers (host only, no device needed) ----
 * dem_cg_material: grain-scale surface energy and drag factor of section 2.4
 * (Table 3: rho, E, nu, e, mu unchanged, gamma x k).
 * dem_cg_diameters: SSW multiplies each fine diameter by k; SSP writes one
 * diameter, k (sum d^3 / n)^(1/3), to every output.  n_fine inputs, n_out
 * outputs (SSW: n_out <= n_fine, the first n_out are used). */
dem_status dem_cg_material(const dem_params* fine, double* gamma_grain, double* drag_factor);
dem_status dem_cg_diameters(int32_t scheme, double k, const double* d_fine, int64_t n_fine,
                            double* d_out, int64_t n_out);
/* eq 37-38 Rayleigh time step with G = E / (2 (1 + nu)). */
double dem_rayleigh_dt(double radius, double rho, double E, double nu);

#ifdef __cplusplus
}
#endif
#endif
