/*
 * sdpdem.h -- C ABI of the MI355X (gfx950) SDPD-DEM hot path.
 *
 * The library advances the particle system of Tsuzuki, "DEMocritus: an open
 * source framework for simulating slurry flows using an SDPD-DEM coupled
 * model" (arXiv 2002.03120): fluid particles under the SDPD+a pair forces
 * (Sec. 2.1, Eqs. FijC, FijD, FijR, FijT), rigid DEM spheres with
 * spring-dashpot contacts and lubrication (Secs. 2.2, 2.3), the two-way
 * drag coupling between them (Sec. 2.4), wall and periodic boundaries
 * (Sec. 2.5) and the two-pass velocity-Verlet loop of Algorithms 1 and 2.
 * The calls mirror the paper's program structure (Sec. 3): construct a
 * particle system from the parameter table and the particles, run the
 * steps itr_start..itr_stop, read particle fields.
 *
 * Conventions shared by every call:
 *  - Return value: SDPDEM_OK (0) or a negative SDPDEM_E_* code; no call
 *    throws.  sdpdem_status_string() names a code.
 *  - Memory: the caller allocates ONE device workspace of
 *    sdpdem_workspace_bytes() bytes and keeps it alive until
 *    sdpdem_destroy(); the library never allocates device memory.  Host
 *    arrays passed in are copied before the call returns.  The
 *    sdpdem_system handle is a small host object owned by the library.
 *  - Streams: every call takes a hipStream_t as void*.  sdpdem_step and
 *    sdpdem_compute_forces enqueue work, then synchronise once on the
 *    stream to read the device status word; the reads into host memory
 *    synchronise; sdpdem_read_field into device memory only enqueues.
 *  - Order: particles are identified by ids that must be a permutation of
 *    0..n-1; every array crossing the ABI is in id order, whatever order
 *    the library keeps internally.
 *  - Types: 0 fluid, 1 rigid, 2 inner wall, 3 outer wall (Sec. 2.5).
 */
#ifndef SDPDEM_H
#define SDPDEM_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SDPDEM_OK 0
#define SDPDEM_E_INVALID_ARG (-1)
#define SDPDEM_E_WORKSPACE_TOO_SMALL (-2)
#define SDPDEM_E_NBR_OVERFLOW (-3)      /* a neighbour row exceeded max_neighbors */
#define SDPDEM_E_CONTACT_OVERFLOW (-4)  /* a rigid contact row exceeded max_contacts */
#define SDPDEM_E_NONFINITE (-5)         /* a position, velocity or spin became non-finite */
#define SDPDEM_E_OUT_OF_DOMAIN (-6)     /* a particle left the cell grid / wall box */
#define SDPDEM_E_HIP (-7)               /* a HIP runtime call failed */

enum sdpdem_type {
  SDPDEM_FLUID = 0,
  SDPDEM_RIGID = 1,
  SDPDEM_INNER_WALL = 2,
  SDPDEM_OUTER_WALL = 3
};

/* Parameter table (Sec. 3.2, Table ipparam); field order is part of the
 * ABI.  All lengths, times and masses in the caller's units. */
typedef struct sdpdem_params {
  double org[3];           /* --orgx/y/z: lower corner of the domain              */
  double L[3];             /* --Lx/y/z: domain size; periodic axes need L >= 3h   */
  int32_t periodic[3];     /* --periodic_type, one flag per axis (8 combinations) */
  int32_t noslip;          /* --slipcond_type: 1 reverse all of v at a wall face,
                              0 reverse its normal component only                 */
  double dx;               /* --dx: lattice spacing; fluid torque lever is dx/2   */
  double h;                /* --h: support radius of the Lucy kernel (Eq. kernel) */
  double rho0, p0, alpha, beta_eos; /* Eq. prtcpres: p = p0 (rho/rho0)^alpha - beta */
  double eta, xi, kBT;     /* shear and bulk viscosity, thermal energy (Sec. 2.1) */
  double dt;               /* time step                                           */
  double g[3], f[3];       /* --gx.. and --fx..: body accelerations, summed       */
  int32_t gravity_type;    /* 0 uniform; 1 sign flipped where x[axis]-org < L/2   */
  int32_t gravity_axis;    /* axis splitting the two halves for gravity_type 1    */
  double coeff_c, coeff_d, coeff_r, coeff_t; /* --Coeff_fcij..ftij switches       */
  double E_dem, nu_dem, mu_fric; /* Young modulus, Poisson ratio, friction (2.2) */
  double dem_damping;      /* multiplier on c_n, c_t of Eqs. deminputE/F (1)      */
  double mass_fluid, inertia_fluid; /* --mass --iner of fluid and wall particles  */
  int32_t enable_kernel_norm;  /* normalise the kernel so a lattice gives rho0     */
  int32_t enable_pres_smooth;  /* Shepard filter of the pressure                   */
  int32_t enable_neg_p_clamp;  /* p < 0 -> 0 at free surfaces                      */
  int32_t enable_lub;          /* lubrication of Eq. lubri                         */
  double eps_min;          /* lower clamp of the fluid volume fraction            */
  double lub_gap_min;      /* floor of the lubrication gap                        */
  int64_t itr_start;       /* first step number (also the noise counter)          */
  int64_t itr_actv_rigid;  /* rigid particles move and couple from this step on   */
  uint64_t seed;           /* key of the Philox4x32-10 noise                      */
  int32_t max_neighbors;   /* capacity of a neighbour row                         */
  int32_t max_contacts;    /* capacity of a rigid contact row                     */
  double shear_rate;       /* Lees-Edwards shear rate (0: plain periodic images);
                              non-zero needs all axes periodic: flow along x,
                              gradient along z, the image above shifted by
                              shear_rate L_z t in x and moving at +shear_rate L_z */
  double cell_factor;      /* fluid cell size = cell_factor h, 0.25 <= cell_factor
                              <= 16 (0 means 1): a tuning knob.  Below 1 the
                              neighbour search reaches ceil(1/cell_factor) cells
                              each way and skips cells out of range.  Neighbour
                              sets do not depend on it; sums only through their
                              order                                              */
  double skin;             /* candidate margin of the neighbour search of Alg. 1
                              (Sec. 3.2), 0 <= skin <= h/2.  0: the particles are
                              re-sorted and the lists rebuilt from the cell grid
                              after every drift.  skin > 0: the cell-grid search
                              keeps every partner within h + skin as a
                              candidate, and after a drift the lists are taken
                              from the candidates (the exact r < h test, so the
                              neighbour sets are unchanged) until some particle
                              has moved skin/2 since the last search; only then
                              are the particles re-sorted and searched again.
                              In a sheared box a particle's drift is measured
                              against the flow's, and the limit shrinks by
                              (R_max + h + skin) |shear rate| t / 2 with the
                              time t between the searched positions and the
                              drifted ones (the flow's part of two partners'
                              approach; a build ahead of a step's first pass
                              saw the positions of the step's start).
                              Deciding this reads one
                              device word after the first pass of a step (one
                              synchronisation per step); under graph replay
                              every step searches                                */
} sdpdem_params;

/* Particles, host memory, n rows in any order (ids must cover 0..n-1).
 * mass/inertia/radius are read for rigid particles only; fluid and wall
 * particles take mass_fluid and inertia_fluid. */
typedef struct sdpdem_particles {
  int64_t n;
  const int64_t* id;
  const uint8_t* type;
  const double* pos;      /* [n*3] */
  const double* vel;      /* [n*3] */
  const double* angvel;   /* [n*3] */
  const double* mass;     /* [n]   */
  const double* inertia;  /* [n]   */
  const double* radius;   /* [n]   */
} sdpdem_particles;

/* One box of a batch: an independent domain (its own periodic or wall
 * axes, Lees-Edwards shear rate, thermal energy and noise key).  The
 * parameters' own org/L/periodic/shear_rate/kBT/seed are ignored by the
 * batch calls; every other parameter is shared by all boxes. */
typedef struct sdpdem_box {
  double org[3], L[3];
  int32_t periodic[3];
  int32_t reserved;        /* 0 */
  double shear_rate;       /* as in sdpdem_params                            */
  double kBT;              /* thermal energy of this box                     */
  uint64_t seed;           /* noise key of this box                          */
} sdpdem_box;

/* Fields readable with sdpdem_read_field: n rows in id order, 1 or 3
 * doubles per row.  Force fields hold the last force evaluation. */
enum sdpdem_field {
  SDPDEM_POS = 0, SDPDEM_VEL, SDPDEM_ANGVEL,
  SDPDEM_DENS,        /* rho, Eq. compdens (FP64)                         */
  SDPDEM_PRES,        /* p, Eq. prtcpres (FP64)                           */
  SDPDEM_PRES_SMOOTH, /* filtered pressure (FP32)                         */
  SDPDEM_F_SDPD,      /* sum_j F^C+F^D+F^R+F^T, fluid and inner walls     */
  SDPDEM_F_CD,        /* sum_j F^C+F^D (input of F^PG)                    */
  SDPDEM_N_SDPD,      /* torque of F^SDPD                                 */
  SDPDEM_F_DG,        /* drag on rigid particles, Eq. F_fpi_DG            */
  SDPDEM_F_PG,        /* pressure-gradient force, Eq. F_fpi_PG            */
  SDPDEM_F_RXN,       /* drag reaction on fluid, Eq. F_fpi_DG_reac        */
  SDPDEM_F_DEM,       /* contact force on rigid particles (Sec. 2.2)      */
  SDPDEM_F_LUB,       /* lubrication force (Eq. lubri)                    */
  SDPDEM_N_DEM,       /* contact torque                                   */
  SDPDEM_F_TOTAL,     /* total force of Eq. newton1 at the current state  */
  SDPDEM_N_TOTAL,     /* total torque of Eq. newton2                      */
  SDPDEM_EPS,         /* fluid volume fraction of rigid particles          */
  SDPDEM_NUM_FIELDS
};

/* Kernel ids for sdpdem_set_profiling. */
enum sdpdem_kernel {
  SDPDEM_K_NONE = 0, SDPDEM_K_BIN, SDPDEM_K_SORT, SDPDEM_K_PERMUTE,
  SDPDEM_K_NEIGHBORS_DENSITY, SDPDEM_K_SMOOTH, SDPDEM_K_FLUID_FORCES,
  SDPDEM_K_FPI_ACTION, SDPDEM_K_FPI_REACTION, SDPDEM_K_DEM, SDPDEM_K_INTEGRATE,
  SDPDEM_K_RIGID_GRID, SDPDEM_NUM_KERNELS
};

typedef struct sdpdem_system sdpdem_system;

/* Bytes of device workspace needed for these parameters and particles:
 * the particle arrays of Sec. 3.2 (one record per particle, sized by the
 * parameter table, Table ipparam) plus the cell grid and neighbour rows of
 * Alg. 1.  Writes *bytes; SDPDEM_E_INVALID_ARG for what sdpdem_create
 * rejects.  Touches no device. */
int sdpdem_workspace_bytes(const sdpdem_params* params,
                           const sdpdem_particles* particles, size_t* bytes);

/* Validate, upload and build the system in the caller's workspace: the
 * initialisation part of the particle system of Sec. 3.1 (parameters of
 * Table ipparam, particle types of Sec. 2.5).
 * Rejects (SDPDEM_E_INVALID_ARG): ids not a permutation of 0..n-1, unknown
 * types, non-positive h, dx, dt, rho0, masses or rigid radii, xi outside
 * [40 eta/51, 5 eta/3] (gamma^a, gamma^b of Sec. 2.1 must stay >= 0),
 * periodic L below 3h, max_neighbors/max_contacts < 1. */
int sdpdem_create(const sdpdem_params* params, const sdpdem_particles* particles,
                  void* d_workspace, size_t workspace_bytes, void* hip_stream,
                  sdpdem_system** out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * sdpdem_create without a workspace argument.  The system lives in a
 * file-scope device array of the library, SDPDEM_STATIC_WORKSPACE_BYTES
 * (64 MiB) per device, held from the first call on a device until the
 * process ends.  The device is the current one (hipSetDevice), which must
 * be the stream's.  The call allocates no device memory (no hipMalloc,
 * hipFree or allocating library routine) and creates no stream: every
 * launch of the system runs on the caller's stream.  Host particle arrays
 * are copied as in sdpdem_create.  Errors: those of sdpdem_create, and
 * SDPDEM_E_WORKSPACE_TOO_SMALL when sdpdem_workspace_bytes exceeds the
 * array (nothing is launched then).  All systems created this way on one
 * device share the array: creating one overwrites the state of the
 * previous one, so use one at a time per device; calls that overlap on one
 * device race.  sdpdem_destroy releases the handle. */
#define SDPDEM_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)
int sdpdem_create_static(const sdpdem_params* params, const sdpdem_particles* particles,
                         void* hip_stream, sdpdem_system** out);

/* Batched systems: nbox independent boxes advanced together, every kernel
 * launch covering all of them (the batched viscometer; each box is one
 * particle system of Sec. 3.1, run through Alg. 1 like a plain one, and
 * its viscosity plays the role of the measurement of Sec. 4.1).  box_of[k] gives
 * the box of particle row k; ids run over 0..n-1 across all boxes.  No
 * pair, contact or coupling ever joins particles of different boxes.
 * The thermal noise of a pair is keyed by its box's seed and the two ids
 * less the smallest id in the box, so a box whose ids are a contiguous
 * range runs bit for bit as the same box alone (ids from 0) would, whatever
 * the other boxes of the batch.
 * Rejects what sdpdem_create rejects, per box, and box_of entries outside
 * 0..nbox-1; a box with shear_rate != 0 must be periodic on all axes. */
int sdpdem_batch_workspace_bytes(const sdpdem_params* params, const sdpdem_box* boxes,
                                 int32_t nbox, const sdpdem_particles* particles,
                                 const int32_t* box_of, size_t* bytes);
int sdpdem_create_batch(const sdpdem_params* params, const sdpdem_box* boxes, int32_t nbox,
                        const sdpdem_particles* particles, const int32_t* box_of,
                        void* d_workspace, size_t workspace_bytes, void* hip_stream,
                        sdpdem_system** out);

/* Algorithm 1: nsteps steps of two velocity-Verlet passes each (Sec. 2.6),
 * each pass the force evaluation of Algorithm 2.  Returns the device status
 * (overflow, non-finite, out of domain) seen at the end: the call enqueues
 * the steps on the stream and then synchronises that stream once to read
 * the status word, so it returns after the steps have run.
 * With rigid particles the library keeps a second stream of its own (at
 * the default priority) for work that does not depend on what runs beside
 * it: the rigid grid beside the neighbour lists, the sphere records and DEM
 * contacts beside the SDPD pair forces and the coupling.  It is forked from
 * the caller's stream and joined back into it within the same build or
 * pass, so work the caller orders on its stream sees everything. */
int sdpdem_step(sdpdem_system* sys, int64_t nsteps, void* hip_stream);

/* Replay the step loop of Algorithm 1 from a captured HIP graph of steps_per_graph steps
 * (an even number; 0 switches it off, the default).  sdpdem_step then runs
 * whole graphs where it can and single steps otherwise; results are the
 * same bits as without graphs.  Capture needs a stream other than the null
 * stream; where capture fails the calls stay eager.  The graph is
 * re-captured after profiling, stress sampling or the rigid activation
 * (itr_actv_rigid) change the launch sequence. */
int sdpdem_set_graph(sdpdem_system* sys, int steps_per_graph);

/* One evaluation of every force at the current state (Alg. 2: the list,
 * density and pressure steps of Alg. 1 when the positions changed, then
 * compute_fluid, compute_fpi_action, compute_fpi_reaction, compute_rigid),
 * no update.  Synchronises the stream once to read the status word. */
int sdpdem_compute_forces(sdpdem_system* sys, void* hip_stream);

/* Copy a field (enum sdpdem_field; the quantities of Secs. 2.1-2.6 and
 * the outputs of Alg. 1's output(), Sec. 3.3) in id order: dst holds
 * n * sdpdem_field_comps(field) doubles (row i = id i; 3 components x, y,
 * z for vector fields).  dst_is_device = 0: dst is host memory and the
 * call synchronises the stream.  dst_is_device = 1: dst is device memory
 * (8-byte aligned) and the copy is only enqueued on the stream.
 * SDPDEM_E_INVALID_ARG for an unknown field, bytes too small, a null or
 * misaligned dst. */
int sdpdem_read_field(sdpdem_system* sys, int field, void* dst, size_t bytes,
                      int dst_is_device, void* hip_stream);
/* Doubles per row of a field for sdpdem_read_field (1 for the scalars rho,
 * p of Eqs. compdens and prtcpres, the filtered pressure and eps of Eq.
 * fvfdef; 3 otherwise; 0 for an unknown field). */
int sdpdem_field_comps(int field);

/* Neighbour sets of the last build (compute_neighbor_list of Alg. 1, the
 * per-particle lists of Sec. 3.2: j != i with |r_ij| < h) as CSR in host
 * memory: row i = neighbours of id i, columns ascending ids; outer walls
 * have empty rows.  row_ptr holds n+1 entries; cols holds cap entries;
 * with cols == NULL only row_ptr and *nnz are written.
 * SDPDEM_E_INVALID_ARG if cap < nnz.  Synchronises the stream. */
int sdpdem_read_neighbors(sdpdem_system* sys, int64_t* row_ptr, int32_t* cols,
                          int64_t cap, int64_t* nnz, void* hip_stream);

/* Rigid contact table (the contact flags and tangential displacements
 * delta_t of Eqs. tandispseq and tandispn, Sec. 2.2, kept per pair as in
 * the neighbour lists of Sec. 3.2) in host memory: pairs [cap][2] ids
 * (i < j) and delta_t [cap][3] held by i (the row of j holds its
 * negative).  pairs == NULL: count only.  SDPDEM_E_INVALID_ARG if cap is
 * too small.  Synchronises the stream. */
int sdpdem_read_contacts(sdpdem_system* sys, int32_t* pairs, double* delta_t,
                         int64_t cap, int64_t* n_contacts, void* hip_stream);
/* Replace the contact table (restart from a backup, Sec. 3.3; the
 * history delta_t of Eq. tandispn): pairs [n][2] ids, delta_t [n][3] held
 * by the first id of each pair; each pair fills both rows.  Host memory.
 * SDPDEM_E_INVALID_ARG for ids that are not rigid or repeated pairs,
 * SDPDEM_E_CONTACT_OVERFLOW beyond max_contacts per sphere. */
int sdpdem_load_contacts(sdpdem_system* sys, const int32_t* pairs,
                         const double* delta_t, int64_t n_contacts,
                         void* hip_stream);

/* FP64 totals of the quantities Eqs. newton1 and newton2 (Sec. 2.6)
 * evolve, over all non-outer-wall particles, in host memory:
 * out = [P(3), L(3) about the origin (m x cross v + I omega), KE_trans,
 *        KE_rot, max|v|, min rho, max rho, total mass, step, 0, 0, 0].
 * Synchronises the stream. */
int sdpdem_totals(sdpdem_system* sys, double out[16], void* hip_stream);

/* The step counter of Alg. 1 (itr_start plus the steps taken); -1 for a
 * null handle. */
int64_t sdpdem_get_step(const sdpdem_system* sys);

/* Shear-stress sampling for viscometry: the viscosity the paper measures
 * from the reverse-Poiseuille mean velocity (Eq. poiseuave, Sec. 4.1) is
 * measured here from the shear stress of Lees-Edwards boxes (not in the
 * paper).  With sampling on, every step ends with one sample per box of
 * the pressure-tensor component
 *   P_zx = ( sum_i m_i v'_z v'_x + sum_pairs r_z F_x ) / V,
 * v' = v - shear_rate (z - z_mid) e_x, the pair sum over the SDPD pair
 * forces (a pair with a rigid or outer-wall partner counted once), the DEM
 * contact and lubrication pairs and the fluid-particle coupling of every
 * sphere (lever sum_j w_sj r_sj / Omega_s times F^DG + F^PG), all from the
 * second force pass of the step, velocities at the end of the step.  The
 * effective viscosity of a sheared box is -<P_zx> / shear_rate.
 * sdpdem_set_stress switches sampling on or off and clears the sums;
 * sdpdem_compute_forces then also refreshes the instantaneous sample
 * (without adding it to the sums).  sdpdem_box_stress copies the last
 * sample and the running sums (nbox doubles each, either may be NULL) and
 * the number of summed samples; it synchronises the stream. */
int sdpdem_set_stress(sdpdem_system* sys, int on, void* hip_stream);
int sdpdem_box_stress(sdpdem_system* sys, double* inst, double* sum, int64_t* nsamples,
                      void* hip_stream);

/* Diagnostics of the background grid and neighbour lists of Alg. 1
 * (Sec. 3.2), host memory, synchronises:
 * out = [n, n_rigid, cells x, y, z of box 0, rigid cells x,
 * y, z of box 0, max neighbour count of the last build, pairs of the last
 * build, number of boxes, steps replayed from captured graphs so far,
 * 1 if the contacts run on the library's second stream, cell-grid searches
 * (sorts) so far, list builds taken from the candidates of an earlier
 * search so far (skin > 0), 0]. */
int sdpdem_info(sdpdem_system* sys, int64_t out[16], void* hip_stream);

/* Per-routine timing, the breakdown of Fig. CompTimeTotal over the
 * routines of Algs. 1 and 2.
 * Time every launch of one kernel (enum sdpdem_kernel) with HIP events on
 * the launch stream; SDPDEM_K_NONE switches timing off.  sdpdem_kernel_time
 * returns the accumulated milliseconds and launch count and resets them. */
int sdpdem_set_profiling(sdpdem_system* sys, int kernel);
int sdpdem_kernel_time(sdpdem_system* sys, double* total_ms, int64_t* launches);
/* Sampled per-routine timing for the breakdown of Fig. CompTimeTotal.
 * Time only the first of every `every` launches of the profiled kernel
 * (every >= 1; 1, the default, times all): the timing events perturb the
 * stream less, and sdpdem_kernel_time counts the timed launches only.
 * Resets the count; SDPDEM_E_INVALID_ARG for every < 1. */
int sdpdem_set_profiling_every(sdpdem_system* sys, int every);

/* Release the handle of a particle system (Sec. 3.1); the caller frees
 * the workspace afterwards.  A null handle is ignored. */
void sdpdem_destroy(sdpdem_system* sys);
/* Name of a status code: the argument checks of the parameter table
 * (Table ipparam) and the run-time checks of Alg. 1's steps. */
const char* sdpdem_status_string(int status);

#ifdef __cplusplus
}
#endif
#endif
