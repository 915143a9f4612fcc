/*
 * sdpdem_oracle.h -- plain FP64 CPU reference of the SDPD-DEM per-step path.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the oracle that the GPU library is
 * checked against.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it; the product path never does.
 * It shares no source, header, table or helper with the GPU library.
 *
 * What it computes follows Tsuzuki, "DEMocritus: an open source framework
 * for simulating slurry flows using an SDPD-DEM coupled model" (arXiv
 * 2002.03120): the governing equation (Eq. govern), the SDPD pair forces
 * (Eqs. FijC, FijD, FijR, FijT with the Lucy kernel, Eqs. kernel and F),
 * the density summation and equation of state (Eqs. compdens, prtcpres),
 * the DEM spring-dashpot contact (Eqs. dem_fnij .. slideref, deminputA ..
 * deminputF), lubrication (Eq. lubri), the fluid-particle coupling
 * (Eqs. F_fpi_PG, F_fpi_DG, beta, F_fpi_DG_reac, fvfdef) and the
 * two-pass velocity-Verlet loop of Algorithms 1 and 2 (Sec. 3.3).
 * Every reading taken where the paper is silent or garbled is stated
 * beside the code that implements it.
 *
 * Parity unpinned: the pressure filter (a Shepard mean, pinned only by its
 * own properties, since the paper gives no formula), the tangential
 * history rules beyond the stick and slide cases, and lubrication between
 * spheres of unequal radii.  Everything else is checked by the tests
 * against closed forms, brute force, invariants or the paper's values.
 *
 * Conventions: host memory only, synchronous, every array in id order
 * (the ids must be a permutation of 0..n-1).  Return 0 on success and a
 * negative ORACLE_E_* code on failure.
 */
#ifndef SDPDEM_ORACLE_H
#define SDPDEM_ORACLE_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ORACLE_OK = 0,
  ORACLE_E_INVALID_ARG = -1,
  ORACLE_E_NBR_OVERFLOW = -3,
  ORACLE_E_CONTACT_OVERFLOW = -4,
  ORACLE_E_NONFINITE = -5,
  ORACLE_E_OUT_OF_DOMAIN = -6,
  ORACLE_E_NOMEM = -8
};

/* particle types (Sec. 2.5 boundary treatment; Sec. 3.2 output types) */
enum { O_FLUID = 0, O_RIGID = 1, O_INNER_WALL = 2, O_OUTER_WALL = 3 };

/* parameter set; names follow the command-line table of Sec. 3.2 */
typedef struct oracle_params {
  double org[3];            /* --orgx/y/z: lower corner of the domain          */
  double L[3];              /* --Lx/y/z: domain size                            */
  int32_t periodic[3];      /* --periodic_type as one flag per axis             */
  int32_t noslip;           /* --slipcond_type: 1 no-slip, 0 slip               */
  double dx;                /* --dx: initial lattice spacing                    */
  double h;                 /* --h: kernel support (cut-off) radius             */
  double rho0, p0, alpha, beta_eos; /* --dens0 --pres0 --alpha --beta           */
  double eta, xi, kBT;      /* --eta --xi --kBT                                 */
  double dt;                /* --dt                                             */
  double g[3], f[3];        /* --gx.. and --fx.. (both accelerations)           */
  int32_t gravity_type;     /* 0: uniform; 1: sign reversed in the lower half   */
  int32_t gravity_axis;     /* axis that splits the two halves                  */
  double coeff_c, coeff_d, coeff_r, coeff_t; /* --Coeff_fcij .. --Coeff_ftij    */
  double E_dem, nu_dem, mu_fric;             /* Young modulus, Poisson, friction */
  double dem_damping;       /* multiplier on c_n and c_t (1 = the paper)        */
  double mass_fluid, inertia_fluid;          /* --mass --iner                   */
  int32_t enable_kernel_norm, enable_pres_smooth, enable_neg_p_clamp, enable_lub;
  double eps_min;           /* lower clamp of the fluid volume fraction         */
  double lub_gap_min;       /* regulariser of the lubrication singularity       */
  int64_t itr_start;        /* --itr_start                                      */
  int64_t itr_actv_rigid;   /* --itr_actv_rigid                                 */
  uint64_t seed;            /* key of the counter-based generator               */
  int32_t max_neighbors, max_contacts;
  /* Lees-Edwards shear rate (0: plain periodic images).  Non-zero needs all
   * three axes periodic: flow along x, gradient along z; the image of the
   * box above is shifted by shear_rate L_z t in x and moves with
   * +shear_rate L_z in x. */
  double shear_rate;
} oracle_params;

typedef struct oracle_system oracle_system;

/* fields readable with oracle_read_field (n rows, comps doubles per row) */
enum {
  OF_POS = 0, OF_VEL, OF_ANGVEL, OF_DENS, OF_PRES, OF_PRES_SMOOTH,
  OF_F_SDPD, OF_F_CD, OF_N_SDPD, OF_F_DG, OF_F_PG, OF_F_RXN,
  OF_F_DEM, OF_F_LUB, OF_N_DEM, OF_F_TOTAL, OF_N_TOTAL, OF_EPS,
  /* per-particle sums of pair-term magnitudes, used to scale tolerances */
  OF_F_SDPD_ABS = 32, OF_F_CD_ABS, OF_N_SDPD_ABS, OF_F_DG_ABS, OF_F_PG_ABS,
  OF_F_RXN_ABS, OF_F_DEM_ABS, OF_F_LUB_ABS, OF_N_DEM_ABS
};

int oracle_field_comps(int field);

int oracle_create(const oracle_params* p, int64_t n, const int64_t* id,
                  const uint8_t* type, const double* pos, const double* vel,
                  const double* angvel, const double* mass,
                  const double* inertia, const double* radius,
                  oracle_system** out);
void oracle_destroy(oracle_system* s);

/* Algorithm 1: nsteps iterations, two velocity-Verlet passes each */
int oracle_step(oracle_system* s, int64_t nsteps);
/* one evaluation of every force at the current state, no update */
int oracle_compute_forces(oracle_system* s);
int oracle_read_field(oracle_system* s, int field, double* dst);
/* neighbour sets as CSR by id, columns ascending (outer walls: empty) */
int oracle_read_neighbors(oracle_system* s, int64_t* row_ptr, int32_t* cols,
                          int64_t cap, int64_t* nnz);
/* rigid contact table: pairs (i<j) and the tangential displacement of i */
int oracle_read_contacts(oracle_system* s, int32_t* pairs, double* delta_t,
                         int64_t cap, int64_t* n_contacts);
int oracle_load_contacts(oracle_system* s, const int32_t* pairs,
                         const double* delta_t, int64_t n_contacts);
int oracle_totals(oracle_system* s, double out[16]);
int64_t oracle_get_step(const oracle_system* s);
/* pressure tensor P_ab (row-major 3x3) of the box: kinetic part from the
 * current velocities (peculiar to the Lees-Edwards profile), virial of the
 * pair forces of the last force evaluation, divided by the box volume */
int oracle_stress(oracle_system* s, double out[9]);
int oracle_num_threads(void);
void oracle_set_num_threads(int n);

/* ---- pure functions, exported so that the tests can pin them ---------- */
double oracle_lucy_w(double r, double h);   /* Eq. kernel                 */
double oracle_lucy_f(double r, double h);   /* Eq. F = -W'(r)/r           */
double oracle_lattice_w_sum(double h, double dx); /* sum_k W(|k| dx)     */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                          uint32_t out[4]);
/* the four standard normals of the pair (a,b) at a given step: three for
 * the thermal force across e_ij, one along it */
void oracle_pair_normals(uint64_t seed, int64_t id_a, int64_t id_b,
                         int64_t step, double z[4]);
/* F^C, F^D, F^R, F^T of one pair, r_ij = xi - xj (already minimum image);
 * d_i, d_j are number densities rho/m_f; ps_* smoothed pressures */
void oracle_pair_force(const oracle_params* p, const double rij[3],
                       const double vi[3], const double vj[3],
                       const double wi[3], const double wj[3], double di,
                       double dj, double psi, double psj, int64_t idi,
                       int64_t idj, int64_t step, double fc[3], double fd[3],
                       double fr[3], double ft[3]);
/* momentum-exchange coefficient beta/(1-eps) of Eq. beta (cancelled form) */
double oracle_drag_b(double eps, double dv_abs, double d, double rho,
                     double mu);
/* one DEM contact evaluation of Sec. 2.2 for a rigid pair (i,j); dij is the
 * minimum-image x_i - x_j, dt_in the stored tangential displacement */
void oracle_dem_pair(const oracle_params* p, const double dij[3],
                     const double vi[3], const double vj[3],
                     const double wi[3], const double wj[3], double Ri,
                     double Rj, double mi, double mj, const double dt_in[3],
                     double fn[3], double ft[3], double dt_out[3],
                     int* sliding);

#ifdef __cplusplus
}
#endif
#endif
