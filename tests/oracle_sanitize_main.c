/*
 * Test driver for the oracle under AddressSanitizer and UndefinedBehavior-
 * Sanitizer (host code only, built with gcc by test_oracle_sanitize.py).
 * It walks every entry point of the oracle over small systems that reach
 * each branch of the method: walls with inner and outer layers, periodic
 * axes, a Lees-Edwards box, thermal noise, rigid spheres in contact and
 * within lubrication range, contact export and restart, the stress tensor,
 * and the error paths.  Exit status 0 means every call returned what it
 * should; a sanitizer report aborts with a non-zero status.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "sdpdem_oracle.h"

#define CHECK(cond)                                                  \
  do {                                                               \
    if (!(cond)) {                                                   \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
      exit(3);                                                       \
    }                                                                \
  } while (0)

static oracle_params base(void) {
  oracle_params p;
  memset(&p, 0, sizeof p);
  for (int a = 0; a < 3; ++a) {
    p.L[a] = 8.0;
    p.periodic[a] = 1;
  }
  p.noslip = 1;
  p.dx = 1.0;
  p.h = 1.5;
  p.rho0 = 1.0;
  p.p0 = 1.0;
  p.alpha = 7.0;
  p.beta_eos = 1.0;
  p.eta = 0.1;
  p.xi = 2.0 / 21.0;
  p.kBT = 1e-3;
  p.dt = 1e-3;
  p.coeff_c = p.coeff_d = p.coeff_r = p.coeff_t = 1.0;
  p.E_dem = 7881.0;
  p.nu_dem = 0.3;
  p.mu_fric = 0.3;
  p.dem_damping = 1.0;
  p.mass_fluid = 1.0;
  p.inertia_fluid = 0.1;
  p.enable_kernel_norm = 1;
  p.enable_pres_smooth = 1;
  p.enable_lub = 1;
  p.eps_min = 0.2;
  p.lub_gap_min = 0.01;
  p.max_neighbors = 64;
  p.max_contacts = 16;
  p.gravity_axis = 2;
  return p;
}

typedef struct {
  int64_t n;
  int64_t* id;
  uint8_t* type;
  double *pos, *vel, *w, *m, *I, *R;
} parts;

static parts make_lattice(int nx, int ny, int nz, int wall_z, uint64_t seed) {
  parts q;
  int64_t nmax = (int64_t)nx * ny * (nz + 6);
  q.id = calloc((size_t)nmax, sizeof(int64_t));
  q.type = calloc((size_t)nmax, 1);
  q.pos = calloc((size_t)nmax * 3, sizeof(double));
  q.vel = calloc((size_t)nmax * 3, sizeof(double));
  q.w = calloc((size_t)nmax * 3, sizeof(double));
  q.m = calloc((size_t)nmax, sizeof(double));
  q.I = calloc((size_t)nmax, sizeof(double));
  q.R = calloc((size_t)nmax, sizeof(double));
  int64_t k = 0;
  uint64_t s = seed * 2654435761u + 1;
  int zlo = wall_z ? -3 : 0, zhi = wall_z ? nz + 3 : nz;
  for (int z = zlo; z < zhi; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        int depth = z < 0 ? -z : (z >= nz ? z - nz + 1 : 0);
        q.id[k] = k;
        q.type[k] = depth == 0 ? O_FLUID : (depth == 1 ? O_INNER_WALL : O_OUTER_WALL);
        q.pos[3 * k] = x + 0.5;
        q.pos[3 * k + 1] = y + 0.5;
        q.pos[3 * k + 2] = z + 0.5;
        for (int a = 0; a < 3 && depth == 0; ++a) {
          s = s * 6364136223846793005ull + 1442695040888963407ull;
          q.vel[3 * k + a] = ((double)(s >> 11) / 9007199254740992.0 - 0.5) * 0.05;
        }
        q.m[k] = 1.0;
        q.I[k] = 0.1;
        q.R[k] = 0.5;
        ++k;
      }
  q.n = k;
  return q;
}

static void free_parts(parts* q) {
  free(q->id);
  free(q->type);
  free(q->pos);
  free(q->vel);
  free(q->w);
  free(q->m);
  free(q->I);
  free(q->R);
}

static void make_rigid(parts* q, int64_t k, double R, const double* x, const double* v) {
  double vs = 4.0 / 3.0 * M_PI * R * R * R;
  q->type[k] = O_RIGID;
  q->R[k] = R;
  q->m[k] = 2.5 * vs;
  q->I[k] = 0.4 * 2.5 * vs * R * R;
  for (int a = 0; a < 3; ++a) {
    q->pos[3 * k + a] = x[a];
    q->vel[3 * k + a] = v[a];
  }
}

static void exercise(oracle_system* s, int64_t n, int steps) {
  CHECK(oracle_step(s, steps) == ORACLE_OK);
  CHECK(oracle_compute_forces(s) == ORACLE_OK);
  double* buf = malloc(sizeof(double) * 3 * (size_t)n);
  for (int f = 0; f <= OF_EPS; ++f) CHECK(oracle_read_field(s, f, buf) == ORACLE_OK);
  for (int f = OF_F_SDPD_ABS; f <= OF_N_DEM_ABS; ++f)
    CHECK(oracle_read_field(s, f, buf) == ORACLE_OK);
  for (int a = 0; a < 3 * n; ++a) CHECK(isfinite(buf[a]));
  free(buf);
  int64_t nnz = 0;
  int64_t* rp = malloc(sizeof(int64_t) * (size_t)(n + 1));
  CHECK(oracle_read_neighbors(s, rp, NULL, 0, &nnz) == ORACLE_OK);
  int32_t* cols = malloc(sizeof(int32_t) * (size_t)(nnz + 1));
  CHECK(oracle_read_neighbors(s, rp, cols, nnz, &nnz) == ORACLE_OK);
  free(cols);
  free(rp);
  int64_t nc = 0;
  CHECK(oracle_read_contacts(s, NULL, NULL, 0, &nc) == ORACLE_OK);
  int32_t* pairs = malloc(sizeof(int32_t) * 2 * (size_t)(nc + 1));
  double* dts = malloc(sizeof(double) * 3 * (size_t)(nc + 1));
  CHECK(oracle_read_contacts(s, pairs, dts, nc, &nc) == ORACLE_OK);
  CHECK(oracle_load_contacts(s, pairs, dts, nc) == ORACLE_OK);
  free(pairs);
  free(dts);
  double tot[16], st[9];
  CHECK(oracle_totals(s, tot) == ORACLE_OK);
  CHECK(oracle_stress(s, st) == ORACLE_OK);
  CHECK(oracle_get_step(s) >= steps);
}

int main(void) {
  oracle_set_num_threads(3);
  /* 1: walls on z (inner and outer layers), spheres in contact and within
   *    lubrication range, noise, gravity */
  {
    oracle_params p = base();
    p.periodic[2] = 0;
    p.g[2] = -1e-3;
    p.L[2] = 8.0;
    parts q = make_lattice(8, 8, 8, 1, 1);
    double xa[3] = {3.0, 3.0, 4.0}, xb[3] = {4.9, 3.1, 4.0}, xc[3] = {3.0, 5.1, 4.2};
    double va[3] = {0.05, 0, 0}, vb[3] = {-0.05, 0, 0}, vc[3] = {0, -0.02, 0};
    make_rigid(&q, 300, 1.0, xa, va);
    make_rigid(&q, 305, 1.0, xb, vb);
    make_rigid(&q, 340, 1.0, xc, vc);
    oracle_system* s = NULL;
    CHECK(oracle_create(&p, q.n, q.id, q.type, q.pos, q.vel, q.w, q.m, q.I, q.R, &s) ==
          ORACLE_OK);
    exercise(s, q.n, 12);
    oracle_destroy(s);
    /* slip walls and the negative-pressure clamp */
    p.noslip = 0;
    p.enable_neg_p_clamp = 1;
    CHECK(oracle_create(&p, q.n, q.id, q.type, q.pos, q.vel, q.w, q.m, q.I, q.R, &s) ==
          ORACLE_OK);
    exercise(s, q.n, 4);
    oracle_destroy(s);
    free_parts(&q);
  }
  /* 2: a Lees-Edwards box, reverse body force */
  {
    oracle_params p = base();
    p.shear_rate = 0.05;
    p.gravity_type = 1;
    p.g[1] = 1e-3;
    p.itr_start = 17;
    parts q = make_lattice(8, 8, 8, 0, 2);
    double xa[3] = {4.0, 4.0, 0.6}, va[3] = {0, 0, -0.1};
    make_rigid(&q, 100, 0.8, xa, va);
    oracle_system* s = NULL;
    CHECK(oracle_create(&p, q.n, q.id, q.type, q.pos, q.vel, q.w, q.m, q.I, q.R, &s) ==
          ORACLE_OK);
    exercise(s, q.n, 10);
    oracle_destroy(s);
    free_parts(&q);
  }
  /* 3: error paths */
  {
    oracle_params p = base();
    parts q = make_lattice(8, 8, 8, 0, 3);
    oracle_system* s = NULL;
    p.xi = 0.0;
    CHECK(oracle_create(&p, q.n, q.id, q.type, q.pos, q.vel, q.w, q.m, q.I, q.R, &s) ==
          ORACLE_E_INVALID_ARG);
    p = base();
    p.max_neighbors = 4;
    CHECK(oracle_create(&p, q.n, q.id, q.type, q.pos, q.vel, q.w, q.m, q.I, q.R, &s) ==
          ORACLE_OK);
    CHECK(oracle_compute_forces(s) == ORACLE_E_NBR_OVERFLOW);
    oracle_destroy(s);
    p = base();
    q.vel[7] = NAN;
    CHECK(oracle_create(&p, q.n, q.id, q.type, q.pos, q.vel, q.w, q.m, q.I, q.R, &s) ==
          ORACLE_OK);
    CHECK(oracle_step(s, 1) == ORACLE_E_NONFINITE);
    oracle_destroy(s);
    free_parts(&q);
  }
  /* the pure functions */
  {
    uint32_t c[4] = {1, 2, 3, 4}, k[2] = {5, 6}, o[4];
    oracle_philox4x32_10(c, k, o);
    double z[4];
    oracle_pair_normals(7, 3, 9, 11, z);
    CHECK(oracle_lattice_w_sum(1.5, 1.0) > 0.0);
    CHECK(oracle_drag_b(0.5, 0.1, 1.0, 1.0, 0.1) > 0.0);
    CHECK(oracle_drag_b(0.9, 1e4, 1.0, 1.0, 0.1) > 0.0);
  }
  printf("oracle sanitizer run ok\n");
  return 0;
}
