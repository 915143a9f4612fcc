/*
 * sdpdem_oracle.c -- plain FP64 CPU reference of the SDPD-DEM per-step path
 * of Tsuzuki, arXiv 2002.03120 ("DEMocritus").
 *
 * TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline
 * leg of the benchmark load this library; the product path never does.  It
 * shares no code with the GPU library.
 *
 * Written to be read against the paper: each routine follows the equation or
 * algorithm it cites, in the paper's order, in double precision, compiled
 * with -ffp-contract=off.  Gather form throughout: every particle sums its
 * own pair terms in ascending neighbour-id order, so the result does not
 * depend on the number of OpenMP threads.  The neighbour search is the
 * background grid with per-cell linked lists that Sec. 3.2 describes; the
 * tests check it against brute force.
 *
 * Readings where the paper is silent, garbled or ambiguous (each is also
 * listed in the design notes of the repository):
 *  R1  F(r) = -W'(r)/r >= 0 (Eq. defF drops the sign; Eq. F agrees).
 *  R2  h is the kernel support radius: W = 0 for r >= h (Eq. kernel).
 *  R3  rho in Eqs. FijC and gamma is the number density d = rho/m_f.
 *  R4  Density sums include the particle itself; every neighbour weighs
 *      m_f (single-pressure hypothesis, Sec. 2.4); the "normalisation of
 *      the coefficient of the kernel function" (Sec. 3.3) is a constant C_W
 *      that makes the ideal cubic lattice give rho0 exactly.
 *  R5  Pressure filtering = Shepard (W-weighted) mean, self included.
 *  R6  dW^S = (dW + dW^T)/2 - tr(dW)/3 * 1 (Eq. reldWij is garbled), the
 *      trace term of Eq. FijT multiplies the identity; dW = sqrt(dt) zeta
 *      with zeta a matrix of independent standard normals.  The matrix
 *      enters only through (sa dW^S + sb tr(dW)/3 1) e, a Gaussian vector
 *      whose law depends on e alone, so that vector is drawn from four
 *      normals (see oracle_pair_force).
 *  R7  Noise comes from Philox4x32-10 keyed by the seed with counter
 *      (min id, max id, step, 0); one block per pair per step, used by
 *      both velocity-Verlet passes, so the per-step variance is sigma^2 dt.
 *  R8  Torque lever: dx/2 for fluid, R for rigid, along -e_ij (Sec. 2.6).
 *  R9  Inner walls: position fixed, velocity and spin updated like fluid.
 *      Outer walls: nothing is updated; rho = rho0, p = p(rho0).
 *  R10 Fluid-particle coupling support H_s = R_s + h, Lucy weights with
 *      that support; eps = 1 - V_s N_r'/V_H (N_r' excludes s), clamped to
 *      [eps_min, 1]; drag acts against the slip, F^DG = -B V_s (v_s - v_f)
 *      with B = beta/(1-eps) in cancelled form; F^PG = (rho0 V_s/m_f) times
 *      the W-weighted mean of the neighbours' F^C + F^D sums; the reaction
 *      is normalised per rigid particle so that it balances exactly.
 *  R11 Tangential history committed once per step (second pass); sliding
 *      truncates the stored displacement to mu|F_n|/k_t; a contact is
 *      dropped when the spheres separate.
 *  R12 Lubrication acts for 0 < gap < h with gap = L - (R_i + R_j), mean
 *      diameter R_i + R_j, gap floored at lub_gap_min.
 *  R13 Body force g + f is an acceleration; gravity_type 1 flips its sign
 *      where x[axis] - org[axis] < L[axis]/2.
 *  R14 Periodic axes use the minimum image (no halo copies); a wall axis
 *      mirrors a particle that leaves [org, org+L] and reverses its velocity
 *      (the normal component of every face crossed for slip; for no-slip
 *      the whole velocity, once per drift even at an edge or corner).
 *  R15 The neighbour test is r^2 < h^2, strict, with
 *      r^2 = (dx*dx + dy*dy) + dz*dz in double precision.
 *  R19 Lees-Edwards shear (not in the paper; for the viscometer): flow
 *      along x, gradient along z.  The image of the box above sits at
 *      x + delta(t), delta = fmod(shear_rate L_z t, L_x) with t the time of
 *      the current positions, and moves with +shear_rate L_z in x.  The
 *      minimum image takes the z image first, then wraps x and y; pair
 *      terms see the image's velocity.  A particle leaving through a z face
 *      re-enters shifted by -/+ delta in x with v_x -/+ shear_rate L_z.
 *  R20 Pressure tensor of the box: P_ab = (sum_i m v'_a v'_b + W_ab) / V
 *      with v' = v - shear_rate (z - z_mid) e_x over fluid, rigid and
 *      inner-wall particles, and W the virial of the pair forces of the
 *      last evaluation: sum over pairs of r_ij,a F_ij,b, a pair computed
 *      from both sides counted half on each side, one-sided SDPD pairs
 *      (fluid on rigid or outer wall) counted once; the fluid-particle
 *      coupling of sphere s counts M_s,a (F^DG_s + F^PG_s)_b with the lever
 *      M_s = sum_j w_sj r_sj / Omega_s.  Body forces are external.
 *
 * Parity unpinned (nothing outside this file fixes them): the Shepard mean
 * of R5 beyond its own properties (a weighted mean of the neighbours'
 * pressures that reproduces a constant field); the history rules of R11
 * beyond the stick and slide cases; the lubrication of R12 between spheres
 * of unequal radii (only the equal-sphere squeeze film is pinned).
 */
#include "sdpdem_oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

struct oracle_system {
  oracle_params P;
  int64_t n;
  uint8_t* type;
  double *pos, *vel, *w, *mass, *iner, *rad;
  double *rho, *p, *ps;
  double *f_sdpd, *f_cd, *n_sdpd, *f_dg, *f_pg, *f_rxn, *f_dem, *f_lub, *n_dem;
  double* eps;
  double *a_sdpd, *a_cd, *a_nsdpd, *a_dg, *a_pg, *a_rxn, *a_dem, *a_lub, *a_ndem;
  double CW;
  /* neighbour sets: fixed-capacity rows */
  int32_t* nb_cnt;
  int32_t* nb_col;
  /* rigid particles in ascending id order */
  int64_t nrig;
  int64_t* rig_id;
  int64_t* rig_of; /* id -> rigid index or -1 */
  double rmax;
  /* coupling sets C_s (Sec. 2.4), rebuilt every pass */
  int32_t* cp_cnt;
  int64_t cp_cap;
  int32_t* cp_col;
  double* cp_w;
  double* cp_omega;
  /* contact table per rigid: partner id and tangential displacement */
  int32_t* ct_cnt;
  int32_t* ct_partner;
  double* ct_dt;
  int64_t step;
  int64_t pos_step;  /* step index of the time of the current positions */
  double le_shift;   /* Lees-Edwards offset at that time (R19) */
  double* vir;       /* per-particle virial W_ab of the last evaluation */
  /* background grid with linked lists (Sec. 3.2) */
  double glo[3], gcs[3];
  int64_t gnc[3];
  int64_t* head;
  int64_t* next;
  int64_t head_cap;
};

/* ------------------------------------------------------------------------ */
/* Lucy kernel, Eqs. kernel and F                                           */

double oracle_lucy_w(double r, double h) {
  if (r >= h) return 0.0;
  double q = r / h;
  double om = 1.0 - q;
  return 105.0 / (16.0 * M_PI * h * h * h) * (1.0 + 3.0 * q) * om * om * om;
}

double oracle_lucy_f(double r, double h) {
  if (r >= h) return 0.0;
  double om = 1.0 - r / h;
  return 315.0 / (4.0 * M_PI * h * h * h * h * h) * om * om;
}

/* Sum of W(|k| dx) over the ideal cubic lattice k in Z^3, self included. */
double oracle_lattice_w_sum(double h, double dx) {
  int K = (int)ceil(h / dx) + 1;
  double s = 0.0;
  for (int a = -K; a <= K; ++a)
    for (int b = -K; b <= K; ++b)
      for (int c = -K; c <= K; ++c) {
        double r = dx * sqrt((double)(a * a + b * b + c * c));
        s += oracle_lucy_w(r, h);
      }
  return s;
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11, "Parallel random
 * numbers: as easy as 1, 2, 3"): ten rounds of two 32x32->64 multiplies
 * with the published multipliers, the key bumped by the published Weyl
 * constants between rounds.                                                */

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                          uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
    uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
    uint32_t y0 = hi1 ^ x1 ^ k0;
    uint32_t y2 = hi0 ^ x3 ^ k1;
    x0 = y0;
    x1 = lo1;
    x2 = y2;
    x3 = lo0;
  }
  out[0] = x0;
  out[1] = x1;
  out[2] = x2;
  out[3] = x3;
}

/* Four standard normals for the unordered pair {a, b} at a step (R6, R7).
 * Uniforms u = ((x >> 8) + 1) 2^-24 in (0, 1] from one Philox block with
 * counter (min id, max id, step, 0); Box-Muller (1958) on (u0,u1) and
 * (u2,u3).                                                               */
void oracle_pair_normals(uint64_t seed, int64_t id_a, int64_t id_b,
                         int64_t step, double z[4]) {
  int64_t lo = id_a < id_b ? id_a : id_b;
  int64_t hi = id_a < id_b ? id_b : id_a;
  uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
  uint32_t ctr[4] = {(uint32_t)lo, (uint32_t)hi, (uint32_t)step, 0u};
  uint32_t x[4];
  oracle_philox4x32_10(ctr, key, x);
  double u[4];
  for (int k = 0; k < 4; ++k) u[k] = ((double)(x[k] >> 8) + 1.0) * (1.0 / 16777216.0);
  for (int m = 0; m < 2; ++m) {
    double rad = sqrt(-2.0 * log(u[2 * m]));
    double ang = 2.0 * M_PI * u[2 * m + 1];
    z[2 * m] = rad * cos(ang);
    z[2 * m + 1] = rad * sin(ang);
  }
}

/* ------------------------------------------------------------------------ */
/* One SDPD+a pair, Eqs. FijC, FijD, FijR, FijT with the gamma and sigma
 * definitions of Sec. 2.1 and readings R1, R3, R6, R7.                    */

void oracle_pair_force(const oracle_params* P, const double rij[3],
                       const double vi[3], const double vj[3],
                       const double wi[3], const double wj[3], double di,
                       double dj, double psi, double psj, int64_t idi,
                       int64_t idj, int64_t step, double fc[3], double fd[3],
                       double fr[3], double ft[3]) {
  double r = sqrt(rij[0] * rij[0] + rij[1] * rij[1] + rij[2] * rij[2]);
  double e[3] = {rij[0] / r, rij[1] / r, rij[2] / r};
  double F = oracle_lucy_f(r, P->h);
  /* conservative force, Eq. FijC */
  double pres = psi / (di * di) + psj / (dj * dj);
  for (int a = 0; a < 3; ++a) fc[a] = P->coeff_c * pres * F * rij[a];
  /* friction coefficients */
  double ga = (20.0 * P->eta / 3.0 - 4.0 * P->xi) * F / (di * dj);
  double gb = (17.0 * P->xi - 40.0 * P->eta / 3.0) * F / (di * dj);
  /* dissipative force, Eq. FijD */
  double v[3] = {vi[0] - vj[0], vi[1] - vj[1], vi[2] - vj[2]};
  double ev = e[0] * v[0] + e[1] * v[1] + e[2] * v[2];
  for (int a = 0; a < 3; ++a)
    fd[a] = P->coeff_d *
            (-ga * (v[a] + e[a] * ev / 3.0) - 2.0 * gb / 3.0 * e[a] * ev);
  /* rotational force, Eq. FijR: -gamma^a (r_ij/2) x (w_i + w_j) */
  double ws[3] = {wi[0] + wj[0], wi[1] + wj[1], wi[2] + wj[2]};
  double half[3] = {rij[0] / 2.0, rij[1] / 2.0, rij[2] / 2.0};
  double cr[3] = {half[1] * ws[2] - half[2] * ws[1],
                  half[2] * ws[0] - half[0] * ws[2],
                  half[0] * ws[1] - half[1] * ws[0]};
  for (int a = 0; a < 3; ++a) fr[a] = P->coeff_r * (-ga * cr[a]);
  /* thermal random force, Eq. FijT */
  for (int a = 0; a < 3; ++a) ft[a] = 0.0;
  if (P->kBT > 0.0 && P->coeff_t != 0.0) {
    double sa = 2.0 * sqrt(P->kBT * ga);
    double sb = 2.0 * sqrt(P->kBT * gb);
    /* Eq. FijT needs dW only as (sa dW^S + sb tr(dW)/3 1) e.  For a matrix
     * of independent standard increments (per sqrt(dt)) that vector is
     * Gaussian with variance 1/2 in each direction across e and
     * sa^2 2/3 + sb^2 1/3 along e (the traceless part's e-e entry has
     * variance 2/3, tr/3 has 1/3, and the three are independent): drawn
     * as s_ij P_perp xi / sqrt(2) with xi = (z0, z1, z2) and
     * P_perp = 1 - e e^T, plus z3 along e (R6).  s_ij = +1 if id_i < id_j,
     * else -1, keeps F^T_ji = -F^T_ij for the shared draw.               */
    double z[4];
    oracle_pair_normals(P->seed, idi, idj, step, z);
    double xe = z[0] * e[0] + z[1] * e[1] + z[2] * e[2];
    double s = idi < idj ? 1.0 : -1.0;
    double cpar = sqrt(sa * sa * (2.0 / 3.0) + sb * sb * (1.0 / 3.0));
    double sq = sqrt(P->dt);
    for (int a = 0; a < 3; ++a) {
      double perp = z[a] - xe * e[a];
      ft[a] = P->coeff_t * (sa * s * perp / sqrt(2.0) + cpar * z[3] * e[a]) / sq;
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Eq. beta divided by (1 - eps): Ergun for eps <= 0.8, Wen-Yu above, with
 * the drag coefficient and particle Reynolds number of Sec. 2.4 (R10).   */

double oracle_drag_b(double eps, double dv, double d, double rho, double mu) {
  if (eps <= 0.8)
    return 150.0 * mu * (1.0 - eps) / (eps * d * d) + 1.75 * rho * dv / d;
  double re = rho * d * eps * dv / mu;
  double cd_dv; /* C_D |v_f - v_i| */
  if (re <= 1000.0)
    cd_dv = 24.0 * mu * (1.0 + 0.15 * pow(re, 0.687)) / (rho * d * eps);
  else
    cd_dv = 0.44 * dv;
  return 0.75 * cd_dv * eps * rho * pow(eps, -2.65) / d;
}

/* ------------------------------------------------------------------------ */
/* DEM contact of Sec. 2.2: Eqs. dem_fnij, tandispn, slideref and the
 * Hertz-Mindlin coefficients deminputA..F (readings R11).  dij is the
 * minimum-image x_i - x_j.                                                */

void oracle_dem_pair(const oracle_params* P, const double dij[3],
                     const double vi[3], const double vj[3],
                     const double wi[3], const double wj[3], double Ri,
                     double Rj, double mi, double mj, const double dt_in[3],
                     double fn[3], double ft[3], double dt_out[3],
                     int* sliding) {
  double L = sqrt(dij[0] * dij[0] + dij[1] * dij[1] + dij[2] * dij[2]);
  double n[3] = {dij[0] / L, dij[1] / L, dij[2] / L};
  double dn[3];
  for (int a = 0; a < 3; ++a) dn[a] = (L - (Ri + Rj)) * n[a];
  double v[3] = {vi[0] - vj[0], vi[1] - vj[1], vi[2] - vj[2]};
  double vn_s = v[0] * n[0] + v[1] * n[1] + v[2] * n[2];
  double vn[3] = {vn_s * n[0], vn_s * n[1], vn_s * n[2]};
  double rw[3] = {Ri * wi[0] + Rj * wj[0], Ri * wi[1] + Rj * wj[1],
                  Ri * wi[2] + Rj * wj[2]};
  double rot[3] = {rw[1] * n[2] - rw[2] * n[1], rw[2] * n[0] - rw[0] * n[2],
                   rw[0] * n[1] - rw[1] * n[0]};
  double vt[3];
  for (int a = 0; a < 3; ++a) vt[a] = v[a] - vn[a] + rot[a];
  double Di = (1.0 - P->nu_dem * P->nu_dem) / (P->E_dem * M_PI);
  double Dj = Di;
  double kn = 4.0 / (3.0 * M_PI) * (1.0 / (Di + Dj)) * sqrt(Ri * Rj / (Ri + Rj));
  double kt = kn / (2.0 * (1.0 + P->nu_dem));
  double mm = 2.0 * mi * mj / (mi + mj);
  double cn = P->dem_damping * 2.0 * sqrt(mm * kn);
  double ct = P->dem_damping * 2.0 * sqrt(mm * kt);
  for (int a = 0; a < 3; ++a) {
    fn[a] = -kn * dn[a] - cn * vn[a];
    ft[a] = -kt * dt_in[a] - ct * vt[a];
  }
  double vt_abs = sqrt(vt[0] * vt[0] + vt[1] * vt[1] + vt[2] * vt[2]);
  double dt_abs =
      sqrt(dt_in[0] * dt_in[0] + dt_in[1] * dt_in[1] + dt_in[2] * dt_in[2]);
  double t[3] = {0.0, 0.0, 0.0};
  if (vt_abs > 0.0) {
    for (int a = 0; a < 3; ++a) t[a] = vt[a] / vt_abs;
  } else if (dt_abs > 0.0) {
    for (int a = 0; a < 3; ++a) t[a] = dt_in[a] / dt_abs;
  }
  double fn_abs = sqrt(fn[0] * fn[0] + fn[1] * fn[1] + fn[2] * fn[2]);
  double ft_abs = sqrt(ft[0] * ft[0] + ft[1] * ft[1] + ft[2] * ft[2]);
  double lim = P->mu_fric * fn_abs;
  if (ft_abs >= lim) {
    for (int a = 0; a < 3; ++a) {
      ft[a] = -lim * t[a];
      dt_out[a] = lim / kt * t[a];
    }
    *sliding = 1;
  } else {
    for (int a = 0; a < 3; ++a) dt_out[a] = dt_abs * t[a] + vt[a] * P->dt;
    *sliding = 0;
  }
}

/* ------------------------------------------------------------------------ */
/* geometry helpers                                                        */

/* Lees-Edwards offset delta(t) of the image above (R19) */
static double le_shift_at(const oracle_params* P, int64_t pstep) {
  if (P->shear_rate == 0.0) return 0.0;
  double t = (double)pstep * P->dt;
  double v = (P->shear_rate * P->L[2]) * t;
  double sft = fmod(v, P->L[0]);
  if (sft < 0.0) sft += P->L[0];
  return sft;
}

static void set_pos_step(oracle_system* s, int64_t pstep) {
  s->pos_step = pstep;
  s->le_shift = le_shift_at(&s->P, pstep);
}

/* minimum-image separation x_i - x_j' (R14, R19); returns k_z, the number
 * of boxes (in z) by which the image j' is displaced, so that j' moves with
 * v_j + k_z shear_rate L_z e_x */
static int min_image(const oracle_system* s, const double* xi,
                     const double* xj, double d[3]) {
  const oracle_params* P = &s->P;
  for (int a = 0; a < 3; ++a) d[a] = xi[a] - xj[a];
  if (P->shear_rate != 0.0) {
    double k = nearbyint(d[2] / P->L[2]);
    d[2] = d[2] - P->L[2] * k;
    d[0] = d[0] - s->le_shift * k;
    d[0] = d[0] - P->L[0] * nearbyint(d[0] / P->L[0]);
    d[1] = d[1] - P->L[1] * nearbyint(d[1] / P->L[1]);
    return (int)k;
  }
  for (int a = 0; a < 3; ++a)
    if (P->periodic[a]) d[a] = d[a] - P->L[a] * nearbyint(d[a] / P->L[a]);
  return 0;
}

/* velocity of the image of j displaced by kz boxes (R19) */
static void image_vel(const oracle_system* s, const double* vj, int kz,
                      double out[3]) {
  out[0] = vj[0] + (double)kz * (s->P.shear_rate * s->P.L[2]);
  out[1] = vj[1];
  out[2] = vj[2];
}

static double norm2(const double d[3]) {
  return (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
}

static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

/* background grid with per-cell linked lists (Sec. 3.2) */
static int grid_build(oracle_system* s) {
  const oracle_params* P = &s->P;
  double cs0 = P->h * (1.0 + 1e-6);
  for (int a = 0; a < 3; ++a) {
    if (P->periodic[a]) {
      s->glo[a] = P->org[a];
      s->gnc[a] = (int64_t)floor(P->L[a] / cs0);
      s->gcs[a] = P->L[a] / (double)s->gnc[a];
    } else {
      double mn = P->org[a], mx = P->org[a] + P->L[a];
      for (int64_t i = 0; i < s->n; ++i) {
        double x = s->pos[3 * i + a];
        if (x < mn) mn = x;
        if (x > mx) mx = x;
      }
      s->gcs[a] = cs0;
      s->glo[a] = mn - cs0;
      s->gnc[a] = (int64_t)floor((mx - s->glo[a]) / cs0) + 2;
    }
  }
  int64_t nc = s->gnc[0] * s->gnc[1] * s->gnc[2];
  if (nc > s->head_cap) {
    free(s->head);
    s->head = (int64_t*)malloc(sizeof(int64_t) * nc);
    if (!s->head) return ORACLE_E_NOMEM;
    s->head_cap = nc;
  }
  for (int64_t c = 0; c < nc; ++c) s->head[c] = -1;
  for (int64_t i = 0; i < s->n; ++i) {
    int64_t c3[3];
    for (int a = 0; a < 3; ++a) {
      int64_t c = (int64_t)floor((s->pos[3 * i + a] - s->glo[a]) / s->gcs[a]);
      if (P->periodic[a]) c = ((c % s->gnc[a]) + s->gnc[a]) % s->gnc[a];
      if (c < 0) c = 0;
      if (c >= s->gnc[a]) c = s->gnc[a] - 1;
      c3[a] = c;
    }
    int64_t c = (c3[2] * s->gnc[1] + c3[1]) * s->gnc[0] + c3[0];
    s->next[i] = s->head[c];
    s->head[c] = i;
  }
  return ORACLE_OK;
}

typedef struct {
  int32_t* v;
  int64_t n, cap;
} ibuf;

static void ibuf_push(ibuf* b, int32_t x) {
  if (b->n == b->cap) {
    b->cap = b->cap ? 2 * b->cap : 256;
    b->v = (int32_t*)realloc(b->v, sizeof(int32_t) * b->cap);
  }
  b->v[b->n++] = x;
}

/* All j != self with |x - x_j| < R (minimum image), sorted by id.
 * type_mask selects the particle types to keep (bit per type).         */
static void query_ball(const oracle_system* s, const double* x, double R,
                       int64_t self, unsigned type_mask, ibuf* out) {
  const oracle_params* P = &s->P;
  out->n = 0;
  int64_t lo[3], cnt[3], c0[3];
  for (int a = 0; a < 3; ++a) {
    c0[a] = (int64_t)floor((x[a] - s->glo[a]) / s->gcs[a]);
    int64_t k = (int64_t)floor(R / s->gcs[a] * (1.0 + 1e-9)) + 1;
    if (P->periodic[a]) {
      c0[a] = ((c0[a] % s->gnc[a]) + s->gnc[a]) % s->gnc[a];
      if (2 * k + 1 >= s->gnc[a]) {
        lo[a] = 0;
        cnt[a] = s->gnc[a];
      } else {
        lo[a] = c0[a] - k;
        cnt[a] = 2 * k + 1;
      }
    } else {
      lo[a] = c0[a] - k;
      cnt[a] = 2 * k + 1;
    }
  }
  double R2 = R * R;
  /* Lees-Edwards: rows seen through a z face are shifted in x, so every x
   * cell of such a row is searched (a superset; the distance test decides) */
  int le = P->shear_rate != 0.0;
  int le_all = le && cnt[2] == s->gnc[2];
  for (int64_t kz = 0; kz < cnt[2]; ++kz) {
    int64_t cz = lo[2] + kz;
    int crossing = le_all || (le && (cz < 0 || cz >= s->gnc[2]));
    if (P->periodic[2]) cz = ((cz % s->gnc[2]) + s->gnc[2]) % s->gnc[2];
    else if (cz < 0 || cz >= s->gnc[2]) continue;
    int64_t xlo = crossing ? 0 : lo[0];
    int64_t xcnt = crossing ? s->gnc[0] : cnt[0];
    for (int64_t ky = 0; ky < cnt[1]; ++ky) {
      int64_t cy = lo[1] + ky;
      if (P->periodic[1]) cy = ((cy % s->gnc[1]) + s->gnc[1]) % s->gnc[1];
      else if (cy < 0 || cy >= s->gnc[1]) continue;
      for (int64_t kx = 0; kx < xcnt; ++kx) {
        int64_t cx = xlo + kx;
        if (P->periodic[0]) cx = ((cx % s->gnc[0]) + s->gnc[0]) % s->gnc[0];
        else if (cx < 0 || cx >= s->gnc[0]) continue;
        int64_t c = (cz * s->gnc[1] + cy) * s->gnc[0] + cx;
        for (int64_t j = s->head[c]; j >= 0; j = s->next[j]) {
          if (j == self) continue;
          if (!((type_mask >> s->type[j]) & 1u)) continue;
          double d[3];
          min_image(s, x, &s->pos[3 * j], d);
          if (norm2(d) < R2) ibuf_push(out, (int32_t)j);
        }
      }
    }
  }
  if (out->n > 1) qsort(out->v, (size_t)out->n, sizeof(int32_t), cmp_i32);
}

#define ALL_TYPES 0xFu
#define MASK(t) (1u << (t))

/* ------------------------------------------------------------------------ */
/* compute_neighbor_list (Alg. 1): neighbour sets N(i) = {j != i : r < h}
 * for every particle that is not an outer wall (outer walls compute
 * nothing, R9).  Also the coupling sets C_s of the rigid particles.      */

static int build_neighbors(oracle_system* s) {
  int rc = grid_build(s);
  if (rc) return rc;
  const oracle_params* P = &s->P;
  int overflow = 0;
#pragma omp parallel
  {
    ibuf b = {0, 0, 0};
#pragma omp for schedule(dynamic, 512) reduction(| : overflow)
    for (int64_t i = 0; i < s->n; ++i) {
      s->nb_cnt[i] = 0;
      if (s->type[i] == O_OUTER_WALL) continue;
      query_ball(s, &s->pos[3 * i], P->h, i, ALL_TYPES, &b);
      int64_t m = b.n;
      if (m > P->max_neighbors) {
        overflow = 1;
        m = P->max_neighbors;
      }
      memcpy(&s->nb_col[i * (int64_t)P->max_neighbors], b.v,
             sizeof(int32_t) * (size_t)m);
      s->nb_cnt[i] = (int32_t)m;
    }
    free(b.v);
  }
  return overflow ? ORACLE_E_NBR_OVERFLOW : ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* compute_particle_dens / compute_particle_pres / smoothe_particle_pres    */

static void density_pressure(oracle_system* s) {
  const oracle_params* P = &s->P;
  double w0 = oracle_lucy_w(0.0, P->h);
  double p_ref = P->p0 * pow(1.0, P->alpha) - P->beta_eos;
  if (P->enable_neg_p_clamp && p_ref < 0.0) p_ref = 0.0;
#pragma omp parallel for schedule(dynamic, 512)
  for (int64_t i = 0; i < s->n; ++i) {
    if (s->type[i] == O_OUTER_WALL) {
      s->rho[i] = P->rho0;
      s->p[i] = p_ref;
      continue;
    }
    /* Eq. compdens with reading R4 */
    double acc = w0;
    const int32_t* nb = &s->nb_col[i * (int64_t)P->max_neighbors];
    for (int k = 0; k < s->nb_cnt[i]; ++k) {
      double d[3];
      min_image(s, &s->pos[3 * i], &s->pos[3 * (int64_t)nb[k]], d);
      acc += oracle_lucy_w(sqrt(norm2(d)), P->h);
    }
    s->rho[i] = s->CW * P->mass_fluid * acc;
    /* Eq. prtcpres, clamped at free surfaces when enabled (Sec. 2.5) */
    double pr = P->p0 * pow(s->rho[i] / P->rho0, P->alpha) - P->beta_eos;
    if (P->enable_neg_p_clamp && pr < 0.0) pr = 0.0;
    s->p[i] = pr;
  }
#pragma omp parallel for schedule(dynamic, 512)
  for (int64_t i = 0; i < s->n; ++i) {
    if (s->type[i] == O_OUTER_WALL || !P->enable_pres_smooth) {
      s->ps[i] = s->p[i];
      continue;
    }
    /* reading R5: Shepard mean of p, self included */
    double num = s->p[i] * w0, den = w0;
    const int32_t* nb = &s->nb_col[i * (int64_t)P->max_neighbors];
    for (int k = 0; k < s->nb_cnt[i]; ++k) {
      int64_t j = nb[k];
      double d[3];
      min_image(s, &s->pos[3 * i], &s->pos[3 * j], d);
      double wij = oracle_lucy_w(sqrt(norm2(d)), P->h);
      num += s->p[j] * wij;
      den += wij;
    }
    s->ps[i] = num / den;
  }
}

static double vabs3(const double* v) {
  return sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
}

/* ------------------------------------------------------------------------ */
/* compute_fluid (Alg. 2): F^SDPD of fluid and inner-wall particles over
 * all their neighbours (rigid ones included, single-pressure hypothesis),
 * the F^C + F^D sums that F^PG needs, and the torque (reading R8).       */

static void compute_fluid(oracle_system* s) {
  const oracle_params* P = &s->P;
  double lever = 0.5 * P->dx;
#pragma omp parallel for schedule(dynamic, 512)
  for (int64_t i = 0; i < s->n; ++i) {
    double F[3] = {0, 0, 0}, Fcd[3] = {0, 0, 0}, N[3] = {0, 0, 0};
    double aF = 0, aCD = 0, aN = 0;
    double* W = &s->vir[9 * i];
    for (int a = 0; a < 9; ++a) W[a] = 0.0;
    if (s->type[i] == O_FLUID || s->type[i] == O_INNER_WALL) {
      double di = s->rho[i] / P->mass_fluid;
      const int32_t* nb = &s->nb_col[i * (int64_t)P->max_neighbors];
      for (int k = 0; k < s->nb_cnt[i]; ++k) {
        int64_t j = nb[k];
        double rij[3], vj[3];
        int kz = min_image(s, &s->pos[3 * i], &s->pos[3 * j], rij);
        image_vel(s, &s->vel[3 * j], kz, vj);
        double dj = s->rho[j] / P->mass_fluid;
        double fc[3], fd[3], fr[3], ft[3];
        oracle_pair_force(P, rij, &s->vel[3 * i], vj, &s->w[3 * i],
                          &s->w[3 * j], di, dj, s->ps[i], s->ps[j], i, j,
                          s->step, fc, fd, fr, ft);
        double r = sqrt(norm2(rij));
        double f[3], cd[3], tq[3], me[3];
        for (int a = 0; a < 3; ++a) {
          f[a] = fc[a] + fd[a] + fr[a] + ft[a];
          cd[a] = fc[a] + fd[a];
          me[a] = -rij[a] / r * lever; /* lever along -e_ij */
        }
        tq[0] = me[1] * f[2] - me[2] * f[1];
        tq[1] = me[2] * f[0] - me[0] * f[2];
        tq[2] = me[0] * f[1] - me[1] * f[0];
        for (int a = 0; a < 3; ++a) {
          F[a] += f[a];
          Fcd[a] += cd[a];
          N[a] += tq[a];
        }
        /* virial (R20): half of a pair that j also evaluates */
        double c = (s->type[j] == O_FLUID || s->type[j] == O_INNER_WALL) ? 0.5 : 1.0;
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) W[3 * a + b] += c * rij[a] * f[b];
        aF += vabs3(f);
        aCD += vabs3(cd);
        aN += vabs3(tq);
      }
    }
    for (int a = 0; a < 3; ++a) {
      s->f_sdpd[3 * i + a] = F[a];
      s->f_cd[3 * i + a] = Fcd[a];
      s->n_sdpd[3 * i + a] = N[a];
    }
    s->a_sdpd[i] = aF;
    s->a_cd[i] = aCD;
    s->a_nsdpd[i] = aN;
  }
}

static int rigid_active(const oracle_system* s) {
  return s->step >= s->P.itr_actv_rigid;
}

/* ------------------------------------------------------------------------ */
/* compute_fpi_action (Alg. 2): eps (Eq. fvfdef, reading R10), the drag
 * F^DG (Eqs. F_fpi_DG and beta) and the pressure-gradient force F^PG
 * (Eq. F_fpi_PG) of every active rigid particle.                          */

static int compute_fpi_action(oracle_system* s) {
  const oracle_params* P = &s->P;
  for (int64_t i = 0; i < s->n; ++i) {
    for (int a = 0; a < 3; ++a) s->f_dg[3 * i + a] = s->f_pg[3 * i + a] = 0.0;
    s->eps[i] = 0.0;
    s->a_dg[i] = s->a_pg[i] = 0.0;
  }
  if (s->nrig == 0 || !rigid_active(s)) {
    for (int64_t r = 0; r < s->nrig; ++r) s->cp_cnt[r] = 0;
    return ORACLE_OK;
  }
  /* capacity of one coupling row: every fluid particle within H_max */
  int err = 0;
#pragma omp parallel
  {
    ibuf b = {0, 0, 0}, rb = {0, 0, 0};
#pragma omp for schedule(dynamic, 4) reduction(| : err)
    for (int64_t r = 0; r < s->nrig; ++r) {
      int64_t si = s->rig_id[r];
      double R = s->rad[si];
      double H = R + P->h;
      const double* xs = &s->pos[3 * si];
      query_ball(s, xs, H, si, MASK(O_FLUID), &b);
      query_ball(s, xs, H, si, MASK(O_RIGID), &rb);
      if (b.n > s->cp_cap) {
        err = 1;
        b.n = s->cp_cap;
      }
      double omega = 0.0, vf[3] = {0, 0, 0}, fcd[3] = {0, 0, 0}, acd = 0.0;
      double lev[3] = {0, 0, 0};
      for (int64_t k = 0; k < b.n; ++k) {
        int64_t j = b.v[k];
        double d[3], vj[3];
        int kz = min_image(s, xs, &s->pos[3 * j], d);
        image_vel(s, &s->vel[3 * j], kz, vj);
        double wsj = oracle_lucy_w(sqrt(norm2(d)), H);
        s->cp_col[r * s->cp_cap + k] = (int32_t)j;
        s->cp_w[r * s->cp_cap + k] = wsj;
        omega += wsj;
        for (int a = 0; a < 3; ++a) {
          vf[a] += wsj * vj[a];
          fcd[a] += wsj * s->f_cd[3 * j + a];
          lev[a] += wsj * d[a];
        }
        acd += wsj * s->a_cd[j];
      }
      s->cp_cnt[r] = (int32_t)b.n;
      s->cp_omega[r] = omega;
      double Vs = 4.0 / 3.0 * M_PI * R * R * R;
      double VH = 4.0 / 3.0 * M_PI * H * H * H;
      double eps = 1.0 - Vs * (double)rb.n / VH;
      if (eps < P->eps_min) eps = P->eps_min;
      if (eps > 1.0) eps = 1.0;
      s->eps[si] = eps;
      if (b.n == 0 || omega <= 0.0) {
        s->cp_cnt[r] = 0;
        continue;
      }
      double dv[3];
      for (int a = 0; a < 3; ++a) dv[a] = s->vel[3 * si + a] - vf[a] / omega;
      double B = oracle_drag_b(eps, vabs3(dv), 2.0 * R, P->rho0, P->eta);
      for (int a = 0; a < 3; ++a) {
        s->f_dg[3 * si + a] = -B * Vs * dv[a];
        s->f_pg[3 * si + a] = P->rho0 * Vs / P->mass_fluid * (fcd[a] / omega);
      }
      /* virial of the coupling (R20), lever M_s = sum_j w_sj r_sj / Omega_s */
      for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c)
          s->vir[9 * si + 3 * a + c] +=
              (lev[a] / omega) * (s->f_dg[3 * si + c] + s->f_pg[3 * si + c]);
      s->a_dg[si] = vabs3(&s->f_dg[3 * si]);
      s->a_pg[si] = P->rho0 * Vs / P->mass_fluid * (acd / omega);
    }
    free(b.v);
    free(rb.v);
  }
  return err ? ORACLE_E_NBR_OVERFLOW : ORACLE_OK;
}

/* compute_fpi_reaction (Alg. 2, Eq. F_fpi_DG_reac with reading R10): the
 * reaction on fluid j is -sum_s F^DG_s w_sj / Omega_s, accumulated with s
 * in ascending id order.                                                  */

static void compute_fpi_reaction(oracle_system* s) {
  for (int64_t i = 0; i < 3 * s->n; ++i) s->f_rxn[i] = 0.0;
  for (int64_t i = 0; i < s->n; ++i) s->a_rxn[i] = 0.0;
  for (int64_t r = 0; r < s->nrig; ++r) {
    int64_t si = s->rig_id[r];
    for (int32_t k = 0; k < s->cp_cnt[r]; ++k) {
      int64_t j = s->cp_col[r * s->cp_cap + k];
      double c = s->cp_w[r * s->cp_cap + k] / s->cp_omega[r];
      for (int a = 0; a < 3; ++a) s->f_rxn[3 * j + a] -= s->f_dg[3 * si + a] * c;
      s->a_rxn[j] += s->a_dg[si] * c;
    }
  }
}

/* compute_rigid (Alg. 2): DEM contacts and lubrication between rigid
 * particles (Secs. 2.2, 2.3).  commit = 1 on the second pass.             */

static int compute_rigid(oracle_system* s, int commit) {
  const oracle_params* P = &s->P;
  for (int64_t i = 0; i < s->n; ++i) {
    for (int a = 0; a < 3; ++a)
      s->f_dem[3 * i + a] = s->f_lub[3 * i + a] = s->n_dem[3 * i + a] = 0.0;
    s->a_dem[i] = s->a_lub[i] = s->a_ndem[i] = 0.0;
  }
  if (s->nrig == 0 || !rigid_active(s)) return ORACLE_OK;
  int err = 0;
  int32_t mc = P->max_contacts;
#pragma omp parallel
  {
    ibuf b = {0, 0, 0};
    int32_t* np = (int32_t*)malloc(sizeof(int32_t) * (size_t)(mc > 0 ? mc : 1));
    double* nd = (double*)malloc(sizeof(double) * 3 * (size_t)(mc > 0 ? mc : 1));
#pragma omp for schedule(dynamic, 16) reduction(| : err)
    for (int64_t r = 0; r < s->nrig; ++r) {
      int64_t si = s->rig_id[r];
      double Rs = s->rad[si];
      query_ball(s, &s->pos[3 * si], Rs + s->rmax + P->h, si, MASK(O_RIGID), &b);
      int32_t ncnt = 0;
      double F[3] = {0, 0, 0}, Fl[3] = {0, 0, 0}, N[3] = {0, 0, 0};
      double aF = 0, aL = 0, aN = 0;
      for (int64_t q = 0; q < b.n; ++q) {
        int64_t k = b.v[q];
        double Rk = s->rad[k];
        double d[3], vk[3];
        int kz = min_image(s, &s->pos[3 * si], &s->pos[3 * k], d);
        image_vel(s, &s->vel[3 * k], kz, vk);
        double L = sqrt(norm2(d));
        if (L < Rs + Rk) {
          double dtin[3] = {0, 0, 0};
          for (int32_t c = 0; c < s->ct_cnt[r]; ++c)
            if (s->ct_partner[r * mc + c] == (int32_t)k) {
              for (int a = 0; a < 3; ++a) dtin[a] = s->ct_dt[(r * mc + c) * 3 + a];
              break;
            }
          double fn[3], ft[3], dto[3];
          int sl;
          oracle_dem_pair(P, d, &s->vel[3 * si], vk,
                          &s->w[3 * si], &s->w[3 * k], Rs, Rk, s->mass[si],
                          s->mass[k], dtin, fn, ft, dto, &sl);
          double tq[3], me[3];
          for (int a = 0; a < 3; ++a) me[a] = -d[a] / L * Rs;
          tq[0] = me[1] * ft[2] - me[2] * ft[1];
          tq[1] = me[2] * ft[0] - me[0] * ft[2];
          tq[2] = me[0] * ft[1] - me[1] * ft[0];
          double f[3];
          for (int a = 0; a < 3; ++a) {
            f[a] = fn[a] + ft[a];
            F[a] += f[a];
            N[a] += tq[a];
          }
          for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c) s->vir[9 * si + 3 * a + c] += 0.5 * d[a] * f[c];
          aF += vabs3(f);
          aN += vabs3(tq);
          if (ncnt >= mc) {
            err = 1;
          } else {
            np[ncnt] = (int32_t)k;
            for (int a = 0; a < 3; ++a) nd[3 * ncnt + a] = dto[a];
            ++ncnt;
          }
        } else if (P->enable_lub) {
          double gap = L - (Rs + Rk);
          if (gap > 0.0 && gap < P->h) {
            double dbar = Rs + Rk;
            double gg = gap > P->lub_gap_min ? gap : P->lub_gap_min;
            double c = 3.0 * M_PI * P->eta * dbar * dbar / (8.0 * gg);
            double fl[3];
            for (int a = 0; a < 3; ++a) {
              fl[a] = c * (vk[a] - s->vel[3 * si + a]);
              Fl[a] += fl[a];
            }
            for (int a = 0; a < 3; ++a)
              for (int e = 0; e < 3; ++e) s->vir[9 * si + 3 * a + e] += 0.5 * d[a] * fl[e];
            aL += vabs3(fl);
          }
        }
      }
      for (int a = 0; a < 3; ++a) {
        s->f_dem[3 * si + a] = F[a];
        s->f_lub[3 * si + a] = Fl[a];
        s->n_dem[3 * si + a] = N[a];
      }
      s->a_dem[si] = aF;
      s->a_lub[si] = aL;
      s->a_ndem[si] = aN;
      if (commit) {
        s->ct_cnt[r] = ncnt;
        for (int32_t c = 0; c < ncnt; ++c) {
          s->ct_partner[r * mc + c] = np[c];
          for (int a = 0; a < 3; ++a) s->ct_dt[(r * mc + c) * 3 + a] = nd[3 * c + a];
        }
      }
    }
    free(b.v);
    free(np);
    free(nd);
  }
  return err ? ORACLE_E_CONTACT_OVERFLOW : ORACLE_OK;
}

/* compute_force (Alg. 2) after the neighbour, density and pressure steps */
static int compute_all(oracle_system* s, int commit) {
  int rc = build_neighbors(s);
  if (rc) return rc;
  density_pressure(s);
  compute_fluid(s);
  rc = compute_fpi_action(s);
  if (rc) return rc;
  compute_fpi_reaction(s);
  return compute_rigid(s, commit);
}

/* ------------------------------------------------------------------------ */
/* totals of Eqs. newton1/newton2 per particle type (Sec. 2.6, R13)       */

static double gsign(const oracle_params* P, const double* x) {
  if (P->gravity_type != 1) return 1.0;
  int a = P->gravity_axis;
  return (x[a] - P->org[a] >= 0.5 * P->L[a]) ? 1.0 : -1.0;
}

static void total_force(const oracle_system* s, int64_t i, double F[3],
                        double N[3]) {
  const oracle_params* P = &s->P;
  double sg = gsign(P, &s->pos[3 * i]);
  for (int a = 0; a < 3; ++a) {
    double body = s->mass[i] * (P->g[a] + P->f[a]) * sg;
    switch (s->type[i]) {
      case O_FLUID:
        F[a] = s->f_sdpd[3 * i + a] + s->f_rxn[3 * i + a] + body;
        N[a] = s->n_sdpd[3 * i + a];
        break;
      case O_INNER_WALL:
        F[a] = s->f_sdpd[3 * i + a] + body;
        N[a] = s->n_sdpd[3 * i + a];
        break;
      case O_RIGID:
        if (rigid_active(s)) {
          F[a] = s->f_pg[3 * i + a] + s->f_dg[3 * i + a] + s->f_dem[3 * i + a] +
                 s->f_lub[3 * i + a] + body;
          N[a] = s->n_dem[3 * i + a];
        } else {
          F[a] = N[a] = 0.0;
        }
        break;
      default:
        F[a] = N[a] = 0.0;
    }
  }
}

/* update(velver): velocity-Verlet half kick, and on the first pass the
 * drift followed by the boundary treatment of Sec. 2.5 (R14).            */

static int update(oracle_system* s, int velver) {
  const oracle_params* P = &s->P;
  int bad = 0, out = 0;
  int act = rigid_active(s);
  /* Lees-Edwards offset at the time the drift moves to (R19) */
  const int le = P->shear_rate != 0.0;
  const double le_new = le_shift_at(P, s->step + 1);
  const double le_dv = P->shear_rate * P->L[2];
#pragma omp parallel for schedule(static) reduction(| : bad, out)
  for (int64_t i = 0; i < s->n; ++i) {
    uint8_t t = s->type[i];
    if (t == O_OUTER_WALL) continue;
    if (t == O_RIGID && !act) continue;
    double F[3], N[3];
    total_force(s, i, F, N);
    for (int a = 0; a < 3; ++a) {
      s->vel[3 * i + a] += 0.5 * P->dt * F[a] / s->mass[i];
      s->w[3 * i + a] += 0.5 * P->dt * N[a] / s->iner[i];
    }
    if (velver == 1 && (t == O_FLUID || t == O_RIGID)) {
      for (int a = 0; a < 3; ++a) s->pos[3 * i + a] += P->dt * s->vel[3 * i + a];
      if (le) {
        /* leaving through a z face: re-enter as the image of the next box */
        double* x = &s->pos[3 * i];
        if (x[2] < P->org[2]) {
          x[2] += P->L[2];
          x[0] += le_new;
          s->vel[3 * i] += le_dv;
        } else if (x[2] >= P->org[2] + P->L[2]) {
          x[2] -= P->L[2];
          x[0] -= le_new;
          s->vel[3 * i] -= le_dv;
        }
        if (x[0] < P->org[0]) x[0] += P->L[0];
        else if (x[0] >= P->org[0] + P->L[0]) x[0] -= P->L[0];
      }
      int hit = 0; /* a wall face was crossed in this drift */
      for (int a = 0; a < 3; ++a) {
        double lo = P->org[a], hi = P->org[a] + P->L[a];
        double* x = &s->pos[3 * i + a];
        if (P->periodic[a]) {
          if (*x < lo) *x += P->L[a];
          else if (*x >= hi) *x -= P->L[a];
        } else if (*x < lo || *x > hi) {
          *x = (*x < lo) ? 2.0 * lo - *x : 2.0 * hi - *x;
          hit = 1;
          if (!P->noslip) s->vel[3 * i + a] = -s->vel[3 * i + a];
          if (*x < lo || *x > hi) out = 1;
        }
      }
      /* no-slip: the whole velocity is reversed once, however many faces
       * (an edge or a corner) the drift crossed */
      if (hit && P->noslip)
        for (int b = 0; b < 3; ++b) s->vel[3 * i + b] = -s->vel[3 * i + b];
    }
    for (int a = 0; a < 3; ++a)
      if (!isfinite(s->vel[3 * i + a]) || !isfinite(s->w[3 * i + a]) ||
          !isfinite(s->pos[3 * i + a]))
        bad = 1;
  }
  if (bad) return ORACLE_E_NONFINITE;
  if (out) return ORACLE_E_OUT_OF_DOMAIN;
  return ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1                                                             */

int oracle_step(oracle_system* s, int64_t nsteps) {
  if (!s || nsteps < 0) return ORACLE_E_INVALID_ARG;
  for (int64_t it = 0; it < nsteps; ++it) {
    for (int velver = 1; velver <= 2; ++velver) {
      int rc = compute_all(s, velver == 2);
      if (rc) return rc;
      rc = update(s, velver);
      if (rc) return rc;
      if (velver == 1) set_pos_step(s, s->step + 1);
    }
    s->step += 1;
  }
  return ORACLE_OK;
}

int oracle_compute_forces(oracle_system* s) {
  if (!s) return ORACLE_E_INVALID_ARG;
  return compute_all(s, 0);
}

/* ------------------------------------------------------------------------ */
/* creation and I/O                                                        */

#define ALLOC(ptr, cnt)                                             \
  do {                                                              \
    (ptr) = calloc((size_t)((cnt) > 0 ? (cnt) : 1), sizeof(*(ptr))); \
    if (!(ptr)) goto nomem;                                         \
  } while (0)

int oracle_create(const oracle_params* p, int64_t n, const int64_t* id,
                  const uint8_t* type, const double* pos, const double* vel,
                  const double* angvel, const double* mass,
                  const double* inertia, const double* radius,
                  oracle_system** out) {
  if (!p || !out || n < 0) return ORACLE_E_INVALID_ARG;
  *out = NULL;
  if (!(p->h > 0) || !(p->dx > 0) || !(p->dt > 0) || !(p->rho0 > 0) ||
      !(p->mass_fluid > 0) || !(p->inertia_fluid > 0) || p->max_neighbors <= 0 ||
      p->max_contacts <= 0 || p->kBT < 0)
    return ORACLE_E_INVALID_ARG;
  /* positivity of gamma^a and gamma^b */
  if (p->xi < 40.0 * p->eta / 51.0 || p->xi > 5.0 * p->eta / 3.0)
    return ORACLE_E_INVALID_ARG;
  for (int a = 0; a < 3; ++a) {
    if (!(p->L[a] > 0)) return ORACLE_E_INVALID_ARG;
    if (p->periodic[a] && p->L[a] < 3.0 * p->h * (1.0 + 1e-6))
      return ORACLE_E_INVALID_ARG;
  }
  if (p->gravity_axis < 0 || p->gravity_axis > 2) return ORACLE_E_INVALID_ARG;
  if (p->shear_rate != 0.0 &&
      (!p->periodic[0] || !p->periodic[1] || !p->periodic[2] || !isfinite(p->shear_rate)))
    return ORACLE_E_INVALID_ARG;
  oracle_system* s = (oracle_system*)calloc(1, sizeof(oracle_system));
  if (!s) return ORACLE_E_NOMEM;
  s->P = *p;
  s->n = n;
  s->step = p->itr_start;
  set_pos_step(s, p->itr_start);
  ALLOC(s->type, n);
  ALLOC(s->pos, 3 * n);
  ALLOC(s->vel, 3 * n);
  ALLOC(s->w, 3 * n);
  ALLOC(s->mass, n);
  ALLOC(s->iner, n);
  ALLOC(s->rad, n);
  ALLOC(s->rho, n);
  ALLOC(s->p, n);
  ALLOC(s->ps, n);
  ALLOC(s->f_sdpd, 3 * n);
  ALLOC(s->f_cd, 3 * n);
  ALLOC(s->n_sdpd, 3 * n);
  ALLOC(s->f_dg, 3 * n);
  ALLOC(s->f_pg, 3 * n);
  ALLOC(s->f_rxn, 3 * n);
  ALLOC(s->f_dem, 3 * n);
  ALLOC(s->f_lub, 3 * n);
  ALLOC(s->n_dem, 3 * n);
  ALLOC(s->eps, n);
  ALLOC(s->a_sdpd, n);
  ALLOC(s->a_cd, n);
  ALLOC(s->a_nsdpd, n);
  ALLOC(s->a_dg, n);
  ALLOC(s->a_pg, n);
  ALLOC(s->a_rxn, n);
  ALLOC(s->a_dem, n);
  ALLOC(s->a_lub, n);
  ALLOC(s->a_ndem, n);
  ALLOC(s->vir, 9 * n);
  ALLOC(s->nb_cnt, n);
  ALLOC(s->nb_col, n * (int64_t)p->max_neighbors);
  ALLOC(s->next, n);
  ALLOC(s->rig_of, n);
  {
    /* ids must be a permutation of 0..n-1 */
    for (int64_t k = 0; k < n; ++k) s->rig_of[k] = -2;
    for (int64_t k = 0; k < n; ++k) {
      int64_t i = id[k];
      if (i < 0 || i >= n || s->rig_of[i] != -2 || type[k] > O_OUTER_WALL) {
        oracle_destroy(s);
        return ORACLE_E_INVALID_ARG;
      }
      s->rig_of[i] = -1;
      s->type[i] = type[k];
      for (int a = 0; a < 3; ++a) {
        s->pos[3 * i + a] = pos[3 * k + a];
        s->vel[3 * i + a] = vel[3 * k + a];
        s->w[3 * i + a] = angvel[3 * k + a];
      }
      if (type[k] == O_RIGID) {
        s->mass[i] = mass[k];
        s->iner[i] = inertia[k];
        s->rad[i] = radius[k];
        if (!(mass[k] > 0) || !(inertia[k] > 0) || !(radius[k] > 0)) {
          oracle_destroy(s);
          return ORACLE_E_INVALID_ARG;
        }
      } else {
        s->mass[i] = p->mass_fluid;
        s->iner[i] = p->inertia_fluid;
        s->rad[i] = 0.5 * p->dx;
      }
    }
    int64_t nr = 0;
    for (int64_t i = 0; i < n; ++i)
      if (s->type[i] == O_RIGID) ++nr;
    s->nrig = nr;
    ALLOC(s->rig_id, nr);
    nr = 0;
    s->rmax = 0.0;
    for (int64_t i = 0; i < n; ++i)
      if (s->type[i] == O_RIGID) {
        s->rig_of[i] = nr;
        s->rig_id[nr++] = i;
        if (s->rad[i] > s->rmax) s->rmax = s->rad[i];
      }
    /* a coupling row holds at most every particle inside the largest H_s */
    double H = s->rmax + p->h;
    double cap = 4.0 / 3.0 * M_PI * (H + p->dx) * (H + p->dx) * (H + p->dx) /
                 (p->dx * p->dx * p->dx) * 2.0 + 64.0;
    s->cp_cap = s->nrig ? (int64_t)cap : 1;
    ALLOC(s->cp_cnt, s->nrig);
    ALLOC(s->cp_omega, s->nrig);
    ALLOC(s->cp_col, s->nrig * s->cp_cap);
    ALLOC(s->cp_w, s->nrig * s->cp_cap);
    ALLOC(s->ct_cnt, s->nrig);
    ALLOC(s->ct_partner, s->nrig * (int64_t)p->max_contacts);
    ALLOC(s->ct_dt, 3 * s->nrig * (int64_t)p->max_contacts);
  }
  if (p->enable_kernel_norm)
    s->CW = p->rho0 / (p->mass_fluid * oracle_lattice_w_sum(p->h, p->dx));
  else
    s->CW = 1.0;
  *out = s;
  return ORACLE_OK;
nomem:
  oracle_destroy(s);
  return ORACLE_E_NOMEM;
}

void oracle_destroy(oracle_system* s) {
  if (!s) return;
  void* ptrs[] = {s->type, s->pos, s->vel, s->w, s->mass, s->iner, s->rad,
                  s->rho, s->p, s->ps, s->f_sdpd, s->f_cd, s->n_sdpd, s->f_dg,
                  s->f_pg, s->f_rxn, s->f_dem, s->f_lub, s->n_dem, s->eps,
                  s->a_sdpd, s->a_cd, s->a_nsdpd, s->a_dg, s->a_pg, s->a_rxn,
                  s->a_dem, s->a_lub, s->a_ndem, s->nb_cnt, s->nb_col,
                  s->rig_id, s->rig_of, s->cp_cnt, s->cp_col, s->cp_w,
                  s->cp_omega, s->ct_cnt, s->ct_partner, s->ct_dt, s->head,
                  s->next, s->vir};
  for (size_t k = 0; k < sizeof(ptrs) / sizeof(ptrs[0]); ++k) free(ptrs[k]);
  free(s);
}

int oracle_field_comps(int field) {
  switch (field) {
    case OF_DENS:
    case OF_PRES:
    case OF_PRES_SMOOTH:
    case OF_EPS:
      return 1;
    default:
      if (field >= OF_F_SDPD_ABS && field <= OF_N_DEM_ABS) return 1;
      if (field >= OF_POS && field <= OF_N_TOTAL) return 3;
      return 0;
  }
}

int oracle_read_field(oracle_system* s, int field, double* dst) {
  if (!s || !dst) return ORACLE_E_INVALID_ARG;
  int64_t n = s->n;
  const double* src = NULL;
  switch (field) {
    case OF_POS: src = s->pos; break;
    case OF_VEL: src = s->vel; break;
    case OF_ANGVEL: src = s->w; break;
    case OF_DENS: src = s->rho; break;
    case OF_PRES: src = s->p; break;
    case OF_PRES_SMOOTH: src = s->ps; break;
    case OF_F_SDPD: src = s->f_sdpd; break;
    case OF_F_CD: src = s->f_cd; break;
    case OF_N_SDPD: src = s->n_sdpd; break;
    case OF_F_DG: src = s->f_dg; break;
    case OF_F_PG: src = s->f_pg; break;
    case OF_F_RXN: src = s->f_rxn; break;
    case OF_F_DEM: src = s->f_dem; break;
    case OF_F_LUB: src = s->f_lub; break;
    case OF_N_DEM: src = s->n_dem; break;
    case OF_EPS: src = s->eps; break;
    case OF_F_SDPD_ABS: src = s->a_sdpd; break;
    case OF_F_CD_ABS: src = s->a_cd; break;
    case OF_N_SDPD_ABS: src = s->a_nsdpd; break;
    case OF_F_DG_ABS: src = s->a_dg; break;
    case OF_F_PG_ABS: src = s->a_pg; break;
    case OF_F_RXN_ABS: src = s->a_rxn; break;
    case OF_F_DEM_ABS: src = s->a_dem; break;
    case OF_F_LUB_ABS: src = s->a_lub; break;
    case OF_N_DEM_ABS: src = s->a_ndem; break;
    case OF_F_TOTAL:
    case OF_N_TOTAL:
      for (int64_t i = 0; i < n; ++i) {
        double F[3], N[3];
        total_force(s, i, F, N);
        for (int a = 0; a < 3; ++a) dst[3 * i + a] = field == OF_F_TOTAL ? F[a] : N[a];
      }
      return ORACLE_OK;
    default:
      return ORACLE_E_INVALID_ARG;
  }
  memcpy(dst, src, sizeof(double) * (size_t)(n * oracle_field_comps(field)));
  return ORACLE_OK;
}

int oracle_read_neighbors(oracle_system* s, int64_t* row_ptr, int32_t* cols,
                          int64_t cap, int64_t* nnz) {
  if (!s || !row_ptr || !nnz) return ORACLE_E_INVALID_ARG;
  int64_t tot = 0;
  row_ptr[0] = 0;
  for (int64_t i = 0; i < s->n; ++i) {
    tot += s->nb_cnt[i];
    row_ptr[i + 1] = tot;
  }
  *nnz = tot;
  if (!cols || cap < tot) return cols ? ORACLE_E_INVALID_ARG : ORACLE_OK;
  for (int64_t i = 0; i < s->n; ++i)
    memcpy(&cols[row_ptr[i]], &s->nb_col[i * (int64_t)s->P.max_neighbors],
           sizeof(int32_t) * (size_t)s->nb_cnt[i]);
  return ORACLE_OK;
}

int oracle_read_contacts(oracle_system* s, int32_t* pairs, double* delta_t,
                         int64_t cap, int64_t* n_contacts) {
  if (!s || !n_contacts) return ORACLE_E_INVALID_ARG;
  int64_t m = 0;
  int32_t mc = s->P.max_contacts;
  for (int64_t r = 0; r < s->nrig; ++r) {
    int64_t si = s->rig_id[r];
    for (int32_t c = 0; c < s->ct_cnt[r]; ++c) {
      int32_t k = s->ct_partner[r * mc + c];
      if (k <= si) continue;
      if (pairs && delta_t && m < cap) {
        pairs[2 * m] = (int32_t)si;
        pairs[2 * m + 1] = k;
        for (int a = 0; a < 3; ++a) delta_t[3 * m + a] = s->ct_dt[(r * mc + c) * 3 + a];
      }
      ++m;
    }
  }
  *n_contacts = m;
  return (pairs && m > cap) ? ORACLE_E_INVALID_ARG : ORACLE_OK;
}

static int add_contact(oracle_system* s, int64_t i, int64_t j, const double* d,
                       double sign) {
  int64_t r = s->rig_of[i];
  int32_t mc = s->P.max_contacts;
  if (r < 0) return ORACLE_E_INVALID_ARG;
  if (s->ct_cnt[r] >= mc) return ORACLE_E_CONTACT_OVERFLOW;
  int32_t c = s->ct_cnt[r]++;
  s->ct_partner[r * mc + c] = (int32_t)j;
  for (int a = 0; a < 3; ++a) s->ct_dt[(r * mc + c) * 3 + a] = sign * d[a];
  return ORACLE_OK;
}

static int cmp_contact_row(const void* a, const void* b) {
  /* rows are (partner, dt[3]) records packed as doubles for sorting */
  double x = ((const double*)a)[0], y = ((const double*)b)[0];
  return (x > y) - (x < y);
}

int oracle_load_contacts(oracle_system* s, const int32_t* pairs,
                         const double* delta_t, int64_t n_contacts) {
  if (!s || (n_contacts > 0 && (!pairs || !delta_t))) return ORACLE_E_INVALID_ARG;
  for (int64_t r = 0; r < s->nrig; ++r) s->ct_cnt[r] = 0;
  for (int64_t m = 0; m < n_contacts; ++m) {
    int64_t i = pairs[2 * m], j = pairs[2 * m + 1];
    if (i < 0 || j < 0 || i >= s->n || j >= s->n || i == j) return ORACLE_E_INVALID_ARG;
    int rc = add_contact(s, i, j, &delta_t[3 * m], 1.0);
    if (rc) return rc;
    rc = add_contact(s, j, i, &delta_t[3 * m], -1.0);
    if (rc) return rc;
  }
  /* keep each row in ascending partner order */
  int32_t mc = s->P.max_contacts;
  double* tmp = (double*)malloc(sizeof(double) * 4 * (size_t)mc);
  if (!tmp) return ORACLE_E_NOMEM;
  for (int64_t r = 0; r < s->nrig; ++r) {
    int32_t c0 = s->ct_cnt[r];
    for (int32_t c = 0; c < c0; ++c) {
      tmp[4 * c] = (double)s->ct_partner[r * mc + c];
      for (int a = 0; a < 3; ++a) tmp[4 * c + 1 + a] = s->ct_dt[(r * mc + c) * 3 + a];
    }
    qsort(tmp, (size_t)c0, 4 * sizeof(double), cmp_contact_row);
    for (int32_t c = 0; c < c0; ++c) {
      s->ct_partner[r * mc + c] = (int32_t)tmp[4 * c];
      for (int a = 0; a < 3; ++a) s->ct_dt[(r * mc + c) * 3 + a] = tmp[4 * c + 1 + a];
    }
  }
  free(tmp);
  return ORACLE_OK;
}

/* FP64 totals over every particle that is not an outer wall:
 * out = [P(3), L(3) about the origin, KE_trans, KE_rot, max|v|, min rho,
 *        max rho, total mass, step, 0, 0, 0]                            */
int oracle_totals(oracle_system* s, double out[16]) {
  if (!s || !out) return ORACLE_E_INVALID_ARG;
  for (int k = 0; k < 16; ++k) out[k] = 0.0;
  out[9] = INFINITY;
  out[10] = -INFINITY;
  for (int64_t i = 0; i < s->n; ++i) {
    if (s->type[i] == O_OUTER_WALL) continue;
    const double* x = &s->pos[3 * i];
    const double* v = &s->vel[3 * i];
    const double* w = &s->w[3 * i];
    double m = s->mass[i], I = s->iner[i];
    for (int a = 0; a < 3; ++a) out[a] += m * v[a];
    out[3] += m * (x[1] * v[2] - x[2] * v[1]) + I * w[0];
    out[4] += m * (x[2] * v[0] - x[0] * v[2]) + I * w[1];
    out[5] += m * (x[0] * v[1] - x[1] * v[0]) + I * w[2];
    double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    out[6] += 0.5 * m * v2;
    out[7] += 0.5 * I * (w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    if (sqrt(v2) > out[8]) out[8] = sqrt(v2);
    if (s->rho[i] < out[9]) out[9] = s->rho[i];
    if (s->rho[i] > out[10]) out[10] = s->rho[i];
    out[11] += m;
  }
  out[12] = (double)s->step;
  return ORACLE_OK;
}

int64_t oracle_get_step(const oracle_system* s) { return s ? s->step : -1; }

/* pressure tensor of the box (R20): kinetic part from the current
 * velocities, virial from the last force evaluation */
int oracle_stress(oracle_system* s, double out[9]) {
  if (!s || !out) return ORACLE_E_INVALID_ARG;
  const oracle_params* P = &s->P;
  double V = P->L[0] * P->L[1] * P->L[2];
  double zmid = P->org[2] + 0.5 * P->L[2];
  double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t i = 0; i < s->n; ++i) {
    if (s->type[i] == O_OUTER_WALL) continue;
    double v[3] = {s->vel[3 * i], s->vel[3 * i + 1], s->vel[3 * i + 2]};
    v[0] -= P->shear_rate * (s->pos[3 * i + 2] - zmid);
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b)
        acc[3 * a + b] += s->mass[i] * v[a] * v[b] + s->vir[9 * i + 3 * a + b];
  }
  for (int k = 0; k < 9; ++k) out[k] = acc[k] / V;
  return ORACLE_OK;
}

int oracle_num_threads(void) { return omp_get_max_threads(); }

void oracle_set_num_threads(int n) {
  if (n > 0) omp_set_num_threads(n);
}
