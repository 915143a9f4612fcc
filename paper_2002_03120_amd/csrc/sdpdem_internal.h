// sdpdem_internal.h -- device data layout and kernel launchers of the
// SDPD-DEM library (shared by the kernel and host translation units).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "sdpdem.h"

namespace sdpdem {

static constexpr int BS = 256;  // threads per block of the particle kernels
// coupling slots per fluid particle: the spheres whose support holds it,
// each with its kernel weight, filled by the action for the reaction
static constexpr int RXN_CAP = 16;
// candidate rounds (64 lanes each) of a sphere's coupling search that the
// action records for the next pass; a longer search is repeated instead
static constexpr int ACT_ROUNDS = 16;

enum : uint8_t { T_FLUID = 0, T_RIGID = 1, T_INNER = 2, T_OUTER = 3 };

// status bits raised by kernels (sticky until the system is destroyed)
enum : int {
  ST_NBR_OVERFLOW = 1,
  ST_CONTACT_OVERFLOW = 2,
  ST_NONFINITE = 4,
  ST_OUT_OF_DOMAIN = 8
};

struct __align__(32) D4 {
  double x, y, z, w;
};
struct __align__(16) F4 {
  float x, y, z, w;
};

// Pair record of one particle for the SDPD force pass, 64 bytes (half a
// cache line, four 16-byte loads): FP64 position, FP32 velocity,
// c_C p~/d^2, spin, 1/d with d = rho/m_f, and the id.  Written with the
// pressure filter after every neighbour build; the velocity and spin are
// refreshed after the second half-kick.
struct __align__(64) PR {
  double x, y, z;
  float vx, vy, vz, pc;
  float wx, wy, wz, invd;
  int gid, type;
};
static_assert(sizeof(PR) == 64, "pair record must be 64 bytes");

// A uniform cell grid.  Periodic axes span [org, org+L) with nc >= 3 cells;
// wall axes span the particle bounding box plus one cell of slack.  Cell
// keys are linear, x fastest.
struct Grid {
  double lo[3];
  double cs[3];
  double inv_cs[3];
  int nc[3];
  int per[3];
  int ncells;
};

// One box of a batch: an independent domain with its own periodic or wall
// axes, optional Lees-Edwards shear (flow x, gradient z), thermal energy and
// noise key, and its own fluid and rigid cell grids.  The boxes' cells are
// numbered consecutively (cell_off, rcell_off), so the counting sort puts
// the particles of a box into one fixed contiguous range [first, first +
// count) of the sorted arrays.
struct BoxD {
  double org[3], L[3], halfL[3];
  double shear;       // shear rate (0: plain images)
  double le_jump;     // shear * L_z: x velocity of the image above
  double le_shift;    // x offset of the image above at the current position time
  double le_next;     // the same at the time the drift of this step moves to
  double vol;         // L_x L_y L_z
  Grid g, rg;         // fluid and rigid grids (local cell numbers)
  int per[3];
  int le;             // shear != 0
  int cell_off, rcell_off;
  int first, count;   // sorted particle range
  int nact;           // its first nact particles move or feel forces; the rest are outer walls
  int wall_off;       // outer walls bin into cells cell_off + wall_off + c (0: the box has none)
  int blk_first;      // the box's first entry in the launch-block table
  int dem_reach;      // rigid-grid cells to search for DEM partners
  double couple_R;    // R_max + h: coupling partners lie within it
  // candidate reuse under shear: the flow brings two particles at most
  // shear_reach t closer (|shear| (R_max + h + skin)); the coupling search
  // reaches act_margin farther, the flow's largest drift before a search
  double shear_reach, act_margin;
  double dem_R;       // 2 R_max + h: DEM and lubrication partners lie within it
  int noise;          // thermal forces on
  float kTf;
  uint32_t key0, key1;
  uint32_t id_base;   // smallest id in the box: noise counters use ids above it
};

// The part of a box the pair loops need, copied into registers once per
// thread (the box table itself could alias the loops' stores).
struct Geo {
  double L[3], halfL[3];
  double lim[3];  // halfL on a periodic axis, infinite on a wall axis
  double inv_Lx;  // 1 / L_x: the sheared x image without a division
  double le_shift, le_jump;
  int per[3];
  int le;
};

// Everything a kernel reads, passed by value.  Particle arrays are in the
// current cell-sorted order; rigid arrays are indexed by rigid slot (the
// rank of the rigid particle's id among all rigid ids).
struct Dev {
  int n, nr, npad, maxn, maxc;
  int nbox;
  int have_rxn;  // the drag reaction of the last evaluation is valid
  int stress;    // accumulate the pair virial of the force pass
  // constants
  int noslip;
  double h, h2, inv_h, dx, lever;
  double rho0, p0, alpha, beta, p_ref, m_f, I_f;
  double cw_m;    // C_W * m_f, density per unit kernel sum
  double w_norm;  // 105 / (16 pi h^3)
  double W0;      // W(0)
  double eta, dt, body[3];
  int gtype, gaxis;
  double E, nu, mu, damp, eps_min, lub_gap_min;
  int lub;
  int clamp;   // negative pressure -> 0
  int smooth;  // Shepard filter of the pressure
  // single-precision pair constants
  float kAf, kBf, kRf;  // folded coefficients of the pair force
  double coef_c;
  float hf, inv_hf, cFf, CAf, CBf, inv_sqrt_dtf, cC, cD, cR, cT, leverf;
  int ncells_all, rncells_all;  // cells of all boxes
  const BoxD* boxes;
  const int2* blk;   // per launch block: (box, first sorted index); box -1 = idle
  int nblk;          // launch blocks: 8 x whole numbers of chunks
  int blk_per;       // launch blocks per chunk
  const int2* ablk;  // the same over the boxes' active parts (outer walls left out)
  int nablk, ablk_per;
  const int* rbox;   // box of every rigid slot
  // particles (current buffer)
  D4* pos;  // x, y, z, radius (lever for fluid and walls)
  D4* vel;  // vx, vy, vz, mass
  D4* om;   // wx, wy, wz, inertia
  uint8_t* type;
  int* gid;
  // sort scratch
  uint32_t* key;
  int* count;
  int* cstart;  // ncells_all + 1
  int* rank;  // per particle: its arrival order in its cell at binning
  int* perm;
  // neighbours and fields
  int* nbr;  // [maxn * npad], neighbour k of particle i at k*npad + i
  int* nbr_cnt;
  // candidate reuse (skin > 0): the partners within h + skin found by the
  // last cell-grid search, in the same column-major form, the positions of
  // that search, and a flag raised by a drift that moved a particle more
  // than skin/2 from them
  int reuse;
  int any_le;      // some box is sheared
  int maxcand;
  double hc, hc2;  // h + skin and its square
  double pad;      // skin/2: how far a particle may be from its cell
  double mv2;      // the flag's threshold: (skin/2)^2, slightly less
  int* cand;       // [maxcand * npad]
  int* cand_cnt;
  D4* xref;
  int* moved;
  // the step whose drift made the positions of the last search (candidate
  // reuse under shear): a drift at step m is (m - sstep) dt later
  int64_t* sstep;
  double* rho;
  double* p;
  D4* xp;   // x, y, z, p of the last build: the pressure filter's neighbour record
  float* ps;
  PR* prec;  // pair records, sorted order
  float* fout;  // 13 planes of npad: F_sdpd(3) N_sdpd(3) F_cd(3) F_rxn(3) W_zx
  // rigid
  int* gid2slot;
  int* rig_sorted;
  int* rig_gid;
  double* f_dg;
  double* f_pg;
  double* f_dem;
  double* f_lub;
  double* n_dem;
  double* eps;
  double* omega;
  double* wzx_r;  // virial W_zx of every rigid slot: [2 s] coupling, [2 s + 1] contacts
  uint32_t* rkey;
  int* rcount;
  int* rstart;
  int* rcursor;
  int* ritems;
  // rigid records in rigid-grid cell order (index t = position in ritems)
  D4* rpos_c;
  D4* rvel_c;
  D4* rom_c;
  D4* rdg_c;       // F^DG / Omega x Lucy normalisation of H_s; w = 1/H_s (0: no coupling)
  // the coupling pairs of the current positions and order (filled by the
  // action of the first pass after a neighbour build, cleared before it):
  int* rxn_cnt;    // spheres whose support holds the particle (0: uncoupled)
  int2* rxn_slot;  // [RXN_CAP][npad]: (cell-ordered sphere record, FP32 Lucy polynomial)
  // per cell-ordered sphere record: the fluid particle of every lane and
  // round of its search (-1: none), and (rounds or -1, rigid centres in H_s)
  int* act_list;  // [nr][ACT_ROUNDS * 64]
  int2* act_meta;
  // per cell-ordered sphere record: the action's sums Omega_s, sum w v (3),
  // sum w (F^C + F^D) (3) and the lever sum w r_z, for the finishing kernel
  double* act_sum;  // [nr][8]
  // device-resident step number (so that a captured graph replays correctly)
  int64_t* dstep;
  int* ct_cnt;      // current contact table
  int* ct_partner;  // partner id
  double* ct_dt;
  // per-box pressure-tensor samples: P_zx now, its running sum and count
  double* st_inst;
  double* st_sum;
  double* st_part;  // per launch block: its particles' share of P_zx V
  int* status;
};

// host-side launchers (sdpdem_kernels.hip)
void launch_fill_i32(int* a, int v, size_t count, hipStream_t st);
void launch_fill_f64(double* a, double v, size_t count, hipStream_t st);
// *dst = *src, dst in host-visible memory
void launch_publish(const int* src, int* dst, hipStream_t st);
void launch_bin(const Dev& d, hipStream_t st);
void launch_bin_rigid(const Dev& d, hipStream_t st);
// exclusive scan of count[0..m) into start[0..m] and (unless null)
// cursor[0..m); count is left all zero, ready for the next binning
void launch_scan(int* count, int m, int* start, int* cursor, int* block_sums,
                 hipStream_t st);
int scan_block_sums_size(int m);
void launch_scatter(const uint32_t* key, int n, int* cursor, int* perm, hipStream_t st);
// perm[start[key[i]] + rank[i]] = i (the ranks the binning handed out)
void launch_scatter_ranked(const uint32_t* key, const int* rank, int n, const int* start,
                           int* perm, hipStream_t st);
// sort each cell's slice of perm by sortkey[perm[k]] (sortkey == null: by value)
void launch_cell_sort(const int* start, int ncells, int* perm, const int* sortkey,
                      hipStream_t st);
void launch_permute(const Dev& d, const D4* spos, const D4* svel, const D4* som,
                    const uint8_t* stype, const int* sgid, hipStream_t st);
// the cell-grid search; with cand (reuse on) also the candidates within
// h + skin and the positions they were found at
void launch_build_density(const Dev& d, bool cand, bool after_drift, hipStream_t st);
// the lists, density and pressure from the candidates of the last search
void launch_filter_density(const Dev& d, hipStream_t st);
// start of a pass: Lees-Edwards offsets of every box for positions at step
// *dstep + add and, with clear_rxn, the reaction's slot counts set to zero
void launch_pass_prep(const Dev& d, BoxD* boxes, int add, bool clear_rxn, hipStream_t st);
// per-box sample of P_zx; with accumulate, also added to the running sums
void launch_box_stress(const Dev& d, int accumulate, hipStream_t st);
void launch_smooth(const Dev& d, bool all, hipStream_t st);
// with t0 and t1, the launch records the two timing events itself
void launch_fluid_forces(const Dev& d, bool noise, hipStream_t st, hipEvent_t t0 = nullptr,
                         hipEvent_t t1 = nullptr);
void launch_rigid_gather(const Dev& d, hipStream_t st);
// the coupling action (the per-sphere gather, then the per-sphere drag and
// pressure-gradient algebra); with fill it also refills the reaction's
// slots (counts cleared) and, unless use_rec, searches and records every
// sphere's partners; use_rec: the partners come from the records of the
// last sort (every particle within skin/2 of where that sort saw it)
void launch_fpi_action(const Dev& d, bool fill, bool use_rec, hipStream_t st);
void launch_fpi_reaction(const Dev& d, hipStream_t st);
void launch_dem(const Dev& d, int commit, int* nxt_cnt, int* nxt_partner, double* nxt_dt,
                hipStream_t st);
// with end_step, block 0 also advances the device step counter; with
// fuse_rxn the launch also forms the drag reaction (launch_fpi_reaction's
// work) of the coupled fluid particles; with track_moved the drift raises
// the moved flag of candidate reuse
void launch_integrate(const Dev& d, int velver, int rigid_active, bool end_step, bool fuse_rxn,
                      bool track_moved, hipStream_t st);
void launch_read_field(const Dev& d, int field, int rigid_active, double* out, hipStream_t st);
int totals_partial_blocks(int n);
void launch_totals(const Dev& d, double* partial, double* out, hipStream_t st);
// neighbour columns k0..k0+kn-1 as ids (-1 past a row's end)
void launch_nbr_cols(const Dev& d, int k0, int kn, int* out, hipStream_t st);

}  // namespace sdpdem
