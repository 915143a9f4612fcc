// sdpdem_api.hip -- host side of the C ABI declared in include/sdpdem.h:
// validation, workspace layout, the per-step launch sequence of
// Algorithms 1 and 2, read-out and diagnostics.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include "sdpdem_internal.h"

using namespace sdpdem;

struct sdpdem_system {
  sdpdem_params P;
  Dev d;
  D4* pos[2];
  D4* vel[2];
  D4* om[2];
  uint8_t* type[2];
  int* gid[2];
  int cur = 0;
  int* ct_cnt[2];
  int* ct_partner[2];
  double* ct_dt[2];
  int ct_cur = 0;
  int* block_sums;
  int* rblock_sums;
  double* field_buf;
  double* tot_part;
  double* tot_out;
  int64_t step = 0;
  bool cache_valid = false;
  // candidate reuse: the candidates and reference positions of a cell-grid
  // search are in place; capturing (every step searches inside a graph);
  // searches and reusing list builds so far
  bool cand_valid = false;
  // the coupling action's per-sphere records hold the partners of every
  // sphere (within H_s + skin) at the current sorted order
  bool rec_valid = false;
  bool capturing = false;
  int64_t searches = 0, reuses = 0;
  // pinned host word the moved flag is copied into, and the event the host
  // polls for that copy (null: a pageable copy and a stream synchronisation)
  int* h_moved = nullptr;
  hipEvent_t ev_moved = nullptr;
  bool fork_marked = false;  // ev_fork already marks the coming build's fork point
  // the reaction's slots hold the coupling pairs of the current positions
  // and sorted order (a neighbour build invalidates them)
  bool rxn_valid = false;
  bool noise = false;
  bool stress = false;
  int64_t stress_samples = 0;
  // captured step loop (graph_steps steps, an even number, per launch)
  int graph_steps = 0;
  hipGraphExec_t gexec = nullptr;
  bool g_act = false, g_stress = false, g_rxn = false, g_rec = false;
  // a second stream of the library's own for work that does not depend on
  // what runs beside it (the rigid grid, the sphere records, the contacts),
  // forked from the caller's stream and joined back into it within the
  // same build or pass (null: one stream)
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_gather = nullptr, ev_join = nullptr;
  int64_t graph_steps_run = 0;  // steps replayed from graphs so far
  // the coming pass's sphere records and contacts are enqueued already
  // (by the build), on the side stream if side_open, whose records event
  // was recorded if gather_ok
  bool rigid_issued = false, side_open = false, gather_ok = true;
  int g_cur = 0, g_ct = 0;  // buffer parity the graph was captured with
  BoxD* boxes = nullptr;  // device copy of the box table
  std::vector<BoxD> h_boxes;
  std::vector<int> h_gid2slot;
  // profiling
  int prof_kernel = SDPDEM_K_NONE;
  int prof_every = 1;      // time the first of every prof_every launches
  int64_t prof_seen = 0;   // launches of the profiled kernel so far
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  size_t ev_used = 0;
  double prof_ms = 0.0;
  int64_t prof_n = 0;
};

namespace {

constexpr double kPi = 3.14159265358979323846;

struct Bump {
  char* base;
  size_t off = 0;
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T* p = reinterpret_cast<T*>(base ? base + off : nullptr);
    off += std::max<size_t>(count, 1) * sizeof(T);
    return p;
  }
};

bool valid_params(const sdpdem_params* P) {
  if (!P) return false;
  if (!(P->h > 0) || !(P->dx > 0) || !(P->dt > 0) || !(P->rho0 > 0) || !(P->mass_fluid > 0) ||
      !(P->inertia_fluid > 0) || !(P->kBT >= 0) || !(P->eta >= 0))
    return false;
  if (P->max_neighbors < 1 || P->max_contacts < 1) return false;
  if (P->xi < 40.0 * P->eta / 51.0 || P->xi > 5.0 * P->eta / 3.0) return false;
  if (P->gravity_axis < 0 || P->gravity_axis > 2) return false;
  if (P->cell_factor != 0.0 && !(P->cell_factor >= 0.25 && P->cell_factor <= 16.0)) return false;
  // a candidate margin up to h/2 keeps h + skin within half of a periodic
  // axis (L >= 3h), where the minimum image is the only one
  if (!(P->skin >= 0.0 && P->skin <= 0.5 * P->h)) return false;
  return true;
}

bool valid_box(const sdpdem_params* P, const sdpdem_box& b) {
  for (int a = 0; a < 3; ++a) {
    if (!(b.L[a] > 0) || !std::isfinite(b.org[a]) || !std::isfinite(b.L[a])) return false;
    if (b.periodic[a] && b.L[a] < 3.0 * P->h * (1.0 + 1e-6)) return false;
  }
  if (!(b.kBT >= 0) || !std::isfinite(b.kBT) || !std::isfinite(b.shear_rate)) return false;
  if (b.shear_rate != 0.0 && (!b.periodic[0] || !b.periodic[1] || !b.periodic[2])) return false;
  return true;
}

bool valid_particles(const sdpdem_particles* q, std::vector<int>* slot_of, int* nrig,
                     double* rmax) {
  if (!q || q->n < 1 || q->n > (int64_t)1 << 30 || !q->id || !q->type || !q->pos || !q->vel ||
      !q->angvel || !q->mass || !q->inertia || !q->radius)
    return false;
  int64_t n = q->n;
  std::vector<char> seen((size_t)n, 0);
  int nr = 0;
  double rm = 0.0;
  for (int64_t k = 0; k < n; ++k) {
    int64_t g = q->id[k];
    if (g < 0 || g >= n || seen[(size_t)g] || q->type[k] > SDPDEM_OUTER_WALL) return false;
    seen[(size_t)g] = 1;
    if (q->type[k] == SDPDEM_RIGID) {
      if (!(q->mass[k] > 0) || !(q->inertia[k] > 0) || !(q->radius[k] > 0)) return false;
      ++nr;
      rm = std::max(rm, q->radius[k]);
    }
  }
  if (slot_of) {
    std::vector<uint8_t> t_by_id((size_t)n);
    for (int64_t k = 0; k < n; ++k) t_by_id[(size_t)q->id[k]] = q->type[k];
    slot_of->assign((size_t)n, -1);
    int s = 0;
    for (int64_t g = 0; g < n; ++g)
      if (t_by_id[(size_t)g] == SDPDEM_RIGID) (*slot_of)[(size_t)g] = s++;
  }
  *nrig = nr;
  *rmax = rm;
  return true;
}

// Cell grid of one box: periodic axes are split into floor(L/cs0) equal
// cells; wall axes cover the box and every one of its particles with one
// cell of slack.
bool make_grid(const sdpdem_box& B, const sdpdem_particles& q, const std::vector<int64_t>& rows,
               double cs0, Grid& g) {
  double total = 1.0;
  for (int a = 0; a < 3; ++a) {
    g.per[a] = B.periodic[a] ? 1 : 0;
    if (g.per[a]) {
      int nc = (int)std::floor(B.L[a] / cs0);
      if (nc < 1) nc = 1;
      g.lo[a] = B.org[a];
      g.nc[a] = nc;
      g.cs[a] = B.L[a] / nc;
    } else {
      double mn = B.org[a], mx = B.org[a] + B.L[a];
      for (int64_t k : rows) {
        double x = q.pos[3 * k + a];
        if (!std::isfinite(x)) return false;
        mn = std::min(mn, x);
        mx = std::max(mx, x);
      }
      g.lo[a] = mn - cs0;
      g.cs[a] = cs0;
      double ncd = std::floor((mx - g.lo[a]) / cs0) + 2.0;
      if (ncd > 1e8) return false;
      g.nc[a] = (int)ncd;
    }
    g.inv_cs[a] = 1.0 / g.cs[a];
    total *= g.nc[a];
  }
  if (total > 1.0e9) return false;
  g.ncells = g.nc[0] * g.nc[1] * g.nc[2];
  return true;
}

double lucy(double r, double h) {
  if (r >= h) return 0.0;
  double q = r / h, om = 1.0 - q;
  return 105.0 / (16.0 * kPi * h * h * h) * (1.0 + 3.0 * q) * om * om * om;
}

// sum of W(|k| dx) over the simple cubic lattice, the particle itself included
double lattice_sum(double h, double dx) {
  int K = (int)std::ceil(h / dx) + 1;
  double s = 0.0;
  for (int a = -K; a <= K; ++a)
    for (int b = -K; b <= K; ++b)
      for (int c = -K; c <= K; ++c) s += lucy(dx * std::sqrt((double)(a * a + b * b + c * c)), h);
  return s;
}

struct Sizes {
  int64_t n, npad, nr;
  int maxn, maxc;
  int maxcand = 0;  // candidate row capacity (0: no reuse)
  int nbox = 1;
  int64_t ncells_all = 0, rncells_all = 0;
  std::vector<BoxD> boxes;
  std::vector<int2> blk;       // launch blocks (box, first sorted index)
  int blk_per = 1;             // launch blocks per chunk (logical_block)
  std::vector<int2> ablk;      // the same over the boxes' active parts
  int ablk_per = 1;
  std::vector<int> rbox;       // box of every rigid slot
  std::vector<int64_t> order;  // initial sorted position -> input row
};

// Carve the workspace (base == nullptr: only measure it).
size_t layout(const Sizes& z, char* base, sdpdem_system* s) {
  Bump b{base};
  size_t n = (size_t)z.n, np = (size_t)z.npad, nr = (size_t)z.nr;
  size_t nc = (size_t)z.ncells_all, rnc = (size_t)z.rncells_all;
  D4 *pos0 = b.take<D4>(np), *pos1 = b.take<D4>(np);
  D4 *vel0 = b.take<D4>(np), *vel1 = b.take<D4>(np);
  D4 *om0 = b.take<D4>(np), *om1 = b.take<D4>(np);
  uint8_t *ty0 = b.take<uint8_t>(np), *ty1 = b.take<uint8_t>(np);
  int *gid0 = b.take<int>(np), *gid1 = b.take<int>(np);
  uint32_t* key = b.take<uint32_t>(np);
  int* count = b.take<int>(nc);
  int* cstart = b.take<int>(nc + 1);
  int* rank = b.take<int>(np);
  int* perm = b.take<int>(np);
  int* bsum = b.take<int>((size_t)scan_block_sums_size((int)nc) + 1);
  int* nbr = b.take<int>((size_t)z.maxn * np);
  int* nbr_cnt = b.take<int>(np);
  int* cand = b.take<int>(z.maxcand ? (size_t)z.maxcand * np : 1);
  int* cand_cnt = b.take<int>(z.maxcand ? np : 1);
  D4* xref = b.take<D4>(z.maxcand ? np : 1);
  double* rho = b.take<double>(np);
  double* p = b.take<double>(np);
  D4* xp = b.take<D4>(np);
  float* ps = b.take<float>(np);
  PR* prec = b.take<PR>(np);
  float* fout = b.take<float>(13 * np);
  int* gid2slot = b.take<int>(np);
  int* rig_sorted = b.take<int>(nr);
  int* rig_gid = b.take<int>(nr);
  double* f_dg = b.take<double>(3 * nr);
  double* f_pg = b.take<double>(3 * nr);
  double* f_dem = b.take<double>(3 * nr);
  double* f_lub = b.take<double>(3 * nr);
  double* n_dem = b.take<double>(3 * nr);
  double* eps = b.take<double>(nr);
  double* omega = b.take<double>(nr);
  double* wzx_r = b.take<double>(2 * nr);
  BoxD* boxes = b.take<BoxD>((size_t)z.nbox);
  int2* blk = b.take<int2>(z.blk.size());
  int2* ablk = b.take<int2>(z.ablk.size());
  int* rbox = b.take<int>(nr);
  double* st_inst = b.take<double>((size_t)z.nbox);
  double* st_part = b.take<double>(z.blk.size());
  double* st_sum = b.take<double>((size_t)z.nbox);
  uint32_t* rkey = b.take<uint32_t>(nr);
  int* rcount = b.take<int>(rnc);
  int* rstart = b.take<int>(rnc + 1);
  int* rcursor = b.take<int>(rnc);
  int* ritems = b.take<int>(nr);
  int* rbsum = b.take<int>((size_t)scan_block_sums_size((int)rnc) + 1);
  D4* rpos_c = b.take<D4>(nr);
  D4* rvel_c = b.take<D4>(nr);
  D4* rom_c = b.take<D4>(nr);
  D4* rdg_c = b.take<D4>(nr);
  int* rxn_cnt = b.take<int>(nr ? np : 1);
  int2* rxn_slot = b.take<int2>(nr ? (size_t)RXN_CAP * np : 1);
  int* act_list = b.take<int>(nr ? (size_t)nr * ACT_ROUNDS * 64 : 1);
  int2* act_meta = b.take<int2>(nr ? nr : 1);
  double* act_sum = b.take<double>(nr ? 8 * (size_t)nr : 1);
  int64_t* dstep = b.take<int64_t>(1);
  int *ctc0 = b.take<int>(nr), *ctc1 = b.take<int>(nr);
  int *ctp0 = b.take<int>(nr * z.maxc), *ctp1 = b.take<int>(nr * z.maxc);
  double *ctd0 = b.take<double>(3 * nr * z.maxc), *ctd1 = b.take<double>(3 * nr * z.maxc);
  int* status = b.take<int>(64);
  double* field_buf = b.take<double>(3 * n);
  double* tot_part = b.take<double>(13 * (size_t)totals_partial_blocks((int)n));
  double* tot_out = b.take<double>(16);
  size_t total = b.off + 256;
  if (s) {
    s->pos[0] = pos0;
    s->pos[1] = pos1;
    s->vel[0] = vel0;
    s->vel[1] = vel1;
    s->om[0] = om0;
    s->om[1] = om1;
    s->type[0] = ty0;
    s->type[1] = ty1;
    s->gid[0] = gid0;
    s->gid[1] = gid1;
    s->ct_cnt[0] = ctc0;
    s->ct_cnt[1] = ctc1;
    s->ct_partner[0] = ctp0;
    s->ct_partner[1] = ctp1;
    s->ct_dt[0] = ctd0;
    s->ct_dt[1] = ctd1;
    s->block_sums = bsum;
    s->rblock_sums = rbsum;
    s->field_buf = field_buf;
    s->tot_part = tot_part;
    s->tot_out = tot_out;
    Dev& d = s->d;
    d.key = key;
    d.count = count;
    d.cstart = cstart;
    d.rank = rank;
    d.perm = perm;
    d.nbr = nbr;
    d.nbr_cnt = nbr_cnt;
    d.cand = cand;
    d.cand_cnt = cand_cnt;
    d.xref = xref;
    d.rho = rho;
    d.p = p;
    d.xp = xp;
    d.ps = ps;
    d.prec = prec;
    d.fout = fout;
    d.gid2slot = gid2slot;
    d.rig_sorted = rig_sorted;
    d.rig_gid = rig_gid;
    d.f_dg = f_dg;
    d.f_pg = f_pg;
    d.f_dem = f_dem;
    d.f_lub = f_lub;
    d.n_dem = n_dem;
    d.eps = eps;
    d.omega = omega;
    d.wzx_r = wzx_r;
    s->boxes = boxes;
    d.boxes = boxes;
    d.blk = blk;
    d.ablk = ablk;
    d.rbox = rbox;
    d.st_inst = st_inst;
    d.st_part = st_part;
    d.st_sum = st_sum;
    d.rkey = rkey;
    d.rcount = rcount;
    d.rstart = rstart;
    d.rcursor = rcursor;
    d.ritems = ritems;
    d.status = status;
    d.moved = status + 32;  // its own 128-byte half of the status block
    d.sstep = reinterpret_cast<int64_t*>(status + 34);
    d.rpos_c = rpos_c;
    d.rvel_c = rvel_c;
    d.rom_c = rom_c;
    d.rdg_c = rdg_c;
    d.rxn_cnt = rxn_cnt;
    d.rxn_slot = rxn_slot;
    d.act_list = act_list;
    d.act_meta = act_meta;
    d.act_sum = act_sum;
    d.dstep = dstep;
  }
  return total;
}

// XCD x runs launch blocks x, x + 8, x + 16, ...; logical_block gives it
// chunks x, x + 8, ... of consecutive table entries, at most max_chunks per
// XCD and at least about a dozen entries long.  Pads the table with idle
// entries to whole rounds of chunks; returns the chunk length.
int pad_chunks(std::vector<int2>& t, size_t max_chunks) {
  const size_t m = std::max<size_t>(1, std::min<size_t>(max_chunks, t.size() / (8 * 12)));
  while (t.size() < 8 * m || t.size() % (8 * m)) t.push_back(make_int2(-1, 0));
  return (int)(t.size() / (8 * m));
}

bool plan(const sdpdem_params* P, const sdpdem_box* boxes, int nbox,
          const sdpdem_particles* q, const int32_t* box_of, Sizes& z,
          std::vector<int>* slot_of) {
  if (!valid_params(P) || !boxes || nbox < 1 || nbox > (1 << 20)) return false;
  for (int b = 0; b < nbox; ++b)
    if (!valid_box(P, boxes[b])) return false;
  int nr = 0;
  double rmax_all = 0.0;
  std::vector<int> slots;
  if (!valid_particles(q, &slots, &nr, &rmax_all)) return false;
  const int64_t n = q->n;
  std::vector<std::vector<int64_t>> rows((size_t)nbox);
  for (int64_t k = 0; k < n; ++k) {
    int b = box_of ? box_of[k] : 0;
    if (b < 0 || b >= nbox) return false;
    rows[(size_t)b].push_back(k);
  }
  z.n = n;
  z.npad = (n + 63) / 64 * 64;
  z.nr = nr;
  z.maxn = P->max_neighbors;
  z.maxc = P->max_contacts;
  if (P->skin > 0.0) {
    // rows grow with the volume of the search sphere
    const double g = (P->h + P->skin) / P->h;
    const double mc = std::ceil((double)P->max_neighbors * g * g * g);
    if (mc > (double)(1 << 20)) return false;
    z.maxcand = (int)mc;
  }
  z.nbox = nbox;
  z.boxes.assign((size_t)nbox, BoxD{});
  z.blk.clear();
  z.ablk.clear();
  z.rbox.assign((size_t)nr, 0);
  z.order.clear();
  z.order.reserve((size_t)n);
  int64_t coff = 0, rcoff = 0, first = 0;
  for (int b = 0; b < nbox; ++b) {
    const sdpdem_box& hb = boxes[b];
    auto& r = rows[(size_t)b];
    // the initial order before the first sort: the particles that move or
    // feel forces, then the outer walls, ids ascending in each part (the
    // sort keeps the outer walls behind, in cells of their own)
    std::sort(r.begin(), r.end(), [&](int64_t a, int64_t c) {
      const bool wa = q->type[a] == SDPDEM_OUTER_WALL, wc = q->type[c] == SDPDEM_OUTER_WALL;
      return wa != wc ? wc : q->id[a] < q->id[c];
    });
    double rmax = 0.0;
    for (int64_t k : r)
      if (q->type[k] == SDPDEM_RIGID) {
        rmax = std::max(rmax, q->radius[k]);
        z.rbox[(size_t)slots[(size_t)q->id[k]]] = b;
      }
    BoxD& B = z.boxes[(size_t)b];
    for (int a = 0; a < 3; ++a) {
      B.org[a] = hb.org[a];
      B.L[a] = hb.L[a];
      B.halfL[a] = 0.5 * hb.L[a];
      B.per[a] = hb.periodic[a] ? 1 : 0;
    }
    B.shear = hb.shear_rate;
    B.le = hb.shear_rate != 0.0 ? 1 : 0;
    B.le_jump = hb.shear_rate * hb.L[2];
    B.le_shift = 0.0;
    B.le_next = 0.0;
    B.vol = hb.L[0] * hb.L[1] * hb.L[2];
    const double cf = P->cell_factor > 0.0 ? P->cell_factor : 1.0;
    if (!make_grid(hb, *q, r, cf * P->h * (1.0 + 1e-6), B.g)) return false;
    for (int a = 0; a < 3; ++a)
      if (B.per[a] && B.g.nc[a] < 3) return false;
    // rigid grid: cells at least H_max = R_max + h wide, so that the fluid
    // particles coupled to a sphere lie in its 27 neighbouring cells
    if (!make_grid(hb, *q, r, (rmax + P->h) * (1.0 + 1e-6), B.rg)) return false;
    // DEM partners lie within R_s + R_k + h <= 2 R_max + h
    double mincs = std::min(B.rg.cs[0], std::min(B.rg.cs[1], B.rg.cs[2]));
    B.dem_reach = std::max(1, (int)std::ceil((2.0 * rmax + P->h) / mincs * (1.0 + 1e-9)));
    B.couple_R = rmax + P->h;
    // under shear every partner within H_s <= R_max + h now was within
    // H_s + skin at the search while 2 D + (R_max + h + skin) |shear| t <
    // skin (D: the largest drift less the flow's, t: time since the search)
    B.shear_reach = std::fabs(hb.shear_rate) * (rmax + P->h + P->skin);
    B.act_margin = (hb.shear_rate != 0.0 && P->skin > 0.0)
                       ? 0.5 * hb.L[2] * P->skin / (rmax + P->h + P->skin)
                       : 0.0;
    B.dem_R = 2.0 * rmax + P->h;
    int64_t nact = 0;
    for (int64_t k : r) nact += q->type[k] != SDPDEM_OUTER_WALL;
    B.nact = (int)nact;
    B.wall_off = nact < (int64_t)r.size() ? B.g.ncells : 0;
    B.cell_off = (int)coff;
    B.rcell_off = (int)rcoff;
    coff += B.g.ncells + B.wall_off;
    rcoff += B.rg.ncells;
    if (coff > (int64_t)1 << 30 || rcoff > (int64_t)1 << 30) return false;
    B.first = (int)first;
    B.count = (int)r.size();
    first += (int64_t)r.size();
    B.noise = (hb.kBT > 0.0 && P->coeff_t != 0.0) ? 1 : 0;
    B.kTf = (float)hb.kBT;
    B.key0 = (uint32_t)(hb.seed & 0xffffffffu);
    B.key1 = (uint32_t)(hb.seed >> 32);
    int64_t id0 = r.empty() ? 0 : q->id[r[0]];
    for (int64_t k : r) id0 = std::min(id0, q->id[k]);
    B.id_base = (uint32_t)id0;
    B.blk_first = (int)z.blk.size();
    for (int c = 0; c < (B.count + BS - 1) / BS; ++c)
      z.blk.push_back(make_int2(b, B.first + c * BS));
    for (int c = 0; c < (B.nact + BS - 1) / BS; ++c)
      z.ablk.push_back(make_int2(b, B.first + c * BS));
    for (int64_t k : r) z.order.push_back(k);
  }
  // The full table (searches, binning) holds regions without work, such as
  // the outer walls above a dam break's water: interleaved chunks give
  // every XCD a share of each.  The active table has work everywhere: one
  // contiguous eighth per XCD keeps each neighbourhood in one L2.
  z.blk_per = pad_chunks(z.blk, 64);
  z.ablk_per = pad_chunks(z.ablk, 1);
  z.ncells_all = coff;
  z.rncells_all = rcoff;
  if (slot_of) *slot_of = slots;
  return true;
}

// the one box of a plain (non-batched) system, from the parameters
sdpdem_box box_from_params(const sdpdem_params* P) {
  sdpdem_box b{};
  for (int a = 0; a < 3; ++a) {
    b.org[a] = P->org[a];
    b.L[a] = P->L[a];
    b.periodic[a] = P->periodic[a];
  }
  b.shear_rate = P->shear_rate;
  b.kBT = P->kBT;
  b.seed = P->seed;
  return b;
}

void fill_constants(sdpdem_system* s, const Sizes& z) {
  const sdpdem_params& P = s->P;
  Dev& d = s->d;
  d.n = (int)z.n;
  d.nr = (int)z.nr;
  d.npad = (int)z.npad;
  d.maxn = z.maxn;
  d.maxc = z.maxc;
  d.nbox = z.nbox;
  d.nblk = (int)z.blk.size();
  d.blk_per = z.blk_per;
  d.nablk = (int)z.ablk.size();
  d.ablk_per = z.ablk_per;
  d.ncells_all = (int)z.ncells_all;
  d.rncells_all = (int)z.rncells_all;
  d.have_rxn = 0;
  d.stress = 0;
  for (int a = 0; a < 3; ++a) d.body[a] = P.g[a] + P.f[a];
  d.noslip = P.noslip;
  d.h = P.h;
  d.h2 = P.h * P.h;
  d.inv_h = 1.0 / P.h;
  d.reuse = z.maxcand > 0 ? 1 : 0;
  d.any_le = 0;
  for (const BoxD& B : z.boxes) d.any_le |= B.le;
  d.maxcand = z.maxcand;
  d.hc = P.h + P.skin;
  d.hc2 = d.hc * d.hc;
  d.pad = d.reuse ? 0.5 * P.skin : 0.0;
  // a partner within h now was within h + 2 (skin/2) of it at the search;
  // the flag's threshold sits a relative 1e-9 inside skin/2, so that FP64
  // rounding of the distances cannot let a partner escape the candidates
  d.mv2 = (0.5 * P.skin * (1.0 - 1e-9)) * (0.5 * P.skin * (1.0 - 1e-9));
  d.dx = P.dx;
  d.lever = 0.5 * P.dx;
  d.rho0 = P.rho0;
  d.p0 = P.p0;
  d.alpha = P.alpha;
  d.beta = P.beta_eos;
  d.clamp = P.enable_neg_p_clamp ? 1 : 0;
  d.smooth = P.enable_pres_smooth ? 1 : 0;
  double pref = P.p0 * std::pow(1.0, P.alpha) - P.beta_eos;
  if (d.clamp && pref < 0.0) pref = 0.0;
  d.p_ref = pref;
  d.m_f = P.mass_fluid;
  d.I_f = P.inertia_fluid;
  d.cw_m = P.enable_kernel_norm ? P.rho0 / lattice_sum(P.h, P.dx) : P.mass_fluid;
  d.w_norm = 105.0 / (16.0 * kPi * P.h * P.h * P.h);
  d.W0 = d.w_norm;
  d.eta = P.eta;
  d.dt = P.dt;
  d.gtype = P.gravity_type;
  d.gaxis = P.gravity_axis;
  d.E = P.E_dem;
  d.nu = P.nu_dem;
  d.mu = P.mu_fric;
  d.damp = P.dem_damping;
  d.eps_min = P.eps_min;
  d.lub_gap_min = P.lub_gap_min;
  d.lub = P.enable_lub ? 1 : 0;
  d.hf = (float)P.h;
  d.inv_hf = (float)(1.0 / P.h);
  d.cFf = (float)(315.0 / (4.0 * kPi * std::pow(P.h, 5)));
  d.CAf = (float)(20.0 * P.eta / 3.0 - 4.0 * P.xi);
  d.CBf = (float)(17.0 * P.xi - 40.0 * P.eta / 3.0);
  d.inv_sqrt_dtf = (float)(1.0 / std::sqrt(P.dt));
  d.cC = (float)P.coeff_c;
  d.coef_c = P.coeff_c;
  {
    double CA = 20.0 * P.eta / 3.0 - 4.0 * P.xi, CB = 17.0 * P.xi - 40.0 * P.eta / 3.0;
    d.kAf = (float)(-P.coeff_d * CA);
    d.kBf = (float)(-P.coeff_d * (CA + 2.0 * CB) / 3.0);
    d.kRf = (float)(-P.coeff_r * CA * 0.5);
  }
  d.cD = (float)P.coeff_d;
  d.cR = (float)P.coeff_r;
  d.cT = (float)P.coeff_t;
  d.leverf = (float)(0.5 * P.dx);
  s->noise = false;
  for (const BoxD& B : z.boxes) s->noise = s->noise || B.noise;
  s->h_boxes = z.boxes;
}

void bind_current(sdpdem_system* s) {
  Dev& d = s->d;
  d.pos = s->pos[s->cur];
  d.vel = s->vel[s->cur];
  d.om = s->om[s->cur];
  d.type = s->type[s->cur];
  d.gid = s->gid[s->cur];
  d.ct_cnt = s->ct_cnt[s->ct_cur];
  d.ct_partner = s->ct_partner[s->ct_cur];
  d.ct_dt = s->ct_dt[s->ct_cur];
}

// ---- profiling: bracket the launches of one kernel with events ----------

void prof_flush(sdpdem_system* s) {
  if (s->ev_used == 0) return;
  if (hipEventSynchronize(s->ev[s->ev_used - 1].second) != hipSuccess) {
    s->ev_used = 0;  // the samples are lost; the kernel's own error surfaces on its stream
    return;
  }
  for (size_t k = 0; k < s->ev_used; ++k) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, s->ev[k].first, s->ev[k].second) == hipSuccess) {
      s->prof_ms += ms;
      s->prof_n += 1;
    }
  }
  s->ev_used = 0;
}

struct Prof {
  sdpdem_system* s;
  hipStream_t st;
  bool on;
  bool ext;  // the launch records the event pair itself (single-kernel scopes)
  Prof(sdpdem_system* s_, int kid, hipStream_t st_, bool ext_ = false)
      : s(s_), st(st_), on(s_->prof_kernel == kid && s_->prof_seen++ % s_->prof_every == 0),
        ext(ext_) {
    if (!on) return;
    if (s->ev_used == s->ev.size()) {
      if (s->ev.size() < 4096) {
        hipEvent_t a, b;
        if (hipEventCreate(&a) != hipSuccess) {
          on = false;
          return;
        }
        if (hipEventCreate(&b) != hipSuccess) {
          (void)hipEventDestroy(a);
          on = false;
          return;
        }
        s->ev.emplace_back(a, b);
      } else {
        prof_flush(s);
      }
    }
    on = ext || hipEventRecord(s->ev[s->ev_used].first, st) == hipSuccess;
  }
  hipEvent_t t0() const { return on && ext ? s->ev[s->ev_used].first : nullptr; }
  hipEvent_t t1() const { return on && ext ? s->ev[s->ev_used].second : nullptr; }
  ~Prof() {
    if (!on) return;
    if (ext || hipEventRecord(s->ev[s->ev_used].second, st) == hipSuccess) s->ev_used += 1;
  }
};

// ---- the per-step launch sequence ----------------------------------------

// (a1)-(a4): sort by cell, permute the state, neighbours + density +
// pressure, smoothing, and the rigid grid.
// Order the side stream after everything enqueued on st so far; false
// (nothing forked) without a side stream or when the events fail.
bool fork_side(sdpdem_system* s, hipStream_t st) {
  return s->side && hipEventRecord(s->ev_fork, st) == hipSuccess &&
         hipStreamWaitEvent(s->side, s->ev_fork, 0) == hipSuccess;
}

// Order st after everything enqueued on the side stream so far.
void join_side(sdpdem_system* s, hipStream_t st) {
  if (hipEventRecord(s->ev_join, s->side) != hipSuccess ||
      hipStreamWaitEvent(st, s->ev_join, 0) != hipSuccess)
    (void)hipStreamSynchronize(s->side);  // no device-side wait: wait here
}

bool rigid_active(const sdpdem_system* s) {
  return s->d.nr > 0 && s->step >= s->P.itr_actv_rigid;
}

// The coming pass's sphere records and contacts on stream rs (the side
// stream when fk); false if the records' event could not be recorded.
bool issue_rigid(sdpdem_system* s, hipStream_t rs, bool fk, int commit) {
  Dev& d = s->d;
  const int nx = s->ct_cur ^ 1;
  {
    Prof pr(s, SDPDEM_K_RIGID_GRID, rs);
    launch_rigid_gather(d, rs);
  }
  const bool ok = !fk || hipEventRecord(s->ev_gather, rs) == hipSuccess;
  {
    Prof pr(s, SDPDEM_K_DEM, rs);
    launch_dem(d, commit, s->ct_cnt[nx], s->ct_partner[nx], s->ct_dt[nx], rs);
  }
  return ok;
}

// How a build gets its lists: sort and search the cell grid; take them
// from the candidates of the last search (every particle is still within
// skin/2 of where it saw it); or the same with the candidate filter already
// enqueued, and the side stream's fork point marked before it.
enum BuildLists { LISTS_SEARCH, LISTS_FILTER, LISTS_FILTERED };

// The neighbour build; with commit_next >= 0 a force pass with that commit
// flag follows at once, and the build already issues that pass's sphere
// records and contacts (which need only the permuted state).  Without a
// search the particles keep their order and cells.  after_drift: the build
// between a step's two passes (else one ahead of the first pass).
void run_build(sdpdem_system* s, hipStream_t st, int commit_next, int lists = LISTS_SEARCH,
               bool after_drift = false) {
  Dev& d = s->d;
  const int nc = d.ncells_all;
  const bool search = lists == LISTS_SEARCH;
  s->rxn_valid = false;  // the positions (and with a search the order) change
  if (search) s->rec_valid = false;  // the coupling records hold old indices
  if (search) {
    {
      Prof pr(s, SDPDEM_K_BIN, st);
      launch_bin(d, st);  // the counts are zero: set at creation, cleared by the scan
    }
    {
      Prof pr(s, SDPDEM_K_SORT, st);
      launch_scan(d.count, nc, d.cstart, nullptr, s->block_sums, st);
      launch_scatter_ranked(d.key, d.rank, d.n, d.cstart, d.perm, st);
      launch_cell_sort(d.cstart, nc, d.perm, s->gid[s->cur], st);
    }
    const int src = s->cur;
    s->cur ^= 1;
    bind_current(s);
    {
      Prof pr(s, SDPDEM_K_PERMUTE, st);
      launch_permute(d, s->pos[src], s->vel[src], s->om[src], s->type[src], s->gid[src], st);
    }
  }
  // the rigid grid, the sphere records and the contacts need the permuted
  // state only: with a side stream they run there beside the neighbour
  // lists and the pressure filter (the pass joins the side stream).  The
  // fork point is marked before the lists are enqueued and the side work
  // after them, so that the main stream never waits on the host enqueuing
  // the many short rigid launches (it does when a step has just read the
  // moved flag and the queue is empty).
  const bool fk0 = d.nr > 0 && s->side &&
                   (lists == LISTS_FILTERED ? s->fork_marked
                                            : hipEventRecord(s->ev_fork, st) == hipSuccess);
  s->fork_marked = false;
  if (search) {
    // inside a graph no step can reuse candidates: the plain search there
    const bool cand = d.reuse && !s->capturing;
    Prof pr(s, SDPDEM_K_NEIGHBORS_DENSITY, st);
    launch_build_density(d, cand, after_drift, st);
    s->cand_valid = cand;
    s->searches += 1;
  } else {
    if (lists == LISTS_FILTER) {
      Prof pr(s, SDPDEM_K_NEIGHBORS_DENSITY, st);
      launch_filter_density(d, st);
    }
    s->reuses += 1;
  }
  const bool fk = fk0 && hipStreamWaitEvent(s->side, s->ev_fork, 0) == hipSuccess;
  hipStream_t rs = fk ? s->side : st;
  if (d.nr > 0) {
    Prof pr(s, SDPDEM_K_RIGID_GRID, rs);
    launch_bin_rigid(d, rs);
    launch_scan(d.rcount, d.rncells_all, d.rstart, d.rcursor, s->rblock_sums, rs);
    launch_scatter(d.rkey, d.nr, d.rcursor, d.ritems, rs);
    launch_cell_sort(d.rstart, d.rncells_all, d.ritems, nullptr, rs);
  }
  if (commit_next >= 0 && rigid_active(s)) {
    s->gather_ok = issue_rigid(s, rs, fk, commit_next);
    s->rigid_issued = true;
  }
  {
    Prof pr(s, SDPDEM_K_SMOOTH, st);
    launch_smooth(d, search, st);
  }
  if (fk) {
    if (s->rigid_issued)
      s->side_open = true;
    else
      join_side(s, st);
  }
}

// whether the coming pass refills the reaction's slots (its pass_prep then
// clears their counts): after a neighbour build, or when they are stale
bool needs_fill(const sdpdem_system* s, bool build) {
  return rigid_active(s) && (build || !s->rxn_valid);
}

// (a5)-(a9): one force evaluation (Alg. 2) and, if asked, the update; fill
// as needs_fill said before the pass's pass_prep.
void run_pass(sdpdem_system* s, int velver, int commit, bool integrate, bool fill,
              hipStream_t st) {
  Dev& d = s->d;
  const bool act = rigid_active(s);
  // The sphere records and the contacts need neither the SDPD forces nor
  // the coupling, and the coupling needs the records but not the contacts:
  // unless the build already issued them, they run on the side stream
  // beside the pair forces (and the contacts beside the coupling chain).
  bool fk = s->side_open;
  if (act && !s->rigid_issued) {
    fk = fork_side(s, st);
    s->gather_ok = issue_rigid(s, fk ? s->side : st, fk, commit);
  }
  s->rigid_issued = false;
  {
    Prof pr(s, SDPDEM_K_FLUID_FORCES, st, true);
    launch_fluid_forces(d, s->noise, st, pr.t0(), pr.t1());
  }
  if (act) {
    if (fk && (!s->gather_ok || hipStreamWaitEvent(st, s->ev_gather, 0) != hipSuccess))
      (void)hipStreamSynchronize(s->side);  // no device-side wait: wait here
    {
      Prof pr(s, SDPDEM_K_FPI_ACTION, st);
      // a filling pass reads the coupling records when the particles kept
      // the order of the sort the records were made at
      const bool use_rec = fill && s->rec_valid;
      launch_fpi_action(d, fill, use_rec, st);
      if (fill) {
        s->rxn_valid = true;
        s->rec_valid = true;  // a search-based fill records every sphere
      }
    }
    // the reaction of an updating pass is formed inside the update
    if (!integrate) {
      Prof pr(s, SDPDEM_K_FPI_REACTION, st);
      launch_fpi_reaction(d, st);
    }
  }
  if (fk) join_side(s, st);
  s->side_open = false;
  if (act) {
    if (commit) {
      s->ct_cur ^= 1;
      bind_current(s);
    }
    d.have_rxn = 1;
  } else {
    d.have_rxn = 0;
  }
  if (integrate) {
    Prof pr(s, SDPDEM_K_INTEGRATE, st);
    // the second pass of a step also advances the device step counter
    // a captured graph never reads the moved flag: no need to raise it
    launch_integrate(d, velver, act ? 1 : 0, velver == 2, act, d.reuse && !s->capturing, st);
  }
}

int status_code(int bits) {
  if (bits & ST_NONFINITE) return SDPDEM_E_NONFINITE;
  if (bits & ST_NBR_OVERFLOW) return SDPDEM_E_NBR_OVERFLOW;
  if (bits & ST_CONTACT_OVERFLOW) return SDPDEM_E_CONTACT_OVERFLOW;
  if (bits & ST_OUT_OF_DOMAIN) return SDPDEM_E_OUT_OF_DOMAIN;
  return SDPDEM_OK;
}

int sync_status(sdpdem_system* s, hipStream_t st) {
  int bits = 0;
  if (hipMemcpyAsync(&bits, s->d.status, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess)
    return SDPDEM_E_HIP;
  if (hipStreamSynchronize(st) != hipSuccess) return SDPDEM_E_HIP;
  if (hipGetLastError() != hipSuccess) return SDPDEM_E_HIP;
  return status_code(bits);
}

}  // namespace


namespace {

void free_side_stream(sdpdem_system* s) {
  for (hipEvent_t* e : {&s->ev_fork, &s->ev_gather, &s->ev_join}) {
    if (*e) (void)hipEventDestroy(*e);
    *e = nullptr;
  }
  if (s->side) (void)hipStreamDestroy(s->side);
  s->side = nullptr;
}

// The side stream (default priority) and its events; without them every
// build and pass stays on the caller's stream.
void make_side_stream(sdpdem_system* s) {
  if (hipStreamCreateWithFlags(&s->side, hipStreamNonBlocking) != hipSuccess) {
    s->side = nullptr;
    return;
  }
  for (hipEvent_t* e : {&s->ev_fork, &s->ev_gather, &s->ev_join})
    if (hipEventCreateWithFlags(e, hipEventDisableTiming) != hipSuccess) {
      *e = nullptr;
      free_side_stream(s);
      return;
    }
}

int create_impl(const sdpdem_params* params, const sdpdem_box* boxes, int nbox,
                const sdpdem_particles* q, const int32_t* box_of, void* d_workspace,
                size_t workspace_bytes, void* hip_stream, sdpdem_system** out,
                bool side_stream = true) {
  if (!out) return SDPDEM_E_INVALID_ARG;
  *out = nullptr;
  Sizes z;
  std::vector<int> slot_of;
  if (!plan(params, boxes, nbox, q, box_of, z, &slot_of)) return SDPDEM_E_INVALID_ARG;
  size_t need = layout(z, nullptr, nullptr);
  if (!d_workspace) return SDPDEM_E_INVALID_ARG;
  if (workspace_bytes < need) return SDPDEM_E_WORKSPACE_TOO_SMALL;
  char* base = reinterpret_cast<char*>(((uintptr_t)d_workspace + 255) & ~(uintptr_t)255);
  if ((size_t)(base - (char*)d_workspace) + need - 256 > workspace_bytes)
    return SDPDEM_E_WORKSPACE_TOO_SMALL;
  sdpdem_system* s = new (std::nothrow) sdpdem_system();
  if (!s) return SDPDEM_E_INVALID_ARG;
  s->P = *params;
  layout(z, base, s);
  fill_constants(s, z);
  s->step = params->itr_start;
  s->cur = 0;
  s->ct_cur = 0;
  s->h_gid2slot = slot_of;
  bind_current(s);
  hipStream_t st = (hipStream_t)hip_stream;
  // stage the particles box by box, ids ascending inside a box: the order
  // the kernels expect before the first sort
  const int64_t n = q->n;
  std::vector<D4> hp((size_t)n), hv((size_t)n), hw((size_t)n);
  std::vector<uint8_t> ht((size_t)n);
  std::vector<int> hg((size_t)n), hrg((size_t)z.nr, 0), hsort((size_t)z.nr, 0);
  for (int64_t at = 0; at < n; ++at) {
    const int64_t k = z.order[(size_t)at];
    int64_t g = q->id[k];
    uint8_t t = q->type[k];
    bool rig = t == SDPDEM_RIGID;
    hp[(size_t)at] = D4{q->pos[3 * k], q->pos[3 * k + 1], q->pos[3 * k + 2],
                        rig ? q->radius[k] : 0.5 * params->dx};
    hv[(size_t)at] = D4{q->vel[3 * k], q->vel[3 * k + 1], q->vel[3 * k + 2],
                        rig ? q->mass[k] : params->mass_fluid};
    hw[(size_t)at] = D4{q->angvel[3 * k], q->angvel[3 * k + 1], q->angvel[3 * k + 2],
                        rig ? q->inertia[k] : params->inertia_fluid};
    ht[(size_t)at] = t;
    hg[(size_t)at] = (int)g;
    if (rig) {
      int sl = slot_of[(size_t)g];
      hrg[(size_t)sl] = (int)g;
      hsort[(size_t)sl] = (int)at;
    }
  }
  Dev& d = s->d;
  bool ok = true;
  ok &= hipMemcpyAsync(s->pos[0], hp.data(), sizeof(D4) * n, hipMemcpyHostToDevice, st) == hipSuccess;
  ok &= hipMemcpyAsync(s->vel[0], hv.data(), sizeof(D4) * n, hipMemcpyHostToDevice, st) == hipSuccess;
  ok &= hipMemcpyAsync(s->om[0], hw.data(), sizeof(D4) * n, hipMemcpyHostToDevice, st) == hipSuccess;
  ok &= hipMemcpyAsync(s->type[0], ht.data(), n, hipMemcpyHostToDevice, st) == hipSuccess;
  ok &= hipMemcpyAsync(s->gid[0], hg.data(), sizeof(int) * n, hipMemcpyHostToDevice, st) == hipSuccess;
  ok &= hipMemcpyAsync(d.gid2slot, slot_of.data(), sizeof(int) * n, hipMemcpyHostToDevice, st) == hipSuccess;
  ok &= hipMemcpyAsync(s->boxes, z.boxes.data(), sizeof(BoxD) * z.nbox, hipMemcpyHostToDevice, st) == hipSuccess;
  ok &= hipMemcpyAsync(const_cast<int2*>(d.blk), z.blk.data(), sizeof(int2) * z.blk.size(),
                       hipMemcpyHostToDevice, st) == hipSuccess;
  ok &= hipMemcpyAsync(const_cast<int2*>(d.ablk), z.ablk.data(), sizeof(int2) * z.ablk.size(),
                       hipMemcpyHostToDevice, st) == hipSuccess;
  {
    const int64_t step0 = params->itr_start;
    ok &= hipMemcpyAsync(d.dstep, &step0, sizeof(int64_t), hipMemcpyHostToDevice, st) == hipSuccess;
  }
  if (z.nr) {
    ok &= hipMemcpyAsync(d.rig_gid, hrg.data(), sizeof(int) * z.nr, hipMemcpyHostToDevice, st) == hipSuccess;
    ok &= hipMemcpyAsync(d.rig_sorted, hsort.data(), sizeof(int) * z.nr, hipMemcpyHostToDevice, st) == hipSuccess;
    ok &= hipMemcpyAsync(const_cast<int*>(d.rbox), z.rbox.data(), sizeof(int) * z.nr,
                         hipMemcpyHostToDevice, st) == hipSuccess;
  }
  // the staging copies read pageable host memory: finish them before the
  // host vectors go out of scope
  ok &= hipStreamSynchronize(st) == hipSuccess;
  launch_fill_i32(s->ct_cnt[0], 0, (size_t)z.nr, st);
  launch_fill_i32(s->ct_cnt[1], 0, (size_t)z.nr, st);
  launch_fill_i32(d.status, 0, 64, st);
  if (z.nr) launch_fill_i32(d.rxn_cnt, 0, (size_t)z.npad, st);
  launch_fill_i32(reinterpret_cast<int*>(d.fout), 0, 13 * (size_t)z.npad, st);
  launch_fill_i32(d.nbr_cnt, 0, (size_t)z.npad, st);
  launch_fill_i32(d.cstart, 0, (size_t)z.ncells_all + 1, st);
  // the binning counts into zeroed arrays; every scan leaves them zero again
  launch_fill_i32(d.count, 0, (size_t)z.ncells_all, st);
  if (z.nr) launch_fill_i32(d.rcount, 0, (size_t)z.rncells_all, st);
  launch_fill_f64(d.f_dg, 0.0, 3 * (size_t)z.nr, st);
  launch_fill_f64(d.f_pg, 0.0, 3 * (size_t)z.nr, st);
  launch_fill_f64(d.f_dem, 0.0, 3 * (size_t)z.nr, st);
  launch_fill_f64(d.f_lub, 0.0, 3 * (size_t)z.nr, st);
  launch_fill_f64(d.n_dem, 0.0, 3 * (size_t)z.nr, st);
  launch_fill_f64(d.eps, 0.0, (size_t)z.nr, st);
  launch_fill_f64(d.omega, 0.0, (size_t)z.nr, st);
  launch_fill_f64(d.wzx_r, 0.0, 2 * (size_t)z.nr, st);
  launch_fill_f64(d.st_inst, 0.0, (size_t)z.nbox, st);
  launch_fill_f64(d.st_sum, 0.0, (size_t)z.nbox, st);
  launch_fill_f64(d.rho, params->rho0, (size_t)z.npad, st);
  launch_fill_f64(d.p, 0.0, (size_t)z.npad, st);
  ok &= hipStreamSynchronize(st) == hipSuccess;
  ok &= hipGetLastError() == hipSuccess;
  if (!ok) {
    delete s;
    return SDPDEM_E_HIP;
  }
  if (z.nr && side_stream) make_side_stream(s);
  // candidate reuse reads one word per step: pinned, where the caller lets
  // the library allocate (the allocation-free variant copies to the stack)
  if (z.maxcand && side_stream) {
    if (hipHostMalloc((void**)&s->h_moved, 64, hipHostMallocDefault) != hipSuccess)
      s->h_moved = nullptr;
    if (hipEventCreateWithFlags(&s->ev_moved, hipEventDisableTiming) != hipSuccess)
      s->ev_moved = nullptr;
  }
  *out = s;
  return SDPDEM_OK;
}

// The allocation-free variant of sdpdem_create keeps its workspace in this
// file-scope device array.  In host code `scratch` names a host-side
// stand-in: its device address is taken with hipGetSymbolAddress once per
// device and only that address is handed to kernels and copies.
constexpr size_t kStaticBytes = SDPDEM_STATIC_WORKSPACE_BYTES;
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void* g_static_ptr[kMaxDevices] = {};

}  // namespace

__device__ __align__(256) unsigned char scratch[kStaticBytes];

namespace {

// device address of `scratch` on the current device (looked up on the first
// call per device)
int static_workspace(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return SDPDEM_E_HIP;
  std::lock_guard<std::mutex> lock(g_static_mu);
  if (!g_static_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
      return SDPDEM_E_HIP;
    g_static_ptr[dev] = ptr;
  }
  *out = g_static_ptr[dev];
  return SDPDEM_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI

extern "C" {

int sdpdem_field_comps(int field) {
  switch (field) {
    case SDPDEM_DENS:
    case SDPDEM_PRES:
    case SDPDEM_PRES_SMOOTH:
    case SDPDEM_EPS:
      return 1;
    default:
      return (field >= 0 && field < SDPDEM_NUM_FIELDS) ? 3 : 0;
  }
}

int sdpdem_workspace_bytes(const sdpdem_params* params, const sdpdem_particles* particles,
                           size_t* bytes) {
  if (!bytes || !params) return SDPDEM_E_INVALID_ARG;
  Sizes z;
  sdpdem_box b = box_from_params(params);
  if (!plan(params, &b, 1, particles, nullptr, z, nullptr)) return SDPDEM_E_INVALID_ARG;
  *bytes = layout(z, nullptr, nullptr);
  return SDPDEM_OK;
}

int sdpdem_create(const sdpdem_params* params, const sdpdem_particles* q, void* d_workspace,
                  size_t workspace_bytes, void* hip_stream, sdpdem_system** out) {
  if (!params) return SDPDEM_E_INVALID_ARG;
  sdpdem_box b = box_from_params(params);
  return create_impl(params, &b, 1, q, nullptr, d_workspace, workspace_bytes, hip_stream, out);
}

int sdpdem_create_static(const sdpdem_params* params, const sdpdem_particles* q,
                         void* hip_stream, sdpdem_system** out) {
  if (!params || !out) return SDPDEM_E_INVALID_ARG;
  *out = nullptr;
  size_t need = 0;
  const int rc = sdpdem_workspace_bytes(params, q, &need);
  if (rc != SDPDEM_OK) return rc;
  // the layout rounds the base up to 256 bytes; the array is 256-aligned
  if (need > kStaticBytes) return SDPDEM_E_WORKSPACE_TOO_SMALL;
  void* base = nullptr;
  const int rs = static_workspace(&base);
  if (rs != SDPDEM_OK) return rs;
  sdpdem_box b = box_from_params(params);
  // no second stream: creating one is a resource the caller did not ask for
  return create_impl(params, &b, 1, q, nullptr, base, kStaticBytes, hip_stream, out,
                     /*side_stream=*/false);
}

int sdpdem_batch_workspace_bytes(const sdpdem_params* params, const sdpdem_box* boxes,
                                 int32_t nbox, const sdpdem_particles* particles,
                                 const int32_t* box_of, size_t* bytes) {
  if (!bytes || !box_of) return SDPDEM_E_INVALID_ARG;
  Sizes z;
  if (!plan(params, boxes, nbox, particles, box_of, z, nullptr)) return SDPDEM_E_INVALID_ARG;
  *bytes = layout(z, nullptr, nullptr);
  return SDPDEM_OK;
}

int sdpdem_create_batch(const sdpdem_params* params, const sdpdem_box* boxes, int32_t nbox,
                        const sdpdem_particles* particles, const int32_t* box_of,
                        void* d_workspace, size_t workspace_bytes, void* hip_stream,
                        sdpdem_system** out) {
  if (!box_of) return SDPDEM_E_INVALID_ARG;
  return create_impl(params, boxes, nbox, particles, box_of, d_workspace, workspace_bytes,
                     hip_stream, out);
}

namespace {

// The moved flag of the drift just enqueued.  A one-thread kernel stores it
// into pinned host memory and the host polls the event behind that kernel,
// which wakes it within microseconds of the drift (a copy command takes
// tens of microseconds, and a blocking synchronisation sleeps for a good
// part of the next kernel's duration).  post_moved enqueues the store
// (false: no pinned word, or the event failed), wait_moved waits for it;
// both answer true (search) on any error.
bool post_moved(sdpdem_system* s, hipStream_t st) {
  if (!s->h_moved || !s->ev_moved) return false;
  *(volatile int*)s->h_moved = 1;
  launch_publish(s->d.moved, s->h_moved, st);  // a failed launch leaves 1: search
  return hipEventRecord(s->ev_moved, st) == hipSuccess;
}
bool wait_moved(sdpdem_system* s) {
  hipError_t e;
  while ((e = hipEventQuery(s->ev_moved)) == hipErrorNotReady) {
  }
  return e != hipSuccess || *(volatile int*)s->h_moved != 0;
}
// without a pinned word: a copy to the stack and a synchronisation
bool read_moved_sync(sdpdem_system* s, hipStream_t st) {
  int moved = 1;
  if (hipMemcpyAsync(&moved, s->d.moved, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return true;
  return moved != 0;
}

// One iteration of Algorithm 1 (enqueue only).
void step_body(sdpdem_system* s, hipStream_t st) {
  Dev& d = s->d;
  // Lees-Edwards offsets for positions at this step and after the drift;
  // the reaction's counts when the pass refills its slots
  const bool fill1 = needs_fill(s, !s->cache_valid);
  launch_pass_prep(d, s->boxes, 0, fill1, st);
  if (!s->cache_valid) run_build(s, st, 0);
  run_pass(s, 1, 0, true, fill1, st);
  // positions moved: sort, neighbours, density and smoothing at x(n+1);
  // they (and the coupling slots) stay valid for the first pass of the
  // next step
  const bool fill2 = needs_fill(s, true);
  launch_pass_prep(d, s->boxes, 1, fill2, st);
  // with candidate reuse, search again only if the drift took some particle
  // skin/2 from where the last search saw it.  The host reads the flag; the
  // candidate filter is enqueued before the answer arrives, so the device
  // does not wait for the host (a search overwrites everything the filter
  // wrote: lists, density, pressure and the filter's records).
  int lists = LISTS_SEARCH;
  if (d.reuse && s->cand_valid && !s->capturing) {
    const bool posted = post_moved(s, st);
    s->fork_marked = d.nr > 0 && s->side && hipEventRecord(s->ev_fork, st) == hipSuccess;
    {
      Prof pr(s, SDPDEM_K_NEIGHBORS_DENSITY, st);
      launch_filter_density(d, st);
    }
    if (!(posted ? wait_moved(s) : read_moved_sync(s, st))) lists = LISTS_FILTERED;
  }
  run_build(s, st, 1, lists, true);
  run_pass(s, 2, 1, true, fill2, st);
  if (s->stress) {
    launch_box_stress(d, 1, st);
    s->stress_samples += 1;
  }
  s->cache_valid = true;
  s->step += 1;
}

void drop_graph(sdpdem_system* s) {
  if (s->gexec) (void)hipGraphExecDestroy(s->gexec);
  s->gexec = nullptr;
}

// Capture graph_steps steps into one executable graph.  Every per-step
// value the kernels need (step number, Lees-Edwards offsets)
// lives in device memory, and the host-side buffer swaps repeat with
// period two, so an even number of captured steps replays correctly.
bool capture(sdpdem_system* s, hipStream_t st) {
  drop_graph(s);
  const int64_t step0 = s->step, samples0 = s->stress_samples;
  const int cur0 = s->cur, ct0 = s->ct_cur;
  const bool rxn0 = s->rxn_valid, cand0 = s->cand_valid, rec0 = s->rec_valid;
  const int64_t searches0 = s->searches;
  hipGraph_t g = nullptr;
  if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) return false;
  s->capturing = true;  // no host decisions inside a graph: every step searches
  for (int k = 0; k < s->graph_steps; ++k) step_body(s, st);
  s->capturing = false;
  const bool ok = hipStreamEndCapture(st, &g) == hipSuccess && g;
  // nothing ran yet: restore the host mirror of the device state
  s->step = step0;
  s->stress_samples = samples0;
  s->rxn_valid = rxn0;
  s->cand_valid = cand0;
  s->rec_valid = rec0;
  s->searches = searches0;
  if (s->cur != cur0 || s->ct_cur != ct0) {
    if (g) (void)hipGraphDestroy(g);
    return false;
  }
  if (!ok) return false;
  hipGraphExec_t ex = nullptr;
  const bool inst = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) == hipSuccess;
  (void)hipGraphDestroy(g);
  if (!inst) return false;
  s->gexec = ex;
  s->g_act = rigid_active(s);
  s->g_rxn = rxn0;
  s->g_rec = rec0;
  s->g_stress = s->stress;
  s->g_cur = s->cur;
  s->g_ct = s->ct_cur;
  return true;
}

}  // namespace

int sdpdem_step(sdpdem_system* s, int64_t nsteps, void* hip_stream) {
  if (!s || nsteps < 0) return SDPDEM_E_INVALID_ARG;
  hipStream_t st = (hipStream_t)hip_stream;
  int64_t left = nsteps;
  while (left > 0) {
    // re-read every round: a failed capture switches graphs off
    const int K = st ? s->graph_steps : 0;  // no capture on the null stream
    // replay whole graphs while nothing that shapes the launch sequence
    // changes inside them (first build done, no timing, rigid activation
    // not crossed)
    const bool act_now = rigid_active(s);
    const bool act_stable =
        s->d.nr == 0 || s->step >= s->P.itr_actv_rigid || s->step + K <= s->P.itr_actv_rigid;
    if (K > 0 && left >= K && s->cache_valid && s->prof_kernel == SDPDEM_K_NONE && act_stable) {
      // the graph bakes in the double buffers' roles (an odd number of
      // eager steps since the capture swaps them) and whether its first
      // pass refills the coupling slots: capture again when either differs
      if (!s->gexec || s->g_act != act_now || s->g_stress != s->stress || s->g_cur != s->cur ||
          s->g_ct != s->ct_cur || s->g_rxn != s->rxn_valid || s->g_rec != s->rec_valid) {
        if (!capture(s, st)) {
          s->graph_steps = 0;  // capture unavailable: stay eager
          continue;
        }
      }
      if (hipGraphLaunch(s->gexec, st) != hipSuccess) return SDPDEM_E_HIP;
      s->rxn_valid = act_now;  // the last pass built and (with the coupling) refilled
      s->cand_valid = false;  // every replayed step searched, without candidates
      s->rec_valid = act_now;  // and (with the coupling) filled by a search
      s->searches += K;
      s->step += K;
      s->graph_steps_run += K;
      if (s->stress) s->stress_samples += K;
      left -= K;
    } else {
      step_body(s, st);
      left -= 1;
    }
  }
  return sync_status(s, st);
}

int sdpdem_set_graph(sdpdem_system* s, int steps_per_graph) {
  if (!s || steps_per_graph < 0 || steps_per_graph % 2) return SDPDEM_E_INVALID_ARG;
  drop_graph(s);
  s->graph_steps = steps_per_graph;
  return SDPDEM_OK;
}

int sdpdem_compute_forces(sdpdem_system* s, void* hip_stream) {
  if (!s) return SDPDEM_E_INVALID_ARG;
  hipStream_t st = (hipStream_t)hip_stream;
  const bool fill = needs_fill(s, !s->cache_valid);
  launch_pass_prep(s->d, s->boxes, 0, fill, st);
  if (!s->cache_valid) {
    run_build(s, st, 0);
    s->cache_valid = true;
  }
  run_pass(s, 1, 0, false, fill, st);
  if (s->stress) launch_box_stress(s->d, 0, st);
  return sync_status(s, st);
}

int sdpdem_set_stress(sdpdem_system* s, int on, void* hip_stream) {
  if (!s) return SDPDEM_E_INVALID_ARG;
  hipStream_t st = (hipStream_t)hip_stream;
  s->stress = on != 0;
  s->d.stress = on ? 1 : 0;
  s->stress_samples = 0;
  launch_fill_f64(s->d.st_sum, 0.0, (size_t)s->d.nbox, st);
  launch_fill_f64(s->d.st_inst, 0.0, (size_t)s->d.nbox, st);
  if (s->d.nr) launch_fill_f64(s->d.wzx_r, 0.0, 2 * (size_t)s->d.nr, st);
  launch_fill_i32(reinterpret_cast<int*>(s->d.fout + 12 * (size_t)s->d.npad), 0,
                  (size_t)s->d.npad, st);
  if (hipStreamSynchronize(st) != hipSuccess) return SDPDEM_E_HIP;
  return hipGetLastError() == hipSuccess ? SDPDEM_OK : SDPDEM_E_HIP;
}

int sdpdem_box_stress(sdpdem_system* s, double* inst, double* sum, int64_t* nsamples,
                      void* hip_stream) {
  if (!s) return SDPDEM_E_INVALID_ARG;
  hipStream_t st = (hipStream_t)hip_stream;
  const size_t nb = (size_t)s->d.nbox;
  if (inst && hipMemcpyAsync(inst, s->d.st_inst, sizeof(double) * nb, hipMemcpyDeviceToHost,
                             st) != hipSuccess)
    return SDPDEM_E_HIP;
  if (sum && hipMemcpyAsync(sum, s->d.st_sum, sizeof(double) * nb, hipMemcpyDeviceToHost, st) !=
                 hipSuccess)
    return SDPDEM_E_HIP;
  if (hipStreamSynchronize(st) != hipSuccess) return SDPDEM_E_HIP;
  if (nsamples) *nsamples = s->stress_samples;
  return hipGetLastError() == hipSuccess ? SDPDEM_OK : SDPDEM_E_HIP;
}

int sdpdem_read_field(sdpdem_system* s, int field, void* dst, size_t bytes, int dst_is_device,
                      void* hip_stream) {
  if (!s || !dst) return SDPDEM_E_INVALID_ARG;
  int comps = sdpdem_field_comps(field);
  if (comps == 0) return SDPDEM_E_INVALID_ARG;
  size_t need = (size_t)s->d.n * comps * sizeof(double);
  if (bytes < need) return SDPDEM_E_INVALID_ARG;
  hipStream_t st = (hipStream_t)hip_stream;
  if (dst_is_device) {
    // the gather kernel writes the id-ordered rows straight into dst
    if ((uintptr_t)dst % alignof(double) != 0) return SDPDEM_E_INVALID_ARG;
    launch_read_field(s->d, field, rigid_active(s) ? 1 : 0, static_cast<double*>(dst), st);
    return hipGetLastError() == hipSuccess ? SDPDEM_OK : SDPDEM_E_HIP;
  }
  launch_read_field(s->d, field, rigid_active(s) ? 1 : 0, s->field_buf, st);
  if (hipMemcpyAsync(dst, s->field_buf, need, hipMemcpyDeviceToHost, st) != hipSuccess)
    return SDPDEM_E_HIP;
  if (hipStreamSynchronize(st) != hipSuccess) return SDPDEM_E_HIP;
  return hipGetLastError() == hipSuccess ? SDPDEM_OK : SDPDEM_E_HIP;
}

int sdpdem_read_neighbors(sdpdem_system* s, int64_t* row_ptr, int32_t* cols, int64_t cap,
                          int64_t* nnz, void* hip_stream) {
  if (!s || !row_ptr || !nnz) return SDPDEM_E_INVALID_ARG;
  hipStream_t st = (hipStream_t)hip_stream;
  const int n = s->d.n;
  const size_t np = (size_t)s->d.npad;
  std::vector<int> cnt((size_t)n), gid((size_t)n);
  if (hipMemcpyAsync(cnt.data(), s->d.nbr_cnt, sizeof(int) * n, hipMemcpyDeviceToHost, st) !=
          hipSuccess ||
      hipMemcpyAsync(gid.data(), s->d.gid, sizeof(int) * n, hipMemcpyDeviceToHost, st) !=
          hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return SDPDEM_E_HIP;
  std::vector<int64_t> rowlen((size_t)n + 1, 0);
  int kmax = 0;
  for (int i = 0; i < n; ++i) {
    rowlen[(size_t)gid[(size_t)i]] = cnt[(size_t)i];
    kmax = std::max(kmax, cnt[(size_t)i]);
  }
  row_ptr[0] = 0;
  for (int g = 0; g < n; ++g) row_ptr[g + 1] = row_ptr[g] + rowlen[(size_t)g];
  *nnz = row_ptr[n];
  if (!cols || *nnz == 0) return SDPDEM_OK;
  if (!s->cache_valid) return SDPDEM_E_INVALID_ARG;  // lists exist only after a build
  if (cap < *nnz) return SDPDEM_E_INVALID_ARG;
  // columns in chunks that fit the field buffer (3n doubles = 6n ints)
  int* dbuf = reinterpret_cast<int*>(s->field_buf);
  const int per = std::max(1, (int)std::min<size_t>(6, (6 * (size_t)n) / np));
  std::vector<int> hb(per * np);
  for (int k0 = 0; k0 < kmax; k0 += per) {
    int kn = std::min(per, kmax - k0);
    launch_nbr_cols(s->d, k0, kn, dbuf, st);
    if (hipMemcpyAsync(hb.data(), dbuf, sizeof(int) * kn * np, hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return SDPDEM_E_HIP;
    for (int i = 0; i < n; ++i) {
      int g = gid[(size_t)i];
      for (int k = 0; k < kn; ++k) {
        int v = hb[(size_t)k * np + i];
        if (v >= 0) cols[row_ptr[g] + k0 + k] = v;
      }
    }
  }
  for (int g = 0; g < n; ++g) std::sort(cols + row_ptr[g], cols + row_ptr[g + 1]);
  return SDPDEM_OK;
}

int sdpdem_read_contacts(sdpdem_system* s, int32_t* pairs, double* delta_t, int64_t cap,
                         int64_t* n_contacts, void* hip_stream) {
  if (!s || !n_contacts) return SDPDEM_E_INVALID_ARG;
  hipStream_t st = (hipStream_t)hip_stream;
  const int nr = s->d.nr, mc = s->d.maxc;
  std::vector<int> cnt((size_t)nr), part((size_t)nr * mc), rg((size_t)nr);
  std::vector<double> dt((size_t)nr * mc * 3);
  if (nr) {
    if (hipMemcpyAsync(cnt.data(), s->d.ct_cnt, sizeof(int) * nr, hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipMemcpyAsync(part.data(), s->d.ct_partner, sizeof(int) * nr * mc, hipMemcpyDeviceToHost,
                       st) != hipSuccess ||
        hipMemcpyAsync(dt.data(), s->d.ct_dt, sizeof(double) * nr * mc * 3, hipMemcpyDeviceToHost,
                       st) != hipSuccess ||
        hipMemcpyAsync(rg.data(), s->d.rig_gid, sizeof(int) * nr, hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return SDPDEM_E_HIP;
  }
  struct Row {
    int i, j;
    double d[3];
  };
  std::vector<Row> rows;
  for (int sl = 0; sl < nr; ++sl) {
    int gi = rg[(size_t)sl];
    for (int c = 0; c < cnt[(size_t)sl] && c < mc; ++c) {
      int gj = part[(size_t)sl * mc + c];
      if (gj <= gi) continue;
      Row r{gi, gj, {dt[((size_t)sl * mc + c) * 3], dt[((size_t)sl * mc + c) * 3 + 1],
                     dt[((size_t)sl * mc + c) * 3 + 2]}};
      rows.push_back(r);
    }
  }
  std::sort(rows.begin(), rows.end(),
            [](const Row& a, const Row& b) { return a.i != b.i ? a.i < b.i : a.j < b.j; });
  *n_contacts = (int64_t)rows.size();
  if (!pairs || !delta_t) return SDPDEM_OK;
  if (cap < (int64_t)rows.size()) return SDPDEM_E_INVALID_ARG;
  for (size_t m = 0; m < rows.size(); ++m) {
    pairs[2 * m] = rows[m].i;
    pairs[2 * m + 1] = rows[m].j;
    for (int a = 0; a < 3; ++a) delta_t[3 * m + a] = rows[m].d[a];
  }
  return SDPDEM_OK;
}

int sdpdem_load_contacts(sdpdem_system* s, const int32_t* pairs, const double* delta_t,
                         int64_t n_contacts, void* hip_stream) {
  if (!s || n_contacts < 0 || (n_contacts > 0 && (!pairs || !delta_t)))
    return SDPDEM_E_INVALID_ARG;
  hipStream_t st = (hipStream_t)hip_stream;
  const int nr = s->d.nr, mc = s->d.maxc, n = s->d.n;
  std::vector<std::vector<std::pair<int, std::array<double, 3>>>> rows((size_t)nr);
  for (int64_t m = 0; m < n_contacts; ++m) {
    int i = pairs[2 * m], j = pairs[2 * m + 1];
    if (i < 0 || j < 0 || i >= n || j >= n || i == j) return SDPDEM_E_INVALID_ARG;
    int si = s->h_gid2slot[(size_t)i], sj = s->h_gid2slot[(size_t)j];
    if (si < 0 || sj < 0) return SDPDEM_E_INVALID_ARG;
    std::array<double, 3> a{delta_t[3 * m], delta_t[3 * m + 1], delta_t[3 * m + 2]};
    std::array<double, 3> b{-a[0], -a[1], -a[2]};
    rows[(size_t)si].push_back({j, a});
    rows[(size_t)sj].push_back({i, b});
  }
  std::vector<int> cnt((size_t)nr, 0), part((size_t)nr * mc, 0);
  std::vector<double> dt((size_t)nr * mc * 3, 0.0);
  for (int sl = 0; sl < nr; ++sl) {
    auto& r = rows[(size_t)sl];
    if ((int)r.size() > mc) return SDPDEM_E_CONTACT_OVERFLOW;
    std::sort(r.begin(), r.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
    cnt[(size_t)sl] = (int)r.size();
    for (size_t c = 0; c < r.size(); ++c) {
      part[(size_t)sl * mc + c] = r[c].first;
      for (int a = 0; a < 3; ++a) dt[((size_t)sl * mc + c) * 3 + a] = r[c].second[a];
    }
  }
  if (nr) {
    if (hipMemcpyAsync(s->d.ct_cnt, cnt.data(), sizeof(int) * nr, hipMemcpyHostToDevice, st) !=
            hipSuccess ||
        hipMemcpyAsync(s->d.ct_partner, part.data(), sizeof(int) * nr * mc, hipMemcpyHostToDevice,
                       st) != hipSuccess ||
        hipMemcpyAsync(s->d.ct_dt, dt.data(), sizeof(double) * nr * mc * 3, hipMemcpyHostToDevice,
                       st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return SDPDEM_E_HIP;
  }
  return SDPDEM_OK;
}

int sdpdem_totals(sdpdem_system* s, double out[16], void* hip_stream) {
  if (!s || !out) return SDPDEM_E_INVALID_ARG;
  hipStream_t st = (hipStream_t)hip_stream;
  launch_totals(s->d, s->tot_part, s->tot_out, st);
  double t[16] = {0};
  if (hipMemcpyAsync(t, s->tot_out, sizeof(double) * 13, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return SDPDEM_E_HIP;
  for (int k = 0; k < 12; ++k) out[k] = t[k];
  out[12] = (double)s->step;
  out[13] = out[14] = out[15] = 0.0;
  return SDPDEM_OK;
}

int64_t sdpdem_get_step(const sdpdem_system* s) { return s ? s->step : -1; }

int sdpdem_info(sdpdem_system* s, int64_t out[16], void* hip_stream) {
  if (!s || !out) return SDPDEM_E_INVALID_ARG;
  for (int k = 0; k < 16; ++k) out[k] = 0;
  out[0] = s->d.n;
  out[1] = s->d.nr;
  for (int a = 0; a < 3; ++a) {
    out[2 + a] = s->h_boxes[0].g.nc[a];
    out[5 + a] = s->h_boxes[0].rg.nc[a];
  }
  out[10] = s->d.nbox;
  out[11] = s->graph_steps_run;
  out[12] = s->side ? 1 : 0;
  out[13] = s->searches;
  out[14] = s->reuses;
  std::vector<int> cnt((size_t)s->d.n);
  hipStream_t st = (hipStream_t)hip_stream;
  if (hipMemcpyAsync(cnt.data(), s->d.nbr_cnt, sizeof(int) * s->d.n, hipMemcpyDeviceToHost, st) !=
          hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return SDPDEM_E_HIP;
  int64_t mx = 0, tot = 0;
  for (int v : cnt) {
    mx = std::max<int64_t>(mx, v);
    tot += v;
  }
  out[8] = mx;
  out[9] = tot;
  return SDPDEM_OK;
}

int sdpdem_set_profiling(sdpdem_system* s, int kernel) {
  if (!s || kernel < 0 || kernel >= SDPDEM_NUM_KERNELS) return SDPDEM_E_INVALID_ARG;
  drop_graph(s);
  prof_flush(s);
  s->prof_kernel = kernel;
  s->prof_ms = 0.0;
  s->prof_n = 0;
  s->prof_seen = 0;
  // create the timing events now, not while the timed launches are being
  // enqueued (creating them there costs host time per launch)
  if (kernel != SDPDEM_K_NONE)
    while (s->ev.size() < 1024) {
      hipEvent_t a, b;
      if (hipEventCreate(&a) != hipSuccess) break;
      if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        break;
      }
      s->ev.emplace_back(a, b);
    }
  return SDPDEM_OK;
}

int sdpdem_set_profiling_every(sdpdem_system* s, int every) {
  if (!s || every < 1) return SDPDEM_E_INVALID_ARG;
  prof_flush(s);
  s->prof_every = every;
  s->prof_seen = 0;
  return SDPDEM_OK;
}

int sdpdem_kernel_time(sdpdem_system* s, double* total_ms, int64_t* launches) {
  if (!s || !total_ms || !launches) return SDPDEM_E_INVALID_ARG;
  prof_flush(s);
  *total_ms = s->prof_ms;
  *launches = s->prof_n;
  s->prof_ms = 0.0;
  s->prof_n = 0;
  return SDPDEM_OK;
}

void sdpdem_destroy(sdpdem_system* s) {
  if (!s) return;
  drop_graph(s);
  prof_flush(s);
  free_side_stream(s);
  if (s->h_moved) (void)hipHostFree(s->h_moved);
  if (s->ev_moved) (void)hipEventDestroy(s->ev_moved);
  for (auto& e : s->ev) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  delete s;
}

const char* sdpdem_status_string(int status) {
  switch (status) {
    case SDPDEM_OK:
      return "ok";
    case SDPDEM_E_INVALID_ARG:
      return "invalid argument";
    case SDPDEM_E_WORKSPACE_TOO_SMALL:
      return "workspace too small";
    case SDPDEM_E_NBR_OVERFLOW:
      return "a neighbour row exceeded max_neighbors";
    case SDPDEM_E_CONTACT_OVERFLOW:
      return "a rigid contact row exceeded max_contacts";
    case SDPDEM_E_NONFINITE:
      return "non-finite position, velocity or spin";
    case SDPDEM_E_OUT_OF_DOMAIN:
      return "a particle left the domain";
    case SDPDEM_E_HIP:
      return "HIP runtime error";
    default:
      return "unknown status";
  }
}

}  // extern "C"
