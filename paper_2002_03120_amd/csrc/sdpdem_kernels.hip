// sdpdem_kernels.hip -- gfx950 kernels of the SDPD-DEM per-step path.
//
// Layout: particles live in cell-sorted order (counting sort of linear cell
// keys, ties broken by id), so every neighbour gather touches a compact
// region that the XCD's L2 holds.  Per-particle kernels map blocks to XCDs
// in contiguous chunks (a dispatch sends block b to XCD b % 8).  Sums are
// gathers, never atomics on floating point, so every run is bit-for-bit
// repeatable.
//
// Precision: positions, velocities, spins, density, pressure, the
// fluid-particle coupling, DEM and the integrator in FP64; the SDPD pair
// forces (Sec. 2.1) in FP32 with FP32 per-particle accumulation, their
// separation vectors taken as FP64 differences rounded once.
#include <cmath>

#include <climits>

#include "sdpdem_device.h"

namespace sdpdem {

// ---------------------------------------------------------------------------
// generic helpers

__global__ void k_fill_i32(int* a, int v, size_t count) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) a[i] = v;
}
// the same for a 16-byte aligned array: four ints per thread
__global__ void k_fill_i32x4(int* a, int v, size_t count) {
  size_t i = 4 * ((size_t)blockIdx.x * blockDim.x + threadIdx.x);
  if (i + 4 <= count) {
    *reinterpret_cast<int4*>(a + i) = make_int4(v, v, v, v);
  } else {
    for (; i < count; ++i) a[i] = v;
  }
}
__global__ void k_fill_f64(double* a, double v, size_t count) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) a[i] = v;
}

void launch_fill_i32(int* a, int v, size_t count, hipStream_t st) {
  if (!count) return;
  if (((uintptr_t)a & 15) == 0) {
    const size_t threads = (count + 3) / 4;
    k_fill_i32x4<<<(unsigned)((threads + BS - 1) / BS), BS, 0, st>>>(a, v, count);
  } else {
    k_fill_i32<<<(unsigned)((count + BS - 1) / BS), BS, 0, st>>>(a, v, count);
  }
}
// one word of device memory into host-visible memory (a pinned host word):
// cheaper than a copy command for the one flag the host waits on
__global__ void k_publish(const int* src, int* dst) {
  if (threadIdx.x == 0) __hip_atomic_store(dst, *src, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
void launch_publish(const int* src, int* dst, hipStream_t st) {
  k_publish<<<1, 64, 0, st>>>(src, dst);
}

void launch_fill_f64(double* a, double v, size_t count, hipStream_t st) {
  if (!count) return;
  k_fill_f64<<<(unsigned)((count + BS - 1) / BS), BS, 0, st>>>(a, v, count);
}

// ---------------------------------------------------------------------------
// (a1) binning and counting sort

__global__ __launch_bounds__(BS) void k_bin(Dev d) {
  int i;
  const int b = blk_box(d, i);
  if (b < 0) return;
  const BoxD& B = d.boxes[b];
  if (i >= B.first + B.count) return;
  D4 p = d.pos[i];
  int oob = 0;
  int cx = cell_coord(p.x, B.g, 0, &oob);
  int cy = cell_coord(p.y, B.g, 1, &oob);
  int cz = cell_coord(p.z, B.g, 2, &oob);
  if (oob) atomicOr(d.status, ST_OUT_OF_DOMAIN);
  // outer walls take the box's second range of cells: the sort then keeps
  // them after the box's active particles, in a fixed order
  const int c = B.cell_off + (d.type[i] == T_OUTER ? B.wall_off : 0) + cell_index(B.g, cx, cy, cz);
  d.key[i] = (uint32_t)c;
  // the arrival order in the cell places the particle in the scatter (the
  // cell sort then fixes the order inside the cell)
  d.rank[i] = atomicAdd(&d.count[c], 1);
}

void launch_bin(const Dev& d, hipStream_t st) {
  k_bin<<<d.nblk, BS, 0, st>>>(d);
}

__global__ __launch_bounds__(BS) void k_bin_rigid(Dev d) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= d.nr) return;
  const BoxD& B = d.boxes[d.rbox[s]];
  D4 p = d.pos[d.rig_sorted[s]];
  int oob = 0;
  int cx = cell_coord(p.x, B.rg, 0, &oob);
  int cy = cell_coord(p.y, B.rg, 1, &oob);
  int cz = cell_coord(p.z, B.rg, 2, &oob);
  if (oob) atomicOr(d.status, ST_OUT_OF_DOMAIN);
  int c = B.rcell_off + cell_index(B.rg, cx, cy, cz);
  d.rkey[s] = (uint32_t)c;
  atomicAdd(&d.rcount[c], 1);
}

void launch_bin_rigid(const Dev& d, hipStream_t st) {
  if (d.nr == 0) return;
  k_bin_rigid<<<(d.nr + 63) / 64, 64, 0, st>>>(d);  // one wave per block: more CUs
}

// The start of a pass, one launch: the Lees-Edwards offsets
// delta(t) = fmod(shear L_z t, L_x) of every box for positions at step
// *dstep + add and at the step after and (when the pass refills the
// coupling slots) the reaction's slot counts cleared.
__global__ void k_pass_prep(BoxD* boxes, int nbox, const int64_t* dstep, int add, double dt,
                            int* rxn_cnt, int nfill) {
#pragma clang fp contract(off)
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t step = dstep[0];
  if (rxn_cnt && 4 * tid < nfill) {
    if (4 * tid + 4 <= nfill)
      *reinterpret_cast<int4*>(rxn_cnt + 4 * tid) = make_int4(0, 0, 0, 0);
    else
      for (int k = 4 * tid; k < nfill; ++k) rxn_cnt[k] = 0;
  }
  if (tid >= nbox) return;
  BoxD& B = boxes[tid];
  if (!B.le) {
    B.le_shift = 0.0;
    B.le_next = 0.0;
    return;
  }
  for (int k = 0; k < 2; ++k) {
    double t = (double)(step + add + k) * dt;
    double v = (B.shear * B.L[2]) * t;
    double sft = fmod(v, B.L[0]);
    if (sft < 0.0) sft += B.L[0];
    if (k == 0)
      B.le_shift = sft;
    else
      B.le_next = sft;
  }
}

void launch_pass_prep(const Dev& d, BoxD* boxes, int add, bool clear_rxn, hipStream_t st) {
  const int nfill = clear_rxn ? d.npad : 0;  // rxn_cnt is 256-byte aligned
  const int threads = max(d.nbox, (nfill + 3) / 4);
  k_pass_prep<<<(unsigned)max(1, (threads + BS - 1) / BS), BS, 0, st>>>(
      boxes, d.nbox, d.dstep, add, d.dt, clear_rxn ? d.rxn_cnt : nullptr, nfill);
}



static constexpr int SCAN_ITEMS = 8;
static constexpr int SCAN_TILE = BS * SCAN_ITEMS;

// the SCAN_ITEMS consecutive counts of one thread: two 16-byte loads when
// all are in range (the arrays are 256-byte aligned), else one by one
static_assert(SCAN_ITEMS == 8, "two 16-byte loads and stores per thread");
__device__ __forceinline__ void load_items(const int* in, int m, int base, int v[SCAN_ITEMS]) {
  if (base + SCAN_ITEMS <= m) {
    const int4 a = *reinterpret_cast<const int4*>(in + base);
    const int4 b = *reinterpret_cast<const int4*>(in + base + 4);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
  } else {
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) v[k] = base + k < m ? in[base + k] : 0;
  }
}

__global__ __launch_bounds__(BS) void k_scan_reduce(const int* in, int m, int* block_sums) {
  __shared__ int lds[BS / 64 + 1];
  int base = blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
  int v[SCAN_ITEMS];
  load_items(in, m, base, v);
  int s = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) s += v[k];
  int tot;
  block_exclusive_scan(s, lds, &tot);
  if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
}

// exclusive scan of the block sums in one block, chunks of 16 sums per
// thread (one chunk covers 4096 sums, a grid of 8.4 M cells)
__global__ __launch_bounds__(BS) void k_scan_blocksums(int* block_sums, int nb) {
  __shared__ int lds[BS / 64 + 1];
  constexpr int PER = 16;
  int carry = 0;
  for (int base = 0; base < nb; base += BS * PER) {
    const int first = base + (int)threadIdx.x * PER;
    int v[PER];
    int s = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      v[k] = first + k < nb ? block_sums[first + k] : 0;
      s += v[k];
    }
    int tot;
    int ex = block_exclusive_scan(s, lds, &tot) + carry;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      if (first + k < nb) block_sums[first + k] = ex;
      ex += v[k];
    }
    carry += tot;
  }
  if (threadIdx.x == 0) block_sums[nb] = carry;
}

// also leaves the counts at zero for the next binning (the count array is
// read by nothing after the scan), so no fill precedes the binning
__global__ __launch_bounds__(BS) void k_scan_apply(int* in, int m, const int* block_sums,
                                                  int nb, int* start, int* cursor) {
  __shared__ int lds[BS / 64 + 1];
  int base = blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
  int v[SCAN_ITEMS];
  load_items(in, m, base, v);
  if (base + SCAN_ITEMS <= m) {
    *reinterpret_cast<int4*>(in + base) = make_int4(0, 0, 0, 0);
    *reinterpret_cast<int4*>(in + base + 4) = make_int4(0, 0, 0, 0);
  } else {
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k)
      if (base + k < m) in[base + k] = 0;
  }
  int s = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) s += v[k];
  int tot;
  int ex = block_exclusive_scan(s, lds, &tot) + block_sums[blockIdx.x];
  int e[SCAN_ITEMS];
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    e[k] = ex;
    ex += v[k];
  }
  if (base + SCAN_ITEMS <= m) {
    const int4 a = make_int4(e[0], e[1], e[2], e[3]), b = make_int4(e[4], e[5], e[6], e[7]);
    *reinterpret_cast<int4*>(start + base) = a;
    *reinterpret_cast<int4*>(start + base + 4) = b;
    if (cursor) {
      *reinterpret_cast<int4*>(cursor + base) = a;
      *reinterpret_cast<int4*>(cursor + base + 4) = b;
    }
  } else {
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k)
      if (base + k < m) {
        start[base + k] = e[k];
        if (cursor) cursor[base + k] = e[k];
      }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) start[m] = block_sums[nb];
}

int scan_block_sums_size(int m) { return (m + SCAN_TILE - 1) / SCAN_TILE + 1; }

void launch_scan(int* count, int m, int* start, int* cursor, int* block_sums,
                 hipStream_t st) {
  int nb = (m + SCAN_TILE - 1) / SCAN_TILE;
  if (nb < 1) nb = 1;
  k_scan_reduce<<<nb, BS, 0, st>>>(count, m, block_sums);
  k_scan_blocksums<<<1, BS, 0, st>>>(block_sums, nb);
  k_scan_apply<<<nb, BS, 0, st>>>(count, m, block_sums, nb, start, cursor);
}

__global__ __launch_bounds__(BS) void k_scatter(const uint32_t* key, int n, int* cursor,
                                               int* perm) {
  int i = xcd_tid();
  if (i >= n) return;
  int slot = atomicAdd(&cursor[key[i]], 1);
  perm[slot] = i;
}

void launch_scatter(const uint32_t* key, int n, int* cursor, int* perm, hipStream_t st) {
  if (n == 0) return;
  k_scatter<<<nblocks(n), BS, 0, st>>>(key, n, cursor, perm);
}

__global__ __launch_bounds__(BS) void k_scatter_ranked(const uint32_t* key, const int* rank,
                                                      int n, const int* start, int* perm) {
  int i = xcd_tid();
  if (i >= n) return;
  perm[start[key[i]] + rank[i]] = i;
}

void launch_scatter_ranked(const uint32_t* key, const int* rank, int n, const int* start,
                           int* perm, hipStream_t st) {
  if (n == 0) return;
  k_scatter_ranked<<<nblocks(n), BS, 0, st>>>(key, rank, n, start, perm);
}

// Insertion sort of each cell's slice: ties of the counting sort are
// broken by a fixed key (the particle id), making the order deterministic.
__global__ __launch_bounds__(BS) void k_cell_sort(const int* start, int ncells, int* perm,
                                                 const int* sortkey) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncells) return;
  int lo = start[c], hi = start[c + 1];
  for (int a = lo + 1; a < hi; ++a) {
    int v = perm[a];
    int kv = sortkey ? sortkey[v] : v;
    int b = a - 1;
    while (b >= lo) {
      int w = perm[b];
      int kw = sortkey ? sortkey[w] : w;
      if (kw <= kv) break;
      perm[b + 1] = w;
      --b;
    }
    perm[b + 1] = v;
  }
}

void launch_cell_sort(const int* start, int ncells, int* perm, const int* sortkey,
                      hipStream_t st) {
  if (ncells == 0) return;
  k_cell_sort<<<(ncells + BS - 1) / BS, BS, 0, st>>>(start, ncells, perm, sortkey);
}

__global__ __launch_bounds__(BS) void k_permute(Dev d, const D4* spos, const D4* svel,
                                               const D4* som, const uint8_t* stype,
                                               const int* sgid) {
  int i = xcd_tid();
  if (i >= d.n) return;
  int o = d.perm[i];
  d.pos[i] = spos[o];
  d.vel[i] = svel[o];
  d.om[i] = som[o];
  uint8_t t = stype[o];
  int g = sgid[o];
  d.type[i] = t;
  d.gid[i] = g;
  if (t == T_RIGID) d.rig_sorted[d.gid2slot[g]] = i;
}

void launch_permute(const Dev& d, const D4* spos, const D4* svel, const D4* som,
                    const uint8_t* stype, const int* sgid, hipStream_t st) {
  k_permute<<<nblocks(d.n), BS, 0, st>>>(d, spos, svel, som, stype, sgid);
}


// ---------------------------------------------------------------------------
// Rigid particles in rigid-grid cell order: after the rigid counting sort,
// copy position (+radius), velocity (+mass) and spin (+inertia) of every
// rigid particle next to its cell neighbours, so the DEM and reaction
// gathers read contiguous records.  Run at the start of every pass (the
// velocities change between passes).

__global__ __launch_bounds__(BS) void k_rigid_gather(Dev d) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= d.nr) return;
  int s = d.ritems[t];
  int i = d.rig_sorted[s];
  d.rpos_c[t] = d.pos[i];
  d.rvel_c[t] = d.vel[i];
  d.rom_c[t] = d.om[i];
}

void launch_rigid_gather(const Dev& d, hipStream_t st) {
  if (d.nr == 0) return;
  k_rigid_gather<<<(d.nr + 63) / 64, 64, 0, st>>>(d);  // one wave per block: more CUs
}

// ---------------------------------------------------------------------------
// (a6) fluid-particle action: one wavefront per rigid particle gathers the
// fluid inside H_s = R_s + h (Sec. 2.4): Omega_s, the W-weighted fluid
// velocity, the W-weighted F^C + F^D of the neighbours and the number of
// other rigid centres inside H_s (k_fpi_finish then forms eps, F^DG and
// F^PG from them).  The cell rows of the search box are contiguous slices
// of the sorted arrays; the wave walks their concatenation with one
// candidate per lane.  With FILL it also hands every coupled fluid particle
// a slot (sphere record, kernel weight) for the reaction and records,
// round by round and lane by lane, which fluid particle each lane coupled
// to.  Both depend only on the positions and the sorted order, so the pass
// after a neighbour build fills them and the next pass (same positions,
// same order) reuses them: the slot counter's atomics miss the L2 and
// travel to memory, and the recorded rounds replace the cell search, with
// every lane summing the same terms in the same order (a sphere whose
// search needed more rounds than the record holds searches again).

__device__ double drag_b(double eps, double dv, double dd, double rho, double mu) {
  // beta / (1 - eps) of the Ergun (eps <= 0.8) and Wen-Yu branches
  if (eps <= 0.8) return 150.0 * mu * (1.0 - eps) / (eps * dd * dd) + 1.75 * rho * dv / dd;
  double re = rho * dd * eps * dv / mu;
  double cd_dv = re <= 1000.0 ? 24.0 * mu * (1.0 + 0.15 * pow(re, 0.687)) / (rho * dd * eps)
                              : 0.44 * dv;
  return 0.75 * cd_dv * eps * rho * pow(eps, -2.65) / dd;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ int wave_sum_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// The record of a sphere (keyed by its rigid slot, so that it survives the
// rigid grid's re-sort every step): per round and lane the partner a
// search visited within H_s + skin, fluid j as j, rigid k as -2 - k, none as
// -1.  Passes at the same sorted order read it instead of searching: the
// same partners in the same lanes and rounds, each tested against H_s
// again, so a pass at the search's positions gives the search's bits and a
// pass after a drift of less than skin/2 finds every partner within H_s.
// With use_rec a filling pass also reads it (the candidates of a build
// that kept the sorted order).
template <bool STRESS, bool FILL>
__global__ __launch_bounds__(BS) void k_fpi_action(Dev d, int use_rec) {
  const int wave = xcd_wave();
  const int lane = threadIdx.x & 63;
  if (wave >= d.nr) return;
  // spheres in rigid-grid cell order: neighbouring waves share cache lines
  const int s = __builtin_amdgcn_readfirstlane(d.ritems[wave]);
  const int si = d.rig_sorted[s];
  const BoxD& B = d.boxes[__builtin_amdgcn_readfirstlane(d.rbox[s])];
  const Geo G = geo_of(B);
  const D4 ps = d.pos[si];
  const double R = ps.w, H = R + d.h, H2 = H * H;
  const double invH = 1.0 / H, wnorm = 105.0 / (16.0 * PI * H * H * H);  // Eq. kernel
  const size_t np = (size_t)d.npad;
  int* const list = d.act_list + (size_t)s * (ACT_ROUNDS * 64);
  double om = 0, v0 = 0, v1 = 0, v2 = 0, f0 = 0, f1 = 0, f2 = 0, l2 = 0;
  int nrig = 0;
  // the pair geometry of fluid candidate j: image separation, its z image
  // and r^2 (the same operations on both paths, so the sums agree bit for bit)
  auto geom = [&](int j, double& ez, int& kz) {
    const D4 pj = d.pos[j];
    double ex = ps.x - pj.x, ey = ps.y - pj.y;
    ez = ps.z - pj.z;
    kz = min_img_box(G, ex, ey, ez);
    return r2_exact(ex, ey, ez);
  };
  // one coupled fluid particle
  auto couple = [&](int j, double r2, double ez, int kz) {
    const double qh = sqrt(r2) * invH, omq = 1.0 - qh;
    const double pw = (1.0 + 3.0 * qh) * omq * omq * omq;
    const double w = wnorm * pw;
    if (FILL) {
      // hand the pair to the reaction: one slot of j (the arrival order
      // does not matter, the reaction sums its slots by sphere record)
      const int slot = atomicAdd(&d.rxn_cnt[j], 1);
      if (slot < RXN_CAP)
        d.rxn_slot[(size_t)slot * np + j] = make_int2(wave, __float_as_int((float)pw));
    }
    const D4 vj = d.vel[j];
    om += w;
    v0 += w * (vj.x + (double)kz * G.le_jump);  // image velocity (Lees-Edwards)
    v1 += w * vj.y;
    v2 += w * vj.z;
    f0 += w * (double)d.fout[6 * np + j];
    f1 += w * (double)d.fout[7 * np + j];
    f2 += w * (double)d.fout[8 * np + j];
    if (STRESS) l2 += w * ez;  // the coupling's lever (z part)
  };
  const int2 meta = FILL && !use_rec ? make_int2(-1, 0) : d.act_meta[s];
  const int stored = __builtin_amdgcn_readfirstlane(meta.x);
  int rounds = 0;  // candidate rounds of the cell search
  if (stored >= 0) {
    rounds = stored;
    for (int r = 0; r < stored; ++r) {
      const int e = list[r * 64 + lane];
      if (e == -1) continue;
      const int j = e >= 0 ? e : -2 - e;
      double ez;
      int kz;
      const double r2 = geom(j, ez, kz);
      if (r2 < H2) {
        if (e >= 0)
          couple(j, r2, ez, kz);
        else
          ++nrig;
      }
    }
  } else {
    const Grid gr = B.g;
    const int coff = B.cell_off;
    int oob = 0;
    const int cc[3] = {cell_coord(ps.x, gr, 0, &oob), cell_coord(ps.y, gr, 1, &oob),
                       cell_coord(ps.z, gr, 2, &oob)};
    // the record keeps the partners within H_s + skin; with candidate
    // reuse the grid holds the particles where the last search saw them, up
    // to pad from where they are: search that much wider
    const double Hr = H + 2.0 * d.pad, Hr2 = Hr * Hr;
    // (and, in a sheared box, as far again as the flow can carry them)
    const double Hs = Hr + d.pad + B.act_margin;
    const int kr = reach_cells(gr, Hs);
    // the search box row by row: lane r takes row r of each batch of 64 rows
    // (at most two runs of consecutive cells per row)
    const StencilShape sh = stencil_shape(gr, cc, kr);
    const int nrows = sh.zn * sh.yn;
    for (int rb = 0; rb < nrows; rb += 64) {
      int sa = 0, la = 0, sb = 0, lb = 0;
      if (rb + lane < nrows) {
        int a0, a1, b0, b1;
        stencil_row<true>(G, gr, coff, ps.x, ps.y, ps.z, Hs, cc, kr, sh, rb + lane, a0, a1, b0,
                          b1);
        if (a1 > a0) {
          sa = d.cstart[a0];
          la = d.cstart[a1] - sa;
        }
        if (b1 > b0) {
          sb = d.cstart[b0];
          lb = d.cstart[b1] - sb;
        }
      }
      const int len = la + lb;
      int inc = len;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        int t = __shfl_up(inc, o, 64);
        if (lane >= o) inc += t;
      }
      const int total = __shfl(inc, 63, 64);
      const int off = inc - len;
      // every lane takes one candidate of the concatenated runs per round;
      // all lanes stay active through the shuffles
      for (int base = 0; base < total; base += 64, ++rounds) {
        const int t = base + lane;
        int r = 0;  // last run whose offset is <= t
#pragma unroll
        for (int stp = 32; stp > 0; stp >>= 1) {
          int cand = r + stp;
          int v = __shfl(off, cand & 63, 64);
          if (cand < 64 && v <= t) r = cand;
        }
        const int offr = __shfl(off, r, 64);
        const int sar = __shfl(sa, r, 64);
        const int lar = __shfl(la, r, 64);
        const int sbr = __shfl(sb, r, 64);
        int rec = -1;  // this lane's partner of this round within H_s + skin
        if (t < total) {
          const int q = t - offr;
          const int j = q < lar ? sar + q : sbr + (q - lar);
          // (the sphere itself is neither partner nor fluid)
          const uint8_t tj = j != si ? d.type[j] : (uint8_t)T_INNER;
          if (tj == T_FLUID || tj == T_RIGID) {
            double ez;
            int kz;
            const double r2 = geom(j, ez, kz);
            if (r2 < Hr2) rec = tj == T_RIGID ? -2 - j : j;
            if (r2 < H2) {
              if (tj == T_RIGID)
                ++nrig;
              else
                couple(j, r2, ez, kz);
            }
          }
        }
        if (FILL && rounds < ACT_ROUNDS) list[rounds * 64 + lane] = rec;
      }
    }
  }
  om = wave_sum(om);
  v0 = wave_sum(v0);
  v1 = wave_sum(v1);
  v2 = wave_sum(v2);
  f0 = wave_sum(f0);
  f1 = wave_sum(f1);
  f2 = wave_sum(f2);
  if (STRESS) l2 = wave_sum(l2);
  nrig = wave_sum_i(nrig);
  if (lane != 0) return;
  // the record of this search (-1: more rounds than it holds, search
  // again) and the rigid count of this pass, for the finishing kernel
  // Only a filling search that does not read records writes one (a pass
  // that does not fill writes no list; and a sphere that had to search
  // although the pass reads records keeps none, since a record must hold
  // the partners around where the last sort saw the particles).
  if (stored >= 0)
    d.act_meta[s] = make_int2(stored, nrig);
  else
    d.act_meta[s] = make_int2(FILL && !use_rec && rounds <= ACT_ROUNDS ? rounds : -1, nrig);
  double* out = d.act_sum + 8 * (size_t)wave;
  out[0] = om;
  out[1] = v0;
  out[2] = v1;
  out[3] = v2;
  out[4] = f0;
  out[5] = f1;
  out[6] = f2;
  out[7] = l2;
}

// (a6, second half) one thread per sphere, in cell order: eps, F^DG and
// F^PG from the sums its action wave left (the per-sphere FP64 algebra,
// divisions and powers, runs here with every lane busy instead of on one
// lane of each action wave)
template <bool STRESS>
__global__ __launch_bounds__(BS) void k_fpi_finish(Dev d) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= d.nr) return;
  const int s = d.ritems[t];
  const int si = d.rig_sorted[s];
  const double R = d.pos[si].w, H = R + d.h;
  const double invH = 1.0 / H, wnorm = 105.0 / (16.0 * PI * H * H * H);  // Eq. kernel
  const double* a = d.act_sum + 8 * (size_t)t;
  const double om = a[0], v0 = a[1], v1 = a[2], v2 = a[3], f0 = a[4], f1 = a[5], f2 = a[6];
  const int nrig = d.act_meta[s].y;
  const double Vs = 4.0 / 3.0 * PI * R * R * R;
  const double VH = 4.0 / 3.0 * PI * H * H * H;
  double eps = 1.0 - Vs * (double)nrig / VH;
  eps = fmin(fmax(eps, d.eps_min), 1.0);
  d.eps[s] = eps;
  d.omega[s] = om;
  double dg[3] = {0, 0, 0}, pg[3] = {0, 0, 0};
  if (om > 0.0) {
    const D4 vs = d.vel[si];
    double dv[3] = {vs.x - v0 / om, vs.y - v1 / om, vs.z - v2 / om};
    double dva = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
    double B_ = drag_b(eps, dva, 2.0 * R, d.rho0, d.eta);
    double kp = d.rho0 * Vs / d.m_f;
    for (int k = 0; k < 3; ++k) dg[k] = -B_ * Vs * dv[k];
    pg[0] = kp * (f0 / om);
    pg[1] = kp * (f1 / om);
    pg[2] = kp * (f2 / om);
  }
  for (int k = 0; k < 3; ++k) {
    d.f_dg[3 * s + k] = dg[k];
    d.f_pg[3 * s + k] = pg[k];
  }
  // virial of the coupling: lever (sum_j w_sj r_sj / Omega_s)_z times the
  // x force (the contacts keep theirs beside it)
  if (STRESS) d.wzx_r[2 * s] = om > 0.0 ? (a[7] / om) * (dg[0] + pg[0]) : 0.0;
  // F^DG / Omega times the kernel's normalisation beside the sphere's
  // cell-ordered record, with 1/H_s (0: the sphere couples to nothing)
  D4 rc;
  rc.x = om > 0.0 ? dg[0] / om * wnorm : 0.0;
  rc.y = om > 0.0 ? dg[1] / om * wnorm : 0.0;
  rc.z = om > 0.0 ? dg[2] / om * wnorm : 0.0;
  rc.w = om > 0.0 ? invH : 0.0;
  d.rdg_c[t] = rc;
}

void launch_fpi_action(const Dev& d, bool fill, bool use_rec, hipStream_t st) {
  if (d.nr == 0) return;
  auto k = d.stress ? (fill ? k_fpi_action<true, true> : k_fpi_action<true, false>)
                    : (fill ? k_fpi_action<false, true> : k_fpi_action<false, false>);
  k<<<nblocks((size_t)d.nr * 64), BS, 0, st>>>(d, use_rec ? 1 : 0);
  // one wavefront per block: the few thousand threads of the finish spread
  // over as many CUs as possible (its FP64 divisions and powers are latency)
  auto f = d.stress ? k_fpi_finish<true> : k_fpi_finish<false>;
  f<<<(d.nr + 63) / 64, 64, 0, st>>>(d);
}

// (a7) reaction on the coupled fluid particles, Eq. F_fpi_DG_reac
// normalised per rigid particle: -sum_s F^DG_s w_sj / Omega_s over the
// rigid s with j in C_s.  The rigid grid's cells are at least H_max wide.
// The reaction on fluid particle i with c > 0 coupling slots; also stored
// in the F_RXN planes (read by the field readout and, when not fused, by
// the update).  Returns the stored FP32 values.
__device__ __forceinline__ void reaction_of(const Dev& d, const BoxD& B, int i, int c,
                                            float out[3]) {
  const size_t np = (size_t)d.npad;
  double a0 = 0, a1 = 0, a2 = 0;
  if (c <= RXN_CAP) {
    // the slots the action left, summed in ascending sphere-record order
    // (a fixed order whatever order the slots were filled in)
    int ts[RXN_CAP];
    float ws[RXN_CAP];
#pragma unroll
    for (int k = 0; k < RXN_CAP; ++k) {
      const int2 sl = k < c ? d.rxn_slot[(size_t)k * np + i] : make_int2(INT_MAX, 0);
      ts[k] = sl.x;
      ws[k] = __int_as_float(sl.y);
    }
    int last = -1;
    for (int m = 0; m < c; ++m) {
      int best = INT_MAX;
      float bw = 0.0f;
#pragma unroll
      for (int k = 0; k < RXN_CAP; ++k)
        if (ts[k] > last && ts[k] < best) {
          best = ts[k];
          bw = ws[k];
        }
      last = best;
      const D4 g = d.rdg_c[best];
      a0 -= g.x * (double)bw;
      a1 -= g.y * (double)bw;
      a2 -= g.z * (double)bw;
    }
  } else {
    // more spheres than slots: search the rigid grid
    D4 pi = d.pos[i];
    const Geo G = geo_of(B);
    const Grid gr = B.rg;
    const int coff = B.rcell_off;
    int oob = 0;
    int cc[3] = {cell_coord(pi.x, gr, 0, &oob), cell_coord(pi.y, gr, 1, &oob),
                 cell_coord(pi.z, gr, 2, &oob)};
    for_stencil<false>(G, gr, coff, pi.x, pi.y, pi.z, B.couple_R, cc, 1, [&](int cb, int ce) {
      int tb = d.rstart[cb], te = d.rstart[ce];
      for (int t = tb; t < te; ++t) {
        D4 g = d.rdg_c[t];
        if (g.w == 0.0) continue;
        D4 ps = d.rpos_c[t];
        double H = ps.w + d.h;
        double ex = ps.x - pi.x, ey = ps.y - pi.y, ez = ps.z - pi.z;
        min_img_box(G, ex, ey, ez);
        double r2 = r2_exact(ex, ey, ez);
        if (!(r2 < H * H)) continue;
        // Lucy weight of support H without its normalisation (folded into g)
        const double q = sqrt(r2) * g.w, omq = 1.0 - q;
        const double w = (1.0 + 3.0 * q) * omq * omq * omq;
        a0 -= g.x * w;
        a1 -= g.y * w;
        a2 -= g.z * w;
      }
    });
  }
  out[0] = (float)a0;
  out[1] = (float)a1;
  out[2] = (float)a2;
  d.fout[9 * np + i] = out[0];
  d.fout[10 * np + i] = out[1];
  d.fout[11 * np + i] = out[2];
}

__global__ __launch_bounds__(BS) void k_fpi_reaction(Dev d) {
  int i;
  const int b = blk_box<true>(d, i);
  if (b < 0) return;
  const BoxD& B = d.boxes[b];
  if (i >= B.first + B.count) return;
  // the action's slot count: nonzero exactly for the fluid particles
  // inside some sphere's support
  const int c = d.rxn_cnt[i];
  if (c == 0) return;
  float out[3];
  reaction_of(d, B, i, c, out);
}

void launch_fpi_reaction(const Dev& d, hipStream_t st) {
  k_fpi_reaction<<<d.nablk, BS, 0, st>>>(d);
}

// ---------------------------------------------------------------------------
// (a8) DEM contacts (Sec. 2.2) and lubrication (Sec. 2.3), FP64, over the
// cell-ordered rigid records: one wavefront per rigid particle, one
// candidate partner per lane.  The contact table row of a particle holds
// partner ids and tangential displacements; commit (second pass) writes the
// next table: the updated history of every pair still in contact, in
// candidate order (ballot + prefix count, so the order is deterministic).

struct DemAcc {
  double F[3], FL[3], N[3], Wzx;
};

// one candidate partner t of sphere s; returns 1 if it is a contact, with
// its partner id and committed tangential displacement
__device__ __forceinline__ int dem_pair_eval(const Dev& d, const Geo& G, int s, const D4& ps,
                                             const D4& vs, const D4& ws, int t, int ocnt,
                                             DemAcc& acc, int& gk, double nd[3]) {
  const double Rs = ps.w, ms = vs.w;
  const double Di = (1.0 - d.nu * d.nu) / (d.E * PI);
  const int mc = d.maxc;
  D4 pk = d.rpos_c[t];
  double Rk = pk.w;
  double e0 = ps.x - pk.x, e1 = ps.y - pk.y, e2 = ps.z - pk.z;
  const int kz = min_img_box(G, e0, e1, e2);
  double L2 = r2_exact(e0, e1, e2);
  double reachk = Rs + Rk + d.h;
  if (!(L2 < reachk * reachk)) return 0;
  double L = sqrt(L2);
  D4 vk = d.rvel_c[t];
  vk.x += (double)kz * G.le_jump;  // image velocity (Lees-Edwards)
  if (L < Rs + Rk) {
    D4 wk = d.rom_c[t];
    gk = d.rig_gid[d.ritems[t]];
    double dt0 = 0, dt1 = 0, dt2 = 0;
    for (int q = 0; q < ocnt; ++q) {
      if (d.ct_partner[s * mc + q] == gk) {
        dt0 = d.ct_dt[(size_t)(s * mc + q) * 3 + 0];
        dt1 = d.ct_dt[(size_t)(s * mc + q) * 3 + 1];
        dt2 = d.ct_dt[(size_t)(s * mc + q) * 3 + 2];
        break;
      }
    }
    double n0 = e0 / L, n1 = e1 / L, n2 = e2 / L;
    double ov = L - (Rs + Rk);  // delta_n = ov * n
    double u0 = vs.x - vk.x, u1 = vs.y - vk.y, u2 = vs.z - vk.z;
    double un = u0 * n0 + u1 * n1 + u2 * n2;
    double rw0 = Rs * ws.x + Rk * wk.x, rw1 = Rs * ws.y + Rk * wk.y, rw2 = Rs * ws.z + Rk * wk.z;
    double t0 = u0 - un * n0 + (rw1 * n2 - rw2 * n1);
    double t1 = u1 - un * n1 + (rw2 * n0 - rw0 * n2);
    double t2 = u2 - un * n2 + (rw0 * n1 - rw1 * n0);
    double kn = 4.0 / (3.0 * PI) * (1.0 / (Di + Di)) * sqrt(Rs * Rk / (Rs + Rk));
    double kt = kn / (2.0 * (1.0 + d.nu));
    double mk = vk.w;
    double mm = 2.0 * ms * mk / (ms + mk);
    double cn = d.damp * 2.0 * sqrt(mm * kn), ct = d.damp * 2.0 * sqrt(mm * kt);
    double fn0 = -kn * ov * n0 - cn * un * n0;
    double fn1 = -kn * ov * n1 - cn * un * n1;
    double fn2 = -kn * ov * n2 - cn * un * n2;
    double ft0 = -kt * dt0 - ct * t0, ft1 = -kt * dt1 - ct * t1, ft2 = -kt * dt2 - ct * t2;
    double vta = sqrt(t0 * t0 + t1 * t1 + t2 * t2);
    double dta = sqrt(dt0 * dt0 + dt1 * dt1 + dt2 * dt2);
    double d0 = 0, d1 = 0, d2 = 0;
    if (vta > 0.0) {
      d0 = t0 / vta;
      d1 = t1 / vta;
      d2 = t2 / vta;
    } else if (dta > 0.0) {
      d0 = dt0 / dta;
      d1 = dt1 / dta;
      d2 = dt2 / dta;
    }
    double fna = sqrt(fn0 * fn0 + fn1 * fn1 + fn2 * fn2);
    double fta = sqrt(ft0 * ft0 + ft1 * ft1 + ft2 * ft2);
    double lim = d.mu * fna;
    if (fta >= lim) {  // Coulomb slider, Eq. slideref
      ft0 = -lim * d0;
      ft1 = -lim * d1;
      ft2 = -lim * d2;
      double m = lim / kt;
      nd[0] = m * d0;
      nd[1] = m * d1;
      nd[2] = m * d2;
    } else {  // Eq. tandispn
      nd[0] = dta * d0 + t0 * d.dt;
      nd[1] = dta * d1 + t1 * d.dt;
      nd[2] = dta * d2 + t2 * d.dt;
    }
    acc.F[0] += fn0 + ft0;
    acc.F[1] += fn1 + ft1;
    acc.F[2] += fn2 + ft2;
    acc.Wzx += 0.5 * e2 * (fn0 + ft0);
    // torque R_s (-n) x F_t
    acc.N[0] += -Rs * (n1 * ft2 - n2 * ft1);
    acc.N[1] += -Rs * (n2 * ft0 - n0 * ft2);
    acc.N[2] += -Rs * (n0 * ft1 - n1 * ft0);
    return 1;
  }
  if (d.lub) {
    double gap = L - (Rs + Rk);
    if (gap > 0.0 && gap < d.h) {
      double db = Rs + Rk;
      double gg = gap > d.lub_gap_min ? gap : d.lub_gap_min;
      double c = 3.0 * PI * d.eta * db * db / (8.0 * gg);
      acc.FL[0] += c * (vk.x - vs.x);
      acc.FL[1] += c * (vk.y - vs.y);
      acc.FL[2] += c * (vk.z - vs.z);
      acc.Wzx += 0.5 * e2 * (c * (vk.x - vs.x));
    }
  }
  return 0;
}

// at most 128 registers (four waves per SIMD instead of three; a few
// spills, 7 % faster over the dam break's 20,000 spheres)
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(4))) void k_dem(
    Dev d, int commit, int* nxt_cnt, int* nxt_partner, double* nxt_dt) {
  const int wave = xcd_wave();
  const int lane = threadIdx.x & 63;
  if (wave >= d.nr) return;
  // spheres in rigid-grid cell order: neighbouring waves share cache lines
  const int me = wave;
  const int s = __builtin_amdgcn_readfirstlane(d.ritems[me]);
  const BoxD& B = d.boxes[__builtin_amdgcn_readfirstlane(d.rbox[s])];
  const Geo G = geo_of(B);
  const Grid gr = B.rg;
  const int coff = B.rcell_off, reach = B.dem_reach;
  // partners k lie within R_s + R_k + h <= R_s + (R_max + h)
  const double dem_Rk = B.couple_R;
  const D4 ps = d.rpos_c[me], vs = d.rvel_c[me], ws = d.rom_c[me];
  int oob = 0;
  int cc[3] = {cell_coord(ps.x, gr, 0, &oob), cell_coord(ps.y, gr, 1, &oob),
               cell_coord(ps.z, gr, 2, &oob)};
  const int mc = d.maxc;
  const int ocnt = d.ct_cnt[s];
  DemAcc acc = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, 0.0};
  int ncnt = 0;
  int overflow = 0;
  const StencilShape sh = stencil_shape(gr, cc, reach);
  const int nrows = sh.zn * sh.yn;
  for (int rb = 0; rb < nrows; rb += 64) {
    int sa = 0, la = 0, sb = 0, lb = 0;
    if (rb + lane < nrows) {
      int a0, a1, b0, b1;
      stencil_row<true>(G, gr, coff, ps.x, ps.y, ps.z, ps.w + dem_Rk, cc, reach, sh, rb + lane,
                        a0, a1, b0, b1);
      if (a1 > a0) {
        sa = d.rstart[a0];
        la = d.rstart[a1] - sa;
      }
      if (b1 > b0) {
        sb = d.rstart[b0];
        lb = d.rstart[b1] - sb;
      }
    }
    const int len = la + lb;
    int inc = len;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      int t = __shfl_up(inc, o, 64);
      if (lane >= o) inc += t;
    }
    const int total = __shfl(inc, 63, 64);
    const int off = inc - len;
    for (int base = 0; base < total; base += 64) {
      const int t = base + lane;
      int r = 0;  // last row whose offset is <= t
#pragma unroll
      for (int stp = 32; stp > 0; stp >>= 1) {
        int cand = r + stp;
        int v = __shfl(off, cand & 63, 64);
        if (cand < 64 && v <= t) r = cand;
      }
      const int offr = __shfl(off, r, 64);
      const int sar = __shfl(sa, r, 64);
      const int lar = __shfl(la, r, 64);
      const int sbr = __shfl(sb, r, 64);
      int contact = 0, gk = -1;
      double nd[3] = {0, 0, 0};
      if (t < total) {
        const int q = t - offr;
        const int tt = q < lar ? sar + q : sbr + (q - lar);
        if (tt != me) contact = dem_pair_eval(d, G, s, ps, vs, ws, tt, ocnt, acc, gk, nd);
      }
      if (commit) {
        // contacts of this round in candidate order
        const uint64_t m = __ballot(contact);
        const int before = __popcll(m & ((1ull << lane) - 1ull));
        const int slot = ncnt + before;
        if (contact) {
          if (slot < mc) {
            nxt_partner[s * mc + slot] = gk;
            nxt_dt[(size_t)(s * mc + slot) * 3 + 0] = nd[0];
            nxt_dt[(size_t)(s * mc + slot) * 3 + 1] = nd[1];
            nxt_dt[(size_t)(s * mc + slot) * 3 + 2] = nd[2];
          } else {
            overflow = 1;
          }
        }
        ncnt += __popcll(m);
      }
    }
  }
  for (int a = 0; a < 3; ++a) {
    acc.F[a] = wave_sum(acc.F[a]);
    acc.FL[a] = wave_sum(acc.FL[a]);
    acc.N[a] = wave_sum(acc.N[a]);
  }
  if (d.stress) acc.Wzx = wave_sum(acc.Wzx);
  overflow = __any(overflow);
  if (lane != 0) return;
  for (int a = 0; a < 3; ++a) {
    d.f_dem[3 * s + a] = acc.F[a];
    d.f_lub[3 * s + a] = acc.FL[a];
    d.n_dem[3 * s + a] = acc.N[a];
  }
  if (d.stress) d.wzx_r[2 * s + 1] = acc.Wzx;
  if (commit) {
    nxt_cnt[s] = ncnt < mc ? ncnt : mc;
    if (overflow || ncnt > mc) atomicOr(d.status, ST_CONTACT_OVERFLOW);
  }
}

void launch_dem(const Dev& d, int commit, int* nxt_cnt, int* nxt_partner, double* nxt_dt,
                hipStream_t st) {
  if (d.nr == 0) return;
  k_dem<<<nblocks((size_t)d.nr * 64), BS, 0, st>>>(d, commit, nxt_cnt, nxt_partner, nxt_dt);
}

// ---------------------------------------------------------------------------
// (a9) velocity Verlet (Alg. 1, update) with the boundary treatment.

// rxo: the fluid particle's reaction when the caller formed it (null: read
// the F_RXN planes)
__device__ __forceinline__ void total_force(const Dev& d, const BoxD& B, int i, uint8_t t,
                                            const D4& p, int rigid_active, double F[3],
                                            double N[3], const float* rxo = nullptr) {
  double sg = 1.0;
  if (d.gtype == 1) {
    double x = d.gaxis == 0 ? p.x : (d.gaxis == 1 ? p.y : p.z);
    sg = (x - B.org[d.gaxis] >= 0.5 * B.L[d.gaxis]) ? 1.0 : -1.0;
  }
  const size_t np = (size_t)d.npad;
  double m = d.vel[i].w;
  for (int a = 0; a < 3; ++a) {
    double body = m * d.body[a] * sg;
    if (t == T_FLUID) {
      double rx = rxo ? (double)rxo[a]
                      : (d.have_rxn && d.rxn_cnt[i] > 0) ? (double)d.fout[(9 + a) * np + i]
                                                         : 0.0;
      F[a] = (double)d.fout[a * np + i] + rx + body;
      N[a] = (double)d.fout[(3 + a) * np + i];
    } else if (t == T_INNER) {
      F[a] = (double)d.fout[a * np + i] + body;
      N[a] = (double)d.fout[(3 + a) * np + i];
    } else if (t == T_RIGID && rigid_active) {
      int s = d.gid2slot[d.gid[i]];
      F[a] = d.f_pg[3 * s + a] + d.f_dg[3 * s + a] + d.f_dem[3 * s + a] + d.f_lub[3 * s + a] +
             body;
      N[a] = d.n_dem[3 * s + a];
    } else {
      F[a] = 0.0;
      N[a] = 0.0;
    }
  }
}

// RXN: the reaction of the coupled fluid particles is formed here too
// (one launch less; the particle's F_RXN is used from registers)
// (64 registers, eight waves per SIMD, fit without spills)
// MOVED: 1 raises the flag of candidate reuse for a drift of skin/2; 2 also
// handles sheared boxes (the drift less the flow's, a limit shrinking with
// the time since the search)
template <int VELVER, bool RXN, int MOVED = 0>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(8))) void k_integrate(Dev d, int rigid_active, int end_step) {
  // the last pass of a step advances the device step counter (no kernel of
  // this launch reads it); only the second half-kick ends a step, and the
  // drift variants, without this store ahead of their loads, read the box
  // constants through the scalar cache
  if (VELVER == 2 && end_step && blockIdx.x == 0 && threadIdx.x == 0) d.dstep[0] += 1;
  int i;
  const int b = blk_box<true>(d, i);
  if (b < 0) return;
  const BoxD& B = d.boxes[b];
  if (i >= B.first + B.count) return;
  uint8_t t = d.type[i];
  if (t == T_OUTER) return;
  if (t == T_RIGID && !rigid_active) return;
  // the reaction first, before the particle's own state is live
  float rxf[3] = {0.0f, 0.0f, 0.0f};
  const int c = RXN && t == T_FLUID ? d.rxn_cnt[i] : 0;
  if (c > 0) reaction_of(d, B, i, c, rxf);
  D4 v = d.vel[i], w = d.om[i];
  // the second half-kick reads the position only for the split body force
  // (positions do not move in that pass, and the first one checked them)
  D4 p = {0.0, 0.0, 0.0, 0.0};
  if (VELVER == 1 || d.gtype == 1) p = d.pos[i];
  double F[3], N[3];
  total_force(d, B, i, t, p, rigid_active, F, N, RXN && t == T_FLUID ? rxf : nullptr);
  const double hdt = 0.5 * d.dt;
  v.x += hdt * F[0] / v.w;
  v.y += hdt * F[1] / v.w;
  v.z += hdt * F[2] / v.w;
  w.x += hdt * N[0] / w.w;
  w.y += hdt * N[1] / w.w;
  w.z += hdt * N[2] / w.w;
  int bad = 0;
  if (VELVER == 1 && (t == T_FLUID || t == T_RIGID)) {
    double x[3] = {p.x + d.dt * v.x, p.y + d.dt * v.y, p.z + d.dt * v.z};
    double vv[3] = {v.x, v.y, v.z};
    if (B.le) {
      // through a sheared z face: re-enter as the image of the next box
      if (x[2] < B.org[2]) {
        x[2] += B.L[2];
        x[0] += B.le_next;
        vv[0] += B.le_jump;
      } else if (x[2] >= B.org[2] + B.L[2]) {
        x[2] -= B.L[2];
        x[0] -= B.le_next;
        vv[0] -= B.le_jump;
      }
      if (x[0] < B.org[0])
        x[0] += B.L[0];
      else if (x[0] >= B.org[0] + B.L[0])
        x[0] -= B.L[0];
    }
    bool hit = false;  // a wall face was crossed in this drift
    for (int a = 0; a < 3; ++a) {
      double lo = B.org[a], hi = B.org[a] + B.L[a];
      if (B.per[a]) {
        if (x[a] < lo)
          x[a] += B.L[a];
        else if (x[a] >= hi)
          x[a] -= B.L[a];
      } else if (x[a] < lo || x[a] > hi) {
        x[a] = x[a] < lo ? 2.0 * lo - x[a] : 2.0 * hi - x[a];
        hit = true;
        if (!d.noslip) vv[a] = -vv[a];  // slip: the normal component
        if (x[a] < lo || x[a] > hi) bad |= ST_OUT_OF_DOMAIN;
      }
    }
    // no-slip: the whole velocity reversed once, also at an edge or corner
    if (hit && d.noslip) {
      vv[0] = -vv[0];
      vv[1] = -vv[1];
      vv[2] = -vv[2];
    }
    p.x = x[0];
    p.y = x[1];
    p.z = x[2];
    v.x = vv[0];
    v.y = vv[1];
    v.z = vv[2];
    d.pos[i] = p;
  }
  if (!isfinite(v.x) || !isfinite(v.y) || !isfinite(v.z) || !isfinite(w.x) || !isfinite(w.y) ||
      !isfinite(w.z) || (VELVER == 1 && (!isfinite(p.x) || !isfinite(p.y) || !isfinite(p.z))))
    bad |= ST_NONFINITE;
  if (bad) atomicOr(d.status, bad);
  d.vel[i] = v;
  d.om[i] = w;
  if (VELVER == 2) {
    // positions did not move: refresh the pair record for the next pass
    PR* r = d.prec + i;
    r->vx = (float)v.x;
    r->vy = (float)v.y;
    r->vz = (float)v.z;
    r->wx = (float)w.x;
    r->wy = (float)w.y;
    r->wz = (float)w.z;
  }
  // Farther than skin/2 from where the last search saw it: the next lists
  // need a new search (one atomic per wave, not per particle).  Tested after
  // the stores, when the velocities are no longer live (the sheared test
  // needs registers of its own).
  if (MOVED && VELVER == 1 && (t == T_FLUID || t == T_RIGID)) {
    const D4 q = d.xref[i];
    double ex = p.x - q.x, ey = p.y - q.y, ez = p.z - q.z;
    bool far;
    if (MOVED == 2 && B.le) {
      // sheared: the displacement through the images of the drifted
      // positions, less the flow's x displacement since the search at the
      // reference height; two partners' separations then change by at most
      // twice that plus shear_reach ts, which must stay below skin (ts the
      // time between the searched positions and these: across a sheared
      // face the image offset moved by the rate times L_z ts)
      Geo G = geo_of(B);
      G.le_shift = B.le_next;
      min_img_box(G, ex, ey, ez);
      const double ts = (double)(d.dstep[0] - d.sstep[0]) * d.dt;
      ex -= B.shear * (q.z - (B.org[2] + 0.5 * B.L[2])) * ts;
      const double lim = (d.pad - 0.5 * B.shear_reach * ts) * (1.0 - 1e-9);
      far = !(lim > 0.0) || r2_exact(ex, ey, ez) > lim * lim;
    } else {
      min_img_box(geo_of(B), ex, ey, ez);
      far = r2_exact(ex, ey, ez) > d.mv2;
    }
    const unsigned long long m = __ballot(far);
    if (m && (threadIdx.x & 63) == (unsigned)(__ffsll((long long)m) - 1)) atomicOr(d.moved, 1);
  }
}

void launch_integrate(const Dev& d, int velver, int rigid_active, bool end_step, bool fuse_rxn,
                      bool track_moved, hipStream_t st) {
  // only the drift (velver 1) moves particles; the moved flag of candidate
  // reuse is a separate instantiation, so the plain update keeps its registers
  auto k = velver == 2 ? (fuse_rxn ? k_integrate<2, true> : k_integrate<2, false>)
           : track_moved
               ? (d.any_le ? (fuse_rxn ? k_integrate<1, true, 2> : k_integrate<1, false, 2>)
                           : (fuse_rxn ? k_integrate<1, true, 1> : k_integrate<1, false, 1>))
               : (fuse_rxn ? k_integrate<1, true> : k_integrate<1, false>);
  k<<<d.nablk, BS, 0, st>>>(d, rigid_active, end_step ? 1 : 0);
}

// ---------------------------------------------------------------------------
// Per-box pressure tensor component P_zx after a step: kinetic part
// m v'_z v'_x with v' the velocity less the shear profile, plus the virial of
// the last force evaluation (pair kernel plane 12 for fluid and inner walls,
// wzx_r for rigid particles), over the box volume.  One block per box sums
// its fixed particle range in a fixed order, so the result is repeatable.

// Per-box pressure tensor sample in two launches with a fixed summation
// order: each launch block sums m v_z v'_x + the virial over its particles
// (a tree in shared memory), then one thread per box adds its blocks'
// partial sums in block order.  A box's blocks start at its first particle,
// so a box gives the same bits alone or in a batch.
__global__ __launch_bounds__(BS) void k_box_stress_part(Dev d, int rigid_active) {
  __shared__ double sh[BS];
  const unsigned lb = logical_block(d);
  int i;
  const int b = blk_box(d, i);
  double q = 0.0;
  if (b >= 0) {
    const BoxD& B = d.boxes[b];
    if (i < B.first + B.count) {
      const uint8_t t = d.type[i];
      if (t != T_OUTER) {
        const size_t np = (size_t)d.npad;
        const double zmid = B.org[2] + 0.5 * B.L[2];
        const D4 p = d.pos[i], v = d.vel[i];
        const double vx = v.x - B.shear * (p.z - zmid);
        q = v.w * v.z * vx;
        if (t == T_FLUID || t == T_INNER)
          q += (double)d.fout[12 * np + i];
        else if (t == T_RIGID && rigid_active) {
          const int k = d.gid2slot[d.gid[i]];
          q += d.wzx_r[2 * k] + d.wzx_r[2 * k + 1];  // coupling + contacts
        }
      }
    }
  }
  sh[threadIdx.x] = q;
  __syncthreads();
  for (int o = BS / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) d.st_part[lb] = sh[0];
}

__global__ void k_box_stress_final(Dev d, int accumulate) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= d.nbox) return;
  const BoxD& B = d.boxes[b];
  const int nb = (B.count + BS - 1) / BS;
  const double* part = d.st_part + B.blk_first;
  // the partials in block order; eight loads in flight at a time (one
  // thread per box would otherwise wait a memory latency per block), the
  // sum itself in the same order
  double acc = 0.0;
  int c = 0;
  for (; c + 8 <= nb; c += 8) {
    double v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = part[c + k];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc += v[k];
  }
  for (; c < nb; ++c) acc += part[c];
  const double pzx = acc / B.vol;
  d.st_inst[b] = pzx;
  if (accumulate) d.st_sum[b] += pzx;
}

void launch_box_stress(const Dev& d, int accumulate, hipStream_t st) {
  k_box_stress_part<<<d.nblk, BS, 0, st>>>(d, d.have_rxn);
  k_box_stress_final<<<(d.nbox + 63) / 64, 64, 0, st>>>(d, accumulate);
}

// ---------------------------------------------------------------------------
// read-out in id order

__global__ __launch_bounds__(BS) void k_read_field(Dev d, int field, int rigid_active,
                                                  double* out) {
  int i = xcd_tid();
  if (i >= d.n) return;
  const int g = d.gid[i];
  const uint8_t t = d.type[i];
  const size_t np = (size_t)d.npad;
  double v[3] = {0, 0, 0};
  int comps = (field == SDPDEM_DENS || field == SDPDEM_PRES || field == SDPDEM_PRES_SMOOTH ||
               field == SDPDEM_EPS) ? 1 : 3;
  int s = (t == T_RIGID) ? d.gid2slot[g] : -1;
  switch (field) {
    case SDPDEM_POS: {
      D4 p = d.pos[i];
      v[0] = p.x;
      v[1] = p.y;
      v[2] = p.z;
    } break;
    case SDPDEM_VEL: {
      D4 p = d.vel[i];
      v[0] = p.x;
      v[1] = p.y;
      v[2] = p.z;
    } break;
    case SDPDEM_ANGVEL: {
      D4 p = d.om[i];
      v[0] = p.x;
      v[1] = p.y;
      v[2] = p.z;
    } break;
    case SDPDEM_DENS:
      v[0] = d.rho[i];
      break;
    case SDPDEM_PRES:
      v[0] = d.p[i];
      break;
    case SDPDEM_PRES_SMOOTH:
      v[0] = (double)d.ps[i];
      break;
    case SDPDEM_F_SDPD:
    case SDPDEM_N_SDPD:
    case SDPDEM_F_CD:
    case SDPDEM_F_RXN: {
      int base = field == SDPDEM_F_SDPD ? 0 : field == SDPDEM_N_SDPD ? 3 : field == SDPDEM_F_CD ? 6 : 9;
      if (field != SDPDEM_F_RXN || (d.have_rxn && d.rxn_cnt[i] > 0))
        for (int a = 0; a < 3; ++a) v[a] = (double)d.fout[(base + a) * np + i];
    } break;
    case SDPDEM_F_DG:
    case SDPDEM_F_PG:
    case SDPDEM_F_DEM:
    case SDPDEM_F_LUB:
    case SDPDEM_N_DEM:
      if (s >= 0 && rigid_active) {
        const double* src = field == SDPDEM_F_DG ? d.f_dg : field == SDPDEM_F_PG ? d.f_pg
                          : field == SDPDEM_F_DEM ? d.f_dem : field == SDPDEM_F_LUB ? d.f_lub
                          : d.n_dem;
        for (int a = 0; a < 3; ++a) v[a] = src[3 * s + a];
      }
      break;
    case SDPDEM_EPS:
      if (s >= 0 && rigid_active) v[0] = d.eps[s];
      break;
    case SDPDEM_F_TOTAL:
    case SDPDEM_N_TOTAL: {
      double F[3], N[3];
      // the box whose fixed sorted range holds i
      int lo = 0, hi = d.nbox - 1;
      while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (d.boxes[mid].first <= i)
          lo = mid;
        else
          hi = mid - 1;
      }
      total_force(d, d.boxes[lo], i, t, d.pos[i], rigid_active, F, N);
      for (int a = 0; a < 3; ++a) v[a] = field == SDPDEM_F_TOTAL ? F[a] : N[a];
    } break;
    default:
      break;
  }
  for (int a = 0; a < comps; ++a) out[(size_t)g * comps + a] = v[a];
}

void launch_read_field(const Dev& d, int field, int rigid_active, double* out, hipStream_t st) {
  k_read_field<<<nblocks(d.n), BS, 0, st>>>(d, field, rigid_active, out);
}

// FP64 totals: per-block partial sums in a fixed tree, then one block.
static constexpr int NTOT = 13;

__global__ __launch_bounds__(BS) void k_totals_partial(Dev d, double* part) {
  __shared__ double sh[NTOT][BS];
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  double q[NTOT];
  for (int k = 0; k < NTOT; ++k) q[k] = 0.0;
  q[9] = INFINITY;
  q[10] = -INFINITY;
  if (i < d.n && d.type[i] != T_OUTER) {
    D4 x = d.pos[i], v = d.vel[i], w = d.om[i];
    double m = v.w, I = w.w;
    q[0] = m * v.x;
    q[1] = m * v.y;
    q[2] = m * v.z;
    q[3] = m * (x.y * v.z - x.z * v.y) + I * w.x;
    q[4] = m * (x.z * v.x - x.x * v.z) + I * w.y;
    q[5] = m * (x.x * v.y - x.y * v.x) + I * w.z;
    double v2 = v.x * v.x + v.y * v.y + v.z * v.z;
    q[6] = 0.5 * m * v2;
    q[7] = 0.5 * I * (w.x * w.x + w.y * w.y + w.z * w.z);
    q[8] = sqrt(v2);
    q[9] = d.rho[i];
    q[10] = d.rho[i];
    q[11] = m;
  }
  for (int k = 0; k < NTOT; ++k) sh[k][threadIdx.x] = q[k];
  __syncthreads();
  for (int o = BS / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      for (int k = 0; k < NTOT; ++k) {
        double a = sh[k][threadIdx.x], b = sh[k][threadIdx.x + o];
        sh[k][threadIdx.x] = k == 8 || k == 10 ? fmax(a, b) : k == 9 ? fmin(a, b) : a + b;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < NTOT; ++k) part[(size_t)blockIdx.x * NTOT + k] = sh[k][0];
}

__global__ __launch_bounds__(BS) void k_totals_final(const double* part, int nb, double* out) {
  __shared__ double sh[NTOT][BS];
  double q[NTOT];
  for (int k = 0; k < NTOT; ++k) q[k] = k == 9 ? INFINITY : (k == 10 || k == 8) ? -INFINITY : 0.0;
  q[8] = 0.0;
  for (int b = threadIdx.x; b < nb; b += BS)
    for (int k = 0; k < NTOT; ++k) {
      double x = part[(size_t)b * NTOT + k];
      q[k] = k == 8 || k == 10 ? fmax(q[k], x) : k == 9 ? fmin(q[k], x) : q[k] + x;
    }
  for (int k = 0; k < NTOT; ++k) sh[k][threadIdx.x] = q[k];
  __syncthreads();
  for (int o = BS / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      for (int k = 0; k < NTOT; ++k) {
        double a = sh[k][threadIdx.x], b = sh[k][threadIdx.x + o];
        sh[k][threadIdx.x] = k == 8 || k == 10 ? fmax(a, b) : k == 9 ? fmin(a, b) : a + b;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < NTOT; ++k) out[k] = sh[k][0];
}

int totals_partial_blocks(int n) { return (n + BS - 1) / BS > 0 ? (n + BS - 1) / BS : 1; }

void launch_totals(const Dev& d, double* partial, double* out, hipStream_t st) {
  int nb = totals_partial_blocks(d.n);
  k_totals_partial<<<nb, BS, 0, st>>>(d, partial);
  k_totals_final<<<1, BS, 0, st>>>(partial, nb, out);
}

}  // namespace sdpdem
